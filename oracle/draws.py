"""The SRFT's random quantities as the library draws them, for tests.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3 draws D's diagonal uniformly on the unit circle (random signs for
real data) and S's l rows without replacement (the paper's experiments).
When the library draws them itself it uses a counter-based generator, so a
draw is a pure function of (seed, draw number, system index); this module
computes the same draw independently, from the generator's published
definition and the sampling rule, so the library's draw can be checked
bit for bit:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): a counter of four 32-bit words and a key of two;
  each of the ten rounds multiplies words 0 and 2 by the constants
  0xD2511F53 and 0xCD9E8D57 (64-bit products, split into high and low
  halves) and mixes: (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key grows
  by (0x9E3779B9, 0xBB67AE85) before every round after the first.
* the words w(c0, c1, c2, c3) of a draw: counter (index, draw, stream,
  system), key (seed mod 2^32, seed div 2^32); stream 0 for the phases,
  stream 1 for the indices.
* phases: u_j = (x0 div 2^5 * 2^26 + x1 div 2^6) / 2^53 from w(j, draw, 0,
  sys); d_j = exp(2 pi i u_j); real data: d_j = 1 - 2 (x2 mod 2).
* indices: Floyd's algorithm for a uniform l-subset of {0, .., N-1}: for
  t = N - l, .., N - 1 (step s = t - (N - l)), r = (y0 2^32 + y1)(t + 1) div
  2^64 from w(s, draw, 1, sys) is uniform on {0, .., t}; add r, or t if r is
  already chosen.  idx lists the subset in increasing order.
"""

from __future__ import annotations

import numpy as np

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    """Philox4x32-10 of counters (array (..., 4) of uint32) under key (k0, k1).

    Returns an array of the same shape (uint32)."""
    c = np.asarray(counter, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = c0 * np.uint64(_M0)  # < 2^64: a 32 x 32-bit product
        p1 = c2 * np.uint64(_M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def _words(seed: int, index, draw: int, stream: int, sys: int):
    index = np.asarray(index, dtype=np.uint64)
    ctr = np.stack([index, np.full_like(index, draw), np.full_like(index, stream), np.full_like(index, sys)], -1)
    return philox4x32_10(ctr, (seed & _MASK, (seed >> 32) & _MASK))


def draw_phases(seed: int, draw: int, sys: int, N: int, real: bool = False) -> np.ndarray:
    """d (N entries): unit-modulus complex128 phases, or +-1 float64 for real data."""
    w = _words(seed, np.arange(N), draw, 0, sys).astype(np.uint64)
    if real:
        return 1.0 - 2.0 * (w[:, 2] & np.uint64(1)).astype(np.float64)
    u = ((w[:, 0] >> np.uint64(5)) * np.uint64(1 << 26) + (w[:, 1] >> np.uint64(6))).astype(np.float64) * 2.0 ** -53
    return np.exp(2j * np.pi * u)


def draw_indices(seed: int, draw: int, sys: int, N: int, l: int) -> np.ndarray:
    """idx (l entries, int32): a uniform l-subset of range(N) in increasing order."""
    N, l = int(N), int(l)
    w = _words(seed, np.arange(l), draw, 1, sys)
    chosen = set()
    for s in range(l):
        t = N - l + s
        x = (int(w[s, 0]) << 32) | int(w[s, 1])
        r = (x * (t + 1)) >> 64
        chosen.add(t if r in chosen else r)
    return np.array(sorted(chosen), dtype=np.int32)


def draw_srft(seed: int, draw: int, sys: int, N: int, l: int, real: bool = False):
    """(d, idx) of one draw."""
    return draw_phases(seed, draw, sys, N, real), draw_indices(seed, draw, sys, N, l)
