"""The oracle's copy of the library's SRFT draw (oracle/draws.py), pinned to
what fixes it independently of any implementation here:

* Philox4x32-10 against the known-answer vectors published with the
  generator's reference implementation (Random123's kat_vectors: counter and
  key all zero; all ones; the hexadecimal digits of pi);
* Floyd's sampling: l distinct indices in increasing order inside [0, N), the
  whole range when l = N, and every l-subset equally likely (chi-square over
  all 56 subsets of 3 out of 8);
* the phases lie on the unit circle with uniformly distributed angle, the
  real signs are balanced, and the words of different draws, streams and
  systems differ.
"""

import itertools

import numpy as np
import pytest

import oracle
from oracle import draws


@pytest.mark.parametrize("ctr,key,out", [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
])
def test_philox_known_answers(ctr, key, out):
    got = oracle.philox4x32_10(np.array([ctr], dtype=np.uint64), key)[0]
    assert tuple(int(v) for v in got) == out


def test_philox_vectorised_matches_single():
    ctr = np.array([[j, 3, 1, 7] for j in range(50)], dtype=np.uint64)
    many = oracle.philox4x32_10(ctr, (11, 12))
    for j in (0, 17, 49):
        one = oracle.philox4x32_10(ctr[j:j + 1], (11, 12))[0]
        assert np.array_equal(one, many[j])


@pytest.mark.parametrize("N,l", [(1, 1), (8, 3), (16, 16), (1024, 256), (4096, 1), (65536, 2048)])
def test_indices_distinct_sorted_in_range(N, l):
    for seed in (0, 1, 2**40 + 5):
        idx = oracle.draw_indices(seed, 0, 0, N, l)
        assert idx.dtype == np.int32 and idx.shape == (l,)
        assert np.all(np.diff(idx) > 0)
        assert idx[0] >= 0 and idx[-1] < N
    if l == N:
        assert np.array_equal(idx, np.arange(N))


def test_indices_uniform_over_subsets():
    """Floyd's algorithm gives every 3-subset of 8 with probability 1/56."""
    subsets = {s: 0 for s in itertools.combinations(range(8), 3)}
    trials = 28000
    for t in range(trials):
        subsets[tuple(int(v) for v in oracle.draw_indices(t, 0, 0, 8, 3))] += 1
    expect = trials / 56
    chi2 = sum((c - expect) ** 2 / expect for c in subsets.values())
    # 55 degrees of freedom: the 0.999 quantile is about 93
    assert chi2 < 93, chi2
    assert min(subsets.values()) > 0


def test_phases_unit_and_uniform():
    d = oracle.draw_phases(5, 0, 0, 1 << 16)
    assert d.dtype == np.complex128
    assert np.max(np.abs(np.abs(d) - 1.0)) < 1e-15
    ang = (np.angle(d) / (2 * np.pi)) % 1.0
    # Kolmogorov-Smirnov distance to U[0, 1): 1.95 / sqrt(n) is the 0.001 level
    srt = np.sort(ang)
    n = srt.size
    ks = max(np.max(np.arange(1, n + 1) / n - srt), np.max(srt - np.arange(n) / n))
    assert ks < 1.95 / np.sqrt(n)
    assert abs(np.mean(d)) < 5.0 / np.sqrt(n)


def test_real_signs_balanced():
    d = oracle.draw_phases(9, 0, 0, 1 << 16, real=True)
    assert set(np.unique(d)) == {-1.0, 1.0}
    assert abs(np.mean(d)) < 5.0 / np.sqrt(d.size)


def test_draws_streams_systems_differ():
    a = oracle.draw_indices(3, 0, 0, 4096, 512)
    assert not np.array_equal(a, oracle.draw_indices(3, 1, 0, 4096, 512))
    assert not np.array_equal(a, oracle.draw_indices(3, 0, 1, 4096, 512))
    assert not np.array_equal(a, oracle.draw_indices(4, 0, 0, 4096, 512))
    assert np.array_equal(a, oracle.draw_indices(3, 0, 0, 4096, 512))
    # phases and indices come from different streams of the same counter range
    w0 = draws._words(3, np.arange(8), 0, 0, 0)
    w1 = draws._words(3, np.arange(8), 0, 1, 0)
    assert not np.array_equal(w0, w1)


def test_seed_splits_into_key_words():
    """The 64-bit seed is the key (low word, high word)."""
    seed = (0x299F31D0 << 32) | 0xA4093822
    w = draws._words(seed, np.array([0x243F6A88]), 0x85A308D3, 0x13198A2E, 0x03707344)[0]
    assert tuple(int(v) for v in w) == (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)
