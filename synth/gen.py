"""Seeded problem generators and random draws.

Everything here is a random draw or a test-problem construction:

* the SRFT's random quantities (Section 3): the diagonal of unit-modulus
  phases D (or random signs for real data) and the l subsample indices, drawn
  without replacement as the paper's own experiments did;
* test matrices shaped like the paper's experiments (Section 7): A = U Sigma V*
  with Haar-distributed factors and log-spaced singular values, plus the
  variants used by the benchmark workloads (plain complex Gaussian A, row-scaled
  Gaussian A with many right-hand sides, batches of uneven real systems).

The generator is numpy's PCG64 seeded explicitly, so every caller that asks for
the same (shape, seed) gets bit-identical arrays.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """Centred complex Gaussian: real and imaginary parts i.i.d. N(0, 1/2)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * np.sqrt(0.5)


def real_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.standard_normal(shape)


def haar_columns(rng: np.random.Generator, rows: int, cols: int, complex_: bool = True) -> np.ndarray:
    """rows x cols matrix with Haar-distributed orthonormal columns.

    QR of a Gaussian matrix with each column multiplied by the conjugate phase
    of the matching diagonal entry of R (Mezzadri's correction).  In exact
    arithmetic this equals Gram-Schmidt on the Gaussian columns, which is how
    the paper's experiments build U and V (Section 7).
    """
    g = complex_gaussian(rng, (rows, cols)) if complex_ else real_gaussian(rng, (rows, cols))
    q, r = np.linalg.qr(g, mode="reduced")
    dg = np.diagonal(r)
    ph = dg / np.where(np.abs(dg) == 0, 1.0, np.abs(dg))
    return q * ph[None, :]


def next_pow2(n: int) -> int:
    """Transform length N: the smallest power of two >= n (rows are zero-padded)."""
    n = int(n)
    return 1 if n <= 1 else 1 << (n - 1).bit_length()


def next_fft_len(n: int) -> int:
    """A transform length N >= n that is not restricted to powers of two: the
    power of two when n <= 512, else the smallest multiple of 256 >= n."""
    if n <= 512:
        return next_pow2(n)
    return -(-n // 256) * 256


def sketch_width(m: int, N: int, factor: int = 4) -> int:
    """l = 4m as Remarks 5.6 and the cost section advise, capped at N."""
    return int(min(factor * int(m), int(N)))


def draw_srft(N: int, l: int, seed: int, real: bool = False):
    """Random quantities of the SRFT T = S F D (Section 3).

    Returns (d, idx):
      d   -- N diagonal entries of D: uniform on the unit circle (complex128),
             or uniform random signs +-1 (float64) when real is True;
      idx -- l distinct indices in [0, N), sorted ascending, int32: the rows of
             F D that the subsampling S keeps, drawn without replacement.
    """
    if not (1 <= l <= N):
        raise ValueError(f"need 1 <= l <= N, got l={l} N={N}")
    g = rng_for(seed)
    if real:
        d = np.where(g.random(N) < 0.5, -1.0, 1.0)
    else:
        theta = g.random(N)
        d = np.exp(2j * np.pi * theta)
    idx = np.sort(g.choice(N, size=l, replace=False)).astype(np.int32)
    return d, idx


def draw_hfactor(N: int, seed: int, real: bool = False):
    """Random quantities of the SRFT's factor H = Theta Pi Z Theta~ Pi~ Z~ (Section 3).

    Returns (theta, perm, zeta, theta_t, perm_t, zeta_t): angles of the two
    rotation chains (N - 1 each, uniform on [0, 2 pi)), two uniformly random
    permutations of range(N) (int32), and two diagonals uniform on the unit
    circle (complex128), or random signs +-1 (float64) when real is True.
    """
    g = rng_for(seed)
    out = []
    for _ in range(2):
        theta = 2.0 * np.pi * g.random(N - 1)
        perm = g.permutation(N).astype(np.int32)
        zeta = np.where(g.random(N) < 0.5, -1.0, 1.0) if real else np.exp(2j * np.pi * g.random(N))
        out.append((theta, perm, zeta))
    return out[0] + out[1]


def make_gaussian(m: int, n: int, seed: int, nrhs: int = 1, complex_: bool = True):
    """A and b with i.i.d. standard Gaussian entries (complex: N(0,1/2) parts)."""
    g = rng_for(seed)
    if complex_:
        A = complex_gaussian(g, (m, n))
        b = complex_gaussian(g, (nrhs, m))
    else:
        A = real_gaussian(g, (m, n))
        b = real_gaussian(g, (nrhs, m))
    return A, (b[0] if nrhs == 1 else b)


def make_svd(m: int, n: int, kappa: float, seed: int, complex_: bool = True, nrhs: int = 1):
    """A = U diag(sigma) V* with Haar U (m x m), V (n x m), sigma log-spaced 1 -> 1/kappa.

    Returns (A, b, (U, sigma, V)).  b is Gaussian.  Shapes follow the paper's
    test matrices of Section 7; kappa sets the condition number.
    """
    g = rng_for(seed)
    U = haar_columns(g, m, m, complex_)
    V = haar_columns(g, n, m, complex_)
    sigma = np.logspace(0.0, -math.log10(kappa), m) if m > 1 else np.ones(1)
    A = (U * sigma[None, :]) @ V.conj().T
    if complex_:
        b = complex_gaussian(g, (nrhs, m))
    else:
        b = real_gaussian(g, (nrhs, m))
    return A, (b[0] if nrhs == 1 else b), (U, sigma, V)


def make_row_scaled(m: int, n: int, nrhs: int, seed: int, decades: float = 2.0):
    """Complex64 Gaussian A with rows scaled by 10^u, u ~ U(-decades, decades).

    Returns (A complex64 (m, n), B complex128 (nrhs, m)).  The complex64 values
    are the problem's data.
    """
    g = rng_for(seed)
    u = g.uniform(-decades, decades, m)
    G = complex_gaussian(g, (m, n))
    A = (G * (10.0 ** u)[:, None]).astype(np.complex64)
    B = complex_gaussian(g, (nrhs, m))
    return A, B


def make_known_answer(m: int, n: int, seed: int, kappa: float = 1e6):
    """The paper's Section 7 test problem with a known minimal-norm solution.

    A = U Sigma V*, Sigma_jj = kappa^{-(j-1)/(m-1)}, p = m^{-1/2} sum_j s_j v_j with
    random signs s_j, b = A p.  p lies in the column span of A*, so it is the
    minimal-norm solution of A p = b.  Returns (A, b, p, sigma).
    """
    g = rng_for(seed)
    U = haar_columns(g, m, m, True)
    V = haar_columns(g, n, m, True)
    j = np.arange(m)
    sigma = kappa ** (-(j / max(m - 1, 1)))
    A = (U * sigma[None, :]) @ V.conj().T
    signs = np.where(g.random(m) < 0.5, -1.0, 1.0)
    p = (V @ signs) / np.sqrt(m)
    b = A @ p
    return A, b, p, sigma


def make_batch_shapes(count: int, seed: int, m_lo: int = 32, m_hi: int = 512,
                      n_lo: int = 2048, n_hi: int = 32768):
    """(m_i, n_i) log-uniform in [m_lo, m_hi] x [n_lo, n_hi], redrawn until n_i >= 4 m_i."""
    g = rng_for(seed)
    shapes = []
    while len(shapes) < count:
        m = int(round(math.exp(g.uniform(math.log(m_lo), math.log(m_hi)))))
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        if n >= 4 * m:
            shapes.append((m, n))
    return shapes


def make_batch(shapes, seed: int, kappa: float = 1e4):
    """Real systems A_i = U_i diag(sigma) V_i^T (sigma log-spaced 1 -> 1/kappa), b_i ~ N(0,1)."""
    out = []
    for k, (m, n) in enumerate(shapes):
        A, b, _ = make_svd(m, n, kappa, seed * 100003 + k, complex_=False)
        out.append((A, b))
    return out


@dataclass(frozen=True)
class Config:
    name: str
    m: int
    n: int
    eps: float
    kind: str
    seed: int
    kappa: float = 1.0
    nrhs: int = 1
    extra: dict = field(default_factory=dict)


# The five benchmark workloads: shapes and conditioning as stated for each.
CONFIGS = {
    "c1_plain_c128": Config("c1_plain_c128", 64, 1024, 1e-12, "gaussian", 0),
    "c2_plain_c128": Config("c2_plain_c128", 512, 65536, 1e-10, "svd", 2, kappa=1e3),
    "c3_mixed_c64": Config("c3_mixed_c64", 2048, 262144, 1e-10, "svd", 3, kappa=1e6),
    "c4_multirhs_c64": Config("c4_multirhs_c64", 4096, 131072, 1e-10, "row_scaled", 4, nrhs=64),
    "c5_batched_f32": Config("c5_batched_f32", 0, 0, 1e-10, "batch", 5, kappa=1e4,
                             extra={"count": 256}),
}
