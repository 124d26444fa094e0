"""Transforms of Section 3: the DFT, the SRFT and its real analogue.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Index conventions are zero-based throughout: the paper's entry (j, k) with
j, k = 1..n is entry (j-1, k-1) here.
"""

from __future__ import annotations

import numpy as np


def dft_matrix(N: int) -> np.ndarray:
    """Dense unitary DFT of eq. (DFT): F[j, k] = N^{-1/2} exp(-2 pi i j k / N).

    Built entry by entry from the formula (exponent reduced mod N so the
    angle stays small), independent of any FFT routine.
    """
    j = np.arange(N, dtype=np.int64)
    jk = np.mod(np.outer(j, j), N).astype(np.float64)
    return np.exp(-2j * np.pi * jk / N) / np.sqrt(N)


def fft_ortho(X: np.ndarray, axis: int = -1) -> np.ndarray:
    """F applied along `axis` via numpy's FFT with the orthonormal scaling.

    numpy's forward FFT uses exp(-2 pi i j k / N); norm="ortho" divides by
    sqrt(N), which is exactly eq. (DFT).
    """
    return np.fft.fft(X, axis=axis, norm="ortho")


def dht_matrix(N: int) -> np.ndarray:
    """Dense orthonormal discrete Hartley transform: cas(2 pi j k / N) / sqrt(N).

    The real-valued counterpart of F used for real data (the paper notes that
    real versions of the scheme are similar; this is the reading taken).
    cas(t) = cos(t) + sin(t).  The matrix is real, symmetric and its own inverse.
    """
    j = np.arange(N, dtype=np.int64)
    t = 2.0 * np.pi * np.mod(np.outer(j, j), N).astype(np.float64) / N
    return (np.cos(t) + np.sin(t)) / np.sqrt(N)


def dht_ortho(X: np.ndarray, axis: int = -1) -> np.ndarray:
    """Orthonormal Hartley transform of real X via the FFT: Re(F x) - Im(F x)."""
    Y = np.fft.fft(X, axis=axis, norm="ortho")
    return Y.real - Y.imag


def srft_matrix(N: int, d: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Dense l x N SRFT with H = I: T = S F D (eqs. SRFT, SRFT2).

    Row k of T is row idx[k] of F times the diagonal D = diag(d).
    """
    F = dft_matrix(N)
    return F[np.asarray(idx), :] * np.asarray(d)[None, :]


def srft_real_matrix(N: int, d: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Real analogue: rows idx of the Hartley matrix times diag(d), d = +-1."""
    Hc = dht_matrix(N)
    return Hc[np.asarray(idx), :] * np.asarray(d)[None, :]


def _pad_rows(A: np.ndarray, N: int) -> np.ndarray:
    m, n = A.shape
    if n == N:
        return A
    out = np.zeros((m, N), dtype=A.dtype)
    out[:, :n] = A
    return out


def sketch(A: np.ndarray, d: np.ndarray, idx: np.ndarray, N: int | None = None) -> np.ndarray:
    """Step 1, eq. (randmat): S = T A*, with T = S F D of size l x N.

    A is m x n.  When n < N, A* is extended by N - n zero rows (A is padded
    with zero columns), which leaves the minimal-norm solution unchanged apart
    from N - n trailing zeros.  Column i of the l x m result is
    (F (d o conj(a_i)))[idx], a_i being row i of A.
    """
    A = np.asarray(A)
    m, n = A.shape
    N = n if N is None else int(N)
    V = _pad_rows(np.conj(A), N) * np.asarray(d)[None, :]
    W = fft_ortho(V, axis=1)
    return np.ascontiguousarray(W[:, np.asarray(idx)].T)


def sketch_real(A: np.ndarray, d: np.ndarray, idx: np.ndarray, N: int | None = None) -> np.ndarray:
    """Real analogue of Step 1: S = T A^T with T = S Hartley D, d = +-1."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    N = n if N is None else int(N)
    V = _pad_rows(A, N) * np.asarray(d)[None, :]
    W = dht_ortho(V, axis=1)
    return np.ascontiguousarray(W[:, np.asarray(idx)].T)


def srft_adjoint(z: np.ndarray, d: np.ndarray, idx: np.ndarray, N: int) -> np.ndarray:
    """Step 3, eq. (nonminnorm): c = T* z = D* F* S* z, a vector of length N.

    S* scatters z into positions idx of a zero vector; F* is the inverse
    orthonormal FFT; D* multiplies by conj(d).
    """
    y = np.zeros(N, dtype=np.complex128)
    y[np.asarray(idx)] = z
    return np.conj(np.asarray(d)) * np.fft.ifft(y, norm="ortho")


def srft_real_adjoint(z: np.ndarray, d: np.ndarray, idx: np.ndarray, N: int) -> np.ndarray:
    """Real analogue of Step 3: c = D Hartley S^T z (the Hartley matrix is symmetric)."""
    y = np.zeros(N, dtype=np.float64)
    y[np.asarray(idx)] = z
    return np.asarray(d) * dht_ortho(y)


# --- The factor H of eq. (Rokhlin_trans) -----------------------------------

def givens_chain_matrix(theta: np.ndarray) -> np.ndarray:
    """Dense Theta of eq. (big_def): the product R_1 R_2 ... R_{N-1}.

    R_k rotates coordinates (k, k+1) (zero-based k-1, k) with the 2 x 2 block
    [[cos t_k, sin t_k], [-sin t_k, cos t_k]].
    """
    N = len(theta) + 1
    M = np.eye(N)
    for k, t in enumerate(theta):
        G = np.eye(N)
        c, s = np.cos(t), np.sin(t)
        G[k, k], G[k, k + 1], G[k + 1, k], G[k + 1, k + 1] = c, s, -s, c
        M = M @ G
    return M


def _givens_chain_apply(theta: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Theta v = R_1 (R_2 ( ... (R_{N-1} v))): rightmost rotation first."""
    v = np.array(v, dtype=np.complex128, copy=True)
    for k in range(len(theta) - 1, -1, -1):
        c, s = np.cos(theta[k]), np.sin(theta[k])
        a, b = v[k], v[k + 1]
        v[k], v[k + 1] = c * a + s * b, -s * a + c * b
    return v


def rokhlin_h_apply(v, theta, perm, zeta, theta_t, perm_t, zeta_t):
    """H v with H = Theta Pi Z Theta~ Pi~ Z~ (eq. Rokhlin_trans).

    Pi is the permutation matrix with (Pi v)[j] = v[perm[j]]; Z = diag(zeta).
    """
    w = np.asarray(zeta_t) * np.asarray(v)
    w = w[np.asarray(perm_t)]
    w = _givens_chain_apply(theta_t, w)
    w = np.asarray(zeta) * w
    w = w[np.asarray(perm)]
    return _givens_chain_apply(theta, w)


def rokhlin_h_matrix(theta, perm, zeta, theta_t, perm_t, zeta_t) -> np.ndarray:
    """Dense H from its six factors, for tiny N."""
    N = len(zeta)
    P = np.eye(N)[np.asarray(perm)]
    Pt = np.eye(N)[np.asarray(perm_t)]
    return (givens_chain_matrix(theta) @ P @ np.diag(zeta)
            @ givens_chain_matrix(theta_t) @ Pt @ np.diag(zeta_t))
