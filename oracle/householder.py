"""Unblocked Householder QR: the factorisation of Step 2 (eq. lineq).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper constructs the minimal-norm z of S* z = b from a QR decomposition of
the l x m sketch S (it points to Golub and Van Loan's Algorithm 5.7.2).  The
upper-triangular factor R of that decomposition is also what the GPU path
keeps as the preconditioner of Step 4.

Convention (the usual complex Householder one): column j is reduced by
H_j = I - tau_j v_j v_j^* with v_j[0] = 1, chosen so that H_j^* x = beta e_1
with beta real and of sign opposite to Re(x[0]).  Hence diag(R) is real.
R is unique up to left multiplication by a diagonal unitary matrix; compare
two R factors only after `normalize_r`.

Works for any numpy floating dtype (float64, complex128, longdouble,
clongdouble): no LAPACK call is involved.
"""

from __future__ import annotations

import numpy as np


def _reflector(x: np.ndarray):
    """(v, tau, beta) with (I - tau v v^*)^* x = beta e_1, v[0] = 1, beta real."""
    alpha = x[0]
    rest = x[1:]
    xnorm2 = np.real(np.vdot(rest, rest)) if rest.size else x.real.dtype.type(0)
    is_cplx = np.iscomplexobj(x)
    if xnorm2 == 0 and (not is_cplx or np.imag(alpha) == 0):
        v = np.zeros_like(x)
        v[0] = 1
        return v, x.dtype.type(0), np.real(alpha)
    norm = np.sqrt(np.real(alpha) ** 2 + (np.imag(alpha) ** 2 if is_cplx else 0) + xnorm2)
    beta = -norm if np.real(alpha) >= 0 else norm
    tau = (beta - alpha) / beta
    v = x / (alpha - beta)
    v[0] = 1
    return v, tau, beta


def householder_qr(S: np.ndarray):
    """Householder QR of an l x m matrix (l >= m), column by column.

    Returns (R, V, tau):
      R   -- m x m upper triangular, real diagonal;
      V   -- l x m, column j holds v_j (unit entry at row j, zeros above);
      tau -- m scalars, S = H_1 H_2 ... H_m [R; 0] with H_j = I - tau_j v_j v_j^*.
    """
    W = np.array(S, copy=True)
    l, m = W.shape
    if l < m:
        raise ValueError("householder_qr needs rows >= columns")
    V = np.zeros_like(W)
    tau = np.zeros(m, dtype=W.dtype)
    for j in range(m):
        v, t, beta = _reflector(W[j:, j])
        V[j:, j] = v
        tau[j] = t
        if j + 1 < m:
            # apply H_j^* = I - conj(tau) v v^* to the trailing columns
            w = v.conj() @ W[j:, j + 1:]
            W[j:, j + 1:] -= np.conj(t) * np.outer(v, w)
        W[j, j] = beta
        W[j + 1:, j] = 0
    return np.triu(W[:m, :]), V, tau


def apply_qh(V: np.ndarray, tau: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Q^* X = H_m^* ... H_1^* X for the reflectors returned by householder_qr."""
    Y = np.array(X, copy=True)
    squeeze = Y.ndim == 1
    if squeeze:
        Y = Y[:, None]
    for j in range(V.shape[1]):
        v = V[j:, j]
        w = v.conj() @ Y[j:, :]
        Y[j:, :] -= np.conj(tau[j]) * np.outer(v, w)
    return Y[:, 0] if squeeze else Y


def normalize_r(R: np.ndarray) -> np.ndarray:
    """D R with D diagonal unitary chosen so diag(D R) is real and >= 0."""
    dg = np.diagonal(R)
    mag = np.abs(dg)
    ph = np.where(mag == 0, 1.0, dg / np.where(mag == 0, 1.0, mag))
    return R * np.conj(ph)[:, None]
