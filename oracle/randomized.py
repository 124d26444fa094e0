"""The randomized algorithm of Section 4, all five steps, on the CPU in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Given A (m x n, full rank, m < n), b, eps and the SRFT's random quantities
(d, idx) of length N >= n (N a power of two, rows zero-padded):

  Step 1  S = T A*                      (eq. randmat)        -> transforms.sketch
  Step 2  z = minimal-norm solution of S* z = b (eq. lineq) via S = Q_S R:
          z = Q_S R^{-*} b = S R^{-1} R^{-*} b               -> householder_qr
  Step 3  c = T* z                      (eq. nonminnorm)     -> transforms.srft_adjoint
  Step 4  y minimising ||A* y - c||^2 to relative precision
          eps^2 l / (alpha N)           (eq. overdet)        -> pcg.pcg_minnorm
  Step 5  x = A* y                      (eq. output)

z and c are not needed by Step 4 in the reading taken (its normal equations
have right-hand side A c = b); they are returned so tests can check the
statements of Lemmas 5.1 and 5.2 on them.
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from .transforms import sketch, sketch_real, srft_adjoint, srft_real_adjoint
from .householder import householder_qr
from .pcg import pcg_minnorm


def randomized_minnorm(A, b, eps: float, d, idx, N: int | None = None, alpha: float = 4.0,
                       rule: str = "P", max_iter: int = 500, real: bool = False,
                       p_exact=None, with_steps23: bool = True):
    A = np.asarray(A)
    b = np.asarray(b)
    m, n = A.shape
    N = n if N is None else int(N)
    l = len(idx)
    # Step 1
    S = sketch_real(A, d, idx, N) if real else sketch(A, d, idx, N)
    # Step 2 (its QR; R is kept as the preconditioner)
    R, V, tau = householder_qr(S)
    out = dict(S=S, R=R, l=l, N=N)
    if with_steps23:
        g = solve_triangular(R, b, trans="C", lower=False)      # R^{-*} b
        z = S @ solve_triangular(R, g, lower=False)             # Q_S R^{-*} b
        # Step 3
        c = srft_real_adjoint(z, d, idx, N) if real else srft_adjoint(z, d, idx, N)
        out.update(z=z, c=c)
    # Step 4
    y, info = pcg_minnorm(A, b, R, eps, l, N, alpha=alpha, rule=rule, max_iter=max_iter,
                          p_exact=p_exact)
    # Step 5
    x = A.conj().T @ y
    out.update(x=x, y=y, info=info)
    return out
