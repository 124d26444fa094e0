"""The classical minimal-norm solver and an extended-precision refined variant.

TEST INFRASTRUCTURE ONLY (see the package docstring).

classical_minnorm -- the O(m^2 n) QR method the paper compares against
  (Section 1; the direct computations of Section 7): A* = Q R by Householder
  QR (LAPACK via scipy), then A = R* Q*, so p = Q u with R* u = b gives
  A p = b with p in the column span of A*, i.e. the minimal-norm solution.

refined_minnorm -- the same factors used for iterative refinement of the
  augmented system  x - A* y = 0,  A x = b  (a published technique: Bjorck's
  refinement for least-squares / minimum-norm problems), with both residuals
  accumulated in numpy longdouble (x86 80-bit, unit roundoff 5.4e-20).  Each
  correction solves the system exactly through the FP64 factors:
      dy = R^{-1} (R^{-*} g - Q* f),   dx = (I - Q Q*) f + Q R^{-*} g,
  with f = A* y - x and g = b - A x.  The fixed point is the minimal-norm
  solution of the stored A to about FP64 roundoff, even when cond(A) * u64
  is far above the target accuracy (cond(A) = 1e6 needs this for 1e-10).

Right-hand sides: b is (m,) or (k, m) with one right-hand side per row; the
returned p has the matching shape (n,) or (k, n).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _as_cols(b):
    b = np.asarray(b)
    return (b[:, None], True) if b.ndim == 1 else (b.T, False)


def _qr_of_adjoint(A):
    Q, R = sla.qr(np.asarray(A).conj().T, mode="economic")
    return Q, R


def classical_minnorm(A, b):
    """p = A^+ b via Householder QR of A* (FP64)."""
    B, single = _as_cols(b)
    Q, R = _qr_of_adjoint(A)
    U = sla.solve_triangular(R, B, trans="C", lower=False)
    P = Q @ U
    return P[:, 0] if single else P.T


def residuals_longdouble(A, x, y, b, chunk_rows: int = 256):
    """f = A* y - x and g = b - A x accumulated in longdouble, row-chunked.

    A, x, y, b are exact FP64 values promoted to longdouble before any
    product, so the only roundoff is longdouble's.  Shapes: x (n, k),
    y (m, k), b (m, k).
    """
    A = np.asarray(A)
    cplx = np.iscomplexobj(A) or np.iscomplexobj(b) or np.iscomplexobj(x)
    ld = np.clongdouble if cplx else np.longdouble
    m, n = A.shape
    k = x.shape[1]
    xl = x.astype(ld)
    yl = y.astype(ld)
    f = -xl.copy()
    g = b.astype(ld).copy()
    for r0 in range(0, m, chunk_rows):
        Al = A[r0:r0 + chunk_rows].astype(ld)
        f += Al.conj().T @ yl[r0:r0 + chunk_rows]
        g[r0:r0 + chunk_rows] -= Al @ xl
    return f, g


def refined_minnorm(A, b, steps: int = 4, tol: float = 1e-17, return_history: bool = False):
    """Minimal-norm solution refined with longdouble residuals (see module doc)."""
    A = np.asarray(A)
    B, single = _as_cols(b)
    Q, R = _qr_of_adjoint(A)
    dt = np.result_type(A, B, np.float64)
    B = B.astype(dt)
    U = sla.solve_triangular(R, B, trans="C", lower=False)
    x = Q @ U
    y = sla.solve_triangular(R, U, lower=False)
    hist = []
    for _ in range(steps):
        f, g = residuals_longdouble(A, x, y, B)
        f64 = f.astype(dt)
        g64 = g.astype(dt)
        h = sla.solve_triangular(R, g64, trans="C", lower=False)  # R^{-*} g
        Qf = Q.conj().T @ f64
        dx = f64 - Q @ Qf + Q @ h
        dy = sla.solve_triangular(R, h - Qf, lower=False)
        x = x + dx
        y = y + dy
        rel = float(np.linalg.norm(dx) / max(np.linalg.norm(x), 1e-300))
        hist.append(rel)
        if rel <= tol:
            break
    out = x[:, 0] if single else x.T
    return (out, hist) if return_history else out
