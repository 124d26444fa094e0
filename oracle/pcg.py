"""Step 4 of Section 4, read as preconditioned conjugate gradients.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Step 4 asks for y minimising f(y) = ||A* y - c||^2 (eq. overdet) to relative
precision delta = eps^2 l / (alpha N), i.e. f(y) - f* <= delta f*, using the
preconditioned iteration of the cited least-squares paper with the same l.
That paper is not reproduced here; the reading taken is:

* Lemma 5.1 gives A c = b (eq. easy), so the normal equations of (overdet)
  are A A* y = b and c never has to be formed;
* the preconditioner is R* R with R the triangular factor of the Step-1
  sketch S = T A* (so Step 2's factorisation is reused);
* the iteration is textbook preconditioned CG (Hestenes-Stiefel) on
  A A* y = b from y_0 = 0, with M^{-1} r = R^{-1} (R^{-*} r).

Scalars carried by the iteration, with r_k = b - A A* y_k:
  rho_k = r_k^* M^{-1} r_k = ||R^{-*} r_k||^2,
  xi_k  = Re(y_k^* (b - r_k)) = ||A* y_k||^2 = ||x_k||^2.
Because T has orthonormal rows, ||R w|| = ||T A* w|| <= ||A* w||, so
(A A*)^{-1} <= (R* R)^{-1} and ||x_k - p||^2 = r_k^* (A A*)^{-1} r_k <= rho_k.

Stopping rules (both use only those scalars):
  "P" -- the paper's tolerance: with f(y_k) - f* = ||x_k - p||^2 (eq. first),
         f* = ||c||^2 - ||p||^2, ||c||^2 = ||z||^2 = rho_0 (eq. intermed1) and
         ||p|| <= sqrt(xi_k) + sqrt(rho_k), stop once
         rho_k <= delta * (rho_0 - (sqrt(xi_k) + sqrt(rho_k))^2),
         which implies f - f* <= delta f*.  When l = N, T is unitary, c = p
         and f* = 0, so rule "R" is used instead.
  "R" -- a direct certificate: stop once rho_k <= (eps / (1 + eps))^2 xi_k,
         which implies ||x_k - p|| <= eps ||p||.
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular


def stop_threshold(rule: str, eps: float, l: int, N: int, alpha: float,
                   rho0: float, rho: float, xi: float) -> bool:
    """True when the stopping rule is met (see the module docstring)."""
    if rule == "P" and l < N:
        delta = eps * eps * l / (alpha * N)
        gap = rho0 - (np.sqrt(xi) + np.sqrt(rho)) ** 2
        return rho <= delta * gap
    tol = eps / (1.0 + eps)
    return rho <= tol * tol * xi


def pcg_minnorm(A, b, R, eps: float, l: int, N: int, alpha: float = 4.0,
                rule: str = "P", max_iter: int = 500, p_exact=None):
    """PCG on A A* y = b preconditioned by R* R; returns (y, info).

    info holds the iteration count, rho_0, the final rho and xi, and (when
    p_exact is given) the per-iteration true errors ||A* y_k - p|| together
    with the certificates sqrt(rho_k).
    """
    A = np.asarray(A)
    b = np.asarray(b)
    Ah = A.conj().T
    y = np.zeros(A.shape[0], dtype=np.result_type(A, b))
    r = b.astype(y.dtype, copy=True)
    s = solve_triangular(R, r, trans="C", lower=False)
    z = solve_triangular(R, s, lower=False)
    rho = float(np.real(np.vdot(s, s)))
    rho0 = rho
    p = z.copy()
    hist_err, hist_cert = [], []
    iters = 0
    converged = rho0 == 0.0
    xi = 0.0
    while not converged and iters < max_iter:
        w = Ah @ p                      # A* p
        q = A @ w                       # A (A* p)
        pq = float(np.real(np.vdot(w, w)))
        a = rho / pq
        y = y + a * p
        r = r - a * q
        s = solve_triangular(R, r, trans="C", lower=False)
        z = solve_triangular(R, s, lower=False)
        rho_new = float(np.real(np.vdot(s, s)))
        xi = float(np.real(np.vdot(y, b - r)))
        iters += 1
        if p_exact is not None:
            hist_err.append(float(np.linalg.norm(Ah @ y - p_exact)))
            hist_cert.append(float(np.sqrt(max(rho_new, 0.0))))
        converged = stop_threshold(rule, eps, l, N, alpha, rho0, rho_new, xi)
        beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
    info = dict(iters=iters, rho0=rho0, rho=rho, xi=xi, converged=converged,
                err_hist=hist_err, cert_hist=hist_cert)
    return y, info
