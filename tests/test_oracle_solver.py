"""Pins for the oracle's solvers: classical, refined and randomized.

The minimal-norm solution p = A^+ b has plain definitions that do not go
through the oracle's code: the SVD pseudo-inverse, the normal-equations
formula A* (A A*)^{-1} b, closed forms for one row and for orthonormal rows,
and the paper's own known-answer construction (Section 7).  The randomized
oracle is further checked against the statements of Lemmas 5.1-5.3 and
Theorem 5.4.
"""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.mark.parametrize("m,n", [(3, 7), (8, 40), (16, 17)])
def test_classical_vs_pinv_and_normal_equations(m, n):
    A, b = synth.make_gaussian(m, n, seed=m + n)
    p = oracle.classical_minnorm(A, b)
    assert _rel(p, np.linalg.pinv(A) @ b) < 1e-12
    assert _rel(p, A.conj().T @ np.linalg.solve(A @ A.conj().T, b)) < 1e-12
    assert _rel(A @ p, b) < 1e-13


def test_classical_multi_rhs_and_real():
    A, B = synth.make_gaussian(6, 30, seed=3, nrhs=4)
    P = oracle.classical_minnorm(A, B)
    assert P.shape == (4, 30)
    for k in range(4):
        assert _rel(P[k], np.linalg.pinv(A) @ B[k]) < 1e-12
    Ar, br = synth.make_gaussian(6, 30, seed=4, complex_=False)
    pr = oracle.classical_minnorm(Ar, br)
    assert pr.dtype == np.float64 and _rel(pr, np.linalg.pinv(Ar) @ br) < 1e-12


def test_closed_forms():
    g = np.random.default_rng(0)
    a = g.standard_normal((1, 9)) + 1j * g.standard_normal((1, 9))
    b = np.array([2.0 - 1.0j])
    p = oracle.classical_minnorm(a, b)
    assert _rel(p, a[0].conj() * b[0] / np.vdot(a[0], a[0]).real) < 1e-14
    # orthonormal rows: A A* = I, so p = A* b
    Q = np.linalg.qr(g.standard_normal((20, 5)) + 1j * g.standard_normal((20, 5)))[0]
    A = Q.conj().T
    b = g.standard_normal(5) + 1j * g.standard_normal(5)
    assert _rel(oracle.classical_minnorm(A, b), A.conj().T @ b) < 1e-14
    d, idx = synth.draw_srft(32, 20, seed=1)
    o = oracle.randomized_minnorm(A, b, 1e-12, d, idx, 32)
    assert _rel(o["x"], A.conj().T @ b) < 1e-12


def test_known_answer_section7():
    A, b, p, sigma = synth.make_known_answer(32, 512, seed=5, kappa=1e3)
    assert abs(sigma[0] / sigma[-1] - 1e3) < 1e-9
    assert _rel(oracle.classical_minnorm(A, b), p) < 1e3 * 1e-14
    assert _rel(oracle.refined_minnorm(A, b), p) < 1e3 * 1e-14


def _longdouble_minnorm(A, b):
    """Householder QR of A* carried out entirely in clongdouble (no LAPACK)."""
    Ah = np.asarray(A).conj().T.astype(np.clongdouble)
    n, m = Ah.shape
    R, V, tau = oracle.householder_qr(Ah)
    # R* u = b by forward substitution in longdouble
    bl = np.asarray(b).astype(np.clongdouble)
    u = np.zeros(m, dtype=np.clongdouble)
    Rh = R.conj().T
    for i in range(m):
        u[i] = (bl[i] - Rh[i, :i] @ u[:i]) / Rh[i, i]
    # p = Q [u; 0] = H_1 ... H_m [u; 0]
    x = np.zeros(n, dtype=np.clongdouble)
    x[:m] = u
    for j in range(m - 1, -1, -1):
        v = V[j:, j]
        x[j:] -= tau[j] * v * (v.conj() @ x[j:])
    return x


@pytest.mark.parametrize("kappa,bound", [(1e4, 2e-15), (1e6, 1e-12)])
def test_refined_reaches_fp64_accuracy(kappa, bound):
    """Plain FP64 QR loses about log10(kappa) digits; the refined solver must not.

    The reference is Householder QR carried out wholly in longdouble, whose own
    forward error is about kappa * 5.4e-20 times a modest dimension factor, so
    the bound at kappa = 1e6 is set well above that (and still 100 times below
    the 1e-10 parity bar the refined oracle serves).
    """
    A, b, _ = synth.make_svd(24, 256, kappa, seed=8)
    p_ld = _longdouble_minnorm(A, b)
    p_ref = oracle.refined_minnorm(A, b)
    err_ref = float(np.linalg.norm((p_ref.astype(np.clongdouble) - p_ld)) / np.linalg.norm(p_ld))
    err_cls = float(np.linalg.norm((oracle.classical_minnorm(A, b).astype(np.clongdouble) - p_ld))
                    / np.linalg.norm(p_ld))
    assert err_ref < bound
    assert err_cls > 10 * err_ref


def test_longdouble_residuals_exact_on_integers():
    A = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    x = np.array([[1.0], [1.0], [1.0]])
    y = np.array([[1.0], [2.0]])
    b = np.array([[6.0], [15.0]])
    f, g = oracle.residuals_longdouble(A, x, y, b)
    assert np.all(f.astype(float)[:, 0] == A.T @ y[:, 0] - x[:, 0])
    assert np.all(g.astype(float) == 0)


@pytest.mark.parametrize("rule", ["P", "R"])
def test_randomized_theorem_5_4(rule):
    A, b, _ = synth.make_svd(16, 200, 1e3, seed=21)
    N = synth.next_pow2(200)
    l = synth.sketch_width(16, N)
    p = oracle.refined_minnorm(A, b)
    for seed in range(20):
        d, idx = synth.draw_srft(N, l, seed=500 + seed)
        for eps in (1e-4, 1e-8):
            o = oracle.randomized_minnorm(A, b, eps, d, idx, N, rule=rule, with_steps23=False)
            assert o["info"]["converged"]
            assert _rel(o["x"], p) <= eps


def test_randomized_lemmas_5_1_and_5_2():
    m, n = 12, 100
    N = synth.next_pow2(n)
    l = 4 * m
    A, b = synth.make_gaussian(m, n, seed=2)
    p = oracle.classical_minnorm(A, b)
    worst_ratio = 0.0
    for seed in range(60):
        d, idx = synth.draw_srft(N, l, seed=seed)
        o = oracle.randomized_minnorm(A, b, 1e-6, d, idx, N)
        S, z, c = o["S"], o["z"], o["c"]
        # z solves S* z = b and lies in range(S)
        assert _rel(S.conj().T @ z, b) < 1e-12
        w = np.linalg.lstsq(S, z, rcond=None)[0]
        assert np.linalg.norm(S @ w - z) < 1e-12 * np.linalg.norm(z)
        # ||z|| = ||c|| (columns of T* orthonormal) and A c = b (Lemma 5.1, eq. easy)
        assert abs(np.linalg.norm(z) - np.linalg.norm(c)) < 1e-12 * np.linalg.norm(z)
        assert _rel(A @ c[:n], b) < 1e-12
        # the projection of c onto range(A*) is p
        Q = np.linalg.qr(A.conj().T)[0]
        assert _rel(Q @ (Q.conj().T @ c[:n]), p) < 1e-12
        worst_ratio = max(worst_ratio, np.linalg.norm(c) / np.linalg.norm(p))
    # Lemma 5.2 (eq. energy) with alpha = 4
    assert worst_ratio <= np.sqrt(4.0 * N / l)


def test_pcg_certificate_and_monotone_error():
    A, b, _ = synth.make_svd(20, 300, 1e2, seed=4)
    N = synth.next_pow2(300)
    d, idx = synth.draw_srft(N, 80, seed=6)
    p = oracle.classical_minnorm(A, b)
    o = oracle.randomized_minnorm(A, b, 1e-10, d, idx, N, p_exact=p, with_steps23=False)
    err = np.array(o["info"]["err_hist"])
    cert = np.array(o["info"]["cert_hist"])
    # ||x_k - p|| <= sqrt(rho_k), up to roundoff at the end
    assert np.all(err <= cert * (1 + 1e-8) + 1e-13 * np.linalg.norm(p))
    # CG minimises the energy norm, here ||x_k - p||: non-increasing
    assert np.all(np.diff(err) <= 1e-12 * np.linalg.norm(p))


def test_l_equals_N_converges_immediately():
    """l = N: T is unitary, R* R = A A*, the preconditioner is exact."""
    A, b = synth.make_gaussian(8, 30, seed=9)
    N = 32
    d, idx = synth.draw_srft(N, N, seed=2)
    o = oracle.randomized_minnorm(A, b, 1e-12, d, idx, N)
    assert o["info"]["iters"] <= 2
    assert _rel(o["x"], oracle.classical_minnorm(A, b)) < 1e-12
    assert _rel(o["c"][:30], oracle.classical_minnorm(A, b)) < 1e-12


def test_zero_padding_is_exact_and_zero_rhs():
    A, b = synth.make_gaussian(10, 45, seed=12)
    N = synth.next_pow2(45)
    d, idx = synth.draw_srft(N, 40, seed=3)
    o = oracle.randomized_minnorm(A, b, 1e-12, d, idx, N)
    assert _rel(o["x"], oracle.classical_minnorm(A, b)) < 1e-12
    o0 = oracle.randomized_minnorm(A, np.zeros(10, complex), 1e-12, d, idx, N)
    assert o0["info"]["iters"] == 0 and np.all(o0["x"] == 0)


def test_randomized_real_variant():
    shapes = synth.make_batch_shapes(3, seed=1, m_lo=8, m_hi=24, n_lo=100, n_hi=400)
    for k, (A, b) in enumerate(synth.make_batch(shapes, seed=2, kappa=1e4)):
        m, n = A.shape
        N = synth.next_pow2(n)
        d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=k, real=True)
        o = oracle.randomized_minnorm(A, b, 1e-10, d, idx, N, real=True)
        assert o["x"].dtype == np.float64
        assert _rel(o["x"], oracle.refined_minnorm(A, b)) < 1e-10
        # A c = b (Lemma 5.1) to roundoff in forming A c, which scales with ||A|| ||c||
        res = np.linalg.norm(A @ o["c"][:n] - b)
        assert res <= 1e-12 * np.linalg.norm(A, 2) * np.linalg.norm(o["c"])
