"""Pins for the oracle's transforms (Section 3) against the formulas themselves.

The dense matrices are built entry by entry from eq. (DFT) and the Hartley
kernel, so they are independent of numpy's FFT; closed forms and unitarity
fix the conventions (sign of the exponent, 1/sqrt(N) scaling, conjugation).
"""

import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("N", [1, 2, 8, 16, 64, 3, 12, 20, 768])
def test_dft_unitary(N):
    F = oracle.dft_matrix(N)
    assert np.allclose(F @ F.conj().T, np.eye(N), atol=1e-13)


@pytest.mark.parametrize("N", [2, 8, 32, 64, 3, 12, 20, 768])
def test_fft_matches_dense_dft(N):
    g = np.random.default_rng(N)
    X = g.standard_normal((5, N)) + 1j * g.standard_normal((5, N))
    F = oracle.dft_matrix(N)
    assert np.allclose(oracle.fft_ortho(X, axis=1), X @ F.T, atol=1e-13)


@pytest.mark.parametrize("N", [16, 12, 768])
def test_dft_closed_forms(N):
    j = np.arange(N)
    # impulse at 0 -> constant 1/sqrt(N)
    e0 = np.zeros(N, complex); e0[0] = 1
    assert np.allclose(oracle.fft_ortho(e0), np.full(N, 1 / np.sqrt(N)))
    # impulse at k0 -> exp(-2 pi i j k0 / N)/sqrt(N)
    k0 = 3
    ek = np.zeros(N, complex); ek[k0] = 1
    assert np.allclose(oracle.fft_ortho(ek), np.exp(-2j * np.pi * j * k0 / N) / np.sqrt(N))
    # pure tone exp(+2 pi i k0 j / N) -> sqrt(N) at index k0
    tone = np.exp(2j * np.pi * k0 * j / N)
    out = oracle.fft_ortho(tone)
    ref = np.zeros(N, complex); ref[k0] = np.sqrt(N)
    assert np.allclose(out, ref, atol=1e-13)


@pytest.mark.parametrize("N", [2, 8, 32, 3, 12, 20])
def test_dht_orthonormal_symmetric(N):
    H = oracle.dht_matrix(N)
    assert np.allclose(H, H.T)
    assert np.allclose(H @ H, np.eye(N), atol=1e-13)
    x = np.random.default_rng(1).standard_normal(N)
    assert np.allclose(oracle.dht_ortho(x), H @ x, atol=1e-13)
    e0 = np.zeros(N); e0[0] = 1
    assert np.allclose(oracle.dht_ortho(e0), np.full(N, 1 / np.sqrt(N)))


@pytest.mark.parametrize("N,l", [(8, 3), (16, 16), (64, 20)])
def test_srft_rows_orthonormal(N, l):
    d, idx = synth.draw_srft(N, l, seed=N + l)
    T = oracle.srft_matrix(N, d, idx)
    assert T.shape == (l, N)
    assert np.allclose(T @ T.conj().T, np.eye(l), atol=1e-13)
    v = np.random.default_rng(2).standard_normal(N) + 0j
    assert np.linalg.norm(T @ v) <= np.linalg.norm(v) * (1 + 1e-14)
    dr, idxr = synth.draw_srft(N, l, seed=N + l, real=True)
    Tr = oracle.srft_real_matrix(N, dr, idxr)
    assert np.allclose(Tr @ Tr.T, np.eye(l), atol=1e-13)


@pytest.mark.parametrize("m,n,N,l", [(3, 8, 8, 6), (4, 13, 16, 12), (5, 40, 64, 20), (1, 2, 2, 2),
                                     (4, 11, 12, 7), (3, 700, 768, 50)])
def test_sketch_equals_dense_T_times_Astar(m, n, N, l):
    g = np.random.default_rng(m * n)
    A = g.standard_normal((m, n)) + 1j * g.standard_normal((m, n))
    d, idx = synth.draw_srft(N, l, seed=7)
    T = oracle.srft_matrix(N, d, idx)
    Astar_pad = np.zeros((N, m), complex)
    Astar_pad[:n, :] = A.conj().T
    S = oracle.sketch(A, d, idx, N)
    assert S.shape == (l, m)
    assert np.allclose(S, T @ Astar_pad, atol=1e-13)


@pytest.mark.parametrize("m,n,N,l", [(3, 8, 8, 6), (4, 13, 16, 12), (5, 40, 64, 20), (4, 11, 12, 7)])
def test_sketch_real_equals_dense(m, n, N, l):
    g = np.random.default_rng(m + n)
    A = g.standard_normal((m, n))
    d, idx = synth.draw_srft(N, l, seed=9, real=True)
    T = oracle.srft_real_matrix(N, d, idx)
    At_pad = np.zeros((N, m))
    At_pad[:n, :] = A.T
    S = oracle.sketch_real(A, d, idx, N)
    assert S.dtype == np.float64
    assert np.allclose(S, T @ At_pad, atol=1e-13)


def test_srft_adjoint_equals_dense():
    N, l = 32, 12
    d, idx = synth.draw_srft(N, l, seed=3)
    T = oracle.srft_matrix(N, d, idx)
    z = np.random.default_rng(0).standard_normal(l) + 1j * np.random.default_rng(1).standard_normal(l)
    assert np.allclose(oracle.srft_adjoint(z, d, idx, N), T.conj().T @ z, atol=1e-13)
    dr, idxr = synth.draw_srft(N, l, seed=3, real=True)
    Tr = oracle.srft_real_matrix(N, dr, idxr)
    zr = np.random.default_rng(5).standard_normal(l)
    assert np.allclose(oracle.srft_real_adjoint(zr, dr, idxr, N), Tr.T @ zr, atol=1e-13)


def test_rokhlin_h_unitary_and_apply():
    N = 12
    g = np.random.default_rng(4)
    th, tht = g.uniform(0, 2 * np.pi, N - 1), g.uniform(0, 2 * np.pi, N - 1)
    pe, pet = g.permutation(N), g.permutation(N)
    ze = np.exp(2j * np.pi * g.random(N))
    zet = np.exp(2j * np.pi * g.random(N))
    H = oracle.rokhlin_h_matrix(th, pe, ze, tht, pet, zet)
    assert np.allclose(H @ H.conj().T, np.eye(N), atol=1e-13)
    v = g.standard_normal(N) + 1j * g.standard_normal(N)
    assert np.allclose(oracle.rokhlin_h_apply(v, th, pe, ze, tht, pet, zet), H @ v, atol=1e-13)
    # a single rotation: R_1 with angle t acts on the first two coordinates
    t = 0.3
    G = oracle.givens_chain_matrix(np.array([t]))
    assert np.allclose(G, [[np.cos(t), np.sin(t)], [-np.sin(t), np.cos(t)]])


def test_lemma_3_1_least_singular_value():
    """Lemma 3.1 under its own hypothesis, with the full T = S F D H.

    alpha = 4, beta = 4, m = 2: eq. (weak) needs l >= alpha^2 beta m^2 /
    (alpha - 1)^2 = 28.4, so l = 29 < n = 128.  The lemma then bounds the
    probability that sigma_min(T Q) < sqrt(l / (alpha n)) by 1/beta.
    """
    m, N, l, alpha, beta = 2, 128, 29, 4.0, 4.0
    assert l >= alpha ** 2 * beta * m ** 2 / (alpha - 1) ** 2
    g = np.random.default_rng(11)
    Q = np.linalg.qr(g.standard_normal((N, m)) + 1j * g.standard_normal((N, m)))[0]
    trials, fails = 200, 0
    for seed in range(trials):
        d, idx = synth.draw_srft(N, l, seed=1000 + seed)
        h = np.random.default_rng(5000 + seed)
        H = oracle.rokhlin_h_matrix(h.uniform(0, 2 * np.pi, N - 1), h.permutation(N),
                                    np.exp(2j * np.pi * h.random(N)),
                                    h.uniform(0, 2 * np.pi, N - 1), h.permutation(N),
                                    np.exp(2j * np.pi * h.random(N)))
        TQ = oracle.srft_matrix(N, d, idx) @ (H @ Q)
        fails += np.linalg.svd(TQ, compute_uv=False)[-1] < np.sqrt(l / (alpha * N))
    assert fails / trials <= 1.0 / beta


@pytest.mark.parametrize("N", [12, 20, 768])
def test_dft_four_step_identity_any_length(N):
    """For N = N1 N2 (N1 any integer), the kept-outputs-only form's identity
    V[k] = sum_{n1} W_N^{n1 k} Z_{n1}[k mod N2], Z_{n1} = DFT_{N2} of
    v[n1 + N1 n2] (eq. DFT regrouped), holds for the oracle's transform."""
    N2 = 4 if N in (12, 20) else 256
    N1 = N // N2
    g = np.random.default_rng(N)
    v = g.standard_normal(N) + 1j * g.standard_normal(N)
    V = oracle.fft_ortho(v) * np.sqrt(N)
    Z = np.array([np.fft.fft(v[n1::N1]) for n1 in range(N1)])
    k = np.arange(N)
    W = np.exp(-2j * np.pi * np.outer(np.arange(N1), k) / N)
    Vk = np.sum(W * Z[:, k % N2], axis=0)
    assert np.allclose(Vk, V, atol=1e-10 * np.abs(V).max())
