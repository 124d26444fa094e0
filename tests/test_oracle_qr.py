"""Pins for the oracle's Householder QR (Step 2's factorisation).

R is checked through properties that fix it up to diagonal phases: upper
triangular with real diagonal, R* R = S* S, Q* S = [R; 0] with Q built from
the stored reflectors, and agreement with LAPACK's R after phase
normalisation.
"""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle


def _rand(g, shape, cplx):
    if cplx:
        return g.standard_normal(shape) + 1j * g.standard_normal(shape)
    return g.standard_normal(shape)


@pytest.mark.parametrize("l,m,cplx", [(12, 5, True), (40, 16, True), (40, 16, False), (7, 7, True), (1, 1, True), (9, 1, False)])
def test_householder_properties(l, m, cplx):
    g = np.random.default_rng(l * 100 + m)
    S = _rand(g, (l, m), cplx)
    R, V, tau = oracle.householder_qr(S)
    assert R.shape == (m, m)
    assert np.allclose(np.tril(R, -1), 0)
    assert np.allclose(np.imag(np.diagonal(R)), 0)
    scale = np.linalg.norm(S) ** 2
    assert np.linalg.norm(R.conj().T @ R - S.conj().T @ S) <= 1e-14 * scale * l
    QhS = oracle.apply_qh(V, tau, S)
    assert np.allclose(QhS[:m], R, atol=1e-13 * np.linalg.norm(S))
    assert np.allclose(QhS[m:], 0, atol=1e-13 * np.linalg.norm(S))
    Rl = sla.qr(S, mode="r")[0][:m]
    assert np.allclose(oracle.normalize_r(R), oracle.normalize_r(Rl), atol=1e-12 * np.linalg.norm(S))


def test_householder_degenerate_columns():
    # first column already a positive multiple of e_1: reflector is the identity (tau = 0)
    S = np.array([[2.0, 1.0], [0.0, 3.0], [0.0, 4.0]])
    R, V, tau = oracle.householder_qr(S)
    assert tau[0] == 0 and R[0, 0] == 2.0
    assert np.isclose(abs(R[1, 1]), 5.0)
    # complex alpha with zero remainder still needs a reflector to make beta real
    Sc = np.array([[1j], [0.0]], dtype=complex)
    Rc, Vc, tc = oracle.householder_qr(Sc)
    assert tc[0] != 0 and np.isclose(abs(Rc[0, 0]), 1.0) and Rc[0, 0].imag == 0


def test_householder_longdouble():
    g = np.random.default_rng(3)
    S = (g.standard_normal((10, 4)) + 1j * g.standard_normal((10, 4))).astype(np.clongdouble)
    R, V, tau = oracle.householder_qr(S)
    assert R.dtype == np.clongdouble
    G = (R.conj().T @ R - S.conj().T @ S)
    assert float(np.max(np.abs(G))) < 1e-16


def test_normalize_r():
    R = np.array([[-2.0 + 0j, 1.0], [0, 1j]])
    Rn = oracle.normalize_r(R)
    assert np.allclose(np.diagonal(Rn), [2.0, 1.0])
    assert np.allclose(Rn.conj().T @ Rn, R.conj().T @ R)
