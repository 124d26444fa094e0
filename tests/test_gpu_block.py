"""GPU parity of the multi-right-hand-side block form against the CPU oracle.

The block form runs k CG recurrences together (split-BF16 matrix-core
products for both passes over A, FP64 refinement and certificate per column).
Every column must meet the method's guarantee ||x_j - p_j|| <= eps ||p_j||
(Theorem 5.4) against the longdouble-refined oracle of the same data, and the
per-column report must account for every column.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _draw(m, n, seed, real=False):
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    d, idx = synth.draw_srft(N, l, seed=seed, real=real)
    return N, d, idx


def _check_cols(X, P, eps):
    errs = [rel(X[k], P[k]) for k in range(P.shape[0])]
    say(f"  max col err {max(errs):.2e}")
    assert max(errs) <= eps
    return errs


@pytest.mark.parametrize("m,n,k,seed", [(128, 4096, 8, 1), (100, 3001, 5, 2), (300, 8192, 64, 3), (16, 700, 2, 4)])
def test_block_c64_row_scaled(m, n, k, seed):
    """complex64 data with rows scaled by 10^U(-2,2) (the multi-RHS workload's recipe)."""
    from paper_0905_4745_amd import api
    say(f"block c64 m={m} n={n} k={k}")
    A, B = synth.make_row_scaled(m, n, k, seed=seed)
    N, d, idx = _draw(m, n, seed)
    X, info = api.minnorm_solve(to_dev(A), to_dev(B), 1e-10, d, idx, N)
    say(f"  iters {info['iters']} refine {info['refine_steps']} cert {info['cert_rel']:.2e}")
    assert info["status"] == 0 and info["nrhs_done"] == k
    P = oracle.refined_minnorm(A.astype(np.complex128), B)
    _check_cols(to_np(X), P, 1e-10)


def test_block_real_f32_and_zero_column():
    from paper_0905_4745_amd import api
    A, B, _ = synth.make_svd(90, 2500, 1e3, seed=5, complex_=False, nrhs=4)
    A32 = A.astype(np.float32)
    B[2] = 0.0
    N, d, idx = _draw(90, 2500, 5, real=True)
    X, info = api.minnorm_solve(to_dev(A32), to_dev(B), 1e-10, d, idx, N)
    assert info["status"] == 0 and info["nrhs_done"] == 4
    X = to_np(X)
    assert np.all(X[2] == 0)
    P = oracle.refined_minnorm(A32.astype(np.float64), B)
    for j in (0, 1, 3):
        assert rel(X[j], P[j]) <= 1e-10


def test_block_mixed_c128_with_c64_copy():
    import torch
    from paper_0905_4745_amd import api
    A, B, _ = synth.make_svd(64, 3000, 1e3, seed=6, nrhs=6)
    N, d, idx = _draw(64, 3000, 6)
    At = to_dev(A)
    X, info = api.minnorm_solve(At, to_dev(B), 1e-10, d, idx, N, A_lo=At.to(torch.complex64))
    assert info["status"] == 0 and info["nrhs_done"] == 6
    _check_cols(to_np(X), oracle.refined_minnorm(A, B), 1e-10)


def test_block_forced_on_plain_c128_matches_one_at_a_time():
    from paper_0905_4745_amd import api
    A, B = synth.make_gaussian(48, 1500, seed=7, nrhs=3)
    N, d, idx = _draw(48, 1500, 7)
    Xb, ib = api.minnorm_solve(to_dev(A), to_dev(B), 1e-11, d, idx, N, opts=api.SolveOptions(block=2))
    X1, i1 = api.minnorm_solve(to_dev(A), to_dev(B), 1e-11, d, idx, N, opts=api.SolveOptions(block=1))
    P = oracle.classical_minnorm(A, B)
    assert ib["status"] == 0 and i1["status"] == 0
    _check_cols(to_np(Xb), P, 1e-11)
    _check_cols(to_np(X1), P, 1e-11)


def test_block_single_column_forced():
    from paper_0905_4745_amd import api
    A, B = synth.make_row_scaled(40, 1200, 1, seed=8)
    N, d, idx = _draw(40, 1200, 8)
    X, info = api.minnorm_solve(to_dev(A), to_dev(B), 1e-10, d, idx, N, opts=api.SolveOptions(block=2))
    assert info["status"] == 0
    P = oracle.refined_minnorm(A.astype(np.complex128), B)
    assert rel(to_np(X)[0], P[0]) <= 1e-10
