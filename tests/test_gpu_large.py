"""GPU parity of the large workloads' own code paths against the CPU oracle.

The 2048 x 262144 mixed-precision workload (cond 1e6, complex64 bulk, FP64
refinement) and the 4096 x 131072 several-right-hand-side workload take code
paths that the small parity tests do not reach: m > 512 (no one-read fused
pass unless the column-major form takes it), single-precision passes
accumulated in FP64 once cond(A) passes 3e4, compensated (double-double)
refinement residuals once cond(A) u64 nears eps, the l > 2048 sketch, and the
block form at m in the thousands.  These tests run those paths at the largest
sizes the oracle solves in seconds to a few minutes on the host and compare
every result with it:

* single system: ||x - p|| <= eps ||p|| (Theorem 5.4) against the longdouble-
  refined oracle, eps = 1e-10;
* block form: the same per column against the classical FP64 oracle (cond(A)
  about 1e4 here, so its own error is near 1e-12);
* sketch: per column of S, relative error <= 20 u32 log2(N) against the
  oracle's FFT sketch with the same (d, idx).
"""

import time

import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu

U32 = 5.96e-8


def _timed(label, fn, *a, **k):
    t0 = time.perf_counter()
    out = fn(*a, **k)
    say(f"  {label}: {time.perf_counter() - t0:.1f} s")
    return out


@pytest.mark.parametrize("m,n,seed", [(640, 8192, 31), (1024, 16384, 32), (2048, 65536, 33)])
def test_mixed_cond_1e6_large_m(m, n, seed):
    """complex128 A with a complex64 copy, cond 1e6, m > 512: the mixed
    workload's passes (FP64-accumulated complex64 bulk, compensated FP64
    refinement) against the longdouble-refined oracle."""
    import torch
    from paper_0905_4745_amd import api
    say(f"mixed c128/c64 cond 1e6 m={m} n={n}: generating")
    A, b, _ = _timed("generate", synth.make_svd, m, n, 1e6, seed=seed)
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    d, idx = synth.draw_srft(N, l, seed=seed)
    At = to_dev(A)
    x, info = api.minnorm_solve(At, to_dev(b), 1e-10, d, idx, N, A_lo=At.to(torch.complex64),
                                raise_on_status=False)
    x = to_np(x)
    del At
    say(f"  gpu status {info['status']} iters {info['iters']} refine {info['refine_steps']} "
        f"cert {info['cert_rel']:.2e}; oracle")
    p = _timed("refined oracle", oracle.refined_minnorm, A, b)
    err = rel(x, p)
    say(f"  err {err:.2e}")
    assert info["status"] == 0
    assert err <= 1e-10


def test_single_precision_problem_large_m():
    """complex64 data as the problem itself (rows scaled by 10^U(-2,2)) at
    m = 1024: single-precision bulk, exact promotion to FP64 in refinement."""
    from paper_0905_4745_amd import api
    m, n = 1024, 16384
    say(f"c64 problem m={m} n={n}")
    A, B = synth.make_row_scaled(m, n, 1, seed=34)
    N = synth.next_pow2(n)
    d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=34)
    X, info = api.minnorm_solve(to_dev(A), to_dev(B), 1e-10, d, idx, N)
    p = _timed("refined oracle", oracle.refined_minnorm, A.astype(np.complex128), B[0])
    err = rel(to_np(X)[0], p)
    say(f"  status {info['status']} iters {info['iters']} err {err:.2e}")
    assert info["status"] == 0
    assert err <= 1e-10


@pytest.mark.parametrize("m,n,seed", [(2048, 16384, 35), (4096, 32768, 36)])
def test_block_form_large_m(m, n, seed):
    """The several-right-hand-side workload's recipe (complex64 rows scaled by
    10^U(-2,2), 64 right-hand sides) at m = 2048 and 4096: split-BF16 block
    products, FP64 refinement per column, against the classical oracle."""
    from paper_0905_4745_amd import api
    k = 64
    say(f"block c64 m={m} n={n} k={k}: generating")
    A, B = _timed("generate", synth.make_row_scaled, m, n, k, seed=seed)
    N = synth.next_pow2(n)
    d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=seed)
    X, info = api.minnorm_solve(to_dev(A), to_dev(B), 1e-10, d, idx, N, raise_on_status=False)
    X = to_np(X)
    say(f"  gpu status {info['status']} done {info['nrhs_done']} iters {info['iters']} "
        f"refine {info['refine_steps']} cert {info['cert_rel']:.2e}; oracle")
    P = _timed("classical oracle", oracle.classical_minnorm, A.astype(np.complex128), B)
    errs = [rel(X[j], P[j]) for j in range(k)]
    say(f"  max col err {max(errs):.2e}")
    assert info["status"] == 0 and info["nrhs_done"] == k
    assert max(errs) <= 1e-10


@pytest.mark.parametrize("m,N,l", [(6, 262144, 8192), (4, 131072, 16384), (3, 262144, 2048)])
def test_sketch_large_l_complex64(m, N, l):
    """The sketch at the mixed workload's (N = 2^18, l = 8192) and the
    several-right-hand-side workload's (N = 2^17, l = 16384) transform sizes,
    complex64, with the launch plan the solver uses by default."""
    from paper_0905_4745_amd import api
    import torch
    say(f"sketch c64 m={m} N={N} l={l}")
    g = np.random.default_rng(N + l)
    A = synth.complex_gaussian(g, (m, N - 37)).astype(np.complex64)
    d, idx = synth.draw_srft(N, l, seed=l)
    S = to_np(api.srft_sketch(to_dev(A), d, idx, N))
    ref = oracle.sketch(A.astype(np.complex128), d, idx, N)
    err = max(float(np.linalg.norm(S[:, i] - ref[:, i]) / np.linalg.norm(ref[:, i])) for i in range(m))
    say(f"  col rel err {err:.2e}")
    assert err <= 20 * U32 * np.log2(N)
