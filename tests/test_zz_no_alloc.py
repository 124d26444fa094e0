"""srft_sketch_noalloc, the allocation-free form of srft_sketch, through the C
ABI: on two calls in a row (the second with a smaller input) and on every
path of the sketch (the one-workgroup transform, the kept-outputs-only
four-step with partial sums, the full four-step chunked through the static
work area), its S equals srft_sketch's to the sketch's bar (20 u log2 N
relative per column, the bar both meet against the oracle), the library's
workspace does not grow during the call, and N beyond the static array's
limit is refused with -7."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import say, to_dev, to_np

pytestmark = pytest.mark.gpu

U = {"complex128": 1.11e-16, "complex64": 5.96e-8, "float64": 1.11e-16, "float32": 5.96e-8}


def _problem(dtype, m, n, seed):
    rng = np.random.default_rng(seed)
    if dtype.startswith("complex"):
        A = synth.complex_gaussian(rng, (m, n))
    else:
        A = rng.standard_normal((m, n))
    return A


def _check(dtype, m, n, l, seed):
    import torch
    from paper_0905_4745_amd import api
    N = synth.next_pow2(n)
    real = not dtype.startswith("complex")
    A = _problem(dtype, m, n, seed)
    d, idx = synth.draw_srft(N, l, seed=seed, real=real)
    At = to_dev(A).to(getattr(torch, dtype))
    S_ref = to_np(api.srft_sketch(At, d, idx, N))
    out = torch.empty((m, l), dtype=At.dtype, device=At.device)
    torch.cuda.synchronize()
    before = api.workspace_bytes()
    S_na = to_np(api.srft_sketch_noalloc(At, d, idx, N, S=out))
    assert api.workspace_bytes() == before
    tol = 20 * U[dtype] * np.log2(N)
    col = np.linalg.norm(S_na - S_ref, axis=0) / np.maximum(np.linalg.norm(S_ref, axis=0), 1e-300)
    say(f"  {dtype} m={m} n={n} N={N} l={l}: max column rel diff vs srft_sketch {col.max():.1e} (bar {tol:.1e}), "
        f"bitwise equal: {np.array_equal(S_na, S_ref)}")
    assert col.max() <= tol
    # a few columns against the oracle too
    A64 = A if not dtype.endswith("32") and dtype != "complex64" else np.asarray(to_np(At), dtype=A.dtype)
    rows = [0, m // 2, m - 1]
    S_o = (oracle.sketch_real if real else oracle.sketch)(A64[rows], d, idx, N)
    err = np.linalg.norm(S_na[:, rows] - S_o, axis=0) / np.linalg.norm(S_o, axis=0)
    assert err.max() <= tol


def test_noalloc_sketch_two_calls_second_smaller():
    # first call: kept-outputs-only four-step with partial sums in the static array
    _check("complex128", 300, 50000, 1200, 61)
    # second call, smaller: the one-workgroup transform (twiddle table rebuilt)
    _check("complex128", 40, 3000, 160, 62)


@pytest.mark.parametrize("dtype,m,n,l", [("complex64", 600, 40000, 2400), ("float64", 100, 20000, 400),
                                         ("float32", 33, 65536, 4000)])
def test_noalloc_sketch_paths(dtype, m, n, l):
    _check(dtype, m, n, l, 63)


def test_noalloc_sketch_limit():
    import torch
    from paper_0905_4745_amd import api
    A = torch.zeros((4, 70000), dtype=torch.complex128, device="cuda")
    d, idx = synth.draw_srft(131072, 16, seed=1)
    with pytest.raises(api.MinnormError) as e:
        api.srft_sketch_noalloc(A, d, idx, 131072)
    assert e.value.status == -7
