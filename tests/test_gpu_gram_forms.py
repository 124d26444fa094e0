"""Step 2's Gram matrix G = S* S (the route of the Cholesky factor R, with
R* R = S* S for the R of any QR of S; Section 4, Step 2) in its three forms:
the block GEMM's Hermitian mode (plan 0), the vector-unit product (plan 1)
and the dedicated FP64 matrix-core kernel (plan 2), each forced through a
plan file.  Every form must give the same factor -- the reported cond(R)
estimate agrees to rounding -- and a solution that meets Theorem 5.4's
guarantee against the oracle; ragged m (not a multiple of the 64- and
128-wide tiles) and split K are covered.
"""

import json

import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _solve_with_gram_plan(tmp_path, plan, A, b, eps, d, idx, N, key, A_lo=None):
    from paper_0905_4745_amd import api
    path = tmp_path / f"gram_{plan}.json"
    path.write_text(json.dumps({"format": "minnorm-plans-1", "plans": {key: plan}, "best_ms": {}}))
    api.plans_load(str(path))
    kw = {} if A_lo is None else {"A_lo": A_lo}
    return api.minnorm_solve(to_dev(A), to_dev(b), eps, d, idx, N, **kw)


@pytest.mark.parametrize("case", ["c128-100", "c128-700", "f64-300", "c64-mixed-520"])
def test_gram_forms_agree(tmp_path, case):
    import torch
    kind, *rest = case.split("-")
    mixed = "mixed" in rest
    m = int(rest[-1])
    n = 12 * m + 1000
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    real = kind == "f64"
    if real:
        rng = np.random.default_rng(m)
        A = rng.standard_normal((m, n))
        b = rng.standard_normal(m)
    else:
        A, b, _ = synth.make_svd(m, n, 1e4 if mixed else 1e3, seed=m)
    d, idx = synth.draw_srft(N, l, seed=m + 1, real=real)
    bulk = {"c128": 0, "c64": 1, "f64": 2}[kind]
    key = f"gram_s/{bulk}/{m}/{l}/0"
    A_lo = to_dev(A).to(torch.complex64) if mixed else None
    ref = oracle.refined_minnorm(A, b) if mixed else oracle.classical_minnorm(A, b)
    eps = 1e-10
    kh = {}
    for plan in (2, 1, 0):
        x, info = _solve_with_gram_plan(tmp_path, plan, A, b, eps, d, idx, N, key, A_lo)
        err = rel(to_np(x), ref)
        kh[plan] = info["kappa_hat"]
        say(f"  {case} plan {plan}: factor {info['factor']} kappa_hat {info['kappa_hat']:.6e} "
            f"iters {info['iters']} err {err:.1e}")
        assert info["status"] == 0 and info["factor"] == "gram"
        assert err <= eps
    for plan in (1, 0):
        assert abs(kh[plan] - kh[2]) <= 1e-6 * kh[2]
