"""The one-read fused pass for m above 512 (column-major copy of the bulk
matrix written by a tiled transpose on the first pass of each solve, then
k_gram_tall): every shape code and several workgroup counts give a solution
that meets Theorem 5.4's guarantee against the classical FP64 oracle, on
ragged shapes (m not a multiple of the copy's 256-row padding, n not a
multiple of any column group) and on every storage type the solver takes."""

import json

import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu

# (m, n, data): complex128 plain; complex128 with a complex64 copy (mixed);
# float64 plain; float32 problem (single-precision bulk, FP64 refinement)
CASES = [(640, 6001, "c128"), (1500, 6001, "c128+c64"), (1100, 4099, "f64"), (2048, 8200, "f32")]


def _problem(m, n, data, seed):
    if data in ("c128", "c128+c64"):
        return synth.make_svd(m, n, 1e3, seed=seed)[:2]
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    if data == "f32":
        A = A.astype(np.float32).astype(np.float64)  # the stored float32 values are the problem
    return A, rng.standard_normal(m)


@pytest.mark.parametrize("m,n,data", CASES)
def test_every_tall_plan_meets_eps(m, n, data, tmp_path):
    import torch
    from paper_0905_4745_amd import api
    say(f"tall pass {data} m={m} n={n}")
    A, b = _problem(m, n, data, seed=m)
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    d, idx = synth.draw_srft(N, l, seed=m + 1, real=data in ("f64", "f32"))
    p = oracle.classical_minnorm(A, b)
    At = to_dev(A)
    kw = {}
    if data == "c128+c64":
        kw["A_lo"] = At.to(torch.complex64)
        bulk, key_dt = "c64", 1
    elif data == "f32":
        At = At.to(torch.float32)
        bulk, key_dt = "f32", 3
    else:
        bulk, key_dt = data, 0 if data == "c128" else 2
    path = tmp_path / "plans.json"
    worst = 0.0
    for code in range(4):
        for wg in (256, 1024):
            plan = wg | 0x80000 | (code << 20)
            path.write_text(json.dumps({"plans": {f"gram/{key_dt}/{m}/{n}/0": plan}}))
            api.plans_load(str(path))
            x, info = api.minnorm_solve(At, to_dev(b), 1e-10, d, idx, N, **kw)
            err = rel(to_np(x), p)
            say(f"  bulk {bulk} plan code {code} wg {wg}: status {info['status']} iters {info['iters']} "
                f"refine {info['refine_steps']} err {err:.2e}")
            assert info["status"] == 0
            assert err <= 1e-10, (code, wg)
            worst = max(worst, err)
    say(f"  worst {worst:.2e}")


@pytest.mark.parametrize("data", ["c128", "c128+c64"])
def test_refined_tall_solve_with_early_copies(data):
    """A refined solve at m above 512 writes its column-major copies on a
    side stream while Step 2 runs (one copy when the bulk is the problem
    matrix itself, two with a separate complex64 bulk); the solve still meets
    eps against the oracle's refined solution at cond 1e6, twice in a row on
    one handle (the second call rewrites the copies after the first call's
    passes)."""
    import torch
    from paper_0905_4745_amd import api
    m, n = 1024, 6000
    A, b, _ = synth.make_svd(m, n, 1e6, seed=17)
    N = synth.next_pow2(n)
    d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=18)
    p = oracle.refined_minnorm(A, b)
    At = to_dev(A)
    if data == "c128":
        kw = {"opts": api.SolveOptions(refine=1)}
    else:
        kw = {"A_lo": At.to(torch.complex64)}
    for rep in range(2):
        x, info = api.minnorm_solve(At, to_dev(b), 1e-10, d, idx, N, **kw)
        err = rel(to_np(x), p)
        say(f"  {data} call {rep}: status {info['status']} iters {info['iters']} refine {info['refine_steps']} "
            f"err {err:.2e}")
        assert info["status"] == 0
        assert err <= 1e-10
