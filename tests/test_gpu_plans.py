"""Autotuned launch plans: chosen by timing on the live operands, kept in the
handle's table, saved to and loaded from JSON; every plan gives a result that
meets the method's guarantee (parity with the oracle is unchanged)."""

import json

import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def test_tuned_plans_roundtrip(tmp_path):
    from paper_0905_4745_amd import api
    A, b, _ = synth.make_svd(200, 12000, 1e3, seed=31)
    N = synth.next_pow2(12000)
    d, idx = synth.draw_srft(N, 800, seed=31)
    before = api.plans_count()
    x, info = api.minnorm_solve(to_dev(A), to_dev(b), 1e-10, d, idx, N, opts=api.SolveOptions(tune=1))
    assert info["status"] == 0
    assert rel(to_np(x), oracle.classical_minnorm(A, b)) <= 1e-10
    assert api.plans_count() >= before + 2  # the fused pass and the four-step chunk
    path = tmp_path / "plans.json"
    api.plans_save(str(path))
    doc = json.loads(path.read_text())
    say(f"  plans {doc['plans']}")
    assert doc["format"] == "minnorm-plans-1"
    key = "gram/0/200/12000/0"
    assert key in doc["plans"] and key in doc["best_ms"]
    plan = doc["plans"][key]
    assert (plan & 0xFFFF) in (256, 512, 1024) and (plan >> 16) in range(16)
    # a hand-written plan file is merged and used
    doc["plans"][key] = 256 | 0x10000
    path.write_text(json.dumps(doc))
    api.plans_load(str(path))
    x2, info2 = api.minnorm_solve(to_dev(A), to_dev(b), 1e-10, d, idx, N)
    assert info2["status"] == 0 and abs(info2["iters"] - info["iters"]) <= 1
    assert rel(to_np(x2), oracle.classical_minnorm(A, b)) <= 1e-10


def test_plan_file_errors(tmp_path):
    from paper_0905_4745_amd import api
    bad = tmp_path / "bad.json"
    bad.write_text('{"format": "x"}')
    with pytest.raises(api.MinnormError) as e:
        api.plans_load(str(bad))
    assert e.value.status == -2
    with pytest.raises(api.MinnormError):
        api.plans_load(str(tmp_path / "missing.json"))


def test_every_fused_plan_meets_eps(tmp_path):
    """Fused-pass plans (workgroup counts, strip widths, strip orders, the
    pass over the column-major copy) give parity with the oracle on a ragged
    shape (n not a multiple of a strip)."""
    from paper_0905_4745_amd import api
    A, b, _ = synth.make_svd(96, 5001, 1e3, seed=32)
    N = synth.next_pow2(5001)
    d, idx = synth.draw_srft(N, 384, seed=32)
    p = oracle.classical_minnorm(A, b)
    path = tmp_path / "p.json"
    for plan in (256, 512, 1024, 256 | 0x10000, 1024 | 0x10000, 512 | 0x20000, 1024 | 0x30000, 512 | 0x40000,
                 256 | 0x70000, 256 | 0xA0000, 1024 | 0x80000, 512 | 0x90000):
        path.write_text(json.dumps({"plans": {"gram/0/96/5001/0": plan}}))
        api.plans_load(str(path))
        x, info = api.minnorm_solve(to_dev(A), to_dev(b), 1e-10, d, idx, N)
        assert info["status"] == 0
        assert rel(to_np(x), p) <= 1e-10, plan


@pytest.mark.parametrize("plan", [512, 256 | 0xA0000])
def test_profile_sampling_counts_live_launches(plan, tmp_path):
    """mn_profile(k): every k-th launch of the fused pass is timed, and only
    launches that ran an iteration are counted.  With the column-major plan
    stored, a single-RHS FP64 solve writes the copy on a side stream during
    Step 2, so every iteration's pass reads it and is eligible, as with the
    row-major plan."""
    from paper_0905_4745_amd import api
    A, b, _ = synth.make_svd(96, 6000, 1e3, seed=33)
    N = synth.next_pow2(6000)
    d, idx = synth.draw_srft(N, 384, seed=33)
    path = tmp_path / "p.json"
    path.write_text(json.dumps({"plans": {"gram/0/96/6000/0": plan}}))
    api.plans_load(str(path))
    At, bt = to_dev(A), to_dev(b)
    counts = {}
    for every in (1, 4):
        api.profile(every)
        x, info = api.minnorm_solve(At, bt, 1e-10, d, idx, N)
        cnt, ms = api.profile_read("gram")
        api.profile(False)
        assert info["status"] == 0
        assert rel(to_np(x), oracle.classical_minnorm(A, b)) <= 1e-10
        say(f"  every {every}: iters {info['iters']} timed launches {cnt} ({ms:.3f} ms)")
        counts[every] = (info["iters"], cnt, ms)
    it1, c1, ms1 = counts[1]
    it4, c4, ms4 = counts[4]
    assert c1 == it1 and ms1 > 0
    assert c4 == (it4 + 3) // 4 and ms4 > 0
    with pytest.raises(ValueError):
        api.profile(-1)


@pytest.mark.parametrize("m,n", [(40, 3001), (130, 7000), (200, 12000), (512, 9000)])
@pytest.mark.parametrize("kind", ["c128", "c64", "f64", "f32"])
def test_column_major_pass_matches_row_major(m, n, kind, tmp_path):
    """The fused pass over the column-major copy (every rows-per-lane class:
    m <= 64, 128, 256, 512; ragged m and n) against the row-major pass on the
    same system: both meet the oracle's bar and take the same iterations up
    to one."""
    import torch
    from paper_0905_4745_amd import api
    say(f"column-major pass {kind} m={m} n={n}")
    real = kind.startswith("f")
    A, b, _ = synth.make_svd(m, n, 1e3, seed=34 + m, complex_=not real)
    N = synth.next_pow2(n)
    d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=35 + m, real=real)
    tdt = {"c128": torch.complex128, "c64": torch.complex64, "f64": torch.float64, "f32": torch.float32}[kind]
    dcode = {"c128": 0, "c64": 1, "f64": 2, "f32": 3}[kind]
    At = to_dev(A, tdt)
    A_used = to_np(At).astype(np.float64 if real else np.complex128)
    p = oracle.refined_minnorm(A_used, b)
    bar = 1e-10
    res = {}
    for plan in (512 | 0x20000, 256 | 0xA0000):
        path = tmp_path / "p.json"
        keys = {f"gram/{dcode}/{m}/{n}/{w}": plan for w in (0, 1)}
        path.write_text(json.dumps({"plans": keys}))
        api.plans_load(str(path))
        x, info = api.minnorm_solve(At, to_dev(b), bar, d, idx, N)
        err = rel(to_np(x), p)
        say(f"  plan {plan:#x}: iters {info['iters']} refine {info['refine_steps']} err {err:.2e}")
        assert info["status"] == 0
        assert err <= bar, plan
        res[plan] = info["iters"]
    assert abs(res[512 | 0x20000] - res[256 | 0xA0000]) <= 1
