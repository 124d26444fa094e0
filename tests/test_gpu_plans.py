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
    assert (plan & 0xFFFF) in (256, 512, 1024) and (plan >> 16) in range(8)
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
    """Fused-pass plans (workgroup counts, strip widths, strip orders) give
    parity with the oracle on a ragged shape (n not a multiple of a strip)."""
    from paper_0905_4745_amd import api
    A, b, _ = synth.make_svd(96, 5001, 1e3, seed=32)
    N = synth.next_pow2(5001)
    d, idx = synth.draw_srft(N, 384, seed=32)
    p = oracle.classical_minnorm(A, b)
    path = tmp_path / "p.json"
    for plan in (256, 512, 1024, 256 | 0x10000, 1024 | 0x10000, 512 | 0x20000, 1024 | 0x30000, 512 | 0x40000,
                 256 | 0x70000):
        path.write_text(json.dumps({"plans": {"gram/0/96/5001/0": plan}}))
        api.plans_load(str(path))
        x, info = api.minnorm_solve(to_dev(A), to_dev(b), 1e-10, d, idx, N)
        assert info["status"] == 0
        assert rel(to_np(x), p) <= 1e-10, plan


def test_profile_sampling_counts_live_launches():
    """mn_profile(k): every k-th launch of the fused pass is timed, and only
    launches that ran an iteration are counted."""
    from paper_0905_4745_amd import api
    A, b, _ = synth.make_svd(96, 6000, 1e3, seed=33)
    N = synth.next_pow2(6000)
    d, idx = synth.draw_srft(N, 384, seed=33)
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
