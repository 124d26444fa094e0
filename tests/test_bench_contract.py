"""Host-side checks of bench.py's contract (no GPU needed):

* more than one GPU is refused with a message and a non-zero status, before
  anything touches a device;
* the counter-measured HBM traffic that the bench line reports is tied to
  the fused-pass source it was measured on: the recorded hashes must match
  the current source (a changed source makes the bench report null, so a
  kernel edit without new counters fails here first) and name shipped plans;
* the shipped launch-plan table is well formed.
"""

import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_traffic_records_match_the_source_and_plans():
    import bench
    with open(bench.DEFAULT_PLANS) as f:
        plans = json.load(f)["plans"]
    for table in (bench.MEASURED_TRAFFIC, bench.MEASURED_TRAFFIC_MIXED):
        for kernel, rec in table.items():
            with open(os.path.join(ROOT, rec["source"]), "rb") as f:
                assert hashlib.sha256(f.read()).hexdigest() == rec["sha256"], kernel
            assert plans.get(rec["plan_key"]) == rec["plan"], kernel
            assert rec["bytes"] > 0


def test_shipped_plans_well_formed():
    import bench
    with open(bench.DEFAULT_PLANS) as f:
        d = json.load(f)
    assert d["format"] == "minnorm-plans-1"
    assert d["plans"] and all(isinstance(v, int) for v in d["plans"].values())
    for k in d["plans"]:
        kind, *dims = k.split("/")
        assert kind and len(dims) == 4 and all(x.lstrip("-").isdigit() for x in dims), k
    assert set(d.get("best_ms", {})) <= set(d["plans"])
