#!/usr/bin/env python3
"""Throughput of the randomized minimal-norm solver on one MI355X.

One step = one whole solve on device-resident inputs: SRFT sketch of A's rows,
Householder QR of the sketch, preconditioned CG on A A* y = b to the paper's
Step-4 precision, x = A* y.  Workload: A = U diag(sigma) V* with Haar U, V,
sigma log-spaced 1 -> 1e-3 (cond 1e3), m = 512, n = 65536, complex128,
eps = 1e-10, l = 4m = 2048, N = n; a fresh (d, idx) draw per step.

Prints one JSON line: solves/s, the average duration and achieved HBM rate of
the dominant pass over A (HIP events on the library's stream, timed region),
the error of the last solve against the CPU oracle, and the CPU oracle's own
throughput on a one-solve sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# the timed region brackets every PROFILE_EVERY-th launch of each pass over A
# with HIP events (the sampled launches give the kernel's average duration)
PROFILE_EVERY = 4
# launch plans tuned on an MI355X for the default workload (written by
# `bench.py --plans-out`), so that every run times the same kernel variants
DEFAULT_PLANS = os.path.join(ROOT, "paper_0905_4745_amd", "plans", "mi355x.json")

# HBM bytes per live launch of the fused pass, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE on this workload, each scaled by what the same counter reads for a
# plain 1 GiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Valid only for the
# kernel source it was measured on: a changed source reports null.
MEASURED_TRAFFIC = {
    "k_gram_cm": {"bytes": 539.14e6, "source": "paper_0905_4745_amd/csrc/gemv.hip",
                  "sha256": "6aec2ea2bd8e3631a42988db9dc8f50d8bfe0db068036f981d8e53fb59ed64fa",
                  "plan_key": "gram/0/512/65536/0", "plan": 655616},
}


def measured_traffic(kernel, plans):
    """Counter-measured HBM bytes per launch, while the kernel source and the
    launch plan this run chose are the ones the counters were taken with."""
    import hashlib
    rec = MEASURED_TRAFFIC.get(kernel)
    if rec is None:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["sha256"]:
            return None
    if plans.get(rec["plan_key"]) != rec["plan"]:
        return None
    return rec["bytes"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle accuracy check")
    ap.add_argument("--m", type=int, default=512)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--kappa", type=float, default=1e3)
    ap.add_argument("--eps", type=float, default=1e-10)
    ap.add_argument("--workload", choices=("plain", "multirhs", "batched", "mixed"), default="plain",
                    help="plain: one complex128 RHS (default); multirhs: complex64 rows scaled by "
                         "10^U(-2,2), 64 RHS through the block path; batched: 256 uneven real "
                         "systems (FP64 data + FP32 copies) in one batched call; mixed: complex128 "
                         "2048 x 262144 at cond 1e6 with a complex64 copy (FP64 refinement)")
    ap.add_argument("--streams", type=int, default=8, help="batched: concurrent lanes")
    ap.add_argument("--no-tune", action="store_true", help="built-in launch plans instead of tuned ones")
    ap.add_argument("--plans-out", default=None, help="write the tuned launch plans (JSON) here")
    ap.add_argument("--plans-in", default=DEFAULT_PLANS if os.path.exists(DEFAULT_PLANS) else None,
                    help="load launch plans (JSON, as written by --plans-out) before the warm-up; "
                         "shapes found there are not tuned again (default: the MI355X table "
                         "shipped with the package, when present)")
    ap.add_argument("--no-plans-in", action="store_true", help="tune every shape on the live operands")
    return ap.parse_args()


def plans_dump(api, args):
    """The handle's launch plans (as saved to JSON), optionally kept on disk."""
    import tempfile
    path = args.plans_out or os.path.join(tempfile.mkdtemp(), "plans.json")
    api.plans_save(path)
    with open(path) as f:
        return json.load(f)["plans"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this solver runs on one GPU: one system's passes over A, its QR and "
                          "its CG recurrences stay on a single device; use --gpus 1"}), flush=True)
        sys.exit(2)

    if args.workload == "multirhs":
        return main_multirhs(args)
    if args.workload == "batched":
        return main_batched(args)
    if args.workload == "mixed":
        return main_mixed(args)

    import numpy as np
    import torch

    import synth
    from paper_0905_4745_amd import api

    dev = torch.device("cuda:0")
    m, n, eps = args.m, args.n, args.eps
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    log(f"[bench] generating A {m}x{n} complex128 cond {args.kappa:g}")
    A, b, _ = synth.make_svd(m, n, args.kappa, seed=2)
    At = torch.from_numpy(A).to(dev)
    bt = torch.from_numpy(b).to(dev)
    draws = []
    for s in range(args.warmup + args.steps):
        d, idx = synth.draw_srft(N, l, seed=1000 + s)
        draws.append((torch.from_numpy(d).to(dev), torch.from_numpy(idx).to(dev)))
    x = torch.empty((1, n), dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()

    # launch plans are tuned on the first warm-up solve (timed candidates on
    # the live operands, outside the timed region) and reused afterwards
    if args.plans_in and not args.no_plans_in:
        log(f"[bench] launch plans from {args.plans_in}")
        api.plans_load(args.plans_in)
    opts = api.SolveOptions(tune=0 if args.no_tune else 1)
    log(f"[bench] warmup {args.warmup}")
    for s in range(args.warmup):
        d, idx = draws[s]
        api.minnorm_solve(At, bt, eps, d, idx, N, x=x, opts=opts)
    torch.cuda.synchronize()

    log(f"[bench] timed {args.steps} solves")
    # every PROFILE_EVERY-th pass over A is bracketed by HIP events (each
    # event pair costs a few microseconds of stream time)
    api.profile(PROFILE_EVERY)
    iters = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        d, idx = draws[args.warmup + s]
        _, info = api.minnorm_solve(At, bt, eps, d, idx, N, x=x, opts=opts)
        iters.append(info["iters"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kstats = {k: api.profile_read(k) for k in ("gemv_adj", "gemv_fwd", "gram")}
    api.profile(False)
    elapsed = t1 - t0
    solves_per_s = args.steps / elapsed
    log(f"[bench] {solves_per_s:.2f} solves/s, {1e3 * elapsed / args.steps:.3f} ms/solve, iters {iters}")

    # dominant kernel: the pass over A with the larger total time
    name = max(kstats, key=lambda k: kstats[k][1])
    plans = plans_dump(api, args)
    # the fused pass reads the column-major copy of A when its plan has bit 19
    cm = (plans.get(f"gram/0/{m}/{n}/0", 0) >> 19) & 1
    kname = {"gemv_adj": "k_gemv_adj", "gemv_fwd": "k_gemv_fwd", "gram": "k_gram_cm" if cm else "k_gram"}[name]
    cnt, tot_ms = kstats[name]
    avg_s = tot_ms / cnt / 1e3
    es = 16
    # A once, plus the vectors: p in and q out (m each) for the fused pass,
    # the m- and n-vector for a single product
    alg_bytes = m * n * es + (2 * m if name == "gram" else m + n) * es
    achieved = alg_bytes / avg_s / 1e9
    kernel_table = {k: {"launches": c, "avg_us": 1e3 * t / max(c, 1)} for k, (c, t) in kstats.items() if c}
    log(f"[bench] kernels {kernel_table}")

    rel_err = None
    if not args.no_check:
        import oracle
        log("[bench] oracle check (classical FP64 QR of A*)")
        p = oracle.classical_minnorm(A, b)
        xh = x[0].cpu().numpy()
        rel_err = float(np.linalg.norm(xh - p) / np.linalg.norm(p))
        log(f"[bench] rel err vs oracle {rel_err:.3e}")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from threadpoolctl import threadpool_info
        threads = max([int(t.get("num_threads", 1)) for t in threadpool_info()] + [1])
        log("[bench] CPU oracle: whole randomized solves of the same workload for about 10 s")
        done = 0
        c0 = time.perf_counter()
        while True:
            d, idx = synth.draw_srft(N, l, seed=1000 + done)
            oracle.randomized_minnorm(A, b, eps, d, idx, N, with_steps23=False)
            done += 1
            if time.perf_counter() - c0 >= 10.0 or done >= 64:
                break
        c1 = time.perf_counter()
        cpu = {"value": done / (c1 - c0), "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"{done} full solves ({m}x{n} complex128, cond {args.kappa:g}, eps {eps:g}: numpy FFT "
                         f"sketch, numpy Householder QR, scipy-triangular-solve PCG, x = A* y), fresh (d, idx) "
                         f"each, took {c1 - c0:.2f} s"}
        log(f"[bench] CPU oracle {done} solves in {c1 - c0:.2f} s on {threads} threads")

    out = {
        "metric": "solves/s at rel-err <= 1e-10 (with HBM GB/s per A-pass)",
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"plain method, complex128, m={m}, n={n}, A = U diag(sigma) V* with Haar "
                               f"factors, cond {args.kappa:g}, eps {eps:g}, l={l}, N={N}, one RHS",
                   "m": m, "n": n, "l": l, "N": N, "eps": eps, "kappa": args.kappa},
        "roofline": {"bound": "hbm", "kernel": kname,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname, plans),
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_us": avg_s * 1e6},
        "kernels": kernel_table,
        "gbps_per_apass": achieved,
        "cg_iters": iters,
        "rel_err": rel_err,
        "cpu_baseline": cpu,
        "plans": plans,
    }
    print(json.dumps(out), flush=True)



BF16_DENSE_PEAK_TFS = 2500.0  # MI355X dense BF16 matrix peak, published


def main_multirhs(args):
    """64 right-hand sides on complex64 A (4096 x 131072, rows scaled by 10^U(-2,2))."""
    import numpy as np
    import torch

    import synth
    from paper_0905_4745_amd import api

    m = args.m if args.m != 512 else 4096
    n = args.n if args.n != 65536 else 131072
    k, eps = 64, args.eps
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    dev = torch.device("cuda:0")
    log(f"[bench] generating A {m}x{n} complex64 (row scales 10^U(-2,2)), {k} RHS")
    A, B = synth.make_row_scaled(m, n, k, seed=4)
    At = torch.from_numpy(A).to(dev)
    Bt = torch.from_numpy(B).to(dev)
    del A
    X = torch.empty((k, n), dtype=torch.complex128, device=dev)
    draws = []
    for s_ in range(args.warmup + args.steps):
        d, idx = synth.draw_srft(N, l, seed=2000 + s_)
        draws.append((torch.from_numpy(d).to(dev), torch.from_numpy(idx).to(dev)))
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup}")
    if args.plans_in and not args.no_plans_in:
        log(f"[bench] launch plans from {args.plans_in}")
        api.plans_load(args.plans_in)
    opts = api.SolveOptions(tune=0 if args.no_tune else 1)
    for s_ in range(args.warmup):
        d, idx = draws[s_]
        _, info = api.minnorm_solve(At, Bt, eps, d, idx, N, x=X, opts=opts)
        log(f"[bench]   info {info}")
    torch.cuda.synchronize()
    log(f"[bench] timed {args.steps} solves of {k} RHS")
    api.profile(PROFILE_EVERY)
    infos = []
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        d, idx = draws[args.warmup + s_]
        _, info = api.minnorm_solve(At, Bt, eps, d, idx, N, x=X, opts=opts)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    names = ("block_adj", "block_fwd", "block_residual")
    kstats = {kk: api.profile_read(kk) for kk in names}
    api.profile(False)
    elapsed = t1 - t0
    table = {kk: {"launches": c, "avg_us": 1e3 * t / max(c, 1)} for kk, (c, t) in kstats.items() if c}
    log(f"[bench] {k * args.steps / elapsed:.1f} RHS/s, {1e3 * elapsed / args.steps:.2f} ms per solve; {table}")
    # the two bulk products read A's split-BF16 planes (8 B per complex entry) once each
    bulk = [kk for kk in ("block_adj", "block_fwd") if kstats[kk][0]]
    kname = max(bulk, key=lambda kk: kstats[kk][1]) if bulk else None
    roof = None
    if kname:
        cnt, tot = kstats[kname]
        avg_s = tot / cnt / 1e3
        alg = m * n * 8 + (n + m) * k * 8
        flops = 3 * 8 * m * n * k
        roof = {"bound": "hbm", "kernel": kname, "achieved": alg / avg_s / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": alg / avg_s / 1e9 / HBM_PEAK_GBS, "traffic": None,
                "alg_bytes_per_launch": alg, "avg_launch_us": avg_s * 1e6,
                "mfma_tflops": flops / avg_s / 1e12, "mfma_frac": flops / avg_s / 1e12 / BF16_DENSE_PEAK_TFS}
    out = {
        "metric": "RHS columns solved/s at rel-err <= 1e-10",
        "value": k * args.steps / elapsed,
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 data; split-bf16 bulk, fp64 refinement",
        "data": "synthetic",
        "config": {"workload": f"multi-RHS block form, complex64 A {m}x{n} (Gaussian rows scaled by "
                               f"10^U(-2,2)), {k} RHS, eps {eps:g}, l={l}, N={N}",
                   "m": m, "n": n, "nrhs": k, "l": l, "N": N, "eps": eps},
        "roofline": roof,
        "kernels": table,
        "iters": [i["iters"] for i in infos],
        "refine_steps": [i["refine_steps"] for i in infos],
        "stage_ms": infos[-1]["stage_ms"],
        "cert_rel_max": max(i["cert_rel"] for i in infos),
        "cpu_baseline": None,
        "plans": plans_dump(api, args),
    }
    print(json.dumps(out), flush=True)


def main_batched(args):
    """256 independent real systems, m log-uniform in [32, 512], n in [2048, 32768], n >= 4m."""
    import numpy as np
    import torch

    import synth
    from paper_0905_4745_amd import api

    count, eps = 256, args.eps
    dev = torch.device("cuda:0")
    log(f"[bench] generating {count} real systems (cond 1e4)")
    shapes = synth.make_batch_shapes(count, seed=5)
    systems = synth.make_batch(shapes, seed=5, kappa=1e4)
    As = [torch.from_numpy(A).to(dev) for A, _ in systems]
    A_los = [a.to(torch.float32) for a in As]
    bs = [torch.from_numpy(b).to(dev) for _, b in systems]
    entries = sum(m * n for m, n in shapes)
    draws = []
    for s_ in range(args.warmup + args.steps):
        ds, idxs, Ns = [], [], []
        for k, (m, n) in enumerate(shapes):
            N = synth.next_pow2(n)
            d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=7919 * s_ + k, real=True)
            ds.append(torch.from_numpy(d).to(dev)), idxs.append(torch.from_numpy(idx).to(dev)), Ns.append(N)
        draws.append((ds, idxs, Ns))
    torch.cuda.synchronize()
    opts = api.SolveOptions(streams=args.streams)
    log(f"[bench] warmup {args.warmup}")
    for s_ in range(args.warmup):
        api.minnorm_solve_batched(As, bs, eps, *draws[s_], A_los=A_los, opts=opts)
    torch.cuda.synchronize()
    log(f"[bench] timed {args.steps} batched calls on {args.streams} lanes")
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        xs, infos = api.minnorm_solve_batched(As, bs, eps, *draws[args.warmup + s_], A_los=A_los, opts=opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    per = count * args.steps / elapsed
    log(f"[bench] {per:.1f} systems/s ({1e3 * elapsed / args.steps:.1f} ms per batch)")
    c0 = time.perf_counter()
    api.minnorm_solve_batched(As, bs, eps, *draws[0], A_los=A_los, opts=api.SolveOptions(streams=1))
    torch.cuda.synchronize()
    serial = count / (time.perf_counter() - c0)
    log(f"[bench] one lane: {serial:.1f} systems/s")
    rel_err = None
    if not args.no_check:
        import oracle
        worst = 0.0
        for k in range(0, count, 32):  # a sample of the systems
            A, b = systems[k]
            p = oracle.refined_minnorm(A, b)
            worst = max(worst, float(np.linalg.norm(xs[k].cpu().numpy() - p) / np.linalg.norm(p)))
        rel_err = worst
        log(f"[bench] worst rel err over 8 sampled systems {worst:.2e}")
    out = {
        "metric": "systems solved/s at rel-err <= 1e-10",
        "value": per,
        "unit": "systems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 data; f32 bulk, f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"batched: {count} real systems A = U diag(sigma) V^T, cond 1e4, m log-uniform "
                               f"[32, 512], n log-uniform [2048, 32768], n >= 4m, eps {eps:g}, "
                               f"{args.streams} concurrent lanes",
                   "count": count, "entries": entries, "streams": args.streams, "eps": eps},
        "one_lane_systems_per_s": serial,
        "iters": [i["iters"] for i in infos[:16]],
        "statuses_ok": sum(1 for i in infos if i["status"] == 0),
        "rel_err": rel_err,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main_mixed(args):
    """complex128 A (2048 x 262144, cond 1e6) with its complex64 copy as the bulk."""
    import torch

    import synth
    from paper_0905_4745_amd import api

    m = args.m if args.m != 512 else 2048
    n = args.n if args.n != 65536 else 262144
    kappa = args.kappa if args.kappa != 1e3 else 1e6
    eps = args.eps
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    dev = torch.device("cuda:0")
    log(f"[bench] generating A {m}x{n} complex128 cond {kappa:g} on the device")
    A, b = synth.make_svd_device(m, n, kappa, seed=3, device=dev)
    A_lo = A.to(torch.complex64)
    x = torch.empty(n, dtype=torch.complex128, device=dev)
    draws = []
    for s_ in range(args.warmup + args.steps):
        d, idx = synth.draw_srft(N, l, seed=3000 + s_)
        draws.append((torch.from_numpy(d).to(dev), torch.from_numpy(idx).to(dev)))
    torch.cuda.synchronize()
    if args.plans_in and not args.no_plans_in:
        log(f"[bench] launch plans from {args.plans_in}")
        api.plans_load(args.plans_in)
    opts = api.SolveOptions(tune=0 if args.no_tune else 1)
    log(f"[bench] warmup {args.warmup}")
    for s_ in range(args.warmup):
        d, idx = draws[s_]
        _, info = api.minnorm_solve(A, b, eps, d, idx, N, A_lo=A_lo, x=x, opts=opts)
        log(f"[bench]   info {info}")
    torch.cuda.synchronize()
    log(f"[bench] timed {args.steps} solves")
    infos = []
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        d, idx = draws[args.warmup + s_]
        _, info = api.minnorm_solve(A, b, eps, d, idx, N, A_lo=A_lo, x=x, opts=opts)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # a property that holds at any size: the FP64 residual of the last x
    res = float(torch.linalg.vector_norm(A @ x - b) / torch.linalg.vector_norm(b))
    log(f"[bench] {args.steps / elapsed:.2f} solves/s; last info {infos[-1]}; |Ax - b|/|b| = {res:.2e}")
    out = {
        "metric": "solves/s at rel-err <= 1e-10 (FP64 certificate)",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 data; c64 bulk, fp64 (compensated) refinement",
        "data": "synthetic",
        "config": {"workload": f"mixed precision, complex128 A {m}x{n} = U diag(sigma) V* (Haar, generated on the "
                               f"device), cond {kappa:g}, complex64 copy as the bulk, eps {eps:g}, l={l}, N={N}",
                   "m": m, "n": n, "l": l, "N": N, "eps": eps, "kappa": kappa},
        "statuses": [i["status"] for i in infos],
        "iters": [i["iters"] for i in infos],
        "refine_steps": [i["refine_steps"] for i in infos],
        "cert_rel_max": max(i["cert_rel"] for i in infos),
        "residual_rel": res,
        "stage_ms": infos[-1]["stage_ms"],
        "roofline": None,
        "cpu_baseline": None,
        "plans": plans_dump(api, args),
    }
    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
