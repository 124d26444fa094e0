#!/usr/bin/env python3
"""Throughput of the randomized minimal-norm solver on one MI355X.

One step = one whole solve on device-resident inputs: the library's draw of
the SRFT (Philox counters, a fresh seed per step), the sketch of A's rows,
Step 2's triangular factor, preconditioned CG on A A* y = b to the paper's
Step-4 precision, x = A* y -- every row of the hot path.

Default workload (`--workload mixed`): complex128 A = U diag(sigma) V*, Haar
U and V, sigma log-spaced 1 -> 1e-6 (cond 1e6), m = 2048, n = 262144, with its
complex64 copy as the bulk (sketch, factor and inner CG in single precision)
and FP64 refinement (compensated residuals) to eps = 1e-10; l = 4m = 8192,
N = n.  Beside it, the plain FP64 GPU path on the same A at the same eps
(`fp64_value`: FP64 bulk, FP64 refinement with the same compensated
residuals), and the classical FP64 oracle timed on the host's cores on a row
sample.  `--workload plain` is the 512 x 65536 complex128 cond-1e3 FP64
method; `multirhs` and `batched` the several-right-hand-side and uneven
batch workloads.

Prints one JSON line: solves/s, the average duration and achieved HBM rate of
the dominant pass over A (HIP events on the library's stream, timed region),
the accuracy reached, and the CPU oracle's throughput.
"""

from __future__ import annotations

import argparse
import dataclasses
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
    "k_gram_cm": {"bytes": 539.15e6, "source": "paper_0905_4745_amd/csrc/gemv.hip",
                  "sha256": "3a931e32285c866c2f0ddf45c965b8d17ea9f0bd90f5b7550d7798aaa6258207",
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
    ap.add_argument("--m", type=int, default=None, help="rows (default: the workload's)")
    ap.add_argument("--n", type=int, default=None, help="columns (default: the workload's)")
    ap.add_argument("--kappa", type=float, default=None, help="cond(A) (default: the workload's)")
    ap.add_argument("--eps", type=float, default=1e-10)
    ap.add_argument("--l", type=int, default=None, help="householder: sketch rows (default 4 m)")
    ap.add_argument("--workload", choices=("plain", "multirhs", "batched", "mixed", "householder"), default="mixed",
                    help="mixed (default): complex128 2048 x 262144 at cond 1e6 with a complex64 copy "
                         "(FP64 refinement), beside the FP64 GPU path; plain: 512 x 65536 complex128 "
                         "cond 1e3, FP64 throughout; multirhs: complex64 rows scaled by 10^U(-2,2), "
                         "64 RHS through the block path; batched: 256 uneven real systems (FP64 data + "
                         "FP32 copies) in one batched call; householder: Step 2's Householder QR "
                         "(build_preconditioner) of a random complex64 l x m sketch (default 8192 x 2048)")
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="mixed: timed solves of the FP64 GPU path (default: steps / 2, at least 2; 0 skips it)")
    ap.add_argument("--inner-digits", type=int, default=None,
                    help="mixed: digits each single-precision inner solve gains (default: the library's)")
    ap.add_argument("--save-a", default=None,
                    help="mixed: generate A and b, save them to this file (torch.save) and exit")
    ap.add_argument("--load-a", default=None,
                    help="mixed: load A and b saved by --save-a instead of generating them (for profiler runs "
                         "that cannot host the generator's QR)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one plain 1 GiB device-to-device copy (the reference kernel for scaling "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE readings) and exit")
    ap.add_argument("--streams", type=int, default=8, help="batched: concurrent lanes")
    ap.add_argument("--no-graph", action="store_true", help="batched: launch every kernel (no graph replay)")
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

    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8}), flush=True)
        return
    if args.workload == "multirhs":
        return main_multirhs(args)
    if args.workload == "batched":
        return main_batched(args)
    if args.workload == "mixed":
        return main_mixed(args)
    if args.workload == "householder":
        return main_householder(args)
    return main_plain(args)


def main_householder(args):
    """Step 2's Householder QR (the fallback factorisation) of a random complex64 sketch."""
    import torch

    from paper_0905_4745_amd import api

    dev = torch.device("cuda:0")
    m = args.m or 2048
    l = args.l or 4 * m
    g = torch.Generator(device=dev).manual_seed(1)
    S = torch.randn((m, l), dtype=torch.complex64, device=dev, generator=g).t()  # column-major l x m
    for _ in range(args.warmup):
        api.build_preconditioner(S)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        api.build_preconditioner(S)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    print(json.dumps({"metric": "Householder factorisations/s", "value": 1.0 / dt, "unit": "factorisations/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
                      "data": "synthetic", "config": {"workload": f"Householder QR of a {l} x {m} complex64 sketch",
                                                      "l": l, "m": m}}), flush=True)


def main_plain(args):
    """complex128 A (512 x 65536, cond 1e3), FP64 throughout, one RHS."""
    import numpy as np
    import torch

    import synth
    from paper_0905_4745_amd import api

    dev = torch.device("cuda:0")
    m, n, eps = args.m or 512, args.n or 65536, args.eps
    kappa = args.kappa or 1e3
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    log(f"[bench] generating A {m}x{n} complex128 cond {kappa:g}")
    A, b, _ = synth.make_svd(m, n, kappa, seed=2)
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
               "sample": f"{done} full solves ({m}x{n} complex128, cond {kappa:g}, eps {eps:g}: numpy FFT "
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
                               f"factors, cond {kappa:g}, eps {eps:g}, l={l}, N={N}, one RHS",
                   "m": m, "n": n, "l": l, "N": N, "eps": eps, "kappa": kappa},
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

    m = args.m or 4096
    n = args.n or 131072
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
        "statuses_ok": sum(1 for i in infos if i["status"] == 0),
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_classical_multi(At, Bt, m, n, k),
        "plans": plans_dump(api, args),
    }
    print(json.dumps(out), flush=True)


def cpu_baseline_classical_multi(A_dev, B_dev, m, n, k):
    """The classical FP64 oracle on the first 512 rows of the same A (promoted
    to complex128) with all k right-hand sides restricted to those rows: one
    QR serves every column; a whole solve costs (m / 512)^2 times the
    sample's time (QR flops ~ 8 n m^2)."""
    import numpy as np

    import oracle
    rows = min(512, m)
    A_s = A_dev[:rows].cpu().numpy().astype(np.complex128)
    B_s = B_dev[:, :rows].cpu().numpy()
    t0 = time.perf_counter()
    oracle.classical_minnorm(A_s, B_s)
    t = time.perf_counter() - t0
    est = t * (m / rows) ** 2
    log(f"[bench] CPU oracle: {rows} rows x {k} RHS in {t:.2f} s -> {est:.1f} s per whole solve")
    return {"value": k / est, "unit": "RHS/s", "cores": blas_threads(), "kind": "oracle",
            "sample": f"classical FP64 minimal-norm solve (scipy Householder QR of A*) of the first {rows} rows of "
                      f"the same {m}x{n} A with its {k} right-hand sides took {t:.2f} s; a whole solve costs "
                      f"(m/{rows})^2 = {(m / rows) ** 2:.0f} times that: {est:.1f} s; host {cpu_model()}, "
                      f"os.cpu_count() = {os.cpu_count()}"}


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
    Ns = [synth.next_pow2(n) for _, n in shapes]
    # the batch is validated once; every call draws its SRFTs in the library
    # (seed = the call's number, sys = the system's index)
    batch_mixed = api.BatchedSystems(As, bs, Ns, A_los)
    batch_fp64 = api.BatchedSystems(As, bs, Ns, None)
    torch.cuda.synchronize()
    opts = api.SolveOptions(streams=args.streams, graph=-1 if args.no_graph else 0)

    def timed(o, batch, steps, warmup):
        for s_ in range(warmup):
            batch.solve(eps, opts=dataclasses.replace(o, seed=s_))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s_ in range(steps):
            xs, infos = batch.solve(eps, opts=dataclasses.replace(o, seed=warmup + s_))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, xs, infos

    log(f"[bench] warmup {args.warmup}, timed {args.steps} batched calls (graph replay "
        f"{'off' if args.no_graph else 'on'})")
    elapsed, xs, infos = timed(opts, batch_mixed, args.steps, args.warmup)
    per = count * args.steps / elapsed
    log(f"[bench] {per:.1f} systems/s ({1e3 * elapsed / args.steps:.1f} ms per batch)")
    # the same calls launching every kernel (no graph replay)
    alt = api.SolveOptions(streams=args.streams, graph=0 if args.no_graph else -1)
    e_alt, _, _ = timed(alt, batch_mixed, max(2, args.steps // 2), 1)
    alt_per = count * max(2, args.steps // 2) / e_alt
    log(f"[bench] graph replay {'on' if args.no_graph else 'off'}: {alt_per:.1f} systems/s")
    # plain FP64 on the same systems (cond 1e4: FP64 alone reaches eps), the
    # comparison the metric asks for
    fsteps = max(2, args.steps // 2)
    e64, _, i64 = timed(api.SolveOptions(streams=args.streams), batch_fp64, fsteps, 1)
    fp64_per = count * fsteps / e64
    log(f"[bench] plain FP64: {fp64_per:.1f} systems/s")
    # fused-pass roofline: one call with every pass timed (launched, not
    # replayed); bytes = each system's FP32 column-major copy once per inner
    # iteration, plus the first pass that reads A's rows and writes the copy
    api.profile(1)
    batch_mixed.solve(eps, opts=api.SolveOptions(streams=args.streams, graph=-1))
    cnt, tot_ms = api.profile_read("gram")
    api.profile(False)
    _, pinfos = batch_mixed.solve(eps, opts=opts)
    pass_bytes = sum(4 * m * n * (inf["iters"] + 1) for (m, n), inf in zip(shapes, pinfos))
    achieved = pass_bytes / (tot_ms / 1e3) / 1e9 if tot_ms > 0 else None
    log(f"[bench] fused passes: {cnt} launches, {tot_ms:.2f} ms, {pass_bytes / 1e9:.2f} GB -> {achieved:.0f} GB/s")
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
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        done, c0 = 0, time.perf_counter()
        while done < count and time.perf_counter() - c0 < 10.0:
            A, b = systems[done]
            oracle.classical_minnorm(A, b)
            done += 1
        ct = time.perf_counter() - c0
        cpu = {"value": done / ct, "unit": "systems/s", "cores": blas_threads(), "kind": "oracle",
               "sample": f"classical FP64 minimal-norm solves (scipy Householder QR of A*) of the first {done} of the "
                         f"same {count} systems, {ct:.2f} s; host {cpu_model()}, os.cpu_count() = {os.cpu_count()}"}
        log(f"[bench] CPU oracle: {done} systems in {ct:.2f} s")
    out = {
        "metric": "systems solved/s at rel-err <= 1e-10, batched mixed precision vs FP64",
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
                               f"[32, 512], n log-uniform [2048, 32768], n >= 4m, eps {eps:g}, one fused call "
                               f"(every stage one launch over all systems), iteration blocks replayed as HIP "
                               f"graphs{' (off)' if args.no_graph else ''}, library-drawn SRFTs (seed = the "
                               f"call's number), the batch validated once and its solutions reused",
                   "count": count, "entries": entries, "eps": eps},
        "graph_replay": not args.no_graph,
        "other_replay_value": alt_per,
        "fp64_value": fp64_per,
        "mixed_over_fp64": per / fp64_per,
        "fp64_config": "the same systems, plain FP64 (no single-precision copy, no refinement)",
        "iters": [i["iters"] for i in infos[:16]],
        "statuses_ok": sum(1 for i in infos if i["status"] == 0),
        "fp64_statuses_ok": sum(1 for i in i64 if i["status"] == 0),
        "rel_err": rel_err,
        "roofline": {"bound": "hbm", "kernel": "kb_gram_cm (+ kb_gram_wt, kb_gram_reduce)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": None,
                     "alg_bytes_per_call": pass_bytes, "pass_ms_per_call": tot_ms, "launches": cnt,
                     "basis": "summed per-system bytes: 4 m n per inner iteration (the FP32 column-major copy) "
                              "plus 8 m n for the pass that writes the copy, over the summed duration of the "
                              "fused-pass stage (HIP events around each launch of it, every kernel launched)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def blas_threads():
    from threadpoolctl import threadpool_info
    return max([int(t.get("num_threads", 1)) for t in threadpool_info() if t.get("user_api") == "blas"] + [1])


def cpu_baseline_classical(A_dev, b_dev, m, n):
    """The classical FP64 oracle (Householder QR of A*, p = Q R^{-*} b) timed
    on the host's cores on the first m' rows of the same A; its cost is
    proportional to n m'^2, so one whole solve is estimated as (m / m')^2
    times the sample's time.  m' = 256, or 512 when that sample is quick."""
    import oracle
    out = None
    for rows in (256, 512):
        if rows > m:
            break
        A_s = A_dev[:rows].cpu().numpy()
        b_s = b_dev[:rows].cpu().numpy()
        t0 = time.perf_counter()
        oracle.classical_minnorm(A_s, b_s)
        t = time.perf_counter() - t0
        est = t * (m / rows) ** 2
        out = {"value": 1.0 / est, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
               "sample": f"classical FP64 minimal-norm solve (scipy Householder QR of A*, LAPACK) of the first "
                         f"{rows} rows of the same {m}x{n} complex128 A took {t:.2f} s; a whole solve costs "
                         f"(m/{rows})^2 = {(m / rows) ** 2:.0f} times that (QR flops ~ 8 n m^2): {est:.1f} s; "
                         f"host {cpu_model()}, os.cpu_count() = {os.cpu_count()}, BLAS threads as reported"}
        log(f"[bench] CPU oracle: {rows} rows in {t:.2f} s -> {est:.1f} s per whole solve")
        del A_s
        if t > 5.0:
            break
    return out


# HBM bytes per live launch of the dominant pass of the mixed workload, from
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (same copy scaling as
# MEASURED_TRAFFIC: the A copy once, plus the workgroups' q partials written);
# valid while the source and the plan are the measured ones
MEASURED_TRAFFIC_MIXED = {
    "k_gram_tall": {"bytes": 4312113357.0, "source": "paper_0905_4745_amd/csrc/gemv.hip",
                    "sha256": "3a931e32285c866c2f0ddf45c965b8d17ea9f0bd90f5b7550d7798aaa6258207",
                    "plan_key": "gram/1/2048/262144/1", "plan": 524800},
}


def main_mixed(args):
    """complex128 A (2048 x 262144, cond 1e6) with its complex64 copy as the
    bulk, FP64 refinement; the FP64 GPU path on the same A beside it."""
    import hashlib

    import torch

    import synth
    from paper_0905_4745_amd import api

    m, n = args.m or 2048, args.n or 262144
    kappa = args.kappa or 1e6
    eps = args.eps
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    dev = torch.device("cuda:0")
    if args.load_a:
        log(f"[bench] loading A, b from {args.load_a}")
        A, b = torch.load(args.load_a, map_location="cpu", weights_only=True)
        A, b = A.to(dev), b.to(dev)
        m, n = A.shape
        N = synth.next_pow2(n)
        l = synth.sketch_width(m, N)
    else:
        log(f"[bench] generating A {m}x{n} complex128 cond {kappa:g} on the device")
        A, b = synth.make_svd_device(m, n, kappa, seed=3, device=dev)
    if args.save_a:
        torch.save((A.cpu(), b.cpu()), args.save_a)
        log(f"[bench] saved A, b to {args.save_a}")
        return
    A_lo = A.to(torch.complex64)
    x = torch.empty(n, dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    if args.plans_in and not args.no_plans_in:
        log(f"[bench] launch plans from {args.plans_in}")
        api.plans_load(args.plans_in)
    tune = 0 if args.no_tune else 1

    def run(steps, warmup, seed0, fp64):
        # one step: the library's draw (fresh seed), sketch, factor, refined CG, x
        opts = (api.SolveOptions(tune=tune, refine=1, inner_digits=6) if fp64 else
                api.SolveOptions(tune=tune, inner_digits=args.inner_digits or 0))
        lo = None if fp64 else A_lo
        for s_ in range(warmup):
            opts.seed = seed0 + s_
            _, info = api.minnorm_solve(A, b, eps, None, None, N, A_lo=lo, x=x, opts=opts, l=l)
            log(f"[bench]   warmup info {info}")
        torch.cuda.synchronize()
        if not fp64:
            api.profile(PROFILE_EVERY)
        infos = []
        t0 = time.perf_counter()
        for s_ in range(steps):
            opts.seed = seed0 + warmup + s_
            _, info = api.minnorm_solve(A, b, eps, None, None, N, A_lo=lo, x=x, opts=opts, l=l)
            infos.append(info)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        kst = None
        if not fp64:
            kst = {k: api.profile_read(k) for k in ("gemv_adj", "gemv_fwd", "gram")}
            api.profile(False)
        return elapsed, infos, kst

    log(f"[bench] mixed: warmup {args.warmup}, timed {args.steps} solves")
    elapsed, infos, kstats = run(args.steps, args.warmup, 3000, False)
    value = args.steps / elapsed
    log(f"[bench] mixed {value:.2f} solves/s; last info {infos[-1]}")
    kernel_table = {k: {"launches": c, "avg_us": 1e3 * t / max(c, 1)} for k, (c, t) in kstats.items() if c}
    log(f"[bench] kernels {kernel_table}")

    fsteps = args.fp64_steps if args.fp64_steps is not None else max(2, args.steps // 2)
    f_elapsed, f_infos, fp64_value = 0.0, [], None
    if fsteps > 0:
        log(f"[bench] FP64 GPU path on the same A: warmup 1, timed {fsteps} solves")
        f_elapsed, f_infos, _ = run(fsteps, 1, 5000, True)
        fp64_value = fsteps / f_elapsed
        log(f"[bench] FP64 {fp64_value:.2f} solves/s; last info {f_infos[-1]}")

    plans = plans_dump(api, args)
    # dominant kernel: the pass over A with the larger total time
    name = max(kstats, key=lambda k: kstats[k][1])
    cnt, tot_ms = kstats[name]
    avg_s = tot_ms / cnt / 1e3
    es = 8  # the complex64 copy
    fused = name == "gram"
    kname = {"gemv_adj": "k_gemv_adj", "gemv_fwd": "k_gemv_fwd",
             "gram": "k_gram_tall" if m > 512 else "k_gram_cm"}[name]
    alg_bytes = m * n * es + (2 * m * 16 if fused else m * 16 + n * 16)
    achieved = alg_bytes / avg_s / 1e9
    traffic = None
    rec = MEASURED_TRAFFIC_MIXED.get(kname)
    if rec:
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            same = hashlib.sha256(f.read()).hexdigest() == rec["sha256"]
        if same and plans.get(rec["plan_key"]) == rec["plan"]:
            traffic = rec["bytes"]

    cpu = None if args.no_cpu_baseline else cpu_baseline_classical(A, b, m, n)

    statuses = [i["status"] for i in infos] + [i["status"] for i in f_infos]
    out = {
        "metric": "solves/s at rel-err <= 1e-10 (with HBM GB/s per A-pass), mixed precision vs FP64",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 bulk (sketch, factor, inner CG), f64 compensated refinement; c128 data",
        "data": "synthetic",
        "config": {"workload": f"mixed precision, complex128 A {m}x{n} = U diag(sigma) V* (Haar factors, "
                               f"generated on the device), cond {kappa:g}, complex64 copy as the bulk, FP64 "
                               f"refinement, eps {eps:g}, l={l}, N={N}, one RHS, library-drawn SRFT per solve",
                   "m": m, "n": n, "l": l, "N": N, "eps": eps, "kappa": kappa},
        "fp64_value": fp64_value,
        "fp64_ms_per_step": 1e3 * f_elapsed / fsteps if fsteps else None,
        "mixed_over_fp64": value / fp64_value if fp64_value else None,
        "fp64_config": "the same A, complex128 bulk (one-read passes over its column-major copy), FP64 "
                       "refinement with the same compensated residuals, inner solves to 6 digits (the fastest of 4, 6, 8, 10 and 12 measured on this workload), same eps",
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_us": avg_s * 1e6},
        "kernels": kernel_table,
        "gbps_per_apass": achieved,
        "rel_err": max(i["cert_rel"] for i in infos),
        "rel_err_kind": "FP64 certificate sqrt(rho/xi) >= ||x - p|| / ||x|| of every timed solve; the same path "
                        "is compared with the longdouble-refined oracle at 2048 x 65536 and smaller in the GPU "
                        "tests (tests/test_gpu_large.py)",
        "fp64_rel_err": max(i["cert_rel"] for i in f_infos) if f_infos else None,
        "statuses_ok": sum(1 for v in statuses if v == 0),
        "solves": len(statuses),
        "iters": [i["iters"] for i in infos],
        "refine_steps": [i["refine_steps"] for i in infos],
        "fp64_iters": [i["iters"] for i in f_infos],
        "fp64_refine_steps": [i["refine_steps"] for i in f_infos],
        "stage_ms": infos[-1]["stage_ms"],
        "fp64_stage_ms": f_infos[-1]["stage_ms"] if f_infos else None,
        "cpu_baseline": cpu,
        "plans": plans,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
