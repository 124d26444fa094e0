"""GPU parity of the whole method (minnorm_solve) against the CPU oracle.

Bars: the method guarantees ||x - p|| <= eps ||p|| (Theorem 5.4), so each
GPU x must lie within eps of the oracle's p (classical FP64 QR, or the
longdouble-refined solver where cond(A) u64 approaches eps).  With the same
(d, idx) the GPU iteration must also track the CPU randomized oracle: equal
iteration counts up to one (rounding can move the stopping test by one step).
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _solve(A, b, eps, d, idx, N, **kw):
    from paper_0905_4745_amd import api
    At = to_dev(A)
    bt = to_dev(b)
    x, info = api.minnorm_solve(At, bt, eps, d, idx, N, **kw)
    return to_np(x), info


@pytest.mark.parametrize("m,n,seed", [(64, 1024, 0), (1, 40, 1), (31, 700, 2), (100, 3000, 3), (200, 2000, 4)])
def test_gaussian_c128(m, n, seed):
    """Plain complex128 method on Gaussian A (the 64 x 1024, eps = 1e-12 workload and ragged sizes)."""
    say(f"solve gaussian c128 m={m} n={n}")
    A, b = synth.make_gaussian(m, n, seed=seed)
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    d, idx = synth.draw_srft(N, l, seed=seed + 10)
    eps = 1e-12
    x, info = _solve(A, b, eps, d, idx, N)
    p = oracle.classical_minnorm(A, b)
    err = rel(x, p)
    o = oracle.randomized_minnorm(A, b, eps, d, idx, N, with_steps23=False)
    say(f"  err {err:.2e} iters gpu {info['iters']} cpu {o['info']['iters']}")
    assert info["status"] == 0
    assert err <= eps
    assert abs(info["iters"] - o["info"]["iters"]) <= 1
    assert rel(x, o["x"]) <= eps


@pytest.mark.parametrize("m,n,kappa,seed", [(128, 8192, 1e3, 5), (96, 5000, 1e3, 6)])
def test_svd_c128_kappa_1e3(m, n, kappa, seed):
    say(f"solve svd c128 m={m} n={n} kappa={kappa}")
    A, b, _ = synth.make_svd(m, n, kappa, seed=seed)
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    d, idx = synth.draw_srft(N, l, seed=seed)
    eps = 1e-10
    x, info = _solve(A, b, eps, d, idx, N)
    p = oracle.classical_minnorm(A, b)
    o = oracle.randomized_minnorm(A, b, eps, d, idx, N, with_steps23=False)
    say(f"  err {rel(x, p):.2e} iters gpu {info['iters']} cpu {o['info']['iters']}")
    assert info["status"] == 0
    assert rel(x, p) <= eps
    assert abs(info["iters"] - o["info"]["iters"]) <= 1


def test_full_size_c128_512x65536():
    """The 512 x 65536, cond 1e3, eps = 1e-10 workload at full size."""
    say("solve svd c128 full size m=512 n=65536")
    A, b, _ = synth.make_svd(512, 65536, 1e3, seed=2)
    N = 65536
    l = 2048
    d, idx = synth.draw_srft(N, l, seed=7)
    x, info = _solve(A, b, 1e-10, d, idx, N)
    p = oracle.classical_minnorm(A, b)
    say(f"  err {rel(x, p):.2e} iters {info['iters']} ms {info['stage_ms']}")
    assert info["status"] == 0
    assert rel(x, p) <= 1e-10


@pytest.mark.parametrize("rule", [0, 1])
def test_stop_rules(rule):
    from paper_0905_4745_amd import api
    A, b, _ = synth.make_svd(48, 1500, 1e2, seed=9)
    N = synth.next_pow2(1500)
    d, idx = synth.draw_srft(N, 192, seed=1)
    x, info = _solve(A, b, 1e-9, d, idx, N, opts=api.SolveOptions(stop_rule=rule))
    o = oracle.randomized_minnorm(A, b, 1e-9, d, idx, N, rule="PR"[rule], with_steps23=False)
    assert rel(x, oracle.classical_minnorm(A, b)) <= 1e-9
    assert abs(info["iters"] - o["info"]["iters"]) <= 1


def test_l_equals_N_and_zero_rhs():
    A, b = synth.make_gaussian(20, 60, seed=3)
    N = 64
    d, idx = synth.draw_srft(N, N, seed=2)
    x, info = _solve(A, b, 1e-12, d, idx, N)
    assert info["iters"] <= 2
    assert rel(x, oracle.classical_minnorm(A, b)) <= 1e-12
    x0, info0 = _solve(A, np.zeros(20, complex), 1e-12, d, idx, N)
    assert info0["iters"] == 0 and np.all(x0 == 0)


def test_orthonormal_rows_and_known_answer():
    g = np.random.default_rng(1)
    Q = np.linalg.qr(synth.complex_gaussian(g, (600, 30)))[0]
    A = np.ascontiguousarray(Q.conj().T)
    b = synth.complex_gaussian(g, 30)
    N = 1024
    d, idx = synth.draw_srft(N, 120, seed=4)
    x, _ = _solve(A, b, 1e-12, d, idx, N)
    assert rel(x, A.conj().T @ b) <= 1e-12
    # the paper's Section 7 construction, cond 1e3
    A, b, p, _ = synth.make_known_answer(64, 2048, seed=5, kappa=1e3)
    d, idx = synth.draw_srft(2048, 256, seed=5)
    x, _ = _solve(A, b, 1e-10, d, idx, 2048)
    assert rel(x, p) <= 1e-10


def test_multi_rhs_c128():
    A, B = synth.make_gaussian(40, 900, seed=11, nrhs=3)
    N = 1024
    d, idx = synth.draw_srft(N, 160, seed=2)
    X, info = _solve(A, B, 1e-11, d, idx, N)
    P = oracle.classical_minnorm(A, B)
    for k in range(3):
        assert rel(X[k], P[k]) <= 1e-11
    assert info["nrhs_done"] == 3


def test_real_f64():
    shapes = synth.make_batch_shapes(3, seed=2, m_lo=16, m_hi=80, n_lo=400, n_hi=3000)
    for k, (A, b) in enumerate(synth.make_batch(shapes, seed=3, kappa=1e4)):
        m, n = A.shape
        N = synth.next_pow2(n)
        d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=k, real=True)
        x, info = _solve(A, b, 1e-10, d, idx, N)
        assert info["status"] == 0
        assert rel(x, oracle.refined_minnorm(A, b)) <= 1e-10


def test_mixed_c128_with_c64_copy_kappa_1e6():
    """complex64 bulk + FP64 refinement at cond 1e6 reaches 1e-10 vs the refined oracle."""
    import torch
    from paper_0905_4745_amd import api
    say("solve mixed c128/c64 kappa 1e6")
    A, b, _ = synth.make_svd(64, 4096, 1e6, seed=3)
    N = 4096
    d, idx = synth.draw_srft(N, 256, seed=3)
    At = to_dev(A)
    x, info = api.minnorm_solve(At, to_dev(b), 1e-10, d, idx, N, A_lo=At.to(torch.complex64))
    p = oracle.refined_minnorm(A, b)
    say(f"  err {rel(to_np(x), p):.2e} iters {info['iters']} refine {info['refine_steps']}")
    assert info["status"] == 0
    assert rel(to_np(x), p) <= 1e-10


def test_mixed_real_f64_with_f32_copy():
    import torch
    from paper_0905_4745_amd import api
    A, b, _ = synth.make_svd(50, 3000, 1e4, seed=8, complex_=False)
    N = 4096
    d, idx = synth.draw_srft(N, 200, seed=8, real=True)
    At = to_dev(A)
    x, info = api.minnorm_solve(At, to_dev(b), 1e-10, d, idx, N, A_lo=At.to(torch.float32))
    assert info["status"] == 0
    assert rel(to_np(x), oracle.refined_minnorm(A, b)) <= 1e-10


def test_single_precision_problem_c64():
    """complex64 data is the problem: refinement promotes it exactly to FP64."""
    from paper_0905_4745_amd import api
    A64, B = synth.make_row_scaled(48, 2000, 2, seed=4)
    N = 2048
    d, idx = synth.draw_srft(N, 192, seed=4)
    X, info = api.minnorm_solve(to_dev(A64), to_dev(B), 1e-10, d, idx, N)
    P = oracle.refined_minnorm(A64.astype(np.complex128), B)
    for k in range(2):
        assert rel(to_np(X[k]), P[k]) <= 1e-10


def test_batched_uneven_real():
    import torch
    from paper_0905_4745_amd import api
    shapes = synth.make_batch_shapes(5, seed=7, m_lo=8, m_hi=64, n_lo=300, n_hi=2000)
    systems = synth.make_batch(shapes, seed=8, kappa=1e4)
    As = [to_dev(A) for A, _ in systems]
    A_los = [a.to(torch.float32) for a in As]
    bs = [to_dev(b) for _, b in systems]
    ds, idxs, Ns = [], [], []
    for k, (m, n) in enumerate(shapes):
        N = synth.next_pow2(n)
        d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=k, real=True)
        ds.append(d), idxs.append(idx), Ns.append(N)
    xs, infos = api.minnorm_solve_batched(As, bs, 1e-10, ds, idxs, Ns, A_los=A_los)
    for (A, b), x, info in zip(systems, xs, infos):
        assert info["status"] == 0
        assert rel(to_np(x), oracle.refined_minnorm(A, b)) <= 1e-10


def test_failure_statuses():
    from paper_0905_4745_amd import api
    # iteration cap -> +2
    A, b, _ = synth.make_svd(32, 1000, 1e3, seed=1)
    N = 1024
    d, idx = synth.draw_srft(N, 128, seed=1)
    x, info = _solve(A, b, 1e-12, d, idx, N, opts=api.SolveOptions(max_iter=1), raise_on_status=False)
    assert info["status"] == 2 and info["iters"] == 1
    # duplicate rows: A not full rank -> sketch rank-deficient (+1)
    A2 = A.copy()
    A2[5] = A2[9]
    with pytest.raises(api.MinnormError) as e:
        _solve(A2, b, 1e-10, d, idx, N)
    assert e.value.status == 1
    # NaN input -> +4
    A3 = A.copy()
    A3[2, 7] = np.nan
    with pytest.raises(api.MinnormError) as e:
        _solve(A3, b, 1e-10, d, idx, N)
    assert e.value.status == 4
    # invalid idx -> -16
    with pytest.raises(api.MinnormError) as e:
        _solve(A, b, 1e-10, d, np.sort(np.concatenate([idx[:-1], idx[:1]])), N)
    assert e.value.status == -16


@pytest.mark.parametrize("m,n,kind", [(640, 6000, "c128"), (700, 5001, "f64"), (96, 3001, "c128")])
def test_unfused_and_unaligned_paths(m, n, kind):
    """m > 512 (separate A* p and A w passes) and rows that are not 16-byte
    aligned (odd n for real data) go through the unfused kernels."""
    say(f"solve {kind} m={m} n={n}")
    real = kind == "f64"
    A, b, _ = synth.make_svd(m, n, 1e2, seed=m, complex_=not real)
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    d, idx = synth.draw_srft(N, l, seed=m, real=real)
    x, info = _solve(A, b, 1e-10, d, idx, N)
    p = oracle.classical_minnorm(A, b)
    say(f"  err {rel(x, p):.2e} iters {info['iters']}")
    assert info["status"] == 0
    assert rel(x, p) <= 1e-10


@pytest.mark.parametrize("form,streams", [(1, 1), (1, 8), (0, 8)])
def test_batched_concurrent_lanes(form, streams):
    """24 uneven real systems (FP64 data + FP32 copies): concurrent lanes (1 and
    8) and the fused form (every stage of all systems in one launch)."""
    import torch
    from paper_0905_4745_amd import api
    say(f"batched 24 systems, form {form}, {streams} lanes")
    shapes = synth.make_batch_shapes(24, seed=11, m_lo=8, m_hi=128, n_lo=300, n_hi=4000)
    systems = synth.make_batch(shapes, seed=12, kappa=1e4)
    As = [to_dev(A) for A, _ in systems]
    A_los = [a.to(torch.float32) for a in As]
    bs = [to_dev(b) for _, b in systems]
    ds, idxs, Ns = [], [], []
    for k, (m, n) in enumerate(shapes):
        N = synth.next_pow2(n)
        d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=100 + k, real=True)
        ds.append(d), idxs.append(idx), Ns.append(N)
    xs, infos = api.minnorm_solve_batched(As, bs, 1e-10, ds, idxs, Ns, A_los=A_los,
                                          opts=api.SolveOptions(streams=streams, batch_form=form))
    worst = 0.0
    for (A, b), x, info in zip(systems, xs, infos):
        assert info["status"] == 0
        worst = max(worst, rel(to_np(x), oracle.refined_minnorm(A, b)))
    say(f"  worst err {worst:.2e}")
    assert worst <= 1e-10


def test_batched_one_bad_idx_others_solved():
    from paper_0905_4745_amd import api
    sys_ = [synth.make_gaussian(m, n, seed=s) for s, (m, n) in enumerate([(20, 500), (33, 900), (12, 300)])]
    As = [to_dev(A) for A, _ in sys_]
    bs = [to_dev(b) for _, b in sys_]
    ds, idxs, Ns = [], [], []
    for k, (A, _) in enumerate(sys_):
        m, n = A.shape
        N = synth.next_pow2(n)
        d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=k)
        if k == 1:
            idx = np.sort(np.concatenate([idx[:-1], idx[:1]]))  # a repeated index
        ds.append(d), idxs.append(idx), Ns.append(N)
    xs, infos = api.minnorm_solve_batched(As, bs, 1e-12, ds, idxs, Ns, opts=api.SolveOptions(streams=3),
                                          raise_on_status=False)
    assert infos[1]["status"] == -14
    for k in (0, 2):
        assert infos[k]["status"] == 0
        A, b = sys_[k]
        assert rel(to_np(xs[k]), oracle.classical_minnorm(A, b)) <= 1e-12


@pytest.mark.parametrize("kind", ["c128", "f64", "c64"])
def test_gram_and_householder_factors_agree(kind):
    """Step 2's R from the Cholesky of the FP64 Gram matrix (default) and from
    Householder QR of S give the same preconditioner: both solves meet eps
    and take the same number of iterations up to one."""
    from paper_0905_4745_amd import api
    real = kind == "f64"
    A, b, _ = synth.make_svd(150, 4000, 1e3, seed=21, complex_=not real)
    if kind == "c64":
        A = A.astype(np.complex64)
    N = synth.next_pow2(4000)
    d, idx = synth.draw_srft(N, 600, seed=21, real=real)
    xg, ig = _solve(A, b, 1e-10, d, idx, N, opts=api.SolveOptions(precond=0))
    xh, ih = _solve(A, b, 1e-10, d, idx, N, opts=api.SolveOptions(precond=1))
    p = oracle.refined_minnorm(A.astype(np.complex128) if kind == "c64" else A, b)
    say(f"  {kind}: gram iters {ig['iters']} err {rel(xg, p):.2e}; householder iters {ih['iters']} err {rel(xh, p):.2e}")
    assert ig["status"] == 0 and ih["status"] == 0
    assert rel(xg, p) <= 1e-10 and rel(xh, p) <= 1e-10
    assert abs(ig["iters"] - ih["iters"]) <= max(1, ih["iters"] // 10)


@pytest.mark.parametrize("kind,m,n", [("c128", 200, 8000), ("f64", 130, 5000), ("c64", 1100, 8800)])
def test_gram_product_routes_agree(kind, m, n, tmp_path):
    """Step 2's Gram matrix S* S on the FP64 matrix cores (plan 0) and on the
    vector units (plan 1, with split-K partials for these shapes) gives the
    same factor: both solves meet eps in the same number of iterations up to
    one.  Ragged m (not a multiple of the 128 x 64 tile)."""
    import json
    from paper_0905_4745_amd import api
    real = kind == "f64"
    A, b, _ = synth.make_svd(m, n, 1e3, seed=23, complex_=not real)
    if kind == "c64":
        A = A.astype(np.complex64)
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    d, idx = synth.draw_srft(N, l, seed=23, real=real)
    dcode = {"c128": 0, "c64": 1, "f64": 2}[kind]
    key = f"gram_s/{dcode}/{m}/{l}/0"
    res = {}
    for plan in (0, 1):
        path = tmp_path / f"plans{plan}.json"
        path.write_text(json.dumps({"format": "minnorm-plans-1", "plans": {key: plan}, "best_ms": {}}))
        api.plans_load(str(path))
        res[plan] = _solve(A, b, 1e-10, d, idx, N)
    p = oracle.refined_minnorm(A.astype(np.complex128) if kind == "c64" else A, b)
    (x0, i0), (x1, i1) = res[0], res[1]
    say(f"  {kind} m={m}: matrix-core iters {i0['iters']} err {rel(x0, p):.2e}; "
        f"vector iters {i1['iters']} err {rel(x1, p):.2e}")
    assert i0["status"] == 0 and i1["status"] == 0
    assert rel(x0, p) <= 1e-10 and rel(x1, p) <= 1e-10
    assert abs(i0["iters"] - i1["iters"]) <= 1


def test_ill_conditioned_falls_back_and_meets_eps():
    """cond 1e7: the Gram route declines (diagonal spread beyond 1e5) and the
    Householder factor is used; the FP64 result still meets eps."""
    A, b, _ = synth.make_svd(40, 1500, 1e7, seed=22)
    N = 2048
    d, idx = synth.draw_srft(N, 160, seed=22)
    x, info = _solve(A, b, 1e-8, d, idx, N)
    assert info["status"] == 0
    assert rel(x, oracle.refined_minnorm(A, b)) <= 1e-8


def _batch_inputs(shapes, seed, complex_, kappa, real_signs):
    ds, idxs, Ns = [], [], []
    for k, (m, n) in enumerate(shapes):
        N = synth.next_pow2(n)
        d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=seed + k, real=real_signs)
        ds.append(d), idxs.append(idx), Ns.append(N)
    return ds, idxs, Ns


def test_batched_fused_plain_c128_matches_lanes():
    """Plain complex128 systems (one with N <= 4096, others four-step; ragged m):
    fused and lane forms both meet eps against the classical oracle, with the
    same iteration counts up to one."""
    from paper_0905_4745_amd import api
    shapes = [(20, 600), (64, 5000), (37, 9000), (130, 4100), (7, 33)]
    systems = [synth.make_svd(m, n, 1e3, seed=40 + k)[:2] for k, (m, n) in enumerate(shapes)]
    As = [to_dev(A) for A, _ in systems]
    bs = [to_dev(b) for _, b in systems]
    ds, idxs, Ns = _batch_inputs(shapes, 50, True, 1e3, False)
    xf, inf_f = api.minnorm_solve_batched(As, bs, 1e-10, ds, idxs, Ns, opts=api.SolveOptions(batch_form=0))
    xl, inf_l = api.minnorm_solve_batched(As, bs, 1e-10, ds, idxs, Ns, opts=api.SolveOptions(batch_form=1))
    for (A, b), a, c, ia, ic in zip(systems, xf, xl, inf_f, inf_l):
        p = oracle.classical_minnorm(A, b)
        assert ia["status"] == 0 and ic["status"] == 0
        assert rel(to_np(a), p) <= 1e-10 and rel(to_np(c), p) <= 1e-10
        assert abs(ia["iters"] - ic["iters"]) <= 1


@pytest.mark.parametrize("bulk", ["f32", "f64"])
def test_batched_fused_four_step_kept_output_classes(bulk):
    """Four-step systems in every kept-outputs-only accumulator class (l <= 512,
    <= 1024, <= 2048, up to l = 2048 at m = 512) in one fused batched call, real
    data: each meets eps against the oracle and takes about the iteration count
    of the same system solved alone (lanes form, whose sketch is the
    single-system kernel).  FP64 bulk (no refinement, the same passes on both
    sides): equal up to one.  FP32 bulk with FP64 refinement: up to three, as
    the fused form builds each FP64 residual A (A* y) in one pass and the lanes
    in two, so the residuals (differences of nearly equal terms) round apart and
    the inner solves they start can end an iteration or two apart."""
    import torch
    from paper_0905_4745_amd import api
    shapes = [(40, 6000), (200, 9000), (300, 20000), (512, 40000), (90, 33000)]
    say(f"batched four-step classes {bulk} {shapes}")
    systems = synth.make_batch(shapes, seed=90, kappa=1e4)
    As = [to_dev(A) for A, _ in systems]
    A_los = [a.to(torch.float32) for a in As] if bulk == "f32" else None
    bs = [to_dev(b) for _, b in systems]
    ds, idxs, Ns = _batch_inputs(shapes, 91, False, 1e4, True)
    xf, inf_f = api.minnorm_solve_batched(As, bs, 1e-10, ds, idxs, Ns, A_los=A_los,
                                          opts=api.SolveOptions(batch_form=0))
    xl, inf_l = api.minnorm_solve_batched(As, bs, 1e-10, ds, idxs, Ns, A_los=A_los,
                                          opts=api.SolveOptions(batch_form=1))
    tol = 3 if bulk == "f32" else 1
    for (A, b), a, c, ia, ic in zip(systems, xf, xl, inf_f, inf_l):
        p = oracle.refined_minnorm(A, b)
        say(f"  iters fused {ia['iters']} lanes {ic['iters']} err {rel(to_np(a), p):.2e}")
        assert ia["status"] == 0 and ic["status"] == 0
        assert rel(to_np(a), p) <= 1e-10 and rel(to_np(c), p) <= 1e-10
        assert abs(ia["iters"] - ic["iters"]) <= tol


def test_batched_fused_mixed_c128_and_fallback():
    """complex128 data with complex64 copies; one system at cond 1e6 makes the
    Gram route decline and is finished by the Householder route."""
    import torch
    from paper_0905_4745_amd import api
    shapes = [(48, 2000), (100, 6000), (32, 1500)]
    kappas = [1e3, 1e4, 1e6]
    systems = [synth.make_svd(m, n, kp, seed=60 + k)[:2] for k, ((m, n), kp) in enumerate(zip(shapes, kappas))]
    As = [to_dev(A) for A, _ in systems]
    A_los = [a.to(torch.complex64) for a in As]
    bs = [to_dev(b) for _, b in systems]
    ds, idxs, Ns = _batch_inputs(shapes, 70, True, 1e3, False)
    xs, infos = api.minnorm_solve_batched(As, bs, 1e-9, ds, idxs, Ns, A_los=A_los)
    for (A, b), x, info in zip(systems, xs, infos):
        assert info["status"] == 0
        assert rel(to_np(x), oracle.refined_minnorm(A, b)) <= 1e-9


@pytest.mark.slow
def test_mixed_kappa_1e6_512x65536():
    """complex128 data, complex64 bulk, cond 1e6 at 512 x 65536: the FP64
    refinement still certifies eps = 1e-10 against the longdouble-refined
    oracle (the rounding of the FP64 residual grows with m and n)."""
    import torch
    from paper_0905_4745_amd import api
    say("mixed c128/c64 kappa 1e6 512x65536")
    A, b, _ = synth.make_svd(512, 65536, 1e6, seed=77)
    N = 65536
    d, idx = synth.draw_srft(N, 2048, seed=77)
    At = to_dev(A)
    x, info = api.minnorm_solve(At, to_dev(b), 1e-10, d, idx, N, A_lo=At.to(torch.complex64), raise_on_status=False)
    p = oracle.refined_minnorm(A, b)
    say(f"  status {info['status']} err {rel(to_np(x), p):.2e} iters {info['iters']} refine {info['refine_steps']} "
        f"cert {info['cert_rel']:.2e} rho0 {info['rho0']:.2e} rho {info['rho']:.2e} xi {info['xi']:.2e}")
    assert info["status"] == 0
    assert rel(to_np(x), p) <= 1e-10


def test_batched_systems_reuse():
    """A batch validated once (api.BatchedSystems) and solved repeatedly: each
    solve equals the one-shot batched call with the same library draws (bitwise:
    the same kernels on the same data), and every solve meets the oracle's
    bar."""
    import torch
    from paper_0905_4745_amd import api
    shapes = [(40, 2300), (64, 5000), (32, 1000), (100, 4000)]
    systems = [synth.make_svd(m, n, 1e3, seed=80 + i)[:2] for i, (m, n) in enumerate(shapes)]
    As = [to_dev(A) for A, _ in systems]
    bs = [to_dev(b) for _, b in systems]
    A_los = [A.to(torch.complex64) for A in As]
    Ns = [synth.next_pow2(n) for _, n in shapes]
    batch = api.BatchedSystems(As, bs, Ns, A_los)
    for seed in (3, 4):
        opts = api.SolveOptions(seed=seed)
        xs, infos = batch.solve(1e-10, opts=opts)
        xs = [x.clone() for x in xs]
        ys, _ = api.minnorm_solve_batched(As, bs, 1e-10, None, None, Ns, A_los=A_los, opts=opts)
        for i, (A, b) in enumerate(systems):
            assert torch.equal(xs[i], ys[i])
            err = rel(to_np(xs[i]), oracle.refined_minnorm(A, b))
            say(f"  seed {seed} system {i}: status {infos[i]['status']} err {err:.1e}")
            assert infos[i]["status"] == 0 and err <= 1e-10
