"""The library's own draw of Step 1's random quantities and the redraw after a
rank-deficient sketch (Remark 4.1), through the C ABI:

* srft_draw equals the oracle's independent Philox4x32-10 / Floyd draw: the
  indices bit for bit, the phases to the rounding of sin and cos;
* a solve with d = idx = NULL uses exactly that draw (bitwise the same x as
  the solve handed srft_draw's output) and meets Theorem 5.4's guarantee;
* a matrix whose first row is built so that the first draw's sketch has a
  zero column (its transformed row vanishes on every kept index) is solved
  after one redraw (info.retries == 1); with redraws switched off, or for a
  matrix that is not of full rank, +1 is returned (after 0, resp. 2 redraws);
* the batched call draws every system (sys = its index) and redraws the
  forced system alone; its one-launch draw of all systems' phases and its
  single copy of the index sets give bit for bit the solutions of the call
  handed srft_draw's output.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,N,l,seed,draw,sys", [
    ("complex128", 4096, 1000, 0, 0, 0),
    ("complex64", 1 << 18, 8192, 12345678901234, 2, 5),
    ("float64", 4096, 4096, 7, 1, 0),
    ("float32", 1 << 16, 300, 2**63 + 11, 0, 3),
])
def test_draw_matches_oracle(dtype, N, l, seed, draw, sys):
    import torch
    from paper_0905_4745_amd import api
    tdt = getattr(torch, dtype)
    real = not tdt.is_complex
    d, idx = api.srft_draw(tdt, seed, draw, sys, N, l)
    d_o, idx_o = oracle.draw_srft(seed, draw, sys, N, l, real=real)
    assert np.array_equal(to_np(idx), idx_o)
    dd = to_np(d)
    if real:
        assert np.array_equal(dd, d_o)
    else:
        # the oracle rounds the argument 2 pi u (relative error u64, so up to
        # 2 pi u64 absolute in the phase) before exp; the library evaluates
        # cos and sin of pi (2u) with an exact argument: both are within a
        # few ulp of exp(2 pi i u), hence 2 pi u64 + 4 u64
        err = float(np.max(np.abs(dd - d_o)))
        say(f"  N={N} l={l}: max |d - d_oracle| = {err:.1e}")
        assert err <= (2 * np.pi + 4) * 1.11e-16


def _forced_row(d, idx, N, real):
    """A row whose transform under (d, idx) vanishes on every kept index."""
    k = int(np.setdiff1d(np.arange(N), idx)[0])
    j = np.arange(N)
    if real:
        cas = (np.cos(2 * np.pi * j * k / N) + np.sin(2 * np.pi * j * k / N)) / np.sqrt(N)
        return d * cas
    return d * np.exp(-2j * np.pi * j * k / N) / np.sqrt(N)


def _forced_problem(m, N, seed, sys, real, rng):
    d0, idx0 = oracle.draw_srft(seed, 0, sys, N, 4 * m, real=real)
    if real:
        A = rng.standard_normal((m, N))
        b = rng.standard_normal(m)
    else:
        A = synth.complex_gaussian(rng, (m, N))
        b = synth.complex_gaussian(rng, (m,))
    A[0] = _forced_row(d0, idx0, N, real)
    S = oracle.sketch_real(A, d0, idx0, N) if real else oracle.sketch(A, d0, idx0, N)
    assert np.linalg.norm(S[:, 0]) < 1e-12 * np.linalg.norm(S)  # the first draw's sketch loses a column
    return A, b


def test_library_draw_is_srft_draw():
    from paper_0905_4745_amd import api
    import torch
    A, b = synth.make_gaussian(64, 1000, seed=3)
    N = 1024
    opts = api.SolveOptions(seed=99)
    x1, info1 = api.minnorm_solve(to_dev(A), to_dev(b), 1e-12, None, None, N, opts=opts)
    d, idx = api.srft_draw(torch.complex128, 99, 0, 0, N, 256)
    x2, info2 = api.minnorm_solve(to_dev(A), to_dev(b), 1e-12, d, idx, N)
    assert info1["status"] == 0 and info1["retries"] == 0
    assert torch.equal(x1, x2) and info1["iters"] == info2["iters"]
    assert rel(to_np(x1), oracle.classical_minnorm(A, b)) <= 1e-12


@pytest.mark.parametrize("real", [False, True])
def test_redraw_after_rank_deficient_sketch(real):
    from paper_0905_4745_amd import api
    rng = np.random.default_rng(5)
    m, N, seed = 8, 256, 4242
    A, b = _forced_problem(m, N, seed, 0, real, rng)
    p = oracle.classical_minnorm(A, b)
    x, info = api.minnorm_solve(to_dev(A), to_dev(b), 1e-12, None, None, N, opts=api.SolveOptions(seed=seed),
                                raise_on_status=False)
    say(f"  forced: status {info['status']} retries {info['retries']} err {rel(to_np(x), p):.1e}")
    assert info["status"] == 0 and info["retries"] == 1
    assert rel(to_np(x), p) <= 1e-12
    # no redraws allowed: the rank-deficient first draw is reported
    _, info = api.minnorm_solve(to_dev(A), to_dev(b), 1e-12, None, None, N,
                                opts=api.SolveOptions(seed=seed, max_reseed=-1), raise_on_status=False)
    assert info["status"] == 1 and info["retries"] == 0
    # a matrix that is not of full rank fails every draw
    A2 = A.copy()
    A2[1] = A2[2]
    _, info = api.minnorm_solve(to_dev(A2), to_dev(b), 1e-12, None, None, N, opts=api.SolveOptions(seed=seed),
                                raise_on_status=False)
    assert info["status"] == 1 and info["retries"] == 2


def test_batched_library_draws_and_redraw():
    from paper_0905_4745_amd import api
    rng = np.random.default_rng(8)
    seed = 77
    shapes = [(8, 300), (16, 1000), (12, 512), (40, 4000)]
    As, bs, Ns = [], [], []
    for i, (m, n) in enumerate(shapes):
        N = synth.next_pow2(n)
        if i == 2:
            A, b = _forced_problem(m, N, seed, 2, False, rng)  # n = N for the forced row
        else:
            A, b = synth.complex_gaussian(rng, (m, n)), synth.complex_gaussian(rng, (m,))
        As.append(A), bs.append(b), Ns.append(N)
    xs, infos = api.minnorm_solve_batched([to_dev(A) for A in As], [to_dev(b) for b in bs], 1e-12, None, None, Ns,
                                          opts=api.SolveOptions(seed=seed), raise_on_status=False)
    for i, (A, b) in enumerate(zip(As, bs)):
        err = rel(to_np(xs[i]), oracle.classical_minnorm(A, b))
        say(f"  system {i}: status {infos[i]['status']} retries {infos[i]['retries']} err {err:.1e}")
        assert infos[i]["status"] == 0
        assert infos[i]["retries"] == (1 if i == 2 else 0)
        assert err <= 1e-12


@pytest.mark.parametrize("real", [False, True])
def test_batched_library_draws_equal_srft_draw(real):
    """The batched call's own draws (every system's phases in one launch, the
    index sets staged and copied at once) are the draws srft_draw makes for
    (seed, draw 0, sys = the system's index): the solutions of the call that
    draws and of the call handed srft_draw's output agree bit for bit, on
    systems of uneven m and N (powers of two and N1 2^k)."""
    import torch
    from paper_0905_4745_amd import api
    rng = np.random.default_rng(31)
    seed = 424242
    shapes = [(24, 900), (48, 2000), (16, 700), (64, 5000), (32, 1500)]
    As, bs, Ns = [], [], []
    for m, n in shapes:
        if real:
            A, b = rng.standard_normal((m, n)), rng.standard_normal(m)
        else:
            A, b = synth.complex_gaussian(rng, (m, n)), synth.complex_gaussian(rng, (m,))
        As.append(to_dev(A))
        bs.append(to_dev(b))
        Ns.append(synth.next_fft_len(n))
    assert any(N & (N - 1) for N in Ns)  # some lengths are not powers of two
    ls = [min(4 * m, N) for (m, _), N in zip(shapes, Ns)]
    opts = api.SolveOptions(seed=seed)
    xs_lib, inf_lib = api.minnorm_solve_batched(As, bs, 1e-12, None, None, Ns, opts=opts, ls=ls)
    tdt = torch.float64 if real else torch.complex128
    ds, idxs = [], []
    for i, (N, l) in enumerate(zip(Ns, ls)):
        d, idx = api.srft_draw(tdt, seed, 0, i, N, l)
        ds.append(d)
        idxs.append(idx)
    xs_cal, inf_cal = api.minnorm_solve_batched(As, bs, 1e-12, ds, idxs, Ns, opts=opts)
    for i in range(len(shapes)):
        say(f"  system {i} N={Ns[i]} l={ls[i]}: status {inf_lib[i]['status']} / {inf_cal[i]['status']}, "
            f"iters {inf_lib[i]['iters']} / {inf_cal[i]['iters']}")
        assert inf_lib[i]["status"] == 0 and inf_cal[i]["status"] == 0
        assert inf_lib[i]["retries"] == 0
        assert torch.equal(xs_lib[i], xs_cal[i])
