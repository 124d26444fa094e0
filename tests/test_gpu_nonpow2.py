"""Transform lengths that are not powers of two (eq. DFT holds for every
length; Section 3): N = N1 2^k with 2^k >= 256 and any N1, run by the
kept-outputs-only form of Step 1, whose identity
V[k] = sum_{n1} W_N^{n1 k} Z_{n1}[k mod 2^k] holds for any N1 (pinned on the
CPU in test_oracle_transforms.py).

* Step 1 against the oracle's FFT sketch at 20 u log2(N) per column, for
  N = 3, 5, 79, 1000 times 256 and 3 x 2^14, 5 x 2^12, ragged n, every dtype,
  l at the 256- and 512-thread forms' capacities;
* whole solves with such N (caller's draw and the library's draw) meet
  Theorem 5.4's guarantee against the oracle;
* the batched form with such N_i agrees with the oracle system by system.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu

U64, U32 = 1.11e-16, 5.96e-8

CASES = [
    # (m, n, N, l)
    (5, 700, 768, 50),          # 3 x 256: one partial block of columns
    (7, 1200, 1280, 300),       # 5 x 256
    (6, 20000, 20480, 1000),    # 5 x 4096
    (9, 20000, 20224, 2048),    # 79 x 256, l at the 256-thread complex128 capacity
    (4, 49000, 49152, 4000),    # 3 x 2^14, l beyond it: the 512-thread form
]


def _colerr(Sg, Sr):
    return max(float(np.linalg.norm(Sg[:, i] - Sr[:, i]) / max(np.linalg.norm(Sr[:, i]), 1e-300))
               for i in range(Sr.shape[1]))


def _sketch_case(m, n, N, l, kind):
    import torch
    from paper_0905_4745_amd import api
    real = kind.startswith("f")
    g = np.random.default_rng(m * 7 + n)
    A = g.standard_normal((m, n)) if real else synth.complex_gaussian(g, (m, n))
    d, idx = synth.draw_srft(N, l, seed=N + l, real=real)
    tdt = {"c128": torch.complex128, "c64": torch.complex64, "f64": torch.float64, "f32": torch.float32}[kind]
    At = to_dev(A, tdt)
    A_used = to_np(At).astype(np.float64 if real else np.complex128)
    S = to_np(api.srft_sketch(At, d, idx, N))
    ref = oracle.sketch_real(A_used, d, idx, N) if real else oracle.sketch(A_used, d, idx, N)
    u = U32 if kind in ("c64", "f32") else U64
    err = _colerr(S.astype(ref.dtype), ref)
    say(f"  {kind} m={m} n={n} N={N} l={l}: col rel err {err:.2e} (bar {20 * u * np.log2(N):.1e})")
    assert err <= 20 * u * np.log2(N)


@pytest.mark.parametrize("m,n,N,l", CASES)
@pytest.mark.parametrize("kind", ["c128", "c64", "f64", "f32"])
def test_sketch_nonpow2(m, n, N, l, kind):
    _sketch_case(m, n, N, l, kind)


@pytest.mark.parametrize("kind", ["c64", "f32"])
def test_sketch_nonpow2_single_wide_l(kind):
    # 1000 x 256 with l = 8000: single precision holds 32 outputs per thread
    _sketch_case(3, 250000, 256000, 8000, kind)


@pytest.mark.parametrize("draw", ["caller", "library"])
def test_solve_nonpow2_c128(draw):
    from paper_0905_4745_amd import api
    m, n = 64, 1100
    N = synth.next_fft_len(n)
    assert N == 1280
    A, b, _ = synth.make_svd(m, n, 1e3, seed=21)
    l = synth.sketch_width(m, N)
    if draw == "caller":
        d, idx = synth.draw_srft(N, l, seed=22)
        x, info = api.minnorm_solve(to_dev(A), to_dev(b), 1e-12, d, idx, N)
    else:
        x, info = api.minnorm_solve(to_dev(A), to_dev(b), 1e-12, None, None, N, l=l)
    err = rel(to_np(x), oracle.classical_minnorm(A, b))
    say(f"  c128 N={N} ({draw} draw): status {info['status']} iters {info['iters']} err {err:.1e}")
    assert info["status"] == 0 and err <= 1e-12


def test_solve_nonpow2_real():
    from paper_0905_4745_amd import api
    m, n = 100, 5000
    N = synth.next_fft_len(n)
    assert N == 5120
    rng = np.random.default_rng(4)
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=5, real=True)
    x, info = api.minnorm_solve(to_dev(A), to_dev(b), 1e-12, d, idx, N)
    err = rel(to_np(x), oracle.classical_minnorm(A, b))
    say(f"  f64 N={N}: status {info['status']} iters {info['iters']} err {err:.1e}")
    assert info["status"] == 0 and err <= 1e-12


def test_solve_nonpow2_mixed():
    import torch
    from paper_0905_4745_amd import api
    m, n = 300, 20000
    N = synth.next_fft_len(n)
    assert N == 20224
    A, b, _ = synth.make_svd(m, n, 1e6, seed=6)
    d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=7)
    At = to_dev(A)
    x, info = api.minnorm_solve(At, to_dev(b), 1e-10, d, idx, N, A_lo=At.to(torch.complex64))
    err = rel(to_np(x), oracle.refined_minnorm(A, b))
    say(f"  mixed N={N}: status {info['status']} iters {info['iters']} refine {info['refine_steps']} err {err:.1e}")
    assert info["status"] == 0 and err <= 1e-10


def test_batched_nonpow2():
    from paper_0905_4745_amd import api
    shapes = [(40, 2300), (64, 5000), (32, 1000)]
    systems = [synth.make_svd(m, n, 1e2, seed=60 + i)[:2] for i, (m, n) in enumerate(shapes)]
    Ns = [synth.next_fft_len(n) for _, n in shapes]
    assert Ns == [2304, 5120, 1024]
    ds, idxs = [], []
    for i, (m, _) in enumerate(shapes):
        d, idx = synth.draw_srft(Ns[i], synth.sketch_width(m, Ns[i]), seed=70 + i)
        ds.append(d)
        idxs.append(idx)
    xs, infos = api.minnorm_solve_batched([to_dev(A) for A, _ in systems], [to_dev(b) for _, b in systems],
                                          [1e-12] * 3, ds, idxs, Ns)
    for i, (A, b) in enumerate(systems):
        err = rel(to_np(xs[i]), oracle.classical_minnorm(A, b))
        say(f"  system {i} N={Ns[i]}: status {infos[i]['status']} err {err:.1e}")
        assert infos[i]["status"] == 0 and err <= 1e-12
