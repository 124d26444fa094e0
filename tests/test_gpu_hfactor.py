"""The paper's full SRFT T = S F D H with H = Theta Pi Z Theta~ Pi~ Z~ on the
GPU (Section 3, eqs. Rokhlin_trans, big_def), against the oracle:

* tiny N: the sketch equals the dense product S F D H [A*; 0] built from
  the oracle's dense H (rokhlin_h_matrix) and SRFT matrix;
* N = 2^16, ragged n: every column of the sketch equals the oracle's sketch
  of the rows transformed by rokhlin_h_apply, to 40 u log2(N) relative
  (the two stages' rotation chains add a few roundings per entry to the
  transform's own);
* a whole solve with H (opts.hfactor) meets Theorem 5.4's guarantee;
* a permutation entry outside [0, N) is refused (-11) before any kernel
  reads through it.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu

U = {"complex128": 1.11e-16, "complex64": 5.96e-8, "float64": 1.11e-16, "float32": 5.96e-8}


def _rows_h(A, N, hp, real):
    """Rows of A zero-padded to N, conjugated (complex), times H (oracle)."""
    m, n = A.shape
    out = np.zeros((m, N), dtype=np.float64 if real else np.complex128)
    for i in range(m):
        v = np.zeros(N, dtype=np.complex128)
        v[:n] = A[i] if real else np.conj(A[i])
        w = oracle.rokhlin_h_apply(v, *hp)
        out[i] = w.real if real else w
    return out


def _oracle_sketch_h(A, d, idx, N, hp, real):
    V = _rows_h(A, N, hp, real)
    # the oracle's sketch conjugates complex rows: hand it conj(H conj(a))
    return oracle.sketch_real(V, d, idx, N) if real else oracle.sketch(np.conj(V), d, idx, N)


@pytest.mark.parametrize("dtype", ["complex128", "float64"])
@pytest.mark.parametrize("N,n,m", [(8, 7, 3), (16, 16, 5), (64, 50, 9)])
def test_sketch_h_dense_tiny(dtype, N, n, m):
    import torch
    from paper_0905_4745_amd import api
    real = dtype == "float64"
    rng = np.random.default_rng(N + m)
    A = rng.standard_normal((m, n)) if real else synth.complex_gaussian(rng, (m, n))
    l = max(1, N // 2)
    d, idx = synth.draw_srft(N, l, seed=N, real=real)
    hp = synth.draw_hfactor(N, seed=N + 1, real=real)
    H = api.HFactor(*hp, complex_=not real)
    S = to_np(api.srft_sketch_h(to_dev(A), d, idx, N, H))
    # dense: T = S F D H, applied to [A*; 0] (real: A^T, Hartley transform)
    Hd = oracle.rokhlin_h_matrix(*hp)
    T = (oracle.srft_real_matrix(N, d, idx) if real else oracle.srft_matrix(N, d, idx)) @ Hd
    Apad = np.zeros((m, N), dtype=A.dtype)
    Apad[:, :n] = A
    S_dense = T @ (Apad.T if real else Apad.conj().T)
    if real:
        S_dense = S_dense.real
    err = np.max(np.abs(S - S_dense)) / np.max(np.abs(S_dense))
    say(f"  {dtype} N={N} n={n} m={m}: max |S - T A*| / max|T A*| = {err:.1e}")
    assert err <= 1e-13


@pytest.mark.parametrize("dtype", ["complex128", "complex64", "float32"])
def test_sketch_h_large(dtype):
    import torch
    from paper_0905_4745_amd import api
    real = not dtype.startswith("complex")
    N, n, m, l = 1 << 16, 50001, 64, 1500
    rng = np.random.default_rng(7)
    A = rng.standard_normal((m, n)) if real else synth.complex_gaussian(rng, (m, n))
    At = to_dev(A).to(getattr(torch, dtype))
    A64 = to_np(At).astype(np.float64 if real else np.complex128)
    d, idx = synth.draw_srft(N, l, seed=8, real=real)
    hp = synth.draw_hfactor(N, seed=9, real=real)
    S = to_np(api.srft_sketch_h(At, d, idx, N, api.HFactor(*hp, complex_=not real)))
    S_o = _oracle_sketch_h(A64, d, idx, N, hp, real)
    col = np.linalg.norm(S - S_o, axis=0) / np.linalg.norm(S_o, axis=0)
    tol = 40 * U[dtype] * np.log2(N)
    say(f"  {dtype}: max column rel err {col.max():.1e} (bar {tol:.1e})")
    assert col.max() <= tol


@pytest.mark.parametrize("case", ["c128", "c64-mixed"])
def test_solve_with_h(case):
    import torch
    from paper_0905_4745_amd import api
    m, n = (64, 1000) if case == "c128" else (300, 20000)
    A, b, _ = synth.make_svd(m, n, 1e3, seed=m)
    N = synth.next_pow2(n)
    l = synth.sketch_width(m, N)
    d, idx = synth.draw_srft(N, l, seed=m + 1)
    H = api.HFactor(*synth.draw_hfactor(N, seed=m + 2))
    At = to_dev(A)
    kw = {"A_lo": At.to(torch.complex64)} if case == "c64-mixed" else {}
    eps = 1e-12 if case == "c128" else 1e-10
    x, info = api.minnorm_solve(At, to_dev(b), eps, d, idx, N, opts=api.SolveOptions(hfactor=H), **kw)
    err = rel(to_np(x), oracle.classical_minnorm(A, b))
    say(f"  {case}: status {info['status']} iters {info['iters']} refine {info['refine_steps']} err {err:.1e}")
    assert info["status"] == 0 and err <= eps


def test_sketch_h_rejects_bad_permutation():
    import torch
    from paper_0905_4745_amd import api
    N = 256
    A = torch.zeros((4, 200), dtype=torch.complex128, device="cuda")
    d, idx = synth.draw_srft(N, 32, seed=1)
    hp = list(synth.draw_hfactor(N, seed=2))
    hp[4] = hp[4].copy()
    hp[4][17] = N  # out of range
    with pytest.raises(api.MinnormError) as e:
        api.srft_sketch_h(A, d, idx, N, api.HFactor(*hp))
    assert e.value.status == -11
