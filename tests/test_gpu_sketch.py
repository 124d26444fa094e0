"""GPU parity of Step 1 (srft_sketch) against the oracle's FFT sketch.

Same (d, idx) on both sides.  Bar: per column of S, the relative error is
at most 20 u log2(N) (u the unit roundoff of the kernel's precision): a
radix-staged FFT with correctly rounded twiddles has error O(u log N).
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu

U64, U32 = 1.11e-16, 5.96e-8

CASES = [
    # (m, n, N, l): tiny, ragged n, one-workgroup FFT, four-step FFT
    (1, 2, 2, 2),
    (3, 13, 16, 9),
    (5, 50, 64, 20),
    (64, 1000, 1024, 256),
    (37, 1024, 1024, 148),
    (33, 4096, 4096, 132),
    (33, 5000, 8192, 132),
    (17, 65536, 65536, 68),
    (3, 100000, 131072, 12),
    (2, 262144, 262144, 8),
]


def _colerr(Sg, Sr):
    return max(float(np.linalg.norm(Sg[:, i] - Sr[:, i]) / max(np.linalg.norm(Sr[:, i]), 1e-300))
               for i in range(Sr.shape[1]))


@pytest.mark.parametrize("m,n,N,l", CASES)
@pytest.mark.parametrize("kind", ["c128", "c64", "f64", "f32"])
def test_sketch_parity(m, n, N, l, kind):
    import torch
    from paper_0905_4745_amd import api
    say(f"sketch {kind} m={m} n={n} N={N} l={l}")
    real = kind.startswith("f")
    g = np.random.default_rng(m * 7 + n)
    if real:
        A = g.standard_normal((m, n))
    else:
        A = synth.complex_gaussian(g, (m, n))
    d, idx = synth.draw_srft(N, l, seed=N + l, real=real)
    tdt = {"c128": torch.complex128, "c64": torch.complex64, "f64": torch.float64, "f32": torch.float32}[kind]
    At = to_dev(A, tdt)
    A_used = to_np(At).astype(np.float64 if real else np.complex128)
    S = to_np(api.srft_sketch(At, d, idx, N))
    ref = oracle.sketch_real(A_used, d, idx, N) if real else oracle.sketch(A_used, d, idx, N)
    u = U32 if kind in ("c64", "f32") else U64
    err = _colerr(S.astype(ref.dtype), ref)
    say(f"  col rel err {err:.2e}")
    assert err <= 20 * u * max(np.log2(N), 1)


def test_sketch_rows_of_identity_give_orthonormal_T():
    """A = I (N x N): S = T, so S S^* = I_l through the GPU kernel."""
    import torch
    from paper_0905_4745_amd import api
    N, l = 64, 24
    d, idx = synth.draw_srft(N, l, seed=3)
    T = to_np(api.srft_sketch(to_dev(np.eye(N, dtype=np.complex128)), d, idx, N))
    assert np.allclose(T @ T.conj().T, np.eye(l), atol=1e-13)
    assert np.allclose(T, oracle.srft_matrix(N, d, idx), atol=1e-14)


def test_sketch_invalid_idx_rejected():
    import torch
    from paper_0905_4745_amd import api
    A = to_dev(np.ones((2, 8), dtype=np.complex128))
    d, idx = synth.draw_srft(8, 4, seed=1)
    with pytest.raises(api.MinnormError) as e:
        api.srft_sketch(A, d, np.array([0, 3, 3, 5], dtype=np.int32), 8)
    assert e.value.status == -10
    with pytest.raises(api.MinnormError) as e:
        api.srft_sketch(A, d, np.array([0, 3, 5, 8], dtype=np.int32), 8)
    assert e.value.status == -10


@pytest.mark.parametrize("m,n,N,l", [(17, 65536, 65536, 68), (3, 100000, 131072, 12), (5, 8192, 8192, 20)])
@pytest.mark.parametrize("kind", ["c128", "f32"])
@pytest.mark.parametrize("split", [1, 2])
def test_sketch_four_step_splits(m, n, N, l, kind, split, tmp_path):
    """Each four-step split (N2 halved `split` times) forced through a loaded
    plan gives the same sketch, to the same bar."""
    import json
    import torch
    from paper_0905_4745_amd import api
    say(f"sketch split {split} {kind} m={m} n={n} N={N}")
    real = kind.startswith("f")
    g = np.random.default_rng(m * 11 + n)
    A = g.standard_normal((m, n)) if real else synth.complex_gaussian(g, (m, n))
    d, idx = synth.draw_srft(N, l, seed=N + 3 * l, real=real)
    tdt = {"c128": torch.complex128, "f32": torch.float32}[kind]
    dcode = {"c128": 0, "f32": 3}[kind]
    plan = (split << 17) | 64
    path = tmp_path / "plans.json"
    path.write_text(json.dumps({"format": "minnorm-plans-1",
                                "plans": {f"sketch_chunk_mb/{dcode}/{m}/{N}/0": plan}, "best_ms": {}}))
    api.plans_load(str(path))
    At = to_dev(A, tdt)
    A_used = to_np(At).astype(np.float64 if real else np.complex128)
    S = to_np(api.srft_sketch(At, d, idx, N))
    ref = oracle.sketch_real(A_used, d, idx, N) if real else oracle.sketch(A_used, d, idx, N)
    u = U32 if kind == "f32" else U64
    err = _colerr(S.astype(ref.dtype), ref)
    say(f"  col rel err {err:.2e}")
    assert err <= 20 * u * max(np.log2(N), 1)


@pytest.mark.parametrize("m,n,N,l", [(17, 65536, 65536, 68), (5, 8192, 8192, 2048), (3, 100000, 131072, 700),
                                     (9, 40000, 65536, 1100), (3, 50000, 65536, 3000), (2, 100000, 131072, 8192)])
@pytest.mark.parametrize("kind", ["c128", "c64", "f64", "f32"])
@pytest.mark.parametrize("bcode,lgng", [(1, 0), (1, 2), (2, 1), (3, 0), (3, 3)])
def test_sketch_pruned_variants(m, n, N, l, kind, bcode, lgng, tmp_path):
    """The kept-outputs-only four-step (B = 16, 8, 4 columns per block; 1 to
    8 column groups per row, partial sums folded) forced through a loaded
    plan gives the oracle's sketch to the same bar, including ragged n,
    l = 2048 (eight kept outputs per thread) and, in single precision,
    l = 3000 and 8192 (16 and 32 per thread; FP64 takes the full four-step
    there)."""
    import json
    import torch
    from paper_0905_4745_amd import api
    say(f"sketch pruned b{bcode} ng{1 << lgng} {kind} m={m} n={n} N={N} l={l}")
    real = kind.startswith("f")
    g = np.random.default_rng(m * 13 + n + l)
    A = g.standard_normal((m, n)) if real else synth.complex_gaussian(g, (m, n))
    d, idx = synth.draw_srft(N, l, seed=N + 5 * l, real=real)
    tdt = {"c128": torch.complex128, "c64": torch.complex64, "f64": torch.float64, "f32": torch.float32}[kind]
    dcode = {"c128": 0, "c64": 1, "f64": 2, "f32": 3}[kind]
    plan = 64 | (bcode << 19) | (lgng << 21)
    path = tmp_path / "plans.json"
    path.write_text(json.dumps({"format": "minnorm-plans-1",
                                "plans": {f"sketch_chunk_mb/{dcode}/{m}/{N}/0": plan}, "best_ms": {}}))
    api.plans_load(str(path))
    At = to_dev(A, tdt)
    A_used = to_np(At).astype(np.float64 if real else np.complex128)
    S = to_np(api.srft_sketch(At, d, idx, N))
    ref = oracle.sketch_real(A_used, d, idx, N) if real else oracle.sketch(A_used, d, idx, N)
    u = U32 if kind in ("c64", "f32") else U64
    err = _colerr(S.astype(ref.dtype), ref)
    say(f"  col rel err {err:.2e}")
    assert err <= 20 * u * max(np.log2(N), 1)


@pytest.mark.parametrize("m,n,N,l", [(3, 50000, 65536, 3000), (2, 100000, 131072, 8192), (4, 262144, 262144, 8192),
                                     (2, 131072, 131072, 16384), (5, 30000, 32768, 600), (3, 70000, 131072, 4096)])
@pytest.mark.parametrize("kind", ["c128", "c64", "f64", "f32"])
@pytest.mark.parametrize("bcode,lgng", [(1, 0), (2, 1), (3, 0), (3, 2)])
def test_sketch_pruned_wide_variants(m, n, N, l, kind, bcode, lgng, tmp_path):
    """The kept-outputs-only form with the wide 512-thread workgroup (N2 =
    8192 / B points per column: N2 = 2048 at B = 4, so that the outer sum
    costs about 8 N flops per row at l = 8192) forced through a loaded plan:
    the oracle's sketch to the same bar, for every B, with and without
    partial sums, up to l = 16384 in single precision (32 kept outputs per
    thread) and l = 4096 in double (FP64 takes the full four-step beyond)."""
    import json
    import torch
    from paper_0905_4745_amd import api
    say(f"sketch pruned wide b{bcode} ng{1 << lgng} {kind} m={m} n={n} N={N} l={l}")
    real = kind.startswith("f")
    g = np.random.default_rng(m * 17 + n + l)
    A = g.standard_normal((m, n)) if real else synth.complex_gaussian(g, (m, n))
    d, idx = synth.draw_srft(N, l, seed=N + 7 * l, real=real)
    tdt = {"c128": torch.complex128, "c64": torch.complex64, "f64": torch.float64, "f32": torch.float32}[kind]
    dcode = {"c128": 0, "c64": 1, "f64": 2, "f32": 3}[kind]
    plan = 64 | (bcode << 19) | (lgng << 21) | (1 << 25)
    path = tmp_path / "plans.json"
    path.write_text(json.dumps({"format": "minnorm-plans-1",
                                "plans": {f"sketch_chunk_mb/{dcode}/{m}/{N}/0": plan}, "best_ms": {}}))
    api.plans_load(str(path))
    At = to_dev(A, tdt)
    A_used = to_np(At).astype(np.float64 if real else np.complex128)
    S = to_np(api.srft_sketch(At, d, idx, N))
    ref = oracle.sketch_real(A_used, d, idx, N) if real else oracle.sketch(A_used, d, idx, N)
    u = U32 if kind in ("c64", "f32") else U64
    err = _colerr(S.astype(ref.dtype), ref)
    say(f"  col rel err {err:.2e}")
    assert err <= 20 * u * max(np.log2(N), 1)
