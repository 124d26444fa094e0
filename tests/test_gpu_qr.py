"""GPU parity of Step 2's factorisation (build_preconditioner).

R is unique up to a diagonal unitary factor; after normalising diag(R) to be
real and positive the GPU R must match the oracle's Householder R to
20 u cond(S) ||S|| (forward error of Householder QR), and R* R = S* S must
hold to 20 u sqrt(l) ||S||^2 (backward stability).
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu

U64, U32 = 1.11e-16, 5.96e-8


@pytest.mark.parametrize("l,m", [(4, 1), (32, 32), (64, 16), (256, 64), (300, 70), (600, 150), (2048, 512)])
@pytest.mark.parametrize("kind", ["c128", "c64", "f64", "f32"])
def test_qr_parity(l, m, kind):
    import torch
    from paper_0905_4745_amd import api
    say(f"qr {kind} l={l} m={m}")
    real = kind.startswith("f")
    g = np.random.default_rng(l + m)
    S = g.standard_normal((l, m)) if real else synth.complex_gaussian(g, (l, m))
    tdt = {"c128": torch.complex128, "c64": torch.complex64, "f64": torch.float64, "f32": torch.float32}[kind]
    # column-major device copy: a row-major (m, l) buffer viewed transposed
    St = to_dev(np.ascontiguousarray(S.T), tdt).t()
    S_used = to_np(St).astype(np.float64 if real else np.complex128)
    R = to_np(api.build_preconditioner(St)).astype(S_used.dtype)
    u = U32 if kind in ("c64", "f32") else U64
    nS = np.linalg.norm(S_used, 2)
    assert np.allclose(np.tril(R, -1), 0)
    assert np.max(np.abs(np.imag(np.diagonal(R)))) == 0
    back = np.linalg.norm(R.conj().T @ R - S_used.conj().T @ S_used, 2)
    say(f"  backward {back / nS**2:.2e}")
    assert back <= 20 * u * np.sqrt(l) * nS ** 2
    Ro, _, _ = oracle.householder_qr(S_used)
    kap = np.linalg.cond(S_used)
    fwd = np.linalg.norm(oracle.normalize_r(R) - oracle.normalize_r(Ro), 2)
    say(f"  forward {fwd / nS:.2e} (cond {kap:.1e})")
    assert fwd <= 20 * u * kap * nS


def test_qr_rank_deficient_flagged():
    import torch
    from paper_0905_4745_amd import api
    g = np.random.default_rng(0)
    S = synth.complex_gaussian(g, (128, 40))
    S[:, 17] = S[:, 3]  # two equal columns
    St = to_dev(np.ascontiguousarray(S.T)).t()
    with pytest.raises(api.MinnormError) as e:
        api.build_preconditioner(St)
    assert e.value.status == 1
    S[:, 17] = 0.0  # a zero column
    St = to_dev(np.ascontiguousarray(S.T)).t()
    with pytest.raises(api.MinnormError) as e:
        api.build_preconditioner(St)
    assert e.value.status == 1
