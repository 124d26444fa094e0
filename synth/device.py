"""Seeded test problems generated on the GPU with torch, for shapes whose host
generation would take minutes (a QR of an n x m Gaussian with n = 262144).
Same recipe as `make_svd` in gen.py (Haar factors by QR with the phase
correction, sigma log-spaced 1 -> 1/kappa, Gaussian b); the random stream is
torch's seeded generator on the device, so values differ from gen.py's.
"""

from __future__ import annotations

import math


def _haar(gen, rows: int, cols: int, device):
    import torch
    g = torch.randn((rows, cols), dtype=torch.complex128, device=device, generator=gen)  # Re, Im ~ N(0, 1/2)
    q, r = torch.linalg.qr(g, mode="reduced")
    d = torch.diagonal(r)
    ph = d / torch.where(d.abs() == 0, torch.ones_like(d.abs()), d.abs())
    return q * ph[None, :]


def make_svd_device(m: int, n: int, kappa: float, seed: int, device="cuda"):
    """(A, b) on `device`: A = U diag(sigma) V* complex128, U m x m, V n x m Haar."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    U = _haar(gen, m, m, device)
    V = _haar(gen, n, m, device)
    sigma = torch.logspace(0.0, -math.log10(kappa), m, dtype=torch.float64, device=device)
    A = (U * sigma[None, :].to(U.dtype)) @ V.conj().T.contiguous()
    b = torch.randn((m,), dtype=torch.complex128, device=device, generator=gen)
    return A, b
