"""HIP-graph replay of the batched lockstep iterations.

The fused batched form captures each block of check_every iterations (every
system's fused pass and CG step) once per parity of the residual ping-pong
and replays it; between replays the host reads the stop flags and, in the
mixed mode, enqueues the FP64 residual pass and the refinement update
eagerly.  Every replay's output feeds the next iteration, so the final x
and the iteration counts of the replayed run equal, bit for bit, those of
the run that launches every kernel (opts.graph = -1); both meet Theorem
5.4's guarantee against the oracle.  check_every = 3 (odd) exercises both
parities' graphs, 8 the single one.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _inputs(shapes, seed, real):
    ds, idxs, Ns = [], [], []
    for k, (m, n) in enumerate(shapes):
        N = synth.next_pow2(n)
        d, idx = synth.draw_srft(N, synth.sketch_width(m, N), seed=seed + k, real=real)
        ds.append(d), idxs.append(idx), Ns.append(N)
    return ds, idxs, Ns


@pytest.mark.parametrize("kind,ce", [("real-mixed", 8), ("real-mixed", 3), ("c128", 8), ("c128", 3)])
def test_graph_replay_matches_launches(kind, ce):
    import torch
    from paper_0905_4745_amd import api
    if kind == "real-mixed":
        shapes = [(40, 3000), (200, 9000), (64, 5000), (300, 20000), (33, 2100), (512, 8192)]
        systems = synth.make_batch(shapes, seed=120, kappa=1e4)
        real = True
    else:
        shapes = [(20, 600), (64, 5000), (37, 9000), (130, 4100)]
        systems = [synth.make_svd(m, n, 1e3, seed=130 + k)[:2] for k, (m, n) in enumerate(shapes)]
        real = False
    As = [to_dev(A) for A, _ in systems]
    A_los = [a.to(torch.float32) for a in As] if kind == "real-mixed" else None
    bs = [to_dev(b) for _, b in systems]
    ds, idxs, Ns = _inputs(shapes, 140, real)
    runs = {}
    for g in (0, -1, 0):  # replay, launches, replay again (graphs rebuilt per call)
        xs, infos = api.minnorm_solve_batched(As, bs, 1e-10, ds, idxs, Ns, A_los=A_los,
                                              opts=api.SolveOptions(check_every=ce, graph=g))
        runs.setdefault(g, []).append(([to_np(x) for x in xs], [i["iters"] for i in infos],
                                       [i["status"] for i in infos]))
    ref_x, ref_it, ref_st = runs[-1][0]
    for xs, its, sts in runs[0]:
        assert sts == ref_st and its == ref_it
        for a, b in zip(xs, ref_x):
            assert np.array_equal(a, b)
    for (A, b), x, s in zip(systems, ref_x, ref_st):
        p = oracle.refined_minnorm(A, b) if kind == "real-mixed" else oracle.classical_minnorm(A, b)
        err = rel(x, p)
        assert s == 0 and err <= 1e-10, err
    say(f"  {kind} check_every {ce}: iterations {ref_it}, replayed runs bitwise equal to launched")
