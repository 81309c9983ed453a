"""Step 1's CG replayed from captured graphs equals eager launches bit for bit.

Each step replays the captured chunks many times with eager work (the other
phases of the step, host convergence checks) in between; the iterates, the
diagnostics and the CG iteration counts must match a context that launches
every kernel eagerly, in FP64 and in mixed precision, in 2D and 3D.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import say, to_host

pytestmark = pytest.mark.gpu


def _dev(a, prec):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64 if prec == 0 else np.float32)).to("cuda")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mk,tau,steps", [(lambda: W.harmonic_2d_32(), 0.1, 6),
                                          (lambda: W.wells_3d(m=20, N=12, seed=4), 30.0, 12)])
def test_graph_chunks_equal_eager(prec, mk, tau, steps):
    from paper_2511_06788_amd import ope
    p = mk()
    say(f"graphs vs eager {p.name} prec={prec}")
    out = []
    for graphs in (True, False):
        with ope.Context(p.grid, p.V, p.N, kinetic=p.kinetic, shift=p.shift, precision=prec) as ctx:
            ope.ope_set_graphs(ctx.handle, graphs)
            U = _dev(p.U0, prec)
            infos = [ope.ope_step(ctx.handle, U, tau) for _ in range(steps)]
            si = ope.ope_solve(ctx.handle, U, tau, 0.0, 3)
            out.append((to_host(U), [(i.energy, i.residual, i.drift, i.inner_iterations) for i in infos],
                        (si.residual, si.inner_iterations)))
    (Ug, ig, sg), (Ue, ie, se) = out
    assert np.array_equal(Ug, Ue)
    assert ig == ie
    assert sg == se
    assert sum(i[3] for i in ig) > 4 * steps      # the chunks did run
