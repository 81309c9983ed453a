"""GPU tests of the batched form (many independent problems stepped together).

* Each problem's batched steps equal ope_step on its own context bit for bit
  (FP64 and mixed, ragged grids and block widths, 2D and 3D, with shared CG
  launches over all problems and with per-problem launches), with the same
  diagnostics; ope_batch_solve equals per-problem ope_solve.
* After the autotuner has changed the sweep shapes, converged batched solves
  still give the dense-eigensolver Ritz values to 1e-10.
* The full batched workload (64 problems, grid edges 24..48, N 16..128) runs
  a step with every invariant intact, and sampled problems' first-step
  energies and residuals equal the CPU oracle's.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W
from tests.gpu_common import say, to_host

pytestmark = pytest.mark.gpu


def _dev(a, prec):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64 if prec == 0 else np.float32)).to("cuda")


def _ragged():
    return [W.wells_3d(m=13, N=5, seed=1), W.wells_3d(m=20, N=17, seed=2), W.harmonic_2d_32(),
            W.wells_3d(m=16, N=34, seed=3), W.wells_3d(m=11, N=3, seed=4), W.wells_3d(m=28, N=48, seed=5)]


@pytest.mark.parametrize("shared", [True, False])
@pytest.mark.parametrize("prec", [0, 1])
def test_batch_steps_equal_single_steps(prec, shared):
    from paper_2511_06788_amd import ope
    probs = _ragged()
    say(f"batch steps vs single prec={prec} shared={shared}")
    # the batch takes one tau for every problem
    tau = 0.5
    with ope.Batch(probs, precision=prec) as b:
        b.set_shared(shared)
        Ub = [_dev(p.U0, prec) for p in probs]
        infos_b = [b.step(Ub, tau) for _ in range(3)]
        Ub = [to_host(U) for U in Ub]
    for i, p in enumerate(probs):
        with ope.Context(p.grid, p.V, p.N, kinetic=p.kinetic, shift=p.shift, precision=prec) as ctx:
            U = _dev(p.U0, prec)
            infos = [ope.ope_step(ctx.handle, U, tau) for _ in range(3)]
            U = to_host(U)
        assert np.array_equal(U, Ub[i]), i
        for k in range(3):
            a, c = infos[k], infos_b[k][i]
            assert (a.energy, a.residual, a.drift, a.inner_iterations) == (c.energy, c.residual, c.drift,
                                                                            c.inner_iterations), (i, k)


def test_batch_solve_equals_single_solves():
    from paper_2511_06788_amd import ope
    # N = 4 closes the lowest two box shells (a wide gap); N = 9 sits inside a shell
    probs = [W.wells_3d(m=12, N=4, seed=5), W.wells_3d(m=15, N=9, seed=6), W.wells_3d(m=10, N=4, seed=7)]
    tau = 30.0
    say("batch solve vs single")
    with ope.Batch(probs) as b:
        Ub = [_dev(p.U0, 0) for p in probs]
        sb = b.solve(Ub, tau, 1e-7, 600)
        Ub = [to_host(U) for U in Ub]
    for i, p in enumerate(probs):
        with ope.Context(p.grid, p.V, p.N) as ctx:
            U = _dev(p.U0, 0)
            si = ope.ope_solve(ctx.handle, U, tau, 1e-7, 600)
            U = to_host(U)
        assert np.array_equal(U, Ub[i]), i
        assert (si.steps, si.converged, si.inner_iterations, si.residual) == (
            sb[i].steps, sb[i].converged, sb[i].inner_iterations, sb[i].residual)
    assert sum(s.converged for s in sb) >= 2


def test_autotuned_batch_converges_to_dense_eigenvalues():
    from paper_2511_06788_amd import ope
    # block widths at shell closures, so that 1e-11 is reached in a few hundred steps
    probs = [W.wells_3d(m=10, N=4, seed=8), W.wells_3d(m=17, N=4, seed=9), W.wells_3d(m=25, N=1, seed=10)]
    tau = 30.0
    say("autotuned batch solve")
    with ope.Batch(probs) as b:
        k = b.autotune()
        assert k == 3
        Ub = [_dev(p.U0, 0) for p in probs]
        sb = b.solve(Ub, tau, 1e-11, 2000)
        ritz = [ope.ope_residual(b.context(i), Ub[i], p.N)[1] for i, p in enumerate(probs)]
        drift = [ope.ope_residual(b.context(i), Ub[i], p.N, want_ritz=False)[2] for i, p in enumerate(probs)]
    for i, p in enumerate(probs):
        H = O.assemble_H(O.Operator(p.grid.m, p.grid.h, p.V)).tocsc()
        w = np.sort(spla.eigsh(H, k=p.N + 2, sigma=0, return_eigenvectors=False))[:p.N]
        assert sb[i].converged == 1
        assert np.max(np.abs(ritz[i] - w) / np.abs(w)) <= 1e-10, i
        assert drift[i] <= 1e-12


def test_autotuned_mixed_batch_steps():
    """The autotuner on FP32 (mixed) problems: after it has picked their sweep
    shapes, mixed batch steps lower the energy and keep the drift small, and
    the first step's energy equals the oracle's energy of the start block."""
    from paper_2511_06788_amd import ope
    probs = [W.wells_3d(m=14, N=9, seed=21), W.wells_3d(m=19, N=32, seed=22), W.wells_3d(m=12, N=17, seed=23)]
    say("autotuned mixed batch")
    with ope.Batch(probs, precision=1) as b:
        assert b.autotune() >= 1
        Ub = [_dev(p.U0, 1) for p in probs]
        i1 = b.step(Ub, 30.0)
        i2 = b.step(Ub, 30.0)
    for i, p in enumerate(probs):
        op = O.Operator(p.grid.m, p.grid.h, p.V)
        U32 = p.U0.astype(np.float32).astype(np.float64)
        assert abs(i1[i].energy - O.energy(op, U32)) <= 1e-6 * abs(i1[i].energy), i
        assert i2[i].energy < i1[i].energy, i
        assert i2[i].drift <= 1e-6, i


def test_full_batched_workload_one_step():
    from paper_2511_06788_amd import ope
    probs = W.batched_problems(64)
    tau = 30.0
    say("full batched workload")
    with ope.Batch(probs) as b:
        b.autotune()
        Ub = [_dev(p.U0, 0) for p in probs]
        i1 = b.step(Ub, tau)
        i2 = b.step(Ub, tau)
    for i in range(len(probs)):
        assert i1[i].status in (0, ope.OPE_ECG_MAXIT)
        assert i2[i].energy < i1[i].energy, i
        assert i2[i].drift <= 1e-12, i
    for i in (0, 17, 63):
        p = probs[i]
        op = O.Operator(p.grid.m, p.grid.h, p.V)
        assert abs(i1[i].energy - O.energy(op, p.U0)) <= 1e-12 * abs(i1[i].energy)
        assert abs(i1[i].residual - O.residual(op, p.U0)) <= 1e-10 * i1[i].residual


def test_batched_workload_step_matches_oracle():
    """The 64-problem workload stepped once as a batch with Step 1 solved to
    1e-13: the three smallest problems' new blocks equal the oracle's exact
    step (Steps 1-4 with a sparse LU for Step 1) to 1e-12, and every problem's
    input energy and residual equal the oracle's."""
    from paper_2511_06788_amd import ope
    probs = W.batched_problems(64)
    order = sorted(range(len(probs)), key=lambda i: probs[i].grid.n)
    pick = order[:3]
    say("batched workload vs oracle step")
    with ope.Batch(probs) as b:
        for i in range(len(probs)):
            ope.ope_set_inner(b.context(i), 0.0, 1e-13, 20000)
        Ub = [_dev(p.U0, 0) for p in probs]
        info = b.step(Ub, 30.0, allow_maxit=False)
        got = {i: to_host(Ub[i]) for i in pick}
    for i in pick:
        p = probs[i]
        op = O.Operator(p.grid.m, p.grid.h, p.V)
        ref = O.steps_1_to_4(p.U0, O.GSolver(op, "sparse"), 30.0)["U"]
        assert np.max(np.abs(got[i] - ref)) <= 1e-12, i
        assert np.max(np.abs(got[i] - p.U0)) > 1e-5, i
        assert abs(info[i].energy - O.energy(op, p.U0)) <= 1e-12 * abs(info[i].energy), i
        assert abs(info[i].residual - O.residual(op, p.U0)) <= 1e-10 * info[i].residual, i
