"""GPU parity of the multigrid-preconditioned Step 1 (ope_set_multigrid)
against the oracle's V-cycle and preconditioned CG (oracle/multigrid.py).

* One V-cycle (ope_mg_vcycle) equals the oracle's ``Hierarchy.vcycle`` to
  1e-12 relative on 3D and 2D grids with odd and even sizes, a kinetic
  factor and a shift, a grid two nodes thick (levels one node thick), even
  and odd N, rows split into slices, and at 64^3 with N = 128 (columns
  compared against the oracle on eight of them); the hierarchy has the
  oracle's number of levels and coarsest size.
* The preconditioned CG capped at k = 1, 2, 3, 5, 6 iterations (eager and
  graph-replayed chunks; N = 40 and 17 at k = 3) equals the oracle's
  ``pcg_source`` iterate.
* Stand-alone Step 1 converges to the sparse direct solution in a few
  iterations; steps with a tight inner solve equal the oracle's exact Steps
  1-4; at 64^3 with N = 128 a step needs far fewer inner iterations than the
  plain CG, keeps the block orthonormal and lowers the energy.
* Batched steps of problems with the preconditioner equal their single steps.
* The preconditioner's default inner factor (0.25; 0.1 again when it is
  switched off, and the caller's factor once ope_set_inner was called).
* Mixed precision: the FP32 V-cycle equals the oracle's to FP32 rounding, and
  a mixed solve with the preconditioner followed by an FP64 one reaches the
  dense eigenvalues.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_common import empty_dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _op(p):
    return O.Operator(p.grid.m, p.grid.h, p.V, kinetic=p.kinetic, shift=p.shift)


def _ctx(p, N=None):
    from paper_2511_06788_amd import ope
    c = ope.Context(p.grid, p.V, p.N if N is None else N, kinetic=p.kinetic, shift=p.shift)
    ope.ope_set_multigrid(c.handle, True)
    return c


def _case(name):
    if name == "wells20_N8":
        return W.wells_3d(m=20, N=8, seed=3)
    if name == "aniso13x11x9_N7":
        g = W.Grid(m=(13, 11, 9), h=(0.07, 0.08, 0.1), lo=(0.0, 0.0, 0.0))
        V = W.harmonic_potential(g, 40.0, (0.5, 0.4, 0.45))
        return W.Problem("aniso", g, V, 7, 1.0, U0=W.initial_block(g.n, 7, 1), kinetic=0.5, shift=2.0)
    if name == "2d_33x27_N6":
        g = W.Grid(m=(33, 27), h=(1.0 / 34, 1.0 / 28), lo=(0.0, 0.0))
        V = W.harmonic_potential(g, 80.0, (0.5, 0.5))
        return W.Problem("2d", g, V, 6, 1.0, U0=W.initial_block(g.n, 6, 2))
    if name == "thin40x2x30_N6":
        # y has two nodes, one on the coarse levels: tiles one column high,
        # whose ring is longer than two columns per thread
        g = W.Grid(m=(40, 2, 30), h=(0.05, 0.05, 0.05), lo=(0.0, 0.0, 0.0))
        V = W.harmonic_potential(g, 30.0, (0.5, 0.5, 0.5))
        return W.Problem("thin", g, V, 6, 1.0, U0=W.initial_block(g.n, 6, 4))
    if name == "wells16_N40":
        return W.wells_3d(m=16, N=40, seed=6)         # rows in two slices of 10 vector pairs
    if name == "wells12_N17":
        return W.wells_3d(m=12, N=17, seed=8)         # odd N: one element per vector group
    raise KeyError(name)


VCYCLE_CASES = ["wells20_N8", "aniso13x11x9_N7", "2d_33x27_N6", "thin40x2x30_N6", "wells16_N40", "wells12_N17"]


@pytest.mark.parametrize("name", VCYCLE_CASES)
def test_vcycle_matches_oracle(name):
    from paper_2511_06788_amd import ope
    p = _case(name)
    op = _op(p)
    hier = O.Hierarchy(op)
    R = np.random.default_rng(7).standard_normal((p.grid.n, p.N))
    ref = hier.vcycle(R)
    say(f"mg vcycle {name}")
    with _ctx(p) as c:
        lv, nc = ope.ope_mg_info(c.handle)
        Z = empty_dev(p.grid.n, p.N)
        ope.ope_mg_vcycle(c.handle, to_dev(R), Z)
        got = to_host(Z)
    assert lv == len(hier.levels) and nc == hier.levels[-1].n
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_vcycle_full_size_matches_oracle_columns():
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=64, N=128, seed=0)
    op = _op(p)
    R = np.random.default_rng(5).standard_normal((p.grid.n, 128))
    cols = [0, 1, 37, 64, 90, 126, 127, 5]
    ref = O.Hierarchy(op).vcycle(R[:, cols])
    say("mg vcycle 64^3 N=128")
    with _ctx(p) as c:
        Z = empty_dev(p.grid.n, 128)
        ope.ope_mg_vcycle(c.handle, to_dev(R), Z)
        got = to_host(Z)[:, cols]
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("k", [1, 2, 3, 5, 6])
def test_capped_pcg_equals_oracle_iterates(k, graphs):
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=13, N=6, seed=11)
    op = _op(p)
    U = W.initial_block(p.grid.n, p.N, 5)
    say(f"capped PCG k={k} graphs={graphs}")
    with _ctx(p) as c:
        ope.ope_set_graphs(c.handle, graphs)
        Yd = empty_dev(p.grid.n, p.N)
        its = ope.ope_source_solve(c.handle, to_dev(U), Yd, None, 1e-15, k, allow_maxit=True)
        Y = to_host(Yd)
    st = {}
    Y_ref = O.pcg_source(op, U, None, tol=1e-15, max_iter=k, stats=st)
    assert its == k and st["iterations"] == k
    assert np.max(np.abs(Y - Y_ref)) <= 1e-12 * np.max(np.abs(Y_ref))


@pytest.mark.parametrize("N", [40, 17])
def test_capped_pcg_equals_oracle_iterates_wide_rows(N):
    """The PCG dot products of the finest post-smoothing with rows split into
    slices (N = 40) and with odd N."""
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=13, N=N, seed=12)
    op = _op(p)
    U = W.initial_block(p.grid.n, p.N, 6)
    say(f"capped PCG N={N}")
    with _ctx(p) as c:
        Yd = empty_dev(p.grid.n, p.N)
        its = ope.ope_source_solve(c.handle, to_dev(U), Yd, None, 1e-15, 3, allow_maxit=True)
        Y = to_host(Yd)
    Y_ref = O.pcg_source(op, U, None, tol=1e-15, max_iter=3)
    assert its == 3
    assert np.max(np.abs(Y - Y_ref)) <= 1e-12 * np.max(np.abs(Y_ref))


def test_capped_pcg_with_a_stopped_slice():
    """Right-hand-side columns that are zero stop before the first iteration;
    with N = 40 the first 20 columns are a whole slice of the row, whose
    V-cycle work-groups return at once (writing zero partial sums) while the
    other slice iterates."""
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=13, N=40, seed=13)
    op = _op(p)
    U = W.initial_block(p.grid.n, p.N, 7)
    U[:, :20] = 0.0
    say("capped PCG N=40 with a stopped slice")
    with _ctx(p) as c:
        Yd = empty_dev(p.grid.n, p.N)
        its = ope.ope_source_solve(c.handle, to_dev(U), Yd, None, 1e-15, 3, allow_maxit=True)
        Y = to_host(Yd)
    Y_ref = O.pcg_source(op, U, None, tol=1e-15, max_iter=3)
    assert its == 3
    assert np.all(Y[:, :20] == 0.0)
    assert np.max(np.abs(Y - Y_ref)) <= 1e-12 * np.max(np.abs(Y_ref))


def test_source_solve_reaches_direct_solution():
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=24, N=5, seed=1)
    op = _op(p)
    ref = O.GSolver(op, "sparse")(p.U0)
    say("PCG source solve")
    with _ctx(p) as c:
        Yd = empty_dev(p.grid.n, p.N)
        its = ope.ope_source_solve(c.handle, to_dev(p.U0), Yd, None, 1e-11, 100)
        Y = to_host(Yd)
    assert its <= 20
    assert np.max(np.abs(Y - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_steps_match_oracle_exact_steps():
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=14, N=12, seed=2)
    op = _op(p)
    G = O.GSolver(op, "sparse")
    tau = 30.0
    say("PCG steps vs oracle")
    with _ctx(p) as c:
        ope.ope_set_inner(c.handle, 0.0, 1e-13, 500)
        U = to_dev(p.U0)
        ref = p.U0
        for _ in range(4):
            info = ope.ope_step(c.handle, U, tau, allow_maxit=False)
            assert abs(info.energy - O.energy(op, ref)) <= 1e-12 * abs(info.energy)
            assert info.inner_iterations <= 40
            ref = O.steps_1_to_4(ref, G, tau)["U"]
        got = to_host(U)
    assert np.max(np.abs(got - ref)) <= 1e-10


def test_full_size_steps_need_few_iterations():
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=64, N=128, seed=0)
    tau = 45.0
    say("PCG steps 64^3 N=128")
    with ope.Context(p.grid, p.V, p.N) as plain, _ctx(p) as c:
        ope.ope_set_inner(c.handle, 0.1, 1e-12, 2000)        # the plain CG's default factor
        Ua, Ub = to_dev(p.U0), to_dev(p.U0)
        ia = [ope.ope_step(plain.handle, Ua, tau) for _ in range(3)]
        ib = [ope.ope_step(c.handle, Ub, tau) for _ in range(3)]
        res_a, _, drift_a = ope.ope_residual(plain.handle, Ua, p.N, want_ritz=False)
        res_b, _, drift_b = ope.ope_residual(c.handle, Ub, p.N, want_ritz=False)
    for a, b in zip(ia, ib):
        # the same input block on the first step
        assert b.inner_iterations * 3 <= a.inner_iterations
    assert ia[0].energy == ib[0].energy
    assert ib[2].energy < ib[1].energy < ib[0].energy
    assert drift_b <= 1e-12
    # both steps meet the same inner tolerance: the iterates stay close
    assert abs(res_b - res_a) <= 0.2 * res_a


def test_inner_factor_defaults():
    """Enabling the preconditioner sets the inner factor to 0.25 and disabling
    it back to 0.1, unless ope_set_inner chose one: steps equal those with the
    factor set explicitly, bit for bit."""
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=16, N=8, seed=5)
    tau = 45.0

    def run(setup):
        with ope.Context(p.grid, p.V, p.N) as c:
            setup(c.handle)
            U = to_dev(p.U0)
            info = [ope.ope_step(c.handle, U, tau) for _ in range(3)]
            return to_host(U), [(i.energy, i.inner_iterations) for i in info]

    say("inner factor defaults")
    mg = lambda h, on=True: ope.ope_set_multigrid(h, on)
    inner = lambda h, eta: ope.ope_set_inner(h, eta, 1e-12, 2000)
    a = run(lambda h: mg(h))
    b = run(lambda h: (inner(h, 0.25), mg(h)))
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
    c = run(lambda h: (inner(h, 0.1), mg(h)))                   # the caller's factor stays
    d = run(lambda h: (mg(h), inner(h, 0.1)))
    assert np.array_equal(c[0], d[0]) and c[1] == d[1]
    assert sum(x[1] for x in c[1]) > sum(x[1] for x in a[1])      # a tighter tolerance costs iterations
    e = run(lambda h: (mg(h), mg(h, False)))
    f = run(lambda h: None)
    assert np.array_equal(e[0], f[0]) and e[1] == f[1]


def test_batched_steps_with_multigrid_equal_single_steps():
    from paper_2511_06788_amd import ope
    probs = [W.wells_3d(m=13, N=5, seed=1), W.wells_3d(m=20, N=17, seed=2), W.harmonic_2d_32()]
    tau = 0.5
    say("batched PCG steps vs single")
    with ope.Batch(probs) as b:
        b.set_shared(True)
        for i in range(len(probs)):
            ope.ope_set_multigrid(b.context(i), True)
        Ub = [to_dev(p.U0) for p in probs]
        ib = [b.step(Ub, tau) for _ in range(2)]
        Ub = [to_host(U) for U in Ub]
    for i, p in enumerate(probs):
        with _ctx(p) as c:
            U = to_dev(p.U0)
            ia = [ope.ope_step(c.handle, U, tau) for _ in range(2)]
            U = to_host(U)
        assert np.array_equal(U, Ub[i]), i
        for k in range(2):
            assert (ia[k].energy, ia[k].inner_iterations) == (ib[k][i].energy, ib[k][i].inner_iterations)


def test_multigrid_refusals():
    from paper_2511_06788_amd import ope
    q = W.wells_3d(m=8, N=257, seed=0)
    with pytest.raises(ope.OpeError) as ei:                  # 257 single-element chunks per row
        ope.Context(q.grid, q.V, q.N)
    assert ei.value.status == ope.OPE_EUNSUPPORTED
    p = W.wells_3d(m=12, N=4, seed=0)
    with ope.Context(p.grid, p.V, p.N) as c:
        R = to_dev(p.U0)
        Z = empty_dev(p.grid.n, p.N)
        with pytest.raises(ope.OpeError):
            ope.ope_mg_vcycle(c.handle, R, Z)            # preconditioner off
        ope.ope_set_multigrid(c.handle, True)
        hier = O.Hierarchy(_op(p))
        assert ope.ope_mg_info(c.handle) == (len(hier.levels), hier.levels[-1].n)
        ope.ope_set_multigrid(c.handle, False)
        assert ope.ope_mg_info(c.handle) == (0, 0)


@pytest.mark.parametrize("name", VCYCLE_CASES)
def test_fp32_vcycle_matches_oracle(name):
    import torch
    from paper_2511_06788_amd import ope
    p = _case(name)
    hier = O.Hierarchy(_op(p))
    R = np.random.default_rng(8).standard_normal((p.grid.n, p.N)).astype(np.float32)
    ref = hier.vcycle(R.astype(np.float64))
    say(f"mg vcycle fp32 {name}")
    with ope.Context(p.grid, p.V, p.N, kinetic=p.kinetic, shift=p.shift, precision=ope.OPE_MIXED) as c:
        ope.ope_set_multigrid(c.handle, True)
        Z = torch.empty((p.grid.n, p.N), dtype=torch.float32, device="cuda")
        ope.ope_mg_vcycle(c.handle, torch.from_numpy(R).to("cuda"), Z)
        got = Z.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 2e-6 * np.max(np.abs(ref))


def test_mixed_solve_with_multigrid_reaches_dense_eigenvalues():
    import torch
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=16, N=8, seed=1)
    op = _op(p)
    w = np.linalg.eigvalsh(O.assemble_H(op).toarray())
    tau = 0.8 * 2.0 / (1.0 / w[0] - 1.0 / w[-1])
    say("mixed + multigrid solve, then FP64 + multigrid")
    with ope.Context(p.grid, p.V, p.N, precision=ope.OPE_MIXED) as cm, _ctx(p) as cd:
        ope.ope_set_multigrid(cm.handle, True)
        U32 = torch.from_numpy(p.U0.astype(np.float32)).to("cuda")
        # the FP32 preconditioned CG floors the mixed phase near 1e-3 (the plain
        # FP32 CG near 1e-4): switch to FP64 there
        sm = ope.ope_solve(cm.handle, U32, tau, 1e-3, 5000)
        assert sm.converged == 1 and sm.inner_iterations < 8 * sm.steps
        U = torch.empty((p.grid.n, p.N), dtype=torch.float64, device="cuda")
        ope.ope_convert(cm.handle, U32, U, p.grid.n * p.N, True)
        sf = ope.ope_solve(cd.handle, U, tau, 1e-10, 20000)
        res, ritz, drift = ope.ope_residual(cd.handle, U, p.N)
    assert sf.converged == 1
    assert np.max(np.abs(ritz - w[:p.N]) / w[:p.N]) <= 1e-10
    assert drift <= 1e-12
