"""GPU tests of the C ABI's set-up and boundary entry points.

* Coercivity check (Section 2.2): an operator with a negative eigenvalue is
  refused with OPE_ENOTSPD; SPD operators whose closed-form bound cannot prove
  it (attractive wells) are accepted, and the Lanczos estimates bracket the
  dense spectrum (lambda_min from above within 1e-8, lambda_max from below).
* Caller-owned workspace (a torch tensor) gives bit-identical steps.
* A block with leading dimension ldu > N gives bit-identical steps, energies
  and residuals to the packed block, and the padding columns are untouched.
* The device-scalar energy and residual equal the host ones bit for bit.
* The generalized problem H u = lambda M u (Section 5's mass inner product):
  ``ope_orthonormalize`` equals the oracle's Cholesky re-orthonormalisation,
  steps with a tight inner solve equal the oracle's Steps 1-4 in the M
  product, and a converged solve reaches the generalized eigenvalues of dense
  ``eigh(K, M)`` to 1e-10 with ``U^T M U = I`` to 1e-12.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W
from tests.gpu_common import say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _ctx(p, N=None):
    from paper_2511_06788_amd import ope
    return ope.Context(p.grid, p.V, p.N if N is None else N, kinetic=p.kinetic, shift=p.shift)


def test_indefinite_operator_is_refused():
    from paper_2511_06788_amd import ope
    p = W.harmonic_2d_32(m=20, N=4)
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    w = np.linalg.eigvalsh(O.assemble_H(op).toarray())
    say("ENOTSPD")
    for shift in (-w[0] - 5.0, -0.5 * (w[0] + w[1])):
        with pytest.raises(ope.OpeError) as ei:
            ope.Context(p.grid, p.V, p.N, shift=shift)
        assert ei.value.status == ope.OPE_ENOTSPD
    # the coarse softened-Coulomb operator with shift 1 has lambda_1 = -4.74 (dense eigvalsh)
    hp = W.hydrogen_softened(m=9, N=8, half=4.0)
    hop = O.Operator(hp.grid.m, hp.grid.h, hp.V, kinetic=hp.kinetic, shift=hp.shift)
    assert np.linalg.eigvalsh(O.assemble_H(hop).toarray())[0] < 0
    with pytest.raises(ope.OpeError) as ei:
        ope.Context(hp.grid, hp.V, hp.N, kinetic=hp.kinetic, shift=hp.shift)
    assert ei.value.status == ope.OPE_ENOTSPD
    # just above the bottom of the spectrum: SPD, accepted
    with ope.Context(p.grid, p.V, p.N, shift=-w[0] + 0.5) as c:
        lo, hi = ope.ope_spectrum_bounds(c.handle)
        assert abs(lo - 0.5) <= 1e-8 * w[-1]


@pytest.mark.parametrize("m,seed,scale", [(12, 4, 1.0), (12, 5, 3.0), (15, 1, 2.0)])
def test_wells_accepted_with_lanczos_bounds(m, seed, scale):
    """Attractive wells deep enough that lambda_min(-Lap_h) + min V <= 0, yet
    lambda_1 > 0 (dense eigvalsh): accepted, with Lanczos estimates inside the
    spectrum and lambda_min accurate."""
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=m, N=4, seed=seed)
    p.V = scale * p.V
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    lap_min = sum(O.sine_eigenvalues_1d(m, h)[0] for h in p.grid.h)
    assert lap_min + p.V.min() <= 0.0
    w = np.linalg.eigvalsh(O.assemble_H(op).toarray())
    assert w[0] > 0
    say(f"lanczos bounds m={m} seed={seed} scale={scale}")
    with _ctx(p) as c:
        lo, hi = ope.ope_spectrum_bounds(c.handle)
    assert w[0] * (1 - 1e-12) <= lo <= w[0] * (1 + 1e-8)
    assert 0.99 * w[-1] <= hi <= w[-1] * (1 + 1e-12)


def test_caller_workspace_is_bitwise_identical():
    import torch
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=14, N=24, seed=3)
    Ua, Ub = to_dev(p.U0), to_dev(p.U0)
    say("caller workspace")
    with _ctx(p) as ca, _ctx(p) as cb:
        nbytes = ope.ope_workspace_size(cb.handle)
        assert nbytes >= 5 * p.grid.n * p.N * 8
        ws = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device="cuda")
        off = (-ws.data_ptr()) % 256
        ope.ope_set_workspace(cb.handle, ws.data_ptr() + off, nbytes)
        for _ in range(3):
            ia = ope.ope_step(ca.handle, Ua, 30.0)
            ib = ope.ope_step(cb.handle, Ub, 30.0)
            assert ia.energy == ib.energy and ia.inner_iterations == ib.inner_iterations
        assert np.array_equal(to_host(Ua), to_host(Ub))
        # hand the workspace back; the library allocates on the next step
        ope.ope_set_workspace(cb.handle, None, 0)
        ope.ope_step(ca.handle, Ua, 30.0)
        ope.ope_step(cb.handle, Ub, 30.0)
        assert np.array_equal(to_host(Ua), to_host(Ub))
        with pytest.raises(ope.OpeError):
            ope.ope_set_workspace(cb.handle, ws.data_ptr() + off, nbytes - 8)


def test_leading_dimension_variants():
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=11, N=9, seed=4)
    n, N = p.grid.n, p.N
    ld = N + 3
    pad = np.full((n, ld), 7.25)
    pad[:, :N] = p.U0
    Up, Ud = to_dev(pad), to_dev(p.U0)
    say("leading dimension")
    with _ctx(p) as c:
        e1 = ope.ope_energy_ld(c.handle, Up, ld)
        e2 = ope.ope_energy(c.handle, Ud)
        assert e1 == e2
        r1 = ope.ope_residual_ld(c.handle, Up, ld, N)
        r2 = ope.ope_residual(c.handle, Ud, N)
        assert r1[0] == r2[0] and r1[2] == r2[2] and np.array_equal(r1[1], r2[1])
        for _ in range(2):
            i1 = ope.ope_step_ld(c.handle, Up, ld, 30.0)
            i2 = ope.ope_step(c.handle, Ud, 30.0)
            assert i1.energy == i2.energy
        got = to_host(Up)
    assert np.array_equal(got[:, :N], to_host(Ud))
    assert np.all(got[:, N:] == 7.25)


def test_device_scalars_equal_host_values():
    import torch
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=13, N=16, seed=5)
    U = to_dev(p.U0)
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    say("device scalars")
    with _ctx(p) as c:
        ope.ope_step(c.handle, U, 30.0)
        ope.ope_energy_d(c.handle, U, out[0:1])
        ope.ope_residual_d(c.handle, U, out[1:2], out[2:3])
        dev = to_host(out)
        e = ope.ope_energy(c.handle, U)
        res, _, drift = ope.ope_residual(c.handle, U, p.N, want_ritz=False)
    assert dev[0] == e and dev[1] == res and dev[2] == drift


def _mass_case(m=(24, 20), N=6, seed=0):
    g = W.unit_box_grid(m)
    V = W.harmonic_potential(g, 60.0, (0.45, 0.55))
    rng = np.random.default_rng(seed)
    d = 1.0 + 0.3 * rng.uniform(size=g.n)
    mu = (0.12, -0.09)
    p = W.Problem("mass", g, V, N, 1.0, U0=W.initial_block(g.n, N, seed))
    op = O.Operator(g.m, g.h, V)
    return p, op, O.Mass(d, mu)


def test_mass_orthonormalize_and_steps_match_oracle():
    from paper_2511_06788_amd import ope
    p, op, mass = _mass_case()
    G = O.GSolver(op, "dense")
    U_ref = O.orthonormalize_M(op, mass, p.U0)
    say("mass orthonormalize and steps")
    with _ctx(p) as c:
        ope.ope_set_mass(c.handle, mass.d, mass.mu)
        ope.ope_set_inner(c.handle, 0.0, 1e-13, 20000)
        U = to_dev(p.U0)
        ope.ope_orthonormalize(c.handle, U)
        Ug = to_host(U)
        assert np.max(np.abs(Ug - U_ref)) <= 1e-12
        X = to_dev(np.random.default_rng(3).standard_normal(p.U0.shape))
        Y = to_dev(np.zeros(p.U0.shape))
        ope.ope_apply_mass(c.handle, X, Y)
        assert np.max(np.abs(to_host(Y) - O.apply_M(op, mass, to_host(X)))) <= 1e-13 * 4
        ref = U_ref
        for k in range(5):
            info = ope.ope_step(c.handle, U, 3.0, allow_maxit=False)
            assert abs(info.energy - O.energy(op, ref)) <= 1e-12 * abs(info.energy)
            assert info.drift <= 1e-12
            assert abs(info.residual - O.residual_M(op, mass, ref)) <= 1e-10 * info.residual
            ref = O.steps_1_to_4_M(op, mass, ref, G, 3.0)["U"]
        assert np.max(np.abs(to_host(U) - ref)) <= 1e-10


def test_mass_solve_converges_to_generalized_eigenvalues():
    from paper_2511_06788_amd import ope
    p, op, mass = _mass_case()
    N = p.N
    K = O.assemble_H(op).toarray()
    Md = O.assemble_M(op, mass).toarray()
    w = sla.eigh(K, Md, eigvals_only=True)
    tcrit = 2.0 / (1.0 / w[0] - 1.0 / w[-1])
    say("mass solve")
    with _ctx(p) as c:
        ope.ope_set_mass(c.handle, mass.d, mass.mu)
        U = to_dev(p.U0)
        ope.ope_orthonormalize(c.handle, U)
        si = ope.ope_solve(c.handle, U, 0.8 * tcrit, 1e-11, 20000)
        res, ritz, drift = ope.ope_residual(c.handle, U, N)
    assert si.converged == 1
    assert np.max(np.abs(ritz - w[:N]) / w[:N]) <= 1e-10
    assert drift <= 1e-12
    assert O.ortho_error_M(op, mass, to_host(U)) <= 1e-12


def test_mass_not_spd_is_refused():
    from paper_2511_06788_amd import ope
    p, op, mass = _mass_case()
    with _ctx(p) as c:
        with pytest.raises(ope.OpeError) as ei:
            ope.ope_set_mass(c.handle, np.full(p.grid.n, 0.3), (0.12, -0.09))
        assert ei.value.status == ope.OPE_ENOTSPD
