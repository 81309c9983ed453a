"""GPU parity of the mixed-precision form (FP32 storage, BF16/FP32 matrix-core
products, FP64 small solve and checks) through the C ABI.

* Building blocks: the three Gram kinds and the two row-block kinds are exact
  on small-integer data (exactly representable in BF16, sums below 2^24); the
  FP32 stencil is within FP32 rounding of the oracle.
* One mixed step equals the oracle's step (delta form, FP64, exact Step 1) to
  the precision of the FP32 block and the BF16 P^T P.
* Converged mixed runs: Ritz values within 1e-6 of the FP64 reference and
  |U^T U - I| < 1e-6; after converting to FP64 and finishing, within 1e-10.
* At 64^3, N = 128: sampled FP32 stencil and the step's invariants.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W
from tests.gpu_common import empty_dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu

EPS32 = float(np.finfo(np.float32).eps)


def _ctx(p, precision=1):
    from paper_2511_06788_amd import ope
    return ope.Context(p.grid, p.V, p.N, kinetic=p.kinetic, shift=p.shift, precision=precision)


def _op(p):
    return O.Operator(p.grid.m, p.grid.h, p.V, kinetic=p.kinetic, shift=p.shift)


def _dev32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


def _empty32(*shape):
    import torch
    return torch.empty(*shape, dtype=torch.float32, device="cuda")


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("n,na,nb", [(1000, 8, 8), (4099, 17, 33), (2048, 128, 128)])
def test_gram_kinds_exact_on_integers(kind, n, na, nb):
    from paper_2511_06788_amd import ope
    rng = np.random.default_rng(n + na + kind)
    A = rng.integers(-8, 9, size=(n, na)).astype(np.float32)
    B = rng.integers(-8, 9, size=(n, nb)).astype(np.float32)
    p = W.harmonic_2d_32(m=8, N=8)
    say(f"gram_f32 kind={kind} n={n} na={na} nb={nb}")
    with _ctx(p) as ctx:
        out = empty_dev(na, nb)
        ope.ope_gram_f32(ctx.handle, kind, _dev32(A), na, na, _dev32(B), nb, nb, n, out)
        G = to_host(out)
    assert np.array_equal(G, A.astype(np.float64).T @ B.astype(np.float64))


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("n,N", [(2048, 128), (3001, 256), (1000, 136)])
def test_gram_kinds_of_a_block_with_itself_exact_on_integers(kind, n, N):
    """X^T X with one pointer for both operands in every arithmetic kind (at
    128 columns the upper block triangle, mirrored; wider, the full product)."""
    from paper_2511_06788_amd import ope
    rng = np.random.default_rng(n + N + kind)
    A = rng.integers(-8, 9, size=(n, N)).astype(np.float32)
    # a context of block width N holds the split-K partials of an N x N Gram
    p = W.Problem("sq", W.Grid(m=(N + 8, 1), h=(1.0, 1.0), lo=(0.0, 0.0)), np.zeros(N + 8), N, 1.0)
    say(f"gram_f32 X^T X kind={kind} n={n} N={N}")
    with _ctx(p) as ctx:
        Ad = _dev32(A)
        out = empty_dev(N, N)
        ope.ope_gram_f32(ctx.handle, kind, Ad, N, N, Ad, N, N, n, out)
        G = to_host(out)
    A64 = A.astype(np.float64)
    assert np.array_equal(G, A64.T @ A64)


@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("m,N", [((40, 30), 8), ((17, 9, 7), 20), ((16, 16, 16), 128)])
def test_rowmm_kinds_exact_on_integers(kind, m, N):
    from paper_2511_06788_amd import ope
    g = W.unit_box_grid(m)
    p = W.Problem("t", g, np.zeros(g.n), N, 1.0)
    rng = np.random.default_rng(N + kind)
    U = rng.integers(-4, 5, size=(g.n, N)).astype(np.float32)
    Y = rng.integers(-4, 5, size=(g.n, N)).astype(np.float32)
    Z = rng.integers(-3, 4, size=(2 * N, N)).astype(np.float32)
    say(f"rowmm_f32 kind={kind} m={m} N={N}")
    with _ctx(p) as ctx:
        Ud = _dev32(U)
        Zd = _dev32(Z)
        # in place with the identity term: U <- U + U Z1 + Y Z2
        ope.ope_rowmm_f32(ctx.handle, kind, Ud, Zd[:N], _dev32(Y), Zd[N:], Ud, 1.0, 1.0, Ud)
        Un = to_host(Ud)
    U64, Y64, Z64 = U.astype(np.float64), Y.astype(np.float64), Z.astype(np.float64)
    assert np.array_equal(Un, U64 + U64 @ Z64[:N] + Y64 @ Z64[N:])


@pytest.mark.parametrize("mk", [lambda: W.harmonic_2d_32(), lambda: W.wells_3d(m=13, N=20, seed=3),
                                lambda: W.wells_3d(m=20, N=128, seed=1)])
def test_apply_h_fp32_within_rounding(mk):
    from paper_2511_06788_amd import ope
    p = mk()
    op = _op(p)
    X = np.random.default_rng(2).standard_normal((p.grid.n, p.N)).astype(np.float32)
    say(f"apply_h fp32 {p.name}")
    with _ctx(p) as ctx:
        Yd = _empty32(p.grid.n, p.N)
        ope.ope_apply_h(ctx.handle, _dev32(X), Yd)
        Y = to_host(Yd).astype(np.float64)
    ref = O.apply_H(op, X.astype(np.float64))
    c = sum(1.0 / h ** 2 for h in op.h)
    bound = 16 * EPS32 * (np.max(np.abs(op.V)) + 4 * c) * np.max(np.abs(X))
    assert np.max(np.abs(Y - ref)) <= bound


@pytest.mark.parametrize("autotune", [False, True])
def test_one_mixed_step_matches_oracle_delta_step(autotune):
    """One mixed step vs the oracle's delta-form step (also after ope_autotune
    has picked the context's sweep shape by timing FP32 CG runs)."""
    from paper_2511_06788_amd import ope
    p = W.harmonic_2d_32()
    op = _op(p)
    U32 = p.U0.astype(np.float32)
    U = U32.astype(np.float64)
    tau = 20.0
    ref = O.step_delta(U, O.GSolver(op, "dense")(U), tau)["U"]
    say(f"one mixed step autotune={autotune}")
    with _ctx(p) as ctx:
        if autotune:
            ope.ope_autotune(ctx.handle)
        ope.ope_set_inner(ctx.handle, 0.0, 1e-7, 20000)
        Ud = _dev32(U32)
        info = ope.ope_step(ctx.handle, Ud, tau)
        Un = to_host(Ud).astype(np.float64)
    step = np.max(np.abs(ref - U))
    assert step > 1e-3
    assert np.max(np.abs(Un - ref)) <= 1e-2 * step
    # energy: FP64 accumulation of U^T (H U) with H U from the FP32 stencil
    assert abs(info.energy - O.energy(op, U)) <= 1e-6 * abs(info.energy)
    # drift: <U,U> accumulated in FP64 from the FP32 iterate
    assert abs(info.drift - O.ortho_error(U)) <= 1e-12


def test_mixed_then_fp64_finish_converges_3d():
    """16^3 wells, N = 17: the mixed phase reaches the FP32 floor with Ritz
    values within 1e-6 and drift below 1e-6; the FP64 finish reaches 1e-10."""
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=16, N=17, seed=0)
    op = _op(p)
    H = O.assemble_H(op)
    w = np.sort(spla.eigsh(H.tocsc(), k=20, sigma=0, return_eigenvectors=False))[:p.N]
    lmax = spla.eigsh(H, k=1, which="LA", return_eigenvectors=False)[0]
    tau = 1.8 / (1 / w[0] - 1 / lmax)
    say("mixed solve 16^3 N=17")
    with _ctx(p, 1) as cm, _ctx(p, 0) as cd:
        U32 = _dev32(p.U0)
        si = ope.ope_solve(cm.handle, U32, tau, 1e-7, 4000)
        res_m, ritz_m, drift_m = ope.ope_residual(cm.handle, U32, p.N)
        U64 = empty_dev(p.grid.n, p.N)
        ope.ope_convert(cm.handle, U32, U64, p.grid.n * p.N, True)
        sf = ope.ope_solve(cd.handle, U64, tau, 1e-11, 4000)
        res_f, ritz_f, drift_f = ope.ope_residual(cd.handle, U64, p.N)
    assert si.steps > 50
    assert res_m <= 1e-5
    assert np.max(np.abs(ritz_m - w) / np.abs(w)) <= 1e-6
    assert drift_m <= 1e-6
    assert sf.converged == 1
    assert np.max(np.abs(ritz_f - w) / np.abs(w)) <= 1e-10
    assert drift_f <= 1e-10


def test_mixed_nan_leaves_U_unchanged():
    from paper_2511_06788_amd import ope
    p = W.harmonic_2d_32()
    U = p.U0.astype(np.float32)
    U[3, 1] = np.nan
    say("mixed nan")
    with _ctx(p) as ctx:
        Ud = _dev32(U)
        st = ope.ope_step_raw(ctx.handle, Ud, 0.1)
        U2 = to_host(Ud)
    assert st == ope.OPE_ENONFINITE
    assert np.array_equal(U2[~np.isnan(U)], U[~np.isnan(U)])


def test_mixed_full_size_invariants():
    """64^3, N = 128: sampled FP32 stencil rows and two mixed steps (energy
    decreases, drift stays at FP32 level)."""
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=64, N=128, seed=0)
    op = _op(p)
    U32 = p.U0.astype(np.float32)
    rows = np.random.default_rng(0).choice(p.grid.n, 4096, replace=False)
    say("mixed full size")
    with _ctx(p) as ctx:
        Ud = _dev32(U32)
        HUd = _empty32(p.grid.n, p.N)
        ope.ope_apply_h(ctx.handle, Ud, HUd)
        HU = to_host(HUd)[rows].astype(np.float64)
        i1 = ope.ope_step(ctx.handle, Ud, 45.0)
        i2 = ope.ope_step(ctx.handle, Ud, 45.0)
        E2 = ope.ope_energy(ctx.handle, Ud)
        res, _, drift = ope.ope_residual(ctx.handle, Ud, p.N, want_ritz=False)
    ref = O.apply_H(op, U32.astype(np.float64))[rows]
    c = sum(1.0 / h ** 2 for h in op.h)
    assert np.max(np.abs(HU - ref)) <= 16 * EPS32 * (np.max(np.abs(op.V)) + 4 * c) * np.max(np.abs(U32))
    assert i2.energy < i1.energy and E2 < i2.energy
    # the device drift check after every update keeps the block below the 1e-6 target
    assert drift <= 1e-6 and i1.drift <= 1e-6 and i2.drift <= 1e-6
