"""GPU parity of each hot-path building block against the FP64 oracle / plain
definitions, through the C ABI (libope.so via its ctypes binding).

Shapes span several tiles with ragged tails (n and N not multiples of the
tile sizes, odd N, N = 1); integer-valued inputs make the Gram and the row-block
products exact in any summation order, so those are compared bit for bit.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_common import EPS, empty_dev, say, stencil_bound, to_dev, to_host

pytestmark = pytest.mark.gpu


def _ctx(problem, N=None):
    from paper_2511_06788_amd import ope
    return ope.Context(problem.grid, problem.V, problem.N if N is None else N, kinetic=problem.kinetic,
                       shift=problem.shift)


def _op(problem):
    return O.Operator(problem.grid.m, problem.grid.h, problem.V, kinetic=problem.kinetic, shift=problem.shift)


CASES = [
    ("2d 32x32 N=8", lambda: W.harmonic_2d_32(), 8),
    ("2d 7x5 N=1", lambda: W.harmonic_2d_32(m=7, N=1), 1),
    ("3d 13x13x13 N=17", lambda: W.wells_3d(m=13, N=17, seed=3), 17),
    ("3d 20^3 N=128", lambda: W.wells_3d(m=20, N=128, seed=1), 128),
    # shift 7: the coarse softened-Coulomb operator has lambda_1 = -5.74 + shift
    ("3d 9^3 N=63 kinetic 0.5 shift", lambda: W.hydrogen_softened(m=9, N=63, half=4.0, shift=7.0), 63),
]


@pytest.mark.parametrize("name,mk,N", CASES, ids=[c[0] for c in CASES])
def test_apply_h_matches_oracle(name, mk, N):
    from paper_2511_06788_amd import ope
    p = mk()
    op = _op(p)
    rng = np.random.default_rng(11)
    X = rng.standard_normal((p.grid.n, N))
    say(f"apply_h {name}")
    with _ctx(p, N) as ctx:
        Xd = to_dev(X)
        Yd = empty_dev(p.grid.n, N)
        ope.ope_apply_h(ctx.handle, Xd, Yd)
        Y = to_host(Yd)
    ref = O.apply_H(op, X)
    assert np.max(np.abs(Y - ref)) <= stencil_bound(op, X)


@pytest.mark.parametrize("n,na,nb", [(1000, 8, 8), (4099, 17, 33), (777, 1, 5), (5003, 128, 128), (2048, 64, 96),
                                     (4099, 17, 17), (3001, 32, 32), (130, 31, 2)])
def test_gram_exact_on_integers(n, na, nb):
    from paper_2511_06788_amd import ope
    rng = np.random.default_rng(n + na)
    A = rng.integers(-8, 9, size=(n, na)).astype(np.float64)
    B = rng.integers(-8, 9, size=(n, nb)).astype(np.float64)
    p = W.harmonic_2d_32(m=8, N=8)
    say(f"gram int n={n} na={na} nb={nb}")
    with _ctx(p) as ctx:
        out = empty_dev(na, nb)
        ope.ope_gram(ctx.handle, to_dev(A), na, na, to_dev(B), nb, nb, n, out)
        G = to_host(out)
    assert np.array_equal(G, A.T @ B)


@pytest.mark.parametrize("n,N", [(5003, 128), (3001, 200), (2048, 256), (4099, 300), (1000, 130)])
def test_gram_of_a_block_with_itself_exact_on_integers(n, N):
    """X^T X with one pointer for both operands: up to 128 columns the kernel
    computes the MFMA blocks on and above the block diagonal and mirrors
    them; wider blocks take the full product (ragged last tiles at 200, 300,
    130)."""
    from paper_2511_06788_amd import ope
    rng = np.random.default_rng(n + N)
    A = rng.integers(-8, 9, size=(n, N)).astype(np.float64)
    # a context of block width N holds the split-K partials of an N x N Gram
    p = W.Problem("sq", W.Grid(m=(N + 8, 1), h=(1.0, 1.0), lo=(0.0, 0.0)), np.zeros(N + 8), N, 1.0)
    say(f"gram X^T X int n={n} N={N}")
    with ope.Context(p.grid, p.V, N) as ctx:
        Ad = to_dev(A)
        out = empty_dev(N, N)
        ope.ope_gram(ctx.handle, Ad, N, N, Ad, N, N, n, out)
        G = to_host(out)
    assert np.array_equal(G, A.T @ A)


@pytest.mark.parametrize("n,lda,na,ldb,nb", [(3001, 40, 33, 24, 20), (3001, 40, 17, 24, 20)])
def test_gram_strided_and_random(n, lda, na, ldb, nb):
    """Strided operands; the second shape takes the narrow (at most 32 columns) kernel."""
    from paper_2511_06788_amd import ope
    rng = np.random.default_rng(5)
    A = rng.standard_normal((n, lda))
    B = rng.standard_normal((n, ldb))
    p = W.harmonic_2d_32(m=8, N=8)
    say("gram strided")
    with _ctx(p) as ctx:
        out = empty_dev(na, nb)
        ope.ope_gram(ctx.handle, to_dev(A), lda, na, to_dev(B), ldb, nb, n, out)
        G = to_host(out)
    ref = A[:, :na].T @ B[:, :nb]
    bound = 2 * n * EPS * (np.abs(A[:, :na]).T @ np.abs(B[:, :nb]))
    assert np.all(np.abs(G - ref) <= bound)


@pytest.mark.parametrize("m,N", [((40, 30), 8), ((17, 9, 7), 17), ((16, 16, 16), 128), ((5, 3), 1),
                                 ((13, 11, 9), 32)])
def test_update_exact_on_integers(m, N):
    """Step 4, U <- U Z1 + Y Z2 in place, with integer data (exact)."""
    from paper_2511_06788_amd import ope
    g = W.unit_box_grid(m)
    p = W.Problem("t", g, np.zeros(g.n), N, 1.0)
    rng = np.random.default_rng(N)
    U = rng.integers(-4, 5, size=(g.n, N)).astype(np.float64)
    Y = rng.integers(-4, 5, size=(g.n, N)).astype(np.float64)
    Z = rng.integers(-3, 4, size=(2 * N, N)).astype(np.float64)
    say(f"update m={m} N={N}")
    with _ctx(p) as ctx:
        Ud = to_dev(U)
        ope.ope_update(ctx.handle, Ud, to_dev(Y), to_dev(Z))
        Un = to_host(Ud)
    assert np.array_equal(Un, U @ Z[:N] + Y @ Z[N:])


@pytest.mark.parametrize("tau", [0.1, 40.0, 1e4])
@pytest.mark.parametrize("exact", [True, False])
def test_small_solve_matches_oracle(tau, exact):
    """Steps 2-3 on the device vs the oracle's elimination (general form when
    <Y,U> is not symmetric)."""
    from paper_2511_06788_amd import ope
    p = W.harmonic_2d_32()
    op = _op(p)
    U = p.U0
    Y = O.GSolver(op, "dense")(U)
    if not exact:
        Y = Y + 1e-4 * np.random.default_rng(2).standard_normal(Y.shape)
    S_a, S_b, T = Y.T @ U, U.T @ Y, Y.T @ Y
    A_ref, B_ref, _ = O.small_solve(S_a, T, tau, S_b=S_b)
    N = p.N
    say(f"small_solve tau={tau} exact={exact}")
    with _ctx(p) as ctx:
        Zd, Ad, Bd = empty_dev(2 * N, N), empty_dev(N, N), empty_dev(N, N)
        ope.ope_small_solve(ctx.handle, to_dev(S_b), to_dev(T), tau, Zd, Ad, Bd)
        Z, A, B = to_host(Zd), to_host(Ad), to_host(Bd)
    assert np.max(np.abs(B - B_ref)) <= 1e-13
    assert np.max(np.abs(A - A_ref)) <= 1e-12 * max(1.0, np.max(np.abs(A_ref)))
    assert np.max(np.abs(Z[:N] - (np.eye(N) - tau * A_ref))) <= 1e-12 * max(1.0, tau * np.max(np.abs(A_ref)))
    assert np.max(np.abs(Z[N:] - tau * B_ref)) <= 1e-13 * tau


def test_small_solve_flags_bad_pivot():
    """A non-finite input must be reported, not silently used."""
    from paper_2511_06788_amd import ope
    p = W.harmonic_2d_32()
    N = p.N
    Sb = np.zeros((N, N))
    T = np.full((N, N), np.nan)
    say("small_solve nan")
    with _ctx(p) as ctx:
        Zd = empty_dev(2 * N, N)
        with pytest.raises(ope.OpeError) as ei:
            ope.ope_small_solve(ctx.handle, to_dev(Sb), to_dev(T), 1.0, Zd)
    assert ei.value.status == ope.OPE_EPIVOT


@pytest.mark.parametrize("name,mk,N", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_source_solve_residual_and_dense(name, mk, N):
    """Step 1: the device CG reaches the requested tolerance on the true residual,
    and agrees with the oracle's exact (dense/sparse) solve."""
    from paper_2511_06788_amd import ope
    p = mk()
    op = _op(p)
    U = W.initial_block(p.grid.n, N, 4)
    tol = 1e-11
    say(f"source_solve {name}")
    with _ctx(p, N) as ctx:
        Yd = empty_dev(p.grid.n, N)
        its = ope.ope_source_solve(ctx.handle, to_dev(U), Yd, None, tol, 20000)
        Y = to_host(Yd)
    assert its > 0
    true_res = np.linalg.norm(U - O.apply_H(op, Y), axis=0)
    assert np.all(true_res <= 20 * tol * np.linalg.norm(U, axis=0))
    Yx = O.GSolver(op)(U)
    assert np.max(np.abs(Y - Yx)) <= 1e-8 * np.max(np.abs(Yx))


@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("k", [1, 2, 3, 5, 6])
def test_capped_cg_equals_textbook_iterates(k, graphs):
    """After exactly k CG iterations (no column converged) the device solution
    equals the oracle's textbook CG iterate: y is updated in pairs of
    iterations on the device, and an odd count ends with the deferred term of
    the last iteration added (with graphs on, k = 5, 6 mix a captured
    4-iteration chunk with eager iterations)."""
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=13, N=6, seed=11)
    op = _op(p)
    U = W.initial_block(p.grid.n, p.N, 5)
    say(f"capped CG k={k} graphs={graphs}")
    with _ctx(p) as ctx:
        ope.ope_set_graphs(ctx.handle, graphs)
        Yd = empty_dev(p.grid.n, p.N)
        its = ope.ope_source_solve(ctx.handle, to_dev(U), Yd, None, 1e-14, k, allow_maxit=True)
        Y = to_host(Yd)
    st = {}
    Y_ref = O.cg_source(op, U, None, tol=1e-14, max_iter=k, stats=st)
    assert its == k and st["iterations"] == k
    assert np.max(np.abs(Y - Y_ref)) <= 1e-12 * np.max(np.abs(Y_ref))


def test_energy_residual_ritz_match_oracle():
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=14, N=24, seed=2)
    op = _op(p)
    U = p.U0
    say("energy/residual/ritz")
    with _ctx(p) as ctx:
        Ud = to_dev(U)
        E = ope.ope_energy(ctx.handle, Ud)
        res, ritz, drift = ope.ope_residual(ctx.handle, Ud, p.N)
    assert abs(E - O.energy(op, U)) <= 1e-13 * abs(O.energy(op, U))
    assert abs(res - O.residual(op, U)) <= 1e-12 * O.residual(op, U)
    r_ref = O.ritz_values(op, U)
    assert np.max(np.abs(ritz - r_ref)) <= 1e-12 * np.max(np.abs(r_ref))
    assert abs(drift - O.ortho_error(U)) <= 1e-14 * p.N


def test_autotune_single_context_keeps_results():
    """ope_autotune picks the fastest sweep shape by timing; H X and the CG
    solution then still match the oracle (a shape changes only the summation
    order of the CG dot products)."""
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=21, N=17, seed=6)
    op = _op(p)
    X = np.random.default_rng(4).standard_normal((p.grid.n, p.N))
    U = W.initial_block(p.grid.n, p.N, 9)
    say("autotune single context")
    with _ctx(p) as ctx:
        ope.ope_autotune(ctx.handle)
        q, mc, wgs = ope.ope_get_sweep_shape(ctx.handle)
        assert q in (1, 2, 4) and mc >= 1 and wgs >= 1
        Yd = empty_dev(p.grid.n, p.N)
        ope.ope_apply_h(ctx.handle, to_dev(X), Yd)
        Y = to_host(Yd)
        Sd = empty_dev(p.grid.n, p.N)
        ope.ope_source_solve(ctx.handle, to_dev(U), Sd, None, 1e-11, 20000)
        S = to_host(Sd)
    assert np.max(np.abs(Y - O.apply_H(op, X))) <= stencil_bound(op, X)
    assert np.all(np.linalg.norm(U - O.apply_H(op, S), axis=0) <= 20 * 1e-11)


@pytest.mark.parametrize("q_max,chunks,flags", [(1, 1, 0), (2, 3, 1), (4, 0, 2), (4, 5, 3), (1, 0, 3),
                                                 (2, 0, 9), (2, 3, 8), (1, 2, 11), (2, 0, 13),
                                                 (2, 0, 17), (2, 2, 19), (2, 0, 21),
                                                 (2, 0, 33), (2, 0, 36), (2, 2, 39), (2, 0, 37)])
def test_sweep_shapes_agree(q_max, chunks, flags):
    """Every launch shape of the marching sweeps computes the same H X, and the
    same CG solution up to the order of the dot-product sums (flags 8: two
    side lines per work-group; with 21 lines the last group is half empty, and
    its x segments of 15 points need segment-end neighbours; with 13 the
    8-vector chunks cover x whole; flags 16: four lines, segments of 7 points,
    the last group three quarters empty; flags 32 with 8-vector chunks: eight
    lines, segments of 8 points, the last group and segment 5/8 full; flags 32
    with whole rows (15 points per pass) falls back to four lines)."""
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=21, N=34, seed=6)
    op = _op(p)
    X = np.random.default_rng(3).standard_normal((p.grid.n, p.N))
    U = W.initial_block(p.grid.n, p.N, 8)
    say(f"sweep shape q={q_max} chunks={chunks} flags={flags}")
    with _ctx(p) as ctx:
        ope.ope_set_sweep_shape(ctx.handle, q_max, chunks, flags)
        Yd = empty_dev(p.grid.n, p.N)
        ope.ope_apply_h(ctx.handle, to_dev(X), Yd)
        Y = to_host(Yd)
        Sd = empty_dev(p.grid.n, p.N)
        ope.ope_source_solve(ctx.handle, to_dev(U), Sd, None, 1e-11, 20000)
        S = to_host(Sd)
    assert np.max(np.abs(Y - O.apply_H(op, X))) <= stencil_bound(op, X)
    assert np.all(np.linalg.norm(U - O.apply_H(op, S), axis=0) <= 20 * 1e-11)


@pytest.mark.parametrize("N", [80, 96, 128])
@pytest.mark.parametrize("narrow", [False, True])
def test_wide_row_chunks_agree(N, narrow):
    """Rows wider than 32 vector columns: by default a work-group takes the
    widest of 32, 16 and 8 vector columns that divides the row (N = 128 in
    FP64: 32, two chunks; N = 96: 16, three; N = 80: 8, five), with the narrow
    flag always 8; H X and the CG solution match the oracle either way."""
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=13, N=N, seed=7)
    op = _op(p)
    X = np.random.default_rng(5).standard_normal((p.grid.n, p.N))
    U = W.initial_block(p.grid.n, p.N, 10)
    say(f"wide row chunks N={N} narrow={narrow}")
    with _ctx(p) as ctx:
        if narrow:
            ope.ope_set_sweep_shape(ctx.handle, 2, 0, ope.OPE_SWEEP_CHUNK_MAJOR | ope.OPE_SWEEP_LINES8
                                    | ope.OPE_SWEEP_NARROW)
        Yd = empty_dev(p.grid.n, p.N)
        ope.ope_apply_h(ctx.handle, to_dev(X), Yd)
        Y = to_host(Yd)
        Sd = empty_dev(p.grid.n, p.N)
        ope.ope_source_solve(ctx.handle, to_dev(U), Sd, None, 1e-11, 20000)
        S = to_host(Sd)
    assert np.max(np.abs(Y - O.apply_H(op, X))) <= stencil_bound(op, X)
    assert np.all(np.linalg.norm(U - O.apply_H(op, S), axis=0) <= 20 * 1e-11)
