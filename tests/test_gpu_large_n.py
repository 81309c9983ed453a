"""GPU parity for block widths above 128 (Steps 2-3 by Newton-Schulz
inversion on the FP64 matrix cores, Step 4 through a side buffer).

* Grams at N = 200 and 512 equal numpy's to rounding.
* ope_small_solve at N = 160, 300 and 512 equals the oracle's Steps 2-3 to
  1e-12, for the well-conditioned Step-2 matrices the scheme produces.
* A full FP64 step at N = 160 equals the oracle's step; at N = 135 a rotated
  eigenbasis stays fixed and its Ritz values (widened Jacobi kernel) are the
  dense eigenvalues.
* The mixed form at 96^3, N = 512 (the large mixed-precision workload) takes
  steps with decreasing energy and FP32-level orthogonality drift, and its
  first-step energy matches the oracle on the same FP32 start block.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W
from tests.gpu_common import empty_dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _ctx(p, precision=0):
    from paper_2511_06788_amd import ope
    return ope.Context(p.grid, p.V, p.N, kinetic=p.kinetic, shift=p.shift, precision=precision)


def _step_inputs(n, N, seed):
    """S_b = U^T Y and T = Y^T Y for an orthonormal U and Y = G U of an SPD
    G with spectrum in [1e-3, 1e-1] plus a small perturbation (the shape the
    scheme produces)."""
    rng = np.random.default_rng(seed)
    U = W.initial_block(n, N, seed)
    Q = W.initial_block(n, n, seed + 1)
    g = rng.uniform(1e-3, 1e-1, n)
    Y = (Q * g) @ (Q.T @ U) + 1e-4 * rng.standard_normal((n, N))
    return U.T @ Y, Y.T @ Y


@pytest.mark.parametrize("N", [160, 300, 512])
def test_small_solve_large_n(N):
    from paper_2511_06788_amd import ope
    n = N + 40
    Sb, T = _step_inputs(n, N, N)
    tau = 30.0
    A_ref, B_ref, _ = O.small_solve(Sb.T, T, tau, S_b=Sb)
    p = W.Problem("ls", W.Grid(m=(n, 1), h=(1.0, 1.0), lo=(0.0, 0.0)), np.zeros(n), N, 1.0)
    say(f"small solve N={N}")
    with ope.Context(p.grid, p.V, N) as ctx:
        Z = empty_dev(2 * N, N)
        A = empty_dev(N, N)
        B = empty_dev(N, N)
        ope.ope_small_solve(ctx.handle, to_dev(Sb), to_dev(T), tau, Z, A, B)
        Bh, Ah, Zh = to_host(B), to_host(A), to_host(Z)
    assert np.max(np.abs(Bh - B_ref)) <= 1e-12 * np.max(np.abs(B_ref))
    assert np.max(np.abs(Ah - A_ref)) <= 1e-12 * np.max(np.abs(A_ref))
    I = np.eye(N)
    assert np.max(np.abs(Zh[:N] - (I - tau * A_ref))) <= 1e-11
    assert np.max(np.abs(Zh[N:] - tau * B_ref)) <= 1e-11


@pytest.mark.parametrize("N", [200, 512])
def test_gram_large_n(N):
    """Grams at N > 128 (the split-K partial buffer is sized per tile count)."""
    from paper_2511_06788_amd import ope
    rng = np.random.default_rng(N)
    A = rng.standard_normal((N, N))
    B = rng.standard_normal((N, N))
    p = W.Problem("sq", W.Grid(m=(N + 8, 1), h=(1.0, 1.0), lo=(0.0, 0.0)), np.zeros(N + 8), N, 1.0)
    say(f"gram N={N}")
    with ope.Context(p.grid, p.V, N) as ctx:
        out = empty_dev(N, N)
        ope.ope_gram(ctx.handle, to_dev(A), N, N, to_dev(B), N, N, N, out)
        G = to_host(out)
    assert np.max(np.abs(G - A.T @ B)) <= 1e-12 * np.max(np.abs(A.T @ B))


def test_fp64_step_large_n_matches_oracle():
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=14, N=160, seed=3)
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    tau = 20.0
    ref = O.steps_1_to_4(p.U0, O.GSolver(op, "dense"), tau)["U"]
    say("fp64 step N=160")
    with _ctx(p) as ctx:
        ope.ope_set_inner(ctx.handle, 0.0, 1e-13, 20000)
        U = to_dev(p.U0)
        info = ope.ope_step(ctx.handle, U, tau)
        Un = to_host(U)
    assert np.max(np.abs(Un - ref)) <= 1e-10
    assert O.ortho_error(Un) <= 1e-12
    assert abs(info.energy - O.energy(op, p.U0)) <= 1e-12 * abs(info.energy)


def test_large_n_eigenbasis_is_fixed_point_and_ritz():
    """A rotated eigenbasis (U* Q) is a fixed point of the step (Remark after
    (3.1)); its Ritz values from the widened Jacobi kernel are the dense
    eigenvalues.  (Converging from a random block at N > 128 takes thousands
    of steps: the relative gap at the cut shrinks with N.)"""
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=11, N=135, seed=3, with_u0=False)
    H = O.assemble_H(O.Operator(p.grid.m, p.grid.h, p.V)).toarray()
    w_all, V = np.linalg.eigh(H)
    w = w_all[:p.N]
    Q = W.initial_block(p.N, p.N, 5)
    U0 = V[:, :p.N] @ Q
    say("fixed point N=135")
    with _ctx(p) as ctx:
        ope.ope_set_inner(ctx.handle, 0.0, 1e-13, 20000)
        U = to_dev(U0)
        res0, ritz, drift = ope.ope_residual(ctx.handle, U, p.N)
        for _ in range(3):
            ope.ope_step(ctx.handle, U, 40.0)
        U1 = to_host(U)
    assert np.max(np.abs(ritz - w) / np.abs(w)) <= 1e-12
    assert res0 <= 1e-12 and drift <= 1e-12
    assert np.max(np.abs(U1 - U0)) <= 1e-10


def test_mixed_96_cubed_n512_steps():
    from paper_2511_06788_amd import ope
    p = W.wells_3d(m=96, N=512, seed=0)
    U32 = p.U0.astype(np.float32)
    rows = np.random.default_rng(0).choice(p.grid.n, 2048, replace=False)
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    say("mixed 96^3 N=512")
    import torch
    with _ctx(p, 1) as ctx:
        U = torch.from_numpy(U32).to("cuda")
        i1 = ope.ope_step(ctx.handle, U, 45.0)
        i2 = ope.ope_step(ctx.handle, U, 45.0)
        res, _, drift = ope.ope_residual(ctx.handle, U, p.N, want_ritz=False)
    U64 = U32.astype(np.float64)
    E_ref = O.energy(op, U64)
    assert abs(i1.energy - E_ref) <= 1e-6 * abs(E_ref)
    assert i2.energy < i1.energy
    # the device drift check after every update keeps the block below the 1e-6 target
    assert i1.drift <= 1e-6 and i2.drift <= 1e-6 and drift <= 1e-6
    assert np.isfinite(res)
