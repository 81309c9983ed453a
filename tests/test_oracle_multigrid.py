"""Pins of the multigrid oracle (oracle/multigrid.py): the preconditioner of
Step 1's CG in the library's preconditioned form.

* The transfers equal brute-force matrices built from their definition
  (weights 3/4 and 1/4 per coarsened axis, tensor products), and
  R = P^T / 2^d exactly.
* P reproduces constant and linear functions away from the boundary (the
  linear interpolation it is meant to be).
* The coarse potential is the mean over the existing children (loop).
* The V-cycle equals the dense two-grid formula B = (I - E) H^{-1} with
  E = (I - S H)(I - P H_c^{-1} R H)(I - S H), S = omega D^{-1}.
* The V-cycle is symmetric and positive definite, with a small condition
  number of B H on a three-level well problem.
* PCG with the identity preconditioner is textbook CG (cg_source), and PCG
  with the V-cycle reaches the sparse direct solution in far fewer iterations.
"""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import multigrid as MG


def _level(m, h=None, seed=0, kinetic=1.0):
    rng = np.random.default_rng(seed)
    h = h or tuple(1.0 / (ma + 1) for ma in m)
    return MG.Level(tuple(m), tuple(h), 10.0 * rng.uniform(size=int(np.prod(m))), kinetic)


def _w(f, I, mf):
    """Weight of coarse node I in fine node f along one coarsened axis."""
    if I == f // 2:
        return 0.75
    J = f // 2 - 1 if f % 2 == 0 else f // 2 + 1
    return 0.25 if I == J else 0.0


def _brute_P(m):
    mc = MG.coarse_shape(m)
    dim = len(m)
    nf, nc = int(np.prod(m)), int(np.prod(mc))
    P = np.zeros((nf, nc))
    fines = list(itertools.product(*[range(m[a]) for a in range(dim)]))
    coarses = list(itertools.product(*[range(mc[a]) for a in range(dim)]))
    lin = lambda idx, mm: sum(idx[a] * int(np.prod(mm[:a])) for a in range(dim))
    for f in fines:
        for I in coarses:
            w = 1.0
            for a in range(dim):
                w *= _w(f[a], I[a], m[a]) if m[a] > 1 else float(f[a] == I[a])
            P[lin(f, m), lin(I, mc)] = w
    return P


@pytest.mark.parametrize("m", [(7, 6), (5, 6, 3), (4, 1, 5), (9, 8, 2)])
def test_transfers_equal_brute_force(m):
    fine = _level(m)
    coarse = _level(MG.coarse_shape(m))
    nf, nc = fine.n, coarse.n
    P = MG.prolong(fine, coarse, np.eye(nc))
    R = MG.restrict(fine, coarse, np.eye(nf))
    assert np.array_equal(P, _brute_P(m))
    d = len(MG.coarsened_axes(m))
    assert np.allclose(R, P.T / 2 ** d, rtol=0, atol=1e-16)


def test_prolongation_reproduces_linear_functions():
    m = (16, 12, 10)
    fine, coarse = _level(m), _level(MG.coarse_shape(m))
    a, b = np.array([0.3, -1.2, 0.7]), 2.5
    # node-centred coordinates in fine-index units: coarse I sits at 2I + 1/2
    cg = np.stack(np.meshgrid(*[2.0 * np.arange(mc) + 0.5 for mc in coarse.m], indexing="ij"), -1)
    fg = np.stack(np.meshgrid(*[np.arange(mf, dtype=float) for mf in m], indexing="ij"), -1)
    ec = (b + cg @ a).transpose(2, 1, 0).reshape(-1, 1)           # x fastest
    ef = MG.prolong(fine, coarse, ec).reshape(m[::-1]).transpose(2, 1, 0)
    want = b + fg @ a
    inner = tuple(slice(1, mf - 1) for mf in m)
    assert np.max(np.abs(ef[inner] - want[inner])) <= 1e-12
    one = MG.prolong(fine, coarse, np.ones((coarse.n, 1))).reshape(m[::-1]).transpose(2, 1, 0)
    assert np.all(one[inner] == 1.0)
    # at the boundary the missing neighbour contributes zero
    assert one[0, 5, 5] == 0.75 and one[-1, 5, 5] == 0.75


@pytest.mark.parametrize("m", [(7, 6, 5), (8, 3)])
def test_coarse_potential_is_the_children_mean(m):
    fine = _level(m, seed=3)
    mc = MG.coarse_shape(m)
    Wc = MG.coarse_potential(fine, mc)
    dim = len(m)
    strides = [int(np.prod(m[:a])) for a in range(dim)]
    cstr = [int(np.prod(mc[:a])) for a in range(dim)]
    for I in itertools.product(*[range(mc[a]) for a in range(dim)]):
        kids = [f for f in itertools.product(*[range(m[a]) for a in range(dim)])
                if all(f[a] // 2 == I[a] for a in range(dim))]
        want = np.mean([fine.W[sum(f[a] * strides[a] for a in range(dim))] for f in kids])
        assert abs(Wc[sum(I[a] * cstr[a] for a in range(dim))] - want) <= 1e-14 * abs(want)


def test_vcycle_equals_dense_two_grid_formula():
    p = W.wells_3d(m=9, N=2, seed=2)
    op = O.Operator((9, 8, 7), tuple(1.0 / (x + 1) for x in (9, 8, 7)), p.V[:9 * 8 * 7], kinetic=0.5, shift=3.0)
    hier = O.Hierarchy(op, coarsest_max=100)
    assert len(hier.levels) == 2
    L0, L1 = hier.levels
    n = L0.n
    H = O.assemble_H(op).toarray()
    S = np.diag(hier.omega / L0.diag)
    P = MG.prolong(L0, L1, np.eye(L1.n))
    R = MG.restrict(L0, L1, np.eye(n))
    Hc = O.assemble_H(L1.op).toarray()
    I = np.eye(n)
    E = (I - S @ H) @ (I - P @ np.linalg.solve(Hc, R @ H)) @ (I - S @ H)
    B = (I - E) @ np.linalg.inv(H)
    Bv = hier.matrix()
    assert np.max(np.abs(Bv - B)) <= 1e-12 * np.max(np.abs(B))
    # L0.diag is the diagonal of the assembled operator
    assert np.allclose(L0.diag, np.diag(H), rtol=1e-15)


def test_vcycle_is_symmetric_positive_definite():
    p = W.wells_3d(m=14, N=2, seed=4)
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    hier = O.Hierarchy(op, coarsest_max=64)          # 14^3 -> 7^3 -> 4^3
    assert len(hier.levels) == 3
    B = hier.matrix()
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B))
    H = O.assemble_H(op).toarray()
    ev = np.sort(np.linalg.eigvals(B @ H).real)
    assert ev[0] > 0.1 and ev[-1] < 1.5
    assert ev[-1] / ev[0] < 8.0


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_pcg_with_identity_is_textbook_cg(k):
    p = W.wells_3d(m=12, N=5, seed=1)
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    a = O.pcg_source(op, p.U0, tol=1e-30, max_iter=k, precond=lambda r: r.copy())
    b = O.cg_source(op, p.U0, tol=1e-30, max_iter=k)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_pcg_reaches_the_direct_solution_in_few_iterations():
    p = W.wells_3d(m=24, N=4, seed=1)
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    G = O.GSolver(op, "sparse")
    ref = G(p.U0)
    st, st_cg = {}, {}
    Y = O.pcg_source(op, p.U0, tol=1e-11, stats=st)
    O.cg_source(op, p.U0, tol=1e-11, stats=st_cg)
    assert st["converged"] and st["iterations"] <= 20 and st_cg["iterations"] >= 100
    assert np.max(np.abs(Y - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_planted_wrong_weight_fails_the_two_grid_pin():
    """A restriction that averages the children only (a plausible slip) is not
    P^T / 2^d; the symmetric-pin check must see it."""
    m = (6, 5, 4)
    fine, coarse = _level(m), _level(MG.coarse_shape(m))
    P = MG.prolong(fine, coarse, np.eye(coarse.n))
    G = MG._grid(np.eye(fine.n), m)
    for a in MG.coarsened_axes(m):
        ax = MG._axis(a, 3)
        mf = G.shape[ax]
        G = np.stack([np.take(G, [f for f in (2 * I, 2 * I + 1) if f < mf], axis=ax).mean(axis=ax)
                      for I in range(MG.coarse_shape(m)[a])], axis=ax)
    R_bad = G.reshape(coarse.n, fine.n)
    assert not np.allclose(R_bad, P.T / 8.0, atol=1e-3)
