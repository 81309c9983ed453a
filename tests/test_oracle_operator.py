"""Pins of the oracle's operator and solvers against closed forms and brute force.

* The discrete Dirichlet Laplacian on a uniform grid has the sine modes
  ``prod_a sin(j_a pi (i_a + 1) / (m_a + 1))`` as exact eigenvectors with
  eigenvalues ``sum_a (4 / h_a^2) sin^2(j_a pi / (2 (m_a + 1)))`` (textbook).
* Brute force: a pure-Python loop over points and neighbours on tiny grids.
* Step 1 (``G = H^{-1}``): the residual ``|H Y - U|`` and agreement of three
  independent solvers (dense Cholesky, sparse LU, per-column CG).
"""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W


def _closed_form_eigs(m, h, kinetic, shift):
    per_axis = [(4.0 / (h[a] ** 2)) * np.sin(np.arange(1, m[a] + 1) * np.pi / (2 * (m[a] + 1))) ** 2
                for a in range(len(m))]
    vals = [kinetic * sum(c) + shift for c in itertools.product(*per_axis)]
    return np.sort(np.array(vals))


def _sine_mode(m, js):
    v = None
    for a in range(len(m)):
        s = np.sin(js[a] * np.pi * (np.arange(m[a]) + 1) / (m[a] + 1))
        v = s if v is None else np.multiply.outer(s, v)   # slower axes outermost
    return v.ravel()


@pytest.mark.parametrize("m,h,kinetic,shift", [
    ((7, 5), (0.125, 1.0 / 6), 1.0, 0.0),
    ((4, 3, 5), (0.2, 0.25, 1.0 / 6), 0.5, 2.5),
])
def test_dense_spectrum_matches_closed_form(m, h, kinetic, shift):
    n = int(np.prod(m))
    op = O.Operator(m, h, np.zeros(n), kinetic=kinetic, shift=shift)
    H = O.assemble_H(op).toarray()
    assert np.allclose(H, H.T)
    w = np.linalg.eigvalsh(H)
    ref = _closed_form_eigs(m, h, kinetic, shift)
    assert np.max(np.abs(w - ref)) <= 1e-12 * np.max(ref)


@pytest.mark.parametrize("m", [(9, 6), (5, 4, 6)])
def test_sine_modes_are_eigenvectors_of_matrix_free_apply(m):
    h = tuple(1.0 / (k + 1) for k in m)
    n = int(np.prod(m))
    c = 3.25
    op = O.Operator(m, h, np.full(n, c))
    cols, lams = [], []
    for js in [(1,) * len(m), (2,) + (1,) * (len(m) - 1), tuple(k for k in m)]:
        cols.append(_sine_mode(m, js))
        lams.append(sum((4.0 / h[a] ** 2) * np.sin(js[a] * np.pi / (2 * (m[a] + 1))) ** 2
                        for a in range(len(m))) + c)
    X = np.stack(cols, axis=1)
    HX = O.apply_H(op, X)
    assert np.max(np.abs(HX - X * np.array(lams)[None, :])) <= 1e-11 * max(lams)


def test_apply_matches_brute_force_loops():
    rng = np.random.default_rng(3)
    m = (4, 3, 5)
    h = (0.3, 0.2, 0.25)
    n = int(np.prod(m))
    V = rng.uniform(-2, 5, n)
    X = rng.standard_normal((n, 3))
    op = O.Operator(m, h, V, kinetic=0.7, shift=0.4)
    Y = np.zeros_like(X)
    for i2, i1, i0 in itertools.product(range(m[2]), range(m[1]), range(m[0])):
        p = i0 + m[0] * (i1 + m[1] * i2)
        idx = (i0, i1, i2)
        acc = np.zeros(3)
        for a in range(3):
            acc += 2.0 * X[p] / h[a] ** 2
            for d in (-1, 1):
                j = list(idx)
                j[a] += d
                if 0 <= j[a] < m[a]:
                    q = j[0] + m[0] * (j[1] + m[1] * j[2])
                    acc -= X[q] / h[a] ** 2
        Y[p] = 0.7 * acc + (V[p] + 0.4) * X[p]
    assert np.allclose(O.apply_H(op, X), Y, rtol=1e-14, atol=1e-12)
    assert np.allclose(O.assemble_H(op) @ X, Y, rtol=1e-14, atol=1e-12)


def test_solvers_agree_and_solve():
    p = W.wells_3d(m=10, N=6, seed=5)
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    U = p.U0
    Yd = O.GSolver(op, "dense")(U)
    Ys = O.GSolver(op, "sparse")(U)
    st = {}
    Yc = O.cg_source(op, U, tol=1e-13, stats=st)
    assert st["converged"]
    for Y in (Yd, Ys, Yc):
        assert np.linalg.norm(O.apply_H(op, Y) - U) <= 1e-11 * np.linalg.norm(U)
    assert np.allclose(Yd, Ys, rtol=0, atol=1e-13)
    assert np.allclose(Yd, Yc, rtol=0, atol=1e-12)


def test_cg_warm_start_exact_solution_takes_no_iterations():
    p = W.wells_3d(m=8, N=4, seed=1)
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    Y = O.GSolver(op, "dense")(p.U0)
    st = {}
    O.cg_source(op, p.U0, Y0=Y, tol=1e-10, stats=st)
    assert st["iterations"] == 0


def test_wells_operator_is_positive_definite():
    """The Gaussian-well family keeps H SPD on small grids (the paper's
    coercivity assumption, Section 2.2); the dense factorisation would raise."""
    for seed in range(3):
        p = W.wells_3d(m=12, N=4, seed=seed, with_u0=False)
        op = O.Operator(p.grid.m, p.grid.h, p.V)
        O.GSolver(op, "dense")
