"""Pins of the oracle's scheme in the inner product of a mass operator M.

Section 5 writes every block in a finite-element basis, so inner products of
coefficient blocks carry the mass matrix and Step 1 solves ``K (GU) = M U``.
The finite-difference stand-in ``M = diag(d) + sum_a mu_a (S_a + S_a^T)`` is
pinned by:

* brute force: ``apply_M`` and ``assemble_M`` against a pure-Python loop over
  points and their axis neighbours;
* closed form: for constant V, d and mu the sine modes diagonalise both K and
  M, so the generalized eigenvalues are ``(c sum_a s_a(j) + V) / (d + 2 sum_a
  mu_a cos(j_a pi / (m_a + 1)))`` (textbook), and ``lowest_eigenpairs`` must
  return the smallest of them;
* M = I reduces every ``*_M`` function to its Euclidean form;
* equivariance: with ``M = L L^T`` (Cholesky), ``U~ = L^T U`` and
  ``K~ = L^{-1} K L^{-T}``, one M-step of U is ``L^{-T}`` times one Euclidean
  step of ``U~`` for the operator ``K~`` (a different computation path);
* (4.1) written densely with the M-product generator equals Steps 1-4_M;
* Theorem 4.1 (``U^T M U`` stays I), Theorem 4.2 (the energy decays), the
  fixed point at an M-orthonormal eigenbasis, and convergence to the
  generalized eigenvalues of dense ``eigh(K, M)`` with ``E = 1/2 sum lambda``;
* ``orthonormalize_M``: ``U^T M U = I`` afterwards and the change of basis is
  upper triangular with a positive diagonal.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W


def _case(m=(9, 7), seed=0, N=4):
    g = W.unit_box_grid(m)
    V = W.harmonic_potential(g, 60.0, (0.45, 0.55))
    op = O.Operator(g.m, g.h, V)
    rng = np.random.default_rng(seed)
    d = 1.0 + 0.3 * rng.uniform(size=g.n)
    mass = O.Mass(d, (0.12, -0.09))
    U0 = W.initial_block(g.n, N, seed)
    return op, mass, U0


def test_apply_and_assemble_match_brute_force():
    m = (4, 3, 5)
    n = int(np.prod(m))
    rng = np.random.default_rng(3)
    op = O.Operator(m, (0.2, 0.25, 1 / 6), rng.standard_normal(n))
    mass = O.Mass(2.0 + rng.uniform(size=n), (0.1, -0.2, 0.3))
    X = rng.standard_normal((n, 3))
    ref = np.zeros_like(X)
    for i2, i1, i0 in itertools.product(range(m[2]), range(m[1]), range(m[0])):
        p = i0 + m[0] * (i1 + m[1] * i2)
        ref[p] = mass.d[p] * X[p]
        idx = [i0, i1, i2]
        for a in range(3):
            for s in (-1, 1):
                j = list(idx)
                j[a] += s
                if 0 <= j[a] < m[a]:
                    q = j[0] + m[0] * (j[1] + m[1] * j[2])
                    ref[p] += mass.mu[a] * X[q]
    assert np.max(np.abs(O.apply_M(op, mass, X) - ref)) <= 1e-13
    assert np.max(np.abs(O.assemble_M(op, mass) @ X - ref)) <= 1e-13


def test_generalized_spectrum_closed_form():
    m = (8, 6)
    h = tuple(1.0 / (k + 1) for k in m)
    n = int(np.prod(m))
    v, d, mu = 3.5, 1.2, (0.2, -0.15)
    op = O.Operator(m, h, np.full(n, v))
    mass = O.Mass(np.full(n, d), mu)
    vals = []
    for j0, j1 in itertools.product(range(1, m[0] + 1), range(1, m[1] + 1)):
        kval = (4 / h[0] ** 2) * np.sin(j0 * np.pi / (2 * (m[0] + 1))) ** 2 \
            + (4 / h[1] ** 2) * np.sin(j1 * np.pi / (2 * (m[1] + 1))) ** 2 + v
        mval = d + 2 * mu[0] * np.cos(j0 * np.pi / (m[0] + 1)) + 2 * mu[1] * np.cos(j1 * np.pi / (m[1] + 1))
        vals.append(kval / mval)
    ref = np.sort(vals)[:10]
    got, vecs, res = O.lowest_eigenpairs(op, 10, mass=mass)
    assert np.max(np.abs(got - ref) / ref) <= 1e-12
    assert np.max(res) <= 1e-9 * ref[-1]


def test_identity_mass_reduces_to_euclidean():
    op, _, U0 = _case()
    mass = O.Mass(np.ones(op.n), (0.0, 0.0))
    G = O.GSolver(op, "dense")
    a = O.steps_1_to_4_M(op, mass, U0, G, 7.0)["U"]
    b = O.steps_1_to_4(U0, G, 7.0)["U"]
    assert np.max(np.abs(a - b)) <= 1e-14
    assert O.residual_M(op, mass, U0) == pytest.approx(O.residual(op, U0), rel=1e-14)
    assert O.ortho_error_M(op, mass, U0) == pytest.approx(O.ortho_error(U0), abs=1e-15)


@pytest.mark.parametrize("tau", [0.5, 9.0])
def test_cholesky_equivariance(tau):
    op, mass, U0 = _case()
    K = O.assemble_H(op).toarray()
    Md = O.assemble_M(op, mass).toarray()
    L = np.linalg.cholesky(Md)
    U = O.orthonormalize_M(op, mass, U0)
    Ut = L.T @ U
    Kt = np.linalg.solve(L, np.linalg.solve(L, K).T)     # L^{-1} K L^{-T} (K symmetric)
    step_t = O.steps_1_to_4(Ut, lambda X: np.linalg.solve(Kt, X), tau)["U"]
    want = np.linalg.solve(L.T, step_t)
    got = O.steps_1_to_4_M(op, mass, U, O.GSolver(op, "dense"), tau)["U"]
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


def test_dense_cayley_equals_steps():
    op, mass, U0 = _case()
    U = O.orthonormalize_M(op, mass, U0)
    G = O.GSolver(op, "dense")
    Md = O.assemble_M(op, mass).toarray()
    out = O.steps_1_to_4_M(op, mass, U, G, 3.0)
    dense = O.step_cayley_dense_M(Md, U, out["Y"], 3.0)
    assert np.max(np.abs(out["U"] - dense)) <= 1e-12
    gen = O.step_general_M(op, mass, U, out["Y"], 3.0)["U"]
    assert np.max(np.abs(out["U"] - gen)) <= 1e-12


def test_orthonormalize_is_upper_triangular_change_of_basis():
    op, mass, U0 = _case()
    U = O.orthonormalize_M(op, mass, U0)
    assert O.ortho_error_M(op, mass, U) <= 1e-13
    R = O.inner_M(op, mass, U, U0)              # U0 = U R
    assert np.max(np.abs(np.tril(R, -1))) <= 1e-13
    assert np.all(np.diag(R) > 0)
    assert np.max(np.abs(U @ R - U0)) <= 1e-13


def test_run_preserves_m_orthonormality_and_converges():
    op, mass, U0 = _case(N=4)
    N = 4
    G = O.GSolver(op, "dense")
    K = O.assemble_H(op).toarray()
    Md = O.assemble_M(op, mass).toarray()
    w, X = sla.eigh(K, Md)
    # fixed point: an M-orthonormal eigenbasis does not move
    Ustar = X[:, :N]
    assert np.max(np.abs(O.steps_1_to_4_M(op, mass, Ustar, G, 5.0)["U"] - Ustar)) <= 1e-12
    tcrit = 2.0 / (1.0 / w[0] - 1.0 / w[-1])
    tau = 0.8 * tcrit
    U = O.orthonormalize_M(op, mass, U0)
    E = O.energy(op, U)
    for k in range(3000):
        U = O.steps_1_to_4_M(op, mass, U, G, tau)["U"]
        E_new = O.energy(op, U)
        assert E_new <= E + 1e-13 * abs(E)
        E = E_new
        assert O.ortho_error_M(op, mass, U) <= 1e-12
        if O.residual_M(op, mass, U) <= 1e-12:
            break
    assert O.residual_M(op, mass, U) <= 1e-12
    ritz = O.ritz_values_M(op, mass, U)
    assert np.max(np.abs(ritz - w[:N]) / w[:N]) <= 1e-12
    assert abs(O.energy(op, U) - 0.5 * w[:N].sum()) <= 1e-12 * w[:N].sum()
