"""Pins of the oracle's time step against the paper's theorems and independent forms.

* Lemma 3.2: ``L_U`` is skew for any U, V, W (not only orthonormal U).
* Lemma 3.1: ``<GU,GU> - <GU,U><GU,U>`` is positive semidefinite, so the Step-2
  matrix is ``>= I``.
* (4.1) three ways: Steps 1-4, a dense n x n Cayley solve and the 2N x 2N
  Woodbury form agree; the general elimination equals the dense solve for an
  inexact Y.
* Theorem 4.1 (orthogonality), Theorem 4.2 (energy decay), the steady state
  of the remark after (3.1) (an eigenbasis, also rotated, does not move), the
  ground-state energy ``E_GS = 1/2 sum lambda_i`` (Section 3.3) and
  convergence to dense ``eigh`` eigenvalues.
* The linearisation at the fixed point: every out-of-span mode is multiplied by
  ``1 - tau (1/lambda_i - 1/mu)`` per step, so the scheme is stable exactly for
  ``tau < 2 / (1/lambda_1 - 1/lambda_max)`` and the slow factor is
  ``1 - tau (1/lambda_N - 1/lambda_{N+1})``; its small-tau limit is the
  continuous rate of Theorem 3.11.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.fixture(scope="module")
def cfg1():
    p = W.harmonic_2d_32()
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    H = O.assemble_H(op).toarray()
    w, X = np.linalg.eigh(H)
    return p, op, O.GSolver(op, "dense"), w, X


def test_generator_is_skew_for_any_blocks():
    rng = np.random.default_rng(0)
    n, N = 40, 5
    U, Y, V, Wb = (rng.standard_normal((n, N)) for _ in range(4))
    lhs = O.inner(V, O.generator_apply(U, Y, Wb)) + O.inner(O.generator_apply(U, Y, V), Wb)
    assert np.max(np.abs(lhs)) <= 1e-12 * np.max(np.abs(O.inner(V, O.generator_apply(U, Y, Wb))))
    L = O.generator_matrix(U, Y)
    assert np.allclose(L, -L.T, atol=1e-13)
    assert np.allclose(L @ V, O.generator_apply(U, Y, V), atol=1e-12)


def test_lemma_3_1_psd_and_step2_matrix(cfg1):
    p, op, G, w, X = cfg1
    U = p.U0
    Y = G(U)
    S = O.inner(Y, U)
    T = O.inner(Y, Y)
    D = T - S @ S
    ev = np.linalg.eigvalsh(0.5 * (D + D.T))
    assert ev.min() >= -1e-14 * np.abs(ev).max()
    for tau in (0.1, 10.0, 1e3):
        A, B, M = O.small_solve(S, T, tau)
        assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() >= 1.0 - 1e-12
        assert np.linalg.norm(B, 2) <= 1.0 + 1e-12


@pytest.mark.parametrize("tau", [0.1, 5.0, 40.0])
def test_three_forms_of_the_step_agree(cfg1, tau):
    p, op, G, w, X = cfg1
    U = p.U0
    out = O.steps_1_to_4(U, G, tau)
    Y = out["Y"]
    Uc = O.step_cayley_dense(U, Y, tau)
    Uw = O.step_woodbury(U, Y, tau)
    Ug = O.step_general(U, Y, tau)["U"]
    for other in (Uc, Uw, Ug):
        assert np.max(np.abs(out["U"] - other)) <= 1e-12


def test_general_elimination_matches_dense_cayley_for_inexact_Y(cfg1):
    p, op, G, w, X = cfg1
    U = p.U0
    rng = np.random.default_rng(7)
    Y = G(U) + 1e-3 * rng.standard_normal(U.shape) / 25.0      # S = Y^T U no longer symmetric
    S = O.inner(Y, U)
    assert np.max(np.abs(S - S.T)) > 1e-6
    tau = 20.0
    Uc = O.step_cayley_dense(U, Y, tau)
    Ug = O.step_general(U, Y, tau)["U"]
    assert np.max(np.abs(Uc - Ug)) <= 1e-12
    assert O.ortho_error(Ug) <= 1e-13           # orthogonality holds for any Y
    # the symmetric-S formula is a different map once S is not symmetric
    Up = U - tau * U @ O.small_solve(S, O.inner(Y, Y), tau)[0] + tau * Y @ O.small_solve(S, O.inner(Y, Y), tau)[1]
    assert np.max(np.abs(Up - Uc)) > 1e-8


def test_cfg1_literal_run_orthogonality_and_energy(cfg1):
    """Theorem 4.1 and Theorem 4.2 on the 32x32 harmonic problem, tau = 0.1, 300 steps."""
    p, op, G, w, X = cfg1
    r = O.run_algorithm1(op, p.U0, 0.1, G, 300)
    E = np.array(r["hist"]["E"])
    assert r["steps"] == 300
    assert max(r["hist"]["ortho"]) <= 1e-12
    assert np.all(np.diff(E) <= 1e-14 * abs(E[0]))
    assert E[-1] < E[0] and E[-1] >= 0.5 * w[:8].sum()


def test_eigenbasis_is_a_fixed_point(cfg1):
    p, op, G, w, X = cfg1
    Ustar = X[:, :8]
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((8, 8)))
    for U in (Ustar, Ustar @ Q):
        for tau in (0.1, 30.0):
            Un = O.steps_1_to_4(U, G, tau)["U"]
            assert np.max(np.abs(Un - U)) <= 1e-12


def test_converges_to_dense_eigenvalues(cfg1):
    p, op, G, w, X = cfg1
    r = O.run_algorithm1(op, p.U0, 40.0, G, 2000, res_tol=1e-11, record=False)
    U = r["U"]
    assert r["hist"]["res"][-1] <= 1e-11
    ritz = O.ritz_values(op, U)
    assert np.max(np.abs(ritz - w[:8]) / w[:8]) <= 1e-12
    assert abs(O.energy(op, U) - 0.5 * w[:8].sum()) <= 1e-12 * w[:8].sum()
    assert O.subspace_distance(U, X[:, :8]) <= 1e-9
    pe = O.paper_eigenvalues(U, G(U))
    assert np.max(np.abs(pe - w[:8]) / w[:8]) <= 1e-11


def _slow_factor(op, U0, G, tau, steps, Ustar):
    U = U0.copy()
    d = []
    for k in range(steps):
        U = O.steps_1_to_4(U, G, tau)["U"]
        d.append(O.subspace_distance(U, Ustar))
    d = np.array(d)
    half = steps // 2
    return np.exp(np.polyfit(np.arange(half, steps), np.log(d[half:]), 1)[0])


def test_stability_threshold_and_rate(cfg1):
    """Fixed-point linearisation: factor 1 - tau*kappa per mode, kappa in
    [1/l_N - 1/l_{N+1}, 1/l_1 - 1/l_max]."""
    p, op, G, w, X = cfg1
    N = 8
    kmax = 1 / w[0] - 1 / w[-1]
    kmin = 1 / w[N - 1] - 1 / w[N]
    tcrit = 2.0 / kmax
    # start close to the fixed point so that only the linearisation matters
    rng = np.random.default_rng(2)
    U0, _ = np.linalg.qr(X[:, :N] + 1e-4 * rng.standard_normal((X.shape[0], N)))
    ok = O.run_algorithm1(op, U0, 0.97 * tcrit, G, 400, record=False)["U"]
    bad = O.run_algorithm1(op, U0, 1.03 * tcrit, G, 400, record=False)["U"]
    assert O.subspace_distance(ok, X[:, :N]) < 1e-6
    assert O.subspace_distance(bad, X[:, :N]) > 1e-3
    tau = 20.0
    f = _slow_factor(op, U0, G, tau, 300, X[:, :N])
    assert abs(f - (1 - tau * kmin)) <= 0.02 * (tau * kmin)


def test_small_tau_rate_is_theorem_3_11(cfg1):
    """For small tau the energy error decays like exp(-2 (1/l_N - 1/l_{N+1}) t)."""
    p, op, G, w, X = cfg1
    N = 8
    kmin = 1 / w[N - 1] - 1 / w[N]
    # perturb the top pair of the block along the next pair, so that only the
    # slowest out-of-span mode is excited
    P = X[:, :N].copy()
    P[:, N - 2:N] += 1e-2 * X[:, N:N + 2]
    U0, _ = np.linalg.qr(P)
    tau = 2.0
    U = U0.copy()
    Egs = 0.5 * w[:N].sum()
    err = []
    for k in range(400):
        U = O.steps_1_to_4(U, G, tau)["U"]
        err.append(O.energy(op, U) - Egs)
    err = np.array(err)
    slope = np.polyfit(np.arange(200, 400) * tau, np.log(err[200:]), 1)[0]
    assert abs(-slope - 2 * kmin) <= 0.05 * 2 * kmin


def test_delta_form_equals_general_step(cfg1):
    """The delta form is Steps 2-4 rewritten (Step 3 substituted into Step 4,
    T - S_a S_b expressed through the projected block): identical to the
    general step for any U (also not orthonormal) and any Y."""
    p, op, G, w, X = cfg1
    U = p.U0
    rng = np.random.default_rng(9)
    E = rng.standard_normal((8, 8)) * 1e-3
    for Uc in (U, U @ (np.eye(8) + 0.5 * (E + E.T))):
        for Y in (G(Uc), G(Uc) + 1e-3 * rng.standard_normal(U.shape) / 25.0):
            for tau in (0.1, 20.0, 45.0):
                a = O.step_general(Uc, Y, tau)["U"]
                b = O.step_delta(Uc, Y, tau)["U"]
                assert np.max(np.abs(a - b)) <= 1e-12
