"""Pins of the oracle against the paper's printed numbers (Table 1) and planted-mistake checks.

Table 1 (Section 5.1) lists, for the 2D harmonic oscillator with N = 15 and a
random orthonormal start, the number of steps until the relative energy error
drops below 1e-10.  The oracle runs a finite-difference analogue (99 x 99
interior grid on (-5.5, 5.5)^2, ``-1/2 Lap + 1/2 |x|^2``) with the same N, step
sizes and stop rule.  The step counts depend only on the spectral gap
``1/lambda_15 - 1/lambda_16``, which the discretisation barely changes, so they
must land close to the printed ones; the eigenvalue errors show the printed
pattern (first ten shells ~1e-13 or better, the top shell much larger).

The planted-mistake tests make a plausible slip in a copy of an oracle formula
and check that a pin fails, so that the pins above are known to bite.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_table1.json")


@pytest.fixture(scope="module")
def oscillator():
    p = W.oscillator_2d_paper(m=99)
    op = O.Operator(p.grid.m, p.grid.h, p.V, kinetic=0.5)
    H = O.assemble_H(op).tocsc()
    w = np.sort(spla.eigsh(H, k=18, sigma=0, return_eigenvectors=False))
    return p, op, O.GSolver(op, "sparse"), w


def test_fd_oscillator_spectrum_near_continuum(oscillator):
    p, op, G, w = oscillator
    ref = json.load(open(GOLDEN))["continuum_eigenvalues_first_16"]
    assert np.max(np.abs(w[:16] - np.array(ref))) < 0.03
    assert w[14] < w[15] - 0.9                         # N = 15 closes a shell


@pytest.mark.parametrize("tau", [0.5, 1.0, 1.5])
def test_table1_step_counts(oscillator, tau):
    p, op, G, w = oscillator
    g = json.load(open(GOLDEN))
    printed = dict(zip(g["tau"], g["steps"]))[tau]
    Egs = 0.5 * w[:15].sum()                            # E(U*) = 1/2 sum lambda_i
    U = p.U0.copy()
    steps = 0
    while True:
        U = O.steps_1_to_4(U, G, tau)["U"]
        steps += 1
        if (O.energy(op, U) - Egs) / Egs < 1e-10 or steps > 3 * printed:
            break
    assert abs(steps - printed) <= 0.15 * printed, (steps, printed)
    err = np.abs(O.ritz_values(op, U) - w[:15]) / w[:15]
    assert err[:10].max() <= max(g["err_first_ten_max"])
    assert err[10:].max() <= max(g["err_last_five_max"])
    assert O.ortho_error(U) <= 1e-12


# ---------------------------------------------------------------------------
# planted mistakes (CPU only): each must be caught by a pin
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_case():
    p = W.harmonic_2d_32(m=12, N=4)
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    G = O.GSolver(op, "dense")
    return p, op, G


def _step_with(U, Y, tau, mutate):
    S = O.inner(Y, U)
    T = O.inner(Y, Y)
    N = U.shape[1]
    I = np.eye(N)
    M = I + 0.25 * tau * tau * (T - S @ S)
    if mutate == "sign_step2":
        M = I - 0.25 * tau * tau * (T - S @ S)
    B = np.linalg.solve(M, I)
    A = (2.0 / tau) * (I - B + 0.5 * tau * S @ B)
    if mutate == "half_A":
        A = (1.0 / tau) * (I - B + 0.5 * tau * S @ B)
    if mutate == "drop_SB":
        A = (2.0 / tau) * (I - B)
    Un = U - tau * U @ A + tau * Y @ B
    if mutate == "sign_update":
        Un = U + tau * U @ A - tau * Y @ B
    if mutate == "swap_AB":
        Un = U - tau * U @ B + tau * Y @ A
    return Un


@pytest.mark.parametrize("mutate", ["sign_step2", "half_A", "drop_SB", "sign_update", "swap_AB"])
def test_planted_step_mistakes_are_caught(small_case, mutate):
    p, op, G, = small_case
    U = p.U0
    Y = G(U)
    tau = 5.0
    good = _step_with(U, Y, tau, None)
    assert np.max(np.abs(good - O.step_cayley_dense(U, Y, tau))) <= 1e-12
    bad = _step_with(U, Y, tau, mutate)
    caught = (np.max(np.abs(bad - O.step_cayley_dense(U, Y, tau))) > 1e-8
              or O.ortho_error(bad) > 1e-8)
    assert caught


@pytest.mark.parametrize("mutate", ["periodic", "h_not_squared", "no_kinetic"])
def test_planted_operator_mistakes_are_caught(mutate):
    m = (6, 5)
    h = (1.0 / 7, 1.0 / 6)
    n = 30
    op = O.Operator(m, h, np.zeros(n), kinetic=0.5)
    X = np.eye(n)
    H = O.apply_H(op, X)
    Hb = H.copy()
    if mutate == "periodic":
        Xg = X.reshape(5, 6, n)
        Hb = H - (np.roll(Xg, 1, axis=1) - np.pad(Xg[:, :-1], ((0, 0), (1, 0), (0, 0)))).reshape(n, n) * 0.5 / h[0] ** 2
    elif mutate == "h_not_squared":
        Hb = H * h[0]
    elif mutate == "no_kinetic":
        Hb = H / 0.5
    w = np.linalg.eigvalsh(0.5 * (Hb + Hb.T))
    ref = np.sort([0.5 * ((4 / h[0] ** 2) * np.sin(i * np.pi / 14) ** 2 + (4 / h[1] ** 2) * np.sin(j * np.pi / 12) ** 2)
                   for i in range(1, 7) for j in range(1, 6)])
    assert np.allclose(np.linalg.eigvalsh(H), ref, rtol=1e-12)
    assert not np.allclose(w, ref, rtol=1e-6)
