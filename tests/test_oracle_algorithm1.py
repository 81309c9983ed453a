"""Pins of Algorithm 1's stopping rule and of the adaptive step choice.

* The stop ``err_E = |E(U^{n+1}) - E(U^n)| / |E(U^n)| <= eps`` (Algorithm 1)
  is checked against the energy history of a fixed-step run: the oracle must
  stop at the first step where the relative change is at most eps, not one
  step earlier or later, and an absolute-change slip (|E| is about 350 here)
  would stop elsewhere.  ``err_E^0 = |E(U^0)|`` makes eps >= |E(U^0)| take no
  step.
* The step counts follow the rate model of the fixed-point linearisation: the
  energy change decays like ``rho^(2n)`` with the slow factor
  ``rho = 1 - tau (1/lambda_N - 1/lambda_{N+1})`` (dense eigenvalues), so
  tightening eps by 1e4 adds ``ln(1e4) / (-2 ln rho)`` steps.
* The adaptive rule: with ``tau_min = tau_max`` it is Algorithm 1 at that
  step, bit for bit; started far above the stability limit it rejects steps,
  keeps every accepted energy non-increasing (Theorem 4.2), stays in
  ``[tau_min, tau_max]`` and converges to the dense eigenvalues, stopping
  at the first step whose relative energy error (Section 5) is below eps.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.fixture(scope="module")
def cfg1():
    p = W.harmonic_2d_32()
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    w = np.linalg.eigvalsh(O.assemble_H(op).toarray())
    return p, op, O.GSolver(op, "dense"), w


def test_energy_stop_is_the_first_relative_change_below_tol(cfg1):
    p, op, G, w = cfg1
    tau = 40.0
    ref = O.run_algorithm1(op, p.U0, tau, G, 400, record=True)
    E = np.array(ref["hist"]["E"])
    assert abs(E[0]) > 100.0
    rel = np.abs(np.diff(E)) / np.abs(E[:-1])
    absd = np.abs(np.diff(E))
    for tol in (1e-4, 1e-8, 1e-11):
        first = int(np.argmax(rel <= tol)) + 1          # steps taken when the rule first holds
        assert rel[first - 1] <= tol and np.all(rel[:first - 1] > tol)
        r = O.run_algorithm1(op, p.U0, tau, G, 1000, energy_tol=tol, record=False)
        assert r["steps"] == first, (tol, r["steps"], first)
        first_abs = int(np.argmax(absd <= tol)) + 1
        assert first_abs != first


def test_initial_err_e_is_the_energy(cfg1):
    p, op, G, w = cfg1
    E0 = O.energy(op, p.U0)
    r = O.run_algorithm1_adaptive(op, p.U0, G, 40.0, 40.0, 40.0, 50, energy_tol=1.01 * abs(E0))
    assert r["steps"] == 0
    r = O.run_algorithm1_adaptive(op, p.U0, G, 40.0, 40.0, 40.0, 50, energy_tol=0.99 * abs(E0))
    assert r["steps"] >= 1


def test_energy_stop_counts_follow_the_rate_model(cfg1):
    p, op, G, w = cfg1
    N = 8
    tau = 40.0
    rho = 1.0 - tau * (1.0 / w[N - 1] - 1.0 / w[N])
    n1 = O.run_algorithm1(op, p.U0, tau, G, 2000, energy_tol=1e-7, record=False)["steps"]
    n2 = O.run_algorithm1(op, p.U0, tau, G, 2000, energy_tol=1e-11, record=False)["steps"]
    predicted = np.log(1e4) / (-2.0 * np.log(rho))
    assert abs((n2 - n1) - predicted) <= 0.12 * predicted, (n1, n2, predicted)


def test_adaptive_with_equal_bounds_is_algorithm1(cfg1):
    p, op, G, w = cfg1
    r1 = O.run_algorithm1(op, p.U0, 40.0, G, 30, record=False)
    r2 = O.run_algorithm1_adaptive(op, p.U0, G, 40.0, 40.0, 40.0, 30)
    assert r2["steps"] == 30 and r2["rejected"] == 0
    assert np.array_equal(r1["U"], r2["U"])
    assert r2["hist"]["tau"] == [40.0] * 30


def test_adaptive_recovers_from_an_unstable_start(cfg1):
    p, op, G, w = cfg1
    N = 8
    tcrit = 2.0 / (1.0 / w[0] - 1.0 / w[-1])
    Egs = 0.5 * w[:N].sum()
    tol = 1e-10
    r = O.run_algorithm1_adaptive(op, p.U0, G, 4.0 * tcrit, 1.0, 4.0 * tcrit, 4000, energy_tol=tol, energy_ref=Egs)
    h = r["hist"]
    assert r["rejected"] > 0
    assert all(1.0 <= t <= 4.0 * tcrit for t in h["tau"])
    E = np.array(h["E"])
    assert np.all(np.diff(E) <= 1e-13 * np.abs(E[:-1]))
    errs = (E - Egs) / Egs
    assert errs[-1] <= tol and errs[-2] > tol
    assert r["steps"] < 4000
    ritz = O.ritz_values(op, r["U"])
    assert np.max(np.abs(ritz - w[:N]) / w[:N]) <= 1e-8
    assert O.ortho_error(r["U"]) <= 1e-12
