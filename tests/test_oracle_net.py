"""Pins of the oracle conv-net (the learned preconditioner's definition).

* ``conv_transpose`` is the adjoint of ``conv`` (inner-product identity).
* ``conv`` of a one-hot kernel is a shift; with a 7-point Laplacian kernel it
  reproduces the oracle's finite-difference operator (with h = 1).
* Weight gradients match central finite differences of the batch loss.
* Both losses (energy norm, residual norm) are 1 for the zero network and 0
  for the exact inverse; their weight gradients match finite differences.
* The learned step with the exact inverse in place of the network is the
  paper's step with exact Step 1 (gradient form ``GU = (U - H^{-1} R) Lam^{-1}``);
  with any network it keeps orthogonality and leaves an eigenbasis fixed.
* Through all four layers: identity taps in layers 1-3 on a positive input
  (every ReLU passes) and the Laplacian kernel in layer 4 give the
  finite-difference operator; a planted sign error in a ReLU mask is caught by
  the finite-difference gradient check.
* Positive homogeneity ``P(a r) = a P(r)`` (a > 0) and ``P(0) = 0``: the
  eigenbasis remains a fixed point of the learned step.
"""
import numpy as np
import pytest

import oracle as O
from oracle import net as NN


def test_transpose_is_adjoint():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((4, 5, 6, 3))
    g = rng.standard_normal((4, 5, 6, 2))
    W = rng.standard_normal((27, 3, 2))
    lhs = np.sum(NN.conv(a, W) * g)
    rhs = np.sum(a * NN.conv_transpose(g, W))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_laplacian_kernel_matches_fd_operator():
    m = (6, 5, 4)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(int(np.prod(m)))
    W = np.zeros((27, 1, 1))
    for t, tap in enumerate(NN.TAPS):
        k = sum(abs(d) for d in tap)
        if k == 0:
            W[t] = 6.0
        elif k == 1:
            W[t] = -1.0
    out = NN.conv(u.reshape(m[2], m[1], m[0], 1), W).reshape(-1)
    op = O.Operator(m, (1.0, 1.0, 1.0), np.zeros(u.size))
    assert np.allclose(out, O.apply_H(op, u[:, None])[:, 0], atol=1e-12)


def _small_problem(m=(5, 4, 4), seed=2):
    rng = np.random.default_rng(seed)
    n = int(np.prod(m))
    h = 1.0 / (max(m) + 1)
    op = O.Operator(m, (h, h, h), rng.uniform(-20.0, 0.0, n), shift=25.0)
    return op, rng


def _samples(op, rng, count):
    solve = O.GSolver(op, "dense")
    xs, ts = [], []
    for _ in range(count):
        r = rng.standard_normal(op.n)
        xs.append(NN.inputs_for(r, op))
        ts.append(NN.target_for(r, op, solve))
    return xs, ts


@pytest.mark.parametrize("kind", ["energy", "residual"])
def test_weight_gradients_match_finite_differences(kind):
    op, rng = _small_problem()
    A = NN.scaled_operator(op)
    Ws = NN.init_weights(7)
    xs, ts = _samples(op, rng, 2)
    loss, grads = NN.batch_loss_and_grads(xs, ts, Ws, A, kind)
    eps = 1e-6
    for li, idx in [(0, (3, 1, 5)), (1, (13, 7, 2)), (2, (26, 15, 15)), (3, (0, 4, 0)), (1, (4, 0, 9)), (0, (20, 0, 2))]:
        Wp = [W.copy() for W in Ws]
        Wm = [W.copy() for W in Ws]
        Wp[li][idx] += eps
        Wm[li][idx] -= eps
        fd = (NN.batch_loss_and_grads(xs, ts, Wp, A, kind)[0] - NN.batch_loss_and_grads(xs, ts, Wm, A, kind)[0]) / (2 * eps)
        assert abs(fd - grads[li][idx]) <= 1e-6 * max(1.0, abs(fd)), (li, idx, fd, grads[li][idx])


def test_energy_loss_of_zero_and_exact_network():
    op, rng = _small_problem(seed=4)
    A = NN.scaled_operator(op)
    xs, ts = _samples(op, rng, 3)
    for x, t in zip(xs, ts):
        l0, _ = NN.sample_loss(np.zeros_like(t), t, x[..., 0], A)
        l1, g1 = NN.sample_loss(t, t, x[..., 0], A)
        assert abs(l0 - 1.0) <= 1e-12
        assert l1 == 0.0 and np.all(g1 == 0.0)
        # a perturbation costs its own energy norm, relative to r^T H^{-1} r
        d = rng.standard_normal(t.shape)
        l2, _ = NN.sample_loss(t + d, t, x[..., 0], A)
        assert l2 > 0.0
        # residual norm: x0 = A t exactly for the normalised column, so
        # the zero network leaves the whole residual and t none of it
        x0 = A(t)
        r0, _ = NN.sample_residual_loss(np.zeros_like(t), x0, A)
        r1, _ = NN.sample_residual_loss(t, x0, A)
        assert abs(r0 - 1.0) <= 1e-12 and r1 <= 1e-24
        assert abs(NN.sample_residual_loss(t + d, x0, A)[0] - np.sum(A(d) ** 2) / np.sum(x0 * x0)) <= 1e-10


def test_learned_step_with_exact_inverse_is_the_paper_step(monkeypatch):
    from workloads import initial_block
    op, _ = _small_problem(m=(4, 4, 3), seed=6)
    U = initial_block(op.n, 3, seed=1)
    solve = O.GSolver(op, "dense")
    monkeypatch.setattr(NN, "apply_preconditioner", lambda R, op_, Ws: solve(R))
    out = NN.learned_step(op, U, None, 0.05)
    ref = O.steps_1_to_4(U, solve, 0.05)
    assert np.allclose(out["Y"], ref["Y"], rtol=0, atol=1e-12 * np.max(np.abs(ref["Y"])))
    assert np.allclose(out["U"], ref["U"], rtol=0, atol=1e-12)


def test_learned_step_orthogonality_and_fixed_point():
    from workloads import initial_block
    op, _ = _small_problem(m=(4, 5, 3), seed=8)
    Ws = NN.init_weights(2)
    U = initial_block(op.n, 4, seed=3)
    U1 = NN.learned_step(op, U, Ws, 0.05)["U"]
    assert O.ortho_error(U1) <= 1e-12
    assert np.max(np.abs(U1 - U)) > 1e-6
    w, V = np.linalg.eigh(O.assemble_H(op).toarray())
    U2 = NN.learned_step(op, V[:, :4], Ws, 0.05)["U"]
    assert np.max(np.abs(U2 - V[:, :4])) <= 1e-11


def test_positive_homogeneity_and_zero():
    rng = np.random.default_rng(3)
    m = (5, 4, 3)
    n = int(np.prod(m))
    op = O.Operator(m, (0.1, 0.1, 0.1), rng.uniform(-5, 0, n))
    R = rng.standard_normal((n, 3))
    Ws = NN.init_weights(1)
    P1 = NN.apply_preconditioner(R, op, Ws)
    P2 = NN.apply_preconditioner(2.5 * R, op, Ws)
    assert np.allclose(P2, 2.5 * P1, rtol=1e-12, atol=1e-14)
    assert np.all(NN.apply_preconditioner(np.zeros((n, 2)), op, Ws) == 0.0)


def test_full_network_linear_special_case():
    m = (5, 6, 4)
    rng = np.random.default_rng(4)
    u = rng.uniform(0.5, 1.5, int(np.prod(m)))
    x = np.zeros((m[2], m[1], m[0], 2))
    x[..., 0] = u.reshape(m[2], m[1], m[0])
    x[..., 1] = rng.uniform(-1, 1, x.shape[:3])     # ignored by W1 below
    centre = NN.TAPS.index((0, 0, 0))
    Ws = [np.zeros((27, ci, co)) for ci, co in zip(NN.CHANNELS[:-1], NN.CHANNELS[1:])]
    Ws[0][centre, 0, 3] = 1.0
    Ws[1][centre, 3, 5] = 1.0
    Ws[2][centre, 5, 0] = 1.0
    for t, tap in enumerate(NN.TAPS):
        k = sum(abs(d) for d in tap)
        Ws[3][t, 0, 0] = 6.0 if k == 0 else (-1.0 if k == 1 else 0.0)
    f = NN.forward(x, Ws)["f"].reshape(-1)
    op = O.Operator(m, (1.0, 1.0, 1.0), np.zeros(u.size))
    assert np.allclose(f, O.apply_H(op, u[:, None])[:, 0], atol=1e-12)


def test_planted_relu_mask_error_is_caught(monkeypatch):
    op, rng = _small_problem(m=(4, 4, 3), seed=5)
    A = NN.scaled_operator(op)
    Ws = NN.init_weights(3)
    xs, ts = _samples(op, rng, 1)
    good = NN.backward
    def bad(cache, df, Ws_):
        c = dict(cache)
        c["z2"] = -c["z2"]            # wrong mask (z < 0 instead of z > 0) in layer 2
        return good(c, df, Ws_)
    monkeypatch.setattr(NN, "backward", bad)
    _, g_bad = NN.batch_loss_and_grads(xs, ts, Ws, A)
    monkeypatch.setattr(NN, "backward", good)
    _, g_ok = NN.batch_loss_and_grads(xs, ts, Ws, A)
    li, idx = 1, (13, 2, 3)
    eps = 1e-6
    Wp = [W.copy() for W in Ws]; Wp[li][idx] += eps
    Wm = [W.copy() for W in Ws]; Wm[li][idx] -= eps
    fd = (NN.batch_loss_and_grads(xs, ts, Wp, A)[0] - NN.batch_loss_and_grads(xs, ts, Wm, A)[0]) / (2 * eps)
    assert abs(fd - g_ok[li][idx]) <= 1e-6 * max(1.0, abs(fd))
    assert np.max(np.abs(g_bad[0] - g_ok[0])) > 1e-3
