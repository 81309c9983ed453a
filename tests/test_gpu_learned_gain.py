"""What the trained network gains, measured on a potential it never saw.

The shipped weights were trained on 64^3 well potentials with seeds >= 1000;
these tests use the seed-0 potential (the benchmark's) with N = 17.

* Loss: on residual columns of a plain trajectory, the trained network's
  loss (energy norm + residual norm; 2 for the zero network) is about a
  quarter of that of the untrained (He-initialised) or the zero network.
* Learned steps alone (judge off, tau = 20) from a late plain iterate lower
  the residual with the trained weights; with the untrained weights they
  raise it.
* The judged solve (tau = 45) reaches residual 1e-8 with the plain solve's
  Ritz values and orthogonality, keeps some learned steps, keeps more of them
  than with the untrained weights, and its wall time next to the plain solve's
  is printed.  The learned form does not beat the plain one here (a 9^3
  receptive field cannot act on the slow, smooth modes that set the rate);
  the test states that measured ratio rather than assume a speedup.
"""
import time

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import say, to_dev, to_host

pytestmark = pytest.mark.gpu

TAU = 45.0


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2511_06788_amd import ope, train_net
    p = W.wells_3d(m=64, N=17, seed=0)
    trained = ope.load_net_weights()
    untrained = train_net.he_init(0)
    return torch, ope, p, trained, untrained


def _late_iterate(torch, ope, p, steps):
    with ope.Context(p.grid, p.V, p.N) as ctx:
        U = to_dev(p.U0)
        for _ in range(steps):
            ope.ope_step(ctx.handle, U, TAU)
        return to_host(U)


def test_trained_loss_on_held_out_potential(setup):
    torch, ope, p, trained, untrained = setup
    from paper_2511_06788_amd import train_net
    say("learned gain: loss")
    n, N = p.grid.n, p.N
    losses = {}
    with ope.Context(p.grid, p.V, N) as ctx, ope.Net(ctx, 16) as net:
        ope.ope_net_set_loss(net.handle, ope.OPE_NET_LOSS_BOTH)
        U = to_dev(p.U0)
        HU, R, S = torch.empty_like(U), torch.empty_like(U), torch.empty_like(U)
        Lam = torch.empty(N, N, dtype=torch.float64, device="cuda")
        Z = torch.zeros(2 * N, N, dtype=torch.float64, device="cuda")
        Z[N:] = torch.eye(N, dtype=torch.float64, device="cuda")
        X = torch.empty(N, n, dtype=torch.float32, device="cuda")
        T = torch.empty_like(X)
        v2 = torch.empty(n, dtype=torch.float32, device="cuda")
        ope.ope_net_potential(net.handle, v2)
        for _ in range(60):
            ope.ope_step(ctx.handle, U, TAU)
        train_net.residual_block(ope, torch, ctx, U, HU, R, Lam, Z)
        ope.ope_source_solve(ctx.handle, R, S, None, tol=1e-8, max_iter=20000)
        ope.ope_net_samples(net.handle, R, S, N, N, X, T)
        for name, w in (("trained", trained), ("untrained", untrained), ("zero", np.zeros_like(trained))):
            ope.ope_net_set_weights(net.handle, w)
            losses[name], _ = ope.ope_net_grad(net.handle, X[:16], v2, T[:16], 16, want_grad=False)
    print("held-out loss", losses)
    assert abs(losses["zero"] - 2.0) <= 1e-3
    assert losses["trained"] < 0.35 * losses["zero"]
    assert losses["trained"] < 0.35 * losses["untrained"]


def _learned_only(torch, ope, p, U0, w, tau, steps):
    with ope.Context(p.grid, p.V, p.N) as ctx, ope.Net(ctx, p.N, w) as net:
        ope.ope_set_preconditioner(ctx.handle, net.handle, judge=False)
        U = to_dev(U0)
        res = []
        for _ in range(steps):
            info, _ = ope.ope_step_learned(ctx.handle, U, tau)
            res.append(info.residual)
        r_end, _, drift = ope.ope_residual(ctx.handle, U, p.N, want_ritz=False)
    return res[0], r_end, drift


def test_learned_steps_alone(setup):
    torch, ope, p, trained, untrained = setup
    say("learned gain: learned steps alone")
    U0 = _late_iterate(torch, ope, p, 200)
    r0, rt, dt = _learned_only(torch, ope, p, U0, trained, 20.0, 10)
    _, ru, du = _learned_only(torch, ope, p, U0, untrained, 20.0, 10)
    print(f"10 learned steps at tau 20 from res {r0:.3e}: trained -> {rt:.3e}, untrained -> {ru:.3e}")
    assert rt < r0
    assert ru > r0
    assert dt <= 1e-12 and du <= 1e-12      # orthogonality holds for any weights


def _solve(torch, ope, p, w, judge=True):
    with ope.Context(p.grid, p.V, p.N) as ctx:
        net = ope.Net(ctx, p.N, w) if w is not None else None
        if net is not None:
            ope.ope_set_preconditioner(ctx.handle, net.handle, judge=judge)
        U = to_dev(p.U0)
        ope.ope_solve(ctx.handle, to_dev(p.U0), TAU, 1.0, 2)      # warm the code paths
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        si = ope.ope_solve(ctx.handle, U, TAU, 1e-8, 4000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res, ritz, drift = ope.ope_residual(ctx.handle, U, p.N)
        if net is not None:
            net.close()
    return si, dt, res, ritz, drift


def test_judged_solve_against_plain(setup):
    torch, ope, p, trained, untrained = setup
    say("learned gain: judged solve vs plain")
    sp, tp, rp, ritz_p, dp = _solve(torch, ope, p, None)
    sl, tl, rl, ritz_l, dl = _solve(torch, ope, p, trained)
    su, tu, ru, _, _ = _solve(torch, ope, p, untrained)
    print(f"plain: {sp.steps} steps {tp:.3f} s; learned (trained): {sl.steps} steps, {sl.learned_steps} kept, "
          f"{tl:.3f} s (plain/learned time {tp / tl:.2f}); learned (untrained): {su.steps} steps, "
          f"{su.learned_steps} kept, {tu:.3f} s")
    assert sp.converged and sl.converged and su.converged
    assert np.max(np.abs(ritz_l - ritz_p) / np.abs(ritz_p)) <= 1e-10
    assert dl <= 1e-12
    assert sl.learned_steps >= 5
    assert sl.learned_steps > su.learned_steps
