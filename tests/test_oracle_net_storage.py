"""Pins of the oracle's optimiser and of its storage-precision network pass.

* ``adam_step`` (Kingma & Ba 2015, Algorithm 1): the first step is
  ``-lr g / (|g| + eps)`` (bias correction makes ``m_hat = g``,
  ``v_hat = g^2``), a constant gradient keeps that step at every count, and
  two steps with gradients 1 and -2 match the moments worked out with exact
  fractions; swapping the two moment updates is caught.
* ``bf16``: bit patterns of representable, halfway (ties to even) and
  just-above-halfway values.
* ``storage_forward``: with integer inputs and sparse +-1 weights every sum
  and every rounding is exact, so it must equal the float64 ``forward`` and
  its bounds vanish away from zero activations; with random weights a float32 re-evaluation (different
  accumulation order and precision, same rounding points) stays inside its
  bounds.
* ``storage_grad``: the float32 re-evaluation of the backward pass (loss
  derivative in float32, bf16 storage of g4..g1, float32 sums) stays within
  2^-5 of the absolute contractions of every weight (four bf16 roundings of
  2^-8 each along the longest path, doubled), and the float64 values equal
  ``backward`` when nothing rounds.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import net as NN


# ---------------------------------------------------------------------------
# Adam
# ---------------------------------------------------------------------------

def test_adam_first_step_is_lr_sign():
    rng = np.random.default_rng(1)
    w = rng.standard_normal(50)
    g = rng.standard_normal(50)
    w1, m1, v1 = NN.adam_step(w, np.zeros(50), np.zeros(50), g, 1, 0.01)
    assert np.max(np.abs(w1 - (w - 0.01 * g / (np.abs(g) + 1e-8)))) <= 1e-15
    assert np.all(np.abs((w - w1) - 0.01 * np.sign(g)) <= 0.01 * 2e-8 / np.abs(g))


def test_adam_constant_gradient_keeps_the_step():
    g = np.array([3.0, -0.5, 1e-3])
    w, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 8):
        w_new, m, v = NN.adam_step(w, m, v, g, t, 0.1)
        assert np.max(np.abs((w - w_new) - 0.1 * g / (np.abs(g) + 1e-8))) <= 1e-12
        w = w_new


def _adam_two_steps_by_hand(lr):
    # g1 = 1, g2 = -2, beta1 = 9/10, beta2 = 999/1000, from zero moments
    b1, b2 = Fraction(9, 10), Fraction(999, 1000)
    m = (1 - b1) * 1
    v = (1 - b2) * 1
    m = b1 * m + (1 - b1) * (-2)
    v = b2 * v + (1 - b2) * 4
    m_hat = m / (1 - b1 ** 2)        # -0.11 / 0.19
    v_hat = v / (1 - b2 ** 2)        # 0.004999 / 0.001999
    return float(m_hat), float(v_hat)


def test_adam_two_steps_match_exact_fractions():
    lr = 0.05
    w0 = np.array([0.7])
    w1, m, v = NN.adam_step(w0, np.zeros(1), np.zeros(1), np.array([1.0]), 1, lr)
    w2, m, v = NN.adam_step(w1, m, v, np.array([-2.0]), 2, lr)
    m_hat, v_hat = _adam_two_steps_by_hand(lr)
    step2 = lr * m_hat / (np.sqrt(v_hat) + 1e-8)
    assert abs(w1[0] - (0.7 - lr / (1.0 + 1e-8))) <= 1e-15
    assert abs(w2[0] - (w1[0] - step2)) <= 1e-15
    assert m_hat == pytest.approx(-0.11 / 0.19, rel=1e-14)


def test_planted_moment_swap_is_caught():
    def swapped(w, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        m = beta2 * m + (1 - beta2) * g
        v = beta1 * v + (1 - beta1) * g * g
        return w - lr * (m / (1 - beta2 ** t)) / (np.sqrt(v / (1 - beta1 ** t)) + eps), m, v
    lr = 0.05
    w1, m, v = swapped(np.array([0.7]), np.zeros(1), np.zeros(1), np.array([1.0]), 1, lr)
    w2, m, v = swapped(w1, m, v, np.array([-2.0]), 2, lr)
    m_hat, v_hat = _adam_two_steps_by_hand(lr)
    assert abs(w2[0] - (w1[0] - lr * m_hat / (np.sqrt(v_hat) + 1e-8))) > 1e-3


# ---------------------------------------------------------------------------
# bf16 rounding
# ---------------------------------------------------------------------------

def test_bf16_rounding_bit_patterns():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20,
                     -(1.0 + 2.0 ** -8 + 2.0 ** -20), 3.0, 2.0 ** -130, 0.0])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -(1.0 + 2.0 ** -7), 3.0, 2.0 ** -130, 0.0])
    assert np.array_equal(NN.bf16(vals), want)
    # 2^-130 is a float32 subnormal with a single bit: representable in bf16
    r = np.random.default_rng(0).standard_normal(1000)
    b = NN.bf16(r)
    assert np.all(np.abs(b - r) <= 2.0 ** -8 * np.abs(r))
    bits = b.astype(np.float32).view(np.uint32)
    assert np.all((bits & 0xFFFF) == 0)


# ---------------------------------------------------------------------------
# storage-precision pass and its bounds
# ---------------------------------------------------------------------------

def _sparse_int_weights(rng, nnz=3):
    Ws = []
    for ci, co in zip(NN.CHANNELS[:-1], NN.CHANNELS[1:]):
        W = np.zeros((27, ci, co))
        for c in range(co):
            for _ in range(nnz):
                W[rng.integers(27), rng.integers(ci), c] = rng.choice([-1.0, 1.0])
        Ws.append(W)
    return Ws


def test_storage_forward_exact_for_integer_data():
    rng = np.random.default_rng(5)
    m = (7, 6, 5)
    x = np.zeros((m[2], m[1], m[0], 2))
    x[..., 0] = rng.integers(-3, 4, size=x.shape[:3])
    x[..., 1] = rng.integers(0, 4, size=x.shape[:3])
    Ws = _sparse_int_weights(rng)
    s = NN.storage_forward(x, Ws)
    ref = NN.forward(x, Ws)
    assert np.array_equal(s["f"], ref["f"])
    assert np.max(np.abs(ref["f"])) > 0
    # intervals round to single values except around zero, where they stay tiny
    for k in ("e_a1", "e_a2", "e_a3"):
        assert np.max(s[k]) <= 1e-3
        assert np.all(s[k][np.abs(s[k[2:]]) >= 1.0] == 0.0)


def _f32_conv(a, W):
    out = np.zeros(a.shape[:3] + (W.shape[2],), dtype=np.float32)
    a32 = a.astype(np.float32)
    W32 = W.astype(np.float32)
    for t in reversed(range(27)):        # another order than the oracle's
        out = (out + NN.shift(a32, NN.TAPS[t]) @ W32[t]).astype(np.float32)
    return out.astype(np.float64)


def _f32_conv_t(g, W):
    out = np.zeros(g.shape[:3] + (W.shape[1],), dtype=np.float32)
    g32 = g.astype(np.float32)
    W32 = W.astype(np.float32)
    for t in reversed(range(27)):
        out = (out + NN.shift(g32, tuple(-d for d in NN.TAPS[t])) @ W32[t].T).astype(np.float32)
    return out.astype(np.float64)


def _f32_forward(x, Ws):
    xb = NN.bf16(x)
    Wb = [NN.bf16(W) for W in Ws]
    a1 = NN.bf16(np.maximum(_f32_conv(xb, Wb[0]), 0.0))
    a2 = NN.bf16(np.maximum(_f32_conv(a1, Wb[1]), 0.0))
    a3 = NN.bf16(np.maximum(_f32_conv(a2, Wb[2]), 0.0))
    return {"xb": xb, "Wb": Wb, "a1": a1, "a2": a2, "a3": a3, "f": _f32_conv(a3, Wb[3])[..., 0]}


def _random_case(seed, m=(9, 8, 7)):
    rng = np.random.default_rng(seed)
    x = np.zeros((m[2], m[1], m[0], 2))
    r = rng.standard_normal(x.shape[:3])
    x[..., 0] = (r / np.linalg.norm(r)).astype(np.float32)
    x[..., 1] = rng.uniform(-0.02, 0.05, size=x.shape[:3]).astype(np.float32)
    Ws = NN.init_weights(seed)
    t = rng.standard_normal(x.shape[:3]).astype(np.float32) * 0.1
    return x, Ws, t


@pytest.mark.parametrize("seed", [0, 1])
def test_storage_forward_bounds_contain_float32_evaluation(seed):
    x, Ws, _ = _random_case(seed)
    s = NN.storage_forward(x, Ws)
    g = _f32_forward(x, Ws)
    assert np.all(np.abs(g["f"] - s["f"]) <= s["e_f"])
    for k in ("a1", "a2", "a3"):
        assert np.all(np.abs(g[k] - s[k]) <= s["e_" + k])
    # the bound is a small fraction of the magnitude of the sums it covers
    mag = NN.conv(np.abs(s["a3"]), np.abs(s["Wb"][3]))[..., 0]
    assert np.max(s["e_f"] / np.maximum(mag, 1e-30)) < 0.1


def _f32_stencil(e, v2, kin):
    e = e.astype(np.float32)
    nb = np.zeros_like(e)
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(1, None)
        hi[ax] = slice(None, -1)
        nb[tuple(lo)] = (nb[tuple(lo)] + e[tuple(hi)]).astype(np.float32)
        nb[tuple(hi)] = (nb[tuple(hi)] + e[tuple(lo)]).astype(np.float32)
    return (np.float32(kin) * (np.float32(6) * e - nb) + v2.astype(np.float32) * e).astype(np.float32)


@pytest.mark.parametrize("kind", ["energy", "residual", "both"])
def test_storage_grad_bounds_contain_float32_evaluation(kind):
    x, Ws, t = _random_case(3)
    v2 = x[..., 1]
    kin = 1.0
    coef, coef_r = 0.7, 0.3
    grads, mags, fw = NN.storage_grad(x, t, v2, Ws, kin, coef, kind=kind, coef_r=coef_r)
    g32 = _f32_forward(x, Ws)
    f = g32["f"].astype(np.float32)
    gsum = np.zeros(f.shape, dtype=np.float64)
    if kind in ("energy", "both"):
        gsum += coef * _f32_stencil((f - t.astype(np.float32)).astype(np.float32), v2, kin).astype(np.float64)
    if kind in ("residual", "both"):
        E = (_f32_stencil(f, v2, kin) - x[..., 0].astype(np.float32)).astype(np.float32)
        gsum += coef_r * _f32_stencil(E, v2, kin).astype(np.float64)
    g4 = NN.bf16(gsum)[..., None]
    Wb = g32["Wb"]
    ref = [None] * 4

    def f32_wgrad(a, g):
        dW = np.zeros((27, a.shape[3], g.shape[3]), dtype=np.float32)
        gf = g.reshape(-1, g.shape[3]).astype(np.float32)
        for tt, tap in enumerate(NN.TAPS):
            dW[tt] = NN.shift(a.astype(np.float32), tap).reshape(-1, a.shape[3]).T @ gf
        return dW.astype(np.float64)

    ref[3] = f32_wgrad(g32["a3"], g4)
    g3 = NN.bf16(_f32_conv_t(g4, Wb[3]) * (g32["a3"] > 0))
    ref[2] = f32_wgrad(g32["a2"], g3)
    g2 = NN.bf16(_f32_conv_t(g3, Wb[2]) * (g32["a2"] > 0))
    ref[1] = f32_wgrad(g32["a1"], g2)
    g1 = NN.bf16(_f32_conv_t(g2, Wb[1]) * (g32["a1"] > 0))
    ref[0] = f32_wgrad(g32["xb"], g1)
    for L in range(4):
        assert np.all(np.abs(ref[L] - grads[L]) <= 2.0 ** -5 * mags[L]), L


def test_storage_grad_equals_backward_without_rounding():
    """With integer data, sparse +-1 weights and a loss derivative that is an
    integer field, no rounding happens and the values are ``backward``'s."""
    rng = np.random.default_rng(9)
    m = (6, 5, 4)
    x = np.zeros((m[2], m[1], m[0], 2))
    x[..., 0] = rng.integers(-2, 3, size=x.shape[:3])
    x[..., 1] = rng.integers(0, 2, size=x.shape[:3])
    Ws = _sparse_int_weights(rng, nnz=2)
    v2 = np.zeros(x.shape[:3])
    t = np.zeros(x.shape[:3])
    grads, mags, fw = NN.storage_grad(x, t, v2, Ws, 1.0, 1.0, kind="energy")
    cache = NN.forward(x, Ws)
    df = NN._stencil(cache["f"], v2, 1.0)
    ref = NN.backward(cache, df, Ws)
    for L in range(4):
        assert np.array_equal(grads[L], ref[L])
