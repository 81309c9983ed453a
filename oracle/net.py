"""Oracle: the small 3D conv-net preconditioner (test infrastructure only).

The learned form replaces ``H^{-1} R`` in the gradient form of the step
(``GU = (U - H^{-1} R) Lam^{-1}``, ``R = HU - U Lam``) by a network applied to
each column of R.  The network here is the plain definition, in float64, of:

    input channels  x_0 = r / |r|,  x_1 = h^2 (V + shift)  (on the grid, zero outside)
    z_1 = W_1 * x,        a_1 = relu(z_1)      2 -> 16 channels
    z_2 = W_2 * a_1,      a_2 = relu(z_2)     16 -> 16
    z_3 = W_3 * a_2,      a_3 = relu(z_3)     16 -> 16
    f   = W_4 * a_3                           16 -> 1
    P(r) = |r| h^2 f

where ``W * a`` is a 3x3x3 cross-correlation with zero padding outside the
grid, ``out[v, co] = sum_{tap, ci} W[tap, ci, co] a[v + tap, ci]``, no biases
(so ``P(0) = 0`` and eigenbases stay fixed points).  The training loss of a
sample is the squared energy-norm error of the preconditioned direction
relative to the exact one,

    (P r - H^{-1} r)^T H (P r - H^{-1} r) / (r^T H^{-1} r)
        = (f - t)^T A (f - t) / (x_0 . t),   t = H^{-1} r / (|r| h^2),  A = h^2 H,

(1 for the zero network, 0 for the exact inverse), averaged over the batch.
The second loss is the residual norm of the preconditioned direction,

    |H P r - r|^2 / |r|^2 = |A f - x_0|^2 / |x_0|^2,

also 1 for the zero network and 0 for the exact inverse; it weights errors at
high frequencies by H^2 instead of H and needs no target.  The grid spacing
must be the same on all three axes.

Layout: a field of C channels on the grid is an array of shape
``(m2, m1, m0, C)`` (x fastest); taps are ordered ``(dz, dy, dx)`` with dx
fastest, each in ``(-1, 0, 1)``.

Two further pieces serve the element-wise comparison with the device kernels:

* ``bf16``, ``storage_forward`` and ``storage_grad`` -- the same network and
  losses evaluated with the storage precision of the device kernels made
  explicit: inputs, weights, the activations after every ReLU, and the
  back-propagated fields rounded to bfloat16 (round to nearest even, via
  float32), everything else in float64.  The forward pass carries beside
  every value an element-wise bound on the distance of a float32-accumulating
  implementation with the same rounding points, by interval arithmetic: a sum
  of K products is off by at most ``K u / (1 - K u)`` times the sum of absolute
  products (u = 2^-24, the float32 unit roundoff); a rounding to bfloat16 is
  monotone, so an input interval ``[z - e, z + e]`` maps to
  ``[bf16(z - e), bf16(z + e)]`` and the bound after it is the width of that
  image (zero whenever the whole interval rounds to one value).  The backward
  pass returns the absolute-value contractions that scale its rounding
  errors; with integer data and sparse +-1 weights every quantity is an
  integer of at most 8 significant bits and the pass is exact.
* ``adam_step`` -- Adam (Kingma & Ba, 2015, Algorithm 1): bias-corrected
  first and second moment estimates and the step ``lr m_hat / (sqrt(v_hat) + eps)``.

Parity: the backward pass is pinned by central finite differences of the loss,
the forward pass by the special case where every ReLU passes and the network
reduces to an explicit stencil, and the loss by its values for the zero and
the exact network; ``bf16`` by the bit patterns of exactly representable and
halfway values; ``storage_forward`` by integer-valued cases where every rounding
is exact (it must then equal ``forward`` with zero bounds), and both
``storage_forward`` by a float32 re-evaluation with the same rounding points
(a different accumulation order and precision) that must stay inside its
bounds, ``storage_grad`` by ``backward`` on exact integer cases and by that
float32 re-evaluation staying within 2^-5 of the absolute contractions; ``adam_step`` by hand-checked
steps (the first step is ``-lr sign(g)`` up to eps, a constant gradient keeps
that step size, two steps with different gradients match values worked out by
hand) and by a planted swap of the moments.
"""
from __future__ import annotations

from typing import Callable, Dict, List, Sequence

import numpy as np

from .operator import Operator, apply_H
from .scheme import step_general

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
CHANNELS = (2, 16, 16, 16, 1)


def shift(a: np.ndarray, tap) -> np.ndarray:
    """``out[v] = a[v + tap]`` with zeros outside the grid (array axes z, y, x, c)."""
    out = np.zeros_like(a)
    src = []
    dst = []
    for ax, d in enumerate(tap):
        n = a.shape[ax]
        if d == 0:
            src.append(slice(0, n))
            dst.append(slice(0, n))
        elif d > 0:
            src.append(slice(d, n))
            dst.append(slice(0, n - d))
        else:
            src.append(slice(0, n + d))
            dst.append(slice(-d, n))
    out[tuple(dst)] = a[tuple(src)]
    return out


def conv(a: np.ndarray, W: np.ndarray) -> np.ndarray:
    """3x3x3 cross-correlation ``out[v, co] = sum_{t, ci} W[t, ci, co] a[v + tap_t, ci]``."""
    out = np.zeros(a.shape[:3] + (W.shape[2],))
    for t, tap in enumerate(TAPS):
        out += shift(a, tap) @ W[t]
    return out


def conv_transpose(g: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of ``conv`` in its input: ``out[v, ci] = sum_{t, co} W[t, ci, co] g[v - tap_t, co]``."""
    out = np.zeros(g.shape[:3] + (W.shape[1],))
    for t, tap in enumerate(TAPS):
        out += shift(g, tuple(-d for d in tap)) @ W[t].T
    return out


def conv_weight_grad(a: np.ndarray, g: np.ndarray) -> np.ndarray:
    """``dW[t, ci, co] = sum_v a[v + tap_t, ci] g[v, co]``."""
    ci, co = a.shape[3], g.shape[3]
    dW = np.zeros((27, ci, co))
    af = a.reshape(-1, ci)
    gf = g.reshape(-1, co)
    for t, tap in enumerate(TAPS):
        dW[t] = shift(a, tap).reshape(-1, ci).T @ gf
    return dW


def init_weights(seed: int) -> List[np.ndarray]:
    """He-style normal initialisation of the four weight tensors ``(27, ci, co)``."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0xC0117]))
    Ws = []
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        Ws.append(rng.standard_normal((27, ci, co)) * np.sqrt(2.0 / (27 * ci)))
    return Ws


def forward(x: np.ndarray, Ws: Sequence[np.ndarray]) -> Dict[str, np.ndarray]:
    """Network on one sample; ``x`` has shape (m2, m1, m0, 2).  Returns the
    pre-activations z1..z3 and the output f (m2, m1, m0)."""
    z1 = conv(x, Ws[0])
    z2 = conv(np.maximum(z1, 0.0), Ws[1])
    z3 = conv(np.maximum(z2, 0.0), Ws[2])
    f = conv(np.maximum(z3, 0.0), Ws[3])[..., 0]
    return {"x": x, "z1": z1, "z2": z2, "z3": z3, "f": f}


def backward(cache: Dict[str, np.ndarray], df: np.ndarray, Ws: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Weight gradients of a scalar with ``d/df = df`` (same shape as f)."""
    g4 = df[..., None]
    a3 = np.maximum(cache["z3"], 0.0)
    dW4 = conv_weight_grad(a3, g4)
    g3 = conv_transpose(g4, Ws[3]) * (cache["z3"] > 0)
    a2 = np.maximum(cache["z2"], 0.0)
    dW3 = conv_weight_grad(a2, g3)
    g2 = conv_transpose(g3, Ws[2]) * (cache["z2"] > 0)
    a1 = np.maximum(cache["z1"], 0.0)
    dW2 = conv_weight_grad(a1, g2)
    g1 = conv_transpose(g2, Ws[1]) * (cache["z1"] > 0)
    dW1 = conv_weight_grad(cache["x"], g1)
    return [dW1, dW2, dW3, dW4]


def scaled_operator(op: Operator) -> Callable[[np.ndarray], np.ndarray]:
    """``A = h^2 H`` acting on a field of shape (m2, m1, m0); equal spacings only."""
    h = op.h[0]
    if any(abs(hh - h) > 1e-12 * h for hh in op.h):
        raise ValueError("the network needs equal grid spacings")
    m = op.m
    shape = (m[2], m[1], m[0])
    return lambda e: h * h * apply_H(op, e.reshape(-1, 1))[:, 0].reshape(shape)


def sample_loss(f: np.ndarray, t: np.ndarray, x0: np.ndarray, apply_A) -> tuple:
    """Energy-norm loss of one sample and its derivative in f."""
    e = f - t
    Ae = apply_A(e)
    den = float(np.sum(x0 * t))
    return float(np.sum(e * Ae)) / den, 2.0 * Ae / den


def sample_residual_loss(f: np.ndarray, x0: np.ndarray, apply_A) -> tuple:
    """Residual-norm loss of one sample and its derivative in f (A is symmetric)."""
    e = apply_A(f) - x0
    xx = float(np.sum(x0 * x0))
    return float(np.sum(e * e)) / xx, 2.0 * apply_A(e) / xx


def batch_loss_and_grads(xs: Sequence[np.ndarray], ts, Ws: Sequence[np.ndarray], apply_A, kind: str = "energy"):
    """Batch-mean loss (``kind`` "energy" or "residual"; targets unused by the
    latter) and its weight gradients."""
    B = len(xs)
    loss = 0.0
    grads = [np.zeros_like(W) for W in Ws]
    for b, x in enumerate(xs):
        c = forward(x, Ws)
        if kind == "energy":
            l, df = sample_loss(c["f"], ts[b], x[..., 0], apply_A)
        elif kind == "residual":
            l, df = sample_residual_loss(c["f"], x[..., 0], apply_A)
        else:
            raise ValueError(kind)
        loss += l / B
        g = backward(c, df / B, Ws)
        for k in range(4):
            grads[k] += g[k]
    return loss, grads


def inputs_for(r_column: np.ndarray, op: Operator) -> np.ndarray:
    """Network input of one residual column (n values, x fastest)."""
    m = op.m
    h = op.h[0]
    shape = (m[2], m[1], m[0])
    x = np.zeros(shape + (2,))
    x[..., 0] = (r_column / np.linalg.norm(r_column)).reshape(shape)
    x[..., 1] = (h * h * (op.V + op.shift)).reshape(shape)
    return x


def target_for(r_column: np.ndarray, op: Operator, solve) -> np.ndarray:
    """``t = H^{-1} r / (|r| h^2)`` on the grid, with ``solve`` applying ``H^{-1}`` to a block."""
    m = op.m
    h = op.h[0]
    y = solve(r_column[:, None])[:, 0]
    return (y / (np.linalg.norm(r_column) * h * h)).reshape(m[2], m[1], m[0])


def apply_preconditioner(R: np.ndarray, op: Operator, Ws: Sequence[np.ndarray]) -> np.ndarray:
    """``P(R)`` column by column: ``|r| h^2 f(r / |r|, h^2 (V + shift))``; zero columns map to zero."""
    h = op.h[0]
    out = np.zeros_like(R)
    for j in range(R.shape[1]):
        nr = np.linalg.norm(R[:, j])
        if nr == 0.0:
            continue
        f = forward(inputs_for(R[:, j], op), Ws)["f"]
        out[:, j] = nr * h * h * f.reshape(-1)
    return out


def learned_step(op: Operator, U: np.ndarray, Ws: Sequence[np.ndarray], tau: float) -> Dict[str, np.ndarray]:
    """The learned form of one step: with ``Lam = U^T H U`` and ``R = HU - U Lam``,
    ``Y = (U - P(R)) Lam^{-1}`` (the gradient form ``GU = (U - H^{-1} R) Lam^{-1}``
    with the network in place of ``H^{-1}``), then Steps 2-4 for that Y."""
    HU = apply_H(op, U)
    Lam = U.T @ HU
    R = HU - U @ Lam
    Y = np.linalg.solve(Lam.T, (U - apply_preconditioner(R, op, Ws)).T).T
    out = step_general(U, Y, tau)
    out["Y"] = Y
    out["R"] = R
    return out


# ---------------------------------------------------------------------------
# optimiser
# ---------------------------------------------------------------------------

def adam_step(w: np.ndarray, m: np.ndarray, v: np.ndarray, g: np.ndarray, t: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) at step count ``t >= 1``:
    ``m = b1 m + (1 - b1) g``, ``v = b2 v + (1 - b2) g^2``,
    ``w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)``.
    Returns the new ``(w, m, v)``."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


# ---------------------------------------------------------------------------
# storage-precision evaluation with element-wise error bounds
# ---------------------------------------------------------------------------

U32 = 2.0 ** -24


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (float64 -> float32 round to nearest, then keep the
    top 16 bits of the float32 word with round to nearest even); returns float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _gamma(k: int) -> float:
    return k * U32 / (1.0 - k * U32)


def _conv_abs(a, W):
    return conv(np.abs(a), np.abs(W))


def _round_interval(z, e, relu: bool):
    """Image of ``[z - e, z + e]`` under (ReLU then) bf16 rounding: the rounded
    centre and the bound on the distance of any image point from it."""
    lo, hi = z - e, z + e
    if relu:
        z, lo, hi = np.maximum(z, 0.0), np.maximum(lo, 0.0), np.maximum(hi, 0.0)
    c, rl, rh = bf16(z), bf16(lo), bf16(hi)
    return c, np.maximum(np.abs(rh - c), np.abs(c - rl))


def _stencil_abs(e: np.ndarray, v2: np.ndarray, kin: float) -> np.ndarray:
    """``|A| e = kin (6 e + sum of neighbours of e) + |v2| e`` for e >= 0 (fields (m2, m1, m0))."""
    nb = np.zeros_like(e)
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(1, None)
        hi[ax] = slice(None, -1)
        nb[tuple(lo)] += e[tuple(hi)]
        nb[tuple(hi)] += e[tuple(lo)]
    return kin * (6.0 * e + nb) + np.abs(v2) * e


def _stencil(e: np.ndarray, v2: np.ndarray, kin: float) -> np.ndarray:
    nb = np.zeros_like(e)
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(1, None)
        hi[ax] = slice(None, -1)
        nb[tuple(lo)] += e[tuple(hi)]
        nb[tuple(hi)] += e[tuple(lo)]
    return kin * (6.0 * e - nb) + v2 * e


def storage_forward(x: np.ndarray, Ws: Sequence[np.ndarray]) -> Dict[str, np.ndarray]:
    """Forward pass with bf16 storage of the input pair, the weights and the
    activations a1..a3 (float32 accumulation assumed for the bounds).  ``x``
    (m2, m1, m0, 2) holds the float32 input values.  Returns the values
    (``xb``, ``Wb``, ``z*``, ``a*``, ``f``) and bounds ``e_a*``, ``e_z*``, ``e_f``."""
    xb = bf16(x)
    Wb = [bf16(W) for W in Ws]
    out = {"xb": xb, "Wb": Wb}
    a, ea = xb, np.zeros_like(xb)
    for L in range(3):
        K = 27 * Wb[L].shape[1]
        z = conv(a, Wb[L])
        ez = conv(ea, np.abs(Wb[L])) + (_gamma(K) + 1e-15) * _conv_abs(np.abs(a) + ea, Wb[L])
        a_new, ea_new = _round_interval(z, ez, relu=True)
        out[f"z{L + 1}"], out[f"e_z{L + 1}"] = z, ez
        out[f"a{L + 1}"], out[f"e_a{L + 1}"] = a_new, ea_new
        a, ea = a_new, ea_new
    K = 27 * 16
    f = conv(a, Wb[3])[..., 0]
    ef = (conv(ea, np.abs(Wb[3])) + (_gamma(K) + 1e-15) * _conv_abs(np.abs(a) + ea, Wb[3]))[..., 0]
    out["f"], out["e_f"] = f, ef
    return out


def storage_grad(x: np.ndarray, t: np.ndarray, v2: np.ndarray, Ws: Sequence[np.ndarray], kin: float,
                 coef: float, kind: str = "energy", coef_r: float = 0.0):
    """Weight gradients of one sample with bf16 storage of the forward
    activations and of the back-propagated fields g4..g1, as the device
    kernels store them.  ``coef`` multiplies ``A (f - t)`` (energy loss) and
    ``coef_r`` multiplies ``A (A f - x0)`` (residual loss): ``kind`` "energy",
    "residual" or "both".  ``v2`` (m2, m1, m0) is the float32 second input
    channel, ``t`` the float32 target.  Returns ``(grads, mags, fields)``:
    the float64 contractions of the stored fields, the contractions of their
    absolute values (the scale of every weight's rounding errors, one bf16
    rounding of a factor moving a term by at most 2^-8 of its size), and the
    fields (forward values; g4..g1 as stored and, as ``g*_raw``, before their
    rounding)."""
    fw = storage_forward(x, Ws)
    f = fw["f"]
    Wb = fw["Wb"]
    x0 = x[..., 0]
    g = np.zeros_like(f)
    if kind in ("energy", "both"):
        g = g + coef * _stencil(f - t, v2, kin)
    if kind in ("residual", "both"):
        g = g + coef_r * _stencil(_stencil(f, v2, kin) - x0, v2, kin)
    fields = dict(fw)
    fields["g4_raw"] = g[..., None]
    gcur = bf16(g)[..., None]
    fields["g4"] = gcur
    grads, mags = [None] * 4, [None] * 4
    grads[3] = conv_weight_grad(fw["a3"], gcur)
    mags[3] = conv_weight_grad(np.abs(fw["a3"]), np.abs(gcur))
    for L in (3, 2, 1):          # weights of layer L + 1 transposed: data gradient at a_L
        raw = conv_transpose(gcur, Wb[L]) * (fw[f"a{L}"] > 0)
        gcur = bf16(raw)
        fields[f"g{L}_raw"], fields[f"g{L}"] = raw, gcur
        prev = fw["xb"] if L == 1 else fw[f"a{L - 1}"]
        grads[L - 1] = conv_weight_grad(prev, gcur)
        mags[L - 1] = conv_weight_grad(np.abs(prev), np.abs(gcur))
    return grads, mags, fields
