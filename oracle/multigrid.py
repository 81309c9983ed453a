"""Oracle: a multigrid V-cycle as the preconditioner of Step 1's CG
(test infrastructure only).

Step 1 of the scheme (Section 4.1) solves the N source problems
``H y_j = u_j`` (``= (M U)_j`` in the generalized case); the paper does not fix
how.  The library's optional preconditioned CG uses one symmetric multigrid
V-cycle per iteration as its preconditioner; this module writes that V-cycle
out from its textbook ingredients, one level at a time, and the preconditioned
CG around it, so that the library's kernels can be checked against it.

Hierarchy (level 0 is the operator itself, ``W_0 = V + shift``):
  * level k+1 coarsens every axis with ``m_a > 1``: ``m_a' = ceil(m_a / 2)``,
    coarse node ``I`` is the parent of fine nodes ``2I`` and ``2I + 1`` (the
    latter only when it exists), ``h_a' = 2 h_a``;
  * ``W_{k+1}(I)`` is the mean of ``W_k`` over the existing children of ``I``;
  * ``H_k = kinetic (-Lap_{h_k}) + diag(W_k)`` (the same finite-difference
    form as the fine operator, on the coarse grid);
  * coarsening stops at the first level k >= 1 with at most ``COARSEST_MAX``
    nodes (level 0 is always coarsened once, unless every axis has a single
    node), whose operator is inverted exactly (Cholesky).

Transfers, per coarsened axis (a tensor product over the axes):
  * prolongation P: fine node ``f`` with parent ``I = f // 2`` takes
    ``3/4 e_I + 1/4 e_J`` with ``J = I - 1`` for even ``f`` and ``I + 1`` for
    odd ``f`` (a missing ``J`` contributes zero) -- linear interpolation
    between node-centred cells;
  * restriction ``R = P^T / 2^d`` (``d`` coarsened axes): coarse ``I`` takes
    ``(3/4 (x_{2I} + x_{2I+1}) + 1/4 (x_{2I-1} + x_{2I+2})) / 2`` per axis,
    missing fine nodes omitted.

V-cycle ``z = B_k b`` (damped Jacobi with ``omega = 0.8``, one sweep before
and one after the coarse correction, so ``B_k`` is symmetric):
    x0 = omega b / d_k                       (d_k the diagonal of H_k)
    r1 = b - H_k x0
    e  = B_{k+1} (R r1)                      (exact solve on the coarsest level)
    x1 = x0 + P e
    z  = x1 + omega (b - H_k x1) / d_k

Preconditioned CG per column (textbook, with the same freezing of converged
columns as ``cg_source``): ``r = u - H y``, ``z = B r``, ``p = z``,
``rho = r^T z``; then ``alpha = rho / p^T H p``, ``y += alpha p``,
``r -= alpha H p``, ``z = B r``, ``beta = r^T z / rho``, ``p = z + beta p``;
column j stops once ``|r_j| <= tol |u_j|``.

Parity: the transfers against brute-force matrices (``R = P^T / 2^d``,
constants and linear functions reproduced by P away from the boundary), the
coarse potential against a loop over children, the V-cycle against the dense
two-grid formula ``B = (I - E) H^{-1}``,
``E = (I - S H)(I - P H_c^{-1} R H)(I - S H)``, its symmetry and positive
definiteness, PCG with the identity preconditioner against ``cg_source``,
and PCG against the sparse direct solution (``tests/test_oracle_multigrid.py``).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.linalg as sla

from .operator import Operator, apply_H, assemble_H

COARSEST_MAX = 64           # nodes of the coarsest level (solved exactly)
OMEGA = 0.8                 # Jacobi damping


@dataclass
class Level:
    m: tuple                # nodes per axis, x first
    h: tuple
    W: np.ndarray           # V + shift on this level, (n,)
    kinetic: float

    @property
    def n(self) -> int:
        return int(np.prod(self.m))

    @property
    def op(self) -> Operator:
        return Operator(self.m, self.h, self.W, kinetic=self.kinetic, shift=0.0)

    @property
    def diag(self) -> np.ndarray:
        return self.W + self.kinetic * sum(2.0 / (h * h) for h in self.h)


def _grid(X: np.ndarray, m: Sequence[int]) -> np.ndarray:
    """(n, N) block -> array indexed [..., y, x, column] (x fastest)."""
    return X.reshape(tuple(reversed(tuple(m))) + (X.shape[1],))


def _axis(a: int, dim: int) -> int:
    """Array axis of grid axis a in the ``_grid`` layout."""
    return dim - 1 - a


def coarsened_axes(m: Sequence[int]) -> List[int]:
    return [a for a in range(len(m)) if m[a] > 1]


def coarse_shape(m: Sequence[int]) -> tuple:
    return tuple((ma + 1) // 2 if ma > 1 else 1 for ma in m)


def prolong_axis(E: np.ndarray, ax: int, mf: int) -> np.ndarray:
    """Linear interpolation along array axis ``ax`` to ``mf`` fine nodes."""
    mc = E.shape[ax]
    shp = list(E.shape)
    shp[ax] = mf
    out = np.zeros(shp)
    for f in range(mf):
        I = f // 2
        J = I - 1 if f % 2 == 0 else I + 1
        dst = [slice(None)] * E.ndim
        dst[ax] = f
        src = [slice(None)] * E.ndim
        src[ax] = I
        val = 0.75 * E[tuple(src)]
        if 0 <= J < mc:
            src[ax] = J
            val = val + 0.25 * E[tuple(src)]
        out[tuple(dst)] = val
    return out


def restrict_axis(X: np.ndarray, ax: int, mc: int) -> np.ndarray:
    """Full-weighting counterpart of ``prolong_axis``: coarse ``I`` takes
    ``(3/4 (x_{2I} + x_{2I+1}) + 1/4 (x_{2I-1} + x_{2I+2})) / 2``."""
    mf = X.shape[ax]
    shp = list(X.shape)
    shp[ax] = mc
    out = np.zeros(shp)
    for I in range(mc):
        acc = 0.0
        for f, w in ((2 * I, 0.75), (2 * I + 1, 0.75), (2 * I - 1, 0.25), (2 * I + 2, 0.25)):
            if 0 <= f < mf:
                src = [slice(None)] * X.ndim
                src[ax] = f
                acc = acc + w * X[tuple(src)]
        dst = [slice(None)] * X.ndim
        dst[ax] = I
        out[tuple(dst)] = acc / 2.0
    return out


def prolong(fine: Level, coarse: Level, E: np.ndarray) -> np.ndarray:
    """P e for an (n_coarse, N) block -> (n_fine, N)."""
    dim = len(fine.m)
    G = _grid(E, coarse.m)
    for a in coarsened_axes(fine.m):
        G = prolong_axis(G, _axis(a, dim), fine.m[a])
    return G.reshape(fine.n, E.shape[1])


def restrict(fine: Level, coarse: Level, X: np.ndarray) -> np.ndarray:
    """R x = P^T x / 2^d for an (n_fine, N) block -> (n_coarse, N)."""
    dim = len(fine.m)
    G = _grid(X, fine.m)
    for a in coarsened_axes(fine.m):
        G = restrict_axis(G, _axis(a, dim), coarse.m[a])
    return G.reshape(coarse.n, X.shape[1])


def coarse_potential(fine: Level, mc: Sequence[int]) -> np.ndarray:
    """Mean of the fine W over the existing children of each coarse node."""
    dim = len(fine.m)
    Wf = _grid(fine.W[:, None], fine.m)[..., 0]
    cax = coarsened_axes(fine.m)
    Wc = np.zeros(tuple(reversed(tuple(mc))))
    for idx in np.ndindex(*Wc.shape):
        choices = []
        for k in range(dim):                   # array axis k holds grid axis dim - 1 - k
            a = dim - 1 - k
            if a in cax:
                choices.append([f for f in (2 * idx[k], 2 * idx[k] + 1) if f < fine.m[a]])
            else:
                choices.append([idx[k]])
        vals = [Wf[t] for t in itertools.product(*choices)]
        Wc[idx] = sum(vals) / len(vals)
    return Wc.reshape(-1)


class Hierarchy:
    """The levels of the V-cycle for an operator (see the module docstring)."""

    def __init__(self, op: Operator, coarsest_max: int = COARSEST_MAX, omega: float = OMEGA):
        self.omega = omega
        lv = [Level(tuple(int(x) for x in op.m), tuple(float(x) for x in op.h),
                    np.asarray(op.V, dtype=np.float64) + op.shift, float(op.kinetic))]
        while len(lv) == 1 or lv[-1].n > coarsest_max:
            f = lv[-1]
            mc = coarse_shape(f.m)
            if mc == f.m:
                break
            hc = tuple(2.0 * f.h[a] if f.m[a] > 1 else f.h[a] for a in range(len(f.m)))
            lv.append(Level(mc, hc, coarse_potential(f, mc), f.kinetic))
        self.levels = lv
        Hc = assemble_H(lv[-1].op).toarray()
        self.coarse_chol = sla.cho_factor(Hc, lower=True)

    def vcycle(self, b: np.ndarray, k: int = 0) -> np.ndarray:
        """z = B_k b for an (n_k, N) block."""
        b = np.asarray(b, dtype=np.float64)
        L = self.levels[k]
        if k == len(self.levels) - 1:
            return sla.cho_solve(self.coarse_chol, b)
        d = L.diag[:, None]
        w = self.omega
        x0 = w * b / d
        r1 = b - apply_H(L.op, x0)
        e = self.vcycle(restrict(L, self.levels[k + 1], r1), k + 1)
        x1 = x0 + prolong(L, self.levels[k + 1], e)
        return x1 + w * (b - apply_H(L.op, x1)) / d

    def matrix(self) -> np.ndarray:
        """Dense B_0 (small grids only)."""
        n = self.levels[0].n
        return self.vcycle(np.eye(n))


def pcg_source(op: Operator, U: np.ndarray, Y0: Optional[np.ndarray] = None, tol: float = 1e-13,
               max_iter: int = 100000, precond: Optional[Callable[[np.ndarray], np.ndarray]] = None,
               stats: Optional[dict] = None) -> np.ndarray:
    """Textbook preconditioned CG, one system ``H y_j = u_j`` per column, with
    ``precond`` (default: one V-cycle of ``Hierarchy(op)``).  Column j stops
    once ``|u_j - H y_j| <= tol |u_j|``; converged columns are frozen."""
    if precond is None:
        precond = Hierarchy(op).vcycle
    U = np.asarray(U, dtype=np.float64)
    Y = np.zeros_like(U) if Y0 is None else np.array(Y0, dtype=np.float64)
    R = U - apply_H(op, Y)
    Z = precond(R)
    P = Z.copy()
    rho = np.einsum("ij,ij->j", R, Z)
    target = (tol * np.linalg.norm(U, axis=0)) ** 2
    active = np.einsum("ij,ij->j", R, R) > target
    it = 0
    while np.any(active) and it < max_iter:
        Q = apply_H(op, P)
        pq = np.einsum("ij,ij->j", P, Q)
        alpha = np.where(active, rho / np.where(active, pq, 1.0), 0.0)
        Y += P * alpha
        R -= Q * alpha
        rr = np.einsum("ij,ij->j", R, R)
        Z = precond(R)
        rho_new = np.einsum("ij,ij->j", R, Z)
        beta = np.where(active, rho_new / np.where(active, rho, 1.0), 0.0)
        P = Z + P * beta
        rho = np.where(active, rho_new, rho)
        active = active & (rr > target)
        it += 1
    if stats is not None:
        stats["iterations"] = it
        stats["converged"] = not bool(np.any(active))
    return Y
