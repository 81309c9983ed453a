"""Oracle: the discrete operator and its inverse (test infrastructure only).

The paper's bilinear form is ``a(u, v) = int grad u . grad v + V u v`` on
``H_0^1`` (Section 2.2), i.e. the operator ``-Lap + V`` with homogeneous
Dirichlet data; its experiments also use ``-1/2 Lap + V`` (Section 5).  Here the
Laplacian is the standard second-order finite-difference one on the interior
nodes of a uniform grid, so the discrete operator is

    H = c * sum_a (I x ... x L_a x ... x I) + diag(V + sigma),
    L_a = (1/h_a^2) tridiag(-1, 2, -1)   (m_a x m_a, zero Dirichlet halo)

with x the fastest point index.  ``G = H^{-1}`` is the paper's solution
operator (Section 3.1); Step 1 of the scheme applies it to N columns.

Parity: ``apply_H`` / ``assemble_H`` pinned by the closed-form sine-mode
eigenpairs and by brute-force loops; ``GSolver`` / ``cg_source`` pinned by the
residual ``|H y - u|`` and by agreement of the three independent solvers.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class Operator:
    """Finite-difference ``H = kinetic * (-Lap_h) + diag(V + shift)``."""

    m: Sequence[int]          # interior nodes per axis, x first
    h: Sequence[float]        # spacing per axis
    V: np.ndarray             # (n,) potential, x fastest
    kinetic: float = 1.0
    shift: float = 0.0

    @property
    def dim(self) -> int:
        return len(self.m)

    @property
    def n(self) -> int:
        return int(np.prod(self.m))


def laplacian_1d(m: int, h: float) -> sp.csr_matrix:
    """``(1/h^2) tridiag(-1, 2, -1)``: the 1D second difference with zero boundary."""
    e = np.ones(m)
    return sp.diags([-e[:-1], 2.0 * e, -e[:-1]], [-1, 0, 1], format="csr") / (h * h)


def assemble_H(op: Operator) -> sp.csr_matrix:
    """Assembled sparse ``H`` as a Kronecker sum (x fastest, so axis 0 is the
    innermost Kronecker factor)."""
    m = list(op.m)
    n = op.n
    H = sp.csr_matrix((n, n))
    for a in range(op.dim):
        left = int(np.prod(m[a + 1:]))   # slower axes
        right = int(np.prod(m[:a]))      # faster axes
        term = sp.kron(sp.kron(sp.identity(left), laplacian_1d(m[a], op.h[a])), sp.identity(right))
        H = H + term
    H = op.kinetic * H + sp.diags(op.V + op.shift)
    return H.tocsr()


def apply_H(op: Operator, X: np.ndarray) -> np.ndarray:
    """Matrix-free ``H X`` for an ``n x N`` block (rows are grid points)."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[1]
    shape = tuple(reversed(op.m)) + (N,)          # (..., y, x, column)
    Xg = X.reshape(shape)
    Y = np.zeros_like(Xg)
    d = op.dim
    for a in range(d):
        ax = d - 1 - a                              # array axis of grid axis a
        inv_h2 = 1.0 / (op.h[a] * op.h[a])
        lap = 2.0 * Xg
        lo = [slice(None)] * (d + 1)
        hi = [slice(None)] * (d + 1)
        lo[ax] = slice(1, None)
        hi[ax] = slice(None, -1)
        # neighbour at index-1 contributes to point index (lap[1:] -= X[:-1]) and vice versa
        lap[tuple(lo)] -= Xg[tuple(hi)]
        lap[tuple(hi)] -= Xg[tuple(lo)]
        Y += inv_h2 * lap
    Y *= op.kinetic
    Y += (op.V + op.shift).reshape(shape[:-1] + (1,)) * Xg
    return Y.reshape(X.shape)


def cg_source(op: Operator, U: np.ndarray, Y0: Optional[np.ndarray] = None, tol: float = 1e-13,
              max_iter: int = 100000, stats: Optional[dict] = None) -> np.ndarray:
    """Textbook conjugate gradients, one independent system ``H y_j = u_j`` per
    column (the paper's Step 1 solves the N source problems independently).
    Column j stops once ``|u_j - H y_j| <= tol * |u_j|``."""
    U = np.asarray(U, dtype=np.float64)
    Y = np.zeros_like(U) if Y0 is None else np.array(Y0, dtype=np.float64)
    R = U - apply_H(op, Y)
    P = R.copy()
    rho = np.einsum("ij,ij->j", R, R)
    target = (tol * np.linalg.norm(U, axis=0)) ** 2
    active = rho > target
    it = 0
    while np.any(active) and it < max_iter:
        Q = apply_H(op, P)
        pq = np.einsum("ij,ij->j", P, Q)
        alpha = np.where(active, rho / np.where(active, pq, 1.0), 0.0)
        Y += P * alpha
        R -= Q * alpha
        rho_new = np.einsum("ij,ij->j", R, R)
        beta = np.where(active, rho_new / np.where(active, rho, 1.0), 0.0)
        P = R + P * beta
        rho = np.where(active, rho_new, rho)
        active = rho > target
        it += 1
    if stats is not None:
        stats["iterations"] = it
        stats["converged"] = not bool(np.any(active))
    return Y


class GSolver:
    """Applies ``G = H^{-1}`` to a block (Step 1).

    ``method``: ``"dense"`` (Cholesky of the assembled matrix, exact up to
    rounding), ``"sparse"`` (SuperLU factorisation, factored once), ``"cg"``
    (per-column CG to ``tol``), or ``"auto"`` (dense up to n = 4096, sparse up
    to n = 40000, CG beyond).
    """

    def __init__(self, op: Operator, method: str = "auto", tol: float = 1e-13):
        self.op = op
        self.tol = tol
        n = op.n
        if method == "auto":
            method = "dense" if n <= 4096 else ("sparse" if n <= 40000 else "cg")
        self.method = method
        if method == "dense":
            Hd = assemble_H(op).toarray()
            self._chol = sla.cho_factor(Hd, lower=True)    # raises LinAlgError if not SPD
        elif method == "sparse":
            self._lu = spla.splu(assemble_H(op).tocsc(), permc_spec="MMD_AT_PLUS_A")
        elif method != "cg":
            raise ValueError(method)
        self.last_stats = {}

    def __call__(self, U: np.ndarray, Y0: Optional[np.ndarray] = None) -> np.ndarray:
        if self.method == "dense":
            return sla.cho_solve(self._chol, U)
        if self.method == "sparse":
            return self._lu.solve(np.asarray(U, dtype=np.float64))
        self.last_stats = {}
        return cg_source(self.op, U, Y0=Y0, tol=self.tol, stats=self.last_stats)
