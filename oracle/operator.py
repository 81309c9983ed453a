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

The paper's experiments work in a finite-element space, where the inner
product of two coefficient vectors is ``c^T M d`` with the mass matrix ``M``
and the stiffness matrix takes the place of H (Section 5, the representation
``U = Phi C``).  ``Mass`` is the finite-difference stand-in for that setting:
an SPD operator ``M = diag(d) + sum_a mu_a (S_a + S_a^T)`` with ``S_a`` the
shift to the next node along axis ``a`` (zero past the boundary), so that the
eigenproblem becomes ``H u = lambda M u``.

``lowest_eigenpairs`` is the plain definition of the converged result of the
method, the N smallest eigenpairs of the SPD matrix ``H`` (or of the pencil
``(H, M)``), computed with a library eigensolver (dense ``eigh`` when small,
else block LOBPCG preconditioned by the exact inverse of ``c(-Lap_h) + s`` via
the discrete sine transform); it never runs the scheme.

Parity: ``apply_H`` / ``assemble_H`` pinned by the closed-form sine-mode
eigenpairs and by brute-force loops; ``GSolver`` / ``cg_source`` pinned by the
residual ``|H y - u|`` and by agreement of the three independent solvers;
``apply_M`` / ``assemble_M`` by brute-force loops and the closed-form spectrum
of a constant-coefficient ``M``; ``lowest_eigenpairs`` by dense ``eigh`` on
small grids and by the closed-form sine spectrum.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy import fft as sfft


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


@dataclass
class Mass:
    """SPD mass operator ``M = diag(d) + sum_a mu_a (S_a + S_a^T)`` on the grid
    of an ``Operator`` (x fastest); ``mu`` has one coefficient per axis."""

    d: np.ndarray             # (n,) diagonal
    mu: Sequence[float]       # off-diagonal coefficient per axis


def assemble_M(op: Operator, mass: Mass) -> sp.csr_matrix:
    """Assembled sparse ``M`` (same Kronecker ordering as ``assemble_H``)."""
    m = list(op.m)
    n = op.n
    M = sp.diags(np.asarray(mass.d, dtype=np.float64)).tocsr()
    for a in range(op.dim):
        if mass.mu[a] == 0.0:
            continue
        left = int(np.prod(m[a + 1:]))
        right = int(np.prod(m[:a]))
        e = np.ones(m[a] - 1)
        off = sp.diags([e, e], [-1, 1], shape=(m[a], m[a]), format="csr")
        M = M + mass.mu[a] * sp.kron(sp.kron(sp.identity(left), off), sp.identity(right))
    return M.tocsr()


def apply_M(op: Operator, mass: Mass, X: np.ndarray) -> np.ndarray:
    """Matrix-free ``M X`` for an ``n x N`` block."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[1]
    shape = tuple(reversed(op.m)) + (N,)
    Xg = X.reshape(shape)
    Y = np.asarray(mass.d, dtype=np.float64).reshape(shape[:-1] + (1,)) * Xg
    d = op.dim
    for a in range(d):
        if mass.mu[a] == 0.0:
            continue
        ax = d - 1 - a
        lo = [slice(None)] * (d + 1)
        hi = [slice(None)] * (d + 1)
        lo[ax] = slice(1, None)
        hi[ax] = slice(None, -1)
        Y[tuple(lo)] += mass.mu[a] * Xg[tuple(hi)]
        Y[tuple(hi)] += mass.mu[a] * Xg[tuple(lo)]
    return Y.reshape(X.shape)


def sine_eigenvalues_1d(m: int, h: float) -> np.ndarray:
    """Eigenvalues ``(4/h^2) sin^2(j pi / (2 (m+1)))``, j = 1..m, of the 1D
    Dirichlet second difference (textbook closed form)."""
    j = np.arange(1, m + 1)
    return (4.0 / (h * h)) * np.sin(j * np.pi / (2.0 * (m + 1))) ** 2


def _dst_preconditioner(op: Operator, s: float):
    """``(c(-Lap_h) + s)^{-1}`` applied to an n x k block by the orthonormal
    type-I discrete sine transform on every axis (exact for that operator)."""
    shape = tuple(reversed(op.m))
    lam = np.zeros(shape)
    for a in range(op.dim):
        ax = op.dim - 1 - a
        w = sine_eigenvalues_1d(op.m[a], op.h[a])
        sh = [1] * op.dim
        sh[ax] = op.m[a]
        lam = lam + w.reshape(sh)
    denom = op.kinetic * lam + s
    axes = tuple(range(op.dim))

    def apply(X):
        X = np.asarray(X, dtype=np.float64)
        k = X.shape[1] if X.ndim == 2 else 1
        Xg = X.reshape(shape + (k,))
        Z = sfft.dstn(Xg, type=1, axes=axes, norm="ortho")
        Z /= denom[..., None]
        return sfft.idstn(Z, type=1, axes=axes, norm="ortho").reshape(X.shape)
    return apply


def lowest_eigenpairs(op: Operator, k: int, mass: Optional[Mass] = None, tol: float = 1e-7,
                      extra: int = 8, seed: int = 12345, max_iter: int = 2000):
    """The ``k`` smallest eigenvalues (ascending) and eigenvectors of ``H``
    (``H x = lambda M x`` when ``mass`` is given).  Dense ``eigh`` for
    n <= 4096; otherwise LOBPCG with ``k + extra`` seeded start vectors, the
    sine-transform preconditioner and residual tolerance ``tol``, followed by
    a Rayleigh-Ritz step on the returned block.  Returns ``(vals, vecs, res)``
    with ``res`` the residual norms ``|H x - lambda M x|`` of unit-M-norm vectors."""
    H = assemble_H(op)
    M = assemble_M(op, mass) if mass is not None else None
    n = op.n
    if n <= 4096:
        Hd = H.toarray()
        if M is None:
            vals, vecs = np.linalg.eigh(Hd)
        else:
            vals, vecs = sla.eigh(Hd, M.toarray())
        vals, vecs = vals[:k], vecs[:, :k]
    else:
        rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x10B9C]))
        X = rng.standard_normal((n, k + extra))
        s = max(1.0, float(np.mean(op.V + op.shift)) + 1.0)
        P = _dst_preconditioner(op, s)
        Pop = spla.LinearOperator((n, n), matvec=P, matmat=P, dtype=np.float64)
        vals, vecs = spla.lobpcg(H, X, B=M, M=Pop, tol=tol, maxiter=max_iter, largest=False)
        # Rayleigh-Ritz on the returned block (orthonormalise in the M product first)
        G = vecs.T @ (M @ vecs if M is not None else vecs)
        L = np.linalg.cholesky(0.5 * (G + G.T))
        Q = np.linalg.solve(L, vecs.T).T
        A = Q.T @ (H @ Q)
        w, Z = np.linalg.eigh(0.5 * (A + A.T))
        vals, vecs = w[:k], (Q @ Z)[:, :k]
    MV = M @ vecs if M is not None else vecs
    res = np.linalg.norm(H @ vecs - MV * vals[None, :], axis=0)
    return vals, vecs, res
