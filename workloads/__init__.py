"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module produces *inputs only*: grid descriptions, potential values on the
grid and an orthonormal starting block.  It holds none of the eigensolver's
arithmetic (no operator application, no Gram products, no time step), so that
the CPU oracle and the HIP library stay independent of each other and can both
be fed from here.

Conventions (stated once, used everywhere):

* A grid is the set of interior nodes of a uniform finite-difference grid with
  homogeneous Dirichlet boundary.  Axis ``a`` has ``m[a]`` interior nodes and
  spacing ``h[a]``; node ``i`` (0-based) of axis ``a`` sits at
  ``lo[a] + (i + 1) * h[a]``.
* Points are numbered with the x index fastest:
  ``p = i0 + m0 * (i1 + m1 * i2)``.  Every n-vector (the potential, one column
  of an orbital block) uses that order.
* An orbital block is an ``n x N`` row-major (point-major) float64 array: the N
  orbital values of one grid point are contiguous.

The paper's initial data is "random data with mutually orthogonal columns"
(Section 5, experiment set-up).  Here it is a seeded standard-normal ``n x N``
matrix orthonormalised by Householder QR with the signs fixed so that
``diag(R) > 0``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "Grid",
    "Problem",
    "harmonic_potential",
    "gaussian_wells",
    "gaussian_wells_params",
    "initial_block",
    "harmonic_2d_32",
    "wells_3d",
    "batched_problems",
    "hydrogen_softened",
    "oscillator_2d_paper",
]


@dataclass(frozen=True)
class Grid:
    """Uniform interior grid with homogeneous Dirichlet boundary."""

    m: Tuple[int, ...]            # interior nodes per axis, x first
    h: Tuple[float, ...]          # spacing per axis
    lo: Tuple[float, ...]         # coordinate of the (excluded) boundary node 0

    @property
    def dim(self) -> int:
        return len(self.m)

    @property
    def n(self) -> int:
        return int(np.prod(self.m))

    def coords(self) -> List[np.ndarray]:
        """Node coordinates as arrays of shape ``m[::-1]`` (z, y, x order)."""
        axes = [self.lo[a] + (np.arange(self.m[a]) + 1.0) * self.h[a] for a in range(self.dim)]
        # meshgrid with 'ij' on reversed axes gives arrays indexed [..., i1, i0]
        grids = np.meshgrid(*axes[::-1], indexing="ij")
        return grids[::-1]  # x-coordinate array first


@dataclass
class Problem:
    """One synthetic eigenproblem instance: grid, operator scaling, potential, start block."""

    name: str
    grid: Grid
    V: np.ndarray                 # (n,) float64, x fastest
    N: int
    tau: float
    kinetic: float = 1.0          # H = kinetic * (-Laplacian_h) + V + shift
    shift: float = 0.0
    U0: np.ndarray = field(default=None, repr=False)  # (n, N) float64 row-major
    meta: dict = field(default_factory=dict)


def unit_box_grid(m: Sequence[int]) -> Grid:
    """Interior nodes of the unit box with ``h = 1/(m+1)`` on every axis."""
    m = tuple(int(v) for v in m)
    return Grid(m=m, h=tuple(1.0 / (v + 1) for v in m), lo=tuple(0.0 for _ in m))


def harmonic_potential(grid: Grid, scale: float, centre: Sequence[float]) -> np.ndarray:
    """``V(x) = scale * 0.5 * |x - c|^2`` sampled on the grid, flattened x-fastest."""
    xs = grid.coords()
    r2 = sum((xs[a] - centre[a]) ** 2 for a in range(grid.dim))
    return np.ascontiguousarray((scale * 0.5 * r2).ravel(), dtype=np.float64)


def gaussian_wells_params(seed: int, count: int = 8, dim: int = 3):
    """Depths, widths and centres of ``count`` wells, drawn in this fixed order:
    depths ~ U[5, 20], widths ~ U[0.05, 0.15], centres ~ U[0.15, 0.85]^dim."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x57E11]))
    depth = rng.uniform(5.0, 20.0, size=count)
    width = rng.uniform(0.05, 0.15, size=count)
    centre = rng.uniform(0.15, 0.85, size=(count, dim))
    return depth, width, centre


def gaussian_wells(grid: Grid, seed: int, count: int = 8) -> np.ndarray:
    """``V(x) = -sum_k d_k exp(-|x - c_k|^2 / (2 w_k^2))`` on the grid (attractive wells)."""
    depth, width, centre = gaussian_wells_params(seed, count, grid.dim)
    xs = grid.coords()
    V = np.zeros(xs[0].shape)
    for k in range(count):
        r2 = sum((xs[a] - centre[k, a]) ** 2 for a in range(grid.dim))
        V -= depth[k] * np.exp(-r2 / (2.0 * width[k] ** 2))
    return np.ascontiguousarray(V.ravel(), dtype=np.float64)


def initial_block(n: int, N: int, seed: int) -> np.ndarray:
    """Seeded standard-normal ``n x N`` block, orthonormalised by Householder QR,
    columns sign-fixed so that ``diag(R) > 0``.  Row-major float64."""
    if N > n:
        raise ValueError(f"cannot build {N} orthonormal columns in dimension {n}")
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x0B17A1]))
    G = rng.standard_normal((n, N))
    Q, R = np.linalg.qr(G, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return np.ascontiguousarray(Q * s[None, :], dtype=np.float64)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def harmonic_2d_32(seed: int = 0, m: int = 32, N: int = 8, tau: float = 0.1) -> Problem:
    """2D 5-point Dirichlet Laplacian on the 32x32 interior grid of the unit
    square (h = 1/33) plus ``V = 100 * 0.5 |x - c|^2`` with ``c = (1/2, 1/2)``,
    N = 8, tau = 0.1."""
    g = unit_box_grid((m, m))
    V = harmonic_potential(g, 100.0, (0.5, 0.5))
    return Problem(name=f"harmonic2d_{m}x{m}_N{N}", grid=g, V=V, N=N, tau=tau,
                   U0=initial_block(g.n, N, seed), meta={"seed": seed, "steps": 300})


def wells_3d(m: int = 64, N: int = 128, seed: int = 0, tau: float = 200.0,
             wells: int = 8, with_u0: bool = True) -> Problem:
    """3D 7-point Dirichlet Laplacian on the m^3 interior grid of the unit cube
    (h = 1/(m+1)) plus ``wells`` seeded Gaussian wells; ``N`` lowest pairs."""
    g = unit_box_grid((m, m, m))
    V = gaussian_wells(g, seed, wells)
    U0 = initial_block(g.n, N, seed) if with_u0 else None
    return Problem(name=f"wells3d_{m}^3_N{N}_s{seed}", grid=g, V=V, N=N, tau=tau, U0=U0,
                   meta={"seed": seed, "wells": wells})


def batched_problems(count: int = 64, seed: int = 0, m_lo: int = 24, m_hi: int = 48,
                     N_lo: int = 16, N_hi: int = 128, tau: float = 200.0) -> List[Problem]:
    """``count`` independent 3D well problems with grid edge ~ U{m_lo..m_hi} and
    N ~ U{N_lo..N_hi}, each with its own well seed; all derived from ``seed``."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0xBA7C4]))
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    Ns = rng.integers(N_lo, N_hi + 1, size=count)
    out = []
    for b in range(count):
        out.append(wells_3d(m=int(ms[b]), N=int(Ns[b]), seed=int(seed) * 1000 + 17 + b, tau=tau))
    return out


def oscillator_2d_paper(m: int = 99, N: int = 15, tau: float = 0.05, seed: int = 0) -> Problem:
    """Finite-difference analogue of the paper's first test problem:
    ``-1/2 Laplacian + 1/2 |x|^2`` on (-5.5, 5.5)^2, N = 15."""
    L = 11.0
    h = L / (m + 1)
    g = Grid(m=(m, m), h=(h, h), lo=(-5.5, -5.5))
    V = harmonic_potential(g, 1.0, (0.0, 0.0))
    return Problem(name=f"oscillator2d_{m}_N{N}", grid=g, V=V, N=N, tau=tau, kinetic=0.5,
                   U0=initial_block(g.n, N, seed), meta={"seed": seed})


def hydrogen_softened(m: int = 63, N: int = 5, tau: float = 1.0, soft: float = 0.1,
                      half: float = 10.0, seed: int = 0, shift: float = 1.0) -> Problem:
    """Finite-difference analogue of the paper's second test problem:
    ``-1/2 Laplacian - 1/sqrt(|x|^2 + soft^2)`` on (-half, half)^3, N = 5.
    The operator is indefinite, so a diagonal shift makes it positive definite."""
    h = 2.0 * half / (m + 1)
    g = Grid(m=(m, m, m), h=(h, h, h), lo=(-half, -half, -half))
    xs = g.coords()
    r2 = xs[0] ** 2 + xs[1] ** 2 + xs[2] ** 2
    V = np.ascontiguousarray((-1.0 / np.sqrt(r2 + soft * soft)).ravel())
    return Problem(name=f"hydrogen_soft_{m}^3_N{N}", grid=g, V=V, N=N, tau=tau, kinetic=0.5,
                   shift=shift, U0=initial_block(g.n, N, seed), meta={"seed": seed, "soft": soft})
