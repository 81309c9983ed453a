"""Pins of the oracle's reference eigensolver (the converged result of the method).

``lowest_eigenpairs`` uses dense ``eigh`` on small grids and preconditioned
LOBPCG above 4096 points.  The LOBPCG branch is checked against

* the closed-form sine spectrum of the Dirichlet Laplacian plus a constant
  (textbook), on an 18^3 grid (multiplicities included);
* scipy's shift-invert Lanczos (``eigsh`` with a sparse factorisation) on a
  Gaussian-well grid above 4096 points, for H and for the pencil (H, M).
"""
import itertools

import numpy as np
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W


def test_lobpcg_branch_matches_closed_form():
    m = (18, 18, 18)
    h = tuple(1.0 / (k + 1) for k in m)
    n = int(np.prod(m))
    op = O.Operator(m, h, np.full(n, 2.0), kinetic=0.5)
    per = [O.sine_eigenvalues_1d(m[a], h[a]) for a in range(3)]
    ref = np.sort([0.5 * (a + b + c) + 2.0 for a, b, c in itertools.product(*per)])[:20]
    got, vecs, res = O.lowest_eigenpairs(op, 20)
    assert np.max(np.abs(got - ref) / ref) <= 1e-11
    assert vecs.shape == (n, 20)
    assert np.max(np.abs(vecs.T @ vecs - np.eye(20))) <= 1e-10


def test_lobpcg_branch_matches_shift_invert_lanczos():
    p = W.wells_3d(m=17, N=12, seed=4, with_u0=False)
    op = O.Operator(p.grid.m, p.grid.h, p.V)
    assert op.n > 4096
    H = O.assemble_H(op).tocsc()
    ref = np.sort(spla.eigsh(H, k=12, sigma=0.0, return_eigenvectors=False))
    got, _, res = O.lowest_eigenpairs(op, 12)
    assert np.max(np.abs(got - ref) / ref) <= 1e-11
    rng = np.random.default_rng(2)
    mass = O.Mass(1.0 + 0.5 * rng.uniform(size=op.n), (0.05, 0.1, -0.08))
    M = O.assemble_M(op, mass).tocsc()
    ref = np.sort(spla.eigsh(H, k=8, M=M, sigma=0.0, return_eigenvectors=False))
    got, _, res = O.lowest_eigenpairs(op, 8, mass=mass)
    assert np.max(np.abs(got - ref) / ref) <= 1e-11
