"""Oracle: the orthogonality-preserving midpoint scheme (test infrastructure only).

Notation (paper, Section 2.1): for blocks ``U = (u_1..u_N)``, ``V`` the inner
matrix is ``<U, V>_ij = (u_i, v_j)``; with Euclidean inner products on grid
vectors that is ``U^T V``.  The Euclidean product differs from the quadrature
weighted ``int u v`` by the constant factor ``prod h_a``, which every N x N
matrix of the scheme is invariant to once ``U^0`` is orthonormal in the same
product.

Functions and the passage each follows:

* ``generator_apply`` / ``generator_matrix`` -- ``L_U V = U<GU, V> - GU<U, V>``
  (eq. (3.2)); as an n x n matrix ``L_U = U Y^T - Y U^T`` with ``Y = GU``.
* ``steps_1_to_4`` -- the scheme (4.1) solved by the paper's Steps 1-4
  (Section 4.1), literally: Step 1 ``Y = GU``; Step 2
  ``(I + tau^2/4 (<Y,Y> - <Y,U><Y,U>)) B = I``; Step 3
  ``tau/2 A = I - B + tau/2 <Y,U> B``; Step 4 ``U' = U - tau U A + tau Y B``.
* ``step_cayley_dense`` -- the same step straight from (4.1):
  ``(I + tau/2 L_U) U' = (I - tau/2 L_U) U`` as an n x n dense solve.  Needs no
  symmetry of ``<Y, U>``, so it is the definition for an inexact Y.
* ``step_general`` -- Steps 2-4 re-derived from (4.1) exactly as the paper does
  but without using ``<Y,U> = <U,Y>`` (which only holds for exact ``Y = GU``):
  ``M = I + tau/2 (S_a - S_b) + tau^2/4 (T - S_a S_b)``, ``B = M^{-1}``,
  ``A = 2/tau (I - B) + S_b B`` with ``S_a = Y^T U``, ``S_b = U^T Y``,
  ``T = Y^T Y``.  Identical to ``steps_1_to_4`` when ``S_a = S_b``.
* ``step_delta`` -- the same step as a correction of U (Step 3 substituted
  into Step 4, ``T - S_a S_b`` rewritten through ``P = Y - U S_b``); equal to
  ``step_general`` for any U and Y.
* ``step_woodbury`` -- (4.1) written with ``L_U = W J W^T``, ``W = [U, Y]``,
  and inverted through the 2N x 2N capacitance matrix (push-through identity).
* ``energy``, ``residual``, ``ritz_values``, ``paper_eigenvalues``,
  ``ortho_error`` -- ``E(U) = 1/2 tr <U,U>_a`` (eq. (2.3)), the eigen-residual,
  Ritz values, the paper's ``eig(<GU,U>^{-1})`` (Section 5 error measure) and
  ``|<U,U> - I|_F`` (Theorem 4.1).
* ``run_algorithm1`` -- Algorithm 1 with a fixed step and either the paper's
  relative-energy-change stop or an eigen-residual stop.
* ``run_algorithm1_adaptive`` -- Algorithm 1 with the step chosen in
  ``[tau_min, tau_max]`` at every iteration.  The paper leaves the choice
  open; the rule here rests on Theorem 4.2 (the energy decays for steps below
  a threshold): a step whose energy rises is redone with the step shrunk
  (never below tau_min), an accepted step lets the next one grow (never above
  tau_max).  Stops on the relative energy change of Algorithm 1, on the
  relative energy error against a reference energy (the stop of the
  experiments, Section 5), or on the eigen-residual.
* ``*_M`` -- the same scheme with the inner product ``<U, V> = U^T M V`` of a
  mass operator M (Section 5: coefficient vectors of a finite-element space,
  where Step 1 reads ``K (GU) = M U``).  ``G = K^{-1} M`` and every inner
  matrix of Steps 2-4 is taken in the M product; Step 4 is unchanged.

Parity: all functions are pinned (tests/test_oracle_scheme.py,
tests/test_oracle_algorithm1.py, tests/test_oracle_mass.py): the three step
forms agree with each other, orthogonality is preserved (Theorem 4.1), energy
decreases (Theorem 4.2), eigenbases are fixed points (Remark after (3.1)),
``L_U`` is skew (Lemma 3.2), the Step-2 matrix is >= I (Lemma 3.1), and the
iteration converges to dense ``eigh`` / closed-form eigenvalues.
"""
from __future__ import annotations

from typing import Callable, Dict, List, Optional

import numpy as np
import scipy.linalg as sla

from .operator import Mass, Operator, apply_H, apply_M


def inner(U: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Inner matrix ``<U, V>_ij = (u_i, v_j)`` (Section 2.1), Euclidean."""
    return U.T @ V


def generator_apply(U: np.ndarray, Y: np.ndarray, V: np.ndarray) -> np.ndarray:
    """``L_U V = U <Y, V> - Y <U, V>`` with ``Y = GU`` (eq. (3.2))."""
    return U @ inner(Y, V) - Y @ inner(U, V)


def generator_matrix(U: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """``L_U`` as an explicit n x n matrix acting on columns: ``U Y^T - Y U^T``."""
    return U @ Y.T - Y @ U.T


def small_solve(S_a: np.ndarray, T: np.ndarray, tau: float, S_b: Optional[np.ndarray] = None):
    """Steps 2 and 3 of Section 4.1.

    With ``S_b`` omitted this is the paper's form (``S = <GU, U>`` symmetric):
    ``B = (I + tau^2/4 (T - S S))^{-1}``, ``A = 2/tau (I - B + tau/2 S B)``.
    With ``S_b = <U, Y>`` given it is the same elimination without assuming
    ``S_a = S_b`` (see ``step_general``).  Returns ``(A, B, M)``."""
    N = S_a.shape[0]
    I = np.eye(N)
    if S_b is None:
        M = I + 0.25 * tau * tau * (T - S_a @ S_a)
        B = np.linalg.solve(M, I)
        A = (2.0 / tau) * (I - B + 0.5 * tau * S_a @ B)
    else:
        M = I + 0.5 * tau * (S_a - S_b) + 0.25 * tau * tau * (T - S_a @ S_b)
        B = np.linalg.solve(M, I)
        A = (2.0 / tau) * (I - B) + S_b @ B
    return A, B, M


def steps_1_to_4(U: np.ndarray, G: Callable[[np.ndarray], np.ndarray], tau: float) -> Dict[str, np.ndarray]:
    """One step of scheme (4.1) by the paper's Steps 1-4 (Section 4.1)."""
    Y = G(U)                                   # Step 1: N source problems
    S = inner(Y, U)                            # <GU, U>
    T = inner(Y, Y)                            # <GU, GU>
    A, B, M = small_solve(S, T, tau)           # Steps 2, 3
    U_next = U - tau * U @ A + tau * Y @ B     # Step 4
    return {"U": U_next, "Y": Y, "A": A, "B": B, "S": S, "T": T, "M": M}


def step_general(U: np.ndarray, Y: np.ndarray, tau: float) -> Dict[str, np.ndarray]:
    """Steps 2-4 for a given block Y (not necessarily exactly GU), eliminated
    from (4.1) without assuming ``<Y,U> = <U,Y>``."""
    S_a = inner(Y, U)
    S_b = inner(U, Y)
    T = inner(Y, Y)
    A, B, M = small_solve(S_a, T, tau, S_b=S_b)
    U_next = U - tau * U @ A + tau * Y @ B
    return {"U": U_next, "A": A, "B": B, "S_a": S_a, "S_b": S_b, "T": T, "M": M}


def step_delta(U: np.ndarray, Y: np.ndarray, tau: float) -> Dict[str, np.ndarray]:
    """Steps 2-4 written as a correction of U (the form the reduced-precision
    path evaluates).  With ``S_b = <U,Y>``, ``C = <U,U>`` and ``P = Y - U S_b``,
    ``T - S_a S_b = P^T P - S_b^T (C - I) S_b`` and Step 3 turns Step 4 into
    ``U' = U - 2 U (I - B) + tau P B``.  Algebraically identical to
    ``step_general`` for any U and Y; both correction terms vanish at a fixed
    point, which is what lets them be evaluated in low precision."""
    N = U.shape[1]
    I = np.eye(N)
    S_b = inner(U, Y)
    P = Y - U @ S_b
    C = inner(U, U)
    Tp = inner(P, P) - S_b.T @ (C - I) @ S_b
    M = I + 0.5 * tau * (S_b.T - S_b) + 0.25 * tau * tau * Tp
    B = np.linalg.solve(M, I)
    Z1 = -2.0 * (I - B)
    Z2 = tau * B
    return {"U": U + U @ Z1 + P @ Z2, "B": B, "S_b": S_b, "P": P, "Tp": Tp, "Z1": Z1, "Z2": Z2, "M": M}


def step_cayley_dense(U: np.ndarray, Y: np.ndarray, tau: float) -> np.ndarray:
    """(4.1) as written: ``(U' - U)/tau = -L_U (U' + U)/2`` solved densely for U'."""
    n = U.shape[0]
    L = generator_matrix(U, Y)
    I = np.eye(n)
    return np.linalg.solve(I + 0.5 * tau * L, (I - 0.5 * tau * L) @ U)


def step_woodbury(U: np.ndarray, Y: np.ndarray, tau: float) -> np.ndarray:
    """(4.1) with ``L_U = W J W^T`` (``W = [U, Y]``, ``J = [[0, I], [-I, 0]]``):
    ``U' = U - tau W (I_2N + tau/2 J W^T W)^{-1} J W^T U``."""
    N = U.shape[1]
    W = np.hstack([U, Y])
    J = np.zeros((2 * N, 2 * N))
    J[:N, N:] = np.eye(N)
    J[N:, :N] = -np.eye(N)
    cap = np.eye(2 * N) + 0.5 * tau * J @ (W.T @ W)
    X = np.linalg.solve(cap, J @ (W.T @ U))
    return U - tau * W @ X


def energy(op: Operator, U: np.ndarray) -> float:
    """``E(U) = 1/2 tr <U, U>_a = 1/2 tr(U^T H U)`` (eq. (2.3))."""
    return 0.5 * float(np.sum(U * apply_H(op, U)))


def ritz_values(op: Operator, U: np.ndarray) -> np.ndarray:
    """Eigenvalues of ``U^T H U`` (ascending)."""
    Lam = U.T @ apply_H(op, U)
    return np.linalg.eigvalsh(0.5 * (Lam + Lam.T))


def paper_eigenvalues(U: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Eigenvalues of ``<GU, U>^{-1}`` with ``Y = GU`` (Section 5 error measure), ascending."""
    S = inner(Y, U)
    w = np.linalg.eigvals(np.linalg.inv(S))
    return np.sort(w.real)


def residual(op: Operator, U: np.ndarray) -> float:
    """``|H U - U Lam|_F / |Lam|_F`` with ``Lam = U^T H U``."""
    HU = apply_H(op, U)
    Lam = U.T @ HU
    return float(np.linalg.norm(HU - U @ Lam) / np.linalg.norm(Lam))


def ortho_error(U: np.ndarray) -> float:
    """``|<U, U> - I|_F`` (the quantity Theorem 4.1 keeps at zero)."""
    return float(np.linalg.norm(U.T @ U - np.eye(U.shape[1])))


def subspace_distance(U: np.ndarray, V: np.ndarray) -> float:
    """Sine of the largest principal angle between span(U) and span(V)."""
    return float(np.sin(np.max(sla.subspace_angles(U, V))))


def run_algorithm1(op: Operator, U0: np.ndarray, tau: float, G: Callable[[np.ndarray], np.ndarray],
                   max_steps: int, res_tol: Optional[float] = None, energy_tol: Optional[float] = None,
                   record: bool = True) -> Dict[str, object]:
    """Algorithm 1 with a fixed step ``tau``.

    Stops after ``max_steps`` steps, or when the eigen-residual drops to
    ``res_tol``, or when the relative energy change
    ``|E(U^{n+1}) - E(U^n)| / |E(U^n)|`` drops to ``energy_tol`` (the rule of
    Algorithm 1).  Step 1 is ``G``."""
    U = np.array(U0, dtype=np.float64)
    E = energy(op, U)
    hist: Dict[str, List[float]] = {"E": [E], "res": [residual(op, U)], "ortho": [ortho_error(U)]}
    steps = 0
    while steps < max_steps:
        if res_tol is not None and hist["res"][-1] <= res_tol:
            break
        out = steps_1_to_4(U, G, tau)
        U = out["U"]
        E_new = energy(op, U)
        errE = abs(E_new - E) / abs(E)
        E = E_new
        steps += 1
        if record or res_tol is not None:
            hist["E"].append(E)
            hist["res"].append(residual(op, U))
            hist["ortho"].append(ortho_error(U))
        if energy_tol is not None and errE <= energy_tol:
            break
    return {"U": U, "steps": steps, "hist": hist}


def run_algorithm1_adaptive(op: Operator, U0: np.ndarray, G: Callable[[np.ndarray], np.ndarray], tau0: float,
                            tau_min: float, tau_max: float, max_steps: int, energy_tol: Optional[float] = None,
                            energy_ref: Optional[float] = None, res_tol: Optional[float] = None,
                            grow: float = 1.5, shrink: float = 0.5, slack: float = 1e-13,
                            step: Optional[Callable] = None) -> Dict[str, object]:
    """Algorithm 1 with ``tau_n`` chosen in ``[tau_min, tau_max]``.

    Iteration n: with the current step tau, compute U' by Steps 1-4 (``step``,
    default ``steps_1_to_4`` with ``G``).  If ``E(U') <= E(U^n) + slack |E(U^n)|``
    (Theorem 4.2's energy decay) or tau is already tau_min, accept: U^{n+1} = U',
    ``err_E^n = |E(U^{n+1}) - E(U^n)| / |E(U^n)|``, and the next step starts at
    ``min(tau_max, grow tau)``.  Otherwise reject U', set
    ``tau = max(tau_min, shrink tau)`` and recompute from U^n.

    Stops (checked before every iteration, in this order): ``res_tol`` on the
    eigen-residual of U^n; with ``energy_ref``, the experiments' relative energy
    error ``(E(U^n) - E_ref) / |E_ref| <= energy_tol``; else Algorithm 1's
    ``err_E <= energy_tol`` with ``err_E^0 = |E(U^0)|``; or ``max_steps``
    accepted steps.  Returns U, the accepted step count, the rejected count,
    and the per-step histories (energy, tau used, residual if ``res_tol``)."""
    if not (0.0 < tau_min <= tau0 <= tau_max):
        raise ValueError("need 0 < tau_min <= tau0 <= tau_max")
    if step is None:
        def step(U, tau):
            return steps_1_to_4(U, G, tau)["U"]
    U = np.array(U0, dtype=np.float64)
    E = energy(op, U)
    errE = abs(E)
    tau = tau0
    hist: Dict[str, List[float]] = {"E": [E], "tau": [], "errE": []}
    if res_tol is not None:
        hist["res"] = [residual(op, U)]
    steps = 0
    rejected = 0
    while True:
        if res_tol is not None and hist["res"][-1] <= res_tol:
            break
        if energy_tol is not None:
            if energy_ref is not None:
                if (E - energy_ref) / abs(energy_ref) <= energy_tol:
                    break
            elif errE <= energy_tol:
                break
        if steps >= max_steps:
            break
        while True:
            U_new = step(U, tau)
            E_new = energy(op, U_new)
            if E_new <= E + slack * abs(E) or tau <= tau_min:
                break
            rejected += 1
            tau = max(tau_min, shrink * tau)
        errE = abs(E_new - E) / abs(E)
        U, E = U_new, E_new
        steps += 1
        hist["E"].append(E)
        hist["tau"].append(tau)
        hist["errE"].append(errE)
        if res_tol is not None:
            hist["res"].append(residual(op, U))
        tau = min(tau_max, grow * tau)
    return {"U": U, "steps": steps, "rejected": rejected, "hist": hist}


# ---------------------------------------------------------------------------
# the scheme in the inner product of a mass operator M
# ---------------------------------------------------------------------------

def inner_M(op: Operator, mass: Mass, U: np.ndarray, V: np.ndarray) -> np.ndarray:
    """``<U, V> = U^T M V``."""
    return U.T @ apply_M(op, mass, V)


def steps_1_to_4_M(op: Operator, mass: Mass, U: np.ndarray, solve_K: Callable[[np.ndarray], np.ndarray],
                   tau: float) -> Dict[str, np.ndarray]:
    """Steps 1-4 of Section 4.1 in the M product: Step 1 solves ``K Y = M U``
    (``solve_K`` applies K^{-1}); ``S = <Y, U>``, ``T = <Y, Y>``; Steps 2-3 as
    ``small_solve``; Step 4 ``U' = U - tau U A + tau Y B``."""
    Y = solve_K(apply_M(op, mass, U))
    S = inner_M(op, mass, Y, U)
    T = inner_M(op, mass, Y, Y)
    A, B, Mb = small_solve(S, T, tau)
    return {"U": U - tau * U @ A + tau * Y @ B, "Y": Y, "A": A, "B": B, "S": S, "T": T}


def step_general_M(op: Operator, mass: Mass, U: np.ndarray, Y: np.ndarray, tau: float) -> Dict[str, np.ndarray]:
    """Steps 2-4 for a given Y in the M product without assuming ``<Y,U> = <U,Y>``."""
    S_a = inner_M(op, mass, Y, U)
    S_b = inner_M(op, mass, U, Y)
    T = inner_M(op, mass, Y, Y)
    A, B, Mb = small_solve(S_a, T, tau, S_b=S_b)
    return {"U": U - tau * U @ A + tau * Y @ B, "A": A, "B": B, "S_a": S_a, "S_b": S_b, "T": T}


def step_cayley_dense_M(Mdense: np.ndarray, U: np.ndarray, Y: np.ndarray, tau: float) -> np.ndarray:
    """(4.1) solved densely with ``L_U V = U <Y, V> - Y <U, V>`` in the M
    product, i.e. ``L_U = (U Y^T - Y U^T) M`` as an n x n matrix."""
    n = U.shape[0]
    L = (U @ Y.T - Y @ U.T) @ Mdense
    I = np.eye(n)
    return np.linalg.solve(I + 0.5 * tau * L, (I - 0.5 * tau * L) @ U)


def residual_M(op: Operator, mass: Mass, U: np.ndarray) -> float:
    """``|K U - M U Lam|_F / |Lam|_F`` with ``Lam = U^T K U``."""
    HU = apply_H(op, U)
    Lam = U.T @ HU
    return float(np.linalg.norm(HU - apply_M(op, mass, U) @ Lam) / np.linalg.norm(Lam))


def ortho_error_M(op: Operator, mass: Mass, U: np.ndarray) -> float:
    """``|<U, U> - I|_F`` in the M product (Theorem 4.1 keeps it at zero)."""
    return float(np.linalg.norm(inner_M(op, mass, U, U) - np.eye(U.shape[1])))


def ritz_values_M(op: Operator, mass: Mass, U: np.ndarray) -> np.ndarray:
    """Eigenvalues of the pencil ``(U^T K U, U^T M U)`` (ascending)."""
    Lam = U.T @ apply_H(op, U)
    C = inner_M(op, mass, U, U)
    return sla.eigh(0.5 * (Lam + Lam.T), 0.5 * (C + C.T), eigvals_only=True)


def orthonormalize_M(op: Operator, mass: Mass, U: np.ndarray) -> np.ndarray:
    """``U R^{-1}`` with ``R`` the upper Cholesky factor of ``U^T M U``
    (``R^T R = U^T M U``, positive diagonal): the unique M-orthonormal block
    with the same column span and an upper-triangular change of basis."""
    C = inner_M(op, mass, U, U)
    R = np.linalg.cholesky(0.5 * (C + C.T)).T
    return sla.solve_triangular(R, U.T, trans="T", lower=False).T
