"""Plain FP64 CPU oracle for the orthogonality-preserving eigensolver step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the test suite, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP library.

Everything here is written from the paper's definitions (Sections 2 and 4.1,
Algorithm 1) in float64 with numpy/scipy primitives, with no blocking or fusion,
so that a reader can check each function against the paper by eye:

* :mod:`oracle.operator` -- the finite-difference operator ``H = c(-Lap_h) + V``
  (assembled and matrix-free), the solution operator ``G = H^{-1}`` (dense
  Cholesky, sparse LU, or textbook CG per column), a mass operator ``M`` for
  the generalized problem ``H u = lambda M u``, and the lowest eigenpairs by a
  library eigensolver (the converged result the scheme must reach).
* :mod:`oracle.scheme`   -- the midpoint scheme (4.1): the paper's Steps 1-4,
  the same step as a dense Cayley solve and as the 2N x 2N Woodbury system,
  the generator ``L_U``, energy, residual, Ritz values, the Algorithm 1 loop
  (fixed and adaptive step) and the scheme in the inner product of M.
* :mod:`oracle.multigrid` -- the symmetric multigrid V-cycle that preconditions
  Step 1's CG in the library's optional preconditioned form, and that
  preconditioned CG per column.
* :mod:`oracle.net`      -- the small 3D conv-net that stands in for ``H^{-1}``
  applied to residual columns in the learned form (forward, backward, loss);
  imported as ``oracle.net``.

Parity status of every function is listed in the module headers; all are pinned
by ``tests/test_oracle_*.py`` against closed forms, brute force, invariants and
the paper's printed numbers.
"""
from .operator import (  # noqa: F401
    Operator,
    laplacian_1d,
    assemble_H,
    apply_H,
    GSolver,
    cg_source,
    Mass,
    assemble_M,
    apply_M,
    sine_eigenvalues_1d,
    lowest_eigenpairs,
)
from .multigrid import Hierarchy, pcg_source  # noqa: F401
from .scheme import (  # noqa: F401
    inner,
    generator_apply,
    generator_matrix,
    steps_1_to_4,
    step_general,
    step_delta,
    step_cayley_dense,
    step_woodbury,
    small_solve,
    energy,
    ritz_values,
    paper_eigenvalues,
    residual,
    ortho_error,
    subspace_distance,
    run_algorithm1,
    run_algorithm1_adaptive,
    inner_M,
    steps_1_to_4_M,
    step_general_M,
    step_cayley_dense_M,
    residual_M,
    ortho_error_M,
    ritz_values_M,
    orthonormalize_M,
)
