/*
 * ope.h -- C ABI of the MI355X (gfx950) orthogonality-preserving eigensolver step.
 *
 * The library computes the N lowest eigenpairs of the finite-difference
 * operator  H = c * (-Lap_h) + diag(V + sigma)  (homogeneous Dirichlet
 * boundary, 5-point stencil in 2D, 7-point in 3D) with the midpoint scheme of
 * the paper's Section 4.1, eq. (4.1):
 *
 *     (U' - U) / tau = -L_U (U' + U) / 2,   L_U V = U <GU, V> - GU <U, V>,
 *     G = H^{-1},
 *
 * solved per step by Steps 1-4 of Section 4.1: Step 1 applies G to the N
 * columns (warm-started conjugate gradients on the device), Steps 2-3 solve a
 * small N x N system in FP64 (the Schur complement of the 2N x 2N capacitance
 * system), Step 4 updates U in place.  Algorithm 1 drives the loop.
 *
 * Conventions shared by every entry point:
 *  - Grid points are numbered x fastest: p = i0 + m0 * (i1 + m1 * i2).
 *  - An orbital block is n x N, row-major ("point-major"): element (p, j) at
 *    offset p * N + j, where n = prod(m).  Block pointers are DEVICE pointers
 *    owned by the caller, 16-byte aligned, and must not overlap unless an
 *    entry point says so.
 *  - Inner matrices <X, Y> = X^T Y are N x N row-major; pointers to them are
 *    device pointers unless the argument says "host".
 *  - Every entry point returns an ope_status; on error no caller buffer
 *    named as an output has been written unless stated otherwise.  Work is
 *    enqueued on the stream given to ope_create (NULL = default stream);
 *    entry points that return host values synchronise that stream.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef OPE_H
#define OPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OPE_OK = 0,
  OPE_EINVAL = 1,      /* invalid argument (sizes, null pointers, dim, N > n ...) */
  OPE_ENOMEM = 2,      /* device or pinned-host allocation failed */
  OPE_EHIP = 3,        /* a HIP runtime call failed */
  OPE_ENONFINITE = 4,  /* a NaN or Inf appeared in a reduction; U left unchanged */
  OPE_ECG_MAXIT = 5,   /* Step 1 hit its iteration cap before the tolerance (step still applied) */
  OPE_EPIVOT = 6,      /* non-positive or tiny pivot in a small FP64 solve; U left unchanged */
  OPE_EUNSUPPORTED = 7,/* valid request the library does not implement */
  OPE_ENOTSPD = 8      /* the operator (or mass operator) is not symmetric positive definite */
} ope_status;

/* OPE_FP64: every block and every operation in FP64.
 * OPE_MIXED: orbital blocks (U and the workspace) stored in FP32; stencil and
 * Step-1 CG in FP32; <U,U> and <U,HU> (energy, drift) accumulated in FP64 on the
 * matrix cores; <U,Y> and the projection P = Y - U<U,Y> in FP32 on the matrix
 * cores; P^T P in BF16 with FP32 accumulation; Step 4 in FP32 on the matrix
 * cores, written in delta form U' = U + U Z1 + P Z2 (Z1 = -2(I - B),
 * Z2 = tau B) so that its rounding vanishes at convergence; the Step-2 matrix uses
 * T - S_a S_b = P^T P - S_b^T (C - I) S_b; the small solves and all checks in FP64.
 * FP32 rounding and the BF16 P^T P add to the drift |U^T U - I|_F that the
 * scheme itself keeps constant, so after every update the drift of the new
 * block is measured (C = U^T U accumulated in FP64) and, above 2.5e-7, the
 * device applies U <- U (3I - C)/2 (one Newton-Schulz step; drift E -> O(E^2))
 * before the block is handed back; a block entering a step with a drift
 * above 1e-6 gets the same correction first.
 * Its accuracy is bounded by FP32 storage (residual floor about 1e-6); convert
 * U to FP64 and continue with an OPE_FP64 context to finish. */
typedef enum { OPE_FP64 = 0, OPE_MIXED = 1 } ope_precision;

/* The discrete operator (paper, Section 2.2 bilinear form a(u,v), discretised
 * by second-order finite differences on the interior nodes of a uniform grid). */
typedef struct {
  int32_t dim;        /* 2 or 3 */
  int64_t m[3];       /* interior nodes per axis, x first (m[2] ignored for dim 2); each >= 1 */
  double h[3];        /* grid spacing per axis (> 0) */
  double kinetic;     /* c > 0: 1.0 for -Lap, 0.5 for -1/2 Lap */
  double shift;       /* sigma added to the diagonal */
  const double* V;    /* HOST pointer to n potential values, x fastest; copied at create */
} ope_op_desc;

typedef struct {
  double energy;      /* E(U) = 1/2 tr(U^T H U) of the iterate entering the step (eq. (2.3)) */
  double residual;    /* |H U - U Lam|_F / |Lam|_F of that iterate, Lam = U^T H U */
  double drift;       /* |U^T U - I|_F of that iterate (Theorem 4.1 keeps it ~ 0) */
  int32_t inner_iterations; /* CG iterations spent in Step 1 */
  int32_t status;     /* ope_status of the step */
} ope_step_info;

typedef struct {
  int32_t steps;      /* steps taken */
  int32_t converged;  /* 1 if the residual reached res_tol */
  double residual;    /* final residual (same definition as ope_step_info) */
  double energy;      /* final energy */
  double drift;       /* final |U^T U - I|_F */
  int64_t inner_iterations; /* total CG iterations */
  int32_t stalled;    /* OPE_MIXED only: 1 if the residual stopped improving (60 steps without a 10% gain) */
  int32_t learned_steps; /* steps taken by the learned form and kept by its judge */
  int32_t rejected;   /* ope_solve_ex: steps redone with a smaller tau (energy rose) */
  int32_t reserved;
  double tau;         /* ope_solve_ex: the step the next iteration would take */
} ope_solve_info;

typedef struct ope_ctx ope_ctx;

/* Create a context for one operator and block width N (1 <= N <= 512,
 * N <= n, odd N at most 256; other N return OPE_EUNSUPPORTED, and so does a plane of the
 * march axis holding 2 GiB or more of FP64 block rows, m0 m1 N 8 bytes in 3D,
 * m0 N 8 in 2D: the stencil addresses one plane through 32-bit offsets).  Copies V to the
 * device, allocates O(N^2) matrices and per-column state (the five n x N
 * workspace blocks in the precision's storage type follow on first use, or come
 * from ope_set_workspace), binds `stream` (a hipStream_t, or NULL), and checks
 * that H is SPD (Section 2.2's coercivity; OPE_ENOTSPD, see
 * ope_spectrum_bounds).
 * Steps 2-3 run as one-work-group Gauss-Jordan kernels for N <= 128 and as
 * Newton-Schulz inversions on the FP64 matrix cores for larger N.
 * precision is an ope_precision.  On error *ctx is set to NULL. */
ope_status ope_create(ope_ctx** ctx, const ope_op_desc* op, int64_t N, int32_t precision, void* stream);

/* Release the context and its device memory (synchronises its stream).  NULL is a no-op. */
ope_status ope_destroy(ope_ctx* ctx);

/* Static text for a status code. */
const char* ope_status_string(ope_status s);

/* Inner-solve policy for Step 1 (the paper does not fix one).  Column j of
 * H Y = U is solved by conjugate gradients warm-started at U Lam^{-1} until
 * |u_j - H y_j| <= eta |u_j|, with eta = max(eta_floor, eta_rel * res) and
 * res the outer residual of the current iterate; at most max_iter iterations.
 * Defaults: eta_rel = 0.1, or 0.25 while the multigrid preconditioner is on,
 * eta_floor = 1e-12 (1e-6 for OPE_MIXED), max_iter = 2000 (measured: Algorithm
 * 1 to residual 1e-8 on 64^3 and 96^3 well problems with N = 17 takes 1.5-1.7x
 * less time than with eta_rel = 1e-2, at a few more steps; with the
 * preconditioner 0.25 takes 1.15-1.45x less time than 0.1).  Once this has
 * been called, ope_set_multigrid no longer changes eta_rel. */
ope_status ope_set_inner(ope_ctx* ctx, double eta_rel, double eta_floor, int32_t max_iter);

/* Multigrid-preconditioned Step 1 (Step 1 of Section 4.1 leaves the solver
 * open).  enable = 1: the CG of every later step, solve and ope_source_solve
 * is preconditioned by one symmetric multigrid V-cycle per iteration (same
 * stopping rule on |u_j - H y_j|, same warm start): hierarchy by halving
 * every axis (m' = ceil(m/2), spacing doubled, potential V + shift averaged
 * over the children), linear prolongation P (weights 3/4, 1/4 per axis),
 * restriction P^T / 2^d, damped Jacobi (omega = 0.8) once before and once
 * after the coarse correction, the first level with at most 64 nodes solved
 * exactly with a dense inverse.  The V-cycle runs in the context's storage
 * type (FP64, or FP32 for OPE_MIXED, its dot products accumulated in FP64).
 * Measured on 64^3 well problems: about 4 preconditioned iterations per step
 * instead of about 66.  Unless ope_set_inner has been called, enabling sets
 * the inner factor eta_rel to 0.25 and disabling to 0.1.  Allocates two n x N blocks plus the coarse levels
 * (about 3/7 of a block); synchronises; enable = 0 frees them.  With the
 * preconditioner on, the host checks the CG's convergence after every
 * iteration (every 2 with graphs on; without the preconditioner every 4).  OPE_EUNSUPPORTED when a point's row has more than 256
 * 16-byte chunks (odd N > 256 in FP64); OPE_ENOTSPD if the coarsest operator
 * is not positive definite.  A problem with the preconditioner on runs its
 * CG on its own stream in batched steps (no shared launches). */
ope_status ope_set_multigrid(ope_ctx* ctx, int32_t enable);
/* Recycled warm start of Step 1 (Step 1 of Section 4.1 leaves the solver
 * open; this changes only where the inner CG starts).  enable = 1: the CG of
 * every later step solves for the correction d = Y - U Lam^{-1}, starting from
 * the previous step's converged correction instead of zero, i.e. from
 * Y0 = U Lam^{-1} + d_prev with r0 = -R Lam^{-1} - H d_prev (same stopping rule
 * on |u_j - H y_j|); after the CG, Y = U Lam^{-1} + d and H d is kept for the
 * next warm start.  Between steps the slowly changing residual leaves the
 * previous correction a close guess, so fewer inner iterations run (measured
 * on well problems: about half with the multigrid preconditioner).  The outer
 * convergence per step can be slower: at 64^3, N = 128 a solve to residual
 * 1e-8 took 654 s with it against 592 s without (more, cheaper steps).
 * ope_solve and ope_solve_ex start every solve with d = 0;
 * successive ope_step calls carry it.  FP64 contexts without a mass operator,
 * outside a batch (else OPE_EUNSUPPORTED); turns CG graph chunks off; allocates
 * two n x N blocks (enable = 0 frees them); synchronises. */
ope_status ope_set_recycle(ope_ctx* ctx, int32_t enable);

/* Levels of the hierarchy (0 when off) and nodes of its coarsest level
 * (host outputs, nullable). */
ope_status ope_mg_info(const ope_ctx* ctx, int32_t* levels, int64_t* coarsest_nodes);
/* One V-cycle Z = B R on n x N device blocks in the context's storage type
 * (the preconditioner alone; R and Z distinct and 16-byte aligned).
 * Synchronises.  OPE_EINVAL when the preconditioner is off. */
ope_status ope_mg_vcycle(ope_ctx* ctx, const void* R, void* Z);

/* --- Hot-path building blocks (each is one row of the step) -------------- */

/* Y = H X for n x N device blocks X, Y (Step 1 operator; a(u,v) of Section
 * 2.2), in the context's storage type (FP64, or FP32 for OPE_MIXED).  X and Y
 * must not overlap. */
ope_status ope_apply_h(ope_ctx* ctx, const void* X, void* Y);

/* Step 1 (OPE_FP64 contexts): Y ~= G U = H^{-1} U column by column by conjugate gradients.  Y0 is
 * an optional device n x N warm start (NULL = zero); Y may equal Y0.  Stops
 * column j when |u_j - H y_j| <= tol |u_j| (recursively updated residual) or
 * after max_iter iterations (then returns OPE_ECG_MAXIT with Y written).
 * *iterations (host, nullable) receives the iteration count. */
ope_status ope_source_solve(ope_ctx* ctx, const double* U, double* Y, const double* Y0,
                            double tol, int32_t max_iter, int32_t* iterations);

/* Inner matrix out = A^T B (na x nb, row-major, device) over `rows` grid
 * rows, for row-major device blocks A (leading dimension lda >= na) and B
 * (ldb >= nb): the products <U,U>, <U,HU>, <U,GU>, <GU,GU> of Steps 2-3.
 * FP64 on the matrix cores; deterministic summation order. 1 <= na, nb <= 512. */
ope_status ope_gram(ope_ctx* ctx, const double* A, int64_t lda, int64_t na,
                    const double* B, int64_t ldb, int64_t nb, int64_t rows, double* out);

/* ope_gram without a context and without any allocation, for callers that
 * cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid allocation).  Same operation, layouts and
 * kernels as ope_gram, enqueued on `stream` (a hipStream_t, NULL = default
 * stream); the split-K partial sums go to a fixed 4 MiB device array of the
 * library (one per GPU, kept until the process ends), so na, nb <= 128
 * (OPE_EINVAL beyond) and rows >= 1.  Calls that overlap on one GPU share that
 * array and race: serialise them (one stream, or events).  The summation order
 * may differ from ope_gram's (a different split of the rows). */
ope_status ope_gram_noalloc(const double* A, int64_t lda, int64_t na, const double* B, int64_t ldb, int64_t nb,
                            int64_t rows, double* out, void* stream);

/* Steps 2-3 (Section 4.1) for the context's N, in FP64, on the device (OPE_FP64 contexts):
 * given S_b = <U, Y> and T = <Y, Y> (N x N device), forms
 *   M = I + tau/2 (S_a - S_b) + tau^2/4 (T - S_a S_b),  S_a = S_b^T,
 * B = M^{-1}, A = 2/tau (I - B) + S_b B, and Z = [I - tau A ; tau B]
 * (2N x N), so that Step 4 is U' = [U, Y] Z.  M reduces to the paper's
 * Step-2 matrix when S is symmetric.  Outputs Z, A, B are device pointers
 * (A, B nullable).  OPE_EPIVOT if elimination meets a pivot <= 1e-300. */
ope_status ope_small_solve(ope_ctx* ctx, const double* S_b, const double* T, double tau,
                           double* Z, double* A, double* B);

/* Step 4: U <- U Z_1 + Y Z_2 in place, Z = [Z_1; Z_2] (2N x N device, as
 * produced by ope_small_solve).  U and Y are n x N FP64 device blocks (OPE_FP64 contexts). */
ope_status ope_update(ope_ctx* ctx, double* U, const double* Y, const double* Z);

/* E(U) = 1/2 tr(U^T H U) (eq. (2.3)) into *energy (host), accumulated in FP64;
 * U in the context's storage type.  Synchronises. */
ope_status ope_energy(ope_ctx* ctx, const void* U, double* energy);

/* FP64 checks of an iterate (host outputs, each nullable):
 *   *residual = |H U - U Lam|_F / |Lam|_F with Lam = U^T H U,
 *   ritz[0..N) = eigenvalues of Lam, ascending (device Jacobi, FP64),
 *   *drift = |U^T U - I|_F.  Synchronises. */
ope_status ope_residual(ope_ctx* ctx, const void* U, double* residual, double* ritz, double* drift);

/* One step of scheme (4.1) in place on the device block U (n x N, in the
 * context's storage type): Steps 1-4 with the inner policy of ope_set_inner.  If info is non-NULL it
 * receives the diagnostics of the iterate entering the step (host struct).
 * On OPE_ENONFINITE or OPE_EPIVOT, U is left unchanged. */
ope_status ope_step(ope_ctx* ctx, void* U, double tau, ope_step_info* info);

/* Algorithm 1 at fixed step tau: repeat ope_step until the residual of the
 * current iterate is <= res_tol or max_steps steps were taken (or, for
 * OPE_MIXED, the residual stalls at the FP32 floor).  info nullable. */
ope_status ope_solve(ope_ctx* ctx, void* U, double tau, double res_tol, int32_t max_steps,
                     ope_solve_info* info);

/* Options of ope_solve_ex: Algorithm 1 (Section 4.1) with the step tau_n
 * chosen in [tau_min, tau_max] at every iteration.  The paper leaves the
 * choice open; the rule here follows Theorem 4.2 (the energy decays for steps
 * below a threshold): a step whose energy E(U') = 1/2 tr(U'^T H U') exceeds
 * E(U) + 1e-13 |E(U)| is redone from U with tau <- max(tau_min, shrink tau)
 * (a step at tau_min is always kept), and after an accepted step the next
 * one starts at min(tau_max, grow tau).  tau_min = tau_max is a fixed step.
 * Stops, checked before every iteration in this order: the residual
 * |HU - U Lam|_F / |Lam|_F <= res_tol (negative: unused); the energy rule
 * (energy_tol negative: unused): with energy_ref NaN, Algorithm 1's
 * err_E = |E(U^{n+1}) - E(U^n)| / |E(U^n)| <= energy_tol (err_E^0 = |E(U^0)|),
 * else the relative energy error of the experiments (Section 5)
 * (E(U^n) - energy_ref) / |energy_ref| <= energy_tol; or max_steps accepted
 * steps (OPE_MIXED also stops when the residual stalls, as ope_solve). */
typedef struct {
  double tau;         /* first step, tau_min <= tau <= tau_max */
  double tau_min;     /* > 0 */
  double tau_max;     /* finite */
  double grow;        /* >= 1 */
  double shrink;      /* in (0, 1) */
  double res_tol;
  double energy_tol;
  double energy_ref;  /* NaN or non-zero */
  int32_t max_steps;  /* >= 0 */
  int32_t reserved;   /* 0 */
} ope_solve_opts;

/* Algorithm 1 with the options above, in place on U (device block in the
 * context's storage type).  An adaptive run (tau_min < tau_max) keeps a copy
 * of U in a library-owned n x N block (allocated on first use).  info
 * (nullable) receives the counts, the final residual, energy and drift, the
 * rejected steps and the next step.  EINVAL on inconsistent options;
 * EUNSUPPORTED with a preconditioner set.  OPE_ECG_MAXIT of single steps is
 * tolerated (the steps are kept). */
ope_status ope_solve_ex(ope_ctx* ctx, void* U, const ope_solve_opts* opts, ope_solve_info* info);

/* Elementwise precision change of `count` values on the context's stream:
 * to_double != 0 converts FP32 src to FP64 dst, else FP64 src to FP32 dst
 * (round to nearest).  Used to hand a mixed-precision iterate to an FP64
 * context for the finishing steps.  src and dst must not overlap. */
ope_status ope_convert(ope_ctx* ctx, const void* src, void* dst, int64_t count, int32_t to_double);

/* Mixed-precision building blocks on FP32 device blocks (kind: 0 = FP64
 * accumulation of FP32 inputs, 1 = FP32 matrix cores, 2 = BF16 inputs with FP32
 * accumulation):
 *   ope_gram_f32: out (na x nb, FP64, device) = A^T B over `rows` rows;
 *   ope_rowmm_f32 (kind 1 or 2): Out = cbeta Cm + ascale (X0 M0 + X1 M1) for
 *     the context's n x N blocks and N x N FP32 matrices (X1/M1 and Cm
 *     nullable); Out may equal X0 or Cm. */
ope_status ope_gram_f32(ope_ctx* ctx, int32_t kind, const float* A, int64_t lda, int64_t na, const float* B,
                        int64_t ldb, int64_t nb, int64_t rows, double* out);
ope_status ope_rowmm_f32(ope_ctx* ctx, int32_t kind, const float* X0, const float* M0, const float* X1,
                         const float* M1, const float* Cm, double cbeta, double ascale, float* Out);

/* --- Operator checks, the generalized problem, workspace, device scalars -- */

/* Estimates of the extreme eigenvalues of H (host outputs, nullable): the
 * extreme Ritz values of a Lanczos run on one seeded pseudo-random vector
 * (FP64, on the device; run once per context, at ope_create when the closed-form
 * bound lambda_min(c (-Lap_h)) + min(V + shift) does not already prove H SPD,
 * else on the first call).  Ritz values lie inside the spectrum, so *lmin is
 * an upper estimate of lambda_min and *lmax a lower estimate of lambda_max;
 * with them the fixed-point stability limit of the step is about
 * 2 / (1/lambda_min - 1/lambda_max).  ope_create returns OPE_ENOTSPD when this
 * run finds a Ritz value <= 0 (then H certainly has an eigenvalue <= 0, and
 * Section 2.2's coercivity fails); an eigenvalue <= 0 whose eigenvector is
 * orthogonal to the Krylov space of the start vector would go unseen. */
ope_status ope_spectrum_bounds(ope_ctx* ctx, double* lmin, double* lmax);

/* The generalized problem H u = lambda M u of the paper's finite-element
 * setting (Section 5: coefficient blocks with the inner product
 * <U, V> = U^T M V and Step 1 solving H (GU) = M U), with the finite-difference
 * mass operator M = diag(d) + sum_a mu_a (S_a + S_a^T), S_a the shift to the
 * next grid node along axis a (zero past the boundary).  d: HOST array of n
 * values, copied; mu: HOST array of dim coefficients.  From then on every
 * inner matrix of Steps 2-4 and of the checks is taken in the M product:
 * C = U^T M U (drift |C - I|_F), Lam = U^T H U (energy 1/2 tr Lam, Ritz values
 * the eigenvalues of Lam, exact for C = I), residual |H U - M U Lam|_F / |Lam|_F,
 * Step 1 solves H Y = M U (CG tolerance relative to |M u_j|), S_b = (MU)^T Y,
 * T = Y^T (MY); Step 4 is unchanged.  U must be M-orthonormal
 * (ope_orthonormalize).  OPE_ENOTSPD unless d_p > 2 sum_a |mu_a| for every p
 * (strict diagonal dominance, a sufficient condition for SPD); EUNSUPPORTED for
 * OPE_MIXED contexts, N > 256 or a preconditioner set.  d = NULL removes M. */
ope_status ope_set_mass(ope_ctx* ctx, const double* d, const double* mu);
/* Y = M X for n x N FP64 device blocks (the mass operator must be set). */
ope_status ope_apply_mass(ope_ctx* ctx, const double* X, double* Y);

/* U <- U R^{-1} in place (OPE_FP64), R the upper Cholesky factor of
 * C = <U, U> (R^T R = C, positive diagonal; the M product when a mass operator
 * is set): an orthonormal start block with the same column span.  OPE_ENOTSPD
 * (U unchanged) when C is not numerically positive definite.  Synchronises. */
ope_status ope_orthonormalize(ope_ctx* ctx, double* U);

/* Size in bytes of the context's workspace of five n x N blocks in its storage
 * type, each rounded up to 256 bytes. */
ope_status ope_workspace_size(const ope_ctx* ctx, size_t* bytes);
/* Give the context caller-owned device memory (>= ope_workspace_size bytes,
 * 256-byte aligned; for instance a torch tensor) for those blocks; the library
 * frees its own copy if it had one and never allocates them again until
 * dptr = NULL hands the workspace back to the library (allocated on next use).
 * The memory must stay valid, and unused by the caller, while the context uses
 * it.  Synchronises the context's stream.  Without this call the library
 * allocates the blocks on first use. */
ope_status ope_set_workspace(ope_ctx* ctx, void* dptr, size_t bytes);

/* Device-scalar forms of ope_energy / ope_residual: enqueue the same
 * evaluation and write E(U), the residual and the drift to DEVICE addresses
 * (each nullable except that one of residual/drift is needed), without
 * synchronising the stream (N <= 128; larger N synchronise inside the
 * Newton-Schulz inversion of Lam). */
ope_status ope_energy_d(ope_ctx* ctx, const void* U, double* d_energy);
ope_status ope_residual_d(ope_ctx* ctx, const void* U, double* d_residual, double* d_drift);

/* ope_step / ope_energy / ope_residual for a block with leading dimension
 * ldu >= N (row p at U + p ldu): ldu = N is the plain call; otherwise the block
 * is copied into a packed library-owned staging block (allocated on first
 * use), processed there, and for ope_step_ld copied back (two extra block
 * copies; ope_step_ld synchronises). */
ope_status ope_step_ld(ope_ctx* ctx, void* U, int64_t ldu, double tau, ope_step_info* info);
ope_status ope_energy_ld(ope_ctx* ctx, const void* U, int64_t ldu, double* energy);
ope_status ope_residual_ld(ope_ctx* ctx, const void* U, int64_t ldu, double* residual, double* ritz, double* drift);

/* --- Learned preconditioner --------------------------------------------
 * Gradient form of Step 1: with R = HU - U Lam, G U = (U - H^{-1} R) Lam^{-1}.
 * The learned form replaces H^{-1} R column by column by a small 3D conv net,
 *   P(r) = |r| h^2 f(r / |r|, h^2 (V + shift)),
 * f: four bias-free 3x3x3 cross-correlations with zero padding, channels
 * 2 -> 16 -> 16 -> 16 -> 1, ReLU after the first three, on BF16 matrix cores
 * with FP32 accumulation (activations stored in BF16).  Weights are FP32
 * masters (BF16 copies feed the matrix cores): OPE_NET_PARAMS values in the
 * order W1[27][2][16], W2[27][16][16], W3[27][16][16], W4[27][16][1], each
 * [tap][in][out] with taps (dz, dy, dx), dx fastest, each in (-1, 0, 1).
 * Training losses of a sample (x = r/|r|, target t = H^{-1} r / (|r| h^2),
 * A = h^2 H), averaged over the batch:
 *   OPE_NET_LOSS_ENERGY    (f - t)^T A (f - t) / (x . t)   the squared H-norm
 *                          error of P r relative to H^{-1} r;
 *   OPE_NET_LOSS_RESIDUAL  |A f - x|^2 / |x|^2   the residual norm of the
 *                          preconditioned direction (no target needed);
 *   OPE_NET_LOSS_BOTH      their sum.
 * Each is 1 for the zero network.  3D grids with equal spacings only.
 * Sample blocks X, T, F are device FP32 [sample][z][y][x] (n values each).
 * The learned step keeps Steps 2-4 (Section 4.1), so orthogonality holds for
 * any weights (Theorem 4.1's argument), and P(0) = 0 keeps eigenbases fixed. */
#define OPE_NET_PARAMS 15120
#define OPE_NET_LOSS_ENERGY 0
#define OPE_NET_LOSS_RESIDUAL 1
#define OPE_NET_LOSS_BOTH 2
typedef struct ope_net ope_net;

/* Network on ctx's grid with activations for up to max_batch (1..4096)
 * samples; its bound second input channel is ctx's h^2 (V + shift).  Weights
 * start at zero.  EUNSUPPORTED for 2D grids or unequal spacings.  Destroy the
 * network before its context. */
ope_status ope_net_create(ope_ctx* ctx, int64_t max_batch, ope_net** net);
ope_status ope_net_destroy(ope_net* net);
/* FP32 weights from / to a HOST array of OPE_NET_PARAMS values (set resets the Adam state). */
ope_status ope_net_set_weights(ope_net* net, const float* w);
ope_status ope_net_get_weights(ope_net* net, float* w);
/* Training loss of ope_net_grad / ope_net_train_step (OPE_NET_LOSS_*; default energy). */
ope_status ope_net_set_loss(ope_net* net, int32_t kind);
/* The bound second input channel h^2 (V + shift) into V2 (device, n FP32). */
ope_status ope_net_potential(ope_net* net, float* V2);
/* F = f(X) for 1 <= B <= max_batch samples.  V2: the second input channel
 * (device, n FP32, shared by the batch), NULL for the bound one. */
ope_status ope_net_forward(ope_net* net, const float* X, const float* V2, int64_t B, float* F);
/* Batch loss into *loss (host, nullable) and its gradient into grad (HOST
 * array of OPE_NET_PARAMS, nullable).  T may be NULL for the residual loss
 * only.
 * ENONFINITE if the loss is not finite. */
ope_status ope_net_grad(ope_net* net, const float* X, const float* V2, const float* T, int64_t B,
                        double* loss, float* grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with
 * learning rate lr > 0; *loss (host, nullable) receives the loss before the step. */
ope_status ope_net_train_step(ope_net* net, const float* X, const float* V2, const float* T, int64_t B,
                              double lr, double* loss);
/* One Adam step (as ope_net_train_step) with a caller-provided gradient
 * (HOST array of OPE_NET_PARAMS values), for callers that form the gradient
 * elsewhere, for instance summed over several processes' ope_net_grad
 * results.  lr > 0. */
ope_status ope_net_apply_grad(ope_net* net, const float* grad, double lr);
/* Training samples from point-major FP64 device blocks R (residual columns)
 * and S = H^{-1} R (leading dimension ld, columns 0..B-1, B <= the context's
 * N): X[b] = r_b / |r_b|, T[b] = s_b / (|r_b| h^2); zero columns give zeros. */
ope_status ope_net_samples(ope_net* net, const double* R, const double* S, int64_t ld, int64_t B,
                           float* X, float* T);

/* Use `net` (created on this context, max_batch >= N) for ope_step_learned
 * and ope_solve, or NULL to go back to plain steps.  OPE_FP64 contexts only.
 * judge = 1: the plain step judges every learned iterate and replaces it when
 * rejected (below); judge = 0: learned iterates are always kept (for study). */
ope_status ope_set_preconditioner(ope_ctx* ctx, ope_net* net, int32_t judge);
/* One learned step in place on U: Y = (U - P(R)) Lam^{-1}, then Steps 2-4.
 * With the judge on, the learned iterate is kept only if its energy is not
 * above the current one (up to 1e-13 relative) and its residual
 * |HU - U Lam|_F / |Lam|_F is not above the current one; otherwise U is
 * restored and one plain step (ope_step) is taken.  *accepted (host,
 * nullable) = 1 if the learned iterate was kept.  info as for ope_step (the
 * input U's energy, residual and drift; inner_iterations 0 when accepted).
 * EINVAL if no network is set. */
ope_status ope_step_learned(ope_ctx* ctx, void* U, double tau, ope_step_info* info, int32_t* accepted);

/* --- Batched form ----------------------------------------------------------
 * Many independent problems (each its own grid, potential and N) stepped
 * together.  Every problem gets its own context and a private stream (default
 * priority); a batch step enqueues the pre-phase of every problem, then rounds
 * of Step-1 CG chunks (two in flight per problem; graph replays when graphs
 * are on) in which each problem drops out as soon as its own columns have
 * converged, then Steps 2-4 of every problem, so the problems' kernels overlap
 * on the GPU.  Each problem's result is exactly that
 * of ope_step on its own context.  The batch is ordered after earlier work on
 * `stream` (NULL: the default stream) and later work on it waits for the batch. */
typedef struct ope_batch ope_batch;

/* count (1..4096) problems: ops[i] (as for ope_create) with block width N[i],
 * all in one precision.  On error *batch is NULL. */
ope_status ope_batch_create(ope_batch** batch, const ope_op_desc* ops, const int64_t* N, int32_t count,
                            int32_t precision, void* stream);
ope_status ope_batch_destroy(ope_batch* batch);
/* The context of problem i (owned by the batch): for its inner policy, sweep
 * shape, residual and energy calls. */
ope_status ope_batch_context(ope_batch* batch, int32_t i, ope_ctx** ctx);
/* One step of every problem; U[i] is problem i's device block (in place).
 * info (host, count entries, nullable) as for ope_step, status per problem;
 * returns the first non-OK status, else OPE_OK. */
ope_status ope_batch_step(ope_batch* batch, void* const* U, double tau, ope_step_info* info);
/* Algorithm 1 for every problem in lock-step rounds (as ope_solve; no stall
 * test and no learned steps).  info: count entries, nullable. */
ope_status ope_batch_solve(ope_batch* batch, void* const* U, double tau, double res_tol, int32_t max_steps,
                           ope_solve_info* info);
/* shared = 1: Step 1's CG sweeps and column reductions of all
 * problems whose column sums fit one work-group (at most 128 columns and
 * 2^15 partial values) run as one launch per phase and class of problems
 * (storage type, vector width, passes per plane, split x lines, line tiles)
 * on a batch stream, each launch's work-groups spread over (problem, tile)
 * work items of every problem's own sweep shape, each problem over all XCDs; same kernels and summation order as the per-problem launches,
 * so the results are identical.  shared = 0 (default): every problem's CG
 * runs on its own stream.  Measured: on the 64-problem workload (grid edges
 * 24..48, N 16..128) per-problem launches are 4-8% faster; on a batch of
 * small problems alone shared launches are faster (2.2x for sixteen 24^3,
 * N = 16 problems), on a batch of large ones slightly slower. */
ope_status ope_batch_set_shared(ope_batch* batch, int32_t shared);
/* Graph-captured batched step: one HIP graph holding a whole step of every
 * problem (residual and warm start on the problems' streams, then exactly
 * `cg_iterations` iterations of Step 1's CG, then Steps 2-4 on the problems'
 * streams), so a step costs one graph launch and no host decision.  The CG
 * follows the batch's launch mode at capture (ope_batch_set_shared): shared
 * launches for the problems that fit them, the problems' own launches on
 * their own streams otherwise.  Columns that converge earlier stop in place
 * (their kernels skip them), so the result is identical to ope_batch_step
 * whenever every problem's CG converges within cg_iterations; otherwise the
 * step is taken with the CG state after cg_iterations and the problem's
 * status is OPE_ECG_MAXIT.  Mixed-precision problems keep Step 4's
 * device-side drift check; the host-decided re-normalisation before a step
 * (driven by the previous step's drift) is not part of the graph.
 * U[i] (device blocks) are fixed at capture: every replay steps the same
 * buffers.  The graph also freezes tau and every problem's settings (inner
 * tolerances, sweep shapes, mass product): capture again after changing any;
 * ope_batch_autotune drops the graph.  Requires N[i] <= 128 (the
 * one-work-group small solves), no kernel timing, cg_iterations even and
 * >= 2; else OPE_EUNSUPPORTED / OPE_EINVAL.  Capture synchronises the device and allocates the graph's own
 * job tables and flags (once per batch); replays may interleave with eager
 * batched steps. */
ope_status ope_batch_capture(ope_batch* batch, void* const* U, double tau, int32_t cg_iterations);
/* Replays the captured step on the batch's stream.  info (host, count
 * entries, nullable): when given, waits for the step and fills it as
 * ope_batch_step does (inner_iterations = the CG iterations each problem
 * counted before converging); returns the first non-OK status.  With info
 * NULL it returns after the launch.  EINVAL if nothing is captured. */
ope_status ope_batch_replay(ope_batch* batch, ope_step_info* info);
/* Autotuner: for every bucket of problems (grid edges and vector-column count
 * in steps of 8) time short CG runs of the first problem over the sweep shapes
 * (passes per plane 1/2 or the two-, four- and eight-line tiles, work-group order,
 * non-temporal stores, column chunking, and the automatic march-chunk count
 * times 1/2, 1, 3/2 or 2) and give every problem of the bucket the fastest
 * (FP64 and FP32 contexts alike).  *tuned (nullable) = number of buckets.
 * Synchronises; uses a temporary n x N block per tuned bucket. */
ope_status ope_batch_autotune(ope_batch* batch, int32_t* tuned);
/* The same search for one context.  The shape changes only the summation
 * order of the CG dot products.  Synchronises; an FP64 context uses a
 * temporary n x N block (an FP32 one its own CG buffers). */
ope_status ope_autotune(ope_ctx* ctx);

/* Step 1's CG runs in chunks of 4 iterations between host convergence checks
 * (preconditioned: 1, or 2 with graphs on);
 * with graphs on each chunk is one replay of a HIP graph captured once per
 * context (on a private stream, replayed on the context's stream), with the
 * same kernels and results as eager launches.  Off by default: eager launches
 * measured about 2% faster (Algorithm 1 to 1e-8 at 64^3 and 96^3, N = 17).
 * enable 0/1. */
ope_status ope_set_graphs(ope_ctx* ctx, int32_t enable);

/* --- Launch shape of the stencil / CG sweeps (tuning) --------------------
 * The sweeps march along the slowest grid axis; a work-group covers q passes
 * of 256/c grid points of one x segment, c the vector columns of its column
 * chunk (q in {1, 2, 4}; more passes per plane mean fewer x segments but
 * more registers), and the march axis is cut
 * into march_chunks ranges (0 = automatic: at least 512 work-groups).  The
 * default shape is q_max = 2, automatic chunks, OPE_SWEEP_CHUNK_MAJOR, plus
 * OPE_SWEEP_LINES8 on 3D grids and OPE_SWEEP_NONTEMPORAL when five n x N
 * blocks of the storage type exceed 256 MiB.
 * q_max = 0 lets the library choose.  flags: OPE_SWEEP_CHUNK_MAJOR puts the
 * work-groups of one column chunk next to each other (so one XCD streams one
 * chunk of every side line) instead of those of one side line;
 * OPE_SWEEP_NONTEMPORAL writes the swept outputs with non-temporal stores;
 * OPE_SWEEP_NARROW gives every work-group an 8-vector column chunk (by
 * default a work-group takes rows of at most 32 vector columns whole, rows
 * of up to 64 in chunks of the widest of 32, 16 and 8 vectors that divides
 * them, and wider rows in chunks of 8);
 * OPE_SWEEP_LINES (3D grids) gives a work-group two adjacent side lines, one
 * per pass over an x segment of 256/c points (q is then 2), OPE_SWEEP_LINES4
 * four, two per pass over segments of half that, OPE_SWEEP_LINES8 eight, four
 * per pass over segments of a quarter (when a pass holds at least 16 points;
 * else as OPE_SWEEP_LINES4); the lines take their inner side neighbours from
 * the staged plane, and only the outer ones load side rows.
 * Results do not depend on the shape beyond the summation order of the CG dot
 * products.  Synchronises; on OPE_EINVAL the previous shape stays. */
#define OPE_SWEEP_CHUNK_MAJOR 1
#define OPE_SWEEP_NONTEMPORAL 2
#define OPE_SWEEP_NARROW 4
#define OPE_SWEEP_LINES 8
#define OPE_SWEEP_LINES4 16
#define OPE_SWEEP_LINES8 32
ope_status ope_set_sweep_shape(ope_ctx* ctx, int32_t q_max, int32_t march_chunks, int32_t flags);

/* The shape in use (outputs nullable, host). */
ope_status ope_get_sweep_shape(const ope_ctx* ctx, int32_t* q, int32_t* march_chunks, int32_t* workgroups);

/* --- Kernel timing (measurement support) ------------------------------ */

typedef enum {
  OPE_KERNEL_STENCIL = 0,   /* H X (stencil SpMM) */
  OPE_KERNEL_CG_SWEEP_A = 1,/* CG sweep A: p^T H p with p formed on the fly */
  OPE_KERNEL_CG_SWEEP_B = 2,/* CG sweep B, both forms: r update with H p and r^T r; odd iterations also y */
  OPE_KERNEL_GRAM = 3,      /* split-K MFMA inner matrices (without their reduction) */
  OPE_KERNEL_ROWMM = 4,     /* MFMA row-block products (residual, warm start, Step 4) */
  OPE_KERNEL_SMALL = 5,     /* one-work-group FP64 small solves */
  OPE_KERNEL_CG_SWEEP_B_Y = 6,/* CG sweep B of odd iterations only (with the paired y update) */
  OPE_KERNEL_CG_REDUCE = 7, /* the two fixed-order column reductions of every CG iteration */
  OPE_KERNEL_MG = 8,        /* one multigrid V-cycle of the preconditioned Step 1 (all its launches) */
  OPE_KERNEL_MG_POST = 9,   /* its finest-level post-smoothing with the PCG dot products (one launch) */
  OPE_KERNEL_COUNT = 10
} ope_kernel_id;

typedef struct {
  int64_t launches;         /* launches timed */
  double total_ms;          /* summed device time between the events around each launch */
} ope_kernel_time;

/* Start timing every launch of `kernel` on the context's stream with a pair of
 * HIP events (until ope_profile_end).  Adds two event records per launch. */
ope_status ope_profile_begin(ope_ctx* ctx, int32_t kernel);

/* Stop timing; synchronises the stream and writes the totals to *out (host). */
ope_status ope_profile_end(ope_ctx* ctx, ope_kernel_time* out);

/* ope_profile_end that also writes, for the first `cap` timed launches in
 * order, the launch's tag (the index of the CG iteration it belongs to, 0 at
 * the start of every Step 1; -1 for launches outside a CG iteration) and its
 * device time in ms (host arrays of `cap` entries; nullable when cap = 0).  A
 * CG iteration past the convergence of every column does no sweep work (or,
 * for sweep B of an odd iteration, only the pending y term), so the tags let
 * a caller average over the iterations that ran (ope_step_info's
 * inner_iterations of the step). */
ope_status ope_profile_end_launches(ope_ctx* ctx, ope_kernel_time* out, int32_t* tags, double* ms, int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* OPE_H */
