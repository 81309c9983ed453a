// Internal declarations of the gfx950 eigensolver-step library.
//
// Data layout in HBM (all FP64):
//   orbital blocks   n x N row-major (point-major): the N orbitals of one grid
//                    point are one contiguous row, so a wavefront reading 64
//                    consecutive lanes touches whole rows (fully coalesced);
//                    stencil neighbours sit at +-N, +-m0*N, +-m0*m1*N elements.
//   inner matrices   N x N row-major.
//   partials         [work-group][column] rows, reduced in a fixed order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "ope.h"

#define OPE_WG 256                  // threads per work-group of the streaming kernels

// Arithmetic of a dense contraction (see k_mfma.hip).
enum { MK_F64 = 0, MK_F32 = 1, MK_BF16 = 2 };
#define OPE_MAX_N_SMALL 512         // largest block width N
#define OPE_MAX_N_ONE_WG 128        // largest N of the one-work-group FP64 small solves

// Default inner tolerance factor eta_rel of Step 1 (|u_j - H y_j| <= eta_rel *
// res |u_j|): plain CG, and CG with the multigrid preconditioner, whose few
// iterations per step make a looser factor pay (measured on 64^3 and 96^3
// well problems: N = 17 to residual 1e-8 in 0.46 / 1.08 s instead of
// 0.53 / 1.58 s at 0.1, and at N = 128 about 4% less time per e-fold of the
// late residual).
constexpr double ETA_REL_CG = 0.1;
constexpr double ETA_REL_MG = 0.25;

struct OpeGrid {
  int dim;
  uint32_t m0, m1, m2;              // interior nodes per axis (m2 = 1 in 2D)
  uint32_t s1, s2;                  // point strides of the y and z neighbours (m0, m0*m1)
  double cx, cy, cz;                // kinetic / h_a^2 per axis (cz = 0 in 2D)
};

// Work decomposition of the plane-marching stencil sweeps (see k_stencil.hip).
struct MarchShape {
  uint32_t ncv;       // vector columns per work-group (column chunk)
  uint32_t pp;        // grid points per pass (OPE_WG / ncv)
  uint32_t q;         // passes per plane (compile-time variant 1, 2, 4 or 8)
  uint32_t xseg;      // x points per segment (q * pp)
  uint32_t nxs;       // x segments
  uint32_t cc;        // column chunks
  uint32_t lines;     // side lines (m1 in 3D, 1 in 2D)
  uint32_t ly;        // side lines per work-group: 1, or q lpp (lpp lines per pass, x segment = pp / lpp)
  uint32_t lpp;       // side lines per pass of a line tile (1 or 2)
  uint32_t lgroups;   // groups of ly side lines
  uint32_t mlen;      // planes along the march axis (m2 in 3D, m1 in 2D)
  uint32_t mc;        // march chunks
  uint32_t mchunk;    // planes per march chunk
  uint32_t side_stride, march_stride;  // point strides of the side and march axes
  uint32_t has_side;
  uint32_t order;     // 0: work-groups of one side line adjacent; 1: of one column chunk adjacent
  uint32_t nt;        // 1: streamed outputs bypass the caches (non-temporal stores)
  double cm, cs;      // stencil coefficients of the march and side axes
};

// State of a device-side Newton-Schulz inversion (N > OPE_MAX_N_ONE_WG).
struct NsState {
  int32_t done;       // 1 converged (its last update still runs), 2 failed
  int32_t upd_skip;   // the update of the current iteration is skipped
  int32_t cur;        // buffer holding the latest iterate
  int32_t iters;
  double res;         // |I - M X_k|_F of the last checked iterate
};

// Device-resident scalars of one context (written by kernels, read by kernels
// and, after a synchronisation, by the host).
struct OpeScalars {
  double energy;      // 1/2 tr Lam
  double residual;    // |HU - U Lam|_F / |Lam|_F
  double drift;       // |U^T U - I|_F
  double lam_fro;     // |Lam|_F
  double eta;         // inner tolerance of this step
  int32_t err;        // ope_status of the device side of the step (0 = ok)
  int32_t cg_iters;   // CG iterations that had at least one active column
  int32_t renorm;     // mixed precision: 1 when the drift check after the update re-normalises U
  int32_t renorms;    // re-normalisations since the context was created
  double drift_after; // mixed precision: |U^T U - I|_F of the updated iterate before the check's correction
};

// predication bits of the row-block products and the predicated copy
enum { ROWMM_IF_OK = 1, ROWMM_IF_RENORM = 2 };

// One level of the multigrid preconditioner (k_mg.hip).  Level 0 is the
// operator itself (its B and E are the caller's residual and result).
#define OPE_MG_MAX_LEVELS 16
struct MgLevel {
  uint32_t m0, m1, m2;          // nodes per axis (1 for absent axes)
  double cx, cy, cz;            // kinetic / h_a^2 on this level (0 for absent axes)
  int64_t n;
  double* diag;                 // diagonal of H on this level (level 0: the context's)
  double* wd;                   // omega / diag (the damped Jacobi factor)
  void *B, *E, *T;              // right-hand side, correction, scratch (n x N each, the context's
                                // storage type; level 0: T only)
};

struct ope_ctx {
  int device;
  hipStream_t stream;
  OpeGrid g;
  double h[3];                  // grid spacings (h[2] = h[1] in 2D)
  double kinetic;               // coefficient of -Lap in H
  int64_t n, N;
  int prec;                     // OPE_FP64 or OPE_MIXED
  int vw;                       // elements per 16-byte row chunk (fewer when N is not a multiple)
  // operator
  double* diag;                 // V + shift + 2 (cx + cy + cz), n values
  float* diag32;                // the same in FP32 (mixed precision)
  // n x N workspace blocks, FP64 (OPE_FP64) or FP32 (OPE_MIXED)
  void* HU;                     // H U, then R = HU - U Lam, then a CG direction buffer
                                // (mixed: finally the projection Y - U <U,Y>)
  void* Y;                      // Step-1 solution G U
  void* Rb[2];                  // CG residuals (double buffered)
  void* Pb;                     // second CG direction buffer (the first is HU)
  // N x N (and 2N x N) matrices, FP64
  double *C, *Lam, *Linv, *Sb, *T, *Z, *A, *B, *Wsm;
  // N > 128: Newton-Schulz workspace (iterates, M X, the matrix, a product), state
  double *ns_x[2], *ns_g, *ns_m, *ns_p, *ns_part;
  NsState* ns;
  NsState* hns;                 // pinned
  // FP32 copies used by the mixed-precision products
  float *Lam32, *Linv32, *Sb32, *Z32;
  // per-column CG state (alpha: 2N, one half per iteration parity)
  double *alpha, *beta, *rho, *target, *cnorm2, *rcol, *rho0;
  int32_t* active;
  // reductions
  double* part;                 // partial sums, part_cap doubles
  int64_t part_cap;
  double* stage;                // second-stage partial sums
  int64_t stage_cap;
  // scalars
  OpeScalars* sc;               // device
  OpeScalars* hsc;              // pinned host mirror
  int32_t* hactive;             // pinned host mirrors of active[] (two slots of N)
  hipEvent_t chunk_ev[2];       // marks each slot's copy
  double* hbuf;                 // pinned host scratch (N doubles)
  // policy
  double eta_rel, eta_floor;
  int32_t eta_user;             // ope_set_inner was called: the preconditioner keeps eta_rel
  // recycled Step-1 correction (ope_set_recycle): the CG runs on the correction
  // d = Y - U Lam^{-1} in Dr, started from the previous step's; HDr = H Dr
  int32_t recycle, have_d, in_batch;
  int32_t cg_on_d;              // the CG being run iterates on Dr (a recycled step's Step 1)
  void* Dr;
  void* HDr;
  int32_t max_iter;
  int32_t check_every;          // CG iterations between host convergence checks (even: graph chunks)
  double drift_seen;            // drift of the last iterate whose scalars reached the host
  double drift_tol;             // mixed precision: drift above which an updated block is re-normalised
  int64_t renorms;              // mixed precision: re-normalisations applied
  int use_graphs;               // replay CG chunks as captured graphs
  int graph_state;              // 0 not built, 1 built, -1 capture failed (eager launches)
  hipStream_t cap_stream;       // private stream used only for capturing
  hipGraphExec_t cg_graph[2];   // first chunk (iterations 0..K-1) and later chunks
  // launch shapes
  int stream_wgs;               // work-groups of the flat streaming kernels
  int stream_pts;               // grid points per flat streaming work-group
  MarchShape ms;                // plane-marching stencil sweeps
  // workspace of the five n x N blocks: library-owned (ws_own) or the caller's (ws_ext)
  void* ws_own;
  void* ws_ext;
  size_t ws_ext_bytes;
  // generalized problem H u = lambda M u: M = diag(mdiag) + sum_a mu_a (S_a + S_a^T) (FP64 only)
  int has_mass;
  double* mdiag;
  double mass_mu[3];
  // staging block for callers' blocks with a leading dimension other than N
  void* Upk;
  // Lanczos estimates of the extreme eigenvalues of H (set-up check)
  int lz_done;
  int lz_iters;
  double lz_min, lz_max;
  // learned form: network (not owned) and the saved iterate its judge restores
  ope_net* net;
  int net_judge;                // 1: the plain step judges each learned iterate and replaces it if rejected
  void* Ubak;
  OpeScalars* hsc2;             // pinned: scalars right after a learned update
  // multigrid-preconditioned Step 1 (ope_set_multigrid; FP64)
  int mg_on;
  int mg_levels;
  MgLevel mg[OPE_MG_MAX_LEVELS];
  double* mg_inv;               // coarsest level: dense inverse, row-major nc x nc
  void* mg_Z;                   // preconditioned residual z (n x N, the context's storage type)
  double* mg_part;              // partial rows of r^T z and r^T r (mg_rows x 2N)
  int64_t mg_rows;
  int64_t mg_rows_used;         // partial rows written by the last V-cycle with dots
  double* mg_dots;              // 2N: r^T z, r^T r
  void* mg_mem;                 // one allocation holding the level blocks
  // kernel timing (ope_profile_begin / ope_profile_end)
  int prof_kernel;              // kernel id being timed, -1 when off
  std::vector<hipEvent_t> prof_events;  // start/stop pairs, reused across sessions
  size_t prof_used;             // events recorded in this session
  std::vector<int32_t> prof_tags;  // per timed launch: the CG iteration index (-1 outside the CG)
  int32_t prof_tag;             // the tag of the launches being enqueued
};

// The conv-net preconditioner (see k_net.hip).  Activations BF16
// [sample][z][y][x][channel]; FP32 fields [sample][z][y][x].
struct ope_net {
  ope_ctx* ctx;                 // grid, stream and bound potential
  int64_t max_batch;
  int64_t n;
  uint32_t m0, m1, m2;
  double hh;                    // h^2
  double kin;                   // kinetic coefficient: h^2 H = kin (6 - neighbours) + h^2 (V + shift)
  int64_t adam_t;               // Adam steps taken
  int32_t loss_kind;            // OPE_NET_LOSS_ENERGY or OPE_NET_LOSS_RESIDUAL
  float *w, *adam_m, *adam_v, *grad;   // FP32 masters, moments, gradient (OPE_NET_PARAMS each)
  uint16_t* wpk;                // packed BF16 operands of the forward and transposed layers
  float* v2;                    // h^2 (V + shift), n values
  uint16_t *x, *a1, *a2, *a3, *g3, *g4;  // input pair, activations, gradients
  float* f;                     // network output
  float* e;                     // residual-norm loss: A f - x
  float* part;                  // weight-gradient partial rows
  double *stage, *lpart, *coef, *dloss, *colsq;
  double* hloss;                // pinned
};

// Brackets one launch with timing events when that kernel is being profiled.
struct ProfScope {
  ope_ctx* c;
  bool on;
  ProfScope(ope_ctx* ctx, int kernel);
  ~ProfScope();
};

// ---------------------------------------------------------------------------
// launchers (each enqueues on ctx->stream and returns hipSuccess or an error)
// ---------------------------------------------------------------------------
hipError_t launch_apply_h(ope_ctx* c, const void* X, void* Y);
// fills c->ms (0 = automatic); narrow = 1 keeps 8-vector column chunks for short rows;
// lines = 1 gives each work-group two side lines, one per pass; lines = 2 four,
// two per pass (3D only)
void march_shape(ope_ctx* c, int q_max, int mc_override, int order, int nt, int narrow, int lines = 0);
int64_t march_rows(const ope_ctx* c);              // partial rows written by the CG sweeps

// CG iteration halves (see k_stencil.hip)
// sweep A: p = r + beta p_old (p = r when first) written to pnew, p^T H p partials
hipError_t launch_cg_pap(ope_ctx* c, const void* r, const void* pold, void* pnew, int first);
// sweep B: rnew = r - alpha H p, rnew^T rnew partials; with y given (odd
// iterations) also y += alpha_prev pprev + alpha p
hipError_t launch_cg_update(ope_ctx* c, const void* r, const void* p, void* rnew, const double* alpha, void* y,
                            const void* pprev, const double* alpha_prev);
// y += alpha p (per column) on stream s: the deferred y term of a CG that
// stopped on an even iteration
hipError_t launch_y_flush(ope_ctx* c, hipStream_t s, void* y, const void* p, const double* alpha);
// y += x over an n x N FP64 block
hipError_t launch_add_block(ope_ctx* c, double* y, const double* x);
hipError_t launch_cg_setup_reduce(ope_ctx* c, int mode);

// multigrid preconditioner (k_mg.hip)
ope_status mg_build(ope_ctx* c);          // the hierarchy for the context's operator and N
void mg_free(ope_ctx* c);
// z = B r (one V-cycle) for the columns still active (all when active is
// NULL); with dots, also the partial rows of r^T z and r^T r into c->mg_part
hipError_t mg_vcycle(ope_ctx* c, const void* r, void* z, const int32_t* active, bool dots);
// PCG scalars from the reduced dots: start (rho = r^T z) and the beta update
hipError_t launch_pcg_start(ope_ctx* c);
hipError_t launch_pcg_beta(ope_ctx* c);

// column sums of partials: out[j] = sum_w part[w*ncols + j], fixed order
// (the CG modes write alpha, default c->alpha)
hipError_t launch_reduce_cols(ope_ctx* c, const double* part, int64_t nrows, int64_t ncols,
                              double* out, int mode, double* alpha = nullptr);
enum { RED_PLAIN = 0, RED_CG_ALPHA = 1, RED_CG_BETA = 2 };

// inner matrix out = A^T B over `rows` rows (partials into c->part, then reduced)
hipError_t launch_gram(ope_ctx* c, const double* A, int64_t lda, int na, const double* B,
                       int64_t ldb, int nb, int64_t rows, double* out);

// out = A^T B for a product the caller knows to be symmetric (U^T H U): up to 128
// columns only the MFMA blocks on and above the block diagonal are computed and
// mirrored, so out is exactly symmetric
hipError_t launch_gram_sym(ope_ctx* c, const double* A, int64_t lda, const double* B, int64_t ldb, int n,
                           int64_t rows, double* out);

// row-block products: Out = cbeta*Cm + ascale*(X0*M0 + X1*M1); optional per-column sums of Out^2
// into c->part (one row per work-group); returns the number of partial rows in *nparts.
hipError_t launch_rowmm(ope_ctx* c, const double* X0, const double* M0, const double* X1,
                        const double* M1, const double* Cm, double cbeta, double ascale, double* Out,
                        int want_colsq, int predicated, int64_t* nparts);
// r0 = U - H Y0 (or U when HY is NULL, zeroing y), per-column sums of r0^2 and U^2 into c->part
hipError_t launch_resid0(ope_ctx* c, const double* U, const double* HY, double* R, double* y);

// mixed precision: FP32 blocks, kind MK_F64 / MK_F32 / MK_BF16
hipError_t launch_gram_f32(ope_ctx* c, int kind, const float* A, int64_t lda, int na, const float* B,
                           int64_t ldb, int nb, int64_t rows, double* out);
hipError_t launch_rowmm_f32(ope_ctx* c, int kind, const float* X0, const float* M0, const float* X1,
                            const float* M1, const float* Cm, double cbeta, double ascale, float* Out,
                            int want_colsq, int predicated, int64_t* nparts);
// elementwise precision conversion (to_double != 0: float -> double)
hipError_t launch_convert(ope_ctx* c, const void* src, void* dst, int64_t count, int to_double);

// one-work-group FP64 kernels
hipError_t launch_prep_small(ope_ctx* c);
hipError_t launch_cg_setup(ope_ctx* c, const double* rho0);
hipError_t launch_small_solve(ope_ctx* c, const double* Sb, const double* T, double tau,
                              double* Z, double* A, double* B);
// mixed: M = I + tau/2 (S_a - S_b) + tau^2/4 (P^T P - S_b^T (C-I) S_b), B = M^{-1}; Z32 = [-2(I-B) ; tau B]
hipError_t launch_small_solve_delta(ope_ctx* c, const double* Sb, const double* Tperp, double tau);
// FP32 copy of an N x N matrix
hipError_t launch_small_to_f32(ope_ctx* c, const double* src, float* dst, int64_t count);
hipError_t launch_jacobi_eig(ope_ctx* c, const double* Asym, double* evals);
// D = alpha op(A) op(B) + beta C + gamma I for N x N FP64 matrices (FP64 matrix
// cores); *skip != 0 makes it a no-op; res (nullable) receives per-work-group
// sums of (delta_ij - D_ij)^2, ((N + 63) / 64)^2 values
hipError_t launch_sqmm(ope_ctx* c, const double* A, int ta, const double* B, int tb, const double* C, double alpha,
                       double beta, double gamma, double* D, uint32_t N, const int32_t* skip, double* res);
// Z32 (N x N, FP32) = (3 I - C) / 2
hipError_t launch_renorm_matrix(ope_ctx* c, const double* C, float* Z32);
// dst = src (bytes, a multiple of 8) unless the step's error flag is set
// (pred = ROWMM_IF_OK), or only when the drift check asked for a
// re-normalisation (pred = ROWMM_IF_RENORM)
hipError_t launch_copy_pred(ope_ctx* c, const void* src, void* dst, uint64_t bytes, int pred = ROWMM_IF_OK);
// drift check after a mixed-precision update: from C = U^T U, sets sc->renorm
// (drift above thr) and writes Z32 = (3 I - C) / 2
hipError_t launch_drift_check(ope_ctx* c, const double* C, float* Z32, double thr);
hipError_t launch_solve_setup(ope_ctx* c, const double* rho0, double tol);

// Batched CG sweeps (k_stencil.hip): one work item range per problem.  The
// fields are the march kernel's arguments (for the odd-iteration sweep B,
// O1 is p of the previous iteration and beta that iteration's alpha).
struct MarchJob {
  const void* F0;
  const void* F1;
  void* O0;
  void* O1;
  void* Yv;
  double* alpha;
  double* beta;
  int32_t* active;
  const void* diag;
  OpeGrid g;
  MarchShape ms;
  uint32_t N, NV;
  double* part;
  OpeScalars* sc;
  uint32_t wg_begin, wg_count;
};
// Batched column reductions (one work-group per problem; ncols <= 128) and the
// gather of every problem's convergence flags into one array.
struct ReduceJob {
  const double* part;
  uint32_t nrows, ncols;
  double *alpha, *beta, *rho;   // alpha: 2 ncols (one half per iteration parity)
  const double* target;
  int32_t* active;
  OpeScalars* sc;
  int32_t* flags_out;      // gather destination (N values)
};
// sweep A, sweep B of an even iteration, sweep B of an odd one (with the y update)
enum { BATCH_SW_PAP = 1, BATCH_SW_UPDATE = 2, BATCH_SW_UPDATE_Y = 3 };
// halo: the class's x lines are split into several segments (nxs > 1);
// ln: its work-groups take two side lines, one per pass (ly = 2)
hipError_t launch_march_batched(hipStream_t s, int prec, int vw, int q, int halo, int ln, int mode, int first,
                                const MarchJob* jobs, uint32_t njobs, uint32_t total_wgs);
hipError_t launch_reduce_batched(hipStream_t s, int mode, int par, const ReduceJob* jobs, uint32_t njobs);
hipError_t launch_gather_flags(hipStream_t s, const ReduceJob* jobs, uint32_t njobs);
// whether a context's CG column sums fit the one-work-group reduction
bool reduce_few_fits(const ope_ctx* c);

// set-up kernels (k_check.hip): Lanczos extreme eigenvalues of H (FP64, one
// vector, temporary device buffers), the Cholesky-based R^{-1} of an N x N SPD
// matrix held in A (overwritten), and copies of a device scalar (0 energy,
// 1 residual, 2 drift) to a caller's device address
hipError_t lanczos_extremes(ope_ctx* c, int max_it, double* lmin, double* lmax, int* iters);
hipError_t launch_chol_rinv(ope_ctx* c, double* A, double* Rinv);
hipError_t launch_scalar_copy(ope_ctx* c, int which, double* out);

// learned form (k_net.hip): column sums of squares of point-major FP64 rows
// (B <= 256) into out, and E = U - P(R) for the context's N columns
hipError_t launch_colsq(ope_ctx* c, const double* R, int64_t ld, int64_t B, double* out);
hipError_t net_apply_residual(ope_net* t, const double* R, const double* colsq, const double* U, double* E);

// device helpers shared by the kernels ---------------------------------------
#ifdef __HIPCC__
// The hardware hands work-group b to XCD (b mod 8).  Map it to a logical index
// so that each XCD works through one contiguous range of the problem and its
// private L2 sees the neighbouring rows it needs.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t G) {
  uint32_t q = G >> 3, r = G & 7u;
  uint32_t x = b & 7u, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}
#endif
