// C ABI of the eigensolver step: context, workspace and the Algorithm 1 driver.
//
// One step of scheme (4.1) (Section 4.1, Steps 1-4) is enqueued as
//   HU = H U                                   (stencil)
//   C = <U,U>, Lam = <U,HU>                    (FP64 MFMA Grams)
//   E, drift, |Lam|_F, Lam^{-1}                (one work-group, FP64)
//   R = HU - U Lam (+ column norms)            -> outer residual, inner tolerance
//   Y = U Lam^{-1}, r = -R Lam^{-1}            (warm start of Step 1: r = U - H Y)
//   CG on H Y = U, column by column            (Step 1; two sweeps per iteration)
//   S_b = <U,Y>, T = <Y,Y>                     (Grams)
//   M, B, A, Z                                 (Steps 2-3, one work-group, FP64)
//   U <- U Z_1 + Y Z_2 in place                (Step 4, predicated on the error flag)
// The host only synchronises to poll CG convergence every few iterations and
// to read the step's scalars at the end.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "ope_internal.h"

#define HIPCHK(x)                               \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return OPE_EHIP;      \
  } while (0)

struct ope_batch {
  int32_t count;
  hipStream_t user;                   // the caller's stream
  hipEvent_t start;
  std::vector<ope_ctx*> ctx;          // one context per problem
  std::vector<hipStream_t> streams;   // its stream
  std::vector<hipEvent_t> done;
  // shared CG launches: one stream, job tables (device + pinned staging), flags
  int shared;                         // 1: one launch per CG phase and class of problems
  hipStream_t cg_stream;
  hipEvent_t cg_ev;
  MarchJob* d_mjobs;
  MarchJob* h_mjobs;
  ReduceJob* d_rjobs;
  ReduceJob* h_rjobs;
  int32_t* d_flags;
  int32_t* h_flags;
  std::vector<uint32_t> flag_off;     // problem i's flags in h_flags
  std::vector<hipStream_t> cls_streams;  // one per class of problems in a shared launch
  std::vector<hipEvent_t> cls_events;
  // a captured batched step (ope_batch_capture / ope_batch_replay): its own job
  // tables and flags, so that eager batched steps between replays leave it intact
  hipStream_t cap_stream;
  hipEvent_t cap_fork, cap_join;
  hipGraphExec_t step_graph;
  MarchJob* d_gmjobs;
  ReduceJob* d_grjobs;
  int32_t* d_gflags;
  int32_t* h_gflags;
  std::vector<uint32_t> gflag_off;
  int32_t cap_iters;
};

namespace {

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  return hipMalloc((void**)p, count * sizeof(T) > 0 ? count * sizeof(T) : 1);
}

hipError_t balloc(void** p, size_t bytes) {
  *p = nullptr;
  return hipMalloc(p, bytes > 0 ? bytes : 1);
}

void drop_graphs(ope_ctx* c);

void free_ctx(ope_ctx* c) {
  if (!c) return;
  mg_free(c);
  void* dptrs[] = {c->diag, c->diag32, c->ws_own, c->C, c->Lam, c->Linv, c->Sb, c->T,
                   c->Z, c->A, c->B, c->Wsm, c->Lam32, c->Linv32, c->Sb32, c->Z32, c->alpha, c->beta, c->rho,
                   c->target, c->cnorm2, c->rcol, c->rho0, c->active, c->part, c->stage, c->sc,
                   c->Ubak, c->ns_x[0], c->ns_x[1], c->ns_g, c->ns_m, c->ns_p, c->ns_part, c->ns,
                   c->mdiag, c->Upk, c->Dr, c->HDr};
  for (void* p : dptrs)
    if (p) (void)hipFree(p);
  if (c->hsc) (void)hipHostFree(c->hsc);
  if (c->hactive) (void)hipHostFree(c->hactive);
  if (c->hbuf) (void)hipHostFree(c->hbuf);
  if (c->hsc2) (void)hipHostFree(c->hsc2);
  if (c->hns) (void)hipHostFree(c->hns);
  for (hipEvent_t e : c->prof_events) (void)hipEventDestroy(e);
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (int k = 0; k < 2; ++k)
    if (c->chunk_ev[k]) (void)hipEventDestroy(c->chunk_ev[k]);
  delete c;
}

ope_status sync_and_read_scalars(ope_ctx* c) {
  HIPCHK(hipMemcpyAsync(c->hsc, c->sc, sizeof(OpeScalars), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return OPE_OK;
}

// Bytes of one n x N block in the workspace (rounded up to 256).
size_t ws_block_bytes(const ope_ctx* c) {
  const size_t esz = c->prec == OPE_FP64 ? sizeof(double) : sizeof(float);
  return ((size_t)c->n * (size_t)c->N * esz + 255) & ~(size_t)255;
}

// The five n x N blocks (HU, Y, two CG residuals, a CG direction) carved from
// one region: the caller's (ope_set_workspace) or one library allocation made
// on first use.
ope_status ensure_ws(ope_ctx* c) {
  if (c->HU) return OPE_OK;
  const size_t bb = ws_block_bytes(c);
  char* base = (char*)c->ws_ext;
  if (!base) {
    if (hipMalloc(&c->ws_own, 5 * bb) != hipSuccess) {
      c->ws_own = nullptr;
      return OPE_ENOMEM;
    }
    base = (char*)c->ws_own;
  }
  c->HU = base;
  c->Y = base + bb;
  c->Rb[0] = base + 2 * bb;
  c->Rb[1] = base + 3 * bb;
  c->Pb = base + 4 * bb;
  return OPE_OK;
}

#define WSCHK(c)                                \
  do {                                          \
    ope_status s_ = ensure_ws(c);               \
    if (s_ != OPE_OK) return s_;                \
  } while (0)

// Y = M X for the mass operator: the stencil sweep with M's diagonal and the
// negated off-diagonal coefficients (the sweep computes d x - sum c_a (x_- + x_+)).
hipError_t apply_mass(ope_ctx* c, const void* X, void* Y) {
  const OpeGrid g0 = c->g;
  const MarchShape ms0 = c->ms;
  double* d0 = c->diag;
  c->g.cx = -c->mass_mu[0];
  c->g.cy = -c->mass_mu[1];
  c->g.cz = c->g.dim == 3 ? -c->mass_mu[2] : 0.0;
  if (c->g.dim == 3) {
    c->ms.cm = c->g.cz;
    c->ms.cs = c->g.cy;
  } else {
    c->ms.cm = c->g.cy;
  }
  c->diag = c->mdiag;
  const hipError_t e = launch_apply_h(c, X, Y);
  c->g = g0;
  c->ms = ms0;
  c->diag = d0;
  return e;
}

// HU, Grams C and Lam, the small prep kernel (energy, drift, Lam^{-1}) and the
// residual R = HU - U Lam written over HU with its column norms in c->rcol.
// FP64: everything in FP64.  Mixed: FP32 stencil, C and Lam accumulated in
// FP64 on the matrix cores (energy and drift stay FP64), R in FP32.
ope_status phase_residual(ope_ctx* c, const void* Uv) {
  const int N = (int)c->N;
  int64_t np = 0;
  HIPCHK(launch_apply_h(c, Uv, c->HU));
  if (c->prec == OPE_FP64 && c->has_mass) {
    // generalized problem: C = U^T M U, Lam = U^T H U, R = HU - MU Lam, and the
    // Step-1 right-hand sides M u_j set the CG tolerances (their norms)
    const double* U = (const double*)Uv;
    double* HU = (double*)c->HU;
    double* MU = (double*)c->Rb[1];
    HIPCHK(apply_mass(c, U, MU));
    HIPCHK(launch_gram(c, U, N, N, MU, N, N, c->n, c->C));
    HIPCHK(launch_gram(c, U, N, N, HU, N, N, c->n, c->Lam));
    HIPCHK(launch_prep_small(c));
    HIPCHK(launch_colsq(c, MU, N, N, c->cnorm2));
    HIPCHK(launch_rowmm(c, MU, c->Lam, nullptr, nullptr, HU, 1.0, -1.0, HU, 1, 0, &np));
  } else if (c->prec == OPE_FP64) {
    const double* U = (const double*)Uv;
    double* HU = (double*)c->HU;
    HIPCHK(launch_gram(c, U, N, N, U, N, N, c->n, c->C));
    HIPCHK(launch_gram_sym(c, U, N, HU, N, N, c->n, c->Lam));     // H is symmetric
    HIPCHK(launch_prep_small(c));
    HIPCHK(launch_rowmm(c, U, c->Lam, nullptr, nullptr, HU, 1.0, -1.0, HU, 1, 0, &np));
  } else {
    const float* U = (const float*)Uv;
    float* HU = (float*)c->HU;
    HIPCHK(launch_gram_f32(c, MK_F64, U, N, N, U, N, N, c->n, c->C));
    HIPCHK(launch_gram_f32(c, MK_F64, U, N, N, HU, N, N, c->n, c->Lam));
    HIPCHK(launch_prep_small(c));
    HIPCHK(launch_rowmm_f32(c, MK_F32, U, c->Lam32, nullptr, nullptr, HU, 1.0, -1.0, HU, 1, 0, &np));
  }
  HIPCHK(launch_reduce_cols(c, c->part, np, N, c->rcol, RED_PLAIN));
  return OPE_OK;
}

// One CG iteration (two sweeps and their fixed-order reductions) with the
// buffer roles of iteration `it` (r and p alternate between two buffers, alpha
// between the two halves of its array).  The y term of an even iteration is
// added by the next iteration's sweep B, together with its own.
hipError_t cg_iteration_body(ope_ctx* c, int it);

// The buffer the CG iterates on: Y, or in a recycled step the correction Dr.
static inline void* cg_y(const ope_ctx* c) { return c->cg_on_d ? c->Dr : c->Y; }

// One CG iteration; its timed launches are tagged with the iteration index.
hipError_t cg_iteration(ope_ctx* c, int it) {
  c->prof_tag = it;
  const hipError_t r = cg_iteration_body(c, it);
  c->prof_tag = -1;
  return r;
}

hipError_t cg_iteration_body(ope_ctx* c, int it) {
  void* r_cur = c->Rb[it & 1];
  void* r_nxt = c->Rb[(it + 1) & 1];
  void* p_old = (it & 1) ? c->Pb : c->HU;    // never read on the first iteration
  void* p_new = (it & 1) ? c->HU : c->Pb;
  double* a_cur = c->alpha + (size_t)(it & 1) * c->N;
  double* a_prev = c->alpha + (size_t)((it + 1) & 1) * c->N;
  const int N = (int)c->N;
  const int first = it == 0;
  hipError_t e;
  // preconditioned form: sweep A forms p from z = B r instead of r
  if ((e = launch_cg_pap(c, c->mg_on ? (const void*)c->mg_Z : r_cur, p_old, p_new, first)) != hipSuccess) return e;
  {
    ProfScope ps(c, OPE_KERNEL_CG_REDUCE);
    if ((e = launch_reduce_cols(c, c->part, march_rows(c), N, nullptr, RED_CG_ALPHA, a_cur)) != hipSuccess) return e;
  }
  if (it & 1) e = launch_cg_update(c, r_cur, p_new, r_nxt, a_cur, cg_y(c), p_old, a_prev);
  else e = launch_cg_update(c, r_cur, p_new, r_nxt, a_cur, nullptr, nullptr, nullptr);
  if (e != hipSuccess) return e;
  if (c->mg_on) {
    // z = B r', then beta = r'^T z / rho and the stop test on |r'|^2
    if ((e = mg_vcycle(c, r_nxt, c->mg_Z, c->active, true)) != hipSuccess) return e;
    ProfScope ps(c, OPE_KERNEL_CG_REDUCE);
    if ((e = launch_reduce_cols(c, c->mg_part, c->mg_rows_used, 2 * N, c->mg_dots, RED_PLAIN)) != hipSuccess)
      return e;
    return launch_pcg_beta(c);
  }
  ProfScope ps(c, OPE_KERNEL_CG_REDUCE);
  return launch_reduce_cols(c, c->part, march_rows(c), N, nullptr, RED_CG_BETA, a_cur);
}

// Preconditioned CG start, after the CG set-up (targets and flags from |r0|^2):
// z0 = B r0 and rho = r0^T z0.
hipError_t pcg_begin(ope_ctx* c) {
  hipError_t e;
  if ((e = mg_vcycle(c, c->Rb[0], c->mg_Z, c->active, true)) != hipSuccess) return e;
  if ((e = launch_reduce_cols(c, c->mg_part, c->mg_rows_used, 2 * c->N, c->mg_dots, RED_PLAIN)) != hipSuccess)
    return e;
  return launch_pcg_start(c);
}

// After `its` CG iterations: when the last one was even, add its deferred y
// term (its p is in Pb, its alpha in the first half), on stream s.
hipError_t cg_flush(ope_ctx* c, int32_t its, hipStream_t s) {
  if (its <= 0 || (its & 1) == 0) return hipSuccess;
  return launch_y_flush(c, s, cg_y(c), c->Pb, c->alpha);
}

void drop_graphs(ope_ctx* c) {
  for (int k = 0; k < 2; ++k) {
    if (c->cg_graph[k]) (void)hipGraphExecDestroy(c->cg_graph[k]);
    c->cg_graph[k] = nullptr;
  }
  c->graph_state = 0;
}

// Capture the two CG chunks (iterations 0..K-1 and K..2K-1, K = check_every,
// even) as graphs on a private stream; they are replayed on the context's
// stream.  Every buffer and launch shape they use is fixed for the context,
// and convergence lives in device-side column masks, so a chunk needs no
// host decision.  On any capture error the context stays on eager launches.
void build_graphs(ope_ctx* c) {
  c->graph_state = -1;
  if (c->check_every % 2 != 0) return;
  if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    c->cap_stream = nullptr;
    return;
  }
  hipStream_t user = c->stream;
  c->stream = c->cap_stream;
  bool ok = true;
  for (int k = 0; k < 2 && ok; ++k) {
    hipGraph_t g = nullptr;
    ok &= hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (!ok) break;
    bool lok = true;
    for (int it = k * c->check_every; it < (k + 1) * c->check_every && lok; ++it) lok = cg_iteration(c, it) == hipSuccess;
    const bool eok = hipStreamEndCapture(c->cap_stream, &g) == hipSuccess;
    ok &= lok && eok && g != nullptr;
    if (ok) ok &= hipGraphInstantiate(&c->cg_graph[k], g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
  }
  c->stream = user;
  if (!ok) {
    (void)hipGetLastError();
    drop_graphs(c);
    c->graph_state = -1;
    return;
  }
  c->graph_state = 1;
}

// Host convergence checks of the preconditioned CG: it converges in a few
// iterations (about 2-4 per step) that each cost about 1 ms, and the chunk
// enqueued behind the one being checked runs past convergence as no-op
// launches (about 0.1 ms per iteration), so every iteration is checked; graph
// chunks hold pairs of iterations.
int mg_check_every(const ope_ctx* c) { return c->use_graphs ? 2 : 1; }

// Enqueues CG iterations up to the next host check (a multiple of
// check_every, or max_iter), the copy of the column flags into host slot
// `slot` and that slot's event.  Whole chunks run as graph replays when graphs
// are on (and no kernel is being timed), the rest as eager launches.
hipError_t cg_chunk(ope_ctx* c, int32_t* it, int32_t max_iter, int slot) {
  const int K = c->check_every;
  const bool graphs = c->use_graphs && c->prof_kernel < 0 && K % 2 == 0 && !c->recycle;
  if (graphs && c->graph_state == 0) build_graphs(c);
  const int32_t end = std::min<int32_t>(max_iter, (*it / K + 1) * K);
  hipError_t e;
  while (*it < end) {
    if (graphs && c->graph_state == 1 && *it % K == 0 && *it + K <= end) {
      if ((e = hipGraphLaunch(c->cg_graph[*it == 0 ? 0 : 1], c->stream)) != hipSuccess) return e;
      *it += K;
    } else {
      if ((e = cg_iteration(c, *it)) != hipSuccess) return e;
      *it += 1;
    }
  }
  if ((e = hipMemcpyAsync(c->hactive + (size_t)slot * c->N, c->active, sizeof(int32_t) * c->N,
                          hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
    return e;
  return hipEventRecord(c->chunk_ev[slot], c->stream);
}

// After host slot `slot` has been filled: true if every column converged.
bool cg_all_done(const ope_ctx* c, int slot) {
  const int32_t* a = c->hactive + (size_t)slot * c->N;
  for (int64_t j = 0; j < c->N; ++j)
    if (a[j] != 0) return false;
  return true;
}

// CG iterations on H Y = U from the state prepared in rho/target/active, with
// r in c->Rb[0]; returns the enqueued iteration count in *iters.  The next
// chunk is enqueued before the flags of the previous one are read, so the GPU
// does not wait for the host; a chunk enqueued after convergence finds every
// column inactive and its kernels do nothing (the sweeps exit, the
// reductions leave inactive columns at alpha = beta = 0).
ope_status run_cg(ope_ctx* c, int32_t max_iter, int32_t* iters, bool* all_done) {
  int32_t it = 0;
  bool done = false;
  int slot_next = 0, head = 0, nout = 0;
  int q[2] = {0, 0};
  for (;;) {
    while (it < max_iter && nout < 2) {
      HIPCHK(cg_chunk(c, &it, max_iter, slot_next));
      q[(head + nout) & 1] = slot_next;
      ++nout;
      slot_next ^= 1;
    }
    if (nout == 0) break;
    const int s = q[head];
    head ^= 1;
    --nout;
    HIPCHK(hipEventSynchronize(c->chunk_ev[s]));
    if (cg_all_done(c, s)) {
      done = true;
      break;
    }
  }
  HIPCHK(cg_flush(c, it, c->stream));
  *iters = it;
  *all_done = done;
  return OPE_OK;
}

void fill_info(ope_ctx* c, ope_step_info* info, int32_t iters, ope_status st) {
  c->drift_seen = c->hsc->drift;
  if (!info) return;
  info->energy = c->hsc->energy;
  info->residual = c->hsc->residual;
  info->drift = c->hsc->drift;
  info->inner_iterations = iters;
  info->status = st;
}

// Warm start of Step 1 (Y = U Lam^{-1}, r = -R Lam^{-1} = U - H Y) and the CG
// start state; R is in c->HU.
ope_status phase_warm_start(ope_ctx* c, const void* Uv) {
  const int N = (int)c->N;
  int64_t np = 0;
  c->cg_on_d = 0;
  if (c->prec == OPE_FP64 && c->recycle) {
    // recycled: the CG solves H d = -R Lam^{-1} from d0 = the previous step's
    // correction (zero at the start), so r0 = -R Lam^{-1} - H d0; Y = U Lam^{-1}
    // + d afterwards (recycle_after_cg)
    HIPCHK(launch_rowmm(c, (const double*)Uv, c->Linv, nullptr, nullptr, nullptr, 0.0, 1.0, (double*)c->Y, 0, 0, &np));
    HIPCHK(launch_rowmm(c, (const double*)c->HU, c->Linv, nullptr, nullptr, c->have_d ? (const double*)c->HDr : nullptr,
                        c->have_d ? -1.0 : 0.0, -1.0, (double*)c->Rb[0], 1, 0, &np));
    if (!c->have_d) HIPCHK(hipMemsetAsync(c->Dr, 0, sizeof(double) * (size_t)c->n * (size_t)N, c->stream));
    c->cg_on_d = 1;
  } else if (c->prec == OPE_FP64) {
    HIPCHK(launch_rowmm(c, (const double*)Uv, c->Linv, nullptr, nullptr, nullptr, 0.0, 1.0, (double*)c->Y, 0, 0, &np));
    HIPCHK(launch_rowmm(c, (const double*)c->HU, c->Linv, nullptr, nullptr, nullptr, 0.0, -1.0, (double*)c->Rb[0], 1,
                        0, &np));
  } else {
    HIPCHK(launch_rowmm_f32(c, MK_F32, (const float*)Uv, c->Linv32, nullptr, nullptr, nullptr, 0.0, 1.0,
                            (float*)c->Y, 0, 0, &np));
    HIPCHK(launch_rowmm_f32(c, MK_F32, (const float*)c->HU, c->Linv32, nullptr, nullptr, nullptr, 0.0, -1.0,
                            (float*)c->Rb[0], 1, 0, &np));
  }
  HIPCHK(launch_reduce_cols(c, c->part, np, N, c->rho0, RED_PLAIN));
  HIPCHK(launch_cg_setup(c, c->rho0));
  if (c->mg_on) HIPCHK(pcg_begin(c));
  return OPE_OK;
}

// After a recycled step's CG: Y = U Lam^{-1} + d, and H d for the next warm
// start (d stays in Dr as the next step's starting correction).
ope_status recycle_after_cg(ope_ctx* c) {
  if (!c->cg_on_d) return OPE_OK;
  HIPCHK(launch_add_block(c, (double*)c->Y, (const double*)c->Dr));
  HIPCHK(launch_apply_h(c, c->Dr, c->HDr));
  c->have_d = 1;
  c->cg_on_d = 0;
  return OPE_OK;
}

// Steps 2-4 after Step 1 (Y in c->Y).
ope_status phase_update(ope_ctx* c, void* Uv, double tau) {
  const int N = (int)c->N;
  const size_t NN = (size_t)N * N;
  int64_t np = 0;
  if (c->prec == OPE_FP64) {
    double* U = (double*)Uv;
    const double* Y = (const double*)c->Y;
    if (c->has_mass) {
      // inner matrices in the M product: S_b = (MU)^T Y, T = Y^T (MY); the CG
      // residual blocks are free once Step 1 has finished
      double* MU = (double*)c->Rb[0];
      double* MY = (double*)c->Rb[1];
      HIPCHK(apply_mass(c, U, MU));
      HIPCHK(apply_mass(c, Y, MY));
      HIPCHK(launch_gram(c, MU, N, N, Y, N, N, c->n, c->Sb));
      HIPCHK(launch_gram(c, Y, N, N, MY, N, N, c->n, c->T));
    } else {
      HIPCHK(launch_gram(c, U, N, N, Y, N, N, c->n, c->Sb));
      HIPCHK(launch_gram(c, Y, N, N, Y, N, N, c->n, c->T));
    }
    HIPCHK(launch_small_solve(c, c->Sb, c->T, tau, c->Z, c->A, c->B));
    if (N <= 128) {
      HIPCHK(launch_rowmm(c, U, c->Z, Y, c->Z + NN, nullptr, 0.0, 1.0, U, 0, 1, &np));
    } else {
      // several column tiles read every column of U: write aside, then copy back
      double* tmp = (double*)c->Pb;
      HIPCHK(launch_rowmm(c, U, c->Z, Y, c->Z + NN, nullptr, 0.0, 1.0, tmp, 0, 1, &np));
      HIPCHK(launch_copy_pred(c, tmp, U, sizeof(double) * (uint64_t)c->n * N));
    }
  } else {
    // S_b = U^T Y (FP32 matrix cores), P = Y - U S_b (FP32), T_perp = P^T P
    // (BF16, FP32 accumulation), FP64 small solve, U += U Z1 + P Z2 (FP32
    // matrix cores: with BF16 operands the rounding of U in U Z1 adds about
    // 1e-4 of drift per early step, with FP32 about 1e-6, at the same speed).
    float* U = (float*)Uv;
    const float* Y = (const float*)c->Y;
    float* P = (float*)c->HU;
    HIPCHK(launch_gram_f32(c, MK_F32, U, N, N, Y, N, N, c->n, c->Sb));
    HIPCHK(launch_small_to_f32(c, c->Sb, c->Sb32, (int64_t)NN));
    HIPCHK(launch_rowmm_f32(c, MK_F32, U, c->Sb32, nullptr, nullptr, Y, 1.0, -1.0, P, 0, 0, &np));
    HIPCHK(launch_gram_f32(c, MK_BF16, P, N, N, P, N, N, c->n, c->T));
    HIPCHK(launch_small_solve_delta(c, c->Sb, c->T, tau));
    if (N <= 128) {
      HIPCHK(launch_rowmm_f32(c, MK_F32, U, c->Z32, P, c->Z32 + NN, U, 1.0, 1.0, U, 0, ROWMM_IF_OK, &np));
    } else {
      float* tmp = (float*)c->Pb;
      HIPCHK(launch_rowmm_f32(c, MK_F32, U, c->Z32, P, c->Z32 + NN, U, 1.0, 1.0, tmp, 0, ROWMM_IF_OK, &np));
      HIPCHK(launch_copy_pred(c, tmp, U, sizeof(float) * (uint64_t)c->n * N));
    }
    // Drift check of the updated iterate: the scheme keeps U^T U constant in
    // exact arithmetic, but the BF16 P^T P perturbs the Step-2 matrix and the
    // FP32 products round, so every mixed step may add drift.  C of the new
    // block (FP64 accumulation) decides on the device whether one
    // Newton-Schulz step U <- U (3I - C)/2 is applied, so that the block handed
    // back stays below the drift target.
    HIPCHK(launch_gram_f32(c, MK_F64, U, N, N, U, N, N, c->n, c->C));
    HIPCHK(launch_drift_check(c, c->C, c->Z32, c->drift_tol));
    if (N <= 128) {
      HIPCHK(launch_rowmm_f32(c, MK_F32, U, c->Z32, nullptr, nullptr, U, 1.0, 1.0, U, 0, ROWMM_IF_RENORM, &np));
    } else {
      float* tmp = (float*)c->Pb;
      HIPCHK(launch_rowmm_f32(c, MK_F32, U, c->Z32, nullptr, nullptr, U, 1.0, 1.0, tmp, 0, ROWMM_IF_RENORM, &np));
      HIPCHK(launch_copy_pred(c, tmp, U, sizeof(float) * (uint64_t)c->n * N, ROWMM_IF_RENORM));
    }
  }
  return OPE_OK;
}

// Mixed precision: when the last observed drift |U^T U - I|_F exceeds 1e-6,
// one Newton-Schulz re-normalisation U <- U + U (I - C) / 2 with C = U^T U
// (FP64 Gram of the FP32 block, FP32 product of the correction) before the
// step: the scheme keeps the drift constant in exact arithmetic, the BF16
// update adds to it, and this takes a drift E to O(E^2).
ope_status mixed_renormalize(ope_ctx* c, void* Uv) {
  if (c->prec != OPE_MIXED || !(c->drift_seen > 1e-6)) return OPE_OK;
  const int N = (int)c->N;
  float* U = (float*)Uv;
  int64_t np = 0;
  HIPCHK(launch_gram_f32(c, MK_F64, U, N, N, U, N, N, c->n, c->C));
  HIPCHK(launch_renorm_matrix(c, c->C, c->Z32));
  if (N <= 128) {
    HIPCHK(launch_rowmm_f32(c, MK_F32, U, c->Z32, nullptr, nullptr, U, 1.0, 1.0, U, 0, 0, &np));
  } else {
    HIPCHK(launch_rowmm_f32(c, MK_F32, U, c->Z32, nullptr, nullptr, U, 1.0, 1.0, (float*)c->Pb, 0, 0, &np));
    HIPCHK(hipMemcpyAsync(U, c->Pb, sizeof(float) * (size_t)c->n * N, hipMemcpyDeviceToDevice, c->stream));
  }
  c->renorms += 1;
  return OPE_OK;
}

// One step (or, with res_tol >= 0, the convergence test of Algorithm 1 and a
// step if the residual is still above res_tol).
ope_status run_step(ope_ctx* c, void* U, double tau, ope_step_info* info, double res_tol, bool* converged) {
  if (converged) *converged = false;
  ope_status st = mixed_renormalize(c, U);
  if (st != OPE_OK) return st;
  st = phase_residual(c, U);
  if (st != OPE_OK) return st;
  st = phase_warm_start(c, U);
  if (st != OPE_OK) return st;
  if (res_tol >= 0.0) {
    st = sync_and_read_scalars(c);
    if (st != OPE_OK) return st;
    if (c->hsc->err != 0) return (ope_status)c->hsc->err;
    if (c->hsc->residual <= res_tol) {
      if (converged) *converged = true;
      fill_info(c, info, 0, OPE_OK);
      return OPE_OK;
    }
  }
  int32_t iters = 0;
  bool cg_done = false;
  st = run_cg(c, c->max_iter, &iters, &cg_done);
  if (st != OPE_OK) return st;
  st = recycle_after_cg(c);
  if (st != OPE_OK) return st;
  st = phase_update(c, U, tau);
  if (st != OPE_OK) return st;
  st = sync_and_read_scalars(c);
  if (st != OPE_OK) return st;
  ope_status out = (ope_status)c->hsc->err;
  if (out == OPE_OK && !cg_done) out = OPE_ECG_MAXIT;
  fill_info(c, info, c->hsc->cg_iters, out);
  return out;
}

// Learned step after phase_residual(U) with its scalars in c->hsc: Y =
// (U - P(R)) Lam^{-1}, Steps 2-4, then the judge (the new iterate's energy and
// residual).  Accepted: U holds the new iterate and its residual phase is done
// (scalars in c->hsc).  Rejected: U is restored and one plain step is taken
// (its diagnostics in *plain).
ope_status learned_core(ope_ctx* c, void* Uv, double tau, bool* accepted, ope_step_info* plain) {
  *accepted = false;
  const int N = (int)c->N;
  const size_t bytes = sizeof(double) * (size_t)c->n * (size_t)N;
  const double E0 = c->hsc->energy, res0 = c->hsc->residual;
  double* U = (double*)Uv;
  int64_t np = 0;
  if (c->net_judge) HIPCHK(hipMemcpyAsync(c->Ubak, U, bytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(net_apply_residual(c->net, (const double*)c->HU, c->rcol, U, (double*)c->Rb[0]));
  HIPCHK(launch_rowmm(c, (const double*)c->Rb[0], c->Linv, nullptr, nullptr, nullptr, 0.0, 1.0, (double*)c->Y, 0, 0,
                      &np));
  ope_status st = phase_update(c, U, tau);
  if (st != OPE_OK) return st;
  if (!c->net_judge) {
    // no judge: the learned iterate is kept unless the small solve failed (then U is unchanged)
    st = sync_and_read_scalars(c);
    if (st != OPE_OK) return st;
    *accepted = c->hsc->err == 0;
    return c->hsc->err == 0 ? OPE_OK : (ope_status)c->hsc->err;
  }
  HIPCHK(hipMemcpyAsync(c->hsc2, c->sc, sizeof(OpeScalars), hipMemcpyDeviceToHost, c->stream));
  st = phase_residual(c, U);
  if (st != OPE_OK) return st;
  HIPCHK(launch_cg_setup(c, c->rcol));   // the residual scalar from the column norms
  st = sync_and_read_scalars(c);
  if (st != OPE_OK) return st;
  const OpeScalars& s = *c->hsc;
  if (c->hsc2->err == 0 && s.err == 0 && s.energy <= E0 + 1e-13 * std::fabs(E0) && s.residual <= res0) {
    *accepted = true;
    return OPE_OK;
  }
  HIPCHK(hipMemcpyAsync(U, c->Ubak, bytes, hipMemcpyDeviceToDevice, c->stream));
  return run_step(c, U, tau, plain, -1.0, nullptr);
}

ope_status check_learned(ope_ctx* c) {
  if (!c->net) return OPE_EINVAL;
  if (c->prec != OPE_FP64) return OPE_EUNSUPPORTED;
  return OPE_OK;
}

// Algorithm 1 with learned steps judged by the plain step.  After a rejected
// learned step the next `backoff` steps are plain (1, 2, 4, ... up to 64,
// reset by an accepted one), so a network that stops helping late in a solve
// costs little more than the plain iteration.
ope_status solve_learned(ope_ctx* c, void* U, double tau, double res_tol, int32_t max_steps, ope_solve_info* si) {
  bool ready = false;      // residual phase of the current U done, scalars in c->hsc
  int32_t skip = 0, backoff = 0;
  ope_status st = OPE_OK;
  for (;;) {
    const bool last = si->steps >= max_steps;
    if (!last && skip > 0) {
      // a plain step (with the convergence test of Algorithm 1 on the way)
      ope_step_info s;
      bool conv = false;
      st = run_step(c, U, tau, &s, res_tol, &conv);
      if (st != OPE_OK && st != OPE_ECG_MAXIT) return st;
      si->residual = s.residual;
      si->energy = s.energy;
      si->drift = s.drift;
      if (conv) {
        si->converged = 1;
        return OPE_OK;
      }
      si->steps += 1;
      si->inner_iterations += s.inner_iterations;
      --skip;
      ready = false;
      continue;
    }
    if (!ready) {
      st = phase_residual(c, U);
      if (st != OPE_OK) return st;
      HIPCHK(launch_cg_setup(c, c->rcol));
      st = sync_and_read_scalars(c);
      if (st != OPE_OK) return st;
      if (c->hsc->err != 0) return (ope_status)c->hsc->err;
    }
    si->residual = c->hsc->residual;
    si->energy = c->hsc->energy;
    si->drift = c->hsc->drift;
    if (c->hsc->residual <= res_tol) {
      si->converged = 1;
      return OPE_OK;
    }
    if (last) return OPE_OK;
    bool acc = false;
    ope_step_info plain;
    memset(&plain, 0, sizeof(plain));
    st = learned_core(c, U, tau, &acc, &plain);
    if (st != OPE_OK && st != OPE_ECG_MAXIT) return st;
    si->steps += 1;
    if (acc) {
      si->learned_steps += 1;
      ready = c->net_judge != 0;   // the judge already evaluated the new iterate
      backoff = 0;
    } else {
      si->inner_iterations += plain.inner_iterations;
      ready = false;
      backoff = backoff ? std::min(2 * backoff, 64) : 1;
      skip = backoff;
    }
  }
}

// ---------------------------------------------------------------------------
// batched form: many independent problems, each on its own context and stream
// ---------------------------------------------------------------------------
struct BatchState {
  std::vector<ope_step_info> info;
  std::vector<ope_status> st;
  std::vector<char> conv, cgdone;
  std::vector<int32_t> it;
};

// A problem takes part in the shared launches when its column sums fit one
// work-group's reduction (the same fixed-order sum its own steps use, so that
// its shared-launch iterates equal those of its own launches bit for bit); its
// work items are the tiles of its own sweep shape.
bool shared_fits(const ope_ctx* c) { return !c->mg_on && reduce_few_fits(c); }

// The shared CG launches of a set of problems: classes of problems that one
// kernel instance can sweep (storage type, vector width, passes per plane,
// split x lines, line tiles), and per class the job tables of its four sweep
// variants (sweep A / B, even / odd iteration), staged in pinned host memory.
struct CgPlan {
  struct Cls {
    int prec, vw, q, halo, ln;
    std::vector<int> idx;
  };
  std::vector<Cls> cls;
  std::vector<uint32_t> cls_off, cls_total;
  uint32_t M = 0;       // problems (reduce jobs)
  uint32_t jobs = 0;    // march jobs
  uint32_t flags = 0;   // convergence flags gathered
};

void plan_cg(ope_batch* b, const std::vector<int>& members, int32_t* d_flags, CgPlan& pl) {
  auto& cls = pl.cls;
  cls.clear();
  for (int i : members) {
    const ope_ctx* c = b->ctx[i];
    const int halo = c->ms.nxs > 1 ? 1 : 0, ln = c->ms.ly > 1 ? 1 : 0;
    bool found = false;
    for (auto& k : cls)
      if (k.prec == c->prec && k.vw == c->vw && k.q == (int)c->ms.q && k.halo == halo && k.ln == ln) {
        k.idx.push_back(i);
        found = true;
        break;
      }
    if (!found) cls.push_back(CgPlan::Cls{c->prec, c->vw, (int)c->ms.q, halo, ln, {i}});
  }
  // job tables: per class, 4 variants (sweep A / B, even / odd iteration)
  pl.M = (uint32_t)members.size();
  pl.cls_off.assign(cls.size(), 0);
  pl.cls_total.assign(cls.size(), 0);
  uint32_t off = 0;
  for (size_t k = 0; k < cls.size(); ++k) {
    pl.cls_off[k] = off;
    uint32_t wg = 0;
    for (int v = 0; v < 4; ++v) {
      wg = 0;
      for (size_t m = 0; m < cls[k].idx.size(); ++m) {
        ope_ctx* c = b->ctx[cls[k].idx[m]];
        const int par = v & 1, upd = v >> 1;
        void* p_old = par ? c->Pb : c->HU;      // as in cg_iteration
        void* p_new = par ? c->HU : c->Pb;
        MarchJob& jb = b->h_mjobs[off + v * cls[k].idx.size() + m];
        jb.F0 = c->Rb[par];
        jb.F1 = upd ? p_new : p_old;
        jb.O0 = upd ? c->Rb[par ^ 1] : nullptr;
        jb.O1 = upd ? (par ? p_old : nullptr) : p_new;     // odd sweep B: p of the previous iteration
        jb.Yv = (upd && par) ? c->Y : nullptr;
        jb.alpha = c->alpha + (size_t)par * c->N;
        jb.beta = (upd && par) ? c->alpha : c->beta;       // odd sweep B: the previous iteration's alpha
        jb.active = c->active;
        jb.diag = c->prec == OPE_FP64 ? (const void*)c->diag : (const void*)c->diag32;
        jb.g = c->g;
        jb.ms = c->ms;
        jb.N = (uint32_t)c->N;
        jb.NV = (uint32_t)(c->N / c->vw);
        jb.part = c->part;
        jb.sc = c->sc;
        jb.wg_begin = wg;
        jb.wg_count = jb.ms.lgroups * jb.ms.nxs * jb.ms.cc * jb.ms.mc;
        wg += (jb.wg_count + 7u) & ~7u;          // whole groups of 8: one per XCD
      }
    }
    pl.cls_total[k] = wg;
    off += 4 * (uint32_t)cls[k].idx.size();
  }
  pl.jobs = off;
  uint32_t foff = 0;
  for (uint32_t m = 0; m < pl.M; ++m) {
    ope_ctx* c = b->ctx[members[m]];
    ReduceJob& rj = b->h_rjobs[m];
    rj.part = c->part;
    rj.nrows = (uint32_t)march_rows(c);
    rj.ncols = (uint32_t)c->N;
    rj.alpha = c->alpha;
    rj.beta = c->beta;
    rj.rho = c->rho;
    rj.target = c->target;
    rj.active = c->active;
    rj.sc = c->sc;
    rj.flags_out = d_flags + foff;
    b->flag_off[members[m]] = foff;
    foff += (uint32_t)c->N;
  }
  pl.flags = foff;
}

// Enqueues `count` CG iterations from iteration it0 of the planned problems on
// stream s (class sweeps forked onto the classes' streams and joined back),
// with the job tables at mjobs / rjobs on the device.  No host synchronisation.
hipError_t enqueue_cg(ope_batch* b, const CgPlan& pl, const MarchJob* mjobs, const ReduceJob* rjobs, int32_t it0,
                      int32_t count, hipStream_t s) {
  hipError_t e;
  const auto& cls = pl.cls;
  while (b->cls_streams.size() < cls.size()) {
    hipStream_t cs;
    hipEvent_t ce;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&ce, hipEventDisableTiming)) != hipSuccess) return e;
    b->cls_streams.push_back(cs);
    b->cls_events.push_back(ce);
  }
  auto sweep = [&](int mode, int par, int first) -> hipError_t {
    hipError_t er;
    const int kmode = (mode == BATCH_SW_UPDATE && par) ? BATCH_SW_UPDATE_Y : mode;
    if (cls.size() == 1) {
      const uint32_t nc = (uint32_t)cls[0].idx.size();
      const uint32_t v = (mode == BATCH_SW_PAP ? 0 : 2) + par;
      return launch_march_batched(s, cls[0].prec, cls[0].vw, cls[0].q, cls[0].halo, cls[0].ln, kmode, first,
                                  mjobs + pl.cls_off[0] + v * nc, nc, pl.cls_total[0]);
    }
    if ((er = hipEventRecord(b->cg_ev, s)) != hipSuccess) return er;
    for (size_t c = 0; c < cls.size(); ++c) {
      hipStream_t cs = b->cls_streams[c];
      const uint32_t nc = (uint32_t)cls[c].idx.size();
      const uint32_t v = (mode == BATCH_SW_PAP ? 0 : 2) + par;
      if ((er = hipStreamWaitEvent(cs, b->cg_ev, 0)) != hipSuccess) return er;
      if ((er = launch_march_batched(cs, cls[c].prec, cls[c].vw, cls[c].q, cls[c].halo, cls[c].ln, kmode, first,
                                     mjobs + pl.cls_off[c] + v * nc, nc, pl.cls_total[c])) != hipSuccess)
        return er;
      if ((er = hipEventRecord(b->cls_events[c], cs)) != hipSuccess) return er;
      if ((er = hipStreamWaitEvent(s, b->cls_events[c], 0)) != hipSuccess) return er;
    }
    return hipSuccess;
  };
  for (int32_t k = 0, it = it0; k < count; ++k, ++it) {
    const int par = it & 1, first = it == 0;
    if ((e = sweep(BATCH_SW_PAP, par, first)) != hipSuccess) return e;
    if ((e = launch_reduce_batched(s, RED_CG_ALPHA, par, rjobs, pl.M)) != hipSuccess) return e;
    if ((e = sweep(BATCH_SW_UPDATE, par, first)) != hipSuccess) return e;
    if ((e = launch_reduce_batched(s, RED_CG_BETA, par, rjobs, pl.M)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// One chunk (check_every iterations) of Step 1's CG for the problems in
// `members`, with one launch per sweep and class of problems and one launch
// per column reduction, then the gather of their convergence flags into
// h_flags (synchronised).  The problems' pre-phases must have completed.
hipError_t batch_cg_chunk(ope_batch* b, const std::vector<int>& members, int32_t* it) {
  CgPlan pl;
  plan_cg(b, members, b->d_flags, pl);
  hipStream_t s = b->cg_stream;
  hipError_t e;
  if ((e = hipMemcpyAsync(b->d_mjobs, b->h_mjobs, sizeof(MarchJob) * pl.jobs, hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(b->d_rjobs, b->h_rjobs, sizeof(ReduceJob) * pl.M, hipMemcpyHostToDevice, s)) != hipSuccess)
    return e;
  const int K = b->ctx[members[0]]->check_every;
  if ((e = enqueue_cg(b, pl, b->d_mjobs, b->d_rjobs, *it, K, s)) != hipSuccess) return e;
  *it += K;
  if ((e = launch_gather_flags(s, b->d_rjobs, pl.M)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(b->h_flags, b->d_flags, sizeof(int32_t) * pl.flags, hipMemcpyDeviceToHost, s)) !=
      hipSuccess)
    return e;
  if ((e = hipEventRecord(b->cg_ev, s)) != hipSuccess) return e;
  return hipEventSynchronize(b->cg_ev);
}

// One round over the problems with run[i] set: the pre-phase of every problem
// (residual, Lam^{-1}, warm start), one host synchronisation, then rounds of
// CG chunks in which each problem leaves as soon as all its columns converged,
// then Steps 2-4 of every problem still running.  With res_tol >= 0 a problem
// whose residual is already <= res_tol is only evaluated (conv set).
ope_status batch_round(ope_batch* b, void* const* U, double tau, double res_tol, const std::vector<char>& run,
                       BatchState& bs) {
  const int P = b->count;
  bs.info.assign(P, ope_step_info{});
  bs.st.assign(P, OPE_OK);
  bs.conv.assign(P, 0);
  bs.cgdone.assign(P, 0);
  bs.it.assign(P, 0);
  std::vector<char> go(run);
  HIPCHK(hipEventRecord(b->start, b->user));
  for (int i = 0; i < P; ++i) {
    if (!go[i]) continue;
    ope_ctx* c = b->ctx[i];
    HIPCHK(hipStreamWaitEvent(c->stream, b->start, 0));
    ope_status st = ensure_ws(c);
    if (st == OPE_OK) st = mixed_renormalize(c, U[i]);
    if (st == OPE_OK) st = phase_residual(c, U[i]);
    if (st == OPE_OK) st = phase_warm_start(c, U[i]);
    if (st == OPE_OK && hipMemcpyAsync(c->hsc, c->sc, sizeof(OpeScalars), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      st = OPE_EHIP;
    if (st != OPE_OK) {
      bs.st[i] = st;
      go[i] = 0;
    }
  }
  for (int i = 0; i < P; ++i) {
    if (!go[i]) continue;
    ope_ctx* c = b->ctx[i];
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->hsc->err != 0) {
      bs.st[i] = (ope_status)c->hsc->err;
      fill_info(c, &bs.info[i], 0, bs.st[i]);
      go[i] = 0;
    } else if (res_tol >= 0.0 && c->hsc->residual <= res_tol) {
      bs.conv[i] = 1;
      fill_info(c, &bs.info[i], 0, OPE_OK);
      go[i] = 0;
    }
  }
  // Step 1: problems whose column sums fit one work-group share one launch per
  // CG phase and class (storage type, vector width, passes per plane, split x
  // lines) on the batch's CG stream; the others run their own chunks on their
  // own streams.
  // Per-problem CG keeps two chunks in flight per problem, as run_cg does: a
  // problem's next chunk is enqueued before the flags of its previous one are
  // read, so the GPU does not drain while the host checks (a chunk enqueued
  // after convergence does nothing).
  std::vector<char> pending(go), shared(P, 0);
  for (int i = 0; i < P; ++i) shared[i] = go[i] && b->shared && shared_fits(b->ctx[i]);
  std::vector<int> head(P, 0), nout(P, 0), slot_next(P, 0), q0(P, 0), q1(P, 0);
  int32_t it_shared = 0;
  for (;;) {
    bool any = false, any_shared = false;
    for (int i = 0; i < P; ++i) {
      if (!pending[i]) continue;
      any = true;
      if (shared[i]) {
        any_shared = true;
        continue;
      }
      ope_ctx* c = b->ctx[i];
      while (bs.it[i] < c->max_iter && nout[i] < 2) {
        if (cg_chunk(c, &bs.it[i], c->max_iter, slot_next[i]) != hipSuccess) {
          bs.st[i] = OPE_EHIP;
          pending[i] = go[i] = 0;
          break;
        }
        (((head[i] + nout[i]) & 1) ? q1 : q0)[i] = slot_next[i];
        ++nout[i];
        slot_next[i] ^= 1;
      }
    }
    if (!any) break;
    if (any_shared) {
      std::vector<int> members;
      for (int i = 0; i < P; ++i)
        if (pending[i] && shared[i]) members.push_back(i);
      HIPCHK(batch_cg_chunk(b, members, &it_shared));
    }
    for (int i = 0; i < P; ++i) {
      if (!pending[i]) continue;
      ope_ctx* c = b->ctx[i];
      if (shared[i]) {
        bs.it[i] = it_shared;
        const int32_t* f = b->h_flags + b->flag_off[i];
        bool done = true;
        for (int64_t j = 0; j < c->N; ++j) done &= f[j] == 0;
        if (done) {
          bs.cgdone[i] = 1;
          pending[i] = 0;
        } else if (it_shared >= c->max_iter) {
          pending[i] = 0;
        }
        continue;
      }
      if (nout[i] == 0) {            // max_iter reached and every chunk read
        pending[i] = 0;
        continue;
      }
      const int slot = (head[i] ? q1 : q0)[i];
      head[i] ^= 1;
      --nout[i];
      HIPCHK(hipEventSynchronize(c->chunk_ev[slot]));
      if (cg_all_done(c, slot)) {
        bs.cgdone[i] = 1;
        pending[i] = 0;
      } else if (bs.it[i] >= c->max_iter && nout[i] == 0) {
        pending[i] = 0;
      }
    }
  }
  for (int i = 0; i < P; ++i) {
    if (!go[i]) continue;
    ope_ctx* c = b->ctx[i];
    ope_status st = cg_flush(c, bs.it[i], c->stream) == hipSuccess ? OPE_OK : OPE_EHIP;   // shared CG: synchronised
    if (st == OPE_OK) st = phase_update(c, U[i], tau);
    if (st == OPE_OK && hipMemcpyAsync(c->hsc, c->sc, sizeof(OpeScalars), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      st = OPE_EHIP;
    if (st != OPE_OK) {
      bs.st[i] = st;
      go[i] = 0;
    }
  }
  for (int i = 0; i < P; ++i) {
    if (!run[i]) continue;
    ope_ctx* c = b->ctx[i];
    if (go[i]) {
      HIPCHK(hipStreamSynchronize(c->stream));
      ope_status out = (ope_status)c->hsc->err;
      if (out == OPE_OK && !bs.cgdone[i]) out = OPE_ECG_MAXIT;
      fill_info(c, &bs.info[i], c->hsc->cg_iters, out);
      bs.st[i] = out;
    }
    // later work on the caller's stream waits for this problem
    HIPCHK(hipEventRecord(b->done[i], c->stream));
    HIPCHK(hipStreamWaitEvent(b->user, b->done[i], 0));
  }
  return OPE_OK;
}

// Seconds per short CG run (8 iterations, best of 3 after a warm-up run) for
// the context's current sweep shape; the set-up is not timed.  FP64: r0 from
// the scratch right-hand side X; FP32 (X unused): r0 is the block with every
// word 0x3F3F3F3F, whose column norms are known on the host.  The inner
// tolerance is 0, so no column converges within the run.
double time_cg(ope_ctx* c, const double* X, hipEvent_t e0, hipEvent_t e1) {
  const int N = (int)c->N;
  std::vector<double> rho;
  if (c->prec != OPE_FP64) {
    const uint32_t bits = 0x3F3F3F3Fu;
    float v;
    memcpy(&v, &bits, sizeof v);
    rho.assign(2 * (size_t)N, (double)c->n * (double)v * (double)v);
  }
  double best = 1e30;
  c->cg_on_d = 0;                // the timed CG iterates on Y
  for (int rep = 0; rep < 4; ++rep) {
    if (c->prec == OPE_FP64) {
      if (launch_resid0(c, X, nullptr, (double*)c->Rb[0], (double*)c->Y) != hipSuccess) return 1e30;
      if (launch_reduce_cols(c, c->part, c->stream_wgs, 2 * c->N, c->rho0, RED_PLAIN) != hipSuccess) return 1e30;
    } else {
      const size_t bytes = sizeof(float) * (size_t)c->n * (size_t)N;
      if (hipMemsetAsync(c->Rb[0], 0x3F, bytes, c->stream) != hipSuccess) return 1e30;
      if (hipMemsetAsync(c->Y, 0, bytes, c->stream) != hipSuccess) return 1e30;
      if (hipMemcpyAsync(c->rho0, rho.data(), sizeof(double) * 2 * N, hipMemcpyHostToDevice, c->stream) !=
          hipSuccess)
        return 1e30;
    }
    if (hipMemcpyAsync(c->cnorm2, c->rho0 + c->N, sizeof(double) * c->N, hipMemcpyDeviceToDevice, c->stream) !=
        hipSuccess)
      return 1e30;
    if (launch_solve_setup(c, c->rho0, 0.0) != hipSuccess) return 1e30;
    if (hipEventRecord(e0, c->stream) != hipSuccess) return 1e30;
    for (int it = 0; it < 8; ++it)
      if (cg_iteration(c, it) != hipSuccess) return 1e30;
    if (hipEventRecord(e1, c->stream) != hipSuccess) return 1e30;
    if (hipEventSynchronize(e1) != hipSuccess) return 1e30;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1e30;
    if (rep > 0 && ms < best) best = ms;      // the first run warms the caches and code
  }
  return best * 1e-3;
}

}  // namespace

ProfScope::ProfScope(ope_ctx* ctx, int kernel) : c(ctx), on(ctx->prof_kernel == kernel) {
  if (!on) return;
  if (c->prof_used + 2 > c->prof_events.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        on = false;
        return;
      }
      c->prof_events.push_back(e);
    }
  }
  (void)hipEventRecord(c->prof_events[c->prof_used], c->stream);
  c->prof_tags.resize(c->prof_used / 2 + 1);
  c->prof_tags[c->prof_used / 2] = c->prof_tag;
}

ProfScope::~ProfScope() {
  if (!on) return;
  (void)hipEventRecord(c->prof_events[c->prof_used + 1], c->stream);
  c->prof_used += 2;
}

// Line-tile level of sweep flags: 0 none, 1, 2, 3 for two, four, eight lines.
static int sweep_lines(int flags) {
  return (flags & OPE_SWEEP_LINES8) ? 3 : ((flags & OPE_SWEEP_LINES4) ? 2 : ((flags & OPE_SWEEP_LINES) ? 1 : 0));
}

// Default sweep flags: chunk-major, eight side lines per work-group on 3D
// grids (four where a pass holds fewer than 16 points; measured: four lines
// 5-17% faster than two at 64^3 and at 96^3 N = 128, 1-3% slower at 96^3
// N = 17, eight lines another 0.7-0.9% at N = 128), and non-temporal stores
// when the CG's working set (about five n x N blocks) exceeds the 256 MiB
// last-level cache.  Measured: streamed stores help once the sweeps' arrays
// cannot stay in that cache and cost while they can.

static int default_sweep_flags(const ope_ctx* c) {
  const double esz = c->prec == OPE_FP64 ? 8.0 : 4.0;
  const bool big = 5.0 * (double)c->n * (double)c->N * esz > 256.0 * 1048576.0;
  return OPE_SWEEP_CHUNK_MAJOR | (c->g.dim == 3 ? OPE_SWEEP_LINES8 : 0) | (big ? OPE_SWEEP_NONTEMPORAL : 0);
}

// Scratch of the allocation-free Gram (ope_gram_noalloc): the split-K
// partial sums, at most GRAM_NOALLOC_SPLITS x 128 x 128 doubles (4 MiB), in a
// file-scope device array.  Every GPU the library runs on holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in).  Calls that overlap on one GPU share it and race.
constexpr int64_t GRAM_NOALLOC_MAX = 128;
constexpr int64_t GRAM_NOALLOC_SPLITS = 32;
constexpr int64_t GRAM_NOALLOC_DOUBLES = GRAM_NOALLOC_SPLITS * GRAM_NOALLOC_MAX * GRAM_NOALLOC_MAX;
static __device__ __align__(256) double scratch[GRAM_NOALLOC_DOUBLES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// The device address of `scratch` on the current device (looked up once per device).
ope_status scratch_address(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OPE_EHIP;
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return OPE_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return OPE_EHIP;
    scratch_ptr[dev] = (double*)ptr;
  }
  *out = scratch_ptr[dev];
  return OPE_OK;
}
}  // namespace

extern "C" {

const char* ope_status_string(ope_status s) {
  switch (s) {
    case OPE_OK: return "ok";
    case OPE_EINVAL: return "invalid argument";
    case OPE_ENOMEM: return "out of memory";
    case OPE_EHIP: return "HIP runtime error";
    case OPE_ENONFINITE: return "non-finite value in a reduction";
    case OPE_ECG_MAXIT: return "inner CG reached its iteration cap";
    case OPE_EPIVOT: return "non-positive pivot in a small FP64 solve";
    case OPE_EUNSUPPORTED: return "not supported by the library";
    case OPE_ENOTSPD: return "operator is not symmetric positive definite";
  }
  return "unknown status";
}

ope_status ope_create(ope_ctx** out, const ope_op_desc* op, int64_t N, int32_t precision, void* stream) {
  if (!out) return OPE_EINVAL;
  *out = nullptr;
  if (!op || !op->V) return OPE_EINVAL;
  if (op->dim != 2 && op->dim != 3) return OPE_EINVAL;
  if (precision != OPE_FP64 && precision != OPE_MIXED) return OPE_EUNSUPPORTED;
  int64_t n = 1;
  for (int a = 0; a < op->dim; ++a) {
    if (op->m[a] < 1 || !(op->h[a] > 0.0)) return OPE_EINVAL;
    n *= op->m[a];
    if (n > (int64_t)1 << 31) return OPE_EINVAL;
  }
  if (!(op->kinetic > 0.0)) return OPE_EINVAL;
  if (N < 1 || N > n) return OPE_EINVAL;
  if (N > OPE_MAX_N_SMALL) return OPE_EUNSUPPORTED;
  // a point's row is split into 16-byte chunks (one element when N is odd),
  // at most one work-group's width of them
  if (N % 2 != 0 && N > OPE_WG) return OPE_EUNSUPPORTED;
  // the stencil sweeps address one plane of the march axis with 32-bit offsets
  const int64_t plane_pts = op->dim == 3 ? op->m[0] * op->m[1] : op->m[0];
  if (plane_pts * N * (int64_t)sizeof(double) >= ((int64_t)1 << 31)) return OPE_EUNSUPPORTED;

  ope_ctx* c = new (std::nothrow) ope_ctx();
  if (!c) return OPE_ENOMEM;
  c->prof_kernel = -1;
  c->prof_used = 0;
  c->prof_tag = -1;
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return OPE_EHIP;
  }
  c->n = n;
  c->N = N;
  c->prec = precision;
  if (precision == OPE_FP64) c->vw = (N % 2 == 0) ? 2 : 1;
  else c->vw = (N % 4 == 0) ? 4 : ((N % 2 == 0) ? 2 : 1);
  const size_t esz = precision == OPE_FP64 ? sizeof(double) : sizeof(float);
  OpeGrid& g = c->g;
  g.dim = op->dim;
  g.m0 = (uint32_t)op->m[0];
  g.m1 = (uint32_t)op->m[1];
  g.m2 = op->dim == 3 ? (uint32_t)op->m[2] : 1u;
  g.s1 = g.m0;
  g.s2 = g.m0 * g.m1;
  g.cx = op->kinetic / (op->h[0] * op->h[0]);
  g.cy = op->kinetic / (op->h[1] * op->h[1]);
  g.cz = op->dim == 3 ? op->kinetic / (op->h[2] * op->h[2]) : 0.0;
  c->h[0] = op->h[0];
  c->h[1] = op->h[1];
  c->h[2] = op->dim == 3 ? op->h[2] : op->h[1];
  c->kinetic = op->kinetic;
  c->eta_rel = ETA_REL_CG;
  c->eta_user = 0;
  c->eta_floor = precision == OPE_FP64 ? 1e-12 : 1e-6;
  c->max_iter = 2000;
  c->check_every = 4;
  c->use_graphs = 0;        // eager launches: measured about 2% faster than graph replays
  c->drift_tol = 2.5e-7;

  // streaming launch shape: about 2048 work-groups, whole passes of points
  const int64_t NV = N / c->vw;
  const int64_t pp = OPE_WG / NV;
  int64_t pts = (n + 2047) / 2048;
  pts = ((pts + pp - 1) / pp) * pp;
  if (pts < pp) pts = pp;
  c->stream_pts = (int)pts;
  c->stream_wgs = (int)((n + pts - 1) / pts);
  {
    const int f = default_sweep_flags(c);
    march_shape(c, 0, 0, 1, (f & OPE_SWEEP_NONTEMPORAL) ? 1 : 0, 0, sweep_lines(f));
  }

  const int64_t blk = n * N;
  const int64_t gtiles = ((N + 63) / 64) * ((N + 63) / 64);
  const int64_t ltiles = ((N + 127) / 128) * ((N + 127) / 128);   // 128 x 128 tiles of the LDS Gram
  int64_t gram_parts = ((1024 + gtiles - 1) / gtiles) * N * N;
  if (((512 + ltiles - 1) / ltiles) * N * N > gram_parts) gram_parts = ((512 + ltiles - 1) / ltiles) * N * N;
  const int64_t row_parts = ((n + 63) / 64) * N;
  int64_t pc = (int64_t)c->stream_wgs * 2 * N;
  if (march_rows(c) * N > pc) pc = march_rows(c) * N;
  if (gram_parts > pc) pc = gram_parts;
  if (row_parts > pc) pc = row_parts;
  c->part_cap = pc;
  c->stage_cap = 64 * (N * N > 2 * N ? N * N : 2 * N);

  std::vector<double> hd((size_t)n);
  const double dsum = 2.0 * (g.cx + g.cy + g.cz);
  for (int64_t p = 0; p < n; ++p) hd[(size_t)p] = op->V[p] + op->shift + dsum;

  bool ok = true;
  ok &= dalloc(&c->diag, n) == hipSuccess;
  // the five n x N blocks are allocated on first use (ensure_ws), or come from the caller
  (void)blk;
  (void)esz;
  if (precision == OPE_MIXED) {
    ok &= dalloc(&c->diag32, n) == hipSuccess;
    ok &= dalloc(&c->Lam32, N * N) == hipSuccess;
    ok &= dalloc(&c->Linv32, N * N) == hipSuccess;
    ok &= dalloc(&c->Sb32, N * N) == hipSuccess;
    ok &= dalloc(&c->Z32, 2 * N * N) == hipSuccess;
  }
  ok &= dalloc(&c->C, N * N) == hipSuccess;
  ok &= dalloc(&c->Lam, N * N) == hipSuccess;
  ok &= dalloc(&c->Linv, N * N) == hipSuccess;
  ok &= dalloc(&c->Sb, N * N) == hipSuccess;
  ok &= dalloc(&c->T, N * N) == hipSuccess;
  ok &= dalloc(&c->Z, 2 * N * N) == hipSuccess;
  ok &= dalloc(&c->A, N * N) == hipSuccess;
  ok &= dalloc(&c->B, N * N) == hipSuccess;
  ok &= dalloc(&c->Wsm, N * N) == hipSuccess;
  ok &= dalloc(&c->alpha, 2 * N) == hipSuccess;   // one half per CG iteration parity
  ok &= dalloc(&c->beta, N) == hipSuccess;
  ok &= dalloc(&c->rho, N) == hipSuccess;
  ok &= dalloc(&c->target, N) == hipSuccess;
  ok &= dalloc(&c->cnorm2, 2 * N) == hipSuccess;
  ok &= dalloc(&c->rcol, 2 * N) == hipSuccess;
  ok &= dalloc(&c->rho0, 2 * N) == hipSuccess;
  ok &= dalloc(&c->active, N) == hipSuccess;
  ok &= dalloc(&c->part, c->part_cap) == hipSuccess;
  ok &= dalloc(&c->stage, c->stage_cap) == hipSuccess;
  ok &= dalloc(&c->sc, 1) == hipSuccess;
  ok &= hipHostMalloc((void**)&c->hsc, sizeof(OpeScalars), hipHostMallocDefault) == hipSuccess;
  ok &= hipHostMalloc((void**)&c->hactive, sizeof(int32_t) * 2 * N, hipHostMallocDefault) == hipSuccess;
  for (int k = 0; k < 2; ++k) ok &= hipEventCreateWithFlags(&c->chunk_ev[k], hipEventDisableTiming) == hipSuccess;
  ok &= hipHostMalloc((void**)&c->hbuf, sizeof(double) * 2 * N, hipHostMallocDefault) == hipSuccess;
  ok &= hipHostMalloc((void**)&c->hsc2, sizeof(OpeScalars), hipHostMallocDefault) == hipSuccess;
  if (N > OPE_MAX_N_ONE_WG) {
    const int64_t t = (N + 63) / 64;
    ok &= dalloc(&c->ns_x[0], N * N) == hipSuccess;
    ok &= dalloc(&c->ns_x[1], N * N) == hipSuccess;
    ok &= dalloc(&c->ns_g, N * N) == hipSuccess;
    ok &= dalloc(&c->ns_m, N * N) == hipSuccess;
    ok &= dalloc(&c->ns_p, N * N) == hipSuccess;
    ok &= dalloc(&c->ns_part, t * t) == hipSuccess;
    ok &= dalloc(&c->ns, 1) == hipSuccess;
    ok &= hipHostMalloc((void**)&c->hns, sizeof(NsState), hipHostMallocDefault) == hipSuccess;
  }
  if (!ok) {
    free_ctx(c);
    return OPE_ENOMEM;
  }
  bool hok = true;
  hok &= hipMemcpy(c->diag, hd.data(), sizeof(double) * n, hipMemcpyHostToDevice) == hipSuccess;
  if (precision == OPE_MIXED) {
    std::vector<float> hf((size_t)n);
    for (int64_t p = 0; p < n; ++p) hf[(size_t)p] = (float)hd[(size_t)p];
    hok &= hipMemcpy(c->diag32, hf.data(), sizeof(float) * n, hipMemcpyHostToDevice) == hipSuccess;
  }
  hok &= hipMemset(c->sc, 0, sizeof(OpeScalars)) == hipSuccess;
  hok &= hipMemset(c->active, 0, sizeof(int32_t) * N) == hipSuccess;
  hok &= hipDeviceSynchronize() == hipSuccess;
  if (!hok) {
    free_ctx(c);
    return OPE_EHIP;
  }
  // Coercivity (Section 2.2): H must be SPD for G = H^{-1} to exist.  The
  // smallest eigenvalue is at least lambda_min(c (-Lap_h)) + min(V + shift)
  // (Weyl), a closed form; when that bound is not positive a Lanczos run on
  // the device decides: a Ritz value <= 0 proves an eigenvalue <= 0.
  double lap_min = 0.0, vmin = 1e300;
  for (int a = 0; a < op->dim; ++a) {
    const double sn = std::sin(M_PI / (2.0 * (double)(op->m[a] + 1)));
    lap_min += op->kinetic * 4.0 * sn * sn / (op->h[a] * op->h[a]);
  }
  for (int64_t p = 0; p < n; ++p) vmin = std::min(vmin, op->V[p] + op->shift);
  if (!(std::isfinite(vmin))) {
    free_ctx(c);
    return OPE_EINVAL;
  }
  if (!(lap_min + vmin > 0.0)) {
    double lo = 0.0, hi = 0.0;
    int its = 0;
    if (lanczos_extremes(c, 1000, &lo, &hi, &its) != hipSuccess) {
      free_ctx(c);
      return OPE_EHIP;
    }
    c->lz_done = 1;
    c->lz_min = lo;
    c->lz_max = hi;
    c->lz_iters = its;
    if (!(lo > 0.0)) {
      free_ctx(c);
      return OPE_ENOTSPD;
    }
  }
  *out = c;
  return OPE_OK;
}

ope_status ope_destroy(ope_ctx* c) {
  if (!c) return OPE_OK;
  (void)hipStreamSynchronize(c->stream);
  free_ctx(c);
  return OPE_OK;
}

ope_status ope_set_inner(ope_ctx* c, double eta_rel, double eta_floor, int32_t max_iter) {
  if (!c || !(eta_rel >= 0.0) || !(eta_floor >= 0.0) || max_iter < 1) return OPE_EINVAL;
  c->eta_rel = eta_rel;
  c->eta_floor = eta_floor;
  c->max_iter = max_iter;
  c->eta_user = 1;
  return OPE_OK;
}

ope_status ope_apply_h(ope_ctx* c, const void* X, void* Y) {
  if (!c || !X || !Y || X == Y) return OPE_EINVAL;
  HIPCHK(launch_apply_h(c, X, Y));
  return OPE_OK;
}

ope_status ope_source_solve(ope_ctx* c, const double* U, double* Y, const double* Y0, double tol, int32_t max_iter,
                            int32_t* iterations) {
  if (!c || !U || !Y || !(tol >= 0.0) || max_iter < 0) return OPE_EINVAL;
  if (U == Y) return OPE_EINVAL;
  if (c->prec != OPE_FP64) return OPE_EUNSUPPORTED;
  WSCHK(c);
  const int N = (int)c->N;
  c->cg_on_d = 0;                // this CG iterates on Y
  // r0 = U - H Y0, column norms of r0 and of U
  if (Y0) {
    HIPCHK(launch_apply_h(c, Y0, c->HU));
    HIPCHK(launch_resid0(c, U, (const double*)c->HU, (double*)c->Rb[0], nullptr));
  } else {
    HIPCHK(launch_resid0(c, U, nullptr, (double*)c->Rb[0], (double*)c->Y));
  }
  HIPCHK(launch_reduce_cols(c, c->part, c->stream_wgs, 2 * N, c->rho0, RED_PLAIN));
  HIPCHK(hipMemcpyAsync(c->cnorm2, c->rho0 + N, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(launch_solve_setup(c, c->rho0, tol));
  if (c->mg_on) HIPCHK(pcg_begin(c));
  if (Y0) HIPCHK(hipMemcpyAsync(c->Y, Y0, sizeof(double) * c->n * N, hipMemcpyDeviceToDevice, c->stream));
  int32_t iters = 0;
  bool done = false;
  ope_status st = run_cg(c, max_iter, &iters, &done);
  if (st != OPE_OK) return st;
  HIPCHK(hipMemcpyAsync(Y, c->Y, sizeof(double) * c->n * N, hipMemcpyDeviceToDevice, c->stream));
  st = sync_and_read_scalars(c);
  if (st != OPE_OK) return st;
  if (iterations) *iterations = c->hsc->cg_iters;
  if (c->hsc->err != 0) return (ope_status)c->hsc->err;
  if (!done) {
    // the last chunk may have converged exactly at the cap
    HIPCHK(hipMemcpy(c->hactive, c->active, sizeof(int32_t) * N, hipMemcpyDeviceToHost));
    int cnt = 0;
    for (int j = 0; j < N; ++j) cnt += c->hactive[j] != 0;
    if (cnt) return OPE_ECG_MAXIT;
  }
  return OPE_OK;
}

ope_status ope_gram(ope_ctx* c, const double* A, int64_t lda, int64_t na, const double* B, int64_t ldb, int64_t nb,
                    int64_t rows, double* out) {
  if (!c || !A || !B || !out) return OPE_EINVAL;
  if (na < 1 || nb < 1 || na > 512 || nb > 512 || lda < na || ldb < nb || rows < 0) return OPE_EINVAL;
  if (na * nb > c->part_cap) return OPE_EUNSUPPORTED;
  if (rows == 0) {
    HIPCHK(hipMemsetAsync(out, 0, sizeof(double) * na * nb, c->stream));
    return OPE_OK;
  }
  HIPCHK(launch_gram(c, A, lda, (int)na, B, ldb, (int)nb, rows, out));
  return OPE_OK;
}

ope_status ope_gram_noalloc(const double* A, int64_t lda, int64_t na, const double* B, int64_t ldb, int64_t nb,
                            int64_t rows, double* out, void* stream) {
  if (!A || !B || !out) return OPE_EINVAL;
  if (na < 1 || nb < 1 || lda < na || ldb < nb || rows < 1 || rows > ((int64_t)1 << 32) - 1) return OPE_EINVAL;
  if (na > GRAM_NOALLOC_MAX || nb > GRAM_NOALLOC_MAX) return OPE_EINVAL;   // beyond the fixed scratch
  double* part = nullptr;
  const ope_status st = scratch_address(&part);
  if (st != OPE_OK) return st;
  // a context-free view for the shared launchers: the partial sums live in the
  // scratch array, there is no stage buffer (the column sums then run in one
  // pass), no timing and no per-step scalars
  ope_ctx v{};
  v.stream = (hipStream_t)stream;
  v.part = part;
  v.part_cap = GRAM_NOALLOC_SPLITS * na * nb;
  v.stage = nullptr;
  v.stage_cap = 0;
  v.prof_kernel = -1;
  v.prof_used = 0;
  v.prof_tag = -1;
  HIPCHK(launch_gram(&v, A, lda, (int)na, B, ldb, (int)nb, rows, out));
  return OPE_OK;
}

ope_status ope_small_solve(ope_ctx* c, const double* Sb, const double* T, double tau, double* Z, double* A,
                           double* B) {
  if (!c || !Sb || !T || !Z || !(tau > 0.0)) return OPE_EINVAL;
  if (c->prec != OPE_FP64) return OPE_EUNSUPPORTED;
  HIPCHK(hipMemsetAsync(&c->sc->err, 0, sizeof(int32_t), c->stream));
  HIPCHK(launch_small_solve(c, Sb, T, tau, Z, A, B));
  ope_status st = sync_and_read_scalars(c);
  if (st != OPE_OK) return st;
  return (ope_status)c->hsc->err;
}

ope_status ope_update(ope_ctx* c, double* U, const double* Y, const double* Z) {
  if (!c || !U || !Y || !Z || U == Y) return OPE_EINVAL;
  if (c->prec != OPE_FP64) return OPE_EUNSUPPORTED;
  WSCHK(c);
  const size_t NN = (size_t)c->N * c->N;
  int64_t np = 0;
  if (c->N <= 128) {
    HIPCHK(launch_rowmm(c, U, Z, Y, Z + NN, nullptr, 0.0, 1.0, U, 0, 0, &np));
  } else {
    HIPCHK(launch_rowmm(c, U, Z, Y, Z + NN, nullptr, 0.0, 1.0, (double*)c->Pb, 0, 0, &np));
    HIPCHK(hipMemcpyAsync(U, c->Pb, sizeof(double) * (size_t)c->n * c->N, hipMemcpyDeviceToDevice, c->stream));
  }
  return OPE_OK;
}

ope_status ope_energy(ope_ctx* c, const void* U, double* energy) {
  if (!c || !U || !energy) return OPE_EINVAL;
  WSCHK(c);
  ope_status st = phase_residual(c, U);
  if (st != OPE_OK) return st;
  st = sync_and_read_scalars(c);
  if (st != OPE_OK) return st;
  *energy = c->hsc->energy;
  return c->hsc->err == OPE_ENONFINITE ? OPE_ENONFINITE : OPE_OK;
}

ope_status ope_residual(ope_ctx* c, const void* U, double* residual, double* ritz, double* drift) {
  if (!c || !U) return OPE_EINVAL;
  WSCHK(c);
  const int N = (int)c->N;
  ope_status st = phase_residual(c, U);
  if (st != OPE_OK) return st;
  HIPCHK(launch_cg_setup(c, c->rcol));   // computes the residual scalar from the column norms
  if (ritz) {
    HIPCHK(launch_jacobi_eig(c, c->Lam, c->rho0));
    HIPCHK(hipMemcpyAsync(c->hbuf, c->rho0, sizeof(double) * N, hipMemcpyDeviceToHost, c->stream));
  }
  st = sync_and_read_scalars(c);
  if (st != OPE_OK) return st;
  if (residual) *residual = c->hsc->residual;
  if (drift) *drift = c->hsc->drift;
  if (ritz) memcpy(ritz, c->hbuf, sizeof(double) * N);
  return c->hsc->err == OPE_ENONFINITE ? OPE_ENONFINITE : OPE_OK;
}

ope_status ope_set_graphs(ope_ctx* c, int32_t enable) {
  if (!c || (enable != 0 && enable != 1)) return OPE_EINVAL;
  c->use_graphs = enable;
  if (c->mg_on) {
    HIPCHK(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->check_every = mg_check_every(c);
  }
  return OPE_OK;
}

ope_status ope_set_multigrid(ope_ctx* c, int32_t enable) {
  if (!c || (enable != 0 && enable != 1)) return OPE_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);               // the captured CG chunks hold the other iteration
  if (!enable) {
    mg_free(c);
    c->check_every = 4;
    if (!c->eta_user) c->eta_rel = ETA_REL_CG;
    return OPE_OK;
  }
  // one thread per row chunk of a point: at most 256 chunks per row
  const int64_t vw = c->prec == OPE_FP64 ? (c->N % 2 == 0 ? 2 : 1) : (c->N % 4 == 0 ? 4 : (c->N % 2 == 0 ? 2 : 1));
  if (c->N / vw > 256) return OPE_EUNSUPPORTED;
  const ope_status st = mg_build(c);
  if (st != OPE_OK) return st;
  c->mg_on = 1;
  c->check_every = mg_check_every(c);
  if (!c->eta_user) c->eta_rel = ETA_REL_MG;
  return OPE_OK;
}

ope_status ope_set_recycle(ope_ctx* c, int32_t enable) {
  if (!c || (enable != 0 && enable != 1)) return OPE_EINVAL;
  if (c->prec != OPE_FP64 || c->has_mass || c->in_batch) return OPE_EUNSUPPORTED;
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  c->have_d = 0;
  c->cg_on_d = 0;
  if (!enable) {
    if (c->Dr) (void)hipFree(c->Dr);
    if (c->HDr) (void)hipFree(c->HDr);
    c->Dr = c->HDr = nullptr;
    c->recycle = 0;
    return OPE_OK;
  }
  const size_t bytes = sizeof(double) * (size_t)c->n * (size_t)c->N;
  if (!c->Dr && hipMalloc(&c->Dr, bytes) != hipSuccess) {
    c->Dr = nullptr;
    return OPE_ENOMEM;
  }
  if (!c->HDr && hipMalloc(&c->HDr, bytes) != hipSuccess) {
    c->HDr = nullptr;
    return OPE_ENOMEM;
  }
  c->recycle = 1;
  return OPE_OK;
}

ope_status ope_mg_info(const ope_ctx* c, int32_t* levels, int64_t* coarsest_nodes) {
  if (!c) return OPE_EINVAL;
  if (levels) *levels = c->mg_on ? c->mg_levels : 0;
  if (coarsest_nodes) *coarsest_nodes = c->mg_on ? c->mg[c->mg_levels - 1].n : 0;
  return OPE_OK;
}

ope_status ope_mg_vcycle(ope_ctx* c, const void* R, void* Zo) {
  if (!c || !R || !Zo || R == (const void*)Zo) return OPE_EINVAL;
  if (!c->mg_on) return OPE_EINVAL;
  if (((((uintptr_t)R) | ((uintptr_t)Zo)) & 15u) != 0) return OPE_EINVAL;
  HIPCHK(mg_vcycle(c, R, Zo, nullptr, false));
  HIPCHK(hipStreamSynchronize(c->stream));
  return OPE_OK;
}

ope_status ope_set_sweep_shape(ope_ctx* c, int32_t q_max, int32_t march_chunks, int32_t flags) {
  if (!c || !(q_max == 0 || q_max == 1 || q_max == 2 || q_max == 4) || march_chunks < 0 || (flags & ~63))
    return OPE_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  const MarchShape keep = c->ms;
  march_shape(c, q_max, march_chunks, flags & OPE_SWEEP_CHUNK_MAJOR, flags & OPE_SWEEP_NONTEMPORAL,
              flags & OPE_SWEEP_NARROW,
              sweep_lines(flags));
  if (march_rows(c) * c->N > c->part_cap) {
    c->ms = keep;
    return OPE_EINVAL;
  }
  return OPE_OK;
}

ope_status ope_get_sweep_shape(const ope_ctx* c, int32_t* q, int32_t* march_chunks, int32_t* workgroups) {
  if (!c) return OPE_EINVAL;
  if (q) *q = (int32_t)c->ms.q;
  if (march_chunks) *march_chunks = (int32_t)c->ms.mc;
  if (workgroups) *workgroups = (int32_t)(c->ms.lgroups * c->ms.nxs * c->ms.cc * c->ms.mc);
  return OPE_OK;
}

ope_status ope_profile_begin(ope_ctx* c, int32_t kernel) {
  if (!c || kernel < 0 || kernel >= OPE_KERNEL_COUNT) return OPE_EINVAL;
  c->prof_kernel = kernel;
  c->prof_used = 0;
  return OPE_OK;
}

ope_status ope_profile_end_launches(ope_ctx* c, ope_kernel_time* out, int32_t* tags, double* ms, int64_t cap) {
  if (!c || !out || cap < 0 || (cap > 0 && (!tags || !ms))) return OPE_EINVAL;
  c->prof_kernel = -1;
  HIPCHK(hipStreamSynchronize(c->stream));
  double total = 0.0;
  for (size_t k = 0; k + 1 < c->prof_used; k += 2) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, c->prof_events[k], c->prof_events[k + 1]));
    total += t;
    const int64_t i = (int64_t)(k / 2);
    if (i < cap) {
      tags[i] = c->prof_tags[i];
      ms[i] = t;
    }
  }
  out->launches = (int64_t)(c->prof_used / 2);
  out->total_ms = total;
  c->prof_used = 0;
  return OPE_OK;
}

ope_status ope_profile_end(ope_ctx* c, ope_kernel_time* out) {
  return ope_profile_end_launches(c, out, nullptr, nullptr, 0);
}

ope_status ope_step(ope_ctx* c, void* U, double tau, ope_step_info* info) {
  if (!c || !U || !(tau > 0.0)) return OPE_EINVAL;
  WSCHK(c);
  return run_step(c, U, tau, info, -1.0, nullptr);
}

ope_status ope_convert(ope_ctx* c, const void* src, void* dst, int64_t count, int32_t to_double) {
  if (!c || !src || !dst || count < 0 || src == dst) return OPE_EINVAL;
  if (count == 0) return OPE_OK;
  HIPCHK(launch_convert(c, src, dst, count, to_double));
  return OPE_OK;
}

ope_status ope_gram_f32(ope_ctx* c, int32_t kind, const float* A, int64_t lda, int64_t na, const float* B,
                        int64_t ldb, int64_t nb, int64_t rows, double* out) {
  if (!c || !A || !B || !out || kind < MK_F64 || kind > MK_BF16) return OPE_EINVAL;
  if (na < 1 || nb < 1 || na > 512 || nb > 512 || lda < na || ldb < nb || rows < 1) return OPE_EINVAL;
  if (na * nb > c->part_cap) return OPE_EUNSUPPORTED;
  HIPCHK(launch_gram_f32(c, kind, A, lda, (int)na, B, ldb, (int)nb, rows, out));
  return OPE_OK;
}

ope_status ope_rowmm_f32(ope_ctx* c, int32_t kind, const float* X0, const float* M0, const float* X1,
                         const float* M1, const float* Cm, double cbeta, double ascale, float* Out) {
  if (!c || !X0 || !M0 || !Out || (X1 && !M1) || (cbeta != 0.0 && !Cm) || (kind != MK_F32 && kind != MK_BF16))
    return OPE_EINVAL;
  if (c->N > 128 && (Out == X0 || Out == X1)) return OPE_EUNSUPPORTED;
  int64_t np = 0;
  HIPCHK(launch_rowmm_f32(c, kind, X0, M0, X1, M1, Cm, cbeta, ascale, Out, 0, 0, &np));
  return OPE_OK;
}

ope_status ope_solve(ope_ctx* c, void* U, double tau, double res_tol, int32_t max_steps, ope_solve_info* info) {
  if (!c || !U || !(tau > 0.0) || !(res_tol >= 0.0) || max_steps < 0) return OPE_EINVAL;
  WSCHK(c);
  ope_solve_info si;
  memset(&si, 0, sizeof(si));
  ope_status st = OPE_OK;
  c->have_d = 0;                 // a solve starts without a recycled correction
  if (c->net) {
    st = solve_learned(c, U, tau, res_tol, max_steps, &si);
    if (info) *info = si;
    return st;
  }
  double best = 1e300;
  int32_t since_best = 0;
  for (;;) {
    ope_step_info s;
    bool conv = false;
    const bool last = si.steps >= max_steps || si.stalled;
    // the final pass only evaluates the iterate (a residual of 1e300 is always reached)
    st = run_step(c, U, tau, &s, last ? 1e300 : res_tol, &conv);
    if (st != OPE_OK && st != OPE_ECG_MAXIT) break;
    si.residual = s.residual;
    si.energy = s.energy;
    si.drift = s.drift;
    if (conv) {
      si.converged = s.residual <= res_tol;
      st = OPE_OK;
      break;
    }
    si.steps += 1;
    si.inner_iterations += s.inner_iterations;
    // the reduced-precision form stops improving at its rounding floor
    if (s.residual < 0.9 * best) {
      best = s.residual;
      since_best = 0;
    } else if (c->prec == OPE_MIXED && ++since_best >= 60) {
      si.stalled = 1;
    }
  }
  if (info) *info = si;
  return st;
}

// Residual phase and Step-1 warm start of the current iterate, scalars on the host.
static ope_status prepare_iterate(ope_ctx* c, void* U) {
  ope_status st = phase_residual(c, U);
  if (st != OPE_OK) return st;
  st = phase_warm_start(c, U);
  if (st != OPE_OK) return st;
  st = sync_and_read_scalars(c);
  if (st != OPE_OK) return st;
  return (ope_status)c->hsc->err;
}

// Algorithm 1 with the step chosen in [tau_min, tau_max]: a step whose energy
// rises above the current one (Theorem 4.2: below a threshold step the energy
// decays) is redone from the saved iterate with the step shrunk, never below
// tau_min; after an accepted step the next one grows, never above tau_max.
static ope_status solve_adaptive(ope_ctx* c, void* U, const ope_solve_opts* o, ope_solve_info* si) {
  const bool adaptive = o->tau_min < o->tau_max;
  const size_t bytes = (c->prec == OPE_FP64 ? sizeof(double) : sizeof(float)) * (size_t)c->n * (size_t)c->N;
  if (adaptive && !c->Ubak) {
    if (balloc(&c->Ubak, sizeof(double) * (size_t)c->n * (size_t)c->N) != hipSuccess) return OPE_ENOMEM;
  }
  const double slack = 1e-13;
  const bool use_ref = !std::isnan(o->energy_ref);
  double tau = o->tau;
  ope_status st = prepare_iterate(c, U);
  if (st != OPE_OK) return st;
  double E = c->hsc->energy, res = c->hsc->residual, drift = c->hsc->drift;
  c->drift_seen = drift;
  double errE = std::fabs(E);
  double best = 1e300;
  int32_t since_best = 0;
  for (;;) {
    si->residual = res;
    si->energy = E;
    si->drift = drift;
    si->tau = tau;
    if (o->res_tol >= 0.0 && res <= o->res_tol) {
      si->converged = 1;
      break;
    }
    if (o->energy_tol >= 0.0) {
      const bool stop = use_ref ? (E - o->energy_ref) / std::fabs(o->energy_ref) <= o->energy_tol
                                : errE <= o->energy_tol;
      if (stop) {
        si->converged = 1;
        break;
      }
    }
    if (si->steps >= o->max_steps || si->stalled) break;
    double E_new = 0.0;
    for (;;) {
      if (adaptive) HIPCHK(hipMemcpyAsync(c->Ubak, U, bytes, hipMemcpyDeviceToDevice, c->stream));
      int32_t iters = 0;
      bool cg_done = false;
      st = run_cg(c, c->max_iter, &iters, &cg_done);
      if (st != OPE_OK) return st;
      st = recycle_after_cg(c);
      if (st != OPE_OK) return st;
      st = phase_update(c, U, tau);
      if (st != OPE_OK) return st;
      HIPCHK(hipMemcpyAsync(c->hsc2, c->sc, sizeof(OpeScalars), hipMemcpyDeviceToHost, c->stream));
      st = phase_residual(c, U);
      if (st == OPE_OK) st = phase_warm_start(c, U);
      if (st == OPE_OK) st = sync_and_read_scalars(c);
      if (st != OPE_OK) return st;
      if (c->hsc2->err != 0) return (ope_status)c->hsc2->err;    // the step failed; U is unchanged
      if (c->hsc->err != 0) return (ope_status)c->hsc->err;
      E_new = c->hsc->energy;
      if (adaptive && !(E_new <= E + slack * std::fabs(E)) && tau > o->tau_min) {
        HIPCHK(hipMemcpyAsync(U, c->Ubak, bytes, hipMemcpyDeviceToDevice, c->stream));
        si->rejected += 1;
        tau = std::max(o->tau_min, o->shrink * tau);
        st = prepare_iterate(c, U);
        if (st != OPE_OK) return st;
        continue;
      }
      si->inner_iterations += c->hsc2->cg_iters;
      break;
    }
    errE = std::fabs(E_new - E) / std::fabs(E);
    E = E_new;
    res = c->hsc->residual;
    drift = c->hsc->drift;
    c->drift_seen = drift;
    si->steps += 1;
    tau = std::min(o->tau_max, o->grow * tau);
    if (res < 0.9 * best) {
      best = res;
      since_best = 0;
    } else if (c->prec == OPE_MIXED && ++since_best >= 60) {
      si->stalled = 1;
    }
  }
  return OPE_OK;
}

ope_status ope_solve_ex(ope_ctx* c, void* U, const ope_solve_opts* o, ope_solve_info* info) {
  if (!c || !U || !o) return OPE_EINVAL;
  if (!(o->tau_min > 0.0) || !(o->tau_min <= o->tau) || !(o->tau <= o->tau_max) || !(o->grow >= 1.0) ||
      !(o->shrink > 0.0 && o->shrink < 1.0) || o->max_steps < 0 || std::isinf(o->tau_max))
    return OPE_EINVAL;
  if (!std::isnan(o->energy_ref) && !(std::fabs(o->energy_ref) > 0.0)) return OPE_EINVAL;
  if (c->net) return OPE_EUNSUPPORTED;
  WSCHK(c);
  ope_solve_info si;
  memset(&si, 0, sizeof(si));
  c->have_d = 0;                 // a solve starts without a recycled correction
  const ope_status st = solve_adaptive(c, U, o, &si);
  if (info) *info = si;
  return st;
}

ope_status ope_set_preconditioner(ope_ctx* c, ope_net* net, int32_t judge) {
  if (!c) return OPE_EINVAL;
  if (!net) {
    c->net = nullptr;
    return OPE_OK;
  }
  if (net->ctx != c || net->max_batch < c->N || (judge != 0 && judge != 1)) return OPE_EINVAL;
  if (c->prec != OPE_FP64 || c->N > 128 || c->has_mass) return OPE_EUNSUPPORTED;
  c->net_judge = judge;
  if (judge && !c->Ubak) {
    if (balloc(&c->Ubak, sizeof(double) * (size_t)c->n * (size_t)c->N) != hipSuccess) return OPE_ENOMEM;
  }
  c->net = net;
  return OPE_OK;
}

ope_status ope_step_learned(ope_ctx* c, void* U, double tau, ope_step_info* info, int32_t* accepted) {
  if (!c || !U || !(tau > 0.0)) return OPE_EINVAL;
  WSCHK(c);
  ope_status st = check_learned(c);
  if (st != OPE_OK) return st;
  if (accepted) *accepted = 0;
  st = phase_residual(c, U);
  if (st != OPE_OK) return st;
  HIPCHK(launch_cg_setup(c, c->rcol));
  st = sync_and_read_scalars(c);
  if (st != OPE_OK) return st;
  if (c->hsc->err != 0) {
    fill_info(c, info, 0, (ope_status)c->hsc->err);
    return (ope_status)c->hsc->err;
  }
  ope_step_info in;
  memset(&in, 0, sizeof(in));
  in.energy = c->hsc->energy;
  in.residual = c->hsc->residual;
  in.drift = c->hsc->drift;
  bool acc = false;
  ope_step_info plain;
  memset(&plain, 0, sizeof(plain));
  st = learned_core(c, U, tau, &acc, &plain);
  in.inner_iterations = acc ? 0 : plain.inner_iterations;
  in.status = st;
  if (info) *info = in;
  if (accepted) *accepted = acc ? 1 : 0;
  return st;
}

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
ope_status ope_batch_create(ope_batch** out, const ope_op_desc* ops, const int64_t* N, int32_t count,
                            int32_t precision, void* stream) {
  if (!out) return OPE_EINVAL;
  *out = nullptr;
  if (!ops || !N || count < 1 || count > 4096) return OPE_EINVAL;
  ope_batch* b = new (std::nothrow) ope_batch();
  if (!b) return OPE_ENOMEM;
  b->count = count;
  b->user = (hipStream_t)stream;
  b->ctx.assign(count, nullptr);
  b->streams.assign(count, nullptr);
  b->done.assign(count, nullptr);
  ope_status st = OPE_OK;
  if (hipEventCreateWithFlags(&b->start, hipEventDisableTiming) != hipSuccess) st = OPE_EHIP;
  for (int32_t i = 0; i < count && st == OPE_OK; ++i) {
    if (hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming) != hipSuccess) {
      st = OPE_EHIP;
      break;
    }
    st = ope_create(&b->ctx[i], &ops[i], N[i], precision, b->streams[i]);
    if (st == OPE_OK) b->ctx[i]->in_batch = 1;
  }
  b->shared = 0;   // per-problem launches: measured as fast as tuned shared launches
  b->flag_off.assign(count, 0);
  if (st == OPE_OK) {
    int64_t nflags = 0;
    for (int32_t i = 0; i < count; ++i) nflags += N[i];
    bool ok = hipStreamCreateWithFlags(&b->cg_stream, hipStreamNonBlocking) == hipSuccess;
    ok &= hipEventCreateWithFlags(&b->cg_ev, hipEventDisableTiming) == hipSuccess;
    ok &= hipMalloc((void**)&b->d_mjobs, sizeof(MarchJob) * 4 * (size_t)count) == hipSuccess;
    ok &= hipHostMalloc((void**)&b->h_mjobs, sizeof(MarchJob) * 4 * (size_t)count, hipHostMallocDefault) == hipSuccess;
    ok &= hipMalloc((void**)&b->d_rjobs, sizeof(ReduceJob) * (size_t)count) == hipSuccess;
    ok &= hipHostMalloc((void**)&b->h_rjobs, sizeof(ReduceJob) * (size_t)count, hipHostMallocDefault) == hipSuccess;
    ok &= hipMalloc((void**)&b->d_flags, sizeof(int32_t) * (size_t)nflags) == hipSuccess;
    ok &= hipHostMalloc((void**)&b->h_flags, sizeof(int32_t) * (size_t)nflags, hipHostMallocDefault) == hipSuccess;
    if (!ok) st = OPE_ENOMEM;
  }
  if (st != OPE_OK) {
    ope_batch_destroy(b);
    return st;
  }
  *out = b;
  return OPE_OK;
}

ope_status ope_batch_set_shared(ope_batch* b, int32_t shared) {
  if (!b || (shared != 0 && shared != 1)) return OPE_EINVAL;
  b->shared = shared;
  return OPE_OK;
}

ope_status ope_batch_destroy(ope_batch* b) {
  if (!b) return OPE_OK;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    if (b->ctx[i]) ope_destroy(b->ctx[i]);
    if (b->streams[i]) (void)hipStreamDestroy(b->streams[i]);
    if (b->done[i]) (void)hipEventDestroy(b->done[i]);
  }
  if (b->start) (void)hipEventDestroy(b->start);
  if (b->cg_ev) (void)hipEventDestroy(b->cg_ev);
  for (hipStream_t cs : b->cls_streams) (void)hipStreamDestroy(cs);
  for (hipEvent_t ce : b->cls_events) (void)hipEventDestroy(ce);
  if (b->cg_stream) (void)hipStreamDestroy(b->cg_stream);
  if (b->d_mjobs) (void)hipFree(b->d_mjobs);
  if (b->d_rjobs) (void)hipFree(b->d_rjobs);
  if (b->d_flags) (void)hipFree(b->d_flags);
  if (b->h_mjobs) (void)hipHostFree(b->h_mjobs);
  if (b->h_rjobs) (void)hipHostFree(b->h_rjobs);
  if (b->h_flags) (void)hipHostFree(b->h_flags);
  if (b->step_graph) (void)hipGraphExecDestroy(b->step_graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->cap_fork) (void)hipEventDestroy(b->cap_fork);
  if (b->cap_join) (void)hipEventDestroy(b->cap_join);
  if (b->d_gmjobs) (void)hipFree(b->d_gmjobs);
  if (b->d_grjobs) (void)hipFree(b->d_grjobs);
  if (b->d_gflags) (void)hipFree(b->d_gflags);
  if (b->h_gflags) (void)hipHostFree(b->h_gflags);
  delete b;
  return OPE_OK;
}

ope_status ope_batch_context(ope_batch* b, int32_t i, ope_ctx** ctx) {
  if (!b || !ctx || i < 0 || i >= b->count) return OPE_EINVAL;
  *ctx = b->ctx[i];
  return OPE_OK;
}

ope_status ope_batch_step(ope_batch* b, void* const* U, double tau, ope_step_info* info) {
  if (!b || !U || !(tau > 0.0)) return OPE_EINVAL;
  for (int32_t i = 0; i < b->count; ++i)
    if (!U[i]) return OPE_EINVAL;
  BatchState bs;
  std::vector<char> run(b->count, 1);
  ope_status st = batch_round(b, U, tau, -1.0, run, bs);
  if (st != OPE_OK) return st;
  ope_status first = OPE_OK;
  for (int32_t i = 0; i < b->count; ++i) {
    if (info) {
      info[i] = bs.info[i];
      info[i].status = bs.st[i];
    }
    if (first == OPE_OK && bs.st[i] != OPE_OK) first = bs.st[i];
  }
  return first;
}

ope_status ope_batch_solve(ope_batch* b, void* const* U, double tau, double res_tol, int32_t max_steps,
                           ope_solve_info* info) {
  if (!b || !U || !(tau > 0.0) || !(res_tol >= 0.0) || max_steps < 0) return OPE_EINVAL;
  for (int32_t i = 0; i < b->count; ++i)
    if (!U[i]) return OPE_EINVAL;
  const int P = b->count;
  std::vector<ope_solve_info> si(P);
  for (auto& x : si) memset(&x, 0, sizeof(x));
  std::vector<char> live(P, 1);
  std::vector<ope_status> fail(P, OPE_OK);
  BatchState bs;
  for (;;) {
    // problems at their step limit are only evaluated in this round
    std::vector<char> run(P, 0), eval_only(P, 0);
    bool any = false;
    for (int i = 0; i < P; ++i) {
      if (!live[i]) continue;
      run[i] = 1;
      any = true;
      eval_only[i] = si[i].steps >= max_steps;
    }
    if (!any) break;
    // problems at their step limit take an evaluation-only round (any residual passes)
    std::vector<char> run_step_set(P, 0), run_eval_set(P, 0);
    for (int i = 0; i < P; ++i) {
      run_step_set[i] = run[i] && !eval_only[i];
      run_eval_set[i] = run[i] && eval_only[i];
    }
    for (int pass = 0; pass < 2; ++pass) {
      const std::vector<char>& set = pass == 0 ? run_step_set : run_eval_set;
      bool has = false;
      for (int i = 0; i < P; ++i) has |= set[i] != 0;
      if (!has) continue;
      ope_status st = batch_round(b, U, tau, pass == 0 ? res_tol : 1e300, set, bs);
      if (st != OPE_OK) return st;
      for (int i = 0; i < P; ++i) {
        if (!set[i]) continue;
        const ope_status s = bs.st[i];
        if (s != OPE_OK && s != OPE_ECG_MAXIT) {
          fail[i] = s;
          live[i] = 0;
          continue;
        }
        si[i].residual = bs.info[i].residual;
        si[i].energy = bs.info[i].energy;
        si[i].drift = bs.info[i].drift;
        if (bs.conv[i]) {
          si[i].converged = bs.info[i].residual <= res_tol;
          live[i] = 0;
          continue;
        }
        si[i].steps += 1;
        si[i].inner_iterations += bs.info[i].inner_iterations;
      }
    }
  }
  ope_status first = OPE_OK;
  for (int i = 0; i < P; ++i) {
    if (info) info[i] = si[i];
    if (first == OPE_OK && fail[i] != OPE_OK) first = fail[i];
  }
  return first;
}

ope_status ope_batch_capture(ope_batch* b, void* const* U, double tau, int32_t cg_iterations) {
  if (!b || !U || !(tau > 0.0) || cg_iterations < 2 || cg_iterations % 2 != 0) return OPE_EINVAL;
  const int P = b->count;
  int64_t nflags = 0;
  for (int i = 0; i < P; ++i) {
    if (!U[i]) return OPE_EINVAL;
    ope_ctx* c = b->ctx[i];
    // one-work-group small solves (no host check) and one-work-group column sums
    if (c->N > OPE_MAX_N_ONE_WG || c->prof_kernel >= 0) return OPE_EUNSUPPORTED;
    ope_status st = ensure_ws(c);
    if (st != OPE_OK) return st;
    nflags += c->N;
  }
  HIPCHK(hipDeviceSynchronize());
  if (b->step_graph) {
    HIPCHK(hipGraphExecDestroy(b->step_graph));
    b->step_graph = nullptr;
  }
  if (!b->cap_stream) {
    HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&b->cap_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&b->cap_join, hipEventDisableTiming));
    if (hipMalloc((void**)&b->d_gmjobs, sizeof(MarchJob) * 4 * (size_t)P) != hipSuccess ||
        hipMalloc((void**)&b->d_grjobs, sizeof(ReduceJob) * (size_t)P) != hipSuccess ||
        hipMalloc((void**)&b->d_gflags, sizeof(int32_t) * (size_t)nflags) != hipSuccess ||
        hipHostMalloc((void**)&b->h_gflags, sizeof(int32_t) * (size_t)nflags, hipHostMallocDefault) != hipSuccess)
      return OPE_ENOMEM;
  }
  // problems in the shared launches (the batch's launch mode), the others run
  // their CG on their own streams; flags of both kinds land in h_gflags
  std::vector<int> members;
  std::vector<char> shared(P, 0);
  for (int i = 0; i < P; ++i)
    if (b->shared && shared_fits(b->ctx[i])) {
      shared[i] = 1;
      members.push_back(i);
    }
  CgPlan pl;
  if (!members.empty()) {
    plan_cg(b, members, b->d_gflags, pl);
    HIPCHK(hipMemcpy(b->d_gmjobs, b->h_mjobs, sizeof(MarchJob) * pl.jobs, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_grjobs, b->h_rjobs, sizeof(ReduceJob) * pl.M, hipMemcpyHostToDevice));
  }
  b->gflag_off.assign(P, 0);
  uint32_t foff = pl.flags;
  for (int i = 0; i < P; ++i) {
    if (shared[i]) {
      b->gflag_off[i] = b->flag_off[i];
    } else {
      b->gflag_off[i] = foff;
      foff += (uint32_t)b->ctx[i]->N;
    }
  }
  hipStream_t cs = b->cap_stream;
  HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  auto finish = [&](int i) -> ope_status {    // Steps 2-4, scalars to the host, join
    ope_ctx* c = b->ctx[i];
    ope_status st = phase_update(c, U[i], tau);
    if (st != OPE_OK) return st;
    HIPCHK(hipMemcpyAsync(c->hsc, c->sc, sizeof(OpeScalars), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipEventRecord(b->done[i], c->stream));
    HIPCHK(hipStreamWaitEvent(cs, b->done[i], 0));
    return OPE_OK;
  };
  auto body = [&]() -> ope_status {
    HIPCHK(hipEventRecord(b->cap_fork, cs));
    for (int i = 0; i < P; ++i) {
      ope_ctx* c = b->ctx[i];
      HIPCHK(hipStreamWaitEvent(c->stream, b->cap_fork, 0));
      ope_status st = phase_residual(c, U[i]);
      if (st == OPE_OK) st = phase_warm_start(c, U[i]);
      if (st != OPE_OK) return st;
      if (shared[i]) {
        HIPCHK(hipEventRecord(b->done[i], c->stream));
        HIPCHK(hipStreamWaitEvent(cs, b->done[i], 0));
        continue;
      }
      // own launches, the whole step on the problem's stream
      for (int32_t it = 0; it < cg_iterations; ++it) HIPCHK(cg_iteration(c, it));
      HIPCHK(cg_flush(c, cg_iterations, c->stream));
      HIPCHK(hipMemcpyAsync(b->h_gflags + b->gflag_off[i], c->active, sizeof(int32_t) * c->N,
                            hipMemcpyDeviceToHost, c->stream));
      if ((st = finish(i)) != OPE_OK) return st;
    }
    if (members.empty()) return OPE_OK;
    HIPCHK(enqueue_cg(b, pl, b->d_gmjobs, b->d_grjobs, 0, cg_iterations, cs));
    HIPCHK(launch_gather_flags(cs, b->d_grjobs, pl.M));
    HIPCHK(hipMemcpyAsync(b->h_gflags, b->d_gflags, sizeof(int32_t) * pl.flags, hipMemcpyDeviceToHost, cs));
    HIPCHK(hipEventRecord(b->cap_join, cs));
    for (int i : members) {
      HIPCHK(hipStreamWaitEvent(b->ctx[i]->stream, b->cap_join, 0));
      ope_status st = finish(i);
      if (st != OPE_OK) return st;
    }
    return OPE_OK;
  };
  const ope_status st = body();
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(cs, &g);
  if (st != OPE_OK || ee != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return st != OPE_OK ? st : OPE_EHIP;
  }
  const hipError_t ie = hipGraphInstantiate(&b->step_graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    b->step_graph = nullptr;
    return OPE_EHIP;
  }
  b->cap_iters = cg_iterations;
  return OPE_OK;
}

ope_status ope_batch_replay(ope_batch* b, ope_step_info* info) {
  if (!b) return OPE_EINVAL;
  if (!b->step_graph) return OPE_EINVAL;
  HIPCHK(hipGraphLaunch(b->step_graph, b->user));
  if (!info) return OPE_OK;
  HIPCHK(hipStreamSynchronize(b->user));
  ope_status first = OPE_OK;
  for (int i = 0; i < b->count; ++i) {
    ope_ctx* c = b->ctx[i];
    const OpeScalars& sc = *c->hsc;
    ope_status st = (ope_status)sc.err;
    if (st == OPE_OK) {
      const int32_t* f = b->h_gflags + b->gflag_off[i];
      for (int64_t j = 0; j < c->N; ++j)
        if (f[j] != 0) st = OPE_ECG_MAXIT;
    }
    info[i].energy = sc.energy;
    info[i].residual = sc.residual;
    info[i].drift = sc.drift;
    info[i].inner_iterations = sc.cg_iters;
    info[i].status = st;
    c->drift_seen = sc.drift;
    if (first == OPE_OK && st != OPE_OK) first = st;
  }
  return first;
}

namespace {

struct TunedShape {
  int q, mc, flags;
};

// The fastest sweep shape of a context for short CG runs (FP64: on the
// scratch right-hand side X, n x N; FP32: X unused): passes per plane 1/2 or the two-, four- and
// eight-line tiles, work-group order, non-temporal stores, column chunking,
// and the automatic march-chunk count times 1/2, 1, 3/2 or 2.  Leaves the
// context on the last shape tried.
TunedShape tune_shape(ope_ctx* c, const double* X, hipEvent_t e0, hipEvent_t e1) {
  const uint32_t NV = (uint32_t)(c->N / c->vw);
  TunedShape pick{2, 0, default_sweep_flags(c)};
  double tbest = 1e30;
  const int narrow_opts = NV <= 32 ? 2 : 1;
  // qs = 3, 4 and 5 stand for the two-, four- and eight-line tiles (q 2)
  for (int qs : {1, 2, 3, 4, 5})
    for (int cm : {0, OPE_SWEEP_CHUNK_MAJOR})
      for (int nt : {0, OPE_SWEEP_NONTEMPORAL})
        for (int nr = 0; nr < narrow_opts; ++nr)
          for (int mcm : {2, 4, 6, 8}) {     // the automatic count times mcm / 4
            if (qs >= 3 && c->g.dim != 3) continue;
            const int q = qs >= 3 ? 2 : qs;
            const int flags = cm | nt | (nr ? OPE_SWEEP_NARROW : 0) | (qs == 3 ? OPE_SWEEP_LINES : 0) |
                              (qs == 4 ? OPE_SWEEP_LINES4 : 0) | (qs == 5 ? OPE_SWEEP_LINES8 : 0);
            if (ope_set_sweep_shape(c, q, 0, flags) != OPE_OK) continue;
            int mc = 0;
            if (mcm != 4) {
              mc = ((int)c->ms.mc * mcm + 2) / 4;
              if (mc < 1) mc = 1;
              if (mc == (int)c->ms.mc) continue;       // the automatic count, timed with mcm = 4
              if (ope_set_sweep_shape(c, q, mc, flags) != OPE_OK) continue;
            }
            const double t = time_cg(c, X, e0, e1);
            if (t < tbest) {
              tbest = t;
              pick = TunedShape{q, mc, flags};
            }
          }
  return pick;
}

}  // namespace

ope_status ope_autotune(ope_ctx* c) {
  if (!c) return OPE_EINVAL;
  WSCHK(c);
  HIPCHK(hipStreamSynchronize(c->stream));
  void* X = nullptr;                                // FP64: the scratch right-hand side
  const size_t bytes = c->prec == OPE_FP64 ? sizeof(double) * (size_t)c->n * (size_t)c->N : 0;
  if (bytes && hipMalloc(&X, bytes) != hipSuccess) return OPE_ENOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipFree(X);
    return OPE_EHIP;
  }
  // any non-zero right-hand side (the sweeps' cost does not depend on it)
  ope_status st = (!X || hipMemsetAsync(X, 0x3F, bytes, c->stream) == hipSuccess) ? OPE_OK : OPE_EHIP;
  if (st == OPE_OK) {
    const TunedShape t = tune_shape(c, (const double*)X, e0, e1);
    if (ope_set_sweep_shape(c, t.q, t.mc, t.flags) != OPE_OK) (void)ope_set_sweep_shape(c, 2, 0, default_sweep_flags(c));
    if (hipStreamSynchronize(c->stream) != hipSuccess) st = OPE_EHIP;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (X) (void)hipFree(X);
  return st;
}

ope_status ope_batch_autotune(ope_batch* b, int32_t* tuned_keys) {
  if (!b) return OPE_EINVAL;
  if (b->step_graph) {       // its job tables hold the old sweep shapes
    (void)hipGraphExecDestroy(b->step_graph);
    b->step_graph = nullptr;
  }
  // bucket of a problem: grid edge and vector-column count, each in steps of 8
  struct Key {
    int dim, prec, vw;
    uint32_t mx, my, mz, nv;
    bool operator<(const Key& o) const {
      return std::tie(dim, prec, vw, mx, my, mz, nv) < std::tie(o.dim, o.prec, o.vw, o.mx, o.my, o.mz, o.nv);
    }
  };
  std::map<Key, TunedShape> best;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return OPE_EHIP;
  }
  ope_status status = OPE_OK;
  for (int32_t i = 0; i < b->count && status == OPE_OK; ++i) {
    ope_ctx* c = b->ctx[i];
    const uint32_t NV = (uint32_t)(c->N / c->vw);
    const Key k{c->g.dim, c->prec, c->vw, (c->g.m0 + 7) / 8, (c->g.m1 + 7) / 8, (c->g.m2 + 7) / 8, (NV + 7) / 8};
    status = ensure_ws(c);
    if (status != OPE_OK) break;
    auto f = best.find(k);
    if (f == best.end()) {
      void* X = nullptr;                          // FP64: the scratch right-hand side
      const size_t bytes = c->prec == OPE_FP64 ? sizeof(double) * (size_t)c->n * (size_t)c->N : 0;
      if (bytes && hipMalloc(&X, bytes) != hipSuccess) {
        status = OPE_ENOMEM;
        break;
      }
      // any non-zero right-hand side (the sweeps' cost does not depend on it)
      if (X) (void)hipMemsetAsync(X, 0x3F, bytes, c->stream);
      const TunedShape pick = tune_shape(c, (const double*)X, e0, e1);
      (void)hipStreamSynchronize(c->stream);
      if (X) (void)hipFree(X);
      best[k] = pick;
      f = best.find(k);
    }
    if (ope_set_sweep_shape(c, f->second.q, f->second.mc, f->second.flags) != OPE_OK) {
      // a shape tuned on a bucket neighbour may not fit this problem's partial buffer
      (void)ope_set_sweep_shape(c, 2, 0, default_sweep_flags(c));
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (tuned_keys) *tuned_keys = (int32_t)best.size();
  return status;
}


ope_status ope_spectrum_bounds(ope_ctx* c, double* lmin, double* lmax) {
  if (!c) return OPE_EINVAL;
  if (!c->lz_done) {
    double lo = 0.0, hi = 0.0;
    int its = 0;
    HIPCHK(lanczos_extremes(c, 1000, &lo, &hi, &its));
    c->lz_done = 1;
    c->lz_min = lo;
    c->lz_max = hi;
    c->lz_iters = its;
  }
  if (lmin) *lmin = c->lz_min;
  if (lmax) *lmax = c->lz_max;
  return OPE_OK;
}

ope_status ope_workspace_size(const ope_ctx* c, size_t* bytes) {
  if (!c || !bytes) return OPE_EINVAL;
  *bytes = 5 * ws_block_bytes(c);
  return OPE_OK;
}

ope_status ope_set_workspace(ope_ctx* c, void* dptr, size_t bytes) {
  if (!c) return OPE_EINVAL;
  if (dptr && (bytes < 5 * ws_block_bytes(c) || (reinterpret_cast<uintptr_t>(dptr) % 256) != 0)) return OPE_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  if (c->ws_own) {
    HIPCHK(hipFree(c->ws_own));
    c->ws_own = nullptr;
  }
  c->HU = c->Y = c->Rb[0] = c->Rb[1] = c->Pb = nullptr;
  c->ws_ext = dptr;
  c->ws_ext_bytes = dptr ? bytes : 0;
  if (dptr) return ensure_ws(c);
  return OPE_OK;
}

ope_status ope_set_mass(ope_ctx* c, const double* d, const double* mu) {
  if (!c) return OPE_EINVAL;
  if (!d) {
    c->has_mass = 0;
    return OPE_OK;
  }
  if (!mu) return OPE_EINVAL;
  if (c->prec != OPE_FP64 || c->net || c->N > 256) return OPE_EUNSUPPORTED;
  const int dims = c->g.dim;
  double off = 0.0;
  for (int a = 0; a < dims; ++a) {
    if (!std::isfinite(mu[a])) return OPE_EINVAL;
    off += 2.0 * std::fabs(mu[a]);
  }
  // strict diagonal dominance with a positive diagonal: M is SPD (Gershgorin)
  for (int64_t p = 0; p < c->n; ++p)
    if (!std::isfinite(d[p])) return OPE_EINVAL;
  for (int64_t p = 0; p < c->n; ++p)
    if (!(d[p] > off)) return OPE_ENOTSPD;
  if (!c->mdiag && dalloc(&c->mdiag, c->n) != hipSuccess) return OPE_ENOMEM;
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(c->mdiag, d, sizeof(double) * c->n, hipMemcpyHostToDevice));
  for (int a = 0; a < 3; ++a) c->mass_mu[a] = a < dims ? mu[a] : 0.0;
  c->has_mass = 1;
  drop_graphs(c);
  return OPE_OK;
}

ope_status ope_apply_mass(ope_ctx* c, const double* X, double* Y) {
  if (!c || !X || !Y || X == Y) return OPE_EINVAL;
  if (!c->has_mass) return OPE_EINVAL;
  HIPCHK(apply_mass(c, X, Y));
  return OPE_OK;
}

ope_status ope_orthonormalize(ope_ctx* c, double* U) {
  if (!c || !U) return OPE_EINVAL;
  if (c->prec != OPE_FP64) return OPE_EUNSUPPORTED;
  WSCHK(c);
  const int N = (int)c->N;
  int64_t np = 0;
  if (c->has_mass) {
    HIPCHK(apply_mass(c, U, c->Rb[1]));
    HIPCHK(launch_gram(c, U, N, N, (const double*)c->Rb[1], N, N, c->n, c->Wsm));
  } else {
    HIPCHK(launch_gram(c, U, N, N, U, N, N, c->n, c->Wsm));
  }
  HIPCHK(hipMemsetAsync(&c->sc->err, 0, sizeof(int32_t), c->stream));
  HIPCHK(launch_chol_rinv(c, c->Wsm, c->Z));
  if (N <= 128) {
    HIPCHK(launch_rowmm(c, U, c->Z, nullptr, nullptr, nullptr, 0.0, 1.0, U, 0, ROWMM_IF_OK, &np));
  } else {
    HIPCHK(launch_rowmm(c, U, c->Z, nullptr, nullptr, nullptr, 0.0, 1.0, (double*)c->Pb, 0, ROWMM_IF_OK, &np));
    HIPCHK(launch_copy_pred(c, c->Pb, U, sizeof(double) * (uint64_t)c->n * N));
  }
  ope_status st = sync_and_read_scalars(c);
  if (st != OPE_OK) return st;
  return (ope_status)c->hsc->err;
}

ope_status ope_energy_d(ope_ctx* c, const void* U, double* d_energy) {
  if (!c || !U || !d_energy) return OPE_EINVAL;
  WSCHK(c);
  ope_status st = phase_residual(c, U);
  if (st != OPE_OK) return st;
  HIPCHK(launch_scalar_copy(c, 0, d_energy));
  return OPE_OK;
}

ope_status ope_residual_d(ope_ctx* c, const void* U, double* d_residual, double* d_drift) {
  if (!c || !U || (!d_residual && !d_drift)) return OPE_EINVAL;
  WSCHK(c);
  ope_status st = phase_residual(c, U);
  if (st != OPE_OK) return st;
  HIPCHK(launch_cg_setup(c, c->rcol));   // computes the residual scalar from the column norms
  if (d_residual) HIPCHK(launch_scalar_copy(c, 1, d_residual));
  if (d_drift) HIPCHK(launch_scalar_copy(c, 2, d_drift));
  return OPE_OK;
}

// Blocks with a leading dimension other than N go through a packed staging
// block: copy in, the packed entry point, copy out (steps only).
static ope_status pack_in(ope_ctx* c, const void* U, int64_t ldu) {
  const size_t esz = c->prec == OPE_FP64 ? sizeof(double) : sizeof(float);
  if (!c->Upk && balloc(&c->Upk, esz * (size_t)c->n * (size_t)c->N) != hipSuccess) return OPE_ENOMEM;
  HIPCHK(hipMemcpy2DAsync(c->Upk, esz * c->N, U, esz * (size_t)ldu, esz * c->N, (size_t)c->n,
                          hipMemcpyDeviceToDevice, c->stream));
  return OPE_OK;
}

static ope_status unpack_out(ope_ctx* c, void* U, int64_t ldu) {
  const size_t esz = c->prec == OPE_FP64 ? sizeof(double) : sizeof(float);
  HIPCHK(hipMemcpy2DAsync(U, esz * (size_t)ldu, c->Upk, esz * c->N, esz * c->N, (size_t)c->n,
                          hipMemcpyDeviceToDevice, c->stream));
  return OPE_OK;
}

ope_status ope_step_ld(ope_ctx* c, void* U, int64_t ldu, double tau, ope_step_info* info) {
  if (!c || !U || !(tau > 0.0) || ldu < c->N) return OPE_EINVAL;
  if (ldu == c->N) return ope_step(c, U, tau, info);
  ope_status st = pack_in(c, U, ldu);
  if (st != OPE_OK) return st;
  st = ope_step(c, c->Upk, tau, info);
  if (st != OPE_OK && st != OPE_ECG_MAXIT) return st;
  const ope_status st2 = unpack_out(c, U, ldu);
  if (st2 != OPE_OK) return st2;
  HIPCHK(hipStreamSynchronize(c->stream));
  return st;
}

ope_status ope_energy_ld(ope_ctx* c, const void* U, int64_t ldu, double* energy) {
  if (!c || !U || !energy || ldu < c->N) return OPE_EINVAL;
  if (ldu == c->N) return ope_energy(c, U, energy);
  ope_status st = pack_in(c, U, ldu);
  if (st != OPE_OK) return st;
  return ope_energy(c, c->Upk, energy);
}

ope_status ope_residual_ld(ope_ctx* c, const void* U, int64_t ldu, double* residual, double* ritz, double* drift) {
  if (!c || !U || ldu < c->N) return OPE_EINVAL;
  if (ldu == c->N) return ope_residual(c, U, residual, ritz, drift);
  ope_status st = pack_in(c, U, ldu);
  if (st != OPE_OK) return st;
  return ope_residual(c, c->Upk, residual, ritz, drift);
}

}  // extern "C"
