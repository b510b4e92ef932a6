// Host orchestration and C ABI of the SNMPBB library (see include/snmf.h).
//
// One outer iteration = W-step then H-step (Section 2.1).  A half-step with variable X
// and partner P launches, in stream order:
//   gram(P) -> rho(G) -> A-pass(P) -> [L X] -> init -> inner_iters x (step1, step2)
// with the Laplacian path (H-step of Graph-SNMPBB) splitting step1/step2 around the
// sparse products L(Z-X), <D, L D> and L S.  All iteration scalars stay on the device;
// every kernel returns at once when the device "done" flag is set, so an outer
// iteration can be captured once as a hipGraph and replayed.  The host only reads the
// flag every check_every outer iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/snmf.h"
#include "common.hpp"
#include "host.hpp"
#include "kernels.hpp"

using namespace snmf;

namespace snmf {
std::string& err_ref() {
  thread_local std::string e;
  return e;
}
}  // namespace snmf

struct snmf_plan {
  snmf_matrix A{};
  snmf_matrix L{};
  snmf_params p{};
  bool lap = false;
  int r = 0;
  int64_t n = 0;
  int prec = SNMF_F32;
  size_t esz = 4;
  hipStream_t s = nullptr;     // private stream of the plan (default priority)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // device memory (one allocation, carved)
  void* pool = nullptr;
  void *Wb = nullptr, *Hb = nullptr, *C = nullptr, *g = nullptr, *Z = nullptr, *D = nullptr;
  void* gs = nullptr;
  void *Bpart = nullptr, *LT = nullptr, *LX = nullptr, *GT[2] = {nullptr, nullptr}, *TT = nullptr;
  double* G64[2] = {nullptr, nullptr};
  double *part = nullptr, *gram_part = nullptr, *lai_part = nullptr, *dots = nullptr;
  double *partsA = nullptr, *partsB = nullptr, *partsC = nullptr, *partsD = nullptr;
  double* trace = nullptr;
  uint16_t *Ahi = nullptr, *Alo = nullptr, *Pthi = nullptr, *Ptlo = nullptr;
  int64_t ldb = 0;
  State* st = nullptr;
  unsigned* counters = nullptr;
  unsigned* flags = nullptr;
  DenseSplit ds{};
  int gram_blocks = 1;
  int grid = 1;  // workgroups of every row-tile kernel of the plan (one partial-sum layout)
  double normA2 = 0.0;
  KParams kp{};
  // captured outer iterations: one, and kGraphRun of them back to back (one launch per
  // run saves the per-launch gap between outer iterations)
  hipGraph_t graph = nullptr, graph_run = nullptr;
  hipGraphExec_t gexec = nullptr, gexec_run = nullptr;
  // the allocation-free solve: pool is the library's static scratch and s the caller's
  // stream, neither owned by the plan
  bool borrowed = false;

  ~snmf_plan() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (gexec_run) (void)hipGraphExecDestroy(gexec_run);
    if (graph_run) (void)hipGraphDestroy(graph_run);
    if (borrowed) return;
    if (pool) (void)hipFree(pool);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (s) (void)hipStreamDestroy(s);
  }
};

namespace snmf {

snmf_status check_params(const snmf_params* p) {
  if (!p) return fail(SNMF_E_ARG, "params is NULL");
  if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) return fail(SNMF_E_ARG, "lambda must be >= 0");
  if (!(p->gamma >= 0.0) || !std::isfinite(p->gamma)) return fail(SNMF_E_ARG, "gamma must be >= 0");
  if (!(p->eta >= 0.0 && p->eta < 1.0)) return fail(SNMF_E_ARG, "eta must lie in [0, 1)");
  if (!(p->theta > 0.0 && p->theta < 1.0)) return fail(SNMF_E_ARG, "theta must lie in (0, 1)");
  if (!(p->phi > 0.0) || !std::isfinite(p->phi)) return fail(SNMF_E_ARG, "phi must be > 0");
  if (!(p->alpha_min > 0.0 && p->alpha_min < p->alpha_max) || !std::isfinite(p->alpha_max))
    return fail(SNMF_E_ARG, "need 0 < alpha_min < alpha_max < inf");
  if (!(p->beta_shrink > 0.0 && p->beta_shrink < 1.0))
    return fail(SNMF_E_ARG, "beta_shrink must lie in (0, 1)");
  if (p->max_ls < 0) return fail(SNMF_E_ARG, "max_ls must be >= 0");
  if (p->inner_iters < 1 || p->inner_iters > kMaxInner)
    return fail(SNMF_E_ARG, "inner_iters must lie in [1, 64]");
  if (p->max_outer < 1) return fail(SNMF_E_ARG, "max_outer must be >= 1");
  if (!(p->target_res >= 0.0)) return fail(SNMF_E_ARG, "target_res must be >= 0");
  if (p->prec < SNMF_F64 || p->prec > SNMF_BF16X3) return fail(SNMF_E_ARG, "unknown precision");
  if (p->fuse_inner != 0 && p->fuse_inner != 1) return fail(SNMF_E_ARG, "fuse_inner must be 0 or 1");
  if (p->accept_at_relaxed && p->project_update)
    return fail(SNMF_E_UNSUPPORTED,
                "accept_at_relaxed needs project_update = 0 (the projected relaxed point has "
                "no closed-form objective)");
  return SNMF_OK;
}

snmf_status check_matrix(const snmf_matrix* A, const char* what) {
  if (!A) return fail(SNMF_E_ARG, std::string(what) + " is NULL");
  if (A->n < 1) return fail(SNMF_E_SHAPE, std::string(what) + ": n must be >= 1");
  switch (A->fmt) {
    case SNMF_DENSE:
      if (!A->dense) return fail(SNMF_E_ARG, std::string(what) + ": dense pointer is NULL");
      if (A->ld < A->n) return fail(SNMF_E_SHAPE, std::string(what) + ": ld < n");
      break;
    case SNMF_CSR:
      if (!A->rowptr || (A->nnz > 0 && (!A->col || !A->val)))
        return fail(SNMF_E_ARG, std::string(what) + ": CSR pointer is NULL");
      if (A->nnz < 0) return fail(SNMF_E_SHAPE, std::string(what) + ": nnz < 0");
      if (A->n >= (int64_t)1 << 31) return fail(SNMF_E_SHAPE, std::string(what) + ": n >= 2^31");
      break;
    case SNMF_LOWRANK:
      if (!A->U || !A->lam) return fail(SNMF_E_ARG, std::string(what) + ": U or lam is NULL");
      if (A->ell < 1 || A->ell > kMaxEll)
        return fail(SNMF_E_SHAPE, std::string(what) + ": ell must lie in [1, 128]");
      break;
    default:
      return fail(SNMF_E_ARG, std::string(what) + ": unknown format");
  }
  return SNMF_OK;
}

KParams kparams_of(const snmf_params& p, bool lap) {
  KParams k{};
  k.lam = p.lambda;
  k.gamma = lap ? p.gamma : 0.0;
  k.eta = p.eta;
  k.theta = p.theta;
  k.phi = p.phi;
  k.amin = p.alpha_min;
  k.amax = p.alpha_max;
  k.shrink = p.beta_shrink;
  k.target = p.target_res;
  k.max_ls = p.max_ls;
  k.relaxed = p.accept_at_relaxed;
  k.project = p.project_update;
  k.max_outer = p.max_outer;
  return k;
}

}  // namespace snmf

namespace {

template <typename T>
snmf_status stats(snmf_plan* pl, const T* x, int64_t rows, int64_t cols, int64_t ld, double* out3) {
  launch_stats2d<T>(x, rows, cols, ld, pl->part, pl->dots, pl->counters + C_NORM, pl->s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out3, pl->dots, 3 * sizeof(double), hipMemcpyDeviceToHost, pl->s));
  HIP_TRY(hipStreamSynchronize(pl->s));
  return SNMF_OK;
}

snmf_status stats_any(snmf_plan* pl, const void* x, int64_t rows, int64_t cols, int64_t ld,
                      double* out3) {
  if (pl->prec == SNMF_F64) return stats<double>(pl, (const double*)x, rows, cols, ld, out3);
  return stats<float>(pl, (const float*)x, rows, cols, ld, out3);
}

snmf_status check_values(const double* st3, const char* what) {
  if (st3[2] > 0) return fail(SNMF_E_NONFINITE, std::string(what) + " has NaN/Inf entries");
  if (st3[1] > 0) return fail(SNMF_E_NEGATIVE, std::string(what) + " has negative entries");
  return SNMF_OK;
}

}  // namespace

namespace snmf {
// Opt-in symmetry check of a dense matrix (params.check_symmetry): E_NOT_SYMMETRIC when an
// entry and its mirror differ by more than kSymTol of the larger.
snmf_status check_dense_symmetry(const snmf_matrix* M, int prec, unsigned* flags, hipStream_t s,
                                 const char* what) {
  HIP_TRY(hipMemsetAsync(flags, 0, 4 * sizeof(unsigned), s));
  if (prec == SNMF_F64)
    launch_dense_symmetry<double>((const double*)M->dense, M->n, M->ld, kSymTol, flags, s);
  else
    launch_dense_symmetry<float>((const float*)M->dense, M->n, M->ld, kSymTol, flags, s);
  HIP_TRY(hipGetLastError());
  unsigned f[4];
  HIP_TRY(hipMemcpyAsync(f, flags, sizeof(f), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (f[3]) return fail(SNMF_E_NOT_SYMMETRIC, std::string(what) + " is not symmetric (" +
                                                  std::to_string(f[3]) + " mismatched entries)");
  return SNMF_OK;
}
}  // namespace snmf

namespace {

snmf_status check_csr(snmf_plan* pl, const snmf_matrix* M, const char* what, bool need_nonneg,
                      double* sumsq) {
  HIP_TRY(hipMemsetAsync(pl->flags, 0, 4 * sizeof(unsigned), pl->s));
  launch_csr_structure(M->rowptr, M->col, M->n, M->nnz, pl->flags, pl->s);
  HIP_TRY(hipGetLastError());
  unsigned f[4];
  HIP_TRY(hipMemcpyAsync(f, pl->flags, sizeof(f), hipMemcpyDeviceToHost, pl->s));
  HIP_TRY(hipStreamSynchronize(pl->s));
  if (f[0] || f[1]) return fail(SNMF_E_SHAPE, std::string(what) + ": malformed CSR structure");
  if (pl->p.validate && f[2] == 0) {
    if (pl->prec == SNMF_F64)
      launch_csr_symmetry<double>(M->rowptr, M->col, (const double*)M->val, M->n, pl->flags, pl->s);
    else
      launch_csr_symmetry<float>(M->rowptr, M->col, (const float*)M->val, M->n, pl->flags, pl->s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(f, pl->flags, sizeof(f), hipMemcpyDeviceToHost, pl->s));
    HIP_TRY(hipStreamSynchronize(pl->s));
    if (f[3]) return fail(SNMF_E_NOT_SYMMETRIC, std::string(what) + " is not symmetric");
  }
  double st3[3] = {0, 0, 0};
  if (M->nnz > 0) SNMF_TRY(stats_any(pl, M->val, 1, M->nnz, M->nnz, st3));
  if (st3[2] > 0) return fail(SNMF_E_NONFINITE, std::string(what) + " has NaN/Inf entries");
  if (need_nonneg && st3[1] > 0) return fail(SNMF_E_NEGATIVE, std::string(what) + " has negative entries");
  if (sumsq) *sumsq = st3[0];
  return SNMF_OK;
}

// outer iterations per replay of the multi-iteration graph
constexpr int kGraphRun = 8;

// ------------------------------------------------------------------ one half-step
// B = A P (partials in Bpart).  With rj.G set, rho = ||G||_2 as well: in one more
// workgroup of the A-pass launch (FP64 dense: a launch of its own just before it).
template <typename T>
snmf_status apass(snmf_plan* pl, const T* P, hipStream_t s, const RhoJob& rj = RhoJob{}) {
  const int64_t n = pl->n;
  const int r = pl->r;
  const int32_t* gate = &pl->st->done;
  if (rj.G && pl->A.fmt == SNMF_DENSE && pl->prec == SNMF_F64) {
    launch_rho(rj.G, rj.r, rj.st, s);
    HIP_TRY(hipGetLastError());
  }
  switch (pl->A.fmt) {
    case SNMF_DENSE:
      if (pl->prec == SNMF_F64) {
        launch_apass_f64((const double*)pl->A.dense, pl->A.ld, (const double*)P, n, r,
                         (double*)pl->Bpart, pl->st, s);
      } else if (pl->prec == SNMF_F32) {
        launch_apass_f32((const float*)pl->A.dense, pl->A.ld, (const float*)P, n, r, pl->ds,
                         (float*)pl->Bpart, n * r, pl->st, s, rj);
      } else {
        launch_split_pt((const float*)P, n, r, pl->ldb, pl->Pthi, pl->Ptlo, pl->st, s);
        launch_apass_bf16x3(pl->Ahi, pl->Alo, pl->ldb, pl->Pthi, pl->Ptlo, pl->ldb, n, r, pl->ds,
                            (float*)pl->Bpart, n * r, pl->st, s, rj);
      }
      break;
    case SNMF_CSR:
      launch_spmm<T>(pl->A.rowptr, pl->A.col, (const T*)pl->A.val, P, n, r, (T*)pl->Bpart, nullptr,
                     nullptr, gate, nullptr, s, rj);
      break;
    default:
      launch_lai<T>((const T*)pl->A.U, (int)pl->A.ell, pl->A.lam, P, n, r, pl->lai_part,
                    (T*)pl->TT, (T*)pl->Bpart, gate, s, rj);
      break;
  }
  HIP_TRY(hipGetLastError());
  return SNMF_OK;
}

int ksplit_of(const snmf_plan* pl) {
  return (pl->A.fmt == SNMF_DENSE && pl->prec != SNMF_F64) ? pl->ds.ksplit : 1;
}

// Start of a half-step up to and including init: G, rho (in or just before the A-pass,
// on the same stream: a second stream would cost more in cross-queue waits than rho
// takes), the A-pass and the gradient.  The first reader of rho is the first inner kernel.
// Inner iterations of this half-step run as fused kernels, one per inner iteration
// (fused_inner_ok), on every half-step without the Laplacian term except the H-step of
// the naive variant.
bool fused_half(const snmf_plan* pl, int is_hstep) {
  return fused_inner_ok(pl->p) && !(pl->lap && is_hstep) && !(pl->p.naive && is_hstep);
}

// dir: init also forms the fused path's direction 0 (fused_half).
template <typename T>
snmf_status half_start(snmf_plan* pl, T* X, const T* P, int is_hstep, bool with_rho,
                       hipStream_t s, bool dir = false) {
  const int64_t n = pl->n;
  const int r = pl->r;
  const int gi = is_hstep ? 1 : 0;
  launch_gram<T>(P, n, r, pl->gram_part, pl->gram_blocks, pl->G64[gi], (T*)pl->GT[gi], pl->st, s);
  HIP_TRY(hipGetLastError());
  RhoJob rj;
  if (with_rho) {
    rj.G = pl->G64[gi];
    rj.r = r;
    rj.st = pl->st;
  }
  SNMF_TRY(apass<T>(pl, P, s, rj));
  const bool lap = pl->lap && is_hstep;
  if (lap) {
    launch_spmm<T>(pl->L.rowptr, pl->L.col, (const T*)pl->L.val, X, n, r, (T*)pl->LX, nullptr,
                   nullptr, &pl->st->done, nullptr, s);
  }
  launch_init<T>(X, P, (const T*)pl->Bpart, ksplit_of(pl), n * r, (T*)pl->C, (T*)pl->g,
                 lap ? (const T*)pl->LX : nullptr, (const T*)pl->GT[gi], n, r, is_hstep, pl->kp,
                 pl->st, pl->partsA, s, BMap{}, pl->grid, lap ? (T*)pl->Z : nullptr,
                 lap ? (T*)pl->D : nullptr, dir ? (T*)pl->D : nullptr,
                 dir ? pl->partsB : nullptr, dir ? (T*)pl->Z : nullptr,
                 dir ? (T*)pl->gs : nullptr);
  HIP_TRY(hipGetLastError());
  return SNMF_OK;
}

// One inner iteration k (Algorithm 1, lines 2-4).  Without a Laplacian: step1, step2.
// H-step of Graph-SNMPBB: step1 phase 1, L(Z-X), step1 phase 2, <D, L D>, step2 phase 1,
// L S, step2 phase 2.
template <typename T>
snmf_status inner_step(snmf_plan* pl, T* X, const T* P, int is_hstep, int k, hipStream_t s) {
  const int64_t n = pl->n;
  const int r = pl->r;
  const int gi = is_hstep ? 1 : 0;
  const T* GT = (const T*)pl->GT[gi];
  T* Z = (T*)pl->Z;
  T* D = (T*)pl->D;
  T* g = (T*)pl->g;
  const bool lap = pl->lap && is_hstep;
  if (!lap) {
    // step 2 forms D again instead of reading it back where the n x r arrays are large
    // (n = 200000, r = 32: 2% faster); at the small sizes (n = 8192, r = 64 and
    // n = 20000, r = 20) storing it measured faster (1.6% and 0.5%)
    const int rd = (int64_t)n * r * (int64_t)sizeof(T) >= kRecomputeDBytes;
    launch_step1<T>(X, g, Z, D, nullptr, GT, pl->G64[0], pl->G64[1], n, r, k, 0, is_hstep, pl->kp,
                    pl->st, pl->partsA, pl->partsB, pl->partsC, pl->trace, s, BMap{}, pl->grid,
                    rd);
    launch_step2<T>(X, g, Z, D, nullptr, (const T*)pl->C, P, nullptr, GT, n, r, k, 0, is_hstep,
                    pl->kp, pl->st, pl->partsB, nullptr, 0, pl->partsC, s, BMap{}, pl->grid,
                    pl->p.inner_iters - 1, rd);
  } else {
    const int64_t* rp = pl->L.rowptr;
    const int32_t* ci = pl->L.col;
    const T* lv = (const T*)pl->L.val;
    T* LT = (T*)pl->LT;
    const int32_t* g1 = &pl->st->done;
    const int32_t* g2 = &pl->st->stop[k];
    // Z and D = Z - X of this iteration come from init (k = 0) or the previous step 2, so
    // the first product runs at once, before this iteration's stop test (made by its
    // phase-2 step 1): it is gated on the solve only, since stop[k] still holds the
    // previous half-step's flag, and a stopped iteration's product is never read
    launch_spmm<T>(rp, ci, lv, D, n, r, LT, nullptr, nullptr, g1, nullptr, s);
    launch_step1<T>(X, g, Z, D, LT, GT, pl->G64[0], pl->G64[1], n, r, k, 2, is_hstep, pl->kp,
                    pl->st, pl->partsA, pl->partsB, pl->partsC, pl->trace, s, BMap{}, pl->grid);
    launch_spmm<T>(rp, ci, lv, D, n, r, nullptr, D, pl->partsD, g1, g2, s);
    launch_step2<T>(X, g, Z, D, nullptr, (const T*)pl->C, P, nullptr, GT, n, r, k, 1, is_hstep,
                    pl->kp, pl->st, pl->partsB, pl->partsD, spmm_dot_grid(n), pl->partsC, s,
                    BMap{}, pl->grid);
    launch_spmm<T>(rp, ci, lv, D, n, r, LT, nullptr, nullptr, g1, g2, s);
    launch_step2<T>(X, g, Z, D, LT, (const T*)pl->C, P, (T*)pl->LX, GT, n, r, k, 2, is_hstep,
                    pl->kp, pl->st, pl->partsB, nullptr, 0, pl->partsC, s, BMap{}, pl->grid);
  }
  HIP_TRY(hipGetLastError());
  return SNMF_OK;
}

// The inner iterations of a half-step: with `fused` (its init ran with dir set) K fused
// kernels, the iterate and the trial update alternating between (X, g) and (Z, gs) and
// the partial sums between partsB and partsD (which the fused path does not otherwise
// use); else K pairs of step 1 and step 2.
template <typename T>
snmf_status inner_steps(snmf_plan* pl, T* X, const T* P, int is_hstep, hipStream_t s,
                        bool fused) {
  const int K = pl->p.inner_iters;
  if (fused) {
    for (int i = 0; i < K; ++i) {
      launch_advance<T>(X, (T*)pl->g, (T*)pl->Z, (T*)pl->gs, (T*)pl->D, (const T*)pl->C, P,
                        (const T*)pl->GT[is_hstep ? 1 : 0], pl->G64[0], pl->G64[1], pl->n, pl->r,
                        K, i, is_hstep, pl->kp, pl->st, (i & 1) ? pl->partsD : pl->partsB,
                        (i & 1) ? pl->partsB : pl->partsD, pl->partsA, pl->partsC, pl->trace, s,
                        pl->grid);
    }
    HIP_TRY(hipGetLastError());
    return SNMF_OK;
  }
  for (int k = 0; k < K; ++k) SNMF_TRY(inner_step<T>(pl, X, P, is_hstep, k, s));
  return SNMF_OK;
}

template <typename T>
snmf_status outer_iteration(snmf_plan* pl, hipStream_t s) {
  T* W = (T*)pl->Wb;
  T* H = (T*)pl->Hb;
  SNMF_TRY(half_start<T>(pl, W, H, 0, true, s, fused_half(pl, 0)));
  SNMF_TRY(inner_steps<T>(pl, W, H, 0, s, fused_half(pl, 0)));
  if (pl->p.naive) {
    // H <- W^T, then an H-step that stops before its first inner iteration: its init
    // (at H = W) and its one step 2 supply the monitor sums of the pair (W, W)
    HIP_TRY(hipMemcpyAsync(H, W, (size_t)pl->n * pl->r * sizeof(T), hipMemcpyDeviceToDevice, s));
    SNMF_TRY(half_start<T>(pl, H, W, 1, false, s));
    launch_naive_hentry(pl->partsA, pl->grid, pl->st, s);
    launch_step2<T>(H, (T*)pl->g, (T*)pl->Z, (T*)pl->D, nullptr, (const T*)pl->C, W, nullptr,
                    (const T*)pl->GT[1], pl->n, pl->r, 0, 0, 1, pl->kp, pl->st, pl->partsB,
                    nullptr, 0, pl->partsC, s, BMap{}, pl->grid, 0, 0);
    HIP_TRY(hipGetLastError());
    return SNMF_OK;
  }
  SNMF_TRY(half_start<T>(pl, H, W, 1, true, s, fused_half(pl, 1)));
  SNMF_TRY(inner_steps<T>(pl, H, W, 1, s, fused_half(pl, 1)));
  return SNMF_OK;
}

snmf_status outer_any(snmf_plan* pl, hipStream_t s) {
  return pl->prec == SNMF_F64 ? outer_iteration<double>(pl, s) : outer_iteration<float>(pl, s);
}

// Monitor record of the last outer iteration: the start of one more W-step, whose first
// inner kernel completes the record and ends the solve (it has reached max_outer).
template <typename T>
snmf_status finalize(snmf_plan* pl, hipStream_t s) {
  T* W = (T*)pl->Wb;
  const T* H = (const T*)pl->Hb;
  SNMF_TRY(half_start<T>(pl, W, H, 0, false, s));
  const int64_t n = pl->n;
  launch_step1<T>(W, (const T*)pl->g, (T*)pl->Z, (T*)pl->D, nullptr, (const T*)pl->GT[0],
                  pl->G64[0], pl->G64[1], n, pl->r, 0, 0, 0, pl->kp, pl->st,
                  pl->partsA, pl->partsB, pl->partsC, pl->trace, s, BMap{}, pl->grid,
                  1);  // D is never read after it
  HIP_TRY(hipGetLastError());
  return SNMF_OK;
}

snmf_status finalize_any(snmf_plan* pl, hipStream_t s) {
  return pl->prec == SNMF_F64 ? finalize<double>(pl, s) : finalize<float>(pl, s);
}

snmf_status build_kparams(snmf_plan* pl) {
  pl->kp = kparams_of(pl->p, pl->lap);
  return SNMF_OK;
}

// Sets up plan pl: checks, scratch (hipMalloc, or the caller's fixed pool of fixed_bytes,
// in which case the plan runs on the user stream and owns nothing), ||A||^2, the split.
snmf_status plan_init(snmf_plan* pl, const snmf_matrix* A, int32_t r, const snmf_params* p,
                      hipStream_t user, void* fixed_pool, size_t fixed_bytes) {
  SNMF_TRY(check_params(p));
  SNMF_TRY(check_matrix(A, "A"));
  if (r < 1 || r > kMaxRank) return fail(SNMF_E_SHAPE, "r must lie in [1, 64]");
  if (r > A->n) return fail(SNMF_E_SHAPE, "r must not exceed n");
  const bool lap = p->L != nullptr && p->gamma > 0.0;
  if (lap) {
    SNMF_TRY(check_matrix(p->L, "L"));
    if (p->L->fmt != SNMF_CSR) return fail(SNMF_E_UNSUPPORTED, "L must be CSR");
    if (p->L->n != A->n) return fail(SNMF_E_SHAPE, "L must be n x n");
  }
  if (p->prec == SNMF_BF16X3 && A->fmt != SNMF_DENSE)
    return fail(SNMF_E_UNSUPPORTED, "BF16X3 applies to dense A only");
  if (p->naive && p->lambda != 0.0)
    return fail(SNMF_E_ARG, "the naive variant has no penalty: lambda must be 0");
  if (p->naive && lap) return fail(SNMF_E_UNSUPPORTED, "the naive variant takes no Laplacian");
  pl->A = *A;
  if (lap) pl->L = *p->L;
  pl->p = *p;
  pl->lap = lap;
  pl->r = r;
  pl->n = A->n;
  pl->prec = p->prec;
  pl->esz = elt_size(p->prec);
  if (fixed_pool) {
    pl->borrowed = true;
    pl->s = user;
    pl->p.use_graph = 0;  // instantiating a graph allocates
  } else {
    HIP_TRY(hipStreamCreateWithFlags(&pl->s, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&pl->ev_in, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&pl->ev_out, hipEventDisableTiming));
    if (user) {
      HIP_TRY(hipEventRecord(pl->ev_in, user));
      HIP_TRY(hipStreamWaitEvent(pl->s, pl->ev_in, 0));
    }
  }
  const int64_t n = pl->n;
  const size_t nr = (size_t)n * r * pl->esz;
  int ksplit = 1;
  if (A->fmt == SNMF_DENSE && pl->prec == SNMF_F32) pl->ds = plan_dense_f32(n, A->ld, r, A->dense);
  if (A->fmt == SNMF_DENSE && pl->prec == SNMF_BF16X3) {
    pl->ds = plan_dense_bf16(n);
    pl->ldb = (n + 63) / 64 * 64;
  }
  if (A->fmt == SNMF_DENSE && pl->prec != SNMF_F64) ksplit = pl->ds.ksplit;
  pl->gram_blocks = gram_blocks(n);
  const int lai_nb = lai_blocks(n);
  // carve one allocation (a fixed table: the allocation-free path allocates nothing on the
  // host either)
  std::pair<void**, size_t> req[40];
  int nreq = 0;
  auto add = [&](void** dst, size_t bytes) { req[nreq++] = {dst, (bytes + 255) / 256 * 256}; };
  add(&pl->Wb, nr);
  add(&pl->Hb, nr);
  add(&pl->C, nr);
  add(&pl->g, nr);
  add(&pl->Z, nr);
  // the fused inner kernels' trial gradient (the trial update itself goes to Z)
  const bool fused = fused_inner_ok(*p);
  if (fused) add(&pl->gs, nr);
  pl->grid = inner_grid(n, r, (int)pl->esz, fused);
  add(&pl->D, nr);
  add(&pl->Bpart, nr * ksplit);
  if (lap) {
    add(&pl->LT, nr);
    add(&pl->LX, nr);
  }
  add(&pl->GT[0], (size_t)r * r * pl->esz);
  add(&pl->GT[1], (size_t)r * r * pl->esz);
  add((void**)&pl->G64[0], (size_t)r * r * 8);
  add((void**)&pl->G64[1], (size_t)r * r * 8);
  add((void**)&pl->part, (size_t)2 * kMaxGrid * kNumPart * 8);
  add((void**)&pl->partsA, (size_t)kInnerGrid * kNumPart * 8);
  add((void**)&pl->partsB, (size_t)kInnerGrid * kNumPart * 8);
  add((void**)&pl->partsC, (size_t)kInnerGrid * kNumPart * 8);
  add((void**)&pl->partsD, (size_t)kInnerGrid * kNumPart * 8);
  add((void**)&pl->gram_part, (size_t)pl->gram_blocks * r * r * 8);
  add((void**)&pl->dots, 64 * 8);
  add((void**)&pl->trace, (size_t)p->max_outer * kTraceFields * 8);
  add((void**)&pl->st, sizeof(State));
  add((void**)&pl->counters, C_COUNT * sizeof(unsigned));
  add((void**)&pl->flags, 4 * sizeof(unsigned));
  if (A->fmt == SNMF_LOWRANK) {
    add((void**)&pl->lai_part, (size_t)lai_nb * A->ell * r * 8);
    add(&pl->TT, (size_t)A->ell * r * pl->esz);
  }
  if (pl->prec == SNMF_BF16X3) {
    add((void**)&pl->Ahi, (size_t)n * pl->ldb * 2);
    add((void**)&pl->Alo, (size_t)n * pl->ldb * 2);
    add((void**)&pl->Pthi, (size_t)r * pl->ldb * 2);
    add((void**)&pl->Ptlo, (size_t)r * pl->ldb * 2);
  }
  size_t total = 0;
  for (int q = 0; q < nreq; ++q) total += req[q].second;
  if (fixed_pool) {
    if (total > fixed_bytes)
      return fail(SNMF_E_SHAPE, "the solve needs " + std::to_string(total) +
                                    " bytes of scratch, more than the " +
                                    std::to_string(fixed_bytes) + " of the static array");
    pl->pool = fixed_pool;
  } else {
    HIP_TRY(hipMalloc(&pl->pool, total));
  }
  size_t off = 0;
  for (int q = 0; q < nreq; ++q) {
    *req[q].first = (char*)pl->pool + off;
    off += req[q].second;
  }
  HIP_TRY(hipMemsetAsync(pl->counters, 0, C_COUNT * sizeof(unsigned), pl->s));
  HIP_TRY(hipMemsetAsync(pl->st, 0, sizeof(State), pl->s));
  // input checks and ||A||^2
  double st3[3] = {0, 0, 0};
  if (A->fmt == SNMF_DENSE) {
    SNMF_TRY(stats_any(pl, A->dense, n, n, A->ld, st3));
    if (p->validate) SNMF_TRY(check_values(st3, "A"));
    if (p->check_symmetry) SNMF_TRY(check_dense_symmetry(A, pl->prec, pl->flags, pl->s, "A"));
    pl->normA2 = st3[0];
  } else if (A->fmt == SNMF_CSR) {
    SNMF_TRY(check_csr(pl, A, "A", p->validate != 0, &pl->normA2));
  } else {
    double lam[kMaxEll];
    HIP_TRY(hipMemcpyAsync(lam, A->lam, A->ell * 8, hipMemcpyDeviceToHost, pl->s));
    HIP_TRY(hipStreamSynchronize(pl->s));
    double s2 = 0.0;
    for (int64_t a = 0; a < A->ell; ++a) {
      const double v = lam[a];
      if (!std::isfinite(v)) return fail(SNMF_E_NONFINITE, "lam has NaN/Inf entries");
      s2 += v * v;
    }
    pl->normA2 = s2;
    if (p->validate) {
      SNMF_TRY(stats_any(pl, A->U, n, A->ell, A->ell, st3));
      if (st3[2] > 0) return fail(SNMF_E_NONFINITE, "U has NaN/Inf entries");
    }
  }
  if (lap) SNMF_TRY(check_csr(pl, &pl->L, "L", false, nullptr));
  if (!(pl->normA2 > 0.0)) return fail(SNMF_E_ARG, "A is zero");
  if (pl->prec == SNMF_BF16X3) {
    launch_split_rows((const float*)A->dense, n, A->ld, pl->ldb, pl->Ahi, pl->Alo, pl->s);
    HIP_TRY(hipGetLastError());
  }
  SNMF_TRY(build_kparams(pl));
  HIP_TRY(hipStreamSynchronize(pl->s));
  return SNMF_OK;
}

snmf_status plan_create(const snmf_matrix* A, int32_t r, const snmf_params* p, hipStream_t user,
                        snmf_plan** out) {
  if (!out) return fail(SNMF_E_ARG, "out is NULL");
  *out = nullptr;
  auto pl = new (std::nothrow) snmf_plan();
  if (!pl) return fail(SNMF_E_OOM, "host allocation failed");
  std::unique_ptr<snmf_plan> guard(pl);
  SNMF_TRY(plan_init(pl, A, r, p, user, nullptr, 0));
  *out = guard.release();
  return SNMF_OK;
}

snmf_status read_info(snmf_plan* pl, snmf_info* info, double* trace) {
  State hs;
  HIP_TRY(hipMemcpyAsync(&hs, pl->st, sizeof(State), hipMemcpyDeviceToHost, pl->s));
  HIP_TRY(hipStreamSynchronize(pl->s));
  const double hz = snmf_clock_rate_hz();
  // the clock ticks of the last record and of the record that met the target
  double ticks_last = 0.0, ticks_conv = 0.0;
  if (hs.trace_len > 0) {
    if (trace)
      HIP_TRY(hipMemcpyAsync(trace, pl->trace, (size_t)hs.trace_len * kTraceFields * 8,
                             hipMemcpyDeviceToHost, pl->s));
    HIP_TRY(hipMemcpyAsync(&ticks_last, pl->trace + (size_t)(hs.trace_len - 1) * kTraceFields + 5,
                           8, hipMemcpyDeviceToHost, pl->s));
    if (hs.converged_at > 0)
      HIP_TRY(hipMemcpyAsync(&ticks_conv,
                             pl->trace + (size_t)(hs.converged_at - 1) * kTraceFields + 5, 8,
                             hipMemcpyDeviceToHost, pl->s));
    HIP_TRY(hipStreamSynchronize(pl->s));
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = hs.status;
    info->outer = hs.outer;
    info->converged_at = hs.converged_at;
    info->inner_total = hs.inner_total;
    info->ls_evals = hs.ls_evals;
    info->ls_exhausted = hs.ls_exhausted;
    info->res_WH = hs.res_last;
    info->res_WWt = hs.resww_last;
    info->sym_gap = hs.sym_last;
    info->pg_norm = hs.pg_last;
    info->objective = hs.f_last;
    info->normA2 = pl->normA2;
    info->seconds = hs.trace_len > 0 ? ticks_last / hz : 0.0;
    info->seconds_to_target = hs.converged_at > 0 ? ticks_conv / hz : -1.0;
  }
  if (hs.status != 0) return fail((snmf_status)hs.status, "numeric breakdown during the solve");
  return SNMF_OK;
}

snmf_status plan_solve(snmf_plan* pl, const void* W0, void* W_out, void* Ht_out, snmf_info* info,
                       hipStream_t user, double* trace) {
  if (!pl) return fail(SNMF_E_ARG, "plan is NULL");
  if (!W0 || !W_out || !Ht_out) return fail(SNMF_E_ARG, "W0, W_out and Ht_out are required");
  const int64_t n = pl->n;
  const int r = pl->r;
  const size_t nr = (size_t)n * r * pl->esz;
  if (pl->borrowed) user = nullptr;  // the plan already runs on the caller's stream
  if (user) {
    HIP_TRY(hipEventRecord(pl->ev_in, user));
    HIP_TRY(hipStreamWaitEvent(pl->s, pl->ev_in, 0));
  }
  if (pl->p.validate) {
    double st3[3];
    SNMF_TRY(stats_any(pl, W0, n, r, r, st3));
    SNMF_TRY(check_values(st3, "W0"));
  }
  HIP_TRY(hipMemcpyAsync(pl->Wb, W0, nr, hipMemcpyDeviceToDevice, pl->s));
  HIP_TRY(hipMemcpyAsync(pl->Hb, W0, nr, hipMemcpyDeviceToDevice, pl->s));
  launch_reset_state(pl->st, pl->normA2, pl->s);
  HIP_TRY(hipGetLastError());
  const int every = std::max(1, pl->p.check_every);
  auto capture = [&](int iters, hipGraph_t* g, hipGraphExec_t* ge) -> snmf_status {
    HIP_TRY(hipStreamBeginCapture(pl->s, hipStreamCaptureModeThreadLocal));
    snmf_status cs = SNMF_OK;
    for (int u = 0; u < iters && cs == SNMF_OK; ++u) cs = outer_any(pl, pl->s);
    hipGraph_t gr = nullptr;
    hipError_t ce = hipStreamEndCapture(pl->s, &gr);
    if (cs != SNMF_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return cs;
    }
    if (ce != hipSuccess) return fail(SNMF_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
    *g = gr;
    HIP_TRY(hipGraphInstantiate(ge, gr, nullptr, nullptr, 0));
    return SNMF_OK;
  };
  const int run = std::min(kGraphRun, every);
  if (pl->p.use_graph && !pl->gexec) SNMF_TRY(capture(1, &pl->graph, &pl->gexec));
  if (pl->p.use_graph && run > 1 && pl->p.max_outer >= run && !pl->gexec_run)
    SNMF_TRY(capture(run, &pl->graph_run, &pl->gexec_run));
  // outer iterations i .. : a captured run when it ends at or before the next check of the
  // done flag and at or before max_outer, else single iterations
  for (int i = 0; i < pl->p.max_outer;) {
    const int next_check = (i / every + 1) * every;
    const int room = std::min(pl->p.max_outer, next_check) - i;
    if (pl->gexec_run && room >= run) {
      HIP_TRY(hipGraphLaunch(pl->gexec_run, pl->s));
      i += run;
    } else if (pl->gexec) {
      HIP_TRY(hipGraphLaunch(pl->gexec, pl->s));
      i += 1;
    } else {
      SNMF_TRY(outer_any(pl, pl->s));
      i += 1;
    }
    if (i % every == 0 && i < pl->p.max_outer) {
      int32_t done = 0;
      HIP_TRY(hipMemcpyAsync(&done, &pl->st->done, sizeof(done), hipMemcpyDeviceToHost, pl->s));
      HIP_TRY(hipStreamSynchronize(pl->s));
      if (done) break;
    }
  }
  SNMF_TRY(finalize_any(pl, pl->s));
  HIP_TRY(hipMemcpyAsync(W_out, pl->Wb, nr, hipMemcpyDeviceToDevice, pl->s));
  HIP_TRY(hipMemcpyAsync(Ht_out, pl->Hb, nr, hipMemcpyDeviceToDevice, pl->s));
  snmf_status rs = read_info(pl, info, trace);
  if (user) {
    HIP_TRY(hipEventRecord(pl->ev_out, pl->s));
    HIP_TRY(hipStreamWaitEvent(user, pl->ev_out, 0));
  }
  return rs;
}

// ------------------------------------------------------------------ allocation-free solve
// The scratch of snmf_solve_noalloc: a file-scope device array (each GPU the library runs
// on holds its own copy until the process ends).  Host code uses its address from
// hipGetSymbolAddress, taken once per device, never the array's name.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

snmf_status scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SNMF_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(SNMF_E_DEVICE, "no device address for the static scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SNMF_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

snmf_status snmf_solve_noalloc(const snmf_matrix* A, int32_t r, const void* W0,
                               const snmf_params* p, void* W_out, void* Ht_out, snmf_info* info,
                               void* stream, double* trace) {
  if (!p) return fail(SNMF_E_ARG, "params is NULL");
  if (p->prec == SNMF_BF16X3)
    return fail(SNMF_E_UNSUPPORTED, "the split copies of A do not fit the static scratch");
  void* sp = nullptr;
  SNMF_TRY(scratch_address(&sp));
  snmf_plan pl;
  SNMF_TRY(plan_init(&pl, A, r, p, (hipStream_t)stream, sp, kScratchBytes));
  return plan_solve(&pl, W0, W_out, Ht_out, info, (hipStream_t)stream, trace);
}

snmf_status snmf_params_default(snmf_params* p) {
  if (!p) return fail(SNMF_E_ARG, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->lambda = 0.0;
  p->gamma = 0.0;
  p->L = nullptr;
  p->eta = 0.85;
  p->theta = 1e-3;
  p->phi = 1.7;
  p->alpha_min = 1e-10;
  p->alpha_max = 1e10;
  p->beta_shrink = 0.5;
  p->max_ls = 20;
  p->inner_iters = 5;
  p->max_outer = 100;
  p->check_every = 8;
  p->target_res = 0.0;
  p->prec = SNMF_F32;
  p->accept_at_relaxed = 0;
  p->project_update = 1;
  p->validate = 1;
  p->use_graph = 1;
  p->fuse_inner = 1;
  return SNMF_OK;
}

snmf_status snmf_plan_create(const snmf_matrix* A, int32_t r, const snmf_params* p, void* stream,
                             snmf_plan** out) {
  return plan_create(A, r, p, (hipStream_t)stream, out);
}

snmf_status snmf_plan_solve(snmf_plan* plan, const void* W0, void* W_out, void* Ht_out,
                            snmf_info* info, void* stream, double* trace) {
  return plan_solve(plan, W0, W_out, Ht_out, info, (hipStream_t)stream, trace);
}

snmf_status snmf_plan_destroy(snmf_plan* plan) {
  if (plan) {
    (void)hipStreamSynchronize(plan->s);
    delete plan;
  }
  return SNMF_OK;
}

snmf_status snmf_solve(const snmf_matrix* A, int32_t r, const void* W0, const snmf_params* p,
                       void* W_out, void* Ht_out, snmf_info* info, void* stream, double* trace) {
  snmf_plan* pl = nullptr;
  SNMF_TRY(plan_create(A, r, p, (hipStream_t)stream, &pl));
  snmf_status s = plan_solve(pl, W0, W_out, Ht_out, info, (hipStream_t)stream, trace);
  std::string keep = snmf::err_ref();
  snmf_plan_destroy(pl);
  snmf::err_ref() = keep;
  return s;
}

snmf_status snmf_plan_half_step(snmf_plan* pl, void* X, const void* P, int32_t is_hstep,
                                void* stream, double* scalars) {
  if (!pl || !X || !P) return fail(SNMF_E_ARG, "plan, X and P are required");
  hipStream_t user = (hipStream_t)stream;
  if (user) {
    HIP_TRY(hipEventRecord(pl->ev_in, user));
    HIP_TRY(hipStreamWaitEvent(pl->s, pl->ev_in, 0));
  }
  launch_reset_state(pl->st, pl->normA2, pl->s);
  const int K = pl->p.inner_iters;
  // the inner iterations, then the entry of one more inner iteration (k = K), which
  // reduces the last update's <S,S>, <S,Y> and forms e_K and alpha_K; its step work only
  // touches scratch (Z, D), never X.
  if (pl->prec == SNMF_F64) {
    SNMF_TRY(half_start<double>(pl, (double*)X, (const double*)P, is_hstep, true, pl->s));
    SNMF_TRY(inner_steps<double>(pl, (double*)X, (const double*)P, is_hstep, pl->s, false));
    launch_step1<double>((const double*)X, (const double*)pl->g, (double*)pl->Z, (double*)pl->D,
                         nullptr, (const double*)pl->GT[is_hstep ? 1 : 0], pl->G64[0], pl->G64[1],
                         pl->n, pl->r, K, (pl->lap && is_hstep) ? 1 : 0, is_hstep, pl->kp, pl->st,
                         pl->partsA, pl->partsB, pl->partsC, pl->trace, pl->s, BMap{},
                         pl->grid, 1);
  } else {
    SNMF_TRY(half_start<float>(pl, (float*)X, (const float*)P, is_hstep, true, pl->s));
    SNMF_TRY(inner_steps<float>(pl, (float*)X, (const float*)P, is_hstep, pl->s, false));
    launch_step1<float>((const float*)X, (const float*)pl->g, (float*)pl->Z, (float*)pl->D,
                        nullptr, (const float*)pl->GT[is_hstep ? 1 : 0], pl->G64[0], pl->G64[1],
                        pl->n, pl->r, K, (pl->lap && is_hstep) ? 1 : 0, is_hstep, pl->kp, pl->st,
                        pl->partsA, pl->partsB, pl->partsC, pl->trace, pl->s, BMap{},
                        pl->grid, 1);
  }
  HIP_TRY(hipGetLastError());
  State hs;
  HIP_TRY(hipMemcpyAsync(&hs, pl->st, sizeof(State), hipMemcpyDeviceToHost, pl->s));
  HIP_TRY(hipStreamSynchronize(pl->s));
  if (scalars) {
    int last = 0;  // last inner iteration that ran
    while (last + 1 < K && !hs.stop[last + 1]) ++last;
    scalars[0] = hs.rho;
    scalars[1] = hs.alpha[last];
    scalars[2] = hs.beta[last];
    scalars[3] = hs.e[last];
    scalars[4] = hs.last_ss;
    scalars[5] = hs.last_sy;
    scalars[6] = (double)hs.ls_evals;
    scalars[7] = (double)hs.inner_total;
  }
  if (user) {
    HIP_TRY(hipEventRecord(pl->ev_out, pl->s));
    HIP_TRY(hipStreamWaitEvent(user, pl->ev_out, 0));
  }
  if (hs.status != 0) return fail((snmf_status)hs.status, "numeric breakdown");
  return SNMF_OK;
}

snmf_status snmf_plan_apass(snmf_plan* pl, const void* P, void* B, void* stream) {
  if (!pl || !P || !B) return fail(SNMF_E_ARG, "plan, P and B are required");
  hipStream_t user = (hipStream_t)stream;
  if (user) {
    HIP_TRY(hipEventRecord(pl->ev_in, user));
    HIP_TRY(hipStreamWaitEvent(pl->s, pl->ev_in, 0));
  }
  HIP_TRY(hipMemsetAsync(pl->st, 0, sizeof(State), pl->s));
  if (pl->prec == SNMF_F64)
    SNMF_TRY(apass<double>(pl, (const double*)P, pl->s));
  else
    SNMF_TRY(apass<float>(pl, (const float*)P, pl->s));
  // add the split-K partials on the device, in the same order as the init kernel
  const int ks = ksplit_of(pl);
  const int64_t nr = pl->n * pl->r;
  if (pl->prec == SNMF_F64)
    launch_sum_parts<double>((const double*)pl->Bpart, ks, nr, (double*)B, nr, pl->s);
  else
    launch_sum_parts<float>((const float*)pl->Bpart, ks, nr, (float*)B, nr, pl->s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(pl->s));
  if (user) {
    HIP_TRY(hipEventRecord(pl->ev_out, pl->s));
    HIP_TRY(hipStreamWaitEvent(user, pl->ev_out, 0));
  }
  return SNMF_OK;
}

snmf_status snmf_plan_time_apass(snmf_plan* pl, const void* P, int32_t reps, double* ms) {
  if (!pl || !P || !ms) return fail(SNMF_E_ARG, "plan, P and ms are required");
  if (reps < 1) return fail(SNMF_E_ARG, "reps must be >= 1");
  HIP_TRY(hipMemsetAsync(pl->st, 0, sizeof(State), pl->s));
  const int64_t n = pl->n;
  const int r = pl->r;
  auto launch = [&]() -> snmf_status {
    if (pl->A.fmt == SNMF_DENSE && pl->prec == SNMF_BF16X3) {
      launch_apass_bf16x3(pl->Ahi, pl->Alo, pl->ldb, pl->Pthi, pl->Ptlo, pl->ldb, n, r, pl->ds,
                          (float*)pl->Bpart, n * r, pl->st, pl->s);
      HIP_TRY(hipGetLastError());
      return SNMF_OK;
    }
    if (pl->prec == SNMF_F64) return apass<double>(pl, (const double*)P, pl->s);
    return apass<float>(pl, (const float*)P, pl->s);
  };
  if (pl->A.fmt == SNMF_DENSE && pl->prec == SNMF_BF16X3) {
    launch_split_pt((const float*)P, n, r, pl->ldb, pl->Pthi, pl->Ptlo, pl->st, pl->s);
    HIP_TRY(hipGetLastError());
  }
  SNMF_TRY(launch());
  ScopedEvent e0, e1;
  HIP_TRY(hipEventCreate(&e0.e));
  HIP_TRY(hipEventCreate(&e1.e));
  HIP_TRY(hipEventRecord(e0.e, pl->s));
  for (int i = 0; i < reps; ++i) SNMF_TRY(launch());
  HIP_TRY(hipEventRecord(e1.e, pl->s));
  HIP_TRY(hipEventSynchronize(e1.e));
  float tot = 0.0f;
  HIP_TRY(hipEventElapsedTime(&tot, e0.e, e1.e));
  *ms = (double)tot / reps;
  return SNMF_OK;
}

snmf_status snmf_plan_gram(snmf_plan* pl, const void* P, double* G, void* stream) {
  if (!pl || !P || !G) return fail(SNMF_E_ARG, "plan, P and G are required");
  hipStream_t user = (hipStream_t)stream;
  if (user) {
    HIP_TRY(hipEventRecord(pl->ev_in, user));
    HIP_TRY(hipStreamWaitEvent(pl->s, pl->ev_in, 0));
  }
  HIP_TRY(hipMemsetAsync(pl->st, 0, sizeof(State), pl->s));
  if (pl->prec == SNMF_F64)
    launch_gram<double>((const double*)P, pl->n, pl->r, pl->gram_part, pl->gram_blocks, pl->G64[0],
                        (double*)pl->GT[0], pl->st, pl->s);
  else
    launch_gram<float>((const float*)P, pl->n, pl->r, pl->gram_part, pl->gram_blocks, pl->G64[0],
                       (float*)pl->GT[0], pl->st, pl->s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(G, pl->G64[0], (size_t)pl->r * pl->r * 8, hipMemcpyDeviceToDevice, pl->s));
  HIP_TRY(hipStreamSynchronize(pl->s));
  return SNMF_OK;
}

snmf_status snmf_rho(const double* G, int32_t r, double* rho, void* stream) {
  if (!G || !rho) return fail(SNMF_E_ARG, "G and rho are required");
  if (r < 1 || r > kMaxRank) return fail(SNMF_E_SHAPE, "r must lie in [1, 64]");
  hipStream_t s = (hipStream_t)stream;
  State* st = nullptr;
  HIP_TRY(hipMalloc(&st, sizeof(State)));
  DevBuf keep;
  keep.p = st;
  HIP_TRY(hipMemsetAsync(st, 0, sizeof(State), s));
  launch_rho(G, r, st, s);
  HIP_TRY(hipGetLastError());
  State hs;
  HIP_TRY(hipMemcpyAsync(&hs, st, sizeof(State), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *rho = hs.rho;
  return SNMF_OK;
}

snmf_status snmf_spmm(const snmf_matrix* M, int32_t prec, const void* X, int32_t r, void* Y,
                      void* stream) {
  SNMF_TRY(check_matrix(M, "M"));
  if (M->fmt != SNMF_CSR) return fail(SNMF_E_UNSUPPORTED, "snmf_spmm needs a CSR matrix");
  if (!X || !Y) return fail(SNMF_E_ARG, "X and Y are required");
  if (r < 1 || r > kMaxRank) return fail(SNMF_E_SHAPE, "r must lie in [1, 64]");
  hipStream_t s = (hipStream_t)stream;
  if (prec == SNMF_F64)
    launch_spmm<double>(M->rowptr, M->col, (const double*)M->val, (const double*)X, M->n, r,
                        (double*)Y, nullptr, nullptr, nullptr, nullptr, s);
  else
    launch_spmm<float>(M->rowptr, M->col, (const float*)M->val, (const float*)X, M->n, r,
                       (float*)Y, nullptr, nullptr, nullptr, nullptr, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return SNMF_OK;
}

snmf_status snmf_split_bf16(const float* x, int64_t count, uint16_t* hi, uint16_t* lo,
                            void* stream) {
  if (!x || !hi || !lo) return fail(SNMF_E_ARG, "x, hi and lo are required");
  if (count < 0) return fail(SNMF_E_SHAPE, "count < 0");
  if (count == 0) return SNMF_OK;
  hipStream_t s = (hipStream_t)stream;
  launch_split_flat(x, count, hi, lo, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return SNMF_OK;
}

double snmf_clock_rate_hz(void) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1e8;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return 1e8;
  return (double)khz * 1e3;
}

const char* snmf_last_error(void) { return snmf::err_ref().c_str(); }

int32_t snmf_abi_version(void) { return SNMF_ABI_VERSION; }

}  // extern "C"
