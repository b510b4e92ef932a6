// Host side and C ABI of NMPBB for rectangular NMF (eq. (1.1); include/snmf.h
// snmf_nmf_solve).  The outer iteration is the W-step (X = W, partner Ht, product V Ht)
// then the H-step (X = Ht, partner W, product V^T W), each Algorithm 1 run by the inner
// kernels of the symmetric solver with lam = 0: their penalty term reads a zero partner
// of X's shape, so only the Gram G = P^T P and the product B carry the true partner.
// Products: dense V by the rectangular product kernel (V P and V^T P read V in place),
// CSR V by the SpMM on V and on its transpose, formed once on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>

#include "../../include/snmf.h"
#include "common.hpp"
#include "host.hpp"
#include "kernels.hpp"

using namespace snmf;

namespace {

struct NmfPlan {
  snmf_matrix V{};
  int64_t m = 0, n = 0, mx = 0;
  int r = 0, prec = SNMF_F32, grid = 1;
  size_t esz = 4;
  snmf_params p{};
  KParams kp{};
  hipStream_t s = nullptr;
  void* pool = nullptr;
  void *Wb = nullptr, *Hb = nullptr, *C = nullptr, *g = nullptr, *Z = nullptr, *D = nullptr,
       *B = nullptr, *Pz = nullptr, *GT[2] = {nullptr, nullptr}, *gs = nullptr;
  void *VT = nullptr, *Bpart = nullptr;  // dense FP32: V^T and the split-K panels
  RectSplit spW, spH;
  double* G64[2] = {nullptr, nullptr};
  double *part = nullptr, *gram_part = nullptr, *dots = nullptr;
  double *partsA = nullptr, *partsB = nullptr, *partsC = nullptr, *partsD = nullptr;
  double* trace = nullptr;
  State* st = nullptr;
  unsigned *counters = nullptr, *flags = nullptr, *cnt = nullptr;
  unsigned long long* cursor = nullptr;
  int64_t* rowptrT = nullptr;
  int32_t* colT = nullptr;
  void* valT = nullptr;
  double normV2 = 0.0;
  ~NmfPlan() {
    if (pool) (void)hipFree(pool);
  }
};

template <typename T>
snmf_status stats(NmfPlan& pl, const T* x, int64_t rows, int64_t cols, int64_t ld, double* out3) {
  launch_stats2d<T>(x, rows, cols, ld, pl.part, pl.dots, pl.counters + C_NORM, pl.s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out3, pl.dots, 3 * sizeof(double), hipMemcpyDeviceToHost, pl.s));
  HIP_TRY(hipStreamSynchronize(pl.s));
  return SNMF_OK;
}

snmf_status check_vals(const double* st3, const char* what) {
  if (st3[2] > 0) return fail(SNMF_E_NONFINITE, std::string(what) + " has NaN/Inf entries");
  if (st3[1] > 0) return fail(SNMF_E_NEGATIVE, std::string(what) + " has negative entries");
  return SNMF_OK;
}

// One half-step of NMF: X (nX rows) with partner P (nP rows); the product of step (trans:
// the H-step's V^T P).
template <typename T>
void half_step(NmfPlan& pl, T* X, int64_t nX, const T* P, int64_t nP, int is_hstep, bool with_rho,
               bool run_inner, hipStream_t s) {
  const int r = pl.r;
  const int gi = is_hstep ? 1 : 0;
  launch_gram<T>(P, nP, r, pl.gram_part, gram_blocks(nP), pl.G64[gi], (T*)pl.GT[gi], pl.st, s);
  // rho of this half-step runs in one more workgroup of the product launch (the FP64
  // dense product: a launch of its own before it)
  RhoJob rj;
  if (with_rho) {
    rj.G = pl.G64[gi];
    rj.r = r;
    rj.st = pl.st;
  }
  T* B = (T*)pl.B;
  int ksplit = 1;
  if (pl.V.fmt == SNMF_DENSE && sizeof(T) == 4) {
    // FP32 MFMA: the H-step's V^T W reads V, the W-step's V Ht its transposed copy
    const RectSplit& sp = is_hstep ? pl.spH : pl.spW;
    const float* A = is_hstep ? (const float*)pl.V.dense : (const float*)pl.VT;
    const int64_t lda = is_hstep ? pl.V.ld : pl.m;
    launch_rect_f32(A, lda, (const float*)P, nP, nX, r, sp, (float*)pl.Bpart, pl.st, s, rj);
    B = (T*)pl.Bpart;
    ksplit = sp.ksplit;
  } else if (pl.V.fmt == SNMF_DENSE) {
    if (with_rho) launch_rho(pl.G64[gi], r, pl.st, s);
    launch_rect_apass<T>((const T*)pl.V.dense, pl.V.ld, nX, nP, is_hstep, P, r, B, pl.st, s);
  } else if (!is_hstep) {
    launch_spmm<T>(pl.V.rowptr, pl.V.col, (const T*)pl.V.val, P, nX, r, B, nullptr, nullptr,
                   &pl.st->done, nullptr, s, rj);
  } else {
    launch_spmm<T>(pl.rowptrT, pl.colT, (const T*)pl.valT, P, nX, r, B, nullptr, nullptr,
                   &pl.st->done, nullptr, s, rj);
  }
  const T* Pz = (const T*)pl.Pz;
  const T* GT = (const T*)pl.GT[gi];
  // one grid for both half-steps: the first inner kernel of a W-step reduces the partial
  // sums of the previous H-step's last kernel together with its own init's
  const int grid = pl.grid;
  T* Z = (T*)pl.Z;
  T* D = (T*)pl.D;
  T* g = (T*)pl.g;
  // one kernel per inner iteration (fused_inner_ok), init then also forming direction 0;
  // partial sums alternate between partsB and partsD
  const bool fused = run_inner && fused_inner_ok(pl.p);
  launch_init<T>(X, Pz, B, ksplit, nX * r, (T*)pl.C, g, nullptr, GT, nX, r, is_hstep, pl.kp,
                 pl.st, pl.partsA, s, BMap{}, grid, nullptr, nullptr, fused ? D : nullptr,
                 fused ? pl.partsB : nullptr, fused ? Z : nullptr, fused ? (T*)pl.gs : nullptr);
  if (fused) {
    const int K = pl.p.inner_iters;
    for (int i = 0; i < K; ++i)
      launch_advance<T>(X, g, Z, (T*)pl.gs, D, (const T*)pl.C, Pz, GT, pl.G64[0], pl.G64[1], nX,
                        r, K, i,
                        is_hstep, pl.kp, pl.st, (i & 1) ? pl.partsD : pl.partsB,
                        (i & 1) ? pl.partsB : pl.partsD, pl.partsA, pl.partsC, pl.trace, s,
                        grid);
    return;
  }
  const int rd = (int64_t)nX * r * (int64_t)sizeof(T) >= kRecomputeDBytes;
  if (!run_inner) {  // the closing entry: completes the monitor record of the last outer
    launch_step1<T>(X, g, Z, D, nullptr, GT, pl.G64[0], pl.G64[1], nX, r, 0, 0, 0, pl.kp, pl.st,
                    pl.partsA, pl.partsB, pl.partsC, pl.trace, s, BMap{}, grid, 1);
    return;
  }
  for (int k = 0; k < pl.p.inner_iters; ++k) {
    launch_step1<T>(X, g, Z, D, nullptr, GT, pl.G64[0], pl.G64[1], nX, r, k, 0, is_hstep, pl.kp,
                    pl.st, pl.partsA, pl.partsB, pl.partsC, pl.trace, s, BMap{}, grid, rd);
    launch_step2<T>(X, g, Z, D, nullptr, (const T*)pl.C, Pz, nullptr, GT, nX, r, k, 0, is_hstep,
                    pl.kp, pl.st, pl.partsB, nullptr, 0, pl.partsC, s, BMap{}, grid,
                    pl.p.inner_iters - 1, rd);
  }
}

template <typename T>
snmf_status run(NmfPlan& pl, const void* W0, const void* Ht0, void* W_out, void* Ht_out,
                snmf_info* info, double* trace) {
  const int64_t m = pl.m, n = pl.n;
  const int r = pl.r;
  hipStream_t s = pl.s;
  HIP_TRY(hipMemcpyAsync(pl.Wb, W0, (size_t)m * r * sizeof(T), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(pl.Hb, Ht0, (size_t)n * r * sizeof(T), hipMemcpyDeviceToDevice, s));
  launch_reset_state(pl.st, pl.normV2, s);
  HIP_TRY(hipGetLastError());
  T* W = (T*)pl.Wb;
  T* H = (T*)pl.Hb;
  const int every = std::max(1, pl.p.check_every);
  for (int i = 0; i < pl.p.max_outer; ++i) {
    half_step<T>(pl, W, m, H, n, 0, true, true, s);
    half_step<T>(pl, H, n, W, m, 1, true, true, s);
    HIP_TRY(hipGetLastError());
    if ((i + 1) % every == 0 && i + 1 < pl.p.max_outer) {
      int32_t done = 0;
      HIP_TRY(hipMemcpyAsync(&done, &pl.st->done, sizeof(done), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (done) break;
    }
  }
  half_step<T>(pl, W, m, H, n, 0, false, false, s);  // the last outer iteration's record
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(W_out, pl.Wb, (size_t)m * r * sizeof(T), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(Ht_out, pl.Hb, (size_t)n * r * sizeof(T), hipMemcpyDeviceToDevice, s));
  State hs;
  HIP_TRY(hipMemcpyAsync(&hs, pl.st, sizeof(State), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double hz = snmf_clock_rate_hz();
  double ticks_last = 0.0, ticks_conv = 0.0;
  if (hs.trace_len > 0) {
    if (trace) {
      HIP_TRY(hipMemcpyAsync(trace, pl.trace, (size_t)hs.trace_len * kTraceFields * 8,
                             hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipMemcpyAsync(&ticks_last, pl.trace + (size_t)(hs.trace_len - 1) * kTraceFields + 5,
                           8, hipMemcpyDeviceToHost, s));
    if (hs.converged_at > 0)
      HIP_TRY(hipMemcpyAsync(&ticks_conv, pl.trace + (size_t)(hs.converged_at - 1) * kTraceFields + 5,
                             8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (trace)  // the symmetric measures have no meaning for W (m x r) and Ht (n x r)
      for (int q = 0; q < hs.trace_len; ++q) {
        trace[(size_t)q * kTraceFields + 1] = NAN;
        trace[(size_t)q * kTraceFields + 2] = NAN;
      }
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
    info->res_WWt = NAN;
    info->sym_gap = NAN;
    info->pg_norm = hs.pg_last;
    info->objective = hs.f_last;
    info->normA2 = pl.normV2;
    info->seconds = hs.trace_len > 0 ? ticks_last / hz : 0.0;
    info->seconds_to_target = hs.converged_at > 0 ? ticks_conv / hz : -1.0;
  }
  if (hs.status != 0) return fail((snmf_status)hs.status, "numeric breakdown during the solve");
  return SNMF_OK;
}

snmf_status nmf_solve(const snmf_matrix* V, int64_t ncols, int32_t r, const void* W0,
                      const void* Ht0, const snmf_params* p, void* W_out, void* Ht_out,
                      snmf_info* info, hipStream_t s, double* trace) {
  SNMF_TRY(check_params(p));
  if (!V) return fail(SNMF_E_ARG, "V is NULL");
  if (!W0 || !Ht0 || !W_out || !Ht_out) return fail(SNMF_E_ARG, "W0, Ht0, W_out and Ht_out are required");
  if (V->fmt == SNMF_LOWRANK) return fail(SNMF_E_UNSUPPORTED, "NMF takes dense or CSR V");
  if (V->fmt != SNMF_DENSE && V->fmt != SNMF_CSR) return fail(SNMF_E_ARG, "V: unknown format");
  if (V->n < 1 || V->n >= ((int64_t)1 << 31)) return fail(SNMF_E_SHAPE, "V: m must lie in [1, 2^31)");
  if (V->fmt == SNMF_DENSE && !V->dense) return fail(SNMF_E_ARG, "V: dense pointer is NULL");
  if (V->fmt == SNMF_CSR) {
    if (!V->rowptr || (V->nnz > 0 && (!V->col || !V->val)))
      return fail(SNMF_E_ARG, "V: CSR pointer is NULL");
    if (V->nnz < 0) return fail(SNMF_E_SHAPE, "V: nnz < 0");
  }
  if (p->prec != SNMF_F32 && p->prec != SNMF_F64)
    return fail(SNMF_E_UNSUPPORTED, "NMF runs in F32 or F64");
  if (p->lambda != 0.0) return fail(SNMF_E_ARG, "NMF has no symmetric penalty: lambda must be 0");
  if (p->L) return fail(SNMF_E_UNSUPPORTED, "NMF takes no Laplacian");
  if (p->naive) return fail(SNMF_E_UNSUPPORTED, "the naive variant is a symmetric one");
  const int64_t m = V->n;
  if (ncols < 1 || ncols >= ((int64_t)1 << 31)) return fail(SNMF_E_SHAPE, "n_cols must lie in [1, 2^31)");
  if (V->fmt == SNMF_DENSE && V->ld < ncols) return fail(SNMF_E_SHAPE, "V: ld < n_cols");
  if (r < 1 || r > kMaxRank) return fail(SNMF_E_SHAPE, "r must lie in [1, 64]");
  if (r > m || r > ncols) return fail(SNMF_E_SHAPE, "r must not exceed m or n");
  NmfPlan pl;
  pl.V = *V;
  pl.m = m;
  pl.n = ncols;
  pl.mx = std::max(m, ncols);
  pl.r = r;
  pl.prec = p->prec;
  pl.esz = elt_size(p->prec);
  pl.p = *p;
  pl.kp = kparams_of(*p, false);
  pl.s = s;
  pl.grid = inner_grid(pl.mx, r, (int)pl.esz, fused_inner_ok(pl.p));
  const size_t xr = (size_t)pl.mx * r * pl.esz;
  std::pair<void**, size_t> req[40];
  int nreq = 0;
  auto add = [&](void** dst, size_t bytes) {
    req[nreq++] = {dst, (std::max<size_t>(bytes, 1) + 255) / 256 * 256};
  };
  add(&pl.Wb, (size_t)m * r * pl.esz);
  add(&pl.Hb, (size_t)ncols * r * pl.esz);
  add(&pl.C, xr);
  add(&pl.g, xr);
  add(&pl.Z, xr);
  add(&pl.gs, xr);  // the fused inner kernels' trial gradient (the trial update goes to Z)
  add(&pl.D, xr);
  add(&pl.B, xr);
  add(&pl.Pz, xr);
  add(&pl.GT[0], (size_t)r * r * pl.esz);
  add(&pl.GT[1], (size_t)r * r * pl.esz);
  add((void**)&pl.G64[0], (size_t)r * r * 8);
  add((void**)&pl.G64[1], (size_t)r * r * 8);
  add((void**)&pl.part, (size_t)2 * kMaxGrid * kNumPart * 8);
  add((void**)&pl.gram_part, (size_t)gram_blocks(pl.mx) * r * r * 8);
  add((void**)&pl.dots, 64 * 8);
  add((void**)&pl.partsA, (size_t)kInnerGrid * kNumPart * 8);
  add((void**)&pl.partsB, (size_t)kInnerGrid * kNumPart * 8);
  add((void**)&pl.partsC, (size_t)kInnerGrid * kNumPart * 8);
  add((void**)&pl.partsD, (size_t)kInnerGrid * kNumPart * 8);
  add((void**)&pl.trace, (size_t)p->max_outer * kTraceFields * 8);
  add((void**)&pl.st, sizeof(State));
  add((void**)&pl.counters, C_COUNT * sizeof(unsigned));
  add((void**)&pl.flags, 4 * sizeof(unsigned));
  if (V->fmt == SNMF_DENSE && p->prec == SNMF_F32) {
    if ((m + 63) / 64 > 65535 || (ncols + 63) / 64 > 65535)
      return fail(SNMF_E_SHAPE, "V: FP32 dense NMF takes m, n_cols <= 4194240");
    pl.spW = rect_split(ncols, m);  // W-step: K = n_cols, output rows m
    pl.spH = rect_split(m, ncols);  // H-step: K = m, output rows n_cols
    add(&pl.VT, (size_t)m * ncols * 4);
    add(&pl.Bpart, (size_t)std::max<int64_t>(pl.spW.ksplit * m, pl.spH.ksplit * ncols) * r * 4);
  }
  if (V->fmt == SNMF_CSR) {
    add((void**)&pl.cnt, (size_t)ncols * sizeof(unsigned));
    add((void**)&pl.cursor, (size_t)ncols * 8);
    add((void**)&pl.rowptrT, (size_t)(ncols + 1) * 8);
    add((void**)&pl.colT, (size_t)V->nnz * 4);
    add(&pl.valT, (size_t)V->nnz * pl.esz);
  }
  size_t total = 0;
  for (int q = 0; q < nreq; ++q) total += req[q].second;
  HIP_TRY(hipMalloc(&pl.pool, total));
  size_t off = 0;
  for (int q = 0; q < nreq; ++q) {
    *req[q].first = (char*)pl.pool + off;
    off += req[q].second;
  }
  HIP_TRY(hipMemsetAsync(pl.counters, 0, C_COUNT * sizeof(unsigned), s));
  HIP_TRY(hipMemsetAsync(pl.st, 0, sizeof(State), s));
  HIP_TRY(hipMemsetAsync(pl.Pz, 0, xr, s));
  double st3[3] = {0, 0, 0};
  if (V->fmt == SNMF_DENSE) {
    if (pl.prec == SNMF_F64)
      SNMF_TRY(stats<double>(pl, (const double*)V->dense, m, ncols, V->ld, st3));
    else
      SNMF_TRY(stats<float>(pl, (const float*)V->dense, m, ncols, V->ld, st3));
    if (p->validate) SNMF_TRY(check_vals(st3, "V"));
  } else {
    HIP_TRY(hipMemsetAsync(pl.flags, 0, 4 * sizeof(unsigned), s));
    launch_csr_check_rect(V->rowptr, V->col, m, ncols, V->nnz, pl.flags, s);
    HIP_TRY(hipGetLastError());
    unsigned f[4];
    HIP_TRY(hipMemcpyAsync(f, pl.flags, sizeof(f), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (f[0] || f[1] || f[2])
      return fail(SNMF_E_SHAPE, "V: malformed CSR (row pointers, columns in [0, n), strictly "
                                "increasing columns per row)");
    if (V->nnz > 0) {
      if (pl.prec == SNMF_F64)
        SNMF_TRY(stats<double>(pl, (const double*)V->val, 1, V->nnz, V->nnz, st3));
      else
        SNMF_TRY(stats<float>(pl, (const float*)V->val, 1, V->nnz, V->nnz, st3));
    }
    if (p->validate) SNMF_TRY(check_vals(st3, "V"));
    if (pl.prec == SNMF_F64)
      launch_csr_transpose<double>(V->rowptr, V->col, (const double*)V->val, m, ncols, V->nnz,
                                   pl.cnt, pl.cursor, pl.rowptrT, pl.colT, (double*)pl.valT, s);
    else
      launch_csr_transpose<float>(V->rowptr, V->col, (const float*)V->val, m, ncols, V->nnz,
                                  pl.cnt, pl.cursor, pl.rowptrT, pl.colT, (float*)pl.valT, s);
    HIP_TRY(hipGetLastError());
  }
  pl.normV2 = st3[0];
  if (!(pl.normV2 > 0.0)) return fail(SNMF_E_ARG, "V is zero");
  if (pl.VT) {
    launch_transpose<float>((const float*)V->dense, m, ncols, V->ld, (float*)pl.VT, s);
    HIP_TRY(hipGetLastError());
  }
  if (p->validate) {
    double w3[3], h3[3];
    if (pl.prec == SNMF_F64) {
      SNMF_TRY(stats<double>(pl, (const double*)W0, m, r, r, w3));
      SNMF_TRY(stats<double>(pl, (const double*)Ht0, ncols, r, r, h3));
    } else {
      SNMF_TRY(stats<float>(pl, (const float*)W0, m, r, r, w3));
      SNMF_TRY(stats<float>(pl, (const float*)Ht0, ncols, r, r, h3));
    }
    SNMF_TRY(check_vals(w3, "W0"));
    SNMF_TRY(check_vals(h3, "Ht0"));
  }
  if (pl.prec == SNMF_F64) return run<double>(pl, W0, Ht0, W_out, Ht_out, info, trace);
  return run<float>(pl, W0, Ht0, W_out, Ht_out, info, trace);
}

}  // namespace

extern "C" {

snmf_status snmf_nmf_solve(const snmf_matrix* V, int64_t n_cols, int32_t r, const void* W0,
                           const void* Ht0, const snmf_params* p, void* W_out, void* Ht_out,
                           snmf_info* info, void* stream, double* trace) {
  return nmf_solve(V, n_cols, r, W0, Ht0, p, W_out, Ht_out, info, (hipStream_t)stream, trace);
}

}  // extern "C"
