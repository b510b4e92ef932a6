// Host side and C ABI of the learned warm start (include/snmf.h, snmf_mlp_* and
// snmf_batch_frame / targets / warmstart).  Every step runs in the kernels of
// k_warmstart.hip and, for the sketch Y = A Omega, in the batch's stacked A-pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/snmf.h"
#include "batch_impl.hpp"
#include "common.hpp"
#include "host.hpp"
#include "kernels.hpp"

using namespace snmf;

namespace {

snmf_status check_mlp(const snmf_mlp* m, bool training) {
  if (!m) return fail(SNMF_E_ARG, "network is NULL");
  if (m->r < 1 || m->r > kMaxRank) return fail(SNMF_E_SHAPE, "network r must lie in [1, 64]");
  if (m->hidden != kMlpHidden) return fail(SNMF_E_UNSUPPORTED, "network hidden width must be 128");
  if (!m->M1 || !m->b1 || !m->M2 || !m->b2 || !m->M1h || !m->M2h)
    return fail(SNMF_E_ARG, "network weight pointers are required");
  if (training && (!m->adam_m || !m->adam_v))
    return fail(SNMF_E_ARG, "training needs the Adam moment arrays");
  return SNMF_OK;
}

MlpDev dev_of(const snmf_mlp* m) {
  MlpDev d{};
  d.r = m->r;
  d.M1 = m->M1;
  d.b1 = m->b1;
  d.M2 = m->M2;
  d.b2 = m->b2;
  d.M1h = m->M1h;
  d.M2h = m->M2h;
  d.mom = m->adam_m;
  d.vel = m->adam_v;
  return d;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct WorkLayout {
  size_t y, a, o, dO, dA, grad, part, total;
};
WorkLayout work_layout(int r, int64_t B) {
  WorkLayout w{};
  size_t at = 0;
  w.y = at;
  at += align256((size_t)B * r * 4);
  w.a = at;
  at += align256((size_t)B * kMlpHidden * 4);
  w.o = at;
  at += align256((size_t)B * r * 4);
  w.dO = at;
  at += align256((size_t)B * r * 4);
  w.dA = at;
  at += align256((size_t)B * kMlpHidden * 4);
  w.grad = at;
  at += align256((size_t)mlp_params(r) * 4);
  w.part = at;
  at += align256(((size_t)kMaxGrid * kNumPart + 1) * 8);
  w.total = at;
  return w;
}

snmf_status begin(snmf_batch* b, hipStream_t user) {
  if (user) {
    HIP_TRY(hipEventRecord(b->ev_in, user));
    HIP_TRY(hipStreamWaitEvent(b->s, b->ev_in, 0));
  }
  return SNMF_OK;
}
snmf_status finish(snmf_batch* b, hipStream_t user) {
  if (user) {
    HIP_TRY(hipEventRecord(b->ev_out, b->s));
    HIP_TRY(hipStreamWaitEvent(user, b->ev_out, 0));
  }
  return SNMF_OK;
}

snmf_status ws_scratch(snmf_batch* b) {
  if (!b->wsR) HIP_TRY(hipMalloc((void**)&b->wsR, std::max<size_t>(8, (size_t)b->total * 8)));
  if (!b->wsI) HIP_TRY(hipMalloc((void**)&b->wsI, (size_t)b->ninst * kMaxRank * 4));
  return SNMF_OK;
}

// Dense problems: the degrees d = A 1 of every problem and a table that hands them to the
// frame kernel (CSR problems sum their rows inside it).
snmf_status dense_degrees(snmf_batch* b) {
  if (!b->wsDeg) {
    int64_t tot = 0;
    for (int g = 0; g < b->nprob; ++g) tot += b->n[g];
    HIP_TRY(hipMalloc((void**)&b->wsDeg, (size_t)tot * 8));
    HIP_TRY(hipMalloc((void**)&b->wsG, (size_t)b->nprob * sizeof(BGraph)));
    std::vector<BGraph> tab(b->nprob);
    int64_t at = 0;
    for (int g = 0; g < b->nprob; ++g) {
      std::memset(&tab[g], 0, sizeof(BGraph));
      tab[g].val = b->A[g].dense;
      tab[g].deg = b->wsDeg + at;
      tab[g].n = b->n[g];
      tab[g].r = b->r[g];
      tab[g].S = b->S;
      at += b->n[g];
    }
    HIP_TRY(hipMemcpyAsync(b->wsG, tab.data(), tab.size() * sizeof(BGraph), hipMemcpyHostToDevice,
                           b->s));
    HIP_TRY(hipStreamSynchronize(b->s));
  }
  int64_t at = 0;
  for (int g = 0; g < b->nprob; ++g) {
    if (b->prec == SNMF_F64)
      launch_dense_rowsum<double>((const double*)b->A[g].dense, b->n[g], b->A[g].ld, b->wsDeg + at,
                                  b->s);
    else
      launch_dense_rowsum<float>((const float*)b->A[g].dense, b->n[g], b->A[g].ld, b->wsDeg + at,
                                 b->s);
    at += b->n[g];
  }
  HIP_TRY(hipGetLastError());
  return SNMF_OK;
}

// Y = A Omega, then the frame of every instance into C (stream b->s).
snmf_status frame_async(snmf_batch* b, const void* Omega, void* Y, void* C, int32_t* anchors) {
  if (b->dense && b->prec == SNMF_BF16X3)
    return fail(SNMF_E_UNSUPPORTED, "the warm start of dense problems runs in F32 or F64");
  SNMF_TRY(ws_scratch(b));
  if (b->dense) SNMF_TRY(dense_degrees(b));
  const BGraph* graphs = b->dense ? b->wsG : b->dgraph;
  launch_breset(b->states, b->dinst, b->ninst, b->s);  // clears the done flags the A-pass reads
  SNMF_TRY(batch_apass_async(b, Omega, Y, b->s));
  int32_t* anc = anchors ? anchors : b->wsI;
  if (b->prec == SNMF_F64)
    launch_ws_frame<double>(b->dinst, b->ninst, b->max_r, graphs, (const double*)Y, b->wsR,
                            (double*)C, anc, b->s);
  else
    launch_ws_frame<float>(b->dinst, b->ninst, b->max_r, graphs, (const float*)Y, b->wsR,
                           (float*)C, anc, b->s);
  HIP_TRY(hipGetLastError());
  return SNMF_OK;
}

}  // namespace

extern "C" {

snmf_status snmf_mlp_sync(const snmf_mlp* m, void* stream) {
  SNMF_TRY(check_mlp(m, false));
  launch_mlp_sync(dev_of(m), (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return SNMF_OK;
}

snmf_status snmf_mlp_forward(const snmf_mlp* m, int64_t rows, const float* C,
                             const float* row_scale, float* Y, void* stream) {
  SNMF_TRY(check_mlp(m, false));
  if (rows < 0) return fail(SNMF_E_SHAPE, "rows < 0");
  if (rows == 0) return SNMF_OK;
  if (!C || !Y) return fail(SNMF_E_ARG, "C and Y are required");
  launch_mlp_forward(dev_of(m), rows, C, row_scale, Y, BMap{}, 0, nullptr, 0, nullptr, nullptr,
                     (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return SNMF_OK;
}

size_t snmf_mlp_workspace_bytes(int32_t r, int64_t batch) {
  if (r < 1 || r > kMaxRank || batch < 1) return 0;
  return work_layout(r, batch).total;
}

snmf_status snmf_mlp_train_step(const snmf_mlp* m, int64_t pool_rows, const float* C,
                                const float* T, const int32_t* idx, int64_t batch, float mu,
                                float lr, int32_t step, void* work, size_t work_bytes,
                                void* stream, double* loss) {
  SNMF_TRY(check_mlp(m, true));
  if (!C || !T || !idx || !work) return fail(SNMF_E_ARG, "C, T, idx and work are required");
  if (pool_rows < 1) return fail(SNMF_E_SHAPE, "pool_rows must be >= 1");
  if (batch < 1 || batch > (int64_t)1 << 24) return fail(SNMF_E_SHAPE, "batch must lie in [1, 2^24]");
  if (step < 1) return fail(SNMF_E_ARG, "step counts from 1");
  if (!(lr > 0.0f) || !(mu >= 0.0f)) return fail(SNMF_E_ARG, "need lr > 0 and mu >= 0");
  const WorkLayout L = work_layout(m->r, batch);
  if (work_bytes < L.total) return fail(SNMF_E_ARG, "workspace too small");
  char* w = (char*)work;
  MlpWork mw{};
  mw.y = (float*)(w + L.y);
  mw.cache_a = (float*)(w + L.a);
  mw.cache_o = (float*)(w + L.o);
  mw.dO = (float*)(w + L.dO);
  mw.dA = (float*)(w + L.dA);
  mw.grad = (float*)(w + L.grad);
  mw.part = (double*)(w + L.part);
  hipStream_t s = (hipStream_t)stream;
  launch_mlp_train_step(dev_of(m), pool_rows, batch, C, T, idx, mu, lr, step, mw, s);
  HIP_TRY(hipGetLastError());
  if (loss) {
    HIP_TRY(hipMemcpyAsync(loss, mw.part + (size_t)kMaxGrid * kNumPart, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return SNMF_OK;
}

snmf_status snmf_batch_frame(snmf_batch* b, const void* Omega, void* Y, void* C,
                             int32_t* anchors, void* stream) {
  if (!b || !Omega || !Y || !C) return fail(SNMF_E_ARG, "batch, Omega, Y and C are required");
  hipStream_t user = (hipStream_t)stream;
  SNMF_TRY(begin(b, user));
  SNMF_TRY(frame_async(b, Omega, Y, C, anchors));
  HIP_TRY(hipStreamSynchronize(b->s));
  return finish(b, user);
}

snmf_status snmf_batch_targets(snmf_batch* b, const void* C, const void* Ht, void* T,
                               int32_t* perm, void* stream) {
  if (!b || !C || !Ht || !T) return fail(SNMF_E_ARG, "batch, C, Ht and T are required");
  SNMF_TRY(ws_scratch(b));
  hipStream_t user = (hipStream_t)stream;
  SNMF_TRY(begin(b, user));
  int32_t* pp = perm ? perm : b->wsI;
  if (b->prec == SNMF_F64)
    launch_ws_match<double>(b->dinst, b->ninst, (const double*)C, (const double*)Ht, (double*)T, pp,
                            b->s);
  else
    launch_ws_match<float>(b->dinst, b->ninst, (const float*)C, (const float*)Ht, (float*)T, pp,
                           b->s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(b->s));
  return finish(b, user);
}

snmf_status snmf_batch_warmstart(snmf_batch* b, int32_t nmodels, const snmf_mlp* models,
                                 const void* Omega, void* W0, void* stream) {
  if (!b || !Omega || !W0 || (nmodels > 0 && !models))
    return fail(SNMF_E_ARG, "batch, models, Omega and W0 are required");
  hipStream_t user = (hipStream_t)stream;
  if (nmodels == 0) {  // the frame alone: W0 = s relu(C) / rms(relu(C))
    SNMF_TRY(begin(b, user));
    SNMF_TRY(frame_async(b, Omega, b->B, b->C, nullptr));
    if (b->prec == SNMF_F64)
      launch_ws_spa_only<double>(b->dinst, b->ninst, (const double*)b->C, (double*)W0, b->s);
    else
      launch_ws_spa_only<float>(b->dinst, b->ninst, (const float*)b->C, (float*)W0, b->s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(b->s));
    return finish(b, user);
  }
  if (b->prec != SNMF_F32) return fail(SNMF_E_UNSUPPORTED, "the warm start network runs in FP32");
  const snmf_mlp* pick[kMaxRank + 1] = {};
  for (int q = 0; q < nmodels; ++q) {
    SNMF_TRY(check_mlp(&models[q], false));
    pick[models[q].r] = &models[q];
  }
  for (const auto& c : b->cls)
    if (!pick[c.r]) return fail(SNMF_E_ARG, "no network for rank " + std::to_string(c.r));
  SNMF_TRY(begin(b, user));
  // the sketch lands in B, the coordinates in C (solve scratch, free between solves)
  SNMF_TRY(frame_async(b, Omega, b->B, b->C, nullptr));
  for (const auto& c : b->cls) {
    launch_mlp_forward(dev_of(pick[c.r]), 0, (const float*)b->C, nullptr, (float*)W0, b->bmap(c),
                       c.blocks, nullptr, 0, nullptr, nullptr, b->s);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(b->s));
  return finish(b, user);
}

snmf_status snmf_warmstart(const snmf_mlp* mlp, const snmf_matrix* A, int32_t r, int32_t prec,
                           const void* Omega, void* W0_out, void* stream) {
  if (!A || !Omega || !W0_out) return fail(SNMF_E_ARG, "A, Omega and W0_out are required");
  if (A->fmt == SNMF_LOWRANK) return fail(SNMF_E_UNSUPPORTED, "the warm start takes dense or CSR A");
  if (prec != SNMF_F32 && prec != SNMF_F64) return fail(SNMF_E_ARG, "prec must be F32 or F64");
  if (mlp) {
    SNMF_TRY(check_mlp(mlp, false));
    if (mlp->r != r) return fail(SNMF_E_SHAPE, "the network's rank differs from r");
    if (prec != SNMF_F32) return fail(SNMF_E_UNSUPPORTED, "the warm start network runs in FP32");
  }
  snmf_params p;
  SNMF_TRY(snmf_params_default(&p));
  p.prec = prec;
  p.max_outer = 1;
  snmf_batch* b = nullptr;
  SNMF_TRY(snmf_batch_create(1, A, &r, nullptr, 1, &p, stream, &b));
  snmf_status s = snmf_batch_warmstart(b, mlp ? 1 : 0, mlp, Omega, W0_out, stream);
  std::string keep = err_ref();
  snmf_batch_destroy(b);
  err_ref() = keep;
  return s;
}

}  // extern "C"
