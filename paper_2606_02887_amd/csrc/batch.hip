// Batched SNMPBB solves: host orchestration and the snmf_batch_* C ABI (include/snmf.h).
//
// Instances (problem g, restart s) are numbered i = g S + s and stored one after another
// (instance-major): every batch buffer (W, Ht, C, g, Z, D, B) holds instance i's n_g x r_g
// block at element offset off_i.  Per half-step, in stream order:
//   Gram of every instance (one launch) -> rho of every instance (one launch)
//   -> A-pass (stacked CSR SpMM: one sweep per problem for all its restarts; dense: one
//   product per instance) -> init -> inner_iters x (step1, step2)
// where init/step1/step2 run one launch per distinct rank (their tile shape depends on
// it), each workgroup finding its instance in a table.  Every instance has its own State
// and partial-sum rows, so it iterates exactly like a single solve of its problem; a
// finished instance's workgroups return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/snmf.h"
#include "common.hpp"
#include "batch_impl.hpp"
#include "host.hpp"
#include "kernels.hpp"

using namespace snmf;

namespace {

// ||x||^2, negative and non-finite counts of a rows x cols array (leading dimension ld).
snmf_status bstats(snmf_batch* b, const void* x, int64_t rows, int64_t cols, int64_t ld,
                   double* out3) {
  if (b->prec == SNMF_F64)
    launch_stats2d<double>((const double*)x, rows, cols, ld, b->part, b->dots,
                           b->counters + C_NORM, b->s);
  else
    launch_stats2d<float>((const float*)x, rows, cols, ld, b->part, b->dots, b->counters + C_NORM,
                          b->s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out3, b->dots, 3 * sizeof(double), hipMemcpyDeviceToHost, b->s));
  HIP_TRY(hipStreamSynchronize(b->s));
  return SNMF_OK;
}

snmf_status bcheck_csr(snmf_batch* b, const snmf_matrix* M, const std::string& what,
                       double* sumsq) {
  HIP_TRY(hipMemsetAsync(b->flags, 0, 4 * sizeof(unsigned), b->s));
  launch_csr_structure(M->rowptr, M->col, M->n, M->nnz, b->flags, b->s);
  HIP_TRY(hipGetLastError());
  unsigned f[4];
  HIP_TRY(hipMemcpyAsync(f, b->flags, sizeof(f), hipMemcpyDeviceToHost, b->s));
  HIP_TRY(hipStreamSynchronize(b->s));
  if (f[0] || f[1]) return fail(SNMF_E_SHAPE, what + ": malformed CSR structure");
  if (b->p.validate && f[2] == 0) {
    if (b->prec == SNMF_F64)
      launch_csr_symmetry<double>(M->rowptr, M->col, (const double*)M->val, M->n, b->flags, b->s);
    else
      launch_csr_symmetry<float>(M->rowptr, M->col, (const float*)M->val, M->n, b->flags, b->s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(f, b->flags, sizeof(f), hipMemcpyDeviceToHost, b->s));
    HIP_TRY(hipStreamSynchronize(b->s));
    if (f[3]) return fail(SNMF_E_NOT_SYMMETRIC, what + " is not symmetric");
  }
  double st3[3] = {0, 0, 0};
  if (M->nnz > 0) SNMF_TRY(bstats(b, M->val, 1, M->nnz, M->nnz, st3));
  if (st3[2] > 0) return fail(SNMF_E_NONFINITE, what + " has NaN/Inf entries");
  if (b->p.validate && st3[1] > 0) return fail(SNMF_E_NEGATIVE, what + " has negative entries");
  *sumsq = st3[0];
  return SNMF_OK;
}

// G64 set (dense BF16X3 only): rho of every instance inside the stacked A-pass launches
// (the product's when its workgroups fit, else the split's), from its Gram in G64
template <typename T>
snmf_status bapass(snmf_batch* b, const T* P, T* B, hipStream_t s,
                   const double* G64 = nullptr) {
  if (!b->dense) {
    launch_bspmm<T>(b->dgraph, b->sblk_tab, b->sblocks, b->states, P, B, s);
    HIP_TRY(hipGetLastError());
    return SNMF_OK;
  }
  if (b->prec == SNMF_BF16X3) {
    // one stacked split-BF16 product per problem: its S restarts are consecutive blocks
    for (int g = 0; g < b->nprob; ++g) {
      const BInst& d = b->hinst[(size_t)g * b->S];
      const DenseSplit& sp = b->ds[g];
      const int64_t snr = (int64_t)b->S * d.n * d.r;
      State* st = b->states + (size_t)g * b->S;
      const double* Grho = G64 ? G64 + d.goff : nullptr;
      // rho rides in the product launch when its workgroups find free slots there, else
      // in the split launch (its tiles are short, so rho sets that launch's length)
      launch_split_pt_stack((const float*)(P + d.off), d.n, d.r, b->S, b->ldb[g], b->Pthi,
                            b->Ptlo, st, b->rho_in_apass ? nullptr : Grho, s);
      const double* Grho_ap = b->rho_in_apass ? Grho : nullptr;
      if (sp.ksplit == 1) {
        launch_apass_bf16x3_stack(b->Ahi[g], b->Alo[g], b->ldb[g], b->Pthi, b->Ptlo, d.n, d.r,
                                  b->S, sp, (float*)(B + d.off), 0, st, Grho_ap, s);
      } else {
        launch_apass_bf16x3_stack(b->Ahi[g], b->Alo[g], b->ldb[g], b->Pthi, b->Ptlo, d.n, d.r,
                                  b->S, sp, (float*)b->Bpart, snr, st, Grho_ap, s);
        launch_sum_parts<float>((const float*)b->Bpart, sp.ksplit, snr, (float*)(B + d.off), snr,
                                s);
      }
      HIP_TRY(hipGetLastError());
    }
    return SNMF_OK;
  }
  for (int i = 0; i < b->ninst; ++i) {
    const BInst& d = b->hinst[i];
    const snmf_matrix& A = b->A[d.prob];
    const int64_t nr = d.n * d.r;
    if (b->prec == SNMF_F64) {
      launch_apass_f64((const double*)A.dense, A.ld, (const double*)(P + d.off), d.n, d.r,
                       (double*)(B + d.off), b->states + i, s);
    } else {
      const DenseSplit& sp = b->ds[d.prob];
      launch_apass_f32((const float*)A.dense, A.ld, (const float*)(P + d.off), d.n, d.r, sp,
                       (float*)b->Bpart, nr, b->states + i, s);
      launch_sum_parts<float>((const float*)b->Bpart, sp.ksplit, nr, (float*)(B + d.off), nr, s);
    }
    HIP_TRY(hipGetLastError());
  }
  return SNMF_OK;
}

template <typename T>
snmf_status bhalf_start(snmf_batch* b, T* X, const T* P, int is_hstep, bool with_rho,
                        hipStream_t s) {
  const int gi = is_hstep ? 1 : 0;
  for (const auto& c : b->cls)
    launch_bgram<T>(P, c.r, b->gblk_tab + c.gtab_off, c.gblocks, b->dinst, b->states, b->gpart, s);
  launch_bgram_reduce<T>(b->dinst, b->ninst, b->max_r, b->states, b->gpart, b->G64[gi],
                         (T*)b->GT[gi], s);
  HIP_TRY(hipGetLastError());
  // dense BF16X3: rho runs inside the stacked A-pass launches (product or split)
  const bool rho_in_apass = b->dense && b->prec == SNMF_BF16X3;
  if (with_rho && !rho_in_apass) {
    launch_brho(b->dinst, b->ninst, b->states, b->G64[gi], s);
    HIP_TRY(hipGetLastError());
  }
  SNMF_TRY(bapass<T>(b, P, (T*)b->B, s, with_rho && rho_in_apass ? b->G64[gi] : nullptr));
  for (const auto& c : b->cls) {
    launch_init<T>(X, P, (const T*)b->B, 1, 0, (T*)b->C, (T*)b->g, nullptr, (const T*)b->GT[gi], 0,
                   c.r, is_hstep, b->kp, b->states, b->partsA, s, b->bmap(c), c.blocks);
  }
  HIP_TRY(hipGetLastError());
  return SNMF_OK;
}

template <typename T>
snmf_status binner(snmf_batch* b, T* X, const T* P, int is_hstep, hipStream_t s) {
  const int gi = is_hstep ? 1 : 0;
  const T* GT = (const T*)b->GT[gi];
  for (int k = 0; k < b->p.inner_iters; ++k) {
    for (const auto& c : b->cls)
      launch_step1<T>(X, (const T*)b->g, (T*)b->Z, (T*)b->D, nullptr, GT, b->G64[0], b->G64[1], 0,
                      c.r, k, 0, is_hstep, b->kp, b->states, b->partsA, b->partsB, b->partsC,
                      b->traces, s, b->bmap(c), c.blocks, 1);
    for (const auto& c : b->cls)
      launch_step2<T>(X, (T*)b->g, (T*)b->Z, (T*)b->D, nullptr, (const T*)b->C, P, nullptr, GT, 0,
                      c.r, k, 0, is_hstep, b->kp, b->states, b->partsB, nullptr, 0, b->partsC, s,
                      b->bmap(c), c.blocks, b->p.inner_iters - 1, 1);
  }
  HIP_TRY(hipGetLastError());
  return SNMF_OK;
}

template <typename T>
snmf_status bouter(snmf_batch* b, hipStream_t s) {
  T* W = (T*)b->Wb;
  T* H = (T*)b->Hb;
  SNMF_TRY(bhalf_start<T>(b, W, H, 0, true, s));
  SNMF_TRY(binner<T>(b, W, H, 0, s));
  SNMF_TRY(bhalf_start<T>(b, H, W, 1, true, s));
  SNMF_TRY(binner<T>(b, H, W, 1, s));
  return SNMF_OK;
}

// Monitor record of the last outer iteration (see the single solve): one more W-step
// start whose first inner kernel completes every instance's record.
template <typename T>
snmf_status bfinalize(snmf_batch* b, hipStream_t s) {
  T* W = (T*)b->Wb;
  const T* H = (const T*)b->Hb;
  SNMF_TRY(bhalf_start<T>(b, W, H, 0, false, s));
  for (const auto& c : b->cls)
    launch_step1<T>(W, (const T*)b->g, (T*)b->Z, (T*)b->D, nullptr, (const T*)b->GT[0], b->G64[0],
                    b->G64[1], 0, c.r, 0, 0, 0, b->kp, b->states, b->partsA, b->partsB, b->partsC,
                    b->traces, s, b->bmap(c), c.blocks, 1);  // D is never read after it
  HIP_TRY(hipGetLastError());
  return SNMF_OK;
}

snmf_status batch_create(int32_t nprob, const snmf_matrix* A, const int32_t* r, const double* lam,
                         int32_t restarts, const snmf_params* p, hipStream_t user,
                         snmf_batch** out) {
  if (!out) return fail(SNMF_E_ARG, "out is NULL");
  *out = nullptr;
  SNMF_TRY(check_params(p));
  if (p->naive) return fail(SNMF_E_UNSUPPORTED, "the naive variant runs as single solves only");
  int tpb_cls[4] = {4, 4, 4, 4};  // row tiles per inner-kernel workgroup, per rank class
  int spmm_rows = 16;              // rows per workgroup of the batched SpMM
  if (p->tuning) {
    const snmf_batch_tuning& t = *p->tuning;
    for (int q = 0; q < 4; ++q) {
      if (t.tiles_per_wg[q] < 1 || t.tiles_per_wg[q] > 64)
        return fail(SNMF_E_ARG, "tuning: tiles_per_wg must lie in [1, 64]");
      tpb_cls[q] = t.tiles_per_wg[q];
    }
    if (t.spmm_rows_per_wg < 1 || t.spmm_rows_per_wg > 4096)
      return fail(SNMF_E_ARG, "tuning: spmm_rows_per_wg must lie in [1, 4096]");
    if (t.reserved[0] || t.reserved[1] || t.reserved[2])
      return fail(SNMF_E_ARG, "tuning: reserved fields must be 0");
    spmm_rows = t.spmm_rows_per_wg;
  }
  if (nprob < 1) return fail(SNMF_E_ARG, "nprob must be >= 1");
  if (restarts < 1) return fail(SNMF_E_ARG, "restarts must be >= 1");
  if (!A || !r) return fail(SNMF_E_ARG, "A and r are required");
  const bool dense = A[0].fmt == SNMF_DENSE;
  if (p->prec == SNMF_BF16X3 && !dense)
    return fail(SNMF_E_UNSUPPORTED, "batched BF16X3 solves take dense A");
  for (int g = 0; g < nprob; ++g) {
    const std::string what = "A[" + std::to_string(g) + "]";
    SNMF_TRY(check_matrix(&A[g], what.c_str()));
    if (A[g].fmt == SNMF_LOWRANK) return fail(SNMF_E_UNSUPPORTED, "batched solves take CSR or dense A");
    if ((A[g].fmt == SNMF_DENSE) != dense)
      return fail(SNMF_E_UNSUPPORTED, "a batch is all CSR or all dense");
    if (r[g] < 1 || r[g] > kMaxRank) return fail(SNMF_E_SHAPE, "r must lie in [1, 64]");
    if (r[g] > A[g].n) return fail(SNMF_E_SHAPE, "r must not exceed n");
    if (lam && (!(lam[g] >= 0.0) || !std::isfinite(lam[g])))
      return fail(SNMF_E_ARG, "lambda must be >= 0");
  }
  const int64_t ninst64 = (int64_t)nprob * restarts;
  if (ninst64 > (1 << 24)) return fail(SNMF_E_SHAPE, "too many instances");
  auto b = new (std::nothrow) snmf_batch();
  if (!b) return fail(SNMF_E_OOM, "host allocation failed");
  std::unique_ptr<snmf_batch> guard(b);
  b->nprob = nprob;
  b->S = restarts;
  b->ninst = (int)ninst64;
  b->p = *p;
  b->prec = p->prec;
  b->esz = elt_size(p->prec);
  b->dense = dense;
  b->kp = kparams_of(*p, false);
  b->A.assign(A, A + nprob);
  b->r.assign(r, r + nprob);
  b->n.resize(nprob);
  for (int g = 0; g < nprob; ++g) b->n[g] = A[g].n;
  HIP_TRY(hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
  if (user) {
    HIP_TRY(hipEventRecord(b->ev_in, user));
    HIP_TRY(hipStreamWaitEvent(b->s, b->ev_in, 0));
  }

  // ---- instance layout, Gram slabs, rank classes, SpMM workgroups
  b->hinst.resize(b->ninst);
  int64_t off = 0, goff = 0, gpoff = 0;
  int gblk = 0;
  for (int g = 0; g < nprob; ++g) {
    const int64_t ng = b->n[g];
    const int rg = b->r[g];
    b->max_r = std::max(b->max_r, rg);
    b->max_nr = std::max(b->max_nr, ng * rg);
    const int gnb = gram_blocks(ng);
    for (int s = 0; s < restarts; ++s) {
      BInst& d = b->hinst[g * restarts + s];
      std::memset(&d, 0, sizeof(d));
      d.off = off;
      d.n = ng;
      d.r = rg;
      d.goff = goff;
      d.gpoff = gpoff;
      d.gnb = gnb;
      d.grpb = (ng + gnb - 1) / gnb;
      d.lam = lam ? lam[g] : p->lambda;
      d.prob = g;
      d.restart = s;
      off += ng * rg;
      goff += (int64_t)rg * rg;
      gpoff += (int64_t)gnb * rg * rg;
      gblk += gnb;
    }
  }
  b->total = off;
  b->gsum = goff;
  b->gpsum = gpoff;
  b->gblocks = gblk;
  std::vector<int32_t> gtab;
  // classes: instances grouped by rank, in instance order within a class
  std::map<int, std::vector<int>> by_r;
  for (int i = 0; i < b->ninst; ++i) by_r[b->hinst[i].r].push_back(i);
  std::vector<int32_t> btab;
  int part_row = 0;
  // row tiles per inner-kernel workgroup: more than one amortises each workgroup's fixed
  // cost (instance lookup, partial-sum reduction, line search, G staging).  The default 4
  // measured best on 256 graphs x 8 restarts (1: 114k, 2: 132k, 4: 138k, 8: 136k instance
  // outer iterations/s); a tuning picks it per rank class.
  for (auto& kv : by_r) {
    snmf_batch::Cls c;
    c.r = kv.first;
    const int rp = rank_pad(c.r);
    const int tpb = tpb_cls[rp <= 8 ? 0 : rp <= 16 ? 1 : rp <= 32 ? 2 : 3];
    c.tab_off = (int64_t)btab.size();
    c.gtab_off = (int64_t)gtab.size();
    int blk = 0, gb = 0;
    for (int i : kv.second) {
      BInst& d = b->hinst[i];
      d.blk0 = blk;
      {
        const int tm = 8 * kThreads / rank_pad(d.r);
        const int64_t nt = std::max<int64_t>(1, (d.n + tm - 1) / tm);
        d.nblk = (int)std::min<int64_t>(kInnerGrid, (nt + tpb - 1) / tpb);
      }
      d.part0 = part_row;
      for (int j = 0; j < d.nblk; ++j) btab.push_back(i);
      blk += d.nblk;
      part_row += d.nblk;
      d.gblk0 = gb;
      for (int j = 0; j < d.gnb; ++j) gtab.push_back(i);
      gb += d.gnb;
    }
    c.blocks = blk;
    c.gblocks = gb;
    if (blk > 0x7fffffff / 2) return fail(SNMF_E_SHAPE, "batch too large");
    b->cls.push_back(c);
  }
  b->part_rows = part_row;
  std::vector<int32_t> stab;
  if (!dense) {
    b->hgraph.resize(nprob);
    int sblk = 0;
    for (int g = 0; g < nprob; ++g) {
      BGraph& G = b->hgraph[g];
      std::memset(&G, 0, sizeof(G));
      G.rowptr = A[g].rowptr;
      G.col = A[g].col;
      G.val = A[g].val;
      G.n = b->n[g];
      G.off0 = b->hinst[g * restarts].off;
      G.r = b->r[g];
      G.S = restarts;
      G.blk0 = sblk;
      G.nblk = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (G.n + spmm_rows - 1) / spmm_rows));
      G.inst0 = g * restarts;
      for (int j = 0; j < G.nblk; ++j) stab.push_back(g);
      sblk += G.nblk;
    }
    b->sblocks = sblk;
  } else if (b->prec == SNMF_F32) {
    b->ds.resize(nprob);
    for (int g = 0; g < nprob; ++g) {
      b->ds[g] = plan_dense_f32(b->n[g], A[g].ld, b->r[g], A[g].dense);
      b->ksplit_max = std::max(b->ksplit_max, b->ds[g].ksplit);
    }
  }
  // BF16X3: one stacked product per problem over its S r columns
  int64_t pt_max = 0, bpart_max = 0;
  if (dense && b->prec == SNMF_BF16X3) {
    b->ds.resize(nprob);
    b->ldb.resize(nprob);
    b->Ahi.assign(nprob, nullptr);
    b->Alo.assign(nprob, nullptr);
    // rho runs inside the product launch when its S workgroups find free slots beside the
    // product's (stack_per_cu() per CU): a rho workgroup that waits for a slot, or holds one
    // a tile workgroup waits for, lengthens the launch by a whole rho (about 55 us at r = 64).
    // Otherwise it runs inside the partner split's launch, whose tiles are short.
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    b->rho_in_apass = true;
    for (int g = 0; g < nprob; ++g) {
      const int64_t R = (int64_t)restarts * b->r[g];
      b->ds[g] = plan_dense_bf16_stack(b->n[g], R);
      if (b->ds[g].nwg + restarts > stack_per_cu() * (int64_t)cus) b->rho_in_apass = false;
      b->ldb[g] = (b->n[g] + 63) / 64 * 64;
      pt_max = std::max(pt_max, R * b->ldb[g]);
      if (b->ds[g].ksplit > 1)
        bpart_max = std::max(bpart_max, (int64_t)b->ds[g].ksplit * R * b->n[g]);
    }
  }
  b->trace_stride = (int64_t)p->max_outer * kTraceFields;

  // ---- one allocation, carved
  std::vector<std::pair<void**, size_t>> req;
  auto add = [&](void** dst, size_t bytes) {
    req.push_back({dst, (std::max<size_t>(bytes, 1) + 255) / 256 * 256});
  };
  const size_t tb = (size_t)b->total * b->esz;
  add(&b->Wb, tb);
  add(&b->Hb, tb);
  add(&b->C, tb);
  add(&b->g, tb);
  add(&b->Z, tb);
  add(&b->D, tb);
  add(&b->B, tb);
  if (dense && b->prec == SNMF_F32) add(&b->Bpart, (size_t)b->ksplit_max * b->max_nr * b->esz);
  if (dense && b->prec == SNMF_BF16X3) {
    for (int g = 0; g < nprob; ++g) {
      add((void**)&b->Ahi[g], (size_t)b->n[g] * b->ldb[g] * 2);
      add((void**)&b->Alo[g], (size_t)b->n[g] * b->ldb[g] * 2);
    }
    add((void**)&b->Pthi, (size_t)pt_max * 2);
    add((void**)&b->Ptlo, (size_t)pt_max * 2);
    if (bpart_max > 0) add(&b->Bpart, (size_t)bpart_max * 4);
  }
  add(&b->GT[0], (size_t)b->gsum * b->esz);
  add(&b->GT[1], (size_t)b->gsum * b->esz);
  add((void**)&b->G64[0], (size_t)b->gsum * 8);
  add((void**)&b->G64[1], (size_t)b->gsum * 8);
  add((void**)&b->gpart, (size_t)b->gpsum * 8);
  add((void**)&b->partsA, (size_t)b->part_rows * kNumPart * 8);
  add((void**)&b->partsB, (size_t)b->part_rows * kNumPart * 8);
  add((void**)&b->partsC, (size_t)b->part_rows * kNumPart * 8);
  add((void**)&b->traces, (size_t)b->ninst * b->trace_stride * 8);
  add((void**)&b->states, (size_t)b->ninst * sizeof(State));
  add((void**)&b->flag, sizeof(int32_t));
  add((void**)&b->part, (size_t)2 * kMaxGrid * kNumPart * 8);
  add((void**)&b->dots, 64 * 8);
  add((void**)&b->counters, C_COUNT * sizeof(unsigned));
  add((void**)&b->flags, 4 * sizeof(unsigned));
  add((void**)&b->dinst, (size_t)b->ninst * sizeof(BInst));
  add((void**)&b->blk_tab, btab.size() * 4);
  add((void**)&b->gblk_tab, gtab.size() * 4);
  if (!dense) {
    add((void**)&b->dgraph, (size_t)nprob * sizeof(BGraph));
    add((void**)&b->sblk_tab, stab.size() * 4);
  }
  size_t bytes = 0;
  for (auto& q : req) bytes += q.second;
  HIP_TRY(hipMalloc(&b->pool, bytes));
  size_t o = 0;
  for (auto& q : req) {
    *q.first = (char*)b->pool + o;
    o += q.second;
  }
  HIP_TRY(hipMemsetAsync(b->counters, 0, C_COUNT * sizeof(unsigned), b->s));
  HIP_TRY(hipMemsetAsync(b->states, 0, (size_t)b->ninst * sizeof(State), b->s));

  // ---- input checks and ||A_g||^2
  b->normA2.resize(nprob);
  for (int g = 0; g < nprob; ++g) {
    const std::string what = "A[" + std::to_string(g) + "]";
    double st3[3] = {0, 0, 0};
    if (dense) {
      SNMF_TRY(bstats(b, A[g].dense, A[g].n, A[g].n, A[g].ld, st3));
      if (p->validate && st3[2] > 0) return fail(SNMF_E_NONFINITE, what + " has NaN/Inf entries");
      if (p->validate && st3[1] > 0) return fail(SNMF_E_NEGATIVE, what + " has negative entries");
      if (p->check_symmetry)
        SNMF_TRY(check_dense_symmetry(&A[g], b->prec, b->flags, b->s, what.c_str()));
      b->normA2[g] = st3[0];
    } else {
      SNMF_TRY(bcheck_csr(b, &A[g], what, &b->normA2[g]));
    }
    if (!(b->normA2[g] > 0.0)) return fail(SNMF_E_ARG, what + " is zero");
  }
  for (int i = 0; i < b->ninst; ++i) b->hinst[i].normA2 = b->normA2[b->hinst[i].prob];
  if (dense && b->prec == SNMF_BF16X3) {
    for (int g = 0; g < nprob; ++g)
      launch_split_rows((const float*)A[g].dense, b->n[g], A[g].ld, b->ldb[g], b->Ahi[g],
                        b->Alo[g], b->s);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipMemcpyAsync(b->dinst, b->hinst.data(), b->hinst.size() * sizeof(BInst),
                         hipMemcpyHostToDevice, b->s));
  HIP_TRY(hipMemcpyAsync(b->blk_tab, btab.data(), btab.size() * 4, hipMemcpyHostToDevice, b->s));
  HIP_TRY(hipMemcpyAsync(b->gblk_tab, gtab.data(), gtab.size() * 4, hipMemcpyHostToDevice, b->s));
  if (!dense) {
    HIP_TRY(hipMemcpyAsync(b->dgraph, b->hgraph.data(), b->hgraph.size() * sizeof(BGraph),
                           hipMemcpyHostToDevice, b->s));
    HIP_TRY(hipMemcpyAsync(b->sblk_tab, stab.data(), stab.size() * 4, hipMemcpyHostToDevice, b->s));
  }
  HIP_TRY(hipStreamSynchronize(b->s));
  *out = guard.release();
  return SNMF_OK;
}

snmf_status outer_any(snmf_batch* b, hipStream_t s) {
  return b->prec == SNMF_F64 ? bouter<double>(b, s) : bouter<float>(b, s);
}

snmf_status batch_solve(snmf_batch* b, const void* const* W0, void* const* W_out,
                        void* const* Ht_out, snmf_info* infos, hipStream_t user,
                        double* traces) {
  if (!b) return fail(SNMF_E_ARG, "batch is NULL");
  if (!W0 || !W_out || !Ht_out) return fail(SNMF_E_ARG, "W0, W_out and Ht_out are required");
  for (int g = 0; g < b->nprob; ++g)
    if (!W0[g] || !W_out[g] || !Ht_out[g])
      return fail(SNMF_E_ARG, "W0, W_out and Ht_out need an array per problem");
  if (user) {
    HIP_TRY(hipEventRecord(b->ev_in, user));
    HIP_TRY(hipStreamWaitEvent(b->s, b->ev_in, 0));
  }
  const int S = b->S;
  for (int g = 0; g < b->nprob; ++g) {
    const int64_t cnt = (int64_t)S * b->n[g] * b->r[g];
    if (b->p.validate) {
      double st3[3];
      SNMF_TRY(bstats(b, W0[g], 1, cnt, cnt, st3));
      if (st3[2] > 0) return fail(SNMF_E_NONFINITE, "W0 has NaN/Inf entries");
      if (st3[1] > 0) return fail(SNMF_E_NEGATIVE, "W0 has negative entries");
    }
    const size_t off = (size_t)b->hinst[g * S].off * b->esz;
    HIP_TRY(hipMemcpyAsync((char*)b->Wb + off, W0[g], cnt * b->esz, hipMemcpyDeviceToDevice, b->s));
    HIP_TRY(hipMemcpyAsync((char*)b->Hb + off, W0[g], cnt * b->esz, hipMemcpyDeviceToDevice, b->s));
  }
  launch_breset(b->states, b->dinst, b->ninst, b->s);
  HIP_TRY(hipGetLastError());
  const int every = std::max(1, b->p.check_every);
  if (b->p.use_graph && !b->gexec) {
    HIP_TRY(hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal));
    snmf_status cs = outer_any(b, b->s);
    hipGraph_t gr = nullptr;
    hipError_t ce = hipStreamEndCapture(b->s, &gr);
    if (cs != SNMF_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return cs;
    }
    if (ce != hipSuccess) return fail(SNMF_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
    b->graph = gr;
    HIP_TRY(hipGraphInstantiate(&b->gexec, gr, nullptr, nullptr, 0));
  }
  for (int it = 0; it < b->p.max_outer; ++it) {
    if (b->gexec) {
      HIP_TRY(hipGraphLaunch(b->gexec, b->s));
    } else {
      SNMF_TRY(outer_any(b, b->s));
    }
    if ((it + 1) % every == 0 && it + 1 < b->p.max_outer) {
      launch_all_done(b->states, b->ninst, b->flag, b->s);
      HIP_TRY(hipGetLastError());
      int32_t done = 0;
      HIP_TRY(hipMemcpyAsync(&done, b->flag, sizeof(done), hipMemcpyDeviceToHost, b->s));
      HIP_TRY(hipStreamSynchronize(b->s));
      if (done) break;
    }
  }
  SNMF_TRY(b->prec == SNMF_F64 ? bfinalize<double>(b, b->s) : bfinalize<float>(b, b->s));
  for (int g = 0; g < b->nprob; ++g) {
    const int64_t cnt = (int64_t)S * b->n[g] * b->r[g];
    const size_t off = (size_t)b->hinst[g * S].off * b->esz;
    HIP_TRY(hipMemcpyAsync(W_out[g], (char*)b->Wb + off, cnt * b->esz, hipMemcpyDeviceToDevice, b->s));
    HIP_TRY(hipMemcpyAsync(Ht_out[g], (char*)b->Hb + off, cnt * b->esz, hipMemcpyDeviceToDevice, b->s));
  }
  std::vector<State> hs(b->ninst);
  HIP_TRY(hipMemcpyAsync(hs.data(), b->states, hs.size() * sizeof(State), hipMemcpyDeviceToHost,
                         b->s));
  if (traces)
    HIP_TRY(hipMemcpyAsync(traces, b->traces, (size_t)b->ninst * b->trace_stride * 8,
                           hipMemcpyDeviceToHost, b->s));
  HIP_TRY(hipStreamSynchronize(b->s));
  const double hz = snmf_clock_rate_hz();
  bool broke = false;
  for (int i = 0; i < b->ninst; ++i) {
    const State& h = hs[i];
    broke = broke || h.status != 0;
    if (!infos) continue;
    snmf_info& info = infos[i];
    std::memset(&info, 0, sizeof(info));
    info.status = h.status;
    info.outer = h.outer;
    info.converged_at = h.converged_at;
    info.inner_total = h.inner_total;
    info.ls_evals = h.ls_evals;
    info.ls_exhausted = h.ls_exhausted;
    info.res_WH = h.res_last;
    info.res_WWt = h.resww_last;
    info.sym_gap = h.sym_last;
    info.pg_norm = h.pg_last;
    info.objective = h.f_last;
    info.normA2 = h.normA2;
    info.seconds = (double)(h.t_hstep - h.t0) / hz;
    info.seconds_to_target = h.converged_at > 0 ? (double)h.t_conv / hz : -1.0;
  }
  if (user) {
    HIP_TRY(hipEventRecord(b->ev_out, b->s));
    HIP_TRY(hipStreamWaitEvent(user, b->ev_out, 0));
  }
  // an instance that broke down (e.g. its factor collapsed to zero, rho = 0) is reported
  // in its own record; the batch call itself succeeds
  (void)broke;
  return SNMF_OK;
}

}  // namespace

snmf_status batch_apass_async(snmf_batch* b, const void* P, void* B, hipStream_t s) {
  if (b->prec == SNMF_F64) return bapass<double>(b, (const double*)P, (double*)B, s);
  return bapass<float>(b, (const float*)P, (float*)B, s);
}

extern "C" {

snmf_status snmf_batch_create(int32_t nprob, const snmf_matrix* A, const int32_t* r,
                              const double* lam, int32_t restarts, const snmf_params* p,
                              void* stream, snmf_batch** out) {
  return batch_create(nprob, A, r, lam, restarts, p, (hipStream_t)stream, out);
}

snmf_status snmf_batch_solve(snmf_batch* b, const void* const* W0, void* const* W_out,
                             void* const* Ht_out, snmf_info* infos, void* stream,
                             double* traces) {
  return batch_solve(b, W0, W_out, Ht_out, infos, (hipStream_t)stream, traces);
}

snmf_status snmf_batch_destroy(snmf_batch* b) {
  if (b) {
    (void)hipStreamSynchronize(b->s);
    delete b;
  }
  return SNMF_OK;
}

snmf_status snmf_solve_batched(int32_t nprob, const snmf_matrix* A, const int32_t* r,
                               const double* lam, int32_t restarts, const void* const* W0,
                               const snmf_params* p, void* const* W_out, void* const* Ht_out,
                               snmf_info* infos, void* stream, double* traces) {
  snmf_batch* b = nullptr;
  SNMF_TRY(batch_create(nprob, A, r, lam, restarts, p, (hipStream_t)stream, &b));
  snmf_status s = batch_solve(b, W0, W_out, Ht_out, infos, (hipStream_t)stream, traces);
  std::string keep = err_ref();
  snmf_batch_destroy(b);
  err_ref() = keep;
  return s;
}

snmf_status snmf_batch_apass(snmf_batch* b, const void* P, void* B, void* stream) {
  if (!b || !P || !B) return fail(SNMF_E_ARG, "batch, P and B are required");
  hipStream_t user = (hipStream_t)stream;
  if (user) {
    HIP_TRY(hipEventRecord(b->ev_in, user));
    HIP_TRY(hipStreamWaitEvent(b->s, b->ev_in, 0));
  }
  launch_breset(b->states, b->dinst, b->ninst, b->s);
  if (b->prec == SNMF_F64)
    SNMF_TRY(bapass<double>(b, (const double*)P, (double*)B, b->s));
  else
    SNMF_TRY(bapass<float>(b, (const float*)P, (float*)B, b->s));
  HIP_TRY(hipStreamSynchronize(b->s));
  if (user) {
    HIP_TRY(hipEventRecord(b->ev_out, b->s));
    HIP_TRY(hipStreamWaitEvent(user, b->ev_out, 0));
  }
  return SNMF_OK;
}

snmf_status snmf_batch_time_apass(snmf_batch* b, const void* P, int32_t reps, double* ms) {
  if (!b || !P || !ms) return fail(SNMF_E_ARG, "batch, P and ms are required");
  if (reps < 1) return fail(SNMF_E_ARG, "reps must be >= 1");
  launch_breset(b->states, b->dinst, b->ninst, b->s);
  auto run = [&]() -> snmf_status {
    if (b->prec == SNMF_F64) return bapass<double>(b, (const double*)P, (double*)b->B, b->s);
    return bapass<float>(b, (const float*)P, (float*)b->B, b->s);
  };
  SNMF_TRY(run());
  ScopedEvent e0, e1;
  HIP_TRY(hipEventCreate(&e0.e));
  HIP_TRY(hipEventCreate(&e1.e));
  HIP_TRY(hipEventRecord(e0.e, b->s));
  for (int i = 0; i < reps; ++i) SNMF_TRY(run());
  HIP_TRY(hipEventRecord(e1.e, b->s));
  HIP_TRY(hipEventSynchronize(e1.e));
  float tot = 0.0f;
  HIP_TRY(hipEventElapsedTime(&tot, e0.e, e1.e));
  *ms = (double)tot / reps;
  return SNMF_OK;
}

snmf_status snmf_batch_size(const snmf_batch* b, int32_t* ninst, int64_t* elements) {
  if (!b) return fail(SNMF_E_ARG, "batch is NULL");
  if (ninst) *ninst = b->ninst;
  if (elements) *elements = b->total;
  return SNMF_OK;
}

}  // extern "C"
