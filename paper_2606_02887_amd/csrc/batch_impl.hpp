// Internal layout of a batched solve (struct snmf_batch of include/snmf.h), shared by
// the batch orchestration and the warm-start entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/snmf.h"
#include "common.hpp"
#include "kernels.hpp"

using snmf::BGraph;
using snmf::BInst;
using snmf::BMap;
using snmf::DenseSplit;
using snmf::KParams;
using snmf::State;

struct snmf_batch {
  int nprob = 0, S = 1, ninst = 0, prec = SNMF_F32;
  size_t esz = 4;
  bool dense = false;
  snmf_params p{};
  KParams kp{};
  std::vector<snmf_matrix> A;
  std::vector<int> r;
  std::vector<int64_t> n;
  std::vector<double> normA2;
  std::vector<BInst> hinst;
  std::vector<BGraph> hgraph;
  std::vector<DenseSplit> ds;
  std::vector<int64_t> ldb;                  // BF16X3: row pitch of A_hi, A_lo, Pt (n up to 64)
  std::vector<uint16_t*> Ahi, Alo;           // BF16X3: split A of every problem
  uint16_t *Pthi = nullptr, *Ptlo = nullptr; // BF16X3: stacked split P of one problem
  bool rho_in_apass = false;                 // BF16X3: rho in the product (else split) launch
  struct Cls {
    int r = 0;
    int blocks = 0;        // inner-kernel workgroups
    int64_t tab_off = 0;   // their first entry in blk_tab
    int gblocks = 0;       // Gram workgroups
    int64_t gtab_off = 0;  // their first entry in gblk_tab
  };
  std::vector<Cls> cls;
  int gblocks = 0, sblocks = 0, max_r = 0, part_rows = 0;
  int64_t total = 0, max_nr = 0, gsum = 0, gpsum = 0;
  int ksplit_max = 1;
  int64_t trace_stride = 0;
  hipStream_t s = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  void* pool = nullptr;
  void *Wb = nullptr, *Hb = nullptr, *C = nullptr, *g = nullptr, *Z = nullptr, *D = nullptr;
  void *B = nullptr, *Bpart = nullptr, *GT[2] = {nullptr, nullptr};
  double* G64[2] = {nullptr, nullptr};
  double *gpart = nullptr, *partsA = nullptr, *partsB = nullptr, *partsC = nullptr;
  double *traces = nullptr, *part = nullptr, *dots = nullptr;
  State* states = nullptr;
  int32_t* flag = nullptr;
  unsigned *counters = nullptr, *flags = nullptr;
  BInst* dinst = nullptr;
  int32_t *blk_tab = nullptr, *gblk_tab = nullptr, *sblk_tab = nullptr;
  BGraph* dgraph = nullptr;
  double* wsR = nullptr;       // warm start: FP64 scratch of the frame (allocated on first use)
  int32_t* wsI = nullptr;      // warm start: anchors / permutations, kMaxRank per instance
  double* wsDeg = nullptr;     // warm start of dense problems: row sums of every A_g
  BGraph* wsG = nullptr;       // warm start of dense problems: their table (deg, n)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;

  BMap bmap(const Cls& c) const {
    BMap m{};
    m.blk_inst = blk_tab + c.tab_off;
    m.inst = dinst;
    m.states = states;
    m.traces = traces;
    m.trace_stride = trace_stride;
    return m;
  }

  ~snmf_batch() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (pool) (void)hipFree(pool);
    if (wsR) (void)hipFree(wsR);
    if (wsI) (void)hipFree(wsI);
    if (wsDeg) (void)hipFree(wsDeg);
    if (wsG) (void)hipFree(wsG);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (s) (void)hipStreamDestroy(s);
  }
};


// The batch's A-pass B = A_g P for every instance, stream-ordered on s (no sync).
snmf_status batch_apass_async(snmf_batch* b, const void* P, void* B, hipStream_t s);
