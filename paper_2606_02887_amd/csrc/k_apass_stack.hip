// The split-BF16 A-pass of a batched dense solve, stacked over restarts: B_s = A P_s for
// the S restarts of one problem in one launch.  All S products share their left operand
// (the per-iteration A-pass of Section 4.1, once per restart), so A_hi and A_lo are
// streamed once for the S right operands: at r = 64 and S = 8 the three BF16 products
// (A_hi P_hi + A_hi P_lo + A_lo P_hi, FP32 accumulation, the split of the single solve)
// become bound by the matrix cores instead of HBM.
//
// Operands: A_hi, A_lo (n x ldb BF16, columns n.. zero); Pt_hi, Pt_lo ((S r) x ldb BF16,
// row s r + m holds column m of P_s, columns n.. zero; k_split_pt_stack writes them).
// The S r stacked columns are cut into blocks of kStackCols (128).  A workgroup (4 waves x
// 32 output rows) computes 128 rows x one column block over one K slice; with one slice it writes
// B directly, else split-K partials that k_sum_parts adds in slice order.  The spectral
// norms rho_s of the restarts' Grams can run in the same launch.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "rho.hpp"

namespace snmf {

// Stacked columns per workgroup, in units of 32: 4 gives 128-column blocks, so each row
// tile's A is requested by half as many workgroups as with 64 (the product is bound by
// those requests through L2); the LDS of such a workgroup leaves one per CU.
constexpr int kStackNNB = 4;
constexpr int kStackCols = 32 * kStackNNB;
constexpr int kStackPerCU = kStackNNB == 2 ? 2 : 1;
int stack_per_cu() { return kStackPerCU; }

typedef float f32x4s __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

namespace {

__device__ __forceinline__ bool stack_done(const State* st, int S) {
  for (int i = 0; i < S; ++i)
    if (!st[i].done) return false;
  return true;
}

// Workgroup id -> (unit, column block), unit = K slice * gx + row tile.  Workgroups go to
// the 8 XCDs in turn (id mod 8).  The G column blocks of one unit get ids of one residue
// mod 8 that are dispatched one after another on that XCD, so they read the same rows of
// A at about the same time through that XCD's L2.  Ids past the last whole group of 8 G
// map in order.
struct StackMap {
  int64_t unit;
  int cb;
};
__device__ __forceinline__ StackMap stack_map(int64_t id, int64_t nwg, int G) {
  const int64_t grp = 8 * (int64_t)G;
  const int64_t full = nwg / grp * grp;
  StackMap m;
  if (id < full) {
    const int64_t x = id & 7, j = id >> 3;
    const int64_t jg = j / G;
    m.unit = jg * 8 + x;
    m.cb = (int)(j - jg * G);
  } else {
    m.unit = id / G;
    m.cb = (int)(id - m.unit * G);
  }
  return m;
}

}  // namespace

template <int V>
using IC = std::integral_constant<int, V>;

// A wave computes 32 rows x 64 columns as 2 x 4 blocks of v_mfma_f32_16x16x32_bf16: a
// lane (l mod 16, l / 16) holds 8 consecutive k of row l mod 16 (A) or of stacked column
// l mod 16 (Pt), so the four lanes of a row read 64 contiguous bytes and one A load
// instruction touches 16 rows (the 32x32x16 shape touched 32 rows with 32 bytes each, and
// the vector cache's per-line work, not the bytes, set the pace).  Per 64-column slab a
// lane loads two 16-byte vectors of each of its two rows from A_hi and A_lo; the slab of
// the block's 64 rows of Pt_hi / Pt_lo is staged in LDS (two buffers) and shared by the
// four waves.  Loads run two slabs ahead: one slab's MFMAs (24 per wave) are shorter than
// a memory round trip, so with one slab ahead every slab waited on its loads.  The A
// vectors go to a ring of three register sets and the Pt vectors to a ring of two; the
// loop is unrolled six slabs deep so every ring index is static.  Past the last slab the
// prefetch re-reads the last slab (in bounds, unused).
//
// Workgroups past the first ntile (one per restart, launched when Grho is set) compute
// rho = ||G_s||_2 of restart s (r x r FP64 Grams r^2 apart) beside the products.
__global__ __launch_bounds__(256, kStackPerCU) void k_apass_bf16x3s(
    const uint16_t* __restrict__ Ahi, const uint16_t* __restrict__ Alo, int64_t ldb,
    const uint16_t* __restrict__ Pthi, const uint16_t* __restrict__ Ptlo, int64_t n, int r,
    int S, int64_t gx, int ncb, int64_t kchunk, int64_t ntile, float* __restrict__ Bout,
    int64_t pstride, State* __restrict__ st, const double* __restrict__ Grho) {
  if ((int64_t)blockIdx.x >= ntile) {
    const int s = (int)((int64_t)blockIdx.x - ntile);
    if (!st[s].done) rho_body(Grho + (int64_t)s * r * r, r, st + s);
    return;
  }
  if (stack_done(st, S)) return;
  constexpr int NNB = kStackNNB;            // the workgroup's stacked columns, in units of 32
  constexpr int CB = 2 * NNB;               // its 16-column blocks
  constexpr int KS = 64;                    // k per slab
  constexpr int PROW = KS + 8;              // LDS row pitch (bf16), keeps 16-byte alignment
  __shared__ __attribute__((aligned(16))) uint16_t sP[2][2][32 * NNB * PROW];  // [buf][hi/lo]
  // running sums of the MFMA accumulators, flushed every six slabs: the matrix cores'
  // FP32 accumulation drifts low by a small fraction of an ulp per instruction (measured
  // mean relative error -1.65e-7 over one chain of 8192 k), so short chains whose sums
  // are added with ordinary FP32 adds keep the product unbiased; [rb * 4 + cb][thread]
  __shared__ f32x4s sAcc[2 * CB][256];
  const StackMap sm = stack_map((int64_t)blockIdx.x, ntile, ncb);
  const int64_t tile = sm.unit % gx, ksl = sm.unit / gx;
  const int64_t R = (int64_t)S * r;
  const int64_t mb = (int64_t)sm.cb * (32 * NNB);  // first stacked column of the block
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ri = lane & 15, g = lane >> 4;
  const int64_t j0 = (tile * 4 + wave) * 32;
  const int64_t kb = ksl * kchunk;
  int64_t ke = kb + kchunk;
  if (ke > ldb) ke = ldb;
  const int64_t nk = (ke - kb) / KS;        // slabs, >= 1
  const int64_t klast = kb + (nk - 1) * KS;
  f32x4s acc[2][CB];                        // [row block][16-column block]
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      acc[rb][cb] = f32x4s{0.0f, 0.0f, 0.0f, 0.0f};
      sAcc[rb * CB + cb][tid] = f32x4s{0.0f, 0.0f, 0.0f, 0.0f};
    }
  // each thread adds its own accumulators into its own LDS slots: no barrier needed
  auto flush = [&]() {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        sAcc[rb * CB + cb][tid] += acc[rb][cb];
        acc[rb][cb] = f32x4s{0.0f, 0.0f, 0.0f, 0.0f};
      }
  };
  // Rows past n and stacked columns past S r read the last valid row of A or Pt instead:
  // they feed only output rows and columns that are never stored, and loads without a
  // condition keep the loop free of branches (the compiler counts loads in flight
  // exactly only in straight-line code; behind a branch it waited for all of them,
  // the prefetch included, before every LDS stage).
  const int64_t ja = j0 + ri < n ? j0 + ri : n - 1;
  const int64_t jb = j0 + 16 + ri < n ? j0 + 16 + ri : n - 1;
  const uint16_t* ah0 = Ahi + ja * ldb + 8 * g;
  const uint16_t* al0 = Alo + ja * ldb + 8 * g;
  const uint16_t* ah1 = Ahi + jb * ldb + 8 * g;
  const uint16_t* al1 = Alo + jb * ldb + 8 * g;
  // Pt staging: 2 (hi, lo) x 64 rows x 64 bf16 = 1024 16-byte vectors, 4 per thread
  constexpr int VPR = KS / 8;               // vectors per row
  constexpr int NVEC = 2 * 32 * NNB * VPR;
  constexpr int NPT = NVEC / 256;
  u16x8 xr[3][2][4];                        // A ring: [slot][hi/lo][row block x k half]
  u16x8 pr[2][NPT];                         // Pt ring
  auto stage_load = [&](u16x8 (&p)[NPT], int64_t k) {
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int e = tid + 256 * q;
      const int which = e / (32 * NNB * VPR);
      const int rem = e - which * (32 * NNB * VPR);
      const int m = rem / VPR, qq = rem - m * VPR;
      const int64_t M = mb + m < R ? mb + m : R - 1;
      p[q] = *(const u16x8*)((which ? Ptlo : Pthi) + M * ldb + k + 8 * qq);
    }
  };
  auto stage_store = [&](const u16x8 (&p)[NPT], int b) {
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int e = tid + 256 * q;
      const int which = e / (32 * NNB * VPR);
      const int rem = e - which * (32 * NNB * VPR);
      const int m = rem / VPR, qq = rem - m * VPR;
      *(u16x8*)&sP[b][which][m * PROW + 8 * qq] = p[q];
    }
  };
  auto load_a = [&](u16x8 (&x)[2][4], int64_t k) {
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      x[0][kh] = *(const u16x8*)(ah0 + k + 32 * kh);
      x[0][2 + kh] = *(const u16x8*)(ah1 + k + 32 * kh);
      x[1][kh] = *(const u16x8*)(al0 + k + 32 * kh);
      x[1][2 + kh] = *(const u16x8*)(al1 + k + 32 * kh);
    }
  };
  auto mma = [&](const u16x8 (&x)[2][4], int b) {
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int m = 16 * cb + ri;
        const u16x8 bh = *(const u16x8*)&sP[b][0][m * PROW + 32 * kh + 8 * g];
        const u16x8 bl = *(const u16x8*)&sP[b][1][m * PROW + 32 * kh + 8 * g];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          const bf16x8 xh = __builtin_bit_cast(bf16x8, x[0][2 * rb + kh]);
          const bf16x8 xl = __builtin_bit_cast(bf16x8, x[1][2 * rb + kh]);
          f32x4s d = acc[rb][cb];
          d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, __builtin_bit_cast(bf16x8, bh), d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, __builtin_bit_cast(bf16x8, bl), d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, __builtin_bit_cast(bf16x8, bh), d, 0, 0, 0);
          acc[rb][cb] = d;
        }
      }
    }
  };
  // slab i (ring phase I = i mod 6): prefetch slab i + 2 into the ring slots that held
  // slab i's Pt (already in LDS) and slab i - 1's A (consumed), multiply slab i, stage
  // slab i + 1's Pt (loaded one step earlier) into the other LDS buffer
  auto step = [&](auto I, int64_t i) {
    constexpr int ia = decltype(I)::value % 3, ip = decltype(I)::value % 2;
    const int64_t kn = i + 2 < nk ? kb + (i + 2) * KS : klast;
    stage_load(pr[ip], kn);
    load_a(xr[(ia + 2) % 3], kn);
    mma(xr[ia], ip);
    stage_store(pr[ip ^ 1], ip ^ 1);
    __syncthreads();
  };
  stage_load(pr[0], kb);
  load_a(xr[0], kb);
  const int64_t k1 = nk > 1 ? kb + KS : klast;
  stage_load(pr[1], k1);
  load_a(xr[1], k1);
  stage_store(pr[0], 0);
  __syncthreads();
  int64_t i = 0;
  for (; i + 6 <= nk; i += 6) {
    step(IC<0>{}, i);
    step(IC<1>{}, i + 1);
    step(IC<2>{}, i + 2);
    step(IC<3>{}, i + 3);
    step(IC<4>{}, i + 4);
    step(IC<5>{}, i + 5);
    flush();
  }
  if (i < nk) step(IC<0>{}, i);
  if (i + 1 < nk) step(IC<1>{}, i + 1);
  if (i + 2 < nk) step(IC<2>{}, i + 2);
  if (i + 3 < nk) step(IC<3>{}, i + 3);
  if (i + 4 < nk) step(IC<4>{}, i + 4);
  flush();
  // D of block (rb, cb): row 4 (l / 16) + v (output row j0 + 16 rb + row), column l mod 16
  // (stacked column mb + 16 cb + column).  Stacked column M is column M mod r of restart
  // M / r, whose n x r block starts at (M / r) n r.
  float* out = Bout + ksl * pstride;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int64_t M = mb + 16 * cb + ri;
    if (M < R) {
      const int64_t s = M / r, m = M - s * r;
      float* o = out + s * n * r + m;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t jj = j0 + 16 * rb + 4 * g + v;
          if (jj < n) o[jj * r] = sAcc[rb * CB + cb][tid][v];
        }
    }
  }
}

// ----------------------------------------------------------------------------- launchers
static int64_t stack_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return cus;
}

// kStackPerCU workgroups per CU: the (row tile, column block) pairs, times K slices of whole
// 64-column slabs while there are fewer pairs than that (at most kMaxKSplit slices).
// n = 8192, S r = 512: 64 x 4 pairs, one slice.
DenseSplit plan_dense_bf16_stack(int64_t n, int64_t R) {
  DenseSplit d;
  const int64_t ldb = (n + 63) / 64 * 64;
  d.gx = (n + 127) / 128;
  const int64_t ncb = (R + kStackCols - 1) / kStackCols;
  const int64_t pairs = d.gx * ncb;
  int64_t ks = (kStackPerCU * stack_cus() + pairs - 1) / pairs;
  const int64_t kmax = ldb / 64;
  if (ks > kmax) ks = kmax;
  if (ks > kMaxKSplit) ks = kMaxKSplit;
  if (ks < 1) ks = 1;
  int64_t kc = (ldb + ks - 1) / ks;
  kc = (kc + 63) / 64 * 64;
  d.kchunk = kc;
  d.ksplit = (int)((ldb + kc - 1) / kc);
  d.nwg = pairs * d.ksplit;
  return d;
}

void launch_apass_bf16x3_stack(const uint16_t* Ahi, const uint16_t* Alo, int64_t ldb,
                               const uint16_t* Pthi, const uint16_t* Ptlo, int64_t n, int r,
                               int S, const DenseSplit& d, float* Bout, int64_t pstride,
                               State* st, const double* Grho, hipStream_t s) {
  const int ncb = (int)(((int64_t)S * r + kStackCols - 1) / kStackCols);
  const int64_t nrho = Grho ? S : 0;
  hipLaunchKernelGGL(k_apass_bf16x3s, dim3((unsigned)(d.nwg + nrho)), dim3(256), 0, s, Ahi, Alo,
                     ldb, Pthi, Ptlo, n, r, S, d.gx, ncb, d.kchunk, d.nwg, Bout, pstride, st,
                     Grho);
}

}  // namespace snmf
