// Sparse and low-rank products of the SNMPBB hot path.
//
// * CSR SpMM  Y = A X  (A symmetric, both triangles stored).  One wavefront per row:
//   lane (slot, c) = (lane / r, lane % r), slot < 64 / r, walks the nonzeros slot,
//   slot + 64 / r, ... of the row and accumulates A_ik X[k][c]; slot 0 adds the other
//   slots' sums in slot order.  (RP, the rank padded to a power of two, only selects the
//   instantiation.)  Used for
//   the A-pass of Graph-SNMPBB and of batched graph problems, and for the Laplacian
//   products L X, L(Z-X), L S of eq. (2.3).  In "dot" mode the kernel writes FP64 partial
//   sums of <X2, A X> per workgroup (the curvature <D, L D>, reduced by the next kernel)
//   instead of storing A X.
// * LAI-SNMPBB (Section 2.3): A P ~= U (lam .* (U^T P)).  T = U^T P is an ell x r
//   reduction over all n rows (FP64 partials per workgroup, then a fixed-order sum that
//   also applies lam); B = U T is a row-local product.
#include "common.hpp"
#include "kernels.hpp"
#include "rho.hpp"

namespace snmf {

// Stands in for an absent gate, so that both gate flags load without a condition (a load
// under a null test waited for its pointer argument and its flag in turn).
__device__ int32_t g_no_gate = 0;

template <typename T, int RP, bool RHO>
__global__ __launch_bounds__(256) void k_spmm(const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col,
                                              const T* __restrict__ val, const T* __restrict__ X,
                                              int64_t n, int r, T* __restrict__ Y,
                                              const T* __restrict__ X2, double* __restrict__ part,
                                              const int32_t* __restrict__ gate,
                                              const int32_t* __restrict__ gate2, RhoJob rj) {
  // gate, gate2: the product is skipped when either flag is set (nullptr: none)
  const int32_t* __restrict__ g1 = gate ? gate : &g_no_gate;
  const int32_t* __restrict__ g2 = gate2 ? gate2 : g1;
  // RHO: workgroup 0 computes rho = ||G||_2 (dispatched first, so it runs beside the
  // product) and the product uses the workgroups after it.  A template flag, so the plain
  // product keeps its lower register count.
  constexpr int64_t b0 = RHO ? 1 : 0;
  if constexpr (RHO) {
    if (blockIdx.x == 0) {
      if (g1[0] | g2[0]) return;
      rho_body(rj.G, rj.r, rj.st);
      return;
    }
  }
  // nonzero slots per wave: lanes s r .. s r + r - 1 serve slot s (at r = 20 three slots,
  // 60 lanes busy, where slots of the padded width RP = 32 would give two)
  const int ns = kWave / r;
  // gathers in flight per lane (each lane's nonzeros are added in the same order for any
  // SU, so the sums do not depend on it).  Measured at the graph workload (A-pass, n =
  // 20000, r = 20) and on a random graph of 6e7 nonzeros (n = 2e6, r = 20), with slots of
  // the padded width: SU = 2 13.8 us / 1.94 ms, 4 12.5 us / 1.59 ms, 8 17.7 us / 2.41 ms
  // (its registers cost resident waves).
  constexpr int SU = 4;
  __shared__ double sred[kThreads / kWave * kNumPart];
  const int lane = threadIdx.x & 63;
  const int slot = lane / r, c = lane - slot * r;
  const bool act = slot < ns;
  const int64_t bid = (int64_t)blockIdx.x - b0;
  const int64_t wave_id = (bid * kThreads + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x - b0) * kThreads / kWave;
  // the first row's extent is loaded before the gates are tested: both round trips overlap
  const int64_t b_first = wave_id < n ? rowptr[wave_id] : 0;
  const int64_t e_first = wave_id < n ? rowptr[wave_id + 1] : 0;
  if (g1[0] | g2[0]) return;
  double dot = 0.0;
  for (int64_t row = wave_id; row < n; row += nwaves) {
    const int64_t b = row == wave_id ? b_first : rowptr[row];
    const int64_t e = row == wave_id ? e_first : rowptr[row + 1];
    T acc = T(0);
    // up to 64 (column, value) pairs per load, broadcast by cross-lane shuffles so that
    // the gathers of four nonzeros per lane group are in flight together
    for (int64_t zb = b; zb < e; zb += kWave) {
      const int cnt = e - zb < kWave ? (int)(e - zb) : kWave;
      const int mc = lane < cnt ? col[zb + lane] : 0;
      const T mv = lane < cnt ? val[zb + lane] : T(0);
      for (int k0 = 0; k0 < cnt; k0 += SU * ns) {  // uniform trip count: all lanes shuffle
        int ck[SU];
        T vk[SU], pk[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          const int k = k0 + slot + u * ns;
          const int src = k < kWave ? k : kWave - 1;
          ck[u] = __shfl(mc, src, kWave);
          vk[u] = __shfl(mv, src, kWave);
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          const int k = k0 + slot + u * ns;
          pk[u] = (act && k < cnt) ? X[(int64_t)ck[u] * r + c] : T(0);
        }
#pragma unroll
        for (int u = 0; u < SU; ++u)
          if (act && k0 + slot + u * ns < cnt) acc += vk[u] * pk[u];
      }
    }
    // slot 0 adds the other slots' sums in slot order
    T tot = acc;
    for (int q = 1; q < ns; ++q) {
      const int src = lane + q * r;
      const T o = __shfl(acc, src < kWave ? src : kWave - 1, kWave);
      tot += o;
    }
    acc = tot;
    if (slot == 0) {
      if (X2)
        dot += (double)X2[row * r + c] * (double)acc;
      else
        Y[row * r + c] = acc;
    }
  }
  if (!X2) return;
  double v[1] = {dot};
  block_sum<1>(v, sred);
  if (threadIdx.x == 0) part[(size_t)bid * kNumPart] = v[0];
}

// ----------------------------------------------------------------------------- batched
// Stacked A-pass of a batched solve: B_s = A P_s for all S restarts of a problem in one
// sweep over its CSR (the restarts form one n x (S r) operand).  One wavefront per row;
// lane c of a chunk of cw columns (cw = 64, or the smallest power of two >= S r) serves
// stacked column c0 + c = s r + j, and the 64 / cw lane groups split the row's nonzeros.
// The wave loads up to 64 (column, value) pairs of the row at once and broadcasts them
// with cross-lane shuffles, so the gathers of four nonzeros are in flight together.
template <typename T>
__global__ __launch_bounds__(256) void k_bspmm(const BGraph* __restrict__ graphs,
                                               const int32_t* __restrict__ sblk_graph,
                                               const State* __restrict__ states,
                                               const T* __restrict__ P, T* __restrict__ B) {
  const BGraph* G = graphs + sblk_graph[blockIdx.x];
  const int r = G->r, S = G->S;
  bool all_done = true;
  for (int s = 0; s < S; ++s) all_done = all_done && states[G->inst0 + s].done;
  if (all_done) return;
  const int64_t n = G->n;
  const int width = r * S;
  int cw = 64;
  while (cw > 1 && cw / 2 >= width) cw >>= 1;
  const int ns = kWave / cw;
  const int lane = threadIdx.x & 63;
  const int c = lane % cw, slot = lane / cw;
  const int64_t wave = ((int64_t)blockIdx.x - G->blk0) * (kThreads / kWave) + threadIdx.x / kWave;
  const int64_t nw = (int64_t)G->nblk * (kThreads / kWave);
  // the CSR arrays come from the graph table, so the compiler cannot see that they are
  // global memory: without the address space it would emit flat loads, which also count
  // against the LDS wait counter
  typedef const __attribute__((address_space(1))) int64_t* GI64;
  typedef const __attribute__((address_space(1))) int32_t* GI32;
  typedef const __attribute__((address_space(1))) T* GT_;
  const GI64 __restrict__ rowptr = (GI64)G->rowptr;
  const GI32 __restrict__ col = (GI32)G->col;
  const GT_ __restrict__ val = (GT_)G->val;
  const int64_t nr = n * r;
  const T* __restrict__ Pg = P + G->off0;
  T* __restrict__ Bg = B + G->off0;
  for (int64_t row = wave; row < n; row += nw) {
    const int64_t b = rowptr[row], e = rowptr[row + 1];
    for (int c0 = 0; c0 < width; c0 += cw) {
      const int cc = c0 + c;
      const bool cok = cc < width;
      const int s = cok ? cc / r : 0;
      const int j = cc - s * r;
      const T* __restrict__ Ps = Pg + s * nr + j;
      T acc = T(0);
      for (int64_t zb = b; zb < e; zb += kWave) {
        const int cnt = e - zb < kWave ? (int)(e - zb) : kWave;
        const int mc = lane < cnt ? col[zb + lane] : 0;
        const T mv = lane < cnt ? val[zb + lane] : T(0);
        for (int k0 = 0; k0 < cnt; k0 += 4 * ns) {  // uniform trip count: all lanes shuffle
          int ck[4];
          T vk[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int k = k0 + slot + u * ns;
            const int src = k < kWave ? k : kWave - 1;
            ck[u] = __shfl(mc, src, kWave);
            vk[u] = __shfl(mv, src, kWave);
          }
          T pk[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int k = k0 + slot + u * ns;
            pk[u] = (cok && k < cnt) ? Ps[(int64_t)ck[u] * r] : T(0);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int k = k0 + slot + u * ns;
            if (k < cnt) acc += vk[u] * pk[u];
          }
        }
      }
      for (int o = cw; o < kWave; o <<= 1) acc += __shfl_xor(acc, o, kWave);
      if (slot == 0 && cok) Bg[s * nr + row * r + j] = acc;
    }
  }
}

template <typename T>
void launch_bspmm(const BGraph* graphs, const int32_t* sblk_graph, int sblocks,
                  const State* states, const T* P, T* B, hipStream_t s) {
  hipLaunchKernelGGL(k_bspmm<T>, dim3(sblocks), dim3(256), 0, s, graphs, sblk_graph, states, P, B);
}
template void launch_bspmm<float>(const BGraph*, const int32_t*, int, const State*, const float*,
                                  float*, hipStream_t);
template void launch_bspmm<double>(const BGraph*, const int32_t*, int, const State*,
                                   const double*, double*, hipStream_t);

// ----------------------------------------------------------------------------- LAI
// Partial T_b = U_b^T P_b over a slab of rows, FP64.  ell <= 128, r <= 64.
template <typename T>
__global__ __launch_bounds__(256) void k_lai_utp(const T* __restrict__ U, int ell,
                                                 const T* __restrict__ P, int64_t n, int r,
                                                 int64_t rows_per_block, double* __restrict__ part,
                                                 const int32_t* __restrict__ gate) {
  if (gate && gate[0]) return;
  constexpr int TR = 16;
  __shared__ double sU[TR][kMaxEll];
  __shared__ double sP[TR][kMaxRank];
  const int ne = ell * r;
  constexpr int NE = kMaxEll * kMaxRank / 256;
  double acc[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) acc[q] = 0.0;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = rb + rows_per_block < n ? rb + rows_per_block : n;
  for (int64_t t0 = rb; t0 < re; t0 += TR) {
    __syncthreads();
    for (int e = threadIdx.x; e < TR * ell; e += 256) {
      const int i = e / ell, a = e - i * ell;
      sU[i][a] = t0 + i < re ? (double)U[(t0 + i) * ell + a] : 0.0;
    }
    for (int e = threadIdx.x; e < TR * r; e += 256) {
      const int i = e / r, cc = e - i * r;
      sP[i][cc] = t0 + i < re ? (double)P[(t0 + i) * r + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = threadIdx.x + q * 256;
      if (e < ne) {
        const int a = e / r, cc = e - a * r;
        double s = acc[q];
#pragma unroll
        for (int i = 0; i < TR; ++i) s = __builtin_fma(sU[i][a], sP[i][cc], s);
        acc[q] = s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = threadIdx.x + q * 256;
    if (e < ne) part[(size_t)blockIdx.x * ne + e] = acc[q];
  }
}

// TT[a][c] = lam[a] * sum_b part[b][a][c], fixed block order.
template <typename T>
__global__ __launch_bounds__(256) void k_lai_reduce(const double* __restrict__ part, int nb, int ell,
                                                    int r, const double* __restrict__ lam,
                                                    T* __restrict__ TT,
                                                    const int32_t* __restrict__ gate) {
  if (gate && gate[0]) return;
  const int ne = ell * r;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= ne) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * ne + e];
  TT[e] = (T)(lam[e / r] * s);
}

// B[i][c] = sum_a U[i][a] TT[a][c]; TT and a 32-row slab of U staged in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_lai_ut(const T* __restrict__ U, int ell,
                                                const T* __restrict__ TT, int64_t n, int r,
                                                T* __restrict__ B, const int32_t* __restrict__ gate) {
  if (gate && gate[0]) return;
  constexpr int TR = 32;
  __shared__ T sT[kMaxEll * kMaxRank];
  __shared__ T sU[TR][kMaxEll + 1];
  for (int e = threadIdx.x; e < ell * r; e += 256) sT[e] = TT[e];
  const int64_t ntiles = (n + TR - 1) / TR;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * TR;
    __syncthreads();
    for (int e = threadIdx.x; e < TR * ell; e += 256) {
      const int i = e / ell, a = e - i * ell;
      sU[i][a] = row0 + i < n ? U[(row0 + i) * ell + a] : T(0);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TR * r; e += 256) {
      const int i = e / r, cc = e - i * r;
      const int64_t row = row0 + i;
      if (row < n) {
        T acc = T(0);
        for (int a = 0; a < ell; ++a) acc += sU[i][a] * sT[a * r + cc];
        B[row * r + cc] = acc;
      }
    }
  }
}

// ----------------------------------------------------------------------------- LAI, FP32
// The FP32 products on MFMA v_mfma_f32_16x16x4f32 with slabs of 64 rows staged in LDS by
// coalesced 16-byte loads (a slab of U or P is one contiguous block of memory).
// Lane l of an MFMA supplies A[l%16][l/16] and B[l/16][l%16] and receives
// D[4(l/16)+v][l%16], v = 0..3.
typedef float f32x4l __attribute__((ext_vector_type(4)));
constexpr int kLaiRows = 64;                    // rows per LDS slab
constexpr int kLaiMaxTiles = 8;                 // 16x16 output tiles per wave
// Grids measured at n = 200000, ell = 64, r = 32 (A-pass time): B = U T with 1024
// workgroups 63 us, 4096 76 us; T = U^T P with 256 partials beat 512.
constexpr int kLaiUtGrid = 1024;   // workgroups of B = U T (pipelined slabs)
constexpr int kLaiUtpGrid = 256;   // workgroups (partials) of T = U^T P
// LDS pitches (dynamic shared memory sized to ell and r): a k-major read (16 consecutive
// columns of 4 rows) is conflict-free with pitch == 16 mod 64, a row-major read (4
// consecutive columns of 16 rows) with pitch == 4 mod 64.
__host__ __device__ inline int lai_pitch_k(int w) { return (w + 63) / 64 * 64 + 16; }
__host__ __device__ inline int lai_pitch_r(int w) { return (w + 63) / 64 * 64 + 4; }

// Stage rows [row0, row0 + 64) of an n x w row-major array into LDS (pitch `pitch`),
// zero beyond n and w; float4 loads when w % 4 == 0.
__device__ __forceinline__ void lai_stage(const float* __restrict__ X, int64_t n, int w,
                                          int64_t row0, float* __restrict__ sX, int pitch) {
  const int64_t rows = n - row0 < kLaiRows ? n - row0 : kLaiRows;
  if ((w & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0) {
    const int w4 = w >> 2;
    const float4* src = reinterpret_cast<const float4*>(X + row0 * w);
    for (int e = threadIdx.x; e < kLaiRows * w4; e += 256) {
      const int i = e / w4, c = (e - i * w4) * 4;
      const float4 v = i < rows ? src[e] : make_float4(0.f, 0.f, 0.f, 0.f);
      *reinterpret_cast<float4*>(&sX[i * pitch + c]) = v;
    }
  } else {
    for (int e = threadIdx.x; e < kLaiRows * w; e += 256) {
      const int i = e / w, c = e - i * w;
      sX[i * pitch + c] = i < rows ? X[(row0 + i) * w + c] : 0.f;
    }
  }
}

// Register-staged slab copy for the pipelined loop: up to NV float4 per thread of the
// 64 x w slab starting at row0 (w % 4 == 0, 16-byte aligned rows); rows >= n read as 0.
template <int NV>
struct SlabRegs {
  float4 v[NV];
  __device__ __forceinline__ void load(const float* __restrict__ X, int64_t n, int w, int64_t row0) {
    const int w4 = w >> 2;
    const int64_t rows = n - row0 < kLaiRows ? n - row0 : kLaiRows;
    const float4* src = reinterpret_cast<const float4*>(X + row0 * w);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = threadIdx.x + q * 256;
      const int i = e / w4;
      v[q] = (e < kLaiRows * w4 && i < rows) ? src[e] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  __device__ __forceinline__ void store(float* __restrict__ sX, int w, int pitch) const {
    const int w4 = w >> 2;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = threadIdx.x + q * 256;
      if (e < kLaiRows * w4) {
        const int i = e / w4, c = (e - i * w4) * 4;
        *reinterpret_cast<float4*>(&sX[i * pitch + c]) = v[q];
      }
    }
  }
};

// Partial T_b = U_b^T P_b over a contiguous slab of rows; FP32 partial (ell x r) per
// workgroup.  Output tiles (ell/16) x (r/16), tile t handled by wave t % 4.
__global__ __launch_bounds__(256) void k_lai_utp32(const float* __restrict__ U, int ell,
                                                   const float* __restrict__ P, int64_t n, int r,
                                                   int64_t rows_per_block,
                                                   float* __restrict__ part,
                                                   const int32_t* __restrict__ gate,
                                                   RhoJob rj) {
  if (gate && gate[0]) return;
  // with rj.G set, the last workgroup computes rho = ||G||_2 beside the slabs
  if (rj.G && blockIdx.x == gridDim.x - 1) {
    rho_body(rj.G, rj.r, rj.st);
    return;
  }
  extern __shared__ __attribute__((aligned(16))) float lai_smem[];
  const int PA = lai_pitch_k(ell), PP = lai_pitch_k(r);
  float* sU = lai_smem;
  float* sP = lai_smem + kLaiRows * PA;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int TL = (ell + 15) / 16, TRr = (r + 15) / 16, nt = TL * TRr;
  f32x4l acc[kLaiMaxTiles];
#pragma unroll
  for (int q = 0; q < kLaiMaxTiles; ++q) acc[q] = f32x4l{0.f, 0.f, 0.f, 0.f};
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = rb + rows_per_block < n ? rb + rows_per_block : n;
  // pipelined when both slabs take 16-byte loads: the next slab is in flight in registers
  // while the MFMAs run on the current one
  const bool vec = (ell & 3) == 0 && (r & 3) == 0 &&
                   ((reinterpret_cast<uintptr_t>(U) | reinterpret_cast<uintptr_t>(P)) & 15) == 0;
  SlabRegs<kLaiRows * kMaxEll / 4 / 256> ru;
  SlabRegs<kLaiRows * kMaxRank / 4 / 256> rp;
  if (vec && rb < re) {
    ru.load(U, re, ell, rb);
    rp.load(P, re, r, rb);
  }
  for (int64_t t0 = rb; t0 < re; t0 += kLaiRows) {
    __syncthreads();
    if (vec) {
      ru.store(sU, ell, PA);
      rp.store(sP, r, PP);
    } else {
      lai_stage(U, re, ell, t0, sU, PA);
      lai_stage(P, re, r, t0, sP, PP);
    }
    __syncthreads();
    if (vec && t0 + kLaiRows < re) {
      ru.load(U, re, ell, t0 + kLaiRows);
      rp.load(P, re, r, t0 + kLaiRows);
    }
#pragma unroll
    for (int q = 0; q < kLaiMaxTiles; ++q) {
      const int t = w + 4 * q;
      if (t < nt) {
        const int i0 = 16 * (t / TRr), j0 = 16 * (t % TRr);
        f32x4l d = acc[q];
        for (int k0 = 0; k0 < kLaiRows; k0 += 4) {
          const int k = k0 + (lane >> 4);
          const float a = sU[k * PA + i0 + (lane & 15)];
          const float b = sP[k * PP + j0 + (lane & 15)];
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d, 0, 0, 0);
        }
        acc[q] = d;
      }
    }
  }
  float* out = part + (size_t)blockIdx.x * ell * r;
#pragma unroll
  for (int q = 0; q < kLaiMaxTiles; ++q) {
    const int t = w + 4 * q;
    if (t < nt) {
      const int i0 = 16 * (t / TRr), j0 = 16 * (t % TRr);
      const int j = j0 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 4 * (lane >> 4) + v;
        if (i < ell && j < r) out[i * r + j] = acc[q][v];
      }
    }
  }
}

// TT[a][c] = lam[a] * sum_b part[b][a][c] in FP64, blocks in order: four threads per
// entry take every fourth block, their sums are added in thread order.
__global__ __launch_bounds__(256) void k_lai_reduce32(const float* __restrict__ part, int nb,
                                                      int ell, int r,
                                                      const double* __restrict__ lam,
                                                      float* __restrict__ TT,
                                                      const int32_t* __restrict__ gate) {
  if (gate && gate[0]) return;
  __shared__ double sq[4][64];
  const int ne = ell * r;
  const int e = blockIdx.x * 64 + (threadIdx.x & 63), q = threadIdx.x >> 6;
  double s = 0.0;
  if (e < ne) {
    int b = q;
    // sixteen of this thread's blocks per round trip, added in block order
    for (; b + 60 < nb; b += 64) {
      float v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = part[(size_t)(b + 4 * u) * ne + e];
#pragma unroll
      for (int u = 0; u < 16; ++u) s += v[u];
    }
    for (; b + 12 < nb; b += 16) {
      const float v0 = part[(size_t)b * ne + e], v1 = part[(size_t)(b + 4) * ne + e];
      const float v2 = part[(size_t)(b + 8) * ne + e], v3 = part[(size_t)(b + 12) * ne + e];
      s += v0;
      s += v1;
      s += v2;
      s += v3;
    }
    for (; b < nb; b += 4) s += part[(size_t)b * ne + e];
  }
  sq[q][threadIdx.x & 63] = s;
  __syncthreads();
  if (q == 0 && e < ne) {
    const double t = ((sq[0][threadIdx.x] + sq[1][threadIdx.x]) + sq[2][threadIdx.x]) + sq[3][threadIdx.x];
    TT[e] = (float)(lam[e / r] * t);
  }
}

// B = U TT, 64-row slabs: output tiles 4 x (r/16), tile t handled by wave t % 4; TT
// (ell x r) staged once per workgroup.
__global__ __launch_bounds__(256) void k_lai_ut32(const float* __restrict__ U, int ell,
                                                  const float* __restrict__ TT, int64_t n, int r,
                                                  float* __restrict__ B,
                                                  const int32_t* __restrict__ gate) {
  if (gate && gate[0]) return;
  extern __shared__ __attribute__((aligned(16))) float lai_smem[];
  const int PA = lai_pitch_r(ell), PT = lai_pitch_k(r);
  const int ellp = (ell + 3) & ~3;  // K padded to the MFMA step (zeros beyond ell)
  float* sU = lai_smem;
  float* sT = lai_smem + kLaiRows * PA;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < ellp * PT; e += 256) {
    const int k = e / PT, c = e - k * PT;
    sT[e] = (k < ell && c < r) ? TT[k * r + c] : 0.f;
  }
  const int TRr = (r + 15) / 16, nt = 4 * TRr;
  const int64_t ntiles = (n + kLaiRows - 1) / kLaiRows;
  // pipelined when U takes 16-byte loads: the workgroup's next slab is in flight in
  // registers while the MFMAs run on the current one
  const bool vec = (ell & 3) == 0 && (reinterpret_cast<uintptr_t>(U) & 15) == 0;
  SlabRegs<kLaiRows * kMaxEll / 4 / 256> ru;
  if (vec && (int64_t)blockIdx.x < ntiles) ru.load(U, n, ell, (int64_t)blockIdx.x * kLaiRows);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * kLaiRows;
    __syncthreads();
    if (vec) {
      ru.store(sU, ell, PA);
    } else {
      lai_stage(U, n, ell, row0, sU, PA);
      if ((ell & 3) != 0)  // zero the K padding columns of the slab
        for (int e = threadIdx.x; e < kLaiRows * (ellp - ell); e += 256)
          sU[(e / (ellp - ell)) * PA + ell + e % (ellp - ell)] = 0.f;
    }
    __syncthreads();
    if (vec && tile + gridDim.x < ntiles) ru.load(U, n, ell, (tile + gridDim.x) * kLaiRows);
    for (int t = w; t < nt; t += 4) {
      const int i0 = 16 * (t / TRr), j0 = 16 * (t % TRr);
      f32x4l d = {0.f, 0.f, 0.f, 0.f};
      for (int k0 = 0; k0 < ellp; k0 += 4) {
        const int k = k0 + (lane >> 4);
        const float a = sU[(i0 + (lane & 15)) * PA + k];
        const float b = sT[k * PT + j0 + (lane & 15)];
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d, 0, 0, 0);
      }
      const int j = j0 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + i0 + 4 * (lane >> 4) + v;
        if (row < n && j < r) B[row * r + j] = d[v];
      }
    }
  }
}

// ----------------------------------------------------------------------------- launchers
#define SNMF_DISPATCH_RP2(rp, ...)                                  \
  switch (rp) {                                                     \
    case 4: { constexpr int RP = 4; __VA_ARGS__; } break;           \
    case 8: { constexpr int RP = 8; __VA_ARGS__; } break;           \
    case 16: { constexpr int RP = 16; __VA_ARGS__; } break;         \
    case 32: { constexpr int RP = 32; __VA_ARGS__; } break;         \
    default: { constexpr int RP = 64; __VA_ARGS__; } break;         \
  }

template <typename T>
void launch_spmm(const int64_t* rowptr, const int32_t* col, const T* val, const T* X, int64_t n,
                 int r, T* Y, const T* X2, double* part, const int32_t* gate,
                 const int32_t* gate2, hipStream_t s, const RhoJob& rj) {
  int64_t nb = (n + 3) / 4;
  if (X2) nb = spmm_dot_grid(n);
  if (nb > 65535 * 4) nb = 65535 * 4;
  if (nb < 1) nb = 1;
  if (rj.G) {
    SNMF_DISPATCH_RP2(rank_pad(r),
                      hipLaunchKernelGGL((k_spmm<T, RP, true>), dim3((unsigned)(nb + 1)), dim3(256),
                                         0, s, rowptr, col, val, X, n, r, Y, X2, part, gate, gate2,
                                         rj))
  } else {
    SNMF_DISPATCH_RP2(rank_pad(r),
                      hipLaunchKernelGGL((k_spmm<T, RP, false>), dim3((unsigned)nb), dim3(256), 0,
                                         s, rowptr, col, val, X, n, r, Y, X2, part, gate, gate2,
                                         rj))
  }
}

int spmm_dot_grid(int64_t n) {
  int64_t nb = (n + 3) / 4;
  if (nb > kInnerGrid) nb = kInnerGrid;
  if (nb < 1) nb = 1;
  return (int)nb;
}

int lai_blocks(int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb > 512) nb = 512;
  if (nb < 1) nb = 1;
  return (int)nb;
}

template <typename T>
void launch_lai(const T* U, int ell, const double* lam, const T* P, int64_t n, int r,
                double* part, T* TT, T* B, const int32_t* gate, hipStream_t s, const RhoJob& rj) {
  if constexpr (sizeof(T) == 4) {
    // FP32 partials, at most lai_blocks(n) of them (the FP64 partial buffer's count)
    int nb = lai_blocks(n);
    if (nb > kLaiUtpGrid) nb = kLaiUtpGrid;
    const int64_t rpb = ((n + nb - 1) / nb + kLaiRows - 1) / kLaiRows * kLaiRows;
    nb = (int)((n + rpb - 1) / rpb);
    static bool attr_set = false;  // allow up to 96 KB of dynamic LDS (ell 128, r 64: 75 KB)
    if (!attr_set) {
      (void)hipFuncSetAttribute((const void*)k_lai_ut32,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
      (void)hipFuncSetAttribute((const void*)k_lai_utp32,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
      attr_set = true;
    }
    const size_t lds1 = (size_t)kLaiRows * (lai_pitch_k(ell) + lai_pitch_k(r)) * 4;
    hipLaunchKernelGGL(k_lai_utp32, dim3(nb + (rj.G ? 1 : 0)), dim3(256), lds1, s,
                       (const float*)U, ell, (const float*)P, n, r, rpb, (float*)part, gate, rj);
    hipLaunchKernelGGL(k_lai_reduce32, dim3((ell * r + 63) / 64), dim3(256), 0, s,
                       (const float*)part, nb, ell, r, lam, (float*)TT, gate);
    int64_t tiles = (n + kLaiRows - 1) / kLaiRows;
    if (tiles > kLaiUtGrid) tiles = kLaiUtGrid;
    const size_t lds2 =
        ((size_t)kLaiRows * lai_pitch_r(ell) + (size_t)((ell + 3) & ~3) * lai_pitch_k(r)) * 4;
    hipLaunchKernelGGL(k_lai_ut32, dim3((unsigned)tiles), dim3(256), lds2, s, (const float*)U,
                       ell, (const float*)TT, n, r, (float*)B, gate);
    return;
  }
  if (rj.G) launch_rho(rj.G, rj.r, rj.st, s);
  const int nb = lai_blocks(n);
  const int64_t rpb = (n + nb - 1) / nb;
  hipLaunchKernelGGL(k_lai_utp<T>, dim3(nb), dim3(256), 0, s, U, ell, P, n, r, rpb, part, gate);
  hipLaunchKernelGGL(k_lai_reduce<T>, dim3((ell * r + 255) / 256), dim3(256), 0, s, part, nb, ell,
                     r, lam, TT, gate);
  int64_t tiles = (n + 31) / 32;
  if (tiles > 8192) tiles = 8192;
  hipLaunchKernelGGL(k_lai_ut<T>, dim3((unsigned)tiles), dim3(256), 0, s, U, ell, TT, n, r, B,
                     gate);
}

#define SNMF_INST_SP(T)                                                                      \
  template void launch_spmm<T>(const int64_t*, const int32_t*, const T*, const T*, int64_t,  \
                               int, T*, const T*, double*, const int32_t*, const int32_t*,   \
                               hipStream_t, const RhoJob&);                                  \
  template void launch_lai<T>(const T*, int, const double*, const T*, int64_t, int, double*, \
                              T*, T*, const int32_t*, hipStream_t, const RhoJob&);
SNMF_INST_SP(float)
SNMF_INST_SP(double)

}  // namespace snmf
