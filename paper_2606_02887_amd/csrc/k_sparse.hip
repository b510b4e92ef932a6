// Sparse and low-rank products of the SNMPBB hot path.
//
// * CSR SpMM  Y = A X  (A symmetric, both triangles stored).  One wavefront per row:
//   lane (slot, c) with c = lane % RP walks the nonzeros slot, slot + 64/RP, ... of the row
//   and accumulates A_ik X[k][c]; the slots are combined with cross-lane adds.  Used for
//   the A-pass of Graph-SNMPBB and of batched graph problems, and for the Laplacian
//   products L X, L(Z-X), L S of eq. (2.3).  In "dot" mode the kernel writes FP64 partial
//   sums of <X2, A X> per workgroup (the curvature <D, L D>, reduced by the next kernel)
//   instead of storing A X.
// * LAI-SNMPBB (Section 2.3): A P ~= U (lam .* (U^T P)).  T = U^T P is an ell x r
//   reduction over all n rows (FP64 partials per workgroup, then a fixed-order sum that
//   also applies lam); B = U T is a row-local product.
#include "common.hpp"
#include "kernels.hpp"

namespace snmf {

template <typename T, int RP>
__global__ __launch_bounds__(256) void k_spmm(const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col,
                                              const T* __restrict__ val, const T* __restrict__ X,
                                              int64_t n, int r, T* __restrict__ Y,
                                              const T* __restrict__ X2, double* __restrict__ part,
                                              const int32_t* __restrict__ gate,
                                              const int32_t* __restrict__ gate2) {
  if ((gate && gate[0]) || (gate2 && gate2[0])) return;
  constexpr int NS = kWave / RP;  // nonzero slots per wave
  __shared__ double sred[kThreads / kWave * kNumPart];
  const int lane = threadIdx.x & 63;
  const int c = lane % RP, slot = lane / RP;
  const int64_t wave_id = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * kThreads / kWave;
  double dot = 0.0;
  for (int64_t row = wave_id; row < n; row += nwaves) {
    const int64_t b = rowptr[row], e = rowptr[row + 1];
    T acc = T(0);
    if (c < r) {
      for (int64_t z = b + slot; z < e; z += NS) acc += val[z] * X[(int64_t)col[z] * r + c];
    }
#pragma unroll
    for (int o = RP; o < kWave; o <<= 1) acc += __shfl_xor(acc, o, kWave);
    if (slot == 0 && c < r) {
      if (X2)
        dot += (double)X2[row * r + c] * (double)acc;
      else
        Y[row * r + c] = acc;
    }
  }
  if (!X2) return;
  double v[1] = {dot};
  block_sum<1>(v, sred);
  if (threadIdx.x == 0) part[(size_t)blockIdx.x * kNumPart] = v[0];
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
  const int64_t* __restrict__ rowptr = G->rowptr;
  const int32_t* __restrict__ col = G->col;
  const T* __restrict__ val = (const T*)G->val;
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
                 const int32_t* gate2, hipStream_t s) {
  int64_t nb = (n + 3) / 4;
  if (X2) nb = spmm_dot_grid(n);
  if (nb > 65535 * 4) nb = 65535 * 4;
  if (nb < 1) nb = 1;
  SNMF_DISPATCH_RP2(rank_pad(r),
                    hipLaunchKernelGGL((k_spmm<T, RP>), dim3((unsigned)nb), dim3(256), 0, s,
                                       rowptr, col, val, X, n, r, Y, X2, part, gate, gate2))
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
                double* part, T* TT, T* B, const int32_t* gate, hipStream_t s) {
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
                               hipStream_t);                                                 \
  template void launch_lai<T>(const T*, int, const double*, const T*, int64_t, int, double*, \
                              T*, T*, const int32_t*, hipStream_t);
SNMF_INST_SP(float)
SNMF_INST_SP(double)

}  // namespace snmf
