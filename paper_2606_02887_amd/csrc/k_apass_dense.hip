// The A-pass B = A P for dense symmetric A: the product that dominates the per-iteration
// cost O(n^2 r) of SNMPBB (Section 4.1 complexity list).  A is streamed once per call.
//
// * FP64: LDS-tiled VALU kernel (parity mode, small n).
// * FP32: MFMA v_mfma_f32_32x32x2f32.  Because A = A^T the kernel computes
//   B^T = P^T A: rows of A feed the MFMA "B" operand, so every lane reads consecutive
//   columns of one row of A and a wave touches two full 128-byte row segments per load.
// * split BF16: A = A_hi + A_lo and P = P_hi + P_lo (round-to-nearest-even BF16), with
//   A P ~= A_hi P_hi + A_hi P_lo + A_lo P_hi accumulated in FP32 on
//   v_mfma_f32_32x32x16_bf16.  P is pre-split and transposed (r x ldp) so both operands
//   are read as 16-byte vectors.
// Every variant writes split-K partial products Bpart[s] (n x r each) that the half-step's
// init kernel adds in a fixed order.
#include "common.hpp"
#include "kernels.hpp"

namespace snmf {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// ----------------------------------------------------------------------------- FP64
__global__ __launch_bounds__(256) void k_apass_f64(const double* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ P, int64_t n, int r,
                                                   double* __restrict__ B,
                                                   const State* __restrict__ st) {
  if (st->done) return;
  constexpr int TR = 32, TK = 64;
  __shared__ double sA[TR][TK + 1];
  __shared__ double sP[TK][kMaxRank];
  const int tid = threadIdx.x, c = tid & 63, rs = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * TR;
  double acc[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) acc[p] = 0.0;
  for (int64_t k0 = 0; k0 < n; k0 += TK) {
    __syncthreads();
    for (int e = tid; e < TR * TK; e += 256) {
      const int i = e / TK, kk = e % TK;
      const int64_t row = row0 + i, col = k0 + kk;
      sA[i][kk] = (row < n && col < n) ? A[row * lda + col] : 0.0;
    }
    for (int e = tid; e < TK * kMaxRank; e += 256) {
      const int kk = e / kMaxRank, cc = e % kMaxRank;
      const int64_t k = k0 + kk;
      sP[kk][cc] = (k < n && cc < r) ? P[k * r + cc] : 0.0;
    }
    __syncthreads();
    if (c < r) {
#pragma unroll 4
      for (int kk = 0; kk < TK; ++kk) {
        const double pv = sP[kk][c];
#pragma unroll
        for (int p = 0; p < 8; ++p) acc[p] = __builtin_fma(sA[rs + 4 * p][kk], pv, acc[p]);
      }
    }
  }
  if (c < r) {
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int64_t row = row0 + rs + 4 * p;
      if (row < n) B[row * r + c] = acc[p];
    }
  }
}

// ----------------------------------------------------------------------------- FP32 MFMA
// Grid: x = blocks of 256 output rows (4 waves x 64), y = K splits of kchunk rows of A.
// Wave w handles output rows j0..j0+63 (two MFMA N-blocks of 32) and all r <= 64
// columns (one or two MFMA M-blocks).  Per k-pair a lane loads A[k+h][j0+c] and
// A[k+h][j0+32+c] (h = lane/32, c = lane%32) and P[k+h][c], P[k+h][32+c].
template <int NMB>
__global__ __launch_bounds__(256) void k_apass_f32(const float* __restrict__ A, int64_t lda,
                                                   const float* __restrict__ P, int64_t n, int r,
                                                   int64_t kchunk, float* __restrict__ Bpart,
                                                   int64_t pstride, const State* __restrict__ st) {
  if (st->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 31, h = lane >> 5;
  const int64_t j0 = ((int64_t)blockIdx.x * 4 + wave) * 64;
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  const int64_t ke = kb + kchunk < n ? kb + kchunk : n;
  f32x16 acc[NMB][2];
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[mb][nb][v] = 0.0f;
  const bool jok0 = j0 + c < n, jok1 = j0 + 32 + c < n;
  const bool mok0 = c < r, mok1 = 32 + c < r;
  const float* arow = A + j0 + c;
  constexpr int U = 8;  // k-pairs per batch of loads
  int64_t k = kb;
  for (; k + 2 * U <= ke; k += 2 * U) {
    float a0[U], a1[U], p0[U], p1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t kk = k + 2 * u + h;
      a0[u] = jok0 ? __builtin_nontemporal_load(arow + kk * lda) : 0.0f;
      a1[u] = jok1 ? __builtin_nontemporal_load(arow + kk * lda + 32) : 0.0f;
      p0[u] = mok0 ? P[kk * r + c] : 0.0f;
      if (NMB > 1) p1[u] = mok1 ? P[kk * r + 32 + c] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(p0[u], a0[u], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(p0[u], a1[u], acc[0][1], 0, 0, 0);
      if (NMB > 1) {
        acc[NMB - 1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(p1[u], a0[u], acc[NMB - 1][0], 0, 0, 0);
        acc[NMB - 1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(p1[u], a1[u], acc[NMB - 1][1], 0, 0, 0);
      }
    }
  }
  for (; k < ke; k += 2) {
    const int64_t kk = k + h;
    const bool kin = kk < ke;
    const float a0 = (kin && jok0) ? arow[kk * lda] : 0.0f;
    const float a1 = (kin && jok1) ? arow[kk * lda + 32] : 0.0f;
    const float p0 = (kin && mok0) ? P[kk * r + c] : 0.0f;
    const float p1 = (NMB > 1 && kin && mok1) ? P[kk * r + 32 + c] : 0.0f;
    acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(p0, a0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(p0, a1, acc[0][1], 0, 0, 0);
    if (NMB > 1) {
      acc[NMB - 1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(p1, a0, acc[NMB - 1][0], 0, 0, 0);
      acc[NMB - 1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(p1, a1, acc[NMB - 1][1], 0, 0, 0);
    }
  }
  // D[m][j] of block (mb, nb): lane holds j = j0 + 32 nb + c and
  // m = 32 mb + 8 (v/4) + 4 h + v%4 in register v.
  float* out = Bpart + (int64_t)blockIdx.y * pstride;
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int64_t j = j0 + 32 * nb + c;
      if (j < n) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int m = 32 * mb + 8 * (v >> 2) + 4 * h + (v & 3);
          if (m < r) out[j * r + m] = acc[mb][nb][v];
        }
      }
    }
}

// ----------------------------------------------------------------------------- split BF16
// Grid: x = blocks of 128 output rows (4 waves x 32), y = K splits (kchunk multiple of 32).
// Per 32-column slab of A a lane loads 16 consecutive BF16 of its row (two 16-byte
// vectors) from A_hi and A_lo; MFMA step s uses lane (h, row) k-values kb+16h+8s..+7,
// and the matching Pt vectors (column m = 32 nb + lane%32).
template <int NNB>
__global__ __launch_bounds__(256) void k_apass_bf16x3(const uint16_t* __restrict__ Ahi,
                                                      const uint16_t* __restrict__ Alo, int64_t ldb,
                                                      const uint16_t* __restrict__ Pthi,
                                                      const uint16_t* __restrict__ Ptlo, int64_t ldp,
                                                      int64_t n, int r, int64_t kchunk,
                                                      float* __restrict__ Bpart, int64_t pstride,
                                                      const State* __restrict__ st) {
  if (st->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 31, h = lane >> 5;
  const int64_t j0 = ((int64_t)blockIdx.x * 4 + wave) * 32;
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  int64_t ke = kb + kchunk;
  if (ke > ldb) ke = ldb;
  f32x16 acc[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[nb][v] = 0.0f;
  const int64_t j = j0 + c;
  const bool jok = j < n;
  const uint16_t* ah = Ahi + (jok ? j : 0) * ldb + 16 * h;
  const uint16_t* al = Alo + (jok ? j : 0) * ldb + 16 * h;
  const uint16_t* ph[NNB];
  const uint16_t* pl[NNB];
  bool mok[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) {
    const int m = 32 * nb + c;
    mok[nb] = m < r;
    ph[nb] = Pthi + (mok[nb] ? m : 0) * ldp + 16 * h;
    pl[nb] = Ptlo + (mok[nb] ? m : 0) * ldp + 16 * h;
  }
  const u16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t k = kb; k < ke; k += 32) {
    u16x8 xa[2][2];  // [hi/lo][step]
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      xa[0][s] = jok ? __builtin_nontemporal_load((const u16x8*)(ah + k + 8 * s)) : zero;
      xa[1][s] = jok ? __builtin_nontemporal_load((const u16x8*)(al + k + 8 * s)) : zero;
    }
#pragma unroll
    for (int nb = 0; nb < NNB; ++nb) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const u16x8 bh = mok[nb] ? *(const u16x8*)(ph[nb] + k + 8 * s) : zero;
        const u16x8 bl = mok[nb] ? *(const u16x8*)(pl[nb] + k + 8 * s) : zero;
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xa[0][s]),
                                                          __builtin_bit_cast(bf16x8, bh), acc[nb], 0, 0, 0);
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xa[0][s]),
                                                          __builtin_bit_cast(bf16x8, bl), acc[nb], 0, 0, 0);
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xa[1][s]),
                                                          __builtin_bit_cast(bf16x8, bh), acc[nb], 0, 0, 0);
      }
    }
  }
  // D[row][col]: row = 8 (v/4) + 4 h + v%4 (output row j0 + row), col = lane%32 (m).
  float* out = Bpart + (int64_t)blockIdx.y * pstride;
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) {
    const int m = 32 * nb + c;
    if (m < r) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t jj = j0 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (jj < n) out[jj * r + m] = acc[nb][v];
      }
    }
  }
}

// ----------------------------------------------------------------------------- partial sum
// out = part[0] + part[1] + ... (left to right, the order the init kernel uses).
template <typename T>
__global__ __launch_bounds__(256) void k_sum_parts(const T* __restrict__ part, int ks,
                                                   int64_t stride, T* __restrict__ out, int64_t N) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256) {
    T b = T(0);
    for (int s = 0; s < ks; ++s) b += part[s * stride + e];
    out[e] = b;
  }
}

template <typename T>
void launch_sum_parts(const T* part, int ks, int64_t stride, T* out, int64_t N, hipStream_t s) {
  int64_t nb = (N + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_sum_parts<T>, dim3((unsigned)nb), dim3(256), 0, s, part, ks, stride, out, N);
}
template void launch_sum_parts<float>(const float*, int, int64_t, float*, int64_t, hipStream_t);
template void launch_sum_parts<double>(const double*, int, int64_t, double*, int64_t, hipStream_t);

// ----------------------------------------------------------------------------- launchers
void launch_apass_f64(const double* A, int64_t lda, const double* P, int64_t n, int r, double* B,
                      const State* st, hipStream_t s) {
  const unsigned gx = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_apass_f64, dim3(gx), dim3(256), 0, s, A, lda, P, n, r, B, st);
}

DenseSplit plan_dense_f32(int64_t n) {
  DenseSplit d;
  const int64_t gx = (n + 255) / 256;
  int64_t ks = (512 + gx - 1) / gx;
  const int64_t kmax = (n + 63) / 64;
  if (ks > kmax) ks = kmax;
  if (ks < 1) ks = 1;
  if (ks > kMaxKSplit) ks = kMaxKSplit;
  int64_t kc = (n + ks - 1) / ks;
  kc = (kc + 15) / 16 * 16;
  d.kchunk = kc;
  d.ksplit = (int)((n + kc - 1) / kc);
  d.gx = gx;
  return d;
}

void launch_apass_f32(const float* A, int64_t lda, const float* P, int64_t n, int r,
                      const DenseSplit& d, float* Bpart, int64_t pstride, const State* st,
                      hipStream_t s) {
  dim3 grid((unsigned)d.gx, (unsigned)d.ksplit);
  if (r > 32)
    hipLaunchKernelGGL(k_apass_f32<2>, grid, dim3(256), 0, s, A, lda, P, n, r, d.kchunk, Bpart,
                       pstride, st);
  else
    hipLaunchKernelGGL(k_apass_f32<1>, grid, dim3(256), 0, s, A, lda, P, n, r, d.kchunk, Bpart,
                       pstride, st);
}

DenseSplit plan_dense_bf16(int64_t n) {
  DenseSplit d;
  const int64_t ldb = (n + 63) / 64 * 64;
  const int64_t gx = (n + 127) / 128;
  int64_t ks = (1024 + gx - 1) / gx;
  const int64_t kmax = ldb / 64;
  if (ks > kmax) ks = kmax;
  if (ks < 1) ks = 1;
  if (ks > kMaxKSplit) ks = kMaxKSplit;
  int64_t kc = (ldb + ks - 1) / ks;
  kc = (kc + 31) / 32 * 32;
  d.kchunk = kc;
  d.ksplit = (int)((ldb + kc - 1) / kc);
  d.gx = gx;
  return d;
}

void launch_apass_bf16x3(const uint16_t* Ahi, const uint16_t* Alo, int64_t ldb,
                         const uint16_t* Pthi, const uint16_t* Ptlo, int64_t ldp, int64_t n, int r,
                         const DenseSplit& d, float* Bpart, int64_t pstride, const State* st,
                         hipStream_t s) {
  dim3 grid((unsigned)d.gx, (unsigned)d.ksplit);
  if (r > 32)
    hipLaunchKernelGGL(k_apass_bf16x3<2>, grid, dim3(256), 0, s, Ahi, Alo, ldb, Pthi, Ptlo, ldp,
                       n, r, d.kchunk, Bpart, pstride, st);
  else
    hipLaunchKernelGGL(k_apass_bf16x3<1>, grid, dim3(256), 0, s, Ahi, Alo, ldb, Pthi, Ptlo, ldp,
                       n, r, d.kchunk, Bpart, pstride, st);
}

}  // namespace snmf
