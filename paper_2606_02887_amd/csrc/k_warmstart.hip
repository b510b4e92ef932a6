// The learned warm start of SNMPBB (not in the paper; the paper's closest analogue is
// the SVD-based start of its numerical experiments, Section 4.2):
//   frame   for every instance (one workgroup each): d = A 1, the sketch rows Y_i / d_i,
//           successive projection (SPA, Gillis & Vavasis 2014) for r anchor rows K, and
//           the coordinates C = Y Y_K^T (Y_K Y_K^T + eps I)^{-1}, eps = 1e-12 tr / r;
//           divided by the entry RMS of relu(C);
//   network W0_i = s relu(c_i + M2 relu(M1 c_i + b1) + b2), r -> H -> r (residual: with
//           M2 = 0, b2 = 0 the frame's own start s relu(c_i)), BF16 weights and FP32
//           arithmetic, s = (sqrt(r) ||A||_F / (n r))^(1/2);
//   targets converged factor columns matched to the anchor order (linear assignment on
//           column cosines, Hungarian method) and divided by their entry RMS;
//   training forward / backward over a minibatch of rows, gradients reduced in a fixed
//           order, Adam (Kingma & Ba 2015), BF16 copies refreshed after every step.
#include "common.hpp"
#include "kernels.hpp"

namespace snmf {

__device__ __forceinline__ float bf16f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf16(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// A training row index, clamped into the row pool [0, pool).
__device__ __forceinline__ int64_t pool_row(const int32_t* idx, int64_t q, int64_t pool) {
  int64_t v = idx[q];
  return v < 0 ? 0 : (v >= pool ? pool - 1 : v);
}

// Block-wide argmax of (value, index): largest value, lowest index among equal values.
// Valid in every thread on return.
__device__ __forceinline__ void block_argmax(double& v, int& idx, double* sv, int* si) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double ov = __shfl_xor(v, o, kWave);
    const int oi = __shfl_xor(idx, o, kWave);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & 63) == 0) {
    sv[w] = v;
    si[w] = idx;
  }
  __syncthreads();
  v = sv[0];
  idx = si[0];
#pragma unroll
  for (int q = 1; q < kThreads / kWave; ++q)
    if (sv[q] > v || (sv[q] == v && si[q] < idx)) {
      v = sv[q];
      idx = si[q];
    }
  __syncthreads();
}

// ----------------------------------------------------------------------------- frame
// One workgroup per instance.  Y: the sketch A Omega (batch buffer); R: FP64 scratch of
// the same layout; C: output coordinates; anchors: kMaxRank ints per instance.
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_ws_frame(const BInst* __restrict__ inst,
                                                       const BGraph* __restrict__ graphs,
                                                       const T* __restrict__ Ybuf,
                                                       double* __restrict__ Rbuf,
                                                       T* __restrict__ Cbuf,
                                                       int32_t* __restrict__ anchors) {
  __shared__ double su[kMaxRank];
  __shared__ double sG[kMaxRank * kMaxRank];
  __shared__ double sM[kMaxRank * kMaxRank];
  __shared__ double sv[kThreads / kWave];
  __shared__ int si[kThreads / kWave];
  __shared__ int sK[kMaxRank];
  const int i = blockIdx.x;
  const BInst d = inst[i];
  const BGraph G = graphs[d.prob];
  const int r = d.r;
  const int64_t n = d.n;
  const T* __restrict__ Y = Ybuf + d.off;
  double* __restrict__ R = Rbuf + d.off;
  // table pointers: cast to global memory so the loads are not flat instructions
  typedef const __attribute__((address_space(1))) int64_t* GI64;
  typedef const __attribute__((address_space(1))) T* GT_;
  const GI64 __restrict__ rowptr = (GI64)G.rowptr;
  const GT_ __restrict__ val = (GT_)G.val;
  // R_i = Y_i / d_i and the first squared norms
  double best = -1.0;
  int bidx = 0;
  const double* __restrict__ degd = G.deg;
  for (int64_t row = threadIdx.x; row < n; row += kThreads) {
    double deg = 0.0;
    if (degd) {
      deg = degd[row];
    } else {
      for (int64_t z = rowptr[row]; z < rowptr[row + 1]; ++z) deg += (double)val[z];
    }
    const double inv = deg > 0.0 ? 1.0 / deg : 0.0;
    double nrm = 0.0;
#pragma unroll
    for (int c = 0; c < RP; ++c) {
      if (c < r) {
        const double x = deg > 0.0 ? (double)Y[row * r + c] * inv : 0.0;
        R[row * r + c] = x;
        nrm = __builtin_fma(x, x, nrm);
      }
    }
    if (nrm > best) {  // rows visited in increasing order: ties keep the lowest index
      best = nrm;
      bidx = (int)row;
    }
  }
  __syncthreads();
  block_argmax(best, bidx, sv, si);
  // successive projection
  for (int j = 0; j < r; ++j) {
    const int k = bidx;
    if (threadIdx.x == 0) sK[j] = k;
    const double nk = best;
    if ((int)threadIdx.x < kMaxRank)
      su[threadIdx.x] = (nk > 0.0 && (int)threadIdx.x < r) ? R[(int64_t)k * r + threadIdx.x] / sqrt(nk) : 0.0;
    __syncthreads();
    best = -1.0;
    bidx = 0;
    for (int64_t row = threadIdx.x; row < n; row += kThreads) {
      double x[RP];
      double dot = 0.0;
#pragma unroll
      for (int c = 0; c < RP; ++c) {
        x[c] = c < r ? R[row * r + c] : 0.0;
        dot = __builtin_fma(x[c], su[c], dot);
      }
      double nrm = 0.0;
#pragma unroll
      for (int c = 0; c < RP; ++c) {
        if (c < r) {
          const double y = x[c] - dot * su[c];
          R[row * r + c] = y;
          nrm = __builtin_fma(y, y, nrm);
        }
      }
      if (nrm > best) {
        best = nrm;
        bidx = (int)row;
      }
    }
    __syncthreads();
    block_argmax(best, bidx, sv, si);
  }
  // Gk = Y_K Y_K^T + eps I, its inverse by Cholesky, M = Y_K^T Gk^{-1}
  for (int e = threadIdx.x; e < r * r; e += kThreads) {
    const int a = e / r, b = e % r;
    double s = 0.0;
    for (int c = 0; c < r; ++c)
      s = __builtin_fma((double)Y[(int64_t)sK[a] * r + c], (double)Y[(int64_t)sK[b] * r + c], s);
    sG[a * kMaxRank + b] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int a = 0; a < r; ++a) tr += sG[a * kMaxRank + a];
    const double eps = 1e-12 * tr / r;
    for (int a = 0; a < r; ++a) sG[a * kMaxRank + a] += eps;
  }
  __syncthreads();
  // Cholesky Gk = L L^T in place (lower triangle), one column at a time
  for (int c = 0; c < r; ++c) {
    if (threadIdx.x == 0) {
      double s = sG[c * kMaxRank + c];
      for (int q = 0; q < c; ++q) s -= sG[c * kMaxRank + q] * sG[c * kMaxRank + q];
      sG[c * kMaxRank + c] = sqrt(fmax(s, 1e-300));
    }
    __syncthreads();
    for (int a = c + 1 + threadIdx.x; a < r; a += kThreads) {
      double s = sG[a * kMaxRank + c];
      for (int q = 0; q < c; ++q) s -= sG[a * kMaxRank + q] * sG[c * kMaxRank + q];
      sG[a * kMaxRank + c] = s / sG[c * kMaxRank + c];
    }
    __syncthreads();
  }
  // column b of Gk^{-1}: solve L z = e_b, then L^T x = z (thread b), into sM
  if ((int)threadIdx.x < r) {
    const int b = threadIdx.x;
    double z[kMaxRank];
    for (int a = 0; a < r; ++a) {
      double s = a == b ? 1.0 : 0.0;
      for (int q = 0; q < a; ++q) s -= sG[a * kMaxRank + q] * z[q];
      z[a] = s / sG[a * kMaxRank + a];
    }
    for (int a = r - 1; a >= 0; --a) {
      double s = z[a];
      for (int q = a + 1; q < r; ++q) s -= sG[q * kMaxRank + a] * z[q];
      z[a] = s / sG[a * kMaxRank + a];
    }
    for (int a = 0; a < r; ++a) sM[a * kMaxRank + b] = z[a];  // Gk^{-1} (symmetric)
  }
  __syncthreads();
  // M = Y_K^T Gk^{-1} (r x r): M[c][b] = sum_a Y[K_a][c] Ginv[a][b]; reuse sG
  for (int e = threadIdx.x; e < r * r; e += kThreads) {
    const int c = e / r, b = e % r;
    double s = 0.0;
    for (int a = 0; a < r; ++a) s = __builtin_fma((double)Y[(int64_t)sK[a] * r + c], sM[a * kMaxRank + b], s);
    sG[c * kMaxRank + b] = s;
  }
  __syncthreads();
  T* __restrict__ Cout = Cbuf + d.off;
  double pos2[1] = {0.0};  // sum of relu(C)^2 of the stored values
  for (int64_t row = threadIdx.x; row < n; row += kThreads) {
    double y[RP];
#pragma unroll
    for (int c = 0; c < RP; ++c) y[c] = c < r ? (double)Y[row * r + c] : 0.0;
    for (int b = 0; b < r; ++b) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < RP; ++c)
        if (c < r) s = __builtin_fma(y[c], sG[c * kMaxRank + b], s);
      const T cv = (T)s;
      Cout[row * r + b] = cv;
      const double p = fmax((double)cv, 0.0);
      pos2[0] = __builtin_fma(p, p, pos2[0]);
    }
  }
  // C divided by the entry RMS of relu(C) (kept if relu(C) = 0): every thread rescales
  // the rows it wrote
  block_sum<1>(pos2, sv);
  const double rms = sqrt(pos2[0] / ((double)n * r));
  if (rms > 0.0) {
    const double kap = 1.0 / rms;
    for (int64_t row = threadIdx.x; row < n; row += kThreads)
      for (int b = 0; b < r; ++b) Cout[row * r + b] = (T)((double)Cout[row * r + b] * kap);
  }
  if ((int)threadIdx.x < r) anchors[(size_t)i * kMaxRank + threadIdx.x] = sK[threadIdx.x];
}

#define SNMF_DISPATCH_WS(rp, ...)                                    \
  switch (rp) {                                                      \
    case 4: { constexpr int RP = 4; __VA_ARGS__; } break;            \
    case 8: { constexpr int RP = 8; __VA_ARGS__; } break;            \
    case 16: { constexpr int RP = 16; __VA_ARGS__; } break;          \
    case 32: { constexpr int RP = 32; __VA_ARGS__; } break;          \
    default: { constexpr int RP = 64; __VA_ARGS__; } break;          \
  }

// Row sums deg[i] = sum_j A[i][j] of a dense matrix in FP64: one wavefront per row, each
// lane adds every 64th entry in order, then a fixed shuffle tree.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dense_rowsum(const T* __restrict__ A, int64_t n,
                                                           int64_t ld, double* __restrict__ deg) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (kThreads / kWave) + (threadIdx.x >> 6);
  if (row >= n) return;
  const T* __restrict__ a = A + row * ld;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += kWave) s += (double)a[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) deg[row] = s;
}

template <typename T>
void launch_dense_rowsum(const T* A, int64_t n, int64_t ld, double* deg, hipStream_t s) {
  const int64_t rows_per = kThreads / kWave;
  hipLaunchKernelGGL(k_dense_rowsum<T>, dim3((unsigned)((n + rows_per - 1) / rows_per)),
                     dim3(kThreads), 0, s, A, n, ld, deg);
}
template void launch_dense_rowsum<float>(const float*, int64_t, int64_t, double*, hipStream_t);
template void launch_dense_rowsum<double>(const double*, int64_t, int64_t, double*, hipStream_t);

template <typename T>
void launch_ws_frame(const BInst* inst, int ninst, int max_r, const BGraph* graphs, const T* Y,
                     double* R, T* C, int32_t* anchors, hipStream_t s) {
  SNMF_DISPATCH_WS(rank_pad(max_r),
                   hipLaunchKernelGGL((k_ws_frame<T, RP>), dim3(ninst), dim3(kThreads), 0, s,
                                      inst, graphs, Y, R, C, anchors))
}
template void launch_ws_frame<float>(const BInst*, int, int, const BGraph*, const float*, double*,
                                     float*, int32_t*, hipStream_t);
template void launch_ws_frame<double>(const BInst*, int, int, const BGraph*, const double*,
                                      double*, double*, int32_t*, hipStream_t);

// ----------------------------------------------------------------------------- targets
// One workgroup per instance: cosines of the columns of C and Ht (FP64), the assignment
// p maximising sum_j cos(C_j, Ht_p[j]) (Hungarian method with potentials on the cost
// -cos, one thread), then Tout[:, j] = Ht[:, p[j]] / rms(Ht).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_ws_match(const BInst* __restrict__ inst,
                                                       const T* __restrict__ Cbuf,
                                                       const T* __restrict__ Hbuf,
                                                       T* __restrict__ Tbuf,
                                                       int32_t* __restrict__ perm) {
  __shared__ double sc[kMaxRank * kMaxRank];
  __shared__ double cn[kMaxRank], hn[kMaxRank];
  __shared__ int sp[kMaxRank];
  const int i = blockIdx.x;
  const BInst d = inst[i];
  const int r = d.r;
  const int64_t n = d.n;
  const T* __restrict__ C = Cbuf + d.off;
  const T* __restrict__ H = Hbuf + d.off;
  // inner products <C_a, H_b>, then column norms: entries e < r*r, norms after
  for (int e = threadIdx.x; e < r * r + 2 * r; e += kThreads) {
    double s = 0.0;
    if (e < r * r) {
      const int a = e / r, b = e % r;
      for (int64_t row = 0; row < n; ++row)
        s = __builtin_fma((double)C[row * r + a], (double)H[row * r + b], s);
      sc[a * kMaxRank + b] = s;
    } else if (e < r * r + r) {
      const int a = e - r * r;
      for (int64_t row = 0; row < n; ++row) s = __builtin_fma((double)C[row * r + a], (double)C[row * r + a], s);
      cn[a] = sqrt(s);
    } else {
      const int b = e - r * r - r;
      for (int64_t row = 0; row < n; ++row) s = __builtin_fma((double)H[row * r + b], (double)H[row * r + b], s);
      hn[b] = sqrt(s);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // cost[a][b] = -cos(C_a, H_b); Hungarian method with row/column potentials (1-based)
    double u[kMaxRank + 1], v[kMaxRank + 1], minv[kMaxRank + 1];
    int p[kMaxRank + 1], way[kMaxRank + 1];
    bool used[kMaxRank + 1];
    for (int q = 0; q <= r; ++q) {
      u[q] = 0.0;
      v[q] = 0.0;
      p[q] = 0;
      way[q] = 0;
    }
    for (int a = 1; a <= r; ++a) {
      p[0] = a;
      int j0 = 0;
      for (int q = 0; q <= r; ++q) {
        minv[q] = 1e300;
        used[q] = false;
      }
      int guard = 0;
      do {
        used[j0] = true;
        const int i0 = p[j0];
        double delta = 1e300;
        int j1 = 0;
        for (int j = 1; j <= r; ++j) {
          if (used[j]) continue;
          const double den = fmax(cn[i0 - 1] * hn[j - 1], 1e-300);
          double cur = -sc[(i0 - 1) * kMaxRank + (j - 1)] / den - u[i0] - v[j];
          if (!(cur < 1e299)) cur = 1e299;  // non-finite costs: progress stays guaranteed
          if (cur < minv[j]) {
            minv[j] = cur;
            way[j] = j0;
          }
          if (minv[j] < delta) {
            delta = minv[j];
            j1 = j;
          }
        }
        for (int j = 0; j <= r; ++j) {
          if (used[j]) {
            u[p[j]] += delta;
            v[j] -= delta;
          } else {
            minv[j] -= delta;
          }
        }
        j0 = j1;
      } while (p[j0] != 0 && ++guard <= kMaxRank);
      guard = 0;
      do {
        const int j1 = way[j0];
        p[j0] = p[j1];
        j0 = j1;
      } while (j0 && ++guard <= kMaxRank);
    }
    for (int j = 1; j <= r; ++j) sp[p[j] - 1] = j - 1;  // anchor p[j]-1 <- column j-1
  }
  __syncthreads();
  // the matched columns divided by their entry RMS (||Ht||_F^2 = sum of the squared
  // column norms, added in column order)
  double h2 = 0.0;
  for (int b = 0; b < r; ++b) h2 = __builtin_fma(hn[b], hn[b], h2);
  const double rms = sqrt(h2 / ((double)n * r));
  const double inv = rms > 0.0 ? 1.0 / rms : 1.0;
  T* __restrict__ Tout = Tbuf + d.off;
  for (int64_t e = threadIdx.x; e < n * r; e += kThreads) {
    const int64_t row = e / r;
    const int a = (int)(e - row * r);
    Tout[e] = (T)((double)H[row * r + sp[a]] * inv);
  }
  if ((int)threadIdx.x < r) perm[(size_t)i * kMaxRank + threadIdx.x] = sp[threadIdx.x];
}

template <typename T>
void launch_ws_match(const BInst* inst, int ninst, const T* C, const T* H, T* Tout, int32_t* perm,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_ws_match<T>, dim3(ninst), dim3(kThreads), 0, s, inst, C, H, Tout, perm);
}
template void launch_ws_match<float>(const BInst*, int, const float*, const float*, float*,
                                     int32_t*, hipStream_t);
template void launch_ws_match<double>(const BInst*, int, const double*, const double*, double*,
                                      int32_t*, hipStream_t);

// ----------------------------------------------------------------------------- frame only
// The ablation without the network: W0 = s relu(C) / rms(relu(C)) per instance (one
// workgroup each; s as for the network's output).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_ws_spa_only(const BInst* __restrict__ inst,
                                                          const T* __restrict__ Cbuf,
                                                          T* __restrict__ Wbuf) {
  __shared__ double sred[kThreads / kWave * kNumPart];
  const BInst d = inst[blockIdx.x];
  const int64_t cnt = d.n * d.r;
  const T* __restrict__ C = Cbuf + d.off;
  double v[1] = {0.0};
  for (int64_t e = threadIdx.x; e < cnt; e += kThreads) {
    const double c = fmax((double)C[e], 0.0);
    v[0] = __builtin_fma(c, c, v[0]);
  }
  block_sum<1>(v, sred);
  const double rms = sqrt(v[0] / (double)cnt);
  const double s = sqrt(sqrt((double)d.r) * sqrt(d.normA2) / ((double)cnt));
  const double f = rms > 0.0 ? s / rms : 0.0;
  T* __restrict__ W = Wbuf + d.off;
  for (int64_t e = threadIdx.x; e < cnt; e += kThreads)
    W[e] = rms > 0.0 ? (T)(fmax((double)C[e], 0.0) * f) : (T)s;
}

template <typename T>
void launch_ws_spa_only(const BInst* inst, int ninst, const T* C, T* W, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_spa_only<T>, dim3(ninst), dim3(kThreads), 0, s, inst, C, W);
}
template void launch_ws_spa_only<float>(const BInst*, int, const float*, float*, hipStream_t);
template void launch_ws_spa_only<double>(const BInst*, int, const double*, double*, hipStream_t);

// ----------------------------------------------------------------------------- network
// Weights staged in LDS as FP32 (dequantised BF16): M1 (H x r) and M2^T (H x r), so row
// k of each is contiguous.  One thread per row: o = c + b2, then for every hidden unit
// a_k = M1_k c + b1_k, h_k = relu(a_k), o += h_k M2[:, k]; y = relu(o).
template <int RP>
struct MlpSmem {
  float M1[kMlpHidden * RP];
  float M2t[kMlpHidden * RP];
  float b1[kMlpHidden];
  float b2[RP];
};

template <int RP>
__device__ __forceinline__ void mlp_stage(const MlpDev& m, MlpSmem<RP>& sm) {
  const int r = m.r;
  for (int e = threadIdx.x; e < kMlpHidden * RP; e += kThreads) {
    const int k = e / RP, c = e % RP;
    sm.M1[e] = c < r ? bf16f(m.M1h[k * r + c]) : 0.f;
    sm.M2t[e] = c < r ? bf16f(m.M2h[c * kMlpHidden + k]) : 0.f;
  }
  for (int e = threadIdx.x; e < kMlpHidden; e += kThreads) sm.b1[e] = m.b1[e];
  for (int e = threadIdx.x; e < RP; e += kThreads) sm.b2[e] = e < r ? m.b2[e] : 0.f;
  __syncthreads();
}

// Forward over rows of a plain N x r array, or (bm.blk_inst != null) over the rows of the
// instances of one rank class, scaled by each instance's s.  Optional cache for training:
// pre-activations a (N x H) and outputs o (N x r).
template <int RP>
__global__ __launch_bounds__(kThreads) void k_mlp_fwd(MlpDev m, int64_t N,
                                                      const float* __restrict__ C,
                                                      const float* __restrict__ row_scale,
                                                      float* __restrict__ Y, BMap bm,
                                                      const int32_t* __restrict__ idx,
                                                      int64_t pool,
                                                      float* __restrict__ cache_a,
                                                      float* __restrict__ cache_o) {
  __shared__ MlpSmem<RP> sm;
  const int r = m.r;
  int64_t off = 0, rows = N, bid = blockIdx.x, nb = gridDim.x;
  float sc = 1.f;
  if (bm.blk_inst) {
    const int i = bm.blk_inst[blockIdx.x];
    const BInst* d = bm.inst + i;
    off = d->off;
    rows = d->n;
    bid = (int64_t)blockIdx.x - d->blk0;
    nb = d->nblk;
    sc = (float)sqrt(sqrt((double)r) * sqrt(d->normA2) / ((double)d->n * r));
  }
  mlp_stage<RP>(m, sm);
  for (int64_t t = bid; t * kThreads < rows; t += nb) {
    const int64_t q = t * kThreads + threadIdx.x;
    if (q >= rows) continue;
    const int64_t row = idx ? pool_row(idx, q, pool) : q;
    float c[RP], o[RP];
#pragma unroll
    for (int j = 0; j < RP; ++j) {
      c[j] = j < r ? C[off + row * r + j] : 0.f;
      o[j] = sm.b2[j] + c[j];  // the residual: o = c + M2 h + b2
    }
    for (int k = 0; k < kMlpHidden; ++k) {
      float a = sm.b1[k];
#pragma unroll
      for (int j = 0; j < RP; ++j) a = fmaf(sm.M1[k * RP + j], c[j], a);
      if (cache_a) cache_a[q * kMlpHidden + k] = a;
      const float h = fmaxf(a, 0.f);
#pragma unroll
      for (int j = 0; j < RP; ++j) o[j] = fmaf(sm.M2t[k * RP + j], h, o[j]);
    }
    const float s = row_scale ? row_scale[row] : sc;
    for (int j = 0; j < r; ++j) {
      if (cache_o) cache_o[q * r + j] = o[j];
      Y[off + q * r + j] = s * fmaxf(o[j], 0.f);
    }
  }
}

// Loss pieces of a minibatch: per-workgroup FP64 partial sums of (y - t)^2, y^2, t^2.
__global__ __launch_bounds__(kThreads) void k_mlp_loss_parts(int64_t B, int r,
                                                             const float* __restrict__ y,
                                                             const float* __restrict__ T,
                                                             const int32_t* __restrict__ idx,
                                                             int64_t pool,
                                                             double* __restrict__ part) {
  __shared__ double sred[kThreads / kWave * kNumPart];
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < B * r;
       e += (int64_t)gridDim.x * kThreads) {
    const int64_t q = e / r;
    const int j = (int)(e - q * r);
    const double yy = y[e], tt = T[pool_row(idx, q, pool) * r + j];
    v[0] += (yy - tt) * (yy - tt);
    v[1] += yy * yy;
    v[2] += tt * tt;
  }
  block_sum<3>(v, sred);
  if (threadIdx.x == 0)
    for (int j = 0; j < 3; ++j) part[(size_t)blockIdx.x * kNumPart + j] = v[j];
}

// do = dL/dy * [o > 0] with dL/dy = 2 (y - t) / N + mu 2 dlt 2 y / N; then
// da = (M2^T do) * [a > 0].  scal: {sum (y-t)^2, sum y^2, sum t^2} after reduction.
template <int RP>
__global__ __launch_bounds__(kThreads) void k_mlp_back_rows(MlpDev m, int64_t B,
                                                            const float* __restrict__ y,
                                                            const float* __restrict__ T,
                                                            const int32_t* __restrict__ idx,
                                                            int64_t pool,
                                                            const float* __restrict__ cache_a,
                                                            const float* __restrict__ cache_o,
                                                            double* __restrict__ part,
                                                            int nparts, float mu,
                                                            float* __restrict__ dO,
                                                            float* __restrict__ dA) {
  __shared__ MlpSmem<RP> sm;
  __shared__ double sred[kThreads / kWave * kNumPart];
  const int r = m.r;
  double sums[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += kThreads)
    for (int j = 0; j < 3; ++j) sums[j] += part[(size_t)b * kNumPart + j];
  block_sum<3>(sums, sred);
  const double N = (double)B * r;
  const float dlt = (float)((sums[1] - sums[2]) / N);
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // the minibatch loss
    const double dd = (sums[1] - sums[2]) / N;
    part[(size_t)kMaxGrid * kNumPart] = sums[0] / N + (double)mu * dd * dd;
  }
  mlp_stage<RP>(m, sm);
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= B) return;
  const int64_t row = pool_row(idx, q, pool);
  float dov[RP];
#pragma unroll
  for (int j = 0; j < RP; ++j) {
    float g = 0.f;
    if (j < r) {
      const float yy = y[q * r + j], tt = T[row * r + j];
      const float dy = (float)(2.0 / N) * (yy - tt) + mu * 2.f * dlt * (float)(2.0 / N) * yy;
      g = cache_o[q * r + j] > 0.f ? dy : 0.f;
      dO[q * r + j] = g;
    }
    dov[j] = g;
  }
  for (int k = 0; k < kMlpHidden; ++k) {
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < RP; ++j) s = fmaf(sm.M2t[k * RP + j], dov[j], s);
    dA[q * kMlpHidden + k] = cache_a[q * kMlpHidden + k] > 0.f ? s : 0.f;
  }
}

// Weight gradients as fixed-order sums over the B minibatch rows (FP64 accumulation),
// one thread per parameter: gM1[k][c] = sum_q dA[q][k] C[row_q][c], gb1[k] = sum dA,
// gM2[j][k] = sum_q dO[q][j] relu(a[q][k]), gb2[j] = sum dO.  Parameters are numbered
// M1 (H r), b1 (H), M2 (r H), b2 (r).
__global__ __launch_bounds__(kThreads) void k_mlp_grad(int r, int64_t B,
                                                       const float* __restrict__ C,
                                                       const int32_t* __restrict__ idx,
                                                       int64_t pool,
                                                       const float* __restrict__ cache_a,
                                                       const float* __restrict__ dO,
                                                       const float* __restrict__ dA,
                                                       float* __restrict__ grad) {
  const int H = kMlpHidden;
  const int np = H * r + H + r * H + r;
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= np) return;
  double s = 0.0;
  if (e < H * r) {
    const int k = e / r, c = e % r;
    for (int64_t q = 0; q < B; ++q) s += (double)dA[q * H + k] * (double)C[pool_row(idx, q, pool) * r + c];
  } else if (e < H * r + H) {
    const int k = e - H * r;
    for (int64_t q = 0; q < B; ++q) s += (double)dA[q * H + k];
  } else if (e < H * r + H + r * H) {
    const int f = e - H * r - H;
    const int j = f / H, k = f % H;
    for (int64_t q = 0; q < B; ++q) s += (double)dO[q * r + j] * (double)fmaxf(cache_a[q * H + k], 0.f);
  } else {
    const int j = e - H * r - H - r * H;
    for (int64_t q = 0; q < B; ++q) s += (double)dO[q * r + j];
  }
  grad[e] = (float)s;
}

// Adam on the FP32 master weights, then the BF16 copies.  step counts from 1.
__global__ __launch_bounds__(kThreads) void k_mlp_adam(MlpDev m, const float* __restrict__ grad,
                                                       float* __restrict__ mom,
                                                       float* __restrict__ vel, int step, float lr,
                                                       float beta1, float beta2, float eps) {
  const int H = kMlpHidden, r = m.r;
  const int np = H * r + H + r * H + r;
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= np) return;
  float* w;
  uint16_t* wh = nullptr;
  int at;
  if (e < H * r) {
    w = m.M1;
    wh = m.M1h;
    at = e;
  } else if (e < H * r + H) {
    w = m.b1;
    at = e - H * r;
  } else if (e < H * r + H + r * H) {
    w = m.M2;
    wh = m.M2h;
    at = e - H * r - H;
  } else {
    w = m.b2;
    at = e - H * r - H - r * H;
  }
  const float g = grad[e];
  const float mm = beta1 * mom[e] + (1.f - beta1) * g;
  const float vv = beta2 * vel[e] + (1.f - beta2) * g * g;
  mom[e] = mm;
  vel[e] = vv;
  const float mh = mm / (1.f - powf(beta1, (float)step));
  const float vh = vv / (1.f - powf(beta2, (float)step));
  const float nw = w[at] - lr * mh / (sqrtf(vh) + eps);
  w[at] = nw;
  if (wh) wh[at] = f2bf16(nw);
}

__global__ __launch_bounds__(kThreads) void k_mlp_sync(MlpDev m) {
  const int H = kMlpHidden, r = m.r;
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < H * r; e += gridDim.x * kThreads) {
    m.M1h[e] = f2bf16(m.M1[e]);
    m.M2h[e] = f2bf16(m.M2[e]);
  }
}

#define SNMF_DISPATCH_MLP(rp, ...)                                   \
  switch (rp) {                                                      \
    case 4: { constexpr int RP = 4; __VA_ARGS__; } break;            \
    case 8: { constexpr int RP = 8; __VA_ARGS__; } break;            \
    case 16: { constexpr int RP = 16; __VA_ARGS__; } break;          \
    case 32: { constexpr int RP = 32; __VA_ARGS__; } break;          \
    default: { constexpr int RP = 64; __VA_ARGS__; } break;          \
  }

int mlp_params(int r) { return kMlpHidden * r * 2 + kMlpHidden + r; }

void launch_mlp_sync(const MlpDev& m, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_sync, dim3((kMlpHidden * m.r + kThreads - 1) / kThreads),
                     dim3(kThreads), 0, s, m);
}

void launch_mlp_forward(const MlpDev& m, int64_t N, const float* C, const float* row_scale,
                        float* Y, const BMap& bm, int grid, const int32_t* idx, int64_t pool,
                        float* cache_a, float* cache_o, hipStream_t s) {
  if (!bm.blk_inst) {
    int64_t g = (N + kThreads - 1) / kThreads;
    grid = (int)(g < 1 ? 1 : (g > 65535 ? 65535 : g));
  }
  SNMF_DISPATCH_MLP(rank_pad(m.r),
                    hipLaunchKernelGGL((k_mlp_fwd<RP>), dim3(grid), dim3(kThreads), 0, s, m, N, C,
                                       row_scale, Y, bm, idx, pool, cache_a, cache_o))
}

void launch_mlp_train_step(const MlpDev& m, int64_t pool, int64_t B, const float* C,
                           const float* T, const int32_t* idx, float mu, float lr, int step,
                           const MlpWork& w, hipStream_t s) {
  launch_mlp_forward(m, B, C, nullptr, w.y, BMap{}, 0, idx, pool, w.cache_a, w.cache_o, s);
  const int np = (int)((B * m.r + kThreads - 1) / kThreads);
  const int nparts = np < 1 ? 1 : (np > kMaxGrid ? kMaxGrid : np);
  hipLaunchKernelGGL(k_mlp_loss_parts, dim3(nparts), dim3(kThreads), 0, s, B, m.r, w.y, T, idx,
                     pool, w.part);
  const int gb = (int)((B + kThreads - 1) / kThreads);
  SNMF_DISPATCH_MLP(rank_pad(m.r),
                    hipLaunchKernelGGL((k_mlp_back_rows<RP>), dim3(gb), dim3(kThreads), 0, s, m,
                                       B, w.y, T, idx, pool, w.cache_a, w.cache_o, w.part, nparts,
                                       mu, w.dO, w.dA))
  const int P = mlp_params(m.r);
  hipLaunchKernelGGL(k_mlp_grad, dim3((P + kThreads - 1) / kThreads), dim3(kThreads), 0, s, m.r,
                     B, C, idx, pool, w.cache_a, w.dO, w.dA, w.grad);
  hipLaunchKernelGGL(k_mlp_adam, dim3((P + kThreads - 1) / kThreads), dim3(kThreads), 0, s, m,
                     w.grad, m.mom, m.vel, step, lr, 0.9f, 0.999f, 1e-8f);
}

}  // namespace snmf
