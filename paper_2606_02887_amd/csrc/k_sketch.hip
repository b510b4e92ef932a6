// Kernels of the randomized range finder of LAI-SNMPBB (Section 2.3) and of the SVD start
// (Section 4.2): wide products A X (X with up to 128 columns), tall-skinny Gram products
// X^T Y in FP64 with a fixed summation order, a one-workgroup Cholesky factorisation with
// the inverse of its triangular factor, tall-skinny products X M, a one-workgroup Jacobi
// eigensolver and the selection of the dominant eigenpairs.
#include "common.hpp"
#include "kernels.hpp"

namespace snmf {

// ----------------------------------------------------------------------------- A X
// CSR: one wavefront per row; lane c owns output columns c and c + 64.  The row's
// (column, value) pairs are loaded 64 at a time and broadcast by cross-lane shuffles;
// the nonzeros are added in storage order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_spmm_wide(const int64_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const T* __restrict__ val,
                                                        const T* __restrict__ X, int64_t n, int w,
                                                        T* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * (kThreads / kWave);
  const bool own0 = lane < w, own1 = lane + 64 < w;
  for (int64_t row = wave; row < n; row += nwaves) {
    const int64_t b = rowptr[row], e = rowptr[row + 1];
    T a0 = T(0), a1 = T(0);
    for (int64_t zb = b; zb < e; zb += kWave) {
      const int cnt = e - zb < kWave ? (int)(e - zb) : kWave;
      const int mc = lane < cnt ? col[zb + lane] : 0;
      const T mv = lane < cnt ? val[zb + lane] : T(0);
      for (int k = 0; k < cnt; ++k) {
        const int ck = __shfl(mc, k, kWave);
        const T vk = __shfl(mv, k, kWave);
        const T* __restrict__ xr = X + (int64_t)ck * w;
        if (own0) a0 += vk * xr[lane];
        if (own1) a1 += vk * xr[lane + 64];
      }
    }
    T* __restrict__ yr = Y + row * w;
    if (own0) yr[lane] = a0;
    if (own1) yr[lane + 64] = a1;
  }
}

// Dense A (n x n, leading dimension ld): 64-row output tiles, K in chunks of 32 staged in
// LDS; thread t owns row t % 64 of the tile and columns t / 64 + 4 q (accumulated in T,
// K in increasing order).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dense_wide(const T* __restrict__ A, int64_t ld,
                                                         const T* __restrict__ X, int64_t n, int w,
                                                         T* __restrict__ Y) {
  __shared__ T sA[64][33];
  __shared__ T sX[32][kSketchMaxW];
  const int t = threadIdx.x, rr = t & 63, cg = t >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  T acc[kSketchMaxW / 4];
#pragma unroll
  for (int q = 0; q < kSketchMaxW / 4; ++q) acc[q] = T(0);
  for (int64_t k0 = 0; k0 < n; k0 += 32) {
    __syncthreads();
    for (int e = t; e < 64 * 32; e += kThreads) {
      const int i = e >> 5, kk = e & 31;
      const int64_t gi = row0 + i, gk = k0 + kk;
      sA[i][kk] = (gi < n && gk < n) ? A[gi * ld + gk] : T(0);
    }
    for (int e = t; e < 32 * w; e += kThreads) {
      const int kk = e / w, c = e - kk * w;
      const int64_t gk = k0 + kk;
      sX[kk][c] = gk < n ? X[gk * w + c] : T(0);
    }
    __syncthreads();
    for (int kk = 0; kk < 32; ++kk) {
      const T a = sA[rr][kk];
#pragma unroll
      for (int q = 0; q < kSketchMaxW / 4; ++q) {
        const int c = cg + 4 * q;
        if (c < w) acc[q] += a * sX[kk][c];
      }
    }
  }
  const int64_t gi = row0 + rr;
  if (gi < n) {
#pragma unroll
    for (int q = 0; q < kSketchMaxW / 4; ++q) {
      const int c = cg + 4 * q;
      if (c < w) Y[gi * w + c] = acc[q];
    }
  }
}

// ----------------------------------------------------------------------------- X^T Y
// Partial C_b = X_b^T Y_b over the rows of slab b = blockIdx.x, output tile
// (ti, tj) = blockIdx.y (32 x 32); thread (tx, ty) of 32 x 8 accumulates entries
// (32 ti + ty + 8 m, 32 tj + tx), m = 0..3, in FP64, rows in increasing order.  The
// entries (i, j) and (j, i) of X^T X are formed by the same products in the same order,
// so the Gram is exactly symmetric.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_tsgram(const T* __restrict__ X,
                                                     const T* __restrict__ Y, int64_t n, int w,
                                                     int64_t rows_per, double* __restrict__ part) {
  __shared__ double sx[32][33], sy[32][33];
  const int nt = (w + 31) / 32;
  const int ti = blockIdx.y / nt, tj = blockIdx.y % nt;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = r0 + rows_per < n ? r0 + rows_per : n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = r0; k0 < r1; k0 += 32) {
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 32; e += kThreads) {
      const int kk = e >> 5, c = e & 31;
      const int64_t gk = k0 + kk;
      const int cx = ti * 32 + c, cy = tj * 32 + c;
      sx[kk][c] = (gk < r1 && cx < w) ? (double)X[gk * w + cx] : 0.0;
      sy[kk][c] = (gk < r1 && cy < w) ? (double)Y[gk * w + cy] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < 32; ++kk) {
      const double yv = sy[kk][tx];
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m] = __builtin_fma(sx[kk][ty + 8 * m], yv, acc[m]);
    }
  }
  double* __restrict__ out = part + (size_t)blockIdx.x * w * w;
  const int c = tj * 32 + tx;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int ri = ti * 32 + ty + 8 * m;
    if (ri < w && c < w) out[ri * w + c] = acc[m];
  }
}

// C = sum over slabs of the partials, in slab order.
__global__ __launch_bounds__(kThreads) void k_tsgram_reduce(const double* __restrict__ part,
                                                            int nb, int ww,
                                                            double* __restrict__ C) {
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= ww) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * ww + e];
  C[e] = s;
}

// ----------------------------------------------------------------------------- Cholesky
// One workgroup: G + s I = R^T R with s = shift_rel tr(G) (R upper triangular, the rows
// eliminated in order), then Rinv = R^{-1} by back substitution, one column per thread.
// R and Rinv are w x w global arrays (w <= 128).  flag[0] is set when a pivot is not
// positive (the sketch has lost rank beyond what the shift covers).
__global__ __launch_bounds__(kThreads) void k_chol_inv(const double* __restrict__ G, int w,
                                                       double shift_rel, double* __restrict__ R,
                                                       double* __restrict__ Rinv,
                                                       int32_t* __restrict__ flag) {
  __shared__ double s_tr, s_piv;
  __shared__ int s_bad;
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < w; ++i) tr += G[i * w + i];
    s_tr = tr;
    s_bad = 0;
  }
  __syncthreads();
  const double sh = shift_rel * s_tr;
  for (int e = threadIdx.x; e < w * w; e += kThreads) {
    const int i = e / w, j = e - i * w;
    R[e] = j >= i ? G[e] + (i == j ? sh : 0.0) : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    if (threadIdx.x == 0) {
      const double d = R[j * w + j];
      if (!(d > 0.0)) s_bad = 1;
      s_piv = d > 0.0 ? sqrt(d) : 1.0;
      R[j * w + j] = s_piv;
    }
    __syncthreads();
    const double p = s_piv;
    for (int k = j + 1 + threadIdx.x; k < w; k += kThreads) R[j * w + k] /= p;
    __syncthreads();
    const int m = w - j - 1;
    for (int e = threadIdx.x; e < m * m; e += kThreads) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k >= i) R[i * w + k] -= R[j * w + i] * R[j * w + k];
    }
    __syncthreads();
  }
  for (int c = threadIdx.x; c < w; c += kThreads) {
    for (int i = c + 1; i < w; ++i) Rinv[i * w + c] = 0.0;
    Rinv[c * w + c] = 1.0 / R[c * w + c];
    for (int i = c - 1; i >= 0; --i) {
      double acc = 0.0;
      for (int k = i + 1; k <= c; ++k) acc = __builtin_fma(R[i * w + k], Rinv[k * w + c], acc);
      Rinv[i * w + c] = -acc / R[i * w + i];
    }
  }
  if (threadIdx.x == 0 && s_bad) flag[0] = 1;
}

// ----------------------------------------------------------------------------- X M
// Q (n x c) = Y (n x w) M (w x c, FP64), optionally |.|: 64-row tiles; M staged in LDS 32
// columns at a time; thread t owns row t / 4 of the tile and columns 8 (t % 4) .. + 7 of
// the chunk; FP64 accumulation over k in increasing order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_tsmm(const T* __restrict__ Y, int64_t n, int w,
                                                   const double* __restrict__ M, int c, int absval,
                                                   T* __restrict__ Q) {
  __shared__ double sM[kSketchMaxW][33];
  const int rr = threadIdx.x >> 2, cq = (threadIdx.x & 3) * 8;
  const int64_t row = (int64_t)blockIdx.x * 64 + rr;
  for (int c0 = 0; c0 < c; c0 += 32) {
    __syncthreads();
    for (int e = threadIdx.x; e < w * 32; e += kThreads) {
      const int k = e >> 5, j = e & 31;
      sM[k][j] = c0 + j < c ? M[k * c + c0 + j] : 0.0;
    }
    __syncthreads();
    if (row < n) {
      double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      const T* __restrict__ yr = Y + row * w;
      for (int k = 0; k < w; ++k) {
        const double y = (double)yr[k];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = __builtin_fma(y, sM[k][cq + u], acc[u]);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = c0 + cq + u;
        if (j < c) Q[row * c + j] = (T)(absval ? fabs(acc[u]) : acc[u]);
      }
    }
  }
}

// ----------------------------------------------------------------------------- Jacobi
// Eigen-decomposition S = V diag(ev) V^T of S = (Tin + Tin^T) / 2 (w x w, FP64) by cyclic
// Jacobi rotations.  A sweep runs w' - 1 rounds (w' = w rounded up to even) of w'/2
// disjoint pairs in the round-robin order: player 0 stays, players 1 .. w'-1 rotate, and
// pairs holding the padding player w are skipped.  For pair (p, q) the rotation
// c = 1/sqrt(1 + t^2), s = t c, t = sgn(th) / (|th| + sqrt(th^2 + 1)),
// th = (a_qq - a_pp) / (2 a_pq) zeroes a_pq; all rotations of a round update the rows
// first, then the columns and V (the pairs are disjoint, so this is their product).
// Sweeps stop when the off-diagonal part is below 1e-15 of the matrix (Frobenius) or
// after 50 sweeps.  A and V are w x w global arrays (w <= 128); one workgroup.
__global__ __launch_bounds__(kThreads) void k_jacobi(const double* __restrict__ Tin, int w,
                                                     double* __restrict__ A,
                                                     double* __restrict__ V,
                                                     double* __restrict__ ev) {
  __shared__ double s_c[kSketchMaxW / 2], s_s[kSketchMaxW / 2];
  __shared__ int s_p[kSketchMaxW / 2], s_q[kSketchMaxW / 2];
  __shared__ double sred[2 * (kThreads / kWave)];
  __shared__ int s_stop;
  const int tid = threadIdx.x;
  const int m = (w + 1) & ~1, np = m / 2;
  for (int e = tid; e < w * w; e += kThreads) {
    const int i = e / w, j = e - i * w;
    A[e] = 0.5 * (Tin[i * w + j] + Tin[j * w + i]);
    V[e] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < w * w; e += kThreads) {
      const int i = e / w, j = e - i * w;
      const double a = A[e];
      tot = __builtin_fma(a, a, tot);
      if (i != j) off = __builtin_fma(a, a, off);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      tot += __shfl_xor(tot, o);
    }
    if ((tid & 63) == 0) {
      sred[2 * (tid >> 6)] = off;
      sred[2 * (tid >> 6) + 1] = tot;
    }
    __syncthreads();
    if (tid == 0) {
      double o2 = 0.0, t2 = 0.0;
      for (int q = 0; q < kThreads / kWave; ++q) {
        o2 += sred[2 * q];
        t2 += sred[2 * q + 1];
      }
      s_stop = !(o2 > 1e-30 * t2);
    }
    __syncthreads();
    if (s_stop) break;
    for (int round = 0; round < m - 1; ++round) {
      if (tid < np) {
        const int a = tid == 0 ? 0 : ((tid - 1 + round) % (m - 1)) + 1;
        const int b = ((m - 2 - tid + round) % (m - 1)) + 1;
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (q < w) {
          const double apq = A[p * w + q];
          if (apq != 0.0) {
            const double th = (A[q * w + q] - A[p * w + p]) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        s_c[tid] = c;
        s_s[tid] = s;
        s_p[tid] = p;
        s_q[tid] = q;
      }
      __syncthreads();
      for (int e = tid; e < np * w; e += kThreads) {
        const int t = e / w, j = e - t * w;
        const int p = s_p[t], q = s_q[t];
        if (q >= w || s_s[t] == 0.0) continue;
        const double c = s_c[t], s = s_s[t];
        const double apj = A[p * w + j], aqj = A[q * w + j];
        A[p * w + j] = c * apj - s * aqj;
        A[q * w + j] = s * apj + c * aqj;
      }
      __syncthreads();
      for (int e = tid; e < np * w; e += kThreads) {
        const int t = e / w, i = e - t * w;
        const int p = s_p[t], q = s_q[t];
        if (q >= w || s_s[t] == 0.0) continue;
        const double c = s_c[t], s = s_s[t];
        const double aip = A[i * w + p], aiq = A[i * w + q];
        A[i * w + p] = c * aip - s * aiq;
        A[i * w + q] = s * aip + c * aiq;
        const double vip = V[i * w + p], viq = V[i * w + q];
        V[i * w + p] = c * vip - s * viq;
        V[i * w + q] = s * vip + c * viq;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < w; i += kThreads) ev[i] = A[i * w + i];
}

// ----------------------------------------------------------------------------- selection
// The k eigenpairs of largest |ev| (ties: lower index first): lam[j] = ev[o_j] and
// M[a][j] = V[a][o_j], times sqrt(|ev[o_j]|) when sqrt_scale is set.  One workgroup.
__global__ __launch_bounds__(kThreads) void k_sketch_select(const double* __restrict__ ev,
                                                            const double* __restrict__ V, int w,
                                                            int k, int sqrt_scale,
                                                            double* __restrict__ lam,
                                                            double* __restrict__ M) {
  __shared__ int order[kSketchMaxW];
  // every slot holds a valid index even if a non-finite eigenvalue breaks the ranking
  for (int i = threadIdx.x; i < kSketchMaxW; i += kThreads) order[i] = i < w ? i : 0;
  __syncthreads();
  for (int i = threadIdx.x; i < w; i += kThreads) {
    const double ai = fabs(ev[i]);
    int rank = 0;
    for (int j = 0; j < w; ++j) {
      const double aj = fabs(ev[j]);
      rank += (aj > ai) || (aj == ai && j < i);
    }
    if (rank < k) order[rank] = i;
  }
  __syncthreads();
  if (lam)
    for (int j = threadIdx.x; j < k; j += kThreads) lam[j] = ev[order[j]];
  for (int e = threadIdx.x; e < w * k; e += kThreads) {
    const int a = e / k, j = e - a * k;
    double v = V[a * w + order[j]];
    if (sqrt_scale) v *= sqrt(fabs(ev[order[j]]));
    M[e] = v;
  }
}

// ----------------------------------------------------------------------------- launchers
template <typename T>
void launch_sketch_spmm(const int64_t* rowptr, const int32_t* col, const T* val, const T* X,
                        int64_t n, int w, T* Y, hipStream_t s) {
  int64_t nb = (n + 3) / 4;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_spmm_wide<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, rowptr, col, val,
                     X, n, w, Y);
}
template <typename T>
void launch_sketch_dense(const T* A, int64_t ld, const T* X, int64_t n, int w, T* Y,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_dense_wide<T>, dim3((unsigned)((n + 63) / 64)), dim3(kThreads), 0, s, A, ld,
                     X, n, w, Y);
}
int sketch_slabs(int64_t n, int64_t* rows_per) {
  int64_t rp = (n + 255) / 256;
  if (rp < 256) rp = 256;
  *rows_per = rp;
  return (int)((n + rp - 1) / rp);
}
template <typename T>
void launch_tsgram(const T* X, const T* Y, int64_t n, int w, double* part, double* C,
                   hipStream_t s) {
  int64_t rp = 0;
  const int nb = sketch_slabs(n, &rp);
  const int nt = (w + 31) / 32;
  hipLaunchKernelGGL(k_tsgram<T>, dim3((unsigned)nb, (unsigned)(nt * nt)), dim3(kThreads), 0, s, X,
                     Y, n, w, rp, part);
  hipLaunchKernelGGL(k_tsgram_reduce, dim3((unsigned)((w * w + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, (const double*)part, nb, w * w, C);
}
void launch_chol_inv(const double* G, int w, double shift_rel, double* R, double* Rinv,
                     int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kThreads), 0, s, G, w, shift_rel, R, Rinv, flag);
}
template <typename T>
void launch_tsmm(const T* Y, int64_t n, int w, const double* M, int c, int absval, T* Q,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_tsmm<T>, dim3((unsigned)((n + 63) / 64)), dim3(kThreads), 0, s, Y, n, w, M,
                     c, absval, Q);
}
void launch_jacobi(const double* Tin, int w, double* A, double* V, double* ev, hipStream_t s) {
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kThreads), 0, s, Tin, w, A, V, ev);
}
void launch_sketch_select(const double* ev, const double* V, int w, int k, int sqrt_scale,
                          double* lam, double* M, hipStream_t s) {
  hipLaunchKernelGGL(k_sketch_select, dim3(1), dim3(kThreads), 0, s, ev, V, w, k, sqrt_scale, lam,
                     M);
}

#define SNMF_SKETCH_INST(T)                                                                       \
  template void launch_sketch_spmm<T>(const int64_t*, const int32_t*, const T*, const T*, int64_t, \
                                      int, T*, hipStream_t);                                      \
  template void launch_sketch_dense<T>(const T*, int64_t, const T*, int64_t, int, T*,             \
                                       hipStream_t);                                              \
  template void launch_tsgram<T>(const T*, const T*, int64_t, int, double*, double*, hipStream_t); \
  template void launch_tsmm<T>(const T*, int64_t, int, const double*, int, int, T*, hipStream_t);
SNMF_SKETCH_INST(float)
SNMF_SKETCH_INST(double)

}  // namespace snmf
