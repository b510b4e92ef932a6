// Kernels of NMPBB for rectangular NMF (eq. (1.1)): the products V P and V^T P of a dense
// m x n matrix with an n x r or m x r partner, and the transpose of a CSR matrix (column
// counts, their scan, the scatter and a per-row sort that makes the result deterministic).
#include "common.hpp"
#include "kernels.hpp"
#include "rho.hpp"

namespace snmf {

// B (rows x r) = V P (trans = 0: V is rows x K, row-major, leading dimension ld) or V^T P
// (trans = 1: V is K x rows).  64 output rows per workgroup, K in chunks of 32 staged in
// LDS; thread t owns row t % 64 and columns t / 64 + 4 q; accumulation in T, K in order.
// Skipped when the solve is done.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_rect_apass(const T* __restrict__ V, int64_t ld,
                                                         int64_t rows, int64_t K, int trans,
                                                         const T* __restrict__ P, int r,
                                                         T* __restrict__ B,
                                                         const State* __restrict__ st) {
  if (st->done) return;
  __shared__ T sA[64][33];
  __shared__ T sP[32][kMaxRank];
  const int t = threadIdx.x, rr = t & 63, cg = t >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  T acc[kMaxRank / 4];
#pragma unroll
  for (int q = 0; q < kMaxRank / 4; ++q) acc[q] = T(0);
  for (int64_t k0 = 0; k0 < K; k0 += 32) {
    __syncthreads();
    for (int e = t; e < 64 * 32; e += kThreads) {
      int i, kk;
      if (trans) {  // consecutive threads read consecutive entries of one row of V
        kk = e >> 6;
        i = e & 63;
      } else {
        i = e >> 5;
        kk = e & 31;
      }
      const int64_t gi = row0 + i, gk = k0 + kk;
      T a = T(0);
      if (gi < rows && gk < K) a = trans ? V[gk * ld + gi] : V[gi * ld + gk];
      sA[i][kk] = a;
    }
    for (int e = t; e < 32 * r; e += kThreads) {
      const int kk = e / r, c = e - kk * r;
      const int64_t gk = k0 + kk;
      sP[kk][c] = gk < K ? P[gk * r + c] : T(0);
    }
    __syncthreads();
    for (int kk = 0; kk < 32; ++kk) {
      const T a = sA[rr][kk];
#pragma unroll
      for (int q = 0; q < kMaxRank / 4; ++q) {
        const int c = cg + 4 * q;
        if (c < r) acc[q] += a * sP[kk][c];
      }
    }
  }
  const int64_t gi = row0 + rr;
  if (gi < rows) {
#pragma unroll
    for (int q = 0; q < kMaxRank / 4; ++q) {
      const int c = cg + 4 * q;
      if (c < r) B[gi * r + c] = acc[q];
    }
  }
}

// CSR of m rows with columns in [0, ncols): flags[0] += bad row pointers, flags[1] +=
// columns out of range, flags[2] += columns not strictly increasing within a row.
__global__ __launch_bounds__(kThreads) void k_csr_check_rect(const int64_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ col,
                                                             int64_t m, int64_t ncols,
                                                             int64_t nnz,
                                                             unsigned* __restrict__ flags) {
  unsigned bp = 0, bc = 0, us = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * kThreads) {
    const int64_t b = rowptr[i], e = rowptr[i + 1];
    if (b < 0 || e < b || e > nnz) {
      ++bp;
      continue;
    }
    int32_t prev = -1;
    for (int64_t z = b; z < e; ++z) {
      const int32_t c = col[z];
      if (c < 0 || c >= ncols) ++bc;
      if (c <= prev) ++us;
      prev = c;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (rowptr[0] != 0 || rowptr[m] != nnz))
    atomicAdd(&flags[0], 1u);
  if (bp) atomicAdd(&flags[0], bp);
  if (bc) atomicAdd(&flags[1], bc);
  if (us) atomicAdd(&flags[2], us);
}

// cnt[c] = entries of column c.
__global__ __launch_bounds__(kThreads) void k_csr_colcount(const int32_t* __restrict__ col,
                                                           int64_t nnz,
                                                           unsigned* __restrict__ cnt) {
  const int64_t z = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (z < nnz) atomicAdd(&cnt[col[z]], 1u);
}

// out[0] = 0, out[i + 1] = out[i] + cnt[i] (one workgroup: chunk sums scanned in thread
// order), and cursor[i] = out[i].
__global__ __launch_bounds__(kThreads) void k_scan_counts(const unsigned* __restrict__ cnt,
                                                          int64_t n, int64_t* __restrict__ out,
                                                          unsigned long long* __restrict__ cursor) {
  __shared__ int64_t tot[kThreads];
  const int64_t chunk = (n + kThreads - 1) / kThreads;
  const int64_t b = (int64_t)threadIdx.x * chunk;
  const int64_t e = b + chunk < n ? b + chunk : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += cnt[i];
  tot[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int q = 0; q < kThreads; ++q) {
      const int64_t v = tot[q];
      tot[q] = run;
      run += v;
    }
    out[n] = run;
  }
  __syncthreads();
  int64_t run = tot[threadIdx.x];
  for (int64_t i = b; i < e; ++i) {
    out[i] = run;
    cursor[i] = (unsigned long long)run;
    run += cnt[i];
  }
}

// Entry (i, c, v) of V goes to row c of V^T at the next free place of that row.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_csr_scatter_t(const int64_t* __restrict__ rowptr,
                                                            const int32_t* __restrict__ col,
                                                            const T* __restrict__ val, int64_t m,
                                                            unsigned long long* __restrict__ cursor,
                                                            int32_t* __restrict__ colT,
                                                            T* __restrict__ valT) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= m) return;
  for (int64_t z = rowptr[i]; z < rowptr[i + 1]; ++z) {
    const unsigned long long p = atomicAdd(&cursor[col[z]], 1ull);
    colT[p] = (int32_t)i;
    valT[p] = val[z];
  }
}

// Sort every row of V^T by column, values alongside (one thread per row; the rows' column
// indices are distinct, so the result is unique).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_csr_sort_pairs(const int64_t* __restrict__ rowptr,
                                                             int64_t n, int32_t* __restrict__ col,
                                                             T* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t b = rowptr[i], e = rowptr[i + 1];
  for (int64_t a = b + 1; a < e; ++a) {
    const int32_t c = col[a];
    const T v = val[a];
    int64_t q = a - 1;
    while (q >= b && col[q] > c) {
      col[q + 1] = col[q];
      val[q + 1] = val[q];
      --q;
    }
    col[q + 1] = c;
    val[q + 1] = v;
  }
}

// ----------------------------------------------------------------------------- FP32 MFMA
typedef float f32x16n __attribute__((ext_vector_type(16)));

// Split-K product panel y of B = A^T P: Bpart[y][j][m] = sum over k in chunk y of
// A[k][j] P[k][m], A K x N row-major (leading dimension lda), P K x r, on
// v_mfma_f32_32x32x2f32.  Grid x: blocks of 256 output rows (4 waves x 64), y: K chunks of
// kchunk rows (kchunk even).  Wave w takes output rows j0 .. j0 + 63 (two MFMA N-blocks)
// and all r <= 64 columns (NMB M-blocks of 32); per k-pair lane (c, h) = (lane % 32,
// lane / 32) loads A[k + h][j0 + c], A[k + h][j0 + 32 + c] and P[k + h][c], P[k + h][32 + c],
// eight k-pairs per batch with the next batch in flight during this one's MFMAs.  With
// A = V (m x n) the panel sums give V^T P (the H-step), with A = V^T (an n x m transposed
// copy) V P (the W-step).  With rj.G set the grid has one more row of workgroups, the
// first (dispatched before the panels, so that it runs beside them from the start), whose
// first workgroup computes rho = ||G||_2 (rho.hpp).  Skipped when the solve is done.
template <int NMB>
__global__ __launch_bounds__(256) void k_rect_f32(const float* __restrict__ A, int64_t lda,
                                                  const float* __restrict__ P, int64_t K,
                                                  int64_t N, int r, int64_t kchunk,
                                                  float* __restrict__ Bpart, int64_t pstride,
                                                  const State* __restrict__ st, RhoJob rj) {
  if (st->done) return;
  int64_t y = blockIdx.y;
  if (rj.G) {
    if (y == 0) {
      if (blockIdx.x == 0) rho_body(rj.G, rj.r, rj.st);  // (issue priority: no gain measured)
      return;
    }
    --y;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 31, h = lane >> 5;
  const int64_t j0 = ((int64_t)blockIdx.x * 4 + wave) * 64;
  const int64_t kb = y * kchunk;
  const int64_t ke = kb + kchunk < K ? kb + kchunk : K;
  f32x16n acc[NMB][2];
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[mb][nb][v] = 0.0f;
  const bool jok0 = j0 + c < N, jok1 = j0 + 32 + c < N;
  const bool mok0 = c < r, mok1 = 32 + c < r;
  const float* arow = A + j0 + c;
  constexpr int U = 8;
  float a0[U], a1[U], p0[U], p1[U];
  float b0[U], b1[U], q0[U], q1[U];
  auto load = [&](float (&x0)[U], float (&x1)[U], float (&y0)[U], float (&y1)[U], int64_t kk0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t kk = kk0 + 2 * u + h;
      x0[u] = jok0 ? __builtin_nontemporal_load(arow + kk * lda) : 0.0f;
      x1[u] = jok1 ? __builtin_nontemporal_load(arow + kk * lda + 32) : 0.0f;
      y0[u] = mok0 ? P[kk * r + c] : 0.0f;
      if (NMB > 1) y1[u] = mok1 ? P[kk * r + 32 + c] : 0.0f;
    }
  };
  auto mma = [&](const float (&x0)[U], const float (&x1)[U], const float (&y0)[U],
                 const float (&y1)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(y0[u], x0[u], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(y0[u], x1[u], acc[0][1], 0, 0, 0);
      if (NMB > 1) {
        acc[NMB - 1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(y1[u], x0[u], acc[NMB - 1][0], 0, 0, 0);
        acc[NMB - 1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(y1[u], x1[u], acc[NMB - 1][1], 0, 0, 0);
      }
    }
  };
  int64_t k = kb;
  if (k + 2 * U <= ke) load(a0, a1, p0, p1, k);
  while (k + 2 * U <= ke) {
    if (k + 4 * U <= ke) {
      load(b0, b1, q0, q1, k + 2 * U);
      mma(a0, a1, p0, p1);
      k += 2 * U;
      if (k + 4 * U <= ke) load(a0, a1, p0, p1, k + 2 * U);
      mma(b0, b1, q0, q1);
      k += 2 * U;
    } else {
      mma(a0, a1, p0, p1);
      k += 2 * U;
    }
  }
  for (; k < ke; k += 2) {
    const int64_t kk = k + h;
    const bool kin = kk < ke;
    const float x0 = (kin && jok0) ? arow[kk * lda] : 0.0f;
    const float x1 = (kin && jok1) ? arow[kk * lda + 32] : 0.0f;
    const float y0 = (kin && mok0) ? P[kk * r + c] : 0.0f;
    const float y1 = (NMB > 1 && kin && mok1) ? P[kk * r + 32 + c] : 0.0f;
    acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(y0, x0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(y0, x1, acc[0][1], 0, 0, 0);
    if (NMB > 1) {
      acc[NMB - 1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(y1, x0, acc[NMB - 1][0], 0, 0, 0);
      acc[NMB - 1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(y1, x1, acc[NMB - 1][1], 0, 0, 0);
    }
  }
  // D[m][j] of block (mb, nb): lane (c, h) holds j = j0 + 32 nb + c and
  // m = 32 mb + 8 (v / 4) + 4 h + v % 4 in register v
  float* out = Bpart + y * pstride;
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int64_t j = j0 + 32 * nb + c;
      if (j < N) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int m = 32 * mb + 8 * (v >> 2) + 4 * h + (v & 3);
          if (m < r) out[j * r + m] = acc[mb][nb][v];
        }
      }
    }
}

// AT (cols x rows) = A^T for A rows x cols (leading dimension lda): 64 x 64 tiles through
// LDS, reads and writes along rows.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T* __restrict__ A, int64_t rows,
                                                   int64_t cols, int64_t lda, T* __restrict__ AT) {
  __shared__ T t[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t rr = r0 + i, cc = c0 + tx;
    t[i][tx] = (rr < rows && cc < cols) ? A[rr * lda + cc] : T(0);
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t cc = c0 + i, rr = r0 + tx;
    if (cc < cols && rr < rows) AT[cc * rows + rr] = t[tx][i];
  }
}

static unsigned nblk(int64_t m) {
  int64_t b = (m + kThreads - 1) / kThreads;
  return (unsigned)(b < 1 ? 1 : b);
}

template <typename T>
void launch_rect_apass(const T* V, int64_t ld, int64_t rows, int64_t K, int trans, const T* P,
                       int r, T* B, const State* st, hipStream_t s) {
  hipLaunchKernelGGL(k_rect_apass<T>, dim3((unsigned)((rows + 63) / 64)), dim3(kThreads), 0, s, V,
                     ld, rows, K, trans, P, r, B, st);
}

void launch_csr_check_rect(const int64_t* rowptr, const int32_t* col, int64_t m, int64_t ncols,
                           int64_t nnz, unsigned* flags, hipStream_t s) {
  unsigned b = nblk(m);
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_csr_check_rect, dim3(b), dim3(kThreads), 0, s, rowptr, col, m, ncols, nnz,
                     flags);
}

template <typename T>
void launch_csr_transpose(const int64_t* rowptr, const int32_t* col, const T* val, int64_t m,
                          int64_t ncols, int64_t nnz, unsigned* cnt, unsigned long long* cursor,
                          int64_t* rowptrT, int32_t* colT, T* valT, hipStream_t s) {
  (void)hipMemsetAsync(cnt, 0, (size_t)ncols * sizeof(unsigned), s);
  if (nnz > 0)
    hipLaunchKernelGGL(k_csr_colcount, dim3(nblk(nnz)), dim3(kThreads), 0, s, col, nnz, cnt);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kThreads), 0, s, (const unsigned*)cnt, ncols,
                     rowptrT, cursor);
  hipLaunchKernelGGL(k_csr_scatter_t<T>, dim3(nblk(m)), dim3(kThreads), 0, s, rowptr, col, val, m,
                     cursor, colT, valT);
  hipLaunchKernelGGL(k_csr_sort_pairs<T>, dim3(nblk(ncols)), dim3(kThreads), 0, s,
                     (const int64_t*)rowptrT, ncols, colT, valT);
}

RectSplit rect_split(int64_t K, int64_t N) {
  RectSplit sp;
  sp.gx = (int)((N + 255) / 256);
  int64_t want = (512 + sp.gx - 1) / sp.gx;          // about two workgroups per CU
  int64_t most = (K + 63) / 64;                      // chunks of at least 64 rows
  if (want > most) want = most;
  if (want < 1) want = 1;
  sp.kchunk = ((K + want - 1) / want + 15) / 16 * 16;  // whole batches of eight k-pairs
  sp.ksplit = (int)((K + sp.kchunk - 1) / sp.kchunk);
  return sp;
}

void launch_rect_f32(const float* A, int64_t lda, const float* P, int64_t K, int64_t N, int r,
                     const RectSplit& sp, float* Bpart, const State* st, hipStream_t s,
                     const RhoJob& rj) {
  const dim3 grid((unsigned)sp.gx, (unsigned)(sp.ksplit + (rj.G ? 1 : 0)));
  if (r > 32)
    hipLaunchKernelGGL(k_rect_f32<2>, grid, dim3(256), 0, s, A, lda, P, K, N, r, sp.kchunk,
                       Bpart, N * r, st, rj);
  else
    hipLaunchKernelGGL(k_rect_f32<1>, grid, dim3(256), 0, s, A, lda, P, K, N, r, sp.kchunk,
                       Bpart, N * r, st, rj);
}

template <typename T>
void launch_transpose(const T* A, int64_t rows, int64_t cols, int64_t lda, T* AT, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose<T>, dim3((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64)),
                     dim3(256), 0, s, A, rows, cols, lda, AT);
}
template void launch_transpose<float>(const float*, int64_t, int64_t, int64_t, float*, hipStream_t);
template void launch_transpose<double>(const double*, int64_t, int64_t, int64_t, double*,
                                       hipStream_t);

template void launch_rect_apass<float>(const float*, int64_t, int64_t, int64_t, int, const float*,
                                       int, float*, const State*, hipStream_t);
template void launch_rect_apass<double>(const double*, int64_t, int64_t, int64_t, int,
                                        const double*, int, double*, const State*, hipStream_t);
template void launch_csr_transpose<float>(const int64_t*, const int32_t*, const float*, int64_t,
                                          int64_t, int64_t, unsigned*, unsigned long long*,
                                          int64_t*, int32_t*, float*, hipStream_t);
template void launch_csr_transpose<double>(const int64_t*, const int32_t*, const double*, int64_t,
                                           int64_t, int64_t, unsigned*, unsigned long long*,
                                           int64_t*, int32_t*, double*, hipStream_t);

}  // namespace snmf
