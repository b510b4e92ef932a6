// Kernels of the graph preprocessing of Graph-SNMPBB (Section 2.2): K nearest neighbours
// by brute force, the union-symmetrised neighbour pattern as CSR, the Gaussian (or
// unweighted) similarity values and the normalised Laplacian I - D^{-1/2} V D^{-1/2} of
// eq. (2.3).  Distances and degrees are formed in FP64, so the integer decisions (which
// points are neighbours) are taken in the precision of the FP64 reference.
#include "common.hpp"
#include "kernels.hpp"

namespace snmf {

// ----------------------------------------------------------------------------- kNN
// One wavefront per query point i; its coordinates are staged in LDS.  Lane l scans the
// candidates j = l, l + 64, ... (increasing j) and keeps the KB smallest (distance, j)
// pairs in a sorted register list (a candidate that ties with a kept one goes after it,
// so within a lane ties keep the lower index).  The wave then takes the K smallest over
// all lanes by K rounds of a (distance, index) minimum across lanes, the winning lane
// dropping its head.  The point itself is skipped.
template <typename T, int KB>
__global__ __launch_bounds__(kThreads) void k_knn(const T* __restrict__ X, int64_t n, int dim,
                                                  int K, int32_t* __restrict__ nbr) {
  __shared__ double sq[kThreads / kWave][kKnnMaxDim];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * (kThreads / kWave) + wv;
  const bool valid = i < n;  // the waves past n stay for the barrier, then leave
  if (valid)
    for (int c = lane; c < dim; c += kWave) sq[wv][c] = (double)X[i * dim + c];
  __syncthreads();
  if (!valid) return;
  double dist[KB];
  int32_t idx[KB];
#pragma unroll
  for (int q = 0; q < KB; ++q) {
    dist[q] = __builtin_inf();
    idx[q] = 0x7fffffff;
  }
  for (int64_t j = lane; j < n; j += kWave) {
    if (j == i) continue;
    const T* __restrict__ xj = X + j * dim;
    double d = 0.0;
    for (int c = 0; c < dim; ++c) {
      const double t = sq[wv][c] - (double)xj[c];
      d = __builtin_fma(t, t, d);
    }
    if (d < dist[KB - 1]) {
#pragma unroll
      for (int q = KB - 1; q > 0; --q) {
        const bool sh = d < dist[q - 1];
        const bool here = !sh && d < dist[q];
        const double nd = sh ? dist[q - 1] : (here ? d : dist[q]);
        const int32_t ni = sh ? idx[q - 1] : (here ? (int32_t)j : idx[q]);
        dist[q] = nd;
        idx[q] = ni;
      }
      if (d < dist[0]) {
        dist[0] = d;
        idx[0] = (int32_t)j;
      }
    }
  }
  for (int t = 0; t < K; ++t) {
    double bd = dist[0];
    int32_t bi = idx[0];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double od = __shfl_xor(bd, o);
      const int32_t oi = __shfl_xor(bi, o);
      if (od < bd || (od == bd && oi < bi)) {
        bd = od;
        bi = oi;
      }
    }
    if (lane == 0) nbr[i * K + t] = bi;
    if (idx[0] == bi) {  // the lane that held the winner drops its head
#pragma unroll
      for (int q = 0; q < KB - 1; ++q) {
        dist[q] = dist[q + 1];
        idx[q] = idx[q + 1];
      }
      dist[KB - 1] = __builtin_inf();
      idx[KB - 1] = 0x7fffffff;
    }
  }
}

// ----------------------------------------------------------------------------- pattern
// True if i is among the K neighbours of j.
__device__ __forceinline__ bool lists(const int32_t* __restrict__ nbr, int K, int64_t j,
                                      int64_t i) {
  for (int t = 0; t < K; ++t)
    if (nbr[j * K + t] == (int32_t)i) return true;
  return false;
}

// cnt[j] += 1 for every edge i -> j whose reverse j -> i is not listed (the union adds i to
// row j).
__global__ __launch_bounds__(kThreads) void k_knn_incount(const int32_t* __restrict__ nbr,
                                                          int64_t n, int K,
                                                          unsigned* __restrict__ cnt) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n * K) return;
  const int64_t i = e / K;
  const int64_t j = nbr[e];
  if (!lists(nbr, K, j, i)) atomicAdd(&cnt[j], 1u);
}

// rowptr[0] = 0, rowptr[i + 1] = rowptr[i] + K + cnt[i] + diag, in one workgroup: thread t
// sums a contiguous chunk of rows, the chunk totals are scanned in thread order.
__global__ __launch_bounds__(kThreads) void k_knn_rowptr(const unsigned* __restrict__ cnt,
                                                         int64_t n, int K, int diag,
                                                         int64_t* __restrict__ rowptr) {
  __shared__ int64_t tot[kThreads];
  const int64_t chunk = (n + kThreads - 1) / kThreads;
  const int64_t b = (int64_t)threadIdx.x * chunk;
  const int64_t e = b + chunk < n ? b + chunk : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += K + (int64_t)cnt[i] + diag;
  tot[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int t = 0; t < kThreads; ++t) {
      const int64_t v = tot[t];
      tot[t] = run;
      run += v;
    }
    rowptr[n] = run;
  }
  __syncthreads();
  int64_t run = tot[threadIdx.x];
  for (int64_t i = b; i < e; ++i) {
    rowptr[i] = run;
    run += K + (int64_t)cnt[i] + diag;
  }
}

// Row i: its own K neighbours (and i itself when diag) first; cursor[i] = where the
// union's additions to row i begin.
__global__ __launch_bounds__(kThreads) void k_knn_own(const int32_t* __restrict__ nbr, int64_t n,
                                                      int K, int diag,
                                                      const int64_t* __restrict__ rowptr,
                                                      int32_t* __restrict__ col,
                                                      unsigned long long* __restrict__ cursor) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  int64_t p = rowptr[i];
  for (int t = 0; t < K; ++t) col[p++] = nbr[i * K + t];
  if (diag) col[p++] = (int32_t)i;
  cursor[i] = (unsigned long long)p;
}

// The union's additions: i is appended to row j for every edge i -> j without its reverse.
__global__ __launch_bounds__(kThreads) void k_knn_add(const int32_t* __restrict__ nbr, int64_t n,
                                                      int K, int32_t* __restrict__ col,
                                                      unsigned long long* __restrict__ cursor) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n * K) return;
  const int64_t i = e / K;
  const int64_t j = nbr[e];
  if (lists(nbr, K, j, i)) return;
  const unsigned long long p = atomicAdd(&cursor[j], 1ull);
  col[p] = (int32_t)i;
}

// Sort every row's columns (insertion sort, one thread per row; the order the additions
// arrived in is not deterministic, the sorted row is).
__global__ __launch_bounds__(kThreads) void k_sort_rows(const int64_t* __restrict__ rowptr,
                                                        int64_t n, int32_t* __restrict__ col) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t b = rowptr[i], e = rowptr[i + 1];
  for (int64_t a = b + 1; a < e; ++a) {
    const int32_t v = col[a];
    int64_t q = a - 1;
    while (q >= b && col[q] > v) {
      col[q + 1] = col[q];
      --q;
    }
    col[q + 1] = v;
  }
}

// ----------------------------------------------------------------------------- values
// v_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)) (sigma > 0) or 1, 0 on the diagonal; the
// degree d_i = sum_j v_ij in column order (FP64).  One thread per row.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_knn_values(const T* __restrict__ X, int64_t n,
                                                         int dim, double sigma,
                                                         const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         double* __restrict__ v,
                                                         double* __restrict__ deg) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const double inv = sigma > 0.0 ? 1.0 / (2.0 * sigma * sigma) : 0.0;
  double d = 0.0;
  for (int64_t z = rowptr[i]; z < rowptr[i + 1]; ++z) {
    const int64_t j = col[z];
    double w = 0.0;
    if (j != i) {
      w = 1.0;
      if (sigma > 0.0) {
        double s2 = 0.0;
        for (int c = 0; c < dim; ++c) {
          const double t = (double)X[i * dim + c] - (double)X[j * dim + c];
          s2 = __builtin_fma(t, t, s2);
        }
        w = exp(-s2 * inv);
      }
    }
    v[z] = w;
    d += w;
  }
  deg[i] = d;
}

// Output values: the similarity itself, or L_ij = [i == j] - s_i v_ij s_j with
// s = d^{-1/2} (0 where d = 0).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_knn_out(int64_t n, int laplacian,
                                                      const int64_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ deg,
                                                      T* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const double si = deg[i] > 0.0 ? 1.0 / sqrt(deg[i]) : 0.0;
  for (int64_t z = rowptr[i]; z < rowptr[i + 1]; ++z) {
    if (!laplacian) {
      val[z] = (T)v[z];
      continue;
    }
    const int64_t j = col[z];
    const double sj = deg[j] > 0.0 ? 1.0 / sqrt(deg[j]) : 0.0;
    val[z] = (T)((j == i ? 1.0 : 0.0) - si * v[z] * sj);
  }
}

// flag[0] += number of non-finite coordinates (the search needs finite distances).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_count_nonfinite(const T* __restrict__ X,
                                                              int64_t count,
                                                              unsigned* __restrict__ flag) {
  unsigned bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * kThreads) {
    const double a = (double)X[e];
    if (!(a - a == 0.0)) ++bad;
  }
  if (bad) atomicAdd(flag, bad);
}

// ----------------------------------------------------------------------------- launchers
template <typename T>
void launch_count_nonfinite(const T* X, int64_t count, unsigned* flag, hipStream_t s) {
  int64_t nb = (count + kThreads - 1) / kThreads;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_count_nonfinite<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, X, count,
                     flag);
}
template void launch_count_nonfinite<float>(const float*, int64_t, unsigned*, hipStream_t);
template void launch_count_nonfinite<double>(const double*, int64_t, unsigned*, hipStream_t);

template <typename T>
void launch_knn(const T* X, int64_t n, int dim, int K, int32_t* nbr, hipStream_t s) {
  const dim3 grid((unsigned)((n + 3) / 4)), blk(kThreads);
  if (K <= 16)
    hipLaunchKernelGGL((k_knn<T, 16>), grid, blk, 0, s, X, n, dim, K, nbr);
  else if (K <= 32)
    hipLaunchKernelGGL((k_knn<T, 32>), grid, blk, 0, s, X, n, dim, K, nbr);
  else
    hipLaunchKernelGGL((k_knn<T, 64>), grid, blk, 0, s, X, n, dim, K, nbr);
}

static unsigned blocks_of(int64_t m) { return (unsigned)((m + kThreads - 1) / kThreads); }

void launch_knn_pattern_count(const int32_t* nbr, int64_t n, int K, int diag, unsigned* cnt,
                              int64_t* rowptr, hipStream_t s) {
  hipLaunchKernelGGL(k_knn_incount, dim3(blocks_of(n * K)), dim3(kThreads), 0, s, nbr, n, K, cnt);
  hipLaunchKernelGGL(k_knn_rowptr, dim3(1), dim3(kThreads), 0, s, (const unsigned*)cnt, n, K, diag,
                     rowptr);
}

void launch_knn_pattern_fill(const int32_t* nbr, int64_t n, int K, int diag,
                             const int64_t* rowptr, int32_t* col, unsigned long long* cursor,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_knn_own, dim3(blocks_of(n)), dim3(kThreads), 0, s, nbr, n, K, diag, rowptr,
                     col, cursor);
  hipLaunchKernelGGL(k_knn_add, dim3(blocks_of(n * K)), dim3(kThreads), 0, s, nbr, n, K, col,
                     cursor);
  hipLaunchKernelGGL(k_sort_rows, dim3(blocks_of(n)), dim3(kThreads), 0, s, rowptr, n, col);
}

template <typename T>
void launch_knn_values(const T* X, int64_t n, int dim, double sigma, int laplacian,
                       const int64_t* rowptr, const int32_t* col, double* v, double* deg, T* val,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_knn_values<T>, dim3(blocks_of(n)), dim3(kThreads), 0, s, X, n, dim, sigma,
                     rowptr, col, v, deg);
  hipLaunchKernelGGL(k_knn_out<T>, dim3(blocks_of(n)), dim3(kThreads), 0, s, n, laplacian, rowptr,
                     col, (const double*)v, (const double*)deg, val);
}

template void launch_knn<float>(const float*, int64_t, int, int, int32_t*, hipStream_t);
template void launch_knn<double>(const double*, int64_t, int, int, int32_t*, hipStream_t);
template void launch_knn_values<float>(const float*, int64_t, int, double, int, const int64_t*,
                                       const int32_t*, double*, double*, float*, hipStream_t);
template void launch_knn_values<double>(const double*, int64_t, int, double, int, const int64_t*,
                                        const int32_t*, double*, double*, double*, hipStream_t);

}  // namespace snmf
