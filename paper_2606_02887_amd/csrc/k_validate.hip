// Input checks of the C ABI run on the device: ||x||^2 with negative / non-finite counts
// over a strided 2-D region, and CSR structure and symmetry checks.
#include "common.hpp"
#include "kernels.hpp"

namespace snmf {

// {sum of squares, negatives, non-finite} over rows x cols with leading dimension ld.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_stats2d(const T* __restrict__ x, int64_t rows,
                                                      int64_t cols, int64_t ld,
                                                      double* __restrict__ part,
                                                      double* __restrict__ out,
                                                      unsigned* __restrict__ counter) {
  __shared__ double sred[kThreads / kWave * 3];
  double v[3] = {0.0, 0.0, 0.0};
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kThreads) {
    const int64_t i = e / cols, j = e - i * cols;
    const double a = (double)x[i * ld + j];
    if (!(a - a == 0.0)) {
      v[2] += 1.0;
    } else {
      v[0] = __builtin_fma(a, a, v[0]);
      v[1] += a < 0.0 ? 1.0 : 0.0;
    }
  }
  block_sum<3>(v, sred);
  if (threadIdx.x == 0)
    for (int j = 0; j < 3; ++j) part[(size_t)blockIdx.x * kNumPart + j] = v[j];
  if (arrive_last(counter, gridDim.x)) {
    double t[3];
    reduce_partials<3>(part, gridDim.x, t, sred);
    if (threadIdx.x == 0)
      for (int j = 0; j < 3; ++j) out[j] = t[j];
  }
}

// CSR structure: flags[0] += bad rowptr, flags[1] += column out of range,
// flags[2] += unsorted or repeated column within a row.
__global__ __launch_bounds__(kThreads) void k_csr_structure(const int64_t* __restrict__ rowptr,
                                                            const int32_t* __restrict__ col,
                                                            int64_t n, int64_t nnz,
                                                            unsigned* __restrict__ flags) {
  unsigned bad_ptr = 0, bad_col = 0, unsorted = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const int64_t b = rowptr[i], e = rowptr[i + 1];
    if (b < 0 || e < b || e > nnz) {
      ++bad_ptr;
      continue;
    }
    int32_t prev = -1;
    for (int64_t z = b; z < e; ++z) {
      const int32_t cc = col[z];
      if (cc < 0 || cc >= n) ++bad_col;
      if (cc <= prev) ++unsorted;
      prev = cc;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (rowptr[0] != 0 || rowptr[n] != nnz) atomicAdd(&flags[0], 1u);
  }
  if (bad_ptr) atomicAdd(&flags[0], bad_ptr);
  if (bad_col) atomicAdd(&flags[1], bad_col);
  if (unsorted) atomicAdd(&flags[2], unsorted);
}

// Symmetry of a CSR matrix with sorted rows: for every stored (i, j, v) row j must hold
// column i with the same value.  flags[3] += mismatches.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_csr_symmetry(const int64_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ col,
                                                           const T* __restrict__ val, int64_t n,
                                                           unsigned* __restrict__ flags) {
  unsigned bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    for (int64_t z = rowptr[i]; z < rowptr[i + 1]; ++z) {
      const int64_t j = col[z];
      int64_t lo = rowptr[j], hi = rowptr[j + 1] - 1;
      bool found = false;
      while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t cm = col[mid];
        if (cm == i) {
          found = val[mid] == val[z];
          break;
        }
        if (cm < i) lo = mid + 1;
        else hi = mid - 1;
      }
      if (!found) ++bad;
    }
  }
  if (bad) atomicAdd(&flags[3], bad);
}

// Symmetry of a dense n x n matrix (leading dimension ld): workgroup (bx, by), by <= bx,
// stages the 32 x 32 tile at (block row by, block column bx) in LDS and compares it with
// the mirrored tile read row by row.  flags[3] += entries with
// |a_ij - a_ji| > tol max(|a_ij|, |a_ji|) (NaN entries count as mismatches).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dense_symmetry(const T* __restrict__ A, int64_t n,
                                                             int64_t ld, double tol,
                                                             unsigned* __restrict__ flags) {
  if (blockIdx.y > blockIdx.x) return;
  __shared__ T tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  for (int q = ty; q < 32; q += 8) {
    const int64_t i = i0 + q, j = j0 + tx;
    tile[q][tx] = (i < n && j < n) ? A[i * ld + j] : T(0);
  }
  __syncthreads();
  unsigned bad = 0;
  for (int q = ty; q < 32; q += 8) {
    const int64_t j = j0 + q, i = i0 + tx;                    // entry (j, i) of the mirror
    if (i < n && j < n) {
      const double a = (double)A[j * ld + i];
      const double b = (double)tile[tx][q];                    // entry (i, j)
      const double m = fmax(fabs(a), fabs(b));
      if (!(fabs(a - b) <= tol * m)) ++bad;
    }
  }
  if (bad) atomicAdd(&flags[3], bad);
}

template <typename T>
void launch_dense_symmetry(const T* A, int64_t n, int64_t ld, double tol, unsigned* flags,
                           hipStream_t s) {
  const int64_t nt = (n + 31) / 32;
  hipLaunchKernelGGL(k_dense_symmetry<T>, dim3((unsigned)nt, (unsigned)nt), dim3(kThreads), 0, s,
                     A, n, ld, tol, flags);
}
template void launch_dense_symmetry<float>(const float*, int64_t, int64_t, double, unsigned*,
                                           hipStream_t);
template void launch_dense_symmetry<double>(const double*, int64_t, int64_t, double, unsigned*,
                                            hipStream_t);

template <typename T>
void launch_stats2d(const T* x, int64_t rows, int64_t cols, int64_t ld, double* part, double* out,
                    unsigned* counter, hipStream_t s) {
  int64_t nb = (rows * cols + kThreads * 8 - 1) / (kThreads * 8);
  if (nb < 1) nb = 1;
  if (nb > kMaxGrid) nb = kMaxGrid;
  hipLaunchKernelGGL(k_stats2d<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, x, rows, cols, ld,
                     part, out, counter);
}

void launch_csr_structure(const int64_t* rowptr, const int32_t* col, int64_t n, int64_t nnz,
                          unsigned* flags, hipStream_t s) {
  int64_t nb = (n + kThreads - 1) / kThreads;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_csr_structure, dim3((unsigned)nb), dim3(kThreads), 0, s, rowptr, col, n,
                     nnz, flags);
}

template <typename T>
void launch_csr_symmetry(const int64_t* rowptr, const int32_t* col, const T* val, int64_t n,
                         unsigned* flags, hipStream_t s) {
  int64_t nb = (n + kThreads - 1) / kThreads;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_csr_symmetry<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, rowptr, col,
                     val, n, flags);
}

template void launch_stats2d<float>(const float*, int64_t, int64_t, int64_t, double*, double*,
                                    unsigned*, hipStream_t);
template void launch_stats2d<double>(const double*, int64_t, int64_t, int64_t, double*, double*,
                                     unsigned*, hipStream_t);
template void launch_csr_symmetry<float>(const int64_t*, const int32_t*, const float*, int64_t,
                                         unsigned*, hipStream_t);
template void launch_csr_symmetry<double>(const int64_t*, const int32_t*, const double*, int64_t,
                                          unsigned*, hipStream_t);

// Solve start: clear the device state, store ||A||^2 and the start time.
__global__ void k_reset_state(State* st, double normA2) {
  if (threadIdx.x == 0) {
    State z = {};
    z.normA2 = normA2;
    z.t0 = wall_clock64();
    *st = z;
  }
}
void launch_reset_state(State* st, double normA2, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, st, normA2);
}

// Batched solve start: one State per instance.
__global__ void k_breset(State* states, const BInst* inst, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) {
    State z = {};
    z.normA2 = inst[i].normA2;
    z.t0 = wall_clock64();
    states[i] = z;
  }
}
void launch_breset(State* states, const BInst* inst, int ninst, hipStream_t s) {
  hipLaunchKernelGGL(k_breset, dim3((ninst + 63) / 64), dim3(64), 0, s, states, inst, ninst);
}

// flag = 1 when every instance of a batched solve is done.
__global__ __launch_bounds__(256) void k_all_done(const State* states, int ninst, int32_t* flag) {
  __shared__ int s_any;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  int open = 0;
  for (int i = threadIdx.x; i < ninst; i += blockDim.x) open |= states[i].done == 0;
  if (open) s_any = 1;
  __syncthreads();
  if (threadIdx.x == 0) flag[0] = s_any ? 0 : 1;
}
void launch_all_done(const State* states, int ninst, int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_all_done, dim3(1), dim3(256), 0, s, states, ninst, flag);
}

// Flat BF16 split of count floats.
__device__ __forceinline__ uint16_t bf16_rne_v(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__global__ __launch_bounds__(kThreads) void k_split_flat(const float* __restrict__ x, int64_t count,
                                                         uint16_t* __restrict__ hi,
                                                         uint16_t* __restrict__ lo) {
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * kThreads) {
    const float a = x[e];
    const uint16_t h = bf16_rne_v(a);
    hi[e] = h;
    lo[e] = bf16_rne_v(a - __uint_as_float((uint32_t)h << 16));
  }
}
void launch_split_flat(const float* x, int64_t count, uint16_t* hi, uint16_t* lo, hipStream_t s) {
  int64_t nb = (count + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_split_flat, dim3((unsigned)nb), dim3(kThreads), 0, s, x, count, hi, lo);
}

}  // namespace snmf
