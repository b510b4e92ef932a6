// Small kernels of the SNMPBB hot path: the Gram matrix G = P^T P, its spectral norm
// rho = ||G||_2 (the first-projection scale of Algorithm 1, Section 2.4), ||A||_F^2 with
// input validation counts, and the BF16 hi/lo split of the precision form.
#include "common.hpp"
#include "kernels.hpp"

namespace snmf {

// ----------------------------------------------------------------------------- Gram
// Each workgroup forms the FP64 Gram of a contiguous slab of rows of P; the last
// workgroup adds the slabs in block order (deterministic) and writes G in FP64 and in
// the iterate type.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gram(const T* __restrict__ P, int64_t n, int r,
                                                   int64_t rows_per_block,
                                                   double* __restrict__ part,
                                                   double* __restrict__ G64, T* __restrict__ GT,
                                                   unsigned* __restrict__ counter,
                                                   const State* __restrict__ st) {
  if (st->done) return;
  constexpr int TR = 32;
  __shared__ double sP[TR][kMaxRank + 1];
  const int rr = r * r;
  double acc[kMaxRank * kMaxRank / kThreads];
  constexpr int NE = kMaxRank * kMaxRank / kThreads;
#pragma unroll
  for (int i = 0; i < NE; ++i) acc[i] = 0.0;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = rb + rows_per_block < n ? rb + rows_per_block : n;
  for (int64_t t0 = rb; t0 < re; t0 += TR) {
    __syncthreads();
    for (int e = threadIdx.x; e < TR * r; e += kThreads) {
      const int i = e / r, c = e - i * r;
      const int64_t row = t0 + i;
      sP[i][c] = row < re ? (double)P[row * r + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = threadIdx.x + q * kThreads;
      if (e < rr) {
        const int a = e / r, b = e - a * r;
        double s = acc[q];
#pragma unroll 8
        for (int i = 0; i < TR; ++i) s = __builtin_fma(sP[i][a], sP[i][b], s);
        acc[q] = s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = threadIdx.x + q * kThreads;
    if (e < rr) part[(size_t)blockIdx.x * rr + e] = acc[q];
  }
  if (arrive_last(counter, gridDim.x)) {
    for (int e = threadIdx.x; e < rr; e += kThreads) {
      double s = 0.0;
      for (unsigned b = 0; b < gridDim.x; ++b) s += part[(size_t)b * rr + e];
      G64[e] = s;
      GT[e] = (T)s;
    }
  }
}

// ----------------------------------------------------------------------------- rho
// Largest eigenvalue of the symmetric positive semidefinite r x r matrix G (r <= 64),
// computed by one wavefront: Lanczos from the all-ones vector with full
// re-orthogonalisation (two classical Gram-Schmidt passes), then bisection with Sturm
// counts on the tridiagonal matrix, 64 trial shifts per round.  G >= 0 elementwise (a
// Gram of a nonnegative block), so its Perron vector is nonnegative and the all-ones
// start has a nonzero component along it.  Also resets the per-half-step scalars.
__global__ __launch_bounds__(kWave) void k_rho(const double* __restrict__ G, int r,
                                                State* __restrict__ st) {
  if (st->done) return;
  constexpr int LD = kMaxRank + 1;
  __shared__ double sQ[kMaxRank * LD];
  __shared__ double sv[kMaxRank];
  __shared__ double sa[kMaxRank], sb[kMaxRank];
  const int i = threadIdx.x;
  double grow[kMaxRank];
  double gn2 = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxRank; ++k) {
    grow[k] = (i < r && k < r) ? G[i * r + k] : 0.0;
    gn2 += grow[k] * grow[k];
  }
  const double gnorm = sqrt(wave_sum(gn2));
  double q = i < r ? 1.0 / sqrt((double)r) : 0.0;
  double qprev = 0.0, bprev = 0.0;
  int m = 0;
  for (int j = 0; j < r; ++j) {
    sQ[i * LD + j] = q;
    sv[i] = q;
    __syncthreads();
    double w = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxRank; ++k) w = __builtin_fma(grow[k], sv[k], w);
    const double a = wave_sum(w * q);
    w -= a * q + bprev * qprev;
    for (int pass = 0; pass < 2; ++pass) {
      __syncthreads();
      sv[i] = w;
      __syncthreads();
      double cj = 0.0;
      if (i <= j)
        for (int k = 0; k < r; ++k) cj = __builtin_fma(sQ[k * LD + i], sv[k], cj);
      __syncthreads();
      sv[i] = i <= j ? cj : 0.0;
      __syncthreads();
      double s = 0.0;
      for (int jj = 0; jj <= j; ++jj) s = __builtin_fma(sQ[i * LD + jj], sv[jj], s);
      w -= s;
    }
    const double b = sqrt(wave_sum(w * w));
    if (i == 0) {
      sa[j] = a;
      sb[j] = b;
    }
    m = j + 1;
    if (!(b > 1e-15 * gnorm)) break;
    qprev = q;
    q = w / b;
    bprev = b;
    __syncthreads();
  }
  __syncthreads();
  // bounds for the largest eigenvalue of T = tridiag(sb, sa, sb)
  double lo = -1e300, hi = -1e300;
  for (int k = 0; k < m; ++k) {
    const double off = (k > 0 ? fabs(sb[k - 1]) : 0.0) + (k + 1 < m ? fabs(sb[k]) : 0.0);
    lo = fmax(lo, sa[k]);
    hi = fmax(hi, sa[k] + off);
  }
  for (int round = 0; round < 40 && hi - lo > 2.0 * 2.220446049250313e-16 * fabs(hi); ++round) {
    const double x = lo + (hi - lo) * (double)(i + 1) / (double)(kWave + 1);
    // Sturm count: number of eigenvalues of T smaller than x (negative LDL^T pivots)
    int cnt = 0;
    double d = 1.0;
    for (int k = 0; k < m; ++k) {
      const double b2 = k > 0 ? sb[k - 1] * sb[k - 1] : 0.0;
      d = (sa[k] - x) - (k > 0 ? b2 / d : 0.0);
      if (fabs(d) < 1e-300) d = -1e-300;
      cnt += d < 0.0;
    }
    // lanes with cnt == m (x above every eigenvalue) form a suffix of the shifts
    const unsigned long long above = __ballot(cnt == m);
    const int first_above = above ? __ffsll((long long)above) - 1 : kWave;
    const double nlo = first_above > 0
                           ? lo + (hi - lo) * (double)first_above / (double)(kWave + 1)
                           : lo;
    const double nhi = first_above < kWave
                           ? lo + (hi - lo) * (double)(first_above + 1) / (double)(kWave + 1)
                           : hi;
    lo = nlo;
    hi = nhi;
  }
  if (i == 0) {
    const double rho = 0.5 * (lo + hi);
    st->rho = rho;
    st->alpha = 1.0 / rho;
    st->e = 0.0;
    st->hs_done = 0;
    st->k = 0;
    if (!(rho > 0.0) || !(rho < 1e308)) {
      st->status = 9;  // SNMF_E_BREAKDOWN
      st->done = 1;
    }
  }
}

// ----------------------------------------------------------------------------- ||A||^2
// Sum of squares in FP64 plus counts of negative and non-finite entries of an array of
// N values; the last workgroup writes {sum, negatives, nonfinite} to out.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_norm2(const T* __restrict__ x, int64_t N,
                                                    double* __restrict__ part,
                                                    double* __restrict__ out,
                                                    unsigned* __restrict__ counter) {
  __shared__ double sred[kThreads / kWave * 3];
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kThreads) {
    const double a = (double)x[i];
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

// ----------------------------------------------------------------------------- BF16 split
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// hi = rne(a), lo = rne(a - hi): rows of A (n x lda, FP32) into n x ldb BF16 arrays whose
// columns n..ldb-1 are zero.
__global__ __launch_bounds__(kThreads) void k_split_rows(const float* __restrict__ A, int64_t n,
                                                         int64_t lda, int64_t ldb,
                                                         uint16_t* __restrict__ hi,
                                                         uint16_t* __restrict__ lo) {
  const int64_t total = n * ldb;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kThreads) {
    const int64_t i = e / ldb, j = e - i * ldb;
    const float a = j < n ? A[i * lda + j] : 0.0f;
    const uint16_t h = bf16_rne(a);
    hi[e] = h;
    lo[e] = bf16_rne(a - bf16_to_f32(h));
  }
}

// P (n x r, FP32) -> Pt_hi, Pt_lo (r x ldp, BF16, transposed, zero beyond n).
__global__ __launch_bounds__(kThreads) void k_split_pt(const float* __restrict__ P, int64_t n, int r,
                                                       int64_t ldp, uint16_t* __restrict__ hi,
                                                       uint16_t* __restrict__ lo,
                                                       const State* __restrict__ st) {
  if (st->done) return;
  const int64_t total = (int64_t)r * ldp;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kThreads) {
    const int64_t m = e / ldp, k = e - m * ldp;
    const float a = k < n ? P[k * r + m] : 0.0f;
    const uint16_t h = bf16_rne(a);
    hi[e] = h;
    lo[e] = bf16_rne(a - bf16_to_f32(h));
  }
}

// ----------------------------------------------------------------------------- launchers
template <typename T>
void launch_gram(const T* P, int64_t n, int r, double* part, int nblk, double* G64, T* GT,
                 unsigned* counter, const State* st, hipStream_t s) {
  int64_t rpb = (n + nblk - 1) / nblk;
  hipLaunchKernelGGL(k_gram<T>, dim3(nblk), dim3(kThreads), 0, s, P, n, r, rpb, part, G64, GT,
                     counter, st);
}
template void launch_gram<float>(const float*, int64_t, int, double*, int, double*, float*,
                                 unsigned*, const State*, hipStream_t);
template void launch_gram<double>(const double*, int64_t, int, double*, int, double*, double*,
                                  unsigned*, const State*, hipStream_t);

void launch_rho(const double* G, int r, State* st, hipStream_t s) {
  hipLaunchKernelGGL(k_rho, dim3(1), dim3(kWave), 0, s, G, r, st);
}

template <typename T>
void launch_norm2(const T* x, int64_t N, double* part, double* out, unsigned* counter,
                  hipStream_t s) {
  int64_t nb = (N + kThreads * 8 - 1) / (kThreads * 8);
  if (nb < 1) nb = 1;
  if (nb > kMaxGrid) nb = kMaxGrid;
  hipLaunchKernelGGL(k_norm2<T>, dim3((unsigned)nb), dim3(kThreads), 0, s, x, N, part, out,
                     counter);
}
template void launch_norm2<float>(const float*, int64_t, double*, double*, unsigned*, hipStream_t);
template void launch_norm2<double>(const double*, int64_t, double*, double*, unsigned*,
                                   hipStream_t);

void launch_split_rows(const float* A, int64_t n, int64_t lda, int64_t ldb, uint16_t* hi,
                       uint16_t* lo, hipStream_t s) {
  int64_t nb = (n * ldb + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_split_rows, dim3((unsigned)nb), dim3(kThreads), 0, s, A, n, lda, ldb, hi,
                     lo);
}

void launch_split_pt(const float* P, int64_t n, int r, int64_t ldp, uint16_t* hi, uint16_t* lo,
                     const State* st, hipStream_t s) {
  int64_t nb = ((int64_t)r * ldp + kThreads - 1) / kThreads;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_split_pt, dim3((unsigned)nb), dim3(kThreads), 0, s, P, n, r, ldp, hi, lo,
                     st);
}

}  // namespace snmf
