// Shared device-side definitions of the SNMPBB HIP library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snmf {

constexpr int kThreads = 256;          // threads per workgroup of the row-tile kernels
constexpr int kWave = 64;
constexpr int kMaxRank = 64;           // largest factorisation rank r of one problem
constexpr int kMaxGrid = 1024;         // row-tile kernels use at most this many workgroups
constexpr int kNumPart = 16;           // FP64 partial sums per workgroup
constexpr int kTraceFields = 10;       // doubles per outer-iteration trace record

// Counters for the "last workgroup finishes the reduction" pattern; one per kernel kind
// so that kernels running concurrently on two streams never share one.
enum Counter { C_GRAM = 0, C_INIT, C_STEP1, C_STEP2, C_NORM, C_LAI, C_LAPRED, C_MISC, C_COUNT };

// Scalars of the iteration that live on the device for the whole solve.  Only the last
// workgroup of a kernel writes them; every other access is a read at kernel start.
struct State {
  // half-step
  double rho;          // ||P^T P||_2
  double alpha;        // BB step for the next inner iteration
  double beta;         // accepted backtracking factor of the current inner iteration
  double e;            // F_k - f(X_k) >= 0 (nonmonotone reference minus objective)
  double ss, sy, gs;   // <S,S>, <S,Y>, <g_k,S> of the last update
  double delta, q, dZ; // <grad f(Z),D>, <D,(G+lam I)D>[+gam<D,LD>], f(Z)-f(X_k)
  double nd2;          // ||D||^2
  double normA2;       // ||A||_F^2
  // monitor staging (written by the H-step, consumed at the next W-step start)
  double m_CX, m_PX, m_XmP2, m_pgH2, m_CP, m_PP, m_XLX;
  double pgW2;         // ||min(W, grad_W)||^2 at the last completed outer iteration
  double res_last, resww_last, sym_last, pg_last, f_last;
  uint64_t t_hstep;    // constant-rate device clock at the end of the last H-step
  uint64_t t0;         // device clock at solve start
  int32_t pending;     // an H-step finished and its monitor record awaits the next W-step
  int32_t pad0;
  int32_t hs_done;     // current half-step stopped early (S = 0)
  int32_t done;        // solve finished: every later kernel returns at once
  int32_t k;           // inner iteration index in the current half-step
  int32_t outer;       // completed outer iterations
  int32_t status;      // 0 ok, otherwise a snmf_status breakdown code
  int32_t converged_at;// first outer iteration whose residual met the target (1-based), 0 none
  int32_t trace_len;
  int32_t is_hstep;
  int64_t ls_evals, ls_exhausted, inner_total;
};

// Scalar parameters passed by value to every kernel that needs them.
struct KParams {
  double lam, gamma, eta, theta, phi, amin, amax, shrink, target;
  int32_t max_ls, relaxed, project, max_outer;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Deterministic block sum of K doubles per thread; result valid in every thread.
// sred must hold kThreads/kWave * K doubles.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* sred) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  constexpr int nw = kThreads / kWave;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double s = wave_sum(v[j]);
    if (lane == 0) sred[wid * K + j] = s;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < nw; ++w) s += sred[w * K + j];
    v[j] = s;
  }
  __syncthreads();
}

// Release this block's partials; returns true in every thread of the last block to
// arrive (which then sees all partials).  The last block resets the counter.
__device__ __forceinline__ bool arrive_last(unsigned int* counter, unsigned int nblocks) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int prev = atomicAdd(counter, 1u);
    s_last = (prev == nblocks - 1) ? 1 : 0;
    if (s_last) atomicExch(counter, 0u);
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __threadfence();
  return last;
}

// Fixed-order reduction of nb rows of K partials (row-major [nb][kNumPart]) by one
// block; the result is valid in every thread.
template <int K>
__device__ __forceinline__ void reduce_partials(const double* part, int nb, double (&out)[K],
                                                double* sred) {
#pragma unroll
  for (int j = 0; j < K; ++j) out[j] = 0.0;
  for (int b = threadIdx.x; b < nb; b += kThreads) {
    const double* p = part + (size_t)b * kNumPart;
#pragma unroll
    for (int j = 0; j < K; ++j) out[j] += p[j];
  }
  block_sum<K>(out, sred);
}


template <typename T> __device__ __forceinline__ T relu(T x) { return x > T(0) ? x : T(0); }

}  // namespace snmf
