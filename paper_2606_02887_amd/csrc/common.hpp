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

constexpr int kMaxInner = 64;         // largest number of inner iterations per half-step
constexpr int kInnerGrid = 1024;       // workgroups of the row-tile kernels (re-reduced)
constexpr int kSketchMaxW = 128;     // widest sketch (rank + oversampling) of the range finder
constexpr int kKnnMaxDim = 64;       // largest point dimension of the K-nearest-neighbour search
constexpr int kKnnMaxK = 64;         // largest K of the K-nearest-neighbour search

// Counters of the setup kernels that finish a reduction in their last workgroup.
enum Counter { C_GRAM = 0, C_INIT, C_STEP1, C_STEP2, C_NORM, C_LAI, C_LAPRED, C_MISC, C_COUNT };

// Scalars of the iteration that live on the device for the whole solve.
// Hot-path kernels never finish a reduction inside themselves: each writes FP64 partial
// sums per workgroup, and the NEXT kernel re-reduces those partials in every workgroup in
// the same fixed order, so all workgroups derive bit-identical scalars (line-search beta,
// BB step, stop decisions) without atomics or device-scope fences.  Workgroup 0 stores
// the scalars here for later kernels.  A kernel never reads a field that it writes: the
// per-inner-iteration values are indexed by the inner iteration k.
struct State {
  double rho;                  // ||P^T P||_2 of the current half-step
  double e[kMaxInner + 1];     // e_k = F_k - f(X_k)
  double alpha[kMaxInner + 1]; // BB step used by inner iteration k
  double beta[kMaxInner + 1];  // accepted backtracking factor of inner iteration k
  int32_t stop[kMaxInner + 1]; // the half-step ended before inner iteration k (S = 0)
  int32_t pad1;
  double normA2;               // ||A||_F^2
  double m_CP;                 // <C, P> of the last H-step (C = A W + lam W, P = W)
  double last_ss, last_sy;     // BB scalars of the last completed update
  double res_last, resww_last, sym_last, pg_last, f_last;
  uint64_t t_hstep;            // device clock when the last H-step update finished
  uint64_t t0;                 // device clock at solve start
  uint64_t t_conv;             // device ticks from t0 to the H-step that met the target
  int32_t pending;             // an H-step finished; its monitor record is still open
  int32_t snap_pending;        // W-step init's copy of pending
  int32_t outer;               // completed (recorded) outer iterations
  int32_t snap_outer;          // W-step init's copy of outer
  int32_t done;                // the solve is finished: every later kernel returns at once
  int32_t status;              // 0 ok, otherwise a snmf_status breakdown code
  int32_t converged_at;        // first outer iteration meeting the target (1-based), 0 none
  int32_t trace_len;
  int64_t ls_evals, ls_exhausted, inner_total;
};

// Scalar parameters passed by value to every kernel that needs them.
struct KParams {
  double lam, gamma, eta, theta, phi, amin, amax, shrink, target;
  int32_t max_ls, relaxed, project, max_outer;
};

// Batched solves: many independent instances (problem g, restart s), each an n x r block
// stored contiguously (instance-major) in shared batch buffers.  Device table entry:
struct BInst {
  int64_t off;     // element offset of the instance's n x r arrays
  int64_t n;
  int32_t r;
  int32_t blk0;    // inner kernels: first workgroup of the instance in its class launch
  int32_t nblk;    //   and its number of workgroups (<= kInnerGrid)
  int32_t part0;   //   first row of its partial sums
  int64_t goff;    // element offset of its r x r Gram (FP64 and iterate-type copies)
  int64_t gpoff;   // element offset of its Gram partials (gnb x r*r)
  int32_t gblk0;   // Gram: first workgroup, number of workgroups, rows per workgroup
  int32_t gnb;
  int64_t grpb;
  double lam;      // its penalty lambda
  double normA2;   // ||A||_F^2 of its problem
  int32_t prob;    // index of its problem
  int32_t restart;
};

// One problem of a batched CSR solve: its restarts are the instances inst0 .. inst0+S-1,
// stored one after another (restart s at element offset off0 + s n r).
struct BGraph {
  const int64_t* rowptr;
  const int32_t* col;
  const void* val;
  const double* deg;  // warm start of dense problems: row sums A 1 (CSR: nullptr)
  int64_t n;
  int64_t off0;
  int32_t r, S;
  int32_t blk0, nblk;  // workgroups of the stacked SpMM launch
  int32_t inst0;
  int32_t pad;
};

// Passed by value to the inner kernels; blk_inst == nullptr means a single solve whose
// pointers, sizes and State come from the kernel arguments.
struct BMap {
  const int32_t* blk_inst;  // workgroup of the launch -> instance
  const BInst* inst;
  State* states;            // one State per instance
  double* traces;           // per-instance traces of trace_stride doubles (nullable)
  int64_t trace_stride;
};

// Cross-lane data movement with DPP (GFX9 encoding).  Lanes whose source is outside the
// row read 0 (bound control), masked-off rows keep 0.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave in a fixed pattern (row shifts 1, 2, 4, 8, then row
// broadcasts 15 and 31); the result is wave-uniform.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0x111>(v);        // row_shr:1
  v += dpp_d<0x112>(v);        // row_shr:2
  v += dpp_d<0x114>(v);        // row_shr:4
  v += dpp_d<0x118>(v);        // row_shr:8
  v += dpp_d<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return readlane_d(v, 63);
}

// Sum over aligned groups of 4 lanes; every lane of the group gets the same bits.
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_d<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);         // quad_perm [2,3,0,1]
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

// Block sums of K <= 16 doubles per thread for the row-tile kernels, in a fixed order that
// does not depend on K: the values go to LDS (stage, kStage doubles), thread 16 s + q adds
// the values of threads 16 u + q of slot s (u = 0..15, even and odd u in two chains), and
// the 16 threads of slot s -- one DPP row -- add their results with row shifts, so lane
// q = 15 holds the total.  Three times faster than a wave reduction per value followed by a
// cross-wave one (0.5 against 1.5 us for 13 values).  slot_sum returns that lane's total
// (and sets s); the callers below broadcast or store it.
constexpr int kStage = 16 * kThreads + 16;
template <int K>
__device__ __forceinline__ double slot_sum(const double (&v)[K], double* stage, int& s) {
  static_assert(K >= 1 && K <= 16, "at most 16 slots");
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < K; ++j) stage[j * kThreads + t] = v[j];
  __syncthreads();
  s = t >> 4;
  const int q = t & 15;
  double a = 0.0;
  if (s < K) {
    double b = 0.0;
#pragma unroll
    for (int u = 0; u < 16; u += 2) {
      a += stage[s * kThreads + u * 16 + q];
      b += stage[s * kThreads + (u + 1) * 16 + q];
    }
    a += b;
    a += dpp_d<0x111>(a);  // row_shr:1
    a += dpp_d<0x112>(a);  // row_shr:2
    a += dpp_d<0x114>(a);  // row_shr:4
    a += dpp_d<0x118>(a);  // row_shr:8
  }
  return a;
}
// Totals in every thread.  The stage may alias buffers no wave reads any more.
template <int K>
__device__ __forceinline__ void block_sum_wide(double (&v)[K], double* stage) {
  int s;
  const double a = slot_sum<K>(v, stage, s);
  if (s < K && (threadIdx.x & 15) == 15) stage[16 * kThreads + s] = a;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < K; ++j) v[j] = stage[16 * kThreads + j];
}
// Totals handed to emit(slot, total), one thread per slot; starts with a barrier, so the
// stage may alias tile buffers that other waves were still reading.
template <int K, typename F>
__device__ __forceinline__ void block_sum_emit(const double (&v)[K], double* stage, F&& emit) {
  __syncthreads();
  int s;
  const double a = slot_sum<K>(v, stage, s);
  if (s < K && (threadIdx.x & 15) == 15) emit(s, a);
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
