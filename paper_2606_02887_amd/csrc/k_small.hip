// Small kernels of the SNMPBB hot path: the Gram matrix G = P^T P, its spectral norm
// rho = ||G||_2 (the first-projection scale of Algorithm 1, Section 2.4), ||A||_F^2 with
// input validation counts, and the BF16 hi/lo split of the precision form.
#include "common.hpp"
#include "kernels.hpp"
#include "rho.hpp"

namespace snmf {

// ----------------------------------------------------------------------------- Gram
// Each workgroup forms the FP64 Gram of a contiguous slab of rows of P on the FP64 matrix
// cores; a second kernel adds the slabs in block order (deterministic) and writes G in
// FP64 and in the iterate type.  The slab is cut into k-steps of four rows, dealt to the
// four wavefronts in turn (k-step j to wavefront j % 4).  RPG, the rank rounded up to a
// power of two, gives NB = max(1, RPG/16) column blocks of 16; a wavefront accumulates the
// NB (NB + 1) / 2 tiles (qa <= qb) of the upper block triangle with
//   D(qa, qb) += A B,  A = P[k rows][16 qa + 0..15]^T (16 x 4),  B = P[k rows][16 qb + 0..15],
// where lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16], both the value of row
// l / 16 of the k-step and column 16 q + l % 16, and holds D[l / 16 + 4 v][l % 16].
// The four wavefront sums are added as (w0 + w1) + (w2 + w3) in LDS, and each entry a <= b
// is written to both (a, b) and (b, a), so the slab Gram is exactly symmetric.
typedef double gd4 __attribute__((ext_vector_type(4)));

template <int RPG>
struct GramCfg {
  static constexpr int NB = RPG >= 16 ? RPG / 16 : 1;  // 16-column blocks
  static constexpr int NT = NB * (NB + 1) / 2;         // upper-triangle tiles
  static constexpr int U = 4;                          // k-steps per batch of loads
};

template <int NB>
__device__ __forceinline__ constexpr int gram_tile(int qa, int qb) {
  // index of tile (qa, qb), qa <= qb, in row-major order of the upper triangle
  return qa * NB - qa * (qa - 1) / 2 + (qb - qa);
}

template <typename T, int RPG>
__device__ __forceinline__ void gram_slab(const T* __restrict__ P, int r, int64_t rb, int64_t re,
                                          double* __restrict__ out) {
  typedef GramCfg<RPG> C;
  constexpr int NB = C::NB, NT = C::NT, U = C::U;
  __shared__ __attribute__((aligned(16))) double sacc[2][NT][4][kWave];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kr = lane >> 4, c16 = lane & 15;
  gd4 acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = gd4{0.0, 0.0, 0.0, 0.0};
  const int64_t nst = (re - rb + 3) / 4;  // k-steps of the slab
  // column of block q: clamped to a valid one, the value masked when out of range
  bool cok[NB];
  int ccl[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int cc = 16 * q + c16;
    cok[q] = cc < r;
    ccl[q] = cc < r ? cc : r - 1;
  }
  // A batch holds the raw values of U k-steps (every address valid: rows past the slab
  // clamped) and a row-in-range flag per k-step; the conversion to FP64 and the masking
  // wait until the MFMAs.  (Masking at the load made the compiler branch around each
  // load and wait for it inside the branch, one memory round trip per k-step.)
  auto load = [&](T (&x)[U][NB], bool (&ok)[U], int64_t j0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = rb + 4 * (j0 + 4 * u) + kr;
      ok[u] = row < re;
      const int64_t rc = row < re ? row : re - 1;
#pragma unroll
      for (int q = 0; q < NB; ++q) x[u][q] = P[rc * r + ccl[q]];
    }
  };
  auto mma = [&](const T (&x)[U][NB], const bool (&ok)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double xd[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) xd[q] = (ok[u] && cok[q]) ? (double)x[u][q] : 0.0;
#pragma unroll
      for (int qa = 0; qa < NB; ++qa)
#pragma unroll
        for (int qb = qa; qb < NB; ++qb) {
          const int tq = gram_tile<NB>(qa, qb);
          acc[tq] = __builtin_amdgcn_mfma_f64_16x16x4f64(xd[qa], xd[qb], acc[tq], 0, 0, 0);
        }
    }
  };
  // wavefront `wave` takes k-steps wave, wave + 4, ...; batches of U of them, two in
  // flight.  The k-steps past the slab load clamped rows and contribute exact zeros, so
  // every load and MFMA of the loop is unconditional: a conditional consumer lets the
  // compiler sink that batch's loads next to their MFMAs, where their latency is exposed.
  const int64_t mine = nst > wave ? (nst - wave + 3) / 4 : 0;
  const int64_t nbat = (mine + U - 1) / U;
  T xa[U][NB], xb[U][NB];
  bool oa[U], ob[U];
  if (nbat > 0) load(xa, oa, wave);
  for (int64_t bt = 0; bt < nbat; bt += 2) {
    const int64_t j0 = wave + 4 * U * bt;
    load(xb, ob, j0 + 4 * U);
    mma(xa, oa);
    load(xa, oa, j0 + 8 * U);
    mma(xb, ob);
  }
  // (w0 + w1) + (w2 + w3): odd waves park their sums, even waves add them; wave 2 parks
  // its pair sum and wave 0 adds it
  auto put = [&](int slot) {
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) sacc[slot][q][v][lane] = acc[q][v];
  };
  auto add = [&](int slot) {
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[q][v] += sacc[slot][q][v][lane];
  };
  if (wave & 1) put(wave >> 1);
  __syncthreads();
  if (!(wave & 1)) add(wave >> 1);
  __syncthreads();
  if (wave == 2) put(0);
  __syncthreads();
  if (wave == 0) {
    add(0);
#pragma unroll
    for (int qa = 0; qa < NB; ++qa)
#pragma unroll
      for (int qb = qa; qb < NB; ++qb) {
        const int tq = gram_tile<NB>(qa, qb);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 16 * qa + kr + 4 * v, b = 16 * qb + c16;
          if (a < r && b < r && (qa < qb || a <= b)) {
            out[a * r + b] = acc[tq][v];
            out[b * r + a] = acc[tq][v];
          }
        }
      }
  }
}

template <typename T, int RPG>
__global__ __launch_bounds__(kThreads) void k_gram(const T* __restrict__ P, int64_t n, int r,
                                                   int64_t rows_per_block,
                                                   double* __restrict__ part,
                                                   const State* __restrict__ st) {
  if (st->done) return;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = rb + rows_per_block < n ? rb + rows_per_block : n;
  gram_slab<T, RPG>(P, r, rb, re, part + (size_t)blockIdx.x * r * r);
}

// Batched: the workgroups of one rank class; workgroup -> (instance, slab) through
// gblk_inst.  The same slabs as a single solve of that instance, so G is bitwise equal.
template <typename T, int RPG>
__global__ __launch_bounds__(kThreads) void k_bgram(const T* __restrict__ P,
                                                    const int32_t* __restrict__ gblk_inst,
                                                    const BInst* __restrict__ inst,
                                                    const State* __restrict__ states,
                                                    double* __restrict__ gpart) {
  const int i = gblk_inst[blockIdx.x];
  const BInst* d = inst + i;
  if (states[i].done) return;
  const int j = (int)blockIdx.x - d->gblk0;
  const int64_t rb = (int64_t)j * d->grpb;
  const int64_t re = rb + d->grpb < d->n ? rb + d->grpb : d->n;
  gram_slab<T, RPG>(P + d->off, d->r, rb, re, gpart + d->gpoff + (size_t)j * d->r * d->r);
}

// Sum over the slabs b = q, q + 4, q + 8, ... (in increasing b) of entry e; the Gram is
// (s_0 + s_1) + s_2 + s_3, the same order in the single and the batched reduction.
__device__ __forceinline__ double gram_sum4(const double* __restrict__ part, int nb, int rr, int e,
                                           int q) {
  double s = 0.0;
  int b = q;
  // sixteen of this thread's slabs per round trip, added in slab order
  for (; b + 60 < nb; b += 64) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = part[(size_t)(b + 4 * u) * rr + e];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += v[u];
  }
  for (; b + 12 < nb; b += 16) {
    const double v0 = part[(size_t)b * rr + e], v1 = part[(size_t)(b + 4) * rr + e];
    const double v2 = part[(size_t)(b + 8) * rr + e], v3 = part[(size_t)(b + 12) * rr + e];
    s += v0;
    s += v1;
    s += v2;
    s += v3;
  }
  for (; b < nb; b += 4) s += part[(size_t)b * rr + e];
  return s;
}

// 64 entries per workgroup, four threads per entry.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gram_reduce(const double* __restrict__ part, int nb,
                                                          int rr, double* __restrict__ G64,
                                                          T* __restrict__ GT,
                                                          const State* __restrict__ st) {
  if (st->done) return;
  __shared__ double sq[4][64];
  const int e = blockIdx.x * 64 + (threadIdx.x & 63), q = threadIdx.x >> 6;
  sq[q][threadIdx.x & 63] = e < rr ? gram_sum4(part, nb, rr, e, q) : 0.0;
  __syncthreads();
  if (q == 0 && e < rr) {
    const int t = threadIdx.x;
    const double s = ((sq[0][t] + sq[1][t]) + sq[2][t]) + sq[3][t];
    G64[e] = s;
    GT[e] = (T)s;
  }
}

// Batched: workgroups (instance, y) add the Gram slabs of elements y kThreads + t (stride
// gridDim.y kThreads) in the order above.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bgram_reduce(const BInst* __restrict__ inst,
                                                           const State* __restrict__ states,
                                                           const double* __restrict__ gpart,
                                                           double* __restrict__ G64,
                                                           T* __restrict__ GT) {
  const int i = blockIdx.x;
  const BInst* d = inst + i;
  if (states[i].done) return;
  const int rr = d->r * d->r;
  const double* part = gpart + d->gpoff;
  for (int e = blockIdx.y * kThreads + threadIdx.x; e < rr; e += gridDim.y * kThreads) {
    const double s = ((gram_sum4(part, d->gnb, rr, e, 0) + gram_sum4(part, d->gnb, rr, e, 1)) +
                      gram_sum4(part, d->gnb, rr, e, 2)) +
                     gram_sum4(part, d->gnb, rr, e, 3);
    G64[d->goff + e] = s;
    GT[d->goff + e] = (T)s;
  }
}

// ----------------------------------------------------------------------------- rho
// rho = ||G||_2 with the body in rho.hpp (Lanczos, then division-free multisection).
__global__ __launch_bounds__(kThreads) void k_rho(const double* __restrict__ G, int r,
                                                  State* __restrict__ st) {
  if (st->done) return;
  rho_body(G, r, st);
}

// Batched: one workgroup per instance.
__global__ __launch_bounds__(kThreads) void k_brho(const BInst* __restrict__ inst,
                                                   State* __restrict__ states,
                                                   const double* __restrict__ G64) {
  const int i = blockIdx.x;
  if (states[i].done) return;
  rho_body(G64 + inst[i].goff, inst[i].r, states + i);
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

typedef unsigned short u16x8s __attribute__((ext_vector_type(8)));

// The P factors of S restarts (S consecutive n x r FP32 blocks) -> Pt_hi, Pt_lo
// ((S r) x ldp BF16, row s r + m = column m of block s, zero beyond n).  A workgroup
// transposes a 64 (k) x 64 (stacked column) tile through LDS, so the reads (rows of P)
// and the writes (rows of Pt) are both contiguous.
//
// Grid: ntile = (ldp / 64) x ceil(S r / 64) tile workgroups, then (Grho set) S more that
// compute rho of restart s from its FP64 Gram at Grho + s r^2 beside the short tiles.
__global__ __launch_bounds__(kThreads) void k_split_pt_stack(const float* __restrict__ P,
                                                             int64_t n, int r, int S, int64_t ldp,
                                                             uint16_t* __restrict__ hi,
                                                             uint16_t* __restrict__ lo,
                                                             State* __restrict__ st,
                                                             const double* __restrict__ Grho) {
  const int64_t nkx = ldp / 64, ntile = nkx * (((int64_t)S * r + 63) / 64);
  if ((int64_t)blockIdx.x >= ntile) {
    const int s = (int)((int64_t)blockIdx.x - ntile);
    __builtin_amdgcn_s_setprio(3);  // rho sets this launch's length: issue priority
    if (!st[s].done) rho_body(Grho + (int64_t)s * r * r, r, st + s);
    return;
  }
  bool all = true;
  for (int i = 0; i < S; ++i)
    if (!st[i].done) all = false;
  if (all) return;
  __shared__ float tile[64][65];
  const int64_t R = (int64_t)S * r;
  const int64_t by = (int64_t)blockIdx.x / nkx;
  const int64_t k0 = ((int64_t)blockIdx.x - by * nkx) * 64, m0 = by * 64;
  const int tid = threadIdx.x;
  // every load is issued (clamped to a valid element) before the first is used, and the
  // padding (k >= n, M >= R) is zeroed afterwards: a load behind a branch would be
  // waited for on its own
  float a[64 * 64 / kThreads];
#pragma unroll
  for (int q = 0; q < 64 * 64 / kThreads; ++q) {
    const int e = tid + kThreads * q;
    const int kk = e >> 6, mm = e & 63;
    const int64_t k = k0 + kk < n ? k0 + kk : n - 1;
    const int64_t M = m0 + mm < R ? m0 + mm : R - 1;
    const int64_t s = M / r, m = M - s * r;
    a[q] = P[(s * n + k) * r + m];
  }
#pragma unroll
  for (int q = 0; q < 64 * 64 / kThreads; ++q) {
    const int e = tid + kThreads * q;
    const int kk = e >> 6, mm = e & 63;
    tile[kk][mm] = (k0 + kk < n && m0 + mm < R) ? a[q] : 0.0f;
  }
  __syncthreads();
  // eight consecutive k of one stacked column per thread: 16-byte stores
#pragma unroll
  for (int q = 0; q < 64 * 64 / 8 / kThreads; ++q) {
    const int e = tid + kThreads * q;
    const int mm = e >> 3, kk0 = (e & 7) * 8;
    const int64_t M = m0 + mm;
    if (M < R) {
      u16x8s vh, vl;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float a = tile[kk0 + t][mm];
        const uint16_t h = bf16_rne(a);
        vh[t] = h;
        vl[t] = bf16_rne(a - bf16_to_f32(h));
      }
      *(u16x8s*)(hi + M * ldp + k0 + kk0) = vh;
      *(u16x8s*)(lo + M * ldp + k0 + kk0) = vl;
    }
  }
}

// ----------------------------------------------------------------------------- launchers
int gram_blocks(int64_t n) {
  int64_t g = (n + 127) / 128;
  if (g < 1) g = 1;
  if (g > 256) g = 256;
  return (int)g;
}

#define SNMF_DISPATCH_RPG(rp, ...)                                  \
  switch (rp) {                                                     \
    case 4: { constexpr int RPG = 4; __VA_ARGS__; } break;          \
    case 8: { constexpr int RPG = 8; __VA_ARGS__; } break;          \
    case 16: { constexpr int RPG = 16; __VA_ARGS__; } break;        \
    case 32: { constexpr int RPG = 32; __VA_ARGS__; } break;        \
    default: { constexpr int RPG = 64; __VA_ARGS__; } break;        \
  }

template <typename T>
void launch_gram(const T* P, int64_t n, int r, double* part, int nblk, double* G64, T* GT,
                 const State* st, hipStream_t s) {
  int64_t rpb = (n + nblk - 1) / nblk;
  SNMF_DISPATCH_RPG(rank_pad(r), hipLaunchKernelGGL((k_gram<T, RPG>), dim3(nblk), dim3(kThreads),
                                                    0, s, P, n, r, rpb, part, st))
  const int rr = r * r;
  hipLaunchKernelGGL(k_gram_reduce<T>, dim3((rr + 63) / 64), dim3(kThreads), 0, s, part, nblk, rr,
                     G64, GT, st);
}
template void launch_gram<float>(const float*, int64_t, int, double*, int, double*, float*,
                                 const State*, hipStream_t);
template void launch_gram<double>(const double*, int64_t, int, double*, int, double*, double*,
                                  const State*, hipStream_t);

void launch_rho(const double* G, int r, State* st, hipStream_t s) {
  hipLaunchKernelGGL(k_rho, dim3(1), dim3(kThreads), 0, s, G, r, st);
}

template <typename T>
void launch_bgram(const T* P, int r, const int32_t* gblk_inst, int gblocks, const BInst* inst,
                  const State* states, double* gpart, hipStream_t s) {
  SNMF_DISPATCH_RPG(rank_pad(r),
                    hipLaunchKernelGGL((k_bgram<T, RPG>), dim3(gblocks), dim3(kThreads), 0, s, P,
                                       gblk_inst, inst, states, gpart))
}
template <typename T>
void launch_bgram_reduce(const BInst* inst, int ninst, int max_r, const State* states,
                         const double* gpart, double* G64, T* GT, hipStream_t s) {
  const int ny = (max_r * max_r + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_bgram_reduce<T>, dim3(ninst, ny), dim3(kThreads), 0, s, inst, states,
                     gpart, G64, GT);
}
template void launch_bgram<float>(const float*, int, const int32_t*, int, const BInst*,
                                  const State*, double*, hipStream_t);
template void launch_bgram<double>(const double*, int, const int32_t*, int, const BInst*,
                                   const State*, double*, hipStream_t);
template void launch_bgram_reduce<float>(const BInst*, int, int, const State*, const double*,
                                         double*, float*, hipStream_t);
template void launch_bgram_reduce<double>(const BInst*, int, int, const State*, const double*,
                                          double*, double*, hipStream_t);

void launch_brho(const BInst* inst, int ninst, State* states, const double* G64, hipStream_t s) {
  hipLaunchKernelGGL(k_brho, dim3(ninst), dim3(kThreads), 0, s, inst, states, G64);
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

void launch_split_pt_stack(const float* P, int64_t n, int r, int S, int64_t ldp, uint16_t* hi,
                           uint16_t* lo, State* st, const double* Grho, hipStream_t s) {
  const int64_t R = (int64_t)S * r;
  const int64_t ntile = (ldp / 64) * ((R + 63) / 64);
  hipLaunchKernelGGL(k_split_pt_stack, dim3((unsigned)(ntile + (Grho ? S : 0))), dim3(kThreads),
                     0, s, P, n, r, S, ldp, hi, lo, st, Grho);
}

void launch_split_pt(const float* P, int64_t n, int r, int64_t ldp, uint16_t* hi, uint16_t* lo,
                     const State* st, hipStream_t s) {
  int64_t nb = ((int64_t)r * ldp + kThreads - 1) / kThreads;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_split_pt, dim3((unsigned)nb), dim3(kThreads), 0, s, P, n, r, ldp, hi, lo,
                     st);
}

}  // namespace snmf
