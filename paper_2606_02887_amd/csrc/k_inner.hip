// Fused row-tile kernels of one SNMPBB half-step (Algorithm 1 with the Section 2.4
// components).  Notation: X is the variable block (n x r), P the fixed partner,
// G = P^T P, C = A P + lam P, so that grad f(X) = X G + lam X - C [+ gam L X]
// (eqs. (2.1)-(2.3) transposed).  f is quadratic in X, hence
//   f(Y + t V) - f(Y) = t <grad f(Y), V> + t^2/2 <V (G + lam I), V> [+ t^2 gam/2 <V, L V>]
// and every line-search trial is scalar work once <grad f(Z), D> and <D, (G+lam I) D>
// are known.  The iteration never forms f itself: it carries e_k = F_k - f(X_k) and the
// differences f(Z) - f(X_k) and f(X_{k+1}) - f(X_k), all accumulated in FP64.
//
// Scalar flow without fences: every kernel writes FP64 partial sums per workgroup; the
// next kernel re-reduces them in every workgroup in one fixed order, so all workgroups
// derive identical scalars, and workgroup 0 records them in the State.
//   init      -> partsA  (H-step: <C,P>; W-step: ||min(W, grad_W)||^2)
//   step1_k   reads partsC of step2_{k-1} (e_k, BB step alpha_k, stop test) or, for
//             k = 0 of a W-step, partsA + partsC of the previous H-step (monitor record);
//             writes partsB = {<grad f(Z),D>, <DG,D>, ||D||^2, f(Z)-f(X)}
//   step2_k   reads partsB [+ partsD = <D,LD>] (line search -> beta_k);
//             writes partsC = {||S||^2, <SG,S>, <g,S>, monitor pieces, <S,LS>}
// Half-steps without the Laplacian term run the fused form instead (k_advance below):
// init also forms direction 0, and each later kernel runs a line search, the update and,
// when the first trial was accepted, the next direction.
//
// A workgroup (256 threads) works on tiles of TM = 8 * 256 / RP rows, RP being the rank
// rounded up to a power of 2; each thread owns 8 elements of a tile (see Lay).  Each
// kernel issues its global loads (partial sums, State scalars, G, the first tile) before
// it waits on any of them.
#include "common.hpp"
#include "kernels.hpp"

namespace snmf {

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Workgroups per CU the row-tile kernels are built for: three for FP32 up to rank 32 (at
// most 168 registers a lane, so three waves share a SIMD; the grid is then three per CU,
// one pass over the tiles with no second round of workgroups), else whatever the
// registers allow.  The general step 2 (V = 2, the Laplacian path) keeps its registers:
// bounded to 168 it spills.
template <typename T, int RP, int V = 0>
__host__ __device__ constexpr int inner_occupancy() {
  return (sizeof(T) == 4 && RP <= 32 && V != 2) ? 3 : 1;
}

// The fused kernels (k_init with the direction, k_advance) hold more values per thread:
// bounded to 168 registers they spill at RP <= 32, so they are built for two workgroups
// per CU, and a plan that uses them caps its grid there (inner_grid).
template <typename T, int RP>
__host__ __device__ constexpr int fused_occupancy() {
  return (sizeof(T) == 4 && RP <= 32) ? 2 : 1;
}

template <int RP>
struct TileCfg {
  static constexpr int RS = kThreads / RP;  // rows per pass (VALU layout)
  static constexpr int TM = RS * 8;         // rows per tile
  static constexpr int NG = (RP * RP + kThreads - 1) / kThreads;  // G entries per thread
};

// Element ownership and the tile product.  Every thread owns 8 elements of a TM x RP
// tile (TM * RP = 2048).
//  * MFMA layout (FP32, RP >= 16): the tile is cut into 8 blocks of 16 x 16 (row-major
//    block order, RP/16 blocks per row); wave w owns blocks 2w and 2w+1; in block b lane l
//    owns rows 4(l/16) + v, v = 0..3, column l%16 -- exactly the output layout of
//    v_mfma_f32_16x16x4f32, so the products land in the owner's registers.
//  * VALU layout (FP64 or RP < 16): thread owns rows tid/RP + p * 256/RP, column tid%RP.
// LDS tiles are zero-padded to RP columns and G to RP x RP; pitches are padded against
// bank conflicts of the MFMA operand reads.
template <typename T, int RP>
struct Lay {
  static constexpr bool MF = sizeof(T) == 4 && RP >= 16;
  static constexpr int TM = TileCfg<RP>::TM;
  static constexpr int YP = MF ? RP + 1 : RP;   // tile pitch
  static constexpr int GP = MF ? RP + 16 : RP;  // G pitch
  __device__ static __forceinline__ void rc(int p, int& lr, int& col) {
    if constexpr (MF) {
      const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
      const int blk = 2 * w + (p >> 2), v = p & 3;
      constexpr int NBC = RP / 16;
      lr = 16 * (blk / NBC) + 4 * (l >> 4) + v;
      col = 16 * (blk % NBC) + (l & 15);
    } else {
      lr = (int)threadIdx.x / RP + p * (kThreads / RP);
      col = (int)threadIdx.x % RP;
    }
  }
};

// LDS tiles are zero-padded, so the products run over a compile-time range and lanes with
// col >= r compute harmless zeros.
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec4<double> {
  typedef double type __attribute__((ext_vector_type(4)));
};
typedef float f32x4m __attribute__((ext_vector_type(4)));

// acc[p] = sum_j sY[row_p][j] * sG[j][col_p] for the owned elements.
template <typename T, int RP>
__device__ __forceinline__ void tile_gemm(const T* __restrict__ sY, const T* __restrict__ sG,
                                          T (&acc)[8]) {
  typedef Lay<T, RP> L;
  if constexpr (L::MF) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int NBC = RP / 16;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int blk = 2 * w + b;
      const int r0 = 16 * (blk / NBC), c0 = 16 * (blk % NBC);
      f32x4m d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < RP; kk += 4) {
        const float a = sY[(r0 + (l & 15)) * L::YP + kk + (l >> 4)];
        const float bb = sG[(kk + (l >> 4)) * L::GP + c0 + (l & 15)];
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bb, d, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[4 * b + v] = d[v];
    }
  } else {
    constexpr int RS = TileCfg<RP>::RS;
    typedef typename Vec4<T>::type V4;
    const int c = threadIdx.x % RP, rs = threadIdx.x / RP;
#pragma unroll
    for (int p = 0; p < 8; ++p) acc[p] = T(0);
#pragma unroll 1
    for (int j = 0; j < RP; j += 4) {
      const T g0 = sG[(j + 0) * RP + c], g1 = sG[(j + 1) * RP + c];
      const T g2 = sG[(j + 2) * RP + c], g3 = sG[(j + 3) * RP + c];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const V4 y = *(const V4*)&sY[(rs + p * RS) * RP + j];
        acc[p] = fmaT(y[0], g0, acc[p]);
        acc[p] = fmaT(y[1], g1, acc[p]);
        acc[p] = fmaT(y[2], g2, acc[p]);
        acc[p] = fmaT(y[3], g3, acc[p]);
      }
    }
  }
}

// The tile buffers share their LDS with the staging area of the block sums (kStage
// doubles), which run before the first tile product or after the last.
template <typename T, int RP>
struct __attribute__((aligned(32))) Smem {
  union {
    struct {
      T G[RP * Lay<T, RP>::GP];
      T a[Lay<T, RP>::TM * Lay<T, RP>::YP];
      T b[Lay<T, RP>::TM * Lay<T, RP>::YP];
    };
    double red[kStage];
  };
};

// G (r x r, row-major in global memory) in registers, then into the zero-padded LDS copy.
template <typename T, int RP>
__device__ __forceinline__ void load_G(const T* __restrict__ GT, int r, T (&v)[TileCfg<RP>::NG]) {
#pragma unroll
  for (int q = 0; q < TileCfg<RP>::NG; ++q) {
    const int e = threadIdx.x + q * kThreads;
    const int a = e / RP, b = e % RP;
    v[q] = (e < RP * RP && a < r && b < r) ? GT[a * r + b] : T(0);
  }
}
template <typename T, int RP>
__device__ __forceinline__ void store_G(T* __restrict__ sG, const T (&v)[TileCfg<RP>::NG]) {
#pragma unroll
  for (int q = 0; q < TileCfg<RP>::NG; ++q) {
    const int e = threadIdx.x + q * kThreads;
    if (e < RP * RP) sG[(e / RP) * Lay<T, RP>::GP + (e % RP)] = v[q];
  }
}

// Thread t adds the rows t, t + 256, ... in that order.  Each pass loads two rows before it
// adds either, so up to 512 workgroups cost one memory round trip, not one per row; the
// first pass is straight-line code (no loop guard between the kernel arguments and the
// loads, so nothing waits for other scalar loads first).  Rows past nb are loaded from an
// in-bounds row and add +0.0, which leaves a sum that started at +0.0 unchanged.  Every
// thread loads, so this suits the fused kernels' plan-wide grids (256 or 512 workgroups);
// load_slots below keeps the plain loop, in which threads past nb load nothing (batches
// re-reduce grids of a few dozen workgroups per instance).
template <int K, typename F>
__device__ __forceinline__ void load_rows(int nb, double (&out)[K], F&& at) {
  auto pass = [&](int b) {
    const int b0 = min(b, nb - 1), b1 = min(b + kThreads, nb - 1);
    double u0[K], u1[K];
#pragma unroll
    for (int j = 0; j < K; ++j) u0[j] = at(b0, j);
#pragma unroll
    for (int j = 0; j < K; ++j) u1[j] = at(b1, j);
    __builtin_amdgcn_sched_barrier(0);  // every load issued before the first add waits
#pragma unroll
    for (int j = 0; j < K; ++j) out[j] += b < nb ? u0[j] : 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) out[j] += b + kThreads < nb ? u1[j] : 0.0;
  };
#pragma unroll
  for (int j = 0; j < K; ++j) out[j] = 0.0;
  pass(threadIdx.x);
  for (int b = threadIdx.x + 2 * kThreads; b < nb; b += 2 * kThreads) pass(b);
}

// This thread's share (workgroups b = tid, tid + 256, ... in increasing b) of K consecutive
// partial-sum slots starting at `first`; block_sum then adds the shares in a fixed order.
template <int K>
__device__ __forceinline__ void load_slots(const double* __restrict__ part, int nb, int first,
                                           double (&out)[K]) {
#pragma unroll
  for (int j = 0; j < K; ++j) out[j] = 0.0;
  for (int b = threadIdx.x; b < nb; b += kThreads) {
#pragma unroll
    for (int j = 0; j < K; ++j) out[j] += part[(size_t)b * kNumPart + first + j];
  }
}

// The partial sums of the fused kernels (kFusedParts slots, below) are slot-major: slot j of
// workgroup b at part[j * kInnerGrid + b].  Every workgroup re-reads all of them, and with
// this layout a wave's load of one slot covers 64 consecutive workgroups (4 cache lines;
// row-major rows would put its 64 lanes on 64 lines).  Each thread adds the same rows in
// the same order as load_slots.
template <int K>
__device__ __forceinline__ void load_cols(const double* __restrict__ part, int nb,
                                          double (&out)[K]) {
  load_rows<K>(nb, out, [&](int b, int j) { return part[(size_t)j * kInnerGrid + b]; });
}

// ----------------------------------------------------------------------------- instances
// Where this workgroup works: a single solve takes everything from the kernel arguments;
// in a batched launch the workgroup looks up its instance (two dependent scalar loads)
// and offsets the batch buffers, Gram copies, partial sums, State and trace by it.
struct Loc {
  int64_t off, n, goff, poff;
  int bid, nb;
  State* st;
  double* trace;
  double lam;
};
__device__ __forceinline__ Loc locate(const BMap& bm, int64_t n, State* st, double* trace,
                                      double lam) {
  Loc l;
  if (bm.blk_inst == nullptr) {
    l.off = 0;
    l.n = n;
    l.goff = 0;
    l.poff = 0;
    l.bid = blockIdx.x;
    l.nb = gridDim.x;
    l.st = st;
    l.trace = trace;
    l.lam = lam;
  } else {
    const int i = bm.blk_inst[blockIdx.x];
    const BInst* d = bm.inst + i;
    l.off = d->off;
    l.n = d->n;
    l.goff = d->goff;
    l.poff = (int64_t)d->part0 * kNumPart;
    l.bid = (int)blockIdx.x - d->blk0;
    l.nb = d->nblk;
    l.st = bm.states + i;
    l.trace = bm.traces ? bm.traces + (size_t)i * bm.trace_stride : nullptr;
    l.lam = d->lam;
  }
  return l;
}

// Element access inside a tile: a uniform base pointer (the tile's first row, held in
// scalar registers) plus this thread's fixed byte offset, so the loads take the
// scalar-base + 32-bit vector-offset form and one offset register serves every array.
// The access goes through a global-address-space pointer: the opaque tile pointer (below)
// hides where the array lives, and a generic pointer would give flat instructions, which
// also count against the LDS wait counter, so every wait on LDS would wait for them too.
template <typename T>
__device__ __forceinline__ T ldo(const T* __restrict__ base, uint32_t bo) {
  typedef const __attribute__((address_space(1))) T* GP;
  return *(GP)(reinterpret_cast<const char*>(base) + bo);
}
template <typename T>
__device__ __forceinline__ void sto(T* __restrict__ base, uint32_t bo, T v) {
  typedef __attribute__((address_space(1))) T* GP;
  *(GP)(reinterpret_cast<char*>(base) + bo) = v;
}
// A tile's pointer into one array, pinned as an opaque uniform (scalar-register) value:
// the empty asm emits nothing, but it stops the compiler from re-associating
// (array + tile) + offset into (array + offset) + tile and hoisting the 64 per-element
// 64-bit sums (array, element) out of the tile loop into vector registers.
template <typename P>
__device__ __forceinline__ P tile_ptr(P base, int64_t tb) {
  P q = base + tb;
  asm volatile("" : "+s"(q));
  return q;
}

// ----------------------------------------------------------------------------- Z and D
// The two projections of Algorithm 1 and the gradient at Z.
template <typename T>
__device__ __forceinline__ T first_proj(T x, T g, T rinv) {  // max(0, X - g / rho)
  return relu(fmaT(-g, rinv, x));
}
template <typename T>
__device__ __forceinline__ T grad_at_z(T g, T dzg, T lam, T dz) {  // g + (Z-X)(G + lam I)
  return fmaT(lam, dz, g + dzg);
}
template <typename T>
__device__ __forceinline__ T second_dir(T z, T gz, T alpha) {  // max(0, Z - alpha gZ) - Z
  return relu(fmaT(-alpha, gz, z)) - z;
}
// The update and its sums, written once so that every kernel forming them (step 2, and
// the fused kernels below, which form the update at beta = 1 one kernel early) produces
// the same bits: X+ = max(0, Z + phi beta D) (no projection when project = 0) and
// g+ = g + S G + lam S.
template <typename T>
__device__ __forceinline__ T next_point(T z, T d, T step, int project) {
  const T y = fmaT(step, d, z);
  return project ? relu(y) : y;
}
template <typename T>
__device__ __forceinline__ T next_grad(T g, T sg, T lam, T s) {
  return fmaT(lam, s, g + sg);
}
// <S,S>, <S G, S>, <g, S> of an update
template <typename T, int K>
__device__ __forceinline__ void update_sums(double (&v)[K], T s, T sg, T g) {
  const double sd = (double)s;
  v[0] = fmaT(sd, sd, v[0]);
  v[1] = fmaT((double)sg, sd, v[1]);
  v[2] = fmaT((double)g, sd, v[2]);
}
// <grad f(Z), D>, ||D||^2 and f(Z) - f(X) = <g + grad f(Z), Z - X>/2 of a direction
template <typename T>
__device__ __forceinline__ void direction_sums(double (&v)[4], T gz, T d, T g, T dz) {
  const double dd = (double)d;
  v[0] = fmaT((double)gz, dd, v[0]);
  v[2] = fmaT(dd, dd, v[2]);
  v[3] = fmaT(0.5 * ((double)g + (double)gz), (double)dz, v[3]);
}
// Monitor sums of the H-step's final X (x) with its gradient g, C and the partner p:
// m = {<C, X>, <P, X>, ||X - P||^2, ||min(X, g)||^2}
template <typename T>
__device__ __forceinline__ void monitor_sums(double* m, T x, T g, T c, T p) {
  const double xd = (double)x, pd = (double)p, dxp = xd - pd;
  const double mn = (double)(x < g ? x : g);
  m[0] = fmaT((double)c, xd, m[0]);
  m[1] = fmaT(pd, xd, m[1]);
  m[2] = fmaT(dxp, dxp, m[2]);
  m[3] = fmaT(mn, mn, m[3]);
}

// ----------------------------------------------------------------------------- direction
// Step 1 of a fused inner iteration on one tile whose X and g are in registers (sm.G
// holds G; sm.a and sm.b are free): Z, grad f(Z), D with step 1's arithmetic (D stored at
// Dt), and the sums the next kernel needs to finish the iteration in one pass
// (kFusedParts of them):
//   ls  = {<grad f(Z),D>, <DG,D>, ||D||^2, f(Z)-f(X)}: the line search;
//   sp  = {||S||^2, <SG,S>, <g,S>} of the update of the trial beta = 1,
//         X+ = max(0, Z + phi D), formed with step 2's arithmetic: the BB step when the
//         line search accepts that trial, the same bits as step 2 would give; that update
//         and its gradient g+ = g + S G + lam S are stored (Xt, gt), so the next kernel
//         has them without forming them again;
//   xp  = {<dZ,dZ>, <dZ,D>, <dZ,dZ G>, <dZ,DG>, <g,dZ>, <g,D>} with dZ = Z - X: the BB
//         step after a backtrack.  A trial beta <= beta_shrink has t = phi beta <= 1
//         (the fused path requires phi beta_shrink <= 1), and Z + t D is then a convex
//         combination of Z >= 0 and Z + D >= 0, so the projection clips nothing and
//         S = dZ + t D: its sums are polynomials in t of these (G symmetric).
// The caller synchronises before reusing sm.a and sm.b.
constexpr int kFusedParts = 13;
template <typename T, int RP>
__device__ __forceinline__ void tile_direction(Smem<T, RP>& sm, const int (&lr)[8],
                                               const int (&cl)[8], const uint32_t (&bo)[8],
                                               int64_t row0, int64_t n, int r, const T (&x)[8],
                                               const T (&gv)[8], T rinv, T alpha, T lam,
                                               T step1, int project, T* __restrict__ Dt,
                                               T* __restrict__ Xt, T* __restrict__ gt,
                                               double (&ls)[4], double (&sp)[3],
                                               double (&xp)[6]) {
  typedef Lay<T, RP> L;
  T z[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const bool ok = row0 + lr[p] < n && cl[p] < r;
    z[p] = first_proj(x[p], gv[p], rinv);
    sm.a[lr[p] * L::YP + cl[p]] = ok ? z[p] - x[p] : T(0);
  }
  __syncthreads();
  T dzg[8];
  tile_gemm<T, RP>(sm.a, sm.G, dzg);
  T d[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const bool ok = row0 + lr[p] < n && cl[p] < r;
    const T dz = z[p] - x[p];
    const T gz = grad_at_z(gv[p], dzg[p], lam, dz);
    const T dd = ok ? second_dir(z[p], gz, alpha) : T(0);
    d[p] = dd;
    if (ok) {
      sto(Dt, bo[p], dd);
      direction_sums(ls, gz, dd, gv[p], dz);
      const double dzd = (double)dz, gd = (double)gv[p];
      xp[0] = fmaT(dzd, dzd, xp[0]);
      xp[1] = fmaT(dzd, (double)dd, xp[1]);
      xp[2] = fmaT(dzd, (double)dzg[p], xp[2]);
      xp[4] = fmaT(gd, dzd, xp[4]);
      xp[5] = fmaT(gd, (double)dd, xp[5]);
    }
    sm.b[lr[p] * L::YP + cl[p]] = dd;
  }
  __syncthreads();
  T dg[8];
  tile_gemm<T, RP>(sm.b, sm.G, dg);
  T xn[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    ls[1] = fmaT((double)dg[p], (double)d[p], ls[1]);
    const bool ok = row0 + lr[p] < n && cl[p] < r;
    if (ok) xp[3] = fmaT((double)(z[p] - x[p]), (double)dg[p], xp[3]);
    xn[p] = ok ? next_point(z[p], d[p], step1, project) : T(0);
    sm.a[lr[p] * L::YP + cl[p]] = ok ? xn[p] - x[p] : T(0);
  }
  __syncthreads();
  T sg[8];
  tile_gemm<T, RP>(sm.a, sm.G, sg);
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    if (row0 + lr[p] < n && cl[p] < r) {
      const T s1 = xn[p] - x[p];
      update_sums(sp, s1, sg[p], gv[p]);
      sto(Xt, bo[p], xn[p]);
      sto(gt, bo[p], next_grad(gv[p], sg[p], lam, s1));
    }
  }
}

// ----------------------------------------------------------------------------- init
// C = (sum of the A-pass partials) + lam P;  g = X G + lam X - C [+ gam LX].  C is stored in
// H-steps only: the outer iteration's monitor sum <C, X> at the final X reads it there.
// DIR (fused inner iterations): also the direction of inner iteration 0 (alpha_0 = 1/rho),
// its sums (tile_direction) into pout and its beta = 1 trial update into (Xs, gs); the
// first fused kernel runs its line search.
template <typename T, int RP, int DIR>
__global__ __launch_bounds__(kThreads, (DIR ? fused_occupancy<T, RP>() : inner_occupancy<T, RP>())) void k_init(
    const T* __restrict__ X, const T* __restrict__ P, const T* __restrict__ Bpart, int ksplit,
    int64_t bstride, T* __restrict__ Cout, T* __restrict__ g, const T* __restrict__ LX,
    const T* __restrict__ GT, int64_t n, int r, int is_hstep, KParams kp, State* __restrict__ st,
    double* __restrict__ partsA, BMap bm, T* __restrict__ Zn, T* __restrict__ Dn,
    T* __restrict__ Dd, double* __restrict__ pout, T* __restrict__ Xs, T* __restrict__ gs) {
  const Loc lc = locate(bm, n, st, nullptr, kp.lam);
  st = lc.st;
  if (st->done) return;
  n = lc.n;
  kp.lam = lc.lam;
  X += lc.off;
  P += lc.off;
  Bpart += lc.off;
  Cout += lc.off;
  g += lc.off;
  if (LX) LX += lc.off;
  GT += lc.goff;
  partsA += lc.poff;
  typedef Lay<T, RP> L;
  constexpr int TM = L::TM;
  __shared__ Smem<T, RP> sm;
  const int tid = threadIdx.x;
  int lr[8], cl[8];
  uint32_t bo[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    L::rc(p, lr[p], cl[p]);
    bo[p] = (uint32_t)((lr[p] * r + cl[p]) * (int)sizeof(T));
  }
  if (!is_hstep && lc.bid == 0 && tid == 0) {
    // snapshot for the monitor record completed by this W-step's first inner kernel
    st->snap_pending = st->pending;
    st->snap_outer = st->outer;
    st->pending = 0;
  }
  T gv[TileCfg<RP>::NG];
  load_G<T, RP>(GT, r, gv);
  const T lam = (T)kp.lam, gam = (T)kp.gamma;
  const T rinv = (Zn || DIR) ? (T)(1.0 / st->rho) : T(0);
  const T step1 = (T)(kp.phi * 1.0);
  double v[1] = {0.0}, ls[4] = {0.0, 0.0, 0.0, 0.0}, sp[3] = {0.0, 0.0, 0.0};
  double xp[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t ntiles = (n + TM - 1) / TM;
  bool first = true;
  for (int64_t t = lc.bid; t < ntiles; t += lc.nb) {
    const int64_t row0 = t * TM, tb = row0 * r;
    const T* __restrict__ Bt = tile_ptr(Bpart, tb);
    T x[8], cv[8], pv[8], lx[8];
    bool ok[8];
    // X, P (and L X) of the tile and the split-K partials of B, the loads of four
    // partials for all eight elements in flight before any is added; each element adds
    // its partials in panel order
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      ok[p] = row0 + lr[p] < n && cl[p] < r;
      x[p] = ok[p] ? ldo(tile_ptr(X, tb), bo[p]) : T(0);
      pv[p] = ok[p] ? ldo(tile_ptr(P, tb), bo[p]) : T(0);
      lx[p] = (ok[p] && LX) ? ldo(tile_ptr(LX, tb), bo[p]) : T(0);
    }
    T b[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) b[p] = T(0);
    int s = 0;
    for (; s + 4 <= ksplit; s += 4) {
      T bq[4][8];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int p = 0; p < 8; ++p)
          bq[u][p] = ok[p] ? ldo(Bt + (s + u) * bstride, bo[p]) : T(0);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int p = 0; p < 8; ++p) b[p] += bq[u][p];
    }
    for (; s < ksplit; ++s) {
      T bs[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) bs[p] = ok[p] ? ldo(Bt + s * bstride, bo[p]) : T(0);
#pragma unroll
      for (int p = 0; p < 8; ++p) b[p] += bs[p];
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) cv[p] = b[p] + lam * pv[p];
    if (first) store_G<T, RP>(sm.G, gv);
    first = false;
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 8; ++p) sm.a[lr[p] * L::YP + cl[p]] = x[p];
    __syncthreads();
    T xg[8], gq[8];
    tile_gemm<T, RP>(sm.a, sm.G, xg);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      gq[p] = T(0);
      if (ok[p]) {
        if (is_hstep) sto(tile_ptr(Cout, tb), bo[p], cv[p]);  // only H-step monitors read C
        T gvv = xg[p] + lam * x[p] - cv[p];
        if (LX) gvv += gam * lx[p];
        gq[p] = gvv;
        sto(tile_ptr(g, tb), bo[p], gvv);
        if (Zn) {  // Laplacian H-step: Z and Z - X of the first inner iteration
          const T zz = first_proj(x[p], gvv, rinv);
          sto(tile_ptr(Zn, tb), bo[p], zz);
          sto(tile_ptr(Dn, tb), bo[p], zz - x[p]);
        }
        if (is_hstep) {
          v[0] = fmaT((double)cv[p], (double)pv[p], v[0]);
        } else {
          const double mn = (double)(x[p] < gvv ? x[p] : gvv);
          v[0] = fmaT(mn, mn, v[0]);
        }
      }
    }
    if constexpr (DIR != 0) {
      __syncthreads();  // every wave is done with the product on sm.a
      tile_direction<T, RP>(sm, lr, cl, bo, row0, n, r, x, gq, rinv, rinv, lam, step1,
                            kp.project, tile_ptr(Dd, tb), tile_ptr(Xs, tb), tile_ptr(gs, tb), ls,
                            sp, xp);
    }
  }
  if constexpr (DIR != 0) {
    const double o[1 + kFusedParts] = {v[0],  ls[0], ls[1], ls[2], ls[3], sp[0], sp[1],
                                       sp[2], xp[0], xp[1], xp[2], xp[3], xp[4], xp[5]};
    double* pa = partsA + (size_t)lc.bid * kNumPart;
    block_sum_emit<1 + kFusedParts>(o, sm.red, [&](int j, double a) {
      if (j)
        pout[(size_t)(j - 1) * kInnerGrid + lc.bid] = a;
      else
        pa[0] = a;
    });
  } else {
    double* pa = partsA + (size_t)lc.bid * kNumPart;
    block_sum_emit<1>(v, sm.red, [&](int j, double a) { pa[j] = a; });
  }
}

// ----------------------------------------------------------------------------- entry
// First kernel of inner iteration k: derive e_k and alpha_k (or, at k = 0, complete the
// monitor record of the previous outer iteration).  `pe` holds this thread's share of
// the partial sums (loaded at kernel start by entry_loads).  Returns kEntryRun, or why
// this inner iteration must not run: the half-step stopped (X_k = X_{k-1}), or the solve
// is over (monitor target or max_outer met, breakdown).
constexpr int kEntryRun = 0, kEntryHalfOver = 1, kEntrySolveOver = 2;
__device__ __forceinline__ void entry_loads(int k, int is_hstep, const double* __restrict__ partsA,
                                            const double* __restrict__ partsC, int nb,
                                            double (&pe)[6]) {
  if (k == 0) {
    double a1[1], m5[5];
    load_slots<1>(partsA, nb, 0, a1);
    if (!is_hstep) {
      load_slots<5>(partsC, nb, 3, m5);
    } else {
#pragma unroll
      for (int j = 0; j < 5; ++j) m5[j] = 0.0;
    }
    pe[0] = a1[0];
#pragma unroll
    for (int j = 0; j < 5; ++j) pe[1 + j] = m5[j];
  } else {
    double s3[3], s1[1];
    load_slots<3>(partsC, nb, 0, s3);
    load_slots<1>(partsC, nb, 8, s1);
    pe[0] = s3[0];
    pe[1] = s3[1];
    pe[2] = s3[2];
    pe[3] = s1[0];
    pe[4] = 0.0;
    pe[5] = 0.0;
  }
}

// e_k and alpha_k of inner iteration k >= 1 from the reduced sums of the last update,
// s4 = {<S,S>, <S G, S>, <g, S>, <S, L S>}; the same return codes as inner_entry.
__device__ int bb_step(int k, const double (&s4)[4], double e_prev, const KParams& kp,
                       State* __restrict__ st, bool w0, double& alpha_out) {
  const double ss = s4[0];
  const double sy = s4[1] + kp.lam * ss + kp.gamma * s4[3];  // <S,Y> = <S(G+lam I),S> [+gam<S,LS>]
  const double dlt = s4[2] + 0.5 * sy;                        // f(X_k) - f(X_{k-1})
  const double e_k = kp.eta * (e_prev - dlt);                 // F_k - f(X_k)
  const double ratio = sy > 0.0 ? ss / sy : 1e308;
  const double alpha_k = fmin(kp.amax, fmax(kp.amin, ratio));
  const bool bad = !(sy == sy) || !(dlt == dlt);
  if (w0) {
    st->last_ss = ss;
    st->last_sy = sy;
    if (bad) {
      st->status = 9;
      st->done = 1;
    }
  }
  if (bad) return kEntrySolveOver;
  if (ss == 0.0) {  // X_k = X_{k-1}: stationary, the half-step is over
    if (w0) st->stop[k] = 1;
    return kEntryHalfOver;
  }
  if (w0) {
    st->e[k] = e_k;
    st->alpha[k] = alpha_k;
    st->stop[k] = 0;
  }
  alpha_out = alpha_k;
  return kEntryRun;
}

template <int RP>
__device__ int inner_entry(int k, int is_hstep, int r, const KParams& kp, State* __restrict__ st,
                            double (&pe)[6], int stop_prev, double e_prev, double rho,
                            const double* __restrict__ Gcur,
                            const double* __restrict__ Gprev, double* __restrict__ trace,
                            double* sred, bool w0, double& alpha_out) {
  double e_k, alpha_k;
  if (k == 0) {
    if (!is_hstep) {
      if (st->snap_pending) {
        // ||min(W, grad_W)||^2, <C,Ht>, <W,Ht>, ||Ht-W||^2, pgH^2, <Ht,LHt>
        block_sum_wide<6>(pe, sred);
        // <W^T W, Ht^T Ht>, ||W^T W||_F^2, ||W||^2 = tr(W^T W); thread t adds the entries
        // t, t + 256, ... in that order, all loaded before the first add (as many per
        // thread as the padded rank needs: one below rank 17)
        constexpr int kGE = (RP * RP + kThreads - 1) / kThreads;
        const int rr = r * r;
        double gp[kGE], gc[kGE];
#pragma unroll
        for (int u = 0; u < kGE; ++u) {
          const int e = min((int)threadIdx.x + u * kThreads, rr - 1);
          gp[u] = Gprev[e];
          gc[u] = Gcur[e];
        }
        const double dg = (int)threadIdx.x < r ? Gprev[threadIdx.x * r + threadIdx.x] : 0.0;
        __builtin_amdgcn_sched_barrier(0);
        double gg[3] = {0.0, 0.0, dg};
#pragma unroll
        for (int u = 0; u < kGE; ++u) {
          if ((int)threadIdx.x + u * kThreads < rr) {
            gg[0] = fma(gp[u], gc[u], gg[0]);
            gg[1] = fma(gp[u], gp[u], gg[1]);
          }
        }
        block_sum_wide<3>(gg, sred);
        const double nA2 = st->normA2;
        const double AWHt = pe[1] - kp.lam * pe[2];     // <A W, Ht>
        const double AWW = st->m_CP - kp.lam * gg[2];   // <A W, W>
        const double res2 = nA2 - 2.0 * AWHt + gg[0];
        const double resw2 = nA2 - 2.0 * AWW + gg[1];
        const double res = sqrt(fmax(res2, 0.0) / nA2);
        const double resw = sqrt(fmax(resw2, 0.0) / nA2);
        const double sym = sqrt(pe[3] / fmax(gg[2], 1e-300));
        const double pg = sqrt(pe[0] + pe[4]);
        const double f = 0.5 * fmax(res2, 0.0) + 0.5 * kp.lam * pe[3] + 0.5 * kp.gamma * pe[5];
        const int o = st->snap_outer;
        const bool conv = kp.target > 0.0 && res <= kp.target;
        const bool bad = !(res == res) || !(pg == pg);
        const bool fin = conv || bad || o + 1 >= kp.max_outer;
        if (w0) {
          if (trace) {
            double* rec = trace + (size_t)o * kTraceFields;
            rec[0] = res;
            rec[1] = resw;
            rec[2] = sym;
            rec[3] = pg;
            rec[4] = f;
            rec[5] = (double)(st->t_hstep - st->t0);
            rec[6] = (double)st->ls_evals;
            rec[7] = (double)st->ls_exhausted;
            rec[8] = st->last_sy > 0.0 ? st->last_ss / st->last_sy : 0.0;
            rec[9] = (double)st->inner_total;
          }
          st->res_last = res;
          st->resww_last = resw;
          st->sym_last = sym;
          st->pg_last = pg;
          st->f_last = f;
          st->outer = o + 1;
          st->trace_len = o + 1;
          if (conv && st->converged_at == 0) {
            st->converged_at = o + 1;
            st->t_conv = st->t_hstep - st->t0;
          }
          if (bad) st->status = 9;
          if (fin) st->done = 1;
        }
        if (fin) return kEntrySolveOver;
      }
    } else {
      double a1[1] = {pe[0]};
      block_sum_wide<1>(a1, sred);                   // <C, P> with P = W
      if (w0) st->m_CP = a1[0];
    }
    // the partner block vanished (rho = 0) or overflowed: breakdown, reported here so
    // that the record of the last completed outer iteration (above) is kept
    if (!(rho > 0.0) || !(rho < 1e308)) {
      if (w0) {
        st->status = 9;
        st->done = 1;
      }
      return kEntrySolveOver;
    }
    e_k = 0.0;
    alpha_k = 1.0 / rho;
  } else {
    if (stop_prev) {
      if (w0) st->stop[k] = 1;
      return kEntryHalfOver;
    }
    double s4[4] = {pe[0], pe[1], pe[2], pe[3]};
    block_sum_wide<4>(s4, sred);
    return bb_step(k, s4, e_prev, kp, st, w0, alpha_out);
  }
  if (w0) {
    st->e[k] = e_k;
    st->alpha[k] = alpha_k;
    st->stop[k] = 0;
  }
  alpha_out = alpha_k;
  return kEntryRun;
}

// ----------------------------------------------------------------------------- step 1
// Z = max(0, X - g/rho);  grad f(Z) = g + (Z - X)(G + lam I) [+ gam L(Z-X)];
// D = max(0, Z - alpha grad f(Z)) - Z.  Partials: <grad f(Z), D>, <D G, D>, ||D||^2 and
// f(Z) - f(X) = <g + grad f(Z), Z - X>/2 (exact for a quadratic).
// phase 0: whole step.  Laplacian path: phase 1 writes Z and Z - X (into D); phase 2
// reads them back together with L(Z - X).
// V = 0: phase 0 only (a compile-time constant, so the Laplacian operands and their
// registers drop out); V = 1: any phase.
template <typename T, int RP, int V>
__global__ __launch_bounds__(kThreads, (inner_occupancy<T, RP>())) void k_step1(
    const T* __restrict__ X, const T* __restrict__ g, T* __restrict__ Z, T* __restrict__ D,
    const T* __restrict__ LdZ, const T* __restrict__ GT, const double* __restrict__ Gcur,
    const double* __restrict__ Gprev, int64_t n, int r, int k, int phase, int is_hstep,
    KParams kp, State* __restrict__ st, const double* __restrict__ partsA,
    double* __restrict__ partsB, const double* __restrict__ partsC, double* __restrict__ trace,
    BMap bm, int rd) {
  if constexpr (V == 0) phase = 0;
  const Loc lc = locate(bm, n, st, trace, kp.lam);
  st = lc.st;
  trace = lc.trace;
  n = lc.n;
  kp.lam = lc.lam;
  X += lc.off;
  g += lc.off;
  Z += lc.off;
  D += lc.off;
  if (LdZ) LdZ += lc.off;
  GT += lc.goff;
  Gcur += lc.goff;
  Gprev += lc.goff;
  partsA += lc.poff;
  partsB += lc.poff;
  partsC += lc.poff;
  typedef Lay<T, RP> L;
  constexpr int TM = L::TM;
  __shared__ Smem<T, RP> sm;
  int lr[8], cl[8];
  uint32_t bo[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    L::rc(p, lr[p], cl[p]);
    bo[p] = (uint32_t)((lr[p] * r + cl[p]) * (int)sizeof(T));
  }
  const int64_t ntiles = (n + TM - 1) / TM;
  // loads first: State scalars, partial sums of the previous kernel, G, the first tile
  const int done = st->done;
  const int km = k > 0 ? k - 1 : 0;
  const int stop_prev = st->stop[km];
  const double e_prev = st->e[km], rho = st->rho;
  double pe[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  entry_loads(k, is_hstep, partsA, partsC, lc.nb, pe);
  T gv[TileCfg<RP>::NG];
  if (phase != 1) load_G<T, RP>(GT, r, gv);
  T x[8], gvv[8], z[8], lz[8];
  auto load_tile = [&](int64_t row0) {
    const int64_t tb = row0 * r;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const bool ok = row0 + lr[p] < n && cl[p] < r;
      x[p] = ok ? ldo(tile_ptr(X, tb), bo[p]) : T(0);
      gvv[p] = ok ? ldo(tile_ptr(g, tb), bo[p]) : T(0);
      z[p] = (ok && phase == 2) ? ldo(tile_ptr(Z, tb), bo[p]) : T(0);
      lz[p] = (ok && phase == 2) ? ldo(tile_ptr(LdZ, tb), bo[p]) : T(0);
    }
  };
  if (lc.bid < ntiles) load_tile((int64_t)lc.bid * TM);
  if (done) return;
  // every phase opens the inner iteration: the Laplacian path launches phase 2 only (its
  // Z and Z - X come from the previous step 2 or from init), phase 1 only as the closing
  // entry of the half-step API
  double alpha_d = 0.0;
  if (inner_entry<RP>(k, is_hstep, r, kp, st, pe, stop_prev, e_prev, rho, Gcur, Gprev, trace,
                  sm.red, lc.bid == 0 && threadIdx.x == 0, alpha_d) != kEntryRun)
    return;
  const T rinv = (T)(1.0 / rho);
  const T alpha = (T)alpha_d;
  const T lam = (T)kp.lam, gam = (T)kp.gamma;
  if (phase == 1) {
    for (int64_t t = lc.bid; t < ntiles; t += lc.nb) {
      if (t != lc.bid) load_tile(t * TM);
      const int64_t tb = t * TM * r;
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        if (t * TM + lr[p] < n && cl[p] < r) {
          const T zz = first_proj(x[p], gvv[p], rinv);
          sto(tile_ptr(Z, tb), bo[p], zz);
          sto(tile_ptr(D, tb), bo[p], zz - x[p]);
        }
      }
    }
    return;
  }
  store_G<T, RP>(sm.G, gv);
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t t = lc.bid; t < ntiles; t += lc.nb) {
    const int64_t row0 = t * TM;
    if (t != lc.bid) load_tile(row0);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const bool ok = row0 + lr[p] < n && cl[p] < r;
      if (phase == 0) z[p] = first_proj(x[p], gvv[p], rinv);
      sm.a[lr[p] * L::YP + cl[p]] = ok ? z[p] - x[p] : T(0);
    }
    __syncthreads();
    T dzg[8];
    tile_gemm<T, RP>(sm.a, sm.G, dzg);
    T d[8];
    const int64_t tb = row0 * r;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const bool ok = row0 + lr[p] < n && cl[p] < r;
      const T dz = z[p] - x[p];
      T gz = grad_at_z(gvv[p], dzg[p], lam, dz);
      if (phase == 2) gz += gam * lz[p];
      const T dd = ok ? second_dir(z[p], gz, alpha) : T(0);
      d[p] = dd;
      if (ok) {
        // phase 0 keeps Z in registers only, and D too when rd is set: step 2 recomputes
        // them from X and g
        if (phase != 0 || !rd) sto(tile_ptr(D, tb), bo[p], dd);
        direction_sums(v, gz, dd, gvv[p], dz);
      }
      sm.b[lr[p] * L::YP + cl[p]] = dd;
    }
    __syncthreads();
    T dg[8];
    tile_gemm<T, RP>(sm.b, sm.G, dg);
#pragma unroll
    for (int p = 0; p < 8; ++p) v[1] = fmaT((double)dg[p], (double)d[p], v[1]);
  }
  double* pb = partsB + (size_t)lc.bid * kNumPart;
  block_sum_emit<4>(v, sm.red, [&](int j, double a) { pb[j] = a; });
}

// ----------------------------------------------------------------------------- line search
// Backtracking from beta = 1 by beta_shrink, at most max_ls reductions (the last beta is
// kept when the cap is hit).  Algorithm 1 accepts beta when
//   f(Z + beta D) <= F_k + theta beta <grad f(Z), D>
// which, with f(Z + beta D) = f(Z) + beta delta + beta^2 q / 2 and F_k = f(X_k) + e_k,
//   (f(Z) - f(X_k)) + (1 - theta) beta delta + beta^2 q / 2 <= e_k.
// The relaxed reading tests Z + phi beta D instead (phi beta in place of beta in f).
__device__ __forceinline__ double line_search(double delta, double q, double dZ, double e,
                                              const KParams& kp, int& evals, int& exhausted) {
  const double c1 = kp.relaxed ? (kp.phi - kp.theta) : (1.0 - kp.theta);
  const double c2 = kp.relaxed ? kp.phi * kp.phi : 1.0;
  double beta = 1.0;
  int t = 0;
  evals = 0;
  exhausted = 0;
  for (;;) {
    ++evals;
    const double lhs = dZ + c1 * beta * delta + 0.5 * c2 * beta * beta * q;
    if (lhs <= e) break;
    if (t >= kp.max_ls) {
      exhausted = 1;
      break;
    }
    beta *= kp.shrink;
    ++t;
  }
  return beta;
}

// ----------------------------------------------------------------------------- step 2
// X+ = max(0, Z + phi beta D);  S = X+ - X;  g+ = g + S (G + lam I) [+ gam L S].
// Partials: ||S||^2, <S G, S>, <g, S>; on the H-step also the monitor pieces
// <C, X+>, <P, X+>, ||X+ - P||^2, ||min(X+, g+)||^2 [and <X+, L X+>]; <S, L S> in slot 8.
// phase 0: whole step.  Laplacian path: phase 1 writes X+ into Z and S into D; phase 2
// reads them back with L S and keeps the buffer L X current (L X+ = L X + L S).
// V = 0: phase 0 of a W-step; V = 1: phase 0 of the last inner iteration of an H-step,
// which also forms the monitor sums; V = 3: phase 0 of an earlier H-step iteration, which
// does not (their monitor sums would be overwritten unread); all three compile-time, so
// unused operands and sums drop out of the registers.  V = 2: any phase and step.
// An H-step that stops early (exact stationarity, stop[k]) forms the monitor sums in the
// first skipped step 2 instead: X and g no longer change, so they are the final ones.
// rd (phase 0): step 1 stored no D; step 2 forms it again from X, g, G and alpha_k with
// the same operations in the same order, so it holds the same bits.
template <typename T, int RP, int V>
__global__ __launch_bounds__(kThreads, (inner_occupancy<T, RP, V>())) void k_step2(
    T* __restrict__ X, T* __restrict__ g, T* __restrict__ Z, T* __restrict__ D,
    const T* __restrict__ LS, const T* __restrict__ C, const T* __restrict__ P,
    T* __restrict__ LXb, const T* __restrict__ GT, int64_t n, int r, int k, int phase,
    int is_hstep, KParams kp, State* __restrict__ st, const double* __restrict__ partsB,
    const double* __restrict__ partsD, int nbD, double* __restrict__ partsC, BMap bm, int rd) {
  if constexpr (V != 2) {
    phase = 0;
    is_hstep = V == 0 ? 0 : 1;
  }
  const Loc lc = locate(bm, n, st, nullptr, kp.lam);
  st = lc.st;
  n = lc.n;
  kp.lam = lc.lam;
  X += lc.off;
  g += lc.off;
  Z += lc.off;
  D += lc.off;
  if (LS) LS += lc.off;
  if (C) C += lc.off;
  if (P) P += lc.off;
  if (LXb) LXb += lc.off;
  GT += lc.goff;
  partsB += lc.poff;
  partsC += lc.poff;
  typedef Lay<T, RP> L;
  constexpr int TM = L::TM;
  __shared__ Smem<T, RP> sm;
  int lr[8], cl[8];
  uint32_t bo[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    L::rc(p, lr[p], cl[p]);
    bo[p] = (uint32_t)((lr[p] * r + cl[p]) * (int)sizeof(T));
  }
  const bool w0 = lc.bid == 0 && threadIdx.x == 0;
  const int64_t ntiles = (n + TM - 1) / TM;
  // loads first: State scalars, partial sums of step 1 (and <D, L D>), G, the first tile
  const int done = st->done;
  const int skip = done | st->stop[k];
  const double e_k = st->e[k], beta_k2 = st->beta[k];
  double pb[4] = {0.0, 0.0, 0.0, 0.0}, pd[1] = {0.0};
  if (phase != 2) {
    load_slots<4>(partsB, lc.nb, 0, pb);
    if (partsD) load_slots<1>(partsD, nbD, 0, pd);
  }
  T gv[TileCfg<RP>::NG];
  if (phase != 1) load_G<T, RP>(GT, r, gv);
  const bool mon = V == 3 ? false : (is_hstep && phase != 1);
  const bool lap = phase == 2;
  // phase 0 (V != 2): Z = max(0, X - g / rho), and with rd also D = max(0, Z - alpha
  // grad f(Z)) - Z, are recomputed from X and g with step 1's arithmetic (the same bits:
  // the same operations on the same operands, the tile product on the same MFMA
  // sequence), so step 1 does not store them.  rd trades a second tile product for two
  // n x r transfers: set where the arrays stream from HBM, clear where the kernels are
  // latency-bound.
  const T rinv = (T)(1.0 / st->rho);
  const T alpha_r = (T)st->alpha[k];
  T x[8], zz[8], dd[8], go[8], cv[8], pv[8], ls[8], lx[8];
  auto load_tile = [&](int64_t row0) {
    const int64_t tb = row0 * r;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const bool ok = row0 + lr[p] < n && cl[p] < r;
      x[p] = ok ? ldo(tile_ptr(X, tb), bo[p]) : T(0);
      if constexpr (V == 2) zz[p] = ok ? ldo(tile_ptr(Z, tb), bo[p]) : T(0);
      if (V == 2 || !rd) dd[p] = (ok && phase != 2) ? ldo(tile_ptr(D, tb), bo[p]) : T(0);
      go[p] = (ok && phase != 1) ? ldo(tile_ptr(g, tb), bo[p]) : T(0);
      cv[p] = (ok && mon) ? ldo(tile_ptr(C, tb), bo[p]) : T(0);
      pv[p] = (ok && mon) ? ldo(tile_ptr(P, tb), bo[p]) : T(0);
      ls[p] = (ok && lap) ? ldo(tile_ptr(LS, tb), bo[p]) : T(0);
      lx[p] = (ok && lap && LXb) ? ldo(tile_ptr(LXb, tb), bo[p]) : T(0);
      if constexpr (V != 2) zz[p] = first_proj(x[p], go[p], rinv);
    }
  };
  if (lc.bid < ntiles) load_tile((int64_t)lc.bid * TM);
  if (skip) {
    if constexpr (V == 1 || V == 3) {
      if (!done) {  // stopped H-step: monitor sums of the final X (S = 0, g unchanged)
        double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t t = lc.bid; t < ntiles; t += lc.nb) {
          const int64_t tb = t * TM * r;
#pragma unroll
          for (int p = 0; p < 8; ++p) {
            if (t * TM + lr[p] < n && cl[p] < r) {
              monitor_sums(v + 3, ldo(tile_ptr(X, tb), bo[p]), ldo(tile_ptr(g, tb), bo[p]),
                           ldo(tile_ptr(C, tb), bo[p]), ldo(tile_ptr(P, tb), bo[p]));
            }
          }
        }
        double* pc = partsC + (size_t)lc.bid * kNumPart;
        block_sum_emit<9>(v, sm.red, [&](int j, double a) { pc[j] = a; });
        if (w0) {  // (set already when an earlier step 2 of this H-step ran)
          st->pending = 1;
          st->t_hstep = wall_clock64();
        }
      }
    }
    return;
  }
  double beta;
  if (phase != 2) {
    block_sum_wide<4>(pb, sm.red);
    double q = pb[1] + kp.lam * pb[2];
    if (partsD) {
      block_sum_wide<1>(pd, sm.red);
      q += kp.gamma * pd[0];
    }
    int evals, exh;
    beta = line_search(pb[0], q, pb[3], e_k, kp, evals, exh);
    if (w0) {
      st->beta[k] = beta;
      st->ls_evals += evals;
      st->ls_exhausted += exh;
      st->inner_total += 1;
    }
  } else {
    beta = beta_k2;
  }
  const T step = (T)(kp.phi * beta);
  const T lam = (T)kp.lam, gam = (T)kp.gamma;
  if (phase == 1) {
    for (int64_t t = lc.bid; t < ntiles; t += lc.nb) {
      if (t != lc.bid) load_tile(t * TM);
      const int64_t tb = t * TM * r;
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        if (t * TM + lr[p] < n && cl[p] < r) {
          const T xn = next_point(zz[p], dd[p], step, kp.project);
          sto(tile_ptr(Z, tb), bo[p], xn);
          sto(tile_ptr(D, tb), bo[p], xn - x[p]);
        }
      }
    }
    return;
  }
  store_G<T, RP>(sm.G, gv);
  double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t t = lc.bid; t < ntiles; t += lc.nb) {
    const int64_t row0 = t * TM;
    if (t != lc.bid) load_tile(row0);
    T xn[8];
    __syncthreads();
    if (V != 2 && rd) {
      // D as step 1 formed it: grad f(Z) = g + (Z - X)(G + lam I), then the projection
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const bool ok = row0 + lr[p] < n && cl[p] < r;
        sm.a[lr[p] * L::YP + cl[p]] = ok ? zz[p] - x[p] : T(0);
      }
      __syncthreads();
      T dzg[8];
      tile_gemm<T, RP>(sm.a, sm.G, dzg);
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const bool ok = row0 + lr[p] < n && cl[p] < r;
        const T gz = grad_at_z(go[p], dzg[p], lam, zz[p] - x[p]);
        dd[p] = ok ? second_dir(zz[p], gz, alpha_r) : T(0);
      }
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const bool ok = row0 + lr[p] < n && cl[p] < r;
      if (phase == 2) {
        xn[p] = zz[p];
      } else {
        xn[p] = ok ? next_point(zz[p], dd[p], step, kp.project) : T(0);
      }
      sm.b[lr[p] * L::YP + cl[p]] = ok ? xn[p] - x[p] : T(0);
    }
    __syncthreads();
    T sg[8];
    tile_gemm<T, RP>(sm.b, sm.G, sg);
    const int64_t tb = row0 * r;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      if (row0 + lr[p] < n && cl[p] < r) {
        const T s = xn[p] - x[p];
        T gn = next_grad(go[p], sg[p], lam, s);
        if (lap) gn += gam * ls[p];
        sto(tile_ptr(X, tb), bo[p], xn[p]);
        sto(tile_ptr(g, tb), bo[p], gn);
        update_sums(v, s, sg[p], go[p]);
        if (lap) v[8] += (double)s * (double)ls[p];
        if (mon) monitor_sums(v + 3, xn[p], gn, cv[p], pv[p]);
        if (lap && LXb) {
          const T lxn = lx[p] + ls[p];
          sto(tile_ptr(LXb, tb), bo[p], lxn);
          if (is_hstep) v[7] += (double)xn[p] * (double)lxn;
        }
        if (lap) {  // Z and Z - X of the next inner iteration, from the final X and g
          const T zn = first_proj(xn[p], gn, rinv);
          sto(tile_ptr(Z, tb), bo[p], zn);
          sto(tile_ptr(D, tb), bo[p], zn - xn[p]);
        }
      }
    }
  }
  double* pc = partsC + (size_t)lc.bid * kNumPart;
  if (mon || lap) {
    block_sum_emit<9>(v, sm.red, [&](int j, double a) { pc[j] = a; });
  } else {  // a step without monitor sums or Laplacian produces only the first three
    const double v3[3] = {v[0], v[1], v[2]};
    block_sum_emit<3>(v3, sm.red, [&](int j, double a) { pc[j] = a; });
    if (threadIdx.x == 0)
      for (int j = 3; j < 9; ++j) pc[j] = 0.0;
  }
  if (is_hstep && w0) {
    st->pending = 1;
    st->t_hstep = wall_clock64();
  }
}

// ----------------------------------------------------------------------------- fused
// Inner iterations with one kernel each (half-steps without the Laplacian term).  An inner
// iteration needs two grid-wide sums: those of its direction (for the line search) and
// those of its update S_k (for the next BB step).  The kernel that forms D_k also forms
// the sums from which the next kernel gets the update's without another reduction
// (tile_direction): for the trial beta = 1 those of the update itself, formed as step 2
// forms them (the same bits), and for any backtracked trial the polynomial coefficients
// of S = dZ + t D.  It also stores that trial update and its gradient.  Kernel i of a
// half-step thus runs the line search of iteration i, derives e_{i+1} and alpha_{i+1},
// takes the stored update when the line search accepted beta = 1 (else it forms the
// update from X_i, g_i, D_i), and forms direction i + 1 in one pass over its tiles;
// kernel K - 1 applies the last update and, in an H-step, forms the monitor sums (into
// partsC, as step 2 does).
// Two buffer pairs (X0, g0) = the half-step's X and g, (X1, g1) scratch, alternate:
// before kernel i, pair i % 2 holds the iterate X_i and its gradient, pair (i + 1) % 2 the
// beta = 1 trial of X_{i+1}.  Kernel i leaves X_{i+1} in pair (i + 1) % 2 (the trial when
// accepted, else overwritten) and the next trial in pair i % 2; the closing kernel copies
// the final X into X0 when it sits in pair 1.  Partial sums alternate between two arrays
// (pin of kernel i = pout of kernel i - 1).  A half-step that stops early (S = 0) marks
// the remaining iterations stopped; their kernels return at once.
template <typename T, int RP, int HS>
__global__ __launch_bounds__(kThreads, (fused_occupancy<T, RP>())) void k_advance(
    T* __restrict__ X0, T* __restrict__ g0, T* __restrict__ X1, T* __restrict__ g1,
    T* __restrict__ D, const T* __restrict__ C, const T* __restrict__ P,
    const T* __restrict__ GT, const double* __restrict__ Gcur, const double* __restrict__ Gprev,
    int64_t n, int r, int K, int i, KParams kp, State* __restrict__ st,
    const double* __restrict__ pin, double* __restrict__ pout, const double* __restrict__ partsA,
    double* __restrict__ partsC, double* __restrict__ trace) {
  typedef Lay<T, RP> L;
  constexpr int TM = L::TM;
  __shared__ Smem<T, RP> sm;
  const int nb = (int)gridDim.x, bid = (int)blockIdx.x;
  const bool w0 = bid == 0 && threadIdx.x == 0;
  T* const Xc = (i & 1) ? X1 : X0;   // X_i, g_i (then the next trial)
  T* const gc = (i & 1) ? g1 : g0;
  T* const Xn = (i & 1) ? X0 : X1;   // the trial of X_{i+1} (then X_{i+1})
  T* const gn_ = (i & 1) ? g0 : g1;
  int lr[8], cl[8];
  uint32_t bo[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    L::rc(p, lr[p], cl[p]);
    bo[p] = (uint32_t)((lr[p] * r + cl[p]) * (int)sizeof(T));
  }
  const int64_t ntiles = (n + TM - 1) / TM;
  // loads first: State scalars, the partial sums (and the k = 0 entry's), G, the trial
  // update of the first tile
  // (unconditional loads, selected afterwards: a load under "i > 0" became a branch that
  // waited for it before any other load was issued)
  const int done = st->done, stop_i = st->stop[i];
  const double rho = st->rho, e_raw = st->e[i];
  const int stopped = i > 0 ? stop_i : 0;
  const double e_i = i > 0 ? e_raw : 0.0;
  double pa[kFusedParts];
  load_cols<kFusedParts>(pin, nb, pa);
  double pe[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (i == 0) entry_loads(0, HS, partsA, partsC, nb, pe);
  T gv[TileCfg<RP>::NG];
  load_G<T, RP>(GT, r, gv);
  T xt[8], gt[8];
  auto load_trial = [&](int64_t row0) {
    const int64_t tb = row0 * r;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const bool ok = row0 + lr[p] < n && cl[p] < r;
      xt[p] = ok ? ldo(tile_ptr(Xn, tb), bo[p]) : T(0);
      gt[p] = ok ? ldo(tile_ptr(gn_, tb), bo[p]) : T(0);
    }
  };
  if (bid < ntiles) load_trial((int64_t)bid * TM);
  if (done || stopped) return;
  if (i == 0) {  // inner iteration 0 opens here: monitor record, <C, P>, rho check
    double a0;
    if (inner_entry<RP>(0, HS, r, kp, st, pe, 0, 0.0, rho, Gcur, Gprev, trace, sm.red, w0, a0) !=
        kEntryRun)
      return;
  }
  block_sum_wide<kFusedParts>(pa, sm.red);
  // line search of iteration i (step 2's)
  const double q = pa[1] + kp.lam * pa[2];
  int evals, exh;
  const double beta = line_search(pa[0], q, pa[3], e_i, kp, evals, exh);
  if (w0) {
    st->beta[i] = beta;
    st->ls_evals += evals;
    st->ls_exhausted += exh;
    st->inner_total += 1;
  }
  const bool trial = beta == 1.0;  // the stored update is X_{i+1}
  // then the next BB step from the sums of this update
  bool dir = false, closing = i + 1 >= K;
  double alpha_d = 0.0;
  if (!closing) {
    double s4[4];
    if (trial) {
      s4[0] = pa[4];
      s4[1] = pa[5];
      s4[2] = pa[6];
    } else {  // S = dZ + t D
      const double t = kp.phi * beta;
      s4[0] = pa[7] + t * (2.0 * pa[8] + t * pa[2]);
      s4[1] = pa[9] + t * (2.0 * pa[10] + t * pa[1]);
      s4[2] = pa[11] + t * pa[12];
    }
    s4[3] = 0.0;
    const int e = bb_step(i + 1, s4, e_i, kp, st, w0, alpha_d);
    if (e == kEntrySolveOver) return;
    dir = e == kEntryRun;
    closing = e == kEntryHalfOver;
  }
  store_G<T, RP>(sm.G, gv);
  const T rinv = (T)(1.0 / rho);
  const T lam = (T)kp.lam;
  const T step = (T)(kp.phi * beta), step1 = (T)(kp.phi * 1.0), alpha = (T)alpha_d;
  double ls[4] = {0.0, 0.0, 0.0, 0.0}, sp[3] = {0.0, 0.0, 0.0};
  double xp[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, mon[4] = {0.0, 0.0, 0.0, 0.0};
  // X_{i+1} and its gradient of one tile: the trial, or step 2's update formed from X_i,
  // g_i and D_i (stored over the trial)
  auto next_tile = [&](int64_t row0, T (&xn)[8], T (&gn)[8]) {
    const int64_t tb = row0 * r;
    if (trial) {
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        xn[p] = xt[p];
        gn[p] = gt[p];
      }
      return;
    }
    T x[8], go[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const bool ok = row0 + lr[p] < n && cl[p] < r;
      x[p] = ok ? ldo(tile_ptr(Xc, tb), bo[p]) : T(0);
      go[p] = ok ? ldo(tile_ptr(gc, tb), bo[p]) : T(0);
      const T dd = ok ? ldo(tile_ptr(D, tb), bo[p]) : T(0);
      const T zz = first_proj(x[p], go[p], rinv);
      xn[p] = ok ? next_point(zz, dd, step, kp.project) : T(0);
      sm.b[lr[p] * L::YP + cl[p]] = ok ? xn[p] - x[p] : T(0);
    }
    __syncthreads();
    T sg[8];
    tile_gemm<T, RP>(sm.b, sm.G, sg);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      gn[p] = T(0);
      if (row0 + lr[p] < n && cl[p] < r) {
        gn[p] = next_grad(go[p], sg[p], lam, xn[p] - x[p]);
        sto(tile_ptr(Xn, tb), bo[p], xn[p]);
        sto(tile_ptr(gn_, tb), bo[p], gn[p]);
      }
    }
  };
  if (closing) {  // the last update, then the H-step's monitor sums of the final X
    for (int64_t t = bid; t < ntiles; t += nb) {
      const int64_t row0 = t * TM, tb = row0 * r;
      T xn[8], gn[8];
      __syncthreads();
      next_tile(row0, xn, gn);
      if (trial && t + nb < ntiles) load_trial(row0 + (int64_t)nb * TM);
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        if (row0 + lr[p] < n && cl[p] < r) {
          if (Xn != X0) sto(tile_ptr(X0, tb), bo[p], xn[p]);
          if (HS)
            monitor_sums(mon, xn[p], gn[p], ldo(tile_ptr(C, tb), bo[p]), ldo(tile_ptr(P, tb), bo[p]));
        }
      }
    }
  } else {  // X_{i+1}, then direction i + 1 and the next trial (into pair i % 2)
    for (int64_t t = bid; t < ntiles; t += nb) {
      const int64_t row0 = t * TM, tb = row0 * r;
      T xn[8], gn[8];
      __syncthreads();
      next_tile(row0, xn, gn);
      // the trial of this workgroup's next tile loads while this one is worked on
      if (trial && t + nb < ntiles) load_trial(row0 + (int64_t)nb * TM);
      // sm.a was last read before this tile's first barrier
      tile_direction<T, RP>(sm, lr, cl, bo, row0, n, r, xn, gn, rinv, alpha, lam, step1,
                            kp.project, tile_ptr(D, tb), tile_ptr(Xc, tb), tile_ptr(gc, tb), ls,
                            sp, xp);
    }
  }
  if (dir) {
    const double o[kFusedParts] = {ls[0], ls[1], ls[2], ls[3], sp[0], sp[1], sp[2],
                                   xp[0], xp[1], xp[2], xp[3], xp[4], xp[5]};
    block_sum_emit<kFusedParts>(o, sm.red,
                                [&](int j, double a) { pout[(size_t)j * kInnerGrid + bid] = a; });
  } else {
    if (HS) {  // slots 0-2 (the last update's sums in step 2) are not read after a half-step
      const double v[9] = {0.0, 0.0, 0.0, mon[0], mon[1], mon[2], mon[3], 0.0, 0.0};
      double* pc = partsC + (size_t)bid * kNumPart;
      block_sum_emit<9>(v, sm.red, [&](int j, double a) { pc[j] = a; });
    }
    if (w0) {
      for (int k = i + 2; k < K; ++k) st->stop[k] = 1;  // (stop[i + 1] set by bb_step)
      if (HS) {
        st->pending = 1;
        st->t_hstep = wall_clock64();
      }
    }
  }
}

// ----------------------------------------------------------------------------- naive variant
// H-step of the naive symmetric variant (H <- W^T after each W-step): after H was set to
// W and the H-step's init ran at H = W, this keeps <C, P> for the monitor (as the first
// inner kernel of an H-step does) and marks the half-step stopped before inner iteration
// 0, so that its one step 2 forms the monitor sums of H = W without moving it.
__global__ __launch_bounds__(kThreads) void k_naive_hentry(const double* __restrict__ partsA,
                                                           int nb, State* __restrict__ st) {
  __shared__ double sred[kStage];
  if (st->done) return;
  double a1[1];
  load_slots<1>(partsA, nb, 0, a1);
  block_sum_wide<1>(a1, sred);
  if (threadIdx.x == 0) {
    st->m_CP = a1[0];
    st->stop[0] = 1;
  }
}

void launch_naive_hentry(const double* partsA, int nb, State* st, hipStream_t s) {
  hipLaunchKernelGGL(k_naive_hentry, dim3(1), dim3(kThreads), 0, s, partsA, nb, st);
}

// ----------------------------------------------------------------------------- launchers
int rank_pad(int r) {
  int rp = 4;
  while (rp < r) rp *= 2;
  return rp;
}

// Compute units of the current device (MI355X: 256), looked up once per device: the
// launchers ask on every launch.
static int64_t inner_cus() {
  static int cached[64] = {0};  // concurrent first lookups store the same value
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev >= 0 && dev < 64 && cached[dev] > 0) return cached[dev];
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  if (dev >= 0 && dev < 64) cached[dev] = cus;
  return cus;
}

// One workgroup per tile up to what stays resident at once (FP32 up to rank 32: three per
// CU, two where the grid also serves the fused kernels), at most kInnerGrid (the
// partial-sum rows).  A grid larger than the resident workgroups runs in two rounds, and
// the second round's workgroups start only when first-round ones end.
int inner_grid(int64_t n, int r, int esz, bool fused) {
  const int rp = rank_pad(r);
  const int tm = 8 * kThreads / rp;
  int64_t nt = (n + tm - 1) / tm;
  if (nt < 1) nt = 1;
  int64_t cap = kInnerGrid;
  if (esz == 4 && rp <= 32) {
    const int per_cu = fused ? fused_occupancy<float, 32>() : inner_occupancy<float, 32>();
    const int64_t res = per_cu * inner_cus();
    if (res < cap) cap = res;
  }
  return (int)(nt < cap ? nt : cap);
}

#define SNMF_DISPATCH_RP(rp, ...)                                   \
  switch (rp) {                                                     \
    case 4: { constexpr int RP = 4; __VA_ARGS__; } break;           \
    case 8: { constexpr int RP = 8; __VA_ARGS__; } break;           \
    case 16: { constexpr int RP = 16; __VA_ARGS__; } break;         \
    case 32: { constexpr int RP = 32; __VA_ARGS__; } break;         \
    default: { constexpr int RP = 64; __VA_ARGS__; } break;         \
  }

template <typename T>
void launch_init(const T* X, const T* P, const T* Bpart, int ksplit, int64_t bstride, T* C, T* g,
                 const T* LX, const T* GT, int64_t n, int r, int is_hstep, const KParams& kp,
                 State* st, double* partsA, hipStream_t s, const BMap& bm, int grid, T* Zn,
                 T* Dn, T* Dd, double* pout, T* Xs, T* gs) {
  if (grid <= 0) grid = inner_grid(n, r, (int)sizeof(T));
  if (Dd) {
    SNMF_DISPATCH_RP(rank_pad(r),
                     hipLaunchKernelGGL((k_init<T, RP, 1>), dim3(grid), dim3(kThreads), 0, s, X,
                                        P, Bpart, ksplit, bstride, C, g, LX, GT, n, r, is_hstep,
                                        kp, st, partsA, bm, Zn, Dn, Dd, pout, Xs, gs))
  } else {
    SNMF_DISPATCH_RP(rank_pad(r),
                     hipLaunchKernelGGL((k_init<T, RP, 0>), dim3(grid), dim3(kThreads), 0, s, X,
                                        P, Bpart, ksplit, bstride, C, g, LX, GT, n, r, is_hstep,
                                        kp, st, partsA, bm, Zn, Dn, Dd, pout, Xs, gs))
  }
}

template <typename T>
void launch_advance(T* X, T* g, T* Xs, T* gs, T* D, const T* C, const T* P, const T* GT,
                    const double* Gcur, const double* Gprev, int64_t n, int r, int K, int i,
                    int is_hstep, const KParams& kp, State* st, const double* pin, double* pout,
                    const double* partsA, double* partsC, double* trace, hipStream_t s,
                    int grid) {
  if (grid <= 0) grid = inner_grid(n, r, (int)sizeof(T));
  if (is_hstep) {
    SNMF_DISPATCH_RP(rank_pad(r),
                     hipLaunchKernelGGL((k_advance<T, RP, 1>), dim3(grid), dim3(kThreads), 0, s,
                                        X, g, Xs, gs, D, C, P, GT, Gcur, Gprev, n, r, K, i, kp,
                                        st, pin, pout, partsA, partsC, trace))
  } else {
    SNMF_DISPATCH_RP(rank_pad(r),
                     hipLaunchKernelGGL((k_advance<T, RP, 0>), dim3(grid), dim3(kThreads), 0, s,
                                        X, g, Xs, gs, D, C, P, GT, Gcur, Gprev, n, r, K, i, kp,
                                        st, pin, pout, partsA, partsC, trace))
  }
}

template <typename T>
void launch_step1(const T* X, const T* g, T* Z, T* D, const T* LdZ, const T* GT,
                  const double* Gcur, const double* Gprev, int64_t n, int r, int k, int phase,
                  int is_hstep, const KParams& kp, State* st, const double* partsA,
                  double* partsB, const double* partsC, double* trace, hipStream_t s,
                  const BMap& bm, int grid, int rd) {
  if (grid <= 0) grid = inner_grid(n, r, (int)sizeof(T));
  if (phase == 0) {
    SNMF_DISPATCH_RP(rank_pad(r),
                     hipLaunchKernelGGL((k_step1<T, RP, 0>), dim3(grid), dim3(kThreads), 0, s, X,
                                        g, Z, D, LdZ, GT, Gcur, Gprev, n, r, k, phase, is_hstep,
                                        kp, st, partsA, partsB, partsC, trace, bm, rd))
  } else {
    SNMF_DISPATCH_RP(rank_pad(r),
                     hipLaunchKernelGGL((k_step1<T, RP, 1>), dim3(grid), dim3(kThreads), 0, s, X,
                                        g, Z, D, LdZ, GT, Gcur, Gprev, n, r, k, phase, is_hstep,
                                        kp, st, partsA, partsB, partsC, trace, bm, rd))
  }
}

template <typename T>
void launch_step2(T* X, T* g, T* Z, T* D, const T* LS, const T* C, const T* P, T* LXb,
                  const T* GT, int64_t n, int r, int k, int phase, int is_hstep,
                  const KParams& kp, State* st, const double* partsB, const double* partsD,
                  int nbD, double* partsC, hipStream_t s, const BMap& bm, int grid,
                  int last_k, int rd) {
  if (grid <= 0) grid = inner_grid(n, r, (int)sizeof(T));
#define SNMF_STEP2(V)                                                                          \
  SNMF_DISPATCH_RP(rank_pad(r),                                                                \
                   hipLaunchKernelGGL((k_step2<T, RP, V>), dim3(grid), dim3(kThreads), 0, s, X, \
                                      g, Z, D, LS, C, P, LXb, GT, n, r, k, phase, is_hstep, kp, \
                                      st, partsB, partsD, nbD, partsC, bm, rd))
  if (phase != 0) {
    SNMF_STEP2(2)
  } else if (is_hstep && k >= last_k) {
    SNMF_STEP2(1)
  } else if (is_hstep) {
    SNMF_STEP2(3)
  } else {
    SNMF_STEP2(0)
  }
#undef SNMF_STEP2
}

#define SNMF_INST(T)                                                                            \
  template void launch_init<T>(const T*, const T*, const T*, int, int64_t, T*, T*, const T*,   \
                               const T*, int64_t, int, int, const KParams&, State*, double*,   \
                               hipStream_t, const BMap&, int, T*, T*, T*, double*, T*, T*);     \
  template void launch_advance<T>(T*, T*, T*, T*, T*, const T*, const T*, const T*,          \
                                  const double*, const double*, int64_t, int, int, int, int,   \
                                  const KParams&, State*, const double*, double*,              \
                                  const double*, double*, double*, hipStream_t, int);          \
  template void launch_step1<T>(const T*, const T*, T*, T*, const T*, const T*, const double*, \
                                const double*, int64_t, int, int, int, int, const KParams&,     \
                                State*, const double*, double*, const double*, double*,         \
                                hipStream_t, const BMap&, int, int);                            \
  template void launch_step2<T>(T*, T*, T*, T*, const T*, const T*, const T*, T*, const T*,    \
                                int64_t, int, int, int, int, const KParams&, State*,            \
                                const double*, const double*, int, double*, hipStream_t,        \
                                const BMap&, int, int, int);
SNMF_INST(float)
SNMF_INST(double)

}  // namespace snmf
