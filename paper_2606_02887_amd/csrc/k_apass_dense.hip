// The A-pass B = A P for dense symmetric A: the product that dominates the per-iteration
// cost O(n^2 r) of SNMPBB (Section 4.1 complexity list).  A is streamed once per call.
//
// * FP64: LDS-tiled VALU kernel (parity mode, small n).
// * FP32: MFMA v_mfma_f32_32x32x2f32.  Because A = A^T the kernel computes
//   B^T = P^T A: rows of A feed the MFMA "B" operand, so every lane reads consecutive
//   columns of one row of A and a wave touches two full 128-byte row segments per load.
// * split BF16: A = A_hi + A_lo and P = P_hi + P_lo (round-to-nearest-even BF16), with
//   A P ~= A_hi P_hi + A_hi P_lo + A_lo P_hi accumulated in FP32 on
//   v_mfma_f32_32x32x16_bf16.  P is pre-split and transposed (r x ldp) so both operands
//   are read as 16-byte vectors.
// Every variant writes split-K partial products Bpart[s] (n x r each) that the half-step's
// init kernel adds in a fixed order.
#include "common.hpp"
#include "kernels.hpp"
#include "rho.hpp"

namespace snmf {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------------------- FP64
__global__ __launch_bounds__(256) void k_apass_f64(const double* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ P, int64_t n, int r,
                                                   double* __restrict__ B,
                                                   const State* __restrict__ st) {
  if (st->done) return;
  constexpr int TR = 32, TK = 64;
  __shared__ double sA[TR][TK + 1];
  __shared__ double sP[TK][kMaxRank];
  const int tid = threadIdx.x, c = tid & 63, rs = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * TR;
  double acc[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) acc[p] = 0.0;
  for (int64_t k0 = 0; k0 < n; k0 += TK) {
    __syncthreads();
    for (int e = tid; e < TR * TK; e += 256) {
      const int i = e / TK, kk = e % TK;
      const int64_t row = row0 + i, col = k0 + kk;
      sA[i][kk] = (row < n && col < n) ? A[row * lda + col] : 0.0;
    }
    for (int e = tid; e < TK * kMaxRank; e += 256) {
      const int kk = e / kMaxRank, cc = e % kMaxRank;
      const int64_t k = k0 + kk;
      sP[kk][cc] = (k < n && cc < r) ? P[k * r + cc] : 0.0;
    }
    __syncthreads();
    if (c < r) {
#pragma unroll 4
      for (int kk = 0; kk < TK; ++kk) {
        const double pv = sP[kk][c];
#pragma unroll
        for (int p = 0; p < 8; ++p) acc[p] = __builtin_fma(sA[rs + 4 * p][kk], pv, acc[p]);
      }
    }
  }
  if (c < r) {
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int64_t row = row0 + rs + 4 * p;
      if (row < n) B[row * r + c] = acc[p];
    }
  }
}

// ----------------------------------------------------------------------------- FP32 MFMA
// Grid: x = blocks of 256 output rows (4 waves x 64), y = K splits of kchunk rows of A.
// Wave w handles output rows j0..j0+63 (two MFMA N-blocks of 32) and all r <= 64
// columns (one or two MFMA M-blocks).  Per k-pair a lane loads A[k+h][j0+c] and
// A[k+h][j0+32+c] (h = lane/32, c = lane%32) and P[k+h][c], P[k+h][32+c].
template <int NMB>
__global__ __launch_bounds__(256) void k_apass_f32(const float* __restrict__ A, int64_t lda,
                                                   const float* __restrict__ P, int64_t n, int r,
                                                   int64_t kchunk, float* __restrict__ Bpart,
                                                   int64_t pstride, const State* __restrict__ st) {
  if (st->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 31, h = lane >> 5;
  const int64_t j0 = ((int64_t)blockIdx.x * 4 + wave) * 64;
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  const int64_t ke = kb + kchunk < n ? kb + kchunk : n;
  f32x16 acc[NMB][2];
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[mb][nb][v] = 0.0f;
  const bool jok0 = j0 + c < n, jok1 = j0 + 32 + c < n;
  const bool mok0 = c < r, mok1 = 32 + c < r;
  const float* arow = A + j0 + c;
  constexpr int U = 8;  // k-pairs per batch of loads
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
  // two batches of loads in flight: the next batch is requested before this one's MFMAs
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
    const float a0 = (kin && jok0) ? arow[kk * lda] : 0.0f;
    const float a1 = (kin && jok1) ? arow[kk * lda + 32] : 0.0f;
    const float p0 = (kin && mok0) ? P[kk * r + c] : 0.0f;
    const float p1 = (NMB > 1 && kin && mok1) ? P[kk * r + 32 + c] : 0.0f;
    acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(p0, a0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(p0, a1, acc[0][1], 0, 0, 0);
    if (NMB > 1) {
      acc[NMB - 1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(p1, a0, acc[NMB - 1][0], 0, 0, 0);
      acc[NMB - 1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(p1, a1, acc[NMB - 1][1], 0, 0, 0);
    }
  }
  // D[m][j] of block (mb, nb): lane holds j = j0 + 32 nb + c and
  // m = 32 mb + 8 (v/4) + 4 h + v%4 in register v.
  float* out = Bpart + (int64_t)blockIdx.y * pstride;
#pragma unroll
  for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int64_t j = j0 + 32 * nb + c;
      if (j < n) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int m = 32 * mb + 8 * (v >> 2) + 4 * h + (v & 3);
          if (m < r) out[j * r + m] = acc[mb][nb][v];
        }
      }
    }
}

// FP32, wide loads (r in (32, 64], r even, lda % 4 == 0): a workgroup computes
// 128-row output tiles over K ranges; its four waves take contiguous quarters of a range.
// Per k-pair a lane loads A[k+h][j0+4c .. +3] (one 16-byte vector) and P[k+h][2c, 2c+1]
// (one 8-byte vector): MFMA N-block q covers the columns j0 + 4c + q, M-block b the ranks
// m = 2c + b.  The four wave tiles are added in LDS in wave order (deterministic) and
// written as coalesced rows of a partial product.
// Balanced split, every workgroup doing about the same MFMA work so the grid fills the CUs
// evenly (two workgroups per CU):
//  * nband full bands of `band` rows of K: workgroup w < nband gx takes rows
//    [b band, (b + 1) band) of tile w % gx (b = w / gx) into partial panel b;
//    consecutive workgroups take consecutive tiles of one band, so the workgroups in
//    flight read the same rows of A at the same time;
//  * the rows left, [nband band, n) of every tile, taken tile by tile, are cut into
//    chunks of `rchunk` rows, one per remaining workgroup; a chunk covers one K range of
//    one tile or the end of one tile and the start of the next.  Tile t receives the
//    chunks of workgroups first(t) .. last(t) (counted from the first such workgroup,
//    first(t) = floor(t lr / rchunk), lr the rows left per tile); workgroup w writes its
//    part of t to panel nband + w - first(t), and last(t) writes zeros to the panels
//    above its own up to nslot - 1.
// So every tile has exactly nslot panels, added in panel order by the consumer.
// With rj.G set, the grid has one more workgroup (number rho_wg): it computes
// rho = ||G||_2 (rho.hpp) beside the tiles.  The register bound of two waves per SIMD and
// the 64 KB of LDS leave room on a CU for it next to a tile workgroup (the tiles take one
// slot fewer than two per CU), so rho (56 us alone at r = 64) adds only the slowdown of
// the tile workgroup that shares its CU.  With two workgroups per CU, workgroups i and
// i + CUs are dispatched to the same CU, so the host places rho at the last index minus
// the CU count, beside the last workgroup: a chunk of the rows after the bands, which
// carries fewer rows than a band.
__global__ __launch_bounds__(256, 2) void k_apass_f32w(const float* __restrict__ A, int64_t lda,
                                                       const float* __restrict__ P, int64_t n,
                                                       int r, int64_t band, int nband,
                                                       int64_t rchunk, int nslot,
                                                       float* __restrict__ Bpart, int64_t pstride,
                                                       const State* __restrict__ st, RhoJob rj,
                                                       int rho_wg) {
  if (st->done) return;
  if (rj.G && (int)blockIdx.x == rho_wg) {
    rho_body(rj.G, rj.r, rj.st);
    return;
  }
  __shared__ float sacc[2 * 8 * 16 * 64];  // [slot][block(mb,nb)][v][lane], 64 KB
  // the wave index is uniform: K ranges, batch counts and loop control stay scalar
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = lane & 31, h = lane >> 5;
  const int64_t w = (rj.G && (int)blockIdx.x > rho_wg) ? blockIdx.x - 1 : blockIdx.x;
  const int64_t gx = (n + 127) / 128;
  const int64_t nfull = (int64_t)nband * gx;
  const int64_t r0 = (int64_t)nband * band;  // first row of K after the full bands
  const int64_t lr = n > r0 ? n - r0 : 0;    // rows of K left per tile
  const int64_t wp = w - nfull;
  // segment cursor over this workgroup's share: one segment in a full band, else
  // [gs, gend) of the tile-major space of the rows left
  int64_t gs = 0, gend = 1;
  if (w >= nfull) {
    gs = wp * rchunk;
    gend = gs + rchunk < gx * lr ? gs + rchunk : gx * lr;
  }
  while (gs < gend) {
    int64_t t, kb, ke;  // tile and its K range [kb, ke)
    int slot, zend;     // panel written; panels slot + 1 .. zend - 1 get zeros
    if (w < nfull) {
      const int64_t bd = w / gx;
      t = w - bd * gx;
      kb = bd * band;
      ke = kb + band < n ? kb + band : n;
      slot = (int)bd;
      zend = slot + 1;
      gs = gend;
    } else {
      t = gs / lr;
      const int64_t o = gs - t * lr;
      kb = r0 + o;
      ke = r0 + (o + (gend - gs) < lr ? o + (gend - gs) : lr);
      slot = nband + (int)(wp - (t * lr) / rchunk);
      const bool last = (t * lr + lr - 1) / rchunk == wp;  // last contributor of tile t
      zend = last ? nslot : slot + 1;
      gs += ke - kb;
    }
    const int64_t j0 = t * 128;
    const int64_t kq = ((ke - kb + 7) / 8) * 2;      // per-wave share, even
    const int64_t wb = kb + wave * kq < ke ? kb + wave * kq : ke;
    const int64_t we = wb + kq < ke ? wb + kq : ke;  // wb <= we <= ke
    f32x16 acc[2][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[mb][nb][v] = 0.0f;
    const int64_t jc = j0 + 4 * c;
    const bool jok = jc + 3 < n;                 // n % 4 == 0 on this path
    const bool mok = 2 * c + 1 < r;              // r even on this path
    // Out-of-range lanes read a clamped, valid address instead of being predicated: the
    // loads stay unconditional (so the compiler keeps the prefetched batch in flight
    // across the MFMAs), and a garbage column of A or rank of P only reaches an output
    // column or rank that is never stored.
    const float* arow = A + (jok ? jc : n - 4);
    const float* prow = P + (mok ? 2 * c : 0);
    constexpr int U = 6;  // k-pairs per batch of loads (2: 91.3 us, 4: 90.7, 6: 89.0; 8 spills)
    f32x4v xa[U], xb[U];
    float2 ya[U], yb[U];
    const f32x4v z4 = {0.f, 0.f, 0.f, 0.f};
    const float2 z2 = {0.f, 0.f};
    auto load = [&](f32x4v (&x)[U], float2 (&y)[U], int64_t k0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t kk = k0 + 2 * u + h;
        x[u] = __builtin_nontemporal_load((const f32x4v*)(arow + kk * lda));
        y[u] = *(const float2*)(prow + kk * r);
      }
    };
    auto mma = [&](const f32x4v (&x)[U], const float2 (&y)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float av[4] = {x[u][0], x[u][1], x[u][2], x[u][3]};
        const float pv[2] = {y[u].x, y[u].y};
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
          for (int mb = 0; mb < 2; ++mb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(pv[mb], av[nb], acc[mb][nb], 0, 0, 0);
      }
    };
    // full batches of U k-pairs, two in flight: each loop step issues the loads of the
    // next two batches among the MFMAs of the current two, one load per four MFMAs (the
    // scheduling-group barriers below fix that order).  A wave issues in order and
    // stalls on a load the memory pipeline cannot take yet, so loads issued in bursts
    // held back MFMAs that were ready (at n = 8192: 106.5 us in bursts, 88-91 us
    // interleaved, TCP stalled on pending data 65% of the cycles with MFMA 49% busy
    // before).  The prefetch of a batch beyond the last one re-reads the last batch (a
    // valid address) and is never used, which keeps every load unconditional.
    const int64_t nbat = (we - wb) / (2 * U);
    const int64_t klast = wb + (nbat > 0 ? nbat - 1 : 0) * 2 * U;
    int64_t k = wb;
    if (nbat > 0) load(xa, ya, k);
    int64_t b = 0;
    for (; b + 2 <= nbat; b += 2) {
      load(xb, yb, k + 2 * U);
      mma(xa, ya);
      load(xa, ya, k + 4 * U < klast ? k + 4 * U : klast);
      mma(xb, yb);
      k += 4 * U;
#pragma unroll
      for (int i = 0; i < 4 * U; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // one global load
        __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);  // four MFMAs
      }
    }
    if (b < nbat) mma(xa, ya);  // odd batch count: xa holds the last batch
    // the rows left (fewer than a batch): one batch of masked loads, all issued before
    // the first wait, and MFMAs for the k-pairs present only
    k = wb + nbat * 2 * U;
    if (k < we) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t kk = k + 2 * u + h;
        const bool kin = kk < we;
        xa[u] = (kin && jok) ? *(const f32x4v*)(arow + kk * lda) : z4;
        ya[u] = (kin && mok) ? *(const float2*)(prow + kk * r) : z2;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k + 2 * u < we) {
          const float av[4] = {xa[u][0], xa[u][1], xa[u][2], xa[u][3]};
          const float pv[2] = {ya[u].x, ya[u].y};
#pragma unroll
          for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(pv[mb], av[nb], acc[mb][nb], 0, 0, 0);
        }
      }
    }
    // the four K-quarter tiles, added pairwise in a fixed order in 64 KB of LDS:
    // (w0 + w1) + (w2 + w3), the total in slot 0
    auto put = [&](int sl) {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
          for (int v = 0; v < 16; ++v) sacc[((sl * 8 + mb * 4 + nb) * 16 + v) * 64 + lane] = acc[mb][nb][v];
    };
    auto add = [&](int sl) {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[mb][nb][v] += sacc[((sl * 8 + mb * 4 + nb) * 16 + v) * 64 + lane];
    };
    if (wave & 1) put(wave >> 1);
    __syncthreads();
    if (!(wave & 1)) add(wave >> 1);
    __syncthreads();
    if (wave == 2) put(0);
    __syncthreads();
    if (wave == 0) {
      add(0);
      put(0);
    }
    __syncthreads();
    // element (jl, m) of the 128 x r tile: jl = 4c + nb, m = 2 mrow + mb with
    // mrow = 8 (v/4) + 4 h + v%4
    float* out = Bpart + (int64_t)slot * pstride;
    for (int e = threadIdx.x; e < 128 * 64; e += 256) {
      const int jl = e >> 6, m = e & 63;
      const int64_t jj = j0 + jl;
      if (m < r && jj < n) {
        const int cc = jl >> 2, nb = jl & 3, mb = m & 1, mrow = m >> 1;
        const int hh = (mrow >> 2) & 1, v = 4 * (mrow >> 3) + (mrow & 3);
        const int idx = ((mb * 4 + nb) * 16 + v) * 64 + 32 * hh + cc;
        out[jj * r + m] = sacc[idx];
        for (int z = slot + 1; z < zend; ++z) Bpart[(int64_t)z * pstride + jj * r + m] = 0.0f;
      }
    }
    __syncthreads();  // sacc is reused by the next range
  }
}

// ----------------------------------------------------------------------------- split BF16
// Grid: x = blocks of 128 output rows (4 waves x 32), y = K splits (kchunk multiple of 64).
// Per 64-column slab of A a lane loads 32 consecutive BF16 of its row (four 16-byte
// vectors, lanes l and l+32 together cover 128 contiguous bytes) from A_hi and A_lo; the
// matching 64-column slab of Pt_hi/Pt_lo (r x 64) is staged once per workgroup in LDS
// (double-buffered) and shared by the four waves.  MFMA step s (0..3) uses lane (h, row)
// k-values k + 32h + 8s .. +7.  The next slab's A vectors are loaded before the current
// slab's MFMAs are issued.
template <int NNB>
__global__ __launch_bounds__(256) void k_apass_bf16x3(const uint16_t* __restrict__ Ahi,
                                                      const uint16_t* __restrict__ Alo, int64_t ldb,
                                                      const uint16_t* __restrict__ Pthi,
                                                      const uint16_t* __restrict__ Ptlo, int64_t ldp,
                                                      int64_t n, int r, int64_t kchunk,
                                                      float* __restrict__ Bpart, int64_t pstride,
                                                      const State* __restrict__ st, RhoJob rj) {
  if (st->done) return;
  // with rj.G set, one more row of workgroups: its first computes rho = ||G||_2 (the grid
  // is resident at once, so it runs beside the tiles)
  if (rj.G && blockIdx.y == gridDim.y - 1) {
    if (blockIdx.x == 0) {
      // rho, not the tiles, sets the length of this launch at r = 64: its waves take
      // issue priority over the tile waves that share its CU (split-BF16 solve at n = 8192:
      // 2712 -> 2895 outer iterations/s)
      __builtin_amdgcn_s_setprio(3);
      rho_body(rj.G, rj.r, rj.st);
    }
    return;
  }
  constexpr int KS = 64;                    // k per slab
  constexpr int PROW = KS + 8;              // LDS row pitch (bf16), keeps 16-byte alignment
  __shared__ __attribute__((aligned(16))) uint16_t sP[2][2][32 * NNB * PROW];  // [buf][hi/lo]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 31, h = lane >> 5;
  const int64_t j0 = ((int64_t)blockIdx.x * 4 + wave) * 32;
  const int64_t kb = (int64_t)blockIdx.y * kchunk;
  int64_t ke = kb + kchunk;
  if (ke > ldb) ke = ldb;
  f32x16 acc[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[nb][v] = 0.0f;
  // Rows past n and Pt rows past r read the last valid row instead: they feed only output
  // rows and columns that are never stored.  Loads without a condition (and a prefetch
  // past the last slab that re-reads it) keep the loop free of branches, so the compiler
  // counts the loads in flight exactly instead of waiting for all of them, the prefetch
  // included, before every LDS stage.
  const int64_t j = j0 + c < n ? j0 + c : n - 1;
  const uint16_t* ah = Ahi + j * ldb + 32 * h;
  const uint16_t* al = Alo + j * ldb + 32 * h;
  // Pt staging: the slab is 32*NNB rows (m) x 64 bf16 for hi and lo, i.e. NVEC 16-byte
  // vectors, NPT per thread.  Global loads of the next slab are issued before the next
  // A vectors and written to LDS only after the current MFMAs, so no wait on the A
  // prefetch is needed to stage.
  constexpr int NVEC = 2 * 32 * NNB * (KS / 8);
  constexpr int NPT = NVEC / 256;
  u16x8 pt[NPT];
  auto stage_load = [&](int64_t k) {
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int e = tid + 256 * q;
      const int which = e / (32 * NNB * (KS / 8));
      const int rem = e - which * (32 * NNB * (KS / 8));
      const int m = rem / (KS / 8), qq = rem - m * (KS / 8);
      const int mm = m < r ? m : r - 1;
      pt[q] = *(const u16x8*)((which ? Ptlo : Pthi) + (int64_t)mm * ldp + k + 8 * qq);
    }
  };
  auto stage_store = [&](int b) {
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int e = tid + 256 * q;
      const int which = e / (32 * NNB * (KS / 8));
      const int rem = e - which * (32 * NNB * (KS / 8));
      const int m = rem / (KS / 8), qq = rem - m * (KS / 8);
      *(u16x8*)&sP[b][which][m * PROW + 8 * qq] = pt[q];
    }
  };
  u16x8 xa[2][4], xn[2][4];
  auto load_a = [&](u16x8 (&x)[2][4], int64_t k) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      x[0][s] = *(const u16x8*)(ah + k + 8 * s);
      x[1][s] = *(const u16x8*)(al + k + 8 * s);
    }
  };
  int buf = 0;
  if (kb < ke) {
    stage_load(kb);
    load_a(xa, kb);
    stage_store(0);
  }
  __syncthreads();
  for (int64_t k = kb; k < ke; k += KS) {
    const int64_t kn = k + KS < ke ? k + KS : k;
    stage_load(kn);
    load_a(xn, kn);
#pragma unroll
    for (int nb = 0; nb < NNB; ++nb) {
      const int m = 32 * nb + c;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const u16x8 bh = *(const u16x8*)&sP[buf][0][m * PROW + 32 * h + 8 * s];
        const u16x8 bl = *(const u16x8*)&sP[buf][1][m * PROW + 32 * h + 8 * s];
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xa[0][s]),
                                                          __builtin_bit_cast(bf16x8, bh), acc[nb], 0, 0, 0);
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xa[0][s]),
                                                          __builtin_bit_cast(bf16x8, bl), acc[nb], 0, 0, 0);
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xa[1][s]),
                                                          __builtin_bit_cast(bf16x8, bh), acc[nb], 0, 0, 0);
      }
    }
    stage_store(buf ^ 1);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      xa[0][s] = xn[0][s];
      xa[1][s] = xn[1][s];
    }
    buf ^= 1;
  }
  // D[row][col]: row = 8 (v/4) + 4 h + v%4 (output row j0 + row), col = lane%32 (m).
  float* out = Bpart + (int64_t)blockIdx.y * pstride;
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) {
    const int m = 32 * nb + c;
    if (m < r) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t jj = j0 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (jj < n) out[jj * r + m] = acc[nb][v];
      }
    }
  }
}

// ----------------------------------------------------------------------------- partial sum
// out = part[0] + part[1] + ... (left to right, the order the init kernel uses).
// ks <= kMaxKSplit: an element's partials are all loaded before the first is added.
template <typename T>
__global__ __launch_bounds__(256) void k_sum_parts(const T* __restrict__ part, int ks,
                                                   int64_t stride, T* __restrict__ out, int64_t N) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256) {
    T v[kMaxKSplit];
#pragma unroll
    for (int s = 0; s < kMaxKSplit; ++s) v[s] = s < ks ? part[s * stride + e] : T(0);
    T b = T(0);
#pragma unroll
    for (int s = 0; s < kMaxKSplit; ++s)
      if (s < ks) b += v[s];
    out[e] = b;
  }
}

template <typename T>
void launch_sum_parts(const T* part, int ks, int64_t stride, T* out, int64_t N, hipStream_t s) {
  int64_t nb = (N + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_sum_parts<T>, dim3((unsigned)nb), dim3(256), 0, s, part, ks, stride, out, N);
}
template void launch_sum_parts<float>(const float*, int, int64_t, float*, int64_t, hipStream_t);
template void launch_sum_parts<double>(const double*, int, int64_t, double*, int64_t, hipStream_t);

// ----------------------------------------------------------------------------- launchers
void launch_apass_f64(const double* A, int64_t lda, const double* P, int64_t n, int r, double* B,
                      const State* st, hipStream_t s) {
  const unsigned gx = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_apass_f64, dim3(gx), dim3(256), 0, s, A, lda, P, n, r, B, st);
}

bool dense_f32_wide(int64_t n, int64_t lda, int r, const void* A) {
  return r > 32 && r % 2 == 0 && n % 4 == 0 && lda % 4 == 0 && ((uintptr_t)A & 15) == 0;
}

// Compute units of the current device (MI355X: 256).
static int64_t device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return cus;
}

constexpr int64_t kDelta = 96;
DenseSplit plan_dense_f32(int64_t n, int64_t lda, int r, const void* A) {
  DenseSplit d;
  if (dense_f32_wide(n, lda, r, A)) {
    d.wide = true;
    d.gx = (n + 127) / 128;
    // two tile workgroups per CU less one slot kept for the rho workgroup (511 at
    // n = 8192): q full bands of one workgroup per tile, the m workgroups left sharing the
    // rows after them.  Bands of at least 256 rows, and at most kMaxKSplit - 3 of them so
    // that q plus the (at most 2) panels of the rows left fit in kMaxKSplit.  At n = 8192:
    // 7 bands of 1040 rows and 63 chunks of 928.  Measured with loads issued in bursts:
    // whole K splits (7 per tile, 448 workgroups) 115.6 us, equal chunks without bands
    // 113.3 us, these bands 107.8 us.
    const int64_t gx = d.gx;
    const int64_t nwg = 2 * device_cus() - 1;
    int64_t q = nwg / gx, m = nwg % gx;
    int64_t qmax = n / 256 < kMaxKSplit - 3 ? n / 256 : kMaxKSplit - 3;
    if (qmax < 1) qmax = 1;
    if (q >= qmax) {
      q = qmax;
      m = 0;
    }
    auto r4 = [](int64_t x) { return (x + 3) / 4 * 4; };
    int64_t band = 0, lr = n, rchunk = 0;
    if (q == 0) {
      rchunk = r4((gx * n + m - 1) / m);
    } else {
      // with rows left over, the chunks of the rows left are about kDelta rows shorter
      // than a band: a chunk that ends inside a tile pays a second pipeline start and
      // epilogue (at n = 8192, kDelta 0 / 48 / 96 / 160: 110.7 / 112.9 / 107.8 / 108.0 us;
      // one workgroup per (tile, band) at 8 bands and no rho slot: 106.0 us)
      band = m ? r4((n * gx + m * kDelta + q * gx + m - 1) / (q * gx + m)) : r4((n + q - 1) / q);
      if (m && q * band >= n) {
        m = 0;
        band = r4((n + q - 1) / q);
      }
      while (q > 1 && (q - 1) * band >= n) --q;
      lr = n > q * band ? n - q * band : 0;
      if (m && lr) rchunk = r4((gx * lr + m - 1) / m);
    }
    if (rchunk && rchunk < 4) rchunk = 4;
    int nslot = (int)q;
    int64_t npart = 0;
    if (rchunk) {
      npart = (gx * lr + rchunk - 1) / rchunk;
      int64_t cnt = 0;
      for (int64_t t = 0; t < gx; ++t) {
        const int64_t c = (t * lr + lr - 1) / rchunk - (t * lr) / rchunk + 1;
        if (c > cnt) cnt = c;
      }
      nslot += (int)cnt;
    }
    d.kchunk = band;
    d.nband = (int)q;
    d.rchunk = rchunk;
    d.ksplit = nslot;  // <= kMaxKSplit
    d.nwg = q * gx + npart;
    return d;
  }
  const int64_t gx = (n + 255) / 256;
  int64_t ks = (512 + gx - 1) / gx;
  const int64_t kmax = (n + 63) / 64;
  if (ks > kmax) ks = kmax;
  if (ks < 1) ks = 1;
  if (ks > kMaxKSplit) ks = kMaxKSplit;
  int64_t kc = (n + ks - 1) / ks;
  kc = (kc + 15) / 16 * 16;
  d.kchunk = kc;
  d.ksplit = (int)((n + kc - 1) / kc);
  d.gx = gx;
  return d;
}

void launch_apass_f32(const float* A, int64_t lda, const float* P, int64_t n, int r,
                      const DenseSplit& d, float* Bpart, int64_t pstride, const State* st,
                      hipStream_t s, const RhoJob& rj) {
  dim3 grid((unsigned)d.gx, (unsigned)d.ksplit);
  if (d.wide) {
    const int64_t total = d.nwg + (rj.G ? 1 : 0);
    int rho_wg = (int)total - 1;
    if (rj.G) {
      int dev = 0, cus = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
          cus > 0 && total - 1 - cus >= 0)
        rho_wg = (int)(total - 1 - cus);
    }
    hipLaunchKernelGGL(k_apass_f32w, dim3((unsigned)total), dim3(256), 0, s, A, lda, P, n, r,
                       d.kchunk, d.nband, d.rchunk, d.ksplit, Bpart, pstride, st, rj, rho_wg);
    return;
  }
  if (rj.G) launch_rho(rj.G, rj.r, rj.st, s);
  if (r > 32)
    hipLaunchKernelGGL(k_apass_f32<2>, grid, dim3(256), 0, s, A, lda, P, n, r, d.kchunk, Bpart,
                       pstride, st);
  else
    hipLaunchKernelGGL(k_apass_f32<1>, grid, dim3(256), 0, s, A, lda, P, n, r, d.kchunk, Bpart,
                       pstride, st);
}

DenseSplit plan_dense_bf16(int64_t n) {
  DenseSplit d;
  const int64_t ldb = (n + 63) / 64 * 64;
  const int64_t gx = (n + 127) / 128;
  int64_t ks = (512 + gx - 1) / gx;
  const int64_t kmax = ldb / 64;
  if (ks > kmax) ks = kmax;
  if (ks < 1) ks = 1;
  if (ks > kMaxKSplit) ks = kMaxKSplit;
  int64_t kc = (ldb + ks - 1) / ks;
  kc = (kc + 63) / 64 * 64;
  d.kchunk = kc;
  d.ksplit = (int)((ldb + kc - 1) / kc);
  d.gx = gx;
  return d;
}

void launch_apass_bf16x3(const uint16_t* Ahi, const uint16_t* Alo, int64_t ldb,
                         const uint16_t* Pthi, const uint16_t* Ptlo, int64_t ldp, int64_t n, int r,
                         const DenseSplit& d, float* Bpart, int64_t pstride, const State* st,
                         hipStream_t s, const RhoJob& rj) {
  dim3 grid((unsigned)d.gx, (unsigned)d.ksplit + (rj.G ? 1u : 0u));
  if (r > 32)
    hipLaunchKernelGGL(k_apass_bf16x3<2>, grid, dim3(256), 0, s, Ahi, Alo, ldb, Pthi, Ptlo, ldp,
                       n, r, d.kchunk, Bpart, pstride, st, rj);
  else
    hipLaunchKernelGGL(k_apass_bf16x3<1>, grid, dim3(256), 0, s, Ahi, Alo, ldb, Pthi, Ptlo, ldp,
                       n, r, d.kchunk, Bpart, pstride, st, rj);
}

}  // namespace snmf
