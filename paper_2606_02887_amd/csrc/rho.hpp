// rho = ||G||_2 = lambda_max(G) of the symmetric positive semidefinite r x r Gram matrix
// G = P^T P: the scale rho_0 = ||H H^T||_2 of the first projection (Section 2.4).  One
// workgroup of 256 threads computes it in two phases; the body is shared by the stand-alone
// kernels and by A-pass kernels that run it in one extra workgroup beside their tiles.
//
// 1. Lanczos from q_1 = r^(-1/2) 1 over the four wavefronts: lane i of wavefront w holds
//    G[i][16w .. 16w+15] in registers, the four partial products of G q are added in LDS
//    in wavefront order (one barrier per step), the two inner products of a step are DPP
//    wave sums, and the normalisation uses b^(-1) = (b^2)^(-1/2) from the hardware
//    estimate plus two Newton steps, so a step has no division and no square root.
//    T = tridiag(b, a, b) has the spectrum of G on the Krylov space; the process stops
//    early when that space is invariant (b^2 <= (1e-15 ||G||_F)^2).  The bounds
//    lo = max a_k <= lambda_max(T) (interlacing) and hi (Gershgorin) are kept on the way.
// 2. Multisection on T: each round places 256 shifts x evenly in [lo, hi], one per
//    thread, and keeps the subinterval where x I - T turns positive definite.  The test
//    runs the leading principal minors s_k = det(x I - T_k),
//        s_k = (x - a_k) s_{k-1} - b_{k-1}^2 s_{k-2},   s_0 = 1, s_{-1} = 0,
//    which are all positive exactly when x > lambda_max(T).  The recurrence has no
//    division; T is scaled by a power of two so that |x - a_k| <= 2 and b_k^2 <= 1, and
//    every four steps the pair (s_k, s_{k-1}) is rescaled by a power of two (exact, signs
//    kept), so neither overflows nor underflows while all minors stay positive.  Lane k
//    holds row k of T, read by every lane of the wave as it goes (no LDS in the loop).  The
//    rounding errors of the recurrence amount to relative perturbations of a few units of
//    roundoff in the entries of x I - T, so the computed answer is exact for a matrix
//    within a few ulps of ||T|| of T.
// Without re-orthogonalisation the extreme Ritz value is still accurate: loss of
// orthogonality only adds copies of converged Ritz values (Paige), and r steps span the
// whole space in exact arithmetic.  G >= 0 elementwise (the Gram of a nonnegative
// factor), so its Perron vector is nonnegative and the all-ones start has a nonzero
// component along it.
#pragma once

#include "common.hpp"

namespace snmf {

// (x)^(-1/2) for x > 0: hardware estimate, then two Newton steps y <- y (3 - x y^2) / 2.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = __builtin_fma(-(x * y), y, 1.0);
    y = __builtin_fma(0.5 * e, y, y);
  }
  return y;
}

// Whole workgroup (kThreads threads) must call; writes st->rho, or flags a breakdown when
// the result is not a positive finite number.
__device__ __forceinline__ void rho_body(const double* __restrict__ G, int r,
                                         State* __restrict__ st) {
  constexpr int kW = kThreads / kWave;   // 4 wavefronts
  constexpr int kC = kMaxRank / kW;      // 16 columns of G per wavefront
  // sv[w]: wavefront w's own copy of the Lanczos vector (written and read by w only);
  // sz[parity][i][w]: partial products (G v)_i over wavefront w's columns, double
  // buffered by step parity so one barrier per step suffices; sA[k] = a_k 2^-e and
  // sB[k] = b_{k-1}^2 2^-2e, the scaled tridiagonal (sB[0] = 0, padding decoupled)
  __shared__ __attribute__((aligned(16))) double sv[kW][kMaxRank];
  __shared__ __attribute__((aligned(16))) double sz[2][kMaxRank][kW];
  __shared__ double sA[kMaxRank], sB[kMaxRank];
  __shared__ double s_lo, s_hi;
  __shared__ int sfirst[kW];
  __shared__ int s_m, s_ex;
  const int t = threadIdx.x;
  const int i = t & (kWave - 1), wv = t / kWave;
  {
    double grow[kC];
    double gn2 = 0.0;
#pragma unroll
    for (int c = 0; c < kC; ++c) {
      const int k = wv * kC + c;
      grow[c] = (i < r && k < r) ? G[i * r + k] : 0.0;
      gn2 = __builtin_fma(grow[c], grow[c], gn2);
    }
    __syncthreads();  // every wave reuses sz[0] below for ||G||_F^2
    sz[0][i][wv] = gn2;
    __syncthreads();
    const double4 g4 = *(const double4*)&sz[0][i][0];
    const double tol2 = 1e-30 * wave_sum((g4.x + g4.y) + (g4.z + g4.w));
    __syncthreads();
    // G v is formed on the unnormalised vector v and scaled by 1/||v|| afterwards, so the
    // reciprocal square root of a step overlaps the broadcast and product of the next.
    // Every wavefront runs the same scalar recurrence on the same data, so all four hold
    // identical a_j, b_j and q (bitwise) without further exchange.
    double v = i < r ? 1.0 : 0.0;
    double rb = 1.0 / sqrt((double)r);
    double q = v * rb, qprev = 0.0, bprev = 0.0;
    double lo = -1e300, hi = -1e300;  // max a_k and the Gershgorin bound, uniform
    double myA = 0.0, myB2 = 0.0;     // lane j keeps a_j and b_j^2
    int m = 0;
    sv[wv][i] = v;
    __builtin_amdgcn_wave_barrier();
    for (int j = 0; j < r; ++j) {
      double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
#pragma unroll
      for (int c = 0; c < kC; c += 4) {
        const double2 u = *(const double2*)&sv[wv][wv * kC + c];
        const double2 u2 = *(const double2*)&sv[wv][wv * kC + c + 2];
        w0 = __builtin_fma(grow[c], u.x, w0);
        w1 = __builtin_fma(grow[c + 1], u.y, w1);
        w2 = __builtin_fma(grow[c + 2], u2.x, w2);
        w3 = __builtin_fma(grow[c + 3], u2.y, w3);
      }
      const int par = j & 1;
      sz[par][i][wv] = (w0 + w1) + (w2 + w3);
      __syncthreads();
      const double4 z4 = *(const double4*)&sz[par][i][0];
      double w = ((z4.x + z4.y) + (z4.z + z4.w)) * rb;  // (G q_j)_i
      const double a = wave_sum(q * w);
      w = __builtin_fma(-a, q, w);
      w = __builtin_fma(-bprev, qprev, w);
      const double ww = wave_sum(w * w);
      m = j + 1;
      // b_j couples rows j and j + 1 of T; it is 0 when the process stops here
      const bool more = ww > tol2 && j + 1 < r;  // false for NaN as well
      if (more) {
        __builtin_amdgcn_wave_barrier();  // this wave has read the old vector
        sv[wv][i] = w;
        __builtin_amdgcn_wave_barrier();
      }
      const double rbn = more ? rsqrt_nr(ww) : 0.0;
      const double b = ww * rbn;
      lo = fmax(lo, a);
      hi = fmax(hi, a + bprev + b);
      if (i == j) {
        myA = a;
        myB2 = more ? ww : 0.0;
      }
      if (!more) break;
      qprev = q;
      q = w * rbn;
      bprev = b;
      rb = rbn;
    }
    if (wv == 0) {
      // scale T by 2^-ex (exact) so that hi lies in [1/2, 1)
      const bool okb = hi > 0.0 && hi < 1e300;
      int ex = 0;
      if (okb) frexp(hi, &ex);
      const int mpad = (m + 3) & ~3;
      if (i < mpad) {
        // padding rows sit two units below lo, so they never bound a shift from above
        sA[i] = i < m ? ldexp(myA, -ex) : ldexp(lo, -ex) - 2.0;
        if (i + 1 < kMaxRank) sB[i + 1] = i + 1 < m ? ldexp(myB2, -2 * ex) : 0.0;
      }
      if (i == 0) {
        sB[0] = 0.0;
        s_m = okb ? m : 0;
        s_ex = ex;
        s_lo = ldexp(lo, -ex);
        s_hi = ldexp(hi, -ex);
      }
    }
  }
  __syncthreads();
  const int m = s_m;  // 0: no positive finite bound, a breakdown
  const int ex = s_ex;
  const int mpad = (m + 3) & ~3;
  // lane k holds row k of the scaled T; each step broadcasts it with a lane read
  const double tA = i < mpad ? sA[i] : 0.0;
  const double tB = i < mpad ? sB[i] : 0.0;
  double L = s_lo, H = s_hi;
  const double div = (double)(kThreads + 1);
  for (int round = 0; m > 0 && round < 40 && H - L > 2.0 * 2.220446049250313e-16 * fabs(H);
       ++round) {
    const double x = L + (H - L) * (double)(t + 1) / div;
    double s1 = 1.0, s0 = 0.0;  // s_{k-1}, s_{k-2}
    bool above = true;
    for (int k = 0; k < mpad; k += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double ak = readlane_d(tA, k + u), bk = readlane_d(tB, k + u);
        const double s2 = __builtin_fma(x - ak, s1, -(bk * s0));
        above = above && s2 > 0.0;
        s0 = s1;
        s1 = s2;
      }
      const int e2 = __builtin_amdgcn_frexp_exp(s1);
      s1 = ldexp(s1, -e2);
      s0 = ldexp(s0, -e2);
    }
    // shifts above lambda_max form a suffix; find its first index
    const unsigned long long ab = __ballot(above);
    if (i == 0) sfirst[wv] = ab ? wv * kWave + __ffsll((long long)ab) - 1 : kThreads;
    __syncthreads();
    const int first = min(min(sfirst[0], sfirst[1]), min(sfirst[2], sfirst[3]));
    __syncthreads();
    const double nlo = L + (H - L) * (double)first / div;
    const double nhi = first < kThreads ? L + (H - L) * (double)(first + 1) / div : H;
    L = first > 0 ? nlo : L;
    H = nhi;
  }
  if (t == 0) {
    // rho = 0 (the partner block vanished) is reported by the first inner kernel of the
    // half-step, after the monitor record of the outer iteration that produced it
    const double rho = m > 0 ? ldexp(0.5 * (L + H), ex) : 0.0;
    st->rho = rho;
  }
}

}  // namespace snmf
