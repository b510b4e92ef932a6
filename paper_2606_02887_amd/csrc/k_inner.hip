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
//
// Thread layout of a workgroup (256 threads): column c = tid % RP, row slot
// rs = tid / RP; a tile holds TM = 8 * 256 / RP rows and each thread owns the 8 elements
// (rs + p * 256/RP, c), p = 0..7, of the tile.  RP is the rank rounded up to a power of 2.
#include "common.hpp"
#include "kernels.hpp"

namespace snmf {

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int RP>
struct TileCfg {
  static constexpr int RS = kThreads / RP;  // rows per pass
  static constexpr int TM = RS * 8;         // rows per tile
};

// acc[p] = sum_j sY[row_p][j] * sG[j][c] for the tile in LDS (row stride r).
template <typename T, int RP>
__device__ __forceinline__ void tile_gemm(const T* __restrict__ sY, const T* __restrict__ sG,
                                          int r, int c, int rs, T (&acc)[8]) {
  constexpr int RS = TileCfg<RP>::RS;
#pragma unroll
  for (int p = 0; p < 8; ++p) acc[p] = T(0);
  if (c >= r) return;
  for (int j = 0; j < r; ++j) {
    const T gj = sG[j * r + c];
#pragma unroll
    for (int p = 0; p < 8; ++p) acc[p] = fmaT(sY[(rs + p * RS) * r + j], gj, acc[p]);
  }
}

template <typename T, int RP>
struct Smem {
  T G[kMaxRank * kMaxRank];
  T a[TileCfg<RP>::TM * RP];
  T b[TileCfg<RP>::TM * RP];
  double red[kThreads / kWave * kNumPart];
};

template <int K>
__device__ __forceinline__ void write_parts(double* __restrict__ parts, const double (&v)[K]) {
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < K; ++j) parts[(size_t)blockIdx.x * kNumPart + j] = v[j];
}

// Partial sums of K consecutive slots starting at slot `first`, reduced over nb
// workgroups in a fixed order; identical in every thread of every workgroup.
template <int K>
__device__ __forceinline__ void reduce_slots(const double* __restrict__ part, int nb, int first,
                                             double (&out)[K], double* sred) {
#pragma unroll
  for (int j = 0; j < K; ++j) out[j] = 0.0;
  for (int b = threadIdx.x; b < nb; b += kThreads) {
    const double* p = part + (size_t)b * kNumPart + first;
#pragma unroll
    for (int j = 0; j < K; ++j) out[j] += p[j];
  }
  block_sum<K>(out, sred);
}

// ----------------------------------------------------------------------------- init
// C = (sum of the A-pass partials) + lam P;  g = X G + lam X - C [+ gam LX].
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_init(
    const T* __restrict__ X, const T* __restrict__ P, const T* __restrict__ Bpart, int ksplit,
    int64_t bstride, T* __restrict__ Cout, T* __restrict__ g, const T* __restrict__ LX,
    const T* __restrict__ GT, int64_t n, int r, int is_hstep, KParams kp, State* __restrict__ st,
    double* __restrict__ partsA) {
  if (st->done) return;
  constexpr int RS = TileCfg<RP>::RS, TM = TileCfg<RP>::TM;
  __shared__ Smem<T, RP> sm;
  const int tid = threadIdx.x, c = tid % RP, rs = tid / RP;
  if (!is_hstep && blockIdx.x == 0 && tid == 0) {
    // snapshot for the monitor record completed by this W-step's first inner kernel
    st->snap_pending = st->pending;
    st->snap_outer = st->outer;
    st->pending = 0;
  }
  for (int e = tid; e < r * r; e += kThreads) sm.G[e] = GT[e];
  const T lam = (T)kp.lam, gam = (T)kp.gamma;
  double v[1] = {0.0};
  const int64_t ntiles = (n + TM - 1) / TM;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * TM;
    T x[8], cv[8], pv[8];
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int lr = rs + p * RS;
      const int64_t row = row0 + lr;
      const bool ok = row < n && c < r;
      const int64_t o = row * r + c;
      T b = T(0);
      if (ok) {
        int s = 0;
        for (; s + 4 <= ksplit; s += 4) {  // four split-K partials in flight, added in order
          const T b0 = Bpart[s * bstride + o], b1 = Bpart[(s + 1) * bstride + o];
          const T b2 = Bpart[(s + 2) * bstride + o], b3 = Bpart[(s + 3) * bstride + o];
          b += b0;
          b += b1;
          b += b2;
          b += b3;
        }
        for (; s < ksplit; ++s) b += Bpart[s * bstride + o];
      }
      x[p] = ok ? X[o] : T(0);
      pv[p] = ok ? P[o] : T(0);
      cv[p] = b + lam * pv[p];
      if (ok) Cout[o] = cv[p];
      if (c < r) sm.a[lr * r + c] = x[p];
    }
    __syncthreads();
    T xg[8];
    tile_gemm<T, RP>(sm.a, sm.G, r, c, rs, xg);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int64_t row = row0 + rs + p * RS;
      if (row < n && c < r) {
        const int64_t o = row * r + c;
        T gv = xg[p] + lam * x[p] - cv[p];
        if (LX) gv += gam * LX[o];
        g[o] = gv;
        if (is_hstep) {
          v[0] += (double)cv[p] * (double)pv[p];
        } else {
          const double mn = (double)(x[p] < gv ? x[p] : gv);
          v[0] += mn * mn;
        }
      }
    }
  }
  block_sum<1>(v, sm.red);
  write_parts<1>(partsA, v);
}

// ----------------------------------------------------------------------------- entry
// First kernel of inner iteration k: derive e_k and alpha_k (or, at k = 0, complete the
// monitor record of the previous outer iteration).  Returns false if this inner
// iteration must not run (solve done, half-step stopped, breakdown).
template <typename T>
__device__ bool inner_entry(int k, int is_hstep, int r, const KParams& kp, State* __restrict__ st,
                            const double* __restrict__ partsA, const double* __restrict__ partsC,
                            int nb, const double* __restrict__ Gcur,
                            const double* __restrict__ Gprev, double* __restrict__ trace,
                            double* sred, double& alpha_out) {
  const bool w0 = blockIdx.x == 0 && threadIdx.x == 0;
  double e_k, alpha_k;
  if (k == 0) {
    if (!is_hstep) {
      if (st->snap_pending) {
        double a1[1], m[5], gg[3] = {0.0, 0.0, 0.0};
        reduce_slots<1>(partsA, nb, 0, a1, sred);   // ||min(W, grad_W)||^2
        reduce_slots<5>(partsC, nb, 3, m, sred);    // <C,Ht>, <W,Ht>, ||Ht-W||^2, pgH^2, <Ht,LHt>
        for (int e = threadIdx.x; e < r * r; e += kThreads) {
          gg[0] += Gprev[e] * Gcur[e];   // <W^T W, Ht^T Ht>
          gg[1] += Gprev[e] * Gprev[e];  // ||W^T W||_F^2
        }
        for (int a = threadIdx.x; a < r; a += kThreads) gg[2] += Gprev[a * r + a];  // ||W||^2
        block_sum<3>(gg, sred);
        const double nA2 = st->normA2;
        const double AWHt = m[0] - kp.lam * m[1];   // <A W, Ht>
        const double AWW = st->m_CP - kp.lam * gg[2];  // <A W, W>
        const double res2 = nA2 - 2.0 * AWHt + gg[0];
        const double resw2 = nA2 - 2.0 * AWW + gg[1];
        const double res = sqrt(fmax(res2, 0.0) / nA2);
        const double resw = sqrt(fmax(resw2, 0.0) / nA2);
        const double sym = sqrt(m[2] / fmax(gg[2], 1e-300));
        const double pg = sqrt(a1[0] + m[3]);
        const double f = 0.5 * fmax(res2, 0.0) + 0.5 * kp.lam * m[2] + 0.5 * kp.gamma * m[4];
        const int o = st->snap_outer;
        const bool conv = kp.target > 0.0 && res <= kp.target;
        const bool bad = !(res == res) || !(pg == pg);
        const bool fin = conv || bad || o + 1 >= kp.max_outer;
        if (w0) {
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
          st->res_last = res;
          st->resww_last = resw;
          st->sym_last = sym;
          st->pg_last = pg;
          st->f_last = f;
          st->outer = o + 1;
          st->trace_len = o + 1;
          if (conv && st->converged_at == 0) st->converged_at = o + 1;
          if (bad) st->status = 9;
          if (fin) st->done = 1;
        }
        if (fin) return false;
      }
    } else {
      double a1[1];
      reduce_slots<1>(partsA, nb, 0, a1, sred);     // <C, P> with P = W
      if (w0) st->m_CP = a1[0];
    }
    e_k = 0.0;
    alpha_k = 1.0 / st->rho;
  } else {
    if (st->stop[k - 1]) {
      if (w0) st->stop[k] = 1;
      return false;
    }
    double s4[3];
    reduce_slots<3>(partsC, nb, 0, s4, sred);
    double sl[1];
    reduce_slots<1>(partsC, nb, 8, sl, sred);
    const double ss = s4[0];
    const double sy = s4[1] + kp.lam * ss + kp.gamma * sl[0];  // <S, Y> = <S(G+lam I),S> [+gam<S,LS>]
    const double dlt = s4[2] + 0.5 * sy;                        // f(X_k) - f(X_{k-1})
    e_k = kp.eta * (st->e[k - 1] - dlt);                        // F_k - f(X_k)
    const double ratio = sy > 0.0 ? ss / sy : 1e308;
    alpha_k = fmin(kp.amax, fmax(kp.amin, ratio));
    const bool bad = !(sy == sy) || !(dlt == dlt);
    if (w0) {
      st->last_ss = ss;
      st->last_sy = sy;
      if (bad) {
        st->status = 9;
        st->done = 1;
      }
    }
    if (bad) return false;
    if (ss == 0.0) {  // X_k = X_{k-1}: stationary, the half-step is over
      if (w0) st->stop[k] = 1;
      return false;
    }
  }
  if (w0) {
    st->e[k] = e_k;
    st->alpha[k] = alpha_k;
    st->stop[k] = 0;
  }
  alpha_out = alpha_k;
  return true;
}

// ----------------------------------------------------------------------------- step 1
// Z = max(0, X - g/rho);  grad f(Z) = g + (Z - X)(G + lam I) [+ gam L(Z-X)];
// D = max(0, Z - alpha grad f(Z)) - Z.  Partials: <grad f(Z), D>, <D G, D>, ||D||^2 and
// f(Z) - f(X) = <g + grad f(Z), Z - X>/2 (exact for a quadratic).
// phase 0: whole step.  Laplacian path: phase 1 writes Z and Z - X (into D); phase 2
// reads them back together with L(Z - X).
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_step1(
    const T* __restrict__ X, const T* __restrict__ g, T* __restrict__ Z, T* __restrict__ D,
    const T* __restrict__ LdZ, const T* __restrict__ GT, const double* __restrict__ Gcur,
    const double* __restrict__ Gprev, int64_t n, int r, int k, int phase, int is_hstep,
    KParams kp, State* __restrict__ st, const double* __restrict__ partsA,
    double* __restrict__ partsB, const double* __restrict__ partsC, double* __restrict__ trace) {
  if (st->done) return;
  constexpr int RS = TileCfg<RP>::RS, TM = TileCfg<RP>::TM;
  __shared__ Smem<T, RP> sm;
  const int tid = threadIdx.x, c = tid % RP, rs = tid / RP;
  double alpha_d = 0.0;
  if (phase != 2) {
    if (!inner_entry<T>(k, is_hstep, r, kp, st, partsA, partsC, gridDim.x, Gcur, Gprev, trace,
                        sm.red, alpha_d))
      return;
  } else {
    if (st->stop[k]) return;
    alpha_d = st->alpha[k];
  }
  const T rinv = (T)(1.0 / st->rho);
  const T alpha = (T)alpha_d;
  const T lam = (T)kp.lam, gam = (T)kp.gamma;
  const int64_t ntiles = (n + TM - 1) / TM;
  if (phase == 1) {
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int64_t row = t * TM + rs + p * RS;
        if (row < n && c < r) {
          const int64_t o = row * r + c;
          const T x = X[o];
          const T z = relu(x - g[o] * rinv);
          Z[o] = z;
          D[o] = z - x;
        }
      }
    }
    return;
  }
  for (int e = tid; e < r * r; e += kThreads) sm.G[e] = GT[e];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * TM;
    T x[8], gv[8], z[8];
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int lr = rs + p * RS;
      const int64_t row = row0 + lr;
      const bool ok = row < n && c < r;
      const int64_t o = row * r + c;
      x[p] = ok ? X[o] : T(0);
      gv[p] = ok ? g[o] : T(0);
      if (phase == 2) {
        z[p] = ok ? Z[o] : T(0);
      } else {
        z[p] = relu(x[p] - gv[p] * rinv);
      }
      if (c < r) sm.a[lr * r + c] = z[p] - x[p];
    }
    __syncthreads();
    T dzg[8];
    tile_gemm<T, RP>(sm.a, sm.G, r, c, rs, dzg);
    T d[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int lr = rs + p * RS;
      const int64_t row = row0 + lr;
      const bool ok = row < n && c < r;
      const int64_t o = row * r + c;
      const T dz = z[p] - x[p];
      T gz = gv[p] + dzg[p] + lam * dz;
      if (phase == 2 && ok) gz += gam * LdZ[o];
      const T dd = ok ? relu(z[p] - alpha * gz) - z[p] : T(0);
      d[p] = dd;
      if (ok) {
        if (phase == 0) Z[o] = z[p];
        D[o] = dd;
        v[0] += (double)gz * (double)dd;
        v[2] += (double)dd * (double)dd;
        v[3] += 0.5 * ((double)gv[p] + (double)gz) * (double)dz;
      }
      if (c < r) sm.b[lr * r + c] = dd;
    }
    __syncthreads();
    T dg[8];
    tile_gemm<T, RP>(sm.b, sm.G, r, c, rs, dg);
#pragma unroll
    for (int p = 0; p < 8; ++p) v[1] += (double)dg[p] * (double)d[p];
  }
  block_sum<4>(v, sm.red);
  write_parts<4>(partsB, v);
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
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_step2(
    T* __restrict__ X, T* __restrict__ g, T* __restrict__ Z, T* __restrict__ D,
    const T* __restrict__ LS, const T* __restrict__ C, const T* __restrict__ P,
    T* __restrict__ LXb, const T* __restrict__ GT, int64_t n, int r, int k, int phase,
    int is_hstep, KParams kp, State* __restrict__ st, const double* __restrict__ partsB,
    const double* __restrict__ partsD, int nbD, double* __restrict__ partsC) {
  if (st->done | st->stop[k]) return;
  constexpr int RS = TileCfg<RP>::RS, TM = TileCfg<RP>::TM;
  __shared__ Smem<T, RP> sm;
  const int tid = threadIdx.x, c = tid % RP, rs = tid / RP;
  const bool w0 = blockIdx.x == 0 && tid == 0;
  double beta;
  if (phase != 2) {
    double b4[4];
    reduce_slots<4>(partsB, gridDim.x, 0, b4, sm.red);
    double q = b4[1] + kp.lam * b4[2];
    if (partsD) {
      double dl[1];
      reduce_slots<1>(partsD, nbD, 0, dl, sm.red);
      q += kp.gamma * dl[0];
    }
    int evals, exh;
    beta = line_search(b4[0], q, b4[3], st->e[k], kp, evals, exh);
    if (w0) {
      st->beta[k] = beta;
      st->ls_evals += evals;
      st->ls_exhausted += exh;
      st->inner_total += 1;
    }
  } else {
    beta = st->beta[k];
  }
  const T step = (T)(kp.phi * beta);
  const T lam = (T)kp.lam, gam = (T)kp.gamma;
  const int64_t ntiles = (n + TM - 1) / TM;
  if (phase == 1) {
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int64_t row = t * TM + rs + p * RS;
        if (row < n && c < r) {
          const int64_t o = row * r + c;
          T xn = Z[o] + step * D[o];
          if (kp.project) xn = relu(xn);
          Z[o] = xn;
          D[o] = xn - X[o];
        }
      }
    }
    return;
  }
  for (int e = tid; e < r * r; e += kThreads) sm.G[e] = GT[e];
  double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * TM;
    T x[8], xn[8];
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int lr = rs + p * RS;
      const int64_t row = row0 + lr;
      const bool ok = row < n && c < r;
      const int64_t o = row * r + c;
      x[p] = ok ? X[o] : T(0);
      if (phase == 2) {
        xn[p] = ok ? Z[o] : T(0);
      } else {
        T y = ok ? Z[o] + step * D[o] : T(0);
        if (kp.project) y = relu(y);
        xn[p] = y;
      }
      if (c < r) sm.a[lr * r + c] = xn[p] - x[p];
    }
    __syncthreads();
    T sg[8];
    tile_gemm<T, RP>(sm.a, sm.G, r, c, rs, sg);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int64_t row = row0 + rs + p * RS;
      if (row < n && c < r) {
        const int64_t o = row * r + c;
        const T s = xn[p] - x[p];
        const T gold = g[o];
        T gn = gold + sg[p] + lam * s;
        if (phase == 2) gn += gam * LS[o];
        X[o] = xn[p];
        g[o] = gn;
        v[0] += (double)s * (double)s;
        v[1] += (double)sg[p] * (double)s;
        v[2] += (double)gold * (double)s;
        if (phase == 2) v[8] += (double)s * (double)LS[o];
        if (is_hstep) {
          const double cx = (double)C[o], px = (double)P[o], xv = (double)xn[p];
          v[3] += cx * xv;
          v[4] += px * xv;
          v[5] += (xv - px) * (xv - px);
          const double mn = (double)(xn[p] < gn ? xn[p] : gn);
          v[6] += mn * mn;
        }
        if (phase == 2 && LXb) {
          const T lxn = LXb[o] + LS[o];
          LXb[o] = lxn;
          if (is_hstep) v[7] += (double)xn[p] * (double)lxn;
        }
      }
    }
  }
  block_sum<9>(v, sm.red);
  write_parts<9>(partsC, v);
  if (is_hstep && w0) {
    st->pending = 1;
    st->t_hstep = wall_clock64();
  }
}

// ----------------------------------------------------------------------------- launchers
int rank_pad(int r) {
  int rp = 4;
  while (rp < r) rp *= 2;
  return rp;
}

int inner_grid(int64_t n, int r) {
  const int tm = 8 * kThreads / rank_pad(r);
  int64_t nt = (n + tm - 1) / tm;
  if (nt < 1) nt = 1;
  return (int)(nt < kInnerGrid ? nt : kInnerGrid);
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
                 State* st, double* partsA, hipStream_t s) {
  const int grid = inner_grid(n, r);
  SNMF_DISPATCH_RP(rank_pad(r),
                   hipLaunchKernelGGL((k_init<T, RP>), dim3(grid), dim3(kThreads), 0, s, X, P,
                                      Bpart, ksplit, bstride, C, g, LX, GT, n, r, is_hstep, kp, st,
                                      partsA))
}

template <typename T>
void launch_step1(const T* X, const T* g, T* Z, T* D, const T* LdZ, const T* GT,
                  const double* Gcur, const double* Gprev, int64_t n, int r, int k, int phase,
                  int is_hstep, const KParams& kp, State* st, const double* partsA,
                  double* partsB, const double* partsC, double* trace, hipStream_t s) {
  const int grid = inner_grid(n, r);
  SNMF_DISPATCH_RP(rank_pad(r),
                   hipLaunchKernelGGL((k_step1<T, RP>), dim3(grid), dim3(kThreads), 0, s, X, g,
                                      Z, D, LdZ, GT, Gcur, Gprev, n, r, k, phase, is_hstep, kp, st,
                                      partsA, partsB, partsC, trace))
}

template <typename T>
void launch_step2(T* X, T* g, T* Z, T* D, const T* LS, const T* C, const T* P, T* LXb,
                  const T* GT, int64_t n, int r, int k, int phase, int is_hstep,
                  const KParams& kp, State* st, const double* partsB, const double* partsD,
                  int nbD, double* partsC, hipStream_t s) {
  const int grid = inner_grid(n, r);
  SNMF_DISPATCH_RP(rank_pad(r),
                   hipLaunchKernelGGL((k_step2<T, RP>), dim3(grid), dim3(kThreads), 0, s, X, g,
                                      Z, D, LS, C, P, LXb, GT, n, r, k, phase, is_hstep, kp, st,
                                      partsB, partsD, nbD, partsC))
}

#define SNMF_INST(T)                                                                            \
  template void launch_init<T>(const T*, const T*, const T*, int, int64_t, T*, T*, const T*,   \
                               const T*, int64_t, int, int, const KParams&, State*, double*,   \
                               hipStream_t);                                                    \
  template void launch_step1<T>(const T*, const T*, T*, T*, const T*, const T*, const double*, \
                                const double*, int64_t, int, int, int, int, const KParams&,     \
                                State*, const double*, double*, const double*, double*,         \
                                hipStream_t);                                                   \
  template void launch_step2<T>(T*, T*, T*, T*, const T*, const T*, const T*, T*, const T*,    \
                                int64_t, int, int, int, int, const KParams&, State*,            \
                                const double*, const double*, int, double*, hipStream_t);
SNMF_INST(float)
SNMF_INST(double)

}  // namespace snmf
