// Fused row-tile kernels of one SNMPBB half-step (Algorithm 1 with the Section 2.4
// components).  Notation: X is the variable block (n x r), P the fixed partner,
// G = P^T P, C = A P + lam P, so that grad f(X) = X G + lam X - C [+ gam L X]
// (eqs. (2.1)-(2.3) transposed).  f is quadratic in X, hence
//   f(Y + t V) - f(Y) = t <grad f(Y), V> + t^2/2 <V (G + lam I), V> [+ t^2 gam/2 <V, L V>]
// and every line-search trial is scalar work once <grad f(Z), D> and <D, (G+lam I) D>
// are known.  The iteration never forms f itself: it carries e = F_k - f(X_k) and the
// differences f(Z) - f(X_k) and f(X_{k+1}) - f(X_k), all accumulated in FP64.
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
  static constexpr int EPT = 8;             // rows per thread
  static constexpr int TM = RS * EPT;       // rows per tile
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

// ----------------------------------------------------------------------------- init
// C = (sum of the A-pass partials) + lam P;  g = X G + lam X - C [+ gam LX].
// W-step: accumulates ||min(W, grad_W)||^2 and, in the last workgroup, completes the
// monitor record of the previous outer iteration (residual from the trace identity
// ||A - W Ht^T||^2 = ||A||^2 - 2 <A W, Ht> + <W^T W, Ht^T Ht>), then decides whether the
// solve is done.  H-step: accumulates <C, P> for the symmetric residual.
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_init(
    const T* __restrict__ X, const T* __restrict__ P, const T* __restrict__ Bpart, int ksplit,
    int64_t bstride, T* __restrict__ Cout, T* __restrict__ g, const T* __restrict__ LX,
    const T* __restrict__ GT, const double* __restrict__ Gcur, const double* __restrict__ Gprev,
    int64_t n, int r, int is_hstep, KParams kp, State* __restrict__ st, double* __restrict__ part,
    unsigned* __restrict__ counter, double* __restrict__ trace) {
  if (st->done) return;
  constexpr int RS = TileCfg<RP>::RS, TM = TileCfg<RP>::TM;
  __shared__ Smem<T, RP> sm;
  const int tid = threadIdx.x, c = tid % RP, rs = tid / RP;
  for (int e = tid; e < r * r; e += kThreads) sm.G[e] = GT[e];
  const T lam = (T)kp.lam, gam = (T)kp.gamma;
  double v[2] = {0.0, 0.0};
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
      if (ok)
        for (int s = 0; s < ksplit; ++s) b += Bpart[s * bstride + o];
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
  block_sum<2>(v, sm.red);
  if (tid == 0) part[(size_t)blockIdx.x * kNumPart] = v[0];
  if (!arrive_last(counter, gridDim.x)) return;
  double tot[1];
  reduce_partials<1>(part, gridDim.x, tot, sm.red);
  if (is_hstep) {
    if (tid == 0) st->m_CP = tot[0];
    return;
  }
  // W-step: the monitor record of the outer iteration that just finished, if any.
  if (!st->pending) return;
  double gg[2] = {0.0, 0.0};
  for (int e = tid; e < r * r; e += kThreads) {
    gg[0] += Gprev[e] * Gcur[e];   // <W^T W, Ht^T Ht>
    gg[1] += Gprev[e] * Gprev[e];  // ||W^T W||_F^2
  }
  block_sum<2>(gg, sm.red);
  if (tid == 0) {
    double trW = 0.0;
    for (int a = 0; a < r; ++a) trW += Gprev[a * r + a];  // ||W||^2
    const double nA2 = st->normA2;
    const double AWHt = st->m_CX - kp.lam * st->m_PX;     // <A W, Ht>
    const double AWW = st->m_CP - kp.lam * trW;           // <A W, W>
    const double res2 = nA2 - 2.0 * AWHt + gg[0];
    const double resw2 = nA2 - 2.0 * AWW + gg[1];
    const double res = sqrt(fmax(res2, 0.0) / nA2);
    const double resw = sqrt(fmax(resw2, 0.0) / nA2);
    const double sym = sqrt(st->m_XmP2 / fmax(trW, 1e-300));
    const double pg = sqrt(tot[0] + st->m_pgH2);
    const double f = 0.5 * fmax(res2, 0.0) + 0.5 * kp.lam * st->m_XmP2 + 0.5 * kp.gamma * st->m_XLX;
    const int o = st->outer;
    double* rec = trace + (size_t)o * kTraceFields;
    rec[0] = res;
    rec[1] = resw;
    rec[2] = sym;
    rec[3] = pg;
    rec[4] = f;
    rec[5] = (double)(st->t_hstep - st->t0);
    rec[6] = (double)st->ls_evals;
    rec[7] = (double)st->ls_exhausted;
    rec[8] = st->alpha;
    rec[9] = (double)st->inner_total;
    st->res_last = res;
    st->resww_last = resw;
    st->sym_last = sym;
    st->pg_last = pg;
    st->f_last = f;
    st->pgW2 = tot[0];
    st->outer = o + 1;
    st->trace_len = o + 1;
    st->pending = 0;
    if (kp.target > 0.0 && res <= kp.target && st->converged_at == 0) {
      st->converged_at = o + 1;
      st->done = 1;
    }
    if (o + 1 >= kp.max_outer) st->done = 1;
    if (!(res == res) || !(pg == pg)) {
      st->status = 9;
      st->done = 1;
    }
  }
}

// ----------------------------------------------------------------------------- step 1
// Z = max(0, X - g/rho);  grad f(Z) = g + (Z - X)(G + lam I) [+ gam L(Z-X)];
// D = max(0, Z - alpha grad f(Z)) - Z.  Partials: <grad f(Z), D>, <D G, D>, ||D||^2 and
// f(Z) - f(X) = <g + grad f(Z), Z - X>/2 (exact for a quadratic).  The last workgroup
// runs the nonmonotone backtracking on the closed-form objective differences.
// With a Laplacian the kernel runs in two phases: phase 1 writes Z and Z - X (into D);
// phase 2 reads them back together with L(Z - X).
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_step1(const T* __restrict__ X, const T* __restrict__ g,
                                                    T* __restrict__ Z, T* __restrict__ D,
                                                    const T* __restrict__ LdZ, T* __restrict__ Dout_dz,
                                                    const T* __restrict__ GT, int64_t n, int r,
                                                    int phase, int lap_dirD, KParams kp,
                                                    State* __restrict__ st, double* __restrict__ part,
                                                    unsigned* __restrict__ counter) {
  if (st->done | st->hs_done) return;
  constexpr int RS = TileCfg<RP>::RS, TM = TileCfg<RP>::TM;
  __shared__ Smem<T, RP> sm;
  const int tid = threadIdx.x, c = tid % RP, rs = tid / RP;
  const T rinv = (T)(1.0 / st->rho);
  const T alpha = (T)st->alpha;
  const T lam = (T)kp.lam, gam = (T)kp.gamma;
  const int64_t ntiles = (n + TM - 1) / TM;
  if (phase == 1) {  // Laplacian path, first pass: Z and Z - X only
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int64_t row = t * TM + rs + p * RS;
        if (row < n && c < r) {
          const int64_t o = row * r + c;
          const T x = X[o];
          const T z = relu(x - g[o] * rinv);
          Z[o] = z;
          Dout_dz[o] = z - x;
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
  if (tid == 0)
    for (int j = 0; j < 4; ++j) part[(size_t)blockIdx.x * kNumPart + j] = v[j];
  if (!arrive_last(counter, gridDim.x)) return;
  double tot[4];
  reduce_partials<4>(part, gridDim.x, tot, sm.red);
  if (tid == 0) {
    st->delta = tot[0];
    st->q = tot[1] + kp.lam * tot[2];
    st->nd2 = tot[2];
    st->dZ = tot[3];
    if (!lap_dirD) line_search(st, kp);
  }
}

// ----------------------------------------------------------------------------- step 2
// X+ = max(0, Z + phi beta D);  S = X+ - X;  g+ = g + S (G + lam I) [+ gam L S].
// Partials: ||S||^2, <S G, S>, <g, S>; on the H-step also the monitor pieces
// <C, X+>, <P, X+>, ||X+ - P||^2 and ||min(X+, g+)||^2.  The last workgroup forms
// <S, Y> = <S G, S> + lam ||S||^2 [+ gam <S, L S>] (the curvature identity of the LAI
// section), f(X+) - f(X) = <g, S> + <S, Y>/2, the nonmonotone update of e and the
// next BB step.  With a Laplacian phase 1 writes X+ into Z and S into D; phase 2 reads
// them back with L S and keeps the buffer L X current (L X+ = L X + L S).
template <typename T, int RP>
__global__ __launch_bounds__(kThreads) void k_step2(T* __restrict__ X, T* __restrict__ g,
                                                    T* __restrict__ Z, T* __restrict__ D,
                                                    const T* __restrict__ LS,
                                                    const T* __restrict__ C, const T* __restrict__ P,
                                                    T* __restrict__ LXb,
                                                    const T* __restrict__ GT, int64_t n, int r,
                                                    int phase, int is_hstep, KParams kp,
                                                    State* __restrict__ st, double* __restrict__ part,
                                                    unsigned* __restrict__ counter) {
  if (st->done | st->hs_done) return;
  constexpr int RS = TileCfg<RP>::RS, TM = TileCfg<RP>::TM;
  __shared__ Smem<T, RP> sm;
  const int tid = threadIdx.x, c = tid % RP, rs = tid / RP;
  const T step = (T)(kp.phi * st->beta);
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
        if (phase == 2 && LXb) {   // keep L X current: L X+ = L X + L S
          const T lxn = LXb[o] + LS[o];
          LXb[o] = lxn;
          if (is_hstep) v[7] += (double)xn[p] * (double)lxn;
        }
      }
    }
  }
  block_sum<9>(v, sm.red);
  if (tid == 0)
    for (int j = 0; j < 9; ++j) part[(size_t)blockIdx.x * kNumPart + j] = v[j];
  if (!arrive_last(counter, gridDim.x)) return;
  double tot[9];
  reduce_partials<9>(part, gridDim.x, tot, sm.red);
  if (tid == 0) {
    const double ss = tot[0];
    const double sy = tot[1] + kp.lam * ss + kp.gamma * tot[8];
    const double gs = tot[2];
    const double dlt = gs + 0.5 * sy;                 // f(X+) - f(X)
    st->ss = ss;
    st->sy = sy;
    st->gs = gs;
    st->e = kp.eta * (st->e - dlt);                   // F_{k+1} - f(X_{k+1})
    const double ratio = sy > 0.0 ? ss / sy : 1e308;
    st->alpha = fmin(kp.amax, fmax(kp.amin, ratio));
    st->k += 1;
    st->inner_total += 1;
    if (ss == 0.0) st->hs_done = 1;
    if (!(sy == sy) || !(dlt == dlt)) {
      st->status = 9;
      st->done = 1;
    }
    if (is_hstep) {
      st->m_CX = tot[3];
      st->m_PX = tot[4];
      st->m_XmP2 = tot[5];
      st->m_pgH2 = tot[6];
      st->m_XLX = tot[7];
      st->pending = 1;
      st->t_hstep = wall_clock64();
    }
  }
}

// ----------------------------------------------------------------------------- line search
// Backtracking from beta = 1 by beta_shrink, at most max_ls reductions (the last beta is
// kept when the cap is hit).  Algorithm 1 accepts beta when
//   f(Z + beta D) <= F_k + theta beta <grad f(Z), D>
// which, with f(Z + beta D) = f(Z) + beta delta + beta^2 q / 2 and F_k = f(X_k) + e, reads
//   (f(Z) - f(X_k)) + (1 - theta) beta delta + beta^2 q / 2 <= e.
// The relaxed reading tests Z + phi beta D instead (phi beta in place of beta in f).
__device__ void line_search(State* st, const KParams& kp) {
  const double delta = st->delta, q = st->q, dZ = st->dZ, e = st->e;
  const double c1 = kp.relaxed ? (kp.phi - kp.theta) : (1.0 - kp.theta);
  const double c2 = kp.relaxed ? kp.phi * kp.phi : 1.0;
  double beta = 1.0;
  int t = 0, evals = 0, exhausted = 0;
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
  st->beta = beta;
  st->ls_evals += evals;
  st->ls_exhausted += exhausted;
}

// Laplacian path: the line search runs after <D, L D> is known.
__global__ void k_line_search(State* st, KParams kp, const double* __restrict__ dLd) {
  if (st->done | st->hs_done) return;
  if (threadIdx.x == 0) {
    st->q += kp.gamma * dLd[0];
    line_search(st, kp);
  }
}

// ----------------------------------------------------------------------------- launchers
static int grid_for(int64_t n, int tm) {
  int64_t nt = (n + tm - 1) / tm;
  if (nt < 1) nt = 1;
  return (int)(nt < kMaxGrid ? nt : kMaxGrid);
}

int rank_pad(int r) {
  int rp = 4;
  while (rp < r) rp *= 2;
  return rp;
}

int inner_grid(int64_t n, int r) {
  const int rp = rank_pad(r);
  return grid_for(n, 8 * kThreads / rp);
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
                 const T* LX, const T* GT, const double* Gcur, const double* Gprev, int64_t n,
                 int r, int is_hstep, const KParams& kp, State* st, double* part,
                 unsigned* counter, double* trace, hipStream_t s) {
  const int grid = inner_grid(n, r);
  SNMF_DISPATCH_RP(rank_pad(r),
                   hipLaunchKernelGGL((k_init<T, RP>), dim3(grid), dim3(kThreads), 0, s, X, P,
                                      Bpart, ksplit, bstride, C, g, LX, GT, Gcur, Gprev, n, r,
                                      is_hstep, kp, st, part, counter, trace))
}

template <typename T>
void launch_step1(const T* X, const T* g, T* Z, T* D, const T* LdZ, T* Ddz, const T* GT,
                  int64_t n, int r, int phase, int lap_dirD, const KParams& kp, State* st,
                  double* part, unsigned* counter, hipStream_t s) {
  const int grid = inner_grid(n, r);
  SNMF_DISPATCH_RP(rank_pad(r),
                   hipLaunchKernelGGL((k_step1<T, RP>), dim3(grid), dim3(kThreads), 0, s, X, g,
                                      Z, D, LdZ, Ddz, GT, n, r, phase, lap_dirD, kp, st, part,
                                      counter))
}

template <typename T>
void launch_step2(T* X, T* g, T* Z, T* D, const T* LS, const T* C, const T* P, T* LXb,
                  const T* GT, int64_t n, int r, int phase, int is_hstep, const KParams& kp,
                  State* st, double* part, unsigned* counter, hipStream_t s) {
  const int grid = inner_grid(n, r);
  SNMF_DISPATCH_RP(rank_pad(r),
                   hipLaunchKernelGGL((k_step2<T, RP>), dim3(grid), dim3(kThreads), 0, s, X, g,
                                      Z, D, LS, C, P, LXb, GT, n, r, phase, is_hstep, kp, st,
                                      part, counter))
}

void launch_line_search(State* st, const KParams& kp, const double* dLd, hipStream_t s) {
  hipLaunchKernelGGL(k_line_search, dim3(1), dim3(64), 0, s, st, kp, dLd);
}

#define SNMF_INST(T)                                                                            \
  template void launch_init<T>(const T*, const T*, const T*, int, int64_t, T*, T*, const T*,   \
                               const T*, const double*, const double*, int64_t, int, int,       \
                               const KParams&, State*, double*, unsigned*, double*,             \
                               hipStream_t);                                                    \
  template void launch_step1<T>(const T*, const T*, T*, T*, const T*, T*, const T*, int64_t,    \
                                int, int, int, const KParams&, State*, double*, unsigned*,      \
                                hipStream_t);                                                   \
  template void launch_step2<T>(T*, T*, T*, T*, const T*, const T*, const T*, T*,               \
                                const T*, int64_t, int, int, int, const KParams&, State*,       \
                                double*, unsigned*, hipStream_t);
SNMF_INST(float)
SNMF_INST(double)

}  // namespace snmf
