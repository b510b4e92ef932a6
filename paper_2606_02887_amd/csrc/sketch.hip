// Host side and C ABI of the randomized range finder of LAI-SNMPBB (Section 2.3) and of
// the SVD start (Section 4.2), include/snmf.h snmf_lai_sketch / snmf_svd_start.
//
// Y = A Omega; Q = orth(Y); power_iters times { Q = orth(A Q); Q = orth(A Q) };
// T = Q^T (A Q); T = P E P^T (Jacobi); the k eigenpairs of largest |E|: U = Q P_k.
// orth() is a shifted Cholesky QR followed by two plain ones (the Gram in FP64 with a
// fixed summation order, the factorisation and its inverse in one workgroup), so every
// step runs on the device and the result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/snmf.h"
#include "common.hpp"
#include "host.hpp"
#include "kernels.hpp"

using namespace snmf;

namespace {

struct SketchBufs {
  void* pool = nullptr;
  void *Y = nullptr, *Q = nullptr;
  double *part = nullptr, *G = nullptr, *R = nullptr, *Rinv = nullptr, *Tm = nullptr,
         *Aj = nullptr, *V = nullptr, *ev = nullptr, *M = nullptr;
  int32_t* flag = nullptr;
  unsigned* cflags = nullptr;
  ~SketchBufs() {
    if (pool) (void)hipFree(pool);
  }
};

snmf_status check_sketch_args(const snmf_matrix* A, int k, int oversample, int power_iters,
                              int prec, const void* Omega, const void* out) {
  SNMF_TRY(check_matrix(A, "A"));
  if (A->fmt == SNMF_LOWRANK) return fail(SNMF_E_UNSUPPORTED, "the range finder takes dense or CSR A");
  if (!Omega || !out) return fail(SNMF_E_ARG, "Omega and the output are required");
  if (prec != SNMF_F32 && prec != SNMF_F64) return fail(SNMF_E_ARG, "prec must be F32 or F64");
  if (k < 1) return fail(SNMF_E_SHAPE, "rank must be >= 1");
  if (oversample < 0) return fail(SNMF_E_SHAPE, "oversample must be >= 0");
  if (k + oversample > kSketchMaxW)
    return fail(SNMF_E_SHAPE, "rank + oversample must not exceed 128");
  if (k + oversample > A->n) return fail(SNMF_E_SHAPE, "rank + oversample must not exceed n");
  if (power_iters < 0 || power_iters > 16) return fail(SNMF_E_ARG, "power_iters must lie in [0, 16]");
  return SNMF_OK;
}

template <typename T>
snmf_status sketch_run(const snmf_matrix* A, int k, int ell, int q, const T* Omega, T* out,
                       double* lam_out, bool svd, hipStream_t s) {
  const int64_t n = A->n;
  SketchBufs b;
  int64_t rp = 0;
  const int nslab = sketch_slabs(n, &rp);
  const size_t ww = (size_t)ell * ell;
  std::vector<std::pair<void**, size_t>> req;
  auto add = [&](void** dst, size_t bytes) { req.push_back({dst, (bytes + 255) / 256 * 256}); };
  add(&b.Y, (size_t)n * ell * sizeof(T));
  add(&b.Q, (size_t)n * ell * sizeof(T));
  add((void**)&b.part, (size_t)nslab * ww * 8);
  add((void**)&b.G, ww * 8);
  add((void**)&b.R, ww * 8);
  add((void**)&b.Rinv, ww * 8);
  add((void**)&b.Tm, ww * 8);
  add((void**)&b.Aj, ww * 8);
  add((void**)&b.V, ww * 8);
  add((void**)&b.ev, (size_t)ell * 8);
  add((void**)&b.M, ww * 8);
  add((void**)&b.flag, 4 * sizeof(int32_t));
  add((void**)&b.cflags, 4 * sizeof(unsigned));
  size_t total = 0;
  for (auto& r : req) total += r.second;
  HIP_TRY(hipMalloc(&b.pool, total));
  size_t off = 0;
  for (auto& r : req) {
    *r.first = (char*)b.pool + off;
    off += r.second;
  }
  HIP_TRY(hipMemsetAsync(b.flag, 0, 4 * sizeof(int32_t), s));
  if (A->fmt == SNMF_CSR) {
    // the products gather rows by column index: the structure must be sound first
    HIP_TRY(hipMemsetAsync(b.cflags, 0, 4 * sizeof(unsigned), s));
    launch_csr_structure(A->rowptr, A->col, n, A->nnz, b.cflags, s);
    HIP_TRY(hipGetLastError());
    unsigned f[4];
    HIP_TRY(hipMemcpyAsync(f, b.cflags, sizeof(f), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (f[0] || f[1]) return fail(SNMF_E_SHAPE, "A: malformed CSR structure");
    if (f[2] == 0) {
      launch_csr_symmetry<T>(A->rowptr, A->col, (const T*)A->val, n, b.cflags, s);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(f, b.cflags, sizeof(f), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (f[3]) return fail(SNMF_E_NOT_SYMMETRIC, "A is not symmetric");
    }
  }
  T* Y = (T*)b.Y;
  T* Q = (T*)b.Q;
  auto apply = [&](const T* X, T* Out) {
    if (A->fmt == SNMF_DENSE)
      launch_sketch_dense<T>((const T*)A->dense, A->ld, X, n, ell, Out, s);
    else
      launch_sketch_spmm<T>(A->rowptr, A->col, (const T*)A->val, X, n, ell, Out, s);
  };
  // shifted Cholesky QR: s = 11 (n ell + ell (ell + 1)) u ||Y||_F^2 with the FP64 unit
  // roundoff keeps the factorisation positive definite whatever the conditioning of Y
  const double shift = 11.0 * ((double)n * ell + (double)ell * (ell + 1)) * 0x1p-53;
  auto chol_pass = [&](const T* X, T* Out, double sh) {
    launch_tsgram<T>(X, X, n, ell, b.part, b.G, s);
    launch_chol_inv(b.G, ell, sh, b.R, b.Rinv, b.flag, s);
    launch_tsmm<T>(X, n, ell, b.Rinv, ell, 0, Out, s);
  };
  auto orth = [&]() {  // Y -> Q (Y is overwritten)
    chol_pass(Y, Q, shift);
    chol_pass(Q, Y, 0.0);
    chol_pass(Y, Q, 0.0);
  };
  apply(Omega, Y);
  orth();
  for (int i = 0; i < q; ++i) {
    apply(Q, Y);
    orth();
    apply(Q, Y);
    orth();
  }
  apply(Q, Y);                                   // Y = A Q
  launch_tsgram<T>(Q, Y, n, ell, b.part, b.Tm, s);  // T = Q^T A Q
  launch_jacobi(b.Tm, ell, b.Aj, b.V, b.ev, s);
  launch_sketch_select(b.ev, b.V, ell, k, svd ? 1 : 0, lam_out, b.M, s);
  launch_tsmm<T>(Q, n, ell, b.M, k, svd ? 1 : 0, out, s);
  HIP_TRY(hipGetLastError());
  int32_t flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, b.flag, sizeof(flag), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (flag) return fail(SNMF_E_BREAKDOWN, "the sketch lost rank: a Cholesky pivot was not positive");
  return SNMF_OK;
}

snmf_status sketch_any(const snmf_matrix* A, int k, int oversample, int q, int prec,
                       const void* Omega, void* out, double* lam_out, bool svd, void* stream) {
  SNMF_TRY(check_sketch_args(A, k, oversample, q, prec, Omega, out));
  hipStream_t s = (hipStream_t)stream;
  const int ell = k + oversample;
  if (prec == SNMF_F64)
    return sketch_run<double>(A, k, ell, q, (const double*)Omega, (double*)out, lam_out, svd, s);
  return sketch_run<float>(A, k, ell, q, (const float*)Omega, (float*)out, lam_out, svd, s);
}

}  // namespace

extern "C" {

snmf_status snmf_lai_sketch(const snmf_matrix* A, int32_t rank, int32_t oversample,
                            int32_t power_iters, int32_t prec, const void* Omega, void* U_out,
                            double* lam_out, void* stream) {
  if (!lam_out) return fail(SNMF_E_ARG, "lam_out is required");
  return sketch_any(A, rank, oversample, power_iters, prec, Omega, U_out, lam_out, false, stream);
}

snmf_status snmf_svd_start(const snmf_matrix* A, int32_t r, int32_t oversample,
                           int32_t power_iters, int32_t prec, const void* Omega, void* W0_out,
                           void* stream) {
  if (r > kMaxRank) return fail(SNMF_E_SHAPE, "r must lie in [1, 64]");
  return sketch_any(A, r, oversample, power_iters, prec, Omega, W0_out, nullptr, true, stream);
}

}  // extern "C"
