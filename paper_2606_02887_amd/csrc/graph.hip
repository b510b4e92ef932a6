// Host side and C ABI of the graph preprocessing of Graph-SNMPBB (Section 2.2; include/
// snmf.h snmf_knn / snmf_knn_graph): neighbours, the union pattern, the similarity values
// and the normalised Laplacian, every step in the kernels of k_graph.hip.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/snmf.h"
#include "common.hpp"
#include "host.hpp"
#include "kernels.hpp"

using namespace snmf;

namespace {

snmf_status check_points(const void* X, int64_t n, int dim, int K, int prec) {
  if (!X) return fail(SNMF_E_ARG, "X is required");
  if (prec != SNMF_F32 && prec != SNMF_F64) return fail(SNMF_E_ARG, "prec must be F32 or F64");
  if (n < 2 || n >= ((int64_t)1 << 31)) return fail(SNMF_E_SHAPE, "n must lie in [2, 2^31)");
  if (dim < 1 || dim > kKnnMaxDim) return fail(SNMF_E_SHAPE, "dim must lie in [1, 64]");
  if (K < 1 || K > kKnnMaxK) return fail(SNMF_E_SHAPE, "K must lie in [1, 64]");
  if (K > n - 1) return fail(SNMF_E_SHAPE, "K must not exceed n - 1");
  return SNMF_OK;
}

// E_NONFINITE unless every coordinate is finite (flag: one device unsigned of scratch).
snmf_status check_finite(const void* X, int64_t count, int prec, unsigned* flag, hipStream_t s) {
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(unsigned), s));
  if (prec == SNMF_F64)
    launch_count_nonfinite<double>((const double*)X, count, flag, s);
  else
    launch_count_nonfinite<float>((const float*)X, count, flag, s);
  HIP_TRY(hipGetLastError());
  unsigned bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (bad) return fail(SNMF_E_NONFINITE, "X has NaN/Inf entries");
  return SNMF_OK;
}

void knn_any(const void* X, int64_t n, int dim, int K, int prec, int32_t* nbr, hipStream_t s) {
  if (prec == SNMF_F64)
    launch_knn<double>((const double*)X, n, dim, K, nbr, s);
  else
    launch_knn<float>((const float*)X, n, dim, K, nbr, s);
}

}  // namespace

extern "C" {

snmf_status snmf_knn(const void* X, int64_t n, int32_t dim, int32_t K, int32_t prec,
                     int32_t* nbr_out, void* stream) {
  SNMF_TRY(check_points(X, n, dim, K, prec));
  if (!nbr_out) return fail(SNMF_E_ARG, "nbr_out is required");
  hipStream_t s = (hipStream_t)stream;
  DevBuf flag;
  HIP_TRY(hipMalloc(&flag.p, 256));
  SNMF_TRY(check_finite(X, n * dim, prec, (unsigned*)flag.p, s));
  knn_any(X, n, dim, K, prec, nbr_out, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return SNMF_OK;
}

snmf_status snmf_knn_graph(const void* X, int64_t n, int32_t dim, int32_t K, double sigma,
                           int32_t laplacian, int32_t prec, int64_t* rowptr_out,
                           int32_t* col_out, void* val_out, int64_t capacity, int64_t* nnz_out,
                           void* stream) {
  SNMF_TRY(check_points(X, n, dim, K, prec));
  if (!rowptr_out || !col_out || !val_out || !nnz_out)
    return fail(SNMF_E_ARG, "rowptr_out, col_out, val_out and nnz_out are required");
  if (!(sigma >= 0.0) || !(sigma < 1e300)) return fail(SNMF_E_ARG, "sigma must be >= 0 and finite");
  const int diag = laplacian ? 1 : 0;
  const int64_t bound = n * (2 * (int64_t)K + diag);
  if (capacity < bound)
    return fail(SNMF_E_SHAPE, "capacity must be at least n (2 K + [laplacian]) = " +
                                  std::to_string(bound));
  hipStream_t s = (hipStream_t)stream;
  // scratch: neighbours, counts, cursors, degrees, FP64 similarity values
  const size_t b_nbr = ((size_t)n * K * 4 + 255) / 256 * 256;
  const size_t b_cnt = ((size_t)n * 4 + 255) / 256 * 256;
  const size_t b_cur = ((size_t)n * 8 + 255) / 256 * 256;
  const size_t b_deg = ((size_t)n * 8 + 255) / 256 * 256;
  const size_t b_v = ((size_t)bound * 8 + 255) / 256 * 256;
  DevBuf pool;
  HIP_TRY(hipMalloc(&pool.p, b_nbr + b_cnt + b_cur + b_deg + b_v + 256));
  char* base = (char*)pool.p;
  SNMF_TRY(check_finite(X, n * dim, prec, (unsigned*)(base + b_nbr + b_cnt + b_cur + b_deg + b_v),
                        s));
  int32_t* nbr = (int32_t*)base;
  unsigned* cnt = (unsigned*)(base + b_nbr);
  unsigned long long* cursor = (unsigned long long*)(base + b_nbr + b_cnt);
  double* deg = (double*)(base + b_nbr + b_cnt + b_cur);
  double* v = (double*)(base + b_nbr + b_cnt + b_cur + b_deg);
  knn_any(X, n, dim, K, prec, nbr, s);
  HIP_TRY(hipMemsetAsync(cnt, 0, (size_t)n * 4, s));
  launch_knn_pattern_count(nbr, n, K, diag, cnt, rowptr_out, s);
  launch_knn_pattern_fill(nbr, n, K, diag, rowptr_out, col_out, cursor, s);
  if (prec == SNMF_F64)
    launch_knn_values<double>((const double*)X, n, dim, sigma, laplacian, rowptr_out, col_out, v,
                              deg, (double*)val_out, s);
  else
    launch_knn_values<float>((const float*)X, n, dim, sigma, laplacian, rowptr_out, col_out, v,
                             deg, (float*)val_out, s);
  HIP_TRY(hipGetLastError());
  int64_t nnz = 0;
  HIP_TRY(hipMemcpyAsync(&nnz, rowptr_out + n, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *nnz_out = nnz;
  return SNMF_OK;
}

}  // extern "C"
