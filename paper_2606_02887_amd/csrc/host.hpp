// Host-side helpers shared by the single-solve and batched-solve orchestration.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/snmf.h"
#include "common.hpp"
#include "kernels.hpp"

namespace snmf {

// The thread-local message behind snmf_last_error().
std::string& err_ref();

inline snmf_status fail(snmf_status s, const std::string& msg) {
  err_ref() = msg;
  return s;
}

#define HIP_TRY(call)                                                                  \
  do {                                                                                 \
    hipError_t _e = (call);                                                            \
    if (_e != hipSuccess)                                                              \
      return ::snmf::fail(_e == hipErrorOutOfMemory ? SNMF_E_OOM : SNMF_E_DEVICE,      \
                          std::string(#call) + ": " + hipGetErrorString(_e));          \
  } while (0)

#define SNMF_TRY(call)                  \
  do {                                  \
    snmf_status _s = (call);            \
    if (_s != SNMF_OK) return _s;       \
  } while (0)

inline size_t elt_size(int prec) { return prec == SNMF_F64 ? 8 : 4; }

// The fused inner kernels (one per inner iteration) serve the half-steps of a solve when
// fuse_inner is set and a backtracked update is never clipped by the projection
// (phi beta_shrink <= 1, no projection, or no backtracking), which their BB step after a
// backtrack relies on.  They beat the two-kernel form at every size measured: where the
// iteration is latency-bound (fewer kernels) and where it streams the n x r arrays (five
// array transfers per inner iteration against six).
inline bool fused_inner_ok(const snmf_params& p) {
  const bool unclipped = !p.project_update || p.max_ls == 0 || p.phi * p.beta_shrink <= 1.0;
  return p.fuse_inner && unclipped;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// A HIP event destroyed with its scope (the timing entry points return early on errors).
struct ScopedEvent {
  hipEvent_t e = nullptr;
  ~ScopedEvent() {
    if (e) (void)hipEventDestroy(e);
  }
};

snmf_status check_params(const snmf_params* p);
snmf_status check_matrix(const snmf_matrix* A, const char* what);
// relative tolerance of the dense symmetry check: about eight FP32 ulps, far above the
// rounding a product such as X X^T leaves between mirrored entries
constexpr double kSymTol = 0x1p-20;
snmf_status check_dense_symmetry(const snmf_matrix* M, int prec, unsigned* flags, hipStream_t s,
                                 const char* what);
KParams kparams_of(const snmf_params& p, bool lap);

}  // namespace snmf
