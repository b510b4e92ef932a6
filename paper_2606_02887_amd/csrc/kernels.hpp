// Host-callable launchers of the SNMPBB kernels (all stream-ordered, no allocation).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace snmf {

constexpr int kMaxEll = 128;     // largest LAI sketch rank
constexpr int kMaxKSplit = 16;   // largest number of split-K partials of a dense A-pass

struct DenseSplit {
  int64_t gx = 1;       // workgroups along the output rows
  int ksplit = 1;       // K splits (partial products)
  int64_t kchunk = 0;   // rows of A per split (wide FP32: rows per full band)
  int nband = 0;        // wide FP32: full bands of K
  int64_t rchunk = 0;   // wide FP32: rows per workgroup over the rows after the bands (0: none)
  int64_t nwg = 0;      // wide FP32: tile workgroups of the balanced split
  bool wide = false;    // FP32: 16-byte A loads (r in (32, 64] even, n and lda multiples of 4)
};

// rho = ||G||_2 of an r x r FP64 Gram, written to st->rho, run inside another kernel's
// launch (G == nullptr: none).
struct RhoJob {
  const double* G = nullptr;
  int r = 0;
  State* st = nullptr;
};

int rank_pad(int r);
int gram_blocks(int64_t n);  // Gram slabs of an n-row partner (shared by single and batched solves)

// ---- learned warm start
constexpr int kMlpHidden = 128;  // hidden width of the warm-start network
struct MlpDev {                  // device view of a warm-start network r -> 128 -> r
  int32_t r;
  float *M1, *b1, *M2, *b2;      // FP32 masters: M1 H x r, b1 H, M2 r x H, b2 r
  uint16_t *M1h, *M2h;           // BF16 copies used by the forward pass
  float *mom, *vel;              // Adam moments (order M1, b1, M2, b2)
};
struct MlpWork {                 // per-minibatch scratch of a training step
  float *y, *cache_a, *cache_o, *dO, *dA, *grad;
  double* part;                  // kMaxGrid x kNumPart loss partials; part[kMaxGrid*kNumPart]: loss
};
int mlp_params(int r);
void launch_mlp_sync(const MlpDev& m, hipStream_t s);
void launch_mlp_forward(const MlpDev& m, int64_t N, const float* C, const float* row_scale,
                        float* Y, const BMap& bm, int grid, const int32_t* idx, int64_t pool,
                        float* cache_a, float* cache_o, hipStream_t s);
void launch_mlp_train_step(const MlpDev& m, int64_t pool, int64_t B, const float* C,
                           const float* T, const int32_t* idx, float mu, float lr, int step,
                           const MlpWork& w, hipStream_t s);
template <typename T>
void launch_dense_rowsum(const T* A, int64_t n, int64_t ld, double* deg, hipStream_t s);
template <typename T>
void launch_ws_frame(const BInst* inst, int ninst, int max_r, const BGraph* graphs, const T* Y,
                     double* R, T* C, int32_t* anchors, hipStream_t s);
template <typename T>
void launch_ws_spa_only(const BInst* inst, int ninst, const T* C, T* W, hipStream_t s);
template <typename T>
void launch_ws_match(const BInst* inst, int ninst, const T* C, const T* H, T* Tout, int32_t* perm,
                     hipStream_t s);
// esz: bytes per element (4 or 8); fused: the grid also serves the fused inner kernels
int inner_grid(int64_t n, int r, int esz, bool fused = false);
int lai_blocks(int64_t n);

template <typename T>
void launch_gram(const T* P, int64_t n, int r, double* part, int nblk, double* G64, T* GT,
                 const State* st, hipStream_t s);
void launch_rho(const double* G, int r, State* st, hipStream_t s);
template <typename T>
void launch_bgram(const T* P, int r, const int32_t* gblk_inst, int gblocks, const BInst* inst,
                  const State* states, double* gpart, hipStream_t s);
template <typename T>
void launch_bgram_reduce(const BInst* inst, int ninst, int max_r, const State* states,
                         const double* gpart, double* G64, T* GT, hipStream_t s);
void launch_brho(const BInst* inst, int ninst, State* states, const double* G64, hipStream_t s);
template <typename T>
void launch_norm2(const T* x, int64_t N, double* part, double* out, unsigned* counter,
                  hipStream_t s);
void launch_split_rows(const float* A, int64_t n, int64_t lda, int64_t ldb, uint16_t* hi,
                       uint16_t* lo, hipStream_t s);
void launch_split_pt(const float* P, int64_t n, int r, int64_t ldp, uint16_t* hi, uint16_t* lo,
                     const State* st, hipStream_t s);

// S consecutive n x r blocks -> (S r) x ldp transposed BF16 hi/lo (ldp a multiple of 64);
// skipped when all S states are done.  With Grho set, rho of restart s (st[s].rho) from
// the FP64 Gram at Grho + s r^2 in the same launch.
void launch_split_pt_stack(const float* P, int64_t n, int r, int S, int64_t ldp, uint16_t* hi,
                           uint16_t* lo, State* st, const double* Grho, hipStream_t s);

template <typename T>
void launch_sum_parts(const T* part, int ks, int64_t stride, T* out, int64_t N, hipStream_t s);
void launch_apass_f64(const double* A, int64_t lda, const double* P, int64_t n, int r, double* B,
                      const State* st, hipStream_t s);
DenseSplit plan_dense_f32(int64_t n, int64_t lda, int r, const void* A);
// With rj.G set, rho is computed in the same launch (wide path) or just before it.
void launch_apass_f32(const float* A, int64_t lda, const float* P, int64_t n, int r,
                      const DenseSplit& d, float* Bpart, int64_t pstride, const State* st,
                      hipStream_t s, const RhoJob& rj = RhoJob{});
DenseSplit plan_dense_bf16(int64_t n);
void launch_apass_bf16x3(const uint16_t* Ahi, const uint16_t* Alo, int64_t ldb,
                         const uint16_t* Pthi, const uint16_t* Ptlo, int64_t ldp, int64_t n, int r,
                         const DenseSplit& d, float* Bpart, int64_t pstride, const State* st,
                         hipStream_t s, const RhoJob& rj = RhoJob{});

// Stacked split-BF16 A-pass of S restarts of one problem (R = S r columns): B_s = A P_s,
// written to Bout + s n r (one K slice) or as d.ksplit partials pstride apart.  With Grho
// set, rho of restart s (st[s].rho) from the FP64 Gram at Grho + s r^2 in the same launch.
DenseSplit plan_dense_bf16_stack(int64_t n, int64_t R);
int stack_per_cu();  // workgroups of the stacked split-BF16 product per CU
void launch_apass_bf16x3_stack(const uint16_t* Ahi, const uint16_t* Alo, int64_t ldb,
                               const uint16_t* Pthi, const uint16_t* Ptlo, int64_t n, int r,
                               int S, const DenseSplit& d, float* Bout, int64_t pstride,
                               State* st, const double* Grho, hipStream_t s);

template <typename T>
void launch_spmm(const int64_t* rowptr, const int32_t* col, const T* val, const T* X, int64_t n,
                 int r, T* Y, const T* X2, double* part, const int32_t* gate,
                 const int32_t* gate2, hipStream_t s, const RhoJob& rj = RhoJob{});
int spmm_dot_grid(int64_t n);
template <typename T>
void launch_bspmm(const BGraph* graphs, const int32_t* sblk_graph, int sblocks,
                  const State* states, const T* P, T* B, hipStream_t s);
void launch_breset(State* states, const BInst* inst, int ninst, hipStream_t s);
void launch_all_done(const State* states, int ninst, int32_t* flag, hipStream_t s);
template <typename T>
void launch_lai(const T* U, int ell, const double* lam, const T* P, int64_t n, int r,
                double* part, T* TT, T* B, const int32_t* gate, hipStream_t s,
                const RhoJob& rj = RhoJob{});

template <typename T>
void launch_init(const T* X, const T* P, const T* Bpart, int ksplit, int64_t bstride, T* C, T* g,
                 const T* LX, const T* GT, int64_t n, int r, int is_hstep, const KParams& kp,
                 State* st, double* partsA, hipStream_t s, const BMap& bm = BMap{}, int grid = 0,
                 T* Zn = nullptr, T* Dn = nullptr,  // Laplacian H-step: Z, Z - X of iteration 0
                 T* Dd = nullptr, double* pout = nullptr,   // fused: direction 0 into Dd,
                 T* Xs = nullptr, T* gs = nullptr);         // its beta = 1 trial into Xs, gs
// Fused inner kernel i (0 <= i < K: line search and update of inner iteration i, direction
// i + 1) of a half-step without the Laplacian term; (X, g) and the scratch pair (Xs, gs)
// alternate as iterate and trial update; pin / pout alternate between two partial-sum
// arrays.
template <typename T>
void launch_advance(T* X, T* g, T* Xs, T* gs, T* D, const T* C, const T* P, const T* GT,
                    const double* Gcur, const double* Gprev, int64_t n, int r, int K, int i,
                    int is_hstep, const KParams& kp, State* st, const double* pin, double* pout,
                    const double* partsA, double* partsC, double* trace, hipStream_t s,
                    int grid = 0);
template <typename T>
void launch_step1(const T* X, const T* g, T* Z, T* D, const T* LdZ, const T* GT,
                  const double* Gcur, const double* Gprev, int64_t n, int r, int k, int phase,
                  int is_hstep, const KParams& kp, State* st, const double* partsA,
                  double* partsB, const double* partsC, double* trace, hipStream_t s,
                  const BMap& bm = BMap{}, int grid = 0, int rd = 0);
template <typename T>
void launch_step2(T* X, T* g, T* Z, T* D, const T* LS, const T* C, const T* P, T* LXb,
                  const T* GT, int64_t n, int r, int k, int phase, int is_hstep,
                  const KParams& kp, State* st, const double* partsB, const double* partsD,
                  int nbD, double* partsC, hipStream_t s, const BMap& bm = BMap{}, int grid = 0,
                  int last_k = 0,  // last inner iteration (its H-step forms the monitor sums)
                  int rd = 0);     // phase 0: step 2 recomputes D (step 1 then stores none)
// Naive variant: the H-step's entry at H = W (<C, P> kept, half-step stopped before k = 0).
void launch_naive_hentry(const double* partsA, int nb, State* st, hipStream_t s);
// Bytes of one n x r array from which a single solve recomputes D in step 2.
constexpr int64_t kRecomputeDBytes = 4 << 20;

template <typename T>
void launch_stats2d(const T* x, int64_t rows, int64_t cols, int64_t ld, double* part, double* out,
                    unsigned* counter, hipStream_t s);
template <typename T>
void launch_dense_symmetry(const T* A, int64_t n, int64_t ld, double tol, unsigned* flags,
                           hipStream_t s);
void launch_csr_structure(const int64_t* rowptr, const int32_t* col, int64_t n, int64_t nnz,
                          unsigned* flags, hipStream_t s);
template <typename T>
void launch_csr_symmetry(const int64_t* rowptr, const int32_t* col, const T* val, int64_t n,
                         unsigned* flags, hipStream_t s);
void launch_reset_state(State* st, double normA2, hipStream_t s);
void launch_split_flat(const float* x, int64_t count, uint16_t* hi, uint16_t* lo, hipStream_t s);



// ---- range finder and SVD start (k_sketch.hip)
template <typename T>
void launch_sketch_spmm(const int64_t* rowptr, const int32_t* col, const T* val, const T* X,
                        int64_t n, int w, T* Y, hipStream_t s);
template <typename T>
void launch_sketch_dense(const T* A, int64_t ld, const T* X, int64_t n, int w, T* Y,
                         hipStream_t s);
int sketch_slabs(int64_t n, int64_t* rows_per);
template <typename T>
void launch_tsgram(const T* X, const T* Y, int64_t n, int w, double* part, double* C,
                   hipStream_t s);
void launch_chol_inv(const double* G, int w, double shift_rel, double* R, double* Rinv,
                     int32_t* flag, hipStream_t s);
template <typename T>
void launch_tsmm(const T* Y, int64_t n, int w, const double* M, int c, int absval, T* Q,
                 hipStream_t s);
void launch_jacobi(const double* Tin, int w, double* A, double* V, double* ev, hipStream_t s);
void launch_sketch_select(const double* ev, const double* V, int w, int k, int sqrt_scale,
                          double* lam, double* M, hipStream_t s);


// ---- graph preprocessing (k_graph.hip)
template <typename T>
void launch_count_nonfinite(const T* X, int64_t count, unsigned* flag, hipStream_t s);
template <typename T>
void launch_knn(const T* X, int64_t n, int dim, int K, int32_t* nbr, hipStream_t s);
void launch_knn_pattern_count(const int32_t* nbr, int64_t n, int K, int diag, unsigned* cnt,
                              int64_t* rowptr, hipStream_t s);
void launch_knn_pattern_fill(const int32_t* nbr, int64_t n, int K, int diag,
                             const int64_t* rowptr, int32_t* col, unsigned long long* cursor,
                             hipStream_t s);
template <typename T>
void launch_knn_values(const T* X, int64_t n, int dim, double sigma, int laplacian,
                       const int64_t* rowptr, const int32_t* col, double* v, double* deg, T* val,
                       hipStream_t s);


// ---- NMPBB for rectangular NMF (k_nmf.hip)
template <typename T>
void launch_rect_apass(const T* V, int64_t ld, int64_t rows, int64_t K, int trans, const T* P,
                       int r, T* B, const State* st, hipStream_t s);
// Split-K panels of B = A^T P on FP32 MFMA (A K x N): gx blocks of 256 output rows, ksplit
// chunks of kchunk rows of K (panel y at Bpart + y N r).
struct RectSplit {
  int gx = 1, ksplit = 1;
  int64_t kchunk = 0;
};
RectSplit rect_split(int64_t K, int64_t N);
void launch_rect_f32(const float* A, int64_t lda, const float* P, int64_t K, int64_t N, int r,
                     const RectSplit& sp, float* Bpart, const State* st, hipStream_t s,
                     const RhoJob& rj = RhoJob{});
template <typename T>
void launch_transpose(const T* A, int64_t rows, int64_t cols, int64_t lda, T* AT, hipStream_t s);
void launch_csr_check_rect(const int64_t* rowptr, const int32_t* col, int64_t m, int64_t ncols,
                           int64_t nnz, unsigned* flags, hipStream_t s);
template <typename T>
void launch_csr_transpose(const int64_t* rowptr, const int32_t* col, const T* val, int64_t m,
                          int64_t ncols, int64_t nnz, unsigned* cnt, unsigned long long* cursor,
                          int64_t* rowptrT, int32_t* colT, T* valT, hipStream_t s);

}  // namespace snmf
