/*
 * snmf.h -- C ABI of the MI355X (gfx950) SNMPBB library.
 *
 * SNMPBB computes a symmetric nonnegative factorisation A ~= W H with W, H^T >= 0 and a
 * penalty that couples W and H^T (Swart & Brust, "A Nonmonotone Gradient-Based Algorithm
 * for Symmetric Nonnegative Matrix Factorization and Graph Clustering"):
 *
 *   minimise  f(W, H) = 1/2 ||A - W H||_F^2 + lam/2 ||W - H^T||_F^2 + gam/2 tr(H L H^T)
 *
 * (eq. (1.3); the last term is the Graph-SNMPBB regulariser of eq. (2.3) with a graph
 * Laplacian L).  The solver alternates a W-step and an H-step (Section 2.1); each is a run
 * of Algorithm 1 (nonmonotone projected Barzilai-Borwein, Section 2.4).  A may be dense,
 * CSR, or the low-rank surrogate U diag(lam) U^T of LAI-SNMPBB (Section 2.3).
 *
 * Conventions shared by every entry point
 *  - All matrices are row-major.  The factor H is exchanged transposed, Ht = H^T (n x r),
 *    so W and Ht have the same shape.
 *  - Array arguments are DEVICE pointers (memory of the current HIP device) unless the
 *    comment says "host".  Struct arguments (snmf_matrix, snmf_params, snmf_info) are host
 *    pointers.  The caller owns every buffer; the library keeps no pointer after a call
 *    returns.  Scratch memory is allocated inside a call (or inside a plan) and freed
 *    before it returns (or when the plan is destroyed).
 *  - `stream` is a hipStream_t (NULL = default stream).  Work is stream-ordered; calls
 *    that return results in host structs synchronise the stream first.
 *  - Errors: argument checks run first and leave every output untouched.  Nothing is
 *    printed, no exception crosses the ABI.  snmf_last_error() returns a thread-local
 *    message describing the last non-OK status.
 *  - Limits: 1 <= r <= 64; sketch rank ell <= 128; n < 2^31 for CSR column indices.
 */
#ifndef SNMF_H
#define SNMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SNMF_ABI_VERSION 4
#define SNMF_TRACE_FIELDS 10

typedef enum snmf_status {
  SNMF_OK = 0,
  SNMF_E_ARG = 1,           /* invalid argument (null pointer, bad parameter value) */
  SNMF_E_SHAPE = 2,         /* inconsistent sizes (r > n, r > 64, bad leading dimension) */
  SNMF_E_NOT_SYMMETRIC = 3, /* CSR pattern/values not symmetric, or a dense A that fails the
                               opt-in check of params.check_symmetry */
  SNMF_E_NEGATIVE = 4,      /* negative entry in A or W0 (A >= 0 and W0 >= 0 are required) */
  SNMF_E_NONFINITE = 5,     /* NaN or Inf in A or W0 */
  SNMF_E_OOM = 6,           /* device allocation failed */
  SNMF_E_DEVICE = 7,        /* a HIP call failed */
  SNMF_E_UNSUPPORTED = 8,   /* valid but unsupported combination (e.g. BF16X3 with CSR) */
  SNMF_E_BREAKDOWN = 9      /* numeric breakdown (rho = 0 or a non-finite scalar); the last
                               finite iterate is written */
} snmf_status;

typedef enum snmf_format { SNMF_DENSE = 0, SNMF_CSR = 1, SNMF_LOWRANK = 2 } snmf_format;

/* Arithmetic of the solve.  F64: every array is double.  F32: every array is float,
 * reductions and line-search scalars are FP64.  BF16X3: as F32, but the dense A-pass
 * multiplies round-to-nearest-even BF16 hi/lo splits of A and of the partner factor on
 * MFMA (A P ~= Ahi Phi + Ahi Plo + Alo Phi, FP32 accumulation); A is given in FP32 and
 * split once per plan. */
typedef enum snmf_precision { SNMF_F64 = 0, SNMF_F32 = 1, SNMF_BF16X3 = 2 } snmf_precision;

/* The symmetric nonnegative input A (n x n), or a graph Laplacian L.  Element type of
 * `dense`, `val` and `U` follows the solve precision (double for F64, float otherwise).
 *  DENSE:   dense[i*ld + j], ld >= n; symmetric: checked only when the solve's
 *           params.check_symmetry is set (O(n^2)), else the caller's promise.  The FP32
 *           A-pass forms A^T P (equal to A P for symmetric A) while the FP64 and split-BF16
 *           forms multiply A P, so an unchecked asymmetric A makes the forms disagree.
 *  CSR:     rowptr[n+1] (int64, device), col[nnz] (int32, device), val[nnz]; both
 *           triangles stored; rows need not be sorted.
 *  LOWRANK: U[i*ell + a] (n x ell, orthonormal columns) and lam[ell] (double, device):
 *           A ~= U diag(lam) U^T.  Products A P are formed as U (lam .* (U^T P)). */
typedef struct snmf_matrix {
  int32_t fmt;
  int32_t reserved;
  int64_t n;
  const void* dense;
  int64_t ld;
  const int64_t* rowptr;
  const int32_t* col;
  const void* val;
  int64_t nnz;
  const void* U;
  int64_t ell;
  const double* lam;
} snmf_matrix;

/* Launch shape of a batched solve (snmf_batch_create), chosen by timing on the batch's
 * own shapes (the package's autotuner caches the choice per device and workload).  Class q
 * holds the instances of rank r with rank padding 8, 16, 32, 64 (q = 0..3: r <= 8,
 * r <= 16, r <= 32, r <= 64).  Any value in range gives the same iteration; only the
 * grouping of the FP64 partial sums, and so their rounding, changes with it. */
typedef struct snmf_batch_tuning {
  int32_t tiles_per_wg[4];  /* row tiles per inner-kernel workgroup of class q, 1..64   [4] */
  int32_t spmm_rows_per_wg; /* rows per workgroup of the batched SpMM (CSR A), 1..4096 [16] */
  int32_t reserved[3];      /* must be 0 */
} snmf_batch_tuning;

/* Solver parameters.  snmf_params_default() fills the values in brackets. */
typedef struct snmf_params {
  double lambda;       /* symmetric penalty lam >= 0 (eq. (1.3))                         [0] */
  double gamma;        /* Laplacian weight gam >= 0 (eq. (2.3)), used when L != NULL     [0] */
  const snmf_matrix* L;/* CSR Laplacian (n x n) or NULL                                [NULL] */
  double eta;          /* nonmonotone memory, 0 <= eta < 1                            [0.85] */
  double theta;        /* Armijo parameter, 0 < theta < 1                             [1e-3] */
  double phi;          /* relaxation factor of W_{k+1} = Z_k + phi beta D_k, phi > 0   [1.7] */
  double alpha_min;    /* BB step clip, 0 < alpha_min < alpha_max                    [1e-10] */
  double alpha_max;    /*                                                             [1e10] */
  double beta_shrink;  /* backtracking factor, 0 < beta_shrink < 1                     [0.5] */
  int32_t max_ls;      /* backtracking reductions per inner iteration, >= 0             [20] */
  int32_t inner_iters; /* inner iterations per half-step, 1..64                           [5] */
  int32_t max_outer;   /* outer (W-step + H-step) iterations, >= 1                      [100] */
  int32_t check_every; /* host checks the stop flag every this many outer iterations     [8] */
  double target_res;   /* stop at the first outer iteration with ||A - W H||/||A|| <= this
                          (0 disables)                                                   [0] */
  int32_t prec;        /* snmf_precision                                          [SNMF_F32] */
  int32_t accept_at_relaxed; /* 0: test f(Z + beta D) (Algorithm 1); 1: test f(Z + phi beta D)
                                (requires project_update = 0)                            [0] */
  int32_t project_update;    /* 1: W_{k+1} = max(0, Z + phi beta D); 0: no projection     [1] */
  int32_t validate;    /* 1: check A >= 0, finite, W0 >= 0 finite, CSR structure        [1] */
  int32_t use_graph;   /* 1: replay one outer iteration as a captured hipGraph           [1] */
  int32_t check_symmetry; /* 1: dense A must satisfy |a_ij - a_ji| <= 2^-20 max(|a_ij|, |a_ji|)
                          for all i, j, else SNMF_E_NOT_SYMMETRIC (one O(n^2) pass over A at
                          plan or batch creation); 0: not checked (CSR symmetry is checked
                          whenever validate is set)                                      [0] */
  int32_t naive;       /* 1: the naive symmetric variant of Section 2.1 in place of the
                          penalty method: each outer iteration runs Algorithm 1 on W with
                          the partner held at the current W and no penalty, then sets
                          H <- W^T (an ablation).  Needs lambda = 0 (E_ARG) and no Laplacian
                          (E_UNSUPPORTED); single solves only (batches: E_UNSUPPORTED)     [0] */
  int32_t fuse_inner;  /* 1: one kernel per inner iteration, 0: two (step 1 and step 2).
                          The fused kernel forms the next BB step from sums its predecessor
                          prepared: for the first backtracking trial (beta = 1) the update's
                          own sums (that update is kept, not formed again), which give the
                          same bits as 0; after a backtrack the sums of S = dZ + phi beta D,
                          which the projection leaves unclipped when phi beta_shrink <= 1
                          (the same scalars up to rounding).  Used on single and NMF solves
                          where phi beta_shrink <= 1, project_update = 0 or max_ls = 0; the
                          H-steps of Graph-SNMPBB and of the naive variant keep two
                          kernels                                                         [1] */
  const snmf_batch_tuning* tuning; /* batched solves: launch shape, or NULL for the
                          defaults (read at snmf_batch_create; values out of range: E_ARG)
                          [NULL] */
} snmf_params;

/* Per-solve results (host struct written on return). */
typedef struct snmf_info {
  int32_t status;        /* snmf_status of the solve */
  int32_t outer;         /* completed outer iterations */
  int32_t converged_at;  /* first outer iteration meeting target_res (1-based), 0 if none */
  int32_t reserved;
  int64_t inner_total;   /* inner iterations run (all half-steps) */
  int64_t ls_evals;      /* line-search trials */
  int64_t ls_exhausted;  /* inner iterations whose backtracking hit max_ls */
  double res_WH;         /* ||A - W Ht^T||_F / ||A||_F at the returned factors */
  double res_WWt;        /* ||A - W W^T||_F / ||A||_F */
  double sym_gap;        /* ||W - Ht||_F / ||W||_F */
  double pg_norm;        /* ||min(W, grad_W f)||^2 + ||min(Ht, grad_Ht f)||^2, square root:
                            zero exactly at first-order stationary points (Section 3.1) */
  double objective;      /* f(W, H) */
  double seconds;        /* device time from solve start to the last completed outer
                            iteration */
  double seconds_to_target; /* device time to converged_at, or -1 */
  double normA2;         /* ||A||_F^2 (surrogate norm sum(lam^2) for LOWRANK) */
} snmf_info;

snmf_status snmf_params_default(snmf_params* p);

/* Solve SNMPBB.  W0 (n x r) is the start of both factors (W = Ht = W0, as H0 = W0^T in
 * Section 4.1).  W_out, Ht_out: n x r outputs (may alias W0 only if W_out == W0).
 * trace: optional host array of max_outer * SNMF_TRACE_FIELDS doubles; record i holds
 * {res_WH, res_WWt, sym_gap, pg_norm, objective, device_ticks, ls_evals, ls_exhausted,
 *  alpha, inner_total} after outer iteration i+1 (device_ticks at the clock rate returned
 * by snmf_clock_rate_hz()). */
snmf_status snmf_solve(const snmf_matrix* A, int32_t r, const void* W0, const snmf_params* p,
                       void* W_out, void* Ht_out, snmf_info* info, void* stream, double* trace);

/* snmf_solve without any allocation, for callers that cannot allocate device memory
 * (serving loops and harnesses that forbid hipMalloc): the same computation as
 * snmf_solve with use_graph = 0 (direct launches; instantiating a graph allocates), with
 * its scratch in the library's static device array of 64 MiB per GPU (held from the
 * first use of the library on a device until the process ends), work on the caller's
 * stream, and no host heap allocation on success.  Limits: F64 or F32 (BF16X3:
 * E_UNSUPPORTED, its split copies of A would not fit); the scratch the problem needs must
 * fit 64 MiB (about 6 n r element sizes plus, for dense F32, the split-K partial panels;
 * dense n = 8192, r = 64 in F32 needs 31 MiB), else E_SHAPE with the size in the message.
 * Every call on a GPU shares that GPU's array, and the library clears what must start at
 * zero on each call: calls that overlap on one GPU (several host threads, or streams that
 * run concurrently) race and must not be issued.  The call synchronises the stream. */
snmf_status snmf_solve_noalloc(const snmf_matrix* A, int32_t r, const void* W0,
                               const snmf_params* p, void* W_out, void* Ht_out, snmf_info* info,
                               void* stream, double* trace);

/* Plans: the same solve with scratch memory and input preprocessing (||A||^2, validation,
 * the BF16 split) kept across calls, for repeated timed solves.  A plan keeps the
 * pointers of A and L given at creation; they must stay valid until destroy. */
typedef struct snmf_plan snmf_plan;
snmf_status snmf_plan_create(const snmf_matrix* A, int32_t r, const snmf_params* p,
                             void* stream, snmf_plan** out);
snmf_status snmf_plan_solve(snmf_plan* plan, const void* W0, void* W_out, void* Ht_out,
                            snmf_info* info, void* stream, double* trace);
snmf_status snmf_plan_destroy(snmf_plan* plan);

/* One half-step of SNMPBB (Algorithm 1 run for inner_iters iterations) with the partner
 * block P fixed: X (n x r, in/out) is W (is_hstep = 0, P = Ht) or Ht (is_hstep = 1,
 * P = W, the Laplacian term applies).  Used to check the method step by step.
 * scalars (host, optional, 8 doubles): {rho, alpha, beta, e of the last inner iteration
 * that ran, <S,S> and <S,Y> of the last update, line-search trials, inner iterations run}.
 * inner_iters <= 64. */
snmf_status snmf_plan_half_step(snmf_plan* plan, void* X, const void* P, int32_t is_hstep,
                                void* stream, double* scalars);

/* Primitives of the hot path, for per-kernel checks.  All arrays are device arrays of the
 * plan's precision type unless stated.
 *  apass:   B = A P (n x r).  For BF16X3 plans the split product above, B in float.
 *  gram:    G = P^T P (r x r, double), accumulated in FP64.
 *  rho:     ||G||_2 of a symmetric PSD r x r double matrix G (device), returned in *rho
 *           (host).
 *  spmm:    Y = M X for a CSR matrix M of the plan's type (e.g. the Laplacian). */
snmf_status snmf_plan_apass(snmf_plan* plan, const void* P, void* B, void* stream);
snmf_status snmf_plan_gram(snmf_plan* plan, const void* P, double* G, void* stream);
snmf_status snmf_rho(const double* G, int32_t r, double* rho, void* stream);
snmf_status snmf_spmm(const snmf_matrix* M, int32_t prec, const void* X, int32_t r, void* Y,
                      void* stream);
/* Average duration (ms) of the A-pass kernels (the dense MFMA product, the CSR SpMM or
 * the three LAI kernels; for BF16X3 the partner split runs once, untimed) over `reps`
 * back-to-back launches on the plan's stream, measured with HIP events after one
 * untimed launch.  P is an n x r device array; the products land in plan scratch. */
snmf_status snmf_plan_time_apass(snmf_plan* plan, const void* P, int32_t reps, double* ms);

/* BF16 round-to-nearest-even split of n*ld floats: hi = bf16(x), lo = bf16(x - hi);
 * hi and lo are uint16 device arrays of n*ld elements. */
snmf_status snmf_split_bf16(const float* x, int64_t count, uint16_t* hi, uint16_t* lo,
                            void* stream);

/* ---------------------------------------------------------------- LAI sketch, SVD start
 * The randomized range finder that builds the low-rank surrogate A ~= U diag(lam) U^T of
 * LAI-SNMPBB (Section 2.3: a random sketch A S = Q R, Q^T A Q = P E P^T, U = Q P).  The
 * paper leaves the sketch open; this library takes S = Omega, a Gaussian n x ell matrix
 * with ell = rank + oversample drawn by the caller, and power_iters rounds of subspace
 * iteration with an orthonormalisation after every product:
 *   Y = A Omega, Q = orth(Y); power_iters times { Q = orth(A Q), Q = orth(A Q) };
 *   T = Q^T A Q = P E P^T; the rank eigenpairs of largest |E| (ties: lower index first):
 *   U = Q P_rank (n x rank, orthonormal columns), lam = E_rank (decreasing |lam|).
 * orth() is a shifted Cholesky QR followed by two plain ones, the Gram products in FP64;
 * the small eigenproblem is solved by Jacobi rotations in FP64.  All on the device.
 * A: dense (read in place; symmetry is the caller's promise) or CSR (structure and
 *    symmetry checked: E_SHAPE, E_NOT_SYMMETRIC); LOWRANK: E_UNSUPPORTED.
 * prec: SNMF_F32 or SNMF_F64, the type of A's values, Omega and U_out.
 * Omega: n x (rank + oversample) device array; U_out: n x rank device array; lam_out:
 *    rank doubles (device).  1 <= rank, 0 <= oversample, rank + oversample <= min(128, n),
 *    0 <= power_iters <= 16 (else E_SHAPE / E_ARG).  E_BREAKDOWN if the sketch has lost
 *    rank beyond what the shifted factorisation absorbs.  Scratch memory is allocated and
 *    freed inside the call; the stream is synchronised before it returns. */
snmf_status snmf_lai_sketch(const snmf_matrix* A, int32_t rank, int32_t oversample,
                            int32_t power_iters, int32_t prec, const void* Omega, void* U_out,
                            double* lam_out, void* stream);
/* The SVD-based start of the numerical experiments (Section 4.2): with the leading r
 * singular triplets A ~= U E V^T, W0 = |U E^(1/2)| (and H0 = |E^(1/2) V^T|, which for a
 * symmetric A is W0^T: the singular triplets are eigenpairs, E = |lam|, V = U sign(lam)).
 * The triplets come from the range finder above with rank = r; W0_out is n x r (device,
 * of the precision's type), ready to be passed as W0 to snmf_solve.  Omega is
 * n x (r + oversample).  Errors as snmf_lai_sketch, and E_SHAPE for r > 64. */
snmf_status snmf_svd_start(const snmf_matrix* A, int32_t r, int32_t oversample,
                           int32_t power_iters, int32_t prec, const void* Omega, void* W0_out,
                           void* stream);

/* ---------------------------------------------------------------- graph preprocessing
 * The similarity matrix of data points that Graph-SNMPBB factors, and the Laplacian of
 * its regulariser (Section 2.2, after Kuang et al.: a Gaussian kernel with parameter sigma,
 * keeping each point's K nearest neighbours; eq. (2.3): L = I - D^{-1/2} V D^{-1/2},
 * d_i = sum_j V_ij).  Readings: Euclidean neighbours, the point itself excluded, ties to
 * the lower index (distances in FP64 on the device); the kernel exp(-||x_i - x_j||^2 /
 * (2 sigma^2)), sigma = 0 for the unweighted graph (kept entries 1); the pattern is
 * symmetrised by union (kept when either point lists the other); an isolated point has
 * L_ii = 1.
 * X: n x dim row-major device array (float for F32, double for F64), 1 <= dim <= 64,
 * 1 <= K <= min(64, n - 1), 2 <= n < 2^31.
 * snmf_knn: nbr_out (n x K int32, device): the neighbours of every point by increasing
 *   distance.
 * snmf_knn_graph: the CSR matrix V (laplacian = 0) or L (laplacian = 1, with the diagonal)
 *   with sorted columns: rowptr_out (n + 1 int64), col_out (int32) and val_out (float or
 *   double) device arrays of `capacity` >= n (2 K + laplacian) entries (the largest
 *   possible union; E_SHAPE otherwise, nothing written); *nnz_out (host) receives the
 *   number of entries.  Scratch memory is allocated and freed inside the call; the stream
 *   is synchronised before it returns. */
snmf_status snmf_knn(const void* X, int64_t n, int32_t dim, int32_t K, int32_t prec,
                     int32_t* nbr_out, void* stream);
snmf_status snmf_knn_graph(const void* X, int64_t n, int32_t dim, int32_t K, double sigma,
                           int32_t laplacian, int32_t prec, int64_t* rowptr_out,
                           int32_t* col_out, void* val_out, int64_t capacity, int64_t* nnz_out,
                           void* stream);

/* ---------------------------------------------------------------- batched solves
 * The batching form: many independent SNMPBB solves (problem g, restart s) run together,
 * every kernel of a half-step covering all of them in one launch (one per distinct rank
 * for the row-tile kernels), the whole outer iteration replayed as one hipGraph.  Each
 * instance keeps its own scalars (rho, BB steps, line search, nonmonotone reference,
 * monitor, stop flag), so instance (g, s) follows exactly the iteration of a single
 * solve of problem g from its start; the restarts of a problem share one sweep over its
 * CSR matrix in the A-pass (B_s = A P_s for all s at once); with dense A in BF16X3 the
 * restarts share one stream of A_hi and A_lo (one stacked split-BF16 product of S r
 * columns).  This form is not in the paper: it serves many-small-graph workloads and
 * multi-start runs.
 *
 * A:        nprob matrices, all CSR or all DENSE, symmetric, n_g >= 1 (LOWRANK and a
 *           Laplacian term are not supported: E_UNSUPPORTED).
 * r:        nprob ranks, 1 <= r_g <= min(64, n_g).
 * lam:      nprob penalties lambda_g (host), or NULL to use p->lambda for every problem.
 * restarts: S >= 1 starts per problem.
 * p:        shared parameters (precision F64 or F32, or BF16X3 for dense A: the A-pass
 *           in split BF16 as for the single solve, everything else in FP32; max_outer,
 *           target_res and check_every apply per instance; gamma and L are ignored).
 *           BF16X3 with CSR A: E_UNSUPPORTED.
 * W0[g]:    device array of S * n_g * r_g values: restart s is the n_g x r_g row-major
 *           block at offset s * n_g * r_g.  W_out[g], Ht_out[g] have the same layout.
 * infos:    host array of nprob * S records, instance g * S + s.
 * traces:   optional host array of nprob * S * max_outer * SNMF_TRACE_FIELDS doubles,
 *           instance-major, the records of snmf_solve.
 * The library keeps the A pointers until destroy; all other buffers are the caller's.
 * Errors as for the single solve, except numeric breakdown: an instance whose iteration
 * breaks down (a non-finite scalar, or rho = 0 after its factor collapsed to zero) stops,
 * keeps its last iterate and reports SNMF_E_BREAKDOWN in infos[i].status while the call
 * returns SNMF_OK.  Trace records beyond infos[i].outer are unspecified. */
typedef struct snmf_batch snmf_batch;
snmf_status snmf_batch_create(int32_t nprob, const snmf_matrix* A, const int32_t* r,
                              const double* lam, int32_t restarts, const snmf_params* p,
                              void* stream, snmf_batch** out);
snmf_status snmf_batch_solve(snmf_batch* b, const void* const* W0, void* const* W_out,
                             void* const* Ht_out, snmf_info* infos, void* stream,
                             double* traces);
snmf_status snmf_batch_destroy(snmf_batch* b);
snmf_status snmf_solve_batched(int32_t nprob, const snmf_matrix* A, const int32_t* r,
                               const double* lam, int32_t restarts, const void* const* W0,
                               const snmf_params* p, void* const* W_out, void* const* Ht_out,
                               snmf_info* infos, void* stream, double* traces);
/* The batch's A-pass alone: P and B are device arrays holding every instance's n_g x r_g
 * block one after another in instance order (g * S + s), B = A_g P for each. */
snmf_status snmf_batch_apass(snmf_batch* b, const void* P, void* B, void* stream);
/* Average duration (ms) of the batch's A-pass (every launch of snmf_batch_apass: for
 * BF16X3 the stacked partner split and the stacked product of each problem) over `reps`
 * back-to-back runs on the batch's stream, measured with HIP events after one untimed
 * run.  P is a batch buffer (device); the products land in batch scratch. */
snmf_status snmf_batch_time_apass(snmf_batch* b, const void* P, int32_t reps, double* ms);
/* Number of instances and the total element count sum_g S n_g r_g of a batch buffer. */
snmf_status snmf_batch_size(const snmf_batch* b, int32_t* ninst, int64_t* elements);

/* ---------------------------------------------------------------- learned warm start
 * Not in the paper (its closest analogue is the SVD-based start of Section 4.2).  A start
 * W0 for each instance of a batch (CSR problems) from a Gaussian sketch Omega:
 *   Y = A Omega; SPA (successive projection, Gillis & Vavasis 2014) on the rows Y_i / d_i,
 *   d = A 1, gives r anchor rows K; C = Y Y_K^T (Y_K Y_K^T + eps I)^{-1},
 *   eps = 1e-12 tr(Y_K Y_K^T) / r (the coordinates in the anchor frame), divided by the
 *   entry RMS of relu(C) (so that every problem's coordinates have one scale);
 *   W0_i = s relu(c_i + M2 relu(M1 c_i + b1) + b2), s = (sqrt(r) ||A||_F / (n r))^(1/2),
 *   a residual network that is the frame's own start s relu(c_i) while M2 = 0, b2 = 0.
 * The network (one per rank r) is trained on converged factors whose columns are matched
 * to the anchor order (linear assignment on column cosines) and divided by their entry
 * RMS (the factor's shape; s sets its scale); the loss is
 * mean((y - t)^2) + mu (mean(y^2) - mean(t^2))^2, the optimiser Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8).  All arrays below are device arrays; the caller owns them. */
typedef struct snmf_mlp {
  int32_t r;          /* 1..64 */
  int32_t hidden;     /* must be 128 */
  float* M1;          /* hidden x r, FP32 master weights */
  float* b1;          /* hidden */
  float* M2;          /* r x hidden */
  float* b2;          /* r */
  uint16_t* M1h;      /* BF16 (round to nearest even) copies of M1, M2 used by the forward */
  uint16_t* M2h;
  float* adam_m;      /* Adam moments, 2 hidden r + hidden + r floats each, in the order */
  float* adam_v;      /*   M1, b1, M2, b2 (needed by training only; zero before step 1) */
} snmf_mlp;
/* Refresh M1h, M2h from M1, M2. */
snmf_status snmf_mlp_sync(const snmf_mlp* m, void* stream);
/* Y (rows x r) = row_scale[i] * net(C_i) for every row (row_scale NULL: scale 1). */
snmf_status snmf_mlp_forward(const snmf_mlp* m, int64_t rows, const float* C,
                             const float* row_scale, float* Y, void* stream);
/* One training step on the `batch` rows idx[0..batch) of the row pools C and T
 * (pool_rows x r each; indices outside [0, pool_rows) are clamped into it): loss,
 * gradients reduced in a fixed order, Adam step number `step` (from 1), BF16 copies
 * refreshed.  work: device scratch of snmf_mlp_workspace_bytes(r, batch) bytes.
 * loss (host, optional): the minibatch loss before the update (synchronises). */
size_t snmf_mlp_workspace_bytes(int32_t r, int64_t batch);
snmf_status snmf_mlp_train_step(const snmf_mlp* m, int64_t pool_rows, const float* C,
                                const float* T, const int32_t* idx, int64_t batch, float mu,
                                float lr, int32_t step, void* work, size_t work_bytes,
                                void* stream, double* loss);
/* The frame of every instance of a CSR batch: Omega, Y, C are batch buffers (the
 * instance-major layout of snmf_batch_apass), C scaled to rms(relu(C)) = 1 per instance;
 * anchors (optional): 64 ints per instance. */
snmf_status snmf_batch_frame(snmf_batch* b, const void* Omega, void* Y, void* C,
                             int32_t* anchors, void* stream);
/* Training targets: T[:, j] = Ht[:, p[j]] / rms(Ht) per instance, p the column assignment
 * maximising sum_j cos(C_j, Ht_p[j]); perm (optional): 64 ints per instance. */
snmf_status snmf_batch_targets(snmf_batch* b, const void* C, const void* Ht, void* T,
                               int32_t* perm, void* stream);
/* W0 (batch buffer) for every instance: frame of Omega, then the network whose r matches
 * the instance's rank (E_ARG if none; FP32 batches only).  nmodels = 0: the frame alone,
 * W0 = s relu(C) / rms(relu(C)) per instance (the ablation without the network).  Dense
 * batches take the degrees d = A 1 from a row sum on the device (BF16X3 dense batches:
 * E_UNSUPPORTED). */
snmf_status snmf_batch_warmstart(snmf_batch* b, int32_t nmodels, const snmf_mlp* models,
                                 const void* Omega, void* W0, void* stream);

/* The warm start of one problem (dense or CSR A, F32 or F64), without a batch: the same
 * sketch, frame and network as snmf_batch_warmstart for a batch of one problem with one
 * start.  Omega (n x r, device, of the precision's type) is the Gaussian sketch matrix,
 * drawn by the caller; W0_out (n x r) receives the start.  mlp = NULL gives the start of
 * the frame alone, W0 = s relu(C) / rms(relu(C)); otherwise mlp->r must equal r and prec
 * must be F32.  Dense A is read in place (its degrees d = A 1 are summed on the device in
 * FP64).  Scratch memory is allocated and freed inside the call.  Errors: E_ARG (null
 * pointers, prec not F32/F64), E_SHAPE (r outside [1, min(64, n)], network rank != r),
 * E_UNSUPPORTED (LOWRANK A, a network with F64), and the input checks of a solve. */
snmf_status snmf_warmstart(const snmf_mlp* mlp, const snmf_matrix* A, int32_t r, int32_t prec,
                           const void* Omega, void* W0_out, void* stream);

/* NMPBB for rectangular NMF, min ||V - W Ht^T||_F^2 / 2 over W, Ht >= 0 (eq. (1.1)), with
 * the alternating scheme of Section 2.1: each outer iteration runs inner_iters iterations
 * of Algorithm 1 on W (the partner Ht, gradient W Ht^T Ht - V Ht), then on Ht (partner W,
 * gradient Ht W^T W - V^T W), with the same first projection, BB steps, nonmonotone line
 * search and stopping tests as the symmetric solve but no penalty term.
 * V: m x n_cols, dense (row-major, ld >= n_cols, read in place) or CSR (m rows, columns in
 *    [0, n_cols) strictly increasing per row; its transpose is formed once on the device
 *    in deterministic order); entries >= 0.  LOWRANK is E_UNSUPPORTED.
 * W0 (m x r), Ht0 (n_cols x r): device, row-major, of the precision's type, >= 0; not
 *    modified.  W_out, Ht_out: device, same shapes, caller-owned.
 * p: prec F32 or F64 (else E_UNSUPPORTED); lambda must be 0 (E_ARG otherwise) and L NULL;
 *    max_outer, inner_iters, line-search and stopping fields as for snmf_solve.
 * info: res_WH = ||V - W Ht^T||_F / ||V||_F, pg_norm the projected gradient of the pair,
 *    objective = res^2 ||V||^2 / 2; res_WWt and sym_gap are NaN.  trace (host, optional,
 *    max_outer x 10 doubles): the per-outer records of snmf_solve, fields 1 and 2 NaN.
 * Scratch memory (about 8 max(m, n_cols) r elements, plus the transpose of a CSR V) is
 * allocated and freed inside the call; the call synchronises the stream.
 * Errors: E_ARG (null pointers, lambda != 0, V zero), E_SHAPE (r outside [1, min(64, m,
 * n_cols)], malformed CSR, ld < n_cols), E_NEGATIVE / E_NONFINITE (inputs), E_BREAKDOWN
 * (a factor collapsed to zero or a scalar overflowed: the outputs hold the last iterate,
 * info the last completed record, as in snmf_solve). */
snmf_status snmf_nmf_solve(const snmf_matrix* V, int64_t n_cols, int32_t r, const void* W0,
                           const void* Ht0, const snmf_params* p, void* W_out, void* Ht_out,
                           snmf_info* info, void* stream, double* trace);

/* Device clock rate (Hz) of the trace ticks and info.seconds. */
double snmf_clock_rate_hz(void);
const char* snmf_last_error(void);
int32_t snmf_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SNMF_H */
