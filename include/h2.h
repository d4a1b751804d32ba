/*
 * h2.h -- C ABI of the MI355X H2 Hessian library.
 *
 * The library builds H2 (nested-basis, strong-admissibility) approximations of
 * symmetric operators that are available only through products with blocks of
 * vectors, applies them (HGEMV) and inverts them by hierarchical Newton-Schulz,
 * following arXiv 2003.10173, "Hierarchical Matrix Approximations of Hessians
 * Arising in Inverse Problems Governed by PDEs":
 *   - format and four-stage product: Sec. 3.1 (Fig. 2, A = D + U S V^T) and
 *     Sec. 3.2 (matrix-vector multiplication; recompression; norms)
 *   - construction from Hessian-vector products (peeling): Sec. 3.3
 *   - Newton-Schulz on H2: Appendix A, Alg. 1 (iteration), Alg. 2 (hierarchical
 *     iteration with a construction threshold per step), Alg. 3 (sampler)
 *
 * Conventions for every entry point
 *   - All functions return h2_status; no C++ exception crosses the ABI.
 *   - "device" pointers are HIP device memory on the current device; "host"
 *     pointers are ordinary host memory.  The caller owns every buffer it
 *     passes; the library owns h2_tree / h2_matrix objects and their device
 *     storage, released by the matching *_destroy call.
 *   - Multivectors are column-major (column j starts at ptr + j*ld) in the
 *     caller's (user) point ordering; the library permutes internally.
 *   - Work is enqueued on the given stream.  Entry points that must decide
 *     sizes from device results (ranks, convergence) synchronise that stream.
 *   - The matrices handled are symmetric (the Hessians of the paper), so the
 *     row basis tree equals the column basis tree (V = U).
 */
#ifndef H2_MI355X_H
#define H2_MI355X_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct h2_tree h2_tree;
typedef struct h2_matrix h2_matrix;
typedef struct h2_mlp h2_mlp;

typedef enum {
  H2_OK = 0,
  H2_EINVAL = -1,         /* bad argument (null pointer, size out of range, ...) */
  H2_ENOMEM = -2,         /* device or host allocation failed */
  H2_EDEVICE = -3,        /* a HIP call failed */
  H2_ECALLBACK = -4,      /* the sampler callback returned nonzero */
  H2_ENUMERIC = -5,       /* NaN/Inf met in samples or factors */
  H2_ENOTCONVERGED = 1,   /* usable best-effort result; a budget was exhausted */
  H2_EDIVERGED = 2        /* Newton-Schulz residual grew above 1 */
} h2_status;

/* storage / GEMM precision of an H2 matrix (vectors of h2_gemv_f32 are FP32) */
typedef enum { H2_FP64 = 0, H2_FP32 = 1, H2_BF16 = 2 } h2_precision;

/*
 * Sampler: Y(:, 0:ncols) = A * Omega(:, 0:ncols)  (Sec. 3.3: the operator is
 * known only through such products; one Hessian-vector product costs one
 * forward and one adjoint PDE solve, Sec. 2).  omega and y are device
 * pointers, column-major, user ordering, FP64.  The callback must only
 * enqueue work on `stream`.  A nonzero return aborts the calling entry point
 * with H2_ECALLBACK after the library has released its temporaries.
 */
typedef int (*h2_sampler_fn)(void* ctx, int n, int ncols, const double* omega, int ld_omega,
                             double* y, int ld_y, hipStream_t stream);

/*
 * Batched sampler: one call applies the operators of many problems at once
 * (the batched construction below, for callers whose Hessian-vector products
 * of many problems run best as one multi-right-hand-side launch).  Packed
 * layout: problem i owns rows row_off[i] .. row_off[i+1] - 1 (its user
 * ordering) of the column-major device blocks omega and y, leading dimension
 * ld = row_off[nprob]; every problem has the same ncols columns.  active[i] = 0:
 * problem i needs no product in this call (its rows of omega are zero and its
 * rows of y are not read).  row_off and active are host arrays, valid during
 * the call.  Only enqueue work on `stream`; nonzero return = H2_ECALLBACK.
 */
typedef int (*h2_batched_sampler_fn)(void* ctx, int nprob, const int64_t* row_off,
                                     const int32_t* active, int ncols, const double* omega,
                                     int ld, double* y, hipStream_t stream);

/* ------------------------------------------------------------------ tree */
/*
 * Cluster tree by KD binary space partition (Sec. 4.2: KD-tree ordering with
 * leaf clusters of size m) and strong-admissibility block lists (Sec. 2 and
 * Sec. 3.1: a block is low rank when its clusters are far apart relative to
 * their size).  Rules: depth L = smallest L with leaf_size * 2^L >= n (0 when
 * n <= leaf_size); a cluster splits along its widest bounding-box dimension
 * (lowest index on ties), points ordered by (coordinate, user index), the left
 * child taking ceil(size/2); (t, s) admissible iff
 *   max(diam2_t, diam2_s) <= (eta*eta) * dist2(t, s)
 * with squared box diameters and box distance summed in dimension order (no
 * fused multiply-add); far pairs at levels >= 1, near pairs at the leaf level.
 * points_host: n x dim, row-major, host.  1 <= dim <= 3.
 */
h2_status h2_tree_create(const double* points_host, int n, int dim, int leaf_size, double eta,
                         h2_tree** out);
void h2_tree_destroy(h2_tree* tree);
/* n, number of levels L (leaves at level L), leaf size, dimension (any may be NULL) */
h2_status h2_tree_info(const h2_tree* tree, int* n, int* levels, int* leaf_size, int* dim);
/* perm_host[i] = user index of tree position i (n entries) */
h2_status h2_tree_perm(const h2_tree* tree, int64_t* perm_host);
/* cluster boundaries of a level: 2^level + 1 tree positions */
h2_status h2_tree_offsets(const h2_tree* tree, int level, int64_t* offsets_host);
/* number of far pairs at `level` (level in 0..L) or near pairs (level = -1) */
h2_status h2_tree_pair_count(const h2_tree* tree, int level, int64_t* count);
/* the pairs (t, s), sorted by (t, s): pairs_host[2*i], pairs_host[2*i+1] */
h2_status h2_tree_pairs(const h2_tree* tree, int level, int32_t* pairs_host);

/* ------------------------------------------------------------------ H2 */
typedef struct {
  int rank_cap;        /* destination H2 rank cap per cluster basis */
  int oversample;      /* p: columns per sampling round = rank_cap + p */
  double tol;          /* relative 2-norm target eps; tau = eps * nu / (4 L) */
  int adaptive;        /* 1: HMT-estimated rounds; 0: one round per level */
  int max_rounds;      /* adaptive round budget per level (>= 2) */
  uint64_t seed;       /* counter-based Gaussian stream seed */
  uint32_t iteration;  /* stream tag (Newton-Schulz iteration index) */
  double norm;         /* ||A||_2 if known (> 0); else estimated (power method) */
  h2_precision prec;   /* FP64 only for construction; see h2_matrix_convert */
  const h2_mlp* learned; /* NULL: plain adaptive sampling.  Otherwise (adaptive
                          mode) the network's predictions set the width of each
                          level's first sampling round (see h2_mlp_create); the
                          estimator still decides when sampling stops */
} h2_opts;

#define H2_MAX_LEVELS 32
typedef struct {
  int levels;
  int weak_rank[H2_MAX_LEVELS];    /* max rank of the sampled sibling blocks, level l */
  int range_cols[H2_MAX_LEVELS];   /* max range-basis width k0 at level l */
  int rounds[H2_MAX_LEVELS];       /* sampling rounds at level l */
  int strong_rank[H2_MAX_LEVELS];  /* max cluster-basis rank at level l (destination) */
  int64_t applies;                 /* sampler columns of the peeling (samples, projections, diagonal) */
  int64_t norm_applies;            /* sampler columns of the norm estimate */
  double norm;                     /* ||A||_2 used for the thresholds */
  int converged;                   /* 1 if every level met the estimator */
  int cap_hit;                     /* 1 if the rank cap truncated a basis */
  double time_ms[8];               /* norm, sample, range, project, diag, recompress, sampler, total */
  int first_cols[H2_MAX_LEVELS];   /* width of the first sampling round at level l */
  int global_rank;                 /* h2_build_lowrank: columns of B (else 0) */
  int64_t global_applies;          /* h2_build_lowrank: sampler columns of the range finder */
  int64_t update_applies;          /* h2_build_lowrank: H2 + low-rank columns of the update */
} h2_build_stats;

/*
 * Batched construction: nprob independent problems (trees, samplers,
 * contexts and options per problem) built level-synchronously on one stream.
 * Every launch of a phase (projections, QR, SVD, subtraction of peeled
 * levels, recompression) covers the blocks of every problem that has that
 * level; the samplers are called problem by problem.  out[i] receives each
 * result; stats (nullable) is an array of nprob.  Each result equals the
 * h2_build of the same problem.  H2_ENOTCONVERGED if any problem ran out of
 * rounds; on an error every out[i] is NULL.
 */
h2_status h2_build_batched(int nprob, const h2_tree* const* trees, const h2_sampler_fn* samplers,
                           void* const* ctxs, const h2_opts* opts, hipStream_t stream,
                           h2_matrix** out, h2_build_stats* stats);

/*
 * The same batched construction with ONE batched sampler for all problems:
 * each phase of each level (the rounds of sampling, the projections, the
 * leaf diagonal, every power-method step of the norm estimates) calls
 * `sampler` once for every problem that needs products in it, over the
 * packed layout (row_off[i] = n_0 + ... + n_{i-1}), with the largest column
 * count requested in that phase (a problem that needs fewer columns gets
 * zero columns beyond its own, whose products are discarded).  So the number
 * of calls grows with levels and rounds, not with problems.  Results equal
 * h2_build_batched with per-problem samplers of the same operators.
 * sampler_calls (nullable) receives the number of calls made.
 */
h2_status h2_build_batched_packed(int nprob, const h2_tree* const* trees,
                                  h2_batched_sampler_fn sampler, void* ctx, const h2_opts* opts,
                                  hipStream_t stream, h2_matrix** out, h2_build_stats* stats,
                                  int64_t* sampler_calls);

/* default options: cap 32, p 10, tol 1e-4, adaptive, 16 rounds, seed 1 */
void h2_opts_default(h2_opts* opts);

/*
 * Construct an H2 approximation of the operator behind `sampler` by
 * randomized peeling on the weak (sibling) partition, level by level from
 * the root (Sec. 3.3), followed by recompression into the strong partition
 * of the tree (Sec. 3.2: QR downsweep, truncated-SVD upsweep, projection).
 * The result is FP64 on the device.
 */
h2_status h2_build(const h2_tree* tree, h2_sampler_fn sampler, void* ctx, const h2_opts* opts,
                   hipStream_t stream, h2_matrix** out, h2_build_stats* stats);

/*
 * Construction combined with a global low-rank approximation (Sec. 3.3, the
 * paragraph on combining with global low-rank approximations: for a data
 * misfit of small global rank, B B^T first, the hierarchical construction of
 * the residual H - B B^T next, and B B^T added back as a low-rank update).
 *   1. nu = ||H||_2 by the power method through `sampler` (unless opts->norm > 0)
 *   2. B (at most global_rank columns) by the two-pass randomized range finder
 *      with global_rank + oversample Gaussian columns: Y = H Omega, Q = qr(Y),
 *      T = Q^T H Q, T = V diag(s) V^T; the s above 1e-13 s_1 give
 *      B = Q V diag(sqrt(s)), so B B^T = Q T Q^T (H symmetric positive
 *      semi-definite)
 *   3. h2_build of the residual, sampler H Omega - B (B^T Omega), threshold
 *      tol * nu / (4 L), basis ranks capped at rank_cap + (columns of B): a
 *      global rank-r term adds up to r to every block's rank
 *   4. the update: h2_build from the sampler A_res Omega + B (B^T Omega) (no
 *      Hessian products), same threshold; its result is *out
 * stats: applies = the Hessian columns of steps 2 and 3 (norm_applies those of
 * step 1), global_rank and global_applies as named, update_applies the
 * columns of step 4; per-level weak ranks and rounds of step 3, strong ranks
 * of the result.  global_rank + oversample <= 1024.
 */
h2_status h2_build_lowrank(const h2_tree* tree, h2_sampler_fn sampler, void* ctx,
                           const h2_opts* opts, int global_rank, hipStream_t stream,
                           h2_matrix** out, h2_build_stats* stats);

/*
 * y = alpha * A x + beta * y for nv columns (Sec. 3.2, four-stage product:
 * upsweep, couplings, downsweep, dense near field).  FP64, device, user order.
 */
h2_status h2_gemv(const h2_matrix* A, int nv, double alpha, const double* x, int ldx,
                  double beta, double* y, int ldy, hipStream_t stream);
/* same with FP32 vectors; the matrix may be stored in FP64, FP32 or BF16 */
h2_status h2_gemv_f32(const h2_matrix* A, int nv, float alpha, const float* x, int ldx,
                      float beta, float* y, int ldy, hipStream_t stream);

/*
 * h2_gemv for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same product (FP64 matrix and vectors, device pointers, user order,
 * column-major) without any allocation.  Its workspace -- tree-order x and y
 * and the basis coefficients, 2 (n + sum of cluster ranks) nv FP64 words --
 * is a fixed array of 2^23 words (64 MiB) that the library holds on every
 * GPU it runs on until the process ends.  A product needing more returns
 * H2_EINVAL before any work is enqueued.  Every call on one GPU uses that
 * GPU's array: calls that overlap in time on one GPU (other streams, other
 * host threads) race and must be serialised by the caller.  The matrix-core
 * tile width is the one an earlier h2_gemv autotuned on the tree, else a
 * fixed rule (no timing runs); every width sums the same products in the
 * same order, so results equal h2_gemv's.
 */
h2_status h2_gemv_noalloc(const h2_matrix* A, int nv, double alpha, const double* x, int ldx,
                          double beta, double* y, int ldy, hipStream_t stream);

/* ||A||_2 by the power method stopped at relative change rel (Sec. 3.2) */
h2_status h2_norm2(const h2_matrix* A, int max_iter, double rel, uint64_t seed,
                   hipStream_t stream, double* out);

/* copy with storage in `prec` (FP32 or BF16 couplings/bases/dense blocks) */
h2_status h2_matrix_convert(const h2_matrix* A, h2_precision prec, h2_matrix** out);
/* scaled copy alpha*A, and the scaled identity alpha*I on a tree */
h2_status h2_matrix_scale(const h2_matrix* A, double alpha, h2_matrix** out);
h2_status h2_matrix_identity(const h2_tree* tree, double alpha, h2_matrix** out);
void h2_destroy(h2_matrix* A);

/*
 * Import / export in the packed host layout (all row-major FP64):
 *   ranks: one int32 per cluster, cluster (l, i) at index 2^l - 1 + i
 *   U:     leaf bases U_i (|leaf_i| x k_i) concatenated over leaves
 *   E:     transfers E_c (k_c x k_parent) for clusters c = 1 .. 2^(L+1)-2
 *   S:     couplings (k_t x k_s) of the far pairs in h2_tree_pairs order,
 *          levels ascending
 *   D:     dense blocks (|t| x |s|) of the near pairs in h2_tree_pairs order
 * h2_matrix_sizes returns the element counts of U, E, S, D for given ranks
 * (ranks_host NULL: the matrix's own ranks; tree from A or from `tree`).
 */
h2_status h2_matrix_sizes(const h2_tree* tree, const int32_t* ranks_host, int64_t* nU,
                          int64_t* nE, int64_t* nS, int64_t* nD);
h2_status h2_matrix_import(const h2_tree* tree, const int32_t* ranks_host, const double* U,
                           const double* E, const double* S, const double* D, h2_matrix** out);
h2_status h2_matrix_ranks(const h2_matrix* A, int32_t* ranks_host);
h2_status h2_matrix_export(const h2_matrix* A, double* U, double* E, double* S, double* D);
/* matrix words per HGEMV (U, E, S, D element counts summed) and storage bytes */
h2_status h2_matrix_words(const h2_matrix* A, int64_t* words, int64_t* bytes);

/* ------------------------------------------------------------------ Newton-Schulz */
typedef struct {
  double eps;          /* stop when E = ||I - A X||_2 <= eps (0: never) */
  int max_iter;        /* iteration budget */
  int x0;              /* 0: X0 = I / ||A||_2;  1: X0 = A^T / ||A||_2^2;
                          2: warm start X0 = x0_matrix (Appendix A.1: the
                          inverse from the previous optimisation step) */
  int dynamic;         /* 1: eps_k = clamp(0.1 E^2, eps_build, 1e-2); 0: eps_build */
  double eps_build;    /* static construction threshold (0: eps / 10) */
  double norm_rel;     /* power-method relative change for ||A||_2 (0: 1e-2) */
  double resid_rel;    /* power-method relative change for E (0: 1e-2) */
  int rank_cap;        /* iterate rank cap (0: the leaf size) */
  int oversample;
  int adaptive;
  int max_rounds;
  uint64_t seed;
  h2_precision prec;   /* H2_FP64: every sampler product in FP64.  H2_FP32: while
                          E > sqrt(eps) the sampler's HGEMVs run on FP32 copies of
                          A and X_k (FP32 matrix cores); the residual E is always
                          FP64, and the iterations after the switch (the
                          refinement) are FP64.  BF16 is refused: BF16 iterates
                          carry 2^-9 relative rounding, a residual floor of about
                          4e-3 cond(A).  Orders above 2 need FP64. */
  int order;           /* hyperpower order l of every step (Appendix A.2):
                          X_{k+1} = X_k (I + R_k + ... + R_k^(l-1)), R_k = I - A X_k,
                          sampled Horner-style (Alg. 4, 2l - 1 HGEMVs per block of
                          samples); 0 or 2: Newton-Schulz (Alg. 3, 3 HGEMVs) */
  int unroll;          /* u > 0: each construction builds u Newton-Schulz steps
                          unrolled in terms of the current iterate (Appendix A.3),
                          X_{k+u} = X_k sum_{i < 2^u} R_k^i, i.e. order 2^u
                          (1 <= u <= 10; order must then be 0) */
  const h2_matrix* x0_matrix; /* x0 = 2: FP64 H2 on A's tree (not modified) */
} h2_ns_opts;

#define H2_MAX_NS_ITERS 128
typedef struct {
  int iterations;
  double norm;                      /* ||A||_2 estimate */
  double resid[H2_MAX_NS_ITERS + 1];/* E_k history, FP64 */
  int64_t applies[H2_MAX_NS_ITERS]; /* sampler columns per iteration */
  int max_rank[H2_MAX_NS_ITERS];    /* largest basis rank of each iterate */
  double time_ms[4];                /* residual, build, refine, total */
  int low_iterations;               /* iterations built from FP32 samples */
} h2_ns_stats;

void h2_ns_opts_default(h2_ns_opts* opts);

/*
 * Hierarchical Newton-Schulz (Appendix A, Alg. 2): X_{k+1} is rebuilt by
 * h2_build from the sampler Y = 2W - X_k (A W), W = X_k Omega (Alg. 3), at
 * threshold eps_k, on the tree and partition of A; iterates are built to
 * absolute accuracy eps_k / ||A||_2.  Returns H2_OK when E <= eps,
 * H2_ENOTCONVERGED when the budget ran out, H2_EDIVERGED on growth above 1.
 * *X_out always receives the last iterate.
 */
h2_status h2_newton_schulz(const h2_matrix* A, const h2_ns_opts* opts, hipStream_t stream,
                           h2_matrix** X_out, h2_ns_stats* stats);

/*
 * Newton-Schulz for nprob independent FP64 matrices in lock step: each
 * iteration evaluates every unfinished problem's residual, then rebuilds all
 * unfinished iterates in one batched construction (h2_build_batched).
 * opts, X_out, stats (nullable) and status (nullable) are arrays of nprob;
 * status[i] is what h2_newton_schulz would return for problem i.
 */
h2_status h2_newton_schulz_batched(int nprob, const h2_matrix* const* A, const h2_ns_opts* opts,
                                   hipStream_t stream, h2_matrix** X_out, h2_ns_stats* stats,
                                   h2_status* status);

/* E = ||I - A X||_2 by the power method on R^T R (four HGEMVs per step) */
h2_status h2_residual_norm(const h2_matrix* A, const h2_matrix* X, double rel, int max_iter,
                           uint64_t seed, uint32_t iteration, hipStream_t stream, double* out);
/* The same for nprob (A[i], X[i]) pairs in lock step: one device-to-host
 * copy per power step for all pairs.  graph != 0: after an eager first step
 * the step's launch sequence (HGEMVs, copies, norms, normalisations of every
 * unfinished pair) is captured once per set of unfinished pairs into a HIP
 * graph and replayed.  out, iters (nullable) have nprob entries; history
 * (nullable, nprob x max_iter) receives the estimate after every step (0
 * after a pair stopped).  Newton-Schulz (batched or not) evaluates its
 * residuals this way with graphs. */
h2_status h2_residual_norm_batched(int nprob, const h2_matrix* const* A, const h2_matrix* const* X,
                                   double rel, int max_iter, uint64_t seed, uint32_t iteration,
                                   int graph, hipStream_t stream, double* out, int* iters,
                                   double* history);

/* ------------------------------------------------------------------ samplers */
/*
 * Built-in samplers for the synthetic Hessians (h2_sampler_fn compatible;
 * pass the returned context as ctx).  They run as HIP kernels on `stream`.
 *   kernel:    H_ij = exp(-|p_i - p_j| / ell) + shift delta_ij, points n x dim
 *   diffusion: H = F^T F / sigma^2 + gamma (I - beta Lap)^2 on a g x g interior
 *              grid (h = 1/(g+1)), F = point observations (obs_count^2 nodes
 *              from obs_index) after explicit Euler heat steps u <- u + dt kappa
 *              Lap u at the listed step numbers; F^T by exact adjoint steps
 *   advdiff:   H = F^T F / sigma^2, upwind advection-diffusion on a g x g grid
 *              with velocity from sum_j s_j sin(pi a_j x) sin(pi b_j y), and
 *              bilinear point observations (x, y in (0,1)) at the listed steps
 */
h2_status h2_sampler_kernel_create(const double* points_host, int n, int dim, double ell,
                                   double shift, void** ctx);
int h2_sampler_kernel_apply(void* ctx, int n, int ncols, const double* omega, int ld_omega,
                            double* y, int ld_y, hipStream_t stream);
h2_status h2_sampler_diffusion_create(int g, double kappa, double dt, int steps,
                                      const int32_t* obs_steps, int n_obs_steps,
                                      const int32_t* obs_index, int obs_count, double sigma,
                                      double gamma, double beta, void** ctx);
int h2_sampler_diffusion_apply(void* ctx, int n, int ncols, const double* omega, int ld_omega,
                               double* y, int ld_y, hipStream_t stream);
h2_status h2_sampler_advdiff_create(int g, double kappa, int steps, const int32_t* obs_steps,
                                    int n_obs_steps, const double* obs_points_host, int n_obs,
                                    double sigma, const int32_t* mode_a, const int32_t* mode_b,
                                    const double* mode_s, int n_modes, void** ctx);
int h2_sampler_advdiff_apply(void* ctx, int n, int ncols, const double* omega, int ld_omega,
                             double* y, int ld_y, hipStream_t stream);
/*
 * minsurf: Hessian of the discrete minimal-surface area (Appendix A, the
 * shape-optimisation example: surface area over the unit square with the
 * boundary heights fixed, on a g x g interior grid, h = 1/(g+1)).
 * heights_host: (g+2) x (g+2) node heights, row-major [iy][ix], boundary
 * included; unknowns are the interior nodes, user index (iy-1) g + (ix-1).
 * Each cell is cut along its anti-diagonal into two triangles on which the
 * height is linear; J = sum_T (h^2/2) sqrt(1 + |grad m|^2) and the sampler
 * applies its exact Hessian at the given surface (a sparse SPD operator).
 */
h2_status h2_sampler_minsurf_create(int g, const double* heights_host, void** ctx);
int h2_sampler_minsurf_apply(void* ctx, int n, int ncols, const double* omega, int ld_omega,
                             double* y, int ld_y, hipStream_t stream);
/*
 * kernel_batched: h2_batched_sampler_fn for nprob kernel matrices (the
 * kernel sampler's H_ij = exp(-|p_i - p_j| / ell_b) + shift_b delta_ij per
 * problem b) in one launch over the packed layout.  points_host: the
 * problems' points stacked in row_off order (row_off[nprob] x dim); ell and
 * shift: one per problem.  Each problem's product equals
 * h2_sampler_kernel_apply's for the same points.
 */
h2_status h2_sampler_kernel_batched_create(int nprob, const int64_t* row_off_host,
                                           const double* points_host, int dim,
                                           const double* ell_host, const double* shift_host,
                                           void** ctx);
int h2_sampler_kernel_batched_apply(void* ctx, int nprob, const int64_t* row_off,
                                    const int32_t* active, int ncols, const double* omega, int ld,
                                    double* y, hipStream_t stream);
/* sampler that applies an H2 matrix (h2_gemv) -- ctx is the h2_matrix pointer */
int h2_sampler_h2_apply(void* ctx, int n, int ncols, const double* omega, int ld_omega,
                        double* y, int ld_y, hipStream_t stream);
void h2_sampler_destroy(void* ctx);

/* ------------------------------------------------------------------ learned counts */
/*
 * Rank predictor for the adaptive range finder of Sec. 3.3 (not from the
 * paper; the estimator stays the stopping rule).  For sibling pair p of
 * level l (t2 = cluster 2p+1) the network maps 16 features to a predicted
 * log(1 + c), c the sample columns the pair held when the estimator accepted
 * it in a plain adaptive build; the first sampling round
 * of the level takes max_p (expm1(y_p), rounded up) + oversample columns
 * (at least rank_cap + oversample, at most 1024 - (rank_cap + oversample)).
 * Features, in order:
 *   l / L;  log2|t2| / 16;  the three box extents of t2, largest first, over
 *   the largest root extent (0 for missing dimensions);  log10((e_max + d) /
 *   (e_min + d)) / 4 over the dimensions, d = 1e-12 root extent (0 in 1D);
 *   dim / 3;  log10(eps) / 10;  for i = 2, 4, ..., 128: max(log10(s_i /
 *   s_1), -16) / 16 over the singular values s of the parent pair's block
 *   (level l - 1, pair p / 2; -1 where it has fewer than i values; 0 at
 *   level 1);  log2(1 + parent rank) / 10 (-1 at level 1).
 * Network: 16 -> 64 -> 64 -> 1, ReLU after the hidden layers; products with
 * BF16 copies of the weights (round to nearest even), FP32 activations and
 * accumulation.  Packed FP32 parameters: W1 (64 x 16, row-major), b1 (64),
 * W2 (64 x 64), b2 (64), W3 (64), b3 (1): H2_MLP_PARAMS floats.
 */
#define H2_MLP_FEATURES 16
#define H2_MLP_HIDDEN 64
#define H2_MLP_PARAMS 5313
/* copies params_host (FP32 masters); Adam moments start at zero */
h2_status h2_mlp_create(const float* params_host, h2_mlp** out);
/* current FP32 master parameters (synchronises the device) */
h2_status h2_mlp_params(const h2_mlp* m, float* params_host);
/* y[0:batch] for X (batch x 16, row-major); device pointers */
h2_status h2_mlp_forward(const h2_mlp* m, int batch, const float* X, float* y, hipStream_t stream);
/* gradient (H2_MLP_PARAMS floats, packed like the parameters) and loss (1
 * float) of the mean squared error against target[0:batch]; device pointers */
h2_status h2_mlp_gradient(const h2_mlp* m, int batch, const float* X, const float* target,
                          float* grad, float* loss, hipStream_t stream);
/* one Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected) on a batch */
h2_status h2_mlp_train_step(h2_mlp* m, int batch, const float* X, const float* target, float lr,
                            hipStream_t stream);
/* loss of the last train step's batch (synchronises the device) */
h2_status h2_mlp_last_loss(const h2_mlp* m, float* loss_host);
void h2_mlp_destroy(h2_mlp* m);
/* Training records: while enabled (h2_records_enable(1) also clears), every
 * adaptive h2_build appends, for each sibling pair of each level, the 16
 * features above and log(1 + c), c the columns the pair held when the
 * estimator accepted it (all its columns if it never did).  h2_records_read returns the count and, if
 * the pointers are not NULL, copies count x 16 features and count targets. */
h2_status h2_records_enable(int on);
h2_status h2_records_read(int64_t* count, float* features, float* targets);

/* Launch timing for roofline reporting (no paper counterpart; a measurement
 * aid).  h2_timing_enable(1) clears the totals and starts bracketing every
 * launch of the library's timed kernels by HIP events recorded on the stream
 * the kernel runs on; h2_timing_enable(0) stops.  h2_timing_read waits for
 * the recorded launches of `kernel` (its name without namespace, e.g.
 * "k_svd_block") and returns their number, summed duration (ms) and summed
 * algorithmic work (flops for the SVD: 14 m n^2 + 8 n^3 per m x n matrix, the
 * Golub-Van Loan count of a thin SVD with both factors, independent of the
 * number of Jacobi sweeps).  Unknown names read as zero launches. */
h2_status h2_timing_enable(int on);
h2_status h2_timing_read(const char* kernel, int64_t* launches, double* total_ms, double* work);
/* dst[0:n] = src[0:n] (device FP64 arrays) by a plain grid-stride kernel
 * (k_stream_copy): the reference transfer of known size used to scale
 * hardware byte counters */
h2_status h2_stream_copy(const double* src, double* dst, int64_t n, hipStream_t stream);

const char* h2_status_string(h2_status s);
/* last error message of this thread (for diagnostics) */
const char* h2_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* H2_MI355X_H */
