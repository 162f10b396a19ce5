/*
 * lrsp.h -- C interface of the MI355X deferred-compression hierarchical solver.
 *
 * The solver computes an approximate factorization of a sparse symmetric
 * positive definite matrix A over a cluster tree (Algorithm 1 of Chen,
 * Cambier, Boman, Rajamanickam, Tuminaro, Darve, "A Robust Hierarchical
 * Solver for Ill-conditioned Systems with Applications to Ice Sheet
 * Modeling") and applies it as a preconditioner (Algorithm 2) inside PCG.
 * The problem statement is "solve Ax = b for sparse SPD A using a clustering
 * of the unknowns" (section "Improved LoRaSp Solver").
 *
 * Conventions
 *   - No C++ exception crosses this interface; every call returns an
 *     lrsp_status.  lrsp_status_str() gives a message.
 *   - "device" pointers are HIP device memory of the current device;
 *     "host" pointers are ordinary host memory.
 *   - Every call enqueues its GPU work on the hip stream passed as
 *     `stream` (a hipStream_t; NULL = the null stream).  lrsp_factor
 *     synchronises that stream once per tree level (the next level's
 *     sizes depend on the compression ranks); lrsp_apply does not
 *     synchronise; lrsp_pcg synchronises once per iteration to test
 *     convergence.
 *   - Handles (lrsp_tree, lrsp_factorization) are not thread-safe; distinct
 *     handles may be used from distinct threads.
 *   - Floating point is IEEE double unless an option says otherwise.
 */
#ifndef LRSP_H
#define LRSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LRSP_OK = 0,
  LRSP_ERR_ARG = 1,       /* invalid argument (sizes, null pointers, tree/matrix mismatch) */
  LRSP_ERR_NOT_SPD = 2,   /* a diagonal-block Cholesky met a pivot <= 0 or NaN */
  LRSP_ERR_HIP = 3,       /* a HIP runtime call failed */
  LRSP_ERR_OOM = 4,       /* device allocation failed */
  LRSP_ERR_NO_CONV = 5,   /* PCG reached maxit; x holds the last iterate */
  LRSP_ERR_INTERNAL = 6   /* a device-side capacity or consistency check failed */
} lrsp_status;

/* Structured extruded grid: nx*ny vertical columns of nz layers with ncomp
 * unknowns per node.  Global DoF id = c + ncomp*(z + nz*(x + nx*y)), so a
 * vertical column is a contiguous range of nz*ncomp ids. */
typedef struct {
  int32_t nx, ny, nz, ncomp;
} lrsp_grid;

/* Sparse SPD matrix in CSR with the FULL symmetric pattern and sorted
 * column indices.  rowptr/col/val are DEVICE pointers.  h_rowptr/h_col are
 * optional HOST copies of the pattern used by the symbolic analysis; when
 * NULL the library copies the pattern from the device.  pattern_id: 0, or a
 * nonzero number the caller gives to this exact pattern.  Precondition: one
 * id is never given to two different patterns.  A factorization whose tree
 * last analysed a pattern of the same nonzero id reuses that analysis after
 * comparing the row pointers in full and the column indices at up to 4096
 * evenly spaced entries instead of all of them (id 0: every entry is
 * compared).  The caller owns all arrays and keeps them alive for the
 * duration of a call. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* rowptr;
  const int32_t* col;
  const double* val;
  const int64_t* h_rowptr;
  const int32_t* h_col;
  uint64_t pattern_id;
} lrsp_csr;

typedef struct lrsp_tree lrsp_tree;
typedef struct lrsp_factorization lrsp_factorization;
typedef struct lrsp_batch lrsp_batch;

/* Factorization options.  Zero-initialise, then set fields. */
typedef struct {
  int32_t tol_mode;   /* 0: relative, rank k = first j with R_jj <= tol*R_00;
                         1: absolute, R_jj <= tol */
  int32_t gemm_prec;  /* Schur-update product: 0 fp64, 1 fp32 inputs with fp32
                         accumulation, 2 bf16 inputs with fp32 accumulation;
                         the result is added to the fp64 matrix */
  int32_t rank_mode;  /* 0: worst-case rank capacities; 1: capacities from
                         learned ranks (see "learned ranks" below) */
  int32_t exec_mode;  /* kernel schedule (results agree to rounding): 0 auto;
                         1 one workgroup per cluster, one launch per colour
                         (the substitution sweeps of lrsp_apply too);
                         2 one workgroup per cluster, one cooperative launch per
                         level; 3 several workgroups per cluster for clusters of
                         96..512 DoFs, else as 2 */
  const float* mlp_weights; /* rank_mode 1: host pointer to the packed MLP
                               parameters (lrsp_mlp_nparams() floats) */
  int32_t autotune;   /* exec_mode 0: 1 = time the candidate schedules of every
                         level now and record the fastest in the autotuner
                         table; 0 = use the table's entry for the level's
                         shape if there is one, else the default schedule */
  int32_t top_dense_threshold; /* 0: the recursion stops at the first level
                         whose cluster graph is complete or has one cluster;
                         T > 0: also at the first level whose unknowns number
                         at most T (Algorithm 1: "small enough" to factor
                         directly), which is then factored by the dense top
                         Cholesky.  0 <= T <= 768 (ERR_ARG otherwise). */
  int32_t scheme;     /* 0: deferred compression (the scaled low-rank
                         elimination); 1: without it, the scheme the paper
                         compares against (section "Deferred-compression
                         Scheme", Eqs. offdiag and sc_old): the unscaled
                         far-field block is compressed, the cluster rotated by
                         U^T on both sides and its fine part eliminated by
                         Cholesky; the coarse unknowns keep that Schur
                         complement as their diagonal block.  Scheme 1 runs
                         one workgroup per cluster (exec_mode 1 or 2; auto
                         and 3 become 2) with the sweeps one launch per
                         colour, fp64 or reduced Schur products; not with
                         rank_mode 1 or the batching form (ERR_ARG). */
  int32_t reserved32b;
  int64_t reserved[4];
} lrsp_opts;

/* ---- cluster tree ------------------------------------------------------
 * Extruded partitioning (section "Extruded Partitioning for Ice Sheets"):
 * the horizontal box [0,nx)x[0,ny) is bisected L times, L the smallest
 * integer with leaf_size*2^L >= N; each split halves the longer side (ties:
 * x) at lo+len/2, left child first; every vertical column stays in one
 * cluster.  Level-l cluster c is the parent of level-(l-1) clusters 2c, 2c+1.
 * ERR_ARG if leaf_size < nz*ncomp or a split would have to cut a column.
 * The tree is allocated by the library; free it with lrsp_tree_free. */
lrsp_status lrsp_tree_build(const lrsp_grid* g, int32_t leaf_size, lrsp_tree** out);

/* Extruded partitioning of an unstructured extruded mesh (same section: one
 * layer partitioned by a graph partitioner, the parts extruded through all
 * layers).  The layer is the graph of ncols vertical columns: adj_ptr
 * [ncols+1] and adj (host arrays, CSR, symmetric, without self loops; the
 * caller keeps ownership).  Column v holds global DoFs
 * c + ncomp*(z + nz*v).  The column set is bisected L times (L as above) by
 * level-structure bisection, which uses the graph alone: a breadth-first
 * search from the smallest column finds the column farthest from it (ties:
 * smallest id), a breadth-first search from that column (neighbours in
 * increasing id, restarting at the smallest unvisited column when a
 * component is exhausted) orders the set, and the first floor(|S|/2)
 * columns of that order form the left child.  Children left, right; a
 * leaf's DoFs sorted by global id.  ERR_ARG for leaf_size < nz*ncomp, an
 * index out of range or a self loop, or a part of one column that would
 * have to be split. */
lrsp_status lrsp_tree_build_graph(int64_t ncols, const int64_t* adj_ptr, const int32_t* adj, int32_t nz,
                                  int32_t ncomp, int32_t leaf_size, lrsp_tree** out);
lrsp_status lrsp_tree_free(lrsp_tree* t);

/* Read-only view of the level-0 clustering.  The arrays are owned by the
 * tree and stay valid until it is freed.  perm lists the global DoFs in
 * cluster order; cluster c holds perm[leaf_ptr[c] .. leaf_ptr[c+1]). */
typedef struct {
  int32_t nlevels;     /* L */
  int32_t nleaves;     /* 2^L */
  int64_t n;
  const int64_t* perm;
  const int64_t* leaf_ptr;
} lrsp_tree_view;
lrsp_status lrsp_tree_export(const lrsp_tree* t, lrsp_tree_view* v);

/* ---- analysis reuse ------------------------------------------------------
 * A tree caches the symbolic analysis of the last matrix pattern factored
 * with it (level graphs, colouring, fill, block layout, descriptors) together
 * with the device workspace of each level.  lrsp_factor reuses a level when
 * the pattern and the sizes of its clusters (the ranks of the level below)
 * are unchanged, and lrsp_factor_free returns the workspace to the tree.
 * A factor alive at the same time as another one from the same tree simply
 * allocates its own workspace.  Results do not depend on reuse. */

/* ---- factorization -----------------------------------------------------
 * Algorithm 1 over the tree: at each level every cluster s, in (colour,
 * index) order of a greedy distance-2 colouring of the level's cluster graph,
 * undergoes the scaled low-rank elimination W_s = P_s G_s E_s S_s
 * (Eqs. scaling, sparse, elim, perm): Cholesky of A_ss, scaling of its block
 * row by G_s^{-1}, column-pivoted QR compression of the scaled far-field
 * block to the rank set by tol, rotation, elimination of the fine DoFs with
 * the Schur update X_nn = A_nn - F^T F.  Recursion stops at the first level
 * whose cluster graph is complete (or has one cluster) with a dense Cholesky.
 * A: device CSR (see lrsp_csr); tol >= 0; opts may be NULL (defaults).
 * On success *F receives a new factor owning its device memory.
 * ERR_NOT_SPD: *F = NULL; lrsp_last_error_info() names level and cluster. */
lrsp_status lrsp_factor(const lrsp_csr* A, lrsp_tree* T, double tol, const lrsp_opts* opts,
                        void* stream, lrsp_factorization** F);
lrsp_status lrsp_factor_free(lrsp_factorization* F);

/* x = M^{-1} b, M the factored approximation of A (Algorithm 2: forward
 * substitution y <- W_i y, coarse solve, backward x <- W_i^T x).
 * b, x: device arrays of n*nrhs doubles, column-major; b == x allowed. */
lrsp_status lrsp_apply(const lrsp_factorization* F, const double* b, double* x, int32_t nrhs,
                       void* stream);

/* Preconditioned conjugate gradients with M = the factor, x0 = 0, stopping
 * when the recursive residual satisfies ||r||_2 <= rtol*||b||_2 (per column)
 * or after maxit iterations.  This is the Krylov solve of the problem
 * statement A x = b (section "Improved LoRaSp Solver") with the factor as
 * preconditioner; the paper wraps the factor in right-preconditioned
 * GMRES(200) instead (section "Numerical Results", test problems; see
 * lrsp_gmres), and PCG is used here because the factor is symmetric
 * positive definite by construction.  b, x: device, n*nrhs column-major.
 * iters[nrhs], relres[nrhs]: host outputs (iteration count = number of
 * matrix-vector products; relres = TRUE ||b - A x||_2/||b||_2).
 * ERR_NO_CONV if some column did not converge (x is still the last iterate). */
lrsp_status lrsp_pcg(const lrsp_csr* A, const lrsp_factorization* F, const double* b, double* x,
                     int32_t nrhs, double rtol, int32_t maxit, int32_t* iters, double* relres,
                     void* stream);

/* Right-preconditioned restarted GMRES(restart) with the factor as
 * preconditioner (M^{-1} applied as in lrsp_apply), as the paper solves its
 * systems: GMRES(200), tolerance 1e-12, at most 1000 iterations (section
 * "Numerical Results", test problems).  x0 = 0; each cycle builds an
 * orthonormal basis of the Krylov space of A M^{-1} (classical Gram-Schmidt
 * applied twice), reduces the Hessenberg matrix by Givens rotations and
 * stops when the least-squares residual satisfies ||r||_2 <= rtol*||b||_2;
 * x = x0 + M^{-1} V y.  b, x: device, n*nrhs column-major, solved column
 * after column.  iters[nrhs]: products with A M^{-1} over all cycles;
 * relres[nrhs]: TRUE ||b - A x||_2/||b||_2.  The basis takes n*(restart+3)
 * doubles of device memory during the call.  ERR_NO_CONV when a column
 * reached maxit (x is the last iterate); ERR_ARG for restart outside
 * 1..4096. */
lrsp_status lrsp_gmres(const lrsp_csr* A, const lrsp_factorization* F, const double* b, double* x,
                       int32_t nrhs, int32_t restart, double rtol, int32_t maxit, int32_t* iters,
                       double* relres, void* stream);

/* lrsp_pcg without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the same iteration, results and errors as lrsp_pcg, with its
 * work vectors (4 n + 528 doubles) in a static device array of the library
 * instead of memory held by F.  Limit: n <= LRSP_PCG_NOALLOC_MAX_N, else
 * ERR_ARG and nothing is launched.  The array is one per GPU, is held from
 * the loading of the library until the process ends, and keeps what the last
 * call left in it (every call initialises what it reads); calls that overlap
 * on one GPU (other threads, other streams) race on it and must not be made.
 * The preconditioner application inside allocates nothing either: it uses
 * the level vectors that F owns. */
#define LRSP_PCG_NOALLOC_MAX_N 1048576
lrsp_status lrsp_pcg_noalloc(const lrsp_csr* A, const lrsp_factorization* F, const double* b,
                             double* x, int32_t nrhs, double rtol, int32_t maxit, int32_t* iters,
                             double* relres, void* stream);

/* ---- introspection -------------------------------------------------------*/
typedef struct {
  int32_t nlevels;       /* levels eliminated before the dense top */
  int32_t top_n;         /* size of the dense top system */
  int32_t top_clusters;
  int32_t reserved;
  double flops[6];       /* algorithmic flops: potrf, trsm, cpqr, applyq, schur, top */
  double bytes_factor;   /* bytes of the stored factor */
  double ms_levels;      /* wall time of lrsp_factor (host clock, ms) */
  int64_t peak_bytes;    /* device bytes held while the factorization ran:
                            the factor, the tree's cached level workspaces
                            and the panel arena */
  double ms_analysis;    /* host time spent on symbolic analysis and setup
                            (zero for levels whose analysis was reused) */
  int32_t levels_reused; /* levels whose analysis and workspace came from the
                            tree's cache (same pattern, same ranks below) */
  int32_t reserved2;
  /* rank_mode 1 (zero otherwise): */
  double rank_bytes;          /* bytes of coarse blocks and panels allocated
                                 from the predicted rank capacities */
  double rank_bytes_worst;    /* the same with worst-case capacities min(m, b) */
  int32_t rank_checks_passed; /* clusters whose rank k <= the predicted k_hat */
  int32_t rank_checks_failed; /* clusters whose QR went on past k_hat */
  /* any rank_mode: a level the tree's cache held is sized from the ranks it
   * found before (k + max(2, k/4)); a rank that reaches such a capacity, or
   * a predicted one, makes the level run again with more room: */
  int32_t rank_redo_levels;   /* levels run again because a rank reached
                                 its capacity (each level counted once) */
  int32_t rank_reruns;        /* runs of levels after the first, in all */
} lrsp_info;
lrsp_status lrsp_factor_info(const lrsp_factorization* F, lrsp_info* info);

/* Per-level schedule and ranks (host arrays owned by F, valid until freed):
 * nclusters, sizes[c] (DoFs at level start), colour[c], order[i] (the i-th
 * processed cluster), ranks[c] (coarse DoFs kept), and the level graph in
 * CSR form (adj_ptr[nclusters+1], adj[]); near[c] and far[c]: the columns
 * of cluster c's near- and far-field blocks when it was eliminated (a and
 * b, structurally nonzero columns only).  level == nlevels describes the
 * dense top (colour/order/ranks/near/far NULL). */
typedef struct {
  int32_t nclusters;
  int32_t ncolours;
  const int32_t* sizes;
  const int32_t* colour;
  const int32_t* order;
  const int32_t* ranks;
  const int32_t* adj_ptr;
  const int32_t* adj;
  const int32_t* near;
  const int32_t* far;
} lrsp_level_view;
lrsp_status lrsp_factor_level(const lrsp_factorization* F, int32_t level, lrsp_level_view* v);

/* Per-level measurements for scaling studies (Complexity Analysis: O(N)
 * work and memory with ranks bounded per level; the paper's per-level
 * breakdown of factor and solve time).  level == nlevels is the dense top.
 * flops: algorithmic flops of the level (the lrsp_info model); sweep_bytes:
 * factor and vector bytes one sweep of the level reads and writes; dofs,
 * coarse: unknowns at level start and kept after it; factor_ms: GPU time
 * from the start of the level's work to the start of the next level's
 * (top: its Cholesky), and solve_ms: GPU time of the level's forward plus
 * backward sweeps summed over the `applies` preconditioner applications
 * (lrsp_apply, and those inside lrsp_pcg / lrsp_gmres) -- both 0 unless
 * timing (lrsp_timing_enable) was on during lrsp_factor and during the
 * applications.  factor_bytes: device bytes of the level's part of the
 * factor (the factor stores the sweeps read and the vector indices);
 * held_bytes: all device bytes the level holds (its workspaces too), the
 * dense top's for level == nlevels; of those, work_bytes: the level-start
 * blocks (diagonal blocks and fine halves), coarse_bytes: the coarse halves
 * (sized by the rank capacities); panel_bytes: the level's share of the
 * panel workspace while it is eliminated (held in the tree's arena, not in
 * held_bytes).  Synchronises the device. */
typedef struct {
  double flops;
  double sweep_bytes;
  double factor_ms;
  double solve_ms;
  int64_t applies;
  int64_t dofs;
  int64_t coarse;
  int32_t nclusters;
  int32_t reserved;
  int64_t factor_bytes;
  int64_t held_bytes;
  int64_t work_bytes;
  int64_t coarse_bytes;
  int64_t panel_bytes;
} lrsp_level_stats;
lrsp_status lrsp_factor_level_stats(const lrsp_factorization* F, int32_t level, lrsp_level_stats* out);

/* ---- learned ranks ---------------------------------------------------------
 * rank_mode 1: before a level is eliminated, every cluster gets 12 features:
 * log2(1+m); log2(1+b), b the level-start size of its far field when it is
 * processed (from the symbolic elimination); from its level-start coupling
 * with its neighbours (Jacobi-scaled, sketched with 8 Gaussian columns drawn
 * from Philox4x32-10) log10 of the Frobenius norm and the 8 sketch singular
 * values over that norm; the fraction of its neighbours processed before it.
 * A 12-64-64-1 ReLU network (fp32) predicts the rank k_hat; the rank
 * capacities, and with them the coarse blocks and panels, are sized
 * ceil(2*k_hat + 4) instead of the worst case min(m, b).  The QR itself
 * is unchanged (it stops at the rank the tolerance sets, so ranks and factor
 * equal rank_mode 0); when a rank reaches a capacity below its worst case
 * the level runs again from its assembled input, those clusters with the
 * worst case and the others with their predicted capacities (at most twice;
 * then every capacity of the level is the worst case).  Parameter vector (fp32, lrsp_mlp_nparams()):
 * mu[12] isd[12] W1[64][12] b1[64] W2[64][64] b2[64] w3[64] b3; the input is
 * (x - mu)*isd.  All arrays of the calls below are device memory. */
int32_t lrsp_mlp_nparams(void);
/* Input statistics of X [n][12] (mu, isd), b3 = mean(t), He-normal weights
 * from Philox4x32-10 with the given seed, zero biases. */
lrsp_status lrsp_mlp_init(float* params, const float* X, const float* t, int64_t n, uint64_t seed,
                          void* stream);
/* Loss 0.5*mean((y - t)^2) (*loss, device, may be NULL) and its gradient
 * grad[nparams] by backpropagation (zero for mu, isd). */
lrsp_status lrsp_mlp_loss_grad(const float* params, const float* X, const float* t, int64_t n,
                               float* grad, float* loss, void* stream);
/* steps full-batch Adam steps (beta 0.9, 0.999) with rate lr; loss_trace
 * [steps] (device, may be NULL) receives the loss before each step. */
lrsp_status lrsp_mlp_train(float* params, const float* X, const float* t, int64_t n, int32_t steps,
                           float lr, float* loss_trace, void* stream);
lrsp_status lrsp_mlp_predict(const float* params, const float* X, int64_t n, float* y, void* stream);
/* Features (host [M][12], fp64) and predicted ranks (host [M]) of one
 * level of a factor computed with rank_mode 1 (either may be NULL). */
lrsp_status lrsp_factor_rank_features(const lrsp_factorization* F, int32_t level, double* feat,
                                      float* pred);

/* ---- batching form -------------------------------------------------------
 * nsys independent systems, each with its own matrix and tree, factored
 * together.  At every tree level the clusters of all systems that are still
 * being eliminated form one work list ordered by colour (clusters of
 * different systems never interact), and one persistent launch eliminates
 * the whole level; systems reach their dense top at their own level, and
 * all tops are factored by one launch.  Each system's factor is the one
 * lrsp_factor computes for it with exec_mode 2 and the same options.
 *
 * Packed vectors: system i occupies rows off_i .. off_i + n_i - 1 with
 * off_i = n_0 + ... + n_{i-1}; ntot = n_0 + ... + n_{nsys-1}; a block of
 * nrhs vectors is ntot x nrhs, column-major, on the device.
 *
 * A[nsys], T[nsys]: as for lrsp_factor (A[i].h_rowptr / h_col recommended).
 * status[nsys]: optional host output, LRSP_OK or LRSP_ERR_NOT_SPD per system.
 * Returns LRSP_ERR_NOT_SPD when some system met a non-positive pivot; *F is
 * then still returned (the other systems' factors are valid).  Any other
 * error leaves *F = NULL.  The trees must outlive the batch. */
lrsp_status lrsp_factor_batched(int32_t nsys, const lrsp_csr* A, lrsp_tree* const* T, double tol,
                                const lrsp_opts* opts, void* stream, lrsp_batch** F,
                                int32_t* status);

/* Numeric refactorization with new values of the same patterns (A[i].val
 * may point to new arrays).  The numeric phase that lrsp_factor_batched
 * recorded (buffer clears, assembly, one elimination launch per level, the
 * tops) is replayed as one captured HIP graph, with no host synchronisation
 * between levels; the ranks are then read back once and compared with the
 * recorded ones.  If some rank differs, the batch is factored again from
 * scratch (lrsp_batch_info counts these fallbacks).  Results equal those of
 * a fresh lrsp_factor_batched. */
lrsp_status lrsp_refactor_batched(lrsp_batch* F, const lrsp_csr* A, void* stream, int32_t* status);
lrsp_status lrsp_batch_free(lrsp_batch* F);

/* x = M^{-1} b for every system (packed, nrhs columns; b == x allowed). */
lrsp_status lrsp_apply_batched(lrsp_batch* F, const double* b, double* x, int32_t nrhs,
                               void* stream);

/* PCG on every (system, column) pair at once: one sparse product with all
 * columns, dot products per pair, updates masked per pair; a pair stops at
 * ||r||_2 <= rtol*||b||_2 while the others go on.  The body of an iteration
 * runs as two captured HIP graphs (before and after the convergence test,
 * which reads one integer).  A: the nsys matrices factored in F.
 * iters, relres: host arrays of nrhs*nsys entries, index c*nsys + i (true
 * relative residual).  ERR_NO_CONV if some pair did not converge. */
lrsp_status lrsp_pcg_batched(const lrsp_csr* A, lrsp_batch* F, const double* b, double* x,
                             int32_t nrhs, double rtol, int32_t maxit, int32_t* iters,
                             double* relres, void* stream);

typedef struct {
  int32_t nsys;
  int32_t nlevels;          /* levels with eliminations (over all systems) */
  int64_t ntot;
  double flops[6];          /* as lrsp_info, summed over systems */
  double ms_factor;         /* host wall time of the last (re)factorization */
  double ms_analysis;       /* host time of planning and setup (first factorization) */
  int64_t peak_bytes;       /* device bytes held by the batch */
  int32_t graph_factor;     /* 1: the last refactorization ran as a graph */
  int32_t graph_pcg;        /* 1: the last batched PCG ran its iterations as graphs */
  int32_t coop_in_graph;    /* always 0: graphs hold ordinary launches whose
                               persistent kernels use a bounded software grid
                               barrier (one workgroup per CU) */
  int32_t refactor_fallbacks;
  int32_t tuned_levels;     /* levels timed by the autotuner in the first factorization */
  int32_t graph_timeouts;   /* graph runs redone eagerly because a grid barrier gave up */
  int32_t sched[16];        /* schedule of levels 0..15 (0 persistent, 1 per colour, 2 split) */
  int32_t grid_cap[16];     /* persistent grid cap of levels 0..15 (0 = full occupancy) */
  int32_t tile[16];         /* split schedule: column tile of the scaling step of
                               levels 0..15 (0: 32 columns per workgroup, 1: 16) */
} lrsp_batch_info;
lrsp_status lrsp_batch_info_get(const lrsp_batch* F, lrsp_batch_info* info);

/* Schedule and ranks of one system of the batch, as lrsp_factor_level
 * (level == the system's number of levels describes its dense top). */
lrsp_status lrsp_batch_level(const lrsp_batch* F, int32_t sys, int32_t level, lrsp_level_view* v);
lrsp_status lrsp_batch_system_levels(const lrsp_batch* F, int32_t sys, int32_t* nlevels);

/* ---- autotuner table -----------------------------------------------------
 * Schedules and tile shapes chosen by timing (opts.autotune = 1): for every
 * level the batch times one persistent launch (full grid and one workgroup
 * per CU), one launch per colour, and the split schedule with either column
 * tile of its scaling step, and keeps the fastest; keyed by level shape,
 * shared by all factorizations of the process; saved and loaded as JSON
 * ({"key", "sched", "grid_cap", "tile", "ms"} per entry). */
lrsp_status lrsp_autotune_save(const char* path);
lrsp_status lrsp_autotune_load(const char* path);
lrsp_status lrsp_autotune_clear(void);
int32_t lrsp_autotune_entries(void);

/* ---- measurement ---------------------------------------------------------
 * When timing is on, the library records a pair of HIP events on the call's
 * stream around every launch of the kernel families below and accumulates,
 * per family, the launch count, the summed event durations and the
 * algorithmic work of those launches (flops of the factorization model:
 * POTRF m^3/3, TRSM m^2(a+b), CPQR and U^T rotation 4(m-j)(b-j), 4(m-j)a per
 * reflector, Schur a(a+1)(m-k); bytes of the sweeps: every stored factor
 * entry read once plus the vector entries read and written).
 * Families: 0 = all cluster-elimination launches, 1 = forward sweep,
 * 2 = backward sweep, 3..9 = the split elimination kernels (3 segment
 * offsets + gather [bytes], 4 Cholesky, 5 triangular scaling, 6 pivoted
 * QR, 7 U^T rotation, 8 Schur update, 9 write-back [bytes]), 10 = the
 * one-workgroup-per-cluster elimination kernel, 11 = the sparse products
 * A p of the PCG iterations [bytes: 12 nnz + 8 (n+1) + 16 n each].
 * lrsp_timing_read synchronises the device. */
typedef struct {
  int64_t launches;
  double total_ms;
  double flops;
  double bytes;
} lrsp_timing;
lrsp_status lrsp_timing_enable(int32_t on);
/* Families that record events while timing is on (bit f = family f; all by
 * default): fewer events, less disturbance of the timed work. */
lrsp_status lrsp_timing_families(uint32_t mask);
lrsp_status lrsp_timing_reset(void);
lrsp_status lrsp_timing_read(int32_t family, lrsp_timing* out);

/* Message of the last failing call on this thread (static storage). */
const char* lrsp_last_error_info(void);
const char* lrsp_status_str(lrsp_status s);

#ifdef __cplusplus
}
#endif
#endif /* LRSP_H */
