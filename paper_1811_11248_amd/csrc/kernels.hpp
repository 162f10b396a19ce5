// kernels.hpp -- host-side launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "desc.hpp"

namespace lrsp {

// Fill n doubles with zero (a kernel, so that it can be graph-captured).
void launch_zero(double* p, int64_t n, hipStream_t st);
void launch_zero_i32(int32_t* p, int64_t n, hipStream_t st);
// Copies what the sweeps read of every cluster of a level (nitems items)
// from its panel into its factor store ItemD::S.
void launch_compact(const ItemD* items, int nitems, LevelState ls, hipStream_t st);

// base[off[e]] = val[e] for every e with off[e] >= 0.
void launch_scatter_vals(const double* val, const int64_t* off, int64_t nnz, double* base,
                         hipStream_t st);
void launch_copy_blocks(const CopyD* tasks, int ntasks, hipStream_t st);
// One ScatterD per system (blockIdx.y), max_nnz = largest nnz.
void launch_scatter_vals_multi(const ScatterD* d, int nd, int64_t max_nnz, hipStream_t st);

// One scaled low-rank elimination per item (all items of one colour), one
// workgroup per cluster.
void launch_slre(const ItemD* items, int nitems, int max_m, int max_nseg, LevelState ls, int level,
                 double tol, int tol_mode, int prec, hipStream_t st);
// All colours of a level in one cooperative launch (grid barrier between
// colours); cstart is a device array of ncolours+1 item offsets.
// grid_cap > 0 limits the persistent grid to grid_cap workgroups.  With
// bar == null the launch is cooperative; with a GridBar (zeroed once) it is
// an ordinary launch of at most one workgroup per CU using the bounded
// software barrier, which can be recorded in a graph.
hipError_t launch_slre_level(const ItemD* items, const int32_t* cstart, int ncolours, int max_items,
                             int max_m, int max_nseg, LevelState ls, int level, double tol,
                             int tol_mode, int prec, hipStream_t st, int grid_cap = 0,
                             GridBar* bar = nullptr);
// Workgroups per CU the persistent elimination kernel can hold at this LDS size.
int slre_level_occupancy(int max_m, int max_nseg);
int device_cus();

// Capacities of one colour for the split (several workgroups per cluster) path.
struct SplitDims {
  int max_m, max_nseg, max_pcap, max_acap, max_bcap;
};
constexpr int kSplitMaxDofs = 512;   // LDS limit of the split kernels
constexpr int kSplitMinDofs = 96;    // below this one workgroup per cluster wins
enum SplitStep {
  kSplitOffsets = 0, kSplitGather, kSplitPotrf, kSplitTrsm, kSplitCpqr, kSplitApplyq, kSplitSchur,
  kSplitWriteback, kSplitSteps
};
// Column tiles of the scaling step (G^{-1} [A_sn | A_sw] on MFMA): 32
// columns per workgroup (default) or 16 (twice the workgroups); the results
// are the same bits either way.
constexpr int kTileWide = 0, kTileNarrow = 1;
void launch_split_step(int step, const ItemD* items, int nitems, const SplitDims& d, LevelState ls,
                       int level, double tol, int tol_mode, int prec, hipStream_t st, int tile = kTileWide);

// Dense Cholesky of the top system (lower, in place).
void launch_top_potrf(double* A, int n, int32_t* err, hipStream_t st);

// Substitution sweeps.  Clusters of at least kSweepSplitM DoFs spread their
// near-field products over units of kSweepCols columns (forward) or
// kSweepRows rows (backward); max_acap bounds the near-field width.
constexpr int kSweepSplitM = 128;
constexpr int kSweepCols = 64;
constexpr int kSweepRows = 32;
// Clusters of at most kSweepWaveM DoFs are swept by one wave; levels of such
// clusters run in workgroups of kSweepWaveThreads threads.
constexpr int kSweepWaveM = 32;
constexpr int kSweepWaveThreads = 512;
constexpr int kSweepWaveVix = 64;  // near-field vector indices staged per cluster
constexpr size_t kSweepWaveTableBytes = 64 + 4 * kSweepWaveVix;  // descriptor, indices
constexpr size_t kSweepWaveTableMax = 96 * 1024;
int sweep_units(bool forward, int max_m, int max_acap);
// The items of one colour (one launch, plus one for the units).  shadow
// (non-null): every item is a cluster of kSweepSplitM..kInvMaxDofs DoFs
// whose store holds W (giok 2) or, with no reflector, G^{-1} (giok 1), as
// after the split schedule on a level of such clusters; the product with W
// then runs in one workgroup per 64 rows, writing to shadow (a vector laid
// out like vec), from where the units read it and copy it back (same
// arithmetic as the product in one workgroup).
void launch_fwd(const ItemD* items, int nitems, int max_m, int max_acap, LevelState ls, double* vec,
                hipStream_t st, double* shadow = nullptr);
// shadow (non-null): the same clusters as for launch_fwd; the units write
// their rows to shadow and the product with W^T, one workgroup per 64
// entries, reads it there and writes the vector (same arithmetic).
void launch_bwd(const ItemD* items, int nitems, int max_m, int max_acap, LevelState ls, double* vec,
                hipStream_t st, double* shadow = nullptr);
// A whole level in one persistent launch; [vlo, vlo + vn) is the level's
// range of the vector buffer (vn = 0: unknown).
hipError_t launch_sweep_level(bool forward, const ItemD* items, const int32_t* cstart, int ncolours,
                              int nitems, int max_items, int max_m, int max_acap, LevelState ls, double* vec,
                              hipStream_t st, int grid_cap = 0, GridBar* bar = nullptr, int64_t vlo = 0,
                              int64_t vn = 0);
void launch_top_solve(const double* L, int n, double* y, hipStream_t st);
// Dense top by the blocked MFMA Cholesky of the split kernels (one
// workgroup of 512 threads, n <= kSplitMaxDofs).
void launch_top_potrf_wg(double* A, int n, int32_t* err, hipStream_t st);
// Dense tops of kSplitMaxDofs < n <= kTopMaxDofs unknowns: blocked Cholesky
// over several workgroups (A: n x (n + 64) doubles, ld n; the last 64
// columns are workspace).  A non-positive pivot sets the error words (bits ==
// 0) or the bit kErrNotSPD of *err (bits != 0, a batched system).  With X
// (n x n, ld n) the lower inverse of the factor is formed there as well
// (cleared first); launch_top_solve then applies it when X = A + n (n + 64),
// using the 64 columns after the factor and 64 more after X (A then holds
// n x (2n + 128) doubles) as its workspace.
constexpr int kTopMaxDofs = 4096;
void launch_top_potrf_blocked(double* A, int n, int32_t* err, int bits, hipStream_t st, double* X = nullptr);
// The tops of a batch with 64..kSplitMaxDofs unknowns by the same kernel
// (the others are skipped); max_n: their largest size.
void launch_top_potrf_wg_batched(const TopD* tops, int ntops, int max_n, hipStream_t st);
// Dense tops of a batch, one workgroup per system (n <= kMaxClusterDofs).
void launch_top_potrf_batched(const TopD* tops, int ntops, int max_n, hipStream_t st);
void launch_top_solve_batched(const TopD* tops, int ntops, int max_n, double* vec, hipStream_t st);

void launch_gather(const double* src, const int64_t* idx, double* dst, int64_t n, hipStream_t st);
void launch_scatter(const double* src, const int64_t* idx, double* dst, int64_t n,
                    hipStream_t st);

// PCG building blocks.
void launch_spmv(const int64_t* rowptr, const int32_t* col, const double* val, const double* x,
                 double* y, int64_t n, hipStream_t st);
// out[0] = x . y (deterministic two-stage reduction; partial has kDotBlocks doubles)
constexpr int kDotBlocks = 512;
void launch_dot(const double* x, const double* y, int64_t n, double* partial, double* out,
                hipStream_t st);
// x += (num/den) p ; r -= (num/den) q
void launch_pcg_xr(double* x, double* r, const double* p, const double* q, int64_t n,
                   const double* num, const double* den, hipStream_t st);
// p = z + (num/den) p
void launch_pcg_p(double* p, const double* z, int64_t n, const double* num, const double* den,
                  hipStream_t st);
// y = b - y
void launch_residual(const double* b, double* y, int64_t n, hipStream_t st);
void launch_copy(const double* src, double* dst, int64_t n, hipStream_t st);

// Restarted GMRES building blocks (krylov.hip).  V is column-major with
// leading dimension ldv; part holds kDotBlocks doubles per column.
// out[c] = V(:, c) . w for c < ncol (deterministic two-stage reduction)
void launch_mdot(const double* V, int64_t ldv, int ncol, const double* w, int64_t n, double* part,
                 double* out, hipStream_t st);
// w = V(:, 0:ncol) h, or w -= V(:, 0:ncol) h when sub
void launch_gemv_cols(const double* V, int64_t ldv, int ncol, const double* h, double* w, int64_t n,
                      bool sub, hipStream_t st);
// v = w / sqrt(nrm2[0]) (0 when nrm2[0] == 0)
void launch_normalize(const double* w, double* v, int64_t n, const double* nrm2, hipStream_t st);
// x += z
void launch_add(double* x, const double* z, int64_t n, hipStream_t st);

// Batching form (packed vectors: column c of system i at c*ldv + off[i]).
void launch_spmm(const int64_t* rowptr, const int32_t* col, const double* val, const double* x,
                 double* y, int64_t n, int64_t ldv, int nrhs, hipStream_t st);
void launch_seg_dot(const double* x, const double* y, const int64_t* off, int64_t ldv, int nsys,
                    int nrhs, double* out, hipStream_t st);
void launch_bpcg_xr(double* x, double* r, const double* p, const double* q, const int32_t* rowsys,
                    int64_t ntot, int nsys, int nrhs, const double* rz, const double* pq,
                    const int32_t* active, hipStream_t st);
void launch_bpcg_p(double* p, const double* z, const int32_t* rowsys, int64_t ntot, int nsys,
                   int nrhs, const double* rz_new, const double* rz, const int32_t* active,
                   hipStream_t st);
void launch_bpcg_state(int mode, int np, double rtol, const double* bb, const double* rr, double* rz,
                       const double* rz_new, int32_t* active, int32_t* iters, int32_t* nactive,
                       hipStream_t st);
void launch_zero_multi(const SpanD* d, int nd, int64_t max_n, hipStream_t st);

}  // namespace lrsp
