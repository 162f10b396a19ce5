// krylov.hip -- kernels of the restarted GMRES wrapper (lrsp_gmres).
//
// The Arnoldi basis V (n x (restart+1), column-major, leading dimension n)
// is orthogonalised by classical Gram-Schmidt applied twice: each pass is
// one block of dot products h = V(:, 0:j)^T w and one update
// w -= V(:, 0:j) h.  Both stream V once per pass at full width (every
// column read with coalesced loads), which is what makes the pass
// HBM-bound rather than latency-bound as column-by-column modified
// Gram-Schmidt would be.  Reductions use a fixed partition of the rows
// (kDotBlocks workgroups) and a fixed summation order, so results do not
// vary from run to run.
#include <hip/hip_runtime.h>

#include "devutil.hpp"
#include "kernels.hpp"

namespace lrsp {

namespace {

constexpr int kColsPerPass = 8;  // columns of V per workgroup of the dot kernel

inline int grid_rows(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (int)(g < 2048 ? (g < 1 ? 1 : g) : 2048);
}

}  // namespace

// part[c * kDotBlocks + blk] = sum over the rows of workgroup blk of
// V[i + c ldv] w[i], for the kColsPerPass columns c of blockIdx.y.
__global__ void __launch_bounds__(256) mdot_partial_kernel(const double* __restrict__ V, int64_t ldv,
                                                           int ncol, const double* __restrict__ w,
                                                           int64_t n, double* __restrict__ part) {
  __shared__ double sh[4][kColsPerPass];
  const int c0 = blockIdx.y * kColsPerPass;
  const int nc = min(kColsPerPass, ncol - c0);
  double acc[kColsPerPass];
#pragma unroll
  for (int c = 0; c < kColsPerPass; ++c) acc[c] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = w[i];
#pragma unroll
    for (int c = 0; c < kColsPerPass; ++c)
      if (c < nc) acc[c] += V[i + (size_t)ldv * (c0 + c)] * wi;
  }
#pragma unroll
  for (int c = 0; c < kColsPerPass; ++c) {
    const double s = wave_sum(acc[c]);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][c] = s;
  }
  __syncthreads();
  if (threadIdx.x < nc) {
    const int c = threadIdx.x;
    part[(size_t)(c0 + c) * kDotBlocks + blockIdx.x] = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
  }
}

// out[c] = sum of part[c * kDotBlocks + 0 .. kDotBlocks), one workgroup per c.
__global__ void __launch_bounds__(256) mdot_final_kernel(const double* __restrict__ part,
                                                         double* __restrict__ out) {
  __shared__ double sh[4];
  const double* p = part + (size_t)blockIdx.x * kDotBlocks;
  double s = 0.0;
  for (int i = threadIdx.x; i < kDotBlocks; i += blockDim.x) s += p[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

void launch_mdot(const double* V, int64_t ldv, int ncol, const double* w, int64_t n, double* part,
                 double* out, hipStream_t st) {
  if (ncol <= 0) return;
  hipLaunchKernelGGL(mdot_partial_kernel, dim3(kDotBlocks, (ncol + kColsPerPass - 1) / kColsPerPass),
                     dim3(256), 0, st, V, ldv, ncol, w, n, part);
  hipLaunchKernelGGL(mdot_final_kernel, dim3(ncol), dim3(256), 0, st, part, out);
}

// sub = 0: w = V(:, 0:ncol) h;  sub = 1: w -= V(:, 0:ncol) h.
__global__ void __launch_bounds__(256) gemv_cols_kernel(const double* __restrict__ V, int64_t ldv,
                                                        int ncol, const double* __restrict__ h,
                                                        double* __restrict__ w, int64_t n, int sub) {
  extern __shared__ double hs[];
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) hs[c] = h[c];
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < ncol; ++c) s += V[i + (size_t)ldv * c] * hs[c];
    w[i] = sub ? w[i] - s : s;
  }
}

void launch_gemv_cols(const double* V, int64_t ldv, int ncol, const double* h, double* w, int64_t n,
                      bool sub, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gemv_cols_kernel, dim3(grid_rows(n)), dim3(256), (size_t)(ncol > 0 ? ncol : 1) * 8, st,
                     V, ldv, ncol, h, w, n, sub ? 1 : 0);
}

// v = w / sqrt(nrm2[0]) (v = 0 when nrm2[0] is 0: a breakdown, which the
// host sees in the same read-back and stops on).
__global__ void normalize_kernel(const double* __restrict__ w, double* __restrict__ v, int64_t n,
                                 const double* __restrict__ nrm2) {
  const double s = nrm2[0] > 0.0 ? 1.0 / sqrt(nrm2[0]) : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = w[i] * s;
}

void launch_normalize(const double* w, double* v, int64_t n, const double* nrm2, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(normalize_kernel, dim3(grid_rows(n)), dim3(256), 0, st, w, v, n, nrm2);
}

__global__ void axpy1_kernel(double* __restrict__ x, const double* __restrict__ z, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] += z[i];
}

void launch_add(double* x, const double* z, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpy1_kernel, dim3(grid_rows(n)), dim3(256), 0, st, x, z, n);
}

}  // namespace lrsp
