// batch.hip -- kernels of the batching form outside the elimination: the
// block-diagonal sparse product with up to four right-hand sides, dot
// products per (system, column), the masked PCG updates of all (system,
// column) pairs, and the multi-buffer fill used when a factorization is
// replayed.
//
// Packed vectors: column c of a batch vector holds system i in rows
// off[i] .. off[i+1]-1 and starts at c*ldv; pair index p = c*nsys + i.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "desc.hpp"
#include "devutil.hpp"
#include "kernels.hpp"

namespace lrsp {

namespace {
constexpr int kMaxRhsPass = 4;  // columns per pass of the sparse product
}

__global__ void __launch_bounds__(256) spmm_kernel(const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ x, double* __restrict__ y,
                                                   int64_t n, int64_t ldv, int nrhs) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc[kMaxRhsPass] = {0.0, 0.0, 0.0, 0.0};
    const int64_t e1 = rowptr[i + 1];
    for (int64_t e = rowptr[i]; e < e1; ++e) {
      const double v = val[e];
      const int64_t j = col[e];
#pragma unroll
      for (int r = 0; r < kMaxRhsPass; ++r)
        if (r < nrhs) acc[r] += v * x[r * ldv + j];
    }
#pragma unroll
    for (int r = 0; r < kMaxRhsPass; ++r)
      if (r < nrhs) y[r * ldv + i] = acc[r];
  }
}

void launch_spmm(const int64_t* rowptr, const int32_t* col, const double* val, const double* x,
                 double* y, int64_t n, int64_t ldv, int nrhs, hipStream_t st) {
  if (n <= 0) return;
  const int g = (int)std::min<int64_t>(8192, (n + 255) / 256);
  for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPass) {
    const int nr = std::min(kMaxRhsPass, nrhs - r0);
    hipLaunchKernelGGL(spmm_kernel, dim3(g), dim3(256), 0, st, rowptr, col, val, x + r0 * ldv,
                       y + r0 * ldv, n, ldv, nr);
  }
}

// out[c*nsys + i] = x_i,c . y_i,c (fixed summation order).
__global__ void __launch_bounds__(256) seg_dot_kernel(const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const int64_t* __restrict__ off, int64_t ldv,
                                                      int nsys, double* __restrict__ out) {
  __shared__ double sh[4];
  const int p = blockIdx.x;
  const int c = p / nsys, i = p - c * nsys;
  const int64_t b = off[i], e = off[i + 1];
  const double* xc = x + c * ldv;
  const double* yc = y + c * ldv;
  double s = 0.0;
  for (int64_t j = b + threadIdx.x; j < e; j += 256) s += xc[j] * yc[j];
  s = group_sum<256>(s, sh);
  if (threadIdx.x == 0) out[p] = s;
}

void launch_seg_dot(const double* x, const double* y, const int64_t* off, int64_t ldv, int nsys,
                    int nrhs, double* out, hipStream_t st) {
  if (nsys <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(seg_dot_kernel, dim3(nsys * nrhs), dim3(256), 0, st, x, y, off, ldv, nsys, out);
}

// x += (rz/pq) p, r -= (rz/pq) q on the rows of active pairs.
__global__ void bpcg_xr_kernel(double* __restrict__ x, double* __restrict__ r,
                               const double* __restrict__ p, const double* __restrict__ q,
                               const int32_t* __restrict__ rowsys, int64_t ntot, int nsys, int nrhs,
                               const double* __restrict__ rz, const double* __restrict__ pq,
                               const int32_t* __restrict__ active) {
  const int64_t total = ntot * nrhs;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = idx / ntot, i = idx - c * ntot;
    const int pr = (int)c * nsys + rowsys[i];
    if (!active[pr]) continue;
    const double a = rz[pr] / pq[pr];
    x[idx] += a * p[idx];
    r[idx] -= a * q[idx];
  }
}

// p = z + (rz_new/rz) p on the rows of active pairs.
__global__ void bpcg_p_kernel(double* __restrict__ p, const double* __restrict__ z,
                              const int32_t* __restrict__ rowsys, int64_t ntot, int nsys, int nrhs,
                              const double* __restrict__ rz_new, const double* __restrict__ rz,
                              const int32_t* __restrict__ active) {
  const int64_t total = ntot * nrhs;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = idx / ntot, i = idx - c * ntot;
    const int pr = (int)c * nsys + rowsys[i];
    if (!active[pr]) continue;
    p[idx] = z[idx] + (rz_new[pr] / rz[pr]) * p[idx];
  }
}

static int vec_grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256)); }

void launch_bpcg_xr(double* x, double* r, const double* p, const double* q, const int32_t* rowsys,
                    int64_t ntot, int nsys, int nrhs, const double* rz, const double* pq,
                    const int32_t* active, hipStream_t st) {
  hipLaunchKernelGGL(bpcg_xr_kernel, dim3(vec_grid(ntot * nrhs)), dim3(256), 0, st, x, r, p, q,
                     rowsys, ntot, nsys, nrhs, rz, pq, active);
}

void launch_bpcg_p(double* p, const double* z, const int32_t* rowsys, int64_t ntot, int nsys,
                   int nrhs, const double* rz_new, const double* rz, const int32_t* active,
                   hipStream_t st) {
  hipLaunchKernelGGL(bpcg_p_kernel, dim3(vec_grid(ntot * nrhs)), dim3(256), 0, st, p, z, rowsys,
                     ntot, nsys, nrhs, rz_new, rz, active);
}

// mode 0 (start): active = (bb > 0), iters = 0.  mode 1 (after an update of
// x and r): active pairs count the iteration and stop when
// sqrt(rr) <= rtol*sqrt(bb).  mode 2 (after p was updated): rz = rz_new on
// active pairs.  In every mode *nactive receives the number of active pairs.
__global__ void __launch_bounds__(1024) bpcg_state_kernel(int mode, int np, double rtol,
                                                          const double* __restrict__ bb,
                                                          const double* __restrict__ rr,
                                                          double* __restrict__ rz,
                                                          const double* __restrict__ rz_new,
                                                          int32_t* __restrict__ active,
                                                          int32_t* __restrict__ iters,
                                                          int32_t* __restrict__ nactive) {
  __shared__ double sh[16];
  int cnt = 0;
  for (int p = threadIdx.x; p < np; p += 1024) {
    int act = active[p];
    if (mode == 0) {
      act = bb[p] > 0.0 ? 1 : 0;
      iters[p] = 0;
    } else if (mode == 1) {
      if (act) {
        iters[p] += 1;
        if (sqrt(rr[p]) <= rtol * sqrt(bb[p])) act = 0;
      }
    } else if (act) {
      rz[p] = rz_new[p];
    }
    active[p] = act;
    cnt += act;
  }
  double c = (double)cnt;
  c = group_sum<1024>(c, sh);
  if (threadIdx.x == 0) *nactive = (int32_t)c;
}

void launch_bpcg_state(int mode, int np, double rtol, const double* bb, const double* rr, double* rz,
                       const double* rz_new, int32_t* active, int32_t* iters, int32_t* nactive,
                       hipStream_t st) {
  hipLaunchKernelGGL(bpcg_state_kernel, dim3(1), dim3(1024), 0, st, mode, np, rtol, bb, rr, rz,
                     rz_new, active, iters, nactive);
}

__global__ void zero_multi_kernel(const SpanD* __restrict__ d) {
  const SpanD t = d[blockIdx.y];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < t.n;
       e += (int64_t)gridDim.x * blockDim.x)
    t.p[e] = 0.0;
}

void launch_zero_multi(const SpanD* d, int nd, int64_t max_n, hipStream_t st) {
  if (nd <= 0 || max_n <= 0) return;
  const int gx = (int)std::min<int64_t>(64, (max_n + 255) / 256);
  hipLaunchKernelGGL(zero_multi_kernel, dim3(gx, nd), dim3(256), 0, st, d);
}

}  // namespace lrsp
