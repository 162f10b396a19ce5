// learned.hip -- kernels of the learned-rank form.
//
//   rank_features   per cluster, at the start of a level: the Jacobi-scaled
//                   coupling B = D_s^{-1/2} A_{s,n(s)} D_n^{-1/2}, its sketch
//                   Y = B Omega (Omega Gaussian from Philox4x32-10), the
//                   singular values of Y from the 8x8 Gram matrix (cyclic
//                   Jacobi), and the 12 features
//                   [log2(1+m), log2(1+b), log10|B|_F, sigma/|B|_F, e]
//                   (b: far-field size when s is processed, e: fraction of
//                   its neighbours processed before it; both symbolic)
//   mlp_predict     12 -> 64 -> 64 -> 1 ReLU network, one thread per sample
//   mlp_grad        loss 0.5 mean (y-t)^2 and its gradient by backpropagation,
//                   64 samples per workgroup, per-workgroup partial sums
//   mlp_reduce      partial sums over workgroups in a fixed order
//   mlp_adam        Adam update of the trained parameters
//   mlp_init        input statistics and He-normal initial weights (Philox)
//
// Parameter vector (fp32): mu[12] isd[12] W1[64][12] b1[64] W2[64][64] b2[64]
// w3[64] b3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "desc.hpp"
#include "devutil.hpp"
#include "learned.hpp"

namespace lrsp {

namespace {

constexpr int kF = kMlpFeatures, kH = kMlpHidden;
constexpr int oMu = 0, oIsd = kF, oW1 = 2 * kF, oB1 = oW1 + kH * kF, oW2 = oB1 + kH,
              oB2 = oW2 + kH * kH, oW3 = oB2 + kH, oB3 = oW3 + kH;
static_assert(oB3 + 1 == kMlpParams, "parameter layout");

// Philox4x32 with 10 rounds (Salmon et al., SC 2011).
__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ void box_muller(uint32_t u0, uint32_t u1, double* g0, double* g1) {
  const double a = ((double)u0 + 0.5) * 0x1p-32, b = ((double)u1 + 0.5) * 0x1p-32;
  const double r = sqrt(-2.0 * log(a));
  const double t = 2.0 * M_PI * b;
  *g0 = r * cos(t);
  *g1 = r * sin(t);
}

// Row j of cluster y's sketch block: 8 Gaussians.
__device__ void omega_row(uint32_t level, uint32_t y, uint32_t j, uint32_t seed, double* out) {
  for (uint32_t call = 0; call < 2; ++call) {
    uint32_t c[4] = {j, y, call, level};
    philox(c, seed, 0u);
    box_muller(c[0], c[1], out + 4 * call, out + 4 * call + 1);
    box_muller(c[2], c[3], out + 4 * call + 2, out + 4 * call + 3);
  }
}

// Eigenvalues of a symmetric 8x8 matrix (row-major, overwritten) by cyclic
// Jacobi rotations; returned on the diagonal.
__device__ void jacobi8(double* a) {
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int p = 0; p < 8; ++p)
      for (int q = 0; q < 8; ++q) {
        tot += a[p * 8 + q] * a[p * 8 + q];
        if (p != q) off += a[p * 8 + q] * a[p * 8 + q];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < 7; ++p)
      for (int q = p + 1; q < 8; ++q) {
        const double apq = a[p * 8 + q];
        if (apq == 0.0) continue;
        const double theta = (a[q * 8 + q] - a[p * 8 + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 8; ++k) {  // columns p, q
          const double akp = a[k * 8 + p], akq = a[k * 8 + q];
          a[k * 8 + p] = c * akp - s * akq;
          a[k * 8 + q] = s * akp + c * akq;
        }
        for (int k = 0; k < 8; ++k) {  // rows p, q
          const double apk = a[p * 8 + k], aqk = a[q * 8 + k];
          a[p * 8 + k] = c * apk - s * aqk;
          a[q * 8 + k] = s * apk + c * aqk;
        }
      }
  }
}

}  // namespace

// LDS: m (D_s^{-1/2}) + 8m (Y) + 8*256 (sketch rows) + 256 (D_y^{-1/2}) doubles.
__global__ void __launch_bounds__(256) rank_features_kernel(const FeatItem* __restrict__ items, int level,
                                                            uint32_t seed, double* feat, float* featf) {
  extern __shared__ double lds[];
  __shared__ double red[4][37];
  const FeatItem it = items[blockIdx.x];
  const int m = it.m, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* dsi = lds;
  double* Y = dsi + m;
  double* om = Y + 8 * m;
  double* djs = om + 8 * 256;
  for (int i = tid; i < m; i += 256) dsi[i] = 1.0 / sqrt(it.Ds[(size_t)i + (size_t)m * i]);
  for (int i = tid; i < 8 * m; i += 256) Y[i] = 0.0;
  __syncthreads();
  double fro = 0.0;
  for (int g = 0; g < it.nseg; ++g) {
    const FeatSeg sg = it.seg[g];
    if (sg.orient == 0) {
      // H: m x ncols block row of s; column c is DoF zl[c] of y
      for (int c0 = 0; c0 < sg.ncols; c0 += 256) {
        const int nc = min(256, sg.ncols - c0);
        if (tid < nc) {
          const int j = sg.zl[c0 + tid];
          omega_row(level, sg.y, j, seed, om + 8 * tid);
          djs[tid] = 1.0 / sqrt(sg.Dy[(size_t)j + (size_t)sg.my * j]);
        }
        __syncthreads();
        for (int i = tid; i < m; i += 256) {
          double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
          for (int cc = 0; cc < nc; ++cc) {
            const double v = sg.H[(size_t)i + (size_t)sg.ld * (c0 + cc)] * dsi[i] * djs[cc];
            fro += v * v;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += v * om[8 * cc + q];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) Y[8 * i + q] += acc[q];
        }
        __syncthreads();
      }
    } else {
      // H: m_y x ncols block row of y; column c is DoF zl[c] of s
      for (int r0 = 0; r0 < sg.ld; r0 += 256) {
        const int nr = min(256, sg.ld - r0);
        if (tid < nr) {
          const int r = r0 + tid;
          omega_row(level, sg.y, r, seed, om + 8 * tid);
          djs[tid] = 1.0 / sqrt(sg.Dy[(size_t)r + (size_t)sg.my * r]);
        }
        __syncthreads();
        for (int c = tid; c < sg.ncols; c += 256) {
          const int jp = sg.zl[c];
          double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
          for (int rr = 0; rr < nr; ++rr) {
            const double v = sg.H[(size_t)(r0 + rr) + (size_t)sg.ld * c] * dsi[jp] * djs[rr];
            fro += v * v;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += v * om[8 * rr + q];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) Y[8 * jp + q] += acc[q];
        }
        __syncthreads();
      }
    }
  }
  // Gram matrix Y^T Y (upper triangle, 36 entries) and |B|_F^2
  double gp[37];
#pragma unroll
  for (int e = 0; e < 37; ++e) gp[e] = 0.0;
  for (int i = tid; i < m; i += 256) {
    int e = 0;
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
      for (int q = p; q < 8; ++q) gp[e++] += Y[8 * i + p] * Y[8 * i + q];
  }
  gp[36] = fro;
#pragma unroll
  for (int e = 0; e < 37; ++e) {
    const double v = wave_sum(gp[e]);
    if (lane == 0) red[wv][e] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double a[64];
    int e = 0;
    for (int p = 0; p < 8; ++p)
      for (int q = p; q < 8; ++q) {
        const double v = red[0][e] + red[1][e] + red[2][e] + red[3][e];
        a[p * 8 + q] = v;
        a[q * 8 + p] = v;
        ++e;
      }
    const double f = sqrt(red[0][36] + red[1][36] + red[2][36] + red[3][36]);
    jacobi8(a);
    double ev[8];
    for (int p = 0; p < 8; ++p) ev[p] = a[p * 8 + p];
    for (int p = 1; p < 8; ++p)  // descending
      for (int q = p; q > 0 && ev[q] > ev[q - 1]; --q) {
        const double t = ev[q];
        ev[q] = ev[q - 1];
        ev[q - 1] = t;
      }
    double out[kF];
    out[0] = log2(1.0 + m);
    out[1] = log2(1.0 + it.bsum);
    out[2] = log10(f + 1e-300);
    for (int p = 0; p < 8; ++p) out[3 + p] = sqrt(fmax(ev[p], 0.0)) / fmax(f, 1e-300);
    out[11] = it.before;
    for (int q = 0; q < kF; ++q) {
      feat[(size_t)it.s * kF + q] = out[q];
      featf[(size_t)it.s * kF + q] = (float)out[q];
    }
  }
}

void launch_rank_features(const FeatItem* items, int nitems, int max_m, int level, uint32_t seed,
                          double* feat, float* featf, hipStream_t st) {
  if (nitems <= 0) return;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(rank_features_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    attr = true;
  }
  const size_t lds = ((size_t)max_m * 9 + 8 * 256 + 256) * sizeof(double);
  hipLaunchKernelGGL(rank_features_kernel, dim3(nitems), dim3(256), lds, st, items, level, seed, feat,
                     featf);
}

// ---- MLP ---------------------------------------------------------------------
__global__ void __launch_bounds__(256) mlp_predict_kernel(const float* __restrict__ P,
                                                          const float* __restrict__ X, int64_t n,
                                                          float* __restrict__ y) {
  __shared__ float w[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += 256) w[i] = P[i];
  __syncthreads();
  const int64_t s = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (s >= n) return;
  float x[kF], h1[kH];
#pragma unroll
  for (int f = 0; f < kF; ++f) x[f] = (X[s * kF + f] - w[oMu + f]) * w[oIsd + f];
  for (int i = 0; i < kH; ++i) {
    float z = w[oB1 + i];
#pragma unroll
    for (int f = 0; f < kF; ++f) z = fmaf(w[oW1 + i * kF + f], x[f], z);
    h1[i] = fmaxf(z, 0.0f);
  }
  float out = w[oB3];
  for (int j = 0; j < kH; ++j) {
    float z = w[oB2 + j];
    for (int i = 0; i < kH; ++i) z = fmaf(w[oW2 + j * kH + i], h1[i], z);
    out = fmaf(w[oW3 + j], fmaxf(z, 0.0f), out);
  }
  y[s] = out;
}

void launch_mlp_predict(const float* params, const float* X, int64_t n, float* y, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(mlp_predict_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, params, X,
                     n, y);
}

// 64 samples per workgroup, 4 threads per sample in the forward and
// backward passes; gradient entries summed over the workgroup's samples in
// sample order.  part[blockIdx][0..kMlpParams) = gradient partial sums of
// the trained parameters, part[blockIdx][kMlpParams] = sum of 0.5 (y-t)^2.
constexpr int kGS = 64;
__global__ void __launch_bounds__(256) mlp_grad_kernel(const float* __restrict__ P,
                                                       const float* __restrict__ X,
                                                       const float* __restrict__ T, int64_t n,
                                                       float inv_n, float* __restrict__ part) {
  __shared__ float w[kMlpParams];
  __shared__ float xs[kGS][kF];
  __shared__ float h1[kGS][kH];   // activations, then dz1
  __shared__ float z2[kGS][kH];   // pre-activations, then dz2
  __shared__ float ys[kGS], dy[kGS];
  const int tid = threadIdx.x;
  for (int i = tid; i < kMlpParams; i += 256) w[i] = P[i];
  __syncthreads();
  const int64_t s0 = (int64_t)blockIdx.x * kGS;
  const int ls = tid >> 2, part4 = tid & 3;  // sample, quarter of the hidden units
  const int64_t s = s0 + ls;
  const bool valid = s < n;
  if (part4 == 0) {
#pragma unroll
    for (int f = 0; f < kF; ++f) xs[ls][f] = valid ? (X[s * kF + f] - w[oMu + f]) * w[oIsd + f] : 0.0f;
  }
  __syncthreads();
  for (int i = part4 * 16; i < part4 * 16 + 16; ++i) {
    float z = w[oB1 + i];
#pragma unroll
    for (int f = 0; f < kF; ++f) z = fmaf(w[oW1 + i * kF + f], xs[ls][f], z);
    h1[ls][i] = fmaxf(z, 0.0f);
  }
  __syncthreads();
  for (int j = part4 * 16; j < part4 * 16 + 16; ++j) {
    float z = w[oB2 + j];
    for (int i = 0; i < kH; ++i) z = fmaf(w[oW2 + j * kH + i], h1[ls][i], z);
    z2[ls][j] = z;
  }
  __syncthreads();
  if (part4 == 0) {
    float o = w[oB3];
    for (int j = 0; j < kH; ++j) o = fmaf(w[oW3 + j], fmaxf(z2[ls][j], 0.0f), o);
    const float r = valid ? o - T[s] : 0.0f;
    ys[ls] = 0.5f * r * r;
    dy[ls] = r * inv_n;
  }
  __syncthreads();
  // gradients of w3, b3 need h2 = relu(z2); dz2 = dy w3 [z2 > 0]
  float* g = part + (size_t)blockIdx.x * (kMlpParams + 1);
  for (int j = tid; j < kH; j += 256) {
    float acc = 0.0f;
    for (int q = 0; q < kGS; ++q) acc = fmaf(dy[q], fmaxf(z2[q][j], 0.0f), acc);
    g[oW3 + j] = acc;
  }
  if (tid == 0) {
    float acc = 0.0f, l = 0.0f;
    for (int q = 0; q < kGS; ++q) {
      acc += dy[q];
      l += ys[q];
    }
    g[oB3] = acc;
    g[kMlpParams] = l;
  }
  __syncthreads();
  for (int j = part4 * 16; j < part4 * 16 + 16; ++j)
    z2[ls][j] = z2[ls][j] > 0.0f ? dy[ls] * w[oW3 + j] : 0.0f;
  __syncthreads();
  // dW2[j][i] = sum_q dz2[q][j] h1[q][i]; db2[j] = sum_q dz2[q][j]
  for (int e = tid; e < kH * kH; e += 256) {
    const int j = e / kH, i = e - j * kH;
    float acc = 0.0f;
    for (int q = 0; q < kGS; ++q) acc = fmaf(z2[q][j], h1[q][i], acc);
    g[oW2 + e] = acc;
  }
  for (int j = tid; j < kH; j += 256) {
    float acc = 0.0f;
    for (int q = 0; q < kGS; ++q) acc += z2[q][j];
    g[oB2 + j] = acc;
  }
  __syncthreads();
  // dz1[i] = sum_j dz2[j] W2[j][i], masked by h1 > 0 (stored over h1)
  float d1[16];
  for (int i = part4 * 16, u = 0; u < 16; ++i, ++u) {
    float acc = 0.0f;
    for (int j = 0; j < kH; ++j) acc = fmaf(z2[ls][j], w[oW2 + j * kH + i], acc);
    d1[u] = h1[ls][i] > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
  for (int u = 0; u < 16; ++u) h1[ls][part4 * 16 + u] = d1[u];
  __syncthreads();
  for (int e = tid; e < kH * kF; e += 256) {
    const int i = e / kF, f = e - i * kF;
    float acc = 0.0f;
    for (int q = 0; q < kGS; ++q) acc = fmaf(h1[q][i], xs[q][f], acc);
    g[oW1 + e] = acc;
  }
  for (int i = tid; i < kH; i += 256) {
    float acc = 0.0f;
    for (int q = 0; q < kGS; ++q) acc += h1[q][i];
    g[oB1 + i] = acc;
  }
  if (tid < 2 * kF) g[tid] = 0.0f;  // mu, isd are not trained
}

__global__ void mlp_reduce_kernel(const float* __restrict__ part, int nblk, float* __restrict__ grad,
                                  float* __restrict__ loss, float inv_n) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e > kMlpParams) return;
  float acc = 0.0f;
  for (int b = 0; b < nblk; ++b) acc += part[(size_t)b * (kMlpParams + 1) + e];
  if (e < kMlpParams) grad[e] = acc;
  else if (loss) *loss = acc * inv_n;
}

void launch_mlp_grad(const float* params, const float* X, const float* t, int64_t n, float* part,
                     float* grad, float* loss, hipStream_t st) {
  const int nblk = (int)((n + kGS - 1) / kGS);
  const float inv_n = 1.0f / (float)n;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(256), 0, st, params, X, t, n, inv_n, part);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kMlpParams + 256) / 256), dim3(256), 0, st, part, nblk,
                     grad, loss, inv_n);
}

int mlp_partial_floats(int64_t n) { return (int)((n + kGS - 1) / kGS) * (kMlpParams + 1); }

__global__ void mlp_adam_kernel(float* __restrict__ P, const float* __restrict__ g, float* __restrict__ m1,
                                float* __restrict__ m2, float lr, float c1, float c2) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < 2 * kF || e >= kMlpParams) return;
  const float b1 = 0.9f, b2 = 0.999f;
  const float a = b1 * m1[e] + (1.0f - b1) * g[e];
  const float v = b2 * m2[e] + (1.0f - b2) * g[e] * g[e];
  m1[e] = a;
  m2[e] = v;
  P[e] -= lr * (a * c1) / (sqrtf(v * c2) + 1e-8f);
}

void launch_mlp_adam(float* params, const float* grad, float* m1, float* m2, float lr, int step,
                     hipStream_t st) {
  const float c1 = 1.0f / (1.0f - powf(0.9f, (float)step));
  const float c2 = 1.0f / (1.0f - powf(0.999f, (float)step));
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, params, grad, m1,
                     m2, lr, c1, c2);
}

// Input statistics (feature mean, inverse deviation) and the target mean,
// one workgroup per column in a fixed summation order; then He-normal
// weights from Philox (counter (index, layer, 0, 0), key (seed_lo, seed_hi)).
__global__ void __launch_bounds__(256) mlp_stats_kernel(const float* __restrict__ X,
                                                        const float* __restrict__ t, int64_t n,
                                                        float* __restrict__ P) {
  __shared__ double sh[4];
  const int f = blockIdx.x;  // kF columns, then the target
  double s = 0.0, s2 = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = f < kF ? X[i * kF + f] : t[i];
    s += v;
    s2 += v * v;
  }
  s = group_sum<256>(s, sh);
  s2 = group_sum<256>(s2, sh);
  if (threadIdx.x == 0) {
    const double mean = s / (double)n;
    const double var = fmax(s2 / (double)n - mean * mean, 0.0);
    if (f < kF) {
      P[oMu + f] = (float)mean;
      P[oIsd + f] = (float)(var > 1e-12 ? 1.0 / sqrt(var) : 1.0);
    } else {
      P[oB3] = (float)mean;
    }
  }
}

__global__ void mlp_weights_kernel(float* __restrict__ P, uint32_t seed_lo, uint32_t seed_hi) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < oW1 || e >= oB3) return;
  float scale = 0.0f;
  if (e < oB1) scale = sqrtf(2.0f / kF);
  else if (e >= oW2 && e < oB2) scale = sqrtf(2.0f / kH);
  else if (e >= oW3) scale = sqrtf(1.0f / kH);
  if (scale == 0.0f) {
    P[e] = 0.0f;  // biases
    return;
  }
  uint32_t c[4] = {(uint32_t)e, 7u, 0u, 0u};
  philox(c, seed_lo, seed_hi);
  double g0, g1;
  box_muller(c[0], c[1], &g0, &g1);
  P[e] = (float)(scale * g0);
}

void launch_mlp_init(float* params, const float* X, const float* t, int64_t n, uint64_t seed,
                     hipStream_t st) {
  hipLaunchKernelGGL(mlp_weights_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, params,
                     (uint32_t)seed, (uint32_t)(seed >> 32));
  hipLaunchKernelGGL(mlp_stats_kernel, dim3(kF + 1), dim3(256), 0, st, X, t, n, params);
}

}  // namespace lrsp
