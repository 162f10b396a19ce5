// devutil.hpp -- device helpers shared by the gfx950 kernels: wave64 and
// workgroup reductions, error reporting, MFMA operand types.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "desc.hpp"

namespace lrsp {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

constexpr double kTie = 1e-10;  // pivot tie window of the column-pivoted QR

// Workgroup barrier that orders LDS only: pending global stores are not
// waited for (for phases that exchange data through LDS alone).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Loads and stores through the global address space, for plain pointers to
// device memory held in descriptors: they count on the vector-memory counter
// only, so that waits for LDS results do not also wait for them (accesses
// through generic pointers count on both).
template <class T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ void gstore(T* p, const T& v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

// Value of v in lane l (l uniform across the wave).
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Data-parallel-primitive lane exchange within rows of 16 lanes (every
// source lane lies in the row, all lanes active).
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <- 7-i in rows of 8
constexpr int kDppMirror = 0x140;     // lane i <- 15-i in rows of 16

// Wave-wide max / min: every 16-lane row reduces by register
// exchanges (each lane of a row ends with the same value), then the four
// row results combine in a fixed order; all lanes get the result.
__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp_d<kDppXor1>(v));
  v = fmax(v, dpp_d<kDppXor2>(v));
  v = fmax(v, dpp_d<kDppHalfMirror>(v));
  v = fmax(v, dpp_d<kDppMirror>(v));
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ int wave_min_dpp(int v) {
  v = min(v, dpp_i<kDppXor1>(v));
  v = min(v, dpp_i<kDppXor2>(v));
  v = min(v, dpp_i<kDppHalfMirror>(v));
  v = min(v, dpp_i<kDppMirror>(v));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Sum over the 64 lanes (all active), every lane gets the result: rows of
// 16 lanes reduce by register exchanges (all lanes of a row end with the
// same value, the additions being commutative), then the row sums combine
// as (r0 + r1) + (r2 + r3).  A fixed order: the same bits on every call.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<kDppXor1>(v);
  v += dpp_d<kDppXor2>(v);
  v += dpp_d<kDppHalfMirror>(v);
  v += dpp_d<kDppMirror>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Sum over the workgroup (nt threads, nt/64 <= 16 waves); every thread gets
// the result.  sh: >= nt/64 doubles of LDS.
template <int NT>
__device__ __forceinline__ double group_sum(double v, double* sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) r += sh[i];
  return r;
}

template <int NT>
__device__ __forceinline__ double group_max(double v, double* sh) {
  v = wave_max_dpp(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) r = fmax(r, sh[i]);
  return r;
}

template <int NT>
__device__ __forceinline__ int group_min_int(int v, int* sh) {
  v = wave_min_dpp(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  int r = sh[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) r = min(r, sh[i]);
  return r;
}

__device__ __forceinline__ void set_error(int32_t* err, int level, int cluster, int code) {
  if (atomicCAS(&err[0], 0, 1) == 0) {
    err[1] = level;
    err[2] = cluster;
    err[3] = code;
  }
}

// Error of the cluster of an item: first error of the level, plus the bit of
// the code in the item's system word.
__device__ __forceinline__ void item_error(const ItemD& it, int32_t* err, int level, int code) {
  set_error(err, level, it.s, code);
  if (it.serr) atomicOr(it.serr, 1 << code);
}

// Grid-wide barrier over nblocks resident workgroups without a cooperative
// launch.  Every wait is bounded: after kBarSpins polls the workgroup gives
// up, records the timeout and goes on, so every wave still exits.
constexpr uint32_t kBarSpins = 1u << 22;
__device__ __forceinline__ void sw_grid_sync(GridBar* b, uint32_t nblocks) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t g = __hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t arrived = __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t spins = 0;
      while (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > kBarSpins) {
          __hip_atomic_store(&b->timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
}

// Column-major lower-triangular tile enumeration: index -> (R, C), R >= C.
__device__ __forceinline__ void tri_tile(int idx, int nt, int& R, int& C) {
  double b = 2.0 * nt + 1.0;
  int c = (int)((b - sqrt(b * b - 8.0 * idx)) * 0.5);
  if (c < 0) c = 0;
  while (c > 0 && (long)c * nt - (long)c * (c - 1) / 2 > idx) --c;
  while ((long)(c + 1) * nt - (long)(c + 1) * c / 2 <= idx) ++c;
  C = c;
  R = c + (idx - (c * nt - c * (c - 1) / 2));
}

__device__ __forceinline__ float round_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

// MFMA tiles, lane l of a wave64 (layouts checked on gfx950):
//   f64 16x16x4 : A[l%16][l/16], B[l/16][l%16], D[4i + l/16][l%16]
//   f32 16x16x4 : A[l%16][l/16], B[l/16][l%16], D[4(l/16) + i][l%16]
//   bf16 16x16x16: A[l%16][4(l/16)+j], B[4(l/16)+j][l%16], D as f32
__device__ __forceinline__ int mfma64_row(int lane, int i) { return 4 * i + (lane >> 4); }
__device__ __forceinline__ int mfma32_row(int lane, int i) { return 4 * (lane >> 4) + i; }

// Copies a rows x cols column-major global block (leading dimension lds_src)
// into LDS with row stride ldd (dst[r*ldd + c]), zero outside `valid`
// (valid(r, c) decides), with NT threads and 8 loads in flight per thread.
template <int NT, class Valid>
__device__ __forceinline__ void load_block_rowmajor(double* dst, int ldd, const double* src, size_t ld_src,
                                                    int rows, int cols, Valid valid) {
  const int n = rows * cols;
  for (int e0 = threadIdx.x; e0 < n; e0 += NT * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT;
      const int c = e / rows, r = e - c * rows;
      v[u] = (e < n && valid(r, c)) ? src[(size_t)r + ld_src * c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT;
      if (e < n) {
        const int c = e / rows, r = e - c * rows;
        dst[r * ldd + c] = v[u];
      }
    }
  }
}

// Stores an LDS block (row stride ldd) to a column-major global block.
template <int NT>
__device__ __forceinline__ void store_block_rowmajor(double* dst, size_t ld_dst, const double* src, int ldd,
                                                     int rows, int cols) {
  const int n = rows * cols;
  for (int e = threadIdx.x; e < n; e += NT) {
    const int c = e / rows, r = e - c * rows;
    dst[(size_t)r + ld_dst * c] = src[r * ldd + c];
  }
}

}  // namespace lrsp
