// split.hip -- elimination of the clusters of one colour when clusters are
// large: each step of the scaled low-rank elimination is its own launch and
// spreads a cluster over several workgroups where the step allows it.
//
//   seg_offsets  segment widths -> panel column offsets, column metadata
//   gather       [A_ss | A_sn | A_sw] -> panel P (several wgs per cluster)
//   potrf        A_ss = G G^T, one 512-thread wg per cluster; up to
//                kInvMaxDofs DoFs also G^{-1}, the matrix held in registers
//   trsm         G^{-1}[A_sn | A_sw] by column chunks: products with G^{-1}
//                on MFMA (up to kInvMaxDofs DoFs), else blocked solves;
//                also the squared norms of the far-field columns
//   cpqr         column-pivoted QR of the scaled far field (one wg)
//   applyq       C = U^T G^{-1} A_sn by column chunks
//   schur        X -= F^T F, 32x32 output tiles on MFMA (f64, f32 or bf16
//                inputs), scattered to the owning blocks
//   writeback    coarse row of s, identity diagonal block
#include <hip/hip_runtime.h>

#include "desc.hpp"
#include "devutil.hpp"
#include "kernels.hpp"

namespace lrsp {

namespace {
constexpr int kRegRows = kMaxClusterDofs / 64;
}

__global__ void __launch_bounds__(256) seg_offsets_kernel(const ItemD* __restrict__ items,
                                                          LevelState ls, int level) {
  extern __shared__ int soff[];
  __shared__ int wsum[4];
  __shared__ int sbad;
  const ItemD& it = items[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nseg = it.nseg;
  if (tid == 0) sbad = 0;
  __syncthreads();
  int carry = 0;
  for (int base = 0; base < nseg; base += 256) {
    const int i = base + tid;
    int w = 0;
    if (i < nseg) {
      const SegD& sg = it.seg[i];
      w = sg.coarse ? ls.k[sg.y] : sg.nfine;
      if (w < 0 || w > sg.cap) {
        sbad = 1;
        w = 0;
      }
    }
    int x = w;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int pre = 0;
    for (int q = 0; q < wv; ++q) pre += wsum[q];
    const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (i < nseg) soff[i] = carry + pre + x - w;
    carry += tot;
    __syncthreads();
  }
  if (tid == 0) soff[nseg] = carry;
  __syncthreads();
  const int total = soff[nseg];
  const int a = soff[it.nsegn];
  if (tid == 0 && total > it.pcap) sbad = 1;
  __syncthreads();
  if (sbad) {
    if (tid == 0) {
      item_error(it, ls.err, level, kErrCapacity);
      ls.a[it.s] = 0;
      ls.b[it.s] = 0;
    }
    return;
  }
  for (int i = tid; i <= nseg; i += 256) it.segoff[i] = soff[i];
  if (tid == 0) {
    ls.a[it.s] = a;
    ls.b[it.s] = total - a;
  }
  for (int c = tid; c < total; c += 256) {
    int lo = 0, hi = nseg - 1;  // last segment starting at or before c
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (soff[mid] <= c) lo = mid;
      else hi = mid - 1;
    }
    const SegD& sg = it.seg[lo];
    const int loc = c - soff[lo];
    const int nat = sg.coarse ? loc : sg.zl[loc];
    it.colseg[c] = lo;
    it.colnat[c] = nat;
    it.vidx[c] = sg.voff + nat;
  }
}

// 32 panel columns per workgroup, eight per wave: the column sources of all
// eight are looked up together, then their rows (R per lane) are loaded
// together and stored.
template <int R>
__global__ void __launch_bounds__(256) gather_panel_kernel(const ItemD* __restrict__ items,
                                                           LevelState ls) {
  const ItemD& it = items[blockIdx.x];
  const int m = it.m;
  if (m == 0) return;
  const int ncols = m + gload(ls.a + it.s) + gload(ls.b + it.s);
  const int c0 = blockIdx.y * 32;
  if (c0 >= ncols) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int sg[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int c = c0 + wv + 4 * q;
    sg[q] = (c >= m && c < ncols) ? gload(it.colseg + (c - m)) : 0;
  }
  const double* src[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int c = c0 + wv + 4 * q;
    if (c < m) {
      src[q] = it.D + (size_t)m * c;
    } else if (c < ncols) {
      const double* base = gload(&it.seg[sg[q]].src);
      src[q] = base + (size_t)m * (c - m - gload(it.segoff + sg[q]));
    } else {
      src[q] = it.D;
    }
  }
  double v[8][R];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int c = c0 + wv + 4 * q;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int r = lane + 64 * t;
      v[q][t] = (c < ncols && r < m) ? gload(src[q] + r) : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int c = c0 + wv + 4 * q;
    double* dst = it.P + (size_t)m * c;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int r = lane + 64 * t;
      if (c < ncols && r < m) gstore(dst + r, v[q][t]);
    }
  }
}

// ---------------------------------------------------------------------------
// Blocked right-looking Cholesky (lower, in place) by one workgroup of NT
// threads.  The 32-wide panel is staged in LDS (row stride 33); its diagonal
// block is factored by wave 0 in registers, the rows below by one thread per
// row; the trailing update runs on v_mfma_f64_16x16x4 in 16x16 lower tiles,
// four tiles per wave loaded before they are updated.
// LDS: m*33 doubles.
template <int NT>
__device__ void potrf_wg(double* A, int ld, int m, double* lds, int* bad) {
  constexpr int NB = 32, LDL = 33, NWV = NT / 64, G = 4;
  double* Lp = lds;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int jb = 0; jb < m; jb += NB) {
    const int w = min(NB, m - jb);
    const int rows = m - jb;
    load_block_rowmajor<NT>(Lp, LDL, A + (size_t)jb * ld + jb, (size_t)ld, rows, NB,
                            [&](int r, int c) { return c < w && c <= r; });
    __syncthreads();
    if (wv == 0) {
      double row[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) row[u] = (lane < w) ? Lp[lane * LDL + u] : 0.0;
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        if (u < w) {
          double d = readlane_d(row[u], u);
          if (!(d > 0.0)) {
            if (lane == 0) *bad = 1;
            d = 1.0;
          }
          d = sqrt(d);
          if (lane == u) row[u] = d;
          else if (lane > u) row[u] = row[u] / d;
#pragma unroll
          for (int v = u + 1; v < NB; ++v) {
            const double lvu = readlane_d(row[u], v);
            if (v < w && lane >= v && lane < w) row[v] -= row[u] * lvu;
          }
        }
      }
      if (lane < w) {
#pragma unroll
        for (int u = 0; u < NB; ++u) Lp[lane * LDL + u] = (u <= lane) ? row[u] : 0.0;
      }
    }
    __syncthreads();
    for (int r = w + tid; r < rows; r += NT) {
      double x[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) x[u] = (u < w) ? Lp[r * LDL + u] : 0.0;
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        if (u < w) {
          double s = x[u];
#pragma unroll
          for (int v = 0; v < u; ++v) s -= Lp[u * LDL + v] * x[v];
          x[u] = s / Lp[u * LDL + u];
        }
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) Lp[r * LDL + u] = x[u];
    }
    __syncthreads();
    for (int e = tid; e < rows * w; e += NT) {
      const int c = e / rows, r = e - c * rows;
      if (c <= r) A[(size_t)(jb + r) + (size_t)ld * (jb + c)] = Lp[r * LDL + c];
    }
    const int rb = rows - w;
    const int nt = (rb + 15) >> 4;
    const int ntiles = nt * (nt + 1) / 2;
    for (int t0 = wv; t0 < ntiles; t0 += NWV * G) {
      int TR[G], TC[G];
      double cur[G][4];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int t = t0 + g * NWV;
        TR[g] = -1;
        TC[g] = 0;
        if (t < ntiles) tri_tile(t, nt, TR[g], TC[g]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 16 * TC[g] + 4 * i + (lane >> 4), r = 16 * TR[g] + (lane & 15);
          cur[g][i] = (TR[g] >= 0 && r < rb && c <= r)
                          ? A[(size_t)(jb + w + r) + (size_t)ld * (jb + w + c)]
                          : 0.0;
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (TR[g] < 0) continue;
        const int cr = 16 * TC[g] + (lane & 15), rr = 16 * TR[g] + (lane & 15);
        d4_t acc = {0.0, 0.0, 0.0, 0.0};
        for (int u0 = 0; u0 < w; u0 += 4) {
          const int u = u0 + (lane >> 4);
          const double av = (cr < rb && u < w) ? Lp[(w + cr) * LDL + u] : 0.0;
          const double bv = (rr < rb && u < w) ? Lp[(w + rr) * LDL + u] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 16 * TC[g] + 4 * i + (lane >> 4), r = 16 * TR[g] + (lane & 15);
          if (r < rb && c <= r) A[(size_t)(jb + w + r) + (size_t)ld * (jb + w + c)] = cur[g][i] - acc[i];
        }
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(512) potrf_kernel(const ItemD* __restrict__ items, LevelState ls,
                                                    int level) {
  extern __shared__ double lds[];
  __shared__ int sbad;
  const ItemD& it = items[blockIdx.x];
  const int m = it.m;
  if (m == 0) return;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  potrf_wg<512>(it.P, m, m, lds, &sbad);
  __syncthreads();
  if (threadIdx.x == 0) ls.giok[it.s] = 0;
  if (sbad && threadIdx.x == 0) item_error(it, ls.err, level, kErrNotSPD);
}

// Dense top of the factorization (n <= kSplitMaxDofs): the same blocked
// Cholesky by one workgroup of 512 threads, the trailing updates on MFMA.
__global__ void __launch_bounds__(512) top_potrf_wg_kernel(double* A, int n, int32_t* err) {
  extern __shared__ double lds[];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  potrf_wg<512>(A, n, n, lds, &sbad);
  __syncthreads();
  if (sbad && threadIdx.x == 0) set_error(err, -1, -1, kErrNotSPD);
}

void launch_top_potrf_wg(double* A, int n, int32_t* err, hipStream_t st) {
  if (n <= 0) return;
  static bool lds_set = false;
  if (!lds_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(top_potrf_wg_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    lds_set = true;
  }
  hipLaunchKernelGGL(top_potrf_wg_kernel, dim3(1), dim3(512), (size_t)n * 33 * 8, st, A, n, err);
}

// The same for the tops of a batch with 64..512 unknowns, one workgroup per
// top (the others are factored by top_potrf_batched_kernel).
__global__ void __launch_bounds__(512) top_potrf_wg_batched_kernel(const TopD* __restrict__ tops) {
  extern __shared__ double lds[];
  __shared__ int sbad;
  const TopD t = tops[blockIdx.x];
  if (t.n < 64 || t.n > kSplitMaxDofs) return;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  potrf_wg<512>(t.L, t.n, t.n, lds, &sbad);
  __syncthreads();
  if (sbad && threadIdx.x == 0) atomicOr(t.err, 1 << kErrNotSPD);
}

void launch_top_potrf_wg_batched(const TopD* tops, int ntops, int max_n, hipStream_t st) {
  if (ntops <= 0 || max_n < 64) return;
  static bool lds_set = false;
  if (!lds_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(top_potrf_wg_batched_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    lds_set = true;
  }
  hipLaunchKernelGGL(top_potrf_wg_batched_kernel, dim3(ntops), dim3(512), (size_t)max_n * 33 * 8, st, tops);
}

// ---------------------------------------------------------------------------
// Cholesky factor G and explicit inverse G^{-1} of the diagonal block of a
// cluster of at most kInvMaxDofs DoFs by one workgroup of 1024 threads, the
// matrix resident in registers: 16x16 tiles in the accumulator layout of
// v_mfma_f64_16x16x4 (lane l, slot v: row 4v + l/16, column l%16).  Tile rows
// r and 15 - r (17 tiles) belong to waves r and r + 8, which take the even
// and the odd tiles of the pair.  Padding beyond m is the identity.
//   G: right-looking by tile columns p.  Wave 0 factors the diagonal tile
//   (readlane broadcasts, reciprocal square roots) and inverts it; the tiles
//   below are G_ip = A_ip G_pp^{-T} on MFMA; the trailing tiles are updated on
//   MFMA.
//   G^{-1}: forward substitution G X = I by tile rows, in the same steps: at
//   step p, once G_pp^{-1} is known, X_pp = G_pp^{-1} and X_pj = G_pp^{-1}
//   acc_pj (j < p, one wave per tile), and with the trailing update the
//   accumulators of the rows i > p take acc_ij -= G_ip X_pj (j <= p; acc_ip
//   starts at zero, the identity having no entries below the diagonal) in
//   the registers of the tiles of G that are final by then.
// G goes to the diagonal block of the panel (lower triangle), G^{-1} to Gi
// (lower tiles, zeros above the diagonal inside the diagonal tiles); no
// thread reads these stores back, so the barriers order LDS only.
constexpr int kInvWaves = 8;          // waves of the Cholesky-inverse workgroup
constexpr int kInvLdP = 17;           // row stride of the LDS tiles
constexpr int kInvLdX = 16 * 16 + 1;  // row stride of the X row-block buffer
constexpr size_t kInvLds = (size_t)(2 * 256 * kInvLdP + 16 * kInvLdP + 2 * 16 * kInvLdX + 16) * sizeof(double);
// Waves of the workgroup: tile rows r and 15 - r (17 tiles) belong to wave r
// (NW = 8), or to waves r and r + 8, which take the even and the odd tiles
// of the pair (NW = 16).
template <int NW>
struct InvMap {
  static constexpr int kSlots = NW == 8 ? 17 : 9;  // tiles per wave
  // Tile (r, c) of slot j of wave w; false when the slot is unused.
  __device__ static __forceinline__ bool slot(int w, int j, int& r, int& c) {
    const int pr = w & 7, g = NW == 8 ? j : 2 * j + (w >> 3);
    if (g <= pr) {
      r = pr;
      c = g;
    } else {
      r = 15 - pr;
      c = g - pr - 1;
    }
    return g < 17;
  }
};

// Look-ahead of chol_inv_kernel: from tile step kLookAheadFrom on, wave
// kLookAheadWave owns no tile below the diagonal step (its tile rows 7 and 8
// are final), so during the trailing phase of step p it forms the diagonal
// tile p + 1 as soon as the owner of that tile has updated it, instead of
// wave 0 after the phase.  The same operations on the same values.
constexpr bool kLookAhead = true;
constexpr int kLookAheadFrom = 8;
constexpr int kLookAheadWave = 7;
// Polls of the look-ahead wave before it gives up on the tile and reports
// the block as failed (a bound only: the owner hands the tile over
// unconditionally).
constexpr uint32_t kLookAheadSpins = 1u << 22;

// Diagonal tile p of chol_inv_kernel by one wave: G_pp (lane r holds row r;
// reciprocal square roots from v_rsq_f64 refined by one Newton step) in Dd,
// and row r of G_pp^{-1} in the same lane by forward substitution across the
// lanes (readlane broadcasts) into the columns 16p.. of Xr (X_pp of the
// inverse).  A pivot that is not > 0 is replaced by 1 and sets *sbad.
__device__ __forceinline__ void inv_diag_tile(double* Dd, double* Xr, int p, int lane, int* sbad) {
  double row[16], Y[16], rdl = 1.0;
  bool bad = false;
#pragma unroll
  for (int u = 0; u < 16; ++u) row[u] = lane < 16 ? Dd[lane * kInvLdP + u] : 0.0;
#pragma unroll
  for (int c = 0; c < 16; ++c) Y[c] = 0.0;
  // pivot u of G_pp, then row u of its inverse, which needs only column u
  // of G_pp (final after pivot u): the two dependency chains are
  // interleaved in one branch-free block (selects instead of lane
  // branches), with the same operations per entry as one after the other
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    double d = readlane_d(row[u], u);
    const bool nonpos = !(d > 0.0);
    bad = bad || nonpos;
    d = nonpos ? 1.0 : d;
    double y = __builtin_amdgcn_rsq(d);
    y = y + y * (0.5 - 0.5 * d * y * y);
    // every lane computes; only the lower part of the tile (lane >= the
    // column, lane < 16) is ever read again, so no lane needs masking
    rdl = lane == u ? y : rdl;
    row[u] = lane == u ? d * y : row[u] * y;
#pragma unroll
    for (int v = u + 1; v < 16; ++v) {
      const double lvu = readlane_d(row[u], v);
      row[v] -= row[u] * lvu;
    }
    // row u of G_pp^{-1}: lane u solves for its entries, the lanes below
    // take its contribution
#pragma unroll
    for (int c = 0; c <= u; ++c) {
      const double t = ((c == u ? 1.0 : 0.0) - Y[c]) * rdl;
      Y[c] = lane == u ? t : Y[c];
    }
#pragma unroll
    for (int c = 0; c <= u; ++c) {
      const double yuc = readlane_d(Y[c], u);
      const double t = Y[c] + row[u] * yuc;
      Y[c] = lane > u ? t : Y[c];
    }
  }
  if (bad && lane == 0) *sbad = 1;
  if (lane < 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      Dd[lane * kInvLdP + u] = u <= lane ? row[u] : 0.0;
      Xr[lane * kInvLdX + 16 * p + u] = u <= lane ? Y[u] : 0.0;
    }
  }
}

template <int NW>
__global__ void __launch_bounds__(NW * 64) chol_inv_kernel(const ItemD* __restrict__ items, LevelState ls,
                                                           int level) {
  using Map = InvMap<NW>;
  constexpr int kInvSlots = Map::kSlots;
  static_assert(NW * 16 * kInvLdP <= 16 * kInvLdX, "staging tiles of the initial load must fit in Ar");
  extern __shared__ double lds[];
  double* Pc = lds;                  // 256 x kInvLdP: tile column p (two buffers
  double* Pc2 = Pc + 256 * kInvLdP;  //   in turn during the Cholesky)
  double* Dd = Pc2 + 256 * kInvLdP;  // 16 x kInvLdP: diagonal tile
  double* Xr = Dd + 16 * kInvLdP;    // 16 x kInvLdX: tile row p of X
  double* Ar = Xr + 16 * kInvLdX;    // 16 x kInvLdX: accumulators of tile row p
  __shared__ int sbad;
  __shared__ int sla;  // last diagonal tile handed to the look-ahead wave
  const ItemD& it = items[blockIdx.x];
  const int m = it.m;
  if (m == 0) return;
  if (m > kInvMaxDofs || !it.Gi) {
    if (threadIdx.x == 0) item_error(it, ls.err, level, kErrTooLarge);
    return;
  }
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // tile coordinates in scalar registers
  const int lr = lane >> 4, lc = lane & 15;
  const int nt = (m + 15) >> 4;
  double* A = it.P;
  double* Xg = it.Gi;
  static_assert(!kLookAhead || (kLookAheadWave & 7) == 7, "the look-ahead wave owns tile rows 7 and 8");
  if (tid == 0) {
    sbad = 0;
    sla = -1;
  }
  // the wave's tiles, loaded with lane l on row l%16 of columns 4v + l/16 (16
  // consecutive rows of a column per 16 lanes), then turned into the
  // accumulator layout through a 16 x 17 staging tile of the wave in Ar (free
  // until the first step's update)
  d4_t T[kInvSlots];
#pragma unroll
  for (int j = 0; j < kInvSlots; ++j) {
    int r, c;
    const bool on = Map::slot(w, j, r, c) && r < nt;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gr = 16 * r + lc, gc = 16 * c + 4 * v + lr;
      double x = 0.0;
      if (on && gc <= gr) x = gr < m ? gload(A + gr + (size_t)m * gc) : (gr == gc ? 1.0 : 0.0);
      T[j][v] = x;
    }
  }
  {
    double* S = Ar + w * 16 * kInvLdP;
#pragma unroll
    for (int j = 0; j < kInvSlots; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) S[lc * kInvLdP + 4 * v + lr] = T[j][v];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
      for (int v = 0; v < 4; ++v) T[j][v] = S[(4 * v + lr) * kInvLdP + lc];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  }
  // ---- G ----
  // tile column 0 to LDS; later columns are put there by the step before
#pragma unroll
  for (int j = 0; j < kInvSlots; ++j) {
    int r, c;
    if (Map::slot(w, j, r, c) && r < nt && c == 0) {
      double* dst = r == 0 ? Dd : Pc + (size_t)16 * r * kInvLdP;
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[(4 * v + lr) * kInvLdP + lc] = T[j][v];
    }
  }
  lds_barrier();
  for (int p = 0; p < nt; ++p) {
    // tile coordinates are recomputed every step rather than kept live
    int wq = w;
    asm volatile("" : "+s"(wq));
    double* Pcur = (p & 1) ? Pc2 : Pc;   // tile column p
    double* Pnext = (p & 1) ? Pc : Pc2;  // tile column p + 1
    // diagonal tile p by wave 0, unless wave 7 formed it during the
    // trailing phase of step p - 1
    if (!(kLookAhead && p > kLookAheadFrom)) {
      if (w == 0) inv_diag_tile(Dd, Xr, p, lane, &sbad);
      lds_barrier();
    }
    // tile column p of G: G_pp from Dd; G_ip = A_ip G_pp^{-T} on MFMA, back to
    // the tile's rows of Pcur for the trailing update
#pragma unroll
    for (int j = 0; j < kInvSlots; ++j) {
      __builtin_amdgcn_sched_barrier(0);
      int r, c;
      if (!Map::slot(wq, j, r, c) || r >= nt || r < p || c != p) continue;
      d4_t x = {0.0, 0.0, 0.0, 0.0};
      if (r == p) {
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] = Dd[(4 * v + lr) * kInvLdP + lc];
      } else {
        double* rows = Pcur + (size_t)16 * r * kInvLdP;
        double av[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) av[s4] = rows[lc * kInvLdP + 4 * s4 + lr];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
          x = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s4], Xr[lc * kInvLdX + 16 * p + 4 * s4 + lr], x, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) rows[(4 * v + lr) * kInvLdP + lc] = x[v];
      }
      T[j] = x;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gr = 16 * r + 4 * v + lr, gc = 16 * p + lc;
        if (gr < m && gc <= gr) gstore(A + gr + (size_t)m * gc, x[v]);
      }
    }
    // tile row p of G^{-1}: X_pj = G_pp^{-1} acc_pj (j < p, the accumulators
    // in Ar) and X_pp = G_pp^{-1}, one tile per wave at a time; X_pj goes to
    // the columns 16j.. of Xr (only the columns 16p.. are read above)
    for (int jt = w; jt <= p; jt += NW) {
      d4_t x = {0.0, 0.0, 0.0, 0.0};
      if (jt < p) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
          x = __builtin_amdgcn_mfma_f64_16x16x4f64(Xr[lc * kInvLdX + 16 * p + 4 * s4 + lr],
                                                   Ar[(4 * s4 + lr) * kInvLdX + 16 * jt + lc], x, 0, 0, 0);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] = Xr[(4 * v + lr) * kInvLdX + 16 * p + lc];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (jt < p) Xr[(4 * v + lr) * kInvLdX + 16 * jt + lc] = x[v];
        const int gr = 16 * p + 4 * v + lr, gc = 16 * jt + lc;
        if (gr < m && gc < m) gstore(Xg + gr + (size_t)m * gc, x[v]);
      }
    }
    lds_barrier();
    // look-ahead: the owner of tile (p + 1, p + 1) updates it first and hands
    // it over in Dd; the look-ahead wave, idle otherwise, forms G and X of
    // diagonal tile p + 1 meanwhile
    const bool la = kLookAhead && p >= kLookAheadFrom && p + 1 < nt;
    if (la) {
#pragma unroll
      for (int j = 0; j < kInvSlots; ++j) {
        __builtin_amdgcn_sched_barrier(0);
        int r, c;
        if (!Map::slot(wq, j, r, c) || r != p + 1 || c != p + 1) continue;
        d4_t acc = T[j];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const double av = Pcur[(16 * r + lc) * kInvLdP + 4 * s4 + lr];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-av, av, acc, 0, 0, 0);
        }
        T[j] = acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) Dd[(4 * v + lr) * kInvLdP + lc] = acc[v];
        __hip_atomic_store(&sla, p + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      if (w == kLookAheadWave) {
        uint32_t spins = 0;
        while (__hip_atomic_load(&sla, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != p + 1) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kLookAheadSpins) {
            if (lane == 0) sbad = 1;
            break;
          }
        }
        inv_diag_tile(Dd, Xr, p + 1, lane, &sbad);
      }
    }
    // rows r > p: trailing tiles T_rc -= G_rp G_cp^T (c > p), the tiles of
    // column p + 1, final now, to Dd and Pnext for the next step
#pragma unroll
    for (int j = 0; j < kInvSlots; ++j) {
      __builtin_amdgcn_sched_barrier(0);
      int r, c;
      if (!Map::slot(wq, j, r, c) || r >= nt || r <= p || c <= p) continue;
      if (la && r == p + 1 && c == p + 1) continue;
      d4_t acc = T[j];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const double av = Pcur[(16 * r + lc) * kInvLdP + 4 * s4 + lr];
        const double bv = Pcur[(16 * c + lc) * kInvLdP + 4 * s4 + lr];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-av, bv, acc, 0, 0, 0);
      }
      T[j] = acc;
      if (c == p + 1) {
        double* dst = r == p + 1 ? Dd : Pnext + (size_t)16 * r * kInvLdP;
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[(4 * v + lr) * kInvLdP + lc] = acc[v];
      }
    }
    // and the inverse's accumulators acc_rc -= G_rp X_pc (c <= p; tile (r, p)
    // held G_rp, which Pcur keeps), those of row p + 1 to Ar for the next step
#pragma unroll
    for (int j = 0; j < kInvSlots; ++j) {
      __builtin_amdgcn_sched_barrier(0);
      int r, c;
      if (!Map::slot(wq, j, r, c) || r >= nt || r <= p || c > p) continue;
      d4_t acc = T[j];
      if (c == p) acc = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const double av = Pcur[(16 * r + lc) * kInvLdP + 4 * s4 + lr];
        const double bv = Xr[(4 * s4 + lr) * kInvLdX + 16 * c + lc];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-av, bv, acc, 0, 0, 0);
      }
      T[j] = acc;
      if (r == p + 1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Ar[(4 * v + lr) * kInvLdX + 16 * c + lc] = acc[v];
      }
    }
    lds_barrier();
  }
  if (sbad) {
    if (tid == 0) item_error(it, ls.err, level, kErrNotSPD);
    return;
  }
  if (tid == 0) ls.giok[it.s] = 1;
}

// B <- G^{-1} B for 32 columns of [A_sn | A_sw] per workgroup with the
// inverse from chol_inv_kernel (512 threads): the column chunk is staged in
// LDS, wave w computes the output tiles of tile rows w and 15 - w on MFMA
// (the k <= i tiles of G^{-1}, eight tiles of it loaded at a time), writes
// them back in place; the squared norms of the far-field columns are summed
// over the tile rows in order.  LDS: kTrsmInvLds bytes.
constexpr int kTrsmInvLdB = 33;
constexpr size_t kTrsmInvLds = (size_t)(256 * kTrsmInvLdB + 16 * 32) * sizeof(double);

// NC = 32 or 16 columns per workgroup (the autotuner's tile choice): every
// column goes through the same MFMA sequence and norm sums either way, so
// the results do not depend on NC.
template <int NC>
__global__ void __launch_bounds__(512) trsm_inv_kernel(const ItemD* __restrict__ items, LevelState ls,
                                                       int level) {
  static_assert(NC == 16 || NC == 32, "column tile");
  extern __shared__ double lds[];
  const ItemD& it = items[blockIdx.x];
  const int m = it.m;
  if (m == 0) return;
  const int a = ls.a[it.s], nb = a + ls.b[it.s];
  const int c0 = blockIdx.y * NC;
  if (c0 >= nb) return;
  if (m > kInvMaxDofs || !it.Gi) {
    if (threadIdx.x == 0) item_error(it, ls.err, level, kErrTooLarge);
    return;
  }
  const int wc = min(NC, nb - c0);
  const int nt = (m + 15) >> 4;
  const int nr = 16 * nt;
  double* Bs = lds;                          // nr x kTrsmInvLdB
  double* red = Bs + 256 * kTrsmInvLdB;      // 16 x 32
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane >> 4, lc = lane & 15;
  double* B = it.P + (size_t)m * (m + c0);
  const double* Gi = it.Gi;
  {
    const int n = nr * NC;
    for (int e0 = tid; e0 < n; e0 += 512 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 512;
        const int c = e / nr, r = e - c * nr;
        v[u] = (e < n && r < m && c < wc) ? gload(B + r + (size_t)m * c) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 512;
        const int c = e / nr, r = e - c * nr;
        if (e < n) Bs[r * kTrsmInvLdB + c] = v[u];
      }
    }
  }
  lds_barrier();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = h == 0 ? w : 15 - w;
    if (i >= nt) continue;
    d4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    const int gr = 16 * i + lc;
    for (int k0 = 0; k0 <= i; k0 += 8) {
      double av[8][4];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int gk = 16 * (k0 + kk) + 4 * s4 + lr;
          av[kk][s4] = (k0 + kk <= i && gr < m && gk < m && gk <= gr) ? gload(Gi + gr + (size_t)m * gk) : 0.0;
        }
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        if (k0 + kk > i) break;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const double* br = Bs + (16 * (k0 + kk) + 4 * s4 + lr) * kTrsmInvLdB;
          acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk][s4], br[lc], acc0, 0, 0, 0);
          if constexpr (NC == 32)
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk][s4], br[16 + lc], acc1, 0, 0, 0);
        }
      }
    }
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * i + 4 * v + lr;
      if (r < m) {
        if (lc < wc) gstore(B + r + (size_t)m * lc, acc0[v]);
        s0 += acc0[v] * acc0[v];
        if constexpr (NC == 32) {
          if (16 + lc < wc) gstore(B + r + (size_t)m * (16 + lc), acc1[v]);
          s1 += acc1[v] * acc1[v];
        }
      }
    }
    s0 += __shfl_xor(s0, 16, 64);
    s0 += __shfl_xor(s0, 32, 64);
    s1 += __shfl_xor(s1, 16, 64);
    s1 += __shfl_xor(s1, 32, 64);
    if (lr == 0) {
      red[i * 32 + lc] = s0;
      if constexpr (NC == 32) red[i * 32 + 16 + lc] = s1;
    }
  }
  lds_barrier();
  if (tid < wc && c0 + tid >= a) {
    double t = 0.0;
    for (int i = 0; i < nt; ++i) t += red[i * 32 + tid];
    gstore(it.norms + c0 + tid - a, t);
  }
}

// ---------------------------------------------------------------------------
// B <- G^{-1} B for BW columns of [A_sn | A_sw] per workgroup.  B chunk and a
// BW-wide panel of G are staged in LDS (rows padded to BW+1).  The diagonal
// block is solved wave-locally (each wave owns BW/4 columns, each column
// spread over 256/BW lanes); the rows below are updated with
// v_mfma_f64_16x16x4.
template <int BW>
__global__ void __launch_bounds__(256) trsm_kernel(const ItemD* __restrict__ items, LevelState ls) {
  extern __shared__ double lds[];
  const ItemD& it = items[blockIdx.x];
  const int m = it.m;
  if (m == 0) return;
  const int a = ls.a[it.s], nb = a + ls.b[it.s];
  const int c0 = blockIdx.y * BW;
  if (c0 >= nb) return;
  const int w = min(BW, nb - c0);
  constexpr int LDB = BW + 1;
  constexpr int LPC = 256 / BW;       // lanes per column in the diagonal solve
  constexpr int RPL = BW / LPC;       // rows of the diagonal block per lane
  double* Bs = lds;
  double* Gs = lds + (size_t)m * LDB;
  const double* G = it.P;
  double* B = it.P + (size_t)m * (m + c0);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  load_block_rowmajor<256>(Bs, LDB, B, (size_t)m, m, BW, [&](int, int c) { return c < w; });
  __syncthreads();
  const int col = wv * (BW / 4) + lane / LPC;  // diagonal-solve column of this lane
  const int g = lane % LPC;                    // its row group
  for (int jb = 0; jb < m; jb += BW) {
    const int jw = min(BW, m - jb);
    const int rows = m - jb;
    load_block_rowmajor<256>(Gs, LDB, G + (size_t)jb * m + jb, (size_t)m, rows, BW,
                             [&](int r, int c) { return c < jw && c <= r; });
    __syncthreads();
    {
      double x[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = g + LPC * t;
        x[t] = (r < jw) ? Bs[(jb + r) * LDB + col] : 0.0;
      }
      for (int u = 0; u < jw; ++u) {
        const int tu = u / LPC, gu = u % LPC;
        double own = x[0];
#pragma unroll
        for (int t = 1; t < RPL; ++t)
          if (t == tu) own = x[t];
        const double xu = __shfl(own, (lane / LPC) * LPC + gu, 64) / Gs[u * LDB + u];
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int r = g + LPC * t;
          if (r == u) x[t] = xu;
          else if (r > u && r < jw) x[t] -= Gs[r * LDB + u] * xu;
        }
      }
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = g + LPC * t;
        if (r < jw) Bs[(jb + r) * LDB + col] = x[t];
      }
    }
    __syncthreads();
    const int rb = rows - jw;
    const int nrt = (rb + 15) >> 4;
    constexpr int nct = BW / 16;
    for (int t = wv; t < nrt * nct; t += 4) {
      const int R0 = (t % nrt) * 16, C0 = (t / nrt) * 16;
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
      const int ar = R0 + (lane & 15);
      for (int u0 = 0; u0 < jw; u0 += 4) {
        const int ka = u0 + (lane >> 4);
        const double av = (ar < rb && ka < jw) ? Gs[(jw + ar) * LDB + ka] : 0.0;
        const double bv = (ka < jw) ? Bs[(jb + ka) * LDB + C0 + (lane & 15)] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = R0 + mfma64_row(lane, i);
        if (r < rb) Bs[(jb + jw + r) * LDB + C0 + (lane & 15)] -= acc[i];
      }
    }
    __syncthreads();
  }
  store_block_rowmajor<256>(B, (size_t)m, Bs, LDB, m, w);
  for (int c = wv; c < w; c += 4) {
    const int pc = c0 + c;
    if (pc < a) continue;
    double s = 0.0;
    for (int r = lane; r < m; r += 64) {
      const double x = Bs[r * LDB + c];
      s += x * x;
    }
    s = wave_sum(s);
    if (lane == 0) it.norms[pc - a] = s;
  }
}

// ---------------------------------------------------------------------------
// Column-pivoted QR of the far-field block (same rules as the fused kernel).
// NT threads; column c belongs to wave (c / CPW) % NW, which streams it in
// and out with R rows per lane.  Per reflector: wave 0 picks the pivot from
// the norms in LDS, the pivot column's wave forms the reflector (it wrote the
// column itself, so it reads it back without a barrier) and stages it in LDS,
// every wave updates its columns and their norms.  The barriers order LDS
// only: no wave waits for the column stores of another.
template <int R, int NT>
__global__ void __launch_bounds__(NT) cpqr_kernel(const ItemD* __restrict__ items, LevelState ls,
                                                  double tol, int tol_mode, int level) {
  constexpr int NW = NT / 64, CPW = (R <= 4 ? 6 : (R <= 8 ? 3 : 2));
  extern __shared__ double lds[];
  __shared__ int s_best, s_code;
  __shared__ double s_rjj, s_tj;
  const ItemD& it = items[blockIdx.x];
  const int m = it.m;
  const int a = gload(ls.a + it.s), b = gload(ls.b + it.s);
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (m == 0 || b == 0) {
    if (tid == 0) gstore(ls.k + it.s, 0);
    return;
  }
  double* nrm = lds;                          // b
  double* vs = lds + b;                       // m
  int* stp = reinterpret_cast<int*>(vs + m);  // b
  double* W = it.P + (size_t)m * (m + a);
  for (int c = tid; c < b; c += NT) {
    nrm[c] = gload(it.norms + c);
    stp[c] = -1;
  }
  lds_barrier();
  const int kmax = min(m, b);
  double r00 = 0.0;  // wave 0 only
  int k = kmax;
  bool over = false;
  for (int j = 0; j < kmax; ++j) {
    if (wv == 0) {
      double mx = 0.0;
      for (int c = lane; c < b; c += 64)
        if (stp[c] < 0) mx = fmax(mx, nrm[c]);
      mx = wave_max_dpp(mx);
      const double thr = (1.0 - kTie) * mx;
      int best = INT_MAX;
      for (int c = lane; c < b; c += 64)
        if (stp[c] < 0 && nrm[c] >= thr) best = min(best, c);
      best = wave_min_dpp(best);
      int code = 0;
      double rjj = 0.0;
      if (best == INT_MAX) {  // only NaN norms left
        code = 1;
      } else {
        rjj = sqrt(nrm[best]);
        if (j == 0) r00 = rjj;
        const bool stop = (tol_mode == 0) ? (rjj <= tol * r00) : (rjj <= tol);
        if (stop || rjj == 0.0) code = 1;
        else if (j >= it.kcap) code = 2;  // rank beyond the capacity
      }
      if (lane == 0) {
        s_best = best;
        s_code = code;
        s_rjj = rjj;
      }
    }
    lds_barrier();
    const int code = __builtin_amdgcn_readfirstlane(s_code);
    if (code) {
      k = code == 2 ? it.kcap : j;
      over = code == 2;
      break;
    }
    const int best = __builtin_amdgcn_readfirstlane(s_best);
    if (wv == (best / CPW) % NW) {
      // reflector j from the pivot column: unit entry at row j, R_jj there
      const double rjj = s_rjj;
      double* x = W + (size_t)m * best;
      double xv[R];
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = lane + 64 * t;
        xv[t] = i < m ? gload(x + i) : 0.0;
      }
      double rest = 0.0, xj = 0.0;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = lane + 64 * t;
        if (i > j && i < m) rest += xv[t] * xv[t];
        xj = t == (j >> 6) ? xv[t] : xj;
      }
      rest = wave_sum(rest);
      const double alpha = readlane_d(xj, j & 63);
      double d, tj;
      if (alpha <= 0.0) {
        d = alpha - rjj;
        tj = (rjj - alpha) / rjj;
      } else {
        d = -rest / (alpha + rjj);
        tj = rest / (rjj * (rjj + alpha));
      }
      if (d == 0.0) tj = 0.0;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = lane + 64 * t;
        if (i < m) {
          double v = 0.0;
          if (i == j) v = 1.0;
          else if (i > j) v = (d != 0.0) ? xv[t] / d : 0.0;
          vs[i] = v;
          if (i == j) gstore(x + i, rjj);
          else if (i > j) gstore(x + i, v);
        }
      }
      if (lane == 0) {
        s_tj = tj;
        stp[best] = j;
        gstore(it.piv + j, best);
        gstore(it.tau + j, tj);
      }
    }
    lds_barrier();
    const double tj = s_tj;
    double vr[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = lane + 64 * t;
      vr[t] = (i >= j && i < m) ? vs[i] : 0.0;
    }
    for (int cb = wv * CPW; cb < b; cb += NW * CPW) {
      double y[CPW][R];
      bool act[CPW];
#pragma unroll
      for (int q = 0; q < CPW; ++q) {
        const int c = cb + q;
        act[q] = c < b && stp[c] < 0;
        const double* yc = W + (size_t)m * (act[q] ? c : best);
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = lane + 64 * t;
          y[q][t] = (act[q] && i >= j && i < m) ? gload(yc + i) : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < CPW; ++q) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) acc += vr[t] * y[q][t];
        const double f = tj * wave_sum(acc);
        if (!act[q]) continue;
        double* yc = W + (size_t)m * (cb + q);
        double nn = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = lane + 64 * t;
          if (i >= j && i < m) {
            const double nv = y[q][t] - f * vr[t];
            gstore(yc + i, nv);
            if (i > j) nn += nv * nv;
          }
        }
        nn = wave_sum(nn);
        if (lane == 0) nrm[cb + q] = nn;
      }
    }
    lds_barrier();
  }
  for (int c = tid; c < b; c += NT) gstore(it.stepof + c, stp[c]);
  if (tid == 0) gstore(ls.k + it.s, k);
  if ((over || k > it.kcap) && tid == 0) item_error(it, ls.err, level, kErrCapacity);
}

// ---------------------------------------------------------------------------
// C <- U^T C for kApplyqCols near-field columns per workgroup (one column
// per wave per pass, R rows per lane in registers); reflectors staged in LDS
// 16 at a time.  The workgroups with blockIdx.y >= ya take the columns of
// G^{-1} instead (clusters whose inverse was formed, k > 0): W = U^T G^{-1}
// replaces G^{-1} in Gi, so that a sweep applies U^T G^{-1} (forward) or its
// transpose G^{-T} U (backward) as one product; the entries of
// G^{-1} above its diagonal tiles are zeros not stored, read as zeros.
constexpr int kApplyqCols = 16;
template <int R>
__global__ void __launch_bounds__(256) applyq_kernel(const ItemD* __restrict__ items, LevelState ls, int ya) {
  extern __shared__ double lds[];
  const ItemD& it = items[blockIdx.x];
  const int m = it.m;
  const int k = min(gload(ls.k + it.s), it.kcap), a = gload(ls.a + it.s);
  const bool winv = (int)blockIdx.y >= ya;
  const int c0 = (winv ? (int)blockIdx.y - ya : (int)blockIdx.y) * kApplyqCols;
  if (m == 0 || k == 0 || c0 >= (winv ? m : a)) return;
  if (winv && (m > kInvMaxDofs || !it.Gi || gload(ls.giok + it.s) == 0)) return;
  const int c1 = min(winv ? m : a, c0 + kApplyqCols);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* Vs = lds;            // 16 x m
  double* ts = lds + 16 * m;   // 16
  int* pv = reinterpret_cast<int*>(ts + 16);  // 16
  const double* W = it.P + (size_t)m * (m + a);
  double* C = winv ? it.Gi : it.P + (size_t)m * m;
  for (int j0 = 0; j0 < k; j0 += 16) {
    const int nj = min(16, k - j0);
    if (j0 > 0) __syncthreads();
    if (tid < nj) {
      ts[tid] = gload(it.tau + j0 + tid);
      pv[tid] = gload(it.piv + j0 + tid);
    }
    lds_barrier();
    for (int e = tid; e < nj * m; e += 256) {
      const int jj = e / m, i = e - jj * m, j = j0 + jj;
      Vs[jj * m + i] = (i == j) ? 1.0 : (i > j ? gload(W + (size_t)m * pv[jj] + i) : 0.0);
    }
    lds_barrier();
    for (int cb = c0 + wv * 4; cb < c1; cb += 16) {
      double y[4][R];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = cb + q;
        // G^{-1}: rows above the diagonal tile of column c are zeros (first
        // pass only; later passes read the full column written by the first)
        const int i0 = (winv && j0 == 0) ? (c & ~15) : 0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = lane + 64 * t;
          y[q][t] = (c < c1 && i >= i0 && i < m) ? gload(C + (size_t)m * c + i) : 0.0;
        }
      }
      for (int jj = 0; jj < nj; ++jj) {
        const double* v = Vs + jj * m;
        double s[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double acc = 0.0;
#pragma unroll
          for (int t = 0; t < R; ++t) {
            const int i = lane + 64 * t;
            if (i < m) acc += v[i] * y[q][t];
          }
          s[q] = wave_sum(acc) * ts[jj];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int t = 0; t < R; ++t) {
            const int i = lane + 64 * t;
            if (i < m) y[q][t] -= s[q] * v[i];
          }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = cb + q;
        if (c >= c1) continue;
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = lane + 64 * t;
          if (i < m) gstore(C + (size_t)m * c + i, y[q][t]);
        }
      }
    }
  }
  // read by the sweeps (later kernels); the workgroups of this launch only
  // test giok for zero
  if (winv && c0 == 0 && tid == 0) ls.giok[it.s] = 2;
}

// ---------------------------------------------------------------------------
// Scatter of one Schur-update element W[rr][cc] (rr >= cc) to its block.
__device__ __forceinline__ void schur_put(const ItemD& it, int rr, int cc, double val, int32_t* err,
                                          int level) {
  const int sr = it.colseg[rr], sc = it.colseg[cc];
  const int nr = it.colnat[rr], nc = it.colnat[cc];
  const int i = min(sr, sc), j = max(sr, sc);
  const PairD& pd = it.pair[j * (j + 1) / 2 + i];
  int row, col;
  if (pd.diag) {
    row = max(nr, nc);
    col = min(nr, nc);
  } else {
    const bool r_rows = (sr == (pd.rows_from_j ? j : i));
    row = r_rows ? nr : nc;
    const int cn = r_rows ? nc : nr;
    col = pd.posmap ? pd.posmap[cn] : cn;
  }
  if (row < 0 || col < 0 || row >= pd.nrows || col >= pd.ncols) {
    item_error(it, err, level, kErrIndex);
    return;
  }
  pd.dst[(size_t)row + (size_t)pd.ld * col] -= val;
}

// X -= F^T F for one 32x32 lower tile of the a x a product; four waves own
// its 16x16 quadrants; the rows of F pass through LDS 64 at a time (16 loads
// in flight per thread).  PREC 0: fp64 MFMA; 1: fp32 inputs, fp32
// accumulate; 2: bf16 inputs (round to nearest even), fp32 accumulate.
constexpr int kSchurRows = 64;
template <int PREC>
__global__ void __launch_bounds__(256) schur_kernel(const ItemD* __restrict__ items, LevelState ls,
                                                    int level) {
  __shared__ double Fr[kSchurRows][33];
  __shared__ double Fc[kSchurRows][33];
  const ItemD& it = items[blockIdx.x];
  const int m = it.m;
  const int k = min(ls.k[it.s], it.kcap), a = ls.a[it.s];
  if (m <= k || a == 0) return;
  const int nt = (a + 31) >> 5;
  if ((int)blockIdx.y >= nt * (nt + 1) / 2) return;
  int R, Cq;
  tri_tile(blockIdx.y, nt, R, Cq);
  const int R0 = 32 * R, C0 = 32 * Cq;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int qr = wv >> 1, qc = wv & 1;
  const bool live = !(R == Cq && qr < qc);  // strictly upper quadrant of a diagonal tile
  const double* C = it.P + (size_t)m * m;
  d4_t acc64 = {0.0, 0.0, 0.0, 0.0};
  f4_t acc32 = {0.f, 0.f, 0.f, 0.f};
  for (int i0 = k; i0 < m; i0 += kSchurRows) {
    // 16 loads in flight per thread: column col of the tile pair, rows ii
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u;
      const int half = e >> 11, ee = e & 2047;
      const int col = ee >> 6, ii = ee & 63;
      const int gi = i0 + ii, gc = (half ? C0 : R0) + col;
      v[u] = (gi < m && gc < a) ? gload(C + (size_t)m * gc + gi) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u;
      const int half = e >> 11, ee = e & 2047;
      const int col = ee >> 6, ii = ee & 63;
      if (half) Fc[ii][col] = v[u];
      else Fr[ii][col] = v[u];
    }
    __syncthreads();
    // the row chunks of 16 in order, each as before (same accumulation order)
    const int nch = min(kSchurRows, ((m - i0 + 15) / 16) * 16);
    if (live) {
      const int ar = 16 * qr + (lane & 15), bc = 16 * qc + (lane & 15);
      for (int c16 = 0; c16 < nch; c16 += 16) {
        if (PREC == 0) {
#pragma unroll
          for (int kk = 0; kk < 16; kk += 4) {
            const int ka = c16 + kk + (lane >> 4);
            acc64 = __builtin_amdgcn_mfma_f64_16x16x4f64(Fr[ka][ar], Fc[ka][bc], acc64, 0, 0, 0);
          }
        } else if (PREC == 1) {
#pragma unroll
          for (int kk = 0; kk < 16; kk += 4) {
            const int ka = c16 + kk + (lane >> 4);
            acc32 = __builtin_amdgcn_mfma_f32_16x16x4f32((float)Fr[ka][ar], (float)Fc[ka][bc], acc32, 0, 0, 0);
          }
        } else {
          s4_t av, bv;
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int ka = c16 + 4 * (lane >> 4) + jj;
            const uint32_t ua = __float_as_uint(round_bf16((float)Fr[ka][ar]));
            const uint32_t ub = __float_as_uint(round_bf16((float)Fc[ka][bc]));
            av[jj] = (short)(ua >> 16);
            bv[jj] = (short)(ub >> 16);
          }
          acc32 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc32, 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  if (!live) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rr = R0 + 16 * qr + (PREC == 0 ? mfma64_row(lane, i) : mfma32_row(lane, i));
    const int cc = C0 + 16 * qc + (lane & 15);
    if (rr < a && cc < a && rr >= cc) {
      const double v = PREC == 0 ? acc64[i] : (double)acc32[i];
      schur_put(it, rr, cc, v, ls.err, level);
    }
  }
}

// ---------------------------------------------------------------------------
// Coarse row of s, written to the blocks that keep it; identity diagonal.
__global__ void __launch_bounds__(256) writeback_kernel(const ItemD* __restrict__ items, LevelState ls,
                                                        int level) {
  const ItemD& it = items[blockIdx.x];
  const int m = it.m;
  const int k = min(ls.k[it.s], it.kcap), a = ls.a[it.s], nb = a + ls.b[it.s];
  if (m == 0 || k == 0) return;
  const int tid = threadIdx.x;
  if (blockIdx.y == 0)
    for (int e = tid; e < k * k; e += 256) {
      const int r = e % k, c = e / k;
      it.D[(size_t)r + (size_t)m * c] = (r == c) ? 1.0 : 0.0;
    }
  const int c0 = blockIdx.y * 64;
  if (c0 >= nb) return;
  const int c1 = min(nb, c0 + 64);
  for (int e = tid; e < k * (c1 - c0); e += 256) {
    const int r = e % k, pc = c0 + e / k;
    const WbD& t = it.wb[it.colseg[pc]];
    const int cn = it.colnat[pc];
    double v = it.P[(size_t)r + (size_t)m * (m + pc)];
    if (pc >= a) {
      const int st = it.stepof[pc - a];
      if (st >= 0 && r > st) v = 0.0;
    }
    const int row = t.trans ? cn : r, col = t.trans ? r : cn;
    if (row >= t.nrows || col >= t.ncols) {
      item_error(it, ls.err, level, kErrIndex);
      continue;
    }
    t.dst[(size_t)row + (size_t)t.ld * col] = v;
  }
}

// ---------------------------------------------------------------------------
void launch_split_step(int step, const ItemD* items, int nitems, const SplitDims& d, LevelState ls,
                       int level, double tol, int tol_mode, int prec, hipStream_t st, int tile) {
  if (nitems <= 0) return;
  static bool lds_set = false;
  if (!lds_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(trsm_kernel<32>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(trsm_kernel<16>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(potrf_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(chol_inv_kernel<kInvWaves>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kInvLds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(trsm_inv_kernel<32>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTrsmInvLds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(trsm_inv_kernel<16>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTrsmInvLds);
    lds_set = true;
  }
  const int mm = d.max_m;
  switch (step) {
    case kSplitOffsets:
      hipLaunchKernelGGL(seg_offsets_kernel, dim3(nitems), dim3(256), (size_t)(d.max_nseg + 1) * 4, st,
                         items, ls, level);
      break;
    case kSplitGather:
      if (mm <= 256)
        hipLaunchKernelGGL(gather_panel_kernel<4>, dim3(nitems, (mm + d.max_pcap + 31) / 32), dim3(256), 0, st, items,
                           ls);
      else
        hipLaunchKernelGGL(gather_panel_kernel<kRegRows>, dim3(nitems, (mm + d.max_pcap + 31) / 32), dim3(256), 0, st,
                           items, ls);
      break;
    case kSplitPotrf:
      if (mm <= kInvMaxDofs)
        hipLaunchKernelGGL(chol_inv_kernel<kInvWaves>, dim3(nitems), dim3(kInvWaves * 64), kInvLds, st, items, ls,
                           level);
      else
        hipLaunchKernelGGL(potrf_kernel, dim3(nitems), dim3(512), (size_t)mm * 33 * 8, st, items, ls,
                           level);
      break;
    case kSplitTrsm:
      if (d.max_pcap <= 0) break;
      if (mm <= kInvMaxDofs && tile == kTileNarrow)
        hipLaunchKernelGGL(trsm_inv_kernel<16>, dim3(nitems, (d.max_pcap + 15) / 16), dim3(512), kTrsmInvLds, st,
                           items, ls, level);
      else if (mm <= kInvMaxDofs)
        hipLaunchKernelGGL(trsm_inv_kernel<32>, dim3(nitems, (d.max_pcap + 31) / 32), dim3(512), kTrsmInvLds, st,
                           items, ls, level);
      else if (mm <= 256)
        hipLaunchKernelGGL(trsm_kernel<32>, dim3(nitems, (d.max_pcap + 31) / 32), dim3(256),
                           (size_t)2 * mm * 33 * 8, st, items, ls);
      else
        hipLaunchKernelGGL(trsm_kernel<16>, dim3(nitems, (d.max_pcap + 15) / 16), dim3(256),
                           (size_t)2 * mm * 17 * 8, st, items, ls);
      break;
    case kSplitCpqr: {
      const size_t lds = (size_t)d.max_pcap * 12 + (size_t)mm * 8 + 64;
      if (mm <= 256)
        hipLaunchKernelGGL((cpqr_kernel<4, 1024>), dim3(nitems), dim3(1024), lds, st, items, ls, tol, tol_mode,
                           level);
      else
        hipLaunchKernelGGL((cpqr_kernel<8, 1024>), dim3(nitems), dim3(1024), lds, st, items, ls, tol, tol_mode,
                           level);
      break;
    }
    case kSplitApplyq: {
      // near-field columns, then (m <= kInvMaxDofs) the columns of G^{-1}
      const int ya = ((d.max_acap > 0 ? d.max_acap : 0) + kApplyqCols - 1) / kApplyqCols;
      if (mm <= kInvMaxDofs)
        hipLaunchKernelGGL(applyq_kernel<4>, dim3(nitems, ya + (mm + kApplyqCols - 1) / kApplyqCols), dim3(256),
                           ((size_t)16 * mm + 24) * 8, st, items, ls, ya);
      else if (ya > 0)
        hipLaunchKernelGGL(applyq_kernel<kRegRows>, dim3(nitems, ya), dim3(256), ((size_t)16 * mm + 24) * 8, st,
                           items, ls, ya);
      break;
    }
    case kSplitSchur: {
      if (d.max_acap <= 0) break;
      const int nt = (d.max_acap + 31) / 32;
      const dim3 g(nitems, nt * (nt + 1) / 2);
      if (prec == 0) hipLaunchKernelGGL(schur_kernel<0>, g, dim3(256), 0, st, items, ls, level);
      else if (prec == 1) hipLaunchKernelGGL(schur_kernel<1>, g, dim3(256), 0, st, items, ls, level);
      else hipLaunchKernelGGL(schur_kernel<2>, g, dim3(256), 0, st, items, ls, level);
      break;
    }
    case kSplitWriteback:
      hipLaunchKernelGGL(writeback_kernel, dim3(nitems, (d.max_pcap + 63) / 64 + 1), dim3(256), 0, st,
                         items, ls, level);
      break;
  }
}

}  // namespace lrsp
