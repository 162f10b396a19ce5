// kernels.hip -- gfx950 kernels of the deferred-compression hierarchical solver.
//
// One workgroup (256 threads = 4 wave64) processes one cluster.  Clusters of
// one colour of the level's distance-2 colouring read and write disjoint
// blocks, so a colour is one launch with one workgroup per cluster.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include <hip/hip_cooperative_groups.h>

#include "desc.hpp"
#include "devutil.hpp"
#include "kernels.hpp"

namespace lrsp {

namespace {

constexpr int kWaves = kThreads / 64;
constexpr int kRegRows = kMaxClusterDofs / 64;  // column slots per lane
constexpr int kColM = 64;  // up to this many rows, column operations run one column per thread

__device__ __forceinline__ double block_sum(double v, double* sh) { return group_sum<kThreads>(v, sh); }
__device__ __forceinline__ double block_max(double v, double* sh) { return group_max<kThreads>(v, sh); }
__device__ __forceinline__ int block_min_int(int v, int* sh) { return group_min_int<kThreads>(v, sh); }

// ---------------------------------------------------------------------------
// Blocked right-looking Cholesky of the lower triangle of the m x m matrix A
// (ld), fused with the triangular solve B <- G^{-1} B of the nb columns B
// (same ld).  Pivots that are not > 0 raise *bad and are replaced by 1 so
// that the sweep stays finite.  LDS: m*kNB + kNB*kNB + kNB*256 doubles.
// TWO: the right-hand side is B (nb columns) followed by B2 (nb2 columns),
// two separate column ranges of the same ld.
template <bool TWO = false>
__device__ __forceinline__ void chol_solve(double* A, int ld, int m, double* B, int nb, double* lds, int* bad,
                                           double* B2 = nullptr, int nb2 = 0) {
  auto colp = [&](int c) -> double* {
    if constexpr (TWO) {
      if (c >= nb) return B2 + (size_t)ld * (c - nb);
    }
    return B + (size_t)ld * c;
  };
  const int nbt = TWO ? nb + nb2 : nb;
  double* Lp = lds;                // (m) x kNB, row-major
  double* Dg = Lp + (size_t)m * kNB;  // kNB x kNB, row-major
  double* Bb = Dg + kNB * kNB;     // kNB x 256, row-major
  const int tid = threadIdx.x;
  for (int jb = 0; jb < m; jb += kNB) {
    const int w = min(kNB, m - jb);
    // (a) factor the diagonal block with wave 0 (lane t holds row t)
    if (tid < 64) {
      double row[kNB];
#pragma unroll
      for (int u = 0; u < kNB; ++u)
        row[u] = (tid < w && u <= tid) ? A[(size_t)(jb + tid) + (size_t)ld * (jb + u)] : 0.0;
#pragma unroll
      for (int u = 0; u < kNB; ++u) {
        if (u < w) {
          double d = readlane_d(row[u], u);
          if (!(d > 0.0)) {
            if (tid == 0) *bad = 1;
            d = 1.0;
          }
          d = sqrt(d);
          if (tid == u) row[u] = d;
          else if (tid > u) row[u] = row[u] / d;
#pragma unroll
          for (int v = u + 1; v < kNB; ++v) {
            const double lvu = readlane_d(row[u], v);
            if (v < w && tid >= v && tid < w) row[v] -= row[u] * lvu;
          }
        }
      }
      if (tid < kNB) {
#pragma unroll
        for (int u = 0; u < kNB; ++u) Dg[tid * kNB + u] = (tid < w && u <= tid) ? row[u] : 0.0;
      }
      if (tid < w) {
#pragma unroll
        for (int u = 0; u < kNB; ++u)
          if (u <= tid) A[(size_t)(jb + tid) + (size_t)ld * (jb + u)] = row[u];
      }
    }
    __syncthreads();
    // (b) panel rows below the diagonal block: x L11^T = a
    const int rem = m - jb - w;
    for (int i = tid; i < rem; i += kThreads) {
      const int gi = jb + w + i;
      double x[kNB];
#pragma unroll
      for (int u = 0; u < kNB; ++u) x[u] = (u < w) ? A[(size_t)gi + (size_t)ld * (jb + u)] : 0.0;
#pragma unroll
      for (int u = 0; u < kNB; ++u) {
        if (u < w) {
          double s = x[u];
#pragma unroll
          for (int v = 0; v < u; ++v) s -= Dg[u * kNB + v] * x[v];
          x[u] = s / Dg[u * kNB + u];
        }
      }
#pragma unroll
      for (int u = 0; u < kNB; ++u) {
        Lp[(size_t)i * kNB + u] = x[u];
        if (u < w) A[(size_t)gi + (size_t)ld * (jb + u)] = x[u];
      }
    }
    __syncthreads();
    // (c) right-hand block: rows jb..jb+w of B, then the rows below
    for (int c0 = 0; c0 < nbt; c0 += 256) {
      const int c = c0 + tid;
      if (c < nbt) {
        double* Bc = colp(c);
        double x[kNB];
#pragma unroll
        for (int u = 0; u < kNB; ++u) x[u] = (u < w) ? Bc[jb + u] : 0.0;
#pragma unroll
        for (int u = 0; u < kNB; ++u) {
          if (u < w) {
            double s = x[u];
#pragma unroll
            for (int v = 0; v < u; ++v) s -= Dg[u * kNB + v] * x[v];
            x[u] = s / Dg[u * kNB + u];
          }
        }
#pragma unroll
        for (int u = 0; u < kNB; ++u) {
          Bb[u * 256 + tid] = x[u];
          if (u < w) Bc[jb + u] = x[u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < kNB; ++u) Bb[u * 256 + tid] = 0.0;
      }
      __syncthreads();
      const int ncol = min(256, nbt - c0);
      const int nR = (rem + 3) >> 2, nC = (ncol + 3) >> 2;
      for (int idx = tid; idx < nR * nC; idx += kThreads) {
        const int R = idx % nR, C = idx / nR;
        double acc[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[r][q] = 0.0;
        for (int u = 0; u < w; ++u) {
          double lr[4], bc[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) lr[r] = (4 * R + r < rem) ? Lp[(size_t)(4 * R + r) * kNB + u] : 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) bc[q] = Bb[u * 256 + 4 * C + q];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[r][q] += lr[r] * bc[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int cc = c0 + 4 * C + q;
          if (4 * C + q < ncol) {
            double* Bc = colp(cc);
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (4 * R + r < rem) Bc[jb + w + 4 * R + r] -= acc[r][q];
          }
        }
      }
      __syncthreads();
    }
    // (d) trailing update of the lower triangle of A
    const int nt = (rem + 3) >> 2;
    const int ntiles = nt * (nt + 1) / 2;
    for (int idx = tid; idx < ntiles; idx += kThreads) {
      int R, C;
      tri_tile(idx, nt, R, C);
      double acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = 0.0;
      for (int u = 0; u < w; ++u) {
        double lr[4], lc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) lr[r] = (4 * R + r < rem) ? Lp[(size_t)(4 * R + r) * kNB + u] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) lc[q] = (4 * C + q < rem) ? Lp[(size_t)(4 * C + q) * kNB + u] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[r][q] += lr[r] * lc[q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cc = 4 * C + q;
        if (cc < rem) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rr = 4 * R + r;
            if (rr < rem && rr >= cc)
              A[(size_t)(jb + w + rr) + (size_t)ld * (jb + w + cc)] -= acc[r][q];
          }
        }
      }
    }
    __syncthreads();
  }
}

// Column-pivoted Householder QR of the m x b far-field block W (ld), truncated
// at the first pivot with R_jj <= tol*R_00 (relative) or <= tol (absolute).
// Pivot: lowest column among those with squared norm >= (1-kTie)*max.
// Reflector j lives in column piv[j] (rows j+1.., unit leading entry); R_jj
// >= 0 sits at row j of that column; other columns hold R in rows < k.
// At most kcap reflectors are stored: when pivot kcap does not meet the stop
// rule, *over is set and kcap is returned.
__device__ __forceinline__ int cpqr(double* W, int ld, int m, int b, double tol, int tol_mode, int kcap, int* piv,
                    int* stepof, double* tau, double* norms, double* shd, int* shi, bool* over) {
  __shared__ double vsh[kColM];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // m <= kColM: one column per thread (its rows loaded together); else one
  // column per wave
  const bool bycol = m <= kColM;
  if (bycol) {
    for (int c = tid; c < b; c += kThreads) {
      const double* y = W + (size_t)ld * c;
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += y[i] * y[i];
      norms[c] = s;
      stepof[c] = -1;
    }
  } else {
    for (int c = wv; c < b; c += kWaves) {
      const double* y = W + (size_t)ld * c;
      double s = 0.0;
      for (int i = lane; i < m; i += 64) s += y[i] * y[i];
      s = wave_sum(s);
      if (lane == 0) {
        norms[c] = s;
        stepof[c] = -1;
      }
    }
  }
  __syncthreads();
  const int kmax = min(m, b);
  double r00 = 0.0;
  int k = kmax;
  for (int j = 0; j < kmax; ++j) {
    double mx = 0.0;
    for (int c = tid; c < b; c += kThreads)
      if (stepof[c] < 0) mx = fmax(mx, norms[c]);
    mx = block_max(mx, shd);
    const double thr = (1.0 - kTie) * mx;
    int best = INT_MAX;
    for (int c = tid; c < b; c += kThreads)
      if (stepof[c] < 0 && norms[c] >= thr) best = min(best, c);
    best = block_min_int(best, shi);
    if (best == INT_MAX) {  // only NaN norms left
      k = j;
      break;
    }
    const double n2 = norms[best];
    const double rjj = sqrt(n2);
    if (j == 0) r00 = rjj;
    const bool stop = (tol_mode == 0) ? (rjj <= tol * r00) : (rjj <= tol);
    if (stop || rjj == 0.0) {
      k = j;
      break;
    }
    if (j >= kcap) {
      k = kcap;
      *over = true;
      break;
    }
    double* x = W + (size_t)ld * best;
    const double alpha = x[j];
    double rest = 0.0;
    for (int i = j + 1 + tid; i < m; i += kThreads) rest += x[i] * x[i];
    rest = block_sum(rest, shd);
    double d, tj;
    if (alpha <= 0.0) {
      d = alpha - rjj;
      tj = (rjj - alpha) / rjj;
    } else {
      d = -rest / (alpha + rjj);
      tj = rest / (rjj * (rjj + alpha));
    }
    if (d == 0.0) tj = 0.0;
    __syncthreads();
    if (d != 0.0)
      for (int i = j + 1 + tid; i < m; i += kThreads) x[i] = x[i] / d;
    if (tid == 0) {
      x[j] = rjj;
      piv[j] = best;
      stepof[best] = j;
      tau[j] = tj;
    }
    __syncthreads();
    if (bycol) {
      // apply H_j to the remaining columns, one per thread, v in LDS
      if (tid < m) vsh[tid] = tid == j ? 1.0 : (tid > j ? x[tid] : 0.0);
      __syncthreads();
      for (int c = tid; c < b; c += kThreads) {
        if (stepof[c] >= 0) continue;
        double* y = W + (size_t)ld * c;
        double s = 0.0;
        for (int i = j; i < m; ++i) s += vsh[i] * y[i];
        const double f = tj * s;
        double nn = 0.0;
        for (int i = j; i < m; ++i) {
          const double nv = y[i] - f * vsh[i];
          y[i] = nv;
          if (i > j) nn += nv * nv;
        }
        norms[c] = nn;
      }
      __syncthreads();
      continue;
    }
    // apply H_j to the remaining columns and recompute their norms below row j
    double v[kRegRows];
#pragma unroll
    for (int t = 0; t < kRegRows; ++t) {
      const int i = lane + 64 * t;
      v[t] = (i > j && i < m) ? x[i] : (i == j ? 1.0 : 0.0);
    }
    for (int c = wv; c < b; c += kWaves) {
      if (stepof[c] >= 0) continue;
      double* y = W + (size_t)ld * c;
      double yr[kRegRows];
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < kRegRows; ++t) {
        const int i = lane + 64 * t;
        yr[t] = (i >= j && i < m) ? y[i] : 0.0;
        s += v[t] * yr[t];
      }
      s = wave_sum(s);
      const double f = tj * s;
      double nn = 0.0;
#pragma unroll
      for (int t = 0; t < kRegRows; ++t) {
        const int i = lane + 64 * t;
        if (i >= j && i < m) {
          const double nv = yr[t] - f * v[t];
          y[i] = nv;
          if (i > j) nn += nv * nv;
        }
      }
      nn = wave_sum(nn);
      if (lane == 0) norms[c] = nn;
    }
    __syncthreads();
  }
  return k;
}

// C <- U^T C for the a columns C (ld): reflectors 0..k-1 in order.  With
// m <= kColM and room in the LDS scratch (scr doubles at lds), the
// reflectors are staged in LDS and C passes through it in chunks of
// columns (row-major in the chunk, so that the column of each thread is
// conflict-free), every column rotated by its own thread; else one column
// per wave from global memory.
__device__ __forceinline__ void apply_qt_cols(double* C, int ld, int m, int a, const double* W, const int* piv,
                              const double* tau, int k, double* lds, size_t scr) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (m <= kColM && scr >= (size_t)(k + 1) * m + k) {
    double* V = lds;                  // k x m, V[j*m + i]
    double* ts = V + (size_t)k * m;   // k
    double* Cs = ts + k;              // m x cw, Cs[i*cw + c]
    const int cw = (int)min<size_t>((size_t)a, (scr - (size_t)k * m - k) / m);
    const int nv = k * m;
    for (int e0 = tid; e0 < nv; e0 += kThreads * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads;
        v[u] = 0.0;
        if (e < nv) {
          const int j = e / m, i = e - j * m;
          v[u] = i == j ? 1.0 : (i > j ? W[(size_t)i + (size_t)ld * piv[j]] : 0.0);
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads;
        if (e < nv) V[e] = v[u];
      }
    }
    for (int j = tid; j < k; j += kThreads) ts[j] = tau[j];
    for (int c0 = 0; c0 < a; c0 += cw) {
      const int nc = min(cw, a - c0), ne = nc * m;
      double* Cg = C + (size_t)ld * c0;
      for (int e0 = tid; e0 < ne; e0 += kThreads * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * kThreads;
          v[u] = 0.0;
          if (e < ne) {
            const int c = e / m, i = e - c * m;
            v[u] = Cg[(size_t)i + (size_t)ld * c];
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * kThreads;
          if (e < ne) {
            const int c = e / m, i = e - c * m;
            Cs[(size_t)i * cw + c] = v[u];
          }
        }
      }
      __syncthreads();
      for (int c = tid; c < nc; c += kThreads) {
        double* y = Cs + c;
        for (int j = 0; j < k; ++j) {
          const double* v = V + (size_t)j * m;
          double s = 0.0;
          for (int i = j; i < m; ++i) s += v[i] * y[(size_t)i * cw];
          const double f = ts[j] * s;
          for (int i = j; i < m; ++i) y[(size_t)i * cw] -= f * v[i];
        }
      }
      __syncthreads();
      for (int e = tid; e < ne; e += kThreads) {
        const int c = e / m, i = e - c * m;
        Cg[(size_t)i + (size_t)ld * c] = Cs[(size_t)i * cw + c];
      }
      __syncthreads();
    }
    return;
  }
  for (int c = wv; c < a; c += kWaves) {
    double* y = C + (size_t)ld * c;
    double yr[kRegRows];
#pragma unroll
    for (int t = 0; t < kRegRows; ++t) {
      const int i = lane + 64 * t;
      yr[t] = (i < m) ? y[i] : 0.0;
    }
    for (int j = 0; j < k; ++j) {
      const double* x = W + (size_t)ld * piv[j];
      double v[kRegRows];
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < kRegRows; ++t) {
        const int i = lane + 64 * t;
        v[t] = (i > j && i < m) ? x[i] : (i == j ? 1.0 : 0.0);
        s += v[t] * yr[t];
      }
      s = wave_sum(s);
      const double f = tau[j] * s;
#pragma unroll
      for (int t = 0; t < kRegRows; ++t) yr[t] -= f * v[t];
    }
#pragma unroll
    for (int t = 0; t < kRegRows; ++t) {
      const int i = lane + 64 * t;
      if (i < m) y[i] = yr[t];
    }
  }
}

// Owning-block entry of the Schur element (rr, cc), cc <= rr, of the
// near-field columns; null, after recording the error, when out of range.
__device__ __forceinline__ double* schur_target(const ItemD& it, int rr, int cc, int32_t* err, int level) {
  const int sr = it.colseg[rr], sc = it.colseg[cc];
  const int nr = it.colnat[rr], nc = it.colnat[cc];
  const int i = min(sr, sc), j = max(sr, sc);
  const PairD& pd = it.pair[j * (j + 1) / 2 + i];
  int row, col;
  if (pd.diag) {
    row = max(nr, nc);
    col = min(nr, nc);
  } else {
    const bool r_is_rowseg = (sr == (pd.rows_from_j ? j : i));
    row = r_is_rowseg ? nr : nc;
    const int cn = r_is_rowseg ? nc : nr;
    col = pd.posmap ? pd.posmap[cn] : cn;
  }
  if (row < 0 || col < 0 || row >= pd.nrows || col >= pd.ncols) {
    item_error(it, err, level, kErrIndex);
    return nullptr;
  }
  return pd.dst + (size_t)row + (size_t)pd.ld * col;
}

// Schur update X -= F^T F, F = rows k..m-1 of the a near-field columns C (ld).
// Each unordered column pair (r >= c) is computed once and scattered to the
// one block that owns it.
__device__ __forceinline__ void schur_scatter(const ItemD& it, const double* C, int ld, int m, int k, int a, int prec,
                              int32_t* err, int level) {
  const int tid = threadIdx.x;
  const int nt = (a + 3) >> 2;
  const int ntiles = nt * (nt + 1) / 2;
  for (int idx = tid; idx < ntiles; idx += kThreads) {
    int R, Cc;
    tri_tile(idx, nt, R, Cc);
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[r][q] = 0.0;
    if (prec == 0) {
      for (int i = k; i < m; ++i) {
        double fr[4], fc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) fr[r] = (4 * R + r < a) ? C[(size_t)i + (size_t)ld * (4 * R + r)] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) fc[q] = (4 * Cc + q < a) ? C[(size_t)i + (size_t)ld * (4 * Cc + q)] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[r][q] += fr[r] * fc[q];
      }
    } else {
      float accf[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) accf[r][q] = 0.0f;
      for (int i = k; i < m; ++i) {
        float fr[4], fc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float t = (4 * R + r < a) ? (float)C[(size_t)i + (size_t)ld * (4 * R + r)] : 0.0f;
          fr[r] = prec == 2 ? round_bf16(t) : t;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float t = (4 * Cc + q < a) ? (float)C[(size_t)i + (size_t)ld * (4 * Cc + q)] : 0.0f;
          fc[q] = prec == 2 ? round_bf16(t) : t;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) accf[r][q] = fmaf(fr[r], fc[q], accf[r][q]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = (double)accf[r][q];
    }
    // all targets first, then all loads, then all stores: sixteen
    // read-modify-writes in flight instead of one after the other
    double* t[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = 4 * R + r, cc = 4 * Cc + q;
        t[r][q] = (rr < a && cc < a && cc <= rr) ? schur_target(it, rr, cc, err, level) : nullptr;
      }
    double old[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) old[r][q] = t[r][q] ? *t[r][q] : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (t[r][q]) *t[r][q] = old[r][q] - acc[r][q];
  }
}

// Staged form of schur_scatter for small panels: F (rows k..m-1 of the a
// columns), the segment and natural index of every column and the pair table
// of the near segments pass through the LDS scratch (scr doubles at lds) in
// one element-parallel copy; each thread then forms its 4x4 tile from LDS
// (same products in the same order as the global form) and resolves its
// targets eight at a time, their posmap loads, old values and stores each
// issued together.  Returns false, doing nothing, when the staging does not fit.
__device__ __forceinline__ bool schur_scatter_staged(const ItemD& it, const double* C, int ld, int m, int k, int a, int prec,
                                     int32_t* err, int level, double* lds, size_t scr) {
  const int tid = threadIdx.x;
  const int nf = m - k;
  const int nsn = it.nsegn;
  const int np = nsn * (nsn + 1) / 2;
  constexpr int kPairD = (int)(sizeof(PairD) / sizeof(double));
  static_assert(sizeof(PairD) % sizeof(double) == 0, "PairD is staged as doubles");
  const size_t need = (size_t)nf * a + (size_t)a + (size_t)kPairD * np + 1;
  if (need > scr) return false;
  double* Fs = lds;                                               // nf x a, ld nf
  int32_t* cs = reinterpret_cast<int32_t*>(Fs + (size_t)nf * a);  // a
  int32_t* cn = cs + a;                                           // a
  PairD* ps = reinterpret_cast<PairD*>(Fs + (size_t)nf * a + a);  // np
  double* dummy = reinterpret_cast<double*>(ps + np);
  {
    const int nF = nf * a;
    for (int e0 = tid; e0 < nF; e0 += kThreads * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads;
        const int c = e / max(nf, 1), r = e - c * nf;
        v[u] = e < nF ? C[(size_t)(k + r) + (size_t)ld * c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads;
        if (e < nF) Fs[e] = v[u];
      }
    }
    for (int c = tid; c < a; c += kThreads) {
      cs[c] = it.colseg[c];
      cn[c] = it.colnat[c];
    }
    const double* src = reinterpret_cast<const double*>(it.pair);
    double* dst = reinterpret_cast<double*>(ps);
    for (int e0 = tid; e0 < kPairD * np; e0 += kThreads * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads;
        v[u] = e < kPairD * np ? src[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads;
        if (e < kPairD * np) dst[e] = v[u];
      }
    }
    if (tid == 0) *dummy = 0.0;
  }
  __syncthreads();
  const int nt = (a + 3) >> 2;
  const int ntiles = nt * (nt + 1) / 2;
  for (int idx = tid; idx < ntiles; idx += kThreads) {
    int R, Cc;
    tri_tile(idx, nt, R, Cc);
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[r][q] = 0.0;
    if (prec == 0) {
      for (int i = 0; i < nf; ++i) {
        double fr[4], fc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) fr[r] = (4 * R + r < a) ? Fs[i + (size_t)nf * (4 * R + r)] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) fc[q] = (4 * Cc + q < a) ? Fs[i + (size_t)nf * (4 * Cc + q)] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[r][q] += fr[r] * fc[q];
      }
    } else {
      float accf[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) accf[r][q] = 0.0f;
      for (int i = 0; i < nf; ++i) {
        float fr[4], fc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float t = (4 * R + r < a) ? (float)Fs[i + (size_t)nf * (4 * R + r)] : 0.0f;
          fr[r] = prec == 2 ? round_bf16(t) : t;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float t = (4 * Cc + q < a) ? (float)Fs[i + (size_t)nf * (4 * Cc + q)] : 0.0f;
          fc[q] = prec == 2 ? round_bf16(t) : t;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) accf[r][q] = fmaf(fr[r], fc[q], accf[r][q]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = (double)accf[r][q];
    }
    // targets, eight at a time: pair and row from LDS, column through the
    // pair's posmap
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int pi[8], row[8], cidx[8];
      bool ok[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int rr = 4 * R + 2 * h + (e >> 2), cc = 4 * Cc + (e & 3);
        ok[e] = rr < a && cc < a && cc <= rr;
        const int rs = ok[e] ? rr : 0, csn = ok[e] ? cc : 0;
        const int sr = cs[rs], sc = cs[csn], nr = cn[rs], ncn = cn[csn];
        const int i = min(sr, sc), j = max(sr, sc);
        pi[e] = j * (j + 1) / 2 + i;
        const bool diag = ps[pi[e]].diag != 0;
        const bool r_is_rowseg = (sr == (ps[pi[e]].rows_from_j ? j : i));
        row[e] = diag ? max(nr, ncn) : (r_is_rowseg ? nr : ncn);
        cidx[e] = diag ? min(nr, ncn) : (r_is_rowseg ? ncn : nr);
      }
      int col[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int32_t* pm = ps[pi[e]].diag ? nullptr : ps[pi[e]].posmap;
        col[e] = *(pm ? pm + cidx[e] : it.colnat);
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int32_t* pm = ps[pi[e]].diag ? nullptr : ps[pi[e]].posmap;
        if (!pm) col[e] = cidx[e];
      }
      double* t[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const PairD& pd = ps[pi[e]];
        t[e] = nullptr;
        if (ok[e]) {
          if (row[e] < 0 || col[e] < 0 || row[e] >= pd.nrows || col[e] >= pd.ncols) item_error(it, err, level, kErrIndex);
          else t[e] = pd.dst + (size_t)row[e] + (size_t)pd.ld * col[e];
        }
      }
      double old[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) old[e] = *(t[e] ? t[e] : dummy);
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (t[e]) *t[e] = old[e] - acc[2 * h + (e >> 2)][e & 3];
    }
  }
  __syncthreads();
  return true;
}

// Widths of the column segments (coarse ones are earlier ranks), their
// exclusive prefix sum into soff[0..nseg] (LDS) and it.segoff, and the near
// and far widths.  Returns false (after recording the error) when a width
// exceeds its capacity.  Its barriers order LDS only (it.segoff is not read
// by the elimination that follows).
__device__ __forceinline__ bool seg_scan(const ItemD& it, LevelState ls, int level, int* soff, int* wsum, int* flag,
                         int& a_out, int& b_out) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nseg = it.nseg;
  if (tid == 0) *flag = 0;
  lds_barrier();
  int carry = 0;
  for (int base = 0; base < nseg; base += kThreads) {
    const int i = base + tid;
    int w = 0;
    if (i < nseg) {
      const SegD* sg = it.seg + i;
      const int coarse = gload(&sg->coarse), y = gload(&sg->y), nfine = gload(&sg->nfine), cap = gload(&sg->cap);
      w = coarse ? gload(ls.k + y) : nfine;
      if (w < 0 || w > cap) {
        *flag = 1;
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
    lds_barrier();
    int pre = 0;
    for (int q = 0; q < wv; ++q) pre += wsum[q];
    int tot = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) tot += wsum[q];
    if (i < nseg) soff[i] = carry + pre + x - w;
    carry += tot;
    lds_barrier();
  }
  if (tid == 0) soff[nseg] = carry;
  lds_barrier();
  a_out = soff[it.nsegn];
  b_out = soff[nseg] - a_out;
  const bool bad = *flag || soff[nseg] > it.pcap;
  for (int i = tid; i <= nseg; i += kThreads) gstore(it.segoff + i, soff[i]);
  if (bad && tid == 0) item_error(it, ls.err, level, kErrCapacity);
  lds_barrier();
  return !bad;
}

// ---------------------------------------------------------------------------
// Clusters of at most kTinyM DoFs whose block row fits kTinyLdsBytes of LDS:
// the block row [A_ss | A_sn | A_sw] is gathered once into LDS and every
// step works on that copy.  The Cholesky and the pivoted QR (serial chains)
// run in wave 0 with cross-lane register exchanges; the scaling and the
// rotation take one column per thread of the workgroup; phases exchange data
// through LDS-only barriers.  The pivot, tie and stop rules are those of
// cpqr.  Whether a cluster takes this form depends on its sizes alone, so
// every schedule gives it the same arithmetic.
constexpr int kTinyM = 32;
constexpr size_t kTinyLdsBytes = 64 * 1024;

// LDS scratch (doubles) of the per-cluster elimination for clusters of at
// most max_m DoFs: the blocked Cholesky's panels, and room for the
// small-cluster form.
__host__ __device__ __forceinline__ size_t slre_scratch(int max_m) {
  const size_t chol = (size_t)max_m * kNB + kNB * kNB + kNB * 256;
  return chol > kTinyLdsBytes / 8 ? chol : kTinyLdsBytes / 8;
}

// Orders LDS accesses of the lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ __forceinline__ size_t tiny_al(size_t x) { return (x + 15) & ~(size_t)15; }

// Byte offsets of the LDS sections of the small-cluster form (the pair
// descriptors last).
struct TinyLayout {
  int ldp;  // odd leading dimension of the panel copy
  size_t p, src, nrm, tau, cseg, cnat, stp, piv, wb, pair, end, end_pairs;
};

__host__ __device__ __forceinline__ TinyLayout tiny_layout(int m, int a, int b, int nseg, int np) {
  TinyLayout L;
  const size_t nc = (size_t)m + a + b;
  L.ldp = m | 1;
  L.p = 0;
  L.src = L.p + tiny_al(8 * (size_t)L.ldp * nc);
  L.nrm = L.src + tiny_al(8 * nc);
  L.tau = L.nrm + tiny_al(8 * (size_t)b);
  L.cseg = L.tau + tiny_al(8 * (size_t)kTinyM);
  L.cnat = L.cseg + tiny_al(4 * ((size_t)a + b));
  L.stp = L.cnat + tiny_al(4 * ((size_t)a + b));
  L.piv = L.stp + tiny_al(4 * (size_t)b);
  L.wb = L.piv + tiny_al(4 * (size_t)kTinyM);
  L.pair = L.wb + tiny_al(sizeof(WbD) * (size_t)nseg);
  L.end = L.pair;
  L.end_pairs = L.pair + tiny_al(sizeof(PairD) * (size_t)np);
  return L;
}

__device__ __forceinline__ bool tiny_fits(int m, int a, int b, int nseg, int nsegn) {
  return m <= kTinyM && tiny_layout(m, a, b, nseg, nsegn * (nsegn + 1) / 2).end_pairs <= kTinyLdsBytes;
}

// Cholesky of the m x m lower triangle of the panel copy (ld ldp) by one
// wave, lane i holding row i; pivots that are not > 0 set bad and are
// replaced by 1.
template <int MB>
__device__ __forceinline__ void tiny_chol(double* Ps, int ldp, int m, int lane, bool& bad) {
  double row[MB];
#pragma unroll
  for (int u = 0; u < MB; ++u) row[u] = (lane < m && u <= lane) ? Ps[lane + ldp * u] : 0.0;
#pragma unroll
  for (int u = 0; u < MB; ++u) {
    if (u < m) {
      double d = readlane_d(row[u], u);
      if (!(d > 0.0)) {
        bad = true;
        d = 1.0;
      }
      d = sqrt(d);
      if (lane == u) row[u] = d;
      else if (lane > u) row[u] = row[u] / d;
#pragma unroll
      for (int v = u + 1; v < MB; ++v) {
        if (v < m) {
          const double lvu = readlane_d(row[u], v);
          if (lane >= v && lane < m) row[v] -= row[u] * lvu;
        }
      }
    }
  }
  if (lane < m) {
#pragma unroll
    for (int u = 0; u < MB; ++u)
      if (u <= lane) Ps[lane + ldp * u] = row[u];
  }
}

// x <- G^{-1} x for the a + b off-diagonal columns of the panel copy, one
// column per thread of the workgroup; squared norms of the far-field
// columns into nrm.
template <int MB>
__device__ __forceinline__ void tiny_scale(double* Ps, int ldp, int m, int a, int b, double* nrm, int* stp) {
  for (int c = threadIdx.x; c < a + b; c += kThreads) {
    double* y = Ps + (size_t)ldp * (m + c);
    double x[MB];
#pragma unroll
    for (int u = 0; u < MB; ++u) x[u] = u < m ? y[u] : 0.0;
#pragma unroll
    for (int u = 0; u < MB; ++u) {
      if (u < m) {
        double s = x[u];
#pragma unroll
        for (int v = 0; v < u; ++v) s -= Ps[u + ldp * v] * x[v];
        x[u] = s / Ps[u + ldp * u];
      }
    }
    double nn = 0.0;
#pragma unroll
    for (int u = 0; u < MB; ++u)
      if (u < m) {
        y[u] = x[u];
        nn += x[u] * x[u];
      }
    if (c >= a) {
      nrm[c - a] = nn;
      stp[c - a] = -1;
    }
  }
}

// Column-pivoted Householder QR of the b scaled far-field columns Wf (ld
// ldp) by one wave: the pivot, tie and stop rules of cpqr, columns held in
// registers while a reflector is applied.  Returns k.
template <int MB>
__device__ __forceinline__ int tiny_cpqr(double* Wf, int ldp, int m, int b, double tol, int tol_mode, int kcap, double* nrm,
                         int* stp, int* pv, double* taus, int32_t* gpiv, double* gtau, int lane, bool& over) {
  const int kmax = min(m, b);
  double r00 = 0.0;
  for (int j = 0; j < kmax; ++j) {
    double mx = 0.0;
    for (int c = lane; c < b; c += 64)
      if (stp[c] < 0) mx = fmax(mx, nrm[c]);
    mx = wave_max_dpp(mx);
    const double thr = (1.0 - kTie) * mx;
    int best = INT_MAX;
    for (int c = lane; c < b; c += 64)
      if (stp[c] < 0 && nrm[c] >= thr) best = min(best, c);
    best = wave_min_dpp(best);
    if (best == INT_MAX) return j;  // only NaN norms left
    const double rjj = sqrt(nrm[best]);
    if (j == 0) r00 = rjj;
    const bool stop = (tol_mode == 0) ? (rjj <= tol * r00) : (rjj <= tol);
    if (stop || rjj == 0.0) return j;
    if (j >= kcap) {
      over = true;
      return kcap;
    }
    double* x = Wf + (size_t)ldp * best;
    double v[MB];
#pragma unroll
    for (int u = 0; u < MB; ++u) v[u] = (u > j && u < m) ? x[u] : 0.0;
    const double alpha = x[j];
    double rest = 0.0;
#pragma unroll
    for (int u = 0; u < MB; ++u) rest += v[u] * v[u];
    double d, tj;
    if (alpha <= 0.0) {
      d = alpha - rjj;
      tj = (rjj - alpha) / rjj;
    } else {
      d = -rest / (alpha + rjj);
      tj = rest / (rjj * (rjj + alpha));
    }
    if (d == 0.0) tj = 0.0;
    // reflector j: unit entry at row j, v / d below
#pragma unroll
    for (int u = 0; u < MB; ++u) {
      if (u == j) v[u] = 1.0;
      else if (u > j && u < m && d != 0.0) v[u] = v[u] / d;
    }
    double mine = 0.0;
#pragma unroll
    for (int u = 0; u < MB; ++u) mine = (u == lane) ? v[u] : mine;
    wave_lds_sync();
    if (lane > j && lane < m) x[lane] = mine;
    if (lane == 0) {
      x[j] = rjj;
      pv[j] = best;
      taus[j] = tj;
      stp[best] = j;
      gstore(gpiv + j, best);
      gstore(gtau + j, tj);
    }
    wave_lds_sync();
    for (int c = lane; c < b; c += 64) {
      if (stp[c] >= 0) continue;
      double* y = Wf + (size_t)ldp * c;
      double yr[MB];
#pragma unroll
      for (int u = 0; u < MB; ++u) yr[u] = (u >= j && u < m) ? y[u] : 0.0;
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < MB; ++u)
        if (u >= j && u < m) s += v[u] * yr[u];
      const double f = tj * s;
      double nn = 0.0;
#pragma unroll
      for (int u = 0; u < MB; ++u)
        if (u >= j && u < m) {
          const double nv = yr[u] - f * v[u];
          y[u] = nv;
          if (u > j) nn += nv * nv;
        }
      nrm[c] = nn;
    }
    wave_lds_sync();
  }
  return kmax;
}

// C <- U^T C for the a near-field columns (ld ldp), one column per thread
// of the workgroup, reflectors 0..k-1 in order.
template <int MB>
__device__ __forceinline__ void tiny_rotate(double* C, const double* Wf, int ldp, int m, int a, int k, const int* pv,
                            const double* taus) {
  for (int c = threadIdx.x; c < a; c += kThreads) {
    double* y = C + (size_t)ldp * c;
    double yr[MB];
#pragma unroll
    for (int u = 0; u < MB; ++u) yr[u] = u < m ? y[u] : 0.0;
    for (int j = 0; j < k; ++j) {
      const double* x = Wf + (size_t)ldp * pv[j];
      double v[MB];
#pragma unroll
      for (int u = 0; u < MB; ++u) v[u] = (u > j && u < m) ? x[u] : (u == j ? 1.0 : 0.0);
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < MB; ++u)
        if (u >= j && u < m) s += v[u] * yr[u];
      const double f = taus[j] * s;
#pragma unroll
      for (int u = 0; u < MB; ++u)
        if (u >= j && u < m) yr[u] -= f * v[u];
    }
#pragma unroll
    for (int u = 0; u < MB; ++u)
      if (u < m) y[u] = yr[u];
  }
}

// Lower-triangle index p -> (rr, cc), cc <= rr, rows of the triangle in order.
__device__ __forceinline__ void tri_index(int p, int& rr, int& cc) {
  int r = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > p) --r;
  while ((r + 1) * (r + 2) / 2 <= p) ++r;
  rr = r;
  cc = p - r * (r + 1) / 2;
}

// Owning-block entry of the Schur element (rr, cc), cc <= rr, of the
// near-field columns (segment and natural index of every column and the pair
// descriptors in LDS); null, after recording the error, when out of range.
__device__ __forceinline__ double* tiny_target(const ItemD& it, int rr, int cc, const int* cseg, const int* cnat,
                                               const PairD* ps, int32_t* err, int level) {
  const int sr = cseg[rr], sc = cseg[cc], nr = cnat[rr], ncn = cnat[cc];
  const int i = min(sr, sc), j = max(sr, sc);
  const PairD& pd = ps[j * (j + 1) / 2 + i];
  int row, col;
  if (pd.diag) {
    row = max(nr, ncn);
    col = min(nr, ncn);
  } else {
    const bool r_is_rowseg = (sr == (pd.rows_from_j ? j : i));
    row = r_is_rowseg ? nr : ncn;
    const int cn = r_is_rowseg ? ncn : nr;
    col = pd.posmap ? gload(pd.posmap + cn) : cn;
  }
  if (row < 0 || col < 0 || row >= pd.nrows || col >= pd.ncols) {
    item_error(it, err, level, kErrIndex);
    return nullptr;
  }
  return pd.dst + (size_t)row + (size_t)pd.ld * col;
}

// Element (rr, cc) of F^T F, F = rows k..m-1 of the columns C (ld ldp, LDS),
// summed in row order.
__device__ __forceinline__ double tiny_dot(const double* C, int ldp, int k, int m, int rr, int cc, int prec) {
  const double* fr = C + (size_t)ldp * rr;
  const double* fc = C + (size_t)ldp * cc;
  if (prec == 0) {
    double acc = 0.0;
    int i = k;
    for (; i + 4 <= m; i += 4) {
      const double r0 = fr[i], r1 = fr[i + 1], r2 = fr[i + 2], r3 = fr[i + 3];
      const double c0 = fc[i], c1 = fc[i + 1], c2 = fc[i + 2], c3 = fc[i + 3];
      acc += r0 * c0;
      acc += r1 * c1;
      acc += r2 * c2;
      acc += r3 * c3;
    }
    for (; i < m; ++i) acc += fr[i] * fc[i];
    return acc;
  }
  float accf = 0.0f;
  for (int i = k; i < m; ++i) {
    float x0 = (float)fr[i], x1 = (float)fc[i];
    if (prec == 2) {
      x0 = round_bf16(x0);
      x1 = round_bf16(x1);
    }
    accf = fmaf(x0, x1, accf);
  }
  return (double)accf;
}

#define LRSP_TINY_DISPATCH(FN, ...)       \
  do {                                    \
    if (m <= 8) FN<8>(__VA_ARGS__);       \
    else if (m <= 16) FN<16>(__VA_ARGS__); \
    else FN<32>(__VA_ARGS__);             \
  } while (0)

// Schur elements whose targets waves 1..3 look up, and whose old values they
// load, while wave 0 factors the diagonal block: (kThreads - 64) * kTinyPre.
constexpr int kTinyPre = 2;
constexpr int kTinyPreN = (kThreads - 64) * kTinyPre;

__device__ __forceinline__ void slre_tiny(const ItemD& it, LevelState ls, int level, double tol, int tol_mode,
                                          int prec, char* lds, const int* soff, int a, int b) {
  __shared__ int sk, sbad2, sover;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m = it.m, nseg = it.nseg, nsn = it.nsegn;
  const int np = nsn * (nsn + 1) / 2;
  const TinyLayout L = tiny_layout(m, a, b, nseg, np);
  const int ldp = L.ldp;
  const int nc = m + a + b;
  double* Ps = reinterpret_cast<double*>(lds + L.p);
  const double** srcp = reinterpret_cast<const double**>(lds + L.src);
  double* nrm = reinterpret_cast<double*>(lds + L.nrm);
  double* taus = reinterpret_cast<double*>(lds + L.tau);
  int* cseg = reinterpret_cast<int*>(lds + L.cseg);
  int* cnat = reinterpret_cast<int*>(lds + L.cnat);
  int* stp = reinterpret_cast<int*>(lds + L.stp);
  int* pv = reinterpret_cast<int*>(lds + L.piv);
  WbD* wbs = reinterpret_cast<WbD*>(lds + L.wb);
  PairD* ps = reinterpret_cast<PairD*>(lds + L.pair);
  // column sources and indices; write-back and pair descriptors to LDS
  for (int pc = tid; pc < a + b; pc += kThreads) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (soff[mid] <= pc) lo = mid;
      else hi = mid - 1;
    }
    const SegD* sg = it.seg + lo;
    const int loc = pc - soff[lo];
    const int coarse = gload(&sg->coarse);
    const int32_t* zl = gload(&sg->zl);
    const double* src = gload(&sg->src);
    const int64_t voff = gload(&sg->voff);
    const int nat = coarse ? loc : gload(zl + loc);
    cseg[pc] = lo;
    cnat[pc] = nat;
    gstore(it.colseg + pc, lo);
    gstore(it.colnat + pc, nat);
    gstore(it.vidx + pc, voff + nat);
    srcp[m + pc] = src + (size_t)m * loc;
  }
  for (int c = tid; c < m; c += kThreads) srcp[c] = it.D + (size_t)m * c;
  {
    constexpr int kW = (int)(sizeof(WbD) / sizeof(double));
    constexpr int kP = (int)(sizeof(PairD) / sizeof(double));
    static_assert(sizeof(WbD) % sizeof(double) == 0 && sizeof(PairD) % sizeof(double) == 0, "staged as doubles");
    const int nw = kW * nseg, npd = kP * np;
    const double* ws = reinterpret_cast<const double*>(it.wb);
    const double* pg = reinterpret_cast<const double*>(it.pair);
    double* wd = reinterpret_cast<double*>(wbs);
    double* pd = reinterpret_cast<double*>(ps);
    for (int e0 = tid; e0 < nw + npd; e0 += kThreads * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads;
        v[u] = e < nw ? gload(ws + e) : (e < nw + npd ? gload(pg + (e - nw)) : 0.0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads;
        if (e < nw) wd[e] = v[u];
        else if (e < nw + npd) pd[e - nw] = v[u];
      }
    }
  }
  if (tid == 0) {
    sbad2 = 0;
    sover = 0;
  }
  lds_barrier();
  // gather the block row, sixteen loads in flight per thread
  const int ne = m * nc;
  for (int e0 = tid; e0 < ne; e0 += kThreads * 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + u * kThreads;
      v[u] = 0.0;
      if (e < ne) {
        const int c = e / m, r = e - c * m;
        v[u] = gload(srcp[c] + r);
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + u * kThreads;
      if (e < ne) {
        const int c = e / m, r = e - c * m;
        Ps[r + (size_t)ldp * c] = v[u];
      }
    }
  }
  lds_barrier();
  // S_s: Cholesky of the diagonal block (wave 0); meanwhile the other waves
  // look up the first Schur targets and load their old values
  const int nel = a * (a + 1) / 2;
  double* tp[kTinyPre] = {};
  double ov[kTinyPre];
  if (wv == 0) {
    bool bad = false;
    LRSP_TINY_DISPATCH(tiny_chol, Ps, ldp, m, lane, bad);
    if (lane == 0 && bad) sbad2 = 1;
  } else {
#pragma unroll
    for (int u = 0; u < kTinyPre; ++u) {
      const int p = (tid - 64) + (kThreads - 64) * u;
      tp[u] = nullptr;
      if (p < nel) {
        int rr, cc;
        tri_index(p, rr, cc);
        tp[u] = tiny_target(it, rr, cc, cseg, cnat, ps, ls.err, level);
      }
    }
#pragma unroll
    for (int u = 0; u < kTinyPre; ++u) ov[u] = tp[u] ? gload(tp[u]) : 0.0;
  }
  lds_barrier();
  LRSP_TINY_DISPATCH(tiny_scale, Ps, ldp, m, a, b, nrm, stp);
  lds_barrier();
  // compression of the scaled far field (wave 0)
  double* Wf = Ps + (size_t)ldp * (m + a);
  if (wv == 0) {
    bool over = false;
    int k = 0;
    LRSP_TINY_DISPATCH(k = tiny_cpqr, Wf, ldp, m, b, tol, tol_mode, it.kcap, nrm, stp, pv, taus, it.piv,
                       it.tau, lane, over);
    if (lane == 0) {
      sk = k;
      sover = over ? 1 : 0;
    }
  }
  lds_barrier();
  const int k = sk;
  if (tid == 0) {
    if (sbad2) item_error(it, ls.err, level, kErrNotSPD);
    if (sover) item_error(it, ls.err, level, kErrCapacity);
  }
  // E_s: rotate the near-field columns, C = U^T G^{-1} A_sn
  double* C = Ps + (size_t)ldp * m;
  if (k > 0) {
    LRSP_TINY_DISPATCH(tiny_rotate, C, Wf, ldp, m, a, k, pv, taus);
    lds_barrier();
  }
  // G_s: X_nn -= F^T F, F = rows k.. of the rotated near-field columns
  if (m > k && a > 0) {
    if (wv > 0) {
#pragma unroll
      for (int u = 0; u < kTinyPre; ++u) {
        const int p = (tid - 64) + (kThreads - 64) * u;
        if (tp[u]) {
          int rr, cc;
          tri_index(p, rr, cc);
          gstore(tp[u], ov[u] - tiny_dot(C, ldp, k, m, rr, cc, prec));
        }
      }
    }
    for (int p0 = kTinyPreN + tid; p0 < nel; p0 += kThreads * 8) {
      double* t[8];
      double val[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int p = p0 + u * kThreads;
        t[u] = nullptr;
        val[u] = 0.0;
        if (p < nel) {
          int rr, cc;
          tri_index(p, rr, cc);
          t[u] = tiny_target(it, rr, cc, cseg, cnat, ps, ls.err, level);
          val[u] = tiny_dot(C, ldp, k, m, rr, cc, prec);
        }
      }
      double old[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) old[u] = t[u] ? gload(t[u]) : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (t[u]) gstore(t[u], old[u] - val[u]);
    }
  }
  // coarse row of s: [I_k | C[:k] | V1^T]
  for (int e = tid; e < k * (a + b); e += kThreads) {
    const int r = e % k, pc = e / k;
    const WbD& t = wbs[cseg[pc]];
    const int cn = cnat[pc];
    double v = Ps[r + (size_t)ldp * (m + pc)];
    if (pc >= a) {
      const int st = stp[pc - a];
      if (st >= 0 && r > st) v = 0.0;
    }
    const int row = t.trans ? cn : r, col = t.trans ? r : cn;
    if (row >= t.nrows || col >= t.ncols) {
      item_error(it, ls.err, level, kErrIndex);
      continue;
    }
    gstore(t.dst + (size_t)row + (size_t)t.ld * col, v);
  }
  // factor pieces for the sweeps (the panel, column-major with ld m)
  for (int e = tid; e < ne; e += kThreads) {
    const int c = e / m, r = e - c * m;
    gstore(it.P + e, Ps[r + (size_t)ldp * c]);
  }
  for (int e = tid; e < k * k; e += kThreads) {
    const int r = e % k, c = e / k;
    gstore(it.D + (size_t)r + (size_t)m * c, (r == c) ? 1.0 : 0.0);
  }
  for (int c = tid; c < b; c += kThreads) gstore(it.stepof + c, stp[c]);
  if (tid == 0) {
    gstore(ls.k + it.s, k);
    gstore(ls.a + it.s, a);
    gstore(ls.b + it.s, b);
    gstore(ls.giok + it.s, 0);
  }
  __syncthreads();
}

// Elimination of one cluster without deferred compression (section
// "Deferred-compression Scheme", Eqs. offdiag and sc_old) on the gathered
// panel P = [A_ss | A_sn | A_sw] (ld m).  The unscaled far-field block is
// compressed by the same column-pivoted QR and rank rule as the scaled form,
// A_sw ~ U_1 V_1^T; A_ss is rotated by U on both sides and A_sn by U^T; the
// fine part of the rotated diagonal block is factored, X_ff = G_f G_f^T, and
// F_c = G_f^{-1} X_fc, F_n = G_f^{-1} (U^T A_sn)_f; the coarse unknowns keep
// D_c = X_cc - F_c^T F_c (its two triangles averaged) and C_cn = (U^T A_sn)_c
// - F_c^T F_n.  On return the panel holds the reflectors of U in A_sw's
// columns, G_f in rows and columns k.. of the diagonal block, F_c below D_c
// in columns ..k, C_cn over F_n in A_sn's columns; returns k.
__device__ __forceinline__ int slre_nodc_core(const ItemD& it, LevelState ls, int level, double tol, int tol_mode,
                                              double* lds, int a, int b, double* shd, int* shi, int* sbad) {
  const int tid = threadIdx.x;
  const int m = it.m;
  double* P = it.P;
  const size_t ld = (size_t)m;
  const size_t scr = (size_t)m * kNB + kNB * kNB + kNB * 256;
  // the assembled diagonal block is valid in its lower triangle: mirror it
  for (int e = tid; e < m * m; e += kThreads) {
    const int r = e % m, c = e / m;
    if (r < c) P[(size_t)r + ld * c] = P[(size_t)c + ld * r];
  }
  if (tid == 0) *sbad = 0;
  __syncthreads();
  double* Wf = P + ld * (m + a);
  int k = 0;
  bool over = false;
  if (b > 0 && m > 0)
    k = cpqr(Wf, m, m, b, tol, tol_mode, it.kcap, it.piv, it.stepof, it.tau, it.norms, shd, shi, &over);
  if (over || k > it.kcap) {
    if (tid == 0) item_error(it, ls.err, level, kErrCapacity);
    k = min(k, it.kcap);
  }
  __syncthreads();
  if (k > 0) {
    apply_qt_cols(P, m, m, m + a, Wf, it.piv, it.tau, k, lds, scr);  // U^T [A_ss | A_sn]
    __syncthreads();
    for (int e = tid; e < m * m; e += kThreads) {  // (U^T A_ss)^T = A_ss U
      const int r = e % m, c = e / m;
      if (r < c) {
        const double x = P[(size_t)r + ld * c];
        P[(size_t)r + ld * c] = P[(size_t)c + ld * r];
        P[(size_t)c + ld * r] = x;
      }
    }
    __syncthreads();
    apply_qt_cols(P, m, m, m, Wf, it.piv, it.tau, k, lds, scr);  // X = U^T A_ss U
    __syncthreads();
  }
  // G_f, F_n and F_c in one fused factor-and-solve
  chol_solve<true>(P + k + ld * k, m, m - k, P + k + ld * m, a, lds, sbad, P + k, k);
  __syncthreads();
  if (*sbad && tid == 0) item_error(it, ls.err, level, kErrNotSPD);
  // rows ..k of the columns of X_cc and of (U^T A_sn): minus F_c^T times the
  // column's rows k.. (F_c, F_n), sixteen rows at a time
  for (int c = tid; c < k + a; c += kThreads) {
    double* col = c < k ? P + ld * c : P + ld * (m + c - k);
    for (int r0 = 0; r0 < k; r0 += 16) {
      double acc[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) acc[t] = 0.0;
      for (int i = k; i < m; ++i) {
        const double f = col[i];
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[t] += P[(size_t)i + ld * min(r0 + t, k - 1)] * f;
      }
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (r0 + t < k) col[r0 + t] -= acc[t];
    }
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += kThreads) {
    const int r = e % k, c = e / k;
    if (r > c) {
      const double v = 0.5 * (P[(size_t)r + ld * c] + P[(size_t)c + ld * r]);
      P[(size_t)r + ld * c] = v;
      P[(size_t)c + ld * r] = v;
    }
  }
  __syncthreads();
  return k;
}

// One scaled low-rank elimination W_s = P_s G_s E_s S_s by one workgroup
// (with ls.nodc, the step without deferred compression instead).
// lds: slre_scratch(m) doubles, then nseg+1 ints.
__device__ __forceinline__ void slre_item(const ItemD& it, LevelState ls, int level, double tol, int tol_mode,
                          int prec, double* lds, int* soff) {
  __shared__ double shd[kWaves];
  __shared__ int shi[kWaves];
  __shared__ int wsum[kWaves];
  __shared__ int sflag, sbad;
  const int tid = threadIdx.x;
  const int m = it.m;
  int a = 0, b = 0;
  if (!seg_scan(it, ls, level, soff, wsum, &sflag, a, b)) {
    if (tid == 0) {
      ls.k[it.s] = 0;
      ls.a[it.s] = 0;
      ls.b[it.s] = 0;
      ls.giok[it.s] = 0;
    }
    return;
  }
  if (!ls.nodc && tiny_fits(m, a, b, it.nseg, it.nsegn)) {
    slre_tiny(it, ls, level, tol, tol_mode, prec, reinterpret_cast<char*>(lds), soff, a, b);
    return;
  }
  double* P = it.P;
  const size_t ld = (size_t)m;
  const int lane = tid & 63, wv = tid >> 6;
  const int ncols = m + a + b;
  // gather [A_ss | A_sn | A_sw].  When the column sources fit in the LDS
  // scratch (free until the Cholesky), every element is copied by its own
  // thread with eight loads in flight; else one column per wave.
  const double** srcp = reinterpret_cast<const double**>(lds);
  const bool table = (size_t)ncols <= (size_t)m * kNB + kNB * kNB + kNB * 256;
  if (table) {
    for (int c = tid; c < ncols; c += kThreads) {
      const double* src;
      if (c < m) {
        src = it.D + ld * c;
      } else {
        const int pc = c - m;
        int lo = 0, hi = it.nseg - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (soff[mid] <= pc) lo = mid;
          else hi = mid - 1;
        }
        const SegD& sg = it.seg[lo];
        const int loc = pc - soff[lo];
        src = sg.src + ld * loc;
        const int nat = sg.coarse ? loc : sg.zl[loc];
        it.colseg[pc] = lo;
        it.colnat[pc] = nat;
        it.vidx[pc] = sg.voff + nat;
      }
      srcp[c] = src;
    }
    __syncthreads();
    const int ne = m * ncols;
    for (int e0 = tid; e0 < ne; e0 += kThreads * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads;
        v[u] = 0.0;
        if (e < ne) {
          const int c = e / m, r = e - c * m;
          v[u] = srcp[c][r];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kThreads;
        if (e < ne) P[e] = v[u];
      }
    }
    __syncthreads();  // the scratch is the Cholesky's from here on
  }
  for (int c = wv; c < (table ? 0 : ncols); c += kWaves) {
    const double* src;
    if (c < m) {
      src = it.D + ld * c;
    } else {
      const int pc = c - m;
      int lo = 0, hi = it.nseg - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (soff[mid] <= pc) lo = mid;
        else hi = mid - 1;
      }
      const SegD& sg = it.seg[lo];
      const int loc = pc - soff[lo];
      src = sg.src + ld * loc;
      if (lane == 0) {
        const int nat = sg.coarse ? loc : sg.zl[loc];
        it.colseg[pc] = lo;
        it.colnat[pc] = nat;
        it.vidx[pc] = sg.voff + nat;
      }
    }
    double v[kRegRows];
#pragma unroll
    for (int t = 0; t < kRegRows; ++t) {
      const int r = lane + 64 * t;
      v[t] = r < m ? src[r] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kRegRows; ++t) {
      const int r = lane + 64 * t;
      if (r < m) P[ld * c + r] = v[t];
    }
  }
  double* C = P + ld * m;
  int k = 0;
  if (ls.nodc) {
    if (!table) __syncthreads();
    k = slre_nodc_core(it, ls, level, tol, tol_mode, lds, a, b, shd, shi, &sbad);
  } else {
    if (tid == 0) sbad = 0;
    __syncthreads();
    // S_s: Cholesky of A_ss and scaling of the block row
    chol_solve(P, m, m, P + ld * m, a + b, lds, &sbad);
    __syncthreads();
    if (sbad && tid == 0) item_error(it, ls.err, level, kErrNotSPD);
    // compression of the scaled far field G^{-1} A_sw
    double* Wf = P + ld * (m + a);
    bool over = false;
    if (b > 0 && m > 0)
      k = cpqr(Wf, m, m, b, tol, tol_mode, it.kcap, it.piv, it.stepof, it.tau, it.norms, shd, shi, &over);
    if (over || k > it.kcap) {
      if (tid == 0) item_error(it, ls.err, level, kErrCapacity);
      k = min(k, it.kcap);
    }
    __syncthreads();
    // E_s: rotate the near-field columns, C = U^T G^{-1} A_sn
    if (k > 0) apply_qt_cols(C, m, m, a, Wf, it.piv, it.tau, k, lds, (size_t)m * kNB + kNB * kNB + kNB * 256);
    __syncthreads();
  }
  // G_s: eliminate the fine DoFs, X_nn -= F^T F (F = rows k.. of C)
  if (m > k && a > 0 &&
      !schur_scatter_staged(it, C, m, m, k, a, prec, ls.err, level, lds, (size_t)m * kNB + kNB * kNB + kNB * 256))
    schur_scatter(it, C, m, m, k, a, prec, ls.err, level);
  // coarse row of s: [I_k | C[:k] | V1^T]
  for (int e = tid; e < k * (a + b); e += kThreads) {
    const int r = e % k, pc = e / k;
    const WbD& t = it.wb[it.colseg[pc]];
    const int cn = it.colnat[pc];
    double v = P[(size_t)r + ld * (m + pc)];
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
  // diagonal block of the coarse unknowns: I_k (without deferred
  // compression D_c)
  for (int e = tid; e < k * k; e += kThreads) {
    const int r = e % k, c = e / k;
    it.D[(size_t)r + ld * c] = ls.nodc ? P[(size_t)r + ld * c] : ((r == c) ? 1.0 : 0.0);
  }
  if (tid == 0) {
    ls.k[it.s] = k;
    ls.a[it.s] = a;
    ls.b[it.s] = b;
    ls.giok[it.s] = ls.nodc ? 3 : 0;
  }
  __syncthreads();
}

}  // namespace

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) slre_kernel(const ItemD* __restrict__ items, LevelState ls,
                                                        int level, double tol, int tol_mode, int prec,
                                                        int max_m) {
  extern __shared__ double lds[];
  int* soff = reinterpret_cast<int*>(lds + slre_scratch(max_m));
  slre_item(items[blockIdx.x], ls, level, tol, tol_mode, prec, lds, soff);
}

// All colours of a level in one persistent launch: workgroups stride over
// the clusters of a colour, then wait at a grid barrier before the next.
// Two consecutive colours of at most one cluster each both run on workgroup
// 0, whose own barrier at the end of a cluster orders them: no grid barrier
// between them (coarse levels are mostly such colours).  No barrier follows
// the last colour.  SW = false: cooperative launch (grid_group barrier);
// SW = true: ordinary launch with a co-resident grid and the bounded
// software barrier `bar`.
template <bool SW>
__global__ void __launch_bounds__(kThreads) slre_level_kernel(const ItemD* __restrict__ items,
                                                              const int32_t* __restrict__ cstart,
                                                              int ncolours, LevelState ls, int level,
                                                              double tol, int tol_mode, int prec,
                                                              int max_m, GridBar* bar) {
  extern __shared__ double lds[];
  int* soff = reinterpret_cast<int*>(lds + slre_scratch(max_m));
  for (int c = 0; c < ncolours; ++c) {
    for (int i = cstart[c] + blockIdx.x; i < cstart[c + 1]; i += gridDim.x)
      slre_item(items[i], ls, level, tol, tol_mode, prec, lds, soff);
    if (c + 1 == ncolours) break;
    if (cstart[c + 1] - cstart[c] <= 1 && cstart[c + 2] - cstart[c + 1] <= 1) {
      __syncthreads();
      continue;
    }
    if constexpr (SW) sw_grid_sync(bar, gridDim.x);
    else cooperative_groups::this_grid().sync();
  }
}

// Kernels that use more than 64 KiB of dynamic LDS must say so once.
static void allow_lds(const void* fn, bool* done) {
  if (*done) return;
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
  *done = true;
}

static size_t slre_lds(int max_m, int max_nseg) {
  return slre_scratch(max_m) * sizeof(double) + (size_t)(max_nseg + 1) * 4;
}

void launch_slre(const ItemD* items, int nitems, int max_m, int max_nseg, LevelState ls, int level,
                 double tol, int tol_mode, int prec, hipStream_t st) {
  if (nitems <= 0) return;
  static bool lds_ok = false;
  allow_lds(reinterpret_cast<const void*>(slre_kernel), &lds_ok);
  hipLaunchKernelGGL(slre_kernel, dim3(nitems), dim3(kThreads), slre_lds(max_m, max_nseg), st, items,
                     ls, level, tol, tol_mode, prec, max_m);
}

int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 1;
  }
  return cus;
}

static int occupancy(const void* fn, size_t lds) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kThreads, lds) != hipSuccess || per < 1)
    per = 1;
  return per;
}

// Co-resident grid for a cooperative launch: at most `want` workgroups and
// at most cap (when > 0).
static int coop_grid(const void* fn, size_t lds, int want, int cap = 0) {
  int g = std::min(want, occupancy(fn, lds) * device_cus());
  if (cap > 0) g = std::min(g, cap);
  return std::max(1, g);
}

int slre_level_occupancy(int max_m, int max_nseg) {
  static bool lds_ok = false;
  allow_lds(reinterpret_cast<const void*>(slre_level_kernel<false>), &lds_ok);
  return occupancy(reinterpret_cast<const void*>(slre_level_kernel<false>), slre_lds(max_m, max_nseg));
}

hipError_t launch_slre_level(const ItemD* items, const int32_t* cstart, int ncolours, int max_items,
                             int max_m, int max_nseg, LevelState ls, int level, double tol,
                             int tol_mode, int prec, hipStream_t st, int grid_cap, GridBar* bar) {
  static bool lds_ok[2] = {false, false};
  const size_t lds = slre_lds(max_m, max_nseg);
  if (bar) {
    // one workgroup per CU at most: every workgroup of the grid is resident
    const void* fn = reinterpret_cast<const void*>(slre_level_kernel<true>);
    allow_lds(fn, &lds_ok[1]);
    int g = std::max(1, std::min(max_items, device_cus()));
    if (grid_cap > 0) g = std::min(g, grid_cap);
    hipLaunchKernelGGL(slre_level_kernel<true>, dim3(g), dim3(kThreads), lds, st, items, cstart, ncolours,
                       ls, level, tol, tol_mode, prec, max_m, bar);
    return hipGetLastError();
  }
  const void* fn = reinterpret_cast<const void*>(slre_level_kernel<false>);
  allow_lds(fn, &lds_ok[0]);
  const int g = coop_grid(fn, lds, max_items, grid_cap);
  GridBar* none = nullptr;
  void* args[] = {(void*)&items, (void*)&cstart, (void*)&ncolours, (void*)&ls, (void*)&level,
                  (void*)&tol, (void*)&tol_mode, (void*)&prec, (void*)&max_m, (void*)&none};
  return hipLaunchCooperativeKernel(fn, dim3(g), dim3(kThreads), args, lds, st);
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) top_potrf_kernel(double* A, int n, int32_t* err) {
  extern __shared__ double lds[];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  chol_solve(A, n, n, nullptr, 0, lds, &sbad);
  __syncthreads();
  if (sbad && threadIdx.x == 0) set_error(err, -1, -1, kErrNotSPD);
}

void launch_top_potrf(double* A, int n, int32_t* err, hipStream_t st) {
  if (n <= 0) return;
  static bool lds_ok = false;
  allow_lds(reinterpret_cast<const void*>(top_potrf_kernel), &lds_ok);
  size_t lds = ((size_t)n * kNB + kNB * kNB + kNB * 256) * sizeof(double);
  hipLaunchKernelGGL(top_potrf_kernel, dim3(1), dim3(kThreads), lds, st, A, n, err);
}

// ---------------------------------------------------------------------------
// Triangular solves of the substitution phase, y in LDS, G (ld) in global.
namespace {

constexpr int kBlkLd = 65;  // row stride of a staged 64x64 block

// y <- G^{-1} y, G lower (m x m, ld), y in LDS.  Per 64-row block: the
// diagonal block is staged in LDS and solved by wave 0 (each lane one row,
// the reciprocals of the diagonal taken first, the solved entries broadcast
// with readlane); the rows below subtract their 64-wide dot products, each
// thread loading sixteen entries of its row at a time.
// blk: 64*65 doubles.
__device__ __forceinline__ void trsv_lower(const double* G, int ld, int m, double* y, double* blk) {
  const int tid = threadIdx.x, lane = tid & 63;
  for (int jb = 0; jb < m; jb += 64) {
    const int w = min(64, m - jb);
    load_block_rowmajor<kThreads>(blk, kBlkLd, G + (size_t)jb * ld + jb, (size_t)ld, w, 64,
                                  [&](int r, int c) { return c < w && c <= r; });
    __syncthreads();
    if (tid < 64) {
      const double* row = blk + lane * kBlkLd;
      const double rd = 1.0 / (lane < w ? blk[lane * kBlkLd + lane] : 1.0);
      double yl = (lane < w) ? y[jb + lane] : 0.0;
#pragma unroll 8
      for (int t = 0; t < 64; ++t) {
        if (t < w) {
          const double yt = readlane_d(yl, t) * readlane_d(rd, t);
          if (lane == t) yl = yt;
          else if (lane > t) yl -= row[t] * yt;
        }
      }
      if (lane < w) y[jb + lane] = yl;
    }
    __syncthreads();
    for (int i = jb + w + tid; i < m; i += kThreads) {
      const double* gi = G + (size_t)i + (size_t)ld * jb;
      double s = 0.0;
      for (int t0 = 0; t0 < w; t0 += 16) {
        double gg[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) gg[t] = (t0 + t < w) ? gi[(size_t)ld * (t0 + t)] : 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t) s += gg[t] * y[jb + min(t0 + t, w - 1)];
      }
      y[i] -= s;
    }
    __syncthreads();
  }
}

// y <- G^{-T} y, G lower (m x m, ld), y in LDS.  From the last 64-row block
// up: subtract the dot products of the block's columns below the block with
// y (one wave per column, four columns in flight), then solve the diagonal
// block transposed in wave 0 (each lane one column, the reciprocals of the
// diagonal taken first, solved entries broadcast with readlane).
template <int R>
__device__ __forceinline__ void trsv_lower_t(const double* G, int ld, int m, double* y, double* blk) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nblk = (m + 63) / 64;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int jb = bi * 64;
    const int w = min(64, m - jb);
    const int r0 = jb + w;
    load_block_rowmajor<kThreads>(blk, kBlkLd, G + (size_t)jb * ld + jb, (size_t)ld, w, 64,
                                  [&](int r, int c) { return c < w && c <= r; });
    double yr[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = r0 + lane + 64 * t;
      yr[t] = i < m ? y[i] : 0.0;
    }
    for (int t0 = wv * 4; t0 < w; t0 += kWaves * 4) {
      double g[4][R];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double* col = G + (size_t)ld * (jb + min(t0 + q, w - 1));
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = r0 + lane + 64 * t;
          g[q][t] = (t0 + q < w && i < m) ? col[i] : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) s += g[q][t] * yr[t];
        s = wave_sum(s);
        if (lane == 0 && t0 + q < w) y[jb + t0 + q] -= s;
      }
    }
    __syncthreads();
    if (tid < 64) {
      const double rd = 1.0 / (lane < w ? blk[lane * kBlkLd + lane] : 1.0);
      double yl = (lane < w) ? y[jb + lane] : 0.0;
#pragma unroll 8
      for (int t = 63; t >= 0; --t) {
        if (t < w) {
          const double yt = readlane_d(yl, t) * readlane_d(rd, t);
          if (lane == t) yl = yt;
          else if (lane < t) yl -= blk[t * kBlkLd + lane] * yt;
        }
      }
      if (lane < w) y[jb + lane] = yl;
    }
    __syncthreads();
  }
}

// Shapes of the cluster matrix in gemv_blk.
constexpr int kGemvLower = 0, kGemvFull = 2;

// y <- M y for M (m x m, ld m, m <= 256) lower triangular or full, y in LDS,
// NT threads: the 64x64 tiles are spread over the waves, each lane one
// row of a tile with the tile's 64 entries of that row loaded at once; the
// partial sums of the column blocks are added in order.  With yg, y is first
// copied from yg (global) into LDS, after the loads of each wave's first tile
// have been issued, so that the two overlap.  red: 4*256 doubles of LDS.
template <int NT = kThreads>
__device__ __forceinline__ void gemv_blk(const double* M, int m, int shape, double* y, double* red,
                                         const double* yg = nullptr) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nb = (m + 63) >> 6;
  const int ntl = shape == kGemvFull ? nb * nb : nb * (nb + 1) / 2;
  double g[64];
  int ib = 0, jb = 0;
  auto load_tile = [&](int t) {
    if (shape == kGemvFull) {
      ib = t % nb;
      jb = t / nb;
    } else {
      int rb = 0;
      while ((rb + 1) * (rb + 2) / 2 <= t) ++rb;
      const int cl = t - rb * (rb + 1) / 2;
      ib = rb;
      jb = cl;
    }
    const int i = 64 * ib + lane;
    const double* Mi = M + min(i, m - 1);
#pragma unroll
    for (int q = 0; q < 64; ++q) {
      const int j = 64 * jb + q;
      const bool ok = i < m && j < m && (shape == kGemvFull || j <= i);
      g[q] = ok ? gload(Mi + (size_t)m * j) : 0.0;
    }
  };
  if (wv < ntl) load_tile(wv);
  if (yg) {
    for (int i = tid; i < m; i += NT) y[i] = gload(yg + i);
    lds_barrier();
  }
  for (int t = wv; t < ntl; t += NT / 64) {
    if (t != wv) load_tile(t);
    const int i = 64 * ib + lane;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 64; ++q) s += g[q] * y[min(64 * jb + q, m - 1)];
    if (i < m) red[jb * 256 + i] = s;
  }
  __syncthreads();
  for (int i = tid; i < m; i += NT) {
    const int ib = i >> 6;
    const int j1 = shape == kGemvLower ? ib + 1 : nb;
    double t = 0.0;
    for (int jb = 0; jb < j1; ++jb) t += red[jb * 256 + i];
    y[i] = t;
  }
  __syncthreads();
}

// y <- M^T y for M (m x m, ld m, m <= 64 R) lower triangular (lower) or full,
// y in LDS: one wave per column of M, QC columns in flight (16 for clusters
// of at most 256 DoFs, else 4), each column's dot product with y summed
// across the wave; the results pass through red (m doubles of LDS) so that
// no wave overwrites y while another still reads it.  NT threads; every
// column's sum has the same order whatever NT and QC.
template <int R, int NT = kThreads>
__device__ __forceinline__ void gemv_t(const double* M, int m, bool lower, double* y, double* red) {
  constexpr int QC = R <= 4 ? 16 : 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double yr[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int i = lane + 64 * t;
    yr[t] = i < m ? y[i] : 0.0;
  }
  for (int cb = wv * QC; cb < m; cb += (NT / 64) * QC) {
    double g[QC][R];
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const int c = min(cb + q, m - 1);
      const double* col = M + (size_t)m * c;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = lane + 64 * t;
        g[q][t] = (cb + q < m && i < m && (!lower || i >= c)) ? gload(col + i) : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < R; ++t) acc += g[q][t] * yr[t];
      acc = wave_sum(acc);
      if (lane == q && cb + q < m) red[cb + q] = acc;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += NT) y[i] = red[i];
  __syncthreads();
}

// Stages reflectors j0..j0+nj-1 (column j of V, m rows) in LDS as
// vs[jj*mp + i] (unit leading entry, zeros above; rows padded to mp),
// sixteen loads in flight per thread.
__device__ __forceinline__ void stage_reflectors(const double* V, int m, int mp, int j0, int nj, double* vs) {
  const int n = nj * mp;
  for (int e0 = threadIdx.x; e0 < n; e0 += kThreads * 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + u * kThreads;
      const int jj = e / mp, i = e - jj * mp, j = j0 + jj;
      v[u] = 0.0;
      if (e < n && i < m) {
        if (i == j) v[u] = 1.0;
        else if (i > j) v[u] = gload(V + (size_t)m * j + i);
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + u * kThreads;
      if (e < n) vs[e] = v[u];
    }
  }
}

// y <- H_{k-1} ... H_0 y (forward: H_0 first) or y <- H_0 ... H_{k-1} y
// (backward: H_{k-1} first) for the k reflectors V (column j = reflector j)
// with factors tau, y in LDS (m).  Reflectors and their tau pass through LDS
// (vs, ts) sixteen at a time; wave 0 applies them with y in registers and
// wave reductions.
template <int R>
__device__ __forceinline__ void apply_reflectors(const double* V, const double* tau, int m, int mp, int k,
                                                 bool fwd, double* y, double* vs, double* ts) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nt = (m + 63) >> 6;
  double yr[R];
  if (wv == 0) {
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = lane + 64 * t;
      yr[t] = (t < nt && i < m) ? y[i] : 0.0;
    }
  }
  const int nchunk = (k + 15) >> 4;
  for (int q = 0; q < nchunk; ++q) {
    const int j0 = fwd ? 16 * q : max(0, k - 16 * (q + 1));
    const int nj = fwd ? min(16, k - j0) : (k - 16 * q) - j0;
    if (tid < nj) ts[tid] = gload(tau + j0 + tid);
    lds_barrier();
    stage_reflectors(V, m, mp, j0, nj, vs);
    __syncthreads();
    if (wv == 0) {
      for (int u = 0; u < nj; ++u) {
        const int jj = fwd ? u : nj - 1 - u;
        const int j = j0 + jj;
        const double* v = vs + jj * mp;
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = lane + 64 * t;
          if (t < nt && i >= j && i < m) s += v[i] * yr[t];
        }
        s = wave_sum(s);
        const double f = ts[jj] * s;
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = lane + 64 * t;
          if (t < nt && i >= j && i < m) yr[t] -= f * v[i];
        }
      }
    }
    __syncthreads();
  }
  if (wv == 0) {
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = lane + 64 * t;
      if (t < nt && i < m) y[i] = yr[t];
    }
  }
  __syncthreads();
}

// y_n -= F^T y_f over the columns [c0, c1) of F = C[k:m, :] (C = U^T G^{-1}
// A_sn in the factor store, ld m): one wave per column, QC columns in flight
// (16 for clusters of at most 256 DoFs, else 4; every column's sum has the
// same order either way).  y (m entries) may be in LDS or global memory.
template <int R>
__device__ __forceinline__ void fwd_near(const ItemD& it, int m, int k, int c0, int c1, const double* y, double* vec) {
  constexpr int QC = R <= 4 ? 16 : 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double yr[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int i = lane + 64 * t;
    yr[t] = (i >= k && i < m) ? y[i] : 0.0;
  }
  const double* C = it.S + (size_t)m * m;
  for (int cb = c0 + wv * QC; cb < c1; cb += kWaves * QC) {
    double g[QC][R];
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const double* f = C + (size_t)m * min(cb + q, c1 - 1);
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = lane + 64 * t;
        g[q][t] = (cb + q < c1 && i >= k && i < m) ? gload(f + i) : 0.0;
      }
    }
    double sv = 0.0;
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < R; ++t) acc += g[q][t] * yr[t];
      acc = wave_sum(acc);
      if (q == lane) sv = acc;
    }
    if (lane < QC && cb + lane < c1) vec[it.vidx[cb + lane]] -= sv;
  }
}

// Without deferred compression (giok 3): y_c -= F_c^T y_f, F_c = rows k.. of
// the panel's columns ..k (ld m), y in LDS; one wave per coarse entry.
__device__ __forceinline__ void nodc_fc_t(const double* P, int m, int k, double* y) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int r = wv; r < k; r += kWaves) {
    const double* f = P + (size_t)m * r;
    double s = 0.0;
    for (int i = k + lane; i < m; i += 64) s += f[i] * y[i];
    s = wave_sum(s);
    if (lane == 0) y[r] -= s;
  }
  __syncthreads();
}

// Without deferred compression: x_f -= F_c x_c, one thread per fine row.
__device__ __forceinline__ void nodc_fc(const double* P, int m, int k, double* x) {
  for (int i = k + threadIdx.x; i < m; i += kThreads) {
    double s = 0.0;
    for (int r = 0; r < k; ++r) s += P[(size_t)i + (size_t)m * r] * x[r];
    x[i] -= s;
  }
  __syncthreads();
}

// Without deferred compression, forward part of the cluster itself:
// y <- U^T y, y_f <- G_f^{-1} y_f, y_c -= F_c^T y_f (y in LDS; S the
// cluster's factor store).
template <int R>
__device__ __forceinline__ void nodc_fwd(const double* S, int m, int k, int a, int mp, double* y, double* blk,
                                         double* vs) {
  const double* V = S + (size_t)m * (m + a);
  apply_reflectors<R>(V, V + (size_t)m * k, m, mp, k, true, y, vs, blk);
  trsv_lower(S + k + (size_t)m * k, m, m - k, y + k, blk);
  nodc_fc_t(S, m, k, y);
}

// Without deferred compression, backward part of the cluster itself (after
// x_f -= F_n x_n): x_f <- G_f^{-T} (x_f - F_c x_c), x <- U x.
template <int R>
__device__ __forceinline__ void nodc_bwd(const double* S, int m, int k, int a, int mp, double* x, double* blk,
                                         double* vs) {
  const double* V = S + (size_t)m * (m + a);
  nodc_fc(S, m, k, x);
  trsv_lower_t<R>(S + k + (size_t)m * k, m, m - k, x + k, blk);
  apply_reflectors<R>(V, V + (size_t)m * k, m, mp, k, false, x, vs, blk);
}

}  // namespace

namespace {

// The cluster's own part of the forward sweep, y <- U^T G^{-1} y (without
// deferred compression the rotation, fine solve and coarse update), from the
// factor store S: gk 2: one product with W = U^T G^{-1} (first copying y from
// yg when yg is given); gk 1: G^{-1} then the reflectors; gk 0: a triangular
// solve with G then the reflectors; gk 3: nodc_fwd.  y in LDS (loaded from yg
// unless yg is null).
template <int R>
__device__ __forceinline__ void own_fwd(const double* S, int gk, int m, int k, int a, int mp, double* y,
                                        const double* yg, double* blk, double* vs) {
  if (gk == 2) {
    gemv_blk(S, m, kGemvFull, y, blk, yg);
    return;
  }
  if (yg) {
    for (int i = threadIdx.x; i < m; i += kThreads) y[i] = yg[i];
    __syncthreads();
  }
  if (gk == 3) {
    nodc_fwd<R>(S, m, k, a, mp, y, blk, vs);
    return;
  }
  if (gk == 1) gemv_blk(S, m, kGemvLower, y, blk);
  else trsv_lower(S, m, m, y, blk);
  const double* V = S + (size_t)m * (m + a);
  apply_reflectors<R>(V, V + (size_t)m * k, m, mp, k, true, y, vs, blk);
}

// The cluster's own part of the backward sweep, x <- G^{-T} U x (the
// transposes of own_fwd), x in LDS.
template <int R>
__device__ __forceinline__ void own_bwd(const double* S, int gk, int m, int k, int a, int mp, double* x,
                                        double* blk, double* vs) {
  if (gk == 2) {
    gemv_t<R>(S, m, false, x, blk);  // W^T = G^{-T} U
    return;
  }
  if (gk == 3) {
    nodc_bwd<R>(S, m, k, a, mp, x, blk, vs);
    return;
  }
  const double* V = S + (size_t)m * (m + a);
  apply_reflectors<R>(V, V + (size_t)m * k, m, mp, k, false, x, vs, blk);
  if (gk == 1) gemv_t<R>(S, m, true, x, blk);  // G^{-T} = (G^{-1})^T
  else trsv_lower_t<R>(S, m, m, x, blk);
}

// Forward substitution of one cluster: y_s <- U^T G^{-1} y_s, y_n -= F^T y_f.
// lds: mp (y) + 64*65 (diagonal block) + 16*mp (reflectors) doubles.
template <int R>
__device__ __forceinline__ void fwd_item(const ItemD& it, LevelState ls, double* vec, double* lds) {
  const int m = it.m;
  if (m == 0) return;
  const int tid = threadIdx.x;
  const int k = ls.k[it.s], a = ls.a[it.s];
  const int mp = ((m + 63) / 64) * 64;
  double* y = lds;
  double* blk = lds + mp;
  double* vs = blk + 64 * kBlkLd;
  double* yg = vec + it.voff;
  own_fwd<R>(it.S, ls.giok[it.s], m, k, a, mp, y, yg, blk, vs);
  fwd_near<R>(it, m, k, 0, a, y, vec);
  for (int i = tid; i < m; i += kThreads) yg[i] = y[i];
  __syncthreads();
}

// Forward sweep of a split cluster, per-cluster part: y_s <- U^T G^{-1} y_s,
// written back to the vector (the near-field product follows in units).
template <int R>
__device__ __forceinline__ void fwd_head(const ItemD& it, LevelState ls, double* vec, double* lds) {
  const int m = it.m;
  if (m == 0) return;
  const int tid = threadIdx.x;
  const int k = ls.k[it.s], a = ls.a[it.s];
  const int mp = ((m + 63) / 64) * 64;
  double* y = lds;
  double* blk = lds + mp;
  double* vs = blk + 64 * kBlkLd;
  double* yg = vec + it.voff;
  own_fwd<R>(it.S, ls.giok[it.s], m, k, a, mp, y, yg, blk, vs);
  for (int i = tid; i < m; i += kThreads) yg[i] = y[i];
  __syncthreads();
}

// Forward sweep of a split cluster, unit `part`: y_n -= F^T y_f over columns
// [part*kSweepCols, (part+1)*kSweepCols) of F, y_s read from the vector.
template <int R>
__device__ __forceinline__ void fwd_unit(const ItemD& it, int part, LevelState ls, double* vec,
                                         const double* ysrc) {
  const int m = it.m;
  const int k = ls.k[it.s], a = ls.a[it.s];
  const int c0 = part * kSweepCols;
  if (m == 0 || c0 >= a) return;
  fwd_near<R>(it, m, k, c0, min(a, c0 + kSweepCols), ysrc + it.voff, vec);
}

// Backward sweep of a split cluster, unit `part`: x_f -= F x_n for the rows
// [part*kSweepRows, (part+1)*kSweepRows) of F that are fine (>= k).  32 rows x
// 8 column groups (two per wave): every row sums its columns group by group
// in a fixed order, then the eight group sums in order.  x_n passes through
// LDS 1024 columns at a time.  lds: 1024 + 256 doubles.
__device__ __forceinline__ void bwd_unit(const ItemD& it, int part, LevelState ls, double* vec, double* lds,
                                         double* shadow = nullptr) {
  const int m = it.m;
  const int k = ls.k[it.s], a = ls.a[it.s];
  const int r0 = part * kSweepRows;
  if (m == 0 || r0 >= m) return;
  if (a == 0 || r0 + kSweepRows <= k) {
    // nothing to subtract: the rows go to the shadow vector unchanged
    if (shadow && threadIdx.x < kSweepRows && r0 + threadIdx.x < m)
      gstore(shadow + it.voff + r0 + threadIdx.x, gload(vec + it.voff + r0 + threadIdx.x));
    return;
  }
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row = r0 + (lane & 31), g = 2 * wv + (lane >> 5);
  const bool act = row >= k && row < m;
  double* xn = lds;
  double* red = lds + 1024;
  const double* C = it.S + (size_t)m * m;
  double s = 0.0;
  for (int c0 = 0; c0 < a; c0 += 1024) {
    const int nc = min(1024, a - c0);
    __syncthreads();
    for (int c = tid; c < nc; c += kThreads) xn[c] = vec[it.vidx[c0 + c]];
    __syncthreads();
    if (act) {
      const double* Cr = C + row + (size_t)m * c0;
      for (int cb = g; cb < nc; cb += 8 * 16) {
        double f[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int c = cb + 8 * q;
          f[q] = c < nc ? Cr[(size_t)m * c] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int c = cb + 8 * q;
          if (c < nc) s += f[q] * xn[c];
        }
      }
    }
  }
  red[g * 32 + (lane & 31)] = s;
  __syncthreads();
  if (tid < 32 && r0 + tid < m) {
    double v = vec[it.voff + r0 + tid];
    if (r0 + tid >= k) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) t += red[q * 32 + tid];
      v -= t;
      if (!shadow) vec[it.voff + r0 + tid] = v;
    }
    if (shadow) gstore(shadow + it.voff + r0 + tid, v);
  }
  __syncthreads();
}

// Backward sweep of a split cluster, per-cluster part (after its units):
// x_s <- G^{-T} U x_s.
template <int R>
__device__ __forceinline__ void bwd_tail(const ItemD& it, LevelState ls, double* vec, double* lds) {
  const int m = it.m;
  if (m == 0) return;
  const int tid = threadIdx.x;
  const int k = ls.k[it.s], a = ls.a[it.s];
  const int mp = ((m + 63) / 64) * 64;
  double* x = lds;
  double* blk = lds + mp;
  double* vs = blk + 64 * kBlkLd;
  double* xg = vec + it.voff;
  for (int i = tid; i < m; i += kThreads) x[i] = xg[i];
  __syncthreads();
  own_bwd<R>(it.S, ls.giok[it.s], m, k, a, mp, x, blk, vs);
  for (int i = tid; i < m; i += kThreads) xg[i] = x[i];
  __syncthreads();
}

// Backward substitution of one cluster: x_f -= F x_n, x_s <- G^{-T} U x_s.
// lds: mp + 64*65 + 16*mp + 1024 doubles.
template <int R>
__device__ __forceinline__ void bwd_item(const ItemD& it, LevelState ls, double* vec, double* lds) {
  const int m = it.m;
  if (m == 0) return;
  const int tid = threadIdx.x;
  const int k = ls.k[it.s], a = ls.a[it.s];
  const int mp = ((m + 63) / 64) * 64;
  double* x = lds;
  double* blk = lds + mp;
  double* vs = blk + 64 * kBlkLd;
  double* xn = vs + 16 * mp;  // 1024-column chunks of x_n
  double* xg = vec + it.voff;
  for (int i = tid; i < m; i += kThreads) x[i] = xg[i];
  const double* C = it.S + (size_t)m * m;
  for (int c0 = 0; c0 < a; c0 += 1024) {
    const int nc = min(1024, a - c0);
    __syncthreads();
    for (int c = tid; c < nc; c += kThreads) xn[c] = vec[it.vidx[c0 + c]];
    __syncthreads();
    for (int i = k + tid; i < m; i += kThreads) {
      double s = 0.0;
      for (int cb = 0; cb < nc; cb += 16) {
        double f[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) f[q] = (cb + q < nc) ? C[(size_t)i + (size_t)m * (c0 + cb + q)] : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (cb + q < nc) s += f[q] * xn[cb + q];
      }
      x[i] -= s;
    }
  }
  __syncthreads();
  own_bwd<R>(it.S, ls.giok[it.s], m, k, a, mp, x, blk, vs);
  for (int i = tid; i < m; i += kThreads) xg[i] = x[i];
  __syncthreads();
}

size_t sweep_lds(int max_m) {
  const size_t mp = (size_t)((max_m + 63) / 64) * 64;
  return (mp + 64 * kBlkLd + 16 * mp + 1024) * sizeof(double);
}

}  // namespace

// ---------------------------------------------------------------------------
// Sweeps of small clusters (m <= kSweepWaveM) by one wave each: lane i holds
// entry i of the cluster's vector, solved entries are broadcast with
// readlane, the near-field products run one lane per column (forward) or
// per row (backward).  MB >= m bounds the row slots kept in registers.

// What a wave needs of a small cluster in the sweeps: its factor store S
// ([G | C | V], ld m) and the reflector factors tau behind it.
struct WaveItem {
  const double* S;
  const double* tau;
  const int64_t* vidx;
  const int32_t* vix;  // LDS copy of the first kSweepWaveVix entries of vidx, or null
  int64_t voff;
  int32_t m, k, a, pad;
};

static_assert(sizeof(WaveItem) + 4 * kSweepWaveVix <= kSweepWaveTableBytes, "wave table entry");

__device__ __forceinline__ WaveItem wave_item(const ItemD& it, LevelState ls) {
  const int m = it.m, k = ls.k[it.s], a = ls.a[it.s];
  return WaveItem{it.S, it.S + (size_t)m * (m + a + k), it.vidx, nullptr, it.voff, m, k, a, 0};
}

// y_s <- U^T G^{-1} y_s; y_n -= F^T y_f.  For MB <= 32 every load that does
// not depend on the computation (G, the reflectors, the first 64 columns of
// F with their targets and the targets' old values) is issued up front.
template <int MB>
__device__ __forceinline__ void fwd_wave(const WaveItem& wi, double* vec) {
  constexpr bool PF = MB <= 32;
  const int lane = threadIdx.x & 63;
  const int m = wi.m;
  if (m == 0) return;
  const int k = wi.k, a = wi.a;
  const bool on = lane < m;
  const double* G = wi.S;
  const double* V = wi.S + (size_t)m * (m + a);
  const double* C = wi.S + (size_t)m * m;
  double g[MB];  // row `lane` of G, columns < lane
#pragma unroll
  for (int j = 0; j < MB; ++j) g[j] = (on && j < lane) ? G[lane + (size_t)m * j] : 0.0;
  const double gd = on ? G[lane + (size_t)m * lane] : 1.0;
  const double tv = lane < k ? wi.tau[lane] : 0.0;
  double* yg = vec + wi.voff;
  double y = on ? yg[lane] : 0.0;
  double vr[PF ? 16 : 1];  // reflector j < 16 at row `lane`
  double f0[PF ? MB : 1];  // column `lane` of F (first 64 columns)
  double old0 = 0.0;
  const bool cv0 = lane < a;
  if constexpr (PF) {
#pragma unroll
    for (int j = 0; j < 16; ++j)
      vr[j] = (j < k) ? (lane == j ? 1.0 : ((on && lane > j) ? V[lane + (size_t)m * j] : 0.0)) : 0.0;
    const double* Cc = C + (size_t)m * (cv0 ? lane : 0);
#pragma unroll
    for (int i = 0; i < MB; ++i) f0[i] = (cv0 && i >= k && i < m) ? Cc[i] : 0.0;
    if (cv0) old0 = vec[wi.vix ? (int64_t)wi.vix[lane] : wi.vidx[lane]];
  }
  const double rd = 1.0 / gd;
  // G^{-1}
#pragma unroll
  for (int j = 0; j < MB; ++j) {
    if (j < m) {
      const double yj = readlane_d(y, j) * readlane_d(rd, j);
      if (lane == j) y = yj;
      else y -= g[j] * yj;
    }
  }
  // U^T: reflectors 0..k-1 (the first 16 prefetched)
  int j1 = 0;
  if constexpr (PF) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j < k) {
        const double sj = wave_sum(vr[j] * y);
        y -= (readlane_d(tv, j) * sj) * vr[j];
      }
    }
    j1 = 16;
  }
  {
    for (int j = j1; j < k; ++j) {
      const double v = lane == j ? 1.0 : ((on && lane > j) ? V[lane + (size_t)m * j] : 0.0);
      const double sj = wave_sum(v * y);
      y -= (readlane_d(tv, j) * sj) * v;
    }
  }
  // y_n -= F^T y_f, F = C[k:m, :], one lane per column
  for (int c0 = 0; c0 < a; c0 += 64) {
    const int c = c0 + lane;
    const bool cv = c < a;
    double s = 0.0;
    if (PF && c0 == 0) {
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        const double yi = readlane_d(y, i);
        if (cv && i >= k && i < m) s += f0[i] * yi;
      }
      if (cv) vec[wi.vix ? (int64_t)wi.vix[c] : wi.vidx[c]] = old0 - s;
      continue;
    }
    const double* Cc = C + (size_t)m * (cv ? c : 0);
    for (int i0 = 0; i0 < m; i0 += 16) {
      double f[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = i0 + u;
        f[u] = (cv && i >= k && i < m) ? Cc[i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = i0 + u;
        const double yi = readlane_d(y, min(i, 63));
        if (cv && i >= k && i < m) s += f[u] * yi;
      }
    }
    if (cv) vec[wi.vidx[c]] -= s;
  }
  if (on) yg[lane] = y;
}

// x_f -= F x_n; x_s <- G^{-T} U x_s.  For MB <= 32 the loads of G, the
// reflectors, the first 32 columns of F and their x_n are issued up front.
template <int MB>
__device__ __forceinline__ void bwd_wave(const WaveItem& wi, double* vec) {
  constexpr bool PF = MB <= 32;
  const int lane = threadIdx.x & 63;
  const int m = wi.m;
  if (m == 0) return;
  const int k = wi.k, a = wi.a;
  const bool on = lane < m;
  const double* G = wi.S;
  const double* V = wi.S + (size_t)m * (m + a);
  const double* C = wi.S + (size_t)m * m;
  const bool fine = on && lane >= k;
  const double gd = on ? G[lane + (size_t)m * lane] : 1.0;
  const double tv = lane < k ? wi.tau[lane] : 0.0;
  double* xg = vec + wi.voff;
  double x = on ? xg[lane] : 0.0;
  double gc[MB];  // column `lane` of G, rows > lane
#pragma unroll
  for (int j = 0; j < MB; ++j) gc[j] = (on && j > lane && j < m) ? G[j + (size_t)m * lane] : 0.0;
  double vr[PF ? 16 : 1];   // reflector j < 16 at row `lane`
  double f0[PF ? 32 : 1];  // row `lane` of F, first 32 columns
  double xn0 = 0.0;
  const int nc0 = min(32, a);
  if constexpr (PF) {
#pragma unroll
    for (int j = 0; j < 16; ++j)
      vr[j] = (j < k) ? (lane == j ? 1.0 : ((on && lane > j) ? V[lane + (size_t)m * j] : 0.0)) : 0.0;
    const double* Cr = C + (size_t)(fine ? lane : 0);
#pragma unroll
    for (int q = 0; q < 32; ++q) f0[q] = (fine && q < nc0) ? Cr[(size_t)m * q] : 0.0;
    if (lane < nc0) xn0 = vec[wi.vix ? (int64_t)wi.vix[lane] : wi.vidx[lane]];
  }
  const double rd = 1.0 / gd;
  // x_f -= F x_n, one lane per row, columns in order
  double s = 0.0;
  int c0 = 0;
  if constexpr (PF) {
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const double xq = readlane_d(xn0, q);
      if (q < nc0) s += f0[q] * xq;
    }
    c0 = nc0;
  }
  for (; c0 < a; c0 += 64) {
    const int nc = min(64, a - c0);
    const double xn = lane < nc ? vec[wi.vidx[c0 + lane]] : 0.0;
    const double* Cr = C + (size_t)(fine ? lane : 0) + (size_t)m * c0;
    for (int cb = 0; cb < nc; cb += 16) {
      double f[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) f[q] = (fine && cb + q < nc) ? Cr[(size_t)m * (cb + q)] : 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double xq = readlane_d(xn, min(cb + q, 63));
        if (cb + q < nc) s += f[q] * xq;
      }
    }
  }
  if (fine) x -= s;
  // U: reflectors k-1..0 (the first 16 prefetched)
  for (int j = k - 1; j >= (PF ? 16 : 0); --j) {
    const double v = lane == j ? 1.0 : ((on && lane > j) ? V[lane + (size_t)m * j] : 0.0);
    const double sj = wave_sum(v * x);
    x -= (readlane_d(tv, j) * sj) * v;
  }
  if constexpr (PF) {
#pragma unroll
    for (int j = 15; j >= 0; --j) {
      if (j < k) {
        const double sj = wave_sum(vr[j] * x);
        x -= (readlane_d(tv, j) * sj) * vr[j];
      }
    }
  }
  // G^{-T}
#pragma unroll
  for (int j = MB - 1; j >= 0; --j) {
    if (j < m) {
      const double xj = readlane_d(x, j) * readlane_d(rd, j);
      if (lane == j) x = xj;
      else x -= gc[j] * xj;
    }
  }
  if (on) xg[lane] = x;
}

#define LRSP_WAVE_DISPATCH(FN, ...)         \
  do {                                      \
    if (wi.m <= 16) FN<16>(__VA_ARGS__);    \
    else FN<32>(__VA_ARGS__);               \
  } while (0)

// One launch per level and sweep direction for levels whose clusters all
// have at most kSweepWaveM DoFs: every wave takes a cluster of the colour;
// one workgroup needs no grid barrier between colours.  With table != 0 the
// descriptors and ranks of all the level's clusters are first copied
// to LDS (kSweepWaveTableBytes per cluster), which takes their loads off the
// path of every colour; with table == 2 also the level-vector indices of the
// first kSweepWaveVix near-field columns (32-bit), so that the vector loads
// of a cluster do not wait for its index loads.
template <bool FWD, bool SW>
__global__ void __launch_bounds__(kSweepWaveThreads) sweep_wave_kernel(const ItemD* __restrict__ items,
                                                                       const int32_t* __restrict__ cstart,
                                                                       int ncolours, LevelState ls,
                                                                       double* vec, GridBar* bar, int table) {
  extern __shared__ double dlds[];
  const int wv = threadIdx.x >> 6, nw = kSweepWaveThreads / 64;
  const int ni = cstart[ncolours];
  WaveItem* tab = reinterpret_cast<WaveItem*>(dlds);
  int32_t* vxs = reinterpret_cast<int32_t*>(tab + (table ? ni : 0));
  if (table) {
    for (int i = threadIdx.x; i < ni; i += kSweepWaveThreads) tab[i] = wave_item(items[i], ls);
    __syncthreads();
    if (table > 1)
      for (int e = threadIdx.x; e < ni * kSweepWaveVix; e += kSweepWaveThreads) {
        const int i = e / kSweepWaveVix, j = e - i * kSweepWaveVix;
        vxs[e] = j < tab[i].a ? (int32_t)tab[i].vidx[j] : 0;
      }
    __syncthreads();
    if (table > 1) {
      for (int i = threadIdx.x; i < ni; i += kSweepWaveThreads) tab[i].vix = vxs + (size_t)kSweepWaveVix * i;
      __syncthreads();
    }
  }
  for (int q = 0; q < ncolours; ++q) {
    const int c = FWD ? q : ncolours - 1 - q;
    for (int i = cstart[c] + blockIdx.x * nw + wv; i < cstart[c + 1]; i += gridDim.x * nw) {
      const ItemD& it = items[i];
      const WaveItem wi = table ? tab[i] : wave_item(it, ls);
      if (FWD) LRSP_WAVE_DISPATCH(fwd_wave, wi, vec);
      else LRSP_WAVE_DISPATCH(bwd_wave, wi, vec);
    }
    if (q + 1 == ncolours) break;
    const int cn = FWD ? c + 1 : c - 1;
    // colours of at most one cluster run on wave 0 of workgroup 0: its own
    // program order orders them (no barrier, no wait for its stores)
    if (cstart[c + 1] - cstart[c] <= 1 && cstart[cn + 1] - cstart[cn] <= 1) {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      continue;
    }
    // colours of at most nw clusters run on workgroup 0 alone
    const bool local = cstart[c + 1] - cstart[c] <= nw && cstart[cn + 1] - cstart[cn] <= nw;
    if (gridDim.x == 1 || local) __syncthreads();
    else if constexpr (SW) sw_grid_sync(bar, gridDim.x);
    else cooperative_groups::this_grid().sync();
  }
}

// Row slots per lane sized to the cluster (the slots beyond m hold zeros and
// add exact zeros, so the results do not depend on the choice).
#define LRSP_ROWS_DISPATCH(FN, ...)                      \
  do {                                                   \
    if (it.m <= 256) FN<4>(__VA_ARGS__);                 \
    else FN<kMaxClusterDofs / 64>(__VA_ARGS__);          \
  } while (0)

// Clusters of at most kSweepWaveM DoFs run the wave form in wave 0 whatever
// the schedule, so that every schedule gives the same bits.
__device__ __forceinline__ void fwd_any(const ItemD& it, bool split, LevelState ls, double* vec, double* lds) {
  if (it.m <= kSweepWaveM && !ls.nodc) {
    if (threadIdx.x < 64) {
      const WaveItem wi = wave_item(it, ls);
      LRSP_WAVE_DISPATCH(fwd_wave, wi, vec);
    }
    __syncthreads();
  } else if (split && it.m >= kSweepSplitM) {
    LRSP_ROWS_DISPATCH(fwd_head, it, ls, vec, lds);
  } else {
    LRSP_ROWS_DISPATCH(fwd_item, it, ls, vec, lds);
  }
}

__device__ __forceinline__ void bwd_any(const ItemD& it, bool split, LevelState ls, double* vec, double* lds) {
  if (it.m <= kSweepWaveM && !ls.nodc) {
    if (threadIdx.x < 64) {
      const WaveItem wi = wave_item(it, ls);
      LRSP_WAVE_DISPATCH(bwd_wave, wi, vec);
    }
    __syncthreads();
  } else if (split && it.m >= kSweepSplitM) {
    LRSP_ROWS_DISPATCH(bwd_tail, it, ls, vec, lds);
  } else {
    LRSP_ROWS_DISPATCH(bwd_item, it, ls, vec, lds);
  }
}

__device__ __forceinline__ void fwd_unit_any(const ItemD& it, int part, LevelState ls, double* vec,
                                             const double* ysrc) {
  if (it.m >= kSweepSplitM) LRSP_ROWS_DISPATCH(fwd_unit, it, part, ls, vec, ysrc);
}

// Items of one colour; with split (a level holding clusters of at least
// kSweepSplitM DoFs) those clusters only do their per-cluster part here.
__global__ void __launch_bounds__(kThreads) fwd_kernel(const ItemD* __restrict__ items, int nitems,
                                                       LevelState ls, double* vec, int split) {
  extern __shared__ double lds[];
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const ItemD& it = items[i];
    fwd_any(it, split != 0, ls, vec, lds);
  }
}

__global__ void __launch_bounds__(kThreads) bwd_kernel(const ItemD* __restrict__ items, int nitems,
                                                       LevelState ls, double* vec, int split) {
  extern __shared__ double lds[];
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const ItemD& it = items[i];
    bwd_any(it, split != 0, ls, vec, lds);
  }
}

// Units of the split clusters of one colour: upi units per item.
__global__ void __launch_bounds__(kThreads) fwd_units_kernel(const ItemD* __restrict__ items, LevelState ls,
                                                             double* vec, int upi, const double* shadow) {
  const ItemD& it = items[blockIdx.x / upi];
  const int part = blockIdx.x % upi;
  // y_s in the shadow vector (rows formed by fwd_rows_kernel): read there,
  // and copied back by the cluster's first unit
  fwd_unit_any(it, part, ls, vec, shadow ? shadow : vec);
  if (shadow && part == 0)
    for (int i = threadIdx.x; i < it.m; i += kThreads) vec[it.voff + i] = gload(shadow + it.voff + i);
}

// Per-cluster part of the forward sweep of a wide colour (see launch_fwd):
// workgroup (i, b) forms rows 64b.. of W y_s (giok 2) or G^{-1} y_s (giok 1)
// into the shadow vector, wave w the partial sums of column block w.  Every
// row's sum has the order of gemv_blk (each tile's 64 products in order,
// then the tiles in order).
__global__ void __launch_bounds__(kThreads) fwd_rows_kernel(const ItemD* __restrict__ items, LevelState ls,
                                                            const double* vec, double* shadow) {
  __shared__ double y[kInvMaxDofs];
  __shared__ double red[4 * 64];
  const ItemD& it = items[blockIdx.x];
  const int m = it.m, ib = blockIdx.y, i0 = 64 * ib;
  if (i0 >= m) return;
  const int gk = ls.giok[it.s];
  if (m > kInvMaxDofs || (gk != 1 && gk != 2)) {
    if (threadIdx.x == 0) item_error(it, ls.err, -1, kErrIndex);
    return;
  }
  const int tid = threadIdx.x, lane = tid & 63, jb = tid >> 6;
  const int nb = (m + 63) >> 6;
  const bool full = gk == 2;
  const bool on = jb < nb && (full || jb <= ib);
  const int i = i0 + lane;
  double g[64];
  if (on) {
    const double* Mi = it.S + min(i, m - 1);
#pragma unroll
    for (int q = 0; q < 64; ++q) {
      const int j = 64 * jb + q;
      g[q] = (i < m && j < m && (full || j <= i)) ? gload(Mi + (size_t)m * j) : 0.0;
    }
  }
  for (int r = tid; r < m; r += kThreads) y[r] = gload(vec + it.voff + r);
  lds_barrier();
  if (on) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 64; ++q) s += g[q] * y[min(64 * jb + q, m - 1)];
    red[jb * 64 + lane] = s;
  }
  lds_barrier();
  if (tid < 64 && i < m) {
    const int j1 = full ? nb : ib + 1;
    double t = 0.0;
    for (int b = 0; b < j1; ++b) t += red[b * 64 + tid];
    gstore(shadow + it.voff + i, t);
  }
}

// Per-cluster part of the backward sweep of a wide colour (see launch_bwd):
// x_s <- W^T x_s (giok 2) or G^{-T} x_s (giok 1, no reflector), x_s read
// from the shadow vector (written by the units), workgroup (i, b) the
// entries 64b.. written to the vector; wave w the 16 columns 64b + 16w..,
// each column's sum formed as in gemv_t (same lanes, same order).
__global__ void __launch_bounds__(kThreads) bwd_cols_kernel(const ItemD* __restrict__ items, LevelState ls,
                                                            double* vec, const double* shadow) {
  constexpr int R = 4, QC = 16;
  const ItemD& it = items[blockIdx.x];
  const int m = it.m, c0 = 64 * blockIdx.y;
  if (c0 >= m) return;
  const int gk = ls.giok[it.s];
  if (m > kInvMaxDofs || (gk != 1 && gk != 2)) {
    if (threadIdx.x == 0) item_error(it, ls.err, -1, kErrIndex);
    return;
  }
  const bool lower = gk != 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int cb = c0 + QC * wv;
  const double* M = it.S;
  double g[QC][R], yr[R];
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    const int c = min(cb + q, m - 1);
    const double* col = M + (size_t)m * c;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = lane + 64 * t;
      g[q][t] = (cb + q < m && i < m && (!lower || i >= c)) ? gload(col + i) : 0.0;
    }
  }
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int i = lane + 64 * t;
    yr[t] = i < m ? gload(shadow + it.voff + i) : 0.0;
  }
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < R; ++t) acc += g[q][t] * yr[t];
    acc = wave_sum(acc);
    if (lane == q && cb + q < m) gstore(vec + it.voff + cb + q, acc);
  }
}

__global__ void __launch_bounds__(kThreads) bwd_units_kernel(const ItemD* __restrict__ items, LevelState ls,
                                                             double* vec, int upi, double* shadow) {
  extern __shared__ double lds[];
  const ItemD& it = items[blockIdx.x / upi];
  if (it.m >= kSweepSplitM) bwd_unit(it, blockIdx.x % upi, ls, vec, lds, shadow);
}

template <bool SW>
__device__ __forceinline__ void level_sync(GridBar* bar) {
  if constexpr (SW) sw_grid_sync(bar, gridDim.x);
  else cooperative_groups::this_grid().sync();
}

// One launch per level and sweep direction; upi > 0: units per item of the
// split clusters (an extra grid barrier per colour).  Without units, two
// consecutive colours of at most one cluster each run on workgroup 0 alone
// and need no grid barrier between them; none follows the last colour.
template <bool SW>
__global__ void __launch_bounds__(kThreads) fwd_level_kernel(const ItemD* __restrict__ items,
                                                             const int32_t* __restrict__ cstart,
                                                             int ncolours, LevelState ls, double* vec,
                                                             GridBar* bar, int upi) {
  extern __shared__ double lds[];
  for (int c = 0; c < ncolours; ++c) {
    for (int i = cstart[c] + blockIdx.x; i < cstart[c + 1]; i += gridDim.x) {
      const ItemD& it = items[i];
      fwd_any(it, upi > 0, ls, vec, lds);
    }
    if (upi == 0) {
      if (c + 1 == ncolours) break;
      if (cstart[c + 1] - cstart[c] <= 1 && cstart[c + 2] - cstart[c + 1] <= 1) {
        __syncthreads();
        continue;
      }
    }
    level_sync<SW>(bar);
    if (upi > 0) {
      const int n = (cstart[c + 1] - cstart[c]) * upi;
      for (int u = blockIdx.x; u < n; u += gridDim.x) {
        const ItemD& it = items[cstart[c] + u / upi];
        fwd_unit_any(it, u % upi, ls, vec, vec);
      }
      level_sync<SW>(bar);
    }
  }
}

template <bool SW>
__global__ void __launch_bounds__(kThreads) bwd_level_kernel(const ItemD* __restrict__ items,
                                                             const int32_t* __restrict__ cstart,
                                                             int ncolours, LevelState ls, double* vec,
                                                             GridBar* bar, int upi) {
  extern __shared__ double lds[];
  for (int c = ncolours - 1; c >= 0; --c) {
    if (upi > 0) {
      const int n = (cstart[c + 1] - cstart[c]) * upi;
      for (int u = blockIdx.x; u < n; u += gridDim.x) {
        const ItemD& it = items[cstart[c] + u / upi];
        if (it.m >= kSweepSplitM) bwd_unit(it, u % upi, ls, vec, lds);
      }
      level_sync<SW>(bar);
    }
    for (int i = cstart[c] + blockIdx.x; i < cstart[c + 1]; i += gridDim.x) {
      const ItemD& it = items[i];
      bwd_any(it, upi > 0, ls, vec, lds);
    }
    if (upi == 0) {
      if (c == 0) break;
      if (cstart[c + 1] - cstart[c] <= 1 && cstart[c] - cstart[c - 1] <= 1) {
        __syncthreads();
        continue;
      }
    }
    level_sync<SW>(bar);
  }
}

// Sweep kernels may use more than 64 KiB of dynamic LDS.
static void allow_sweep_lds() {
  static bool done[6] = {false, false, false, false, false, false};
  allow_lds(reinterpret_cast<const void*>(fwd_kernel), &done[0]);
  allow_lds(reinterpret_cast<const void*>(bwd_kernel), &done[1]);
  allow_lds(reinterpret_cast<const void*>(fwd_level_kernel<false>), &done[2]);
  allow_lds(reinterpret_cast<const void*>(bwd_level_kernel<false>), &done[3]);
  allow_lds(reinterpret_cast<const void*>(fwd_level_kernel<true>), &done[4]);
  allow_lds(reinterpret_cast<const void*>(bwd_level_kernel<true>), &done[5]);
}

int sweep_units(bool forward, int max_m, int max_acap) {
  if (max_m < kSweepSplitM) return 0;
  return forward ? std::max(1, (max_acap + kSweepCols - 1) / kSweepCols)
                 : (max_m + kSweepRows - 1) / kSweepRows;
}

void launch_fwd(const ItemD* items, int nitems, int max_m, int max_acap, LevelState ls, double* vec,
                hipStream_t st, double* shadow) {
  if (nitems <= 0) return;
  allow_sweep_lds();
  const int upi = sweep_units(true, max_m, max_acap);
  if (!(shadow && upi > 0 && max_m <= kInvMaxDofs && !ls.nodc)) shadow = nullptr;
  if (shadow)
    hipLaunchKernelGGL(fwd_rows_kernel, dim3(nitems, (max_m + 63) / 64), dim3(kThreads), 0, st, items, ls, vec,
                       shadow);
  else
    hipLaunchKernelGGL(fwd_kernel, dim3(nitems), dim3(kThreads), sweep_lds(max_m), st, items, nitems, ls, vec,
                       upi > 0 ? 1 : 0);
  if (upi > 0)
    hipLaunchKernelGGL(fwd_units_kernel, dim3(nitems * upi), dim3(kThreads), 0, st, items, ls, vec, upi, shadow);
}

void launch_bwd(const ItemD* items, int nitems, int max_m, int max_acap, LevelState ls, double* vec,
                hipStream_t st, double* shadow) {
  if (nitems <= 0) return;
  allow_sweep_lds();
  const int upi = sweep_units(false, max_m, max_acap);
  if (!(shadow && upi > 0 && max_m <= kInvMaxDofs && !ls.nodc)) shadow = nullptr;
  if (upi > 0)
    hipLaunchKernelGGL(bwd_units_kernel, dim3(nitems * upi), dim3(kThreads), (1024 + 256) * sizeof(double), st,
                       items, ls, vec, upi, shadow);
  if (shadow)
    hipLaunchKernelGGL(bwd_cols_kernel, dim3(nitems, (max_m + 63) / 64), dim3(kThreads), 0, st, items, ls, vec,
                       shadow);
  else
    hipLaunchKernelGGL(bwd_kernel, dim3(nitems), dim3(kThreads), sweep_lds(max_m), st, items, nitems, ls, vec,
                       upi > 0 ? 1 : 0);
}

hipError_t launch_sweep_level(bool forward, const ItemD* items, const int32_t* cstart, int ncolours,
                              int nitems, int max_items, int max_m, int max_acap, LevelState ls, double* vec,
                              hipStream_t st, int grid_cap, GridBar* bar, int64_t vlo, int64_t vn) {
  if (max_m <= kSweepWaveM) {
    constexpr int nw = kSweepWaveThreads / 64;
    int want = std::max(1, (max_items + nw - 1) / nw);
    if (grid_cap > 0) want = std::min(want, grid_cap);
    static bool lds_ok[4] = {false, false, false, false};
    const size_t tbytes = (size_t)nitems * kSweepWaveTableBytes;
    int table = tbytes <= kSweepWaveTableMax ? 1 : 0;
    // 32-bit vector indices when the whole level vector lies below 2^31
    if (table && vn > 0 && vlo + vn < ((int64_t)1 << 31)) table = 2;
    const size_t lds = table ? tbytes : 0;
    if (want == 1 || bar) {
      const int g = std::min(want, device_cus());
      const void* fn = forward ? reinterpret_cast<const void*>(sweep_wave_kernel<true, true>)
                               : reinterpret_cast<const void*>(sweep_wave_kernel<false, true>);
      allow_lds(fn, &lds_ok[forward ? 0 : 1]);
      if (forward)
        hipLaunchKernelGGL((sweep_wave_kernel<true, true>), dim3(g), dim3(kSweepWaveThreads), lds, st, items, cstart,
                           ncolours, ls, vec, bar, table);
      else
        hipLaunchKernelGGL((sweep_wave_kernel<false, true>), dim3(g), dim3(kSweepWaveThreads), lds, st, items,
                           cstart, ncolours, ls, vec, bar, table);
      return hipGetLastError();
    }
    const void* fn = forward ? reinterpret_cast<const void*>(sweep_wave_kernel<true, false>)
                             : reinterpret_cast<const void*>(sweep_wave_kernel<false, false>);
    allow_lds(fn, &lds_ok[forward ? 2 : 3]);
    const int g = coop_grid(fn, lds, want, grid_cap);
    GridBar* none = nullptr;
    void* args[] = {(void*)&items, (void*)&cstart, (void*)&ncolours, (void*)&ls, (void*)&vec, (void*)&none,
                    (void*)&table};
    return hipLaunchCooperativeKernel(fn, dim3(g), dim3(kSweepWaveThreads), args, lds, st);
  }
  allow_sweep_lds();
  const size_t lds = sweep_lds(max_m);
  int upi = sweep_units(forward, max_m, max_acap);
  const int want = std::max(max_items, max_items * upi);
  if (bar) {
    int g = std::max(1, std::min(want, device_cus()));
    if (grid_cap > 0) g = std::min(g, grid_cap);
    if (forward)
      hipLaunchKernelGGL(fwd_level_kernel<true>, dim3(g), dim3(kThreads), lds, st, items, cstart, ncolours,
                         ls, vec, bar, upi);
    else
      hipLaunchKernelGGL(bwd_level_kernel<true>, dim3(g), dim3(kThreads), lds, st, items, cstart, ncolours,
                         ls, vec, bar, upi);
    return hipGetLastError();
  }
  const void* fn = forward ? reinterpret_cast<const void*>(fwd_level_kernel<false>)
                           : reinterpret_cast<const void*>(bwd_level_kernel<false>);
  const int g = coop_grid(fn, lds, want, grid_cap);
  GridBar* none = nullptr;
  void* args[] = {(void*)&items, (void*)&cstart, (void*)&ncolours, (void*)&ls, (void*)&vec, (void*)&none,
                  (void*)&upi};
  return hipLaunchCooperativeKernel(fn, dim3(g), dim3(kThreads), args, lds, st);
}

__global__ void __launch_bounds__(kThreads) top_solve_kernel(const double* L, int n, double* yg) {
  extern __shared__ double lds[];
  double* y = lds;
  double* blk = lds + ((n + 63) / 64) * 64;  // 64*65 doubles
  for (int i = threadIdx.x; i < n; i += kThreads) y[i] = yg[i];
  __syncthreads();
  trsv_lower(L, n, n, y, blk);
  trsv_lower_t<kMaxClusterDofs / 64>(L, n, n, y, blk);
  for (int i = threadIdx.x; i < n; i += kThreads) yg[i] = y[i];
}



// ---------------------------------------------------------------------------
// Dense tops larger than one workgroup's Cholesky (kSplitMaxDofs < n <=
// kTopMaxDofs): right-looking blocked Cholesky over blocks of kTB columns,
// three launches per block: the diagonal block factored and inverted by one
// workgroup in LDS; every row tile below it, L_ip = A_ip L_pp^{-T} on MFMA
// f64 (one workgroup each); every tile of the trailing lower triangle, A_ij
// -= L_ip L_jp^T on MFMA f64 (one workgroup each).  The buffer holds n x (n
// + kTB) doubles (ld n): the last kTB columns receive, in the rows of each
// diagonal block, its inverse (read by the panel and by the solve).
constexpr int kTB = 64, kTLd = kTB + 1;

// Row-major kTB x kTB tile (rows r0.., columns c0.. of the column-major A,
// ld) into LDS with row stride kTLd; entries beyond nr rows or nc columns
// are zeros.
__device__ __forceinline__ void load_tile(const double* A, size_t ld, int r0, int c0, int nr, int nc, double* T) {
  for (int e0 = threadIdx.x; e0 < kTB * kTB; e0 += kThreads * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kThreads, c = e / kTB, r = e - c * kTB;
      v[u] = (e < kTB * kTB && r < nr && c < nc) ? A[(size_t)(r0 + r) + ld * (size_t)(c0 + c)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kThreads, c = e / kTB, r = e - c * kTB;
      if (e < kTB * kTB) T[r * kTLd + c] = v[u];
    }
  }
}

// The transpose: T[c * kTLd + r] = X(r0 + r, c0 + c) (rows r < nr, columns
// c < nc; zeros elsewhere), so that tile_abt multiplies by X itself.
__device__ __forceinline__ void load_tile_t(const double* X, size_t ld, int r0, int c0, int nr, int nc, double* T) {
  for (int e0 = threadIdx.x; e0 < kTB * kTB; e0 += kThreads * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kThreads, c = e / kTB, r = e - c * kTB;
      v[u] = (e < kTB * kTB && r < nr && c < nc) ? X[(size_t)(r0 + r) + ld * (size_t)(c0 + c)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kThreads, c = e / kTB, r = e - c * kTB;
      if (e < kTB * kTB) T[c * kTLd + r] = v[u];
    }
  }
}

// X = As Bs^T for two kTB x kTB tiles in LDS (row stride kTLd): wave w
// computes the 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 tiles of
// v_mfma_f64_16x16x4; acc[a][b][v] is X(32 (w/2) + 16 a + 4 v + lane/16,
// 32 (w%2) + 16 b + lane%16).
__device__ __forceinline__ void tile_abt(const double* As, const double* Bs, d4_t acc[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane >> 4, lc = lane & 15;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int s4 = 0; s4 < kTB / 4; ++s4) {
    double av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = As[(r0 + 16 * a + lc) * kTLd + 4 * s4 + lr];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = Bs[(c0 + 16 * b + lc) * kTLd + 4 * s4 + lr];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
}

// Stores acc (the tile_abt layout) into rows r0.., columns c0.. of A (ld):
// op 0 stores, op 1 subtracts; rows >= nr, columns >= nc and, with lower,
// entries above the diagonal are left alone.
__device__ __forceinline__ void store_tile(double* A, size_t ld, int r0, int c0, int nr, int nc, bool lower, int op,
                                           const d4_t acc[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane >> 4, lc = lane & 15;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 32 * (w >> 1) + 16 * a + 4 * v + lr, c = 32 * (w & 1) + 16 * b + lc;
        if (r < nr && c < nc && (!lower || r >= c)) {
          double* x = A + (size_t)(r0 + r) + ld * (size_t)(c0 + c);
          *x = op ? *x - acc[a][b][v] : acc[a][b][v];
        }
      }
}

// Diagonal block p of a large top, one workgroup, in LDS: Cholesky by
// 16-column panels (the 16 x 16 diagonal part by wave 0 with its rows in
// registers and readlane broadcasts, the rows below by one thread each, the
// trailing triangle by all threads), then thread c forms column c of the
// inverse by forward substitution (four partial sums per entry).  Stores
// L_pp (lower) in place and L_pp^{-1} in the extra columns.  A pivot that is
// not > 0 is replaced by 1 and reported in the error words (bits == 0) or as
// the error bit of a batched system.
// S: kTB x kTLd doubles of LDS, rd: kTB, Xs: kTB x kTB, sbad: an int of LDS
// (kTB (kTLd + kTB + 1) doubles in all).
constexpr int kDiagLds = kTB * (kTLd + kTB + 1);
__device__ __forceinline__ void dense_diag_block(double* A, int n, int p, int32_t* err, int bits, double* S,
                                                 double* rd, double* Xs, int& sbad) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rp = p * kTB, np = min(kTB, n - rp);
  // the block (identity beyond np), eight loads in flight per thread
  for (int e0 = tid; e0 < kTB * kTB; e0 += kThreads * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kThreads, c = e / kTB, r = e - c * kTB;
      v[u] = (r < np && c < np) ? (r >= c ? A[(size_t)(rp + r) + (size_t)n * (rp + c)] : 0.0) : (r == c ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kThreads, c = e / kTB, r = e - c * kTB;
      S[r * kTLd + c] = v[u];
    }
  }
  if (tid == 0) sbad = 0;
  __syncthreads();
#pragma unroll
  for (int kb = 0; kb < kTB; kb += 16) {
    if (wv == 0) {
      double row[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) row[u] = (lane < 16 && u <= lane) ? S[(kb + lane) * kTLd + kb + u] : 0.0;
      bool bad = false;
      double rdl = 1.0;
      // one branch-free block: the pivot test and lane u's reciprocal are
      // selects, so the pivots' dependency chains can be scheduled together
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        double d = readlane_d(row[u], u);
        const bool nonpos = !(d > 0.0);
        bad = bad || (nonpos && kb + u < np);
        d = nonpos ? 1.0 : d;
        // 1 / sqrt(d) from v_rsq_f64 refined by two Newton steps, sqrt(d)
        // as d times it (no divide or square-root sequence on the chain)
        double rs = __builtin_amdgcn_rsq(d);
        rs = rs + rs * (0.5 - 0.5 * d * rs * rs);
        rs = rs + rs * (0.5 - 0.5 * d * rs * rs);
        const double piv = d * rs;
        // every lane computes; only the lower part of the panel's diagonal
        // tile (lane >= the column, lane < 16) is ever read again
        rdl = lane == u ? rs : rdl;
        row[u] = lane == u ? piv : row[u] * rs;
#pragma unroll
        for (int v = u + 1; v < 16; ++v) {
          const double lvu = readlane_d(row[u], v);
          row[v] -= row[u] * lvu;
        }
      }
      if (lane < 16) {
        rd[kb + lane] = rdl;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (u <= lane) S[(kb + lane) * kTLd + kb + u] = row[u];
      }
      if (bad && lane == 0) sbad = 1;
    }
    __syncthreads();
    // rows below: x L11^T = a, one thread per row
    for (int r = kb + 16 + tid; r < kTB; r += kThreads) {
      double x[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) x[u] = S[r * kTLd + kb + u];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        double t = x[u];
#pragma unroll
        for (int v = 0; v < u; ++v) t -= x[v] * S[(kb + u) * kTLd + kb + v];
        x[u] = t * rd[kb + u];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) S[r * kTLd + kb + u] = x[u];
    }
    __syncthreads();
    // trailing triangle: S[r][c] -= sum_k S[r][kb+k] S[c][kb+k], r >= c >= kb + 16
    const int rem = kTB - kb - 16;
    for (int e = tid; e < rem * (rem + 1) / 2; e += kThreads) {
      int rr = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while ((rr + 1) * (rr + 2) / 2 <= e) ++rr;
      while (rr * (rr + 1) / 2 > e) --rr;
      const int cc = e - rr * (rr + 1) / 2;
      const int r = kb + 16 + rr, c = kb + 16 + cc;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) acc += S[r * kTLd + kb + k] * S[c * kTLd + kb + k];
      S[r * kTLd + c] -= acc;
    }
    __syncthreads();
  }
  // the factor to A
  for (int e = tid; e < kTB * kTB; e += kThreads) {
    const int c = e / kTB, r = e - c * kTB;
    if (r < np && c < np && r >= c) A[(size_t)(rp + r) + (size_t)n * (rp + c)] = S[r * kTLd + c];
  }
  // L_pp^{-1} by 16 x 16 tiles in Xs (64 x 64, ld 64): wave w inverts the
  // diagonal tile w (lane c < 16 forms column c by forward substitution),
  // then the tiles below the diagonal follow on MFMA by distance from it,
  // X_ij = -X_ii (sum_{k=j}^{i-1} L_ik X_kj) for i - j = 1, 2, 3 in turn
  {
    const int w0 = 16 * wv;
    if (lane < 16) {
      double x[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < r; ++q) s += S[(w0 + r) * kTLd + w0 + q] * x[q];
        x[r] = ((r == lane ? 1.0 : 0.0) - s) * rd[w0 + r];
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) Xs[(w0 + r) * kTB + w0 + lane] = x[r];
    }
    __syncthreads();
    const int lr = lane >> 4, lc = lane & 15;
    for (int d = 1; d < 4; ++d) {
      const int ti = wv + d, tj = wv;  // this wave's tile at distance d
      if (ti < 4) {
        d4_t t = {0.0, 0.0, 0.0, 0.0};
        for (int kt = tj; kt < ti; ++kt) {
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
            t = __builtin_amdgcn_mfma_f64_16x16x4f64(S[(16 * ti + lc) * kTLd + 16 * kt + 4 * s4 + lr],
                                                     Xs[(16 * kt + 4 * s4 + lr) * kTB + 16 * tj + lc], t, 0, 0, 0);
        }
        d4_t x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
          x = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[(16 * ti + lc) * kTB + 16 * ti + 4 * s4 + lr], t[s4], x, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) Xs[(16 * ti + 4 * v + lr) * kTB + 16 * tj + lc] = -x[v];
      }
      __syncthreads();
    }
    // to the extra columns, zeros above the diagonal
    for (int e = tid; e < kTB * kTB; e += kThreads) {
      const int c = e / kTB, r = e - c * kTB;
      if (r < np && c < np) A[(size_t)n * n + (size_t)(rp + r) + (size_t)n * c] = r >= c ? Xs[r * kTB + c] : 0.0;
    }
  }
  if (sbad && tid == 0) {
    if (bits) atomicOr(err, 1 << kErrNotSPD);
    else set_error(err, -1, -1, kErrNotSPD);
  }
}

__global__ void __launch_bounds__(kThreads) dense_diag_kernel(double* A, int n, int p, int32_t* err, int bits) {
  extern __shared__ double lds[];  // the block (row-major, lower part used), 1 / L_jj, the inverse
  __shared__ int sbad;
  dense_diag_block(A, n, p, err, bits, lds, lds + kTB * kTLd, lds + kTB * kTLd + kTB, sbad);
}

// Panel launch of step p: workgroup b < T takes row tile i = p + 1 + b, L_ip
// = A_ip L_pp^{-T} with the inverse from dense_diag_kernel; with the
// inverse X of the whole factor being formed (X != null), workgroup T + c
// (c <= p) finishes tile (p, c) of X: X_pp = L_pp^{-1}, X_pc = L_pp^{-1}
// R_pc, where R_pc = -sum_{q<p} L_pq X_qc has been accumulated in place.
__global__ void __launch_bounds__(kThreads) dense_panel_kernel(double* A, int n, int p, int T, double* X) {
  extern __shared__ double lds[];
  double* As = lds;
  double* Bs = lds + kTB * kTLd;
  const int rp = p * kTB, np = min(kTB, n - rp);
  if ((int)blockIdx.x >= T) {
    const int c = blockIdx.x - T, rc = c * kTB;
    if (c == p) {
      for (int e = threadIdx.x; e < np * np; e += kThreads) {
        const int cc = e / np, r = e - cc * np;
        X[(size_t)(rp + r) + (size_t)n * (rp + cc)] = A[(size_t)n * n + (size_t)(rp + r) + (size_t)n * cc];
      }
      return;
    }
    load_tile(A + (size_t)n * n, n, rp, 0, np, np, As);  // L_pp^{-1}
    load_tile_t(X, n, rp, rc, np, kTB, Bs);              // R_pc
    __syncthreads();
    d4_t acc[2][2];
    tile_abt(As, Bs, acc);
    store_tile(X, n, rp, rc, np, kTB, false, 0, acc);
    return;
  }
  const int i = p + 1 + blockIdx.x;
  const int ri = i * kTB;
  const int ni = min(kTB, n - ri);
  load_tile(A, n, ri, rp, ni, np, As);                 // A_ip
  load_tile(A + (size_t)n * n, n, rp, 0, np, np, Bs);  // L_pp^{-1}
  __syncthreads();
  d4_t acc[2][2];
  tile_abt(As, Bs, acc);  // A_ip L_pp^{-T}
  store_tile(A, n, ri, rp, ni, np, false, 0, acc);
}

// Update launch of step p: workgroup t < T(T+1)/2 takes lower tile (i, j),
// p < j <= i, in row order of the triangle; with X, the further workgroups
// take the tiles (i, c), i > p, c <= p, of the inverse's accumulators:
// R_ic -= L_ip X_pc.  Workgroup 0, whose tile (p+1, p+1) is then final,
// goes on to factor and invert that diagonal block (the diagonal step of
// step p + 1, while the other tiles are still being updated).
__global__ void __launch_bounds__(kThreads) dense_update_kernel(double* A, int n, int p, int T, double* X,
                                                                int32_t* err, int bits) {
  extern __shared__ double lds[];
  __shared__ int sbad;
  double* As = lds;
  double* Bs = lds + kTB * kTLd;
  const int ntri = T * (T + 1) / 2;
  if ((int)blockIdx.x >= ntri) {
    const int u = blockIdx.x - ntri;
    const int i = p + 1 + u / (p + 1), c = u % (p + 1);
    const int ri = i * kTB, rp = p * kTB, rc = c * kTB;
    const int ni = min(kTB, n - ri), np = min(kTB, n - rp);
    load_tile(A, n, ri, rp, ni, np, As);    // L_ip
    load_tile_t(X, n, rp, rc, np, kTB, Bs);  // X_pc
    __syncthreads();
    d4_t acc[2][2];
    tile_abt(As, Bs, acc);
    store_tile(X, n, ri, rc, ni, kTB, false, 1, acc);
    return;
  }
  const int t = blockIdx.x;
  int ii = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
  while (ii * (ii + 1) / 2 > t) --ii;
  const int jj = t - ii * (ii + 1) / 2;
  const int i = p + 1 + ii, j = p + 1 + jj;
  const int ri = i * kTB, rj = j * kTB, rp = p * kTB;
  const int ni = min(kTB, n - ri), nj = min(kTB, n - rj), np = min(kTB, n - rp);
  load_tile(A, n, ri, rp, ni, np, As);  // L_ip
  load_tile(A, n, rj, rp, nj, np, Bs);  // L_jp
  __syncthreads();
  d4_t acc[2][2];
  tile_abt(As, Bs, acc);
  store_tile(A, n, ri, rj, ni, nj, i == j, 1, acc);
  if (t == 0) {
    // the stores above, made visible to the whole workgroup (device-scope
    // fences on both sides of the barrier, so no stale cached line is read)
    __threadfence();
    __syncthreads();
    __threadfence();
    dense_diag_block(A, n, p + 1, err, bits, lds, lds + kTB * kTLd, lds + kTB * kTLd + kTB, sbad);
  }
}

void launch_top_potrf_blocked(double* A, int n, int32_t* err, int bits, hipStream_t st, double* X) {
  if (n <= 0) return;
  static bool done[3] = {false, false, false};
  allow_lds(reinterpret_cast<const void*>(dense_panel_kernel), &done[0]);
  allow_lds(reinterpret_cast<const void*>(dense_update_kernel), &done[1]);
  allow_lds(reinterpret_cast<const void*>(dense_diag_kernel), &done[2]);
  const size_t lds = (size_t)2 * kTB * kTLd * sizeof(double);
  static_assert(kDiagLds <= 2 * kTB * kTLd, "the update launch's LDS holds the diagonal step's");
  const int nt = (n + kTB - 1) / kTB;
  if (X) launch_zero(X, (int64_t)n * n, st);
  // the diagonal block of step p + 1 is factored by the update launch of
  // step p (its workgroup 0), the first one by a launch of its own
  hipLaunchKernelGGL(dense_diag_kernel, dim3(1), dim3(kThreads), (size_t)kDiagLds * sizeof(double), st, A, n, 0,
                     err, bits);
  for (int p = 0; p < nt; ++p) {
    const int T = nt - p - 1;
    const int gp = T + (X ? p + 1 : 0);
    if (gp > 0)
      hipLaunchKernelGGL(dense_panel_kernel, dim3(gp), dim3(kThreads), lds, st, A, n, p, T, X);
    const int gu = T * (T + 1) / 2 + (X ? T * (p + 1) : 0);
    if (gu > 0)
      hipLaunchKernelGGL(dense_update_kernel, dim3(gu), dim3(kThreads), lds, st, A, n, p, T, X, err, bits);
  }
}

// y <- X^T X y for the lower inverse X (n x n, ld n) of a large top's
// factor, over the 64 x 64 tiles (i, c), i >= c, of its lower triangle (one
// workgroup per tile, T(T+1)/2 of them for T = ceil(n / 64) tile rows) in
// three launches: P_c(i) = X_ic y_c; then z_i = sum_{c <= i} P_c(i) (every
// tile of row i forms the same z_i, in the order c = 0..i) and Q_i(c) =
// X_ic^T z_i; then y_c = sum_{i >= c} Q_i(c) in the order i = c..T-1.  P and
// Q hold T x n doubles each (P_c at P + c n, Q_i at Q + i n).  Every sum has
// one fixed order: four interleaved partial sums combined as (0+1)+(2+3).
__global__ void __launch_bounds__(kThreads) top_inv_part_kernel(const double* X, int n, const double* y,
                                                                double* P) {
  __shared__ double red[4 * 64];
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  int i, c;
  tri_index(blockIdx.x, i, c);
  const int ri = i * kTB, rc = c * kTB, ni = min(kTB, n - ri), nc = min(kTB, n - rc);
  double xv[16], yv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int col = g * 16 + u;
    const bool ok = o < ni && col < nc && (i != c || col <= o);
    xv[u] = ok ? X[(size_t)(ri + o) + (size_t)n * (rc + col)] : 0.0;
    yv[u] = col < nc ? y[rc + col] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s += xv[u] * yv[u];
  red[g * 64 + o] = s;
  __syncthreads();
  if (threadIdx.x < ni)
    P[(size_t)c * n + ri + threadIdx.x] =
        (red[threadIdx.x] + red[64 + threadIdx.x]) + (red[128 + threadIdx.x] + red[192 + threadIdx.x]);
}

__global__ void __launch_bounds__(kThreads) top_inv_mid_kernel(const double* X, int n, const double* P,
                                                               double* Q) {
  __shared__ double S[kTB * kTLd];  // S[col * kTLd + r] = X_ic(r, col)
  __shared__ double zs[kTB];
  __shared__ double red[4 * 64];
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  int i, c;
  tri_index(blockIdx.x, i, c);
  const int ri = i * kTB, rc = c * kTB, ni = min(kTB, n - ri), nc = min(kTB, n - rc);
  double xv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int col = g * 16 + u;
    const bool ok = o < ni && col < nc && (i != c || col <= o);
    xv[u] = ok ? X[(size_t)(ri + o) + (size_t)n * (rc + col)] : 0.0;
  }
  double s = 0.0;
  if (o < ni)
    for (int cp = g; cp <= i; cp += 4) s += P[(size_t)cp * n + ri + o];
  red[g * 64 + o] = s;
#pragma unroll
  for (int u = 0; u < 16; ++u) S[(g * 16 + u) * kTLd + o] = xv[u];
  __syncthreads();
  if (threadIdx.x < kTB)
    zs[threadIdx.x] = (red[threadIdx.x] + red[64 + threadIdx.x]) + (red[128 + threadIdx.x] + red[192 + threadIdx.x]);
  __syncthreads();
  // column o of the tile against z_i, rows g*16 .. g*16 + 15
  s = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s += S[o * kTLd + g * 16 + u] * zs[g * 16 + u];
  red[g * 64 + o] = s;
  __syncthreads();
  if (threadIdx.x < nc)
    Q[(size_t)i * n + rc + threadIdx.x] =
        (red[threadIdx.x] + red[64 + threadIdx.x]) + (red[128 + threadIdx.x] + red[192 + threadIdx.x]);
}

__global__ void __launch_bounds__(kThreads) top_inv_sum_kernel(const double* Q, int n, int T, double* y) {
  __shared__ double red[4 * 64];
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int c = blockIdx.x, rc = c * kTB, nc = min(kTB, n - rc);
  double s = 0.0;
  if (o < nc)
    for (int i = c + g; i < T; i += 4) s += Q[(size_t)i * n + rc + o];
  red[g * 64 + o] = s;
  __syncthreads();
  if (threadIdx.x < nc)
    y[rc + threadIdx.x] = (red[threadIdx.x] + red[64 + threadIdx.x]) + (red[128 + threadIdx.x] + red[192 + threadIdx.x]);
}

void launch_top_solve(const double* L, int n, double* y, hipStream_t st) {
  if (n <= 0) return;
  size_t lds = ((size_t)((n + 63) / 64) * 64 + 64 * kBlkLd) * sizeof(double);
  if (n > kSplitMaxDofs) {
    // the factor's inverse X (formed by the blocked Cholesky) sits after the
    // n x (n + 64) factor; the 64 columns after the factor hold P, the 64
    // after X hold Q (T <= 64 tile rows since n <= kTopMaxDofs)
    const double* X = L + (size_t)n * (n + 64);
    double* P = const_cast<double*>(L) + (size_t)n * n;
    double* Q = const_cast<double*>(X) + (size_t)n * n;
    const int nt = (n + kTB - 1) / kTB, ntile = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(top_inv_part_kernel, dim3(ntile), dim3(kThreads), 0, st, X, n, y, P);
    hipLaunchKernelGGL(top_inv_mid_kernel, dim3(ntile), dim3(kThreads), 0, st, X, n, P, Q);
    hipLaunchKernelGGL(top_inv_sum_kernel, dim3(nt), dim3(kThreads), 0, st, Q, n, nt, y);
    return;
  }
  static bool lds_ok = false;
  allow_lds(reinterpret_cast<const void*>(top_solve_kernel), &lds_ok);
  hipLaunchKernelGGL(top_solve_kernel, dim3(1), dim3(kThreads), lds, st, L, n, y);
}

// Dense tops of a batch: one workgroup per system.
__global__ void __launch_bounds__(kThreads) top_potrf_batched_kernel(const TopD* __restrict__ tops) {
  extern __shared__ double lds[];
  __shared__ int sbad;
  const TopD t = tops[blockIdx.x];
  // tops of 64..512 unknowns take the MFMA Cholesky of one workgroup, larger
  // ones the blocked Cholesky over several (as a single system's top does,
  // so that each system's factor is the same bits)
  if (t.n <= 0 || t.n >= 64) return;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  chol_solve(t.L, t.n, t.n, nullptr, 0, lds, &sbad);
  __syncthreads();
  if (sbad && threadIdx.x == 0) atomicOr(t.err, 1 << kErrNotSPD);
}

void launch_top_potrf_batched(const TopD* tops, int ntops, int max_n, hipStream_t st) {
  if (ntops <= 0 || max_n <= 0) return;
  static bool lds_ok = false;
  allow_lds(reinterpret_cast<const void*>(top_potrf_batched_kernel), &lds_ok);
  size_t lds = ((size_t)max_n * kNB + kNB * kNB + kNB * 256) * sizeof(double);
  hipLaunchKernelGGL(top_potrf_batched_kernel, dim3(ntops), dim3(kThreads), lds, st, tops);
  if (max_n >= 64) launch_top_potrf_wg_batched(tops, ntops, std::min(max_n, kSplitMaxDofs), st);
}

__global__ void __launch_bounds__(kThreads) top_solve_batched_kernel(const TopD* __restrict__ tops,
                                                                     double* vec) {
  extern __shared__ double lds[];
  const TopD t = tops[blockIdx.x];
  const int n = t.n;
  if (n <= 0) return;
  double* y = lds;
  double* blk = lds + ((n + 63) / 64) * 64;
  double* yg = vec + t.voff;
  for (int i = threadIdx.x; i < n; i += kThreads) y[i] = yg[i];
  __syncthreads();
  trsv_lower(t.L, n, n, y, blk);
  trsv_lower_t<kMaxClusterDofs / 64>(t.L, n, n, y, blk);
  for (int i = threadIdx.x; i < n; i += kThreads) yg[i] = y[i];
}

void launch_top_solve_batched(const TopD* tops, int ntops, int max_n, double* vec, hipStream_t st) {
  if (ntops <= 0 || max_n <= 0) return;
  static bool lds_ok = false;
  allow_lds(reinterpret_cast<const void*>(top_solve_batched_kernel), &lds_ok);
  size_t lds = ((size_t)((max_n + 63) / 64) * 64 + 64 * kBlkLd) * sizeof(double);
  hipLaunchKernelGGL(top_solve_batched_kernel, dim3(ntops), dim3(kThreads), lds, st, tops, vec);
}

// ---------------------------------------------------------------------------
__global__ void zero_kernel(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}
__global__ void zero_i32_kernel(int32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Factor store of one cluster after its level (one workgroup per cluster):
// S = [M0 | C | V | tau] with M0 the m x m diagonal-block factor (W = U^T
// G^{-1} or G^{-1} when the factorization formed them, else the panel's
// diagonal block: G, or without deferred compression G_f with F_c and D_c),
// C the panel's a near-field columns, V the k reflectors in step order
// (column j = the far-field column of pivot j) and tau their factors.  A
// cluster whose k or a exceed the store's capacities (ranks other than the
// layout was planned for, which the host detects and answers by a new
// factorization) is left alone.
__global__ void __launch_bounds__(256) compact_kernel(const ItemD* __restrict__ items, LevelState ls) {
  const ItemD& it = items[blockIdx.x];
  const int m = it.m;
  if (m == 0 || !it.S) return;
  const int k = ls.k[it.s], a = ls.a[it.s], gk = ls.giok[it.s];
  if (k > it.sk || a > it.sa) return;
  const size_t mm = (size_t)m * m;
  const double* M0 = (gk == 1 || gk == 2) ? it.Gi : it.P;
  double* S = it.S;
  const size_t n0 = mm + (size_t)m * a, nv = (size_t)m * k;
  for (size_t e0 = threadIdx.x; e0 < n0; e0 += 256 * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const size_t e = e0 + (size_t)u * 256;
      v[u] = e < n0 ? (e < mm ? M0[e] : it.P[e]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const size_t e = e0 + (size_t)u * 256;
      if (e < n0) S[e] = v[u];
    }
  }
  const double* Wf = it.P + (size_t)m * (m + a);
  double* V = S + n0;
  for (size_t e = threadIdx.x; e < nv; e += 256) {
    const int j = (int)(e / m), i = (int)(e - (size_t)j * m);
    V[e] = Wf[(size_t)m * it.piv[j] + i];
  }
  for (int j = threadIdx.x; j < k; j += 256) V[nv + j] = it.tau[j];
}

static int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

void launch_compact(const ItemD* items, int nitems, LevelState ls, hipStream_t st) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(compact_kernel, dim3(nitems), dim3(256), 0, st, items, ls);
}

void launch_zero(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n);
}
void launch_zero_i32(int32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n);
}

__global__ void scatter_vals_kernel(const double* val, const int64_t* off, int64_t nnz, double* base) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = off[e];
    if (o >= 0) base[o] = val[e];
  }
}
void launch_scatter_vals(const double* val, const int64_t* off, int64_t nnz, double* base,
                         hipStream_t st) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(scatter_vals_kernel, dim3(grid_for(nnz)), dim3(256), 0, st, val, off, nnz,
                     base);
}

__global__ void scatter_vals_multi_kernel(const ScatterD* __restrict__ d) {
  const ScatterD t = d[blockIdx.y];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < t.nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = t.off[e];
    if (o >= 0) t.base[o] = t.val[e];
  }
}

void launch_scatter_vals_multi(const ScatterD* d, int nd, int64_t max_nnz, hipStream_t st) {
  if (nd <= 0 || max_nnz <= 0) return;
  const int gx = (int)std::min<int64_t>(64, (max_nnz + 255) / 256);
  hipLaunchKernelGGL(scatter_vals_multi_kernel, dim3(gx, nd), dim3(256), 0, st, d);
}

__global__ void copy_blocks_kernel(const CopyD* tasks) {
  const CopyD t = tasks[blockIdx.x];
  const int64_t n = (int64_t)t.rows * t.cols;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = (int)(e % t.rows), c = (int)(e / t.rows);
    const double v = t.trans ? t.src[(size_t)c + (size_t)t.sld * r] : t.src[(size_t)r + (size_t)t.sld * c];
    t.dst[(size_t)r + (size_t)t.dld * c] = v;
  }
}
void launch_copy_blocks(const CopyD* tasks, int ntasks, hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(copy_blocks_kernel, dim3(ntasks), dim3(256), 0, st, tasks);
}

__global__ void gather_kernel(const double* src, const int64_t* idx, double* dst, int64_t n) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x)
    dst[j] = src[idx[j]];
}
__global__ void scatter_kernel(const double* src, const int64_t* idx, double* dst, int64_t n) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x)
    dst[idx[j]] = src[j];
}
void launch_gather(const double* src, const int64_t* idx, double* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gather_kernel, dim3(grid_for(n)), dim3(256), 0, st, src, idx, dst, n);
}
void launch_scatter(const double* src, const int64_t* idx, double* dst, int64_t n,
                    hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(n)), dim3(256), 0, st, src, idx, dst, n);
}

// ---------------------------------------------------------------------------
__global__ void spmv_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                            const double* __restrict__ val, const double* __restrict__ x,
                            double* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) s += val[e] * x[col[e]];
    y[i] = s;
  }
}
void launch_spmv(const int64_t* rowptr, const int32_t* col, const double* val, const double* x,
                 double* y, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(spmv_kernel, dim3(grid_for(n)), dim3(256), 0, st, rowptr, col, val, x, y, n);
}

__global__ void __launch_bounds__(256) dot_partial_kernel(const double* x, const double* y, int64_t n,
                                                          double* partial) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
__global__ void __launch_bounds__(256) dot_final_kernel(const double* partial, int np, double* out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += partial[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
void launch_dot(const double* x, const double* y, int64_t n, double* partial, double* out,
                hipStream_t st) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(kDotBlocks), dim3(256), 0, st, x, y, n, partial);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(256), 0, st, partial, kDotBlocks, out);
}

__global__ void pcg_xr_kernel(double* x, double* r, const double* p, const double* q, int64_t n,
                              const double* num, const double* den) {
  const double al = num[0] / den[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += al * p[i];
    r[i] -= al * q[i];
  }
}
void launch_pcg_xr(double* x, double* r, const double* p, const double* q, int64_t n,
                   const double* num, const double* den, hipStream_t st) {
  hipLaunchKernelGGL(pcg_xr_kernel, dim3(grid_for(n)), dim3(256), 0, st, x, r, p, q, n, num, den);
}
__global__ void pcg_p_kernel(double* p, const double* z, int64_t n, const double* num,
                             const double* den) {
  const double be = num[0] / den[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + be * p[i];
}
void launch_pcg_p(double* p, const double* z, int64_t n, const double* num, const double* den,
                  hipStream_t st) {
  hipLaunchKernelGGL(pcg_p_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, z, n, num, den);
}
__global__ void residual_kernel(const double* b, double* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = b[i] - y[i];
}
void launch_residual(const double* b, double* y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(residual_kernel, dim3(grid_for(n)), dim3(256), 0, st, b, y, n);
}
__global__ void copy_kernel(const double* s, double* d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}
void launch_copy(const double* src, double* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, st, src, dst, n);
}

}  // namespace lrsp
