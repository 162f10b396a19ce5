// desc.hpp -- plain-old-data work descriptors shared by the host planner and
// the gfx950 kernels.
//
// Storage of a tree level (all fp64, column-major):
//   D_x         diagonal block of cluster x, m_x x m_x; only its lower
//               triangle is meaningful.
//   fine half   for a linked pair {e,l} with e processed before l and linked
//               when e is processed: the block row of e restricted to the
//               columns Z(e,l) of l that can be nonzero there (m_e x |Z|).
//   coarse half for every pair {e,l} linked by the end of the level: the
//               coupling of l's rows with e's coarse DoFs (m_l x kcap_e);
//               after l is processed its first k_l rows hold the
//               coarse-coarse coupling that the next level assembles.
//   panel P_s   the block row [A_ss | A_sn | A_sw] of cluster s gathered when
//               s is processed; afterwards it holds the factor pieces of s:
//               G (lower), C = U^T G^{-1} A_sn (rows k.. are F), and the
//               reflectors of U in the far-field part.
#pragma once
#include <cstdint>

namespace lrsp {

constexpr int kThreads = 256;       // threads of a cluster workgroup
constexpr int kNB = 16;             // panel width of the blocked Cholesky
constexpr int kMaxClusterDofs = 768;
constexpr int kInvMaxDofs = 256;    // clusters whose G^{-1} is formed explicitly

// One column segment of the block row of the cluster being processed.
struct SegD {
  const double* src;   // m_s rows (ld = m_s); columns of this segment
  const int32_t* zl;   // fine: natural column indices in cluster y; coarse: null
  int64_t voff;        // offset of cluster y in the level vector
  int32_t y;           // cluster id within the level
  int32_t coarse;      // 1: y processed earlier, width = k[y]; 0: fine
  int32_t nfine;       // fine width
  int32_t cap;         // column capacity of the source block
  int32_t isw;         // 0 near field n(s), 1 far field w(s)
  int32_t pad;
};

// Schur-update target of the near-field segment pair (i <= j); stored at
// index j*(j+1)/2 + i.
struct PairD {
  double* dst;
  const int32_t* posmap;  // block column of a natural index of the column
                          // cluster; null = identity
  int32_t ld;
  int32_t rows_from_j;    // rows come from segment j (else from i)
  int32_t diag;           // i == j: lower triangle of a diagonal block
  int32_t nrows;          // bounds of the target block (checked)
  int32_t ncols;
  int32_t pad;
};

// Write-back target of segment i for the coarse row of s.
struct WbD {
  double* dst;
  int32_t ld;
  int32_t trans;  // 0: dst[r + ld*c] (r coarse row of s, c column index);
                  // 1: dst[c + ld*r]
  int32_t nrows;
  int32_t ncols;
};

struct ItemD {
  int32_t s, m, nseg, nsegn;
  int32_t pcap;   // panel column capacity beyond the m diagonal columns
  int32_t kcap;   // capacity for the rank of s
  const SegD* seg;
  const PairD* pair;
  const WbD* wb;
  double* D;        // m x m
  double* P;        // m x (m + pcap)
  double* Gi;       // m x m, G^{-1} (lower) for m <= kInvMaxDofs on levels that
                    // may take the split schedule, else null
  double* S;        // factor store read by the sweeps: [M0 (m x m) | C (m x sa)
                    // | V (m x sk) | tau (sk)], ld m, filled after the level
  int32_t sa, sk;   // near-field columns and rank the store holds room for
  int32_t* colseg;  // [pcap] segment of each panel column
  int32_t* colnat;  // [pcap] natural index of each panel column
  int64_t* vidx;    // [pcap] level-vector index of each near-field column
  int32_t* piv;     // [kcap] far-field column of reflector j
  int32_t* stepof;  // [pcap] reflector step of a far-field column, -1 if none
  double* tau;      // [kcap]
  double* norms;    // [pcap] scratch
  int32_t* segoff;  // [nseg+1] scratch
  int64_t voff;     // offset of s in the level vector
  int32_t* serr;    // error bits (1 << ErrCode) of the system s belongs to,
                    // or null (batched factorizations)
};

// Per-level dynamic results, indexed by cluster.
struct LevelState {
  int32_t* k;     // rank (coarse DoFs kept)
  int32_t* a;     // near-field columns
  int32_t* b;     // far-field columns
  int32_t* err;   // [4]: flag, level, cluster, code (then 4 words of grid barrier)
  int32_t* giok;  // 1: the factorization left G^{-1} in ItemD::Gi;
                  // 2: Gi holds W = U^T G^{-1} (k > 0 reflectors folded in, all
                  //    m x m entries); the backward sweep applies its transpose;
                  // 3: eliminated without deferred compression (the panel holds
                  //    the reflectors of U, the fine factor G_f in rows/columns
                  //    k.. of the diagonal block, F_c in its columns ..k and F_n)
  int32_t nodc = 0;  // 1: eliminate without deferred compression (fused kernels)
};

// dst[r + dld*c] = trans ? src[c + sld*r] : src[r + sld*c], r < rows, c < cols
struct CopyD {
  const double* src;
  double* dst;
  int32_t sld, dld, rows, cols, trans, pad;
};

// Dense top system of one system of a batch: L (n x n, lower after the
// factorization) and its segment of the vector buffer.
struct TopD {
  double* L;
  int64_t voff;
  int32_t* err;  // error bits of the system
  int32_t n;
  int32_t pad;
};

// base[off[e]] = val[e] for e < nnz with off[e] >= 0 (one system of a batch).
struct ScatterD {
  const double* val;
  const int64_t* off;
  double* base;
  int64_t nnz;
};

// Software grid barrier of a persistent launch that is not cooperative
// (launches recorded in graphs).  count returns to 0 after every barrier;
// timeout is set when a wait gave up, after which results are invalid.
struct GridBar {
  uint32_t count;
  uint32_t gen;
  int32_t timeout;
  int32_t pad;
};

// Rank features: one level-start neighbour block of cluster s.
struct FeatSeg {
  const double* H;     // fine half holding the coupling of s and y
  const int32_t* zl;   // natural indices of H's columns
  const double* Dy;    // diagonal block of y (m_y x m_y)
  int32_t ld;          // rows of H
  int32_t ncols;       // columns of H
  int32_t y;           // neighbour cluster
  int32_t my;          // its size
  int32_t orient;      // 0: H = block row of s (columns in y); 1: H = block row of y (columns in s)
  int32_t pad;
};

struct FeatItem {
  const double* Ds;    // diagonal block of s
  const FeatSeg* seg;
  double before;       // fraction of the neighbours processed before s
  int32_t m, nseg, s;
  int32_t bsum;        // summed level-start sizes of the far field of s
};

// n doubles at p (buffer fills of a batch).
struct SpanD {
  double* p;
  int64_t n;
};

enum ErrCode : int32_t {
  kErrNone = 0,
  kErrNotSPD = 1,
  kErrCapacity = 2,
  kErrIndex = 3,
  kErrTooLarge = 4,
};

}  // namespace lrsp
