// api.cpp -- C interface of the hierarchical solver (see include/lrsp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lrsp.h"
#include "desc.hpp"
#include "kernels.hpp"
#include "plan.hpp"

using namespace lrsp;

namespace {

thread_local std::string g_last_error;

lrsp_status fail(lrsp_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

// Event timing of kernel families (lrsp_timing_*).
constexpr int kFamilies = 11;
struct TimingState {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[kFamilies];
  int64_t launches[kFamilies] = {};
  double ms[kFamilies] = {};
  double flops[kFamilies] = {};
  double bytes[kFamilies] = {};
};
TimingState g_tm;

hipEvent_t tm_event() {
  if (!g_tm.pool.empty()) {
    hipEvent_t e = g_tm.pool.back();
    g_tm.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Records the start event of a timed launch; returns the pending index.
struct TimedLaunch {
  int fam;
  hipStream_t st;
  hipEvent_t a = nullptr;
  TimedLaunch(int f, hipStream_t s) : fam(f), st(s) {
    if (!g_tm.on) return;
    a = tm_event();
    (void)hipEventRecord(a, st);
  }
  ~TimedLaunch() {
    if (!a) return;
    hipEvent_t b = tm_event();
    (void)hipEventRecord(b, st);
    g_tm.pending[fam].push_back({a, b});
    g_tm.launches[fam]++;
  }
};

void tm_collect() {
  for (int f = 0; f < kFamilies; ++f) {
    for (auto& pr : g_tm.pending[f]) {
      float ms = 0.f;
      (void)hipEventSynchronize(pr.second);
      if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) g_tm.ms[f] += ms;
      g_tm.pool.push_back(pr.first);
      g_tm.pool.push_back(pr.second);
    }
    g_tm.pending[f].clear();
  }
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(LRSP_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_));          \
  } while (0)

// Device buffer owned by the factor (stream-ordered allocator, cached pool).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

bool g_pool_init = false;

hipError_t dalloc(DevBuf* b, size_t bytes, hipStream_t st) {
  if (!g_pool_init) {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
      }
    }
    g_pool_init = true;
  }
  b->bytes = bytes;
  return hipMallocAsync(&b->p, std::max<size_t>(bytes, 256), st);
}

void dfree(DevBuf* b, hipStream_t st) {
  if (b->p) (void)hipFreeAsync(b->p, st);
  b->p = nullptr;
  b->bytes = 0;
}

uint64_t g_level_ids = 0;

struct LevelDev {
  const uint64_t id = ++g_level_ids;  // unique per workspace
  LevelPlan plan;
  std::vector<int> k, a, b;
  int max_m = 0;
  DevBuf work, wints;      // D / fine / coarse halves; posmaps and column lists
  DevBuf fac;              // panels, tau, norms (doubles)
  DevBuf fints;            // colseg, colnat, stepof, piv, segoff (int32)
  DevBuf fvidx;            // vidx (int64)
  DevBuf desc;             // SegD / PairD / WbD / ItemD
  DevBuf state;            // k, a, b, err
  ItemD* d_items = nullptr;
  LevelState ls{};
  int64_t vbase = 0;       // offset of this level in the vector buffer
  std::vector<int64_t> voff;
  int64_t nvec = 0;
  DevBuf gidx;             // level >= 1: indices into the previous level's vector
  // adjacency export
  std::vector<int> adj_ptr, adj, sizes_i, colour_i, order_i;
  std::vector<double> sweep_bytes;  // per colour: bytes one sweep of it moves
  std::vector<SplitDims> cdims;     // per colour capacities
  int max_items = 0;                // largest colour
  int max_nseg = 0;
  bool split = false;               // several workgroups per cluster
  const int32_t* d_cstart = nullptr;
  DevBuf vals_off;                  // level 0: CSR entry -> work-arena offset
  DevBuf tasks;                     // level >= 1: assembly copy tasks
  int ntasks = 0;
  uint64_t tasks_src = 0;           // id of the level the tasks read from
  void free_all(hipStream_t st) {
    dfree(&work, st); dfree(&wints, st); dfree(&fac, st); dfree(&fints, st); dfree(&fvidx, st);
    dfree(&desc, st); dfree(&state, st); dfree(&gidx, st); dfree(&vals_off, st); dfree(&tasks, st);
  }
};

// Analysis of the last pattern factored with a tree, and level workspaces
// returned by freed factors.
struct TreeCache {
  bool have = false;
  uint64_t hash = 0;
  int64_t nnz = -1;
  std::vector<std::vector<int>> adj0;
  std::unordered_map<uint64_t, std::vector<uint64_t>> z0;
  std::vector<std::unique_ptr<LevelDev>> levels;
  hipStream_t stream = nullptr;
  ~TreeCache() {
    for (auto& L : levels)
      if (L) L->free_all(stream);
    (void)hipStreamSynchronize(stream);
  }
};

uint64_t pattern_hash(const int64_t* rp, const int32_t* cl, int64_t n, int64_t nnz) {
  uint64_t h = 1469598103934665603ull ^ (uint64_t)n ^ ((uint64_t)nnz << 32);
  for (int64_t i = 0; i <= n; ++i) h = (h ^ (uint64_t)rp[i]) * 1099511628211ull;
  for (int64_t e = 0; e < nnz; ++e) h = (h ^ (uint32_t)cl[e]) * 1099511628211ull;
  return h;
}

}  // namespace

struct lrsp_tree {
  TreeH t;
  std::shared_ptr<TreeCache> cache = std::make_shared<TreeCache>();
};

struct lrsp_factorization {
  int64_t n = 0;
  std::vector<std::unique_ptr<LevelDev>> levels;
  // dense top
  int top_n = 0;
  int top_level = 0;
  DevBuf top;             // L (n_top x n_top)
  int64_t top_vbase = 0;
  DevBuf top_gidx;        // indices into the last level's vector (or unused)
  std::vector<int> top_sizes, top_adj_ptr, top_adj;
  DevBuf perm;            // level-0 cluster order
  DevBuf vec;             // all level vectors
  int64_t vec_total = 0;
  DevBuf scratch;         // PCG work vectors / scalars
  size_t scratch_n = 0;
  lrsp_info info{};
  hipStream_t stream = nullptr;
  std::weak_ptr<TreeCache> cache;
  uint64_t pattern = 0;
  ~lrsp_factorization() {
    std::shared_ptr<TreeCache> c = cache.lock();
    const bool give = c && c->have && c->hash == pattern;
    for (size_t l = 0; l < levels.size(); ++l) {
      if (!levels[l]) continue;
      if (give) {
        if (c->levels.size() <= l) c->levels.resize(l + 1);
        if (c->levels[l]) c->levels[l]->free_all(stream);
        c->levels[l] = std::move(levels[l]);
        c->stream = stream;
      } else {
        levels[l]->free_all(stream);
      }
    }
    dfree(&top, stream); dfree(&top_gidx, stream); dfree(&perm, stream); dfree(&vec, stream);
    dfree(&scratch, stream);
    (void)hipStreamSynchronize(stream);
  }
};

namespace {

template <class T>
T* at(const DevBuf& b, int64_t off) {
  return reinterpret_cast<T*>(b.p) + off;
}

// Coupling c(x,y) between the coarse DoFs of two linked clusters of a
// finished level: returns the source block and whether it is transposed.
bool coupling(const LevelDev& L, int x, int y, const double** src, int* sld, int* trans) {
  const LevelPlan& p = L.plan;
  if (!std::binary_search(p.adj2[x].begin(), p.adj2[x].end(), y)) return false;
  const int later = p.pos[x] > p.pos[y] ? x : y;
  const int earlier = later == x ? y : x;
  auto it = p.hc_off.find(pkey(later, earlier));
  if (it == p.hc_off.end()) return false;
  *src = at<double>(L.work, it->second);
  *sld = p.m[later];
  *trans = (later == x) ? 0 : 1;
  return true;
}

// Tasks that move the coarse-coarse couplings of finished level `prev` into
// block storage of the next level (fine halves of edges, diagonal blocks).
bool assembly_tasks(const LevelDev& prev, const LevelDev& cur, std::vector<CopyD>* tasks) {
  const LevelPlan& q = cur.plan;
  const std::vector<int>& k = prev.k;
  auto add = [&](const double* src, int sld, int trans, double* dst, int dld, int rows, int cols) {
    if (rows <= 0 || cols <= 0) return;
    CopyD c{src, dst, sld, dld, rows, cols, trans, 0};
    tasks->push_back(c);
  };
  for (int P = 0; P < q.M; ++P) {
    const int L = 2 * P, R = 2 * P + 1;
    double* D = at<double>(cur.work, q.d_off[P]);
    const int mP = q.m[P];
    add(at<double>(prev.work, prev.plan.d_off[L]), prev.plan.m[L], 0, D, mP, k[L], k[L]);
    add(at<double>(prev.work, prev.plan.d_off[R]), prev.plan.m[R], 0, D + (size_t)k[L] * mP + k[L],
        mP, k[R], k[R]);
    const double* src;
    int sld, tr;
    if (coupling(prev, R, L, &src, &sld, &tr)) add(src, sld, tr, D + k[L], mP, k[R], k[L]);
  }
  for (auto& kv : q.hf_off) {
    const int e = (int)(kv.first >> 32), l = (int)(kv.first & 0xffffffffu);
    if (!std::binary_search(q.adj[e].begin(), q.adj[e].end(), l)) continue;  // fill only
    if ((int)q.zfin.at(kv.first).size() != q.m[l]) return false;
    double* H = at<double>(cur.work, kv.second);
    const int me = q.m[e];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const int x = 2 * e + a, y = 2 * l + b;
        const double* src;
        int sld, tr;
        if (!coupling(prev, x, y, &src, &sld, &tr)) continue;
        const int ro = a ? k[2 * e] : 0, co = b ? k[2 * l] : 0;
        add(src, sld, tr, H + ro + (size_t)me * co, me, k[x], k[y]);
      }
  }
  return true;
}

// Copies a host array into a new device buffer; waits for the copy, since
// the host array may be pageable and short-lived.
lrsp_status upload(DevBuf* b, const void* src, size_t bytes, hipStream_t st) {
  HIPCHK(dalloc(b, bytes, st));
  if (bytes) HIPCHK(hipMemcpyAsync(b->p, src, bytes, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return LRSP_OK;
}

// Builds device storage and descriptors of one planned level.
lrsp_status setup_level(LevelDev* L, hipStream_t st, int64_t vbase) {
  LevelPlan& p = L->plan;
  const int M = p.M;
  plan_layout(&p);
  L->max_m = 0;
  for (int x = 0; x < M; ++x) L->max_m = std::max(L->max_m, p.m[x]);
  if (L->max_m > kMaxClusterDofs)
    return fail(LRSP_ERR_ARG, "cluster larger than " + std::to_string(kMaxClusterDofs) +
                                  " DoFs; use a smaller leaf size");
  HIPCHK(dalloc(&L->work, sizeof(double) * p.work_doubles, st));
  launch_zero(at<double>(L->work, 0), p.work_doubles, st);
  // int arena: posmaps (-1 = absent) and column lists
  std::vector<int32_t> hints(p.work_ints, -1);
  for (auto& kv : p.zfin) {
    const std::vector<int>& z = kv.second;
    int32_t* pm = hints.data() + p.pos_off[kv.first];
    for (size_t i = 0; i < z.size(); ++i) pm[z[i]] = (int32_t)i;
    std::copy(z.begin(), z.end(), hints.data() + p.zl_off[kv.first]);
  }
  if (lrsp_status s = upload(&L->wints, hints.data(), hints.size() * 4, st)) return s;
  // factor arenas
  int64_t fd = 0, fi = 0, fv = 0;
  std::vector<int64_t> poff(M), toff(M), noff(M), csoff(M), cnoff(M), stoff(M), pvoff(M),
      sgoff(M), vxoff(M);
  auto al = [](int64_t v) { return (v + 31) & ~(int64_t)31; };
  for (int s = 0; s < M; ++s) {
    const int64_t pc = p.acap[s] + p.bcap[s];
    const int nseg = (int)(p.nlist[s].size() + p.wlist[s].size());
    poff[s] = fd; fd += al((int64_t)p.m[s] * (p.m[s] + pc));
    toff[s] = fd; fd += al(p.kcap[s]);
    noff[s] = fd; fd += al(pc);
    csoff[s] = fi; fi += al(pc);
    cnoff[s] = fi; fi += al(pc);
    stoff[s] = fi; fi += al(pc);
    pvoff[s] = fi; fi += al(p.kcap[s]);
    sgoff[s] = fi; fi += al(nseg + 1);
    vxoff[s] = fv; fv += al(pc);
  }
  HIPCHK(dalloc(&L->fac, sizeof(double) * fd, st));
  HIPCHK(dalloc(&L->fints, sizeof(int32_t) * fi, st));
  HIPCHK(dalloc(&L->fvidx, sizeof(int64_t) * fv, st));
  HIPCHK(dalloc(&L->state, sizeof(int32_t) * (3 * (size_t)M + 8), st));
  int32_t* sb = at<int32_t>(L->state, 0);
  L->ls.k = sb;
  L->ls.a = sb + M;
  L->ls.b = sb + 2 * M;
  L->ls.err = sb + 3 * M;
  launch_zero_i32(sb, 3 * (int64_t)M + 8, st);
  // level vector offsets
  L->voff.assign(M, 0);
  int64_t vo = 0;
  for (int x = 0; x < M; ++x) {
    L->voff[x] = vbase + vo;
    vo += p.m[x];
  }
  L->vbase = vbase;
  L->nvec = vo;
  // descriptors
  std::vector<SegD> segs;
  std::vector<PairD> pairs;
  std::vector<WbD> wbs;
  std::vector<ItemD> items(M);
  std::vector<int64_t> seg0(M), pair0(M), wb0(M);
  double* W = at<double>(L->work, 0);
  int32_t* WI = at<int32_t>(L->wints, 0);
  for (int idx = 0; idx < M; ++idx) {
    const int s = p.order[idx];
    const std::vector<int>& nl = p.nlist[s];
    const std::vector<int>& wl = p.wlist[s];
    seg0[s] = (int64_t)segs.size();
    wb0[s] = (int64_t)wbs.size();
    for (int pass = 0; pass < 2; ++pass)
      for (int y : (pass ? wl : nl)) {
        SegD sg{};
        sg.y = y;
        sg.isw = pass;
        sg.voff = L->voff[y];
        WbD wb{};
        if (p.pos[y] < p.pos[s]) {
          const int64_t o = p.hc_off.at(pkey(s, y));
          sg.src = W + o;
          sg.zl = nullptr;
          sg.coarse = 1;
          sg.cap = p.kcap[y];
          wb.dst = W + o;
          wb.ld = p.m[s];
          wb.trans = 0;
          wb.nrows = p.m[s];
          wb.ncols = p.kcap[y];
        } else {
          const uint64_t key = pkey(s, y);
          sg.src = W + p.hf_off.at(key);
          sg.zl = WI + p.zl_off.at(key);
          sg.coarse = 0;
          sg.nfine = (int)p.zfin.at(key).size();
          sg.cap = sg.nfine;
          wb.dst = W + p.hc_off.at(pkey(y, s));
          wb.ld = p.m[y];
          wb.trans = 1;
          wb.nrows = p.m[y];
          wb.ncols = p.kcap[s];
        }
        segs.push_back(sg);
        wbs.push_back(wb);
      }
    pair0[s] = (int64_t)pairs.size();
    const int nn = (int)nl.size();
    for (int j = 0; j < nn; ++j)
      for (int i = 0; i <= j; ++i) {
        PairD pd{};
        const int pi = nl[i], qj = nl[j];
        if (i == j) {
          pd.dst = W + p.d_off[pi];
          pd.ld = p.m[pi];
          pd.diag = 1;
          pd.nrows = p.m[pi];
          pd.ncols = p.m[pi];
        } else {
          const int e = p.pos[pi] < p.pos[qj] ? pi : qj;
          const int l = e == pi ? qj : pi;
          if (p.pos[e] < p.pos[s]) {
            pd.dst = W + p.hc_off.at(pkey(l, e));
            pd.ld = p.m[l];
            pd.rows_from_j = (l == qj);
            pd.nrows = p.m[l];
            pd.ncols = p.kcap[e];
          } else {
            const uint64_t key = pkey(e, l);
            pd.dst = W + p.hf_off.at(key);
            pd.posmap = WI + p.pos_off.at(key);
            pd.ld = p.m[e];
            pd.rows_from_j = (e == qj);
            pd.nrows = p.m[e];
            pd.ncols = (int)p.zfin.at(key).size();
          }
        }
        pairs.push_back(pd);
      }
  }
  const size_t bs = sizeof(SegD) * segs.size(), bp = sizeof(PairD) * pairs.size(),
               bw = sizeof(WbD) * wbs.size(), bi = sizeof(ItemD) * M,
               bc = sizeof(int32_t) * (p.ncolours + 1);
  const size_t o1 = (bs + 255) & ~(size_t)255, o2 = o1 + ((bp + 255) & ~(size_t)255),
               o3 = o2 + ((bw + 255) & ~(size_t)255), o4 = o3 + ((bi + 255) & ~(size_t)255);
  HIPCHK(dalloc(&L->desc, o4 + bc, st));
  char* db = reinterpret_cast<char*>(L->desc.p);
  double* F = at<double>(L->fac, 0);
  int32_t* FI = at<int32_t>(L->fints, 0);
  int64_t* FV = at<int64_t>(L->fvidx, 0);
  for (int idx = 0; idx < M; ++idx) {
    const int s = p.order[idx];
    ItemD& it = items[idx];
    it.s = s;
    it.m = p.m[s];
    it.nseg = (int)(p.nlist[s].size() + p.wlist[s].size());
    it.nsegn = (int)p.nlist[s].size();
    it.pcap = p.acap[s] + p.bcap[s];
    it.kcap = p.kcap[s];
    it.seg = reinterpret_cast<const SegD*>(db) + seg0[s];
    it.pair = reinterpret_cast<const PairD*>(db + o1) + pair0[s];
    it.wb = reinterpret_cast<const WbD*>(db + o2) + wb0[s];
    it.D = W + p.d_off[s];
    it.P = F + poff[s];
    it.tau = F + toff[s];
    it.norms = F + noff[s];
    it.colseg = FI + csoff[s];
    it.colnat = FI + cnoff[s];
    it.stepof = FI + stoff[s];
    it.piv = FI + pvoff[s];
    it.segoff = FI + sgoff[s];
    it.vidx = FV + vxoff[s];
    it.voff = L->voff[s];
  }
  std::vector<char> blob(o4 + bc, 0);
  if (bs) std::memcpy(blob.data(), segs.data(), bs);
  if (bp) std::memcpy(blob.data() + o1, pairs.data(), bp);
  if (bw) std::memcpy(blob.data() + o2, wbs.data(), bw);
  std::memcpy(blob.data() + o3, items.data(), bi);
  std::memcpy(blob.data() + o4, p.cstart.data(), bc);
  HIPCHK(hipMemcpyAsync(db, blob.data(), blob.size(), hipMemcpyHostToDevice, st));
  L->d_items = reinterpret_cast<ItemD*>(db + o3);
  L->d_cstart = reinterpret_cast<const int32_t*>(db + o4);
  // per-colour capacities
  L->cdims.assign(p.ncolours, SplitDims{0, 0, 0, 0});
  L->max_items = 0;
  L->max_nseg = 0;
  for (int c = 0; c < p.ncolours; ++c) {
    L->max_items = std::max(L->max_items, p.cstart[c + 1] - p.cstart[c]);
    SplitDims& d = L->cdims[c];
    for (int idx = p.cstart[c]; idx < p.cstart[c + 1]; ++idx) {
      const ItemD& it = items[idx];
      d.max_m = std::max(d.max_m, it.m);
      d.max_nseg = std::max(d.max_nseg, it.nseg);
      d.max_pcap = std::max(d.max_pcap, it.pcap);
      d.max_acap = std::max(d.max_acap, p.acap[it.s]);
    }
    L->max_nseg = std::max(L->max_nseg, d.max_nseg);
  }
  // hipMemcpyAsync from pageable memory may return before the copy is done
  HIPCHK(hipStreamSynchronize(st));
  // export copies
  L->sizes_i = p.m;
  L->colour_i = p.colour;
  L->order_i = p.order;
  L->adj_ptr.assign(1, 0);
  L->adj.clear();
  for (int x = 0; x < M; ++x) {
    L->adj.insert(L->adj.end(), p.adj[x].begin(), p.adj[x].end());
    L->adj_ptr.push_back((int)L->adj.size());
  }
  return LRSP_OK;
}

bool complete_graph(const std::vector<std::vector<int>>& adj) {
  const int M = (int)adj.size();
  for (int x = 0; x < M; ++x)
    if ((int)adj[x].size() != M - 1) return false;
  return true;
}

}  // namespace

extern "C" {

const char* lrsp_status_str(lrsp_status s) {
  switch (s) {
    case LRSP_OK: return "ok";
    case LRSP_ERR_ARG: return "invalid argument";
    case LRSP_ERR_NOT_SPD: return "matrix (or an approximate Schur complement) not positive definite";
    case LRSP_ERR_HIP: return "HIP runtime error";
    case LRSP_ERR_OOM: return "out of device memory";
    case LRSP_ERR_NO_CONV: return "PCG did not converge";
    case LRSP_ERR_INTERNAL: return "internal consistency check failed";
  }
  return "unknown status";
}

const char* lrsp_last_error_info(void) { return g_last_error.c_str(); }

lrsp_status lrsp_tree_build(const lrsp_grid* g, int32_t leaf_size, lrsp_tree** out) {
  if (!g || !out) return fail(LRSP_ERR_ARG, "null argument");
  auto t = std::make_unique<lrsp_tree>();
  if (build_tree(g->nx, g->ny, g->nz, g->ncomp, leaf_size, &t->t) != 0)
    return fail(LRSP_ERR_ARG, "invalid grid/leaf size (leaf < nz*ncomp or a column would be split)");
  *out = t.release();
  return LRSP_OK;
}

lrsp_status lrsp_tree_free(lrsp_tree* t) {
  delete t;
  return LRSP_OK;
}

lrsp_status lrsp_tree_export(const lrsp_tree* t, lrsp_tree_view* v) {
  if (!t || !v) return fail(LRSP_ERR_ARG, "null argument");
  v->nlevels = t->t.L;
  v->nleaves = (int32_t)t->t.leaf_ptr.size() - 1;
  v->n = t->t.n;
  v->perm = t->t.perm.data();
  v->leaf_ptr = t->t.leaf_ptr.data();
  return LRSP_OK;
}

lrsp_status lrsp_factor_free(lrsp_factorization* F) {
  delete F;
  return LRSP_OK;
}

static lrsp_status factor_impl(const lrsp_csr* A, lrsp_tree* T, double tol, const lrsp_opts* opts,
                               void* stream, lrsp_factorization** out) {
  if (!A || !T || !out) return fail(LRSP_ERR_ARG, "null argument");
  *out = nullptr;
  const TreeH& tr = T->t;
  if (A->n != tr.n) return fail(LRSP_ERR_ARG, "matrix size does not match the tree");
  if (!(tol >= 0.0)) return fail(LRSP_ERR_ARG, "tol must be >= 0");
  if (!A->rowptr || !A->col || !A->val) return fail(LRSP_ERR_ARG, "null CSR array");
  lrsp_opts o{};
  if (opts) o = *opts;
  if (o.gemm_prec < 0 || o.gemm_prec > 2 || o.tol_mode < 0 || o.tol_mode > 1 || o.exec_mode < 0 ||
      o.exec_mode > 3)
    return fail(LRSP_ERR_ARG, "invalid option");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  // host copy of the pattern
  std::vector<int64_t> hrp;
  std::vector<int32_t> hcol;
  const int64_t* rp = A->h_rowptr;
  const int32_t* cl = A->h_col;
  if (!rp || !cl) {
    hrp.resize(A->n + 1);
    hcol.resize(A->nnz);
    HIPCHK(hipMemcpyAsync(hrp.data(), A->rowptr, sizeof(int64_t) * (A->n + 1),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hcol.data(), A->col, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rp = hrp.data();
    cl = hcol.data();
  }
  if (rp[A->n] != A->nnz) return fail(LRSP_ERR_ARG, "rowptr[n] != nnz");
  auto F = std::make_unique<lrsp_factorization>();
  F->n = A->n;
  F->stream = st;
  double ms_an = 0.0;
  auto tick = [] { return std::chrono::steady_clock::now(); };
  auto ms_since = [](std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
  };
  std::shared_ptr<TreeCache> cache = T->cache;
  F->cache = cache;
  // level 0 clusters and graph
  std::vector<int> sizes(tr.leaf_ptr.size() - 1);
  for (size_t c = 0; c + 1 < tr.leaf_ptr.size(); ++c)
    sizes[c] = (int)(tr.leaf_ptr[c + 1] - tr.leaf_ptr[c]);
  const uint64_t ph = pattern_hash(rp, cl, A->n, A->nnz);
  F->pattern = ph;
  if (!(cache->have && cache->hash == ph && cache->nnz == A->nnz)) {
    const auto ta = tick();
    for (auto& Lc : cache->levels)
      if (Lc) Lc->free_all(st);
    cache->levels.clear();
    cache->have = false;
    level0_graph(tr, rp, cl, &cache->adj0);
    // initial fine column sets of level-0 blocks
    cache->z0.clear();
    for (int64_t i = 0; i < tr.n; ++i) {
      const int p = tr.dof_cluster[i];
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = cl[e];
        if (j < 0 || j >= tr.n) return fail(LRSP_ERR_ARG, "column index out of range");
        const int q = tr.dof_cluster[j];
        if (q == p) continue;
        std::vector<uint64_t>& b = cache->z0[pkey(p, q)];
        if (b.empty()) b.assign((sizes[q] + 63) / 64, 0);
        const int lj = tr.dof_local[j];
        b[lj >> 6] |= 1ull << (lj & 63);
      }
    }
    cache->have = true;
    cache->hash = ph;
    cache->nnz = A->nnz;
    ms_an += ms_since(ta);
  }
  std::vector<std::vector<int>> adj = cache->adj0;
  int reused = 0;
  HIPCHK(dalloc(&F->perm, sizeof(int64_t) * tr.n, st));
  HIPCHK(hipMemcpyAsync(F->perm.p, tr.perm.data(), sizeof(int64_t) * tr.n, hipMemcpyHostToDevice, st));
  double flops[6] = {0, 0, 0, 0, 0, 0};
  int64_t vbase = 0;
  int level = 0;
  LevelDev* prev = nullptr;
  std::vector<int32_t> herr(4);
  while (true) {
    const int M = (int)sizes.size();
    if (M == 1 || complete_graph(adj)) break;
    std::unique_ptr<LevelDev> Lp;
    bool reuse = false;
    if ((int)cache->levels.size() > level && cache->levels[level] &&
        cache->levels[level]->plan.m == sizes && cache->levels[level]->vbase == vbase) {
      Lp = std::move(cache->levels[level]);
      reuse = true;
      ++reused;
    }
    const auto ta = tick();
    if (!reuse) {
      Lp = std::make_unique<LevelDev>();
      Lp->plan.M = M;
      Lp->plan.m = sizes;
      Lp->plan.adj = adj;
      plan_level(&Lp->plan, level == 0 ? &cache->z0 : nullptr);
      if (lrsp_status s = setup_level(Lp.get(), st, vbase)) return s;
    } else {
      launch_zero(at<double>(Lp->work, 0), Lp->plan.work_doubles, st);
      launch_zero_i32(at<int32_t>(Lp->state, 0), 3 * (int64_t)M + 8, st);
    }
    LevelDev* L = Lp.get();
    vbase += L->nvec;
    // assemble the level's matrix
    if (level == 0 && L->vals_off.p) {
      launch_scatter_vals(A->val, at<int64_t>(L->vals_off, 0), A->nnz, at<double>(L->work, 0), st);
    } else if (level == 0) {
      std::vector<int64_t> off(A->nnz, -1);
      const LevelPlan& p = L->plan;
      for (int64_t i = 0; i < tr.n; ++i) {
        const int pc = tr.dof_cluster[i], li = tr.dof_local[i];
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
          const int j = cl[e];
          const int q = tr.dof_cluster[j], lj = tr.dof_local[j];
          if (q == pc) {
            off[e] = p.d_off[pc] + li + (int64_t)p.m[pc] * lj;
          } else if (p.pos[pc] < p.pos[q]) {
            const uint64_t key = pkey(pc, q);
            const std::vector<int>& z = p.zfin.at(key);
            const int col = (int)(std::lower_bound(z.begin(), z.end(), lj) - z.begin());
            if (col >= (int)z.size() || z[col] != lj)
              return fail(LRSP_ERR_INTERNAL, "level-0 entry outside its fine column set");
            off[e] = p.hf_off.at(key) + li + (int64_t)p.m[pc] * col;
          }
        }
      }
      if (lrsp_status s = upload(&L->vals_off, off.data(), off.size() * 8, st)) return s;
      launch_scatter_vals(A->val, at<int64_t>(L->vals_off, 0), A->nnz, at<double>(L->work, 0), st);
    } else {
      if (!(reuse && L->tasks_src == prev->id)) {
        std::vector<CopyD> tasks;
        if (!assembly_tasks(*prev, *L, &tasks))
          return fail(LRSP_ERR_INTERNAL, "coarse fine-half block is not dense");
        dfree(&L->tasks, st);
        L->ntasks = (int)tasks.size();
        if (!tasks.empty())
          if (lrsp_status s = upload(&L->tasks, tasks.data(), tasks.size() * sizeof(CopyD), st)) return s;
        L->tasks_src = prev->id;
        // gather indices into the previous level's vector
        std::vector<int64_t> g;
        g.reserve(L->nvec);
        for (int P = 0; P < M; ++P)
          for (int c = 0; c < 2; ++c) {
            const int x = 2 * P + c;
            for (int i = 0; i < prev->k[x]; ++i) g.push_back(prev->voff[x] + i);
          }
        dfree(&L->gidx, st);
        if (lrsp_status s = upload(&L->gidx, g.data(), g.size() * 8, st)) return s;
      }
      if (L->ntasks > 0) launch_copy_blocks(at<CopyD>(L->tasks, 0), L->ntasks, st);
    }
    if (!reuse) ms_an += ms_since(ta);
    // eliminate the clusters colour by colour
    const LevelPlan& p = L->plan;
    const int mode = o.exec_mode == 0 ? 3 : o.exec_mode;
    L->split = mode == 3 && L->max_m >= kSplitMinDofs && L->max_m <= kSplitMaxDofs;
    bool done = false;
    if (L->split) {
      for (int c = 0; c < p.ncolours; ++c) {
        TimedLaunch tall(0, st);
        for (int step = 0; step < kSplitSteps; ++step) {
          static const int fam[kSplitSteps] = {3, 3, 4, 5, 6, 7, 8, 9};
          TimedLaunch ts(fam[step], st);
          launch_split_step(step, L->d_items + p.cstart[c], p.cstart[c + 1] - p.cstart[c], L->cdims[c],
                            L->ls, level, tol, o.tol_mode, o.gemm_prec, st);
        }
      }
      done = true;
    } else if (mode >= 2) {
      TimedLaunch tall(0, st), tf(10, st);
      done = launch_slre_level(L->d_items, L->d_cstart, p.ncolours, L->max_items, L->max_m,
                               L->max_nseg, L->ls, level, tol, o.tol_mode, o.gemm_prec,
                               st) == hipSuccess;
      if (!done) (void)hipGetLastError();
    }
    if (!done) {
      for (int c = 0; c < p.ncolours; ++c) {
        TimedLaunch tall(0, st), tf(10, st);
        launch_slre(L->d_items + p.cstart[c], p.cstart[c + 1] - p.cstart[c], L->max_m, L->max_nseg,
                    L->ls, level, tol, o.tol_mode, o.gemm_prec, st);
      }
    }
    HIPCHK(hipGetLastError());
    L->k.resize(M);
    L->a.resize(M);
    L->b.resize(M);
    HIPCHK(hipMemcpyAsync(L->k.data(), L->ls.k, 4 * (size_t)M, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(L->a.data(), L->ls.a, 4 * (size_t)M, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(L->b.data(), L->ls.b, 4 * (size_t)M, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(herr.data(), L->ls.err, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (herr[0]) {
      if (herr[3] == kErrNotSPD)
        return fail(LRSP_ERR_NOT_SPD, "non-positive pivot in the diagonal block of cluster " +
                                          std::to_string(herr[2]) + " at level " +
                                          std::to_string(herr[1]));
      return fail(LRSP_ERR_INTERNAL, "device check failed (code " + std::to_string(herr[3]) +
                                         ") at level " + std::to_string(herr[1]) + " cluster " +
                                         std::to_string(herr[2]));
    }
    double lvl_flops = 0.0;
    L->sweep_bytes.assign(p.ncolours, 0.0);
    for (int s = 0; s < M; ++s) {
      const double m = p.m[s], a = L->a[s], b = L->b[s], k = L->k[s];
      double f[5] = {m * m * m / 3.0, m * m * (a + b), 0.0, 0.0, a * (a + 1.0) * (m - k)};
      for (int j = 0; j < k; ++j) {
        f[2] += 4.0 * (m - j) * (b - j);
        f[3] += 4.0 * (m - j) * a;
      }
      for (int i = 0; i < 5; ++i) {
        flops[i] += f[i];
        lvl_flops += f[i];
      }
      if (g_tm.on && L->split) {
        for (int i = 0; i < 5; ++i) g_tm.flops[4 + i] += f[i];
        g_tm.bytes[3] += 16.0 * m * (m + a + b);  // panel gathered: read + write
        g_tm.bytes[9] += 16.0 * k * (a + b);
      }
      // one sweep reads G (lower), the k reflectors and F once, and reads
      // and writes the cluster's and its near field's vector entries
      L->sweep_bytes[p.colour[s]] +=
          8.0 * (m * (m + 1) / 2.0 + k * m + (m - k) * a) + 8.0 * (2.0 * m + 2.0 * a);
    }
    if (g_tm.on) {
      g_tm.flops[0] += lvl_flops;
      if (!L->split) g_tm.flops[10] += lvl_flops;
    }
    // next level
    std::vector<int> nsz(M / 2);
    for (int P = 0; P < M / 2; ++P) nsz[P] = L->k[2 * P] + L->k[2 * P + 1];
    std::vector<std::vector<int>> nadj;
    coarsen_square(adj, &nadj);
    sizes.swap(nsz);
    adj.swap(nadj);
    prev = L;
    F->levels.push_back(std::move(Lp));
    ++level;
  }
  // dense top
  const int M = (int)sizes.size();
  int ntop = 0;
  std::vector<int64_t> toff(M + 1, 0);
  for (int x = 0; x < M; ++x) toff[x + 1] = toff[x] + sizes[x];
  ntop = (int)toff[M];
  if (ntop > kMaxClusterDofs)
    return fail(LRSP_ERR_ARG, "dense top system larger than " + std::to_string(kMaxClusterDofs));
  F->top_n = ntop;
  F->top_level = level;
  F->top_sizes = sizes;
  F->top_adj_ptr.assign(1, 0);
  for (int x = 0; x < M; ++x) {
    F->top_adj.insert(F->top_adj.end(), adj[x].begin(), adj[x].end());
    F->top_adj_ptr.push_back((int)F->top_adj.size());
  }
  HIPCHK(dalloc(&F->top, sizeof(double) * std::max<int64_t>(1, (int64_t)ntop * ntop), st));
  double* Tm = at<double>(F->top, 0);
  launch_zero(Tm, (int64_t)ntop * ntop, st);
  if (level == 0) {
    std::vector<int64_t> off(A->nnz, -1);
    for (int64_t i = 0; i < tr.n; ++i) {
      const int pc = tr.dof_cluster[i], li = tr.dof_local[i];
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = cl[e];
        const int q = tr.dof_cluster[j], lj = tr.dof_local[j];
        off[e] = (toff[pc] + li) + (int64_t)ntop * (toff[q] + lj);
      }
    }
    DevBuf doff;
    if (lrsp_status s = upload(&doff, off.data(), off.size() * 8, st)) return s;
    launch_scatter_vals(A->val, at<int64_t>(doff, 0), A->nnz, Tm, st);
    dfree(&doff, st);
  } else {
    std::vector<CopyD> tasks;
    const std::vector<int>& k = prev->k;
    const int Mp = prev->plan.M;
    std::vector<int64_t> xo(Mp);
    for (int x = 0; x < Mp; ++x) xo[x] = toff[x / 2] + ((x & 1) ? k[x - 1] : 0);
    for (int x = 0; x < Mp; ++x) {
      if (k[x] > 0)
        tasks.push_back(CopyD{at<double>(prev->work, prev->plan.d_off[x]), Tm + xo[x] + (size_t)ntop * xo[x],
                              prev->plan.m[x], ntop, k[x], k[x], 0, 0});
      for (int y : prev->plan.adj2[x]) {
        const double* src;
        int sld, trn;
        if (k[x] > 0 && k[y] > 0 && coupling(*prev, x, y, &src, &sld, &trn))
          tasks.push_back(CopyD{src, Tm + xo[x] + (size_t)ntop * xo[y], sld, ntop, k[x], k[y], trn, 0});
      }
    }
    DevBuf dt;
    if (!tasks.empty()) {
      if (lrsp_status s = upload(&dt, tasks.data(), tasks.size() * sizeof(CopyD), st)) return s;
      launch_copy_blocks(at<CopyD>(dt, 0), (int)tasks.size(), st);
      dfree(&dt, st);
    }
    std::vector<int64_t> g;
    for (int P = 0; P < M; ++P)
      for (int c = 0; c < 2; ++c) {
        const int x = 2 * P + c;
        for (int i = 0; i < k[x]; ++i) g.push_back(prev->voff[x] + i);
      }
    if (lrsp_status s = upload(&F->top_gidx, g.data(), g.size() * 8, st)) return s;
  }
  DevBuf terr;
  HIPCHK(dalloc(&terr, 16, st));
  launch_zero_i32(at<int32_t>(terr, 0), 4, st);
  launch_top_potrf(Tm, ntop, at<int32_t>(terr, 0), st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(herr.data(), terr.p, 16, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  dfree(&terr, st);
  if (herr[0]) return fail(LRSP_ERR_NOT_SPD, "non-positive pivot in the dense top factorization");
  flops[5] = (double)ntop * ntop * ntop / 3.0;
  F->top_vbase = vbase;
  F->vec_total = vbase + ntop;
  HIPCHK(dalloc(&F->vec, sizeof(double) * std::max<int64_t>(1, F->vec_total), st));
  launch_zero(at<double>(F->vec, 0), F->vec_total, st);
  HIPCHK(hipStreamSynchronize(st));
  const auto t1 = std::chrono::steady_clock::now();
  lrsp_info& inf = F->info;
  inf.nlevels = (int)F->levels.size();
  inf.top_n = ntop;
  inf.top_clusters = M;
  for (int i = 0; i < 6; ++i) inf.flops[i] = flops[i];
  double fb = 8.0 * ntop * ntop;
  for (auto& L : F->levels) fb += (double)L->fac.bytes;
  inf.bytes_factor = fb;
  inf.ms_levels = std::chrono::duration<double, std::milli>(t1 - t0).count();
  inf.ms_analysis = ms_an;
  inf.levels_reused = reused;
  int64_t held = 0;
  for (auto& L : F->levels)
    held += (int64_t)(L->work.bytes + L->wints.bytes + L->fac.bytes + L->fints.bytes + L->fvidx.bytes +
                      L->desc.bytes + L->state.bytes + L->gidx.bytes + L->vals_off.bytes + L->tasks.bytes);
  inf.peak_bytes = held + (int64_t)(F->top.bytes + F->vec.bytes + F->perm.bytes);
  *out = F.release();
  return LRSP_OK;
}

lrsp_status lrsp_factor(const lrsp_csr* A, lrsp_tree* T, double tol, const lrsp_opts* opts,
                        void* stream, lrsp_factorization** out) {
  try {
    return factor_impl(A, T, tol, opts, stream, out);
  } catch (const std::bad_alloc&) {
    return fail(LRSP_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(LRSP_ERR_INTERNAL, std::string("planner: ") + e.what());
  }
}

static lrsp_status apply_one(const lrsp_factorization* F, const double* b, double* x, hipStream_t st) {
  double* V = at<double>(F->vec, 0);
  const int64_t n = F->n;
  const int nl = (int)F->levels.size();
  double* v0 = V + (nl ? F->levels[0]->vbase : F->top_vbase);
  launch_gather(b, at<int64_t>(F->perm, 0), v0, n, st);
  for (int l = 0; l < nl; ++l) {
    const LevelDev& L = *F->levels[l];
    const LevelPlan& p = L.plan;
    {
      TimedLaunch tl(1, st);
      if (launch_sweep_level(true, L.d_items, L.d_cstart, p.ncolours, L.max_items, L.max_m, L.ls, V,
                             st) != hipSuccess) {
        (void)hipGetLastError();
        for (int c = 0; c < p.ncolours; ++c)
          launch_fwd(L.d_items + p.cstart[c], p.cstart[c + 1] - p.cstart[c], L.max_m, L.ls, V, st);
      }
      if (g_tm.on)
        for (double by : L.sweep_bytes) g_tm.bytes[1] += by;
    }
    if (l + 1 < nl) {
      const LevelDev& N = *F->levels[l + 1];
      launch_gather(V, at<int64_t>(N.gidx, 0), V + N.vbase, N.nvec, st);
    } else {
      launch_gather(V, at<int64_t>(F->top_gidx, 0), V + F->top_vbase, F->top_n, st);
    }
  }
  launch_top_solve(at<double>(F->top, 0), F->top_n, V + F->top_vbase, st);
  for (int l = nl - 1; l >= 0; --l) {
    const LevelDev& L = *F->levels[l];
    const LevelPlan& p = L.plan;
    if (l + 1 < nl) {
      const LevelDev& N = *F->levels[l + 1];
      launch_scatter(V + N.vbase, at<int64_t>(N.gidx, 0), V, N.nvec, st);
    } else {
      launch_scatter(V + F->top_vbase, at<int64_t>(F->top_gidx, 0), V, F->top_n, st);
    }
    {
      TimedLaunch tl(2, st);
      if (launch_sweep_level(false, L.d_items, L.d_cstart, p.ncolours, L.max_items, L.max_m, L.ls, V,
                             st) != hipSuccess) {
        (void)hipGetLastError();
        for (int c = p.ncolours - 1; c >= 0; --c)
          launch_bwd(L.d_items + p.cstart[c], p.cstart[c + 1] - p.cstart[c], L.max_m, L.ls, V, st);
      }
      if (g_tm.on)
        for (double by : L.sweep_bytes) g_tm.bytes[2] += by;
    }
  }
  launch_scatter(v0, at<int64_t>(F->perm, 0), x, n, st);
  HIPCHK(hipGetLastError());
  return LRSP_OK;
}

lrsp_status lrsp_apply(const lrsp_factorization* F, const double* b, double* x, int32_t nrhs, void* stream) {
  if (!F || !b || !x || nrhs < 1) return fail(LRSP_ERR_ARG, "invalid argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int r = 0; r < nrhs; ++r)
    if (lrsp_status s = apply_one(F, b + (size_t)r * F->n, x + (size_t)r * F->n, st)) return s;
  return LRSP_OK;
}

lrsp_status lrsp_pcg(const lrsp_csr* A, const lrsp_factorization* F, const double* b, double* x,
                     int32_t nrhs, double rtol, int32_t maxit, int32_t* iters, double* relres,
                     void* stream) {
  if (!A || !F || !b || !x || nrhs < 1 || !iters || !relres || A->n != F->n || maxit < 0)
    return fail(LRSP_ERR_ARG, "invalid argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  lrsp_factorization* Fm = const_cast<lrsp_factorization*>(F);
  const int64_t n = A->n;
  const size_t need = 4 * (size_t)n + kDotBlocks + 16;
  if (Fm->scratch_n < need) {
    dfree(&Fm->scratch, st);
    HIPCHK(dalloc(&Fm->scratch, need * sizeof(double), st));
    Fm->scratch_n = need;
  }
  double* r = at<double>(Fm->scratch, 0);
  double* z = r + n;
  double* p = z + n;
  double* q = p + n;
  double* part = q + n;
  double* sc = part + kDotBlocks;  // [0] rz, [1] rz_new, [2] pq, [3] rr, [4] bb
  lrsp_status result = LRSP_OK;
  for (int rhs = 0; rhs < nrhs; ++rhs) {
    const double* bb = b + (size_t)rhs * n;
    double* xx = x + (size_t)rhs * n;
    launch_zero(xx, n, st);
    launch_dot(bb, bb, n, part, sc + 4, st);
    double hb = 0.0;
    HIPCHK(hipMemcpyAsync(&hb, sc + 4, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double nb = std::sqrt(hb);
    int it = 0;
    bool conv = nb == 0.0;
    if (!conv) {
      launch_copy(bb, r, n, st);
      if (lrsp_status s = apply_one(F, r, z, st)) return s;
      launch_dot(r, z, n, part, sc + 0, st);
      launch_copy(z, p, n, st);
      while (it < maxit) {
        launch_spmv(A->rowptr, A->col, A->val, p, q, n, st);
        launch_dot(p, q, n, part, sc + 2, st);
        launch_pcg_xr(xx, r, p, q, n, sc + 0, sc + 2, st);
        launch_dot(r, r, n, part, sc + 3, st);
        double hr = 0.0;
        HIPCHK(hipMemcpyAsync(&hr, sc + 3, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        ++it;
        if (std::sqrt(hr) <= rtol * nb) {
          conv = true;
          break;
        }
        if (lrsp_status s = apply_one(F, r, z, st)) return s;
        launch_dot(r, z, n, part, sc + 1, st);
        launch_pcg_p(p, z, n, sc + 1, sc + 0, st);
        launch_copy(sc + 1, sc + 0, 1, st);
      }
    }
    // true residual
    launch_spmv(A->rowptr, A->col, A->val, xx, q, n, st);
    launch_residual(bb, q, n, st);
    launch_dot(q, q, n, part, sc + 3, st);
    double ht = 0.0;
    HIPCHK(hipMemcpyAsync(&ht, sc + 3, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    iters[rhs] = it;
    relres[rhs] = nb > 0 ? std::sqrt(ht) / nb : 0.0;
    if (!conv) result = LRSP_ERR_NO_CONV;
  }
  if (result != LRSP_OK) g_last_error = "PCG reached maxit";
  return result;
}

lrsp_status lrsp_timing_enable(int32_t on) {
  g_tm.on = on != 0;
  return LRSP_OK;
}

lrsp_status lrsp_timing_reset(void) {
  tm_collect();
  for (int f = 0; f < kFamilies; ++f) {
    g_tm.launches[f] = 0;
    g_tm.ms[f] = g_tm.flops[f] = g_tm.bytes[f] = 0.0;
  }
  return LRSP_OK;
}

lrsp_status lrsp_timing_read(int32_t family, lrsp_timing* out) {
  if (family < 0 || family >= kFamilies || !out) return fail(LRSP_ERR_ARG, "invalid timing family");
  tm_collect();
  out->launches = g_tm.launches[family];
  out->total_ms = g_tm.ms[family];
  out->flops = g_tm.flops[family];
  out->bytes = g_tm.bytes[family];
  return LRSP_OK;
}

lrsp_status lrsp_factor_info(const lrsp_factorization* F, lrsp_info* info) {
  if (!F || !info) return fail(LRSP_ERR_ARG, "null argument");
  *info = F->info;
  return LRSP_OK;
}

lrsp_status lrsp_factor_level(const lrsp_factorization* F, int32_t level, lrsp_level_view* v) {
  if (!F || !v || level < 0 || level > (int)F->levels.size())
    return fail(LRSP_ERR_ARG, "invalid level");
  if (level == (int)F->levels.size()) {
    v->nclusters = (int32_t)F->top_sizes.size();
    v->ncolours = 0;
    v->sizes = F->top_sizes.data();
    v->colour = nullptr;
    v->order = nullptr;
    v->ranks = nullptr;
    v->adj_ptr = F->top_adj_ptr.data();
    v->adj = F->top_adj.data();
    return LRSP_OK;
  }
  const LevelDev& L = *F->levels[level];
  v->nclusters = L.plan.M;
  v->ncolours = L.plan.ncolours;
  v->sizes = L.sizes_i.data();
  v->colour = L.colour_i.data();
  v->order = L.order_i.data();
  v->ranks = L.k.data();
  v->adj_ptr = L.adj_ptr.data();
  v->adj = L.adj.data();
  return LRSP_OK;
}

}  // extern "C"
