// runtime.cpp -- host runtime shared by the single-system and batched
// factorizations (see runtime.hpp).
#include "runtime.hpp"

#include <algorithm>
#include <climits>
#include <cstring>

namespace lrsp {
namespace rt {

namespace {
thread_local std::string g_last_error;
uint64_t g_level_ids = 0;
}  // namespace

lrsp_status fail(lrsp_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

const char* last_error() { return g_last_error.c_str(); }

uint64_t next_level_id() { return ++g_level_ids; }

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

static bool g_pool_init = false;

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

void pool_trim() {
  int dev = 0;
  hipMemPool_t pool;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess)
    (void)hipMemPoolTrimTo(pool, kPoolKeepBytes);
}

void dfree(DevBuf* b, hipStream_t st) {
  if (b->p) (void)hipFreeAsync(b->p, st);
  b->p = nullptr;
  b->bytes = 0;
}

bool coupling(const LevelDev& L, int x, int y, const double** src, int* sld, int* trans) {
  const LevelPlan& p = L.plan;
  if (!std::binary_search(p.adj2[x].begin(), p.adj2[x].end(), y)) return false;
  const int later = p.pos[x] > p.pos[y] ? x : y;
  const int earlier = later == x ? y : x;
  auto it = p.hc_off.find(pkey(later, earlier));
  if (it == p.hc_off.end()) return false;
  *src = at<double>(L.coarse, it->second);
  *sld = p.m[later];
  *trans = (later == x) ? 0 : 1;
  return true;
}

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

void coarse_gather_indices(const LevelDev& prev, int nparents, std::vector<int64_t>* g) {
  g->clear();
  for (int P = 0; P < nparents; ++P)
    for (int c = 0; c < 2; ++c) {
      const int x = 2 * P + c;
      for (int i = 0; i < prev.k[x]; ++i) g->push_back(prev.voff[x] + i);
    }
}

lrsp_status upload(DevBuf* b, const void* src, size_t bytes, hipStream_t st) {
  HIPCHK(dalloc(b, bytes, st));
  if (bytes) HIPCHK(hipMemcpyAsync(b->p, src, bytes, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return LRSP_OK;
}

lrsp_status setup_level(LevelDev* L, hipStream_t st, int64_t vbase, int sbase,
                        const LevelState* shared, int32_t* serr, PanelArena* arena) {
  if (lrsp_status s = setup_level_a(L, st, vbase)) return s;
  return setup_level_b(L, st, sbase, shared, serr, arena);
}

lrsp_status setup_level_a(LevelDev* L, hipStream_t st, int64_t vbase) {
  LevelPlan& p = L->plan;
  const int M = p.M;
  plan_layout(&p);
  L->max_m = 0;
  L->min_m = M > 0 ? p.m[0] : 0;
  for (int x = 0; x < M; ++x) {
    L->max_m = std::max(L->max_m, p.m[x]);
    L->min_m = std::min(L->min_m, p.m[x]);
  }
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
  // level vector offsets
  L->voff.assign(M, 0);
  int64_t vo = 0;
  for (int x = 0; x < M; ++x) {
    L->voff[x] = vbase + vo;
    vo += p.m[x];
  }
  L->vbase = vbase;
  L->nvec = vo;
  return LRSP_OK;
}

namespace {

int64_t al32(int64_t v) { return (v + 31) & ~(int64_t)31; }

// Panel workspace of a level (doubles): panel, tau, norms and, where the
// split schedule may form it, the inverse of every cluster; returns the
// total.
struct PanelLayout {
  std::vector<int64_t> poff, toff, noff, gioff;
};
int64_t panel_layout(const LevelPlan& p, bool want_gi, PanelLayout* o) {
  const int M = p.M;
  o->poff.assign(M, 0);
  o->toff.assign(M, 0);
  o->noff.assign(M, 0);
  o->gioff.assign(M, -1);
  int64_t fd = 0;
  for (int s = 0; s < M; ++s) {
    const int64_t pc = p.acap[s] + p.bcap[s];
    o->poff[s] = fd; fd += al32((int64_t)p.m[s] * (p.m[s] + pc));
    o->toff[s] = fd; fd += al32(p.kcap[s]);
    o->noff[s] = fd; fd += al32(pc);
    if (want_gi && p.m[s] > 0 && p.m[s] <= kInvMaxDofs) {
      o->gioff[s] = fd;
      fd += al32((int64_t)p.m[s] * p.m[s]);
    }
  }
  return fd;
}

// The panel workspace of a level: its own buffer, or the start of the
// shared arena (grown when too small; a user on another stream is waited
// for first).
lrsp_status panel_base(LevelDev* L, int64_t fd, hipStream_t st, PanelArena* arena, double** base) {
  dfree(&L->fac, st);
  if (!arena) {
    HIPCHK(dalloc(&L->fac, sizeof(double) * (size_t)fd, st));
    *base = at<double>(L->fac, 0);
    return LRSP_OK;
  }
  if (lrsp_status s = arena_reserve(arena, L->arena_off + fd, st)) return s;
  L->arena_gen = arena->gen;
  L->arena_doubles = fd;
  *base = at<double>(arena->buf, 0) + L->arena_off;
  return LRSP_OK;
}

void point_items(const LevelPlan& p, const PanelLayout& lay, double* F, std::vector<ItemD>* items) {
  for (int idx = 0; idx < p.M; ++idx) {
    const int s = p.order[idx];
    ItemD& it = (*items)[idx];
    it.P = F + lay.poff[s];
    it.Gi = lay.gioff[s] >= 0 ? F + lay.gioff[s] : nullptr;
    it.tau = F + lay.toff[s];
    it.norms = F + lay.noff[s];
  }
}

}  // namespace

void arena_use(PanelArena* arena, hipStream_t st) {
  if (arena->used && arena->stream != st) (void)hipStreamSynchronize(arena->stream);
  arena->stream = st;
  arena->used = true;
}

lrsp_status arena_reserve(PanelArena* arena, int64_t doubles, hipStream_t st) {
  arena_use(arena, st);
  if (arena->buf.bytes < sizeof(double) * (size_t)doubles) {
    dfree(&arena->buf, st);
    HIPCHK(dalloc(&arena->buf, sizeof(double) * (size_t)doubles, st));
    ++arena->gen;
  }
  return LRSP_OK;
}

int64_t panel_doubles(const LevelDev& L) {
  PanelLayout lay;
  return panel_layout(L.plan, L.want_gi, &lay);
}

lrsp_status rebind_panels(LevelDev* L, hipStream_t st, PanelArena* arena) {
  PanelLayout lay;
  const int64_t fd = panel_layout(L->plan, L->want_gi, &lay);
  double* F = nullptr;
  if (lrsp_status s = panel_base(L, fd, st, arena, &F)) return s;
  point_items(L->plan, lay, F, &L->h_items);
  HIPCHK(hipMemcpyAsync(L->d_items, L->h_items.data(), sizeof(ItemD) * (size_t)L->plan.M, hipMemcpyHostToDevice,
                        st));
  return LRSP_OK;
}

lrsp_status setup_level_b(LevelDev* L, hipStream_t st, int sbase, const LevelState* shared,
                          int32_t* serr, PanelArena* arena) {
  LevelPlan& p = L->plan;
  const int M = p.M;
  // coarse halves (layout from the current rank capacities)
  plan_layout(&p);
  dfree(&L->coarse, st);
  dfree(&L->fints, st);
  dfree(&L->fvidx, st);
  dfree(&L->desc, st);
  HIPCHK(dalloc(&L->coarse, sizeof(double) * p.coarse_doubles, st));
  launch_zero(at<double>(L->coarse, 0), p.coarse_doubles, st);
  // panel workspace and index arenas
  PanelLayout lay;
  double* F = nullptr;
  if (lrsp_status s = panel_base(L, panel_layout(p, L->want_gi, &lay), st, arena, &F)) return s;
  int64_t fi = 0, fv = 0;
  std::vector<int64_t> csoff(M), cnoff(M), stoff(M), pvoff(M), sgoff(M), vxoff(M);
  auto al = al32;
  for (int s = 0; s < M; ++s) {
    const int64_t pc = p.acap[s] + p.bcap[s];
    const int nseg = (int)(p.nlist[s].size() + p.wlist[s].size());
    csoff[s] = fi; fi += al(pc);
    cnoff[s] = fi; fi += al(pc);
    stoff[s] = fi; fi += al(pc);
    pvoff[s] = fi; fi += al(p.kcap[s]);
    sgoff[s] = fi; fi += al(nseg + 1);
    vxoff[s] = fv; fv += al(pc);
  }
  HIPCHK(dalloc(&L->fints, sizeof(int32_t) * fi, st));
  HIPCHK(dalloc(&L->fvidx, sizeof(int64_t) * fv, st));
  L->sbase = sbase;
  if (shared) {
    L->ls = *shared;
  } else {
    dfree(&L->state, st);
    HIPCHK(dalloc(&L->state, sizeof(int32_t) * (4 * (size_t)M + 8), st));
    int32_t* sb = at<int32_t>(L->state, 0);
    L->ls.k = sb;
    L->ls.a = sb + M;
    L->ls.b = sb + 2 * M;
    L->ls.err = sb + 3 * M;
    L->ls.giok = sb + 3 * M + 8;
    launch_zero_i32(sb, 4 * (int64_t)M + 8, st);
  }
  // descriptors
  std::vector<SegD> segs;
  std::vector<PairD> pairs;
  std::vector<WbD> wbs;
  std::vector<ItemD> items(M);
  std::vector<int64_t> seg0(M), pair0(M), wb0(M);
  double* W = at<double>(L->work, 0);
  double* CR = at<double>(L->coarse, 0);
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
        sg.y = sbase + y;
        sg.isw = pass;
        sg.voff = L->voff[y];
        WbD wb{};
        if (p.pos[y] < p.pos[s]) {
          const int64_t o = p.hc_off.at(pkey(s, y));
          sg.src = CR + o;
          sg.zl = nullptr;
          sg.coarse = 1;
          sg.cap = p.kcap[y];
          wb.dst = CR + o;
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
          wb.dst = CR + p.hc_off.at(pkey(y, s));
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
            pd.dst = CR + p.hc_off.at(pkey(l, e));
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
  int32_t* FI = at<int32_t>(L->fints, 0);
  int64_t* FV = at<int64_t>(L->fvidx, 0);
  for (int idx = 0; idx < M; ++idx) {
    const int s = p.order[idx];
    ItemD& it = items[idx];
    it.s = sbase + s;
    it.serr = serr;
    it.m = p.m[s];
    it.nseg = (int)(p.nlist[s].size() + p.wlist[s].size());
    it.nsegn = (int)p.nlist[s].size();
    it.pcap = p.acap[s] + p.bcap[s];
    it.kcap = p.kcap[s];
    it.seg = reinterpret_cast<const SegD*>(db) + seg0[s];
    it.pair = reinterpret_cast<const PairD*>(db + o1) + pair0[s];
    it.wb = reinterpret_cast<const WbD*>(db + o2) + wb0[s];
    it.D = W + p.d_off[s];
    it.colseg = FI + csoff[s];
    it.colnat = FI + cnoff[s];
    it.stepof = FI + stoff[s];
    it.piv = FI + pvoff[s];
    it.segoff = FI + sgoff[s];
    it.vidx = FV + vxoff[s];
    it.voff = L->voff[s];
  }
  point_items(p, lay, F, &items);
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
  L->cdims.assign(p.ncolours, SplitDims{0, 0, 0, 0, 0});
  L->max_items = 0;
  L->max_nseg = 0;
  L->max_acap = 0;
  for (int c = 0; c < p.ncolours; ++c) {
    L->max_items = std::max(L->max_items, p.cstart[c + 1] - p.cstart[c]);
    SplitDims& d = L->cdims[c];
    for (int idx = p.cstart[c]; idx < p.cstart[c + 1]; ++idx) {
      const ItemD& it = items[idx];
      d.max_m = std::max(d.max_m, it.m);
      d.max_nseg = std::max(d.max_nseg, it.nseg);
      d.max_pcap = std::max(d.max_pcap, it.pcap);
      d.max_acap = std::max(d.max_acap, p.acap[it.s - sbase]);
      d.max_bcap = std::max(d.max_bcap, p.bcap[it.s - sbase]);
    }
    L->max_nseg = std::max(L->max_nseg, d.max_nseg);
    L->max_acap = std::max(L->max_acap, d.max_acap);
  }
  // hipMemcpyAsync from pageable memory may return before the copy is done
  HIPCHK(hipStreamSynchronize(st));
  L->h_items = std::move(items);
  L->sol_k.clear();  // the new items carry no stores yet
  L->sol_a.clear();
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

lrsp_status plan_stores(LevelDev* L, hipStream_t st, bool* changed) {
  *changed = false;
  const LevelPlan& p = L->plan;
  const int M = p.M;
  if (L->sol.p && L->sol_k == L->k && L->sol_a == L->a) return LRSP_OK;
  auto al = [](int64_t v) { return (v + 31) & ~(int64_t)31; };
  std::vector<int64_t> off(M);
  int64_t tot = 0;
  for (int idx = 0; idx < M; ++idx) {
    const int s = p.order[idx];
    const int64_t m = p.m[s], a = L->a[s], k = L->k[s];
    off[idx] = tot;
    tot += al(m * (m + a + k) + k);
  }
  dfree(&L->sol, st);
  HIPCHK(dalloc(&L->sol, sizeof(double) * (size_t)std::max<int64_t>(tot, 1), st));
  double* base = at<double>(L->sol, 0);
  for (int idx = 0; idx < M; ++idx) {
    const int s = p.order[idx];
    ItemD& it = L->h_items[idx];
    it.S = base + off[idx];
    it.sa = L->a[s];
    it.sk = L->k[s];
  }
  L->sol_k = L->k;
  L->sol_a = L->a;
  *changed = true;
  return LRSP_OK;
}

bool complete_graph(const std::vector<std::vector<int>>& adj) {
  const int M = (int)adj.size();
  for (int x = 0; x < M; ++x)
    if ((int)adj[x].size() != M - 1) return false;
  return true;
}

lrsp_status level0_offsets(const TreeH& tr, const int64_t* rp, const int32_t* cl, int64_t nnz,
                           const LevelPlan& p, std::vector<int64_t>* off) {
  off->assign(nnz, -1);
  for (int64_t i = 0; i < tr.n; ++i) {
    const int pc = tr.dof_cluster[i], li = tr.dof_local[i];
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int j = cl[e];
      const int q = tr.dof_cluster[j], lj = tr.dof_local[j];
      if (q == pc) {
        (*off)[e] = p.d_off[pc] + li + (int64_t)p.m[pc] * lj;
      } else if (p.pos[pc] < p.pos[q]) {
        const uint64_t key = pkey(pc, q);
        const std::vector<int>& z = p.zfin.at(key);
        const int col = (int)(std::lower_bound(z.begin(), z.end(), lj) - z.begin());
        if (col >= (int)z.size() || z[col] != lj)
          return fail(LRSP_ERR_INTERNAL, "level-0 entry outside its fine column set");
        (*off)[e] = p.hf_off.at(key) + li + (int64_t)p.m[pc] * col;
      }
    }
  }
  return LRSP_OK;
}

void top_offsets_level0(const TreeH& tr, const int64_t* rp, const int32_t* cl, int64_t nnz,
                        const std::vector<int64_t>& toff, int ntop, std::vector<int64_t>* off) {
  off->assign(nnz, -1);
  for (int64_t i = 0; i < tr.n; ++i) {
    const int pc = tr.dof_cluster[i], li = tr.dof_local[i];
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int j = cl[e];
      const int q = tr.dof_cluster[j], lj = tr.dof_local[j];
      (*off)[e] = (toff[pc] + li) + (int64_t)ntop * (toff[q] + lj);
    }
  }
}

void top_tasks(const LevelDev& prev, const std::vector<int64_t>& toff, int ntop, double* Tm,
               std::vector<CopyD>* tasks) {
  const std::vector<int>& k = prev.k;
  const int Mp = prev.plan.M;
  std::vector<int64_t> xo(Mp);
  for (int x = 0; x < Mp; ++x) xo[x] = toff[x / 2] + ((x & 1) ? k[x - 1] : 0);
  for (int x = 0; x < Mp; ++x) {
    if (k[x] > 0)
      tasks->push_back(CopyD{at<double>(prev.work, prev.plan.d_off[x]),
                             Tm + xo[x] + (size_t)ntop * xo[x], prev.plan.m[x], ntop, k[x], k[x], 0, 0});
    for (int y : prev.plan.adj2[x]) {
      const double* src;
      int sld, trn;
      if (k[x] > 0 && k[y] > 0 && coupling(prev, x, y, &src, &sld, &trn))
        tasks->push_back(CopyD{src, Tm + xo[x] + (size_t)ntop * xo[y], sld, ntop, k[x], k[y], trn, 0});
    }
  }
}

void level_stats(LevelDev* L, double flops[5]) {
  const LevelPlan& p = L->plan;
  for (int i = 0; i < 5; ++i) flops[i] = 0.0;
  L->sweep_bytes.assign(p.ncolours, 0.0);
  for (int s = 0; s < p.M; ++s) {
    const double m = p.m[s], a = L->a[s], b = L->b[s], k = L->k[s];
    double f[5] = {m * m * m / 3.0, m * m * (a + b), 0.0, 0.0, a * (a + 1.0) * (m - k)};
    for (int j = 0; j < k; ++j) {
      f[2] += 4.0 * (m - j) * (b - j);
      f[3] += 4.0 * (m - j) * a;
    }
    for (int i = 0; i < 5; ++i) flops[i] += f[i];
    // one sweep reads G (lower), the k reflectors and F once, and reads and
    // writes the cluster's and its near field's vector entries
    L->sweep_bytes[p.colour[s]] +=
        8.0 * (m * (m + 1) / 2.0 + k * m + (m - k) * a) + 8.0 * (2.0 * m + 2.0 * a);
  }
}

}  // namespace rt
}  // namespace lrsp
