// api.cpp -- C interface of the hierarchical solver (see include/lrsp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lrsp.h"
#include "desc.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "learned.hpp"
#include "runtime.hpp"

using namespace lrsp;
using namespace lrsp::rt;

namespace {

// Analysis of the last pattern factored with a tree (with a copy of that
// pattern to recognise it), and level workspaces returned by freed factors.
struct TreeCache {
  bool have = false;
  uint64_t gen = 0;  // advanced whenever the analysed pattern changes
  uint64_t id = 0;   // the caller's pattern id of that pattern (0: none)
  // the last factorization reused every level and found the ranks (k, a, b)
  // of the one before: the next one may assume them (spec_ok)
  bool spec_ok = false;
  int64_t nnz = -1;
  std::vector<int64_t> rp;
  std::vector<int32_t> cl;
  std::vector<std::vector<int>> adj0;
  std::unordered_map<uint64_t, std::vector<uint64_t>> z0;
  std::vector<std::unique_ptr<LevelDev>> levels;
  DevBuf perm;  // the tree's DoF permutation on the device, returned by freed factors
  PanelArena arena;  // panel workspace shared by the levels
  hipStream_t stream = nullptr;
  ~TreeCache() {
    int64_t held = 0;
    for (auto& L : levels)
      if (L) {
        held += L->held_bytes();
        L->free_all(stream);
      }
    dfree(&perm, stream);
    if (arena.used && arena.stream != stream) (void)hipStreamSynchronize(arena.stream);
    held += (int64_t)arena.buf.bytes;
    dfree(&arena.buf, stream);
    (void)hipStreamSynchronize(stream);
    if (held > (int64_t)kPoolKeepBytes) pool_trim();
  }
  bool same_pattern(const int64_t* r, const int32_t* c, int64_t n, int64_t z, uint64_t pid) const {
    if (!have || nnz != z || (int64_t)rp.size() != n + 1) return false;
    if (std::memcmp(rp.data(), r, sizeof(int64_t) * (size_t)(n + 1)) != 0) return false;
    if (pid != 0 && pid == id) {
      // a named pattern: the row pointers are equal; the column indices are
      // checked at up to 4096 evenly spaced entries (a pattern with the same
      // id but other columns is caught there unless it differs only between
      // the samples, which the id's contract excludes)
      const int64_t step = z > 4096 ? z / 4096 : 1;
      for (int64_t i = 0; i < z; i += step)
        if (cl[(size_t)i] != c[i]) return false;
      return z == 0 || cl[(size_t)z - 1] == c[z - 1];
    }
    return std::memcmp(cl.data(), c, sizeof(int32_t) * (size_t)z) == 0;
  }
};

}  // namespace

struct lrsp_tree {
  TreeH t;
  std::shared_ptr<TreeCache> cache = std::make_shared<TreeCache>();
};

struct lrsp_factorization {
  int64_t n = 0;
  int exec_mode = 0;  // 1: the sweeps too run one launch per colour
  bool nodc = false;  // eliminated without deferred compression (sweeps per colour)
  std::vector<std::unique_ptr<LevelDev>> levels;
  // dense top
  int top_n = 0;
  int top_level = 0;
  DevBuf top;             // L (n_top x n_top)
  int64_t top_vbase = 0;
  DevBuf top_gidx;        // indices into the last level's vector (or unused)
  std::vector<int> top_sizes, top_adj_ptr, top_adj;
  DevBuf perm;            // level-0 cluster order
  DevBuf vec;             // all level vectors, then their shadow copy
  int64_t vec_total = 0;
  DevBuf scratch;         // PCG work vectors / scalars
  size_t scratch_n = 0;
  lrsp_info info{};
  hipStream_t stream = nullptr;
  std::weak_ptr<TreeCache> cache;
  uint64_t pattern = 0;  // TreeCache::gen of the pattern factored
  // Per-level statistics (lrsp_factor_level_stats).  With timing on, an
  // event at the start of every level, one before and one after the dense
  // top, and one pair around each level's forward and backward sweep of
  // every apply.
  std::vector<double> lev_flops, lev_sweep_bytes;
  std::vector<hipEvent_t> lev_ev;
  mutable std::vector<std::vector<std::pair<hipEvent_t, hipEvent_t>>> sweep_ev;
  mutable int64_t timed_applies = 0;
  hipEvent_t new_event() {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~lrsp_factorization() {
    for (hipEvent_t e : lev_ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& v : sweep_ev)
      for (auto& pr : v) {
        if (pr.first) (void)hipEventDestroy(pr.first);
        if (pr.second) (void)hipEventDestroy(pr.second);
      }
    std::shared_ptr<TreeCache> c = cache.lock();
    const bool give = c && c->have && c->gen == pattern;
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
    if (c && perm.p) {  // the permutation belongs to the tree: back to its cache
      dfree(&c->perm, stream);
      c->perm = perm;
      c->stream = stream;
      perm = DevBuf{};
    }
    dfree(&top, stream); dfree(&top_gidx, stream); dfree(&perm, stream); dfree(&vec, stream);
    dfree(&scratch, stream);
    (void)hipStreamSynchronize(stream);
    if (!give && info.peak_bytes > (int64_t)kPoolKeepBytes) pool_trim();
  }
};


const TreeH& lrsp::rt::tree_of(const lrsp_tree* t) { return t->t; }

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

const char* lrsp_last_error_info(void) { return last_error(); }

lrsp_status lrsp_tree_build(const lrsp_grid* g, int32_t leaf_size, lrsp_tree** out) {
  if (!g || !out) return fail(LRSP_ERR_ARG, "null argument");
  auto t = std::make_unique<lrsp_tree>();
  if (build_tree(g->nx, g->ny, g->nz, g->ncomp, leaf_size, &t->t) != 0)
    return fail(LRSP_ERR_ARG, "invalid grid/leaf size (leaf < nz*ncomp or a column would be split)");
  *out = t.release();
  return LRSP_OK;
}

lrsp_status lrsp_tree_build_graph(int64_t ncols, const int64_t* adj_ptr, const int32_t* adj, int32_t nz,
                                  int32_t ncomp, int32_t leaf_size, lrsp_tree** out) {
  if (!out || !adj_ptr) return fail(LRSP_ERR_ARG, "null argument");
  auto t = std::make_unique<lrsp_tree>();
  if (build_tree_graph(ncols, adj_ptr, adj, nz, ncomp, leaf_size, &t->t) != 0)
    return fail(LRSP_ERR_ARG,
                "invalid layer graph or leaf size (leaf < nz*ncomp, an index out of range, a self loop, "
                "or a part that would have to split a column)");
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

// Rank capacities of a level from the ranks k a previous factorization of the
// same pattern found: k plus a quarter, at least 2 more.
static std::vector<int> reuse_caps(const std::vector<int>& k) {
  std::vector<int> c(k.size());
  for (size_t i = 0; i < k.size(); ++i) c[i] = k[i] + std::max(2, k[i] / 4);
  return c;
}

// *retry: set when a level assumed the ranks of the previous factorization
// wrongly; the caller then runs factor_impl again, which no longer assumes.
static lrsp_status factor_impl(const lrsp_csr* A, lrsp_tree* T, double tol, const lrsp_opts* opts,
                               void* stream, lrsp_factorization** out, bool* retry) {
  *retry = false;
  if (!A || !T || !out) return fail(LRSP_ERR_ARG, "null argument");
  *out = nullptr;
  const TreeH& tr = T->t;
  if (A->n != tr.n) return fail(LRSP_ERR_ARG, "matrix size does not match the tree");
  if (!(tol >= 0.0)) return fail(LRSP_ERR_ARG, "tol must be >= 0");
  if (!A->rowptr || !A->col || !A->val) return fail(LRSP_ERR_ARG, "null CSR array");
  lrsp_opts o{};
  if (opts) o = *opts;
  if (o.gemm_prec < 0 || o.gemm_prec > 2 || o.tol_mode < 0 || o.tol_mode > 1 || o.exec_mode < 0 ||
      o.exec_mode > 3 || o.rank_mode < 0 || o.rank_mode > 1 || o.autotune < 0 || o.autotune > 1 ||
      o.top_dense_threshold < 0 || o.top_dense_threshold > kTopMaxDofs || o.scheme < 0 || o.scheme > 1)
    return fail(LRSP_ERR_ARG, "invalid option");
  const bool learned = o.rank_mode == 1;
  if (learned && !o.mlp_weights) return fail(LRSP_ERR_ARG, "rank_mode 1 needs mlp_weights");
  const bool nodc = o.scheme == 1;
  if (nodc && learned) return fail(LRSP_ERR_ARG, "scheme 1 (no deferred compression) with rank_mode 1");
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
  F->exec_mode = o.exec_mode;
  F->nodc = nodc;
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
  if (cache->same_pattern(rp, cl, A->n, A->nnz, A->pattern_id)) {
    cache->id = A->pattern_id;
  } else {
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
    cache->rp.assign(rp, rp + A->n + 1);
    cache->cl.assign(cl, cl + A->nnz);
    cache->have = true;
    cache->id = A->pattern_id;
    ++cache->gen;
    cache->nnz = A->nnz;
    ms_an += ms_since(ta);
  }
  F->pattern = cache->gen;
  std::vector<std::vector<int>> adj = cache->adj0;
  int reused = 0;
  if (cache->perm.p) {  // uploaded by an earlier factorization with this tree
    F->perm = cache->perm;
    cache->perm = DevBuf{};
  } else {
    HIPCHK(dalloc(&F->perm, sizeof(int64_t) * tr.n, st));
    HIPCHK(hipMemcpyAsync(F->perm.p, tr.perm.data(), sizeof(int64_t) * tr.n, hipMemcpyHostToDevice, st));
  }
  double flops[6] = {0, 0, 0, 0, 0, 0};
  int64_t vbase = 0;
  int level = 0;
  LevelDev* prev = nullptr;
  std::vector<int32_t> herr(4);
  DevBuf d_mlp;  // learned ranks: the network's parameters on the device
  if (learned) {
    if (lrsp_status s = upload(&d_mlp, o.mlp_weights, sizeof(float) * kMlpParams, st)) return s;
  }
  double cap_bytes = 0.0, worst_bytes = 0.0;
  int checks_pass = 0, checks_fail = 0, cap_redo = 0, cap_reruns = 0;
  // With spec, a reused level assumes the k, a, b of the previous
  // factorization of this pattern (held by its workspace) instead of waiting
  // for them: its read-back goes to pinned memory and is compared after the
  // last kernel; a difference runs the whole factorization again without
  // assuming.  The host then queues level after level while the GPU works.
  const bool spec_on = !learned && cache->spec_ok;
  cache->spec_ok = false;  // set again only by a factorization that completes
  std::vector<LevelDev*> specs;
  bool same_ranks = true;  // every level reused, read-back k, a, b as assumed
  // Checks the levels that assumed their ranks, in level order, once the
  // stream has been synchronized: a level's error words are its own (the
  // levels below it were checked first), then its ranks.  1: ranks differ,
  // run again; 0: all as assumed.
  auto check_specs = [&](lrsp_status* err) -> int {
    *err = LRSP_OK;
    for (LevelDev* Ls : specs) {
      const int Ms = Ls->plan.M;
      const int32_t* h = Ls->h_kab;
      const int32_t* e = h + 3 * Ms;
      if (e[0] && e[3] == kErrCapacity) {  // a rank outgrew a capacity: run again, per level
        cache->spec_ok = false;
        *retry = true;
        return 1;
      }
      if (e[0]) {
        if (e[3] == kErrNotSPD)
          *err = fail(LRSP_ERR_NOT_SPD, "non-positive pivot in the diagonal block of cluster " +
                                            std::to_string(e[2]) + " at level " + std::to_string(e[1]));
        else
          *err = fail(LRSP_ERR_INTERNAL, "device check failed (code " + std::to_string(e[3]) + ") at level " +
                                             std::to_string(e[1]) + " cluster " + std::to_string(e[2]));
        return 0;
      }
      if (!std::equal(Ls->k.begin(), Ls->k.end(), h) || !std::equal(Ls->a.begin(), Ls->a.end(), h + Ms) ||
          !std::equal(Ls->b.begin(), Ls->b.end(), h + 2 * Ms)) {
        cache->spec_ok = false;
        *retry = true;
        return 1;
      }
    }
    specs.clear();
    return 0;
  };
  // a level whose coarse halves were allocated anew: the assembly tasks of
  // the next level, which copy from them, are built again
  auto next_level_tasks_stale = [&](int l) {
    if ((int)cache->levels.size() > l + 1 && cache->levels[l + 1]) cache->levels[l + 1]->tasks_src = 0;
  };
  while (true) {
    const int M = (int)sizes.size();
    if (M == 1 || complete_graph(adj)) break;
    if (o.top_dense_threshold > 0) {  // "small enough": the dense top takes the rest
      int64_t tot = 0;
      for (int x : sizes) tot += x;
      if (tot <= o.top_dense_threshold) break;
    }
    std::unique_ptr<LevelDev> Lp;
    bool reuse = false;
    // the split schedule (auto or forced) needs room for explicit inverses
    const bool want_gi = !nodc && (o.exec_mode == 0 || o.exec_mode == 3);
    if (!learned && (int)cache->levels.size() > level && cache->levels[level] &&
        (cache->levels[level]->want_gi || !want_gi) &&
        cache->levels[level]->plan.m == sizes && cache->levels[level]->vbase == vbase) {
      Lp = std::move(cache->levels[level]);
      reuse = true;
      ++reused;
    }
    const auto ta = tick();
    if (!reuse) {
      Lp = std::make_unique<LevelDev>();
      Lp->want_gi = want_gi;
      Lp->plan.M = M;
      Lp->plan.m = sizes;
      Lp->plan.adj = adj;
      plan_level(&Lp->plan, level == 0 ? &cache->z0 : nullptr);
      if (lrsp_status s = setup_level_a(Lp.get(), st, vbase)) return s;
      if (learned) {
        // what the worst-case capacities min(m, b) would allocate
        worst_bytes += 8.0 * (double)(Lp->plan.coarse_doubles + plan_panel_doubles(Lp->plan));
      } else if (lrsp_status s = setup_level_b(Lp.get(), st, 0, nullptr, nullptr, &cache->arena)) {
        return s;
      }
    } else {
      launch_zero(at<double>(Lp->work, 0), Lp->plan.work_doubles, st);
      launch_zero(at<double>(Lp->coarse, 0), Lp->plan.coarse_doubles, st);
      launch_zero_i32(at<int32_t>(Lp->state, 0), 4 * (int64_t)M + 8, st);
      if (!Lp->capped && (int)Lp->k.size() == M) {
        // the level ran before with the worst-case rank capacities: from now
        // on the ranks it found, with some room, size its coarse halves and
        // panels (a rank that outgrows them makes the level run again with
        // more room, as with learned ranks)
        Lp->caps = reuse_caps(Lp->k);
        plan_capacities(&Lp->plan, &Lp->caps);
        Lp->capped = true;
        Lp->cap_tries = 0;
        if (lrsp_status s = setup_level_b(Lp.get(), st, 0, nullptr, nullptr, &cache->arena)) return s;
        next_level_tasks_stale(level);
      } else if (Lp->arena_gen != cache->arena.gen) {
        // the shared panel arena was allocated anew since the level last ran
        if (lrsp_status s = rebind_panels(Lp.get(), st, &cache->arena)) return s;
      } else {
        arena_use(&cache->arena, st);
      }
    }
    LevelDev* L = Lp.get();
    vbase += L->nvec;
    if (g_tm.on) {  // start of this level's GPU work (its assembly included)
      hipEvent_t e = F->new_event();
      if (e) (void)hipEventRecord(e, st);
      F->lev_ev.push_back(e);
    }
    // assemble the level's matrix
    if (level == 0 && L->vals_off.p) {
      launch_scatter_vals(A->val, at<int64_t>(L->vals_off, 0), A->nnz, at<double>(L->work, 0), st);
    } else if (level == 0) {
      std::vector<int64_t> off;
      if (lrsp_status s = level0_offsets(tr, rp, cl, A->nnz, L->plan, &off)) return s;
      if (lrsp_status s = upload(&L->vals_off, off.data(), off.size() * 8, st)) return s;
      launch_scatter_vals(A->val, at<int64_t>(L->vals_off, 0), A->nnz, at<double>(L->work, 0), st);
    } else {
      if (!(reuse && L->tasks_src == prev->id && L->tasks.p)) {
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
        coarse_gather_indices(*prev, M, &g);
        dfree(&L->gidx, st);
        if (lrsp_status s = upload(&L->gidx, g.data(), g.size() * 8, st)) return s;
      }
      if (L->ntasks > 0) launch_copy_blocks(at<CopyD>(L->tasks, 0), L->ntasks, st);
    }
    if (learned) {
      // level-start features -> predicted ranks -> rank capacities
      if (lrsp_status s = predict_level(L, level, tol, at<float>(d_mlp, 0), st, &L->feat, &L->pred)) return s;
      L->caps = rank_caps(L->pred);
      plan_capacities(&L->plan, &L->caps);
      L->capped = true;
      L->cap_tries = 0;
      if (lrsp_status s = setup_level_b(L, st, 0, nullptr, nullptr, &cache->arena)) return s;
    }
    if (!reuse) ms_an += ms_since(ta);
    // eliminate the clusters colour by colour
    const LevelPlan& p = L->plan;
    // without deferred compression: one workgroup per cluster (the fused
    // kernels), persistent unless one launch per colour was asked for
    const int mode = nodc ? (o.exec_mode == 1 ? 1 : 2) : (o.exec_mode == 0 ? 3 : o.exec_mode);
    L->split = mode == 3 && L->max_m >= kSplitMinDofs && L->max_m <= kSplitMaxDofs;
    L->ls.nodc = nodc ? 1 : 0;
  eliminate_level:
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
    // k, a, b and the error words lie back to back in the state buffer: one copy
    const size_t nkab = 3 * (size_t)M + 4;
    const bool spec = spec_on && reuse && L->k.size() == (size_t)M && L->a.size() == (size_t)M &&
                      L->b.size() == (size_t)M;
    if (spec) {
      if (L->h_kab_n < nkab) {
        if (L->h_kab) {
          HIPCHK(hipStreamSynchronize(st));
          HIPCHK(hipHostFree(L->h_kab));
          L->h_kab = nullptr;
          L->h_kab_n = 0;
        }
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&L->h_kab), 4 * nkab, hipHostMallocDefault));
        L->h_kab_n = nkab;
      }
      HIPCHK(hipMemcpyAsync(L->h_kab, L->ls.k, 4 * nkab, hipMemcpyDeviceToHost, st));
      specs.push_back(L);
      herr.assign(4, 0);
    } else {
      std::vector<int32_t> kab(nkab);
      HIPCHK(hipMemcpyAsync(kab.data(), L->ls.k, 4 * kab.size(), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (!specs.empty()) {  // this level's input rests on the assumed ranks below it
        lrsp_status e;
        if (check_specs(&e)) return LRSP_ERR_INTERNAL;
        if (e) return e;
      }
      if (!reuse || L->k.size() != (size_t)M || !std::equal(L->k.begin(), L->k.end(), kab.begin()) ||
          !std::equal(L->a.begin(), L->a.end(), kab.begin() + M) ||
          !std::equal(L->b.begin(), L->b.end(), kab.begin() + 2 * M))
        same_ranks = false;
      L->k.assign(kab.begin(), kab.begin() + M);
      L->a.assign(kab.begin() + M, kab.begin() + 2 * M);
      L->b.assign(kab.begin() + 2 * M, kab.begin() + 3 * M);
      herr.assign(kab.begin() + 3 * M, kab.end());
    }
    if (herr[0] && herr[3] == kErrCapacity && L->capped) {
      // a rank reached its capacity (predicted, or from the ranks found
      // before): the clusters whose QR stopped at a capacity below their
      // worst case min(m, b) get the worst case,
      // the others keep theirs, and the level runs again from its assembled
      // input.  A cluster eliminated after a truncated one can see other
      // values in the new run, so this repeats, at most kCapRetries times
      // before every capacity of the level is the worst case.
      if (L->cap_tries++ == 0) ++cap_redo;
      ++cap_reruns;
      bool raised = false;
      for (int x = 0; x < M; ++x) {
        const int worst = std::min(p.m[x], p.bcap[x]);
        if (L->k[x] >= p.kcap[x] && p.kcap[x] < worst) {
          L->caps[x] = std::numeric_limits<int>::max();
          raised = true;
        }
      }
      if (raised && L->cap_tries <= kCapRetries) {
        plan_capacities(&L->plan, &L->caps);
      } else {
        plan_capacities(&L->plan, nullptr);
        L->capped = false;
      }
      if (lrsp_status s = setup_level_b(L, st, 0, nullptr, nullptr, &cache->arena)) return s;
      next_level_tasks_stale(level);
      launch_zero(at<double>(L->work, 0), L->plan.work_doubles, st);
      if (level == 0) {
        launch_scatter_vals(A->val, at<int64_t>(L->vals_off, 0), A->nnz, at<double>(L->work, 0), st);
      } else if (L->ntasks > 0) {
        launch_copy_blocks(at<CopyD>(L->tasks, 0), L->ntasks, st);
      }
      L->split = mode == 3 && L->max_m >= kSplitMinDofs && L->max_m <= kSplitMaxDofs;
      goto eliminate_level;
    }
    if (herr[0]) {
      if (herr[3] == kErrNotSPD)
        return fail(LRSP_ERR_NOT_SPD, "non-positive pivot in the diagonal block of cluster " +
                                          std::to_string(herr[2]) + " at level " +
                                          std::to_string(herr[1]));
      return fail(LRSP_ERR_INTERNAL, "device check failed (code " + std::to_string(herr[3]) +
                                         ") at level " + std::to_string(herr[1]) + " cluster " +
                                         std::to_string(herr[2]));
    }
    if (learned) {
      cap_bytes += 8.0 * (double)(L->plan.coarse_doubles + plan_panel_doubles(L->plan));
      for (int x = 0; x < M; ++x) {
        // check of the predicted rank: the pivot after the predicted rank
        // already met the stop rule (k <= k_hat), or the QR went on
        if (L->k[x] <= (int)std::lround(std::max(0.0f, L->pred[x]))) ++checks_pass;
        else ++checks_fail;
      }
    }
    {  // what the sweeps read, into the clusters' factor stores
      bool changed = false;
      if (lrsp_status s = plan_stores(L, st, &changed)) return s;
      if (changed)
        HIPCHK(hipMemcpyAsync(L->d_items, L->h_items.data(), sizeof(ItemD) * (size_t)M, hipMemcpyHostToDevice, st));
      TimedLaunch tall(0, st);
      launch_compact(L->d_items, M, L->ls, st);
    }
    double f[5];
    level_stats(L, f);
    double lvl_flops = 0.0;
    for (int i = 0; i < 5; ++i) {
      flops[i] += f[i];
      lvl_flops += f[i];
      if (g_tm.on && L->split) g_tm.flops[4 + i] += f[i];
    }
    if (g_tm.on && L->split) {
      for (int s = 0; s < M; ++s) {
        const double m = p.m[s], a = L->a[s], b = L->b[s], k = L->k[s];
        g_tm.bytes[3] += 16.0 * m * (m + a + b);  // panel gathered: read + write
        g_tm.bytes[9] += 16.0 * k * (a + b);
      }
    }
    if (g_tm.on) {
      g_tm.flops[0] += lvl_flops;
      if (!L->split) g_tm.flops[10] += lvl_flops;
    }
    F->lev_flops.push_back(lvl_flops);
    {
      double by = 0.0;
      for (double v : L->sweep_bytes) by += v;
      F->lev_sweep_bytes.push_back(by);
    }
    // next level
    std::vector<int> nsz(M / 2);
    for (int P = 0; P < M / 2; ++P) nsz[P] = L->k[2 * P] + L->k[2 * P + 1];
    // the next graph depends on the structure only: kept with the level's
    // workspace and reused with it
    if (!reuse || L->next_adj.size() != (size_t)(M + 1) / 2) coarsen_square(adj, &L->next_adj);
    std::vector<std::vector<int>> nadj = L->next_adj;
    sizes.swap(nsz);
    adj.swap(nadj);
    prev = L;
    F->levels.push_back(std::move(Lp));
    ++level;
  }
  // dense top
  if (g_tm.on) {
    hipEvent_t e = F->new_event();
    if (e) (void)hipEventRecord(e, st);
    F->lev_ev.push_back(e);
  }
  const int M = (int)sizes.size();
  int ntop = 0;
  std::vector<int64_t> toff(M + 1, 0);
  for (int x = 0; x < M; ++x) toff[x + 1] = toff[x] + sizes[x];
  ntop = (int)toff[M];
  if (ntop > kTopMaxDofs)
    return fail(LRSP_ERR_ARG, "dense top system larger than " + std::to_string(kTopMaxDofs));
  F->top_n = ntop;
  F->top_level = level;
  F->top_sizes = sizes;
  F->top_adj_ptr.assign(1, 0);
  for (int x = 0; x < M; ++x) {
    F->top_adj.insert(F->top_adj.end(), adj[x].begin(), adj[x].end());
    F->top_adj_ptr.push_back((int)F->top_adj.size());
  }
  // n x (n + 64) (the blocked Cholesky of large tops forms its diagonal
  // blocks' inverses in the last 64 columns), then for such tops the n x n
  // inverse of the factor and 64 columns of the solve's partial sums (the
  // solve keeps its other partial sums in the factor's 64 extra columns)
  const int64_t top_cols = ntop > kSplitMaxDofs ? 2 * (int64_t)ntop + 128 : (int64_t)ntop + 64;
  HIPCHK(dalloc(&F->top, sizeof(double) * std::max<int64_t>(1, (int64_t)ntop * top_cols), st));
  double* Tm = at<double>(F->top, 0);
  launch_zero(Tm, (int64_t)ntop * ntop, st);
  if (level == 0) {
    std::vector<int64_t> off;
    top_offsets_level0(tr, rp, cl, A->nnz, toff, ntop, &off);
    DevBuf doff;
    if (lrsp_status s = upload(&doff, off.data(), off.size() * 8, st)) return s;
    launch_scatter_vals(A->val, at<int64_t>(doff, 0), A->nnz, Tm, st);
    dfree(&doff, st);
  } else {
    std::vector<CopyD> tasks;
    top_tasks(*prev, toff, ntop, Tm, &tasks);
    DevBuf dt;
    if (!tasks.empty()) {
      if (lrsp_status s = upload(&dt, tasks.data(), tasks.size() * sizeof(CopyD), st)) return s;
      launch_copy_blocks(at<CopyD>(dt, 0), (int)tasks.size(), st);
      dfree(&dt, st);
    }
    std::vector<int64_t> g;
    coarse_gather_indices(*prev, M, &g);
    if (lrsp_status s = upload(&F->top_gidx, g.data(), g.size() * 8, st)) return s;
  }
  DevBuf terr;
  HIPCHK(dalloc(&terr, 16, st));
  launch_zero_i32(at<int32_t>(terr, 0), 4, st);
  if (ntop >= 64 && ntop <= kSplitMaxDofs) launch_top_potrf_wg(Tm, ntop, at<int32_t>(terr, 0), st);
  else if (ntop > kSplitMaxDofs)  // with the factor's inverse, which the solve applies
    launch_top_potrf_blocked(Tm, ntop, at<int32_t>(terr, 0), 0, st, Tm + (size_t)ntop * (ntop + 64));
  else launch_top_potrf(Tm, ntop, at<int32_t>(terr, 0), st);
  HIPCHK(hipGetLastError());
  if (g_tm.on) {
    hipEvent_t e = F->new_event();
    if (e) (void)hipEventRecord(e, st);
    F->lev_ev.push_back(e);
  }
  HIPCHK(hipMemcpyAsync(herr.data(), terr.p, 16, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  dfree(&terr, st);
  {  // the levels that assumed their ranks
    lrsp_status e;
    if (check_specs(&e)) return LRSP_ERR_INTERNAL;
    if (e) return e;
  }
  // every level reused and every rank as the workspace held it (the assumed
  // ones were just checked): the next factorization may assume them
  cache->spec_ok = !learned && level > 0 && reused == level && same_ranks;
  const size_t arena_held = cache->arena.buf.bytes;  // held while the levels ran
  {  // an arena far larger than this factorization's levels needed (sized by
     // worst-case capacities before) is given back; the next factorization
     // allocates what it needs
    int64_t need = 0;
    for (auto& L : F->levels) need = std::max(need, L->arena_off + L->arena_doubles);
    if (cache->arena.buf.bytes > sizeof(double) * (size_t)need + (sizeof(double) * (size_t)need) / 2) {
      dfree(&cache->arena.buf, st);
      ++cache->arena.gen;
    }
  }
  if (herr[0]) return fail(LRSP_ERR_NOT_SPD, "non-positive pivot in the dense top factorization");
  flops[5] = (double)ntop * ntop * ntop / 3.0;
  F->top_vbase = vbase;
  F->vec_total = vbase + ntop;
  // the level vectors, then a shadow copy laid out the same way (the
  // forward products of split levels write there)
  HIPCHK(dalloc(&F->vec, sizeof(double) * std::max<int64_t>(1, 2 * F->vec_total), st));
  launch_zero(at<double>(F->vec, 0), 2 * F->vec_total, st);
  HIPCHK(hipStreamSynchronize(st));
  const auto t1 = std::chrono::steady_clock::now();
  lrsp_info& inf = F->info;
  inf.nlevels = (int)F->levels.size();
  inf.top_n = ntop;
  inf.top_clusters = M;
  for (int i = 0; i < 6; ++i) inf.flops[i] = flops[i];
  double fb = (double)F->top.bytes;
  for (auto& L : F->levels) fb += (double)L->factor_bytes();
  inf.bytes_factor = fb;
  inf.ms_levels = std::chrono::duration<double, std::milli>(t1 - t0).count();
  inf.ms_analysis = ms_an;
  inf.levels_reused = reused;
  inf.rank_bytes = learned ? cap_bytes : 0.0;
  inf.rank_bytes_worst = learned ? worst_bytes : 0.0;
  inf.rank_checks_passed = checks_pass;
  inf.rank_checks_failed = checks_fail;
  inf.rank_redo_levels = cap_redo;
  inf.rank_reruns = cap_reruns;
  int64_t held = 0;
  for (auto& L : F->levels) held += L->held_bytes();
  inf.peak_bytes = held + (int64_t)(F->top.bytes + F->vec.bytes + F->perm.bytes + arena_held);
  *out = F.release();
  return LRSP_OK;
}

lrsp_status lrsp_factor(const lrsp_csr* A, lrsp_tree* T, double tol, const lrsp_opts* opts,
                        void* stream, lrsp_factorization** out) {
  try {
    bool retry = false;
    const lrsp_status s = factor_impl(A, T, tol, opts, stream, out, &retry);
    return retry ? factor_impl(A, T, tol, opts, stream, out, &retry) : s;
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
  const bool lev_t = g_tm.on;
  if (lev_t) {
    if (F->sweep_ev.size() < (size_t)nl + 1) F->sweep_ev.resize(nl + 1);
    ++F->timed_applies;
  }
  auto lev_event = [&](int l) -> hipEvent_t {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    (void)hipEventRecord(e, st);
    (void)l;
    return e;
  };
  for (int l = 0; l < nl; ++l) {
    const LevelDev& L = *F->levels[l];
    const LevelPlan& p = L.plan;
    hipEvent_t fa = lev_t ? lev_event(l) : nullptr;
    {
      TimedLaunch tl(1, st);
      // levels with split clusters run one launch per colour (plus its units)
      const bool per_colour = F->exec_mode == 1 || F->nodc || sweep_units(true, L.max_m, L.max_acap) > 0;
      if (per_colour ||
          launch_sweep_level(true, L.d_items, L.d_cstart, p.ncolours, p.cstart.back(), L.max_items, L.max_m, L.max_acap, L.ls, V,
                             st, 0, nullptr, L.vbase, L.nvec) != hipSuccess) {
        if (!per_colour) (void)hipGetLastError();
        // after the split schedule every cluster of kSweepSplitM..kInvMaxDofs
        // DoFs keeps W (or G^{-1} when it has no reflector)
        const bool wide = L.split && L.min_m >= kSweepSplitM && L.max_m <= kInvMaxDofs && !F->nodc;
        for (int c = 0; c < p.ncolours; ++c)
          launch_fwd(L.d_items + p.cstart[c], p.cstart[c + 1] - p.cstart[c], L.max_m, L.max_acap, L.ls, V, st,
                     wide ? V + F->vec_total : nullptr);
      }
      if (g_tm.on)
        for (double by : L.sweep_bytes) g_tm.bytes[1] += by;
    }
    if (lev_t) F->sweep_ev[l].push_back({fa, lev_event(l)});
    if (l + 1 < nl) {
      const LevelDev& N = *F->levels[l + 1];
      launch_gather(V, at<int64_t>(N.gidx, 0), V + N.vbase, N.nvec, st);
    } else {
      launch_gather(V, at<int64_t>(F->top_gidx, 0), V + F->top_vbase, F->top_n, st);
    }
  }
  {
    hipEvent_t ta = lev_t ? lev_event(nl) : nullptr;
    launch_top_solve(at<double>(F->top, 0), F->top_n, V + F->top_vbase, st);
    if (lev_t) F->sweep_ev[nl].push_back({ta, lev_event(nl)});
  }
  for (int l = nl - 1; l >= 0; --l) {
    const LevelDev& L = *F->levels[l];
    const LevelPlan& p = L.plan;
    if (l + 1 < nl) {
      const LevelDev& N = *F->levels[l + 1];
      launch_scatter(V + N.vbase, at<int64_t>(N.gidx, 0), V, N.nvec, st);
    } else {
      launch_scatter(V + F->top_vbase, at<int64_t>(F->top_gidx, 0), V, F->top_n, st);
    }
    hipEvent_t ba = lev_t ? lev_event(l) : nullptr;
    {
      TimedLaunch tl(2, st);
      const bool per_colour = F->exec_mode == 1 || F->nodc || sweep_units(false, L.max_m, L.max_acap) > 0;
      if (per_colour ||
          launch_sweep_level(false, L.d_items, L.d_cstart, p.ncolours, p.cstart.back(), L.max_items, L.max_m, L.max_acap, L.ls, V,
                             st, 0, nullptr, L.vbase, L.nvec) != hipSuccess) {
        if (!per_colour) (void)hipGetLastError();
        const bool wide = L.split && L.min_m >= kSweepSplitM && L.max_m <= kInvMaxDofs && !F->nodc;
        for (int c = p.ncolours - 1; c >= 0; --c)
          launch_bwd(L.d_items + p.cstart[c], p.cstart[c + 1] - p.cstart[c], L.max_m, L.max_acap, L.ls, V, st,
                     wide ? V + F->vec_total : nullptr);
      }
      if (g_tm.on)
        for (double by : L.sweep_bytes) g_tm.bytes[2] += by;
    }
    if (lev_t) F->sweep_ev[l].push_back({ba, lev_event(l)});
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

// Algorithmic bytes of one sparse product y = A x: the CSR arrays (8-byte
// values, 4-byte column indices, 8-byte row pointers), x read and y written
// once.
static double spmv_bytes(int64_t n, int64_t nnz) {
  return 12.0 * (double)nnz + 8.0 * (double)(n + 1) + 16.0 * (double)n;
}

// PCG on every right-hand side in turn with the work vectors in `work`
// (4 n + kDotBlocks + 16 doubles of device memory: r, z, p, q, the partial
// sums of the dot products and the scalars).
static lrsp_status pcg_impl(const lrsp_csr* A, const lrsp_factorization* F, const double* b, double* x,
                            int32_t nrhs, double rtol, int32_t maxit, int32_t* iters, double* relres,
                            hipStream_t st, double* work) {
  const int64_t n = A->n;
  double* r = work;
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
        {
          TimedLaunch tl(11, st);
          launch_spmv(A->rowptr, A->col, A->val, p, q, n, st);
          if (g_tm.on) g_tm.bytes[11] += spmv_bytes(n, A->nnz);
        }
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
  if (result != LRSP_OK) (void)fail(result, "PCG reached maxit");
  return result;
}

lrsp_status lrsp_pcg(const lrsp_csr* A, const lrsp_factorization* F, const double* b, double* x,
                     int32_t nrhs, double rtol, int32_t maxit, int32_t* iters, double* relres,
                     void* stream) {
  if (!A || !F || !b || !x || nrhs < 1 || !iters || !relres || A->n != F->n || maxit < 0)
    return fail(LRSP_ERR_ARG, "invalid argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  lrsp_factorization* Fm = const_cast<lrsp_factorization*>(F);
  const size_t need = 4 * (size_t)A->n + kDotBlocks + 16;
  if (Fm->scratch_n < need) {
    dfree(&Fm->scratch, st);
    HIPCHK(dalloc(&Fm->scratch, need * sizeof(double), st));
    Fm->scratch_n = need;
  }
  return pcg_impl(A, F, b, x, nrhs, rtol, maxit, iters, relres, st, at<double>(Fm->scratch, 0));
}

// Work vectors of lrsp_pcg_noalloc: one array per GPU, resident from the
// loading of the library until the process ends (33.6 MB).
static __device__ __align__(256) double scratch[4 * (size_t)LRSP_PCG_NOALLOC_MAX_N + kDotBlocks + 16];

// Device address of `scratch` on each GPU, looked up once per device with
// that device current (the host-side name of the array is not a device
// address and must not be handed to kernels or copies).
static double* scratch_ptr(hipError_t* err) {
  static std::mutex mu;
  static std::unordered_map<int, double*> ptrs;
  int dev = -1;
  if ((*err = hipGetDevice(&dev)) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = ptrs.find(dev);
  if (it != ptrs.end()) return it->second;
  void* p = nullptr;
  if ((*err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess || !p) {
    if (*err == hipSuccess) *err = hipErrorInvalidSymbol;
    return nullptr;
  }
  ptrs[dev] = static_cast<double*>(p);
  return static_cast<double*>(p);
}

lrsp_status lrsp_pcg_noalloc(const lrsp_csr* A, const lrsp_factorization* F, const double* b, double* x,
                             int32_t nrhs, double rtol, int32_t maxit, int32_t* iters, double* relres,
                             void* stream) {
  if (!A || !F || !b || !x || nrhs < 1 || !iters || !relres || maxit < 0)
    return fail(LRSP_ERR_ARG, "invalid argument");
  if (A->n > LRSP_PCG_NOALLOC_MAX_N)
    return fail(LRSP_ERR_ARG, "lrsp_pcg_noalloc: n = " + std::to_string(A->n) +
                                  " exceeds the static work area (n <= " +
                                  std::to_string(LRSP_PCG_NOALLOC_MAX_N) + "); use lrsp_pcg");
  if (A->n != F->n) return fail(LRSP_ERR_ARG, "invalid argument");
  hipError_t e = hipSuccess;
  double* work = scratch_ptr(&e);
  if (!work) return fail(LRSP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  return pcg_impl(A, F, b, x, nrhs, rtol, maxit, iters, relres, reinterpret_cast<hipStream_t>(stream), work);
}

// Restarted GMRES with the factor as right preconditioner: A M^{-1} u = b,
// x = M^{-1} u.  Arnoldi by classical Gram-Schmidt applied twice (two
// block passes over the basis per step), Givens rotations and the
// least-squares solve on the host (the Hessenberg column is read back once
// per step, which is also the convergence test).
static lrsp_status gmres_one(const lrsp_csr* A, const lrsp_factorization* F, const double* b, double* x,
                             int m, double rtol, int maxit, int* iters, double* relres, bool* conv_out,
                             hipStream_t st, double* work) {
  const int64_t n = A->n;
  double* V = work;                          // n x (m + 1)
  double* z = V + (size_t)n * (m + 1);       // M^{-1} v, and M^{-1} V y
  double* w = z + n;                         // A z, residuals
  double* part = w + n;                      // kDotBlocks x (m + 1)
  double* hd = part + (size_t)kDotBlocks * (m + 1);  // [h1 (m+1) | h2 (m+1) | nrm2 | bb]
  double* h2 = hd + (m + 1);
  double* nrm = h2 + (m + 1);
  double* ydev = nrm + 2;                    // m
  std::vector<double> hh(2 * (size_t)(m + 1) + 1), y(m), g(m + 1), cs(m), sn(m);
  std::vector<double> H((size_t)(m + 1) * m);  // column-major (m + 1) x m
  auto Hc = [&](int i, int j) -> double& { return H[(size_t)i + (size_t)(m + 1) * j]; };
  launch_zero(x, n, st);
  launch_dot(b, b, n, part, nrm + 1, st);
  double hb = 0.0;
  HIPCHK(hipMemcpyAsync(&hb, nrm + 1, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double nb = std::sqrt(hb);
  int it = 0;
  bool conv = nb == 0.0;
  while (!conv && it < maxit) {
    // r = b - A x, v0 = r / ||r||
    launch_spmv(A->rowptr, A->col, A->val, x, w, n, st);
    launch_residual(b, w, n, st);
    launch_dot(w, w, n, part, nrm, st);
    double hr = 0.0;
    HIPCHK(hipMemcpyAsync(&hr, nrm, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double beta = std::sqrt(hr);
    if (beta <= rtol * nb) {
      conv = true;
      break;
    }
    launch_normalize(w, V, n, nrm, st);
    const int mm = std::min(m, maxit - it);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < mm; ++j) {
      double* vj = V + (size_t)n * j;
      if (lrsp_status s = apply_one(F, vj, z, st)) return s;
      launch_spmv(A->rowptr, A->col, A->val, z, w, n, st);
      launch_mdot(V, n, j + 1, w, n, part, hd, st);
      launch_gemv_cols(V, n, j + 1, hd, w, n, true, st);
      launch_mdot(V, n, j + 1, w, n, part, h2, st);
      launch_gemv_cols(V, n, j + 1, h2, w, n, true, st);
      launch_dot(w, w, n, part, nrm, st);
      HIPCHK(hipMemcpyAsync(hh.data(), hd, sizeof(double) * (2 * (size_t)(m + 1) + 1), hipMemcpyDeviceToHost, st));
      launch_normalize(w, V + (size_t)n * (j + 1), n, nrm, st);
      HIPCHK(hipStreamSynchronize(st));
      for (int i = 0; i <= j; ++i) Hc(i, j) = hh[i] + hh[(size_t)(m + 1) + i];
      Hc(j + 1, j) = std::sqrt(std::max(0.0, hh[2 * (size_t)(m + 1)]));
      for (int i = 0; i < j; ++i) {  // earlier rotations on the new column
        const double t = cs[i] * Hc(i, j) + sn[i] * Hc(i + 1, j);
        Hc(i + 1, j) = -sn[i] * Hc(i, j) + cs[i] * Hc(i + 1, j);
        Hc(i, j) = t;
      }
      const double a = Hc(j, j), bb = Hc(j + 1, j);
      if (bb == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        const double r = std::hypot(a, bb);
        cs[j] = a / r;
        sn[j] = bb / r;
      }
      Hc(j, j) = cs[j] * a + sn[j] * bb;
      Hc(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      k = j + 1;
      if (std::fabs(g[j + 1]) <= rtol * nb) {
        conv = true;
        break;
      }
      if (Hc(j, j) == 0.0) break;  // breakdown: the least-squares solve below ends the cycle
    }
    for (int i = k - 1; i >= 0; --i) {  // back substitution
      double s = g[i];
      for (int l = i + 1; l < k; ++l) s -= Hc(i, l) * y[l];
      y[i] = Hc(i, i) != 0.0 ? s / Hc(i, i) : 0.0;
    }
    HIPCHK(hipMemcpyAsync(ydev, y.data(), sizeof(double) * (size_t)std::max(k, 1), hipMemcpyHostToDevice, st));
    launch_gemv_cols(V, n, k, ydev, w, n, false, st);
    if (lrsp_status s = apply_one(F, w, z, st)) return s;
    launch_add(x, z, n, st);
    HIPCHK(hipStreamSynchronize(st));  // y stays alive until the copy is done
    if (k == 0) break;
  }
  launch_spmv(A->rowptr, A->col, A->val, x, w, n, st);
  launch_residual(b, w, n, st);
  launch_dot(w, w, n, part, nrm, st);
  double ht = 0.0;
  HIPCHK(hipMemcpyAsync(&ht, nrm, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *iters = it;
  *relres = nb > 0 ? std::sqrt(ht) / nb : 0.0;
  *conv_out = conv;
  return LRSP_OK;
}

lrsp_status lrsp_gmres(const lrsp_csr* A, const lrsp_factorization* F, const double* b, double* x,
                       int32_t nrhs, int32_t restart, double rtol, int32_t maxit, int32_t* iters,
                       double* relres, void* stream) {
  if (!A || !F || !b || !x || nrhs < 1 || restart < 1 || restart > 4096 || !iters || !relres ||
      A->n != F->n || maxit < 0)
    return fail(LRSP_ERR_ARG, "invalid argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t n = A->n;
  const int m = restart;
  const size_t need = (size_t)n * (m + 3) + (size_t)kDotBlocks * (m + 1) + 3 * (size_t)(m + 1) + 8;
  DevBuf buf;
  HIPCHK(dalloc(&buf, need * sizeof(double), st));
  lrsp_status result = LRSP_OK;
  for (int r = 0; r < nrhs; ++r) {
    bool conv = false;
    int it = 0;
    lrsp_status s = gmres_one(A, F, b + (size_t)r * n, x + (size_t)r * n, m, rtol, maxit, &it, relres + r,
                              &conv, st, at<double>(buf, 0));
    if (s != LRSP_OK) {
      dfree(&buf, st);
      return s;
    }
    iters[r] = it;
    if (!conv) result = LRSP_ERR_NO_CONV;
  }
  dfree(&buf, st);
  if (result != LRSP_OK) (void)fail(result, "GMRES reached maxit");
  return result;
}

lrsp_status lrsp_timing_enable(int32_t on) {
  g_tm.on = on != 0;
  return LRSP_OK;
}

lrsp_status lrsp_timing_families(uint32_t mask) {
  g_tm.mask = mask;
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

lrsp_status lrsp_factor_rank_features(const lrsp_factorization* F, int32_t level, double* feat,
                                      float* pred) {
  if (!F || level < 0 || level >= (int)F->levels.size()) return fail(LRSP_ERR_ARG, "invalid level");
  const LevelDev& L = *F->levels[level];
  if (L.feat.empty()) return fail(LRSP_ERR_ARG, "the factor was not computed with learned ranks");
  if (feat) std::copy(L.feat.begin(), L.feat.end(), feat);
  if (pred) std::copy(L.pred.begin(), L.pred.end(), pred);
  return LRSP_OK;
}

lrsp_status lrsp_factor_level_stats(const lrsp_factorization* F, int32_t level, lrsp_level_stats* out) {
  if (!F || !out || level < 0 || level > (int)F->levels.size())
    return fail(LRSP_ERR_ARG, "invalid level");
  const int nl = (int)F->levels.size();
  lrsp_level_stats r{};
  if (level < nl) {
    r.flops = F->lev_flops[level];
    r.sweep_bytes = F->lev_sweep_bytes[level];
    const LevelDev& L = *F->levels[level];
    for (int x = 0; x < L.plan.M; ++x) {
      r.dofs += L.plan.m[x];
      r.coarse += L.k[x];
    }
    r.nclusters = L.plan.M;
    r.factor_bytes = L.factor_bytes();
    r.held_bytes = L.held_bytes();
    r.work_bytes = (int64_t)(L.work.bytes + L.wints.bytes);
    r.coarse_bytes = (int64_t)L.coarse.bytes;
    r.panel_bytes = L.fac.p ? (int64_t)L.fac.bytes : 8 * L.arena_doubles;
  } else {
    r.flops = F->info.flops[5];
    r.dofs = F->top_n;
    r.nclusters = (int32_t)F->top_sizes.size();
    r.factor_bytes = (int64_t)F->top.bytes;
    r.held_bytes = (int64_t)F->top.bytes;
  }
  // factor time: from the start of this level to the start of the next
  // (the top: its factorization alone)
  if ((int)F->lev_ev.size() == nl + 2) {
    HIPCHK(hipEventSynchronize(F->lev_ev[nl + 1]));
    float ms = 0.f;
    if (F->lev_ev[level] && F->lev_ev[level + 1] &&
        hipEventElapsedTime(&ms, F->lev_ev[level], F->lev_ev[level + 1]) == hipSuccess)
      r.factor_ms = ms;
  }
  if ((size_t)level < F->sweep_ev.size()) {
    for (auto& pr : F->sweep_ev[level]) {
      float ms = 0.f;
      if (!pr.first || !pr.second) continue;
      HIPCHK(hipEventSynchronize(pr.second));
      if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) r.solve_ms += ms;
    }
    r.applies = F->timed_applies;
  }
  *out = r;
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
    v->near = nullptr;
    v->far = nullptr;
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
  v->near = L.a.data();
  v->far = L.b.data();
  return LRSP_OK;
}

}  // extern "C"
