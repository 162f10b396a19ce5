// batch.cpp -- batching form: many independent systems factored and solved
// together (see the batching section of include/lrsp.h).
//
// Level l of a batch is the union of level l of every system that is still
// being eliminated.  Each system is planned on its own (in parallel host
// threads); its level storage and descriptors are built with cluster ids
// shifted into one batch-wide LevelState, so one merged work list, ordered
// by colour, drives one launch for the whole level.  Clusters of different
// systems touch disjoint storage, hence the colours of different systems can
// share a round.
//
// Vector buffer: block 0 holds every system's level-0 (or dense top) vector
// at its packed offset; block l >= 1 holds, in system order, the level-l
// vectors of the systems eliminated at l and the top vectors of the systems
// whose top starts at l, gathered from block l-1 by one index list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lrsp.h"
#include "desc.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "runtime.hpp"
#include "tune.hpp"

using namespace lrsp;
using namespace lrsp::rt;

namespace {

// Runs fn(i) for i < n on up to 16 host threads.
template <class Fn>
void parallel_for(int n, Fn fn) {
  const int nt = std::max(1, std::min<int>({16, n, (int)std::thread::hardware_concurrency()}));
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&] {
      for (int i = next++; i < n; i = next++) fn(i);
    });
  for (auto& t : th) t.join();
}

struct BSys {
  const TreeH* tr = nullptr;
  int64_t n = 0, nnz = 0, off = 0;
  std::vector<int64_t> hrp;
  std::vector<int32_t> hcol;
  const int64_t* rp = nullptr;
  const int32_t* cl = nullptr;
  std::vector<std::unique_ptr<LevelDev>> levels;
  std::vector<int> sizes;                 // cluster sizes at the current level
  std::vector<std::vector<int>> adj;      // cluster graph at the current level
  std::unordered_map<uint64_t, std::vector<uint64_t>> z0;
  bool stopped = false;
  int top_level = -1;
  int top_n = 0;
  int64_t top_vbase = 0;
  DevBuf top;
  DevBuf off0;                            // level-0 CSR entry -> offset (level-0 work or top)
  std::vector<int> top_sizes, top_adj_ptr, top_adj;
};

// Items of colour c of a system's level, in processing order.
void append_colour(const LevelDev& L, int c, std::vector<ItemD>* items) {
  const LevelPlan& p = L.plan;
  items->insert(items->end(), L.h_items.begin() + p.cstart[c], L.h_items.begin() + p.cstart[c + 1]);
}

struct BLevel {
  std::vector<int> sys;    // systems eliminated at this level
  std::vector<int> stop;   // systems whose dense top starts at this level
  int Mtot = 0;
  DevBuf state;            // k, a, b [Mtot], err [8]
  LevelState ls{};
  DevBuf desc;             // merged items + colour starts
  ItemD* d_items = nullptr;
  const int32_t* d_cstart = nullptr;
  std::vector<int> cstart;
  int ncolours = 0, max_items = 0, max_m = 0, max_nseg = 0, max_acap = 0;
  std::vector<SplitDims> cdims;
  DevBuf zero;             // SpanD: buffers cleared before assembly
  int nzero = 0;
  int64_t max_zero = 0;
  DevBuf scat;             // level 0: ScatterD per system
  int nscat = 0;
  int64_t max_nnz = 0;
  DevBuf tasks;            // level >= 1: CopyD assembly tasks (levels and tops)
  int ntasks = 0;
  int64_t vbase = 0, nvec = 0;  // vector block
  DevBuf gidx;             // level >= 1: sources of the block in block l-1
  tune::Choice sched;
  std::vector<int> rec_k;  // ranks recorded by the first factorization
  std::vector<double> sweep_bytes;
  void free_all(hipStream_t st) {
    dfree(&state, st); dfree(&desc, st); dfree(&zero, st); dfree(&scat, st); dfree(&tasks, st);
    dfree(&gidx, st);
  }
};

}  // namespace

struct lrsp_batch {
  int nsys = 0;
  int64_t ntot = 0;
  double tol = 0.0;
  lrsp_opts o{};
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;       // private stream on which graphs are recorded
  std::vector<BSys> sys;
  std::vector<BLevel> lv;          // vector blocks 0..nb-1
  PanelArena arena;                // panel workspace: the systems of a level side by side
  int nlevels = 0;                 // blocks with eliminations
  DevBuf perm;                     // packed index -> block-0 index
  DevBuf offs;                     // [nsys+1] packed offsets
  DevBuf rowsys;                   // [ntot] system of each packed row
  DevBuf serr;                     // [nsys] error bits
  DevBuf tops;                     // TopD [nsys]
  DevBuf bars;                     // GridBar [2 * blocks]: graph-mode sweep barriers
  int max_top = 0;
  int64_t vec_total = 0;
  DevBuf vec;                      // vec_total * vec_cols
  int vec_cols = 0;
  // replay graph of the numeric phase
  hipGraph_t g_factor = nullptr;
  hipGraphExec_t ge_factor = nullptr;
  // merged matrix of the batched PCG
  DevBuf mrowptr, mcol, mval, mtasks;
  int nmtasks = 0;
  // PCG work
  DevBuf pcg;
  size_t pcg_doubles = 0;
  int pcg_nrhs = 0;
  hipGraphExec_t ge_pcg[2] = {nullptr, nullptr};
  hipGraph_t g_pcg[2] = {nullptr, nullptr};
  const double* pcg_key[3] = {nullptr, nullptr, nullptr};
  double pcg_rtol = -1.0;
  bool pcg_no_graph = false;
  lrsp_batch_info info{};
  void free_graphs() {
    if (ge_factor) (void)hipGraphExecDestroy(ge_factor);
    if (g_factor) (void)hipGraphDestroy(g_factor);
    ge_factor = nullptr;
    g_factor = nullptr;
    free_pcg_graphs();
  }
  void free_pcg_graphs() {
    for (int i = 0; i < 2; ++i) {
      if (ge_pcg[i]) (void)hipGraphExecDestroy(ge_pcg[i]);
      if (g_pcg[i]) (void)hipGraphDestroy(g_pcg[i]);
      ge_pcg[i] = nullptr;
      g_pcg[i] = nullptr;
    }
  }
  void free_device() {
    for (auto& s : sys) {
      for (auto& L : s.levels)
        if (L) L->free_all(stream);
      s.levels.clear();
      dfree(&s.top, stream);
      dfree(&s.off0, stream);
    }
    for (auto& B : lv) B.free_all(stream);
    lv.clear();
    dfree(&arena.buf, stream);
    dfree(&perm, stream); dfree(&offs, stream); dfree(&rowsys, stream); dfree(&serr, stream);
    dfree(&tops, stream); dfree(&bars, stream); dfree(&vec, stream); dfree(&mrowptr, stream); dfree(&mcol, stream);
    dfree(&mval, stream); dfree(&mtasks, stream); dfree(&pcg, stream);
    vec_cols = 0;
    pcg_doubles = 0;
  }
  ~lrsp_batch() {
    free_graphs();
    free_device();
    (void)hipStreamSynchronize(stream);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

lrsp_status upload_vec(DevBuf* b, const void* src, size_t bytes, hipStream_t st) {
  dfree(b, st);
  return upload(b, src, bytes, st);
}

// Tops of more than kSplitMaxDofs unknowns: the blocked Cholesky, system by
// system (their error bit as the batched kernels report it).
void top_potrf_large(lrsp_batch* F, hipStream_t st) {
  for (int i = 0; i < F->nsys; ++i) {
    BSys& S = F->sys[i];
    if (S.top_n > kSplitMaxDofs)
      launch_top_potrf_blocked(at<double>(S.top, 0), S.top_n, at<int32_t>(F->serr, i), 1, st);
  }
}

// Clears and assembles the input of block B (levels and tops starting at B).
void assemble(const BLevel& B, hipStream_t st) {
  if (B.Mtot > 0) launch_zero_i32(B.ls.k, 4 * (int64_t)B.Mtot + 8, st);
  launch_zero_multi(at<SpanD>(B.zero, 0), B.nzero, B.max_zero, st);
  if (B.nscat > 0) launch_scatter_vals_multi(at<ScatterD>(B.scat, 0), B.nscat, B.max_nnz, st);
  if (B.ntasks > 0) launch_copy_blocks(at<CopyD>(B.tasks, 0), B.ntasks, st);
}

// Barrier words of the level's persistent launch in graph mode (behind the
// error words of its state; cleared with the state by assemble()).
GridBar* level_bar(const BLevel& B) { return reinterpret_cast<GridBar*>(B.ls.err + 4); }

// Eliminates every cluster of block B with the chosen schedule.  graph:
// the launches are being recorded, so the persistent schedule uses the
// software grid barrier instead of a cooperative launch.
lrsp_status eliminate(const BLevel& B, int level, double tol, const lrsp_opts& o,
                      const tune::Choice& c, bool graph, hipStream_t st) {
  if (B.Mtot == 0) return LRSP_OK;
  TimedLaunch tall(0, st);
  if (c.sched == tune::kSchedPersistent) {
    TimedLaunch tf(10, st);
    if (launch_slre_level(B.d_items, B.d_cstart, B.ncolours, B.max_items, B.max_m, B.max_nseg, B.ls,
                          level, tol, o.tol_mode, o.gemm_prec, st, c.grid_cap,
                          graph ? level_bar(B) : nullptr) == hipSuccess)
      return LRSP_OK;
    if (graph) return fail(LRSP_ERR_HIP, "persistent level launch failed");
    (void)hipGetLastError();
  }
  if (c.sched == tune::kSchedSplit && B.max_m >= kSplitMinDofs && B.max_m <= kSplitMaxDofs) {
    for (int col = 0; col < B.ncolours; ++col)
      for (int step = 0; step < kSplitSteps; ++step)
        launch_split_step(step, B.d_items + B.cstart[col], B.cstart[col + 1] - B.cstart[col],
                          B.cdims[col], B.ls, level, tol, o.tol_mode, o.gemm_prec, st, c.tile);
  } else {
    TimedLaunch tf(10, st);
    for (int col = 0; col < B.ncolours; ++col)
      launch_slre(B.d_items + B.cstart[col], B.cstart[col + 1] - B.cstart[col], B.max_m, B.max_nseg,
                  B.ls, level, tol, o.tol_mode, o.gemm_prec, st);
  }
  HIPCHK(hipGetLastError());
  return LRSP_OK;
}

// Times the candidate schedules of block B (re-assembling its input before
// every run) and returns the fastest.
lrsp_status autotune_level(const BLevel& B, int level, double tol, const lrsp_opts& o, hipStream_t st,
                           tune::Choice* best) {
  std::vector<tune::Choice> cand;
  cand.push_back({tune::kSchedPersistent, 0, 0.0});
  const int occ = slre_level_occupancy(B.max_m, B.max_nseg);
  if (occ > 1) cand.push_back({tune::kSchedPersistent, device_cus(), 0.0});
  cand.push_back({tune::kSchedPerColour, 0, 0.0});
  if (B.max_m >= kSplitMinDofs && B.max_m <= kSplitMaxDofs) {
    cand.push_back({tune::kSchedSplit, 0, 0.0, kTileWide});
    if (B.max_m <= 256) cand.push_back({tune::kSchedSplit, 0, 0.0, kTileNarrow});
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const bool was_on = g_tm.on;
  g_tm.on = false;
  double best_ms = 1e300;
  for (auto& c : cand) {
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {  // the first run warms caches and code
      assemble(B, st);
      HIPCHK(hipEventRecord(e0, st));
      if (lrsp_status s = eliminate(B, level, tol, o, c, false, st)) {
        g_tm.on = was_on;
        return s;
      }
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    }
    c.ms = ms;
    if (ms < best_ms) {
      best_ms = ms;
      *best = c;
    }
  }
  g_tm.on = was_on;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return LRSP_OK;
}

lrsp_status check_opts(const lrsp_opts& o) {
  if (o.gemm_prec < 0 || o.gemm_prec > 2 || o.tol_mode < 0 || o.tol_mode > 1 || o.exec_mode < 0 ||
      o.exec_mode > 3 || o.autotune < 0 || o.autotune > 1 || o.scheme != 0 || o.top_dense_threshold < 0 ||
      o.top_dense_threshold > kMaxClusterDofs)
    return fail(LRSP_ERR_ARG, "invalid option");
  if (o.rank_mode != 0) return fail(LRSP_ERR_ARG, "batched factorizations use rank_mode 0");
  return LRSP_OK;
}

// Planning, setup and the first numeric factorization of a batch.
lrsp_status batch_factor(lrsp_batch* F, const lrsp_csr* A, const TreeH* const* T, int32_t* status) {
  const hipStream_t st = F->stream;
  const int nsys = F->nsys;
  const auto t0 = std::chrono::steady_clock::now();
  double ms_an = 0.0;
  auto ms_since = [](std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
  };
  F->sys.clear();
  F->sys.resize(nsys);
  int64_t off = 0;
  for (int i = 0; i < nsys; ++i) {
    BSys& S = F->sys[i];
    S.tr = T[i];
    if (A[i].n != S.tr->n) return fail(LRSP_ERR_ARG, "matrix size does not match the tree of system " + std::to_string(i));
    if (!A[i].rowptr || !A[i].col || !A[i].val) return fail(LRSP_ERR_ARG, "null CSR array");
    S.n = A[i].n;
    S.nnz = A[i].nnz;
    S.off = off;
    off += S.n;
    // the batch keeps its own copy of the pattern (replanning, merged matrix)
    S.hrp.resize(S.n + 1);
    S.hcol.resize(S.nnz);
    if (A[i].h_rowptr && A[i].h_col) {
      std::memcpy(S.hrp.data(), A[i].h_rowptr, 8 * (S.n + 1));
      std::memcpy(S.hcol.data(), A[i].h_col, 4 * S.nnz);
    } else {
      HIPCHK(hipMemcpyAsync(S.hrp.data(), A[i].rowptr, 8 * (S.n + 1), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(S.hcol.data(), A[i].col, 4 * S.nnz, hipMemcpyDeviceToHost, st));
    }
    S.rp = S.hrp.data();
    S.cl = S.hcol.data();
  }
  HIPCHK(hipStreamSynchronize(st));
  F->ntot = off;
  for (int i = 0; i < nsys; ++i)
    if (F->sys[i].rp[F->sys[i].n] != F->sys[i].nnz) return fail(LRSP_ERR_ARG, "rowptr[n] != nnz");
  // level-0 analysis of every system
  auto ta = std::chrono::steady_clock::now();
  std::vector<int> bad(nsys, 0);
  parallel_for(nsys, [&](int i) {
    BSys& S = F->sys[i];
    const TreeH& tr = *S.tr;
    S.sizes.resize(tr.leaf_ptr.size() - 1);
    for (size_t c = 0; c + 1 < tr.leaf_ptr.size(); ++c) S.sizes[c] = (int)(tr.leaf_ptr[c + 1] - tr.leaf_ptr[c]);
    for (int64_t e = 0; e < S.nnz; ++e)
      if (S.cl[e] < 0 || S.cl[e] >= tr.n) {
        bad[i] = 1;
        return;
      }
    level0_graph(tr, S.rp, S.cl, &S.adj);
    for (int64_t r = 0; r < tr.n; ++r) {
      const int p = tr.dof_cluster[r];
      for (int64_t e = S.rp[r]; e < S.rp[r + 1]; ++e) {
        const int q = tr.dof_cluster[S.cl[e]];
        if (q == p) continue;
        std::vector<uint64_t>& b = S.z0[pkey(p, q)];
        if (b.empty()) b.assign((S.sizes[q] + 63) / 64, 0);
        const int lj = tr.dof_local[S.cl[e]];
        b[lj >> 6] |= 1ull << (lj & 63);
      }
    }
  });
  for (int i = 0; i < nsys; ++i)
    if (bad[i]) return fail(LRSP_ERR_ARG, "column index out of range in system " + std::to_string(i));
  ms_an += ms_since(ta);
  HIPCHK(dalloc(&F->serr, 4 * (size_t)nsys, st));
  launch_zero_i32(at<int32_t>(F->serr, 0), nsys, st);
  {
    std::vector<int64_t> po(nsys + 1);
    std::vector<int64_t> perm(F->ntot);
    std::vector<int32_t> rs(F->ntot);
    for (int i = 0; i < nsys; ++i) {
      const BSys& S = F->sys[i];
      po[i] = S.off;
      for (int64_t j = 0; j < S.n; ++j) {
        perm[S.off + j] = S.off + S.tr->perm[j];
        rs[S.off + j] = i;
      }
    }
    po[nsys] = F->ntot;
    if (lrsp_status s = upload(&F->offs, po.data(), po.size() * 8, st)) return s;
    if (lrsp_status s = upload(&F->perm, perm.data(), perm.size() * 8, st)) return s;
    if (lrsp_status s = upload(&F->rowsys, rs.data(), rs.size() * 4, st)) return s;
  }
  double flops[6] = {0, 0, 0, 0, 0, 0};
  int64_t cursor = F->ntot;
  int tuned = 0;
  std::vector<int32_t> herr(8);
  for (int l = 0;; ++l) {
    BLevel B;
    for (int i = 0; i < nsys; ++i) {
      BSys& S = F->sys[i];
      if (S.stopped) continue;
      int64_t tot = 0;
      for (int x : S.sizes) tot += x;
      if (S.sizes.size() == 1 || complete_graph(S.adj) ||
          (F->o.top_dense_threshold > 0 && tot <= F->o.top_dense_threshold))
        B.stop.push_back(i);
      else B.sys.push_back(i);
    }
    if (B.sys.empty() && B.stop.empty()) break;
    ta = std::chrono::steady_clock::now();
    // vector block
    std::vector<int64_t> vb(nsys, -1);
    {
      int64_t run = 0;
      std::vector<char> in(nsys, 0);
      for (int i : B.sys) in[i] = 1;
      for (int i : B.stop) in[i] = 1;
      for (int i = 0; i < nsys; ++i) {
        if (!in[i]) continue;
        const BSys& S = F->sys[i];
        int64_t len = 0;
        for (int m : S.sizes) len += m;
        vb[i] = l == 0 ? S.off : cursor + run;
        run += len;
      }
      B.vbase = l == 0 ? 0 : cursor;
      B.nvec = run;
      if (l > 0) cursor += run;
    }
    // plan the eliminated systems in parallel, then set them up
    std::vector<std::unique_ptr<LevelDev>> Ls(B.sys.size());
    for (size_t j = 0; j < B.sys.size(); ++j) {
      BSys& S = F->sys[B.sys[j]];
      Ls[j] = std::make_unique<LevelDev>();
      Ls[j]->plan.M = (int)S.sizes.size();
      Ls[j]->plan.m = S.sizes;
      Ls[j]->plan.adj = S.adj;
    }
    parallel_for((int)B.sys.size(), [&](int j) {
      BSys& S = F->sys[B.sys[j]];
      plan_level(&Ls[j]->plan, l == 0 ? &S.z0 : nullptr);
    });
    std::vector<int> sbase(B.sys.size());
    for (size_t j = 0; j < B.sys.size(); ++j) {
      sbase[j] = B.Mtot;
      B.Mtot += Ls[j]->plan.M;
    }
    if (B.Mtot > 0) {
      HIPCHK(dalloc(&B.state, 4 * (4 * (size_t)B.Mtot + 8), st));
      int32_t* sb = at<int32_t>(B.state, 0);
      B.ls = LevelState{sb, sb + B.Mtot, sb + 2 * B.Mtot, sb + 3 * B.Mtot, sb + 3 * B.Mtot + 8};
      launch_zero_i32(sb, 4 * (int64_t)B.Mtot + 8, st);
    }
    {  // the systems' panels side by side in the shared arena
      int64_t off = 0;
      for (auto& L : Ls) {
        L->arena_off = off;
        off += panel_doubles(*L);
      }
      if (lrsp_status s = arena_reserve(&F->arena, off, st)) return s;
    }
    for (size_t j = 0; j < B.sys.size(); ++j) {
      const int i = B.sys[j];
      if (lrsp_status s = setup_level(Ls[j].get(), st, vb[i], sbase[j], &B.ls, at<int32_t>(F->serr, i),
                                      &F->arena))
        return s;
    }
    // assembly of the block's input
    std::vector<SpanD> zeros;
    std::vector<ScatterD> scats;
    std::vector<CopyD> tasks;
    std::vector<int64_t> gidx;
    for (size_t j = 0; j < B.sys.size(); ++j) {
      LevelDev& L = *Ls[j];
      zeros.push_back(SpanD{at<double>(L.work, 0), L.plan.work_doubles});
      zeros.push_back(SpanD{at<double>(L.coarse, 0), L.plan.coarse_doubles});
    }
    for (int i : B.stop) {
      BSys& S = F->sys[i];
      const int M = (int)S.sizes.size();
      std::vector<int64_t> toff(M + 1, 0);
      for (int x = 0; x < M; ++x) toff[x + 1] = toff[x] + S.sizes[x];
      S.top_n = (int)toff[M];
      if (S.top_n > kMaxClusterDofs)
        return fail(LRSP_ERR_ARG, "dense top of system " + std::to_string(i) + " larger than " +
                                      std::to_string(kMaxClusterDofs));
      S.top_level = l;
      S.top_vbase = vb[i];
      S.top_sizes = S.sizes;
      S.top_adj_ptr.assign(1, 0);
      S.top_adj.clear();
      for (int x = 0; x < M; ++x) {
        S.top_adj.insert(S.top_adj.end(), S.adj[x].begin(), S.adj[x].end());
        S.top_adj_ptr.push_back((int)S.top_adj.size());
      }
      HIPCHK(dalloc(&S.top, sizeof(double) * std::max<int64_t>(1, (int64_t)S.top_n * (S.top_n + 64)), st));
      zeros.push_back(SpanD{at<double>(S.top, 0), (int64_t)S.top_n * S.top_n});
      F->max_top = std::max(F->max_top, S.top_n);
      if (l == 0) {
        std::vector<int64_t> o0;
        top_offsets_level0(*S.tr, S.rp, S.cl, S.nnz, toff, S.top_n, &o0);
        if (lrsp_status s = upload_vec(&S.off0, o0.data(), o0.size() * 8, st)) return s;
        scats.push_back(ScatterD{A[i].val, at<int64_t>(S.off0, 0), at<double>(S.top, 0), S.nnz});
      } else {
        top_tasks(*S.levels.back(), toff, S.top_n, at<double>(S.top, 0), &tasks);
      }
    }
    for (size_t j = 0; j < B.sys.size(); ++j) {
      const int i = B.sys[j];
      BSys& S = F->sys[i];
      LevelDev& L = *Ls[j];
      if (l == 0) {
        std::vector<int64_t> o0;
        if (lrsp_status s = level0_offsets(*S.tr, S.rp, S.cl, S.nnz, L.plan, &o0)) return s;
        if (lrsp_status s = upload_vec(&S.off0, o0.data(), o0.size() * 8, st)) return s;
        scats.push_back(ScatterD{A[i].val, at<int64_t>(S.off0, 0), at<double>(L.work, 0), S.nnz});
      } else if (!assembly_tasks(*S.levels.back(), L, &tasks)) {
        return fail(LRSP_ERR_INTERNAL, "coarse fine-half block is not dense");
      }
    }
    if (l > 0) {
      // gather list in the block's system order
      std::vector<char> in(nsys, 0);
      for (int i : B.sys) in[i] = 1;
      for (int i : B.stop) in[i] = 1;
      std::vector<int64_t> g;
      for (int i = 0; i < nsys; ++i) {
        if (!in[i]) continue;
        const BSys& S = F->sys[i];
        coarse_gather_indices(*S.levels.back(), (int)S.sizes.size(), &g);
        gidx.insert(gidx.end(), g.begin(), g.end());
      }
      if ((int64_t)gidx.size() != B.nvec) return fail(LRSP_ERR_INTERNAL, "vector block size mismatch");
      if (lrsp_status s = upload(&B.gidx, gidx.data(), gidx.size() * 8, st)) return s;
    }
    B.nzero = (int)zeros.size();
    for (auto& z : zeros) B.max_zero = std::max(B.max_zero, z.n);
    if (!zeros.empty())
      if (lrsp_status s = upload(&B.zero, zeros.data(), zeros.size() * sizeof(SpanD), st)) return s;
    B.nscat = (int)scats.size();
    for (auto& sc : scats) B.max_nnz = std::max(B.max_nnz, sc.nnz);
    if (!scats.empty())
      if (lrsp_status s = upload(&B.scat, scats.data(), scats.size() * sizeof(ScatterD), st)) return s;
    B.ntasks = (int)tasks.size();
    if (!tasks.empty())
      if (lrsp_status s = upload(&B.tasks, tasks.data(), tasks.size() * sizeof(CopyD), st)) return s;
    // merged work list, by colour
    if (B.Mtot > 0) {
      std::vector<ItemD> items;
      B.cstart.assign(1, 0);
      for (auto& L : Ls) B.ncolours = std::max(B.ncolours, L->plan.ncolours);
      B.cdims.assign(B.ncolours, SplitDims{0, 0, 0, 0, 0});
      for (int c = 0; c < B.ncolours; ++c) {
        for (auto& L : Ls) {
          const LevelPlan& p = L->plan;
          if (c >= p.ncolours) continue;
          append_colour(*L, c, &items);
          SplitDims& d = B.cdims[c];
          const SplitDims& e = L->cdims[c];
          d.max_m = std::max(d.max_m, e.max_m);
          d.max_nseg = std::max(d.max_nseg, e.max_nseg);
          d.max_pcap = std::max(d.max_pcap, e.max_pcap);
          d.max_acap = std::max(d.max_acap, e.max_acap);
          d.max_bcap = std::max(d.max_bcap, e.max_bcap);
        }
        B.cstart.push_back((int)items.size());
        B.max_items = std::max(B.max_items, B.cstart[c + 1] - B.cstart[c]);
        B.max_acap = std::max(B.max_acap, B.cdims[c].max_acap);
      }
      for (auto& L : Ls) {
        B.max_m = std::max(B.max_m, L->max_m);
        B.max_nseg = std::max(B.max_nseg, L->max_nseg);
      }
      const size_t bi = sizeof(ItemD) * items.size(), o4 = (bi + 255) & ~(size_t)255;
      std::vector<char> blob(o4 + 4 * B.cstart.size(), 0);
      std::memcpy(blob.data(), items.data(), bi);
      std::memcpy(blob.data() + o4, B.cstart.data(), 4 * B.cstart.size());
      if (lrsp_status s = upload(&B.desc, blob.data(), blob.size(), st)) return s;
      B.d_items = at<ItemD>(B.desc, 0);
      B.d_cstart = reinterpret_cast<const int32_t*>(reinterpret_cast<char*>(B.desc.p) + o4);
    }
    ms_an += ms_since(ta);
    // assemble and eliminate
    if (B.Mtot > 0) {
      const std::string key = tune::key(true, B.max_m, (int)B.cstart.back(), B.ncolours);
      if (F->o.exec_mode == 1) B.sched = tune::Choice{tune::kSchedPerColour, 0, 0.0};
      else if (F->o.exec_mode == 2) B.sched = tune::Choice{tune::kSchedPersistent, 0, 0.0};
      else if (F->o.exec_mode == 3) B.sched = tune::Choice{tune::kSchedSplit, 0, 0.0};
      else if (F->o.autotune) {
        if (lrsp_status s = autotune_level(B, l, F->tol, F->o, st, &B.sched)) return s;
        tune::store(key, B.sched);
        ++tuned;
      } else if (!tune::lookup(key, &B.sched)) {
        B.sched = tune::Choice{tune::kSchedPersistent, 0, 0.0};
      }
    }
    assemble(B, st);
    if (lrsp_status s = eliminate(B, l, F->tol, F->o, B.sched, false, st)) return s;
    // read back the ranks
    if (B.Mtot > 0) {
      std::vector<int32_t> kab(3 * (size_t)B.Mtot);
      HIPCHK(hipMemcpyAsync(kab.data(), B.ls.k, 4 * kab.size(), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(herr.data(), B.ls.err, 16, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (herr[0] && herr[3] != kErrNotSPD)
        return fail(LRSP_ERR_INTERNAL, "device check failed (code " + std::to_string(herr[3]) +
                                           ") at level " + std::to_string(herr[1]));
      B.rec_k.assign(kab.begin(), kab.begin() + B.Mtot);
      B.sweep_bytes.clear();
      for (size_t j = 0; j < B.sys.size(); ++j) {
        LevelDev& L = *Ls[j];
        const int M = L.plan.M;
        L.k.assign(kab.begin() + sbase[j], kab.begin() + sbase[j] + M);
        L.a.assign(kab.begin() + B.Mtot + sbase[j], kab.begin() + B.Mtot + sbase[j] + M);
        L.b.assign(kab.begin() + 2 * B.Mtot + sbase[j], kab.begin() + 2 * B.Mtot + sbase[j] + M);
        bool changed = false;
        if (lrsp_status s = plan_stores(&L, st, &changed)) return s;
        double f[5];
        level_stats(&L, f);
        for (int q = 0; q < 5; ++q) flops[q] += f[q];
        if (B.sweep_bytes.size() < L.sweep_bytes.size()) B.sweep_bytes.resize(L.sweep_bytes.size(), 0.0);
        for (size_t c = 0; c < L.sweep_bytes.size(); ++c) B.sweep_bytes[c] += L.sweep_bytes[c];
      }
      // the merged work list again, now pointing at the factor stores, and
      // what the sweeps read copied into them
      std::vector<ItemD> items;
      for (int c = 0; c < B.ncolours; ++c)
        for (auto& L : Ls)
          if (c < L->plan.ncolours) append_colour(*L, c, &items);
      HIPCHK(hipMemcpyAsync(B.d_items, items.data(), sizeof(ItemD) * items.size(), hipMemcpyHostToDevice, st));
      launch_compact(B.d_items, (int)items.size(), B.ls, st);
      HIPCHK(hipStreamSynchronize(st));
    }
    // next level of every eliminated system; the stopped ones are done
    for (size_t j = 0; j < B.sys.size(); ++j) {
      BSys& S = F->sys[B.sys[j]];
      LevelDev& L = *Ls[j];
      const int M = L.plan.M;
      std::vector<int> nsz(M / 2);
      for (int P = 0; P < M / 2; ++P) nsz[P] = L.k[2 * P] + L.k[2 * P + 1];
      std::vector<std::vector<int>> nadj;
      coarsen_square(S.adj, &nadj);
      S.sizes.swap(nsz);
      S.adj.swap(nadj);
      S.levels.push_back(std::move(Ls[j]));
    }
    for (int i : B.stop) F->sys[i].stopped = true;
    if (B.Mtot > 0) F->nlevels = l + 1;
    F->lv.push_back(std::move(B));
  }
  // levels set up before the arena last grew: their items to the new buffer
  for (size_t l = 0; l < F->lv.size(); ++l) {
    BLevel& B = F->lv[l];
    if (B.Mtot == 0) continue;
    std::vector<LevelDev*> Ls;
    bool stale = false;
    for (int i : B.sys) {
      LevelDev* L = F->sys[i].levels[l].get();
      Ls.push_back(L);
      stale = stale || L->arena_gen != F->arena.gen;
    }
    if (!stale) continue;
    for (LevelDev* L : Ls)
      if (lrsp_status s = rebind_panels(L, st, &F->arena)) return s;
    std::vector<ItemD> items;
    for (int c = 0; c < B.ncolours; ++c)
      for (LevelDev* L : Ls)
        if (c < L->plan.ncolours) append_colour(*L, c, &items);
    HIPCHK(hipMemcpyAsync(B.d_items, items.data(), sizeof(ItemD) * items.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  // dense tops
  std::vector<TopD> tops(nsys);
  for (int i = 0; i < nsys; ++i) {
    BSys& S = F->sys[i];
    tops[i] = TopD{at<double>(S.top, 0), S.top_vbase, at<int32_t>(F->serr, i), S.top_n, 0};
    flops[5] += (double)S.top_n * S.top_n * S.top_n / 3.0;
  }
  if (lrsp_status s = upload(&F->tops, tops.data(), tops.size() * sizeof(TopD), st)) return s;
  launch_top_potrf_batched(at<TopD>(F->tops, 0), nsys, F->max_top, st);
  top_potrf_large(F, st);
  HIPCHK(hipGetLastError());
  std::vector<int32_t> se(nsys);
  HIPCHK(hipMemcpyAsync(se.data(), F->serr.p, 4 * (size_t)nsys, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  F->vec_total = cursor;
  HIPCHK(dalloc(&F->bars, sizeof(GridBar) * 2 * std::max<size_t>(1, F->lv.size()), st));
  launch_zero_i32(at<int32_t>(F->bars, 0), 8 * (int64_t)std::max<size_t>(1, F->lv.size()), st);
  // info
  lrsp_batch_info& inf = F->info;
  inf = lrsp_batch_info{};
  inf.nsys = nsys;
  inf.nlevels = F->nlevels;
  inf.ntot = F->ntot;
  for (int q = 0; q < 6; ++q) inf.flops[q] = flops[q];
  inf.ms_factor = ms_since(t0);
  inf.ms_analysis = ms_an;
  inf.tuned_levels = tuned;
  for (size_t l = 0; l < F->lv.size() && l < 16; ++l) {
    inf.sched[l] = F->lv[l].sched.sched;
    inf.grid_cap[l] = F->lv[l].sched.grid_cap;
    inf.tile[l] = F->lv[l].sched.tile;
  }
  int64_t held = 0;
  for (auto& S : F->sys) {
    for (auto& L : S.levels) held += L->held_bytes();
    held += (int64_t)(S.top.bytes + S.off0.bytes);
  }
  for (auto& B : F->lv)
    held += (int64_t)(B.state.bytes + B.desc.bytes + B.zero.bytes + B.scat.bytes + B.tasks.bytes + B.gidx.bytes);
  inf.peak_bytes = held + (int64_t)F->arena.buf.bytes;
  lrsp_status rs = LRSP_OK;
  for (int i = 0; i < nsys; ++i) {
    const bool notspd = (se[i] & (1 << kErrNotSPD)) != 0;
    if (se[i] & ~(1 << kErrNotSPD))
      return fail(LRSP_ERR_INTERNAL, "device check failed in system " + std::to_string(i));
    if (status) status[i] = notspd ? LRSP_ERR_NOT_SPD : LRSP_OK;
    if (notspd && rs == LRSP_OK) rs = fail(LRSP_ERR_NOT_SPD, "non-positive pivot in system " + std::to_string(i));
  }
  return rs;
}

// The numeric phase of a planned batch: clears, assembly, eliminations,
// tops.  No host synchronisation; with graph = true it can be recorded.
lrsp_status numeric_phase(lrsp_batch* F, bool graph, hipStream_t st) {
  launch_zero_i32(at<int32_t>(F->serr, 0), F->nsys, st);
  for (size_t l = 0; l < F->lv.size(); ++l) {
    const BLevel& B = F->lv[l];
    assemble(B, st);
    if (lrsp_status s = eliminate(B, (int)l, F->tol, F->o, B.sched, graph, st)) return s;
    if (B.Mtot > 0) launch_compact(B.d_items, B.cstart.back(), B.ls, st);
  }
  launch_top_potrf_batched(at<TopD>(F->tops, 0), F->nsys, F->max_top, st);
  top_potrf_large(F, st);
  HIPCHK(hipGetLastError());
  return LRSP_OK;
}

// Records fn(stream) into an executable graph on the batch's private stream
// (the caller's stream may be the null stream, which cannot record); the
// graph is then launched on the caller's stream.  Returns false (after
// clearing the error state) if recording or instantiation fails.
template <class Fn>
bool capture(lrsp_batch* F, hipGraph_t* g, hipGraphExec_t* ge, Fn fn) {
  *g = nullptr;
  *ge = nullptr;
  if (!F->cap && hipStreamCreateWithFlags(&F->cap, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    F->cap = nullptr;
    return false;
  }
  hipStream_t st = F->cap;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  const lrsp_status s = fn(st);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &graph);
  (void)hipGetLastError();
  if (s != LRSP_OK || e != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return false;
  }
  if (hipGraphInstantiate(ge, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(graph);
    *ge = nullptr;
    return false;
  }
  *g = graph;
  return true;
}

// Barrier words of the sweeps of level l in graph mode.
GridBar* sweep_bar(const lrsp_batch* F, size_t l, bool forward) {
  return at<GridBar>(F->bars, 2 * (int64_t)l + (forward ? 0 : 1));
}

// One application of the preconditioner to nrhs packed columns.  graph: the
// launches are being recorded (persistent sweeps use the software barrier).
lrsp_status apply_cols(lrsp_batch* F, const double* b, double* x, int nrhs, bool graph,
                       hipStream_t st) {
  for (int r = 0; r < nrhs; ++r) {
    double* V = at<double>(F->vec, (int64_t)r * F->vec_total);
    launch_gather(b + (size_t)r * F->ntot, at<int64_t>(F->perm, 0), V, F->ntot, st);
    for (size_t l = 0; l < F->lv.size(); ++l) {
      const BLevel& B = F->lv[l];
      if (l > 0) launch_gather(V, at<int64_t>(B.gidx, 0), V + B.vbase, B.nvec, st);
      if (B.Mtot == 0) continue;
      TimedLaunch tl(1, st);
      // levels with split clusters run one launch per colour (plus its units)
      const bool per_colour = sweep_units(true, B.max_m, B.max_acap) > 0;
      if (per_colour ||
          launch_sweep_level(true, B.d_items, B.d_cstart, B.ncolours, B.cstart.back(), B.max_items, B.max_m, B.max_acap, B.ls, V, st, 0,
                             graph ? sweep_bar(F, l, true) : nullptr, 0, F->vec_total) != hipSuccess) {
        if (!per_colour) {
          if (graph) return fail(LRSP_ERR_HIP, "persistent sweep launch failed");
          (void)hipGetLastError();
        }
        for (int c = 0; c < B.ncolours; ++c)
          launch_fwd(B.d_items + B.cstart[c], B.cstart[c + 1] - B.cstart[c], B.max_m, B.max_acap, B.ls, V, st);
      }
      if (g_tm.on)
        for (double by : B.sweep_bytes) g_tm.bytes[1] += by;
    }
    launch_top_solve_batched(at<TopD>(F->tops, 0), F->nsys, F->max_top, V, st);
    for (int l = (int)F->lv.size() - 1; l >= 0; --l) {
      const BLevel& B = F->lv[l];
      if (B.Mtot > 0) {
        TimedLaunch tl(2, st);
        const bool per_colour = sweep_units(false, B.max_m, B.max_acap) > 0;
        if (per_colour ||
            launch_sweep_level(false, B.d_items, B.d_cstart, B.ncolours, B.cstart.back(), B.max_items, B.max_m, B.max_acap, B.ls, V,
                               st, 0, graph ? sweep_bar(F, l, false) : nullptr, 0, F->vec_total) != hipSuccess) {
          if (!per_colour) {
            if (graph) return fail(LRSP_ERR_HIP, "persistent sweep launch failed");
            (void)hipGetLastError();
          }
          for (int c = B.ncolours - 1; c >= 0; --c)
            launch_bwd(B.d_items + B.cstart[c], B.cstart[c + 1] - B.cstart[c], B.max_m, B.max_acap, B.ls, V, st);
        }
        if (g_tm.on)
          for (double by : B.sweep_bytes) g_tm.bytes[2] += by;
      }
      if (l > 0) launch_scatter(V + B.vbase, at<int64_t>(B.gidx, 0), V, B.nvec, st);
    }
    launch_scatter(V, at<int64_t>(F->perm, 0), x + (size_t)r * F->ntot, F->ntot, st);
  }
  HIPCHK(hipGetLastError());
  return LRSP_OK;
}

lrsp_status ensure_vec(lrsp_batch* F, int nrhs, hipStream_t st) {
  if (F->vec_cols >= nrhs) return LRSP_OK;
  F->free_pcg_graphs();
  dfree(&F->vec, st);
  HIPCHK(dalloc(&F->vec, sizeof(double) * std::max<int64_t>(1, F->vec_total * nrhs), st));
  launch_zero(at<double>(F->vec, 0), F->vec_total * nrhs, st);
  F->vec_cols = nrhs;
  return LRSP_OK;
}

lrsp_status check_status(lrsp_batch* F, int32_t* status, hipStream_t st) {
  std::vector<int32_t> se(F->nsys);
  HIPCHK(hipMemcpyAsync(se.data(), F->serr.p, 4 * se.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  lrsp_status rs = LRSP_OK;
  for (int i = 0; i < F->nsys; ++i) {
    if (se[i] & ~(1 << kErrNotSPD))
      return fail(LRSP_ERR_INTERNAL, "device check failed in system " + std::to_string(i));
    const bool notspd = (se[i] & (1 << kErrNotSPD)) != 0;
    if (status) status[i] = notspd ? LRSP_ERR_NOT_SPD : LRSP_OK;
    if (notspd && rs == LRSP_OK) rs = fail(LRSP_ERR_NOT_SPD, "non-positive pivot in system " + std::to_string(i));
  }
  return rs;
}

}  // namespace

extern "C" {

lrsp_status lrsp_factor_batched(int32_t nsys, const lrsp_csr* A, lrsp_tree* const* T, double tol,
                                const lrsp_opts* opts, void* stream, lrsp_batch** out,
                                int32_t* status) {
  if (!out || nsys < 1 || !A || !T) return fail(LRSP_ERR_ARG, "invalid argument");
  *out = nullptr;
  if (!(tol >= 0.0)) return fail(LRSP_ERR_ARG, "tol must be >= 0");
  for (int i = 0; i < nsys; ++i)
    if (!T[i]) return fail(LRSP_ERR_ARG, "null tree");
  try {
    auto F = std::make_unique<lrsp_batch>();
    F->nsys = nsys;
    F->tol = tol;
    if (opts) F->o = *opts;
    if (lrsp_status s = check_opts(F->o)) return s;
    F->stream = reinterpret_cast<hipStream_t>(stream);
    std::vector<const TreeH*> trees(nsys);
    for (int i = 0; i < nsys; ++i) trees[i] = &tree_of(T[i]);
    lrsp_status s = batch_factor(F.get(), A, trees.data(), status);
    if (s != LRSP_OK && s != LRSP_ERR_NOT_SPD) return s;
    *out = F.release();
    return s;
  } catch (const std::bad_alloc&) {
    return fail(LRSP_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(LRSP_ERR_INTERNAL, std::string("planner: ") + e.what());
  }
}

lrsp_status lrsp_refactor_batched(lrsp_batch* F, const lrsp_csr* A, void* stream, int32_t* status) {
  if (!F || !A) return fail(LRSP_ERR_ARG, "invalid argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  F->stream = st;
  const auto t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < F->nsys; ++i)
    if (A[i].n != F->sys[i].n || A[i].nnz != F->sys[i].nnz || !A[i].val)
      return fail(LRSP_ERR_ARG, "matrix " + std::to_string(i) + " does not match the batch");
  // new value pointers into the level-0 scatter descriptors
  if (!F->lv.empty() && F->lv[0].nscat > 0) {
    std::vector<ScatterD> sc(F->lv[0].nscat);
    int j = 0;
    for (int i : F->lv[0].stop) sc[j++] = ScatterD{A[i].val, at<int64_t>(F->sys[i].off0, 0), at<double>(F->sys[i].top, 0), F->sys[i].nnz};
    for (size_t q = 0; q < F->lv[0].sys.size(); ++q) {
      const int i = F->lv[0].sys[q];
      sc[j++] = ScatterD{A[i].val, at<int64_t>(F->sys[i].off0, 0), at<double>(F->sys[i].levels[0]->work, 0),
                         F->sys[i].nnz};
    }
    HIPCHK(hipMemcpyAsync(F->lv[0].scat.p, sc.data(), sc.size() * sizeof(ScatterD), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  const bool was_on = g_tm.on;
  if (!F->ge_factor) {
    g_tm.on = false;  // no timing events inside the recorded graph
    (void)capture(F, &F->g_factor, &F->ge_factor, [&](hipStream_t s) { return numeric_phase(F, true, s); });
    g_tm.on = was_on;
  }
  bool graph = F->ge_factor != nullptr;
  if (graph) {
    HIPCHK(hipGraphLaunch(F->ge_factor, st));
  } else if (lrsp_status s = numeric_phase(F, false, st)) {
    return s;
  }
  // ranks (and barrier time-outs) of every level against the recorded ones
  auto read_levels = [&](std::vector<std::vector<int32_t>>* ks, std::vector<std::array<int32_t, 8>>* es) -> lrsp_status {
    ks->assign(F->lv.size(), {});
    es->assign(F->lv.size(), {});
    for (size_t l = 0; l < F->lv.size(); ++l) {
      const BLevel& B = F->lv[l];
      if (B.Mtot == 0) continue;
      (*ks)[l].resize(B.Mtot);
      HIPCHK(hipMemcpyAsync((*ks)[l].data(), B.ls.k, 4 * (size_t)B.Mtot, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync((*es)[l].data(), B.ls.err, 32, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    return LRSP_OK;
  };
  std::vector<std::vector<int32_t>> ks;
  std::vector<std::array<int32_t, 8>> es;
  if (lrsp_status s = read_levels(&ks, &es)) return s;
  bool timed_out = false;
  for (auto& e : es) timed_out = timed_out || e[6] != 0;
  if (graph && timed_out) {
    // a software barrier gave up: discard the graph, redo the phase eagerly
    F->free_graphs();
    F->info.graph_timeouts += 1;
    graph = false;
    if (lrsp_status s = numeric_phase(F, false, st)) return s;
    if (lrsp_status s = read_levels(&ks, &es)) return s;
  }
  F->info.graph_factor = graph ? 1 : 0;
  F->info.coop_in_graph = 0;
  bool same = true;
  for (size_t l = 0; l < F->lv.size() && same; ++l)
    if (F->lv[l].Mtot > 0 && ks[l] != F->lv[l].rec_k) same = false;
  if (!same) {
    // different ranks: plan again from scratch with the new values
    std::vector<const TreeH*> keep(F->nsys);
    for (int i = 0; i < F->nsys; ++i) keep[i] = F->sys[i].tr;
    F->free_graphs();
    F->free_device();
    const int fb = F->info.refactor_fallbacks + 1;
    lrsp_status s = batch_factor(F, A, keep.data(), status);
    F->info.refactor_fallbacks = fb;
    F->info.ms_factor = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return s;
  }
  lrsp_status s = check_status(F, status, st);
  F->info.ms_factor = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return s;
}

lrsp_status lrsp_batch_free(lrsp_batch* F) {
  delete F;
  return LRSP_OK;
}

lrsp_status lrsp_apply_batched(lrsp_batch* F, const double* b, double* x, int32_t nrhs, void* stream) {
  if (!F || !b || !x || nrhs < 1) return fail(LRSP_ERR_ARG, "invalid argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (lrsp_status s = ensure_vec(F, nrhs, st)) return s;
  return apply_cols(F, b, x, nrhs, true, st);
}

lrsp_status lrsp_pcg_batched(const lrsp_csr* A, lrsp_batch* F, const double* b, double* x,
                             int32_t nrhs, double rtol, int32_t maxit, int32_t* iters,
                             double* relres, void* stream) {
  if (!A || !F || !b || !x || nrhs < 1 || !iters || !relres || maxit < 0 || !(rtol >= 0.0))
    return fail(LRSP_ERR_ARG, "invalid argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int nsys = F->nsys;
  const int64_t ntot = F->ntot;
  for (int i = 0; i < nsys; ++i)
    if (A[i].n != F->sys[i].n || A[i].nnz != F->sys[i].nnz || !A[i].val)
      return fail(LRSP_ERR_ARG, "matrix " + std::to_string(i) + " does not match the batch");
  if (lrsp_status s = ensure_vec(F, nrhs, st)) return s;
  // merged block-diagonal matrix: pattern once, values every call
  int64_t nnzt = 0;
  for (auto& S : F->sys) nnzt += S.nnz;
  if (!F->mrowptr.p) {
    std::vector<int64_t> rp(ntot + 1);
    std::vector<int32_t> cl(nnzt);
    int64_t e0 = 0;
    for (auto& S : F->sys) {
      for (int64_t r = 0; r < S.n; ++r) rp[S.off + r] = e0 + S.rp[r];
      for (int64_t e = 0; e < S.nnz; ++e) cl[e0 + e] = (int32_t)(S.off + S.cl[e]);
      e0 += S.nnz;
    }
    rp[ntot] = e0;
    if (lrsp_status s = upload(&F->mrowptr, rp.data(), rp.size() * 8, st)) return s;
    if (lrsp_status s = upload(&F->mcol, cl.data(), cl.size() * 4, st)) return s;
    HIPCHK(dalloc(&F->mval, 8 * (size_t)std::max<int64_t>(1, nnzt), st));
  }
  {
    constexpr int64_t kChunk = 1 << 16;
    std::vector<CopyD> t;
    int64_t e0 = 0;
    for (int i = 0; i < nsys; ++i) {
      for (int64_t c = 0; c < F->sys[i].nnz; c += kChunk) {
        const int rows = (int)std::min<int64_t>(kChunk, F->sys[i].nnz - c);
        t.push_back(CopyD{A[i].val + c, at<double>(F->mval, e0 + c), rows, rows, rows, 1, 0, 0});
      }
      e0 += F->sys[i].nnz;
    }
    if ((int)t.size() > F->nmtasks) {
      dfree(&F->mtasks, st);
      HIPCHK(dalloc(&F->mtasks, t.size() * sizeof(CopyD), st));
      F->nmtasks = (int)t.size();
    }
    HIPCHK(hipMemcpyAsync(F->mtasks.p, t.data(), t.size() * sizeof(CopyD), hipMemcpyHostToDevice, st));
    launch_copy_blocks(at<CopyD>(F->mtasks, 0), (int)t.size(), st);
    HIPCHK(hipStreamSynchronize(st));
  }
  // work: r z p q (ntot*nrhs each), 5 scalars per pair, 2 ints per pair + 1
  const int np = nsys * nrhs;
  const size_t nv = (size_t)ntot * nrhs;
  const size_t need = 4 * nv + 5 * (size_t)np + (2 * (size_t)np + 2 + 1) / 2 + 1;
  if (F->pcg_doubles < need || F->pcg_nrhs != nrhs) {
    F->free_pcg_graphs();
    dfree(&F->pcg, st);
    HIPCHK(dalloc(&F->pcg, need * 8, st));
    F->pcg_doubles = need;
    F->pcg_nrhs = nrhs;
  }
  double* r = at<double>(F->pcg, 0);
  double* z = r + nv;
  double* p = z + nv;
  double* q = p + nv;
  double* bb = q + nv;
  double* rz = bb + np;
  double* rzn = rz + np;
  double* pq = rzn + np;
  double* rr = pq + np;
  int32_t* active = reinterpret_cast<int32_t*>(rr + np);
  int32_t* its = active + np;
  int32_t* nact = its + np;
  const int64_t* offs = at<int64_t>(F->offs, 0);
  const int32_t* rowsys = at<int32_t>(F->rowsys, 0);
  const int64_t* mrp = at<int64_t>(F->mrowptr, 0);
  const int32_t* mcl = at<int32_t>(F->mcol, 0);
  const double* mv = at<double>(F->mval, 0);
  launch_zero(x, (int64_t)nv, st);
  launch_seg_dot(b, b, offs, ntot, nsys, nrhs, bb, st);
  launch_bpcg_state(0, np, rtol, bb, rr, rz, rzn, active, its, nact, st);
  launch_copy(b, r, (int64_t)nv, st);
  if (lrsp_status s = apply_cols(F, r, z, nrhs, true, st)) return s;
  launch_seg_dot(r, z, offs, ntot, nsys, nrhs, rz, st);
  launch_copy(z, p, (int64_t)nv, st);
  int32_t hact = 0;
  HIPCHK(hipMemcpyAsync(&hact, nact, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  auto body1 = [&](hipStream_t s) -> lrsp_status {
    launch_spmm(mrp, mcl, mv, p, q, ntot, ntot, nrhs, s);
    launch_seg_dot(p, q, offs, ntot, nsys, nrhs, pq, s);
    launch_bpcg_xr(x, r, p, q, rowsys, ntot, nsys, nrhs, rz, pq, active, s);
    launch_seg_dot(r, r, offs, ntot, nsys, nrhs, rr, s);
    launch_bpcg_state(1, np, rtol, bb, rr, rz, rzn, active, its, nact, s);
    HIPCHK(hipGetLastError());
    return LRSP_OK;
  };
  bool in_graph = false;
  auto body2 = [&](hipStream_t s) -> lrsp_status {
    if (lrsp_status e = apply_cols(F, r, z, nrhs, in_graph, s)) return e;
    launch_seg_dot(r, z, offs, ntot, nsys, nrhs, rzn, s);
    launch_bpcg_p(p, z, rowsys, ntot, nsys, nrhs, rzn, rz, active, s);
    launch_bpcg_state(2, np, rtol, bb, rr, rz, rzn, active, its, nact, s);
    HIPCHK(hipGetLastError());
    return LRSP_OK;
  };
  // the graphs bake in x and rtol; capture again when they change
  if (F->pcg_key[0] != x || F->pcg_rtol != rtol) {
    F->free_pcg_graphs();
    F->pcg_key[0] = x;
    F->pcg_rtol = rtol;
  }
  const bool timing = g_tm.on;  // timed runs record events, outside graphs
  if (!timing && hact > 0 && !F->ge_pcg[0] && !F->pcg_no_graph) {
    in_graph = true;
    if (!capture(F, &F->g_pcg[0], &F->ge_pcg[0], body1) || !capture(F, &F->g_pcg[1], &F->ge_pcg[1], body2))
      F->free_pcg_graphs();
    in_graph = false;
  }
  const bool graphs = !timing && F->ge_pcg[0] && F->ge_pcg[1];
  F->info.graph_pcg = graphs ? 1 : 0;
  for (int it = 0; it < maxit && hact > 0; ++it) {
    if (graphs) HIPCHK(hipGraphLaunch(F->ge_pcg[0], st));
    else if (lrsp_status s = body1(st)) return s;
    HIPCHK(hipMemcpyAsync(&hact, nact, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hact == 0 || it + 1 == maxit) break;
    if (graphs) HIPCHK(hipGraphLaunch(F->ge_pcg[1], st));
    else if (lrsp_status s = body2(st)) return s;
  }
  // true residuals
  launch_spmm(mrp, mcl, mv, x, q, ntot, ntot, nrhs, st);
  launch_residual(b, q, (int64_t)nv, st);
  launch_seg_dot(q, q, offs, ntot, nsys, nrhs, rr, st);
  std::vector<double> hrr(np), hbb(np);
  std::vector<int32_t> hact_v(np);
  HIPCHK(hipMemcpyAsync(hrr.data(), rr, 8 * (size_t)np, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hbb.data(), bb, 8 * (size_t)np, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(iters, its, 4 * (size_t)np, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(hact_v.data(), active, 4 * (size_t)np, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (graphs) {
    // a software barrier that gave up invalidates the run: solve again
    // without graphs (and do not record them again for this batch)
    std::vector<GridBar> hb(2 * F->lv.size());
    HIPCHK(hipMemcpyAsync(hb.data(), F->bars.p, hb.size() * sizeof(GridBar), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool to = false;
    for (auto& g : hb) to = to || g.timeout != 0;
    if (to) {
      F->free_pcg_graphs();
      F->pcg_no_graph = true;
      F->info.graph_timeouts += 1;
      launch_zero_i32(at<int32_t>(F->bars, 0), 4 * (int64_t)hb.size(), st);
      return lrsp_pcg_batched(A, F, b, x, nrhs, rtol, maxit, iters, relres, stream);
    }
  }
  bool conv = true;
  for (int j = 0; j < np; ++j) {
    relres[j] = hbb[j] > 0 ? std::sqrt(hrr[j] / hbb[j]) : 0.0;
    if (hact_v[j]) conv = false;
  }
  if (!conv) return fail(LRSP_ERR_NO_CONV, "PCG reached maxit");
  return LRSP_OK;
}

lrsp_status lrsp_batch_info_get(const lrsp_batch* F, lrsp_batch_info* info) {
  if (!F || !info) return fail(LRSP_ERR_ARG, "null argument");
  *info = F->info;
  return LRSP_OK;
}

lrsp_status lrsp_batch_system_levels(const lrsp_batch* F, int32_t sys, int32_t* nlevels) {
  if (!F || !nlevels || sys < 0 || sys >= F->nsys) return fail(LRSP_ERR_ARG, "invalid argument");
  *nlevels = (int32_t)F->sys[sys].levels.size();
  return LRSP_OK;
}

lrsp_status lrsp_batch_level(const lrsp_batch* F, int32_t sys, int32_t level, lrsp_level_view* v) {
  if (!F || !v || sys < 0 || sys >= F->nsys) return fail(LRSP_ERR_ARG, "invalid argument");
  const BSys& S = F->sys[sys];
  if (level < 0 || level > (int)S.levels.size()) return fail(LRSP_ERR_ARG, "invalid level");
  if (level == (int)S.levels.size()) {
    v->nclusters = (int32_t)S.top_sizes.size();
    v->ncolours = 0;
    v->sizes = S.top_sizes.data();
    v->colour = nullptr;
    v->order = nullptr;
    v->ranks = nullptr;
    v->adj_ptr = S.top_adj_ptr.data();
    v->adj = S.top_adj.data();
    v->near = nullptr;
    v->far = nullptr;
    return LRSP_OK;
  }
  const LevelDev& L = *S.levels[level];
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

lrsp_status lrsp_autotune_save(const char* path) { return tune::save(path); }
lrsp_status lrsp_autotune_load(const char* path) { return tune::load(path); }
lrsp_status lrsp_autotune_clear(void) {
  tune::clear();
  return LRSP_OK;
}
int32_t lrsp_autotune_entries(void) { return tune::entries(); }

}  // extern "C"
