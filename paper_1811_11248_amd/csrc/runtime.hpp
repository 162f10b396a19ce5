// runtime.hpp -- host runtime shared by the single-system and batched
// factorizations: error reporting, launch timing, device buffers, the device
// storage of one planned tree level and the level-assembly helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/lrsp.h"
#include "desc.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace lrsp {
namespace rt {

// Records msg as the thread's last error and returns s.
lrsp_status fail(lrsp_status s, const std::string& msg);
const char* last_error();

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ::lrsp::rt::fail(LRSP_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// Event timing of kernel families (lrsp_timing_*).
constexpr int kFamilies = 12;
struct TimingState {
  bool on = false;
  uint32_t mask = ~0u;  // families that record events
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[kFamilies];
  int64_t launches[kFamilies] = {};
  double ms[kFamilies] = {};
  double flops[kFamilies] = {};
  double bytes[kFamilies] = {};
};
extern TimingState g_tm;
hipEvent_t tm_event();
void tm_collect();

// Records events around the launches issued during its lifetime.
struct TimedLaunch {
  int fam;
  hipStream_t st;
  hipEvent_t a = nullptr;
  TimedLaunch(int f, hipStream_t s) : fam(f), st(s) {
    if (!g_tm.on || !((g_tm.mask >> f) & 1u)) return;
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

// Device buffer from the stream-ordered allocator (cached pool).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};
hipError_t dalloc(DevBuf* b, size_t bytes, hipStream_t st);
// Unused device memory the default pool keeps once a factorization or a
// tree has been released (and its stream synchronized); the rest goes back to
// the device, so that one very large factorization does not leave the next
// one of another shape to allocate around its free blocks.
constexpr size_t kPoolKeepBytes = (size_t)16 << 30;
void pool_trim();
void dfree(DevBuf* b, hipStream_t st);

template <class T>
T* at(const DevBuf& b, int64_t off) {
  return reinterpret_cast<T*>(b.p) + off;
}

uint64_t next_level_id();

// Workspace of the panels (with the inverses, tau and norms) shared by the
// levels of one tree's factorizations: a level needs its panels only while it
// is eliminated (the sweeps read the factor stores), so every level lays them
// out from the arena's start.
struct PanelArena {
  DevBuf buf;
  uint64_t gen = 0;              // advanced whenever buf is allocated anew
  hipStream_t stream = nullptr;  // stream of the last user
  bool used = false;
};
// Before a factorization on stream st works in the arena: waits for the
// last user's stream when it is another.
void arena_use(PanelArena* arena, hipStream_t st);
// Makes the arena hold at least `doubles` (allocated anew, with a new
// generation, when it is smaller); includes arena_use.
lrsp_status arena_reserve(PanelArena* arena, int64_t doubles, hipStream_t st);

// Device storage, descriptors and results of one planned tree level.
struct LevelDev {
  const uint64_t id = next_level_id();  // unique per workspace
  LevelPlan plan;
  std::vector<int> k, a, b;
  int max_m = 0, min_m = 0;
  DevBuf work, wints;      // D / fine halves; posmaps and column lists
  DevBuf coarse;           // coarse halves (sized by the rank capacities)
  DevBuf fac;              // panels, inverses, tau, norms (doubles): the level's workspace
                           // (empty when the level uses a shared arena)
  uint64_t arena_gen = 0;  // generation of the shared arena the items point into
  int64_t arena_off = 0;   // where in the arena the level's panels start (doubles)
  int64_t arena_doubles = 0;
  DevBuf sol;              // factor stores (ItemD::S) of the clusters: what the sweeps read
  std::vector<int> sol_k, sol_a;  // ranks and near-field widths the stores are laid out for
  DevBuf fints;            // colseg, colnat, stepof, piv, segoff (int32)
  DevBuf fvidx;            // vidx (int64)
  DevBuf desc;             // SegD / PairD / WbD / ItemD
  DevBuf state;            // k, a, b, err (unless the level shares a batch state)
  ItemD* d_items = nullptr;
  std::vector<ItemD> h_items;  // host copy, in processing order
  LevelState ls{};
  int sbase = 0;           // cluster id offset in a shared state
  int64_t vbase = 0;       // offset of this level in the vector buffer
  std::vector<int64_t> voff;
  int64_t nvec = 0;
  DevBuf gidx;             // level >= 1: indices into the previous level's vector
  // adjacency export
  std::vector<int> adj_ptr, adj, sizes_i, colour_i, order_i;
  std::vector<double> sweep_bytes;  // per colour: bytes one sweep of it moves
  std::vector<SplitDims> cdims;     // per colour capacities
  int max_items = 0;                // largest colour
  int max_acap = 0;                 // widest near field (capacity)
  int max_nseg = 0;
  bool split = false;               // several workgroups per cluster
  bool want_gi = true;              // room for the explicit inverses (split schedule)
  const int32_t* d_cstart = nullptr;
  DevBuf vals_off;                  // level 0: CSR entry -> work-arena offset
  DevBuf tasks;                     // level >= 1: assembly copy tasks
  int ntasks = 0;
  uint64_t tasks_src = 0;           // id of the level the tasks read from
  std::vector<std::vector<int>> next_adj;  // cluster graph of the next level (structure only)
  bool capped = false;              // rank capacities from predicted ranks
  std::vector<double> feat;         // learned ranks: features [M][12]
  std::vector<float> pred;          // and predicted ranks [M]
  std::vector<int> caps;            // rank capacities the level runs with
  int cap_tries = 0;                // runs of the level after a capacity overflow
  int32_t* h_kab = nullptr;         // pinned host copy of k, a, b and the error words
  size_t h_kab_n = 0;
  void free_all(hipStream_t st) {
    dfree(&work, st); dfree(&wints, st); dfree(&coarse, st); dfree(&fac, st); dfree(&fints, st);
    dfree(&fvidx, st); dfree(&sol, st);
    dfree(&desc, st); dfree(&state, st); dfree(&gidx, st); dfree(&vals_off, st); dfree(&tasks, st);
    if (h_kab) {
      (void)hipStreamSynchronize(st);
      (void)hipHostFree(h_kab);
    }
    h_kab = nullptr;
    h_kab_n = 0;
  }
  int64_t held_bytes() const {
    return (int64_t)(work.bytes + wints.bytes + coarse.bytes + fac.bytes + sol.bytes + fints.bytes + fvidx.bytes + desc.bytes +
                     state.bytes + gidx.bytes + vals_off.bytes + tasks.bytes);
  }
  // bytes of the level's part of the factor: the stores and the vector indices
  int64_t factor_bytes() const { return (int64_t)(sol.bytes + fvidx.bytes); }
};

// Lays out the factor stores of a finished level for its ranks L->k and
// near-field widths L->a (host copies), allocates them and points the host
// items at them; *changed tells whether the device items must be uploaded
// again (false when the stores already have this layout).
lrsp_status plan_stores(LevelDev* L, hipStream_t st, bool* changed);

// Coupling c(x,y) between the coarse DoFs of two linked clusters of a
// finished level: the source block and whether it is transposed.
bool coupling(const LevelDev& L, int x, int y, const double** src, int* sld, int* trans);

// Tasks that move the coarse-coarse couplings of finished level `prev` into
// the block storage of the next level.  False if a fill block is not dense.
bool assembly_tasks(const LevelDev& prev, const LevelDev& cur, std::vector<CopyD>* tasks);

// Indices of the coarse DoFs of finished level `prev`, in the order of the
// next level's (or the top's) clusters (parent P = children 2P, 2P+1).
void coarse_gather_indices(const LevelDev& prev, int nparents, std::vector<int64_t>* g);

// Copies a host array into a new device buffer and waits for the copy.
lrsp_status upload(DevBuf* b, const void* src, size_t bytes, hipStream_t st);

// Builds the device storage and descriptors of a planned level.  With
// `shared` the level's k/a/b/err live in a batch-wide state at cluster ids
// sbase.. (items and segments carry the shifted ids) and items report their
// errors also to *serr.
lrsp_status setup_level(LevelDev* L, hipStream_t st, int64_t vbase, int sbase = 0,
                        const LevelState* shared = nullptr, int32_t* serr = nullptr,
                        PanelArena* arena = nullptr);
// Doubles of the panel workspace of a planned level (at its capacities).
int64_t panel_doubles(const LevelDev& L);
// The two phases of setup_level.  A: layout, work arena (diagonal blocks and
// fine halves, cleared), column lists, vector offsets -- everything the
// level's assembly needs, independent of the rank capacities.  B: coarse
// region (cleared), panels and descriptors for the current capacities; it
// may be called again after the capacities change.
lrsp_status setup_level_a(LevelDev* L, hipStream_t st, int64_t vbase);
lrsp_status setup_level_b(LevelDev* L, hipStream_t st, int sbase = 0,
                          const LevelState* shared = nullptr, int32_t* serr = nullptr,
                          PanelArena* arena = nullptr);
// Points the items of a level that uses the shared arena at its current
// buffer (after the arena was allocated anew; the level's panels at
// arena_off, which the caller has reserved) and uploads them to the level's
// own item array.
lrsp_status rebind_panels(LevelDev* L, hipStream_t st, PanelArena* arena);

bool complete_graph(const std::vector<std::vector<int>>& adj);

// Level-0 CSR entry -> offset in the level's work arena (-1: not stored).
lrsp_status level0_offsets(const TreeH& tr, const int64_t* rp, const int32_t* cl, int64_t nnz,
                           const LevelPlan& p, std::vector<int64_t>* off);

// Dense top assembled from the CSR (no level eliminated): entry -> offset in
// the ntop x ntop matrix (clusters in order, toff their first rows).
void top_offsets_level0(const TreeH& tr, const int64_t* rp, const int32_t* cl, int64_t nnz,
                        const std::vector<int64_t>& toff, int ntop, std::vector<int64_t>* off);

// Dense top assembled from the coarse rows of the finished level `prev`.
void top_tasks(const LevelDev& prev, const std::vector<int64_t>& toff, int ntop, double* Tm,
               std::vector<CopyD>* tasks);

// Learned ranks of a level whose work arena holds the level-start matrix:
// features (host, [M][12]) and the network's predicted ranks (host, [M]).
lrsp_status predict_level(LevelDev* L, int level, double tol, const float* d_params, hipStream_t st,
                          std::vector<double>* feat, std::vector<float>* pred);
// Rank capacities from predicted ranks: ceil(kRankCapScale*max(y,0) + kRankCapSlack).
constexpr double kRankCapScale = 2.0;
constexpr double kRankCapSlack = 4.0;
// Targeted runs of a level after a rank overflowed its capacity before every
// capacity of the level falls back to the worst case.
constexpr int kCapRetries = 2;
std::vector<int> rank_caps(const std::vector<float>& pred);

// The cluster tree held by a tree handle.
const TreeH& tree_of(const lrsp_tree* t);

// Algorithmic flops (potrf, trsm, cpqr, applyq, schur) of a finished level
// and the bytes of one sweep per colour (into L->sweep_bytes).
void level_stats(LevelDev* L, double flops[5]);

}  // namespace rt
}  // namespace lrsp
