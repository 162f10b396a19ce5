// plan.hpp -- host planner of the hierarchical factorization.
//
// For one tree level the planner fixes, from the level's cluster graph alone
// (no values): the distance-2 colouring and processing order, the near and far
// field of every cluster at the time it is processed, the column sets of the
// fine blocks (which columns of a neighbour can be nonzero), capacities for
// the value-dependent ranks, and the device layout and descriptors of all
// blocks.  Sizes of the next level depend on the ranks, which the host reads
// back once per level.
#pragma once
#include <cstdint>
#include <unordered_map>
#include <vector>

#include "desc.hpp"

namespace lrsp {

struct TreeH {
  int nx = 0, ny = 0, nz = 0, nc = 0;
  int leaf = 0;
  int L = 0;
  int64_t n = 0;
  std::vector<int64_t> perm;       // DoFs in level-0 cluster order
  std::vector<int64_t> leaf_ptr;   // [nleaves+1]
  std::vector<int32_t> dof_cluster;
  std::vector<int32_t> dof_local;
};

// Returns 0 on success, -1 on invalid arguments.
int build_tree(int nx, int ny, int nz, int nc, int leaf, TreeH* t);
// Extruded partitioning of an unstructured layer: the graph of the ncols
// vertical columns (CSR, symmetric, no self loops) is bisected L times by
// level-structure bisection (breadth-first order from a far vertex, cut in
// the middle); column v holds DoFs v*nz*nc .. (v+1)*nz*nc - 1.
int build_tree_graph(int64_t ncols, const int64_t* adj_ptr, const int32_t* adj, int nz, int nc, int leaf,
                     TreeH* t);

inline uint64_t pkey(int p, int q) { return ((uint64_t)(uint32_t)p << 32) | (uint32_t)q; }

struct LevelPlan {
  int M = 0;
  std::vector<int> m;                     // sizes at level start
  std::vector<std::vector<int>> adj;      // level graph, sorted
  std::vector<std::vector<int>> adj2;     // clusters within two hops, sorted
  std::vector<int> colour, order, pos;
  int ncolours = 0;
  std::vector<int> cstart;                // [ncolours+1] ranges of order per colour
  std::vector<std::vector<int>> nlist, wlist;
  std::unordered_map<uint64_t, std::vector<int>> zfin;  // (s,y): y later, linked at s
  std::vector<int> kcap, acap, bcap;

  // layout (offsets in doubles / ints, relative to the arenas).  The work
  // arena holds the diagonal blocks and fine halves, whose sizes do not depend
  // on the rank capacities; the coarse halves live in a region of their own.
  int64_t work_doubles = 0;
  int64_t coarse_doubles = 0;
  std::vector<int64_t> d_off;                        // D_x
  std::unordered_map<uint64_t, int64_t> hc_off;      // (l,e): coarse half, m_l x kcap_e (coarse region)
  std::unordered_map<uint64_t, int64_t> hf_off;      // (e,l): fine half, m_e x |zfin|
  std::unordered_map<uint64_t, int64_t> pos_off;     // (e,l): posmap (m_l ints) in int arena
  std::unordered_map<uint64_t, int64_t> zl_off;      // (e,l): zfin list in int arena
  int64_t work_ints = 0;
};

// Level graph of level 0 from the CSR pattern.
void level0_graph(const TreeH& t, const int64_t* rowptr, const int32_t* col,
                  std::vector<std::vector<int>>* adj);
// Parents (c -> c/2) of all pairs within two hops.
void coarsen_square(const std::vector<std::vector<int>>& adj, std::vector<std::vector<int>>* out);

// Colouring, order, symbolic fill and capacities.  zinit(p,q) gives the
// initial fine column set of block (p,q) for every edge; nullptr = dense.
void plan_level(LevelPlan* lp,
                const std::unordered_map<uint64_t, std::vector<uint64_t>>* zinit);

// Rank capacities kcap (and the near/far column capacities acap/bcap that
// follow from them) in processing order: kcap_s = min(m_s, bcap_s, caps[s])
// (caps == nullptr: the worst case min(m_s, bcap_s)).
void plan_capacities(LevelPlan* lp, const std::vector<int>* caps);

// Layout of D and the fine halves (work arena), posmaps and column lists
// (int arena), and the coarse halves (coarse region).
void plan_layout(LevelPlan* lp);

// Doubles of all panels P_s (m_s x (m_s + acap_s + bcap_s)).
int64_t plan_panel_doubles(const LevelPlan& lp);

}  // namespace lrsp
