// plan.cpp -- host planner (tree, level graphs, colouring, symbolic fill).
#include "plan.hpp"

#include <algorithm>
#include <climits>
#include <set>

namespace lrsp {

int build_tree(int nx, int ny, int nz, int nc, int leaf, TreeH* t) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || nc <= 0 || leaf <= 0) return -1;
  const int64_t col = (int64_t)nz * nc;
  if (leaf < col) return -1;
  const int64_t n = (int64_t)nx * ny * col;
  int L = 0;
  while (((int64_t)leaf << L) < n) ++L;
  struct Box { int x0, x1, y0, y1; };
  std::vector<Box> boxes{{0, nx, 0, ny}};
  for (int d = 0; d < L; ++d) {
    std::vector<Box> nxt;
    nxt.reserve(boxes.size() * 2);
    for (const Box& b : boxes) {
      const int lx = b.x1 - b.x0, ly = b.y1 - b.y0;
      if (lx >= ly) {
        if (lx < 2) return -1;
        const int mid = b.x0 + lx / 2;
        nxt.push_back({b.x0, mid, b.y0, b.y1});
        nxt.push_back({mid, b.x1, b.y0, b.y1});
      } else {
        const int mid = b.y0 + ly / 2;
        nxt.push_back({b.x0, b.x1, b.y0, mid});
        nxt.push_back({b.x0, b.x1, mid, b.y1});
      }
    }
    boxes.swap(nxt);
  }
  t->nx = nx; t->ny = ny; t->nz = nz; t->nc = nc; t->leaf = leaf; t->L = L; t->n = n;
  t->perm.clear();
  t->perm.reserve(n);
  t->leaf_ptr.assign(1, 0);
  t->dof_cluster.assign(n, -1);
  t->dof_local.assign(n, -1);
  for (size_t c = 0; c < boxes.size(); ++c) {
    const Box& b = boxes[c];
    int loc = 0;
    // increasing (y, x, z) is increasing global id
    for (int y = b.y0; y < b.y1; ++y)
      for (int x = b.x0; x < b.x1; ++x) {
        const int64_t base = col * ((int64_t)x + (int64_t)nx * y);
        for (int64_t z = 0; z < col; ++z) {
          t->perm.push_back(base + z);
          t->dof_cluster[base + z] = (int32_t)c;
          t->dof_local[base + z] = loc++;
        }
      }
    t->leaf_ptr.push_back((int64_t)t->perm.size());
  }
  return 0;
}

// Breadth-first order of the ascending vertex set S over the subgraph it
// induces (neighbours in increasing id, restarts at the smallest unvisited
// vertex of S when the queue empties).  mark[v] == tag marks v in S and is
// set to tag + 1 once v is visited; dist (optional) receives the distances
// within start's component (-1 elsewhere).
static void bfs_order(const std::vector<int32_t>& S, const int64_t* adj_ptr, const int32_t* adj,
                      int32_t start, std::vector<int32_t>& mark, int32_t tag, std::vector<int32_t>* order,
                      std::vector<int32_t>* dist) {
  order->clear();
  order->reserve(S.size());
  mark[start] = tag + 1;
  order->push_back(start);
  if (dist) (*dist)[start] = 0;
  size_t head = 0, next_unvisited = 0;
  bool first_comp = true;
  while (order->size() < S.size()) {
    if (head == order->size()) {
      while (mark[S[next_unvisited]] != tag) ++next_unvisited;
      const int32_t v = S[next_unvisited];
      mark[v] = tag + 1;
      order->push_back(v);
      first_comp = false;
    }
    const int32_t u = (*order)[head++];
    for (int64_t e = adj_ptr[u]; e < adj_ptr[u + 1]; ++e) {
      const int32_t w = adj[e];
      if (mark[w] != tag) continue;
      mark[w] = tag + 1;
      order->push_back(w);
      if (dist && first_comp && (*dist)[u] >= 0) (*dist)[w] = (*dist)[u] + 1;
    }
  }
}

int build_tree_graph(int64_t ncols, const int64_t* adj_ptr, const int32_t* adj, int nz, int nc, int leaf,
                     TreeH* t) {
  if (ncols <= 0 || nz <= 0 || nc <= 0 || leaf <= 0 || !adj_ptr || (!adj && adj_ptr[ncols] > 0)) return -1;
  const int64_t col = (int64_t)nz * nc;
  if (leaf < col || ncols > INT32_MAX) return -1;
  for (int64_t v = 0; v < ncols; ++v) {
    if (adj_ptr[v + 1] < adj_ptr[v]) return -1;
    for (int64_t e = adj_ptr[v]; e < adj_ptr[v + 1]; ++e)
      if (adj[e] < 0 || adj[e] >= ncols || adj[e] == v) return -1;
  }
  const int64_t n = ncols * col;
  int L = 0;
  while (((int64_t)leaf << L) < n) ++L;
  std::vector<std::vector<int32_t>> sets(1);
  sets[0].resize(ncols);
  for (int64_t v = 0; v < ncols; ++v) sets[0][v] = (int32_t)v;
  // mark[v]: the tag of the set being split (even), +1 once visited
  std::vector<int32_t> mark(ncols, -2), dist(ncols, -1), order;
  int32_t tag = 0;
  for (int d = 0; d < L; ++d) {
    std::vector<std::vector<int32_t>> nxt;
    nxt.reserve(sets.size() * 2);
    for (const auto& S : sets) {
      if (S.size() < 2) return -1;
      // search 1 from the smallest vertex: the far vertex of its component
      tag += 2;
      for (int32_t v : S) {
        mark[v] = tag;
        dist[v] = -1;
      }
      bfs_order(S, adj_ptr, adj, S[0], mark, tag, &order, &dist);
      int32_t far = -1, r = S[0];
      for (int32_t v : S)  // ascending ids: the first of the largest distance
        if (dist[v] > far) {
          far = dist[v];
          r = v;
        }
      // search 2 from it; cut its order in the middle
      tag += 2;
      for (int32_t v : S) mark[v] = tag;
      bfs_order(S, adj_ptr, adj, r, mark, tag, &order, nullptr);
      const size_t h = S.size() / 2;
      std::vector<int32_t> left(order.begin(), order.begin() + h), right(order.begin() + h, order.end());
      std::sort(left.begin(), left.end());
      std::sort(right.begin(), right.end());
      nxt.push_back(std::move(left));
      nxt.push_back(std::move(right));
    }
    sets.swap(nxt);
  }
  t->nx = (int)ncols; t->ny = 1; t->nz = nz; t->nc = nc; t->leaf = leaf; t->L = L; t->n = n;
  t->perm.clear();
  t->perm.reserve(n);
  t->leaf_ptr.assign(1, 0);
  t->dof_cluster.assign(n, -1);
  t->dof_local.assign(n, -1);
  for (size_t c = 0; c < sets.size(); ++c) {
    int loc = 0;
    for (int32_t v : sets[c])
      for (int64_t z = 0; z < col; ++z) {
        const int64_t g = col * (int64_t)v + z;
        t->perm.push_back(g);
        t->dof_cluster[g] = (int32_t)c;
        t->dof_local[g] = loc++;
      }
    t->leaf_ptr.push_back((int64_t)t->perm.size());
  }
  return 0;
}

void level0_graph(const TreeH& t, const int64_t* rowptr, const int32_t* col,
                  std::vector<std::vector<int>>* adj) {
  const int M = (int)t.leaf_ptr.size() - 1;
  std::vector<std::set<int>> s(M);
  for (int64_t i = 0; i < t.n; ++i) {
    const int p = t.dof_cluster[i];
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int q = t.dof_cluster[col[e]];
      if (p != q) {
        s[p].insert(q);
        s[q].insert(p);
      }
    }
  }
  adj->assign(M, {});
  for (int p = 0; p < M; ++p) (*adj)[p].assign(s[p].begin(), s[p].end());
}

static void two_hop(const std::vector<std::vector<int>>& adj, std::vector<std::vector<int>>* out) {
  const int M = (int)adj.size();
  out->assign(M, {});
  for (int s = 0; s < M; ++s) {
    std::set<int> near(adj[s].begin(), adj[s].end());
    for (int q : adj[s]) near.insert(adj[q].begin(), adj[q].end());
    near.erase(s);
    (*out)[s].assign(near.begin(), near.end());
  }
}

void coarsen_square(const std::vector<std::vector<int>>& adj, std::vector<std::vector<int>>* out) {
  std::vector<std::vector<int>> a2;
  two_hop(adj, &a2);
  const int M = (int)adj.size();
  const int P = (M + 1) / 2;
  std::vector<std::set<int>> s(P);
  for (int x = 0; x < M; ++x)
    for (int y : a2[x])
      if (x / 2 != y / 2) s[x / 2].insert(y / 2);
  out->assign(P, {});
  for (int p = 0; p < P; ++p) (*out)[p].assign(s[p].begin(), s[p].end());
}

namespace {
using Bits = std::vector<uint64_t>;

void bits_or(Bits& dst, const std::vector<int>& idx, int nbits) {
  if (dst.empty()) dst.assign((nbits + 63) / 64, 0);
  for (int i : idx) dst[i >> 6] |= 1ull << (i & 63);
}

std::vector<int> bits_list(const Bits& b) {
  std::vector<int> out;
  for (size_t w = 0; w < b.size(); ++w) {
    uint64_t v = b[w];
    while (v) {
      const int t = __builtin_ctzll(v);
      out.push_back((int)(w * 64 + t));
      v &= v - 1;
    }
  }
  return out;
}
}  // namespace

void plan_level(LevelPlan* lp, const std::unordered_map<uint64_t, std::vector<uint64_t>>* zinit) {
  const int M = lp->M;
  two_hop(lp->adj, &lp->adj2);
  // greedy distance-2 colouring in index order
  lp->colour.assign(M, -1);
  int ncol = 0;
  for (int s = 0; s < M; ++s) {
    std::vector<char> used(lp->adj2[s].size() + 1, 0);
    for (int q : lp->adj2[s]) {
      const int c = lp->colour[q];
      if (c >= 0 && c < (int)used.size()) used[c] = 1;
    }
    int c = 0;
    while (used[c]) ++c;
    lp->colour[s] = c;
    ncol = std::max(ncol, c + 1);
  }
  lp->ncolours = ncol;
  lp->order.resize(M);
  for (int s = 0; s < M; ++s) lp->order[s] = s;
  std::stable_sort(lp->order.begin(), lp->order.end(),
                   [&](int a, int b) { return lp->colour[a] < lp->colour[b]; });
  lp->pos.assign(M, 0);
  for (int i = 0; i < M; ++i) lp->pos[lp->order[i]] = i;
  lp->cstart.assign(ncol + 1, 0);
  for (int s = 0; s < M; ++s) lp->cstart[lp->colour[s] + 1]++;
  for (int c = 0; c < ncol; ++c) lp->cstart[c + 1] += lp->cstart[c];

  // symbolic elimination in processing order
  std::unordered_map<uint64_t, Bits> Z;
  for (int p = 0; p < M; ++p)
    for (int q : lp->adj[p]) {
      Bits& z = Z[pkey(p, q)];
      if (zinit) {
        auto it = zinit->find(pkey(p, q));
        if (it != zinit->end()) z = it->second;
        else z.assign((lp->m[q] + 63) / 64, 0);
      } else {
        std::vector<int> all(lp->m[q]);
        for (int i = 0; i < lp->m[q]; ++i) all[i] = i;
        bits_or(z, all, lp->m[q]);
      }
    }
  std::vector<std::set<int>> linked(M);
  for (int p = 0; p < M; ++p) linked[p].insert(lp->adj[p].begin(), lp->adj[p].end());
  std::vector<char> done(M, 0);
  lp->nlist.assign(M, {});
  lp->wlist.assign(M, {});
  lp->kcap.assign(M, 0);
  lp->acap.assign(M, 0);
  lp->bcap.assign(M, 0);
  lp->zfin.clear();
  for (int idx = 0; idx < M; ++idx) {
    const int s = lp->order[idx];
    const std::vector<int>& nl = lp->adj[s];
    std::vector<int> wl;
    for (int q : linked[s])
      if (!std::binary_search(nl.begin(), nl.end(), q)) wl.push_back(q);
    lp->nlist[s] = nl;
    lp->wlist[s] = wl;
    int64_t acap = 0, bcap = 0;
    for (int pass = 0; pass < 2; ++pass) {
      const std::vector<int>& lst = pass ? wl : nl;
      for (int y : lst) {
        int w;
        if (done[y]) {
          w = lp->kcap[y];
        } else {
          std::vector<int> z = bits_list(Z[pkey(s, y)]);
          w = (int)z.size();
          lp->zfin[pkey(s, y)] = std::move(z);
        }
        (pass ? bcap : acap) += w;
      }
    }
    lp->acap[s] = (int)acap;
    lp->bcap[s] = (int)bcap;
    lp->kcap[s] = (int)std::min<int64_t>(lp->m[s], bcap);
    // fill among the near field
    for (int p : nl)
      for (int q : nl) {
        if (p == q) continue;
        linked[p].insert(q);
        if (!done[p] && !done[q]) bits_or(Z[pkey(p, q)], lp->zfin[pkey(s, q)], lp->m[q]);
      }
    done[s] = 1;
  }
}

void plan_capacities(LevelPlan* lp, const std::vector<int>* caps) {
  const int M = lp->M;
  std::vector<char> done(M, 0);
  for (int idx = 0; idx < M; ++idx) {
    const int s = lp->order[idx];
    int64_t acap = 0, bcap = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (int y : pass ? lp->wlist[s] : lp->nlist[s])
        (pass ? bcap : acap) += done[y] ? lp->kcap[y] : (int64_t)lp->zfin.at(pkey(s, y)).size();
    lp->acap[s] = (int)acap;
    lp->bcap[s] = (int)bcap;
    int64_t kc = std::min<int64_t>(lp->m[s], bcap);
    if (caps) kc = std::min<int64_t>(kc, std::max(0, (*caps)[s]));
    lp->kcap[s] = (int)kc;
    done[s] = 1;
  }
}

void plan_layout(LevelPlan* lp) {
  const int M = lp->M;
  int64_t off = 0, ioff = 0;
  lp->d_off.assign(M, 0);
  lp->hc_off.clear();
  lp->hf_off.clear();
  lp->pos_off.clear();
  lp->zl_off.clear();
  auto al = [](int64_t v) { return (v + 31) & ~(int64_t)31; };
  for (int x = 0; x < M; ++x) {
    lp->d_off[x] = off;
    off += al((int64_t)lp->m[x] * lp->m[x]);
  }
  for (auto& kv : lp->zfin) {
    const int e = (int)(kv.first >> 32), l = (int)(kv.first & 0xffffffffu);
    lp->hf_off[kv.first] = off;
    off += al((int64_t)lp->m[e] * (int64_t)kv.second.size());
    lp->pos_off[kv.first] = ioff;
    ioff += (lp->m[l] + 7) & ~7;
    lp->zl_off[kv.first] = ioff;
    ioff += ((int64_t)kv.second.size() + 7) & ~7;
  }
  lp->work_doubles = off;
  lp->work_ints = ioff;
  // coarse halves: their own region, the only one that depends on kcap
  int64_t coff = 0;
  for (int x = 0; x < M; ++x)
    for (int y : lp->adj2[x]) {
      if (y <= x) continue;
      const int e = lp->pos[x] < lp->pos[y] ? x : y;
      const int l = e == x ? y : x;
      lp->hc_off[pkey(l, e)] = coff;
      coff += al((int64_t)lp->m[l] * lp->kcap[e]);
    }
  lp->coarse_doubles = coff;
}

int64_t plan_panel_doubles(const LevelPlan& lp) {
  int64_t t = 0;
  for (int s = 0; s < lp.M; ++s)
    t += (int64_t)lp.m[s] * (lp.m[s] + lp.acap[s] + lp.bcap[s]);
  return t;
}

}  // namespace lrsp
