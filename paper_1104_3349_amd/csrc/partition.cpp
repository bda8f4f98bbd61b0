// Substructuring of C into subdomain interiors and an interface (separator).
//
// The paper obtains P^T C P = [D E; F G] with block-diagonal D from a graph
// partitioner (section 1; section 3.3) and aggregates consecutively numbered
// interface nodes (section 3.1 step 1; Algorithm 1 breakpoints r_i).  It does
// not fix the partitioner, so this file implements one deterministic scheme:
//
//   1. pressure-like rows: diagonal absent or exactly 0.0;
//   2. H = symmetrised pattern without self-loops;
//   3. recursive level-set bisection: components of H[V] by smallest index,
//      each rooted at a pseudo-peripheral node (from the smallest index, move
//      to the least-degree, then smallest-index, node of the last BFS level
//      while the eccentricity grows); separator level t = first level whose
//      cumulative count times mV reaches |V| ceil(mV/2); pressure nodes of
//      level t move to the near side and pull their far-side neighbours into
//      the separator (the separator holds velocity nodes only); parts are
//      numbered depth first, near side first;
//   4. closure: every interior pressure component whose constant vector lies
//      in the null space of its interior block (sum over the component of
//      C(v, q) is exactly 0.0 for every adjacent interior velocity row v)
//      gives up one node to the separator, paired with an interface velocity
//      neighbour: the unclaimed pair with the strongest coupling relative to
//      the rows' largest entries (a weakly coupled pair leaves the interface
//      block nearly singular);
//   5. reverse Cuthill-McKee per interior component; separator in ascending
//      index with each closure node right after its pair;
//   6. aggregates of sz consecutive separator positions, never separating a
//      closure node from its pair;
//   7. D-ranges: the not-yet-taken interior velocity neighbours of each
//      aggregate's nodes, walking the separator in order (section 3.1 step 2b
//      allows a D-range "slightly larger" than the aggregate; the example of
//      section 3.2 takes the D nodes with direct edges to the aggregate).
//
// Only integer work, apart from the exact zero test of step 4.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "internal.h"

namespace addns {
namespace {

struct Graph {
  std::vector<int32_t> ptr, adj;  // symmetric, sorted, no self loops
  int32_t n() const { return (int32_t)ptr.size() - 1; }
};

Graph symmetrise(int32_t N, const int32_t* rowptr, const int32_t* colidx) {
  std::vector<int64_t> cnt(N + 1, 0);
  for (int32_t i = 0; i < N; ++i)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      int32_t j = colidx[e];
      if (j == i) continue;
      cnt[i + 1]++;
      cnt[j + 1]++;
    }
  for (int32_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> tmp(cnt[N]);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int32_t i = 0; i < N; ++i)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      int32_t j = colidx[e];
      if (j == i) continue;
      tmp[pos[i]++] = j;
      tmp[pos[j]++] = i;
    }
  Graph g;
  g.ptr.assign(N + 1, 0);
  g.adj.reserve(tmp.size());
  for (int32_t i = 0; i < N; ++i) {
    auto b = tmp.begin() + cnt[i], e = tmp.begin() + cnt[i + 1];
    std::sort(b, e);
    auto u = std::unique(b, e);
    g.adj.insert(g.adj.end(), b, u);
    g.ptr[i + 1] = (int32_t)g.adj.size();
  }
  return g;
}

// Work space for BFS on induced subgraphs.  `member[v] == tag` marks v as a
// vertex of the current induced subgraph.
struct Bfs {
  const Graph& g;
  std::vector<int32_t> member, level, deg;
  int32_t tag = 0;
  explicit Bfs(const Graph& g_) : g(g_), member(g_.n(), -1), level(g_.n(), -1), deg(g_.n(), 0) {}

  void select(const std::vector<int32_t>& V) {
    ++tag;
    for (int32_t v : V) member[v] = tag;
    for (int32_t v : V) {
      int32_t d = 0;
      for (int32_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) d += member[g.adj[e]] == tag;
      deg[v] = d;
    }
  }
  bool in(int32_t v) const { return member[v] == tag; }

  // BFS levels from root inside the current subgraph; returns the visited
  // nodes grouped by level (levels[d] ascending by discovery).
  int32_t levels_from(int32_t root, std::vector<int32_t>& order, std::vector<int32_t>& lstart) {
    order.clear();
    lstart.clear();
    order.push_back(root);
    level[root] = 0;
    lstart.push_back(0);
    size_t head = 0;
    int32_t cur = 0;
    while (head < order.size()) {
      int32_t u = order[head];
      if (level[u] != cur) {
        cur = level[u];
        lstart.push_back((int32_t)head);
      }
      ++head;
      for (int32_t e = g.ptr[u]; e < g.ptr[u + 1]; ++e) {
        int32_t w = g.adj[e];
        if (in(w) && level[w] < 0) {
          level[w] = cur + 1;
          order.push_back(w);
        }
      }
    }
    lstart.push_back((int32_t)order.size());
    return cur;  // eccentricity
  }
  void clear_levels(const std::vector<int32_t>& order) {
    for (int32_t v : order) level[v] = -1;
  }

  // Pseudo-peripheral root of the component of `start`; leaves the level
  // structure of the returned root in (order, lstart).
  int32_t pseudo_peripheral(int32_t start, std::vector<int32_t>& order,
                            std::vector<int32_t>& lstart) {
    int32_t r = start;
    int32_t ecc = levels_from(r, order, lstart);
    std::vector<int32_t> o2, l2;
    while (true) {
      int32_t best = -1;
      for (int32_t i = lstart[ecc]; i < lstart[ecc + 1]; ++i) {
        int32_t v = order[i];
        if (best < 0 || deg[v] < deg[best] || (deg[v] == deg[best] && v < best)) best = v;
      }
      clear_levels(order);
      int32_t ecc_c = levels_from(best, o2, l2);
      if (ecc_c > ecc) {
        r = best;
        ecc = ecc_c;
        order.swap(o2);
        lstart.swap(l2);
      } else {
        clear_levels(o2);
        levels_from(r, order, lstart);
        return r;
      }
    }
  }

  // Components of the current subgraph in order of their smallest vertex;
  // V must be sorted ascending.  Returns the smallest vertex of each.
  std::vector<int32_t> component_starts(const std::vector<int32_t>& V) {
    std::vector<int32_t> starts, order, lstart;
    for (int32_t v : V) {
      if (level[v] >= 0) continue;
      starts.push_back(v);
      levels_from(v, order, lstart);  // marks the component
    }
    for (int32_t v : V) level[v] = -1;
    return starts;
  }
};

struct Bisection {
  const Graph& g;
  const std::vector<uint8_t>& is_p;
  Bfs bfs;
  std::vector<int32_t>& part;
  int32_t next_id = 0;
  Bisection(const Graph& g_, const std::vector<uint8_t>& p_, std::vector<int32_t>& part_)
      : g(g_), is_p(p_), bfs(g_), part(part_) {}

  void run(std::vector<int32_t> V, int32_t mV) {
    if (mV == 1) {
      for (int32_t v : V) part[v] = next_id;
      ++next_id;
      return;
    }
    if (V.empty()) {
      next_id += mV;
      return;
    }
    const int32_t mA = (mV + 1) / 2;
    bfs.select(V);
    std::vector<int32_t> starts = bfs.component_starts(V);
    // concatenated level sets
    std::vector<std::vector<int32_t>> levels;
    std::vector<int32_t> order, lstart;
    for (int32_t s : starts) {
      bfs.pseudo_peripheral(s, order, lstart);
      for (size_t d = 0; d + 1 < lstart.size(); ++d)
        levels.emplace_back(order.begin() + lstart[d], order.begin() + lstart[d + 1]);
      bfs.clear_levels(order);
    }
    int64_t cum = 0;
    size_t t = 0;
    for (; t < levels.size(); ++t) {
      cum += (int64_t)levels[t].size();
      if (cum * mV >= (int64_t)V.size() * mA) break;
    }
    // side: 0 = near (A), 1 = separator, 2 = far (B); stored in bfs.level
    for (size_t d = 0; d < levels.size(); ++d)
      for (int32_t v : levels[d]) bfs.level[v] = d < t ? 0 : (d == t ? 1 : 2);
    std::vector<int32_t> sp;
    for (int32_t v : levels[t])
      if (is_p[v]) sp.push_back(v);
    std::sort(sp.begin(), sp.end());
    for (int32_t q : sp) {
      bfs.level[q] = 0;
      for (int32_t e = g.ptr[q]; e < g.ptr[q + 1]; ++e) {
        int32_t w = g.adj[e];
        if (bfs.in(w) && bfs.level[w] == 2) bfs.level[w] = 1;
      }
    }
    std::vector<int32_t> A, B;
    for (int32_t v : V) {
      int32_t s = bfs.level[v];
      if (s == 0) A.push_back(v);
      else if (s == 2) B.push_back(v);
      else part[v] = -1;
    }
    for (int32_t v : V) bfs.level[v] = -1;
    run(std::move(A), mA);
    run(std::move(B), mV - mA);
  }
};

// Reverse Cuthill-McKee of H[nodes] (nodes sorted ascending), component by
// component in order of their smallest vertex.
void rcm(Bfs& bfs, const std::vector<int32_t>& nodes, std::vector<int32_t>& out) {
  if (nodes.empty()) return;
  bfs.select(nodes);
  const Graph& g = bfs.g;
  std::vector<int32_t> starts = bfs.component_starts(nodes);
  std::vector<int32_t> order, lstart, cm, nb;
  std::vector<uint8_t> seen(0);
  for (int32_t s : starts) {
    int32_t root = bfs.pseudo_peripheral(s, order, lstart);
    bfs.clear_levels(order);
    cm.clear();
    cm.push_back(root);
    bfs.level[root] = 0;  // used as "visited"
    for (size_t head = 0; head < cm.size(); ++head) {
      int32_t u = cm[head];
      nb.clear();
      for (int32_t e = g.ptr[u]; e < g.ptr[u + 1]; ++e) {
        int32_t w = g.adj[e];
        if (bfs.in(w) && bfs.level[w] < 0) nb.push_back(w);
      }
      std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
        return bfs.deg[a] != bfs.deg[b] ? bfs.deg[a] < bfs.deg[b] : a < b;
      });
      for (int32_t w : nb) {
        bfs.level[w] = 0;
        cm.push_back(w);
      }
    }
    out.insert(out.end(), cm.rbegin(), cm.rend());
  }
  for (int32_t v : nodes) bfs.level[v] = -1;
}

}  // namespace

int build_partition(int32_t N, const int32_t* rowptr, const int32_t* colidx, const double* vals,
                    int32_t m, int32_t sz, PartitionData& P) {
  P = PartitionData();
  P.N = N;
  P.m = m;
  P.sz = sz;
  P.rowptr.assign(rowptr, rowptr + N + 1);
  P.colidx.assign(colidx, colidx + rowptr[N]);

  // 1. pressure-like rows
  P.is_p.assign(N, 1);
  for (int32_t i = 0; i < N; ++i)
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
      if (colidx[e] == i) P.is_p[i] = vals[e] == 0.0;
  const std::vector<uint8_t>& is_p = P.is_p;

  // 2. symmetric pattern
  Graph g = symmetrise(N, rowptr, colidx);

  // 3. recursive bisection
  P.part.assign(N, -1);
  {
    Bisection bis(g, is_p, P.part);
    std::vector<int32_t> all(N);
    std::iota(all.begin(), all.end(), 0);
    bis.run(std::move(all), m);
  }
  std::vector<int32_t>& part = P.part;

  // 4. closure of interior pressure components
  std::vector<double> rowmax(N, 0.0);
  for (int32_t r = 0; r < N; ++r)
    for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) rowmax[r] = std::max(rowmax[r], std::fabs(vals[e]));
  std::vector<int32_t> pair_of(N, -1);
  std::vector<uint8_t> claimed(N, 0);
  {
    std::vector<std::vector<int32_t>> members(m);
    for (int32_t v = 0; v < N; ++v)
      if (part[v] >= 0) members[part[v]].push_back(v);
    std::vector<int32_t> comp(N, -1);
    std::vector<uint8_t> inK(N, 0);
    for (int32_t j = 0; j < m; ++j) {
      const std::vector<int32_t>& nodes = members[j];
      // components of the pressure/velocity bipartite graph of the interior,
      // discovered from pressure nodes in ascending order (so each
      // component's first pressure node is its smallest)
      std::vector<std::vector<int32_t>> Ks, Vs;
      for (int32_t q0 : nodes) {
        if (!is_p[q0] || comp[q0] >= 0) continue;
        int32_t cid = (int32_t)Ks.size();
        Ks.emplace_back();
        Vs.emplace_back();
        std::vector<int32_t> stack{q0};
        comp[q0] = cid;
        while (!stack.empty()) {
          int32_t u = stack.back();
          stack.pop_back();
          (is_p[u] ? Ks : Vs)[cid].push_back(u);
          for (int32_t e = g.ptr[u]; e < g.ptr[u + 1]; ++e) {
            int32_t w = g.adj[e];
            if (part[w] != j || comp[w] >= 0 || is_p[w] == is_p[u]) continue;
            comp[w] = cid;
            stack.push_back(w);
          }
        }
      }
      for (size_t c = 0; c < Ks.size(); ++c) {
        std::vector<int32_t>& K = Ks[c];
        std::vector<int32_t>& Vv = Vs[c];
        std::sort(K.begin(), K.end());
        std::sort(Vv.begin(), Vv.end());
        for (int32_t q : K) inK[q] = 1;
        bool closed = true;
        for (int32_t v : Vv) {
          double s = 0.0;
          for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e)
            if (inK[colidx[e]]) s += vals[e];
          if (s != 0.0) {
            closed = false;
            break;
          }
        }
        for (int32_t q : K) inK[q] = 0;
        if (!closed) continue;
        // candidate pairs (q in K, separator velocity neighbour f), ranked by
        // the strength of their coupling relative to each row's largest
        // entry, |C(q,f)|/max|C(q,:)| then |C(f,q)|/max|C(f,:)|, ties to the
        // smaller q, then the smaller f; the best unclaimed f wins
        struct Cand {
          double s1, s2;
          int32_t q, f;
        };
        auto better = [](const Cand& a, const Cand& b) {
          if (a.s1 != b.s1) return a.s1 > b.s1;
          if (a.s2 != b.s2) return a.s2 > b.s2;
          if (a.q != b.q) return a.q < b.q;
          return a.f < b.f;
        };
        auto coef = [&](int32_t r, int32_t c) {
          for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e)
            if (colidx[e] == c) return std::fabs(vals[e]);
          return 0.0;
        };
        bool any = false, any_free = false;
        Cand best{}, best_free{};
        for (int32_t q : K) {
          for (int32_t e = g.ptr[q]; e < g.ptr[q + 1]; ++e) {
            const int32_t f = g.adj[e];
            if (part[f] >= 0 || is_p[f]) continue;
            const Cand c{rowmax[q] > 0.0 ? coef(q, f) / rowmax[q] : 0.0,
                         rowmax[f] > 0.0 ? coef(f, q) / rowmax[f] : 0.0, q, f};
            if (!any || better(c, best)) best = c;
            any = true;
            if (!claimed[f] && (!any_free || better(c, best_free))) best_free = c;
            any_free = any_free || !claimed[f];
          }
        }
        if (!any) continue;
        int32_t pick_q = best_free.q, pick_f = best_free.f;
        if (!any_free) {
          pick_q = best.q;
          pick_f = best.f;
          P.status = ADDNS_WARN_SHARED_PAIR;
        }
        part[pick_q] = -1;
        claimed[pick_f] = 1;
        pair_of[pick_q] = pick_f;
      }
      for (int32_t v : nodes) comp[v] = -1;
    }
  }

  // 5. orderings
  Bfs bfs(g);
  P.perm.clear();
  P.perm.reserve(N);
  P.int_offsets.assign(1, 0);
  {
    std::vector<std::vector<int32_t>> members(m);
    for (int32_t v = 0; v < N; ++v)
      if (part[v] >= 0) members[part[v]].push_back(v);
    for (int32_t j = 0; j < m; ++j) {
      rcm(bfs, members[j], P.perm);
      P.int_offsets.push_back((int32_t)P.perm.size());
    }
  }
  {
    std::vector<std::vector<int32_t>> reps(N);
    for (int32_t q = 0; q < N; ++q)
      if (pair_of[q] >= 0) reps[pair_of[q]].push_back(q);
    for (int32_t s = 0; s < N; ++s) {
      if (part[s] >= 0 || pair_of[s] >= 0) continue;
      P.perm.push_back(s);
      P.pair.push_back(-1);
      for (int32_t q : reps[s]) {  // ascending by construction
        P.perm.push_back(q);
        P.pair.push_back(s);
      }
    }
  }
  const int32_t n_int = P.int_offsets.back();
  const int32_t nsep = (int32_t)P.perm.size() - n_int;
  if ((int32_t)P.perm.size() != N) {
    set_error("partition: closure node paired with a node outside the separator");
    return ADDNS_ERR_PARTITION;
  }

  // 6. aggregates
  P.agg_offsets.assign(1, 0);
  for (int32_t r = 0; r < nsep;) {
    int32_t e = std::min(r + sz, nsep);
    while (e < nsep && P.pair[e] >= 0) ++e;
    P.agg_offsets.push_back(e);
    r = e;
  }

  // 7. D-ranges
  P.drange_offsets.assign(1, 0);
  P.drange_nodes.clear();
  {
    std::vector<uint8_t> taken(N, 0);
    const int32_t k = (int32_t)P.agg_offsets.size() - 1;
    for (int32_t i = 0; i < k; ++i) {
      for (int32_t s = P.agg_offsets[i]; s < P.agg_offsets[i + 1]; ++s) {
        int32_t gnode = P.perm[n_int + s];
        for (int32_t e = g.ptr[gnode]; e < g.ptr[gnode + 1]; ++e) {
          int32_t w = g.adj[e];
          if (part[w] >= 0 && !is_p[w] && !taken[w]) {
            taken[w] = 1;
            P.drange_nodes.push_back(w);
          }
        }
      }
      P.drange_offsets.push_back((int32_t)P.drange_nodes.size());
    }
  }
  return P.status;
}

}  // namespace addns
