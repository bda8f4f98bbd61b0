// Host planning of the coarse-grid correction of the interface solve (the
// coarse grid correction proposed in section 6).  The coarse space Z is built
// from the pattern of C and the partition only:
//   * H = symmetrised pattern without self-loops; velocity classes = the
//     connected components of H over the non-pressure nodes, numbered by
//     their smallest node;
//   * two separator nodes are near when they share a class and are adjacent
//     in H or have a common neighbour in H;
//   * pieces: walking the separator in order, each non-pressure node not yet
//     in a piece starts one, grown breadth first through near nodes not yet
//     in a piece (neighbours in ascending position) up to P nodes;
//   * each piece gives the normalised constant and, with at least three
//     nodes, the normalised, mean-free breadth-first level along the piece
//     from the node last reached from its first node (ties: smaller
//     position).
// Then the device plan: the (subdomain, coarse column) solves that form
// D^{-1} E Z, the row pattern of S Z = G Z - F D^{-1} E Z, and the row groups
// of the restriction kernel.  Integer work plus the coarse vectors' values.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <set>

#include "precond.h"

namespace addns {

namespace {

// Breadth-first levels over adjacency lists restricted by `in` (local ids).
std::vector<int32_t> levels(const std::vector<std::vector<int32_t>>& adj, int32_t start, int32_t n) {
  std::vector<int32_t> lev(n, -1);
  std::vector<int32_t> frontier{start}, next;
  lev[start] = 0;
  while (!frontier.empty()) {
    next.clear();
    for (int32_t a : frontier)
      for (int32_t b : adj[a])
        if (lev[b] < 0) {
          lev[b] = lev[a] + 1;
          next.push_back(b);
        }
    frontier.swap(next);
  }
  return lev;
}

}  // namespace

void build_coarse_space(const PartitionData& P, int32_t piece, CoarseSpace& cs) {
  if (piece < 1) throw ArgError("coarse piece size must be >= 1");
  const int32_t N = P.N, ni = P.n_int(), ns = P.sep_size();
  cs = CoarseSpace{};
  cs.piece = piece;
  // symmetrised pattern without loops
  std::vector<std::vector<int32_t>> H(N);
  for (int32_t r = 0; r < N; ++r)
    for (int32_t e = P.rowptr[r]; e < P.rowptr[r + 1]; ++e) {
      const int32_t c = P.colidx[e];
      if (c == r) continue;
      H[r].push_back(c);
      H[c].push_back(r);
    }
  for (auto& v : H) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  // velocity classes: components over non-pressure nodes, visited from the
  // smallest node up, so class ids follow the smallest node
  std::vector<int32_t> cls(N, -1);
  int32_t ncls = 0;
  {
    std::vector<int32_t> stack;
    for (int32_t s = 0; s < N; ++s) {
      if (P.is_p[s] || cls[s] >= 0) continue;
      cls[s] = ncls;
      stack.assign(1, s);
      while (!stack.empty()) {
        const int32_t a = stack.back();
        stack.pop_back();
        for (int32_t b : H[a])
          if (!P.is_p[b] && cls[b] < 0) {
            cls[b] = ncls;
            stack.push_back(b);
          }
      }
      ++ncls;
    }
  }
  // near adjacency between separator positions of one class
  std::vector<int32_t> where(N, -1);
  for (int32_t p = 0; p < ns; ++p) where[P.perm[ni + p]] = p;
  std::vector<std::vector<int32_t>> adj(ns);
  std::vector<int32_t> mark(ns, -1);
  for (int32_t p = 0; p < ns; ++p) {
    const int32_t g = P.perm[ni + p];
    if (P.is_p[g]) continue;
    auto add = [&](int32_t x) {
      const int32_t q = where[x];
      if (q >= 0 && q != p && cls[x] == cls[g] && mark[q] != p) {
        mark[q] = p;
        adj[p].push_back(q);
      }
    };
    for (int32_t c : H[g]) {
      add(c);
      for (int32_t d : H[c]) add(d);
    }
    std::sort(adj[p].begin(), adj[p].end());
  }
  // pieces
  std::vector<int32_t> owner(ns, -1);
  cs.node_piece.assign(ns, -1);
  cs.node_z0.assign(ns, 0.0);
  cs.node_z1.assign(ns, 0.0);
  cs.piece_off.assign(1, 0);
  cs.piece_pos.clear();
  cs.col_piece.clear();
  cs.col_kind.clear();
  cs.piece_col0.clear();
  cs.piece_col1.clear();
  std::vector<int32_t> members, frontier, next;
  for (int32_t p = 0; p < ns; ++p) {
    if (P.is_p[P.perm[ni + p]] || owner[p] >= 0) continue;
    const int32_t c = (int32_t)cs.piece_off.size() - 1;
    members.assign(1, p);
    owner[p] = c;
    frontier.assign(1, p);
    while (!frontier.empty() && (int32_t)members.size() < piece) {
      next.clear();
      for (int32_t a : frontier)
        for (int32_t b : adj[a])
          if (owner[b] < 0 && (int32_t)members.size() < piece) {
            owner[b] = c;
            members.push_back(b);
            next.push_back(b);
          }
      frontier.swap(next);
    }
    const int32_t s = (int32_t)members.size();
    for (int32_t q : members) cs.piece_pos.push_back(q);
    cs.piece_off.push_back((int32_t)cs.piece_pos.size());
    const double z0 = 1.0 / std::sqrt((double)s);
    for (int32_t q : members) {
      cs.node_piece[q] = c;
      cs.node_z0[q] = z0;
    }
    cs.piece_col0.push_back((int32_t)cs.col_piece.size());
    cs.col_piece.push_back(c);
    cs.col_kind.push_back(0);
    int32_t col1 = -1;
    if (s >= 3) {
      // adjacency inside the piece, in local ids (members' order)
      std::vector<int32_t> loc(s);
      std::vector<std::vector<int32_t>> inner(s);
      for (int32_t a = 0; a < s; ++a) mark[members[a]] = -2 - a;  // local id lookup
      for (int32_t a = 0; a < s; ++a)
        for (int32_t b : adj[members[a]])
          if (owner[b] == c) inner[a].push_back(-2 - mark[b]);
      for (int32_t a = 0; a < s; ++a) mark[members[a]] = -1;
      std::vector<int32_t> lev0 = levels(inner, 0, s);
      const int32_t far = *std::max_element(lev0.begin(), lev0.end());
      int32_t r = -1;
      for (int32_t a = 0; a < s; ++a)
        if (lev0[a] == far && (r < 0 || members[a] < members[r])) r = a;
      std::vector<int32_t> lev = levels(inner, r, s);
      double mean = 0.0;
      for (int32_t a = 0; a < s; ++a) mean += lev[a];
      mean /= s;
      std::vector<double> t(s);
      double nt = 0.0;
      for (int32_t a = 0; a < s; ++a) {
        t[a] = lev[a] - mean;
        nt += t[a] * t[a];
      }
      nt = std::sqrt(nt);
      if (nt > 0.0) {
        col1 = (int32_t)cs.col_piece.size();
        cs.col_piece.push_back(c);
        cs.col_kind.push_back(1);
        for (int32_t a = 0; a < s; ++a) cs.node_z1[members[a]] = t[a] / nt;
      }
    }
    cs.piece_col1.push_back(col1);
  }
  cs.npieces = (int32_t)cs.piece_off.size() - 1;
  cs.nc = (int32_t)cs.col_piece.size();
}

void build_coarse_plan(const PartitionData& P, const Plan& pl, int32_t piece, CoarsePlan& cp) {
  build_coarse_space(P, piece, cp.space);
  const CoarseSpace& z = cp.space;
  const int32_t ni = pl.n_int, ns = pl.nsep, nc = z.nc, m = pl.m;
  std::vector<int32_t> sub_of(ni, 0);
  for (int32_t j = 0; j < m; ++j)
    for (int32_t r = pl.subs[j].int_off; r < pl.subs[j].int_off + pl.subs[j].n; ++r) sub_of[r] = j;
  cp.sub_of = sub_of;
  // subdomains touched by each piece through E (column pattern of E)
  std::vector<std::vector<int32_t>> subs_of_piece(z.npieces);
  for (int32_t r = 0; r < ni; ++r)
    for (int32_t t = pl.e_rowptr[r]; t < pl.e_rowptr[r + 1]; ++t) {
      const int32_t pc = z.node_piece[pl.e_colidx[t]];
      if (pc >= 0) subs_of_piece[pc].push_back(sub_of[r]);
    }
  for (auto& v : subs_of_piece) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  cp.pair_sub.clear();
  cp.pair_col.clear();
  cp.pair_off.clear();
  cp.cpair_ptr.assign(1, 0);
  cp.pair_total = 0;
  for (int32_t c = 0; c < nc; ++c) {
    for (int32_t j : subs_of_piece[z.col_piece[c]]) {
      cp.pair_sub.push_back(j);
      cp.pair_col.push_back(c);
      cp.pair_off.push_back(cp.pair_total);
      cp.pair_total += pl.subs[j].npad;
    }
    cp.cpair_ptr.push_back((int32_t)cp.pair_sub.size());
  }
  // separator rows that F couples to each subdomain
  std::vector<std::vector<int32_t>> rows_of_sub(m);
  for (int32_t s = 0; s < ns; ++s)
    for (int32_t t = pl.f_rowptr[s]; t < pl.f_rowptr[s + 1]; ++t) rows_of_sub[sub_of[pl.f_colidx[t]]].push_back(s);
  for (auto& v : rows_of_sub) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  // rows of S Z(:, c): G's rows touching the piece, F's rows of its subdomains
  std::vector<std::vector<int32_t>> rows_of_piece(z.npieces);
  for (int32_t s = 0; s < ns; ++s) {
    const int32_t r = ni + s;
    for (int32_t t = pl.cp_rowptr[r]; t < pl.cp_rowptr[r + 1]; ++t) {
      const int32_t c = pl.cp_colidx[t];
      if (c < ni) continue;
      const int32_t pc = z.node_piece[c - ni];
      if (pc >= 0) rows_of_piece[pc].push_back(s);
    }
  }
  for (int32_t pc = 0; pc < z.npieces; ++pc) {
    auto& v = rows_of_piece[pc];
    for (int32_t j : subs_of_piece[pc]) v.insert(v.end(), rows_of_sub[j].begin(), rows_of_sub[j].end());
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  std::vector<std::vector<int32_t>> cols_of_row(ns);
  for (int32_t c = 0; c < nc; ++c)
    for (int32_t s : rows_of_piece[z.col_piece[c]]) cols_of_row[s].push_back(c);
  cp.sz_rowptr.assign(ns + 1, 0);
  cp.sz_col.clear();
  for (int32_t s = 0; s < ns; ++s) {
    cp.sz_col.insert(cp.sz_col.end(), cols_of_row[s].begin(), cols_of_row[s].end());
    cp.sz_rowptr[s + 1] = (int32_t)cp.sz_col.size();
  }
  // row groups of the restriction kernel: every piece, then the remaining
  // separator rows (closure nodes) in runs of at most 64
  cp.grp_off.assign(1, 0);
  cp.grp_rows.clear();
  cp.grp_col0.clear();
  cp.grp_col1.clear();
  for (int32_t pc = 0; pc < z.npieces; ++pc) {
    for (int32_t t = z.piece_off[pc]; t < z.piece_off[pc + 1]; ++t) cp.grp_rows.push_back(z.piece_pos[t]);
    cp.grp_off.push_back((int32_t)cp.grp_rows.size());
    cp.grp_col0.push_back(z.piece_col0[pc]);
    cp.grp_col1.push_back(z.piece_col1[pc]);
  }
  std::vector<int32_t> rest;
  for (int32_t s = 0; s < ns; ++s)
    if (z.node_piece[s] < 0) rest.push_back(s);
  for (size_t a = 0; a < rest.size(); a += 64) {
    for (size_t b = a; b < std::min(rest.size(), a + 64); ++b) cp.grp_rows.push_back(rest[b]);
    cp.grp_off.push_back((int32_t)cp.grp_rows.size());
    cp.grp_col0.push_back(-1);
    cp.grp_col1.push_back(-1);
  }
  // per group, the union of the S Z columns on its rows (and the blocks of
  // E_c below)
  cp.grp_coff.assign(1, 0);
  cp.grp_cols.clear();
  std::vector<int32_t> u;
  for (size_t g = 0; g + 1 < cp.grp_off.size(); ++g) {
    u.clear();
    if (cp.grp_col0[g] >= 0)
      for (int32_t t = cp.grp_off[g]; t < cp.grp_off[g + 1]; ++t) {
        const int32_t s = cp.grp_rows[t];
        u.insert(u.end(), cp.sz_col.begin() + cp.sz_rowptr[s], cp.sz_col.begin() + cp.sz_rowptr[s + 1]);
      }
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    cp.grp_cols.insert(cp.grp_cols.end(), u.begin(), u.end());
    cp.grp_coff.push_back((int32_t)cp.grp_cols.size());
  }
  // blocks of E_c: columns joined when an entry E_c(c', c) can be nonzero
  // (c' a column of a group, c in the group's list), then every component
  // widened to the contiguous run of columns it spans, overlapping runs merged
  std::vector<int32_t> parent(nc);
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int32_t x) {
    while (parent[x] != x) x = parent[x] = parent[parent[x]];
    return x;
  };
  auto unite = [&](int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a != b) parent[std::max(a, b)] = std::min(a, b);
  };
  for (size_t g = 0; g + 1 < cp.grp_off.size(); ++g) {
    const int32_t c0 = cp.grp_col0[g], c1 = cp.grp_col1[g];
    if (c0 < 0) continue;
    if (c1 >= 0) unite(c0, c1);
    for (int32_t t = cp.grp_coff[g]; t < cp.grp_coff[g + 1]; ++t) unite(c0, cp.grp_cols[t]);
  }
  std::vector<int32_t> hi(nc, -1);  // last column of each component, at its root
  for (int32_t c = 0; c < nc; ++c) hi[find(c)] = std::max(hi[find(c)], c);
  cp.blk_off.assign(1, 0);
  cp.blk_eoff.assign(1, 0);
  cp.col_blk.assign(nc, 0);
  cp.blk_max = 0;
  for (int32_t c = 0, end = -1; c < nc; ++c) {
    end = std::max(end, hi[find(c)]);
    if (c == end) {  // the run [blk_off.back(), c] closes here
      const int32_t b = (int32_t)cp.blk_off.size() - 1, a = cp.blk_off.back(), sz = c + 1 - a;
      for (int32_t x = a; x <= c; ++x) cp.col_blk[x] = b;
      cp.blk_off.push_back(c + 1);
      cp.blk_eoff.push_back(cp.blk_eoff.back() + (int64_t)sz * sz);
      cp.blk_max = std::max(cp.blk_max, sz);
    }
  }
}

}  // namespace addns

extern "C" int addns_partition_coarse_space(addns_partition_t p, int32_t piece, int32_t* npieces, int32_t* ncols,
                                            int32_t* piece_offsets, int32_t* piece_pos, int32_t* col_piece,
                                            int32_t* col_kind, double* z0, double* z1) {
  return addns::guarded("addns_partition_coarse_space", [&]() -> int {
    if (!p) throw addns::ArgError("null handle");
    if (piece < 1 || piece > 64) throw addns::ArgError("piece size must lie in 1..64");
    addns::CoarseSpace cs;
    addns::build_coarse_space(p->d, piece, cs);
    if (npieces) *npieces = cs.npieces;
    if (ncols) *ncols = cs.nc;
    auto cp32 = [](int32_t* dst, const std::vector<int32_t>& src) {
      if (dst && !src.empty()) std::copy(src.begin(), src.end(), dst);
    };
    cp32(piece_offsets, cs.piece_off);
    cp32(piece_pos, cs.piece_pos);
    cp32(col_piece, cs.col_piece);
    cp32(col_kind, cs.col_kind);
    if (z0) std::copy(cs.node_z0.begin(), cs.node_z0.end(), z0);
    if (z1) std::copy(cs.node_z1.begin(), cs.node_z1.end(), z1);
    return ADDNS_OK;
  });
}
