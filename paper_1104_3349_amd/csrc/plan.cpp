// Host-side integer planning for the device setup: the permuted CSR of C~,
// band-storage gather maps of the interior blocks A_jj, the CSR structure of
// the coupling blocks E and F, and the dense gather maps of the aggregate
// blocks G_i, D_{r_i}, E_i, F_i (Algorithm 1).  No floating-point work.
#include <algorithm>
#include <cstdlib>
#include <numeric>

#include "precond.h"

namespace addns {

static int32_t round_up(int32_t a, int32_t b) { return (a + b - 1) / b * b; }

// Row width of the overlap chain matrices for aggregates of at most smax
// nodes (0: too large for the chain kernel).
int overlap_chain_width(int32_t smax) { return smax <= 64 ? 64 : (smax <= 80 ? 80 : (smax <= 128 ? 128 : 0)); }

void build_plan(const PartitionData& P, Plan& pl, int schur_mode, int block_mult, int overlap,
                bool per_interior) {
  const int32_t N = P.N;
  pl.N = N;
  pl.m = P.m;
  pl.k = P.k();
  pl.n_int = P.n_int();
  pl.nsep = P.sep_size();
  pl.perm = P.perm;
  pl.iperm.assign(N, 0);
  for (int32_t r = 0; r < N; ++r) pl.iperm[P.perm[r]] = r;

  // permuted CSR, rows in new order, columns sorted in new numbering
  pl.cp_rowptr.assign(N + 1, 0);
  pl.cp_colidx.resize(P.colidx.size());
  pl.cp_src.resize(P.colidx.size());
  pl.cp_orow.resize(P.colidx.size());
  {
    std::vector<std::pair<int32_t, int32_t>> row;
    int32_t t = 0;
    for (int32_t r = 0; r < N; ++r) {
      int32_t o = P.perm[r];
      row.clear();
      for (int32_t e = P.rowptr[o]; e < P.rowptr[o + 1]; ++e) row.emplace_back(pl.iperm[P.colidx[e]], e);
      std::sort(row.begin(), row.end());
      for (auto& ce : row) {
        pl.cp_colidx[t] = ce.first;
        pl.cp_src[t] = ce.second;
        pl.cp_orow[t] = o;
        ++t;
      }
      pl.cp_rowptr[r + 1] = t;
    }
  }
  const std::vector<int32_t>& rp = pl.cp_rowptr;
  const std::vector<int32_t>& ci = pl.cp_colidx;

  // interior bandwidths, per subdomain
  const int32_t m = P.m;
  std::vector<int32_t> sub_of(N, -1);
  for (int32_t j = 0; j < m; ++j)
    for (int32_t r = P.int_offsets[j]; r < P.int_offsets[j + 1]; ++r) sub_of[r] = j;
  std::vector<int32_t> kl(m, 0), ku(m, 0);
  for (int32_t r = 0; r < pl.n_int; ++r)
    for (int32_t t = rp[r]; t < rp[r + 1]; ++t) {
      int32_t c = ci[t];
      if (c < pl.n_int && sub_of[c] == sub_of[r]) {
        kl[sub_of[r]] = std::max(kl[sub_of[r]], r - c);
        ku[sub_of[r]] = std::max(ku[sub_of[r]], c - r);
      }
    }
  // lower blocks hold at least kl columns (the window carry then comes only
  // from the previous block), upper blocks at least kl + ku rows (U is then
  // block bidiagonal); nbu = 2 nbl lets one padding serve both sweeps
  // One block size for every subdomain: each sweep step costs about one
  // memory round trip whatever its size, so a subdomain with a narrower band
  // must not get more (smaller) steps than the widest one.  Per interior:
  // each its own minimum, fewer stored entries (the inverted diagonal blocks
  // grow with the block) for a sweep bound by memory traffic.
  pl.block_mult = std::max(1, block_mult);
  pl.per_interior = per_interior;
  auto min_nbl = [&](int32_t j) { return round_up(std::max({1, kl[j], (kl[j] + ku[j] + 1) / 2}), 8); };
  int32_t nbl_all = 1;
  for (int32_t j = 0; j < m; ++j) nbl_all = std::max(nbl_all, min_nbl(j));
  nbl_all *= pl.block_mult;
  pl.subs.assign(m, SubInfo{});
  pl.lblks.clear();
  pl.ublks.clear();
  pl.KL = pl.KU = pl.nbL = pl.nbU = pl.maxW = 0;
  int64_t band = 0, vec = 0, lm = 0, lp = 0, lw = 0, uo = 0;
  for (int32_t j = 0; j < m; ++j) {
    SubInfo& q = pl.subs[j];
    q.n = P.int_offsets[j + 1] - P.int_offsets[j];
    q.kl = kl[j];
    q.ku = ku[j];
    q.nbl = per_interior ? min_nbl(j) * pl.block_mult : nbl_all;
    q.nbu = 2 * q.nbl;
    q.npad = q.n == 0 ? 0 : round_up(q.n, q.nbu);
    q.ldab = 2 * q.kl + q.ku + 1;
    q.vec_off = (int32_t)vec;
    q.int_off = P.int_offsets[j];
    q.band_off = band;
    q.lblk0 = (int32_t)pl.lblks.size();
    q.ublk0 = (int32_t)pl.ublks.size();
    q.lmat_off = lm;
    q.lperm_off = lp;
    q.u_off = uo;
    const int32_t W = q.nbl + q.kl;
    for (int32_t b = 0; b < q.npad / q.nbl; ++b) {
      pl.lblks.push_back(LBlk{j, b, lm, lp, lw});
      lm += (int64_t)W * q.nbl;
      lp += W;
      lw += (int64_t)W * q.nbl + (int64_t)q.nbl * q.nbl;
    }
    for (int32_t b = 0; b < q.npad / q.nbu; ++b) {
      pl.ublks.push_back(UBlk{j, b, uo});
      uo += (int64_t)q.nbu * q.nbu;
    }
    band += (int64_t)q.ldab * q.npad;
    vec += q.npad;
    pl.KL = std::max(pl.KL, q.kl);
    pl.KU = std::max(pl.KU, q.ku);
    pl.nbL = std::max(pl.nbL, q.nbl);
    pl.nbU = std::max(pl.nbU, q.nbu);
    pl.maxW = std::max(pl.maxW, W);
  }
  pl.band_total = band;
  pl.npad_total = vec;
  pl.lmat_total = lm;
  pl.lperm_total = lp;
  pl.lwork_total = lw;
  pl.u_total = uo;
  pl.band_dst.clear();
  pl.band_src.clear();
  for (int32_t r = 0; r < pl.n_int; ++r) {
    const SubInfo& q = pl.subs[sub_of[r]];
    for (int32_t t = rp[r]; t < rp[r + 1]; ++t) {
      int32_t c = ci[t];
      if (c >= pl.n_int || sub_of[c] != sub_of[r]) continue;
      int32_t lr = r - q.int_off, lc = c - q.int_off;
      pl.band_dst.push_back(q.band_off + (int64_t)lc * q.ldab + (q.kl + q.ku + lr - lc));
      pl.band_src.push_back(t);
    }
  }

  // E: interior rows x separator cols; F: separator rows x interior cols
  pl.e_rowptr.assign(pl.n_int + 1, 0);
  pl.e_colidx.clear();
  pl.e_src.clear();
  for (int32_t r = 0; r < pl.n_int; ++r) {
    for (int32_t t = rp[r]; t < rp[r + 1]; ++t)
      if (ci[t] >= pl.n_int) {
        pl.e_colidx.push_back(ci[t] - pl.n_int);
        pl.e_src.push_back(t);
      }
    pl.e_rowptr[r + 1] = (int32_t)pl.e_colidx.size();
  }
  pl.f_rowptr.assign(pl.nsep + 1, 0);
  pl.f_colidx.clear();
  pl.f_src.clear();
  for (int32_t s = 0; s < pl.nsep; ++s) {
    int32_t r = pl.n_int + s;
    for (int32_t t = rp[r]; t < rp[r + 1]; ++t)
      if (ci[t] < pl.n_int) {
        pl.f_colidx.push_back(ci[t]);
        pl.f_src.push_back(t);
      }
    pl.f_rowptr[s + 1] = (int32_t)pl.f_colidx.size();
  }

  // (subdomain, separator column) couplings for the exact interface blocks
  pl.pair_sub.clear();
  pl.pair_col.clear();
  pl.pair_off.clear();
  pl.pcol_ptr.assign(1, 0);
  pl.pair_total = 0;
  if (schur_mode == ADDNS_SCHUR_EXACT_BJ) {
    std::vector<std::vector<int32_t>> subs_of_col(pl.nsep);
    for (int32_t r = 0; r < pl.n_int; ++r)
      for (int32_t t = pl.e_rowptr[r]; t < pl.e_rowptr[r + 1]; ++t) subs_of_col[pl.e_colidx[t]].push_back(sub_of[r]);
    for (int32_t c = 0; c < pl.nsep; ++c) {
      std::vector<int32_t>& v = subs_of_col[c];
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
      for (int32_t j : v) {
        pl.pair_sub.push_back(j);
        pl.pair_col.push_back(c);
        pl.pair_off.push_back(pl.pair_total);
        pl.pair_total += pl.subs[j].npad;
      }
      pl.pcol_ptr.push_back((int32_t)pl.pair_sub.size());
    }
  }

  // dense aggregate blocks
  const int32_t k = pl.k;
  pl.agg_of.assign(pl.nsep, 0);
  for (int32_t i = 0; i < k; ++i)
    for (int32_t c = P.agg_offsets[i]; c < P.agg_offsets[i + 1]; ++c) pl.agg_of[c] = i;
  pl.agg_off = P.agg_offsets;
  pl.agg_s.resize(k);
  pl.agg_d.resize(k);
  for (int32_t i = 0; i < k; ++i) pl.agg_s[i] = P.agg_offsets[i + 1] - P.agg_offsets[i];
  // overlapped aggregates: aggregate i also takes the first w_i positions of
  // aggregate i+1, w_i < s_i and w_i <= s_{i+1}; the last one takes none
  pl.overlap = overlap;
  pl.agg_w.assign(k, 0);
  pl.agg_e.resize(k);
  if (overlap > 0)
    for (int32_t i = 0; i + 1 < k; ++i)
      pl.agg_w[i] = std::max(0, std::min(overlap, std::min(pl.agg_s[i] - 1, pl.agg_s[i + 1])));
  for (int32_t i = 0; i < k; ++i) pl.agg_e[i] = pl.agg_s[i] + pl.agg_w[i];
  std::vector<std::vector<int32_t>> drange(k);  // new numbering
  for (int32_t i = 0; i < k; ++i) {
    if (schur_mode == ADDNS_SCHUR_MSCN || schur_mode == ADDNS_SCHUR_MSCNR) {
      // an extended aggregate's D-range: its own, then that of aggregate i+1
      const int32_t last = pl.agg_w[i] > 0 ? i + 1 : i;
      for (int32_t j = i; j <= last; ++j)
        for (int32_t t = P.drange_offsets[j]; t < P.drange_offsets[j + 1]; ++t)
          drange[i].push_back(pl.iperm[P.drange_nodes[t]]);
    } else if (schur_mode == ADDNS_SCHUR_MSCN_LITERAL) {
      for (int32_t s = P.agg_offsets[i]; s < P.agg_offsets[i + 1]; ++s) drange[i].push_back(s);
    }
    pl.agg_d[i] = (int32_t)drange[i].size();
  }
  pl.g_off.assign(k + 1, 0);
  pl.dd_off.assign(k + 1, 0);
  pl.de_off.assign(k + 1, 0);
  pl.df_off.assign(k + 1, 0);
  pl.sinv_off.assign(k + 1, 0);
  pl.l_off.assign(k + 1, 0);
  pl.m_off.assign(k + 1, 0);
  {
    int32_t smax = 0;
    for (int32_t i = 0; i < k; ++i) smax = std::max(smax, pl.agg_s[i]);
    pl.ovl_width = overlap > 0 ? overlap_chain_width(smax) : 0;
  }
  for (int32_t i = 0; i < k; ++i) {
    int64_t s = pl.agg_s[i], e = pl.agg_e[i], d = pl.agg_d[i];
    pl.g_off[i + 1] = pl.g_off[i] + e * e;
    pl.dd_off[i + 1] = pl.dd_off[i] + d * d;
    pl.de_off[i + 1] = pl.de_off[i] + d * e;
    pl.df_off[i + 1] = pl.df_off[i] + e * d;
    pl.sinv_off[i + 1] = pl.sinv_off[i] + s * s;
    pl.l_off[i + 1] = pl.l_off[i] + (int64_t)pl.agg_w[i] * s;
    pl.m_off[i + 1] = pl.m_off[i] + (i > 0 ? s * pl.ovl_width : 0);
  }
  // learned-correction samples: separator velocity rows, five stencil slots
  pl.smp_row.clear();
  pl.smp_nb.clear();
  pl.smp_loc.clear();
  {
    for (int32_t c = 0; c < pl.nsep; ++c) {
      const int32_t r = pl.n_int + c;
      const int32_t g = pl.perm[r];
      if (P.is_p[g]) continue;
      // velocity neighbours in the original numbering, nearest first on each side
      std::vector<std::pair<int32_t, int32_t>> lo, hi;  // (distance, permuted column)
      for (int32_t t = rp[r]; t < rp[r + 1]; ++t) {
        const int32_t o = pl.perm[ci[t]];
        if (o == g || P.is_p[o]) continue;
        (o < g ? lo : hi).emplace_back(std::abs(o - g), ci[t]);
      }
      std::sort(lo.begin(), lo.end());
      std::sort(hi.begin(), hi.end());
      int32_t nb[5] = {lo.size() > 1 ? lo[1].second : -1, lo.size() > 0 ? lo[0].second : -1, r,
                       hi.size() > 0 ? hi[0].second : -1, hi.size() > 1 ? hi[1].second : -1};
      const int32_t i = pl.agg_of[c];
      const int32_t a = c - P.agg_offsets[i], s = pl.agg_e[i];  // row stride of the dense block
      pl.smp_row.push_back(r);
      for (int q = 0; q < 5; ++q) {
        pl.smp_nb.push_back(nb[q]);
        int64_t loc = -1;
        if (nb[q] >= pl.n_int) {
          const int32_t cc = nb[q] - pl.n_int;
          if (cc >= P.agg_offsets[i] && cc < P.agg_offsets[i + 1])
            loc = pl.g_off[i] + (int64_t)a * s + (cc - P.agg_offsets[i]);
        }
        pl.smp_loc.push_back(loc);
      }
    }
  }
  pl.g_total = pl.g_off[k];
  pl.dd_total = pl.dd_off[k];
  pl.de_total = pl.de_off[k];
  pl.df_total = pl.df_off[k];
  const int64_t base_dd = pl.g_total, base_de = base_dd + pl.dd_total, base_df = base_de + pl.de_total;
  pl.dense_dst.clear();
  pl.dense_src.clear();
  std::vector<int32_t> posA(N, -1), posD(N, -1);
  for (int32_t i = 0; i < k; ++i) {
    const int32_t s = pl.agg_e[i], d = pl.agg_d[i];  // extended size (= s_i without overlap)
    for (int32_t a = 0; a < s; ++a) posA[pl.n_int + pl.agg_off[i] + a] = a;
    for (int32_t a = 0; a < d; ++a) posD[drange[i][a]] = a;
    // rows of the aggregate: G_i and F_i
    for (int32_t a = 0; a < s; ++a) {
      int32_t r = pl.n_int + pl.agg_off[i] + a;
      for (int32_t t = rp[r]; t < rp[r + 1]; ++t) {
        int32_t c = ci[t];
        if (posA[c] >= 0) {
          pl.dense_dst.push_back(pl.g_off[i] + (int64_t)a * s + posA[c]);
          pl.dense_src.push_back(t);
        }
        if (posD[c] >= 0) {
          pl.dense_dst.push_back(base_df + pl.df_off[i] + (int64_t)a * d + posD[c]);
          pl.dense_src.push_back(t);
        }
      }
    }
    // rows of the D-range: D_i and E_i
    for (int32_t a = 0; a < d; ++a) {
      int32_t r = drange[i][a];
      for (int32_t t = rp[r]; t < rp[r + 1]; ++t) {
        int32_t c = ci[t];
        if (posD[c] >= 0) {
          pl.dense_dst.push_back(base_dd + pl.dd_off[i] + (int64_t)a * d + posD[c]);
          pl.dense_src.push_back(t);
        }
        if (posA[c] >= 0) {
          pl.dense_dst.push_back(base_de + pl.de_off[i] + (int64_t)a * s + posA[c]);
          pl.dense_src.push_back(t);
        }
      }
    }
    for (int32_t a = 0; a < s; ++a) posA[pl.n_int + pl.agg_off[i] + a] = -1;
    for (int32_t a = 0; a < d; ++a) posD[drange[i][a]] = -1;
  }
}

}  // namespace addns
