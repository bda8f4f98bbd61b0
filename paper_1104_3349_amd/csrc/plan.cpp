// Host-side integer planning for the device setup: the permuted CSR of C~,
// band-storage gather maps of the interior blocks A_jj, the CSR structure of
// the coupling blocks E and F, and the dense gather maps of the aggregate
// blocks G_i, D_{r_i}, E_i, F_i (Algorithm 1).  No floating-point work.
#include <algorithm>
#include <numeric>

#include "precond.h"

namespace addns {

static int32_t round_up(int32_t a, int32_t b) { return (a + b - 1) / b * b; }

void build_plan(const PartitionData& P, Plan& pl, int schur_mode, int block_mult) {
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
  // must not get more (smaller) steps than the widest one.
  pl.block_mult = std::max(1, block_mult);
  int32_t nbl_all = 1;
  for (int32_t j = 0; j < m; ++j) nbl_all = std::max({nbl_all, kl[j], (kl[j] + ku[j] + 1) / 2});
  nbl_all = round_up(nbl_all, 8) * pl.block_mult;
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
    q.nbl = nbl_all;
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

  // dense aggregate blocks
  const int32_t k = pl.k;
  pl.agg_off = P.agg_offsets;
  pl.agg_s.resize(k);
  pl.agg_d.resize(k);
  std::vector<std::vector<int32_t>> drange(k);  // new numbering
  for (int32_t i = 0; i < k; ++i) {
    pl.agg_s[i] = P.agg_offsets[i + 1] - P.agg_offsets[i];
    if (schur_mode == ADDNS_SCHUR_MSCN) {
      for (int32_t t = P.drange_offsets[i]; t < P.drange_offsets[i + 1]; ++t)
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
  for (int32_t i = 0; i < k; ++i) {
    int64_t s = pl.agg_s[i], d = pl.agg_d[i];
    pl.g_off[i + 1] = pl.g_off[i] + s * s;
    pl.dd_off[i + 1] = pl.dd_off[i] + d * d;
    pl.de_off[i + 1] = pl.de_off[i] + d * s;
    pl.df_off[i + 1] = pl.df_off[i] + s * d;
    pl.sinv_off[i + 1] = pl.sinv_off[i] + s * s;
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
    const int32_t s = pl.agg_s[i], d = pl.agg_d[i];
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
