// C-ABI entry points: setup_precond (Algorithm 1 + interior factorisation),
// apply_precond (Algorithm 2) and gmres_solve (restarted right-preconditioned
// (F)GMRES with MGS Arnoldi and Givens rotations).  Host code only orders
// kernel launches, moves a few scalars and owns device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <new>

#include "precond.h"

using namespace addns;

// Scratch of addns_apply_precond_static, for callers that cannot allocate:
// the permuted input and output vectors and the interior sweeps' two padded
// work vectors (2 N + 2 npad doubles), at most 32 MiB.  Every GPU the
// library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns on that
// device (the array's name is a host-side stand-in, not a device address).
constexpr int64_t kStaticScratchDoubles = int64_t(4) << 20;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

int prec_bytes(int prec) { return prec == P64 ? 8 : (prec == P32 ? 4 : 2); }

// Extra streams per device (index idx) for setup work that can run beside
// the interior factorisation (default priority; created once, kept until
// the process ends).
hipStream_t side_stream(int idx) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, hipStream_t>* streams = new std::map<std::pair<int, int>, hipStream_t>();
  int dev = 0;
  ADDNS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams->find({dev, idx});
  if (it != streams->end()) return it->second;
  hipStream_t st;
  ADDNS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  (*streams)[{dev, idx}] = st;
  return st;
}

void setup_coarse(addns_precond* pc, const PartitionData* P, int32_t piece, hipStream_t s, PlanCache* cache,
                  const std::function<void()>& side_work);

// Factor and interface storage of one preconditioner.
// Builds the plan from P (or keeps the handle's plan when P is null: a
// refactor) and computes every numeric part of the preconditioner.
// side_work, if given, is called once, with a stream of its own that has
// seen the final interior factors, while the coarse setup's kernels (when
// there are any) are queued on s; it must leave that stream drained.
void setup_device(addns_precond* pc, const PartitionData* P, const int32_t* d_rowptr, const int32_t* d_colidx,
                  const double* d_vals, const addns_precond_opts& o, hipStream_t s, PlanCache* cache = nullptr,
                  const std::function<void(hipStream_t)>& side_work = {}) {
  Plan& pl = pc->plan;
  if (P) {
    // the host plan depends on the partition and on (schur, block_mult,
    // overlap) only: reuse the partition's copy when those match
    const bool per = o.block_sizing == 2;
    if (cache && cache->have_plan && cache->schur == o.schur && cache->block_mult == std::max(1, o.block_mult) &&
        cache->overlap == o.overlap && cache->per_interior == (int)per) {
      pl = cache->plan;
    } else {
      build_plan(*P, pl, o.schur, o.block_mult, o.overlap, per);
      if (cache) {
        cache->plan = pl;
        cache->maps_dev = -1;
        cache->zs_choice = -1;
        cache->have_plan = true;
        cache->have_coarse = false;
        cache->cmaps_dev = -1;
        cache->schur = o.schur;
        cache->block_mult = std::max(1, o.block_mult);
        cache->overlap = o.overlap;
        cache->per_interior = (int)per;
      }
    }
  }
  const int32_t N = pl.N;
  const int64_t nnz = (int64_t)pl.cp_colidx.size();

  // the plan's maps: kept on the partition's cache for later setups
  PlanMaps local_maps;
  PlanMaps* maps = &local_maps;
  {
    int dev = 0;
    ADDNS_HIP(hipGetDevice(&dev));
    if (cache) {
      maps = &cache->maps;
      if (cache->maps_dev != dev) {
        cache->maps.upload(pl, s);
        cache->maps_dev = dev;
      }
    } else {
      local_maps.upload(pl, s);
    }
  }
  // -- permuted, row-scaled C~
  const DevBuf& d_src = maps->cp_src;
  const DevBuf& d_orow = maps->cp_orow;
  pc->perm.copy_from(maps->perm, s);
  pc->iperm.copy_from(maps->iperm, s);
  pc->R.alloc(sizeof(double) * N);
  launch_row_scale(d_rowptr, d_vals, N, o.row_scale, pc->R.as<double>(), s);
  pc->cp_rowptr.copy_from(maps->cp_rowptr, s);
  pc->cp_colidx.copy_from(maps->cp_colidx, s);
  pc->cp_vals.alloc(sizeof(double) * nnz);
  launch_gather_scaled(d_src.as<int32_t>(), d_orow.as<int32_t>(), d_vals, pc->R.as<double>(), nnz,
                       pc->cp_vals.as<double>(), s);
  const double* cpv = pc->cp_vals.as<double>();

  // -- E and F
  {
    const DevBuf& es = maps->e_src;
    const DevBuf& fs = maps->f_src;
    pc->e_rowptr.copy_from(maps->e_rowptr, s);
    pc->e_colidx.copy_from(maps->e_colidx, s);
    pc->e_vals.alloc(sizeof(double) * pl.e_src.size());
    launch_gather(es.as<int32_t>(), cpv, (int64_t)pl.e_src.size(), pc->e_vals.as<double>(), s);
    pc->f_rowptr.copy_from(maps->f_rowptr, s);
    pc->f_colidx.copy_from(maps->f_colidx, s);
    pc->f_vals.alloc(sizeof(double) * pl.f_src.size());
    launch_gather(fs.as<int32_t>(), cpv, (int64_t)pl.f_src.size(), pc->f_vals.as<double>(), s);
  }

  // -- interior blocks: band LU, then block-bidiagonal sweep form
  const int32_t m = pl.m;
  pc->subs.copy_from(maps->subs, s);
  pc->lblks.copy_from(maps->lblks, s);
  pc->ublks.copy_from(maps->ublks, s);
  const int64_t npad_total = pl.npad_total;
  pc->ypad.alloc(sizeof(double) * std::max<int64_t>(npad_total, 1));
  pc->zpad.alloc(sizeof(double) * std::max<int64_t>(npad_total, 1));
  const int32_t nL = (int32_t)pl.lblks.size(), nU = (int32_t)pl.ublks.size();
  const int fb = prec_bytes(o.interior_prec == ADDNS_F32 ? P32 : P64);
  const int iprec = o.interior_prec == ADDNS_F32 ? P32 : P64;
  DevBuf info;
  info.alloc(sizeof(int32_t) * (m + 4));
  ADDNS_HIP(hipMemsetAsync(info.p, 0, sizeof(int32_t) * (m + 4), s));
  if (pl.KL + pl.KU > 1024 || pl.nbU > 1024)
    throw ArgError("interior bandwidth too large (the band LU and the sweep take KL + KU up to 1024)");
  // the point the interface setup may start from (the info reset and the
  // permuted matrix done), before the interior work is queued
  hipEvent_t ready;
  ADDNS_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t e;
    ~EvGuard() { (void)hipEventDestroy(e); }
  } ready_guard{ready};
  ADDNS_HIP(hipEventRecord(ready, s));
  // device buffers of the interior factorisation: kept to the end of the
  // setup, since its work runs while the interface is set up
  DevBuf ab, ipiv, work, colnorm, d_nnz;
  const DevBuf& bdst = maps->band_dst;
  const DevBuf& bsrc = maps->band_src;
  const bool interior = m > 0 && npad_total > 0;
  if (interior) {
    ab.alloc(sizeof(double) * pl.band_total);
    ADDNS_HIP(hipMemsetAsync(ab.p, 0, sizeof(double) * pl.band_total, s));
    ipiv.alloc(sizeof(int32_t) * npad_total);
    launch_scatter_band(bdst.as<int64_t>(), bsrc.as<int32_t>(), cpv, (int64_t)pl.band_dst.size(), ab.as<double>(), s);
    launch_band_pad_identity(pc->subs.as<SubInfo>(), m, ab.as<double>(), s);
    colnorm.alloc(sizeof(double) * npad_total);
    int32_t npad_max = 0;
    for (const SubInfo& q : pl.subs) npad_max = std::max(npad_max, q.npad);
    // the column norms scale the incomplete factorisation's drops only: the
    // exact LU (tau = 0) multiplies them by zero
    if (o.ilu_tol > 0.0)
      launch_band_colnorm(ab.as<double>(), pc->subs.as<SubInfo>(), m, npad_max, colnorm.as<double>(), s);
    else
      ADDNS_HIP(hipMemsetAsync(colnorm.p, 0, sizeof(double) * npad_total, s));
    int32_t kl_max = 0, kv_max = 0, nbl_max = 0, nbu_max = 0;
    for (const SubInfo& q : pl.subs) {
      // the blocked band LU factors whole panels
      if (q.npad % kNpadMultiple != 0) throw std::logic_error("padded interior size is not a multiple of 16");
      kl_max = std::max(kl_max, q.kl);
      kv_max = std::max(kv_max, q.kl + q.ku);
      nbl_max = std::max(nbl_max, q.nbl);
      nbu_max = std::max(nbu_max, q.nbu);
    }
    pc->lperm.alloc(sizeof(int32_t) * pl.lperm_total);
    // the sweep's last row slot may read up to 64 * 5 rows past a block's
    // end; the zeroed tail keeps that overrun inside the allocation
    const int64_t tail = kSweepOverrunBytes;
    pc->lmat.alloc((int64_t)fb * pl.lmat_total + tail);
    pc->uinv.alloc((int64_t)fb * pl.u_total + tail);
    pc->u12.alloc((int64_t)fb * pl.u_total + tail);
    for (DevBuf* d : {&pc->lmat, &pc->uinv, &pc->u12})
      ADDNS_HIP(hipMemsetAsync(static_cast<char*>(d->p) + d->bytes - tail, 0, tail, s));
    work.alloc(sizeof(double) * std::max(pl.lwork_total, pl.u_total));
    // The band LU takes as long as its widest bands: their panels hold the
    // most rows per lane.  The subdomains that need fewer register rows go
    // to a second stream with a launch of their own (fewer rows per lane),
    // and the conversion of their blocks starts as soon as they are done,
    // beside the widest bands' elimination.  A zero pivot of the LU is
    // reported below; the conversions of such factors run but are discarded.
    auto rows_of = [](int32_t kl) { return (kl + 8 + 63) / 64; };  // panel rows per lane
    const int32_t rows_max = rows_of(kl_max);
    if (!convert_slabs(nbl_max, kl_max, nbu_max, kv_max))
      throw std::logic_error("interior blocks beyond the slab conversions");
    // bands too wide for the blocked LU take the unblocked elimination, one
    // launch over every subdomain
    const bool blocked = band_lu_blocked(kl_max);
    // group 0: the widest bands (on the caller's stream); group 1: the rest
    // (on a second stream), empty when every band needs the same rows
    std::vector<int8_t> gof(m);
    for (int32_t j = 0; j < m; ++j) gof[j] = (!blocked || rows_of(pl.subs[j].kl) == rows_max) ? 0 : 1;
    struct Launch {
      std::vector<int32_t> list;
      int32_t kl_max = 0, kv_max = 0, nb_max = 0;
      DevBuf d;
    };
    struct Group {
      Launch lu;
      std::vector<std::unique_ptr<Launch>> lower, upper;  // by block size class
    } grp[2];
    for (int32_t j = 0; j < m; ++j) {
      Launch& L = grp[gof[j]].lu;
      L.list.push_back(j);
      L.kl_max = std::max(L.kl_max, pl.subs[j].kl);
      L.kv_max = std::max(L.kv_max, pl.subs[j].kl + pl.subs[j].ku);
    }
    // the slab conversions size their LDS for the largest block of a launch:
    // one launch per size class (blocks of up to 32, 64, 128, ... rows), so
    // that small blocks of per-interior sizing keep many workgroups per CU
    auto classify = [&](std::vector<std::unique_ptr<Launch>>& out, int32_t nblk, bool upper) {
      std::map<int, Launch*> byc;
      for (int32_t i = 0; i < nblk; ++i) {
        const SubInfo& q = pl.subs[upper ? pl.ublks[i].sub : pl.lblks[i].sub];
        const int32_t nb = upper ? q.nbu : q.nbl;
        int c = 0;
        while ((32 << c) < nb) ++c;
        Launch*& L = byc[gof[upper ? pl.ublks[i].sub : pl.lblks[i].sub] * 64 + c];
        if (!L) {
          out.emplace_back(new Launch());
          L = out.back().get();
        }
        L->list.push_back(i);
        L->nb_max = std::max(L->nb_max, nb);
        L->kl_max = std::max(L->kl_max, q.kl);
        L->kv_max = std::max(L->kv_max, q.kl + q.ku);
      }
    };
    std::vector<std::unique_ptr<Launch>> lower_all, upper_all;
    classify(lower_all, nL, false);
    classify(upper_all, nU, true);
    for (auto& L : lower_all) grp[gof[pl.lblks[L->list[0]].sub]].lower.push_back(std::move(L));
    for (auto& L : upper_all) grp[gof[pl.ublks[L->list[0]].sub]].upper.push_back(std::move(L));
    // lists uploaded before any stream forks (a copy from pageable memory
    // waits for its stream's earlier work)
    for (Group& g : grp) {
      g.lu.d.upload(g.lu.list, s);
      for (auto& L : g.lower) L->d.upload(L->list, s);
      for (auto& L : g.upper) L->d.upload(L->list, s);
    }
    const bool split = !grp[1].lu.list.empty();
    hipStream_t s1 = split ? side_stream(1) : s;
    hipEvent_t ev[2];
    for (hipEvent_t& e : ev) ADDNS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    struct EvGuard2 {
      hipEvent_t* e;
      ~EvGuard2() {
        (void)hipEventDestroy(e[0]);
        (void)hipEventDestroy(e[1]);
      }
    } ev_guard{ev};
    if (split) {
      ADDNS_HIP(hipEventRecord(ev[0], s));  // the band, its norms, the lists and the tails ready
      ADDNS_HIP(hipStreamWaitEvent(s1, ev[0], 0));
    }
    for (int gi = 1; gi >= 0; --gi) {
      Group& g = grp[gi];
      if (g.lu.list.empty()) continue;
      hipStream_t sg = gi == 0 ? s : s1;
      if (blocked)
        launch_band_lu(ab.as<double>(), ipiv.as<int32_t>(), pc->subs.as<SubInfo>(), (int32_t)g.lu.list.size(),
                       info.as<int32_t>(), colnorm.as<double>(), o.ilu_tol, g.lu.kl_max, g.lu.kv_max,
                       g.lu.d.as<int32_t>(), sg);
      else
        launch_band_lu(ab.as<double>(), ipiv.as<int32_t>(), pc->subs.as<SubInfo>(), m, info.as<int32_t>(),
                       colnorm.as<double>(), o.ilu_tol, kl_max, kv_max, nullptr, sg);
      for (auto& L : g.lower)
        launch_convert_lower(ab.as<double>(), ipiv.as<int32_t>(), pc->subs.as<SubInfo>(), pc->lblks.as<LBlk>(),
                             (int32_t)L->list.size(), work.as<double>(), pc->lperm.as<int32_t>(), pc->lmat.p, iprec,
                             info.as<int32_t>() + m, L->nb_max, L->kl_max, L->d.as<int32_t>(), sg);
      for (auto& L : g.upper)
        launch_convert_upper(ab.as<double>(), pc->subs.as<SubInfo>(), pc->ublks.as<UBlk>(), (int32_t)L->list.size(),
                             work.as<double>(), pc->uinv.p, pc->u12.p, iprec, info.as<int32_t>() + m, L->nb_max,
                             L->kv_max, L->d.as<int32_t>(), sg);
    }
    if (split) {
      ADDNS_HIP(hipEventRecord(ev[1], s1));
      ADDNS_HIP(hipStreamWaitEvent(s, ev[1], 0));
    }
    d_nnz.alloc(sizeof(int64_t) * m);
    int32_t n_max = 0;
    for (const SubInfo& q : pl.subs) n_max = std::max(n_max, q.n);
    launch_band_nnz(ab.as<double>(), pc->subs.as<SubInfo>(), m, n_max, d_nnz.as<int64_t>(), s);
  }
  // reads the interior's results once its work has finished
  auto finish_interior = [&]() {
    if (!interior) return;
    std::vector<int32_t> h_info(m + 1);
    std::vector<int64_t> h_nnz(m);
    ADDNS_HIP(hipMemcpyAsync(h_info.data(), info.p, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToHost, s));
    ADDNS_HIP(hipMemcpyAsync(h_nnz.data(), d_nnz.p, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s));
    ADDNS_HIP(hipStreamSynchronize(s));
    for (int32_t j = 0; j < m; ++j)
      if (h_info[j] != 0)
        throw SingularError("interior block " + std::to_string(j) + " has a zero pivot at column " +
                            std::to_string(h_info[j] - 1));
    if (h_info[m] == 1) throw SingularError("an interior U factor has a zero diagonal");
    if (h_info[m] == 2)
      throw SingularError("the interior block factors are not finite in the storage type (overflow of the "
                          "inverted diagonal blocks)");
    pc->interior_nnz = 0;
    for (int64_t c : h_nnz) pc->interior_nnz += c;
  };

  // -- interface: dense blocks, mini Schur complements, inverses.  Except
  // for the exact block Jacobi form (which needs the interior factors) it
  // runs on a second stream while the interior factorisation, which fills
  // only one compute unit per subdomain, runs on the first.
  const int32_t k = pl.k;
  const int sprec = o.schur_prec == ADDNS_F64 ? P64 : (o.schur_prec == ADDNS_F32 ? P32 : P16S);
  auto interface_setup = [&](hipStream_t s) {
    pc->agg_off.upload(pl.agg_off, s);
    pc->agg_s.upload(pl.agg_s, s);
    pc->sinv_off.upload(pl.sinv_off, s);
    pc->schur_prec = sprec;
    pc->interior_prec = iprec;
    if (k > 0) {
      int32_t smax = 0;
      for (int32_t i = 0; i < k; ++i) smax = std::max(smax, pl.agg_s[i]);
      if (smax > 1024) throw ArgError("aggregates larger than 1024 nodes are not supported");
      if (o.overlap > 0 && smax > 128) throw ArgError("overlapped aggregates need aggregates of at most 128 nodes");
      if (o.overlap > 0 && k > kMaxOverlapAggregates)
        throw ArgError("overlapped aggregates: at most 12000 aggregates");
      const int64_t dense_n = pl.g_total + pl.dd_total + pl.de_total + pl.df_total;
      DevBuf dense, agg_d, g_off, dd_off, de_off, df_off, work;
      const DevBuf& ddst = maps->dense_dst;
      const DevBuf& dsrc = maps->dense_src;
      dense.alloc(sizeof(double) * dense_n);
      ADDNS_HIP(hipMemsetAsync(dense.p, 0, sizeof(double) * dense_n, s));
      launch_dense_scatter(ddst.as<int64_t>(), dsrc.as<int32_t>(), cpv, (int64_t)pl.dense_dst.size(), dense.as<double>(),
                           s);
      agg_d.upload(pl.agg_d, s);
      g_off.upload(pl.g_off, s);
      dd_off.upload(pl.dd_off, s);
      de_off.upload(pl.de_off, s);
      df_off.upload(pl.df_off, s);
      double* G = dense.as<double>();
      const int64_t nsmp = (int64_t)pl.smp_row.size();
      pc->learned_count = nsmp;
      if (o.schur == ADDNS_SCHUR_LEARNED) {
        pc->smp_row.upload(pl.smp_row, s);
        pc->smp_nb.upload(pl.smp_nb, s);
        pc->smp_loc.upload(pl.smp_loc, s);
      } else {  // keep G: learning targets are S_i - G_i of this (teacher) mode
        pc->g_copy.alloc(sizeof(double) * pl.g_total);
        ADDNS_HIP(hipMemcpyAsync(pc->g_copy.p, G, sizeof(double) * pl.g_total, hipMemcpyDeviceToDevice, s));
      }
      if (o.schur == ADDNS_SCHUR_LEARNED && nsmp > 0) {
        // S_i ~ G_i + Delta_i: features of each separator velocity row, the
        // network's corrections on G's stencil slots inside the aggregate
        const int np = mlp_param_count();
        DevBuf wts, img, X, Dl;
        wts.alloc(sizeof(float) * np);
        img.alloc(sizeof(float) * mlp_image_floats());
        ADDNS_HIP(hipMemcpyAsync(wts.p, o.learned_model, sizeof(float) * np, hipMemcpyHostToDevice, s));
        launch_mlp_image(wts.as<float>(), img.as<float>(), s);
        X.alloc(sizeof(float) * 7 * nsmp);
        Dl.alloc(sizeof(float) * 5 * nsmp);
        launch_dtn_features(nsmp, pc->smp_row.as<int32_t>(), pc->smp_nb.as<int32_t>(), pc->cp_rowptr.as<int32_t>(),
                            pc->cp_colidx.as<int32_t>(), cpv, pc->perm.as<int32_t>(), pc->R.as<double>(),
                            X.as<float>(), s);
        launch_mlp_forward(img.as<float>(), X.as<float>(), Dl.as<float>(), nsmp, o.learned_bf16 ? 1 : 0, s);
        launch_dtn_correct(nsmp, pc->smp_loc.as<int64_t>(), Dl.as<float>(), G, s);
        ADDNS_HIP(hipStreamSynchronize(s));
      }
      if (o.schur == ADDNS_SCHUR_EXACT_BJ) {
        const int32_t np = (int32_t)pl.pair_sub.size();
        DevBuf psub, pcol, poff, pptr, aggof, U, scratch;
        psub.upload(pl.pair_sub, s);
        pcol.upload(pl.pair_col, s);
        poff.upload(pl.pair_off, s);
        pptr.upload(pl.pcol_ptr, s);
        aggof.upload(pl.agg_of, s);
        U.alloc(sizeof(double) * std::max<int64_t>(pl.pair_total, 1));
        scratch.alloc(sizeof(double) * std::max<int64_t>(pl.pair_total, 1));
        launch_column_solves(pc, np, psub.as<int32_t>(), pcol.as<int32_t>(), poff.as<int64_t>(), scratch.as<double>(),
                             U.as<double>(), s);
        launch_exact_schur_update(pl.nsep, pptr.as<int32_t>(), psub.as<int32_t>(), poff.as<int64_t>(),
                                  pc->subs.as<SubInfo>(), aggof.as<int32_t>(), pc->agg_off.as<int32_t>(),
                                  g_off.as<int64_t>(), pc->f_rowptr.as<int32_t>(), pc->f_colidx.as<int32_t>(),
                                  pc->f_vals.as<double>(), U.as<double>(), G, s);
        ADDNS_HIP(hipStreamSynchronize(s));
      }
      DevBuf agg_e;  // extended aggregate sizes (= agg_s without overlap)
      agg_e.upload(pl.agg_e, s);
      if (o.schur == ADDNS_SCHUR_MSCN || o.schur == ADDNS_SCHUR_MSCN_LITERAL || o.schur == ADDNS_SCHUR_MSCNR)
        launch_schur_blocks(k, agg_e.as<int32_t>(), agg_d.as<int32_t>(), g_off.as<int64_t>(), dd_off.as<int64_t>(),
                            de_off.as<int64_t>(), df_off.as<int64_t>(), G, G + pl.g_total,
                            G + pl.g_total + pl.dd_total, G + pl.g_total + pl.dd_total + pl.de_total,
                            info.as<int32_t>() + m + 1, o.schur == ADDNS_SCHUR_MSCNR ? 1 : 0, s);
      pc->schur_S.alloc(sizeof(double) * pl.g_total);
      ADDNS_HIP(hipMemcpyAsync(pc->schur_S.p, G, sizeof(double) * pl.g_total, hipMemcpyDeviceToDevice, s));
      const int64_t a_total = pl.sinv_off[k];
      pc->sinv.alloc((int64_t)prec_bytes(sprec) * a_total);
      pc->sinv_scale.alloc(sizeof(float) * k);
      work.alloc(sizeof(double) * 2 * a_total);
      if (o.overlap == 0) {
        launch_invert_dense(k, pc->agg_s.as<int32_t>(), g_off.as<int64_t>(), G, work.as<double>(),
                            info.as<int32_t>() + m + 2, pc->sinv_off.as<int64_t>(), pc->sinv.p,
                            pc->sinv_scale.as<float>(), sprec, s);
      } else {
        // Shat block lower bidiagonal: invert its diagonal blocks A_i, then
        // form the chain matrices M_i from the FP64 inverses
        DevBuf agg_w, l_off, A, L;
        agg_w.upload(pl.agg_w, s);
        l_off.upload(pl.l_off, s);
        A.alloc(sizeof(double) * std::max<int64_t>(a_total, 1));
        L.alloc(sizeof(double) * std::max<int64_t>(pl.l_off[k], 1));
        launch_overlap_split(k, pc->agg_s.as<int32_t>(), agg_w.as<int32_t>(), g_off.as<int64_t>(),
                             pc->sinv_off.as<int64_t>(), l_off.as<int64_t>(), G, A.as<double>(), L.as<double>(), s);
        launch_invert_dense(k, pc->agg_s.as<int32_t>(), pc->sinv_off.as<int64_t>(), A.as<double>(), work.as<double>(),
                            info.as<int32_t>() + m + 2, pc->sinv_off.as<int64_t>(), pc->sinv.p,
                            pc->sinv_scale.as<float>(), sprec, s);
        const int mdbl = sprec == P64 ? 1 : 0;
        pc->ovl_moff.upload(pl.m_off, s);
        pc->ovl_m.alloc((mdbl ? 8 : 4) * std::max<int64_t>(pl.m_off[k], 1));
        launch_overlap_m(k, pc->agg_s.as<int32_t>(), agg_w.as<int32_t>(), pc->sinv_off.as<int64_t>(),
                         l_off.as<int64_t>(), pc->ovl_moff.as<int64_t>(), pl.ovl_width, work.as<double>(),
                         L.as<double>(), pc->ovl_m.p, mdbl, s);
        pc->overlap_chain = k > 1 ? pl.ovl_width : 0;
        // the chain in segments: responses of each segment's aggregates to the
        // previous segment's last one
        pc->ovl_seg = overlap_segment_length(k, o.overlap_segment);
        if (pc->overlap_chain && (k + pc->ovl_seg - 1) / pc->ovl_seg > 1) {
          pc->ovl_q.alloc((mdbl ? 8 : 4) * std::max<int64_t>(pl.m_off[k], 1));
          launch_overlap_q(pc, s);
        } else {
          pc->ovl_q.reset();
        }
        ADDNS_HIP(hipStreamSynchronize(s));
      }
      int32_t h2[2];
      ADDNS_HIP(hipMemcpyAsync(h2, info.as<int32_t>() + m + 1, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s));
      ADDNS_HIP(hipStreamSynchronize(s));
      if (h2[0]) throw SingularError("a D-range block D_{r_i} is singular");
      if (h2[1]) throw SingularError("an interface block S_i is singular");
    }
    ADDNS_HIP(hipStreamSynchronize(s));
  };
  if (o.schur == ADDNS_SCHUR_EXACT_BJ) {
    finish_interior();
    interface_setup(s);
  } else {
    hipStream_t s2 = side_stream(0);
    ADDNS_HIP(hipStreamWaitEvent(s2, ready, 0));
    interface_setup(s2);
    finish_interior();
  }

  // -- coarse-grid correction of the interface solve (section 6), with the
  // caller's side work on another stream beside its kernels
  ADDNS_HIP(hipEventRecord(ready, s));  // the interior factors are final
  auto side = [&]() {
    if (!side_work) return;
    hipStream_t cs = side_stream(0);
    ADDNS_HIP(hipStreamWaitEvent(cs, ready, 0));
    side_work(cs);
  };
  pc->coarse_nc = 0;
  if (o.coarse > 0 && pl.nsep > 0) setup_coarse(pc, P, o.coarse, s, cache, side);
  else side();

  // permuted in/out vectors of addns_apply_precond: allocated here so that
  // an apply launches kernels only (and can be captured in a graph)
  pc->vperm_in.alloc(sizeof(double) * N);
  pc->vperm_out.alloc(sizeof(double) * N);

  // -- byte accounting
  int64_t fbytes = 0;
  fbytes += pl.lmat_total * fb + pl.lperm_total * 4;
  fbytes += 2 * pl.u_total * fb;
  const int64_t a_total = k > 0 ? pl.sinv_off[k] : 0;
  // chain matrices read once, and the responses once more when the chain
  // runs in segments
  const int64_t m_bytes = pc->overlap_chain ? pl.m_off[k] * (sprec == P64 ? 8 : 4) *
                                                  ((k + pc->ovl_seg - 1) / pc->ovl_seg > 1 ? 2 : 1)
                                            : 0;
  fbytes += a_total * prec_bytes(sprec) + m_bytes;
  pc->factor_bytes = fbytes;
  // algorithmic bytes of one apply: band factors L (KL) and U (KL+KU+1) per
  // interior row read twice, pivots, E and F (value + index), Shat^-1, and six
  // vector passes
  int64_t band = 0;
  for (int32_t j = 0; j < m; ++j) band += (int64_t)pl.subs[j].n * (2 * pl.subs[j].kl + pl.subs[j].ku + 1);
  pc->bytes_apply = 2 * band * fb + 2 * 4 * (int64_t)pl.n_int +
                    (int64_t)(pl.e_src.size() + pl.f_src.size()) * 12 + a_total * prec_bytes(sprec) + m_bytes +
                    6 * (int64_t)N * 8;
  // coarse correction: E_c^{-1}, S Z (value + column), the coarse vectors
  // and piece ids, and t written once and read once
  if (pc->coarse_nc > 0)
    pc->bytes_apply += pc->coarse.blk_eoff.back() * 8 + (int64_t)pc->coarse.sz_col.size() * 12 +
                       (int64_t)pl.nsep * (4 + 8 + 8 + 16);
}

// Coarse-grid correction of the interface solve: the coarse space from the
// partition (a refactor keeps it), S Z = G Z - F D^{-1} E Z from one interior
// sweep per (subdomain, coarse column) pair, E_c = Z^T S Z and its inverse.
// side_work is called once, after all of that is queued on s and before the
// host waits for it.
void setup_coarse(addns_precond* pc, const PartitionData* P, int32_t piece, hipStream_t s, PlanCache* cache,
                  const std::function<void()>& side_work) {
  const Plan& pl = pc->plan;
  CoarsePlan& cp = pc->coarse;
  pc->coarse_nc = 0;
  if (P) {
    if (cache && cache->have_coarse && cache->piece == piece) {
      cp = cache->coarse;
    } else {
      build_coarse_plan(*P, pl, piece, cp);
      if (cache && cache->have_plan) {
        cache->coarse = cp;
        cache->have_coarse = true;
        cache->piece = piece;
        cache->cmaps_dev = -1;
      }
    }
  }
  const CoarseSpace& z = cp.space;
  const int32_t nc = z.nc;
  if (nc > kMaxCoarseColumns)
    throw ArgError("coarse space of " + std::to_string(nc) + " columns exceeds 8192 (use a larger piece size)");
  // the coarse plan's arrays: kept on the partition's cache for later setups
  CoarseMaps local_maps;
  CoarseMaps* cm = &local_maps;
  {
    int dev = 0;
    ADDNS_HIP(hipGetDevice(&dev));
    if (P && cache && cache->have_coarse && cache->piece == piece) {
      cm = &cache->cmaps;
      if (cache->cmaps_dev != dev) {
        cache->cmaps.upload(cp, pl, s);
        cache->cmaps_dev = dev;
      }
    } else {
      local_maps.upload(cp, pl, s);
    }
  }
  pc->cz_piece.copy_from(cm->piece, s);
  pc->cz_z0.copy_from(cm->z0, s);
  pc->cz_z1.copy_from(cm->z1, s);
  pc->cz_colp.copy_from(cm->colp, s);
  pc->cz_colk.copy_from(cm->colk, s);
  pc->cz_p0.copy_from(cm->p0, s);
  pc->cz_p1.copy_from(cm->p1, s);
  pc->cz_szp.copy_from(cm->szp, s);
  pc->cz_szc.copy_from(cm->szc, s);
  pc->cz_szv.alloc(sizeof(double) * cp.sz_col.size());
  pc->cz_goff.copy_from(cm->goff, s);
  pc->cz_grows.copy_from(cm->grows, s);
  pc->cz_gc0.copy_from(cm->gc0, s);
  pc->cz_gc1.copy_from(cm->gc1, s);
  pc->cz_gcoff.copy_from(cm->gcoff, s);
  pc->cz_gcols.copy_from(cm->gcols, s);
  pc->cz_t.alloc(sizeof(double) * std::max<int32_t>(pl.nsep, 1));
  pc->cz_g.alloc(sizeof(double) * std::max<int32_t>(nc, 1));
  pc->cz_y.alloc(sizeof(double) * std::max<int32_t>(nc, 1));
  pc->cz_boff.copy_from(cm->boff, s);
  pc->cz_cblk.copy_from(cm->cblk, s);
  pc->cz_beoff.copy_from(cm->beoff, s);
  const int64_t ec_total = cp.blk_eoff.empty() ? 0 : cp.blk_eoff.back();
  pc->cz_einv.alloc(sizeof(double) * std::max<int64_t>(ec_total, 1));
  if (nc == 0) {
    side_work();
    return;
  }
  const DevBuf &psub = cm->psub, &pcol = cm->pcol, &poff = cm->poff, &cpp = cm->cpp, &subof = cm->subof,
               &ioff = cm->ioff;
  DevBuf W, scratch, perm, work, info;
  W.alloc(sizeof(double) * std::max<int64_t>(cp.pair_total, 1));
  scratch.alloc(sizeof(double) * std::max<int64_t>(cp.pair_total, 1));
  const int32_t npairs = (int32_t)cp.pair_sub.size();
  launch_coarse_column_solves(pc, npairs, psub.as<int32_t>(), pcol.as<int32_t>(), poff.as<int64_t>(),
                              scratch.as<double>(), W.as<double>(), 0, s);
  // one FP64 refinement step: E_c^{-1} amplifies errors of S Z by cond(E_c),
  // and the sweep's explicitly inverted blocks (or FP32 factors) leave
  // W = D^{-1} E Z accurate only to eps * cond(A_jj) of the storage
  DevBuf dW;
  dW.alloc(sizeof(double) * std::max<int64_t>(cp.pair_total, 1));
  launch_coarse_refine(pc, npairs, psub.as<int32_t>(), pcol.as<int32_t>(), poff.as<int64_t>(), W.as<double>(),
                       scratch.as<double>(), dW.as<double>(), s);
  launch_coarse_sz(pc, subof.as<int32_t>(), psub.as<int32_t>(), cpp.as<int32_t>(), poff.as<int64_t>(),
                   ioff.as<int32_t>(), W.as<double>(), s);
  double* Ec = pc->cz_einv.as<double>();
  ADDNS_HIP(hipMemsetAsync(Ec, 0, sizeof(double) * (size_t)ec_total, s));
  launch_coarse_ec(pc, nc, Ec, s);
  perm.alloc(sizeof(int32_t) * nc);
  work.alloc(sizeof(double) * (cp.blk_off.size() + 2 * (size_t)nc));
  info.alloc(sizeof(int32_t));
  ADDNS_HIP(hipMemsetAsync(info.p, 0, sizeof(int32_t), s));
  launch_gj_invert(pc, Ec, perm.as<int32_t>(), work.as<double>(), info.as<int32_t>(), s);
  // the whole chain is queued: the side work runs beside it (before the
  // read of the pivot flag, which waits for the chain)
  side_work();
  int32_t h_info = 0;
  ADDNS_HIP(hipMemcpyAsync(&h_info, info.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  ADDNS_HIP(hipStreamSynchronize(s));
  if (h_info) throw SingularError("the coarse matrix Z^T S Z is singular (pivot " + std::to_string(h_info - 1) + ")");
  pc->coarse_nc = nc;
}

// ypad, zpad: the two padded vectors of the interior sweeps (NULL: the
// handle's own)
void apply_permuted(addns_precond* pc, const double* yp, double* xp, hipStream_t s, double* ypad = nullptr,
                    double* zpad = nullptr) {
  const Plan& pl = pc->plan;
  // z1 = D^{-1} y1 (into the interior part of xp)
  launch_interior_solve(pc, yp, xp, 0, nullptr, nullptr, s, ypad);
  // two-level interface solve: t = y2 - F z1 and Z^T t, then y = E_c^{-1} Z^T t
  if (pc->coarse_nc > 0) {
    launch_coarse_restrict(pc, yp, xp, s);
    launch_coarse_solve(pc, s);
  }
  // x2 = Shat^{-1} (y2 - F z1): blockwise, then (overlapped aggregates) the
  // forward substitution over Shat's lower blocks
  launch_interface_solve(pc, yp, xp, xp, s);
  launch_overlap_chain(pc, xp + pl.n_int, s);
  // x1 = z1 - D^{-1} (E x2), in place
  if (pl.k > 0) launch_interior_solve(pc, nullptr, xp, 1, xp + pl.n_int, xp, s, zpad);
}

// Mean duration (ms) of a few interior solves on the handle's own factors.
float time_interior_solve(addns_precond* pc, hipStream_t s) {
  const Plan& pl = pc->plan;
  if (pl.n_int == 0 || pl.m == 0) return 0.0f;
  DevBuf y, z;
  y.alloc(sizeof(double) * pl.n_int);
  z.alloc(sizeof(double) * pl.n_int);
  ADDNS_HIP(hipMemsetAsync(y.p, 0, sizeof(double) * pl.n_int, s));
  hipEvent_t e0, e1;
  ADDNS_HIP(hipEventCreate(&e0));
  ADDNS_HIP(hipEventCreate(&e1));
  launch_interior_solve(pc, y.as<double>(), z.as<double>(), 0, nullptr, nullptr, s);
  ADDNS_HIP(hipEventRecord(e0, s));
  const int reps = 2;
  for (int r = 0; r < reps; ++r) launch_interior_solve(pc, y.as<double>(), z.as<double>(), 0, nullptr, nullptr, s);
  ADDNS_HIP(hipEventRecord(e1, s));
  ADDNS_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  ADDNS_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

// Chunk count of the interior sweep.  requested 1: none; >= 2: that many;
// 0: the p that minimises a fixed model of the chunked solve, from the plan
// and the device's CU count only (never from a timing, so the choice, and
// with it the rounding of every solve, is the same on every run and box):
// the longest chunk sweeps ceil(nU / p) of the nU upper blocks at
// kSweepBlockUs each, every chunk boundary adds kSweepBoundaryUs for the two
// recurrences, and p is capped at one workgroup per CU over the m interiors.
// The constants are the per-block step and per-boundary costs measured on
// the 128 x 128 workload (0.21 ms over 12 upper blocks; about 5 us).
constexpr double kSweepBlockUs = 17.5, kSweepBoundaryUs = 5.0;

int model_sweep_chunks(const Plan& pl, int cus) {
  if (pl.m == 0 || pl.n_int == 0) return 1;
  int32_t nu = 1;
  for (const SubInfo& q : pl.subs) nu = std::max(nu, q.npad / q.nbu);
  const int pcap = std::min(max_sweep_chunks(pl), std::max(1, cus / pl.m));
  int p = 1;
  double best = nu * kSweepBlockUs;
  for (int c = 2; c <= pcap; ++c) {
    const double model = (double)((nu + c - 1) / c) * kSweepBlockUs + kSweepBoundaryUs * (c - 1);
    if (model < best) {
      best = model;
      p = c;
    }
  }
  return p;
}

void choose_sweep_chunks(addns_precond* pc, int requested, hipStream_t s) {
  const Plan& pl = pc->plan;
  release_chunked_sweep(pc);
  if (requested == 1 || pl.m == 0 || pl.n_int == 0) return;
  const int pmax = max_sweep_chunks(pl);
  if (requested >= 2) {
    if (requested > pmax) throw ArgError("sweep_chunks exceeds the upper blocks of an interior");
    build_chunked_sweep(pc, requested, s);
    return;
  }
  hipDeviceProp_t prop;
  ADDNS_HIP(hipGetDeviceProperties(&prop, pc->device));
  const int p = model_sweep_chunks(pl, prop.multiProcessorCount);
  if (p < 2) return;
  build_chunked_sweep(pc, p, s);
}

// Zero-slot form of the sweep in use (single-workgroup or chunked): the
// caller's choice, or the faster of the two by timing.  Both give the same
// result bit for bit, so the timing never changes numerics.  A later setup
// on the same plan (the partition's cache) and device with the same interior
// precision, chunk count and drop tolerance takes the choice timed before.
void choose_zero_skip(addns_precond* pc, int requested, double ilu_tol, hipStream_t s, PlanCache* cache) {
  if (requested != 0) {
    pc->zero_skip = requested == 2 ? 1 : 0;
    return;
  }
  if (cache && cache->zs_choice >= 0 && cache->zs_dev == pc->device && cache->zs_prec == pc->interior_prec &&
      cache->zs_chunks == pc->sweep_chunks && cache->zs_ilu == ilu_tol) {
    pc->zero_skip = cache->zs_choice;
    pc->tuned_ms = cache->zs_ms;
    return;
  }
  float ms[2];
  for (int z = 0; z < 2; ++z) {
    pc->zero_skip = z;
    ms[z] = time_interior_solve(pc, s);
  }
  pc->zero_skip = ms[1] < ms[0] ? 1 : 0;
  pc->tuned_ms = std::min(ms[0], ms[1]);
  if (cache) {
    cache->zs_choice = pc->zero_skip;
    cache->zs_dev = pc->device;
    cache->zs_prec = pc->interior_prec;
    cache->zs_chunks = pc->sweep_chunks;
    cache->zs_ilu = ilu_tol;
    cache->zs_ms = pc->tuned_ms;
  }
}

struct GmresWork {
  double *V, *Z, *w, *xp, *bp, *rp, *H, *g, *cs, *sn, *y, *pa, *pb, *scal;
  double *ca, *cb, *hc;  // CGS2 partial tables ((restart+1) x 1024 each) and coefficients
};

GmresWork gmres_work(addns_precond* pc, int restart, int flexible) {
  const int32_t N = pc->plan.N;
  if (pc->gm_restart < restart || !pc->V.p) {
    pc->V.alloc(sizeof(double) * (int64_t)(restart + 1) * N);
    pc->Z.alloc(sizeof(double) * (int64_t)restart * N);
    pc->w.alloc(sizeof(double) * N);
    pc->xp.alloc(sizeof(double) * N);
    pc->bp.alloc(sizeof(double) * N);
    pc->rp.alloc(sizeof(double) * N);
    const int ldh = restart + 1;
    pc->Hd.alloc(sizeof(double) * ((int64_t)ldh * restart + 4 * ldh));
    pc->partials.alloc(sizeof(double) * 2 * 1024);
    pc->cgs.alloc(sizeof(double) * ((int64_t)2 * ldh * 1024 + ldh));
    pc->scal.alloc(sizeof(double) * 8);
    pc->gm_restart = restart;
    if (!pc->host_pinned) ADDNS_HIP(hipHostMalloc(&pc->host_pinned, 64, hipHostMallocDefault));
  }
  (void)flexible;
  GmresWork g;
  const int ldh = pc->gm_restart + 1;
  g.V = pc->V.as<double>();
  g.Z = pc->Z.as<double>();
  g.w = pc->w.as<double>();
  g.xp = pc->xp.as<double>();
  g.bp = pc->bp.as<double>();
  g.rp = pc->rp.as<double>();
  g.H = pc->Hd.as<double>();
  g.g = g.H + (int64_t)ldh * pc->gm_restart;
  g.cs = g.g + ldh;
  g.sn = g.cs + ldh;
  g.y = g.sn + ldh;
  g.pa = pc->partials.as<double>();
  g.pb = g.pa + 1024;
  g.ca = pc->cgs.as<double>();
  g.cb = g.ca + (int64_t)ldh * 1024;
  g.hc = g.cb + (int64_t)ldh * 1024;
  g.scal = pc->scal.as<double>();
  return g;
}

double read_scalar(addns_precond* pc, const double* d, hipStream_t s) {
  double* h = static_cast<double*>(pc->host_pinned);
  ADDNS_HIP(hipMemcpyAsync(h, d, sizeof(double), hipMemcpyDeviceToHost, s));
  ADDNS_HIP(hipStreamSynchronize(s));
  return h[0];
}

}  // namespace

extern "C" {

int addns_setup_precond(addns_partition_t p, int32_t N, const int32_t* d_rowptr, const int32_t* d_colidx,
                        const double* d_vals, const addns_precond_opts* opts, void* stream, addns_precond_t* out) {
  return guarded("addns_setup_precond", [&]() -> int {
    if (!p || !out || !d_rowptr || !d_colidx || !d_vals) throw ArgError("null argument");
    if (N != p->d.N) throw ArgError("N does not match the partition");
    // buffers released since the last setup become reusable
    pool_sync();
    addns_precond_opts o{ADDNS_SCHUR_MSCN, ADDNS_F64, ADDNS_F64, 1, nullptr, 1, 0, 0, 0.0, 0, 0, 0, 0, 0};
    if (opts) o = *opts;
    if (o.overlap_segment < 0) throw ArgError("overlap_segment must be >= 0");
    if (o.block_sizing < 0 || o.block_sizing > 2) throw ArgError("block_sizing must be 0, 1 or 2");
    if (o.block_sizing == 0) {
      // With at most one interior per compute unit the sweep takes as long as
      // its longest chain of dependent steps, which a shared block size keeps
      // short; with more interiors than compute units the workgroups queue,
      // and the total work, which each interior's own size keeps small, counts.
      hipDeviceProp_t prop;
      int dev = 0;
      ADDNS_HIP(hipGetDevice(&dev));
      ADDNS_HIP(hipGetDeviceProperties(&prop, dev));
      o.block_sizing = p->d.m > prop.multiProcessorCount ? 2 : 1;
    }
    if (o.sweep_zero_skip < 0 || o.sweep_zero_skip > 2) throw ArgError("sweep_zero_skip must be 0, 1 or 2");
    if (o.coarse < 0 || o.coarse > 64) throw ArgError("coarse piece size must lie in 0..64");
    if (o.coarse > 0 && o.overlap > 0) throw ArgError("the coarse correction is built for non-overlapping aggregates");
    if (o.schur < 0 || o.schur > ADDNS_SCHUR_MSCNR) throw ArgError("unknown schur mode");
    if (o.overlap < 0) throw ArgError("overlap must be >= 0");
    if (o.overlap > 0 && o.schur != ADDNS_SCHUR_MSCN && o.schur != ADDNS_SCHUR_MSCNR && o.schur != ADDNS_SCHUR_LUM)
      throw ArgError("overlapped aggregates are defined for MSCN, MSCNR and LUM");
    if (o.block_mult < 0 || o.block_mult > 4) throw ArgError("block_mult must be 0..4");
    if (!(o.ilu_tol >= 0.0 && o.ilu_tol < 1.0)) throw ArgError("ilu_tol must lie in [0, 1)");
    if (o.sweep_chunks < 0) throw ArgError("sweep_chunks must be >= 0");
    const bool autotune = o.block_mult == 0;
    if (o.schur == ADDNS_SCHUR_LEARNED && !o.learned_model) throw ArgError("LEARNED mode needs learned_model");
    if (o.interior_prec != ADDNS_F64 && o.interior_prec != ADDNS_F32) throw ArgError("interior_prec");
    if (o.schur_prec < ADDNS_F64 || o.schur_prec > ADDNS_F16_SCALED) throw ArgError("schur_prec");
    if (o.schur == ADDNS_SCHUR_MSCN_LITERAL && p->d.n_int() < p->d.sep_size())
      throw ArgError("literal D-range pairing needs |D| >= |Sigma|");
    auto make = [&](int mult) {
      std::unique_ptr<addns_precond> pc(new addns_precond());
      pc->schur_mode = o.schur;
      pc->row_scale = o.row_scale;
      ADDNS_HIP(hipGetDevice(&pc->device));
      addns_precond_opts oo = o;
      oo.block_mult = mult;
      if (!p->cache) p->cache = std::make_shared<PlanCache>();
      // the chunk count from the plan model, and the chunked sweep's
      // responses built beside the coarse setup
      auto chunks = [&](hipStream_t cs) { choose_sweep_chunks(pc.get(), o.sweep_chunks, cs); };
      setup_device(pc.get(), &p->d, d_rowptr, d_colidx, d_vals, oo, as_stream(stream), p->cache.get(), chunks);
      pc->opts = oo;
      if (o.schur == ADDNS_SCHUR_LEARNED) {
        pc->learned_w.assign(o.learned_model, o.learned_model + mlp_param_count());
        pc->opts.learned_model = nullptr;  // the caller's array is not kept
      }
      // then the zero-slot form of the sweep that will run
      choose_zero_skip(pc.get(), o.sweep_zero_skip, o.ilu_tol, as_stream(stream), p->cache.get());
      pc->opts.sweep_chunks = pc->sweep_chunks;
      return pc;
    };
    // block_mult = 0: a fixed choice (1), not a timing: the sweep block size
    // regroups the same factors but changes the rounding of a solve
    *out = make(autotune ? 1 : o.block_mult).release();
    return ADDNS_OK;
  });
}

int addns_precond_refactor(addns_precond_t pc, const int32_t* d_rowptr, const int32_t* d_colidx,
                           const double* d_vals, void* stream) {
  return guarded("addns_precond_refactor", [&]() -> int {
    if (!pc || !d_rowptr || !d_colidx || !d_vals) throw ArgError("null argument");
    addns_precond_opts o = pc->opts;
    if (o.schur == ADDNS_SCHUR_LEARNED) o.learned_model = pc->learned_w.data();
    pc->valid = 0;
    // the chunk responses belong to the factors
    setup_device(pc, nullptr, d_rowptr, d_colidx, d_vals, o, as_stream(stream), nullptr, [&](hipStream_t cs) {
      if (pc->sweep_chunks > 1) build_chunked_sweep(pc, pc->sweep_chunks, cs);
    });
    pc->valid = 1;
    return ADDNS_OK;
  });
}

int addns_apply_precond(addns_precond_t pc, const double* d_y, double* d_x, void* stream) {
  return guarded("addns_apply_precond", [&]() -> int {
    if (!pc || !d_y || !d_x) throw ArgError("null argument");
    require_factors(pc);
    if (d_y == d_x) throw ArgError("y and x must not alias");
    hipStream_t s = as_stream(stream);
    const int32_t N = pc->plan.N;
    launch_permute(pc->perm.as<int32_t>(), d_y, pc->vperm_in.as<double>(), N, 0, nullptr, s);
    apply_permuted(pc, pc->vperm_in.as<double>(), pc->vperm_out.as<double>(), s);
    launch_permute(pc->perm.as<int32_t>(), pc->vperm_out.as<double>(), d_x, N, 1, nullptr, s);
    ADDNS_HIP(hipGetLastError());
    return ADDNS_OK;
  });
}

// Device address of `scratch` on device dev, looked up once per device
// with that device current.
static double* static_scratch(int dev) {
  static std::mutex mu;
  static double* ptr[256] = {};
  if (dev < 0 || dev >= 256) throw ArgError("device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    ADDNS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw HipError("hipGetSymbolAddress returned a null address for the static scratch");
    ptr[dev] = static_cast<double*>(p);
  }
  return ptr[dev];
}

int addns_apply_precond_static(addns_precond_t pc, const double* d_y, double* d_x, void* stream) {
  return guarded("addns_apply_precond_static", [&]() -> int {
    if (!pc || !d_y || !d_x) throw ArgError("null argument");
    require_factors(pc);
    if (d_y == d_x) throw ArgError("y and x must not alias");
    const Plan& pl = pc->plan;
    const int32_t N = pl.N;
    const int64_t npad = std::max<int64_t>(pl.npad_total, 1);
    const int64_t need = 2 * (int64_t)N + 2 * npad;
    if (need > kStaticScratchDoubles)
      throw ArgError("this system needs " + std::to_string(need) + " doubles of scratch; the static array holds " +
                     std::to_string(kStaticScratchDoubles) + " (use addns_apply_precond)");
    int dev = -1;
    ADDNS_HIP(hipGetDevice(&dev));
    if (dev != pc->device)
      throw ArgError("the current device (" + std::to_string(dev) + ") is not the handle's (" +
                     std::to_string(pc->device) + ")");
    double* w = static_scratch(dev);
    double* vin = w;
    double* vout = w + N;
    double* ypad = w + 2 * (int64_t)N;
    double* zpad = ypad + npad;
    hipStream_t s = as_stream(stream);
    launch_permute(pc->perm.as<int32_t>(), d_y, vin, N, 0, nullptr, s);
    apply_permuted(pc, vin, vout, s, ypad, zpad);
    launch_permute(pc->perm.as<int32_t>(), vout, d_x, N, 1, nullptr, s);
    ADDNS_HIP(hipGetLastError());
    return ADDNS_OK;
  });
}

int addns_interior_solve(addns_precond_t pc, const double* d_y1, double* d_z1, void* stream) {
  return guarded("addns_interior_solve", [&]() -> int {
    if (!pc || !d_y1 || !d_z1) throw ArgError("null argument");
    require_factors(pc);
    if (d_y1 == d_z1) throw ArgError("y1 and z1 must not alias");
    launch_interior_solve(pc, d_y1, d_z1, 0, nullptr, nullptr, as_stream(stream));
    ADDNS_HIP(hipGetLastError());
    return ADDNS_OK;
  });
}

int addns_gmres_solve(addns_precond_t pc, const double* d_b, double* d_x, const addns_gmres_opts* opts,
                      addns_gmres_result* res, void* stream) {
  return guarded("addns_gmres_solve", [&]() -> int {
    if (!pc || !d_b || !d_x || !opts || !res) throw ArgError("null argument");
    require_factors(pc);
    const int restart = opts->restart, maxit = opts->maxit;
    if (restart < 1 || restart > 1024 || maxit < 0 || !(opts->tol > 0.0))
      throw ArgError("1 <= restart <= 1024, maxit >= 0, tol > 0");
    if (opts->ortho != ADDNS_ORTHO_MGS && opts->ortho != ADDNS_ORTHO_CGS2) throw ArgError("unknown ortho");
    hipStream_t s = as_stream(stream);
    const int32_t N = pc->plan.N;
    const Plan& pl = pc->plan;
    GmresWork g = gmres_work(pc, restart, opts->flexible);
    const int ldh = pc->gm_restart + 1;
    const int nparts = krylov_grid(N);
    const int32_t* rp = pc->cp_rowptr.as<int32_t>();
    const int32_t* ci = pc->cp_colidx.as<int32_t>();
    const double* cv = pc->cp_vals.as<double>();
    double* hist = res->resid_hist;
    res->iters = 0;
    res->cycles = 0;
    res->converged = 0;
    res->true_relres = 0.0;
    res->est_relres = 0.0;
    // b~ = R b and x in the permuted numbering
    launch_permute(pc->perm.as<int32_t>(), d_b, g.bp, N, 0, pc->R.as<double>(), s);
    if (opts->use_x0) launch_permute(pc->perm.as<int32_t>(), d_x, g.xp, N, 0, nullptr, s);
    else ADDNS_HIP(hipMemsetAsync(g.xp, 0, sizeof(double) * N, s));
    launch_dot_partials(g.bp, g.bp, N, g.pa, s);
    launch_norm_finalize(g.pa, nparts, g.scal, 2, s);
    const double bnorm = read_scalar(pc, g.scal + 2, s);
    if (bnorm == 0.0) {
      ADDNS_HIP(hipMemsetAsync(d_x, 0, sizeof(double) * N, s));
      res->converged = 1;
      if (hist) hist[0] = 0.0;
      ADDNS_HIP(hipStreamSynchronize(s));
      return ADDNS_OK;
    }
    launch_residual(rp, ci, cv, g.xp, g.bp, g.rp, N, g.pa, s);
    launch_norm_finalize(g.pa, nparts, g.scal, 3, s);
    double beta = read_scalar(pc, g.scal + 3, s);
    double relres = beta / bnorm;
    int its = 0;
    bool converged = relres <= opts->tol;
    struct Events {
      hipEvent_t e[2] = {nullptr, nullptr};
      ~Events() {
        for (hipEvent_t x : e)
          if (x) (void)hipEventDestroy(x);
      }
    } ev;
    for (hipEvent_t& x : ev.e) ADDNS_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
    while (!converged && its < maxit) {
      res->cycles++;
      launch_scale_copy(g.rp, g.V, g.scal, 3, N, s);
      ADDNS_HIP(hipMemsetAsync(g.g, 0, sizeof(double) * ldh, s));
      ADDNS_HIP(hipMemcpyAsync(g.g, g.scal + 3, sizeof(double), hipMemcpyDeviceToDevice, s));
      int jdone = 0;
      // Iteration j's residual estimate is read only after iteration j + 1 is
      // queued, so the GPU never waits for the host between iterations.  An
      // iteration queued past the one that stops is discarded: it writes only
      // H(:, j), g[j], g[j+1], V[j+1] and Z[j], which the update below does not
      // read, so the result is that of stopping in place.
      double* hbuf = static_cast<double*>(pc->host_pinned) + 2;
      void* hdev = nullptr;  // the same pinned buffer as the device addresses it
      ADDNS_HIP(hipHostGetDevicePointer(&hdev, pc->host_pinned, 0));
      double* hbuf_dev = static_cast<double*>(hdev) + 2;
      auto queue_iteration = [&](int j) {
        double* vj = g.V + (int64_t)j * N;
        double* zj = opts->flexible ? g.Z + (int64_t)j * N : g.Z;
        apply_permuted(pc, vj, zj, s);
        double* pin = g.pa;
        int pnorm_parts = nparts;
        if (opts->ortho == ADDNS_ORTHO_CGS2) {
          // h = V^T w; w -= V h; c = V^T w; w -= V c; h += c (a fixed number of launches)
          double* hcol = g.H + (int64_t)j * ldh;
          const int cparts = cgs_parts(N);
          launch_spmv_dots(rp, ci, cv, zj, g.w, g.V, j + 1, N, g.ca, s);
          launch_cgs_coeffs(g.ca, cparts, j + 1, g.hc, hcol, 0, s);
          launch_cgs_update(g.w, g.V, j + 1, g.hc, N, g.cb, 0, s);
          launch_cgs_coeffs(g.cb, cparts, j + 1, g.hc, hcol, 1, s);
          launch_cgs_update(g.w, g.V, j + 1, g.hc, N, g.pa, 1, s);
          pnorm_parts = cparts;
        } else {
          launch_spmv_dot(rp, ci, cv, zj, g.w, g.V, N, g.pa, s);
          double* pout = g.pb;
          for (int i = 0; i <= j; ++i) {
            const double* vnext = i < j ? g.V + (int64_t)(i + 1) * N : nullptr;
            launch_mgs_step(g.w, g.V + (int64_t)i * N, vnext, N, pin, pout, g.H + (int64_t)j * ldh + i, nparts, s);
            std::swap(pin, pout);
          }
        }
        // the estimate goes straight to pinned host memory (no copy launch);
        // the same launch scales w into v_{j+1}
        launch_finalize(g.H, g.g, g.cs, g.sn, pin, pnorm_parts, j, ldh, g.scal, hbuf_dev + 2 * (j & 1), g.w,
                        g.V + (int64_t)(j + 1) * N, N, s);
        ADDNS_HIP(hipEventRecord(ev.e[j & 1], s));
      };
      // true: the cycle stops after iteration j
      auto finish_iteration = [&](int j) -> bool {
        ADDNS_HIP(hipEventSynchronize(ev.e[j & 1]));
        const double hn = hbuf[2 * (j & 1)], est = hbuf[2 * (j & 1) + 1];
        ++its;
        jdone = j + 1;
        res->est_relres = est / bnorm;
        if (hist) hist[its - 1] = est / bnorm;
        if (!std::isfinite(est)) throw HipError("non-finite residual estimate");
        return est <= opts->tol * bnorm || its >= maxit || hn == 0.0;
      };
      for (int j = 0; j < restart; ++j) {
        queue_iteration(j);
        if (j > 0 && finish_iteration(j - 1)) break;
        if (j == restart - 1) {
          finish_iteration(j);
          break;
        }
      }
      launch_backsolve(g.H, g.g, jdone, ldh, g.y, s);
      if (opts->flexible) {
        launch_combine(g.Z, N, g.y, jdone, N, g.xp, 1, s);
      } else {
        launch_combine(g.V, N, g.y, jdone, N, g.w, 0, s);
        apply_permuted(pc, g.w, g.Z, s);
        launch_combine(g.Z, N, nullptr, 1, N, g.xp, 1, s);
      }
      launch_residual(rp, ci, cv, g.xp, g.bp, g.rp, N, g.pa, s);
      launch_norm_finalize(g.pa, nparts, g.scal, 3, s);
      beta = read_scalar(pc, g.scal + 3, s);
      relres = beta / bnorm;
      converged = relres <= opts->tol;
    }
    launch_permute(pc->perm.as<int32_t>(), g.xp, d_x, N, 1, nullptr, s);
    ADDNS_HIP(hipStreamSynchronize(s));
    (void)pl;
    res->iters = its;
    res->converged = converged ? 1 : 0;
    res->true_relres = relres;
    if (!converged) {
      set_error("GMRES reached maxit with relative residual " + std::to_string(relres));
      return ADDNS_ERR_NOCONV;
    }
    return ADDNS_OK;
  });
}

int addns_gmres_solve_batched(addns_precond_t pc, int32_t nsys, const int32_t* sys_offsets, const double* d_b,
                              double* d_x, const addns_gmres_opts* opts, addns_gmres_result* res, void* stream) {
  return guarded("addns_gmres_solve_batched", [&]() -> int {
    if (!pc || !sys_offsets || !d_b || !d_x || !opts || !res || nsys < 1) throw ArgError("null argument");
    require_factors(pc);
    const int restart = opts->restart, maxit = opts->maxit;
    if (restart < 1 || restart > 1024 || maxit < 0 || !(opts->tol > 0.0))
      throw ArgError("1 <= restart <= 1024, maxit >= 0, tol > 0");
    if (!opts->flexible) throw ArgError("the batched solver is flexible GMRES only");
    if (opts->ortho != ADDNS_ORTHO_MGS) throw ArgError("the batched solver orthogonalises by MGS (ortho = 0)");
    const Plan& pl = pc->plan;
    const int32_t N = pl.N;
    if (sys_offsets[0] != 0 || sys_offsets[nsys] != N) throw ArgError("sys_offsets must run from 0 to N");
    for (int32_t q = 0; q < nsys; ++q)
      if (sys_offsets[q + 1] <= sys_offsets[q]) throw ArgError("sys_offsets must be increasing");
    hipStream_t s = as_stream(stream);
    // rows of every system in the permuted numbering, as contiguous chunks
    std::vector<int32_t> sys_of(N);
    for (int32_t q = 0; q < nsys; ++q)
      for (int32_t o = sys_offsets[q]; o < sys_offsets[q + 1]; ++o) sys_of[pl.iperm[o]] = q;
    std::vector<std::vector<Chunk>> per(nsys);
    const int32_t cmax = seg_chunk_rows();
    for (int32_t r = 0; r < N;) {
      int32_t q = sys_of[r], e = r;
      while (e < N && sys_of[e] == q && e - r < cmax) ++e;
      per[q].push_back(Chunk{r, e, q});
      r = e;
    }
    std::vector<Chunk> chunks;
    std::vector<int32_t> coff(1, 0);
    for (int32_t q = 0; q < nsys; ++q) {
      chunks.insert(chunks.end(), per[q].begin(), per[q].end());
      coff.push_back((int32_t)chunks.size());
    }
    const int nch = (int)chunks.size();
    DevBuf d_ch, d_coff, d_live, d_jdone, state, parts, scal;
    d_ch.upload(chunks, s);
    d_coff.upload(coff, s);
    d_live.alloc(sizeof(int32_t) * nsys);
    // the apply skips the subdomains, aggregates and coarse groups of the
    // systems that have converged: their system ids, and the live flags
    // below, stay on the handle for the duration of the solve
    {
      std::vector<int32_t> sub_sys(std::max(pl.m, 1), 0), agg_sys(std::max(pl.k, 1), 0);
      for (int32_t j = 0; j < pl.m; ++j)
        if (pl.subs[j].n > 0) sub_sys[j] = sys_of[pl.subs[j].int_off];
      for (int32_t i = 0; i < pl.k; ++i)
        if (pl.agg_off[i + 1] > pl.agg_off[i]) agg_sys[i] = sys_of[pl.n_int + pl.agg_off[i]];
      const CoarsePlan& cp = pc->coarse;
      std::vector<int32_t> grp_sys(std::max<size_t>(cp.grp_col0.size(), 1), 0);
      for (size_t g = 0; g + 1 < cp.grp_off.size(); ++g)
        if (cp.grp_off[g + 1] > cp.grp_off[g]) grp_sys[g] = sys_of[pl.n_int + cp.grp_rows[cp.grp_off[g]]];
      pc->mask_sub.upload(sub_sys, s);
      pc->mask_agg.upload(agg_sys, s);
      pc->mask_grp.upload(grp_sys, s);
      ADDNS_HIP(hipStreamSynchronize(s));  // the host vectors end with this block
    }
    struct MaskGuard {
      addns_precond* pc;
      ~MaskGuard() { pc->mask_live = nullptr; }
    } mask_guard{pc};
    pc->mask_live = d_live.as<int32_t>();
    d_jdone.alloc(sizeof(int32_t) * nsys);
    const int ldh = restart + 1;
    const int64_t st = (int64_t)ldh * restart + 4 * ldh;
    state.alloc(sizeof(double) * st * nsys);
    ADDNS_HIP(hipMemsetAsync(state.p, 0, sizeof(double) * st * nsys, s));
    parts.alloc(sizeof(double) * 2 * nch);
    scal.alloc(sizeof(double) * 4 * nsys);
    GmresWork g = gmres_work(pc, restart, 1);
    double* pa = parts.as<double>();
    double* pb = pa + nch;
    double* sc = scal.as<double>();
    const int32_t* rp = pc->cp_rowptr.as<int32_t>();
    const int32_t* ci = pc->cp_colidx.as<int32_t>();
    const double* cv = pc->cp_vals.as<double>();
    std::vector<int32_t> live(nsys, 1), active(nsys, 0), jdone(nsys, 0), its(nsys, 0), conv(nsys, 0), cyc(nsys, 0);
    std::vector<double> h_sc(4 * nsys), bnorm(nsys), relres(nsys);
    auto put = [&](DevBuf& d, const std::vector<int32_t>& h) {
      ADDNS_HIP(hipMemcpyAsync(d.p, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, s));
    };
    auto get_scal = [&]() {
      ADDNS_HIP(hipMemcpyAsync(h_sc.data(), sc, sizeof(double) * 4 * nsys, hipMemcpyDeviceToHost, s));
      ADDNS_HIP(hipStreamSynchronize(s));
    };
    launch_permute(pc->perm.as<int32_t>(), d_b, g.bp, N, 0, pc->R.as<double>(), s);
    if (opts->use_x0) launch_permute(pc->perm.as<int32_t>(), d_x, g.xp, N, 0, nullptr, s);
    else ADDNS_HIP(hipMemsetAsync(g.xp, 0, sizeof(double) * N, s));
    put(d_live, live);
    launch_seg_dot(g.bp, g.bp, d_ch.as<Chunk>(), nch, pa, s);
    launch_seg_norm(pa, d_coff.as<int32_t>(), nullptr, nsys, sc, 2, s);
    launch_seg_residual(rp, ci, cv, g.xp, g.bp, g.rp, d_ch.as<Chunk>(), nch, d_live.as<int32_t>(), pa, s);
    launch_seg_norm(pa, d_coff.as<int32_t>(), nullptr, nsys, sc, 3, s);
    get_scal();
    for (int32_t q = 0; q < nsys; ++q) {
      bnorm[q] = h_sc[4 * q + 2];
      relres[q] = bnorm[q] > 0.0 ? h_sc[4 * q + 3] / bnorm[q] : 0.0;
      conv[q] = relres[q] <= opts->tol;
      active[q] = !conv[q] && maxit > 0;
    }
    auto any = [](const std::vector<int32_t>& v) {
      for (int32_t x : v)
        if (x) return true;
      return false;
    };
    while (any(active)) {
      put(d_live, active);
      for (int32_t q = 0; q < nsys; ++q) {
        jdone[q] = 0;
        if (active[q]) cyc[q]++;
      }
      launch_seg_scale_copy(g.rp, g.V, sc, 3, d_ch.as<Chunk>(), nch, d_live.as<int32_t>(), s);
      launch_seg_init_g(state.as<double>(), st, d_live.as<int32_t>(), nsys, ldh, restart, sc, 3, s);
      std::vector<int32_t> lv = active;
      for (int j = 0; j < restart && any(lv); ++j) {
        put(d_live, lv);
        double* vj = g.V + (int64_t)j * N;
        double* zj = g.Z + (int64_t)j * N;
        apply_permuted(pc, vj, zj, s);
        launch_seg_spmv_dot(rp, ci, cv, zj, g.w, g.V, d_ch.as<Chunk>(), nch, d_live.as<int32_t>(), pa, s);
        double* pin = pa;
        double* pout = pb;
        for (int i = 0; i <= j; ++i) {
          const double* vnext = i < j ? g.V + (int64_t)(i + 1) * N : nullptr;
          launch_seg_mgs_step(g.w, g.V + (int64_t)i * N, vnext, d_ch.as<Chunk>(), nch, d_coff.as<int32_t>(),
                              d_live.as<int32_t>(), pin, pout, state.as<double>(), st, (int64_t)j * ldh + i, s);
          std::swap(pin, pout);
        }
        launch_seg_finalize(state.as<double>(), st, pin, d_coff.as<int32_t>(), d_live.as<int32_t>(), nsys, j, ldh,
                            restart, sc, s);
        launch_seg_scale_copy(g.w, g.V + (int64_t)(j + 1) * N, sc, 0, d_ch.as<Chunk>(), nch, d_live.as<int32_t>(), s);
        get_scal();
        for (int32_t q = 0; q < nsys; ++q) {
          if (!lv[q]) continue;
          const double hn = h_sc[4 * q], est = h_sc[4 * q + 1];
          its[q]++;
          jdone[q] = j + 1;
          res[q].est_relres = est / bnorm[q];
          if (res[q].resid_hist) res[q].resid_hist[its[q] - 1] = est / bnorm[q];
          if (!std::isfinite(est)) throw HipError("non-finite residual estimate in system " + std::to_string(q));
          if (est <= opts->tol * bnorm[q] || its[q] >= maxit || hn == 0.0) lv[q] = 0;
        }
      }
      put(d_jdone, jdone);
      put(d_live, active);
      launch_seg_backsolve(state.as<double>(), st, d_jdone.as<int32_t>(), nsys, ldh, restart, s);
      launch_seg_combine(g.Z, N, state.as<double>(), st, d_jdone.as<int32_t>(), ldh, restart, d_ch.as<Chunk>(), nch,
                         g.xp, s);
      launch_seg_residual(rp, ci, cv, g.xp, g.bp, g.rp, d_ch.as<Chunk>(), nch, d_live.as<int32_t>(), pa, s);
      launch_seg_norm(pa, d_coff.as<int32_t>(), d_live.as<int32_t>(), nsys, sc, 3, s);
      get_scal();
      for (int32_t q = 0; q < nsys; ++q) {
        if (!active[q]) continue;
        relres[q] = h_sc[4 * q + 3] / bnorm[q];
        conv[q] = relres[q] <= opts->tol;
        if (conv[q] || its[q] >= maxit) active[q] = 0;
      }
    }
    launch_permute(pc->perm.as<int32_t>(), g.xp, d_x, N, 1, nullptr, s);
    ADDNS_HIP(hipStreamSynchronize(s));
    bool all = true;
    for (int32_t q = 0; q < nsys; ++q) {
      res[q].iters = its[q];
      res[q].cycles = cyc[q];
      res[q].converged = conv[q];
      res[q].true_relres = relres[q];
      all = all && conv[q];
    }
    if (!all) {
      set_error("some systems reached maxit above tol");
      return ADDNS_ERR_NOCONV;
    }
    return ADDNS_OK;
  });
}

int addns_precond_info(addns_precond_t pc, int32_t* kl, int32_t* ku, int32_t* nb_lower, int32_t* nb_upper,
                       int64_t* factor_bytes, int64_t* bytes_apply, int64_t* learned_count, int32_t* block_mult,
                       int64_t* interior_nnz, int32_t* sweep_chunks, int64_t* chunk_bytes, int64_t* band_words) {
  if (!pc) {
    set_error("addns_precond_info: null handle");
    return ADDNS_ERR_ARG;
  }
  if (kl) *kl = pc->plan.KL;
  if (ku) *ku = pc->plan.KU;
  if (nb_lower) *nb_lower = pc->plan.nbL;
  if (nb_upper) *nb_upper = pc->plan.nbU;
  if (factor_bytes) *factor_bytes = pc->factor_bytes;
  if (bytes_apply) *bytes_apply = pc->bytes_apply + 2 * pc->chunk_bytes;
  if (learned_count) *learned_count = pc->learned_count;
  if (block_mult) *block_mult = pc->plan.block_mult;
  if (interior_nnz) *interior_nnz = pc->interior_nnz;
  if (sweep_chunks) *sweep_chunks = pc->sweep_chunks;
  if (chunk_bytes) *chunk_bytes = pc->chunk_bytes;
  if (band_words) {
    int64_t w = 0;
    for (const SubInfo& q : pc->plan.subs) w += (int64_t)q.n * (2 * q.kl + q.ku + 1);
    *band_words = w;
  }
  return ADDNS_OK;
}

int addns_precond_fill(addns_precond_t pc, int64_t* nnz_precond, int64_t* nnz_c) {
  if (!pc) {
    set_error("addns_precond_fill: null handle");
    return ADDNS_ERR_ARG;
  }
  const Plan& pl = pc->plan;
  int64_t shat = 0;
  for (int32_t i = 0; i < pl.k; ++i) shat += (int64_t)pl.agg_s[i] * pl.agg_s[i];
  if (pl.overlap > 0) shat += pl.l_off[pl.k];
  if (nnz_precond)
    *nnz_precond = pc->interior_nnz + shat + (int64_t)pl.e_src.size() + (int64_t)pl.f_src.size();
  if (nnz_c) *nnz_c = (int64_t)pl.cp_colidx.size();
  return ADDNS_OK;
}

int addns_precond_schur_blocks(addns_precond_t pc, double* h_out, int64_t count) {
  return guarded("addns_precond_schur_blocks", [&]() -> int {
    if (!pc || !h_out) throw ArgError("null argument");
    require_factors(pc);
    if (count != pc->plan.g_total) throw ArgError("count must equal the sum of |agg_i|^2");
    if (count > 0) ADDNS_HIP(hipMemcpy(h_out, pc->schur_S.p, sizeof(double) * count, hipMemcpyDeviceToHost));
    return ADDNS_OK;
  });
}

void addns_precond_destroy(addns_precond_t pc) { delete pc; }

int64_t addns_release_cached_memory(void) { return (int64_t)pool_trim(); }

}  // extern "C"
