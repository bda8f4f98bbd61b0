// Internal state of a preconditioner handle and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "internal.h"

namespace addns {

#define ADDNS_HIP(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      throw HipError(std::string(#call) + ": " + hipGetErrorString(e_));             \
    }                                                                                \
  } while (0)

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct SingularError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// Owning device buffer.
// Caching device allocator (device_pool.cpp): blocks released to a
// per-device pool are reused only after a device synchronisation that
// followed their release (pool_sync, at the start of every allocating entry
// point); pool_trim gives every cached block back (returns the bytes).
void* pool_alloc(size_t n, size_t* cap, int* dev);
void pool_free(void* p, size_t cap, int dev);
void pool_sync();
size_t pool_trim();

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;  // requested size
  size_t cap = 0;    // size of the block behind p (>= bytes)
  int dev = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { reset(); }
  void reset() {
    if (p) pool_free(p, cap, dev);
    p = nullptr;
    bytes = cap = 0;
  }
  // keeps the allocation (and its address) when the size is unchanged, so
  // that a refactor on the same plan leaves every device pointer in place
  void alloc(size_t n) {
    if (n == 0) n = 8;
    if (p && bytes == n) return;
    reset();
    p = pool_alloc(n, &cap, &dev);
    bytes = n;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
  template <class T>
  void upload(const std::vector<T>& v, hipStream_t s) {
    alloc(v.size() * sizeof(T));
    if (!v.empty()) ADDNS_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  // a device-side copy of another buffer (same size)
  void copy_from(const DevBuf& o, hipStream_t s) {
    alloc(o.bytes);
    ADDNS_HIP(hipMemcpyAsync(p, o.p, o.bytes, hipMemcpyDeviceToDevice, s));
  }
};

// Per-subdomain sweep geometry (POD, shared by host and device).
struct SubInfo {
  int32_t n, npad;        // interior size and padded size (multiple of nbu)
  int32_t kl, ku;         // lower / upper bandwidth of A_jj
  int32_t nbl, nbu;       // lower / upper block sizes (nbu = 2 nbl >= kl + ku, nbl >= kl)
  int32_t ldab;           // band storage leading dimension 2 kl + ku + 1
  int32_t vec_off;        // offset into padded work vectors (and pivots)
  int32_t int_off;        // offset of the interior in the permuted numbering
  int32_t lblk0, ublk0;   // first lower / upper block
  int32_t pad_;
  int64_t band_off;       // offset of the band storage (elements)
  int64_t lmat_off;       // first lower block matrix (elements); blocks are W x nbl each
  int64_t lperm_off;      // first lower block gather indices; W each
  int64_t u_off;          // first upper block (elements); nbu x nbu each
};
struct LBlk {             // one lower block: W = nbl + kl window rows
  int32_t sub, idx;
  int64_t moff;           // offset of [inv(L11); L21 inv(L11)] (W x nbl, elements)
  int64_t poff;           // offset of the window gather indices (W)
  int64_t woff;           // conversion work offset (W nbl + nbl nbl doubles)
};
struct UBlk {             // one upper block: nbu x nbu inverse and coupling
  int32_t sub, idx;
  int64_t off;            // offset into inv(U_bb) and U_{b,b+1} (elements); also work offset
};

// A contiguous row range of one system (segmented Krylov reductions).
struct Chunk {
  int32_t start, end, sys;
};

// Host-side integer plan: every gather map the device setup needs.  Built
// from the partition and the pattern only.
struct Plan {
  int32_t N = 0, m = 0, k = 0, n_int = 0, nsep = 0;
  int32_t KL = 0, KU = 0;     // largest interior bandwidths (reported)
  int32_t nbL = 0, nbU = 0;   // largest block sizes
  int32_t maxW = 0;           // largest lower window nbl + kl
  int32_t block_mult = 1;     // lower block size = block_mult x its minimum
  bool per_interior = false;  // block sizes per interior (else one for all)
  // permuted CSR of C~ (new numbering) and the source entry of each value
  std::vector<int32_t> cp_rowptr, cp_colidx, cp_src, cp_orow;
  std::vector<int32_t> perm, iperm;
  // interior blocks
  std::vector<SubInfo> subs;
  std::vector<LBlk> lblks;
  std::vector<UBlk> ublks;
  int64_t band_total = 0, npad_total = 0, lmat_total = 0, lperm_total = 0, lwork_total = 0, u_total = 0;
  std::vector<int64_t> band_dst;                 // band element index per interior C~p entry
  std::vector<int32_t> band_src;                 //   ... and its C~p entry
  // E (interior rows x separator cols) and F (separator rows x interior cols), CSR
  std::vector<int32_t> e_rowptr, e_colidx, e_src;
  std::vector<int32_t> f_rowptr, f_colidx, f_src;
  // dense Schur blocks (aggregate i: s_i = |agg|, d_i = |D-range|)
  std::vector<int32_t> agg_off, agg_s, agg_d;    // agg_off: k+1 separator positions
  std::vector<int64_t> g_off, dd_off, de_off, df_off, sinv_off;  // element offsets
  // overlapped aggregates: width w_i, extended size e_i = s_i + w_i (the
  // dense G/E/F blocks are e_i wide), the lower blocks L_i (w_i x s_i) of
  // Shat and the chain matrices M_i = A_i^{-1} [L_{i-1}; 0] (s_i x s_{i-1},
  // rows stored ovl_width wide, zero-padded)
  int32_t overlap = 0, ovl_width = 0;
  std::vector<int32_t> agg_w, agg_e;
  std::vector<int64_t> l_off, m_off;
  std::vector<int64_t> dense_dst;                // scratch element index
  std::vector<int32_t> dense_src;                // C~p entry
  int64_t g_total = 0, dd_total = 0, de_total = 0, df_total = 0;
  // exact block-Jacobi interface blocks: (subdomain, separator column) solves
  std::vector<int32_t> agg_of;                   // per separator position
  std::vector<int32_t> pair_sub, pair_col, pcol_ptr;
  std::vector<int64_t> pair_off;
  int64_t pair_total = 0;
  // learned interface correction: one sample per separator velocity row;
  // five stencil slots [far lower, near lower, diagonal, near upper, far upper]
  std::vector<int32_t> smp_row;                  // permuted row index
  std::vector<int32_t> smp_nb;                   // 5 per sample: permuted column or -1
  std::vector<int64_t> smp_loc;                  // 5 per sample: element of the dense G/S block or -1
};

// per_interior: each interior's own lower block size (else the widest band's
// for all)
void build_plan(const PartitionData& P, Plan& pl, int schur_mode, int block_mult, int overlap,
                bool per_interior);

// Coarse space of the two-level interface solve: pieces of at most `piece`
// separator velocity nodes, one constant and (pieces of three nodes or
// more) one linear column each.  Positions are separator positions.
struct CoarseSpace {
  int32_t piece = 0, npieces = 0, nc = 0;
  std::vector<int32_t> piece_off, piece_pos;      // pieces, members in joining order
  std::vector<int32_t> col_piece, col_kind;       // per column: piece, 0 constant / 1 linear
  std::vector<int32_t> piece_col0, piece_col1;    // per piece: its columns (-1 if none)
  std::vector<int32_t> node_piece;                // per separator position (-1: pressure-like)
  std::vector<double> node_z0, node_z1;           // per position: constant and linear values
};
// Device plan of the coarse correction.
struct CoarsePlan {
  CoarseSpace space;
  std::vector<int32_t> sub_of;                    // subdomain of every interior row
  // (subdomain, coarse column) solves D_j^{-1} E_j z_c, ordered by column
  std::vector<int32_t> pair_sub, pair_col, cpair_ptr;
  std::vector<int64_t> pair_off;
  int64_t pair_total = 0;
  // row pattern of S Z (CSR over separator rows, coarse columns ascending)
  std::vector<int32_t> sz_rowptr, sz_col;
  // restriction groups (<= 64 rows each): the pieces, then the other rows
  std::vector<int32_t> grp_off, grp_rows, grp_col0, grp_col1;
  std::vector<int32_t> grp_coff, grp_cols;        // per group: the columns of S Z on its rows, ascending
  // E_c is block diagonal over runs of coarse columns that no entry couples
  // (for concatenated systems, at least one block per system): block b holds
  // columns [blk_off[b], blk_off[b+1]) and its dense inverse starts at
  // element blk_eoff[b]
  std::vector<int32_t> blk_off, col_blk;
  std::vector<int64_t> blk_eoff;
  int32_t blk_max = 0;
};
void build_coarse_space(const PartitionData& P, int32_t piece, CoarseSpace& cs);
void build_coarse_plan(const PartitionData& P, const Plan& pl, int32_t piece, CoarsePlan& cp);

// Host plans of one partition, keyed by the options they depend on.
// Device copies of a plan's gather and scatter maps (the setup's index
// arrays that do not depend on the matrix values).
struct PlanMaps {
  DevBuf cp_src, cp_orow, e_src, f_src, band_dst, band_src, dense_dst, dense_src;
  // the plan's structure that every handle keeps a copy of
  DevBuf perm, iperm, cp_rowptr, cp_colidx, e_rowptr, e_colidx, f_rowptr, f_colidx, subs, lblks, ublks;
  void upload(const Plan& pl, hipStream_t s) {
    perm.upload(pl.perm, s);
    iperm.upload(pl.iperm, s);
    cp_rowptr.upload(pl.cp_rowptr, s);
    cp_colidx.upload(pl.cp_colidx, s);
    e_rowptr.upload(pl.e_rowptr, s);
    e_colidx.upload(pl.e_colidx, s);
    f_rowptr.upload(pl.f_rowptr, s);
    f_colidx.upload(pl.f_colidx, s);
    subs.upload(pl.subs, s);
    lblks.upload(pl.lblks, s);
    ublks.upload(pl.ublks, s);
    cp_src.upload(pl.cp_src, s);
    cp_orow.upload(pl.cp_orow, s);
    e_src.upload(pl.e_src, s);
    f_src.upload(pl.f_src, s);
    band_dst.upload(pl.band_dst, s);
    band_src.upload(pl.band_src, s);
    dense_dst.upload(pl.dense_dst, s);
    dense_src.upload(pl.dense_src, s);
  }
};

// Device copies of a coarse plan's arrays: those every handle keeps a copy
// of, and the (subdomain, column) pair lists of the setup's column solves.
struct CoarseMaps {
  DevBuf piece, z0, z1, colp, colk, p0, p1, szp, szc, goff, grows, gc0, gc1, gcoff, gcols, boff, cblk, beoff;
  DevBuf psub, pcol, poff, cpp, subof, ioff;
  void upload(const CoarsePlan& cp, const Plan& pl, hipStream_t s) {
    const CoarseSpace& z = cp.space;
    piece.upload(z.node_piece, s);
    z0.upload(z.node_z0, s);
    z1.upload(z.node_z1, s);
    colp.upload(z.col_piece, s);
    colk.upload(z.col_kind, s);
    p0.upload(z.piece_col0, s);
    p1.upload(z.piece_col1, s);
    szp.upload(cp.sz_rowptr, s);
    szc.upload(cp.sz_col, s);
    goff.upload(cp.grp_off, s);
    grows.upload(cp.grp_rows, s);
    gc0.upload(cp.grp_col0, s);
    gc1.upload(cp.grp_col1, s);
    gcoff.upload(cp.grp_coff, s);
    gcols.upload(cp.grp_cols, s);
    boff.upload(cp.blk_off, s);
    cblk.upload(cp.col_blk, s);
    beoff.upload(cp.blk_eoff, s);
    psub.upload(cp.pair_sub, s);
    pcol.upload(cp.pair_col, s);
    poff.upload(cp.pair_off, s);
    cpp.upload(cp.cpair_ptr, s);
    subof.upload(cp.sub_of, s);
    std::vector<int32_t> int_off(pl.m);
    for (int32_t j = 0; j < pl.m; ++j) int_off[j] = pl.subs[j].int_off;
    ioff.upload(int_off, s);
  }
};

struct PlanCache {
  bool have_plan = false, have_coarse = false;
  int schur = -1, block_mult = -1, overlap = -1, piece = -1, per_interior = -1;
  Plan plan;
  CoarsePlan coarse;
  // the plan's maps on device maps_dev (-1: none yet, or the plan changed):
  // a repeated setup of the same partition does not upload them again
  int maps_dev = -1;
  PlanMaps maps;
  // the timed zero-slot choice of the sweep on this plan (-1: none yet),
  // with the interior precision, chunk count and ILU drop tolerance it was
  // timed for
  // the coarse plan's arrays on device cmaps_dev (-1: none yet, or the
  // coarse plan changed)
  int cmaps_dev = -1;
  CoarseMaps cmaps;
  int zs_choice = -1, zs_prec = -1, zs_chunks = -1, zs_dev = -1;
  double zs_ilu = -1.0;
  float zs_ms = 0.0f;
};

// Largest coarse space the two-level interface solve accepts (its dense
// inverse is nc^2 FP64 and its Gauss-Jordan setup takes 2 nc launches).
constexpr int32_t kMaxCoarseColumns = 8192;

// Bytes past the end of each interior factor array that the sweep may read
// (its last row slot can overrun a block by up to 64 * 5 - 1 FP64 rows).
constexpr int64_t kSweepOverrunBytes = 4096;
constexpr int kSweepMaxSlots = 5;  // row slots of 64 rows per wave in a sweep GEMV
static_assert(kSweepOverrunBytes >= (64 * kSweepMaxSlots - 1) * (int64_t)sizeof(double),
              "the zeroed tail must cover the largest row-slot overrun");

// Largest aggregate count of the overlapped interface solve (its chain
// keeps 12 bytes per aggregate in LDS).
constexpr int32_t kMaxOverlapAggregates = 12000;

// Storage precision tags
enum Prec { P64 = 0, P32 = 1, P16S = 2 };

}  // namespace addns

struct addns_precond {
  addns::Plan plan;
  int schur_mode = 0, interior_prec = 0, schur_prec = 0, row_scale = 1;
  addns_precond_opts opts{};                          // as set up (block_mult: the one in use)
  std::vector<float> learned_w;                       // LEARNED: the network weights, for refactors
  int valid = 1;                                      // 0 after a failed refactor: no usable factors
  int device = 0;
  // vectors / matrices (device)
  addns::DevBuf perm, iperm, R;                       // R in original numbering
  addns::DevBuf cp_rowptr, cp_colidx, cp_vals;        // C~ permuted (fp64)
  addns::DevBuf e_rowptr, e_colidx, e_vals, f_rowptr, f_colidx, f_vals;
  // interior factors in block form
  addns::DevBuf subs, lblks, ublks;                   // SubInfo / LBlk / UBlk tables
  addns::DevBuf lperm;                                // per L-block window gather indices
  addns::DevBuf lmat;                                 // per L-block [inv(L11); L21 inv(L11)]
  addns::DevBuf uinv, u12;                            // per U-block
  // interface
  addns::DevBuf agg_off, agg_s, sinv_off, sinv, sinv_scale, schur_S;
  // overlapped aggregates: chain matrices M_i (FP64 with FP64 interface
  // storage, else FP32) applied by the block forward substitution over Shat
  addns::DevBuf ovl_m, ovl_moff;
  int overlap_chain = 0;                              // 0: none, else the chain matrices' row width (64, 80, 128)
  addns::DevBuf ovl_q;                                // segment responses Q_i (same layout as M_i)
  int32_t ovl_seg = 1;                                // chain segment length L
  // scratch
  addns::DevBuf ypad, zpad, z1, x2tmp;                // padded interior work vectors
  addns::DevBuf vperm_in, vperm_out;                  // permuted apply in/out
  int64_t factor_bytes = 0, bytes_apply = 0;
  int64_t interior_nnz = 0;                           // stored entries of the interior L and U factors
  int64_t learned_count = 0;
  float tuned_ms = 0.0f;                              // autotuner timing of the interior solve
  int zero_skip = 0;                                  // sweep skips structural-zero row slots (autotuned)
  // chunked interior sweep: p chunks per interior swept side by side, joined
  // through each chunk's response to its incoming carry (lower) or state
  // (upper); per (subdomain, chunk) the offsets of X_c, LP_c, Y_c, UP_c
  int sweep_chunks = 1, ch_klmax = 0;
  int64_t chunk_bytes = 0;                            // response matrices, read once per interior solve
  addns::DevBuf ch_off, ch_lx, ch_lp, ch_uy, ch_up;   // offsets (int64) and response matrices
  addns::DevBuf ch_cz, ch_xs, ch_uin;                 // zero-state carries and upper outputs, E x2
  addns::DevBuf ch_nz, ch_nzo;                        // coupling columns of the chunk boundaries
  addns::DevBuf ch_prow, ch_np, ch_npo;               // pure carry rows and coupled carry positions
  addns::DevBuf g_copy;                               // G blocks before the update (learning targets S - G)
  // coarse-grid correction of the interface solve (opts.coarse > 0)
  addns::CoarsePlan coarse;
  int32_t coarse_nc = 0;
  addns::DevBuf cz_piece, cz_z0, cz_z1, cz_colp, cz_colk, cz_p0, cz_p1;   // per position / column / piece
  addns::DevBuf cz_szp, cz_szc, cz_szv;              // S Z, CSR over separator rows
  addns::DevBuf cz_einv;                              // (Z^T S Z)^{-1}, nc x nc row-major FP64
  addns::DevBuf cz_goff, cz_grows, cz_gc0, cz_gc1;    // restriction groups
  addns::DevBuf cz_gcoff, cz_gcols;                   //   and their S Z column lists
  addns::DevBuf cz_boff, cz_cblk, cz_beoff;            // blocks of E_c
  addns::DevBuf cz_t, cz_g, cz_y;                     // apply scratch: t, Z^T t, y
  // while a batched solve runs: per-system live flags (device) and the
  // system of every subdomain, aggregate and restriction group; the apply
  // kernels then skip the work units of systems that have converged
  const int32_t* mask_live = nullptr;
  addns::DevBuf mask_sub, mask_agg, mask_grp;
  addns::DevBuf smp_row, smp_nb, smp_loc;             // learned-correction sample table
  // GMRES work space (grown on demand)
  addns::DevBuf V, Z, w, xp, bp, rp, Hd, gd, partials, scal;
  addns::DevBuf cgs;                                  // CGS2: two (restart+1) x 1024 partial tables and h
  int gm_restart = 0;
  void* host_pinned = nullptr;
  ~addns_precond() {
    if (host_pinned) (void)hipHostFree(host_pinned);
  }
};

namespace addns {
inline void require_factors(const addns_precond* pc) {
  if (!pc->valid) throw ArgError("the handle holds no factors: its last refactor failed");
}

// launchers (kernels_*.hip)
void launch_row_scale(const int32_t* rowptr, const double* vals, int32_t N, int scale, double* R,
                      hipStream_t s);
void launch_gather_scaled(const int32_t* src, const int32_t* orow, const double* vals, const double* R,
                          int64_t n, double* out, hipStream_t s);
void launch_gather(const int32_t* src, const double* in, int64_t n, double* out, hipStream_t s);
void launch_scatter_band(const int64_t* dst, const int32_t* src, const double* cpv, int64_t n, double* ab,
                         hipStream_t s);
void launch_band_pad_identity(const SubInfo* subs, int32_t m, double* ab, hipStream_t s);
// Every padded interior size is a multiple of this (block sizes are multiples
// of 8 and the upper block is twice the lower one); the blocked band LU's
// panels of 8 columns rely on it.
constexpr int32_t kNpadMultiple = 16;
void launch_band_lu(double* ab, int32_t* ipiv, const SubInfo* subs, int32_t m, int32_t* info, const double* colnorm,
                    double tau, int32_t kl_max, int32_t kv_max, const int32_t* sub_list, hipStream_t s);
// true when bands of at most kl_max take the blocked LU (which takes subdomain
// lists: m workgroups for sub_list[0 .. m))
bool band_lu_blocked(int32_t kl_max);
// true when the slab conversions (which take block lists) apply
bool convert_slabs(int32_t nbl_max, int32_t kl_max, int32_t nbu_max, int32_t kv_max);
void launch_band_colnorm(const double* ab, const SubInfo* subs, int32_t m, int32_t npad_max, double* colnorm,
                         hipStream_t s);
void launch_band_nnz(const double* ab, const SubInfo* subs, int32_t m, int32_t n_max, int64_t* counts,
                     hipStream_t s);
// The conversions raise *info to 1 for a zero diagonal of U and to 2 for a
// block not finite in the storage type.
void launch_convert_lower(const double* ab, const int32_t* ipiv, const SubInfo* subs, const LBlk* lb, int32_t nblk,
                          double* work, int32_t* lperm, void* lmat, int prec, int32_t* info, int32_t nbl_max,
                          int32_t kl_max, const int32_t* blk_list, hipStream_t s);
void launch_convert_upper(const double* ab, const SubInfo* subs, const UBlk* ub, int32_t nblk, double* work,
                          void* uinv, void* u12, int prec, int32_t* info, int32_t nbu_max, int32_t kv_max,
                          const int32_t* blk_list, hipStream_t s);
void launch_dense_scatter(const int64_t* dst, const int32_t* src, const double* cpv, int64_t n, double* out,
                          hipStream_t s);
void launch_schur_blocks(int32_t k, const int32_t* agg_s, const int32_t* agg_d, const int64_t* g_off,
                         const int64_t* dd_off, const int64_t* de_off, const int64_t* df_off, double* G,
                         double* Dd, double* De, double* Df, int32_t* info, int rowsum, hipStream_t s);
void launch_invert_dense(int32_t k, const int32_t* agg_s, const int64_t* g_off, const double* S,
                         double* work, int32_t* info, const int64_t* sinv_off, void* sinv, float* scale,
                         int prec, hipStream_t s);
// work: the padded vector the sweep uses (NULL: the handle's ypad / zpad)
void launch_interior_solve(const addns_precond* pc, const double* yin, double* out, int second,
                           const double* x2, const double* z1, hipStream_t s, double* work = nullptr);
int max_sweep_chunks(const Plan& pl);
void build_chunked_sweep(addns_precond* pc, int p, hipStream_t s);
void release_chunked_sweep(addns_precond* pc);
void launch_column_solves(const addns_precond* pc, int32_t npairs, const int32_t* pair_sub, const int32_t* pair_col,
                          const int64_t* pair_off, double* scratch, double* out, hipStream_t s);
void launch_exact_schur_update(int32_t nsep, const int32_t* pcol_ptr, const int32_t* pair_sub, const int64_t* pair_off,
                               const SubInfo* subs, const int32_t* agg_of, const int32_t* agg_off, const int64_t* g_off,
                               const int32_t* f_rowptr, const int32_t* f_colidx, const double* f_vals,
                               const double* U, double* S, hipStream_t s);
void launch_interface_solve(const addns_precond* pc, const double* y, const double* z1, double* x2out,
                            hipStream_t s);
// coarse correction (kernels_coarse.hip, column solves in kernels_apply.hip)
// rhs_given = 0: right-hand sides E_j z_c formed in the scratch; 1: taken
// from the scratch as stored there
void launch_coarse_column_solves(const addns_precond* pc, int32_t npairs, const int32_t* pair_sub,
                                 const int32_t* pair_col, const int64_t* pair_off, double* scratch, double* out,
                                 int rhs_given, hipStream_t s);
// one step of iterative refinement of the column solves: scratch = E_j z_c -
// A_jj W (FP64), then W += A_jj^{-1} scratch through the sweep
void launch_coarse_refine(const addns_precond* pc, int32_t npairs, const int32_t* pair_sub, const int32_t* pair_col,
                          const int64_t* pair_off, double* W, double* scratch, double* dW, hipStream_t s);
void launch_coarse_sz(const addns_precond* pc, const int32_t* sub_of, const int32_t* pair_sub,
                      const int32_t* cpair_ptr, const int64_t* pair_off, const int32_t* int_off,
                      const double* W, hipStream_t s);
void launch_coarse_ec(const addns_precond* pc, int32_t nc, double* Ec, hipStream_t s);
// Gauss-Jordan inverses of the diagonal blocks of E_c in place (blockwise
// storage); work: nb + 2 nc doubles; info: first failing step + 1 (0 = ok)
void launch_gj_invert(const addns_precond* pc, double* A, int32_t* perm, double* work, int32_t* info, hipStream_t s);
void launch_coarse_restrict(const addns_precond* pc, const double* y, const double* z1, hipStream_t s);
void launch_coarse_solve(const addns_precond* pc, hipStream_t s);
void launch_overlap_split(int32_t k, const int32_t* agg_s, const int32_t* agg_w, const int64_t* g_off,
                          const int64_t* a_off, const int64_t* l_off, const double* Se, double* A, double* L,
                          hipStream_t s);
void launch_overlap_m(int32_t k, const int32_t* agg_s, const int32_t* agg_w, const int64_t* a_off,
                      const int64_t* l_off, const int64_t* m_off, int32_t width, const double* winv, const double* L,
                      void* M, int m_double, hipStream_t s);
void launch_overlap_chain(const addns_precond* pc, double* x2, hipStream_t s);
void launch_overlap_q(const addns_precond* pc, hipStream_t s);
int32_t overlap_segment_length(int32_t k, int32_t requested);
int overlap_chain_width(int32_t smax);
void launch_permute(const int32_t* perm, const double* in, double* out, int32_t n, int inverse,
                    const double* scale, hipStream_t s);
// krylov
void launch_spmv(const int32_t* rowptr, const int32_t* colidx, const double* vals, const double* x,
                 double* y, int32_t n, hipStream_t s);
int krylov_grid(int32_t n);
void launch_spmv_dot(const int32_t* rowptr, const int32_t* colidx, const double* vals, const double* x,
                     double* w, const double* v0, int32_t n, double* partials, hipStream_t s);
void launch_residual(const int32_t* rowptr, const int32_t* colidx, const double* vals, const double* x,
                     const double* b, double* r, int32_t n, double* partials, hipStream_t s);
int cgs_parts(int32_t n);  // partials per basis vector of the CGS2 kernels
void launch_spmv_dots(const int32_t* rowptr, const int32_t* colidx, const double* vals, const double* z, double* w,
                      const double* V, int nvec, int32_t n, double* partials, hipStream_t s);
void launch_cgs_coeffs(const double* partials, int nparts, int nvec, double* h, double* Hcol, int add, hipStream_t s);
void launch_cgs_update(double* w, const double* V, int nvec, const double* h, int32_t n, double* partials, int mode,
                       hipStream_t s);
void launch_mgs_step(double* w, const double* vi, const double* vnext, int32_t n, const double* partials_in,
                     double* partials_out, double* h_out, int nparts, hipStream_t s);
void launch_finalize(double* H, double* g, double* cs, double* sn, const double* partials, int nparts,
                     int32_t j, int32_t ldh, double* scal, double* hostout, const double* w, double* v,
                     int32_t n, hipStream_t s);
void launch_scale_copy(const double* w, double* v, const double* scal, int idx, int32_t n, hipStream_t s);
void launch_norm_finalize(const double* partials, int nparts, double* scal, int idx, hipStream_t s);
void launch_backsolve(const double* H, const double* g, int32_t j, int32_t ldh, double* y, hipStream_t s);
void launch_combine(const double* Z, int64_t ldz, const double* y, int32_t j, int32_t n, double* x, int add,
                    hipStream_t s);
void launch_dot_partials(const double* a, const double* b, int32_t n, double* partials, hipStream_t s);
// segmented Krylov (batched systems)
int seg_chunk_rows();
void launch_seg_spmv_dot(const int32_t* rp, const int32_t* ci, const double* cv, const double* z, double* w,
                         const double* v0, const Chunk* ch, int nch, const int32_t* live, double* parts, hipStream_t s);
void launch_seg_residual(const int32_t* rp, const int32_t* ci, const double* cv, const double* x, const double* b,
                         double* r, const Chunk* ch, int nch, const int32_t* live, double* parts, hipStream_t s);
void launch_seg_dot(const double* a, const double* b, const Chunk* ch, int nch, double* parts, hipStream_t s);
void launch_seg_mgs_step(double* w, const double* vi, const double* vnext, const Chunk* ch, int nch,
                         const int32_t* coff, const int32_t* live, const double* pin, double* pout, double* state,
                         int64_t st, int64_t hidx, hipStream_t s);
void launch_seg_finalize(double* state, int64_t st, const double* parts, const int32_t* coff, const int32_t* live,
                         int nsys, int32_t j, int32_t ldh, int32_t restart, double* scal, hipStream_t s);
void launch_seg_norm(const double* parts, const int32_t* coff, const int32_t* live, int nsys, double* scal, int idx,
                     hipStream_t s);
void launch_seg_init_g(double* state, int64_t st, const int32_t* live, int nsys, int32_t ldh, int32_t restart,
                       const double* scal, int idx, hipStream_t s);
void launch_seg_scale_copy(const double* w, double* v, const double* scal, int idx, const Chunk* ch, int nch,
                           const int32_t* live, hipStream_t s);
void launch_seg_backsolve(double* state, int64_t st, const int32_t* jdone, int nsys, int32_t ldh, int32_t restart,
                          hipStream_t s);
void launch_seg_combine(const double* Z, int64_t ldz, const double* state, int64_t st, const int32_t* jdone,
                        int32_t ldh, int32_t restart, const Chunk* ch, int nch, double* x, hipStream_t s);
// learned interface correction (kernels_dtn.hip)
int mlp_param_count();
int mlp_grad_groups(int64_t count);  // workgroups (partials) of launch_mlp_grad
void launch_dtn_features(int64_t count, const int32_t* smp_row, const int32_t* smp_nb, const int32_t* rp,
                         const int32_t* ci, const double* cv, const int32_t* perm, const double* R, float* X,
                         hipStream_t s);
void launch_dtn_targets(int64_t count, const int64_t* smp_loc, const double* S, const double* G, float* Y, float* M,
                        hipStream_t s);
void launch_dtn_correct(int64_t count, const int64_t* smp_loc, const float* D, double* G, hipStream_t s);
// The network kernels read the weights as an image (the LDS layout of the
// padded weight tiles, mlp_image_floats() floats), built by
// launch_mlp_image from the packed parameters and updated by every Adam step.
int mlp_image_floats();
void launch_mlp_image(const float* wts, float* img, hipStream_t s);
void launch_mlp_forward(const float* img, const float* X, float* P, int64_t count, int bf16, hipStream_t s);
void launch_mlp_grad(const float* img, const float* X, const float* Y, const float* M, const int32_t* idx,
                     int64_t count, float scale, float* gpart, float* lpart, hipStream_t s);
void launch_mlp_reduce_adam(const float* gpart, int nwg, float* grad, float* wts, float* img, float* m1, float* m2,
                            int adam, float lr, float b1, float b2, float eps, float bc1, float bc2, hipStream_t s);

// Runs an entry point's body, turning exceptions into status codes and a
// thread-local message: no C++ exception crosses the C boundary.
template <class F>
int guarded(const char* what, F&& f) {
  try {
    return f();
  } catch (const ArgError& e) {
    set_error(std::string(what) + ": " + e.what());
    return ADDNS_ERR_ARG;
  } catch (const SingularError& e) {
    set_error(std::string(what) + ": " + e.what());
    return ADDNS_ERR_SINGULAR;
  } catch (const HipError& e) {
    set_error(std::string(what) + ": " + e.what());
    return ADDNS_ERR_HIP;
  } catch (const std::bad_alloc&) {
    set_error(std::string(what) + ": out of host memory");
    return ADDNS_ERR_NOMEM;
  } catch (const std::exception& e) {
    set_error(std::string(what) + ": " + e.what());
    return ADDNS_ERR_HIP;
  }
}
}  // namespace addns
