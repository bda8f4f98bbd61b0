// Apply kernels: Algorithm 2, x = B^{-1} y in the permuted numbering.
//
//   interior solve   z1 = D^{-1} y1           (one workgroup per subdomain, or
//                                               per chunk of it: see below)
//   interface solve  x2 = Shat^{-1}(y2 - F z1) (one workgroup per aggregate)
//   interior solve   x1 = z1 - D^{-1} (E x2)   (E x2 formed in a first pass)
//
// Each interior solve is a forward sweep over the lower blocks followed by a
// backward sweep over the upper blocks.  Every block step is a gather plus
// one or two dense GEMVs whose matrices are streamed from HBM column-major:
// a wavefront reads 64 consecutive rows of one column per load (coalesced),
// the vector operand sits in LDS and is read as a broadcast, and column
// groups are reduced through LDS in a fixed order.  The matrices do not
// depend on the data, so their loads run ahead of the step that uses them.
// Factors are stored in FP64 or FP32; accumulation is always FP64.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "precond.h"

namespace addns {
namespace {

constexpr int kSweepThreads = 1024;
constexpr int kWaves = kSweepThreads / 64;

template <class T>
__device__ inline double ld(const T* p) { return (double)(*p); }
constexpr int kIfRows = 4;  // rows a wave loads together in the interface solve
template <>
__device__ inline double ld<__half>(const __half* p) { return (double)__half2float(*p); }

// Column chunk of one wave: CB columns x S row slots of a block, plus the
// window-gather indices of those columns (lower sweep only).  Register
// resident; a wave keeps two chunks so that the loads of the next chunk (or
// of the next block, across the barriers of a step) are in flight while the
// current one is consumed.
template <class T>
constexpr int chunk_cols(int S) {
  // the widest chunks whose two copies fit in the registers of 1024 threads
  return sizeof(T) == 4 ? (S <= 2 ? 12 : (S == 3 ? 9 : (S == 4 ? 6 : 5)))
                        : (S <= 2 ? 4 : (S == 3 ? 3 : 2));
}

template <class T, int S>
struct Chunk {
  static constexpr int CB = chunk_cols<T>(S);
  T v[CB][S];
  int32_t gi[CB];
};

// Geometry of one wave in a GEMV with R rows and K columns: waves form RG
// row groups (64 S rows each) x CG column groups; this wave owns the rows
// r0 + 64 s + lane and the columns [kb, ke).  The same for every block of a
// sweep, so it is computed once per sweep.
struct Geo {
  int R, K, CG, cg, kb, ke, r0;
  bool act;
};

template <int S>
__device__ __attribute__((always_inline)) inline Geo make_geo(int R, int K) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  Geo g;
  g.R = R;
  g.K = K;
  const int RG = (R + 64 * S - 1) / (64 * S);
  g.CG = max(1, kWaves / RG);
  g.act = w < RG * g.CG;
  const int rg = w % RG;
  g.cg = w / RG;
  g.kb = K * g.cg / g.CG;
  g.ke = K * (g.cg + 1) / g.CG;
  g.r0 = rg * 64 * S;
  return g;
}

// Loads columns k0 .. k0+CB-1 of M (column-major, leading dimension R).
// The blocks store their structural zeros, so the plain form needs no
// per-lane mask: each column's base address is wave-uniform (scalar
// registers) and the lane's row is the only per-lane part of an address.
// With Z, each lane loads only rows inside its column's nonzero range (and
// below R); the others keep an exact zero: fewer bytes (no slot or row past
// the structure is fetched), more instructions.  Few subdomains leave the
// sweep bound by per-CU issue and latency, many subdomains by HBM, so the
// setup times both forms on the actual factors and keeps the faster (they
// give the same result bit for bit):
//   kind 2: upper        M(r,k) = 0 for r > k
//   kind 3: band-shifted M(r,k) = 0 for r < k - par
//   kind 4: [lower; full] M(r,k) = 0 for r < min(k, par)
// In the plain form the last slot may run past row R - 1 (at most 64 S - 1
// rows): those products land in rows that are never stored, and every
// factor allocation is padded so that the overrun stays inside it.  Columns
// past the wave's range repeat its last column (their vector weight is 0).
template <class T, int S, int kind, bool Z>
__device__ __attribute__((always_inline)) inline void load_chunk(Chunk<T, S>& c, const Geo& g, const T* M, int par,
                                                                 const int32_t* gidx, int k0) {
  constexpr int CB = Chunk<T, S>::CB;
  const uint32_t lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int k = __builtin_amdgcn_readfirstlane(min(k0 + j, g.ke - 1));
    const T* col = M + (int64_t)k * g.R;
    const int hi = kind == 2 ? min(g.R, k + 1) : g.R;  // rows [lo, hi) may be nonzero
    const int lo = kind == 3 ? max(0, k - par) : (kind == 4 ? min(k, par) : 0);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = g.r0 + 64 * s + (int)lane;
      T x = T(0);
      if (!Z || (r >= lo && r < hi)) x = col[(uint32_t)r];
      c.v[j][s] = x;
    }
    if (gidx) c.gi[j] = gidx[k];
  }
}

template <class T, int S>
__device__ __attribute__((always_inline)) inline void fma_chunk(const Chunk<T, S>& c, const Geo& g, int k0, const double* vin, bool gather,
                                 double (&acc)[S]) {
  constexpr int CB = Chunk<T, S>::CB;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int k = k0 + j;
    const double vk = k < g.ke ? vin[gather ? c.gi[j] : k] : 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] += (double)c.v[j][s] * vk;
  }
}

// Issues the first two chunks of a GEMV (the rest follow inside run_gemv).
template <class T, int S, int kind, bool Z>
__device__ __attribute__((always_inline)) inline void prefetch_gemv(Chunk<T, S>& A, Chunk<T, S>& B, const Geo& g, const T* M, int par,
                                     const int32_t* gidx) {
  constexpr int CB = Chunk<T, S>::CB;
  // a wave whose column range is empty (K below the column groups) loads
  // nothing: its first column would be kb - 1, outside the matrix
  if (!g.act || g.kb >= g.ke) return;
  load_chunk<T, S, kind, Z>(A, g, M, par, gidx, g.kb);
  if (g.kb + CB < g.ke) load_chunk<T, S, kind, Z>(B, g, M, par, gidx, g.kb + CB);
}

// part[cg * R + r] = sum over the wave's columns of M(r, k) vec(k); A and B
// hold the first two chunks (prefetch_gemv), later chunks are loaded two
// ahead of their use.  The caller synchronises and reduces over the CG
// column groups in a fixed order.
template <class T, int S, int kind, bool Z>
__device__ __attribute__((always_inline)) inline int run_gemv(Chunk<T, S>& A, Chunk<T, S>& B, const Geo& g, const T* M, int par,
                               const int32_t* gidx, const double* vin, double* part) {
  constexpr int CB = Chunk<T, S>::CB;
  if (g.act) {
    double acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = 0.0;
    const bool gather = gidx != nullptr;
    for (int k0 = g.kb; k0 < g.ke; k0 += 2 * CB) {
      fma_chunk<T, S>(A, g, k0, vin, gather, acc);
      if (k0 + 2 * CB < g.ke) load_chunk<T, S, kind, Z>(A, g, M, par, gidx, k0 + 2 * CB);
      if (k0 + CB < g.ke) {
        fma_chunk<T, S>(B, g, k0 + CB, vin, gather, acc);
        if (k0 + 3 * CB < g.ke) load_chunk<T, S, kind, Z>(B, g, M, par, gidx, k0 + 3 * CB);
      }
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = g.r0 + 64 * s + lane;
      if (r < g.R) part[g.cg * g.R + r] = acc[s];
    }
  }
  return g.CG;
}

__device__ inline double sum_parts(const double* part, int R, int CG, int r) {
  double s = 0.0;
  for (int c = 0; c < CG; ++c) s += part[c * R + r];
  return s;
}

struct SweepArgs {
  int32_t maxW, maxU;
  const SubInfo* subs;
  const LBlk* lb;
  const UBlk* ub;
  const int32_t* lperm;
  const void* lmat;
  const void* uinv;
  const void* u12;
  const int32_t* e_rowptr;
  const int32_t* e_colidx;
  const double* e_vals;
  double* ypad;      // padded intermediate (after the lower sweep)
  // mode 2 (column solves): workgroup p solves A_jj^{-1} E(int_j, c), j = pair_sub[p],
  // c = pair_col[p]; scratch and output at pair_off[p] (padded length of j)
  const int32_t* pair_sub;
  const int32_t* pair_col;
  const int64_t* pair_off;
  // mode 2 with a coarse space: pair_col names a coarse column z_c and the
  // right-hand side is E(int_j, :) z_c, z_c held per separator position as
  // (piece, constant value, linear value)
  const int32_t* cz_piece;
  const double* cz_z0;
  const double* cz_z1;
  const int32_t* cz_colp;
  const int32_t* cz_colk;
  int32_t pair_rhs_given;  // mode 2: the right-hand side is already in the scratch
  // modes 0 and 1 of a batched solve: workgroups of subdomains whose system
  // has converged (live[unit_sys[sub]] == 0) do nothing
  const int32_t* live;
  const int32_t* unit_sys;
};

// One workgroup per subdomain.  mode 0: out[int] = D^{-1} yin[int].
// mode 1: input u = E x2 (x2 = separator part, CSR E), and
// out[int] = z1[int] - D^{-1} u.  mode 2: one workgroup per (subdomain,
// separator column) pair, out[pair_off + row] = (A_jj^{-1} E(int_j, c))(row).
//
// Lower sweep, block b (window rows b*nbl .. b*nbl+W-1, W = nbl+kl):
//   v = P_b w;  [x_b; c] = [inv(L11); L21 inv(L11)] v_top;  carry = v_bot - c
// Upper sweep, block b (rows b*nbu ..):  x_b = inv(U_bb) (y_b - U_b,b+1 x_b+1)
//
// The block matrices do not depend on the data, so the loads of the next
// GEMV's first chunks are issued before the barriers and reductions of the
// current step, and the next step's input rows are fetched before the
// current GEMV: the sweep waits for memory once per step at most, not once
// per chunk.
template <class T, int S, bool Z>
__global__ void __launch_bounds__(kSweepThreads)
k_interior_solve(SweepArgs a, const double* __restrict__ yin, double* out, int mode, const double* x2,
                 const double* z1) {
  extern __shared__ double smem[];
  if (mode != 2 && a.live && !a.live[a.unit_sys[blockIdx.x]]) return;
  const SubInfo q = a.subs[mode == 2 ? a.pair_sub[blockIdx.x] : blockIdx.x];
  const int32_t pcol = mode == 2 ? a.pair_col[blockIdx.x] : -1;
  const int64_t poff = mode == 2 ? a.pair_off[blockIdx.x] : 0;
  const int32_t n = q.n, npad = q.npad;
  if (n == 0) return;
  const int32_t ioff = q.int_off, voff = q.vec_off;
  const int32_t KL = q.kl, nbL = q.nbl, nbU = q.nbu, W = nbL + KL, KV = q.kl + q.ku;
  const int tid = threadIdx.x;
  double* wA = smem;             // maxW
  double* wB = wA + a.maxW;      // maxW
  double* t = wB + a.maxW;       // maxU
  double* xn = t + a.maxU;       // maxU
  double* part = xn + a.maxU;    // kWaves * max(maxW, maxU)
  double* ypad = a.ypad + (mode == 2 ? poff : (int64_t)voff);
  const T* lmat = (const T*)a.lmat + q.lmat_off;
  const T* uinv = (const T*)a.uinv + q.u_off;
  const T* u12 = (const T*)a.u12 + q.u_off;
  const int32_t* lperm = a.lperm + q.lperm_off;
  const int32_t nL = npad / nbL, nU = npad / nbU;
  const Geo gl = make_geo<S>(W, nbL);
  const Geo gu = make_geo<S>(nbU, nbU);
  Chunk<T, S> A, B;
  // first GEMV of the sweep in flight while the input is prepared
  if (nL > 0) prefetch_gemv<T, S, 4, Z>(A, B, gl, lmat, nbL, lperm);
  // modes 1 and 2: the sweep input (E x2, or column pcol of E) into ypad;
  // the lower sweep writes ypad only below the rows it still has to read
  if (mode != 0 && !(mode == 2 && a.pair_rhs_given)) {
    const int32_t zp = (mode == 2 && a.cz_piece) ? a.cz_colp[pcol] : -1;
    const double* zv = (mode == 2 && a.cz_piece) ? (a.cz_colk[pcol] ? a.cz_z1 : a.cz_z0) : nullptr;
    for (int32_t r = tid; r < n; r += blockDim.x) {
      double s = 0.0;
      for (int32_t e = a.e_rowptr[ioff + r]; e < a.e_rowptr[ioff + r + 1]; ++e) {
        const int32_t c = a.e_colidx[e];
        if (mode == 1) s += a.e_vals[e] * x2[c];
        else if (zv) {
          if (a.cz_piece[c] == zp) s += a.e_vals[e] * zv[c];
        } else if (c == pcol) s += a.e_vals[e];
      }
      ypad[r] = s;
    }
    __syncthreads();
  }
  const double* src = mode == 0 ? yin + ioff : ypad;
  // ---- forward sweep over lower blocks
  double* wc = wA;
  double* wn = wB;
  for (int32_t r = tid; r < W; r += blockDim.x) wc[r] = r < n ? src[r] : 0.0;
  __syncthreads();
  for (int32_t b = 0; b < nL; ++b) {
    const int32_t* idx = lperm + (int64_t)b * W;
    const T* M = lmat + (int64_t)b * W * nbL;
    // next window's new rows and this block's carry gather indices, fetched
    // before this step's GEMV so that the reduction below waits for neither
    const int32_t rin = (b + 1) * nbL + KL + tid;
    const double nin = (tid < nbL && rin < n) ? src[rin] : 0.0;
    const int32_t cidx = (tid >= nbL && tid < W) ? idx[tid] : 0;
    const int CG = run_gemv<T, S, 4, Z>(A, B, gl, M, nbL, idx, wc, part);
    if (b + 1 < nL) prefetch_gemv<T, S, 4, Z>(A, B, gl, M + (int64_t)W * nbL, nbL, idx + W);
    else if (nU > 0) prefetch_gemv<T, S, 2, Z>(A, B, gu, uinv + (int64_t)(nU - 1) * nbU * nbU, 0, nullptr);
    __syncthreads();
    for (int32_t r = tid; r < W; r += blockDim.x) {
      const double v = sum_parts(part, W, CG, r);
      if (r < nbL) ypad[b * nbL + r] = v;
      else wn[r - nbL] = wc[r == tid ? cidx : idx[r]] - v;
    }
    if (tid < nbL) wn[KL + tid] = nin;
    __syncthreads();
    double* tmp = wc;
    wc = wn;
    wn = tmp;
  }
  // ---- backward sweep over upper blocks
  for (int32_t b = nU - 1; b >= 0; --b) {
    const int64_t uoff = (int64_t)b * nbU * nbU;
    const double yb = tid < nbU ? ypad[b * nbU + tid] : 0.0;
    if (b < nU - 1) {
      const int CG = run_gemv<T, S, 3, Z>(A, B, gu, u12 + uoff, KV - nbU, nullptr, xn, part);
      prefetch_gemv<T, S, 2, Z>(A, B, gu, uinv + uoff, 0, nullptr);
      __syncthreads();
      if (tid < nbU) t[tid] = yb - sum_parts(part, nbU, CG, tid);
    } else {
      if (tid < nbU) t[tid] = yb;
    }
    __syncthreads();
    const int CG = run_gemv<T, S, 2, Z>(A, B, gu, uinv + uoff, 0, nullptr, t, part);
    if (b > 0) prefetch_gemv<T, S, 3, Z>(A, B, gu, u12 + uoff - (int64_t)nbU * nbU, KV - nbU, nullptr);
    __syncthreads();
    if (tid < nbU) {
      const double x = sum_parts(part, nbU, CG, tid);
      xn[tid] = x;
      const int32_t row = b * nbU + tid;
      if (row < n) {
        if (mode == 1) out[ioff + row] = z1[ioff + row] - x;
        else if (mode == 2) out[poff + row] = x;
        else out[ioff + row] = x;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Chunked interior sweep.  The lower recurrence passes a KL-long carry from
// block to block, the upper one the solution block x_{b+1}; both are linear.
// Cutting every interior at p - 1 upper-block boundaries (chunk c holds upper
// blocks [u_c, u_{c+1}), u_c = floor(nU c / p), and lower blocks [2u_c,
// 2u_{c+1})), each chunk is swept side by side from a zero carry or state and
// then corrected:
//   lower  y_c = y0_c + X_c d_c,   d_1 = g_0,
//          d_c = g_{c-1} + sum_i (T_{c-1} ... T_{c-1-i}) g_{c-2-i}
//   upper  x_c = x0_c + Y_c s_c,   s_{p-2} = f_{p-1},
//          s_c = f_{c+1} + sum_i (Yt_{c+1} ... Yt_{c+1+i}) f_{c+2+i}
// with g_c the zero-carry carry out of chunk c, f_c the first block of x0_c,
// X_c / T_c the response of chunk c's outputs / carry out to a unit carry in,
// Y_c / Yt_c that of its outputs / first block to a unit state above.  The
// single-chunk responses are swept once per factorisation (mode 3, one
// workgroup per chunk and unit); the products over chunk ranges follow from
// them by small GEMMs (k_chunk_products) and are stored side by side, so each
// chunk finds its carry and state with one GEMV instead of a chain of
// dependent ones.  Three launches per solve: zero-carry lower chunks; carry,
// lower correction and zero-state upper chunk; state, upper correction and
// output.
//   LP_c = [T_{c-1}, T_{c-1}T_{c-2}, ..., T_{c-1}...T_1]   KL x (c-1) KL
//   UP_c = [R_{c+1}, R_{c+1}R_{c+2}, ..., R_{c+1}...R_{p-2}]
// The state above chunk c reaches it only through the nonzero columns of the
// coupling block U_{b,b+1}, b = u_{c+1} - 1 (found at setup in the stored
// factors): a unit state in any other column has exactly zero response.  So
// the upper responses are taken only for those ns_c columns nz_c, the state
// s_c is carried only in them, Y_c is rows_c x ns_c, and R_c = Yt_c(nz_{c-1}, :)
// is ns_{c-1} x ns_c (UP_c: ns_c x (ns_{c+1} + ... + ns_{p-2})).
// Likewise a carry position at a lower boundary is "pure" when its value is
// still one raw input (its row of every block matrix it passed is zero, and
// it entered the window as an input): the chunk starts it from that input
// (prow), and only the other nsl_c positions np_c are corrected, so d_c, X_c
// (rows_c x nsl_c), T_c and LP_c (nsl_c x (nsl_1 + ... + nsl_{c-1})) live on
// them.
// ---------------------------------------------------------------------------
struct ChunkArgs {
  int32_t p, klmax, stk;  // chunks, carry stride, LDS words of the stacked recurrence vector
  const int64_t* off;     // per (subdomain, chunk): element offsets of X_c, LP_c, Y_c, UP_c
  void* lx;
  void* lp;
  void* uy;
  void* up;
  double* cz;          // zero-carry carry out of each chunk (klmax per (subdomain, chunk))
  double* xs;          // zero-state upper outputs, padded interior numbering
  double* uin;         // mode 1: the sweep input E x2, padded interior numbering
  const int32_t* nz;   // coupling columns nz_c of every (subdomain, boundary c) ...
  const int32_t* nzo;  // ... at nz[nzo[j p + c] .. nzo[j p + c + 1])
  const int32_t* prow; // lower boundary c: input row of each pure carry position, else -1 (klmax each)
  const int32_t* np;   // coupled carry positions np_c of every (subdomain, boundary c) ...
  const int32_t* npo;  // ... at np[npo[j p + c] .. npo[j p + c + 1]) (empty for c = 0)
  const int32_t* job;  // mode 3: (subdomain, first chunk, end chunk, unit) per workgroup
};

__host__ __device__ inline int32_t chunk_ub(int32_t nU, int32_t p, int32_t c) { return (int32_t)((int64_t)nU * c / p); }

// Lower chunks.  mode 0: input yin; mode 1: input E x2 (each chunk forms the
// rows it reads); mode 3: the response of chunks [c, ce) to the unit carry
// `unit` into chunk c: X_c (single chunk) and the carry out into LP_ce.
template <class T, int S, bool Z>
__global__ void __launch_bounds__(kSweepThreads)
k_chunk_lower(SweepArgs a, ChunkArgs ca, const double* __restrict__ yin, int mode, const double* __restrict__ x2) {
  extern __shared__ double smem[];
  const int32_t jb = blockIdx.x;
  const int32_t j = mode == 3 ? ca.job[4 * jb] : jb / ca.p;
  const int32_t c = mode == 3 ? ca.job[4 * jb + 1] : jb % ca.p;
  const int32_t ce = mode == 3 ? ca.job[4 * jb + 2] : c + 1;
  const int32_t unit = mode == 3 ? ca.job[4 * jb + 3] : -1;
  const SubInfo q = a.subs[j];
  const int32_t n = q.n;
  if (n == 0) return;
  const int32_t ioff = q.int_off, voff = q.vec_off;
  const int32_t KL = q.kl, nbL = q.nbl, W = nbL + KL, nU = q.npad / q.nbu;
  const int32_t b0 = 2 * chunk_ub(nU, ca.p, c), b1 = 2 * chunk_ub(nU, ca.p, ce);
  const int32_t r0 = b0 * nbL, r1 = b1 * nbL, rows = r1 - r0;
  const int tid = threadIdx.x;
  double* wA = smem;
  double* wB = wA + a.maxW;
  double* part = wB + a.maxW;  // kWaves * maxW
  const T* lmat = (const T*)a.lmat + q.lmat_off;
  const int32_t* lperm = a.lperm + q.lperm_off;
  const Geo gl = make_geo<S>(W, nbL);
  Chunk<T, S> A, B;
  if (b0 < b1) prefetch_gemv<T, S, 4, Z>(A, B, gl, lmat + (int64_t)b0 * W * nbL, nbL, lperm + (int64_t)b0 * W);
  const double* src = mode == 0 ? yin + ioff : ca.uin + voff;
  if (mode == 1) {
    // the rows this chunk reads: its own after the carry rows, and the
    // carry rows of the next chunk (which enter through the last window)
    const int32_t lo = c == 0 ? 0 : r0 + KL, hi = min(r1 + KL, n);
    for (int32_t r = lo + tid; r < hi; r += blockDim.x) {
      double s = 0.0;
      for (int32_t e = a.e_rowptr[ioff + r]; e < a.e_rowptr[ioff + r + 1]; ++e) s += a.e_vals[e] * x2[a.e_colidx[e]];
      ca.uin[voff + r] = s;
    }
    __syncthreads();
  }
  auto input = [&](int32_t row) -> double { return (mode == 3 || row >= n) ? 0.0 : src[row]; };
  // a pure carry position starts from its input row (mode 1: E x2 formed here,
  // the row may belong to the previous chunk)
  auto pure_input = [&](int32_t row) -> double {
    if (row < 0 || row >= n) return 0.0;
    if (mode == 0) return yin[ioff + row];
    double s = 0.0;
    for (int32_t e = a.e_rowptr[ioff + row]; e < a.e_rowptr[ioff + row + 1]; ++e) s += a.e_vals[e] * x2[a.e_colidx[e]];
    return s;
  };
  const int32_t* prow = ca.prow + ((int64_t)j * ca.p + c) * ca.klmax;
  const int32_t o_c = ca.npo[(int64_t)j * ca.p + c];
  double* wc = wA;
  double* wn = wB;
  for (int32_t r = tid; r < W; r += blockDim.x) {
    double v;
    if (c == 0 || r >= KL) v = input(r0 + r);
    else if (mode == 3) v = r == ca.np[o_c + unit] ? 1.0 : 0.0;
    else v = pure_input(prow[r]);
    wc[r] = v;
  }
  __syncthreads();
  double* ypad = a.ypad + voff;
  T* X = (mode == 3 && ce == c + 1) ? (T*)ca.lx + ca.off[4 * ((int64_t)j * ca.p + c)] + (int64_t)unit * rows : nullptr;
  for (int32_t b = b0; b < b1; ++b) {
    const int32_t* idx = lperm + (int64_t)b * W;
    const T* M = lmat + (int64_t)b * W * nbL;
    const int32_t rin = (b + 1) * nbL + KL + tid;
    const double nin = (tid < nbL && b + 1 < b1) ? input(rin) : 0.0;
    const int32_t cidx = (tid >= nbL && tid < W) ? idx[tid] : 0;
    const int CG = run_gemv<T, S, 4, Z>(A, B, gl, M, nbL, idx, wc, part);
    if (b + 1 < b1) prefetch_gemv<T, S, 4, Z>(A, B, gl, M + (int64_t)W * nbL, nbL, idx + W);
    __syncthreads();
    for (int32_t r = tid; r < W; r += blockDim.x) {
      const double v = sum_parts(part, W, CG, r);
      if (r < nbL) {
        if (mode != 3) ypad[b * nbL + r] = v;
        else if (X) X[b * nbL + r - r0] = (T)v;
      } else {
        wn[r - nbL] = wc[r == tid ? cidx : idx[r]] - v;
      }
    }
    if (tid < nbL) wn[KL + tid] = nin;
    __syncthreads();
    double* tmp = wc;
    wc = wn;
    wn = tmp;
  }
  // the carry out of the chunk on the coupled positions of the next boundary
  if (ce < ca.p) {
    const int32_t o1 = ca.npo[(int64_t)j * ca.p + ce], n1 = ca.npo[(int64_t)j * ca.p + ce + 1] - o1;
    if (mode == 3) {
      // column `unit` of T_c (block 0 of LP_{c+1}: n1 rows)
      T* L = (T*)ca.lp + ca.off[4 * ((int64_t)j * ca.p + ce) + 1] + (int64_t)unit * n1;
      for (int32_t k = tid; k < n1; k += blockDim.x) L[k] = (T)wc[ca.np[o1 + k]];
    } else {
      for (int32_t k = tid; k < n1; k += blockDim.x) ca.cz[((int64_t)j * ca.p + c) * ca.klmax + k] = wc[ca.np[o1 + k]];
    }
  }
}

// Carry and lower correction of chunk c (modes 0/1), then its upper blocks
// from a zero state above; mode 3: the response of chunks [c, ce) (swept
// downwards) to the unit state `unit` above chunk ce - 1: Y_c (single chunk)
// and the first block of chunk c into UP_{c-1}.
template <class T, int S, bool Z>
__global__ void __launch_bounds__(kSweepThreads)
k_chunk_upper(SweepArgs a, ChunkArgs ca, int mode) {
  extern __shared__ double smem[];
  const int32_t jb = blockIdx.x;
  const int32_t j = mode == 3 ? ca.job[4 * jb] : jb / ca.p;
  const int32_t c = mode == 3 ? ca.job[4 * jb + 1] : jb % ca.p;
  const int32_t ce = mode == 3 ? ca.job[4 * jb + 2] : c + 1;
  const int32_t unit = mode == 3 ? ca.job[4 * jb + 3] : -1;
  const SubInfo q = a.subs[j];
  if (q.n == 0) return;
  const int32_t voff = q.vec_off, nbU = q.nbu, KV = q.kl + q.ku, nU = q.npad / nbU;
  const int32_t u0 = chunk_ub(nU, ca.p, c), u1 = chunk_ub(nU, ca.p, ce);
  const int32_t r0 = u0 * nbU, rows = (u1 - u0) * nbU;
  const int tid = threadIdx.x;
  double* t = smem;
  double* xn = t + a.maxU;
  double* dv = xn + a.maxU;
  double* stk = dv + a.maxW;
  double* part = stk + ca.stk;
  const int64_t* off = ca.off + 4 * ((int64_t)j * ca.p + c);
  double* ypad = a.ypad + voff;
  const T* uinv = (const T*)a.uinv + q.u_off;
  const T* u12 = (const T*)a.u12 + q.u_off;
  const Geo gu = make_geo<S>(nbU, nbU);
  const bool state_in = mode == 3;
  Chunk<T, S> A, B;
  const int32_t* zl = ca.npo + (int64_t)j * ca.p;  // coupled carry positions per boundary
  const int32_t nsl = zl[c + 1] - zl[c];
  if (mode != 3 && c >= 1 && nsl > 0) {
    const double* cz = ca.cz + (int64_t)j * ca.p * ca.klmax;
    const Geo gx = make_geo<S>(rows, nsl);
    const T* X = (const T*)ca.lx + off[0];
    // K = nsl_1 + ... + nsl_{c-1}: block i of LP_c takes g_{c-2-i} (boundary c-1-i)
    const int32_t K = zl[c] - zl[1];
    if (c >= 2 && K > 0) {
      // d_c = g_{c-1} + LP_c [g_{c-2}; ...; g_0]
      const Geo gp = make_geo<S>(nsl, K);
      const T* LP = (const T*)ca.lp + off[1];
      prefetch_gemv<T, S, 0, false>(A, B, gp, LP, 0, nullptr);
      for (int32_t e = tid; e < K; e += blockDim.x) {
        // entries of boundary bb occupy [zl[c] - zl[bb + 1], zl[c] - zl[bb])
        int32_t bb = c - 1;
        while (e >= zl[c] - zl[bb]) --bb;
        stk[e] = cz[(int64_t)(bb - 1) * ca.klmax + (e - (zl[c] - zl[bb + 1]))];
      }
      __syncthreads();
      const int CG = run_gemv<T, S, 0, false>(A, B, gp, LP, 0, nullptr, stk, part);
      prefetch_gemv<T, S, 0, false>(A, B, gx, X, 0, nullptr);
      __syncthreads();
      for (int32_t r = tid; r < nsl; r += blockDim.x) dv[r] = cz[(int64_t)(c - 1) * ca.klmax + r] + sum_parts(part, nsl, CG, r);
    } else {
      prefetch_gemv<T, S, 0, false>(A, B, gx, X, 0, nullptr);
      for (int32_t r = tid; r < nsl; r += blockDim.x) dv[r] = cz[(int64_t)(c - 1) * ca.klmax + r];
    }
    __syncthreads();
    // y_c += X_c d_c
    const int CG = run_gemv<T, S, 0, false>(A, B, gx, X, 0, nullptr, dv, part);
    if (u0 < u1) prefetch_gemv<T, S, 2, Z>(A, B, gu, uinv + (int64_t)(u1 - 1) * nbU * nbU, 0, nullptr);
    __syncthreads();
    for (int32_t r = tid; r < rows; r += blockDim.x) ypad[r0 + r] += sum_parts(part, rows, CG, r);
    __syncthreads();
  } else if (state_in) {
    const int32_t col = ca.nz[ca.nzo[(int64_t)j * ca.p + c] + unit];
    for (int32_t r = tid; r < nbU; r += blockDim.x) xn[r] = r == col ? 1.0 : 0.0;
    if (u0 < u1) prefetch_gemv<T, S, 3, Z>(A, B, gu, u12 + (int64_t)(u1 - 1) * nbU * nbU, KV - nbU, nullptr);
    __syncthreads();
  } else if (u0 < u1) {
    prefetch_gemv<T, S, 2, Z>(A, B, gu, uinv + (int64_t)(u1 - 1) * nbU * nbU, 0, nullptr);
  }
  T* Y = mode == 3 ? (T*)ca.uy + off[2] + (int64_t)unit * rows : nullptr;
  double* xs = ca.xs + voff;
  for (int32_t b = u1 - 1; b >= u0; --b) {
    const int64_t uoff = (int64_t)b * nbU * nbU;
    const double yb = (mode != 3 && tid < nbU) ? ypad[b * nbU + tid] : 0.0;
    if (b < u1 - 1 || state_in) {
      const int CG = run_gemv<T, S, 3, Z>(A, B, gu, u12 + uoff, KV - nbU, nullptr, xn, part);
      prefetch_gemv<T, S, 2, Z>(A, B, gu, uinv + uoff, 0, nullptr);
      __syncthreads();
      if (tid < nbU) t[tid] = yb - sum_parts(part, nbU, CG, tid);
    } else {
      if (tid < nbU) t[tid] = yb;
    }
    __syncthreads();
    const int CG = run_gemv<T, S, 2, Z>(A, B, gu, uinv + uoff, 0, nullptr, t, part);
    if (b > u0) prefetch_gemv<T, S, 3, Z>(A, B, gu, u12 + uoff - (int64_t)nbU * nbU, KV - nbU, nullptr);
    __syncthreads();
    if (tid < nbU) {
      const double x = sum_parts(part, nbU, CG, tid);
      xn[tid] = x;
      const int32_t row = b * nbU + tid;
      if (mode != 3) xs[row] = x;
      else Y[row - r0] = (T)x;
    }
    __syncthreads();
  }
  if (mode == 3 && c >= 1) {
    // R_c column `unit` (block 0 of UP_{c-1}): the first block at nz_{c-1}
    const int32_t o = ca.nzo[(int64_t)j * ca.p + c - 1], ns = ca.nzo[(int64_t)j * ca.p + c] - o;
    T* R = (T*)ca.up + ca.off[4 * ((int64_t)j * ca.p + c - 1) + 3] + (int64_t)unit * ns;
    for (int32_t k = tid; k < ns; k += blockDim.x) R[k] = (T)xn[ca.nz[o + k]];
  }
}

// State and upper correction of chunk c, and the output: mode 0 out = x,
// mode 1 out = z1 - x (interior rows).
template <class T, int S>
__global__ void __launch_bounds__(kSweepThreads)
k_chunk_fix(SweepArgs a, ChunkArgs ca, int mode, double* out, const double* z1) {
  extern __shared__ double smem[];
  const int32_t j = blockIdx.x / ca.p, c = blockIdx.x % ca.p, p = ca.p;
  const SubInfo q = a.subs[j];
  const int32_t n = q.n;
  if (n == 0) return;
  const int32_t ioff = q.int_off, voff = q.vec_off, nbU = q.nbu, nU = q.npad / nbU;
  const int32_t u0 = chunk_ub(nU, p, c), u1 = chunk_ub(nU, p, c + 1);
  const int32_t r0 = u0 * nbU, rows = (u1 - u0) * nbU;
  const int tid = threadIdx.x;
  double* s = smem;
  double* stk = s + a.maxU;
  double* part = stk + ca.stk;
  const double* xs = ca.xs + voff;
  const int64_t* off = ca.off + 4 * ((int64_t)j * p + c);
  int CG = 0;
  const int32_t o = ca.nzo[(int64_t)j * p + c], ns = c + 1 < p ? ca.nzo[(int64_t)j * p + c + 1] - o : 0;
  if (ns > 0) {
    Chunk<T, S> A, B;
    const Geo gy = make_geo<S>(rows, ns);
    const T* Y = (const T*)ca.uy + off[2];
    const int32_t uf = chunk_ub(nU, p, c + 1);
    // K = ns_{c+1} + ... + ns_{p-2}: the stacked restricted first blocks
    const int32_t K = c + 2 < p ? ca.nzo[(int64_t)j * p + p - 1] - ca.nzo[(int64_t)j * p + c + 1] : 0;
    if (K > 0) {
      // s_c = f_{c+1}(nz_c) + UP_c [f_{c+2}(nz_{c+1}); ...; f_{p-1}(nz_{p-2})]
      const Geo gp = make_geo<S>(ns, K);
      const T* UP = (const T*)ca.up + off[3];
      prefetch_gemv<T, S, 0, false>(A, B, gp, UP, 0, nullptr);
      const int32_t ob = ca.nzo[(int64_t)j * p + c + 1];
      for (int32_t e = tid; e < K; e += blockDim.x) {
        // entry e belongs to boundary c2 (first block of chunk c2 + 1)
        int32_t c2 = c + 1;
        while (ca.nzo[(int64_t)j * p + c2 + 1] <= ob + e) ++c2;
        stk[e] = xs[(int64_t)chunk_ub(nU, p, c2 + 1) * nbU + ca.nz[ob + e]];
      }
      __syncthreads();
      const int CGp = run_gemv<T, S, 0, false>(A, B, gp, UP, 0, nullptr, stk, part);
      prefetch_gemv<T, S, 0, false>(A, B, gy, Y, 0, nullptr);
      __syncthreads();
      for (int32_t k = tid; k < ns; k += blockDim.x) s[k] = xs[uf * nbU + ca.nz[o + k]] + sum_parts(part, ns, CGp, k);
    } else {
      prefetch_gemv<T, S, 0, false>(A, B, gy, Y, 0, nullptr);
      for (int32_t k = tid; k < ns; k += blockDim.x) s[k] = xs[uf * nbU + ca.nz[o + k]];
    }
    __syncthreads();
    CG = run_gemv<T, S, 0, false>(A, B, gy, Y, 0, nullptr, s, part);
    __syncthreads();
  }
  for (int32_t r = tid; r < rows; r += blockDim.x) {
    const int32_t row = r0 + r;
    if (row >= n) continue;
    const double x = xs[row] + (ns > 0 ? sum_parts(part, rows, CG, r) : 0.0);
    out[ioff + row] = mode == 1 ? z1[ioff + row] - x : x;
  }
}

// One level of the product responses, for every subdomain: P_c(:, w0 ..) =
// P_c(:, 0 .. w0) P_nx, with P_c(:, 0 .. w0) the single-chunk block
// (upper: P = UP, nx = c + 1, rows ns_c, w0 = ns_{c+1}, P_nx ns_{c+1} x K_{c+1};
// lower: P = LP, nx = c - 1, rows nsl_c, w0 = nsl_{c-1}, P_nx nsl_{c-1} x
// (nsl_1 + ... + nsl_{c-2})).  FP64 accumulation, one thread per output entry.
template <class T>
__global__ void k_chunk_products(const SubInfo* __restrict__ subs, const int64_t* __restrict__ off,
                                 const int32_t* __restrict__ cnt, int32_t p, int32_t c, int upper, T* P) {
  const int32_t j = blockIdx.y;
  const SubInfo q = subs[j];
  if (q.n == 0) return;
  const int32_t* z = cnt + (int64_t)j * p;  // upper: coupling columns; lower: coupled carry positions
  int32_t rows, w0, cols, nx;
  if (upper) {
    rows = z[c + 1] - z[c];
    w0 = z[c + 2] - z[c + 1];
    cols = z[p - 1] - z[c + 2];
    nx = c + 1;
  } else {
    rows = z[c + 1] - z[c];
    w0 = z[c] - z[c - 1];
    cols = z[c - 1] - z[1];
    nx = c - 1;
  }
  const int64_t total = (int64_t)rows * cols;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int32_t r = (int32_t)(e % rows);
  const int64_t col = e / rows;
  const int slot = upper ? 3 : 1;
  T* Pc = P + off[4 * ((int64_t)j * p + c) + slot];
  const T* Px = P + off[4 * ((int64_t)j * p + nx) + slot];
  double acc = 0.0;
  for (int32_t k = 0; k < w0; ++k) acc += (double)Pc[(int64_t)k * rows + r] * (double)Px[col * w0 + k];
  Pc[((int64_t)w0 + col) * rows + r] = (T)acc;
}

// Coupling columns of each chunk boundary: flags[(j p + c) ld + k] = 1 if
// column k of U_{b,b+1}, b = u_{c+1} - 1, holds a nonzero (ld: the largest
// upper block size, a stride shared by every interior).
template <class T>
__global__ void k_chunk_nzcols(const SubInfo* __restrict__ subs, const T* __restrict__ u12_all, int32_t p,
                               int32_t ld, uint8_t* __restrict__ flags) {
  const int32_t j = blockIdx.x / (p - 1), c = blockIdx.x % (p - 1);
  const SubInfo q = subs[j];
  const int32_t nbU = q.nbu;
  uint8_t* f = flags + ((int64_t)j * p + c) * ld;
  if (q.n == 0) {
    for (int32_t k = threadIdx.x; k < nbU; k += blockDim.x) f[k] = 0;
    return;
  }
  const int32_t nU = q.npad / nbU, b = chunk_ub(nU, p, c + 1) - 1;
  const T* M = u12_all + q.u_off + (int64_t)b * nbU * nbU;
  for (int32_t k = threadIdx.x; k < nbU; k += blockDim.x) {
    bool nzc = false;
    for (int32_t r = 0; r < nbU && !nzc; ++r) nzc = M[(int64_t)k * nbU + r] != T(0);
    f[k] = nzc ? 1 : 0;
  }
}

// Zero rows of the lower block matrices: flags[blk * klmax + r] = 1 if row
// nbl + r of block blk's [inv(L11); L21 inv(L11)] is zero (its carry entry
// passes through the block unchanged).
template <class T>
__global__ void k_lower_zero_rows(const LBlk* __restrict__ lb, const SubInfo* __restrict__ subs,
                                  const T* __restrict__ lmat, int32_t klmax, uint8_t* __restrict__ flags) {
  const LBlk L = lb[blockIdx.x];
  const SubInfo q = subs[L.sub];
  const int32_t nbL = q.nbl, W = nbL + q.kl;
  const T* M = lmat + L.moff;
  for (int32_t r = threadIdx.x; r < q.kl; r += blockDim.x) {
    bool zero = true;
    for (int32_t k = 0; k < nbL && zero; ++k) zero = M[(int64_t)k * W + nbL + r] == T(0);
    flags[(int64_t)blockIdx.x * klmax + r] = zero ? 1 : 0;
  }
}

// One workgroup per aggregate: t = y2 - F z1 on the aggregate's rows, then
// x2 = S_i^{-1} t with S_i^{-1} column-major.  Thread (r, cs) owns row r of
// the GEMV and column chunk cs (Rp rows, CS = 1024 / Rp chunks); up to 128
// rows, a chunk fits kIfPref registers and is loaded before the gather of t
// (it does not depend on t), so the two memory latencies overlap.  The
// chunk partials meet in LDS in a fixed order.
constexpr int kIfPref = 16;

// With a coarse space (cz.t non-null) the kernel is the last step of the
// two-level interface solve: t comes precomputed (with y = E_c^{-1} Z^T t
// already formed), the block solve acts on r = t - (S Z) y and the coarse
// part Z y is added to the result.
struct CoarseApply {
  const double* t;       // separator vector t = y2 - F z1
  const double* y;       // coarse solution
  const int32_t* szp;    // S Z, CSR over separator rows
  const int32_t* szc;
  const double* szv;
  const int32_t* piece;  // per separator position
  const double* z0;
  const double* z1;
  const int32_t* p0;     // per piece: constant / linear column (-1 none)
  const int32_t* p1;
};

template <class T>
__global__ void __launch_bounds__(1024)
k_interface_solve(int32_t n_int, const int32_t* __restrict__ agg_off, const int32_t* __restrict__ f_rowptr,
                  const int32_t* __restrict__ f_colidx, const double* __restrict__ f_vals,
                  const int64_t* __restrict__ sinv_off, const T* __restrict__ sinv, const float* __restrict__ scale,
                  int scaled, const double* __restrict__ y, const double* __restrict__ z1, double* __restrict__ out,
                  CoarseApply cz, const int32_t* __restrict__ live, const int32_t* __restrict__ agg_sys) {
  __shared__ double t[1024];
  __shared__ double part[1024];
  const int i = blockIdx.x;
  if (live && !live[agg_sys[i]]) return;
  const int32_t a0 = agg_off[i], s = agg_off[i + 1] - a0;
  const int tid = threadIdx.x;
  const T* M = sinv + sinv_off[i];
  const int Rp = s <= 64 ? 64 : (s <= 128 ? 128 : (s <= 256 ? 256 : 1024));
  const int CS = 1024 / Rp;
  const int r = tid % Rp, cs = tid / Rp;
  const int32_t kb = (int32_t)((int64_t)s * cs / CS), ke = (int32_t)((int64_t)s * (cs + 1) / CS);
  const bool pref = s <= 128;  // then ke - kb <= 128 / 8 = kIfPref
  double mv[kIfPref];
  if (pref) {
#pragma unroll
    for (int q = 0; q < kIfPref; ++q) {
      const int32_t k = kb + q;
      mv[q] = (r < s && k < ke) ? ld(M + (int64_t)k * s + r) : 0.0;
    }
  }
  // t = y2 - F z1 (or t - S Z y with a coarse space) on the aggregate's
  // rows: each wave takes kIfRows rows at a time, its lanes load the rows'
  // entries and their vector values together (two memory rounds for all of
  // them), and each row's terms are summed by a fixed butterfly over the
  // wave's lanes before they are subtracted
  {
    const int lane = tid & 63, wave = tid >> 6, nw = (int)(blockDim.x >> 6);
    const int32_t* rp = cz.t ? cz.szp : f_rowptr;
    const int32_t* cix = cz.t ? cz.szc : f_colidx;
    const double* val = cz.t ? cz.szv : f_vals;
    const double* vec = cz.t ? cz.y : z1;
    for (int32_t q0 = wave; q0 < s; q0 += nw * kIfRows) {
      int32_t e0[kIfRows], e1[kIfRows];
      double w[kIfRows], x[kIfRows], acc[kIfRows];
#pragma unroll
      for (int g = 0; g < kIfRows; ++g) {
        const int32_t q = q0 + g * nw;
        const int32_t row = a0 + min(q, s - 1);
        e0[g] = q < s ? rp[row] : 0;
        e1[g] = q < s ? rp[row + 1] : 0;
        acc[g] = q < s ? (cz.t ? cz.t[row] : y[n_int + row]) : 0.0;
      }
#pragma unroll
      for (int g = 0; g < kIfRows; ++g) {
        const int32_t e = e0[g] + lane;
        const bool in = e < e1[g];
        w[g] = in ? val[e] : 0.0;
        x[g] = in ? vec[cix[e]] : 0.0;
      }
#pragma unroll
      for (int g = 0; g < kIfRows; ++g) {
        const int32_t q = q0 + g * nw;
        if (q >= s) continue;
        double sum = w[g] * x[g];
        // entries past the first 64 (rare): the next ones, 64 at a time
        for (int32_t eb = e0[g] + 64; eb < e1[g]; eb += 64) {
          const int32_t e = eb + lane;
          if (e < e1[g]) sum += val[e] * vec[cix[e]];
        }
        for (int off = 32; off >= 1; off >>= 1) sum += __shfl_xor(sum, off);
        if (lane == 0) t[q] = acc[g] - sum;
      }
    }
  }
  __syncthreads();
  // Z y on row `row` (separator position), 0 without a coarse space
  auto zy = [&](int32_t row) -> double {
    if (!cz.t) return 0.0;
    const int32_t pc = cz.piece[row];
    if (pc < 0) return 0.0;
    const int32_t c1 = cz.p1[pc];
    return cz.z0[row] * cz.y[cz.p0[pc]] + (c1 >= 0 ? cz.z1[row] * cz.y[c1] : 0.0);
  };
  if (pref) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kIfPref; ++q)
      if (kb + q < ke) acc += mv[q] * t[kb + q];
    part[cs * Rp + r] = acc;
    __syncthreads();
    if (cs == 0 && r < s) {
      double acc2 = 0.0;
      for (int c = 0; c < CS; ++c) acc2 += part[c * Rp + r];
      if (scaled) acc2 *= (double)scale[i];
      out[n_int + a0 + r] = acc2 + zy(a0 + r);
    }
    return;
  }
  for (int32_t rb = 0; rb < s; rb += Rp) {
    const int32_t row = rb + r;
    double acc = 0.0;
    if (row < s)
      for (int32_t k = kb; k < ke; ++k) acc += ld(M + (int64_t)k * s + row) * t[k];
    part[cs * Rp + r] = acc;
    __syncthreads();
    if (cs == 0 && row < s) {
      double acc2 = 0.0;
      for (int c = 0; c < CS; ++c) acc2 += part[c * Rp + r];
      if (scaled) acc2 *= (double)scale[i];
      out[n_int + a0 + row] = acc2 + zy(a0 + row);
    }
    __syncthreads();
  }
}

__global__ void k_permute(const int32_t* __restrict__ perm, const double* __restrict__ in, double* __restrict__ out,
                          int32_t n, int inverse, const double* __restrict__ scale) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int32_t o = perm[r];
  if (inverse) out[o] = in[r];
  else out[r] = scale ? in[o] * scale[o] : in[o];
}

}  // namespace

size_t sweep_smem_bytes(int32_t maxW, int32_t maxU) {
  return sizeof(double) * (size_t)(2 * maxW + 2 * maxU + kWaves * std::max(maxW, maxU));
}

template <class T, int S, bool Z>
static void launch_sweep(const SweepArgs& a, int m, size_t smem, const double* yin, double* out, int mode,
                         const double* x2, const double* z1, hipStream_t s) {
  // raise the kernel's dynamic-LDS limit once per size (the setup's own
  // sweeps do it before any caller could capture an apply in a graph)
  static size_t raised = 64 * 1024;
  if (smem > raised) {
    ADDNS_HIP(hipFuncSetAttribute((const void*)k_interior_solve<T, S, Z>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    raised = smem;
  }
  k_interior_solve<T, S, Z><<<m, kSweepThreads, smem, s>>>(a, yin, out, mode, x2, z1);
}

template <class T, bool Z>
static void dispatch_sweep(int S, const SweepArgs& a, int m, size_t smem, const double* yin, double* out, int mode,
                           const double* x2, const double* z1, hipStream_t s) {
  switch (S) {
    case 1: launch_sweep<T, 1, Z>(a, m, smem, yin, out, mode, x2, z1, s); break;
    case 2: launch_sweep<T, 2, Z>(a, m, smem, yin, out, mode, x2, z1, s); break;
    case 3: launch_sweep<T, 3, Z>(a, m, smem, yin, out, mode, x2, z1, s); break;
    case 4: launch_sweep<T, 4, Z>(a, m, smem, yin, out, mode, x2, z1, s); break;
    case 5: launch_sweep<T, 5, Z>(a, m, smem, yin, out, mode, x2, z1, s); break;
    default: throw ArgError("sweep row slots out of range");
  }
}

static SweepArgs sweep_args(const addns_precond* pc) {
  const Plan& pl = pc->plan;
  SweepArgs a{};
  a.maxW = pl.maxW;
  a.maxU = pl.nbU;
  a.subs = pc->subs.as<SubInfo>();
  a.lb = pc->lblks.as<LBlk>();
  a.ub = pc->ublks.as<UBlk>();
  a.lperm = pc->lperm.as<int32_t>();
  a.lmat = pc->lmat.p;
  a.uinv = pc->uinv.p;
  a.u12 = pc->u12.p;
  a.e_rowptr = pc->e_rowptr.as<int32_t>();
  a.e_colidx = pc->e_colidx.as<int32_t>();
  a.e_vals = pc->e_vals.as<double>();
  return a;
}

static void run_sweep(const addns_precond* pc, const SweepArgs& a, int grid, const double* yin, double* out, int mode,
                      const double* x2, const double* z1, hipStream_t s) {
  const Plan& pl = pc->plan;
  const size_t smem = sweep_smem_bytes(pl.maxW, pl.nbU);
  if (smem > 160 * 1024 || pl.nbU > kSweepThreads)
    throw ArgError("interior bandwidth too large for the LDS-staged sweep");
  const int S = std::min(kSweepMaxSlots, (std::max(pl.maxW, pl.nbU) + 63) / 64);
  // zero-slot skipping is a tile choice of the autotuner: skipped slots hold
  // exact zeros, so both forms give bitwise the same result
  const bool z = pc->zero_skip != 0;
  if (pc->interior_prec == P64) {
    if (z) dispatch_sweep<double, true>(S, a, grid, smem, yin, out, mode, x2, z1, s);
    else dispatch_sweep<double, false>(S, a, grid, smem, yin, out, mode, x2, z1, s);
  } else {
    if (z) dispatch_sweep<float, true>(S, a, grid, smem, yin, out, mode, x2, z1, s);
    else dispatch_sweep<float, false>(S, a, grid, smem, yin, out, mode, x2, z1, s);
  }
}

// ---- chunked sweep ---------------------------------------------------------
static int32_t chunk_stack_words(int p, int32_t klmax, int32_t maxU) {
  return std::max(0, p - 2) * std::max(klmax, maxU);
}

static size_t chunk_smem_bytes(int32_t maxW, int32_t maxU, int S, int32_t stk) {
  return sizeof(double) * (size_t)(2 * maxW + 2 * maxU + stk +
                                   std::max<int64_t>((int64_t)kWaves * std::max(maxW, maxU), 1024 * S));
}

template <class T>
struct TypeTag {
  using type = T;
};

// f(TypeTag<T>, integral_constant<int, S>, integral_constant<bool, Z>) for the
// handle's storage type, row slots and zero-slot choice
template <class F>
static void with_sweep_shape(const addns_precond* pc, F&& f) {
  const Plan& pl = pc->plan;
  const int S = std::min(kSweepMaxSlots, (std::max(pl.maxW, pl.nbU) + 63) / 64);
  auto by_s = [&](auto tt, auto zz) {
    switch (S) {
      case 1: f(tt, std::integral_constant<int, 1>{}, zz); break;
      case 2: f(tt, std::integral_constant<int, 2>{}, zz); break;
      case 3: f(tt, std::integral_constant<int, 3>{}, zz); break;
      case 4: f(tt, std::integral_constant<int, 4>{}, zz); break;
      case 5: f(tt, std::integral_constant<int, 5>{}, zz); break;
      default: throw ArgError("sweep row slots out of range");
    }
  };
  auto by_z = [&](auto tt) {
    if (pc->zero_skip) by_s(tt, std::true_type{});
    else by_s(tt, std::false_type{});
  };
  if (pc->interior_prec == P64) by_z(TypeTag<double>{});
  else by_z(TypeTag<float>{});
}

template <class K>
static void raise_lds(K kernel, size_t smem) {
  if (smem > 64 * 1024)
    ADDNS_HIP(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
}

static ChunkArgs chunk_args(const addns_precond* pc) {
  ChunkArgs ca{};
  ca.p = pc->sweep_chunks;
  ca.klmax = pc->ch_klmax;
  ca.stk = chunk_stack_words(ca.p, ca.klmax, pc->plan.nbU);
  ca.off = pc->ch_off.as<int64_t>();
  ca.lx = pc->ch_lx.p;
  ca.lp = pc->ch_lp.p;
  ca.uy = pc->ch_uy.p;
  ca.up = pc->ch_up.p;
  ca.cz = pc->ch_cz.as<double>();
  ca.xs = pc->ch_xs.as<double>();
  ca.uin = pc->ch_uin.as<double>();
  ca.nz = pc->ch_nz.as<int32_t>();
  ca.nzo = pc->ch_nzo.as<int32_t>();
  ca.prow = pc->ch_prow.as<int32_t>();
  ca.np = pc->ch_np.as<int32_t>();
  ca.npo = pc->ch_npo.as<int32_t>();
  return ca;
}

static void run_chunked(const addns_precond* pc, const SweepArgs& a, const double* yin, double* out, int mode,
                        const double* x2, const double* z1, hipStream_t s) {
  const Plan& pl = pc->plan;
  const ChunkArgs ca = chunk_args(pc);
  const int grid = pl.m * ca.p;
  with_sweep_shape(pc, [&](auto tt, auto ss, auto zz) {
    using T = typename decltype(tt)::type;
    constexpr int S = decltype(ss)::value;
    constexpr bool Z = decltype(zz)::value;
    const size_t smem = chunk_smem_bytes(pl.maxW, pl.nbU, S, ca.stk);
    k_chunk_lower<T, S, Z><<<grid, kSweepThreads, smem, s>>>(a, ca, yin, mode, x2);
    k_chunk_upper<T, S, Z><<<grid, kSweepThreads, smem, s>>>(a, ca, mode);
    k_chunk_fix<T, S><<<grid, kSweepThreads, smem, s>>>(a, ca, mode, out, z1);
  });
}

int max_sweep_chunks(const Plan& pl) {
  int32_t p = 0;
  for (const SubInfo& q : pl.subs)
    if (q.n > 0) p = p == 0 ? q.npad / q.nbu : std::min(p, q.npad / q.nbu);
  return std::max(p, 1);
}

void release_chunked_sweep(addns_precond* pc) {
  pc->sweep_chunks = 1;
  pc->chunk_bytes = 0;
  for (DevBuf* d : {&pc->ch_off, &pc->ch_lx, &pc->ch_lp, &pc->ch_uy, &pc->ch_up, &pc->ch_cz, &pc->ch_xs, &pc->ch_uin,
                    &pc->ch_nz, &pc->ch_nzo, &pc->ch_prow, &pc->ch_np, &pc->ch_npo})
    d->reset();
}

// Offsets and response matrices of the chunked sweep with p chunks, swept on
// the handle's current factors (mode 3 of the chunk kernels, one workgroup per
// chunk range and unit).
void build_chunked_sweep(addns_precond* pc, int p, hipStream_t s) {
  const Plan& pl = pc->plan;
  if (p < 2 || p > max_sweep_chunks(pl)) throw ArgError("sweep_chunks exceeds the upper blocks of an interior");
  const int S = std::min(kSweepMaxSlots, (std::max(pl.maxW, pl.nbU) + 63) / 64);
  const int m = pl.m;
  const int fb = pc->interior_prec == P64 ? 8 : 4;
  int32_t klmax = 1;
  for (const SubInfo& q : pl.subs) klmax = std::max(klmax, q.kl);
  if (chunk_smem_bytes(pl.maxW, pl.nbU, S, chunk_stack_words(p, klmax, pl.nbU)) > 160 * 1024)
    throw ArgError("sweep_chunks too large for the chunk kernels' LDS");
  // coupling columns of every chunk boundary, from the stored U_{b,b+1},
  // and the zero rows of the lower block matrices with the gather indices
  // (for the pure carry positions below): one wait for both
  const int32_t nlb = (int32_t)pl.lblks.size();
  std::vector<uint8_t> flags((size_t)m * p * pl.nbU, 0);
  std::vector<uint8_t> zrow((size_t)std::max(nlb, 1) * klmax, 0);
  std::vector<int32_t> h_lperm((size_t)std::max<int64_t>(pl.lperm_total, 1));
  {
    DevBuf d_flags, d_z;
    d_flags.alloc(flags.size());
    d_z.alloc(zrow.size());
    ADDNS_HIP(hipMemsetAsync(d_flags.p, 0, flags.size(), s));
    if (pc->interior_prec == P64)
      k_chunk_nzcols<double><<<m * (p - 1), 256, 0, s>>>(pc->subs.as<SubInfo>(), pc->u12.as<double>(), p,
                                                         pl.nbU, d_flags.as<uint8_t>());
    else
      k_chunk_nzcols<float><<<m * (p - 1), 256, 0, s>>>(pc->subs.as<SubInfo>(), pc->u12.as<float>(), p,
                                                        pl.nbU, d_flags.as<uint8_t>());
    if (nlb > 0) {
      if (pc->interior_prec == P64)
        k_lower_zero_rows<double><<<nlb, 256, 0, s>>>(pc->lblks.as<LBlk>(), pc->subs.as<SubInfo>(), pc->lmat.as<double>(),
                                                      klmax, d_z.as<uint8_t>());
      else
        k_lower_zero_rows<float><<<nlb, 256, 0, s>>>(pc->lblks.as<LBlk>(), pc->subs.as<SubInfo>(), pc->lmat.as<float>(),
                                                     klmax, d_z.as<uint8_t>());
    }
    ADDNS_HIP(hipMemcpyAsync(flags.data(), d_flags.p, flags.size(), hipMemcpyDeviceToHost, s));
    if (nlb > 0) ADDNS_HIP(hipMemcpyAsync(zrow.data(), d_z.p, zrow.size(), hipMemcpyDeviceToHost, s));
    if (pl.lperm_total > 0)
      ADDNS_HIP(hipMemcpyAsync(h_lperm.data(), pc->lperm.p, sizeof(int32_t) * pl.lperm_total, hipMemcpyDeviceToHost, s));
    ADDNS_HIP(hipStreamSynchronize(s));
  }
  std::vector<int32_t> nz, nzo((size_t)m * p + 1, 0);
  for (int32_t j = 0; j < m; ++j)
    for (int32_t c = 0; c < p; ++c) {
      nzo[(size_t)j * p + c] = (int32_t)nz.size();
      if (c + 1 < p && pl.subs[j].n > 0)
        for (int32_t k = 0; k < pl.subs[j].nbu; ++k)
          if (flags[((size_t)j * p + c) * pl.nbU + k]) nz.push_back(k);
    }
  nzo[(size_t)m * p] = (int32_t)nz.size();
  // pure carry positions at every lower chunk boundary: follow each window
  // position through the blocks
  std::vector<int32_t> prow((size_t)m * p * klmax, -1), np, npo((size_t)m * p + 1, 0);
  for (int32_t j = 0; j < m; ++j) {
    const SubInfo& q = pl.subs[j];
    std::vector<std::vector<int32_t>> lists(p);
    if (q.n > 0) {
      const int32_t KL = q.kl, nbL = q.nbl, W = nbL + KL, nU = q.npad / q.nbu, nL = q.npad / nbL;
      std::vector<uint8_t> pure(KL, 1), npure(KL);
      std::vector<int32_t> row(KL), nrow(KL);
      for (int32_t r = 0; r < KL; ++r) row[r] = r;
      int32_t cnext = 1;
      for (int32_t b = 0; b <= nL; ++b) {
        // at chunk boundary c (block 2 u_c) record the state before block b
        while (cnext < p && 2 * chunk_ub(nU, p, cnext) == b) {
          for (int32_t r = 0; r < KL; ++r) {
            if (pure[r]) prow[((size_t)j * p + cnext) * klmax + r] = row[r];
            else lists[cnext].push_back(r);
          }
          ++cnext;
        }
        if (b == nL) break;
        const LBlk& L = pl.lblks[(size_t)q.lblk0 + b];
        const uint8_t* zr = &zrow[((size_t)q.lblk0 + b) * klmax];
        for (int32_t r = 0; r < KL; ++r) {
          const int32_t pos = h_lperm[(size_t)L.poff + nbL + r];
          if (pos < 0 || pos >= W) throw HipError("lower gather index out of range");
          const bool src_pure = pos >= KL ? true : pure[pos] != 0;
          npure[r] = (zr[r] && src_pure) ? 1 : 0;
          nrow[r] = pos >= KL ? b * nbL + pos : row[pos];
        }
        pure.swap(npure);
        row.swap(nrow);
      }
    }
    for (int32_t c = 0; c < p; ++c) {
      npo[(size_t)j * p + c] = (int32_t)np.size();
      np.insert(np.end(), lists[c].begin(), lists[c].end());
    }
  }
  npo[(size_t)m * p] = (int32_t)np.size();
  std::vector<int64_t> off((size_t)4 * m * p, 0);
  std::vector<int32_t> jl, ju;
  int64_t nlx = 0, nlp = 0, nuy = 0, nup = 0;
  for (int32_t j = 0; j < m; ++j) {
    const SubInfo& q = pl.subs[j];
    if (q.n == 0) continue;
    const int32_t nU = q.npad / q.nbu, nbU = q.nbu;
    const int32_t* zl = &npo[(size_t)j * p];
    for (int32_t c = 0; c < p; ++c) {
      const int32_t rows = (int32_t)(((int64_t)nU * (c + 1) / p - (int64_t)nU * c / p) * nbU);
      if (rows > 1024 * S) throw ArgError("sweep chunk too tall for the chunk kernels' GEMVs");
      int64_t* o = &off[(size_t)4 * ((int64_t)j * p + c)];
      const int32_t nsl = zl[c + 1] - zl[c];
      if (c >= 1) {
        o[0] = nlx;
        nlx += (int64_t)rows * nsl;
      }
      if (c >= 2) {
        o[1] = nlp;
        nlp += (int64_t)nsl * (zl[c] - zl[1]);
      }
      const int32_t* z = &nzo[(size_t)j * p];
      if (c + 1 < p) {
        o[2] = nuy;
        nuy += (int64_t)rows * (z[c + 1] - z[c]);
      }
      if (c + 2 < p) {
        o[3] = nup;
        nup += (int64_t)(z[c + 1] - z[c]) * (z[p - 1] - z[c + 1]);
      }
    }
    // single chunks: lower c >= 1 (X_c, and T_c into block 0 of LP_{c+1}),
    // upper c <= p - 2 (Y_c, and Yt_c into block 0 of UP_{c-1}); the longer
    // products follow from them (k_chunk_products)
    for (int32_t c = 1; c < p; ++c)
      for (int32_t u = 0; u < npo[(size_t)j * p + c + 1] - npo[(size_t)j * p + c]; ++u) jl.insert(jl.end(), {j, c, c + 1, u});
    for (int32_t c = 0; c + 1 < p; ++c)
      for (int32_t u = 0; u < nzo[(size_t)j * p + c + 1] - nzo[(size_t)j * p + c]; ++u)
        ju.insert(ju.end(), {j, c, c + 1, u});
  }
  // Every buffer is sized for the largest structure the plan admits (all nbu
  // columns coupled, no pure carry position), which depends on the plan and
  // p only: a refactor whose factors couple other columns or rows rebuilds
  // into the same allocations, so an apply captured before it stays valid.
  int64_t cap_nz = 0, cap_np = 0, cap[4] = {0, 0, 0, 0};
  for (const SubInfo& q : pl.subs) {
    if (q.n == 0) continue;
    const int64_t nU = q.npad / q.nbu, kl = q.kl, nb = q.nbu;
    cap_nz += (int64_t)(p - 1) * nb;
    cap_np += (int64_t)(p - 1) * kl;
    for (int32_t c = 0; c < p; ++c) {
      const int64_t rows = (nU * (c + 1) / p - nU * c / p) * nb;
      if (c >= 1) cap[0] += rows * kl;
      if (c >= 2) cap[1] += kl * (c - 1) * kl;
      if (c + 1 < p) cap[2] += rows * nb;
      if (c + 2 < p) cap[3] += nb * (p - 2 - c) * nb;
    }
  }
  const int64_t cnt[4] = {nlx, nlp, nuy, nup};
  if ((int64_t)nz.size() > cap_nz || (int64_t)np.size() > cap_np || nlx > cap[0] || nlp > cap[1] || nuy > cap[2] ||
      nup > cap[3])
    throw HipError("chunked sweep structure exceeds its plan bound");
  nz.resize((size_t)cap_nz, 0);
  np.resize((size_t)cap_np, 0);
  pc->sweep_chunks = p;
  pc->ch_klmax = klmax;
  pc->chunk_bytes = (int64_t)fb * (nlx + nlp + nuy + nup);
  pc->ch_off.upload(off, s);
  // the chunk GEMVs' last row slot may read up to 64 * 5 rows past a
  // matrix; the zeroed rest of the allocation (unused capacity and a tail)
  // keeps that overrun inside it
  const int64_t tail = kSweepOverrunBytes;
  DevBuf* mats[4] = {&pc->ch_lx, &pc->ch_lp, &pc->ch_uy, &pc->ch_up};
  for (int i = 0; i < 4; ++i) {
    mats[i]->alloc((size_t)(fb * cap[i] + tail));
    ADDNS_HIP(hipMemsetAsync(static_cast<char*>(mats[i]->p) + fb * cnt[i], 0, mats[i]->bytes - fb * cnt[i], s));
  }
  pc->ch_cz.alloc(sizeof(double) * (size_t)m * p * klmax);
  pc->ch_xs.alloc(sizeof(double) * (size_t)std::max<int64_t>(pl.npad_total, 1));
  pc->ch_uin.alloc(sizeof(double) * (size_t)std::max<int64_t>(pl.npad_total, 1));
  pc->ch_nz.upload(nz, s);
  pc->ch_nzo.upload(nzo, s);
  pc->ch_prow.upload(prow, s);
  pc->ch_np.upload(np, s);
  pc->ch_npo.upload(npo, s);
  DevBuf d_jl, d_ju;
  d_jl.upload(jl, s);
  d_ju.upload(ju, s);
  SweepArgs a = sweep_args(pc);
  a.ypad = pc->ypad.as<double>();
  ChunkArgs ca = chunk_args(pc);
  with_sweep_shape(pc, [&](auto tt, auto ss, auto zz) {
    using T = typename decltype(tt)::type;
    constexpr int S2 = decltype(ss)::value;
    constexpr bool Z = decltype(zz)::value;
    const size_t smem = chunk_smem_bytes(pl.maxW, pl.nbU, S2, ca.stk);
    raise_lds(k_chunk_lower<T, S2, Z>, smem);
    raise_lds(k_chunk_upper<T, S2, Z>, smem);
    raise_lds(k_chunk_fix<T, S2>, smem);
    ca.job = d_jl.as<int32_t>();
    if (!jl.empty()) k_chunk_lower<T, S2, Z><<<(int)(jl.size() / 4), kSweepThreads, smem, s>>>(a, ca, nullptr, 3, nullptr);
    ca.job = d_ju.as<int32_t>();
    if (!ju.empty()) k_chunk_upper<T, S2, Z><<<(int)(ju.size() / 4), kSweepThreads, smem, s>>>(a, ca, 3);
    // UP_c = [R_{c+1}, R_{c+1} UP_{c+1}] for c = p-4 down to 0;
    // LP_c = [T_{c-1}, T_{c-1} LP_{c-1}] for c = 3 up to p-1
    for (int32_t c = p - 4; c >= 0; --c) {
      int64_t tot = 1;
      for (int32_t j = 0; j < m; ++j) {
        const int32_t* z = &nzo[(size_t)j * p];
        tot = std::max<int64_t>(tot, (int64_t)(z[c + 1] - z[c]) * (z[p - 1] - z[c + 2]));
      }
      k_chunk_products<T><<<dim3((unsigned)((tot + 255) / 256), m), 256, 0, s>>>(
          pc->subs.as<SubInfo>(), pc->ch_off.as<int64_t>(), pc->ch_nzo.as<int32_t>(), p, c, 1, (T*)pc->ch_up.p);
    }
    for (int32_t c = 3; c < p; ++c) {
      int64_t tot = 1;
      for (int32_t j = 0; j < m; ++j) {
        const int32_t* zl = &npo[(size_t)j * p];
        tot = std::max<int64_t>(tot, (int64_t)(zl[c + 1] - zl[c]) * (zl[c - 1] - zl[1]));
      }
      k_chunk_products<T><<<dim3((unsigned)((tot + 255) / 256), m), 256, 0, s>>>(
          pc->subs.as<SubInfo>(), pc->ch_off.as<int64_t>(), pc->ch_npo.as<int32_t>(), p, c, 0, (T*)pc->ch_lp.p);
    }
  });
  ADDNS_HIP(hipGetLastError());
  ADDNS_HIP(hipStreamSynchronize(s));
}

void launch_interior_solve(const addns_precond* pc, const double* yin, double* out, int second, const double* x2,
                           const double* z1, hipStream_t s, double* work) {
  const Plan& pl = pc->plan;
  if (pl.m == 0 || pl.n_int == 0) return;
  SweepArgs a = sweep_args(pc);
  a.ypad = work ? work : (second ? pc->zpad.as<double>() : pc->ypad.as<double>());
  if (pc->mask_live && pc->sweep_chunks <= 1) {
    a.live = pc->mask_live;
    a.unit_sys = pc->mask_sub.as<int32_t>();
  }
  if (pc->sweep_chunks > 1) run_chunked(pc, a, yin, out, second ? 1 : 0, x2, z1, s);
  else run_sweep(pc, a, pl.m, yin, out, second ? 1 : 0, x2, z1, s);
}

void launch_column_solves(const addns_precond* pc, int32_t npairs, const int32_t* pair_sub, const int32_t* pair_col,
                          const int64_t* pair_off, double* scratch, double* out, hipStream_t s) {
  if (npairs == 0) return;
  SweepArgs a = sweep_args(pc);
  a.ypad = scratch;
  a.pair_sub = pair_sub;
  a.pair_col = pair_col;
  a.pair_off = pair_off;
  run_sweep(pc, a, npairs, nullptr, out, 2, nullptr, nullptr, s);
}

void launch_coarse_column_solves(const addns_precond* pc, int32_t npairs, const int32_t* pair_sub,
                                 const int32_t* pair_col, const int64_t* pair_off, double* scratch, double* out,
                                 int rhs_given, hipStream_t s) {
  if (npairs == 0) return;
  SweepArgs a = sweep_args(pc);
  a.pair_rhs_given = rhs_given;
  a.ypad = scratch;
  a.pair_sub = pair_sub;
  a.pair_col = pair_col;
  a.pair_off = pair_off;
  a.cz_piece = pc->cz_piece.as<int32_t>();
  a.cz_z0 = pc->cz_z0.as<double>();
  a.cz_z1 = pc->cz_z1.as<double>();
  a.cz_colp = pc->cz_colp.as<int32_t>();
  a.cz_colk = pc->cz_colk.as<int32_t>();
  run_sweep(pc, a, npairs, nullptr, out, 2, nullptr, nullptr, s);
}

void launch_interface_solve(const addns_precond* pc, const double* y, const double* z1, double* out, hipStream_t s) {
  const Plan& pl = pc->plan;
  if (pl.k == 0) return;
  CoarseApply cz{};
  if (pc->coarse_nc > 0) {
    cz.t = pc->cz_t.as<double>();
    cz.y = pc->cz_y.as<double>();
    cz.szp = pc->cz_szp.as<int32_t>();
    cz.szc = pc->cz_szc.as<int32_t>();
    cz.szv = pc->cz_szv.as<double>();
    cz.piece = pc->cz_piece.as<int32_t>();
    cz.z0 = pc->cz_z0.as<double>();
    cz.z1 = pc->cz_z1.as<double>();
    cz.p0 = pc->cz_p0.as<int32_t>();
    cz.p1 = pc->cz_p1.as<int32_t>();
  }
  const int32_t* ao = pc->agg_off.as<int32_t>();
  const int32_t* fr = pc->f_rowptr.as<int32_t>();
  const int32_t* fc = pc->f_colidx.as<int32_t>();
  const double* fv = pc->f_vals.as<double>();
  const int64_t* so = pc->sinv_off.as<int64_t>();
  if (pc->schur_prec == P64)
    k_interface_solve<double><<<pl.k, 1024, 0, s>>>(pl.n_int, ao, fr, fc, fv, so, pc->sinv.as<double>(), nullptr, 0, y,
                                                   z1, out, cz, pc->mask_live, pc->mask_agg.as<int32_t>());
  else if (pc->schur_prec == P32)
    k_interface_solve<float><<<pl.k, 1024, 0, s>>>(pl.n_int, ao, fr, fc, fv, so, pc->sinv.as<float>(), nullptr, 0, y,
                                                  z1, out, cz, pc->mask_live, pc->mask_agg.as<int32_t>());
  else
    k_interface_solve<__half><<<pl.k, 1024, 0, s>>>(pl.n_int, ao, fr, fc, fv, so, pc->sinv.as<__half>(),
                                                   pc->sinv_scale.as<float>(), 1, y, z1, out, cz, pc->mask_live,
                                                   pc->mask_agg.as<int32_t>());
}

void launch_permute(const int32_t* perm, const double* in, double* out, int32_t n, int inverse, const double* scale,
                    hipStream_t s) {
  if (n > 0) k_permute<<<(n + 255) / 256, 256, 0, s>>>(perm, in, out, n, inverse, scale);
}

}  // namespace addns
