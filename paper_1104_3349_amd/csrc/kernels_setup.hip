// Setup kernels (Algorithm 1 and the exact interior factorisations):
//   - row scaling by the largest absolute entry (section 5);
//   - gathers of C~ into its permuted CSR, band storage of each A_jj, and
//     dense aggregate blocks;
//   - band LU with partial pivoting of every A_jj (one workgroup each);
//   - conversion of the band factors into block-bidiagonal sweeps whose
//     diagonal blocks are stored inverted (the apply then runs dense
//     triangular GEMVs instead of a row-by-row recurrence);
//   - mini Schur complements S_i = G_i - F_i D_{r_i}^{-1} E_i: Gaussian
//     elimination of [D_{r_i} | E_i], back substitution, and the product
//     F_i X_i on FP64 matrix cores (MFMA); then S_i^{-1} by Gauss-Jordan
//     with partial pivoting, stored in the requested precision.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <stdexcept>

#include "precond.h"

namespace addns {
namespace {

constexpr int kSetupThreads = 1024;
constexpr int kMaxBandLU = 1024;  // KL + KU limit of k_band_lu (the sweep's own limit is the same)
constexpr double kPivotTie = 1e-12;  // band LU: candidates this close to the largest count as equal

__global__ void k_row_scale(const int32_t* __restrict__ rowptr, const double* __restrict__ vals, int32_t N,
                            int scale, double* __restrict__ R) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  if (!scale) {
    R[i] = 1.0;
    return;
  }
  double mx = 0.0;
  for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) mx = fmax(mx, fabs(vals[e]));
  R[i] = mx > 0.0 ? 1.0 / mx : 1.0;
}

__global__ void k_gather_scaled(const int32_t* __restrict__ src, const int32_t* __restrict__ orow,
                                const double* __restrict__ vals, const double* __restrict__ R, int64_t n,
                                double* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = R[orow[t]] * vals[src[t]];
}

__global__ void k_gather(const int32_t* __restrict__ src, const double* __restrict__ in, int64_t n,
                         double* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = in[src[t]];
}

__global__ void k_scatter(const int64_t* __restrict__ dst, const int32_t* __restrict__ src,
                          const double* __restrict__ cpv, int64_t n, double* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[dst[t]] = cpv[src[t]];
}

__global__ void k_band_pad_identity(const SubInfo* subs, double* ab) {
  const SubInfo q = subs[blockIdx.x];
  for (int32_t c = q.n + threadIdx.x; c < q.npad; c += blockDim.x)
    ab[q.band_off + (int64_t)c * q.ldab + q.kl + q.ku] = 1.0;
}

// ---------------------------------------------------------------------------
// Band LU with partial pivoting, one workgroup per interior block.  Band
// storage is column-major with leading dimension ldab = 2KL+KU+1; entry
// (r, c) lives at row KV + r - c of column c, KV = KL + KU, so the factor U
// may fill KL extra superdiagonals.  ipiv[j] = row swapped with row j at
// step j (subdomain-local).  info[sub] = first zero pivot + 1 (0 if none).
// tau > 0 makes it the threshold ILU used as an inexact interior solver in
// the experiments of section 5: at step j a multiplier whose entry before
// division is below tau ||A(:,j)||_2 is dropped (stored as zero, its row not
// updated), and so is an entry u_jk of the pivot row below tau ||A(:,k)||_2;
// the pivot is never dropped.  colnorm holds the column norms of the blocks
// before elimination (k_band_colnorm).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kSetupThreads)
k_band_lu(double* __restrict__ ab_all, int32_t* __restrict__ ipiv_all, const SubInfo* __restrict__ subs,
          int32_t* __restrict__ info, const double* __restrict__ colnorm_all, double tau) {
  const int sub = blockIdx.x;
  const SubInfo q = subs[sub];
  const int32_t n = q.npad, ldab = q.ldab, KL = q.kl, KU = q.ku;
  double* ab = ab_all + q.band_off;
  int32_t* ipiv = ipiv_all + q.vec_off;
  const double* cn = colnorm_all + q.vec_off;
  const int32_t KV = KL + KU;
  __shared__ double s_piv;
  __shared__ double s_top;
  __shared__ int32_t s_p;
  __shared__ int32_t s_ju;
  __shared__ int32_t s_info;
  __shared__ double s_l[kMaxBandLU + 1];  // multipliers of the current column
  __shared__ double s_u[kMaxBandLU];      // pivot row of U right of the diagonal
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    s_ju = 0;
    s_info = 0;
  }
  __syncthreads();
  for (int32_t j = 0; j < n; ++j) {
    const int32_t km = min(KL, n - 1 - j);
    double* colj = ab + (int64_t)j * ldab + KV;
    // pivot search over rows j..j+km: the first row whose magnitude is
    // within a relative kPivotTie of the largest (a rounding-independent
    // choice among equal candidates)
    if (wave == 0) {
      double best = 0.0;
      for (int32_t i = lane; i <= km; i += 64) best = fmax(best, fabs(colj[i]));
      for (int off = 32; off >= 1; off >>= 1) best = fmax(best, __shfl_xor(best, off));
      const double thr = (1.0 - kPivotTie) * best;
      int32_t bi = km + 1;
      for (int32_t i = lane; i <= km; i += 64)
        if (fabs(colj[i]) >= thr) {
          bi = i;
          break;
        }
      for (int off = 32; off >= 1; off >>= 1) bi = min(bi, __shfl_xor(bi, off));
      if (bi > km) bi = 0;  // an all-zero column: a zero pivot at row j
      if (lane == 0) {
        // a column without a nonzero candidate: with dropping (tau > 0) the
        // pivot becomes tau ||A(:, j)|| (compensation of the dropped fill);
        // the exact LU reports it
        double pv = colj[bi];
        if (pv == 0.0 && tau > 0.0) pv = tau * cn[j];
        s_p = bi;
        s_piv = pv;
        s_top = colj[0];
        ipiv[j] = j + bi;
        if (pv == 0.0 && s_info == 0) s_info = j + 1;
        int32_t ju = max(s_ju, min(j + KU + bi, n - 1));
        s_ju = ju;
      }
    }
    __syncthreads();
    const int32_t p = s_p;
    const double piv = s_piv;
    const int32_t ju = s_ju;
    if (piv != 0.0) {
      // multipliers of column j (after the row swap) and the swap of columns
      // j+1..ju; both also go to LDS for the update below
      const double rinv = 1.0 / piv;
      const double drop_l = tau * cn[j];
      for (int32_t i = tid; i <= km; i += blockDim.x) {
        if (i == 0) continue;
        const double a = (i == p) ? s_top : colj[i];
        const double l = fabs(a) < drop_l ? 0.0 : a * rinv;
        colj[i] = l;
        s_l[i] = l;
      }
      if (tid == 0) colj[0] = piv;
      for (int32_t c = j + 1 + tid; c <= ju; c += blockDim.x) {
        double* col = ab + (int64_t)c * ldab + KV + j - c;
        double a = col[0];
        if (p != 0) {
          const double b = col[p];
          col[p] = a;
          a = b;
        }
        if (fabs(a) < tau * cn[c]) a = 0.0;
        col[0] = a;
        s_u[c - j - 1] = a;
      }
    }
    __syncthreads();
    if (piv != 0.0 && km > 0) {
      // rank-1 update of rows 1..km of columns j+1..ju: every thread loads
      // its Q elements before it stores any (independent addresses)
      constexpr int Q = 24;  // two batches cover KL x (KL+KU) = 130 x 260 with 1024 threads
      const int32_t total = (ju - j) * km;
      for (int32_t base = 0; base < total; base += Q * (int32_t)blockDim.x) {
        double v[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int32_t t = base + q * (int32_t)blockDim.x + tid;
          const int32_t c = t / km, i = 1 + t % km;
          v[q] = t < total ? ab[(int64_t)(j + 1 + c) * ldab + KV - 1 - c + i] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int32_t t = base + q * (int32_t)blockDim.x + tid;
          const int32_t c = t / km, i = 1 + t % km;
          if (t < total) ab[(int64_t)(j + 1 + c) * ldab + KV - 1 - c + i] = v[q] - s_l[i] * s_u[c];
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) info[sub] = s_info;
}

// ---------------------------------------------------------------------------
// Blocked form of the same band LU (identical pivots and factor entries,
// bit for bit): panels of kPanel columns.  One wave factors a panel (rows
// j0 .. j0+KL+nb-1) with the rows in its registers and full-row interchanges
// inside the panel (getrf style); the panel's interchanges are then applied
// to the trailing columns j0+nb .. ju and the panel rows of those columns are
// solved with the panel's unit lower triangle (one thread per column, with
// the ILU drop of U entries); the rows below the panel receive one rank-nb
// update, each entry's terms subtracted in the unblocked elimination's order
// (a step that skipped a column contributes an exact zero).  Finally each
// panel column's multipliers are returned to band storage order (the later
// interchanges of the same panel undone), which is what the sweep conversion
// reads.  The trailing window is read and written once per panel instead of
// once per column.  Bands whose panel does not fit 4 x 64 rows per lane use
// the unblocked kernel.
// ---------------------------------------------------------------------------
constexpr int kPanel = 8;
static_assert(kNpadMultiple % kPanel == 0, "panels must tile every padded block");
// Threads of the blocked band LU: 12 waves (three a SIMD) leave each lane
// the registers that the lookahead needs (the panel in wave 0's registers
// next to the update tiles of the others) without spilling, and give the
// trailing update 11 waves.
constexpr int kLuThreads = 768;

__device__ inline double readlane_d(double x, int32_t l) {
  const int64_t bits = __double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)bits, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(bits >> 32), l);
  return __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
}

template <int CTRL, int ROW_MASK>
__device__ inline uint32_t dpp_umax_step(uint32_t v) {
  return max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false));
}

// Largest unsigned value over the wave (0 is the identity): a prefix maximum
// within each row of 16 lanes by DPP row shifts, then the row maxima
// combined by row broadcasts, read from lane 63.  Lanes whose DPP source
// does not exist receive 0.
__device__ inline uint32_t wave_umax(uint32_t x) {
  x = dpp_umax_step<0x111, 0xf>(x);  // row_shr:1
  x = dpp_umax_step<0x112, 0xf>(x);  // row_shr:2
  x = dpp_umax_step<0x114, 0xf>(x);  // row_shr:4
  x = dpp_umax_step<0x118, 0xf>(x);  // row_shr:8
  x = dpp_umax_step<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x = dpp_umax_step<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Largest value over the wave of non-negative, non-NaN doubles x, exactly:
// such doubles order as their bit patterns, so the maximum is the largest
// high word, then the largest low word among the lanes that hold it (32-bit
// integer steps instead of double ones).
__device__ inline double wave_max_nonneg(double x) {
  const uint64_t bits = (uint64_t)__double_as_longlong(x);
  const uint32_t hi = (uint32_t)(bits >> 32), lo = (uint32_t)bits;
  const uint32_t hmax = wave_umax(hi);
  const uint32_t lmax = wave_umax(hi == hmax ? lo : 0u);
  return __longlong_as_double((int64_t)(((uint64_t)hmax << 32) | lmax));
}

// The same panel factorisation with the panel in registers: lane l holds
// rows l + 64k (k < NS) of the kPanel columns (every padded block holds a
// multiple of kPanel columns, so panels are always full); the pivot search
// uses one max reduction and ballots, and the pivot row and row c reach
// every lane by readlane.  Per column c only the later columns are interchanged in
// registers: the earlier ones hold finished multipliers that the panel no
// longer reads, so their interchanges are applied afterwards in LDS (lane c
// replays the steps after c on its column, in order).  Each entry sees the
// same operations in the same order as with every interchange applied at
// its step, so the results are identical.
template <int NS>
__device__ __attribute__((always_inline)) inline void panel_regs(
    double* s_pan, int32_t prmax, int32_t prows, int32_t j0, int32_t n, int32_t KL, int32_t KU, int lane,
    double tau, const double* cn, int32_t* ipiv, int32_t* s_pv, int32_t* s_ok, int32_t* s_juc, int32_t& s_ju,
    int32_t& s_info) {
  double a[NS][kPanel];
#pragma unroll
  for (int k = 0; k < NS; ++k)
#pragma unroll
    for (int c = 0; c < kPanel; ++c) {
      const int32_t r = lane + 64 * k;
      a[k][c] = r < prows ? s_pan[c * prmax + r] : 0.0;
    }
  // drop thresholds of the panel columns, loaded once
  double dropc[kPanel];
#pragma unroll
  for (int c = 0; c < kPanel; ++c) dropc[c] = tau * cn[j0 + c];
  int32_t ju = s_ju, info = s_info;
#pragma unroll
  for (int c = 0; c < kPanel; ++c) {
    const int32_t jj = j0 + c, km = min(KL, n - 1 - jj);
    // pivot: the first row of c .. c+km within the tie tolerance of the largest
    double best = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int32_t r = lane + 64 * k;
      if (r >= c && r <= c + km) best = fmax(best, fabs(a[k][c]));
    }
    best = wave_max_nonneg(best);
    const double thr = (1.0 - kPivotTie) * best;
    int32_t prow = c;
    bool found = false;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int32_t r = lane + 64 * k;
      const uint64_t msk = __ballot(r >= c && r <= c + km && fabs(a[k][c]) >= thr);
      if (!found && msk != 0) {
        prow = 64 * k + (int32_t)__builtin_ctzll(msk);
        found = true;
      }
    }
    const int32_t p = __builtin_amdgcn_readfirstlane(prow - c);
    const int32_t pl = (c + p) & 63, pk = (c + p) >> 6;
    // the pivot row in columns c.. (slot pk chosen uniformly, then read from
    // lane pl) and row c of column c
    double vp[kPanel];
#pragma unroll
    for (int cc = 0; cc < kPanel; ++cc) {
      if (cc < c) continue;
      double v = a[0][cc];
#pragma unroll
      for (int k = 1; k < NS; ++k)
        if (pk == k) v = a[k][cc];
      vp[cc] = readlane_d(v, pl);
    }
    double piv = vp[c];
    const double top = readlane_d(a[0][c], c);
    // no nonzero candidate: the compensated pivot tau ||A(:, j)|| of the
    // incomplete factorisation (zero, so reported, for the exact LU)
    if (piv == 0.0) piv = dropc[c];
    const bool ok = piv != 0.0;
    ju = max(ju, min(jj + KU + p, n - 1));
    if (lane == 0) {
      s_pv[c] = p;
      s_ok[c] = ok;
      s_juc[c] = ju;
      ipiv[jj] = jj + p;
    }
    if (!ok) {
      if (info == 0) info = jj + 1;
      continue;
    }
    // the interchange of rows c and c + p in the later columns; row c becomes
    // U (dropped below the threshold)
    double u[kPanel];
#pragma unroll
    for (int cc = c + 1; cc < kPanel; ++cc) {
      const double rc = readlane_d(a[0][cc], c);
      u[cc] = vp[cc];
      if (j0 + cc <= ju && fabs(vp[cc]) < dropc[cc]) u[cc] = 0.0;
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (k == pk && lane == pl) a[k][cc] = rc;
      if (lane == c) a[0][cc] = u[cc];
    }
    // multipliers of column c from its values before the interchange
    const double rinv = 1.0 / piv, drop_l = dropc[c];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int32_t r = lane + 64 * k;
      if (r > c && r <= c + km) {
        const double v = (r == c + p) ? top : a[k][c];
        a[k][c] = fabs(v) < drop_l ? 0.0 : v * rinv;
      }
    }
    if (lane == c) a[0][c] = piv;
    // rank-1 update of the later panel columns
#pragma unroll
    for (int cc = c + 1; cc < kPanel; ++cc) {
      if (j0 + cc > ju) continue;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int32_t r = lane + 64 * k;
        if (r > c && r <= c + km) a[k][cc] -= a[k][c] * u[cc];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k)
#pragma unroll
    for (int c = 0; c < kPanel; ++c) {
      const int32_t r = lane + 64 * k;
      if (r < prows) s_pan[c * prmax + r] = a[k][c];
    }
  // the later steps' interchanges in the multiplier columns (same wave: the
  // stores above are seen by these reads in program order)
  if (lane < kPanel) {
    double* pc = s_pan + lane * prmax;
    for (int32_t c2 = lane + 1; c2 < kPanel; ++c2) {
      const int32_t p2 = s_ok[c2] ? s_pv[c2] : 0;
      if (p2 != 0) {
        const double x = pc[c2];
        pc[c2] = pc[c2 + p2];
        pc[c2 + p2] = x;
      }
    }
  }
  if (lane == 0) {
    s_ju = ju;
    s_info = info;
  }
}

// Rank-kPanel update of rows j0+kPanel .. rmax of the trailing columns tcol
// in [t_lo, t_hi) (tcol counts from column j0+kPanel): lane l keeps the
// multipliers of rows rc0 + l + 64k (k < 3) in registers, wave w of W takes
// columns t_lo + w, t_lo + w + W, ... four at a time; U12 of a column is a
// broadcast LDS read (its skipped steps hold zero).  Rows past nrows and
// columns past t_hi read the last valid row or column instead (every load is
// unconditional) and store nothing.  With s_dst the results go to the panel
// buffer s_dst (column tcol, panel row = row - (j0 + kPanel)) instead of the
// band.
__device__ __attribute__((always_inline)) inline void lu_rank_update(
    double* ab, int32_t ldab, int32_t KV, const double* s_pan, const double* s_u12, int32_t prmax, int32_t ntmax,
    int32_t j0, int32_t nrows, int32_t t_lo, int32_t t_hi, int w, int W, int lane, double* s_dst) {
  if (nrows <= 0 || t_lo >= t_hi) return;
  const int32_t c0 = j0 + kPanel;  // first trailing column (and first row below the panel)
  for (int32_t rc0 = 0; rc0 < nrows; rc0 += 3 * 64) {
    double L[3][kPanel];
    int32_t ro[3];
    bool rv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int32_t r = rc0 + lane + 64 * k;
      rv[k] = r < nrows;
      ro[k] = min(r, nrows - 1);
#pragma unroll
      for (int c = 0; c < kPanel; ++c) L[k][c] = s_pan[c * prmax + kPanel + ro[k]];
    }
    for (int32_t t0 = t_lo + w; t0 < t_hi; t0 += 4 * W) {
      double a[4][3];
      int32_t tc[4];
#pragma unroll
      for (int bq = 0; bq < 4; ++bq) {
        tc[bq] = min(t0 + bq * W, t_hi - 1);
        // entry (c0 + ro, c0 + tc) of the band
        const double* col = ab + (int64_t)(c0 + tc[bq]) * ldab + KV - tc[bq];
#pragma unroll
        for (int k = 0; k < 3; ++k) a[bq][k] = col[ro[k]];
      }
#pragma unroll
      for (int bq = 0; bq < 4; ++bq) {
        const bool cv = t0 + bq * W < t_hi;
        double u[kPanel];
#pragma unroll
        for (int c = 0; c < kPanel; ++c) u[c] = s_u12[c * ntmax + tc[bq]];
        double* col = ab + (int64_t)(c0 + tc[bq]) * ldab + KV - tc[bq];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          double x = a[bq][k];
#pragma unroll
          for (int c = 0; c < kPanel; ++c) x -= L[k][c] * u[c];
          if (cv && rv[k]) {
            if (s_dst) s_dst[tc[bq] * prmax + ro[k]] = x;
            else col[ro[k]] = x;
          }
        }
      }
    }
  }
}

// Lookahead: panel k+1 is factored by wave 0 while the other waves apply
// panel k's rank-kPanel update to the columns after panel k+1 and store
// panel k-1.  Per panel k:
//   (1) all threads: interchanges and unit lower solve of every trailing
//       column (U12 of the panel);
//   (2) all waves: the rank-kPanel update of the next panel's columns,
//       written to its LDS buffer, and its other entries from memory;
//   (3) wave 0 factors panel k+1; waves 1.. update the remaining columns and
//       return panel k-1 to memory with its multipliers in band order.
// Three panel buffers rotate (panel k+1 factored, k applied, k-1 stored).
// A panel's columns stay in LDS from the update that forms them until they
// are stored, and no other step reads them from memory in between.  Every
// entry receives the same operations in the same order as without
// lookahead, so pivots and factors are unchanged bit for bit.
template <int NS>
__global__ void __launch_bounds__(kLuThreads)
k_band_lu_blocked(double* __restrict__ ab_all, int32_t* __restrict__ ipiv_all, const SubInfo* __restrict__ subs,
                  int32_t* __restrict__ info, const double* __restrict__ colnorm_all, double tau, int32_t prmax,
                  int32_t ntmax, const int32_t* __restrict__ sub_list) {
  extern __shared__ double s_dyn[];
  // panel buffer b: column c at s_dyn + (b * kPanel + c) * prmax; U12 row c
  // at s_u12 + c * ntmax
  double* const s_u12 = s_dyn + 3 * kPanel * prmax;
  __shared__ int32_t s_pv[3][kPanel], s_juc[3][kPanel], s_ok[3][kPanel];
  __shared__ int32_t s_ju, s_info;
  const int sub = sub_list ? sub_list[blockIdx.x] : (int)blockIdx.x;
  const SubInfo q = subs[sub];
  const int32_t n = q.npad, ldab = q.ldab, KL = q.kl, KU = q.ku, KV = KL + KU;
  double* ab = ab_all + q.band_off;
  int32_t* ipiv = ipiv_all + q.vec_off;
  const double* cn = colnorm_all + q.vec_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = (int)(blockDim.x >> 6);
  if (n == 0) return;  // an empty interior (info stays 0)
  // entry (r, c) of the block lives at ab[c * ldab + KV + r - c] for -KV <= r - c <= KL
  auto at = [&](int32_t r, int32_t c) -> double& { return ab[(int64_t)c * ldab + KV + r - c]; };
  auto pan = [&](int b) { return s_dyn + b * kPanel * prmax; };
  // entries (c, rr) of panel j0 from memory, except those with c < c_upd and
  // rr < r_upd (written by the update), by threads t0, t0 + nth, ...
  auto load_panel = [&](int b, int32_t j0, int32_t c_upd, int32_t r_upd, int t0, int nth) {
    const int32_t prows = min(KL + kPanel, n - j0);
    double* P = pan(b);
    for (int32_t e = t0; e < kPanel * prows; e += nth) {
      const int32_t c = e / prows, rr = e % prows, d = rr - c;
      if (c < c_upd && rr < r_upd) continue;
      P[c * prmax + rr] = (d <= KL && d >= -KV) ? at(j0 + rr, j0 + c) : 0.0;
    }
  };
  // panel j0 (buffer b) to memory, its multipliers in band storage order: the
  // panel's later interchanges undone, each entry's row traced through them
  // (the undo swaps, for c2 from the last column down to c + 1, rows c2 and
  // c2 + p_c2 of column c), by threads t0, t0 + nth, ...
  auto store_panel = [&](int b, int32_t j0, int t0, int nth) {
    const int32_t prows = min(KL + kPanel, n - j0);
    const double* P = pan(b);
    for (int32_t e = t0; e < kPanel * prows; e += nth) {
      const int32_t c = e / prows, rr = e % prows;
      int32_t pos = rr;
      for (int32_t c2 = kPanel - 1; c2 > c; --c2) {
        const int32_t p2 = s_ok[b][c2] ? s_pv[b][c2] : 0;
        if (p2 == 0) continue;
        if (pos == c2) pos = c2 + p2;
        else if (pos == c2 + p2) pos = c2;
      }
      const int32_t d = pos - c;
      if (d <= KL && d >= -KV) at(j0 + pos, j0 + c) = P[c * prmax + rr];
    }
  };
  if (tid == 0) {
    s_ju = 0;
    s_info = 0;
  }
  // panel 0
  load_panel(0, 0, 0, 0, tid, blockDim.x);
  __syncthreads();
  if (wave == 0)
    panel_regs<NS>(pan(0), prmax, min(KL + kPanel, n), 0, n, KL, KU, lane, tau, cn, ipiv, s_pv[0], s_ok[0], s_juc[0],
                   s_ju, s_info);
  __syncthreads();
  for (int32_t k = 0;; ++k) {
    const int b = k % 3, bn = (k + 1) % 3, bp = (k + 2) % 3;  // panels k, k+1, k-1
    const int32_t j0 = k * kPanel;  // < n: n is a multiple of kPanel
    constexpr int32_t nb = kPanel;
    const int32_t ju = s_ju, nt = ju - (j0 + nb) + 1;
    const double* P = pan(b);
    double* U = s_u12;
    // ---- (1) trailing columns j0+nb .. ju: interchanges, then the panel rows
    // (unit lower triangular solve), in registers, one column per thread
    for (int32_t tcol = tid; tcol < nt; tcol += blockDim.x) {
      const int32_t jc = j0 + nb + tcol;
      const double drop_u = tau * cn[jc];
      double v[kPanel];
#pragma unroll
      for (int c = 0; c < kPanel; ++c) v[c] = jc <= s_juc[b][c] ? at(j0 + c, jc) : 0.0;
#pragma unroll
      for (int c = 0; c < kPanel; ++c) {
        if (!s_ok[b][c] || jc > s_juc[b][c]) continue;
        const int32_t p = s_pv[b][c];
        if (p == 0) continue;
        if (c + p < nb) {
          // both rows inside the panel
#pragma unroll
          for (int c2 = 0; c2 < kPanel; ++c2)
            if (c2 == c + p) {
              const double x = v[c2];
              v[c2] = v[c];
              v[c] = x;
            }
        } else {
          double& g = at(j0 + c + p, jc);
          const double x = g;
          g = v[c];
          v[c] = x;
        }
      }
#pragma unroll
      for (int c = 0; c < kPanel; ++c) {
        double u = 0.0;
        if (s_ok[b][c] && jc <= s_juc[b][c]) {
          u = v[c];
          if (fabs(u) < drop_u) u = 0.0;
          v[c] = u;
#pragma unroll
          for (int i = 1; i < kPanel; ++i)
            if (c + i < kPanel) v[c + i] -= P[c * prmax + c + i] * u;
        }
        U[c * ntmax + tcol] = u;
      }
#pragma unroll
      for (int c = 0; c < kPanel; ++c)
        if (jc <= s_juc[b][c]) at(j0 + c, jc) = v[c];
    }
    __syncthreads();
    const int32_t rmax = min(j0 + nb - 1 + KL, n - 1), nrows = rmax - (j0 + nb) + 1;
    const int32_t jn = j0 + nb;
    const bool next = jn < n;
    const int32_t nlook = next ? min(kPanel, max(nt, 0)) : 0;
    // ---- (2) the next panel into its buffer: the update of its first nlook
    // columns (rows below this panel), everything else from memory
    if (next) {
      lu_rank_update(ab, ldab, KV, P, U, prmax, ntmax, j0, nrows, 0, nlook, wave, nwaves, lane, pan(bn));
      load_panel(bn, jn, nlook, max(nrows, 0), tid, blockDim.x);
      __syncthreads();
    }
    // ---- (3) wave 0: factor the next panel; the other waves: the rest of
    // this panel's update, then the previous panel to memory
    if (wave == 0) {
      if (next)
        panel_regs<NS>(pan(bn), prmax, min(KL + kPanel, n - jn), jn, n, KL, KU, lane, tau, cn, ipiv, s_pv[bn],
                       s_ok[bn], s_juc[bn], s_ju, s_info);
    } else {
      lu_rank_update(ab, ldab, KV, P, U, prmax, ntmax, j0, nrows, nlook, max(nt, 0), wave - 1, nwaves - 1, lane,
                     nullptr);
      if (k > 0) store_panel(bp, j0 - kPanel, tid - 64, (int)blockDim.x - 64);
    }
    __syncthreads();
    if (!next) {
      // the last panel
      store_panel(b, j0, tid, blockDim.x);
      break;
    }
  }
  if (tid == 0) info[sub] = s_info;
}

// Column 2-norms of every padded interior block before elimination: column
// c holds its original entries in band rows KL .. ldab-1.
__global__ void k_band_colnorm(const double* __restrict__ ab_all, const SubInfo* __restrict__ subs,
                               double* __restrict__ colnorm_all) {
  const SubInfo q = subs[blockIdx.y];
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= q.npad) return;
  const double* col = ab_all + q.band_off + (int64_t)c * q.ldab;
  double acc = 0.0;
  for (int32_t r = q.kl; r < q.ldab; ++r) acc += col[r] * col[r];
  colnorm_all[q.vec_off + c] = sqrt(acc);
}

// Stored entries of the factors of every block (multipliers below the unit
// diagonal and U, real rows and columns only): counts[sub] += the count of
// this workgroup's kNnzCols columns (grid: column chunks x subdomains;
// counts zeroed first; integer sums, so the order does not matter).
constexpr int kNnzCols = 64;
__global__ void __launch_bounds__(256)
k_band_nnz(const double* __restrict__ ab_all, const SubInfo* __restrict__ subs, unsigned long long* __restrict__ counts) {
  const SubInfo q = subs[blockIdx.y];
  const int32_t n = q.n, ldab = q.ldab, KV = q.kl + q.ku;
  const int32_t c0 = blockIdx.x * kNnzCols, c1 = min(n, c0 + kNnzCols);
  if (c0 >= c1) return;
  const double* ab = ab_all + q.band_off + (int64_t)c0 * ldab;
  unsigned long long cnt = 0;
  for (int32_t t = threadIdx.x; t < (c1 - c0) * ldab; t += blockDim.x) {
    const int32_t c = c0 + t / ldab, r = t % ldab;
    const int32_t row = c + r - KV;  // U rows r <= KV, multiplier rows r > KV
    if (row >= 0 && row < n && (r <= KV || row <= c + q.kl) && ab[t] != 0.0) ++cnt;
  }
  __shared__ unsigned long long s_cnt[256 / 64];
  for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
  if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long v = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += s_cnt[w];
    atomicAdd(counts + blockIdx.y, v);
  }
}

// max |x_t| over n contiguous doubles, in every thread of the block (ends
// with a barrier)
__device__ inline double block_absmax(const double* x, int64_t n, double* s_wmax) {
  double m = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) m = fmax(m, fabs(x[t]));
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) s_wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, s_wmax[w]);
  __syncthreads();
  return r;
}

template <class T>
__device__ inline T to_store(double v) { return (T)v; }
template <>
__device__ inline __half to_store<__half>(double v) { return __float2half((float)v); }

// ---------------------------------------------------------------------------
// Lower sweep blocks.  For block b of subdomain sub (columns c0 = b*nbL ..
// c0+nbL-1) the row operations of the band LU touch only the window rows
// c0 .. c0+nbL+KL-1.  Their product is L~^{-1} P with P the window
// permutation and L~ = [L11 0; L21 I] the multipliers after the later swaps
// of the block, so that for the permuted window v = P w
//     x_b = inv(L11) v_top,   carry = v_bot - (L21 inv(L11)) v_top.
// Stored per block: the gather indices of P (W = nbL+KL) and one column-major
// W x nbL matrix [inv(L11); L21 inv(L11)], applied to v_top as one GEMV.
// Two launches.  k_convert_lower_prep (one workgroup per block): the
// multipliers with the block's later swaps applied, each band entry's row
// traced through those swaps (a permutation of its column, so the entries
// land where the swaps in order put them), and the window indices permuted
// in LDS.  k_convert_lower_slab (grid: slabs x blocks): columns c0 ..
// c0+sw-1 of inv(L11) in LDS by forward elimination of the unit lower L11
// (column c receives the steps i >= c only: rows r > i lose Lw(r, i) X(i, c),
// Lw's column i read into LDS one step ahead), then the rows below as dot
// products of Lw's rows with the slab's columns over k = c .. nbL-1 in
// increasing k.  Every element's operations and their order depend only on
// the block, not on the slab split, so any slab width gives the same result
// bit for bit.
__global__ void __launch_bounds__(kSetupThreads)
k_convert_lower_prep(const double* __restrict__ ab_all, const int32_t* __restrict__ ipiv_all,
                     const SubInfo* __restrict__ subs, const LBlk* __restrict__ lb, double* __restrict__ work_all,
                     int32_t* __restrict__ lperm_all, const int32_t* __restrict__ blk_list) {
  extern __shared__ int32_t s_i[];  // piv[nbL], idx[W]
  const LBlk B = lb[blk_list ? blk_list[blockIdx.x] : blockIdx.x];
  const SubInfo q = subs[B.sub];
  const int32_t nbL = q.nbl, KL = q.kl, ldab = q.ldab, KV = q.kl + q.ku;
  const int32_t c0 = B.idx * nbL, W = nbL + KL;
  const double* ab = ab_all + q.band_off;
  const int32_t* ipiv = ipiv_all + q.vec_off;
  double* Lw = work_all + B.woff;
  int32_t* piv = s_i;
  int32_t* idx = s_i + nbL;
  const int tid = threadIdx.x;
  for (int32_t s = tid; s < nbL; s += blockDim.x) piv[s] = ipiv[c0 + s] - c0;
  for (int64_t t = tid; t < (int64_t)W * nbL; t += blockDim.x) Lw[t] = 0.0;
  __syncthreads();
  if (tid == 0) {
    for (int32_t r = 0; r < W; ++r) idx[r] = r;
    for (int32_t s = 0; s < nbL; ++s) {
      const int32_t p = piv[s], a = idx[s];
      idx[s] = idx[p];
      idx[p] = a;
    }
  }
  // band entries (c + i, c), 1 <= i <= KL, to their rows after the swaps
  // s = c+1 .. nbL-1
  for (int64_t t = tid; t < (int64_t)KL * nbL; t += blockDim.x) {
    const int32_t c = (int32_t)(t / KL), i = 1 + (int32_t)(t % KL);
    int32_t pos = c + i;
    for (int32_t s = c + 1; s < nbL; ++s) {
      const int32_t p = piv[s];
      if (p == s) continue;
      if (pos == s) pos = p;
      else if (pos == p) pos = s;
    }
    Lw[(int64_t)c * W + pos] = ab[(int64_t)(c0 + c) * ldab + KV + i];
  }
  __syncthreads();
  int32_t* op = lperm_all + B.poff;
  for (int32_t r = tid; r < W; r += blockDim.x) op[r] = idx[r];
}

constexpr int kLSlabThreads = 256;
template <class T>
__global__ void __launch_bounds__(kLSlabThreads)
k_convert_lower_slab(const SubInfo* __restrict__ subs, const LBlk* __restrict__ lb, const double* __restrict__ work_all,
                     int32_t slab, T* __restrict__ lmat_all, int32_t* __restrict__ info,
                     const int32_t* __restrict__ blk_list) {
  extern __shared__ double s_x[];
  const LBlk B = lb[blk_list ? blk_list[blockIdx.y] : blockIdx.y];
  const SubInfo q = subs[B.sub];
  const int32_t nbL = q.nbl, KL = q.kl, W = nbL + KL;
  const int32_t a0 = blockIdx.x * slab;
  if (a0 >= nbL) return;
  const int32_t sw = min(slab, nbL - a0), ldx = nbL + 1;
  const double* Lw = work_all + B.woff;  // W x nbL, column-major
  double* X = s_x;                        // slab column cc at X + cc * ldx (rows 0 .. nbL-1)
  double* lcol = s_x + (int64_t)slab * ldx;  // two buffers of nbL: Lw(0 .. nbL-1, i)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = kLSlabThreads / 64;
  for (int32_t e = tid; e < sw * nbL; e += kLSlabThreads) {
    const int32_t cc = e / nbL, r = e % nbL;
    X[cc * ldx + r] = r == a0 + cc ? 1.0 : 0.0;
  }
  auto put = [&](int32_t i) {
    if (i > nbL - 2) return;
    double* buf = lcol + (i & 1) * nbL;
    for (int32_t r = tid; r < nbL; r += kLSlabThreads) buf[r] = r > i ? Lw[(int64_t)i * W + r] : 0.0;
  };
  put(a0);
  __syncthreads();
  // forward elimination: rows r > i of the slab columns c <= i
  for (int32_t i = a0; i < nbL - 1; ++i) {
    const double* lc = lcol + (i & 1) * nbL;
    for (int32_t r = i + 1 + lane; r < nbL; r += 64) {
      const double l = lc[r];
      for (int32_t cc = wave; cc < sw; cc += nw)
        if (a0 + cc <= i) X[cc * ldx + r] -= l * X[cc * ldx + i];
    }
    put(i + 1);
    __syncthreads();
  }
  // rows below: sum over k = c .. nbL-1 of Lw(r, k) X(k, c), in increasing k
  T* lm = lmat_all + B.moff;
  bool bad = false;
  constexpr int kCols = 8;  // slab columns per wave at a time
  for (int32_t cb = wave * kCols; cb < sw; cb += nw * kCols) {
    for (int32_t rb = nbL; rb < W; rb += 64) {
      const int32_t r = rb + lane;
      const int32_t rr = min(r, W - 1);
      double acc[kCols];
#pragma unroll
      for (int j = 0; j < kCols; ++j) acc[j] = 0.0;
      for (int32_t k = a0 + cb; k < nbL; ++k) {
        const double l = Lw[(int64_t)k * W + rr];
#pragma unroll
        for (int j = 0; j < kCols; ++j)
          if (cb + j < sw && a0 + cb + j <= k) acc[j] += l * X[(cb + j) * ldx + k];
      }
      if (r < W)
#pragma unroll
        for (int j = 0; j < kCols; ++j)
          if (cb + j < sw) {
            const T st = to_store<T>(acc[j]);
            if (!isfinite((double)st)) bad = true;
            lm[(int64_t)(a0 + cb + j) * W + r] = st;
          }
    }
  }
  for (int32_t e = tid; e < sw * nbL; e += kLSlabThreads) {
    const int32_t cc = e / nbL, r = e % nbL;
    const T st = to_store<T>(X[cc * ldx + r]);
    if (!isfinite((double)st)) bad = true;
    lm[(int64_t)(a0 + cc) * W + r] = st;
  }
  if (bad) atomicMax(info, 2);
}

// ---------------------------------------------------------------------------
// Upper sweep blocks (rows r0 = b*nbU .. r0+nbU-1, nbU >= KL+KU so that U is
// block bidiagonal): inv(U_bb) (column-major) and U_{b,b+1} (column-major).
// ---------------------------------------------------------------------------
// inv(U_bb) by back substitution on all columns at once: steps i = nbU-1 ..
// 0 scale row i by 1 / U(i, i) and take U(r, i) X(i, :) from the rows r < i
// (a zero U(r, i) skipped).  By slabs of columns (grid: slabs x blocks), the
// slab in LDS: column c receives steps i <= c only, and step i touches rows
// i - KV .. i - 1 (U is banded), so a slab of columns c0 .. c0+sw-1 runs
// steps c0+sw-1 .. 0 on its own.  U's column i is read into LDS one step
// ahead.  Wave w takes columns w, w + 4, ... of the slab, lane l rows l,
// l + 64, ... of a step; every element's operations and their order depend
// only on the block, so any slab width gives the same result bit for bit.
constexpr int kUSlabThreads = 256;
constexpr int kUFetch = 5;  // entries of U's column per thread: KV + 1 <= 5 * 256
template <class T>
__global__ void __launch_bounds__(kUSlabThreads)
k_convert_upper_slab(const double* __restrict__ ab_all, const SubInfo* __restrict__ subs,
                     const UBlk* __restrict__ ub, int32_t slab, int32_t kv_max, T* __restrict__ uinv_all,
                     T* __restrict__ u12_all, int32_t* __restrict__ info, const int32_t* __restrict__ blk_list) {
  extern __shared__ double s_x[];
  const UBlk B = ub[blk_list ? blk_list[blockIdx.y] : blockIdx.y];
  const SubInfo q = subs[B.sub];
  const int32_t nbU = q.nbu, ldab = q.ldab, n = q.npad, KV = q.kl + q.ku;
  const int32_t c0 = blockIdx.x * slab;
  if (c0 >= nbU) return;
  const int32_t sw = min(slab, nbU - c0), ldx = nbU + 1;
  const int32_t r0 = B.idx * nbU;
  const double* ab = ab_all + q.band_off;
  double* X = s_x;                                  // column cc of the slab at X + cc * ldx
  double* ucol = s_x + (int64_t)slab * ldx;         // two buffers of kv_max + 1: U(i - KV .. i, i)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = kUSlabThreads / 64;
  auto U = [&](int32_t r, int32_t c) -> double {  // subdomain-local (r, c)
    const int32_t d = c - r;
    return (d >= 0 && d <= KV && c < n) ? ab[(int64_t)c * ldab + KV + r - c] : 0.0;
  };
  // buffer entry j of step i holds U(i - KV + j, i), j = 0 .. KV (the last
  // is the diagonal)
  auto fetch = [&](int32_t i, double (&v)[kUFetch]) {
#pragma unroll
    for (int t = 0; t < kUFetch; ++t) {
      const int32_t j = tid + t * kUSlabThreads, r = i - KV + j;
      v[t] = (i >= 0 && j <= KV && r >= 0) ? U(r0 + r, r0 + i) : 0.0;
    }
  };
  auto put = [&](int32_t i, const double (&v)[kUFetch]) {
    double* buf = ucol + (i & 1) * (kv_max + 1);
#pragma unroll
    for (int t = 0; t < kUFetch; ++t) {
      const int32_t j = tid + t * kUSlabThreads;
      if (j <= KV) buf[j] = v[t];
    }
  };
  for (int32_t e = tid; e < sw * nbU; e += kUSlabThreads) {
    const int32_t cc = e / nbU, r = e % nbU;
    X[cc * ldx + r] = r == c0 + cc ? 1.0 : 0.0;
  }
  const int32_t itop = c0 + sw - 1;
  {
    double v[kUFetch];
    fetch(itop, v);
    put(itop, v);
  }
  __syncthreads();
  for (int32_t i = itop; i >= 0; --i) {
    const double* uc = ucol + (i & 1) * (kv_max + 1);  // uc[KV + r - i] = U(r, i)
    double v[kUFetch];
    fetch(i - 1, v);  // the next step's column, in flight during this one
    const double d = uc[KV];
    if (d == 0.0) {
      if (tid == 0) atomicMax(info, 1);
      return;
    }
    const double dinv = 1.0 / d;
    if (tid < sw && c0 + tid >= i) X[tid * ldx + i] *= dinv;
    __syncthreads();
    const int32_t rlo = max(0, i - KV);
    for (int32_t rb = rlo; rb < i; rb += 64) {
      const int32_t r = rb + lane;
      const double u = r < i ? uc[KV + r - i] : 0.0;
      if (u != 0.0)
        for (int32_t cc = wave; cc < sw; cc += nw)
          if (c0 + cc >= i) X[cc * ldx + r] -= u * X[cc * ldx + i];
    }
    if (i > 0) put(i - 1, v);
    __syncthreads();
  }
  T* ui = uinv_all + B.off;
  T* u12 = u12_all + B.off;
  bool bad = false;
  for (int32_t e = tid; e < sw * nbU; e += kUSlabThreads) {
    const int32_t cc = e / nbU, r = e % nbU, c = c0 + cc;
    const int64_t t = (int64_t)c * nbU + r;
    const T a = to_store<T>(X[cc * ldx + r]), b = to_store<T>(U(r0 + r, r0 + nbU + c));
    if (!isfinite((double)a) || !isfinite((double)b)) bad = true;
    ui[t] = a;
    u12[t] = b;
  }
  if (bad) atomicMax(info, 2);
}

// ---------------------------------------------------------------------------
// Mini Schur complements, one workgroup per aggregate.
//   G (s x s), D (d x d), E (d x s), F (s x d), all row-major FP64.
// Gaussian elimination with partial pivoting of [D | E] turns E into
// L^{-1} P E; back substitution with U gives X = D^{-1} E; then
// G <- G - F X on MFMA (v_mfma_f64_16x16x4f64).
// rowsum != 0 (the rowsum variant of section 3.1): E is first collapsed to
// its row sums e = E 1 (kept in E's column 0), the elimination carries that
// one column, and the correction c = F D^{-1} e is subtracted from G's
// diagonal, so each row of S_i keeps the row sum of the full mini Schur
// complement.
// ---------------------------------------------------------------------------
typedef double double4_t __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kSetupThreads)
k_schur_blocks(const int32_t* __restrict__ agg_s, const int32_t* __restrict__ agg_d,
               const int64_t* __restrict__ g_off, const int64_t* __restrict__ dd_off,
               const int64_t* __restrict__ de_off, const int64_t* __restrict__ df_off, double* __restrict__ Gall,
               double* __restrict__ Dall, double* __restrict__ Eall, double* __restrict__ Fall,
               int32_t* __restrict__ info, int rowsum) {
  const int i = blockIdx.x;
  const int32_t s = agg_s[i], d = agg_d[i];
  if (d == 0) return;
  double* G = Gall + g_off[i];
  double* D = Dall + dd_off[i];
  double* E = Eall + de_off[i];
  double* F = Fall + df_off[i];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t se = rowsum ? 1 : s;  // right-hand sides carried through the elimination
  const int32_t w = d + se;           // augmented row length
  if (rowsum) {
    // one thread per row: its sum in column order, stored over column 0
    for (int32_t r = tid; r < d; r += blockDim.x) {
      double a = 0.0;
      for (int32_t q = 0; q < s; ++q) a += E[(int64_t)r * s + q];
      E[(int64_t)r * s] = a;
    }
    __syncthreads();
  }
  auto A = [&](int32_t r, int32_t c) -> double& { return c < d ? D[(int64_t)r * d + c] : E[(int64_t)r * s + (c - d)]; };
  __shared__ int32_t s_p;
  __shared__ double s_piv;
  __shared__ int s_bad;
  __shared__ double s_wmax[kSetupThreads / 64];
  if (tid == 0) s_bad = 0;
  // a pivot at or below 1e-13 max|D_r| marks the block singular
  const double tiny = 1e-13 * block_absmax(D, (int64_t)d * d, s_wmax);
  for (int32_t c = 0; c < d; ++c) {
    if (wave == 0) {
      double best = -1.0;
      int32_t bi = c;
      for (int32_t r = c + lane; r < d; r += 64) {
        double a = fabs(A(r, c));
        if (a > best) {
          best = a;
          bi = r;
        }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        double ob = __shfl_xor(best, off);
        int32_t oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) {
        s_p = bi;
        s_piv = A(bi, c);
        if (fabs(s_piv) <= tiny) s_bad = 1;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const int32_t p = s_p;
    if (p != c)
      for (int32_t q = c + tid; q < w; q += blockDim.x) {
        double a = A(c, q);
        A(c, q) = A(p, q);
        A(p, q) = a;
      }
    __syncthreads();
    const double rinv = 1.0 / s_piv;
    const int32_t rows = d - 1 - c, cols = w - c - 1;
    for (int64_t t = tid; t < (int64_t)rows * cols; t += blockDim.x) {
      int32_t r = c + 1 + (int32_t)(t / cols), q = c + 1 + (int32_t)(t % cols);
      double l = A(r, c) * rinv;
      A(r, q) -= l * A(c, q);
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) atomicMax(info, 1);
    return;
  }
  // back substitution: E <- U^{-1} E (rows from the bottom)
  for (int32_t r = d - 1; r >= 0; --r) {
    const double dinv = 1.0 / A(r, r);
    for (int32_t q = tid; q < se; q += blockDim.x) E[(int64_t)r * s + q] *= dinv;
    __syncthreads();
    for (int64_t t = tid; t < (int64_t)r * se; t += blockDim.x) {
      int32_t rr = (int32_t)(t / se), q = (int32_t)(t % se);
      E[(int64_t)rr * s + q] -= D[(int64_t)rr * d + r] * E[(int64_t)r * s + q];
    }
    __syncthreads();
  }
  if (rowsum) {
    // G(r, r) <- G(r, r) - sum_k F(r, k) x(k), x = D^{-1} e in E's column 0
    for (int32_t r = tid; r < s; r += blockDim.x) {
      double a = 0.0;
      for (int32_t k = 0; k < d; ++k) a += F[(int64_t)r * d + k] * E[(int64_t)k * s];
      G[(int64_t)r * s + r] -= a;
    }
    return;
  }
  // G <- G - F X with 16x16 output tiles, k in steps of 4 (FP64 MFMA).
  // Lane layout of v_mfma_f64_16x16x4f64 (checked on gfx950): A operand lane
  // l holds A(l%16, l/16), B operand lane l holds B(l/16, l%16), result
  // register v of lane l holds C(4*v + l/16, l%16).
  const int32_t tiles = ((s + 15) / 16);
  for (int32_t tile = wave; tile < tiles * tiles; tile += blockDim.x / 64) {
    const int32_t ti = tile / tiles, tj = tile % tiles;
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    const int32_t ar = ti * 16 + (lane & 15), bc = tj * 16 + (lane & 15), kk = lane >> 4;
    for (int32_t k0 = 0; k0 < d; k0 += 4) {
      int32_t k = k0 + kk;
      double a = (ar < s && k < d) ? F[(int64_t)ar * d + k] : 0.0;
      double b = (k < d && bc < s) ? E[(int64_t)k * s + bc] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    for (int v = 0; v < 4; ++v) {
      int32_t r = ti * 16 + 4 * v + (lane >> 4), c = tj * 16 + (lane & 15);
      if (r < s && c < s) G[(int64_t)r * s + c] -= acc[v];
    }
  }
}

// ---------------------------------------------------------------------------
// S_i^{-1} by Gauss-Jordan with partial pivoting on [S | I], stored
// column-major in the requested precision (FP16 with one scale per block).
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(kSetupThreads)
k_invert_dense(const int32_t* __restrict__ agg_s, const int64_t* __restrict__ g_off, const double* __restrict__ Sall,
               double* __restrict__ work_all, int32_t* __restrict__ info, const int64_t* __restrict__ sinv_off,
               T* __restrict__ sinv_all, float* __restrict__ scale_all, int prec) {
  const int i = blockIdx.x;
  const int32_t s = agg_s[i];
  const double* S = Sall + g_off[i];
  double* A = work_all + 2 * g_off[i];  // s x 2s row-major
  const int32_t w = 2 * s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int64_t t = tid; t < (int64_t)s * w; t += blockDim.x) {
    int32_t r = (int32_t)(t / w), c = (int32_t)(t % w);
    A[t] = c < s ? S[(int64_t)r * s + c] : (c - s == r ? 1.0 : 0.0);
  }
  __shared__ int32_t s_p;
  __shared__ double s_piv;
  __shared__ int s_bad;
  __shared__ double s_red[16];
  __shared__ double s_wmax[kSetupThreads / 64];
  if (tid == 0) s_bad = 0;
  // a pivot at or below 1e-13 max|S_i| marks the block singular
  const double tiny = 1e-13 * block_absmax(S, (int64_t)s * s, s_wmax);
  for (int32_t c = 0; c < s; ++c) {
    if (wave == 0) {
      double best = -1.0;
      int32_t bi = c;
      for (int32_t r = c + lane; r < s; r += 64) {
        double a = fabs(A[(int64_t)r * w + c]);
        if (a > best) {
          best = a;
          bi = r;
        }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        double ob = __shfl_xor(best, off);
        int32_t oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) {
        s_p = bi;
        s_piv = A[(int64_t)bi * w + c];
        if (fabs(s_piv) <= tiny) s_bad = 1;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const int32_t p = s_p;
    if (p != c)
      for (int32_t q = tid; q < w; q += blockDim.x) {
        double a = A[(int64_t)c * w + q];
        A[(int64_t)c * w + q] = A[(int64_t)p * w + q];
        A[(int64_t)p * w + q] = a;
      }
    __syncthreads();
    const double rinv = 1.0 / s_piv;
    for (int32_t q = tid; q < w; q += blockDim.x) A[(int64_t)c * w + q] *= rinv;
    __syncthreads();
    for (int64_t t = tid; t < (int64_t)s * w; t += blockDim.x) {
      int32_t r = (int32_t)(t / w), q = (int32_t)(t % w);
      if (r == c || q == c) continue;
      A[(int64_t)r * w + q] -= A[(int64_t)r * w + c] * A[(int64_t)c * w + q];
    }
    __syncthreads();
    for (int32_t r = tid; r < s; r += blockDim.x)
      if (r != c) A[(int64_t)r * w + c] = 0.0;
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) atomicMax(info, 1);
    return;
  }
  float scl = 1.0f;
  if (prec == P16S) {
    double mx = 0.0;
    for (int64_t t = tid; t < (int64_t)s * s; t += blockDim.x) {
      int32_t r = (int32_t)(t / s), c = (int32_t)(t % s);
      mx = fmax(mx, fabs(A[(int64_t)r * w + s + c]));
    }
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if (lane == 0) s_red[wave] = mx;
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int q = 0; q < (int)(blockDim.x / 64); ++q) m = fmax(m, s_red[q]);
      s_red[0] = m > 0.0 ? m : 1.0;
      scale_all[i] = (float)s_red[0];
    }
    __syncthreads();
    scl = (float)s_red[0];
  }
  T* out = sinv_all + sinv_off[i];
  for (int64_t t = tid; t < (int64_t)s * s; t += blockDim.x) {
    int32_t c = (int32_t)(t / s), r = (int32_t)(t % s);  // column-major output
    double v = A[(int64_t)r * w + s + c];
    if (prec == P16S) v /= (double)scl;
    out[t] = to_store<T>(v);
  }
}


// ---------------------------------------------------------------------------
// Exact block-Jacobi interface blocks: S(agg_i, agg_i) = G_ii - sum_j F(agg_i,
// int_j) A_jj^{-1} E(int_j, agg_i).  One workgroup per separator column c;
// its (subdomain, column) solves U_p = A_jj^{-1} E(int_j, c) are applied in
// ascending subdomain order (deterministic), rows of the aggregate in
// parallel.
// ---------------------------------------------------------------------------
__global__ void k_exact_schur_update(const int32_t* __restrict__ pcol_ptr, const int32_t* __restrict__ pair_sub,
                                     const int64_t* __restrict__ pair_off, const SubInfo* __restrict__ subs,
                                     const int32_t* __restrict__ agg_of, const int32_t* __restrict__ agg_off,
                                     const int64_t* __restrict__ g_off, const int32_t* __restrict__ f_rowptr,
                                     const int32_t* __restrict__ f_colidx, const double* __restrict__ f_vals,
                                     const double* __restrict__ U, double* __restrict__ S) {
  const int32_t c = blockIdx.x;
  const int32_t i = agg_of[c];
  const int32_t a0 = agg_off[i], s = agg_off[i + 1] - a0, b = c - a0;
  for (int32_t a = threadIdx.x; a < s; a += blockDim.x) {
    double acc = 0.0;
    for (int32_t p = pcol_ptr[c]; p < pcol_ptr[c + 1]; ++p) {
      const SubInfo q = subs[pair_sub[p]];
      const double* u = U + pair_off[p];
      for (int32_t e = f_rowptr[a0 + a]; e < f_rowptr[a0 + a + 1]; ++e) {
        const int32_t col = f_colidx[e] - q.int_off;
        if (col >= 0 && col < q.n) acc += f_vals[e] * u[col];
      }
    }
    S[g_off[i] + (int64_t)a * s + b] -= acc;
  }
}

// ---------------------------------------------------------------------------
// Overlapped aggregates.  The extended block S_i^e (e = s + w, row-major)
// splits into its diagonal part A_i = S_i^e[0:s, 0:s] and the lower part
// L_i = S_i^e[s:e, 0:s], which Shat holds below A_i in the first w rows of
// aggregate i+1 (column-wise assembly).
// ---------------------------------------------------------------------------
__global__ void k_overlap_split(const int32_t* __restrict__ agg_s, const int32_t* __restrict__ agg_w,
                                const int64_t* __restrict__ g_off, const int64_t* __restrict__ a_off,
                                const int64_t* __restrict__ l_off, const double* __restrict__ Se_all,
                                double* __restrict__ A_all, double* __restrict__ L_all) {
  const int i = blockIdx.x;
  const int32_t s = agg_s[i], w = agg_w[i], e = s + w;
  const double* Se = Se_all + g_off[i];
  double* A = A_all + a_off[i];
  double* L = L_all + l_off[i];
  for (int64_t t = threadIdx.x; t < (int64_t)e * s; t += blockDim.x) {
    const int32_t r = (int32_t)(t / s), c = (int32_t)(t % s);
    const double v = Se[(int64_t)r * e + c];
    if (r < s) A[(int64_t)r * s + c] = v;
    else L[(int64_t)(r - s) * s + c] = v;
  }
}

// Chain matrices of the block forward substitution over Shat:
//   x_i = A_i^{-1} t_i - M_i x_{i-1},  M_i = A_i^{-1}[:, 0:w_{i-1}] L_{i-1}
// (s_i x s_{i-1}, row-major, rows `width` long with zeros past s_{i-1}),
// from the FP64 inverse that k_invert_dense leaves in the right half of its
// s x 2s work rows; FP64 sums in index order, stored as T.
template <class T>
__global__ void k_overlap_m(const int32_t* __restrict__ agg_s, const int32_t* __restrict__ agg_w,
                            const int64_t* __restrict__ a_off, const int64_t* __restrict__ l_off,
                            const int64_t* __restrict__ m_off, int32_t width, const double* __restrict__ work,
                            const double* __restrict__ L_all, T* __restrict__ M_all) {
  const int i = blockIdx.x + 1;
  const int32_t s = agg_s[i], sp = agg_s[i - 1], wp = agg_w[i - 1];
  const double* Winv = work + 2 * a_off[i];  // row r: [I | A_i^{-1}] of width 2s
  const double* L = L_all + l_off[i - 1];      // wp x sp
  const int32_t spp = width;
  T* M = M_all + m_off[i];
  for (int64_t t = threadIdx.x; t < (int64_t)s * spp; t += blockDim.x) {
    const int32_t r = (int32_t)(t / spp), c = (int32_t)(t % spp);
    double acc = 0.0;
    if (c < sp)
      for (int32_t q = 0; q < wp; ++q) acc += Winv[(int64_t)r * 2 * s + s + q] * L[(int64_t)q * sp + c];
    M[t] = (T)acc;
  }
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_overlap_split(int32_t k, const int32_t* agg_s, const int32_t* agg_w, const int64_t* g_off,
                          const int64_t* a_off, const int64_t* l_off, const double* Se, double* A, double* L,
                          hipStream_t s) {
  if (k > 0) k_overlap_split<<<k, 256, 0, s>>>(agg_s, agg_w, g_off, a_off, l_off, Se, A, L);
}

void launch_overlap_m(int32_t k, const int32_t* agg_s, const int32_t* agg_w, const int64_t* a_off,
                      const int64_t* l_off, const int64_t* m_off, int32_t width, const double* winv, const double* L,
                      void* M, int m_double, hipStream_t s) {
  if (k < 2) return;
  if (m_double)
    k_overlap_m<double><<<k - 1, 256, 0, s>>>(agg_s, agg_w, a_off, l_off, m_off, width, winv, L, (double*)M);
  else
    k_overlap_m<float><<<k - 1, 256, 0, s>>>(agg_s, agg_w, a_off, l_off, m_off, width, winv, L, (float*)M);
}

void launch_exact_schur_update(int32_t nsep, const int32_t* pcol_ptr, const int32_t* pair_sub, const int64_t* pair_off,
                               const SubInfo* subs, const int32_t* agg_of, const int32_t* agg_off, const int64_t* g_off,
                               const int32_t* f_rowptr, const int32_t* f_colidx, const double* f_vals,
                               const double* U, double* S, hipStream_t s) {
  if (nsep > 0)
    k_exact_schur_update<<<nsep, 64, 0, s>>>(pcol_ptr, pair_sub, pair_off, subs, agg_of, agg_off, g_off, f_rowptr,
                                             f_colidx, f_vals, U, S);
}
void launch_row_scale(const int32_t* rowptr, const double* vals, int32_t N, int scale, double* R, hipStream_t s) {
  if (N > 0) k_row_scale<<<nblocks(N, 256), 256, 0, s>>>(rowptr, vals, N, scale, R);
}
void launch_gather_scaled(const int32_t* src, const int32_t* orow, const double* vals, const double* R, int64_t n,
                          double* out, hipStream_t s) {
  if (n > 0) k_gather_scaled<<<nblocks(n, 256), 256, 0, s>>>(src, orow, vals, R, n, out);
}
void launch_gather(const int32_t* src, const double* in, int64_t n, double* out, hipStream_t s) {
  if (n > 0) k_gather<<<nblocks(n, 256), 256, 0, s>>>(src, in, n, out);
}
void launch_scatter_band(const int64_t* dst, const int32_t* src, const double* cpv, int64_t n, double* ab,
                         hipStream_t s) {
  if (n > 0) k_scatter<<<nblocks(n, 256), 256, 0, s>>>(dst, src, cpv, n, ab);
}
void launch_dense_scatter(const int64_t* dst, const int32_t* src, const double* cpv, int64_t n, double* out,
                          hipStream_t s) {
  if (n > 0) k_scatter<<<nblocks(n, 256), 256, 0, s>>>(dst, src, cpv, n, out);
}
void launch_band_pad_identity(const SubInfo* subs, int32_t m, double* ab, hipStream_t s) {
  if (m > 0) k_band_pad_identity<<<m, 256, 0, s>>>(subs, ab);
}
void launch_band_colnorm(const double* ab, const SubInfo* subs, int32_t m, int32_t npad_max, double* colnorm,
                         hipStream_t s) {
  if (m > 0 && npad_max > 0) k_band_colnorm<<<dim3((npad_max + 255) / 256, m), 256, 0, s>>>(ab, subs, colnorm);
}
void launch_band_nnz(const double* ab, const SubInfo* subs, int32_t m, int32_t n_max, int64_t* counts,
                     hipStream_t s) {
  if (m == 0) return;
  ADDNS_HIP(hipMemsetAsync(counts, 0, sizeof(int64_t) * m, s));
  if (n_max > 0)
    k_band_nnz<<<dim3((n_max + kNnzCols - 1) / kNnzCols, m), 256, 0, s>>>(ab, subs,
                                                                         reinterpret_cast<unsigned long long*>(counts));
}
template <int NS>
void run_band_lu(double* ab, int32_t* ipiv, const SubInfo* subs, int32_t m, int32_t* info, const double* colnorm,
                 double tau, int32_t prmax, int32_t ntmax, const int32_t* sub_list, hipStream_t s) {
  const size_t smem = sizeof(double) * ((size_t)3 * kPanel * prmax + (size_t)kPanel * ntmax);
  static size_t raised = 64 * 1024;
  if (smem > raised) {
    ADDNS_HIP(hipFuncSetAttribute((const void*)k_band_lu_blocked<NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)smem));
    raised = smem;
  }
  k_band_lu_blocked<NS><<<m, kLuThreads, smem, s>>>(ab, ipiv, subs, info, colnorm, tau, prmax, ntmax, sub_list);
}
bool band_lu_blocked(int32_t kl_max) { return (kl_max + kPanel + 63) / 64 <= 4; }
void launch_band_lu(double* ab, int32_t* ipiv, const SubInfo* subs, int32_t m, int32_t* info, const double* colnorm,
                    double tau, int32_t kl_max, int32_t kv_max, const int32_t* sub_list, hipStream_t s) {
  if (m == 0) return;
  if (sub_list && !band_lu_blocked(kl_max)) throw std::logic_error("a subdomain list needs the blocked band LU");
  const int32_t prmax = kl_max + kPanel, ntmax = std::max(kv_max, 1);
  // panel rows per lane in registers (64 * NS >= prmax); wider bands take the
  // unblocked elimination
  switch ((prmax + 63) / 64) {
    case 1: run_band_lu<1>(ab, ipiv, subs, m, info, colnorm, tau, prmax, ntmax, sub_list, s); break;
    case 2: run_band_lu<2>(ab, ipiv, subs, m, info, colnorm, tau, prmax, ntmax, sub_list, s); break;
    case 3: run_band_lu<3>(ab, ipiv, subs, m, info, colnorm, tau, prmax, ntmax, sub_list, s); break;
    case 4: run_band_lu<4>(ab, ipiv, subs, m, info, colnorm, tau, prmax, ntmax, sub_list, s); break;
    default: k_band_lu<<<m, kSetupThreads, 0, s>>>(ab, ipiv, subs, info, colnorm, tau); break;
  }
}
template <class T>
void run_convert_lower_slab(const SubInfo* subs, const LBlk* lb, int32_t nblk, int32_t slab, int32_t nbl_max,
                            const double* work, T* lmat, int32_t* info, const int32_t* blk_list, hipStream_t s) {
  const size_t smem = sizeof(double) * ((size_t)slab * (nbl_max + 1) + 2 * (size_t)nbl_max);
  static size_t raised = 64 * 1024;
  if (smem > raised) {
    ADDNS_HIP(hipFuncSetAttribute((const void*)k_convert_lower_slab<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)smem));
    raised = smem;
  }
  const dim3 grid((unsigned)((nbl_max + slab - 1) / slab), (unsigned)nblk);
  k_convert_lower_slab<T><<<grid, kLSlabThreads, smem, s>>>(subs, lb, work, slab, lmat, info, blk_list);
}
// slabs of up to 32 columns within 96 KB of LDS
static int32_t lower_slab(int32_t nbl_max) {
  return (int32_t)std::min<int64_t>(32, (96 * 1024 / 8 - 2 * (int64_t)nbl_max) / ((int64_t)nbl_max + 1));
}
static int32_t upper_slab(int32_t nbu_max) {
  return (int32_t)std::min<int64_t>(32, (96 * 1024 / 8) / ((int64_t)nbu_max + 1));
}
bool convert_slabs(int32_t nbl_max, int32_t kl_max, int32_t nbu_max, int32_t kv_max) {
  return lower_slab(nbl_max) >= 1 && sizeof(int32_t) * (2 * (size_t)nbl_max + kl_max) <= 64 * 1024 &&
         upper_slab(nbu_max) >= 1 && kv_max < kUFetch * kUSlabThreads;
}
void launch_convert_lower(const double* ab, const int32_t* ipiv, const SubInfo* subs, const LBlk* lb, int32_t nblk,
                          double* work, int32_t* lperm, void* lmat, int prec, int32_t* info, int32_t nbl_max,
                          int32_t kl_max, const int32_t* blk_list, hipStream_t s) {
  if (nblk == 0) return;
  const int32_t slab = lower_slab(nbl_max);
  const size_t prep_smem = sizeof(int32_t) * (2 * (size_t)nbl_max + kl_max);
  if (slab >= 1 && prep_smem <= 64 * 1024) {
    k_convert_lower_prep<<<nblk, kSetupThreads, prep_smem, s>>>(ab, ipiv, subs, lb, work, lperm, blk_list);
    if (prec == P64)
      run_convert_lower_slab<double>(subs, lb, nblk, slab, nbl_max, work, (double*)lmat, info, blk_list, s);
    else
      run_convert_lower_slab<float>(subs, lb, nblk, slab, nbl_max, work, (float*)lmat, info, blk_list, s);
    return;
  }
  throw std::logic_error("lower block too wide for the slab conversion");
}
template <class T>
void run_convert_upper_slab(const double* ab, const SubInfo* subs, const UBlk* ub, int32_t nblk, int32_t slab,
                            int32_t nbu_max, int32_t kv_max, T* uinv, T* u12, int32_t* info, const int32_t* blk_list,
                            hipStream_t s) {
  const size_t smem = sizeof(double) * ((size_t)slab * (nbu_max + 1) + 2 * (size_t)(kv_max + 1));
  static size_t raised = 64 * 1024;
  if (smem > raised) {
    ADDNS_HIP(hipFuncSetAttribute((const void*)k_convert_upper_slab<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)smem));
    raised = smem;
  }
  const dim3 grid((unsigned)((nbu_max + slab - 1) / slab), (unsigned)nblk);
  k_convert_upper_slab<T><<<grid, kUSlabThreads, smem, s>>>(ab, subs, ub, slab, kv_max, uinv, u12, info, blk_list);
}
void launch_convert_upper(const double* ab, const SubInfo* subs, const UBlk* ub, int32_t nblk, double* work,
                          void* uinv, void* u12, int prec, int32_t* info, int32_t nbu_max, int32_t kv_max,
                          const int32_t* blk_list, hipStream_t s) {
  if (nblk == 0) return;
  // slabs of up to 32 columns within 96 KB of LDS; U's column fits the
  // values per thread of the step buffer
  const int32_t slab = upper_slab(nbu_max);
  if (slab >= 1 && kv_max < kUFetch * kUSlabThreads) {
    if (prec == P64)
      run_convert_upper_slab<double>(ab, subs, ub, nblk, slab, nbu_max, kv_max, (double*)uinv, (double*)u12, info,
                                     blk_list, s);
    else
      run_convert_upper_slab<float>(ab, subs, ub, nblk, slab, nbu_max, kv_max, (float*)uinv, (float*)u12, info,
                                    blk_list, s);
    return;
  }
  throw std::logic_error("upper block too wide for the slab conversion");
}
void launch_schur_blocks(int32_t k, const int32_t* agg_s, const int32_t* agg_d, const int64_t* g_off,
                         const int64_t* dd_off, const int64_t* de_off, const int64_t* df_off, double* G, double* Dd,
                         double* De, double* Df, int32_t* info, int rowsum, hipStream_t s) {
  if (k > 0)
    k_schur_blocks<<<k, kSetupThreads, 0, s>>>(agg_s, agg_d, g_off, dd_off, de_off, df_off, G, Dd, De, Df, info,
                                              rowsum);
}
void launch_invert_dense(int32_t k, const int32_t* agg_s, const int64_t* g_off, const double* S, double* work,
                         int32_t* info, const int64_t* sinv_off, void* sinv, float* scale, int prec, hipStream_t s) {
  if (k == 0) return;
  if (prec == P64)
    k_invert_dense<double><<<k, kSetupThreads, 0, s>>>(agg_s, g_off, S, work, info, sinv_off, (double*)sinv, scale,
                                                        prec);
  else if (prec == P32)
    k_invert_dense<float><<<k, kSetupThreads, 0, s>>>(agg_s, g_off, S, work, info, sinv_off, (float*)sinv, scale, prec);
  else
    k_invert_dense<__half><<<k, kSetupThreads, 0, s>>>(agg_s, g_off, S, work, info, sinv_off, (__half*)sinv, scale,
                                                        prec);
}

}  // namespace addns
