// Kernels of the coarse-grid correction of the interface solve (section 6
// proposes a coarse grid correction; the two-level form is
//   y = E_c^{-1} Z^T t,   x2 = Z y + Shat^{-1} (t - S Z y),
// with E_c = Z^T S Z and S = G - F D^{-1} E the interface Schur complement).
//
// Setup: S Z column by column from its definition (the columns D_j^{-1} E_j z_c
// come from the interior sweep), E_c = Z^T S Z, and E_c^{-1} by Gauss-Jordan
// elimination with partial pivoting.  Apply: the restriction t, Z^T t; the
// coarse solve y = E_c^{-1} (Z^T t); the block solve on t - S Z y with Z y
// added (k_interface_solve).  Every reduction runs in a fixed order, so the
// results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <stdexcept>
#include <string>


#include "precond.h"

namespace addns {
namespace {

// Sum over the 64 lanes of a wave in a fixed butterfly order.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wave per separator row of S Z: the entry for coarse column c is
//   (G z_c)(row) - sum_j F(row, int_j) W_(j,c),
// W_(j,c) = D_j^{-1} E_j z_c from the column solves.
__global__ void k_coarse_sz(int32_t ns, int32_t n_int, const int32_t* __restrict__ cp_rowptr,
                            const int32_t* __restrict__ cp_colidx, const double* __restrict__ cp_vals,
                            const int32_t* __restrict__ f_rowptr, const int32_t* __restrict__ f_colidx,
                            const double* __restrict__ f_vals, const int32_t* __restrict__ piece,
                            const double* __restrict__ z0, const double* __restrict__ z1,
                            const int32_t* __restrict__ colp, const int32_t* __restrict__ colk,
                            const int32_t* __restrict__ szp, const int32_t* __restrict__ szc,
                            const int32_t* __restrict__ sub_of, const int32_t* __restrict__ int_off,
                            const int32_t* __restrict__ pair_sub, const int32_t* __restrict__ cpair_ptr,
                            const int64_t* __restrict__ pair_off, const double* __restrict__ W,
                            double* __restrict__ szv) {
  const int32_t row = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= ns) return;
  const int32_t r = n_int + row;
  for (int32_t e = szp[row] + lane; e < szp[row + 1]; e += 64) {
    const int32_t c = szc[e];
    const int32_t pc = colp[c];
    const double* zv = colk[c] ? z1 : z0;
    double acc = 0.0;
    for (int32_t t = cp_rowptr[r]; t < cp_rowptr[r + 1]; ++t) {
      const int32_t col = cp_colidx[t];
      if (col >= n_int && piece[col - n_int] == pc) acc += cp_vals[t] * zv[col - n_int];
    }
    for (int32_t t = f_rowptr[row]; t < f_rowptr[row + 1]; ++t) {
      const int32_t col = f_colidx[t];
      const int32_t j = sub_of[col];
      int64_t off = -1;
      for (int32_t q = cpair_ptr[c]; q < cpair_ptr[c + 1]; ++q)
        if (pair_sub[q] == j) off = pair_off[q];
      if (off >= 0) acc -= f_vals[t] * W[off + (col - int_off[j])];
    }
    szv[e] = acc;
  }
}

// One wave per restriction group (a piece): the rows of E_c that belong to
// the group's columns, E_c(c', c) = sum over the group's rows, in their stored
// order, of z_c'(row) S Z(row, c).  Each lane owns columns c of the group's
// column list and accumulates them in registers (S Z(row, c) found by binary
// search in the row's ascending column list); no element is written twice.
__global__ void k_coarse_ec(int32_t ngrp, const int32_t* __restrict__ goff, const int32_t* __restrict__ grows,
                            const int32_t* __restrict__ gc0, const int32_t* __restrict__ gc1,
                            const int32_t* __restrict__ gcoff, const int32_t* __restrict__ gcols,
                            const double* __restrict__ z0, const double* __restrict__ z1,
                            const int32_t* __restrict__ szp, const int32_t* __restrict__ szc,
                            const double* __restrict__ szv, const int32_t* __restrict__ boff,
                            const int32_t* __restrict__ cblk, const int64_t* __restrict__ beoff,
                            double* __restrict__ Ec) {
  const int32_t g = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (g >= ngrp) return;
  const int32_t c0 = gc0[g], c1 = gc1[g];
  if (c0 < 0) return;
  // the group's columns and all columns it couples to share one block
  const int32_t b = cblk[c0], o = boff[b], n = boff[b + 1] - o;
  double* E = Ec + beoff[b];
  for (int32_t q = gcoff[g] + lane; q < gcoff[g + 1]; q += 64) {
    const int32_t c = gcols[q];
    double a0 = 0.0, a1 = 0.0;
    for (int32_t t = goff[g]; t < goff[g + 1]; ++t) {
      const int32_t row = grows[t];
      int32_t lo = szp[row], hi = szp[row + 1];
      while (lo < hi) {
        const int32_t mid = (lo + hi) / 2;
        if (szc[mid] < c) lo = mid + 1;
        else hi = mid;
      }
      if (lo < szp[row + 1] && szc[lo] == c) {
        const double v = szv[lo];
        a0 += z0[row] * v;
        a1 += z1[row] * v;
      }
    }
    E[(int64_t)(c0 - o) * n + (c - o)] = a0;
    if (c1 >= 0) E[(int64_t)(c1 - o) * n + (c - o)] = a1;
  }
}

// Residual of the (subdomain, coarse column) solves in FP64, one workgroup
// per pair: scratch = E_j z_c - A_jj W on the interior rows of subdomain j,
// both read from the permuted, scaled C (separator columns: E; columns of
// the same interior: A_jj).
__global__ void k_pair_residual(int32_t n_int, const SubInfo* __restrict__ subs, const int32_t* __restrict__ pair_sub,
                                const int32_t* __restrict__ pair_col, const int64_t* __restrict__ pair_off,
                                const int32_t* __restrict__ cp_rowptr, const int32_t* __restrict__ cp_colidx,
                                const double* __restrict__ cp_vals, const int32_t* __restrict__ piece,
                                const double* __restrict__ z0, const double* __restrict__ z1,
                                const int32_t* __restrict__ colp, const int32_t* __restrict__ colk,
                                const double* __restrict__ W, double* __restrict__ scratch) {
  const int32_t q = blockIdx.x;
  const SubInfo sb = subs[pair_sub[q]];
  const int32_t c = pair_col[q], pc = colp[c];
  const double* zv = colk[c] ? z1 : z0;
  const int64_t off = pair_off[q];
  for (int32_t r = threadIdx.x; r < sb.n; r += blockDim.x) {
    const int32_t R = sb.int_off + r;
    double acc = 0.0;
    for (int32_t t = cp_rowptr[R]; t < cp_rowptr[R + 1]; ++t) {
      const int32_t col = cp_colidx[t];
      if (col >= n_int) {
        if (piece[col - n_int] == pc) acc += cp_vals[t] * zv[col - n_int];
      } else if (col >= sb.int_off && col < sb.int_off + sb.n) {
        acc -= cp_vals[t] * W[off + (col - sb.int_off)];
      }
    }
    scratch[off + r] = acc;
  }
}

// W += dW on the interior rows of every pair.
__global__ void k_pair_add(const SubInfo* __restrict__ subs, const int32_t* __restrict__ pair_sub,
                           const int64_t* __restrict__ pair_off, const double* __restrict__ dW, double* __restrict__ W) {
  const int32_t q = blockIdx.x;
  const int32_t n = subs[pair_sub[q]].n;
  const int64_t off = pair_off[q];
  for (int32_t r = threadIdx.x; r < n; r += blockDim.x) W[off + r] += dW[off + r];
}

// Largest |A| of every diagonal block (one workgroup per block), the scale
// of the singularity test.
__global__ void __launch_bounds__(1024) k_absmax(const double* __restrict__ A, const int32_t* __restrict__ boff,
                                                 const int64_t* __restrict__ beoff, double* __restrict__ out) {
  __shared__ double red[1024];
  const int32_t b = blockIdx.x;
  const int64_t n2 = beoff[b + 1] - beoff[b];
  const double* E = A + beoff[b];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n2; i += blockDim.x) m = fmax(m, fabs(E[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = red[0];
}

// Gauss-Jordan step k on every block of more than k columns, part 1 (one
// workgroup per block): pivot = first row i >= k of largest |A(i,k)|; copies
// of the pivot row and of column k (after the interchange), then the swap of
// rows k and pivot.  work: amax[nb], prow[nc], mcol[nc] (block b at boff[b]).
__global__ void __launch_bounds__(1024) k_gj_pivot(double* __restrict__ A, int32_t nb, int32_t k,
                                                   const int32_t* __restrict__ boff,
                                                   const int64_t* __restrict__ beoff, int32_t* __restrict__ perm,
                                                   double* __restrict__ work, int32_t nc, int32_t* __restrict__ info) {
  __shared__ double bv[1024];
  __shared__ int32_t bi[1024];
  const int32_t b = blockIdx.x;
  const int32_t o = boff[b], n = boff[b + 1] - o;
  if (k >= n) return;
  double* E = A + beoff[b];
  const int tid = threadIdx.x;
  double best = -1.0;
  int32_t bidx = n;
  for (int32_t i = k + tid; i < n; i += blockDim.x) {
    const double v = fabs(E[(int64_t)i * n + k]);
    if (v > best) {
      best = v;
      bidx = i;
    }
  }
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (tid < s) {
      const double v2 = bv[tid + s];
      const int32_t i2 = bi[tid + s];
      if (v2 > bv[tid] || (v2 == bv[tid] && i2 < bi[tid])) {
        bv[tid] = v2;
        bi[tid] = i2;
      }
    }
    __syncthreads();
  }
  const int32_t p = bi[0];
  if (tid == 0) {
    perm[o + k] = p;
    if (!(bv[0] > 1e-13 * work[b]) && info[0] == 0) info[0] = o + k + 1;
  }
  double* prow = work + nb + o;
  double* mcol = work + nb + nc + o;
  // copies first, from the matrix before the interchange (rows k and p
  // trade places); every load has returned before its thread reaches the
  // barrier, so the interchange below cannot overtake them
  for (int32_t i = tid; i < n; i += blockDim.x) {
    const int32_t src = i == k ? p : (i == p ? k : i);
    mcol[i] = E[(int64_t)src * n + k];
  }
  for (int32_t j = tid; j < n; j += blockDim.x) prow[j] = E[(int64_t)p * n + j];
  __syncthreads();
  if (p != k)
    for (int32_t j = tid; j < n; j += blockDim.x) {
      const double x = E[(int64_t)k * n + j], y = E[(int64_t)p * n + j];
      E[(int64_t)k * n + j] = y;
      E[(int64_t)p * n + j] = x;
    }
}

// Gauss-Jordan step k, part 2: in-place inverse update of every block with
// more than k columns, from the copied pivot row and column (every element
// reads only the copies and itself).  Grid: x over columns, y over the
// coarse rows of all blocks.
__global__ void k_gj_update(double* __restrict__ A, int32_t nb, int32_t nc, int32_t k,
                            const int32_t* __restrict__ boff, const int32_t* __restrict__ cblk,
                            const int64_t* __restrict__ beoff, const double* __restrict__ work) {
  const int32_t r = blockIdx.y;
  const int32_t b = cblk[r];
  const int32_t o = boff[b], n = boff[b + 1] - o;
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || j >= n) return;
  const int32_t i = r - o;
  const double* prow = work + nb + o;
  const double* mcol = work + nb + nc + o;
  const double piv = prow[k];
  const double inv = 1.0 / piv;
  double& a = A[beoff[b] + (int64_t)i * n + j];
  if (i == k) a = j == k ? inv : prow[j] * inv;
  else if (j == k) a = -mcol[i] * inv;
  else a -= mcol[i] * (prow[j] * inv);
}

// The same Gauss-Jordan inversion with every step in one workgroup per
// block (one launch instead of two per step): the block's largest |entry|,
// then per step k the pivot (first row of largest |A(i,k)| among rows >= k,
// by one wave), the copies of pivot row and column, the interchange and the
// update, and finally the column interchanges undone.  Blocks of at most
// kGjLds columns are worked in LDS, larger ones in place in memory.  Each
// element receives the operations of k_gj_pivot, k_gj_update and
// k_gj_colswap in the same order, so the inverse is the same bit for bit.
constexpr int kGjLds = 88;
constexpr int kGjFusedMax = 1024;
template <bool LDS>
__global__ void __launch_bounds__(1024) k_gj_fused(double* __restrict__ A, const int32_t* __restrict__ boff,
                                                   const int64_t* __restrict__ beoff, int32_t* __restrict__ perm,
                                                   int32_t* __restrict__ info) {
  __shared__ double s_E[LDS ? kGjLds * kGjLds : 1];
  __shared__ double prow[kGjFusedMax], mcol[kGjFusedMax];
  __shared__ double red[16];
  __shared__ int32_t s_p[kGjFusedMax];
  const int32_t b = blockIdx.x;
  const int32_t o = boff[b], n = boff[b + 1] - o;
  double* G = A + beoff[b];
  double* E = LDS ? s_E : G;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = (int)(blockDim.x >> 6);
  double m = 0.0;
  for (int32_t e = tid; e < n * n; e += blockDim.x) {
    const double x = G[e];
    if (LDS) E[e] = x;
    m = fmax(m, fabs(x));
  }
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if (lane == 0) red[wave] = m;
  __syncthreads();
  double amax = 0.0;
  for (int w = 0; w < nw; ++w) amax = fmax(amax, red[w]);
  for (int32_t k = 0; k < n; ++k) {
    if (wave == 0) {
      // pivot: largest |A(i,k)|, the smallest such row on ties
      double best = -1.0;
      int32_t bidx = n;
      for (int32_t i = k + lane; i < n; i += 64) {
        const double v = fabs(E[i * n + k]);
        if (v > best) {
          best = v;
          bidx = i;
        }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        const double v2 = __shfl_xor(best, off);
        const int32_t i2 = __shfl_xor(bidx, off);
        if (v2 > best || (v2 == best && i2 < bidx)) {
          best = v2;
          bidx = i2;
        }
      }
      if (lane == 0) {
        s_p[k] = bidx;
        if (!(best > 1e-13 * amax) && info[0] == 0) info[0] = o + k + 1;
      }
    }
    __syncthreads();
    const int32_t p = s_p[k];
    // copies from the matrix before the interchange
    for (int32_t i = tid; i < n; i += blockDim.x) {
      const int32_t src = i == k ? p : (i == p ? k : i);
      mcol[i] = E[src * n + k];
      prow[i] = E[p * n + i];
    }
    __syncthreads();
    if (p != k)
      for (int32_t j = tid; j < n; j += blockDim.x) {
        const double x = E[k * n + j], y = E[p * n + j];
        E[k * n + j] = y;
        E[p * n + j] = x;
      }
    __syncthreads();
    const double inv = 1.0 / prow[k];
    for (int32_t e = tid; e < n * n; e += blockDim.x) {
      const int32_t i = e / n, j = e % n;
      double& a = E[e];
      if (i == k) a = j == k ? inv : prow[j] * inv;
      else if (j == k) a = -mcol[i] * inv;
      else a -= mcol[i] * (prow[j] * inv);
    }
    __syncthreads();
  }
  // the pivot rows go to memory once, after the loop
  for (int32_t k = tid; k < n; k += blockDim.x) perm[o + k] = s_p[k];
  // column interchanges undone, one thread per row
  for (int32_t r = tid; r < n; r += blockDim.x) {
    double* row = E + r * n;
    for (int32_t k = n - 1; k >= 0; --k) {
      const int32_t p = s_p[k];
      if (p != k) {
        const double t = row[k];
        row[k] = row[p];
        row[p] = t;
      }
    }
  }
  if (LDS) {
    __syncthreads();
    for (int32_t e = tid; e < n * n; e += blockDim.x) G[e] = E[e];
  }
}

// The same again with the block in registers: thread t holds column t % n,
// rows t / n + R m (m < M) with R = 1024 / n row groups, for blocks with
// n <= R M.  A step moves only column k, rows k and p and the pivot through
// LDS, so the matrix is read from and written to memory once.  Every wave
// finds the pivot itself (the same search over the same column, so the same
// row), and the update of step k leaves column k + 1 in the other of two
// column buffers: two barriers a step.  Same operations on every element in
// the same order, so the same inverse bit for bit.
constexpr int kGjRegs = 26;
template <int M>
__global__ void __launch_bounds__(1024) k_gj_regs(double* __restrict__ A, const int32_t* __restrict__ boff,
                                                  const int64_t* __restrict__ beoff, int32_t* __restrict__ perm,
                                                  int32_t* __restrict__ info) {
  __shared__ double colk[2][kGjFusedMax], rowp[kGjFusedMax], rowk[kGjFusedMax];
  __shared__ double red[16];
  __shared__ int32_t s_p[kGjFusedMax];
  const int32_t b = blockIdx.x;
  const int32_t o = boff[b], n = boff[b + 1] - o;
  double* G = A + beoff[b];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = (int)(blockDim.x >> 6);
  const int32_t R = 1024 / n, j = tid % n, g = tid / n;
  const bool jv = g < R;
  double a[M];
  double m = 0.0;
#pragma unroll
  for (int q = 0; q < M; ++q) {
    const int32_t i = g + R * q;
    a[q] = (jv && i < n) ? G[i * n + j] : 0.0;
    m = fmax(m, fabs(a[q]));
    if (jv && j == 0 && i < n) colk[0][i] = a[q];
  }
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if (lane == 0) red[wave] = m;
  __syncthreads();
  double amax = 0.0;
  for (int w = 0; w < nw; ++w) amax = fmax(amax, red[w]);
  for (int32_t k = 0; k < n; ++k) {
    const double* ck = colk[k & 1];
    double* cn = colk[(k + 1) & 1];
    double best = -1.0;
    int32_t bidx = n;
    for (int32_t i = k + lane; i < n; i += 64) {
      const double v = fabs(ck[i]);
      if (v > best) {
        best = v;
        bidx = i;
      }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const double v2 = __shfl_xor(best, off);
      const int32_t i2 = __shfl_xor(bidx, off);
      if (v2 > best || (v2 == best && i2 < bidx)) {
        best = v2;
        bidx = i2;
      }
    }
    // lane 0's row, as one search would give it
    const int32_t p = __shfl(bidx, 0);
    if (tid == 0) {
      s_p[k] = p;
      if (!(best > 1e-13 * amax) && info[0] == 0) info[0] = o + k + 1;
    }
    if (jv)
#pragma unroll
      for (int q = 0; q < M; ++q) {
        const int32_t i = g + R * q;
        if (i == p) rowp[j] = a[q];
        if (i == k) rowk[j] = a[q];
      }
    __syncthreads();
    // mcol(i) = column k after the interchange, prow = row p before it
    const double inv = 1.0 / rowp[k];
    if (jv) {
      const double pj = rowp[j], kj = rowk[j];
#pragma unroll
      for (int q = 0; q < M; ++q) {
        const int32_t i = g + R * q;
        if (i >= n) continue;
        const int32_t src = i == k ? p : (i == p ? k : i);
        const double x = i == p ? kj : (i == k ? pj : a[q]);  // the interchange
        if (i == k) a[q] = j == k ? inv : pj * inv;
        else if (j == k) a[q] = -ck[src] * inv;
        else a[q] = x - ck[src] * (pj * inv);
        if (j == k + 1) cn[i] = a[q];
      }
    }
    __syncthreads();
  }
  // the pivot rows go to memory once, after the loop: a store in a step
  // would hold the step's barrier until it completes
  for (int32_t k = tid; k < n; k += blockDim.x) perm[o + k] = s_p[k];
  // column interchanges undone: column j ends where the swaps k = n-1 .. 0,
  // applied in order, move it
  if (jv) {
    int32_t c = j;
    for (int32_t k = n - 1; k >= 0; --k) {
      const int32_t p = s_p[k];
      if (p == k) continue;
      if (c == k) c = p;
      else if (c == p) c = k;
    }
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const int32_t i = g + R * q;
      if (i < n) G[i * n + c] = a[q];
    }
  }
}

// Undo the row interchanges on the columns of each block's inverse: inv(A)
// is inv(P A) with its columns swapped back in reverse order.  One thread
// per coarse row.
__global__ void k_gj_colswap(double* __restrict__ A, int32_t nc, const int32_t* __restrict__ boff,
                             const int32_t* __restrict__ cblk, const int64_t* __restrict__ beoff,
                             const int32_t* __restrict__ perm) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nc) return;
  const int32_t b = cblk[r], o = boff[b], n = boff[b + 1] - o;
  double* row = A + beoff[b] + (int64_t)(r - o) * n;
  for (int32_t k = n - 1; k >= 0; --k) {
    const int32_t p = perm[o + k];
    if (p != k) {
      const double t = row[k];
      row[k] = row[p];
      row[p] = t;
    }
  }
}

// Restriction (one wave per group): t = y2 - F z1 on the group's rows, and
// for a piece its two entries of g = Z^T t.
__global__ void k_coarse_restrict(int32_t ngrp, int32_t n_int, const int32_t* __restrict__ goff,
                                  const int32_t* __restrict__ grows, const int32_t* __restrict__ gc0,
                                  const int32_t* __restrict__ gc1, const int32_t* __restrict__ f_rowptr,
                                  const int32_t* __restrict__ f_colidx, const double* __restrict__ f_vals,
                                  const double* __restrict__ z0, const double* __restrict__ z1,
                                  const double* __restrict__ y, const double* __restrict__ zin,
                                  double* __restrict__ t, double* __restrict__ g, const int32_t* __restrict__ live,
                                  const int32_t* __restrict__ grp_sys) {
  const int32_t grp = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (grp >= ngrp) return;
  // a piece lies inside one system; the groups of pressure-like rows that
  // hold no coarse column may span systems and are always computed
  if (live && gc0[grp] >= 0 && !live[grp_sys[grp]]) return;
  const int32_t a = goff[grp], cnt = goff[grp + 1] - a;
  double p0 = 0.0, p1 = 0.0;
  if (lane < cnt) {
    const int32_t row = grows[a + lane];
    double acc = y[n_int + row];
    for (int32_t e = f_rowptr[row]; e < f_rowptr[row + 1]; ++e) acc -= f_vals[e] * zin[f_colidx[e]];
    t[row] = acc;
    p0 = z0[row] * acc;
    p1 = z1[row] * acc;
  }
  const int32_t c0 = gc0[grp], c1 = gc1[grp];
  if (c0 >= 0) {
    p0 = wave_sum(p0);
    p1 = wave_sum(p1);
    if (lane == 0) {
      g[c0] = p0;
      if (c1 >= 0) g[c1] = p1;
    }
  }
}

// Coarse solve y = E_c^{-1} g blockwise, one wave per coarse row (a row of
// its block's row-major inverse).
__global__ void k_coarse_solve(int32_t nc, const double* __restrict__ Einv, const int32_t* __restrict__ boff,
                               const int32_t* __restrict__ cblk, const int64_t* __restrict__ beoff,
                               const double* __restrict__ g, double* __restrict__ y) {
  const int32_t i = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (i >= nc) return;
  const int32_t b = cblk[i], o = boff[b], n = boff[b + 1] - o;
  const double* row = Einv + beoff[b] + (int64_t)(i - o) * n;
  const double* gb = g + o;
  double acc = 0.0;
  for (int32_t j = lane; j < n; j += 64) acc += row[j] * gb[j];
  acc = wave_sum(acc);
  if (lane == 0) y[i] = acc;
}

}  // namespace

void launch_coarse_sz(const addns_precond* pc, const int32_t* sub_of, const int32_t* pair_sub,
                      const int32_t* cpair_ptr, const int64_t* pair_off, const int32_t* int_off,
                      const double* W, hipStream_t s) {
  const Plan& pl = pc->plan;
  if (pl.nsep == 0) return;
  const int waves = 4;
  k_coarse_sz<<<(pl.nsep + waves - 1) / waves, 64 * waves, 0, s>>>(
      pl.nsep, pl.n_int, pc->cp_rowptr.as<int32_t>(), pc->cp_colidx.as<int32_t>(), pc->cp_vals.as<double>(),
      pc->f_rowptr.as<int32_t>(), pc->f_colidx.as<int32_t>(), pc->f_vals.as<double>(), pc->cz_piece.as<int32_t>(),
      pc->cz_z0.as<double>(), pc->cz_z1.as<double>(), pc->cz_colp.as<int32_t>(), pc->cz_colk.as<int32_t>(),
      pc->cz_szp.as<int32_t>(), pc->cz_szc.as<int32_t>(), sub_of, int_off, pair_sub, cpair_ptr, pair_off, W,
      pc->cz_szv.as<double>());
}

void launch_coarse_refine(const addns_precond* pc, int32_t npairs, const int32_t* pair_sub, const int32_t* pair_col,
                          const int64_t* pair_off, double* W, double* scratch, double* dW, hipStream_t s) {
  if (npairs == 0) return;
  k_pair_residual<<<npairs, 256, 0, s>>>(pc->plan.n_int, pc->subs.as<SubInfo>(), pair_sub, pair_col, pair_off,
                                         pc->cp_rowptr.as<int32_t>(), pc->cp_colidx.as<int32_t>(),
                                         pc->cp_vals.as<double>(), pc->cz_piece.as<int32_t>(), pc->cz_z0.as<double>(),
                                         pc->cz_z1.as<double>(), pc->cz_colp.as<int32_t>(), pc->cz_colk.as<int32_t>(),
                                         W, scratch);
  launch_coarse_column_solves(pc, npairs, pair_sub, pair_col, pair_off, scratch, dW, 1, s);
  k_pair_add<<<npairs, 256, 0, s>>>(pc->subs.as<SubInfo>(), pair_sub, pair_off, dW, W);
}

void launch_coarse_ec(const addns_precond* pc, int32_t nc, double* Ec, hipStream_t s) {
  const int32_t ngrp = (int32_t)pc->coarse.grp_col0.size();
  if (ngrp == 0 || nc == 0) return;
  const int waves = 4;
  k_coarse_ec<<<(ngrp + waves - 1) / waves, 64 * waves, 0, s>>>(
      ngrp, pc->cz_goff.as<int32_t>(), pc->cz_grows.as<int32_t>(), pc->cz_gc0.as<int32_t>(),
      pc->cz_gc1.as<int32_t>(), pc->cz_gcoff.as<int32_t>(), pc->cz_gcols.as<int32_t>(), pc->cz_z0.as<double>(),
      pc->cz_z1.as<double>(), pc->cz_szp.as<int32_t>(), pc->cz_szc.as<int32_t>(), pc->cz_szv.as<double>(),
      pc->cz_boff.as<int32_t>(), pc->cz_cblk.as<int32_t>(), pc->cz_beoff.as<int64_t>(), Ec);
}

void launch_gj_invert(const addns_precond* pc, double* A, int32_t* perm, double* work, int32_t* info, hipStream_t s) {
  const CoarsePlan& cp = pc->coarse;
  const int32_t nb = (int32_t)cp.blk_off.size() - 1, nc = cp.space.nc;
  if (nb <= 0 || nc == 0) return;
  const int32_t* boff = pc->cz_boff.as<int32_t>();
  const int32_t* cblk = pc->cz_cblk.as<int32_t>();
  const int64_t* beoff = pc->cz_beoff.as<int64_t>();
  // the form: the block in LDS, in registers, in memory, or one launch
  // pair per step; every form gives the same inverse bit for bit.  The
  // ADDNS_COARSE_GJ environment variable (lds, registers, memory, steps)
  // forces one, for tests; a form too small for the blocks is an error.
  const bool lds_ok = cp.blk_max <= kGjLds;
  const bool regs_ok = cp.blk_max <= 1024 && (1024 / cp.blk_max) * kGjRegs >= cp.blk_max;
  const bool mem_ok = cp.blk_max <= kGjFusedMax;
  const char* force = std::getenv("ADDNS_COARSE_GJ");
  std::string form = force ? force : "";
  if (form.empty()) form = lds_ok ? "lds" : (regs_ok ? "registers" : (mem_ok ? "memory" : "steps"));
  if ((form == "lds" && !lds_ok) || (form == "registers" && !regs_ok) || (form == "memory" && !mem_ok) ||
      (form != "lds" && form != "registers" && form != "memory" && form != "steps"))
    throw ArgError("ADDNS_COARSE_GJ=" + form + " does not fit coarse blocks of " +
                                std::to_string(cp.blk_max) + " columns");
  if (form == "lds") {
    k_gj_fused<true><<<nb, 1024, 0, s>>>(A, boff, beoff, perm, info);
    return;
  }
  if (form == "registers") {
    k_gj_regs<kGjRegs><<<nb, 1024, 0, s>>>(A, boff, beoff, perm, info);
    return;
  }
  if (form == "memory") {
    k_gj_fused<false><<<nb, 1024, 0, s>>>(A, boff, beoff, perm, info);
    return;
  }
  k_absmax<<<nb, 1024, 0, s>>>(A, boff, beoff, work);
  const dim3 grid((unsigned)((cp.blk_max + 255) / 256), (unsigned)nc);
  for (int32_t k = 0; k < cp.blk_max; ++k) {
    k_gj_pivot<<<nb, 1024, 0, s>>>(A, nb, k, boff, beoff, perm, work, nc, info);
    k_gj_update<<<grid, 256, 0, s>>>(A, nb, nc, k, boff, cblk, beoff, work);
  }
  k_gj_colswap<<<(nc + 255) / 256, 256, 0, s>>>(A, nc, boff, cblk, beoff, perm);
}

void launch_coarse_restrict(const addns_precond* pc, const double* y, const double* z1, hipStream_t s) {
  const int32_t ngrp = (int32_t)pc->coarse.grp_col0.size();
  if (ngrp == 0) return;
  const int waves = 4;
  k_coarse_restrict<<<(ngrp + waves - 1) / waves, 64 * waves, 0, s>>>(
      ngrp, pc->plan.n_int, pc->cz_goff.as<int32_t>(), pc->cz_grows.as<int32_t>(), pc->cz_gc0.as<int32_t>(),
      pc->cz_gc1.as<int32_t>(), pc->f_rowptr.as<int32_t>(), pc->f_colidx.as<int32_t>(), pc->f_vals.as<double>(),
      pc->cz_z0.as<double>(), pc->cz_z1.as<double>(), y, z1, pc->cz_t.as<double>(), pc->cz_g.as<double>(),
      pc->mask_live, pc->mask_grp.as<int32_t>());
}

void launch_coarse_solve(const addns_precond* pc, hipStream_t s) {
  const int32_t nc = pc->coarse_nc;
  if (nc == 0) return;
  const int waves = 4;
  k_coarse_solve<<<(nc + waves - 1) / waves, 64 * waves, 0, s>>>(
      nc, pc->cz_einv.as<double>(), pc->cz_boff.as<int32_t>(), pc->cz_cblk.as<int32_t>(), pc->cz_beoff.as<int64_t>(),
      pc->cz_g.as<double>(), pc->cz_y.as<double>());
}

}  // namespace addns
