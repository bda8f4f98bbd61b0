// Krylov kernels of restarted (F)GMRES in FP64: CSR SpMV, fused
// axpy + next-dot steps of modified Gram-Schmidt, Givens rotations and the
// cycle-end update.  Dot products reduce per workgroup with wavefront
// shuffles and write one partial per workgroup; the consumer of a dot
// re-reduces all partials in a fixed order, so every result is bitwise
// reproducible run to run.
#include <hip/hip_runtime.h>

#include "precond.h"

namespace addns {
namespace {

constexpr int kKT = 256;          // threads per reduction workgroup
constexpr int kPerThread = 4;     // elements per thread per grid pass
constexpr int kMaxParts = 1024;
constexpr int kMaxRestart = 1024;  // Krylov dimension per cycle handled by k_finalize

__device__ inline double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sum of v over the workgroup (every thread gets the result).
__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q];
  return s;
}

// Fixed-order sum of nparts partials (identical in every workgroup).
__device__ inline double reduce_parts(const double* __restrict__ parts, int nparts, double* red) {
  double v = 0.0;
  for (int q = threadIdx.x; q < nparts; q += blockDim.x) v += parts[q];
  return block_sum(v, red);
}

// CSR row dot with 4 lanes per row would not pay at ~6 entries per row:
// one thread per row, rows assigned so that a wavefront covers 64 rows.
__device__ inline double row_dot(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                 const double* __restrict__ vals, const double* __restrict__ x, int32_t r) {
  double s = 0.0;
  for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) s += vals[e] * x[colidx[e]];
  return s;
}

__global__ void __launch_bounds__(kKT) k_spmv(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                             const double* __restrict__ vals, const double* __restrict__ x,
                                             double* __restrict__ y, int32_t n) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) y[r] = row_dot(rowptr, colidx, vals, x, r);
}

// w = A z and the partial of <w, v0>.
__global__ void __launch_bounds__(kKT)
k_spmv_dot(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx, const double* __restrict__ vals,
           const double* __restrict__ z, double* __restrict__ w, const double* __restrict__ v0, int32_t n,
           double* __restrict__ partials) {
  __shared__ double red[kKT / 64];
  double acc = 0.0;
  for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    double y = row_dot(rowptr, colidx, vals, z, r);
    w[r] = y;
    acc += y * v0[r];
  }
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// r = b - A x and the partial of <r, r>.
__global__ void __launch_bounds__(kKT)
k_residual(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx, const double* __restrict__ vals,
           const double* __restrict__ x, const double* __restrict__ b, double* __restrict__ r, int32_t n,
           double* __restrict__ partials) {
  __shared__ double red[kKT / 64];
  double acc = 0.0;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double y = b[i] - row_dot(rowptr, colidx, vals, x, i);
    r[i] = y;
    acc += y * y;
  }
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kKT)
k_dot_partials(const double* __restrict__ a, const double* __restrict__ b, int32_t n, double* __restrict__ partials) {
  __shared__ double red[kKT / 64];
  double acc = 0.0;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) acc += a[i] * b[i];
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// One modified Gram-Schmidt step: h = <w, v_i> from the partials of the
// previous kernel; w -= h v_i; partial of <w, v_next> (or <w, w> when
// v_next is null).  Workgroup 0 stores h.
__global__ void __launch_bounds__(kKT)
k_mgs_step(double* __restrict__ w, const double* __restrict__ vi, const double* __restrict__ vnext, int32_t n,
           const double* __restrict__ pin, double* __restrict__ pout, double* __restrict__ h_out, int nparts) {
  __shared__ double red[kKT / 64];
  // the vector loads do not depend on h: issue them before reducing the
  // partials of <w, v_i>, so that the two memory latencies overlap
  const int32_t stride = gridDim.x * blockDim.x, i0 = blockIdx.x * blockDim.x + threadIdx.x;
  double wv[kPerThread], vv[kPerThread], nv[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int32_t i = i0 + k * stride;
    wv[k] = i < n ? w[i] : 0.0;
    vv[k] = i < n ? vi[i] : 0.0;
    nv[k] = (i < n && vnext) ? vnext[i] : 0.0;
  }
  const double h = reduce_parts(pin, nparts, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) *h_out = h;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int32_t i = i0 + k * stride;
    if (i < n) {
      const double y = wv[k] - h * vv[k];
      w[i] = y;
      acc += y * (vnext ? nv[k] : y);
    }
  }
  for (int32_t i = i0 + kPerThread * stride; i < n; i += stride) {  // grids capped at kMaxParts
    const double y = w[i] - h * vi[i];
    w[i] = y;
    acc += y * (vnext ? vnext[i] : y);
  }
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) pout[blockIdx.x] = s;
}

// h_{j+1,j} = ||w||; rotations 0..j-1 applied to column j of H; rotation j
// from (h_jj, h_{j+1,j}) with t = hypot(a, b), c = a/t, s = b/t (b = 0 gives
// c = 1, s = 0); g_{j+1} = -s g_j, g_j = c g_j; and the next basis vector
// v_{j+1} = w / h_{j+1,j} (an unchanged copy when the norm is zero).
// Every workgroup reduces the norm partials itself (the same fixed order,
// so the same value) and scales its rows; workgroup 0 also updates H, the
// rotations and g.  scal[0] = h_{j+1,j}, scal[1] = |g_{j+1}|.
__global__ void __launch_bounds__(kKT)
k_finalize(double* __restrict__ H, double* __restrict__ g, double* __restrict__ cs, double* __restrict__ sn,
           const double* __restrict__ partials, int nparts, int32_t j, int32_t ldh, double* __restrict__ scal,
           double* __restrict__ hostout, const double* __restrict__ w, double* __restrict__ v, int32_t n) {
  __shared__ double red[kKT / 64];
  __shared__ double s_col[kMaxRestart + 1], s_cs[kMaxRestart], s_sn[kMaxRestart];
  const bool lead = blockIdx.x == 0;
  double* col = H + (int64_t)j * ldh;
  // stage column j and the rotations in LDS (parallel loads that overlap the
  // reduction), so the serial rotation loop below reads no global memory
  if (lead)
    for (int32_t i = threadIdx.x; i <= j; i += blockDim.x) {
      s_col[i] = col[i];
      if (i < j) {
        s_cs[i] = cs[i];
        s_sn[i] = sn[i];
      }
    }
  const double hn = sqrt(reduce_parts(partials, nparts, red));  // synchronises the block
  const int32_t row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row < n) v[row] = hn != 0.0 ? w[row] / hn : w[row];
  if (!lead || threadIdx.x != 0) return;
  for (int32_t i = 0; i < j; ++i) {
    double t = s_cs[i] * s_col[i] + s_sn[i] * s_col[i + 1];
    s_col[i + 1] = -s_sn[i] * s_col[i] + s_cs[i] * s_col[i + 1];
    s_col[i] = t;
  }
  for (int32_t i = 0; i < j; ++i) col[i] = s_col[i];
  double a = s_col[j], b = hn, c, s;
  if (b == 0.0) {
    c = 1.0;
    s = 0.0;
  } else {
    double t = hypot(a, b);
    c = a / t;
    s = b / t;
  }
  cs[j] = c;
  sn[j] = s;
  col[j] = c * a + s * b;
  col[j + 1] = 0.0;
  g[j + 1] = -s * g[j];
  g[j] = c * g[j];
  scal[0] = hn;
  scal[1] = fabs(g[j + 1]);
  if (hostout) {
    // the host reads these after an event recorded behind this kernel
    hostout[0] = hn;
    hostout[1] = fabs(g[j + 1]);
    __threadfence_system();
  }
}

// ---------------------------------------------------------------------------
// Classical Gram-Schmidt applied twice (CGS2): every basis vector's inner
// product in one pass over the rows.  A workgroup's rows of w stay in
// registers (kPerThread per thread, rows beyond that on a grid-stride tail);
// per basis vector the wave partials meet in LDS, and partials[i * nparts +
// workgroup] receives the workgroup's sum in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kDotChunk = 16;  // basis vectors per round: independent loads, then interleaved reductions
constexpr int kCgsRows = 1;    // rows per thread held in registers by the CGS2 kernels (more workgroups in flight)

// Grid of the CGS2 kernels: kCgsRows rows per thread, at most kMaxParts
// workgroups (rows beyond that on a grid-stride tail).
inline int cgs_grid(int32_t n) {
  int g = (int)((n + kKT * kCgsRows - 1) / (kKT * kCgsRows));
  return std::max(1, std::min(g, kMaxParts));
}

// Loads are unconditional (rows clamped to n-1, vectors past the chunk's
// end clamped to its last one; the clamped products are zero or dropped) so
// that the compiler issues a chunk's loads together.
__device__ inline void basis_dots(const double (&wv)[kCgsRows], const double* __restrict__ w,
                                  const double* __restrict__ V, int nvec, int32_t n, double* __restrict__ partials,
                                  int nparts, double (*s_part)[kKT / 64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t stride = gridDim.x * blockDim.x, i0 = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t rc[kCgsRows];
#pragma unroll
  for (int k = 0; k < kCgsRows; ++k) rc[k] = min(i0 + k * stride, n - 1);
  for (int c0 = 0; c0 < nvec; c0 += kDotChunk) {
    const int cn = min(kDotChunk, nvec - c0);
    double acc[kDotChunk];
#pragma unroll
    for (int c = 0; c < kDotChunk; ++c) {
      const double* vi = V + (int64_t)(c0 + min(c, cn - 1)) * n;
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < kCgsRows; ++k) a += wv[k] * vi[rc[k]];
      acc[c] = a;
    }
    for (int32_t r = i0 + kCgsRows * stride; r < n; r += stride) {
      const double y = w[r];
#pragma unroll
      for (int c = 0; c < kDotChunk; ++c) acc[c] += y * V[(int64_t)(c0 + min(c, cn - 1)) * n + r];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
      for (int c = 0; c < kDotChunk; ++c) acc[c] += __shfl_xor(acc[c], off);
    }
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < kDotChunk; ++c)
        if (c < cn) s_part[c][wave] = acc[c];
    }
    __syncthreads();
    if ((int)threadIdx.x < cn) {
      double s = 0.0;
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += s_part[threadIdx.x][q];
      partials[(int64_t)(c0 + threadIdx.x) * nparts + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// w = A z and the partials of <w, V_i>, i < nvec.
__global__ void __launch_bounds__(kKT)
k_spmv_dots(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx, const double* __restrict__ vals,
            const double* __restrict__ z, double* __restrict__ w, const double* __restrict__ V, int nvec, int32_t n,
            double* __restrict__ partials) {
  __shared__ double s_part[kDotChunk][kKT / 64];
  const int32_t stride = gridDim.x * blockDim.x, i0 = blockIdx.x * blockDim.x + threadIdx.x;
  double wv[kCgsRows];
#pragma unroll
  for (int k = 0; k < kCgsRows; ++k) {
    const int32_t r = i0 + k * stride;
    wv[k] = r < n ? row_dot(rowptr, colidx, vals, z, r) : 0.0;
    if (r < n) w[r] = wv[k];
  }
  for (int32_t r = i0 + kCgsRows * stride; r < n; r += stride) w[r] = row_dot(rowptr, colidx, vals, z, r);
  basis_dots(wv, w, V, nvec, n, partials, gridDim.x, s_part);  // tail rows: re-read by their own thread
}

// h_i = sum of the partials of basis vector i, one workgroup per vector
// (fixed-order tree); Hcol = h, or Hcol += h for the second pass.
__global__ void __launch_bounds__(kKT)
k_cgs_coeffs(const double* __restrict__ partials, int nparts, double* __restrict__ h, double* __restrict__ Hcol,
             int add) {
  __shared__ double red[kKT / 64];
  const int i = blockIdx.x;
  const double s = reduce_parts(partials + (int64_t)i * nparts, nparts, red);
  if (threadIdx.x == 0) {
    h[i] = s;
    Hcol[i] = add ? Hcol[i] + s : s;
  }
}

// w -= sum_i h_i V_i (i ascending), then the partials of <w, V_i> (mode 0)
// or of <w, w> (mode 1, into partials[workgroup]).
__global__ void __launch_bounds__(kKT)
k_cgs_update(double* __restrict__ w, const double* __restrict__ V, int nvec, const double* __restrict__ h, int32_t n,
             double* __restrict__ partials, int mode) {
  __shared__ double s_h[kMaxRestart + 1];
  __shared__ double s_part[kDotChunk][kKT / 64];
  __shared__ double red[kKT / 64];
  for (int i = threadIdx.x; i < nvec; i += blockDim.x) s_h[i] = h[i];
  const int32_t stride = gridDim.x * blockDim.x, i0 = blockIdx.x * blockDim.x + threadIdx.x;
  double wv[kCgsRows];
  int32_t rc[kCgsRows];
#pragma unroll
  for (int k = 0; k < kCgsRows; ++k) {
    const int32_t r = i0 + k * stride;
    rc[k] = min(r, n - 1);
    wv[k] = r < n ? w[r] : 0.0;
  }
  __syncthreads();
  for (int i = 0; i < nvec; ++i) {
    const double* vi = V + (int64_t)i * n;
    const double hi = s_h[i];
#pragma unroll
    for (int k = 0; k < kCgsRows; ++k) wv[k] -= hi * vi[rc[k]];
  }
#pragma unroll
  for (int k = 0; k < kCgsRows; ++k) {
    const int32_t r = i0 + k * stride;
    if (r < n) w[r] = wv[k];
    else wv[k] = 0.0;
  }
  for (int32_t r = i0 + kCgsRows * stride; r < n; r += stride) {
    double y = w[r];
    for (int i = 0; i < nvec; ++i) y -= s_h[i] * V[(int64_t)i * n + r];
    w[r] = y;
  }
  if (mode == 0) {
    basis_dots(wv, w, V, nvec, n, partials, gridDim.x, s_part);
  } else {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kCgsRows; ++k) acc += wv[k] * wv[k];
    for (int32_t r = i0 + kCgsRows * stride; r < n; r += stride) acc += w[r] * w[r];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

__global__ void k_norm_finalize(const double* __restrict__ partials, int nparts, double* __restrict__ scal, int idx) {
  __shared__ double red[kKT / 64];
  const double s = reduce_parts(partials, nparts, red);
  if (threadIdx.x == 0) scal[idx] = sqrt(s);
}

// v = w / scal[idx] (unchanged copy when the norm is zero).
__global__ void k_scale_copy(const double* __restrict__ w, double* __restrict__ v, const double* __restrict__ scal,
                             int idx, int32_t n) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = scal[idx];
  v[i] = d != 0.0 ? w[i] / d : w[i];
}

// y = R^{-1} g for the leading j x j triangle of H (one thread).
__global__ void k_backsolve(const double* __restrict__ H, const double* __restrict__ g, int32_t j, int32_t ldh,
                            double* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int32_t i = j - 1; i >= 0; --i) {
    double s = g[i];
    for (int32_t q = i + 1; q < j; ++q) s -= H[(int64_t)q * ldh + i] * y[q];
    y[i] = s / H[(int64_t)i * ldh + i];
  }
}

// x (+)= sum_i y_i Z_i with the sum in ascending i (y == null: all ones).
__global__ void k_combine(const double* __restrict__ Z, int64_t ldz, const double* __restrict__ y, int32_t j,
                          int32_t n, double* __restrict__ x, int add) {
  int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double s = 0.0;
  for (int32_t i = 0; i < j; ++i) s += (y ? y[i] : 1.0) * Z[(int64_t)i * ldz + e];
  x[e] = add ? x[e] + s : s;
}

// ---------------------------------------------------------------------------
// Segmented forms for many independent systems solved in lockstep.  Rows of
// every system are split into chunks of at most kKT * kPerThread rows, one
// workgroup each; a system's scalars are fixed-order sums over its chunks'
// partials.  live[sys] == 0 freezes a system (its chunks do nothing).
// Per-system Krylov state: H (ldh x restart, column-major), then g, cs, sn,
// y (ldh each), stride st = ldh * restart + 4 ldh.
// ---------------------------------------------------------------------------
__device__ inline double seg_sum(const double* __restrict__ parts, const int32_t* __restrict__ coff, int sys,
                                 double* red) {
  double v = 0.0;
  for (int q = coff[sys] + threadIdx.x; q < coff[sys + 1]; q += blockDim.x) v += parts[q];
  return block_sum(v, red);
}

__device__ inline double seg_sum_serial(const double* __restrict__ parts, const int32_t* __restrict__ coff, int sys) {
  double v = 0.0;
  for (int q = coff[sys]; q < coff[sys + 1]; ++q) v += parts[q];
  return v;
}

__global__ void __launch_bounds__(kKT)
k_seg_spmv_dot(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx, const double* __restrict__ vals,
               const double* __restrict__ z, double* __restrict__ w, const double* __restrict__ v0,
               const Chunk* __restrict__ ch, const int32_t* __restrict__ live, double* __restrict__ partials) {
  __shared__ double red[kKT / 64];
  const Chunk c = ch[blockIdx.x];
  if (!live[c.sys]) return;
  double acc = 0.0;
  for (int32_t r = c.start + threadIdx.x; r < c.end; r += blockDim.x) {
    double y = row_dot(rowptr, colidx, vals, z, r);
    w[r] = y;
    acc += y * v0[r];
  }
  double sm = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = sm;
}

__global__ void __launch_bounds__(kKT)
k_seg_residual(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx, const double* __restrict__ vals,
               const double* __restrict__ x, const double* __restrict__ b, double* __restrict__ r,
               const Chunk* __restrict__ ch, const int32_t* __restrict__ live, double* __restrict__ partials) {
  __shared__ double red[kKT / 64];
  const Chunk c = ch[blockIdx.x];
  if (!live[c.sys]) return;
  double acc = 0.0;
  for (int32_t i = c.start + threadIdx.x; i < c.end; i += blockDim.x) {
    double y = b[i] - row_dot(rowptr, colidx, vals, x, i);
    r[i] = y;
    acc += y * y;
  }
  double sm = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = sm;
}

__global__ void __launch_bounds__(kKT)
k_seg_dot(const double* __restrict__ a, const double* __restrict__ b, const Chunk* __restrict__ ch,
          double* __restrict__ partials) {
  __shared__ double red[kKT / 64];
  const Chunk c = ch[blockIdx.x];
  double acc = 0.0;
  for (int32_t i = c.start + threadIdx.x; i < c.end; i += blockDim.x) acc += a[i] * b[i];
  double sm = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = sm;
}

__global__ void __launch_bounds__(kKT)
k_seg_mgs_step(double* __restrict__ w, const double* __restrict__ vi, const double* __restrict__ vnext,
               const Chunk* __restrict__ ch, const int32_t* __restrict__ coff, const int32_t* __restrict__ live,
               const double* __restrict__ pin, double* __restrict__ pout, double* __restrict__ state, int64_t st,
               int64_t hidx) {
  __shared__ double red[kKT / 64];
  const Chunk c = ch[blockIdx.x];
  if (!live[c.sys]) return;
  // vector loads first (they do not depend on h), then the partials
  double wv[kPerThread], vv[kPerThread], nv[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int32_t i = c.start + threadIdx.x + k * blockDim.x;
    wv[k] = i < c.end ? w[i] : 0.0;
    vv[k] = i < c.end ? vi[i] : 0.0;
    nv[k] = (i < c.end && vnext) ? vnext[i] : 0.0;
  }
  const double h = seg_sum(pin, coff, c.sys, red);
  if (blockIdx.x == coff[c.sys] && threadIdx.x == 0) state[c.sys * st + hidx] = h;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int32_t i = c.start + threadIdx.x + k * blockDim.x;
    if (i < c.end) {
      const double y = wv[k] - h * vv[k];
      w[i] = y;
      acc += y * (vnext ? nv[k] : y);
    }
  }
  for (int32_t i = c.start + threadIdx.x + kPerThread * blockDim.x; i < c.end; i += blockDim.x) {
    const double y = w[i] - h * vi[i];
    w[i] = y;
    acc += y * (vnext ? vnext[i] : y);
  }
  double sm = block_sum(acc, red);
  if (threadIdx.x == 0) pout[blockIdx.x] = sm;
}

// one thread per system: norm, rotations, new rotation, g update
__global__ void k_seg_finalize(double* __restrict__ state, int64_t st, const double* __restrict__ partials,
                               const int32_t* __restrict__ coff, const int32_t* __restrict__ live, int nsys,
                               int32_t j, int32_t ldh, int32_t restart, double* __restrict__ scal) {
  const int sys = blockIdx.x * blockDim.x + threadIdx.x;
  if (sys >= nsys || !live[sys]) return;
  double* H = state + sys * st;
  double* g = H + (int64_t)ldh * restart;
  double* cs = g + ldh;
  double* sn = cs + ldh;
  const double hn = sqrt(seg_sum_serial(partials, coff, sys));
  double* col = H + (int64_t)j * ldh;
  for (int32_t i = 0; i < j; ++i) {
    double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  double a = col[j], b = hn, c, sv;
  if (b == 0.0) {
    c = 1.0;
    sv = 0.0;
  } else {
    double t = hypot(a, b);
    c = a / t;
    sv = b / t;
  }
  cs[j] = c;
  sn[j] = sv;
  col[j] = c * a + sv * b;
  col[j + 1] = 0.0;
  g[j + 1] = -sv * g[j];
  g[j] = c * g[j];
  scal[4 * sys + 0] = hn;
  scal[4 * sys + 1] = fabs(g[j + 1]);
}

__global__ void k_seg_norm(const double* __restrict__ partials, const int32_t* __restrict__ coff,
                           const int32_t* __restrict__ live, int nsys, double* __restrict__ scal, int idx) {
  const int sys = blockIdx.x * blockDim.x + threadIdx.x;
  if (sys >= nsys || (live && !live[sys])) return;
  scal[4 * sys + idx] = sqrt(seg_sum_serial(partials, coff, sys));
}

// start of a cycle: g = beta e_1 with beta = scal[4 sys + idx]
__global__ void k_seg_init_g(double* __restrict__ state, int64_t st, const int32_t* __restrict__ live, int nsys,
                             int32_t ldh, int32_t restart, const double* __restrict__ scal, int idx) {
  const int sys = blockIdx.x;
  if (sys >= nsys || !live[sys]) return;
  double* g = state + sys * st + (int64_t)ldh * restart;
  for (int32_t q = threadIdx.x; q < ldh; q += blockDim.x) g[q] = q == 0 ? scal[4 * sys + idx] : 0.0;
}

__global__ void __launch_bounds__(kKT)
k_seg_scale_copy(const double* __restrict__ w, double* __restrict__ v, const double* __restrict__ scal, int idx,
                 const Chunk* __restrict__ ch, const int32_t* __restrict__ live) {
  const Chunk c = ch[blockIdx.x];
  if (!live[c.sys]) return;
  const double d = scal[4 * c.sys + idx];
  for (int32_t i = c.start + threadIdx.x; i < c.end; i += blockDim.x) v[i] = d != 0.0 ? w[i] / d : w[i];
}

__global__ void k_seg_backsolve(double* __restrict__ state, int64_t st, const int32_t* __restrict__ jdone, int nsys,
                                int32_t ldh, int32_t restart) {
  const int sys = blockIdx.x * blockDim.x + threadIdx.x;
  if (sys >= nsys) return;
  const int32_t j = jdone[sys];
  double* H = state + sys * st;
  const double* g = H + (int64_t)ldh * restart;
  double* y = H + (int64_t)ldh * restart + 3 * ldh;
  for (int32_t i = j - 1; i >= 0; --i) {
    double sm = g[i];
    for (int32_t q = i + 1; q < j; ++q) sm -= H[(int64_t)q * ldh + i] * y[q];
    y[i] = sm / H[(int64_t)i * ldh + i];
  }
}

__global__ void __launch_bounds__(kKT)
k_seg_combine(const double* __restrict__ Z, int64_t ldz, const double* __restrict__ state, int64_t st,
              const int32_t* __restrict__ jdone, int32_t ldh, int32_t restart, const Chunk* __restrict__ ch,
              double* __restrict__ x) {
  const Chunk c = ch[blockIdx.x];
  const int32_t j = jdone[c.sys];
  if (j == 0) return;
  const double* y = state + c.sys * st + (int64_t)ldh * restart + 3 * ldh;
  for (int32_t e = c.start + threadIdx.x; e < c.end; e += blockDim.x) {
    double sm = 0.0;
    for (int32_t i = 0; i < j; ++i) sm += y[i] * Z[(int64_t)i * ldz + e];
    x[e] += sm;
  }
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int krylov_grid(int32_t n) {
  int g = (int)((n + kKT * kPerThread - 1) / (kKT * kPerThread));
  return std::max(1, std::min(g, kMaxParts));
}

void launch_spmv(const int32_t* rowptr, const int32_t* colidx, const double* vals, const double* x, double* y,
                 int32_t n, hipStream_t s) {
  if (n > 0) k_spmv<<<nb(n, kKT), kKT, 0, s>>>(rowptr, colidx, vals, x, y, n);
}
void launch_spmv_dot(const int32_t* rowptr, const int32_t* colidx, const double* vals, const double* x, double* w,
                     const double* v0, int32_t n, double* partials, hipStream_t s) {
  k_spmv_dot<<<krylov_grid(n), kKT, 0, s>>>(rowptr, colidx, vals, x, w, v0, n, partials);
}
void launch_residual(const int32_t* rowptr, const int32_t* colidx, const double* vals, const double* x,
                     const double* b, double* r, int32_t n, double* partials, hipStream_t s) {
  k_residual<<<krylov_grid(n), kKT, 0, s>>>(rowptr, colidx, vals, x, b, r, n, partials);
}
void launch_dot_partials(const double* a, const double* b, int32_t n, double* partials, hipStream_t s) {
  k_dot_partials<<<krylov_grid(n), kKT, 0, s>>>(a, b, n, partials);
}
void launch_mgs_step(double* w, const double* vi, const double* vnext, int32_t n, const double* pin, double* pout,
                     double* h_out, int nparts, hipStream_t s) {
  k_mgs_step<<<krylov_grid(n), kKT, 0, s>>>(w, vi, vnext, n, pin, pout, h_out, nparts);
}
void launch_finalize(double* H, double* g, double* cs, double* sn, const double* partials, int nparts, int32_t j,
                     int32_t ldh, double* scal, double* hostout, const double* w, double* v, int32_t n,
                     hipStream_t s) {
  k_finalize<<<std::max(1u, nb(n, kKT)), kKT, 0, s>>>(H, g, cs, sn, partials, nparts, j, ldh, scal, hostout, w, v, n);
}
int cgs_parts(int32_t n) { return cgs_grid(n); }
void launch_spmv_dots(const int32_t* rowptr, const int32_t* colidx, const double* vals, const double* z, double* w,
                      const double* V, int nvec, int32_t n, double* partials, hipStream_t s) {
  k_spmv_dots<<<cgs_grid(n), kKT, 0, s>>>(rowptr, colidx, vals, z, w, V, nvec, n, partials);
}
void launch_cgs_coeffs(const double* partials, int nparts, int nvec, double* h, double* Hcol, int add, hipStream_t s) {
  if (nvec > 0) k_cgs_coeffs<<<nvec, kKT, 0, s>>>(partials, nparts, h, Hcol, add);
}
void launch_cgs_update(double* w, const double* V, int nvec, const double* h, int32_t n, double* partials, int mode,
                       hipStream_t s) {
  k_cgs_update<<<cgs_grid(n), kKT, 0, s>>>(w, V, nvec, h, n, partials, mode);
}
void launch_norm_finalize(const double* partials, int nparts, double* scal, int idx, hipStream_t s) {
  k_norm_finalize<<<1, kKT, 0, s>>>(partials, nparts, scal, idx);
}
void launch_scale_copy(const double* w, double* v, const double* scal, int idx, int32_t n, hipStream_t s) {
  if (n > 0) k_scale_copy<<<nb(n, 256), 256, 0, s>>>(w, v, scal, idx, n);
}
void launch_backsolve(const double* H, const double* g, int32_t j, int32_t ldh, double* y, hipStream_t s) {
  k_backsolve<<<1, 64, 0, s>>>(H, g, j, ldh, y);
}
void launch_combine(const double* Z, int64_t ldz, const double* y, int32_t j, int32_t n, double* x, int add,
                    hipStream_t s) {
  if (n > 0) k_combine<<<nb(n, 256), 256, 0, s>>>(Z, ldz, y, j, n, x, add);
}

}  // namespace addns

namespace addns {
int seg_chunk_rows() { return kKT * kPerThread; }
void launch_seg_spmv_dot(const int32_t* rp, const int32_t* ci, const double* cv, const double* z, double* w,
                         const double* v0, const Chunk* ch, int nch, const int32_t* live, double* parts, hipStream_t s) {
  k_seg_spmv_dot<<<nch, kKT, 0, s>>>(rp, ci, cv, z, w, v0, ch, live, parts);
}
void launch_seg_residual(const int32_t* rp, const int32_t* ci, const double* cv, const double* x, const double* b,
                         double* r, const Chunk* ch, int nch, const int32_t* live, double* parts, hipStream_t s) {
  k_seg_residual<<<nch, kKT, 0, s>>>(rp, ci, cv, x, b, r, ch, live, parts);
}
void launch_seg_dot(const double* a, const double* b, const Chunk* ch, int nch, double* parts, hipStream_t s) {
  k_seg_dot<<<nch, kKT, 0, s>>>(a, b, ch, parts);
}
void launch_seg_mgs_step(double* w, const double* vi, const double* vnext, const Chunk* ch, int nch,
                         const int32_t* coff, const int32_t* live, const double* pin, double* pout, double* state,
                         int64_t st, int64_t hidx, hipStream_t s) {
  k_seg_mgs_step<<<nch, kKT, 0, s>>>(w, vi, vnext, ch, coff, live, pin, pout, state, st, hidx);
}
void launch_seg_finalize(double* state, int64_t st, const double* parts, const int32_t* coff, const int32_t* live,
                         int nsys, int32_t j, int32_t ldh, int32_t restart, double* scal, hipStream_t s) {
  k_seg_finalize<<<(nsys + 63) / 64, 64, 0, s>>>(state, st, parts, coff, live, nsys, j, ldh, restart, scal);
}
void launch_seg_norm(const double* parts, const int32_t* coff, const int32_t* live, int nsys, double* scal, int idx,
                     hipStream_t s) {
  k_seg_norm<<<(nsys + 63) / 64, 64, 0, s>>>(parts, coff, live, nsys, scal, idx);
}
void launch_seg_init_g(double* state, int64_t st, const int32_t* live, int nsys, int32_t ldh, int32_t restart,
                       const double* scal, int idx, hipStream_t s) {
  k_seg_init_g<<<nsys, 64, 0, s>>>(state, st, live, nsys, ldh, restart, scal, idx);
}
void launch_seg_scale_copy(const double* w, double* v, const double* scal, int idx, const Chunk* ch, int nch,
                           const int32_t* live, hipStream_t s) {
  k_seg_scale_copy<<<nch, kKT, 0, s>>>(w, v, scal, idx, ch, live);
}
void launch_seg_backsolve(double* state, int64_t st, const int32_t* jdone, int nsys, int32_t ldh, int32_t restart,
                          hipStream_t s) {
  k_seg_backsolve<<<(nsys + 63) / 64, 64, 0, s>>>(state, st, jdone, nsys, ldh, restart);
}
void launch_seg_combine(const double* Z, int64_t ldz, const double* state, int64_t st, const int32_t* jdone,
                        int32_t ldh, int32_t restart, const Chunk* ch, int nch, double* x, hipStream_t s) {
  k_seg_combine<<<nch, kKT, 0, s>>>(Z, ldz, state, st, jdone, ldh, restart, ch, x);
}
}  // namespace addns
