// Apply kernels: Algorithm 2, x = B^{-1} y in the permuted numbering.
//
//   interior solve   z1 = D^{-1} y1           (one workgroup per subdomain)
//   interface solve  x2 = Shat^{-1}(y2 - F z1) (one workgroup per aggregate)
//   interior solve   x1 = z1 - D^{-1} (E x2)   (E x2 formed while loading)
//
// Each interior solve is a forward sweep over the lower blocks followed by a
// backward sweep over the upper blocks.  Every block step is a gather plus
// one or two dense GEMVs whose matrices are streamed from HBM column-major:
// a wavefront reads 64 consecutive rows of one column per load (coalesced),
// the vector operand sits in LDS and is read as a broadcast, and column
// chunks are reduced through LDS in a fixed order.  Factors are stored in
// FP64 or FP32; accumulation is always FP64.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "precond.h"

namespace addns {
namespace {

constexpr int kSweepThreads = 1024;
constexpr int kWaves = kSweepThreads / 64;

template <class T>
__device__ inline double ld(const T* p) { return (double)(*p); }
template <>
__device__ inline double ld<__half>(const __half* p) { return (double)__half2float(*p); }

// y[r] = sum_k M(r,k) v[k] for r < R, k restricted per row to
// [lo(r), hi(r)), M column-major with leading dimension R.
// kind 0: full; 1: lower (k <= r); 2: upper (k >= r); 3: k <= r + shift.
// Result into out[0..R) (LDS).  part: LDS scratch of kWaves * R doubles.
template <class T>
__device__ void block_gemv(const T* __restrict__ M, int R, int K, const double* v, double* out, double* part,
                           int kind, int shift) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int RT = (R + 63) >> 6;
  const int CS = max(1, kWaves / RT);
  if (wave < RT * CS) {
    const int tile = wave % RT, cs = wave / RT;
    const int r = tile * 64 + lane;
    int kb = (int)((int64_t)K * cs / CS), ke = (int)((int64_t)K * (cs + 1) / CS);
    const int rmin = tile * 64, rmax = min(R, rmin + 64) - 1;
    if (kind == 1) ke = min(ke, rmax + 1);
    else if (kind == 2) kb = max(kb, rmin);
    else if (kind == 3) ke = min(ke, rmax + shift + 1);
    int lo = 0, hi = K;
    if (kind == 1) hi = r + 1;
    else if (kind == 2) lo = r;
    else if (kind == 3) hi = r + shift + 1;
    double acc = 0.0;
    if (r < R) {
      const T* col = M + (int64_t)kb * R + r;
      int k = kb;
#pragma unroll 4
      for (; k < ke; ++k, col += R) {
        if (k >= lo && k < hi) acc += ld(col) * v[k];
      }
    }
    if (r < R) part[cs * R + r] = acc;
  }
  __syncthreads();
  for (int r = tid; r < R; r += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < CS; ++c) s += part[c * R + r];
    out[r] = s;
  }
  __syncthreads();
}

struct SweepArgs {
  int32_t KL, nbL, nbU, KV;
  const int32_t* sub_n;
  const int32_t* sub_npad;
  const int32_t* sub_int_off;
  const int32_t* sub_vec_off;
  const int32_t* sub_lblk0;
  const int32_t* sub_ublk0;
  const int32_t* lperm;
  const void* l11inv;
  const void* l21;
  const void* uinv;
  const void* u12;
  const int32_t* e_rowptr;
  const int32_t* e_colidx;
  const double* e_vals;
  double* ypad;      // padded intermediate (after the lower sweep)
};

// One workgroup per subdomain.  second == 0: out[int] = D^{-1} yin[int].
// second == 1: input u = E x2 (x2 = separator part, CSR E), and
// out[int] = z1[int] - D^{-1} u.
template <class T>
__global__ void __launch_bounds__(kSweepThreads)
k_interior_solve(SweepArgs a, const double* __restrict__ yin, double* __restrict__ out, int second,
                 const double* __restrict__ x2, const double* __restrict__ z1) {
  extern __shared__ double smem[];
  const int sub = blockIdx.x;
  const int32_t n = a.sub_n[sub], npad = a.sub_npad[sub];
  if (n == 0) return;
  const int32_t ioff = a.sub_int_off[sub], voff = a.sub_vec_off[sub];
  const int32_t KL = a.KL, nbL = a.nbL, nbU = a.nbU, W = nbL + KL;
  const int tid = threadIdx.x;
  double* w = smem;                 // W
  double* v = w + W;                // W
  double* xb = v + W;               // max(nbL, nbU)
  double* t = xb + nbU;             // nbU
  double* part = t + nbU;           // kWaves * max(W, nbU)
  double* ypad = a.ypad + voff;
  auto input = [&](int32_t r) -> double {
    if (r >= n) return 0.0;
    if (!second) return yin[ioff + r];
    double s = 0.0;
    for (int32_t e = a.e_rowptr[ioff + r]; e < a.e_rowptr[ioff + r + 1]; ++e) s += a.e_vals[e] * x2[a.e_colidx[e]];
    return s;
  };
  // ---- forward sweep over lower blocks: window = [carry (KL); next nbL rows]
  for (int32_t r = tid; r < KL; r += blockDim.x) w[r] = input(r);
  const int32_t nL = npad / nbL;
  const int32_t lb0 = a.sub_lblk0[sub];
  for (int32_t b = 0; b < nL; ++b) {
    const int64_t blk = lb0 + b;
    for (int32_t r = tid; r < nbL; r += blockDim.x) w[KL + r] = input(b * nbL + KL + r);
    __syncthreads();
    const int32_t* idx = a.lperm + blk * W;
    for (int32_t r = tid; r < W; r += blockDim.x) v[r] = w[idx[r]];
    __syncthreads();
    block_gemv<T>((const T*)a.l11inv + blk * nbL * nbL, nbL, nbL, v, xb, part, 1, 0);
    for (int32_t r = tid; r < nbL; r += blockDim.x) ypad[b * nbL + r] = xb[r];
    block_gemv<T>((const T*)a.l21 + blk * KL * nbL, KL, nbL, xb, t, part, 0, 0);
    for (int32_t r = tid; r < KL; r += blockDim.x) w[r] = v[nbL + r] - t[r];
    __syncthreads();
  }
  // ---- backward sweep over upper blocks
  const int32_t nU = npad / nbU;
  const int32_t ub0 = a.sub_ublk0[sub];
  for (int32_t b = nU - 1; b >= 0; --b) {
    const int64_t blk = ub0 + b;
    if (b < nU - 1) {
      block_gemv<T>((const T*)a.u12 + blk * nbU * nbU, nbU, nbU, xb, t, part, 3, a.KV - nbU);
      for (int32_t r = tid; r < nbU; r += blockDim.x) t[r] = ypad[b * nbU + r] - t[r];
    } else {
      for (int32_t r = tid; r < nbU; r += blockDim.x) t[r] = ypad[b * nbU + r];
    }
    __syncthreads();
    block_gemv<T>((const T*)a.uinv + blk * nbU * nbU, nbU, nbU, t, xb, part, 2, 0);
    for (int32_t r = tid; r < nbU; r += blockDim.x) {
      int32_t row = b * nbU + r;
      if (row < n) {
        if (second) out[ioff + row] = z1[ioff + row] - xb[r];
        else out[ioff + row] = xb[r];
      }
    }
    __syncthreads();
  }
}

// One workgroup per aggregate: t = y2 - F z1 on the aggregate's rows, then
// x2 = S_i^{-1} t with S_i^{-1} column-major.
template <class T>
__global__ void __launch_bounds__(256)
k_interface_solve(int32_t n_int, const int32_t* __restrict__ agg_off, const int32_t* __restrict__ f_rowptr,
                  const int32_t* __restrict__ f_colidx, const double* __restrict__ f_vals,
                  const int64_t* __restrict__ sinv_off, const T* __restrict__ sinv, const float* __restrict__ scale,
                  int scaled, const double* __restrict__ y, const double* __restrict__ z1, double* __restrict__ out) {
  __shared__ double t[1024];
  __shared__ double part[4 * 256];
  const int i = blockIdx.x;
  const int32_t a0 = agg_off[i], s = agg_off[i + 1] - a0;
  const int tid = threadIdx.x;
  for (int32_t r = tid; r < s; r += blockDim.x) {
    int32_t row = a0 + r;
    double acc = y[n_int + row];
    for (int32_t e = f_rowptr[row]; e < f_rowptr[row + 1]; ++e) acc -= f_vals[e] * z1[f_colidx[e]];
    t[r] = acc;
  }
  __syncthreads();
  const T* M = sinv + sinv_off[i];
  // rows r = tid % Rp, column chunk tid / Rp
  const int Rp = s <= 64 ? 64 : (s <= 128 ? 128 : 256);
  const int CS = 256 / Rp;
  const int r = tid % Rp, cs = tid / Rp;
  for (int32_t rb = 0; rb < s; rb += Rp) {
    const int32_t row = rb + r;
    double acc = 0.0;
    if (row < s) {
      int32_t kb = (int32_t)((int64_t)s * cs / CS), ke = (int32_t)((int64_t)s * (cs + 1) / CS);
      for (int32_t k = kb; k < ke; ++k) acc += ld(M + (int64_t)k * s + row) * t[k];
    }
    part[cs * 256 + r] = acc;
    __syncthreads();
    if (cs == 0 && row < s) {
      double acc2 = 0.0;
      for (int c = 0; c < CS; ++c) acc2 += part[c * 256 + r];
      if (scaled) acc2 *= (double)scale[i];
      out[n_int + a0 + row] = acc2;
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

size_t sweep_smem_bytes(int32_t KL, int32_t nbL, int32_t nbU) {
  int32_t W = nbL + KL;
  return sizeof(double) * (size_t)(2 * W + 2 * nbU + kWaves * std::max(W, nbU));
}

void launch_interior_solve(const addns_precond* pc, const double* yin, double* out, int second, const double* x2,
                           const double* z1, hipStream_t s) {
  const Plan& pl = pc->plan;
  if (pl.m == 0 || pl.n_int == 0) return;
  SweepArgs a;
  a.KL = pl.KL;
  a.nbL = pl.nbL;
  a.nbU = pl.nbU;
  a.KV = pl.KL + pl.KU;
  a.sub_n = pc->sub_n.as<int32_t>();
  a.sub_npad = pc->sub_npad.as<int32_t>();
  a.sub_int_off = pc->sub_int_off.as<int32_t>();
  a.sub_vec_off = pc->sub_vec_off.as<int32_t>();
  a.sub_lblk0 = pc->sub_lblk0.as<int32_t>();
  a.sub_ublk0 = pc->sub_ublk0.as<int32_t>();
  a.lperm = pc->lperm.as<int32_t>();
  a.l11inv = pc->l11inv.p;
  a.l21 = pc->l21.p;
  a.uinv = pc->uinv.p;
  a.u12 = pc->u12.p;
  a.e_rowptr = pc->e_rowptr.as<int32_t>();
  a.e_colidx = pc->e_colidx.as<int32_t>();
  a.e_vals = pc->e_vals.as<double>();
  a.ypad = second ? pc->zpad.as<double>() : pc->ypad.as<double>();
  size_t smem = sweep_smem_bytes(pl.KL, pl.nbL, pl.nbU);
  if (smem > 160 * 1024) throw ArgError("interior bandwidth too large for the LDS-staged sweep");
  if (smem > 64 * 1024) {
    if (pc->interior_prec == P64)
      ADDNS_HIP(hipFuncSetAttribute((const void*)k_interior_solve<double>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    else
      ADDNS_HIP(hipFuncSetAttribute((const void*)k_interior_solve<float>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  }
  if (pc->interior_prec == P64)
    k_interior_solve<double><<<pl.m, kSweepThreads, smem, s>>>(a, yin, out, second, x2, z1);
  else
    k_interior_solve<float><<<pl.m, kSweepThreads, smem, s>>>(a, yin, out, second, x2, z1);
}

void launch_interface_solve(const addns_precond* pc, const double* y, const double* z1, double* out, hipStream_t s) {
  const Plan& pl = pc->plan;
  if (pl.k == 0) return;
  const int32_t* ao = pc->agg_off.as<int32_t>();
  const int32_t* fr = pc->f_rowptr.as<int32_t>();
  const int32_t* fc = pc->f_colidx.as<int32_t>();
  const double* fv = pc->f_vals.as<double>();
  const int64_t* so = pc->sinv_off.as<int64_t>();
  if (pc->schur_prec == P64)
    k_interface_solve<double><<<pl.k, 256, 0, s>>>(pl.n_int, ao, fr, fc, fv, so, pc->sinv.as<double>(), nullptr, 0, y,
                                                   z1, out);
  else if (pc->schur_prec == P32)
    k_interface_solve<float><<<pl.k, 256, 0, s>>>(pl.n_int, ao, fr, fc, fv, so, pc->sinv.as<float>(), nullptr, 0, y,
                                                  z1, out);
  else
    k_interface_solve<__half><<<pl.k, 256, 0, s>>>(pl.n_int, ao, fr, fc, fv, so, pc->sinv.as<__half>(),
                                                   pc->sinv_scale.as<float>(), 1, y, z1, out);
}

void launch_permute(const int32_t* perm, const double* in, double* out, int32_t n, int inverse, const double* scale,
                    hipStream_t s) {
  if (n > 0) k_permute<<<(n + 255) / 256, 256, 0, s>>>(perm, in, out, n, inverse, scale);
}

}  // namespace addns
