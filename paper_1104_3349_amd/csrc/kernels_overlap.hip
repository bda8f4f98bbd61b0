// Interface solve with overlapped aggregates (the overlap Remark of
// section 3.1; Algorithm 1's overlapped branch).  Shat is block lower
// bidiagonal: its diagonal blocks A_i are applied by the blockwise
// interface kernel (u_i = A_i^{-1} t_i), and the forward substitution
// x_i = u_i - M_i x_{i-1}, M_i = A_i^{-1} [L_{i-1}; 0], runs here.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "precond.h"

namespace addns {
namespace {

// Sum over aligned groups of 4 lanes with two DPP quad permutations; every
// lane of a quad ends with the same fixed-order sum.
template <int CTRL>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <class A>
__device__ inline A quad_sum(A p) {
  p += dpp_mov<0xB1>(p);  // quad_perm [1,0,3,2]
  p += dpp_mov<0x4E>(p);  // quad_perm [2,3,0,1]
  return p;
}

// Overlapped aggregates: Shat is block lower bidiagonal, so after the
// blockwise u_i = A_i^{-1} t_i (k_interface_solve, in place in x2) the
// forward substitution x_i = u_i - M_i x_{i-1} remains.  It runs in
// segments of L aggregates (segment g: aggregates g L .. g L + L - 1):
//   (1) every segment sweeps its own chain from a zero start, z_i = u_i -
//       M_i z_{i-1} past its first aggregate (z = u there), side by side;
//   (2) one workgroup chains the segment ends: x_b = z_b - Q_b x_{b'} (b' the
//       previous segment's last aggregate), with the response
//       Q_i = M_i for a segment's first aggregate, Q_i = -M_i Q_{i-1} after it;
//   (3) every other aggregate of segments 1.. takes x_i = z_i - Q_i x_{b'}.
// With one segment, (1) is the whole chain and (2), (3) do not run.
//
// The chain kernel runs one sequence of aggregates per workgroup: the
// aggregates of segment blockIdx.x (ends = 0) or the segment ends (ends =
// 1), with the matrices Mall (M_i, or Q_i for the ends).  One workgroup of
// 4 ROWS threads; aggregates hold at most ROWS nodes; the matrix rows are
// stored 4 CQ wide (zero past the previous aggregate's size).  Row r belongs
// to the quad of lanes 4r..4r+3, each holding CQ consecutive columns, whose
// partial sums meet in quad_sum; products are formed in T (FP32 with FP32
// chain matrices, so x_{i-1} is read rounded to FP32) and x_i is formed in
// FP64.  The matrices and u_i do not depend on the chain: they arrive in two
// register rings of P steps each, one filled while the other is consumed, so
// every load has P steps to land.  x_{i-1} and x_i alternate between two LDS
// rows (zero at the start, so padded columns multiply finite values); one
// barrier per step.  The sequence's offsets are staged in LDS first
// (dynamic: 16 (L + 1) bytes), so no step waits on a scalar memory load.
__host__ __device__ inline int32_t seg_last(int32_t g, int32_t L, int32_t k) { return ((g + 1) * L < k ? (g + 1) * L : k) - 1; }

template <class T, int ROWS, int CQ, int P>
__global__ void __launch_bounds__(4 * ROWS)
k_overlap_chain(int32_t k, int32_t L, int ends, const int32_t* __restrict__ agg_off_g,
                const int64_t* __restrict__ m_off_g, const T* __restrict__ Mall, double* __restrict__ x2) {
  constexpr int W = 4 * CQ;  // stored row width of the matrices
  __shared__ T xs[2][W];
  extern __shared__ int64_t chain_lds[];
  // the sequence: J aggregates; step j (1 <= j < J) forms aggregate seq(j)
  // from seq(j - 1)
  const int32_t nseg = (k + L - 1) / L;
  const int32_t first = blockIdx.x * L;
  const int32_t J = ends ? nseg : min(L, k - first);
  auto seq = [&](int32_t j) { return ends ? seg_last(j, L, k) : first + j; };
  int64_t* m_off = chain_lds;                                    // J entries
  int32_t* a0s = reinterpret_cast<int32_t*>(chain_lds + J);      // J entries
  int32_t* szs = a0s + J;                                        // J entries
  const int tid = threadIdx.x, r = tid >> 2, c0 = (tid & 3) * CQ;
  for (int q = tid; q < 2 * W; q += blockDim.x) xs[q / W][q % W] = T(0);
  for (int32_t q = tid; q < J; q += blockDim.x) {
    const int32_t g = seq(q);
    m_off[q] = m_off_g[g];
    a0s[q] = agg_off_g[g];
    szs[q] = agg_off_g[g + 1] - agg_off_g[g];
  }
  __syncthreads();
  for (int32_t q = tid; q < szs[0]; q += blockDim.x) xs[0][q] = (T)x2[a0s[0] + q];
  if (J < 2) return;
  T m[2][P][CQ];
  double u[2][P];
  // Every lane loads and stores unconditionally (so that the compiler can
  // count the loads in flight exactly): steps past the end repeat step J-1,
  // and rows past the aggregate's size repeat its last row (computing and
  // storing the same value as that row's own lanes).
  auto load = [&](int32_t j, int b, int jj) {
    j = min(j, J - 1);
    const int32_t a0 = a0s[j], re = min(r, szs[j] - 1);
    const T* M = Mall + m_off[j] + (int64_t)re * W + c0;
#pragma unroll
    for (int q = 0; q < CQ; ++q) m[b][jj][q] = M[q];
    u[b][jj] = x2[a0 + re];
  };
  // one step of the chain from ring slot (b, jj); false past the last step
  auto step = [&](int32_t j, int b, int jj) -> bool {
    if (j >= J) return false;
    const int32_t a0 = a0s[j], re = min(r, szs[j] - 1);
    const T* xp = xs[(j - 1) & 1] + c0;
    T p = T(0);
#pragma unroll
    for (int q = 0; q < CQ; ++q) p += m[b][jj][q] * xp[q];
    p = quad_sum(p);
    const double v = u[b][jj] - (double)p;
    xs[j & 1][re] = (T)v;
    x2[a0 + re] = v;
    __syncthreads();
    return true;
  };
#pragma unroll
  for (int jj = 0; jj < P; ++jj) load(1 + jj, 0, jj);
  __syncthreads();
  for (int32_t g0 = 1; g0 < J; g0 += 2 * P) {
#pragma unroll
    for (int jj = 0; jj < P; ++jj) load(g0 + P + jj, 1, jj);
#pragma unroll
    for (int jj = 0; jj < P; ++jj)
      if (!step(g0 + jj, 0, jj)) return;
#pragma unroll
    for (int jj = 0; jj < P; ++jj) load(g0 + 2 * P + jj, 0, jj);
#pragma unroll
    for (int jj = 0; jj < P; ++jj)
      if (!step(g0 + P + jj, 1, jj)) return;
  }
}

// Step (3): one workgroup per aggregate i of segments 1.. other than the
// segment's last: x_i = z_i - Q_i x_{b'}, with x_{b'} (the previous
// segment's last aggregate, final after step 2) staged in LDS.  The same
// quad layout and the same product type as the chain.
template <class T, int ROWS, int CQ>
__global__ void __launch_bounds__(4 * ROWS)
k_overlap_fix(int32_t k, int32_t L, const int32_t* __restrict__ agg_off, const int64_t* __restrict__ q_off,
              const T* __restrict__ Qall, double* __restrict__ x2) {
  constexpr int W = 4 * CQ;
  __shared__ T xs[W];
  const int32_t i = blockIdx.x, g = i / L;
  if (g == 0 || i == seg_last(g, L, k)) return;
  const int32_t bp = g * L - 1;  // previous segment's last aggregate
  const int32_t pa = agg_off[bp], ps = agg_off[bp + 1] - pa;
  const int tid = threadIdx.x, r = tid >> 2, c0 = (tid & 3) * CQ;
  for (int q = tid; q < W; q += blockDim.x) xs[q] = q < ps ? (T)x2[pa + q] : T(0);
  __syncthreads();
  const int32_t a0 = agg_off[i], s = agg_off[i + 1] - a0;
  if (r >= s) return;
  const T* Q = Qall + q_off[i] + (int64_t)r * W + c0;
  T p = T(0);
#pragma unroll
  for (int q = 0; q < CQ; ++q) p += Q[q] * xs[c0 + q];
  p = quad_sum(p);
  if ((tid & 3) == 0) x2[a0 + r] = x2[a0 + r] - (double)p;
}

// Setup of the responses: one workgroup per segment g >= 1, its aggregates
// in order: Q_i = M_i at the segment's first aggregate, then
// Q_i = -M_i Q_{i-1} (rows of M_i: 4 CQ wide, its columns are the previous
// aggregate's nodes; Q_{i-1} rows the previous aggregate's nodes), in FP64
// from the stored matrices, stored like them.
template <class T>
__global__ void k_overlap_q(int32_t k, int32_t L, int32_t W, const int32_t* __restrict__ agg_off,
                            const int64_t* __restrict__ m_off, const T* __restrict__ Mall, T* __restrict__ Qall) {
  const int32_t g = blockIdx.x + 1, a = g * L, b = seg_last(g, L, k);
  for (int32_t i = a; i <= b; ++i) {
    const int32_t s = agg_off[i + 1] - agg_off[i], sp = agg_off[i] - agg_off[i - 1];
    const T* M = Mall + m_off[i];
    T* Q = Qall + m_off[i];
    const T* Qp = Qall + m_off[i - 1];
    for (int32_t t = threadIdx.x; t < s * W; t += blockDim.x) {
      if (i == a) {
        Q[t] = M[t];
      } else {
        const int32_t rr = t / W, c = t % W;
        double acc = 0.0;
        for (int32_t q = 0; q < sp; ++q) acc += (double)M[(int64_t)rr * W + q] * (double)Qp[(int64_t)q * W + c];
        Q[t] = (T)(-acc);
      }
    }
    __syncthreads();
  }
}

}  // namespace

template <class T, int ROWS, int CQ, int P>
void run_overlap_chain(int32_t k, int32_t L, const int32_t* ao, const int64_t* mo, const T* M, const T* Q,
                       double* x2, hipStream_t s) {
  const int32_t nseg = (k + L - 1) / L;
  const size_t smem = 16 * (size_t)std::max(L, nseg);
  static size_t raised = 64 * 1024;
  if (smem > raised) {
    ADDNS_HIP(hipFuncSetAttribute((const void*)k_overlap_chain<T, ROWS, CQ, P>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    raised = smem;
  }
  k_overlap_chain<T, ROWS, CQ, P><<<nseg, 4 * ROWS, smem, s>>>(k, L, 0, ao, mo, M, x2);
  if (nseg > 1) {
    k_overlap_chain<T, ROWS, CQ, P><<<1, 4 * ROWS, smem, s>>>(k, L, 1, ao, mo, Q, x2);
    k_overlap_fix<T, ROWS, CQ><<<k, 4 * ROWS, 0, s>>>(k, L, ao, mo, Q, x2);
  }
}

// Segment length of the chain: the requested one, else the L that balances
// the segment sweeps (L steps) against the chain of segment ends (k / L).
int32_t overlap_segment_length(int32_t k, int32_t requested) {
  if (requested > 0) return std::min(requested, std::max(k, 1));
  int32_t L = 1;
  while ((int64_t)L * L < k) ++L;
  return L;
}

void launch_overlap_q(const addns_precond* pc, hipStream_t s) {
  const Plan& pl = pc->plan;
  const int32_t k = pl.k, L = pc->ovl_seg;
  const int32_t nseg = (k + L - 1) / L;
  if (!pc->overlap_chain || nseg < 2) return;
  const int32_t* ao = pc->agg_off.as<int32_t>();
  const int64_t* mo = pc->ovl_moff.as<int64_t>();
  if (pc->schur_prec == P64)
    k_overlap_q<double><<<nseg - 1, 256, 0, s>>>(k, L, pc->overlap_chain, ao, mo, pc->ovl_m.as<double>(),
                                                 pc->ovl_q.as<double>());
  else
    k_overlap_q<float><<<nseg - 1, 256, 0, s>>>(k, L, pc->overlap_chain, ao, mo, pc->ovl_m.as<float>(),
                                                pc->ovl_q.as<float>());
}

void launch_overlap_chain(const addns_precond* pc, double* x2, hipStream_t s) {
  const Plan& pl = pc->plan;
  if (!pc->overlap_chain || pl.k < 2) return;
  const int32_t* ao = pc->agg_off.as<int32_t>();
  const int64_t* mo = pc->ovl_moff.as<int64_t>();
  const int32_t L = pc->ovl_seg;
  const bool dbl = pc->schur_prec == P64;
  const double* Md = pc->ovl_m.as<double>();
  const float* Mf = pc->ovl_m.as<float>();
  const double* Qd = pc->ovl_q.as<double>();
  const float* Qf = pc->ovl_q.as<float>();
  switch (pc->overlap_chain) {
    case 64:
      if (dbl) run_overlap_chain<double, 64, 16, 2>(pl.k, L, ao, mo, Md, Qd, x2, s);
      else run_overlap_chain<float, 64, 16, 4>(pl.k, L, ao, mo, Mf, Qf, x2, s);
      break;
    case 80:
      if (dbl) run_overlap_chain<double, 80, 20, 2>(pl.k, L, ao, mo, Md, Qd, x2, s);
      else run_overlap_chain<float, 80, 20, 4>(pl.k, L, ao, mo, Mf, Qf, x2, s);
      break;
    default:
      if (dbl) run_overlap_chain<double, 128, 32, 1>(pl.k, L, ao, mo, Md, Qd, x2, s);
      else run_overlap_chain<float, 128, 32, 2>(pl.k, L, ao, mo, Mf, Qf, x2, s);
  }
}

}  // namespace addns
