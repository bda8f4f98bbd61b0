// Interface solve with overlapped aggregates (the overlap Remark of
// section 3.1; Algorithm 1's overlapped branch).  Shat is block lower
// bidiagonal: its diagonal blocks A_i are applied by the blockwise
// interface kernel (u_i = A_i^{-1} t_i), and the forward substitution
// x_i = u_i - M_i x_{i-1}, M_i = A_i^{-1} [L_{i-1}; 0], runs here.
#include <hip/hip_runtime.h>

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
// blockwise u_i = A_i^{-1} t_i (k_interface_solve, in place in x2) one
// workgroup of 4 ROWS threads runs the forward substitution
// x_i = u_i - M_i x_{i-1} over i = 1..k-1.  Aggregates hold at most ROWS
// nodes; M_i rows are stored 4 CQ wide (zero past s_{i-1}).  Row r belongs
// to the quad of lanes 4r..4r+3, each holding CQ consecutive columns, whose
// partial sums meet in quad_sum; products are formed in T (FP32 with FP32
// chain matrices, so x_{i-1} is read rounded to FP32) and x_i is formed in
// FP64.  M_i and u_i do not depend on the chain: they arrive in two register
// rings of P steps each, one filled while the other is consumed, so every
// load has P steps to land.  x_{i-1} and x_i alternate between two LDS rows
// (zero at the start, so padded columns multiply finite values); one
// barrier per step.  Aggregate and M_i offsets are staged in LDS first
// (dynamic: 8k + 4(k+1) bytes), so no step waits on a scalar memory load.
template <class T, int ROWS, int CQ, int P>
__global__ void __launch_bounds__(4 * ROWS)
k_overlap_chain(int32_t k, const int32_t* __restrict__ agg_off_g, const int64_t* __restrict__ m_off_g,
                const T* __restrict__ Mall, double* __restrict__ x2) {
  constexpr int W = 4 * CQ;  // stored row width of M_i
  __shared__ T xs[2][W];
  extern __shared__ int64_t chain_lds[];
  int64_t* m_off = chain_lds;                                    // k entries
  int32_t* agg_off = reinterpret_cast<int32_t*>(chain_lds + k);  // k + 1 entries
  const int tid = threadIdx.x, r = tid >> 2, c0 = (tid & 3) * CQ;
  for (int q = tid; q < 2 * W; q += blockDim.x) xs[q / W][q % W] = T(0);
  for (int32_t q = tid; q < k; q += blockDim.x) m_off[q] = m_off_g[q];
  for (int32_t q = tid; q <= k; q += blockDim.x) agg_off[q] = agg_off_g[q];
  __syncthreads();
  {
    const int32_t s0 = agg_off[1] - agg_off[0];
    for (int32_t q = tid; q < s0; q += blockDim.x) xs[0][q] = (T)x2[agg_off[0] + q];
  }
  T m[2][P][CQ];
  double u[2][P];
  // Every lane loads and stores unconditionally (so that the compiler can
  // count the loads in flight exactly): steps past the end repeat step k-1,
  // and rows past s_i repeat row s_i - 1 (computing and storing the same
  // value as that row's own lanes).
  auto load = [&](int32_t i, int b, int j) {
    i = min(i, k - 1);
    const int32_t a0 = agg_off[i], re = min(r, agg_off[i + 1] - a0 - 1);
    const T* M = Mall + m_off[i] + (int64_t)re * W + c0;
#pragma unroll
    for (int q = 0; q < CQ; ++q) m[b][j][q] = M[q];
    u[b][j] = x2[a0 + re];
  };
  // one step of the chain from ring slot (b, j); false past the last step
  auto step = [&](int32_t i, int b, int j) -> bool {
    if (i >= k) return false;
    const int32_t a0 = agg_off[i], re = min(r, agg_off[i + 1] - a0 - 1);
    const T* xp = xs[(i - 1) & 1] + c0;
    T p = T(0);
#pragma unroll
    for (int q = 0; q < CQ; ++q) p += m[b][j][q] * xp[q];
    p = quad_sum(p);
    const double v = u[b][j] - (double)p;
    xs[i & 1][re] = (T)v;
    x2[a0 + re] = v;
    __syncthreads();
    return true;
  };
#pragma unroll
  for (int j = 0; j < P; ++j) load(1 + j, 0, j);
  __syncthreads();
  for (int32_t g0 = 1; g0 < k; g0 += 2 * P) {
#pragma unroll
    for (int j = 0; j < P; ++j) load(g0 + P + j, 1, j);
#pragma unroll
    for (int j = 0; j < P; ++j)
      if (!step(g0 + j, 0, j)) return;
#pragma unroll
    for (int j = 0; j < P; ++j) load(g0 + 2 * P + j, 0, j);
#pragma unroll
    for (int j = 0; j < P; ++j)
      if (!step(g0 + P + j, 1, j)) return;
  }
}

}  // namespace

template <class T, int ROWS, int CQ, int P>
void run_overlap_chain(int32_t k, const int32_t* ao, const int64_t* mo, const T* M, double* x2, hipStream_t s) {
  const size_t smem = 8 * (size_t)k + 4 * (size_t)(k + 1);
  static size_t raised = 64 * 1024;
  if (smem > raised) {
    ADDNS_HIP(hipFuncSetAttribute((const void*)k_overlap_chain<T, ROWS, CQ, P>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    raised = smem;
  }
  k_overlap_chain<T, ROWS, CQ, P><<<1, 4 * ROWS, smem, s>>>(k, ao, mo, M, x2);
}

// Row width of the chain matrices for aggregates of at most smax nodes (0:
// too large for the chain kernel).
int overlap_chain_width(int32_t smax) { return smax <= 64 ? 64 : (smax <= 80 ? 80 : (smax <= 128 ? 128 : 0)); }

void launch_overlap_chain(const addns_precond* pc, double* x2, hipStream_t s) {
  const Plan& pl = pc->plan;
  if (!pc->overlap_chain || pl.k < 2) return;
  const int32_t* ao = pc->agg_off.as<int32_t>();
  const int64_t* mo = pc->ovl_moff.as<int64_t>();
  const bool dbl = pc->schur_prec == P64;
  switch (pc->overlap_chain) {
    case 64:
      if (dbl) run_overlap_chain<double, 64, 16, 2>(pl.k, ao, mo, pc->ovl_m.as<double>(), x2, s);
      else run_overlap_chain<float, 64, 16, 4>(pl.k, ao, mo, pc->ovl_m.as<float>(), x2, s);
      break;
    case 80:
      if (dbl) run_overlap_chain<double, 80, 20, 2>(pl.k, ao, mo, pc->ovl_m.as<double>(), x2, s);
      else run_overlap_chain<float, 80, 20, 4>(pl.k, ao, mo, pc->ovl_m.as<float>(), x2, s);
      break;
    default:
      if (dbl) run_overlap_chain<double, 128, 32, 1>(pl.k, ao, mo, pc->ovl_m.as<double>(), x2, s);
      else run_overlap_chain<float, 128, 32, 2>(pl.k, ao, mo, pc->ovl_m.as<float>(), x2, s);
  }
}

}  // namespace addns
