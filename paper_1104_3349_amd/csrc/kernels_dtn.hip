// Learned interface correction (an extension, not a method of the paper):
// a small MLP maps local stencil features of a separator velocity row to
// corrections of that row of G_i on G's own pattern, trained on interface
// blocks S_i that the library computes (a teacher mode, MSCN by default).
//
//   features (7): the five scaled stencil coefficients of the row in the slots
//     [far lower, near lower, diagonal, near upper, far upper] and the two
//     convective (skew-symmetric) coupling differences, near and far:
//       k_s = R_g (C(g,s) - C(s,g)) / 2;  f5 = k_nu - k_nl, f6 = k_fu - k_fl;
//   network: 7 -> 64 (ReLU) -> 64 (ReLU) -> 5, row-major weights
//     W1[64][7] b1[64] W2[64][64] b2[64] W3[5][64] b3[5]  (4997 parameters);
//   loss: (1/count) sum_k sum_s mask_ks (p_ks - y_ks)^2.
// Training runs in FP32 (minibatch gradients reduced in a fixed order, Adam);
// inference optionally rounds weights and activations to BF16.
#include <hip/hip_runtime.h>

#include "precond.h"

namespace addns {
namespace {

constexpr int kIn = 7, kH = 64, kOut = 5;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kOut * kH, kNP = oB3 + kOut;
static_assert(kNP == 4997, "parameter count");

__device__ inline float bf16_round(float x) {
  // round to nearest even on the upper 16 bits (finite inputs)
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __builtin_bit_cast(float, u & 0xffff0000u);
}

// ---------------------------------------------------------------------------
// features / targets / corrections
// ---------------------------------------------------------------------------
__device__ inline double csr_val(const int32_t* rp, const int32_t* ci, const double* cv, int32_t r, int32_t c) {
  int32_t lo = rp[r], hi = rp[r + 1];
  while (lo < hi) {  // columns are sorted
    int32_t mid = (lo + hi) >> 1;
    if (ci[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  return (lo < rp[r + 1] && ci[lo] == c) ? cv[lo] : 0.0;
}

__global__ void k_dtn_features(int64_t count, const int32_t* __restrict__ smp_row, const int32_t* __restrict__ smp_nb,
                               const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const double* __restrict__ cv, const int32_t* __restrict__ perm,
                               const double* __restrict__ R, float* __restrict__ X) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int32_t r = smp_row[k];
  const double Rg = R[perm[r]];
  double f[5], sk[5];
  for (int q = 0; q < 5; ++q) {
    const int32_t s = smp_nb[5 * k + q];
    f[q] = 0.0;
    sk[q] = 0.0;
    if (s < 0) continue;
    f[q] = csr_val(rp, ci, cv, r, s);
    if (q != 2) sk[q] = 0.5 * (f[q] - csr_val(rp, ci, cv, s, r) * Rg / R[perm[s]]);
  }
  float* x = X + kIn * k;
  for (int q = 0; q < 5; ++q) x[q] = (float)f[q];
  x[5] = (float)(sk[3] - sk[1]);
  x[6] = (float)(sk[4] - sk[0]);
}

__global__ void k_dtn_targets(int64_t count, const int64_t* __restrict__ smp_loc, const double* __restrict__ S,
                              const double* __restrict__ G, float* __restrict__ Y, float* __restrict__ M) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  for (int q = 0; q < 5; ++q) {
    const int64_t l = smp_loc[5 * k + q];
    Y[kOut * k + q] = l >= 0 ? (float)(S[l] - G[l]) : 0.0f;
    M[kOut * k + q] = l >= 0 ? 1.0f : 0.0f;
  }
}

__global__ void k_dtn_correct(int64_t count, const int64_t* __restrict__ smp_loc, const float* __restrict__ D,
                              double* __restrict__ G) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  for (int q = 0; q < 5; ++q) {
    const int64_t l = smp_loc[5 * k + q];
    if (l >= 0) G[l] += (double)D[kOut * k + q];
  }
}

// ---------------------------------------------------------------------------
// network
// ---------------------------------------------------------------------------
template <bool BF>
__device__ inline void mlp_fwd(const float* __restrict__ w, const float* x, float* h1, float* h2, float* p) {
  for (int i = 0; i < kH; ++i) {
    float a = w[oB1 + i];
#pragma unroll
    for (int j = 0; j < kIn; ++j) a += w[oW1 + i * kIn + j] * x[j];
    a = a > 0.0f ? a : 0.0f;
    h1[i] = BF ? bf16_round(a) : a;
  }
  for (int i = 0; i < kH; ++i) {
    float a = w[oB2 + i];
    for (int j = 0; j < kH; ++j) a += w[oW2 + i * kH + j] * h1[j];
    a = a > 0.0f ? a : 0.0f;
    h2[i] = BF ? bf16_round(a) : a;
  }
  for (int i = 0; i < kOut; ++i) {
    float a = w[oB3 + i];
    for (int j = 0; j < kH; ++j) a += w[oW3 + i * kH + j] * h2[j];
    p[i] = a;
  }
}

// one thread per sample; weights staged in LDS (rounded to BF16 when asked)
__global__ void __launch_bounds__(256)
k_mlp_forward(const float* __restrict__ wts, const float* __restrict__ X, float* __restrict__ P, int64_t count,
              int bf16) {
  __shared__ float w[kNP];
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) w[i] = bf16 ? bf16_round(wts[i]) : wts[i];
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  float x[kIn], h1[kH], h2[kH], p[kOut];
  for (int j = 0; j < kIn; ++j) x[j] = bf16 ? bf16_round(X[kIn * k + j]) : X[kIn * k + j];
  if (bf16) mlp_fwd<true>(w, x, h1, h2, p);
  else mlp_fwd<false>(w, x, h1, h2, p);
  for (int i = 0; i < kOut; ++i) P[kOut * k + i] = p[i];
}

// Partial gradient of one workgroup's samples (32 per workgroup, 64 threads):
// forward and backward per sample, then parameter-wise sums over the
// workgroup's samples in sample order.  gpart[wg][kNP], lpart[wg] = loss sum.
constexpr int kGS = 32;
__global__ void __launch_bounds__(64)
k_mlp_grad(const float* __restrict__ wts, const float* __restrict__ X, const float* __restrict__ Y,
           const float* __restrict__ M, const int32_t* __restrict__ idx, int64_t count, float scale,
           float* __restrict__ gpart, float* __restrict__ lpart) {
  __shared__ float w[kNP];
  __shared__ float sx[kGS][kIn], sh1[kGS][kH], sh2[kGS][kH], sd1[kGS][kH], sd2[kGS][kH], sdp[kGS][kOut];
  __shared__ float sl[kGS];
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) w[i] = wts[i];
  __syncthreads();
  const int t = threadIdx.x;
  const int64_t k = (int64_t)blockIdx.x * kGS + t;
  if (t < kGS) {
    float x[kIn], h1[kH], h2[kH], p[kOut], dp[kOut];
    const bool ok = k < count;
    const int64_t sk = ok ? (idx ? idx[k] : k) : 0;
    for (int j = 0; j < kIn; ++j) x[j] = ok ? X[kIn * sk + j] : 0.0f;
    mlp_fwd<false>(w, x, h1, h2, p);
    float loss = 0.0f;
    for (int i = 0; i < kOut; ++i) {
      const float m = ok ? M[kOut * sk + i] : 0.0f;
      const float d = p[i] - (ok ? Y[kOut * sk + i] : 0.0f);
      loss += m * d * d;
      dp[i] = 2.0f * m * d * scale;
    }
    sl[t] = loss;
    for (int i = 0; i < kOut; ++i) sdp[t][i] = dp[i];
    for (int j = 0; j < kIn; ++j) sx[t][j] = x[j];
    for (int i = 0; i < kH; ++i) {
      sh1[t][i] = h1[i];
      sh2[t][i] = h2[i];
    }
    // dh2 = W3^T dp, through ReLU
    for (int j = 0; j < kH; ++j) {
      float a = 0.0f;
      for (int i = 0; i < kOut; ++i) a += w[oW3 + i * kH + j] * dp[i];
      sd2[t][j] = h2[j] > 0.0f ? a : 0.0f;
    }
    // dh1 = W2^T dh2, through ReLU
    for (int j = 0; j < kH; ++j) {
      float a = 0.0f;
      for (int i = 0; i < kH; ++i) a += w[oW2 + i * kH + j] * sd2[t][i];
      sd1[t][j] = h1[j] > 0.0f ? a : 0.0f;
    }
  }
  __syncthreads();
  float* g = gpart + (int64_t)blockIdx.x * kNP;
  for (int prm = t; prm < kNP; prm += blockDim.x) {
    float a = 0.0f;
    if (prm < oB1) {
      const int i = prm / kIn, j = prm % kIn;
      for (int q = 0; q < kGS; ++q) a += sd1[q][i] * sx[q][j];
    } else if (prm < oW2) {
      const int i = prm - oB1;
      for (int q = 0; q < kGS; ++q) a += sd1[q][i];
    } else if (prm < oB2) {
      const int i = (prm - oW2) / kH, j = (prm - oW2) % kH;
      for (int q = 0; q < kGS; ++q) a += sd2[q][i] * sh1[q][j];
    } else if (prm < oW3) {
      const int i = prm - oB2;
      for (int q = 0; q < kGS; ++q) a += sd2[q][i];
    } else if (prm < oB3) {
      const int i = (prm - oW3) / kH, j = (prm - oW3) % kH;
      for (int q = 0; q < kGS; ++q) a += sdp[q][i] * sh2[q][j];
    } else {
      const int i = prm - oB3;
      for (int q = 0; q < kGS; ++q) a += sdp[q][i];
    }
    g[prm] = a;
  }
  if (t == 0) {
    float a = 0.0f;
    for (int q = 0; q < kGS; ++q) a += sl[q];
    lpart[blockIdx.x] = a;
  }
}

// fixed-order sum of the workgroup partials, then (optionally) one Adam step
__global__ void k_mlp_reduce_adam(const float* __restrict__ gpart, int nwg, float* __restrict__ grad,
                                  float* __restrict__ wts, float* __restrict__ m1, float* __restrict__ m2, int adam,
                                  float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const int prm = blockIdx.x * blockDim.x + threadIdx.x;
  if (prm >= kNP) return;
  float g = 0.0f;
  for (int q = 0; q < nwg; ++q) g += gpart[(int64_t)q * kNP + prm];
  grad[prm] = g;
  if (!adam) return;
  const float a = b1 * m1[prm] + (1.0f - b1) * g;
  const float v = b2 * m2[prm] + (1.0f - b2) * g * g;
  m1[prm] = a;
  m2[prm] = v;
  wts[prm] -= lr * (a / bc1) / (sqrtf(v / bc2) + eps);
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int mlp_param_count() { return kNP; }
int mlp_grad_group() { return kGS; }

void launch_dtn_features(int64_t count, const int32_t* smp_row, const int32_t* smp_nb, const int32_t* rp,
                         const int32_t* ci, const double* cv, const int32_t* perm, const double* R, float* X,
                         hipStream_t s) {
  if (count > 0) k_dtn_features<<<nb(count, 256), 256, 0, s>>>(count, smp_row, smp_nb, rp, ci, cv, perm, R, X);
}
void launch_dtn_targets(int64_t count, const int64_t* smp_loc, const double* S, const double* G, float* Y, float* M,
                        hipStream_t s) {
  if (count > 0) k_dtn_targets<<<nb(count, 256), 256, 0, s>>>(count, smp_loc, S, G, Y, M);
}
void launch_dtn_correct(int64_t count, const int64_t* smp_loc, const float* D, double* G, hipStream_t s) {
  if (count > 0) k_dtn_correct<<<nb(count, 256), 256, 0, s>>>(count, smp_loc, D, G);
}
void launch_mlp_forward(const float* wts, const float* X, float* P, int64_t count, int bf16, hipStream_t s) {
  if (count > 0) k_mlp_forward<<<nb(count, 256), 256, 0, s>>>(wts, X, P, count, bf16);
}
void launch_mlp_grad(const float* wts, const float* X, const float* Y, const float* M, const int32_t* idx,
                     int64_t count, float scale, float* gpart, float* lpart, hipStream_t s) {
  if (count > 0) k_mlp_grad<<<nb(count, kGS), 64, 0, s>>>(wts, X, Y, M, idx, count, scale, gpart, lpart);
}
void launch_mlp_reduce_adam(const float* gpart, int nwg, float* grad, float* wts, float* m1, float* m2, int adam,
                            float lr, float b1, float b2, float eps, float bc1, float bc2, hipStream_t s) {
  k_mlp_reduce_adam<<<nb(kNP, 256), 256, 0, s>>>(gpart, nwg, grad, wts, m1, m2, adam, lr, b1, b2, eps, bc1, bc2);
}

}  // namespace addns
