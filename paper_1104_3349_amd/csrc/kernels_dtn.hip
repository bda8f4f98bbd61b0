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

#include <algorithm>

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
// network on the matrix cores
// ---------------------------------------------------------------------------
// One wave evaluates a tile of 16 samples.  Features are the row dimension
// of every product and samples the column dimension, so each layer is
//   Out (F_out x 16) = W (F_out x F_in) In (F_in x 16) + b
// on 16 x 16 MFMA tiles (FP32: v_mfma_f32_16x16x4f32; BF16 inference:
// v_mfma_f32_16x16x16bf16_1k, FP32 accumulation).  Lane l = 16 g + c holds
// rows 4 g + r (r = 0..3) of column c of an accumulator tile, which is the
// B operand of the next product if that product's K index runs over
// {4 g + r} for a fixed r (FP32) or over 4 g + r, r = 0..3 (BF16): the
// matching A operand (a weight row) is read with the same K order, so the
// layers chain in registers.  The first layer carries its bias as an
// eighth input fixed to 1; the others start from the bias.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));

// LDS copy of the weights, rows padded by one word (W1 with its bias as
// column 7, W3 padded to 16 rows of zeros).
constexpr int kLd1 = 9, kLd2 = kH + 1, kLd3 = kH + 1;
constexpr int kLdsW1 = kH * kLd1, kLdsW2 = kH * kLd2, kLdsW3 = 16 * kLd3;
struct alignas(16) WLds {
  float w1[kLdsW1];  // [64][9]: W1 | b1 | 0
  float w2[kLdsW2];  // [64][65]
  float w3[kLdsW3];  // [16][65], rows 5..15 zero
  float b2[kH];
  float b3[16];      // 5..15 zero
};
// The same layout in device memory (the weight image): built from the packed
// parameters once (k_mlp_image) and kept current by the Adam step, so that a
// workgroup stages it with wide, independent loads.
constexpr int kImgW1 = 0, kImgW2 = kImgW1 + kLdsW1, kImgW3 = kImgW2 + kLdsW2, kImgB2 = kImgW3 + kLdsW3,
              kImgB3 = kImgB2 + kH, kImg = kImgB3 + 16;
static_assert(sizeof(WLds) == sizeof(float) * kImg && kImg % 4 == 0, "weight image layout");

// image position of packed parameter prm
__device__ inline int img_pos(int prm) {
  if (prm < oB1) return kImgW1 + (prm / kIn) * kLd1 + prm % kIn;
  if (prm < oW2) return kImgW1 + (prm - oB1) * kLd1 + kIn;
  if (prm < oB2) return kImgW2 + ((prm - oW2) / kH) * kLd2 + (prm - oW2) % kH;
  if (prm < oW3) return kImgB2 + (prm - oB2);
  if (prm < oB3) return kImgW3 + ((prm - oW3) / kH) * kLd3 + (prm - oW3) % kH;
  return kImgB3 + (prm - oB3);
}

// one workgroup: zero the image (its padding stays zero), then place every
// parameter
__global__ void __launch_bounds__(256) k_mlp_image(const float* __restrict__ wts, float* __restrict__ img) {
  for (int i = threadIdx.x; i < kImg; i += blockDim.x) img[i] = 0.0f;
  __syncthreads();
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) img[img_pos(i)] = wts[i];
}

__device__ void stage_weights(WLds& L, const float* __restrict__ img, bool bf) {
  const float4* src = reinterpret_cast<const float4*>(img);
  float4* dst = reinterpret_cast<float4*>(&L);
#pragma unroll 8
  for (int i = threadIdx.x; i < kImg / 4; i += blockDim.x) {
    float4 v = src[i];
    if (bf) {
      v.x = bf16_round(v.x);
      v.y = bf16_round(v.y);
      v.z = bf16_round(v.z);
      v.w = bf16_round(v.w);
    }
    dst[i] = v;
  }
}

__device__ inline f32x4 relu4(f32x4 a) {
  f32x4 o;
#pragma unroll
  for (int r = 0; r < 4; ++r) o[r] = a[r] > 0.0f ? a[r] : 0.0f;
  return o;
}

// FP32 forward of one tile.  x[q] = input k = 4 q + g of sample c (k = 7:
// the constant 1 of a present sample).  h1, h2: hidden tiles; returns the
// output tile (rows 4 g + r < 5 meaningful).
__device__ inline f32x4 fwd_f32(const WLds& L, const float (&x)[2], f32x4 (&h1)[4], f32x4 (&h2)[4]) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < 2; ++q)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(L.w1[(16 * mt + c) * kLd1 + 4 * q + g], x[q], acc, 0, 0, 0);
    h1[mt] = relu4(acc);
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = L.b2[16 * mt + 4 * g + r];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(L.w2[(16 * mt + c) * kLd2 + 16 * kt + 4 * g + r], h1[kt][r], acc,
                                                   0, 0, 0);
    h2[mt] = relu4(acc);
  }
  f32x4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = L.b3[4 * g + r];
#pragma unroll
  for (int kt = 0; kt < 4; ++kt)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(L.w3[c * kLd3 + 16 * kt + 4 * g + r], h2[kt][r], acc, 0, 0, 0);
  return acc;
}

__device__ inline short bf16_bits(float x) { return (short)(__builtin_bit_cast(uint32_t, x) >> 16); }

// BF16 forward of one tile (weights in L already rounded to BF16; the
// inputs and the hidden activations are rounded here).  x[e] = input
// k = 4 g + e of sample c.
__device__ inline f32x4 fwd_bf16(const WLds& L, const float (&x)[4]) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  i16x4 xb;
#pragma unroll
  for (int e = 0; e < 4; ++e) xb[e] = bf16_bits(bf16_round(x[e]));
  i16x4 hb[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    i16x4 a;
#pragma unroll
    for (int e = 0; e < 4; ++e) a[e] = g < 2 ? bf16_bits(L.w1[(16 * mt + c) * kLd1 + 4 * g + e]) : (short)0;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, xb, acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) hb[mt][r] = bf16_bits(bf16_round(acc[r] > 0.0f ? acc[r] : 0.0f));
  }
  i16x4 h2b[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = L.b2[16 * mt + 4 * g + r];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
      i16x4 a;
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = bf16_bits(L.w2[(16 * mt + c) * kLd2 + 16 * kt + 4 * g + e]);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, hb[kt], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) h2b[mt][r] = bf16_bits(bf16_round(acc[r] > 0.0f ? acc[r] : 0.0f));
  }
  f32x4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = L.b3[4 * g + r];
#pragma unroll
  for (int kt = 0; kt < 4; ++kt) {
    i16x4 a;
#pragma unroll
    for (int e = 0; e < 4; ++e) a[e] = bf16_bits(L.w3[c * kLd3 + 16 * kt + 4 * g + e]);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, h2b[kt], acc, 0, 0, 0);
  }
  return acc;
}

// Inference: 4 waves per workgroup, each wave one tile of 16 samples at a
// time (grid-stride over tiles); weights staged once per workgroup.
constexpr int kFwdWaves = 4;
__global__ void __launch_bounds__(64 * kFwdWaves)
k_mlp_forward(const float* __restrict__ img, const float* __restrict__ X, float* __restrict__ P, int64_t count,
              int bf16) {
  __shared__ WLds L;
  stage_weights(L, img, bf16 != 0);
  __syncthreads();
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const int64_t tiles = (count + 15) / 16;
  for (int64_t t = (int64_t)blockIdx.x * kFwdWaves + (threadIdx.x >> 6); t < tiles;
       t += (int64_t)gridDim.x * kFwdWaves) {
    const int64_t k = 16 * t + c;
    const bool ok = k < count;
    f32x4 p;
    if (bf16) {
      float x[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = 4 * g + e;
        x[e] = !ok || j > kIn ? 0.0f : (j == kIn ? 1.0f : X[kIn * k + j]);
      }
      p = fwd_bf16(L, x);
    } else {
      float x[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int j = 4 * q + g;
        x[q] = !ok ? 0.0f : (j == kIn ? 1.0f : X[kIn * k + j]);
      }
      f32x4 h1[4], h2[4];
      p = fwd_f32(L, x, h1, h2);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * g + r;
      if (ok && o < kOut) P[kOut * k + o] = p[r];
    }
  }
}

// Partial gradient of one workgroup's samples (one wave; workgroup w takes
// the contiguous samples [w per, (w + 1) per), per a multiple of 16, in
// tiles of 16 in order): forward and backward per tile on the matrix cores,
// then the parameter gradients, which sum over samples, as products whose K
// index is the sample: the tiles are transposed through LDS (features on the
// lane's column, samples on its K slot) and accumulated in registers across
// the tiles.  gpart[wg][kNP] and lpart[wg] = loss sum.  The number of
// workgroups depends on the sample count only (mlp_grad_groups), so the
// summation order, and the result, is fixed for a given count.
constexpr int kMaxGradGroups = 1024;
constexpr int kLT = 17;  // LDS row stride of a transposed tile [feature][sample]
struct GLds {
  float h1[kH * kLT], h2[kH * kLT], d1[kH * kLT], d2[kH * kLT];
  float x[8 * kLT], dp[8 * kLT];
  float loss[64];
};

__global__ void __launch_bounds__(64)
k_mlp_grad(const float* __restrict__ img, const float* __restrict__ X, const float* __restrict__ Y,
           const float* __restrict__ M, const int32_t* __restrict__ idx, int64_t count, int64_t per,
           float scale, float* __restrict__ gpart, float* __restrict__ lpart) {
  __shared__ WLds L;
  __shared__ GLds T;
  stage_weights(L, img, false);
  const int l = threadIdx.x, g = l >> 4, c = l & 15;
  const f32x4 z4 = {0.0f, 0.0f, 0.0f, 0.0f};
  f32x4 gw1[4], gw2[4][4], gw3[4], gb2[4], gb3 = z4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    gw1[i] = z4;
    gw3[i] = z4;
    gb2[i] = z4;
#pragma unroll
    for (int j = 0; j < 4; ++j) gw2[i][j] = z4;
  }
  float loss = 0.0f;
  __syncthreads();
  const int64_t k0 = (int64_t)blockIdx.x * per, k1 = min(count, k0 + per);
  for (int64_t kt0 = k0; kt0 < k1; kt0 += 16) {
    const int64_t k = kt0 + c;
    const bool ok = k < k1;
    const int64_t sk = ok ? (idx ? idx[k] : k) : 0;
    float x[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int j = 4 * q + g;
      x[q] = !ok ? 0.0f : (j == kIn ? 1.0f : X[kIn * sk + j]);
    }
    f32x4 h1[4], h2[4];
    const f32x4 p = fwd_f32(L, x, h1, h2);
    // output error (rows 4 g + r < 5)
    f32x4 dp;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * g + r;
      dp[r] = 0.0f;
      if (ok && o < kOut) {
        const float m = M[kOut * sk + o];
        const float d = p[r] - Y[kOut * sk + o];
        loss += m * d * d;
        dp[r] = 2.0f * m * d * scale;
      }
    }
    // dH2 = W3^T dp through the ReLU (K over the outputs 4 g + r)
    f32x4 d2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 acc = z4;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(L.w3[(4 * g + r) * kLd3 + 16 * mt + c], dp[r], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) d2[mt][r] = h2[mt][r] > 0.0f ? acc[r] : 0.0f;
    }
    // dH1 = W2^T dH2 through the ReLU
    f32x4 d1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 acc = z4;
#pragma unroll
      for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(L.w2[(16 * kt + 4 * g + r) * kLd2 + 16 * mt + c], d2[kt][r],
                                                     acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) d1[mt][r] = h1[mt][r] > 0.0f ? acc[r] : 0.0f;
    }
    // transpose the tile through LDS: [feature][sample]
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = (16 * mt + 4 * g + r) * kLT + c;
        T.h1[f] = h1[mt][r];
        T.h2[f] = h2[mt][r];
        T.d1[f] = d1[mt][r];
        T.d2[f] = d2[mt][r];
      }
#pragma unroll
    for (int q = 0; q < 2; ++q) T.x[(4 * q + g) * kLT + c] = x[q];
    if (g < 2) {
#pragma unroll
      for (int r = 0; r < 4; ++r) T.dp[(4 * g + r) * kLT + c] = dp[r];
    }
    __syncthreads();
    // parameter gradients, K = the 16 samples in 4 steps of 4
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int sc = 4 * q + g;  // this lane's sample slot in step q
      float a2[4], b1[4], a1[4], b2[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a2[t] = T.d2[(16 * t + c) * kLT + sc];
        b1[t] = T.h1[(16 * t + c) * kLT + sc];
        a1[t] = T.d1[(16 * t + c) * kLT + sc];
        b2[t] = T.h2[(16 * t + c) * kLT + sc];
      }
      const float bx = c < 8 ? T.x[c * kLT + sc] : 0.0f;
      const float ap = c < kOut ? T.dp[c * kLT + sc] : 0.0f;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) gw2[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[mt], b1[nt], gw2[mt][nt], 0, 0, 0);
        gb2[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[mt], 1.0f, gb2[mt], 0, 0, 0);
        gw1[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[mt], bx, gw1[mt], 0, 0, 0);
        gw3[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ap, b2[mt], gw3[mt], 0, 0, 0);
      }
      gb3 = __builtin_amdgcn_mfma_f32_16x16x4f32(ap, 1.0f, gb3, 0, 0, 0);
    }
    __syncthreads();  // the next tile overwrites T
  }
  // every parameter written once: lane (g, c) holds rows 4 g + r of column c
  float* gout = gpart + (int64_t)blockIdx.x * kNP;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = 16 * mt + 4 * g + r;
      if (c < kIn) gout[oW1 + f * kIn + c] = gw1[mt][r];
      else if (c == kIn) gout[oB1 + f] = gw1[mt][r];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) gout[oW2 + f * kH + 16 * nt + c] = gw2[mt][nt][r];
      if (c == 0) gout[oB2 + f] = gb2[mt][r];
    }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * g + r;
      if (o < kOut) gout[oW3 + o * kH + 16 * nt + c] = gw3[nt][r];
    }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int o = 4 * g + r;
    if (c == 0 && o < kOut) gout[oB3 + o] = gb3[r];
  }
  // loss: fixed-order sum over the lanes
  T.loss[l] = loss;
  __syncthreads();
  if (l == 0) {
    float a = 0.0f;
    for (int q = 0; q < 64; ++q) a += T.loss[q];
    lpart[blockIdx.x] = a;
  }
}

// fixed-order sum of the workgroup partials, then (optionally) one Adam step
__global__ void k_mlp_reduce_adam(const float* __restrict__ gpart, int nwg, float* __restrict__ grad,
                                  float* __restrict__ wts, float* __restrict__ img, float* __restrict__ m1,
                                  float* __restrict__ m2, int adam, float lr, float b1, float b2, float eps, float bc1,
                                  float bc2) {
  const int prm = blockIdx.x * blockDim.x + threadIdx.x;
  if (prm >= kNP) return;
  // loads in batches of 8 (independent), added in partial order
  float g = 0.0f;
  int q = 0;
  for (; q + 8 <= nwg; q += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = gpart[(int64_t)(q + u) * kNP + prm];
#pragma unroll
    for (int u = 0; u < 8; ++u) g += v[u];
  }
  for (; q < nwg; ++q) g += gpart[(int64_t)q * kNP + prm];
  grad[prm] = g;
  if (!adam) return;
  const float a = b1 * m1[prm] + (1.0f - b1) * g;
  const float v = b2 * m2[prm] + (1.0f - b2) * g * g;
  m1[prm] = a;
  m2[prm] = v;
  const float wn = wts[prm] - lr * (a / bc1) / (sqrtf(v / bc2) + eps);
  wts[prm] = wn;
  img[img_pos(prm)] = wn;
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int mlp_param_count() { return kNP; }
int mlp_grad_groups(int64_t count) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((count + 15) / 16, kMaxGradGroups));
}

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
int mlp_image_floats() { return kImg; }
void launch_mlp_image(const float* wts, float* img, hipStream_t s) { k_mlp_image<<<1, 256, 0, s>>>(wts, img); }
void launch_mlp_forward(const float* img, const float* X, float* P, int64_t count, int bf16, hipStream_t s) {
  if (count <= 0) return;
  const int64_t tiles = (count + 15) / 16;
  const unsigned grid = (unsigned)std::min<int64_t>((tiles + kFwdWaves - 1) / kFwdWaves, 2048);
  k_mlp_forward<<<grid, 64 * kFwdWaves, 0, s>>>(img, X, P, count, bf16);
}
void launch_mlp_grad(const float* img, const float* X, const float* Y, const float* M, const int32_t* idx,
                     int64_t count, float scale, float* gpart, float* lpart, hipStream_t s) {
  if (count <= 0) return;
  const int nwg = mlp_grad_groups(count);
  const int64_t per = ((count + nwg - 1) / nwg + 15) / 16 * 16;
  k_mlp_grad<<<nwg, 64, 0, s>>>(img, X, Y, M, idx, count, per, scale, gpart, lpart);
}
void launch_mlp_reduce_adam(const float* gpart, int nwg, float* grad, float* wts, float* img, float* m1, float* m2,
                            int adam, float lr, float b1, float b2, float eps, float bc1, float bc2, hipStream_t s) {
  k_mlp_reduce_adam<<<nb(kNP, 256), 256, 0, s>>>(gpart, nwg, grad, wts, img, m1, m2, adam, lr, b1, b2, eps, bc1, bc2);
}

}  // namespace addns
