// bessel_mlp.hip -- learned bracket predictor for the FP32 path.
//
// A small network maps the features of an element to its integration bracket
// [t0, t1] (the range of Section 2.1, Eq. (7)-(8)), so the peak and bracket
// searches of Sections 2.2-2.3 are skipped.  It is trained on brackets produced
// by the method's own range finder (find_bracket at the FP32 margin).  Every
// predicted bracket is checked after the bins; elements that fail are
// compacted into a worklist and recomputed by the Newton path, which therefore
// remains both the fallback and the reference for the predictor's error.
//
//   features  z = ((log max(|v|, 1e-3) - m_v) / s_v, (log x - m_x) / s_x)
//   network   h1 = clamp(W1 z + b1, -1, 1), h2 = phi(W2 h1 + b2), y = W3 h2 + b3
//             (2 -> 64 -> 64 -> 2; FP32 master weights)
//   activations  tanh-shaped, without transcendentals: the first layer's is
//             the clamp to [-1, 1] (slope 1 inside, 0 outside), the second's
//             phi(a) = u (3 - u^2) / 2 with u = clamp(a / 1.5, -1, 1), a cubic
//             sigmoid (odd, slope 1 at 0, flat at +-1 from |a| = 1.5,
//             continuously differentiable), phi'(a) = 1 - u^2; inference
//             evaluates both in packed f16 arithmetic
//   bracket   t0 = max(0, y0 - margin_t0) exp(y1), t1 = exp(y1 + margin_t1)
//   targets   y0* = t0/t1, y1* = log t1 of the Newton bracket
//   loss      mean of 1/2 (w0 e0^2 + w1 e1^2), e = y - y*, with weight alpha on
//             the unsafe side (t0 too large, t1 too small)
//
// Parameter vector (floats): W1 (64 x 2, row-major), b1[64], W2 (64 x 64,
// W2[i][j] multiplies h1[j]), b2[64], W3 (2 x 64), b3[2]  -- 4482 trainable
// values -- then m_v, s_v, m_x, s_x, margin_t1, margin_t0, 0, 0.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "bessel.h"
#include "bessel_device.hpp"
#include "bessel_internal.hpp"
#include "bessel_learned.hpp"

namespace bk {

constexpr int kH = 64;
constexpr int kNW = BESSEL_MLP_NWEIGHTS;  // 4482
constexpr int kNP = BESSEL_MLP_NPARAMS;   // 4490
constexpr int oW1 = 0, ob1 = 128, oW2 = 192, ob2 = 4288, oW3 = 4352, ob3 = 4480, oMeta = 4482;
constexpr float kMarginF32 = 15.9423851528787422f;  // -log 2^-23

// ---------------------------------------------------------------------------
// Shared device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mlp_features(const float* __restrict__ P, float v, float x, float& z0, float& z1) {
  const float lv = kLn2F * hlog2(fmaxf(fabsf(v), kVFloor));
  const float lx = kLn2F * hlog2(x);
  z0 = (lv - P[oMeta + 0]) / P[oMeta + 1];
  z1 = (lx - P[oMeta + 2]) / P[oMeta + 3];
}

// The activation: phi(a) = u (3 - u^2) / 2, u = clamp(a / kActC, -1, 1), and
// its derivative (3 / (2 kActC)) (1 - u^2), which is 1 - u^2 at kActC = 1.5.
constexpr float kActC = 1.5f;
__device__ __forceinline__ float act_phi(float a, float& dphi) {
  const float u = fminf(fmaxf(a * (1.0f / kActC), -1.0f), 1.0f);
  const float u2 = u * u;
  dphi = (1.5f / kActC) * (1.0f - u2);
  return 0.5f * u * (3.0f - u2);
}
__device__ __forceinline__ float act_phi(float a) {
  float d;
  return act_phi(a, d);
}
// The first layer's activation: clamp(a, -1, 1), derivative 1 inside.
__device__ __forceinline__ float act_clamp(float a, float& d) {
  d = fabsf(a) < 1.0f ? 1.0f : 0.0f;
  return fminf(fmaxf(a, -1.0f), 1.0f);
}

// splitmix64 (Steele, Lea, Flood 2014): counter-based draws for minibatches.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Labels: the Newton bracket at the FP32 margin.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_mlp_labels(int64_t n, const float* __restrict__ v,
                                                       const float* __restrict__ x, float* __restrict__ t0,
                                                       float* __restrict__ t1) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const Bracket b = find_bracket<false>(fabs((double)v[i]), (double)x[i], kMarginF32);
  t0[i] = b.t0;
  t1[i] = b.t1;
}

// ---------------------------------------------------------------------------
// Training: forward and backward of a block of 64 samples (FP32), per-block
// partial gradients, then a fixed-order reduction over blocks (deterministic).
// Four wavefronts per block; wavefront w owns hidden-unit tile w (units
// 16w..16w+15) of both layers.  Of the three 64 x 64 x 64 products of a block
// -- the second layer forward (W2 H1), its backward (W2^T D2) and the weight
// gradient (D2 H1^T) -- each wavefront computes the 16 rows of its tile, on
// v_mfma_f32_16x16x4f32 (FP32 operands, FP32 accumulation); the rest runs on
// the VALU.  Matrices pass through LDS sample-major, [sample][unit], one pad
// column so that fragment reads along either index hit distinct banks.
//
// v_mfma_f32_16x16x4f32, lane l:  A (16 x 4) element [l % 16][l / 16],
// B (4 x 16) element [l / 16][l % 16], D (16 x 16) elements
// [4 (l / 16) + r][l % 16], r = 0..3.
// ---------------------------------------------------------------------------
constexpr int kTB = 64;          // samples per training block
constexpr int kTW = kH / 16;     // wavefronts per training block, one per unit tile
constexpr int kTT = kTB * kTW;   // threads per training block
static_assert(oMeta - oW3 <= 3 * kTB && kH <= kTB && oW2 <= 3 * kTB, "the VALU sums fit the block's lanes");

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct TrainLds {
  float h1[kTB][kH + 1];  // layer-1 activations
  float g1[kTB][kH + 1];  // the derivatives of their activation
  float d2[kTB][kH + 1];  // layer-2 deltas
  float c[kTB][kH + 1];   // layer-2 activations, then layer-1 deltas
  float z[kTB][2];
  float tg[kTB][2];       // targets t0/t1, log t1
  float dy[kTB][2];
  float yp[kTW][kTB][2];  // each tile's share of the outputs
  float loss[kTB];
  int valid[kTB];
};

// sampled: sample s of the step is index splitmix64(seed ^ step-key ^ s) mod n;
// otherwise sample s is element s.  Partial gradients of block b go to
// partial[b * (kNW + 1) .. + kNW), the partial loss to partial[b * (kNW + 1) + kNW].
__global__ __launch_bounds__(kTT) void k_mlp_grad(const float* __restrict__ P, int64_t n, int64_t batch,
                                                  int sampled, uint64_t seed, int64_t step,
                                                  const float* __restrict__ v, const float* __restrict__ x,
                                                  const float* __restrict__ lt0, const float* __restrict__ lt1,
                                                  float alpha, float* __restrict__ partial) {
  __shared__ TrainLds S;
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63;  // w: the unit tile (wavefront-uniform)
  const int lr = l & 15, lg = l >> 4;
  // layer 1, one sample per lane, the tile's 16 units; wavefront 0 also
  // keeps the features and the targets
  {
    const int64_t s = (int64_t)blockIdx.x * kTB + l;
    const bool valid = s < batch;
    float z0 = 0.0f, z1 = 0.0f;
    int64_t idx = 0;
    if (valid) {
      idx = sampled ? (int64_t)(splitmix64(seed ^ ((uint64_t)step * 0x100000001b3ULL) ^ (uint64_t)s) % (uint64_t)n)
                    : s;
      mlp_features(P, v[idx], x[idx], z0, z1);
    }
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * w + jj;
      float d = 0.0f;
      S.h1[l][j] = valid ? act_clamp(fmaf(P[oW1 + 2 * j], z0, fmaf(P[oW1 + 2 * j + 1], z1, P[ob1 + j])), d) : 0.0f;
      S.g1[l][j] = d;
    }
    if (w == 0) {
      float y0t = 0.0f, y1t = 0.0f;
      if (valid) {
        const float T0 = lt0[idx], T1 = lt1[idx];
        y0t = T0 / T1;
        y1t = logf(T1);
      }
      S.z[l][0] = z0;
      S.z[l][1] = z1;
      S.tg[l][0] = y0t;
      S.tg[l][1] = y1t;
      S.valid[l] = valid ? 1 : 0;
    }
  }
  __syncthreads();

  // layer 2 of the tile: A2 = W2 H1 + b2, tiles [w][sample tile st]
  f32x4 acc[4];
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[st][r] = P[ob2 + 16 * w + 4 * lg + r];
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) {
    const float a = P[oW2 + (16 * w + lr) * kH + 4 * ks + lg];
    float b[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) b[st] = S.h1[16 * st + lr][4 * ks + lg];
#pragma unroll
    for (int st = 0; st < 4; ++st) acc[st] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[st], acc[st], 0, 0, 0);
  }
  // h2 = phi(A2) and the tile's share of y = W3 h2 + b3: each lane holds 4
  // units of each of its 4 samples; the 4 lanes of a sample (l % 16 equal)
  // add up, then the shares of the tiles meet in LDS
  float y0p[4] = {0.0f, 0.0f, 0.0f, 0.0f}, y1p[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  float g2[4][4];  // phi'(a2)
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * w + 4 * lg + r;
      const float h = act_phi(acc[st][r], g2[st][r]);
      acc[st][r] = h;
      y0p[st] = fmaf(P[oW3 + i], h, y0p[st]);
      y1p[st] = fmaf(P[oW3 + kH + i], h, y1p[st]);
    }
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    y0p[st] += __shfl_xor(y0p[st], 16);
    y0p[st] += __shfl_xor(y0p[st], 32);
    y1p[st] += __shfl_xor(y1p[st], 16);
    y1p[st] += __shfl_xor(y1p[st], 32);
    if (lg == 0) {
      S.yp[w][16 * st + lr][0] = y0p[st];
      S.yp[w][16 * st + lr][1] = y1p[st];
    }
  }
  __syncthreads();
  // output errors (every wavefront, the same sums in the same order)
  float dy0[4], dy1[4];
  const float inv_b = 1.0f / (float)batch;
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int q = 16 * st + lr;
    dy0[st] = 0.0f;
    dy1[st] = 0.0f;
    float lossv = 0.0f;
    if (S.valid[q]) {
      const float y0 = (S.yp[0][q][0] + S.yp[1][q][0]) + (S.yp[2][q][0] + S.yp[3][q][0]);
      const float y1 = (S.yp[0][q][1] + S.yp[1][q][1]) + (S.yp[2][q][1] + S.yp[3][q][1]);
      const float e0 = (y0 + P[ob3]) - S.tg[q][0];
      const float e1 = (y1 + P[ob3 + 1]) - S.tg[q][1];
      const float w0 = e0 > 0.0f ? alpha : 1.0f;
      const float w1 = e1 < 0.0f ? alpha : 1.0f;
      lossv = 0.5f * (w0 * e0 * e0 + w1 * e1 * e1) * inv_b;
      dy0[st] = w0 * e0 * inv_b;
      dy1[st] = w1 * e1 * inv_b;
    }
    if (w == 0 && lg == 0) {
      S.dy[q][0] = dy0[st];
      S.dy[q][1] = dy1[st];
      S.loss[q] = lossv;
    }
  }
  // layer-2 deltas of the tile (zero for invalid samples, whose dy is zero)
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * w + 4 * lg + r, q = 16 * st + lr;
      S.c[q][i] = acc[st][r];
      S.d2[q][i] = fmaf(P[oW3 + i], dy0[st], P[oW3 + kH + i] * dy1[st]) * g2[st][r];
    }
  __syncthreads();

  float* out = partial + (int64_t)blockIdx.x * (kNW + 1);
  if (t < oMeta - oW3) {
    // W3, b3 (VALU: 130 values over the 64 samples), wavefronts 0-2
    const int e = oW3 + t;
    float a = 0.0f;
    if (e < ob3) {
      const int o = (e - oW3) >> 6, i = (e - oW3) & 63;
      for (int q = 0; q < kTB; ++q) a = fmaf(S.dy[q][o], S.c[q][i], a);
    } else {
      const int o = e - ob3;
      for (int q = 0; q < kTB; ++q) a += S.dy[q][o];
    }
    out[e] = a;
  } else if (t >= 3 * kTB && t < 3 * kTB + kH) {
    // b2 (VALU), wavefront 3
    const int i = t - 3 * kTB;
    float a = 0.0f;
    for (int q = 0; q < kTB; ++q) a += S.d2[q][i];
    out[ob2 + i] = a;
  }
  // layer-1 deltas of the tile: D1 = (W2^T D2) (1 - h1^2), tiles [w][sample tile st]
  f32x4 acc1[4];
#pragma unroll
  for (int st = 0; st < 4; ++st) acc1[st] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) {
    const float a = P[oW2 + (4 * ks + lg) * kH + 16 * w + lr];
    float b[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) b[st] = S.d2[16 * st + lr][4 * ks + lg];
#pragma unroll
    for (int st = 0; st < 4; ++st) acc1[st] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[st], acc1[st], 0, 0, 0);
  }
  // W2 gradient, rows of the tile: D2 H1^T, tiles [w][unit tile jt], k over samples
  f32x4 accw[4];
#pragma unroll
  for (int jt = 0; jt < 4; ++jt) accw[jt] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) {
    const float a = S.d2[4 * ks + lg][16 * w + lr];
    float b[4];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) b[jt] = S.h1[4 * ks + lg][16 * jt + lr];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) accw[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[jt], accw[jt], 0, 0, 0);
  }
#pragma unroll
  for (int jt = 0; jt < 4; ++jt)
#pragma unroll
    for (int r = 0; r < 4; ++r) out[oW2 + (16 * w + 4 * lg + r) * kH + 16 * jt + lr] = accw[jt][r];
  __syncthreads();  // every read of S.c (the W3 sums) is done
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * w + 4 * lg + r, q = 16 * st + lr;
      S.c[q][j] = acc1[st][r] * S.g1[q][j];
    }
  __syncthreads();  // the layer-1 deltas in S.c
  if (t < oW2) {
    // W1, b1 (VALU: 192 values), wavefronts 0-2
    const int e = t;
    float a = 0.0f;
    if (e < ob1) {
      const int j = e >> 1, k = e & 1;
      for (int q = 0; q < kTB; ++q) a = fmaf(S.c[q][j], S.z[q][k], a);
    } else {
      const int j = e - ob1;
      for (int q = 0; q < kTB; ++q) a += S.c[q][j];
    }
    out[e] = a;
  } else if (t == 3 * kTB) {
    float ls = 0.0f;
    for (int q = 0; q < kTB; ++q) ls += S.loss[q];
    out[kNW] = ls;
  }
}

// grad[e] = sum over blocks of partial[b][e] in block order; loss likewise.
// Sum over blocks of value e of the partials, in block order (deterministic);
// 32 loads in flight per group (the sum is latency-bound: a few hundred
// threads in all).
__device__ __forceinline__ float reduce_partials(const float* __restrict__ partial, int nblocks, int e) {
  constexpr int kFly = 32;
  double acc = 0.0;
  int b = 0;
  for (; b + kFly <= nblocks; b += kFly) {
    float p[kFly];
#pragma unroll
    for (int j = 0; j < kFly; ++j) p[j] = partial[(int64_t)(b + j) * (kNW + 1) + e];
#pragma unroll
    for (int j = 0; j < kFly; ++j) acc += (double)p[j];
  }
  for (; b < nblocks; ++b) acc += (double)partial[(int64_t)b * (kNW + 1) + e];
  return (float)acc;
}

__global__ __launch_bounds__(kBlock) void k_mlp_reduce(const float* __restrict__ partial, int nblocks,
                                                       float* __restrict__ grad, float* __restrict__ loss) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e > kNW) return;
  const float g = reduce_partials(partial, nblocks, e);
  if (e < kNW) grad[e] = g;
  else if (loss) *loss = g;
}

// Adam (Kingma & Ba) with bias correction; step counts from 1.
__device__ __forceinline__ void adam_update(float* __restrict__ P, float g, float* __restrict__ m,
                                            float* __restrict__ s2, int e, int64_t step, float lr, float beta1,
                                            float beta2, float eps) {
  const float mm = beta1 * m[e] + (1.0f - beta1) * g;
  const float ss = beta2 * s2[e] + (1.0f - beta2) * g * g;
  m[e] = mm;
  s2[e] = ss;
  const float mh = mm / (1.0f - powf(beta1, (float)step));
  const float sh = ss / (1.0f - powf(beta2, (float)step));
  P[e] -= lr * mh / (sqrtf(sh) + eps);
}

__global__ __launch_bounds__(kBlock) void k_mlp_adam(float* __restrict__ P, const float* __restrict__ grad,
                                                     float* __restrict__ m, float* __restrict__ s2, int64_t step,
                                                     float lr, float beta1, float beta2, float eps) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= kNW) return;
  adam_update(P, grad[e], m, s2, e, step, lr, beta1, beta2, eps);
}

// One training step's tail in one launch: the ordered reduction of the block
// partials and the Adam update of each parameter; the batch loss goes to *loss.
__global__ __launch_bounds__(kBlock) void k_mlp_reduce_adam(const float* __restrict__ partial, int nblocks,
                                                            float* __restrict__ P, float* __restrict__ m,
                                                            float* __restrict__ s2, int64_t step, float lr,
                                                            float beta1, float beta2, float eps,
                                                            float* __restrict__ loss) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e > kNW) return;
  const float g = reduce_partials(partial, nblocks, e);
  if (e < kNW)
    adam_update(P, g, m, s2, e, step, lr, beta1, beta2, eps);
  else
    *loss = g;
}

// ---------------------------------------------------------------------------
// Inference
// ---------------------------------------------------------------------------

// FP32 reference forward, one element per lane, the activation in FP32 (for
// parity tests).
__global__ __launch_bounds__(kBlock) void k_mlp_forward_f32(const float* __restrict__ P, int64_t n,
                                                            const float* __restrict__ v, const float* __restrict__ x,
                                                            float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float z0, z1;
  mlp_features(P, v[i], x[i], z0, z1);
  float h1[kH];
  for (int j = 0; j < kH; ++j) {
    float d;
    h1[j] = act_clamp(fmaf(P[oW1 + 2 * j], z0, fmaf(P[oW1 + 2 * j + 1], z1, P[ob1 + j])), d);
  }
  float y0 = P[ob3], y1 = P[ob3 + 1];
  for (int k = 0; k < kH; ++k) {
    float a = P[ob2 + k];
    for (int j = 0; j < kH; ++j) a = fmaf(P[oW2 + k * kH + j], h1[j], a);
    const float h2 = act_phi(a);
    y0 = fmaf(P[oW3 + k], h2, y0);
    y1 = fmaf(P[oW3 + kH + k], h2, y1);
  }
  y[2 * i] = y0;
  y[2 * i + 1] = y1;
}

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Inference operands, rebuilt from the FP32 parameters whenever they change
// (k_mlp_pack) so that a wavefront loads its fragments with a few 16-byte loads.
// Each layer's MFMA produces A = k a + 1/2 for its pre-activation a, with
// k = 1/2 (first layer) or 1 / (2 kActC) (second), so that w = clamp(A, 0, 1)
// is the conversion to f16 with its clamp, and the activations are
//   clamp(a, -1, 1) = 2 w - 1,   phi(a) = 2 S(w) - 1,  S(w) = w^2 (3 - 2 w);
// the next layer takes w or S through  W (2 X - 1) + b = 2 W X + (b - sum W).
//   header  z0 = log2 max(|v|, 1e-3) * c_v + d_v,  z1 = log2 x * c_x + d_x
//           (c = ln 2 / s, d = -m / s), e^{margin_t1}, margin_t0, b3'[2]
//   A1      layer-1 fragments: for hidden tile ht and row lr, the eight f16
//           values (Wh0, Wh0, Wl0, Wh1, Wh1, Wl1, bh, bl) -- hi/lo splits of
//           W1 / 2 and b1 / 2 + 1/2 -- which meet
//           (zh0, zl0, zh0, zh1, zl1, zh1, 1, 1)
//   A2      layer-2 fragments (f16 of W2 / kActC) per output tile, k-block and
//           lane, columns in the order the layer-1 results reach the lane
//   B2      (b2 - sum_j W2[., j]) / (2 kActC) + 1/2 in accumulator order
//   A3      layer-3 fragments (f16 of 2 W3) per element tile et and k-block:
//           output c on row 4 et + c, zero rows elsewhere, so that the four
//           tiles share one accumulator and each lane ends with the outputs of
//           its own element;  b3' = b3 - sum_i W3[., i]
constexpr int qA1 = 16, qA2 = qA1 + 4 * 16 * 4, qB2 = qA2 + 4 * 2 * 64 * 4, qA3 = qB2 + kH,
              kNQ = qA3 + 4 * 2 * 64 * 4;
constexpr float kPreScale1 = 0.5f;          // layer 1: A = a / 2 + 1/2
constexpr float kPreScale = 0.5f / kActC;  // layer 2: A = a / (2 kActC) + 1/2

// hidden unit fed by k-slot j of lane group g in k-block kb of layer 2: the
// layer-1 accumulators of tiles 2kb and 2kb+1 hold rows 4g..4g+3 of each
__host__ __device__ constexpr int l2_col(int kb, int g, int j) { return 32 * kb + (j < 4 ? 4 * g + j : 16 + 4 * g + j - 4); }

__global__ __launch_bounds__(kBlock) void k_mlp_pack(const float* __restrict__ P, float* __restrict__ Q) {
  const int t = threadIdx.x;
  _Float16* a1 = reinterpret_cast<_Float16*>(Q + qA1);
  _Float16* a2 = reinterpret_cast<_Float16*>(Q + qA2);
  if (t < kH) {
    const int h = t;  // = 16 ht + lr
    const float w[3] = {kPreScale1 * P[oW1 + 2 * h], kPreScale1 * P[oW1 + 2 * h + 1],
                        fmaf(kPreScale1, P[ob1 + h], 0.5f)};
    _Float16 hi[3], lo[3];
    for (int k = 0; k < 3; ++k) {
      hi[k] = (_Float16)w[k];
      lo[k] = (_Float16)(w[k] - (float)hi[k]);
    }
    const _Float16 e[8] = {hi[0], hi[0], lo[0], hi[1], hi[1], lo[1], hi[2], lo[2]};
    for (int j = 0; j < 8; ++j) a1[h * 8 + j] = e[j];
    double rs = (double)P[ob2 + h];
    for (int j = 0; j < kH; ++j) rs -= (double)P[oW2 + h * kH + j];
    Q[qB2 + h] = (float)fma((double)kPreScale, rs, 0.5);  // 16 ho + 4 g + r is the natural order
  }
  _Float16* a3 = reinterpret_cast<_Float16*>(Q + qA3);
  for (int idx = t; idx < 4 * 2 * 64 * 8; idx += kBlock) {
    const int j = idx & 7, l = (idx >> 3) & 63, kb = (idx >> 9) & 1, hi = idx >> 10;
    const int row = 16 * hi + (l & 15);
    a2[idx] = (_Float16)(2.0f * kPreScale * P[oW2 + row * kH + l2_col(kb, l >> 4, j)]);
    // layer 3 for element tile et = hi: output c on row 4 et + c
    const int c = (l & 15) - 4 * hi;
    a3[idx] = (c == 0 || c == 1) ? (_Float16)(2.0f * P[oW3 + c * kH + l2_col(kb, l >> 4, j)]) : (_Float16)0.0f;
  }
  if (t < 2) {
    double s = (double)P[ob3 + t];
    for (int i = 0; i < kH; ++i) s -= (double)P[oW3 + t * kH + i];
    Q[qHdr + 6 + t] = (float)s;
  }
  if (t == 0) {
    Q[qHdr + 0] = kLn2F / P[oMeta + 1];
    Q[qHdr + 1] = -P[oMeta + 0] / P[oMeta + 1];
    Q[qHdr + 2] = kLn2F / P[oMeta + 3];
    Q[qHdr + 3] = -P[oMeta + 2] / P[oMeta + 3];
    Q[qHdr + 4] = hexp2(kLog2eF * P[oMeta + 4]);
    Q[qHdr + 5] = P[oMeta + 5];
    for (int k = 8; k < 16; ++k) Q[qHdr + k] = 0.0f;
  }
}

// clamp(A, 0, 1) for two accumulators as packed f16: the clamp rides on the
// conversion (v_cvt_pk_f16_f32 with its clamp bit), one instruction.
__device__ __forceinline__ f16x2 clamp_pair(float a, float b) {
  const _Float16 zero = (_Float16)0.0f, one = (_Float16)1.0f;
  const f16x2 w = (f16x2){(_Float16)a, (_Float16)b};
  return __builtin_elementwise_min(__builtin_elementwise_max(w, (f16x2){zero, zero}), (f16x2){one, one});
}

// S(clamp(A, 0, 1)) for two accumulators: the conversion with its clamp, then
// one packed FMA and two packed products; 4 instructions for 2 activations.
__device__ __forceinline__ f16x2 cubic_pair(float a, float b) {
  const _Float16 two = (_Float16)2.0f, three = (_Float16)3.0f;
  const f16x2 w = clamp_pair(a, b);
  return (w * w) * (w * (f16x2){-two, -two} + (f16x2){three, three});
}

// The activations of one 16 x 16 accumulator pair (rows 4g..4g+3 of two
// tiles), packed as the next layer's f16x8 k-slots: w (CUBIC false) or S(w).
template <bool CUBIC>
__device__ __forceinline__ f16x8 act_tiles(f32x4 d0, f32x4 d1) {
  auto pair = [](float a, float b) { return CUBIC ? cubic_pair(a, b) : clamp_pair(a, b); };
  const f16x4 p = __builtin_shufflevector(pair(d0[0], d0[1]), pair(d0[2], d0[3]), 0, 1, 2, 3);
  const f16x4 q = __builtin_shufflevector(pair(d1[0], d1[1]), pair(d1[2], d1[3]), 0, 1, 2, 3);
  return __builtin_shufflevector(p, q, 0, 1, 2, 3, 4, 5, 6, 7);
}

// One wavefront evaluates the network for its 64 elements (lane = element),
// every layer on v_mfma_f32_16x16x32_f16 or the VALU:
//   A (16 x 32):  lane l holds row l%16, k-slots 8(l/16)..8(l/16)+7
//   B (32 x 16):  lane l holds column l%16, k-slots 8(l/16)..8(l/16)+7
//   D (16 x 16):  lane l holds column l%16, rows 4(l/16)..4(l/16)+3
// Layer 1: D[hidden][element] = A1 * Z, where element tile et takes the
// features only from lane group et (its own elements), zeros elsewhere.
// Layer 2: D[hidden out][element] = A2 * W1^T + B2; the layer-1 activations
// of a lane are already its B fragments (k-slots permuted as l2_col).
// Layer 3: D[4 et + c][element] += A3(et) * S2^T over the four element tiles
// into one accumulator; lane l = 16 g + e ends with rows 4g, 4g + 1 of column
// e, the two outputs of its own element.
// Every lane of the wavefront must call it.
__device__ __forceinline__ void mlp_wave_mfma(const float* __restrict__ Q, float z0, float z1, float& y0, float& y1) {
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lg = l >> 4;
  f16x8 zf;
  {
    const _Float16 z0h = (_Float16)z0, z1h = (_Float16)z1;
    const _Float16 z0l = (_Float16)(z0 - (float)z0h), z1l = (_Float16)(z1 - (float)z1h);
    const _Float16 one = (_Float16)1.0f;
    zf[0] = z0h;
    zf[1] = z0l;
    zf[2] = z0h;
    zf[3] = z1h;
    zf[4] = z1l;
    zf[5] = z1h;
    zf[6] = one;
    zf[7] = one;
  }
  f16x8 zero;
#pragma unroll
  for (int j = 0; j < 8; ++j) zero[j] = (_Float16)0.0f;
  const f16x8* A1 = reinterpret_cast<const f16x8*>(Q + qA1);
  const f16x8* A2 = reinterpret_cast<const f16x8*>(Q + qA2);
  f16x8 a1[4], a2[4][2], a3[4][2];
  f32x4 b2[4];
#pragma unroll
  for (int ht = 0; ht < 4; ++ht) a1[ht] = A1[ht * 16 + lr];
#pragma unroll
  for (int ho = 0; ho < 4; ++ho) {
    a2[ho][0] = A2[(ho * 2 + 0) * 64 + l];
    a2[ho][1] = A2[(ho * 2 + 1) * 64 + l];
    b2[ho] = *reinterpret_cast<const f32x4*>(Q + qB2 + 16 * ho + 4 * lg);
    const f16x8* A3 = reinterpret_cast<const f16x8*>(Q + qA3);
    a3[ho][0] = A3[(ho * 2 + 0) * 64 + l];  // ho doubles as the element tile here
    a3[ho][1] = A3[(ho * 2 + 1) * 64 + l];
  }
  f32x4 acc = {Q[qHdr + 6], Q[qHdr + 7], 0.0f, 0.0f};  // rows 4g + c start at b3'[c]
#pragma unroll
  for (int et = 0; et < 4; ++et) {
    const f16x8 bz = (lg == et) ? zf : zero;
    f32x4 d1[4];
#pragma unroll
    for (int ht = 0; ht < 4; ++ht) {
      d1[ht] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
      d1[ht] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1[ht], bz, d1[ht], 0, 0, 0);
    }
    const f16x8 h[2] = {act_tiles<false>(d1[0], d1[1]), act_tiles<false>(d1[2], d1[3])};
    f32x4 d2[4];
#pragma unroll
    for (int ho = 0; ho < 4; ++ho) {
      d2[ho] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2[ho][0], h[0], b2[ho], 0, 0, 0);
      d2[ho] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2[ho][1], h[1], d2[ho], 0, 0, 0);
    }
    const f16x8 h3[2] = {act_tiles<true>(d2[0], d2[1]), act_tiles<true>(d2[2], d2[3])};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a3[et][0], h3[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a3[et][1], h3[1], acc, 0, 0, 0);
  }
  y0 = acc[0];
  y1 = acc[1];
}

__global__ __launch_bounds__(kBlock) void k_mlp_forward_mfma(const float* __restrict__ Q, int64_t n,
                                                             const float* __restrict__ v,
                                                             const float* __restrict__ x, float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  float z0 = 0.0f, z1 = 0.0f;
  if (i < n) mlp_features_q(Q, v[i], x[i], z0, z1);
  float y0, y1;
  mlp_wave_mfma(Q, z0, z1, y0, y1);
  if (i < n) {
    y[2 * i] = y0;
    y[2 * i + 1] = y1;
  }
}

// Tabulated network (range mode BESSEL_RANGE_MLP_TABLE).  The features are
// two-dimensional, so the network's outputs can be tabulated once per change
// of the parameters: k_mlp_tab_nodes runs the f16-MFMA inference above on a
// kTab x kTab grid of the feature plane, z in [-kTabZ, kTabZ]^2, and
// k_mlp_tab_cells stores per cell the bilinear coefficients of both outputs
// (value, d/du, d/dw, d2/dudw; 8 floats = one aligned 32-byte record).  An
// element then costs one record load and six FMAs instead of 128 activations.
// Interpolation moves the outputs by ~1e-3 (y0) and ~4e-4 (y1) on the scale
// workload, far inside the margins; the check after the bins still decides.
// grid: kTab * kTab / kBlock blocks (every lane a node; the whole wavefront
// takes part in the MFMAs)
__global__ __launch_bounds__(kBlock) void k_mlp_tab_nodes(const float* __restrict__ Q, float* __restrict__ nodes) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  const int i = g / kTab, j = g - i * kTab;
  const float step = 2.0f * kTabZ / (float)(kTab - 1);
  float y0, y1;
  mlp_wave_mfma(Q, fmaf(step, (float)i, -kTabZ), fmaf(step, (float)j, -kTabZ), y0, y1);
  nodes[2 * g] = y0;
  nodes[2 * g + 1] = y1;
}

__global__ __launch_bounds__(kBlock) void k_mlp_tab_cells(const float* __restrict__ nodes, float4* __restrict__ cells) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= kCells * kCells) return;
  const int i = c / kCells, j = c - i * kCells;
  const float* a = nodes + 2 * (i * kTab + j);  // (i, j)
  const float* b = a + 2;                       // (i, j + 1)
  const float* d = a + 2 * kTab;                // (i + 1, j)
  const float* e = d + 2;                       // (i + 1, j + 1)
  cells[2 * c] = make_float4(a[0], d[0] - a[0], b[0] - a[0], (e[0] - d[0]) - (b[0] - a[0]));
  cells[2 * c + 1] = make_float4(a[1], d[1] - a[1], b[1] - a[1], (e[1] - d[1]) - (b[1] - a[1]));
}

__global__ __launch_bounds__(kBlock) void k_mlp_forward_table(const float* __restrict__ Q,
                                                              const float4* __restrict__ cells, int64_t n,
                                                              const float* __restrict__ v,
                                                              const float* __restrict__ x, float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float z0, z1, y0, y1;
  mlp_features_q(Q, v[i], x[i], z0, z1);
  mlp_table(cells, z0, z1, y0, y1);
  y[2 * i] = y0;
  y[2 * i + 1] = y1;
}

// Fused: network (f16 MFMA, or its table with TAB) -> bracket -> checked FP32
// bins -> outputs, or the element index onto the worklist (count at work[0],
// indices from work[1]).
template <bool GRAD, int NB, bool TAB>
__global__ __launch_bounds__(kBlock) void k_logk_mlp(const float* __restrict__ Q, const float4* __restrict__ cells,
                                                     int64_t n, int nbins,
                                                     const float* __restrict__ vin, const float* __restrict__ xin,
                                                     const float* __restrict__ gout, float* __restrict__ logk,
                                                     float* __restrict__ dv, float* __restrict__ dx,
                                                     float* __restrict__ t0o, float* __restrict__ t1o,
                                                     float* __restrict__ tpo, float* __restrict__ gpo,
                                                     uint8_t* __restrict__ fb, int* __restrict__ work) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int nb = NB > 0 ? NB : nbins;
  const bool in = i < n;
  const float vs = in ? vin[i] : 1.0f;
  const float xf = in ? xin[i] : 1.0f;
  double lk = 0.0, dvv = 0.0, dxv = 0.0;
  const bool special = in && domain_special((double)vs, (double)xf, lk, dvv, dxv);
  // the whole wavefront takes part in the network
  float z0 = 0.0f, z1 = 0.0f;
  if (in && !special) mlp_features_q(Q, vs, xf, z0, z1);
  float y0, y1;
  if constexpr (TAB) mlp_table(cells, z0, z1, y0, y1);
  else mlp_wave_mfma(Q, z0, z1, y0, y1);
  bool ok = true;
  LearnedBracket lb{};
  if (in && !special) {
    const float v = fabsf(vs);
    BinSums s;
    ok = learned_bins<GRAD ? 1 : 0>(Q, (double)v, (double)xf, y0, y1, nb, lb, s);
    if (ok) {
      const double h = ((double)lb.t1 - (double)lb.t0) / (double)nb;
      const double rS0 = rcp_of<false>(s.S0);
      lk = (double)lb.G + log_of<false>(h * s.S0);
      if (GRAD) {
        dvv = (v == 0.0f) ? 0.0 : copysign(s.Sv * rS0, (double)vs);
        dxv = -s.Sx * rS0;
      }
    }
  }
  // compaction of the failures: the block's wavefronts count theirs in LDS
  // and one atomic per block (not per wavefront: a single global counter
  // serialises its atomics, which costs as much as the kernel itself when a
  // few percent of the elements fail) reserves the block's stretch of the list
  __shared__ int s_count, s_base;
  const bool fail = in && !special && !ok;
  const unsigned long long mask = __ballot(fail);
  const int lane = threadIdx.x & 63;
  if (threadIdx.x == 0) s_count = 0;
  __syncthreads();
  int woff = 0;
  if (lane == 0 && mask) woff = atomicAdd(&s_count, __popcll(mask));
  woff = __shfl(woff, 0);
  __syncthreads();
  if (threadIdx.x == 0 && s_count > 0) s_base = atomicAdd(work, s_count);
  __syncthreads();
  if (fail) work[1 + s_base + woff + __popcll(mask & ((1ULL << lane) - 1ULL))] = (int)i;
  if (!in) return;
  if (fb) fb[i] = fail ? 1 : 0;
  if (fail) return;
  if (logk) logk[i] = (float)lk;
  if (GRAD) {
    if (gout) {
      const double go = (double)gout[i];
      dvv *= go;
      dxv *= go;
    }
    dv[i] = (float)dvv;
    dx[i] = (float)dxv;
  }
  if (t0o) {
    t0o[i] = special ? __builtin_nanf("") : lb.t0;
    t1o[i] = special ? __builtin_nanf("") : lb.t1;
    if (tpo) tpo[i] = special ? __builtin_nanf("") : lb.tg;
    if (gpo) gpo[i] = special ? __builtin_nanf("") : lb.G;
  }
}

// Persistent fallback over the worklist: the Newton path of k_logk<float>,
// element by element.  Every lane leaves when the list is exhausted.
template <bool GRAD, int NB>
__global__ __launch_bounds__(kBlock) void k_logk_fallback(int nbins, const int* __restrict__ work,
                                                          const float* __restrict__ vin, const float* __restrict__ xin,
                                                          const float* __restrict__ gout, float* __restrict__ logk,
                                                          float* __restrict__ dv, float* __restrict__ dx,
                                                          float* __restrict__ t0o, float* __restrict__ t1o,
                                                          float* __restrict__ tpo, float* __restrict__ gpo) {
  const int64_t count = work[0];
  const int nb = NB > 0 ? NB : nbins;
  // 64-bit: with every element on the list, k + stride can pass 2^31
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < count; k += (int64_t)gridDim.x * kBlock) {
    const int64_t i = work[1 + k];
    const double vs = (double)vin[i];
    const double x = (double)xin[i];
    const double v = fabs(vs);
    const Bracket b = find_bracket<false>(v, x, kMarginF32);
    if (t0o) {
      t0o[i] = b.t0;
      t1o[i] = b.t1;
      if (tpo) tpo[i] = b.tp;
      if (gpo) gpo[i] = (float)b.G;
      if (!logk && !dv) continue;
    }
    const BinSums s = bins_f32<GRAD>(nb, v, x, b.G, (double)b.t0, (double)b.t1);
    const double h = ((double)b.t1 - (double)b.t0) / (double)nb;
    const double rS0 = rcp_of<false>(s.S0);
    if (logk) logk[i] = (float)(b.G + log_of<false>(h * s.S0));
    if (GRAD) {
      double dvv = (v == 0.0) ? 0.0 : copysign(s.Sv * rS0, vs);
      double dxv = -s.Sx * rS0;
      if (gout) {
        const double go = (double)gout[i];
        dvv *= go;
        dxv *= go;
      }
      dv[i] = (float)dvv;
      dx[i] = (float)dxv;
    }
  }
}

__global__ void k_zero_int(int* p) { *p = 0; }

}  // namespace bk

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------
struct bessel_mlp {
  float* params = nullptr;  // [kNP]
  float* packed = nullptr;  // [kNQ] inference operands derived from params
  bool packed_stale = true; // params changed since the last k_mlp_pack
  float* tab_nodes = nullptr;     // [2 kTab^2] network outputs on the grid (range mode table)
  int64_t cap_tab_nodes = 0;
  float4* tab_cells = nullptr;    // [2 kCells^2] bilinear records
  int64_t cap_tab_cells = 0;
  bool table_stale = true;  // packed operands rebuilt since the table was
  float* adam_m = nullptr;  // [kNW]
  float* adam_s = nullptr;  // [kNW]
  float* grad = nullptr;    // [kNW + 1] (last: loss)
  float* partial = nullptr;
  int64_t cap_partial_blocks = 0;
  float* labels = nullptr;  // [2 * cap_labels]
  int64_t cap_labels = 0;
  float* losses = nullptr;  // [cap_losses]
  int64_t cap_losses = 0;
  int* work = nullptr;  // [1 + cap_work]
  int64_t cap_work = 0;
  int64_t adam_step = 0;
};

using namespace bk;

namespace {

int hip_fail(hipError_t e, const char* what) {
  return set_error(BESSEL_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Grow a device buffer (contents not preserved).  Stream-ordered so the hot
// path never synchronises; the old buffer is released after prior work.
template <typename T>
int ensure(T*& p, int64_t& cap, int64_t need, hipStream_t st, const char* what) {
  if (need <= cap && p) return BESSEL_OK;
  if (p) {
    hipError_t e = hipFreeAsync(p, st);
    if (e != hipSuccess) return hip_fail(e, what);
    p = nullptr;
    cap = 0;
  }
  hipError_t e = hipMallocAsync((void**)&p, (size_t)need * sizeof(T), st);
  if (e != hipSuccess) return hip_fail(e, what);
  cap = need;
  return BESSEL_OK;
}

}  // namespace

extern "C" int bessel_mlp_create(const float* params, int64_t nparams, bessel_mlp** out) {
  if (!out) return set_error(BESSEL_ERR_ARG, "out must be non-NULL");
  *out = nullptr;
  if (params && nparams != kNP) return set_error(BESSEL_ERR_ARG, "nparams must be %d", kNP);
  bessel_mlp* m = new (std::nothrow) bessel_mlp();
  if (!m) return set_error(BESSEL_ERR_ARG, "out of host memory");
  hipError_t e = hipMalloc((void**)&m->params, kNP * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&m->packed, kNQ * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&m->adam_m, kNW * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&m->adam_s, kNW * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&m->grad, (kNW + 1) * sizeof(float));
  // the network's table (2.6 MB) is allocated here, so that building it later
  // (on the first call in the table mode after a parameter change) allocates
  // nothing
  if (e == hipSuccess) e = hipMalloc((void**)&m->tab_nodes, (size_t)2 * kTab * kTab * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&m->tab_cells, (size_t)2 * kCells * kCells * sizeof(float4));
  if (e == hipSuccess) {
    m->cap_tab_nodes = (int64_t)2 * kTab * kTab;
    m->cap_tab_cells = (int64_t)2 * kCells * kCells;
  }
  if (e == hipSuccess) e = hipMemset(m->adam_m, 0, kNW * sizeof(float));
  if (e == hipSuccess) e = hipMemset(m->adam_s, 0, kNW * sizeof(float));
  if (e == hipSuccess) {
    if (params) {
      e = hipMemcpy(m->params, params, kNP * sizeof(float), hipMemcpyHostToDevice);
    } else {
      float host[kNP];
      memset(host, 0, sizeof(host));
      host[oMeta + 1] = 1.0f;
      host[oMeta + 3] = 1.0f;
      e = hipMemcpy(m->params, host, sizeof(host), hipMemcpyHostToDevice);
    }
  }
  if (e != hipSuccess) {
    int rc = hip_fail(e, "bessel_mlp_create");
    bessel_mlp_destroy(m);
    return rc;
  }
  *out = m;
  return BESSEL_OK;
}

extern "C" int bessel_mlp_destroy(bessel_mlp* m) {
  if (!m) return BESSEL_OK;
  (void)hipDeviceSynchronize();
  void* sync_ptrs[] = {m->params, m->packed, m->adam_m, m->adam_s, m->grad, m->tab_nodes, m->tab_cells};
  for (void* p : sync_ptrs)
    if (p) (void)hipFree(p);
  void* async_ptrs[] = {m->partial, m->labels, m->losses, m->work};  // hipMallocAsync
  for (void* p : async_ptrs)
    if (p) (void)hipFreeAsync(p, nullptr);
  (void)hipDeviceSynchronize();
  delete m;
  return BESSEL_OK;
}

extern "C" int bessel_mlp_set_params(bessel_mlp* m, const float* params, int64_t nparams) {
  if (!m || !params) return set_error(BESSEL_ERR_ARG, "mlp and params must be non-NULL");
  if (nparams != kNP) return set_error(BESSEL_ERR_ARG, "nparams must be %d", kNP);
  hipError_t e = hipMemcpy(m->params, params, kNP * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->adam_m, 0, kNW * sizeof(float));
  if (e == hipSuccess) e = hipMemset(m->adam_s, 0, kNW * sizeof(float));
  if (e != hipSuccess) return hip_fail(e, "bessel_mlp_set_params");
  m->adam_step = 0;
  m->packed_stale = true;
  return BESSEL_OK;
}

extern "C" int bessel_mlp_get_params(const bessel_mlp* m, float* params, int64_t nparams) {
  if (!m || !params) return set_error(BESSEL_ERR_ARG, "mlp and params must be non-NULL");
  if (nparams != kNP) return set_error(BESSEL_ERR_ARG, "nparams must be %d", kNP);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(params, m->params, kNP * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "bessel_mlp_get_params");
  return BESSEL_OK;
}

// Per-block partial gradients of a batch (k_mlp_grad); returns the block count.
static int launch_partials(bessel_mlp* m, int64_t n, int64_t batch, int sampled, uint64_t seed, int64_t step,
                           const float* v, const float* x, const float* t0, const float* t1, float alpha,
                           hipStream_t st, int64_t& nblocks) {
  nblocks = (batch + kTB - 1) / kTB;
  int rc = ensure(m->partial, m->cap_partial_blocks, nblocks * (kNW + 1), st, "partial gradients");
  if (rc) return rc;
  k_mlp_grad<<<dim3((unsigned)nblocks), kTT, 0, st>>>(m->params, n, batch, sampled, seed, step, v, x, t0, t1,
                                                      alpha, m->partial);
  return check_launch("k_mlp_grad");
}

static int launch_grad(bessel_mlp* m, int64_t n, int64_t batch, int sampled, uint64_t seed, int64_t step,
                       const float* v, const float* x, const float* t0, const float* t1, float alpha,
                       hipStream_t st) {
  int64_t nblocks = 0;
  int rc = launch_partials(m, n, batch, sampled, seed, step, v, x, t0, t1, alpha, st, nblocks);
  if (rc) return rc;
  k_mlp_reduce<<<dim3((kNW + 1 + kBlock - 1) / kBlock), kBlock, 0, st>>>(m->partial, (int)nblocks, m->grad,
                                                                        m->grad + kNW);
  return check_launch("k_mlp_reduce");
}

extern "C" int bessel_mlp_loss_grad(bessel_mlp* m, int64_t n, const float* v, const float* x, const float* t0,
                                    const float* t1, float alpha, float* loss, float* grad, void* hip_stream) {
  if (!m || !v || !x || !t0 || !t1 || !loss || !grad) return set_error(BESSEL_ERR_ARG, "NULL argument");
  if (n <= 0 || n > (1LL << 30)) return set_error(BESSEL_ERR_ARG, "n = %lld outside [1, 2^30]", (long long)n);
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = launch_grad(m, n, n, 0, 0, 0, v, x, t0, t1, alpha, st);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(grad, m->grad, kNW * sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(loss, m->grad + kNW, sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "bessel_mlp_loss_grad");
  return BESSEL_OK;
}

extern "C" int bessel_mlp_train(bessel_mlp* m, const bessel_mlp_train_cfg* cfg, int64_t n, const float* v,
                                const float* x, float* loss_host, void* hip_stream) {
  if (!m || !cfg || !v || !x) return set_error(BESSEL_ERR_ARG, "NULL argument");
  if (n <= 0 || n > (1LL << 30)) return set_error(BESSEL_ERR_ARG, "n = %lld outside [1, 2^30]", (long long)n);
  if (cfg->steps < 0 || cfg->batch <= 0 || cfg->batch > (1LL << 24))
    return set_error(BESSEL_ERR_ARG, "steps must be >= 0 and batch in [1, 2^24]");
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = ensure(m->labels, m->cap_labels, 2 * n, st, "labels");
  if (rc) return rc;
  rc = ensure(m->losses, m->cap_losses, cfg->steps > 0 ? cfg->steps : 1, st, "losses");
  if (rc) return rc;
  float* t0 = m->labels;
  float* t1 = m->labels + n;
  dim3 grid;
  rc = grid_for(n, grid);
  if (rc) return rc;
  k_mlp_labels<<<grid, kBlock, 0, st>>>(n, v, x, t0, t1);
  rc = check_launch("k_mlp_labels");
  if (rc) return rc;
  // two launches per step: partial gradients, then the ordered reduction
  // fused with the Adam update (which also records the step's loss)
  for (int64_t k = 0; k < cfg->steps; ++k) {
    int64_t nblocks = 0;
    rc = launch_partials(m, n, cfg->batch, 1, cfg->seed, k, v, x, t0, t1, cfg->alpha, st, nblocks);
    if (rc) return rc;
    // exponential decay from lr to lr_final over the run
    const double frac = cfg->steps > 1 ? (double)k / (double)(cfg->steps - 1) : 0.0;
    const float lr = (float)(cfg->lr * pow((double)cfg->lr_final / (double)cfg->lr, frac));
    m->adam_step += 1;
    k_mlp_reduce_adam<<<dim3((kNW + 1 + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        m->partial, (int)nblocks, m->params, m->adam_m, m->adam_s, m->adam_step, lr, cfg->beta1, cfg->beta2,
        cfg->adam_eps, m->losses + k);
    m->packed_stale = true;
    rc = check_launch("k_mlp_reduce_adam");
    if (rc) return rc;
  }
  if (loss_host && cfg->steps > 0) {
    hipError_t e = hipMemcpyAsync(loss_host, m->losses, cfg->steps * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "loss readback");
  }
  return BESSEL_OK;
}

extern "C" int bessel_mlp_adam_step(bessel_mlp* m, const float* grad, float lr, float beta1, float beta2, float eps,
                                    void* hip_stream) {
  if (!m || !grad) return set_error(BESSEL_ERR_ARG, "NULL argument");
  hipStream_t st = (hipStream_t)hip_stream;
  m->adam_step += 1;
  m->packed_stale = true;
  k_mlp_adam<<<dim3((kNW + kBlock - 1) / kBlock), kBlock, 0, st>>>(m->params, grad, m->adam_m, m->adam_s,
                                                                   m->adam_step, lr, beta1, beta2, eps);
  return check_launch("k_mlp_adam");
}

// Rebuild the inference operands on the caller's stream if the parameters
// changed since they were last built.
static int refresh_packed(const bessel_mlp* mc, hipStream_t st) {
  bessel_mlp* m = const_cast<bessel_mlp*>(mc);
  if (!m->packed_stale) return BESSEL_OK;
  k_mlp_pack<<<1, kBlock, 0, st>>>(m->params, m->packed);
  const int rc = check_launch("k_mlp_pack");
  if (rc == BESSEL_OK) {
    m->packed_stale = false;
    m->table_stale = true;
  }
  return rc;
}

// Rebuild the network's table (after the operands) on the caller's stream if
// the operands changed since it was last built.
static int refresh_table(const bessel_mlp* mc, hipStream_t st) {
  bessel_mlp* m = const_cast<bessel_mlp*>(mc);
  int rc = refresh_packed(m, st);
  if (rc || !m->table_stale) return rc;
  if (!m->tab_nodes || !m->tab_cells) return set_error(BESSEL_ERR_ARG, "the handle has no table buffers");
  static_assert((kTab * kTab) % kBlock == 0, "the node grid fills whole blocks");
  k_mlp_tab_nodes<<<kTab * kTab / kBlock, kBlock, 0, st>>>(m->packed, m->tab_nodes);
  rc = check_launch("k_mlp_tab_nodes");
  if (rc) return rc;
  k_mlp_tab_cells<<<(kCells * kCells + kBlock - 1) / kBlock, kBlock, 0, st>>>(m->tab_nodes, m->tab_cells);
  rc = check_launch("k_mlp_tab_cells");
  if (rc == BESSEL_OK) m->table_stale = false;
  return rc;
}

namespace bk {

int mlp_table_operands(const bessel_mlp* m, hipStream_t st, const float** Q, const float4** cells) {
  const int rc = refresh_table(m, st);
  if (rc) return rc;
  *Q = m->packed;
  *cells = m->tab_cells;
  return BESSEL_OK;
}

}  // namespace bk

extern "C" int bessel_mlp_forward(const bessel_mlp* m, int64_t n, const float* v, const float* x, float* y, int mode,
                                  void* hip_stream) {
  if (!m || (n > 0 && (!v || !x || !y))) return set_error(BESSEL_ERR_ARG, "NULL argument");
  if (mode < 0 || mode > 2) return set_error(BESSEL_ERR_ARG, "mode must be 0 (FP32), 1 (f16 MFMA) or 2 (table)");
  if (n == 0) return BESSEL_OK;
  dim3 grid;
  int rc = grid_for(n, grid);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  if (mode == 0) {
    k_mlp_forward_f32<<<grid, kBlock, 0, st>>>(m->params, n, v, x, y);
  } else if (mode == 1) {
    rc = refresh_packed(m, st);
    if (rc) return rc;
    k_mlp_forward_mfma<<<grid, kBlock, 0, st>>>(m->packed, n, v, x, y);
  } else {
    rc = refresh_table(m, st);
    if (rc) return rc;
    k_mlp_forward_table<<<grid, kBlock, 0, st>>>(m->packed, m->tab_cells, n, v, x, y);
  }
  return check_launch("k_mlp_forward");
}

namespace bk {

// Fused learned-range pass + fallback (shared by logk, logk_dv_dx and range).
template <bool GRAD, bool TAB>
static void launch_fused(dim3 grid, hipStream_t st, const bessel_mlp* m, int64_t n, int nbins, const float* v,
                         const float* x, const float* go, float* lk, float* dv, float* dx, float* t0, float* t1,
                         float* tp, float* gp, uint8_t* fb) {
  const float4* cells = TAB ? m->tab_cells : nullptr;
  switch (nbins) {
    case 64:
      k_logk_mlp<GRAD, 64, TAB><<<grid, kBlock, 0, st>>>(m->packed, cells, n, nbins, v, x, go, lk, dv, dx, t0, t1,
                                                         tp, gp, fb, m->work);
      break;
    case 128:
      k_logk_mlp<GRAD, 128, TAB><<<grid, kBlock, 0, st>>>(m->packed, cells, n, nbins, v, x, go, lk, dv, dx, t0, t1,
                                                          tp, gp, fb, m->work);
      break;
    case 256:
      k_logk_mlp<GRAD, 256, TAB><<<grid, kBlock, 0, st>>>(m->packed, cells, n, nbins, v, x, go, lk, dv, dx, t0, t1,
                                                          tp, gp, fb, m->work);
      break;
    default:
      k_logk_mlp<GRAD, 0, TAB><<<grid, kBlock, 0, st>>>(m->packed, cells, n, nbins, v, x, go, lk, dv, dx, t0, t1,
                                                        tp, gp, fb, m->work);
      break;
  }
}

template <bool GRAD>
static int run_mlp(int64_t n, const float* v, const float* x, const float* go, float* lk, float* dv, float* dx,
                   float* t0, float* t1, float* tp, float* gp, uint8_t* fb, int nbins, const bessel_mlp* mc,
                   bool table, hipStream_t st) {
  bessel_mlp* m = const_cast<bessel_mlp*>(mc);
  dim3 grid;
  int rc = grid_for(n, grid);
  if (rc) return rc;
  if (n > 0x7fffffffLL - 1) return set_error(BESSEL_ERR_ARG, "n too large for the learned-range worklist");
  rc = ensure(m->work, m->cap_work, n + 1, st, "worklist");
  if (rc) return rc;
  rc = table ? refresh_table(m, st) : refresh_packed(m, st);
  if (rc) return rc;
  k_zero_int<<<1, 1, 0, st>>>(m->work);
  if (table)
    launch_fused<GRAD, true>(grid, st, m, n, nbins, v, x, go, lk, dv, dx, t0, t1, tp, gp, fb);
  else
    launch_fused<GRAD, false>(grid, st, m, n, nbins, v, x, go, lk, dv, dx, t0, t1, tp, gp, fb);
  rc = check_launch("k_logk_mlp");
  if (rc) return rc;
  // persistent fallback grid: 4 blocks per CU, fewer for small batches (the
  // worklist never holds more than n elements)
  const dim3 fgrid((unsigned)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock));
  switch (nbins) {
    case 64:
      k_logk_fallback<GRAD, 64><<<fgrid, kBlock, 0, st>>>(nbins, m->work, v, x, go, lk, dv, dx, t0, t1, tp, gp);
      break;
    case 128:
      k_logk_fallback<GRAD, 128><<<fgrid, kBlock, 0, st>>>(nbins, m->work, v, x, go, lk, dv, dx, t0, t1, tp, gp);
      break;
    case 256:
      k_logk_fallback<GRAD, 256><<<fgrid, kBlock, 0, st>>>(nbins, m->work, v, x, go, lk, dv, dx, t0, t1, tp, gp);
      break;
    default:
      k_logk_fallback<GRAD, 0><<<fgrid, kBlock, 0, st>>>(nbins, m->work, v, x, go, lk, dv, dx, t0, t1, tp, gp);
      break;
  }
  return check_launch("k_logk_fallback");
}

int logk_mlp(int64_t n, const float* v, const float* x, const float* go, float* lk, float* dv, float* dx, int nbins,
             bool grad, const bessel_mlp* mlp, bool table, hipStream_t st) {
  // Small batches (at most the split threshold) run the Newton bracket on the
  // 16-lanes-per-element layout, one launch: there one lane per element
  // leaves most of the chip idle, and the predictor saves nothing; the
  // handle's fallback count reads 0 afterwards.
  if (n <= split_threshold())
    return logk_newton(BESSEL_F32, n, v, x, go, lk, dv, dx, nbins, grad, st, mlp->work, true);
  if (grad)
    return run_mlp<true>(n, v, x, go, lk, dv, dx, nullptr, nullptr, nullptr, nullptr, nullptr, nbins, mlp, table, st);
  return run_mlp<false>(n, v, x, nullptr, lk, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nbins, mlp,
                        table, st);
}

int range_mlp(int64_t n, const float* v, const float* x, float* t0, float* t1, float* tp, float* gpk,
              uint8_t* fallback, const bessel_mlp* mlp, bool table, hipStream_t st) {
  return run_mlp<false>(n, v, x, nullptr, nullptr, nullptr, nullptr, t0, t1, tp, gpk, fallback, 128, mlp, table, st);
}

}  // namespace bk

extern "C" int bessel_mlp_fallback_count(const bessel_mlp* m, int* count_host) {
  if (!m || !count_host) return set_error(BESSEL_ERR_ARG, "NULL argument");
  if (!m->work) {
    *count_host = 0;
    return BESSEL_OK;
  }
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(count_host, m->work, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "bessel_mlp_fallback_count");
  return BESSEL_OK;
}
