// bessel_learned.hpp -- the learned bracket on the device: the network's
// features, its bilinear table, the shift and the check of a predicted
// bracket, shared by the fused learned-range kernels (bessel_mlp.hip) and the
// per-set sums (bessel_gh.hip).
//
// The predictor's outputs (y0, y1) approximate (t0 / t1, log t1) of the
// method's bracket (Section 2.1, Eq. (7)-(8), as Sections 2.2-2.3 find it);
// every predicted bracket is integrated with the checked FP32 bins and
// accepted only if its end terms are below eps of the shift and its even and
// odd node sums agree, so correctness never rests on the network.
#pragma once

#include "bessel_device.hpp"

namespace bk {

constexpr float kVFloor = 1e-3f;

// Header of the packed inference operands (k_mlp_pack): the features'
// affine maps z0 = log2 max(|v|, kVFloor) * Q[0] + Q[1], z1 = log2 x * Q[2] +
// Q[3], then e^{margin_t1}, margin_t0, and the output biases.
constexpr int qHdr = 0;

__device__ __forceinline__ void mlp_features_q(const float* __restrict__ Q, float v, float x, float& z0, float& z1) {
  z0 = fmaf(hlog2(fmaxf(fabsf(v), kVFloor)), Q[qHdr + 0], Q[qHdr + 1]);
  z1 = fmaf(hlog2(x), Q[qHdr + 2], Q[qHdr + 3]);
}

// The network's table (range mode BESSEL_RANGE_MLP_TABLE): kTab x kTab nodes
// on z in [-kTabZ, kTabZ]^2, per cell the bilinear coefficients of both
// outputs (value, d/du, d/dw, d2/dudw) in one 32-byte record.
constexpr int kTab = 256;
constexpr float kTabZ = 4.0f;
constexpr int kCells = kTab - 1;

// Bilinear lookup; features outside the table are clamped to its edge (their
// brackets are then usually rejected by the check and recomputed).
__device__ __forceinline__ void mlp_table(const float4* __restrict__ cells, float z0, float z1, float& y0,
                                          float& y1) {
  const float s = (float)(kTab - 1) / (2.0f * kTabZ);
  const float u = fminf(fmaxf((z0 + kTabZ) * s, 0.0f), (float)kCells - 1e-3f);
  const float w = fminf(fmaxf((z1 + kTabZ) * s, 0.0f), (float)kCells - 1e-3f);
  const int i = (int)u, j = (int)w;
  const float fu = u - (float)i, fw = w - (float)j;
  const float4 r0 = cells[2 * (i * kCells + j)];
  const float4 r1 = cells[2 * (i * kCells + j) + 1];
  y0 = fmaf(fw, fmaf(fu, r0.w, r0.z), fmaf(fu, r0.y, r0.x));
  y1 = fmaf(fw, fmaf(fu, r1.w, r1.z), fmaf(fu, r1.y, r1.x));
}

// g at one point for the shift of a learned bracket, FP32 hardware form.  Any
// finite shift is exact (log K = G + log(h S0) with S0 relative to the same
// G); inside the bracket g >= max g - L, so the exponents stay below L and
// FP32 cannot overflow.
__device__ __forceinline__ float shift_at(float v, float x, float t) {
  const float e = hexp2(kLog2eF * t);
  return log_cosh_f32(v * t) - 0.5f * x * (e + hrcp(e));
}

// Acceptance of a learned bracket after its bins (all relative to e^{G}):
//   coverage   the end terms are at most eps_32 (t0 = 0 needs no lower test);
//              since G <= max g, this bounds g at the ends by max g + log eps;
//   resolution the even-node and odd-node rules (step 2h) agree to 1e-5, so
//              the full rule's error is far below FP32 resolution;
//   finiteness of every sum.
__device__ __forceinline__ bool accept_bins(const BinSums& s, float t0) {
  const float tau = 1.1920929e-07f;
  const bool cover = (t0 == 0.0f || s.term0 <= tau) && s.termN <= tau;
  const bool resolved = fabs(s.Seven - s.Sodd) <= 1e-5 * 0.5 * (s.Seven + s.Sodd);
  return cover && resolved && isfinite(s.S0) && s.S0 > 0.0;
}

// A learned bracket from the network's outputs (y0, y1) for v >= 0 and finite
// x > 0, with its shift and its checked FP32 bins (DER as bins_f32).  The
// bracket and the shift are computed from v and x rounded to FP32; the bins
// take v and x as given.
//   t0 = max(0, y0 - margin_t0) e^{y1},  t1 = e^{y1} e^{margin_t1};
//   G = g(tg), tg the best of the bracket's midpoint, asinh(v/x) (the peak
//   when v t_p >> 1) clamped into the bracket and, when t0 = 0, 0 (g(0) = -x).
// Returns true when the bracket passed accept_bins; s then holds its sums.
struct LearnedBracket {
  float t0, t1, tg, G;
};

template <int DER>
__device__ __forceinline__ bool learned_bins(const float* __restrict__ Q, double vd, double xd, float y0, float y1,
                                             int nb, LearnedBracket& lb, BinSums& s) {
  const float v = (float)vd, x = (float)xd;
  const float t1r = hexp2(kLog2eF * y1);  // predicted t1 before widening
  lb.t0 = fmaxf(0.0f, y0 - Q[qHdr + 5]) * t1r;
  lb.t1 = t1r * Q[qHdr + 4];
  const float r = fminf(v * hrcp(x), 1e18f);
  const float ta = fminf(fmaxf(kLn2F * hlog2(r + hsqrt(fmaf(r, r, 1.0f))), lb.t0), lb.t1);
  const float tm = 0.5f * (lb.t0 + lb.t1);
  const float gm = shift_at(v, x, tm), ga = shift_at(v, x, ta);
  lb.G = fmaxf(gm, ga);
  lb.tg = (ga >= gm) ? ta : tm;
  if (lb.t0 == 0.0f && -x > lb.G) {
    lb.G = -x;
    lb.tg = 0.0f;
  }
  if (!(isfinite(lb.t1) && lb.t1 > lb.t0 && isfinite(lb.G))) return false;
  s = bins_f32<DER, true>(nb, vd, xd, (double)lb.G, (double)lb.t0, (double)lb.t1);
  return accept_bins(s, lb.t0);
}

}  // namespace bk
