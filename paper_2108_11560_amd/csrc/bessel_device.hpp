// bessel_device.hpp -- gfx950 device code for log K_v(x): arithmetic helpers,
// the bracket finder and the fixed-bin log-space trapezoid.
//
// Method: Takekawa, arXiv 2108.11560.
//   Section 2, Eq. (1)-(2):   K_v(x) = int_0^inf cosh(v t) exp(-x cosh t) dt
//   Section 2.1, Eq. (3)-(5): g(t) = log cosh(v t) - x cosh t, g', g''
//   Section 2.1, Eq. (7)-(8): truncation set {t : g(t) >= g(t_p) + log eps}
//   Section 2.2-2.3:          peak t_p and the ends t0, t1
//   Section 2.4, Eq. (9)-(11), Eq. (int): n-bin trapezoid, summed relative to g(t_p)
//   Section 4.1, Eq. (13):    d/dv and d/dx integrands
//
// Precision layout, chosen for gfx950 rates (FP64 FMA at the full vector rate,
// FP32 exp2/log2/rcp/sqrt at half rate, no FP64 transcendentals in hardware):
//   - bracket search (t_p, t0, t1): FP32 hardware transcendentals, with one
//     extra nat of margin that absorbs their rounding; every returned end is on
//     the outside of its crossing, so the bracket is a superset;
//   - the shift G ~ g(t_p): any finite value gives the same log K (it is
//     subtracted in every node's exponent and added back to log K), so it is
//     formed in FP32 arithmetic, with x subtracted exactly in FP64;
//   - per-bin argument g(t_m) - G: FP64, from linear recurrences (e^{t_m} - 1
//     and 1 - e^{-t_m}, or cosh t_m, and 1 - e^{-2 v t_m}), so no
//     transcendental is spent on them;
//   - per-bin exponential and sums: FP32 hardware exp2 (F32 path) or a
//     table-driven FP64 exp (F64 path), summed in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bk {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;
constexpr float kLog2eF = 1.44269504089f;
constexpr float kLn2F = 0.693147180560f;

// ---------------------------------------------------------------------------
// FP32 hardware transcendentals (v_exp_f32, v_log_f32, v_rcp_f32, v_sqrt_f32).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float hexp2(float a) { return __builtin_amdgcn_exp2f(a); }
__device__ __forceinline__ float hlog2(float a) { return __builtin_amdgcn_logf(a); }
__device__ __forceinline__ float hrcp(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ float hsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }

// ---------------------------------------------------------------------------
// FP64 elementary functions written for this kernel's argument ranges.
//
// exp: a = k ln2 + r with k = nearest integer to a log2(e), obtained by adding
// 1.5 * 2^52 (the sum's low mantissa bits are k); r = a - k ln2 with ln 2 split
// into its double rounding and the residual (Cody-Waite), each applied with a
// fused multiply-add; e^r by a degree-10 polynomial with minimax relative error
// 3.0e-16 on |r| <= ln2/2 (coefficients from gen_exp_poly.py); 2^k applied by
// ldexp.
// ---------------------------------------------------------------------------
constexpr double kLn2D = 6.93147180559945286227e-01;   // ln 2 rounded to double
constexpr double kLn2Lo = 2.31904681384629955842e-17;  // ln 2 - kLn2D
constexpr double kRoundMagic = 6755399441055744.0;     // 1.5 * 2^52

struct ExpParts {
  double em1;  // e^r - 1
  int k;       // e^a = 2^k (1 + em1)
};

__device__ __forceinline__ ExpParts exp_parts(double a) {
  a = fmax(a, -708.0);  // keeps 2^k normal; e^-708 is below every term that matters
  const double kd = fma(a, kLog2e, kRoundMagic);
  const double kf = kd - kRoundMagic;
  const double r = fma(-kf, kLn2Lo, fma(-kf, kLn2D, a));
  double p = 2.748844352290197e-07;
  p = fma(p, r, 2.7639768251354328e-06);
  p = fma(p, r, 2.480191768787707e-05);
  p = fma(p, r, 0.00019841171384225596);
  p = fma(p, r, 0.001388888849913829);
  p = fma(p, r, 0.008333333384665794);
  p = fma(p, r, 0.041666666668426014);
  p = fma(p, r, 0.16666666666557742);
  p = fma(p, r, 0.49999999999997286);
  p = fma(p, r, 1.0000000000000064);
  ExpParts e;
  e.em1 = p * r;
  e.k = __double2loint(kd);
  return e;
}

// x * 2^k (v_ldexp_f64: one full-rate operation, exact while the result is
// normal, which the callers' ranges keep it).
__device__ __forceinline__ double scale2k(double x, int k) { return __builtin_amdgcn_ldexp(x, k); }

__device__ __forceinline__ double exp_f64(double a) {
  const ExpParts e = exp_parts(a);
  return scale2k(1.0 + e.em1, e.k);
}

// e^a for the nodes of the FP64 bins, from a table: with K the nearest integer
// to 256 a log2(e), a = K ln2/256 + r and |r| <= ln2/512, so
//   e^a = 2^{floor(K/256)} 2^{(K mod 256)/256} e^r,
// the middle factor read from a 256-entry table in LDS (exp2_table, built by
// every block that uses it) and e^r by a degree-3 minimax polynomial (relative
// error 1.8e-14 on |r| <= ln2/512; gen_exp_poly.py 3 512).  One multiply and
// one ldexp apply the table entry and 2^k; the per-node cost is 12 VALU slots
// against 15 for a degree-9 polynomial on |r| <= ln2/2, at the same accuracy.
__shared__ double s_exp2_table[256];
// 2^{j/256} - 1 to full relative accuracy (expm1_pair_tab).
__shared__ double s_exp2m1_table[256];

// Every thread of a block calls it before any thread of the block reaches
// exp_node_f64 or expm1_pair_tab, then the block synchronises.  Blocks have
// kBlock = 256 threads, one entry each.
__device__ __forceinline__ void exp2_table_init() {
  const int j = threadIdx.x & 255;
  const ExpParts e = exp_parts((double)j * (kLn2D / 256.0));  // k = 0 for j < 128, 1 above
  const double T = scale2k(1.0 + e.em1, e.k);
  s_exp2_table[j] = T;
  s_exp2m1_table[j] = (e.k == 0) ? e.em1 : T - 1.0;  // T - 1 exact for T in [1, 2]
}

__device__ __forceinline__ double exp_node_f64(double a) {
  a = fmax(a, -708.0);
  const double kd = fma(a, 256.0 * kLog2e, kRoundMagic);
  const double kf = kd - kRoundMagic;
  const double r = fma(-kf, kLn2Lo / 256.0, fma(-kf, kLn2D / 256.0, a));
  double p = 0.1666666514027065;
  p = fma(p, r, 0.5000000763659442);
  p = fma(p, r, 1.0000000000000384);
  p = fma(p, r, 0.9999999999999825);
  const int K = __double2loint(kd);
  return scale2k(s_exp2_table[K & 255] * p, K >> 8);  // K >> 8 = floor(K / 256)
}

// 1 - e^{-z} for z >= 0 with relative accuracy as z -> 0.
__device__ __forceinline__ double one_minus_exp_neg(double z) {
  const ExpParts e = exp_parts(-z);
  return (e.k == 0) ? -e.em1 : 1.0 - scale2k(1.0 + e.em1, e.k);
}

// e^{-z} and 1 - e^{-z} from one exponential: bitwise exp_f64(-z) and
// one_minus_exp_neg(z).
struct ExpNeg {
  double q, om;
};

__device__ __forceinline__ ExpNeg exp_neg_pair(double z) {
  const ExpParts e = exp_parts(-z);
  const double q = scale2k(1.0 + e.em1, e.k);
  return {q, (e.k == 0) ? -e.em1 : 1.0 - q};
}

// 1/y: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp_f64(double y) {
  double r = __builtin_amdgcn_rcp(y);
  double e = fma(-y, r, 1.0);
  r = fma(r, e, r);
  e = fma(-y, r, 1.0);
  return fma(r, e, r);
}

// log y for finite y > 0 in the normal range: y = 2^e m with m in
// [sqrt(1/2), sqrt(2)), log m = 2 atanh(s), s = (m - 1)/(m + 1), |s| <= 0.1716,
// series in s^2 to s^22 (truncation < 1e-17 relative).
__device__ __forceinline__ double log_f64(double y) {
  int hi = __double2hiint(y);
  int e = (hi >> 20) - 1023;
  hi = (hi & 0x000fffff) | 0x3ff00000;  // m in [1, 2)
  if (hi > 0x3ff6a09e) {                 // m > sqrt(2): halve
    hi -= 0x00100000;
    e += 1;
  }
  const double m = __hiloint2double(hi, __double2loint(y));
  const double num = m - 1.0;
  const double den = m + 1.0;
  const double rd = rcp_f64(den);
  double s = num * rd;
  s = fma(fma(-den, s, num), rd, s);  // one correction step on the quotient
  const double s2 = s * s;
  double p = 1.0 / 23.0;
  p = fma(p, s2, 1.0 / 21.0);
  p = fma(p, s2, 1.0 / 19.0);
  p = fma(p, s2, 1.0 / 17.0);
  p = fma(p, s2, 1.0 / 15.0);
  p = fma(p, s2, 1.0 / 13.0);
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  const double lm = fma(2.0 * s * s2, p, 2.0 * s);
  return fma((double)e, kLn2D, lm);
}

// cosh t for t >= 0 from e^t and its reciprocal.
__device__ __forceinline__ double cosh_f64(double t) {
  const double E = exp_f64(t);
  return 0.5 * (E + rcp_f64(E));
}

// log cosh z for z >= 0: z + log(1 + e^{-2z}) - log 2 (absolute error ~1e-16 |z|).
__device__ __forceinline__ double log_cosh_f64(double z) {
  return z + log_f64(1.0 + exp_f64(-2.0 * z)) - kLn2;
}

// g_{v,x}(t) = log cosh(v t) - x cosh t (Eq. 3) in FP64; v >= 0, t >= 0.
__device__ __forceinline__ double g_f64(double v, double x, double t) {
  return log_cosh_f64(v * t) - x * cosh_f64(t);
}

// e^t - 1 and 1 - e^{-t} for t >= 0, each to a few ulp relative (also as
// t -> 0); their product is 2 (cosh t - 1).
struct Expm1Pair {
  double ep, em;  // e^t - 1 and 1 - e^{-t}
};

__device__ __forceinline__ Expm1Pair expm1_pair(double t) {
  const ExpParts e = exp_parts(t);
  const double m = (e.k == 0) ? e.em1 : scale2k(1.0 + e.em1, e.k) - 1.0;  // e^t >= e^{ln2/2} when k > 0
  return {m, m * rcp_f64(1.0 + m)};
}

// The same pair from the block's tables (exp2_table_init), for t >= 0: with
// K = round(256 t log2 e) = 256 k + j and |r| <= ln2/512 as in exp_node_f64,
// e^t = 2^k T_j e^r, and for k = 0 e^t - 1 = (T_j - 1) + T_j (e^r - 1) with
// T_j - 1 from its own table, so no term cancels; e^r - 1 by its Taylor
// polynomial of degree 5 (remainder below 1e-20 on |r| <= ln2/512).  For
// k >= 1, e^t >= 2 and e^t - 1 has no cancellation.  About 25 slots against
// 40 for expm1_pair.
__device__ __forceinline__ Expm1Pair expm1_pair_tab(double t) {
  const double kd = fma(t, 256.0 * kLog2e, kRoundMagic);
  const double kf = kd - kRoundMagic;
  const double r = fma(-kf, kLn2Lo / 256.0, fma(-kf, kLn2D / 256.0, t));
  double p = fma(r, 1.0 / 120.0, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  const double q = p * r;  // e^r - 1
  const int K = __double2loint(kd);
  const int j = K & 255, k = K >> 8;
  const double e0 = fma(s_exp2_table[j], q, s_exp2m1_table[j]);  // T_j e^r - 1
  const double m = (k == 0) ? e0 : scale2k(1.0 + e0, k) - 1.0;
  return {m, m * rcp_f64(1.0 + m)};
}

__device__ __forceinline__ double coshm1_f64(double t) {
  const Expm1Pair p = expm1_pair(t);
  return 0.5 * (p.ep * p.em);
}

// g(t) + x = log cosh(v t) - x (cosh t - 1), without the cancellation of
// x cosh t against x for large x.
__device__ __forceinline__ double g_plus_x_f64(double v, double x, double t) {
  return log_cosh_f64(v * t) - x * coshm1_f64(t);
}

// log cosh z for z >= 0, FP32 hardware form (absolute error ~1e-7 |z|).
__device__ __forceinline__ float log_cosh_f32(float z) {
  const float q = hexp2(-2.0f * kLog2eF * z);
  return z + (hlog2(1.0f + q) - 1.0f) * kLn2F;
}

// Domain conventions (see include/bessel.h).  Returns true when the element is
// outside v real, 0 < x < inf, or outside the range the FP32 bracket search
// represents; then logk, dv, dx hold the convention's values.
// Smallest x: the upper end solves x cosh t = L with L up to ~37 (FP64
// margin), so L / x must stay below the FP32 maximum.  Largest x: x itself
// and g(t_p) ~ -x must stay well inside the FP32 range.  Largest |v|: the
// search's margin for its own FP32 rounding grows as 1e-6 |g(t_p)| ~ 1e-6 v t_p,
// so the bracket's half-width stays near sqrt(2e-6 t_p) while the integrand's
// width 1/sqrt(v) shrinks; from |v| ~ 1e7 on, 128 bins no longer resolve it.
// Largest v / x: the upper end's acosh((...) / x) in the fixed-count search
// (which runs at every order) forms ~2 v / x in FP32, which overflows near
// 1.7e38.
// Finite inputs beyond these give NaN (documented in the header), as do NaN
// inputs and x < 0.
constexpr double kMinX = 1e-36;
constexpr double kMaxX = 1e36;
constexpr double kMaxV = 1e6;
constexpr double kMaxVoverX = 1.2e38;

__device__ __forceinline__ bool domain_special(double v, double x, double& logk, double& dv, double& dx) {
  const double nan_ = __builtin_nan("");
  const bool finite_v = !__builtin_isinf(v);
  const bool beyond = (x > 0.0 && x < kMinX) || (x > kMaxX && !__builtin_isinf(x)) ||
                      (finite_v && (fabs(v) > kMaxV || (x > 0.0 && fabs(v) > kMaxVoverX * x)));
  if (__builtin_isnan(v) || __builtin_isnan(x) || x < 0.0 || beyond) {
    logk = nan_; dv = nan_; dx = nan_;
    return true;
  }
  if (x == 0.0) {
    logk = __builtin_inf(); dv = nan_; dx = nan_;
    return true;
  }
  if (__builtin_isinf(x)) {
    logk = -__builtin_inf(); dv = nan_; dx = nan_;
    return true;
  }
  if (__builtin_isinf(v)) {
    logk = __builtin_inf(); dv = nan_; dx = nan_;
    return true;
  }
  return false;
}

// Final step of a path in the precision of its output: log(h S0) and 1/S0.
// FP32 outputs take the hardware log2 and reciprocal (errors of ~1 ulp of
// FP32, far below the FP32 bar); FP64 outputs the FP64 routines above.
template <bool F64>
__device__ __forceinline__ double log_of(double y) {
  if constexpr (F64) return log_f64(y);
  else return (double)(kLn2F * hlog2((float)y));
}

template <bool F64>
__device__ __forceinline__ double rcp_of(double y) {
  if constexpr (F64) return rcp_f64(y);
  else return (double)hrcp((float)y);
}

// ---------------------------------------------------------------------------
// Bracket (Sections 2.1-2.3), redesigned for fixed trip counts so a wavefront
// never waits on a slow lane.  All loops below have compile-time trip counts.
// ---------------------------------------------------------------------------
struct Bracket {
  double G;    // the shift: g(t_p) (see find_bracket for its arithmetic)
  double Gx;   // G + x, formed without cancellation (the FP64 bins' shift)
  float tp;    // peak location (at or to the right of the true peak)
  float t0;    // lower end (0, or at/left of the crossing)
  float t1;    // upper end (at/right of the crossing)
};

constexpr int kPeakIters = 4;   // Newton steps for t_p (g(t_p) within ~1e-4 nats of max g)
constexpr int kUpperIters = 2;  // fixed-point steps before the final Newton step for t1
constexpr int kLowerIters = 3;  // fixed-point steps for t0

// The x cosh t and x sinh t terms below are formed as x e^{t} = 2^{t log2 e +
// log2 x} and x e^{-t}, never as x times e^{t}: for x down to ~1e-30 the peak
// and the upper end sit near t = log(2v/x) ~ 70-90, where e^{t} alone would
// leave the FP32 range while x e^{t} stays moderate.  lx = log2 x.

// Peak t_p > 0 when v^2 > x (Section 2.1).  g' = v tanh(v t) - x sinh t is
// concave on t >= 0 (g''' <= 0), zero at 0 and at t_p, and g'(t) <= v - x sinh t
// < 0 for t > asinh(v/x).  Newton steps started at asinh(v/x), right of the
// root, on a concave function decreasing through the root stay right of it and
// decrease monotonically; each step is clamped to [0, t] so FP32 rounding can
// only stall it, never move it left of the root by more than the rounding.
__device__ __forceinline__ float peak_f32(float v, float x, float lx) {
  // asinh(r), r = v/x, without squaring r: log(r) + log(1 + sqrt(1 + 1/r^2))
  const float rr = x * hrcp(v);
  float t = kLn2F * (hlog2(v) - lx + hlog2(1.0f + hsqrt(fmaf(rr, rr, 1.0f))));
#pragma unroll
  for (int k = 0; k < kPeakIters; ++k) {
    const float q = hexp2(-2.0f * kLog2eF * v * t);  // e^{-2 v t}
    const float rq = hrcp(1.0f + q);
    const float th = (1.0f - q) * rq;                  // tanh(v t)
    const float sech2 = 4.0f * q * rq * rq;            // sech^2(v t)
    const float xe = hexp2(fmaf(kLog2eF, t, lx));      // x e^{t}
    const float xei = hexp2(fmaf(-kLog2eF, t, lx));    // x e^{-t}
    const float gp = v * th - 0.5f * (xe - xei);       // g'(t)   (Eq. 4)
    const float gpp = v * v * sech2 - 0.5f * (xe + xei);  // g''(t)  (Eq. 5), < 0 here
    const float tn = t - gp * hrcp(gpp);
    t = fminf(t, fmaxf(tn, 0.0f));
  }
  return t;
}

// Upper end t1: F(t) = g(t) - G + L is concave and decreasing beyond the peak.
// The map T(t) = acosh((log cosh(v t) - G + L) / x) is increasing, has t1 as
// its fixed point and contracts there (T'(t1) = v tanh(v t1) / (x sinh t1) < 1
// because g'(t1) < 0); from t_p, inside the bracket, its iterates increase
// toward t1.  A final Newton step from such an inside point of a concave F
// lands at or beyond the root, so the returned t1 is outside.
__device__ __forceinline__ float upper_f32(float v, float x, float lx, float tp, float G, float L) {
  const float rx = hrcp(x);
  float t = tp;
#pragma unroll
  for (int k = 0; k < kUpperIters; ++k) {
    const float y = fmaxf((log_cosh_f32(v * t) - G + L) * rx, 1.0f);
    // acosh(y) = log(y + sqrt(y - 1) sqrt(y + 1)): no y^2, which would
    // overflow for y > 1.8e19 (x below ~1e-18)
    t = kLn2F * hlog2(y + hsqrt(y - 1.0f) * hsqrt(y + 1.0f));
  }
  const float q = hexp2(-2.0f * kLog2eF * v * t);
  const float lc = v * t + (hlog2(1.0f + q) - 1.0f) * kLn2F;
  const float xe = hexp2(fmaf(kLog2eF, t, lx));
  const float xei = hexp2(fmaf(-kLog2eF, t, lx));
  const float F = lc - 0.5f * (xe + xei) - G + L;
  const float Fp = v * (1.0f - q) * hrcp(1.0f + q) - 0.5f * (xe - xei);
  const float tn = t - F * hrcp(Fp);
  // Fp < 0 strictly right of the peak; keep t if rounding made the step useless.
  return (Fp < 0.0f && tn >= t) ? tn : t;
}

// Lower end t0 > 0, used only when g(0) - G <= -L (Section 2.3).  The map
// U(t) = acosh(exp(x cosh t + G - L)) / v is increasing with fixed point t0;
// from t = 0 (outside, where F <= 0) its iterates increase toward t0 and stay
// outside, so every iterate is a valid lower end.
__device__ __forceinline__ float lower_f32(float v, float lx, float tp, float G, float L) {
  const float rv = hrcp(v);
  float t = 0.0f;
#pragma unroll
  for (int k = 0; k < kLowerIters; ++k) {
    const float xch = 0.5f * (hexp2(fmaf(kLog2eF, t, lx)) + hexp2(fmaf(-kLog2eF, t, lx)));  // x cosh t
    const float y = fmaxf(xch + (G - L), 0.0f);
    // acosh(e^y) = y + log(1 + sqrt(1 - e^{-2y}))
    const float s = hsqrt(fmaxf(1.0f - hexp2(-2.0f * kLog2eF * y), 0.0f));
    t = (y + kLn2F * hlog2(1.0f + s)) * rv;
  }
  return fminf(t, tp);
}

// Large orders (|v| above the validated 1e3, peak t_p > 0).  The steps of
// upper_f32 / lower_f32 move ~L / v per iteration while the bracket's
// half-width is ~sqrt(2 L / v), so for large v a fixed count of them stops far
// from the ends (the bracket stays valid but widens several-fold, and the bins
// lose resolution).  Here each end starts from a bound instead.  The third
// derivative of g is <= 0 on t >= 0 (that of log cosh(v t) and that of
// -x cosh t both are), so g'' decreases:
//   right of t_p (where g'(t_p) <= 0: the peak search ends at or right of the
//   root) g lies below the parabola g(t_p) - a d^2 / 2, a = -g''(t_p), so
//   t_p + sqrt(2 L / a) is outside;
//   left of t_p, over [t_l, t_p] the curvature is at least a_l = -g''(t_l), so
//   if w = sqrt(2 L / a_l) <= t_p - t_l, t_p - w is outside.
// For large v these bounds are nearly tight (F ~ 0 there, within the FP32
// rounding of F), so each start sits kLargeOut times further out (F ~ -0.56 L).
// From an outside point Newton steps on the concave F = g - G + L stay outside
// and converge (the tangent lies above F).  The fixed-count searches above run
// as well, and each end takes the tighter of the two valid results: near a
// flat peak (x ~ v^2, where -g''(t_p) is small) their bracket is the narrower
// one, and they are the result where a start is not outside by the FP32
// evaluation of F.
struct GDerivs {
  float F, gp, a;  // F = g - G + L, g', -g''
};
__device__ __forceinline__ GDerivs g_derivs_f32(float v, float lx, float t, float G, float L) {
  const float q = hexp2(-2.0f * kLog2eF * v * t);  // e^{-2 v t}
  const float rq = hrcp(1.0f + q);
  const float xe = hexp2(fmaf(kLog2eF, t, lx));    // x e^{t}
  const float xei = hexp2(fmaf(-kLog2eF, t, lx));  // x e^{-t}
  GDerivs d;
  d.F = v * t + (hlog2(1.0f + q) - 1.0f) * kLn2F - 0.5f * (xe + xei) - G + L;
  d.gp = v * (1.0f - q) * rq - 0.5f * (xe - xei);
  d.a = 0.5f * (xe + xei) - v * v * (4.0f * q * rq * rq);
  return d;
}

constexpr float kLargeV = 1e3f;  // above it the ends start from the bounds
constexpr int kLargeNewton = 2;  // Newton steps from each outside start
constexpr float kLargeOut = 1.25f;

__device__ __forceinline__ float upper_large_f32(float v, float x, float lx, float tp, float G, float L) {
  const float t_fixed = upper_f32(v, x, lx, tp, G, L);
  const GDerivs d0 = g_derivs_f32(v, lx, tp, G, L);
  float t = tp + kLargeOut * hsqrt(2.0f * L * hrcp(d0.a));
  GDerivs d = g_derivs_f32(v, lx, t, G, L);
  if (!(d0.a > 0.0f && d.F < 0.0f && d.gp < 0.0f)) return t_fixed;
#pragma unroll
  for (int k = 0; k < kLargeNewton; ++k) {
    const float tn = t - d.F * hrcp(d.gp);
    const GDerivs dn = g_derivs_f32(v, lx, tn, G, L);
    // keep only steps that stay outside (F < 0) and move inward
    if (!(dn.F < 0.0f && dn.gp < 0.0f && tn < t)) break;
    t = tn;
    d = dn;
  }
  return fminf(t, t_fixed);
}

__device__ __forceinline__ float lower_large_f32(float v, float lx, float tp, float G, float L) {
  const float t_fixed = lower_f32(v, lx, tp, G, L);
  const GDerivs dp = g_derivs_f32(v, lx, tp, G, L);
  const float D = 2.0f * hsqrt(2.0f * L * hrcp(dp.a));
  const float tl = fmaxf(tp - D, 0.0f);
  const GDerivs dl = g_derivs_f32(v, lx, tl, G, L);
  const float w = kLargeOut * hsqrt(2.0f * L * hrcp(dl.a));
  float t = tp - w;
  GDerivs d = g_derivs_f32(v, lx, t, G, L);
  if (!(dp.a > 0.0f && dl.a > 0.0f && w <= tp - tl && d.F < 0.0f && d.gp > 0.0f)) return t_fixed;
#pragma unroll
  for (int k = 0; k < kLargeNewton; ++k) {
    const float tn = t - d.F * hrcp(d.gp);
    const GDerivs dn = g_derivs_f32(v, lx, tn, G, L);
    if (!(dn.F < 0.0f && dn.gp > 0.0f && tn > t)) break;
    t = tn;
    d = dn;
  }
  return fminf(fmaxf(t, t_fixed), tp);
}

// Full bracket for v >= 0 and finite x > 0.  log_eps_margin = -log eps of the
// output dtype.  The search margin adds one nat plus a term proportional to
// the magnitudes that FP32 rounds, so the FP32 search cannot land inside the
// exact log-eps set.
// The shift G = g(t_p) and Gx = G + x.  Any finite shift gives the same
// log K (log K = G + log(h S0) with S0 taken relative to the same G), so the
// kernels take Gx = log cosh(v t_p) - x (cosh t_p - 1) in FP32 hardware
// arithmetic (cosh t - 1 = 2 sinh^2(t/2)) and G = Gx - x in FP64: its rounding
// (~1e-7 of log cosh(v t_p) and of x cosh t_p ~ v near the peak; x itself
// enters exactly) moves the exponents by far less than the margin, for ~20
// slots against ~90 for the FP64 form.  G64 (bessel_range's FP64 output,
// which reports g(t_p) itself) forms both in FP64.
template <bool G64 = true>
__device__ __forceinline__ Bracket find_bracket(double v, double x, float log_eps_margin) {
  Bracket b;
  const float vf = (float)v, xf = (float)x;
  const float lx = hlog2(xf);
  float tp = 0.0f;
  if (v * v > x) tp = peak_f32(vf, xf, lx);
  const float xcp = hexp2(fmaf(kLog2eF, tp, lx)) + hexp2(fmaf(-kLog2eF, tp, lx));  // 2 x cosh t_p
  double G, Gx;
  if constexpr (G64) {
    Gx = g_plus_x_f64(v, x, (double)tp);
    G = Gx - x;
  } else {
    const float eh = hexp2(0.5f * kLog2eF * tp);
    const float sh = 0.5f * (eh - hrcp(eh));  // sinh(t_p / 2)
    Gx = (double)fmaf(-2.0f * xf, sh * sh, log_cosh_f32(vf * tp));
    G = Gx - x;
  }
  const float Gf = (float)G;
  const float L = log_eps_margin + 1.0f + 1e-6f * (fabsf(Gf) + xcp);
  b.G = G;
  b.Gx = Gx;
  b.tp = tp;
  const bool need_t0 = (-x - G + (double)L) <= 0.0;
  if (vf > kLargeV && tp > 0.0f) {
    b.t1 = upper_large_f32(vf, xf, lx, tp, Gf, L);
    b.t0 = need_t0 ? lower_large_f32(vf, lx, tp, Gf, L) : 0.0f;
  } else {
    b.t1 = upper_f32(vf, xf, lx, tp, Gf, L);
    b.t0 = need_t0 ? lower_f32(vf, lx, tp, Gf, L) : 0.0f;
  }
  return b;
}

// ---------------------------------------------------------------------------
// Bins (Section 2.4, Eq. (9)-(11) and Eq. (int)).
//
// With q = e^{-2 v t} and r = 1 - q, the integrand and its companions are
//   f        = cosh(v t) e^{-x cosh t}        = e^{A} (2 - r)
//   d/dv f   = t sinh(v t) e^{-x cosh t}      = e^{A} r t
//   -d/dx f  = cosh t cosh(v t) e^{-x cosh t} = e^{A} (2 - r) cosh t
// with A = v t - x cosh t - log 2, so each node needs one exponential of the
// shifted argument A - G.  Along t_m = t0 + m h every other factor follows by
// cheap recurrences instead of transcendentals:
//   e^{t+h} - 1 = (e^t - 1) e^h + (e^h - 1), and the same for 1 - e^{-t}
//                                                        (FP64 path, re-anchored)
//   cosh(t+h) = 2 cosh(h) cosh(t) - cosh(t-h)            (FP32 path)
//   r(t+h) = r(t) e^{-2vh} + (1 - e^{-2vh})               (only positive terms,
//                                                           so r = 1 - q stays
//                                                           accurate as v -> 0)
// The sums are S0 = sum c_m f_m, Sv = sum c_m d/dv f_m, Sx = sum c_m (-d/dx f_m),
// with c_0 = c_n = 1/2 (Eq. (11)); then
//   log K = G + log(h S0),  d/dv log K = Sv / S0,  d/dx log K = -Sx / S0.
// ---------------------------------------------------------------------------
struct BinSums {
  double S0, Sv, Sx;
  // second-derivative sums (DER == 2).  FP32 bins: t^2 f, cosh^2 t f and
  // t cosh t sinh(vt) e^{-x cosh t}.  FP64 bins: moments about centres a, b
  // near the peak (bins_f64), so that the variances they form do not cancel:
  // Svv = sum f (t - a)^2, Sxx = sum f (C - b)^2, Svx = sum d/dv f (C - b),
  // and Sv1 = sum f (t - a), Sx1 = sum f (C - b), Sq = sum 2 e^{A} e^{-2vt} t,
  // the last being sum (t f - d/dv f) with C = cosh t, f = e^{A} (1 + e^{-2vt}).
  double Svv, Sxx, Svx;
  double Sv1, Sx1, Sq;
  // Filled only by the checked FP32 variant (learned brackets): the sums over
  // even and over odd nodes (each a trapezoid / midpoint rule of step 2h; their
  // difference measures the quadrature error), and the unweighted terms at the
  // two ends, relative to e^{G}.
  double Seven, Sodd;
  float term0, termN;
};

constexpr int kChunk = 16;    // nodes per unrolled chunk (FP64 bins)
constexpr int kChunk32 = 32;  // nodes per unrolled chunk (FP32 bins)

// Second-order moments of one FP64 node (DER == 2), about the centres a (t)
// and b (cosh t; C and b may both be given less 1): with wu = e^{A} u (f),
// wr = e^{A} r (d/dv f / t) and d = t - a (formed by the caller),
//   M0 += wu d^2,  M1 += wu (C - b)^2,  M2 += wr t (C - b),
//   M3 += wu d,    M4 += wu (C - b),    M5 += (wu - wr) t.
// Six sums, 12 operations a node against 6 for the raw moments t^2 f,
// C^2 f, t C d/dv f; each sum is its own chain, so no even/odd split.
__device__ __forceinline__ void moments(double wu, double wr, double t, double d, double C, double b, double* M) {
  const double Y = C - b;
  const double wuY = wu * Y, wud = wu * d;
  M[1] = fma(wuY, Y, M[1]);
  M[4] += wuY;
  M[2] = fma(wr * t, Y, M[2]);
  M[0] = fma(wud, d, M[0]);
  M[3] += wud;
  M[5] = fma(wu - wr, t, M[5]);
}

// FP64 bins.  The argument of a node's exponential is formed relative to
// g(t_p) + x: A - G = v t - x (cosh t - 1) - (g(t_p) + x) - log 2, so that for
// large x (where g(t_p) ~ -x and cosh t ~ 1 across the bracket) no term of
// size x cancels.  cosh t - 1 = (e^t - 1)(1 - e^{-t}) / 2, a product of two
// positive factors, each by a recurrence with positive terms:
//   e^{t+h} - 1 = (e^t - 1) e^h + (e^h - 1),
//   1 - e^{-(t+h)} = (1 - e^{-t}) e^{-h} + (1 - e^{-h}),
// (relative error within ~m ulp after m steps, also as t -> 0), both
// recomputed at each chunk start (every kChunk nodes) from the block's tables
// (expm1_pair_tab; the kernels build them with exp2_table_init).  f at a node is
// e^{A} u with u = 2 - r = 1 + e^{-2vt} by its own recurrence (as in the FP32
// bins); even and odd nodes are summed apart (independent FMA chains).
// S_x = sum f cosh t is returned as S0 + sum f (cosh t - 1).
// Along a chunk, v t - (g(t_p) + x) - log 2 advances by fma(v, h, .), t and
// t - ca by adding h, from the chunk's first node (one operation each, no
// per-node constant b h to materialise).  Each step rounds by at most half an
// ulp of the running value, so after the kChunk - 1 steps the error is of the
// order of v ulp(t), which the direct form v (t_a + b h) carries at every
// node; t - ca, small near the peak, keeps a finer ulp than t - ca formed
// from t.
// DER: 0 = S0 only, 1 = also S_v, S_x, 2 = also the second-derivative sums,
// taken about the centres ca (for t) and 1 + cb1 (for cosh t): the caller
// passes the peak and its cosh - 1, within a few widths of the integrand's
// means.  Gx ~ g(t_p) + x, formed without cancellation (Bracket::Gx).
template <int DER>
__device__ __forceinline__ BinSums bins_f64(int nb, double v, double x, double Gx, double t0, double t1,
                                            double ca = 0.0, double cb1 = 0.0) {
  constexpr bool GRAD = DER >= 1;
  const double h = (t1 - t0) / (double)nb;
  const double Gs = Gx + kLn2;
  const double xh = 0.5 * x;
  const Expm1Pair hh = expm1_pair_tab(h);
  const double eh = 1.0 + hh.ep, ehi = 1.0 - hh.em;
  const ExpNeg qh = exp_neg_pair(2.0 * v * h);
  const double Q = qh.q, E2 = qh.om;  // e^{-2vh}, 1 - Q
  double r = one_minus_exp_neg(2.0 * v * t0);
  double u = 2.0 - r;
  BinSums s{};
  double S[2] = {0.0, 0.0}, Sv[2] = {0.0, 0.0}, Sx[2] = {0.0, 0.0};
  double M[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // second-order moments (DER == 2)
  const int nchunks = nb / kChunk;
  for (int c = 0; c < nchunks; ++c) {
    const double ta = fma((double)(c * kChunk), h, t0);
    Expm1Pair an = expm1_pair_tab(ta);
    double L = fma(v, ta, -Gs), t = ta, d = ta - ca;
#pragma unroll
    for (int b = 0; b < kChunk; ++b) {
      if (b > 0) {
        L = fma(v, h, L);  // an explicit FMA, whatever the compiler's contraction
        if (GRAD) t += h;
        if (DER >= 2) d += h;
      }
      const double P = an.ep * an.em;  // 2 (cosh t - 1)
      double w = exp_node_f64(fma(-xh, P, L));
      if (b == 0) w *= (c == 0) ? 0.5 : 1.0;
      S[b & 1] = fma(w, u, S[b & 1]);
      if (GRAD) {
        const double wr = w * r, wu = w * u;
        Sv[b & 1] = fma(wr, t, Sv[b & 1]);
        Sx[b & 1] = fma(wu, P, Sx[b & 1]);
        if (DER >= 2) moments(wu, wr, t, d, 0.5 * P, cb1, M);
        r = fma(r, Q, E2);
      }
      u = fma(u, Q, E2);
      an.ep = fma(an.ep, eh, hh.ep);
      an.em = fma(an.em, ehi, hh.em);
    }
  }
  // remainder nodes (nb not a multiple of kChunk) and the last node m = nb
  for (int m = nchunks * kChunk; m <= nb; ++m) {
    const double t = (m == nb) ? t1 : fma((double)m, h, t0);
    const Expm1Pair an = expm1_pair_tab(t);
    const double P = an.ep * an.em;
    double w = exp_node_f64(fma(-xh, P, fma(v, t, -Gs)));
    if (m == 0 || m == nb) w *= 0.5;
    S[m & 1] = fma(w, u, S[m & 1]);
    if (GRAD) {
      const double wr = w * r, wu = w * u;
      Sv[m & 1] = fma(wr, t, Sv[m & 1]);
      Sx[m & 1] = fma(wu, P, Sx[m & 1]);
      if (DER >= 2) moments(wu, wr, t, t - ca, 0.5 * P, cb1, M);
      r = fma(r, Q, E2);
    }
    u = fma(u, Q, E2);
  }
  s.S0 = S[0] + S[1];
  if (GRAD) {
    s.Sv = Sv[0] + Sv[1];
    s.Sx = fma(0.5, Sx[0] + Sx[1], s.S0);
  }
  if (DER >= 2) {
    s.Svv = M[0];
    s.Sxx = M[1];
    s.Svx = M[2];
    s.Sv1 = M[3];
    s.Sx1 = M[4];
    s.Sq = M[5];
  }
  return s;
}

// FP32 bins: the argument A - G is formed in FP64 (v t, x cosh t and G reach
// ~1e3 and nearly cancel, which FP32 could not resolve), pre-scaled by log2 e;
// then one hardware exp2 per node, whose FP32 result is widened and
// accumulated in FP64 against u = 2 - r = 1 + e^{-2vt}.  u, r and cosh t
// follow linear recurrences (one FMA each per node):
//   u_{m+1} = Q u_m + (1 - Q),  r_{m+1} = Q r_m + (1 - Q),  Q = e^{-2vh},
// whose terms are positive (relative error ~ m eps), and the three-term
// C_{m+1} = 2 cosh h C_m - C_{m-1} (relative error ~ m eps / (2 sinh h)).
// r (for d/dv) is kept by its own recurrence rather than as 2 - u, which would
// lose its relative accuracy as v -> 0.  The forward and derivative variants
// accumulate S0 with identical operations.
template <int DER, bool CHECK = false>
__device__ __forceinline__ BinSums bins_f32(int nb, double v, double x, double G, double t0, double t1) {
  constexpr bool GRAD = DER >= 1;
  const double h = (t1 - t0) / (double)nb;
  const double vl = v * kLog2e;
  const double xl = x * kLog2e;
  const double Gl = (G + kLn2) * kLog2e;
  const double dL = vl * h;
  const double eh = exp_f64(h);
  const double ehi = rcp_f64(eh);
  const double c2 = eh + ehi;  // 2 cosh h
  const double E0 = exp_f64(t0);
  const double E0i = rcp_f64(E0);
  double Cp = 0.5 * (E0 * ehi + E0i * eh);  // cosh(t0 - h)
  double C = 0.5 * (E0 + E0i);              // cosh(t0)
  const ExpNeg qh = exp_neg_pair(2.0 * v * h);
  const double Q = qh.q, E2 = qh.om;  // e^{-2vh}, 1 - Q
  double r = one_minus_exp_neg(2.0 * v * t0);
  double u = 2.0 - r;
  const double L0 = fma(vl, t0, -Gl);  // (v t - G - log 2) log2 e
  BinSums s{};
  // even and odd nodes go to separate sums (two independent FMA chains; the
  // checked variant also needs them apart); chunk starts are even
  double S[2] = {0.0, 0.0}, Sv[2] = {0.0, 0.0}, Sx[2] = {0.0, 0.0};
  double Svv[2] = {0.0, 0.0}, Sxx[2] = {0.0, 0.0}, Svx[2] = {0.0, 0.0};
  const int nchunks = nb / kChunk32;
  for (int c = 0; c < nchunks; ++c) {
    // the linear part runs by addition inside a chunk (error <= kChunk32 ulp of |L|)
    double L = fma((double)(c * kChunk32), dL, L0);
    // node time, by addition likewise: an index literal in fma(b, h, t) would
    // cost a copy per node (the three-operand FMA takes no literal)
    double t = fma((double)(c * kChunk32), h, t0);
#pragma unroll
    for (int b = 0; b < kChunk32; ++b) {
      float w = hexp2((float)fma(-xl, C, L));
      if (CHECK && b == 0 && c == 0) s.term0 = w * (float)u;
      if (b == 0) w *= (c == 0) ? 0.5f : 1.0f;
      const double wd = (double)w;
      S[b & 1] = fma(wd, u, S[b & 1]);
      if (GRAD) {
        const double wr = wd * r, wu = wd * u;
        Sv[b & 1] = fma(wr, t, Sv[b & 1]);
        Sx[b & 1] = fma(wu, C, Sx[b & 1]);
        if (DER >= 2) {
          Svv[b & 1] = fma(wu * t, t, Svv[b & 1]);
          Sxx[b & 1] = fma(wu * C, C, Sxx[b & 1]);
          Svx[b & 1] = fma(wr * t, C, Svx[b & 1]);
        }
        r = fma(r, Q, E2);
        t += h;
      }
      u = fma(u, Q, E2);
      L += dL;
      const double Cn = fma(c2, C, -Cp);
      Cp = C;
      C = Cn;
    }
  }
  for (int m = nchunks * kChunk32; m <= nb; ++m) {
    const double L = (m == nb) ? fma(vl, t1, -Gl) : fma((double)m, dL, L0);
    float w = hexp2((float)fma(-xl, C, L));
    if (CHECK && m == 0) s.term0 = w * (float)u;
    if (CHECK && m == nb) s.termN = w * (float)u;
    if (m == 0 || m == nb) w *= 0.5f;
    const double wd = (double)w;
    S[m & 1] = fma(wd, u, S[m & 1]);
    if (GRAD) {
      const double t = (m == nb) ? t1 : fma((double)m, h, t0), wr = wd * r, wu = wd * u;
      Sv[m & 1] = fma(wr, t, Sv[m & 1]);
      Sx[m & 1] = fma(wu, C, Sx[m & 1]);
      if (DER >= 2) {
        Svv[m & 1] = fma(wu * t, t, Svv[m & 1]);
        Sxx[m & 1] = fma(wu * C, C, Sxx[m & 1]);
        Svx[m & 1] = fma(wr * t, C, Svx[m & 1]);
      }
      r = fma(r, Q, E2);
    }
    u = fma(u, Q, E2);
    const double Cn = fma(c2, C, -Cp);
    Cp = C;
    C = Cn;
  }
  s.S0 = S[0] + S[1];
  if (CHECK) {
    s.Seven = S[0];
    s.Sodd = S[1];
  }
  if (GRAD) {
    s.Sv = Sv[0] + Sv[1];
    s.Sx = Sx[0] + Sx[1];
  }
  if (DER >= 2) {
    s.Svv = Svv[0] + Svv[1];
    s.Sxx = Sxx[0] + Sxx[1];
    s.Svx = Svx[0] + Svx[1];
  }
  return s;
}

// ---------------------------------------------------------------------------
// Bins of one sub-range, for kernels that split an element's nodes over
// several lanes (small batches, where one lane per element would leave most
// of the chip idle): nodes m in [m_lo, m_hi), and the last node m = nb when
// with_end (then m_hi == nb).  The per-node arithmetic is that of bins_f32 /
// bins_f64 with every recurrence started at m_lo; c_0 = c_nb = 1/2.
// ---------------------------------------------------------------------------
template <int DER>
__device__ __forceinline__ BinSums sub_bins_f32(int nb, int m_lo, int m_hi, bool with_end, double v, double x,
                                                double G, double t0, double t1) {
  constexpr bool GRAD = DER >= 1;
  const double h = (t1 - t0) / (double)nb;
  const double vl = v * kLog2e;
  const double xl = x * kLog2e;
  const double Gl = (G + kLn2) * kLog2e;
  const double dL = vl * h;
  const double ta = fma((double)m_lo, h, t0);
  const double eh = exp_f64(h);
  const double ehi = rcp_f64(eh);
  const double c2 = eh + ehi;
  const double Ea = exp_f64(ta);
  const double Eai = rcp_f64(Ea);
  double Cp = 0.5 * (Ea * ehi + Eai * eh);
  double C = 0.5 * (Ea + Eai);
  const ExpNeg qh = exp_neg_pair(2.0 * v * h);
  const double Q = qh.q, E2 = qh.om;
  double r = one_minus_exp_neg(2.0 * v * ta);
  double u = 2.0 - r;
  double L = fma((double)m_lo, dL, fma(vl, t0, -Gl));
  BinSums s{};
  for (int m = m_lo; m <= m_hi; ++m) {
    if (m == m_hi) {
      if (!with_end) break;
      L = fma(vl, t1, -Gl);
    }
    float w = hexp2((float)fma(-xl, C, L));
    if (m == 0 || m == nb) w *= 0.5f;
    const double wd = (double)w;
    s.S0 = fma(wd, u, s.S0);
    if (GRAD) {
      const double t = (m == nb) ? t1 : fma((double)m, h, t0);
      const double wr = wd * r, wu = wd * u;
      s.Sv = fma(wr, t, s.Sv);
      s.Sx = fma(wu, C, s.Sx);
      if (DER >= 2) {
        s.Svv = fma(wu * t, t, s.Svv);
        s.Sxx = fma(wu * C, C, s.Sxx);
        s.Svx = fma(wr * t, C, s.Svx);
      }
      r = fma(r, Q, E2);
    }
    u = fma(u, Q, E2);
    L += dL;
    const double Cn = fma(c2, C, -Cp);
    Cp = C;
    C = Cn;
  }
  return s;
}

template <int DER>
__device__ __forceinline__ BinSums sub_bins_f64(int nb, int m_lo, int m_hi, bool with_end, double v, double x,
                                                double Gx, double t0, double t1, double ca = 0.0, double cb1 = 0.0) {
  constexpr bool GRAD = DER >= 1;
  const double h = (t1 - t0) / (double)nb;
  const double Gs = Gx + kLn2;
  const double xh = 0.5 * x;
  const Expm1Pair hh = expm1_pair_tab(h);
  const double eh = 1.0 + hh.ep, ehi = 1.0 - hh.em;
  const ExpNeg qh = exp_neg_pair(2.0 * v * h);
  const double Q = qh.q, E2 = qh.om;
  double r = one_minus_exp_neg(2.0 * v * fma((double)m_lo, h, t0));
  double u = 2.0 - r;
  Expm1Pair an{0.0, 0.0};
  double M[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // second-order moments (DER == 2)
  double SxP = 0.0;
  BinSums s{};
  for (int m = m_lo; m <= m_hi; ++m) {
    if (m == m_hi && !with_end) break;
    const double t = (m == nb) ? t1 : fma((double)m, h, t0);
    if ((m - m_lo) % kChunk == 0 || m == nb) an = expm1_pair_tab(t);  // recurrences re-anchored every kChunk nodes
    const double P = an.ep * an.em;  // 2 (cosh t - 1)
    double w = exp_node_f64(fma(-xh, P, fma(v, t, -Gs)));
    if (m == 0 || m == nb) w *= 0.5;
    s.S0 = fma(w, u, s.S0);
    if (GRAD) {
      const double wr = w * r, wu = w * u;
      s.Sv = fma(wr, t, s.Sv);
      SxP = fma(wu, P, SxP);
      if (DER >= 2) moments(wu, wr, t, t - ca, 0.5 * P, cb1, M);
      r = fma(r, Q, E2);
    }
    u = fma(u, Q, E2);
    an.ep = fma(an.ep, eh, hh.ep);
    an.em = fma(an.em, ehi, hh.em);
  }
  // S_x = sum f cosh t as the sum of f and of f (cosh t - 1): the split kernels
  // add each lane's S0 and Sx over the group, so Sx carries both parts
  if (GRAD) s.Sx = fma(0.5, SxP, s.S0);
  if (DER >= 2) {
    s.Svv = M[0];
    s.Sxx = M[1];
    s.Svx = M[2];
    s.Sv1 = M[3];
    s.Sx1 = M[4];
    s.Sq = M[5];
  }
  return s;
}

}  // namespace bk
