// bessel_deriv.hip -- derivatives of K_v(x) itself of any orders a (in v) and
// b (in x), each integrand over its own peak and bracket (Section 4.1,
// Eq. (13)), and the C ABI entry point bessel_logdk.
//
// Differentiating Eq. (1) under the integral,
//   d^a/dv^a d^b/dx^b K_v(x) = (-1)^b int_0^inf t^a cosh^b(t) C_a(v t) e^{-x cosh t} dt,
// with C_a = cosh for even a and sinh for odd a.  For v >= 0 the integrand is
// non-negative with log
//   g_ab(t) = a log t + b log cosh t + log C_a(v t) - x cosh t,
// which has a single peak: g_ab' = sinh(t) (phi(t) - x) where
// phi = (a/t + b tanh t + v T(v t)) / sinh t (T = tanh for even a, coth for odd
// a) is strictly decreasing, so g_ab' changes sign once.  Each element then
// runs the method of Section 2 on g_ab instead of g: peak, the bracket where
// g_ab is within log eps of the peak, and the fixed-bin trapezoid in log space.
//
// This is the accuracy path for derivatives.  The companion sums of
// bessel_logk_dv_dx and bessel_logk_hess reuse f's bracket, which is enough
// for first and second orders; higher orders move the integrand's mass away
// from f's (t^a and cosh^b t grow), and only brackets of their own keep the
// FP64 bar.  All arithmetic is FP64 (both dtypes): the searches evaluate
// g_ab with FP64 exp and log, and the bins use the FP64 node exponential.
// The searches have data-dependent trip counts (a doubling search, as
// Algorithm 1 of the paper, for each end), bounded by fixed limits.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "bessel.h"
#include "bessel_device.hpp"
#include "bessel_internal.hpp"

namespace bk {
namespace {

// Past this t the factor x cosh t exceeds every level the searches compare
// against for any x >= 1e-36 (x cosh 700 > 1e267): g_ab is taken as -inf.
constexpr double kDkTMax = 700.0;
// bisection steps in log t for the peak, then safeguarded Newton steps (the
// peak only sets the shift and the start of the end searches: any point near
// it gives a valid bracket)
constexpr int kDkPeakBisect = 8;
constexpr int kDkPeakNewton = 4;
// each end: at most kDkDoubling doublings of the step, then kDkRefine rounds
// of one bisection and one safeguarded Newton step
constexpr int kDkDoubling = 64;
constexpr int kDkRefine = 3;

struct GabAt {
  double g;   // g_ab(t)
  double g1;  // g_ab'(t)
  double g2;  // g_ab''(t)
};

// g_ab and its first two t-derivatives at t > 0 (v >= 0; v > 0 for odd a).
// With q = e^{-2vt}, r = 1 - q and u = 1 + q:
//   log C_a(vt) = vt - log 2 + log(u or r),   v T(vt) = v (r/u or u/r),
//   d/dt v T(vt) = +-4 v^2 q / (u or r)^2.
template <bool VAL, bool D2>
__device__ __forceinline__ GabAt gab_at(double v, double x, int a, int b, double t) {
  GabAt o;
  if (t > kDkTMax) {
    o.g = -__builtin_inf();
    o.g1 = -__builtin_inf();
    o.g2 = -__builtin_inf();
    return o;
  }
  const ExpParts et = exp_parts(t);
  const double E = scale2k(1.0 + et.em1, et.k);
  const double Ei = rcp_f64(E);
  const double ch = 0.5 * (E + Ei);
  // sinh t from e^t - 1 when t is small (|t| <= log(2)/2: 2^k = 1), so it
  // keeps its relative accuracy
  const double sh = (et.k == 0) ? 0.5 * et.em1 * (1.0 + Ei) : 0.5 * (E - Ei);
  const ExpParts eq = exp_parts(-2.0 * v * t);
  const double q = scale2k(1.0 + eq.em1, eq.k);
  const double r = (eq.k == 0) ? -eq.em1 : 1.0 - q;
  const double u = 1.0 + q;
  const bool odd = a & 1;
  const double num = odd ? u : r;
  const double den = odd ? r : u;
  const double rden = rcp_f64(den);
  const double rt = rcp_f64(t);
  const double rch = rcp_f64(ch);
  o.g1 = (double)a * rt + (double)b * sh * rch + v * num * rden - x * sh;
  if (VAL) {
    // a log t + b log cosh t = b (t - log 2) + log(t^a (1 + e^{-2t})^b): one
    // log for both while the product is a normal number ((1 + e^{-2t})^b <= 2^8
    // and t <= 700 bound it above; a tiny t^a takes the two logs apart)
    double pw = 1.0;
    for (int k = 0; k < a; ++k) pw *= t;
    const double c2 = 1.0 + Ei * Ei;
    for (int k = 0; k < b; ++k) pw *= c2;
    double g = (v * t - kLn2 + log_f64(den)) - x * ch;
    if (b) g = fma((double)b, t - kLn2, g);
    if (pw >= 1e-290) {
      if (a || b) g += log_f64(pw);
    } else {
      g += (double)a * log_f64(t) + (double)b * log_f64(c2);
    }
    o.g = g;
  }
  if (D2) {
    const double tq = 4.0 * v * v * q * rden * rden;
    o.g2 = -(double)a * rt * rt + (double)b * rch * rch + (odd ? -tq : tq) - x * ch;
  }
  return o;
}

// Peak of g_ab.  At t = 0 when a = 0 and b + v^2 <= x (then g_ab''(0) <= 0 and
// phi decreasing keep g_ab' <= 0).  Otherwise the root of g_ab' lies below
//   T = min(t*, max(1, t**)),  t* = ((b+v) + sqrt((b+v)^2 + 4x(a+1))) / (2x),
//   t** = log(1 + 2(a+1+b+v)/x),
// since g_ab' <= (a+1)/t + b + v - x sinh t, negative beyond t* (sinh t > t) and
// beyond max(1, t**) (sinh t > (e^t - 1)/2, (a+1)/t <= a+1).  Bisection in
// log t over 40 octaves below T, then Newton steps kept inside the bracket.
__device__ __forceinline__ double gab_peak(double v, double x, int a, int b) {
  if (a == 0 && (double)b + v * v <= x) return 0.0;
  const double c = (double)b + v;
  const double ts = (c + sqrt(fma(c, c, 4.0 * x * (double)(a + 1)))) / (2.0 * x);
  const double tss = log_f64(1.0 + 2.0 * ((double)(a + 1) + c) / x);
  const double T = fmin(ts, fmax(1.0, tss)) * 1.0625;
  double shi = log_f64(T);
  double slo = shi - 40.0 * kLn2;
  for (int k = 0; k < kDkPeakBisect; ++k) {
    const double sm = 0.5 * (slo + shi);
    if (gab_at<false, false>(v, x, a, b, exp_f64(sm)).g1 > 0.0) slo = sm;
    else shi = sm;
  }
  double lo = exp_f64(slo), hi = exp_f64(shi);
  double t = sqrt(lo * hi);
  for (int k = 0; k < kDkPeakNewton; ++k) {
    const GabAt p = gab_at<false, true>(v, x, a, b, t);
    if (p.g1 > 0.0) lo = t;
    else hi = t;
    double tn = (p.g2 < 0.0) ? t - p.g1 / p.g2 : 0.5 * (lo + hi);
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    t = tn;
  }
  return t;
}

struct DkBracket {
  double tp, G, t0, t1;
};

// Bracket [t0, t1] containing {t : g_ab(t) >= G - L}, G = g_ab(t_p).  Each end:
// steps from t_p doubling from d0 = sqrt(2L / -g_ab''(t_p)) (the width of a
// Gaussian with that curvature, capped at max(t_p, 1)) until F = g_ab - G + L
// is negative, then rounds of one bisection and one Newton step from the
// outer end, keeping F >= 0 inside and F < 0 outside.  The outer end is
// returned, so the bracket is a superset.
__device__ __forceinline__ DkBracket gab_bracket(double v, double x, int a, int b, double L) {
  DkBracket br;
  const double tp = gab_peak(v, x, a, b);
  double G, curv;
  if (tp > 0.0) {
    const GabAt p = gab_at<true, true>(v, x, a, b, tp);
    G = p.g;
    curv = -p.g2;
  } else {
    G = -x;
    curv = x - (double)b - v * v;
  }
  br.tp = tp;
  br.G = G;
  const double cap = fmax(tp, 1.0);
  const double d0 = (curv > 0.0) ? fmin(sqrt(2.0 * L / curv), cap) : cap;

  // upper end
  {
    double lo = tp, d = d0, hi = tp + d;
    GabAt ph = gab_at<true, false>(v, x, a, b, hi);
    for (int k = 0; k < kDkDoubling && ph.g - G + L >= 0.0; ++k) {
      lo = hi;
      d *= 2.0;
      hi = tp + d;
      ph = gab_at<true, false>(v, x, a, b, hi);
    }
    for (int it = 0; it < kDkRefine; ++it) {
      const double mid = 0.5 * (lo + hi);
      const GabAt pm = gab_at<true, false>(v, x, a, b, mid);
      if (pm.g - G + L >= 0.0) {
        lo = mid;
      } else {
        hi = mid;
        ph = pm;
      }
      const double tn = hi - (ph.g - G + L) / ph.g1;  // F < 0 and F' < 0 at hi
      if (tn > lo && tn < hi) {
        const GabAt pn = gab_at<true, false>(v, x, a, b, tn);
        if (pn.g - G + L >= 0.0) {
          lo = tn;
        } else {
          hi = tn;
          ph = pn;
        }
      }
    }
    br.t1 = hi;
  }

  // lower end: 0 when the peak is at 0 or g_0b(0) = -x is inside the set
  if (tp == 0.0 || (a == 0 && -x - G + L >= 0.0)) {
    br.t0 = 0.0;
  } else {
    double hi = tp, d = d0, lo = tp - d;
    GabAt pl{};
    bool outside = false;
    for (int k = 0; k < kDkDoubling && lo > 0.0; ++k) {
      pl = gab_at<true, false>(v, x, a, b, lo);
      if (pl.g - G + L < 0.0) {
        outside = true;
        break;
      }
      hi = lo;
      d *= 2.0;
      lo = tp - d;
    }
    // otherwise 0 is the outer end: F(0) < 0 here, since a > 0 (g_ab -> -inf)
    // or -x - G + L < 0
    if (!outside) lo = 0.0;
    for (int it = 0; it < kDkRefine; ++it) {
      const double mid = 0.5 * (lo + hi);
      const GabAt pm = gab_at<true, false>(v, x, a, b, mid);
      if (pm.g - G + L >= 0.0) {
        hi = mid;
      } else {
        lo = mid;
        pl = pm;
      }
      if (lo > 0.0) {
        const double tn = lo - (pl.g - G + L) / pl.g1;  // F < 0 and F' > 0 at lo
        if (tn > lo && tn < hi) {
          const GabAt pn = gab_at<true, false>(v, x, a, b, tn);
          if (pn.g - G + L >= 0.0) {
            hi = tn;
          } else {
            lo = tn;
            pl = pn;
          }
        }
      }
    }
    br.t0 = lo;
  }
  return br;
}

// The trapezoid of Eq. (int) on g_ab: sum_m c_m e^{g_ab(t_m) - G} with
//   e^{g_ab(t) - G} = e^{A(t) - A(t_p)} (t/t_p)^a (cosh t / cosh t_p)^b rho(t),
//   A(t) = v t - x cosh t,  rho = (u or r)(t) / (u or r)(t_p),
// where rho follows the linear recurrence of u and r (scaled by the constant
// 1/(u or r)(t_p)) and e^{t_m}, e^{-t_m} run by products re-anchored every
// kChunk nodes, as in the log K bins.
__device__ __forceinline__ double gab_bins(int nb, double v, double x, int a, int b, const DkBracket& br) {
  const double t0 = br.t0, t1 = br.t1, tp = br.tp;
  const double h = (t1 - t0) / (double)nb;
  const bool odd = a & 1;
  const double Ep = exp_f64(tp);
  const double chp = 0.5 * (Ep + rcp_f64(Ep));
  const double rchp = rcp_f64(chp);
  const double rtp = (a > 0) ? rcp_f64(tp) : 0.0;
  const double Ap = fma(v, tp, -x * chp);
  const double rp = one_minus_exp_neg(2.0 * v * tp);
  const double rfp = rcp_f64(odd ? rp : 2.0 - rp);
  const double Q = exp_f64(-2.0 * v * h);
  const double E2s = one_minus_exp_neg(2.0 * v * h) * rfp;
  const double r0 = one_minus_exp_neg(2.0 * v * t0);
  double rho = (odd ? r0 : 2.0 - r0) * rfp;
  const double xh = 0.5 * x;
  const double eh = exp_f64(h), ehi = rcp_f64(eh);
  double S[2] = {0.0, 0.0};
  const int nchunks = (nb + 1 + kChunk - 1) / kChunk;
  for (int c = 0; c < nchunks; ++c) {
    const int m0 = c * kChunk;
    const double ta = fma((double)m0, h, t0);
    double E = exp_f64(ta);
    double Ei = rcp_f64(E);
    for (int j = 0; j < kChunk; ++j) {
      const int m = m0 + j;
      if (m > nb) break;
      const double t = (m == nb) ? t1 : fma((double)j, h, ta);
      const double ch2 = E + Ei;
      // clamped below the overflow of 2^k; arguments that large do not occur
      // inside the validated domain
      double w = exp_node_f64(fmin(fma(-xh, ch2, fma(v, t, -Ap)), 708.0));
      double p = rho;
      const double tt = t * rtp;
      for (int k = 0; k < a; ++k) p *= tt;
      const double cc = 0.5 * ch2 * rchp;
      for (int k = 0; k < b; ++k) p *= cc;
      if (m == 0 || m == nb) w *= 0.5;
      S[m & 1] = fma(w, p, S[m & 1]);
      rho = fma(rho, Q, E2s);
      E *= eh;
      Ei *= ehi;
    }
  }
  return h * (S[0] + S[1]);
}

// -log eps of the output dtype plus one nat of margin.
template <typename T>
__device__ __forceinline__ double dk_margin() {
  return (sizeof(T) == 8 ? 36.0436533891171560 : 15.9423851528787422) + 1.0;
}

template <typename T, int NB>
__global__ __launch_bounds__(kBlock) void k_logdk(int64_t n, int nbins, int a, int b, const T* __restrict__ vin,
                                                  const T* __restrict__ xin, T* __restrict__ out,
                                                  T* __restrict__ sgn) {
  exp2_table_init();  // the bins run in FP64 for both output types
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int nb = NB > 0 ? NB : nbins;
  const double vs = (double)vin[i];
  const double x = (double)xin[i];
  const double nan_ = __builtin_nan("");
  double s = (b & 1) ? -1.0 : 1.0;
  if ((a & 1) && vs < 0.0) s = -s;
  double res;
  if (__builtin_isnan(vs) || __builtin_isnan(x) || x < 0.0 || (x > 0.0 && x < kMinX)) {
    res = nan_;
    s = nan_;
  } else if ((a & 1) && vs == 0.0) {
    res = -__builtin_inf();  // an odd v-derivative of a function even in v
    s = 0.0;
  } else if (x == 0.0 || __builtin_isinf(vs)) {
    res = __builtin_inf();
  } else if (__builtin_isinf(x)) {
    res = -__builtin_inf();
  } else {
    const double v = fabs(vs);
    const DkBracket br = gab_bracket(v, x, a, b, dk_margin<T>());
    res = br.G + log_f64(gab_bins(nb, v, x, a, b, br));
  }
  out[i] = (T)res;
  if (sgn) sgn[i] = (T)s;
}

template <typename T>
void launch_logdk(dim3 grid, hipStream_t st, int64_t n, int nbins, int a, int b, const void* v, const void* x,
                  void* out, void* sgn) {
  const T* vv = (const T*)v;
  const T* xx = (const T*)x;
  T* o = (T*)out;
  T* s = (T*)sgn;
  switch (nbins) {
    case 64: k_logdk<T, 64><<<grid, kBlock, 0, st>>>(n, nbins, a, b, vv, xx, o, s); break;
    case 128: k_logdk<T, 128><<<grid, kBlock, 0, st>>>(n, nbins, a, b, vv, xx, o, s); break;
    case 256: k_logdk<T, 256><<<grid, kBlock, 0, st>>>(n, nbins, a, b, vv, xx, o, s); break;
    default: k_logdk<T, 0><<<grid, kBlock, 0, st>>>(n, nbins, a, b, vv, xx, o, s); break;
  }
}

}  // namespace
}  // namespace bk

using namespace bk;

extern "C" int bessel_logdk(int dtype, int64_t n, const void* v, const void* x, int order_v, int order_x,
                            void* logdk, void* sign, int nbins, void* hip_stream) {
  if (dtype != BESSEL_F32 && dtype != BESSEL_F64) return set_error(BESSEL_ERR_DTYPE, "dtype %d is not F32/F64", dtype);
  if (n < 0) return set_error(BESSEL_ERR_ARG, "n = %lld < 0", (long long)n);
  if (n > 0 && (!v || !x)) return set_error(BESSEL_ERR_ARG, "v and x must be non-NULL");
  if (order_v < 0 || order_v > BESSEL_MAX_ORDER || order_x < 0 || order_x > BESSEL_MAX_ORDER)
    return set_error(BESSEL_ERR_ORDER, "orders (%d, %d) outside [0, %d]", order_v, order_x, BESSEL_MAX_ORDER);
  if (nbins < BESSEL_MIN_BINS || nbins > BESSEL_MAX_BINS)
    return set_error(BESSEL_ERR_NBINS, "nbins = %d outside [%d, %d]", nbins, BESSEL_MIN_BINS, BESSEL_MAX_BINS);
  if (n == 0) return BESSEL_OK;
  if (!logdk) return set_error(BESSEL_ERR_ARG, "logdk must be non-NULL");
  const size_t nb = (size_t)n * (dtype == BESSEL_F64 ? 8 : 4);
  void* outs[2] = {logdk, sign};
  for (int k = 0; k < 2; ++k)
    if (overlaps(outs[k], nb, v, nb) || overlaps(outs[k], nb, x, nb))
      return set_error(BESSEL_ERR_ALIAS, "an output overlaps an input");
  if (overlaps(logdk, nb, sign, nb)) return set_error(BESSEL_ERR_ALIAS, "logdk overlaps sign");
  dim3 grid;
  int rc = grid_for(n, grid);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  if (dtype == BESSEL_F64)
    launch_logdk<double>(grid, st, n, nbins, order_v, order_x, v, x, logdk, sign);
  else
    launch_logdk<float>(grid, st, n, nbins, order_v, order_x, v, x, logdk, sign);
  return check_launch("k_logdk");
}
