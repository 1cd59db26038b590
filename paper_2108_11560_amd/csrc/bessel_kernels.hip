// bessel_kernels.hip -- gfx950 kernels and the C ABI (include/bessel.h) for
// batched log K_v(x), its v/x derivatives and the integration range.
//
// One (v, x) element per lane, SoA inputs loaded coalesced, all per-element
// state in registers, a fixed bin count per launch so every lane of a
// wavefront runs the same instruction stream (Section 2.4: the fixed number of
// divisions is what makes the time per element uniform).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "bessel.h"
#include "bessel_device.hpp"
#include "bessel_internal.hpp"

namespace bk {

// -log eps of the output dtype: eps = 2^-52 (FP64), 2^-23 (FP32).
constexpr float kMarginF64 = 36.0436533891171560f;
constexpr float kMarginF32 = 15.9423851528787422f;

template <typename T>
__device__ __forceinline__ float margin_of() {
  return sizeof(T) == 8 ? kMarginF64 : kMarginF32;
}

template <typename T, int DER>
__device__ __forceinline__ BinSums run_bins(int nb, double v, double x, const Bracket& b) {
  if constexpr (sizeof(T) == 8) {
    return bins_f64<DER>(nb, v, x, b.Gx, (double)b.t0, (double)b.t1);
  } else {
    return bins_f32<DER>(nb, v, x, b.G, (double)b.t0, (double)b.t1);
  }
}

// NB > 0: bin count fixed at compile time; NB == 0: runtime nbins.
template <typename T, int NB, bool GRAD>
__global__ __launch_bounds__(kBlock) void k_logk(int64_t n, int nbins, const T* __restrict__ vin,
                                                 const T* __restrict__ xin, const T* __restrict__ gout,
                                                 T* __restrict__ logk, T* __restrict__ dv,
                                                 T* __restrict__ dx) {
  if constexpr (sizeof(T) == 8) {
    exp2_table_init();
    __syncthreads();
  }
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int nb = NB > 0 ? NB : nbins;
  const double vs = (double)vin[i];
  const double x = (double)xin[i];
  double lk, dvv, dxv;
  if (!domain_special(vs, x, lk, dvv, dxv)) {
    const double v = fabs(vs);
    const Bracket b = find_bracket<false>(v, x, margin_of<T>());
    const BinSums s = run_bins<T, GRAD ? 1 : 0>(nb, v, x, b);
    const double h = ((double)b.t1 - (double)b.t0) / (double)nb;
    constexpr bool F64 = sizeof(T) == 8;
    lk = b.G + log_of<F64>(h * s.S0);
    if (GRAD) {
      const double rS0 = rcp_of<F64>(s.S0);
      dvv = (v == 0.0) ? 0.0 : copysign(s.Sv * rS0, vs);
      dxv = -s.Sx * rS0;
    }
  }
  if (GRAD) {
    if (gout) {
      const double go = (double)gout[i];
      dvv *= go;
      dxv *= go;
    }
    dv[i] = (T)dvv;
    dx[i] = (T)dxv;
    if (logk) logk[i] = (T)lk;
  } else {
    logk[i] = (T)lk;
  }
}

// log K with its first and second derivatives in v and x from one pass over
// the bins (Section 4.1, Eq. (13) with n + m <= 2).  Under the normalised
// integrand p = f / K, with tau = tanh(v t) and C = cosh t,
//   d2/dv2 log K = E[t^2] - E[t tau]^2,  d2/dx2 log K = Var C,
//   d2/dvdx log K = -Cov(t tau, C)   (odd in v, like d/dv).
// FP32 outputs form them from the raw sums (S_vv/S - (S_v/S)^2 and so on).
// FP64 outputs take the sums about centres a = t_p and b = cosh t_p (the FP64
// bins' moments, of cosh t - 1 about cosh t_p - 1): where the integrand is narrow (large v with small x, or
// large x) E[C^2] exceeds Var C by up to ~1e8, and the raw difference would
// lose that many digits.  With D = E[t] - a and Dx = E[C] - b from the
// centred first moments,
//   Var C = E[(C - b)^2] - Dx^2,  Cov(t tau, C) = E[t tau (C - b)] - E[t tau] Dx,
//   E[t^2] - E[t tau]^2 = E[(t - a)^2] - D^2 + E[t - t tau] (E[t] + E[t tau]),
// where E[t - t tau] = E[2 e^{-2vt} t / (1 + e^{-2vt})] comes from its own
// positive sum, not as a difference of the two nearly equal means.
// Every output is nullable.
// The six outputs of k_logk_hess from an element's bracket and sums (the
// bracket's t_p is the centre of the FP64 moments).
template <bool F64>
__device__ __forceinline__ void hess_outputs(double vs, double v, const Bracket& b, const BinSums& s, int nb,
                                             double& lk, double& lv, double& lx, double& lvv, double& lxx,
                                             double& lvx) {
  const double h = ((double)b.t1 - (double)b.t0) / (double)nb;
  // first order as bessel_logk_dv_dx (same operations, same results); the
  // second order takes FP64 1/S0
  const double rS0o = rcp_of<F64>(s.S0);
  lk = b.G + log_of<F64>(h * s.S0);
  lv = (v == 0.0) ? 0.0 : copysign(s.Sv * rS0o, vs);
  lx = -s.Sx * rS0o;
  const double rS0 = rcp_f64(s.S0);
  const double ev = s.Sv * rS0, ex = s.Sx * rS0;
  double mvx;  // -Cov(t tau, C), any sign: flip it for v < 0, do not replace it
  if constexpr (F64) {
    const double D = s.Sv1 * rS0, Dx = s.Sx1 * rS0;
    lvv = fma(-D, D, s.Svv * rS0) + (s.Sq * rS0) * (((double)b.tp + D) + ev);
    lxx = fma(-Dx, Dx, s.Sxx * rS0);
    mvx = fma(ev, Dx, -s.Svx * rS0);
  } else {
    lvv = fma(-ev, ev, s.Svv * rS0);
    lxx = fma(-ex, ex, s.Sxx * rS0);
    mvx = fma(ev, ex, -s.Svx * rS0);
  }
  lvx = (v == 0.0) ? 0.0 : (vs < 0.0 ? -mvx : mvx);
}

template <typename T, int NB>
__global__ __launch_bounds__(kBlock) void k_logk_hess(int64_t n, int nbins, const T* __restrict__ vin,
                                                      const T* __restrict__ xin, T* __restrict__ logk,
                                                      T* __restrict__ dv, T* __restrict__ dx, T* __restrict__ dvv,
                                                      T* __restrict__ dxx, T* __restrict__ dvx) {
  if constexpr (sizeof(T) == 8) {
    exp2_table_init();
    __syncthreads();
  }
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int nb = NB > 0 ? NB : nbins;
  const double vs = (double)vin[i];
  const double x = (double)xin[i];
  double lk, lv, lx;
  double lvv = __builtin_nan(""), lxx = __builtin_nan(""), lvx = __builtin_nan("");
  if (!domain_special(vs, x, lk, lv, lx)) {
    const double v = fabs(vs);
    const Bracket b = find_bracket<false>(v, x, margin_of<T>());
    constexpr bool F64 = sizeof(T) == 8;
    BinSums s;
    if constexpr (F64) {
      const double ca = (double)b.tp;  // centres of the FP64 moments
      s = bins_f64<2>(nb, v, x, b.Gx, (double)b.t0, (double)b.t1, ca, coshm1_f64(ca));
    } else {
      s = bins_f32<2>(nb, v, x, b.G, (double)b.t0, (double)b.t1);
    }
    hess_outputs<F64>(vs, v, b, s, nb, lk, lv, lx, lvv, lxx, lvx);
  }
  if (logk) logk[i] = (T)lk;
  if (dv) dv[i] = (T)lv;
  if (dx) dx[i] = (T)lx;
  if (dvv) dvv[i] = (T)lvv;
  if (dxx) dxx[i] = (T)lxx;
  if (dvx) dvx[i] = (T)lvx;
}

// Small batches: kSplit lanes per element.  Every lane of an element's group
// finds the same bracket (the search is short and deterministic, so nothing
// is broadcast), integrates 1/kSplit of the nodes, and the group adds its
// FP64 partial sums with butterfly shuffles; lane 0 of the group writes.
// Lanes past n work on a dummy element so that every lane reaches the shuffles.
constexpr int kSplit = 16;

__device__ __forceinline__ double group_sum(double a) {
#pragma unroll
  for (int m = kSplit / 2; m >= 1; m >>= 1) a += __shfl_xor(a, m);
  return a;
}

// clear (nullable): a counter set to 0 by the first thread (the worklist count
// of a learned-range handle whose small call runs here).
template <typename T, int NB, bool GRAD>
__global__ __launch_bounds__(kBlock) void k_logk_split(int64_t n, int nbins, const T* __restrict__ vin,
                                                       const T* __restrict__ xin, const T* __restrict__ gout,
                                                       T* __restrict__ logk, T* __restrict__ dv,
                                                       T* __restrict__ dx, int* __restrict__ clear) {
  if constexpr (sizeof(T) == 8) {
    exp2_table_init();
    __syncthreads();
  }
  if (clear && blockIdx.x == 0 && threadIdx.x == 0) *clear = 0;
  const int64_t e = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kSplit;
  const int k = (int)(threadIdx.x % kSplit);
  const bool in = e < n;
  const int nb = NB > 0 ? NB : nbins;
  const double vs = in ? (double)vin[e] : 1.0;
  const double x = in ? (double)xin[e] : 1.0;
  double lk, dvv, dxv;
  const bool special = domain_special(vs, x, lk, dvv, dxv);
  const double v = fabs(vs);
  BinSums s{};
  Bracket b{};
  if (!special) {
    b = find_bracket<false>(v, x, margin_of<T>());
    const int m_lo = (k * nb) / kSplit, m_hi = ((k + 1) * nb) / kSplit;
    if constexpr (sizeof(T) == 8)
      s = sub_bins_f64<GRAD ? 1 : 0>(nb, m_lo, m_hi, k == kSplit - 1, v, x, b.Gx, (double)b.t0, (double)b.t1);
    else
      s = sub_bins_f32<GRAD ? 1 : 0>(nb, m_lo, m_hi, k == kSplit - 1, v, x, b.G, (double)b.t0, (double)b.t1);
  }
  const double S0 = group_sum(s.S0);
  const double Sv = GRAD ? group_sum(s.Sv) : 0.0;
  const double Sx = GRAD ? group_sum(s.Sx) : 0.0;
  if (!in || k != 0) return;
  if (!special) {
    const double h = ((double)b.t1 - (double)b.t0) / (double)nb;
    constexpr bool F64 = sizeof(T) == 8;
    lk = b.G + log_of<F64>(h * S0);
    if (GRAD) {
      const double rS0 = rcp_of<F64>(S0);
      dvv = (v == 0.0) ? 0.0 : copysign(Sv * rS0, vs);
      dxv = -Sx * rS0;
    }
  }
  if (GRAD) {
    if (gout) {
      const double go = (double)gout[e];
      dvv *= go;
      dxv *= go;
    }
    dv[e] = (T)dvv;
    dx[e] = (T)dxv;
    if (logk) logk[e] = (T)lk;
  } else {
    logk[e] = (T)lk;
  }
}

// Second derivatives for small batches: the layout of k_logk_split (kSplit
// lanes per element, each summing 1/kSplit of the nodes; the group adds its
// FP64 partial sums with butterfly shuffles) with the sums of k_logk_hess.
template <typename T, int NB>
__global__ __launch_bounds__(kBlock) void k_logk_hess_split(int64_t n, int nbins, const T* __restrict__ vin,
                                                            const T* __restrict__ xin, T* __restrict__ logk,
                                                            T* __restrict__ dv, T* __restrict__ dx,
                                                            T* __restrict__ dvv, T* __restrict__ dxx,
                                                            T* __restrict__ dvx) {
  if constexpr (sizeof(T) == 8) {
    exp2_table_init();
    __syncthreads();
  }
  constexpr bool F64 = sizeof(T) == 8;
  const int64_t e = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kSplit;
  const int k = (int)(threadIdx.x % kSplit);
  const bool in = e < n;
  const int nb = NB > 0 ? NB : nbins;
  const double vs = in ? (double)vin[e] : 1.0;
  const double x = in ? (double)xin[e] : 1.0;
  double lk, lv, lx;
  double lvv = __builtin_nan(""), lxx = __builtin_nan(""), lvx = __builtin_nan("");
  const bool special = domain_special(vs, x, lk, lv, lx);
  const double v = fabs(vs);
  BinSums s{};
  Bracket b{};
  if (!special) {
    b = find_bracket<false>(v, x, margin_of<T>());
    const int m_lo = (k * nb) / kSplit, m_hi = ((k + 1) * nb) / kSplit;
    if constexpr (F64) {
      const double ca = (double)b.tp;
      s = sub_bins_f64<2>(nb, m_lo, m_hi, k == kSplit - 1, v, x, b.Gx, (double)b.t0, (double)b.t1, ca,
                          coshm1_f64(ca));
    } else {
      s = sub_bins_f32<2>(nb, m_lo, m_hi, k == kSplit - 1, v, x, b.G, (double)b.t0, (double)b.t1);
    }
  }
  s.S0 = group_sum(s.S0);
  s.Sv = group_sum(s.Sv);
  s.Sx = group_sum(s.Sx);
  s.Svv = group_sum(s.Svv);
  s.Sxx = group_sum(s.Sxx);
  s.Svx = group_sum(s.Svx);
  if constexpr (F64) {
    s.Sv1 = group_sum(s.Sv1);
    s.Sx1 = group_sum(s.Sx1);
    s.Sq = group_sum(s.Sq);
  }
  if (!in || k != 0) return;
  if (!special) hess_outputs<F64>(vs, v, b, s, nb, lk, lv, lx, lvv, lxx, lvx);
  if (logk) logk[e] = (T)lk;
  if (dv) dv[e] = (T)lv;
  if (dx) dx[e] = (T)lx;
  if (dvv) dvv[e] = (T)lvv;
  if (dxx) dxx[e] = (T)lxx;
  if (dvx) dvx[e] = (T)lvx;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_range(int64_t n, const T* __restrict__ vin, const T* __restrict__ xin,
                                                  T* __restrict__ t0, T* __restrict__ t1, T* __restrict__ tp,
                                                  T* __restrict__ gpk) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double v = fabs((double)vin[i]);
  const double x = (double)xin[i];
  double a, b_, c;
  if (domain_special((double)vin[i], x, a, b_, c)) {
    const T nan_ = (T)__builtin_nan("");
    t0[i] = nan_; t1[i] = nan_;
    if (tp) tp[i] = nan_;
    if (gpk) gpk[i] = nan_;
    return;
  }
  const Bracket b = find_bracket<sizeof(T) == 8>(v, x, margin_of<T>());
  t0[i] = (T)b.t0;
  t1[i] = (T)b.t1;
  if (tp) tp[i] = (T)b.tp;
  if (gpk) gpk[i] = (T)b.G;
}

// grad_v = go * dv, grad_x = go * dx (either output may be NULL).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_backward(int64_t n, const T* __restrict__ go, const T* __restrict__ dv,
                                                     const T* __restrict__ dx, T* __restrict__ gv,
                                                     T* __restrict__ gx) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const T g = go[i];
  if (gv) gv[i] = g * dv[i];
  if (gx) gx[i] = g * dx[i];
}

// Vector-Jacobian product of (d/dv, d/dx) log K with the symmetric Hessian:
//   grad_v = g_dv dvv + g_dx dvx,  grad_x = g_dv dvx + g_dx dxx  (either output,
//   and either upstream gradient, may be NULL).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_hess_vjp(int64_t n, const T* __restrict__ gdv, const T* __restrict__ gdx,
                                                     const T* __restrict__ dvv, const T* __restrict__ dxx,
                                                     const T* __restrict__ dvx, T* __restrict__ gv,
                                                     T* __restrict__ gx) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const T a = gdv ? gdv[i] : (T)0;
  const T b = gdx ? gdx[i] : (T)0;
  const T m = dvx[i];
  if (gv) gv[i] = gdx ? (gdv ? fma(a, dvv[i], b * m) : b * m) : a * dvv[i];
  if (gx) gx[i] = gdv ? (gdx ? fma(a, m, b * dxx[i]) : a * m) : b * dxx[i];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

const char* last_error() { return g_err; }

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  if (!a || !b || abytes == 0 || bbytes == 0) return false;
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

int check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(BESSEL_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return BESSEL_OK;
}

int grid_for(int64_t n, dim3& grid) {
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffLL) return set_error(BESSEL_ERR_ARG, "n = %lld exceeds the launch limit", (long long)n);
  grid = dim3((unsigned)blocks);
  return BESSEL_OK;
}

// Batches of at most this many elements run kSplit lanes per element.
static std::atomic<int64_t> g_split_threshold{kDefaultSplitThreshold};

int64_t split_threshold() { return g_split_threshold.load(std::memory_order_relaxed); }

template <typename T, bool GRAD>
static void launch_logk(dim3 grid, hipStream_t st, int64_t n, int nbins, const T* v, const T* x, const T* go, T* lk,
                        T* dv, T* dx, int* clear, bool force_split) {
  if (force_split || n <= g_split_threshold.load(std::memory_order_relaxed)) {
    const dim3 sgrid((unsigned)((n * kSplit + kBlock - 1) / kBlock));
    switch (nbins) {
      case 64: k_logk_split<T, 64, GRAD><<<sgrid, kBlock, 0, st>>>(n, nbins, v, x, go, lk, dv, dx, clear); break;
      case 128: k_logk_split<T, 128, GRAD><<<sgrid, kBlock, 0, st>>>(n, nbins, v, x, go, lk, dv, dx, clear); break;
      case 256: k_logk_split<T, 256, GRAD><<<sgrid, kBlock, 0, st>>>(n, nbins, v, x, go, lk, dv, dx, clear); break;
      default: k_logk_split<T, 0, GRAD><<<sgrid, kBlock, 0, st>>>(n, nbins, v, x, go, lk, dv, dx, clear); break;
    }
    return;
  }
  switch (nbins) {
    case 64: k_logk<T, 64, GRAD><<<grid, kBlock, 0, st>>>(n, nbins, v, x, go, lk, dv, dx); break;
    case 128: k_logk<T, 128, GRAD><<<grid, kBlock, 0, st>>>(n, nbins, v, x, go, lk, dv, dx); break;
    case 256: k_logk<T, 256, GRAD><<<grid, kBlock, 0, st>>>(n, nbins, v, x, go, lk, dv, dx); break;
    default: k_logk<T, 0, GRAD><<<grid, kBlock, 0, st>>>(n, nbins, v, x, go, lk, dv, dx); break;
  }
}

int logk_newton(int dtype, int64_t n, const void* v, const void* x, const void* go, void* lk, void* dv, void* dx,
                int nbins, bool grad, hipStream_t st, int* clear, bool force_split) {
  dim3 grid;
  int rc = grid_for(n, grid);
  if (rc) return rc;
  if (dtype == BESSEL_F64) {
    if (grad)
      launch_logk<double, true>(grid, st, n, nbins, (const double*)v, (const double*)x, (const double*)go,
                                (double*)lk, (double*)dv, (double*)dx, clear, force_split);
    else
      launch_logk<double, false>(grid, st, n, nbins, (const double*)v, (const double*)x, nullptr, (double*)lk,
                                 nullptr, nullptr, clear, force_split);
  } else {
    if (grad)
      launch_logk<float, true>(grid, st, n, nbins, (const float*)v, (const float*)x, (const float*)go, (float*)lk,
                               (float*)dv, (float*)dx, clear, force_split);
    else
      launch_logk<float, false>(grid, st, n, nbins, (const float*)v, (const float*)x, nullptr, (float*)lk, nullptr,
                                nullptr, clear, force_split);
  }
  return check_launch("k_logk");
}

template <typename T>
static void launch_hess(dim3 grid, hipStream_t st, int64_t n, int nbins, const void* v, const void* x, void* const* o) {
  const T* vv = (const T*)v;
  const T* xx = (const T*)x;
  T* p[6];
  for (int k = 0; k < 6; ++k) p[k] = (T*)o[k];
  if (n <= g_split_threshold.load(std::memory_order_relaxed)) {
    const dim3 sgrid((unsigned)((n * kSplit + kBlock - 1) / kBlock));
    switch (nbins) {
      case 64: k_logk_hess_split<T, 64><<<sgrid, kBlock, 0, st>>>(n, nbins, vv, xx, p[0], p[1], p[2], p[3], p[4], p[5]); break;
      case 128: k_logk_hess_split<T, 128><<<sgrid, kBlock, 0, st>>>(n, nbins, vv, xx, p[0], p[1], p[2], p[3], p[4], p[5]); break;
      case 256: k_logk_hess_split<T, 256><<<sgrid, kBlock, 0, st>>>(n, nbins, vv, xx, p[0], p[1], p[2], p[3], p[4], p[5]); break;
      default: k_logk_hess_split<T, 0><<<sgrid, kBlock, 0, st>>>(n, nbins, vv, xx, p[0], p[1], p[2], p[3], p[4], p[5]); break;
    }
    return;
  }
  switch (nbins) {
    case 64: k_logk_hess<T, 64><<<grid, kBlock, 0, st>>>(n, nbins, vv, xx, p[0], p[1], p[2], p[3], p[4], p[5]); break;
    case 128: k_logk_hess<T, 128><<<grid, kBlock, 0, st>>>(n, nbins, vv, xx, p[0], p[1], p[2], p[3], p[4], p[5]); break;
    case 256: k_logk_hess<T, 256><<<grid, kBlock, 0, st>>>(n, nbins, vv, xx, p[0], p[1], p[2], p[3], p[4], p[5]); break;
    default: k_logk_hess<T, 0><<<grid, kBlock, 0, st>>>(n, nbins, vv, xx, p[0], p[1], p[2], p[3], p[4], p[5]); break;
  }
}

int range_newton(int dtype, int64_t n, const void* v, const void* x, void* t0, void* t1, void* tp, void* gpk,
                 hipStream_t st) {
  dim3 grid;
  int rc = grid_for(n, grid);
  if (rc) return rc;
  if (dtype == BESSEL_F64)
    k_range<double><<<grid, kBlock, 0, st>>>(n, (const double*)v, (const double*)x, (double*)t0, (double*)t1,
                                             (double*)tp, (double*)gpk);
  else
    k_range<float><<<grid, kBlock, 0, st>>>(n, (const float*)v, (const float*)x, (float*)t0, (float*)t1, (float*)tp,
                                            (float*)gpk);
  return check_launch("k_range");
}

}  // namespace bk

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace bk;

static size_t elem_size(int dtype) { return dtype == BESSEL_F64 ? 8 : 4; }

static int common_checks(int dtype, int64_t n, const void* v, const void* x, int range_mode, const bessel_mlp* mlp) {
  if (dtype != BESSEL_F32 && dtype != BESSEL_F64) return set_error(BESSEL_ERR_DTYPE, "dtype %d is not F32/F64", dtype);
  if (n < 0) return set_error(BESSEL_ERR_ARG, "n = %lld < 0", (long long)n);
  if (n > 0 && (!v || !x)) return set_error(BESSEL_ERR_ARG, "v and x must be non-NULL");
  if (range_mode != BESSEL_RANGE_NEWTON && range_mode != BESSEL_RANGE_MLP && range_mode != BESSEL_RANGE_MLP_TABLE)
    return set_error(BESSEL_ERR_RANGE_MODE, "unknown range_mode %d", range_mode);
  const bool learned = range_mode != BESSEL_RANGE_NEWTON;
  if (learned && !mlp) return set_error(BESSEL_ERR_RANGE_MODE, "a learned range_mode needs an mlp");
  if (learned && dtype != BESSEL_F32)
    return set_error(BESSEL_ERR_UNSUPPORTED, "the learned range is provided for F32 only");
  return BESSEL_OK;
}

extern "C" int bessel_logk(int dtype, int64_t n, const void* v, const void* x, void* logk, int nbins, int range_mode,
                           const bessel_mlp* mlp, void* hip_stream) {
  int rc = common_checks(dtype, n, v, x, range_mode, mlp);
  if (rc) return rc;
  if (nbins < BESSEL_MIN_BINS || nbins > BESSEL_MAX_BINS)
    return set_error(BESSEL_ERR_NBINS, "nbins = %d outside [%d, %d]", nbins, BESSEL_MIN_BINS, BESSEL_MAX_BINS);
  if (n == 0) return BESSEL_OK;
  if (!logk) return set_error(BESSEL_ERR_ARG, "logk must be non-NULL");
  const size_t nb = (size_t)n * elem_size(dtype);
  if (overlaps(logk, nb, v, nb) || overlaps(logk, nb, x, nb))
    return set_error(BESSEL_ERR_ALIAS, "logk overlaps an input");
  hipStream_t st = (hipStream_t)hip_stream;
  if (range_mode != BESSEL_RANGE_NEWTON)
    return logk_mlp(n, (const float*)v, (const float*)x, nullptr, (float*)logk, nullptr, nullptr, nbins, false, mlp,
                    range_mode == BESSEL_RANGE_MLP_TABLE, st);
  return logk_newton(dtype, n, v, x, nullptr, logk, nullptr, nullptr, nbins, false, st);
}

extern "C" int bessel_logk_dv_dx(int dtype, int64_t n, const void* v, const void* x, const void* grad_out, void* logk,
                                 void* dv, void* dx, int nbins, int range_mode, const bessel_mlp* mlp,
                                 void* hip_stream) {
  int rc = common_checks(dtype, n, v, x, range_mode, mlp);
  if (rc) return rc;
  if (nbins < BESSEL_MIN_BINS || nbins > BESSEL_MAX_BINS)
    return set_error(BESSEL_ERR_NBINS, "nbins = %d outside [%d, %d]", nbins, BESSEL_MIN_BINS, BESSEL_MAX_BINS);
  if (n == 0) return BESSEL_OK;
  if (!dv || !dx) return set_error(BESSEL_ERR_ARG, "dv and dx must be non-NULL");
  const size_t nb = (size_t)n * elem_size(dtype);
  const void* ins[3] = {v, x, grad_out};
  void* outs[3] = {dv, dx, logk};
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b)
      if (overlaps(outs[a], nb, ins[b], nb)) return set_error(BESSEL_ERR_ALIAS, "an output overlaps an input");
    for (int b = a + 1; b < 3; ++b)
      if (overlaps(outs[a], nb, outs[b], nb)) return set_error(BESSEL_ERR_ALIAS, "two outputs overlap");
  }
  hipStream_t st = (hipStream_t)hip_stream;
  if (range_mode != BESSEL_RANGE_NEWTON)
    return logk_mlp(n, (const float*)v, (const float*)x, (const float*)grad_out, (float*)logk, (float*)dv, (float*)dx,
                    nbins, true, mlp, range_mode == BESSEL_RANGE_MLP_TABLE, st);
  return logk_newton(dtype, n, v, x, grad_out, logk, dv, dx, nbins, true, st);
}

extern "C" int bessel_logk_hess(int dtype, int64_t n, const void* v, const void* x, void* logk, void* dv, void* dx,
                                void* dvv, void* dxx, void* dvx, int nbins, void* hip_stream) {
  int rc = common_checks(dtype, n, v, x, BESSEL_RANGE_NEWTON, nullptr);
  if (rc) return rc;
  if (nbins < BESSEL_MIN_BINS || nbins > BESSEL_MAX_BINS)
    return set_error(BESSEL_ERR_NBINS, "nbins = %d outside [%d, %d]", nbins, BESSEL_MIN_BINS, BESSEL_MAX_BINS);
  if (n == 0) return BESSEL_OK;
  void* outs[6] = {logk, dv, dx, dvv, dxx, dvx};
  bool any = false;
  for (void* o : outs) any = any || (o != nullptr);
  if (!any) return set_error(BESSEL_ERR_ARG, "at least one output must be non-NULL");
  const size_t nb = (size_t)n * elem_size(dtype);
  for (int a = 0; a < 6; ++a) {
    if (overlaps(outs[a], nb, v, nb) || overlaps(outs[a], nb, x, nb))
      return set_error(BESSEL_ERR_ALIAS, "an output overlaps an input");
    for (int b = a + 1; b < 6; ++b)
      if (overlaps(outs[a], nb, outs[b], nb)) return set_error(BESSEL_ERR_ALIAS, "two outputs overlap");
  }
  dim3 grid;
  rc = grid_for(n, grid);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  if (dtype == BESSEL_F64)
    launch_hess<double>(grid, st, n, nbins, v, x, outs);
  else
    launch_hess<float>(grid, st, n, nbins, v, x, outs);
  return check_launch("k_logk_hess");
}

extern "C" int bessel_range(int dtype, int64_t n, const void* v, const void* x, void* t0, void* t1, void* tp,
                            void* logf_peak, int range_mode, const bessel_mlp* mlp, uint8_t* fallback,
                            void* hip_stream) {
  int rc = common_checks(dtype, n, v, x, range_mode, mlp);
  if (rc) return rc;
  if (n == 0) return BESSEL_OK;
  if (!t0 || !t1) return set_error(BESSEL_ERR_ARG, "t0 and t1 must be non-NULL");
  const size_t nb = (size_t)n * elem_size(dtype);
  const void* ins[2] = {v, x};
  void* outs[4] = {t0, t1, tp, logf_peak};
  for (int a = 0; a < 4; ++a) {
    for (int b = 0; b < 2; ++b)
      if (overlaps(outs[a], nb, ins[b], nb)) return set_error(BESSEL_ERR_ALIAS, "an output overlaps an input");
    for (int b = a + 1; b < 4; ++b)
      if (overlaps(outs[a], nb, outs[b], nb)) return set_error(BESSEL_ERR_ALIAS, "two outputs overlap");
    if (fallback && overlaps(outs[a], nb, fallback, (size_t)n))
      return set_error(BESSEL_ERR_ALIAS, "fallback overlaps an output");
  }
  hipStream_t st = (hipStream_t)hip_stream;
  if (range_mode != BESSEL_RANGE_NEWTON)
    return range_mlp(n, (const float*)v, (const float*)x, (float*)t0, (float*)t1, (float*)tp, (float*)logf_peak,
                     fallback, mlp, range_mode == BESSEL_RANGE_MLP_TABLE, st);
  return range_newton(dtype, n, v, x, t0, t1, tp, logf_peak, st);
}

extern "C" int bessel_logk_backward(int dtype, int64_t n, const void* grad_out, const void* dv, const void* dx,
                                    void* grad_v, void* grad_x, void* hip_stream) {
  if (dtype != BESSEL_F32 && dtype != BESSEL_F64) return set_error(BESSEL_ERR_DTYPE, "dtype %d is not F32/F64", dtype);
  if (n < 0) return set_error(BESSEL_ERR_ARG, "n = %lld < 0", (long long)n);
  if (n == 0) return BESSEL_OK;
  if (!grad_out || (grad_v && !dv) || (grad_x && !dx))
    return set_error(BESSEL_ERR_ARG, "grad_out, and dv/dx for each requested gradient, must be non-NULL");
  const size_t nb = (size_t)n * elem_size(dtype);
  const void* ins[3] = {grad_out, dv, dx};
  for (int b = 0; b < 3; ++b)
    if (overlaps(grad_v, nb, ins[b], nb) || overlaps(grad_x, nb, ins[b], nb))
      return set_error(BESSEL_ERR_ALIAS, "an output overlaps an input");
  if (overlaps(grad_v, nb, grad_x, nb)) return set_error(BESSEL_ERR_ALIAS, "grad_v overlaps grad_x");
  dim3 grid;
  int rc = grid_for(n, grid);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  if (dtype == BESSEL_F64)
    k_backward<double><<<grid, kBlock, 0, st>>>(n, (const double*)grad_out, (const double*)dv, (const double*)dx,
                                                (double*)grad_v, (double*)grad_x);
  else
    k_backward<float><<<grid, kBlock, 0, st>>>(n, (const float*)grad_out, (const float*)dv, (const float*)dx,
                                               (float*)grad_v, (float*)grad_x);
  return check_launch("k_backward");
}

extern "C" int bessel_hess_vjp(int dtype, int64_t n, const void* g_dv, const void* g_dx, const void* dvv,
                               const void* dxx, const void* dvx, void* grad_v, void* grad_x, void* hip_stream) {
  if (dtype != BESSEL_F32 && dtype != BESSEL_F64) return set_error(BESSEL_ERR_DTYPE, "dtype %d is not F32/F64", dtype);
  if (n < 0) return set_error(BESSEL_ERR_ARG, "n = %lld < 0", (long long)n);
  if (n == 0) return BESSEL_OK;
  if (!g_dv && !g_dx) return set_error(BESSEL_ERR_ARG, "g_dv and g_dx cannot both be NULL");
  if (!dvx || (g_dv && grad_v && !dvv) || (g_dx && grad_x && !dxx))
    return set_error(BESSEL_ERR_ARG, "dvx, and dvv/dxx where they are used, must be non-NULL");
  const size_t nb = (size_t)n * elem_size(dtype);
  const void* ins[5] = {g_dv, g_dx, dvv, dxx, dvx};
  for (int b = 0; b < 5; ++b)
    if (overlaps(grad_v, nb, ins[b], nb) || overlaps(grad_x, nb, ins[b], nb))
      return set_error(BESSEL_ERR_ALIAS, "an output overlaps an input");
  if (overlaps(grad_v, nb, grad_x, nb)) return set_error(BESSEL_ERR_ALIAS, "grad_v overlaps grad_x");
  dim3 grid;
  int rc = grid_for(n, grid);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  if (dtype == BESSEL_F64)
    k_hess_vjp<double><<<grid, kBlock, 0, st>>>(n, (const double*)g_dv, (const double*)g_dx, (const double*)dvv,
                                                (const double*)dxx, (const double*)dvx, (double*)grad_v,
                                                (double*)grad_x);
  else
    k_hess_vjp<float><<<grid, kBlock, 0, st>>>(n, (const float*)g_dv, (const float*)g_dx, (const float*)dvv,
                                               (const float*)dxx, (const float*)dvx, (float*)grad_v, (float*)grad_x);
  return check_launch("k_hess_vjp");
}

extern "C" int bessel_set_split_threshold(int64_t n, int64_t* previous) {
  if (n < 0) return set_error(BESSEL_ERR_ARG, "threshold %lld < 0", (long long)n);
  if (n > BESSEL_MAX_SPLIT_THRESHOLD)
    return set_error(BESSEL_ERR_ARG, "threshold %lld above %lld", (long long)n, (long long)BESSEL_MAX_SPLIT_THRESHOLD);
  const int64_t old = g_split_threshold.exchange(n);
  if (previous) *previous = old;
  return BESSEL_OK;
}

extern "C" const char* bessel_last_error(void) { return last_error(); }

#define BK_STR2(a) #a
#define BK_STR(a) BK_STR2(a)
extern "C" const char* bessel_version(void) {
  return "libbessel gfx950, HIP " BK_STR(HIP_VERSION_MAJOR) "." BK_STR(HIP_VERSION_MINOR) ", " __VERSION__;
}
