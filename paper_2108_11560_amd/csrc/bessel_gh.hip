// bessel_gh.hip -- per-set sums of log K over shared samples, with the
// gradients of each sum with respect to the set's parameters.
//
// For set i with parameters (lambda, alpha, delta, mu) and samples y_j:
//   v = lambda - 1/2,  r_j = sqrt(delta^2 + (y_j - mu)^2),  x_j = alpha r_j,
//   S_i = sum_j log K_v(x_j)
// (the shape of a generalised-hyperbolic log-likelihood, whose Bessel factor
// motivates the method in the paper's introduction).  Each (i, j) runs the
// FP32 path with derivatives (Sections 2 and 4.1); the chain rule gives
//   dS/dlambda = sum dv,  dS/dalpha = sum dx r,  dS/ddelta = sum dx alpha delta / r,
//   dS/dmu = sum dx alpha (mu - y) / r.
// One block per (set, chunk of kBlock samples): wavefront shuffle sums and an
// LDS sum give one FP64 partial per block; a second kernel adds the partials
// of each set in chunk order (deterministic).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <mutex>

#include "bessel.h"
#include "bessel_device.hpp"
#include "bessel_internal.hpp"
#include "bessel_learned.hpp"

namespace bk {

constexpr int kGhQ = 5;  // sum, d/dlambda, d/dalpha, d/ddelta, d/dmu
constexpr float kMarginGh = 15.9423851528787422f;  // FP32 eps

__device__ __forceinline__ double wave_sum(double a) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) a += __shfl_xor(a, m);
  return a;
}

// TAB: the bracket from the network's table (range mode BESSEL_RANGE_MLP_TABLE;
// Q, cells: the handle's operands), checked after its bins; an element whose
// learned bracket fails the check takes the Newton bracket in the same lane.
template <int NB, bool TAB>
__global__ __launch_bounds__(kBlock) void k_gh_partial(int64_t nsamp, int64_t nchunks, int nbins,
                                                       const float* __restrict__ lam, const float* __restrict__ alpha,
                                                       const float* __restrict__ delta, const float* __restrict__ mu,
                                                       const float* __restrict__ y, const float* __restrict__ Q,
                                                       const float4* __restrict__ cells, double* __restrict__ partial) {
  __shared__ double red[kBlock / 64][kGhQ];
  const int64_t set = (int64_t)blockIdx.x / nchunks;
  const int64_t chunk = (int64_t)blockIdx.x - set * nchunks;
  const int64_t j = chunk * kBlock + threadIdx.x;
  const int nb = NB > 0 ? NB : nbins;
  double c[kGhQ] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (j < nsamp) {
    const double vs = (double)lam[set] - 0.5;
    const double a = (double)alpha[set], d = (double)delta[set], m = (double)mu[set];
    const double dy = (double)y[j] - m;
    const double r = sqrt(fma(d, d, dy * dy));
    const double x = a * r;
    double lk, dv, dx;
    if (!domain_special(vs, x, lk, dv, dx)) {
      const double v = fabs(vs);
      BinSums s;
      double G = 0.0, t0 = 0.0, t1 = 0.0;
      bool ok = false;
      if constexpr (TAB) {
        float z0, z1, y0, y1;
        mlp_features_q(Q, (float)v, (float)x, z0, z1);
        mlp_table(cells, z0, z1, y0, y1);
        LearnedBracket lb;
        ok = learned_bins<1>(Q, v, x, y0, y1, nb, lb, s);
        G = (double)lb.G, t0 = (double)lb.t0, t1 = (double)lb.t1;
      }
      if (!ok) {
        const Bracket b = find_bracket<false>(v, x, kMarginGh);
        s = bins_f32<true>(nb, v, x, b.G, (double)b.t0, (double)b.t1);
        G = b.G, t0 = (double)b.t0, t1 = (double)b.t1;
      }
      const double h = (t1 - t0) / (double)nb;
      const double rS0 = rcp_of<false>(s.S0);
      lk = G + log_of<false>(h * s.S0);
      dv = (v == 0.0) ? 0.0 : copysign(s.Sv * rS0, vs);
      dx = -s.Sx * rS0;
    }
    const double rr = rcp_f64(r);
    c[0] = lk;
    c[1] = dv;
    c[2] = dx * r;
    c[3] = dx * a * d * rr;
    c[4] = -dx * a * dy * rr;
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kGhQ; ++q) {
    const double s = wave_sum(c[q]);
    if ((threadIdx.x & 63) == 0) red[w][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < kGhQ) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) s += red[k][threadIdx.x];
    partial[(int64_t)blockIdx.x * kGhQ + threadIdx.x] = s;
  }
}

__global__ __launch_bounds__(kBlock) void k_gh_final(int64_t nsets, int64_t nchunks, const double* __restrict__ partial,
                                                     const float* __restrict__ gsum, float* __restrict__ sum,
                                                     float* __restrict__ g_lam, float* __restrict__ g_alpha,
                                                     float* __restrict__ g_delta, float* __restrict__ g_mu) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nsets) return;
  double acc[kGhQ] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t c = 0; c < nchunks; ++c)
#pragma unroll
    for (int q = 0; q < kGhQ; ++q) acc[q] += partial[(i * nchunks + c) * kGhQ + q];
  const double g = gsum ? (double)gsum[i] : 1.0;
  sum[i] = (float)acc[0];
  if (g_lam) g_lam[i] = (float)(g * acc[1]);
  if (g_alpha) g_alpha[i] = (float)(g * acc[2]);
  if (g_delta) g_delta[i] = (float)(g * acc[3]);
  if (g_mu) g_mu[i] = (float)(g * acc[4]);
}

// Partials of bessel_gh_logk_sum_noalloc: one record of kGhQ doubles per
// (set, chunk) block, at most kGhScratchBlocks blocks (10 MiB: 1024 sets of
// 65536 samples).  Each GPU holds its own copy for the life of the process;
// host code reaches it only through the address hipGetSymbolAddress returns
// for that GPU (gh_scratch below), never through the array's name.
constexpr int64_t kGhScratchBlocks = BESSEL_GH_NOALLOC_MAX_BLOCKS;
static __device__ __align__(256) double scratch[kGhScratchBlocks * kGhQ];

constexpr int kMaxDevices = 64;
static std::atomic<double*> g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// The device address of `scratch` on the device that runs work queued on st
// (the stream's device, or the current device for the null stream), looked up
// once per device with that device current.
static int gh_scratch(hipStream_t st, double** out) {
  int dev = 0;
  hipError_t e = st ? hipStreamGetDevice(st, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(BESSEL_ERR_HIP, "device of the stream: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(BESSEL_ERR_ARG, "device %d beyond %d", dev, kMaxDevices);
  double* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
    if (!p) {
      int cur = 0;
      e = hipGetDevice(&cur);
      if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
      void* addr = nullptr;
      if (e == hipSuccess) e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
      const hipError_t e2 = (cur != dev) ? hipSetDevice(cur) : hipSuccess;
      if (e == hipSuccess) e = e2;
      if (e != hipSuccess || !addr)
        return set_error(BESSEL_ERR_HIP, "address of the static partials: %s", hipGetErrorString(e));
      p = static_cast<double*>(addr);
      g_scratch_ptr[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return BESSEL_OK;
}

namespace {

// Argument checks shared by both entry points; nblocks receives the number of
// (set, chunk) blocks, i.e. of partial records the call needs.
int gh_checks(int64_t nsets, const float* lam, const float* alpha, const float* delta, const float* mu,
              int64_t nsamp, const float* y, const float* grad_sum, float* sum, float* g_lam, float* g_alpha,
              float* g_delta, float* g_mu, int nbins, int range_mode, const bessel_mlp* mlp, int64_t& nchunks,
              int64_t& nblocks) {
  if (nsets < 0 || nsamp < 0) return set_error(BESSEL_ERR_ARG, "nsets and nsamp must be >= 0");
  if (range_mode == BESSEL_RANGE_MLP)
    return set_error(BESSEL_ERR_UNSUPPORTED, "the per-set sums take the Newton bracket or the network's table");
  if (range_mode != BESSEL_RANGE_NEWTON && range_mode != BESSEL_RANGE_MLP_TABLE)
    return set_error(BESSEL_ERR_RANGE_MODE, "unknown range_mode %d", range_mode);
  if (range_mode == BESSEL_RANGE_MLP_TABLE && !mlp)
    return set_error(BESSEL_ERR_RANGE_MODE, "BESSEL_RANGE_MLP_TABLE needs an mlp");
  if (nbins < BESSEL_MIN_BINS || nbins > BESSEL_MAX_BINS)
    return set_error(BESSEL_ERR_NBINS, "nbins = %d outside [%d, %d]", nbins, BESSEL_MIN_BINS, BESSEL_MAX_BINS);
  nchunks = nsamp > 0 ? (nsamp + kBlock - 1) / kBlock : 1;
  nblocks = 0;
  if (nsets == 0) return BESSEL_OK;
  if (!lam || !alpha || !delta || !mu || !sum || (nsamp > 0 && !y))
    return set_error(BESSEL_ERR_ARG, "lam, alpha, delta, mu, sum and y must be non-NULL");
  const size_t sb = (size_t)nsets * sizeof(float);
  const void* ins[6] = {lam, alpha, delta, mu, grad_sum, y};
  const size_t inb[6] = {sb, sb, sb, sb, sb, (size_t)nsamp * sizeof(float)};
  void* outs[5] = {sum, g_lam, g_alpha, g_delta, g_mu};
  for (int a = 0; a < 5; ++a) {
    for (int b = 0; b < 6; ++b)
      if (overlaps(outs[a], sb, ins[b], inb[b])) return set_error(BESSEL_ERR_ALIAS, "an output overlaps an input");
    for (int b = a + 1; b < 5; ++b)
      if (overlaps(outs[a], sb, outs[b], sb)) return set_error(BESSEL_ERR_ALIAS, "two outputs overlap");
  }
  if (nchunks > 0x7fffffffLL / nsets) return set_error(BESSEL_ERR_ARG, "nsets x nsamp too large for one launch");
  nblocks = nsets * nchunks;
  return BESSEL_OK;
}

template <bool TAB>
void gh_partials(dim3 grid, hipStream_t st, int64_t nsamp, int64_t nchunks, int nbins, const float* lam,
                 const float* alpha, const float* delta, const float* mu, const float* y, const float* Q,
                 const float4* cells, double* partial) {
  switch (nbins) {
    case 64:
      k_gh_partial<64, TAB><<<grid, kBlock, 0, st>>>(nsamp, nchunks, nbins, lam, alpha, delta, mu, y, Q, cells, partial);
      break;
    case 128:
      k_gh_partial<128, TAB><<<grid, kBlock, 0, st>>>(nsamp, nchunks, nbins, lam, alpha, delta, mu, y, Q, cells, partial);
      break;
    case 256:
      k_gh_partial<256, TAB><<<grid, kBlock, 0, st>>>(nsamp, nchunks, nbins, lam, alpha, delta, mu, y, Q, cells, partial);
      break;
    default:
      k_gh_partial<0, TAB><<<grid, kBlock, 0, st>>>(nsamp, nchunks, nbins, lam, alpha, delta, mu, y, Q, cells, partial);
      break;
  }
}

// The two kernels of a call, with the partial records at `partial`
// (nblocks * kGhQ doubles, every one written by k_gh_partial before
// k_gh_final reads it, so nothing needs clearing).  With the table range the
// handle's operands are refreshed first (kernel launches only).
int gh_launch(int64_t nsets, const float* lam, const float* alpha, const float* delta, const float* mu,
              int64_t nsamp, const float* y, const float* grad_sum, float* sum, float* g_lam, float* g_alpha,
              float* g_delta, float* g_mu, int nbins, int range_mode, const bessel_mlp* mlp, int64_t nchunks,
              int64_t nblocks, double* partial, hipStream_t st) {
  const dim3 grid((unsigned)nblocks);
  if (range_mode == BESSEL_RANGE_MLP_TABLE) {
    const float* Q = nullptr;
    const float4* cells = nullptr;
    const int rc = mlp_table_operands(mlp, st, &Q, &cells);
    if (rc) return rc;
    gh_partials<true>(grid, st, nsamp, nchunks, nbins, lam, alpha, delta, mu, y, Q, cells, partial);
  } else {
    gh_partials<false>(grid, st, nsamp, nchunks, nbins, lam, alpha, delta, mu, y, nullptr, nullptr, partial);
  }
  int rc = check_launch("k_gh_partial");
  if (rc) return rc;
  k_gh_final<<<dim3((unsigned)((nsets + kBlock - 1) / kBlock)), kBlock, 0, st>>>(nsets, nchunks, partial, grad_sum,
                                                                             sum, g_lam, g_alpha, g_delta, g_mu);
  return check_launch("k_gh_final");
}

}  // namespace

}  // namespace bk

using namespace bk;

extern "C" int bessel_gh_logk_sum(int64_t nsets, const float* lam, const float* alpha, const float* delta,
                                  const float* mu, int64_t nsamp, const float* y, const float* grad_sum, float* sum,
                                  float* g_lam, float* g_alpha, float* g_delta, float* g_mu, int nbins,
                                  int range_mode, const bessel_mlp* mlp, void* hip_stream) {
  int64_t nchunks = 0, nblocks = 0;
  int rc = gh_checks(nsets, lam, alpha, delta, mu, nsamp, y, grad_sum, sum, g_lam, g_alpha, g_delta, g_mu, nbins,
                     range_mode, mlp, nchunks, nblocks);
  if (rc || nsets == 0) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  double* partial = nullptr;
  hipError_t e = hipMallocAsync((void**)&partial, (size_t)nblocks * kGhQ * sizeof(double), st);
  if (e != hipSuccess) return set_error(BESSEL_ERR_HIP, "partials: %s", hipGetErrorString(e));
  rc = gh_launch(nsets, lam, alpha, delta, mu, nsamp, y, grad_sum, sum, g_lam, g_alpha, g_delta, g_mu, nbins,
                 range_mode, mlp, nchunks, nblocks, partial, st);
  e = hipFreeAsync(partial, st);
  if (rc == BESSEL_OK && e != hipSuccess) return set_error(BESSEL_ERR_HIP, "partials: %s", hipGetErrorString(e));
  return rc;
}

extern "C" int bessel_gh_logk_sum_noalloc(int64_t nsets, const float* lam, const float* alpha, const float* delta,
                                          const float* mu, int64_t nsamp, const float* y, const float* grad_sum,
                                          float* sum, float* g_lam, float* g_alpha, float* g_delta, float* g_mu,
                                          int nbins, int range_mode, const bessel_mlp* mlp, void* hip_stream) {
  int64_t nchunks = 0, nblocks = 0;
  int rc = gh_checks(nsets, lam, alpha, delta, mu, nsamp, y, grad_sum, sum, g_lam, g_alpha, g_delta, g_mu, nbins,
                     range_mode, mlp, nchunks, nblocks);
  if (rc || nsets == 0) return rc;
  if (nblocks > kGhScratchBlocks)
    return set_error(BESSEL_ERR_ARG, "nsets x ceil(nsamp / %d) = %lld exceeds the %lld records of the static partials",
                     kBlock, (long long)nblocks, (long long)kGhScratchBlocks);
  hipStream_t st = (hipStream_t)hip_stream;
  double* partial = nullptr;
  rc = gh_scratch(st, &partial);
  if (rc) return rc;
  return gh_launch(nsets, lam, alpha, delta, mu, nsamp, y, grad_sum, sum, g_lam, g_alpha, g_delta, g_mu, nbins,
                   range_mode, mlp, nchunks, nblocks, partial, st);
}
