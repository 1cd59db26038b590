// valu_rates.hip -- issue rates of the instruction classes the log K kernels
// are built from, on the GPU at hand (gfx950).
//
// The roofline of the kernels counts VALU work in lane-slots: one full-rate
// VALU instruction on one lane is one slot, and the peak is
// CUs x 64 lanes x clock.  This program measures, per instruction class, how
// many lane-operations per clock per CU the chip sustains, which gives each
// class its slot cost (64 / rate).  Every kernel runs 8 independent dependent
// chains per lane in 256-thread blocks, enough waves to fill every SIMD, and
// stores its chains so nothing is folded away.  The MFMA entry counts flops of
// v_mfma_f32_16x16x32_bf16 (4 independent accumulators per wavefront).
//
// Output: one JSON object per line.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kChains = 8;
constexpr int kIter = 2048;
constexpr int kThreads = 256;
constexpr int kBlocks = 8192;

typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));

enum Op {
  FMA_F32,
  FMA_F64,
  MUL_F64,
  ADD_F64,
  EXP_F32,
  LOG_F32,
  RCP_F32,
  SQRT_F32,
  RCP_F64,
  FMA64x4_EXP32,  // 4 FP64 FMAs and one FP32 exp per step, independent chains
  SIGMOID,        // 1 / (1 + 2^a): exp, add, rcp
  LDEXP_F64,      // x 2^k (k = 0 at run time, so the chain keeps its value)
  EXP_F16,        // v_exp_f16
  RCP_F16,        // v_rcp_f16
  SIGMOID_F16X2,  // two activations in half precision: pack, exp, add, rcp
  kNumOps
};

template <int OP>
__global__ __launch_bounds__(kThreads) void k_rate(float* __restrict__ of, double* __restrict__ od, float pf,
                                                  double pd, int pk) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  float af[kChains];
  double ad[kChains];
  _Float16 ah[kChains];
  float ag[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    af[i] = 0.5f + 0.01f * (float)(i + (gid & 7));
    ad[i] = 0.5 + 0.01 * (double)(i + (gid & 7));
    ah[i] = (_Float16)af[i];
    ag[i] = -af[i];
  }
  for (int it = 0; it < kIter; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
      if (OP == FMA_F32) af[i] = fmaf(af[i], pf, 1e-7f);
      if (OP == FMA_F64) ad[i] = fma(ad[i], pd, 1e-7);
      if (OP == MUL_F64) ad[i] = ad[i] * pd;
      if (OP == ADD_F64) ad[i] = ad[i] + pd;
      if (OP == EXP_F32) af[i] = __builtin_amdgcn_exp2f(-af[i]);
      if (OP == LOG_F32) af[i] = __builtin_amdgcn_logf(af[i] + 1.0f);
      if (OP == RCP_F32) af[i] = __builtin_amdgcn_rcpf(af[i]);
      if (OP == SQRT_F32) af[i] = __builtin_amdgcn_sqrtf(af[i]);
      if (OP == RCP_F64) ad[i] = __builtin_amdgcn_rcp(ad[i]);
      if (OP == FMA64x4_EXP32) {
        ad[i] = fma(ad[i], pd, 1e-7);
        ad[i] = fma(ad[i], pd, 1e-7);
        ad[i] = fma(ad[i], pd, 1e-7);
        ad[i] = fma(ad[i], pd, 1e-7);
        af[i] = __builtin_amdgcn_exp2f(-af[i]);
      }
      if (OP == SIGMOID) af[i] = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(af[i]));
      if (OP == LDEXP_F64) ad[i] = __builtin_amdgcn_ldexp(ad[i], pk);
      if (OP == EXP_F16) ah[i] = __builtin_elementwise_exp2(-ah[i]);
      if (OP == RCP_F16) ah[i] = __builtin_amdgcn_rcph(ah[i]);
      if (OP == SIGMOID_F16X2) {
        const h16x2 p = __builtin_bit_cast(h16x2, __builtin_amdgcn_cvt_pkrtz(af[i], ag[i]));
        h16x2 e = __builtin_elementwise_exp2(p);
        e = e + (h16x2){(_Float16)1.0f, (_Float16)1.0f};
        af[i] = (float)__builtin_amdgcn_rcph(e[0]);
        ag[i] = (float)__builtin_amdgcn_rcph(e[1]);
      }
    }
  }
  float sf = 0.0f;
  double sd = 0.0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    sf += af[i] + ag[i] + (float)ah[i];
    sd += ad[i];
  }
  of[gid] = sf;
  od[gid] = sd;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaIter = 4096;

// VALU_WORK: also one exp per accumulator element per step on independent
// values, to see whether matrix-core work and VALU work overlap.
template <bool VALU_WORK>
__global__ __launch_bounds__(kThreads) void k_mfma(float* __restrict__ of, float pf) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  bf16x8 a, b;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)(0.01f * (float)((gid + j) & 15));
    b[j] = (__bf16)(0.02f * (float)((gid + 3 * j) & 15));
  }
  f32x4 acc[4];
  float e[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc[c][r] = 0.0f;
      e[c][r] = pf * (float)(c + r);
    }
  for (int it = 0; it < kMfmaIter; ++it) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
      if (VALU_WORK)
#pragma unroll
        for (int r = 0; r < 4; ++r) e[c][r] = __builtin_amdgcn_exp2f(-e[c][r]);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) s += acc[c][r] + e[c][r];
  of[gid] = s;
}

int g_cus = 0;
double g_clock_hz = 0.0;

template <typename F>
float best_ms(F launch) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0f;
  launch();
  if (hipDeviceSynchronize() != hipSuccess) return -1.0f;
  float best = 1e30f;
  for (int r = 0; r < 5; ++r) {
    float ms = 0.0f;
    if (hipEventRecord(a, nullptr) != hipSuccess) return -1.0f;
    launch();
    if (hipEventRecord(b, nullptr) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess)
      return -1.0f;
    if (ms < best) best = ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

void report(const char* name, double ops, float ms, const char* unit_note) {
  const double rate = ops / (ms * 1e-3);
  const double per_cu_clk = rate / ((double)g_cus * g_clock_hz);
  printf("{\"op\": \"%s\", \"ms\": %.4f, \"lane_ops_per_s\": %.5g, \"lane_ops_per_clk_per_cu\": %.2f, "
         "\"slots\": %.3f, \"note\": \"%s\"}\n",
         name, ms, rate, per_cu_clk, 64.0 / per_cu_clk, unit_note);
}

template <int OP>
int run_rate(const char* name, int ops_per_step, float* of, double* od, const char* note) {
  const float ms = best_ms([&] { k_rate<OP><<<kBlocks, kThreads>>>(of, od, 0.999999f, 0.999999, 0); });
  if (ms < 0.0f) return 1;
  report(name, (double)kBlocks * kThreads * kIter * kChains * ops_per_step, ms, note);
  return 0;
}

template <bool VALU_WORK>
int run_mfma(const char* name, float* of) {
  const float ms = best_ms([&] { k_mfma<VALU_WORK><<<kBlocks, kThreads>>>(of, 0.5f); });
  if (ms < 0.0f) return 1;
  const double waves = (double)kBlocks * kThreads / 64.0;
  const double flops = waves * kMfmaIter * 4 * (16.0 * 16.0 * 32.0 * 2.0);
  printf("{\"op\": \"%s\", \"ms\": %.4f, \"tflops\": %.2f, \"flops_per_clk_per_cu\": %.1f}\n", name, ms,
         flops / (ms * 1e-3) * 1e-12, flops / (ms * 1e-3) / ((double)g_cus * g_clock_hz));
  return 0;
}

}  // namespace

int main() {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, 0) != hipSuccess) {
    fprintf(stderr, "no HIP device\n");
    return 1;
  }
  g_cus = p.multiProcessorCount;
  g_clock_hz = (double)p.clockRate * 1e3;
  printf("{\"device\": \"%s\", \"cus\": %d, \"clock_hz\": %.0f}\n", p.gcnArchName, g_cus, g_clock_hz);
  const size_t n = (size_t)kBlocks * kThreads;
  float* of = nullptr;
  double* od = nullptr;
  if (hipMalloc((void**)&of, n * sizeof(float)) != hipSuccess) return 1;
  if (hipMalloc((void**)&od, n * sizeof(double)) != hipSuccess) return 1;
  int rc = 0;
  rc |= run_rate<FMA_F32>("v_fma_f32", 1, of, od, "");
  rc |= run_rate<FMA_F64>("v_fma_f64", 1, of, od, "");
  rc |= run_rate<MUL_F64>("v_mul_f64", 1, of, od, "");
  rc |= run_rate<ADD_F64>("v_add_f64", 1, of, od, "");
  rc |= run_rate<EXP_F32>("v_exp_f32", 1, of, od, "");
  rc |= run_rate<LOG_F32>("v_log_f32 (+ v_add_f32)", 1, of, od, "one op per step counted: the add is extra");
  rc |= run_rate<RCP_F32>("v_rcp_f32", 1, of, od, "");
  rc |= run_rate<SQRT_F32>("v_sqrt_f32", 1, of, od, "");
  rc |= run_rate<RCP_F64>("v_rcp_f64", 1, of, od, "");
  rc |= run_rate<FMA64x4_EXP32>("4 v_fma_f64 + 1 v_exp_f32", 5, of, od,
                                "5 ops per step: slots > 1 means the exp does not overlap the FMAs");
  rc |= run_rate<SIGMOID>("1/(1+2^a): exp + add + rcp", 1, of, od, "slots per activation");
  rc |= run_rate<LDEXP_F64>("v_ldexp_f64", 1, of, od, "");
  rc |= run_rate<EXP_F16>("v_exp_f16", 1, of, od, "");
  rc |= run_rate<RCP_F16>("v_rcp_f16", 1, of, od, "");
  rc |= run_rate<SIGMOID_F16X2>("2 x 1/(1+2^a) in half precision (with conversions)", 2, of, od,
                                "slots per activation");
  rc |= run_mfma<false>("v_mfma_f32_16x16x32_bf16", of);
  rc |= run_mfma<true>("v_mfma_f32_16x16x32_bf16 + 4 v_exp_f32 per MFMA", of);
  (void)hipFree(of);
  (void)hipFree(od);
  return rc;
}
