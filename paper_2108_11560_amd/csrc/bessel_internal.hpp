// bessel_internal.hpp -- declarations shared by the library's translation units
// (not part of the public ABI in include/bessel.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "bessel.h"

namespace bk {

constexpr int kBlock = 256;  // 4 wave64 per workgroup
// Batches of at most this many elements take the kernels that split each
// element's nodes over 16 lanes (log K and first derivatives, Newton bracket).
constexpr int64_t kDefaultSplitThreshold = 16384;

int set_error(int code, const char* fmt, ...);
const char* last_error();
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes);
int check_launch(const char* what);
int grid_for(int64_t n, dim3& grid);

// Plain Newton-range paths (bessel_kernels.hip).  clear (nullable): a device
// counter the first thread sets to 0; force_split: the kSplit-lanes layout
// whatever the batch-size policy says.
int logk_newton(int dtype, int64_t n, const void* v, const void* x, const void* go, void* lk, void* dv, void* dx,
                int nbins, bool grad, hipStream_t st, int* clear = nullptr, bool force_split = false);
// The batch-size policy: batches of at most this many elements take the
// kSplit-lanes layouts (bessel_set_split_threshold).
int64_t split_threshold();
int range_newton(int dtype, int64_t n, const void* v, const void* x, void* t0, void* t1, void* tp, void* gpk,
                 hipStream_t st);

// Learned-range paths (bessel_mlp.hip), F32 only.
// table: the network's bilinear table instead of its per-element inference.
int logk_mlp(int64_t n, const float* v, const float* x, const float* go, float* lk, float* dv, float* dx, int nbins,
             bool grad, const bessel_mlp* mlp, bool table, hipStream_t st);
// The handle's packed inference operands and its network table, rebuilt on
// st first if the parameters changed (kernel launches only, no allocation).
int mlp_table_operands(const bessel_mlp* mlp, hipStream_t st, const float** Q, const float4** cells);
int range_mlp(int64_t n, const float* v, const float* x, float* t0, float* t1, float* tp, float* gpk,
              uint8_t* fallback, const bessel_mlp* mlp, bool table, hipStream_t st);

}  // namespace bk
