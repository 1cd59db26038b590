// bessel_mlp.hip -- learned bracket predictor (placeholder until the MLP kernels land).
#include <hip/hip_runtime.h>

#include "bessel.h"
#include "bessel_internal.hpp"

namespace bk {

int logk_mlp(int64_t, const float*, const float*, const float*, float*, float*, float*, int, bool, const bessel_mlp*,
             hipStream_t) {
  return set_error(BESSEL_ERR_UNSUPPORTED, "learned range not built yet");
}

int range_mlp(int64_t, const float*, const float*, float*, float*, float*, float*, uint8_t*, const bessel_mlp*,
              hipStream_t) {
  return set_error(BESSEL_ERR_UNSUPPORTED, "learned range not built yet");
}

}  // namespace bk
