// ozaki.hip -- split-form dd Rgemm (placeholder until the kernels land).
#include <hip/hip_runtime.h>

#include "../../include/mpdd.h"
#include "kernels.hpp"

namespace mpdd {

int ozaki_gemm(const void*, bool, bool, int64_t, int64_t, int64_t, double, double, const double*,
               const double*, int64_t, const double*, const double*, int64_t, double, double,
               double*, double*, int64_t, hipStream_t) {
  return MPDD_ERR_UNSUPPORTED;
}

}  // namespace mpdd
