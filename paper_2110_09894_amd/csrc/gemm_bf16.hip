// Split-precision complex GEMM, BF16 hi+lo instantiations.
#include "gemm_split.h"

namespace qx {
hipError_t launch_gemm_bf16(const GemmArgs& a, int tile, hipStream_t s) {
  return launch_split_tile<QX_SPLIT_BF16>(a, tile, s);
}
}  // namespace qx
