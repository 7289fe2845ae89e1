// Host-side launchers of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include "kargs.h"

namespace qx {

enum GemmTile { GEMM_TILE_128x128 = 0, GEMM_TILE_64x64 = 1 };

hipError_t launch_simt(const SimtArgs& a, hipStream_t s);
hipError_t launch_gemm(const GemmArgs& a, int precision, int tile, hipStream_t s);
hipError_t launch_dot(const DotArgs& a, hipStream_t s);
void permute_setup(PermArgs& a);
void gemm_epilogue_setup(GemmArgs& g);  // fills ep_bit from the output strides  // fills the tile / outer-bit fields from rank and in_pos
hipError_t launch_permute(const PermArgs& a, hipStream_t s);
hipError_t launch_slice_sum(const SliceSumArgs& a, hipStream_t s);
hipError_t launch_gather(const GatherArgs& a, hipStream_t s);
hipError_t launch_absmax(const AbsmaxArgs& a, hipStream_t s);  // grid <= 1024 work-groups
constexpr int ABSMAX_PARTIALS = 1024;

}  // namespace qx
