// Host-side launchers of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include "kargs.h"

namespace qx {

// Work-group tile shapes of the matrix-core GEMMs (qx_gemm_tile).  The P3 / P4 shapes are the
// software-pipelined split-precision form with 3 / 4 LDS stages (one work-group per CU);
// complex64 runs them as the plain 128x128 shape.  THIN is the memory-bound kernel for
// products with a side of at most 32 and K at most 32 (other products run their default tile).
enum GemmTile {
  GEMM_TILE_128x128 = 0,
  GEMM_TILE_64x64 = 1,
  GEMM_TILE_128x64 = 2,
  GEMM_TILE_64x128 = 3,
  GEMM_TILE_256x128 = 4,
  GEMM_TILE_128x256 = 5,
  GEMM_TILE_128x128P3 = 6,
  GEMM_TILE_128x128P4 = 7,
  GEMM_TILE_THIN = 8,  // memory-bound thin products (gemm_thin_fits), any precision
  GEMM_N_TILES = 9
};
inline void gemm_tile_dims(int tile, int& bm, int& bn) {
  static const int d[GEMM_N_TILES][2] = {{128, 128}, {64, 64}, {128, 64}, {64, 128}, {256, 128},
                                         {128, 256}, {128, 128}, {128, 128}, {32, 256}};
  bm = d[tile][0];
  bn = d[tile][1];
}
// K the split BF16 / FP16 tile kernels accept (8, or a multiple of 16)
inline bool gemm_split_k_ok(const GemmArgs& a) { return a.K % 16 == 0 || a.K == 8; }
inline bool gemm_tile_pipelined(int tile) { return tile == GEMM_TILE_128x128P3 || tile == GEMM_TILE_128x128P4; }
// The thin kernel's domain: one side of at most 32 rows and K at most 32.
bool gemm_thin_fits(const GemmArgs& a);
hipError_t launch_gemm_thin(const GemmArgs& a, hipStream_t s);
// Default tile for a product of the given sizes (used without autotuning).
int gemm_default_tile(int64_t M, int64_t N);

hipError_t launch_simt(const SimtArgs& a, hipStream_t s);
hipError_t launch_gemm(const GemmArgs& a, int precision, int tile, hipStream_t s);
hipError_t launch_gemm_c64(const GemmArgs& a, int tile, hipStream_t s);
hipError_t launch_gemm_bf16(const GemmArgs& a, int tile, hipStream_t s);  // operands stored split BF16
hipError_t launch_gemm_fp16(const GemmArgs& a, int tile, hipStream_t s);  // operands stored split FP16
hipError_t launch_dot(const DotArgs& a, hipStream_t s);
bool dot_outer_shape(const DotArgs& a, int& nfa, int& nfb);  // k_dot_outer applies (needs a.part)
void permute_setup(PermArgs& a);  // fills the tile / outer-bit fields from rank and in_pos
void gemm_args_setup(GemmArgs& g);  // fills the epilogue bit order and the k-tile steps
hipError_t launch_permute(const PermArgs& a, hipStream_t s);
hipError_t launch_slice_sum(const SliceSumArgs& a, hipStream_t s);
hipError_t launch_gather(const GatherArgs& a, hipStream_t s);
hipError_t launch_split_planes(const SplitPlanesArgs& a, hipStream_t s);
hipError_t launch_split_inplace(const SplitInplaceArgs& a, hipStream_t s);  // n % 8 == 0
hipError_t launch_block_init(const BlockArgs& a, hipStream_t s);
hipError_t launch_block_advance(const BlockArgs& a, hipStream_t s);
hipError_t launch_block_finish(const BlockArgs& a, double* amp, hipStream_t s);
hipError_t launch_absmax(const AbsmaxArgs& a, hipStream_t s);  // grid <= 1024 work-groups
hipError_t launch_scale_from_max(const ScaleFromMaxArgs& a, hipStream_t s);
constexpr int ABSMAX_PARTIALS = 1024;

}  // namespace qx
