// Complex GEMM on FP32 matrix cores: kernel and launchers (complex64 path).
#include "gemm_common.h"

namespace qx {

// ---------------------------------------------------------------------------
// Complex GEMM on FP32 matrix cores (v_mfma_f32_32x32x2_f32).
// Work-group tile BM x BN, 4 waves in a 2x2 grid, K tile of 16 complex values.
// Both operand tiles are staged in LDS as [row][k] (k contiguous), so each lane
// fetches its 8 consecutive k values with wide LDS reads.  Lane group g = l/32
// owns k in [8g, 8g+8); step s of the 8 MFMA steps uses k = 8g + s for both
// operands, which is a valid split of the k-sum.  A complex product is four
// real MFMAs into separate real / imaginary accumulators.
// ---------------------------------------------------------------------------
// Tiles of 128x64 up to 128x128 are held to 256 registers per lane (accumulators in VGPRs), so two
// work-groups share a CU: at 128x128 this took the c64 products from one to two waves per SIMD.
template <int BM, int BN, bool A_KC, bool B_KC>
__global__ __launch_bounds__(256, (BM * BN > 64 * 64 && BM * BN <= 128 * 128) ? 2 : 1) void k_gemm_f32(GemmArgs p) {
  constexpr int BK = 16;
  constexpr int PITCH = BK + 2;            // complex per LDS row (+16 B against bank conflicts)
  constexpr int WM = BM / 2, WN = BN / 2;  // wave tile
  constexpr int FM = WM / 32, FN = WN / 32;
  using LA = TileLoader<BM, A_KC>;
  using LB = TileLoader<BN, B_KC>;
  // one LDS area: double-buffered operand tiles, reused by the epilogue's
  // per-wave 32 x 33 staging blocks
  constexpr int SA = 2 * BM * PITCH, SB = 2 * BN * PITCH, SE = 4 * 32 * 33;
  __shared__ __attribute__((aligned(16))) QxCplx smem[(SA + SB) > SE ? (SA + SB) : SE];
  QxCplx (*As)[BM * PITCH] = reinterpret_cast<QxCplx (*)[BM * PITCH]>(smem);
  QxCplx (*Bs)[BN * PITCH] = reinterpret_cast<QxCplx (*)[BN * PITCH]>(smem + SA);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const TileCoord tc = tile_coord(p, BM, BN);
  const QxCplx* __restrict__ A = p.a + tc.aoff;
  const QxCplx* __restrict__ B = p.b + tc.boff;
  const int64_t m0 = tc.tm * BM, n0 = tc.tn * BN;

  const OperandView va = view_a(p, A), vb = view_b(p, B);
  LA la;
  LB lb;
  la.init(va, m0, tid);
  lb.init(vb, n0, tid);
  QxCplx ra[LA::P][8], rb[LB::P][8];
  int64_t kao = 0, kbo = 0;  // offsets of the k tile last loaded
  auto load_tiles = [&](int64_t k0) {
    la.load(va, k0, kao, ra);
    lb.load(vb, k0, kbo, rb);
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int ps = 0; ps < LA::P; ++ps) {
      const int c = tid + ps * 256;
      if (c < LA::CH) {
        int r, kg;
        LA::row_kg(c, r, kg);
        QxCplx* dst = &As[buf][r * PITCH + kg * 8];
#pragma unroll
        for (int j = 0; j < 8; j += 2)
          *(v4f*)(dst + j) = v4f{ra[ps][j].x, ra[ps][j].y, ra[ps][j + 1].x, ra[ps][j + 1].y};
      }
    }
#pragma unroll
    for (int ps = 0; ps < LB::P; ++ps) {
      const int c = tid + ps * 256;
      if (c < LB::CH) {
        int r, kg;
        LB::row_kg(c, r, kg);
        QxCplx* dst = &Bs[buf][r * PITCH + kg * 8];
#pragma unroll
        for (int j = 0; j < 8; j += 2)
          *(v4f*)(dst + j) = v4f{rb[ps][j].x, rb[ps][j].y, rb[ps][j + 1].x, rb[ps][j + 1].y};
      }
    }
  };

  v16f cr[FM][FN], ci[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      cr[a][b] = v16f{0};
      ci[a][b] = v16f{0};
    }

  const int64_t nk = (p.K + BK - 1) / BK;
  load_tiles(0);
  store_tiles(0);
  __syncthreads();
  const int lrow = lane & 31, g = lane >> 5;
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nk) {
      const int z = __builtin_ctzll(~(uint64_t)kt);
      kao += p.a_kinc[z];
      kbo += p.b_kinc[z];
      load_tiles((kt + 1) * BK);
    }
    QxCplx fa[FM][8], fb[FN][8];
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const QxCplx* src = &As[buf][(wm * WM + a * 32 + lrow) * PITCH + g * 8];
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        v4f v = *(const v4f*)(src + j);
        fa[a][j] = {v[0], v[1]};
        fa[a][j + 1] = {v[2], v[3]};
      }
    }
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      const QxCplx* src = &Bs[buf][(wn * WN + b * 32 + lrow) * PITCH + g * 8];
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        v4f v = *(const v4f*)(src + j);
        fb[b][j] = {v[0], v[1]};
        fb[b][j + 1] = {v[2], v[3]};
      }
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          cr[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[a][s].x, fb[b][s].x, cr[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          ci[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[a][s].x, fb[b][s].y, ci[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          cr[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(-fa[a][s].y, fb[b][s].y, cr[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          ci[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[a][s].y, fb[b][s].x, ci[a][b], 0, 0, 0);
    }
    if (kt + 1 < nk) store_tiles(buf ^ 1);
    __syncthreads();
  }

  const OutMap om = out_map(p, m0, n0);
  store_blocks<FM, FN, WM, WN, false, 0>(p, tc.coff, om, m0, n0, wm, wn, lane, cr, ci, 1.f, smem + wave * (32 * 33));
}

template <int BM, int BN>
static hipError_t launch_f32(const GemmArgs& a, hipStream_t s) {
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  const int64_t nwg = tiles * (int64_t)a.n_items * (1LL << a.nh);
  if (nwg <= 0) return hipSuccess;
  if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool akc = gemm_a_kc(a), bkc = gemm_b_kc(a);
  dim3 grid((unsigned)nwg), block(256);
  if (akc && bkc) hipLaunchKernelGGL((k_gemm_f32<BM, BN, true, true>), grid, block, 0, s, a);
  else if (akc) hipLaunchKernelGGL((k_gemm_f32<BM, BN, true, false>), grid, block, 0, s, a);
  else if (bkc) hipLaunchKernelGGL((k_gemm_f32<BM, BN, false, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_gemm_f32<BM, BN, false, false>), grid, block, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gemm_c64(const GemmArgs& a, int tile, hipStream_t s) {
  switch (tile) {
    case GEMM_TILE_64x64: return launch_f32<64, 64>(a, s);
    case GEMM_TILE_128x64: return launch_f32<128, 64>(a, s);
    case GEMM_TILE_64x128: return launch_f32<64, 128>(a, s);
    case GEMM_TILE_256x128: return launch_f32<256, 128>(a, s);
    case GEMM_TILE_128x256: return launch_f32<128, 256>(a, s);
    default: return launch_f32<128, 128>(a, s);
  }
}

}  // namespace qx
