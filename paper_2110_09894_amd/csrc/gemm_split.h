// Split-precision complex GEMM kernel template (internal header).
#pragma once
#include "gemm_common.h"

#include <type_traits>

namespace qx {

// ---------------------------------------------------------------------------
// Split-precision complex GEMM on BF16 / FP16 matrix cores.
// Each FP32 value x is split into hi = round(x) and lo = round(x - hi) in the
// 16-bit format when the tile is staged in LDS, and
//   A B ~= Ah Bh + Ah Bl + Al Bh
// is accumulated in FP32 (v_mfma_f32_32x32x16_{bf16,f16}).  For FP16 both
// operands are first scaled by powers of two that bring their largest
// magnitude near 2^14 (exact, undone in the epilogue).  LDS holds four planes
// per operand (re hi, re lo, im hi, im lo) as [row][k]; lane group g = l/32
// supplies k in [8g, 8g+8) of one 16-wide step for both operands.
// ---------------------------------------------------------------------------
template <int PREC> struct Half16;
template <> struct Half16<QX_SPLIT_BF16> {
  typedef __bf16 T;
  typedef __bf16 V8 __attribute__((ext_vector_type(8)));
  __device__ static inline T cvt(float x) { return (T)x; }
  __device__ static inline v16f mfma(V8 a, V8 b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Half16<QX_SPLIT_FP16> {
  typedef _Float16 T;
  typedef _Float16 V8 __attribute__((ext_vector_type(8)));
  __device__ static inline T cvt(float x) { return (T)x; }
  __device__ static inline v16f mfma(V8 a, V8 b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <int BM, int BN, bool A_KC, bool B_KC, int PREC>
__global__ __launch_bounds__(256) void k_gemm_split(GemmArgs p) {
  using H = Half16<PREC>;
  using T = typename H::T;
  using V8 = typename H::V8;
  constexpr int BK = 16;
  constexpr int P16 = BK + 8;              // 16-bit elements per LDS row (+16 B pad)
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 32, FN = WN / 32;
  using LA = TileLoader<BM, A_KC>;
  using LB = TileLoader<BN, B_KC>;
  // one LDS area: double-buffered hi/lo operand planes, reused by the
  // epilogue's per-wave 32 x 33 complex staging blocks
  constexpr int SA = 2 * 4 * BM * P16, SB = 2 * 4 * BN * P16;     // 16-bit elements
  constexpr int SE = 4 * 32 * 33 * 4;                               // complex64 as 16-bit units
  __shared__ __attribute__((aligned(16))) T smem[(SA + SB) > SE ? (SA + SB) : SE];
  T (*As)[4][BM * P16] = reinterpret_cast<T (*)[4][BM * P16]>(smem);
  T (*Bs)[4][BN * P16] = reinterpret_cast<T (*)[4][BN * P16]>(smem + SA);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const TileCoord tc = tile_coord(p, BM, BN);
  const QxCplx* __restrict__ A = p.a + tc.aoff;
  const QxCplx* __restrict__ B = p.b + tc.boff;
  const int64_t m0 = tc.tm * BM, n0 = tc.tn * BN;
  const float sa = p.a_scale ? p.a_scale[0] : 1.f;
  const float sb = p.b_scale ? p.b_scale[0] : 1.f;

  const OperandView va = view_a(p, A), vb = view_b(p, B);
  LA la;
  LB lb;
  la.init(va, m0, tid);
  lb.init(vb, n0, tid);
  // PF register sets: with two, tile t lives in set t & 1 and global loads run two
  // k tiles ahead; the 256-wide tiles keep one set (two would spill)
  constexpr int PF = (BM * BN > 128 * 128) ? 1 : 2;
  QxCplx ra[PF][LA::P][8], rb[PF][LB::P][8];
  auto load_tiles = [&](int64_t k0, auto set) {
    la.load(va, k0, ra[decltype(set)::value % PF]);
    lb.load(vb, k0, rb[decltype(set)::value % PF]);
  };
  // split 8 complex values into the four planes and store 16 bytes per plane
  auto split_store = [&](T* p0, T* p1, T* p2, T* p3, const QxCplx (&v)[8], float sc) {
    V8 rh, rl, ih, il;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float xr = v[j].x * sc, xi = v[j].y * sc;
      const T hr = H::cvt(xr), hi = H::cvt(xi);
      rh[j] = hr;
      rl[j] = H::cvt(xr - (float)hr);
      ih[j] = hi;
      il[j] = H::cvt(xi - (float)hi);
    }
    *(V8*)p0 = rh;
    *(V8*)p1 = rl;
    *(V8*)p2 = ih;
    *(V8*)p3 = il;
  };
  auto store_tiles = [&](int buf, auto set) {
    constexpr int S = decltype(set)::value;
#pragma unroll
    for (int ps = 0; ps < LA::P; ++ps) {
      const int c = tid + ps * 256;
      if (c < LA::CH) {
        int r, kg;
        LA::row_kg(c, r, kg);
        const int o = r * P16 + kg * 8;
        split_store(&As[buf][0][o], &As[buf][1][o], &As[buf][2][o], &As[buf][3][o], ra[S % PF][ps], sa);
      }
    }
#pragma unroll
    for (int ps = 0; ps < LB::P; ++ps) {
      const int c = tid + ps * 256;
      if (c < LB::CH) {
        int r, kg;
        LB::row_kg(c, r, kg);
        const int o = r * P16 + kg * 8;
        split_store(&Bs[buf][0][o], &Bs[buf][1][o], &Bs[buf][2][o], &Bs[buf][3][o], rb[S % PF][ps], sb);
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
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  load_tiles(0, S0{});
  if (PF == 1) {
    store_tiles(0, S0{});
  } else {
    if (nk > 1) load_tiles(BK, S1{});
    store_tiles(0, S0{});
  }
  __syncthreads();
  const int lrow = lane & 31, g = lane >> 5;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  // One k tile from LDS buffer S: prefetch tile kt+2 into register set S, run half
  // of the MFMAs, convert + store tile kt+1 (register set S^1) into the other LDS
  // buffer while they execute, run the other half.
  auto step = [&](int64_t kt, const int cur, auto set) {
    constexpr int S = decltype(set)::value;
    using SN = std::integral_constant<int, S ^ 1>;
    // the last two tiles re-load the final tile (in bounds) so the body has no branch
    if (PF == 2) load_tiles((kt + 2 < nk ? kt + 2 : nk - 1) * BK, set);
    if (PF == 1 && kt + 1 < nk) load_tiles((kt + 1) * BK, SN{});
    V8 arh[FM], arl[FM], aih[FM], ail[FM], naih[FM], nail[FM];
    V8 brh[FN], brl[FN], bih[FN], bil[FN];
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const int o = (wm * WM + a * 32 + lrow) * P16 + g * 8;
      arh[a] = *(const V8*)&As[cur][0][o];
      arl[a] = *(const V8*)&As[cur][1][o];
      aih[a] = *(const V8*)&As[cur][2][o];
      ail[a] = *(const V8*)&As[cur][3][o];
      u4 t0 = *(u4*)&aih[a], t1 = *(u4*)&ail[a];
      t0 ^= 0x80008000u;  // flip the sign of both 16-bit halves
      t1 ^= 0x80008000u;
      naih[a] = *(V8*)&t0;
      nail[a] = *(V8*)&t1;
    }
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      const int o = (wn * WN + b * 32 + lrow) * P16 + g * 8;
      brh[b] = *(const V8*)&Bs[cur][0][o];
      brl[b] = *(const V8*)&Bs[cur][1][o];
      bih[b] = *(const V8*)&Bs[cur][2][o];
      bil[b] = *(const V8*)&Bs[cur][3][o];
    }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        cr[a][b] = H::mfma(arh[a], brh[b], cr[a][b]);
        ci[a][b] = H::mfma(arh[a], bih[b], ci[a][b]);
      }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        cr[a][b] = H::mfma(naih[a], bih[b], cr[a][b]);
        ci[a][b] = H::mfma(aih[a], brh[b], ci[a][b]);
      }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        cr[a][b] = H::mfma(arh[a], brl[b], cr[a][b]);
        ci[a][b] = H::mfma(arh[a], bil[b], ci[a][b]);
      }
    if (PF == 2) store_tiles(cur ^ 1, SN{});  // on the last tile this fills the idle buffer
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        cr[a][b] = H::mfma(arl[a], brh[b], cr[a][b]);
        ci[a][b] = H::mfma(arl[a], bih[b], ci[a][b]);
      }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        cr[a][b] = H::mfma(naih[a], bil[b], cr[a][b]);
        ci[a][b] = H::mfma(aih[a], brl[b], ci[a][b]);
      }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        cr[a][b] = H::mfma(nail[a], bih[b], cr[a][b]);
        ci[a][b] = H::mfma(ail[a], brh[b], ci[a][b]);
      }
    if (PF == 1 && kt + 1 < nk) store_tiles(cur ^ 1, SN{});
    if (PF == 2) {
      // interleave: each MFMA followed by a few VALU (hi/lo conversion) and LDS ops
#pragma unroll
      for (int i = 0; i < 12 * FM * FN; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // VALU
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
        __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS write
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // global read
      }
    }
    __syncthreads();
  };
  if (PF == 2) {
    for (int64_t kt = 0; kt < nk; kt += 2) {
      step(kt, 0, S0{});
      if (kt + 1 < nk) step(kt + 1, 1, S1{});
    }
  } else {
    for (int64_t kt = 0; kt < nk; ++kt) step(kt, (int)(kt & 1), S1{});
  }

  const float unscale = 1.f / (sa * sb);
  const OutMap om = out_map(p, m0, n0);
  store_blocks<FM, FN, WM, WN, true>(p, tc.coff, om, m0, n0, wm, wn, lane, cr, ci, unscale,
                               reinterpret_cast<QxCplx*>(smem) + wave * (32 * 33));
}

template <int BM, int BN, int PREC>
static hipError_t launch_split(const GemmArgs& a, hipStream_t s) {
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  const int64_t nwg = tiles * (int64_t)a.n_items * (1LL << a.nh);
  if (nwg <= 0) return hipSuccess;
  if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool akc = gemm_a_kc(a), bkc = gemm_b_kc(a);
  dim3 grid((unsigned)nwg), block(256);
  if (akc && bkc) hipLaunchKernelGGL((k_gemm_split<BM, BN, true, true, PREC>), grid, block, 0, s, a);
  else if (akc) hipLaunchKernelGGL((k_gemm_split<BM, BN, true, false, PREC>), grid, block, 0, s, a);
  else if (bkc) hipLaunchKernelGGL((k_gemm_split<BM, BN, false, true, PREC>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_gemm_split<BM, BN, false, false, PREC>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <int PREC>
static hipError_t launch_split_tile(const GemmArgs& a, int tile, hipStream_t s) {
  switch (tile) {
    case GEMM_TILE_64x64: return launch_split<64, 64, PREC>(a, s);
    case GEMM_TILE_128x64: return launch_split<128, 64, PREC>(a, s);
    case GEMM_TILE_64x128: return launch_split<64, 128, PREC>(a, s);
    case GEMM_TILE_256x128: return launch_split<256, 128, PREC>(a, s);
    case GEMM_TILE_128x256: return launch_split<128, 256, PREC>(a, s);
    default: return launch_split<128, 128, PREC>(a, s);
  }
}

}  // namespace qx
