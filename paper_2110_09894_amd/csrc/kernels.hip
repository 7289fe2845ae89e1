// HIP kernels for gfx950 (CDNA4): the tensor primitives of a sliced network
// contraction (Sec. III-B: slicing, permuting, contracting, recombination).
//
//   k_simt      small / memory-bound pairwise contraction, any bit layout
//   k_gemm_f32  complex matrix product on FP32 MFMA (Sec. IV-A: contractions
//               mapped to matrix multiplications)
//   k_dot       long inner products (the root of a slice's tree)
//   k_permute   LDS-tiled index permutation of dim-2 tensors
//   k_slice_sum FP64 sum of per-slice values (Eq. 2), fixed order
//   k_gather    per-bitstring offsets for the output closure (Sec. II)
#include <hip/hip_runtime.h>

#include <utility>
#include "kargs.h"
#include "kernels.h"
#include "qxtn.h"

namespace qx {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ QxCplx cmul_acc(QxCplx acc, QxCplx a, QxCplx b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
  return acc;
}

// ---------------------------------------------------------------------------
// Small contraction: one thread per output element, contracted bits looped.
// The low (up to 8) contracted bits' offsets are tabulated in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_simt(SimtArgs p) {
  __shared__ int64_t ka[256], kb[256];
  const int nklo = p.n_k < 8 ? p.n_k : 8;
  const int nlo = 1 << nklo;
  for (int i = threadIdx.x; i < nlo; i += blockDim.x) {
    int64_t oa = 0, ob = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < nklo && ((i >> j) & 1)) { oa += p.a_ks[j]; ob += p.b_ks[j]; }
    ka[i] = oa;
    kb[i] = ob;
  }
  __syncthreads();
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int item = blockIdx.y;
  if (o >= ((int64_t)1 << p.n_out)) return;
  int64_t ao = (int64_t)item * p.a_item + (p.a_gather ? p.a_gather[item] : 0);
  int64_t bo = (int64_t)item * p.b_item + (p.b_gather ? p.b_gather[item] : 0);
#pragma unroll
  for (int i = 0; i < QX_MAX_BITS; ++i)
    if (i < p.n_out && ((o >> i) & 1)) { ao += p.a_os[i]; bo += p.b_os[i]; }
  QxCplx acc = {0.f, 0.f};
  const int nkhi = p.n_k - nklo;
  for (int64_t kh = 0; kh < ((int64_t)1 << nkhi); ++kh) {
    int64_t ah = ao, bh = bo;
#pragma unroll
    for (int j = 0; j < QX_MAX_KBITS - 8; ++j)
      if (j < nkhi && ((kh >> j) & 1)) { ah += p.a_ks[8 + j]; bh += p.b_ks[8 + j]; }
    for (int kl = 0; kl < nlo; ++kl) acc = cmul_acc(acc, p.a[ah + ka[kl]], p.b[bh + kb[kl]]);
  }
  p.c[(int64_t)item * p.c_item + o] = acc;
}

// ---------------------------------------------------------------------------
// Operand tile loader shared by the matrix-product kernels.  A tile is ROWS
// rows x 16 k of complex64; every chunk is 8 consecutive k of one row.  For a
// k-contiguous operand a thread reads its chunk with 16-byte loads; otherwise
// consecutive lanes take consecutive rows, so a row-contiguous operand is read
// with coalesced 8-byte loads.  Row offsets are fixed per thread for the whole
// kernel; the k offset of the tile origin is recomputed per k tile.
// ---------------------------------------------------------------------------
__device__ inline int64_t scatter_bits(int64_t v, const int64_t* st, int n) {
  int64_t off = 0;
  for (int i = 0; i < n; ++i)
    if ((v >> i) & 1) off += st[i];
  return off;
}

struct OperandView {
  const QxCplx* X;
  int64_t rows, K;
  int64_t ld_r, ld_k;        // linear mode
  const int64_t *rs, *ks;    // bit mode
  int nr, nk;
  bool bits, kc, vec;
};

template <int ROWS, bool KC>
struct TileLoader {
  static constexpr int BK = 16;
  static constexpr int CH = ROWS * (BK / 8);
  static constexpr int P = (CH + 255) / 256;
  int64_t roff[P];           // offset of the chunk's row
  int64_t kgoff[P];          // offset of the chunk's first k within the tile
  int rloc[P], kgl[P];
  bool rok[P];
  __device__ static inline void row_kg(int c, int& r, int& kg) {
    r = KC ? c / (BK / 8) : c % ROWS;
    kg = KC ? c % (BK / 8) : c / ROWS;
  }
  __device__ inline int64_t koff(const OperandView& v, int64_t k) const {
    return v.bits ? scatter_bits(k, v.ks, v.nk) : k * v.ld_k;
  }
  __device__ inline void init(const OperandView& v, int64_t r0, int tid) {
    const int64_t rbase = v.bits ? scatter_bits(r0, v.rs, v.nr) : r0 * v.ld_r;
#pragma unroll
    for (int ps = 0; ps < P; ++ps) {
      const int c = tid + ps * 256;
      int r = 0, kg = 0;
      if (c < CH) row_kg(c, r, kg);
      rloc[ps] = r;
      kgl[ps] = kg;
      rok[ps] = c < CH && r0 + r < v.rows;
      roff[ps] = rbase + (v.bits ? scatter_bits(r, v.rs, v.nr) : (int64_t)r * v.ld_r);
      kgoff[ps] = koff(v, kg * 8);
    }
  }
  // offset of k0 (a multiple of 16): bits 4 and up
  __device__ inline int64_t kbase(const OperandView& v, int64_t k0) const { return koff(v, k0); }
  __device__ inline void load(const OperandView& v, int64_t k0, QxCplx (&reg)[P][8]) const {
    const int64_t kb0 = kbase(v, k0);
#pragma unroll
    for (int ps = 0; ps < P; ++ps) {
      const int64_t kb = k0 + kgl[ps] * 8;
      const QxCplx* src = v.X + roff[ps] + kb0 + kgoff[ps];
      if (KC && v.vec && rok[ps] && kb + 8 <= v.K) {
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          v4f x = *(const v4f*)(src + j);
          reg[ps][j] = {x[0], x[1]};
          reg[ps][j + 1] = {x[2], x[3]};
        }
      } else if (KC) {
#pragma unroll
        for (int j = 0; j < 8; ++j) reg[ps][j] = (rok[ps] && kb + j < v.K) ? src[j] : QxCplx{0.f, 0.f};
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int64_t jo = v.bits ? ((j & 1) ? v.ks[0] : 0) + ((j & 2) ? v.ks[1] : 0) + ((j & 4) ? v.ks[2] : 0)
                                    : (int64_t)j * v.ld_k;
          reg[ps][j] = (rok[ps] && kb + j < v.K) ? src[jo] : QxCplx{0.f, 0.f};
        }
      }
    }
  }
};

__device__ inline OperandView view_a(const GemmArgs& p, const QxCplx* X) {
  OperandView v;
  v.X = X; v.rows = p.M; v.K = p.K; v.ld_r = p.a_ms; v.ld_k = p.a_ks; v.rs = p.a_rs; v.ks = p.a_kst;
  v.nr = p.nm; v.nk = p.nk; v.bits = p.bits != 0; v.kc = p.bits ? p.a_kc != 0 : p.a_ks == 1; v.vec = p.vec_a != 0;
  return v;
}
__device__ inline OperandView view_b(const GemmArgs& p, const QxCplx* X) {
  OperandView v;
  v.X = X; v.rows = p.N; v.K = p.K; v.ld_r = p.b_ns; v.ld_k = p.b_ks; v.rs = p.b_rs; v.ks = p.b_kst;
  v.nr = p.nn; v.nk = p.nk; v.bits = p.bits != 0; v.kc = p.bits ? p.b_kc != 0 : p.b_ks == 1; v.vec = p.vec_b != 0;
  return v;
}

// Output offset of (m, n): m0 / n0 are tile origins, lm / ln offsets inside the tile.
struct OutMap {
  int64_t mbase, nbase;
  __device__ inline int64_t m(const GemmArgs& p, int64_t lm) const {
    return p.bits ? mbase + scatter_bits(lm, p.c_mst, p.nm) : mbase + lm * p.c_ms;
  }
  __device__ inline int64_t n(const GemmArgs& p, int64_t ln) const {
    return p.bits ? nbase + scatter_bits(ln, p.c_nst, p.nn) : nbase + ln;
  }
};
__device__ inline OutMap out_map(const GemmArgs& p, int64_t m0, int64_t n0) {
  OutMap o;
  o.mbase = p.bits ? scatter_bits(m0, p.c_mst, p.nm) : m0 * p.c_ms;
  o.nbase = p.bits ? scatter_bits(n0, p.c_nst, p.nn) : n0;
  return o;
}

// Work-group -> (batch item, hyper index, tile) with an XCD-aware order:
// hardware deals work-groups round-robin over the 8 XCDs, so each XCD gets a
// contiguous run of logical tiles and neighbours share its L2.
struct TileCoord {
  int item;
  int64_t tm, tn, aoff, boff, coff;
};
__device__ inline TileCoord tile_coord(const GemmArgs& p, int BM, int BN) {
  const int64_t tiles_n = (p.N + BN - 1) / BN;
  const int64_t tiles = ((p.M + BM - 1) / BM) * tiles_n;
  const int64_t nwg = (int64_t)gridDim.x;
  int64_t w = blockIdx.x;
  const int64_t per = nwg / 8;
  if (per > 0 && w < per * 8) w = (w % 8) * per + w / 8;
  const int64_t z = w / tiles, t = w % tiles;
  TileCoord tc;
  tc.tm = t / tiles_n;
  tc.tn = t % tiles_n;
  tc.item = (int)(z >> p.nh);
  const int64_t h = z & ((1LL << p.nh) - 1);
  tc.aoff = (int64_t)tc.item * p.a_item + (p.a_gather ? p.a_gather[tc.item] : 0);
  tc.boff = (int64_t)tc.item * p.b_item + (p.b_gather ? p.b_gather[tc.item] : 0);
  tc.coff = (int64_t)tc.item * p.c_item;
#pragma unroll
  for (int i = 0; i < QX_MAX_HBITS; ++i)
    if (i < p.nh && ((h >> i) & 1)) { tc.aoff += p.a_hs[i]; tc.boff += p.b_hs[i]; tc.coff += p.c_hs[i]; }
  return tc;
}

// Epilogue: each 32x32 accumulator block goes through LDS and is stored in the
// order of ascending output address, so the stores form contiguous runs for
// any output index order.  Element e of a block (10 bits, ordered by output
// stride) is split into a lane part (bits 0..5) and a store-step part (bits
// 6..9); both offsets are sums of precomputed per-bit strides.
// stage: per-wave LDS area of 32 x 33 complex.
template <int FM, int FN, int WM, int WN, bool UNROLL>
__device__ inline void store_blocks(const GemmArgs& p, QxCplx* __restrict__ C, const OutMap& om, int64_t m0,
                                    int64_t n0, int wm, int wn, int lane, const v16f (&cr)[FM][FN],
                                    const v16f (&ci)[FM][FN], float scale, QxCplx* stage) {
  const int lrow = lane & 31, g = lane >> 5;
  int lm_lane = 0, ln_lane = 0;
  int64_t off_lane = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b)
    if ((lane >> b) & 1) {
      lm_lane += p.ep_lm[b];
      ln_lane += p.ep_ln[b];
      off_lane += p.ep_st[b];
    }
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 16; ++i)
        stage[(8 * (i / 4) + 4 * g + (i % 4)) * 33 + lrow] = QxCplx{cr[a][b][i] * scale, ci[a][b][i] * scale};
      __syncthreads();
      const int64_t lm0 = wm * WM + a * 32, ln0 = wn * WN + b * 32;
      QxCplx* __restrict__ Cb = C + om.m(p, lm0) + om.n(p, ln0) + off_lane;
      auto put = [&](int j) {
        int lm = lm_lane, ln = ln_lane;
        int64_t off = 0;
#pragma unroll
        for (int b2 = 0; b2 < 4; ++b2)
          if ((j >> b2) & 1) {
            lm += p.ep_lm[6 + b2];
            ln += p.ep_ln[6 + b2];
            off += p.ep_st[6 + b2];
          }
        if (m0 + lm0 + lm < p.M && n0 + ln0 + ln < p.N) Cb[off] = stage[lm * 33 + ln];
      };
      // a rolled loop keeps the FP32 kernel's registers low enough for two waves per SIMD
      if (UNROLL) {
#pragma unroll
        for (int j = 0; j < 16; ++j) put(j);
      } else {
#pragma unroll 1
        for (int j = 0; j < 16; ++j) put(j);
      }
    }
}

// ---------------------------------------------------------------------------
// Complex GEMM on FP32 matrix cores (v_mfma_f32_32x32x2_f32).
// Work-group tile BM x BN, 4 waves in a 2x2 grid, K tile of 16 complex values.
// Both operand tiles are staged in LDS as [row][k] (k contiguous), so each lane
// fetches its 8 consecutive k values with wide LDS reads.  Lane group g = l/32
// owns k in [8g, 8g+8); step s of the 8 MFMA steps uses k = 8g + s for both
// operands, which is a valid split of the k-sum.  A complex product is four
// real MFMAs into separate real / imaginary accumulators.
// ---------------------------------------------------------------------------
template <int BM, int BN, bool A_KC, bool B_KC>
__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs p) {
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
  auto load_tiles = [&](int64_t k0) {
    la.load(va, k0, ra);
    lb.load(vb, k0, rb);
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
    if (kt + 1 < nk) load_tiles((kt + 1) * BK);
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

  QxCplx* __restrict__ C = p.c + tc.coff;
  const OutMap om = out_map(p, m0, n0);
  store_blocks<FM, FN, WM, WN, false>(p, C, om, m0, n0, wm, wn, lane, cr, ci, 1.f, smem + wave * (32 * 33));
}

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
  QxCplx ra[LA::P][8], rb[LB::P][8];
  auto load_tiles = [&](int64_t k0) {
    la.load(va, k0, ra);
    lb.load(vb, k0, rb);
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
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int ps = 0; ps < LA::P; ++ps) {
      const int c = tid + ps * 256;
      if (c < LA::CH) {
        int r, kg;
        LA::row_kg(c, r, kg);
        const int o = r * P16 + kg * 8;
        split_store(&As[buf][0][o], &As[buf][1][o], &As[buf][2][o], &As[buf][3][o], ra[ps], sa);
      }
    }
#pragma unroll
    for (int ps = 0; ps < LB::P; ++ps) {
      const int c = tid + ps * 256;
      if (c < LB::CH) {
        int r, kg;
        LB::row_kg(c, r, kg);
        const int o = r * P16 + kg * 8;
        split_store(&Bs[buf][0][o], &Bs[buf][1][o], &Bs[buf][2][o], &Bs[buf][3][o], rb[ps], sb);
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
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nk) load_tiles((kt + 1) * BK);
    V8 arh[FM], arl[FM], aih[FM], ail[FM], naih[FM], nail[FM];
    V8 brh[FN], brl[FN], bih[FN], bil[FN];
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const int o = (wm * WM + a * 32 + lrow) * P16 + g * 8;
      arh[a] = *(const V8*)&As[buf][0][o];
      arl[a] = *(const V8*)&As[buf][1][o];
      aih[a] = *(const V8*)&As[buf][2][o];
      ail[a] = *(const V8*)&As[buf][3][o];
      u4 t0 = *(u4*)&aih[a], t1 = *(u4*)&ail[a];
      t0 ^= 0x80008000u;  // flip the sign of both 16-bit halves
      t1 ^= 0x80008000u;
      naih[a] = *(V8*)&t0;
      nail[a] = *(V8*)&t1;
    }
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      const int o = (wn * WN + b * 32 + lrow) * P16 + g * 8;
      brh[b] = *(const V8*)&Bs[buf][0][o];
      brl[b] = *(const V8*)&Bs[buf][1][o];
      bih[b] = *(const V8*)&Bs[buf][2][o];
      bil[b] = *(const V8*)&Bs[buf][3][o];
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
    if (kt + 1 < nk) store_tiles(buf ^ 1);
    __syncthreads();
  }

  const float unscale = 1.f / (sa * sb);
  QxCplx* __restrict__ C = p.c + tc.coff;
  const OutMap om = out_map(p, m0, n0);
  store_blocks<FM, FN, WM, WN, true>(p, C, om, m0, n0, wm, wn, lane, cr, ci, unscale,
                               reinterpret_cast<QxCplx*>(smem) + wave * (32 * 33));
}

// ---------------------------------------------------------------------------
// Long inner products: one work-group per output element; FP32 partial sums
// per lane, reduced across the wavefront with cross-lane shuffles and across
// the 4 waves through LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dot(DotArgs p) {
  __shared__ float red[2][4];
  const int64_t o = blockIdx.x;
  const int item = blockIdx.y;
  int64_t ao = (int64_t)item * p.a_item + (p.a_gather ? p.a_gather[item] : 0);
  int64_t bo = (int64_t)item * p.b_item + (p.b_gather ? p.b_gather[item] : 0);
#pragma unroll
  for (int i = 0; i < QX_MAX_BITS; ++i)
    if (i < p.n_out && ((o >> i) & 1)) { ao += p.a_os[i]; bo += p.b_os[i]; }
  const QxCplx* __restrict__ A = p.a + ao;
  const QxCplx* __restrict__ B = p.b + bo;
  // four independent partial sums per lane keep the sequential chains short
  QxCplx acc0 = {0.f, 0.f}, acc1 = {0.f, 0.f}, acc2 = {0.f, 0.f}, acc3 = {0.f, 0.f};
  const bool vec = ((((uintptr_t)A) | ((uintptr_t)B)) & 15) == 0 && (p.K & 3) == 0;
  if (vec) {
    for (int64_t k = 4 * (int64_t)threadIdx.x; k < p.K; k += 4 * blockDim.x) {
      const v4f a0 = *(const v4f*)(A + k), a1 = *(const v4f*)(A + k + 2);
      const v4f b0 = *(const v4f*)(B + k), b1 = *(const v4f*)(B + k + 2);
      acc0 = cmul_acc(acc0, QxCplx{a0[0], a0[1]}, QxCplx{b0[0], b0[1]});
      acc1 = cmul_acc(acc1, QxCplx{a0[2], a0[3]}, QxCplx{b0[2], b0[3]});
      acc2 = cmul_acc(acc2, QxCplx{a1[0], a1[1]}, QxCplx{b1[0], b1[1]});
      acc3 = cmul_acc(acc3, QxCplx{a1[2], a1[3]}, QxCplx{b1[2], b1[3]});
    }
  } else {
    for (int64_t k = threadIdx.x; k < p.K; k += blockDim.x) acc0 = cmul_acc(acc0, A[k], B[k]);
  }
  QxCplx acc = {(acc0.x + acc1.x) + (acc2.x + acc3.x), (acc0.y + acc1.y) + (acc2.y + acc3.y)};
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    acc.x += __shfl_xor(acc.x, off, 64);
    acc.y += __shfl_xor(acc.y, off, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wave] = acc.x;
    red[1][wave] = acc.y;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    QxCplx r = {(red[0][0] + red[0][1]) + (red[0][2] + red[0][3]),
                (red[1][0] + red[1][1]) + (red[1][2] + red[1][3])};
    p.c[(int64_t)item * p.c_item + o] = r;
  }
}

// ---------------------------------------------------------------------------
// Index permutation.  A tile is the set of elements that differ only in the
// output's lowest bits and the bits at the input's lowest positions, so a tile
// is read in runs contiguous in the input and written in runs contiguous in
// the output, transposing through LDS.  The outer bits select the tile.  Each
// work-group builds its offset tables once and then walks many tiles.
// ---------------------------------------------------------------------------
constexpr int PERM_TB = 5;
__global__ __launch_bounds__(256) void k_permute(PermArgs p) {
  __shared__ QxCplx buf[1 << (2 * PERM_TB)];
  __shared__ long long tin[1 << (2 * PERM_TB)];   // load order v -> input offset inside tile
  __shared__ short tlu[1 << (2 * PERM_TB)];       // load order v -> LDS slot
  __shared__ long long tout[1 << (2 * PERM_TB)];  // LDS slot u -> output offset inside tile
  const int nt = p.nt;
  const int tsz = 1 << nt;
  for (int v = threadIdx.x; v < tsz; v += blockDim.x) {
    long long inoff = 0, outoff = 0;
    int u = 0;
    for (int b = 0; b < nt; ++b)
      if ((v >> b) & 1) {
        inoff += 1LL << p.in_pos[p.tl[p.ll[b]]];
        u |= 1 << p.ll[b];
        outoff += 1LL << p.tl[b];
      }
    tin[v] = inoff;
    tlu[v] = (short)u;
    tout[v] = outoff;
  }
  const int64_t n_tiles = (int64_t)1 << p.n_outer;
  const int64_t total = n_tiles * p.n_items;
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int64_t item = t >> p.n_outer;
    int64_t w = t & (n_tiles - 1), ibase = item * p.in_item, obase = item * p.out_item;
    for (int i = 0; w; ++i, w >>= 1)
      if (w & 1) { ibase += p.outer_in[i]; obase += p.outer_out[i]; }
    __syncthreads();  // tables ready / previous tile's LDS reads done
    const QxCplx* __restrict__ in = p.in + ibase;
    for (int v = threadIdx.x; v < tsz; v += blockDim.x) buf[tlu[v]] = in[tin[v]];
    __syncthreads();
    QxCplx* __restrict__ out = p.out + obase;
    for (int u = threadIdx.x; u < tsz; u += blockDim.x) out[tout[u]] = buf[u];
  }
}

// ---------------------------------------------------------------------------
// FP64 sum over the slices of one block, ascending slice order (deterministic).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_slice_sum(SliceSumArgs p) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= p.n_items) return;
  const int64_t base = (int64_t)item * p.root_item + (p.root_gather ? p.root_gather[item] : 0);
  double sr = 0.0, si = 0.0;
  for (int s = p.s_lo; s < p.s_hi; ++s) {
    int64_t off = base;
#pragma unroll
    for (int j = 0; j < QX_MAX_SBITS; ++j)
      if (j < p.n_sbits && ((s >> j) & 1)) off += p.s_stride[j];
    const QxCplx v = p.root[off];
    sr += (double)v.x;
    si += (double)v.y;
  }
  p.amp[2 * item] += sr;
  p.amp[2 * item + 1] += si;
}

constexpr int ABSMAX_GRID = 1024;
__global__ __launch_bounds__(256) void k_absmax(AbsmaxArgs p) {
  __shared__ float red[4];
  __shared__ int last;
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += (int64_t)gridDim.x * blockDim.x) {
    const QxCplx v = p.x[i];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    p.partial[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __threadfence();
    last = atomicAdd(p.ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  float mm = 0.f;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) mm = fmaxf(mm, __ldg(&p.partial[i]));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mm = fmaxf(mm, __shfl_xor(mm, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mm;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    float sc = 1.f;
    if (mx > 0.f && mx < 3.0e38f) {
      int e;
      frexpf(mx, &e);  // mx < 2^e
      int k = 14 - e;
      k = k > 100 ? 100 : (k < -100 ? -100 : k);
      sc = ldexpf(1.f, k);
    }
    p.scale[0] = sc;
    *p.ticket = 0u;
  }
}

__global__ __launch_bounds__(256) void k_gather(GatherArgs p) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= p.n_items) return;
  const uint64_t x = p.x[item];
  int64_t off = 0;
#pragma unroll
  for (int j = 0; j < 64; ++j)
    if (j < p.n_q && ((x >> p.q[j]) & 1ULL)) off += p.stride[j];
  p.out[item] = off;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_simt(const SimtArgs& a, hipStream_t s) {
  const int64_t n = (int64_t)1 << a.n_out;
  const int threads = n < 256 ? (n < 64 ? 64 : (int)n) : 256;
  dim3 grid((unsigned)((n + threads - 1) / threads), (unsigned)a.n_items);
  hipLaunchKernelGGL(k_simt, grid, dim3(threads), 0, s, a);
  return hipGetLastError();
}

template <int BM, int BN, int PREC>
static hipError_t launch_gemm_tile(const GemmArgs& a, hipStream_t s) {
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  const int64_t nwg = tiles * (int64_t)a.n_items * (1LL << a.nh);
  if (nwg <= 0) return hipSuccess;
  if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool akc = a.bits ? a.a_kc != 0 : a.a_ks == 1;
  const bool bkc = a.bits ? a.b_kc != 0 : a.b_ks == 1;
  dim3 grid((unsigned)nwg), block(256);
  if (PREC == QX_C64) {
    if (akc && bkc) hipLaunchKernelGGL((k_gemm_f32<BM, BN, true, true>), grid, block, 0, s, a);
    else if (akc) hipLaunchKernelGGL((k_gemm_f32<BM, BN, true, false>), grid, block, 0, s, a);
    else if (bkc) hipLaunchKernelGGL((k_gemm_f32<BM, BN, false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_gemm_f32<BM, BN, false, false>), grid, block, 0, s, a);
  } else {
    constexpr int PR = PREC == QX_C64 ? QX_SPLIT_BF16 : PREC;
    if (akc && bkc) hipLaunchKernelGGL((k_gemm_split<BM, BN, true, true, PR>), grid, block, 0, s, a);
    else if (akc) hipLaunchKernelGGL((k_gemm_split<BM, BN, true, false, PR>), grid, block, 0, s, a);
    else if (bkc) hipLaunchKernelGGL((k_gemm_split<BM, BN, false, true, PR>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_gemm_split<BM, BN, false, false, PR>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& a, int precision, int tile, hipStream_t s) {
  const bool small = tile == GEMM_TILE_64x64;
  switch (precision) {
    case QX_SPLIT_BF16:
      return small ? launch_gemm_tile<64, 64, QX_SPLIT_BF16>(a, s) : launch_gemm_tile<128, 128, QX_SPLIT_BF16>(a, s);
    case QX_SPLIT_FP16:
      return small ? launch_gemm_tile<64, 64, QX_SPLIT_FP16>(a, s) : launch_gemm_tile<128, 128, QX_SPLIT_FP16>(a, s);
    default:
      return small ? launch_gemm_tile<64, 64, QX_C64>(a, s) : launch_gemm_tile<128, 128, QX_C64>(a, s);
  }
}

hipError_t launch_dot(const DotArgs& a, hipStream_t s) {
  dim3 grid((unsigned)(1LL << a.n_out), (unsigned)a.n_items);
  hipLaunchKernelGGL(k_dot, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

void permute_setup(PermArgs& a) {
  const int r = a.rank;
  const int tb = r < PERM_TB ? r : PERM_TB;
  int nt = 0, no = 0;
  for (int i = 0; i < r; ++i) {
    if (i < tb || a.in_pos[i] < tb) {
      a.tl[nt++] = i;
    } else {
      a.outer_in[no] = 1LL << a.in_pos[i];
      a.outer_out[no] = 1LL << i;
      ++no;
    }
  }
  int nl = 0;
  for (int pos = 0; pos < r && nl < nt; ++pos)
    for (int j = 0; j < nt; ++j)
      if (a.in_pos[a.tl[j]] == pos) a.ll[nl++] = j;
  a.nt = nt;
  a.n_outer = no;
}

hipError_t launch_permute(const PermArgs& a, hipStream_t s) {
  const int64_t total = ((int64_t)1 << a.n_outer) * a.n_items;
  const int64_t grid = total < 4096 ? total : 4096;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute, dim3((unsigned)grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_slice_sum(const SliceSumArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.n_items + 255) / 256));
  hipLaunchKernelGGL(k_slice_sum, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

void gemm_epilogue_setup(GemmArgs& g) {
  // the ten bits of a 32x32 block (m 0..4, n 0..4) in ascending order of output stride
  int64_t st[10];
  int id[10];
  for (int i = 0; i < 5; ++i) {
    id[i] = i;
    id[5 + i] = 8 + i;
    if (g.bits) {
      st[i] = i < g.nm ? g.c_mst[i] : ((int64_t)1 << 62) + i;
      st[5 + i] = i < g.nn ? g.c_nst[i] : ((int64_t)1 << 62) + 5 + i;
    } else {
      st[i] = g.c_ms << i;
      st[5 + i] = (int64_t)1 << i;
    }
  }
  for (int i = 1; i < 10; ++i)
    for (int j = i; j > 0 && st[j] < st[j - 1]; --j) {
      std::swap(st[j], st[j - 1]);
      std::swap(id[j], id[j - 1]);
    }
  for (int i = 0; i < 10; ++i) {
    const bool isn = id[i] >= 8;
    const int bit = isn ? id[i] - 8 : id[i];
    g.ep_lm[i] = isn ? 0 : 1 << bit;
    g.ep_ln[i] = isn ? 1 << bit : 0;
    g.ep_st[i] = st[i] >= ((int64_t)1 << 62) ? 0 : st[i];
  }
}

hipError_t launch_absmax(const AbsmaxArgs& a, hipStream_t s) {
  const int64_t want = (a.n + 255) / 256;
  const int grid = (int)(want < 1 ? 1 : (want > ABSMAX_GRID ? ABSMAX_GRID : want));
  hipLaunchKernelGGL(k_absmax, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.n_items + 255) / 256));
  hipLaunchKernelGGL(k_gather, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace qx
