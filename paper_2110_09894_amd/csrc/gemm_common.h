// Device code shared by the matrix-core GEMM kernels (internal header).
#pragma once
#include <hip/hip_runtime.h>

#include "kargs.h"
#include "kernels.h"
#include "qxtn.h"
#include "split_format.h"

namespace qx {


typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ QxCplx cmul_acc(QxCplx acc, QxCplx a, QxCplx b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
  return acc;
}

// ---------------------------------------------------------------------------
// Operand tile loader shared by the matrix-product kernels.  A tile is ROWS
// rows x 16 k of complex64; every chunk is 8 consecutive k of one row.  For a
// k-contiguous operand a thread reads its chunk with 16-byte loads; otherwise
// consecutive lanes take consecutive rows, so a row-contiguous operand is read
// with coalesced 8-byte loads.  Row offsets are fixed per thread for the whole
// kernel; the k offset of the tile origin is recomputed per k tile.
// ---------------------------------------------------------------------------
// Offset of index v under per-bit strides st[0..n): sum of st[i] over the set bits
// i of v.  NB bounds the bits v can have; the loop is unrolled so the strides are
// fetched together instead of one dependent load per bit.
template <int NB = QX_GEMM_BITS>
__device__ inline int64_t scatter_bits(int64_t v, const int64_t* st, int n) {
  int64_t off = 0;
#pragma unroll
  for (int i = 0; i < NB; ++i) off += (i < n && ((v >> i) & 1)) ? st[i] : 0;
  return off;
}
// The same for a wave-uniform v with few set bits (tile origins): one step per set bit.
__device__ inline int64_t scatter_set_bits(uint64_t v, const int64_t* st, int n) {
  int64_t off = 0;
  for (; v; v &= v - 1) {
    const int i = __builtin_ctzll(v);
    if (i >= n) break;
    off += st[i];
  }
  return off;
}

// k-contiguous loading (8 consecutive k values with 16-byte loads) needs the
// operand's k stride to be 1 for k bits 0..2, 16-byte alignment and K % 8 == 0.
__host__ __device__ inline bool gemm_a_kc(const GemmArgs& p) {
  return (p.bits ? p.a_kc != 0 : p.a_ks == 1) && p.vec_a && p.K % 8 == 0;
}
__host__ __device__ inline bool gemm_b_kc(const GemmArgs& p) {
  return (p.bits ? p.b_kc != 0 : p.b_ks == 1) && p.vec_b && p.K % 8 == 0;
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
    const int64_t rbase = v.bits ? scatter_set_bits(r0, v.rs, v.nr) : r0 * v.ld_r;
#pragma unroll
    for (int ps = 0; ps < P; ++ps) {
      const int c = tid + ps * 256;
      int r = 0, kg = 0;
      if (c < CH) row_kg(c, r, kg);
      rloc[ps] = r;
      kgl[ps] = kg;
      rok[ps] = c < CH && r0 + r < v.rows;
      roff[ps] = rbase + (v.bits ? scatter_bits<8>(r, v.rs, v.nr) : (int64_t)r * v.ld_r);
      kgoff[ps] = v.bits ? scatter_bits<4>(kg * 8, v.ks, v.nk) : kg * 8 * v.ld_k;
    }
  }
  // offset of k0 (a multiple of 16): bits 4 and up
  __device__ inline int64_t kbase(const OperandView& v, int64_t k0) const { return koff(v, k0); }
  // Branch-free: invalid rows, and k chunks past K, read row 0 of the tile origin
  // (a valid address) and are zeroed with selects, so the compiler can keep several
  // tiles of loads in flight.  A k-contiguous operand is only used when the host has
  // checked 16-byte alignment and K % 8 == 0 (so a chunk is wholly inside or outside
  // K); every other operand takes the row-contiguous path.
  __device__ inline void load(const OperandView& v, int64_t k0, QxCplx (&reg)[P][8]) const {
    load(v, k0, kbase(v, k0), reg);
  }
  // kb0: offset of k0, when the caller tracks it incrementally
  __device__ inline void load(const OperandView& v, int64_t k0, int64_t kb0, QxCplx (&reg)[P][8]) const {
#pragma unroll
    for (int ps = 0; ps < P; ++ps) {
      const int64_t kb = k0 + kgl[ps] * 8;
      const bool ok = rok[ps] && (!KC || kb < v.K);
      const QxCplx* src = v.X + (ok ? roff[ps] : 0) + kb0 + kgoff[ps];
      if (KC) {
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          const v4f x = *(const v4f*)(src + j);
          reg[ps][j] = {ok ? x[0] : 0.f, ok ? x[1] : 0.f};
          reg[ps][j + 1] = {ok ? x[2] : 0.f, ok ? x[3] : 0.f};
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const bool okj = ok && kb + j < v.K;
          const int64_t jo = v.bits ? ((j & 1) ? v.ks[0] : 0) + ((j & 2) ? v.ks[1] : 0) + ((j & 4) ? v.ks[2] : 0)
                                    : (int64_t)j * v.ld_k;
          const QxCplx x = src[okj ? jo : 0];
          reg[ps][j] = {okj ? x.x : 0.f, okj ? x.y : 0.f};
        }
      }
    }
  }
};

__device__ inline OperandView view_a(const GemmArgs& p, const QxCplx* X) {
  OperandView v;
  v.X = X; v.rows = p.M; v.K = p.K; v.ld_r = p.a_ms; v.ld_k = p.a_ks; v.rs = p.a_rs; v.ks = p.a_kst;
  v.nr = p.nm; v.nk = p.nk; v.bits = p.bits != 0; v.kc = gemm_a_kc(p); v.vec = p.vec_a != 0;
  return v;
}
__device__ inline OperandView view_b(const GemmArgs& p, const QxCplx* X) {
  OperandView v;
  v.X = X; v.rows = p.N; v.K = p.K; v.ld_r = p.b_ns; v.ld_k = p.b_ks; v.rs = p.b_rs; v.ks = p.b_kst;
  v.nr = p.nn; v.nk = p.nk; v.bits = p.bits != 0; v.kc = gemm_b_kc(p); v.vec = p.vec_b != 0;
  return v;
}

// Output offset of (m, n): m0 / n0 are tile origins, lm / ln (< 256) offsets inside the tile.
struct OutMap {
  int64_t mbase, nbase;
  __device__ inline int64_t m(const GemmArgs& p, int64_t lm) const {
    return p.bits ? mbase + scatter_bits<8>(lm, p.c_mst, p.nm) : mbase + lm * p.c_ms;
  }
  __device__ inline int64_t n(const GemmArgs& p, int64_t ln) const {
    return p.bits ? nbase + scatter_bits<8>(ln, p.c_nst, p.nn) : nbase + ln;
  }
};
__device__ inline OutMap out_map(const GemmArgs& p, int64_t m0, int64_t n0) {
  OutMap o;
  o.mbase = p.bits ? scatter_set_bits(m0, p.c_mst, p.nm) : m0 * p.c_ms;
  o.nbase = p.bits ? scatter_set_bits(n0, p.c_nst, p.nn) : n0;
  return o;
}

// Work-group -> (batch item, hyper index, tile) with an XCD-aware order:
// hardware deals work-groups round-robin over the 8 XCDs, so each XCD gets a
// contiguous run of logical tiles and neighbours share its L2.  Inside one
// product the tiles run in groups of QX_TILE_GROUP tile rows, m fastest, so the
// work-groups resident on one XCD at a time cover a square-ish patch of C and
// read few A and B panels, each shared by several of them through the L2.
constexpr uint32_t QX_TILE_GROUP = 8;
struct TileCoord {
  int item;
  int64_t tm, tn, aoff, boff, coff;
};
// (the launchers keep the grid below 2^31 work-groups, so 32-bit division suffices)
__device__ inline TileCoord tile_coord(const GemmArgs& p, int BM, int BN) {
  const uint32_t tiles_m = (uint32_t)((p.M + BM - 1) / BM);
  const uint32_t tiles_n = (uint32_t)((p.N + BN - 1) / BN);
  const uint32_t tiles = tiles_m * tiles_n;
  const uint32_t nwg = gridDim.x;
  uint32_t w = blockIdx.x;
  const uint32_t per = nwg / 8;
  if (per > 0 && w < per * 8) w = (w % 8) * per + w / 8;
  const uint32_t z = w / tiles, t = w % tiles;
  const uint32_t group = QX_TILE_GROUP * tiles_n;
  const uint32_t g = t / group, first = g * QX_TILE_GROUP, r = t - g * group;
  const uint32_t gsz = tiles_m - first < QX_TILE_GROUP ? tiles_m - first : QX_TILE_GROUP;
  TileCoord tc;
  tc.tm = first + r % gsz;
  tc.tn = r / gsz;
  tc.item = (int)(z >> p.nh);
  const int64_t h = z & ((1LL << p.nh) - 1);
  tc.aoff = (int64_t)tc.item * p.a_item + (p.a_gather ? p.a_gather[tc.item] : 0);
  tc.boff = (int64_t)tc.item * p.b_item + (p.b_gather ? p.b_gather[tc.item] : 0);
  tc.coff = (int64_t)tc.item * p.c_item;
  for (uint32_t hb = h; hb; hb &= hb - 1) {
    const int i = __builtin_ctz(hb);
    tc.aoff += p.a_hs[i];
    tc.boff += p.b_hs[i];
    tc.coff += p.c_hs[i];
  }
  return tc;
}

// Complex64 product outputs are read by a later op, not by this one: their stores (each wave
// instruction a run of consecutive elements) are non-temporal, so they do not displace the operand
// panels the resident work-groups share in the L2.  The split kernels keep ordinary stores: a lane
// writes a chunk's four planes in four instructions, which the L2 merges into whole lines (and the
// non-temporal form in their unused complex64 branch made the 128x128 BF16 kernel spill).
__device__ __forceinline__ void store_out(QxCplx* dst, QxCplx v) {
  __builtin_nontemporal_store(qx_f32x2{v.x, v.y}, reinterpret_cast<qx_f32x2*>(dst));
}

// Orders this wave's LDS accesses before and after it (a wave's LDS operations
// complete in issue order; the empty asm statements keep the compiler from
// moving memory accesses across).  Unlike __syncthreads() it neither waits for
// the other waves nor for outstanding global stores.
__device__ __forceinline__ void wave_lds_fence() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// Epilogue: each 32x32 accumulator block goes through LDS and is stored in the
// order of ascending output address, so the stores form contiguous runs for
// any output index order.  Element e of a block (10 bits, ordered by output
// stride) is split into a lane part (bits 0..5) and a store-step part (bits
// 6..9); both offsets are sums of precomputed per-bit strides.  coff: element
// offset of the work-group's output (item and shared-slice offsets).  With
// c_split the output is written in split BF16 form.
// stage: per-wave LDS area of 32 x 33 complex.  The caller has passed a
// work-group barrier after the last LDS read of the k loop, so the stage areas
// (which alias the operand buffers) are free; afterwards each wave only touches
// its own area.
// Planes of a value already multiplied by the output's scale factor: BF16 (KIND 1) or FP16 (KIND 2).
template <int KIND>
__device__ __forceinline__ void split_scaled(QxCplx v, uint32_t& hi, uint32_t& lo) {
  if constexpr (KIND == 2) split_pair_f16(v, hi, lo);
  else split_pair(v, hi, lo);
}

// scale multiplies every accumulator before it is stored (split FP16: the output's scale over the
// operands'); KIND is the split storage written when p.c_split is set, 0 for the complex64 kernel
// (whose products never write split storage, and whose plain stores are non-temporal).
template <int FM, int FN, int WM, int WN, bool UNROLL, int KIND = 1>
__device__ inline void store_blocks(const GemmArgs& p, int64_t coff, const OutMap& om, int64_t m0,
                                    int64_t n0, int wm, int wn, int lane, const v16f (&cr)[FM][FN],
                                    const v16f (&ci)[FM][FN], float scale, QxCplx* stage) {
  const int lrow = lane & 31, g = lane >> 5;
  if (p.c_split && p.ep_reg) {
    // A lane's accumulator group j (entries 8j .. 8j + 7) holds block rows 16j + 4g + {0..3, 8..11}
    // of column lrow: with m bits 0, 1, 3 at output strides 1, 2, 4 that is one 8-element chunk,
    // converted and written as four 16-byte stores without going through LDS.
    uint16_t* __restrict__ C16 = reinterpret_cast<uint16_t*>(p.c);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int64_t lm0 = wm * WM + a * 32, ln0 = wn * WN + b * 32;
        if (n0 + ln0 + lrow >= p.N) continue;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (m0 + lm0 + 16 * j >= p.M) continue;
          uint32_t pl[4][4];
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            uint32_t hi0, lo0, hi1, lo1, w[4];
            split_scaled<KIND>(QxCplx{cr[a][b][8 * j + 2 * d] * scale, ci[a][b][8 * j + 2 * d] * scale}, hi0, lo0);
            split_scaled<KIND>(QxCplx{cr[a][b][8 * j + 2 * d + 1] * scale, ci[a][b][8 * j + 2 * d + 1] * scale}, hi1,
                               lo1);
            split_words(hi0, lo0, hi1, lo1, w);
#pragma unroll
            for (int q = 0; q < 4; ++q) pl[q][d] = w[q];
          }
          const int64_t e0 = coff + om.m(p, lm0 + 16 * j + 4 * g) + om.n(p, ln0 + lrow);  // a multiple of 8
#pragma unroll
          for (int q = 0; q < 4; ++q)
            *(v4u*)(C16 + split_chunk(e0) + 8 * q) = v4u{pl[q][0], pl[q][1], pl[q][2], pl[q][3]};
        }
      }
    return;
  }
  // split output in chunks: this lane's two chunks (block-element bits 3..9 = lane + 64 s),
  // their output offsets inside a block and the LDS stage index of each element
  struct {
    int64_t off[2];
    int sidx[2][8];
  } ck;
  if (p.c_split && p.ep_chunk) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int ch = lane + 64 * s;
      int lm = 0, ln = 0;
      int64_t off = 0;
#pragma unroll
      for (int b2 = 0; b2 < 7; ++b2)
        if ((ch >> b2) & 1) {
          lm += p.ep_lm[3 + b2];
          ln += p.ep_ln[3 + b2];
          off += p.ep_st[3 + b2];
        }
      ck.off[s] = off;
#pragma unroll
      for (int i = 0; i < 8; ++i)
        ck.sidx[s][i] = (lm + ((i & 1) ? p.ep_lm[0] : 0) + ((i & 2) ? p.ep_lm[1] : 0) + ((i & 4) ? p.ep_lm[2] : 0)) * 33 +
                        ln + ((i & 1) ? p.ep_ln[0] : 0) + ((i & 2) ? p.ep_ln[1] : 0) + ((i & 4) ? p.ep_ln[2] : 0);
    }
  }
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
      wave_lds_fence();
#pragma unroll
      for (int i = 0; i < 16; ++i)
        stage[(8 * (i / 4) + 4 * g + (i % 4)) * 33 + lrow] = QxCplx{cr[a][b][i] * scale, ci[a][b][i] * scale};
      wave_lds_fence();
      const int64_t lm0 = wm * WM + a * 32, ln0 = wn * WN + b * 32;
      if (p.c_split && p.ep_chunk) {
        // split output whose 8-element chunks lie inside the block: a lane converts
        // one chunk (block-element bits 0..2) and writes its four planes as 16-byte stores
        uint16_t* __restrict__ C16 = reinterpret_cast<uint16_t*>(p.c);
        const int64_t ebase = coff + om.m(p, lm0) + om.n(p, ln0);
        const bool inside = m0 + lm0 + 32 <= p.M && n0 + ln0 + 32 <= p.N;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          uint32_t pl[4][4];
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            uint32_t hi0, lo0, hi1, lo1, w[4];
            split_scaled<KIND>(stage[ck.sidx[s][2 * d]], hi0, lo0);
            split_scaled<KIND>(stage[ck.sidx[s][2 * d + 1]], hi1, lo1);
            split_words(hi0, lo0, hi1, lo1, w);
#pragma unroll
            for (int q = 0; q < 4; ++q) pl[q][d] = w[q];
          }
          const int64_t e0 = ebase + ck.off[s];  // a multiple of 8
          if (inside) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              *(v4u*)(C16 + split_chunk(e0) + 8 * q) = v4u{pl[q][0], pl[q][1], pl[q][2], pl[q][3]};
          } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const int lmi = ck.sidx[s][i] / 33, lni = ck.sidx[s][i] % 33;
              if (m0 + lm0 + lmi < p.M && n0 + ln0 + lni < p.N) store_split(C16, e0 + i, stage[ck.sidx[s][i]], KIND);
            }
          }
        }
        continue;
      }
      const int64_t eb = coff + om.m(p, lm0) + om.n(p, ln0) + off_lane;
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
        if (m0 + lm0 + lm < p.M && n0 + ln0 + ln < p.N) {
          const QxCplx v = stage[lm * 33 + ln];
          if (p.c_split) store_split(reinterpret_cast<uint16_t*>(p.c), eb + off, v, KIND);
          else if constexpr (KIND == 0) store_out(p.c + eb + off, v);
          else p.c[eb + off] = v;
        }
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

}  // namespace qx
