// Split-precision complex GEMM on BF16 or FP16 matrix cores with pre-split operands.
//
// Both operands are stored split (split_format.h: 64-byte chunks of 8 elements
// holding hi re, lo re, hi im, lo im), so the k loop converts nothing:
//   A B ~= Ah Bh + Ah Bl + Al Bh
// per real product, accumulated in FP32 by v_mfma_f32_32x32x16_bf16 (or _f16),
// with the complex product as four real ones (the sign of Im A Im B is applied
// by flipping the sign bits of the Im A fragments).  FP16 operands hold the
// values times their tensors' power-of-two scales; the epilogue divides them
// out (and applies the output's own scale when it is stored split FP16).
//
// Staging.  A tile is ROWS rows x 16 k; in LDS a row is 128 bytes = eight
// 16-byte slots, one per (k half g, plane q), and slot (g, q) of row r sits at
// position (4 g + q) ^ f(r), f(r) = (r & 7) ^ ((r >> 3) & 1), so the 8 or 16
// consecutive rows one fragment load reads at a time hit distinct banks.  A
// k-contiguous operand row is one 128-byte line in memory (two 64-byte chunks
// when k bit 3 is not the next stride), copied global -> LDS directly
// (global_load_lds_dwordx4: each lane moves 16 bytes, and a wave's 64 lanes
// fill 1 KB = 8 rows), leaving no staging registers; other operands go through
// registers.  NS LDS stages rotate: the copy of tile k + NS - 1 runs while tile
// k is multiplied.
#include <type_traits>

#include "gemm_common.h"

namespace qx {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

// slot position of (k half g, plane q) in LDS row r
__device__ __forceinline__ int slot_of(int r, int gq) { return gq ^ ((r & 7) ^ ((r >> 3) & 1)); }

// offset of tile-local row r < 256 (its bits are disjoint from those of the tile origin)
__device__ __forceinline__ int64_t row_offset(const OperandView& v, int r) {
  return v.bits ? scatter_bits<8>(r, v.rs, v.nr) : (int64_t)r * v.ld_r;
}
__device__ __forceinline__ int64_t origin_offset(const OperandView& v, int64_t r0) {
  return v.bits ? scatter_set_bits(r0, v.rs, v.nr) : r0 * v.ld_r;
}
// k < 16
__device__ __forceinline__ int64_t k_offset(const OperandView& v, int k) {
  return v.bits ? scatter_bits<4>(k, v.ks, v.nk) : (int64_t)k * v.ld_k;
}

// Direct global -> LDS copy of a k-contiguous operand tile.  The ROWS / 8
// one-KB pieces (8 rows each) are dealt to the NW waves round-robin; lane l of
// a piece fills slot l & 7 of row l >> 3.  Element offsets of chunk starts are
// multiples of 8 (k bits 0..2 are the three lowest strides), so a chunk's
// plane q is the 16 bytes at BF16 offset 4 e0 + 8 q.
template <int ROWS, int NW>
struct DmaTile {
  static constexpr int NP = ROWS / 8;
  static constexpr int NJ = NP / NW;  // pieces per wave
  static constexpr int NI = NJ;       // direct copies per wave per k tile
  static_assert(NJ * NW == NP, "pieces must divide evenly among the waves");
  int64_t goff[NJ];  // BF16 offset of this lane's 16 bytes, relative to the k tile origin
  __device__ inline void init(const OperandView& v, int64_t r0, int wave, int lane) {
    const int64_t k8 = k_offset(v, 8), base = origin_offset(v, r0);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int row = (wave + NW * j) * 8 + (lane >> 3);
      const int gq = slot_of(row, lane & 7);  // slot_of is its own inverse
      // rows past the end read row 0 of the tile: their results are never stored
      const int r = r0 + row < v.rows ? row : 0;
      goff[j] = 4 * (base + row_offset(v, r) + ((gq >> 2) ? k8 : 0)) + 8 * (gq & 3);
    }
  }
  // kb: element offset of the k tile origin (a multiple of 8)
  __device__ inline void issue(const uint16_t* X, int64_t kb, char* region, int wave) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const uint16_t* src = X + 4 * kb + goff[j];
      // (device pass only: the host pass of a kernel that names this builtin would drop its launch stub)
#if defined(__HIP_DEVICE_COMPILE__)
      __builtin_amdgcn_global_load_lds(src, (lds_void*)(region + (wave + NW * j) * 1024), 16, 0, 0);
#endif
    }
  }
  // the copies land in LDS by themselves
  __device__ inline void store(char*, int, int) const {}
};

// Register-staged copy for an operand that is not k-contiguous: consecutive
// lanes take consecutive rows, each lane gathers 8 k values of one row.
template <int ROWS, int NT>
struct RegTile {
  static constexpr int CH = ROWS * 2;
  static constexpr int P = (CH + NT - 1) / NT;
  static constexpr int NI = 0;  // no direct copies
  int64_t roff[P];
  int row[P], kg[P];
  u32x4 reg[P][4];
  __device__ inline void init(const OperandView& v, int64_t r0, int tid) {
    const int64_t base = origin_offset(v, r0);
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int c = tid + NT * s;
      row[s] = c < CH ? c % ROWS : -1;
      kg[s] = (c / ROWS) & 1;
      const int rr = c % ROWS;
      const int r = r0 + rr < v.rows ? rr : 0;
      roff[s] = base + row_offset(v, r) + k_offset(v, kg[s] * 8);
    }
  }
  __device__ inline void load(const OperandView& v, const uint16_t* X, int64_t kb) {
    int64_t jo[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) jo[j] = k_offset(v, j);
#pragma unroll
    for (int s = 0; s < P; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t e0 = roff[s] + kb + jo[2 * j], e1 = roff[s] + kb + jo[2 * j + 1];
          reg[s][q][j] = (uint32_t)X[split_off(e0, q)] | ((uint32_t)X[split_off(e1, q)] << 16);
        }
  }
  __device__ inline void store(char* region) const {
#pragma unroll
    for (int s = 0; s < P; ++s)
      if (row[s] >= 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          *(u32x4*)(region + row[s] * 128 + slot_of(row[s], kg[s] * 4 + q) * 16) = reg[s][q];
      }
  }
};

__device__ __forceinline__ v16f mfma(bf16x8 a, bf16x8 b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v16f mfma(f16x8 a, f16x8 b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}
// sign flip of all 8 values (BF16 and FP16 both keep the sign in bit 15)
template <class T>
__device__ __forceinline__ T neg(T x) {
  u32x4 t = __builtin_bit_cast(u32x4, x);
  t ^= 0x80008000u;
  return __builtin_bit_cast(T, t);
}

// s_waitcnt for "at most n vector-memory operations outstanding" (expcnt and
// lgkmcnt left at their maxima)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int I>
using Int = std::integral_constant<int, I>;

// Work-group barrier for the k loop.  __syncthreads() adds a release fence that
// waits for every outstanding vector-memory operation, including the direct
// copies still in flight into later stages; here the caller has already waited
// for exactly the copies that must have landed (wait_vm), and LDS operations are
// drained explicitly.  The empty asm statements keep the compiler from moving
// memory accesses across the barrier.
__device__ __forceinline__ void stage_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS reads and writes are done
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

}  // namespace

// BM x BN work-group tile computed by WGM x WGN waves; NS LDS stages.  Each
// wave takes its fragments of k tile t into registers before tile t is
// multiplied, so the copies of tiles t + 1 .. t + NS are in flight meanwhile.
template <int BM, int BN, int WGM, int WGN, int NS, bool A_KC, bool B_KC, bool F16>
__device__ __forceinline__ void gemm_split16(const GemmArgs& p) {
  using frag = typename std::conditional<F16, f16x8, bf16x8>::type;
  constexpr int NW = WGM * WGN, NT = 64 * NW;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int ABYTES = BM * 128, BBYTES = BN * 128, BUF = ABYTES + BBYTES;
  constexpr int STAGE = NW * 32 * 33 * 8;
  constexpr int SMEM = NS * BUF > STAGE ? NS * BUF : STAGE;
  __shared__ __attribute__((aligned(1024))) char smem[SMEM];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const TileCoord tc = tile_coord(p, BM, BN);
  // split storage is addressed from the tensor base by element offset (split_off)
  const uint16_t* __restrict__ A = reinterpret_cast<const uint16_t*>(p.a);
  const uint16_t* __restrict__ B = reinterpret_cast<const uint16_t*>(p.b);
  const int64_t m0 = tc.tm * BM, n0 = tc.tn * BN;
  const OperandView va = view_a(p, nullptr), vb = view_b(p, nullptr);

  typename std::conditional<A_KC, DmaTile<BM, NW>, RegTile<BM, NT>>::type sa;
  typename std::conditional<B_KC, DmaTile<BN, NW>, RegTile<BN, NT>>::type sb;
  if constexpr (A_KC) sa.init(va, m0, wave, lane);
  else sa.init(va, m0, tid);
  if constexpr (B_KC) sb.init(vb, n0, wave, lane);
  else sb.init(vb, n0, tid);
  constexpr int NI = decltype(sa)::NI + decltype(sb)::NI;  // direct copies per wave per k tile

  const int64_t nk = (p.K + 15) / 16;  // K is a multiple of 16, or 8 (checked by the launcher)
  // last k tile fetched and the element offsets of its origin in A and B
  int64_t kf = 0, ka = tc.aoff, kb = tc.boff;
  // start the copy of k tile kf into LDS buffer bi (register-staged operands: the loads only)
  auto fetch = [&](auto bsel) {
    char* buf = smem + decltype(bsel)::value * BUF;
    if constexpr (A_KC) sa.issue(A, ka, buf, wave);
    else sa.load(va, A, ka);
    if constexpr (B_KC) sb.issue(B, kb, buf + ABYTES, wave);
    else sb.load(vb, B, kb);
  };
  auto commit = [&](auto bsel) {
    char* buf = smem + decltype(bsel)::value * BUF;
    if constexpr (!A_KC) sa.store(buf);
    else sa.store(buf, wave, lane);
    if constexpr (!B_KC) sb.store(buf + ABYTES);
    else sb.store(buf + ABYTES, wave, lane);
  };
  auto advance = [&]() {
    const int z = __builtin_ctzll(~(uint64_t)kf);
    ka += p.a_kinc[z];
    kb += p.b_kinc[z];
    ++kf;
  };

  v16f cr[FM][FN], ci[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      cr[a][b] = v16f{0};
      ci[a][b] = v16f{0};
    }

  // prologue: tiles 0 .. NS - 1, one per LDS buffer; then wait for tile 0
  fetch(Int<0>{});
  commit(Int<0>{});
  if (nk > 1) {
    advance();
    fetch(Int<1>{});
    commit(Int<1>{});
  }
  if constexpr (NS > 2) {
    if (nk > 2) {
      advance();
      fetch(Int<2>{});
      commit(Int<2>{});
    }
  }
  if constexpr (NS > 3) {
    if (nk > 3) {
      advance();
      fetch(Int<3>{});
      commit(Int<3>{});
    }
  }
  if (nk >= NS) wait_vm<(NS - 1) * NI>();
  else wait_vm<0>();
  stage_barrier();
  if (p.K == 8) {
    // one k tile whose upper half (k 8..15) does not exist: the copies filled those
    // slots with the lower half again (k bit 3 has no stride), so zero them
    for (int i = tid; i < 4 * (BM + BN); i += NT) {
      const int row = i >> 2, q = i & 3;
      char* base = row < BM ? smem + row * 128 : smem + ABYTES + (row - BM) * 128;
      const int r = row < BM ? row : row - BM;
      *(u32x4*)(base + slot_of(r, 4 + q) * 16) = u32x4{0, 0, 0, 0};
    }
    stage_barrier();
  }

  // fragment addresses: this lane's tile row (mod 32) and the four slots of its k half
  const int frow = lane & 31;
  int fo[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) fo[q] = frow * 128 + slot_of(frow, (lane >> 5) * 4 + q) * 16;

  // One k tile: every wave reads all its fragments of tile kt (buffer BI), a barrier
  // frees the buffer, and the copy of tile kt + NS into it starts before the products
  // run, so a copy has NS steps to land instead of NS - 1.
  auto step = [&](int64_t kt, auto bsel) {
    constexpr int BI = decltype(bsel)::value;
    const bool more = kt + NS < nk;
    const char* bufA = smem + BI * BUF;
    const char* bufB = bufA + ABYTES;
    frag arh[FM], arl[FM], aih[FM], ail[FM], brh[FN], brl[FN], bih[FN], bil[FN];
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const char* r = bufA + (wm * WM + a * 32) * 128;
      arh[a] = *(const frag*)(r + fo[0]);
      arl[a] = *(const frag*)(r + fo[1]);
      aih[a] = *(const frag*)(r + fo[2]);
      ail[a] = *(const frag*)(r + fo[3]);
    }
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      const char* r = bufB + (wn * WN + b * 32) * 128;
      brh[b] = *(const frag*)(r + fo[0]);
      brl[b] = *(const frag*)(r + fo[1]);
      bih[b] = *(const frag*)(r + fo[2]);
      bil[b] = *(const frag*)(r + fo[3]);
    }
    stage_barrier();
    if (more) {
      advance();
      fetch(bsel);
    }
    // Im C += Im A Re B; Re C += Re A Re B; Im C += Re A Im B; Re C -= Im A Im B
    // (hi hi, hi lo, lo hi each); consecutive products update different accumulators
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) ci[a][b] = mfma(aih[a], brh[b], ci[a][b]);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) cr[a][b] = mfma(arh[a], brh[b], cr[a][b]);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) ci[a][b] = mfma(aih[a], brl[b], ci[a][b]);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) cr[a][b] = mfma(arh[a], brl[b], cr[a][b]);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) ci[a][b] = mfma(ail[a], brh[b], ci[a][b]);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) cr[a][b] = mfma(arl[a], brh[b], cr[a][b]);
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      aih[a] = neg(aih[a]);
      ail[a] = neg(ail[a]);
    }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) ci[a][b] = mfma(arh[a], bih[b], ci[a][b]);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) cr[a][b] = mfma(aih[a], bih[b], cr[a][b]);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) ci[a][b] = mfma(arh[a], bil[b], ci[a][b]);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) cr[a][b] = mfma(aih[a], bil[b], cr[a][b]);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) ci[a][b] = mfma(arl[a], bih[b], ci[a][b]);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) cr[a][b] = mfma(ail[a], bih[b], cr[a][b]);
    if (more) commit(bsel);
    // this wave's copies of tile kt + 1 have landed once at most the later tiles'
    // copies are outstanding; the barrier then publishes every wave's pieces
    if (kt + 1 < nk) {
      if (more) wait_vm<(NS - 1) * NI>();
      else wait_vm<0>();
      stage_barrier();
    }
  };
  int64_t kt = 0;
  for (; kt + NS <= nk; kt += NS) {
    step(kt, Int<0>{});
    step(kt + 1, Int<1>{});
    if constexpr (NS > 2) step(kt + 2, Int<2>{});
    if constexpr (NS > 3) step(kt + 3, Int<3>{});
  }
  if (kt < nk) step(kt, Int<0>{});
  if constexpr (NS > 2)
    if (kt + 1 < nk) step(kt + 1, Int<1>{});
  if constexpr (NS > 3)
    if (kt + 2 < nk) step(kt + 2, Int<2>{});

  const OutMap om = out_map(p, m0, n0);
  // FP16: divide out the operands' scales, apply the output's when it is stored split (powers of two: exact)
  const float f = F16 ? (p.c_split ? out_scale(p.c_scale) : 1.f) / (out_scale(p.a_scale) * out_scale(p.b_scale))
                      : 1.f;
  store_blocks<FM, FN, WM, WN, true, F16 ? 2 : 1>(p, tc.coff, om, m0, n0, wm, wn, lane, cr, ci, f,
                                                 reinterpret_cast<QxCplx*>(smem) + wave * (32 * 33));
}

// A wave's fragments of one k tile: for each of its FM (FN) 32-row blocks of A (B), the four
// planes of its lane's 8 consecutive k.
template <class frag, int FM, int FN>
struct Frags {
  frag arh[FM], arl[FM], aih[FM], ail[FM], brh[FN], brl[FN], bih[FN], bil[FN];
};

template <class frag, int FM, int FN>
__device__ __forceinline__ void read_frags(Frags<frag, FM, FN>& f, const char* bufA, const char* bufB,
                                           const int (&fo)[4]) {
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    const char* r = bufA + a * 32 * 128;
    f.arh[a] = *(const frag*)(r + fo[0]);
    f.arl[a] = *(const frag*)(r + fo[1]);
    f.aih[a] = *(const frag*)(r + fo[2]);
    f.ail[a] = *(const frag*)(r + fo[3]);
  }
#pragma unroll
  for (int b = 0; b < FN; ++b) {
    const char* r = bufB + b * 32 * 128;
    f.brh[b] = *(const frag*)(r + fo[0]);
    f.brl[b] = *(const frag*)(r + fo[1]);
    f.bih[b] = *(const frag*)(r + fo[2]);
    f.bil[b] = *(const frag*)(r + fo[3]);
  }
}

// The complex product of one k tile as 12 real MFMAs per accumulator pair (hi hi, hi lo, lo hi of
// Re A Re B, Re A Im B, Im A Re B and -Im A Im B); consecutive MFMAs update different accumulators.
template <class frag, int FM, int FN>
__device__ __forceinline__ void mma_tile(Frags<frag, FM, FN>& f, v16f (&cr)[FM][FN], v16f (&ci)[FM][FN]) {
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) ci[a][b] = mfma(f.aih[a], f.brh[b], ci[a][b]);
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) cr[a][b] = mfma(f.arh[a], f.brh[b], cr[a][b]);
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) ci[a][b] = mfma(f.aih[a], f.brl[b], ci[a][b]);
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) cr[a][b] = mfma(f.arh[a], f.brl[b], cr[a][b]);
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) ci[a][b] = mfma(f.ail[a], f.brh[b], ci[a][b]);
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) cr[a][b] = mfma(f.arl[a], f.brh[b], cr[a][b]);
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    f.aih[a] = neg(f.aih[a]);
    f.ail[a] = neg(f.ail[a]);
  }
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) ci[a][b] = mfma(f.arh[a], f.bih[b], ci[a][b]);
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) cr[a][b] = mfma(f.aih[a], f.bih[b], cr[a][b]);
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) ci[a][b] = mfma(f.arh[a], f.bil[b], ci[a][b]);
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) cr[a][b] = mfma(f.aih[a], f.bil[b], cr[a][b]);
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) ci[a][b] = mfma(f.arl[a], f.bih[b], ci[a][b]);
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) cr[a][b] = mfma(f.ail[a], f.bih[b], cr[a][b]);
}

// Software-pipelined form for one work-group per CU (one wavefront per SIMD, so the
// accumulators and two fragment sets fit in its registers): NS LDS stages hold k tiles
// t .. t + NS - 1.  Step t, after one barrier (tile t + 1 has landed; every wave's reads of
// tile t are done, so its buffer is free), issues the copy of tile t + NS into that buffer,
// issues the LDS reads of tile t + 1's fragments, and runs tile t's MFMAs on the fragments
// read during step t - 1, so the reads overlap the products and a copy has NS - 1 steps to land.
template <int BM, int BN, int WGM, int WGN, int NS, bool A_KC, bool B_KC, bool F16>
__device__ __forceinline__ void gemm_split16_pipe(const GemmArgs& p) {
  using frag = typename std::conditional<F16, f16x8, bf16x8>::type;
  constexpr int NW = WGM * WGN, NT = 64 * NW;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int ABYTES = BM * 128, BBYTES = BN * 128, BUF = ABYTES + BBYTES;
  constexpr int STAGE = NW * 32 * 33 * 8;
  constexpr int SMEM = NS * BUF > STAGE ? NS * BUF : STAGE;
  static_assert(NS >= 2 && NS <= 4, "stages");
  __shared__ __attribute__((aligned(1024))) char smem[SMEM];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const TileCoord tc = tile_coord(p, BM, BN);
  const uint16_t* __restrict__ A = reinterpret_cast<const uint16_t*>(p.a);
  const uint16_t* __restrict__ B = reinterpret_cast<const uint16_t*>(p.b);
  const int64_t m0 = tc.tm * BM, n0 = tc.tn * BN;
  const OperandView va = view_a(p, nullptr), vb = view_b(p, nullptr);

  typename std::conditional<A_KC, DmaTile<BM, NW>, RegTile<BM, NT>>::type sa;
  typename std::conditional<B_KC, DmaTile<BN, NW>, RegTile<BN, NT>>::type sb;
  if constexpr (A_KC) sa.init(va, m0, wave, lane);
  else sa.init(va, m0, tid);
  if constexpr (B_KC) sb.init(vb, n0, wave, lane);
  else sb.init(vb, n0, tid);
  constexpr int NI = decltype(sa)::NI + decltype(sb)::NI;  // direct copies per wave per k tile

  const int64_t nk = (p.K + 15) / 16;  // K is a multiple of 16, or 8 (checked by the launcher)
  int64_t kf = 0, ka = tc.aoff, kb = tc.boff;
  // register-staged loads first, so a later wait for them leaves the direct copies in flight
  auto fetch = [&](int bi) {
    char* buf = smem + bi * BUF;
    if constexpr (!A_KC) sa.load(va, A, ka);
    if constexpr (!B_KC) sb.load(vb, B, kb);
    if constexpr (A_KC) sa.issue(A, ka, buf, wave);
    if constexpr (B_KC) sb.issue(B, kb, buf + ABYTES, wave);
  };
  auto commit = [&](int bi) {
    char* buf = smem + bi * BUF;
    if constexpr (!A_KC) sa.store(buf);
    if constexpr (!B_KC) sb.store(buf + ABYTES);
  };
  auto advance = [&]() {
    const int z = __builtin_ctzll(~(uint64_t)kf);
    ka += p.a_kinc[z];
    kb += p.b_kinc[z];
    ++kf;
  };

  v16f cr[FM][FN], ci[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      cr[a][b] = v16f{0};
      ci[a][b] = v16f{0};
    }

  // prologue: tiles 0 .. NS - 1 into buffers 0 .. NS - 1; wait for tile 0
  fetch(0);
  commit(0);
#pragma unroll
  for (int j = 1; j < NS; ++j)
    if (j < nk) {
      advance();
      fetch(j);
      commit(j);
    }
  if (nk >= NS) wait_vm<(NS - 1) * NI>();
  else wait_vm<0>();
  stage_barrier();
  if (p.K == 8) {
    // one k tile whose upper half (k 8..15) does not exist: zero those slots
    for (int i = tid; i < 4 * (BM + BN); i += NT) {
      const int row = i >> 2, q = i & 3;
      char* base = row < BM ? smem + row * 128 : smem + ABYTES + (row - BM) * 128;
      const int r = row < BM ? row : row - BM;
      *(u32x4*)(base + slot_of(r, 4 + q) * 16) = u32x4{0, 0, 0, 0};
    }
    stage_barrier();
  }

  const int frow = lane & 31;
  int fo[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) fo[q] = frow * 128 + slot_of(frow, (lane >> 5) * 4 + q) * 16;
  const int aoff = wm * WM * 128, boff = ABYTES + wn * WN * 128;

  Frags<frag, FM, FN> f0, f1;
  read_frags(f0, smem + aoff, smem + boff, fo);
  int cur = 0;  // buffer of tile t
  auto pstep = [&](int64_t t, Frags<frag, FM, FN>& fc, Frags<frag, FM, FN>& fn) {
    const bool has_next = t + 1 < nk, refill = t + NS < nk;
    if (has_next) {
      if (t + NS - 1 < nk) wait_vm<(NS - 2) * NI>();
      else wait_vm<0>();
    }
    stage_barrier();  // this wave's reads of tile t have landed (lgkmcnt 0); tile t + 1 is visible
    if (refill) {
      advance();
      fetch(cur);
    }
    const int nxt = cur + 1 == NS ? 0 : cur + 1;
    if (has_next) read_frags(fn, smem + nxt * BUF + aoff, smem + nxt * BUF + boff, fo);
    mma_tile(fc, cr, ci);
    if (refill) commit(cur);
    cur = nxt;
  };
  for (int64_t t = 0; t < nk; t += 2) {
    pstep(t, f0, f1);
    if (t + 1 < nk) pstep(t + 1, f1, f0);
  }

  // the last step's barrier followed every wave's last LDS read: the stage areas are free
  const OutMap om = out_map(p, m0, n0);
  const float f = F16 ? (p.c_split ? out_scale(p.c_scale) : 1.f) / (out_scale(p.a_scale) * out_scale(p.b_scale))
                      : 1.f;
  store_blocks<FM, FN, WM, WN, true, F16 ? 2 : 1>(p, tc.coff, om, m0, n0, wm, wn, lane, cr, ci, f,
                                                 reinterpret_cast<QxCplx*>(smem) + wave * (32 * 33));
}

// Two wavefronts per SIMD where the LDS stages allow two work-groups per CU.
#define QX_SPLIT16_BOUNDS \
  __launch_bounds__(64 * WGM * WGN, (!PIPE && (WGM * WGN == 8 || NS * 128 * (BM + BN) <= 80 * 1024)) ? 2 : 1)

// PIPE: the software-pipelined form, one work-group per CU.
template <int BM, int BN, int WGM, int WGN, int NS, bool A_KC, bool B_KC, bool PIPE>
__global__ QX_SPLIT16_BOUNDS void k_gemm_bf16s(GemmArgs p) {
  if constexpr (PIPE) gemm_split16_pipe<BM, BN, WGM, WGN, NS, A_KC, B_KC, false>(p);
  else gemm_split16<BM, BN, WGM, WGN, NS, A_KC, B_KC, false>(p);
}
template <int BM, int BN, int WGM, int WGN, int NS, bool A_KC, bool B_KC, bool PIPE>
__global__ QX_SPLIT16_BOUNDS void k_gemm_fp16s(GemmArgs p) {
  if constexpr (PIPE) gemm_split16_pipe<BM, BN, WGM, WGN, NS, A_KC, B_KC, true>(p);
  else gemm_split16<BM, BN, WGM, WGN, NS, A_KC, B_KC, true>(p);
}

template <int BM, int BN, int WGM, int WGN, int NS, bool A_KC, bool B_KC, bool F16, bool PIPE>
static void launch_kernel(dim3 grid, dim3 block, hipStream_t s, const GemmArgs& a) {
  if constexpr (F16)
    hipLaunchKernelGGL((k_gemm_fp16s<BM, BN, WGM, WGN, NS, A_KC, B_KC, PIPE>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_gemm_bf16s<BM, BN, WGM, WGN, NS, A_KC, B_KC, PIPE>), grid, block, 0, s, a);
}

template <int BM, int BN, int WGM, int WGN, int NS, bool F16, bool PIPE = false>
static hipError_t launch_bf16s(const GemmArgs& a, hipStream_t s) {
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  const int64_t nwg = tiles * (int64_t)a.n_items * (1LL << a.nh);
  if (nwg <= 0) return hipSuccess;
  if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool akc = gemm_a_kc(a), bkc = gemm_b_kc(a);
  dim3 grid((unsigned)nwg), block(64 * WGM * WGN);
  if (akc && bkc) launch_kernel<BM, BN, WGM, WGN, NS, true, true, F16, PIPE>(grid, block, s, a);
  else if (akc) launch_kernel<BM, BN, WGM, WGN, NS, true, false, F16, PIPE>(grid, block, s, a);
  else if (bkc) launch_kernel<BM, BN, WGM, WGN, NS, false, true, F16, PIPE>(grid, block, s, a);
  else launch_kernel<BM, BN, WGM, WGN, NS, false, false, F16, PIPE>(grid, block, s, a);
  return hipGetLastError();
}

template <bool F16>
static hipError_t launch_split16(const GemmArgs& a, int tile, hipStream_t s) {
  // operands must be stored split, and K a multiple of the 16-wide k tile (or 8: one half tile)
  if (!a.a_split || !a.b_split || !gemm_split_k_ok(a)) return hipErrorInvalidValue;
  switch (tile) {
    case GEMM_TILE_64x64: return launch_bf16s<64, 64, 2, 2, 2, F16>(a, s);
    case GEMM_TILE_128x64: return launch_bf16s<128, 64, 2, 2, 3, F16>(a, s);
    case GEMM_TILE_64x128: return launch_bf16s<64, 128, 2, 2, 3, F16>(a, s);
    case GEMM_TILE_256x128: return launch_bf16s<256, 128, 4, 2, 3, F16>(a, s);
    case GEMM_TILE_128x256: return launch_bf16s<128, 256, 2, 4, 3, F16>(a, s);
    case GEMM_TILE_128x128P3: return launch_bf16s<128, 128, 2, 2, 3, F16, true>(a, s);
    case GEMM_TILE_128x128P4: return launch_bf16s<128, 128, 2, 2, 4, F16, true>(a, s);
    default: return launch_bf16s<128, 128, 2, 2, 2, F16>(a, s);
  }
}

hipError_t launch_gemm_bf16(const GemmArgs& a, int tile, hipStream_t s) { return launch_split16<false>(a, tile, s); }
hipError_t launch_gemm_fp16(const GemmArgs& a, int tile, hipStream_t s) { return launch_split16<true>(a, tile, s); }

}  // namespace qx
