// Thin complex products: one operand ("W") of at most 32 rows and K at most 32,
// the other ("X") long.  Such a product reads X once and writes an output of
// about X's size, so HBM bandwidth bounds it, not the matrix cores.
//
// Work is spread over independent wavefronts (no work-group barrier): a wave
// owns eight (four for K > 16) consecutive 16-row blocks of X, keeps all of W
// in registers as matrix-core fragments, loads every block of X it owns
// straight into fragment registers (all those loads in flight together),
// multiplies each block on a 16x16 matrix-core shape and writes the 16 x S
// result through a per-wave LDS stage in ascending output-address order, so
// the stores form contiguous runs whatever the output's index order.
//
// A complex product as real matrix products (Sec. IV-A): with X' = [Re X, Im X]
// along k, W'r = [Re W, -Im W] and W'i = [Im W, Re W],
//   Re C = X' W'r,   Im C = X' W'i.
// Complex64 operands run v_mfma_f32_16x16x4_f32 with Re / Im interleaved along
// k; split operands (hi + lo planes, split_format.h) run
// v_mfma_f32_16x16x32_bf16 / _f16 with the terms hi hi + hi lo + lo hi, as the
// large products do.  The k order of the real products is free as long as
// X' and W' lanes agree, which both fragment layouts below guarantee.
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "gemm_common.h"

namespace qx {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int THIN_MAX_S = 32;  // rows of W
constexpr int THIN_MAX_K = 32;
constexpr int THIN_EP = 9;      // index bits of a 16 x 32 output block

// The product C = X W^T in thin form, built on the host from the matrix-product arguments.
// Every offset is a sum of per-bit strides (linear layouts too: bit b of an index with stride
// s contributes s << b), in elements.
struct ThinArgs {
  const void* x;
  const void* w;
  void* c;
  int64_t L;                        // rows of X
  int32_t S, K;                     // rows of W, contracted length
  int32_t nr;                       // bits of a row index of X
  int32_t kind;                     // storage of X and W: 0 complex64, 1 split BF16, 2 split FP16 (scaled)
  int32_t c_kind;                   // storage of C, likewise
  int32_t kc, w_kc;                 // X's / W's k bits 0..2 have strides 1, 2, 4 and 16-byte alignment holds
  const float *x_scale, *w_scale, *c_scale;  // FP16 tensor scales (null = 1)
  int64_t x_rst[QX_GEMM_BITS], c_rst[QX_GEMM_BITS];  // X row bits in X and in C
  int64_t x_kst[5], w_kst[5], w_sst[5], c_sst[5];    // k bits in X and W; W row bits in W and in C
  int64_t x_item, w_item, c_item;
  const int64_t *x_gather, *w_gather;
  int32_t n_items, nh;
  int64_t x_hs[QX_MAX_HBITS], w_hs[QX_MAX_HBITS], c_hs[QX_MAX_HBITS];
  // the bits of a 16 x SP output block in ascending order of output stride: stride and
  // contribution to the block row i / to s (bits that do not exist sort last with stride 0)
  int64_t ep_st[THIN_EP];
  int32_t ep_i[THIN_EP], ep_s[THIN_EP];
  int32_t ep_chunk;                 // split C whose three lowest block strides are 1, 2, 4
};

__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(v4u a, v4u b, v4f c, bf16x8) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                 0);
}
__device__ __forceinline__ v4f mfma16(v4u a, v4u b, v4f c, f16x8) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0,
                                                0);
}

__device__ __forceinline__ v4u pack8(const uint16_t (&h)[8]) {
  return v4u{(uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16),
             (uint32_t)h[4] | ((uint32_t)h[5] << 16), (uint32_t)h[6] | ((uint32_t)h[7] << 16)};
}

// Fragments of one 16-row block of X held by one lane.  Lane (i = lane % 16, q = lane / 16)
// supplies row i of the block.  Complex64: the KP / 2 real k values q KP/2 .. of X' with
// Re / Im interleaved, i.e. complex k in [q KP/4, (q + 1) KP/4).  Split: per 16-k chunk c,
// the 8 values of plane (hi, lo) of component q / 2 at complex k 16 c + 8 (q % 2) + 0..7.
template <int KIND, int KP>
struct XFrag;
template <int KP>
struct XFrag<0, KP> {
  float a[KP / 2];
};
template <int KP>
struct XFrag<1, KP> {
  v4u hi[KP / 16], lo[KP / 16];
};
template <int KP>
struct XFrag<2, KP> : XFrag<1, KP> {};

}  // namespace

// 16-row blocks per wave: eight (K up to 16) or four (K up to 32), all loaded at once.
template <int KP>
constexpr int thin_nb() {
  return KP == 32 ? 4 : 8;
}

// Sum of st[b] over the set bits b < N of v (a select per bit, no branch).
template <int N, class T>
__device__ __forceinline__ int64_t bit_sum(int v, const T* st) {
  int64_t o = 0;
#pragma unroll
  for (int b = 0; b < N; ++b) o += ((v >> b) & 1) ? (int64_t)st[b] : 0;
  return o;
}

// KIND: operand storage; KP: K rounded up to 16 or 32 (complex64 also 4 or 8); SP: S rounded up to
// 16 or 32; XKC: X is
// k-contiguous (16-byte fragment loads).  Every load is issued unconditionally (lanes outside an
// operand read a valid element of it), so no load waits behind a branch.
template <int KIND, int KP, int SP, bool XKC>
__global__ __launch_bounds__(256) void k_gemm_thin(ThinArgs p) {
  constexpr int NCB = SP / 16;               // 16-column blocks of the output
  constexpr int NKC = KP / 16;               // 16-k chunks (split)
  constexpr int PITCH = SP + 1;              // stage row pitch in complex values
  constexpr int NE = 16 * SP;                // elements of an output block
  constexpr int NB = thin_nb<KP>();
  using hfrag = typename std::conditional<KIND == 2, f16x8, bf16x8>::type;
  __shared__ QxCplx stage_all[4 * 16 * PITCH];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  QxCplx* stage = stage_all + wave * (16 * PITCH);
  const int64_t L = p.L;
  const int64_t wpz = (L + 16 * NB - 1) / (16 * NB);  // waves per batch item / shared-slice index
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave;
  if (gw >= wpz * ((int64_t)p.n_items << p.nh)) return;
  const int64_t z = gw / wpz;
  const int64_t rw0 = (gw - z * wpz) * (16 * NB);  // first row of the wave (bits 0 .. log2(16 NB) - 1 clear)
  const int item = (int)(z >> p.nh);
  int64_t xo = (int64_t)item * p.x_item + (p.x_gather ? p.x_gather[item] : 0);
  int64_t wo = (int64_t)item * p.w_item + (p.w_gather ? p.w_gather[item] : 0);
  int64_t co = (int64_t)item * p.c_item;
  for (uint32_t hb = (uint32_t)(z & ((1LL << p.nh) - 1)); hb; hb &= hb - 1) {
    const int i = __builtin_ctz(hb);
    xo += p.x_hs[i];
    wo += p.w_hs[i];
    co += p.c_hs[i];
  }
  const int64_t xw = xo + scatter_set_bits(rw0, p.x_rst, p.nr);  // row rw0 in X and in C
  const int64_t cw = co + scatter_set_bits(rw0, p.c_rst, p.nr);
  // strides in registers: row bits 0..6 (inside the wave), k bits, W row bits, output block bits
  int64_t xrs[7], crs[7], xks[5], wks[5], wss[5], est[THIN_EP];
  int ei[THIN_EP], es[THIN_EP];
#pragma unroll
  for (int b = 0; b < 7; ++b) {
    xrs[b] = p.x_rst[b];
    crs[b] = p.c_rst[b];
  }
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    xks[b] = p.x_kst[b];
    wks[b] = p.w_kst[b];
    wss[b] = p.w_sst[b];
  }
#pragma unroll
  for (int b = 0; b < THIN_EP; ++b) {
    est[b] = p.ep_st[b];
    ei[b] = p.ep_i[b];
    es[b] = p.ep_s[b];
  }
  const int K = p.K, S = p.S;
  const bool wkc = p.w_kc != 0;
  const int li = lane & 15, q = lane >> 4;
  const int64_t xr_lane = bit_sum<4>(li, xrs);

  // ---- X fragments of all NB blocks, their loads in flight together.  Lanes past the last row
  // read row rw0, and k slots at or past K read k mod K of the same row: neither value needs a
  // mask (W' is zero at k >= K, and rows past the end are never stored), so no load has to
  // complete before the next is issued.
  XFrag<KIND, KP> xf[NB];
  constexpr int NKO = KIND == 0 ? (XKC ? 1 : KP / 4) : (XKC ? NKC : NKC * 8);
  int64_t xko[NKO];  // k offsets of this lane's fragment values
#pragma unroll
  for (int j = 0; j < NKO; ++j) {
    int k;
    if constexpr (KIND == 0) k = q * (KP / 4) + (XKC ? 0 : j);
    else k = 16 * (XKC ? j : j / 8) + 8 * (q & 1) + (XKC ? 0 : j % 8);
    xko[j] = bit_sum<5>(k < K ? k : k % K, xks);
  }
#pragma unroll
  for (int blk = 0; blk < NB; ++blk) {
    const int64_t xr = rw0 + 16 * blk + li < L ? xw + bit_sum<7>(blk << 4, xrs) + xr_lane : xw;
    if constexpr (KIND == 0) {
      const QxCplx* __restrict__ X = static_cast<const QxCplx*>(p.x);
      if constexpr (XKC) {
        const float* src = reinterpret_cast<const float*>(X + xr + xko[0]);
#pragma unroll
        for (int j = 0; j < KP / 8; ++j) {
          const v4f v = *reinterpret_cast<const v4f*>(src + 4 * j);
#pragma unroll
          for (int e = 0; e < 4; ++e) xf[blk].a[4 * j + e] = v[e];
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < KP / 4; ++kk) {
          const QxCplx v = X[xr + xko[kk]];
          xf[blk].a[2 * kk] = v.x;
          xf[blk].a[2 * kk + 1] = v.y;
        }
      }
    } else {
      const uint16_t* __restrict__ X16 = static_cast<const uint16_t*>(p.x);
      const int pl = 2 * (q >> 1);
#pragma unroll
      for (int c = 0; c < NKC; ++c) {
        if constexpr (XKC) {
          const v4u* src = reinterpret_cast<const v4u*>(X16 + split_chunk(xr + xko[c]) + 8 * pl);  // a multiple of 8
          xf[blk].hi[c] = src[0];
          xf[blk].lo[c] = src[1];
        } else {
          uint16_t h[8], l[8];
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            const int64_t e = xr + xko[8 * c + v];
            h[v] = X16[split_off(e, pl)];
            l[v] = X16[split_off(e, pl + 1)];
          }
          xf[blk].hi[c] = pack8(h);
          xf[blk].lo[c] = pack8(l);
        }
      }
    }
  }

  // ---- W as B-operand fragments: lane (j = li, q) holds column s = 16 cb + j
  float bre[NCB][KIND == 0 ? KP / 2 : 1], bim[NCB][KIND == 0 ? KP / 2 : 1];
  v4u brh[NCB][NKC], brl[NCB][NKC], bih[NCB][NKC], bil[NCB][NKC];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int s = 16 * cb + li;
    const bool sok = s < S;
    const int64_t so = wo + bit_sum<5>(s, wss);
    if constexpr (KIND == 0) {
      const QxCplx* __restrict__ W = static_cast<const QxCplx*>(p.w);
      const int64_t kq = bit_sum<5>(q * (KP / 4), wks);
#pragma unroll
      for (int kk = 0; kk < KP / 4; ++kk) {
        const int k = q * (KP / 4) + kk;
        const bool ok = sok && k < K;
        const QxCplx v = W[ok ? so + kq + bit_sum<5>(kk, wks) : wo];
        const float re = ok ? v.x : 0.f, im = ok ? v.y : 0.f;
        bre[cb][2 * kk] = re;
        bre[cb][2 * kk + 1] = -im;
        bim[cb][2 * kk] = im;
        bim[cb][2 * kk + 1] = re;
      }
    } else {
      const uint16_t* __restrict__ W16 = static_cast<const uint16_t*>(p.w);
#pragma unroll
      for (int c = 0; c < NKC; ++c) {
        const int k0 = 16 * c + 8 * (q & 1);
        v4u rh, rl, ih, il;
        if (wkc) {
          // 8 consecutive k of one row form one chunk: its four planes are 16-byte loads
          const bool ok = sok && k0 < K;
          const int64_t e0 = ok ? so + bit_sum<5>(k0, wks) : wo;  // a multiple of 8
          const v4u* src = reinterpret_cast<const v4u*>(W16 + split_chunk(e0));
          const v4u zero = v4u{0, 0, 0, 0};
          rh = ok ? src[0] : zero;
          rl = ok ? src[1] : zero;
          ih = ok ? src[2] : zero;
          il = ok ? src[3] : zero;
        } else {
          uint16_t h[4][8];
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            const bool ok = sok && k0 + v < K;
            const int64_t e = ok ? so + bit_sum<5>(k0 + v, wks) : wo;
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) {
              const uint16_t x = W16[split_off(e, pl)];
              h[pl][v] = ok ? x : (uint16_t)0;
            }
          }
          rh = pack8(h[0]);
          rl = pack8(h[1]);
          ih = pack8(h[2]);
          il = pack8(h[3]);
        }
        // k' of W'r: Re W for q < 2, -Im W for q >= 2; of W'i: Im W, then Re W
        const bool lo_half = q < 2;
        brh[cb][c] = lo_half ? rh : (ih ^ 0x80008000u);
        brl[cb][c] = lo_half ? rl : (il ^ 0x80008000u);
        bih[cb][c] = lo_half ? ih : rh;
        bil[cb][c] = lo_half ? il : rl;
      }
    }
  }

  const float fscale = (p.c_kind == 2 ? out_scale(p.c_scale) : 1.f) /
                       (KIND == 2 ? out_scale(p.x_scale) * out_scale(p.w_scale) : 1.f);
  const int c_kind = KIND == 0 ? 0 : p.c_kind;  // complex64 operands give a complex64 product
  const bool chunked = c_kind != 0 && p.ep_chunk != 0;
  // this lane's element of an output block (block bits 0..5), and the 8-element chunk whose plane
  // lane % 4 it writes (chunk bits 3..6 = lane / 4)
  const int ep_li = (int)bit_sum<6>(lane, ei);
  const int ep_ls = (int)bit_sum<6>(lane, es);
  const int64_t ep_lo = bit_sum<6>(lane, est);
  const int qi_lane = (int)bit_sum<4>(lane >> 2, ei + 3);
  const int qs_lane = (int)bit_sum<4>(lane >> 2, es + 3);
  const int64_t qo_lane = bit_sum<4>(lane >> 2, est + 3);

  // ---- products and output, block by block
#pragma unroll
  for (int blk = 0; blk < NB; ++blk) {
    const int64_t r0 = rw0 + 16 * blk;
    if (r0 >= L) break;
    v4f cr[NCB], ci[NCB], cr2[NCB], ci2[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) cr[cb] = ci[cb] = cr2[cb] = ci2[cb] = v4f{0.f, 0.f, 0.f, 0.f};
    if constexpr (KIND == 0) {
#pragma unroll
      for (int t = 0; t < KP / 2; t += 2)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          cr[cb] = mfma16(xf[blk].a[t], bre[cb][t], cr[cb]);
          ci[cb] = mfma16(xf[blk].a[t], bim[cb][t], ci[cb]);
          cr2[cb] = mfma16(xf[blk].a[t + 1], bre[cb][t + 1], cr2[cb]);
          ci2[cb] = mfma16(xf[blk].a[t + 1], bim[cb][t + 1], ci2[cb]);
        }
    } else {
#pragma unroll
      for (int c = 0; c < NKC; ++c)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          cr[cb] = mfma16(xf[blk].hi[c], brh[cb][c], cr[cb], hfrag{});
          ci[cb] = mfma16(xf[blk].hi[c], bih[cb][c], ci[cb], hfrag{});
          cr2[cb] = mfma16(xf[blk].hi[c], brl[cb][c], cr2[cb], hfrag{});
          ci2[cb] = mfma16(xf[blk].hi[c], bil[cb][c], ci2[cb], hfrag{});
          cr2[cb] = mfma16(xf[blk].lo[c], brh[cb][c], cr2[cb], hfrag{});
          ci2[cb] = mfma16(xf[blk].lo[c], bih[cb][c], ci2[cb], hfrag{});
        }
    }
    // accumulator r of a lane is block row 4 q + r, column li
    wave_lds_fence();
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        stage[(4 * q + r) * PITCH + 16 * cb + li] =
            QxCplx{(cr[cb][r] + cr2[cb][r]) * fscale, (ci[cb][r] + ci2[cb][r]) * fscale};
    wave_lds_fence();
    const int64_t cb0 = cw + bit_sum<7>(blk << 4, crs);
    const int64_t rows = L - r0;  // valid rows of this block (may exceed 16)
    if (KIND != 0 && chunked && rows >= 16) {
      // Block bits 0..2 have output strides 1, 2, 4, so the block is NE / 8 chunks of 8 elements.
      // Four consecutive lanes write the four 16-byte planes of one chunk (plane q = hi / lo of the
      // real / imaginary parts), so a store instruction covers 16 whole chunks, contiguous where the
      // chunks are; a lane reads its component of the chunk's 8 values and forms its plane.  S is a
      // power of two, so a chunk is wholly inside the output (its first s below S) or wholly outside.
      uint16_t* __restrict__ C16 = static_cast<uint16_t*>(p.c);
      const float* stage_f = reinterpret_cast<const float*>(stage);
      const int q = lane & 3, comp = q >> 1;
      const bool low = (q & 1) != 0;
#pragma unroll
      for (int r = 0; r < NE / 8 / 16; ++r) {
        // chunk (lane >> 2) + 16 r: block bits 3..6 from the lane, 7 and 8 from the round
        const int ci = qi_lane + (int)bit_sum<2>(r, ei + 7), cs = qs_lane + (int)bit_sum<2>(r, es + 7);
        const int64_t co_ = qo_lane + bit_sum<2>(r, est + 7);
        if (cs < S) {
          uint32_t pw[4];
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            float x[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int v = 2 * d + h;
              const int i = ci + (int)bit_sum<3>(v, ei), sv = cs + (int)bit_sum<3>(v, es);
              x[h] = stage_f[2 * (i * PITCH + sv) + comp];
            }
            // the same component of elements 2d and 2d + 1 as a pair: split_value gives their hi
            // plane word and their lo plane word
            uint32_t hw, lw;
            split_value(c_kind, 1.f, QxCplx{x[0], x[1]}, hw, lw);
            pw[d] = low ? lw : hw;
          }
          *reinterpret_cast<v4u*>(C16 + split_chunk(cb0 + co_) + 8 * q) = v4u{pw[0], pw[1], pw[2], pw[3]};
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < NE / 64; ++t) {
        const int i = ep_li + (int)bit_sum<3>(t, ei + 6);
        const int s = ep_ls + (int)bit_sum<3>(t, es + 6);
        const int64_t off = ep_lo + bit_sum<3>(t, est + 6);
        if (i < rows && s < S) {
          const QxCplx v = stage[i * PITCH + s];
          if (KIND != 0 && c_kind) store_split(static_cast<uint16_t*>(p.c), cb0 + off, v, c_kind, 1.f);
          else static_cast<QxCplx*>(p.c)[cb0 + off] = v;
        }
      }
    }
  }
}

bool gemm_thin_fits(const GemmArgs& a) {
  const bool a_small = a.M <= a.N;
  const int64_t S = a_small ? a.M : a.N, L = a_small ? a.N : a.M;
  return S <= THIN_MAX_S && a.K >= 1 && a.K <= THIN_MAX_K && a.a_split == a.b_split && (a.a_split || !a.c_split) &&
         L < (1LL << 32);
}

// Thin form of a matrix product: X is the long operand, W the short one, C[x row][w row].
static void thin_args(const GemmArgs& g, ThinArgs& t) {
  std::memset(&t, 0, sizeof(t));
  const bool a_small = g.M <= g.N;  // then X = B (rows n) and W = A (rows m)
  t.x = a_small ? (const void*)g.b : (const void*)g.a;
  t.w = a_small ? (const void*)g.a : (const void*)g.b;
  t.c = g.c;
  t.L = a_small ? g.N : g.M;
  t.S = (int32_t)(a_small ? g.M : g.N);
  t.K = (int32_t)g.K;
  t.kind = g.a_split;
  t.c_kind = g.c_split;
  t.x_scale = a_small ? g.b_scale : g.a_scale;
  t.w_scale = a_small ? g.a_scale : g.b_scale;
  t.c_scale = g.c_scale;
  t.kc = a_small ? gemm_b_kc(g) : gemm_a_kc(g);
  t.w_kc = a_small ? gemm_a_kc(g) : gemm_b_kc(g);
  int nr = 0;
  while (nr < QX_GEMM_BITS && (1LL << nr) < t.L) ++nr;
  t.nr = nr;
  if (g.bits) {
    const int xn = a_small ? g.nn : g.nm, wn = a_small ? g.nm : g.nn;
    for (int b = 0; b < xn; ++b) {
      t.x_rst[b] = a_small ? g.b_rs[b] : g.a_rs[b];
      t.c_rst[b] = a_small ? g.c_nst[b] : g.c_mst[b];
    }
    for (int b = 0; b < wn && b < 5; ++b) {
      t.w_sst[b] = a_small ? g.a_rs[b] : g.b_rs[b];
      t.c_sst[b] = a_small ? g.c_mst[b] : g.c_nst[b];
    }
    for (int b = 0; b < g.nk && b < 5; ++b) {
      t.x_kst[b] = a_small ? g.b_kst[b] : g.a_kst[b];
      t.w_kst[b] = a_small ? g.a_kst[b] : g.b_kst[b];
    }
  } else {
    // A[m][k] at m a_ms + k a_ks, B[k][n] at k b_ks + n b_ns, C[m][n] at m c_ms + n
    const int64_t x_rs = a_small ? g.b_ns : g.a_ms, x_ks = a_small ? g.b_ks : g.a_ks;
    const int64_t w_ss = a_small ? g.a_ms : g.b_ns, w_ks = a_small ? g.a_ks : g.b_ks;
    const int64_t c_rs = a_small ? 1 : g.c_ms, c_ss = a_small ? g.c_ms : 1;
    for (int b = 0; b < nr; ++b) {
      t.x_rst[b] = x_rs << b;
      t.c_rst[b] = c_rs << b;
    }
    for (int b = 0; b < 5; ++b) {
      t.x_kst[b] = x_ks << b;
      t.w_kst[b] = w_ks << b;
      t.w_sst[b] = w_ss << b;
      t.c_sst[b] = c_ss << b;
    }
  }
  if (g.bits && nr > 4) {
    // Rows are independent, so their bits may be numbered in any order.  A block's rows (bits 0..3)
    // are the four with the lowest output strides (contiguous output runs, and split chunks inside
    // a block); a wave's blocks (bits 4..6) differ in the row bits with the lowest strides in X
    // (longer contiguous runs of X per wave); a work-group's waves (bits 7, 8) in the next output
    // bits; the rest follow by output stride.
    std::vector<int> by_c(nr), by_x(nr), order;
    for (int b = 0; b < nr; ++b) by_c[b] = by_x[b] = b;
    std::stable_sort(by_c.begin(), by_c.end(), [&](int u, int v) { return t.c_rst[u] < t.c_rst[v]; });
    std::stable_sort(by_x.begin(), by_x.end(), [&](int u, int v) { return t.x_rst[u] < t.x_rst[v]; });
    std::vector<bool> used(nr, false);
    auto take = [&](const std::vector<int>& from, int n) {
      for (int b : from)
        if (n > 0 && !used[b]) {
          used[b] = true;
          order.push_back(b);
          --n;
        }
    };
    take(by_c, 4);
    take(by_x, 3);
    take(by_c, nr);
    int64_t xr[QX_GEMM_BITS], cr[QX_GEMM_BITS];
    for (int b = 0; b < nr; ++b) {
      xr[b] = t.x_rst[order[b]];
      cr[b] = t.c_rst[order[b]];
    }
    std::memcpy(t.x_rst, xr, sizeof(int64_t) * nr);
    std::memcpy(t.c_rst, cr, sizeof(int64_t) * nr);
  }
  t.x_item = a_small ? g.b_item : g.a_item;
  t.w_item = a_small ? g.a_item : g.b_item;
  t.c_item = g.c_item;
  t.x_gather = a_small ? g.b_gather : g.a_gather;
  t.w_gather = a_small ? g.a_gather : g.b_gather;
  t.n_items = g.n_items;
  t.nh = g.nh;
  for (int i = 0; i < g.nh; ++i) {
    t.x_hs[i] = a_small ? g.b_hs[i] : g.a_hs[i];
    t.w_hs[i] = a_small ? g.a_hs[i] : g.b_hs[i];
    t.c_hs[i] = g.c_hs[i];
  }
  // output block bits: row bits 0..3, then column bits 0..log2(SP) - 1, ordered by output stride
  const int sp_bits = t.S <= 16 ? 4 : 5;
  struct Bit {
    bool exists;
    int64_t st;
    int di, ds;
  } bits[THIN_EP];
  int n = 0;
  for (int b = 0; b < 4; ++b) bits[n++] = {b < nr, t.c_rst[b], 1 << b, 0};
  int ns = 0;
  while ((1 << ns) < t.S) ++ns;
  for (int b = 0; b < sp_bits; ++b) bits[n++] = {b < ns, t.c_sst[b], 0, 1 << b};
  std::stable_sort(bits, bits + n, [](const Bit& x, const Bit& y) {
    if (x.exists != y.exists) return x.exists;
    return x.exists && x.st < y.st;
  });
  for (int b = 0; b < n; ++b) {
    t.ep_st[b] = bits[b].exists ? bits[b].st : 0;
    t.ep_i[b] = bits[b].di;
    t.ep_s[b] = bits[b].ds;
  }
  t.ep_chunk = t.c_kind != 0 && (t.S & (t.S - 1)) == 0 && bits[0].exists && bits[1].exists && bits[2].exists && bits[0].st == 1 &&
               bits[1].st == 2 && bits[2].st == 4;
}

template <int KIND, int KP, int SP>
static void launch_thin(const ThinArgs& t, unsigned nwg, hipStream_t s) {
  // 16-byte fragment loads need at least 2 complex k per lane (KP >= 8)
  if constexpr (KP >= 8) {
    if (t.kc) {
      hipLaunchKernelGGL((k_gemm_thin<KIND, KP, SP, true>), dim3(nwg), dim3(256), 0, s, t);
      return;
    }
  }
  hipLaunchKernelGGL((k_gemm_thin<KIND, KP, SP, false>), dim3(nwg), dim3(256), 0, s, t);
}

template <int KIND>
static void launch_thin_kind(const ThinArgs& t, unsigned nwg, hipStream_t s) {
  // complex64 with K <= 4 or <= 8: a lane loads 1 or 2 complex k of a row (4 lanes cover the sum)
  // instead of 4 slots of which the ones past K repeat the row's values
  if constexpr (KIND == 0) {
    if (t.K <= 4) {
      if (t.S <= 16) launch_thin<KIND, 4, 16>(t, nwg, s);
      else launch_thin<KIND, 4, 32>(t, nwg, s);
      return;
    }
    if (t.K <= 8) {
      if (t.S <= 16) launch_thin<KIND, 8, 16>(t, nwg, s);
      else launch_thin<KIND, 8, 32>(t, nwg, s);
      return;
    }
  }
  if (t.K <= 16) {
    if (t.S <= 16) launch_thin<KIND, 16, 16>(t, nwg, s);
    else launch_thin<KIND, 16, 32>(t, nwg, s);
  } else {
    if (t.S <= 16) launch_thin<KIND, 32, 16>(t, nwg, s);
    else launch_thin<KIND, 32, 32>(t, nwg, s);
  }
}

hipError_t launch_gemm_thin(const GemmArgs& a, hipStream_t s) {
  if (!gemm_thin_fits(a)) return hipErrorInvalidValue;
  ThinArgs t;
  thin_args(a, t);
  const int64_t rows = 16LL * (t.K <= 16 ? thin_nb<16>() : thin_nb<32>());  // rows per wave
  const int64_t waves = (t.L + rows - 1) / rows * ((int64_t)a.n_items << a.nh);
  const int64_t nwg = (waves + 3) / 4;
  if (nwg <= 0) return hipSuccess;
  if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
  switch (t.kind) {
    case 0: launch_thin_kind<0>(t, (unsigned)nwg, s); break;
    case 1: launch_thin_kind<1>(t, (unsigned)nwg, s); break;
    case 2: launch_thin_kind<2>(t, (unsigned)nwg, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qx
