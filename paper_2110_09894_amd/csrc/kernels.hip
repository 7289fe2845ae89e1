// HIP kernels for gfx950 (CDNA4): the tensor primitives of a sliced network
// contraction (Sec. III-B: slicing, permuting, contracting, recombination).
//
//   k_simt      small / memory-bound pairwise contraction, any bit layout
//   k_dot_outer long inner products whose outputs form an outer product per shared
//               index value (the root of a slice block's tree): every operand row read once
//   k_dot       other long inner products; k_dot_wave for K <= 16384
//   k_permute   LDS-tiled index permutation of dim-2 tensors
//   k_slice_sum FP64 sum of per-slice values (Eq. 2), fixed order, a wave per value
//   k_gather    per-bitstring offsets for the output closure (Sec. II)
//   k_absmax, k_scale_from_max   FP16 operand scales from calibration maxima
// The matrix-core products (Sec. IV-A: contractions mapped to matrix
// multiplications) are in gemm_f32.hip (complex64) and gemm_bf16.hip (split BF16 / FP16).
#include <hip/hip_runtime.h>

#include <utility>
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
// Small contraction: one thread per output element, contracted bits looped.
// The low (up to 8) contracted bits' offsets are tabulated in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_simt(SimtArgs p) {
  __shared__ int64_t ka[256], kb[256];
  __shared__ __attribute__((aligned(16))) uint16_t sp[256 * 4];  // split output of the block's 256 elements
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
  // the block covers outputs [o0, o0 + blockDim): o0's bits (uniform) and the thread's bits are disjoint
  const int tid = threadIdx.x;
  const int64_t o0 = (int64_t)blockIdx.x * blockDim.x, o = o0 + tid;
  const int64_t n = (int64_t)1 << p.n_out;
  const int item = blockIdx.y;
  // split output of full 256-element blocks goes through LDS and out as 16-byte stores
  const bool chunked = p.c_split && blockDim.x == 256 && n >= 256;
  if (o >= n) return;  // never taken by a chunked block
  int64_t ao = (int64_t)item * p.a_item + (p.a_gather ? p.a_gather[item] : 0);
  int64_t bo = (int64_t)item * p.b_item + (p.b_gather ? p.b_gather[item] : 0);
  if (p.block) {
    const int64_t sb = p.block[0];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i < p.nfix_a && ((sb >> p.fix_ja[i]) & 1)) ao += p.fix_sa[i];
      if (i < p.nfix_b && ((sb >> p.fix_jb[i]) & 1)) bo += p.fix_sb[i];
    }
  }
#pragma unroll
  for (int i = 0; i < QX_MAX_BITS; ++i)
    if (i < p.n_out && ((o0 >> i) & 1)) { ao += p.a_os[i]; bo += p.b_os[i]; }
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (i < p.n_out && ((tid >> i) & 1)) { ao += p.a_os[i]; bo += p.b_os[i]; }
  QxCplx acc = {0.f, 0.f};
  if (p.n_k <= 3) {
    // up to 8 terms: uniform offsets, every load issued before the first product
    QxCplx xa[8], xb[8];
#pragma unroll
    for (int kl = 0; kl < 8; ++kl) {
      if (kl < nlo) {
        const int64_t oa = ((kl & 1) ? p.a_ks[0] : 0) + ((kl & 2) ? p.a_ks[1] : 0) + ((kl & 4) ? p.a_ks[2] : 0);
        const int64_t ob = ((kl & 1) ? p.b_ks[0] : 0) + ((kl & 2) ? p.b_ks[1] : 0) + ((kl & 4) ? p.b_ks[2] : 0);
        xa[kl] = p.a[ao + oa];
        xb[kl] = p.b[bo + ob];
      }
    }
#pragma unroll
    for (int kl = 0; kl < 8; ++kl)
      if (kl < nlo) acc = cmul_acc(acc, xa[kl], xb[kl]);
  } else {
    const int nkhi = p.n_k - nklo;
    for (int64_t kh = 0; kh < ((int64_t)1 << nkhi); ++kh) {
      int64_t ah = ao, bh = bo;
#pragma unroll
      for (int j = 0; j < QX_MAX_KBITS - 8; ++j)
        if (j < nkhi && ((kh >> j) & 1)) { ah += p.a_ks[8 + j]; bh += p.b_ks[8 + j]; }
      for (int kl = 0; kl < nlo; ++kl) acc = cmul_acc(acc, p.a[ah + ka[kl]], p.b[bh + kb[kl]]);
    }
  }
  const int64_t e = (int64_t)item * p.c_item + o;
  if (chunked) {
    uint32_t hi, lo;
    split_value(p.c_split, out_scale(p.c_scale), acc, hi, lo);
    sp[split_off(tid, 0)] = (uint16_t)hi;
    sp[split_off(tid, 1)] = (uint16_t)lo;
    sp[split_off(tid, 2)] = (uint16_t)(hi >> 16);
    sp[split_off(tid, 3)] = (uint16_t)(lo >> 16);
    __syncthreads();
    // the block's elements e - tid .. e - tid + 255 (a multiple of 8 onwards) are 2 KB of split storage
    if (tid < 128)
      *(v4u*)(reinterpret_cast<uint16_t*>(p.c) + split_chunk(e - tid) + 8 * tid) = *(const v4u*)(sp + 8 * tid);
  } else if (p.c_split) {
    store_split(reinterpret_cast<uint16_t*>(p.c), e, acc, p.c_split, out_scale(p.c_scale));
  } else {
    p.c[e] = acc;
  }
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
    if (p.c_split)
      store_split(reinterpret_cast<uint16_t*>(p.c), (int64_t)item * p.c_item + o, r, p.c_split, out_scale(p.c_scale));
    else p.c[(int64_t)item * p.c_item + o] = r;
  }
}

// Shorter inner products (K <= 16384): a group of L lanes per output (L = 16,
// 32 or 64 for K >= 256, 512, 1024, so a lane sums at least 16 terms), 256 / L
// outputs per work-group, reduced with cross-lane shuffles inside the group
// only (no LDS, no barrier).  A lane keeps four partial sums of at most
// K / (4 L) terms each.
template <int L>
__global__ __launch_bounds__(256) void k_dot_wave(DotArgs p) {
  const int sub = threadIdx.x & (L - 1);
  const int64_t o = (int64_t)blockIdx.x * (256 / L) + (threadIdx.x / L);
  if (o >= ((int64_t)1 << p.n_out)) return;  // whole lane groups only; shuffles stay inside a group
  const int item = blockIdx.y;
  int64_t ao = (int64_t)item * p.a_item + (p.a_gather ? p.a_gather[item] : 0);
  int64_t bo = (int64_t)item * p.b_item + (p.b_gather ? p.b_gather[item] : 0);
#pragma unroll
  for (int i = 0; i < QX_MAX_BITS; ++i)
    if (i < p.n_out && ((o >> i) & 1)) { ao += p.a_os[i]; bo += p.b_os[i]; }
  const QxCplx* __restrict__ A = p.a + ao;
  const QxCplx* __restrict__ B = p.b + bo;
  QxCplx acc0 = {0.f, 0.f}, acc1 = {0.f, 0.f}, acc2 = {0.f, 0.f}, acc3 = {0.f, 0.f};
  const bool vec = ((((uintptr_t)A) | ((uintptr_t)B)) & 15) == 0 && (p.K & 3) == 0;
  if (vec) {
    for (int64_t k = 4 * (int64_t)sub; k < p.K; k += 4 * L) {
      const v4f a0 = *(const v4f*)(A + k), a1 = *(const v4f*)(A + k + 2);
      const v4f b0 = *(const v4f*)(B + k), b1 = *(const v4f*)(B + k + 2);
      acc0 = cmul_acc(acc0, QxCplx{a0[0], a0[1]}, QxCplx{b0[0], b0[1]});
      acc1 = cmul_acc(acc1, QxCplx{a0[2], a0[3]}, QxCplx{b0[2], b0[3]});
      acc2 = cmul_acc(acc2, QxCplx{a1[0], a1[1]}, QxCplx{b1[0], b1[1]});
      acc3 = cmul_acc(acc3, QxCplx{a1[2], a1[3]}, QxCplx{b1[2], b1[3]});
    }
  } else {
    for (int64_t k = sub; k < p.K; k += L) acc0 = cmul_acc(acc0, A[k], B[k]);
  }
  QxCplx acc = {(acc0.x + acc1.x) + (acc2.x + acc3.x), (acc0.y + acc1.y) + (acc2.y + acc3.y)};
#pragma unroll
  for (int off = L / 2; off >= 1; off >>= 1) {
    acc.x += __shfl_xor(acc.x, off, 64);
    acc.y += __shfl_xor(acc.y, off, 64);
  }
  if (sub == 0) {
    if (p.c_split)
      store_split(reinterpret_cast<uint16_t*>(p.c), (int64_t)item * p.c_item + o, acc, p.c_split,
                  out_scale(p.c_scale));
    else p.c[(int64_t)item * p.c_item + o] = acc;
  }
}

// Long inner products whose outputs form an NA x NB outer product per value of
// the shared bits h (A only bits Fa, B only bits Fb, 2 <= NA, NB <= 8): a
// work-group owns one (item, h) and a range of k, reads each of the NA rows of
// A and NB rows of B once (16-byte loads along k) and keeps all NA * NB partial
// sums per lane, instead of one work-group per output re-reading a row NB (NA)
// times.  Lanes are reduced by a reduce-scatter butterfly (after step s a lane
// keeps half of its remaining sums: the one it holds at the end is lane >> (6 -
// log2(NA NB))), then the 4 waves through LDS, in a fixed order.  With the k
// range split over ks work-groups the partial results go to p.part and
// k_dot_outer_finish adds them in split order.
template <int NA, int NB>
__global__ __launch_bounds__(256) void k_dot_outer(DotArgs p, int nfa, int nfb, int kslog) {
  constexpr int NACC = NA * NB;
  constexpr int LOG = NACC >= 64 ? 6 : (NACC >= 32 ? 5 : (NACC >= 16 ? 4 : (NACC >= 8 ? 3 : 2)));
  __shared__ float red[2][4][NACC];
  const int nh = p.n_out - nfa - nfb;
  const int64_t gid = blockIdx.x;
  const int64_t split = gid & ((1LL << kslog) - 1), wg = gid >> kslog;
  const int64_t h = wg & ((1LL << nh) - 1);
  const int item = (int)(wg >> nh);
  int64_t ao = (int64_t)item * p.a_item + (p.a_gather ? p.a_gather[item] : 0);
  int64_t bo = (int64_t)item * p.b_item + (p.b_gather ? p.b_gather[item] : 0);
#pragma unroll
  for (int i = 0; i < QX_MAX_BITS; ++i)
    if (i < nh && ((h >> i) & 1)) { ao += p.a_os[nfa + nfb + i]; bo += p.b_os[nfa + nfb + i]; }
  int64_t ar[NA], br[NB];
#pragma unroll
  for (int r = 0; r < NA; ++r) {
    ar[r] = ao;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (j < nfa && ((r >> j) & 1)) ar[r] += p.a_os[nfb + j];
  }
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    br[r] = bo;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (j < nfb && ((r >> j) & 1)) br[r] += p.b_os[j];
  }
  float vr[NACC], vi[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) vr[i] = vi[i] = 0.f;
  const int64_t kc = p.K >> kslog, k0 = split * kc, k1 = k0 + kc;
  const int tid = threadIdx.x;
  // rows start at multiples of K (>= 1024) past 16-byte aligned bases
  const bool vec = ((((uintptr_t)(p.a + ao)) | ((uintptr_t)(p.b + bo))) & 15) == 0 && (p.K & 3) == 0;
  if (vec) {
    for (int64_t k = k0 + 2 * tid; k < k1; k += 512) {
      v4f xa[NA], xb[NB];
#pragma unroll
      for (int r = 0; r < NA; ++r) xa[r] = *(const v4f*)(p.a + ar[r] + k);
#pragma unroll
      for (int r = 0; r < NB; ++r) xb[r] = *(const v4f*)(p.b + br[r] + k);
#pragma unroll
      for (int ra = 0; ra < NA; ++ra)
#pragma unroll
        for (int rb = 0; rb < NB; ++rb) {
          const int i = ra * NB + rb;
          float re = vr[i], im = vi[i];
          re = fmaf(xa[ra][0], xb[rb][0], re);
          re = fmaf(-xa[ra][1], xb[rb][1], re);
          im = fmaf(xa[ra][0], xb[rb][1], im);
          im = fmaf(xa[ra][1], xb[rb][0], im);
          re = fmaf(xa[ra][2], xb[rb][2], re);
          re = fmaf(-xa[ra][3], xb[rb][3], re);
          im = fmaf(xa[ra][2], xb[rb][3], im);
          im = fmaf(xa[ra][3], xb[rb][2], im);
          vr[i] = re;
          vi[i] = im;
        }
    }
  } else {
    for (int64_t k = k0 + tid; k < k1; k += 256) {
      QxCplx xa[NA], xb[NB];
#pragma unroll
      for (int r = 0; r < NA; ++r) xa[r] = p.a[ar[r] + k];
#pragma unroll
      for (int r = 0; r < NB; ++r) xb[r] = p.b[br[r] + k];
#pragma unroll
      for (int ra = 0; ra < NA; ++ra)
#pragma unroll
        for (int rb = 0; rb < NB; ++rb) {
          const QxCplx c = cmul_acc(QxCplx{vr[ra * NB + rb], vi[ra * NB + rb]}, xa[ra], xb[rb]);
          vr[ra * NB + rb] = c.x;
          vi[ra * NB + rb] = c.y;
        }
    }
  }
  // reduce-scatter over the wave: at offset d a lane keeps the upper half of its sums if bit d is set
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int st = 0; st < LOG; ++st) {
    const int d = 32 >> st, half = NACC >> (st + 1);
    const bool up = (lane & d) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const float sr = up ? vr[i] : vr[i + half], si = up ? vi[i] : vi[i + half];
      const float kr = up ? vr[i + half] : vr[i], ki = up ? vi[i + half] : vi[i];
      vr[i] = kr + __shfl_xor(sr, d, 64);
      vi[i] = ki + __shfl_xor(si, d, 64);
    }
  }
#pragma unroll
  for (int d = 32 >> LOG; d >= 1; d >>= 1) {
    vr[0] += __shfl_xor(vr[0], d, 64);
    vi[0] += __shfl_xor(vi[0], d, 64);
  }
  if ((lane & ((64 >> LOG) - 1)) == 0) {
    red[0][wave][lane >> (6 - LOG)] = vr[0];
    red[1][wave][lane >> (6 - LOG)] = vi[0];
  }
  __syncthreads();
  if (tid < NACC) {
    const QxCplx r = {(red[0][0][tid] + red[0][1][tid]) + (red[0][2][tid] + red[0][3][tid]),
                      (red[1][0][tid] + red[1][1][tid]) + (red[1][2][tid] + red[1][3][tid])};
    if (kslog > 0) {
      p.part[gid * NACC + tid] = r;
    } else {
      const int64_t e = (int64_t)item * p.c_item + h * NACC + tid;
      if (p.c_split) store_split(reinterpret_cast<uint16_t*>(p.c), e, r, p.c_split, out_scale(p.c_scale));
      else p.c[e] = r;
    }
  }
}

// Sums of k_dot_outer's split partial results, in split order: one thread per output.
__global__ __launch_bounds__(256) void k_dot_outer_finish(DotArgs p, int nacc, int nh, int kslog) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = ((int64_t)p.n_items << nh) * nacc;
  if (g >= n) return;
  const int64_t wg = g / nacc, t = g - wg * nacc;
  QxCplx r = {0.f, 0.f};
  for (int64_t sp = 0; sp < (1LL << kslog); ++sp) {
    const QxCplx v = p.part[((wg << kslog) + sp) * nacc + t];
    r.x += v.x;
    r.y += v.y;
  }
  const int64_t h = wg & ((1LL << nh) - 1);
  const int item = (int)(wg >> nh);
  const int64_t e = (int64_t)item * p.c_item + h * nacc + t;
  if (p.c_split) store_split(reinterpret_cast<uint16_t*>(p.c), e, r, p.c_split, out_scale(p.c_scale));
  else p.c[e] = r;
}

// Complex64 matrices -> split BF16 form [item][row][kp], k >= K zero-filled.
__global__ __launch_bounds__(256) void k_split_planes(SplitPlanesArgs p) {
  const int64_t per = p.rows * p.kp;
  const int64_t n = per * p.n_items;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t item = e / per, rk = e - item * per;
    const int64_t r = rk / p.kp, k = rk - r * p.kp;
    const QxCplx v = k < p.K ? p.in[item * p.in_item + r * p.ld_r + k * p.ld_k] : QxCplx{0.f, 0.f};
    store_split(p.out, e, v, p.kind);
  }
}

// In-place conversion of a complex64 tensor to split FP16 form (x * scale): a thread reads one
// 64-byte chunk of 8 elements and writes back their four planes in the same 64 bytes.  (Leaves
// start at any 8-byte boundary, so the accesses are 8 bytes wide.)
__global__ __launch_bounds__(256) void k_split_inplace(SplitInplaceArgs p) {
  const float sc = out_scale(p.scale);
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < p.n / 8; c += (int64_t)gridDim.x * blockDim.x) {
    QxCplx* x = p.x + 8 * c;
    QxCplx v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = x[j];
    uint32_t w[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t hi0, lo0, hi1, lo1, q[4];
      split_value(2, sc, v[2 * j], hi0, lo0);
      split_value(2, sc, v[2 * j + 1], hi1, lo1);
      split_words(hi0, lo0, hi1, lo1, q);
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) w[pl][j] = q[pl];
    }
    uint2* o = reinterpret_cast<uint2*>(x);
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
      o[2 * pl] = uint2{w[pl][0], w[pl][1]};
      o[2 * pl + 1] = uint2{w[pl][2], w[pl][3]};
    }
  }
}

// ---------------------------------------------------------------------------
// Index permutation.  A tile is the set of elements that differ only in the
// output's lowest bits and the bits at the input's lowest positions, so a tile
// is read in runs contiguous in the input and written in runs contiguous in
// the output, transposing through LDS.  The outer bits select the tile.  Each
// work-group builds its offset tables once and then walks many tiles.
// ---------------------------------------------------------------------------
constexpr int PERM_TB = QX_PERM_TB;
constexpr int PERM_TSZ = 1 << (2 * PERM_TB);     // largest tile (elements)
constexpr int PERM_PAIRS = PERM_TSZ / 2 / 256;   // element pairs per thread per tile
constexpr int PERM_HALF = 1 << PERM_TB;          // entries of each half-table
__global__ __launch_bounds__(256) void k_permute(PermArgs p) {
  __shared__ QxCplx buf[PERM_TSZ];
  // offsets split into the low and high PERM_TB bits of the load order v / LDS slot u:
  // in(v) = tin[0][v & 63] + tin[1][v >> 6], slot(v) = tlu[0][..] | tlu[1][..], out(u) likewise
  __shared__ long long tin[2][PERM_HALF], tout[2][PERM_HALF];
  __shared__ int tlu[2][PERM_HALF];
  const int nt = p.nt;
  const int tsz = 1 << nt;
  for (int x = threadIdx.x; x < 2 * PERM_HALF; x += blockDim.x) {
    const int h = x / PERM_HALF, e = x % PERM_HALF;
    long long inoff = 0, outoff = 0;
    int u = 0;
    for (int c = 0; c < PERM_TB; ++c) {
      const int b = h * PERM_TB + c;
      if (b < nt && ((e >> c) & 1)) {
        inoff += 1LL << p.in_pos[p.tl[p.ll[b]]];
        u |= 1 << p.ll[b];
        outoff += 1LL << p.tl[b];
      }
    }
    tin[h][e] = inoff;
    tlu[h][e] = u;
    tout[h][e] = outoff;
  }
  auto in_off = [&](int v) { return tin[0][v & (PERM_HALF - 1)] + tin[1][v >> PERM_TB]; };
  auto slot = [&](int v) { return tlu[0][v & (PERM_HALF - 1)] | tlu[1][v >> PERM_TB]; };
  auto out_off = [&](int u) { return tout[0][u & (PERM_HALF - 1)] + tout[1][u >> PERM_TB]; };
  const int64_t n_tiles = (int64_t)1 << p.n_outer;
  const int64_t total = n_tiles * p.n_items;
  auto bases = [&](int64_t t, int64_t& ib, int64_t& ob) {
    const int64_t item = t >> p.n_outer;
    int64_t w = t & (n_tiles - 1);
    ib = item * p.in_item;
    ob = item * p.out_item;
    for (int i = 0; w; ++i, w >>= 1)
      if (w & 1) { ib += p.outer_in[i]; ob += p.outer_out[i]; }
  };
  if (!p.vec) {
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
      int64_t ibase, obase;
      bases(t, ibase, obase);
      __syncthreads();  // tables ready / previous tile's LDS reads done
      const QxCplx* __restrict__ in = p.in + ibase;
      for (int v = threadIdx.x; v < tsz; v += blockDim.x) buf[slot(v)] = in[in_off(v)];
      __syncthreads();
      QxCplx* __restrict__ out = p.out + obase;
      for (int u = threadIdx.x; u < tsz; u += blockDim.x) out[out_off(u)] = buf[u];
    }
    return;
  }
  // Pairs: load-order bit 0 is input bit 0 and LDS slot bit 0 is output bit 0, so elements 2i and
  // 2i + 1 are adjacent in the input (load order) and in the output (slot order): 16-byte accesses.
  // The next tile's loads are issued before the current tile is written out.
  const int npair = tsz >> 1;
  __syncthreads();  // tables ready
  int64_t t = blockIdx.x;
  if (t >= total) return;  // uniform over the work-group
  int64_t ibase, obase;
  bases(t, ibase, obase);
  v4f cur[PERM_PAIRS];
#pragma unroll
  for (int r = 0; r < PERM_PAIRS; ++r) {
    const int i = threadIdx.x + 256 * r;
    if (i < npair) cur[r] = *(const v4f*)(p.in + ibase + in_off(2 * i));
  }
  for (; t < total; t += gridDim.x) {
#pragma unroll
    for (int r = 0; r < PERM_PAIRS; ++r) {
      const int i = threadIdx.x + 256 * r;
      if (i < npair) {
        buf[slot(2 * i)] = QxCplx{cur[r][0], cur[r][1]};
        buf[slot(2 * i + 1)] = QxCplx{cur[r][2], cur[r][3]};
      }
    }
    __syncthreads();
    const int64_t tn = t + gridDim.x;
    int64_t ib2 = 0, ob2 = obase;
    if (tn < total) {
      bases(tn, ib2, ob2);
#pragma unroll
      for (int r = 0; r < PERM_PAIRS; ++r) {
        const int i = threadIdx.x + 256 * r;
        if (i < npair) cur[r] = *(const v4f*)(p.in + ib2 + in_off(2 * i));
      }
    }
#pragma unroll
    for (int r = 0; r < PERM_PAIRS; ++r) {
      const int i = threadIdx.x + 256 * r;
      if (i < npair) {
        const QxCplx a = buf[2 * i], b = buf[2 * i + 1];
        *(v4f*)(p.out + obase + out_off(2 * i)) = v4f{a.x, a.y, b.x, b.y};
      }
    }
    __syncthreads();  // LDS reads done before the next tile is written
    obase = ob2;
  }
}

// ---------------------------------------------------------------------------
// FP64 sum over the slices of one block in a fixed order (deterministic): one
// wavefront per value (bitstring v >> n_obits, open-qubit assignment j = the low
// n_obits bits of v); lane l sums slices lo + l, lo + l + 64, ... in ascending
// order, then the 64 partial sums meet in a fixed butterfly.  A block of 2^js
// slices thus takes about 2^js / 64 dependent steps per lane, whatever js is.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_slice_sum(SliceSumArgs p) {
  const int lane = threadIdx.x & 63;
  const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= p.n_items) return;
  const int item = v >> p.n_obits;
  int64_t base = (int64_t)item * p.root_item + (p.root_gather ? p.root_gather[item] : 0);
#pragma unroll
  for (int i = 0; i < QX_MAX_OBITS; ++i)
    if (i < p.n_obits && ((v >> i) & 1)) base += p.o_stride[i];
  const int lo = p.block ? (int)p.block[1] : p.s_lo, hi = p.block ? (int)p.block[2] : p.s_hi;
  double sr = 0.0, si = 0.0;
  for (int s = lo + lane; s < hi; s += 64) {
    int64_t off = base;
#pragma unroll
    for (int j = 0; j < QX_MAX_SBITS; ++j)
      if (j < p.n_sbits && ((s >> j) & 1)) off += p.s_stride[j];
    const QxCplx x = p.root[off];
    sr += (double)x.x;
    si += (double)x.y;
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    sr += __shfl_xor(sr, m, 64);
    si += __shfl_xor(si, m, 64);
  }
  if (lane == 0) {
    p.amp[2 * (int64_t)v] += sr;
    p.amp[2 * (int64_t)v + 1] += si;
  }
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
  for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) mm = fmaxf(mm, p.partial[i]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mm = fmaxf(mm, __shfl_xor(mm, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mm;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    p.maxv[0] = fmaxf(p.maxv[0], mx);
    *p.ticket = 0u;
  }
}

__global__ __launch_bounds__(256) void k_scale_from_max(ScaleFromMaxArgs p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const float mx = p.v[i];
  float sc = 1.f;
  if (mx > 0.f && mx < 3.0e38f) {
    int e;
    frexpf(mx, &e);  // mx < 2^e
    int k = p.target_exp - e;
    k = k > 100 ? 100 : (k < -100 ? -100 : k);
    sc = ldexpf(1.f, k);
  }
  p.v[i] = sc;
}

// Start of a contract call: block state and zeroed FP64 accumulator.
__global__ __launch_bounds__(256) void k_block_init(BlockArgs p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    p.state[3] = p.first_block;
    p.state[4] = p.slice_begin;
    p.state[5] = p.slice_end;
    p.state[6] = p.js;
  }
  if (i < p.n_items) {
    p.acc[2 * i] = 0.0;
    p.acc[2 * i + 1] = 0.0;
  }
}

// Head of every block program: take the next block and its local slice range.
__global__ void k_block_advance(BlockArgs p) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t bb = p.state[3];
  const int js = (int)p.state[6];
  const int64_t base = bb << js, bsz = 1LL << js;
  const int64_t s0 = p.state[4], s1 = p.state[5];
  p.state[0] = base;
  p.state[1] = (s0 > base ? s0 : base) - base;
  p.state[2] = (s1 < base + bsz ? s1 : base + bsz) - base;
  p.state[3] = bb + 1;
}

// End of a contract call: caller's amplitudes += accumulated slice sums.
__global__ __launch_bounds__(256) void k_block_finish(BlockArgs p, double* amp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p.n_items) {
    amp[2 * i] += p.acc[2 * i];
    amp[2 * i + 1] += p.acc[2 * i + 1];
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

hipError_t launch_gemm(const GemmArgs& a, int precision, int tile, hipStream_t s) {
  // the split tile kernels take K of 8 or a multiple of 16; shorter sums run on the thin kernel
  if (tile == GEMM_TILE_THIN || (precision != QX_C64 && !gemm_split_k_ok(a))) {
    if (gemm_thin_fits(a)) return launch_gemm_thin(a, s);
    tile = gemm_default_tile(a.M, a.N);
  }
  switch (precision) {
    case QX_SPLIT_BF16: return launch_gemm_bf16(a, tile, s);
    case QX_SPLIT_FP16: return launch_gemm_fp16(a, tile, s);
    default: return launch_gemm_c64(a, tile, s);
  }
}

int gemm_default_tile(int64_t M, int64_t N) {
  if (M >= 128 && N >= 128) return GEMM_TILE_128x128;
  if (M >= 128) return GEMM_TILE_128x64;
  if (N >= 128) return GEMM_TILE_64x128;
  return GEMM_TILE_64x64;
}

// Outer-product form of a dot (k_dot_outer): the lowest nfb output bits are B's only, the next nfa A's
// only, the rest shared; 1 <= nfa, nfb <= 3 and K >= 1024.
bool dot_outer_shape(const DotArgs& a, int& nfa, int& nfb) {
  nfa = nfb = 0;
  int i = 0;
  while (i < a.n_out && a.a_os[i] == 0 && a.b_os[i] != 0) ++i, ++nfb;
  while (i < a.n_out && a.b_os[i] == 0 && a.a_os[i] != 0) ++i, ++nfa;
  for (; i < a.n_out; ++i)
    if (a.a_os[i] == 0 || a.b_os[i] == 0) return false;
  return a.part != nullptr && nfa >= 1 && nfa <= 3 && nfb >= 1 && nfb <= 3 && a.K >= 1024;
}

template <int NA, int NB>
static void launch_outer(const DotArgs& a, int nfa, int nfb, int kslog, int64_t nwg, hipStream_t s) {
  hipLaunchKernelGGL((k_dot_outer<NA, NB>), dim3((unsigned)nwg), dim3(256), 0, s, a, nfa, nfb, kslog);
}

hipError_t launch_dot(const DotArgs& a, hipStream_t s) {
  int nfa, nfb;
  // (a grid beyond 2^31 work-groups keeps the per-output kernels)
  if (dot_outer_shape(a, nfa, nfb) && a.n_out - nfa - nfb < 31 &&
      ((int64_t)a.n_items << (a.n_out - nfa - nfb)) <= 0x7fffffffLL) {
    const int nh = a.n_out - nfa - nfb;
    const int64_t wgs = (int64_t)a.n_items << nh;
    const int nacc = 1 << (nfa + nfb);
    // split the sum while the grid is short of 1024 work-groups (chunks of at least 4096 terms)
    int kslog = 0;
    while ((wgs << kslog) < 1024 && (a.K & (a.K - 1)) == 0 && (a.K >> (kslog + 1)) >= 4096) ++kslog;
    if (kslog > 0 && ((wgs << kslog) > 0x7fffffffLL || (wgs << kslog) * nacc > QX_DOT_PART_ELEMS)) kslog = 0;
    const int64_t nwg = wgs << kslog;
    switch (nfa * 4 + nfb) {
      case 1 * 4 + 1: launch_outer<2, 2>(a, nfa, nfb, kslog, nwg, s); break;
      case 1 * 4 + 2: launch_outer<2, 4>(a, nfa, nfb, kslog, nwg, s); break;
      case 1 * 4 + 3: launch_outer<2, 8>(a, nfa, nfb, kslog, nwg, s); break;
      case 2 * 4 + 1: launch_outer<4, 2>(a, nfa, nfb, kslog, nwg, s); break;
      case 2 * 4 + 2: launch_outer<4, 4>(a, nfa, nfb, kslog, nwg, s); break;
      case 2 * 4 + 3: launch_outer<4, 8>(a, nfa, nfb, kslog, nwg, s); break;
      case 3 * 4 + 1: launch_outer<8, 2>(a, nfa, nfb, kslog, nwg, s); break;
      case 3 * 4 + 2: launch_outer<8, 4>(a, nfa, nfb, kslog, nwg, s); break;
      default: launch_outer<8, 8>(a, nfa, nfb, kslog, nwg, s); break;
    }
    if (kslog > 0) {
      const int64_t n = wgs * nacc;
      hipLaunchKernelGGL(k_dot_outer_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, nacc, nh, kslog);
    }
    return hipGetLastError();
  }
  if (a.K <= 16384) {
    const int64_t n = 1LL << a.n_out;
    if (a.K >= 1024) {
      hipLaunchKernelGGL(k_dot_wave<64>, dim3((unsigned)((n + 3) / 4), (unsigned)a.n_items), dim3(256), 0, s, a);
    } else if (a.K >= 512) {
      hipLaunchKernelGGL(k_dot_wave<32>, dim3((unsigned)((n + 7) / 8), (unsigned)a.n_items), dim3(256), 0, s, a);
    } else {
      hipLaunchKernelGGL(k_dot_wave<16>, dim3((unsigned)((n + 15) / 16), (unsigned)a.n_items), dim3(256), 0, s, a);
    }
  } else {
    dim3 grid((unsigned)(1LL << a.n_out), (unsigned)a.n_items);
    hipLaunchKernelGGL(k_dot, grid, dim3(256), 0, s, a);
  }
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

hipError_t launch_permute(const PermArgs& a_in, hipStream_t s) {
  PermArgs a = a_in;
  const int64_t total = ((int64_t)1 << a.n_outer) * a.n_items;
  const int64_t grid = total < 4096 ? total : 4096;
  if (grid <= 0) return hipSuccess;
  // pair accesses need 16-byte aligned tile bases: aligned pointers and even item strides (outer
  // strides are at least 2^PERM_TB elements); a one-element tile has no pairs
  a.vec = a.nt >= 1 && ((((uintptr_t)a.in) | ((uintptr_t)a.out)) & 15) == 0 && (a.in_item & 1) == 0 &&
          (a.out_item & 1) == 0;
  hipLaunchKernelGGL(k_permute, dim3((unsigned)grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_slice_sum(const SliceSumArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.n_items + 3) / 4));  // a wavefront per value
  hipLaunchKernelGGL(k_slice_sum, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

void gemm_args_setup(GemmArgs& g) {
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
  g.ep_chunk = g.ep_st[0] == 1 && g.ep_st[1] == 2 && g.ep_st[2] == 4;
  // k-tile steps: tile t -> t + 1 sets bit z of t (its lowest zero bit) and clears the bits below
  for (int z = 0; z < QX_GEMM_BITS; ++z) {
    int64_t ia = 0, ib = 0;
    if (!g.bits) {
      ia = 16 * g.a_ks;
      ib = 16 * g.b_ks;
    } else if (4 + z < g.nk) {
      ia = g.a_kst[4 + z];
      ib = g.b_kst[4 + z];
      for (int i = 0; i < z; ++i) {
        ia -= g.a_kst[4 + i];
        ib -= g.b_kst[4 + i];
      }
    }
    g.a_kinc[z] = ia;
    g.b_kinc[z] = ib;
  }
}

hipError_t launch_absmax(const AbsmaxArgs& a, hipStream_t s) {
  const int64_t want = (a.n + 255) / 256;
  const int grid = (int)(want < 1 ? 1 : (want > ABSMAX_GRID ? ABSMAX_GRID : want));
  hipLaunchKernelGGL(k_absmax, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_scale_from_max(const ScaleFromMaxArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_from_max, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_block_init(const BlockArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_block_init, dim3((unsigned)((a.n_items + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_block_advance(const BlockArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_block_advance, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_block_finish(const BlockArgs& a, double* amp, hipStream_t s) {
  hipLaunchKernelGGL(k_block_finish, dim3((unsigned)((a.n_items + 255) / 256)), dim3(256), 0, s, a, amp);
  return hipGetLastError();
}

hipError_t launch_split_planes(const SplitPlanesArgs& a, hipStream_t s) {
  const int64_t n = a.rows * a.kp * a.n_items;
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + 255) / 256;
  hipLaunchKernelGGL(k_split_planes, dim3((unsigned)(want < 8192 ? want : 8192)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_split_inplace(const SplitInplaceArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.n % 8 != 0) return hipErrorInvalidValue;
  const int64_t want = (a.n / 8 + 255) / 256;
  hipLaunchKernelGGL(k_split_inplace, dim3((unsigned)(want < 4096 ? want : 4096)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.n_items + 255) / 256));
  hipLaunchKernelGGL(k_gather, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace qx
