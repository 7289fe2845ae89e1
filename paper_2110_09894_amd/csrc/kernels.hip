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
#include "kargs.h"
#include "kernels.h"

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
  constexpr int CHA = BM * (BK / 8), CHB = BN * (BK / 8);  // 8-element chunks per tile
  constexpr int PA = (CHA + 255) / 256, PB = (CHB + 255) / 256;
  __shared__ __attribute__((aligned(16))) QxCplx As[2][BM * PITCH];
  __shared__ __attribute__((aligned(16))) QxCplx Bs[2][BN * PITCH];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t tiles_m = (p.M + BM - 1) / BM, tiles_n = (p.N + BN - 1) / BN;
  const int64_t tiles = tiles_m * tiles_n;
  const int64_t nwg = (int64_t)gridDim.x;
  // XCD-aware order: hardware deals work-groups round-robin over 8 XCDs; give
  // each XCD a contiguous run of logical tiles so neighbours share its L2.
  int64_t w = blockIdx.x;
  const int64_t per = nwg / 8;
  if (per > 0 && w < per * 8) w = (w % 8) * per + w / 8;
  const int64_t z = w / tiles, t = w % tiles;
  const int64_t tm = t / tiles_n, tn = t % tiles_n;
  const int item = (int)(z >> p.nh);
  const int64_t h = z & ((1LL << p.nh) - 1);
  int64_t aoff = (int64_t)item * p.a_item + (p.a_gather ? p.a_gather[item] : 0);
  int64_t boff = (int64_t)item * p.b_item + (p.b_gather ? p.b_gather[item] : 0);
  int64_t coff = (int64_t)item * p.c_item;
#pragma unroll
  for (int i = 0; i < QX_MAX_HBITS; ++i)
    if (i < p.nh && ((h >> i) & 1)) { aoff += p.a_hs[i]; boff += p.b_hs[i]; coff += p.c_hs[i]; }
  const QxCplx* __restrict__ A = p.a + aoff;
  const QxCplx* __restrict__ B = p.b + boff;
  const int64_t m0 = tm * BM, n0 = tn * BN;

  QxCplx ra[PA][8], rb[PB][8];

  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int ps = 0; ps < PA; ++ps) {
      const int c = tid + ps * 256;
      if (c < CHA) {
        const int r = A_KC ? c / (BK / 8) : c % BM;
        const int kg = A_KC ? c % (BK / 8) : c / BM;
        const int64_t m = m0 + r, kb = k0 + kg * 8;
        if (A_KC) {
          const QxCplx* src = A + m * p.a_ms + kb;
          if (p.vec_a && m < p.M && kb + 8 <= p.K) {
#pragma unroll
            for (int j = 0; j < 8; j += 2) {
              v4f v = *(const v4f*)(src + j);
              ra[ps][j] = {v[0], v[1]};
              ra[ps][j + 1] = {v[2], v[3]};
            }
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
              ra[ps][j] = (m < p.M && kb + j < p.K) ? src[j] : QxCplx{0.f, 0.f};
          }
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            ra[ps][j] = (m < p.M && kb + j < p.K) ? A[(kb + j) * p.a_ks + m] : QxCplx{0.f, 0.f};
        }
      }
    }
#pragma unroll
    for (int ps = 0; ps < PB; ++ps) {
      const int c = tid + ps * 256;
      if (c < CHB) {
        const int r = B_KC ? c / (BK / 8) : c % BN;
        const int kg = B_KC ? c % (BK / 8) : c / BN;
        const int64_t n = n0 + r, kb = k0 + kg * 8;
        if (B_KC) {
          const QxCplx* src = B + n * p.b_ns + kb;
          if (p.vec_b && n < p.N && kb + 8 <= p.K) {
#pragma unroll
            for (int j = 0; j < 8; j += 2) {
              v4f v = *(const v4f*)(src + j);
              rb[ps][j] = {v[0], v[1]};
              rb[ps][j + 1] = {v[2], v[3]};
            }
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
              rb[ps][j] = (n < p.N && kb + j < p.K) ? src[j] : QxCplx{0.f, 0.f};
          }
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            rb[ps][j] = (n < p.N && kb + j < p.K) ? B[(kb + j) * p.b_ks + n] : QxCplx{0.f, 0.f};
        }
      }
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int ps = 0; ps < PA; ++ps) {
      const int c = tid + ps * 256;
      if (c < CHA) {
        const int r = A_KC ? c / (BK / 8) : c % BM;
        const int kg = A_KC ? c % (BK / 8) : c / BM;
        QxCplx* dst = &As[buf][r * PITCH + kg * 8];
#pragma unroll
        for (int j = 0; j < 8; j += 2)
          *(v4f*)(dst + j) = v4f{ra[ps][j].x, ra[ps][j].y, ra[ps][j + 1].x, ra[ps][j + 1].y};
      }
    }
#pragma unroll
    for (int ps = 0; ps < PB; ++ps) {
      const int c = tid + ps * 256;
      if (c < CHB) {
        const int r = B_KC ? c / (BK / 8) : c % BN;
        const int kg = B_KC ? c % (BK / 8) : c / BN;
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

  QxCplx* __restrict__ C = p.c + coff;
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t m = m0 + wm * WM + a * 32 + 8 * (i / 4) + 4 * g + (i % 4);
        const int64_t n = n0 + wn * WN + b * 32 + lrow;
        if (m < p.M && n < p.N) C[m * p.c_ms + n] = QxCplx{cr[a][b][i], ci[a][b][i]};
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
  QxCplx acc = {0.f, 0.f};
  const bool vec = ((((uintptr_t)A) | ((uintptr_t)B)) & 15) == 0 && (p.K & 1) == 0;
  if (vec) {
    for (int64_t k = 2 * (int64_t)threadIdx.x; k < p.K; k += 2 * blockDim.x) {
      v4f va = *(const v4f*)(A + k);
      v4f vb = *(const v4f*)(B + k);
      acc = cmul_acc(acc, QxCplx{va[0], va[1]}, QxCplx{vb[0], vb[1]});
      acc = cmul_acc(acc, QxCplx{va[2], va[3]}, QxCplx{vb[2], vb[3]});
    }
  } else {
    for (int64_t k = threadIdx.x; k < p.K; k += blockDim.x) acc = cmul_acc(acc, A[k], B[k]);
  }
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

template <int BM, int BN>
static hipError_t launch_gemm_tile(const GemmArgs& a, hipStream_t s) {
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  const int64_t nwg = tiles * (int64_t)a.n_items * (1LL << a.nh);
  if (nwg <= 0) return hipSuccess;
  if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool akc = a.a_ks == 1, bkc = a.b_ks == 1;
  dim3 grid((unsigned)nwg), block(256);
  if (akc && bkc) hipLaunchKernelGGL((k_gemm_f32<BM, BN, true, true>), grid, block, 0, s, a);
  else if (akc) hipLaunchKernelGGL((k_gemm_f32<BM, BN, true, false>), grid, block, 0, s, a);
  else if (bkc) hipLaunchKernelGGL((k_gemm_f32<BM, BN, false, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_gemm_f32<BM, BN, false, false>), grid, block, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& a, int precision, int tile, hipStream_t s) {
  (void)precision;
  switch (tile) {
    case GEMM_TILE_64x64: return launch_gemm_tile<64, 64>(a, s);
    default: return launch_gemm_tile<128, 128>(a, s);
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

hipError_t launch_gather(const GatherArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.n_items + 255) / 256));
  hipLaunchKernelGGL(k_gather, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace qx
