// Thin complex products: one operand small (at most 32 rows, K at most 32), the
// other large.  Such a product reads the large operand once and writes an output
// of the same size, so HBM bandwidth bounds it, not the matrix cores: the small
// operand goes to LDS once per work-group, and each thread streams one row of the
// large operand (its K values) and writes that row's outputs.  Operands and
// output may be complex64 or split (BF16 planes, or FP16 planes of scaled
// values); the arithmetic is FP32.
#include "gemm_common.h"

namespace qx {

namespace {

constexpr int THIN_MAX_S = 32;  // rows of the small operand
constexpr int THIN_MAX_K = 32;

__device__ __forceinline__ float f16_value(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// Element e of a tensor stored as kind 0 (complex64), 1 (split BF16) or 2 (split FP16 of x * scale;
// inv = 1 / scale).
__device__ __forceinline__ QxCplx load_elem(const QxCplx* X, int kind, float inv, int64_t e) {
  if (kind == 0) return X[e];
  const uint16_t* P = reinterpret_cast<const uint16_t*>(X);
  const int64_t c = split_chunk(e) + (e & 7);
  if (kind == 1)
    return QxCplx{bf16_value(P[c]) + bf16_value(P[c + 8]), bf16_value(P[c + 16]) + bf16_value(P[c + 24])};
  return QxCplx{(f16_value(P[c]) + f16_value(P[c + 8])) * inv, (f16_value(P[c + 16]) + f16_value(P[c + 24])) * inv};
}

}  // namespace

// A_SMALL: A (M <= 32 rows) is the small operand and a thread owns one column n of B and C;
// otherwise B (N <= 32 columns) is small and a thread owns one row m of A and C.
template <bool A_SMALL>
__global__ __launch_bounds__(256) void k_gemm_thin(GemmArgs p) {
  __shared__ QxCplx sm[THIN_MAX_S * THIN_MAX_K];
  const int64_t L = A_SMALL ? p.N : p.M;
  const int S = (int)(A_SMALL ? p.M : p.N), K = (int)p.K;
  const int64_t chunks = (L + 255) / 256;
  const int64_t z = blockIdx.x / chunks, ch = blockIdx.x - z * chunks;
  const int item = (int)(z >> p.nh);
  int64_t aoff = (int64_t)item * p.a_item + (p.a_gather ? p.a_gather[item] : 0);
  int64_t boff = (int64_t)item * p.b_item + (p.b_gather ? p.b_gather[item] : 0);
  int64_t coff = (int64_t)item * p.c_item;
  for (uint32_t hb = (uint32_t)(z & ((1LL << p.nh) - 1)); hb; hb &= hb - 1) {
    const int i = __builtin_ctz(hb);
    aoff += p.a_hs[i];
    boff += p.b_hs[i];
    coff += p.c_hs[i];
  }
  const float inva = 1.f / out_scale(p.a_scale), invb = 1.f / out_scale(p.b_scale);
  // the small operand, [s][k], into LDS
  for (int i = threadIdx.x; i < S * K; i += 256) {
    const int sidx = i / K, k = i - sidx * K;
    int64_t e;
    if (A_SMALL) e = aoff + (p.bits ? scatter_bits<5>(sidx, p.a_rs, p.nm) + scatter_bits<5>(k, p.a_kst, p.nk)
                                    : (int64_t)sidx * p.a_ms + (int64_t)k * p.a_ks);
    else e = boff + (p.bits ? scatter_bits<5>(sidx, p.b_rs, p.nn) + scatter_bits<5>(k, p.b_kst, p.nk)
                            : (int64_t)sidx * p.b_ns + (int64_t)k * p.b_ks);
    sm[i] = A_SMALL ? load_elem(p.a, p.a_split, inva, e) : load_elem(p.b, p.b_split, invb, e);
  }
  __syncthreads();
  const int64_t l = ch * 256 + threadIdx.x;
  if (l >= L) return;
  // this thread's row of the large operand: its K values
  QxCplx x[THIN_MAX_K];
  {
    const QxCplx* X = A_SMALL ? p.b : p.a;
    const int kind = A_SMALL ? p.b_split : p.a_split;
    const float inv = A_SMALL ? invb : inva;
    int64_t base;
    if (A_SMALL) base = boff + (p.bits ? scatter_bits(l, p.b_rs, p.nn) : l * p.b_ns);
    else base = aoff + (p.bits ? scatter_bits(l, p.a_rs, p.nm) : l * p.a_ms);
#pragma unroll
    for (int k = 0; k < THIN_MAX_K; ++k) {
      if (k < K) {
        const int64_t ko = p.bits ? scatter_bits<5>(k, A_SMALL ? p.b_kst : p.a_kst, p.nk)
                                  : (int64_t)k * (A_SMALL ? p.b_ks : p.a_ks);
        x[k] = load_elem(X, kind, inv, base + ko);
      }
    }
  }
  const float cs = p.c_split == 2 ? out_scale(p.c_scale) : 1.f;
  const int64_t lo = p.bits ? (A_SMALL ? scatter_bits(l, p.c_nst, p.nn) : scatter_bits(l, p.c_mst, p.nm))
                            : (A_SMALL ? l : l * p.c_ms);
  for (int sidx = 0; sidx < S; ++sidx) {
    QxCplx acc = {0.f, 0.f};
#pragma unroll
    for (int k = 0; k < THIN_MAX_K; ++k)
      if (k < K) acc = cmul_acc(acc, sm[sidx * K + k], x[k]);
    const int64_t so = p.bits ? (A_SMALL ? scatter_bits<5>(sidx, p.c_mst, p.nm) : scatter_bits<5>(sidx, p.c_nst, p.nn))
                              : (A_SMALL ? (int64_t)sidx * p.c_ms : sidx);
    const int64_t e = coff + lo + so;
    if (p.c_split) store_split(reinterpret_cast<uint16_t*>(p.c), e, acc, p.c_split, cs);
    else p.c[e] = acc;
  }
}

bool gemm_thin_fits(const GemmArgs& a) {
  return (a.M < a.N ? a.M : a.N) <= THIN_MAX_S && a.K <= THIN_MAX_K;
}

hipError_t launch_gemm_thin(const GemmArgs& a, hipStream_t s) {
  if (!gemm_thin_fits(a)) return hipErrorInvalidValue;
  const bool a_small = a.M <= a.N;
  const int64_t L = a_small ? a.N : a.M;
  const int64_t nwg = ((L + 255) / 256) * (int64_t)a.n_items * (1LL << a.nh);
  if (nwg <= 0) return hipSuccess;
  if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
  if (a_small) hipLaunchKernelGGL(k_gemm_thin<true>, dim3((unsigned)nwg), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_gemm_thin<false>, dim3((unsigned)nwg), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace qx
