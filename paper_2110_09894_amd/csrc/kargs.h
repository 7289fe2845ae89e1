// Kernel argument blocks shared by the plan compiler (host) and the HIP kernels.
//
// Every tensor is a dense array of complex64 (float2) whose indices all have
// dimension 2, so an element's offset is a sum of per-index ("bit") strides.
// A tensor may also carry a batch dimension over bitstrings ("items").
// Operands are addressed as
//   base + item * item_stride + gather[item] + sum_i bit_i(index) * stride_i
// where gather[] holds, per bitstring, the offset selected by that bitstring's
// qubit values on the operand's open output indices (output closure, Sec. II),
// and base already includes the offset chosen by the fixed sliced indices of
// the current slice (Eq. 2).
#pragma once
#include <stdint.h>

#define QX_MAX_BITS 48      // bits of one tensor (incl. open output and slice bits)
#define QX_MAX_KBITS 24     // contracted bits of one small contraction
#define QX_MAX_HBITS 16     // shared slice bits of one matrix product (batch)
#define QX_MAX_SBITS 24     // slice bits carried to the root
#define QX_MAX_OBITS 16     // open output qubits (amplitudes per bitstring = 2^m)
#define QX_PERM_TB 6        // a permute tile: the output's 6 lowest bits and the input's 6 lowest positions

struct QxCplx { float x, y; };

// Small / memory-bound contraction, one thread per output element:
//   C[item][o] = sum_k A[..o..k] * B[..o..k]     (C dense in o)
struct SimtArgs {
  const QxCplx *a, *b;
  QxCplx *c;
  // fixed sliced indices of leaf operands: offset += bit j of the block's first
  // slice (block[0]) times stride
  const int64_t *block;
  int32_t nfix_a, nfix_b;
  int32_t fix_ja[4], fix_jb[4];
  int64_t fix_sa[4], fix_sb[4];
  int64_t a_item, b_item, c_item;        // item strides (0 = operand shared by all items)
  const int64_t *a_gather, *b_gather;    // per-item offsets, or null
  int32_t n_out, n_k, n_items;
  int32_t pad_;
  int32_t c_split, pad2_;                // C's storage: 0 complex64, 1 split BF16, 2 split FP16 of C * *c_scale
  const float *c_scale;                  // split FP16: C's power-of-two scale
  int64_t a_os[QX_MAX_BITS], b_os[QX_MAX_BITS];   // strides of output bit i (0 if absent)
  int64_t a_ks[QX_MAX_KBITS], b_ks[QX_MAX_KBITS]; // strides of contracted bit j
};

// Batched complex matrix product on the matrix cores:
//   C[z][m][n] = sum_k A[z][m][k] B[z][k][n],  z = item * 2^nh + h
// Element addressing has two modes.  Linear: A(m, k) at m*a_ms + k*a_ks, B(k, n)
// at k*b_ks + n*b_ns, C(m, n) at m*c_ms + n.  Bit-scattered (bits != 0, M, N, K
// powers of two): every bit of m, n, k has its own stride in each operand, so
// any index order of a dim-2 tensor can be read or written in place:
//   A(m, k) at sum_i bit_i(m) a_rs[i] + sum_j bit_j(k) a_kst[j], etc.
// a_kc / b_kc: k bits 0..2 are unit-stride-contiguous (8 consecutive k values
// are 8 consecutive elements), which enables 16-byte loads along k.
// a_split / b_split / c_split: the operand's storage, 0 complex64, 1 split BF16
// planes, 2 split FP16 planes of the value times the tensor's power-of-two
// scale (*a_scale, *b_scale, *c_scale; split_format.h).
#define QX_GEMM_BITS 32
struct GemmArgs {
  const QxCplx *a, *b;
  QxCplx *c;
  int64_t M, N, K;
  int64_t a_ms, a_ks, b_ks, b_ns, c_ms;  // linear mode
  int64_t a_item, b_item, c_item;
  const int64_t *a_gather, *b_gather;
  int32_t n_items, nh;                   // nh = number of shared-slice bits
  int32_t vec_a, vec_b;                  // 16-byte vector loads allowed along k (alignment)
  const float *a_scale, *b_scale, *c_scale;  // split FP16: power-of-two tensor scales (null = 1)
  int32_t bits, nm, nn, nk;              // bit-scattered mode and log2 of M, N, K
  int32_t a_kc, b_kc;
  int32_t a_split, b_split, c_split, pad_split_;
  // epilogue: the ten bits of a 32x32 block in ascending order of output stride,
  // each with its output stride and its contribution to the block-local m / n
  int64_t ep_st[10];
  int32_t ep_lm[10], ep_ln[10];
  int32_t ep_chunk;                      // the three lowest of those strides are 1, 2, 4
  int32_t ep_reg;                        // split output: m bits 0, 1, 3 have output strides 1, 2, 4
  int64_t a_hs[QX_MAX_HBITS], b_hs[QX_MAX_HBITS], c_hs[QX_MAX_HBITS];
  int64_t a_rs[QX_GEMM_BITS], a_kst[QX_GEMM_BITS];
  int64_t b_rs[QX_GEMM_BITS], b_kst[QX_GEMM_BITS];
  int64_t c_mst[QX_GEMM_BITS], c_nst[QX_GEMM_BITS];
  // k-tile offset steps: moving from 16-wide k tile t to t + 1 adds a_kinc[z]
  // (b_kinc[z]) to the operand offset, z = number of trailing one bits of t
  int64_t a_kinc[QX_GEMM_BITS], b_kinc[QX_GEMM_BITS];
};

// Long inner products (root of a slice's tree):
//   C[item][o] = sum_{k<K} A[..o..][k] * B[..o..][k]   (k contiguous in both)
// Output bits fastest first: those of B only, those of A only, those of both.
// Scratch for sums split over work-groups: at most QX_DOT_PART_ELEMS complex values.
#define QX_DOT_PART_ELEMS (2048 * 64)

struct DotArgs {
  const QxCplx *a, *b;
  QxCplx *c;
  QxCplx *part;                         // QX_DOT_PART_ELEMS of scratch for split sums, or null
  int64_t K;
  int64_t a_item, b_item, c_item;
  const int64_t *a_gather, *b_gather;
  int32_t n_out, n_items;
  int32_t c_split, pad2_;                // C's storage: 0 complex64, 1 split BF16, 2 split FP16 of C * *c_scale
  const float *c_scale;
  int64_t a_os[QX_MAX_BITS], b_os[QX_MAX_BITS];
};

// Bit permutation: out[item][o] = in[item][sum_i bit_i(o) << in_pos[i]]
// The host splits the bits into a tile (the output's lowest bits plus the bits
// at the input's lowest positions, at most 2 QX_PERM_TB) and outer bits.
struct PermArgs {
  const QxCplx *in;
  QxCplx *out;
  int64_t in_item, out_item;
  int32_t rank, n_items;
  int32_t in_pos[QX_MAX_BITS];
  int32_t nt, n_outer;                  // tile bits, outer bits
  int32_t tl[2 * QX_PERM_TB];           // tile bits (output-bit indices), ascending
  int32_t ll[2 * QX_PERM_TB];           // tile-bit slots in ascending input position
  int64_t outer_in[QX_MAX_BITS], outer_out[QX_MAX_BITS];  // strides of outer bit i
  int32_t vec, pad_;                    // 16-byte pair accesses (aligned pointers, even item strides)
};

// Sum over the slices of one block, FP64, ascending slice order:
//   amp[item] += sum_{s in [s_lo, s_hi)} root[item-offset + sum_j bit_j(s) * s_stride[j]]
struct SliceSumArgs {
  const QxCplx *root;
  const int64_t *block;                 // if set, the slice range is block[1], block[2]
  int64_t root_item;
  const int64_t *root_gather;
  double *amp;                          // [items][2^n_obits][2]
  int32_t n_items, n_sbits;             // n_items counts values: bitstrings << n_obits
  int32_t s_lo, s_hi;
  int64_t s_stride[QX_MAX_SBITS];
  int32_t n_obits, pad_;                // open output qubits: value j's bit i selects o_stride[i]
  int64_t o_stride[QX_MAX_OBITS];
};

// Largest magnitude of a tensor, folded into a running maximum (one per FP16 operand
// scale, over several calibration passes).  Work-groups write partial maxima; the last
// one to finish (ticket counter) reduces them, updates maxv and resets the counter for
// the next launch.
struct AbsmaxArgs {
  const QxCplx *x;
  int64_t n;                            // complex elements
  float *partial;                       // [gridDim.x]
  unsigned int *ticket;                 // zero before the first launch; left zero after each
  float *maxv;                          // running largest |Re|, |Im|: maxv[0] = max(maxv[0], max of x)
};

// Running maxima -> power-of-two FP16 operand scales, in place:
//   v[i] = 2^(target_exp - e) with v[i] < 2^e (clamped to 2^-100..2^100); 1 where v[i] is zero
struct ScaleFromMaxArgs {
  float *v;
  int32_t n, target_exp;
};

// Slice-block state kept on the device so one captured block program can be
// replayed for every block:  state[0] first slice of the current block,
// state[1], state[2] local slice range [lo, hi), state[3] next block index,
// state[4], state[5] the call's slice range, state[6] log2 slices per block.
struct BlockArgs {
  int64_t *state;
  double *acc;                          // [n_items][2] FP64 accumulator (zeroed by k_block_init);
                                        // n_items counts values: bitstrings << open qubits
  int64_t first_block, slice_begin, slice_end;
  int32_t js, n_items;
};

// Complex64 matrices -> split form (kind 1 BF16, 2 FP16 at unit scale), k padded with zeros to kp:
//   out[item][r][k'] (split) = in[item * in_item + r * ld_r + k' * ld_k] for k' < K, else 0
struct SplitPlanesArgs {
  const QxCplx *in;
  uint16_t *out;
  int64_t rows, K, kp, ld_r, ld_k, in_item;
  int32_t n_items, kind;
};

// A complex64 tensor of n elements (n a multiple of 8) rewritten in place in split FP16
// form of x * *scale: every 64-byte chunk of 8 elements becomes their four planes.
struct SplitInplaceArgs {
  QxCplx *x;
  int64_t n;
  const float *scale;
};

// Per-bitstring gather offsets: out[item] = sum_j bit_{q_j}(x[item]) * stride_j
struct GatherArgs {
  const uint64_t *x;
  int64_t *out;
  int32_t n_items, n_q;
  int32_t q[64];
  int64_t stride[64];
};
