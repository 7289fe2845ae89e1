/*
 * qxtn.h -- C-ABI of the sliced tensor-network amplitude library for AMD MI355X (gfx950).
 *
 * What is computed.  A tensor network is a product of tensors summed over the
 * indices they share (Sec. II, Eq. 1).  For a quantum circuit, the network built
 * from its gates has one open index per qubit; closing each open index with the
 * value of that qubit in a bitstring x turns the network's value into the
 * amplitude <x|U|0...0> (Sec. II).  Slicing fixes a chosen set of indices to
 * each of their values: the network's value is the sum of the values of the
 * 2^k sliced networks, which are independent (Sec. III-A, Eq. 2).  Each sliced
 * network is contracted as a sequence of pairwise contractions along a given
 * contraction tree (Sec. III-A), each pairwise contraction being an index
 * permutation followed by a complex matrix product (Sec. IV-A: contractions
 * mapped to matrix multiplications).
 *
 * Two calls carry the method:
 *   qx_plan_create(network, contraction_tree, sliced_indices) -> plan
 *   qx_contract(plan, bitstrings, slice_range) -> amplitudes (accumulated)
 *
 * Conventions shared by all calls.
 *   - Every index has dimension 2.  A tensor of rank r holds 2^r complex
 *     values, row-major in the order of its listed indices (first index
 *     slowest).
 *   - Bitstrings are packed uint64: bit q is the value of qubit q (q < 64).
 *   - Slice s in [0, 2^k) sets the j-th sliced index to bit j of s.
 *   - Device buffers are HIP device pointers; "stream" is a hipStream_t passed
 *     as void* (NULL = the default stream).
 *   - Every function returns a qx_status; on error a message is available from
 *     qx_last_error() (thread-local, valid until the next call on the thread).
 *     Errors are detected on the host before any work is enqueued, and a failed
 *     call leaves the plan usable.
 */
#ifndef QXTN_H
#define QXTN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QX_OK = 0,
  QX_ERR_INVALID_ARG = -1,     /* bad pointer, size or range */
  QX_ERR_INVALID_NETWORK = -2, /* label used other than twice (once for an output wire), ... */
  QX_ERR_INVALID_TREE = -3,    /* not one SSA binary tree consuming every tensor once */
  QX_ERR_UNSUPPORTED = -4,     /* e.g. a dimension other than 2, more than 64 qubits */
  QX_ERR_OUT_OF_BUDGET = -5,   /* the plan's device memory would exceed hbm_budget_bytes */
  QX_ERR_HIP = -6,             /* a HIP runtime call failed */
  QX_ERR_DRY_RUN = -7          /* device work requested from a host-only plan */
} qx_status;

typedef enum {
  QX_C64 = 0,        /* complex64 storage, FP32 MFMA matrix products */
  QX_SPLIT_BF16 = 1, /* matrix products as BF16 hi+lo terms on MFMA, FP32 accumulation */
  QX_SPLIT_FP16 = 2  /* matrix products as FP16 hi+lo terms on MFMA, FP32 accumulation; each
                        operand tensor is stored times a power-of-two scale fixed at plan creation
                        by four complex64 calibration passes over pseudo-random bitstrings and
                        slice blocks spread over the range (its largest magnitude there then lies
                        below 2^6, about 1000x below FP16's limit; a later value beyond that
                        headroom gives non-finite amplitudes) */
} qx_precision;

/* The network: leaves only.  Output wires are open indices, not tensors. */
typedef struct {
  int32_t n_tensors;           /* number of leaf tensors, >= 1 */
  const int64_t *index_ptr;    /* [n_tensors+1] CSR offsets into index_ids */
  const int64_t *index_ids;    /* labels (>= 0); each label appears in exactly two tensors,
                                  or in one tensor if it is an output wire */
  const int64_t *data_ptr;     /* [n_tensors+1] offsets into data, in complex elements;
                                  tensor t holds 2^(rank t) elements */
  const double *data;          /* complex128 values, interleaved (re, im) */
  int32_t n_qubits;            /* 0..64 */
  const int64_t *output_index; /* [n_qubits] label of qubit q's output wire */
} qx_network;

typedef struct {
  int32_t precision;           /* qx_precision */
  int32_t max_bitstrings;      /* largest B a qx_contract call may pass (>= 1) */
  int32_t slice_batch_log2;    /* sliced indices 0..j-1 vary inside one device pass; -1 = auto:
                                  the cheapest estimated j (matrix work plus launches per block)
                                  whose plan fits hbm_budget_bytes, or when that is 0, 96 GiB and
                                  (unless dry_run) 80% of the device's free memory */
  int32_t dry_run;             /* non-zero: compile on the host only, touch no device */
  int64_t hbm_budget_bytes;    /* 0 = no limit */
  int32_t autotune;            /* non-zero: time every matrix-core tile shape that fits each
                                  per-call / per-block product at plan creation and keep the
                                  fastest (results cached per shape for the process) */
  int32_t eager;               /* non-zero: launch every op of every slice block individually;
                                  0: capture one block's ops in a HIP graph per batch size and
                                  replay it for every block (always eager while timing is on) */
  uint64_t open_qubits;        /* bit q set: qubit q's output wire stays open, so each bitstring
                                  yields the 2^m amplitudes of all values of those m qubits
                                  (Sec. II: output indices left open give a batch of amplitudes);
                                  m <= 16 and max_bitstrings * 2^m <= 2^24.  0 = all closed */
  int32_t gemm_tile;           /* matrix-core work-group tile of every product: 0 = automatic (the
                                  autotuner's choice when autotune is set, else a default by shape);
                                  t + 1 = force qx_gemm_tile t for every product (autotune is then
                                  ignored); other values are rejected */
  int32_t reserved_;           /* must be 0 */
} qx_plan_options;

/* Work-group tile shapes (rows of A x columns of B) of the matrix-core products.
 * Options and qx_cgemm take the tile as (value + 1), 0 meaning automatic.  The P3
 * and P4 shapes are the split-precision products' software-pipelined form (one
 * work-group per CU, three or four LDS stages); complex64 runs them as 128x128.
 * THIN is the memory-bound kernel for products with one side of at most 32 and
 * K of at most 32 (16x16 matrix-core shapes, independent wavefronts, any
 * storage), and the default for them; forced on another product it runs that
 * product's default tile.  Split-precision products whose K is neither 8 nor a
 * multiple of 16 (large contractions with a short side and a sum of 2 or 4
 * terms) run THIN whatever tile is asked for. */
typedef enum {
  QX_TILE_128x128 = 0,
  QX_TILE_64x64 = 1,
  QX_TILE_128x64 = 2,
  QX_TILE_64x128 = 3,
  QX_TILE_256x128 = 4,
  QX_TILE_128x256 = 5,
  QX_TILE_128x128P3 = 6,
  QX_TILE_128x128P4 = 7,
  QX_TILE_THIN = 8,
  QX_N_TILES = 9
} qx_gemm_tile;

typedef struct {
  int64_t device_bytes;        /* device memory the plan holds (leaves, constants, arena, per-call
                                  state; 1 MiB of inner-product partial sums in plans that have one) */
  int64_t arena_bytes;         /* part of device_bytes used as per-call working memory */
  int32_t n_leaves;
  int32_t n_sliced;
  int32_t slice_batch_log2;    /* effective value */
  int32_t width;               /* log2 elements of the largest per-slice intermediate */
  int32_t n_ops_const;         /* device ops run once at plan creation */
  int32_t n_ops_call;          /* device ops run once per qx_contract call */
  int32_t n_ops_block;         /* device ops run once per slice block */
  int32_t n_gemm_block;        /* of which matrix-core products */
  double flops_per_slice;      /* 8*M*N*K summed over the tree for one slice and one bitstring */
  double flops_block;          /* complex flops executed per slice block at max_bitstrings */
  double gemm_flops_block;     /* of which on matrix cores */
  double flops_call;           /* complex flops executed once per call */
  int32_t n_open;              /* m: open output qubits (amplitudes per bitstring = 2^m) */
  int32_t reserved;
} qx_plan_info;

typedef struct qx_plan qx_plan;

/*
 * Compile a plan: validate the network and the tree, choose each
 * intermediate's memory layout, lay out the device arena, upload the leaves
 * (rounded to complex64) and pre-contract the sub-trees that depend neither on
 * the bitstring nor on the slice.  Sec. III-A (contraction order, slicing),
 * Sec. IV-A (simulation plan separated from the tensor primitives).
 *
 *   net            host; copied, may be freed on return.
 *   tree           host int32 [n_tensors-1][2]; step t contracts ids (a, b) and
 *                  creates id n_tensors + t.  Ids refer to leaves (< n_tensors)
 *                  or earlier steps.  The last step is the root.
 *   sliced         host int64 [n_sliced] labels to slice; none may be an output
 *                  wire; n_sliced <= 40.
 *   opt            host; NULL = defaults (QX_C64, max_bitstrings 1, auto, 0, 0, 0, 0, 0).
 *   stream         hipStream_t used for uploads and pre-contraction.
 *   out            receives the plan (owned by the caller; free with qx_plan_destroy).
 */
qx_status qx_plan_create(const qx_network *net, const int32_t *tree, const int64_t *sliced,
                         int32_t n_sliced, const qx_plan_options *opt, void *stream,
                         qx_plan **out);

/* Sizes and work figures of a plan (host only; valid for dry-run plans). */
qx_status qx_plan_get_info(const qx_plan *plan, qx_plan_info *info);

/*
 * Device memory the same network, tree and slice set would hold as a plan with
 * another bitstring capacity or slice batch (Sec. III-B: device memory is the
 * second, tighter bottleneck; Sec. III-A: slicing trades memory for repeated
 * work).  Host only: the plan is recompiled on the host with those two values
 * (nothing is allocated on the device), so it is valid on dry-run plans and
 * costs milliseconds; the figure is what qx_plan_get_info's device_bytes
 * would report for that plan (leaves, constants, arena, gather tables, scale
 * slots, slice-block state and FP64 accumulator), excluding the caller's
 * bitstring and amplitude buffers (8 * B and 16 * B * 2^m bytes).
 *
 *   plan              any plan (dry-run or not); not modified.
 *   n_bitstrings      0 = the plan's max_bitstrings, else 1..2^20 with
 *                     n_bitstrings * 2^m <= 2^24.
 *   slice_batch_log2  -1 = the plan's effective slice batch, else
 *                     0..min(n_sliced, 24): 2^j slices computed per pass.
 *   bytes             receives the figure.
 * Errors: QX_ERR_INVALID_ARG (NULL pointer, value out of range).
 */
qx_status qx_plan_peak_bytes(const qx_plan *plan, int32_t n_bitstrings, int32_t slice_batch_log2,
                             int64_t *bytes);

/*
 * Accumulate amplitudes: for each of the B bitstrings x_b,
 *   d_amplitudes[b] += sum over slices s in [slice_begin, slice_end) of the value
 *                      of slice s's network closed by x_b        (Eq. 2, Sec. II)
 * With m open qubits q_0 < ... < q_{m-1} the network is closed by x_b on the
 * other qubits only and d_amplitudes[b][j] receives the amplitude of x_b with
 * qubit q_i set to bit i of j (x_b's own bits at open qubits are ignored).
 * Per-slice values are formed in FP32 complex; the sum over slices and the
 * accumulation are FP64 in a fixed order (blocks in ascending order; inside a
 * block, 64 ascending strided partial sums joined by a fixed butterfly), so the
 * result is bitwise reproducible for a given plan, range and B.
 *
 *   d_bitstrings   device uint64 [B].
 *   B              1..max_bitstrings.
 *   slice range    0 <= slice_begin <= slice_end <= 2^n_sliced (empty is a no-op).
 *   d_amplitudes   device double [B][2^m][2] (re, im), caller-zeroed, ACCUMULATED (+=);
 *                  m = 0 unless the plan has open qubits.  Its size is not checked here.
 *   stream         all work is enqueued on it; the call does not synchronise.
 * Calls on one plan must not overlap in time (the plan's arena is shared):
 * serialise them on one stream.  Caller buffers must stay alive until the
 * stream has completed the work.
 */
qx_status qx_contract(qx_plan *plan, const uint64_t *d_bitstrings, int32_t B,
                      int64_t slice_begin, int64_t slice_end, double *d_amplitudes,
                      void *stream);

/* Release every device and host resource of the plan (NULL is a no-op).
 * First waits for the plan's own device work: the pre-contraction at creation
 * and the work enqueued by its last qx_contract call (an event recorded at the
 * end of each call on the call's stream); other work on the device is not
 * waited for. */
void qx_plan_destroy(qx_plan *plan);

/* Message of the last failed call on this thread ("" if none). */
const char *qx_last_error(void);

/* ---- measurement ---------------------------------------------------------- */

/* Classes of device launches a plan makes. */
typedef enum {
  QX_OPCLASS_GEMM = 0,      /* complex matrix products on the matrix cores */
  QX_OPCLASS_SIMT = 1,      /* small / memory-bound contractions */
  QX_OPCLASS_DOT = 2,       /* long inner products (root of a slice's tree) */
  QX_OPCLASS_PERMUTE = 3,   /* index permutations */
  QX_OPCLASS_SLICESUM = 4,  /* FP64 sum over slices */
  QX_OPCLASS_GATHER = 5,    /* per-bitstring gather offsets */
  QX_OPCLASS_SCALE = 6,     /* operand magnitude reductions for FP16 scaling */
  QX_N_OPCLASS = 7
} qx_opclass;

typedef struct {
  int64_t launches;
  double seconds;   /* sum of HIP-event durations bracketing each launch */
  double flops;     /* algorithmic complex flops (8 M N K per product) */
  double bytes;     /* algorithmic bytes (each operand read once, result written once) */
} qx_op_timing;

/* One device operation of a compiled plan (host only; valid for dry-run plans). */
typedef struct {
  int32_t phase;     /* 0 run once at plan creation, 1 once per qx_contract call, 2 once per slice block */
  int32_t op_class;  /* qx_opclass */
  int64_t M, N, K;   /* matrix product: C[M][N] += A[M][K] B[K][N]; other ops: output elements, 1, summed
                        elements (K = 1 for permutes and magnitude reductions) */
  int64_t batch;     /* independent products per launch at max_bitstrings (bitstring items times
                        shared varying-slice combinations) */
  int32_t tile;      /* qx_gemm_tile the product launches with (autotuned or forced), -1 otherwise */
  int32_t batched;   /* the op's batch scales with the call's B (one copy per bitstring) */
  double flops;      /* algorithmic complex flops at max_bitstrings (8 M N K batch for products) */
  double bytes;      /* algorithmic bytes at max_bitstrings (operands read once, result written once) */
} qx_op_info;

/* Ops are numbered in launch order: index 0 .. n_ops_const + n_ops_call + n_ops_block - 1 (qx_plan_info);
 * the plan-time ops first, then the per-call ops, then the per-block ops.  QX_ERR_INVALID_ARG for an index
 * out of range. */
qx_status qx_plan_get_op_info(const qx_plan *plan, int32_t index, qx_op_info *info);

/* enable != 0: every launch made by qx_contract on this plan is bracketed by a
 * pair of HIP events recorded on the launch's stream. */
qx_status qx_plan_set_timing(qx_plan *plan, int32_t enable);

/* Wait for the recorded events and return per-class totals since the last
 * reset (out: host array [QX_N_OPCLASS]).  reset != 0 clears the totals. */
qx_status qx_plan_get_timing(qx_plan *plan, qx_op_timing *out, int32_t reset);

/* ---- kernel-level entry points (the primitives a plan is built from) ------ */

/*
 * Index permutation of a batch of rank-r dim-2 tensors (Sec. III-B: permute
 * primitive).  With bits numbered from the fastest (bit 0), output element o
 * of item z is read from input element  sum_i bit_i(o) << in_pos[i]:
 *   out[z][o] = in[z][ sum_i ((o >> i) & 1) << in_pos[i] ].
 * in_pos (host, int32 [rank]) must be a permutation of 0..rank-1; rank <= 40.
 * d_in, d_out: device complex64 (float2) [items][2^rank], not overlapping.
 */
qx_status qx_permute_c64(const void *d_in, void *d_out, int32_t rank, const int32_t *in_pos,
                         int64_t items, void *stream);

/*
 * Strided-batched complex matrix product on the matrix cores (Sec. IV-A:
 * contractions mapped to matrix multiplications):
 *   C[z][m][n] = sum_k A[z][m][k] * B[z][k][n],   0 <= z < batch
 * Element (m, k) of A item z is at d_a + z*stride_a + m*a_ms + k*a_ks; one of
 * a_ms, a_ks must be 1.  B likewise with (k, n) strides b_ks, b_ns.  C item z
 * is dense row-major [M][N] at d_c + z*stride_c.  All strides in complex
 * elements.  precision: qx_precision.  M, N, K >= 1.  tile: 0 = a default
 * work-group tile by shape, t + 1 = qx_gemm_tile t (any tile is valid for any
 * M, N).  Asynchronous on stream.
 * The split precisions first split A and B into stream-ordered temporaries
 * (hipMallocAsync, 8*batch*(M+N)*roundup(K,16) bytes, freed on the stream;
 * FP16 planes at unit scale, so A and B should lie within FP16's range: values
 * of magnitude 2^-3 .. 2^15 keep 22 significant bits); the split products of a
 * plan read operands their producers stored split and allocate nothing.  Errors: QX_ERR_INVALID_ARG (NULL pointer,
 * sizes, strides, tile), QX_ERR_HIP (launch or allocation failure).
 */
qx_status qx_cgemm(const void *d_a, const void *d_b, void *d_c, int64_t M, int64_t N, int64_t K,
                   int64_t a_ms, int64_t a_ks, int64_t b_ks, int64_t b_ns, int64_t stride_a,
                   int64_t stride_b, int64_t stride_c, int64_t batch, int32_t precision,
                   int32_t tile, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): the product of
 * qx_cgemm, same arguments and same kernels, allocating nothing.  The split
 * operand copies that qx_cgemm puts in stream-ordered allocations go to a
 * scratch array compiled into the library instead: each device the library
 * runs on holds QX_CGEMM_NOALLOC_SCRATCH_BYTES of it until the process ends.
 * QX_C64 uses no scratch.
 *   Limit: with a split precision, 8 * batch * (M + N) * roundup(K, 16) bytes must
 *   not exceed QX_CGEMM_NOALLOC_SCRATCH_BYTES, else QX_ERR_INVALID_ARG before
 *   anything is enqueued.
 *   Sharing: every call on a device uses that device's one scratch, which keeps
 *   the last call's contents (each call overwrites all it reads); calls whose
 *   work overlaps in time on one device (other streams, other host threads)
 *   race and must be serialised, e.g. on one stream.
 *   Set-up: the first call made with a device current looks up that device's
 *   scratch address (hipGetSymbolAddress); no call allocates or frees memory.
 * Other errors as qx_cgemm.
 */
#define QX_CGEMM_NOALLOC_SCRATCH_BYTES (64LL << 20)
qx_status qx_cgemm_noalloc(const void *d_a, const void *d_b, void *d_c, int64_t M, int64_t N, int64_t K,
                           int64_t a_ms, int64_t a_ks, int64_t b_ks, int64_t b_ns, int64_t stride_a,
                           int64_t stride_b, int64_t stride_c, int64_t batch, int32_t precision,
                           int32_t tile, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QXTN_H */
