// C-ABI entry points and the plan executor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "plan.h"
#include "qxtn.h"
#include "split_format.h"

using namespace qx;

static thread_local std::string g_err;

// Host BF16 rounding (nearest even), for leaves that are stored split.
static uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static float bf16_float(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

static qx_status fail(qx_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(QX_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

struct PendingEvent {
  int cls;
  hipEvent_t a, b;
  double flops, bytes;
};

struct qx_plan {
  PlanCore pc;
  bool timing = false;
  std::vector<PendingEvent> pending;
  std::vector<hipEvent_t> pool;
  qx_op_timing acc[QX_N_OPCLASS];
  bool dry = true;
  int device = 0;
  QxCplx* d_leaves = nullptr;
  char* d_arena = nullptr;
  int64_t* d_gather = nullptr;
  float* d_misc = nullptr;            // FP16 operand scales, absmax partials, absmax ticket
  int64_t* d_state = nullptr;         // slice-block state (8 int64), FP64 accumulator [max_b][2], dot partials
  int64_t device_bytes = 0;
  bool eager = false;
  hipStream_t cap_stream = nullptr;   // stream used to capture block programs
  std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs;  // per batch size
  hipEvent_t done = nullptr;          // recorded after the plan's latest device work
  // host copies of the compile inputs, so the plan can be recompiled with another
  // bitstring capacity or slice batch (qx_plan_peak_bytes)
  std::vector<int64_t> net_index_ptr, net_index_ids, net_data_ptr, net_output;
  int32_t net_n_qubits = 0;
  std::vector<int32_t> tree;
  std::vector<int64_t> sliced;
  qx_plan_options opt{};
};

// d_state: slice-block state (64 bytes), the FP64 accumulator, then (plans with a long inner product)
// the partial sums of inner products split over work-groups
static int64_t acc_bytes(const PlanCore& pc) { return ((int64_t)pc.max_b << pc.n_open) * 16; }
static int64_t state_bytes(const PlanCore& pc) {
  bool dot = false;
  for (const Op& o : pc.ops) dot = dot || o.kind == OP_DOT;
  return 64 + acc_bytes(pc) + (dot ? (int64_t)QX_DOT_PART_ELEMS * 8 : 0);
}

static int64_t misc_bytes(const PlanCore& pc) {
  return ((int64_t)pc.n_scale_slots + ABSMAX_PARTIALS + 64) * 4;
}

static int64_t plan_device_bytes(const PlanCore& pc) {
  return ((pc.leaf_pool_elems * 8 + 255) / 256) * 256 + pc.arena_bytes +
         (int64_t)pc.gathers.size() * pc.max_b * 8 + misc_bytes(pc) + state_bytes(pc);
}

static QxCplx* tensor_ptr(qx_plan* p, int tid) {
  const Tensor& t = p->pc.tensors[tid];
  return t.is_leaf ? p->d_leaves + t.leaf_off : reinterpret_cast<QxCplx*>(p->d_arena + t.arena_off);
}

static const int64_t* gather_ptr(qx_plan* p, int g) {
  return g < 0 ? nullptr : p->d_gather + (int64_t)g * p->pc.max_b;
}

static float* scale_ptr(qx_plan* p, int slot) { return slot < 0 ? nullptr : p->d_misc + 64 + ABSMAX_PARTIALS + slot; }

// Split FP16 tensors are stored as x * 2^(FP16_TARGET_EXP - e) with max |x| < 2^e measured in the
// calibration pass: the largest value lands below 2^6, leaving FP16's range (65504) a factor of about
// 1000 of headroom, while values down to 2^-3 keep 22 significant bits and smaller ones an absolute
// error of at most 2^-25, i.e. 2^-30 of the tensor's largest value.
constexpr int FP16_TARGET_EXP = 6;

static void resolve_pointers(qx_plan* p) {
  for (Op& op : p->pc.ops) {
    QxCplx* a = op.in_a >= 0 ? tensor_ptr(p, op.in_a) : nullptr;
    QxCplx* b = op.in_b >= 0 ? tensor_ptr(p, op.in_b) : nullptr;
    QxCplx* c = op.out >= 0 ? tensor_ptr(p, op.out) : nullptr;
    // split FP16 output: the producer applies the output tensor's scale
    const float* cs = op.out >= 0 ? scale_ptr(p, p->pc.tensors[op.out].scale_slot) : nullptr;
    switch (op.kind) {
      case OP_SIMT:
        op.simt.a = a; op.simt.b = b; op.simt.c = c;
        op.simt.a_gather = gather_ptr(p, op.gather_a);
        op.simt.b_gather = gather_ptr(p, op.gather_b);
        op.simt.block = (op.fix_a.empty() && op.fix_b.empty()) ? nullptr : p->d_state;
        op.simt.c_scale = cs;
        op.simt.nfix_a = (int)op.fix_a.size();
        op.simt.nfix_b = (int)op.fix_b.size();
        for (size_t i = 0; i < op.fix_a.size(); ++i) {
          op.simt.fix_ja[i] = op.fix_a[i].j;
          op.simt.fix_sa[i] = op.fix_a[i].stride;
        }
        for (size_t i = 0; i < op.fix_b.size(); ++i) {
          op.simt.fix_jb[i] = op.fix_b[i].j;
          op.simt.fix_sb[i] = op.fix_b[i].stride;
        }
        break;
      case OP_GEMM:
        op.gemm.a = a; op.gemm.b = b; op.gemm.c = c;
        op.gemm.a_gather = gather_ptr(p, op.gather_a);
        op.gemm.b_gather = gather_ptr(p, op.gather_b);
        op.gemm.a_scale = scale_ptr(p, op.scale_slot);
        op.gemm.b_scale = op.scale_slot >= 0 ? scale_ptr(p, op.scale_slot + 1) : nullptr;
        op.gemm.c_scale = cs;
        break;
      case OP_ABSMAX:
        op.absmax.x = a;
        op.absmax.ticket = reinterpret_cast<unsigned int*>(p->d_misc);
        op.absmax.partial = p->d_misc + 64;
        op.absmax.maxv = scale_ptr(p, op.scale_slot);
        break;
      case OP_DOT:
        op.dot.a = a; op.dot.b = b; op.dot.c = c;
        op.dot.a_gather = gather_ptr(p, op.gather_a);
        op.dot.b_gather = gather_ptr(p, op.gather_b);
        op.dot.c_scale = cs;
        op.dot.part = reinterpret_cast<QxCplx*>(reinterpret_cast<char*>(p->d_state) + 64 + acc_bytes(p->pc));
        break;
      case OP_PERM:
        op.perm.in = a; op.perm.out = c;
        break;
    }
  }
}

static hipEvent_t take_event(qx_plan* p) {
  if (!p->pool.empty()) {
    hipEvent_t e = p->pool.back();
    p->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch through f(), bracketed by events when timing is enabled.
template <class F>
static hipError_t timed(qx_plan* p, int cls, double flops, double bytes, hipStream_t s, F f) {
  if (!p->timing) return f();
  PendingEvent ev{cls, take_event(p), take_event(p), flops, bytes};
  if (!ev.a || !ev.b) return hipErrorOutOfMemory;
  hipEventRecord(ev.a, s);
  hipError_t e = f();
  hipEventRecord(ev.b, s);
  p->pending.push_back(ev);
  return e;
}

static int op_class(int kind) {
  switch (kind) {
    case OP_GEMM: return QX_OPCLASS_GEMM;
    case OP_DOT: return QX_OPCLASS_DOT;
    case OP_PERM: return QX_OPCLASS_PERMUTE;
    case OP_ABSMAX: return QX_OPCLASS_SCALE;
    default: return QX_OPCLASS_SIMT;
  }
}

// How run_op launches an op.  RUN: the plan's own kernels; magnitude reductions
// are skipped.  CALIBRATE (split FP16 plans, at creation): every tensor is kept
// in complex64 and the products run on the complex64 kernel, so the magnitude
// reductions see the values the split FP16 tensors will hold.
enum RunMode { MODE_RUN = 0, MODE_CALIBRATE = 1 };

// Fixed sliced indices only occur on leaf operands of small contractions,
// whose kernel adds them from the device-side block state.
static qx_status run_op(qx_plan* p, const Op& op, int B, hipStream_t s, int mode = MODE_RUN) {
  if (op.kind == OP_ABSMAX && mode != MODE_CALIBRATE) return QX_OK;
  const bool cal = mode == MODE_CALIBRATE;
  const bool outb = op.out >= 0 ? p->pc.tensors[op.out].batched : false;
  const double scale = outb ? (double)B / p->pc.max_b : 1.0;
  hipError_t e = timed(p, op_class(op.kind), op.flops * scale, op.bytes * scale, s, [&]() -> hipError_t {
  switch (op.kind) {
    case OP_SIMT: {
      SimtArgs a = op.simt;
      if (outb) a.n_items = B;
      if (cal) a.c_split = 0;
      return launch_simt(a, s);
    }
    case OP_GEMM: {
      GemmArgs g = op.gemm;
      if (outb) g.n_items = B;
      if (cal) {
        g.a_split = g.b_split = g.c_split = 0;
        g.a_scale = g.b_scale = g.c_scale = nullptr;
        return launch_gemm(g, QX_C64, op.tile, s);
      }
      return launch_gemm(g, p->pc.precision, op.tile, s);
    }
    case OP_DOT: {
      DotArgs d = op.dot;
      if (outb) d.n_items = B;
      if (cal) d.c_split = 0;
      return launch_dot(d, s);
    }
    case OP_ABSMAX: {
      AbsmaxArgs m = op.absmax;
      const Tensor& t = p->pc.tensors[op.in_a];
      m.n = t.elems() * (t.batched ? B : 1);
      return launch_absmax(m, s);
    }
    case OP_PERM: {
      PermArgs q = op.perm;
      if (outb) q.n_items = B;
      return launch_permute(q, s);
    }
  }
  return hipErrorInvalidValue;
  });
  if (e != hipSuccess) return fail(QX_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return QX_OK;
}

// Estimated seconds for a whole slice range: matrix-core work, plus a launch cost per op
// (magnitude reductions only run at plan creation).
static double est_cost(const PlanCore& pc) {
  const double blocks = std::ldexp(1.0, pc.n_sliced - pc.js);
  const double flops = pc.flops_block * blocks + pc.flops_call;
  int n_block = 0, n_call = 0;
  for (const Op& o : pc.ops)
    if (o.kind != OP_ABSMAX) {
      if (o.phase == PH_BLOCK) ++n_block;
      else if (o.phase == PH_CALL) ++n_call;
    }
  return flops / 60e12 + blocks * (n_block + 1) * 6e-6 + n_call * 6e-6;
}

// One slice block: take the next block, run the block ops, add its slices'
// values into the plan's FP64 accumulator.  Reads the block from device state
// only, so the same launches can be captured once and replayed per block.
static qx_status run_block(qx_plan* p, int B, hipStream_t s, int mode = MODE_RUN) {
  const PlanCore& pc = p->pc;
  BlockArgs ba;
  std::memset(&ba, 0, sizeof(ba));
  ba.state = p->d_state;
  ba.acc = reinterpret_cast<double*>(p->d_state + 8);
  ba.n_items = B;
  hipError_t e = timed(p, QX_OPCLASS_SLICESUM, 0.0, 0.0, s, [&] { return launch_block_advance(ba, s); });
  if (e != hipSuccess) return fail(QX_ERR_HIP, std::string("block advance launch: ") + hipGetErrorString(e));
  for (int i = pc.n_const + pc.n_call; i < (int)pc.ops.size(); ++i) {
    qx_status r = run_op(p, pc.ops[i], B, s, mode);
    if (r != QX_OK) return r;
  }
  const Tensor& rt = pc.tensors[pc.root];
  SliceSumArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.root = tensor_ptr(p, pc.root);
  sa.block = p->d_state;
  sa.root_item = rt.batched ? rt.elems() : 0;
  sa.root_gather = gather_ptr(p, pc.root_gather);
  sa.amp = ba.acc;
  sa.n_items = B << pc.n_open;
  sa.n_sbits = pc.js;
  for (int j = 0; j < pc.js; ++j) sa.s_stride[j] = pc.root_sstride[j];
  sa.n_obits = pc.n_open;
  for (int i = 0; i < pc.n_open; ++i) sa.o_stride[i] = pc.root_ostride[i];
  const double sbytes = (8.0 * std::ldexp(1.0, pc.js) + 32.0) * ((int64_t)B << pc.n_open);
  e = timed(p, QX_OPCLASS_SLICESUM, 0.0, sbytes, s, [&] { return launch_slice_sum(sa, s); });
  if (e != hipSuccess) return fail(QX_ERR_HIP, std::string("slice-sum launch: ") + hipGetErrorString(e));
  return QX_OK;
}

// Per-bitstring offsets of every output closure (one gather per OPEN -> BATCHED edge).
static qx_status run_gathers(qx_plan* p, const uint64_t* d_bitstrings, int B, hipStream_t s) {
  const PlanCore& pc = p->pc;
  for (size_t g = 0; g < pc.gathers.size(); ++g) {
    const GatherDesc& gd = pc.gathers[g];
    GatherArgs ga;
    std::memset(&ga, 0, sizeof(ga));
    ga.x = d_bitstrings;
    ga.out = p->d_gather + (int64_t)g * pc.max_b;
    ga.n_items = B;
    ga.n_q = (int)gd.q.size();
    for (size_t j = 0; j < gd.q.size(); ++j) {
      ga.q[j] = gd.q[j];
      ga.stride[j] = gd.stride[j];
    }
    hipError_t e = timed(p, QX_OPCLASS_GATHER, 0.0, 16.0 * B, s, [&] { return launch_gather(ga, s); });
    if (e != hipSuccess) return fail(QX_ERR_HIP, std::string("gather launch: ") + hipGetErrorString(e));
  }
  return QX_OK;
}

// Calibration passes of a split FP16 plan and the bitstrings they use: SplitMix64
// (Steele, Lea and Flood, 2014) of the pass and item, cut to the circuit's qubits.
constexpr int FP16_CAL_PASSES = 4;
static uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// Split FP16 plans: fixes every split tensor's power-of-two scale from complex64
// passes (plan-time ops once; then, per pass, the per-call ops and one slice
// block for max_bitstrings pseudo-random bitstrings, the passes spread over the
// slice blocks), then rewrites the split leaves in split FP16 form and recomputes
// the plan-time ops in it.  A tensor's scale follows the largest magnitude it
// held in any pass.  Bitstrings matter: the two-qubit gates of the random
// circuits keep many tensor entries exactly zero, so one fixed bitstring can
// leave whole batched tensors zero.  Later calls reuse the scales: a value more
// than about 1000 times the largest its tensor held in calibration would overflow
// FP16 and make the amplitudes it reaches non-finite.
static qx_status calibrate_fp16(qx_plan* p, hipStream_t s) {
  const PlanCore& pc = p->pc;
  for (int i = 0; i < pc.n_const; ++i) {
    const qx_status r = run_op(p, pc.ops[i], 1, s, MODE_CALIBRATE);
    if (r != QX_OK) return r;
  }
  const int nq = pc.n_qubits;
  const uint64_t qmask = nq >= 64 ? ~0ULL : ((1ULL << nq) - 1);
  std::vector<uint64_t> bits((size_t)FP16_CAL_PASSES * pc.max_b);
  for (size_t i = 0; i < bits.size(); ++i) bits[i] = splitmix64(0x51ce0000ULL + i) & qmask;
  uint64_t* d_bits = nullptr;
  HIP_TRY(hipMalloc((void**)&d_bits, bits.size() * sizeof(uint64_t)));
  struct Free {
    uint64_t* q;
    ~Free() { hipFree(q); }
  } free_bits{d_bits};
  HIP_TRY(hipMemcpyAsync(d_bits, bits.data(), bits.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  const int64_t n_blocks = (int64_t)1 << (pc.n_sliced - pc.js);
  for (int pass = 0; pass < FP16_CAL_PASSES; ++pass) {
    qx_status r = run_gathers(p, d_bits + (size_t)pass * pc.max_b, pc.max_b, s);
    if (r != QX_OK) return r;
    const int64_t blk = pass * n_blocks / FP16_CAL_PASSES;
    BlockArgs ba;
    std::memset(&ba, 0, sizeof(ba));
    ba.state = p->d_state;
    ba.acc = reinterpret_cast<double*>(p->d_state + 8);
    ba.first_block = blk;
    ba.slice_begin = blk << pc.js;
    ba.slice_end = (blk + 1) << pc.js;
    ba.js = pc.js;
    ba.n_items = pc.max_b << pc.n_open;
    HIP_TRY(launch_block_init(ba, s));
    for (int i = pc.n_const; i < pc.n_const + pc.n_call; ++i) {
      r = run_op(p, pc.ops[i], pc.max_b, s, MODE_CALIBRATE);
      if (r != QX_OK) return r;
    }
    r = run_block(p, pc.max_b, s, MODE_CALIBRATE);
    if (r != QX_OK) return r;
  }
  ScaleFromMaxArgs sa{scale_ptr(p, 0), pc.n_scale_slots, FP16_TARGET_EXP};
  HIP_TRY(launch_scale_from_max(sa, s));
  for (const Tensor& t : pc.tensors)
    if (t.is_leaf && t.split) {
      SplitInplaceArgs a{p->d_leaves + t.leaf_off, t.elems(), scale_ptr(p, t.scale_slot)};
      HIP_TRY(launch_split_inplace(a, s));
    }
  for (int i = 0; i < pc.n_const; ++i) {
    const qx_status r = run_op(p, pc.ops[i], 1, s);
    if (r != QX_OK) return r;
  }
  // the bitstring buffer is freed on return: wait for the passes that read it
  HIP_TRY(hipStreamSynchronize(s));
  return QX_OK;
}

// Tile autotuner: times every tile shape that fits a product and keeps the
// fastest; results are cached per (precision, shape, batch, operand modes).
struct TileKey {
  int prec, nh, items, akc, bkc;
  int64_t M, N, K;
  bool operator<(const TileKey& o) const {
    return std::tie(prec, nh, items, akc, bkc, M, N, K) < std::tie(o.prec, o.nh, o.items, o.akc, o.bkc, o.M, o.N, o.K);
  }
};
static std::mutex g_tune_mu;
static std::map<TileKey, int> g_tune_cache;

static qx_status autotune_plan(qx_plan* p, hipStream_t s) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  for (int i = p->pc.n_const; i < (int)p->pc.ops.size(); ++i) {
    Op& op = p->pc.ops[i];
    if (op.kind != OP_GEMM) continue;
    const GemmArgs& g = op.gemm;
    const TileKey key{p->pc.precision, g.nh, g.n_items, g.a_kc, g.b_kc, g.M, g.N, g.K};
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        op.tile = it->second;
        continue;
      }
    }
    // candidate shapes: one untimed warm-up each, then rounds that time every candidate once, in turn,
    // so clock drift affects them alike; at least 2 rounds, up to 5 while a round stays short.  Keep the
    // shape with the smallest time.
    std::vector<int> cand;
    for (int t = 0; t < GEMM_N_TILES; ++t) {
      if (gemm_tile_pipelined(t) && p->pc.precision == QX_C64) continue;  // same kernel as the plain shape
      if (t == GEMM_TILE_THIN) {
        if (gemm_thin_fits(g)) cand.push_back(t);
        continue;
      }
      if (p->pc.precision != QX_C64 && !gemm_split_k_ok(g)) continue;  // such a product runs thin
      int bm, bn;
      gemm_tile_dims(t, bm, bn);
      if (bm <= std::max<int64_t>(64, g.M) && bn <= std::max<int64_t>(64, g.N)) cand.push_back(t);
    }
    int best = op.tile;
    if (!cand.empty()) {
      std::vector<float> ms_min(cand.size(), 1e30f);
      float round_ms = 0.f;
      for (size_t c = 0; c < cand.size(); ++c) {
        HIP_TRY(hipEventRecord(e0, s));
        HIP_TRY(launch_gemm(g, p->pc.precision, cand[c], s));
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        round_ms += ms;
      }
      const int rounds = std::max(2, std::min(5, (int)(200.f / std::max(round_ms, 1e-3f))));
      for (int r = 0; r < rounds; ++r)
        for (size_t c = 0; c < cand.size(); ++c) {
          HIP_TRY(hipEventRecord(e0, s));
          HIP_TRY(launch_gemm(g, p->pc.precision, cand[c], s));
          HIP_TRY(hipEventRecord(e1, s));
          HIP_TRY(hipEventSynchronize(e1));
          float ms = 0.f;
          HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
          ms_min[c] = std::min(ms_min[c], ms);
        }
      size_t bi = 0;
      for (size_t c = 1; c < cand.size(); ++c)
        if (ms_min[c] < ms_min[bi]) bi = c;
      best = cand[bi];
      if (getenv("QX_DUMP_TUNE")) {
        fprintf(stderr, "tune prec %d M %lld N %lld K %lld items %d nh %d:", p->pc.precision, (long long)g.M,
                (long long)g.N, (long long)g.K, g.n_items, g.nh);
        for (size_t c = 0; c < cand.size(); ++c) fprintf(stderr, " t%d=%.3f", cand[c], ms_min[c]);
        fprintf(stderr, " -> %d\n", best);
      }
    }
    op.tile = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return QX_OK;
}

static qx_status contract_enqueue(qx_plan* p, const uint64_t* d_bitstrings, int32_t B, int64_t slice_begin,
                                  int64_t slice_end, double* d_amplitudes, hipStream_t s);

extern "C" {

const char* qx_last_error(void) { return g_err.c_str(); }

qx_status qx_plan_create(const qx_network* net, const int32_t* tree, const int64_t* sliced,
                         int32_t n_sliced, const qx_plan_options* opt_in, void* stream,
                         qx_plan** out) {
  g_err.clear();
  if (!out) return fail(QX_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!net) return fail(QX_ERR_INVALID_ARG, "net is NULL");
  if (net->n_tensors < 1) return fail(QX_ERR_INVALID_NETWORK, "network has no tensors");
  if (!net->index_ptr || !net->data_ptr || !net->data) return fail(QX_ERR_INVALID_ARG, "network arrays are NULL");
  if (net->index_ptr[net->n_tensors] > 0 && !net->index_ids) return fail(QX_ERR_INVALID_ARG, "index_ids is NULL");
  if (net->n_qubits < 0 || net->n_qubits > 64) return fail(QX_ERR_UNSUPPORTED, "n_qubits must be in 0..64");
  if (net->n_qubits > 0 && !net->output_index) return fail(QX_ERR_INVALID_ARG, "output_index is NULL");
  if (net->n_tensors > 1 && !tree) return fail(QX_ERR_INVALID_ARG, "tree is NULL");
  if (n_sliced < 0 || n_sliced > 40) return fail(QX_ERR_UNSUPPORTED, "n_sliced must be in 0..40");
  if (n_sliced > 0 && !sliced) return fail(QX_ERR_INVALID_ARG, "sliced is NULL");
  for (int t = 0; t < net->n_tensors; ++t) {
    const int64_t r = net->index_ptr[t + 1] - net->index_ptr[t];
    if (r < 0 || r > 40) return fail(QX_ERR_UNSUPPORTED, "tensor rank must be in 0..40");
  }
  qx_plan_options opt;
  std::memset(&opt, 0, sizeof(opt));
  opt.precision = QX_C64;
  opt.max_bitstrings = 1;
  opt.slice_batch_log2 = -1;
  if (opt_in) opt = *opt_in;
  if (opt.gemm_tile < 0 || opt.gemm_tile > GEMM_N_TILES)
    return fail(QX_ERR_INVALID_ARG, "gemm_tile must be 0 (automatic) or 1..9 (tile + 1)");
  if (opt.reserved_ != 0) return fail(QX_ERR_INVALID_ARG, "reserved_ must be 0");
  if (opt.precision < QX_C64 || opt.precision > QX_SPLIT_FP16)
    return fail(QX_ERR_INVALID_ARG, "unknown precision");
  if (opt.max_bitstrings < 1 || opt.max_bitstrings > (1 << 20))
    return fail(QX_ERR_INVALID_ARG, "max_bitstrings must be in 1..2^20");
  if (opt.slice_batch_log2 < -1 || opt.slice_batch_log2 > std::min(n_sliced, QX_MAX_SBITS))
    return fail(QX_ERR_INVALID_ARG, "slice_batch_log2 must be -1 or in 0..min(n_sliced, 24)");
  if (opt.hbm_budget_bytes < 0) return fail(QX_ERR_INVALID_ARG, "hbm_budget_bytes < 0");
  if (net->n_qubits < 64 && (opt.open_qubits >> net->n_qubits) != 0)
    return fail(QX_ERR_INVALID_ARG, "open_qubits names a qubit >= n_qubits");
  const int n_open = __builtin_popcountll(opt.open_qubits);
  if (n_open > QX_MAX_OBITS) return fail(QX_ERR_UNSUPPORTED, "at most 16 open qubits");
  if (((int64_t)opt.max_bitstrings << n_open) > ((int64_t)1 << 24))
    return fail(QX_ERR_UNSUPPORTED, "max_bitstrings * 2^(open qubits) must be <= 2^24");

  qx_plan* p = new (std::nothrow) qx_plan();
  if (!p) return fail(QX_ERR_INVALID_ARG, "out of host memory");
  std::string err;
  qx_status st;
  if (opt.slice_batch_log2 >= 0) {
    st = compile_plan(net, tree, sliced, n_sliced, opt, opt.slice_batch_log2, p->pc, err);
  } else {
    int64_t limit = opt.hbm_budget_bytes > 0 ? opt.hbm_budget_bytes : (int64_t)96 << 30;
    if (opt.hbm_budget_bytes <= 0 && !opt.dry_run) {
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) limit = std::min<int64_t>(limit, (int64_t)(0.8 * free_b));
    }
    double best = 1e300;
    int best_js = -1;
    st = QX_OK;
    for (int js = 0; js <= std::min(n_sliced, 8); ++js) {
      PlanCore cand;
      st = compile_plan(net, tree, sliced, n_sliced, opt, js, cand, err);
      if (st != QX_OK) break;
      if (plan_device_bytes(cand) > limit && js > 0) continue;
      const double c = est_cost(cand);
      if (c < best * 0.97 || best_js < 0) {
        best = c;
        best_js = js;
      }
    }
    if (st == QX_OK) st = compile_plan(net, tree, sliced, n_sliced, opt, best_js < 0 ? 0 : best_js, p->pc, err);
  }
  if (st != QX_OK) {
    delete p;
    return fail(st, err);
  }
  p->device_bytes = plan_device_bytes(p->pc);
  if (opt.hbm_budget_bytes > 0 && p->device_bytes > opt.hbm_budget_bytes) {
    const int64_t need = p->device_bytes;
    delete p;
    return fail(QX_ERR_OUT_OF_BUDGET, "plan needs " + std::to_string(need) + " device bytes, budget is " +
                                          std::to_string(opt.hbm_budget_bytes));
  }
  p->dry = opt.dry_run != 0;
  p->eager = opt.eager != 0;
  if (opt.gemm_tile > 0)
    for (Op& op : p->pc.ops)
      if (op.kind == OP_GEMM) op.tile = opt.gemm_tile - 1;
  {
    const int n = net->n_tensors;
    p->net_index_ptr.resize(n + 1);
    p->net_data_ptr.resize(n + 1);
    for (int t = 0; t <= n; ++t) {
      p->net_index_ptr[t] = net->index_ptr[t] - net->index_ptr[0];
      p->net_data_ptr[t] = net->data_ptr[t] - net->data_ptr[0];
    }
    p->net_index_ids.assign(net->index_ids + net->index_ptr[0], net->index_ids + net->index_ptr[n]);
    p->net_n_qubits = net->n_qubits;
    p->net_output.assign(net->output_index, net->output_index + net->n_qubits);
    if (n > 1) p->tree.assign(tree, tree + 2 * (n - 1));
    p->sliced.assign(sliced, sliced + n_sliced);
    p->opt = opt;
  }
  for (const Op& op : p->pc.ops)
    if (op.kind != OP_SIMT && (!op.fix_a.empty() || !op.fix_b.empty())) {
      delete p;
      return fail(QX_ERR_INVALID_TREE, "internal: fixed sliced index on a non-small contraction");
    } else if (op.fix_a.size() > 4 || op.fix_b.size() > 4) {
      delete p;
      return fail(QX_ERR_UNSUPPORTED, "a leaf carries more than 4 sliced indices");
    }
  if (!p->dry) {
    hipStream_t s = (hipStream_t)stream;
    auto cleanup = [&](qx_status code, const std::string& m) {
      qx_plan_destroy(p);
      return fail(code, m);
    };
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) return cleanup(QX_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    const int64_t leaf_bytes = std::max<int64_t>(256, p->pc.leaf_pool_elems * 8);
    if ((e = hipMalloc((void**)&p->d_leaves, leaf_bytes)) != hipSuccess)
      return cleanup(QX_ERR_HIP, std::string("hipMalloc(leaves): ") + hipGetErrorString(e));
    if ((e = hipMalloc((void**)&p->d_arena, std::max<int64_t>(256, p->pc.arena_bytes))) != hipSuccess)
      return cleanup(QX_ERR_HIP, std::string("hipMalloc(arena): ") + hipGetErrorString(e));
    if ((e = hipMalloc((void**)&p->d_state, state_bytes(p->pc))) != hipSuccess)
      return cleanup(QX_ERR_HIP, std::string("hipMalloc(state): ") + hipGetErrorString(e));
    if ((e = hipMemsetAsync(p->d_state, 0, state_bytes(p->pc), s)) != hipSuccess)
      return cleanup(QX_ERR_HIP, std::string("hipMemsetAsync(state): ") + hipGetErrorString(e));
    if ((e = hipMalloc((void**)&p->d_misc, misc_bytes(p->pc))) != hipSuccess)
      return cleanup(QX_ERR_HIP, std::string("hipMalloc(misc): ") + hipGetErrorString(e));
    if ((e = hipMemsetAsync(p->d_misc, 0, misc_bytes(p->pc), s)) != hipSuccess)
      return cleanup(QX_ERR_HIP, std::string("hipMemsetAsync(misc): ") + hipGetErrorString(e));
    const int64_t gb = std::max<int64_t>(256, (int64_t)p->pc.gathers.size() * p->pc.max_b * 8);
    if ((e = hipMalloc((void**)&p->d_gather, gb)) != hipSuccess)
      return cleanup(QX_ERR_HIP, std::string("hipMalloc(gather): ") + hipGetErrorString(e));
    // leaves: complex128 -> complex64, round to nearest even; a leaf read by a split-BF16
    // product holds its split BF16 form (64-byte chunks of 8 elements: hi re, lo re,
    // hi im, lo im) in the same bytes
    std::vector<float> h(2 * p->pc.leaf_pool_elems);
    for (size_t i = 0; i < h.size(); ++i) h[i] = (float)p->pc.leaf_data[i];
    for (const Tensor& t : p->pc.tensors) {
      if (!t.is_leaf || !t.split || p->pc.precision != QX_SPLIT_BF16) continue;
      const int64_t E = t.elems();
      std::vector<uint16_t> planes(4 * E);
      for (int64_t e = 0; e < E; ++e) {
        const float re = h[2 * (t.leaf_off + e)], im = h[2 * (t.leaf_off + e) + 1];
        const uint16_t rh = bf16_rne(re), ih = bf16_rne(im);
        planes[split_off(e, 0)] = rh;
        planes[split_off(e, 1)] = bf16_rne(re - bf16_float(rh));
        planes[split_off(e, 2)] = ih;
        planes[split_off(e, 3)] = bf16_rne(im - bf16_float(ih));
      }
      std::memcpy(&h[2 * t.leaf_off], planes.data(), planes.size() * sizeof(uint16_t));
    }
    if ((e = hipMemcpyAsync(p->d_leaves, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
      return cleanup(QX_ERR_HIP, std::string("hipMemcpyAsync(leaves): ") + hipGetErrorString(e));
    resolve_pointers(p);
    if (p->pc.precision == QX_SPLIT_FP16) {
      qx_status r = calibrate_fp16(p, s);
      if (r != QX_OK) {
        std::string m = g_err;
        return cleanup(r, m);
      }
    } else {
      for (int i = 0; i < p->pc.n_const; ++i) {
        qx_status r = run_op(p, p->pc.ops[i], 1, s);
        if (r != QX_OK) {
          std::string m = g_err;
          return cleanup(r, m);
        }
      }
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess)
      return cleanup(QX_ERR_HIP, std::string("plan pre-contraction: ") + hipGetErrorString(e));
    if ((e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming)) != hipSuccess)
      return cleanup(QX_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
    if (opt.autotune && opt.gemm_tile == 0) {
      // gather offsets of zero keep every timing launch's reads inside its operands
      if ((e = hipMemsetAsync(p->d_gather, 0, gb, s)) != hipSuccess)
        return cleanup(QX_ERR_HIP, std::string("hipMemsetAsync(gather): ") + hipGetErrorString(e));
      qx_status r = autotune_plan(p, s);
      if (r != QX_OK) {
        std::string m = g_err;
        return cleanup(r, m);
      }
    }
  }
  *out = p;
  return QX_OK;
}

qx_status qx_plan_get_info(const qx_plan* p, qx_plan_info* info) {
  g_err.clear();
  if (!p || !info) return fail(QX_ERR_INVALID_ARG, "NULL argument");
  const PlanCore& pc = p->pc;
  std::memset(info, 0, sizeof(*info));
  info->device_bytes = p->device_bytes;
  info->arena_bytes = pc.arena_bytes;
  info->n_leaves = pc.n_leaves;
  info->n_sliced = pc.n_sliced;
  info->slice_batch_log2 = pc.js;
  info->width = pc.width;
  info->n_ops_const = pc.n_const;
  info->n_ops_call = pc.n_call;
  info->n_ops_block = pc.n_block;
  info->n_gemm_block = pc.n_gemm_block;
  info->flops_per_slice = pc.flops_per_slice;
  info->flops_block = pc.flops_block;
  info->gemm_flops_block = pc.gemm_flops_block;
  info->flops_call = pc.flops_call;
  info->n_open = pc.n_open;
  info->reserved = 0;
  return QX_OK;
}

qx_status qx_plan_get_op_info(const qx_plan* p, int32_t index, qx_op_info* info) {
  g_err.clear();
  if (!p || !info) return fail(QX_ERR_INVALID_ARG, "NULL argument");
  if (index < 0 || index >= (int32_t)p->pc.ops.size()) return fail(QX_ERR_INVALID_ARG, "op index out of range");
  const Op& op = p->pc.ops[index];
  std::memset(info, 0, sizeof(*info));
  info->phase = op.phase;
  info->op_class = op_class(op.kind);
  info->tile = -1;
  info->flops = op.flops;
  info->bytes = op.bytes;
  info->batched = op.out >= 0 && p->pc.tensors[op.out].batched ? 1 : 0;
  switch (op.kind) {
    case OP_GEMM:
      info->M = op.gemm.M; info->N = op.gemm.N; info->K = op.gemm.K;
      info->batch = (int64_t)op.gemm.n_items << op.gemm.nh;
      info->tile = op.tile;
      break;
    case OP_SIMT:
      info->M = (int64_t)1 << op.simt.n_out; info->N = 1; info->K = (int64_t)1 << op.simt.n_k;
      info->batch = op.simt.n_items;
      break;
    case OP_DOT:
      info->M = (int64_t)1 << op.dot.n_out; info->N = 1; info->K = op.dot.K;
      info->batch = op.dot.n_items;
      break;
    case OP_PERM:
      info->M = (int64_t)1 << op.perm.rank; info->N = 1; info->K = 1;
      info->batch = op.perm.n_items;
      break;
    default: {
      const Tensor& t = p->pc.tensors[op.in_a];
      info->M = t.elems(); info->N = 1; info->K = 1;
      info->batch = t.batched ? p->pc.max_b : 1;
      info->batched = t.batched ? 1 : 0;
    }
  }
  return QX_OK;
}

qx_status qx_plan_peak_bytes(const qx_plan* p, int32_t n_bitstrings, int32_t slice_batch_log2, int64_t* bytes) {
  g_err.clear();
  if (!p || !bytes) return fail(QX_ERR_INVALID_ARG, "NULL argument");
  const int B = n_bitstrings == 0 ? p->pc.max_b : n_bitstrings;
  if (B < 1 || B > (1 << 20)) return fail(QX_ERR_INVALID_ARG, "n_bitstrings must be 0 or in 1..2^20");
  if (((int64_t)B << p->pc.n_open) > ((int64_t)1 << 24))
    return fail(QX_ERR_INVALID_ARG, "n_bitstrings * 2^(open qubits) must be <= 2^24");
  const int js = slice_batch_log2 < 0 ? p->pc.js : slice_batch_log2;
  if (slice_batch_log2 < -1 || js > std::min(p->pc.n_sliced, QX_MAX_SBITS))
    return fail(QX_ERR_INVALID_ARG, "slice_batch_log2 must be -1 or in 0..min(n_sliced, 24)");
  if (B == p->pc.max_b && js == p->pc.js) {
    *bytes = p->device_bytes;
    return QX_OK;
  }
  qx_network net;
  net.n_tensors = p->pc.n_leaves;
  net.index_ptr = p->net_index_ptr.data();
  net.index_ids = p->net_index_ids.data();
  net.data_ptr = p->net_data_ptr.data();
  net.data = p->pc.leaf_data.data();
  net.n_qubits = p->net_n_qubits;
  net.output_index = p->net_output.data();
  qx_plan_options opt = p->opt;
  opt.max_bitstrings = B;
  PlanCore pc;
  std::string err;
  const qx_status st = compile_plan(&net, p->tree.empty() ? nullptr : p->tree.data(), p->sliced.data(),
                                    (int32_t)p->sliced.size(), opt, js, pc, err);
  if (st != QX_OK) return fail(st, err);
  *bytes = plan_device_bytes(pc);
  return QX_OK;
}

qx_status qx_contract(qx_plan* p, const uint64_t* d_bitstrings, int32_t B, int64_t slice_begin,
                      int64_t slice_end, double* d_amplitudes, void* stream) {
  g_err.clear();
  if (!p) return fail(QX_ERR_INVALID_ARG, "plan is NULL");
  const PlanCore& pc = p->pc;
  if (B < 1 || B > pc.max_b)
    return fail(QX_ERR_INVALID_ARG, "B must be in 1..max_bitstrings (" + std::to_string(pc.max_b) + ")");
  const int64_t nsl = (int64_t)1 << pc.n_sliced;
  if (slice_begin < 0 || slice_end < slice_begin || slice_end > nsl)
    return fail(QX_ERR_INVALID_ARG, "slice range must satisfy 0 <= begin <= end <= 2^n_sliced");
  if (!d_amplitudes) return fail(QX_ERR_INVALID_ARG, "d_amplitudes is NULL");
  if (!d_bitstrings) return fail(QX_ERR_INVALID_ARG, "d_bitstrings is NULL");
  if (p->dry) return fail(QX_ERR_DRY_RUN, "plan was compiled with dry_run");
  if (slice_begin == slice_end) return QX_OK;
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != p->device) return fail(QX_ERR_INVALID_ARG, "current device differs from the plan's device");
  hipStream_t s = (hipStream_t)stream;
  const qx_status st = contract_enqueue(p, d_bitstrings, B, slice_begin, slice_end, d_amplitudes, s);
  // whatever was enqueued, qx_plan_destroy waits for it through this event
  const hipError_t e = hipEventRecord(p->done, s);
  if (st == QX_OK && e != hipSuccess) return fail(QX_ERR_HIP, std::string("hipEventRecord: ") + hipGetErrorString(e));
  return st;
}

}  // extern "C"

// Enqueues one validated qx_contract call on stream s.
static qx_status contract_enqueue(qx_plan* p, const uint64_t* d_bitstrings, int32_t B, int64_t slice_begin,
                                  int64_t slice_end, double* d_amplitudes, hipStream_t s) {
  const PlanCore& pc = p->pc;
  qx_status r0 = run_gathers(p, d_bitstrings, B, s);
  if (r0 != QX_OK) return r0;
  for (int i = pc.n_const; i < pc.n_const + pc.n_call; ++i) {
    qx_status r = run_op(p, pc.ops[i], B, s);
    if (r != QX_OK) return r;
  }
  const int64_t first = slice_begin >> pc.js, last = (slice_end - 1) >> pc.js;
  BlockArgs ba;
  std::memset(&ba, 0, sizeof(ba));
  ba.state = p->d_state;
  ba.acc = reinterpret_cast<double*>(p->d_state + 8);
  ba.first_block = first;
  ba.slice_begin = slice_begin;
  ba.slice_end = slice_end;
  ba.js = pc.js;
  ba.n_items = B << pc.n_open;  // accumulated values
  HIP_TRY(launch_block_init(ba, s));
  const bool use_graph = !p->eager && !p->timing && last > first;
  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    auto it = p->graphs.find(B);
    if (it == p->graphs.end()) {
      if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
      HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
      qx_status r = run_block(p, B, p->cap_stream);
      hipGraph_t graph = nullptr;
      hipError_t ce = hipStreamEndCapture(p->cap_stream, &graph);
      if (r != QX_OK) {
        if (graph) hipGraphDestroy(graph);
        return r;
      }
      if (ce != hipSuccess) return fail(QX_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
      hipGraphExec_t ge = nullptr;
      hipError_t ie = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        hipGraphDestroy(graph);
        return fail(QX_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
      }
      it = p->graphs.emplace(B, std::make_pair(graph, ge)).first;
    }
    exec = it->second.second;
  }
  for (int64_t bb = first; bb <= last; ++bb) {
    if (exec) {
      HIP_TRY(hipGraphLaunch(exec, s));
    } else {
      qx_status r = run_block(p, B, s);
      if (r != QX_OK) return r;
    }
  }
  HIP_TRY(launch_block_finish(ba, d_amplitudes, s));
  return QX_OK;
}

extern "C" {

qx_status qx_plan_set_timing(qx_plan* p, int32_t enable) {
  g_err.clear();
  if (!p) return fail(QX_ERR_INVALID_ARG, "plan is NULL");
  if (p->dry && enable) return fail(QX_ERR_DRY_RUN, "plan was compiled with dry_run");
  p->timing = enable != 0;
  return QX_OK;
}

qx_status qx_plan_get_timing(qx_plan* p, qx_op_timing* out, int32_t reset) {
  g_err.clear();
  if (!p || !out) return fail(QX_ERR_INVALID_ARG, "NULL argument");
  for (PendingEvent& ev : p->pending) {
    HIP_TRY(hipEventSynchronize(ev.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
    qx_op_timing& t = p->acc[ev.cls];
    t.launches += 1;
    t.seconds += ms * 1e-3;
    t.flops += ev.flops;
    t.bytes += ev.bytes;
    p->pool.push_back(ev.a);
    p->pool.push_back(ev.b);
  }
  p->pending.clear();
  for (int i = 0; i < QX_N_OPCLASS; ++i) out[i] = p->acc[i];
  if (reset) std::memset(p->acc, 0, sizeof(p->acc));
  return QX_OK;
}

void qx_plan_destroy(qx_plan* p) {
  if (!p) return;
  if (!p->dry) {
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(p->device);
    // the plan's own work only: the last contract call (or the creation) recorded p->done
    if (p->done) hipEventSynchronize(p->done);
    if (p->cap_stream) hipStreamSynchronize(p->cap_stream);
    for (PendingEvent& ev : p->pending) {
      hipEventDestroy(ev.a);
      hipEventDestroy(ev.b);
    }
    for (hipEvent_t e : p->pool) hipEventDestroy(e);
    if (p->d_leaves) hipFree(p->d_leaves);
    if (p->d_arena) hipFree(p->d_arena);
    if (p->d_gather) hipFree(p->d_gather);
    if (p->d_misc) hipFree(p->d_misc);
    if (p->d_state) hipFree(p->d_state);
    for (auto& kv : p->graphs) {
      hipGraphExecDestroy(kv.second.second);
      hipGraphDestroy(kv.second.first);
    }
    if (p->cap_stream) hipStreamDestroy(p->cap_stream);
    if (p->done) hipEventDestroy(p->done);
    hipSetDevice(cur);
  }
  delete p;
}

qx_status qx_permute_c64(const void* d_in, void* d_out, int32_t rank, const int32_t* in_pos, int64_t items,
                         void* stream) {
  g_err.clear();
  if (!d_in || !d_out || !in_pos) return fail(QX_ERR_INVALID_ARG, "NULL argument");
  if (rank < 0 || rank > 40) return fail(QX_ERR_UNSUPPORTED, "rank must be in 0..40");
  if (items < 0 || items > 65535) return fail(QX_ERR_INVALID_ARG, "items must be in 0..65535");
  uint64_t seen = 0;
  for (int i = 0; i < rank; ++i) {
    if (in_pos[i] < 0 || in_pos[i] >= rank || ((seen >> in_pos[i]) & 1))
      return fail(QX_ERR_INVALID_ARG, "in_pos is not a permutation of 0..rank-1");
    seen |= 1ULL << in_pos[i];
  }
  if (items == 0) return QX_OK;
  PermArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = (const QxCplx*)d_in;
  a.out = (QxCplx*)d_out;
  a.rank = rank;
  a.n_items = (int)items;
  a.in_item = a.out_item = (int64_t)1 << rank;
  for (int i = 0; i < rank; ++i) a.in_pos[i] = in_pos[i];
  permute_setup(a);
  HIP_TRY(launch_permute(a, (hipStream_t)stream));
  return QX_OK;
}

// Shared by qx_cgemm and qx_cgemm_noalloc.  Split precision splits A and B into
// temporaries first: in `scratch` when given (it holds at least
// cgemm_split_bytes(...) bytes), else in stream-ordered allocations.
static int64_t cgemm_split_bytes(int64_t M, int64_t N, int64_t K, int64_t batch) {
  const int64_t kp = (K + 15) / 16 * 16;
  return 8 * batch * (M + N) * kp;
}

static qx_status cgemm_check(const void* d_a, const void* d_b, void* d_c, int64_t M, int64_t N, int64_t K,
                             int64_t a_ms, int64_t a_ks, int64_t b_ks, int64_t b_ns, int64_t batch,
                             int32_t precision, int32_t tile_opt) {
  if (!d_a || !d_b || !d_c) return fail(QX_ERR_INVALID_ARG, "NULL argument");
  if (tile_opt < 0 || tile_opt > GEMM_N_TILES) return fail(QX_ERR_INVALID_ARG, "tile must be 0 or 1..9");
  if (M < 1 || N < 1 || K < 1 || batch < 0) return fail(QX_ERR_INVALID_ARG, "M, N, K must be >= 1, batch >= 0");
  if (!(a_ms == 1 || a_ks == 1) || !(b_ks == 1 || b_ns == 1) || a_ms < 1 || a_ks < 1 || b_ks < 1 || b_ns < 1)
    return fail(QX_ERR_INVALID_ARG, "one stride of each operand must be 1 and all strides >= 1");
  if (precision < QX_C64 || precision > QX_SPLIT_FP16) return fail(QX_ERR_INVALID_ARG, "unknown precision");
  if (batch > 0x7fffffff) return fail(QX_ERR_INVALID_ARG, "batch too large");
  return QX_OK;
}

static qx_status cgemm_run(const void* d_a, const void* d_b, void* d_c, int64_t M, int64_t N, int64_t K,
                           int64_t a_ms, int64_t a_ks, int64_t b_ks, int64_t b_ns, int64_t stride_a,
                           int64_t stride_b, int64_t stride_c, int64_t batch, int32_t precision, int32_t tile_opt,
                           hipStream_t s, uint16_t* scratch) {
  if (batch == 0) return QX_OK;
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.a = (const QxCplx*)d_a;
  g.b = (const QxCplx*)d_b;
  g.c = (QxCplx*)d_c;
  g.M = M; g.N = N; g.K = K;
  g.a_ms = a_ms; g.a_ks = a_ks; g.b_ks = b_ks; g.b_ns = b_ns; g.c_ms = N;
  g.a_item = stride_a; g.b_item = stride_b; g.c_item = stride_c;
  g.n_items = (int)batch;
  g.nh = 0;
  // 16-byte vector loads along k need even strides and an aligned base
  g.vec_a = a_ks == 1 && a_ms % 2 == 0 && stride_a % 2 == 0 && ((uintptr_t)d_a) % 16 == 0;
  g.vec_b = b_ks == 1 && b_ns % 2 == 0 && stride_b % 2 == 0 && ((uintptr_t)d_b) % 16 == 0;
  const int tile = tile_opt > 0 ? tile_opt - 1 : gemm_default_tile(M, N);
  if (precision == QX_C64) {
    gemm_args_setup(g);
    HIP_TRY(launch_gemm(g, precision, tile, s));
    return QX_OK;
  }
  // split precision: the product reads pre-split operands, so split A and B into
  // temporaries [item][row][kp] (k zero-padded to a multiple of 16) first; FP16
  // planes at unit scale
  const int64_t kp = (K + 15) / 16 * 16;
  const int64_t pa = batch * M * kp, pb = batch * N * kp;
  uint16_t *ta = scratch, *tb = scratch ? scratch + 4 * pa : nullptr;
  if (!scratch) {
    HIP_TRY(hipMallocAsync((void**)&ta, pa * 8, s));
    hipError_t e = hipMallocAsync((void**)&tb, pb * 8, s);
    if (e != hipSuccess) {
      hipFreeAsync(ta, s);
      return fail(QX_ERR_HIP, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    }
  }
  const int32_t kind = precision == QX_SPLIT_FP16 ? 2 : 1;
  SplitPlanesArgs sa{(const QxCplx*)d_a, ta, M, K, kp, a_ms, a_ks, stride_a, (int32_t)batch, kind};
  SplitPlanesArgs sb{(const QxCplx*)d_b, tb, N, K, kp, b_ns, b_ks, stride_b, (int32_t)batch, kind};
  hipError_t e = launch_split_planes(sa, s);
  if (e == hipSuccess) e = launch_split_planes(sb, s);
  if (e == hipSuccess) {
    g.a = (const QxCplx*)ta;
    g.b = (const QxCplx*)tb;
    g.K = kp;
    g.a_ms = kp; g.a_ks = 1; g.b_ns = kp; g.b_ks = 1;
    g.a_item = M * kp; g.b_item = N * kp;
    g.a_split = g.b_split = kind;
    g.vec_a = g.vec_b = 1;
    gemm_args_setup(g);
    e = launch_gemm(g, precision, tile, s);
  }
  if (!scratch) {
    hipFreeAsync(ta, s);
    hipFreeAsync(tb, s);
  }
  if (e != hipSuccess) return fail(QX_ERR_HIP, std::string("split product: ") + hipGetErrorString(e));
  return QX_OK;
}

}  // extern "C"

// Scratch of qx_cgemm_noalloc: the split operand copies of one call.  Every
// device the library runs on holds its own instance until the process ends.  Host
// code must not pass this name to a kernel (on the host it is only a stand-in
// for the symbol): the device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) uint16_t scratch[QX_CGEMM_NOALLOC_SCRATCH_BYTES / 2];

static std::mutex g_scratch_mu;
static std::map<int, uint16_t*> g_scratch;  // device -> address of its scratch

// Address of the current device's scratch, looked up on the first call made
// with that device current.
static qx_status noalloc_scratch(uint16_t** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(QX_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = g_scratch.emplace(dev, static_cast<uint16_t*>(ptr)).first;
  }
  *out = it->second;
  return QX_OK;
}

extern "C" {

qx_status qx_cgemm_noalloc(const void* d_a, const void* d_b, void* d_c, int64_t M, int64_t N, int64_t K,
                           int64_t a_ms, int64_t a_ks, int64_t b_ks, int64_t b_ns, int64_t stride_a,
                           int64_t stride_b, int64_t stride_c, int64_t batch, int32_t precision, int32_t tile_opt,
                           void* stream) {
  g_err.clear();
  const qx_status st = cgemm_check(d_a, d_b, d_c, M, N, K, a_ms, a_ks, b_ks, b_ns, batch, precision, tile_opt);
  if (st != QX_OK) return st;
  uint16_t* scr = nullptr;
  if (precision != QX_C64 && batch > 0) {
    const double need = 8.0 * (double)batch * ((double)M + (double)N) * (double)((K + 15) / 16 * 16);
    if (need > (double)QX_CGEMM_NOALLOC_SCRATCH_BYTES)
      return fail(QX_ERR_INVALID_ARG, "split operand copies need " + std::to_string((int64_t)need) +
                                          " bytes; the allocation-free product's scratch holds " +
                                          std::to_string((int64_t)QX_CGEMM_NOALLOC_SCRATCH_BYTES));
    const qx_status sst = noalloc_scratch(&scr);
    if (sst != QX_OK) return sst;
  }
  return cgemm_run(d_a, d_b, d_c, M, N, K, a_ms, a_ks, b_ks, b_ns, stride_a, stride_b, stride_c, batch, precision,
                   tile_opt, (hipStream_t)stream, scr);
}

qx_status qx_cgemm(const void* d_a, const void* d_b, void* d_c, int64_t M, int64_t N, int64_t K, int64_t a_ms,
                   int64_t a_ks, int64_t b_ks, int64_t b_ns, int64_t stride_a, int64_t stride_b,
                   int64_t stride_c, int64_t batch, int32_t precision, int32_t tile_opt, void* stream) {
  g_err.clear();
  const qx_status st = cgemm_check(d_a, d_b, d_c, M, N, K, a_ms, a_ks, b_ks, b_ns, batch, precision, tile_opt);
  if (st != QX_OK) return st;
  return cgemm_run(d_a, d_b, d_c, M, N, K, a_ms, a_ks, b_ks, b_ns, stride_a, stride_b, stride_c, batch, precision,
                   tile_opt, (hipStream_t)stream, nullptr);
}

}  // extern "C"
