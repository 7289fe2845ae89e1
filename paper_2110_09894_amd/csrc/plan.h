// Plan compiler data structures (internal to the library).
//
// A plan turns (network, contraction tree, sliced indices) into three lists of
// device operations:
//   CONST  run once at plan creation: sub-trees that depend neither on the
//          bitstring nor on the slice block (their open output indices are kept
//          as ordinary indices, so every bitstring's variant is precomputed);
//   CALL   run once per qx_contract call: sub-trees that depend on the
//          bitstrings (carrying one copy per bitstring) but not on the block;
//   BLOCK  run once per block of 2^j consecutive slices: everything that
//          touches a sliced index fixed for the block.
// The j lowest sliced indices vary inside a block and are carried as ordinary
// indices up to the root, so one pass computes 2^j slices' values at once;
// the remaining sliced indices are fixed per block by offsetting leaf reads
// (Eq. 2).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "kargs.h"
#include "qxtn.h"

namespace qx {

enum Phase { PH_CONST = 0, PH_CALL = 1, PH_BLOCK = 2 };
enum OpKind { OP_SIMT = 0, OP_GEMM = 1, OP_DOT = 2, OP_PERM = 3, OP_ABSMAX = 4 };

struct Tensor {
  bool is_leaf = false;
  int64_t leaf_off = 0;          // complex offset in the leaf pool
  std::vector<int> lay;          // label ids, FASTEST first (lay[i] has stride 2^i)
  bool batched = false;          // one copy per bitstring
  int phase = PH_CONST;
  int64_t arena_off = -1;        // byte offset in the arena (non-leaf)
  int first_op = -1, last_op = -1;
  bool split = false;            // stored split (operand of a split-precision product)
  int scale_slot = -1;           // split FP16: slot of the tensor's power-of-two scale
  int64_t elems() const { return (int64_t)1 << lay.size(); }
};

struct FixTerm {   // offset contribution of a fixed sliced index: bit j of the block's first slice
  int j;
  int64_t stride;
};

struct Op {
  OpKind kind;
  int phase;
  int in_a = -1, in_b = -1, out = -1;  // tensor ids
  int gather_a = -1, gather_b = -1;    // gather table ids
  std::vector<FixTerm> fix_a, fix_b;
  int tile = 0;
  double flops = 0.0;                  // complex flops at max_bitstrings (8 M N K per product)
  double bytes = 0.0;                  // algorithmic HBM bytes at max_bitstrings
  SimtArgs simt;
  GemmArgs gemm;
  DotArgs dot;
  PermArgs perm;
  AbsmaxArgs absmax;
  int scale_slot = -1;                 // ABSMAX: slot written; GEMM: slot of A (B = slot + 1)
};

struct GatherDesc {
  int tensor;                          // tensor whose open output indices are gathered
  std::vector<int> q;                  // qubits
  std::vector<int64_t> stride;
};

struct PlanCore {
  // inputs (copied)
  int n_leaves = 0, n_qubits = 0, n_sliced = 0;
  int precision = QX_C64;
  int max_b = 1;
  int js = 0;                          // varying sliced indices per block
  std::vector<int64_t> label_of;       // dense label id -> user label
  std::vector<int> kind;               // per label id: 0 regular, 1 output, 2 sliced
  std::vector<int> aux;                // qubit (output) or slice index j (sliced)
  std::vector<int> open_bit;           // per label id: bit i of the open-qubit value index, or -1
  int n_open = 0;                      // open output qubits m (a regular index each, up to the root)
  std::vector<int> aux_label_id;       // dense label id of every index entry of the network
  std::vector<double> leaf_data;       // complex128 interleaved, leaf pool order
  int64_t leaf_pool_elems = 0;
  // compiled program
  std::vector<Tensor> tensors;
  std::vector<Op> ops;                 // CONST ops, then CALL ops, then BLOCK ops
  int n_const = 0, n_call = 0, n_block = 0;
  std::vector<GatherDesc> gathers;
  int root = -1;                       // tensor id of the root
  int root_gather = -1;
  std::vector<int64_t> root_sstride;   // stride of varying sliced index j in the root
  std::vector<int64_t> root_ostride;   // stride of open-qubit bit i in the root
  int64_t arena_bytes = 0;
  int width = 0;
  double flops_per_slice = 0, flops_block = 0, gemm_flops_block = 0, flops_call = 0;
  int n_gemm_block = 0;
  int n_scale_slots = 0;
};

// Host-only compilation; returns QX_OK or an error with a message.
qx_status compile_plan(const qx_network* net, const int32_t* tree, const int64_t* sliced,
                       int32_t n_sliced, const qx_plan_options& opt, int js, PlanCore& pc,
                       std::string& err);

}  // namespace qx
