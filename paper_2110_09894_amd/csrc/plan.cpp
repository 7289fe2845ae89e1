// Plan compiler: network + contraction tree + sliced indices -> device program.
//
// Sec. III-A: a network is contracted as a sequence of pairwise contractions
// along a tree; slicing fixes indices and sums the independent sliced networks
// (Eq. 2).  Sec. II: closing the output wires with a bitstring gives one
// amplitude.  Sec. IV-A: the plan (index accounting, order) is kept apart from
// the tensor primitives that execute it.
//
// Index roles.  Every label is regular (joins two tensors), an output wire
// (one tensor; closed by the bitstring) or sliced.  Sliced index j < js
// "varies": it is carried as an ordinary index up to the root, so a block of
// 2^js consecutive slices is computed in one pass.  Sliced index j >= js is
// "fixed" for the block and is applied as an offset when a leaf is read.
//
// Output wires.  A node is OPEN if 2^(number of output wires below it) <= the
// bitstring batch: its output wires are kept as ordinary indices, so one
// tensor holds every bitstring's variant.  Otherwise it is BATCHED: it holds
// one tensor per bitstring, and its open children are read at the offset the
// bitstring selects (a gather).
//
// Op classes.  A pairwise contraction with free dims M, N and contracted K
// (all powers of two) runs as
//   GEMM  complex matrix product on the matrix cores when M, N >= 16, K >= 8;
//         its operands must hold the free and contracted indices as two
//         contiguous groups at the fast end, else an LDS-tiled permute copies
//         them into that layout;
//   DOT   long inner products (K >= 256, not a matrix-core product): one
//         work-group reduces each output, never one thread;
//   SIMT  otherwise (any layout, one thread per output element).
#include "plan.h"
#include "kernels.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <unordered_map>

namespace qx {

namespace {

constexpr int KIND_REG = 0, KIND_OUT = 1, KIND_SLICE = 2;
constexpr int CLS_SIMT = 0, CLS_GEMM = 1, CLS_DOT = 2;
constexpr int INF_OP = 1 << 30;

struct Node {
  int a = -1, b = -1, parent = -1;
  bool leaf = false;
  bool has_fixed = false;   // a leaf carrying a fixed sliced index
  bool depF = false;        // sub-tree touches a fixed sliced index
  int nq = 0;               // output wires below
  bool batched = false;
  int phase = PH_CONST;
  std::vector<int> bits;    // label ids of the stored result (sorted)
  std::vector<int> K, H, Fa, Fb;  // contraction sets (sorted)
  int cls = CLS_SIMT;
  int tensor = -1;
};

struct View {
  std::vector<FixTerm> fix;
  std::vector<std::pair<int, int64_t>> gath;  // (qubit, stride)
};

bool contains(const std::vector<int>& sorted, int x) {
  return std::binary_search(sorted.begin(), sorted.end(), x);
}
std::vector<int> set_and(const std::vector<int>& a, const std::vector<int>& b) {
  std::vector<int> r;
  std::set_intersection(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
  return r;
}
std::vector<int> set_minus(const std::vector<int>& a, const std::vector<int>& b) {
  std::vector<int> r;
  std::set_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
  return r;
}
std::vector<int> set_or(const std::vector<int>& a, const std::vector<int>& b) {
  std::vector<int> r;
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
  return r;
}
bool same_set(std::vector<int> a, std::vector<int> b) {
  std::sort(a.begin(), a.end());
  std::sort(b.begin(), b.end());
  return a == b;
}

struct Compiler {
  PlanCore& pc;
  std::string& err;
  std::vector<Node> nodes;
  std::vector<Op> ops;  // emission order (phases sorted later)

  Compiler(PlanCore& p, std::string& e) : pc(p), err(e) {}

  // split-precision plans store every matrix-product operand split (BF16 or scaled FP16 planes)
  bool split() const { return pc.precision == QX_SPLIT_BF16 || pc.precision == QX_SPLIT_FP16; }
  int split_kind() const { return pc.precision == QX_SPLIT_FP16 ? 2 : 1; }

  bool is_fixed(int lab) const { return pc.kind[lab] == KIND_SLICE && pc.aux[lab] >= pc.js; }
  bool is_vary(int lab) const { return pc.kind[lab] == KIND_SLICE && pc.aux[lab] < pc.js; }
  bool is_out(int lab) const { return pc.kind[lab] == KIND_OUT; }

  int pos_in(const Tensor& t, int lab) const {
    for (size_t i = 0; i < t.lay.size(); ++i)
      if (t.lay[i] == lab) return (int)i;
    return -1;
  }

  View view(const Tensor& t, bool consumer_batched) const {
    View v;
    for (size_t i = 0; i < t.lay.size(); ++i) {
      const int lab = t.lay[i];
      const int64_t stride = (int64_t)1 << i;
      if (is_fixed(lab)) v.fix.push_back({pc.aux[lab], stride});
      else if (is_out(lab) && consumer_batched && !t.batched) v.gath.push_back({pc.aux[lab], stride});
    }
    return v;
  }

  int add_gather(int tensor, const View& v) {
    if (v.gath.empty()) return -1;
    GatherDesc g;
    g.tensor = tensor;
    for (auto& qs : v.gath) {
      g.q.push_back(qs.first);
      g.stride.push_back(qs.second);
    }
    pc.gathers.push_back(g);
    return (int)pc.gathers.size() - 1;
  }

  // Operand labels the contraction sees (fixed and gathered indices removed).
  std::vector<int> visible(const Node& c, bool consumer_batched) const {
    std::vector<int> r;
    for (int lab : c.bits)
      if (!(is_out(lab) && consumer_batched && !c.batched)) r.push_back(lab);
    return r;
  }

  // F and K at the fast end as two contiguous groups?  kfirst: K is the fastest group.
  bool ready(const Tensor& t, const std::vector<int>& F, const std::vector<int>& K, bool& kfirst,
             std::vector<int>& korder, std::vector<int>& forder) const {
    const size_t nf = F.size(), nk = K.size();
    if (t.lay.size() < nf + nk) return false;
    auto in = [&](const std::vector<int>& s, size_t lo, size_t hi) {
      for (size_t i = lo; i < hi; ++i)
        if (!contains(s, t.lay[i])) return false;
      return true;
    };
    if (in(K, 0, nk) && in(F, nk, nk + nf)) {
      kfirst = true;
      korder.assign(t.lay.begin(), t.lay.begin() + nk);
      forder.assign(t.lay.begin() + nk, t.lay.begin() + nk + nf);
      return true;
    }
    if (in(F, 0, nf) && in(K, nf, nf + nk)) {
      kfirst = false;
      forder.assign(t.lay.begin(), t.lay.begin() + nf);
      korder.assign(t.lay.begin() + nf, t.lay.begin() + nf + nk);
      return true;
    }
    return false;
  }

  // Copy tensor ti into layout [korder][F in ti's order][rest in ti's order] (fastest first).
  int emit_permute(int ti, const std::vector<int>& korder, const std::vector<int>& F) {
    const Tensor src = pc.tensors[ti];
    if (src.split) err = "internal: permute of a split tensor";
    Tensor dst;
    dst.batched = src.batched;
    dst.phase = src.phase;
    dst.lay = korder;
    for (int lab : src.lay)
      if (contains(F, lab)) dst.lay.push_back(lab);
    for (int lab : src.lay)
      if (std::find(dst.lay.begin(), dst.lay.end(), lab) == dst.lay.end()) dst.lay.push_back(lab);
    pc.tensors.push_back(dst);
    const int di = (int)pc.tensors.size() - 1;
    Op op;
    op.kind = OP_PERM;
    op.phase = src.phase;
    op.in_a = ti;
    op.out = di;
    std::memset(&op.perm, 0, sizeof(op.perm));
    op.perm.rank = (int)dst.lay.size();
    op.perm.n_items = src.batched ? pc.max_b : 1;
    op.perm.in_item = src.batched ? src.elems() : 0;
    op.perm.out_item = src.batched ? dst.elems() : 0;
    for (size_t i = 0; i < dst.lay.size(); ++i) op.perm.in_pos[i] = pos_in(src, dst.lay[i]);
    permute_setup(op.perm);
    const double items = src.batched ? pc.max_b : 1;
    op.bytes = 16.0 * (double)src.elems() * items;
    ops.push_back(op);
    return di;
  }

  bool build(const qx_network* net, const int32_t* tree) {
    const int n = pc.n_leaves;
    const int nn = 2 * n - 1;
    nodes.assign(nn, Node());
    // leaves
    int64_t off = 0;
    for (int t = 0; t < n; ++t) {
      Node& nd = nodes[t];
      nd.leaf = true;
      Tensor tt;
      tt.is_leaf = true;
      tt.leaf_off = off;
      const int64_t r = net->index_ptr[t + 1] - net->index_ptr[t];
      off += (int64_t)1 << r;
      // listed order is slowest first; lay is fastest first
      for (int64_t i = r - 1; i >= 0; --i) tt.lay.push_back((int)pc.aux_label_id[net->index_ptr[t] + i]);
      for (int lab : tt.lay) {
        if (is_fixed(lab)) { nd.has_fixed = true; nd.depF = true; }
        else nd.bits.push_back(lab);
        if (is_out(lab)) nd.nq++;
      }
      std::sort(nd.bits.begin(), nd.bits.end());
      nd.tensor = (int)pc.tensors.size();
      pc.tensors.push_back(tt);
    }
    int logb = 0;
    while ((1 << (logb + 1)) <= pc.max_b) ++logb;
    // internal nodes: sets, modes, classes
    for (int t = 0; t < n - 1; ++t) {
      const int p = n + t;
      Node& nd = nodes[p];
      nd.a = tree[2 * t];
      nd.b = tree[2 * t + 1];
      nodes[nd.a].parent = p;
      nodes[nd.b].parent = p;
      const Node& A = nodes[nd.a];
      const Node& B = nodes[nd.b];
      nd.nq = A.nq + B.nq;
      nd.depF = A.depF || B.depF;
      nd.batched = A.batched || B.batched || nd.nq > logb;
      nd.phase = nd.depF ? PH_BLOCK : (nd.batched ? PH_CALL : PH_CONST);
      const std::vector<int> va = visible(A, nd.batched), vb = visible(B, nd.batched);
      const std::vector<int> both = set_and(va, vb);
      for (int lab : both) {
        if (is_vary(lab)) nd.H.push_back(lab);
        else if (pc.kind[lab] == KIND_REG) nd.K.push_back(lab);
        else {
          err = "internal: unexpected shared label";
          return false;
        }
      }
      nd.Fa = set_minus(va, vb);
      nd.Fb = set_minus(vb, va);
      nd.bits = set_or(set_or(nd.Fa, nd.Fb), nd.H);
      const int m = (int)nd.Fa.size(), nb = (int)nd.Fb.size(), k = (int)nd.K.size();
      const bool leaf_fixed = A.has_fixed || B.has_fixed;
      // a large result from a long operand and a short one (at most 32 rows, at most 32 terms
      // summed): the memory-bound thin matrix-product kernel reads the long operand once, in
      // its own order, where one thread per output would read it scattered and once per short row
      const bool big = (int)nd.bits.size() + (nd.batched ? logb : 0) >= 20;
      const bool thin = std::min(m, nb) >= 1 && std::min(m, nb) <= 5 && std::max(m, nb) >= 4 && k >= 1 && k <= 5;
      if (!leaf_fixed && m >= 4 && nb >= 4 && k >= 3 && m + nb + k >= 15) nd.cls = CLS_GEMM;
      else if (!leaf_fixed && big && thin) nd.cls = CLS_GEMM;
      else if (!leaf_fixed && k >= 8) nd.cls = CLS_DOT;  // long sums: parallel reduction, never one thread
      else nd.cls = CLS_SIMT;
      if ((int)nd.bits.size() > QX_MAX_BITS) {
        err = "an intermediate has more than 48 indices (including open output and slice indices)";
        return false;
      }
      if (nd.cls == CLS_SIMT && k > QX_MAX_KBITS) {
        err = "a small contraction sums over more than 24 indices";
        return false;
      }
      if ((int)nd.H.size() > QX_MAX_HBITS) {
        err = "too many varying sliced indices shared by one contraction";
        return false;
      }
      // per-slice, per-bitstring work (regular indices only)
      int reg = 0;
      for (int lab : set_or(set_or(nd.Fa, nd.Fb), nd.K))
        if (pc.kind[lab] == KIND_REG) ++reg;
      pc.flops_per_slice += 8.0 * std::ldexp(1.0, reg);
      int regw = 0;
      for (int lab : nd.bits)
        if (pc.kind[lab] == KIND_REG) ++regw;
      pc.width = std::max(pc.width, regw);
    }
    // split plans store every matrix-product operand split; leaves are split at upload (BF16) or after
    // the scale calibration at plan creation (FP16)
    if (split())
      for (int t = 0; t < n; ++t)
        if (nodes[t].parent >= 0 && nodes[nodes[t].parent].cls == CLS_GEMM) pc.tensors[nodes[t].tensor].split = true;
    for (int t = 0; t < n - 1; ++t)
      if (!emit_node(n + t) || !err.empty()) return false;
    pc.root = nodes[nn - 1].tensor;
    return true;
  }

  // Preferred storage order (fastest first) of node p's result for its consumer.
  // For a matrix-product parent: the contracted indices lowest -- the sibling's
  // three lowest if they are contracted there, so both operands can be read
  // k-contiguously -- then the parent's free indices, then the rest.  For a
  // dot parent the sibling's contracted order must be matched exactly.
  // Otherwise: the free indices of the larger child first (coalesced writes).
  std::vector<int> preferred_layout(int p, int ta, int tb) {
    const Node& nd = nodes[p];
    const int q = nd.parent;
    const Tensor& TA = pc.tensors[ta];
    const Tensor& TB = pc.tensors[tb];
    const Tensor& big = TA.elems() >= TB.elems() ? TA : TB;
    const Tensor& small = TA.elems() >= TB.elems() ? TB : TA;
    std::vector<int> ff;
    auto push = [&](int lab) {
      if (contains(nd.bits, lab) && std::find(ff.begin(), ff.end(), lab) == ff.end()) ff.push_back(lab);
    };
    if (q >= 0 && (nodes[q].cls == CLS_GEMM || nodes[q].cls == CLS_DOT)) {
      const Node& Q = nodes[q];
      const std::vector<int> vis = visible(nd, Q.batched);
      const std::vector<int> kq = set_and(vis, Q.K);
      const std::vector<int> fq = set_minus(set_minus(vis, Q.K), Q.H);
      const int sib = Q.a == p ? Q.b : Q.a;
      bool matched = false;
      if (nodes[sib].tensor >= 0) {
        const Tensor& st = pc.tensors[nodes[sib].tensor];
        if (Q.cls == CLS_DOT) {
          std::vector<int> ko = kq;
          std::sort(ko.begin(), ko.end(), [&](int x, int y) { return pos_in(st, x) < pos_in(st, y); });
          for (int lab : ko) push(lab);
          matched = true;
        } else if (st.lay.size() >= 3 && contains(kq, st.lay[0]) && contains(kq, st.lay[1]) &&
                   contains(kq, st.lay[2])) {
          for (int i = 0; i < 3; ++i) push(st.lay[i]);
          matched = true;
        }
      }
      if (!matched || Q.cls == CLS_GEMM) {
        std::vector<int> kord;
        for (int lab : big.lay)
          if (contains(kq, lab)) kord.push_back(lab);
        for (int lab : small.lay)
          if (contains(kq, lab) && std::find(kord.begin(), kord.end(), lab) == kord.end()) kord.push_back(lab);
        if (!matched && Q.cls == CLS_GEMM && split())
          for (int lab : register_epilogue_lead(p, sib, kord)) push(lab);
        for (int lab : kord) push(lab);
      }
      for (int lab : big.lay)
        if (contains(fq, lab)) push(lab);
      for (int lab : small.lay)
        if (contains(fq, lab)) push(lab);
    }
    for (int lab : big.lay) push(lab);
    for (int lab : small.lay) push(lab);
    return ff;
  }

  // Node p and its sibling sib are the two operands of a split matrix product
  // and p is laid out first; the sibling will copy p's three lowest indices
  // (contracted ones, so both operands are read k-contiguously).  A split
  // matrix product writes its result straight from the accumulators when its
  // three lowest output indices lie on one operand side holding at least four
  // free indices, so pick, from the contracted indices in the order kord, three
  // that allow this for both producing products if possible, else for the one
  // with the larger result.  Empty when neither can have it.
  std::vector<int> register_epilogue_lead(int p, int sib, const std::vector<int>& kord) {
    const Node& P = nodes[p];
    const Node& S = nodes[sib];
    auto side = [](const Node& x, int lab) { return contains(x.Fa, lab) ? 1 : contains(x.Fb, lab) ? 2 : 0; };
    auto fits = [](const Node& x, int s) {
      return (s == 1 && x.Fa.size() >= 4) || (s == 2 && x.Fb.size() >= 4);
    };
    auto weight = [&](const Node& x) {
      return x.cls == CLS_GEMM ? std::ldexp(1.0, (int)x.bits.size()) * (x.batched ? pc.max_b : 1) : 0.0;
    };
    const double wp = weight(P), ws = weight(S);
    std::vector<int> best;
    double best_w = 0.0;
    // sp / ss: required side in P / S, 0 = no requirement
    for (int sp = 0; sp <= 2; ++sp)
      for (int ss = 0; ss <= 2; ++ss) {
        if ((sp && (wp == 0.0 || !fits(P, sp))) || (ss && (ws == 0.0 || !fits(S, ss)))) continue;
        const double w = (sp ? wp : 0.0) + (ss ? ws : 0.0);
        if (w <= best_w) continue;
        std::vector<int> c;
        for (int lab : kord)
          if ((!sp || side(P, lab) == sp) && (!ss || side(S, lab) == ss) && c.size() < 3) c.push_back(lab);
        if (c.size() == 3) {
          best = c;
          best_w = w;
        }
      }
    return best;
  }

  // Matrix product in bit-scattered mode: operands are read in their stored
  // layouts and the result is written in the layout its consumer prefers.
  void emit_gemm(Node& nd, int ta, int tb, Tensor& out, Op& op, double items) {
    const int p = (int)(&nd - nodes.data());
    out.lay = preferred_layout(p, ta, tb);
    // the N side (whose rows vary across lanes in the epilogue) owns the lowest output index
    bool a_is_n = nd.Fa.size() > nd.Fb.size();
    for (int lab : out.lay) {
      if (contains(nd.Fa, lab)) { a_is_n = true; break; }
      if (contains(nd.Fb, lab)) { a_is_n = false; break; }
    }
    // A split output whose three lowest indices all come from one side can be written
    // straight from the accumulators: that side becomes M, numbered so that m bits 0, 1, 3
    // (the rows one lane holds in its accumulator groups) are those three indices.
    bool ep_reg = false;
    if (split() && out.split && out.lay.size() >= 3) {
      const bool fa = contains(nd.Fa, out.lay[0]) && contains(nd.Fa, out.lay[1]) && contains(nd.Fa, out.lay[2]);
      const bool fb = contains(nd.Fb, out.lay[0]) && contains(nd.Fb, out.lay[1]) && contains(nd.Fb, out.lay[2]);
      if ((fa && nd.Fa.size() >= 4) || (fb && nd.Fb.size() >= 4)) {
        ep_reg = true;
        a_is_n = !fa;
      }
    }
    const int tA = a_is_n ? tb : ta, tB = a_is_n ? ta : tb;
    const std::vector<int>& FA = a_is_n ? nd.Fb : nd.Fa;
    const std::vector<int>& FB = a_is_n ? nd.Fa : nd.Fb;
    const Tensor& XA = pc.tensors[tA];
    const Tensor& XB = pc.tensors[tB];
    const View va = view(XA, nd.batched), vb = view(XB, nd.batched);
    op.in_a = tA;
    op.in_b = tB;
    op.gather_a = add_gather(tA, va);
    op.gather_b = add_gather(tB, vb);
    auto by_out = [&](std::vector<int> v) {
      std::sort(v.begin(), v.end(), [&](int x, int y) { return pos_in(out, x) < pos_in(out, y); });
      return v;
    };
    std::vector<int> mlab = by_out(FA);
    const std::vector<int> nlab = by_out(FB);
    if (ep_reg) std::swap(mlab[2], mlab[3]);
    // k numbering: three unit-stride k bits first when an operand has them lowest
    auto low3 = [&](const Tensor& t) {
      return t.lay.size() >= 3 && contains(nd.K, t.lay[0]) && contains(nd.K, t.lay[1]) &&
             contains(nd.K, t.lay[2]);
    };
    const bool a3 = low3(XA), b3 = low3(XB);
    bool kca = false, kcb = false;
    std::vector<int> klab;
    const Tensor* kref = XA.elems() >= XB.elems() ? &XA : &XB;
    if (a3 && b3 && std::equal(XA.lay.begin(), XA.lay.begin() + 3, XB.lay.begin())) {
      kca = kcb = true;
      klab.assign(XA.lay.begin(), XA.lay.begin() + 3);
    } else if (a3 && (!b3 || XA.elems() >= XB.elems())) {
      kca = true;
      klab.assign(XA.lay.begin(), XA.lay.begin() + 3);
      kref = &XA;
    } else if (b3) {
      kcb = true;
      klab.assign(XB.lay.begin(), XB.lay.begin() + 3);
      kref = &XB;
    }
    std::vector<int> krest = nd.K;
    std::sort(krest.begin(), krest.end(), [&](int x, int y) { return pos_in(*kref, x) < pos_in(*kref, y); });
    for (int lab : krest)
      if (std::find(klab.begin(), klab.end(), lab) == klab.end()) klab.push_back(lab);
    std::vector<int> horder = nd.H;
    std::sort(horder.begin(), horder.end(), [&](int x, int y) { return pos_in(XA, x) < pos_in(XA, y); });

    GemmArgs& g = op.gemm;
    std::memset(&g, 0, sizeof(g));
    g.bits = 1;
    g.nm = (int)mlab.size();
    g.nn = (int)nlab.size();
    g.nk = (int)klab.size();
    g.M = (int64_t)1 << g.nm;
    g.N = (int64_t)1 << g.nn;
    g.K = (int64_t)1 << g.nk;
    for (int i = 0; i < g.nm; ++i) {
      g.a_rs[i] = (int64_t)1 << pos_in(XA, mlab[i]);
      g.c_mst[i] = (int64_t)1 << pos_in(out, mlab[i]);
    }
    for (int i = 0; i < g.nn; ++i) {
      g.b_rs[i] = (int64_t)1 << pos_in(XB, nlab[i]);
      g.c_nst[i] = (int64_t)1 << pos_in(out, nlab[i]);
    }
    for (int j = 0; j < g.nk; ++j) {
      g.a_kst[j] = (int64_t)1 << pos_in(XA, klab[j]);
      g.b_kst[j] = (int64_t)1 << pos_in(XB, klab[j]);
    }
    g.a_kc = kca;
    g.b_kc = kcb;
    if (split()) {
      if (!XA.split || !XB.split) err = "internal: matrix-product operand not stored split";
      g.a_split = g.b_split = split_kind();
    }
    // 16-byte loads need 8-element alignment: arena tensors are 256-byte aligned and every
    // non-k stride of a k-contiguous operand is a multiple of 8
    g.vec_a = kca && (!XA.is_leaf || XA.leaf_off % 8 == 0);
    g.vec_b = kcb && (!XB.is_leaf || XB.leaf_off % 8 == 0);
    g.a_item = XA.batched ? XA.elems() : 0;
    g.b_item = XB.batched ? XB.elems() : 0;
    g.n_items = (int)items;
    g.nh = (int)horder.size();
    for (size_t i = 0; i < horder.size(); ++i) {
      g.a_hs[i] = (int64_t)1 << pos_in(XA, horder[i]);
      g.b_hs[i] = (int64_t)1 << pos_in(XB, horder[i]);
      g.c_hs[i] = (int64_t)1 << pos_in(out, horder[i]);
    }
    gemm_args_setup(g);
    g.ep_reg = ep_reg;
    op.kind = OP_GEMM;
    if (pc.precision == QX_SPLIT_FP16) {
      // each operand's scale slot (a tensor has one consumer); the magnitude reductions that fill
      // them run only in the calibration pass at plan creation
      op.scale_slot = pc.n_scale_slots;
      pc.n_scale_slots += 2;
      pc.tensors[tA].scale_slot = op.scale_slot;
      pc.tensors[tB].scale_slot = op.scale_slot + 1;
      for (int side = 0; side < 2; ++side) {
        const int ti = side == 0 ? tA : tB;
        Op am;
        am.kind = OP_ABSMAX;
        am.phase = pc.tensors[ti].phase;
        am.in_a = ti;
        am.out = -1;
        am.scale_slot = op.scale_slot + side;
        std::memset(&am.absmax, 0, sizeof(am.absmax));
        am.bytes = 8.0 * (double)pc.tensors[ti].elems() * (pc.tensors[ti].batched ? pc.max_b : 1);
        ops.push_back(am);
      }
    }
    op.flops = 8.0 * (double)g.M * g.N * g.K * std::ldexp(1.0, g.nh) * items;
    op.tile = (std::min(g.M, g.N) <= 32 && g.K <= 32) ? (int)GEMM_TILE_THIN : gemm_default_tile(g.M, g.N);
  }

  bool emit_node(int p) {
    Node& nd = nodes[p];
    const Node& NA = nodes[nd.a];
    const Node& NB = nodes[nd.b];
    int ta = NA.tensor, tb = NB.tensor;
    Tensor out;
    out.batched = nd.batched;
    out.phase = nd.phase;
    out.split = split() && nd.parent >= 0 && nodes[nd.parent].cls == CLS_GEMM;
    Op op;
    op.phase = nd.phase;
    const double items = nd.batched ? pc.max_b : 1;
    const int q = nd.parent;
    if (nd.cls == CLS_GEMM) {
      emit_gemm(nd, ta, tb, out, op, items);
    } else if (nd.cls == CLS_DOT) {
      const bool need_kfirst = true;
      bool ka = false, kb = false;
      std::vector<int> koa, kob, foa, fob;
      bool ra = ready(pc.tensors[ta], nd.Fa, nd.K, ka, koa, foa) && (!need_kfirst || ka);
      bool rb = ready(pc.tensors[tb], nd.Fb, nd.K, kb, kob, fob) && (!need_kfirst || kb);
      if (ra && rb && koa != kob) {
        if (pc.tensors[ta].elems() <= pc.tensors[tb].elems()) ra = false;
        else rb = false;
      }
      if (!ra && !rb) {
        std::vector<int> ko = nd.K;  // canonical: sorted label ids
        ta = emit_permute(ta, ko, nd.Fa);
        tb = emit_permute(tb, ko, nd.Fb);
      } else if (!ra) {
        ta = emit_permute(ta, kob, nd.Fa);
      } else if (!rb) {
        tb = emit_permute(tb, koa, nd.Fb);
      }
      const View va = view(pc.tensors[ta], nd.batched), vb = view(pc.tensors[tb], nd.batched);
      op.in_a = ta;
      op.in_b = tb;
      op.gather_a = add_gather(ta, va);
      op.gather_b = add_gather(tb, vb);
      std::vector<int> horder = nd.H;
      std::sort(horder.begin(), horder.end(),
                [&](int x, int y) { return pos_in(pc.tensors[ta], x) < pos_in(pc.tensors[ta], y); });
      const Tensor& TA = pc.tensors[ta];
      const Tensor& TB = pc.tensors[tb];
      {
        // DOT: output bits fastest-first = Fb, Fa, H
        out.lay = nd.Fb;
        out.lay.insert(out.lay.end(), nd.Fa.begin(), nd.Fa.end());
        out.lay.insert(out.lay.end(), horder.begin(), horder.end());
        DotArgs& d = op.dot;
        std::memset(&d, 0, sizeof(d));
        d.K = (int64_t)1 << nd.K.size();
        d.n_out = (int)out.lay.size();
        for (size_t i = 0; i < out.lay.size(); ++i) {
          const int pa = pos_in(TA, out.lay[i]), pb = pos_in(TB, out.lay[i]);
          d.a_os[i] = pa >= 0 ? ((int64_t)1 << pa) : 0;
          d.b_os[i] = pb >= 0 ? ((int64_t)1 << pb) : 0;
        }
        d.a_item = TA.batched ? TA.elems() : 0;
        d.b_item = TB.batched ? TB.elems() : 0;
        d.n_items = (int)items;
        op.kind = OP_DOT;
        op.flops = 8.0 * (double)d.K * std::ldexp(1.0, d.n_out) * items;
      }
    } else {
      // SIMT: any layout can be written, so write the one the consumer prefers
      const Tensor& TA = pc.tensors[ta];
      const Tensor& TB = pc.tensors[tb];
      std::vector<int> ff = preferred_layout(p, ta, tb);
      if (ff.size() != nd.bits.size()) {
        err = "internal: output layout incomplete";
        return false;
      }
      out.lay = ff;
      const View va = view(TA, nd.batched), vb = view(TB, nd.batched);
      op.in_a = ta;
      op.in_b = tb;
      op.gather_a = add_gather(ta, va);
      op.gather_b = add_gather(tb, vb);
      op.fix_a = va.fix;
      op.fix_b = vb.fix;
      SimtArgs& s = op.simt;
      std::memset(&s, 0, sizeof(s));
      s.n_out = (int)ff.size();
      s.n_k = (int)nd.K.size();
      for (size_t i = 0; i < ff.size(); ++i) {
        const int pa = pos_in(TA, ff[i]), pb = pos_in(TB, ff[i]);
        s.a_os[i] = pa >= 0 ? ((int64_t)1 << pa) : 0;
        s.b_os[i] = pb >= 0 ? ((int64_t)1 << pb) : 0;
      }
      for (size_t j = 0; j < nd.K.size(); ++j) {
        s.a_ks[j] = (int64_t)1 << pos_in(TA, nd.K[j]);
        s.b_ks[j] = (int64_t)1 << pos_in(TB, nd.K[j]);
      }
      s.a_item = TA.batched ? TA.elems() : 0;
      s.b_item = TB.batched ? TB.elems() : 0;
      s.n_items = (int)items;
      op.kind = OP_SIMT;
      op.flops = 8.0 * std::ldexp(1.0, s.n_out + s.n_k) * items;
    }
    pc.tensors.push_back(out);
    const int oi = (int)pc.tensors.size() - 1;
    nd.tensor = oi;
    op.out = oi;
    const Tensor& O = pc.tensors[oi];
    const double ia = pc.tensors[op.in_a].batched ? pc.max_b : 1;
    const double ib = pc.tensors[op.in_b].batched ? pc.max_b : 1;
    op.bytes = 8.0 * ((double)pc.tensors[op.in_a].elems() * ia + (double)pc.tensors[op.in_b].elems() * ib +
                      (double)O.elems() * items);
    const int64_t citem = O.batched ? O.elems() : 0;
    const int csplit = O.split ? split_kind() : 0;
    if (op.kind == OP_SIMT) { op.simt.c_item = citem; op.simt.c_split = csplit; }
    if (op.kind == OP_GEMM) { op.gemm.c_item = citem; op.gemm.c_split = csplit; }
    if (op.kind == OP_DOT) { op.dot.c_item = citem; op.dot.c_split = csplit; }
    ops.push_back(op);
    return true;
  }
};

}  // namespace

qx_status compile_plan(const qx_network* net, const int32_t* tree, const int64_t* sliced,
                       int32_t n_sliced, const qx_plan_options& opt, int js, PlanCore& pc,
                       std::string& err) {
  pc = PlanCore();
  const int n = net->n_tensors;
  pc.n_leaves = n;
  pc.n_qubits = net->n_qubits;
  pc.n_sliced = n_sliced;
  pc.precision = opt.precision;
  pc.max_b = opt.max_bitstrings;
  pc.js = js;
  // dense label ids
  std::unordered_map<int64_t, int> id;
  std::vector<int> count;
  const int64_t nidx = net->index_ptr[n];
  pc.aux_label_id.resize(nidx);
  for (int t = 0; t < n; ++t) {
    for (int64_t i = net->index_ptr[t]; i < net->index_ptr[t + 1]; ++i) {
      const int64_t lab = net->index_ids[i];
      for (int64_t i2 = net->index_ptr[t]; i2 < i; ++i2)
        if (net->index_ids[i2] == lab) {
          err = "label " + std::to_string(lab) + " appears twice in one tensor (traces are not supported)";
          return QX_ERR_INVALID_NETWORK;
        }
      auto it = id.find(lab);
      int d;
      if (it == id.end()) {
        d = (int)pc.label_of.size();
        id[lab] = d;
        pc.label_of.push_back(lab);
        count.push_back(0);
      } else {
        d = it->second;
      }
      count[d]++;
      pc.aux_label_id[i] = d;
    }
  }
  const int L = (int)pc.label_of.size();
  pc.kind.assign(L, KIND_REG);
  pc.aux.assign(L, -1);
  for (int qb = 0; qb < net->n_qubits; ++qb) {
    auto it = id.find(net->output_index[qb]);
    if (it == id.end()) {
      err = "output wire of qubit " + std::to_string(qb) + " is not an index of any tensor";
      return QX_ERR_INVALID_NETWORK;
    }
    if (pc.kind[it->second] == KIND_OUT) {
      err = "two qubits share one output wire";
      return QX_ERR_INVALID_NETWORK;
    }
    pc.kind[it->second] = KIND_OUT;
    pc.aux[it->second] = qb;
  }
  for (int d = 0; d < L; ++d) {
    const int want = pc.kind[d] == KIND_OUT ? 1 : 2;
    if (count[d] != want) {
      err = "label " + std::to_string(pc.label_of[d]) + " appears in " + std::to_string(count[d]) +
            " tensors (" + (want == 1 ? "output wires need 1" : "need 2") + ")";
      return QX_ERR_INVALID_NETWORK;
    }
  }
  for (int j = 0; j < n_sliced; ++j) {
    auto it = id.find(sliced[j]);
    if (it == id.end()) {
      err = "sliced label " + std::to_string(sliced[j]) + " is not in the network";
      return QX_ERR_INVALID_ARG;
    }
    if (pc.kind[it->second] == KIND_OUT) {
      err = "sliced label " + std::to_string(sliced[j]) + " is an output wire";
      return QX_ERR_INVALID_ARG;
    }
    if (pc.kind[it->second] == KIND_SLICE) {
      err = "sliced label " + std::to_string(sliced[j]) + " listed twice";
      return QX_ERR_INVALID_ARG;
    }
    pc.kind[it->second] = KIND_SLICE;
    pc.aux[it->second] = j;
  }
  // open output qubits: their wires become regular indices that no contraction sums, so they
  // reach the root, which then holds 2^m values per bitstring
  pc.open_bit.assign(L, -1);
  pc.n_open = 0;
  for (int qb = 0; qb < net->n_qubits; ++qb)
    if ((opt.open_qubits >> qb) & 1ULL) {
      const int d = id.find(net->output_index[qb])->second;
      pc.kind[d] = KIND_REG;
      pc.aux[d] = -1;
      pc.open_bit[d] = pc.n_open++;
    }
  // tree validity: SSA, each id consumed once, all consumed
  std::vector<char> used(2 * n - 1, 0);
  for (int t = 0; t < n - 1; ++t) {
    for (int s = 0; s < 2; ++s) {
      const int c = tree[2 * t + s];
      if (c < 0 || c >= n + t) {
        err = "tree step " + std::to_string(t) + " refers to id " + std::to_string(c) + " not yet defined";
        return QX_ERR_INVALID_TREE;
      }
      if (used[c]) {
        err = "tree consumes id " + std::to_string(c) + " twice";
        return QX_ERR_INVALID_TREE;
      }
      used[c] = 1;
    }
  }
  // leaf data
  pc.leaf_pool_elems = 0;
  for (int t = 0; t < n; ++t) {
    const int64_t r = net->index_ptr[t + 1] - net->index_ptr[t];
    if (net->data_ptr[t + 1] - net->data_ptr[t] != ((int64_t)1 << r)) {
      err = "tensor " + std::to_string(t) + " does not hold 2^rank elements (every index must have dimension 2)";
      return QX_ERR_UNSUPPORTED;
    }
    pc.leaf_pool_elems += (int64_t)1 << r;
  }
  pc.leaf_data.assign(net->data + 2 * net->data_ptr[0], net->data + 2 * net->data_ptr[n]);

  Compiler cc(pc, err);
  if (!cc.build(net, tree)) return QX_ERR_UNSUPPORTED;

  // order ops by phase (stable: dependencies only point to equal or earlier phases)
  std::vector<Op> sorted;
  for (int ph = PH_CONST; ph <= PH_BLOCK; ++ph)
    for (auto& o : cc.ops)
      if (o.phase == ph) sorted.push_back(o);
  pc.ops = sorted;
  for (auto& o : pc.ops) {
    if (o.phase == PH_CONST) pc.n_const++;
    else if (o.phase == PH_CALL) pc.n_call++;
    else pc.n_block++;
  }
  // liveness
  for (auto& t : pc.tensors) {
    t.first_op = -1;
    t.last_op = -1;
  }
  for (int i = 0; i < (int)pc.ops.size(); ++i) {
    const Op& o = pc.ops[i];
    if (o.out >= 0) {
      Tensor& out = pc.tensors[o.out];
      out.first_op = i;
      out.last_op = std::max(out.last_op, i);
    }
    for (int in : {o.in_a, o.in_b}) {
      if (in < 0) continue;
      Tensor& ti = pc.tensors[in];
      const int produced_phase = ti.phase;
      ti.last_op = (produced_phase < o.phase) ? INF_OP : std::max(ti.last_op, i);
    }
  }
  Tensor& rt = pc.tensors[pc.root];
  if (!rt.is_leaf) rt.last_op = INF_OP;
  // first-fit interval allocation in the arena
  struct Iv { int64_t off, size; int last; };
  std::vector<int> order;
  for (int i = 0; i < (int)pc.tensors.size(); ++i)
    if (!pc.tensors[i].is_leaf && pc.tensors[i].first_op >= 0) order.push_back(i);
  std::sort(order.begin(), order.end(),
            [&](int x, int y) { return pc.tensors[x].first_op < pc.tensors[y].first_op; });
  std::vector<Iv> live;
  int64_t arena = 0;
  for (int ti : order) {
    Tensor& t = pc.tensors[ti];
    const int64_t sz = ((t.elems() * (t.batched ? pc.max_b : 1) * 8) + 255) / 256 * 256;
    std::vector<Iv> keep;
    for (auto& iv : live)
      if (iv.last >= t.first_op) keep.push_back(iv);
    live.swap(keep);
    std::sort(live.begin(), live.end(), [](const Iv& x, const Iv& y) { return x.off < y.off; });
    int64_t cand = 0;
    for (auto& iv : live) {
      if (cand + sz <= iv.off) break;
      cand = std::max(cand, iv.off + iv.size);
    }
    t.arena_off = cand;
    live.push_back({cand, sz, t.last_op});
    arena = std::max(arena, cand + sz);
  }
  pc.arena_bytes = arena;
  if (getenv("QX_DUMP_PLAN")) {
    static const char* kn[] = {"SIMT", "GEMM", "DOT", "PERM"};
    for (size_t i = 0; i < pc.ops.size(); ++i) {
      const Op& o = pc.ops[i];
      if (o.kind == OP_ABSMAX || (o.phase != PH_BLOCK && o.kind != OP_PERM && o.kind != OP_GEMM)) continue;
      fprintf(stderr, "op %zu ph %d %s in %d(%zu b%d) %d out %d(%zu b%d) flops %.3g bytes %.3g", i, o.phase,
              kn[o.kind], o.in_a, pc.tensors[o.in_a].lay.size(), (int)pc.tensors[o.in_a].batched, o.in_b,
              o.out, pc.tensors[o.out].lay.size(), (int)pc.tensors[o.out].batched, o.flops, o.bytes);
      if (o.kind == OP_GEMM)
        fprintf(stderr, " M %lld N %lld K %lld nh %d akc %d bkc %d csplit %d epreg %d", (long long)o.gemm.M,
                (long long)o.gemm.N, (long long)o.gemm.K, o.gemm.nh, o.gemm.a_kc, o.gemm.b_kc, o.gemm.c_split,
                o.gemm.ep_reg);
      if (o.kind == OP_GEMM) {
        fprintf(stderr, " ep");
        for (int j = 0; j < 10; ++j) fprintf(stderr, " %s%d:%lld", o.gemm.ep_lm[j] ? "m" : "n",
                                             o.gemm.ep_lm[j] ? o.gemm.ep_lm[j] : o.gemm.ep_ln[j],
                                             (long long)o.gemm.ep_st[j]);
        fprintf(stderr, " hs");
        for (int j = 0; j < o.gemm.nh; ++j) fprintf(stderr, " %lld", (long long)o.gemm.c_hs[j]);
        fprintf(stderr, " a_rs");
        for (int j = 0; j < o.gemm.nm; ++j) fprintf(stderr, " %lld", (long long)o.gemm.a_rs[j]);
        fprintf(stderr, " b_rs");
        for (int j = 0; j < o.gemm.nn; ++j) fprintf(stderr, " %lld", (long long)o.gemm.b_rs[j]);
        fprintf(stderr, " a_kst");
        for (int j = 0; j < o.gemm.nk; ++j) fprintf(stderr, " %lld", (long long)o.gemm.a_kst[j]);
        fprintf(stderr, " b_kst");
        for (int j = 0; j < o.gemm.nk; ++j) fprintf(stderr, " %lld", (long long)o.gemm.b_kst[j]);
        fprintf(stderr, " c_mst");
        for (int j = 0; j < o.gemm.nm; ++j) fprintf(stderr, " %lld", (long long)o.gemm.c_mst[j]);
        fprintf(stderr, " c_nst");
        for (int j = 0; j < o.gemm.nn; ++j) fprintf(stderr, " %lld", (long long)o.gemm.c_nst[j]);
      }
      if (o.kind == OP_SIMT) {
        fprintf(stderr, " nout %d nk %d fixa %zu fixb %zu gath %d %d", o.simt.n_out, o.simt.n_k, o.fix_a.size(),
                o.fix_b.size(), o.gather_a, o.gather_b);
        fprintf(stderr, " a_os");
        for (int j = 0; j < o.simt.n_out; ++j) fprintf(stderr, " %lld", (long long)o.simt.a_os[j]);
        fprintf(stderr, " b_os");
        for (int j = 0; j < o.simt.n_out; ++j) fprintf(stderr, " %lld", (long long)o.simt.b_os[j]);
        fprintf(stderr, " a_ks");
        for (int j = 0; j < o.simt.n_k; ++j) fprintf(stderr, " %lld", (long long)o.simt.a_ks[j]);
        fprintf(stderr, " b_ks");
        for (int j = 0; j < o.simt.n_k; ++j) fprintf(stderr, " %lld", (long long)o.simt.b_ks[j]);
      }
      if (o.kind == OP_DOT) {
        fprintf(stderr, " K %lld nout %d a_os", (long long)o.dot.K, o.dot.n_out);
        for (int j = 0; j < o.dot.n_out; ++j) fprintf(stderr, " %lld", (long long)o.dot.a_os[j]);
        fprintf(stderr, " b_os");
        for (int j = 0; j < o.dot.n_out; ++j) fprintf(stderr, " %lld", (long long)o.dot.b_os[j]);
      }
      if (o.kind == OP_PERM) {
        fprintf(stderr, " in_pos");
        for (int j = 0; j < o.perm.rank; ++j) fprintf(stderr, " %d", o.perm.in_pos[j]);
      }
      fprintf(stderr, "\n");
    }
  }
  // root read-out
  {
    const Tensor& r = pc.tensors[pc.root];
    pc.root_sstride.assign(js, 0);
    pc.root_ostride.assign(pc.n_open, -1);
    GatherDesc g;
    g.tensor = pc.root;
    for (size_t i = 0; i < r.lay.size(); ++i) {
      const int lab = r.lay[i];
      if (pc.kind[lab] == KIND_SLICE && pc.aux[lab] < js) pc.root_sstride[pc.aux[lab]] = (int64_t)1 << i;
      else if (pc.open_bit[lab] >= 0) pc.root_ostride[pc.open_bit[lab]] = (int64_t)1 << i;
      else if (pc.kind[lab] == KIND_OUT && !r.batched) {
        g.q.push_back(pc.aux[lab]);
        g.stride.push_back((int64_t)1 << i);
      } else if (pc.kind[lab] != KIND_SLICE) {
        err = "internal: root carries an uncontracted index";
        return QX_ERR_INVALID_TREE;
      }
    }
    for (int j = 0; j < js; ++j)
      if (pc.root_sstride[j] == 0) {
        err = "internal: a varying sliced index does not reach the root";
        return QX_ERR_INVALID_TREE;
      }
    for (int i = 0; i < pc.n_open; ++i)
      if (pc.root_ostride[i] < 0) {
        err = "internal: an open output qubit does not reach the root";
        return QX_ERR_INVALID_TREE;
      }
    if (!g.q.empty()) {
      pc.gathers.push_back(g);
      pc.root_gather = (int)pc.gathers.size() - 1;
    }
  }
  for (auto& o : pc.ops) {
    if (o.phase == PH_BLOCK) {
      pc.flops_block += o.flops;
      if (o.kind == OP_GEMM) {
        pc.gemm_flops_block += o.flops;
        pc.n_gemm_block++;
      }
    } else if (o.phase == PH_CALL) {
      pc.flops_call += o.flops;
    }
  }
  return QX_OK;
}

}  // namespace qx
