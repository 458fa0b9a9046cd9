// Host-side contraction-DAG data structures: the merged DAG (Sec. II-B), the
// schedulers (Sec. III), the memory model (Sec. II-C) and the budgeted plan.
// Pure C++17; no GPU calls.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace cdag {

// Named kinds K22, K32, K33 and the general contractions C1, C2, C3 of the
// last c axes of the left operand with the first c axes of the right one
// (operand and output ranks 2..4); a general contraction with the ranks of a
// named kind is stored as that kind.
// NARY marks a node of a general DAG (any number of children, sizes given
// by the caller), which is scheduled and simulated but never executed.
enum Kind : int32_t { K22 = 0, K32 = 1, K33 = 2, HCA = 3, C1 = 4, C2 = 5, C3 = 6, NARY = 7, LEAF = -1 };
constexpr int kMinRank = 2, kMaxRank = 4;
// Kind kSpecBase + i: a contraction over any index pairs, the context's spec i.
constexpr int32_t kSpecBase = 16;
inline bool is_spec(int32_t kind) { return kind >= kSpecBase; }

// A contraction over any index pairs (rank_l, rank_r operands): axis pair_l[k]
// of the left operand is summed against axis pair_r[k] of the right one; the
// output lists the left operand's free axes in order, then the right one's,
// and output axis j is axis perm[j] of that list.
struct Spec {
  int32_t rank_l, rank_r, n_pairs;
  int32_t pair_l[3], pair_r[3], perm[4];
};
inline int contracted_axes(int kind) {
  switch (kind) {
    case K22: case K32: case C1: return 1;
    case K33: case C2: return 2;
    case C3: return 3;
    default: return 0;
  }
}

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Structure-of-arrays DAG.  Ids: leaves 0..n_leaves-1, then contractions in
// order of first appearance, so every child id is smaller than its parent's.
struct Dag {
  int64_t n_leaves = 0;
  std::vector<int32_t> kind, rank, nvec, nt;
  std::vector<int64_t> left, right;         // binary nodes; -1 otherwise
  std::vector<int64_t> child_off, child;    // CSR children in operand order (left, right)
  std::vector<int64_t> par_off, par;        // CSR parents, one entry per edge, in creation order
  std::vector<int64_t> root_of_graph;       // per input graph
  std::vector<int64_t> tree_root;           // unique roots, first-appearance order
  std::vector<int64_t> tree_off, tree_nodes;  // per tree: node set in post-order (left first)
  std::vector<int64_t> ctree_off, ctree;    // per node: ascending tree indices containing it
  // per input graph: correlator id and weight
  std::vector<int32_t> corr;
  std::vector<double> w_re, w_im;
  std::vector<Spec> specs;                  // contraction specs (kinds kSpecBase + i)
  // A general DAG (build_general) carries per-node sizes in bytes instead of
  // tensor shapes; it can be scheduled and simulated, not planned or run.
  bool general = false;
  std::vector<int64_t> fixed_size;

  int64_t n_nodes() const { return (int64_t)kind.size(); }
  bool is_leaf(int64_t u) const { return kind[u] < 0; }
  int64_t n_parents(int64_t u) const { return par_off[u + 1] - par_off[u]; }
  int64_t n_children(int64_t u) const { return child_off[u + 1] - child_off[u]; }
  const int64_t* children_begin(int64_t u) const { return child.data() + child_off[u]; }
  const int64_t* children_end(int64_t u) const { return child.data() + child_off[u + 1]; }
  int64_t elems(int64_t u) const {
    int64_t e = nt[u];
    for (int r = 0; r < rank[u]; ++r) e *= nvec[u];
    return e;
  }
  // Bytes of u's tensor in a mode with elem_bytes per complex element; a root's
  // per-t scalar goes straight into the correlator buffer and counts 0.
  int64_t size(int64_t u, int elem_bytes) const {
    if (general) return fixed_size[u];
    return kind[u] == HCA ? 0 : elems(u) * elem_bytes;
  }
  bool in_tree(int64_t u, int64_t t) const;   // binary search in ctree(u)
  // Summed axes of contraction u (named, general or spec kind).
  int axes(int64_t u) const { return is_spec(kind[u]) ? specs[kind[u] - kSpecBase].n_pairs : contracted_axes(kind[u]); }
  // Algorithmic flops of contraction u (8 per complex multiply-add).
  double flops(int64_t u) const;
  // Exterior contraction u as a complex GEMM per time slice: M = N^(rl - c),
  // Ncols = N^(rr - c), K = N^c for operand ranks rl, rr and c contracted axes.
  void gemm_shape(int64_t u, int64_t* M, int64_t* Ncols, int64_t* K) const;
};

struct LeafIn { int32_t rank, nvec, nt; };
struct OpIn { int32_t kind, left, right; };
struct GraphIn { int32_t n_ops, corr; const OpIn* ops; double w_re, w_im; };

// specs: the contraction specs that op kinds kSpecBase + i name.  A spec equal
// to C1, C2 or C3 on its operands (the last c axes of the left one against the
// first c of the right one, in order, natural output order) is stored as that
// kind.
Dag build(const std::vector<LeafIn>& leaves, const std::vector<GraphIn>& graphs,
          const std::vector<Spec>& specs = {});
// A general DAG: nodes 0..n_leaves-1 are leaves, every other node lists its
// children (child_off/child, CSR, ids smaller than its own, no repeats) and
// size[u] is the bytes of u's tensor.  Trees are rooted at the non-leaf nodes
// without parents, in id order.  Throws Error(CDAG_E_INVALID) on bad input.
Dag build_general(int64_t n_nodes, int64_t n_leaves, const int64_t* size, const int64_t* child_off,
                  const int64_t* child);

std::vector<int64_t> sched_input(const Dag& d);
// Sibling needs every contraction to have exactly two children.
std::vector<int64_t> sched_sibling(const Dag& d);
// Tree scheduler; sizes in bytes of elem_bytes per element.  check=true
// recomputes each live tree's gain from scratch at every selection and throws
// Error(CDAG_E_STATE) on a mismatch with the incremental tgain.
std::vector<int64_t> sched_tree(const Dag& d, int elem_bytes, bool check);
// Node-based gain scheduler: the ready contraction with the largest gain
// M - M' under the memory model runs next (ties to the lowest id).  check=true
// recomputes every ready gain at each pick and throws Error(CDAG_E_STATE) if a
// cached gain is stale or the pick is not the largest.
std::vector<int64_t> sched_node(const Dag& d, int elem_bytes, bool check);

struct MemSim { std::vector<int64_t> M; int64_t peak_post = 0, peak_live = 0; };
MemSim memsim(const Dag& d, const std::vector<int64_t>& order, int elem_bytes);

// ---------------------------------------------------------------- plan
enum PlanOp : int32_t { OP_D2H = 0, OP_DROP = 1, OP_H2D = 2, OP_ALLOC = 3, OP_EXEC = 4, OP_FREE = 5 };

struct PlanRec {
  int32_t op;
  int64_t node, step;
  // physical placement (filled by place()): arena offset of the tensor's
  // allocation for H2D/ALLOC; host spill offset for D2H/H2D of intermediates.
  int64_t dev_off = -1, host_off = -1;
  // EXEC: arena offsets of the left and right operands (dev_off: the output).
  int64_t a_off = -1, b_off = -1;
  // Synchronisation between the three streams (compute, upload, spill), as
  // steps of the same chunk whose work must have finished (-1: none):
  //   D2H    wait_comp: kernels that last touched the tensor;
  //          wait_h2d:  an upload that last read the host range it writes;
  //   H2D    wait_comp: kernels that last touched the arena range it writes;
  //          wait_d2h:  a spill that last read that arena range, or that
  //                     wrote the tensor's host copy;
  //   ALLOC  wait_d2h:  a spill that last read the arena range (the kernels
  //                     of the step wait for it before writing the output).
  int64_t wait_comp = -1, wait_h2d = -1, wait_d2h = -1;
};

struct PlanOpts {
  int elem_bytes = 16;
  int64_t budget = INT64_MAX;
  bool batched = false;
  int64_t wave_max = 4096;
  int64_t lookahead = 0;
  bool leaves_resident = false;
  // Time-slice chunks: every contraction and trace acts on each time slice t
  // on its own, so the DAG can run as t_chunks passes over nt / t_chunks
  // slices of every tensor.  Passes alternate between two halves of the
  // budget, so the uploads of one pass overlap the kernels of the previous
  // one.  Each pass follows the same plan, made for tensors of
  // size / t_chunks bytes under budget / 2 (the whole budget when
  // t_chunks = 1).
  int64_t t_chunks = 1;
};

// Plan of one pass (t_chunks = 1: the whole execution).  Counters and the
// resident peak are those of one pass; plan_totals() gives the execution's.
struct Plan {
  PlanOpts opts;
  std::vector<std::vector<int64_t>> steps;  // contractions per step
  std::vector<PlanRec> recs;
  std::vector<int64_t> rec_off;             // per step: first record index
  int64_t peak_resident = 0, n_evict = 0, n_h2d = 0, h2d_bytes = 0, n_d2h = 0, d2h_bytes = 0;
  // placement
  int64_t pool_bytes = 0;                   // physical high-water of one pass's tensor pool
  int64_t host_spill_bytes = 0;             // host spill range of one pass
  std::vector<int64_t> leaf_off;            // leaves_resident: offsets in the leaf region
  int64_t leaf_region_bytes = 0;            // whole leaves (all time slices)
  int64_t chunks() const { return opts.t_chunks; }
  int64_t halves() const { return opts.t_chunks > 1 ? 2 : 1; }
  // Bytes of u's tensor in one pass.
  int64_t tsize(const Dag& d, int64_t u) const { return d.size(u, opts.elem_bytes) / opts.t_chunks; }
};

// Counters of the whole execution: one pass's times t_chunks; the resident
// peak of one pass per half of the budget in use.
struct PlanTotals { int64_t steps, peak_resident, n_evict, n_h2d, h2d_bytes, n_d2h, d2h_bytes; };
PlanTotals plan_totals(const Plan& p);

std::vector<std::vector<int64_t>> cut_waves(const Dag& d, const std::vector<int64_t>& order,
                                            const std::vector<int64_t>& size, int64_t budget,
                                            int64_t wave_max, int64_t lookahead);
// Throws Error(CDAG_E_INVALID) when t_chunks < 1 or does not divide the nt of
// every node, Error(CDAG_E_BUDGET) when a step does not fit.
Plan make_plan(const Dag& d, const std::vector<int64_t>& order, const PlanOpts& o);
// Assign arena offsets (256-byte aligned, best fit) and host spill offsets,
// and derive the cross-stream waits.
void place(const Dag& d, Plan& p);

}  // namespace cdag
