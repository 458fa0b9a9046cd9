// CDAG formation (Sec. II-B): merge binary contraction trees into one DAG by
// hash-consing structurally identical contractions.
#include <algorithm>
#include <climits>
#include <unordered_map>

#include "host.hpp"
#include "../../../include/cdag.h"

namespace cdag {

namespace {
struct KeyHash {
  size_t operator()(const std::tuple<int32_t, int64_t, int64_t>& k) const {
    uint64_t h = (uint64_t)std::get<0>(k) * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)std::get<1>(k) + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)std::get<2>(k) + 0x8CB92BA72F3D8DD7ull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

int64_t ipow(int64_t n, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= n;
  return r;
}

[[noreturn]] void invalid(const std::string& m) { throw Error(CDAG_E_INVALID, m); }

// Parents, tree node sets and per-node tree lists from the children and the
// tree roots.
void finish(Dag& d) {
  const int64_t n = d.n_nodes();
  // parents in edge-creation order: node by node, children in operand order
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t x : d.child) cnt[x]++;
  d.par_off.assign(n + 1, 0);
  for (int64_t u = 0; u < n; ++u) d.par_off[u + 1] = d.par_off[u] + cnt[u];
  d.par.assign(d.par_off[n], -1);
  std::vector<int64_t> fill(d.par_off.begin(), d.par_off.end() - 1);
  for (int64_t u = d.n_leaves; u < n; ++u)
    for (const int64_t* x = d.children_begin(u); x != d.children_end(u); ++x) d.par[fill[*x]++] = u;
  // tree node sets: post-order DFS from each unique root, children in order
  const int64_t k = (int64_t)d.tree_root.size();
  d.tree_off.assign(1, 0);
  std::vector<int64_t> mark(n, -1);
  std::vector<std::vector<int64_t>> ct(n);
  for (int64_t t = 0; t < k; ++t) {
    // iterative post-order: (node, state) pairs, state 0 = expand, 1 = emit
    std::vector<std::pair<int64_t, int>> st{{d.tree_root[t], 0}};
    while (!st.empty()) {
      auto [u, s] = st.back();
      st.pop_back();
      if (s == 1) { d.tree_nodes.push_back(u); ct[u].push_back(t); continue; }
      if (mark[u] == t) continue;
      mark[u] = t;
      st.push_back({u, 1});
      for (const int64_t* x = d.children_end(u); x != d.children_begin(u);) st.push_back({*--x, 0});
    }
    d.tree_off.push_back((int64_t)d.tree_nodes.size());
  }
  d.ctree_off.assign(n + 1, 0);
  for (int64_t u = 0; u < n; ++u) d.ctree_off[u + 1] = d.ctree_off[u] + (int64_t)ct[u].size();
  d.ctree.reserve(d.ctree_off[n]);
  for (int64_t u = 0; u < n; ++u) d.ctree.insert(d.ctree.end(), ct[u].begin(), ct[u].end());
}
}  // namespace

bool Dag::in_tree(int64_t u, int64_t t) const {
  return std::binary_search(ctree.begin() + ctree_off[u], ctree.begin() + ctree_off[u + 1], t);
}

void Dag::gemm_shape(int64_t u, int64_t* M, int64_t* Ncols, int64_t* K) const {
  const int c = axes(u);
  const int64_t n = nvec[u];
  *M = ipow(n, rank[left[u]] - c);
  *Ncols = ipow(n, rank[right[u]] - c);
  *K = ipow(n, c);
}

double Dag::flops(int64_t u) const {
  if (kind[u] < 0) return 0.0;
  if (kind[u] == HCA) return 8.0 * nt[u] * (double)nvec[u] * nvec[u];
  int64_t M, N, K;
  gemm_shape(u, &M, &N, &K);
  return 8.0 * nt[u] * (double)M * (double)N * (double)K;
}

// Checks spec s against operand ranks (rl, rr); returns its output rank and
// sets *canonical when it is C_c in the engine's own order.
static int check_spec(const Spec& s, int rl, int rr, const std::string& where, bool* canonical) {
  if (s.rank_l != rl || s.rank_r != rr) invalid(where + "operand ranks differ from the spec's");
  const int c = s.n_pairs, ro = rl + rr - 2 * c;
  if (c < 1 || c > 3 || ro < kMinRank || ro > kMaxRank) invalid(where + "spec ranks out of range");
  int seen_l = 0, seen_r = 0;
  bool canon = true;
  for (int k = 0; k < c; ++k) {
    const int a = s.pair_l[k], b = s.pair_r[k];
    if (a < 0 || a >= rl || b < 0 || b >= rr || (seen_l >> a & 1) || (seen_r >> b & 1))
      invalid(where + "spec axes out of range or repeated");
    seen_l |= 1 << a;
    seen_r |= 1 << b;
    canon = canon && a == rl - c + k && b == k;
  }
  int seen_o = 0;
  for (int j = 0; j < ro; ++j) {
    const int q = s.perm[j];
    if (q < 0 || q >= ro || (seen_o >> q & 1)) invalid(where + "spec perm is not a permutation of the output axes");
    seen_o |= 1 << q;
    canon = canon && q == j;
  }
  *canonical = canon;
  return ro;
}

Dag build(const std::vector<LeafIn>& leaves, const std::vector<GraphIn>& graphs, const std::vector<Spec>& specs) {
  Dag d;
  d.n_leaves = (int64_t)leaves.size();
  d.specs = specs;
  for (const auto& l : leaves) {
    if (l.rank < kMinRank || l.rank > kMaxRank || l.nvec < 1 || l.nt < 1)
      invalid("leaf: rank must be 2..4, nvec and nt >= 1");
    d.kind.push_back(LEAF);
    d.rank.push_back(l.rank);
    d.nvec.push_back(l.nvec);
    d.nt.push_back(l.nt);
    d.left.push_back(-1);
    d.right.push_back(-1);
  }
  std::unordered_map<std::tuple<int32_t, int64_t, int64_t>, int64_t, KeyHash> table;
  std::vector<int64_t> local, consumed;
  std::vector<char> root_seen;
  for (size_t gi = 0; gi < graphs.size(); ++gi) {
    const GraphIn& g = graphs[gi];
    if (g.n_ops < 1 || !g.ops) invalid("graph " + std::to_string(gi) + ": no ops");
    if (g.corr < 0) invalid("graph " + std::to_string(gi) + ": negative corr_id");
    local.assign(g.n_ops, -1);
    consumed.assign(g.n_ops, 0);
    for (int32_t oi = 0; oi < g.n_ops; ++oi) {
      const OpIn& op = g.ops[oi];
      std::string where = "graph " + std::to_string(gi) + " op " + std::to_string(oi) + ": ";
      if ((op.kind < K22 || op.kind > C3) && !(is_spec(op.kind) && op.kind - kSpecBase < (int64_t)specs.size()))
        invalid(where + "unknown kind");
      if ((op.kind == HCA) != (oi == g.n_ops - 1)) invalid(where + "the root, and only the root, must be HCA");
      int64_t ids[2];
      const int32_t xs[2] = {op.left, op.right};
      for (int s = 0; s < 2; ++s) {
        int32_t x = xs[s];
        if (x >= 0) {
          if (x >= d.n_leaves) invalid(where + "leaf id out of range");
          ids[s] = x;
        } else {
          int64_t j = -(int64_t)x - 1;
          if (j >= oi) invalid(where + "forward or self reference");
          consumed[j] += 1;
          ids[s] = local[j];
        }
      }
      if (ids[0] == ids[1]) invalid(where + "identical operands");
      const int rl = d.rank[ids[0]], rr = d.rank[ids[1]];
      int32_t kind = op.kind;
      int ro;
      if (kind == HCA) {
        if (rl != 2 || rr != 2) invalid(where + "operand rank mismatch");
        ro = 0;
      } else {
        int c;
        if (is_spec(kind)) {
          const Spec& sp = specs[kind - kSpecBase];
          bool canonical = false;
          ro = check_spec(sp, rl, rr, where, &canonical);
          c = sp.n_pairs;
          if (canonical) kind = c == 1 ? C1 : c == 2 ? C2 : C3;
        } else {
          c = contracted_axes(kind);
          ro = rl + rr - 2 * c;
        }
        if (kind == K22 && (rl != 2 || rr != 2)) invalid(where + "operand rank mismatch");
        if (kind == K32 && (rl != 3 || rr != 2)) invalid(where + "operand rank mismatch");
        if (kind == K33 && (rl != 3 || rr != 3)) invalid(where + "operand rank mismatch");
        if (ro < kMinRank || ro > kMaxRank) invalid(where + "output rank out of range");
        const int64_t n = d.nvec[ids[0]];
        if (ipow(n, std::max(std::max(rl - c, rr - c), c)) > (int64_t)INT32_MAX)
          invalid(where + "a GEMM dimension of the contraction exceeds 2^31");
        // a general contraction with the ranks of a named kind is that kind
        if (kind == C1 && rl == 2 && rr == 2) kind = K22;
        if (kind == C1 && rl == 3 && rr == 2) kind = K32;
        if (kind == C2 && rl == 3 && rr == 3) kind = K33;
      }
      if (d.nvec[ids[0]] != d.nvec[ids[1]] || d.nt[ids[0]] != d.nt[ids[1]])
        invalid(where + "operand N or Nt mismatch");
      auto key = std::make_tuple(kind, ids[0], ids[1]);
      auto it = table.find(key);
      int64_t u;
      if (it == table.end()) {
        u = d.n_nodes();
        table.emplace(key, u);
        d.kind.push_back(kind);
        d.rank.push_back(ro);
        d.nvec.push_back(d.nvec[ids[0]]);
        d.nt.push_back(d.nt[ids[0]]);
        d.left.push_back(ids[0]);
        d.right.push_back(ids[1]);
      } else {
        u = it->second;
      }
      local[oi] = u;
    }
    for (int32_t oi = 0; oi + 1 < g.n_ops; ++oi)
      if (consumed[oi] != 1)
        invalid("graph " + std::to_string(gi) + ": every non-root op must be used exactly once");
    int64_t root = local[g.n_ops - 1];
    d.root_of_graph.push_back(root);
    d.corr.push_back(g.corr);
    d.w_re.push_back(g.w_re);
    d.w_im.push_back(g.w_im);
    if ((int64_t)root_seen.size() < d.n_nodes()) root_seen.resize(d.n_nodes(), 0);
    if (!root_seen[root]) {
      root_seen[root] = 1;
      d.tree_root.push_back(root);
    }
  }
  const int64_t n = d.n_nodes();
  d.child_off.assign(n + 1, 0);
  for (int64_t u = 0; u < n; ++u) d.child_off[u + 1] = d.child_off[u] + (d.is_leaf(u) ? 0 : 2);
  d.child.reserve(d.child_off[n]);
  for (int64_t u = d.n_leaves; u < n; ++u) {
    d.child.push_back(d.left[u]);
    d.child.push_back(d.right[u]);
  }
  finish(d);
  return d;
}

Dag build_general(int64_t n_nodes, int64_t n_leaves, const int64_t* size, const int64_t* child_off,
                  const int64_t* child) {
  if (n_leaves < 0 || n_nodes < n_leaves || n_nodes >= (1LL << 31)) invalid("general: need 0 <= n_leaves <= n_nodes < 2^31");
  if (n_nodes > 0 && (!size || !child_off)) invalid("general: size or child_off is NULL");
  if (n_nodes > 0 && child_off[0] != 0) invalid("general: child_off[0] must be 0");
  Dag d;
  d.general = true;
  d.n_leaves = n_leaves;
  d.kind.assign(n_nodes, NARY);
  d.rank.assign(n_nodes, 0);
  d.nvec.assign(n_nodes, 0);
  d.nt.assign(n_nodes, 0);
  d.left.assign(n_nodes, -1);
  d.right.assign(n_nodes, -1);
  d.fixed_size.assign(size, size + n_nodes);
  d.child_off.assign(n_nodes + 1, 0);
  std::vector<int64_t> last_parent(n_nodes, -1);
  for (int64_t u = 0; u < n_nodes; ++u) {
    const std::string where = "general: node " + std::to_string(u) + ": ";
    if (size[u] < 0) invalid(where + "negative size");
    const int64_t b = child_off[u], e = child_off[u + 1];
    if (e < b) invalid(where + "child_off must not decrease");
    if (u < n_leaves) {
      if (e != b) invalid(where + "a leaf has no children");
      d.kind[u] = LEAF;
    } else {
      if (e == b) invalid(where + "a non-leaf node needs at least one child");
      if (!child) invalid("general: child is NULL");
      for (int64_t j = b; j < e; ++j) {
        const int64_t x = child[j];
        if (x < 0 || x >= u) invalid(where + "child ids must lie in [0, u)");
        if (last_parent[x] == u) invalid(where + "repeated child");
        last_parent[x] = u;
        d.child.push_back(x);
      }
      if (e - b == 2) {
        d.left[u] = child[b];
        d.right[u] = child[b + 1];
      }
    }
    d.child_off[u + 1] = (int64_t)d.child.size();
  }
  std::vector<char> has_parent(n_nodes, 0);
  for (int64_t x : d.child) has_parent[x] = 1;
  for (int64_t u = n_leaves; u < n_nodes; ++u)
    if (!has_parent[u]) d.tree_root.push_back(u);
  d.root_of_graph = d.tree_root;
  finish(d);
  return d;
}

}  // namespace cdag
