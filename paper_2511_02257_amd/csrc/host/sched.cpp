// Contraction schedulers (Sec. III): input order, Sibling (Algs. 1-3), Tree
// (Algs. 4-8) and a node-based gain scheduler (the conclusions' future work),
// plus the Sec. II-C memory model.
//
// Readings where the paper is silent or garbled:
//   * Sibling picks the waiting leaf with the smallest id when all queues are
//     empty; queues are FIFO; the sibling subtree's leaves are brought in left
//     child first; "the sibling of u under v" is v's other child.
//   * Tree: TR-INIT accumulates the individual gains igain (not the counts g)
//     into tgain; PROCESS-CHILD removes u from x's AVAIL parents; ties in the
//     argmax go to the lowest tree index; PROCESS-CTREE visits each not yet
//     processed node of the tree once, in post-order, left child first.
//   * Input order and Tree take any number of children per node (in operand
//     order); Sibling, which uses a node's sibling, needs exactly two.
#include <algorithm>
#include <deque>
#include <functional>
#include <queue>

#include "host.hpp"
#include "../../../include/cdag.h"

namespace cdag {

std::vector<int64_t> sched_input(const Dag& d) {
  std::vector<char> done(d.n_nodes(), 0);
  std::vector<int64_t> order;
  order.reserve(d.n_nodes() - d.n_leaves);
  std::vector<std::pair<int64_t, int>> st;
  for (int64_t r : d.root_of_graph) {
    st.assign(1, {r, 0});
    while (!st.empty()) {
      auto [u, s] = st.back();
      st.pop_back();
      if (d.is_leaf(u) || done[u]) continue;
      if (s == 1) { done[u] = 1; order.push_back(u); continue; }
      st.push_back({u, 1});
      for (const int64_t* x = d.children_end(u); x != d.children_begin(u);) st.push_back({*--x, 0});
    }
  }
  return order;
}

// ---------------------------------------------------------------- Sibling
// Sibling (Sec. III-A) as an event machine.  Ready contractions wait in one
// FIFO per rank of Eq. (1); the highest non-empty rank runs next, and when
// every rank is empty the lowest-id leaf not yet in memory is brought in.  A
// tensor that arrives in memory (a leaf brought in, a contraction run) is an
// event for each of its parents in turn: the parent's count of missing
// children drops; with one child missing, the leaves still waiting in that
// sibling's subtree are brought in, depth first, left before right (each such
// leaf being an arrival of its own, handled before the next pending event);
// with none missing, the parent joins its rank's FIFO.  Pending work is kept
// on an explicit stack, so deep subtrees need no recursion.
namespace {
enum SbState : uint8_t { WAITING, QUEUED, INMEM, RELEASED };

class SiblingMachine {
 public:
  explicit SiblingMachine(const Dag& dd) : d(dd) {
    const int64_t n = d.n_nodes();
    for (int64_t u = d.n_leaves; u < n; ++u)
      if (d.n_children(u) != 2)
        throw Error(CDAG_E_INVALID, "sibling: node " + std::to_string(u) + " does not have two children");
    rank.assign(n, 0);
    int32_t top = 0;
    for (int64_t u = d.n_leaves; u < n; ++u) {   // Eq. (1); ids are topological
      rank[u] = 1 + std::max(rank[d.left[u]], rank[d.right[u]]);
      top = std::max(top, rank[u]);
    }
    users.resize(n);
    missing.resize(n);
    for (int64_t u = 0; u < n; ++u) {
      users[u] = d.n_parents(u);
      missing[u] = d.is_leaf(u) ? 0 : 2;
    }
    state.assign(n, WAITING);
    ready.resize(top + 1);
  }

  std::vector<int64_t> run() {
    const int64_t n_contr = d.n_nodes() - d.n_leaves;
    int64_t next_leaf = 0;
    while ((int64_t)order.size() < n_contr) {
      while (high >= 1 && ready[high].empty()) --high;
      if (high >= 1) {
        const int64_t v = ready[high].front();
        ready[high].pop_front();
        contract(v);
      } else {
        while (next_leaf < d.n_leaves && state[next_leaf] != WAITING) ++next_leaf;
        if (next_leaf >= d.n_leaves) throw Error(CDAG_E_STATE, "sibling: no waiting leaf left");
        bring(next_leaf);
      }
      drain();
    }
    return std::move(order);
  }

 private:
  // Stack work: NOTIFY walks the parents of an arrived tensor (edge = the next
  // parent edge); FETCH brings in the waiting leaves of a subtree.
  enum Kind : uint8_t { NOTIFY, FETCH };
  struct Work { Kind kind; int64_t node, edge; };

  const Dag& d;
  std::vector<int32_t> rank;
  std::vector<int64_t> users, missing;     // parents still to run; children not yet in memory
  std::vector<uint8_t> state;
  std::vector<std::deque<int64_t>> ready;  // FIFO per rank
  int32_t high = 0;                        // no rank above this one holds work
  std::vector<Work> stack;
  std::vector<int64_t> order;

  void arrived(int64_t u) {
    state[u] = INMEM;
    stack.push_back({NOTIFY, u, d.par_off[u]});
  }
  void bring(int64_t leaf) { arrived(leaf); }
  void contract(int64_t v) {
    order.push_back(v);
    arrived(v);
    for (int64_t c : {d.left[v], d.right[v]})
      if (--users[c] == 0) state[c] = RELEASED;
    if (d.n_parents(v) == 0) state[v] = RELEASED;   // a root's value leaves at once
  }
  void drain() {
    while (!stack.empty()) {
      Work& w = stack.back();
      if (w.kind == FETCH) {
        const int64_t u = w.node;
        stack.pop_back();
        if (state[u] != WAITING) continue;
        if (d.is_leaf(u)) {
          bring(u);
        } else {                                    // left subtree first
          stack.push_back({FETCH, d.right[u], 0});
          stack.push_back({FETCH, d.left[u], 0});
        }
        continue;
      }
      if (w.edge == d.par_off[w.node + 1]) {
        stack.pop_back();
        continue;
      }
      const int64_t u = w.node, v = d.par[w.edge++];
      if (--missing[v] == 1) {
        const int64_t sib = d.left[v] == u ? d.right[v] : d.left[v];
        if (state[sib] == WAITING) stack.push_back({FETCH, sib, 0});
      } else if (missing[v] == 0) {
        ready[rank[v]].push_back(v);
        state[v] = QUEUED;
        high = std::max(high, rank[v]);
      }
    }
  }
};
}  // namespace

std::vector<int64_t> sched_sibling(const Dag& d) { return SiblingMachine(d).run(); }

// ---------------------------------------------------------------- Tree
namespace {
enum TrState : uint8_t { AVAIL, TR_INMEM, TR_RELEASED };

// Per (node x, successor tree T): tau = unprocessed parents of x inside T.
// The paper's delta (unprocessed parents of x outside T) is not stored: it is
// out_av[x] - tau, so processing a parent outside T needs no per-tree update.
struct Pred { int64_t tree, tau; bool in_pred; };

struct TreeSched {
  const Dag& d;
  const int64_t k;
  std::vector<int64_t> size;
  std::vector<uint8_t> state;
  std::vector<int64_t> out_av;              // |u.outAv|
  std::vector<int64_t> igain;               // aligned with ctree: igain(T_i, u)
  std::vector<std::vector<Pred>> td;        // per node: one entry per successor tree, by tree
  // per node: tau value -> indices into td[node] (entries whose tau changed
  // since they were filed are stale and skipped)
  std::vector<std::vector<std::vector<int32_t>>> bucket;
  std::vector<int64_t> cnt;                 // scratch: per tree counter
  std::vector<int64_t> touched;             // scratch: trees with a nonzero counter
  std::vector<int64_t> tgain, cgain;
  std::vector<char> alive;
  // (tgain, -tree) entries of live trees in a max-heap; an entry whose gain
  // is no longer the tree's current gain, or whose tree is processed, is stale
  // and skipped when it reaches the top (the top is max tgain, lowest index)
  std::priority_queue<std::pair<int64_t, int64_t>> pq;
  std::vector<int64_t> order;
  std::vector<int64_t> visit_mark;

  TreeSched(const Dag& dd, int elem_bytes)
      : d(dd), k((int64_t)dd.tree_root.size()) {
    const int64_t n = d.n_nodes();
    size.resize(n);
    for (int64_t u = 0; u < n; ++u) size[u] = d.size(u, elem_bytes);
    visit_mark.assign(n, -1);
    cnt.assign(k, 0);
  }

  // cnt[t] = number of parents of u inside tree t (trees listed in touched).
  void count_parents_in_trees(int64_t u) {
    for (int64_t e = d.par_off[u]; e < d.par_off[u + 1]; ++e) {
      const int64_t p = d.par[e];
      for (int64_t j = d.ctree_off[p]; j < d.ctree_off[p + 1]; ++j) {
        const int64_t t = d.ctree[j];
        if (cnt[t]++ == 0) touched.push_back(t);
      }
    }
  }
  void clear_counts() {
    for (int64_t t : touched) cnt[t] = 0;
    touched.clear();
  }

  void set_gain(int64_t t, int64_t delta) {
    if (delta == 0) return;
    tgain[t] += delta;
    if (alive[t]) pq.push({tgain[t], -t});
  }

  void init() {                                   // TR-INIT
    const int64_t n = d.n_nodes();
    state.assign(n, AVAIL);
    out_av.resize(n);
    for (int64_t u = 0; u < n; ++u) out_av[u] = d.n_parents(u);
    tgain.assign(k, 0);
    cgain.assign(k, 0);
    alive.assign(k, 1);
    td.assign(n, {});
    bucket.assign(n, {});
    igain.assign(d.ctree.size(), 0);
    // g(u, T_i) = |outAv(u)| minus the edges (u, v) with v also in T_i, i.e.
    // the number of u's parents outside T_i.  Parents inside each tree are
    // counted from the parents' tree lists: O(sum over edges of |ctree|).
    for (int64_t u = 0; u < n; ++u) {
      count_parents_in_trees(u);
      for (int64_t j = d.ctree_off[u]; j < d.ctree_off[u + 1]; ++j) {
        const int64_t t = d.ctree[j];
        const int64_t g = out_av[u] - cnt[t];
        igain[j] = g == 0 ? 0 : -size[u];
        tgain[t] += igain[j];
      }
      clear_counts();
    }
    for (int64_t t = 0; t < k; ++t) pq.push({tgain[t], -t});
  }

  void process_child(int64_t u, int64_t x) {      // PROCESS-CHILD
    std::vector<Pred>& v = td[x];
    const int64_t a = out_av[x];                  // before u is counted as processed
    // Trees without u: delta = a - tau drops by one.  It reaches 0 (case 2.a)
    // exactly for the entries with tau == a - 1.
    if (a - 1 >= 1) {
      for (int32_t i : bucket[x][a - 1]) {
        const Pred& e = v[i];
        if (!e.in_pred || e.tau != a - 1 || d.in_tree(u, e.tree)) continue;
        cgain[e.tree] += size[x];
        set_gain(e.tree, +size[x]);
      }
    }
    // Trees with u: tau drops by one, delta stays (case 1).
    for (int64_t j = d.ctree_off[u]; j < d.ctree_off[u + 1]; ++j) {
      const int64_t t = d.ctree[j];
      const auto it = std::lower_bound(v.begin(), v.end(), t,
                                       [](const Pred& e, int64_t tr) { return e.tree < tr; });
      Pred& e = *it;                              // every tree of a parent of x has an entry
      if (!e.in_pred) continue;
      if (e.tau == 1 && a - e.tau == 0) {         // case 1.a
        cgain[t] -= size[x];
        set_gain(t, -size[x]);
      }
      if (--e.tau == 0)
        e.in_pred = false;
      else
        bucket[x][e.tau].push_back((int32_t)(it - v.begin()));
    }
    if (--out_av[x] == 0) state[x] = TR_RELEASED;
  }

  void process_node(int64_t u) {                  // PROCESS-NODE
    for (int64_t j = d.ctree_off[u]; j < d.ctree_off[u + 1]; ++j) set_gain(d.ctree[j], -igain[j]);
    // all of u's parents are AVAIL here (children are processed first)
    count_parents_in_trees(u);
    std::vector<Pred>& v = td[u];
    v.clear();
    std::sort(touched.begin(), touched.end());
    for (int64_t t : touched) v.push_back({t, cnt[t], true});
    clear_counts();
    auto& b = bucket[u];
    b.assign((size_t)d.n_parents(u) + 1, {});
    for (size_t i = 0; i < v.size(); ++i) {
      b[v[i].tau].push_back((int32_t)i);
      if (out_av[u] - v[i].tau == 0) {            // delta == 0
        cgain[v[i].tree] += size[u];
        set_gain(v[i].tree, +size[u]);
      }
    }
    state[u] = out_av[u] == 0 ? TR_RELEASED : TR_INMEM;
  }

  void process_ctree(int64_t t) {                 // PROCESS-CTREE
    std::vector<std::pair<int64_t, int>> st{{d.tree_root[t], 0}};
    while (!st.empty()) {
      auto [u, s] = st.back();
      st.pop_back();
      if (state[u] != AVAIL) continue;
      if (s == 1) {
        if (!d.is_leaf(u)) {
          for (const int64_t* x = d.children_begin(u); x != d.children_end(u); ++x) process_child(u, *x);
          order.push_back(u);
        }
        process_node(u);
        continue;
      }
      if (visit_mark[u] == t) continue;
      visit_mark[u] = t;
      st.push_back({u, 1});
      for (const int64_t* x = d.children_end(u); x != d.children_begin(u);) st.push_back({*--x, 0});
    }
  }

  // M - M' for tree t from the current states (no incremental fields).
  int64_t brute_gain(int64_t t) const {
    std::vector<int64_t> todo, touched;
    for (int64_t j = d.tree_off[t]; j < d.tree_off[t + 1]; ++j)
      if (state[d.tree_nodes[j]] == AVAIL) todo.push_back(d.tree_nodes[j]);
    std::sort(todo.begin(), todo.end());
    touched = todo;
    for (int64_t u : todo) touched.insert(touched.end(), d.children_begin(u), d.children_end(u));
    std::sort(touched.begin(), touched.end());
    touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
    auto in_todo = [&](int64_t x) { return std::binary_search(todo.begin(), todo.end(), x); };
    int64_t before = 0, after = 0;
    for (int64_t x : touched) {
      bool proc = state[x] != AVAIL;
      bool pending_b = false, pending_a = false;
      for (int64_t e = d.par_off[x]; e < d.par_off[x + 1]; ++e) {
        int64_t p = d.par[e];
        if (state[p] == AVAIL) {
          pending_b = true;
          if (!in_todo(p)) pending_a = true;
        }
      }
      if (proc && pending_b) before += size[x];
      if ((proc || in_todo(x)) && pending_a) after += size[x];
    }
    return before - after;
  }

  void run(bool check) {                          // TR-SCHEDULER
    init();
    for (int64_t it = 0; it < k; ++it) {
      if (check)
        for (int64_t t = 0; t < k; ++t)
          if (alive[t] && brute_gain(t) != tgain[t])
            throw Error(CDAG_E_STATE, "tree: incremental tgain of tree " + std::to_string(t) +
                                          " is " + std::to_string(tgain[t]) + ", M - M' is " +
                                          std::to_string(brute_gain(t)));
      while (!alive[-pq.top().second] || pq.top().first != tgain[-pq.top().second]) pq.pop();
      const int64_t best = -pq.top().second;      // max tgain, lowest index on ties
      pq.pop();
      alive[best] = 0;
      process_ctree(best);
    }
  }
};
}  // namespace

std::vector<int64_t> sched_tree(const Dag& d, int elem_bytes, bool check) {
  TreeSched s(d, elem_bytes);
  s.run(check);
  return std::move(s.order);
}

// ---------------------------------------------------------------- node gain
// Node-based gain scheduler: the Tree scheduler's gain M - M' (Sec. III-B)
// taken down to single contractions, as the conclusions propose.  Running v
// under the Sec. II-C model brings in v's leaf children that are not yet
// resident, adds v's output (nothing for a contraction without parents, whose
// output is released at once) and releases every child whose last pending
// parent is v, so gain(v) = released - brought - output.  A contraction is
// ready once its non-leaf children have run; the ready one with the largest
// gain runs next, ties to the lowest id.  Running v changes another node's
// gain in two cases only: a leaf child of v that v brought in no longer costs
// its other parents anything, and a child left with one pending parent is
// released by that parent.  Those gains are recomputed and pushed again (each
// leaf's parents are scanned once, each child's once when one parent is left,
// so O(E) scans in all); stale heap entries are skipped.
std::vector<int64_t> sched_node(const Dag& d, int elem_bytes, bool check) {
  const int64_t n = d.n_nodes();
  std::vector<int64_t> pending(n), waiting(n, 0), gain(n, 0);
  std::vector<char> resident(n, 0), done(n, 0);
  for (int64_t u = 0; u < n; ++u) pending[u] = d.n_parents(u);
  for (int64_t u = d.n_leaves; u < n; ++u)
    for (const int64_t* px = d.children_begin(u); px != d.children_end(u); ++px) waiting[u] += !d.is_leaf(*px);
  auto eval = [&](int64_t v) {
    int64_t g = d.n_parents(v) ? -d.size(v, elem_bytes) : 0;
    for (const int64_t* px = d.children_begin(v); px != d.children_end(v); ++px) {
      const int64_t sx = d.size(*px, elem_bytes);
      if (!resident[*px]) g -= sx;            // a leaf not brought in yet
      if (pending[*px] == 1) g += sx;         // v is its last pending parent
    }
    return g;
  };
  std::priority_queue<std::pair<int64_t, int64_t>> pq;   // (gain, -id): largest gain, then lowest id
  for (int64_t u = d.n_leaves; u < n; ++u)
    if (waiting[u] == 0) {
      gain[u] = eval(u);
      pq.push({gain[u], -u});
    }
  std::vector<int64_t> order;
  order.reserve(n - d.n_leaves);
  while (!pq.empty()) {
    const int64_t g = pq.top().first, v = -pq.top().second;
    pq.pop();
    if (done[v] || g != gain[v]) continue;
    if (check)   // every ready gain current, and v the largest (lowest id on ties)
      for (int64_t q = d.n_leaves; q < n; ++q) {
        if (done[q] || waiting[q] != 0) continue;
        const int64_t e = eval(q);
        if (e != gain[q]) throw Error(CDAG_E_STATE, "node scheduler: a stale gain at node " + std::to_string(q));
        if (e > g || (e == g && q < v)) throw Error(CDAG_E_STATE, "node scheduler: a better node was passed over");
      }
    done[v] = 1;
    order.push_back(v);
    auto refresh = [&](int64_t q) {
      if (done[q] || waiting[q] != 0) return;
      const int64_t ng = eval(q);
      if (ng != gain[q]) {
        gain[q] = ng;
        pq.push({ng, -q});
      }
    };
    for (const int64_t* px = d.children_begin(v); px != d.children_end(v); ++px) {
      const int64_t x = *px;
      const bool brought = !resident[x];
      resident[x] = --pending[x] > 0;
      if (pending[x] == 0) continue;
      if (brought) {
        for (int64_t pi = d.par_off[x]; pi < d.par_off[x + 1]; ++pi) refresh(d.par[pi]);
      } else if (pending[x] == 1) {
        for (int64_t pi = d.par_off[x]; pi < d.par_off[x + 1]; ++pi)
          if (!done[d.par[pi]]) {
            refresh(d.par[pi]);
            break;
          }
      }
    }
    resident[v] = pending[v] > 0;
    for (int64_t pi = d.par_off[v]; pi < d.par_off[v + 1]; ++pi) {
      const int64_t q = d.par[pi];
      if (--waiting[q] == 0) {
        gain[q] = eval(q);
        pq.push({gain[q], -q});
      }
    }
  }
  if ((int64_t)order.size() != n - d.n_leaves) throw Error(CDAG_E_STATE, "node scheduler: a contraction never became ready");
  return order;
}

// ---------------------------------------------------------------- memory model
MemSim memsim(const Dag& d, const std::vector<int64_t>& order, int elem_bytes) {
  const int64_t n = d.n_nodes();
  std::vector<int64_t> remaining(n);
  for (int64_t u = 0; u < n; ++u) remaining[u] = d.n_parents(u);
  std::vector<char> in_mem(n, 0), seen(n, 0);
  MemSim r;
  int64_t M = 0;
  if ((int64_t)order.size() != n - d.n_leaves) throw Error(CDAG_E_INVALID, "memsim: order must list every contraction once");
  for (int64_t c : order) {
    if (c < d.n_leaves || c >= n || seen[c]) throw Error(CDAG_E_INVALID, "memsim: order must list every contraction once");
    seen[c] = 1;
    int64_t brought = 0;
    for (const int64_t* px = d.children_begin(c); px != d.children_end(c); ++px) {
      const int64_t x = *px;
      if (!in_mem[x]) {
        if (!d.is_leaf(x)) throw Error(CDAG_E_INVALID, "memsim: order is not topological");
        in_mem[x] = 1;
        brought += d.size(x, elem_bytes);
      }
    }
    r.peak_live = std::max(r.peak_live, M + brought + d.size(c, elem_bytes));
    M += brought + d.size(c, elem_bytes);
    in_mem[c] = 1;
    for (const int64_t* px = d.children_begin(c); px != d.children_end(c); ++px)
      if (--remaining[*px] == 0) { in_mem[*px] = 0; M -= d.size(*px, elem_bytes); }
    if (remaining[c] == 0) { in_mem[c] = 0; M -= d.size(c, elem_bytes); }
    r.M.push_back(M);
    r.peak_post = std::max(r.peak_post, M);
  }
  return r;
}

}  // namespace cdag
