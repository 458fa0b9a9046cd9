// Drives every host entry point of the C ABI on seeded DAGs (meson rings,
// baryon chains, general DAGs) and on malformed input; built with
// -fsanitize=address,undefined by tests/test_host_sanitizers.py.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "cdag.h"

namespace {
uint64_t g_state = 0x9e3779b97f4a7c15ULL;
uint64_t next_u64() {                       // splitmix64
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
int pick(int n) { return (int)(next_u64() % (uint64_t)n); }

int g_fail = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (%s)\n", what, cdag_last_error());
    g_fail = 1;
  }
}

// Meson rings over leaves [0, nm) (rank 2) and baryon chains over baryons
// [nm, nm + nb) (rank 3); all leaves N = n, Nt = nt, no host data.
void build_mixed(cdag_ctx* c, int nm, int nb, int n_graphs, int n) {
  std::vector<cdag_leaf> leaves;
  for (int i = 0; i < nm; ++i) leaves.push_back({2, n, 2, CDAG_C128, nullptr});
  for (int i = 0; i < nb; ++i) leaves.push_back({3, n, 2, CDAG_C128, nullptr});
  std::vector<std::vector<cdag_op>> ops(n_graphs);
  std::vector<cdag_graph> graphs(n_graphs);
  for (int g = 0; g < n_graphs; ++g) {
    std::vector<cdag_op>& o = ops[g];
    if (nb >= 2 && g % 3 == 2) {
      const int a = nm + pick(nb), b = pick(nm);
      int c2 = nm + pick(nb - 1);
      if (c2 >= a) ++c2;
      int d = pick(nm - 1);
      if (d >= b) ++d;
      o.push_back({CDAG_K32, a, b});
      o.push_back({CDAG_K33, -1, c2});
      o.push_back({CDAG_HCA, -2, d});
    } else {
      const int len = 3 + pick(4);
      std::vector<int> seq;
      while ((int)seq.size() < len) {
        const int x = pick(nm);
        bool dup = false;
        for (int y : seq) dup |= y == x;
        if (!dup) seq.push_back(x);
      }
      int cur = seq[0];
      for (int k = 1; k + 1 < len; ++k) {
        o.push_back({CDAG_K22, cur, seq[k]});
        cur = -(int)o.size();
      }
      o.push_back({CDAG_HCA, cur, seq[len - 1]});
    }
    graphs[g] = cdag_graph{(int32_t)o.size(), g % 3, o.data(), 1.0, 0.0};
  }
  expect(build_cdag(c, leaves.data(), (int64_t)leaves.size(), graphs.data(), n_graphs) == CDAG_OK, "build_cdag");
}

void exercise(cdag_ctx* c, bool general_dag) {
  int64_t nv = 0, ne = 0, nt = 0;
  double fv = 0, fe = 0;
  expect(cdag_dag_stats(c, &nv, &ne, &nt, &fv, &fe) == CDAG_OK, "dag_stats");
  for (int policy = 0; policy <= 3; ++policy) {
    int64_t n = 0;
    if (schedule(c, policy, nullptr, 0, &n) != CDAG_OK) continue;   // Sibling may refuse
    std::vector<int64_t> order(n), M(n);
    expect(schedule(c, policy | (policy == 2 ? CDAG_SCHED_CHECK : 0), order.data(), n, &n) == CDAG_OK, "schedule");
    int64_t pp = 0, pl = 0;
    expect(cdag_memsim(c, order.data(), n, 16, M.data(), &pp, &pl) == CDAG_OK, "memsim");
    expect(cdag_set_order(c, order.data(), n) == CDAG_OK, "set_order");
    for (uint64_t frac : {0ULL, 3ULL, 6ULL}) {
      set_mem_budget(c, frac ? (uint64_t)pl / frac : UINT64_MAX);
      for (int batched = 0; batched <= 1; ++batched)
        for (int resident = 0; resident <= 1; ++resident) {
          cdag_set_options(c, resident, 64, batched ? 4 : 0, 1);
          cdag_plan_stats ps;
          const int rc = cdag_plan(c, CDAG_FP64, batched, &ps);
          if (general_dag) {
            expect(rc == CDAG_E_STATE, "a general DAG is not planned");
            continue;
          }
          expect(rc == CDAG_OK || rc == CDAG_E_BUDGET, "plan");
          if (rc != CDAG_OK) continue;
          int64_t m = 0;
          expect(cdag_plan_ops(c, nullptr, nullptr, nullptr, 0, &m) == CDAG_OK, "plan_ops count");
          std::vector<int32_t> op(m);
          std::vector<int64_t> node(m), step(m);
          expect(cdag_plan_ops(c, op.data(), node.data(), step.data(), m, &m) == CDAG_OK, "plan_ops");
        }
    }
    set_mem_budget(c, UINT64_MAX);
  }
  int64_t m = 0;
  expect(cdag_get_nodes(c, nullptr, nullptr, nullptr, 0, &m) == CDAG_OK, "get_nodes count");
  std::vector<int32_t> kind(m);
  std::vector<int64_t> l(m), r(m);
  expect(cdag_get_nodes(c, kind.data(), l.data(), r.data(), m, &m) == CDAG_OK, "get_nodes");
  cdag_exec_stats es;
  expect(execute(c, CDAG_FP64, 1, &es) != CDAG_OK, "execute without a device fails");
}

void general(cdag_ctx* c, int n_leaves, int n_inner) {
  std::vector<int64_t> size, off{0}, child;
  for (int u = 0; u < n_leaves; ++u) { size.push_back(1 + pick(1000)); off.push_back(0); }
  for (int u = n_leaves; u < n_leaves + n_inner; ++u) {
    const int k = 1 + pick(4);
    std::vector<int64_t> kids;
    while ((int)kids.size() < k) {
      const int64_t x = pick(u);
      bool dup = false;
      for (int64_t y : kids) dup |= y == x;
      if (!dup) kids.push_back(x);
    }
    for (int64_t x : kids) child.push_back(x);
    size.push_back(pick(1001));
    off.push_back((int64_t)child.size());
  }
  expect(cdag_build_general(c, n_leaves + n_inner, n_leaves, size.data(), off.data(), child.data()) == CDAG_OK,
         "build_general");
}

void malformed(cdag_ctx* c) {
  cdag_leaf L[3] = {{2, 4, 1, CDAG_C128, nullptr}, {2, 4, 1, CDAG_C128, nullptr}, {3, 4, 1, CDAG_C128, nullptr}};
  const cdag_op bad[][2] = {{{CDAG_K22, 0, 0}, {CDAG_HCA, -1, 1}},  {{CDAG_K22, 0, 9}, {CDAG_HCA, -1, 1}},
                            {{CDAG_K22, 0, -2}, {CDAG_HCA, -1, 1}}, {{CDAG_HCA, 0, 1}, {CDAG_K22, 0, 1}},
                            {{CDAG_K22, 2, 1}, {CDAG_HCA, -1, 1}},  {{7, 0, 1}, {CDAG_HCA, -1, 1}}};
  for (const auto& ops : bad) {
    cdag_graph g = {2, 0, ops, 1.0, 0.0};
    expect(build_cdag(c, L, 3, &g, 1) == CDAG_E_INVALID, "malformed graph refused");
  }
  expect(build_cdag(c, nullptr, 3, nullptr, 1) == CDAG_E_INVALID, "NULL arrays refused");
  const int64_t sz[3] = {1, 1, 1}, off[4] = {0, 0, 0, 2}, dup[2] = {0, 0};
  expect(cdag_build_general(c, 3, 2, sz, off, dup) == CDAG_E_INVALID, "repeated child refused");
  const int64_t order[1] = {0};
  expect(cdag_set_order(c, order, 1) != CDAG_OK, "bad order refused");
  expect(cdag_set_specs(c, nullptr, 2) == CDAG_E_INVALID, "NULL specs refused");
}

// Contractions over index pairs: a chain through a spec on two baryons
// (pairs (2,0) and (0,2), output reversed), scheduled and planned; then a
// spec that does not fit its operands.
void index_pairs(cdag_ctx* c) {
  const cdag_spec specs[2] = {{3, 3, 2, {2, 0, 0}, {0, 2, 0}, {1, 0, 0, 0}},
                              {3, 2, 1, {0, 0, 0}, {1, 0, 0}, {2, 0, 1, 0}}};
  expect(cdag_set_specs(c, specs, 2) == CDAG_OK, "set_specs");
  cdag_leaf L[4] = {{3, 4, 2, CDAG_C128, nullptr}, {3, 4, 2, CDAG_C128, nullptr},
                    {2, 4, 2, CDAG_C128, nullptr}, {2, 4, 2, CDAG_C128, nullptr}};
  const cdag_op ops[3] = {{CDAG_SPEC_BASE + 1, 0, 2}, {CDAG_SPEC_BASE, -1, 1}, {CDAG_HCA, -2, 3}};
  cdag_graph g = {3, 0, ops, 1.0, 0.0};
  expect(build_cdag(c, L, 4, &g, 1) == CDAG_OK, "build with specs");
  int64_t n = 0;
  expect(schedule(c, CDAG_SCHED_TREE, nullptr, 0, &n) == CDAG_OK && n == 3, "schedule with specs");
  cdag_plan_stats st;
  expect(cdag_plan(c, CDAG_FP64, 1, &st) == CDAG_OK, "plan with specs");
  expect(cdag_plan(c, CDAG_BF16X3, 1, &st) == CDAG_E_INVALID, "split-BF16 refuses specs");
  std::vector<cdag_plan_stats> again(1);
  expect(cdag_plan(c, CDAG_FP32, 0, again.data()) == CDAG_OK, "per-contraction plan with specs");
  const cdag_op wrong[2] = {{CDAG_SPEC_BASE + 1, 0, 1}, {CDAG_HCA, -1, 3}};
  cdag_graph w = {2, 0, wrong, 1.0, 0.0};
  expect(build_cdag(c, L, 4, &w, 1) == CDAG_E_INVALID, "spec on the wrong ranks refused");
  expect(cdag_set_specs(c, nullptr, 0) == CDAG_OK, "clear specs");
}
}  // namespace

int main() {
  cdag_ctx* c = nullptr;
  expect(cdag_create(&c) == CDAG_OK, "create");
  for (int round = 0; round < 6; ++round) {
    build_mixed(c, 6 + round, round % 3 == 0 ? 0 : 3 + round % 2, 20 + 15 * round, 3 + round % 3);
    exercise(c, false);
    general(c, 5 + round, 20 + 10 * round);
    exercise(c, true);
  }
  malformed(c);
  index_pairs(c);
  build_mixed(c, 8, 4, 40, 4);
  exercise(c, false);
  expect(cdag_destroy(c) == CDAG_OK, "destroy");
  if (!g_fail) std::printf("sanitizer driver: ok\n");
  return g_fail;
}
