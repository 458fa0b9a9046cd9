// C ABI of the contraction-DAG engine (include/cdag.h).  Every entry point
// catches all exceptions and returns a status code.
#include <chrono>
#include <cstring>
#include <string>

#include "ctx.hpp"

struct cdag_ctx {
  cdag::Ctx c;
};

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}

template <class F>
int guard(F&& f) {
  try {
    g_err.clear();
    f();
    return CDAG_OK;
  } catch (const cdag::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(CDAG_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(CDAG_E_INVALID, e.what());
  } catch (...) {
    return fail(CDAG_E_INVALID, "unknown error");
  }
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void need(bool ok, int code, const char* m) {
  if (!ok) throw cdag::Error(code, m);
}

int elem_bytes_prec(int prec) {
  need(prec == CDAG_FP64 || prec == CDAG_FP32 || prec == CDAG_BF16X3 || prec == CDAG_BF16X6, CDAG_E_INVALID,
       "unknown precision");
  return prec == CDAG_FP64 ? 16 : 8;
}
}  // namespace

namespace cdag {
void ensure_plan(Ctx& c, int prec, int batched) {
  need(c.built, CDAG_E_STATE, "build_cdag first");
  need(!c.dag.general, CDAG_E_STATE, "a general DAG has no tensor shapes: it can be scheduled and simulated only");
  need(c.scheduled, CDAG_E_STATE, "schedule first");
  const int eb = elem_bytes_prec(prec);
  batched = batched ? 1 : 0;
  if (c.planned && c.plan_version == c.version && c.plan_prec == prec && c.plan_batched == batched) return;
  c.planned = false;
  double t0 = now();
  PlanOpts o;
  o.elem_bytes = eb;
  o.budget = c.budget;
  o.batched = batched != 0;
  o.wave_max = c.wave_max;
  o.lookahead = c.wave_lookahead;
  o.leaves_resident = c.leaves_resident;
  o.t_chunks = c.t_chunks;
  c.plan = make_plan(c.dag, c.order, o);
  place(c.dag, c.plan);
  c.kplan = make_kernel_plan(c.dag, c.plan, prec, c.tiles, c.fuse_traces);
  // host result buffers sized with the plan (an execute then writes them
  // without allocating)
  c.corr_host.resize(c.kplan.corr_bytes / 8);
  c.sums_host.resize(c.kplan.sums_bytes / 8);
  MemSim ms = memsim(c.dag, c.order, eb);
  c.peak_post = ms.peak_post;
  c.peak_live = ms.peak_live;
  c.t_plan = now() - t0;
  c.plan_version = c.version;
  c.plan_prec = prec;
  c.plan_batched = batched;
  c.plan_serial++;
  c.planned = true;
}
}  // namespace cdag

extern "C" {

const char* cdag_last_error(void) { return g_err.c_str(); }

int cdag_create(cdag_ctx** out) {
  if (!out) return fail(CDAG_E_INVALID, "out is NULL");
  return guard([&] { *out = new cdag_ctx(); });
}

int cdag_destroy(cdag_ctx* c) {
  if (!c) return CDAG_OK;
  return guard([&] {
    cdag::device_destroy(c->c.dev);
    c->c.dev = nullptr;
    delete c;
  });
}

int build_cdag(cdag_ctx* h, const cdag_leaf* leaves, int64_t n_leaves, const cdag_graph* graphs,
               int64_t n_graphs) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    need(n_leaves >= 0 && n_graphs >= 0, CDAG_E_INVALID, "negative count");
    need(n_leaves == 0 || leaves, CDAG_E_INVALID, "leaves is NULL");
    need(n_graphs == 0 || graphs, CDAG_E_INVALID, "graphs is NULL");
    need(n_leaves < (1LL << 31) && n_graphs < (1LL << 31), CDAG_E_INVALID, "too many leaves or graphs");
    cdag::Ctx& c = h->c;
    std::vector<cdag::LeafIn> L(n_leaves);
    int64_t with_data = 0;
    for (int64_t i = 0; i < n_leaves; ++i) {
      L[i] = {leaves[i].rank, leaves[i].nvec, leaves[i].nt};
      with_data += leaves[i].host != nullptr;
      need(leaves[i].dtype == CDAG_C128 || leaves[i].dtype == CDAG_C64, CDAG_E_INVALID, "leaf dtype must be C128 or C64");
    }
    need(with_data == 0 || with_data == n_leaves, CDAG_E_INVALID, "either every leaf has host data or none");
    std::vector<cdag::GraphIn> G(n_graphs);
    static_assert(sizeof(cdag::OpIn) == sizeof(cdag_op), "op layout");
    for (int64_t g = 0; g < n_graphs; ++g)
      G[g] = {graphs[g].n_ops, graphs[g].corr_id, reinterpret_cast<const cdag::OpIn*>(graphs[g].ops),
              graphs[g].w_re, graphs[g].w_im};
    cdag::Dag d = cdag::build(L, G, c.specs);
    // every correlator's graphs must share Nt
    int32_t n_corr = 0;
    for (int32_t x : d.corr) n_corr = std::max(n_corr, x + 1);
    std::vector<int32_t> cnt(n_corr, -1);
    for (size_t g = 0; g < d.corr.size(); ++g) {
      int32_t nt = d.nt[d.root_of_graph[g]];
      need(cnt[d.corr[g]] < 0 || cnt[d.corr[g]] == nt, CDAG_E_INVALID, "graphs of one correlator differ in Nt");
      cnt[d.corr[g]] = nt;
    }
    std::vector<std::vector<uint8_t>> data;
    std::vector<int32_t> dtypes(n_leaves);
    if (with_data) {
      data.resize(n_leaves);
      for (int64_t i = 0; i < n_leaves; ++i) {
        const int64_t bytes = d.elems(i) * (leaves[i].dtype == CDAG_C64 ? 8 : 16);
        const uint8_t* src = static_cast<const uint8_t*>(leaves[i].host);
        data[i].assign(src, src + bytes);
        dtypes[i] = leaves[i].dtype;
      }
    }
    c.dag = std::move(d);
    c.leaf_data = std::move(data);
    c.leaf_dtype = std::move(dtypes);
    c.has_data = with_data > 0 || n_leaves == 0;   // an empty DAG executes trivially
    c.n_corr = n_corr;
    c.built = true;
    c.data_version++;
    c.scheduled = false;
    c.planned = false;
    c.have_results = false;
    c.version++;
  });
}

int cdag_set_specs(cdag_ctx* h, const cdag_spec* specs, int64_t n) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    need(n >= 0 && n <= 1024 && (n == 0 || specs), CDAG_E_INVALID, "specs: 0..1024 entries, non-NULL");
    std::vector<cdag::Spec> v(n);
    static_assert(sizeof(cdag::Spec) == sizeof(cdag_spec), "spec layout");
    for (int64_t i = 0; i < n; ++i) std::memcpy(&v[i], &specs[i], sizeof(cdag_spec));
    h->c.specs = std::move(v);
  });
}

int cdag_build_general(cdag_ctx* h, int64_t n_nodes, int64_t n_leaves, const int64_t* size_bytes,
                       const int64_t* child_off, const int64_t* child) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    cdag::Ctx& c = h->c;
    cdag::Dag d = cdag::build_general(n_nodes, n_leaves, size_bytes, child_off, child);
    c.dag = std::move(d);
    c.leaf_data.clear();
    c.leaf_dtype.clear();
    c.has_data = false;
    c.n_corr = 0;
    c.built = true;
    c.data_version++;
    c.scheduled = false;
    c.planned = false;
    c.have_results = false;
    c.version++;
  });
}

int schedule(cdag_ctx* h, int policy, int64_t* order_out, int64_t cap, int64_t* n_out) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    cdag::Ctx& c = h->c;
    need(c.built, CDAG_E_STATE, "build_cdag first");
    const bool check = (policy & CDAG_SCHED_CHECK) != 0;
    const int p = policy & 0xff;
    double t0 = now();
    std::vector<int64_t> o;
    if (p == CDAG_SCHED_INPUT) o = cdag::sched_input(c.dag);
    else if (p == CDAG_SCHED_SIBLING) o = cdag::sched_sibling(c.dag);
    else if (p == CDAG_SCHED_TREE) o = cdag::sched_tree(c.dag, 16, check);
    else if (p == CDAG_SCHED_NODE) o = cdag::sched_node(c.dag, 16, check);
    else throw cdag::Error(CDAG_E_INVALID, "unknown policy");
    double t = now() - t0;
    if (n_out) *n_out = (int64_t)o.size();
    if (order_out) {
      need(cap >= (int64_t)o.size(), CDAG_E_RANGE, "order_out capacity too small");
      std::memcpy(order_out, o.data(), o.size() * sizeof(int64_t));
    }
    c.order = std::move(o);
    c.t_sched = t;
    c.scheduled = true;
    c.version++;
  });
}

int cdag_set_order(cdag_ctx* h, const int64_t* order, int64_t n) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    cdag::Ctx& c = h->c;
    need(c.built, CDAG_E_STATE, "build_cdag first");
    const cdag::Dag& d = c.dag;
    need(n == d.n_nodes() - d.n_leaves, CDAG_E_INVALID, "order must list every contraction once");
    need(n == 0 || order != nullptr, CDAG_E_INVALID, "order is NULL");
    std::vector<char> done(d.n_nodes(), 0);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t u = order[i];
      need(u >= d.n_leaves && u < d.n_nodes(), CDAG_E_INVALID, "order: id out of range or a leaf");
      need(!done[u], CDAG_E_INVALID, "order: a contraction is listed twice");
      for (const int64_t* px = d.children_begin(u); px != d.children_end(u); ++px)
        need(d.is_leaf(*px) || done[*px], CDAG_E_INVALID, "order: a contraction comes before its child");
      done[u] = 1;
    }
    c.order.assign(order, order + n);
    c.t_sched = 0.0;
    c.scheduled = true;
    c.version++;
  });
}

int set_mem_budget(cdag_ctx* h, uint64_t bytes) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    h->c.budget = bytes >= (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)bytes;
    h->c.version++;
  });
}

int cdag_set_options(cdag_ctx* h, int leaves_resident, int wave_max, int64_t wave_lookahead,
                     int use_graphs) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    need(wave_max >= 1, CDAG_E_INVALID, "wave_max must be >= 1");
    need(wave_lookahead >= 0, CDAG_E_INVALID, "wave_lookahead must be >= 0");
    need(use_graphs >= 0 && use_graphs <= 2, CDAG_E_INVALID, "use_graphs must be 0, 1 or 2");
    h->c.leaves_resident = leaves_resident != 0;
    h->c.wave_max = wave_max;
    h->c.wave_lookahead = wave_lookahead;
    h->c.use_graphs = use_graphs;
    h->c.version++;
  });
}

int cdag_set_time_chunks(cdag_ctx* h, int64_t t_chunks) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    need(t_chunks >= 1, CDAG_E_INVALID, "t_chunks must be >= 1");
    h->c.t_chunks = t_chunks;
    h->c.version++;
  });
}

int cdag_set_trace_fusion(cdag_ctx* h, int on) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    h->c.fuse_traces = on != 0;
    h->c.version++;
  });
}

int cdag_set_timing(cdag_ctx* h, int timing) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] { h->c.timing = timing != 0; });
}

int cdag_launch_records(cdag_ctx* h, cdag_launch_record* out, int64_t cap, int64_t* n_out) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    need(cap >= 0 && (cap == 0 || out != nullptr), CDAG_E_INVALID, "out is NULL");
    const auto& r = h->c.records;
    const int64_t n = std::min<int64_t>(cap, (int64_t)r.size());
    for (int64_t i = 0; i < n; ++i) out[i] = r[i];
    if (n_out) *n_out = (int64_t)r.size();
  });
}

int cdag_trace_execute(cdag_ctx* h, int prec, int batched, cdag_trace_rec* out, int64_t cap, int64_t* n_out,
                       int64_t fail_at) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    need(cap >= 0 && (cap == 0 || out != nullptr), CDAG_E_INVALID, "out is NULL");
    cdag::ensure_plan(h->c, prec, batched);
    std::vector<cdag_trace_rec> t;
    cdag::trace_execute(h->c, prec, t, fail_at);
    const int64_t n = std::min<int64_t>(cap, (int64_t)t.size());
    if (n > 0) std::memcpy(out, t.data(), (size_t)n * sizeof(cdag_trace_rec));
    if (n_out) *n_out = (int64_t)t.size();
  });
}

int cdag_set_tile(cdag_ctx* h, int prec, int kind, int nvec, int tile, int grid, int lds_stages, int split_k) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    elem_bytes_prec(prec);
    need(kind >= CDAG_K22 && kind <= CDAG_C3 && kind != CDAG_HCA, CDAG_E_INVALID,
         "kind must be an exterior contraction (K22, K32, K33, C1, C2, C3)");
    need(nvec >= 1, CDAG_E_INVALID, "nvec must be >= 1");
    need(tile >= -1 && tile < cdag::kNumTiles, CDAG_E_INVALID, "tile out of range");
    need(grid >= 0 && grid < cdag::kNumGrids, CDAG_E_INVALID, "grid must be 0 or 1");
    need(lds_stages == 1 || lds_stages == 2, CDAG_E_INVALID, "lds_stages must be 1 or 2");
    need(split_k == 0 || split_k == 1, CDAG_E_INVALID, "split_k must be 0 or 1");
    auto key = std::make_tuple(prec, kind, nvec);
    if (tile < 0)
      h->c.tiles.erase(key);
    else
      h->c.tiles[key] = cdag::choice_of(cdag::variant_of(tile, grid, lds_stages), split_k != 0);
    h->c.version++;
  });
}

int cdag_get_tile(cdag_ctx* h, int prec, int kind, int nvec, int* tile, int* grid, int* lds_stages,
                  int* split_k) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    elem_bytes_prec(prec);
    need(tile != nullptr && grid != nullptr && lds_stages != nullptr && split_k != nullptr, CDAG_E_INVALID,
         "NULL output");
    auto it = h->c.tiles.find(std::make_tuple(prec, kind, nvec));
    const int ch = it != h->c.tiles.end() ? it->second : cdag::default_tile(prec, kind, nvec);
    const int v = cdag::choice_variant(ch);
    *split_k = cdag::choice_split_k(ch) ? 1 : 0;
    *tile = cdag::variant_tile(v);
    *grid = cdag::variant_grid(v);
    *lds_stages = cdag::variant_stages(v);
  });
}

int cdag_memsim(cdag_ctx* h, const int64_t* order, int64_t n, int elem_bytes, int64_t* M_out,
                int64_t* peak_post, int64_t* peak_live) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    cdag::Ctx& c = h->c;
    need(c.built, CDAG_E_STATE, "build_cdag first");
    need(elem_bytes == 8 || elem_bytes == 16, CDAG_E_INVALID, "elem_bytes must be 8 or 16");
    need(n >= 0 && (n == 0 || order), CDAG_E_INVALID, "order is NULL");
    std::vector<int64_t> o(order, order + n);
    cdag::MemSim ms = cdag::memsim(c.dag, o, elem_bytes);
    if (M_out) std::memcpy(M_out, ms.M.data(), ms.M.size() * sizeof(int64_t));
    if (peak_post) *peak_post = ms.peak_post;
    if (peak_live) *peak_live = ms.peak_live;
  });
}

static void fill_plan_stats(const cdag::Ctx& c, cdag_plan_stats* s) {
  const cdag::Plan& p = c.plan;
  const cdag::PlanTotals t = cdag::plan_totals(p);
  std::memset(s, 0, sizeof(*s));
  s->n_nodes = c.dag.n_nodes();
  s->n_leaves = c.dag.n_leaves;
  s->n_contr = c.dag.n_nodes() - c.dag.n_leaves;
  s->n_roots = (int64_t)c.dag.tree_root.size();
  s->n_steps = t.steps;
  s->peak_post = c.peak_post;
  s->peak_live = c.peak_live;
  s->peak_resident = t.peak_resident;
  s->n_evict = t.n_evict;
  s->n_h2d = t.n_h2d;
  s->h2d_bytes = t.h2d_bytes;
  s->n_d2h = t.n_d2h;
  s->d2h_bytes = t.d2h_bytes;
  s->budget = c.budget;
  s->arena_bytes = c.kplan.total_bytes;
  s->tensor_highwater = p.leaf_region_bytes + p.halves() * p.pool_bytes;
  s->host_spill_bytes = p.halves() * p.host_spill_bytes;
  s->hec_items = c.kplan.hec_items;
  s->flops = c.kplan.flops;
  s->t_sched_s = c.t_sched;
  s->t_plan_s = c.t_plan;
}

int cdag_plan(cdag_ctx* h, int prec, int batched, cdag_plan_stats* out) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    cdag::ensure_plan(h->c, prec, batched);
    if (out) fill_plan_stats(h->c, out);
  });
}

int cdag_plan_ops(cdag_ctx* h, int32_t* op, int64_t* node, int64_t* step, int64_t cap, int64_t* n_out) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    const cdag::Ctx& c = h->c;
    need(c.planned, CDAG_E_STATE, "cdag_plan first");
    const auto& r = c.plan.recs;
    if (n_out) *n_out = (int64_t)r.size();
    if (op || node || step) {
      need(cap >= (int64_t)r.size(), CDAG_E_RANGE, "capacity too small");
      for (size_t i = 0; i < r.size(); ++i) {
        if (op) op[i] = r[i].op;
        if (node) node[i] = r[i].node;
        if (step) step[i] = r[i].step;
      }
    }
  });
}

int cdag_get_nodes(cdag_ctx* h, int32_t* kind, int64_t* left, int64_t* right, int64_t cap, int64_t* n_out) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    const cdag::Ctx& c = h->c;
    need(c.built, CDAG_E_STATE, "build_cdag first");
    const int64_t n = c.dag.n_nodes();
    if (n_out) *n_out = n;
    if (kind || left || right) {
      need(cap >= n, CDAG_E_RANGE, "capacity too small");
      for (int64_t u = 0; u < n; ++u) {
        if (kind) kind[u] = c.dag.kind[u];
        if (left) left[u] = c.dag.left[u];
        if (right) right[u] = c.dag.right[u];
      }
    }
  });
}

int cdag_graph_roots(cdag_ctx* h, int64_t* roots, int64_t cap) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    const cdag::Ctx& c = h->c;
    need(c.built, CDAG_E_STATE, "build_cdag first");
    need(roots != nullptr, CDAG_E_INVALID, "roots is NULL");
    need(cap >= (int64_t)c.dag.root_of_graph.size(), CDAG_E_RANGE, "capacity too small");
    std::memcpy(roots, c.dag.root_of_graph.data(), c.dag.root_of_graph.size() * sizeof(int64_t));
  });
}

int cdag_dag_stats(cdag_ctx* h, int64_t* n_vertices, int64_t* n_edges, int64_t* n_trees, double* f_v,
                   double* f_e) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    need(h->c.built, CDAG_E_STATE, "build_cdag first");
    const cdag::Dag& d = h->c.dag;
    const int64_t V = d.n_nodes(), E = (int64_t)d.child.size();
    double sv = 0, se = 0;
    for (int64_t u = 0; u < V; ++u) {
      const int64_t c = d.ctree_off[u + 1] - d.ctree_off[u];
      sv += (double)c;
      se += (double)d.n_children(u) * (double)c;
    }
    if (n_vertices) *n_vertices = V;
    if (n_edges) *n_edges = E;
    if (n_trees) *n_trees = (int64_t)d.tree_root.size();
    if (f_v) *f_v = V ? sv / (double)V : 0.0;
    if (f_e) *f_e = E ? se / (double)E : 0.0;
  });
}

int cdag_bind_device(cdag_ctx* h, int device, void* compute_stream, void* copy_stream) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    need(compute_stream && copy_stream && compute_stream != copy_stream, CDAG_E_INVALID,
         "two distinct non-NULL streams are required");
    cdag::device_bind(h->c, device, compute_stream, copy_stream);
  });
}

int cdag_bind_arena(cdag_ctx* h, void* arena, uint64_t bytes) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    need(arena != nullptr && bytes > 0, CDAG_E_INVALID, "arena is NULL or empty");
    need(((uintptr_t)arena & 255) == 0, CDAG_E_INVALID, "arena must be 256-byte aligned");
    cdag::device_bind_arena(h->c, arena, bytes);
  });
}

int execute(cdag_ctx* h, int prec, int batched, cdag_exec_stats* out) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    cdag::Ctx& c = h->c;
    need(c.built, CDAG_E_STATE, "build_cdag first");
    need(c.has_data, CDAG_E_STATE, "the DAG was built without leaf data");
    need(c.scheduled, CDAG_E_STATE, "schedule first");
    need(c.dev != nullptr, CDAG_E_STATE, "cdag_bind_device first");
    cdag::ensure_plan(c, prec, batched);
    cdag_exec_stats st;
    std::memset(&st, 0, sizeof(st));
    c.have_results = false;
    cdag::device_execute(c, prec, batched, &st);
    fill_plan_stats(c, &st.plan);
    c.have_results = true;
    if (out) *out = st;
  });
}

int cdag_execute_static(cdag_ctx* h, int prec, int batched, cdag_exec_stats* out) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    cdag::Ctx& c = h->c;
    need(c.built, CDAG_E_STATE, "build_cdag first");
    need(c.has_data, CDAG_E_STATE, "the DAG was built without leaf data");
    need(c.dev != nullptr, CDAG_E_STATE, "cdag_bind_device first");
    elem_bytes_prec(prec);
    static_assert(CDAG_STATIC_SCRATCH_BYTES == (64LL << 20), "scratch size in the header");
    // planning allocates host memory: the plan must exist already
    need(c.planned && c.plan_version == c.version && c.plan_prec == prec && c.plan_batched == (batched ? 1 : 0),
         CDAG_E_STATE, "cdag_plan for the same precision and batching first");
    c.have_results = false;
    cdag_exec_stats st;
    std::memset(&st, 0, sizeof(st));
    cdag::device_execute_static(c, prec, &st);
    fill_plan_stats(c, &st.plan);
    c.have_results = true;
    if (out) *out = st;
  });
}

int cdag_autotune(cdag_ctx* h, int prec, int batched, int reps, int mode, int64_t* n_tuned) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    cdag::Ctx& c = h->c;
    need(reps >= 1, CDAG_E_INVALID, "reps must be >= 1");
    need(mode >= 0 && mode <= 2, CDAG_E_INVALID, "mode must be 0 (synthetic), 1 (in situ) or 2 (synthetic, uniform)");
    need(c.dev != nullptr, CDAG_E_STATE, "cdag_bind_device first");
    need(mode == 0 || c.has_data, CDAG_E_STATE, "in-situ tuning needs leaf data");
    cdag::ensure_plan(c, prec, batched);
    int64_t n = mode == 1 ? cdag::device_autotune_insitu(c, prec, batched, reps)
                          : cdag::device_autotune(c, prec, batched, reps, mode == 2);
    c.version++;
    c.have_results = false;
    if (n_tuned) *n_tuned = n;
  });
}

int fetch_correlators(cdag_ctx* h, double* out, int64_t cap) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    const cdag::Ctx& c = h->c;
    need(c.have_results, CDAG_E_STATE, "execute first");
    need(out != nullptr, CDAG_E_INVALID, "out is NULL");
    const cdag::Dag& d = c.dag;
    std::vector<int64_t> tree_of(d.n_nodes(), -1);
    for (size_t t = 0; t < d.tree_root.size(); ++t) tree_of[d.tree_root[t]] = (int64_t)t;
    int64_t total = 0;
    for (int64_t r : d.root_of_graph) total += 2LL * d.nt[r];
    need(cap >= total, CDAG_E_RANGE, "capacity too small");
    int64_t o = 0;
    for (int64_t r : d.root_of_graph) {
      const int64_t off = c.kplan.tree_corr_off[tree_of[r]] / 8;
      std::memcpy(out + o, c.corr_host.data() + off, 2 * d.nt[r] * sizeof(double));
      o += 2LL * d.nt[r];
    }
  });
}

int cdag_fetch_sums(cdag_ctx* h, double* out, int64_t cap) {
  if (!h) return fail(CDAG_E_INVALID, "ctx is NULL");
  return guard([&] {
    const cdag::Ctx& c = h->c;
    need(c.have_results, CDAG_E_STATE, "execute first");
    need(out != nullptr, CDAG_E_INVALID, "out is NULL");
    int64_t total = 0;
    for (int32_t nt : c.kplan.sum_nt) total += 2LL * nt;
    need(cap >= total, CDAG_E_RANGE, "capacity too small");
    std::memcpy(out, c.sums_host.data(), total * sizeof(double));
  });
}

}  // extern "C"
