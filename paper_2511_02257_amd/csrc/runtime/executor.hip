// Device runtime: leaf staging in pinned host memory, the arena borrowed from
// the caller, and execution of a placed plan on three HIP streams.
//
// Eager execution: per step s the spill stream copies the step's evicted
// intermediates to the host (D2H) and records ev_d2h[s]; the upload stream
// copies its missing operands in (H2D) and records ev_h2d[s]; the compute
// stream waits for the uploads of the step (and, where an output reuses
// memory a spill was still reading, for that spill), launches the step's
// kernels and records ev_comp[s].  A transfer into memory that kernels last
// touched at step k first waits for ev_comp[k]; an upload into memory a spill
// was reading, or of a tensor a spill wrote out, waits for that spill; a
// spill into host memory an upload was reading waits for that upload.  All
// waits come from the plan (place()), so uploads, spills and kernels overlap
// whenever the memory they use is already free.
// Time-slice passes (t_chunks > 1) repeat the plan on slices of every tensor,
// alternating between two halves of the memory; a pass waits for the one two
// before it (same half) to be done with that half.
// Graph replay: the same walk captured on one stream (segments of steps, the
// stream order carries every dependency), or added to one graph node by node
// with the walk's waits as explicit edges (no capture).  The eager walk can also be
// recorded instead of issued (trace_execute), so that its ordering can be
// checked on a host without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <cstdlib>
#include <thread>
#include <tuple>

#include "../ctx.hpp"
#include "../kernels/kernels.hpp"

namespace cdag {

namespace {
inline void ignore_last_error() { (void)hipGetLastError(); }
// A failed call also leaves its code as the thread's last error; it is read
// (and so cleared) here, or a later launch check would report it again.
void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    ignore_last_error();
    throw Error(CDAG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  }
}
#define HIPC(x) hip_check((x), #x)
inline void ignore(hipError_t) {}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Stream roles; trace records and event ids use these numbers.
enum StreamRole : int { S_COMP = 0, S_H2D = 1, S_D2H = 2, kStreams = 3 };
}  // namespace

// ---------------------------------------------------------------- static scratch
// Device memory for cdag_execute_static, which allocates nothing: a fixed
// array that every GPU the library runs on holds until the process ends.  In
// host code `scratch` only names the symbol; its device address (one per GPU)
// comes from hipGetSymbolAddress when a context binds a device, and only that
// address is ever passed to kernels or copies.
constexpr int64_t kScratchBytes = CDAG_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;   // device ordinal -> device address of `scratch`

// Called with `device` current; once per device.
void ensure_scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return;
  void* ptr = nullptr;
  hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  g_scratch_ptr[device] = static_cast<char*>(ptr);
}

char* scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}
}  // namespace

struct Device {
  int device = -1;
  hipStream_t comp = nullptr, copy = nullptr;   // borrowed: kernels, uploads
  hipStream_t spill_s = nullptr;                // owned: spills to the host
  char* arena = nullptr;
  uint64_t arena_bytes = 0;
  uint64_t arena_epoch = 0;                 // bumped when the arena is rebound
  // pinned staging of leaves in device layout, per precision mode
  std::vector<void*> stage[4];
  uint64_t stage_version[4] = {0, 0, 0, 0};
  // host spill pool: pinned, or pageable when a pinned allocation of the
  // plan's size fails (then steps run eagerly, without captured segments)
  void* spill = nullptr;
  int64_t spill_bytes = 0;
  bool spill_pageable = false;
  // pinned result buffer
  void* results = nullptr;
  int64_t results_bytes = 0;
  // per step of every pass and per stream role; then per pass, the pass-end
  // events of the three streams
  std::vector<hipEvent_t> ev[kStreams], ev_end[kStreams];
  hipEvent_t t0 = nullptr, t1 = nullptr;
  // what is currently uploaded
  uint64_t blob_key = 0, blob_epoch = 0;
  int resident_prec = -1;
  uint64_t resident_key = 0, resident_epoch = 0;
  // captured step sequence: one graph per segment of consecutive steps
  hipStream_t cap = nullptr;        // stream the one-stream segments are captured on
  hipEvent_t ev_join[2] = {nullptr, nullptr};
  std::vector<hipGraph_t> seg_graph;
  std::vector<hipGraphExec_t> seg_exec;
  uint64_t graph_key = 0, graph_epoch = 0, graph_stage = 0;
  int graph_mode = 0;
  void* graph_spill = nullptr;

  void drop_graphs() {
    for (auto g : seg_exec) ignore(hipGraphExecDestroy(g));
    for (auto g : seg_graph) ignore(hipGraphDestroy(g));
    seg_exec.clear();
    seg_graph.clear();
    graph_key = 0;
  }
  // timing mode: event pairs around kernel launches and host transfers
  std::vector<hipEvent_t> tpool;
  size_t tnext = 0;
  struct TPair {
    int64_t launch;          // launch index; -1: cross sum; -2: a transfer
    int32_t type, kinds;     // transfers: CDAG_LAUNCH_H2D / D2H and the tensor's kind bit
    int64_t step;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<TPair> tpairs;

  hipEvent_t timing_event() {
    if (tnext == tpool.size()) {
      hipEvent_t e;
      HIPC(hipEventCreate(&e));
      tpool.push_back(e);
    }
    return tpool[tnext++];
  }

  ~Device() {
    if (device >= 0) ignore(hipSetDevice(device));
    drop_graphs();
    if (cap) ignore(hipStreamDestroy(cap));
    if (spill_s) ignore(hipStreamDestroy(spill_s));
    for (int r = 0; r < kStreams; ++r) {
      for (auto e : ev[r]) ignore(hipEventDestroy(e));
      for (auto e : ev_end[r]) ignore(hipEventDestroy(e));
    }
    for (auto e : tpool) ignore(hipEventDestroy(e));
    if (t0) ignore(hipEventDestroy(t0));
    if (t1) ignore(hipEventDestroy(t1));
    for (auto e : ev_join)
      if (e) ignore(hipEventDestroy(e));
    for (auto& v : stage)
      for (void* p : v)
        if (p) ignore(hipHostFree(p));
    free_spill();
    if (results) ignore(hipHostFree(results));
  }
  void free_spill() {
    if (spill && spill_pageable) std::free(spill);
    else if (spill) ignore(hipHostFree(spill));
    spill = nullptr;
    spill_bytes = 0;
    spill_pageable = false;
  }
};

void device_destroy(Device* d) { delete d; }

void device_bind(Ctx& c, int device, void* compute_stream, void* copy_stream) {
  int n = 0;
  HIPC(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) throw Error(CDAG_E_INVALID, "device ordinal out of range");
  if (!c.dev || c.dev->device != device) {
    delete c.dev;
    c.dev = nullptr;
    c.dev = new Device();
    c.dev->device = device;
  }
  HIPC(hipSetDevice(device));
  ensure_scratch_address(device);
  c.dev->comp = (hipStream_t)compute_stream;
  c.dev->copy = (hipStream_t)copy_stream;
  if (!c.dev->t0) {
    // library-owned streams keep the default priority
    HIPC(hipEventCreate(&c.dev->t0));
    HIPC(hipEventCreate(&c.dev->t1));
    for (auto& e : c.dev->ev_join) HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPC(hipStreamCreateWithFlags(&c.dev->spill_s, hipStreamNonBlocking));
    HIPC(hipStreamCreateWithFlags(&c.dev->cap, hipStreamNonBlocking));
  }
}

void device_bind_arena(Ctx& c, void* arena, uint64_t bytes) {
  if (!c.dev) throw Error(CDAG_E_STATE, "cdag_bind_device first");
  c.dev->arena = (char*)arena;
  c.dev->arena_bytes = bytes;
  c.dev->arena_epoch++;
}

namespace {
// Interleaved complex [nt][e] (S = double or float) -> planar [nt][2][e] in T.
template <typename S, typename T>
void to_device_layout(const S* src, T* dst, int64_t nt, int64_t e) {
  for (int64_t t = 0; t < nt; ++t) {
    const S* s = src + 2 * t * e;
    T* re = dst + 2 * t * e;
    T* im = re + e;
    for (int64_t i = 0; i < e; ++i) {
      re[i] = (T)s[2 * i];
      im[i] = (T)s[2 * i + 1];
    }
  }
}

void ensure_stage(Ctx& c, int prec) {
  Device& D = *c.dev;
  if (D.stage_version[prec] == c.data_version && !D.stage[prec].empty()) return;
  const int64_t L = c.dag.n_leaves;
  const int eb = prec == CDAG_FP64 ? 16 : 8;
  for (void* p : D.stage[prec])
    if (p) ignore(hipHostFree(p));
  D.stage[prec].assign(L, nullptr);
  for (int64_t u = 0; u < L; ++u)
    HIPC(hipHostMalloc(&D.stage[prec][u], (size_t)c.dag.size(u, eb), hipHostMallocDefault));
  const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned w = 0; w < nth; ++w)
    th.emplace_back([&, w] {
      for (int64_t u = w; u < L; u += nth) {
        const int64_t e = c.dag.elems(u) / c.dag.nt[u];
        const void* src = c.leaf_data[u].data();
        const bool c64 = c.leaf_dtype[u] == CDAG_C64;
        if (prec == CDAG_FP64) {
          if (c64) to_device_layout<float, double>((const float*)src, (double*)D.stage[prec][u], c.dag.nt[u], e);
          else to_device_layout<double, double>((const double*)src, (double*)D.stage[prec][u], c.dag.nt[u], e);
        } else {
          if (c64) to_device_layout<float, float>((const float*)src, (float*)D.stage[prec][u], c.dag.nt[u], e);
          else to_device_layout<double, float>((const double*)src, (float*)D.stage[prec][u], c.dag.nt[u], e);
        }
      }
    });
  for (auto& t : th) t.join();
  D.stage_version[prec] = c.data_version;
}

void ensure_events(Device& D, size_t steps, size_t passes) {
  for (int r = 0; r < kStreams; ++r) {
    for (auto* v : {&D.ev[r], &D.ev_end[r]}) {
      const size_t n = v == &D.ev[r] ? steps : passes;
      while (v->size() < n) {
        hipEvent_t e;
        HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        v->push_back(e);
      }
    }
  }
}

// The spill pool holds the plan's spilled intermediates at once.  Pinned
// memory of that size may be refused; pageable memory then takes its place.
void ensure_spill(Device& D, int64_t need_bytes) {
  if (D.spill && D.spill_bytes >= need_bytes) return;
  D.free_spill();
  if (need_bytes <= 0) return;
  if (hipHostMalloc(&D.spill, (size_t)need_bytes, hipHostMallocDefault) != hipSuccess) {
    ignore_last_error();
    D.spill = std::malloc((size_t)need_bytes);
    if (!D.spill) throw Error(CDAG_E_NOMEM, "host spill pool of " + std::to_string(need_bytes) + " bytes");
    D.spill_pageable = true;
  }
  D.spill_bytes = need_bytes;
}

void ensure_pinned(void*& p, int64_t& have, int64_t need_bytes) {
  if (have >= need_bytes && p) return;
  if (p) ignore(hipHostFree(p));
  p = nullptr;
  have = 0;
  if (need_bytes <= 0) return;
  HIPC(hipHostMalloc(&p, (size_t)need_bytes, hipHostMallocDefault));
  have = need_bytes;
}

hipError_t call_of(const Launch& L, int prec, char* arena, KernelCall* k) {
  switch (L.type) {
    case L_HEC:
      return hec_call(prec, L.tile, L.interior != 0, arena, L.desc_off, L.n_desc, L.n_items, k, L.tr_desc_off,
                      L.tr_n_desc, L.tr_n_items);
    case L_RED: return reduce_call(prec, arena, L.desc_off, L.n_desc, L.n_items, k);
    case L_HCA: return hca_call(prec, arena, L.desc_off, L.n_desc, L.n_items, k);
    default: throw Error(CDAG_E_STATE, "bad launch type");
  }
}

hipError_t launch_one(const Launch& L, int prec, char* arena, hipStream_t st) {
  KernelCall k;
  const hipError_t e = call_of(L, prec, arena, &k);
  return e != hipSuccess ? e : launch(k, st);
}

// Kernels of global step g; with `timed`, every launch is bracketed by an
// event pair.
int64_t launch_step(const KernelPlan& kp, int64_t g, int prec, char* arena, hipStream_t st, Device* timed) {
  int64_t n = 0;
  for (int64_t li = kp.launch_off[g]; li < kp.launch_off[g + 1]; ++li) {
    const Launch& L = kp.launches[li];
    if (timed) {
      hipEvent_t a = timed->timing_event(), b = timed->timing_event();
      HIPC(hipEventRecord(a, st));
      HIPC(launch_one(L, prec, arena, st));
      HIPC(hipEventRecord(b, st));
      timed->tpairs.push_back({li, 0, 0, g, 0.0, a, b});
    } else {
      HIPC(launch_one(L, prec, arena, st));
    }
    ++n;
  }
  return n;
}

// Where pass k of a time-chunked execution keeps its data: the tensor pool and
// workspace of half k % 2 of the arena, half k % 2 of the host spill pool, and
// slices [k nt / C, (k + 1) nt / C) of every tensor (bytes(u) per pass).
struct PassMap {
  const Ctx& c;
  int64_t k, dev_shift, host_shift;
  PassMap(const Ctx& ctx, int64_t pass)
      : c(ctx), k(pass), dev_shift((pass % 2) * ctx.kplan.half_bytes),
        host_shift((pass % 2) * ctx.plan.host_spill_bytes) {}
  int64_t bytes(int64_t u) const { return c.plan.tsize(c.dag, u); }
  int64_t dev(int64_t off) const { return off + dev_shift; }
  int64_t host(int64_t off) const { return off + host_shift; }
  int64_t stage(int64_t u) const { return k * bytes(u); }   // in the leaf's staging buffer
  // arena offset of operand x planned at `planned`: a resident leaf's slices of
  // this pass, else the planned offset in the pass's half
  int64_t operand(int64_t x, int64_t planned) const {
    if (c.plan.opts.leaves_resident && c.dag.is_leaf(x)) return c.plan.leaf_off[x] + k * bytes(x);
    return dev(planned);
  }
};

// Walk global steps [g0, g1), g = k * S + s being step s of pass k: each
// step's spills (after the kernels that last touched the tensor and any upload
// still reading the host range), its uploads (after the kernels and spills
// that last used the arena range, and the spill that wrote a re-uploaded
// tensor), then its kernels (after the step's uploads and any spill still
// reading an output's memory).  With one_stream (how one-stream segments are
// captured) every dependency is the stream order and no event is used.  In a
// captured segment, waits on steps before g0 are left out: the segments' graphs
// run one after another on one stream, so everything before g0 has finished
// when the segment starts.  Ops issues the work (HipOps) or records it
// (TraceOps).
template <class Ops>
int64_t walk_steps(const Ctx& c, int64_t g0, int64_t g1, bool one_stream, bool in_capture, Ops& ops) {
  const Plan& p = c.plan;
  const int64_t S = (int64_t)p.steps.size(), C = p.chunks();
  // waited[to][from]: newest step of stream `from` that stream `to` has waited
  // for; events of one stream complete in step order, so older ones are implied
  int64_t waited[kStreams][kStreams];
  for (auto& row : waited)
    for (auto& x : row) x = in_capture ? g0 - 1 : -1;
  auto wait = [&](int to, int from, int64_t g) {
    if (one_stream || g < 0 || g <= waited[to][from]) return;
    ops.wait(to, from, g, g);
    waited[to][from] = g;
  };
  int64_t n_launch = 0;
  for (int64_t g = g0; g < g1; ++g) {
    const int64_t k = g / S, s = g % S, kS = k * S;
    const PassMap m(c, k);
    auto at = [&](int64_t step) { return step >= 0 ? kS + step : -1; };
    if (s == 0 && k >= 2 && !one_stream && !(in_capture && (k - 1) * S <= g0)) {
      // pass k - 2 used the same half of the arena and of the spill pool
      ops.wait_pass(S_H2D, S_COMP, k - 2, g);
      ops.wait_pass(S_H2D, S_D2H, k - 2, g);
      ops.wait_pass(S_D2H, S_H2D, k - 2, g);
      ops.wait_pass(S_COMP, S_D2H, k - 2, g);
    }
    bool any_d2h = false, any_h2d = false;
    int64_t alloc_d2h = -1;
    for (int64_t ri = p.rec_off[s]; ri < p.rec_off[s + 1]; ++ri) {
      const PlanRec& r = p.recs[ri];
      if (r.op != OP_D2H) continue;
      wait(S_D2H, S_COMP, at(r.wait_comp));
      wait(S_D2H, S_H2D, at(r.wait_h2d));
      ops.transfer(r, m, g);
      any_d2h = true;
    }
    if (any_d2h && !one_stream) ops.record(S_D2H, g);
    for (int64_t ri = p.rec_off[s]; ri < p.rec_off[s + 1]; ++ri) {
      const PlanRec& r = p.recs[ri];
      if (r.op == OP_H2D) {
        wait(S_H2D, S_COMP, at(r.wait_comp));
        wait(S_H2D, S_D2H, at(r.wait_d2h));
        ops.transfer(r, m, g);
        any_h2d = true;
      } else if (r.op == OP_ALLOC) {
        alloc_d2h = std::max(alloc_d2h, at(r.wait_d2h));
      }
    }
    if (any_h2d && !one_stream) ops.record(S_H2D, g);
    if (any_h2d) wait(S_COMP, S_H2D, g);
    wait(S_COMP, S_D2H, alloc_d2h);
    n_launch += ops.launch(g, m);
    if (!one_stream) {
      ops.record(S_COMP, g);
      if (s == S - 1 && k + 2 < C)
        for (int r = 0; r < kStreams; ++r) ops.record_pass(r, k, g);
    }
  }
  return n_launch;
}

// The issuing form: kernels on st[S_COMP], uploads on st[S_H2D], spills on
// st[S_D2H], with the device's per-step and per-pass events.
struct HipOps {
  const Ctx& c;
  Device& D;
  int prec;
  hipStream_t st[kStreams];
  Device* timed;

  void wait(int to, int from, int64_t g, int64_t) { HIPC(hipStreamWaitEvent(st[to], D.ev[from][g], 0)); }
  void record(int r, int64_t g) { HIPC(hipEventRecord(D.ev[r][g], st[r])); }
  void wait_pass(int to, int from, int64_t k, int64_t) { HIPC(hipStreamWaitEvent(st[to], D.ev_end[from][k], 0)); }
  void record_pass(int r, int64_t k, int64_t) { HIPC(hipEventRecord(D.ev_end[r][k], st[r])); }
  int64_t launch(int64_t g, const PassMap&) { return launch_step(c.kplan, g, prec, D.arena, st[S_COMP], timed); }
  void transfer(const PlanRec& r, const PassMap& m, int64_t g) {
    const size_t sz = (size_t)m.bytes(r.node);
    hipStream_t cs = st[r.op == OP_D2H ? S_D2H : S_H2D];
    hipEvent_t ta = nullptr, tb = nullptr;
    if (timed) {
      ta = timed->timing_event();
      tb = timed->timing_event();
      HIPC(hipEventRecord(ta, cs));
    }
    char* spill = (char*)D.spill;
    if (r.op == OP_D2H) {
      HIPC(hipMemcpyAsync(spill + m.host(r.host_off), D.arena + m.dev(r.dev_off), sz, hipMemcpyDeviceToHost, cs));
    } else {
      const void* src = c.dag.is_leaf(r.node) ? (const void*)((const char*)D.stage[prec][r.node] + m.stage(r.node))
                                              : (const void*)(spill + m.host(r.host_off));
      HIPC(hipMemcpyAsync(D.arena + m.dev(r.dev_off), src, sz, hipMemcpyHostToDevice, cs));
    }
    if (timed) {
      HIPC(hipEventRecord(tb, cs));
      const int32_t kd = c.dag.kind[r.node];
      timed->tpairs.push_back({-2, r.op == OP_D2H ? CDAG_LAUNCH_D2H : CDAG_LAUNCH_H2D,
                               kd >= 0 ? (1 << kd) : 0, g, (double)sz, ta, tb});
    }
  }
};

int64_t issue_steps(Ctx& c, Device& D, int prec, int64_t g0, int64_t g1, hipStream_t comp, hipStream_t h2d,
                    hipStream_t d2h, Device* timed, bool in_capture) {
  HipOps ops{c, D, prec, {comp, h2d, d2h}, timed};
  return walk_steps(c, g0, g1, comp == h2d, in_capture, ops);
}

// The recording form: the same walk with no HIP call, writing what each stream
// would do (event records and waits, and the byte ranges that every transfer
// and every step's kernels read and write).  Event ids: kStreams * g + stream
// for the step events, kStreams * (passes * S + k) + stream for the pass-end
// events.  fail_at >= 0 throws at that record, as a failed HIP call would.
struct TraceOps {
  const Ctx& c;
  int prec;
  std::vector<cdag_trace_rec>& out;
  int64_t fail_at;
  int64_t seq = 0;

  void put(const cdag_trace_rec& r) {
    if ((int64_t)out.size() == fail_at)
      throw Error(CDAG_E_HIP, "injected failure at trace record " + std::to_string(fail_at));
    out.push_back(r);
  }
  static cdag_trace_rec blank(int32_t op, int32_t stream, int64_t step) {
    cdag_trace_rec r{};
    r.op = op;
    r.stream = stream;
    r.step = step;
    r.seq = r.node = r.event = -1;
    return r;
  }
  int64_t pass_event(int64_t k, int r) const {
    return kStreams * (c.plan.chunks() * (int64_t)c.plan.steps.size() + k) + r;
  }
  void event(int32_t op, int32_t stream, int64_t id, int64_t g) {
    cdag_trace_rec r = blank(op, stream, g);
    r.event = id;
    put(r);
  }
  void access(int32_t op, int32_t stream, int64_t g, int64_t node, int32_t space, int64_t off, int64_t bytes) {
    cdag_trace_rec r = blank(op, stream, g);
    r.seq = seq;
    r.node = node;
    r.space = space;
    r.off = off;
    r.bytes = bytes;
    put(r);
  }
  void wait(int to, int from, int64_t ev_g, int64_t g) { event(CDAG_TR_WAIT, to, kStreams * ev_g + from, g); }
  void record(int r, int64_t g) { event(CDAG_TR_RECORD, r, kStreams * g + r, g); }
  void wait_pass(int to, int from, int64_t k, int64_t g) { event(CDAG_TR_WAIT, to, pass_event(k, from), g); }
  void record_pass(int r, int64_t k, int64_t g) { event(CDAG_TR_RECORD, r, pass_event(k, r), g); }
  void transfer(const PlanRec& r, const PassMap& m, int64_t g) {
    const int64_t bytes = m.bytes(r.node);
    if (r.op == OP_D2H) {
      access(CDAG_TR_READ, S_D2H, g, r.node, CDAG_SPACE_ARENA, m.dev(r.dev_off), bytes);
      access(CDAG_TR_WRITE, S_D2H, g, r.node, CDAG_SPACE_SPILL, m.host(r.host_off), bytes);
    } else {
      if (c.dag.is_leaf(r.node)) access(CDAG_TR_READ, S_H2D, g, r.node, CDAG_SPACE_STAGE, m.stage(r.node), bytes);
      else access(CDAG_TR_READ, S_H2D, g, r.node, CDAG_SPACE_SPILL, m.host(r.host_off), bytes);
      access(CDAG_TR_WRITE, S_H2D, g, r.node, CDAG_SPACE_ARENA, m.dev(r.dev_off), bytes);
    }
    ++seq;
  }
  int64_t launch(int64_t g, const PassMap& m) {
    const Plan& p = c.plan;
    const int64_t S = (int64_t)p.steps.size(), s = g % S;
    for (int64_t ri = p.rec_off[s]; ri < p.rec_off[s + 1]; ++ri) {
      const PlanRec& r = p.recs[ri];
      if (r.op != OP_EXEC) continue;
      const int64_t* ch = c.dag.children_begin(r.node);
      access(CDAG_TR_READ, S_COMP, g, ch[0], CDAG_SPACE_ARENA, m.operand(ch[0], r.a_off), m.bytes(ch[0]));
      access(CDAG_TR_READ, S_COMP, g, ch[1], CDAG_SPACE_ARENA, m.operand(ch[1], r.b_off), m.bytes(ch[1]));
      if (c.dag.kind[r.node] != HCA)
        access(CDAG_TR_WRITE, S_COMP, g, r.node, CDAG_SPACE_ARENA, m.dev(r.dev_off), m.bytes(r.node));
    }
    ++seq;
    return c.kplan.launch_off[g + 1] - c.kplan.launch_off[g];
  }
};

// The graph form: the same walk adding the transfers and kernels to a HIP
// graph as nodes with explicit dependencies (no stream capture).  A node
// depends on the previous node of its stream and on the nodes its stream
// waited for since; an event stands for its stream's last node (joined with
// that stream's pending waits) at the time it is recorded.
struct GraphOps {
  const Ctx& c;
  Device& D;
  int prec;
  hipGraph_t graph;
  hipGraphNode_t last[kStreams] = {nullptr, nullptr, nullptr};
  std::vector<hipGraphNode_t> pending[kStreams];
  std::vector<hipGraphNode_t> ev_node[kStreams];     // per global step
  std::vector<hipGraphNode_t> pass_node[kStreams];   // per pass
  std::vector<hipGraphNode_t> deps;

  GraphOps(const Ctx& ctx, Device& dev, int p, hipGraph_t g) : c(ctx), D(dev), prec(p), graph(g) {
    const size_t G = (size_t)(ctx.plan.chunks() * (int64_t)ctx.plan.steps.size());
    for (int r = 0; r < kStreams; ++r) {
      ev_node[r].assign(G, nullptr);
      pass_node[r].assign((size_t)ctx.plan.chunks(), nullptr);
    }
  }
  void deps_of(int r) {
    deps = pending[r];
    if (last[r]) deps.push_back(last[r]);
  }
  void added(int r, hipGraphNode_t n) {
    last[r] = n;
    pending[r].clear();
  }
  hipGraphNode_t head(int r) {
    if (pending[r].empty()) return last[r];
    deps_of(r);
    hipGraphNode_t n = nullptr;
    HIPC(hipGraphAddEmptyNode(&n, graph, deps.data(), deps.size()));
    added(r, n);
    return n;
  }
  void wait(int to, int from, int64_t g, int64_t) {
    if (ev_node[from][g]) pending[to].push_back(ev_node[from][g]);
  }
  void record(int r, int64_t g) { ev_node[r][g] = head(r); }
  void wait_pass(int to, int from, int64_t k, int64_t) {
    if (pass_node[from][k]) pending[to].push_back(pass_node[from][k]);
  }
  void record_pass(int r, int64_t k, int64_t) { pass_node[r][k] = head(r); }
  void transfer(const PlanRec& r, const PassMap& m, int64_t) {
    const size_t sz = (size_t)m.bytes(r.node);
    const int sr = r.op == OP_D2H ? S_D2H : S_H2D;
    char* spill = (char*)D.spill;
    void* dst;
    const void* src;
    hipMemcpyKind kind;
    if (r.op == OP_D2H) {
      dst = spill + m.host(r.host_off);
      src = D.arena + m.dev(r.dev_off);
      kind = hipMemcpyDeviceToHost;
    } else {
      dst = D.arena + m.dev(r.dev_off);
      src = c.dag.is_leaf(r.node) ? (const void*)((const char*)D.stage[prec][r.node] + m.stage(r.node))
                                  : (const void*)(spill + m.host(r.host_off));
      kind = hipMemcpyHostToDevice;
    }
    deps_of(sr);
    hipGraphNode_t n = nullptr;
    HIPC(hipGraphAddMemcpyNode1D(&n, graph, deps.data(), deps.size(), dst, src, sz, kind));
    added(sr, n);
  }
  int64_t launch(int64_t g, const PassMap&) {
    const KernelPlan& kp = c.kplan;
    for (int64_t li = kp.launch_off[g]; li < kp.launch_off[g + 1]; ++li) {
      KernelCall k;
      HIPC(call_of(kp.launches[li], prec, D.arena, &k));
      k.bind();
      hipKernelNodeParams np{};
      np.func = const_cast<void*>(k.fn);
      np.gridDim = dim3(k.grid);
      np.blockDim = dim3(k.block);
      np.sharedMemBytes = 0;
      np.kernelParams = k.args;
      np.extra = nullptr;
      deps_of(S_COMP);
      hipGraphNode_t n = nullptr;
      HIPC(hipGraphAddKernelNode(&n, graph, deps.data(), deps.size(), &np));
      added(S_COMP, n);
    }
    return kp.launch_off[g + 1] - kp.launch_off[g];
  }
};

constexpr int64_t kSegmentSteps = 64;   // steps per one-stream graph when transfers are present
}  // namespace

// Autotuner: for every distinct (kind, N) among the exterior contractions,
// time each kernel choice on a synthetic contraction of that shape (operands
// in the arena's tensor pool, which holds nothing between executes).  uniform
// = false keeps the fastest choice per time slice of each shape; uniform =
// true keeps the one choice whose time over the whole DAG (per-slice time x
// the slices of that shape in the DAG, summed over shapes) is least, so that
// every wave runs its exterior contractions in one grouped launch.  The
// choices enter the tile table of the context.
int64_t device_autotune(Ctx& c, int prec, int batched, int reps, bool uniform) {
  Device& D = *c.dev;
  HIPC(hipSetDevice(D.device));
  const Plan& p = c.plan;
  const KernelPlan& kp = c.kplan;
  if (!D.arena) throw Error(CDAG_E_STATE, "cdag_bind_arena first");
  if ((uint64_t)kp.total_bytes > D.arena_bytes) throw Error(CDAG_E_NOMEM, "arena smaller than the plan");
  (void)batched;
  const int64_t eb = prec == CDAG_FP64 ? 16 : 8, acc = prec == CDAG_FP64 ? 8 : 4;
  auto al = [](int64_t x) { return (x + 255) / 256 * 256; };
  const int64_t lo = al(p.leaf_region_bytes), hi = kp.ws_off + kp.ws_bytes;
  const auto shapes = tune_shapes(c.dag);
  // slices of each shape in the DAG (the uniform choice's weights)
  std::map<std::pair<int, int>, double> weight;
  for (int64_t u = c.dag.n_leaves; u < c.dag.n_nodes(); ++u)
    if (c.dag.kind[u] != HCA) weight[{c.dag.kind[u], c.dag.nvec[u]}] += c.dag.nt[u];
  std::map<std::pair<int, int>, std::vector<double>> per_slice;   // shape -> time per slice, per choice
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  int64_t tuned = 0;
  try {
    for (const auto& sh : shapes) {
      const int kind = sh.first.first, n = sh.first.second;
      double best = 1e300;
      int best_tile = -1;
      const int snt = sh.second.nt;
      std::vector<double>& row = per_slice[sh.first];
      row.assign(kNumChoices, 1e300);
      for (int ch = 0; ch < kNumChoices; ++ch) {
        HecDesc h{};
        decompose(sh.second.gemm, snt, ch, prec, &h);   // split count of a real contraction
        if (!choice_split_k(ch)) {
          HecDesc a{};
          decompose(sh.second.gemm, snt, choice_variant(ch), prec, &a);
          if (a.splits == 1) {                          // same work items as the split choice
            row[ch] = row[choice_of(choice_variant(ch), true)];
            continue;
          }
        }
        const int64_t slice_items = (int64_t)h.tiles_m * h.tiles_n * h.splits;
        const int64_t slice = (int64_t)h.M * h.K * eb + (int64_t)h.K * h.N * eb + (int64_t)h.M * h.N * eb;
        const int64_t wslice = h.splits > 1 ? (int64_t)h.splits * 2 * h.M * h.N * acc : 0;
        // A wave holds many contractions of one shape: time a batch of slices
        // with at least 4096 work items (at most 64 contractions' worth).
        int64_t want = std::max<int64_t>(snt, (4096 + slice_items - 1) / slice_items);
        want = std::min<int64_t>(want, 64LL * snt);
        int64_t nt = std::min<int64_t>(want, (hi - lo - 4096) / std::max<int64_t>(1, slice + wslice + 1024));
        if (nt < 1 || nt * slice_items > INT32_MAX) continue;
        h.nt = (int32_t)nt;
        h.tile_count = (int32_t)(nt * slice_items);
        const int64_t a = lo, b = a + al(nt * h.M * h.K * eb), cc = b + al(nt * h.K * h.N * eb);
        const int64_t ws = cc + al(nt * h.M * h.N * eb);
        const int64_t ws_bytes = h.splits > 1 ? al((int64_t)h.splits * nt * 2 * h.M * h.N * acc) : 0;
        const int64_t desc = ws + ws_bytes;
        if (desc + 256 > hi) continue;
        h.a_off = a;
        h.b_off = b;
        h.c_off = cc;
        h.ws_off = h.splits > 1 ? ws : -1;
        h.tile_begin = 0;
        RedDesc r{ws, cc, h.M * h.N, (int32_t)nt, h.splits, 0};
        const int64_t red_items = (2LL * nt * h.M * h.N + 255) / 256;
        HIPC(hipMemsetAsync(D.arena + a, 0, (size_t)(ws - a), D.comp));
        HIPC(hipMemcpyAsync(D.arena + desc, &h, sizeof(h), hipMemcpyHostToDevice, D.comp));
        HIPC(hipMemcpyAsync(D.arena + desc + 128, &r, sizeof(r), hipMemcpyHostToDevice, D.comp));
        const int v = choice_variant(ch);
        const bool interior =
            hec_interior(h, kTileShapes[variant_tile(v)].bm, kTileShapes[variant_tile(v)].bn, k_step(prec));
        auto once = [&] {
          HIPC(launch_hec(prec, v, interior, D.arena, desc, 1, h.tile_count, D.comp));
          if (h.splits > 1) HIPC(launch_reduce(prec, D.arena, desc + 128, 1, red_items, D.comp));
        };
        once();
        HIPC(hipEventRecord(e0, D.comp));
        for (int k = 0; k < reps; ++k) once();
        HIPC(hipEventRecord(e1, D.comp));
        HIPC(hipEventSynchronize(e1));
        float ms = 0;
        HIPC(hipEventElapsedTime(&ms, e0, e1));
        const double t_slice = ms / reps / (double)nt;
        row[ch] = t_slice;
        if (t_slice < best) { best = t_slice; best_tile = ch; }
      }
      if (best_tile >= 0 && !uniform) {
        c.tiles[std::make_tuple(prec, kind, n)] = best_tile;
        ++tuned;
      }
    }
    if (uniform && !per_slice.empty()) {
      double best = 1e300;
      int best_ch = -1;
      for (int ch = 0; ch < kNumChoices; ++ch) {
        double t = 0;
        for (const auto& kv : per_slice) t += weight[kv.first] * kv.second[ch];
        if (t < best) { best = t; best_ch = ch; }
      }
      if (best_ch >= 0 && best < 1e299)
        for (const auto& kv : per_slice) {
          c.tiles[std::make_tuple(prec, kv.first.first, kv.first.second)] = best_ch;
          ++tuned;
        }
    }
  } catch (...) {
    ignore(hipEventDestroy(e0));
    ignore(hipEventDestroy(e1));
    throw;
  }
  ignore(hipEventDestroy(e0));
  ignore(hipEventDestroy(e1));
  HIPC(hipStreamSynchronize(D.comp));
  return tuned;
}

// In-situ autotuner: for every distinct (kind, N) in turn, run the planned DAG
// `reps` times with each kernel variant for that shape (the other shapes keep
// their current choice), with HIP events around every launch, and keep the
// variant whose fastest execute spends the least time in exterior
// contractions plus split-K reductions.
int64_t device_autotune_insitu(Ctx& c, int prec, int batched, int reps) {
  const auto shapes = tune_shapes(c.dag);
  const bool timing = c.timing;
  const auto tiles = c.tiles;                  // restored if a trial execute throws
  c.timing = true;
  int64_t tuned = 0;
  try {
    for (const auto& sh : shapes) {
      const auto key = std::make_tuple(prec, sh.first.first, sh.first.second);
      double best = 1e300;
      int best_v = -1;
      for (int v = 0; v < kNumChoices; ++v) {
        if (!choice_split_k(v)) {
          // the no-split setting only differs where the rule would split
          HecDesc h{};
          decompose(sh.second.gemm, sh.second.nt, choice_variant(v), prec, &h);
          if (h.splits == 1) continue;
        }
        c.tiles[key] = v;
        c.version++;
        ensure_plan(c, prec, batched);
        if ((uint64_t)c.kplan.total_bytes > c.dev->arena_bytes) continue;
        double t = 1e300;                        // fastest of the reps (robust to noise)
        for (int r = 0; r < reps; ++r) {
          cdag_exec_stats st{};
          device_execute(c, prec, batched, &st);
          double tr = 0;
          for (const cdag_launch_record& rec : c.records)
            if (rec.type == CDAG_LAUNCH_HEC || rec.type == CDAG_LAUNCH_REDUCE) tr += rec.ms;
          t = std::min(t, tr);
        }
        if (t < best) { best = t; best_v = v; }
      }
      if (best_v >= 0) {
        c.tiles[key] = best_v;
        ++tuned;
      } else {
        c.tiles.erase(key);
      }
      c.version++;
    }
  } catch (...) {
    c.timing = timing;
    c.tiles = tiles;
    c.version++;
    throw;
  }
  c.timing = timing;
  return tuned;
}

void trace_execute(const Ctx& c, int prec, std::vector<cdag_trace_rec>& out, int64_t fail_at) {
  out.clear();
  TraceOps ops{c, prec, out, fail_at};
  walk_steps(c, 0, c.plan.chunks() * (int64_t)c.plan.steps.size(), false, false, ops);
}

namespace {
// Capture global steps [g0, g1) into one graph on one stream (stream order
// carries every dependency).
hipGraph_t capture_steps(Ctx& c, Device& D, int prec, int64_t g0, int64_t g1) {
  hipGraph_t g = nullptr;
  HIPC(hipStreamBeginCapture(D.cap, hipStreamCaptureModeThreadLocal));
  try {
    issue_steps(c, D, prec, g0, g1, D.cap, D.cap, D.cap, nullptr, true);
  } catch (...) {
    ignore(hipStreamEndCapture(D.cap, &g));
    if (g) ignore(hipGraphDestroy(g));
    throw;
  }
  HIPC(hipStreamEndCapture(D.cap, &g));
  return g;
}

// Build the whole step sequence as one graph over the three streams' work,
// with the plan's waits as explicit edges.
hipGraph_t build_graph(Ctx& c, Device& D, int prec) {
  hipGraph_t g = nullptr;
  HIPC(hipGraphCreate(&g, 0));
  try {
    GraphOps ops(c, D, prec, g);
    walk_steps(c, 0, c.plan.chunks() * (int64_t)c.plan.steps.size(), false, false, ops);
  } catch (...) {
    ignore(hipGraphDestroy(g));
    throw;
  }
  return g;
}
}  // namespace

void device_execute(Ctx& c, int prec, int batched, cdag_exec_stats* st) {
  (void)batched;
  Device& D = *c.dev;
  const double tw0 = now();
  HIPC(hipSetDevice(D.device));
  const Plan& p = c.plan;
  const KernelPlan& kp = c.kplan;
  if (!D.arena) throw Error(CDAG_E_STATE, "cdag_bind_arena first");
  if ((uint64_t)kp.total_bytes > D.arena_bytes)
    throw Error(CDAG_E_NOMEM, "arena has " + std::to_string(D.arena_bytes) + " bytes, the plan needs " +
                                  std::to_string(kp.total_bytes));
  const int eb = prec == CDAG_FP64 ? 16 : 8;
  ensure_stage(c, prec);
  ensure_spill(D, p.halves() * p.host_spill_bytes);
  ensure_pinned(D.results, D.results_bytes, kp.corr_bytes + kp.sums_bytes);
  const int64_t S = (int64_t)p.steps.size(), G = p.chunks() * S;
  ensure_events(D, (size_t)std::max<int64_t>(G, 1), (size_t)p.chunks());

  // descriptor tables: one upload per (plan, arena)
  const uint64_t pkey = c.plan_serial;
  if (D.blob_key != pkey || D.blob_epoch != D.arena_epoch) {
    HIPC(hipMemcpyAsync(D.arena + kp.blob_off, kp.blob.data(), kp.blob.size(), hipMemcpyHostToDevice, D.comp));
    HIPC(hipStreamSynchronize(D.comp));
    D.blob_key = pkey;
    D.blob_epoch = D.arena_epoch;
  }
  // leaves kept resident in their own region: one upload per (precision, arena, build)
  if (c.leaves_resident &&
      (D.resident_prec != prec || D.resident_epoch != D.arena_epoch || D.resident_key != D.stage_version[prec])) {
    for (int64_t u = 0; u < c.dag.n_leaves; ++u)
      HIPC(hipMemcpyAsync(D.arena + p.leaf_off[u], D.stage[prec][u], (size_t)c.dag.size(u, eb),
                          hipMemcpyHostToDevice, D.copy));
    HIPC(hipStreamSynchronize(D.copy));
    D.resident_prec = prec;
    D.resident_epoch = D.arena_epoch;
    D.resident_key = D.stage_version[prec];
  }
  // a plan with the leaves on the host keeps its own tensors where a resident
  // plan keeps the leaves, so the next resident execute uploads them again
  if (!c.leaves_resident) D.resident_prec = -1;

  bool has_copies = false;
  for (const PlanRec& r : p.recs)
    if (r.op == OP_H2D || r.op == OP_D2H) { has_copies = true; break; }

  int64_t n_launch = 0, n_segments = 0;
  D.tnext = 0;
  D.tpairs.clear();
  Device* timed = c.timing ? &D : nullptr;
  HIPC(hipEventRecord(D.t0, D.comp));
  if (c.use_graphs && !c.timing && !D.spill_pageable) {
    // replay graphs: one-stream segments of kSegmentSteps steps when there are
    // transfers (else one), or one graph built over the three streams
    const bool one = c.use_graphs == 1;
    const int64_t seg = one && has_copies ? kSegmentSteps : std::max<int64_t>(G, 1);
    if (D.graph_key != pkey || D.graph_epoch != D.arena_epoch || D.graph_spill != D.spill ||
        D.graph_stage != D.stage_version[prec] || D.graph_mode != c.use_graphs) {
      D.drop_graphs();
      for (int64_t g0 = 0; g0 < G; g0 += seg) {
        hipGraph_t g = nullptr;
        try {
          g = one ? capture_steps(c, D, prec, g0, std::min(G, g0 + seg)) : build_graph(c, D, prec);
        } catch (...) {
          D.drop_graphs();
          throw;
        }
        D.seg_graph.push_back(g);
        hipGraphExec_t ge = nullptr;
        HIPC(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        D.seg_exec.push_back(ge);
      }
      D.graph_key = pkey;
      D.graph_epoch = D.arena_epoch;
      D.graph_spill = D.spill;
      D.graph_stage = D.stage_version[prec];
      D.graph_mode = c.use_graphs;
    }
    for (hipGraphExec_t ge : D.seg_exec) HIPC(hipGraphLaunch(ge, D.comp));
    n_segments = (int64_t)D.seg_exec.size();
    for (int64_t g = 0; g < G; ++g) n_launch += kp.launch_off[g + 1] - kp.launch_off[g];
  } else {
    n_launch += issue_steps(c, D, prec, 0, G, D.comp, D.copy, D.spill_s, timed, false);
    // the results copy and the caller's later work follow every transfer
    HIPC(hipEventRecord(D.ev_join[0], D.copy));
    HIPC(hipEventRecord(D.ev_join[1], D.spill_s));
    HIPC(hipStreamWaitEvent(D.comp, D.ev_join[0], 0));
    HIPC(hipStreamWaitEvent(D.comp, D.ev_join[1], 0));
  }
  if (timed) {
    hipEvent_t a = D.timing_event(), b = D.timing_event();
    HIPC(hipEventRecord(a, D.comp));
    HIPC(launch_xsum(D.arena, kp.xsum.desc_off, kp.xsum_entries_off, kp.xsum.n_desc, D.comp));
    HIPC(hipEventRecord(b, D.comp));
    D.tpairs.push_back({-1, 0, 0, -1, 0.0, a, b});
  } else {
    HIPC(launch_xsum(D.arena, kp.xsum.desc_off, kp.xsum_entries_off, kp.xsum.n_desc, D.comp));
  }
  n_launch++;
  HIPC(hipEventRecord(D.t1, D.comp));
  if (kp.corr_bytes + kp.sums_bytes > 0)
    HIPC(hipMemcpyAsync(D.results, D.arena + kp.corr_off, (size_t)(kp.corr_bytes + kp.sums_bytes),
                        hipMemcpyDeviceToHost, D.comp));
  HIPC(hipStreamSynchronize(D.comp));
  HIPC(hipStreamSynchronize(D.copy));
  HIPC(hipStreamSynchronize(D.spill_s));
  float ms = 0;
  HIPC(hipEventElapsedTime(&ms, D.t0, D.t1));
  c.corr_host.assign((const double*)D.results, (const double*)D.results + kp.corr_bytes / 8);
  c.sums_host.assign((const double*)((const char*)D.results + kp.corr_bytes),
                     (const double*)((const char*)D.results + kp.corr_bytes) + kp.sums_bytes / 8);
  double t_hec = 0, t_kern = 0, t_copy = 0;
  if (timed) {
    c.records.clear();
    for (const Device::TPair& pr : D.tpairs) {
      float x = 0;
      HIPC(hipEventElapsedTime(&x, pr.a, pr.b));
      cdag_launch_record r{};
      r.step = pr.step;
      r.ms = x;
      if (pr.launch == -2) {
        r.type = pr.type;
        r.kinds = pr.kinds;
        r.n_items = 1;
        r.bytes = pr.bytes;
        c.records.push_back(r);
        t_copy += x * 1e-3;
        continue;
      }
      t_kern += x * 1e-3;
      const Launch& L = pr.launch >= 0 ? kp.launches[pr.launch] : kp.xsum;
      r.type = L.type;
      r.variant = L.type == L_HEC ? L.tile : 0;
      r.interior = L.type == L_HEC ? L.interior : 0;
      r.kinds = L.kinds;
      r.n_items = L.n_items;
      r.flops = L.flops;
      r.bytes = L.bytes;
      r.trace_items = L.tr_n_items;
      r.trace_flops = L.tr_flops;
      r.trace_bytes = L.tr_bytes;
      c.records.push_back(r);
      if (L.type == L_HEC) t_hec += x * 1e-3;
    }
  }
  int64_t n_hec = 0;
  for (const Launch& L : kp.launches) n_hec += L.type == L_HEC;
  st->t_hec_s = t_hec;
  st->t_kernels_s = t_kern;
  st->t_copy_s = t_copy;
  st->arena_highwater = kp.total_bytes;
  st->hec_flops = kp.hec_flops;
  st->hec_bytes = kp.hec_bytes;
  st->n_hec_launches = n_hec;
  st->t_total_s = now() - tw0;
  st->t_device_s = ms * 1e-3;
  st->n_launches = n_launch;
  st->n_graph_segments = n_segments;
}

// ---------------------------------------------------------------- no allocation
namespace {
// The one-stream walk with every byte in the static scratch: leaf uploads copy
// the library's interleaved host copy into a staging range at the end of the
// scratch and convert it into place on the device.
struct StaticOps {
  const Ctx& c;
  int prec;
  char* base;
  int64_t staging;    // offset of the staging range in the scratch
  hipStream_t st;

  void wait(int, int, int64_t, int64_t) {}
  void record(int, int64_t) {}
  void wait_pass(int, int, int64_t, int64_t) {}
  void record_pass(int, int64_t, int64_t) {}
  void upload_leaf(int64_t u, int64_t dev_off) const {
    const bool src_double = c.leaf_dtype[u] == CDAG_C128;
    const int64_t nt = c.dag.nt[u], e = c.dag.elems(u) / nt;
    HIPC(hipMemcpyAsync(base + staging, c.leaf_data[u].data(), c.leaf_data[u].size(), hipMemcpyHostToDevice, st));
    HIPC(launch_to_planar(src_double, prec == CDAG_FP64, base + staging, base + dev_off, nt, e, st));
  }
  void transfer(const PlanRec& r, const PassMap&, int64_t) {
    if (r.op != OP_H2D || !c.dag.is_leaf(r.node)) throw Error(CDAG_E_STATE, "static execute: a spill in the plan");
    upload_leaf(r.node, r.dev_off);
  }
  int64_t launch(int64_t g, const PassMap&) { return launch_step(c.kplan, g, prec, base, st, nullptr); }
};
}  // namespace

void device_execute_static(Ctx& c, int prec, cdag_exec_stats* st) {
  Device& D = *c.dev;
  const double tw0 = now();
  HIPC(hipSetDevice(D.device));
  char* base = scratch_address(D.device);
  if (!base) throw Error(CDAG_E_STATE, "static scratch not set up on this device");
  const Plan& p = c.plan;
  const KernelPlan& kp = c.kplan;
  if (p.chunks() != 1) throw Error(CDAG_E_STATE, "static execute runs whole tensors (t_chunks 1)");
  if (p.n_d2h > 0) throw Error(CDAG_E_BUDGET, "static execute: the plan spills to host memory");
  int64_t staging = 0;
  for (int64_t u = 0; u < c.dag.n_leaves; ++u) staging = std::max<int64_t>(staging, (int64_t)c.leaf_data[u].size());
  const int64_t stage_off = (kp.total_bytes + 255) / 256 * 256;
  if (stage_off + staging > kScratchBytes)
    throw Error(CDAG_E_NOMEM, "static execute needs " + std::to_string(stage_off + staging) +
                                  " bytes of device memory, the static scratch holds " + std::to_string(kScratchBytes));
  if ((int64_t)c.corr_host.size() * 8 < kp.corr_bytes || (int64_t)c.sums_host.size() * 8 < kp.sums_bytes)
    throw Error(CDAG_E_STATE, "static execute: result buffers not sized by the plan");
  hipStream_t s = D.comp;
  StaticOps ops{c, prec, base, stage_off, s};
  // descriptor tables (every call: another context may have used the scratch)
  HIPC(hipMemcpyAsync(base + kp.blob_off, kp.blob.data(), kp.blob.size(), hipMemcpyHostToDevice, s));
  if (c.leaves_resident)
    for (int64_t u = 0; u < c.dag.n_leaves; ++u) ops.upload_leaf(u, p.leaf_off[u]);
  const int64_t G = (int64_t)p.steps.size();
  int64_t n_launch = walk_steps(c, 0, G, true, false, ops);
  HIPC(launch_xsum(base, kp.xsum.desc_off, kp.xsum_entries_off, kp.xsum.n_desc, s));
  ++n_launch;
  HIPC(hipMemcpyAsync(c.corr_host.data(), base + kp.corr_off, (size_t)kp.corr_bytes, hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(c.sums_host.data(), base + kp.sums_off, (size_t)kp.sums_bytes, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  int64_t n_hec = 0;
  for (const Launch& L : kp.launches) n_hec += L.type == L_HEC;
  st->hec_flops = kp.hec_flops;
  st->hec_bytes = kp.hec_bytes;
  st->n_hec_launches = n_hec;
  st->n_launches = n_launch;
  st->arena_highwater = stage_off + staging;
  st->t_total_s = now() - tw0;
}

}  // namespace cdag
