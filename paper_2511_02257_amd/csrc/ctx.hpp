// Library context shared by the C ABI (capi.cpp) and the device runtime
// (runtime/executor.hip).
#pragma once

#include <cstdint>
#include <vector>

#include "host/host.hpp"
#include "host/kplan.hpp"
#include "../../include/cdag.h"

namespace cdag {

struct Device;   // device-side state, defined in runtime/executor.hip

struct Ctx {
  // contraction specs (op kinds kSpecBase + i) for the next build_cdag
  std::vector<Spec> specs;
  // build
  bool built = false;
  Dag dag;
  bool has_data = false;
  std::vector<std::vector<uint8_t>> leaf_data;  // interleaved host copies, dtype leaf_dtype
  std::vector<int32_t> leaf_dtype;              // CDAG_C128 or CDAG_C64 per leaf
  int32_t n_corr = 0;
  uint64_t data_version = 0;     // bumped by build_cdag (leaf data changed)
  // schedule
  bool scheduled = false;
  std::vector<int64_t> order;
  double t_sched = 0;
  // options
  int64_t budget = INT64_MAX;
  bool leaves_resident = false;
  int64_t wave_max = 4096;
  int64_t wave_lookahead = 0;
  int use_graphs = 1;            // 0 eager, 1 one-stream segments, 2 three-stream graph
  int64_t t_chunks = 1;
  bool fuse_traces = true;       // a step's traces ride in one of its contraction launches
  bool timing = false;
  TileTable tiles;               // (prec, kind, N) -> kernel variant overrides
  uint64_t version = 1;          // bumped by every change that invalidates a plan
  // last plan
  bool planned = false;
  uint64_t plan_version = 0;
  uint64_t plan_serial = 0;      // bumped each time a plan is (re)built
  int plan_prec = -1, plan_batched = -1;
  Plan plan;
  KernelPlan kplan;
  int64_t peak_post = 0, peak_live = 0;
  double t_plan = 0;
  // device
  Device* dev = nullptr;
  // results of the last execute
  bool have_results = false;
  std::vector<double> corr_host, sums_host;   // corr buffer (per tree), sums buffer
  std::vector<cdag_launch_record> records;    // per launch of the last timed execute
};

// Plans for (prec, batched) unless the cached plan already matches.
void ensure_plan(Ctx& c, int prec, int batched);

void device_destroy(Device* d);
void device_bind(Ctx& c, int device, void* compute_stream, void* copy_stream);
void device_bind_arena(Ctx& c, void* arena, uint64_t bytes);
void device_execute(Ctx& c, int prec, int batched, cdag_exec_stats* st);
// The planned execute on the compute stream alone, with the static scratch
// as the arena and no allocation (see cdag_execute_static).
void device_execute_static(Ctx& c, int prec, cdag_exec_stats* st);
// The eager two-stream issue order of the planned execute, recorded instead of
// issued (no HIP call); fail_at >= 0 throws Error(CDAG_E_HIP) at that record.
void trace_execute(const Ctx& c, int prec, std::vector<cdag_trace_rec>& out, int64_t fail_at);
int64_t device_autotune(Ctx& c, int prec, int batched, int reps, bool uniform);
int64_t device_autotune_insitu(Ctx& c, int prec, int batched, int reps);

}  // namespace cdag
