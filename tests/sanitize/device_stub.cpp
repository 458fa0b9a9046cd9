// Host-only build of the library for the sanitizer test: the device runtime
// (HIP) is replaced by functions that fail with CDAG_E_STATE, so every host
// entry point (build, schedule, memory model, plan) runs under ASan/UBSan.
#include "ctx.hpp"

namespace cdag {
namespace {
[[noreturn]] void no_device() { throw Error(CDAG_E_STATE, "no device in the sanitizer build"); }
}  // namespace
void device_destroy(Device*) {}
void device_bind(Ctx&, int, void*, void*) { no_device(); }
void device_bind_arena(Ctx&, void*, uint64_t) { no_device(); }
void device_execute(Ctx&, int, int, cdag_exec_stats*) { no_device(); }
void device_execute_static(Ctx&, int, cdag_exec_stats*) { no_device(); }
int64_t device_autotune(Ctx&, int, int, int, bool) { no_device(); }
int64_t device_autotune_insitu(Ctx&, int, int, int) { no_device(); }
void trace_execute(const Ctx&, int, std::vector<cdag_trace_rec>&, int64_t) { no_device(); }
}  // namespace cdag
