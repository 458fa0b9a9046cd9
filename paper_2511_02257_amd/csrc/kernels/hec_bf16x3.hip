// Kernel table of the exterior contractions in split BF16 with three pieces: every tile, LDS
// stage count, grid policy, interior flag and carried traces.
#include "hec.hpp"
#include "kernels.hpp"

namespace cdag {
namespace {
template <class TL, int ST, bool PF, bool IN, bool TR>
struct Kern {
  static const void* fn() { return reinterpret_cast<const void*>(&hec_bf16<TL, ST, PF, 3, IN, TR>); }
};
}  // namespace

const void* hec_kernel_bf16x3(int tile, int stages, bool persistent, bool interior, bool traces) {
  return hec_table<Kern>(tile, stages, persistent, interior, traces);
}

}  // namespace cdag
