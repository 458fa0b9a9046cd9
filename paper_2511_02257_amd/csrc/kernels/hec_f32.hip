// Kernel table of the exterior contractions in complex FP32: every tile, LDS
// stage count, grid policy, interior flag and carried traces. Also the general kernel
// (contractions over any index pairs).
#include "hec.hpp"
#include "kernels.hpp"

namespace cdag {
namespace {
template <class TL, int ST, bool PF, bool IN, bool TR>
struct Kern {
  static const void* fn() { return reinterpret_cast<const void*>(&hec_mfma<float, TL, ST, PF, false, IN, TR>); }
};
}  // namespace

const void* hec_kernel_f32(int tile, int stages, bool persistent, bool interior, bool traces) {
  return hec_table<Kern>(tile, stages, persistent, interior, traces);
}

const void* hec_general_f32() {
  return reinterpret_cast<const void*>(&hec_mfma<float, Tile1, 2, false, true, false>);
}

}  // namespace cdag
