// Launchers of the HIP kernels (kernels.hip).  Every launcher takes the arena
// base and arena-relative descriptor offsets; prec: 0 FP64, 1 FP32, 2 split-BF16.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdag {

hipError_t launch_hec(int prec, int variant, char* arena, int64_t desc_off, int n_desc, int64_t n_items,
                      hipStream_t s);
hipError_t launch_reduce(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, hipStream_t s);
hipError_t launch_hca(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, hipStream_t s);
hipError_t launch_xsum(char* arena, int64_t desc_off, int64_t entries_off, int n_desc, hipStream_t s);

}  // namespace cdag
