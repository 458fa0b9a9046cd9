// Launchers of the HIP kernels (kernels.hip, hec_*.hip).  Every launcher takes the arena
// base and arena-relative descriptor offsets; prec: 0 FP64, 1 FP32, 2 split-BF16
// (two pieces), 3 split-BF16 (three pieces).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdag {

// One kernel launch as a function and its arguments, so that it can be
// launched on a stream or added to a graph as a kernel node.  Kernels take
// (arena, descriptors, n_desc, n_items); the exterior contractions also
// (trace descriptors, n_tdesc, n_titems) for the traces they may carry; the
// cross sum takes (arena, descriptors, entries, n_desc).  bind() points args
// at the fields; a copied KernelCall must be bound again.
struct KernelCall {
  const void* fn = nullptr;
  unsigned grid = 1, block = 1;
  char* arena = nullptr;
  const void* desc = nullptr;
  const void* entries = nullptr;
  int n_desc = 0;
  int64_t n_items = 0;
  const void* tdesc = nullptr;
  int n_tdesc = 0;
  int64_t n_titems = 0;
  int n_args = 4;
  void* args[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  void bind();
};
hipError_t launch(KernelCall& k, hipStream_t s);

// Exterior-contraction launch of kernel variant `variant`; interior: every
// contraction of the launch passes hec_interior (desc.hpp) for the variant's
// tile and the precision's k-step.  n_titems > 0: the launch also carries
// n_titems root traces (n_tdesc HcaDesc at arena offset tdesc_off) in
// hec_trace_blocks() more workgroups; only variants of one workgroup per
// item, not the general kernel, and the grid must stay within kMaxGrid
// (hipErrorInvalidValue otherwise).
hipError_t hec_call(int prec, int variant, bool interior, char* arena, int64_t desc_off, int n_desc,
                    int64_t n_items, KernelCall* k, int64_t tdesc_off = 0, int n_tdesc = 0, int64_t n_titems = 0);
hipError_t reduce_call(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, KernelCall* k);
hipError_t hca_call(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, KernelCall* k);
hipError_t xsum_call(char* arena, int64_t desc_off, int64_t entries_off, int n_desc, KernelCall* k);

hipError_t launch_hec(int prec, int variant, bool interior, char* arena, int64_t desc_off, int n_desc,
                      int64_t n_items, hipStream_t s);
hipError_t launch_reduce(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, hipStream_t s);
hipError_t launch_hca(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, hipStream_t s);
hipError_t launch_xsum(char* arena, int64_t desc_off, int64_t entries_off, int n_desc, hipStream_t s);
// Kernel tables of the exterior contractions, one translation unit per
// precision (hec_f64.hip, hec_f32.hip, hec_bf16x2.hip, hec_bf16x3.hip): the
// kernel of tile `tile` (index into kTileShapes), `stages` LDS stages (1 or 2),
// persistent grid or one workgroup per item, interior launch or not, with the
// step's traces carried or not; nullptr for a tile out of range or for traces
// on a persistent grid.  hec_general_*: the kernel of contractions over any
// index pairs.
const void* hec_kernel_f64(int tile, int stages, bool persistent, bool interior, bool traces);
const void* hec_kernel_f32(int tile, int stages, bool persistent, bool interior, bool traces);
const void* hec_kernel_bf16x2(int tile, int stages, bool persistent, bool interior, bool traces);
const void* hec_kernel_bf16x3(int tile, int stages, bool persistent, bool interior, bool traces);
const void* hec_general_f64();
const void* hec_general_f32();
// Interleaved complex [nt][e] (double or float) -> device layout [nt][2][e]
// (double or float), both in device memory.
hipError_t launch_to_planar(bool src_double, bool dst_double, const void* src, void* dst, int64_t nt, int64_t e,
                           hipStream_t s);

}  // namespace cdag
