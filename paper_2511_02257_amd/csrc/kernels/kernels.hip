// HIP kernels for gfx950 (CDNA4) besides the exterior contractions (hec.hpp,
// hec_*.hip): fixed-order split-K reduction, the FP64 root trace, the FP64
// cross-diagram sum, the layout conversion of uploaded leaves, and every
// launcher.  Tensor layout and descriptors: desc.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "desc.hpp"
#include "hec.hpp"
#include "kernels.hpp"

namespace cdag {

// ------------------------------------------------------------------ split-K reduce
template <typename T>
__global__ void __launch_bounds__(256) splitk_reduce(char* __restrict__ arena, const RedDesc* __restrict__ descs,
                                                     int n_desc, int64_t n_items) {
  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int di = find_desc(&descs[0].item_begin, sizeof(RedDesc) / 4, n_desc, item);
    const RedDesc& r = descs[di];
    const int64_t total = 2LL * r.nt * r.mn;
    const int64_t e = (item - r.item_begin) * 256 + threadIdx.x;
    if (e >= total) continue;
    const T* W = reinterpret_cast<const T*>(arena + r.ws_off);
    double s = 0.0;
    for (int k = 0; k < r.splits; ++k) s += (double)W[(int64_t)k * total + e];   // fixed order
    reinterpret_cast<T*>(arena + r.c_off)[e] = (T)s;
  }
}

// ------------------------------------------------------------------ root trace (FP64)
// The traces of one launch (device code and summation order: hec.hpp), in one
// of two layouts of the same order.  WG = false: one wave per (root, t), four
// per workgroup, for launches with many traces.  WG = true: one workgroup per
// (root, t), for launches with few traces (small waves), which one wave each
// would spread over few compute units with several rounds of loads per wave.
template <typename T, bool WG>
__global__ void __launch_bounds__(256, 3) hca_trace(char* __restrict__ arena, const HcaDesc* __restrict__ descs,
                                                    int n_desc, int64_t n_items) {
  if constexpr (WG) {
    __shared__ double part[2][4];
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x)
      trace_group<T, 4>(arena, descs, n_desc, item, true, (int)threadIdx.x, part);
  } else {
    const int wave = (int)threadIdx.x >> 6;
    for (int64_t base = (int64_t)blockIdx.x * 4; base < n_items; base += (int64_t)gridDim.x * 4) {
      const int64_t item = base + wave;
      if (item >= n_items) break;
      trace_wave<T, 4>(arena, descs, n_desc, item);
    }
  }
}

// ------------------------------------------------------------------ cross-diagram sum (FP64)
// One workgroup per correlator.  Thread i sums the entries i, i + 256, ... in
// that order; the 256 partial sums are then added in a fixed tree.  The order
// is fixed, so the result does not change from run to run.
__global__ void __launch_bounds__(256) xsum_kernel(char* __restrict__ arena, const XsumDesc* __restrict__ descs,
                                                   const XsumEntry* __restrict__ entries, int n_desc) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  for (int c = blockIdx.x; c < n_desc; c += gridDim.x) {
    const XsumDesc& x = descs[c];
    double* out = reinterpret_cast<double*>(arena + x.out_off);
    for (int t = 0; t < x.nt; ++t) {
      double sr = 0.0, si = 0.0;
      for (int e = x.e_begin + tid; e < x.e_end; e += 256) {
        const double* C = reinterpret_cast<const double*>(arena + entries[e].root_off);
        const double cr = C[2 * t], ci = C[2 * t + 1];
        sr += entries[e].w_re * cr - entries[e].w_im * ci;
        si += entries[e].w_re * ci + entries[e].w_im * cr;
      }
      red[0][tid] = sr;
      red[1][tid] = si;
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
          red[0][tid] += red[0][tid + w];
          red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
      }
      if (tid == 0) {
        out[2 * t] = red[0][0];
        out[2 * t + 1] = red[1][0];
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ layout conversion
// Interleaved complex [nt][e] (S: double or float) -> the device layout
// [nt][2][e] in T, converted on the device (the path that copies host data
// straight into device memory, without a pinned staging copy in device layout).
template <typename S, typename T>
__global__ void __launch_bounds__(256) to_planar(const S* __restrict__ src, T* __restrict__ dst, int64_t nt,
                                                 int64_t e) {
  const int64_t total = nt * e;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t t = i / e, x = i - t * e;
    const S re = src[2 * i], im = src[2 * i + 1];
    dst[2 * t * e + x] = (T)re;
    dst[(2 * t + 1) * e + x] = (T)im;
  }
}

// ------------------------------------------------------------------ launchers
namespace {
// Persistent launches: at most as many workgroups as can be resident at once
// (compute units x occupancy of the kernel); each loops over work items with
// a grid stride.  The occupancy query is made once per kernel.
unsigned persistent_grid(const void* kernel, int block, int64_t items) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;   // (kernel, device) -> resident workgroups
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  const auto key = std::make_pair(kernel, dev);
  int resident;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it == cache.end()) {
      int cus = 0, per_cu = 0;
      if (dev < 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
        resident = 1 << 16;
      else
        resident = cus * per_cu;
      cache.emplace(key, resident);
    } else {
      resident = it->second;
    }
  }
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(items, resident));
}
// traces per launch from which one wave per trace still fills 256 compute
// units with a workgroup of four waves each
constexpr int64_t kHcaWaveItems = 4 * 256;
unsigned grid_for(int64_t items) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(items, kMaxGrid)); }

void set_args(KernelCall& k, char* arena, const void* desc, int n_desc, int64_t n_items) {
  k.arena = arena;
  k.desc = desc;
  k.n_desc = n_desc;
  k.n_items = n_items;
  k.n_args = 4;
}
}  // namespace

void KernelCall::bind() {
  args[0] = &arena;
  args[1] = &desc;
  if (n_args == 5) {
    args[2] = &entries;
    args[3] = &n_desc;
    args[4] = nullptr;
  } else {
    args[2] = &n_desc;
    args[3] = &n_items;
    if (n_args == 7) {
      args[4] = &tdesc;
      args[5] = &n_tdesc;
      args[6] = &n_titems;
    }
  }
}

hipError_t launch(KernelCall& k, hipStream_t s) {
  k.bind();
  return hipLaunchKernel(k.fn, dim3(k.grid), dim3(k.block), k.args, 0, s);
}

// variant = tile + kNumTiles * (grid + 2 * stage_choice), stage_choice 0: two
// LDS stages, 1: one; grid 0: persistent, 1: one workgroup per work item.
// interior: every contraction of the launch passes hec_interior for the
// variant's tile and the precision's k-step (the host checks it).
hipError_t hec_call(int prec, int variant, bool interior, char* arena, int64_t desc_off, int n_desc, int64_t n_items,
                    KernelCall* k, int64_t tdesc_off, int n_tdesc, int64_t n_titems) {
  const bool traces = n_titems > 0;
  if (variant == kGenVariantId) {        // contractions over any index pairs: FP64 and FP32
    if (prec > 1 || traces) return hipErrorInvalidValue;
    k->fn = prec == 0 ? hec_general_f64() : hec_general_f32();
    k->block = kTileShapes[1].nth;
    k->grid = grid_for(n_items);
    set_args(*k, arena, arena + desc_off, n_desc, n_items);
    k->n_args = 7;
    return hipSuccess;
  }
  if (variant < 0 || variant >= 4 * kNumTiles || prec < 0 || prec > 3) return hipErrorInvalidValue;
  const int tile = variant % kNumTiles;
  const bool persistent = (variant / kNumTiles) % 2 == 0;
  const int stages = variant / (2 * kNumTiles) == 0 ? 2 : 1;
  const void* fn = prec == 0   ? hec_kernel_f64(tile, stages, persistent, interior, traces)
                   : prec == 1 ? hec_kernel_f32(tile, stages, persistent, interior, traces)
                   : prec == 2 ? hec_kernel_bf16x2(tile, stages, persistent, interior, traces)
                               : hec_kernel_bf16x3(tile, stages, persistent, interior, traces);
  if (fn == nullptr) return hipErrorInvalidValue;
  k->fn = fn;
  k->block = kTileShapes[tile].nth;
  set_args(*k, arena, arena + desc_off, n_desc, n_items);
  k->n_args = 7;
  if (traces) {
    // one workgroup per contraction work item, then the trace workgroups
    const int64_t blocks = n_items + trace_blocks(k->block, n_titems);
    if (blocks > kMaxGrid) return hipErrorInvalidValue;
    k->grid = (unsigned)blocks;
    k->tdesc = arena + tdesc_off;
    k->n_tdesc = n_tdesc;
    k->n_titems = n_titems;
  } else {
    k->grid = persistent ? persistent_grid(fn, k->block, n_items) : grid_for(n_items);
    k->tdesc = nullptr;
    k->n_tdesc = 0;
    k->n_titems = 0;
  }
  return hipSuccess;
}

hipError_t reduce_call(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, KernelCall* k) {
  k->fn = prec == 0 ? reinterpret_cast<const void*>(&splitk_reduce<double>)
                    : reinterpret_cast<const void*>(&splitk_reduce<float>);
  k->grid = grid_for(n_items);
  k->block = 256;
  set_args(*k, arena, arena + desc_off, n_desc, n_items);
  return hipSuccess;
}

// The trace layout by launch size: one wave per trace while that still gives
// every compute unit a workgroup (256 CUs), else one workgroup per trace.
hipError_t hca_call(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, KernelCall* k) {
  const bool wg = n_items < kHcaWaveItems;
  k->fn = prec == 0 ? (wg ? reinterpret_cast<const void*>(&hca_trace<double, true>)
                          : reinterpret_cast<const void*>(&hca_trace<double, false>))
                    : (wg ? reinterpret_cast<const void*>(&hca_trace<float, true>)
                          : reinterpret_cast<const void*>(&hca_trace<float, false>));
  k->grid = grid_for(wg ? n_items : (n_items + 3) / 4);
  k->block = 256;
  set_args(*k, arena, arena + desc_off, n_desc, n_items);
  return hipSuccess;
}

hipError_t xsum_call(char* arena, int64_t desc_off, int64_t entries_off, int n_desc, KernelCall* k) {
  k->fn = reinterpret_cast<const void*>(&xsum_kernel);
  k->grid = grid_for(n_desc);
  k->block = 256;
  set_args(*k, arena, arena + desc_off, n_desc, 0);
  k->entries = arena + entries_off;
  k->n_args = 5;
  return hipSuccess;
}

hipError_t launch_hec(int prec, int variant, bool interior, char* arena, int64_t desc_off, int n_desc,
                      int64_t n_items, hipStream_t s) {
  KernelCall k;
  hipError_t e = hec_call(prec, variant, interior, arena, desc_off, n_desc, n_items, &k);
  return e != hipSuccess ? e : launch(k, s);
}

hipError_t launch_reduce(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, hipStream_t s) {
  KernelCall k;
  const hipError_t e = reduce_call(prec, arena, desc_off, n_desc, n_items, &k);
  return e != hipSuccess ? e : launch(k, s);
}

hipError_t launch_hca(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, hipStream_t s) {
  KernelCall k;
  const hipError_t e = hca_call(prec, arena, desc_off, n_desc, n_items, &k);
  return e != hipSuccess ? e : launch(k, s);
}

hipError_t launch_to_planar(bool src_double, bool dst_double, const void* src, void* dst, int64_t nt, int64_t e,
                           hipStream_t s) {
  const dim3 grid(grid_for((nt * e + 255) / 256)), block(256);
  if (src_double && dst_double)
    hipLaunchKernelGGL((to_planar<double, double>), grid, block, 0, s, (const double*)src, (double*)dst, nt, e);
  else if (src_double)
    hipLaunchKernelGGL((to_planar<double, float>), grid, block, 0, s, (const double*)src, (float*)dst, nt, e);
  else if (dst_double)
    hipLaunchKernelGGL((to_planar<float, double>), grid, block, 0, s, (const float*)src, (double*)dst, nt, e);
  else
    hipLaunchKernelGGL((to_planar<float, float>), grid, block, 0, s, (const float*)src, (float*)dst, nt, e);
  return hipGetLastError();
}

hipError_t launch_xsum(char* arena, int64_t desc_off, int64_t entries_off, int n_desc, hipStream_t s) {
  KernelCall k;
  const hipError_t e = xsum_call(arena, desc_off, entries_off, n_desc, &k);
  return e != hipSuccess ? e : launch(k, s);
}

}  // namespace cdag
