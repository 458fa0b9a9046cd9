// HIP kernels for gfx950 (CDNA4) besides the exterior contractions (hec.hpp,
// hec_*.hip): fixed-order split-K reduction, the FP64 root trace, the FP64
// cross-diagram sum, the layout conversion of uploaded leaves, and every
// launcher.  Tensor layout and descriptors: desc.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

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
// 4 consecutive elements of one row: vector loads when all 4 are in range and
// the row is 4-element aligned, otherwise element-wise with zero fill.
template <typename T>
__device__ __forceinline__ void load4(T (&r)[4], const T* src, int valid, bool vec) {
  if (vec && valid == 4) {
    typedef typename Vec2<T>::V V;
    constexpr int W = Vec2<T>::n;
    const V* s = reinterpret_cast<const V*>(src);
#pragma unroll
    for (int q = 0; q < 4 / W; ++q) {
      V v = s[q];
      const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
      for (int x = 0; x < W; ++x) r[q * W + x] = e[x];
    }
  } else {
#pragma unroll
    for (int x = 0; x < 4; ++x) r[x] = x < valid ? src[x] : T(0);
  }
}

// Four consecutive elements from a 16-byte aligned address, as vector loads.
template <typename T>
__device__ __forceinline__ void load4v(T (&r)[4], const T* src) {
  typedef typename Vec2<T>::V V;
  constexpr int W = Vec2<T>::n;
  const V* s = reinterpret_cast<const V*>(src);
#pragma unroll
  for (int q = 0; q < 4 / W; ++q) {
    V v = s[q];
    const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
    for (int x = 0; x < W; ++x) r[q * W + x] = e[x];
  }
}

// C(t) = sum_ij P[i,j] Q[j,i] over 4 x 4 blocks b = 0 .. nb^2 - 1 (block row
// ib = b / nb, block column jb = b % nb, nb = ceil(N / 4)).  A block's loads
// are 4 rows of P over columns 4jb.. and 4 rows of Q over columns 4ib.., so
// every load is a row segment and the transpose happens in registers.
// Summation order, the same in both layouts below: 256 partial sums, sum v
// adding (by fused multiply-adds, in FP64; exact products for FP32 inputs)
// the blocks v, v + 256, v + 512, ... in that order; sums 64w .. 64w + 63 meet
// in a fixed butterfly across a wave's lanes, and the four results are added
// in order w = 0, 1, 2, 3.  The result depends only on the data and N.
// Layouts: WG = false, one wave per (root, t), four per workgroup, lane l
// keeping the sums l, l + 64, l + 128, l + 192 (launches with many traces);
// WG = true, one workgroup per (root, t), thread x keeping sum x (launches
// with few traces, which one wave each would spread over few compute units
// with several rounds of loads per wave).
template <typename T, bool WG>
__global__ void __launch_bounds__(256, 3) hca_trace(char* __restrict__ arena, const HcaDesc* __restrict__ descs,
                                                 int n_desc, int64_t n_items) {
  __shared__ double part[2][4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NS = WG ? 1 : 4;      // partial sums per thread
  constexpr int W = WG ? 256 : 64;    // distance between a thread's sums' first blocks
  const int x = WG ? tid : lane;
  const int64_t first = WG ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * 4 + wave;
  const int64_t stride = WG ? (int64_t)gridDim.x : (int64_t)gridDim.x * 4;
  for (int64_t item = first; item - (WG ? 0 : wave) < n_items; item += stride) {
    if (!WG && item >= n_items) break;
    const int di = find_desc(&descs[0].item_begin, sizeof(HcaDesc) / 4, n_desc, item);
    const HcaDesc& h = descs[di];
    const int t = (int)(item - h.item_begin), n = h.n;
    const int64_t nn = (int64_t)n * n;
    const T* P = reinterpret_cast<const T*>(arena + h.p_off) + (int64_t)t * 2 * nn;
    const T* Q = reinterpret_cast<const T*>(arena + h.q_off) + (int64_t)t * 2 * nn;
    const int nb = (n + 3) >> 2, nbb = nb * nb;
    double sr[NS], si[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) sr[j] = si[j] = 0.0;
    T pr[4][4], pi[4][4], qr[4][4], qi[4][4];
    auto accumulate = [&]() {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double xr = (double)pr[a][c], xi = (double)pi[a][c];
          const double yr = (double)qr[c][a], yi = (double)qi[c][a];
          sr[0] = __builtin_fma(xr, yr, sr[0]);
          sr[0] = __builtin_fma(-xi, yi, sr[0]);
          si[0] = __builtin_fma(xr, yi, si[0]);
          si[0] = __builtin_fma(xi, yr, si[0]);
        }
    };
    // chunk c0: one block for each of the thread's sums (block c0 + W j for
    // sum j), each added into sum 0, after which the sums rotate by one, so
    // that the chunk ends with every sum back in its place (the loop stays
    // rolled, which keeps one block's registers live at a time).  WHOLE: N a
    // multiple of 4, so every block is whole and every row segment a 16-byte
    // aligned run, loaded as plain vector loads (masks would let the compiler
    // merge them into element-wise loads).
    auto sweep = [&](auto whole) {
      constexpr bool WHOLE = decltype(whole)::value;
      for (int c0 = x; c0 < nbb; c0 += W * NS) {
#pragma unroll 1
        for (int q = 0; q < NS; ++q) {
          // a block past the end reloads block c0 (in bounds) and is not added
          const int b = c0 + W * q < nbb ? c0 + W * q : c0;
          const int i0 = 4 * (b / nb), j0 = 4 * (b % nb);
          const int vj = min(4, n - j0), vi = min(4, n - i0);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t po = (int64_t)(i0 + r) * n + j0, qo = (int64_t)(j0 + r) * n + i0;
            if constexpr (WHOLE) {
              load4v<T>(pr[r], P + po);
              load4v<T>(pi[r], P + nn + po);
              load4v<T>(qr[r], Q + qo);
              load4v<T>(qi[r], Q + nn + qo);
            } else {
              load4<T>(pr[r], P + po, i0 + r < n ? vj : 0, false);
              load4<T>(pi[r], P + nn + po, i0 + r < n ? vj : 0, false);
              load4<T>(qr[r], Q + qo, j0 + r < n ? vi : 0, false);
              load4<T>(qi[r], Q + nn + qo, j0 + r < n ? vi : 0, false);
            }
          }
          // every load of the block ahead of its first use, so that they are
          // all in flight at once
          __builtin_amdgcn_sched_barrier(0);
          if (c0 + W * q < nbb) accumulate();
          __builtin_amdgcn_sched_barrier(0);
          if constexpr (NS > 1) {
            const double r0 = sr[0], i0s = si[0];
#pragma unroll
            for (int j = 0; j + 1 < NS; ++j) {
              sr[j] = sr[j + 1];
              si[j] = si[j + 1];
            }
            sr[NS - 1] = r0;
            si[NS - 1] = i0s;
          }
        }
      }
    };
    if ((n & 3) == 0) sweep(std::true_type{});
    else sweep(std::false_type{});
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        sr[j] += __shfl_xor(sr[j], o);
        si[j] += __shfl_xor(si[j], o);
      }
    double* out = reinterpret_cast<double*>(arena + h.out_off);
    if constexpr (WG) {
      if (lane == 0) {
        part[0][wave] = sr[0];
        part[1][wave] = si[0];
      }
      __syncthreads();
      if (tid == 0) {
        out[2 * t] = ((part[0][0] + part[0][1]) + part[0][2]) + part[0][3];
        out[2 * t + 1] = ((part[1][0] + part[1][1]) + part[1][2]) + part[1][3];
      }
      __syncthreads();
    } else if (lane == 0) {
      out[2 * t] = ((sr[0] + sr[1]) + sr[2]) + sr[3];
      out[2 * t + 1] = ((si[0] + si[1]) + si[2]) + si[3];
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
constexpr int64_t kMaxGrid = 1 << 20;
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
                    KernelCall* k) {
  if (variant == kGenVariantId) {        // contractions over any index pairs: FP64 and FP32
    if (prec > 1) return hipErrorInvalidValue;
    k->fn = prec == 0 ? hec_general_f64() : hec_general_f32();
    k->block = kTileShapes[1].nth;
    k->grid = grid_for(n_items);
    set_args(*k, arena, arena + desc_off, n_desc, n_items);
    return hipSuccess;
  }
  if (variant < 0 || variant >= 4 * kNumTiles || prec < 0 || prec > 3) return hipErrorInvalidValue;
  const int tile = variant % kNumTiles;
  const bool persistent = (variant / kNumTiles) % 2 == 0;
  const int stages = variant / (2 * kNumTiles) == 0 ? 2 : 1;
  const void* fn = prec == 0   ? hec_kernel_f64(tile, stages, persistent, interior)
                   : prec == 1 ? hec_kernel_f32(tile, stages, persistent, interior)
                   : prec == 2 ? hec_kernel_bf16x2(tile, stages, persistent, interior)
                               : hec_kernel_bf16x3(tile, stages, persistent, interior);
  if (fn == nullptr) return hipErrorInvalidValue;
  k->fn = fn;
  k->block = kTileShapes[tile].nth;
  k->grid = persistent ? persistent_grid(fn, k->block, n_items) : grid_for(n_items);
  set_args(*k, arena, arena + desc_off, n_desc, n_items);
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
