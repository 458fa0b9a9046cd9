// Launch planning: turn a placed plan into per-step kernel launches with
// arena-relative descriptor tables, and fix the arena layout.  Pure host code.
#pragma once

#include <cstdint>
#include <map>
#include <tuple>
#include <vector>

#include "host.hpp"
#include "../kernels/desc.hpp"

namespace cdag {

enum LaunchType : int32_t { L_HEC = 0, L_RED = 1, L_HCA = 2, L_XSUM = 3 };

struct Launch {
  int32_t type;
  int32_t tile;       // HEC: kernel variant (tile shape and grid policy)
  int32_t n_desc;
  int64_t desc_off;   // arena offset of the first descriptor
  int64_t n_items;    // HEC: tiles; RED: 256-element blocks; HCA: (root, t) pairs; XSUM: correlators
  int64_t host_desc;  // byte offset of the first descriptor in KernelPlan::blob
  double flops = 0;   // algorithmic flops of the launch (HEC, HCA)
  double bytes = 0;   // HEC, HCA: algorithmic bytes; RED: workspace read + output write
  int32_t kinds = 0;  // bit k set when a contraction of kind k is in the launch
  int32_t interior = 0;   // HEC: every contraction interior (hec_interior) for the variant's tile
  // HEC carrying the root traces of its step (trace fusion): tr_n_desc HcaDesc
  // at tr_desc_off (blob offset tr_host_desc), tr_n_items (root, t) items, and
  // their algorithmic flops and bytes (not in flops and bytes above)
  int32_t tr_n_desc = 0;
  int64_t tr_desc_off = 0, tr_host_desc = 0, tr_n_items = 0;
  double tr_flops = 0, tr_bytes = 0;
};

// Kernel variant of an exterior contraction: a tile shape (index into
// kTileShapes), a grid policy and the LDS stages, encoded as
// tile + kNumTiles * (grid + 2 * (2 - stages)) with grid 0 = persistent
// (compute units x occupancy workgroups striding over the work list),
// grid 1 = one workgroup per work item, and stages 2 (double buffer) or 1.
constexpr int kNumGrids = 2, kNumVariants = kNumTiles * kNumGrids * 2;
inline int variant_of(int tile, int grid, int stages = 2) {
  return tile + kNumTiles * (grid + 2 * (2 - stages));
}
inline int variant_tile(int v) { return v % kNumTiles; }
inline int variant_grid(int v) { return (v / kNumTiles) % 2; }
inline int variant_stages(int v) { return 2 - v / (2 * kNumTiles); }
// A kernel choice is a variant plus the split-K mode:
// choice = variant + kNumVariants * (split-K allowed ? 0 : 1).  Split-K, when
// allowed, follows the per-contraction rule of decompose(); either way the
// split count depends only on the contraction and the choice, never on how
// contractions are grouped into launches.
constexpr int kNumChoices = 2 * kNumVariants;
// Contractions over any index pairs run in their own launches of the general
// kernel (index-mapped loads and stores, 32 x 32 tiles of 256 threads, no
// split-K), launch variant kGenVariant; FP64 and FP32 only.
constexpr int kGenVariant = kNumVariants;
constexpr int kGenTile = 1;
static_assert(kGenVariant == kGenVariantId, "general kernel's launch variant");
inline int choice_of(int variant, bool split_k) { return variant + kNumVariants * (split_k ? 0 : 1); }
inline int choice_variant(int c) { return c % kNumVariants; }
inline bool choice_split_k(int c) { return c < kNumVariants; }
// Choice per (precision, kind, N): an explicit table entry (set through the
// ABI or by the autotuner) wins, else default_tile().
using TileTable = std::map<std::tuple<int, int, int>, int>;
int default_tile(int prec, int kind, int n);   // returns a choice
// Complex GEMM per time slice of an exterior contraction (Dag::gemm_shape).
struct Gemm { int64_t M, N, K; };
// GEMM dimensions, tile counts and split-K of one contraction with GEMM g, nt
// time slices and kernel `choice` (offsets and tile_begin unset).  nt_run > 0:
// the descriptor covers nt_run of the nt slices (one pass of a time-chunked
// execution); the split count still follows all nt.
void decompose(const Gemm& g, int nt, int choice, int prec, HecDesc* h, int nt_run = 0);
// Distinct (kind, N) among the exterior contractions of d (the keys of the
// kernel-choice table), each with its largest Nt and its largest GEMM (a
// general kind can occur with several operand ranks).
struct TuneShape { int nt; Gemm gemm; };
std::map<std::pair<int, int>, TuneShape> tune_shapes(const Dag& d);
// k-step of the matrix-core kernels: FP64 uses 16, FP32 and split-BF16 32.
inline int k_step(int prec) { return prec == 0 ? 16 : 32; }
// Split-K: aim for at least this many work items per contraction, keeping at
// least kMinKSplit of K per split.
constexpr int kSplitTarget = 512, kMinKSplit = 256;

struct KernelPlan {
  int prec = 0;
  int64_t chunks = 1;                // passes over the time slices (PlanOpts::t_chunks)
  std::vector<int64_t> launch_off;   // per step of each pass (k * n_steps + s): first launch index
                                     // (size chunks * n_steps + 1)
  std::vector<Launch> launches;
  Launch xsum{};
  int64_t xsum_entries_off = 0;     // arena offset of the XsumEntry table
  std::vector<uint8_t> blob;         // all descriptor tables, uploaded to blob_off
  // arena layout
  int64_t tensors_end = 0;           // leaf region + tensor pool and workspace of each half
  int64_t half_bytes = 0;            // tensor pool + workspace of one half (a pass's memory)
  int64_t ws_off = 0, ws_bytes = 0;  // workspace of half 0 (half 1: + half_bytes)
  int64_t blob_off = 0;
  int64_t corr_off = 0, corr_bytes = 0;   // per tree: [nt][2] doubles
  int64_t sums_off = 0, sums_bytes = 0;   // per correlator: [nt][2] doubles
  int64_t total_bytes = 0;
  std::vector<int64_t> tree_corr_off;     // per tree: byte offset inside the corr buffer
  std::vector<int64_t> sum_corr_off;      // per correlator: byte offset inside the sums buffer
  std::vector<int32_t> sum_nt;            // per correlator
  double flops = 0;
  double hec_flops = 0, hec_bytes = 0;
  int64_t hec_items = 0;                  // summed over all exterior-contraction launches
};

int64_t elem_bytes_of(int prec);                 // 16 for FP64, 8 otherwise
// Strides of spec s on tensors of dimension n (desc.hpp, IndexMap).
IndexMap index_map(const Spec& s, int n);
// fuse_traces: a step's root traces ride in one of its exterior-contraction
// launches (the last of one workgroup per item, not the general kernel) when
// it has one, instead of a launch of their own; either way the traces give
// the same bits.
KernelPlan make_kernel_plan(const Dag& d, const Plan& p, int prec, const TileTable& tiles, bool fuse_traces = false);

}  // namespace cdag
