// Launch descriptors shared by the host launch planner and the HIP kernels.
// Every address is a byte offset from the arena base passed to the kernel, so
// a descriptor table stays valid for any arena address and can be uploaded
// once per plan.
//
// Tensor layout in the arena (all precisions): [nt][2][N^rank] -- per time
// slice the real plane, then the imaginary plane, each row-major.  A
// contraction is then, per t, the complex GEMM C_t (M x N) = A_t (M x K) B_t
// (K x N) with row-major planes:
//   K22: (M, N, K) = (n, n, n)
//   K32: (M, N, K) = (n^2, n, n)     A = X[i,j | k], B = Y[k | l]
//   K33: (M, N, K) = (n, n, n^2)     A = X[i | j,l], B = Y[j,l | m]
#pragma once
#include <stdint.h>

namespace cdag {

// Exterior-contraction tile shapes (workgroup output tile BM x BN, threads).
// The kernels instantiate exactly these, in this order.
struct TileShape { int32_t bm, bn, nth; };
constexpr int kNumTiles = 6;
constexpr TileShape kTileShapes[kNumTiles] = {
    {64, 64, 256}, {32, 32, 256}, {48, 48, 64}, {128, 64, 256}, {64, 32, 256}, {64, 64, 512}};

// Launch variant of the general kernel (contractions over any index pairs):
// one past the tile x grid x stages variants.
constexpr int kGenVariantId = 4 * kNumTiles;

// Most workgroups in one launch; a launch with more work items strides.
constexpr int64_t kMaxGrid = 1 << 20;
// Root traces that one workgroup of `nth` threads takes when an exterior-
// contraction launch carries its step's traces (a group of four waves per
// trace; a 64-thread workgroup takes one as a single wave), and the
// workgroups that n of them need.
constexpr int traces_per_block(int nth) { return nth >= 256 ? nth / 256 : 1; }
constexpr int64_t trace_blocks(int nth, int64_t n) {
  return (n + traces_per_block(nth) - 1) / traces_per_block(nth);
}

// One exterior contraction inside a grouped launch.
struct HecDesc {
  int64_t a_off, b_off, c_off;   // t = 0 slice of A, B and C
  int64_t ws_off;                // split-K partials [splits][nt][2][M*N] (accumulator type), or -1
  int64_t map_off;               // IndexMap of a contraction over any index pairs, or -1
  int32_t M, N, K, nt;
  int32_t tiles_m, tiles_n, splits, k_split;   // k_split: K range per split (multiple of the k-step)
  int32_t tile_begin, tile_count;              // this op's work items in the launch
};

// An interior contraction for a tile of bm x bn and a k-step bk: every work
// item is a whole tile with whole k-slices, rows of A and B hold a multiple of
// 8 elements, and both operand slices start 16-byte aligned (planes and time
// slices then stay aligned).  A launch whose contractions are all interior
// runs the kernel form with unpredicated vector loads and stores.
inline bool hec_interior(const HecDesc& h, int bm, int bn, int bk) {
  return h.map_off < 0 && h.M % bm == 0 && h.N % bn == 0 && h.K % 8 == 0 && h.N % 8 == 0 && h.K % bk == 0 &&
         h.k_split % bk == 0 && (h.a_off & 15) == 0 && (h.b_off & 15) == 0;
}

// Element strides of a contraction over any index pairs, digit by digit.  The
// GEMM indices m (the left operand's free axes, in order), k (the summed axes,
// in pair order) and n (the right operand's free axes) are mixed-radix numbers
// in N, most significant digit first; the element offset within one plane is
// A(m, k) = sum_d m_d a_m[d] + sum_d k_d a_k[d], and likewise for B(k, n) and
// for C(m, n), whose strides carry the output's axis order.
struct IndexMap {
  int32_t n, dm, dk, dn;         // radix N; digits of m, k and n
  int64_t a_m[3], a_k[3];
  int64_t b_k[3], b_n[3];
  int64_t c_m[3], c_n[3];
};

// Fixed-order reduction of split-K partials into C (one per split op).
struct RedDesc {
  int64_t ws_off, c_off;
  int32_t mn, nt, splits, item_begin;          // items: ceil(2*nt*mn / 256) blocks
};

// Root trace C(t) = sum_ij P[t,i,j] Q[t,j,i] into the FP64 correlator buffer.
struct HcaDesc {
  int64_t p_off, q_off, out_off;               // out: [nt][2] doubles
  int32_t n, nt, item_begin, pad;              // items: one per time slice
};

// Cross-diagram sum for one correlator: sum over entries [e_begin, e_end)
// (ascending input graph) of w * C_root(t), in a fixed order.
struct XsumDesc {
  int64_t out_off;                             // [nt][2] doubles
  int32_t e_begin, e_end, nt, pad;
};
struct XsumEntry {
  int64_t root_off;                            // [nt][2] doubles
  double w_re, w_im;
};

}  // namespace cdag
