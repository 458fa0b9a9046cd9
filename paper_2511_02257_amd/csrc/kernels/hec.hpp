// Device code of the grouped exterior contractions on the matrix cores
// (gfx950, CDNA4), shared by the per-precision kernel tables (hec_*.hip) and
// the other kernels (kernels.hip).  Tensor layout and descriptors: desc.hpp.
//
// Exterior contraction = per time slice a complex GEMM C = A B with planar
// (re, im) operands.  With real matrix-core products only, either
//   Re C = Ar Br - Ai Bi,  Im C = Ar Bi + Ai Br              (four products)
// or Gauss's form with three,
//   P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi),  Re C = P1 - P2,
//   Im C = P3 - (P1 + P2).
// Flop counts use the ZGEMM convention (8 flops per complex multiply-add)
// whichever form runs.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "desc.hpp"

namespace cdag {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v8s __attribute__((ext_vector_type(8)));

// Largest i with first[i * stride] <= item, where first[0] == 0 and the
// values strictly increase.  Called by all 64 lanes of a wave with the same
// item: each round the lanes read the starts of 64 equal blocks of the
// remaining range and a ballot picks the block holding the item, so n
// descriptors take ceil(log64 n) dependent loads instead of log2 n.
__device__ __forceinline__ int find_desc(const int32_t* first, int stride_words, int n, int64_t item) {
  const int lane = threadIdx.x & 63;
  int lo = 0, cnt = n;
  while (cnt > 1) {
    const int step = (cnt + 63) >> 6;
    const bool in_range = lane * step < cnt;
    const bool ok = in_range && (int64_t)first[(int64_t)(lo + lane * step) * stride_words] <= item;
    const unsigned long long m = __ballot(ok);
    const int last = 63 - __clzll(m);       // lane 0 always holds: first[lo] <= item
    lo += last * step;
    cnt = min(step, cnt - last * step);
  }
  return lo;
}

// Tile configuration: WGM x WGN waves per workgroup, each holding TM x TN
// blocks of 16 x 16 outputs; the workgroup tile is BM x BN.
template <int WGM_, int WGN_, int TM_, int TN_>
struct Tile {
  static constexpr int WGM = WGM_, WGN = WGN_, TM = TM_, TN = TN_;
  static constexpr int NTH = 64 * WGM * WGN;
  static constexpr int BM = 16 * WGM * TM, BN = 16 * WGN * TN;
};
// Must match kTileShapes in desc.hpp, entry by entry.
typedef Tile<2, 2, 2, 2> Tile0;   //  64 x 64, 256 threads
typedef Tile<2, 2, 1, 1> Tile1;   //  32 x 32, 256 threads
typedef Tile<1, 1, 3, 3> Tile2;   //  48 x 48,  64 threads
typedef Tile<2, 2, 4, 2> Tile3;   // 128 x 64, 256 threads
typedef Tile<2, 2, 2, 1> Tile4;   //  64 x 32, 256 threads
typedef Tile<2, 4, 2, 1> Tile5;   //  64 x 64, 512 threads (half the accumulators per wave)

// Occupancy target of an exterior-contraction kernel: the waves per SIMD that
// its register budget must allow (the compiler keeps each lane within
// 512 / waves registers).  P: 0 FP64, 1 FP32, 2 split BF16 (either piece
// count); 1 leaves the register budget to the compiler.
template <int P, class TL, int ST, bool PF>
struct Occupancy {
  static constexpr int waves = 1;
};
// Targets that shrink a variant's registers without spilling, where LDS leaves
// room for the extra workgroups (measured: split-BF16 K33 on the 64 x 64 / 256
// tile +3 %; the others within noise).  Only the grids of one workgroup per
// item take them: squeezed to 127 registers, the persistent FP32 one-stage
// 64 x 64 kernels with 32-deep k-slices gave wrong results.
#define CDAG_OCCUPANCY(P, TL, ST, W) \
  template <> struct Occupancy<P, TL, ST, false> { static constexpr int waves = W; };
CDAG_OCCUPANCY(0, Tile0, 1, 3)
CDAG_OCCUPANCY(0, Tile0, 2, 2)
CDAG_OCCUPANCY(0, Tile4, 1, 3)
CDAG_OCCUPANCY(0, Tile4, 2, 2)
CDAG_OCCUPANCY(0, Tile1, 1, 4)
CDAG_OCCUPANCY(1, Tile0, 1, 4)
CDAG_OCCUPANCY(1, Tile0, 2, 4)
CDAG_OCCUPANCY(1, Tile3, 1, 3)
CDAG_OCCUPANCY(1, Tile4, 1, 4)
CDAG_OCCUPANCY(1, Tile4, 2, 4)
CDAG_OCCUPANCY(2, Tile0, 1, 3)
CDAG_OCCUPANCY(2, Tile3, 1, 2)
#undef CDAG_OCCUPANCY

struct WorkItem {
  const HecDesc* h;
  int t, m0, n0, sp, kbeg, kend;
};

template <int BM, int BN>
__device__ __forceinline__ WorkItem decode_item(const HecDesc* descs, int n_desc, int64_t item) {
  WorkItem w;
  const int di = find_desc(&descs[0].tile_begin, sizeof(HecDesc) / 4, n_desc, item);
  const HecDesc* h = &descs[di];
  int64_t local = item - h->tile_begin;
  // XCD-aware order.  Workgroups go to the eight XCDs round robin (item mod 8
  // for one workgroup per item, and for a persistent grid of a multiple of 8
  // workgroups).  When the contraction's items start on a multiple of 8 and Nt
  // is one, item x + 8 j takes time slice x + 8 (j / T), tile j mod T (T tiles
  // per slice): every tile of a slice runs on one XCD, one after another, so
  // the operand panels they share come from that XCD's L2, and each XCD reads
  // only its own slices.  A bijection of the contraction's items; with T = 1
  // it is the identity.
  const int64_t T = (int64_t)h->splits * h->tiles_n * h->tiles_m;
  if (T > 1 && ((h->tile_begin | h->nt) & 7) == 0) {
    const int32_t x = (int32_t)(local & 7), j = (int32_t)(local >> 3), T32 = (int32_t)T;
    local = (int64_t)(x + 8 * (j / T32)) * T + (j % T32);
  }
  w.sp = (int)(local % h->splits);
  local /= h->splits;
  const int tn = (int)(local % h->tiles_n);
  local /= h->tiles_n;
  const int tm = (int)(local % h->tiles_m);
  w.t = (int)(local / h->tiles_m);
  w.m0 = tm * BM;
  w.n0 = tn * BN;
  w.kbeg = w.sp * h->k_split;
  w.kend = min(h->K, w.kbeg + h->k_split);
  w.h = h;
  return w;
}

// Operand view of one work item: the contraction's descriptor, the A and B
// slices of its time slice, and the tile and K range.
template <typename T>
struct ItemView {
  const HecDesc* h;
  const T* A;
  const T* B;
  int M, N, K, t, sp, m0, n0, kbeg, kend;
  bool avec;         // rows of A allow 8-element vector loads
  const IndexMap* map;   // a contraction over any index pairs, else nullptr
};

// Element offset of a mixed-radix index x (nd digits in radix n, most
// significant first) with per-digit strides st.
__device__ __forceinline__ int64_t digit_offset(int64_t x, int nd, int n, const int64_t* st) {
  int64_t off = 0;
#pragma unroll
  for (int d = 2; d >= 0; --d) {
    if (d < nd) {
      off += (x % n) * st[d];
      x /= n;
    }
  }
  return off;
}

template <typename T, int BM, int BN>
__device__ __forceinline__ ItemView<T> view_item(char* arena, const HecDesc* descs, int n_desc, int64_t item) {
  const WorkItem w = decode_item<BM, BN>(descs, n_desc, item);
  ItemView<T> v;
  v.h = w.h;
  v.M = w.h->M;
  v.N = w.h->N;
  v.K = w.h->K;
  v.t = w.t;
  v.sp = w.sp;
  v.m0 = w.m0;
  v.n0 = w.n0;
  v.kbeg = w.kbeg;
  v.kend = w.kend;
  v.A = reinterpret_cast<const T*>(arena + w.h->a_off) + (int64_t)w.t * 2 * v.M * v.K;
  v.B = reinterpret_cast<const T*>(arena + w.h->b_off) + (int64_t)w.t * 2 * v.K * v.N;
  v.map = w.h->map_off >= 0 ? reinterpret_cast<const IndexMap*>(arena + w.h->map_off) : nullptr;
  v.avec = (v.K & 7) == 0 && v.map == nullptr;
  return v;
}

// ------------------------------------------------------------------ FP64 / FP32
template <typename T> struct Mfma;
// Output layout of one 16x16 block: lane l, register v holds column l % 16 and
// row row(l / 16, v).  The f64 instruction interleaves rows across the four
// 16-lane groups; the f32 one gives each group four consecutive rows
// (both checked on the device with a single-instruction probe).
template <> struct Mfma<double> {
  typedef v4d V;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int grp, int v) { return grp + 4 * v; }
};
template <> struct Mfma<float> {
  typedef v4f V;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int grp, int v) { return 4 * grp + v; }
};

template <typename T> struct Vec2;
template <> struct Vec2<double> { typedef double2 V; static constexpr int n = 2; };
template <> struct Vec2<float> { typedef float4 V; static constexpr int n = 4; };
// 16 bytes of T as one register tuple.  Loaded operands are kept in these, so
// that every 16-byte load fills a whole tuple that stays live until its LDS
// store (a load into a tuple the compiler only partly keeps makes it wait for
// that load before the tuple's registers are reused, which stalls the
// prefetch of the next k-slice behind its own latency).
template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef double V __attribute__((ext_vector_type(2))); };
template <> struct Vec16<float> { typedef float V __attribute__((ext_vector_type(4))); };

// Wait for every vector memory operation of this wave (s_waitcnt vmcnt(0);
// expcnt and lgkmcnt left free).  Called where the loaded k-slice is stored to
// LDS, which needs it anyway: past this point no load is in flight on any
// path, so the compiler has nothing to wait for when the next loads reuse
// registers.
__device__ __forceinline__ void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// Scheduling fence: the compiler moves no instruction across it.  Keeps a
// k-slice's prefetch loads ahead of its products (the scheduler would
// otherwise sink them next to their LDS store, exposing their latency) and
// the LDS store behind them.
__device__ __forceinline__ void fence() { __builtin_amdgcn_sched_barrier(0); }

// 8 consecutive elements of one row: vector loads when fully in range and the
// row is 8-element aligned, otherwise element-wise with zero fill.
template <typename T>
__device__ __forceinline__ void load8(T (&r)[8], const T* src, int valid, bool vec) {
  if (vec && valid == 8) {
    typedef typename Vec2<T>::V V;
    constexpr int W = Vec2<T>::n;
    const V* s = reinterpret_cast<const V*>(src);
#pragma unroll
    for (int q = 0; q < 8 / W; ++q) {
      V v = s[q];
      const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
      for (int i = 0; i < W; ++i) r[q * W + i] = e[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = i < valid ? src[i] : T(0);
  }
}

// One 16-byte chunk (W = 16 / sizeof(T) elements) of a row: a vector load when
// all W are in range and rows are W-element aligned, otherwise element-wise
// with zero fill.
template <typename T>
__device__ __forceinline__ void load16b(T (&r)[16 / sizeof(T)], const T* src, int valid, bool vec) {
  constexpr int W = 16 / (int)sizeof(T);
  typedef typename Vec2<T>::V V;
  static_assert(sizeof(V) == 16, "one vector per chunk");
  if (vec && valid == W) {
    V v = *reinterpret_cast<const V*>(src);
    const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
    for (int i = 0; i < W; ++i) r[i] = e[i];
  } else {
#pragma unroll
    for (int i = 0; i < W; ++i) r[i] = i < valid ? src[i] : T(0);
  }
}

// ------------------------------------------------------------------ root traces
// K consecutive elements of one row (K = 2 or 4): WHOLE, vector loads from a
// K-element aligned address; otherwise element-wise, the first `valid` of
// them, with zero fill: every lane loads (element 0 in place of one past the
// run, and `safe`, an address in range, when the run is empty), so that no
// load sits behind a branch and the addresses need not stay live.
template <typename T, int K, bool WHOLE>
__device__ __forceinline__ void load_run(T (&r)[K], const T* src, int valid, const T* safe) {
  if constexpr (WHOLE) {
    constexpr int V = (int)(16 / sizeof(T)) < K ? (int)(16 / sizeof(T)) : K;   // elements per load
    typedef T VT __attribute__((ext_vector_type(V)));
#pragma unroll
    for (int q = 0; q < K / V; ++q) {
      const VT v = *reinterpret_cast<const VT*>(src + q * V);
#pragma unroll
      for (int x = 0; x < V; ++x) r[q * V + x] = v[x];
    }
  } else {
    const T* base = valid > 0 ? src : safe;
#pragma unroll
    for (int x = 0; x < K; ++x) {
      const T v = base[x < valid ? x : 0];
      r[x] = x < valid ? v : T(0);
    }
  }
}

// C(t) = sum_ij P[i,j] Q[j,i] over 4 x 4 blocks b = 0 .. nb^2 - 1 (block row
// ib = b / nb, block column jb = b % nb, nb = ceil(N / 4)).  A block reads 4
// rows of P over columns 4jb.. and 4 rows of Q over columns 4ib.., so every
// load is a row segment and the transpose happens in registers; within a
// block the terms P[a][c] Q[c][a] are added for a = 0..3, c = 0..3 in that
// order.  Summation order, the same in every layout: 256 partial sums, sum v
// adding (by fused multiply-adds, in FP64; exact products for FP32 inputs) the
// blocks v, v + 256, v + 512, ... in that order; sums 64w .. 64w + 63 meet in
// a fixed butterfly across a wave's lanes, and the four results are added in
// order w = 0, 1, 2, 3.  The result depends only on the data and N.
//
// The NS partial sums of one thread: sum j takes the blocks x + W j + 256 r,
// r = 0, 1, ... (x: the thread's place in its layout; W NS = 256).  A chunk
// brings one block for each of the sums, each added into sum 0, after which
// the sums rotate by one, so that the chunk ends with every sum back in its
// place (the loop stays rolled, which keeps one block's registers live at a
// time).  A block is loaded RPB rows of P (a = h RPB ..) at a time, with the
// matching RPB columns of Q's 4 rows: RPB = 4, all of it at once; RPB = 2, in
// two halves, which halves the registers (the order of the terms is the
// same).  WHOLE: N a multiple of 4, so every block is whole and every row
// segment aligned, loaded as plain vector loads (masks would let the
// compiler merge them into element-wise loads).
template <typename T, int NS, bool WHOLE, int RPB>
__device__ __forceinline__ void trace_sums(const T* P, const T* Q, int n, int x, double (&sr)[NS],
                                           double (&si)[NS]) {
  constexpr int W = 256 / NS;
  const int64_t nn = (int64_t)n * n;
  const int nb = (n + 3) >> 2, nbb = nb * nb;
  T pr[RPB][4], pi[RPB][4], qr[4][RPB], qi[4][RPB];
#pragma unroll 1
  for (int c0 = x; c0 < nbb; c0 += 256) {
#pragma unroll 1
    for (int q = 0; q < NS; ++q) {
      // a block past the end reloads block c0 (in bounds) and is not added
      const bool add = c0 + W * q < nbb;
      const int b = add ? c0 + W * q : c0;
      const int i0 = 4 * (b / nb), j0 = 4 * (b % nb);
#pragma unroll
      for (int h = 0; h < 4 / RPB; ++h) {
        const int ia = i0 + h * RPB;    // first P row (and Q column) of this part
#pragma unroll
        for (int r = 0; r < RPB; ++r) {
          const int64_t po = (int64_t)(ia + r) * n + j0;
          const int valid = ia + r < n ? min(4, n - j0) : 0;
          load_run<T, 4, WHOLE>(pr[r], P + po, valid, P);
          load_run<T, 4, WHOLE>(pi[r], P + nn + po, valid, P);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t qo = (int64_t)(j0 + c) * n + ia;
          const int valid = j0 + c < n ? max(0, min(RPB, n - ia)) : 0;
          load_run<T, RPB, WHOLE>(qr[c], Q + qo, valid, Q);
          load_run<T, RPB, WHOLE>(qi[c], Q + nn + qo, valid, Q);
        }
        // every load of the part ahead of its first use, so that they are all
        // in flight at once
        __builtin_amdgcn_sched_barrier(0);
        if (add) {
#pragma unroll
          for (int a = 0; a < RPB; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const double xr = (double)pr[a][c], xi = (double)pi[a][c];
              const double yr = (double)qr[c][a], yi = (double)qi[c][a];
              sr[0] = __builtin_fma(xr, yr, sr[0]);
              sr[0] = __builtin_fma(-xi, yi, sr[0]);
              si[0] = __builtin_fma(xr, yi, si[0]);
              si[0] = __builtin_fma(xi, yr, si[0]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // the next part's loads stay after this part's products (the
        // compiler would otherwise merge Q's adjacent column pairs of the two
        // halves into one load, and hold both halves' registers)
        if constexpr (RPB < 4) asm volatile("" ::: "memory");
      }
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
}

// Where trace item `item` reads and writes (every lane of the wave calls it
// with the same item).
template <typename T>
struct TraceItem {
  const T *P, *Q;
  int n, t;
  double* out;
  __device__ __forceinline__ TraceItem(char* arena, const HcaDesc* descs, int n_desc, int64_t item) {
    const HcaDesc& h = descs[find_desc(&descs[0].item_begin, sizeof(HcaDesc) / 4, n_desc, item)];
    t = (int)(item - h.item_begin);
    n = h.n;
    const int64_t nn = (int64_t)n * n;
    P = reinterpret_cast<const T*>(arena + h.p_off) + (int64_t)t * 2 * nn;
    Q = reinterpret_cast<const T*>(arena + h.q_off) + (int64_t)t * 2 * nn;
    out = reinterpret_cast<double*>(arena + h.out_off) + 2 * t;
  }
  template <int NS, int RPB>
  __device__ __forceinline__ void sums(int x, double (&sr)[NS], double (&si)[NS]) const {
#pragma unroll
    for (int j = 0; j < NS; ++j) sr[j] = si[j] = 0.0;
    if ((n & 3) == 0) trace_sums<T, NS, true, RPB>(P, Q, n, x, sr, si);
    else trace_sums<T, NS, false, RPB>(P, Q, n, x, sr, si);
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        sr[j] += __shfl_xor(sr[j], o);
        si[j] += __shfl_xor(si[j], o);
      }
  }
};

// Wave layout: one trace per wave, lane l keeping the sums l, l + 64, l + 128,
// l + 192.  No barrier.
template <typename T, int RPB>
__device__ __forceinline__ void trace_wave(char* arena, const HcaDesc* descs, int n_desc, int64_t item) {
  const TraceItem<T> it(arena, descs, n_desc, item);
  double sr[4], si[4];
  it.template sums<4, RPB>(threadIdx.x & 63, sr, si);
  if ((threadIdx.x & 63) == 0) {
    it.out[0] = ((sr[0] + sr[1]) + sr[2]) + sr[3];
    it.out[1] = ((si[0] + si[1]) + si[2]) + si[3];
  }
}

// Workgroup layout: one trace per group of four waves (g_tid = 0 .. 255, the
// thread's place in its group), thread x keeping sum x; the four wave sums
// meet in `part` (the group's LDS).  Holds two workgroup barriers, so every
// thread of the workgroup calls it equally often; a group with active = false
// takes part in the barriers only.
template <typename T, int RPB>
__device__ __forceinline__ void trace_group(char* arena, const HcaDesc* descs, int n_desc, int64_t item, bool active,
                                            int g_tid, double (&part)[2][4]) {
  const int wave = g_tid >> 6;
  double sr[1] = {0.0}, si[1] = {0.0};
  double* out = nullptr;
  if (active) {
    const TraceItem<T> it(arena, descs, n_desc, item);
    it.template sums<1, RPB>(g_tid, sr, si);
    out = it.out;
    if ((g_tid & 63) == 0) {
      part[0][wave] = sr[0];
      part[1][wave] = si[0];
    }
  }
  __syncthreads();
  if (active && g_tid == 0) {
    out[0] = ((part[0][0] + part[0][1]) + part[0][2]) + part[0][3];
    out[1] = ((part[1][0] + part[1][1]) + part[1][2]) + part[1][3];
  }
  __syncthreads();
}

// Traces carried by an exterior-contraction launch (the traces of the same
// plan step, which read only earlier steps' outputs): block b after the
// contractions' work items takes traces b * G .. b * G + G - 1, G = NTH / 256
// (traces_per_block) in the workgroup layout, or one in the wave layout for
// 64-thread tiles; blocks load in halves, so that the trace path needs no
// more registers than the contractions do.
template <typename T, int NTH>
__device__ __forceinline__ void trace_block(char* arena, const HcaDesc* descs, int n_desc, int64_t n_items,
                                            int64_t b) {
  if constexpr (NTH >= 256) {
    static_assert(NTH % 256 == 0, "whole groups of four waves");
    constexpr int G = traces_per_block(NTH);
    __shared__ double part[G][2][4];
    const int g = (int)threadIdx.x / 256;
    const int64_t item = b * G + g;
    trace_group<T, 2>(arena, descs, n_desc, item, item < n_items, (int)threadIdx.x % 256, part[g]);
  } else {
    static_assert(NTH == 64, "one wave");
    if (b < n_items) trace_wave<T, 2>(arena, descs, n_desc, b);
  }
}

// Store one 16x16 block pair (Re, Im) of accumulators with the instruction's
// row layout; rows and columns outside M x N are skipped (INNER: the block is
// known to lie inside).  NT: non-temporal stores, which keep a launch's
// outputs (read by a later wave, long after the caches have turned over) from
// displacing the operands that its other work items are still reading from L2.
template <typename T, typename V, bool NT, bool INNER = false>
__device__ __forceinline__ void store_block(T* C, int M, int N, int row0, int col, const V& re, const V& im,
                                           int lk, const IndexMap* map = nullptr) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int m = row0 + Mfma<T>::row(lk, v);
    if (INNER || (m < M && col < N)) {
      // a general contraction writes C(m, n) at its output axis order
      const int64_t off = map ? digit_offset(m, map->dm, map->n, map->c_m) + digit_offset(col, map->dn, map->n, map->c_n)
                              : (int64_t)m * N + col;
      T* pr = &C[off];
      T* pi = &C[(int64_t)M * N + off];
      if (NT) {
        __builtin_nontemporal_store(re[v], pr);
        __builtin_nontemporal_store(im[v], pi);
      } else {
        *pr = re[v];
        *pi = im[v];
      }
    }
  }
}

// ST: LDS stages.  2 = double buffer (one barrier per k-chunk); 1 = one
// buffer refilled from the register prefetch (two barriers per k-chunk, half
// the LDS, more workgroups per compute unit).  PF: a workgroup that strides
// over several items (persistent grid) prefetches its next item.
// GEN: every work item is a contraction over any index pairs; operands are
// loaded and the output stored through its IndexMap, element by element.
// FULL: every contraction of the launch is interior (hec_interior): operands
// load with unpredicated 16-byte loads and outputs store without bounds tests.
// TR: the launch also carries the root traces of its plan step (n_titems
// (root, t) items described by tdescs), in the workgroups after the
// contractions' work items (one workgroup per item; trace_block); without TR
// the last three arguments are unused.
template <typename T, class TL, int ST, bool PF, bool GEN = false, bool FULL = false, bool TR = false>
__global__ void __launch_bounds__(TL::NTH, (Occupancy<sizeof(T) == 8 ? 0 : 1, TL, ST, PF>::waves))
hec_mfma(char* __restrict__ arena, const HecDesc* __restrict__ descs, int n_desc, int64_t n_items,
         const HcaDesc* __restrict__ tdescs, int n_tdesc, int64_t n_titems) {
  static_assert(!(GEN && FULL), "a general contraction is never interior");
  static_assert(!(TR && (PF || GEN)), "traces ride only in launches of one workgroup per item");
  typedef typename Mfma<T>::V V;
  constexpr int NTH = TL::NTH, BM = TL::BM, BN = TL::BN, TM = TL::TM, TN = TL::TN;
  // k-slice: 16 (FP64) or 32 (FP32) k per LDS stage, so that a K = 64
  // contraction's item runs four or two slices.  A rows are padded so that
  // the 16 rows read by one instruction fall in distinct LDS banks.
  constexpr int BK = sizeof(T) == 8 ? 16 : 32, APAD = BK + (sizeof(T) == 8 ? 1 : 4), BPAD = BN + 16;
  constexpr int SPR = BK / 8;   // 8-element A segments per row
  // The A tile is split into 8-element row segments ([plane][row][k / 8]); the
  // B tile into 16-byte row chunks of W elements ([plane][k][n / W]), so that
  // consecutive lanes load and store consecutive 16 bytes (coalesced loads,
  // LDS stores free of bank conflicts).
  constexpr int W = 16 / (int)sizeof(T);
  constexpr int SEGA = 2 * BM * SPR, SEGB = 2 * BK * (BN / W);
  constexpr int LA = (SEGA + NTH - 1) / NTH, LB = (SEGB + NTH - 1) / NTH;
  static_assert(BN % W == 0, "B chunks must tile the row");
  // CT: the FP32 output tile of an interior launch goes through LDS, so that
  // every thread stores whole 16-byte pieces of 128-byte lines (the f32
  // accumulator layout alone gives 64-byte row segments per 16 lanes, and
  // the memory then writes 1.3 x the output bytes).  The tile [plane][m][n]
  // reuses the operand stages' LDS once the item's last slice is done.
  constexpr bool CT = FULL && sizeof(T) == 4;
  constexpr int CPAD = BN + 4;          // 16-lane row groups of one instruction in distinct banks
  constexpr int A_ELEMS = ST * 2 * BM * APAD, B_ELEMS = ST * 2 * BK * BPAD, C_ELEMS = CT ? 2 * BM * CPAD : 0;
  constexpr int SMEM = A_ELEMS + B_ELEMS > C_ELEMS ? A_ELEMS + B_ELEMS : C_ELEMS;
  __shared__ __attribute__((aligned(16))) T smem[SMEM];
  T (&As)[ST][2][BM][APAD] = *reinterpret_cast<T (*)[ST][2][BM][APAD]>(smem);            // [stage][plane][m][k]
  T (&Bs)[ST][2][BK][BPAD] = *reinterpret_cast<T (*)[ST][2][BK][BPAD]>(smem + A_ELEMS);  // [stage][plane][k][n]
  T (&Cs)[2][BM][CPAD] = *reinterpret_cast<T (*)[2][BM][CPAD]>(smem);                   // [plane][m][n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / TL::WGN, wn = wave % TL::WGN, li = lane & 15, lk = lane >> 4;

  typedef typename Vec16<T>::V VL;
  constexpr int NA = 8 / W;     // 16-byte tuples per A segment
  VL ra[LA][NA], rb[LB];
  auto gload = [&](const ItemView<T>& o, int k0) {
    if constexpr (FULL) {
      // interior tile, whole k-slice: unpredicated 16-byte loads
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        const int seg = tid + q * NTH;
        if (SEGA % NTH == 0 || seg < SEGA) {
          const int p = seg / (SPR * BM), r = (seg % (SPR * BM)) / SPR, hh = seg % SPR;
          const VL* src = reinterpret_cast<const VL*>(o.A + (int64_t)p * o.M * o.K + (int64_t)(o.m0 + r) * o.K +
                                                      k0 + 8 * hh);
#pragma unroll
          for (int j = 0; j < NA; ++j) ra[q][j] = src[j];
        }
      }
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int seg = tid + q * NTH;
        if (SEGB % NTH == 0 || seg < SEGB) {
          const int p = seg / (BK * (BN / W)), rem = seg % (BK * (BN / W));
          const int kk = rem / (BN / W), cw = rem % (BN / W);
          rb[q] = *reinterpret_cast<const VL*>(o.B + (int64_t)p * o.K * o.N + (int64_t)(k0 + kk) * o.N + o.n0 +
                                               W * cw);
        }
      }
      return;
    }
    // ragged or general: element-wise where a row or k range ends
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int seg = tid + q * NTH;
      if (SEGA % NTH == 0 || seg < SEGA) {
        const int p = seg / (SPR * BM), r = (seg % (SPR * BM)) / SPR, hh = seg % SPR;
        const int am = o.m0 + r, ak = k0 + 8 * hh;
        T e[8];
        if constexpr (GEN) {
          const IndexMap& mp = *o.map;
          const T* plane = o.A + (int64_t)p * o.M * o.K;
          const int64_t row = am < o.M ? digit_offset(am, mp.dm, mp.n, mp.a_m) : 0;
#pragma unroll
          for (int i = 0; i < 8; ++i)
            e[i] = (am < o.M && ak + i < o.kend) ? plane[row + digit_offset(ak + i, mp.dk, mp.n, mp.a_k)] : T(0);
        } else {
          const int av = am < o.M ? max(0, min(8, o.kend - ak)) : 0;
          load8<T>(e, o.A + (int64_t)p * o.M * o.K + (int64_t)am * o.K + ak, av, o.avec);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) ra[q][i / W][i % W] = e[i];
      }
    }
    const bool bvw = (o.N % W) == 0;
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int seg = tid + q * NTH;
      if (SEGB % NTH == 0 || seg < SEGB) {
        const int p = seg / (BK * (BN / W)), rem = seg % (BK * (BN / W));
        const int kk = rem / (BN / W), cw = rem % (BN / W);
        const int bkk = k0 + kk, bn = o.n0 + W * cw;
        T e[W];
        if constexpr (GEN) {
          const IndexMap& mp = *o.map;
          const T* plane = o.B + (int64_t)p * o.K * o.N;
          const int64_t row = bkk < o.kend ? digit_offset(bkk, mp.dk, mp.n, mp.b_k) : 0;
#pragma unroll
          for (int i = 0; i < W; ++i)
            e[i] = (bkk < o.kend && bn + i < o.N) ? plane[row + digit_offset(bn + i, mp.dn, mp.n, mp.b_n)] : T(0);
        } else {
          const int bv = bkk < o.kend ? max(0, min(W, o.N - bn)) : 0;
          load16b<T>(e, o.B + (int64_t)p * o.K * o.N + (int64_t)bkk * o.N + bn, bv, bvw);
        }
#pragma unroll
        for (int i = 0; i < W; ++i) rb[q][i] = e[i];
      }
    }
  };
  auto sstore = [&](int st) {
    wait_loads();
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int seg = tid + q * NTH;
      if (SEGA % NTH == 0 || seg < SEGA) {
        const int p = seg / (SPR * BM), r = (seg % (SPR * BM)) / SPR, hh = seg % SPR;
#pragma unroll
        for (int i = 0; i < 8; ++i) As[st][p][r][8 * hh + i] = ra[q][i / W][i % W];
      }
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int seg = tid + q * NTH;
      if (SEGB % NTH == 0 || seg < SEGB) {
        const int p = seg / (BK * (BN / W)), rem = seg % (BK * (BN / W));
        const int kk = rem / (BN / W), cw = rem % (BN / W);
        *reinterpret_cast<VL*>(&Bs[st][p][kk][W * cw]) = rb[q];
      }
    }
  };

  int64_t item = blockIdx.x;
  if constexpr (TR) {
    if (item >= n_items) {
      trace_block<T, NTH>(arena, tdescs, n_tdesc, n_titems, item - n_items);
      return;
    }
  }
  if (item >= n_items) return;
  ItemView<T> cur = view_item<T, BM, BN>(arena, descs, n_desc, item);
  gload(cur, cur.kbeg);
  for (;;) {
    // With PF the next item is located now and its first k-slice is loaded
    // during this item's last slice, so the workgroup never waits for a fresh
    // item's first loads.
    const int64_t next = item + gridDim.x;
    const bool has_next = next < n_items;
    ItemView<T> nxt = cur;
    if (PF && has_next) nxt = view_item<T, BM, BN>(arena, descs, n_desc, next);

    // Complex products.  With G3 (Gauss), three real products per complex one:
    // P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi), then Re = P1 - P2 and
    // Im = P3 - (P1 + P2).  Otherwise four, Re (in P1) += Ar Br + Ai (-Bi) and
    // Im (in P3) += Ar Bi + Ai Br.  G3 needs a third accumulator, so it is used
    // only where a wave holds at most two 16 x 16 blocks.
    constexpr bool G3 = TM * TN <= 2;
    V p1[TM][TN], p2[TM][TN], p3[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        p1[i][j] = V{0, 0, 0, 0};
        p2[i][j] = V{0, 0, 0, 0};
        p3[i][j] = V{0, 0, 0, 0};
      }

    // One k-slice of products from LDS stage st.
    auto mma_slice = [&](int st) {
#pragma unroll
      for (int k4 = 0; k4 < BK / 4; ++k4) {
        const int kk = 4 * k4 + lk;
        T a_r[TM], a_i[TM], b_r[TN], b_i[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          a_r[i] = As[st][0][(wm * TM + i) * 16 + li][kk];
          a_i[i] = As[st][1][(wm * TM + i) * 16 + li][kk];
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          b_r[j] = Bs[st][0][kk][(wn * TN + j) * 16 + li];
          b_i[j] = Bs[st][1][kk][(wn * TN + j) * 16 + li];
        }
        if constexpr (G3) {
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              p1[i][j] = Mfma<T>::mma(a_r[i], b_r[j], p1[i][j]);
              p2[i][j] = Mfma<T>::mma(a_i[i], b_i[j], p2[i][j]);
              p3[i][j] = Mfma<T>::mma(a_r[i] + a_i[i], b_r[j] + b_i[j], p3[i][j]);
            }
        } else {
          T b_n[TN];
#pragma unroll
          for (int j = 0; j < TN; ++j) b_n[j] = -b_i[j];
          // Consecutive instructions go to different accumulators; each
          // accumulator still adds its two products in the same order.
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              p1[i][j] = Mfma<T>::mma(a_r[i], b_r[j], p1[i][j]);
              p3[i][j] = Mfma<T>::mma(a_r[i], b_i[j], p3[i][j]);
            }
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              p1[i][j] = Mfma<T>::mma(a_i[i], b_n[j], p1[i][j]);
              p3[i][j] = Mfma<T>::mma(a_i[i], b_r[j], p3[i][j]);
            }
        }
      }
    };
    // Each slice but the last loads the next one while its products run; the
    // last loads the next item's first slice (PF).  The last slice is peeled
    // off so that every pass of the loop stores what it loaded: no load is in
    // flight when the loop comes round, and the compiler has no reason to wait
    // for the prefetch before the products.
    const int nk = (cur.kend - cur.kbeg + BK - 1) / BK;
    int c = 0;
    if (ST == 2) {
      sstore(0);
      __syncthreads();
      for (; c + 1 < nk; ++c) {
        gload(cur, cur.kbeg + (c + 1) * BK);
        fence();
        mma_slice(c & 1);
        fence();
        sstore((c & 1) ^ 1);
        __syncthreads();
      }
    } else {
      for (; c + 1 < nk; ++c) {
        sstore(0);
        __syncthreads();
        gload(cur, cur.kbeg + (c + 1) * BK);
        fence();
        mma_slice(0);
        __syncthreads();
      }
      if (nk > 0) {
        sstore(0);
        __syncthreads();
      }
    }
    if (PF && has_next) gload(nxt, nxt.kbeg);
    fence();
    if (nk > 0) {
      mma_slice(ST == 2 ? (c & 1) : 0);
      __syncthreads();
    }

    const HecDesc& h = *cur.h;
    const int M = cur.M, N = cur.N;
    T* C;
    if (h.splits > 1)
      C = reinterpret_cast<T*>(arena + h.ws_off) + ((int64_t)cur.sp * h.nt + cur.t) * 2 * M * N;
    else
      C = reinterpret_cast<T*>(arena + h.c_off) + (int64_t)cur.t * 2 * M * N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        V re = p1[i][j], im = p3[i][j];
        if constexpr (G3) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            re[v] = p1[i][j][v] - p2[i][j][v];
            im[v] = p3[i][j][v] - (p1[i][j][v] + p2[i][j][v]);
          }
        }
        if constexpr (CT) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = (wm * TM + i) * 16 + Mfma<T>::row(lk, v), cc = (wn * TN + j) * 16 + li;
            Cs[0][r][cc] = re[v];
            Cs[1][r][cc] = im[v];
          }
        } else {
          store_block<T, V, true, FULL>(C, M, N, cur.m0 + (wm * TM + i) * 16, cur.n0 + (wn * TN + j) * 16 + li,
                                        re, im, lk, GEN ? cur.map : nullptr);
        }
      }
    if constexpr (CT) {
      __syncthreads();
      typedef typename Vec16<T>::V VC;
      constexpr int QR = BN / 4;   // 16-byte pieces per tile row
#pragma unroll
      for (int e = tid; e < 2 * BM * QR; e += NTH) {
        const int p = e / (BM * QR), rem = e % (BM * QR), r = rem / QR, c4 = rem % QR;
        const VC val = *reinterpret_cast<const VC*>(&Cs[p][r][4 * c4]);
        T* dst = C + (int64_t)p * M * N + (int64_t)(cur.m0 + r) * N + cur.n0 + 4 * c4;
        __builtin_nontemporal_store(val, reinterpret_cast<VC*>(dst));
      }
      __syncthreads();   // the next item's first LDS store reuses Cs
    }
    if (!has_next) break;
    item = next;
    if (PF) {
      cur = nxt;
    } else {
      cur = view_item<T, BM, BN>(arena, descs, n_desc, item);
      gload(cur, cur.kbeg);
    }
  }
}

// ------------------------------------------------------------------ split BF16
// Each FP32 operand x is split into P bf16 pieces by repeated rounding:
// p0 = bf16(x), p1 = bf16(x - p0), p2 = bf16(x - p0 - p1) (each difference is
// exact in FP32).  A piece is at most 2^-8 of the one before, so a real
// product x y is approximated by the piece products p_i q_j with i + j < P:
//   P = 2: hi*hi + hi*lo + lo*hi (three products; the dropped lo*lo and the
//          remainders of the split leave up to ~3 * 2^-16 relative error);
//   P = 3: the six products with i + j <= 2 (the dropped terms and the
//          remainder are of order 2^-24, the FP32 rounding of the inputs).
// The products accumulate in FP32 on the bf16 matrix cores, smallest first.
template <int P>
__device__ __forceinline__ void split_bf16(float x, __bf16 (&piece)[P]) {
  float rest = x;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    piece[i] = (__bf16)rest;
    rest -= (float)piece[i];
  }
}

// The same split for two values at once: each rounding is one packed
// conversion of the pair (v_cvt_pk_bf16_f32), each difference two FP32
// subtractions, with the same results as split_bf16 on each value.
typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf_t __attribute__((ext_vector_type(2)));
typedef __bf16 v4bf_t __attribute__((ext_vector_type(4)));
template <int P>
__device__ __forceinline__ void split_bf16_pair(v2f_t x, v2bf_t (&piece)[P]) {
  v2f_t rest = x;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    piece[i] = __builtin_convertvector(rest, v2bf_t);
    rest = rest - __builtin_convertvector(piece[i], v2f_t);
  }
}
__device__ __forceinline__ v8bf cat_bf16(v2bf_t a, v2bf_t b, v2bf_t c, v2bf_t d) {
  const v4bf_t ab = __builtin_shufflevector(a, b, 0, 1, 2, 3), cd = __builtin_shufflevector(c, d, 0, 1, 2, 3);
  return __builtin_shufflevector(ab, cd, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Piece products kept for P pieces, smallest first: term t multiplies piece
// term_x(t) of A by piece term_y(t) of B.
template <int P> __device__ constexpr int n_terms() { return P == 2 ? 3 : 6; }
template <int P> __device__ constexpr int term_x(int t) {
  return P == 2 ? (t == 0 ? 1 : 0) : (t == 0 ? 2 : (t == 2 || t == 3) ? 1 : 0);
}
template <int P> __device__ constexpr int term_y(int t) {
  return P == 2 ? (t == 1 ? 1 : 0) : (t == 1 ? 2 : (t == 2 || t == 4) ? 1 : 0);
}

// TR as in hec_mfma (the traces read the FP32 storage of these modes).
template <class TL, int ST_, bool PF, int P, bool FULL = false, bool TR = false>
__global__ void __launch_bounds__(TL::NTH, (Occupancy<2, TL, ST_, PF>::waves))
hec_bf16(char* __restrict__ arena, const HecDesc* __restrict__ descs, int n_desc, int64_t n_items,
         const HcaDesc* __restrict__ tdescs, int n_tdesc, int64_t n_titems) {
  static_assert(!(TR && PF), "traces ride only in launches of one workgroup per item");
  constexpr int NTH = TL::NTH, BM = TL::BM, BN = TL::BN, TM = TL::TM, TN = TL::TN;
  constexpr int BK = 32, PAD = BK + 8;     // bf16 per LDS row (16-byte aligned rows)
  // Two stages of three pieces of the 128 x 64 tile would exceed the 160 KB of
  // LDS; that variant keeps one stage (the arithmetic is the same either way).
  constexpr int ST = (ST_ == 2 && 2 * 2 * P * (BM + BN) * PAD * 2 > 160 * 1024) ? 1 : ST_;
  // A: segments of 8 consecutive k of one row m.  B: segments of 8 consecutive
  // k of two adjacent columns n (consecutive lanes take consecutive column
  // pairs, so each of the 8 loads is coalesced), which become two 16-byte rows
  // of the transposed LDS tile.
  constexpr int SEGA = 2 * BM * (BK / 8), SEGB = 2 * (BK / 8) * (BN / 2);
  constexpr int LA = (SEGA + NTH - 1) / NTH, LB = (SEGB + NTH - 1) / NTH;
  static_assert(BN % 2 == 0, "B column pairs");
  // [stage][plane][piece][row][k]: A rows are m, B rows are n (B is stored transposed)
  __shared__ __attribute__((aligned(16))) __bf16 As[ST][2][P][BM][PAD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[ST][2][P][BN][PAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / TL::WGN, wn = wave % TL::WGN, li = lane & 15, lk = lane >> 4;

  // loaded operands as whole register tuples (see Vec16)
  typedef float v2f __attribute__((ext_vector_type(2)));
  v4f ra[LA][2];
  v2f rb[LB][8];
  auto gload = [&](const ItemView<float>& o, int k0) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int seg = tid + q * NTH;
      if (SEGA % NTH == 0 || seg < SEGA) {
        const int p = seg / (4 * BM), r = (seg % (4 * BM)) >> 2, qq = seg & 3;
        const int am = o.m0 + r, ak = k0 + 8 * qq;
        const float* src = o.A + (int64_t)p * o.M * o.K + (int64_t)am * o.K + ak;
        if constexpr (FULL) {
          ra[q][0] = reinterpret_cast<const v4f*>(src)[0];
          ra[q][1] = reinterpret_cast<const v4f*>(src)[1];
        } else {
          float e[8];
          const int av = am < o.M ? max(0, min(8, o.kend - ak)) : 0;
          load8<float>(e, src, av, o.avec);
#pragma unroll
          for (int i = 0; i < 8; ++i) ra[q][i / 4][i % 4] = e[i];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int seg = tid + q * NTH;
      if (SEGB % NTH == 0 || seg < SEGB) {
        const int p = seg / ((BK / 8) * (BN / 2)), rem = seg % ((BK / 8) * (BN / 2));
        const int g = rem / (BN / 2), cp = rem % (BN / 2);
        const int bk0 = k0 + 8 * g, bn = o.n0 + 2 * cp;
        const float* src = o.B + (int64_t)p * o.K * o.N + (int64_t)bk0 * o.N + bn;
        if (FULL || (bk0 + 8 <= o.kend && bn + 2 <= o.N && (o.N & 1) == 0)) {
#pragma unroll
          for (int i = 0; i < 8; ++i) rb[q][i] = *reinterpret_cast<const v2f*>(src + (int64_t)i * o.N);
        } else {
#pragma unroll
          for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int c = 0; c < 2; ++c)
              rb[q][i][c] = (bk0 + i < o.kend && bn + c < o.N) ? src[(int64_t)i * o.N + c] : 0.0f;
        }
      }
    }
  };
  auto sstore = [&](int st) {
    wait_loads();
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int seg = tid + q * NTH;
      if (SEGA % NTH == 0 || seg < SEGA) {
        const int p = seg / (4 * BM), r = (seg % (4 * BM)) >> 2, qq = seg & 3;
        // the 8 values as 4 adjacent pairs; each piece is one 16-byte row segment
        v2bf_t pc[4][P];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          split_bf16_pair<P>(v2f_t{ra[q][j / 2][2 * (j % 2)], ra[q][j / 2][2 * (j % 2) + 1]}, pc[j]);
#pragma unroll
        for (int x = 0; x < P; ++x)
          *reinterpret_cast<v8bf*>(&As[st][p][x][r][8 * qq]) = cat_bf16(pc[0][x], pc[1][x], pc[2][x], pc[3][x]);
      }
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int seg = tid + q * NTH;
      if (SEGB % NTH == 0 || seg < SEGB) {
        const int p = seg / ((BK / 8) * (BN / 2)), rem = seg % ((BK / 8) * (BN / 2));
        const int g = rem / (BN / 2), cp = rem % (BN / 2);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          // column c's 8 values of k as 4 pairs of consecutive k
          v2bf_t pc[4][P];
#pragma unroll
          for (int j = 0; j < 4; ++j) split_bf16_pair<P>(v2f_t{rb[q][2 * j][c], rb[q][2 * j + 1][c]}, pc[j]);
#pragma unroll
          for (int x = 0; x < P; ++x)
            *reinterpret_cast<v8bf*>(&Bs[st][p][x][2 * cp + c][8 * g]) =
                cat_bf16(pc[0][x], pc[1][x], pc[2][x], pc[3][x]);
        }
      }
    }
  };

  int64_t item = blockIdx.x;
  if constexpr (TR) {
    if (item >= n_items) {
      trace_block<float, NTH>(arena, tdescs, n_tdesc, n_titems, item - n_items);
      return;
    }
  }
  if (item >= n_items) return;
  ItemView<float> cur = view_item<float, BM, BN>(arena, descs, n_desc, item);
  gload(cur, cur.kbeg);
  for (;;) {
    // with PF: next item located now, its first k-slice loaded during this
    // item's last slice
    const int64_t next = item + gridDim.x;
    const bool has_next = next < n_items;
    ItemView<float> nxt = cur;
    if (PF && has_next) nxt = view_item<float, BM, BN>(arena, descs, n_desc, next);

    v4f cr[TM][TN], ci[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) { cr[i][j] = v4f{0, 0, 0, 0}; ci[i][j] = v4f{0, 0, 0, 0}; }

    // One k-slice of products from LDS stage st.
    auto mma_slice = [&](int st) {
      // one 16x16x32 step: lane holds k = 8*lk .. 8*lk+7 of row li (A) / column li (B)
      v8bf a[TM][2][P], b[TN][2][P], bn[TN][P];   // [block][plane][piece]; bn: pieces of -Bi
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int x = 0; x < P; ++x)
            a[i][p][x] = *reinterpret_cast<const v8bf*>(&As[st][p][x][(wm * TM + i) * 16 + li][8 * lk]);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int x = 0; x < P; ++x)
            b[j][p][x] = *reinterpret_cast<const v8bf*>(&Bs[st][p][x][(wn * TN + j) * 16 + li][8 * lk]);
        // -Bi: flip the bf16 sign bits
#pragma unroll
        for (int x = 0; x < P; ++x) {
          v8s sg = *reinterpret_cast<v8s*>(&b[j][1][x]) ^ (short)0x8000;
          bn[j][x] = *reinterpret_cast<v8bf*>(&sg);
        }
      }
      // Re += Ar Br - Ai Bi ; Im += Ar Bi + Ai Br.  Each real product is the sum
      // of the piece products (x, y) with x + y < P, smallest terms first:
      // (1,0) (0,1) (0,0) for P = 2; (2,0) (0,2) (1,1) (1,0) (0,1) (0,0) for
      // P = 3.  Term by term over all accumulators, so that consecutive
      // instructions are independent; each accumulator adds its terms in the
      // same order.
#define MM(acc, u, v) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(u, v, acc, 0, 0, 0)
#define TERM(CR_X, CR_Y, CI_X, CI_Y)            \
  _Pragma("unroll") for (int i = 0; i < TM; ++i) \
  _Pragma("unroll") for (int j = 0; j < TN; ++j) { MM(cr[i][j], CR_X, CR_Y); MM(ci[i][j], CI_X, CI_Y); }
#pragma unroll
      for (int t = 0; t < n_terms<P>(); ++t) {
        const int x = term_x<P>(t), y = term_y<P>(t);
        TERM(a[i][0][x], b[j][0][y], a[i][0][x], b[j][1][y])
      }
#pragma unroll
      for (int t = 0; t < n_terms<P>(); ++t) {
        const int x = term_x<P>(t), y = term_y<P>(t);
        TERM(a[i][1][x], bn[j][y], a[i][1][x], b[j][0][y])
      }
#undef TERM
#undef MM
    };
    // The last slice is peeled off, as in hec_mfma: every pass of the loop
    // stores what it loaded.
    const int nk = (cur.kend - cur.kbeg + BK - 1) / BK;
    int c = 0;
    if (ST == 2) {
      sstore(0);
      __syncthreads();
      for (; c + 1 < nk; ++c) {
        gload(cur, cur.kbeg + (c + 1) * BK);
        fence();
        mma_slice(c & 1);
        fence();
        sstore((c & 1) ^ 1);
        __syncthreads();
      }
    } else {
      for (; c + 1 < nk; ++c) {
        sstore(0);
        __syncthreads();
        gload(cur, cur.kbeg + (c + 1) * BK);
        fence();
        mma_slice(0);
        __syncthreads();
      }
      if (nk > 0) {
        sstore(0);
        __syncthreads();
      }
    }
    if (PF && has_next) gload(nxt, nxt.kbeg);
    fence();
    if (nk > 0) {
      mma_slice(ST == 2 ? (c & 1) : 0);
      __syncthreads();
    }

    const HecDesc& h = *cur.h;
    const int M = cur.M, N = cur.N;
    float* C;
    if (h.splits > 1)
      C = reinterpret_cast<float*>(arena + h.ws_off) + ((int64_t)cur.sp * h.nt + cur.t) * 2 * M * N;
    else
      C = reinterpret_cast<float*>(arena + h.c_off) + (int64_t)cur.t * 2 * M * N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        store_block<float, v4f, false, FULL>(C, M, N, cur.m0 + (wm * TM + i) * 16, cur.n0 + (wn * TN + j) * 16 + li,
                                             cr[i][j], ci[i][j], lk);
    if (!has_next) break;
    item = next;
    if (PF) {
      cur = nxt;
    } else {
      cur = view_item<float, BM, BN>(arena, descs, n_desc, item);
      gload(cur, cur.kbeg);
    }
  }
}

static_assert(Tile0::BM == kTileShapes[0].bm && Tile0::BN == kTileShapes[0].bn && Tile0::NTH == kTileShapes[0].nth, "tile 0");
static_assert(Tile1::BM == kTileShapes[1].bm && Tile1::BN == kTileShapes[1].bn && Tile1::NTH == kTileShapes[1].nth, "tile 1");
static_assert(Tile2::BM == kTileShapes[2].bm && Tile2::BN == kTileShapes[2].bn && Tile2::NTH == kTileShapes[2].nth, "tile 2");
static_assert(Tile3::BM == kTileShapes[3].bm && Tile3::BN == kTileShapes[3].bn && Tile3::NTH == kTileShapes[3].nth, "tile 3");
static_assert(Tile4::BM == kTileShapes[4].bm && Tile4::BN == kTileShapes[4].bn && Tile4::NTH == kTileShapes[4].nth, "tile 4");
static_assert(Tile5::BM == kTileShapes[5].bm && Tile5::BN == kTileShapes[5].bn && Tile5::NTH == kTileShapes[5].nth, "tile 5");

// Kernel of one launch variant in a per-precision table: K<TL, ST, PF, IN, TR>::fn()
// is the kernel for tile TL, ST LDS stages, persistent grid PF, interior
// launch IN (every contraction interior, hec_interior) and carried traces TR
// (grids of one workgroup per item only: nullptr for a persistent one).
template <template <class, int, bool, bool, bool> class K, class TL, int ST>
const void* hec_pick_st(bool persistent, bool interior, bool traces) {
  if (persistent) {
    if (traces) return nullptr;
    return interior ? K<TL, ST, true, true, false>::fn() : K<TL, ST, true, false, false>::fn();
  }
  if (traces) return interior ? K<TL, ST, false, true, true>::fn() : K<TL, ST, false, false, true>::fn();
  return interior ? K<TL, ST, false, true, false>::fn() : K<TL, ST, false, false, false>::fn();
}
template <template <class, int, bool, bool, bool> class K, class TL>
const void* hec_pick(int stages, bool persistent, bool interior, bool traces) {
  return stages == 2 ? hec_pick_st<K, TL, 2>(persistent, interior, traces)
                     : hec_pick_st<K, TL, 1>(persistent, interior, traces);
}
template <template <class, int, bool, bool, bool> class K>
const void* hec_table(int tile, int stages, bool persistent, bool interior, bool traces) {
  switch (tile) {
    case 0: return hec_pick<K, Tile0>(stages, persistent, interior, traces);
    case 1: return hec_pick<K, Tile1>(stages, persistent, interior, traces);
    case 2: return hec_pick<K, Tile2>(stages, persistent, interior, traces);
    case 3: return hec_pick<K, Tile3>(stages, persistent, interior, traces);
    case 4: return hec_pick<K, Tile4>(stages, persistent, interior, traces);
    case 5: return hec_pick<K, Tile5>(stages, persistent, interior, traces);
    default: return nullptr;
  }
}

}  // namespace cdag
