// HIP kernels for gfx950 (CDNA4): grouped exterior contractions on the matrix
// cores, fixed-order split-K reduction, the FP64 root trace and the FP64
// cross-diagram sum.  Tensor layout and descriptors: desc.hpp.
//
// Exterior contraction = per time slice a complex GEMM C = A B with planar
// (re, im) operands.  With real matrix-core products only, either
//   Re C = Ar Br - Ai Bi,  Im C = Ar Bi + Ai Br              (four products)
// or Gauss's form with three,
//   P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi),  Re C = P1 - P2,
//   Im C = P3 - (P1 + P2).
// Flop counts use the ZGEMM convention (8 flops per complex multiply-add)
// whichever form runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "desc.hpp"
#include "kernels.hpp"

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

// Store one 16x16 block pair (Re, Im) of accumulators with the instruction's
// row layout; rows and columns outside M x N are skipped.  NT: non-temporal
// stores, which keep a launch's outputs (read by a later wave, long after the
// caches have turned over) from displacing the operands that its other work
// items are still reading from L2.
template <typename T, typename V, bool NT>
__device__ __forceinline__ void store_block(T* C, int M, int N, int row0, int col, const V& re, const V& im,
                                           int lk, const IndexMap* map = nullptr) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int m = row0 + Mfma<T>::row(lk, v);
    if (m < M && col < N) {
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
template <typename T, class TL, int ST, bool PF, bool GEN = false>
__global__ void __launch_bounds__(TL::NTH) hec_mfma(char* __restrict__ arena, const HecDesc* __restrict__ descs,
                                                     int n_desc, int64_t n_items) {
  typedef typename Mfma<T>::V V;
  constexpr int NTH = TL::NTH, BM = TL::BM, BN = TL::BN, TM = TL::TM, TN = TL::TN;
  constexpr int BK = 16, APAD = BK + 1, BPAD = BN + 16;
  // The A tile is split into 8-element row segments ([plane][row][k / 8]); the
  // B tile into 16-byte row chunks of W elements ([plane][k][n / W]), so that
  // consecutive lanes load and store consecutive 16 bytes (coalesced loads,
  // LDS stores free of bank conflicts).
  constexpr int W = 16 / (int)sizeof(T);
  constexpr int SEGA = 2 * BM * (BK / 8), SEGB = 2 * BK * (BN / W);
  constexpr int LA = (SEGA + NTH - 1) / NTH, LB = (SEGB + NTH - 1) / NTH;
  static_assert(BN % W == 0, "B chunks must tile the row");
  __shared__ __attribute__((aligned(16))) T As[ST][2][BM][APAD];   // [stage][plane][m][k]
  __shared__ __attribute__((aligned(16))) T Bs[ST][2][BK][BPAD];   // [stage][plane][k][n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / TL::WGN, wn = wave % TL::WGN, li = lane & 15, lk = lane >> 4;

  T ra[LA][8], rb[LB][W];
  auto gload = [&](const ItemView<T>& o, int k0) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int seg = tid + q * NTH;
      if (seg < SEGA) {
        const int p = seg / (2 * BM), r = (seg % (2 * BM)) >> 1, hh = seg & 1;
        const int am = o.m0 + r, ak = k0 + 8 * hh;
        if constexpr (GEN) {
          const IndexMap& mp = *o.map;
          const T* plane = o.A + (int64_t)p * o.M * o.K;
          const int64_t row = am < o.M ? digit_offset(am, mp.dm, mp.n, mp.a_m) : 0;
#pragma unroll
          for (int i = 0; i < 8; ++i)
            ra[q][i] = (am < o.M && ak + i < o.kend) ? plane[row + digit_offset(ak + i, mp.dk, mp.n, mp.a_k)] : T(0);
        } else {
          const int av = am < o.M ? max(0, min(8, o.kend - ak)) : 0;
          load8<T>(ra[q], o.A + (int64_t)p * o.M * o.K + (int64_t)am * o.K + ak, av, o.avec);
        }
      }
    }
    const bool bvw = (o.N % W) == 0;
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int seg = tid + q * NTH;
      if (seg < SEGB) {
        const int p = seg / (BK * (BN / W)), rem = seg % (BK * (BN / W));
        const int kk = rem / (BN / W), cw = rem % (BN / W);
        const int bkk = k0 + kk, bn = o.n0 + W * cw;
        if constexpr (GEN) {
          const IndexMap& mp = *o.map;
          const T* plane = o.B + (int64_t)p * o.K * o.N;
          const int64_t row = bkk < o.kend ? digit_offset(bkk, mp.dk, mp.n, mp.b_k) : 0;
#pragma unroll
          for (int i = 0; i < W; ++i)
            rb[q][i] = (bkk < o.kend && bn + i < o.N) ? plane[row + digit_offset(bn + i, mp.dn, mp.n, mp.b_n)] : T(0);
        } else {
          const int bv = bkk < o.kend ? max(0, min(W, o.N - bn)) : 0;
          load16b<T>(rb[q], o.B + (int64_t)p * o.K * o.N + (int64_t)bkk * o.N + bn, bv, bvw);
        }
      }
    }
  };
  auto sstore = [&](int st) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int seg = tid + q * NTH;
      if (seg < SEGA) {
        const int p = seg / (2 * BM), r = (seg % (2 * BM)) >> 1, hh = seg & 1;
#pragma unroll
        for (int i = 0; i < 8; ++i) As[st][p][r][8 * hh + i] = ra[q][i];
      }
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int seg = tid + q * NTH;
      if (seg < SEGB) {
        const int p = seg / (BK * (BN / W)), rem = seg % (BK * (BN / W));
        const int kk = rem / (BN / W), cw = rem % (BN / W);
#pragma unroll
        for (int i = 0; i < W; ++i) Bs[st][p][kk][W * cw + i] = rb[q][i];
      }
    }
  };

  int64_t item = blockIdx.x;
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

    const int nk = (cur.kend - cur.kbeg + BK - 1) / BK;
    if (ST == 2) {
      sstore(0);
      __syncthreads();
    }
    for (int c = 0; c < nk; ++c) {
      const int st = ST == 2 ? (c & 1) : 0;
      if (ST == 1) {
        sstore(0);
        __syncthreads();
      }
      if (c + 1 < nk)
        gload(cur, cur.kbeg + (c + 1) * BK);
      else if (PF && has_next)
        gload(nxt, nxt.kbeg);
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
      if (ST == 2 && c + 1 < nk) sstore(st ^ 1);
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
        store_block<T, V, true>(C, M, N, cur.m0 + (wm * TM + i) * 16, cur.n0 + (wn * TN + j) * 16 + li, re, im,
                                lk, GEN ? cur.map : nullptr);
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

// Piece products kept for P pieces, smallest first: term t multiplies piece
// term_x(t) of A by piece term_y(t) of B.
template <int P> __device__ constexpr int n_terms() { return P == 2 ? 3 : 6; }
template <int P> __device__ constexpr int term_x(int t) {
  return P == 2 ? (t == 0 ? 1 : 0) : (t == 0 ? 2 : (t == 2 || t == 3) ? 1 : 0);
}
template <int P> __device__ constexpr int term_y(int t) {
  return P == 2 ? (t == 1 ? 1 : 0) : (t == 1 ? 2 : (t == 2 || t == 4) ? 1 : 0);
}

template <class TL, int ST_, bool PF, int P>
__global__ void __launch_bounds__(TL::NTH) hec_bf16(char* __restrict__ arena, const HecDesc* __restrict__ descs,
                                                     int n_desc, int64_t n_items) {
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

  float ra[LA][8], rb[LB][8][2];
  auto gload = [&](const ItemView<float>& o, int k0) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int seg = tid + q * NTH;
      if (seg < SEGA) {
        const int p = seg / (4 * BM), r = (seg % (4 * BM)) >> 2, qq = seg & 3;
        const int am = o.m0 + r, ak = k0 + 8 * qq;
        const int av = am < o.M ? max(0, min(8, o.kend - ak)) : 0;
        load8<float>(ra[q], o.A + (int64_t)p * o.M * o.K + (int64_t)am * o.K + ak, av, o.avec);
      }
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int seg = tid + q * NTH;
      if (seg < SEGB) {
        const int p = seg / ((BK / 8) * (BN / 2)), rem = seg % ((BK / 8) * (BN / 2));
        const int g = rem / (BN / 2), cp = rem % (BN / 2);
        const int bk0 = k0 + 8 * g, bn = o.n0 + 2 * cp;
        const float* src = o.B + (int64_t)p * o.K * o.N + (int64_t)bk0 * o.N + bn;
        if (bk0 + 8 <= o.kend && bn + 2 <= o.N && (o.N & 1) == 0) {
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const float2 v = *reinterpret_cast<const float2*>(src + (int64_t)i * o.N);
            rb[q][i][0] = v.x;
            rb[q][i][1] = v.y;
          }
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
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int seg = tid + q * NTH;
      if (seg < SEGA) {
        const int p = seg / (4 * BM), r = (seg % (4 * BM)) >> 2, qq = seg & 3;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          __bf16 pc[P];
          split_bf16<P>(ra[q][i], pc);
#pragma unroll
          for (int x = 0; x < P; ++x) As[st][p][x][r][8 * qq + i] = pc[x];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int seg = tid + q * NTH;
      if (seg < SEGB) {
        const int p = seg / ((BK / 8) * (BN / 2)), rem = seg % ((BK / 8) * (BN / 2));
        const int g = rem / (BN / 2), cp = rem % (BN / 2);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          v8bf pv[P];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            __bf16 pc[P];
            split_bf16<P>(rb[q][i][c], pc);
#pragma unroll
            for (int x = 0; x < P; ++x) pv[x][i] = pc[x];
          }
#pragma unroll
          for (int x = 0; x < P; ++x) *reinterpret_cast<v8bf*>(&Bs[st][p][x][2 * cp + c][8 * g]) = pv[x];
        }
      }
    }
  };

  int64_t item = blockIdx.x;
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

    const int nk = (cur.kend - cur.kbeg + BK - 1) / BK;
    if (ST == 2) {
      sstore(0);
      __syncthreads();
    }
    for (int c = 0; c < nk; ++c) {
      const int st = ST == 2 ? (c & 1) : 0;
      if (ST == 1) {
        sstore(0);
        __syncthreads();
      }
      if (c + 1 < nk)
        gload(cur, cur.kbeg + (c + 1) * BK);
      else if (PF && has_next)
        gload(nxt, nxt.kbeg);
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
      if (ST == 2 && c + 1 < nk) sstore(st ^ 1);
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
        store_block<float, v4f, false>(C, M, N, cur.m0 + (wm * TM + i) * 16, cur.n0 + (wn * TN + j) * 16 + li,
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

// C(t) = sum_ij P[i,j] Q[j,i]: one wave per (root, t), four per workgroup.
// Lane l takes the 4 x 4 blocks b = l, l + 64, ... with block row ib = b / nb
// and block column jb = b % nb (nb = ceil(N / 4)): it reads rows 4ib.. of P
// over columns 4jb.. and rows 4jb.. of Q over columns 4ib.., so every load is
// a row segment and the transpose happens in registers (no LDS, no barrier).
// Products and sums in FP64 (exact products for FP32 inputs); each lane adds
// its blocks in order and the 64 lane sums meet in a fixed butterfly, so the
// result depends only on the data and N.
template <typename T>
__global__ void __launch_bounds__(256) hca_trace(char* __restrict__ arena, const HcaDesc* __restrict__ descs,
                                                 int n_desc, int64_t n_items) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < n_items; base += (int64_t)gridDim.x * 4) {
    const int64_t item = base + wave;
    if (item >= n_items) break;
    const int di = find_desc(&descs[0].item_begin, sizeof(HcaDesc) / 4, n_desc, item);
    const HcaDesc& h = descs[di];
    const int t = (int)(item - h.item_begin), n = h.n;
    const int64_t nn = (int64_t)n * n;
    const T* P = reinterpret_cast<const T*>(arena + h.p_off) + (int64_t)t * 2 * nn;
    const T* Q = reinterpret_cast<const T*>(arena + h.q_off) + (int64_t)t * 2 * nn;
    const int nb = (n + 3) >> 2;
    double sr = 0.0, si = 0.0;
    // FP32 blocks are half the bytes, so the whole-block path keeps two of
    // them in flight per lane (the same bytes as one FP64 block).
    constexpr int BPI = sizeof(T) == 4 ? 2 : 1;
    T pr[BPI][4][4], pi[BPI][4][4], qr[BPI][4][4], qi[BPI][4][4];
    auto accumulate = [&](int u) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double xr = (double)pr[u][a][c], xi = (double)pi[u][a][c];
          const double yr = (double)qr[u][c][a], yi = (double)qi[u][c][a];
          sr += xr * yr - xi * yi;
          si += xr * yi + xi * yr;
        }
    };
    if ((n & 3) == 0) {
      // N a multiple of 4: every block is whole and every row segment is a
      // 16-byte aligned run, so the loads are plain vector loads (no masks,
      // which would otherwise be merged into element-wise loads).
      for (int b0 = lane; b0 < nb * nb; b0 += 64 * BPI) {
#pragma unroll
        for (int u = 0; u < BPI; ++u) {
          // a block past the end reloads block b0 (in bounds) and is not added
          const int b = b0 + 64 * u < nb * nb ? b0 + 64 * u : b0;
          const int i0 = 4 * (b / nb), j0 = 4 * (b % nb);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t po = (int64_t)(i0 + r) * n + j0, qo = (int64_t)(j0 + r) * n + i0;
            load4v<T>(pr[u][r], P + po);
            load4v<T>(pi[u][r], P + nn + po);
            load4v<T>(qr[u][r], Q + qo);
            load4v<T>(qi[u][r], Q + nn + qo);
          }
        }
        // Keep every load of the iteration ahead of its first use, so that
        // the wave has them all in flight at once instead of waiting between
        // groups of loads.
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < BPI; ++u)
          if (b0 + 64 * u < nb * nb) accumulate(u);
      }
    } else {
      for (int b = lane; b < nb * nb; b += 64) {
        const int i0 = 4 * (b / nb), j0 = 4 * (b % nb);
        const int vj = min(4, n - j0), vi = min(4, n - i0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t po = (int64_t)(i0 + r) * n + j0, qo = (int64_t)(j0 + r) * n + i0;
          load4<T>(pr[0][r], P + po, i0 + r < n ? vj : 0, false);
          load4<T>(pi[0][r], P + nn + po, i0 + r < n ? vj : 0, false);
          load4<T>(qr[0][r], Q + qo, j0 + r < n ? vi : 0, false);
          load4<T>(qi[0][r], Q + nn + qo, j0 + r < n ? vi : 0, false);
        }
        accumulate(0);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      sr += __shfl_xor(sr, o);
      si += __shfl_xor(si, o);
    }
    if (lane == 0) {
      double* out = reinterpret_cast<double*>(arena + h.out_off);
      out[2 * t] = sr;
      out[2 * t + 1] = si;
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
unsigned grid_for(int64_t items) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(items, kMaxGrid)); }

template <class TL, int ST, bool PF>
const void* hec_kernel(int prec) {
  if (prec == 0) return reinterpret_cast<const void*>(&hec_mfma<double, TL, ST, PF>);
  if (prec == 1) return reinterpret_cast<const void*>(&hec_mfma<float, TL, ST, PF>);
  if (prec == 2) return reinterpret_cast<const void*>(&hec_bf16<TL, ST, PF, 2>);
  return reinterpret_cast<const void*>(&hec_bf16<TL, ST, PF, 3>);
}

template <class TL, int ST>
void hec_tile(KernelCall& k, int prec, bool persistent, int64_t n_items) {
  k.fn = persistent ? hec_kernel<TL, ST, true>(prec) : hec_kernel<TL, ST, false>(prec);
  k.block = TL::NTH;
  k.grid = persistent ? persistent_grid(k.fn, TL::NTH, n_items) : grid_for(n_items);
}

template <int ST>
void hec_stages(KernelCall& k, int prec, int tile, bool persistent, int64_t n_items) {
  switch (tile) {
    case 0: hec_tile<Tile0, ST>(k, prec, persistent, n_items); break;
    case 1: hec_tile<Tile1, ST>(k, prec, persistent, n_items); break;
    case 2: hec_tile<Tile2, ST>(k, prec, persistent, n_items); break;
    case 3: hec_tile<Tile3, ST>(k, prec, persistent, n_items); break;
    case 4: hec_tile<Tile4, ST>(k, prec, persistent, n_items); break;
    default: hec_tile<Tile5, ST>(k, prec, persistent, n_items); break;
  }
}

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
hipError_t hec_call(int prec, int variant, char* arena, int64_t desc_off, int n_desc, int64_t n_items,
                    KernelCall* k) {
  if (variant == kGenVariantId) {        // contractions over any index pairs: FP64 and FP32
    if (prec > 1) return hipErrorInvalidValue;
    k->fn = prec == 0 ? reinterpret_cast<const void*>(&hec_mfma<double, Tile1, 2, false, true>)
                      : reinterpret_cast<const void*>(&hec_mfma<float, Tile1, 2, false, true>);
    k->block = Tile1::NTH;
    k->grid = grid_for(n_items);
    set_args(*k, arena, arena + desc_off, n_desc, n_items);
    return hipSuccess;
  }
  if (variant < 0 || variant >= 4 * kNumTiles || prec < 0 || prec > 3) return hipErrorInvalidValue;
  const int tile = variant % kNumTiles;
  const bool persistent = (variant / kNumTiles) % 2 == 0;
  if (variant / (2 * kNumTiles) == 0)
    hec_stages<2>(*k, prec, tile, persistent, n_items);
  else
    hec_stages<1>(*k, prec, tile, persistent, n_items);
  set_args(*k, arena, arena + desc_off, n_desc, n_items);
  return hipSuccess;
}

static_assert(Tile0::BM == kTileShapes[0].bm && Tile0::BN == kTileShapes[0].bn && Tile0::NTH == kTileShapes[0].nth, "tile 0");
static_assert(Tile1::BM == kTileShapes[1].bm && Tile1::BN == kTileShapes[1].bn && Tile1::NTH == kTileShapes[1].nth, "tile 1");
static_assert(Tile2::BM == kTileShapes[2].bm && Tile2::BN == kTileShapes[2].bn && Tile2::NTH == kTileShapes[2].nth, "tile 2");
static_assert(Tile3::BM == kTileShapes[3].bm && Tile3::BN == kTileShapes[3].bn && Tile3::NTH == kTileShapes[3].nth, "tile 3");
static_assert(Tile4::BM == kTileShapes[4].bm && Tile4::BN == kTileShapes[4].bn && Tile4::NTH == kTileShapes[4].nth, "tile 4");
static_assert(Tile5::BM == kTileShapes[5].bm && Tile5::BN == kTileShapes[5].bn && Tile5::NTH == kTileShapes[5].nth, "tile 5");

hipError_t reduce_call(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, KernelCall* k) {
  k->fn = prec == 0 ? reinterpret_cast<const void*>(&splitk_reduce<double>)
                    : reinterpret_cast<const void*>(&splitk_reduce<float>);
  k->grid = grid_for(n_items);
  k->block = 256;
  set_args(*k, arena, arena + desc_off, n_desc, n_items);
  return hipSuccess;
}

hipError_t hca_call(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, KernelCall* k) {
  k->fn = prec == 0 ? reinterpret_cast<const void*>(&hca_trace<double>)
                    : reinterpret_cast<const void*>(&hca_trace<float>);
  k->grid = grid_for((n_items + 3) / 4);
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

hipError_t launch_hec(int prec, int variant, char* arena, int64_t desc_off, int n_desc, int64_t n_items,
                      hipStream_t s) {
  KernelCall k;
  hipError_t e = hec_call(prec, variant, arena, desc_off, n_desc, n_items, &k);
  return e != hipSuccess ? e : launch(k, s);
}

hipError_t launch_reduce(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, hipStream_t s) {
  KernelCall k;
  reduce_call(prec, arena, desc_off, n_desc, n_items, &k);
  return launch(k, s);
}

hipError_t launch_hca(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, hipStream_t s) {
  KernelCall k;
  hca_call(prec, arena, desc_off, n_desc, n_items, &k);
  return launch(k, s);
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
  xsum_call(arena, desc_off, entries_off, n_desc, &k);
  return launch(k, s);
}

}  // namespace cdag
