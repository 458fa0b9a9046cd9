// HIP kernels for gfx950 (CDNA4): grouped exterior contractions on the matrix
// cores, fixed-order split-K reduction, the FP64 root trace and the FP64
// cross-diagram sum.  Tensor layout and descriptors: desc.hpp.
//
// Exterior contraction = per time slice a complex GEMM C = A B with planar
// (re, im) operands.  With real matrix-core products only:
//   Re C = Ar Br - Ai Bi,  Im C = Ar Bi + Ai Br
// i.e. four real products per complex multiply-add (the 8-flop ZGEMM count).
#include <hip/hip_runtime.h>

#include "desc.hpp"
#include "kernels.hpp"

namespace cdag {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v8s __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, NTH = 256;

__device__ __forceinline__ int find_desc(const int32_t* first, int stride_words, int n, int64_t item) {
  // largest i with first[i * stride] <= item (first[0] == 0)
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if ((int64_t)first[(int64_t)mid * stride_words] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
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

constexpr int BK = 16;
constexpr int APAD = BK + 1;    // A tile row stride in LDS (elements)
constexpr int BPAD = BN + 16;   // B tile row stride in LDS (elements)

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

template <typename T>
__global__ void __launch_bounds__(NTH) hec_mfma(char* __restrict__ arena, const HecDesc* __restrict__ descs,
                                                 int n_desc, int64_t n_items) {
  typedef typename Mfma<T>::V V;
  __shared__ T As[2][2][BM][APAD];   // [stage][plane][m][k]
  __shared__ T Bs[2][2][BK][BPAD];   // [stage][plane][k][n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, li = lane & 15, lk = lane >> 4;
  // load roles
  const int ap = tid >> 7, ar = (tid >> 1) & 63, ah = tid & 1;
  const int bp = tid >> 7, bk = (tid >> 3) & 15, bs = tid & 7;

  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int di = find_desc(&descs[0].tile_begin, sizeof(HecDesc) / 4, n_desc, item);
    const HecDesc& h = descs[di];
    int64_t local = item - h.tile_begin;
    const int sp = (int)(local % h.splits);
    local /= h.splits;
    const int tn = (int)(local % h.tiles_n);
    local /= h.tiles_n;
    const int tm = (int)(local % h.tiles_m);
    const int t = (int)(local / h.tiles_m);
    const int M = h.M, N = h.N, K = h.K;
    const int m0 = tm * BM, n0 = tn * BN;
    const int kbeg = sp * h.k_split, kend = min(K, kbeg + h.k_split);
    const T* A = reinterpret_cast<const T*>(arena + h.a_off) + (int64_t)t * 2 * M * K;
    const T* B = reinterpret_cast<const T*>(arena + h.b_off) + (int64_t)t * 2 * K * N;
    const bool avec = (K & 7) == 0, bvec = (N & 7) == 0;

    V cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) { cr[i][j] = V{0, 0, 0, 0}; ci[i][j] = V{0, 0, 0, 0}; }

    T ra[8], rb[8];
    auto gload = [&](int k0) {
      const int am = m0 + ar, ak = k0 + 8 * ah;
      const int av = am < M ? max(0, min(8, kend - ak)) : 0;
      load8<T>(ra, A + (int64_t)ap * M * K + (int64_t)am * K + ak, av, avec);
      const int bkk = k0 + bk, bn = n0 + 8 * bs;
      const int bv = bkk < kend ? max(0, min(8, N - bn)) : 0;
      load8<T>(rb, B + (int64_t)bp * K * N + (int64_t)bkk * N + bn, bv, bvec);
    };
    auto sstore = [&](int st) {
#pragma unroll
      for (int i = 0; i < 8; ++i) As[st][ap][ar][8 * ah + i] = ra[i];
#pragma unroll
      for (int i = 0; i < 8; ++i) Bs[st][bp][bk][8 * bs + i] = rb[i];
    };

    const int nk = (kend - kbeg + BK - 1) / BK;
    gload(kbeg);
    sstore(0);
    __syncthreads();
    for (int c = 0; c < nk; ++c) {
      const int st = c & 1;
      if (c + 1 < nk) gload(kbeg + (c + 1) * BK);
#pragma unroll
      for (int k4 = 0; k4 < BK / 4; ++k4) {
        const int kk = 4 * k4 + lk;
        T a_r[2], a_i[2], b_r[2], b_i[2], b_n[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a_r[i] = As[st][0][wm * 32 + i * 16 + li][kk];
          a_i[i] = As[st][1][wm * 32 + i * 16 + li][kk];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          b_r[j] = Bs[st][0][kk][wn * 32 + j * 16 + li];
          b_i[j] = Bs[st][1][kk][wn * 32 + j * 16 + li];
          b_n[j] = -b_i[j];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            cr[i][j] = Mfma<T>::mma(a_r[i], b_r[j], cr[i][j]);
            cr[i][j] = Mfma<T>::mma(a_i[i], b_n[j], cr[i][j]);
            ci[i][j] = Mfma<T>::mma(a_r[i], b_i[j], ci[i][j]);
            ci[i][j] = Mfma<T>::mma(a_i[i], b_r[j], ci[i][j]);
          }
      }
      if (c + 1 < nk) sstore(st ^ 1);
      __syncthreads();
    }

    // epilogue: lane holds rows Mfma<T>::row(lk, v), column li of each 16x16 sub-tile
    T* C;
    if (h.splits > 1)
      C = reinterpret_cast<T*>(arena + h.ws_off) + ((int64_t)sp * h.nt + t) * 2 * M * N;
    else
      C = reinterpret_cast<T*>(arena + h.c_off) + (int64_t)t * 2 * M * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = n0 + wn * 32 + j * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = m0 + wm * 32 + i * 16 + Mfma<T>::row(lk, v);
          if (m < M && n < N) {
            C[(int64_t)m * N + n] = cr[i][j][v];
            C[(int64_t)M * N + (int64_t)m * N + n] = ci[i][j][v];
          }
        }
      }
  }
}

// ------------------------------------------------------------------ split BF16
// Each FP32 operand x is split as hi = bf16(x), lo = bf16(x - hi); a real
// product is approximated by hi*hi' + hi*lo' + lo*hi' (the lo*lo' term is
// dropped), accumulated in FP32 on the bf16 matrix cores.
constexpr int BK3 = 32;
constexpr int A3PAD = BK3 + 8;   // bf16 elements per A row in LDS (16-byte aligned rows)
constexpr int B3PAD = BK3 + 8;   // B is stored transposed: [n][k]

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

__global__ void __launch_bounds__(NTH) hec_bf16x3(char* __restrict__ arena, const HecDesc* __restrict__ descs,
                                                   int n_desc, int64_t n_items) {
  // [stage][plane][hi/lo][row][k]: A rows are m, B rows are n (transposed)
  __shared__ __attribute__((aligned(16))) __bf16 As[2][2][2][BM][A3PAD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][2][2][BN][B3PAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, li = lane & 15, lk = lane >> 4;
  // A: 64 rows x 32 k x 2 planes = 4096 floats, 16 per thread: plane, row, half
  const int ap = tid >> 7, ar = (tid >> 1) & 63, ah = tid & 1;
  // B: 32 k x 64 n x 2 planes: plane, k row, 16-column segment
  const int bp = tid >> 7, bk = (tid >> 2) & 31, bs = tid & 3;

  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int di = find_desc(&descs[0].tile_begin, sizeof(HecDesc) / 4, n_desc, item);
    const HecDesc& h = descs[di];
    int64_t local = item - h.tile_begin;
    const int sp = (int)(local % h.splits);
    local /= h.splits;
    const int tn = (int)(local % h.tiles_n);
    local /= h.tiles_n;
    const int tm = (int)(local % h.tiles_m);
    const int t = (int)(local / h.tiles_m);
    const int M = h.M, N = h.N, K = h.K;
    const int m0 = tm * BM, n0 = tn * BN;
    const int kbeg = sp * h.k_split, kend = min(K, kbeg + h.k_split);
    const float* A = reinterpret_cast<const float*>(arena + h.a_off) + (int64_t)t * 2 * M * K;
    const float* B = reinterpret_cast<const float*>(arena + h.b_off) + (int64_t)t * 2 * K * N;
    const bool avec = (K & 7) == 0, bvec = (N & 7) == 0;

    v4f cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) { cr[i][j] = v4f{0, 0, 0, 0}; ci[i][j] = v4f{0, 0, 0, 0}; }

    float ra[16], rb[16];
    auto gload = [&](int k0) {
      const int am = m0 + ar;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int ak = k0 + 16 * ah + 8 * q;
        const int av = am < M ? max(0, min(8, kend - ak)) : 0;
        float tmp[8];
        load8<float>(tmp, A + (int64_t)ap * M * K + (int64_t)am * K + ak, av, avec);
#pragma unroll
        for (int i = 0; i < 8; ++i) ra[8 * q + i] = tmp[i];
      }
      const int bkk = k0 + bk;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int bn = n0 + 16 * bs + 8 * q;
        const int bv = bkk < kend ? max(0, min(8, N - bn)) : 0;
        float tmp[8];
        load8<float>(tmp, B + (int64_t)bp * K * N + (int64_t)bkk * N + bn, bv, bvec);
#pragma unroll
        for (int i = 0; i < 8; ++i) rb[8 * q + i] = tmp[i];
      }
    };
    auto sstore = [&](int st) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        __bf16 hi, lo;
        split_bf16(ra[i], hi, lo);
        As[st][ap][0][ar][16 * ah + i] = hi;
        As[st][ap][1][ar][16 * ah + i] = lo;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        __bf16 hi, lo;
        split_bf16(rb[i], hi, lo);
        Bs[st][bp][0][16 * bs + i][bk] = hi;
        Bs[st][bp][1][16 * bs + i][bk] = lo;
      }
    };

    const int nk = (kend - kbeg + BK3 - 1) / BK3;
    gload(kbeg);
    sstore(0);
    __syncthreads();
    for (int c = 0; c < nk; ++c) {
      const int st = c & 1;
      if (c + 1 < nk) gload(kbeg + (c + 1) * BK3);
      // one 16x16x32 step: lane holds k = 8*lk .. 8*lk+7 of row li (A) / column li (B)
      v8bf a[2][2][2], b[2][2][2], bn_hi[2], bn_lo[2];   // [sub][plane][hi/lo]
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int s = 0; s < 2; ++s)
            a[i][p][s] = *reinterpret_cast<const v8bf*>(&As[st][p][s][wm * 32 + i * 16 + li][8 * lk]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int s = 0; s < 2; ++s)
            b[j][p][s] = *reinterpret_cast<const v8bf*>(&Bs[st][p][s][wn * 32 + j * 16 + li][8 * lk]);
        // -Bi: flip the bf16 sign bits
        v8s hs = *reinterpret_cast<v8s*>(&b[j][1][0]) ^ (short)0x8000;
        v8s ls = *reinterpret_cast<v8s*>(&b[j][1][1]) ^ (short)0x8000;
        bn_hi[j] = *reinterpret_cast<v8bf*>(&hs);
        bn_lo[j] = *reinterpret_cast<v8bf*>(&ls);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          // Re += Ar Br - Ai Bi ; Im += Ar Bi + Ai Br, each with hi*hi + hi*lo + lo*hi
#define MM(acc, x, y) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc, 0, 0, 0)
          MM(cr[i][j], a[i][0][1], b[j][0][0]);
          MM(cr[i][j], a[i][0][0], b[j][0][1]);
          MM(cr[i][j], a[i][0][0], b[j][0][0]);
          MM(cr[i][j], a[i][1][1], bn_hi[j]);
          MM(cr[i][j], a[i][1][0], bn_lo[j]);
          MM(cr[i][j], a[i][1][0], bn_hi[j]);
          MM(ci[i][j], a[i][0][1], b[j][1][0]);
          MM(ci[i][j], a[i][0][0], b[j][1][1]);
          MM(ci[i][j], a[i][0][0], b[j][1][0]);
          MM(ci[i][j], a[i][1][1], b[j][0][0]);
          MM(ci[i][j], a[i][1][0], b[j][0][1]);
          MM(ci[i][j], a[i][1][0], b[j][0][0]);
#undef MM
        }
      if (c + 1 < nk) sstore(st ^ 1);
      __syncthreads();
    }

    float* C;
    if (h.splits > 1)
      C = reinterpret_cast<float*>(arena + h.ws_off) + ((int64_t)sp * h.nt + t) * 2 * M * N;
    else
      C = reinterpret_cast<float*>(arena + h.c_off) + (int64_t)t * 2 * M * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = n0 + wn * 32 + j * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = m0 + wm * 32 + i * 16 + 4 * lk + v;
          if (m < M && n < N) {
            C[(int64_t)m * N + n] = cr[i][j][v];
            C[(int64_t)M * N + (int64_t)m * N + n] = ci[i][j][v];
          }
        }
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
template <typename T>
__global__ void __launch_bounds__(256) hca_trace(char* __restrict__ arena, const HcaDesc* __restrict__ descs,
                                                 int n_desc, int64_t n_items) {
  __shared__ T Qs[2][32][33];
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int di = find_desc(&descs[0].item_begin, sizeof(HcaDesc) / 4, n_desc, item);
    const HcaDesc& h = descs[di];
    const int t = (int)(item - h.item_begin), n = h.n;
    const int64_t nn = (int64_t)n * n;
    const T* P = reinterpret_cast<const T*>(arena + h.p_off) + (int64_t)t * 2 * nn;
    const T* Q = reinterpret_cast<const T*>(arena + h.q_off) + (int64_t)t * 2 * nn;
    double sr = 0.0, si = 0.0;
    for (int bi = 0; bi < n; bi += 32)
      for (int bj = 0; bj < n; bj += 32) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {           // Qs[p][r][c] = Q[p][bj + r][bi + c]
          const int idx = tid + 256 * q, r = idx >> 5, c = idx & 31;
          const bool ok = bj + r < n && bi + c < n;
          const int64_t o = (int64_t)(bj + r) * n + bi + c;
          Qs[0][r][c] = ok ? Q[o] : T(0);
          Qs[1][r][c] = ok ? Q[nn + o] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {           // P[bi + r][bj + c] * Q[bj + c][bi + r]
          const int idx = tid + 256 * q, r = idx >> 5, c = idx & 31;
          if (bi + r < n && bj + c < n) {
            const int64_t o = (int64_t)(bi + r) * n + bj + c;
            const double pr = (double)P[o], pi = (double)P[nn + o];
            const double qr = (double)Qs[0][c][r], qi = (double)Qs[1][c][r];
            sr += pr * qr - pi * qi;
            si += pr * qi + pi * qr;
          }
        }
      }
    red[0][tid] = sr;
    red[1][tid] = si;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {         // fixed-order tree
      if (tid < w) {
        red[0][tid] += red[0][tid + w];
        red[1][tid] += red[1][tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      double* out = reinterpret_cast<double*>(arena + h.out_off);
      out[2 * t] = red[0][0];
      out[2 * t + 1] = red[1][0];
    }
    __syncthreads();
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

// ------------------------------------------------------------------ launchers
namespace {
constexpr int64_t kMaxGrid = 1 << 20;
unsigned grid_for(int64_t items) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(items, kMaxGrid)); }
}  // namespace

hipError_t launch_hec(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, hipStream_t s) {
  const HecDesc* d = reinterpret_cast<const HecDesc*>(arena + desc_off);
  if (prec == 0)
    hipLaunchKernelGGL(hec_mfma<double>, dim3(grid_for(n_items)), dim3(NTH), 0, s, arena, d, n_desc, n_items);
  else if (prec == 1)
    hipLaunchKernelGGL(hec_mfma<float>, dim3(grid_for(n_items)), dim3(NTH), 0, s, arena, d, n_desc, n_items);
  else
    hipLaunchKernelGGL(hec_bf16x3, dim3(grid_for(n_items)), dim3(NTH), 0, s, arena, d, n_desc, n_items);
  return hipGetLastError();
}

hipError_t launch_reduce(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, hipStream_t s) {
  const RedDesc* d = reinterpret_cast<const RedDesc*>(arena + desc_off);
  if (prec == 0)
    hipLaunchKernelGGL(splitk_reduce<double>, dim3(grid_for(n_items)), dim3(256), 0, s, arena, d, n_desc, n_items);
  else
    hipLaunchKernelGGL(splitk_reduce<float>, dim3(grid_for(n_items)), dim3(256), 0, s, arena, d, n_desc, n_items);
  return hipGetLastError();
}

hipError_t launch_hca(int prec, char* arena, int64_t desc_off, int n_desc, int64_t n_items, hipStream_t s) {
  const HcaDesc* d = reinterpret_cast<const HcaDesc*>(arena + desc_off);
  if (prec == 0)
    hipLaunchKernelGGL(hca_trace<double>, dim3(grid_for(n_items)), dim3(256), 0, s, arena, d, n_desc, n_items);
  else
    hipLaunchKernelGGL(hca_trace<float>, dim3(grid_for(n_items)), dim3(256), 0, s, arena, d, n_desc, n_items);
  return hipGetLastError();
}

hipError_t launch_xsum(char* arena, int64_t desc_off, int64_t entries_off, int n_desc, hipStream_t s) {
  const XsumDesc* d = reinterpret_cast<const XsumDesc*>(arena + desc_off);
  const XsumEntry* e = reinterpret_cast<const XsumEntry*>(arena + entries_off);
  hipLaunchKernelGGL(xsum_kernel, dim3(grid_for(n_desc)), dim3(256), 0, s, arena, d, e, n_desc);
  return hipGetLastError();
}

}  // namespace cdag
