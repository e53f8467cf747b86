// The general batched action: d-dimensional operands for any d >= 1
// (Section 2.1 generalises the summation to n-D arrays), rectangular factors
// op(F_k) of size m_k x n_k with op in {N, T, C} and complex entries (Section
// 2.2), alpha and beta, and factors that may change along the batch (the
// case Section 6 names).  Real FP32 / FP64 and complex (C: FP32 pairs, Z:
// FP64 pairs).
//
// The action is d mode products, fastest index first, each one pass over
// HBM through the caller's workspace (ping-pong arrays), the way the paper
// builds its 3-D kernel from a 2-D stage and a batched GEMM through a work
// array (Section 4).  The fused 2-D / 3-D kernels keep every stage in
// registers; this path instead covers any size and any d, and its one kernel
// is the mode product
//
//     Out[u, i, v] = sum_a op(F)(i, a) * In[u, a, v],  u < pre, i < m, a < n, v < post
//
// on the 16x16x4 matrix cores: a tile is 16 output rows i by 16 "columns"
// c = u * post + v, contracted in steps of four a.  When post > 1 the data
// columns are the MFMA's B operand (lanes of a row group read 16 consecutive
// v), when post == 1 (the fastest index) the data is the A operand (each lane
// reads consecutive a of one u).  Complex products take four real MFMAs per
// step: re += Fr xr - Fi xi, im += Fr xi + Fi xr.  With factors per operand
// a tile's columns never straddle two operands.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kron.h"
#include "kron_launch.hpp"

namespace kron {
namespace {

constexpr int kNdMaxDim = 8;
// 16-column sub-tiles per tile of kron_mode_kernel: four keep 4 KiB of loads
// in flight per wavefront for real data (the pass is latency-bound with one:
// 4-D n = 16 2.17 -> 1.97 ms, 2-D n = 32 1.85 -> 1.23 ms); complex data,
// twice the registers per column, measured 3 % slower with four.
template <bool kC>
constexpr int nd_sub_tiles() {
  return kC ? 1 : 4;
}

// Offset of column c of a pass: its digits, fastest first, each times its
// stride (digit j = (c / prod_{i<j} mod_i) % mod_j; the last digit takes the
// rest), plus `along` times the contracted (input) or produced (output)
// index.  Dense intermediates have two digits (v < post, then u); the first
// pass may read and the last pass may write strided storage (up to three
// digits: the slower indices, then the operand).
struct NdIndex {
  int nlev;           // 1..3
  int64_t mod[3];     // radix of digits 0 .. nlev - 2
  int64_t stride[3];  // element stride of each digit
  int64_t along;      // element stride of the contracted / produced index
};

__device__ __forceinline__ int64_t nd_offset(const NdIndex& ix, int64_t c) {
  int64_t off = 0;
  for (int j = 0; j < ix.nlev - 1; ++j) {
    off += (c % ix.mod[j]) * ix.stride[j];
    c /= ix.mod[j];
  }
  return off + c * ix.stride[ix.nlev - 1];
}

// Digits of a column, kept up to date by additions as a wavefront walks its
// tiles (a 64-bit division per tile would cost more than the tile's MFMAs).
struct Digits {
  int64_t d[3];
  __device__ __forceinline__ void set(const NdIndex& ix, int64_t c) {
    for (int j = 0; j < ix.nlev - 1; ++j) {
      d[j] = c % ix.mod[j];
      c /= ix.mod[j];
    }
    d[ix.nlev - 1] = c;
  }
  // column += k (k >= 0), carrying into the slower digits
  __device__ __forceinline__ void add(const NdIndex& ix, int64_t k) {
    d[0] += k;
    if (ix.nlev == 1) return;
    while (d[0] >= ix.mod[0]) {
      d[0] -= ix.mod[0];
      ++d[1];
    }
    if (ix.nlev == 2) return;
    while (d[1] >= ix.mod[1]) {
      d[1] -= ix.mod[1];
      ++d[2];
    }
  }
  __device__ __forceinline__ int64_t offset(const NdIndex& ix) const {
    int64_t off = d[0] * ix.stride[0];
    for (int j = 1; j < ix.nlev; ++j) off += d[j] * ix.stride[j];
    return off;
  }
};

// A wavefront's tiles are one contiguous range; within it the tile
// coordinates (row chunk fastest, then column chunk, then group) advance by
// additions.
struct TileWalk {
  int64_t t, t1, grp, ch;
  int ic;
  __device__ __forceinline__ TileWalk(int64_t ntiles, int rows, int64_t chunks, int64_t wave, int64_t nwaves) {
    const int64_t per = (ntiles + nwaves - 1) / nwaves;
    t = wave * per;
    t1 = t + per < ntiles ? t + per : ntiles;
    ic = 0;
    grp = ch = 0;
    if (t < t1) {
      ic = (int)(t % rows);
      const int64_t ct = t / rows;
      grp = ct / chunks;
      ch = ct % chunks;
    }
  }
  // next tile; returns 0 (same columns), 1 (next chunk of the group) or 2 (next group)
  __device__ __forceinline__ int next(int rows, int64_t chunks) {
    ++t;
    if (++ic < rows) return 0;
    ic = 0;
    if (++ch < chunks) return 1;
    ch = 0;
    ++grp;
    return 2;
  }
};

// One mode product.  Element counts and offsets are in elements (a complex
// element is one unit; its two parts follow each other in memory).
struct NdPass {
  const void* X;
  void* Y;
  const void* F;
  int64_t ldfp;   // factor stride between operands (0: shared)
  int ld;         // leading dimension of the stored factor
  int op;         // 0 N, 1 T, 2 C
  int m, n;       // output / input extent of the contracted index
  int conjx;      // conjugate the input elements (op(X) = X^* of the 2-D interface)
  NdIndex in, out;
  int64_t cols;   // columns per group (a group shares one factor)
  int64_t cols_groups;  // number of groups
  int64_t chunks; // 16-column chunks per group
  int rows;       // 16-row chunks of the output index
};

template <typename T>
struct NdAcc;
template <>
struct NdAcc<float> {
  using type = f32x4;
  __device__ static f32x4 mma(float a, float b, f32x4 c) { return mfma_f32(a, b, c); }
  __device__ static constexpr int drow(int g, int r) { return 4 * g + r; }
};
template <>
struct NdAcc<double> {
  using type = f64x4;
  __device__ static f64x4 mma(double a, double b, f64x4 c) { return mfma_f64(a, b, c); }
  __device__ static constexpr int drow(int g, int r) { return g + 4 * r; }
};

// Input reads are non-temporal unless `keep`: a pass whose output index has
// more than 16 rows reads each input column once per 16-row block, back to
// back in the same wavefront, and the later reads then hit the L2 cache.
template <typename T>
__device__ __forceinline__ T ld1(const T* p, bool keep) {
  return keep ? *in_global(p) : __builtin_nontemporal_load(in_global(p));
}

template <typename T, bool kC>
__device__ __forceinline__ void ld_elem(const T* p, int64_t e, T& re, T& im, bool keep = false) {
  if constexpr (kC) {
    re = ld1(p + 2 * e, keep);
    im = ld1(p + 2 * e + 1, keep);
  } else {
    re = ld1(p + e, keep);
    im = T(0);
  }
}

template <typename T, bool kC>
__device__ __forceinline__ void st_elem(T* p, int64_t e, T re, T im) {
  if constexpr (kC) {
    __builtin_nontemporal_store(re, in_global(p) + 2 * e);
    __builtin_nontemporal_store(im, in_global(p) + 2 * e + 1);
  } else {
    __builtin_nontemporal_store(re, in_global(p) + e);
  }
}

// NS consecutive scalars at p (p aligned to min(16, NS * sizeof(T)) bytes),
// in 16-byte (or, below 16 bytes, NS-scalar) vector accesses, non-temporal
// unless `keep` (as ld_elem).
template <typename T, int NS>
__device__ __forceinline__ void ldv(const T* p, T (&o)[NS], bool keep = false) {
  constexpr int W = (NS * sizeof(T) >= 16) ? 16 / (int)sizeof(T) : NS;
  typedef T V __attribute__((ext_vector_type(W)));
#pragma unroll
  for (int q = 0; q < NS / W; ++q) {
    const V v = ld1(reinterpret_cast<const V*>(p) + q, keep);
#pragma unroll
    for (int e = 0; e < W; ++e) o[q * W + e] = v[e];
  }
}

template <typename T, int NS>
__device__ __forceinline__ void stv(T* p, const T (&o)[NS]) {
  constexpr int W = (NS * sizeof(T) >= 16) ? 16 / (int)sizeof(T) : NS;
  typedef T V __attribute__((ext_vector_type(W)));
#pragma unroll
  for (int q = 0; q < NS / W; ++q) {
    V v;
#pragma unroll
    for (int e = 0; e < W; ++e) v[e] = o[q * W + e];
    __builtin_nontemporal_store(v, in_global(reinterpret_cast<V*>(p)) + q);
  }
}

// op(F)(i, a) of the stored factor (zero outside m x n); complex parts in
// fr, fi with the conjugation of op 'C' applied.
template <typename T, bool kC>
__device__ __forceinline__ void factor_entry(const NdPass& P, const T* F, int i, int a, T& fr, T& fi) {
  fr = T(0);
  fi = T(0);
  if (i < P.m && a < P.n) {
    const int64_t e = P.op == 0 ? i + (int64_t)P.ld * a : a + (int64_t)P.ld * i;
    if constexpr (kC) {
      fr = in_global(F)[2 * e];
      fi = in_global(F)[2 * e + 1];
      if (P.op == 2) fi = -fi;
    } else {
      fr = in_global(F)[e];
    }
  }
}

// Dense passes whose faster extent `post` is a multiple of kW: a tile is 16
// output rows by 16 * kW consecutive columns, and lane L owns the kW columns
// cb + kW * L .. + kW - 1, which lie in one u and are consecutive in memory,
// so they are loaded and stored as vectors.  Each of them is one MFMA's B
// operand (the factor is shared), so the tile is kW (complex: 4 kW) MFMAs
// per contraction step.  X and Y are 16-byte aligned.
template <typename T, bool kC, int kW, bool kBeta>
__global__ __launch_bounds__(kBlock) void kron_mode_wide_kernel(NdPass P, int64_t ntiles, T ar, T ai, T br, T bi) {
  using A = NdAcc<T>;
  using acc_t = typename A::type;
  constexpr int kS = kC ? 2 : 1;   // scalars per element
  constexpr int NS = kW * kS;      // scalars per lane and row
  const T* __restrict__ X = static_cast<const T*>(P.X);
  T* __restrict__ Y = static_cast<T*>(P.Y);
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const int nk = (P.n + 15) / 16;
  const bool keep = P.rows > 1;
  const int64_t post = P.in.mod[0];
  TileWalk w(ntiles, P.rows, P.chunks, wave, nwaves);
  Digits dc;  // digits (v, u) of the tile's first column
  if (w.t < w.t1) dc.set(P.in, w.grp * P.cols + w.ch * (16 * kW));
  for (; w.t < w.t1;) {
    const int ic = w.ic;
    const int64_t grp = w.grp;
    const int64_t cl = grp * P.cols + w.ch * (16 * kW) + kW * L;  // this lane's first column
    const bool colok = cl < (grp + 1) * P.cols;
    const T* F = static_cast<const T*>(P.F) + grp * P.ldfp * kS;
    // this lane's (u, v): the tile's digits plus kW * L columns
    int64_t u = dc.d[1], v0 = dc.d[0] + kW * L;
    if (v0 >= post) {
      const uint32_t q = (uint32_t)((uint64_t)v0 / (uint64_t)post);
      u += q;
      v0 -= (int64_t)q * post;
    }
    const int64_t xb = u * P.n * post + v0, yb = u * P.m * post + v0;
    acc_t dr[kW], di[kW];
#pragma unroll
    for (int j = 0; j < kW; ++j) {
      dr[j] = acc_t{0, 0, 0, 0};
      di[j] = acc_t{0, 0, 0, 0};
    }
    for (int kc = 0; kc < nk; ++kc) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        // real data: step s contracts indices 4s .. 4s + 3 of the block, one
        // per lane group, so a load instruction covers four consecutive rows
        // (complex data keeps rows 4g + s, measured faster for it)
        const int a = kC ? 16 * kc + 4 * g + s : 16 * kc + 4 * s + g;
        T x[NS];
        if (colok && a < P.n) {
          ldv<T, NS>(X + (xb + (int64_t)a * post) * kS, x, keep);
        } else {
#pragma unroll
          for (int q = 0; q < NS; ++q) x[q] = T(0);
        }
        T fr, fi;
        factor_entry<T, kC>(P, F, 16 * ic + L, a, fr, fi);
#pragma unroll
        for (int j = 0; j < kW; ++j) {
          if constexpr (kC) {
            dr[j] = A::mma(fr, x[2 * j], dr[j]);
            dr[j] = A::mma(-fi, x[2 * j + 1], dr[j]);
            di[j] = A::mma(fr, x[2 * j + 1], di[j]);
            di[j] = A::mma(fi, x[2 * j], di[j]);
          } else {
            dr[j] = A::mma(fr, x[j], dr[j]);
          }
        }
      }
    }
    // Real results: register r of lane group g becomes row 4r + g, so a
    // store instruction (one r) writes four consecutive rows.  FP64
    // accumulators already hold rows g + 4r; FP32 ones (rows 4g + r) trade
    // lane groups and registers first.  Complex results keep rows drow(g, r).
    if constexpr (sizeof(T) == 4 && !kC) {
#pragma unroll
      for (int j = 0; j < kW; ++j) transpose_groups_regs(dr[j]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = kC ? 16 * ic + A::drow(g, r) : 16 * ic + 4 * r + g;
      if (i >= P.m || !colok) continue;
      T* yp = Y + (yb + (int64_t)i * post) * kS;
      T o[NS];
#pragma unroll
      for (int j = 0; j < kW; ++j) {
        const T re = dr[j][r], im = kC ? di[j][r] : T(0);
        o[j * kS] = ar * re - ai * im;
        if constexpr (kC) o[j * kS + 1] = ar * im + ai * re;
      }
      if constexpr (kBeta) {
        T old[NS];
        ldv<T, NS>(yp, old);
#pragma unroll
        for (int j = 0; j < kW; ++j) {
          if constexpr (kC) {
            const T orr = old[2 * j], oi = old[2 * j + 1];
            o[2 * j] += br * orr - bi * oi;
            o[2 * j + 1] += br * oi + bi * orr;
          } else {
            o[j] += br * old[j];
          }
        }
      }
      stv<T, NS>(yp, o);
    }
    const int step = w.next(P.rows, P.chunks);
    if (step == 1) dc.add(P.in, 16 * kW);
    else if (step == 2 && w.t < w.t1) dc.set(P.in, w.grp * P.cols);
  }
}

// 4 x 4 transpose inside each quad of lanes (DPP quad permutations): lane
// 4q + j, register r ends up with what lane 4q + r held in register j.
template <int kCtrl>
__device__ __forceinline__ float dpp_move(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kCtrl, 0xF, 0xF, false));
}
template <int kCtrl>
__device__ __forceinline__ double dpp_move(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, kCtrl, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ void quad_transpose(T (&v)[4]) {
  constexpr int kXor1 = 0xB1;  // quad_perm(1, 0, 3, 2)
  constexpr int kXor2 = 0x4E;  // quad_perm(2, 3, 0, 1)
  const int j = threadIdx.x & 3;
#pragma unroll
  for (int base = 0; base < 4; base += 2) {
    const T recv = dpp_move<kXor1>((j & 1) ? v[base] : v[base + 1]);
    if (j & 1) v[base] = recv;
    else v[base + 1] = recv;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const T recv = dpp_move<kXor2>((j & 2) ? v[r] : v[r + 2]);
    if (j & 2) v[r] = recv;
    else v[r + 2] = recv;
  }
}

// kDataA: the data is the MFMA's A operand (post == 1); otherwise B.
// kBeta: Out <- alpha * product + beta * Out (the last pass); otherwise
// Out <- alpha * product.
// kVecA (kDataA, dense input, n a multiple of 4, X 16-byte aligned): the
// four contraction indices 4g .. 4g + 3 of a lane are consecutive in memory
// and come in as one vector.
template <typename T, bool kC, bool kDataA, bool kBeta, bool kVecA>
__global__ __launch_bounds__(kBlock) void kron_mode_kernel(NdPass P, int64_t ntiles, T ar, T ai, T br, T bi) {
  static_assert(!kVecA || kDataA, "vector loads of the A operand");
  using A = NdAcc<T>;
  using acc_t = typename A::type;
  constexpr int kS = kC ? 2 : 1;
  constexpr int kU = nd_sub_tiles<kC>();  // 16-column sub-tiles per tile (more loads in flight per wavefront)
  constexpr int kCols = 16 * kU;
  const T* __restrict__ X = static_cast<const T*>(P.X);
  T* __restrict__ Y = static_cast<T*>(P.Y);
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const int nk = (P.n + 15) / 16;
  const bool keep = P.rows > 1;
  // vector stores of the output (kDataA): the produced index is the fastest,
  // m and the column stride are multiples of 4, Y is 16-byte aligned
  const bool vec_out = kDataA && !kC && P.out.along == 1 && P.m % 4 == 0 && P.out.stride[0] % 4 == 0 &&
                       (reinterpret_cast<uintptr_t>(P.Y) & 15) == 0;
  TileWalk w(ntiles, P.rows, P.chunks, wave, nwaves);
  Digits din, dout;
  if (w.t < w.t1) {
    din.set(P.in, w.grp * P.cols + w.ch * kCols);
    dout.set(P.out, w.grp * P.cols + w.ch * kCols);
  }
  for (; w.t < w.t1;) {
    const int ic = w.ic;
    const int64_t grp = w.grp;
    const int64_t cb = grp * P.cols + w.ch * kCols;  // first column of the tile
    const int64_t cend = (grp + 1) * P.cols;
    const T* F = static_cast<const T*>(P.F) + grp * P.ldfp * kS;
    // The columns of a tile usually share every digit but the fastest (cb's
    // fastest digit + kCols - 1 stays below its radix): one offset for the
    // tile plus the column's step.  Otherwise every column is decomposed.
    const bool fast_in = P.in.nlev == 1 || din.d[0] + kCols <= P.in.mod[0];
    const bool fast_out = P.out.nlev == 1 || dout.d[0] + kCols <= P.out.mod[0];
    const int64_t in0 = din.offset(P.in), out0 = dout.offset(P.out);
    // sub-tile j: columns cb + 16 j .. + 15; this lane loads column cb + 16 j + L
    bool colok[kU];
    int64_t xb[kU];
#pragma unroll
    for (int j = 0; j < kU; ++j) {
      const int64_t cl = cb + 16 * j + L;
      colok[j] = cl < cend;
      xb[j] = fast_in ? in0 + (16 * j + L) * P.in.stride[0] : (colok[j] ? nd_offset(P.in, cl) : 0);
    }
    const int fi_row = 16 * ic + L;  // factor row held by this lane
    acc_t dr[kU], di[kU];
#pragma unroll
    for (int j = 0; j < kU; ++j) {
      dr[j] = acc_t{0, 0, 0, 0};
      di[j] = acc_t{0, 0, 0, 0};
    }
    for (int kc = 0; kc < nk; ++kc) {
      // the operands of every sub-tile first (loads in flight together)
      T xv[kU][4 * kS];
#pragma unroll
      for (int j = 0; j < kU; ++j) {
        if constexpr (kVecA) {
          if (colok[j] && 16 * kc + 4 * g < P.n) {
            ldv<T, 4 * kS>(X + (xb[j] + 16 * kc + 4 * g) * kS, xv[j], keep);
          } else {
#pragma unroll
            for (int q = 0; q < 4 * kS; ++q) xv[j][q] = T(0);
          }
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int a = 16 * kc + 4 * g + s;
            T xr = 0, xi = 0;
            if (colok[j] && a < P.n) ld_elem<T, kC>(X, xb[j] + (int64_t)a * P.in.along, xr, xi, keep);
            xv[j][s * kS] = xr;
            if constexpr (kC) xv[j][s * kS + 1] = xi;
          }
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int a = 16 * kc + 4 * g + s;
        T fr, fi;
        factor_entry<T, kC>(P, F, fi_row, a, fr, fi);
#pragma unroll
        for (int j = 0; j < kU; ++j) {
          const T xr = xv[j][s * kS];
          T xi = T(0);
          if constexpr (kC) xi = P.conjx ? -xv[j][s * kS + 1] : xv[j][s * kS + 1];
          if constexpr (kDataA) {
            dr[j] = A::mma(xr, fr, dr[j]);
            if constexpr (kC) {
              dr[j] = A::mma(xi, -fi, dr[j]);
              di[j] = A::mma(xi, fr, di[j]);
              di[j] = A::mma(xr, fi, di[j]);
            }
          } else {
            dr[j] = A::mma(fr, xr, dr[j]);
            if constexpr (kC) {
              dr[j] = A::mma(-fi, xi, dr[j]);
              di[j] = A::mma(fr, xi, di[j]);
              di[j] = A::mma(fi, xr, di[j]);
            }
          }
        }
      }
    }
    if constexpr (kDataA && !kC) {
      // Output index fastest, dense and 16-byte aligned: a quad transpose
      // gives each lane four consecutive outputs of one column, written as
      // one vector (instead of four scattered scalars).
      if (vec_out && fast_out && out0 % 4 == 0) {
#pragma unroll
        for (int j = 0; j < kU; ++j) {
          T o[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) o[r] = ar * dr[j][r];
          quad_transpose(o);
          const int i0 = 16 * ic + 4 * (L >> 2);
          const int jc = 16 * j + A::drow(g, L & 3);
          if (i0 >= P.m || cb + jc >= cend) continue;
          T* yp = Y + out0 + jc * P.out.stride[0] + i0;
          if constexpr (kBeta) {
            T old[4];
            ldv<T, 4>(yp, old);
#pragma unroll
            for (int r = 0; r < 4; ++r) o[r] += br * old[r];
          }
          stv<T, 4>(yp, o);
        }
        goto next_tile;
      }
    }
#pragma unroll
    for (int j = 0; j < kU; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = kDataA ? 16 * ic + L : 16 * ic + A::drow(g, r);
        const int jc = 16 * j + (kDataA ? A::drow(g, r) : L);  // column of the tile
        if (i >= P.m || cb + jc >= cend) continue;
        const int64_t e =
            (fast_out ? out0 + jc * P.out.stride[0] : nd_offset(P.out, cb + jc)) + (int64_t)i * P.out.along;
        T yr = ar * dr[j][r] - ai * di[j][r];
        T yi = ar * di[j][r] + ai * dr[j][r];
        if constexpr (kBeta) {
          T or_, oi;
          ld_elem<T, kC>(Y, e, or_, oi);
          yr = yr + (br * or_ - bi * oi);
          yi = yi + (br * oi + bi * or_);
        }
        st_elem<T, kC>(Y, e, yr, yi);
      }
    }
  next_tile:
    const int step = w.next(P.rows, P.chunks);
    if (step == 1) {
      din.add(P.in, kCols);
      dout.add(P.out, kCols);
    } else if (step == 2 && w.t < w.t1) {
      din.set(P.in, w.grp * P.cols);
      dout.set(P.out, w.grp * P.cols);
    }
  }
}

template <typename T, bool kC, bool kDataA, bool kBeta, bool kVecA>
void launch_mode(const NdPass& P, int64_t ntiles, T ar, T ai, T br, T bi, hipStream_t stream) {
  auto k = kron_mode_kernel<T, kC, kDataA, kBeta, kVecA>;
  hipLaunchKernelGGL(k, dim3(grid_blocks(ntiles, occupancy_blocks(k), 0)), dim3(kBlock), 0, stream, P, ntiles, ar, ai,
                     br, bi);
}

template <typename T, bool kC, int kW, bool kBeta>
void launch_wide(NdPass P, T ar, T ai, T br, T bi, hipStream_t stream) {
  P.chunks = (P.cols + 16 * kW - 1) / (16 * kW);
  const int64_t ntiles = (P.cols > 0 ? P.cols_groups : 0) * P.chunks * P.rows;
  auto k = kron_mode_wide_kernel<T, kC, kW, kBeta>;
  hipLaunchKernelGGL(k, dim3(grid_blocks(ntiles, occupancy_blocks(k), 0)), dim3(kBlock), 0, stream, P, ntiles, ar, ai,
                     br, bi);
}

template <typename T, bool kC, bool kBeta>
void run_pass_b(const NdPass& P, int64_t ntiles, bool dense, T ar, T ai, T br, T bi, hipStream_t s) {
  const int64_t post = P.in.nlev == 2 ? P.in.mod[0] : 1;
  const bool aligned = ((reinterpret_cast<uintptr_t>(P.X) | reinterpret_cast<uintptr_t>(P.Y)) & 15) == 0;
  if (dense && aligned && post % 4 == 0) {
    launch_wide<T, kC, 4, kBeta>(P, ar, ai, br, bi, s);
  } else if (dense && aligned && post % 2 == 0) {
    launch_wide<T, kC, 2, kBeta>(P, ar, ai, br, bi, s);
  } else {
    launch_mode<T, kC, false, kBeta, false>(P, ntiles, ar, ai, br, bi, s);
  }
}

// One pass: the data as A operand when post == 1 (vector loads when the input
// is dense, n is a multiple of 4 and X 16-byte aligned), else as B operand
// (the wide tiles when both sides are dense, aligned, and post allows).
template <typename T, bool kC>
void run_pass(const NdPass& P, int64_t ntiles, bool data_a, bool dense_in, bool dense_out, bool beta, T ar, T ai,
              T br, T bi, hipStream_t s) {
  if (data_a) {
    const bool vec = dense_in && P.n % 4 == 0 && (reinterpret_cast<uintptr_t>(P.X) & 15) == 0;
    if (vec) {
      if (beta) launch_mode<T, kC, true, true, true>(P, ntiles, ar, ai, br, bi, s);
      else launch_mode<T, kC, true, false, true>(P, ntiles, ar, ai, br, bi, s);
    } else {
      if (beta) launch_mode<T, kC, true, true, false>(P, ntiles, ar, ai, br, bi, s);
      else launch_mode<T, kC, true, false, false>(P, ntiles, ar, ai, br, bi, s);
    }
  } else {
    if (beta) run_pass_b<T, kC, true>(P, ntiles, dense_in && dense_out, ar, ai, br, bi, s);
    else run_pass_b<T, kC, false>(P, ntiles, dense_in && dense_out, ar, ai, br, bi, s);
  }
}

int op_code(char c) {
  switch (c) {
    case 'N': case 'n': return 0;
    case 'T': case 't': return 1;
    case 'C': case 'c': return 2;
    default: return -1;
  }
}

// Elements after pass k (k = d..0: d is the input, 0 the output): extents
// n_0 .. n_{k-1}, m_k .. m_{d-1}.
int64_t extent_after(int d, const int* m, const int* n, int k) {
  int64_t s = 1;
  for (int j = 0; j < d; ++j) s *= j < k ? n[j] : m[j];
  return s;
}

// Scalars of one intermediate array (the largest one), 0 when d == 1.
int64_t nd_inter_elems(int d, const int* m, const int* n, int64_t batch) {
  int64_t big = 0;
  for (int k = 1; k < d; ++k) {
    const int64_t e = extent_after(d, m, n, k) * batch;
    if (e > big) big = e;
  }
  return big;
}

size_t nd_ws_bytes(int d, const int* m, const int* n, int64_t batch, size_t elem) {
  const int64_t inter = nd_inter_elems(d, m, n, batch);
  const int copies = d >= 3 ? 2 : (d == 2 ? 1 : 0);
  const size_t one = ((size_t)inter * elem + 255) / 256 * 256;
  return one * (size_t)copies;
}

bool sizes_ok(int d, const int* m, const int* n) {
  if (d < 1 || d > kNdMaxDim || !m || !n) return false;
  double ex = 1, ey = 1;
  for (int k = 0; k < d; ++k) {
    if (m[k] < 1 || n[k] < 1 || m[k] > KRON_ND_MAX_EXTENT || n[k] > KRON_ND_MAX_EXTENT) return false;
    ex *= n[k];
    ey *= m[k];
  }
  return ex < 9e15 && ey < 9e15;
}

// Strided operand storage of the first pass's input or the last pass's
// output (d <= 3): element stride of each index and between operands.
struct NdStrides {
  int64_t s[3];
  int64_t sp;
};

// Index of a dense pass: In[u, a, v] / Out[u, i, v] with v < post and
// extent e of the middle index.
NdIndex dense_index(int64_t e, int64_t post) {
  NdIndex ix{};
  if (post == 1) {
    ix.nlev = 1;
    ix.stride[0] = e;
    ix.along = 1;
  } else {
    ix.nlev = 2;
    ix.mod[0] = post;
    ix.stride[0] = 1;
    ix.stride[1] = e * post;
    ix.along = post;
  }
  return ix;
}

// Index of strided storage with extents ext[0..d-1] when index k0 is the
// contracted one (the fastest, d - 1, for the first pass) or the produced
// one (the slowest, 0, for the last pass): the other indices are the
// digits, fastest first, then the operand.
NdIndex strided_index(int d, const int* ext, const NdStrides& st, int k0) {
  NdIndex ix{};
  int lev = 0;
  for (int j = d - 1; j >= 0; --j) {
    if (j == k0) continue;
    ix.mod[lev] = ext[j];
    ix.stride[lev] = st.s[j];
    ++lev;
  }
  ix.stride[lev] = st.sp;
  ix.nlev = lev + 1;
  ix.along = st.s[k0];
  return ix;
}

// Argument positions of kron_nd_batched_*: d 1, m 2, n 3, ops 4, alpha 5,
// factors 6, ldf 7, ldfp 8, X 9, beta 10, Y 11, batch 12, ws 13, ws_bytes 14.
// xs / ys: strided storage of X and Y (d <= 3), or nullptr for packed
// operands; conjx conjugates X on the way in.  The caller checks them.
template <typename T, bool kC>
int nd_run(int d, const int* m, const int* n, const char* ops, T ar, T ai, const T* const* F, const int* ldf,
           const int64_t* ldfp, const T* X, T br, T bi, T* Y, int64_t batch, void* ws, size_t ws_bytes,
           hipStream_t stream, const NdStrides* xs = nullptr, const NdStrides* ys = nullptr, bool conjx = false) {
  if (d < 1 || d > kNdMaxDim) return -1;
  if (!m || !sizes_ok(d, m, n)) return -2;
  if (!n) return -3;
  if (!ops) return -4;
  int opc[kNdMaxDim];
  for (int k = 0; k < d; ++k)
    if ((opc[k] = op_code(ops[k])) < 0) return -4;  // 'C' on real data is 'T'
  if (!F) return -6;
  for (int k = 0; k < d; ++k)
    if (!F[k]) return -6;
  if (!ldf) return -7;
  for (int k = 0; k < d; ++k)
    if (ldf[k] < (opc[k] == 0 ? m[k] : n[k])) return -7;
  if (!ldfp) return -8;
  for (int k = 0; k < d; ++k)
    if (ldfp[k] < 0) return -8;
  if (!X) return -9;
  if (!Y || (const void*)Y == (const void*)X) return -11;
  if (batch < 0) return -12;
  if (batch == 0) return 0;
  const size_t elem = sizeof(T) * (kC ? 2 : 1);
  const size_t need = nd_ws_bytes(d, m, n, batch, elem);
  if (need > 0 && (!ws || reinterpret_cast<uintptr_t>(ws) % 16 != 0)) return -13;
  if (ws_bytes < need) return -14;
  const size_t half = d >= 3 ? need / 2 : need;
  T* buf[2] = {static_cast<T*>(ws), reinterpret_cast<T*>(static_cast<uint8_t*>(ws) + half)};
  const bool has_beta = br != T(0) || bi != T(0);
  const void* in = X;
  int which = 0;
  for (int k = d - 1; k >= 0; --k) {
    NdPass P;
    P.X = in;
    P.Y = k == 0 ? static_cast<void*>(Y) : static_cast<void*>(buf[which]);
    P.F = F[k];
    P.ldfp = ldfp[k];
    P.ld = ldf[k];
    P.op = opc[k];
    P.m = m[k];
    P.n = n[k];
    P.conjx = conjx && k == d - 1;
    int64_t pre = 1, post = 1;
    for (int j = 0; j < k; ++j) pre *= n[j];
    for (int j = k + 1; j < d; ++j) post *= m[j];
    P.in = (k == d - 1 && xs) ? strided_index(d, n, *xs, d - 1) : dense_index(n[k], post);
    if (k == 0 && ys) {
      P.out = strided_index(d, m, *ys, 0);
    } else {
      P.out = dense_index(m[k], post);
    }
    const bool shared = ldfp[k] == 0;
    P.cols = shared ? batch * pre * post : pre * post;
    const int64_t groups = shared ? 1 : batch;
    P.cols_groups = groups;
    P.chunks = (P.cols + 16 * nd_sub_tiles<kC>() - 1) / (16 * nd_sub_tiles<kC>());
    P.rows = (m[k] + 15) / 16;
    const int64_t ntiles = groups * P.chunks * P.rows;
    const bool last = k == 0;
    const bool dense_in = !(k == d - 1 && xs), dense_out = !(k == 0 && ys);
    run_pass<T, kC>(P, ntiles, post == 1, dense_in, dense_out, last && has_beta, last ? ar : T(1), last ? ai : T(0),
                    br, bi, stream);
    in = P.Y;
    which ^= 1;
  }
  return 0;
}

// Checks shared by the TKRON-style entry points (Section 3's argument lists
// with rectangular factors): returns 0 or -position.
int rect_op(char c) { return op_code(c); }
bool extent_ok(int v) { return v >= 1 && v <= KRON_ND_MAX_EXTENT; }

// Workspace check at the caller's argument positions (kws: ws, kws + 1: ws_bytes).
int rect_ws_check(int d, const int* m, const int* n, int64_t batch, size_t elem, const void* ws, size_t ws_bytes,
                  int kws) {
  if (batch <= 0) return 0;
  const size_t need = nd_ws_bytes(d, m, n, batch, elem);
  if (need > 0 && (!ws || reinterpret_cast<uintptr_t>(ws) % 16 != 0)) return -kws;
  if (ws_bytes < need) return -(kws + 1);
  return 0;
}

template <typename T, bool kC>
int rect_run(int d, const char* ops, const int* m, const int* nn, int64_t batch, T ar, T ai, const T* const* F,
             const int* ld, const T* X, const NdStrides& xs, T br, T bi, T* Y, const NdStrides& ys, bool conjx,
             void* ws, size_t ws_bytes, hipStream_t stream) {
  int64_t ldfp[3] = {0, 0, 0};
  const int rc = nd_run<T, kC>(d, m, nn, ops, ar, ai, F, ld, ldfp, X, br, bi, Y, batch, ws, ws_bytes, stream, &xs,
                               &ys, conjx);
  if (rc != 0) return rc;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

}  // namespace
}  // namespace kron

extern "C" {

size_t kron_nd_workspace_size(int d, const int* m, const int* n, int64_t batch, int type) {
  if (!kron::sizes_ok(d, m, n) || batch < 0) return 0;
  size_t elem;
  switch (type) {
    case KRON_MODE_F32: elem = 4; break;
    case KRON_MODE_F64: elem = 8; break;
    case KRON_TYPE_C32: elem = 8; break;
    case KRON_TYPE_C64: elem = 16; break;
    default: return 0;
  }
  return kron::nd_ws_bytes(d, m, n, batch, elem);
}

int kron_nd_batched_f32(int d, const int* m, const int* n, const char* ops, float alpha, const float* const* factors,
                        const int* ldf, const int64_t* ldfp, const float* X, float beta, float* Y, int64_t batch,
                        void* ws, size_t ws_bytes, hipStream_t stream) {
  int rc = kron::nd_run<float, false>(d, m, n, ops, alpha, 0.f, factors, ldf, ldfp, X, beta, 0.f, Y, batch, ws,
                                      ws_bytes, stream);
  if (rc != 0) return rc;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

int kron_nd_batched_f64(int d, const int* m, const int* n, const char* ops, double alpha,
                        const double* const* factors, const int* ldf, const int64_t* ldfp, const double* X,
                        double beta, double* Y, int64_t batch, void* ws, size_t ws_bytes, hipStream_t stream) {
  int rc = kron::nd_run<double, false>(d, m, n, ops, alpha, 0.0, factors, ldf, ldfp, X, beta, 0.0, Y, batch, ws,
                                       ws_bytes, stream);
  if (rc != 0) return rc;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

int kron_nd_batched_c32(int d, const int* m, const int* n, const char* ops, kron_c32_t alpha,
                        const kron_c32_t* const* factors, const int* ldf, const int64_t* ldfp, const kron_c32_t* X,
                        kron_c32_t beta, kron_c32_t* Y, int64_t batch, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  int rc = kron::nd_run<float, true>(d, m, n, ops, alpha.re, alpha.im,
                                     reinterpret_cast<const float* const*>(factors), ldf, ldfp,
                                     reinterpret_cast<const float*>(X), beta.re, beta.im,
                                     reinterpret_cast<float*>(Y), batch, ws, ws_bytes, stream);
  if (rc != 0) return rc;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

int kron_nd_batched_c64(int d, const int* m, const int* n, const char* ops, kron_c64_t alpha,
                        const kron_c64_t* const* factors, const int* ldf, const int64_t* ldfp, const kron_c64_t* X,
                        kron_c64_t beta, kron_c64_t* Y, int64_t batch, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  int rc = kron::nd_run<double, true>(d, m, n, ops, alpha.re, alpha.im,
                                      reinterpret_cast<const double* const*>(factors), ldf, ldfp,
                                      reinterpret_cast<const double*>(X), beta.re, beta.im,
                                      reinterpret_cast<double*>(Y), batch, ws, ws_bytes, stream);
  if (rc != 0) return rc;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

}  // extern "C"

// ---- TKRON1 / TKRON2 / TKRON3 with rectangular factors (Section 3) ---------

#define KRON_RECT_TYPES(F) \
  F(f32, float, float, false, a, 0.f, b, 0.f) \
  F(f64, double, double, false, a, 0.0, b, 0.0) \
  F(c32, float, kron_c32_t, true, a.re, a.im, b.re, b.im) \
  F(c64, double, kron_c64_t, true, a.re, a.im, b.re, b.im)

// 1-D: positions opA 1, ma 2, na 3, batch 4, alpha 5, A 6, lda 7, X 8,
// ldxp 9, beta 10, Y 11, ldyp 12, ws 13, ws_bytes 14.
#define KRON_RECT1(TAG, R, E, CPLX, AR, AI, BR, BI)                                                              \
  int kron1d_batched_rect_##TAG(char opA, int ma, int na, int64_t batch, E a, const E* A, int lda, const E* X,  \
                                int64_t ldxp, E b, E* Y, int64_t ldyp, void* ws, size_t ws_bytes,               \
                                hipStream_t stream) {                                                           \
    if (kron::rect_op(opA) < 0) return -1;                                                                      \
    if (!kron::extent_ok(ma)) return -2;                                                                        \
    if (!kron::extent_ok(na)) return -3;                                                                        \
    if (batch < 0) return -4;                                                                                   \
    if (!A) return -6;                                                                                          \
    if (lda < (kron::rect_op(opA) == 0 ? ma : na)) return -7;                                                   \
    if (!X) return -8;                                                                                          \
    if (ldxp < 0) return -9;                                                                                    \
    if (!Y || (const void*)Y == (const void*)X) return -11;                                                     \
    if (ldyp < ma) return -12;                                                                                  \
    const int m[1] = {ma}, n[1] = {na}, ld[1] = {lda};                                                          \
    const char ops[1] = {opA};                                                                                  \
    const R* F[1] = {reinterpret_cast<const R*>(A)};                                                            \
    const kron::NdStrides xs{{1, 0, 0}, ldxp}, ys{{1, 0, 0}, ldyp};                                              \
    return kron::rect_run<R, CPLX>(1, ops, m, n, batch, AR, AI, F, ld, reinterpret_cast<const R*>(X), xs, BR,   \
                                   BI, reinterpret_cast<R*>(Y), ys, false, ws, ws_bytes, stream);               \
  }

// 2-D: positions opA 1, opB 2, opX 3, ma 4, na 5, mb 6, nb 7, batch 8,
// alpha 9, A 10, lda 11, B 12, ldb 13, X 14, ldx 15, ldxp 16, beta 17,
// Y 18, ldy 19, ldyp 20, ws 21, ws_bytes 22.
#define KRON_RECT2(TAG, R, E, CPLX, AR, AI, BR, BI)                                                              \
  int kron2d_batched_rect_##TAG(char opA, char opB, char opX, int ma, int na, int mb, int nb, int64_t batch,    \
                                E a, const E* A, int lda, const E* B, int ldb, const E* X, int64_t ldx,         \
                                int64_t ldxp, E b, E* Y, int64_t ldy, int64_t ldyp, void* ws, size_t ws_bytes,  \
                                hipStream_t stream) {                                                           \
    const int oa = kron::rect_op(opA), ob = kron::rect_op(opB), ox = kron::rect_op(opX);                        \
    if (oa < 0) return -1;                                                                                      \
    if (ob < 0) return -2;                                                                                      \
    if (ox < 0) return -3;                                                                                      \
    if (!kron::extent_ok(ma)) return -4;                                                                        \
    if (!kron::extent_ok(na)) return -5;                                                                        \
    if (!kron::extent_ok(mb)) return -6;                                                                        \
    if (!kron::extent_ok(nb)) return -7;                                                                        \
    if (batch < 0) return -8;                                                                                   \
    if (!A) return -10;                                                                                         \
    if (lda < (oa == 0 ? ma : na)) return -11;                                                                  \
    if (!B) return -12;                                                                                         \
    if (ldb < (ob == 0 ? mb : nb)) return -13;                                                                  \
    if (!X) return -14;                                                                                         \
    if (ldx < 0) return -15;                                                                                    \
    if (ldxp < 0) return -16;                                                                                   \
    if (!Y || (const void*)Y == (const void*)X) return -18;                                                     \
    if (ldy < mb) return -19;                                                                                   \
    if (ldyp < ldy * ma) return -20;                                                                            \
    const int m[2] = {ma, mb}, n[2] = {na, nb}, ld[2] = {lda, ldb};                                             \
    if (int rc = kron::rect_ws_check(2, m, n, batch, sizeof(E), ws, ws_bytes, 21)) return rc;                  \
    const char ops[2] = {opA, opB};                                                                             \
    const R* F[2] = {reinterpret_cast<const R*>(A), reinterpret_cast<const R*>(B)};                             \
    /* op(X_p)(a0, a1), a1 the fast index: X_p(a1, a0) at a1 + ldx a0, or (op T / C) X_p(a0, a1) at */          \
    /* a0 + ldx a1 */                                                                                           \
    const kron::NdStrides xs = ox == 0 ? kron::NdStrides{{ldx, 1, 0}, ldxp} : kron::NdStrides{{1, ldx, 0}, ldxp}; \
    const kron::NdStrides ys{{ldy, 1, 0}, ldyp};                                                                \
    return kron::rect_run<R, CPLX>(2, ops, m, n, batch, AR, AI, F, ld, reinterpret_cast<const R*>(X), xs, BR,   \
                                   BI, reinterpret_cast<R*>(Y), ys, ox == 2, ws, ws_bytes, stream);             \
  }

// 3-D: positions opA 1, opB 2, opC 3, ma 4, na 5, mb 6, nb 7, mc 8, nc 9,
// batch 10, alpha 11, A 12, lda 13, B 14, ldb 15, C 16, ldc 17, X 18,
// ldx 19, ldx2 20, ldxp 21, beta 22, Y 23, ldy 24, ldy2 25, ldyp 26, ws 27,
// ws_bytes 28.
#define KRON_RECT3(TAG, R, E, CPLX, AR, AI, BR, BI)                                                              \
  int kron3d_batched_rect_##TAG(char opA, char opB, char opC, int ma, int na, int mb, int nb, int mc, int nc,   \
                                int64_t batch, E a, const E* A, int lda, const E* B, int ldb, const E* C,       \
                                int ldc, const E* X, int64_t ldx, int64_t ldx2, int64_t ldxp, E b, E* Y,        \
                                int64_t ldy, int64_t ldy2, int64_t ldyp, void* ws, size_t ws_bytes,             \
                                hipStream_t stream) {                                                           \
    const int oa = kron::rect_op(opA), ob = kron::rect_op(opB), oc = kron::rect_op(opC);                        \
    if (oa < 0) return -1;                                                                                      \
    if (ob < 0) return -2;                                                                                      \
    if (oc < 0) return -3;                                                                                      \
    if (!kron::extent_ok(ma)) return -4;                                                                        \
    if (!kron::extent_ok(na)) return -5;                                                                        \
    if (!kron::extent_ok(mb)) return -6;                                                                        \
    if (!kron::extent_ok(nb)) return -7;                                                                        \
    if (!kron::extent_ok(mc)) return -8;                                                                        \
    if (!kron::extent_ok(nc)) return -9;                                                                        \
    if (batch < 0) return -10;                                                                                  \
    if (!A) return -12;                                                                                         \
    if (lda < (oa == 0 ? ma : na)) return -13;                                                                  \
    if (!B) return -14;                                                                                         \
    if (ldb < (ob == 0 ? mb : nb)) return -15;                                                                  \
    if (!C) return -16;                                                                                         \
    if (ldc < (oc == 0 ? mc : nc)) return -17;                                                                  \
    if (!X) return -18;                                                                                         \
    if (ldx < 0) return -19;                                                                                    \
    if (ldx2 < 0) return -20;                                                                                   \
    if (ldxp < 0) return -21;                                                                                   \
    if (!Y || (const void*)Y == (const void*)X) return -23;                                                     \
    if (ldy < mc) return -24;                                                                                   \
    if (ldy2 < ldy * mb) return -25;                                                                            \
    if (ldyp < ldy2 * ma) return -26;                                                                           \
    const int m[3] = {ma, mb, mc}, n[3] = {na, nb, nc}, ld[3] = {lda, ldb, ldc};                                \
    if (int rc = kron::rect_ws_check(3, m, n, batch, sizeof(E), ws, ws_bytes, 27)) return rc;                  \
    const char ops[3] = {opA, opB, opC};                                                                        \
    const R* F[3] = {reinterpret_cast<const R*>(A), reinterpret_cast<const R*>(B), reinterpret_cast<const R*>(C)}; \
    const kron::NdStrides xs{{ldx2, ldx, 1}, ldxp}, ys{{ldy2, ldy, 1}, ldyp};                                   \
    return kron::rect_run<R, CPLX>(3, ops, m, n, batch, AR, AI, F, ld, reinterpret_cast<const R*>(X), xs, BR,   \
                                   BI, reinterpret_cast<R*>(Y), ys, false, ws, ws_bytes, stream);               \
  }

extern "C" {
KRON_RECT_TYPES(KRON_RECT1)
KRON_RECT_TYPES(KRON_RECT2)
KRON_RECT_TYPES(KRON_RECT3)
}  // extern "C"
