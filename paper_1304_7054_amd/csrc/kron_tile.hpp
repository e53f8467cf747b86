// Device building blocks of the batched Kronecker action on gfx950.
//
// One wavefront (64 lanes) owns one "tile": a 16 x 16 (2-D) or 16 x 16 x 16
// (3-D) block of slots.  For n = 16 a tile is one operand.  For smaller n,
// Q = 16 / n operands are packed along every axis (Q^2 or Q^3 operands per
// tile) and the shared factors are expanded to block-diagonal 16 x 16 tiles
// diag(M, ..., M, 0); the cross terms vanish, so each packed operand sees its
// own action (the paper's batched update of Section 2.2 with the factors
// constant across the batch, Section 1).
//
// Every mode product is a 16-slot contraction done on the matrix cores with
// the 16x16 MFMA family.  Register picture per lane (l = lane, L = l % 16,
// g = l / 16):
//   * operand "A" of an MFMA takes row L and contraction slots k(g, s);
//   * operand "B" takes column L and the same contraction slots;
//   * the 4-element accumulator holds rows drow(g, r), column L, where
//     drow(g, r) = 4g + r for FP32 and bf16 MFMAs and g + 4r for FP64.
// A stage's accumulator can feed the next stage as either operand without
// any data movement: the index held on rows becomes the contraction index,
// the column index stays on L.  Which of the two roles it takes decides
// where the new index appears, and the stage order is chosen so that both
// the operand load and the result store are contiguous 16-byte accesses for
// FP32 at n = 16.  Only the 3-D path needs one exchange: the slab index
// (which register) trades places with the row-group index (which lane group)
// through two rounds of gfx950 permlane swaps, 64 instructions per tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kron {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kSlots = 16;

// Address-space views.  HIP pointers are generic; where a pointer crosses an
// out-of-line call the compiler can no longer tell global memory from LDS and
// falls back to flat instructions, which count against both the memory and
// the LDS wait counters (an LDS wait then also waits for every global load
// in flight).  Every access below goes through one of these views instead.
template <typename T>
using global_ptr = __attribute__((address_space(1))) T*;
template <typename T>
using lds_ptr = __attribute__((address_space(3))) T*;
template <typename T>
__device__ __forceinline__ global_ptr<T> in_global(T* p) {
  return (global_ptr<T>)p;
}
template <typename T>
__device__ __forceinline__ lds_ptr<T> in_lds(T* p) {
  return (lds_ptr<T>)p;
}

// ---- tile geometry ---------------------------------------------------------

template <int N>
struct Geo {
  static_assert(N >= 1 && N <= 16, "n must be in 1..16");
  static constexpr int Q = kSlots / N;   // operands packed per axis
  static constexpr int U = Q * N;        // used slots per axis
  // When fewer than 16 slots hold data, logical index u sits in slot
  // 4 * (u % 4) + u / 4 (row group u % 4, register u / 4): the used slots
  // then fill the first kSteps contraction steps, and the remaining steps
  // (all zero) are skipped.  Every axis, the data and the factor tiles use the
  // same placement, so the contractions are unchanged.
  static constexpr bool kPerm = U < 16;
  static constexpr int kSteps = kPerm ? (U + 3) / 4 : 4;
  static constexpr bool kVec = (N % 4) == 0 && !kPerm;  // 4 consecutive slots = 4 consecutive elements
};

// slot -> (packed-operand index along the axis, index inside the operand)
template <int N>
struct Slot {
  int sub, idx;
  bool valid;
  __device__ __forceinline__ explicit Slot(int s) {
    const int u = Geo<N>::kPerm ? 4 * (s % 4) + s / 4 : s;
    sub = u / N;
    idx = u % N;
    valid = u < Geo<N>::U;
  }
};

// logical index u (0 <= u < U) -> its slot (the inverse of Slot: the
// placement is its own inverse)
template <int N>
__device__ __forceinline__ constexpr int slot_of(int u) {
  return Geo<N>::kPerm ? 4 * (u % 4) + u / 4 : u;
}

template <int N>
__device__ __forceinline__ constexpr bool slot_live(int s) {
  return (Geo<N>::kPerm ? 4 * (s % 4) + s / 4 : s) < Geo<N>::U;
}

// ---- bf16 helpers ------------------------------------------------------------

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }  // round to nearest even
__device__ __forceinline__ float from_bf16(__bf16 h) { return (float)h; }
__device__ __forceinline__ __bf16 bits_to_bf16(uint16_t b) { return __builtin_bit_cast(__bf16, b); }
__device__ __forceinline__ uint16_t bf16_to_bits(__bf16 h) { return __builtin_bit_cast(uint16_t, h); }

// x = hi + lo + O(2^-16 |x|): hi = bf16(x), lo = bf16(x - hi); x - hi is exact in FP32.
__device__ __forceinline__ void split4(const f32x4& x, bf16x4& hi, bf16x4& lo) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    __bf16 h = to_bf16(x[e]);
    hi[e] = h;
    lo[e] = to_bf16(x[e] - from_bf16(h));
  }
}

__device__ __forceinline__ bf16x8 cat8(const bf16x4& a, const bf16x4& b) {
  bf16x8 r;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    r[e] = a[e];
    r[e + 4] = b[e];
  }
  return r;
}

// ---- MFMA wrappers -------------------------------------------------------------

__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_bf16_k16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_bf16_k32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---- factor tiles -----------------------------------------------------------------
//
// Each lane keeps, for every shared factor M, the four values
//   Mt(L, k(g, s)), s = 0..3,
// of the block-diagonal tile Mt = diag(M, ..., M, 0).  M is column-major
// (M(i, j) at i + n*j); with kTrans the tile of M^T is taken instead.
// `kmap` selects the contraction-slot order: 0 -> 4g + s, 1 -> drow(g, s).

template <int N, bool kTrans, typename T>
__device__ __forceinline__ T tile_entry(const T* M, int row, int col) {
  Slot<N> r(row), c(col);
  if (!(r.valid && c.valid) || r.sub != c.sub) return T(0);
  return kTrans ? in_global(M)[c.idx + N * r.idx] : in_global(M)[r.idx + N * c.idx];
}

// ---- precision modes -----------------------------------------------------------------
//
// Each mode provides
//   io_t      element type in memory
//   acc_t     accumulator (four values per lane)
//   fac_t     per-lane factor values for one stage
//   drow(g,r) accumulator row held by lane group g, register r
//   load_fac  the factor values for contraction-slot map kmap
//   da(f, x)  stage with the data as MFMA operand A (row L, slots k(g, s) in x[s])
//   db(f, x)  stage with the data as MFMA operand B
//   da_in     the first stage, fed straight from memory values

struct ModeF32 {
  using io_t = float;
  using acc_t = f32x4;
  using elem_t = float;
  using fac_t = f32x4;
  static constexpr int kBytes = 4;
  __device__ static constexpr int drow(int g, int r) { return 4 * g + r; }
  template <int N, bool kTrans>
  __device__ static fac_t load_fac(const io_t* M, int L, int g, int kmap) {
    fac_t f;
#pragma unroll
    for (int s = 0; s < 4; ++s) f[s] = tile_entry<N, kTrans>(M, L, kmap == 0 ? 4 * g + s : drow(g, s));
    return f;
  }
  template <int kSteps = 4>
  __device__ static acc_t da(const fac_t& f, const acc_t& x) {
    acc_t c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < kSteps; ++s) c = mfma_f32(x[s], f[s], c);
    return c;
  }
  template <int kSteps = 4>
  __device__ static acc_t db(const fac_t& f, const acc_t& x) {
    acc_t c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < kSteps; ++s) c = mfma_f32(f[s], x[s], c);
    return c;
  }
  template <int kSteps = 4>
  __device__ static acc_t da_in(const fac_t& f, const acc_t& x) { return da<kSteps>(f, x); }
  __device__ static acc_t to_acc(const f32x4& v) { return v; }
};

struct ModeF64 {
  using io_t = double;
  using acc_t = f64x4;
  using elem_t = double;
  using fac_t = f64x4;
  static constexpr int kBytes = 8;
  __device__ static constexpr int drow(int g, int r) { return g + 4 * r; }
  template <int N, bool kTrans>
  __device__ static fac_t load_fac(const io_t* M, int L, int g, int kmap) {
    fac_t f;
#pragma unroll
    for (int s = 0; s < 4; ++s) f[s] = tile_entry<N, kTrans>(M, L, kmap == 0 ? 4 * g + s : drow(g, s));
    return f;
  }
  // An FP64 accumulator holds rows g + 4r, so when it feeds the next stage
  // step s contracts slots 4s..4s+3, which under the placement of Geo hold
  // logical indices s, s+4, s+8, s+12: every step can hold data, and da/db
  // always take all four.  Only the first stage, fed in slot order 4g + s
  // (step s = logical 4s..4s+3), skips the empty steps.
  template <int kSteps = 4>
  __device__ static acc_t da(const fac_t& f, const acc_t& x) {
    acc_t c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) c = mfma_f64(x[s], f[s], c);
    return c;
  }
  template <int kSteps = 4>
  __device__ static acc_t db(const fac_t& f, const acc_t& x) {
    acc_t c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) c = mfma_f64(f[s], x[s], c);
    return c;
  }
  template <int kSteps = 4>
  __device__ static acc_t da_in(const fac_t& f, const acc_t& x) {
    acc_t c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kSteps; ++s) c = mfma_f64(x[s], f[s], c);
    return c;
  }
};

// bf16x3: every FP32 value v is split as hi + lo; a product v*m is taken as
// hi*mlo + lo*mhi (the small terms first) + hi*mhi, lo*lo' dropped.  Both
// steps are K=32 bf16 MFMAs on the same packed data [hi | lo]: the first
// pairs it with [mlo | mhi], the second with [mhi | 0].  The two are chained
// through the accumulator with the same instruction on purpose: a K=32
// result fed as the accumulator of a K=16 bf16 MFMA came out stale on
// gfx950 with the wait states the compiler inserts.
struct ModeBF16x3 {
  using io_t = float;
  using acc_t = f32x4;
  struct fac_t {
    bf16x8 small;  // [mlo | mhi]
    bf16x8 big;    // [mhi | 0]
  };
  static constexpr int kBytes = 4;
  __device__ static constexpr int drow(int g, int r) { return 4 * g + r; }
  template <int N, bool kTrans>
  __device__ static fac_t load_fac(const io_t* M, int L, int g, int kmap) {
    f32x4 v;
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = tile_entry<N, kTrans>(M, L, kmap == 0 ? 4 * g + s : drow(g, s));
    bf16x4 hi, lo, zero;
    split4(v, hi, lo);
#pragma unroll
    for (int e = 0; e < 4; ++e) zero[e] = to_bf16(0.f);
    return fac_t{cat8(lo, hi), cat8(hi, zero)};
  }
  template <int kSteps = 4>
  __device__ static acc_t da(const fac_t& f, const acc_t& x) {
    bf16x4 hi, lo;
    split4(x, hi, lo);
    const bf16x8 d = cat8(hi, lo);
    acc_t c = {0.f, 0.f, 0.f, 0.f};
    c = mfma_bf16_k32(d, f.small, c);
    return mfma_bf16_k32(d, f.big, c);
  }
  template <int kSteps = 4>
  __device__ static acc_t db(const fac_t& f, const acc_t& x) {
    bf16x4 hi, lo;
    split4(x, hi, lo);
    const bf16x8 d = cat8(hi, lo);
    acc_t c = {0.f, 0.f, 0.f, 0.f};
    c = mfma_bf16_k32(f.small, d, c);
    return mfma_bf16_k32(f.big, d, c);
  }
  template <int kSteps = 4>
  __device__ static acc_t da_in(const fac_t& f, const acc_t& x) { return da(f, x); }
};

// bf16x6: every FP32 value v is split three ways, v = h + m + l with
// h = bf16(v), m = bf16(v - h), l = bf16(v - h - m); both differences are
// exact in FP32 and l takes the last bits exactly, so the three parts hold
// all 24 significant bits.  A product v*w is taken as six bf16 products,
// smallest first: h*wl + l*wh, then h*wm + m*wh, then h*wh + m*wm, each pair
// one K=32 MFMA on packed data ([h | l] or [h | m]) chained through the
// accumulator; the dropped terms (m*wl, l*wm, l*wl) are below 2^-23 of |v*w|.
// Three MFMAs per step instead of bf16x3's two, for results as accurate as
// plain FP32 on any data (bf16x3 keeps 16 significant bits per value).
__device__ __forceinline__ void split3(const f32x4& x, bf16x4& h, bf16x4& m, bf16x4& l) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const __bf16 a = to_bf16(x[e]);
    const float r1 = x[e] - from_bf16(a);
    const __bf16 b = to_bf16(r1);
    h[e] = a;
    m[e] = b;
    l[e] = to_bf16(r1 - from_bf16(b));
  }
}

struct ModeBF16x6 {
  using io_t = float;
  using acc_t = f32x4;
  struct fac_t {
    bf16x8 lh;  // [wl | wh]: pairs with data [h | l]
    bf16x8 mh;  // [wm | wh]: pairs with data [h | m]
    bf16x8 hm;  // [wh | wm]: pairs with data [h | m]
  };
  static constexpr int kBytes = 4;
  __device__ static constexpr int drow(int g, int r) { return 4 * g + r; }
  template <int N, bool kTrans>
  __device__ static fac_t load_fac(const io_t* M, int L, int g, int kmap) {
    f32x4 v;
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = tile_entry<N, kTrans>(M, L, kmap == 0 ? 4 * g + s : drow(g, s));
    bf16x4 h, m, l;
    split3(v, h, m, l);
    return fac_t{cat8(l, h), cat8(m, h), cat8(h, m)};
  }
  template <int kSteps = 4>
  __device__ static acc_t da(const fac_t& f, const acc_t& x) {
    bf16x4 h, m, l;
    split3(x, h, m, l);
    const bf16x8 dhl = cat8(h, l), dhm = cat8(h, m);
    acc_t c = {0.f, 0.f, 0.f, 0.f};
    c = mfma_bf16_k32(dhl, f.lh, c);
    c = mfma_bf16_k32(dhm, f.mh, c);
    return mfma_bf16_k32(dhm, f.hm, c);
  }
  template <int kSteps = 4>
  __device__ static acc_t db(const fac_t& f, const acc_t& x) {
    bf16x4 h, m, l;
    split3(x, h, m, l);
    const bf16x8 dhl = cat8(h, l), dhm = cat8(h, m);
    acc_t c = {0.f, 0.f, 0.f, 0.f};
    c = mfma_bf16_k32(f.lh, dhl, c);
    c = mfma_bf16_k32(f.mh, dhm, c);
    return mfma_bf16_k32(f.hm, dhm, c);
  }
  template <int kSteps = 4>
  __device__ static acc_t da_in(const fac_t& f, const acc_t& x) { return da(f, x); }
};

// bf16 storage: the factors and the operands are exact bf16 values.  The
// first stage multiplies bf16 by bf16 exactly (one K=16 MFMA); later stages
// split the FP32 intermediate into hi + lo and take hi*m + lo*m in one K=32
// MFMA.  The result is rounded to bf16 on the way out.
struct ModeBF16 {
  using io_t = uint16_t;
  using acc_t = f32x4;
  using fac_t = bf16x4;
  static constexpr int kBytes = 2;
  __device__ static constexpr int drow(int g, int r) { return 4 * g + r; }
  template <int N, bool kTrans>
  __device__ static fac_t load_fac(const io_t* M, int L, int g, int kmap) {
    fac_t f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int col = kmap == 0 ? 4 * g + s : drow(g, s);
      Slot<N> r(L), c(col);
      uint16_t b = 0;
      if (r.valid && c.valid && r.sub == c.sub) b = kTrans ? in_global(M)[c.idx + N * r.idx] : in_global(M)[r.idx + N * c.idx];
      f[s] = bits_to_bf16(b);
    }
    return f;
  }
  template <int kSteps = 4>
  __device__ static acc_t da(const fac_t& f, const acc_t& x) {
    bf16x4 hi, lo;
    split4(x, hi, lo);
    acc_t c = {0.f, 0.f, 0.f, 0.f};
    return mfma_bf16_k32(cat8(hi, lo), cat8(f, f), c);
  }
  template <int kSteps = 4>
  __device__ static acc_t db(const fac_t& f, const acc_t& x) {
    bf16x4 hi, lo;
    split4(x, hi, lo);
    acc_t c = {0.f, 0.f, 0.f, 0.f};
    return mfma_bf16_k32(cat8(f, f), cat8(hi, lo), c);
  }
  // first stage: x holds exact bf16 values widened to FP32
  template <int kSteps = 4>
  __device__ static acc_t da_in(const fac_t& f, const acc_t& x) {
    bf16x4 h;
#pragma unroll
    for (int e = 0; e < 4; ++e) h[e] = to_bf16(x[e]);
    acc_t c = {0.f, 0.f, 0.f, 0.f};
    return mfma_bf16_k16(h, f, c);
  }
};

// Waits until every vector-memory load of the wavefront has returned
// (s_waitcnt vmcnt(0)).  Called once after a kernel's factor loads: in a loop
// that requests the next tile's data ahead of the current tile's arithmetic,
// the first use of a factor register could otherwise be compiled as a full
// wait, which also waits for those requests in every iteration.
__device__ __forceinline__ void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// ---- lane-group <-> slab exchange (3-D) --------------------------------------------
//
// Before: lane group g, register (slab b, r) holds the element with row index
// i = drow(g, r) and slab b.  After: lane group G holds, in register
// (slab 4*g_old + rb, r), the element of row drow(g_old, r) and slab 4G + rb.
// permlane32_swap(x, y) exchanges x's upper 32 lanes with y's lower 32 lanes;
// permlane16_swap(x, y) exchanges x's odd 16-lane rows with y's even rows.
// Pairing registers whose slab differs in bit 3 (then bit 2) swaps lane bit 5
// (then 4) with that slab bit.

__device__ __forceinline__ void swap32(float& x, float& y) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap16(float& x, float& y) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap32(double& x, double& y) {
  uint64_t xb = __builtin_bit_cast(uint64_t, x), yb = __builtin_bit_cast(uint64_t, y);
  auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)xb, (uint32_t)yb, false, false);
  auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(xb >> 32), (uint32_t)(yb >> 32), false, false);
  x = __builtin_bit_cast(double, ((uint64_t)hi[0] << 32) | lo[0]);
  y = __builtin_bit_cast(double, ((uint64_t)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ void swap16(double& x, double& y) {
  uint64_t xb = __builtin_bit_cast(uint64_t, x), yb = __builtin_bit_cast(uint64_t, y);
  auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)xb, (uint32_t)yb, false, false);
  auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(xb >> 32), (uint32_t)(yb >> 32), false, false);
  x = __builtin_bit_cast(double, ((uint64_t)hi[0] << 32) | lo[0]);
  y = __builtin_bit_cast(double, ((uint64_t)hi[1] << 32) | lo[1]);
}

// Within one accumulator: lane group g, register r -> lane group r,
// register g (lane bit 5 trades with register bit 1, then lane bit 4 with
// register bit 0).  For an FP64 accumulator (rows g + 4r) this leaves rows
// 4g .. 4g + 3 in lane group g, i.e. four consecutive elements per lane.
template <typename V>
__device__ __forceinline__ void transpose_groups_regs(V& v) {
  auto a = v[0], b = v[1], c = v[2], d = v[3];
  swap32(a, c);
  swap32(b, d);
  swap16(a, b);
  swap16(c, d);
  v[0] = a;
  v[1] = b;
  v[2] = c;
  v[3] = d;
}

// The same exchange on an array whose logical slab b sits at t[H(b)].
template <int (*H)(int), typename V>
__device__ __forceinline__ void exchange_groups_slabs_at(V (&t)[16]) {
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      auto x = t[H(b)][r], y = t[H(b + 8)][r];
      swap32(x, y);
      t[H(b)][r] = x;
      t[H(b + 8)][r] = y;
    }
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    if (b & 4) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      auto x = t[H(b)][r], y = t[H(b + 4)][r];
      swap16(x, y);
      t[H(b)][r] = x;
      t[H(b + 4)][r] = y;
    }
  }
}

template <typename V>
__device__ __forceinline__ void exchange_groups_slabs(V (&t)[16]) {
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      auto x = t[b][r], y = t[b + 8][r];
      swap32(x, y);
      t[b][r] = x;
      t[b + 8][r] = y;
    }
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    if (b & 4) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      auto x = t[b][r], y = t[b + 4][r];
      swap16(x, y);
      t[b][r] = x;
      t[b + 4][r] = y;
    }
  }
}

}  // namespace kron
