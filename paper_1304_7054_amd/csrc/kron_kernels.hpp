// Per-tile routines of the batched Kronecker action (2-D and 3-D).
//
// 2-D (Section 2, (A (x) B) vec(X) = vec(B X A^T)).  In memory an operand is
// X(u, v) at u*n + v (u = column of the column-major matrix, the slow index;
// v = row, the fast index), and Y(i, j) = sum_{u,v} A(i, u) B(j, v) X(u, v).
//   load    lane (L, g) holds X(u = slot L, v = slots 4g..4g+3)
//   stage 1 contract v with B, data as MFMA operand A  -> rows u, column j
//   stage 2 contract u with A, data as MFMA operand A  -> rows j, column i
//   store   lane (L, g) holds Y(i = slot L, j = slots drow(g, 0..3))
//
// 3-D (Section 2.1; the library's (A (x) B (x) C) is the paper's K(C, B, A)).
// Element (a, b, c) at a*n^2 + b*n + c and
// Y(i, j, k) = sum A(i, a) B(j, b) C(k, c) X(a, b, c).
//   load    lane (L, g), slab b holds X(a = slot L, b, c = slots 4g..4g+3)
//   stage 1 contract c with C, data as operand A  -> rows a, column k   (per slab b)
//   stage 2 contract a with A, data as operand B  -> rows i, column k   (per slab b)
//   exchange lane groups <-> slabs                 -> slab i, slots b on (g, s)
//   stage 3 contract b with B, data as operand A  -> rows k, column j   (per slab i)
//   store   lane (L, g), slab i holds Y(i, j = slot L, k = slots drow(g, 0..3))
// Unlike the paper's Algorithm 1 there is no intermediate array in memory:
// all three mode products run on data held in registers.
#pragma once

#include "kron_tile.hpp"

namespace kron {

// ---- memory access of four elements ------------------------------------------------

template <typename io_t>
struct Mem;

template <>
struct Mem<float> {
  using acc = f32x4;
  static constexpr int kAlign = 16;
  __device__ static f32x4 load4(const float* p) { return __builtin_nontemporal_load(in_global(reinterpret_cast<const f32x4*>(p))); }
  __device__ static void store4(float* p, const f32x4& v) { __builtin_nontemporal_store(v, in_global(reinterpret_cast<f32x4*>(p))); }
  __device__ static float load1(const float* p) { return __builtin_nontemporal_load(in_global(p)); }
  __device__ static void store1(float* p, float v) { __builtin_nontemporal_store(v, in_global(p)); }
};

template <>
struct Mem<double> {
  using acc = f64x4;
  typedef double f64x2 __attribute__((ext_vector_type(2)));
  static constexpr int kAlign = 16;
  __device__ static f64x4 load4(const double* p) {
    f64x2 a = __builtin_nontemporal_load(in_global(reinterpret_cast<const f64x2*>(p)));
    f64x2 b = __builtin_nontemporal_load(in_global(reinterpret_cast<const f64x2*>(p + 2)));
    return f64x4{a[0], a[1], b[0], b[1]};
  }
  __device__ static void store4(double* p, const f64x4& v) {
    __builtin_nontemporal_store(f64x2{v[0], v[1]}, in_global(reinterpret_cast<f64x2*>(p)));
    __builtin_nontemporal_store(f64x2{v[2], v[3]}, in_global(reinterpret_cast<f64x2*>(p + 2)));
  }
  __device__ static double load1(const double* p) { return __builtin_nontemporal_load(in_global(p)); }
  __device__ static void store1(double* p, double v) { __builtin_nontemporal_store(v, in_global(p)); }
};

// bf16 storage: values are widened to FP32 on load and rounded to nearest even on store
template <>
struct Mem<uint16_t> {
  using acc = f32x4;
  static constexpr int kAlign = 8;
  __device__ static f32x4 load4(const uint16_t* p) {
    u16x4 b = __builtin_nontemporal_load(in_global(reinterpret_cast<const u16x4*>(p)));
    return f32x4{from_bf16(bits_to_bf16(b[0])), from_bf16(bits_to_bf16(b[1])), from_bf16(bits_to_bf16(b[2])),
                 from_bf16(bits_to_bf16(b[3]))};
  }
  __device__ static void store4(uint16_t* p, const f32x4& v) {
    u16x4 b = {bf16_to_bits(to_bf16(v[0])), bf16_to_bits(to_bf16(v[1])), bf16_to_bits(to_bf16(v[2])),
               bf16_to_bits(to_bf16(v[3]))};
    __builtin_nontemporal_store(b, in_global(reinterpret_cast<u16x4*>(p)));
  }
  __device__ static float load1(const uint16_t* p) { return from_bf16(bits_to_bf16(__builtin_nontemporal_load(in_global(p)))); }
  __device__ static void store1(uint16_t* p, float v) { __builtin_nontemporal_store(bf16_to_bits(to_bf16(v)), in_global(p)); }
};

template <typename V>
__device__ __forceinline__ bool all_finite(const V& v) {
  return __builtin_isfinite(v[0]) && __builtin_isfinite(v[1]) && __builtin_isfinite(v[2]) && __builtin_isfinite(v[3]);
}

// Output stores.  kBeta: the BLAS-style output update Y <- v + beta * Y of
// Section 3's interface, reading the old value at the address it writes, in
// the same lane, so the update needs no synchronisation.
template <bool kBeta, typename io_t, typename V, typename S>
__device__ __forceinline__ void put4(io_t* p, V v, S beta) {
  if constexpr (kBeta) {
    const V y = Mem<io_t>::load4(p);
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = v[r] + beta * y[r];
  }
  Mem<io_t>::store4(p, v);
}

template <bool kBeta, typename io_t, typename E, typename S>
__device__ __forceinline__ void put1(io_t* p, E v, S beta) {
  if constexpr (kBeta) v = v + beta * Mem<io_t>::load1(p);
  Mem<io_t>::store1(p, v);
}

// Offset (elements, relative to the tile's first operand) and packed-operand
// number contributed by one axis.  `stride` is the element stride of the axis
// inside an operand (n^2, n or 1); `opmul` its packed-operand multiplier
// (Q^2, Q or 1); E the operand size n^d.
template <int N, int E>
struct AxisPart {
  int off, op;
  bool valid;
  __device__ __forceinline__ AxisPart(int slot, int stride, int opmul) {
    Slot<N> s(slot);
    op = s.sub * opmul;
    off = op * E + s.idx * stride;
    valid = s.valid;
  }
};

// ---- 2-D tile ---------------------------------------------------------------------

// kTX: the operands are read transposed (op(X_p) = X_p^T of Section 2.2's
// 2-D interface): the slow and fast element strides of the loads swap, the
// packed-operand numbering does not, and the loads are scalar.
template <class M, int N, bool kVec, bool kTrans, bool kTX = false>
struct Tile2D {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  using fac_t = typename M::fac_t;
  static constexpr int Q = Geo<N>::Q;
  static constexpr int kOps = Q * Q;  // operands per tile
  static constexpr int E = N * N;     // elements per operand
  // FP64 accumulators hold rows g + 4r; with vector I/O they are regrouped
  // (rows 4g .. 4g + 3 per lane) before the store, so every lane writes 32
  // contiguous bytes instead of four scattered 8-byte values.
  static constexpr bool kRegroup = kVec && M::drow(0, 1) != 1;
  static constexpr bool kStoreVec = kVec;

  static constexpr bool kLoadVec = kVec && !kTX;

  fac_t fB, fA;
  AxisPart<N, E> pL;            // slot L on the slow axis (store)
  AxisPart<N, E> pLi;           // slot L on the slow axis (load; stride 1 when kTX)
  int offI[4], opI[4];          // load: fast slots 4g + s
  bool vI[4];
  int offO[4], opO[4];          // store: fast slots drow(g, r)
  bool vO[4];

  __device__ __forceinline__ Tile2D(const io_t* A, const io_t* B, int L, int g)
      : pL(L, N, Q), pLi(L, kTX ? 1 : N, Q) {
    fB = M::template load_fac<N, kTrans>(B, L, g, 0);
    fA = M::template load_fac<N, kTrans>(A, L, g, 1);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      AxisPart<N, E> pi(4 * g + s, kTX ? N : 1, 1), po(kRegroup ? 4 * g + s : M::drow(g, s), 1, 1);
      offI[s] = pi.off; opI[s] = pi.op; vI[s] = pi.valid;
      offO[s] = po.off; opO[s] = po.op; vO[s] = po.valid;
    }
  }

  // rem = operands from the tile's first one to the end of the batch (>= 1);
  // only >= 0 restricts the access to that one operand of the tile.
  __device__ static __forceinline__ bool take(int op, int64_t rem, int only) {
    return op < rem && (only < 0 || op == only);
  }

  __device__ __forceinline__ acc_t load(const io_t* Xt, int64_t rem, int only = -1) const {
    acc_t x;
    if constexpr (N == 16 && kLoadVec) {
      x = Mem<io_t>::load4(Xt + pLi.off + offI[0]);
    } else if constexpr (kLoadVec) {
      bool ok = pLi.valid && vI[0] && take(pLi.op + opI[0], rem, only);
      if (ok) x = Mem<io_t>::load4(Xt + pLi.off + offI[0]);
      else x = acc_t{0, 0, 0, 0};
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        bool ok = pLi.valid && vI[s] && take(pLi.op + opI[s], rem, only);
        x[s] = ok ? Mem<io_t>::load1(Xt + pLi.off + offI[s]) : 0;
      }
    }
    return x;
  }

  static constexpr int kS = Geo<N>::kSteps;
  __device__ __forceinline__ acc_t compute(const acc_t& x) const {
    return M::template da<kS>(fA, M::template da_in<kS>(fB, x));
  }

  template <bool kBeta = false, typename S = float>
  __device__ __forceinline__ void store(io_t* Yt, int64_t rem, const acc_t& y_in, int only = -1, S beta = S(0)) const {
    acc_t y = y_in;
    if constexpr (kRegroup) transpose_groups_regs(y);
    if constexpr (N == 16 && kStoreVec) {
      put4<kBeta>(Yt + pL.off + offO[0], y, beta);
    } else if constexpr (kStoreVec) {
      if (pL.valid && vO[0] && take(pL.op + opO[0], rem, only)) put4<kBeta>(Yt + pL.off + offO[0], y, beta);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (pL.valid && vO[r] && take(pL.op + opO[r], rem, only)) put1<kBeta>(Yt + pL.off + offO[r], y[r], beta);
    }
  }

  // Packed tiles (Q > 1): a NaN or Inf in one operand would reach its tile
  // neighbours through the zero blocks of the factor tiles (0 * Inf = NaN).
  // When a tile's result holds any non-finite value, it is redone one
  // operand at a time so that IEEE propagation stays inside each operand.
  template <bool kBeta = false, typename S = float>
  __device__ __forceinline__ void finish(const io_t* Xt, io_t* Yt, int64_t rem, const acc_t& y, S beta = S(0)) const {
    if constexpr (kOps > 1) {
      if (__any(!all_finite(y))) {
        const int last = rem < kOps ? (int)rem : kOps;
        for (int o = 0; o < last; ++o) store<kBeta>(Yt, rem, compute(load(Xt, rem, o)), o, beta);
        return;
      }
    }
    store<kBeta>(Yt, rem, y, -1, beta);
  }
};

// ---- 3-D tile ---------------------------------------------------------------------

template <class M, int N, bool kVec, bool kTrans, bool kContig = false>
struct Tile3D {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  using fac_t = typename M::fac_t;
  static constexpr int Q = Geo<N>::Q;
  static constexpr int kOps = Q * Q * Q;
  static constexpr int E = N * N * N;
  static constexpr bool kStoreVec = kVec && (kContig || M::drow(0, 1) == 1);

  fac_t fC, fA, fB;
  AxisPart<N, E> pLi;   // load: slot L on the slow axis a (kContig: on the middle axis b)
  AxisPart<N, E> pLo;   // store: slot L on the middle axis j
  int offI[4], opI[4];  // load: fast slots 4g + s
  bool vI[4];
  int offO[4], opO[4];  // store: fast slots drow(g, r)
  bool vO[4];

  __device__ __forceinline__ Tile3D(const io_t* A, const io_t* B, const io_t* C, int L, int g)
      : pLi(L, kContig ? N : N * N, kContig ? Q : Q * Q), pLo(L, N, Q) {
    fC = M::template load_fac<N, kTrans>(C, L, g, 0);
    if constexpr (kContig) {
      fB = M::template load_fac<N, kTrans>(B, L, g, 1);
      fA = M::template load_fac<N, kTrans>(A, L, g, 0);
    } else {
      fA = M::template load_fac<N, kTrans>(A, L, g, 1);
      fB = M::template load_fac<N, kTrans>(B, L, g, 0);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      AxisPart<N, E> pi(4 * g + s, 1, 1), po(kContig ? 4 * g + s : M::drow(g, s), 1, 1);
      offI[s] = pi.off; opI[s] = pi.op; vI[s] = pi.valid;
      offO[s] = po.off; opO[s] = po.op; vO[s] = po.valid;
    }
  }

  __device__ static __forceinline__ bool take(int op, int64_t rem, int only) {
    return op < rem && (only < 0 || op == only);
  }

  __device__ __forceinline__ void load_slab(const io_t* Xt, int64_t rem, int b, acc_t& v, int only = -1) const {
    // slab on the middle axis (kContig: on the slow axis)
    AxisPart<N, E> pS(b, kContig ? N * N : N, kContig ? Q * Q : Q);
    if constexpr (N == 16 && kVec) {
      v = Mem<io_t>::load4(Xt + pLi.off + pS.off + offI[0]);
    } else if constexpr (kVec) {
      bool ok = pS.valid && pLi.valid && vI[0] && take(pLi.op + pS.op + opI[0], rem, only);
      if (ok) v = Mem<io_t>::load4(Xt + pLi.off + pS.off + offI[0]);
      else v = acc_t{0, 0, 0, 0};
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        bool ok = pS.valid && pLi.valid && vI[s] && take(pLi.op + pS.op + opI[s], rem, only);
        v[s] = ok ? Mem<io_t>::load1(Xt + pLi.off + pS.off + offI[s]) : 0;
      }
    }
  }

  __device__ __forceinline__ void load(const io_t* Xt, int64_t rem, acc_t (&t)[16], int only = -1) const {
#pragma unroll
    for (int b = 0; b < 16; ++b) load_slab(Xt, rem, b, t[b], only);
  }

  // After exchange_groups_slabs, the value for output slab `o` and
  // contraction slots 4g + s sits in register [4 * g_old + s][r_old] where
  // (g_old, r_old) held row o before the exchange.
  __device__ __forceinline__ static void regather(const acc_t (&t)[16], int o, acc_t& z) {
    int gi = 0, ri = 0;
#pragma unroll
    for (int gg = 0; gg < 4; ++gg)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        if (M::drow(gg, rr) == o) { gi = gg; ri = rr; }
#pragma unroll
    for (int s = 0; s < 4; ++s) z[s] = t[4 * gi + s][ri];
  }

  static constexpr int kS = Geo<N>::kSteps;
  // slabs whose slot holds no element stay zero and are not computed
  __device__ static constexpr bool live(int slab) { return slot_live<N>(slab); }

  // Stages 1 and 2 touch one slab at a time.
  __device__ __forceinline__ void stage12(acc_t& v) const {
    if constexpr (kContig) {
      // slab a of X(a, b = slot L, c = slots 4g+s): contract c (rows b, column k), then b (rows k, column j)
      v = M::template da<kS>(fB, M::template da_in<kS>(fC, v));
    } else {
      // slab b of X(a = slot L, b, c = slots 4g+s): contract c (rows a, column k), then a (rows i, column k)
      v = M::template db<kS>(fA, M::template da_in<kS>(fC, v));
    }
  }

  // Position in t of the stage-3 result for output slab o while it is still
  // in the exchanged arrangement: output o = drow(g, r) is computed from the
  // four slabs 4g .. 4g + 3 alone, so it can be written back into slab 4g + r
  // of that same group (the identity for FP32, where drow(g, r) = 4g + r).
  __device__ static constexpr int home(int o) {
    int h = 0;
    for (int gg = 0; gg < 4; ++gg)
      for (int rr = 0; rr < 4; ++rr)
        if (M::drow(gg, rr) == o) h = 4 * gg + rr;
    return h;
  }

  // The third mode needs every slab: exchange lane groups and slabs, contract,
  // and (kContig) exchange back so that the result is stored in 1 KiB rows.
  __device__ __forceinline__ void stage3(acc_t (&t)[16]) const {
    exchange_groups_slabs(t);
    if constexpr (kContig && Q == 1) {
      // In place, one group of four slabs at a time (a 4-slab copy instead of
      // a second 16-slab array): the results of group g go to t[4g + r].
      // Packed tiles (Q > 1) keep the two-array form below, which the
      // compiler schedules with fewer spills there.
#pragma unroll
      for (int gg = 0; gg < 4; ++gg) {
        acc_t src[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) src[s] = t[4 * gg + s];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int k = M::drow(gg, rr);
          if (!live(k)) {
            t[4 * gg + rr] = acc_t{0, 0, 0, 0};
            continue;
          }
          acc_t z;
#pragma unroll
          for (int s = 0; s < 4; ++s) z[s] = src[s][rr];
          t[4 * gg + rr] = M::template db<kS>(fA, z);  // contract a: rows i, column j, slab k
        }
      }
      exchange_groups_slabs_at<home>(t);  // -> slab i, slots k on (g, s), still at home(k)
      // slab i = drow(g, r) takes element r of the results for slabs 4g + s,
      // which sit at home(4g + s): both sets are the same four registers
#pragma unroll
      for (int gg = 0; gg < 4; ++gg) {
        acc_t src[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) src[s] = t[home(4 * gg + s)];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          acc_t z;
#pragma unroll
          for (int s = 0; s < 4; ++s) z[s] = src[s][rr];
          t[M::drow(gg, rr)] = z;
        }
      }
    } else if constexpr (kContig) {
      acc_t u[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (!live(k)) {
          u[k] = acc_t{0, 0, 0, 0};
          continue;
        }
        acc_t z;
        regather(t, k, z);
        u[k] = M::template db<kS>(fA, z);  // contract a: rows i, column j, slab k
      }
      exchange_groups_slabs(u);  // -> slab i, slots k on (g, s)
#pragma unroll
      for (int i = 0; i < 16; ++i) regather(u, i, t[i]);
    } else {
      acc_t u[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (!live(i)) {
          u[i] = acc_t{0, 0, 0, 0};
          continue;
        }
        acc_t z;
        regather(t, i, z);
        u[i] = M::template da<kS>(fB, z);  // contract b: rows k, column j, slab i
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) t[i] = u[i];
    }
  }

  // t: loaded slabs in, results (slab i) out
  __device__ __forceinline__ void compute(acc_t (&t)[16]) const {
#pragma unroll
    for (int b = 0; b < 16; ++b)
      if (live(b)) stage12(t[b]);
    stage3(t);
  }

  template <bool kBeta = false, typename S = float>
  __device__ __forceinline__ void store_slab(io_t* Yt, int64_t rem, int i, const acc_t& v, int only = -1,
                                             S beta = S(0)) const {
    AxisPart<N, E> pS(i, N * N, Q * Q);  // slab on the slow axis
    if constexpr (N == 16 && kStoreVec) {
      put4<kBeta>(Yt + pS.off + pLo.off + offO[0], v, beta);
    } else if constexpr (kStoreVec) {
      if (pS.valid && pLo.valid && vO[0] && take(pS.op + pLo.op + opO[0], rem, only))
        put4<kBeta>(Yt + pS.off + pLo.off + offO[0], v, beta);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (pS.valid && pLo.valid && vO[r] && take(pS.op + pLo.op + opO[r], rem, only))
          put1<kBeta>(Yt + pS.off + pLo.off + offO[r], v[r], beta);
    }
  }

  template <bool kBeta = false, typename S = float>
  __device__ __forceinline__ void store(io_t* Yt, int64_t rem, const acc_t (&t)[16], int only = -1,
                                        S beta = S(0)) const {
#pragma unroll
    for (int i = 0; i < 16; ++i) store_slab<kBeta>(Yt, rem, i, t[i], only, beta);
  }

  // Same isolation rule as the 2-D tile: a packed tile whose result holds a
  // non-finite value is recomputed one operand at a time.
  template <bool kBeta = false, typename S = float>
  __device__ __forceinline__ void finish(const io_t* Xt, io_t* Yt, int64_t rem, acc_t (&t)[16], S beta = S(0)) const {
    if constexpr (kOps > 1) {
      bool fin = true;
#pragma unroll
      for (int i = 0; i < 16; ++i) fin = fin && all_finite(t[i]);
      if (__any(!fin)) {
        const int last = rem < kOps ? (int)rem : kOps;
        for (int o = 0; o < last; ++o) {
          load(Xt, rem, t, o);
          compute(t);
          store<kBeta>(Yt, rem, t, o, beta);
        }
        return;
      }
    }
    store<kBeta>(Yt, rem, t, -1, beta);
  }
};

// ---- persistent kernels ---------------------------------------------------------------
//
// 256-thread workgroups; every wavefront walks the tiles with a grid stride.
// The 2-D kernel keeps kTiles tiles in flight per wavefront.

constexpr int kBlock = 256;

template <class M, int N, bool kVec, bool kTrans, int kTiles>
__global__ __launch_bounds__(kBlock) void kron2d_kernel(const typename M::io_t* __restrict__ A,
                                                        const typename M::io_t* __restrict__ B,
                                                        const typename M::io_t* __restrict__ X,
                                                        typename M::io_t* __restrict__ Y, int64_t batch,
                                                        int64_t ntiles) {
  using T = Tile2D<M, N, kVec, kTrans>;
  using acc_t = typename M::acc_t;
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const T tile(A, B, L, g);
  for (int64_t base = wave * kTiles; base < ntiles; base += nwaves * kTiles) {
    acc_t x[kTiles];
#pragma unroll
    for (int j = 0; j < kTiles; ++j) {
      const int64_t t = base + j;
      if (t < ntiles) x[j] = tile.load(X + t * T::kOps * T::E, batch - t * T::kOps);
      else x[j] = acc_t{0, 0, 0, 0};
    }
#pragma unroll
    for (int j = 0; j < kTiles; ++j) x[j] = tile.compute(x[j]);
#pragma unroll
    for (int j = 0; j < kTiles; ++j) {
      const int64_t t = base + j;
      if (t < ntiles) tile.finish(X + t * T::kOps * T::E, Y + t * T::kOps * T::E, batch - t * T::kOps, x[j]);
    }
  }
}

// Loop structure of the 3-D kernel (the variant chosen per (mode, n)):
//   kPipe    the loads of a wavefront's next tile are issued before the
//            current tile is computed;
//   kWindow  > 0: slab loads are kept to a window of kWindow slabs in flight
//            and stages 1-2 run on each slab as it lands (scheduling barriers
//            keep the compiler from hoisting every load to the top).  Fewer
//            bytes in flight per wavefront keep HBM queues short.
// FP64 tiles hold twice the registers of FP32 ones; without a hint the
// compiler spends them all and one wavefront runs per SIMD, which leaves the
// slab loads of a single wavefront to cover HBM latency.  Two per SIMD fit
// without spilling once stage 3 runs in place, for n = 16 (packed and padded
// tiles carry more per-lane addressing and would spill).
template <class M, int N>
constexpr int kernel3d_waves() {
  return sizeof(typename M::io_t) == 8 && N == 16 ? 2 : 1;
}

template <class M, int N, bool kVec, bool kTrans, bool kPipe, bool kContig, int kWindow>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kernel3d_waves<M, N>()))) void kron3d_kernel(const typename M::io_t* __restrict__ A,
                                                        const typename M::io_t* __restrict__ B,
                                                        const typename M::io_t* __restrict__ C,
                                                        const typename M::io_t* __restrict__ X,
                                                        typename M::io_t* __restrict__ Y, int64_t batch,
                                                        int64_t ntiles) {
  using T = Tile3D<M, N, kVec, kTrans, kContig>;
  using acc_t = typename M::acc_t;
  constexpr int64_t kStep = (int64_t)T::kOps * T::E;
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const T tile(A, B, C, L, g);
  if constexpr (kWindow > 0) {
    // pre: the first kWindow slabs of the wavefront's next tile.  With kPipe
    // they are requested before the current tile's third stage, otherwise
    // after its stores.
    acc_t pre[kWindow];
    int64_t t = wave;
    if (t < ntiles) {
#pragma unroll
      for (int b = 0; b < kWindow; ++b) tile.load_slab(X + t * kStep, batch - t * T::kOps, b, pre[b]);
    }
    for (; t < ntiles; t += nwaves) {
      const typename M::io_t* Xt = X + t * kStep;
      const int64_t rem = batch - t * T::kOps;
      const int64_t tn = t + nwaves;
      acc_t v[16];
#pragma unroll
      for (int b = 0; b < kWindow; ++b) v[b] = pre[b];
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        __builtin_amdgcn_sched_barrier(0);
        if (T::live(b)) tile.stage12(v[b]);
        if (b + kWindow < 16) tile.load_slab(Xt, rem, b + kWindow, v[b + kWindow]);
      }
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (kPipe) {
        if (tn < ntiles) {
#pragma unroll
          for (int b = 0; b < kWindow; ++b) tile.load_slab(X + tn * kStep, batch - tn * T::kOps, b, pre[b]);
        }
      }
      tile.stage3(v);
      tile.finish(Xt, Y + t * kStep, rem, v);
      if constexpr (!kPipe) {
        if (tn < ntiles) {
#pragma unroll
          for (int b = 0; b < kWindow; ++b) tile.load_slab(X + tn * kStep, batch - tn * T::kOps, b, pre[b]);
        }
      }
    }
  } else if constexpr (kPipe) {
    int64_t t = wave;
    if (t >= ntiles) return;
    acc_t cur[16];
    tile.load(X + t * kStep, batch - t * T::kOps, cur);
    for (; t < ntiles; t += nwaves) {
      const int64_t tn = t + nwaves;
      acc_t nxt[16];
      if (tn < ntiles) tile.load(X + tn * kStep, batch - tn * T::kOps, nxt);
      tile.compute(cur);
      tile.finish(X + t * kStep, Y + t * kStep, batch - t * T::kOps, cur);
#pragma unroll
      for (int i = 0; i < 16; ++i) cur[i] = nxt[i];
    }
  } else {
    for (int64_t t = wave; t < ntiles; t += nwaves) {
      acc_t v[16];
      tile.load(X + t * kStep, batch - t * T::kOps, v);
      tile.compute(v);
      tile.finish(X + t * kStep, Y + t * kStep, batch - t * T::kOps, v);
    }
  }
}

// The extended interface's cases that the plain kernels do not cover
// (Section 2.2's update Y_p <- K(op(X_p)) + beta Y_p; alpha and op on the
// factors are folded into the factors by the caller):
//   kBeta  beta != 0: every lane reads the old output where it stores;
//   kTX    (2-D) the operands are read transposed.
// The tile loops of the plain kernels: 2-D keeps four tiles in flight per
// wavefront, 3-D walks contiguous 1 KiB rows.  FP32 and FP64 storage only
// (io_t is the arithmetic type).
template <class M, int N, bool kVec, int kDim, bool kBeta, bool kTX>
__global__ __launch_bounds__(kBlock) void kron_ex_kernel(const typename M::io_t* __restrict__ A,
                                                         const typename M::io_t* __restrict__ B,
                                                         const typename M::io_t* __restrict__ C,
                                                         const typename M::io_t* __restrict__ X,
                                                         typename M::io_t* __restrict__ Y, int64_t batch,
                                                         int64_t ntiles, typename M::io_t beta) {
  static_assert(kDim == 2 || !kTX, "op on the operands exists in 2-D only");
  using acc_t = typename M::acc_t;
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  if constexpr (kDim == 2) {
    using T = Tile2D<M, N, kVec, false, kTX>;
    constexpr int kTiles = 4;
    const T tile(A, B, L, g);
    for (int64_t base = wave * kTiles; base < ntiles; base += nwaves * kTiles) {
      acc_t x[kTiles];
#pragma unroll
      for (int j = 0; j < kTiles; ++j) {
        const int64_t t = base + j;
        if (t < ntiles) x[j] = tile.load(X + t * T::kOps * T::E, batch - t * T::kOps);
        else x[j] = acc_t{0, 0, 0, 0};
      }
#pragma unroll
      for (int j = 0; j < kTiles; ++j) x[j] = tile.compute(x[j]);
#pragma unroll
      for (int j = 0; j < kTiles; ++j) {
        const int64_t t = base + j;
        if (t < ntiles)
          tile.template finish<kBeta>(X + t * T::kOps * T::E, Y + t * T::kOps * T::E, batch - t * T::kOps, x[j],
                                      beta);
      }
    }
  } else {
    using T = Tile3D<M, N, kVec, false, true>;
    constexpr int64_t kStep = (int64_t)T::kOps * T::E;
    const T tile(A, B, C, L, g);
    for (int64_t t = wave; t < ntiles; t += nwaves) {
      acc_t v[16];
      tile.load(X + t * kStep, batch - t * T::kOps, v);
      tile.compute(v);
      tile.template finish<kBeta>(X + t * kStep, Y + t * kStep, batch - t * T::kOps, v, beta);
    }
  }
}

// n = 16 (one operand per tile): the result of tile t is written one slab
// at a time, and between two slab stores the wavefront runs stages 1-2 on a
// slab of its next tile and requests the slab kWindow further on.  Reads and
// writes then alternate per 1 KiB row instead of a whole tile of each in a
// burst; contiguous-row stage order, so every access is one 1 KiB row.
// At most 16 + kWindow slabs are live at once (a result slab dies as it is
// stored): with 4-byte elements that fits three wavefronts per SIMD, with
// 8-byte ones two (stage 3 in place).
template <class M>
constexpr int stream_waves() {
  return sizeof(typename M::io_t) == 8 ? 2 : 3;
}

template <class M, bool kTrans, int kWindow>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(stream_waves<M>()))) void kron3d_stream_kernel(const typename M::io_t* __restrict__ A,
                                                               const typename M::io_t* __restrict__ B,
                                                               const typename M::io_t* __restrict__ C,
                                                               const typename M::io_t* __restrict__ X,
                                                               typename M::io_t* __restrict__ Y, int64_t ntiles) {
  using T = Tile3D<M, 16, true, kTrans, true>;
  using acc_t = typename M::acc_t;
  static_assert(T::kOps == 1, "one operand per tile");
  constexpr int64_t kStep = T::E;
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const T tile(A, B, C, L, g);
  int64_t t = wave;
  if (t >= ntiles) return;
  acc_t v[16], nx[16];
  {
    const typename M::io_t* Xt = X + t * kStep;
#pragma unroll
    for (int b = 0; b < kWindow; ++b) tile.load_slab(Xt, 1, b, v[b]);
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      __builtin_amdgcn_sched_barrier(0);
      tile.stage12(v[b]);
      if (b + kWindow < 16) tile.load_slab(Xt, 1, b + kWindow, v[b + kWindow]);
    }
    __builtin_amdgcn_sched_barrier(0);
    tile.stage3(v);
  }
  for (;;) {
    typename M::io_t* Yt = Y + t * kStep;
    const int64_t tn = t + nwaves;
    if (tn >= ntiles) {
      tile.store(Yt, 1, v);
      return;
    }
    const typename M::io_t* Xn = X + tn * kStep;
#pragma unroll
    for (int b = 0; b < kWindow; ++b) tile.load_slab(Xn, 1, b, nx[b]);
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      __builtin_amdgcn_sched_barrier(0);
      tile.store_slab(Yt, 1, b, v[b]);
      tile.stage12(nx[b]);
      if (b + kWindow < 16) tile.load_slab(Xn, 1, b + kWindow, nx[b + kWindow]);
    }
    __builtin_amdgcn_sched_barrier(0);
    tile.stage3(nx);
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = nx[b];
    t = tn;
  }
}

}  // namespace kron
