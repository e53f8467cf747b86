// LDS-staged tile I/O for the sizes whose tiles do not map onto 16-byte rows
// (every n except 16): packed tiles (n <= 8) and padded ones (9 <= n <= 15).
//
// A tile's operands are consecutive in memory (tile t holds operands
// t*kOps .. t*kOps + kOps - 1, packed back to back), so the wavefront copies
// the whole run, min(rem, kOps) * n^d elements, into its own LDS slice with
// coalesced 4-element loads, zero-fills the rest of the slice for a ragged
// last tile, and then reads its MFMA operand slots out of LDS: per lane one
// offset per row-group slot, plus a compile-time offset per slab; slots that
// hold no element read a zero cell.  Results go the opposite way.  Only the
// wavefront that owns a slice touches it, so wavefront-scope fences order
// the phases; no workgroup barrier is needed.
#pragma once

#include "kron_kernels.hpp"

namespace kron {

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// element in memory -> compute type (bf16 bits -> FP32; FP32 and FP64 as they are)
template <typename io_t>
__device__ __forceinline__ auto widen(io_t v) {
  if constexpr (sizeof(io_t) == 2) return from_bf16(bits_to_bf16(v));
  else return v;
}

template <typename io_t, typename T>
__device__ __forceinline__ io_t narrow(T v) {
  if constexpr (sizeof(io_t) == 2) return bf16_to_bits(to_bf16((float)v));
  else return (io_t)v;
}

// Copy `count` consecutive elements from global memory into an LDS slice.
template <typename io_t>
__device__ __forceinline__ void copy_in(const io_t* __restrict__ src, io_t* lds, int count, int lane) {
  const bool vec = ((reinterpret_cast<uintptr_t>(src) % Mem<io_t>::kAlign) == 0) &&
                   ((reinterpret_cast<uintptr_t>(lds) % 16) == 0) && (count % 4 == 0);
  if (vec) {
    for (int i = lane * 4; i < count; i += 256) {
      if constexpr (sizeof(io_t) == 4) {
        *reinterpret_cast<f32x4*>(lds + i) = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(src + i));
      } else if constexpr (sizeof(io_t) == 8) {
        typedef double f64x2 __attribute__((ext_vector_type(2)));
        *reinterpret_cast<f64x2*>(lds + i) = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(src + i));
        *reinterpret_cast<f64x2*>(lds + i + 2) = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(src + i + 2));
      } else {
        *reinterpret_cast<u16x4*>(lds + i) = __builtin_nontemporal_load(reinterpret_cast<const u16x4*>(src + i));
      }
    }
  } else {
    for (int i = lane; i < count; i += 64) lds[i] = __builtin_nontemporal_load(src + i);
  }
}

template <typename io_t>
__device__ __forceinline__ void zero_fill(io_t* lds, int from, int to, int lane) {
  for (int i = from + lane; i < to; i += 64) lds[i] = io_t(0);
}

template <typename io_t>
__device__ __forceinline__ void copy_out(io_t* __restrict__ dst, const io_t* lds, int count, int lane) {
  const bool vec = ((reinterpret_cast<uintptr_t>(dst) % Mem<io_t>::kAlign) == 0) &&
                   ((reinterpret_cast<uintptr_t>(lds) % 16) == 0) && (count % 4 == 0);
  if (vec) {
    for (int i = lane * 4; i < count; i += 256) {
      if constexpr (sizeof(io_t) == 4) {
        __builtin_nontemporal_store(*reinterpret_cast<const f32x4*>(lds + i), reinterpret_cast<f32x4*>(dst + i));
      } else if constexpr (sizeof(io_t) == 8) {
        typedef double f64x2 __attribute__((ext_vector_type(2)));
        __builtin_nontemporal_store(*reinterpret_cast<const f64x2*>(lds + i), reinterpret_cast<f64x2*>(dst + i));
        __builtin_nontemporal_store(*reinterpret_cast<const f64x2*>(lds + i + 2), reinterpret_cast<f64x2*>(dst + i + 2));
      } else {
        __builtin_nontemporal_store(*reinterpret_cast<const u16x4*>(lds + i), reinterpret_cast<u16x4*>(dst + i));
      }
    }
  } else {
    for (int i = lane; i < count; i += 64) __builtin_nontemporal_store(lds[i], dst + i);
  }
}

// Element offsets of a tile's slots (memory axes 0 slow, 1, 2 fast).
template <int N, int Dim>
struct TileGeom {
  static constexpr int Q = Geo<N>::Q;
  static constexpr int E = Dim == 3 ? N * N * N : N * N;
  __device__ static constexpr int stride(int ax) {
    return Dim == 3 ? (ax == 0 ? N * N : ax == 1 ? N : 1) : (ax == 0 ? N : 1);
  }
  __device__ static constexpr int opmul(int ax) {
    return Dim == 3 ? (ax == 0 ? Q * Q : ax == 1 ? Q : 1) : (ax == 0 ? Q : 1);
  }
};

// Per-lane part of the slot offsets: `base[s]` (0 for a slot that holds no
// element, whose value is then replaced by 0) plus a compile-time slab part,
// so that every LDS access is one address register + an immediate offset.
template <int N, int Dim>
struct LaneSlots {
  using G = TileGeom<N, Dim>;
  int base[4];
  bool ok[4];
  __device__ __forceinline__ LaneSlots(int L, int lax, int g, int gax, bool drow64) {
    AxisPart<N, G::E> pl(L, G::stride(lax), G::opmul(lax));
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      AxisPart<N, G::E> pg(drow64 ? g + 4 * s : 4 * g + s, G::stride(gax), G::opmul(gax));
      ok[s] = pl.valid && pg.valid;
      base[s] = ok[s] ? pl.off + pg.off : 0;
    }
  }
};

// ---- 3-D (slabs on the slow axis, L on the middle axis, row-group slots
// on the fast axis, for both X and Y: the contiguous-row stage order) --------

template <class M, int N, bool kTrans>
struct Staged3D {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  using Tile = Tile3D<M, N, false, kTrans, true>;
  using G = TileGeom<N, 3>;
  static constexpr int Q = Geo<N>::Q;
  static constexpr int kOps = Q * Q * Q;
  static constexpr int E = G::E;
  static constexpr int kElems = kOps * E;
  static constexpr int kSlice = (kElems + 7) / 8 * 8;

  Tile tile;
  LaneSlots<N, 3> ls;

  __device__ __forceinline__ Staged3D(const io_t* A, const io_t* B, const io_t* C, int L, int g)
      : tile(A, B, C, L, g), ls(L, 1, g, 2, false) {}

  __device__ __forceinline__ acc_t read(const io_t* lds, int a) const {
    AxisPart<N, E> ps(a, G::stride(0), G::opmul(0));
    acc_t v = acc_t{0, 0, 0, 0};
    if (!ps.valid) return v;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const auto x = widen(lds[ls.base[s] + ps.off]);
      v[s] = ls.ok[s] ? x : decltype(x)(0);
    }
    return v;
  }

  __device__ __forceinline__ void write(io_t* lds, int i, const acc_t& v) const {
    AxisPart<N, E> ps(i, G::stride(0), G::opmul(0));
    if (!ps.valid) return;
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (ls.ok[s]) lds[ls.base[s] + ps.off] = narrow<io_t>(v[s]);
  }
};

// One tile through an LDS slice of at least S::kSlice elements.  Packed
// tiles (several operands) whose result holds a non-finite value are redone
// one operand at a time: the slice is zeroed, only operand o is copied in (at
// its own place), the same code runs, and only operand o is copied out, so
// IEEE propagation stays inside operand o.
template <class S>
__device__ __forceinline__ void staged3d_tile(const S& st, typename S::io_t* lds, const typename S::io_t* Xt,
                                              typename S::io_t* Yt, int64_t rem, int l) {
  using acc_t = typename S::acc_t;
  const int nops = (int)(rem < S::kOps ? rem : S::kOps);
  for (int o = -1;;) {
    // o < 0: the whole tile; o >= 0: operand o alone
    const int first = o < 0 ? 0 : o * S::E;
    const int count = o < 0 ? nops * S::E : S::E;
    wave_sync_lds();  // the previous copy-out has read the slice
    if (o >= 0) zero_fill(lds, 0, S::kElems, l);
    else zero_fill(lds, count, S::kElems, l);
    wave_sync_lds();
    copy_in(Xt + first, lds + first, count, l);
    wave_sync_lds();
    acc_t v[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      v[a] = st.read(lds, a);
      if (S::Tile::live(a)) st.tile.stage12(v[a]);
    }
    st.tile.stage3(v);
    if constexpr (S::kOps > 1) {
      if (o < 0) {
        bool fin = true;
#pragma unroll
        for (int i = 0; i < 16; ++i) fin = fin && all_finite(v[i]);
        if (__any(!fin)) {
          o = 0;
          continue;
        }
      }
    }
    wave_sync_lds();  // every lane has read its slots
#pragma unroll
    for (int i = 0; i < 16; ++i) st.write(lds, i, v[i]);
    wave_sync_lds();
    copy_out(Yt + first, lds + first, count, l);
    if (o < 0 || ++o >= nops) break;
  }
}

template <class M, int N, bool kTrans>
__global__ __launch_bounds__(kBlock) void kron3d_staged_kernel(const typename M::io_t* __restrict__ A,
                                                               const typename M::io_t* __restrict__ B,
                                                               const typename M::io_t* __restrict__ C,
                                                               const typename M::io_t* __restrict__ X,
                                                               typename M::io_t* __restrict__ Y, int64_t batch,
                                                               int64_t ntiles) {
  using S = Staged3D<M, N, kTrans>;
  using io_t = typename M::io_t;
  __shared__ __attribute__((aligned(16))) io_t slices[kBlock / kWave][S::kSlice];
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  io_t* lds = slices[threadIdx.x >> 6];
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const S st(A, B, C, L, g);
  for (int64_t t = wave; t < ntiles; t += nwaves)
    staged3d_tile(st, lds, X + t * S::kElems, Y + t * S::kElems, batch - t * S::kOps, l);
}

// ---- 2-D (X: L on the slow axis, slots 4g + s on the fast axis; Y: L on the
// slow axis, slots drow(g, r) on the fast axis) -------------------------------

template <class M, int N, bool kTrans>
struct Staged2D {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  using Tile = Tile2D<M, N, false, kTrans>;
  using G = TileGeom<N, 2>;
  static constexpr int Q = Geo<N>::Q;
  static constexpr int kOps = Q * Q;
  static constexpr int E = G::E;
  static constexpr int kElems = kOps * E;
  static constexpr int kSlice = (kElems + 7) / 8 * 8;

  Tile tile;
  LaneSlots<N, 2> in, out;

  __device__ __forceinline__ Staged2D(const io_t* A, const io_t* B, int L, int g)
      : tile(A, B, L, g), in(L, 0, g, 1, false), out(L, 0, g, 1, M::drow(0, 1) != 1) {}

  __device__ __forceinline__ acc_t read(const io_t* lds) const {
    acc_t v;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const auto x = widen(lds[in.base[s]]);
      v[s] = in.ok[s] ? x : decltype(x)(0);
    }
    return v;
  }

  __device__ __forceinline__ void write(io_t* lds, const acc_t& v) const {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (out.ok[r]) lds[out.base[r]] = narrow<io_t>(v[r]);
  }
};

// kT consecutive tiles (from tile t0, at most `last` - t0 of them) through
// kT LDS slices of S::kSlice elements each; a packed tile with a non-finite
// result is redone per operand as in 3-D.
template <class S, int kT>
__device__ __forceinline__ void staged2d_tiles(const S& st, typename S::io_t* slices, const typename S::io_t* X,
                                               typename S::io_t* Y, int64_t t0, int64_t last, int64_t batch,
                                               int l) {
  using io_t = typename S::io_t;
  using acc_t = typename S::acc_t;
  int nops[kT];
#pragma unroll
  for (int j = 0; j < kT; ++j) {
    const int64_t t = t0 + j;
    const int64_t rem = t < last ? batch - t * S::kOps : 0;
    nops[j] = (int)(rem < S::kOps ? rem : S::kOps);
  }
  wave_sync_lds();
#pragma unroll
  for (int j = 0; j < kT; ++j) zero_fill(slices + j * S::kSlice, nops[j] * S::E, S::kElems, l);
#pragma unroll
  for (int j = 0; j < kT; ++j)
    if (nops[j] > 0) copy_in(X + (t0 + j) * S::kElems, slices + j * S::kSlice, nops[j] * S::E, l);
  wave_sync_lds();
  acc_t v[kT];
#pragma unroll
  for (int j = 0; j < kT; ++j) v[j] = st.tile.compute(st.read(slices + j * S::kSlice));
  bool bad[kT];
#pragma unroll
  for (int j = 0; j < kT; ++j) bad[j] = S::kOps > 1 && nops[j] > 0 && __any(!all_finite(v[j]));
  wave_sync_lds();
#pragma unroll
  for (int j = 0; j < kT; ++j)
    if (!bad[j]) st.write(slices + j * S::kSlice, v[j]);
  wave_sync_lds();
#pragma unroll
  for (int j = 0; j < kT; ++j)
    if (nops[j] > 0 && !bad[j]) copy_out(Y + (t0 + j) * S::kElems, slices + j * S::kSlice, nops[j] * S::E, l);
  if constexpr (S::kOps > 1) {
    for (int j = 0; j < kT; ++j) {
      if (!bad[j]) continue;
      io_t* sl = slices + j * S::kSlice;
      const io_t* Xt = X + (t0 + j) * S::kElems;
      io_t* Yt = Y + (t0 + j) * S::kElems;
      // this tile's results were not written back: redo it operand by operand
      for (int o = 0; o < nops[j]; ++o) {
        wave_sync_lds();
        zero_fill(sl, 0, S::kElems, l);
        wave_sync_lds();
        copy_in(Xt + o * S::E, sl + o * S::E, S::E, l);
        wave_sync_lds();
        const acc_t y = st.tile.compute(st.read(sl));
        wave_sync_lds();
        st.write(sl, y);
        wave_sync_lds();
        copy_out(Yt + o * S::E, sl + o * S::E, S::E, l);
      }
    }
  }
}

template <class M, int N, bool kTrans>
__global__ __launch_bounds__(kBlock) void kron2d_staged_kernel(const typename M::io_t* __restrict__ A,
                                                               const typename M::io_t* __restrict__ B,
                                                               const typename M::io_t* __restrict__ X,
                                                               typename M::io_t* __restrict__ Y, int64_t batch,
                                                               int64_t ntiles) {
  using S = Staged2D<M, N, kTrans>;
  using io_t = typename M::io_t;
  constexpr int kT = 4;
  __shared__ __attribute__((aligned(16))) io_t slices[kBlock / kWave][kT * S::kSlice];
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  io_t* mine = slices[threadIdx.x >> 6];
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const S st(A, B, L, g);
  for (int64_t base = wave * kT; base < ntiles; base += nwaves * kT)
    staged2d_tiles<S, kT>(st, mine, X, Y, base, ntiles, batch, l);
}

}  // namespace kron
