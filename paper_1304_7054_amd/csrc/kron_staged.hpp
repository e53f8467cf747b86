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

// Copies between global memory and an LDS slice.  A slice is placed at the
// same offset modulo 16 bytes as the global run it receives (stage_base), so
// both sides of the copy are vector-aligned for any tile size and start:
// a scalar head, 16-byte vectors, a scalar tail.  Each lane issues a batch of
// loads before it writes any of them to LDS, so a wavefront has several
// requests in flight instead of one round trip per element group.  When the
// two sides still differ modulo 16 bytes (an output array aligned unlike the
// input), the copy goes element by element, also in batches.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kStagePad = 8;  // spare elements per slice for the alignment shift

template <typename io_t>
__device__ __forceinline__ io_t* stage_base(io_t* lds, const io_t* src) {
  return lds + (int)((reinterpret_cast<uintptr_t>(src) & 15) / sizeof(io_t));
}

template <typename T, int kB>
__device__ __forceinline__ void batched_in(const T* __restrict__ src, T* lds, int n, int lane) {
  for (int b = 0; b < n; b += 64 * kB) {
    T r[kB];
#pragma unroll
    for (int k = 0; k < kB; ++k) {
      const int i = b + 64 * k + lane;
      if (i < n) r[k] = __builtin_nontemporal_load(in_global(src) + i);
    }
#pragma unroll
    for (int k = 0; k < kB; ++k) {
      const int i = b + 64 * k + lane;
      if (i < n) in_lds(lds)[i] = r[k];
    }
  }
}

template <typename T, int kB>
__device__ __forceinline__ void batched_out(T* __restrict__ dst, const T* lds, int n, int lane) {
  for (int b = 0; b < n; b += 64 * kB) {
    T r[kB];
#pragma unroll
    for (int k = 0; k < kB; ++k) {
      const int i = b + 64 * k + lane;
      if (i < n) r[k] = in_lds(lds)[i];
    }
#pragma unroll
    for (int k = 0; k < kB; ++k) {
      const int i = b + 64 * k + lane;
      if (i < n) __builtin_nontemporal_store(r[k], in_global(dst) + i);
    }
  }
}

// elements before `p` reaches a 16-byte boundary (at most count)
template <typename io_t>
__device__ __forceinline__ int head_elems(const io_t* p, int count) {
  const int h = (int)(((16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15) / sizeof(io_t));
  return h < count ? h : count;
}

template <typename io_t>
__device__ __forceinline__ bool same_phase16(const void* a, const void* b) {
  return ((reinterpret_cast<uintptr_t>(a) ^ reinterpret_cast<uintptr_t>(b)) & 15) == 0;
}

// Copy `count` consecutive elements from global memory into an LDS slice.
template <typename io_t>
__device__ __forceinline__ void copy_in(const io_t* __restrict__ src, io_t* lds, int count, int lane) {
  constexpr int V = 16 / sizeof(io_t);
  if (!same_phase16<io_t>(src, lds)) {
    batched_in<io_t, 16>(src, lds, count, lane);
    return;
  }
  const int head = head_elems(src, count);
  if (lane < head) in_lds(lds)[lane] = __builtin_nontemporal_load(in_global(src) + lane);
  const int nv = (count - head) / V;
  batched_in<u32x4, 8>(reinterpret_cast<const u32x4*>(src + head), reinterpret_cast<u32x4*>(lds + head), nv, lane);
  const int done = head + nv * V;
  if (lane < count - done) in_lds(lds)[done + lane] = __builtin_nontemporal_load(in_global(src) + done + lane);
}

template <typename io_t>
__device__ __forceinline__ void zero_fill(io_t* lds, int from, int to, int lane) {
  for (int i = from + lane; i < to; i += 64) in_lds(lds)[i] = io_t(0);
}

// Copy `count` consecutive elements from an LDS slice to global memory.
template <typename io_t>
__device__ __forceinline__ void copy_out(io_t* __restrict__ dst, const io_t* lds, int count, int lane) {
  constexpr int V = 16 / sizeof(io_t);
  if (!same_phase16<io_t>(dst, lds)) {
    batched_out<io_t, 16>(dst, lds, count, lane);
    return;
  }
  const int head = head_elems(dst, count);
  if (lane < head) __builtin_nontemporal_store(in_lds(lds)[lane], in_global(dst) + lane);
  const int nv = (count - head) / V;
  batched_out<u32x4, 8>(reinterpret_cast<u32x4*>(dst + head), reinterpret_cast<const u32x4*>(lds + head), nv, lane);
  const int done = head + nv * V;
  if (lane < count - done) __builtin_nontemporal_store(in_lds(lds)[done + lane], in_global(dst) + done + lane);
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
  static constexpr int kSlice = (kElems + kStagePad + 7) / 8 * 8;

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
      const auto x = widen(in_lds(lds)[ls.base[s] + ps.off]);
      v[s] = ls.ok[s] ? x : decltype(x)(0);
    }
    return v;
  }

  __device__ __forceinline__ void write(io_t* lds, int i, const acc_t& v) const {
    AxisPart<N, E> ps(i, G::stride(0), G::opmul(0));
    if (!ps.valid) return;
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (ls.ok[s]) in_lds(lds)[ls.base[s] + ps.off] = narrow<io_t>(v[s]);
  }
};

// Prefetch of a run of operands into registers: the run's head elements
// (up to the first 16-byte boundary), its first kPre 16-byte vectors per lane
// and its tail elements are loaded by issue(); commit() writes them into an
// LDS slice placed at the run's 16-byte phase (stage_base) and copies any
// vectors beyond the first 64 * kPre directly.  Issued for the next tile
// before the current one is computed, the loads overlap that work.
template <typename io_t, int kMaxElems>
struct RunPrefetch {
  static constexpr int V = 16 / (int)sizeof(io_t);
  static constexpr int kAll = (kMaxElems / V + 63) / 64;
  static constexpr int kPre = kAll < 8 ? kAll : 8;
  u32x4 r[kPre];
  io_t hv, tv;
  const io_t* src;
  int count, head, nv;

  __device__ __forceinline__ void issue(const io_t* src_, int count_, int lane) {
    src = src_;
    count = count_;
    head = head_elems(src, count);
    nv = (count - head) / V;
    const u32x4* s4 = reinterpret_cast<const u32x4*>(src + head);
    if (lane < head) hv = __builtin_nontemporal_load(in_global(src) + lane);
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
      const int i = lane + 64 * k;
      if (i < nv) r[k] = __builtin_nontemporal_load(in_global(s4) + i);
    }
    const int done = head + nv * V;
    if (lane < count - done) tv = __builtin_nontemporal_load(in_global(src) + done + lane);
  }

  // lds: the slice base for this run (stage_base(slice, src))
  __device__ __forceinline__ void commit(io_t* lds, int lane) const {
    u32x4* d4 = reinterpret_cast<u32x4*>(lds + head);
    if (lane < head) in_lds(lds)[lane] = hv;
#pragma unroll
    for (int k = 0; k < kPre; ++k) {
      const int i = lane + 64 * k;
      if (i < nv) in_lds(d4)[i] = r[k];
    }
    if constexpr (kAll > kPre) {
      const u32x4* s4 = reinterpret_cast<const u32x4*>(src + head);
      batched_in<u32x4, 8>(s4 + 64 * kPre, d4 + 64 * kPre, nv - 64 * kPre, lane);
    }
    const int done = head + nv * V;
    if (lane < count - done) in_lds(lds)[done + lane] = tv;
  }
};

// Results of a tile (or span) left in an LDS slice, copied out later.  With
// two slices per wavefront the copy-out of tile t is issued after tile
// t + 1's prefetched operands are committed to the other slice: the commit
// waits for those loads, and one counter covers both loads and stores here,
// so stores issued just before it would be waited for as well.  Issued after
// it, they complete while tile t + 1 is computed.
template <typename io_t>
struct Pending {
  io_t* dst = nullptr;
  const io_t* src = nullptr;
  int count = 0;

  __device__ __forceinline__ void hold(io_t* dst_, const io_t* src_, int count_) {
    dst = dst_;
    src = src_;
    count = count_;
  }
  __device__ __forceinline__ void write(int lane) {
    if (count > 0) copy_out(dst, src, count, lane);
    count = 0;
  }
};

// Two slices per wavefront when both fit in LDS at four wavefronts per SIMD
// (16 per CU, 160 KiB of LDS), one otherwise.
template <int kSliceBytes>
constexpr int stage_buffers() {
  return 2 * kSliceBytes * 16 <= 160 * 1024 ? 2 : 1;
}

// One tile through an LDS slice of S::kSlice elements (16-byte aligned).
// Packed tiles (several operands) whose result holds a non-finite value are
// redone one operand at a time: the slice is zeroed, only operand o is copied
// in (at its own place), the same code runs, and only operand o is copied
// out, so IEEE propagation stays inside operand o.
template <class S>
__device__ __forceinline__ void staged3d_tile(const S& st, typename S::io_t* slice, const typename S::io_t* Xt,
                                              typename S::io_t* Yt, int64_t rem, int l) {
  using acc_t = typename S::acc_t;
  typename S::io_t* lds = stage_base(slice, Xt);
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

// One tile of a prefetched sequence: its prefetched operands are committed
// to `slice`, then (kDefer) the previous tile's results, left in the
// wavefront's other slice, are copied out, the next tile's operands
// requested, this tile computed, and its results left in `slice` and held in
// `po`.  Without kDefer (one slice) the results are copied out at once.  A
// packed tile with a non-finite result is redone one operand at a time as
// in staged3d_tile, each operand written out at once.
template <bool kDefer, class S, class P>
__device__ __forceinline__ void staged3d_step(const S& st, typename S::io_t* slice, const typename S::io_t* Xt,
                                              typename S::io_t* Yt, int64_t rem, int l, P& pf,
                                              Pending<typename S::io_t>& po, const typename S::io_t* Xnext,
                                              int64_t rem_next) {
  using acc_t = typename S::acc_t;
  typename S::io_t* lds = stage_base(slice, Xt);
  const int nops = (int)(rem < S::kOps ? rem : S::kOps);
  for (int o = -1;;) {
    // o < 0: the whole tile; o >= 0: operand o alone
    const int first = o < 0 ? 0 : o * S::E;
    const int count = o < 0 ? nops * S::E : S::E;
    wave_sync_lds();  // this slice's last copy-out has read it
    if (o >= 0) zero_fill(lds, 0, S::kElems, l);
    else zero_fill(lds, count, S::kElems, l);
    if (o < 0) {
      pf.commit(lds, l);
      if constexpr (kDefer) po.write(l);
    } else {
      wave_sync_lds();
      copy_in(Xt + first, lds + first, count, l);
    }
    wave_sync_lds();
    if (o < 0 && Xnext) pf.issue(Xnext, (int)(rem_next < S::kOps ? rem_next : S::kOps) * S::E, l);
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
    if (kDefer && o < 0) {
      po.hold(Yt, lds, count);
      break;
    }
    wave_sync_lds();
    copy_out(Yt + first, lds + first, count, l);
    if (o < 0 || ++o >= nops) break;
  }
}

// Waves per SIMD the 3-D staged kernel is held to: single-operand tiles for
// n = 9 .. 13 fit four (their LDS slices are small); the larger tiles are
// limited by LDS to two anyway and are left unconstrained (1).
template <int N>
constexpr int staged3d_waves() {
  return N >= 9 && N <= 13 ? 4 : 1;
}

// kDefer selects the prefetch pipeline of staged3d_step: two slices per
// wavefront with each tile's copy-out issued after the next tile's commit,
// and one wait for the factor loads before the loop (launch variant 11);
// otherwise one slice, results written out as soon as they are in it
// (variant 8).  Which is faster depends on the size; the launch table picks.
template <class M, int N, bool kTrans, bool kDefer>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(staged3d_waves<N>()))) void kron3d_staged_kernel(const typename M::io_t* __restrict__ A,
                                                               const typename M::io_t* __restrict__ B,
                                                               const typename M::io_t* __restrict__ C,
                                                               const typename M::io_t* __restrict__ X,
                                                               typename M::io_t* __restrict__ Y, int64_t batch,
                                                               int64_t ntiles) {
  using S = Staged3D<M, N, kTrans>;
  using io_t = typename M::io_t;
  using P = RunPrefetch<io_t, S::kElems>;
  // small tiles: the next tile's operands (at most 4 vectors per lane) are
  // loaded while the current one is computed; larger tiles would give up
  // occupancy for the registers
  constexpr bool kPf = P::kAll <= 4;
  constexpr int kBuf = kPf && kDefer ? stage_buffers<S::kSlice * (int)sizeof(io_t)>() : 1;
  __shared__ __attribute__((aligned(16))) io_t slices[kBlock / kWave][kBuf][S::kSlice];
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const int w = threadIdx.x >> 6;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const S st(A, B, C, L, g);
  if constexpr (kDefer) wait_loads();
  if constexpr (kPf) {
    P pf;
    Pending<io_t> po;
    int64_t t = wave;
    int b = 0;
    if (t < ntiles) pf.issue(X + t * S::kElems, (int)((batch - t * S::kOps) < S::kOps ? batch - t * S::kOps : S::kOps) * S::E, l);
    for (; t < ntiles; t += nwaves, b ^= kBuf - 1) {
      const int64_t tn = t + nwaves;
      staged3d_step<kBuf == 2>(st, slices[w][b], X + t * S::kElems, Y + t * S::kElems, batch - t * S::kOps, l, pf, po,
                               tn < ntiles ? X + tn * S::kElems : nullptr, batch - tn * S::kOps);
    }
    wave_sync_lds();
    po.write(l);
  } else {
    for (int64_t t = wave; t < ntiles; t += nwaves)
      staged3d_tile(st, slices[w][0], X + t * S::kElems, Y + t * S::kElems, batch - t * S::kOps, l);
  }
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
  // Consecutive tiles sit back to back in LDS as they do in memory, so that
  // a group of kT tiles moves as one span; kT is sized for about 4 KB per
  // wavefront and group (the copy size that keeps HBM busiest), 2..8 tiles.
  static constexpr int kTileBytes = kElems * (int)sizeof(io_t);
  static constexpr int kT = 4096 / kTileBytes < 2 ? 2 : 4096 / kTileBytes > 8 ? 8 : 4096 / kTileBytes;
  static constexpr int kSpan = (kT * kElems + kStagePad + 7) / 8 * 8;

  Tile tile;
  LaneSlots<N, 2> in, out;

  __device__ __forceinline__ Staged2D(const io_t* A, const io_t* B, int L, int g)
      : tile(A, B, L, g), in(L, 0, g, 1, false), out(L, 0, g, 1, M::drow(0, 1) != 1) {}

  __device__ __forceinline__ acc_t read(const io_t* lds) const {
    acc_t v;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const auto x = widen(in_lds(lds)[in.base[s]]);
      v[s] = in.ok[s] ? x : decltype(x)(0);
    }
    return v;
  }

  __device__ __forceinline__ void write(io_t* lds, const acc_t& v) const {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (out.ok[r]) in_lds(lds)[out.base[r]] = narrow<io_t>(v[r]);
  }
};

// A span is kT consecutive tiles (from tile t0; those at or past `last` hold
// nothing) that move through the wavefront's LDS as one piece: the run of
// operands they hold is copied in as one piece, the tail of the span
// zero-filled, and the results copied out as one piece.
// Elements of the operands in the span of tiles t0 .. min(t0 + kT, last) - 1.
template <class S>
__device__ __forceinline__ int span_elems(int64_t t0, int64_t last, int64_t batch) {
  const int64_t ops_left = batch - t0 * S::kOps;
  const int64_t tiles_left = last - t0;
  const int64_t cap = (tiles_left < S::kT ? tiles_left : S::kT) * S::kOps;
  return (int)(ops_left < cap ? ops_left : cap) * S::E;
}

// The fallback of a span with a non-finite packed tile (results of the
// other tiles already in the span): every tile is written out at once, the
// bad ones recomputed operand by operand.
template <class S>
__device__ __forceinline__ void staged2d_redo(const S& st, typename S::io_t* span, const typename S::io_t* Xs,
                                              typename S::io_t* Ys, int nops_all, const bool (&bad)[S::kT], int l) {
  using io_t = typename S::io_t;
  using acc_t = typename S::acc_t;
  constexpr int kT = S::kT;
  if constexpr (S::kOps > 1) {
    for (int j = 0; j < kT; ++j) {
      const int nops = nops_all - j * S::kOps;
      if (nops <= 0) break;
      const int nj = nops < S::kOps ? nops : S::kOps;
      io_t* sl = span + j * S::kElems;
      if (!bad[j]) {
        copy_out(Ys + j * S::kElems, sl, nj * S::E, l);
        continue;
      }
      const io_t* Xt = Xs + j * S::kElems;
      io_t* Yt = Ys + j * S::kElems;
      // this tile's results were not written back: redo it operand by operand
      for (int o = 0; o < nj; ++o) {
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

// A span of a prefetched sequence, as staged3d_step (kDefer: two slices per
// wavefront, the previous span's copy-out issued after this span's commit).
// A span with a non-finite packed tile is finished by staged2d_redo (every
// part written out at once, the bad tiles redone per operand as in 3-D).
template <bool kDefer, class S, class P>
__device__ __forceinline__ void staged2d_step(const S& st, typename S::io_t* span, const typename S::io_t* X,
                                              typename S::io_t* Y, int64_t t0, int64_t last, int64_t batch, int l,
                                              P& pf, Pending<typename S::io_t>& po, int64_t tn) {
  using io_t = typename S::io_t;
  using acc_t = typename S::acc_t;
  constexpr int kT = S::kT;
  const int count = span_elems<S>(t0, last, batch);
  const int nops_all = count / S::E;
  const io_t* Xs = X + t0 * S::kElems;
  io_t* Ys = Y + t0 * S::kElems;
  span = stage_base(span, Xs);
  wave_sync_lds();  // this span's last copy-out has read it
  zero_fill(span, count, kT * S::kElems, l);
  pf.commit(span, l);
  if constexpr (kDefer) po.write(l);
  wave_sync_lds();
  if (tn < last) pf.issue(X + tn * S::kElems, span_elems<S>(tn, last, batch), l);
  acc_t v[kT];
#pragma unroll
  for (int j = 0; j < kT; ++j) v[j] = st.tile.compute(st.read(span + j * S::kElems));
  bool bad[kT];
  bool any_bad = false;
#pragma unroll
  for (int j = 0; j < kT; ++j) {
    const int nops = nops_all - j * S::kOps;
    bad[j] = S::kOps > 1 && nops > 0 && __any(!all_finite(v[j]));
    any_bad |= bad[j];
  }
  wave_sync_lds();
#pragma unroll
  for (int j = 0; j < kT; ++j)
    if (!bad[j]) st.write(span + j * S::kElems, v[j]);
  wave_sync_lds();
  if (!any_bad) {
    if constexpr (kDefer) po.hold(Ys, span, count);
    else copy_out(Ys, span, count, l);
    return;
  }
  staged2d_redo(st, span, Xs, Ys, nops_all, bad, l);
}

// kDefer as for the 3-D kernel (launch variant 4; variant 3 without).
template <class M, int N, bool kTrans, bool kDefer>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void kron2d_staged_kernel(const typename M::io_t* __restrict__ A,
                                                               const typename M::io_t* __restrict__ B,
                                                               const typename M::io_t* __restrict__ X,
                                                               typename M::io_t* __restrict__ Y, int64_t batch,
                                                               int64_t ntiles) {
  using S = Staged2D<M, N, kTrans>;
  using io_t = typename M::io_t;
  constexpr int kT = S::kT;
  constexpr int kBuf = kDefer ? stage_buffers<S::kSpan * (int)sizeof(io_t)>() : 1;
  __shared__ __attribute__((aligned(16))) io_t slices[kBlock / kWave][kBuf][S::kSpan];
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const int w = threadIdx.x >> 6;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const S st(A, B, L, g);
  if constexpr (kDefer) wait_loads();
  // the next span's operands (at most about 4 KiB) are loaded while the
  // current span is computed
  RunPrefetch<io_t, kT * S::kElems> pf;
  Pending<io_t> po;
  int64_t base = wave * kT;
  int b = 0;
  if (base < ntiles) pf.issue(X + base * S::kElems, span_elems<S>(base, ntiles, batch), l);
  for (; base < ntiles; base += nwaves * kT, b ^= kBuf - 1)
    staged2d_step<kBuf == 2>(st, slices[w][b], X, Y, base, ntiles, batch, l, pf, po, base + nwaves * kT);
  wave_sync_lds();
  po.write(l);
}

}  // namespace kron
