// One persistent launch over many (dim, n) groups of operands, each group
// with its own shared factors: the paper's batched action (Section 2.2) for
// a batch that mixes sizes and 2-D / 3-D operands.
//
// kron_grouped_prepare writes a small plan into the caller's device
// workspace: a header, the group descriptors, and for each of two phases
// (2-D groups, 3-D groups) the list of its groups with the number of work
// units before each.  With groups of both dimensions kron_grouped_launch
// runs both phases in one persistent kernel: some wavefronts start on the
// 2-D phase, the others on the 3-D phase, and each moves on to the other
// phase when its first has no work left, so that the 2-D phase's short,
// latency-bound units overlap the 3-D phase's streaming.  A batch of one
// dimension runs that phase's own kernel: the 2-D one keeps small LDS
// slices and more wavefronts per SIMD, which a 3-D tile of up to 16 KiB per
// wavefront would otherwise deny every group.
//
// Inside a phase, the groups' units (a unit is one 3-D tile or a run of 2-D
// tiles) form one sequence, groups with the costliest units first, cut into
// chunks that shrink along the sequence (guided self-scheduling: a chunk
// holds about the remaining work over twice the wavefront count, never less
// than a floor), so that the last chunks to be claimed are small.
// Wavefronts claim chunks in sequence order from a counter in the workspace,
// the next one while they work on the current one.  Neighbouring chunks therefore run at the same time, as
// neighbouring tiles do in the single-group kernels, a wavefront loads a
// group's factors only when its next chunk belongs to another group, and
// the load balances itself whatever the cost estimates are.  The wavefront
// that finishes last puts the counters back to zero, so the next launch, or
// a graph replay, starts from a clean state with no memset.  Which
// wavefront computes a chunk does not change its result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <queue>
#include <vector>

#include "kron.h"
#include "kron_kernels.hpp"
#include "kron_launch.hpp"
#include "kron_runtime.hpp"
#include "kron_staged.hpp"

namespace kron {

namespace {

constexpr uint64_t kMagic = 0x4b524f4e47525031ull;  // "KRONGRP1"

struct alignas(16) GroupDesc {
  int32_t dim, n, mode, vec;
  const void* A;
  const void* B;
  const void* C;
  const void* X;
  void* Y;
  int64_t count;
  int64_t ntiles;
};

// One phase: the groups of one dimension in sequence order.
struct PhaseDesc {
  int32_t ngroups, blocks;
  int64_t nchunks;
  int64_t list_off;     // ngroups x int32 group index (padded to 8 bytes), then
                        // ngroups + 1 x int64 units before each entry, then
                        // nchunks + 1 x int64 first unit of each chunk
  int64_t counter_off;  // uint64 next chunk, uint32 wavefronts done
};

struct alignas(64) Header {
  uint64_t magic;
  int32_t ngroups;
  int32_t split16;  // one launch for both phases: wavefronts with (index mod 16) below this start on the 2-D one
  int64_t groups_off, total_bytes;
  PhaseDesc phase[2];
};

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---- device side ----------------------------------------------------------------

// The item routines stay out of line: inlining all (mode, n) paths into one
// kernel made the register allocator spill heavily.  Sizes other than 16 go
// through the wavefront's LDS slice (kron_staged.hpp); the slice of each
// phase holds its largest staged tile (group) plus the alignment pad.
constexpr int kGroupSlice3 = 4096 + kStagePad;  // floats per wavefront: a 16^3-slot tile
constexpr int kGroupSlice2 = 1024 + kStagePad;  // floats per wavefront: a 4 KiB group of 2-D tiles

// Tiles per 2-D unit: a span of the staged path, or 4 tiles of the direct
// n = 16 path.  Used on both sides, so host and device count units alike.
template <class M, int N>
constexpr int units2d_tiles() {
  if constexpr (N != 16) return Staged2D<M, N, false>::kT;
  else return 4;
}

// Chunk claiming.  Lane 0 takes the next chunk index from the phase counter;
// the value is read (and broadcast) only when it is needed, so the atomic's
// latency overlaps the current chunk's work.
// First unit of each chunk of a phase (nchunks + 1 entries).
struct ChunkTable {
  const int64_t* start;
  int64_t nchunks;
  __device__ __forceinline__ int64_t first(int64_t c) const { return in_global(start)[c]; }
};

struct Claim {
  unsigned long long* next;
  __device__ __forceinline__ unsigned long long issue() const {
    unsigned long long c = 0;
    if ((threadIdx.x & 63) == 0) c = __hip_atomic_fetch_add(in_global(next), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return c;
  }
  __device__ static __forceinline__ int64_t value(unsigned long long c) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)c);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(c >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
  }
};

// The chunks of one group that a wavefront claims in a row, starting with
// chunk c.  The group's units are u0 .. u1 - 1 of the phase sequence; chunk
// c holds units cstart[c] .. cstart[c + 1] - 1.  Returns the first claimed
// chunk that is not this group's (or one past the last chunk).
template <class M, int N, bool kVec>
__device__ __attribute__((noinline)) int64_t run_group_2d(const GroupDesc& gd, int64_t c, const ChunkTable& ct,
                                                          int64_t u0, int64_t u1, Claim cl, int L, int g,
                                                          float* slice) {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  const io_t* X = static_cast<const io_t*>(gd.X);
  io_t* Y = static_cast<io_t*>(gd.Y);
  const int64_t ntiles = gd.ntiles;
  constexpr int kT = units2d_tiles<M, N>();
  if constexpr (N != 16) {
    using S = Staged2D<M, N, false>;
    static_assert(S::kSpan * sizeof(io_t) <= kGroupSlice2 * sizeof(float), "2-D span exceeds the wavefront's LDS");
    const S st(static_cast<const io_t*>(gd.A), static_cast<const io_t*>(gd.B), L, g);
    const int lane = threadIdx.x & 63;
    // the next unit of the chunk is loaded into registers while the current
    // one is computed and written out (as in the single-group kernel)
    RunPrefetch<io_t, kT * S::kElems> pf;
    Pending<io_t> po;  // one slice per wavefront: results are written out at once
    do {
      const unsigned long long nx = cl.issue();
      int64_t u = ct.first(c) - u0;
      const int64_t ue = ct.first(c + 1) - u0;
      if (u < ue) pf.issue(X + u * kT * S::kElems, span_elems<S>(u * kT, ntiles, gd.count), lane);
      for (; u < ue; ++u)
        staged2d_step<false>(st, slice, X, Y, u * kT, ntiles, gd.count, lane, pf, po,
                             u + 1 < ue ? (u + 1) * kT : ntiles);
      c = Claim::value(nx);
    } while (c < ct.nchunks && ct.first(c) < u1);
  } else {
    using T = Tile2D<M, N, kVec, false>;
    const T tile(static_cast<const io_t*>(gd.A), static_cast<const io_t*>(gd.B), L, g);
    do {
      const unsigned long long nx = cl.issue();
      for (int64_t u = ct.first(c) - u0, ue = ct.first(c + 1) - u0; u < ue; ++u) {
        const int64_t base = u * kT;
        acc_t x[kT];
#pragma unroll
        for (int j = 0; j < kT; ++j) {
          const int64_t t = base + j;
          if (t < ntiles) x[j] = tile.load(X + t * T::kOps * T::E, gd.count - t * T::kOps);
          else x[j] = acc_t{0, 0, 0, 0};
        }
#pragma unroll
        for (int j = 0; j < kT; ++j) x[j] = tile.compute(x[j]);
#pragma unroll
        for (int j = 0; j < kT; ++j) {
          const int64_t t = base + j;
          if (t < ntiles) tile.finish(X + t * T::kOps * T::E, Y + t * T::kOps * T::E, gd.count - t * T::kOps, x[j]);
        }
      }
      c = Claim::value(nx);
    } while (c < ct.nchunks && ct.first(c) < u1);
  }
  return c;
}

// As run_group_2d for a 3-D group (a unit is one tile).
template <class M, int N, bool kVec>
__device__ __attribute__((noinline)) int64_t run_group_3d(const GroupDesc& gd, int64_t c, const ChunkTable& ct,
                                                          int64_t u0, int64_t u1, Claim cl, int L, int g,
                                                          float* slice) {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  const io_t* X = static_cast<const io_t*>(gd.X);
  io_t* Y = static_cast<io_t*>(gd.Y);
  const io_t* A = static_cast<const io_t*>(gd.A);
  const io_t* B = static_cast<const io_t*>(gd.B);
  const io_t* C = static_cast<const io_t*>(gd.C);
  const int64_t ntiles = gd.ntiles;
  if constexpr (N != 16) {
    using S = Staged3D<M, N, false>;
    static_assert(S::kSlice * sizeof(io_t) <= kGroupSlice3 * sizeof(float), "3-D slice exceeds the wavefront's LDS");
    const S st(A, B, C, L, g);
    const int lane = threadIdx.x & 63;
    // the next tile of the chunk is loaded into registers while the current
    // one is computed (up to 8 vectors per lane; larger tiles copy the rest
    // when they are committed)
    RunPrefetch<io_t, S::kElems> pf;
    Pending<io_t> po;  // one slice per wavefront: results are written out at once
    auto ops_of = [&](int64_t t) { return (int)((gd.count - t * S::kOps) < S::kOps ? gd.count - t * S::kOps : S::kOps); };
    do {
      const unsigned long long nx = cl.issue();
      int64_t t = ct.first(c) - u0;
      const int64_t te = ct.first(c + 1) - u0;
      if (t < te) pf.issue(X + t * S::kElems, ops_of(t) * S::E, lane);
      for (; t < te; ++t)
        staged3d_step<false>(st, slice, X + t * S::kElems, Y + t * S::kElems,
                             gd.count - t * S::kOps, lane, pf, po, t + 1 < te ? X + (t + 1) * S::kElems : nullptr,
                             gd.count - (t + 1) * S::kOps);
      c = Claim::value(nx);
    } while (c < ct.nchunks && ct.first(c) < u1);
  } else {
    using T = Tile3D<M, N, kVec, false, true>;
    constexpr int kWindow = 2;
    constexpr int64_t kStep = (int64_t)T::kOps * T::E;
    const T tile(A, B, C, L, g);
    do {
      const unsigned long long nx = cl.issue();
      for (int64_t t = ct.first(c) - u0, te = ct.first(c + 1) - u0; t < te; ++t) {
        const io_t* Xt = X + t * kStep;
        const int64_t rem = gd.count - t * T::kOps;
        acc_t v[16];
#pragma unroll
        for (int b = 0; b < kWindow; ++b) tile.load_slab(Xt, rem, b, v[b]);
#pragma unroll
        for (int b = 0; b < 16; ++b) {
          __builtin_amdgcn_sched_barrier(0);
          tile.stage12(v[b]);
          if (b + kWindow < 16) tile.load_slab(Xt, rem, b + kWindow, v[b + kWindow]);  // n == 16: all live
        }
        __builtin_amdgcn_sched_barrier(0);
        tile.stage3(v);
        tile.finish(Xt, Y + t * kStep, rem, v);
      }
      c = Claim::value(nx);
    } while (c < ct.nchunks && ct.first(c) < u1);
  }
  return c;
}

template <class M, int Dim>
__device__ __forceinline__ int64_t run_group(const GroupDesc& gd, int64_t c, const ChunkTable& ct, int64_t u0,
                                             int64_t u1, Claim cl, int L, int g, float* slice) {
#define KRON_G_CASE(NN)                                                                                 \
  case NN:                                                                                              \
    if constexpr (Dim == 2) {                                                                           \
      if (NN == 16 && gd.vec) return run_group_2d<M, NN, NN == 16>(gd, c, ct, u0, u1, cl, L, g, slice); \
      return run_group_2d<M, NN, false>(gd, c, ct, u0, u1, cl, L, g, slice);                           \
    } else {                                                                                            \
      if (NN == 16 && gd.vec) return run_group_3d<M, NN, NN == 16>(gd, c, ct, u0, u1, cl, L, g, slice); \
      return run_group_3d<M, NN, false>(gd, c, ct, u0, u1, cl, L, g, slice);                           \
    }
  switch (gd.n) { KRON_N_CASES(KRON_G_CASE) }
#undef KRON_G_CASE
  return ct.nchunks;
}

// One phase's chunks, claimed until none are left; then the wavefront
// counts itself out of the phase (the last one resets the phase's counters).
template <int Dim>
__device__ __forceinline__ void grouped_phase(const uint8_t* __restrict__ ws, float* slice) {
  const Header* h = reinterpret_cast<const Header*>(ws);
  const PhaseDesc& ph = h->phase[Dim - 2];
  const GroupDesc* groups = reinterpret_cast<const GroupDesc*>(ws + h->groups_off);
  const size_t ng = (size_t)ph.ngroups;
  const int32_t* list = reinterpret_cast<const int32_t*>(ws + ph.list_off);
  const int64_t* ubefore = reinterpret_cast<const int64_t*>(ws + ph.list_off + align_up(4 * ng, 8));
  const ChunkTable ct{ubefore + ng + 1, ph.nchunks};
  unsigned long long* next = reinterpret_cast<unsigned long long*>(const_cast<uint8_t*>(ws) + ph.counter_off);
  unsigned int* done = reinterpret_cast<unsigned int*>(const_cast<uint8_t*>(ws) + ph.counter_off + 8);
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const Claim cl{next};
  int64_t c = Claim::value(cl.issue());
  int k = 0;
  while (c < ct.nchunks) {
    const int64_t u = ct.first(c);
    while (ubefore[k + 1] <= u) ++k;  // a wavefront's claims only grow
    const GroupDesc gd = groups[list[k]];
    if (gd.mode == KRON_MODE_BF16X3) c = run_group<ModeBF16x3, Dim>(gd, c, ct, ubefore[k], ubefore[k + 1], cl, L, g, slice);
    else c = run_group<ModeF32, Dim>(gd, c, ct, ubefore[k], ubefore[k + 1], cl, L, g, slice);
  }
  // every wavefront has made its last claim once `done` reaches the launch's
  // wavefront count: the last one resets both counters for the next launch
  if (l == 0) {
    const unsigned int nw = (gridDim.x * kBlock) / kWave;
    if (__hip_atomic_fetch_add(in_global(done), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u == nw) {
      __hip_atomic_exchange(in_global(next), 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_exchange(in_global(done), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 4))) void kron_grouped2d_kernel(
    const uint8_t* __restrict__ ws) {
  __shared__ __attribute__((aligned(16))) float slices[kBlock / kWave][kGroupSlice2];
  grouped_phase<2>(ws, slices[threadIdx.x >> 6]);
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void kron_grouped3d_kernel(
    const uint8_t* __restrict__ ws) {
  __shared__ __attribute__((aligned(16))) float slices[kBlock / kWave][kGroupSlice3];
  grouped_phase<3>(ws, slices[threadIdx.x >> 6]);
}

// Both phases in one launch: a share of the wavefronts (split16 of every 16)
// starts on the 2-D phase and the rest on the 3-D phase; each moves to the
// other phase once its first one has no chunks left.  The 2-D phase's short,
// latency-bound units then run beside the 3-D phase's streaming instead of
// after it.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void kron_grouped_kernel(
    const uint8_t* __restrict__ ws) {
  __shared__ __attribute__((aligned(16))) float slices[kBlock / kWave][kGroupSlice3];
  const Header* h = reinterpret_cast<const Header*>(ws);
  const int wave = (int)((blockIdx.x * kBlock + threadIdx.x) >> 6);
  float* slice = slices[threadIdx.x >> 6];
  if ((wave & 15) < h->split16) {
    grouped_phase<2>(ws, slice);
    grouped_phase<3>(ws, slice);
  } else {
    grouped_phase<3>(ws, slice);
    grouped_phase<2>(ws, slice);
  }
}

// ---- host side ------------------------------------------------------------------

struct Plan {
  int blocks[2];  // per phase; 0 = nothing to run
  int merged;     // > 0: one launch of kron_grouped_kernel with this many blocks
  size_t bytes;
};
std::mutex g_plans_mu;
std::map<const void*, Plan> g_plans;

int64_t tiles_of(int dim, int n, int64_t count) {
  const int64_t q = 16 / n;
  const int64_t ops = dim == 3 ? q * q * q : q * q;
  return (count + ops - 1) / ops;
}

template <class M>
int tiles_per_unit2d(int n) {
  switch (n) {
#define KRON_U_CASE(NN) \
  case NN:              \
    return units2d_tiles<M, NN>();
    KRON_N_CASES(KRON_U_CASE)
#undef KRON_U_CASE
    default:
      return 1;
  }
}

int64_t units_of(const kron_group_t& d) {
  const int64_t nt = tiles_of(d.dim, d.n, d.count);
  if (d.dim == 3) return nt;
  const int per = d.mode == KRON_MODE_BF16X3 ? tiles_per_unit2d<ModeBF16x3>(d.n) : tiles_per_unit2d<ModeF32>(d.n);
  return (nt + per - 1) / per;
}

int grouped_blocks(int dim) {
  static const int occ2 = std::max(1, occupancy_blocks(kron_grouped2d_kernel));
  static const int occ3 = std::max(1, occupancy_blocks(kron_grouped3d_kernel));
  return device_cus() * (dim == 2 ? occ2 : occ3);
}

int merged_blocks() {
  static const int occ = std::max(1, occupancy_blocks(kron_grouped_kernel));
  return device_cus() * occ;
}

struct Layout {
  size_t groups_off, list_off[2], counter_off[2], total;
};

Layout layout_for(int ngroups, const int (&nlist)[2], const int64_t (&nchunks)[2]) {
  Layout lo;
  lo.groups_off = align_up(sizeof(Header), 64);
  size_t at = lo.groups_off + sizeof(GroupDesc) * (size_t)ngroups;
  for (int ph = 0; ph < 2; ++ph) {
    lo.list_off[ph] = align_up(at, 64);
    at = lo.list_off[ph] + align_up(4 * (size_t)nlist[ph], 8) + 8 * ((size_t)nlist[ph] + 1) +
         8 * ((size_t)nchunks[ph] + 1);
  }
  for (int ph = 0; ph < 2; ++ph) {
    lo.counter_off[ph] = align_up(at, 64);
    at = lo.counter_off[ph] + 64;
  }
  lo.total = align_up(at, 256);
  return lo;
}

// Relative cost of one unit: the larger of its matrix-core time (MFMA
// cycles per SIMD) and its HBM time (bytes moved at ~2.2 bytes per SIMD
// cycle, the full-chip bandwidth), plus a fixed per-unit overhead.
double unit_cost(const kron_group_t& d) {
  const int q = 16 / d.n;
  const double elems = d.dim == 3 ? (double)q * q * q * d.n * d.n * d.n : (double)q * q * d.n * d.n;
  const double mem = 2.0 * 4.0 * elems / 2.2;
  const int steps = (q * d.n + 3) / 4;
  double mfma;
  if (d.dim == 3) mfma = d.mode == KRON_MODE_BF16X3 ? 3 * 16 * 2 * 16.0 : 3 * 16 * steps * 32.0;
  else mfma = d.mode == KRON_MODE_BF16X3 ? 2 * 2 * 16.0 : 2 * steps * 32.0;
  const double per_tile = std::max(mem, mfma) + 200.0;
  if (d.dim == 3) return per_tile;
  const int per = d.mode == KRON_MODE_BF16X3 ? tiles_per_unit2d<ModeBF16x3>(d.n) : tiles_per_unit2d<ModeF32>(d.n);
  return per_tile * per;
}

// Guided chunking: a chunk holds about (remaining cost) / (kGuide x
// wavefronts), at least kMinChunkCost (a couple of tiles of work), and never
// crosses a group boundary.
constexpr double kGuide = 2.0;
constexpr double kMinChunkCost = 40000.0;

// Order a phase's groups by unit cost (costliest first) and cut the unit
// sequence into chunks.  Fills the units before each group and the first
// unit of each chunk (plus the end); returns the number of chunks.
int64_t cut_chunks(const kron_group_t* g, std::vector<int>& list, int nwaves, std::vector<int64_t>& ubefore,
                   std::vector<int64_t>& cstart) {
  std::stable_sort(list.begin(), list.end(), [&](int a, int b) { return unit_cost(g[a]) > unit_cost(g[b]); });
  double remaining = 0;
  for (int i : list) remaining += unit_cost(g[i]) * (double)units_of(g[i]);
  ubefore.assign(1, 0);
  cstart.clear();
  const double waves = (double)std::max(nwaves, 1);
  for (int i : list) {
    const int64_t units = units_of(g[i]);
    const double uc = unit_cost(g[i]);
    int64_t u = 0;
    while (u < units) {
      const double want = std::max(remaining / (kGuide * waves), kMinChunkCost);
      const int64_t take = std::min<int64_t>(units - u, std::max<int64_t>(1, (int64_t)(want / uc)));
      cstart.push_back(ubefore.back() + u);
      u += take;
      remaining -= uc * (double)take;
    }
    ubefore.push_back(ubefore.back() + units);
  }
  cstart.push_back(ubefore.back());
  return (int64_t)cstart.size() - 1;
}

int check_groups(const kron_group_t* g, int ngroups) {
  if (!g || ngroups <= 0) return -1;
  for (int i = 0; i < ngroups; ++i) {
    const kron_group_t& d = g[i];
    if ((d.dim != 2 && d.dim != 3) || d.n < 1 || d.n > KRON_MAX_N) return -1;
    if (d.mode != KRON_MODE_F32 && d.mode != KRON_MODE_BF16X3) return -1;
    if (d.count < 0) return -1;
    if (d.count > 0 && (!d.A || !d.B || (d.dim == 3 && !d.C) || !d.X || !d.Y || d.X == d.Y)) return -1;
  }
  return 0;
}

// The non-empty groups of each phase, in descriptor order.
void phase_lists(const kron_group_t* g, int ngroups, std::vector<int> (&lists)[2], int (&nlist)[2]) {
  for (int ph = 0; ph < 2; ++ph) {
    lists[ph].clear();
    for (int i = 0; i < ngroups; ++i)
      if (g[i].dim == ph + 2 && g[i].count > 0) lists[ph].push_back(i);
    nlist[ph] = (int)lists[ph].size();
  }
}

}  // namespace

// Both phases' sequences and chunk tables.
struct Phases {
  std::vector<int> lists[2];
  int nlist[2];
  std::vector<int64_t> ubefore[2], cstart[2];
  int64_t nchunks[2];
  int blocks[2];
  int merged;   // blocks of the one-launch kernel when both phases have groups, else 0
  int split16;  // its wavefronts (of every 16) that start on the 2-D phase
};

// With groups of both dimensions, both phases run in one launch of
// kron_grouped_kernel (their chunks cut for that launch's wavefronts), half
// of its wavefronts starting on each phase.  The 2-D phase's units are short
// and bound by memory latency, so its share of the time exceeds its share of
// the bytes; on the 500,000-operand mixed batch any start share from 4 to 10
// of 16 wavefronts gave the same time, 1 to 3 were slower.
void build_phases(const kron_group_t* g, int ngroups, Phases& p) {
  phase_lists(g, ngroups, p.lists, p.nlist);
  const bool both = p.nlist[0] > 0 && p.nlist[1] > 0;
  p.merged = both ? merged_blocks() : 0;
  p.split16 = both ? 8 : 0;
  for (int ph = 0; ph < 2; ++ph) {
    p.blocks[ph] = both ? p.merged : grouped_blocks(ph + 2);
    p.nchunks[ph] = cut_chunks(g, p.lists[ph], p.blocks[ph] * (kBlock / kWave), p.ubefore[ph], p.cstart[ph]);
  }
}

size_t grouped_workspace_bytes(const kron_group_t* g, int ngroups) {
  if (check_groups(g, ngroups) != 0) return 0;
  Phases p;
  build_phases(g, ngroups, p);
  return layout_for(ngroups, p.nlist, p.nchunks).total;
}

int grouped_prepare(const kron_group_t* g, int ngroups, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (check_groups(g, ngroups) != 0) return -1;
  if (!ws) return -3;
  Phases p;
  build_phases(g, ngroups, p);
  const Layout lo = layout_for(ngroups, p.nlist, p.nchunks);
  if (ws_bytes < lo.total) return -4;

  std::vector<uint8_t> host(lo.total, 0);  // counters start at zero
  Header h{};
  h.magic = kMagic;
  h.ngroups = ngroups;
  h.groups_off = (int64_t)lo.groups_off;
  h.total_bytes = (int64_t)lo.total;
  h.split16 = p.split16;
  Plan plan{{0, 0}, p.merged, lo.total};
  for (int ph = 0; ph < 2; ++ph) {
    const size_t ng = (size_t)p.nlist[ph];
    h.phase[ph].ngroups = p.nlist[ph];
    h.phase[ph].blocks = ng > 0 ? p.blocks[ph] : 0;
    h.phase[ph].nchunks = p.nchunks[ph];
    h.phase[ph].list_off = (int64_t)lo.list_off[ph];
    h.phase[ph].counter_off = (int64_t)lo.counter_off[ph];
    plan.blocks[ph] = h.phase[ph].blocks;
    uint8_t* at = host.data() + lo.list_off[ph];
    for (size_t k = 0; k < ng; ++k) reinterpret_cast<int32_t*>(at)[k] = p.lists[ph][k];
    at += align_up(4 * ng, 8);
    std::memcpy(at, p.ubefore[ph].data(), 8 * p.ubefore[ph].size());
    at += 8 * p.ubefore[ph].size();
    std::memcpy(at, p.cstart[ph].data(), 8 * p.cstart[ph].size());
  }
  std::memcpy(host.data(), &h, sizeof(h));
  GroupDesc* gd = reinterpret_cast<GroupDesc*>(host.data() + lo.groups_off);
  for (int i = 0; i < ngroups; ++i) {
    const kron_group_t& d = g[i];
    const uintptr_t mask = 15;
    const bool vec = ((uintptr_t)d.X & mask) == 0 && ((uintptr_t)d.Y & mask) == 0;
    gd[i] = GroupDesc{d.dim, d.n, d.mode, vec ? 1 : 0, d.A, d.B, d.C, d.X, d.Y, d.count,
                      tiles_of(d.dim, d.n, d.count)};
  }

  hipError_t e = hipMemcpyAsync(ws, host.data(), lo.total, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lk(g_plans_mu);
  g_plans[ws] = plan;
  return 0;
}

int grouped_launch(const void* ws, hipStream_t stream) {
  if (!ws) return -1;
  Plan plan;
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    auto f = g_plans.find(ws);
    if (f == g_plans.end()) return -1;
    plan = f->second;
  }
  const uint8_t* w = static_cast<const uint8_t*>(ws);
  if (plan.merged > 0) {
    hipLaunchKernelGGL(kron_grouped_kernel, dim3(plan.merged), dim3(kBlock), 0, stream, w);
    return 0;
  }
  if (plan.blocks[0] > 0) hipLaunchKernelGGL(kron_grouped2d_kernel, dim3(plan.blocks[0]), dim3(kBlock), 0, stream, w);
  if (plan.blocks[1] > 0) hipLaunchKernelGGL(kron_grouped3d_kernel, dim3(plan.blocks[1]), dim3(kBlock), 0, stream, w);
  return 0;
}

}  // namespace kron
