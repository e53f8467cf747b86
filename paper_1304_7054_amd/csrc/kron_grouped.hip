// One persistent launch over many (dim, n) groups of operands, each group
// with its own shared factors: the paper's batched action (Section 2.2) for
// a batch that mixes sizes and 2-D / 3-D operands.
//
// kron_grouped_prepare builds, on the host, a work list in the caller's
// device workspace:
//   header | group descriptors | per-wavefront item ranges | items
// An item is a run of consecutive tiles of one group.  Tiles are priced with
// a cost model (matrix-core cycles vs HBM bytes of the tile, whichever is
// larger), each group is cut into items of about equal cost, and items are
// handed to wavefronts largest first, each to the wavefront with the least
// work so far.  The assignment is static, so a captured graph can replay the
// launch with no counters to reset, and results do not depend on timing.
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

struct alignas(16) Item {
  int32_t group;
  int32_t ntiles;
  int64_t first_tile;
};

struct alignas(64) Header {
  uint64_t magic;
  int32_t ngroups;
  int32_t nwaves;
  int32_t nitems;
  int32_t blocks;
  int64_t groups_off, starts_off, items_off, total_bytes;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---- device side ----------------------------------------------------------------

// The item routines stay out of line: inlining all (mode, dim, n) paths into
// the one kernel made the register allocator spill heavily.  Sizes other
// than 16 go through the wavefront's LDS slice (kron_staged.hpp).
constexpr int kGroupSlice = 4096 + 8;  // floats per wavefront: the largest 3-D tile

template <class M, int N, bool kVec>
__device__ __attribute__((noinline)) void run_item_2d(const GroupDesc& gd, const Item& it, int L, int g,
                                                      float* slice) {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  const io_t* X = static_cast<const io_t*>(gd.X);
  io_t* Y = static_cast<io_t*>(gd.Y);
  const int64_t end = it.first_tile + it.ntiles;
  if constexpr (N != 16) {
    using S = Staged2D<M, N, false>;
    static_assert(S::kSpan * sizeof(io_t) <= kGroupSlice * sizeof(float), "2-D span exceeds the wavefront's LDS");
    const S st(static_cast<const io_t*>(gd.A), static_cast<const io_t*>(gd.B), L, g);
    for (int64_t base = it.first_tile; base < end; base += S::kT)
      staged2d_tiles<S>(st, slice, X, Y, base, end, gd.count, threadIdx.x & 63);
  } else {
    constexpr int kT = 4;
    using T = Tile2D<M, N, kVec, false>;
    const T tile(static_cast<const io_t*>(gd.A), static_cast<const io_t*>(gd.B), L, g);
    for (int64_t base = it.first_tile; base < end; base += kT) {
      acc_t x[kT];
#pragma unroll
      for (int j = 0; j < kT; ++j) {
        const int64_t t = base + j;
        if (t < end) x[j] = tile.load(X + t * T::kOps * T::E, gd.count - t * T::kOps);
        else x[j] = acc_t{0, 0, 0, 0};
      }
#pragma unroll
      for (int j = 0; j < kT; ++j) x[j] = tile.compute(x[j]);
#pragma unroll
      for (int j = 0; j < kT; ++j) {
        const int64_t t = base + j;
        if (t < end) tile.finish(X + t * T::kOps * T::E, Y + t * T::kOps * T::E, gd.count - t * T::kOps, x[j]);
      }
    }
  }
}

template <class M, int N, bool kVec>
__device__ __attribute__((noinline)) void run_item_3d(const GroupDesc& gd, const Item& it, int L, int g,
                                                      float* slice) {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  const io_t* X = static_cast<const io_t*>(gd.X);
  io_t* Y = static_cast<io_t*>(gd.Y);
  const io_t* A = static_cast<const io_t*>(gd.A);
  const io_t* B = static_cast<const io_t*>(gd.B);
  const io_t* C = static_cast<const io_t*>(gd.C);
  const int64_t end = it.first_tile + it.ntiles;
  if constexpr (N != 16) {
    using S = Staged3D<M, N, false>;
    static_assert(S::kSlice <= kGroupSlice, "3-D slice exceeds the wavefront's LDS");
    const S st(A, B, C, L, g);
    for (int64_t t = it.first_tile; t < end; ++t)
      staged3d_tile(st, slice, X + t * S::kElems, Y + t * S::kElems, gd.count - t * S::kOps, threadIdx.x & 63);
  } else {
    using T = Tile3D<M, N, kVec, false, true>;
    constexpr int kWindow = 2;
    constexpr int64_t kStep = (int64_t)T::kOps * T::E;
    const T tile(A, B, C, L, g);
    for (int64_t t = it.first_tile; t < end; ++t) {
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
  }
}

template <class M>
__device__ __forceinline__ void run_item(const GroupDesc& gd, const Item& it, int L, int g, float* slice) {
#define KRON_G_CASE(NN)                                                                  \
  case NN:                                                                               \
    if (gd.dim == 2) {                                                                   \
      if (NN == 16 && gd.vec) run_item_2d<M, NN, NN == 16>(gd, it, L, g, slice);         \
      else run_item_2d<M, NN, false>(gd, it, L, g, slice);                               \
    } else {                                                                             \
      if (NN == 16 && gd.vec) run_item_3d<M, NN, NN == 16>(gd, it, L, g, slice);         \
      else run_item_3d<M, NN, false>(gd, it, L, g, slice);                               \
    }                                                                                    \
    break;
  switch (gd.n) { KRON_N_CASES(KRON_G_CASE) }
#undef KRON_G_CASE
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void kron_grouped_kernel(
    const uint8_t* __restrict__ ws) {
  const Header* h = reinterpret_cast<const Header*>(ws);
  const GroupDesc* groups = reinterpret_cast<const GroupDesc*>(ws + h->groups_off);
  const int32_t* starts = reinterpret_cast<const int32_t*>(ws + h->starts_off);
  const Item* items = reinterpret_cast<const Item*>(ws + h->items_off);
  __shared__ __attribute__((aligned(16))) float slices[kBlock / kWave][kGroupSlice];
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  float* slice = slices[threadIdx.x >> 6];
  const int wave = (int)(((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6);
  if (wave >= h->nwaves) return;
  const int i1 = starts[wave + 1];
  for (int i = starts[wave]; i < i1; ++i) {
    const Item it = items[i];
    const GroupDesc gd = groups[it.group];
    if (gd.mode == KRON_MODE_BF16X3) run_item<ModeBF16x3>(gd, it, L, g, slice);
    else run_item<ModeF32>(gd, it, L, g, slice);
  }
}

// ---- host side ------------------------------------------------------------------

struct Plan {
  int blocks;
  size_t bytes;
};
std::mutex g_plans_mu;
std::map<const void*, Plan> g_plans;

int64_t tiles_of(int dim, int n, int64_t count) {
  const int64_t q = 16 / n;
  const int64_t ops = dim == 3 ? q * q * q : q * q;
  return (count + ops - 1) / ops;
}

// Relative cost of one tile: the larger of its matrix-core time (MFMA
// cycles per SIMD) and its HBM time (bytes moved / ~2.2 bytes per SIMD cycle
// at full-chip bandwidth).
double tile_cost(int dim, int n, int mode) {
  const int q = 16 / n;
  const double elems = dim == 3 ? (double)q * q * q * n * n * n : (double)q * q * n * n;
  const double mem = 2.0 * 4.0 * elems / 2.2;
  double mfma;
  if (dim == 3) mfma = mode == KRON_MODE_BF16X3 ? 3 * 16 * 2 * 16.0 : 3 * 16 * 4 * 32.0;
  else mfma = mode == KRON_MODE_BF16X3 ? 2 * 2 * 16.0 : 2 * 4 * 32.0;
  return std::max(mem, mfma) + 200.0;  // fixed per-tile overhead
}

int grouped_blocks() {
  static const int occ = std::max(1, occupancy_blocks(kron_grouped_kernel));
  return device_cus() * occ;
}

struct Layout {
  size_t groups_off, starts_off, items_off, total;
};

Layout layout_for(int ngroups, int nwaves, int64_t nitems) {
  Layout lo;
  lo.groups_off = align_up(sizeof(Header), 64);
  lo.starts_off = align_up(lo.groups_off + sizeof(GroupDesc) * (size_t)ngroups, 64);
  lo.items_off = align_up(lo.starts_off + sizeof(int32_t) * ((size_t)nwaves + 1), 64);
  lo.total = align_up(lo.items_off + sizeof(Item) * (size_t)nitems, 256);
  return lo;
}

// Items per wavefront the splitter aims at (finer items balance better,
// coarser ones reload the factors less often).
constexpr int kItemsPerWave = 4;

// Cut every group into runs of consecutive tiles of about equal cost.
void split_items(const kron_group_t* g, int ngroups, int nwaves, std::vector<Item>& items, std::vector<double>& cost) {
  double total = 0;
  for (int i = 0; i < ngroups; ++i)
    total += tile_cost(g[i].dim, g[i].n, g[i].mode) * (double)tiles_of(g[i].dim, g[i].n, g[i].count);
  const double target = total / ((double)nwaves * kItemsPerWave);
  items.clear();
  cost.clear();
  for (int i = 0; i < ngroups; ++i) {
    const int64_t nt = tiles_of(g[i].dim, g[i].n, g[i].count);
    if (nt == 0) continue;
    const double c = tile_cost(g[i].dim, g[i].n, g[i].mode);
    double perd = target / c;
    int64_t per = perd < 1.0 ? 1 : (perd > (double)(1 << 30) ? (int64_t)(1 << 30) : (int64_t)perd);
    for (int64_t t0 = 0; t0 < nt; t0 += per) {
      const int64_t k = std::min<int64_t>(per, nt - t0);
      items.push_back(Item{i, (int32_t)k, t0});
      cost.push_back(c * (double)k);
    }
  }
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

}  // namespace

size_t grouped_workspace_bytes(const kron_group_t* g, int ngroups) {
  if (check_groups(g, ngroups) != 0) return 0;
  const int nwaves = grouped_blocks() * (kBlock / kWave);
  std::vector<Item> items;
  std::vector<double> cost;
  split_items(g, ngroups, nwaves, items, cost);
  return layout_for(ngroups, nwaves, (int64_t)items.size()).total;
}

int grouped_prepare(const kron_group_t* g, int ngroups, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (check_groups(g, ngroups) != 0) return -1;
  if (!ws) return -3;
  const int blocks = grouped_blocks();
  const int nwaves = blocks * (kBlock / kWave);
  std::vector<Item> items;
  std::vector<double> cost;
  split_items(g, ngroups, nwaves, items, cost);
  const Layout lo = layout_for(ngroups, nwaves, (int64_t)items.size());
  if (ws_bytes < lo.total) return -4;

  // largest first, each to the least loaded wavefront
  std::vector<int> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  using Slot = std::pair<double, int>;
  std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
  for (int w = 0; w < nwaves; ++w) heap.push({0.0, w});
  std::vector<std::vector<int>> per_wave(nwaves);
  for (int idx : order) {
    Slot s = heap.top();
    heap.pop();
    per_wave[s.second].push_back(idx);
    heap.push({s.first + cost[idx], s.second});
  }

  std::vector<uint8_t> host(lo.total, 0);
  Header h{};
  h.magic = kMagic;
  h.ngroups = ngroups;
  h.nwaves = nwaves;
  h.nitems = (int32_t)items.size();
  h.blocks = blocks;
  h.groups_off = (int64_t)lo.groups_off;
  h.starts_off = (int64_t)lo.starts_off;
  h.items_off = (int64_t)lo.items_off;
  h.total_bytes = (int64_t)lo.total;
  std::memcpy(host.data(), &h, sizeof(h));
  GroupDesc* gd = reinterpret_cast<GroupDesc*>(host.data() + lo.groups_off);
  for (int i = 0; i < ngroups; ++i) {
    const kron_group_t& d = g[i];
    const uintptr_t mask = 15;
    const bool vec = ((uintptr_t)d.X & mask) == 0 && ((uintptr_t)d.Y & mask) == 0;
    gd[i] = GroupDesc{d.dim, d.n, d.mode, vec ? 1 : 0, d.A, d.B, d.C, d.X, d.Y, d.count,
                      tiles_of(d.dim, d.n, d.count)};
  }
  int32_t* starts = reinterpret_cast<int32_t*>(host.data() + lo.starts_off);
  Item* it = reinterpret_cast<Item*>(host.data() + lo.items_off);
  int32_t k = 0;
  for (int w = 0; w < nwaves; ++w) {
    starts[w] = k;
    for (int idx : per_wave[w]) it[k++] = items[idx];
  }
  starts[nwaves] = k;

  hipError_t e = hipMemcpyAsync(ws, host.data(), lo.total, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lk(g_plans_mu);
  g_plans[ws] = Plan{blocks, lo.total};
  return 0;
}

int grouped_launch(const void* ws, hipStream_t stream) {
  if (!ws) return -1;
  int blocks;
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    auto f = g_plans.find(ws);
    if (f == g_plans.end()) return -1;
    blocks = f->second.blocks;
  }
  hipLaunchKernelGGL(kron_grouped_kernel, dim3(blocks), dim3(kBlock), 0, stream, static_cast<const uint8_t*>(ws));
  return 0;
}

}  // namespace kron
