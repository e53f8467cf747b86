// Host-side launch of the forward kernels: n dispatch, alignment choice and
// grid size.  Included by one translation unit per precision mode.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <mutex>
#include <unordered_map>

#include "kron_kernels.hpp"
#include "kron_staged.hpp"
#include "kron_runtime.hpp"

namespace kron {

// Resident workgroups per CU for a kernel, queried once per kernel (keyed by
// its address: kernels of one signature must not share the value).
inline int occupancy_blocks_of(const void* kernel) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(kernel);
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
  cache.emplace(kernel, nb);
  return nb;
}

template <typename K>
int occupancy_blocks(K kernel) {
  return occupancy_blocks_of(reinterpret_cast<const void*>(kernel));
}

// Workgroups to launch: enough to cover the work, at most `per_cu` (or the
// occupancy limit when per_cu <= 0) on every CU.
inline unsigned grid_blocks(int64_t waves_needed, int occ, int per_cu) {
  const int64_t need = (waves_needed + kBlock / kWave - 1) / (kBlock / kWave);
  const int64_t cap = (int64_t)device_cus() * (per_cu > 0 ? per_cu : occ);
  int64_t g = need < cap ? need : cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

inline bool aligned_to(const void* p, int bytes) { return (reinterpret_cast<uintptr_t>(p) % bytes) == 0; }

template <class M, int N, bool kTrans, bool kVec, int kTiles>
void launch2d_k(const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* X,
                typename M::io_t* Y, int64_t batch, int64_t ntiles, int per_cu, hipStream_t stream) {
  auto k = kron2d_kernel<M, N, kVec, kTrans, kTiles>;
  const int64_t waves = (ntiles + kTiles - 1) / kTiles;
  hipLaunchKernelGGL(k, dim3(grid_blocks(waves, occupancy_blocks(k), per_cu)), dim3(kBlock), 0, stream, A, B, X, Y,
                     batch, ntiles);
}

template <class M, int N, bool kTrans, bool kVec>
void launch2d_v(int variant, const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* X,
                typename M::io_t* Y, int64_t batch, int64_t ntiles, int per_cu, hipStream_t stream) {
  switch (variant) {
    case 1:
      launch2d_k<M, N, kTrans, kVec, 8>(A, B, X, Y, batch, ntiles, per_cu, stream);
      break;
    case 2:
      launch2d_k<M, N, kTrans, kVec, 2>(A, B, X, Y, batch, ntiles, per_cu, stream);
      break;
    default:
      launch2d_k<M, N, kTrans, kVec, 4>(A, B, X, Y, batch, ntiles, per_cu, stream);
  }
}

// Sizes that read their tiles through LDS: every n but 16 (an FP64 3-D
// slice is up to 32 KiB per wavefront, 128 KiB per workgroup).
template <class M, int N, int Dim>
constexpr bool kStageable = N != 16;

// 2-D variants: tiles kept in flight per wavefront, 0 -> 4, 1 -> 8, 2 -> 2;
// 3 -> tiles staged through LDS (n != 16), 4 -> the same with two LDS slices
// per wavefront and each span's copy-out issued after the next span's
// operands are committed (n = 16 runs variant 0).
template <class M, int N, bool kTrans>
int launch2d_n(const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* X,
               typename M::io_t* Y, int64_t batch, hipStream_t stream, int mode) {
  using io_t = typename M::io_t;
  constexpr int64_t ops = (int64_t)Geo<N>::Q * Geo<N>::Q;
  const int64_t ntiles = (batch + ops - 1) / ops;
  const LaunchShape sh = launch_shape(mode, 2, N);
  if constexpr (kStageable<M, N, 2>) {
    if (sh.variant == 3 || sh.variant == 4) {
      auto k = sh.variant == 4 ? kron2d_staged_kernel<M, N, kTrans, true> : kron2d_staged_kernel<M, N, kTrans, false>;
      constexpr int kT = Staged2D<M, N, kTrans>::kT;
      const int64_t waves = (ntiles + kT - 1) / kT;
      hipLaunchKernelGGL(k, dim3(grid_blocks(waves, occupancy_blocks(k), sh.blocks_per_cu)), dim3(kBlock), 0,
                         stream, A, B, X, Y, batch, ntiles);
      return 0;
    }
  }
  if constexpr (Geo<N>::kVec) {
    if (aligned_to(X, Mem<io_t>::kAlign) && aligned_to(Y, Mem<io_t>::kAlign)) {
      launch2d_v<M, N, kTrans, true>(sh.variant, A, B, X, Y, batch, ntiles, sh.blocks_per_cu, stream);
      return 0;
    }
  }
  launch2d_v<M, N, kTrans, false>(sh.variant, A, B, X, Y, batch, ntiles, sh.blocks_per_cu, stream);
  return 0;
}

template <class M, int N, bool kTrans, bool kVec, bool kPipe, bool kContig, int kWindow>
void launch3d_k(const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
                const typename M::io_t* X, typename M::io_t* Y, int64_t batch, int64_t ntiles, int per_cu,
                hipStream_t stream) {
  auto k = kron3d_kernel<M, N, kVec, kTrans, kPipe, kContig, kWindow>;
  hipLaunchKernelGGL(k, dim3(grid_blocks(ntiles, occupancy_blocks(k), per_cu)), dim3(kBlock), 0, stream, A, B, C, X,
                     Y, batch, ntiles);
}

template <class M, int N, bool kTrans, bool kVec>
void launch3d_v(int variant, const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
                const typename M::io_t* X, typename M::io_t* Y, int64_t batch, int64_t ntiles, int per_cu,
                hipStream_t stream) {
  switch (variant) {
    case 1:
      launch3d_k<M, N, kTrans, kVec, true, false, 0>(A, B, C, X, Y, batch, ntiles, per_cu, stream);
      break;
    case 2:
      launch3d_k<M, N, kTrans, kVec, false, true, 0>(A, B, C, X, Y, batch, ntiles, per_cu, stream);
      break;
    case 3:
      launch3d_k<M, N, kTrans, kVec, true, true, 0>(A, B, C, X, Y, batch, ntiles, per_cu, stream);
      break;
    case 4:
      launch3d_k<M, N, kTrans, kVec, false, true, 2>(A, B, C, X, Y, batch, ntiles, per_cu, stream);
      break;
    case 5:
      launch3d_k<M, N, kTrans, kVec, false, true, 4>(A, B, C, X, Y, batch, ntiles, per_cu, stream);
      break;
    case 6:
      launch3d_k<M, N, kTrans, kVec, true, true, 2>(A, B, C, X, Y, batch, ntiles, per_cu, stream);
      break;
    case 7:
      launch3d_k<M, N, kTrans, kVec, true, true, 4>(A, B, C, X, Y, batch, ntiles, per_cu, stream);
      break;
    case 9:
    case 10:
      if constexpr (N == 16 && kVec) {
        auto k = variant == 9 ? kron3d_stream_kernel<M, kTrans, 2> : kron3d_stream_kernel<M, kTrans, 4>;
        hipLaunchKernelGGL(k, dim3(grid_blocks(ntiles, occupancy_blocks(k), per_cu)), dim3(kBlock), 0, stream, A, B,
                           C, X, Y, ntiles);
      } else {
        // same stage order (contiguous rows), slab window 2
        launch3d_k<M, N, kTrans, kVec, false, true, 2>(A, B, C, X, Y, batch, ntiles, per_cu, stream);
      }
      break;
    default:
      launch3d_k<M, N, kTrans, kVec, false, false, 0>(A, B, C, X, Y, batch, ntiles, per_cu, stream);
  }
}

// 3-D variants: 0 plain, 1 next tile prefetched, 2 contiguous 1 KiB rows
// (operand slabs along the slow axis, a second lane-group exchange),
// 3 = 1 + 2, 4/5 contiguous rows with a window of 2/4 slab loads in flight,
// 6/7 = 4/5 with the next tile's first slabs requested before stage 3,
// 8 = tiles staged through LDS (n != 16; n = 16 falls back to variant 0), 9/10 = n = 16 with the result stores
// interleaved with the next tile's loads and stages 1-2, window 2/4 (other
// sizes and unaligned arrays run variant 4, the same stage order), 11 = 8
// with two LDS slices per wavefront where they fit and each tile's copy-out
// issued after the next tile's operands are committed (n = 16: variant 0).
template <class M, int N, bool kTrans>
int launch3d_n(const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
               const typename M::io_t* X, typename M::io_t* Y, int64_t batch, hipStream_t stream, int mode) {
  using io_t = typename M::io_t;
  constexpr int64_t ops = (int64_t)Geo<N>::Q * Geo<N>::Q * Geo<N>::Q;
  const int64_t ntiles = (batch + ops - 1) / ops;
  const LaunchShape sh = launch_shape(mode, 3, N);
  if constexpr (kStageable<M, N, 3>) {
    if (sh.variant == 8 || sh.variant == 11) {
      auto k = sh.variant == 11 ? kron3d_staged_kernel<M, N, kTrans, true> : kron3d_staged_kernel<M, N, kTrans, false>;
      hipLaunchKernelGGL(k, dim3(grid_blocks(ntiles, occupancy_blocks(k), sh.blocks_per_cu)), dim3(kBlock), 0,
                         stream, A, B, C, X, Y, batch, ntiles);
      return 0;
    }
  }
  if constexpr (Geo<N>::kVec) {
    if (aligned_to(X, Mem<io_t>::kAlign) && aligned_to(Y, Mem<io_t>::kAlign)) {
      launch3d_v<M, N, kTrans, true>(sh.variant, A, B, C, X, Y, batch, ntiles, sh.blocks_per_cu, stream);
      return 0;
    }
  }
  launch3d_v<M, N, kTrans, false>(sh.variant, A, B, C, X, Y, batch, ntiles, sh.blocks_per_cu, stream);
  return 0;
}

// kron_ex_kernel (beta != 0, or 2-D operands read transposed): the vector
// path when X and Y are aligned, a persistent grid sized by occupancy.
template <class M, int Dim, int N, bool kBeta, bool kTX>
void launch_ex_k(const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
                 const typename M::io_t* X, typename M::io_t* Y, int64_t batch, typename M::io_t beta,
                 hipStream_t stream) {
  using io_t = typename M::io_t;
  constexpr int64_t Q = Geo<N>::Q;
  constexpr int64_t ops = Dim == 2 ? Q * Q : Q * Q * Q;
  const int64_t ntiles = (batch + ops - 1) / ops;
  const int64_t waves = Dim == 2 ? (ntiles + 3) / 4 : ntiles;  // 2-D: four tiles per wavefront step
  auto run = [&](auto k) {
    hipLaunchKernelGGL(k, dim3(grid_blocks(waves, occupancy_blocks(k), 0)), dim3(kBlock), 0, stream, A, B, C, X, Y,
                       batch, ntiles, beta);
  };
  if constexpr (Geo<N>::kVec) {
    if (aligned_to(X, Mem<io_t>::kAlign) && aligned_to(Y, Mem<io_t>::kAlign)) {
      run(kron_ex_kernel<M, N, true, Dim, kBeta, kTX>);
      return;
    }
  }
  run(kron_ex_kernel<M, N, false, Dim, kBeta, kTX>);
}

template <class M, int Dim, int N>
int launch_ex_n(const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
                const typename M::io_t* X, typename M::io_t* Y, int64_t batch, typename M::io_t beta, bool transx,
                hipStream_t stream) {
  const bool has_beta = beta != typename M::io_t(0);
  if constexpr (Dim == 2) {
    if (transx) {
      if (has_beta) launch_ex_k<M, 2, N, true, true>(A, B, C, X, Y, batch, beta, stream);
      else launch_ex_k<M, 2, N, false, true>(A, B, C, X, Y, batch, beta, stream);
      return 0;
    }
  }
  if (!has_beta || transx) return -2;  // nothing this kernel adds: the caller runs the plain kernels
  launch_ex_k<M, Dim, N, true, false>(A, B, C, X, Y, batch, beta, stream);
  return 0;
}

#define KRON_N_CASES(F) \
  F(1) F(2) F(3) F(4) F(5) F(6) F(7) F(8) F(9) F(10) F(11) F(12) F(13) F(14) F(15) F(16)

template <class M, bool kTrans>
int launch2d(int n, const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* X,
             typename M::io_t* Y, int64_t batch, hipStream_t stream, int mode) {
  switch (n) {
#define KRON_CASE(NN) \
  case NN:            \
    return launch2d_n<M, NN, kTrans>(A, B, X, Y, batch, stream, mode);
    KRON_N_CASES(KRON_CASE)
#undef KRON_CASE
    default:
      return -1;
  }
}

template <class M, int Dim>
int launch_ex(int n, const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
              const typename M::io_t* X, typename M::io_t* Y, int64_t batch, typename M::io_t beta, bool transx,
              hipStream_t stream) {
  switch (n) {
#define KRON_CASE(NN) \
  case NN:            \
    return launch_ex_n<M, Dim, NN>(A, B, C, X, Y, batch, beta, transx, stream);
    KRON_N_CASES(KRON_CASE)
#undef KRON_CASE
    default:
      return -1;
  }
}

// n in [NLO, NHI] (one translation unit per range keeps builds parallel)
template <class M, bool kTrans, int NN, int NHI>
int launch3d_range(int n, const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
                   const typename M::io_t* X, typename M::io_t* Y, int64_t batch, hipStream_t stream, int mode) {
  if constexpr (NN > NHI) {
    return -1;
  } else {
    if (n == NN) return launch3d_n<M, NN, kTrans>(A, B, C, X, Y, batch, stream, mode);
    return launch3d_range<M, kTrans, NN + 1, NHI>(n, A, B, C, X, Y, batch, stream, mode);
  }
}

}  // namespace kron
