// Section 3's interface with leading dimensions: factors with lda/ldb/ldc,
// operands and results at arbitrary element strides (ldx, ldx2, ldxp and
// ldy, ldy2, ldyp), op on every factor, op on the operands in 2-D, alpha and
// beta.  FP32 and FP64.
//
// The MFMA contractions are those of the dense tiles (Tile2D / Tile3D
// compute); only the addressing differs.  Every lane computes the element
// offsets of its slots from the strides at run time (64-bit), reads and
// writes one element at a time (3-D n = 16 with strides in multiples of 4
// elements: 16-byte vectors), and keeps the dense kernels' rules: packed
// tiles for n < 16, dead slots skipped, a tile with a non-finite result redone
// one operand at a time.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kron.h"
#include "kron_kernels.hpp"
#include "kron_launch.hpp"

namespace kron {
namespace {

// Element strides of one array: s1 between columns (2-D) or along the middle
// index (3-D), s2 along the slowest index (3-D), sp between operands.
struct Strides {
  int64_t s1, s2, sp;
};

// op(M) with leading dimension ld, alpha on the first factor, written dense
// (factor f at out + f * n^2, column-major).
template <typename T>
__global__ __launch_bounds__(256) void prepare_strided_factors_kernel(int n, int nf, const T* __restrict__ A, int lda,
                                                                      const T* __restrict__ B, int ldb,
                                                                      const T* __restrict__ C, int ldc, unsigned tmask,
                                                                      T alpha, T* __restrict__ out) {
  const int nn = n * n;
  for (int e = threadIdx.x; e < nf * nn; e += blockDim.x) {
    const int f = e / nn, idx = e % nn, i = idx % n, j = idx / n;
    const T* M = f == 0 ? A : f == 1 ? B : C;
    const int ld = f == 0 ? lda : f == 1 ? ldb : ldc;
    const T v = ((tmask >> f) & 1u) ? M[j + (int64_t)ld * i] : M[i + (int64_t)ld * j];
    out[e] = f == 0 ? alpha * v : v;
  }
}

// One element access of a lane: its offset inside the tile's first operand
// block and the packed operand it belongs to.
struct Site {
  int64_t off;
  int op;
  bool valid;
};

template <bool kBeta, typename T>
__device__ __forceinline__ void put(T* p, T v, T beta) {
  if constexpr (kBeta) v = v + beta * Mem<T>::load1(p);
  Mem<T>::store1(p, v);
}

// kVec (3-D, n = 16, every stride a multiple of 4 elements, 16-byte aligned
// bases): the four fast-axis elements of a lane are contiguous and move as
// one vector, as in the dense kernels.
template <class M, int N, int kDim, bool kBeta, bool kTX, bool kVec>
__global__ __launch_bounds__(kBlock) void kron_strided_kernel(const typename M::io_t* __restrict__ A,
                                                              const typename M::io_t* __restrict__ B,
                                                              const typename M::io_t* __restrict__ C,
                                                              const typename M::io_t* __restrict__ X, Strides xs,
                                                              typename M::io_t* __restrict__ Y, Strides ys,
                                                              int64_t batch, int64_t ntiles, typename M::io_t beta) {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  constexpr int Q = Geo<N>::Q;
  static_assert(!kVec || (kDim == 3 && N == 16), "vector accesses: 3-D, n = 16");
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  const Slot<N> sL(L);
  if constexpr (kDim == 2) {
    // lane (L, g) holds element (row = slot 4g + s, column = slot L) of op(X_p)
    // and stores Y(row = slot drow(g, r), column = slot L)
    using Tl = Tile2D<M, N, false, false>;
    constexpr int kOps = Tl::kOps;
    const Tl tile(A, B, L, g);
    Site in[4], out[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const Slot<N> sf(4 * g + s), so(M::drow(g, s));
      in[s].op = sL.sub * Q + sf.sub;
      in[s].off = in[s].op * xs.sp + (kTX ? sL.idx + xs.s1 * sf.idx : sf.idx + xs.s1 * sL.idx);
      in[s].valid = sL.valid && sf.valid;
      out[s].op = sL.sub * Q + so.sub;
      out[s].off = out[s].op * ys.sp + so.idx + ys.s1 * sL.idx;
      out[s].valid = sL.valid && so.valid;
    }
    auto load = [&](const io_t* Xt, int64_t rem, int only) {
      acc_t x;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bool ok = in[s].valid && in[s].op < rem && (only < 0 || in[s].op == only);
        x[s] = ok ? Mem<io_t>::load1(Xt + in[s].off) : io_t(0);
      }
      return x;
    };
    auto store = [&](io_t* Yt, int64_t rem, int only, const acc_t& y) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (out[r].valid && out[r].op < rem && (only < 0 || out[r].op == only)) put<kBeta>(Yt + out[r].off, y[r], beta);
    };
    // four tiles in flight per wavefront: their loads, then products and stores
    constexpr int kTiles = 4;
    for (int64_t base = wave * kTiles; base < ntiles; base += nwaves * kTiles) {
      acc_t x[kTiles];
#pragma unroll
      for (int j = 0; j < kTiles; ++j) {
        const int64_t t = base + j;
        x[j] = t < ntiles ? load(X + t * kOps * xs.sp, batch - t * kOps, -1) : acc_t{0, 0, 0, 0};
      }
#pragma unroll
      for (int j = 0; j < kTiles; ++j) {
        const int64_t t = base + j;
        if (t >= ntiles) continue;
        const io_t* Xt = X + t * kOps * xs.sp;
        io_t* Yt = Y + t * kOps * ys.sp;
        const int64_t rem = batch - t * kOps;
        const acc_t y = tile.compute(x[j]);
        if (kOps > 1 && __any(!all_finite(y))) {
          const int last = rem < kOps ? (int)rem : kOps;
          for (int o = 0; o < last; ++o) store(Yt, rem, o, tile.compute(load(Xt, rem, o)));
        } else {
          store(Yt, rem, -1, y);
        }
      }
    }
  } else {
    // contiguous-row stage order of Tile3D: lane (L, g), slab b holds
    // X(fast = slot 4g + s, middle = slot L, slow = slot b); results come back
    // in the same arrangement
    using Tl = Tile3D<M, N, false, false, true>;
    constexpr int kOps = Tl::kOps;
    const Tl tile(A, B, C, L, g);
    Site fx[4], fy[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const Slot<N> sf(4 * g + s);
      const int op = sL.sub * Q + sf.sub;
      fx[s] = Site{op * xs.sp + sf.idx + xs.s1 * sL.idx, op, sL.valid && sf.valid};
      fy[s] = Site{op * ys.sp + sf.idx + ys.s1 * sL.idx, op, sL.valid && sf.valid};
    }
    auto load = [&](const io_t* Xt, int64_t rem, int only, acc_t (&v)[16]) {
      if constexpr (kVec) {  // one operand per tile, every slot live
#pragma unroll
        for (int b = 0; b < 16; ++b) v[b] = Mem<io_t>::load4(Xt + b * xs.s2 + fx[0].off);
        return;
      }
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const Slot<N> sb(b);
        const int opb = sb.sub * Q * Q;
        const int64_t offb = opb * xs.sp + sb.idx * xs.s2;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int op = opb + fx[s].op;
          const bool ok = sb.valid && fx[s].valid && op < rem && (only < 0 || op == only);
          v[b][s] = ok ? Mem<io_t>::load1(Xt + offb + fx[s].off) : io_t(0);
        }
      }
    };
    auto store = [&](io_t* Yt, int64_t rem, int only, const acc_t (&v)[16]) {
      if constexpr (kVec) {
#pragma unroll
        for (int i = 0; i < 16; ++i) put4<kBeta>(Yt + i * ys.s2 + fy[0].off, v[i], beta);
        return;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const Slot<N> si(i);
        const int opi = si.sub * Q * Q;
        const int64_t offi = opi * ys.sp + si.idx * ys.s2;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int op = opi + fy[s].op;
          if (si.valid && fy[s].valid && op < rem && (only < 0 || op == only))
            put<kBeta>(Yt + offi + fy[s].off, v[i][s], beta);
        }
      }
    };
    for (int64_t t = wave; t < ntiles; t += nwaves) {
      const io_t* Xt = X + t * kOps * xs.sp;
      io_t* Yt = Y + t * kOps * ys.sp;
      const int64_t rem = batch - t * kOps;
      acc_t v[16];
      load(Xt, rem, -1, v);
      tile.compute(v);
      bool fin = true;
#pragma unroll
      for (int i = 0; i < 16; ++i) fin = fin && all_finite(v[i]);
      if (kOps > 1 && __any(!fin)) {
        const int last = rem < kOps ? (int)rem : kOps;
        for (int o = 0; o < last; ++o) {
          load(Xt, rem, o, v);
          tile.compute(v);
          store(Yt, rem, o, v);
        }
      } else {
        store(Yt, rem, -1, v);
      }
    }
  }
}

inline bool vec_strides(const Strides& s, const void* base) {
  return s.s1 % 4 == 0 && s.s2 % 4 == 0 && s.sp % 4 == 0 && reinterpret_cast<uintptr_t>(base) % 16 == 0;
}

template <class M, int Dim, int N, bool kBeta, bool kTX>
void launch_strided_k(const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
                      const typename M::io_t* X, Strides xs, typename M::io_t* Y, Strides ys, int64_t batch,
                      typename M::io_t beta, hipStream_t stream) {
  constexpr int64_t Q = Geo<N>::Q;
  constexpr int64_t ops = Dim == 2 ? Q * Q : Q * Q * Q;
  const int64_t ntiles = (batch + ops - 1) / ops;
  const int64_t waves = Dim == 2 ? (ntiles + 3) / 4 : ntiles;  // 2-D: four tiles per wavefront step
  auto run = [&](auto k) {
    hipLaunchKernelGGL(k, dim3(grid_blocks(waves, occupancy_blocks(k), 0)), dim3(kBlock), 0, stream, A, B, C, X,
                       xs, Y, ys, batch, ntiles, beta);
  };
  if constexpr (Dim == 3 && N == 16) {
    if (vec_strides(xs, X) && vec_strides(ys, Y)) {
      run(kron_strided_kernel<M, N, Dim, kBeta, kTX, true>);
      return;
    }
  }
  run(kron_strided_kernel<M, N, Dim, kBeta, kTX, false>);
}

template <class M, int Dim, int N>
void launch_strided_n(const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
                      const typename M::io_t* X, Strides xs, typename M::io_t* Y, Strides ys, int64_t batch,
                      typename M::io_t beta, bool transx, hipStream_t stream) {
  const bool has_beta = beta != typename M::io_t(0);
  if constexpr (Dim == 2) {
    if (transx) {
      if (has_beta) launch_strided_k<M, 2, N, true, true>(A, B, C, X, xs, Y, ys, batch, beta, stream);
      else launch_strided_k<M, 2, N, false, true>(A, B, C, X, xs, Y, ys, batch, beta, stream);
      return;
    }
  }
  if (has_beta) launch_strided_k<M, Dim, N, true, false>(A, B, C, X, xs, Y, ys, batch, beta, stream);
  else launch_strided_k<M, Dim, N, false, false>(A, B, C, X, xs, Y, ys, batch, beta, stream);
}

template <class M, int Dim>
int launch_strided(int n, const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
                   const typename M::io_t* X, Strides xs, typename M::io_t* Y, Strides ys, int64_t batch,
                   typename M::io_t beta, bool transx, hipStream_t stream) {
  switch (n) {
#define KRON_CASE(NN)                                                                           \
  case NN:                                                                                      \
    launch_strided_n<M, Dim, NN>(A, B, C, X, xs, Y, ys, batch, beta, transx, stream);           \
    return 0;
    KRON_N_CASES(KRON_CASE)
#undef KRON_CASE
    default:
      return -1;
  }
}

// ---- 1-D: TKRON1, y_p <- alpha op(A) x_p + beta y_p ---------------------------
//
// One tile is 16 vectors: D = Aop * [x_p .. x_p+15] on the 16x16 MFMA, with
// Aop = alpha op(A) padded to 16 x 16 with zeros.  Lane (L, g) supplies row L
// of Aop and column L (vector p + L) of the block at contraction slots
// 4g + s, and receives rows drow(g, r) of that column (FP64: regrouped to
// 4g + r).  Each output column sees only its own vector, so a NaN stays in
// its vector.  Four tiles are in flight per wavefront.  kVec (n = 16, strides
// multiples of 4 elements, 16-byte aligned bases): one 16-byte load and store
// per lane and tile.
template <class M, bool kVec, bool kBeta>
__global__ __launch_bounds__(kBlock) void kron1d_kernel(int n, const typename M::io_t* __restrict__ Aop,
                                                        const typename M::io_t* __restrict__ X, int64_t ldxp,
                                                        typename M::io_t* __restrict__ Y, int64_t ldyp,
                                                        int64_t batch, int64_t ntiles, typename M::io_t beta) {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  io_t a[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 4 * g + s;
    a[s] = (L < n && k < n) ? Aop[L + n * k] : io_t(0);
  }
  constexpr int kTiles = 4;  // tiles in flight per wavefront: all loads, then the products, then the stores
  for (int64_t base = wave * kTiles; base < ntiles; base += nwaves * kTiles) {
    acc_t x[kTiles];
#pragma unroll
    for (int j = 0; j < kTiles; ++j) {
      const int64_t p = (base + j) * 16 + L;
      const bool live = p < batch;
      if constexpr (kVec) {
        x[j] = live ? Mem<io_t>::load4(X + p * ldxp + 4 * g) : acc_t{0, 0, 0, 0};
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = 4 * g + s;
          x[j][s] = (live && k < n) ? Mem<io_t>::load1(X + p * ldxp + k) : io_t(0);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kTiles; ++j) {
      const int64_t p = (base + j) * 16 + L;
      const bool live = p < batch;
      acc_t y = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if constexpr (sizeof(io_t) == 8) y = mfma_f64(a[s], x[j][s], y);
        else y = mfma_f32(a[s], x[j][s], y);
      }
      if constexpr (M::drow(0, 1) != 1) transpose_groups_regs(y);  // rows 4g + r
      if constexpr (kVec) {
        if (live) put4<kBeta>(Y + p * ldyp + 4 * g, y, beta);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * g + r;
          if (live && i < n) put<kBeta>(Y + p * ldyp + i, y[r], beta);
        }
      }
    }
  }
}

// alpha op(A) with leading dimension lda, written dense
template <typename T>
__global__ __launch_bounds__(256) void prepare_tkron1_kernel(int n, const T* __restrict__ A, int lda, int trans,
                                                             T alpha, T* __restrict__ out) {
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e % n, j = e / n;
    out[e] = alpha * (trans ? A[j + (int64_t)lda * i] : A[i + (int64_t)lda * j]);
  }
}

int op_code(char op) { return (op == 'N' || op == 'n') ? 0 : (op == 'T' || op == 't') ? 1 : -1; }

// Positions: n 1, opA 2, alpha 3, A 4, lda 5, X 6, ldxp 7, beta 8, Y 9,
// ldyp 10, batch 11, ws 12, ws_bytes 13.
template <class M>
int tkron1_call(int n, char opA, typename M::io_t alpha, const typename M::io_t* A, int lda,
                const typename M::io_t* X, int64_t ldxp, typename M::io_t beta, typename M::io_t* Y, int64_t ldyp,
                int64_t batch, void* ws, size_t ws_bytes, hipStream_t stream) {
  using T = typename M::io_t;
  if (n < 1 || n > KRON_MAX_N) return -1;
  const int trans = op_code(opA);
  if (trans < 0) return -2;
  if (!A) return -4;
  if (lda < n) return -5;
  if (!X || reinterpret_cast<uintptr_t>(X) % sizeof(T) != 0) return -6;
  if (ldxp < 0) return -7;
  if (!Y || reinterpret_cast<uintptr_t>(Y) % sizeof(T) != 0 || (const void*)Y == (const void*)X) return -9;
  if (ldyp < n) return -10;
  if (batch < 0) return -11;
  if (batch == 0) return 0;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % sizeof(T) != 0) return -12;
  if (ws_bytes < (size_t)n * n * sizeof(T)) return -13;
  T* P = static_cast<T*>(ws);
  hipLaunchKernelGGL(prepare_tkron1_kernel<T>, dim3(1), dim3(256), 0, stream, n, A, lda, trans, alpha, P);
  const int64_t ntiles = (batch + 15) / 16;
  const bool vec = n == 16 && ldxp % 4 == 0 && ldyp % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(Y) % 16 == 0;
  const bool has_beta = beta != T(0);
  auto run = [&](auto k) {
    hipLaunchKernelGGL(k, dim3(grid_blocks((ntiles + 3) / 4, occupancy_blocks(k), 0)), dim3(kBlock), 0, stream, n, P,
                       X, ldxp, Y, ldyp, batch, ntiles, beta);
  };
  if (vec) {
    if (has_beta) run(kron1d_kernel<M, true, true>);
    else run(kron1d_kernel<M, true, false>);
  } else {
    if (has_beta) run(kron1d_kernel<M, false, true>);
    else run(kron1d_kernel<M, false, false>);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

// Argument checks and launches shared by the four entry points.  The
// argument positions of the C signatures: n 1, the ops 2-4, alpha 5, then
// (factor, ld) pairs from 6, then X and its strides, beta, Y and its
// strides, batch, ws, ws_bytes.
template <class M>
int strided_call(int dim, int n, const char* ops, typename M::io_t alpha, const typename M::io_t* const* mats,
                 const int* lds, const typename M::io_t* X, const int64_t* ldx, typename M::io_t beta,
                 typename M::io_t* Y, const int64_t* ldy, int64_t batch, void* ws, size_t ws_bytes,
                 hipStream_t stream) {
  using T = typename M::io_t;
  if (n < 1 || n > KRON_MAX_N) return -1;
  unsigned tmask = 0;
  bool transx = false;
  for (int f = 0; f < 3; ++f) {
    const int b = op_code(ops[f]);
    if (b < 0) return -(2 + f);
    if (f < dim) tmask |= (unsigned)b << f;
    else transx = b != 0;
  }
  int k = 6;  // position of A
  for (int f = 0; f < dim; ++f, k += 2) {
    if (!mats[f]) return -k;
    if (lds[f] < n) return -(k + 1);
  }
  // X: pointer at k, then its dim strides (ldx, [ldx2,] ldxp)
  const int kX = k, kBeta = kX + dim + 1, kY = kBeta + 1, kBatch = kY + dim + 1;
  if (!X || reinterpret_cast<uintptr_t>(X) % sizeof(T) != 0) return -kX;
  if (!Y || reinterpret_cast<uintptr_t>(Y) % sizeof(T) != 0 || (const void*)Y == (const void*)X) return -kY;
  // X is only read, so its strides may be any non-negative values (an
  // operand stride of 0 applies the action to one array batch times).  Y's
  // must give every output element its own address: ldy >= n, and each
  // further stride at least n times the previous one.
  for (int j = 0; j < dim; ++j)
    if (ldx[j] < 0) return -(kX + 1 + j);
  if (ldy[0] < n) return -(kY + 1);
  for (int j = 1; j < dim; ++j)
    if (ldy[j] < ldy[j - 1] * n) return -(kY + 1 + j);
  if (batch < 0) return -kBatch;
  if (batch == 0) return 0;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % sizeof(T) != 0) return -(kBatch + 1);
  if (ws_bytes < (size_t)dim * n * n * sizeof(T)) return -(kBatch + 2);
  T* P = static_cast<T*>(ws);
  hipLaunchKernelGGL(prepare_strided_factors_kernel<T>, dim3(1), dim3(256), 0, stream, n, dim, mats[0], lds[0],
                     mats[1], lds[1], dim == 3 ? mats[2] : mats[1], dim == 3 ? lds[2] : lds[1], tmask, alpha, P);
  const Strides xs{ldx[0], dim == 3 ? ldx[1] : 0, ldx[dim - 1]};
  const Strides ys{ldy[0], dim == 3 ? ldy[1] : 0, ldy[dim - 1]};
  const int rc = dim == 2 ? launch_strided<M, 2>(n, P, P + n * n, P + n * n, X, xs, Y, ys, batch, beta, transx, stream)
                          : launch_strided<M, 3>(n, P, P + n * n, P + 2 * n * n, X, xs, Y, ys, batch, beta, false,
                                                 stream);
  if (rc != 0) return rc;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

}  // namespace
}  // namespace kron

extern "C" {

int kron1d_batched_f32(int n, char opA, float alpha, const float* A, int lda, const float* X, int64_t ldxp,
                       float beta, float* Y, int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes,
                       hipStream_t stream) {
  return kron::tkron1_call<kron::ModeF32>(n, opA, alpha, A, lda, X, ldxp, beta, Y, ldyp, batch, ws, ws_bytes, stream);
}

int kron1d_batched_f64(int n, char opA, double alpha, const double* A, int lda, const double* X, int64_t ldxp,
                       double beta, double* Y, int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes,
                       hipStream_t stream) {
  return kron::tkron1_call<kron::ModeF64>(n, opA, alpha, A, lda, X, ldxp, beta, Y, ldyp, batch, ws, ws_bytes, stream);
}

int kron2d_batched_strided_f32(int n, char opA, char opB, char opX, float alpha, const float* A, int lda,
                               const float* B, int ldb, const float* X, int64_t ldx, int64_t ldxp, float beta,
                               float* Y, int64_t ldy, int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
  const char ops[3] = {opA, opB, opX};
  const float* mats[2] = {A, B};
  const int lds[2] = {lda, ldb};
  const int64_t lx[2] = {ldx, ldxp}, ly[2] = {ldy, ldyp};
  return kron::strided_call<kron::ModeF32>(2, n, ops, alpha, mats, lds, X, lx, beta, Y, ly, batch, ws, ws_bytes,
                                           stream);
}

int kron2d_batched_strided_f64(int n, char opA, char opB, char opX, double alpha, const double* A, int lda,
                               const double* B, int ldb, const double* X, int64_t ldx, int64_t ldxp, double beta,
                               double* Y, int64_t ldy, int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
  const char ops[3] = {opA, opB, opX};
  const double* mats[2] = {A, B};
  const int lds[2] = {lda, ldb};
  const int64_t lx[2] = {ldx, ldxp}, ly[2] = {ldy, ldyp};
  return kron::strided_call<kron::ModeF64>(2, n, ops, alpha, mats, lds, X, lx, beta, Y, ly, batch, ws, ws_bytes,
                                           stream);
}

int kron3d_batched_strided_f32(int n, char opA, char opB, char opC, float alpha, const float* A, int lda,
                               const float* B, int ldb, const float* C, int ldc, const float* X, int64_t ldx,
                               int64_t ldx2, int64_t ldxp, float beta, float* Y, int64_t ldy, int64_t ldy2,
                               int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes, hipStream_t stream) {
  const char ops[3] = {opA, opB, opC};
  const float* mats[3] = {A, B, C};
  const int lds[3] = {lda, ldb, ldc};
  const int64_t lx[3] = {ldx, ldx2, ldxp}, ly[3] = {ldy, ldy2, ldyp};
  return kron::strided_call<kron::ModeF32>(3, n, ops, alpha, mats, lds, X, lx, beta, Y, ly, batch, ws, ws_bytes,
                                           stream);
}

int kron3d_batched_strided_f64(int n, char opA, char opB, char opC, double alpha, const double* A, int lda,
                               const double* B, int ldb, const double* C, int ldc, const double* X, int64_t ldx,
                               int64_t ldx2, int64_t ldxp, double beta, double* Y, int64_t ldy, int64_t ldy2,
                               int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes, hipStream_t stream) {
  const char ops[3] = {opA, opB, opC};
  const double* mats[3] = {A, B, C};
  const int lds[3] = {lda, ldb, ldc};
  const int64_t lx[3] = {ldx, ldx2, ldxp}, ly[3] = {ldy, ldy2, ldyp};
  return kron::strided_call<kron::ModeF64>(3, n, ops, alpha, mats, lds, X, lx, beta, Y, ly, batch, ws, ws_bytes,
                                           stream);
}

}  // extern "C"
