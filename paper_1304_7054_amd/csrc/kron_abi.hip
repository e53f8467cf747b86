// C ABI of libkron: argument checks, status codes and dispatch to the
// per-mode launchers.  The declarations and their documentation are in
// include/kron.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "kron.h"
#include "kron_runtime.hpp"

namespace kron {

constexpr int kNumModesAbi = 5;  // modes the launch table and the autotuner know

int device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    cache[dev].store(cus, std::memory_order_relaxed);
    v = cus;
  }
  return v;
}

namespace {
constexpr int kNumModes = kNumModesAbi;
// Launch shapes per (mode, dim - 2, n), packed as blocks_per_cu * 16 + variant.
// -1 = not set: the built-in default applies.
std::atomic<int> g_shape[kNumModes][2][17];

void init_shapes() {
  // thread-safe one-time initialisation (C++11 static local)
  static const bool done = [] {
    for (auto& m : g_shape)
      for (auto& d : m)
        for (auto& v : d) v.store(-1, std::memory_order_relaxed);
    return true;
  }();
  (void)done;
}

// Built-in defaults, measured on MI355X at n = 16 with 1 GiB batches (the
// autotuner refines them per n).
LaunchShape default_shape(int mode, int dim, int n) {
  if (n != 16) return LaunchShape{0, dim == 2 ? 3 : 8};  // staged through LDS
  if (dim == 3) {
    switch (mode) {
      case 0: return LaunchShape{2, 9};   // FP32: stores interleaved with the next tile, 2-slab window
      case 1: return LaunchShape{2, 7};   // FP64: 4-slab window + next tile
      case 2: return LaunchShape{2, 9};   // bf16x3: as FP32
      case 4: return LaunchShape{2, 9};   // bf16x6: as FP32
      default: return LaunchShape{0, 10}; // bf16 storage: stores interleaved, 4-slab window
    }
  }
  switch (mode) {
    case 0: return LaunchShape{2, 0};  // FP32 2-D: 4 tiles in flight, 2 workgroups per CU
    case 1: return LaunchShape{3, 1};  // FP64 2-D: 8 tiles in flight, 3 workgroups per CU
    default: return LaunchShape{0, 0};
  }
}
}  // namespace

LaunchShape launch_shape(int mode, int dim, int n) {
  init_shapes();
  if (mode < 0 || mode >= kNumModes || dim < 2 || dim > 3 || n < 1 || n > 16) return LaunchShape{0, 0};
  const int v = g_shape[mode][dim - 2][n].load(std::memory_order_relaxed);
  if (v < 0) return default_shape(mode, dim, n);
  return LaunchShape{v >> 4, v & 15};
}

int set_launch_shape(int mode, int dim, int n, int blocks_per_cu, int variant) {
  init_shapes();
  if (mode < 0 || mode >= kNumModes) return -1;
  if (dim < 2 || dim > 3) return -2;
  if (n < 1 || n > 16) return -3;
  if (blocks_per_cu < -1 || blocks_per_cu > 64) return -4;
  if (variant < 0 || variant > (dim == 3 ? 11 : 4)) return -5;
  g_shape[mode][dim - 2][n].store(blocks_per_cu < 0 ? -1 : blocks_per_cu * 16 + variant, std::memory_order_relaxed);
  return 0;
}

int fwd3d_f32(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
              hipStream_t s, bool trans) {
  return n <= 8 ? fwd3d_f32_lo(n, A, B, C, X, Y, batch, s, trans) : fwd3d_f32_hi(n, A, B, C, X, Y, batch, s, trans);
}
int fwd3d_f64(int n, const double* A, const double* B, const double* C, const double* X, double* Y,
              int64_t batch, hipStream_t s, bool trans) {
  return n <= 8 ? fwd3d_f64_lo(n, A, B, C, X, Y, batch, s, trans) : fwd3d_f64_hi(n, A, B, C, X, Y, batch, s, trans);
}
int fwd3d_bf16x3(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                 hipStream_t s) {
  return n <= 8 ? fwd3d_bf16x3_lo(n, A, B, C, X, Y, batch, s) : fwd3d_bf16x3_hi(n, A, B, C, X, Y, batch, s);
}
int fwd3d_bf16x6(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                 hipStream_t s) {
  return n <= 8 ? fwd3d_bf16x6_lo(n, A, B, C, X, Y, batch, s) : fwd3d_bf16x6_hi(n, A, B, C, X, Y, batch, s);
}
int fwd3d_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* C, const uint16_t* X, uint16_t* Y,
               int64_t batch, hipStream_t s) {
  return n <= 8 ? fwd3d_bf16_lo(n, A, B, C, X, Y, batch, s) : fwd3d_bf16_hi(n, A, B, C, X, Y, batch, s);
}

}  // namespace kron

namespace {

// Launch errors surface through hipGetLastError; return them as positive codes.
int finish_launch(int rc) {
  if (rc != 0) return rc;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

// Common checks of the forward entry points.  Argument positions follow the
// C signatures: n is 1, then the factors, then X, Y, batch.
int check2d(int n, const void* A, const void* B, const void* X, const void* Y, int64_t batch) {
  if (n < 1 || n > KRON_MAX_N) return -1;
  if (!A) return -2;
  if (!B) return -3;
  if (!X) return -4;
  if (!Y || Y == X) return -5;
  if (batch < 0) return -6;
  return 0;
}

int check3d(int n, const void* A, const void* B, const void* C, const void* X, const void* Y, int64_t batch) {
  if (n < 1 || n > KRON_MAX_N) return -1;
  if (!A) return -2;
  if (!B) return -3;
  if (!C) return -4;
  if (!X) return -5;
  if (!Y || Y == X) return -6;
  if (batch < 0) return -7;
  return 0;
}

// op(M) per factor and alpha on the first factor, written once to `out`
// (factor f at out + f * n^2, column-major).
template <typename T>
__global__ __launch_bounds__(256) void kron_prepare_factors_kernel(int n, int nf, const T* __restrict__ A,
                                                                   const T* __restrict__ B, const T* __restrict__ C,
                                                                   unsigned tmask, T alpha, T* __restrict__ out) {
  const int nn = n * n;
  for (int e = threadIdx.x; e < nf * nn; e += blockDim.x) {
    const int f = e / nn, idx = e % nn, i = idx % n, j = idx / n;
    const T* M = f == 0 ? A : f == 1 ? B : C;
    const T v = ((tmask >> f) & 1u) ? M[j + n * i] : M[i + n * j];
    out[e] = f == 0 ? alpha * v : v;
  }
}

// 0 for 'N'/'n', 1 for 'T'/'t', -1 otherwise
int op_bit(char op) { return (op == 'N' || op == 'n') ? 0 : (op == 'T' || op == 't') ? 1 : -1; }

// Checks and factor preparation shared by the extended entry points.
// Positions follow their C signatures: n, the ops (one per factor, then opX
// in 2-D), alpha, the factors, X, beta, Y, batch, ws, ws_bytes.  Returns 0,
// with the prepared factors being written to ws on `stream` and *transx set,
// or -k.
template <typename T>
int prepare_ex(int dim, int n, const char* ops, T alpha, const T* const* mats, const T* X, const T* Y,
               int64_t batch, void* ws, size_t ws_bytes, hipStream_t stream, bool* skip, bool* transx) {
  *skip = false;
  *transx = false;
  if (n < 1 || n > KRON_MAX_N) return -1;
  const int nops = 3;  // 2-D: opA, opB, opX; 3-D: opA, opB, opC
  unsigned tmask = 0;
  for (int f = 0; f < nops; ++f) {
    const int b = op_bit(ops[f]);
    if (b < 0) return -(2 + f);
    if (f < dim) tmask |= (unsigned)b << f;
    else *transx = b != 0;
  }
  const int kA = nops + 3;  // position of A (after n, the ops and alpha)
  for (int f = 0; f < dim; ++f)
    if (!mats[f]) return -(kA + f);
  const int kX = kA + dim;
  if (!X) return -kX;
  if (!Y || (const void*)Y == (const void*)X) return -(kX + 2);
  if (batch < 0) return -(kX + 3);
  if (batch == 0) {
    *skip = true;
    return 0;
  }
  if (!ws || reinterpret_cast<uintptr_t>(ws) % sizeof(T) != 0) return -(kX + 4);
  if (ws_bytes < (size_t)dim * n * n * sizeof(T)) return -(kX + 5);
  hipLaunchKernelGGL(kron_prepare_factors_kernel<T>, dim3(1), dim3(256), 0, stream, n, dim, mats[0], mats[1],
                     dim == 3 ? mats[2] : mats[1], tmask, alpha, static_cast<T*>(ws));
  return 0;
}

}  // namespace

namespace {

// Shared checks of the backward entry points.  k0 is the position of X.
template <typename T>
int check_backward(int dim, int n, const T* X, const T* dY, const T* dX, const void* gA, const void* gB,
                   const void* gC, int64_t batch, const void* ws, size_t ws_bytes, int k0) {
  const bool factors = gA || gB || gC;
  if (factors && !X && batch > 0) return -k0;
  if (!dY && batch > 0) return -(k0 + 1);
  if (dX && (dX == dY || dX == X)) return -(k0 + 2);
  const int kb = k0 + 3 + dim;  // position of batch
  if (batch < 0) return -kb;
  if (factors && batch > 0) {
    if (!ws) return -(kb + 1);
    if (ws_bytes < kron::grad_workspace_bytes(dim, n, batch, (int)sizeof(T))) return -(kb + 2);
  }
  return 0;
}

}  // namespace

namespace {

// Shared body of the 3-D FP32 extended entry points: checks, factor
// preparation into ws, then the plain kernels (beta == 0) or the beta kernel
// on the prepared factors, all on `stream`.
int ex3d_f32_call(int n, char opA, char opB, char opC, float alpha, const float* A, const float* B, const float* C,
                  const float* X, float beta, float* Y, int64_t batch, void* ws, size_t ws_bytes,
                  hipStream_t stream) {
  const char ops[3] = {opA, opB, opC};
  const float* mats[3] = {A, B, C};
  bool skip, transx;
  if (int rc = prepare_ex<float>(3, n, ops, alpha, mats, X, Y, batch, ws, ws_bytes, stream, &skip, &transx))
    return rc;
  if (skip) return 0;
  const float* P = static_cast<const float*>(ws);
  return finish_launch(beta != 0.0f ? kron::ex3d_f32(n, P, P + n * n, P + 2 * n * n, X, Y, batch, beta, stream)
                                     : kron::fwd3d_f32(n, P, P + n * n, P + 2 * n * n, X, Y, batch, stream, false));
}

// The allocation-free entry point's workspace: the three prepared n x n
// FP32 factors of one call (3 KiB at n = 16).  Every device holds its own
// copy for the life of the process.  Host code never passes the array's
// name to a kernel: it is a host-side stand-in, not a device address.  The
// device address is looked up once per device (with that device current)
// and kept per device ordinal.
constexpr size_t kNoAllocScratchBytes = 3 * KRON_MAX_N * KRON_MAX_N * sizeof(float);
static __device__ __align__(256) float scratch[kNoAllocScratchBytes / sizeof(float)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device; 0 or a hipError_t.
int noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!p) return (int)hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace

extern "C" {

int kron2d_batched_f32(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch,
                       hipStream_t stream) {
  if (int rc = check2d(n, A, B, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd2d_f32(n, A, B, X, Y, batch, stream, false));
}

int kron2d_batched_f64(int n, const double* A, const double* B, const double* X, double* Y, int64_t batch,
                       hipStream_t stream) {
  if (int rc = check2d(n, A, B, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd2d_f64(n, A, B, X, Y, batch, stream, false));
}

int kron3d_batched_f32(int n, const float* A, const float* B, const float* C, const float* X, float* Y,
                       int64_t batch, hipStream_t stream) {
  if (int rc = check3d(n, A, B, C, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd3d_f32(n, A, B, C, X, Y, batch, stream, false));
}

int kron3d_batched_f64(int n, const double* A, const double* B, const double* C, const double* X, double* Y,
                       int64_t batch, hipStream_t stream) {
  if (int rc = check3d(n, A, B, C, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd3d_f64(n, A, B, C, X, Y, batch, stream, false));
}

int kron2d_batched_f32_bf16x3(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch,
                              hipStream_t stream) {
  if (int rc = check2d(n, A, B, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd2d_bf16x3(n, A, B, X, Y, batch, stream));
}

int kron3d_batched_f32_bf16x3(int n, const float* A, const float* B, const float* C, const float* X, float* Y,
                              int64_t batch, hipStream_t stream) {
  if (int rc = check3d(n, A, B, C, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd3d_bf16x3(n, A, B, C, X, Y, batch, stream));
}

int kron2d_batched_f32_bf16x6(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch,
                              hipStream_t stream) {
  if (int rc = check2d(n, A, B, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd2d_bf16x6(n, A, B, X, Y, batch, stream));
}

int kron3d_batched_f32_bf16x6(int n, const float* A, const float* B, const float* C, const float* X, float* Y,
                              int64_t batch, hipStream_t stream) {
  if (int rc = check3d(n, A, B, C, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd3d_bf16x6(n, A, B, C, X, Y, batch, stream));
}

int kron2d_batched_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* X, uint16_t* Y,
                        int64_t batch, hipStream_t stream) {
  if (int rc = check2d(n, A, B, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd2d_bf16(n, A, B, X, Y, batch, stream));
}

int kron3d_batched_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* C, const uint16_t* X,
                        uint16_t* Y, int64_t batch, hipStream_t stream) {
  if (int rc = check3d(n, A, B, C, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd3d_bf16(n, A, B, C, X, Y, batch, stream));
}

int kron2d_batched_adjoint_f32(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch,
                               hipStream_t stream) {
  if (int rc = check2d(n, A, B, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd2d_f32(n, A, B, X, Y, batch, stream, true));
}

int kron3d_batched_adjoint_f32(int n, const float* A, const float* B, const float* C, const float* X, float* Y,
                               int64_t batch, hipStream_t stream) {
  if (int rc = check3d(n, A, B, C, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd3d_f32(n, A, B, C, X, Y, batch, stream, true));
}

int kron2d_batched_adjoint_f64(int n, const double* A, const double* B, const double* X, double* Y,
                               int64_t batch, hipStream_t stream) {
  if (int rc = check2d(n, A, B, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd2d_f64(n, A, B, X, Y, batch, stream, true));
}

int kron3d_batched_adjoint_f64(int n, const double* A, const double* B, const double* C, const double* X,
                               double* Y, int64_t batch, hipStream_t stream) {
  if (int rc = check3d(n, A, B, C, X, Y, batch)) return rc;
  if (batch == 0) return 0;
  return finish_launch(kron::fwd3d_f64(n, A, B, C, X, Y, batch, stream, true));
}

size_t kron_backward_workspace_size(int dim, int n, int64_t batch, int mode) {
  if ((dim != 2 && dim != 3) || n < 1 || n > KRON_MAX_N || batch < 0) return 0;
  if (mode != KRON_MODE_F32 && mode != KRON_MODE_F64) return 0;
  return kron::grad_workspace_bytes(dim, n, batch, mode == KRON_MODE_F64 ? 8 : 4);
}


int kron2d_backward_f32(int n, const float* A, const float* B, const float* X, const float* dY, float* dX,
                        float* dA, float* dB, int64_t batch, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (n < 1 || n > KRON_MAX_N) return -1;
  if (!A) return -2;
  if (!B) return -3;
  if (int rc = check_backward<float>(2, n, X, dY, dX, dA, dB, nullptr, batch, ws, ws_bytes, 4)) return rc;
  if (dX && batch > 0) {
    if (int rc = finish_launch(kron::fwd2d_f32(n, A, B, dY, dX, batch, stream, true))) return rc;
  }
  if (dA || dB) return finish_launch(kron::grad2d_f32(n, A, B, X, dY, dA, dB, batch, ws, stream));
  return 0;
}

int kron3d_backward_f32(int n, const float* A, const float* B, const float* C, const float* X, const float* dY,
                        float* dX, float* dA, float* dB, float* dC, int64_t batch, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  if (n < 1 || n > KRON_MAX_N) return -1;
  if (!A) return -2;
  if (!B) return -3;
  if (!C) return -4;
  if (int rc = check_backward<float>(3, n, X, dY, dX, dA, dB, dC, batch, ws, ws_bytes, 5)) return rc;
  if (n == 16 && (dA || dB || dC) && kron::backward3d16_usable(X, dY, dX))
    return finish_launch(kron::backward3d16_f32(A, B, C, X, dY, dX, dA, dB, dC, batch, ws, stream));
  if (dX && batch > 0) {
    if (int rc = finish_launch(kron::fwd3d_f32(n, A, B, C, dY, dX, batch, stream, true))) return rc;
  }
  if (dA || dB || dC) return finish_launch(kron::grad3d_f32(n, A, B, C, X, dY, dA, dB, dC, batch, ws, stream));
  return 0;
}

int kron2d_backward_f64(int n, const double* A, const double* B, const double* X, const double* dY, double* dX,
                        double* dA, double* dB, int64_t batch, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (n < 1 || n > KRON_MAX_N) return -1;
  if (!A) return -2;
  if (!B) return -3;
  if (int rc = check_backward<double>(2, n, X, dY, dX, dA, dB, nullptr, batch, ws, ws_bytes, 4)) return rc;
  if (dX && batch > 0) {
    if (int rc = finish_launch(kron::fwd2d_f64(n, A, B, dY, dX, batch, stream, true))) return rc;
  }
  if (dA || dB) return finish_launch(kron::grad2d_f64(n, A, B, X, dY, dA, dB, batch, ws, stream));
  return 0;
}

int kron3d_backward_f64(int n, const double* A, const double* B, const double* C, const double* X,
                        const double* dY, double* dX, double* dA, double* dB, double* dC, int64_t batch, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
  if (n < 1 || n > KRON_MAX_N) return -1;
  if (!A) return -2;
  if (!B) return -3;
  if (!C) return -4;
  if (int rc = check_backward<double>(3, n, X, dY, dX, dA, dB, dC, batch, ws, ws_bytes, 5)) return rc;
  if (dX && batch > 0) {
    if (int rc = finish_launch(kron::fwd3d_f64(n, A, B, C, dY, dX, batch, stream, true))) return rc;
  }
  if (dA || dB || dC) return finish_launch(kron::grad3d_f64(n, A, B, C, X, dY, dA, dB, dC, batch, ws, stream));
  return 0;
}

}  // extern "C"

namespace {

// Validity of one backward group descriptor (before anything is launched).
bool grad_group_ok(const kron_group_grad_t& d) {
  if ((d.dim != 2 && d.dim != 3) || d.n < 1 || d.n > KRON_MAX_N || d.count < 0) return false;
  if (d.mode != KRON_MODE_F32 && d.mode != KRON_MODE_F64) return false;
  if (d.count == 0) return true;
  if (!d.A || !d.B || (d.dim == 3 && !d.C) || !d.dY) return false;
  const bool factors = d.dA || d.dB || (d.dim == 3 && d.dC);
  if (factors && !d.X) return false;
  if (d.dX && (d.dX == d.dY || d.dX == d.X)) return false;
  return true;
}

// Workspace slice of one group: its backward workspace, 256-byte aligned.
size_t grad_group_bytes(const kron_group_grad_t& d) {
  const size_t b = kron_backward_workspace_size(d.dim, d.n, d.count, d.mode);
  return (b + 255) / 256 * 256;
}

}  // namespace

extern "C" {

size_t kron_grouped_backward_workspace_size(const kron_group_grad_t* groups, int ngroups) {
  if (!groups || ngroups < 1) return 0;
  size_t total = 0;
  for (int i = 0; i < ngroups; ++i) {
    if (!grad_group_ok(groups[i])) return 0;
    total += grad_group_bytes(groups[i]);
  }
  return total;
}

namespace {

// Streams the grouped backward spreads its groups over (per device, created
// on first use, default priority, never destroyed): one group's kernels are
// too small to fill the GPU on their own.
constexpr int kBwdStreams = 8;
std::mutex g_bwd_mu;
hipStream_t g_bwd_streams[64][kBwdStreams];
bool g_bwd_ready[64];

const hipStream_t* bwd_streams() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_bwd_mu);
  if (!g_bwd_ready[dev]) {
    for (int i = 0; i < kBwdStreams; ++i) {
      if (hipStreamCreateWithFlags(&g_bwd_streams[dev][i], hipStreamNonBlocking) != hipSuccess) {
        for (int j = 0; j < i; ++j) (void)hipStreamDestroy(g_bwd_streams[dev][j]);
        return nullptr;
      }
    }
    g_bwd_ready[dev] = true;
  }
  return g_bwd_streams[dev];
}

int grad_group_run(const kron_group_grad_t& d, void* w, size_t b, hipStream_t stream) {
  if (d.mode == KRON_MODE_F32) {
    using T = float;
    if (d.dim == 2)
      return kron2d_backward_f32(d.n, (const T*)d.A, (const T*)d.B, (const T*)d.X, (const T*)d.dY, (T*)d.dX,
                                 (T*)d.dA, (T*)d.dB, d.count, w, b, stream);
    return kron3d_backward_f32(d.n, (const T*)d.A, (const T*)d.B, (const T*)d.C, (const T*)d.X, (const T*)d.dY,
                               (T*)d.dX, (T*)d.dA, (T*)d.dB, (T*)d.dC, d.count, w, b, stream);
  }
  using T = double;
  if (d.dim == 2)
    return kron2d_backward_f64(d.n, (const T*)d.A, (const T*)d.B, (const T*)d.X, (const T*)d.dY, (T*)d.dX,
                               (T*)d.dA, (T*)d.dB, d.count, w, b, stream);
  return kron3d_backward_f64(d.n, (const T*)d.A, (const T*)d.B, (const T*)d.C, (const T*)d.X, (const T*)d.dY,
                             (T*)d.dX, (T*)d.dA, (T*)d.dB, (T*)d.dC, d.count, w, b, stream);
}

}  // namespace

int kron_grouped_backward(const kron_group_grad_t* groups, int ngroups, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
  if (!groups) return -1;
  if (ngroups < 1) return -2;
  size_t need = 0;
  for (int i = 0; i < ngroups; ++i) {
    if (!grad_group_ok(groups[i])) return -1;
    need += grad_group_bytes(groups[i]);
  }
  if (need > 0 && !ws) return -3;
  if (ws_bytes < need) return -4;
  // Fork: the worker streams wait for the work already on `stream`; the
  // groups go to them in turn; join: `stream` waits for every worker.  Each
  // group's kernels stay in order on one stream, and its result does not
  // depend on what runs beside it.  Without worker streams (or with one
  // group) the groups run on `stream` in descriptor order.
  const hipStream_t* workers = ngroups > 1 ? bwd_streams() : nullptr;
  hipEvent_t fork = nullptr;
  if (workers) {
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) {
      workers = nullptr;
    } else {
      hipError_t e = hipEventRecord(fork, stream);
      for (int w = 0; w < kBwdStreams && e == hipSuccess; ++w) e = hipStreamWaitEvent(workers[w], fork, 0);
      if (e != hipSuccess) {
        (void)hipEventDestroy(fork);
        return (int)e;
      }
    }
  }
  // Each group's workspace slice, in descriptor order.
  std::vector<size_t> off(ngroups);
  {
    size_t o = 0;
    for (int i = 0; i < ngroups; ++i) {
      off[i] = o;
      o += grad_group_bytes(groups[i]);
    }
  }
  // Largest groups first, each to the stream with the least work so far
  // (elements read and written, plus a fixed cost per group for its launches).
  std::vector<int> order(ngroups);
  std::vector<double> cost(ngroups);
  for (int i = 0; i < ngroups; ++i) {
    const kron_group_grad_t& d = groups[i];
    const double e = (double)d.count * (d.dim == 3 ? (double)d.n * d.n * d.n : (double)d.n * d.n);
    cost[i] = 3.0 * e + 2.0e5;
    order[i] = i;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  double load[kBwdStreams] = {};
  uint8_t* base = static_cast<uint8_t*>(ws);
  int rc = 0;
  for (int k = 0; k < ngroups && rc == 0; ++k) {
    const int i = order[k];
    const kron_group_grad_t& d = groups[i];
    const size_t b = grad_group_bytes(d);
    hipStream_t s = stream;
    if (workers) {
      int w = 0;
      for (int j = 1; j < kBwdStreams; ++j)
        if (load[j] < load[w]) w = j;
      load[w] += cost[i];
      s = workers[w];
    }
    // descriptors were checked above, so only a launch failure can end the loop
    rc = grad_group_run(d, b ? base + off[i] : nullptr, b, s);
  }
  if (workers) {
    for (int w = 0; w < kBwdStreams; ++w) {
      hipEvent_t done = nullptr;
      hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(done, workers[w]);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, done, 0);
      if (done) (void)hipEventDestroy(done);
      if (e != hipSuccess && rc == 0) rc = (int)e;
    }
    (void)hipEventDestroy(fork);
  }
  if (rc > 0) return rc;
  if (rc < 0) return -1;
  return 0;
}

size_t kron_grouped_workspace_size(const kron_group_t* groups, int ngroups) {
  return kron::grouped_workspace_bytes(groups, ngroups);
}

int kron_grouped_prepare(const kron_group_t* groups, int ngroups, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!groups) return -1;
  if (ngroups <= 0) return -2;
  return kron::grouped_prepare(groups, ngroups, ws, ws_bytes, stream);
}

int kron_grouped_launch(const void* ws, hipStream_t stream) {
  if (!ws) return -1;
  return finish_launch(kron::grouped_launch(ws, stream));
}

int kron_graph_capture_grouped(const void* ws, void** graph_exec) {
  if (!ws) return -1;
  if (!graph_exec) return -2;
  *graph_exec = nullptr;
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return (int)e;
  hipGraph_t graph = nullptr;
  int rc = 0;
  e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = kron::grouped_launch(ws, s);
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (rc == 0 && e2 != hipSuccess) rc = (int)e2;
  } else {
    rc = (int)e;
  }
  if (rc == 0) {
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = (int)e;
    else *graph_exec = exec;
  }
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(s);
  return rc;
}

int kron_graph_launch(void* graph_exec, hipStream_t stream) {
  if (!graph_exec) return -1;
  hipError_t e = hipGraphLaunch(static_cast<hipGraphExec_t>(graph_exec), stream);
  return e == hipSuccess ? 0 : (int)e;
}

int kron_graph_destroy(void* graph_exec) {
  if (!graph_exec) return -1;
  hipError_t e = hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph_exec));
  return e == hipSuccess ? 0 : (int)e;
}

size_t kron_ex_workspace_size(int dim, int n, int mode) {
  if ((dim != 2 && dim != 3) || n < 1 || n > KRON_MAX_N) return 0;
  if (mode != KRON_MODE_F32 && mode != KRON_MODE_F64) return 0;
  return (size_t)dim * n * n * (mode == KRON_MODE_F64 ? 8 : 4);
}

int kron2d_batched_ex_f32(int n, char opA, char opB, char opX, float alpha, const float* A, const float* B,
                          const float* X, float beta, float* Y, int64_t batch, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
  const char ops[3] = {opA, opB, opX};
  const float* mats[2] = {A, B};
  bool skip, transx;
  if (int rc = prepare_ex<float>(2, n, ops, alpha, mats, X, Y, batch, ws, ws_bytes, stream, &skip, &transx))
    return rc;
  if (skip) return 0;
  const float* P = static_cast<const float*>(ws);
  return finish_launch(beta != 0.0f || transx ? kron::ex2d_f32(n, P, P + n * n, X, Y, batch, beta, transx, stream)
                                              : kron::fwd2d_f32(n, P, P + n * n, X, Y, batch, stream, false));
}

int kron2d_batched_ex_f64(int n, char opA, char opB, char opX, double alpha, const double* A, const double* B,
                          const double* X, double beta, double* Y, int64_t batch, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
  const char ops[3] = {opA, opB, opX};
  const double* mats[2] = {A, B};
  bool skip, transx;
  if (int rc = prepare_ex<double>(2, n, ops, alpha, mats, X, Y, batch, ws, ws_bytes, stream, &skip, &transx))
    return rc;
  if (skip) return 0;
  const double* P = static_cast<const double*>(ws);
  return finish_launch(beta != 0.0 || transx ? kron::ex2d_f64(n, P, P + n * n, X, Y, batch, beta, transx, stream)
                                             : kron::fwd2d_f64(n, P, P + n * n, X, Y, batch, stream, false));
}

int kron3d_batched_ex_f32(int n, char opA, char opB, char opC, float alpha, const float* A, const float* B,
                          const float* C, const float* X, float beta, float* Y, int64_t batch, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
  return ex3d_f32_call(n, opA, opB, opC, alpha, A, B, C, X, beta, Y, batch, ws, ws_bytes, stream);
}

// The allocation-free variant: the prepared factors go to this library's
// own device array instead of a caller workspace.
int kron3d_batched_ex_f32_noalloc(int n, char opA, char opB, char opC, float alpha, const float* A,
                                  const float* B, const float* C, const float* X, float beta, float* Y,
                                  int64_t batch, hipStream_t stream) {
  if (n < 1 || n > KRON_MAX_N) return -1;
  if ((size_t)3 * n * n * sizeof(float) > kNoAllocScratchBytes) return -1;  // beyond the array's capacity
  void* ws = nullptr;
  if (int rc = noalloc_scratch(&ws)) return rc;
  return ex3d_f32_call(n, opA, opB, opC, alpha, A, B, C, X, beta, Y, batch, ws, kNoAllocScratchBytes, stream);
}

int kron3d_batched_ex_f64(int n, char opA, char opB, char opC, double alpha, const double* A, const double* B,
                          const double* C, const double* X, double beta, double* Y, int64_t batch, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
  const char ops[3] = {opA, opB, opC};
  const double* mats[3] = {A, B, C};
  bool skip, transx;
  if (int rc = prepare_ex<double>(3, n, ops, alpha, mats, X, Y, batch, ws, ws_bytes, stream, &skip, &transx))
    return rc;
  if (skip) return 0;
  const double* P = static_cast<const double*>(ws);
  return finish_launch(beta != 0.0 ? kron::ex3d_f64(n, P, P + n * n, P + 2 * n * n, X, Y, batch, beta, stream)
                                    : kron::fwd3d_f64(n, P, P + n * n, P + 2 * n * n, X, Y, batch, stream, false));
}

const char* kron_status_string(int status) {
  if (status == 0) return "success";
  if (status < 0) {
    static const char* names[] = {"invalid argument 1", "invalid argument 2",  "invalid argument 3",
                                  "invalid argument 4", "invalid argument 5",  "invalid argument 6",
                                  "invalid argument 7", "invalid argument 8",  "invalid argument 9",
                                  "invalid argument 10", "invalid argument 11", "invalid argument 12",
                                  "invalid argument 13", "invalid argument 14", "invalid argument 15"};
    int k = -status;
    return k <= 15 ? names[k - 1] : "invalid argument";
  }
  return hipGetErrorString((hipError_t)status);
}

const char* kron_version(void) { return "kron 0.1 gfx950"; }

int kron_set_launch(int mode, int dim, int n, int blocks_per_cu, int variant) {
  return kron::set_launch_shape(mode, dim, n, blocks_per_cu, variant);
}

int kron_autotune(int mode, int dim, int n, const void* A, const void* B, const void* C, const void* X, void* Y,
                  int64_t batch, int reps, hipStream_t stream, int* best_blocks, int* best_variant,
                  float* best_ms) {
  if (mode < 0 || mode >= kron::kNumModesAbi) return -1;
  if (dim < 2 || dim > 3) return -2;
  if (n < 1 || n > KRON_MAX_N) return -3;
  if (!A) return -4;
  if (!B) return -5;
  if (dim == 3 && !C) return -6;
  if (!X) return -7;
  if (!Y || Y == X) return -8;
  if (batch <= 0) return -9;
  if (reps < 1) return -10;
  auto run = [&]() -> int {
    switch (mode * 2 + (dim - 2)) {
      case 0: return kron2d_batched_f32(n, (const float*)A, (const float*)B, (const float*)X, (float*)Y, batch, stream);
      case 1: return kron3d_batched_f32(n, (const float*)A, (const float*)B, (const float*)C, (const float*)X, (float*)Y, batch, stream);
      case 2: return kron2d_batched_f64(n, (const double*)A, (const double*)B, (const double*)X, (double*)Y, batch, stream);
      case 3: return kron3d_batched_f64(n, (const double*)A, (const double*)B, (const double*)C, (const double*)X, (double*)Y, batch, stream);
      case 4: return kron2d_batched_f32_bf16x3(n, (const float*)A, (const float*)B, (const float*)X, (float*)Y, batch, stream);
      case 5: return kron3d_batched_f32_bf16x3(n, (const float*)A, (const float*)B, (const float*)C, (const float*)X, (float*)Y, batch, stream);
      case 8: return kron2d_batched_f32_bf16x6(n, (const float*)A, (const float*)B, (const float*)X, (float*)Y, batch, stream);
      case 9: return kron3d_batched_f32_bf16x6(n, (const float*)A, (const float*)B, (const float*)C, (const float*)X, (float*)Y, batch, stream);
      case 6: return kron2d_batched_bf16(n, (const uint16_t*)A, (const uint16_t*)B, (const uint16_t*)X, (uint16_t*)Y, batch, stream);
      default: return kron3d_batched_bf16(n, (const uint16_t*)A, (const uint16_t*)B, (const uint16_t*)C, (const uint16_t*)X, (uint16_t*)Y, batch, stream);
    }
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return (int)e;
  }
  // candidate variants: 2-D 0-3 plus 4 (n != 16); 3-D 0-7 plus 9-10
  // (n = 16) or 8 and 11 (other n)
  int vars[12], nvar = 0;
  for (int v = 0; v <= (dim == 3 ? 11 : 4); ++v) {
    bool use;
    if (dim == 2) use = v < 4 || n != 16;
    else if (v == 8 || v == 11) use = n != 16;
    else if (v == 9 || v == 10) use = n == 16;
    else use = true;
    if (use) vars[nvar++] = v;
  }
  const int blocks[] = {0, 1, 2, 3, 4};
  constexpr int kNB = sizeof(blocks) / sizeof(blocks[0]);
  // Every shape is timed in three sweeps (forward, reverse, forward) and
  // scored by its mean: clocks that are still rising during the first shapes
  // of a sweep cannot decide the choice, and neither can one lucky timing of
  // a shape whose time varies from launch to launch.  Each timing follows
  // three untimed launches of the same shape.
  constexpr int kSweeps = 3;
  float times[11 * kNB];
  for (float& t : times) t = 0.f;
  int rc = 0;
  const int nshape = nvar * kNB;
  for (int sweep = 0; sweep < kSweeps && rc == 0; ++sweep) {
    for (int q = 0; q < nshape && rc == 0; ++q) {
      const int idx = sweep % 2 == 0 ? q : nshape - 1 - q;
      const int v = vars[idx / kNB], b = blocks[idx % kNB];
      kron::set_launch_shape(mode, dim, n, b, v);
      for (int w = 0; w < 3 && rc == 0; ++w) rc = run();  // warm-up (first: code object load)
      if (rc != 0) break;
      if ((e = hipEventRecord(e0, stream)) != hipSuccess) { rc = (int)e; break; }
      for (int r = 0; r < reps && rc == 0; ++r) rc = run();
      if (rc != 0) break;
      if ((e = hipEventRecord(e1, stream)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
        rc = (int)e;
        break;
      }
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { rc = (int)e; break; }
      times[idx] += ms / (float)reps / (float)kSweeps;
    }
  }
  float best = 3.4e38f;
  int bb = 0, bv = 0;
  for (int idx = 0; idx < nshape; ++idx)
    if (times[idx] < best) {
      best = times[idx];
      bv = vars[idx / kNB];
      bb = blocks[idx % kNB];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != 0) {
    kron::set_launch_shape(mode, dim, n, -1, 0);
    return rc;
  }
  kron::set_launch_shape(mode, dim, n, bb, bv);
  if (best_blocks) *best_blocks = bb;
  if (best_variant) *best_variant = bv;
  if (best_ms) *best_ms = best;
  return 0;
}

int kron_get_launch(int mode, int dim, int n, int* blocks_per_cu, int* variant) {
  if (mode < 0 || mode >= kron::kNumModesAbi) return -1;
  if (dim < 2 || dim > 3) return -2;
  if (n < 1 || n > 16) return -3;
  if (!blocks_per_cu) return -4;
  if (!variant) return -5;
  const kron::LaunchShape sh = kron::launch_shape(mode, dim, n);
  *blocks_per_cu = sh.blocks_per_cu;
  *variant = sh.variant;
  return 0;
}

}  // extern "C"
