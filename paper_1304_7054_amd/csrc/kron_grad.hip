// Launch of the factor-gradient kernels (FP32 and FP64).
#include "kron_grad.hpp"
#include "kron_launch.hpp"

namespace kron {

// Wavefronts of the partial kernel: a fixed function of the batch and the
// device, so the summation order (and the result) is the same on every call.
int64_t grad_waves(int dim, int n, int64_t batch) {
  const int64_t q = 16 / n;
  const int64_t ops = dim == 3 ? q * q * q : q * q;
  const int64_t ntiles = (batch + ops - 1) / ops;
  const int64_t cap = (int64_t)device_cus() * 8;
  int64_t w = ntiles < cap ? ntiles : cap;
  w = (w + 3) / 4 * 4;  // whole 256-thread workgroups
  return w < 4 ? 4 : w;
}

size_t grad_workspace_bytes(int dim, int n, int64_t batch, int elem_bytes) {
  return (size_t)grad_waves(dim, n, batch) * 3 * 256 * (size_t)elem_bytes;
}

template <class M, int N, int Dim>
int grad_n(const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
           const typename M::io_t* X, const typename M::io_t* dY, typename M::io_t* dA, typename M::io_t* dB,
           typename M::io_t* dC, int64_t batch, void* ws, hipStream_t stream) {
  using T = typename M::elem_t;
  constexpr int64_t q = Geo<N>::Q;
  constexpr int64_t ops = Dim == 3 ? q * q * q : q * q;
  const int64_t ntiles = (batch + ops - 1) / ops;
  const int which = (dA ? 1 : 0) | (dB ? 2 : 0) | (dC ? 4 : 0);
  T* part = static_cast<T*>(ws);
  int64_t nwaves = 0;
  if (batch > 0) {
    nwaves = grad_waves(Dim, N, batch);
    hipLaunchKernelGGL((kron_grad_partial_kernel<M, N, Dim>), dim3((unsigned)(nwaves / 4)), dim3(kGradBlock), 0,
                       stream, A, B, C, X, dY, part, batch, ntiles, which);
  }
  hipLaunchKernelGGL((kron_grad_reduce_kernel<typename M::io_t, T, N>), dim3(3 * N * N), dim3(kGradBlock), 0, stream,
                     part, nwaves, dA, dB, dC);
  return 0;
}

// 3-D n = 16 FP32 with 16-byte aligned arrays: dX and the factor gradients
// in one pass (kron3d_backward16_kernel), then the shared reduction.  The
// workgroup count is a fixed function of the batch and the device.
int backward3d16_f32(const float* A, const float* B, const float* C, const float* X, const float* dY, float* dX,
                     float* dA, float* dB, float* dC, int64_t batch, void* ws, hipStream_t stream) {
  const int which = (dA ? 1 : 0) | (dB ? 2 : 0) | (dC ? 4 : 0);
  float* part = static_cast<float*>(ws);
  int64_t nblocks = 0;
  if (batch > 0) {
    const int64_t cap = (int64_t)device_cus() * occupancy_blocks(kron3d_backward16_kernel);
    nblocks = batch < cap ? batch : cap;
    hipLaunchKernelGGL(kron3d_backward16_kernel, dim3((unsigned)nblocks), dim3(kGradBlock), 0, stream, A, B, C, X,
                       dY, dX, part, batch, which);
  }
  if (which) {
    hipLaunchKernelGGL((kron_grad_reduce_kernel<float, float, 16>), dim3(3 * 16 * 16), dim3(kGradBlock), 0, stream,
                       part, nblocks, dA, dB, dC);
  }
  return 0;
}

bool backward3d16_usable(const void* X, const void* dY, const void* dX) {
  const uintptr_t m = 15;
  return (((uintptr_t)X | (uintptr_t)dY | (uintptr_t)dX) & m) == 0;
}

template <class M, int Dim>
int grad_dispatch(int n, const typename M::io_t* A, const typename M::io_t* B, const typename M::io_t* C,
                  const typename M::io_t* X, const typename M::io_t* dY, typename M::io_t* dA,
                  typename M::io_t* dB, typename M::io_t* dC, int64_t batch, void* ws, hipStream_t s) {
  switch (n) {
#define KRON_CASE(NN) \
  case NN:            \
    return grad_n<M, NN, Dim>(A, B, C, X, dY, dA, dB, dC, batch, ws, s);
    KRON_N_CASES(KRON_CASE)
#undef KRON_CASE
    default:
      return -1;
  }
}

int grad2d_f32(int n, const float* A, const float* B, const float* X, const float* dY, float* dA, float* dB,
               int64_t batch, void* ws, hipStream_t s) {
  return grad_dispatch<ModeF32, 2>(n, A, B, nullptr, X, dY, dA, dB, nullptr, batch, ws, s);
}
int grad3d_f32(int n, const float* A, const float* B, const float* C, const float* X, const float* dY, float* dA,
               float* dB, float* dC, int64_t batch, void* ws, hipStream_t s) {
  return grad_dispatch<ModeF32, 3>(n, A, B, C, X, dY, dA, dB, dC, batch, ws, s);
}
int grad2d_f64(int n, const double* A, const double* B, const double* X, const double* dY, double* dA, double* dB,
               int64_t batch, void* ws, hipStream_t s) {
  return grad_dispatch<ModeF64, 2>(n, A, B, nullptr, X, dY, dA, dB, nullptr, batch, ws, s);
}
int grad3d_f64(int n, const double* A, const double* B, const double* C, const double* X, const double* dY,
               double* dA, double* dB, double* dC, int64_t batch, void* ws, hipStream_t s) {
  return grad_dispatch<ModeF64, 3>(n, A, B, C, X, dY, dA, dB, dC, batch, ws, s);
}

}  // namespace kron
