// Host runtime shared by the translation units of libkron: device facts,
// launch tuning table and the per-mode launch entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct kron_group;

namespace kron {

// Compute units of the current device (cached per device ordinal).
int device_cus();

// Launch shape for (mode, dim, n): workgroups per CU (0 = as many as are
// resident at once) and kernel variant.  Defaults come from a table measured
// on MI355X; kron_set_launch / kron_autotune replace them.
struct LaunchShape {
  int blocks_per_cu;
  int variant;
};
LaunchShape launch_shape(int mode, int dim, int n);
int set_launch_shape(int mode, int dim, int n, int blocks_per_cu, int variant);

// Forward launches of each precision mode, defined in kron_<mode>.hip.
// Return 0, or -1 for an n outside 1..16.
int fwd2d_f32(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch, hipStream_t s,
              bool trans);
int fwd3d_f32(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
              hipStream_t s, bool trans);
int fwd2d_f64(int n, const double* A, const double* B, const double* X, double* Y, int64_t batch, hipStream_t s,
              bool trans);
int fwd3d_f64(int n, const double* A, const double* B, const double* C, const double* X, double* Y,
              int64_t batch, hipStream_t s, bool trans);
int fwd2d_bf16x3(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch, hipStream_t s);
int fwd3d_bf16x3(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                 hipStream_t s);
int fwd2d_bf16x6(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch, hipStream_t s);
int fwd3d_bf16x6(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                 hipStream_t s);
int fwd2d_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* X, uint16_t* Y, int64_t batch,
               hipStream_t s);
int fwd3d_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* C, const uint16_t* X, uint16_t* Y,
               int64_t batch, hipStream_t s);

// 3-D launches split by n range (kron_<mode>_3d_lo/hi.hip).
int fwd3d_f32_lo(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                hipStream_t s, bool trans);
int fwd3d_f32_hi(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                hipStream_t s, bool trans);
int fwd3d_f64_lo(int n, const double* A, const double* B, const double* C, const double* X, double* Y, int64_t batch,
                hipStream_t s, bool trans);
int fwd3d_f64_hi(int n, const double* A, const double* B, const double* C, const double* X, double* Y, int64_t batch,
                hipStream_t s, bool trans);
int fwd3d_bf16x3_lo(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                hipStream_t s);
int fwd3d_bf16x3_hi(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                hipStream_t s);
int fwd3d_bf16x6_lo(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                hipStream_t s);
int fwd3d_bf16x6_hi(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                hipStream_t s);
int fwd3d_bf16_lo(int n, const uint16_t* A, const uint16_t* B, const uint16_t* C, const uint16_t* X, uint16_t* Y, int64_t batch,
                hipStream_t s);
int fwd3d_bf16_hi(int n, const uint16_t* A, const uint16_t* B, const uint16_t* C, const uint16_t* X, uint16_t* Y, int64_t batch,
                hipStream_t s);

// Y <- K(op(X)) + beta Y (kron_ex_<mode>.hip) for beta != 0 or, in 2-D,
// transposed operands (transx); alpha and op on the factors are already in
// the factors.  Return 0, -1 for an n outside 1..16, or -2 when beta == 0
// and !transx (the plain kernels cover that case).
int ex2d_f32(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch, float beta, bool transx,
             hipStream_t s);
int ex3d_f32(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
             float beta, hipStream_t s);
int ex2d_f64(int n, const double* A, const double* B, const double* X, double* Y, int64_t batch, double beta,
             bool transx, hipStream_t s);
int ex3d_f64(int n, const double* A, const double* B, const double* C, const double* X, double* Y, int64_t batch,
             double beta, hipStream_t s);

// Grouped launch (kron_grouped.hip).
size_t grouped_workspace_bytes(const struct kron_group* g, int ngroups);
int grouped_prepare(const struct kron_group* g, int ngroups, void* ws, size_t ws_bytes, hipStream_t stream);
int grouped_launch(const void* ws, hipStream_t stream);

// Factor gradients (kron_grad.hip).  ws holds grad_workspace_bytes().
int64_t grad_waves(int dim, int n, int64_t batch);
size_t grad_workspace_bytes(int dim, int n, int64_t batch, int elem_bytes);
int grad2d_f32(int n, const float* A, const float* B, const float* X, const float* dY, float* dA, float* dB,
               int64_t batch, void* ws, hipStream_t s);
int grad3d_f32(int n, const float* A, const float* B, const float* C, const float* X, const float* dY, float* dA,
               float* dB, float* dC, int64_t batch, void* ws, hipStream_t s);
// 3-D n = 16 FP32 backward in one pass (dX and the factor gradients); usable
// when X, dY and dX (if given) are 16-byte aligned.
int backward3d16_f32(const float* A, const float* B, const float* C, const float* X, const float* dY, float* dX,
                     float* dA, float* dB, float* dC, int64_t batch, void* ws, hipStream_t stream);
bool backward3d16_usable(const void* X, const void* dY, const void* dX);
int grad2d_f64(int n, const double* A, const double* B, const double* X, const double* dY, double* dA, double* dB,
               int64_t batch, void* ws, hipStream_t s);
int grad3d_f64(int n, const double* A, const double* B, const double* C, const double* X, const double* dY,
               double* dA, double* dB, double* dC, int64_t batch, void* ws, hipStream_t s);

}  // namespace kron
