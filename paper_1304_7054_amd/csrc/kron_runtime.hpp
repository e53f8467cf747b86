// Host runtime shared by the translation units of libkron: device facts,
// launch tuning table and the per-mode launch entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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
int fwd2d_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* X, uint16_t* Y, int64_t batch,
               hipStream_t s);
int fwd3d_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* C, const uint16_t* X, uint16_t* Y,
               int64_t batch, hipStream_t s);

}  // namespace kron
