// FP32 forward and transposed actions (plain FP32 products and sums on the
// 16x16x4 FP32 matrix-core instruction).
#include "kron_launch.hpp"

namespace kron {

int fwd2d_f32(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch, hipStream_t s,
              bool trans) {
  return trans ? launch2d<ModeF32, true>(n, A, B, X, Y, batch, s, 0)
               : launch2d<ModeF32, false>(n, A, B, X, Y, batch, s, 0);
}

int fwd3d_f32(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
              hipStream_t s, bool trans) {
  return trans ? launch3d<ModeF32, true>(n, A, B, C, X, Y, batch, s, 0)
               : launch3d<ModeF32, false>(n, A, B, C, X, Y, batch, s, 0);
}

}  // namespace kron
