// FP32 2-D actions, forward and transposed (plain FP32 products and sums on the
// 16x16x4 FP32 matrix-core instruction).
#include "kron_launch.hpp"

namespace kron {

int fwd2d_f32(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch, hipStream_t s,
            bool trans) {
  return trans ? launch2d<ModeF32, true>(n, A, B, X, Y, batch, s, 0)
               : launch2d<ModeF32, false>(n, A, B, X, Y, batch, s, 0);
}

}  // namespace kron
