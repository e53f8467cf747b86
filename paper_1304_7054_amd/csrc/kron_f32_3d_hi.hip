// FP32 3-D actions, forward and transposed, n in [9, 16] (plain FP32
// products and sums on the 16x16x4 FP32 matrix-core instruction).
#include "kron_launch.hpp"

namespace kron {

int fwd3d_f32_hi(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                    hipStream_t s, bool trans) {
  return trans ? launch3d_range<ModeF32, true, 9, 16>(n, A, B, C, X, Y, batch, s, 0)
               : launch3d_range<ModeF32, false, 9, 16>(n, A, B, C, X, Y, batch, s, 0);
}

}  // namespace kron
