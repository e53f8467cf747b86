// FP32 actions with the output update Y <- K X + beta Y (beta != 0), 2-D and 3-D.
#include "kron_launch.hpp"

namespace kron {

int beta2d_f32(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch, float beta, hipStream_t s) {
  return launch_beta<ModeF32, 2>(n, A, B, B, X, Y, batch, beta, s);
}

int beta3d_f32(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch, float beta,
               hipStream_t s) {
  return launch_beta<ModeF32, 3>(n, A, B, C, X, Y, batch, beta, s);
}

}  // namespace kron
