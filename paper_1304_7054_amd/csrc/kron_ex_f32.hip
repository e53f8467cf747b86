// FP32 actions of the extended interface that the plain kernels do not
// cover: the output update Y <- K X + beta Y (beta != 0), 2-D and 3-D, and
// 2-D operands read transposed.
#include "kron_launch.hpp"

namespace kron {

int ex2d_f32(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch, float beta, bool transx,
             hipStream_t s) {
  return launch_ex<ModeF32, 2>(n, A, B, B, X, Y, batch, beta, transx, s);
}

int ex3d_f32(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch, float beta,
             hipStream_t s) {
  return launch_ex<ModeF32, 3>(n, A, B, C, X, Y, batch, beta, false, s);
}

}  // namespace kron
