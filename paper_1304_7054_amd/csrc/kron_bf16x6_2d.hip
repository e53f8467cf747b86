// FP32 in/out 2-D action through the bf16x6 three-way split on the bf16 matrix cores.
#include "kron_launch.hpp"

namespace kron {

int fwd2d_bf16x6(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch, hipStream_t s) {
  return launch2d<ModeBF16x6, false>(n, A, B, X, Y, batch, s, 4);
}

}  // namespace kron
