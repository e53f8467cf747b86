// FP32 in/out 3-D action through the bf16x6 three-way split, n in [1, 8].
#include "kron_launch.hpp"

namespace kron {

int fwd3d_bf16x6_lo(int n, const float* A, const float* B, const float* C, const float* X, float* Y, int64_t batch,
                       hipStream_t s) {
  return launch3d_range<ModeBF16x6, false, 1, 8>(n, A, B, C, X, Y, batch, s, 4);
}

}  // namespace kron
