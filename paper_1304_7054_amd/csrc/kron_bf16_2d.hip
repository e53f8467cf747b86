// bf16-storage 2-D action with FP32 sums on the bf16 matrix cores.
#include "kron_launch.hpp"

namespace kron {

int fwd2d_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* X, uint16_t* Y, int64_t batch, hipStream_t s) {
  return launch2d<ModeBF16, false>(n, A, B, X, Y, batch, s, 3);
}

}  // namespace kron
