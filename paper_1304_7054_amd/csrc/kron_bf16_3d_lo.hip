// bf16-storage 3-D action with FP32 sums, n in [1, 8].
#include "kron_launch.hpp"

namespace kron {

int fwd3d_bf16_lo(int n, const uint16_t* A, const uint16_t* B, const uint16_t* C, const uint16_t* X, uint16_t* Y, int64_t batch,
                     hipStream_t s) {
  return launch3d_range<ModeBF16, false, 1, 8>(n, A, B, C, X, Y, batch, s, 3);
}

}  // namespace kron
