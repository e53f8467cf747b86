// bf16 storage with FP32 sums on the bf16 matrix cores.
#include "kron_launch.hpp"

namespace kron {

int fwd2d_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* X, uint16_t* Y, int64_t batch,
               hipStream_t s) {
  return launch2d<ModeBF16, false>(n, A, B, X, Y, batch, s, 3);
}

int fwd3d_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* C, const uint16_t* X, uint16_t* Y,
               int64_t batch, hipStream_t s) {
  return launch3d<ModeBF16, false>(n, A, B, C, X, Y, batch, s, 3);
}

}  // namespace kron
