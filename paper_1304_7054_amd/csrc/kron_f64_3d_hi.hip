// FP64 3-D actions, forward and transposed, n in [9, 16] (16x16x4 FP64
// matrix-core instruction).
#include "kron_launch.hpp"

namespace kron {

int fwd3d_f64_hi(int n, const double* A, const double* B, const double* C, const double* X, double* Y, int64_t batch,
                    hipStream_t s, bool trans) {
  return trans ? launch3d_range<ModeF64, true, 9, 16>(n, A, B, C, X, Y, batch, s, 1)
               : launch3d_range<ModeF64, false, 9, 16>(n, A, B, C, X, Y, batch, s, 1);
}

}  // namespace kron
