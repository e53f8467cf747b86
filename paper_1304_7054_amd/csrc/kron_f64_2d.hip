// FP64 2-D actions, forward and transposed (16x16x4 FP64 matrix-core instruction).
#include "kron_launch.hpp"

namespace kron {

int fwd2d_f64(int n, const double* A, const double* B, const double* X, double* Y, int64_t batch, hipStream_t s,
            bool trans) {
  return trans ? launch2d<ModeF64, true>(n, A, B, X, Y, batch, s, 1)
               : launch2d<ModeF64, false>(n, A, B, X, Y, batch, s, 1);
}

}  // namespace kron
