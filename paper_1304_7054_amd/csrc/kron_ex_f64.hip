// FP64 actions of the extended interface that the plain kernels do not
// cover: the output update Y <- K X + beta Y (beta != 0), 2-D and 3-D, and
// 2-D operands read transposed.
#include "kron_launch.hpp"

namespace kron {

int ex2d_f64(int n, const double* A, const double* B, const double* X, double* Y, int64_t batch, double beta, bool transx,
             hipStream_t s) {
  return launch_ex<ModeF64, 2>(n, A, B, B, X, Y, batch, beta, transx, s);
}

int ex3d_f64(int n, const double* A, const double* B, const double* C, const double* X, double* Y, int64_t batch, double beta,
             hipStream_t s) {
  return launch_ex<ModeF64, 3>(n, A, B, C, X, Y, batch, beta, false, s);
}

}  // namespace kron
