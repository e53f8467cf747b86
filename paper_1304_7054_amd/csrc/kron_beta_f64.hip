// FP64 actions with the output update Y <- K X + beta Y (beta != 0), 2-D and 3-D.
#include "kron_launch.hpp"

namespace kron {

int beta2d_f64(int n, const double* A, const double* B, const double* X, double* Y, int64_t batch, double beta, hipStream_t s) {
  return launch_beta<ModeF64, 2>(n, A, B, B, X, Y, batch, beta, s);
}

int beta3d_f64(int n, const double* A, const double* B, const double* C, const double* X, double* Y, int64_t batch, double beta,
               hipStream_t s) {
  return launch_beta<ModeF64, 3>(n, A, B, C, X, Y, batch, beta, s);
}

}  // namespace kron
