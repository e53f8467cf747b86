/*
 * CPU oracle for the batched Kronecker-product action (Jhurani, "Batched
 * Kronecker product for 2-D matrices and 3-D arrays on NVIDIA GPUs").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or constant with the GPU library.
 *
 * Storage (Section 3, "Batched function interface"): every matrix and every
 * operand is column-major with the smallest leading dimensions, and operand p
 * starts at p*n^2 (2-D) or p*n^3 (3-D) elements, as in the measured setting of
 * Section 5.
 *
 * 2-D (Section 2, the defining identity (A (x) B) vec(X) = vec(B X A^T)):
 *     X_p is n x n, element (l, m) at l + n*m, and Y_p = B * X_p * A^T.
 *     Computed as T = B * X_p (sum over l ascending), then Y_p = T * A^T
 *     (sum over m ascending): 4 n^3 flops per operand (Section 5 flop model).
 *
 * 3-D (Section 2.1, the triple summation and vec(Y) = (C (x) B (x) A) vec(X)):
 *     the paper's operator K(P, Q, R) applies P to the fastest (first,
 *     column-major) index, Q to the middle one and R to the slowest:
 *         Y_ijk = sum_{l,m,n} P_il Q_jm R_kn X_lmn,  X_lmn at l + n*m + n^2*n'.
 *     The library's kron3d(A, B, C) is vec(Y) = (A (x) B (x) C) vec(X) on the
 *     memory-order vector, which is the paper's K(C, B, A): C contracts the
 *     fastest index, B the middle one, A the slowest.  Three mode products
 *     in the fixed order fastest, middle, slowest: 6 n^4 flops per operand.
 *
 * Gradients of L = sum_p <dY_p, Y_p> (inner product of the flattened arrays)
 * with respect to X_p and to the shared matrices, summed over the batch.
 * They are written out from the summation forms above:
 *   2-D: dX_p = B^T dY_p A;  dA = sum_p dY_p^T (B X_p);  dB = sum_p dY_p (X_p A^T)^T
 *   3-D: dX = K(C^T, B^T, A^T) dY; dA/dB/dC contract dY with X after the two
 *        other factors have been applied (see the functions below).
 *
 * The float variants keep storage and accumulation in float and must be built
 * with -ffp-contract=off so that no multiply-add is fused.
 */
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

#define ORACLE_API __attribute__((visibility("default")))

/* ---- generic bodies, instantiated for double and float ---------------- */

/* Y_p = B X_p A^T, column-major n x n, for p in [0, batch). */
#define DEFINE_KRON2D(NAME, T)                                                   \
  ORACLE_API void NAME(int n, const T* A, const T* B, const T* X, T* Y,          \
                       int64_t batch) {                                         \
    const int64_t nn = (int64_t)n * n;                                           \
    _Pragma("omp parallel for schedule(static)")                                 \
    for (int64_t p = 0; p < batch; ++p) {                                        \
      T tmp[16 * 16];                                                            \
      const T* x = X + p * nn;                                                   \
      T* y = Y + p * nn;                                                         \
      /* T = B * X: T(r, m) = sum_l B(r, l) X(l, m) */                           \
      for (int m = 0; m < n; ++m)                                                \
        for (int r = 0; r < n; ++r) {                                            \
          T s = 0;                                                               \
          for (int l = 0; l < n; ++l) s += B[r + n * l] * x[l + n * m];          \
          tmp[r + n * m] = s;                                                    \
        }                                                                        \
      /* Y = T * A^T: Y(r, c) = sum_m T(r, m) A(c, m) */                         \
      for (int c = 0; c < n; ++c)                                                \
        for (int r = 0; r < n; ++r) {                                            \
          T s = 0;                                                               \
          for (int m = 0; m < n; ++m) s += tmp[r + n * m] * A[c + n * m];        \
          y[r + n * c] = s;                                                      \
        }                                                                        \
    }                                                                            \
  }

/* Paper's K(P, Q, R) on column-major n x n x n arrays:
 *   Y(i,j,k) = sum_{l,m,q} P(i,l) Q(j,m) R(k,q) X(l,m,q),
 *   element (l, m, q) at l + n*m + n*n*q.
 * Done as three mode products: first index (P), then second (Q), then third (R). */
#define DEFINE_KPQR(NAME, T)                                                     \
  static void NAME(int n, const T* P, const T* Q, const T* R, const T* x,        \
                   T* y, T* w1, T* w2) {                                         \
    const int nn = n * n;                                                        \
    /* w1(i, m, q) = sum_l P(i, l) x(l, m, q) */                                 \
    for (int q = 0; q < n; ++q)                                                  \
      for (int m = 0; m < n; ++m)                                                \
        for (int i = 0; i < n; ++i) {                                            \
          T s = 0;                                                               \
          for (int l = 0; l < n; ++l) s += P[i + n * l] * x[l + n * m + nn * q]; \
          w1[i + n * m + nn * q] = s;                                            \
        }                                                                        \
    /* w2(i, j, q) = sum_m Q(j, m) w1(i, m, q) */                                \
    for (int q = 0; q < n; ++q)                                                  \
      for (int j = 0; j < n; ++j)                                                \
        for (int i = 0; i < n; ++i) {                                            \
          T s = 0;                                                               \
          for (int m = 0; m < n; ++m) s += Q[j + n * m] * w1[i + n * m + nn * q];\
          w2[i + n * j + nn * q] = s;                                            \
        }                                                                        \
    /* y(i, j, k) = sum_q R(k, q) w2(i, j, q) */                                 \
    for (int k = 0; k < n; ++k)                                                  \
      for (int j = 0; j < n; ++j)                                                \
        for (int i = 0; i < n; ++i) {                                            \
          T s = 0;                                                               \
          for (int q = 0; q < n; ++q) s += R[k + n * q] * w2[i + n * j + nn * q];\
          y[i + n * j + nn * k] = s;                                             \
        }                                                                        \
  }

/* vec(Y_p) = (A (x) B (x) C) vec(X_p) = paper's K(C, B, A)(X_p). */
#define DEFINE_KRON3D(NAME, KPQR, T)                                             \
  ORACLE_API void NAME(int n, const T* A, const T* B, const T* C, const T* X,    \
                       T* Y, int64_t batch) {                                    \
    const int64_t nnn = (int64_t)n * n * n;                                      \
    _Pragma("omp parallel for schedule(static)")                                 \
    for (int64_t p = 0; p < batch; ++p) {                                        \
      T w1[16 * 16 * 16], w2[16 * 16 * 16];                                      \
      KPQR(n, C, B, A, X + p * nnn, Y + p * nnn, w1, w2);                        \
    }                                                                            \
  }

DEFINE_KRON2D(oracle_kron2d_f64, double)
DEFINE_KRON2D(oracle_kron2d_f32, float)
DEFINE_KPQR(kpqr_f64, double)
DEFINE_KPQR(kpqr_f32, float)
DEFINE_KRON3D(oracle_kron3d_f64, kpqr_f64, double)
DEFINE_KRON3D(oracle_kron3d_f32, kpqr_f32, float)

/* ---- Section 3's interface on the same storage (double only) ---------------
 *   Y_p <- alpha * K(op(A), op(B)[, op(C)]) X_p + beta * Y_p,
 *   op(M) = M for 'N' (or 'n') and M^T for 'T' (or 't').
 * As in BLAS, beta == 0 means Y is not read (its old contents, even NaN, do
 * not matter).  Written out plainly: the op matrices are formed explicitly,
 * the action is taken with the functions above into a temporary, and the
 * alpha/beta update is applied element by element. */

static void op_matrix(int n, char op, const double* M, double* out) {
  const int t = (op == 'T' || op == 't');
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) out[i + n * j] = t ? M[j + n * i] : M[i + n * j];
}

static void axpby(double alpha, const double* z, double beta, double* y, int64_t count) {
  for (int64_t e = 0; e < count; ++e) y[e] = beta == 0.0 ? alpha * z[e] : alpha * z[e] + beta * y[e];
}

/* 2-D: Y_p <- alpha * K(op(A), op(B))(op(X_p)) + beta * Y_p.  Only in 2-D
 * may op act on the operands too (Section 2.2); op(X_p) is formed
 * explicitly, operand by operand, before the plain action. */
ORACLE_API void oracle_kron2d_ex_f64(int n, char opA, char opB, char opX, double alpha, const double* A,
                                     const double* B, const double* X, double beta, double* Y, int64_t batch) {
  double Ao[256], Bo[256];
  op_matrix(n, opA, A, Ao);
  op_matrix(n, opB, B, Bo);
  const int64_t nn = (int64_t)n * n, count = batch * nn;
  double* xo = (double*)calloc(count ? count : 1, sizeof(double));
  for (int64_t p = 0; p < batch; ++p) op_matrix(n, opX, X + p * nn, xo + p * nn);
  double* z = (double*)calloc(count ? count : 1, sizeof(double));
  oracle_kron2d_f64(n, Ao, Bo, xo, z, batch);
  axpby(alpha, z, beta, Y, count);
  free(z);
  free(xo);
}

ORACLE_API void oracle_kron3d_ex_f64(int n, char opA, char opB, char opC, double alpha, const double* A,
                                     const double* B, const double* C, const double* X, double beta, double* Y,
                                     int64_t batch) {
  double Ao[256], Bo[256], Co[256];
  op_matrix(n, opA, A, Ao);
  op_matrix(n, opB, B, Bo);
  op_matrix(n, opC, C, Co);
  const int64_t count = batch * n * n * n;
  double* z = (double*)calloc(count ? count : 1, sizeof(double));
  oracle_kron3d_f64(n, Ao, Bo, Co, X, z, batch);
  axpby(alpha, z, beta, Y, count);
  free(z);
}

/* 1-D (Section 3's TKRON1, a batched matrix-vector product):
 *     y_p <- alpha * op(A) x_p + beta * y_p,  p = 0 .. batch-1,
 * with x_p at X + p*ldxp and y_p at Y + p*ldyp (n elements each).  The sum
 * runs over j ascending; Y is not read when beta == 0. */
ORACLE_API void oracle_kron1d_ex_f64(int n, char opA, double alpha, const double* A, const double* X, int64_t ldxp,
                                     double beta, double* Y, int64_t ldyp, int64_t batch) {
  double Ao[256];
  op_matrix(n, opA, A, Ao);
  for (int64_t p = 0; p < batch; ++p) {
    const double* x = X + p * ldxp;
    double* y = Y + p * ldyp;
    for (int i = 0; i < n; ++i) {
      double s = 0;
      for (int j = 0; j < n; ++j) s += Ao[i + n * j] * x[j];
      y[i] = beta == 0.0 ? alpha * s : alpha * s + beta * y[i];
    }
  }
}

/* ---- gradients (double only) ------------------------------------------ */

static void transpose_n(int n, const double* M, double* Mt) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Mt[j + n * i] = M[i + n * j];
}

static double* zalloc(size_t count) { return (double*)calloc(count ? count : 1, sizeof(double)); }

/* 2-D: Y_p = B X_p A^T with L = sum_p <dY_p, Y_p>.
 *   dX_p = B^T dY_p A                                 (the adjoint action)
 *   dA(c, m) = sum_p sum_r dY_p(r, c) (B X_p)(r, m)   (dA = sum_p dY_p^T B X_p)
 *   dB(r, l) = sum_p sum_c dY_p(r, c) (X_p A^T)(l, c) (dB = sum_p dY_p A X_p^T)
 * Any output pointer may be NULL to skip it.  dA/dB are overwritten. */
ORACLE_API void oracle_kron2d_grad_f64(int n, const double* A, const double* B,
                                       const double* X, const double* dY,
                                       double* dX, double* dA, double* dB,
                                       int64_t batch) {
  const int64_t nn = (int64_t)n * n;
  if (dX) {
    double At[256], Bt[256];
    transpose_n(n, A, At);
    transpose_n(n, B, Bt);
    /* B^T dY A = Bt dY (At)^T, i.e. the forward action with (At, Bt). */
    oracle_kron2d_f64(n, At, Bt, dY, dX, batch);
  }
  if (dA) memset(dA, 0, sizeof(double) * nn);
  if (dB) memset(dB, 0, sizeof(double) * nn);
  if (!dA && !dB) return;
  for (int64_t p = 0; p < batch; ++p) {
    const double* x = X + p * nn;
    const double* dy = dY + p * nn;
    if (dA) {
      double bx[256];
      for (int m = 0; m < n; ++m)
        for (int r = 0; r < n; ++r) {
          double s = 0;
          for (int l = 0; l < n; ++l) s += B[r + n * l] * x[l + n * m];
          bx[r + n * m] = s;
        }
      for (int m = 0; m < n; ++m)
        for (int c = 0; c < n; ++c) {
          double s = 0;
          for (int r = 0; r < n; ++r) s += dy[r + n * c] * bx[r + n * m];
          dA[c + n * m] += s;
        }
    }
    if (dB) {
      double xa[256]; /* xa(l, c) = sum_m X(l, m) A(c, m) */
      for (int c = 0; c < n; ++c)
        for (int l = 0; l < n; ++l) {
          double s = 0;
          for (int m = 0; m < n; ++m) s += x[l + n * m] * A[c + n * m];
          xa[l + n * c] = s;
        }
      for (int l = 0; l < n; ++l)
        for (int r = 0; r < n; ++r) {
          double s = 0;
          for (int c = 0; c < n; ++c) s += dy[r + n * c] * xa[l + n * c];
          dB[r + n * l] += s;
        }
    }
  }
}

/* 3-D: memory index of operand element (a, b, c) is a*n^2 + b*n + c, and
 *   Y(i, j, k) = sum_{a,b,c} A(i, a) B(j, b) C(k, c) X(a, b, c),
 * with matrices column-major (A(i, a) at i + n*a).  With L = sum_p <dY_p, Y_p>:
 *   dX(a, b, c) = sum_{i,j,k} A(i, a) B(j, b) C(k, c) dY(i, j, k)
 *   dA(i, a) = sum_p sum_{j,k} dY(i, j, k) U(a, j, k),  U = X with B on b, C on c
 *   dB(j, b) = sum_p sum_{i,k} dY(i, j, k) V(i, b, k),  V = X with A on a, C on c
 *   dC(k, c) = sum_p sum_{i,j} dY(i, j, k) W(i, j, c),  W = X with A on a, B on b
 * The partial products U, V, W are formed with the same K(P, Q, R) helper by
 * passing the identity for the factor that is left out.  dA/dB/dC are
 * overwritten; any output may be NULL. */
ORACLE_API void oracle_kron3d_grad_f64(int n, const double* A, const double* B,
                                       const double* C, const double* X,
                                       const double* dY, double* dX, double* dA,
                                       double* dB, double* dC, int64_t batch) {
  const int64_t nn = (int64_t)n * n, nnn = nn * n;
  double At[256], Bt[256], Ct[256], I[256];
  transpose_n(n, A, At);
  transpose_n(n, B, Bt);
  transpose_n(n, C, Ct);
  for (int i = 0; i < n * n; ++i) I[i] = 0.0;
  for (int i = 0; i < n; ++i) I[i + n * i] = 1.0;
  if (dX) oracle_kron3d_f64(n, At, Bt, Ct, dY, dX, batch);
  if (dA) memset(dA, 0, sizeof(double) * nn);
  if (dB) memset(dB, 0, sizeof(double) * nn);
  if (dC) memset(dC, 0, sizeof(double) * nn);
  if (!dA && !dB && !dC) return;
  double* u = zalloc(nnn);
  double* w1 = zalloc(nnn);
  double* w2 = zalloc(nnn);
  for (int64_t p = 0; p < batch; ++p) {
    const double* x = X + p * nnn;
    const double* dy = dY + p * nnn;
    if (dA) { /* U = K(C, B, I) x: C on the fastest index c, B on b, a untouched */
      kpqr_f64(n, C, B, I, x, u, w1, w2);
      for (int i = 0; i < n; ++i)
        for (int a = 0; a < n; ++a) {
          double s = 0;
          for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) s += dy[i * nn + j * n + k] * u[a * nn + j * n + k];
          dA[i + n * a] += s;
        }
    }
    if (dB) { /* V = K(C, I, A) x */
      kpqr_f64(n, C, I, A, x, u, w1, w2);
      for (int j = 0; j < n; ++j)
        for (int b = 0; b < n; ++b) {
          double s = 0;
          for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) s += dy[i * nn + j * n + k] * u[i * nn + b * n + k];
          dB[j + n * b] += s;
        }
    }
    if (dC) { /* W = K(I, B, A) x */
      kpqr_f64(n, I, B, A, x, u, w1, w2);
      for (int k = 0; k < n; ++k)
        for (int c = 0; c < n; ++c) {
          double s = 0;
          for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) s += dy[i * nn + j * n + k] * u[i * nn + j * n + c];
          dC[k + n * c] += s;
        }
    }
  }
  free(u);
  free(w1);
  free(w2);
}

/* Number of OpenMP threads the oracle would use (for reporting). */
ORACLE_API int oracle_num_threads(void) {
  int t = 1;
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  t = omp_get_max_threads();
#endif
  return t;
}

/* Set the number of OpenMP threads of later calls (for timing on a given
   core count); n < 1 is ignored. */
ORACLE_API void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---- d-dimensional arrays, rectangular, complex, per-operand factors -------
 *
 * Section 2.1 generalises the action to n-D arrays for any n >= 1 (the
 * summation gains one index and one factor per dimension), Section 2.2
 * allows op(M) in {M, M^T, M^*} with op(M) of size m x n, complex entries,
 * and alpha / beta, and Section 6 names the case where the factors change
 * along the batch.  Written out for operand p:
 *
 *   Y_p(i_0, .., i_{d-1}) <- alpha * sum_{a_0, .., a_{d-1}}
 *        op(F_0)(i_0, a_0) * .. * op(F_{d-1})(i_{d-1}, a_{d-1}) * X_p(a_0, .., a_{d-1})
 *      + beta * Y_p(i_0, .., i_{d-1})
 *
 * with the library's convention that the last index is the fastest in
 * memory (element (a_0, .., a_{d-1}) of X_p at sum_k a_k * prod_{j>k} n_j, and
 * vec(Y_p) = (op(F_0) (x) .. (x) op(F_{d-1})) vec(X_p)).  X_p has extents
 * n_0 .. n_{d-1} and starts at p * prod(n); Y_p has extents m_0 .. m_{d-1}
 * and starts at p * prod(m).  F_k of operand p starts at F[k] + p * ldfp[k]
 * (ldfp[k] = 0: one matrix shared by the batch) and is stored column-major
 * with leading dimension ldf[k]; the stored matrix is m_k x n_k for 'N' and
 * n_k x m_k for 'T' / 'C' ('C' also conjugates).  beta == 0 does not read Y.
 *
 * Computed as d mode products, fastest index first: contracting index k
 * replaces extent n_k by m_k.  Complex numbers are (re, im) pairs of doubles.
 */
#include <complex.h>

#define ND_MAX_DIM 8

static int64_t nd_prod(const int* e, int d) {
  int64_t s = 1;
  for (int k = 0; k < d; ++k) s *= e[k];
  return s;
}

/* op(F)(i, a) for the stored matrix M with leading dimension ld */
#define ND_OP_ENTRY(T, CONJ, M, ld, op, i, a)                                        \
  ((op) == 'N' || (op) == 'n' ? (M)[(i) + (int64_t)(ld) * (a)]                       \
   : ((op) == 'T' || (op) == 't') ? (M)[(a) + (int64_t)(ld) * (i)]                   \
   : CONJ((M)[(a) + (int64_t)(ld) * (i)]))

#define DEFINE_KRON_ND(NAME, T, CONJ)                                                \
  static void NAME(int d, const int* m, const int* n, const char* ops, T alpha,      \
                   const T* const* F, const int* ldf, const int64_t* ldfp,           \
                   const T* X, T beta, T* Y, int64_t batch) {                        \
    const int64_t nx = nd_prod(n, d), ny = nd_prod(m, d);                            \
    int64_t big = 1; /* largest intermediate: max over passes of its extents */      \
    for (int k = d; k >= 0; --k) {                                                   \
      int e[ND_MAX_DIM];                                                             \
      for (int j = 0; j < d; ++j) e[j] = j < k ? n[j] : m[j];                        \
      const int64_t s = nd_prod(e, d);                                               \
      if (s > big) big = s;                                                          \
    }                                                                                \
    _Pragma("omp parallel for schedule(dynamic)")                                    \
    for (int64_t p = 0; p < batch; ++p) {                                            \
      T* cur = (T*)malloc(sizeof(T) * big);                                          \
      T* nxt = (T*)malloc(sizeof(T) * big);                                          \
      int e[ND_MAX_DIM];                                                             \
      for (int j = 0; j < d; ++j) e[j] = n[j];                                       \
      for (int64_t q = 0; q < nx; ++q) cur[q] = X[p * nx + q];                       \
      for (int k = d - 1; k >= 0; --k) {                                             \
        /* cur has extents e; contract index k: pre x n_k x post -> pre x m_k x post */ \
        int64_t pre = 1, post = 1;                                                   \
        for (int j = 0; j < k; ++j) pre *= e[j];                                     \
        for (int j = k + 1; j < d; ++j) post *= e[j];                                \
        const T* M = F[k] + p * ldfp[k];                                             \
        for (int64_t u = 0; u < pre; ++u)                                            \
          for (int i = 0; i < m[k]; ++i)                                             \
            for (int64_t v = 0; v < post; ++v) {                                     \
              T s = 0;                                                               \
              for (int a = 0; a < n[k]; ++a)                                         \
                s += ND_OP_ENTRY(T, CONJ, M, ldf[k], ops[k], i, a) *                 \
                     cur[(u * n[k] + a) * post + v];                                 \
              nxt[(u * m[k] + i) * post + v] = s;                                    \
            }                                                                        \
        e[k] = m[k];                                                                 \
        T* t = cur; cur = nxt; nxt = t;                                              \
      }                                                                              \
      for (int64_t q = 0; q < ny; ++q) {                                             \
        T v = alpha * cur[q];                                                        \
        Y[p * ny + q] = beta == (T)0 ? v : v + beta * Y[p * ny + q];                 \
      }                                                                              \
      free(cur);                                                                     \
      free(nxt);                                                                     \
    }                                                                                \
  }

#define ND_NO_CONJ(x) (x)
DEFINE_KRON_ND(kron_nd_real, double, ND_NO_CONJ)
DEFINE_KRON_ND(kron_nd_cplx, double _Complex, conj)

/* Real FP64. */
ORACLE_API void oracle_kron_nd_f64(int d, const int* m, const int* n, const char* ops, double alpha,
                                   const double* const* F, const int* ldf, const int64_t* ldfp, const double* X,
                                   double beta, double* Y, int64_t batch) {
  kron_nd_real(d, m, n, ops, alpha, F, ldf, ldfp, X, beta, Y, batch);
}

/* Complex FP64: every array holds (re, im) pairs of doubles. */
ORACLE_API void oracle_kron_nd_z64(int d, const int* m, const int* n, const char* ops, double alpha_re,
                                   double alpha_im, const double* const* F, const int* ldf, const int64_t* ldfp,
                                   const double* X, double beta_re, double beta_im, double* Y, int64_t batch) {
  const double _Complex alpha = alpha_re + alpha_im * I, beta = beta_re + beta_im * I;
  kron_nd_cplx(d, m, n, ops, alpha, (const double _Complex* const*)F, ldf, ldfp, (const double _Complex*)X, beta,
               (double _Complex*)Y, batch);
}
