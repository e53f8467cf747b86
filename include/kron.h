/*
 * kron.h -- C ABI of the MI355X (gfx950) batched Kronecker-product action.
 *
 * Operation (Jhurani, "Batched Kronecker product for 2-D matrices and 3-D
 * arrays on NVIDIA GPUs"):
 *
 *   2-D, Section 2, the identity (A (x) B) vec(X) = vec(B X A^T):
 *       Y_p = B * X_p * A^T                       for p = 0 .. batch-1
 *   3-D, Section 2.1, the triple summation and its vec form:
 *       vec(Y_p) = (A (x) B (x) C) vec(X_p)
 *     which is the paper's K(C, B, A): C acts on the fastest memory index,
 *     B on the middle one and A on the slowest.  With operand element
 *     (a, b, c) stored at a*n*n + b*n + c:
 *       Y_p(i, j, k) = sum_{a,b,c} A(i, a) B(j, b) C(k, c) X_p(a, b, c).
 *   Both are the batched update of Section 2.2 with alpha = 1, beta = 0 and
 *   op = N everywhere (the setting the paper measures in Section 5).  The
 *   general update (alpha, beta, op on the factors and on 2-D operands,
 *   leading dimensions) and the 1-D TKRON1 of Section 3 have entry points
 *   of their own further below.
 *
 * Layout (Section 3): every matrix is n x n column-major with leading
 * dimension n (element (i, j) at i + n*j); operands are packed back to back
 * with the smallest strides (n*n for 2-D, n*n*n for 3-D), 2-D operands
 * column-major.  One rule covers both: vec(Y_p) = kron(F1, kron(F2, ...))
 * vec(X_p) on memory-order vectors, with the factors in argument order.
 * 1 <= n <= 16 (the paper's size range, Table 1).
 *
 * Ownership: the caller owns all memory; every pointer is a device pointer
 * (the grouped and backward entry points also take a caller-owned device
 * workspace; see their notes).  The library never allocates device memory
 * (the work-array convention of Section 4).  Calls are asynchronous on
 * `stream` (0 = the null stream) unless noted.
 *
 * Aliasing: X and Y must not overlap; X == Y is rejected, partial overlap is
 * undefined.  In the plain entry points Y is write-only (beta = 0): its
 * previous contents, NaN included, never reach the result.
 *
 * Return value: 0 on success; -k when argument k (1-based) is invalid;
 * a positive hipError_t when a HIP call fails.  batch == 0 returns 0 and
 * launches nothing.  kron_status_string() names any status.
 */
#ifndef KRON_H
#define KRON_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KRON_SUCCESS 0
#define KRON_MAX_N 16

/* Precision modes (the grouped descriptors and the autotuner use them). */
enum kron_mode {
  KRON_MODE_F32 = 0,    /* FP32 in/out, FP32 products and sums */
  KRON_MODE_F64 = 1,    /* FP64 in/out, FP64 products and sums */
  KRON_MODE_BF16X3 = 2, /* FP32 in/out; each FP32 factor split into bf16 hi + lo,
                           products hi*hi' + hi*lo' + lo*hi' on bf16 matrix cores,
                           FP32 sums */
  KRON_MODE_BF16 = 3,   /* bf16 storage of A, B, C, X, Y (uint16_t bit patterns),
                           FP32 sums, intermediates kept as bf16 hi + lo pairs,
                           output rounded to nearest even */
  KRON_MODE_BF16X6 = 4  /* FP32 in/out; each FP32 value split three ways into bf16
                           h + m + l (all 24 bits), six bf16 products per FP32 product
                           (terms below 2^-23 dropped), FP32 sums */
};

/* ---- plain forward ------------------------------------------------------- */

/* Y_p = B X_p A^T (2-D, Section 2), FP32.  A, B: n*n; X, Y: batch*n*n. */
int kron2d_batched_f32(int n, const float* A, const float* B, const float* X,
                       float* Y, int64_t batch, hipStream_t stream);
/* Same in FP64. */
int kron2d_batched_f64(int n, const double* A, const double* B, const double* X,
                       double* Y, int64_t batch, hipStream_t stream);

/* vec(Y_p) = (A (x) B (x) C) vec(X_p) (3-D, Section 2.1), FP32.
   A, B, C: n*n; X, Y: batch*n^3. */
int kron3d_batched_f32(int n, const float* A, const float* B, const float* C,
                       const float* X, float* Y, int64_t batch, hipStream_t stream);
/* Same in FP64. */
int kron3d_batched_f64(int n, const double* A, const double* B, const double* C,
                       const double* X, double* Y, int64_t batch, hipStream_t stream);

/* ---- precision modes (same operations, same layouts) -------------------- */

/* FP32 in/out computed with the bf16x3 split on bf16 matrix cores
   (KRON_MODE_BF16X3).  The split keeps 16 significant bits of every value:
   on N(0,1) data and on the log-uniform precision workload at n = 16 the
   normwise error stays within FP32's 1e-5 gate; on log-uniform data at
   small n (few dominant products per output) it can reach about 2e-5. */
int kron2d_batched_f32_bf16x3(int n, const float* A, const float* B, const float* X,
                              float* Y, int64_t batch, hipStream_t stream);
int kron3d_batched_f32_bf16x3(int n, const float* A, const float* B, const float* C,
                              const float* X, float* Y, int64_t batch, hipStream_t stream);

/* FP32 in/out computed with the three-way bf16x6 split (KRON_MODE_BF16X6):
   every value is held exactly as three bf16 parts and each FP32 product is
   formed from six bf16 products on the matrix cores, so the results are as
   accurate as plain FP32 on any data (normwise and per operand). */
int kron2d_batched_f32_bf16x6(int n, const float* A, const float* B, const float* X,
                              float* Y, int64_t batch, hipStream_t stream);
int kron3d_batched_f32_bf16x6(int n, const float* A, const float* B, const float* C,
                              const float* X, float* Y, int64_t batch, hipStream_t stream);

/* bf16 storage (KRON_MODE_BF16): every array holds bf16 bit patterns
   (uint16_t); sums in FP32; Y rounded to nearest even. */
int kron2d_batched_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* X,
                        uint16_t* Y, int64_t batch, hipStream_t stream);
int kron3d_batched_bf16(int n, const uint16_t* A, const uint16_t* B, const uint16_t* C,
                        const uint16_t* X, uint16_t* Y, int64_t batch, hipStream_t stream);

/* ---- transposed action (the adjoint) ------------------------------------ */

/* The same actions with every factor transposed: Y_p = B^T X_p A (2-D) and
   vec(Y_p) = (A^T (x) B^T (x) C^T) vec(X_p) (3-D).  The paper transposes the
   constant matrices once instead of per operand (Section 2.2); here the
   transpose is folded into how each wave loads the factors.  This is the
   gradient with respect to X. */
int kron2d_batched_adjoint_f32(int n, const float* A, const float* B, const float* X,
                               float* Y, int64_t batch, hipStream_t stream);
int kron3d_batched_adjoint_f32(int n, const float* A, const float* B, const float* C,
                               const float* X, float* Y, int64_t batch, hipStream_t stream);
int kron2d_batched_adjoint_f64(int n, const double* A, const double* B, const double* X,
                               double* Y, int64_t batch, hipStream_t stream);
int kron3d_batched_adjoint_f64(int n, const double* A, const double* B, const double* C,
                               const double* X, double* Y, int64_t batch, hipStream_t stream);

/* ---- mixed batches: one launch over many groups ----------------------------- */

/* One group of operands sharing the factors A, B (and C for dim 3), stored as
   for kron2d/kron3d_batched; `mode` is KRON_MODE_F32 or KRON_MODE_BF16X3
   (FP32 arrays).  C may be NULL for dim 2. */
typedef struct kron_group {
  int32_t dim;      /* 2 or 3 */
  int32_t n;        /* 1..16 */
  int32_t mode;     /* KRON_MODE_F32 or KRON_MODE_BF16X3 */
  int32_t reserved; /* set to 0 */
  const void* A;
  const void* B;
  const void* C;
  const void* X;
  void* Y;
  int64_t count; /* operands in the group, >= 0 */
} kron_group_t;

/* The batched action of Section 2.2 over a batch that mixes sizes and 2-D /
   3-D operands, in two persistent kernel launches (2-D groups, then 3-D
   groups; one graph capture holds both).  kron_grouped_prepare builds the
   plan on the host and copies it into `ws`, caller-owned device memory of
   at least kron_grouped_workspace_size() bytes; it synchronises `stream`.
   The plan orders each phase's groups, cuts their tiles into chunks that
   shrink towards the end of the sequence, and holds one counter per phase
   from which the kernels' wavefronts claim chunks; the last wavefront of a
   launch resets the counter, so every launch (and graph replay) starts from
   the prepared state.  Launches that share one `ws` must therefore be
   ordered (same stream, or synchronised): concurrent ones race on the
   counter.  Results do not depend on which wavefront ran which chunk.  The
   plan keeps the group pointers: the arrays must stay valid while it is
   used.  kron_grouped_launch(ws) runs every group; it is asynchronous and
   takes no host-side work besides the launches.  The plan is bound to this
   process and to the device it was prepared on; preparing the same `ws`
   again replaces it.  Returns 0 or -k (argument k invalid: -1 also for any
   bad group descriptor; -4 workspace too small). */
size_t kron_grouped_workspace_size(const kron_group_t* groups, int ngroups);
int kron_grouped_prepare(const kron_group_t* groups, int ngroups, void* ws, size_t ws_bytes,
                         hipStream_t stream);
int kron_grouped_launch(const void* ws, hipStream_t stream);

/* HIP graphs for launch-bound callers: capture one kron_grouped_launch(ws)
   into an instantiated graph (`*graph_exec`), replay it on any stream, and
   release it.  Capture happens on a private stream of default priority. */
int kron_graph_capture_grouped(const void* ws, void** graph_exec);
int kron_graph_launch(void* graph_exec, hipStream_t stream);
int kron_graph_destroy(void* graph_exec);

/* ---- Section 3's interface: per-factor op, alpha and beta ---------------------- */

/* Y_p <- alpha * K(op(A), op(B)[, op(C)]) X_p + beta * Y_p (Section 2.2's
   batched update) with op(M) = M ('N' or 'n') or M^T ('T' or 't'), on the
   same storage as the plain entry points (2-D: Y_p = alpha * op(B) op(X_p)
   op(A)^T + beta * Y_p, where opX may transpose each operand as the paper's
   2-D interface allows; 3-D: vec(Y_p) = alpha * (op(A) (x) op(B) (x) op(C))
   vec(X_p) + beta * vec(Y_p)).  Following the paper's transpose-once remark
   (Section 2.2), op and alpha are applied once to the n x n factors, written
   to the caller's workspace `ws` (device memory aligned to the element size,
   at least kron_ex_workspace_size(dim, n, mode) bytes, mode KRON_MODE_F32 or
   KRON_MODE_F64; owned by the caller).
   beta == 0: Y is written and never read (NaN in Y does not propagate), and
   the plain forward kernels run on the prepared factors, so the batch costs
   the same as the plain call.
   beta != 0: every output element is read once and updated in place by the
   lane that computes it (one more pass over Y; NaN in Y propagates as in
   BLAS).
   opX = 'T' (2-D): each X_p is read transposed by the computing lanes (no
   copy of X is made).
   Returns 0 or -k (argument k invalid; a bad op character counts as
   invalid); batch == 0 is a no-op.  Asynchronous on `stream`; `ws` must stay
   valid until the call's kernels have run. */
size_t kron_ex_workspace_size(int dim, int n, int mode);
int kron2d_batched_ex_f32(int n, char opA, char opB, char opX, float alpha, const float* A, const float* B,
                          const float* X, float beta, float* Y, int64_t batch, void* ws, size_t ws_bytes,
                          hipStream_t stream);
int kron2d_batched_ex_f64(int n, char opA, char opB, char opX, double alpha, const double* A, const double* B,
                          const double* X, double beta, double* Y, int64_t batch, void* ws, size_t ws_bytes,
                          hipStream_t stream);
int kron3d_batched_ex_f32(int n, char opA, char opB, char opC, float alpha, const float* A, const float* B,
                          const float* C, const float* X, float beta, float* Y, int64_t batch, void* ws,
                          size_t ws_bytes, hipStream_t stream);
int kron3d_batched_ex_f64(int n, char opA, char opB, char opC, double alpha, const double* A, const double* B,
                          const double* C, const double* X, double beta, double* Y, int64_t batch, void* ws,
                          size_t ws_bytes, hipStream_t stream);

/* ---- the general action: d dimensions, rectangular, complex, varying factors ---- */

/* Complex scalars: (re, im) pairs, the layout of C99 float/double _Complex. */
typedef struct kron_c32 {
  float re, im;
} kron_c32_t;
typedef struct kron_c64 {
  double re, im;
} kron_c64_t;

#define KRON_TYPE_C32 5 /* element type codes of kron_nd_workspace_size beside */
#define KRON_TYPE_C64 6 /* KRON_MODE_F32 and KRON_MODE_F64 */
#define KRON_ND_MAX_DIM 8
#define KRON_ND_MAX_EXTENT 65536

/* vec(Y_p) <- alpha * (op(F_0) (x) op(F_1) (x) ... (x) op(F_{d-1})) vec(X_p)
                + beta * vec(Y_p),   p = 0 .. batch-1.
   Section 2.1 extends the summation to arrays of any dimension d >= 1,
   Section 2.2 gives op(M) in {M, M^T, M^*} of size m x n, complex types,
   alpha and beta, and Section 6 names factors that change along the batch:
     Y_p(i_0..i_{d-1}) = alpha * sum_{a_0..a_{d-1}} prod_k op(F_k)(i_k, a_k)
                         * X_p(a_0..a_{d-1}) + beta * Y_p(i_0..i_{d-1}).
   Layout: the last index is the fastest; X_p has extents n[0] .. n[d-1]
   (element (a_0..a_{d-1}) at sum_k a_k * prod_{j>k} n[j]) and starts at
   X + p * prod(n); Y_p has extents m[0] .. m[d-1] and starts at
   Y + p * prod(m).  For d = 2 and 3 with square factors this is the plain
   action of kron2d/kron3d_batched (F_0 = A on the slowest index).
   ops[k]: 'N' (op(F) = F, stored m[k] x n[k]), 'T' (F^T, stored n[k] x m[k])
   or 'C' (conjugate transpose; the same as 'T' for real types).  factors[k]
   is column-major with leading dimension ldf[k] >= the stored row count; the
   matrix of operand p starts at factors[k] + p * ldfp[k] elements (ldfp[k]
   = 0: one matrix for the whole batch).  1 <= m[k], n[k] <= 65536,
   1 <= d <= 8.  beta == 0 does not read Y.  X and Y must not overlap.
   Computed as d mode products (fastest index first), each one pass over
   device memory through the caller's workspace `ws` (16-byte aligned, at
   least kron_nd_workspace_size(d, m, n, batch, type) bytes; none for d = 1)
   with type KRON_MODE_F32, KRON_MODE_F64, KRON_TYPE_C32 or KRON_TYPE_C64.
   Returns 0, -k (argument k invalid: 1 d, 2 m, 3 n, 4 ops, 6 factors, 7 ldf,
   8 ldfp, 9 X, 11 Y, 12 batch, 13 ws, 14 ws_bytes) or a positive hipError_t;
   asynchronous on `stream`. */
size_t kron_nd_workspace_size(int d, const int* m, const int* n, int64_t batch, int type);
int kron_nd_batched_f32(int d, const int* m, const int* n, const char* ops, float alpha, const float* const* factors,
                        const int* ldf, const int64_t* ldfp, const float* X, float beta, float* Y, int64_t batch,
                        void* ws, size_t ws_bytes, hipStream_t stream);
int kron_nd_batched_f64(int d, const int* m, const int* n, const char* ops, double alpha,
                        const double* const* factors, const int* ldf, const int64_t* ldfp, const double* X,
                        double beta, double* Y, int64_t batch, void* ws, size_t ws_bytes, hipStream_t stream);
int kron_nd_batched_c32(int d, const int* m, const int* n, const char* ops, kron_c32_t alpha,
                        const kron_c32_t* const* factors, const int* ldf, const int64_t* ldfp, const kron_c32_t* X,
                        kron_c32_t beta, kron_c32_t* Y, int64_t batch, void* ws, size_t ws_bytes,
                        hipStream_t stream);
int kron_nd_batched_c64(int d, const int* m, const int* n, const char* ops, kron_c64_t alpha,
                        const kron_c64_t* const* factors, const int* ldf, const int64_t* ldfp, const kron_c64_t* X,
                        kron_c64_t beta, kron_c64_t* Y, int64_t batch, void* ws, size_t ws_bytes,
                        hipStream_t stream);

/* Section 3's TKRON1 / TKRON2 / TKRON3 argument lists with rectangular
   factors, leading dimensions, op in {N, T, C}, alpha, beta, and the types
   S, D, C, Z of the paper (f32, f64, c32, c64), on the engine above (one
   pass per dimension; the first pass reads the strided X, the last writes
   the strided Y).  Factor roles are this library's: A acts on the slowest
   index of each operand, B on the fastest (2-D) or the middle one (3-D), C
   on the fastest (3-D), i.e. these compute the paper's K(B, A) and K(C, B, A)
   in its index naming.
     1-D: y_p <- alpha op(A) x_p + beta y_p;  op(A) ma x na; x_p (na contiguous
          elements) at X + p*ldxp; y_p (ma elements) at Y + p*ldyp.
     2-D: Y_p <- alpha op(B) op(X_p) op(A)^T + beta Y_p;  op(A) ma x na,
          op(B) mb x nb, op(X_p) nb x na, Y_p mb x ma column-major with
          leading dimension ldy, at Y + p*ldyp.  X_p is stored nb x na
          (opX 'N') or na x nb (opX 'T' / 'C') with leading dimension ldx, at
          X + p*ldxp.
     3-D: vec(Y_p) <- alpha (op(A) (x) op(B) (x) op(C)) vec(X_p) + beta vec(Y_p);
          X_p(a, b, c) (a < na slowest, c < nc fastest) at
          X + p*ldxp + a*ldx2 + b*ldx + c, Y_p(i, j, k) at
          Y + p*ldyp + i*ldy2 + j*ldy + k.
   Factors: column-major, lda >= ma (op 'N') or na (op 'T' / 'C'), likewise
   ldb, ldc.  X strides may be any values >= 0 (X is only read); Y strides
   must give every output element its own address: ldy >= mb (2-D) or mc
   (3-D), ldy2 >= ldy*mb, ldyp >= ldy*ma (2-D) or ldy2*ma (3-D) or ma (1-D).
   Every extent is in 1..65536.  beta == 0 does not read Y; X and Y must not
   overlap.  ws: at least kron_nd_workspace_size(d, m, n, batch, type) bytes
   with m = {ma, mb[, mc]}, n = {na, nb[, nc]} (none for 1-D).  Returns 0,
   -k (argument k invalid, counting from 1 in the order of the signature),
   or a positive hipError_t; asynchronous on `stream`. */
int kron1d_batched_rect_f32(char opA, int ma, int na, int64_t batch, float alpha, const float* A, int lda,
                            const float* X, int64_t ldxp, float beta, float* Y, int64_t ldyp, void* ws, size_t ws_bytes,
                            hipStream_t stream);
int kron2d_batched_rect_f32(char opA, char opB, char opX, int ma, int na, int mb, int nb, int64_t batch,
                            float alpha, const float* A, int lda, const float* B, int ldb, const float* X, int64_t ldx,
                            int64_t ldxp, float beta, float* Y, int64_t ldy, int64_t ldyp, void* ws, size_t ws_bytes,
                            hipStream_t stream);
int kron3d_batched_rect_f32(char opA, char opB, char opC, int ma, int na, int mb, int nb, int mc, int nc,
                            int64_t batch, float alpha, const float* A, int lda, const float* B, int ldb, const float* C,
                            int ldc, const float* X, int64_t ldx, int64_t ldx2, int64_t ldxp, float beta, float* Y,
                            int64_t ldy, int64_t ldy2, int64_t ldyp, void* ws, size_t ws_bytes, hipStream_t stream);

int kron1d_batched_rect_f64(char opA, int ma, int na, int64_t batch, double alpha, const double* A, int lda,
                            const double* X, int64_t ldxp, double beta, double* Y, int64_t ldyp, void* ws, size_t ws_bytes,
                            hipStream_t stream);
int kron2d_batched_rect_f64(char opA, char opB, char opX, int ma, int na, int mb, int nb, int64_t batch,
                            double alpha, const double* A, int lda, const double* B, int ldb, const double* X, int64_t ldx,
                            int64_t ldxp, double beta, double* Y, int64_t ldy, int64_t ldyp, void* ws, size_t ws_bytes,
                            hipStream_t stream);
int kron3d_batched_rect_f64(char opA, char opB, char opC, int ma, int na, int mb, int nb, int mc, int nc,
                            int64_t batch, double alpha, const double* A, int lda, const double* B, int ldb, const double* C,
                            int ldc, const double* X, int64_t ldx, int64_t ldx2, int64_t ldxp, double beta, double* Y,
                            int64_t ldy, int64_t ldy2, int64_t ldyp, void* ws, size_t ws_bytes, hipStream_t stream);

int kron1d_batched_rect_c32(char opA, int ma, int na, int64_t batch, kron_c32_t alpha, const kron_c32_t* A, int lda,
                            const kron_c32_t* X, int64_t ldxp, kron_c32_t beta, kron_c32_t* Y, int64_t ldyp, void* ws, size_t ws_bytes,
                            hipStream_t stream);
int kron2d_batched_rect_c32(char opA, char opB, char opX, int ma, int na, int mb, int nb, int64_t batch,
                            kron_c32_t alpha, const kron_c32_t* A, int lda, const kron_c32_t* B, int ldb, const kron_c32_t* X, int64_t ldx,
                            int64_t ldxp, kron_c32_t beta, kron_c32_t* Y, int64_t ldy, int64_t ldyp, void* ws, size_t ws_bytes,
                            hipStream_t stream);
int kron3d_batched_rect_c32(char opA, char opB, char opC, int ma, int na, int mb, int nb, int mc, int nc,
                            int64_t batch, kron_c32_t alpha, const kron_c32_t* A, int lda, const kron_c32_t* B, int ldb, const kron_c32_t* C,
                            int ldc, const kron_c32_t* X, int64_t ldx, int64_t ldx2, int64_t ldxp, kron_c32_t beta, kron_c32_t* Y,
                            int64_t ldy, int64_t ldy2, int64_t ldyp, void* ws, size_t ws_bytes, hipStream_t stream);

int kron1d_batched_rect_c64(char opA, int ma, int na, int64_t batch, kron_c64_t alpha, const kron_c64_t* A, int lda,
                            const kron_c64_t* X, int64_t ldxp, kron_c64_t beta, kron_c64_t* Y, int64_t ldyp, void* ws, size_t ws_bytes,
                            hipStream_t stream);
int kron2d_batched_rect_c64(char opA, char opB, char opX, int ma, int na, int mb, int nb, int64_t batch,
                            kron_c64_t alpha, const kron_c64_t* A, int lda, const kron_c64_t* B, int ldb, const kron_c64_t* X, int64_t ldx,
                            int64_t ldxp, kron_c64_t beta, kron_c64_t* Y, int64_t ldy, int64_t ldyp, void* ws, size_t ws_bytes,
                            hipStream_t stream);
int kron3d_batched_rect_c64(char opA, char opB, char opC, int ma, int na, int mb, int nb, int mc, int nc,
                            int64_t batch, kron_c64_t alpha, const kron_c64_t* A, int lda, const kron_c64_t* B, int ldb, const kron_c64_t* C,
                            int ldc, const kron_c64_t* X, int64_t ldx, int64_t ldx2, int64_t ldxp, kron_c64_t beta, kron_c64_t* Y,
                            int64_t ldy, int64_t ldy2, int64_t ldyp, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- allocation-free variant ------------------------------------------------------ */

/* kron3d_batched_ex_f32 without a workspace argument, for callers that cannot
   allocate device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid allocation).  The prepared factors go to a device
   array of the library (3 * 16 * 16 floats, 3 KiB: every n in 1..16 fits;
   each GPU the library runs on holds its own copy until the process ends).
   The call allocates nothing: no hipMalloc, hipFree or allocating library
   routine.  Arguments, layout, results and status codes are those of
   kron3d_batched_ex_f32 (an n beyond KRON_MAX_N, hence beyond the array,
   returns -1); the device is the current one, as for every call.  On its
   first call on a device the library looks up that device's array address
   (a failure there is returned as a positive hipError_t).
   Every call on one GPU shares that GPU's array, which keeps the last call's
   prepared factors: calls that may overlap on one GPU (issued on different
   streams without ordering between them, or from several host threads)
   race and must be serialised by the caller.  Calls ordered on one stream
   are safe. */
int kron3d_batched_ex_f32_noalloc(int n, char opA, char opB, char opC, float alpha, const float* A,
                                  const float* B, const float* C, const float* X, float beta, float* Y,
                                  int64_t batch, hipStream_t stream);

/* ---- Section 3's interface with leading dimensions ------------------------------ */

/* The extended update above on strided storage, with the argument layout of
   the paper's TKRON2 / TKRON3 (Section 3) restricted to square n x n factors.
   The factor roles keep this library's convention, not TKRON's: the first
   factor argument acts on the slowest operand index and the last one on the
   fastest, so in the paper's notation these calls compute
   K(op(C), op(B), op(A)) in 3-D and K(op(B), op(A)) in 2-D (TKRON names A the
   factor of the first, fastest index).  The kron{2,3}d_tkron_* entry points
   below take TKRON's roles and rectangular factors.
     factor M (A, B, C): column-major with leading dimension ld >= n;
     2-D operand p: X_p(l, m) at X[l + ldx*m + ldxp*p], result likewise in Y
       with ldy, ldyp;
     3-D operand p: X_p(l, m, k) at X[l + ldx*m + ldx2*k + ldxp*p] (l is the
       fastest index, the one C contracts; ldx2 is the paper's distance
       between adjacent planes), result likewise with ldy, ldy2, ldyp.
   X is only read: its strides may be any values >= 0 (an operand stride of
   0 applies the action to one array `batch` times).  Y's strides must give
   every output element its own address: ldy >= n, ldy2 >= n*ldy (3-D), and
   ldyp >= n*ldy (2-D) or n*ldy2 (3-D).  X and Y must not overlap.  The
   library cannot see buffer sizes: the caller guarantees that every address
   the strides reach lies inside its arrays.
   ops, alpha, beta, ws (kron_ex_workspace_size bytes) and stream as for the
   _ex entry points; opX (2-D) transposes each operand.  Any stride and any
   element-aligned address is accepted: elements are read and written one at
   a time, except in 3-D with n = 16 when every X and Y stride is a multiple
   of 4 elements and both bases are 16-byte aligned (then 16-byte vectors).
   Contiguous arrays run faster through the _ex entry points.  Returns 0 or -k (argument k invalid; positions beyond 15 are
   reported by kron_status_string as "invalid argument"). */
int kron2d_batched_strided_f32(int n, char opA, char opB, char opX, float alpha, const float* A, int lda,
                               const float* B, int ldb, const float* X, int64_t ldx, int64_t ldxp, float beta,
                               float* Y, int64_t ldy, int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes,
                               hipStream_t stream);
int kron2d_batched_strided_f64(int n, char opA, char opB, char opX, double alpha, const double* A, int lda,
                               const double* B, int ldb, const double* X, int64_t ldx, int64_t ldxp, double beta,
                               double* Y, int64_t ldy, int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes,
                               hipStream_t stream);
int kron3d_batched_strided_f32(int n, char opA, char opB, char opC, float alpha, const float* A, int lda,
                               const float* B, int ldb, const float* C, int ldc, const float* X, int64_t ldx,
                               int64_t ldx2, int64_t ldxp, float beta, float* Y, int64_t ldy, int64_t ldy2,
                               int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes, hipStream_t stream);
int kron3d_batched_strided_f64(int n, char opA, char opB, char opC, double alpha, const double* A, int lda,
                               const double* B, int ldb, const double* C, int ldc, const double* X, int64_t ldx,
                               int64_t ldx2, int64_t ldxp, double beta, double* Y, int64_t ldy, int64_t ldy2,
                               int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- 1-D: TKRON1 (Section 3), a batched matrix-vector product ------------------- */

/* y_p <- alpha * op(A) x_p + beta * y_p for p = 0 .. batch-1, with x_p the
   n elements at X + p*ldxp and y_p those at Y + p*ldyp; A is n x n,
   column-major with leading dimension lda >= n; op 'N'/'n' or 'T'/'t'.
   ldxp >= 0 (0 repeats one vector), ldyp >= n; X and Y must not overlap.
   ws: at least kron_ex_workspace_size(2, n, mode) bytes of device memory
   (alpha * op(A) is written there once per call).  beta == 0 does not read
   Y.  Each output vector depends only on its own input vector (a NaN stays
   in its vector).  16 vectors per wavefront and MFMA tile; 16-byte accesses
   when n = 16, both strides are multiples of 4 elements and X, Y are 16-byte
   aligned.  Returns 0 or -k (argument k invalid); asynchronous on `stream`. */
int kron1d_batched_f32(int n, char opA, float alpha, const float* A, int lda, const float* X, int64_t ldxp,
                       float beta, float* Y, int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes,
                       hipStream_t stream);
int kron1d_batched_f64(int n, char opA, double alpha, const double* A, int lda, const double* X, int64_t ldxp,
                       double beta, double* Y, int64_t ldyp, int64_t batch, void* ws, size_t ws_bytes,
                       hipStream_t stream);

/* ---- backward ---------------------------------------------------------------- */

/* Gradients of L = sum_p <dY_p, Y_p> for the forward actions above (the
   shared factors enter every operand, so their gradients are summed over the
   batch; the paper's transpose-once remark of Section 2.2 gives dX as the
   transposed action):
     2-D: dX_p = B^T dY_p A,  dA = sum_p dY_p^T (B X_p),  dB = sum_p dY_p A X_p^T
     3-D: dX = (A^T (x) B^T (x) C^T) dY;  in operand indices (element (a, b, c)
          at a*n^2 + b*n + c):
          dA(i, a) = sum_p sum_{j,k} dY(i, j, k) sum_{b,c} B(j, b) C(k, c) X(a, b, c)
          and likewise dB over (i, k), dC over (i, j).
   Layouts as in the forward calls; dA, dB, dC are n x n column-major and are
   overwritten (zero for batch == 0).  Any of dX, dA, dB, dC may be NULL to
   skip it; X may be NULL when only dX is wanted.  dX must not alias X or dY.
   `ws` is caller-owned device memory of at least
   kron_backward_workspace_size(dim, n, batch, mode) bytes (per-wavefront or
   per-workgroup partial sums; needed only for dA/dB/dC).  For 3-D n = 16
   FP32 with 16-byte aligned X, dY and dX and at least one factor gradient
   requested, dX and the factor gradients come from one pass over X and dY.
   The summation order is fixed, so repeated calls on the same device give
   identical bits.  FP32 partial sums, final sums in FP64.  Asynchronous on
   `stream`. */
size_t kron_backward_workspace_size(int dim, int n, int64_t batch, int mode);
int kron2d_backward_f32(int n, const float* A, const float* B, const float* X, const float* dY,
                        float* dX, float* dA, float* dB, int64_t batch, void* ws, size_t ws_bytes,
                        hipStream_t stream);
int kron3d_backward_f32(int n, const float* A, const float* B, const float* C, const float* X,
                        const float* dY, float* dX, float* dA, float* dB, float* dC, int64_t batch,
                        void* ws, size_t ws_bytes, hipStream_t stream);
int kron2d_backward_f64(int n, const double* A, const double* B, const double* X, const double* dY,
                        double* dX, double* dA, double* dB, int64_t batch, void* ws, size_t ws_bytes,
                        hipStream_t stream);
int kron3d_backward_f64(int n, const double* A, const double* B, const double* C, const double* X,
                        const double* dY, double* dX, double* dA, double* dB, double* dC, int64_t batch,
                        void* ws, size_t ws_bytes, hipStream_t stream);

/* Backward over a mixed batch: the gradients above for every group of a
   batch that mixes sizes and 2-D / 3-D operands (Section 2.2's batched
   update with one set of shared factors per group).  Each group's dA, dB, dC
   are summed over that group's operands only.  mode is KRON_MODE_F32 or
   KRON_MODE_F64 (the arrays' element type); C and dC are ignored for dim 2;
   any of dX, dA, dB, dC may be NULL to skip it, and X may be NULL in a group
   that requests no factor gradient.  `ws` is caller-owned device memory of at
   least kron_grouped_backward_workspace_size() bytes (each group's partial
   sums in its own slice).  Every descriptor is checked before anything is
   launched; each group then runs as kron{2,3}d_backward_{f32,f64} would.
   The groups are spread, largest first, over eight streams the library owns
   (per device, created on the first call, default priority, never freed),
   which wait for the work already on `stream` and which `stream` waits for
   afterwards (events); one group, or a device where the streams cannot be
   created, runs on `stream` itself.  Asynchronous with respect to the host.
   Returns 0; -1 (groups NULL or an invalid descriptor), -2 (ngroups < 1), -3
   (ws NULL while needed), -4 (ws_bytes too small), or a positive
   hipError_t.  The result of every group is the single-group call's, bit for
   bit. */
typedef struct kron_group_grad {
  int32_t dim;      /* 2 or 3 */
  int32_t n;        /* 1..16 */
  int32_t mode;     /* KRON_MODE_F32 or KRON_MODE_F64 */
  int32_t reserved; /* set to 0 */
  const void* A;
  const void* B;
  const void* C;
  const void* X;    /* count * n^dim */
  const void* dY;   /* count * n^dim */
  void* dX;         /* count * n^dim, or NULL */
  void* dA;         /* n * n each, or NULL */
  void* dB;
  void* dC;
  int64_t count;    /* operands in the group, >= 0 */
} kron_group_grad_t;
size_t kron_grouped_backward_workspace_size(const kron_group_grad_t* groups, int ngroups);
int kron_grouped_backward(const kron_group_grad_t* groups, int ngroups, void* ws, size_t ws_bytes,
                          hipStream_t stream);

/* ---- measurement reference ----------------------------------------------------- */

/* Copies `bytes` bytes from src to dst with 16-byte non-temporal loads and
   stores on a persistent grid, in the fastest shape of a copy sweep on
   MI355X (2 KiB per wavefront step, two workgroups per compute unit): the
   achievable device-memory bandwidth the Kronecker kernels are compared
   with.  src and dst: 16-byte aligned device pointers that must not
   overlap; bytes: a multiple of 16.  Returns 0, -1 (src), -2 (dst), -3
   (bytes) or a positive hipError_t; asynchronous on `stream`. */
int kron_copy_bytes(const void* src, void* dst, size_t bytes, hipStream_t stream);

/* ---- launch shape ----------------------------------------------------------- */

/* How the kernels for (mode, dim, n) are launched: `blocks_per_cu` 256-thread
   workgroups per compute unit (0 = as many as can be resident; -1 = back to
   the built-in default) and a kernel `variant`:
     2-D: 0/1/2 = 4/8/2 tiles in flight per wavefront, direct loads;
          3 = tiles staged through LDS (n != 16); 4 = 3 with two LDS slices
          per wavefront, each span's stores issued after the next span's
          prefetched operands are in LDS (n != 16; otherwise variant 0).
     3-D: 0 plain; 1 next tile prefetched; 2 contiguous 1 KiB rows (a second
          register exchange); 3 = 1 + 2; 4/5 = contiguous rows with a window
          of 2/4 slab loads in flight; 6/7 = 4/5 with the next tile's first
          slabs requested early; 8 = tiles staged through LDS (n != 16;
          otherwise variant 0); 9/10 = n = 16,
          contiguous rows, the result stores interleaved with the next
          tile's slab loads (window 2/4; otherwise variant 4); 11 = 8 with
          the stores deferred as in 2-D variant 4 (n != 16; otherwise
          variant 0).  The paper
   picks its kernel method by matrix size and fixes the number of thread
   blocks (Sections 4 and 5); here the choice is a per-(mode, dim, n) table
   that an autotuner can fill.  Process-wide, not thread-safe against
   concurrent launches of the same (mode, dim, n).  Returns 0 or -k. */
int kron_set_launch(int mode, int dim, int n, int blocks_per_cu, int variant);
int kron_get_launch(int mode, int dim, int n, int* blocks_per_cu, int* variant);

/* Autotuner: time every launch shape (variants x 0..4 workgroups per CU) of
   (mode, dim, n) on the caller's device buffers (A, B, C, X read; Y is
   overwritten; C may be NULL for dim 2; element type as for the mode's
   entry points), `reps` timed launches each on `stream` with HIP events, in
   three sweeps over all shapes (forward, reverse, forward; three untimed
   launches before each timing), keep the shape with the lowest mean time in
   the launch-shape table and report it with that mean (any out pointer may
   be NULL).  Synchronises `stream`.  On error the entry is reset to the
   built-in default. */
int kron_autotune(int mode, int dim, int n, const void* A, const void* B, const void* C,
                  const void* X, void* Y, int64_t batch, int reps, hipStream_t stream,
                  int* best_blocks, int* best_variant, float* best_ms);

/* ---- status -------------------------------------------------------------- */

/* Static string describing a status returned by any entry point. */
const char* kron_status_string(int status);

/* Library version and build target, e.g. "kron 0.1 gfx950". */
const char* kron_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KRON_H */
