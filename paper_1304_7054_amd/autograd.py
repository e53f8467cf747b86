"""torch.autograd front end of the batched Kronecker action.

Torch-level convention: X is (batch, n, n) or (batch, n, n, n), contiguous,
and the factors are ordinary (row-major) n x n tensors, so that

    2-D:  Y[p, i, j]    = sum_{u,v}   A[i, u] B[j, v] X[p, u, v]
    3-D:  Y[p, i, j, k] = sum_{a,b,c} A[i, a] B[j, b] C[k, c] X[p, a, b, c]

i.e. factor m acts along operand axis m.  On the memory-order vector this is
vec(Y_p) = (A kron B (kron C)) vec(X_p), the library's C ABI convention; for
2-D it is the paper's Y_p = B X_p A^T on the column-major view of X_p.  The
wrapper gives the kernels the column-major copies of the n x n factors (the
paper's transpose-once, Section 2.2); all batch work runs in libkron.
Backward: dX from the transposed action, dA/dB/dC batch-reduced by the
factor-gradient kernels (deterministic).  The backward is first order only:
its kernels write plain tensors with no graph, so asking for a second
derivative through it raises instead of silently treating it as constant.
"""
import torch

from . import _binding as kb

_FWD = {
    (2, torch.float32, "f32"): kb.kron2d_batched_f32,
    (3, torch.float32, "f32"): kb.kron3d_batched_f32,
    (2, torch.float64, "f64"): kb.kron2d_batched_f64,
    (3, torch.float64, "f64"): kb.kron3d_batched_f64,
    (2, torch.float32, "bf16x3"): kb.kron2d_batched_f32_bf16x3,
    (3, torch.float32, "bf16x3"): kb.kron3d_batched_f32_bf16x3,
}
_BWD = {
    (2, torch.float32): (kb.kron2d_backward_f32, kb.MODE_F32),
    (3, torch.float32): (kb.kron3d_backward_f32, kb.MODE_F32),
    (2, torch.float64): (kb.kron2d_backward_f64, kb.MODE_F64),
    (3, torch.float64): (kb.kron3d_backward_f64, kb.MODE_F64),
}


def _colmajor(M):
    return M.detach().t().contiguous()


def _check(X, mats):
    dim = X.dim() - 1
    if dim not in (2, 3):
        raise ValueError("X must be (batch, n, n) or (batch, n, n, n)")
    n = X.shape[-1]
    if any(s != n for s in X.shape[1:]):
        raise ValueError("operands must be n x n (x n)")
    if len(mats) != dim:
        raise ValueError(f"{dim}-D action needs {dim} factors")
    for M in mats:
        if M.shape != (n, n) or M.dtype != X.dtype or M.device != X.device:
            raise ValueError("factors must be n x n tensors of X's dtype and device")
    return dim, n


class KronFn(torch.autograd.Function):
    """Y = K(A, B[, C]) X with a hand-written backward."""

    @staticmethod
    def forward(ctx, mode, X, *mats):
        dim, n = _check(X, mats)
        X = X.contiguous()
        cm = [_colmajor(M) for M in mats]
        Y = torch.empty_like(X)
        fn = _FWD[(dim, X.dtype, mode)]
        fn(n, *cm, X, Y, X.shape[0])
        ctx.save_for_backward(X, *cm)
        ctx.dim, ctx.n = dim, n
        return Y

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, dY):
        X, *cm = ctx.saved_tensors
        dim, n = ctx.dim, ctx.n
        batch = X.shape[0]
        dY = dY.contiguous()
        need = ctx.needs_input_grad
        dX = torch.empty_like(X) if need[1] else None
        grads = [torch.empty(n * n, dtype=X.dtype, device=X.device) if need[2 + m] else None for m in range(dim)]
        fn, mode = _BWD[(dim, X.dtype)]
        ws = None
        if any(g is not None for g in grads):
            ws = torch.empty(max(1, kb.kron_backward_workspace_size(dim, n, batch, mode)), dtype=torch.uint8,
                             device=X.device)
        if dX is not None or ws is not None:
            fn(n, *cm, X, dY, dX, *grads, batch, ws)
        # the kernels return column-major n x n gradients; view them as torch matrices
        gm = [g.view(n, n).t() if g is not None else None for g in grads]
        return (None, dX, *gm)


def kron2d(X, A, B, mode="f32"):
    """Y[p, i, j] = sum A[i, u] B[j, v] X[p, u, v] (mode 'f32'/'f64' follows dtype; 'bf16x3' for FP32)."""
    if X.dtype == torch.float64:
        mode = "f64"
    return KronFn.apply(mode, X, A, B)


def kron3d(X, A, B, C, mode="f32"):
    """Y[p, i, j, k] = sum A[i, a] B[j, b] C[k, c] X[p, a, b, c]."""
    if X.dtype == torch.float64:
        mode = "f64"
    return KronFn.apply(mode, X, A, B, C)
