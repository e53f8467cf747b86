"""CPU oracle for the batched Kronecker-product action.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the library itself never does.
It shares no code with the HIP library (``paper_1304_7054_amd``) and imports
nothing from it.

All arrays are numpy arrays in memory order:

* matrices are n x n **column-major**, passed as flat length-n^2 arrays
  (element (i, j) at i + n*j), as in the paper's interface section;
* 2-D operand p occupies elements [p*n^2, (p+1)*n^2) and is column-major;
  the action is Y_p = B X_p A^T, i.e. vec(Y_p) = (A kron B) vec(X_p)
  (the defining identity of Section 2);
* 3-D operand p occupies [p*n^3, (p+1)*n^3) with element (a, b, c) at
  a*n^2 + b*n + c, and vec(Y_p) = (A kron B kron C) vec(X_p), which is the
  paper's K(C, B, A) of Section 2.1 (C on the fastest index).

Functions follow the C source ``kron_oracle.c`` one to one; FP64 is the
truth, the float variants accumulate in float without fused multiply-adds.
Gradients are for L = sum_p <dY_p, Y_p> and are FP64 only.
"""
import ctypes
import os

import numpy as np

from . import build as _build


class Oracle:
    """Bindings to one build of the oracle library (the default one, or a
    test build of a deliberately altered copy)."""

    def __init__(self, path):
        lib = ctypes.CDLL(path)
        i64 = ctypes.c_int64
        p = ctypes.c_void_p
        for name in ("oracle_kron2d_f64", "oracle_kron2d_f32"):
            getattr(lib, name).argtypes = [ctypes.c_int, p, p, p, p, i64]
            getattr(lib, name).restype = None
        for name in ("oracle_kron3d_f64", "oracle_kron3d_f32"):
            getattr(lib, name).argtypes = [ctypes.c_int, p, p, p, p, p, i64]
            getattr(lib, name).restype = None
        lib.oracle_kron2d_grad_f64.argtypes = [ctypes.c_int, p, p, p, p, p, p, p, i64]
        lib.oracle_kron2d_grad_f64.restype = None
        lib.oracle_kron3d_grad_f64.argtypes = [ctypes.c_int, p, p, p, p, p, p, p, p, p, i64]
        lib.oracle_kron3d_grad_f64.restype = None
        d, ch = ctypes.c_double, ctypes.c_char
        lib.oracle_kron2d_ex_f64.argtypes = [ctypes.c_int, ch, ch, ch, d, p, p, p, d, p, i64]
        lib.oracle_kron2d_ex_f64.restype = None
        lib.oracle_kron3d_ex_f64.argtypes = [ctypes.c_int, ch, ch, ch, d, p, p, p, p, d, p, i64]
        lib.oracle_kron3d_ex_f64.restype = None
        lib.oracle_kron1d_ex_f64.argtypes = [ctypes.c_int, ch, d, p, p, i64, d, p, i64, i64]
        lib.oracle_kron1d_ex_f64.restype = None
        ip, lp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)
        lib.oracle_kron_nd_f64.argtypes = [ctypes.c_int, ip, ip, ctypes.c_char_p, d, ctypes.POINTER(p), ip, lp,
                                           p, d, p, i64]
        lib.oracle_kron_nd_f64.restype = None
        lib.oracle_kron_nd_z64.argtypes = [ctypes.c_int, ip, ip, ctypes.c_char_p, d, d, ctypes.POINTER(p), ip, lp,
                                           p, d, d, p, i64]
        lib.oracle_kron_nd_z64.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        self.lib = lib
        self.path = path

    def kron2d(self, n, A, B, X, batch, precision="f64"):
        """Y_p = B X_p A^T for p < batch (column-major n x n); flat array out."""
        dt, tag = _dtype(precision)
        A = _prep(A, dt, n * n)
        B = _prep(B, dt, n * n)
        X = _prep(X, dt, batch * n * n)
        Y = np.empty(batch * n * n, dtype=dt)
        getattr(self.lib, f"oracle_kron2d_{tag}")(n, _ptr(A), _ptr(B), _ptr(X), _ptr(Y), batch)
        return Y

    def kron3d(self, n, A, B, C, X, batch, precision="f64"):
        """vec(Y_p) = (A kron B kron C) vec(X_p) in memory order; flat array out."""
        dt, tag = _dtype(precision)
        A = _prep(A, dt, n * n)
        B = _prep(B, dt, n * n)
        C = _prep(C, dt, n * n)
        X = _prep(X, dt, batch * n ** 3)
        Y = np.empty(batch * n ** 3, dtype=dt)
        getattr(self.lib, f"oracle_kron3d_{tag}")(n, _ptr(A), _ptr(B), _ptr(C), _ptr(X), _ptr(Y), batch)
        return Y

    def kron2d_grad(self, n, A, B, X, dY, batch):
        """(dX, dA, dB) of L = sum_p <dY_p, Y_p> for the 2-D action, in FP64."""
        dt = np.float64
        A, B = _prep(A, dt, n * n), _prep(B, dt, n * n)
        X, dY = _prep(X, dt, batch * n * n), _prep(dY, dt, batch * n * n)
        dX = np.empty_like(X)
        dA = np.empty(n * n, dt)
        dB = np.empty(n * n, dt)
        self.lib.oracle_kron2d_grad_f64(n, _ptr(A), _ptr(B), _ptr(X), _ptr(dY),
                                        _ptr(dX), _ptr(dA), _ptr(dB), batch)
        return dX, dA, dB

    def kron3d_grad(self, n, A, B, C, X, dY, batch):
        """(dX, dA, dB, dC) of L = sum_p <dY_p, Y_p> for the 3-D action, in FP64."""
        dt = np.float64
        A, B, C = (_prep(M, dt, n * n) for M in (A, B, C))
        X, dY = _prep(X, dt, batch * n ** 3), _prep(dY, dt, batch * n ** 3)
        dX = np.empty_like(X)
        dA, dB, dC = (np.empty(n * n, dt) for _ in range(3))
        self.lib.oracle_kron3d_grad_f64(n, _ptr(A), _ptr(B), _ptr(C), _ptr(X), _ptr(dY),
                                        _ptr(dX), _ptr(dA), _ptr(dB), _ptr(dC), batch)
        return dX, dA, dB, dC

    def kron2d_ex(self, n, opA, opB, alpha, A, B, X, beta, Y, batch, opX="N"):
        """Y_p <- alpha * op(B) op(X_p) op(A)^T + beta * Y_p (op 'N' or 'T'; Y
        not read when beta == 0), in FP64; returns the new Y (a copy)."""
        dt = np.float64
        A, B = _prep(A, dt, n * n), _prep(B, dt, n * n)
        X = _prep(X, dt, batch * n * n)
        Y = np.array(_prep(Y, dt, batch * n * n), copy=True)
        self.lib.oracle_kron2d_ex_f64(n, opA.encode(), opB.encode(), opX.encode(), alpha, _ptr(A), _ptr(B),
                                      _ptr(X), beta, _ptr(Y), batch)
        return Y

    def kron1d_ex(self, n, opA, alpha, A, X, beta, Y, batch, ldxp=None, ldyp=None):
        """y_p <- alpha * op(A) x_p + beta * y_p with x_p at X[p*ldxp:], y_p at
        Y[p*ldyp:] (default n), in FP64; returns the new Y (a copy)."""
        dt = np.float64
        ldxp = n if ldxp is None else int(ldxp)
        ldyp = n if ldyp is None else int(ldyp)
        A = _prep(A, dt, n * n)
        X = np.ascontiguousarray(np.asarray(X, dt).reshape(-1))
        Y = np.array(np.asarray(Y, dt).reshape(-1), copy=True)
        if batch > 0 and (X.size < (batch - 1) * ldxp + n or Y.size < (batch - 1) * ldyp + n):
            raise ValueError("X or Y too small for batch and strides")
        self.lib.oracle_kron1d_ex_f64(n, opA.encode(), alpha, _ptr(A), _ptr(X), ldxp, beta, _ptr(Y), ldyp, batch)
        return Y

    def kron3d_ex(self, n, opA, opB, opC, alpha, A, B, C, X, beta, Y, batch):
        """vec(Y_p) <- alpha * (op(A) kron op(B) kron op(C)) vec(X_p) + beta * vec(Y_p),
        in FP64; returns the new Y (a copy)."""
        dt = np.float64
        A, B, C = (_prep(M, dt, n * n) for M in (A, B, C))
        X = _prep(X, dt, batch * n ** 3)
        Y = np.array(_prep(Y, dt, batch * n ** 3), copy=True)
        self.lib.oracle_kron3d_ex_f64(n, opA.encode(), opB.encode(), opC.encode(), alpha, _ptr(A), _ptr(B),
                                      _ptr(C), _ptr(X), beta, _ptr(Y), batch)
        return Y

    def kron_nd(self, m, n, ops, alpha, factors, X, beta, Y, batch, ldf=None, ldfp=None):
        """vec(Y_p) <- alpha (op(F_0) kron .. kron op(F_{d-1})) vec(X_p) + beta vec(Y_p)
        for d-dimensional operands (last index fastest), op(F_k) m[k] x n[k]
        ('N', 'T' or 'C'), F_k of operand p at factors[k][p * ldfp[k]:]
        (column-major, leading dimension ldf[k]); real FP64, or complex128
        when any input is complex.  Returns the new Y (a copy)."""
        d = len(m)
        if not (1 <= d <= 8 and len(n) == d and len(ops) == d and len(factors) == d):
            raise ValueError("d must be in 1..8 with one size, op and factor per dimension")
        cplx = any(np.iscomplexobj(a) for a in list(factors) + [X, Y, alpha, beta])
        dt = np.complex128 if cplx else np.float64
        ldf = [int(m[k] if ops[k] in "Nn" else n[k]) for k in range(d)] if ldf is None else [int(v) for v in ldf]
        ldfp = [0] * d if ldfp is None else [int(v) for v in ldfp]
        fs = [np.ascontiguousarray(np.asarray(f).reshape(-1), dtype=dt) for f in factors]
        for k in range(d):
            rows, cols = (m[k], n[k]) if ops[k] in "Nn" else (n[k], m[k])
            need = (rows + ldf[k] * (cols - 1)) + (batch - 1) * ldfp[k] if batch > 0 else 0
            if ldf[k] < rows or fs[k].size < need:
                raise ValueError(f"factor {k}: leading dimension or size too small")
        nx, ny = int(np.prod(n)), int(np.prod(m))
        X = _prep(X, dt, batch * nx)
        Y = np.array(_prep(Y, dt, batch * ny), copy=True)
        ci = (ctypes.c_int * d)
        fp = (ctypes.c_void_p * d)(*[f.ctypes.data for f in fs])
        args = (d, ci(*m), ci(*n), "".join(ops).encode(), )
        if cplx:
            a, b = complex(alpha), complex(beta)
            self.lib.oracle_kron_nd_z64(*args, a.real, a.imag, fp, ci(*ldf), (ctypes.c_int64 * d)(*ldfp),
                                        _ptr(X), b.real, b.imag, _ptr(Y), batch)
        else:
            self.lib.oracle_kron_nd_f64(*args, float(alpha), fp, ci(*ldf), (ctypes.c_int64 * d)(*ldfp), _ptr(X),
                                        float(beta), _ptr(Y), batch)
        return Y

    def num_threads(self):
        """OpenMP threads the oracle uses."""
        return int(self.lib.oracle_num_threads())

    def set_num_threads(self, n):
        """OpenMP threads of later calls (timing on a stated core count)."""
        self.lib.oracle_set_num_threads(int(n))


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _prep(a, dtype, size=None):
    a = np.ascontiguousarray(np.asarray(a).reshape(-1), dtype=dtype)
    if size is not None and a.size != size:
        raise ValueError(f"expected {size} elements, got {a.size}")
    return a


def _dtype(precision):
    if precision in ("f64", np.float64):
        return np.float64, "f64"
    if precision in ("f32", np.float32):
        return np.float32, "f32"
    raise ValueError(f"precision must be 'f64' or 'f32', not {precision!r}")


_DEFAULT = None


def default():
    """The oracle built from kron_oracle.c (rebuilt when the source is newer)."""
    global _DEFAULT
    if _DEFAULT is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _DEFAULT = Oracle(path)
    return _DEFAULT


def kron2d(*args, **kw):
    return default().kron2d(*args, **kw)


def kron3d(*args, **kw):
    return default().kron3d(*args, **kw)


def kron2d_grad(*args, **kw):
    return default().kron2d_grad(*args, **kw)


def kron3d_grad(*args, **kw):
    return default().kron3d_grad(*args, **kw)


def num_threads():
    return default().num_threads()


def kron2d_ex(*args, **kw):
    return default().kron2d_ex(*args, **kw)


def kron1d_ex(*args, **kw):
    return default().kron1d_ex(*args, **kw)


def kron3d_ex(*args, **kw):
    return default().kron3d_ex(*args, **kw)


def kron_nd(*args, **kw):
    return default().kron_nd(*args, **kw)
