"""ctypes binding of libkron (include/kron.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Arrays are
torch tensors on the GPU (their storage is passed as a raw pointer); the
binding checks device, dtype, contiguity and sizes so that a kernel never
reads or writes outside the tensors it is given, then calls the library on
the current (or given) stream.  All arithmetic happens in the HIP kernels;
there is no other code path.  If libkron.so is missing, every call raises.
"""
import ctypes
import os

import numpy as np

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkron.so")

MODE_F32, MODE_F64, MODE_BF16X3, MODE_BF16, MODE_BF16X6 = 0, 1, 2, 3, 4


class KronError(RuntimeError):
    """A non-zero status returned by libkron."""

    def __init__(self, func, status, text):
        super().__init__(f"{func} returned {status}: {text}")
        self.status = status


_LIB = None


class KronGroup(ctypes.Structure):
    """kron_group_t of include/kron.h."""
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("C", ctypes.c_void_p), ("X", ctypes.c_void_p), ("Y", ctypes.c_void_p),
                ("count", ctypes.c_int64)]

class KronGroupGrad(ctypes.Structure):
    """kron_group_grad_t of include/kron.h."""
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("C", ctypes.c_void_p), ("X", ctypes.c_void_p), ("dY", ctypes.c_void_p),
                ("dX", ctypes.c_void_p), ("dA", ctypes.c_void_p), ("dB", ctypes.c_void_p),
                ("dC", ctypes.c_void_p), ("count", ctypes.c_int64)]

class KronC32(ctypes.Structure):
    """kron_c32_t of include/kron.h (a complex float, by value)."""
    _fields_ = [("re", ctypes.c_float), ("im", ctypes.c_float)]


class KronC64(ctypes.Structure):
    """kron_c64_t of include/kron.h (a complex double, by value)."""
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


KRON_TYPE_C32, KRON_TYPE_C64 = 5, 6

# (name, argument kinds); 'i' int, 'l' int64, 'p' pointer, 'S' stream, 'z' size_t,
# 'c' char, 'f' float, 'd' double
SIGNATURES = {
    "kron2d_batched_f32": "ipppplS",
    "kron2d_batched_f64": "ipppplS",
    "kron3d_batched_f32": "ippppplS",
    "kron3d_batched_f64": "ippppplS",
    "kron2d_batched_f32_bf16x3": "ipppplS",
    "kron3d_batched_f32_bf16x3": "ippppplS",
    "kron2d_batched_f32_bf16x6": "ipppplS",
    "kron3d_batched_f32_bf16x6": "ippppplS",
    "kron2d_batched_bf16": "ipppplS",
    "kron3d_batched_bf16": "ippppplS",
    "kron2d_batched_adjoint_f32": "ipppplS",
    "kron3d_batched_adjoint_f32": "ippppplS",
    "kron2d_batched_adjoint_f64": "ipppplS",
    "kron3d_batched_adjoint_f64": "ippppplS",
    "kron2d_backward_f32": "ippppppplpzS",
    "kron3d_backward_f32": "ippppppppplpzS",
    "kron2d_backward_f64": "ippppppplpzS",
    "kron3d_backward_f64": "ippppppppplpzS",
    "kron2d_batched_ex_f32": "icccfpppfplpzS",
    "kron2d_batched_ex_f64": "icccdpppdplpzS",
    "kron3d_batched_ex_f32": "icccfppppfplpzS",
    "kron3d_batched_ex_f64": "icccdppppdplpzS",
    "kron3d_batched_ex_f32_noalloc": "icccfppppfplS",
    "kron1d_batched_f32": "icfpiplfpllpzS",
    "kron1d_batched_f64": "icdpipldpllpzS",
    "kron2d_batched_strided_f32": "icccfpipipllfplllpzS",
    "kron2d_batched_strided_f64": "icccdpipiplldplllpzS",
    "kron3d_batched_strided_f32": "icccfpipipiplllfpllllpzS",
    "kron3d_batched_strided_f64": "icccdpipipipllldpllllpzS",
}

_CT = {"i": ctypes.c_int, "l": ctypes.c_int64, "p": ctypes.c_void_p, "S": ctypes.c_void_p,
       "z": ctypes.c_size_t, "c": ctypes.c_char, "f": ctypes.c_float, "d": ctypes.c_double,
       "C": KronC32, "Z": KronC64}

_RECT_SCALAR = {"f32": "f", "f64": "d", "c32": "C", "c64": "Z"}
for _t, _k in _RECT_SCALAR.items():
    SIGNATURES[f"kron1d_batched_rect_{_t}"] = f"ciil{_k}pipl{_k}plpzS"
    SIGNATURES[f"kron2d_batched_rect_{_t}"] = f"ccciiiil{_k}pipipll{_k}pllpzS"
    SIGNATURES[f"kron3d_batched_rect_{_t}"] = f"ccciiiiiil{_k}pipipiplll{_k}plllpzS"


def lib():
    """The loaded libkron (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libkron.so not found at {LIB_PATH}; build it with "
                               "`python paper_1304_7054_amd/build.py` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, kinds in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = [_CT[k] for k in kinds]
            f.restype = ctypes.c_int
        L.kron_status_string.argtypes = [ctypes.c_int]
        L.kron_status_string.restype = ctypes.c_char_p
        L.kron_version.argtypes = []
        L.kron_version.restype = ctypes.c_char_p
        L.kron_backward_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int]
        L.kron_backward_workspace_size.restype = ctypes.c_size_t
        L.kron_ex_workspace_size.argtypes = [ctypes.c_int] * 3
        L.kron_ex_workspace_size.restype = ctypes.c_size_t
        L.kron_grouped_workspace_size.argtypes = [ctypes.POINTER(KronGroup), ctypes.c_int]
        L.kron_grouped_workspace_size.restype = ctypes.c_size_t
        L.kron_grouped_prepare.argtypes = [ctypes.POINTER(KronGroup), ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_size_t, ctypes.c_void_p]
        L.kron_grouped_prepare.restype = ctypes.c_int
        L.kron_grouped_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.kron_grouped_launch.restype = ctypes.c_int
        ip, lp, cp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64), ctypes.c_char_p
        L.kron_nd_workspace_size.argtypes = [ctypes.c_int, ip, ip, ctypes.c_int64, ctypes.c_int]
        L.kron_nd_workspace_size.restype = ctypes.c_size_t
        for name, sc in (("kron_nd_batched_f32", ctypes.c_float), ("kron_nd_batched_f64", ctypes.c_double),
                         ("kron_nd_batched_c32", KronC32), ("kron_nd_batched_c64", KronC64)):
            f = getattr(L, name)
            f.argtypes = [ctypes.c_int, ip, ip, cp, sc, ctypes.POINTER(ctypes.c_void_p), ip, lp, ctypes.c_void_p, sc,
                          ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
            f.restype = ctypes.c_int
        L.kron_copy_bytes.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.kron_copy_bytes.restype = ctypes.c_int
        L.kron_grouped_backward_workspace_size.argtypes = [ctypes.POINTER(KronGroupGrad), ctypes.c_int]
        L.kron_grouped_backward_workspace_size.restype = ctypes.c_size_t
        L.kron_grouped_backward.argtypes = [ctypes.POINTER(KronGroupGrad), ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_size_t, ctypes.c_void_p]
        L.kron_grouped_backward.restype = ctypes.c_int
        L.kron_graph_capture_grouped.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
        L.kron_graph_capture_grouped.restype = ctypes.c_int
        L.kron_graph_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.kron_graph_launch.restype = ctypes.c_int
        L.kron_graph_destroy.argtypes = [ctypes.c_void_p]
        L.kron_graph_destroy.restype = ctypes.c_int
        L.kron_autotune.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p] * 5 + [
            ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float)]
        L.kron_autotune.restype = ctypes.c_int
        L.kron_set_launch.argtypes = [ctypes.c_int] * 5
        L.kron_set_launch.restype = ctypes.c_int
        L.kron_get_launch.argtypes = [ctypes.c_int] * 3 + [ctypes.POINTER(ctypes.c_int)] * 2
        L.kron_get_launch.restype = ctypes.c_int
        _LIB = L
        _apply_shipped_table()
    return _LIB


APPLIED_TABLE = {"path": None, "entries": 0}


def _apply_shipped_table():
    """Apply the launch table measured by the autotuner for this GPU's
    architecture (tuning/<arch>.json), unless KRON_TUNE_CACHE names another
    table; entries keyed for another device or HIP version are ignored."""
    if os.environ.get("KRON_TUNE_CACHE") or not torch.cuda.is_available():
        return
    from . import tune
    arch = tune.device_key().split("|")[0]
    path = os.path.join(HERE, "tuning", f"{arch}.json")
    if os.path.exists(path):
        APPLIED_TABLE["entries"] = tune.load(path)
        APPLIED_TABLE["path"] = os.path.relpath(path, os.path.dirname(HERE))


def status_string(status: int) -> str:
    return lib().kron_status_string(int(status)).decode()


def version() -> str:
    return lib().kron_version().decode()


def kron_set_launch(mode, dim, n, blocks_per_cu, variant):
    """Set the launch shape of (mode, dim, n); blocks_per_cu -1 restores the default."""
    return _call("kron_set_launch", int(mode), int(dim), int(n), int(blocks_per_cu), int(variant))


def kron_get_launch(mode, dim, n):
    """(blocks_per_cu, variant) currently used for (mode, dim, n)."""
    b, v = ctypes.c_int(0), ctypes.c_int(0)
    _call("kron_get_launch", int(mode), int(dim), int(n), ctypes.byref(b), ctypes.byref(v))
    return b.value, v.value


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _scratch(need, device, stream):
    """A workspace the binding allocates on the caller's behalf.  The caching
    allocator tracks the current stream; when the kernels run on another
    stream the block is recorded on that stream too, so it is not handed to
    a new tensor before those kernels have read it."""
    ws = torch.empty(need, dtype=torch.uint8, device=device)
    if stream is not None:
        ts = torch.cuda.ExternalStream(stream, device=device) if isinstance(stream, int) else stream
        if ts.cuda_stream != torch.cuda.current_stream(device).cuda_stream:
            ws.record_stream(ts)
    return ws


def _arr(t, dtype, min_numel, what):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{what} must live on the GPU, not {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{what} must have dtype {dtype}, not {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() < min_numel:
        raise ValueError(f"{what} holds {t.numel()} elements, needs {min_numel}")
    return ctypes.c_void_p(t.data_ptr())


def _call(name, *args):
    rc = getattr(lib(), name)(*args)
    if rc != 0:
        raise KronError(name, rc, status_string(rc))
    return rc


def _dim_call(name, dim, dtype, n, mats, X, Y, batch, stream):
    n, batch = int(n), int(batch)
    if not 1 <= n <= 16:
        raise ValueError(f"n must be in 1..16, got {n}")
    if batch < 0:
        raise ValueError("batch must be >= 0")
    ptrs = [_arr(M, dtype, n * n, f"factor {i}") for i, M in enumerate(mats)]
    size = batch * n ** dim
    px = _arr(X, dtype, size, "X")
    py = _arr(Y, dtype, size, "Y")
    if X.data_ptr() == Y.data_ptr() and size > 0:
        raise ValueError("X and Y must not overlap")
    return _call(name, n, *ptrs, px, py, batch, _stream(stream))


def kron2d_batched_f32(n, A, B, X, Y, batch, stream=None):
    """Y_p = B X_p A^T, FP32 (see include/kron.h)."""
    return _dim_call("kron2d_batched_f32", 2, torch.float32, n, (A, B), X, Y, batch, stream)


def kron2d_batched_f64(n, A, B, X, Y, batch, stream=None):
    return _dim_call("kron2d_batched_f64", 2, torch.float64, n, (A, B), X, Y, batch, stream)


def kron3d_batched_f32(n, A, B, C, X, Y, batch, stream=None):
    """vec(Y_p) = (A kron B kron C) vec(X_p), FP32 (see include/kron.h)."""
    return _dim_call("kron3d_batched_f32", 3, torch.float32, n, (A, B, C), X, Y, batch, stream)


def kron3d_batched_f64(n, A, B, C, X, Y, batch, stream=None):
    return _dim_call("kron3d_batched_f64", 3, torch.float64, n, (A, B, C), X, Y, batch, stream)


def kron2d_batched_f32_bf16x3(n, A, B, X, Y, batch, stream=None):
    return _dim_call("kron2d_batched_f32_bf16x3", 2, torch.float32, n, (A, B), X, Y, batch, stream)


def kron3d_batched_f32_bf16x3(n, A, B, C, X, Y, batch, stream=None):
    return _dim_call("kron3d_batched_f32_bf16x3", 3, torch.float32, n, (A, B, C), X, Y, batch, stream)


def kron2d_batched_f32_bf16x6(n, A, B, X, Y, batch, stream=None):
    return _dim_call("kron2d_batched_f32_bf16x6", 2, torch.float32, n, (A, B), X, Y, batch, stream)


def kron3d_batched_f32_bf16x6(n, A, B, C, X, Y, batch, stream=None):
    return _dim_call("kron3d_batched_f32_bf16x6", 3, torch.float32, n, (A, B, C), X, Y, batch, stream)


def kron2d_batched_bf16(n, A, B, X, Y, batch, stream=None):
    """bf16 storage: tensors of dtype torch.bfloat16 (or int16/uint16 bit patterns viewed as bfloat16)."""
    return _dim_call("kron2d_batched_bf16", 2, torch.bfloat16, n, (A, B), X, Y, batch, stream)


def kron3d_batched_bf16(n, A, B, C, X, Y, batch, stream=None):
    return _dim_call("kron3d_batched_bf16", 3, torch.bfloat16, n, (A, B, C), X, Y, batch, stream)


def kron2d_batched_adjoint_f32(n, A, B, X, Y, batch, stream=None):
    """Y_p = B^T X_p A, FP32."""
    return _dim_call("kron2d_batched_adjoint_f32", 2, torch.float32, n, (A, B), X, Y, batch, stream)


def kron3d_batched_adjoint_f32(n, A, B, C, X, Y, batch, stream=None):
    return _dim_call("kron3d_batched_adjoint_f32", 3, torch.float32, n, (A, B, C), X, Y, batch, stream)


def kron2d_batched_adjoint_f64(n, A, B, X, Y, batch, stream=None):
    return _dim_call("kron2d_batched_adjoint_f64", 2, torch.float64, n, (A, B), X, Y, batch, stream)


def kron3d_batched_adjoint_f64(n, A, B, C, X, Y, batch, stream=None):
    return _dim_call("kron3d_batched_adjoint_f64", 3, torch.float64, n, (A, B, C), X, Y, batch, stream)


def kron_backward_workspace_size(dim, n, batch, mode):
    """Bytes of device workspace the factor gradients need."""
    return int(lib().kron_backward_workspace_size(int(dim), int(n), int(batch), int(mode)))


def _backward_call(name, dim, dtype, mode, n, mats, X, dY, dX, grads, batch, ws, stream):
    n, batch = int(n), int(batch)
    if not 1 <= n <= 16:
        raise ValueError(f"n must be in 1..16, got {n}")
    if batch < 0:
        raise ValueError("batch must be >= 0")
    size = batch * n ** dim
    pm = [_arr(M, dtype, n * n, f"factor {i}") for i, M in enumerate(mats)]
    px = _arr(X, dtype, size, "X")
    pdy = _arr(dY, dtype, size, "dY")
    pdx = _arr(dX, dtype, size, "dX")
    pg = [_arr(G, dtype, n * n, f"gradient {i}") for i, G in enumerate(grads)]
    for t in [dX] + list(grads):
        if t is not None and size > 0 and any(o is not None and t.data_ptr() == o.data_ptr() for o in (X, dY)):
            raise ValueError("outputs must not alias X or dY")
    need = kron_backward_workspace_size(dim, n, batch, mode) if any(G is not None for G in grads) else 0
    if need and ws is None:
        ws = _scratch(need, dY.device, stream)
    if need and ws.numel() * ws.element_size() < need:
        raise ValueError(f"workspace must hold {need} bytes")
    pws = ctypes.c_void_p(ws.data_ptr()) if ws is not None else None
    nbytes = ws.numel() * ws.element_size() if ws is not None else 0
    return _call(name, n, *pm, px, pdy, pdx, *pg, batch, pws, nbytes, _stream(stream))


def kron2d_backward_f32(n, A, B, X, dY, dX, dA, dB, batch, ws=None, stream=None):
    """dX, dA, dB of L = sum_p <dY_p, Y_p> (see include/kron.h); None skips an output."""
    return _backward_call("kron2d_backward_f32", 2, torch.float32, MODE_F32, n, (A, B), X, dY, dX, (dA, dB),
                          batch, ws, stream)


def kron3d_backward_f32(n, A, B, C, X, dY, dX, dA, dB, dC, batch, ws=None, stream=None):
    return _backward_call("kron3d_backward_f32", 3, torch.float32, MODE_F32, n, (A, B, C), X, dY, dX,
                          (dA, dB, dC), batch, ws, stream)


def kron2d_backward_f64(n, A, B, X, dY, dX, dA, dB, batch, ws=None, stream=None):
    return _backward_call("kron2d_backward_f64", 2, torch.float64, MODE_F64, n, (A, B), X, dY, dX, (dA, dB),
                          batch, ws, stream)


def kron3d_backward_f64(n, A, B, C, X, dY, dX, dA, dB, dC, batch, ws=None, stream=None):
    return _backward_call("kron3d_backward_f64", 3, torch.float64, MODE_F64, n, (A, B, C), X, dY, dX,
                          (dA, dB, dC), batch, ws, stream)


def kron_ex_workspace_size(dim, n, mode):
    """Bytes of workspace the extended entry points need (0 for invalid arguments)."""
    return int(lib().kron_ex_workspace_size(int(dim), int(n), int(mode)))


def _op_char(op, what):
    if op not in ("N", "n", "T", "t"):
        raise ValueError(f"{what} must be 'N' or 'T', got {op!r}")
    return op.encode()


def _ex_call(name, dim, dtype, mode, n, ops, alpha, mats, X, beta, Y, batch, ws, stream):
    n, batch = int(n), int(batch)
    if not 1 <= n <= 16:
        raise ValueError(f"n must be in 1..16, got {n}")
    if batch < 0:
        raise ValueError("batch must be >= 0")
    opc = [_op_char(op, f"op{i}") for i, op in enumerate(ops)]
    ptrs = [_arr(M, dtype, n * n, f"factor {i}") for i, M in enumerate(mats)]
    size = batch * n ** dim
    px = _arr(X, dtype, size, "X")
    py = _arr(Y, dtype, size, "Y")
    if X.data_ptr() == Y.data_ptr() and size > 0:
        raise ValueError("X and Y must not overlap")
    need = kron_ex_workspace_size(dim, n, mode)
    if ws is None:
        ws = _scratch(need, X.device, stream)
    pw = _arr(ws, torch.uint8, need, "workspace")
    return _call(name, n, *opc, alpha, *ptrs, px, beta, py, batch, pw, ws.numel(), _stream(stream))


def kron2d_batched_ex_f32(n, opA, opB, opX, alpha, A, B, X, beta, Y, batch, ws=None, stream=None):
    """Y_p = alpha op(B) op(X_p) op(A)^T + beta Y_p, FP32 (see include/kron.h)."""
    return _ex_call("kron2d_batched_ex_f32", 2, torch.float32, MODE_F32, n, (opA, opB, opX), float(alpha), (A, B),
                    X, float(beta), Y, batch, ws, stream)


def kron2d_batched_ex_f64(n, opA, opB, opX, alpha, A, B, X, beta, Y, batch, ws=None, stream=None):
    return _ex_call("kron2d_batched_ex_f64", 2, torch.float64, MODE_F64, n, (opA, opB, opX), float(alpha), (A, B),
                    X, float(beta), Y, batch, ws, stream)


def kron3d_batched_ex_f32(n, opA, opB, opC, alpha, A, B, C, X, beta, Y, batch, ws=None, stream=None):
    """vec(Y_p) = alpha (op(A) kron op(B) kron op(C)) vec(X_p) + beta vec(Y_p), FP32."""
    return _ex_call("kron3d_batched_ex_f32", 3, torch.float32, MODE_F32, n, (opA, opB, opC), float(alpha),
                    (A, B, C), X, float(beta), Y, batch, ws, stream)


def kron3d_batched_ex_f64(n, opA, opB, opC, alpha, A, B, C, X, beta, Y, batch, ws=None, stream=None):
    return _ex_call("kron3d_batched_ex_f64", 3, torch.float64, MODE_F64, n, (opA, opB, opC), float(alpha),
                    (A, B, C), X, float(beta), Y, batch, ws, stream)


def kron3d_batched_ex_f32_noalloc(n, opA, opB, opC, alpha, A, B, C, X, beta, Y, batch, stream=None):
    """kron3d_batched_ex_f32 with no workspace: the library keeps the prepared
    factors in its own device array (calls that overlap on one GPU race)."""
    n, batch = int(n), int(batch)
    if not 1 <= n <= 16:
        raise ValueError(f"n must be in 1..16, got {n}")
    if batch < 0:
        raise ValueError("batch must be >= 0")
    opc = [_op_char(op, f"op{i}") for i, op in enumerate((opA, opB, opC))]
    ptrs = [_arr(M, torch.float32, n * n, f"factor {i}") for i, M in enumerate((A, B, C))]
    size = batch * n ** 3
    px = _arr(X, torch.float32, size, "X")
    py = _arr(Y, torch.float32, size, "Y")
    if X.data_ptr() == Y.data_ptr() and size > 0:
        raise ValueError("X and Y must not overlap")
    return _call("kron3d_batched_ex_f32_noalloc", n, *opc, float(alpha), *ptrs, px, float(beta), py, batch,
                 _stream(stream))


_ND_TYPES = {torch.float32: ("f32", MODE_F32), torch.float64: ("f64", MODE_F64),
             torch.complex64: ("c32", KRON_TYPE_C32), torch.complex128: ("c64", KRON_TYPE_C64)}


def kron_nd_workspace_size(m, n, batch, type_code):
    """Bytes of workspace kron_nd_batched_* needs (0 for invalid arguments)."""
    d = len(m)
    ci = ctypes.c_int * max(1, d)
    return int(lib().kron_nd_workspace_size(d, ci(*m), ci(*n), int(batch), int(type_code)))


def _nd_call(tag, m, n, ops, alpha, factors, ldf, ldfp, X, beta, Y, batch, ws, stream):
    dtype = {"f32": torch.float32, "f64": torch.float64, "c32": torch.complex64, "c64": torch.complex128}[tag]
    code = _ND_TYPES[dtype][1]
    m, n = [int(v) for v in m], [int(v) for v in n]
    d, batch = len(m), int(batch)
    if not 1 <= d <= 8 or len(n) != d or len(ops) != d or len(factors) != d:
        raise ValueError("d must be in 1..8 with one size, op and factor per dimension")
    if min(m + n) < 1 or max(m + n) > 65536:
        raise ValueError("every extent must be in 1..65536")
    if batch < 0:
        raise ValueError("batch must be >= 0")
    for o in ops:
        if o not in "NnTtCc":
            raise ValueError(f"op must be 'N', 'T' or 'C', got {o!r}")
    rows = [m[k] if ops[k] in "Nn" else n[k] for k in range(d)]
    cols = [n[k] if ops[k] in "Nn" else m[k] for k in range(d)]
    ldf = list(rows) if ldf is None else [int(v) for v in ldf]
    ldfp = [0] * d if ldfp is None else [int(v) for v in ldfp]
    ptrs = []
    for k in range(d):
        if ldf[k] < rows[k] or ldfp[k] < 0:
            raise ValueError(f"factor {k}: leading dimension or operand stride too small")
        one = rows[k] + ldf[k] * (cols[k] - 1)
        need = one + (batch - 1) * ldfp[k] if batch > 0 else one
        ptrs.append(_arr(factors[k], dtype, need, f"factor {k}").value)
    nx, ny = batch * int(np.prod(n)), batch * int(np.prod(m))
    px = _arr(X, dtype, nx, "X")
    py = _arr(Y, dtype, ny, "Y")
    if nx > 0 and ny > 0:
        esz = X.element_size()
        x0, y0 = X.data_ptr(), Y.data_ptr()
        if x0 < y0 + ny * esz and y0 < x0 + nx * esz:
            raise ValueError("X and Y must not overlap")
    need = kron_nd_workspace_size(m, n, batch, code)
    if ws is None and need > 0:
        ws = _scratch(need, Y.device, stream)
    pw = _arr(ws, torch.uint8, need, "workspace") if need > 0 else None
    ci = ctypes.c_int * d
    if tag in ("c32", "c64"):
        S = KronC32 if tag == "c32" else KronC64
        a, b = complex(alpha), complex(beta)
        alpha_c, beta_c = S(a.real, a.imag), S(b.real, b.imag)
    else:
        alpha_c, beta_c = float(alpha), float(beta)
    return _call(f"kron_nd_batched_{tag}", d, ci(*m), ci(*n), "".join(ops).encode(), alpha_c,
                 (ctypes.c_void_p * d)(*ptrs), ci(*ldf), (ctypes.c_int64 * d)(*ldfp), px, beta_c, py, batch, pw,
                 0 if ws is None else ws.numel(), _stream(stream))


def kron_nd_batched_f32(m, n, ops, alpha, factors, X, beta, Y, batch, ldf=None, ldfp=None, ws=None, stream=None):
    """vec(Y_p) = alpha (op(F_0) kron .. kron op(F_{d-1})) vec(X_p) + beta vec(Y_p), FP32 (include/kron.h)."""
    return _nd_call("f32", m, n, ops, alpha, factors, ldf, ldfp, X, beta, Y, batch, ws, stream)


def kron_nd_batched_f64(m, n, ops, alpha, factors, X, beta, Y, batch, ldf=None, ldfp=None, ws=None, stream=None):
    return _nd_call("f64", m, n, ops, alpha, factors, ldf, ldfp, X, beta, Y, batch, ws, stream)


def kron_nd_batched_c32(m, n, ops, alpha, factors, X, beta, Y, batch, ldf=None, ldfp=None, ws=None, stream=None):
    """Complex FP32 pairs (torch.complex64)."""
    return _nd_call("c32", m, n, ops, alpha, factors, ldf, ldfp, X, beta, Y, batch, ws, stream)


def kron_nd_batched_c64(m, n, ops, alpha, factors, X, beta, Y, batch, ldf=None, ldfp=None, ws=None, stream=None):
    """Complex FP64 pairs (torch.complex128)."""
    return _nd_call("c64", m, n, ops, alpha, factors, ldf, ldfp, X, beta, Y, batch, ws, stream)


def kron_nd_batched(m, n, ops, alpha, factors, X, beta, Y, batch, ldf=None, ldfp=None, ws=None, stream=None):
    """The kron_nd_batched_* entry point of X's dtype."""
    if X.dtype not in _ND_TYPES:
        raise TypeError(f"unsupported dtype {X.dtype}")
    return _nd_call(_ND_TYPES[X.dtype][0], m, n, ops, alpha, factors, ldf, ldfp, X, beta, Y, batch, ws, stream)


def _span(exts, strides, batch, sp):
    """Elements from an operand array's first element to one past its last
    element over the whole batch (0 for an empty batch)."""
    if batch <= 0:
        return 0
    return 1 + sum((e - 1) * st for e, st in zip(exts, strides)) + (batch - 1) * sp


def _rect_call(tag, d, ops, m, n, batch, alpha, mats, lds, X, xstrides, xsp, beta, Y, ystrides, ysp, ws, stream):
    dtype = {"f32": torch.float32, "f64": torch.float64, "c32": torch.complex64, "c64": torch.complex128}[tag]
    code = _ND_TYPES[dtype][1]
    m, n, batch = [int(v) for v in m], [int(v) for v in n], int(batch)
    for o in ops:
        if o not in "NnTtCc":
            raise ValueError(f"op must be 'N', 'T' or 'C', got {o!r}")
    if min(m + n) < 1 or max(m + n) > 65536 or batch < 0:
        raise ValueError("extents must be in 1..65536 and batch >= 0")
    ptrs = []
    for k in range(d):
        rows, cols = (m[k], n[k]) if ops[k] in "Nn" else (n[k], m[k])
        if int(lds[k]) < rows:
            raise ValueError(f"leading dimension of factor {k} too small")
        ptrs += [_arr(mats[k], dtype, rows + int(lds[k]) * (cols - 1), f"factor {k}"), int(lds[k])]
    if min(list(xstrides) + [xsp]) < 0:
        raise ValueError("X strides must be >= 0")
    ex = _span(n if d != 2 or ops[2] in "Nn" else n, xstrides, batch, xsp)
    ey = _span(m, ystrides, batch, ysp)
    px, py = _arr(X, dtype, ex, "X"), _arr(Y, dtype, ey, "Y")
    if ex > 0 and ey > 0:
        esz = X.element_size()
        x0, y0 = X.data_ptr(), Y.data_ptr()
        if x0 < y0 + ey * esz and y0 < x0 + ex * esz:
            raise ValueError("X and Y must not overlap")
    need = kron_nd_workspace_size(m, n, batch, code)
    if ws is None and need > 0:
        ws = _scratch(need, Y.device, stream)
    pw = _arr(ws, torch.uint8, need, "workspace") if need > 0 else None
    if tag in ("c32", "c64"):
        S = KronC32 if tag == "c32" else KronC64
        a, b = complex(alpha), complex(beta)
        alpha, beta = S(a.real, a.imag), S(b.real, b.imag)
    else:
        alpha, beta = float(alpha), float(beta)
    return alpha, beta, ptrs, px, py, pw, 0 if ws is None else ws.numel()


def _rect1(tag, opA, ma, na, batch, alpha, A, lda, X, ldxp, beta, Y, ldyp, ws=None, stream=None):
    if int(ldyp) < int(ma):
        raise ValueError("ldyp must be >= ma")
    a, b, ptrs, px, py, pw, wb = _rect_call(tag, 1, opA, [ma], [na], batch, alpha, [A], [lda], X, [1], int(ldxp),
                                            beta, Y, [1], int(ldyp), ws, stream)
    return _call(f"kron1d_batched_rect_{tag}", _op_any(opA), int(ma), int(na), int(batch), a, *ptrs, px,
                 int(ldxp), b, py, int(ldyp), pw, wb, _stream(stream))


def _rect2(tag, opA, opB, opX, ma, na, mb, nb, batch, alpha, A, lda, B, ldb, X, ldx, ldxp, beta, Y, ldy, ldyp,
           ws=None, stream=None):
    ldx, ldxp, ldy, ldyp = int(ldx), int(ldxp), int(ldy), int(ldyp)
    if ldy < int(mb) or ldyp < ldy * int(ma):
        raise ValueError("Y strides must give every output element its own address (ldy >= mb, ldyp >= ldy*ma)")
    xs = [ldx, 1] if opX in "Nn" else [1, ldx]       # strides of (slow a0, fast a1) of op(X_p)
    a, b, ptrs, px, py, pw, wb = _rect_call(tag, 2, opA + opB + opX, [ma, mb], [na, nb], batch, alpha, [A, B],
                                            [lda, ldb], X, xs, ldxp, beta, Y, [ldy, 1], ldyp, ws, stream)
    return _call(f"kron2d_batched_rect_{tag}", _op_any(opA), _op_any(opB), _op_any(opX), int(ma), int(na), int(mb),
                 int(nb), int(batch), a, *ptrs, px, ldx, ldxp, b, py, ldy, ldyp, pw, wb, _stream(stream))


def _rect3(tag, opA, opB, opC, ma, na, mb, nb, mc, nc, batch, alpha, A, lda, B, ldb, C, ldc, X, ldx, ldx2, ldxp,
           beta, Y, ldy, ldy2, ldyp, ws=None, stream=None):
    ldx, ldx2, ldxp = int(ldx), int(ldx2), int(ldxp)
    ldy, ldy2, ldyp = int(ldy), int(ldy2), int(ldyp)
    if ldy < int(mc) or ldy2 < ldy * int(mb) or ldyp < ldy2 * int(ma):
        raise ValueError("Y strides must give every output element its own address")
    a, b, ptrs, px, py, pw, wb = _rect_call(tag, 3, opA + opB + opC, [ma, mb, mc], [na, nb, nc], batch, alpha,
                                            [A, B, C], [lda, ldb, ldc], X, [ldx2, ldx, 1], ldxp, beta, Y,
                                            [ldy2, ldy, 1], ldyp, ws, stream)
    return _call(f"kron3d_batched_rect_{tag}", _op_any(opA), _op_any(opB), _op_any(opC), int(ma), int(na), int(mb),
                 int(nb), int(mc), int(nc), int(batch), a, *ptrs, px, ldx, ldx2, ldxp, b, py, ldy, ldy2, ldyp, pw, wb,
                 _stream(stream))


def _op_any(op):
    if op not in ("N", "n", "T", "t", "C", "c"):
        raise ValueError(f"op must be 'N', 'T' or 'C', got {op!r}")
    return op.encode()


def _make_rect(tag):
    def k1(opA, ma, na, batch, alpha, A, lda, X, ldxp, beta, Y, ldyp, ws=None, stream=None):
        return _rect1(tag, opA, ma, na, batch, alpha, A, lda, X, ldxp, beta, Y, ldyp, ws, stream)

    def k2(opA, opB, opX, ma, na, mb, nb, batch, alpha, A, lda, B, ldb, X, ldx, ldxp, beta, Y, ldy, ldyp, ws=None,
           stream=None):
        return _rect2(tag, opA, opB, opX, ma, na, mb, nb, batch, alpha, A, lda, B, ldb, X, ldx, ldxp, beta, Y, ldy,
                      ldyp, ws, stream)

    def k3(opA, opB, opC, ma, na, mb, nb, mc, nc, batch, alpha, A, lda, B, ldb, C, ldc, X, ldx, ldx2, ldxp, beta, Y,
           ldy, ldy2, ldyp, ws=None, stream=None):
        return _rect3(tag, opA, opB, opC, ma, na, mb, nb, mc, nc, batch, alpha, A, lda, B, ldb, C, ldc, X, ldx, ldx2,
                      ldxp, beta, Y, ldy, ldy2, ldyp, ws, stream)
    for f, dd in ((k1, 1), (k2, 2), (k3, 3)):
        f.__name__ = f.__qualname__ = f"kron{dd}d_batched_rect_{tag}"
        f.__doc__ = f"TKRON{dd} with rectangular factors ({tag}); see include/kron.h."
    return k1, k2, k3


(kron1d_batched_rect_f32, kron2d_batched_rect_f32, kron3d_batched_rect_f32) = _make_rect("f32")
(kron1d_batched_rect_f64, kron2d_batched_rect_f64, kron3d_batched_rect_f64) = _make_rect("f64")
(kron1d_batched_rect_c32, kron2d_batched_rect_c32, kron3d_batched_rect_c32) = _make_rect("c32")
(kron1d_batched_rect_c64, kron2d_batched_rect_c64, kron3d_batched_rect_c64) = _make_rect("c64")


def _extent(n, strides):
    """Elements spanned by one array with the given strides (fast stride 1),
    from its first element to one past its last."""
    return (n - 1) * (1 + sum(strides)) + 1


def _strided_call(name, dim, dtype, mode, n, ops, alpha, mats, lds, X, ldx, beta, Y, ldy, batch, ws, stream):
    n, batch = int(n), int(batch)
    if not 1 <= n <= 16:
        raise ValueError(f"n must be in 1..16, got {n}")
    if batch < 0:
        raise ValueError("batch must be >= 0")
    opc = [_op_char(op, f"op{i}") for i, op in enumerate(ops)]
    lds = [int(v) for v in lds]
    ldx, ldy = [int(v) for v in ldx], [int(v) for v in ldy]
    for i, ld in enumerate(lds):
        if ld < n:
            raise ValueError(f"leading dimension of factor {i} must be >= n")
    if min(ldx) < 0:
        raise ValueError("X strides must be >= 0")
    if ldy[0] < n or any(ldy[j] < ldy[j - 1] * n for j in range(1, dim)):
        raise ValueError("Y strides must give every output element its own address "
                         "(ldy >= n, each further stride >= n times the previous)")
    ptrs = []
    for i, (M, ld) in enumerate(zip(mats, lds)):
        ptrs += [_arr(M, dtype, (n - 1) * ld + n, f"factor {i}"), ld]
    # one array spans its in-array strides; the batch adds (batch - 1) operand strides
    ex = _extent(n, ldx[:-1]) + (batch - 1) * ldx[-1] if batch > 0 else 0
    ey = _extent(n, ldy[:-1]) + (batch - 1) * ldy[-1] if batch > 0 else 0
    px = _arr(X, dtype, ex, "X")
    py = _arr(Y, dtype, ey, "Y")
    if batch > 0:
        esz = X.element_size()
        x0, y0 = X.data_ptr(), Y.data_ptr()
        if x0 < y0 + ey * esz and y0 < x0 + ex * esz:
            raise ValueError("X and Y must not overlap")
    need = kron_ex_workspace_size(dim, n, mode)
    if ws is None:
        ws = _scratch(need, Y.device, stream)
    pw = _arr(ws, torch.uint8, need, "workspace")
    return _call(name, n, *opc, alpha, *ptrs, px, *ldx, beta, py, *ldy, batch, pw, ws.numel(), _stream(stream))


def kron2d_batched_strided_f32(n, opA, opB, opX, alpha, A, lda, B, ldb, X, ldx, ldxp, beta, Y, ldy, ldyp, batch,
                               ws=None, stream=None):
    """Y_p = alpha op(B) op(X_p) op(A)^T + beta Y_p with leading dimensions
    (X_p(l, m) at X[l + ldx*m + ldxp*p]), FP32 (see include/kron.h)."""
    return _strided_call("kron2d_batched_strided_f32", 2, torch.float32, MODE_F32, n, (opA, opB, opX),
                         float(alpha), (A, B), (lda, ldb), X, (ldx, ldxp), float(beta), Y, (ldy, ldyp), batch, ws,
                         stream)


def kron2d_batched_strided_f64(n, opA, opB, opX, alpha, A, lda, B, ldb, X, ldx, ldxp, beta, Y, ldy, ldyp, batch,
                               ws=None, stream=None):
    return _strided_call("kron2d_batched_strided_f64", 2, torch.float64, MODE_F64, n, (opA, opB, opX),
                         float(alpha), (A, B), (lda, ldb), X, (ldx, ldxp), float(beta), Y, (ldy, ldyp), batch, ws,
                         stream)


def kron3d_batched_strided_f32(n, opA, opB, opC, alpha, A, lda, B, ldb, C, ldc, X, ldx, ldx2, ldxp, beta, Y, ldy,
                               ldy2, ldyp, batch, ws=None, stream=None):
    """3-D with leading dimensions: X_p(l, m, k) at X[l + ldx*m + ldx2*k + ldxp*p], FP32."""
    return _strided_call("kron3d_batched_strided_f32", 3, torch.float32, MODE_F32, n, (opA, opB, opC),
                         float(alpha), (A, B, C), (lda, ldb, ldc), X, (ldx, ldx2, ldxp), float(beta), Y,
                         (ldy, ldy2, ldyp), batch, ws, stream)


def kron3d_batched_strided_f64(n, opA, opB, opC, alpha, A, lda, B, ldb, C, ldc, X, ldx, ldx2, ldxp, beta, Y, ldy,
                               ldy2, ldyp, batch, ws=None, stream=None):
    return _strided_call("kron3d_batched_strided_f64", 3, torch.float64, MODE_F64, n, (opA, opB, opC),
                         float(alpha), (A, B, C), (lda, ldb, ldc), X, (ldx, ldx2, ldxp), float(beta), Y,
                         (ldy, ldy2, ldyp), batch, ws, stream)


def _tkron1_call(name, dtype, mode, n, opA, alpha, A, lda, X, ldxp, beta, Y, ldyp, batch, ws, stream):
    n, batch, lda, ldxp, ldyp = int(n), int(batch), int(lda), int(ldxp), int(ldyp)
    if not 1 <= n <= 16:
        raise ValueError(f"n must be in 1..16, got {n}")
    if batch < 0:
        raise ValueError("batch must be >= 0")
    if lda < n or ldxp < 0 or ldyp < n:
        raise ValueError("need lda >= n, ldxp >= 0, ldyp >= n")
    opc = _op_char(opA, "opA")
    pa = _arr(A, dtype, (n - 1) * lda + n, "A")
    ex = (batch - 1) * ldxp + n if batch > 0 else 0
    ey = (batch - 1) * ldyp + n if batch > 0 else 0
    px = _arr(X, dtype, ex, "X")
    py = _arr(Y, dtype, ey, "Y")
    if batch > 0:
        esz = X.element_size()
        x0, y0 = X.data_ptr(), Y.data_ptr()
        if x0 < y0 + ey * esz and y0 < x0 + ex * esz:
            raise ValueError("X and Y must not overlap")
    need = kron_ex_workspace_size(2, n, mode)
    if ws is None:
        ws = _scratch(need, Y.device, stream)
    pw = _arr(ws, torch.uint8, need, "workspace")
    return _call(name, n, opc, alpha, pa, lda, px, ldxp, beta, py, ldyp, batch, pw, ws.numel(), _stream(stream))


def kron1d_batched_f32(n, opA, alpha, A, lda, X, ldxp, beta, Y, ldyp, batch, ws=None, stream=None):
    """TKRON1: y_p = alpha op(A) x_p + beta y_p, x_p at X[p*ldxp:], FP32 (see include/kron.h)."""
    return _tkron1_call("kron1d_batched_f32", torch.float32, MODE_F32, n, opA, float(alpha), A, lda, X, ldxp,
                        float(beta), Y, ldyp, batch, ws, stream)


def kron1d_batched_f64(n, opA, alpha, A, lda, X, ldxp, beta, Y, ldyp, batch, ws=None, stream=None):
    return _tkron1_call("kron1d_batched_f64", torch.float64, MODE_F64, n, opA, float(alpha), A, lda, X, ldxp,
                        float(beta), Y, ldyp, batch, ws, stream)


def _groups_array(groups):
    """groups: iterable of dicts with dim, n, A, B, (C), X, Y, count and optional
    mode (MODE_F32 default or MODE_BF16X3); tensors are FP32 on the GPU."""
    groups = list(groups)
    arr = (KronGroup * max(1, len(groups)))()
    for i, g in enumerate(groups):
        dim, n, count = int(g["dim"]), int(g["n"]), int(g["count"])
        mode = int(g.get("mode", MODE_F32))
        if dim not in (2, 3) or not 1 <= n <= 16 or count < 0:
            raise ValueError(f"group {i}: bad dim/n/count")
        if mode not in (MODE_F32, MODE_BF16X3):
            raise ValueError(f"group {i}: mode must be MODE_F32 or MODE_BF16X3")
        size = count * n ** dim
        mats = [_arr(g[k], torch.float32, n * n, f"group {i} {k}") for k in ("A", "B", "C")[:dim]]
        px = _arr(g["X"], torch.float32, size, f"group {i} X")
        py = _arr(g["Y"], torch.float32, size, f"group {i} Y")
        if size > 0 and g["X"].data_ptr() == g["Y"].data_ptr():
            raise ValueError(f"group {i}: X and Y must not overlap")
        arr[i] = KronGroup(dim, n, mode, 0, mats[0], mats[1], mats[2] if dim == 3 else None, px, py, count)
    return arr, len(groups)


def _grad_groups_array(groups):
    """groups: iterable of dicts with dim, n, A, B, (C), X, dY, count, the
    optional outputs dX, dA, dB, (dC) and an optional mode (MODE_F32 default
    or MODE_F64, the tensors' dtype)."""
    groups = list(groups)
    arr = (KronGroupGrad * max(1, len(groups)))()
    for i, g in enumerate(groups):
        dim, n, count = int(g["dim"]), int(g["n"]), int(g["count"])
        mode = int(g.get("mode", MODE_F32))
        if dim not in (2, 3) or not 1 <= n <= 16 or count < 0:
            raise ValueError(f"group {i}: bad dim/n/count")
        if mode not in (MODE_F32, MODE_F64):
            raise ValueError(f"group {i}: mode must be MODE_F32 or MODE_F64")
        dt = _MODE_DTYPE[mode]
        size = count * n ** dim
        names = ("A", "B", "C")[:dim]
        mats = [_arr(g[k], dt, n * n, f"group {i} {k}") for k in names]
        want = [g.get(k) for k in ("dA", "dB", "dC")[:dim]]
        outs = [_arr(t, dt, n * n, f"group {i} d{k}") if t is not None else None for t, k in zip(want, names)]
        px = _arr(g["X"], dt, size, f"group {i} X") if g.get("X") is not None else None
        if px is None and any(t is not None for t in want) and count > 0:
            raise ValueError(f"group {i}: X is needed for factor gradients")
        pdy = _arr(g["dY"], dt, size, f"group {i} dY")
        pdx = None
        if g.get("dX") is not None:
            pdx = _arr(g["dX"], dt, size, f"group {i} dX")
            for other in ("X", "dY"):
                if g.get(other) is not None and size > 0 and g["dX"].data_ptr() == g[other].data_ptr():
                    raise ValueError(f"group {i}: dX must not alias {other}")
        arr[i] = KronGroupGrad(dim, n, mode, 0, mats[0], mats[1], mats[2] if dim == 3 else None, px, pdy, pdx,
                               outs[0], outs[1], outs[2] if dim == 3 else None, count)
    return arr, len(groups)


def kron_grouped_backward_workspace_size(groups):
    arr, k = _grad_groups_array(groups)
    return int(lib().kron_grouped_backward_workspace_size(arr, k))


def kron_grouped_backward(groups, ws=None, stream=None):
    """dX, dA, dB, dC of every group of a mixed batch (see include/kron.h);
    ws (uint8 tensor) defaults to a fresh buffer recorded on the stream."""
    arr, k = _grad_groups_array(groups)
    need = int(lib().kron_grouped_backward_workspace_size(arr, k))
    if need == 0:
        raise ValueError("invalid group descriptors")
    if ws is None:
        dev = next(iter(groups))["dY"].device
        ws = _scratch(need, dev, stream)
    pw = _arr(ws, torch.uint8, need, "workspace")
    return _call("kron_grouped_backward", arr, k, pw, ws.numel(), _stream(stream))


def kron_copy_bytes(src, dst, stream=None):
    """Streaming copy of src into dst (same byte size, 16-byte multiples): the
    bandwidth reference of the measurements."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous and of the same byte size")
    return _call("kron_copy_bytes", ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nb,
                 _stream(stream))


def kron_grouped_workspace_size(groups):
    arr, k = _groups_array(groups)
    return int(lib().kron_grouped_workspace_size(arr, k))


def kron_grouped_prepare(groups, ws, stream=None):
    """Build the work plan of `groups` into device workspace `ws` (uint8 tensor);
    the group tensors must outlive every launch of the plan."""
    arr, k = _groups_array(groups)
    return _call("kron_grouped_prepare", arr, k, ctypes.c_void_p(ws.data_ptr()),
                 ws.numel() * ws.element_size(), _stream(stream))


def kron_grouped_launch(ws, stream=None):
    return _call("kron_grouped_launch", ctypes.c_void_p(ws.data_ptr()), _stream(stream))


def kron_graph_capture_grouped(ws):
    """Instantiated HIP graph (an opaque handle) holding one grouped launch."""
    h = ctypes.c_void_p(0)
    _call("kron_graph_capture_grouped", ctypes.c_void_p(ws.data_ptr()), ctypes.byref(h))
    return h.value


def kron_graph_launch(graph_exec, stream=None):
    return _call("kron_graph_launch", ctypes.c_void_p(graph_exec), _stream(stream))


def kron_graph_destroy(graph_exec):
    return _call("kron_graph_destroy", ctypes.c_void_p(graph_exec))


_MODE_DTYPE = {MODE_F32: torch.float32, MODE_F64: torch.float64, MODE_BF16X3: torch.float32,
               MODE_BF16: torch.bfloat16, MODE_BF16X6: torch.float32}


def kron_autotune(mode, dim, n, A, B, C, X, Y, batch, reps=10, stream=None):
    """Time every launch shape of (mode, dim, n) on these buffers, keep the
    fastest; returns (blocks_per_cu, variant, ms)."""
    dt = _MODE_DTYPE[int(mode)]
    n, batch = int(n), int(batch)
    size = batch * n ** dim
    mats = [_arr(M, dt, n * n, f"factor {i}") for i, M in enumerate((A, B, C)[:dim])]
    if dim == 2:
        mats.append(None)
    px, py = _arr(X, dt, size, "X"), _arr(Y, dt, size, "Y")
    b, v, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_float(0)
    _call("kron_autotune", int(mode), int(dim), n, *mats, px, py, batch, int(reps), _stream(stream),
          ctypes.byref(b), ctypes.byref(v), ctypes.byref(ms))
    return b.value, v.value, ms.value
