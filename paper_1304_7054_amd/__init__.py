"""MI355X (gfx950) batched Kronecker-product action.

The compute lives in ``libkron.so`` (hand-written HIP kernels, C ABI declared
in ``include/kron.h``).  This package is its thin Python binding: the
functions carry the names of the C entry points and only marshal arguments.
"""
from ._binding import (  # noqa: F401
    KronError,
    LIB_PATH,
    MODE_BF16,
    MODE_BF16X3,
    MODE_BF16X6,
    MODE_F32,
    MODE_F64,
    SIGNATURES,
    kron2d_backward_f32,
    kron2d_backward_f64,
    kron3d_backward_f32,
    kron3d_backward_f64,
    kron_backward_workspace_size,
    kron2d_batched_ex_f32,
    kron2d_batched_ex_f64,
    kron3d_batched_ex_f32,
    kron3d_batched_ex_f32_noalloc,
    kron3d_batched_ex_f64,
    kron_ex_workspace_size,
    kron_nd_batched,
    kron1d_batched_rect_f32,
    kron1d_batched_rect_f64,
    kron1d_batched_rect_c32,
    kron1d_batched_rect_c64,
    kron2d_batched_rect_f32,
    kron2d_batched_rect_f64,
    kron2d_batched_rect_c32,
    kron2d_batched_rect_c64,
    kron3d_batched_rect_f32,
    kron3d_batched_rect_f64,
    kron3d_batched_rect_c32,
    kron3d_batched_rect_c64,
    kron_nd_batched_c32,
    kron_nd_batched_c64,
    kron_nd_batched_f32,
    kron_nd_batched_f64,
    kron_nd_workspace_size,
    KRON_TYPE_C32,
    KRON_TYPE_C64,
    KronC32,
    KronC64,
    kron1d_batched_f32,
    kron1d_batched_f64,
    kron2d_batched_strided_f32,
    kron2d_batched_strided_f64,
    kron3d_batched_strided_f32,
    kron3d_batched_strided_f64,
    kron2d_batched_adjoint_f32,
    kron2d_batched_adjoint_f64,
    kron2d_batched_bf16,
    kron2d_batched_f32,
    kron2d_batched_f32_bf16x3,
    kron2d_batched_f32_bf16x6,
    kron2d_batched_f64,
    kron3d_batched_adjoint_f32,
    kron3d_batched_adjoint_f64,
    kron3d_batched_bf16,
    kron3d_batched_f32,
    kron3d_batched_f32_bf16x3,
    kron3d_batched_f32_bf16x6,
    kron3d_batched_f64,
    kron_graph_capture_grouped,
    kron_graph_destroy,
    kron_graph_launch,
    kron_grouped_launch,
    kron_grouped_prepare,
    kron_grouped_workspace_size,
    kron_copy_bytes,
    kron_grouped_backward,
    kron_grouped_backward_workspace_size,
    KronGroupGrad,
    KronGroup,
    kron_autotune,
    kron_get_launch,
    kron_set_launch,
    lib,
    status_string,
    version,
)


def _load_tuning():
    """KRON_TUNE_CACHE, when set, names the launch table to apply (see
    tune.py); the shipped per-architecture table is applied otherwise, on the
    first call into the library on a GPU."""
    import os
    path = os.environ.get("KRON_TUNE_CACHE")
    if path and os.path.exists(path):
        from . import tune
        tune.load(path)


try:
    _load_tuning()
except Exception as exc:  # a stale or foreign table must not break import
    import warnings
    warnings.warn(f"KRON_TUNE_CACHE not applied: {exc}")
