"""The C-ABI boundary without a GPU: the built library loads, exports every
function include/kron.h declares, and the Python binding gives each one a
ctypes signature.  Only host-side entry points are called (version, status
strings, launch-table queries); nothing launches a kernel."""
import ctypes
import os
import re

import pytest

import paper_1304_7054_amd as kron
from paper_1304_7054_amd import _binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kron.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)       # block comments
    text = re.sub(r"//[^\n]*", " ", text)                      # line comments
    names = re.findall(r"(?:^|[;{}\s])(?:const\s+char\s*\*|size_t|int)\s+(kron\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    for must in ("kron2d_batched_f32", "kron3d_batched_f32", "kron3d_batched_f64", "kron3d_batched_f32_bf16x3",
                 "kron3d_batched_bf16", "kron3d_batched_adjoint_f32", "kron3d_backward_f32",
                 "kron_backward_workspace_size", "kron_grouped_workspace_size", "kron_grouped_prepare",
                 "kron_grouped_launch", "kron_graph_capture_grouped", "kron_graph_launch", "kron_graph_destroy",
                 "kron_set_launch", "kron_get_launch", "kron_autotune", "kron_status_string", "kron_version"):
        assert must in names, must
    assert len(names) >= 28, names


def test_library_exports_every_declared_function():
    raw = ctypes.CDLL(_binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, missing


def test_binding_types_every_declared_function():
    L = kron.lib()
    untyped = [n for n in declared_functions() if getattr(L, n).argtypes is None]
    assert not untyped, untyped
    # the typed wrappers carry the same names as the C entry points
    for name in _binding.SIGNATURES:
        assert hasattr(kron, name) or hasattr(_binding, name), name


def test_host_side_entry_points():
    assert kron.version()
    assert kron.status_string(0)
    assert "argument" in kron.status_string(-3).lower()
    # launch table: defaults are readable and out-of-range requests are rejected
    for mode in (kron.MODE_F32, kron.MODE_F64, kron.MODE_BF16X3, kron.MODE_BF16):
        for dim in (2, 3):
            blocks, variant = kron.kron_get_launch(mode, dim, 16)
            assert blocks >= 0 and variant >= 0
    with pytest.raises(kron.KronError):
        kron.kron_set_launch(kron.MODE_F32, 3, 0, 0, 0)
