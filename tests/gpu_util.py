"""Helpers of the GPU parity tests: upload seeded numpy inputs, call the
library through its C ABI binding, fetch results, and measure errors."""
import numpy as np
import torch

import paper_1304_7054_amd as kron
import workloads

DEV = "cuda:0"

FWD = {
    ("f32", 2): kron.kron2d_batched_f32,
    ("f32", 3): kron.kron3d_batched_f32,
    ("f64", 2): kron.kron2d_batched_f64,
    ("f64", 3): kron.kron3d_batched_f64,
    ("bf16x3", 2): kron.kron2d_batched_f32_bf16x3,
    ("bf16x3", 3): kron.kron3d_batched_f32_bf16x3,
    ("bf16x6", 2): kron.kron2d_batched_f32_bf16x6,
    ("bf16x6", 3): kron.kron3d_batched_f32_bf16x6,
    ("bf16", 2): kron.kron2d_batched_bf16,
    ("bf16", 3): kron.kron3d_batched_bf16,
    ("adj_f32", 2): kron.kron2d_batched_adjoint_f32,
    ("adj_f32", 3): kron.kron3d_batched_adjoint_f32,
    ("adj_f64", 2): kron.kron2d_batched_adjoint_f64,
    ("adj_f64", 3): kron.kron3d_batched_adjoint_f64,
}

IO_DTYPE = {"f32": np.float32, "bf16x3": np.float32, "bf16x6": np.float32, "adj_f32": np.float32,
            "f64": np.float64, "adj_f64": np.float64}


def to_dev(a, mode):
    """numpy (float values) -> device tensor in the mode's storage type."""
    if mode == "bf16":
        bits = workloads.f32_to_bf16_bits(np.asarray(a, dtype=np.float32))
        return torch.from_numpy(bits.view(np.int16)).to(DEV).view(torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(a, dtype=IO_DTYPE[mode])).to(DEV)


def from_dev(t, mode):
    if mode == "bf16":
        return workloads.bf16_bits_to_f32(t.view(torch.int16).cpu().numpy().view(np.uint16))
    return t.cpu().numpy()


def run(mode, dim, n, mats, X, batch, poison=True, x_offset=0, y_offset=0):
    """Run one forward call; X is a numpy array of batch*n^dim values.
    x_offset/y_offset shift the operand arrays inside larger buffers (in elements)."""
    fn = FWD[(mode, dim)]
    tm = [to_dev(M, mode) for M in mats]
    size = batch * n ** dim
    tx_full = to_dev(np.concatenate([np.zeros(x_offset), np.asarray(X).reshape(-1)]), mode)
    tx = tx_full[x_offset:]
    ty_full = torch.empty(size + y_offset, dtype=tx.dtype, device=DEV)
    if poison:
        ty_full.fill_(float("nan"))
    ty = ty_full[y_offset:]
    fn(n, *tm, tx, ty, batch)
    torch.cuda.synchronize()
    return from_dev(ty, mode)


def rounded_inputs(mode, arrs):
    """The values the library actually sees (bf16 storage rounds its inputs)."""
    if mode == "bf16":
        return [workloads.bf16_bits_to_f32(workloads.f32_to_bf16_bits(np.asarray(a, np.float32))).astype(np.float64)
                for a in arrs]
    return [np.asarray(a, dtype=np.float64) for a in arrs]


def errors(got, want, batch):
    """(normwise relative error over the whole batch, max per-operand relative error)."""
    g = np.asarray(got, dtype=np.float64).reshape(batch, -1)
    w = np.asarray(want, dtype=np.float64).reshape(batch, -1)
    d = g - w
    norm = np.linalg.norm(d) / max(np.linalg.norm(w), 1e-300)
    per = np.linalg.norm(d, axis=1) / np.maximum(np.linalg.norm(w, axis=1), 1e-300)
    return float(norm), float(per.max()) if batch else 0.0


TOL = {"f32": 1e-5, "adj_f32": 1e-5, "bf16x3": 1e-5, "bf16x6": 1e-5, "f64": 1e-13, "adj_f64": 1e-13, "bf16": 1e-2}


def tiles_batch(dim, n, tiles=3, extra=1):
    """A batch that spans several tiles of the library's packing and a ragged tail."""
    q = 16 // n
    per_tile = q ** dim
    return tiles * per_tile + max(extra, per_tile // 3)
