"""Seeded synthetic inputs for the batched Kronecker-product action.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic.  Both the CPU oracle and the HIP library are fed from
here, so they always see the same values.

Memory conventions (shared by the oracle and the library): matrices are n x n
column-major flat arrays; 2-D operands are n x n column-major blocks of n^2
elements, 3-D operands are blocks of n^3 elements with element (a, b, c) at
a*n^2 + b*n + c, packed back to back (the smallest leading dimensions, as in
the paper's measured setting).

Workloads (seed = 13047054 + index; draws in the order A, B, C, X, dY):

0. 2-D, n = 4, 4096 operands, A, B, X ~ U[-1, 1].
1. 2-D, n = 16 (1,048,576 operands) or n = 10 (2,684,354): 1 GiB of FP32
   operands; A, B ~ U[-1, 1], X ~ N(0, 1).  FP64 uses half the batch.
2. 3-D, n = 16 (65,536 arrays) or n = 10 (268,435): 1 GiB of FP32 operands;
   distinct A, B, C ~ U[-1, 1], X ~ N(0, 1).  FP64 uses half the batch.
3. 3-D, n = 16, 65,536 arrays, every entry of A, B, C and X log-uniform in
   magnitude on [1e-3, 1e3] with a random sign (precision stress).
4. 500,000 mixed operands: n in 2..16 with weight 3 on 6..10 and 1 elsewhere,
   2-D with probability 0.7 else 3-D; one group per (dim, n) holding its own
   A, B (, C) ~ U[-1, 1]; X, dY ~ N(0, 1); groups in increasing (dim, n).
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 13047054

ONE_GIB = 1 << 30

# operand counts that make 1 GiB of FP32 operands
BATCH_2D = {16: 1_048_576, 10: 2_684_354}
BATCH_3D = {16: 65_536, 10: 268_435}
MIXED_COUNT = 500_000


def rng_for(index: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + index)


def uniform(rng, size, dtype=np.float64):
    """U[-1, 1] drawn in float64, cast to dtype."""
    return rng.uniform(-1.0, 1.0, size).astype(dtype)


def normal(rng, size, dtype=np.float64, chunk=1 << 25):
    """N(0, 1) drawn in float64 (in chunks, to bound host memory), cast to dtype."""
    out = np.empty(size, dtype=dtype)
    for s in range(0, size, chunk):
        e = min(size, s + chunk)
        out[s:e] = rng.standard_normal(e - s)
    return out


def log_uniform(rng, size, dtype=np.float64, lo=1e-3, hi=1e3):
    """Magnitude exp(U[ln lo, ln hi]) with sign +-1 at probability 1/2 each."""
    mag = np.exp(rng.uniform(np.log(lo), np.log(hi), size))
    sign = np.where(rng.random(size) < 0.5, -1.0, 1.0)
    return (sign * mag).astype(dtype)


def log_uniform_device_(t, gen, lo=1e-3, hi=1e3):
    """In place on a device tensor: the log_uniform distribution (magnitude
    exp(U[ln lo, ln hi]), sign +-1 at probability 1/2) drawn with a seeded
    torch generator; for the 1 GiB workloads, where host draws take long."""
    import torch
    mag = torch.empty(t.shape, dtype=torch.float32, device=t.device)
    mag.uniform_(float(np.log(lo)), float(np.log(hi)), generator=gen).exp_()
    sign = torch.empty_like(mag).bernoulli_(0.5, generator=gen).mul_(2).sub_(1)
    t.copy_(mag * sign)
    return t


@dataclass
class Problem:
    """One (dim, n) group of operands with its shared matrices."""
    dim: int
    n: int
    batch: int
    A: np.ndarray
    B: np.ndarray
    C: Optional[np.ndarray]
    X: np.ndarray
    dY: Optional[np.ndarray] = None

    @property
    def elems(self) -> int:
        return self.n ** self.dim

    def flops(self) -> int:
        """Paper's flop model: 4 n^3 (2-D) or 6 n^4 (3-D) per operand."""
        return self.batch * (4 * self.n ** 3 if self.dim == 2 else 6 * self.n ** 4)


def dense(dim: int, n: int, batch: int, index: int, dtype=np.float32,
          x_dist: str = "normal", mat_dist: str = "uniform", with_dy: bool = False) -> Problem:
    """A single-group problem drawn in the order A, B, (C), X, (dY)."""
    rng = rng_for(index)
    size = batch * n ** dim
    mdraw = {"uniform": uniform, "log_uniform": log_uniform}[mat_dist]
    A = mdraw(rng, n * n, dtype)
    B = mdraw(rng, n * n, dtype)
    C = mdraw(rng, n * n, dtype) if dim == 3 else None
    xdraw = {"normal": normal, "uniform": uniform, "log_uniform": log_uniform}[x_dist]
    X = xdraw(rng, size, dtype)
    dY = normal(rng, size, dtype) if with_dy else None
    return Problem(dim, n, batch, A, B, C, X, dY)


def workload0(dtype=np.float32) -> Problem:
    return dense(2, 4, 4096, 0, dtype, x_dist="uniform")


def workload1(n: int = 16, dtype=np.float32, batch: Optional[int] = None) -> Problem:
    b = batch if batch is not None else (BATCH_2D[n] if dtype == np.float32 else BATCH_2D[n] // 2)
    return dense(2, n, b, 1, dtype)


def workload2(n: int = 16, dtype=np.float32, batch: Optional[int] = None) -> Problem:
    b = batch if batch is not None else (BATCH_3D[n] if dtype == np.float32 else BATCH_3D[n] // 2)
    return dense(3, n, b, 2, dtype)


def workload3(batch: int = BATCH_3D[16]) -> Problem:
    return dense(3, 16, batch, 3, np.float32, x_dist="log_uniform", mat_dist="log_uniform")


def mixed_sizes(count: int = MIXED_COUNT, index: int = 4):
    """Per-operand (dim, n) draws of the mixed workload."""
    rng = rng_for(index)
    ns = np.arange(2, 17)
    w = np.where((ns >= 6) & (ns <= 10), 3.0, 1.0)
    n_draw = rng.choice(ns, size=count, p=w / w.sum())
    dim_draw = np.where(rng.random(count) < 0.7, 2, 3)
    return rng, dim_draw, n_draw


def workload4(count: int = MIXED_COUNT, dtype=np.float32) -> List[Problem]:
    """Mixed workload: one Problem per (dim, n) group present, with dY."""
    rng, dims, ns = mixed_sizes(count)
    groups = []
    for dim in (2, 3):
        for n in range(2, 17):
            b = int(np.count_nonzero((dims == dim) & (ns == n)))
            if b == 0:
                continue
            A = uniform(rng, n * n, dtype)
            B = uniform(rng, n * n, dtype)
            C = uniform(rng, n * n, dtype) if dim == 3 else None
            X = normal(rng, b * n ** dim, dtype)
            dY = normal(rng, b * n ** dim, dtype)
            groups.append(Problem(dim, n, b, A, B, C, X, dY))
    return groups


# ---- bf16 storage helpers (input preparation) -----------------------------

def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 with round-to-nearest-even; returns uint16 bits."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    nan = np.isnan(np.asarray(x, dtype=np.float32))
    out = rounded.astype(np.uint16)
    out[nan] = 0x7FC0
    return out


def bf16_bits_to_f32(h: np.ndarray) -> np.ndarray:
    return (np.asarray(h, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


# ---- structured matrices for exactness checks ------------------------------

def identity_cm(n: int, dtype=np.float32) -> np.ndarray:
    return np.eye(n, dtype=dtype).reshape(-1, order="F")


def permutation_cm(n: int, perm: np.ndarray, dtype=np.float32) -> np.ndarray:
    """Column-major P with P[i, perm[i]] = 1, so (P v)_i = v[perm[i]]."""
    P = np.zeros((n, n), dtype=dtype)
    P[np.arange(n), perm] = 1
    return P.reshape(-1, order="F")


def small_integers(rng, size, lo, hi, dtype=np.float32) -> np.ndarray:
    return rng.integers(lo, hi + 1, size).astype(dtype)
