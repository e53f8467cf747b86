"""Parity at the full workload sizes (1 GiB of FP32 operands), in the launch
configuration bench.py times (the built-in defaults): every output element
is written and finite (Y starts as NaN), and sampled operands (first, last
and random ones) match the FP64 oracle computed one by one on the host.
The backward is checked at full size through an identity that holds at any
size: L = sum_p <dY_p, Y_p> is linear in each of X, A, B, C, so
<dX, X> = <dA, A> = <dB, B> = <dC, C> = L (Euler's theorem for homogeneous
functions of degree one)."""
import numpy as np
import pytest
import torch

import bench
import oracle
import workloads

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


FULL = [
    ("f32", 3, 16, workloads.BATCH_3D[16]),
    ("f32", 3, 10, workloads.BATCH_3D[10]),
    ("f32", 2, 16, workloads.BATCH_2D[16]),
    ("f32", 2, 10, workloads.BATCH_2D[10]),
    ("f64", 3, 16, workloads.BATCH_3D[16] // 2),
    ("f64", 2, 16, workloads.BATCH_2D[16] // 2),
    ("bf16x3", 3, 16, workloads.BATCH_3D[16]),
    ("bf16", 3, 16, workloads.BATCH_3D[16]),
]
TOL = {"f32": 1e-5, "f64": 1e-13, "bf16x3": 1e-5, "bf16": 1e-2}


@pytest.mark.parametrize("mode,dim,n,batch", FULL)
def test_full_size_sampled(mode, dim, n, batch):
    _need_gpu()
    mats, X, Y = bench.make_inputs(torch, dim, n, batch, mode, 3)
    if mode in ("bf16x3", "bf16"):
        gen = torch.Generator(device="cuda").manual_seed(workloads.SEED_BASE + 3)
        for t in mats + [X]:
            workloads.log_uniform_device_(t, gen)
    Y.fill_(float("nan"))
    fn = bench.fn_for(mode, dim)
    assert fn(n, *mats, X, Y, batch) == 0
    torch.cuda.synchronize()
    assert bool(torch.isfinite(Y).all()), "unwritten or non-finite outputs"
    # sampled operands against the FP64 oracle on the exact device input values
    rng = np.random.default_rng(batch + n)
    idx = np.unique(np.concatenate([[0, 1, batch - 2, batch - 1], rng.integers(0, batch, 24)]))
    e = n ** dim
    hm = [m.double().cpu().numpy() for m in mats]
    num = den = 0.0
    for p in idx:
        x = X[p * e:(p + 1) * e].double().cpu().numpy()
        y = Y[p * e:(p + 1) * e].double().cpu().numpy()
        want = oracle.kron2d(n, *hm, x, 1) if dim == 2 else oracle.kron3d(n, *hm, x, 1)
        num += float(np.sum((y - want) ** 2))
        den += float(np.sum(want ** 2))
    assert np.sqrt(num / den) <= TOL[mode], (mode, dim, n, np.sqrt(num / den))


def test_full_size_backward_identity():
    _need_gpu()
    import paper_1304_7054_amd as kron
    n, batch = 16, workloads.BATCH_3D[16]
    mats, X, Y = bench.make_inputs(torch, 3, n, batch, "f32", 4)
    gen = torch.Generator(device="cuda").manual_seed(workloads.SEED_BASE + 4)
    dY = torch.randn(X.numel(), generator=gen, device="cuda")
    kron.kron3d_batched_f32(n, *mats, X, Y, batch)
    dX = torch.full_like(X, float("nan"))
    grads = [torch.full((n * n,), float("nan"), device="cuda") for _ in range(3)]
    ws = torch.empty(kron.kron_backward_workspace_size(3, n, batch, kron.MODE_F32), dtype=torch.uint8, device="cuda")
    kron.kron3d_backward_f32(n, *mats, X, dY, dX, *grads, batch, ws)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(dX).all())
    L = float((dY.double() * Y.double()).sum())
    scale = float((dY.double().abs() * Y.double().abs()).sum())
    checks = {"dX": float((dX.double() * X.double()).sum())}
    for name, g, m in zip(("dA", "dB", "dC"), grads, mats):
        checks[name] = float((g.double() * m.double()).sum())
    for name, v in checks.items():
        assert abs(v - L) <= 1e-5 * scale, (name, v, L, scale)
