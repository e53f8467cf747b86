"""Backward over the mixed batch: the 500,000-operand mixed workload (n in
2..16 weighted toward 6..10, 70/30 2-D/3-D, one group per (dim, n) with its
own factors, upstream gradients dY ~ N(0, 1)) through kron_grouped_backward.

* every group's dA, dB (, dC) element by element against the FP64 oracle's
  gradient over the whole group, and dX on sampled operands;
* central finite differences in FP64 (h = 1e-3) on the first 64 operands of
  every group: every factor entry and 256 random operand entries.  The loss
  L = sum_p <dY_p, Y_p> is linear in each factor and in X, so a central
  difference equals the derivative up to rounding;
* the grouped call equals the single-group entry points bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-5


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _mats(p):
    return [m for m in (p.A, p.B, p.C) if m is not None]


def _upload(probs, dtype=torch.float32, count=None):
    groups = []
    for p in probs:
        b = p.batch if count is None else min(count, p.batch)
        e = p.n ** p.dim
        g = {"dim": p.dim, "n": p.n, "count": b,
             "mode": 0 if dtype == torch.float32 else 1,
             "X": torch.from_numpy(np.ascontiguousarray(p.X[:b * e])).to(DEV).to(dtype),
             "dY": torch.from_numpy(np.ascontiguousarray(p.dY[:b * e])).to(DEV).to(dtype)}
        g["dX"] = torch.full_like(g["X"], float("nan"))
        for k, m in zip("ABC", _mats(p)):
            g[k] = torch.from_numpy(m).to(DEV).to(dtype)
            g["d" + k] = torch.full((p.n * p.n,), float("nan"), device=DEV, dtype=dtype)
        groups.append(g)
    return groups


@pytest.fixture(scope="module")
def mixed():
    return workloads.workload4()


def test_grouped_backward_full_size_against_oracle(mixed):
    _need_gpu()
    import paper_1304_7054_amd as kron
    groups = _upload(mixed)
    kron.kron_grouped_backward(groups)
    torch.cuda.synchronize()
    rng = np.random.default_rng(404)
    for p, g in zip(mixed, groups):
        assert bool(torch.isfinite(g["dX"]).all()), (p.dim, p.n)
        mats = [m.astype(np.float64) for m in _mats(p)]
        grad = oracle.kron2d_grad if p.dim == 2 else oracle.kron3d_grad
        want = grad(p.n, *mats, p.X.astype(np.float64), p.dY.astype(np.float64), p.batch)
        for k, w in zip("ABC", want[1:]):
            got = g["d" + k].double().cpu().numpy()
            err = np.linalg.norm(got - w) / np.linalg.norm(w)
            assert err <= TOL, (p.dim, p.n, k, err)
        e = p.n ** p.dim
        idx = np.unique(np.concatenate([[0, p.batch - 1], rng.integers(0, p.batch, 30)]))
        got = torch.stack([g["dX"][q * e:(q + 1) * e] for q in idx]).double().cpu().numpy()
        wdx = np.stack([want[0][q * e:(q + 1) * e] for q in idx])
        err = np.linalg.norm(got - wdx) / np.linalg.norm(wdx)
        assert err <= TOL, (p.dim, p.n, "dX", err)


def test_grouped_backward_finite_differences(mixed):
    """FP32 gradients of the first 64 operands of every group against central
    differences of the FP64 forward (the library's, itself checked against
    the FP64 oracle) at h = 1e-3."""
    _need_gpu()
    import paper_1304_7054_amd as kron
    h = 1e-3
    count = 64
    groups = _upload(mixed, torch.float32, count)
    kron.kron_grouped_backward(groups)
    torch.cuda.synchronize()
    rng = np.random.default_rng(505)
    for p, g in zip(mixed, groups):
        b = g["count"]
        fwd = kron.kron2d_batched_f64 if p.dim == 2 else kron.kron3d_batched_f64
        mats = [g[k].double() for k in "ABC"[:p.dim]]
        X, dY = g["X"].double(), g["dY"].double()
        Y = torch.empty_like(X)

        def loss(ms, x):
            fwd(p.n, *ms, x, Y, b)
            return float((dY * Y).sum())

        fd, an = [], []
        for f in range(p.dim):
            for e in range(p.n * p.n):
                up = [m.clone() for m in mats]
                dn = [m.clone() for m in mats]
                up[f][e] += h
                dn[f][e] -= h
                fd.append((loss(up, X) - loss(dn, X)) / (2 * h))
            an.append(g["d" + "ABC"[f]].double().cpu().numpy())
        an = np.concatenate(an)
        fd = np.array(fd)
        err = np.linalg.norm(an - fd) / np.linalg.norm(fd)
        assert err <= TOL, (p.dim, p.n, "factors", err)
        xi = rng.integers(0, X.numel(), 256)
        fdx = []
        for q in xi:
            xu, xd = X.clone(), X.clone()
            xu[q] += h
            xd[q] -= h
            fdx.append((loss(mats, xu) - loss(mats, xd)) / (2 * h))
        got = g["dX"].double().cpu().numpy()[xi]
        fdx = np.array(fdx)
        err = np.linalg.norm(got - fdx) / np.linalg.norm(fdx)
        assert err <= TOL, (p.dim, p.n, "dX", err)


def test_grouped_backward_equals_single_group_calls():
    """Each group of a small mixed batch (FP32 and FP64) gives the single-group
    backward's bits; empty groups write zero factor gradients."""
    _need_gpu()
    import paper_1304_7054_amd as kron
    probs = workloads.workload4(count=3000)
    for dtype in (torch.float32, torch.float64):
        groups = _upload(probs, dtype)
        groups[0]["count"] = 0
        kron.kron_grouped_backward(groups)
        torch.cuda.synchronize()
        for p, g in zip(probs, groups):
            b = g["count"]
            tag = "f32" if dtype == torch.float32 else "f64"
            fn = getattr(kron, f"kron{p.dim}d_backward_{tag}")
            dX = torch.full_like(g["X"], float("nan"))
            outs = [torch.full_like(g["A"], float("nan")) for _ in range(p.dim)]
            fn(p.n, *[g[k] for k in "ABC"[:p.dim]], g["X"], g["dY"], dX, *outs, b)
            torch.cuda.synchronize()
            for k, o in zip("ABC", outs):
                assert torch.equal(g["d" + k], o), (p.dim, p.n, k)
            if b > 0:
                e = p.n ** p.dim
                assert torch.equal(g["dX"][:b * e], dX[:b * e]), (p.dim, p.n)
            else:
                assert all(bool((g["d" + k] == 0).all()) for k in "ABC"[:p.dim])


def test_grouped_backward_rejects_bad_descriptors():
    _need_gpu()
    import paper_1304_7054_amd as kron
    L = kron.lib()
    arr = (kron.KronGroupGrad * 1)()
    t = torch.zeros(64, device=DEV)
    arr[0] = kron.KronGroupGrad(2, 17, 0, 0, t.data_ptr(), t.data_ptr(), None, t.data_ptr(), t.data_ptr(), None,
                                None, None, None, 1)
    assert L.kron_grouped_backward_workspace_size(arr, 1) == 0
    assert L.kron_grouped_backward(arr, 1, t.data_ptr(), 256, None) == -1
    assert L.kron_grouped_backward(arr, 0, t.data_ptr(), 256, None) == -2
    arr[0] = kron.KronGroupGrad(2, 4, 0, 0, t.data_ptr(), t.data_ptr(), None, t.data_ptr(), t.data_ptr(), None,
                                t.data_ptr(), None, None, 1)
    need = L.kron_grouped_backward_workspace_size(arr, 1)
    assert need > 0
    assert L.kron_grouped_backward(arr, 1, None, need, None) == -3
    assert L.kron_grouped_backward(arr, 1, t.data_ptr(), need - 1, None) == -4
