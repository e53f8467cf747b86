"""GPU parity of the backward: dX (transposed action) and the batch-reduced
factor gradients dA, dB, dC, through the C ABI and through the
torch.autograd front end.  References: the FP64 oracle gradient, central
finite differences of the library's own FP64 forward (exact up to rounding
because L = sum <dY, Y> is linear in each argument), and
torch.autograd.gradcheck in FP64."""
import numpy as np
import pytest
import torch

import oracle
from pins import cm, mat

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _abi_backward(dim, n, mats, X, dY, batch, dtype, want=(True, True, True, True)):
    import paper_1304_7054_amd as kron
    T = {np.float32: torch.float32, np.float64: torch.float64}[dtype]
    tm = [torch.from_numpy(np.asarray(m, dtype)).to(DEV) for m in mats]
    tx = torch.from_numpy(np.asarray(X, dtype)).to(DEV)
    tdy = torch.from_numpy(np.asarray(dY, dtype)).to(DEV)
    dX = torch.full_like(tx, float("nan")) if want[0] else None
    grads = [torch.full((n * n,), float("nan"), dtype=T, device=DEV) if w else None for w in want[1:1 + dim]]
    mode = kron.MODE_F32 if dtype == np.float32 else kron.MODE_F64
    ws = torch.empty(max(1, kron.kron_backward_workspace_size(dim, n, batch, mode)), dtype=torch.uint8, device=DEV)
    fn = {(2, np.float32): kron.kron2d_backward_f32, (3, np.float32): kron.kron3d_backward_f32,
          (2, np.float64): kron.kron2d_backward_f64, (3, np.float64): kron.kron3d_backward_f64}[(dim, dtype)]
    fn(n, *tm, tx, tdy, dX, *grads, batch, ws)
    torch.cuda.synchronize()
    out = [dX.cpu().numpy() if dX is not None else None] + [g.cpu().numpy() if g is not None else None for g in grads]
    return out


def _oracle_grad(dim, n, mats, X, dY, batch):
    if dim == 2:
        return oracle.kron2d_grad(n, mats[0], mats[1], X, dY, batch)
    return oracle.kron3d_grad(n, mats[0], mats[1], mats[2], X, dY, batch)


@pytest.mark.parametrize("n", list(range(1, 17)))
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_backward_matches_oracle(prec, dim, n):
    _need_gpu()
    dtype = np.float32 if prec == "f32" else np.float64
    q = 16 // n
    batch = 3 * q ** dim + 2
    rng = np.random.default_rng(500 + 17 * dim + n)
    mats = [rng.uniform(-1, 1, n * n).astype(dtype) for _ in range(dim)]
    X = rng.standard_normal(batch * n ** dim).astype(dtype)
    dY = rng.standard_normal(batch * n ** dim).astype(dtype)
    got = _abi_backward(dim, n, mats, X, dY, batch, dtype)
    want = _oracle_grad(dim, n, [m.astype(np.float64) for m in mats], X.astype(np.float64), dY.astype(np.float64), batch)
    tol = 1e-5 if prec == "f32" else 1e-12
    for name, g, w in zip(["dX", "dA", "dB", "dC"], got, want):
        assert np.all(np.isfinite(g)), name
        assert _rel(g, w) <= tol, (name, _rel(g, w))


@pytest.mark.parametrize("dim", [2, 3])
def test_backward_partial_outputs_and_zero_batch(dim):
    """Skipped outputs stay untouched; a zero batch gives zero gradients."""
    _need_gpu()
    n = 5
    rng = np.random.default_rng(3)
    mats = [rng.uniform(-1, 1, n * n) for _ in range(dim)]
    X = rng.standard_normal(7 * n ** dim)
    dY = rng.standard_normal(7 * n ** dim)
    only_b = _abi_backward(dim, n, mats, X, dY, 7, np.float64, want=(False, False, True, False))
    full = _oracle_grad(dim, n, mats, X, dY, 7)
    assert only_b[0] is None and only_b[1] is None
    assert _rel(only_b[2], full[2]) <= 1e-12
    zero = _abi_backward(dim, n, mats, X[:0], dY[:0], 0, np.float64)
    for g in zero[1:]:
        assert np.all(g == 0)


def test_backward_is_deterministic():
    _need_gpu()
    n, batch = 16, 3000
    rng = np.random.default_rng(4)
    mats = [rng.uniform(-1, 1, n * n).astype(np.float32) for _ in range(3)]
    X = rng.standard_normal(batch * n ** 3).astype(np.float32)
    dY = rng.standard_normal(batch * n ** 3).astype(np.float32)
    a = _abi_backward(3, n, mats, X, dY, batch, np.float32)
    b = _abi_backward(3, n, mats, X, dY, batch, np.float32)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("dim,n", [(2, 3), (2, 16), (3, 2), (3, 5)])
def test_autograd_gradcheck_fp64(dim, n):
    _need_gpu()
    from paper_1304_7054_amd.autograd import kron2d, kron3d
    torch.manual_seed(0)
    batch = 3
    X = torch.randn((batch,) + (n,) * dim, dtype=torch.float64, device=DEV, requires_grad=True)
    mats = [torch.randn(n, n, dtype=torch.float64, device=DEV, requires_grad=True) for _ in range(dim)]
    f = kron2d if dim == 2 else kron3d
    assert torch.autograd.gradcheck(lambda x, *m: f(x, *m), (X, *mats), eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("dim,n", [(2, 7), (2, 16), (3, 4), (3, 16)])
def test_autograd_matches_torch_reference_fp32(dim, n):
    """The front end's forward and gradients against the same computation in
    plain torch FP64 ops (einsum on the CPU)."""
    _need_gpu()
    from paper_1304_7054_amd.autograd import kron2d, kron3d
    torch.manual_seed(1)
    batch = 11
    X = torch.randn((batch,) + (n,) * dim, device=DEV, requires_grad=True)
    mats = [torch.randn(n, n, device=DEV, requires_grad=True) for _ in range(dim)]
    f = kron2d if dim == 2 else kron3d
    Y = f(X, *mats)
    dY = torch.randn_like(Y)
    Y.backward(dY)
    Xc = X.detach().double().cpu().requires_grad_()
    mc = [m.detach().double().cpu().requires_grad_() for m in mats]
    if dim == 2:
        Yr = torch.einsum("iu,jv,puv->pij", mc[0], mc[1], Xc)
    else:
        Yr = torch.einsum("ia,jb,kc,pabc->pijk", mc[0], mc[1], mc[2], Xc)
    Yr.backward(dY.double().cpu())
    assert _rel(Y.detach().cpu(), Yr.detach()) <= 1e-5
    assert _rel(X.grad.cpu(), Xc.grad) <= 1e-5
    for m, r in zip(mats, mc):
        assert _rel(m.grad.cpu(), r.grad) <= 1e-5


def test_second_derivative_raises():
    """The hand-written backward is first order: a double backward through it
    must raise rather than treat its outputs as constants."""
    _need_gpu()
    from paper_1304_7054_amd.autograd import kron3d
    n, batch = 4, 3
    X = torch.randn((batch, n, n, n), device=DEV, requires_grad=True)
    mats = [torch.randn(n, n, device=DEV, requires_grad=True) for _ in range(3)]
    Y = kron3d(X, *mats)
    (gx,) = torch.autograd.grad(Y.square().sum(), X, create_graph=True)
    with pytest.raises(RuntimeError):
        gx.sum().backward()


def test_mixed_shapes_finite_differences_fp64():
    """The mixed workload's group shapes (a few (dim, n) groups, FP64), with
    gradients checked by central differences (h = 1e-3) of the library's own
    forward: on all entries of A, B, C and on 64 random entries of X."""
    _need_gpu()
    from paper_1304_7054_amd.autograd import kron2d, kron3d
    rng = np.random.default_rng(44)
    h = 1e-3
    for dim, n, batch in ((2, 6, 64), (2, 9, 40), (3, 7, 20), (3, 10, 8), (2, 16, 16), (3, 2, 64)):
        X = torch.from_numpy(rng.standard_normal((batch,) + (n,) * dim)).to(DEV).requires_grad_()
        mats = [torch.from_numpy(rng.uniform(-1, 1, (n, n))).to(DEV).requires_grad_() for _ in range(dim)]
        dY = torch.from_numpy(rng.standard_normal((batch,) + (n,) * dim)).to(DEV)
        f = kron2d if dim == 2 else kron3d
        f(X, *mats).backward(dY)

        def L(Xv, ms):
            with torch.no_grad():
                return float((f(Xv, *ms) * dY).sum())

        for m_idx in range(dim):
            fd = np.empty((n, n))
            for i in range(n):
                for j in range(n):
                    ms_p = [m.detach().clone() for m in mats]
                    ms_m = [m.detach().clone() for m in mats]
                    ms_p[m_idx][i, j] += h
                    ms_m[m_idx][i, j] -= h
                    fd[i, j] = (L(X.detach(), ms_p) - L(X.detach(), ms_m)) / (2 * h)
            assert _rel(mats[m_idx].grad.cpu().numpy(), fd) <= 1e-8, (dim, n, m_idx)
        flat = X.detach().reshape(-1)
        idx = rng.choice(flat.numel(), size=64, replace=False)
        gx = X.grad.reshape(-1).cpu().numpy()
        for e in idx:
            xp, xm = flat.clone(), flat.clone()
            xp[e] += h
            xm[e] -= h
            fd = (L(xp.view_as(X), [m.detach() for m in mats]) - L(xm.view_as(X), [m.detach() for m in mats])) / (2 * h)
            assert abs(gx[e] - fd) <= 1e-8 * (1 + abs(fd)), (dim, n, e)


@pytest.mark.parametrize("want", [(True, True, True, True), (False, True, False, False), (True, False, True, True),
                                  (False, False, False, True)])
def test_fused_16_backward_subsets_and_unfused_agree(want):
    """3-D n = 16 FP32 takes the one-pass backward (dX and the factor
    gradients from one read of X and dY) when the arrays are 16-byte aligned;
    a batch above the workgroup count runs several tiles per workgroup.
    Requested outputs match the FP64 oracle, skipped ones stay untouched, and
    the unfused path (reached through arrays one element off alignment)
    agrees within the FP32 tolerance."""
    _need_gpu()
    import paper_1304_7054_amd as kron
    n, batch = 16, 2000
    rng = np.random.default_rng(61)
    mats = [rng.uniform(-1, 1, n * n).astype(np.float32) for _ in range(3)]
    X = rng.standard_normal(batch * n ** 3).astype(np.float32)
    dY = rng.standard_normal(batch * n ** 3).astype(np.float32)
    ref = _oracle_grad(3, n, [m.astype(np.float64) for m in mats], X.astype(np.float64), dY.astype(np.float64), batch)
    got = _abi_backward(3, n, mats, X, dY, batch, np.float32, want=want)
    for name, w, g, r in zip(["dX", "dA", "dB", "dC"], want, got, ref):
        if w:
            assert np.all(np.isfinite(g)) and _rel(g, r) <= 1e-5, (name, _rel(g, r))
        else:
            assert g is None
    # the same call on arrays that start one element past an aligned address
    tm = [torch.from_numpy(m).to(DEV) for m in mats]
    xb = torch.empty(X.size + 1, device=DEV)
    yb = torch.empty(X.size + 1, device=DEV)
    xb[1:] = torch.from_numpy(X).to(DEV)
    yb[1:] = torch.from_numpy(dY).to(DEV)
    dxb = torch.full((X.size + 1,), float("nan"), device=DEV) if want[0] else None
    grads = [torch.full((n * n,), float("nan"), device=DEV) if w else None for w in want[1:]]
    ws = torch.empty(kron.kron_backward_workspace_size(3, n, batch, kron.MODE_F32), dtype=torch.uint8, device=DEV)
    kron.kron3d_backward_f32(n, *tm, xb[1:], yb[1:], dxb[1:] if dxb is not None else None, *grads, batch, ws)
    torch.cuda.synchronize()
    other = [dxb[1:].cpu().numpy() if dxb is not None else None] + [gg.cpu().numpy() if gg is not None else None for gg in grads]
    for name, a, b in zip(["dX", "dA", "dB", "dC"], got, other):
        if a is not None:
            assert _rel(a, b) <= 2e-6, (name, _rel(a, b))
