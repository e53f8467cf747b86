"""Parity of the extended entry points, Y <- alpha K(op(A), op(B)[, op(C)]) X
(Section 3's batched interface with op in {N, T}; beta = 0), against the
FP64 oracle's extended interface: every op combination, several n (tiled and
staged paths, ragged batches), alpha values including 0 and negative ones,
Y filled with NaN so that an unwritten or read output shows.  A non-zero
beta, a bad op character and a short workspace are rejected with their
argument's position."""
import itertools

import numpy as np
import pytest
import torch

import oracle
import paper_1304_7054_amd as kron

pytestmark = pytest.mark.gpu
TOL = {"f32": 1e-5, "f64": 1e-13}
DT = {"f32": torch.float32, "f64": torch.float64}


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(mode, dim, n, ops, alpha, batch, seed):
    rng = np.random.default_rng(seed)
    mats = [rng.uniform(-1, 1, n * n) for _ in range(dim)]
    X = rng.standard_normal(batch * n ** dim)
    dt = DT[mode]
    tm = [torch.tensor(m, dtype=dt, device="cuda") for m in mats]
    tx = torch.tensor(X, dtype=dt, device="cuda")
    ty = torch.full_like(tx, float("nan"))
    fn = getattr(kron, f"kron{dim}d_batched_ex_{mode}")
    assert fn(n, *ops, alpha, *tm, tx, 0.0, ty, batch) == 0
    torch.cuda.synchronize()
    got = ty.double().cpu().numpy()
    hm = [t.double().cpu().numpy() for t in tm]
    hx = tx.double().cpu().numpy()
    nan = np.full(hx.size, np.nan)
    if dim == 2:
        want = oracle.kron2d_ex(n, *ops, alpha, *hm, hx, 0.0, nan, batch)
    else:
        want = oracle.kron3d_ex(n, *ops, alpha, *hm, hx, 0.0, nan, batch)
    assert np.all(np.isfinite(got))
    den = np.linalg.norm(want)
    err = np.linalg.norm(got - want) / den if den > 0 else np.linalg.norm(got)
    assert err <= TOL[mode], (mode, dim, n, ops, alpha, err)


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("n", [3, 10, 16])
@pytest.mark.parametrize("ops", list(itertools.product("NT", repeat=3)))
def test_ex3d_all_ops(mode, n, ops):
    _need_gpu()
    _run(mode, 3, n, ops, -1.75, 37, 11 + n)


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("n", [1, 5, 16])
@pytest.mark.parametrize("ops", list(itertools.product("NT", repeat=2)))
def test_ex2d_all_ops(mode, n, ops):
    _need_gpu()
    _run(mode, 2, n, ops, 0.5, 301, 21 + n)


@pytest.mark.parametrize("alpha", [0.0, 1.0, 3.0])
def test_ex_alpha_values(alpha):
    _need_gpu()
    _run("f32", 3, 16, ("T", "n", "t"), alpha, 129, 5)
    _run("f64", 2, 12, ("n", "T"), alpha, 77, 6)


def test_ex_identity_ops_equal_plain_call():
    """op = N, alpha = 1 gives bitwise the plain entry point's result (the
    prepared factors are copies of the inputs and the same kernels run)."""
    _need_gpu()
    g = torch.Generator(device="cuda").manual_seed(3)
    n, batch = 16, 1000
    mats = [torch.rand(n * n, generator=g, device="cuda") - 0.5 for _ in range(3)]
    X = torch.randn(batch * n ** 3, generator=g, device="cuda")
    Y1, Y2 = torch.empty_like(X), torch.empty_like(X)
    kron.kron3d_batched_f32(n, *mats, X, Y1, batch)
    kron.kron3d_batched_ex_f32(n, "N", "N", "N", 1.0, *mats, X, 0.0, Y2, batch)
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)


def test_ex_rejections():
    _need_gpu()
    n, batch = 4, 3
    mats = [torch.zeros(n * n, device="cuda") for _ in range(3)]
    X = torch.zeros(batch * n ** 3, device="cuda")
    Y = torch.zeros_like(X)
    L = kron.lib()
    ws = torch.empty(kron.kron_ex_workspace_size(3, n, kron.MODE_F32), dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    p = [m.data_ptr() for m in mats]

    def call(opA=b"N", beta=0.0, wsb=ws.numel(), wsp=ws.data_ptr()):
        return L.kron3d_batched_ex_f32(n, opA, b"N", b"T", 1.0, *p, X.data_ptr(), beta, Y.data_ptr(), batch,
                                       wsp, wsb, s)

    assert call() == 0
    assert call(opA=b"C") == -2           # op of A
    assert call(beta=1.0) == -10          # beta (10th argument)
    assert call(wsp=0) == -13             # workspace
    assert call(wsb=ws.numel() - 1) == -14
    torch.cuda.synchronize()
    with pytest.raises(kron.KronError):
        kron.kron3d_batched_ex_f32(n, "N", "N", "N", 1.0, *mats, X, 0.5, Y, batch)
    with pytest.raises(ValueError):
        kron.kron2d_batched_ex_f32(n, "X", "N", 1.0, mats[0], mats[1], X, 0.0, Y, batch)
