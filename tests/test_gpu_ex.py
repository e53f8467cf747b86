"""Parity of the extended entry points, Y <- alpha K(op(A), op(B)[, op(C)]) X
+ beta Y (Section 3's batched interface with op in {N, T}), against the
FP64 oracle's extended interface: every op combination, several n (tiled and
staged paths, ragged batches), alpha values including 0 and negative ones.
In 2-D, op may also transpose the operands (opX).  With beta = 0, Y starts
as NaN so that an unwritten or read output shows;
with beta != 0, Y starts as seeded values that the update must read.  A bad
op character and a short or missing workspace are rejected with their
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


def _run(mode, dim, n, ops, alpha, batch, seed, beta=0.0, offset=0, opX="N"):
    rng = np.random.default_rng(seed)
    mats = [rng.uniform(-1, 1, n * n) for _ in range(dim)]
    X = rng.standard_normal(batch * n ** dim)
    Y0 = rng.standard_normal(batch * n ** dim)
    dt = DT[mode]
    size = batch * n ** dim
    tm = [torch.tensor(m, dtype=dt, device="cuda") for m in mats]
    # offset > 0: X and Y start `offset` elements into their allocations (unaligned arrays)
    bx = torch.zeros(size + offset, dtype=dt, device="cuda")
    by = torch.zeros(size + offset, dtype=dt, device="cuda")
    tx, ty = bx[offset:], by[offset:]
    tx.copy_(torch.tensor(X, dtype=dt))
    if beta == 0.0:
        ty.fill_(float("nan"))
    else:
        ty.copy_(torch.tensor(Y0, dtype=dt))
    hy0 = ty.double().cpu().numpy()
    fn = getattr(kron, f"kron{dim}d_batched_ex_{mode}")
    cops = tuple(ops) + ((opX,) if dim == 2 else ())
    assert fn(n, *cops, alpha, *tm, tx, beta, ty, batch) == 0
    torch.cuda.synchronize()
    got = ty.double().cpu().numpy()
    hm = [t.double().cpu().numpy() for t in tm]
    hx = tx.double().cpu().numpy()
    if dim == 2:
        want = oracle.kron2d_ex(n, *ops, alpha, *hm, hx, beta, hy0, batch, opX=opX)
    else:
        want = oracle.kron3d_ex(n, *ops, alpha, *hm, hx, beta, hy0, batch)
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


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("n", [1, 2, 4, 5, 7, 8, 10, 13, 16])
@pytest.mark.parametrize("dim", [2, 3])
def test_ex_beta_nonzero(mode, n, dim):
    """beta != 0: the update reads the old Y (every n: packed tiles, ragged
    last tile)."""
    _need_gpu()
    batch = 301 if dim == 2 else 37
    ops = ("T", "N", "T")[:dim]
    _run(mode, dim, n, ops, -0.75, batch, 400 + n + dim, beta=1.25)


@pytest.mark.parametrize("alpha,beta", [(0.0, 2.0), (1.0, -1.0), (2.5, 0.5)])
def test_ex_beta_values(alpha, beta):
    _need_gpu()
    _run("f32", 3, 16, ("N", "T", "N"), alpha, 257, 9, beta=beta)
    _run("f64", 2, 16, ("T", "T"), alpha, 1001, 10, beta=beta)


@pytest.mark.parametrize("mode", ["f32", "f64"])
def test_ex_beta_unaligned(mode):
    """X and Y one element past a 16-byte boundary: the scalar store path."""
    _need_gpu()
    _run(mode, 3, 16, ("T", "T", "T"), 1.5, 9, 12, beta=-2.0, offset=1)
    _run(mode, 2, 8, ("N", "T"), 1.5, 33, 13, beta=-2.0, offset=1)


def test_ex_beta_isolates_nonfinite_operands():
    """A NaN in one operand of a packed tile (n = 5: several operands per
    tile) stays in that operand; the others match the oracle."""
    _need_gpu()
    n, batch = 5, 64
    rng = np.random.default_rng(31)
    mats = [rng.uniform(-1, 1, n * n) for _ in range(3)]
    X = rng.standard_normal(batch * n ** 3)
    X[7 * n ** 3 + 3] = np.nan
    Y0 = rng.standard_normal(batch * n ** 3)
    tm = [torch.tensor(m, dtype=torch.float64, device="cuda") for m in mats]
    tx = torch.tensor(X, device="cuda")
    ty = torch.tensor(Y0, device="cuda")
    kron.kron3d_batched_ex_f64(n, "N", "T", "N", 1.0, *tm, tx, 0.5, ty, batch)
    torch.cuda.synchronize()
    got = ty.cpu().numpy().reshape(batch, -1)
    want = oracle.kron3d_ex(n, "N", "T", "N", 1.0, *mats, X, 0.5, Y0, batch).reshape(batch, -1)
    assert np.isnan(got[7]).any()
    keep = np.arange(batch) != 7
    np.testing.assert_allclose(got[keep], want[keep], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 9, 12, 16])
@pytest.mark.parametrize("beta", [0.0, -0.5])
def test_ex2d_op_x(mode, n, beta):
    """op(X_p) = X_p^T in 2-D, with and without the beta update, packed and
    ragged tiles."""
    _need_gpu()
    _run(mode, 2, n, ("T", "N"), 1.25, 203, 500 + n, beta=beta, opX="T")


@pytest.mark.parametrize("ops", list(itertools.product("NT", repeat=2)))
def test_ex2d_op_x_all_factor_ops(ops):
    _need_gpu()
    _run("f32", 2, 16, ops, -1.0, 64, 77, opX="t")
    _run("f64", 2, 7, ops, 0.5, 50, 78, beta=2.0, opX="T")


@pytest.mark.parametrize("mode", ["f32", "f64"])
def test_ex2d_op_x_unaligned(mode):
    _need_gpu()
    _run(mode, 2, 16, ("N", "N"), 1.0, 17, 14, beta=0.25, offset=1, opX="T")
    _run(mode, 2, 6, ("N", "T"), 1.0, 17, 15, offset=3, opX="T")


def test_ex2d_op_x_equals_transposed_input():
    """opX = T gives bitwise what the plain action gives on explicitly
    transposed operands (the same products in the same order)."""
    _need_gpu()
    g = torch.Generator(device="cuda").manual_seed(4)
    n, batch = 16, 4096
    A, B = (torch.rand(n * n, generator=g, device="cuda") - 0.5 for _ in range(2))
    X = torch.randn(batch * n * n, generator=g, device="cuda")
    Xt = X.view(batch, n, n).transpose(1, 2).contiguous().view(-1)
    Y1, Y2 = torch.empty_like(X), torch.empty_like(X)
    kron.kron2d_batched_ex_f32(n, "N", "N", "T", 1.0, A, B, X, 0.0, Y1, batch)
    kron.kron2d_batched_ex_f32(n, "N", "N", "N", 1.0, A, B, Xt, 0.0, Y2, batch)
    torch.cuda.synchronize()
    # the two calls run different kernels (tile loop vs tuned kernel): same
    # MFMA sequence per tile, so equal to rounding of the same sums
    torch.testing.assert_close(Y1, Y2, rtol=0, atol=0)


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
    assert call(beta=1.0) == 0
    assert call(opA=b"C") == -2           # op of A
    assert call(wsp=0) == -13             # workspace
    assert call(wsp=ws.data_ptr() + 2) == -13
    assert call(wsb=ws.numel() - 1) == -14
    torch.cuda.synchronize()
    with pytest.raises(ValueError):       # short workspace, caught by the binding
        kron.kron3d_batched_ex_f32(n, "N", "N", "N", 1.0, *mats, X, 0.5, Y, batch, ws=ws[:8])
    with pytest.raises(ValueError):
        kron.kron2d_batched_ex_f32(n, "X", "N", "N", 1.0, mats[0], mats[1], X, 0.0, Y, batch)
    with pytest.raises(ValueError):
        kron.kron2d_batched_ex_f32(n, "N", "N", "C", 1.0, mats[0], mats[1], X, 0.0, Y, batch)
    # opX is argument 4 of the 2-D entry points
    X2, Y2 = X[: batch * n * n], Y[: batch * n * n]
    assert L.kron2d_batched_ex_f32(n, b"N", b"N", b"Q", 1.0, p[0], p[1], X2.data_ptr(), 0.0, Y2.data_ptr(), batch,
                                   ws.data_ptr(), ws.numel(), s) == -4


@pytest.mark.parametrize("dim", [2, 3])
def test_internal_workspace_on_side_stream(dim):
    """The binding allocates the factor workspace itself when none is given.
    With the kernels on a side stream, a tensor allocated on the current
    stream right after the call must not reuse that block before the side
    stream's kernels have read it: the result still matches the oracle."""
    _need_gpu()
    n, batch = 16, 4096
    rng = np.random.default_rng(77 + dim)
    mats = [rng.uniform(-1, 1, n * n) for _ in range(dim)]
    X = rng.standard_normal(batch * n ** dim)
    tm = [torch.tensor(m, dtype=torch.float32, device="cuda") for m in mats]
    tx = torch.tensor(X, dtype=torch.float32, device="cuda")
    ty = torch.full_like(tx, float("nan"))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    ops = ("T", "N", "N") if dim == 2 else ("T", "N", "T")
    fn = getattr(kron, f"kron{dim}d_batched_ex_f32")
    # keep the side stream busy first so that its kernels start late
    with torch.cuda.stream(side):
        big = torch.randn(1 << 24, device="cuda")
        for _ in range(20):
            big = big * 1.0001
    fn(n, *ops, 1.25, *tm, tx, 0.0, ty, batch, None, side)
    # allocations on the current stream right after the call, overwritten at once
    junk = [torch.full((kron.kron_ex_workspace_size(dim, n, kron.MODE_F32) // 4,), 1e30, device="cuda")
            for _ in range(8)]
    torch.cuda.synchronize()
    del junk, big
    got = ty.double().cpu().numpy()
    hm = [t.double().cpu().numpy() for t in tm]
    if dim == 2:
        want = oracle.kron2d_ex(n, ops[0], ops[1], 1.25, *hm, X.astype(np.float32).astype(np.float64), 0.0,
                                np.zeros(X.size), batch, opX="N")
    else:
        want = oracle.kron3d_ex(n, *ops, 1.25, *hm, X.astype(np.float32).astype(np.float64), 0.0, np.zeros(X.size),
                                batch)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert np.all(np.isfinite(got)) and err <= 1e-5, err
