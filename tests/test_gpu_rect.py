"""GPU parity of Section 3's TKRON1 / TKRON2 / TKRON3 argument lists with
rectangular factors (kron{1,2,3}d_batched_rect_{f32,f64,c32,c64}): op in
{N, T, C} on every factor and on the 2-D operands, alpha, beta, padded
leading dimensions on factors, operands and results.  The oracle runs on
dense copies of exactly the device values (gathered from the strided
storage); the results are compared at the strided addresses, and every
output element between them must keep its sentinel value, bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f32": 1e-5, "c32": 1e-5, "f64": 1e-13, "c64": 1e-13}
NDT = {"f32": np.float32, "f64": np.float64, "c32": np.complex64, "c64": np.complex128}


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _draw(rng, size, tag):
    v = rng.uniform(-1, 1, size)
    if tag[0] == "c":
        v = v + 1j * rng.uniform(-1, 1, size)
    return v.astype(NDT[tag])


def _factor(rng, tag, op, m, n, pad):
    rows, cols = (m, n) if op == "N" else (n, m)
    ld = rows + pad
    return _draw(rng, ld * cols, tag), ld


def _index(exts, strides, batch, sp):
    """Flat offsets of every element (operand-major, last index fastest)."""
    grids = np.meshgrid(*[np.arange(e) for e in exts], indexing="ij")
    one = sum(g * s for g, s in zip(grids, strides)).reshape(-1)
    return (np.arange(batch)[:, None] * sp + one[None, :]).reshape(-1)


def _compare(tag, Y, got, yidx, want, sentinel):
    assert np.all(np.isfinite(got[yidx])), "unwritten or non-finite outputs"
    err = np.linalg.norm(got[yidx] - want) / max(np.linalg.norm(want), 1e-300)
    assert err <= TOL[tag], err
    gaps = np.ones(got.size, bool)
    gaps[yidx] = False
    assert np.array_equal(got[gaps], sentinel[gaps]), "elements outside the addressed outputs changed"


CASES2 = [  # ops (A, B, X), ma, na, mb, nb, pad
    ("NNN", 3, 5, 4, 2, 0),
    ("TNT", 16, 16, 9, 12, 3),
    ("NTN", 7, 1, 1, 7, 1),
    ("CNC", 5, 6, 7, 4, 2),
    ("NCT", 20, 17, 3, 18, 1),
]


@pytest.mark.parametrize("tag", ["f32", "f64", "c32", "c64"])
@pytest.mark.parametrize("case", range(len(CASES2)))
@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_rect2d(tag, case, beta):
    _need_gpu()
    import paper_1304_7054_amd as kron
    ops, ma, na, mb, nb, pad = CASES2[case]
    if tag[0] == "f":
        ops = ops.replace("C", "T")   # conjugation of real data is the transpose
    rng = np.random.default_rng(10 * case + len(tag))
    batch = 13
    A, lda = _factor(rng, tag, ops[0], ma, na, pad)
    B, ldb = _factor(rng, tag, ops[1], mb, nb, pad + 1)
    xrows = nb if ops[2] == "N" else na
    ldx = xrows + pad
    ldxp = ldx * (na if ops[2] == "N" else nb) + pad
    X = _draw(rng, ldxp * batch, tag)
    ldy, ldyp = mb + pad + 1, (mb + pad + 1) * ma + 2
    Ysent = _draw(rng, ldyp * batch, tag)
    alpha = (1.5 - 0.25j) if tag[0] == "c" else -1.25
    beta_v = (beta * (1 + 1j)) if tag[0] == "c" else beta
    tY = torch.from_numpy(Ysent.copy()).to(DEV)
    fn = getattr(kron, f"kron2d_batched_rect_{tag}")
    fn(ops[0], ops[1], ops[2], ma, na, mb, nb, batch, alpha, torch.from_numpy(A).to(DEV), lda,
       torch.from_numpy(B).to(DEV), ldb, torch.from_numpy(X).to(DEV), ldx, ldxp, beta_v, tY, ldy, ldyp)
    torch.cuda.synchronize()
    got = tY.cpu().numpy()
    # op(X_p)(a0, a1) with a1 the fast index: X_p(a1, a0) at a1 + ldx*a0, or (op T / C) at a0 + ldx*a1
    xs = [ldx, 1] if ops[2] == "N" else [1, ldx]
    xd = X[_index([na, nb], xs, batch, ldxp)]
    if ops[2] == "C":
        xd = xd.conj()
    yidx = _index([ma, mb], [ldy, 1], batch, ldyp)
    want = oracle.kron_nd([ma, mb], [na, nb], ops[:2], alpha, [A, B], xd, beta_v, Ysent[yidx], batch, ldf=[lda, ldb])
    _compare(tag, tY, got, yidx, want, Ysent if beta == 0.0 else got)


CASES3 = [  # ops, (ma, na, mb, nb, mc, nc), pad
    ("NNN", (3, 5, 4, 2, 6, 3), 0),
    ("TNT", (16, 16, 12, 16, 16, 9), 2),
    ("CTN", (5, 1, 1, 5, 7, 7), 1),
    ("NCC", (18, 4, 3, 17, 2, 20), 1),
]


@pytest.mark.parametrize("tag", ["f32", "f64", "c32", "c64"])
@pytest.mark.parametrize("case", range(len(CASES3)))
@pytest.mark.parametrize("beta", [0.0, -2.0])
def test_rect3d(tag, case, beta):
    _need_gpu()
    import paper_1304_7054_amd as kron
    ops, (ma, na, mb, nb, mc, nc), pad = CASES3[case]
    if tag[0] == "f":
        ops = ops.replace("C", "T")
    rng = np.random.default_rng(100 + 10 * case + len(tag))
    batch = 7
    A, lda = _factor(rng, tag, ops[0], ma, na, pad)
    B, ldb = _factor(rng, tag, ops[1], mb, nb, pad)
    C, ldc = _factor(rng, tag, ops[2], mc, nc, pad + 2)
    ldx, ldx2 = nc + pad, (nc + pad) * nb + 1
    ldxp = ldx2 * na + pad
    X = _draw(rng, ldxp * batch, tag)
    ldy, ldy2 = mc + 1, (mc + 1) * mb + pad
    ldyp = ldy2 * ma + 3
    Ysent = _draw(rng, ldyp * batch, tag)
    alpha = (0.5 + 0.75j) if tag[0] == "c" else 2.0
    beta_v = complex(beta, 0.5) if tag[0] == "c" and beta != 0 else beta
    tY = torch.from_numpy(Ysent.copy()).to(DEV)
    fn = getattr(kron, f"kron3d_batched_rect_{tag}")
    fn(ops[0], ops[1], ops[2], ma, na, mb, nb, mc, nc, batch, alpha, torch.from_numpy(A).to(DEV), lda,
       torch.from_numpy(B).to(DEV), ldb, torch.from_numpy(C).to(DEV), ldc, torch.from_numpy(X).to(DEV), ldx, ldx2,
       ldxp, beta_v, tY, ldy, ldy2, ldyp)
    torch.cuda.synchronize()
    got = tY.cpu().numpy()
    xd = X[_index([na, nb, nc], [ldx2, ldx, 1], batch, ldxp)]
    yidx = _index([ma, mb, mc], [ldy2, ldy, 1], batch, ldyp)
    want = oracle.kron_nd([ma, mb, mc], [na, nb, nc], ops, alpha, [A, B, C], xd, beta_v, Ysent[yidx], batch,
                          ldf=[lda, ldb, ldc])
    _compare(tag, tY, got, yidx, want, Ysent if beta == 0.0 else got)


@pytest.mark.parametrize("tag", ["f32", "f64", "c32", "c64"])
@pytest.mark.parametrize("ma,na,op", [(5, 3, "N"), (16, 16, "T"), (1, 20, "C"), (33, 7, "N")])
def test_rect1d(tag, ma, na, op):
    _need_gpu()
    import paper_1304_7054_amd as kron
    if tag[0] == "f":
        op = op.replace("C", "T")
    rng = np.random.default_rng(ma * 7 + na)
    batch = 45
    A, lda = _factor(rng, tag, op, ma, na, 2)
    ldxp, ldyp = na + 3, ma + 1
    X = _draw(rng, ldxp * batch, tag)
    Ysent = _draw(rng, ldyp * batch, tag)
    alpha = (2 - 1j) if tag[0] == "c" else 0.5
    beta = (0.25 + 0.25j) if tag[0] == "c" else -1.0
    tY = torch.from_numpy(Ysent.copy()).to(DEV)
    getattr(kron, f"kron1d_batched_rect_{tag}")(op, ma, na, batch, alpha, torch.from_numpy(A).to(DEV), lda,
                                               torch.from_numpy(X).to(DEV), ldxp, beta, tY, ldyp)
    torch.cuda.synchronize()
    got = tY.cpu().numpy()
    xd = X[_index([na], [1], batch, ldxp)]
    yidx = _index([ma], [1], batch, ldyp)
    want = oracle.kron_nd([ma], [na], op, alpha, [A], xd, beta, Ysent[yidx], batch, ldf=[lda])
    _compare(tag, tY, got, yidx, want, got)
    gaps = np.ones(got.size, bool)
    gaps[yidx] = False
    assert np.array_equal(got[gaps], Ysent[gaps])


def test_rect_argument_checks():
    _need_gpu()
    import paper_1304_7054_amd as kron
    L = kron.lib()
    t = torch.zeros(4096, device=DEV)
    y = torch.zeros(4096, device=DEV)
    p, q = t.data_ptr(), y.data_ptr()
    ws = torch.empty(kron.kron_nd_workspace_size([3, 5], [4, 6], 2, kron.MODE_F32), dtype=torch.uint8, device=DEV)
    ok = [b"N", b"N", b"N", 3, 4, 5, 6, 2, 1.0, p, 3, p, 5, p, 6, 24, 0.0, q, 5, 15, ws.data_ptr(), ws.numel(), None]
    f = L.kron2d_batched_rect_f32
    assert f(*ok) == 0
    for pos, val in ((1, b"X"), (3, b"Q"), (4, 0), (7, 70000), (8, -1), (11, 2), (13, 4), (15, -1), (18, p),
                     (19, 4), (20, 14), (21, None), (22, ws.numel() - 1)):
        bad = list(ok)
        bad[pos - 1] = val
        assert f(*bad) == -pos, pos
    torch.cuda.synchronize()
