"""Parity of the strided entry points (Section 3's TKRON2 / TKRON3 argument
layout with leading dimensions) against the FP64 oracle's extended
interface.  Operands are gathered from the strided buffers on the host into
dense arrays for the oracle; the result is compared at the strided output
positions, and every element of the output buffer between them must keep
its sentinel value bitwise (nothing outside the addressed elements is
written).  Covers padded columns, planes and operands, the operand stride 0
(one array broadcast), op on every factor and on 2-D operands, alpha, beta,
leading dimensions of the factors, packed tiles for n < 16 and ragged
batches, and the argument checks."""
import itertools

import numpy as np
import pytest
import torch

import oracle
import paper_1304_7054_amd as kron

pytestmark = pytest.mark.gpu
DT = {"f32": torch.float32, "f64": torch.float64}
TOL = {"f32": 1e-5, "f64": 1e-13}
SENTINEL = -7.25


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _index(n, dim, strides, batch):
    """Flat buffer index of every element, in dense (p, slow .., fast) order."""
    r = np.arange(n)
    if dim == 2:
        ld, ldp = strides
        idx = r[None, None, :] + ld * r[None, :, None] + ldp * np.arange(batch)[:, None, None]
    else:
        ld, ld2, ldp = strides
        idx = (r[None, None, None, :] + ld * r[None, None, :, None] + ld2 * r[None, :, None, None]
               + ldp * np.arange(batch)[:, None, None, None])
    return idx.reshape(-1)


def _padded_factor(rng, n, ld):
    """n x n factor in a column-major buffer with leading dimension ld
    (padding rows filled with a value that would show if read)."""
    buf = np.full(ld * n, 1e6)
    M = rng.uniform(-1, 1, (n, n))  # M[i, j]
    for j in range(n):
        buf[j * ld:j * ld + n] = M[:, j]
    dense = M.T.reshape(-1)  # column-major flat
    return buf, dense


def _run(mode, dim, n, ops, alpha, beta, lds, ldx, ldy, batch, seed):
    rng = np.random.default_rng(seed)
    dt = DT[mode]
    facs = [_padded_factor(rng, n, ld) for ld in lds]
    xi = _index(n, dim, ldx, batch)
    yi = _index(n, dim, ldy, batch)
    xbuf = rng.standard_normal(int(xi.max()) + 1 + 3)
    ybuf = np.full(int(yi.max()) + 1 + 3, SENTINEL)
    y0 = rng.standard_normal(yi.size)
    if beta != 0.0:
        ybuf[yi] = y0
    tm = [torch.tensor(b, dtype=dt, device="cuda") for b, _ in facs]
    tx = torch.tensor(xbuf, dtype=dt, device="cuda")
    ty = torch.tensor(ybuf, dtype=dt, device="cuda")
    ybefore = ty.double().cpu().numpy()
    args = []
    for t, ld in zip(tm, lds):
        args += [t, ld]
    fn = getattr(kron, f"kron{dim}d_batched_strided_{mode}")
    assert fn(n, *ops, alpha, *args, tx, *ldx, beta, ty, *ldy, batch) == 0
    torch.cuda.synchronize()
    got = ty.double().cpu().numpy()
    # the oracle on dense copies of exactly the device values
    hx = tx.double().cpu().numpy()[xi]
    hm = [t.double().cpu().numpy()[np.concatenate([np.arange(j * ld, j * ld + n) for j in range(n)])]
          for t, ld in zip(tm, lds)]
    hy0 = ybefore[yi]
    if dim == 2:
        want = oracle.kron2d_ex(n, ops[0], ops[1], alpha, *hm, hx, beta, hy0, batch, opX=ops[2])
    else:
        want = oracle.kron3d_ex(n, *ops, alpha, *hm, hx, beta, hy0, batch)
    out = got[yi]
    den = np.linalg.norm(want)
    err = np.linalg.norm(out - want) / den if den > 0 else np.linalg.norm(out)
    assert err <= TOL[mode], (mode, dim, n, ops, err)
    gaps = np.ones(got.size, bool)
    gaps[yi] = False
    assert np.array_equal(got[gaps], ybefore[gaps]), "elements outside the addressed ones were written"


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("n", [1, 3, 4, 5, 8, 11, 16])
def test_strided2d_padded(mode, n):
    _need_gpu()
    ldx, ldy = n + 3, n + 1
    _run(mode, 2, n, ("T", "N", "N"), 1.5, 0.0, (n + 2, n), (ldx, ldx * n + 5), (ldy, ldy * n + 2), 45, 600 + n)


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("n", [1, 2, 4, 5, 7, 10, 16])
def test_strided3d_padded(mode, n):
    _need_gpu()
    ldx, ldy = n + 1, n + 2
    _run(mode, 3, n, ("N", "T", "N"), -0.5, 0.0, (n, n + 1, n + 4),
         (ldx, ldx * n + 3, (ldx * n + 3) * n + 7), (ldy, ldy * n, ldy * n * n + 1), 13, 700 + n)


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_strided3d_vector_path(mode, beta):
    """3-D n = 16 with every stride a multiple of 4 elements: the 16-byte
    vector accesses (padded columns, planes and operands)."""
    _need_gpu()
    n = 16
    _run(mode, 3, n, ("T", "N", "N"), 1.25, beta, (n, n, n + 3), (20, 320, 320 * 16 + 8), (16, 260, 260 * 16),
         23, 950)


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("dim", [2, 3])
def test_strided_dense_layout_matches_ex(mode, dim):
    """Dense strides through the strided kernel give the _ex result (same
    products in the same order, so equal to the last bit)."""
    _need_gpu()
    n, batch = 16, 300 if dim == 2 else 40
    g = torch.Generator(device="cuda").manual_seed(8)
    dt = DT[mode]
    mats = [torch.rand(n * n, generator=g, device="cuda", dtype=dt) - 0.5 for _ in range(dim)]
    X = torch.randn(batch * n ** dim, generator=g, device="cuda", dtype=dt)
    Y0 = torch.randn(batch * n ** dim, generator=g, device="cuda", dtype=dt)
    Y1, Y2 = Y0.clone(), Y0.clone()
    if dim == 2:
        getattr(kron, f"kron2d_batched_ex_{mode}")(n, "T", "N", "T", 0.5, *mats, X, 2.0, Y1, batch)
        getattr(kron, f"kron2d_batched_strided_{mode}")(n, "T", "N", "T", 0.5, mats[0], n, mats[1], n, X, n, n * n,
                                                        2.0, Y2, n, n * n, batch)
    else:
        getattr(kron, f"kron3d_batched_ex_{mode}")(n, "T", "N", "T", 0.5, *mats, X, 2.0, Y1, batch)
        getattr(kron, f"kron3d_batched_strided_{mode}")(n, "T", "N", "T", 0.5, mats[0], n, mats[1], n, mats[2], n,
                                                        X, n, n * n, n ** 3, 2.0, Y2, n, n * n, n ** 3, batch)
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)


@pytest.mark.parametrize("ops", list(itertools.product("NT", repeat=3)))
def test_strided_all_ops_with_beta(ops):
    _need_gpu()
    n = 6
    _run("f64", 3, n, ops, 0.75, -1.25, (n + 1, n, n + 2), (n, n * n + 1, n ** 3 + 9), (n + 1, (n + 1) * n, (n + 1) * n * n),
         11, 800)
    _run("f32", 2, 9, ops, 0.75, 0.5, (9, 10), (11, 99 + 4), (9, 81), 70, 801)


def test_strided_broadcast_operand():
    """ldxp = 0: every output is the action on the same array."""
    _need_gpu()
    n = 5
    _run("f32", 3, n, ("N", "N", "N"), 1.0, 0.0, (n, n, n), (n, n * n, 0), (n, n * n, n ** 3), 29, 900)
    _run("f64", 2, 16, ("N", "T", "T"), 1.0, 0.0, (16, 16), (16, 0), (17, 17 * 16), 21, 901)


def test_strided_nonfinite_isolation():
    """A NaN in one operand of a packed tile stays in that operand."""
    _need_gpu()
    n, batch = 4, 40
    rng = np.random.default_rng(5)
    mats = [torch.tensor(rng.uniform(-1, 1, n * n), device="cuda") for _ in range(3)]
    ldp = n ** 3 + 2
    X = torch.tensor(rng.standard_normal(ldp * batch), device="cuda")
    X[9 * ldp + 5] = float("nan")
    Y = torch.zeros(ldp * batch, dtype=torch.float64, device="cuda")
    kron.kron3d_batched_strided_f64(n, "N", "N", "N", 1.0, mats[0], n, mats[1], n, mats[2], n, X, n, n * n, ldp, 0.0,
                                    Y, n, n * n, ldp, batch)
    torch.cuda.synchronize()
    y = Y.cpu().numpy().reshape(batch, ldp)[:, :n ** 3]
    assert np.isnan(y[9]).any()
    assert np.isfinite(np.delete(y, 9, axis=0)).all()


def test_strided_argument_checks():
    _need_gpu()
    n, batch = 4, 3
    A = torch.zeros(n * n, device="cuda")
    X = torch.zeros(batch * n * n, device="cuda")
    Y = torch.zeros(batch * n * n, device="cuda")
    ws = torch.empty(kron.kron_ex_workspace_size(2, n, kron.MODE_F32), dtype=torch.uint8, device="cuda")
    L = kron.lib()
    s = torch.cuda.current_stream().cuda_stream
    a = A.data_ptr()

    def call(lda=n, ldx=n, ldxp=n * n, ldy=n, ldyp=n * n, opX=b"N", y=None):
        return L.kron2d_batched_strided_f32(n, b"N", b"N", opX, 1.0, a, lda, a, n, X.data_ptr(), ldx, ldxp, 0.0,
                                            Y.data_ptr() if y is None else y, ldy, ldyp, batch, ws.data_ptr(),
                                            ws.numel(), s)

    assert call() == 0
    assert call(opX=b"Z") == -4
    assert call(lda=n - 1) == -7
    assert call(ldx=-1) == -11
    assert call(ldy=n - 1) == -15
    assert call(ldyp=n * n - 1) == -16
    assert call(y=X.data_ptr()) == -14
    torch.cuda.synchronize()
    with pytest.raises(ValueError):   # Y too small for its strides
        kron.kron2d_batched_strided_f32(n, "N", "N", "N", 1.0, A, n, A, n, X, n, n * n, 0.0, Y, n, n * n + 1, batch)
    with pytest.raises(ValueError):   # overlapping X and Y
        kron.kron2d_batched_strided_f32(n, "N", "N", "N", 1.0, A, n, A, n, X, n, n * n, 0.0, X, n, n * n, batch)


@pytest.mark.parametrize("n", [3, 16])
def test_factor_axis_roles_with_permutations(n):
    """Which factor acts on which axis of the strided 3-D entry point: with
    distinct permutation factors and index-coded X, the result is exactly the
    gathered copy Y[l, m, k] = X[pc[l], pb[m], pa[k]] (l fastest): C acts on
    the fastest index l, B on m and A on the slowest index k, i.e. the paper's
    K(C, B, A) in TKRON3's argument roles.  Padded strides, bitwise."""
    _need_gpu()
    rng = np.random.default_rng(5150 + n)
    pa, pb, pc = (rng.permutation(n) for _ in range(3))
    batch, ld = 5, n + 3
    ld2, ldp = ld * (n + 1), ld * (n + 1) * (n + 2)

    def perm_cm(p):
        P = np.zeros((n, n))
        P[np.arange(n), p] = 1.0
        return torch.tensor(P.T.reshape(-1), dtype=torch.float32, device="cuda")

    xi = _index(n, 3, (ld, ld2, ldp), batch)
    xbuf = np.zeros(int(xi.max()) + 1)
    xbuf[xi] = np.arange(xi.size) + 1.0
    ybuf = np.full(int(xi.max()) + 1, SENTINEL)
    tx = torch.tensor(xbuf, dtype=torch.float32, device="cuda")
    ty = torch.tensor(ybuf, dtype=torch.float32, device="cuda")
    kron.kron3d_batched_strided_f32(n, "N", "N", "N", 1.0, perm_cm(pa), n, perm_cm(pb), n, perm_cm(pc), n, tx, ld,
                                    ld2, ldp, 0.0, ty, ld, ld2, ldp, batch)
    torch.cuda.synchronize()
    got = ty.double().cpu().numpy()[xi].reshape(batch, n, n, n)   # [p, k, m, l]
    Xv = (np.arange(xi.size) + 1.0).reshape(batch, n, n, n)
    want = Xv[:, pa][:, :, pb][:, :, :, pc]
    assert np.array_equal(got, want)
