"""Parity of TKRON1 (Section 3's 1-D interface, y_p <- alpha op(A) x_p +
beta y_p) against the FP64 oracle: every n, both ops, alpha and beta,
padded and broadcast strides, a leading dimension on A, ragged batches
(not a multiple of the 16 vectors of a tile), the 16-byte path at n = 16,
a NaN that must stay in its own vector, the output gaps left untouched,
and the argument checks."""
import numpy as np
import pytest
import torch

import oracle
import paper_1304_7054_amd as kron

pytestmark = pytest.mark.gpu
DT = {"f32": torch.float32, "f64": torch.float64}
TOL = {"f32": 1e-5, "f64": 1e-13}
SENTINEL = 3.5


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(mode, n, op, alpha, beta, lda, ldxp, ldyp, batch, seed, nan_at=None):
    rng = np.random.default_rng(seed)
    dt = DT[mode]
    Abuf = np.full(lda * n, 1e6)
    Ad = rng.uniform(-1, 1, (n, n))
    for j in range(n):
        Abuf[j * lda:j * lda + n] = Ad[:, j]
    X = rng.standard_normal(max((batch - 1) * ldxp + n, 1) + 2)
    if nan_at is not None:
        X[nan_at * ldxp + n // 2] = np.nan
    ysize = (batch - 1) * ldyp + n + 2
    Y = np.full(ysize, SENTINEL)
    yi = (np.arange(batch)[:, None] * ldyp + np.arange(n)[None, :]).reshape(-1)
    if beta != 0.0:
        Y[yi] = rng.standard_normal(yi.size)
    tA, tX, tY = (torch.tensor(a, dtype=dt, device="cuda") for a in (Abuf, X, Y))
    ybefore = tY.double().cpu().numpy()
    fn = getattr(kron, f"kron1d_batched_{mode}")
    assert fn(n, op, alpha, tA, lda, tX, ldxp, beta, tY, ldyp, batch) == 0
    torch.cuda.synchronize()
    got = tY.double().cpu().numpy()
    hA = tA.double().cpu().numpy()[np.concatenate([np.arange(j * lda, j * lda + n) for j in range(n)])]
    want = oracle.kron1d_ex(n, op, alpha, hA, tX.double().cpu().numpy(), beta, ybefore, batch, ldxp, ldyp)
    gaps = np.ones(got.size, bool)
    gaps[yi] = False
    assert np.array_equal(got[gaps], ybefore[gaps]), "elements outside the output vectors were written"
    if nan_at is None:
        err = np.linalg.norm(got[yi] - want[yi]) / max(np.linalg.norm(want[yi]), 1e-300)
        assert err <= TOL[mode], (mode, n, op, err)
    else:
        g2, w2 = got[yi].reshape(batch, n), want[yi].reshape(batch, n)
        assert np.isnan(g2[nan_at]).any()
        keep = np.arange(batch) != nan_at
        assert np.isfinite(g2[keep]).all()
        np.testing.assert_allclose(g2[keep], w2[keep], rtol=TOL[mode] * 10, atol=TOL[mode])


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("n", list(range(1, 17)))
def test_tkron1_dense(mode, n):
    _need_gpu()
    _run(mode, n, "N", 1.0, 0.0, n, n, n, 1000 + 7, 1100 + n)


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("op", ["N", "T"])
@pytest.mark.parametrize("n", [3, 8, 16])
def test_tkron1_strided_alpha_beta(mode, op, n):
    _need_gpu()
    _run(mode, n, op, -0.75, 1.5, n + 2, n + 3, n + 1, 333, 1200 + n)


@pytest.mark.parametrize("mode", ["f32", "f64"])
@pytest.mark.parametrize("beta", [0.0, 2.0])
def test_tkron1_vector_path(mode, beta):
    """n = 16 with strides in multiples of 4 elements: 16-byte accesses."""
    _need_gpu()
    _run(mode, 16, "T", 0.5, beta, 16, 20, 24, 517, 1300)


def test_tkron1_broadcast_and_small_batch():
    _need_gpu()
    _run("f32", 7, "N", 1.0, 0.0, 7, 0, 7, 40, 1400)      # one vector repeated
    _run("f64", 16, "N", 1.0, 0.0, 16, 16, 16, 1, 1401)   # a single vector
    _run("f64", 5, "T", 2.0, -1.0, 5, 5, 5, 15, 1402)     # less than one tile


def test_tkron1_nan_stays_in_its_vector():
    _need_gpu()
    _run("f32", 16, "N", 1.0, 0.0, 16, 16, 16, 64, 1500, nan_at=21)
    _run("f64", 6, "N", 1.0, 0.0, 6, 6, 6, 64, 1501, nan_at=5)


def test_tkron1_argument_checks():
    _need_gpu()
    n, batch = 4, 10
    A = torch.zeros(n * n, device="cuda")
    X = torch.zeros(batch * n, device="cuda")
    Y = torch.zeros(batch * n, device="cuda")
    ws = torch.empty(kron.kron_ex_workspace_size(2, n, kron.MODE_F32), dtype=torch.uint8, device="cuda")
    L = kron.lib()
    s = torch.cuda.current_stream().cuda_stream

    def call(n_=n, op=b"N", lda=n, ldxp=n, ldyp=n, y=None, wsb=None):
        return L.kron1d_batched_f32(n_, op, 1.0, A.data_ptr(), lda, X.data_ptr(), ldxp, 0.0,
                                    Y.data_ptr() if y is None else y, ldyp, batch, ws.data_ptr(),
                                    ws.numel() if wsb is None else wsb, s)

    assert call() == 0
    assert call(n_=17) == -1
    assert call(op=b"C") == -2
    assert call(lda=n - 1) == -5
    assert call(ldxp=-1) == -7
    assert call(y=X.data_ptr()) == -9
    assert call(ldyp=n - 1) == -10
    assert call(wsb=4) == -13
    torch.cuda.synchronize()
    with pytest.raises(ValueError):
        kron.kron1d_batched_f32(n, "N", 1.0, A, n, X, n, 0.0, Y, n + 1, batch)   # Y too small
