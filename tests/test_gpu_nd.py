"""GPU parity of the general action (kron_nd_batched_{f32,f64,c32,c64}):
d-dimensional operands (d = 1..5), rectangular factors with op in {N, T, C},
sizes above 16 (several 16-slot chunks per index), complex types, alpha and
beta, padded leading dimensions and factors per operand, element by element
against the FP64 / complex128 oracle on the same values.

Tolerances: normwise relative error over the batch <= 1e-5 for FP32 and
complex FP32 (both parts), <= 1e-13 for FP64 and complex FP64.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f32": 1e-5, "c32": 1e-5, "f64": 1e-13, "c64": 1e-13}
TDT = {"f32": torch.float32, "f64": torch.float64, "c32": torch.complex64, "c64": torch.complex128}
NDT = {"f32": np.float32, "f64": np.float64, "c32": np.complex64, "c64": np.complex128}


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _draw(rng, size, tag):
    v = rng.uniform(-1, 1, size)
    if tag in ("c32", "c64"):
        v = v + 1j * rng.uniform(-1, 1, size)
    return v.astype(NDT[tag])


def _case(seed, m, n, ops, tag, batch, varying=False, pad=0):
    rng = np.random.default_rng(seed)
    d = len(m)
    fs, ldf, ldfp = [], [], []
    for k in range(d):
        rows, cols = (m[k], n[k]) if ops[k] == "N" else (n[k], m[k])
        ld = rows + pad
        stride = ld * cols + pad if varying else 0
        size = (batch - 1) * stride + ld * cols if varying else ld * cols
        fs.append(_draw(rng, size, tag))
        ldf.append(ld)
        ldfp.append(stride)
    X = _draw(rng, batch * int(np.prod(n)), tag)
    Y0 = _draw(rng, batch * int(np.prod(m)), tag)
    return fs, ldf, ldfp, X, Y0


def _run(tag, m, n, ops, alpha, fs, ldf, ldfp, X, beta, Y0, batch, poison=False):
    import paper_1304_7054_amd as kron
    dt = TDT[tag]
    tf = [torch.from_numpy(f).to(DEV) for f in fs]
    tx = torch.from_numpy(X).to(DEV)
    ty = torch.from_numpy(Y0).to(DEV)
    if poison:
        ty.fill_(float("nan"))
    fn = getattr(kron, f"kron_nd_batched_{tag}")
    fn(m, n, ops, alpha, tf, tx, beta, ty, batch, ldf=ldf, ldfp=ldfp)
    torch.cuda.synchronize()
    assert ty.dtype == dt
    return ty.cpu().numpy()


def _check(tag, got, want):
    got = got.astype(np.complex128 if tag[0] == "c" else np.float64)
    assert np.all(np.isfinite(got)), "unwritten or non-finite outputs"
    err = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)
    assert err <= TOL[tag], err
    return err


SHAPES = [
    ([5], [3], "N"),
    ([16], [16], "T"),
    ([40], [23], "N"),
    ([3, 7], [5, 2], "NT"),
    ([16, 16], [16, 16], "NN"),
    ([17, 9], [12, 33], "TN"),
    ([4, 3, 5], [2, 6, 3], "NTN"),
    ([10, 10, 10], [10, 10, 10], "TNT"),
    ([16, 12, 16], [12, 16, 16], "NNT"),
    ([20, 18, 3], [19, 17, 5], "NTN"),
    ([3, 4, 2, 5], [2, 3, 4, 3], "NTTN"),
    ([6, 6, 6, 6], [6, 6, 6, 6], "NNNN"),
    ([2, 3, 2, 2, 3], [3, 2, 2, 3, 2], "TNTNT"),
    ([8, 32], [5, 32], "TN"),            # a pass with 32 faster elements: two columns per lane
    ([3, 4, 16], [2, 4, 16], "NTN"),     # 64 faster elements: four columns per lane
    ([7, 64], [9, 64], "NN"),
]


@pytest.mark.parametrize("tag", ["f32", "f64", "c32", "c64"])
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_nd_matches_oracle(tag, shape):
    _need_gpu()
    m, n, ops = SHAPES[shape]
    if tag[0] == "c":
        ops = ops.replace("T", "C") if shape % 2 else ops  # conjugate transposes on half the shapes
    batch = 37
    fs, ldf, ldfp, X, Y0 = _case(100 * shape + len(tag), m, n, ops, tag, batch)
    alpha = (1.25 - 0.5j) if tag[0] == "c" else -1.5
    got = _run(tag, m, n, ops, alpha, fs, ldf, ldfp, X, 0.0, Y0, batch, poison=True)
    want = oracle.kron_nd(m, n, ops, alpha, fs, X, 0.0, np.zeros(Y0.size), batch, ldf=ldf, ldfp=ldfp)
    _check(tag, got, want)


@pytest.mark.parametrize("tag", ["f32", "f64", "c32", "c64"])
@pytest.mark.parametrize("shape", [1, 4, 6, 9, 10])
def test_nd_beta_padding_and_per_operand_factors(tag, shape):
    """beta != 0 (Y read and updated), padded leading dimensions, and each
    operand with its own factors (ldfp > 0)."""
    _need_gpu()
    m, n, ops = SHAPES[shape]
    if tag[0] == "c":
        ops = ops.replace("N", "C", 1)
    batch = 11
    fs, ldf, ldfp, X, Y0 = _case(7 + shape, m, n, ops, tag, batch, varying=True, pad=3)
    alpha = (0.5 + 2j) if tag[0] == "c" else 0.75
    beta = (-0.25 + 0.5j) if tag[0] == "c" else 1.5
    got = _run(tag, m, n, ops, alpha, fs, ldf, ldfp, X, beta, Y0, batch)
    want = oracle.kron_nd(m, n, ops, alpha, fs, X, beta, Y0, batch, ldf=ldf, ldfp=ldfp)
    _check(tag, got, want)


def test_nd_per_operand_factors_differ():
    """Factors per operand give each operand its own action: the result for
    operand p equals a shared-factor call with operand p's factors."""
    _need_gpu()
    m, n, ops = [16, 5, 16], [16, 7, 16], "NTN"
    batch = 5
    fs, ldf, ldfp, X, Y0 = _case(91, m, n, ops, "f32", batch, varying=True)
    got = _run("f32", m, n, ops, 1.0, fs, ldf, ldfp, X, 0.0, Y0, batch)
    nx, ny = int(np.prod(n)), int(np.prod(m))
    for p in range(batch):
        one = [f[p * s:p * s + ld * (mm if o == "N" else nn)] for f, s, ld, mm, nn, o in zip(fs, ldfp, ldf, n, m, ops)]
        ref = _run("f32", m, n, ops, 1.0, one, ldf, [0] * 3, X[p * nx:(p + 1) * nx], 0.0, Y0[:ny], 1)
        assert np.array_equal(got[p * ny:(p + 1) * ny], ref), p


def test_nd_square_matches_plain_action():
    """Square real shared factors in 2-D and 3-D: the same action as the plain
    entry points (within FP32 rounding: the arithmetic order differs)."""
    _need_gpu()
    import paper_1304_7054_amd as kron
    rng = np.random.default_rng(5)
    for d, n in ((2, 16), (3, 16), (3, 7)):
        batch = 29
        mats = [rng.uniform(-1, 1, n * n).astype(np.float32) for _ in range(d)]
        X = rng.standard_normal(batch * n ** d).astype(np.float32)
        tm = [torch.from_numpy(M).to(DEV) for M in mats]
        tx = torch.from_numpy(X).to(DEV)
        y1, y2 = torch.empty_like(tx), torch.empty_like(tx)
        (kron.kron2d_batched_f32 if d == 2 else kron.kron3d_batched_f32)(n, *tm, tx, y1, batch)
        kron.kron_nd_batched_f32([n] * d, [n] * d, "N" * d, 1.0, tm, tx, 0.0, y2, batch)
        torch.cuda.synchronize()
        err = float((y1 - y2).double().norm() / y1.double().norm())
        assert err <= 1e-6, (d, n, err)


def test_nd_zero_batch_and_bad_arguments():
    _need_gpu()
    import ctypes
    import paper_1304_7054_amd as kron
    L = kron.lib()
    t = torch.zeros(4096, device=DEV)
    y = torch.full_like(t, 3.0)
    ci = ctypes.c_int * 2
    F = (ctypes.c_void_p * 2)(t.data_ptr(), t.data_ptr())
    ld = ci(4, 4)
    ldp = (ctypes.c_int64 * 2)(0, 0)
    ws = torch.empty(1 << 16, dtype=torch.uint8, device=DEV)
    call = lambda d, m, n, ops, ldf, ldfp, X, Y, b, w, wb: L.kron_nd_batched_f32(
        d, ci(*m), ci(*n), ops, 1.0, F, ldf, ldfp, X, 0.0, Y, b, w, wb, None)
    ok = (2, (4, 4), (4, 4), b"NN", ld, ldp, t.data_ptr(), y.data_ptr(), 3, ws.data_ptr(), ws.numel())
    assert call(*ok) == 0
    assert call(2, (4, 4), (4, 4), b"NN", ld, ldp, t.data_ptr(), y.data_ptr(), 0, None, 0) == 0   # batch 0: no-op
    bad = list(ok); bad[0] = 9; assert call(*bad) == -1
    bad = list(ok); bad[1] = (0, 4); assert call(*bad) == -2
    bad = list(ok); bad[3] = b"NX"; assert call(*bad) == -4
    bad = list(ok); bad[4] = ci(3, 4); assert call(*bad) == -7
    bad = list(ok); bad[5] = (ctypes.c_int64 * 2)(-1, 0); assert call(*bad) == -8
    bad = list(ok); bad[7] = t.data_ptr(); assert call(*bad) == -11
    bad = list(ok); bad[8] = -1; assert call(*bad) == -12
    bad = list(ok); bad[9] = None; assert call(*bad) == -13
    bad = list(ok); bad[10] = 16; assert call(*bad) == -14
    torch.cuda.synchronize()


@pytest.mark.parametrize("case", ["f32 4-D n=16", "c32 3-D n=16", "f32 2-D n=32", "f32 3-D varying n=16"])
def test_nd_full_size_sampled(case):
    """The benchmarked general-action workloads at full size (1 GiB of
    operands): every output finite, sampled operands against the oracle."""
    _need_gpu()
    import bench
    run = bench.ND_CASES[case]
    out = run(torch, check_only=True)
    assert out["sampled_rel_err"] <= TOL[out["tag"]], out
