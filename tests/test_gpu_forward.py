"""GPU parity of the forward and transposed actions against the CPU oracle.

Every call goes through the C ABI (ctypes binding).  Inputs are seeded
(workloads module), results are compared with the FP64 oracle on the exact
values the library received, element by element:
  * FP32 plain: normwise and per-operand relative error <= 1e-5
  * bf16x3: normwise <= 1e-5 (per-operand maximum <= 4e-5, reported)
  * bf16x6: normwise and per-operand <= 1e-5 (as plain FP32)
  * FP64: <= 1e-13
  * bf16 storage: <= 1e-2 against the FP64 oracle on the bf16-rounded inputs
Bit-exact cases (identity and permutation factors, small integers) compare
every element exactly.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from pins import cm, mat

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import gpu_util as gu

MODES = ["f32", "f64", "bf16x3", "bf16", "bf16x6"]
NS = list(range(1, 17))


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle(dim, n, mats, X, batch, transpose=False):
    if transpose:
        mats = [cm(mat(M, n).T) for M in mats]
    if dim == 2:
        return oracle.kron2d(n, mats[0], mats[1], X, batch, "f64")
    return oracle.kron3d(n, mats[0], mats[1], mats[2], X, batch, "f64")


def _inputs(dim, n, batch, seed, mode):
    rng = np.random.default_rng(seed)
    mats = [rng.uniform(-1, 1, n * n) for _ in range(dim)]
    X = rng.standard_normal(batch * n ** dim)
    if mode in ("f32", "bf16x3", "bf16x6", "adj_f32"):
        mats = [m.astype(np.float32) for m in mats]
        X = X.astype(np.float32)
    return mats, X


@pytest.mark.parametrize("n", NS)
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", MODES + ["adj_f32", "adj_f64"])
def test_forward_matches_oracle(mode, dim, n):
    _need_gpu()
    batch = gu.tiles_batch(dim, n)
    mats, X = _inputs(dim, n, batch, 1000 * dim + n, mode)
    got = gu.run(mode, dim, n, mats, X, batch)
    exact_in = gu.rounded_inputs(mode, mats + [X])
    want = _oracle(dim, n, exact_in[:-1], exact_in[-1], batch, transpose=mode.startswith("adj"))
    norm, per = gu.errors(got, want, batch)
    tol = gu.TOL[mode]
    assert np.all(np.isfinite(got)), "unwritten or non-finite outputs"
    assert norm <= tol, (mode, dim, n, norm)
    if mode in ("f32", "f64", "adj_f32", "adj_f64", "bf16x6"):
        # plain modes and bf16x6: the per-operand maximum is gated too
        assert per <= tol, (mode, dim, n, per)
    elif mode == "bf16x3":
        # the split keeps 16 significant bits per factor; operands with few
        # elements average less, so only the batch-normwise error is the gate
        assert per <= 4 * tol, (mode, dim, n, per)


# bf16x3 keeps 16 significant bits of every value (hi + lo); on log-uniform
# data few products dominate each output, so the batch-normwise error of the
# split averages over fewer terms.  Emulated worst case over n = 1..16 with
# these seeds: 1.1e-5 (3-D n = 4); the precision workload's own size (3-D
# n = 16) stays under the FP32 gate.
LOGU_TOL = {"f32": 1e-5, "bf16x3": 2e-5, "bf16x6": 1e-5, "bf16": 1e-2}


@pytest.mark.parametrize("n", NS)
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", ["f32", "bf16x3", "bf16x6", "bf16"])
def test_forward_log_uniform(mode, dim, n):
    """The precision workload's distribution at every n: every entry of the
    factors and the operands log-uniform in magnitude on [1e-3, 1e3] with a
    random sign, element-wise against the FP64 oracle.  bf16 storage is
    gated against the oracle on both the rounded inputs and the original
    FP32 values."""
    _need_gpu()
    batch = gu.tiles_batch(dim, n)
    rng = np.random.default_rng(5000 + 100 * dim + n)
    mats = [workloads.log_uniform(rng, n * n, np.float32) for _ in range(dim)]
    X = workloads.log_uniform(rng, batch * n ** dim, np.float32)
    got = gu.run(mode, dim, n, mats, X, batch)
    assert np.all(np.isfinite(got)), "unwritten or non-finite outputs"
    exact_in = gu.rounded_inputs(mode, mats + [X])
    want = _oracle(dim, n, exact_in[:-1], exact_in[-1], batch)
    norm, per = gu.errors(got, want, batch)
    tol = 1e-5 if (mode == "bf16x3" and dim == 3 and n == 16) else LOGU_TOL[mode]
    assert norm <= tol, (mode, dim, n, norm)
    if mode in ("f32", "bf16x6"):
        assert per <= tol, (mode, dim, n, per)
    if mode == "bf16":
        orig = _oracle(dim, n, [m.astype(np.float64) for m in mats], X.astype(np.float64), batch)
        norm_i, _ = gu.errors(got, orig, batch)
        assert norm_i <= 1e-2, (dim, n, norm_i)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 12, 16])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", MODES)
def test_identity_is_bit_exact(mode, dim, n):
    _need_gpu()
    batch = gu.tiles_batch(dim, n)
    rng = np.random.default_rng(7)
    X = rng.standard_normal(batch * n ** dim).astype(np.float32)
    if mode == "bf16x3":
        # the hi + lo split holds 16 significant bits; such values pass exactly
        X = (X.view(np.uint32) & np.uint32(0xFFFFFF00)).view(np.float32)
    I = workloads.identity_cm(n, np.float64)
    got = gu.run(mode, dim, n, [I] * dim, X, batch)
    want = gu.rounded_inputs(mode, [X])[0]
    assert np.array_equal(got.astype(np.float64), want)


def _perm_cm(n, perm):
    P = np.zeros((n, n))
    P[np.arange(n), perm] = 1.0
    return cm(P)


@pytest.mark.parametrize("n", [2, 3, 4, 6, 7, 10, 13, 16])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", MODES)
def test_permutation_is_bit_exact(mode, dim, n):
    """Distinct permutations per factor and index-coded X: Y must be the
    gathered copy X[pa[i], pb[j](, pc[k])] exactly (factor <-> axis mapping)."""
    _need_gpu()
    batch = gu.tiles_batch(dim, n)
    rng = np.random.default_rng(100 + n)
    perms = [rng.permutation(n) for _ in range(dim)]
    size = batch * n ** dim
    # values exactly representable: 8 significant bits for bf16 storage, 16 for
    # the bf16x3 split, 24 for FP32
    limit = {"bf16": 256, "bf16x3": 1 << 16}.get(mode, 1 << 24)   # bf16x6 holds all 24 bits
    X = (np.arange(size) % limit).astype(np.float64) + 1.0
    got = gu.run(mode, dim, n, [_perm_cm(n, p) for p in perms], X, batch)
    Xv = X.reshape((batch,) + (n,) * dim)
    if dim == 2:
        want = Xv[:, perms[0]][:, :, perms[1]]
    else:
        want = Xv[:, perms[0]][:, :, perms[1]][:, :, :, perms[2]]
    assert np.array_equal(got.astype(np.float64), want.reshape(-1))


@pytest.mark.parametrize("n", [3, 5, 8, 11, 16])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", MODES)
def test_small_integers_are_bit_exact(mode, dim, n):
    """A, B, C in {-2..2}, X in {-8..8}: all partial sums are exact in FP32,
    so the library must equal the oracle bit for bit (bf16 storage: the
    exact result rounded to bf16, nearest even)."""
    _need_gpu()
    batch = gu.tiles_batch(dim, n)
    rng = np.random.default_rng(300 + n)
    mats = [rng.integers(-2, 3, n * n).astype(np.float64) for _ in range(dim)]
    X = rng.integers(-8, 9, batch * n ** dim).astype(np.float64)
    got = gu.run(mode, dim, n, mats, X, batch)
    want = _oracle(dim, n, mats, X, batch)
    if mode == "bf16":
        want = torch.from_numpy(want.astype(np.float32)).to(torch.bfloat16).float().numpy()
    assert np.array_equal(got.astype(np.float64), want.astype(np.float64))


@pytest.mark.parametrize("n", [2, 5, 16])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", ["f32", "f64", "bf16x3", "bf16x6"])
def test_nan_stays_in_its_operand(mode, dim, n):
    """A NaN in one operand affects that operand's output only (packed tiles
    included), and a NaN-filled Y never leaks into the result."""
    _need_gpu()
    batch = gu.tiles_batch(dim, n)
    mats, X = _inputs(dim, n, batch, 55, mode)
    q = batch // 2
    X = X.copy()
    X[q * n ** dim + (n ** dim) // 2] = np.nan
    got = gu.run(mode, dim, n, mats, X, batch).reshape(batch, -1)
    bad = [p for p in range(batch) if not np.all(np.isfinite(got[p]))]
    assert bad == [q], bad
    exact_in = gu.rounded_inputs(mode, mats + [X])
    want = _oracle(dim, n, exact_in[:-1], exact_in[-1], batch).reshape(batch, -1)
    keep = np.arange(batch) != q
    norm, _ = gu.errors(got[keep], want[keep], batch - 1)
    assert norm <= gu.TOL[mode]


@pytest.mark.parametrize("n", [3, 16])
@pytest.mark.parametrize("dim", [2, 3])
def test_unaligned_pointers(dim, n):
    """Operand arrays that do not start on a 16-byte boundary (X and Y
    offset alike or differently) take the element-wise or shifted-staging
    paths and give the same bits."""
    _need_gpu()
    batch = gu.tiles_batch(dim, n)
    mats, X = _inputs(dim, n, batch, 77, "f32")
    a = gu.run("f32", dim, n, mats, X, batch)
    b = gu.run("f32", dim, n, mats, X, batch, x_offset=1, y_offset=3)
    assert np.array_equal(a, b)
    c = gu.run("f32", dim, n, mats, X, batch, x_offset=2, y_offset=2)   # same phase, not 16-byte aligned
    assert np.array_equal(a, c)


@pytest.mark.parametrize("dim", [2, 3])
def test_zero_batch_and_bad_arguments(dim):
    _need_gpu()
    import paper_1304_7054_amd as kron
    n = 4
    t = torch.zeros(n ** dim * 2, device=gu.DEV)
    M = torch.zeros(n * n, device=gu.DEV)
    fn = gu.FWD[("f32", dim)]
    mats = [M] * dim
    y = torch.full_like(t, 7.0)
    assert fn(n, *mats, t, y, 0) == 0                           # batch 0: no-op
    assert torch.all(y == 7.0)
    raw = getattr(kron.lib(), fn.__name__)
    p = [M.data_ptr()] * dim
    assert raw(n, *p, t.data_ptr(), t.data_ptr(), 1, None) == -(dim + 3)   # X == Y
    assert raw(0, *p, t.data_ptr(), y.data_ptr(), 1, None) == -1
    assert raw(n, *p, t.data_ptr(), y.data_ptr(), -1, None) == -(dim + 4)
    with pytest.raises(ValueError):
        fn(n, *mats, t, t, 1)                                   # the binding rejects overlap too
    with pytest.raises(ValueError):
        fn(17, *mats, t, torch.empty_like(t), 1)
    with pytest.raises(ValueError):
        fn(n, *mats, t, torch.empty_like(t), 3)                 # too small for 3 operands


def test_repeated_runs_are_bitwise_identical():
    _need_gpu()
    mats, X = _inputs(3, 16, 64, 5, "f32")
    a = gu.run("f32", 3, 16, mats, X, 64)
    b = gu.run("f32", 3, 16, mats, X, 64)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n", [4, 7, 10, 16])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", ["f32", "bf16x3", "f64", "bf16", "bf16x6"])
def test_launch_variants_agree(mode, dim, n):
    """Every launch shape gives a correct result, and shapes that share an
    arithmetic order give the same bits.  One workgroup per CU forces the
    grid-stride loops to run many tiles per wavefront.  The 3-D variants with
    bit 1 set contract the modes in another order (C, B, A instead of C, A, B),
    so they are compared with the oracle, not bit for bit with the others."""
    _need_gpu()
    import paper_1304_7054_amd as kron
    mcode = {"f32": kron.MODE_F32, "bf16x3": kron.MODE_BF16X3, "f64": kron.MODE_F64, "bf16": kron.MODE_BF16,
             "bf16x6": kron.MODE_BF16X6}[mode]
    q = 16 // n
    batch = 256 * 4 * 3 * q ** dim + 5     # several tiles per wavefront at 1 block per CU
    if mode == "f64":
        batch = batch // 4 + 3
    mats, X = _inputs(dim, n, batch, 99, mode)
    want = _oracle(dim, n, gu.rounded_inputs(mode, mats), gu.rounded_inputs(mode, [X])[0], batch)
    refs = {}
    try:
        for variant in (list(range(12)) if dim == 3 else [0, 1, 2, 3, 4]):
            # 3-D variants 2..7, 8 and 11 (LDS-staged) and 9/10 (stores
            # interleaved with the next tile, n = 16; variant 4 otherwise)
            # contract C, B, A; 0 and 1 contract C, A, B.  Variants 8 and 11
            # at a size they cannot use run variant 0.
            stageable = n != 16
            if dim == 2:
                order = 0
            elif variant in (8, 11):
                order = 1 if stageable else 0
            elif variant in (9, 10):
                order = 1
            else:
                order = 1 if variant >= 2 else 0
            for blocks in (0, 1):
                kron.kron_set_launch(mcode, dim, n, blocks, variant)
                got = gu.run(mode, dim, n, mats, X, batch)
                assert gu.errors(got, want, batch)[0] <= gu.TOL[mode], (variant, blocks)
                if order in refs:
                    assert np.array_equal(got, refs[order]), (variant, blocks)
                else:
                    refs[order] = got
    finally:
        kron.kron_set_launch(mcode, dim, n, -1, 0)


@pytest.mark.parametrize("n", [2, 5, 10])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_nan_isolation_in_both_staged_pipelines(mode, dim, n):
    """The NaN rule holds in both LDS-staged pipelines whatever the launch
    table picks: the single-slice one (2-D variant 3, 3-D variant 8) and the
    one with two slices and deferred stores (2-D 4, 3-D 11), which writes a
    tile's results out only after the next tile's operands are in LDS."""
    _need_gpu()
    import paper_1304_7054_amd as kron
    mcode = {"f32": kron.MODE_F32, "bf16x3": kron.MODE_BF16X3}[mode]
    # several tiles (2-D: spans of up to 8 tiles) per wavefront at one
    # workgroup per CU on 256 CUs, plus a ragged tail
    per_tile = (16 // n) ** dim
    batch = 1024 * 3 * per_tile * (8 if dim == 2 else 1) + max(1, per_tile // 3)
    mats, X = _inputs(dim, n, batch, 57, mode)
    q = batch // 3
    X = X.copy()
    X[q * n ** dim + (n ** dim) // 3] = np.nan
    exact_in = gu.rounded_inputs(mode, mats + [X])
    want = _oracle(dim, n, exact_in[:-1], exact_in[-1], batch).reshape(batch, -1)
    keep = np.arange(batch) != q
    outs = []
    try:
        for variant in ((3, 4) if dim == 2 else (8, 11)):
            kron.kron_set_launch(mcode, dim, n, 1, variant)  # one workgroup per CU: many tiles per wavefront
            got = gu.run(mode, dim, n, mats, X, batch).reshape(batch, -1)
            bad = np.nonzero(~np.all(np.isfinite(got), axis=1))[0].tolist()
            assert bad == [q], (variant, bad[:8])
            norm, _ = gu.errors(got[keep], want[keep], batch - 1)
            assert norm <= gu.TOL[mode], variant
            outs.append(got)
    finally:
        kron.kron_set_launch(mcode, dim, n, -1, 0)
    assert np.array_equal(outs[0][keep], outs[1][keep])
