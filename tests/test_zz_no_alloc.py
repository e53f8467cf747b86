"""The allocation-free entry point kron3d_batched_ex_f32_noalloc against the
workspace entry point kron3d_batched_ex_f32 (same kernels on the same
prepared factors: equal bit for bit) and against the FP64 oracle, on two
calls in a row, the second with a smaller input."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


def _case(rng, n, batch):
    mats = [rng.uniform(-1, 1, n * n).astype(np.float32) for _ in range(3)]
    X = rng.standard_normal(batch * n ** 3).astype(np.float32)
    Y0 = rng.standard_normal(batch * n ** 3).astype(np.float32)
    return mats, X, Y0


def _run_pair(kron, n, ops, alpha, beta, mats, X, Y0, batch):
    dev = "cuda:0"
    tm = [torch.from_numpy(m).to(dev) for m in mats]
    tx = torch.from_numpy(X).to(dev)
    y_ref = torch.from_numpy(Y0).to(dev)
    y_na = torch.from_numpy(Y0).to(dev)
    if beta == 0.0:
        y_ref.fill_(float("nan"))
        y_na.fill_(float("nan"))
    ws = torch.empty(kron.kron_ex_workspace_size(3, n, kron.MODE_F32), dtype=torch.uint8, device=dev)
    assert kron.kron3d_batched_ex_f32(n, *ops, alpha, *tm, tx, beta, y_ref, batch, ws) == 0
    # through the C ABI directly: no workspace argument exists
    raw = kron.lib().kron3d_batched_ex_f32_noalloc
    rc = raw(n, *[o.encode() for o in ops], alpha, *[t.data_ptr() for t in tm], tx.data_ptr(), beta,
             y_na.data_ptr(), batch, torch.cuda.current_stream().cuda_stream)
    assert rc == 0, kron.status_string(rc)
    torch.cuda.synchronize()
    return y_ref.cpu().numpy(), y_na.cpu().numpy()


def test_noalloc_matches_workspace_entry_point_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1304_7054_amd as kron
    rng = np.random.default_rng(20260)
    # first call: n = 16, beta != 0, mixed ops; second: smaller n and batch, beta = 0
    for n, batch, ops, alpha, beta in ((16, 37, ("T", "N", "T"), -1.5, 0.5), (5, 9, ("N", "T", "N"), 2.0, 0.0)):
        mats, X, Y0 = _case(rng, n, batch)
        ref, got = _run_pair(kron, n, ops, alpha, beta, mats, X, Y0, batch)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref), (n, batch)
        want = oracle.kron3d_ex(n, *ops, alpha, *[m.astype(np.float64) for m in mats], X.astype(np.float64), beta,
                                Y0.astype(np.float64), batch)
        err = np.linalg.norm(got.astype(np.float64) - want) / np.linalg.norm(want)
        assert err <= 1e-5, (n, err)


def test_noalloc_rejects_bad_arguments():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1304_7054_amd as kron
    raw = kron.lib().kron3d_batched_ex_f32_noalloc
    t = torch.zeros(16 ** 3, device="cuda:0")
    M = torch.zeros(256, device="cuda:0")
    y = torch.full_like(t, 3.0)
    p = M.data_ptr()
    assert raw(17, b"N", b"N", b"N", 1.0, p, p, p, t.data_ptr(), 0.0, y.data_ptr(), 1, None) == -1
    assert raw(16, b"X", b"N", b"N", 1.0, p, p, p, t.data_ptr(), 0.0, y.data_ptr(), 1, None) == -2
    assert raw(16, b"N", b"N", b"N", 1.0, p, p, p, t.data_ptr(), 0.0, t.data_ptr(), 1, None) == -11
    assert raw(16, b"N", b"N", b"N", 1.0, p, p, p, t.data_ptr(), 0.0, y.data_ptr(), -1, None) == -12
    assert raw(16, b"N", b"N", b"N", 1.0, p, p, p, t.data_ptr(), 0.0, y.data_ptr(), 0, None) == 0
    torch.cuda.synchronize()
    assert bool((y == 3.0).all())
