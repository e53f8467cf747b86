"""One persistent launch over mixed (dim, n) groups, eager and replayed from
a captured HIP graph, against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _make_groups(spec, seed, mode=0):
    """spec: list of (dim, n, count); returns (device groups, host arrays)."""
    rng = np.random.default_rng(seed)
    groups, host = [], []
    for dim, n, count in spec:
        mats = [rng.uniform(-1, 1, n * n).astype(np.float32) for _ in range(dim)]
        X = rng.standard_normal(count * n ** dim).astype(np.float32)
        g = {"dim": dim, "n": n, "count": count, "mode": mode,
             "X": torch.from_numpy(X).to(DEV), "Y": torch.full((count * n ** dim,), float("nan"), device=DEV)}
        for k, m in zip("ABC", mats):
            g[k] = torch.from_numpy(m).to(DEV)
        groups.append(g)
        host.append((mats, X))
    return groups, host


def _check(groups, host, tol=1e-5):
    for g, (mats, X) in zip(groups, host):
        n, dim, count = g["n"], g["dim"], g["count"]
        got = g["Y"].cpu().numpy().astype(np.float64)
        if count == 0:
            continue
        want = (oracle.kron2d if dim == 2 else oracle.kron3d)(n, *[m.astype(np.float64) for m in mats],
                                                               X.astype(np.float64), count, "f64")
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert np.all(np.isfinite(got)) and err <= tol, (dim, n, count, err)


@pytest.mark.parametrize("mode", [0, 2])
def test_grouped_all_sizes(mode):
    import paper_1304_7054_amd as kron
    _need_gpu()
    spec = [(d, n, (37 if d == 2 else 5) * (16 // n) ** (d - 1) + 3) for d in (2, 3) for n in range(1, 17)]
    spec += [(2, 7, 0), (3, 16, 1)]
    groups, host = _make_groups(spec, 11, mode)
    ws = torch.empty(kron.kron_grouped_workspace_size(groups), dtype=torch.uint8, device=DEV)
    kron.kron_grouped_prepare(groups, ws)
    kron.kron_grouped_launch(ws)
    torch.cuda.synchronize()
    _check(groups, host)


def test_grouped_graph_replay_matches_eager():
    import paper_1304_7054_amd as kron
    _need_gpu()
    spec = [(2, 6, 2000), (2, 9, 900), (3, 8, 300), (3, 10, 120), (3, 16, 40), (2, 16, 500)]
    groups, host = _make_groups(spec, 12)
    ws = torch.empty(kron.kron_grouped_workspace_size(groups), dtype=torch.uint8, device=DEV)
    kron.kron_grouped_prepare(groups, ws)
    kron.kron_grouped_launch(ws)
    torch.cuda.synchronize()
    _check(groups, host)
    eager = [g["Y"].clone() for g in groups]
    exe = kron.kron_graph_capture_grouped(ws)
    try:
        for rep in range(4):
            for g in groups:
                g["Y"].fill_(float("nan"))          # eager work between replays
            torch.cuda.synchronize()
            kron.kron_graph_launch(exe)
            torch.cuda.synchronize()
            for g, e in zip(groups, eager):
                assert torch.equal(g["Y"], e), rep
    finally:
        kron.kron_graph_destroy(exe)


def test_grouped_rejects_bad_plans():
    import paper_1304_7054_amd as kron
    _need_gpu()
    groups, _ = _make_groups([(3, 5, 10)], 13)
    need = kron.kron_grouped_workspace_size(groups)
    small = torch.empty(max(1, need // 2), dtype=torch.uint8, device=DEV)
    with pytest.raises(kron.KronError):
        kron.kron_grouped_prepare(groups, small)
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    other = torch.empty(need, dtype=torch.uint8, device=DEV)
    with pytest.raises(kron.KronError):
        kron.kron_grouped_launch(other)                 # never prepared
    kron.kron_grouped_prepare(groups, ws)
    kron.kron_grouped_launch(ws)


def test_mixed_workload_sampled():
    """The 500,000-operand mixed workload (seeded), one launch, checked on
    sampled operands of every group against the FP64 oracle."""
    import paper_1304_7054_amd as kron
    _need_gpu()
    probs = workloads.workload4()
    groups = []
    for p in probs:
        g = {"dim": p.dim, "n": p.n, "count": p.batch, "X": torch.from_numpy(p.X).to(DEV),
             "Y": torch.empty(p.X.size, device=DEV)}
        for k, m in zip("ABC", (p.A, p.B, p.C)):
            if m is not None:
                g[k] = torch.from_numpy(m).to(DEV)
        groups.append(g)
    assert sum(p.batch for p in probs) == workloads.MIXED_COUNT
    ws = torch.empty(kron.kron_grouped_workspace_size(groups), dtype=torch.uint8, device=DEV)
    kron.kron_grouped_prepare(groups, ws)
    kron.kron_grouped_launch(ws)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for p, g in zip(probs, groups):
        e = p.n ** p.dim
        idx = np.unique(np.concatenate([[0, p.batch - 1], rng.integers(0, p.batch, 16)]))
        Y = g["Y"].cpu().numpy()
        mats = [m.astype(np.float64) for m in (p.A, p.B, p.C) if m is not None]
        for q in idx:
            want = (oracle.kron2d if p.dim == 2 else oracle.kron3d)(p.n, *mats, p.X[q * e:(q + 1) * e], 1, "f64")
            got = Y[q * e:(q + 1) * e]
            assert np.linalg.norm(got - want) <= 1e-5 * np.linalg.norm(want), (p.dim, p.n, q)
