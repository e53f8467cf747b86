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


@pytest.mark.parametrize("dims", [(2,), (3,)])
def test_grouped_one_phase_matches_single_group_kernels(dims):
    """Plans with only 2-D or only 3-D groups (the other phase empty), an
    unaligned group among them; every group's result equals, bit for bit,
    the single-group FP32 entry point on the same arrays (same tile code and
    stage order at the default launch shapes)."""
    import paper_1304_7054_amd as kron
    _need_gpu()
    spec = [(d, n, c) for d in dims for n, c in ((3, 700), (7, 333), (10, 250), (16, 97))]
    groups, host = _make_groups(spec, 21)
    # one unaligned group: X and Y start one element into their buffers
    g0 = groups[-1]
    xs = torch.empty(g0["X"].numel() + 1, device=DEV)
    xs[1:] = g0["X"]
    ys = torch.full((g0["Y"].numel() + 1,), float("nan"), device=DEV)
    g0["X"], g0["Y"] = xs[1:], ys[1:]
    ws = torch.empty(kron.kron_grouped_workspace_size(groups), dtype=torch.uint8, device=DEV)
    kron.kron_grouped_prepare(groups, ws)
    kron.kron_grouped_launch(ws)
    torch.cuda.synchronize()
    _check(groups, host)
    for g in groups:
        ref = torch.full_like(g["Y"], float("nan"))
        mats = [g[k] for k in "ABC"[:g["dim"]]]
        fn = kron.kron2d_batched_f32 if g["dim"] == 2 else kron.kron3d_batched_f32
        fn(g["n"], *mats, g["X"], ref, g["count"])
        torch.cuda.synchronize()
        assert torch.equal(ref, g["Y"]), (g["dim"], g["n"])


def test_grouped_counters_return_to_zero():
    """The chunk counters in the workspace are back at zero after every
    launch (the last wavefront resets them), so launches and graph replays
    start clean; repeated launches give the same bits."""
    import struct
    import paper_1304_7054_amd as kron
    _need_gpu()
    spec = [(2, 5, 3000), (2, 12, 800), (3, 4, 500), (3, 9, 300), (3, 16, 60)]
    groups, host = _make_groups(spec, 31)
    ws = torch.empty(kron.kron_grouped_workspace_size(groups), dtype=torch.uint8, device=DEV)
    kron.kron_grouped_prepare(groups, ws)
    first = None
    for rep in range(5):
        for g in groups:
            g["Y"].fill_(float("nan"))
        kron.kron_grouped_launch(ws)
        torch.cuda.synchronize()
        raw = ws.cpu().numpy().tobytes()
        for ph in range(2):
            counter_off = struct.unpack_from("<q", raw, 32 + 32 * ph + 24)[0]
            nxt, done = struct.unpack_from("<QI", raw, counter_off)
            assert (nxt, done) == (0, 0), (rep, ph, nxt, done)
        ys = [g["Y"].clone() for g in groups]
        if first is None:
            _check(groups, host)
            first = ys
        else:
            for a, b in zip(first, ys):
                assert torch.equal(a, b), rep


@pytest.mark.parametrize("spec", [
    [(2, 5, 3), (3, 16, 3000), (3, 10, 2000)],        # a tiny 2-D phase beside a large 3-D one
    [(2, 16, 60000), (2, 3, 20000), (3, 2, 7)],        # a tiny 3-D phase beside a large 2-D one
    [(2, 1, 1), (3, 1, 1)],                            # one operand per phase
])
def test_grouped_one_launch_skewed_phases(spec):
    """Both phases in one launch when one of them is tiny: every wavefront
    works through both chunk sequences (half start on each), the results
    match the oracle, every group equals the single-group entry point bit
    for bit, and repeated launches leave the counters at zero and give the
    same bits."""
    import struct
    import paper_1304_7054_amd as kron
    _need_gpu()
    groups, host = _make_groups(spec, 41)
    ws = torch.empty(kron.kron_grouped_workspace_size(groups), dtype=torch.uint8, device=DEV)
    kron.kron_grouped_prepare(groups, ws)
    first = None
    for rep in range(3):
        for g in groups:
            g["Y"].fill_(float("nan"))
        kron.kron_grouped_launch(ws)
        torch.cuda.synchronize()
        raw = ws.cpu().numpy().tobytes()
        for ph in range(2):
            counter_off = struct.unpack_from("<q", raw, 32 + 32 * ph + 24)[0]
            assert struct.unpack_from("<QI", raw, counter_off) == (0, 0), (rep, ph)
        ys = [g["Y"].clone() for g in groups]
        if first is None:
            _check(groups, host)
            first = ys
        else:
            for a, b in zip(first, ys):
                assert torch.equal(a, b), rep
    for g in groups:
        ref = torch.full_like(g["Y"], float("nan"))
        mats = [g[k] for k in "ABC"[:g["dim"]]]
        fn = kron.kron2d_batched_f32 if g["dim"] == 2 else kron.kron3d_batched_f32
        fn(g["n"], *mats, g["X"], ref, g["count"])
        torch.cuda.synchronize()
        assert torch.equal(ref, g["Y"]), (g["dim"], g["n"])
