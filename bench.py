"""Benchmark of the batched Kronecker-product action on one MI355X.

Headline workload: 3-D, n = 16, FP32, 65,536 arrays of 16^3 (1 GiB of X and
1 GiB of Y), A, B, C ~ U[-1, 1], X ~ N(0, 1), all resident in HBM before the
timed region.  One step is one launch of kron3d_batched_f32 over the whole
batch.  GFLOP/s uses the paper's flop model (Section 5): 6 n^4 per 3-D
operand, 4 n^3 per 2-D operand.

Printed: one JSON line with the headline value, the roofline of the dominant
kernel (algorithmic bytes = read X once + write Y once, over its average
launch time measured with HIP events on its stream), the same measurement
for the other precision modes and sizes, sampled parity against the FP64
oracle, and the CPU oracle timed on a bounded sample of the workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure
PAPER_K20C = {("f32", 3, 16): 268, ("f32", 2, 16): 285, ("f32", 3, 10): 126, ("f32", 2, 10): 143,
              ("f64", 3, 16): 169, ("f64", 2, 16): 152, ("f64", 3, 10): 103, ("f64", 2, 10): 108}
KERNEL_SOURCES = ["paper_1304_7054_amd/csrc/kron_tile.hpp", "paper_1304_7054_amd/csrc/kron_kernels.hpp",
                  "paper_1304_7054_amd/csrc/kron_launch.hpp", "paper_1304_7054_amd/csrc/kron_abi.hip"]


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--device-warm", type=float, default=0.5,
                   help="seconds of untimed launches before each measurement's warm-up steps (steady clocks)")
    p.add_argument("--only-headline", action="store_true", help="skip the other modes")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--summarize-profiles", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                   help="read rocprofv3 outputs of this script (kernel trace, FETCH_SIZE, WRITE_SIZE runs "
                        "with --copy-calibration) and write the summary and traffic record under profiles/")
    p.add_argument("--summarize-trace", metavar="TRACE_DIR",
                   help="read a rocprofv3 --kernel-trace --stats run of the whole benchmark and write the per-kernel "
                        "summary profiles/bench_kernels.md")
    p.add_argument("--copy-calibration", action="store_true",
                   help="first run three plain 1 GiB device copies (a kernel of known traffic for "
                        "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return p.parse_args()


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def flops_per_op(dim, n):
    return 4 * n ** 3 if dim == 2 else 6 * n ** 4


def make_inputs(torch, dim, n, batch, mode, seed):
    """Seeded synthetic inputs on the GPU: factors U[-1, 1] from the workload
    seed (numpy), operands N(0, 1) from a seeded device generator."""
    import workloads
    rng = workloads.rng_for(seed)
    mats = [workloads.uniform(rng, n * n, np.float64) for _ in range(dim)]
    gen = torch.Generator(device="cuda").manual_seed(workloads.SEED_BASE + seed)
    dt = {"f32": torch.float32, "bf16x3": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[mode]
    X = torch.randn(batch * n ** dim, generator=gen, device="cuda", dtype=torch.float32 if dt != torch.float64 else dt)
    X = X.to(dt)
    tm = [torch.from_numpy(m).to("cuda").to(dt) for m in mats]
    Y = torch.empty_like(X)
    return tm, X, Y


def fn_for(mode, dim):
    import paper_1304_7054_amd as kron
    return {
        ("f32", 2): kron.kron2d_batched_f32, ("f32", 3): kron.kron3d_batched_f32,
        ("f64", 2): kron.kron2d_batched_f64, ("f64", 3): kron.kron3d_batched_f64,
        ("bf16x3", 2): kron.kron2d_batched_f32_bf16x3, ("bf16x3", 3): kron.kron3d_batched_f32_bf16x3,
        ("bf16", 2): kron.kron2d_batched_bf16, ("bf16", 3): kron.kron3d_batched_bf16,
    }[(mode, dim)]


DEVICE_WARM_S = 0.5


def time_launches(torch, fn, args, steps, warmup):
    """Run `steps` launches bracketed by synchronisation; HIP events around
    every launch on the stream it is issued on.  Returns (wall ms/step,
    mean kernel ms, min kernel ms)."""
    stream = torch.cuda.current_stream()
    # bring the device to its steady clocks first (untimed), then the W warm-up steps
    t_end = time.perf_counter() + DEVICE_WARM_S
    while time.perf_counter() < t_end:
        for _ in range(20):
            fn(*args, stream=stream)
        torch.cuda.synchronize()
    for _ in range(warmup):
        fn(*args, stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn(*args, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    ks = [a.elapsed_time(b) for a, b in ev]
    return wall, float(np.mean(ks)), float(np.min(ks))


def sampled_error(torch, mode, dim, n, mats, X, Y, batch, samples=24, seed=0):
    """Normwise error of sampled operands against the FP64 oracle (computed
    operand by operand on the host from the same device values)."""
    import oracle
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([[0, batch - 1], rng.integers(0, batch, samples)]))
    e = n ** dim
    hm = [m.double().cpu().numpy() for m in mats]
    num = den = 0.0
    for p in idx:
        x = X[p * e:(p + 1) * e].double().cpu().numpy()
        y = Y[p * e:(p + 1) * e].double().cpu().numpy()
        want = oracle.kron2d(n, *hm, x, 1) if dim == 2 else oracle.kron3d(n, *hm, x, 1)
        num += float(np.sum((y - want) ** 2))
        den += float(np.sum(want ** 2))
    return float(np.sqrt(num / den))


def measure(torch, mode, dim, n, batch, steps, warmup, seed):
    mats, X, Y = make_inputs(torch, dim, n, batch, mode, seed)
    fn = fn_for(mode, dim)
    args = (n, *mats, X, Y, batch)
    wall, kmean, kmin = time_launches(torch, fn, args, steps, warmup)
    bytes_per = X.element_size() * n ** dim * 2
    alg_bytes = bytes_per * batch
    gflops = batch * flops_per_op(dim, n) / (kmean * 1e-3) / 1e9
    gbs = alg_bytes / (kmean * 1e-3) / 1e9
    err = sampled_error(torch, mode, dim, n, mats, X, Y, batch)
    out = {"mode": mode, "dim": dim, "n": n, "batch": batch, "ms": round(kmean, 4), "ms_min": round(kmin, 4),
           "wall_ms_per_step": round(wall, 4), "gflops": round(gflops, 1), "gbs": round(gbs, 1),
           "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes": alg_bytes, "sampled_rel_err": err}
    k20 = PAPER_K20C.get((mode, dim, n))
    if k20:
        out["paper_k20c_gflops"] = k20
    del mats, X, Y
    torch.cuda.empty_cache()
    return out


def measure_grouped(torch, steps, warmup):
    """The 500,000-operand mixed workload (n in 2..16, 70/30 2-D/3-D, one
    group per (dim, n)) in one persistent launch, replayed from a HIP graph."""
    import paper_1304_7054_amd as kron
    import workloads
    probs = workloads.workload4()
    groups, flops, alg = [], 0, 0
    for p in probs:
        g = {"dim": p.dim, "n": p.n, "count": p.batch, "X": torch.from_numpy(p.X).to("cuda"),
             "Y": torch.empty(p.X.size, device="cuda")}
        for k, m in zip("ABC", (p.A, p.B, p.C)):
            if m is not None:
                g[k] = torch.from_numpy(m).to("cuda")
        groups.append(g)
        flops += p.flops()
        alg += 2 * 4 * p.X.size
    ws = torch.empty(kron.kron_grouped_workspace_size(groups), dtype=torch.uint8, device="cuda")
    kron.kron_grouped_prepare(groups, ws)
    exe = kron.kron_graph_capture_grouped(ws)
    try:
        wall, kmean, kmin = time_launches(torch, lambda stream=None: kron.kron_graph_launch(exe, stream), (),
                                          steps, warmup)
        ewall, emean, emin = time_launches(torch, lambda stream=None: kron.kron_grouped_launch(ws, stream), (),
                                           steps, warmup)
    finally:
        kron.kron_graph_destroy(exe)
    torch.cuda.synchronize()
    # sampled parity of the graph replay
    import oracle
    rng = np.random.default_rng(7)
    worst = 0.0
    for p, g in zip(probs, groups):
        e = p.n ** p.dim
        Y = g["Y"]
        mats = [m.astype(np.float64) for m in (p.A, p.B, p.C) if m is not None]
        for q in rng.integers(0, p.batch, 4):
            want = (oracle.kron2d if p.dim == 2 else oracle.kron3d)(p.n, *mats, p.X[q * e:(q + 1) * e], 1, "f64")
            got = Y[q * e:(q + 1) * e].double().cpu().numpy()
            worst = max(worst, float(np.linalg.norm(got - want) / np.linalg.norm(want)))
    del groups, ws
    torch.cuda.empty_cache()
    return {"mode": "f32 grouped (graph replay)", "operands": workloads.MIXED_COUNT, "groups": len(probs),
            "ms": round(kmean, 4), "ms_min": round(kmin, 4), "eager_ms": round(emean, 4),
            "gflops": round(flops / (kmean * 1e-3) / 1e9, 1), "gbs": round(alg / (kmean * 1e-3) / 1e9, 1),
            "hbm_frac": round(alg / (kmean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes": alg,
            "sampled_max_rel_err": worst}


def measure_ex(torch, steps, warmup, beta=0.0):
    """Section 3's interface on the 3-D n=16 FP32 workload: alpha = -1.5 and
    op = (T, N, T) (per-call factor preparation included).  beta = 0 writes
    Y (2 GiB of traffic); beta != 0 also reads it (3 GiB)."""
    import paper_1304_7054_amd as kron
    import workloads
    n, batch = 16, workloads.BATCH_3D[16]
    mats, X, Y = make_inputs(torch, 3, n, batch, "f32", 5)
    Y.normal_()
    ws = torch.empty(kron.kron_ex_workspace_size(3, n, kron.MODE_F32), dtype=torch.uint8, device="cuda")
    # beta != 0: the timed calls update Y in place (|beta| < 1 keeps it
    # bounded); the parity sample is taken on one more call, from a saved
    # copy of the sampled arrays
    rng = np.random.default_rng(5)
    e = n ** 3
    idx = rng.integers(0, batch, 16)
    fn = lambda stream=None: kron.kron3d_batched_ex_f32(n, "T", "N", "T", -1.5, *mats, X, beta, Y, batch, ws, stream)
    wall, kmean, kmin = time_launches(torch, fn, (), max(10, steps // 2), warmup)
    torch.cuda.synchronize()
    import oracle
    hm = [m.double().cpu().numpy() for m in mats]
    y0 = {int(q): Y[q * e:(q + 1) * e].double().cpu().numpy() for q in idx}
    fn()
    torch.cuda.synchronize()
    num = den = 0.0
    for q in idx:
        q = int(q)
        x = X[q * e:(q + 1) * e].double().cpu().numpy()
        want = oracle.kron3d_ex(n, "T", "N", "T", -1.5, *hm, x, beta, y0[q], 1)
        got = Y[q * e:(q + 1) * e].double().cpu().numpy()
        num += float(np.sum((got - want) ** 2))
        den += float(np.sum(want ** 2))
    alg = (2 if beta == 0.0 else 3) * X.numel() * 4
    del mats, X, Y, ws
    torch.cuda.empty_cache()
    return {"mode": f"f32 extended 3-D n=16 (alpha=-1.5, ops T,N,T, beta={beta})", "batch": batch,
            "ms": round(kmean, 4), "ms_min": round(kmin, 4), "wall_ms_per_step": round(wall, 4),
            "gflops": round(batch * flops_per_op(3, n) / (kmean * 1e-3) / 1e9, 1),
            "gbs": round(alg / (kmean * 1e-3) / 1e9, 1),
            "hbm_frac": round(alg / (kmean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes": alg,
            "sampled_rel_err": float(np.sqrt(num / den))}


def measure_ex2d_transx(torch, steps, warmup):
    """2-D n=16 FP32 with op(X_p) = X_p^T (Section 2.2's 2-D interface):
    operands read transposed, beta = 0 (2 GiB of traffic)."""
    import paper_1304_7054_amd as kron
    import workloads
    n, batch = 16, workloads.BATCH_2D[16]
    mats, X, Y = make_inputs(torch, 2, n, batch, "f32", 6)
    ws = torch.empty(kron.kron_ex_workspace_size(2, n, kron.MODE_F32), dtype=torch.uint8, device="cuda")
    fn = lambda stream=None: kron.kron2d_batched_ex_f32(n, "N", "N", "T", 1.0, *mats, X, 0.0, Y, batch, ws, stream)
    wall, kmean, kmin = time_launches(torch, fn, (), max(10, steps // 2), warmup)
    torch.cuda.synchronize()
    import oracle
    rng = np.random.default_rng(6)
    hm = [m.double().cpu().numpy() for m in mats]
    e, num, den = n * n, 0.0, 0.0
    for q in rng.integers(0, batch, 16):
        x = X[q * e:(q + 1) * e].double().cpu().numpy()
        want = oracle.kron2d_ex(n, "N", "N", 1.0, *hm, x, 0.0, np.zeros(e), 1, opX="T")
        got = Y[q * e:(q + 1) * e].double().cpu().numpy()
        num += float(np.sum((got - want) ** 2))
        den += float(np.sum(want ** 2))
    alg = 2 * X.numel() * 4
    del mats, X, Y, ws
    torch.cuda.empty_cache()
    return {"mode": "f32 extended 2-D n=16 (op(X) = X^T, beta=0)", "batch": batch, "ms": round(kmean, 4),
            "ms_min": round(kmin, 4), "wall_ms_per_step": round(wall, 4),
            "gflops": round(batch * flops_per_op(2, n) / (kmean * 1e-3) / 1e9, 1),
            "gbs": round(alg / (kmean * 1e-3) / 1e9, 1),
            "hbm_frac": round(alg / (kmean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes": alg,
            "sampled_rel_err": float(np.sqrt(num / den))}


def measure_strided(torch, steps, warmup, ld=17):
    """3-D n=16 FP32 through the strided entry point on padded storage:
    columns of ld elements (ldx = ldy = ld, ldx2 = ld*16, ldxp = ld*256),
    beta = 0; ld = 17 takes the element-wise path, ld = 20 the 16-byte
    vectors.  Algorithmic bytes count the elements addressed (2 GiB)."""
    import paper_1304_7054_amd as kron
    import workloads
    n, batch = 16, workloads.BATCH_3D[16]
    ld2, ldp = ld * n, ld * n * n
    g = torch.Generator(device="cuda").manual_seed(workloads.SEED_BASE + 7)
    mats = [torch.rand(n * n, generator=g, device="cuda") * 2 - 1 for _ in range(3)]
    X = torch.randn(ldp * batch, generator=g, device="cuda")
    Y = torch.empty_like(X)
    ws = torch.empty(kron.kron_ex_workspace_size(3, n, kron.MODE_F32), dtype=torch.uint8, device="cuda")
    fn = lambda stream=None: kron.kron3d_batched_strided_f32(n, "N", "N", "N", 1.0, mats[0], n, mats[1], n, mats[2],
                                                             n, X, ld, ld2, ldp, 0.0, Y, ld, ld2, ldp, batch, ws,
                                                             stream)
    wall, kmean, kmin = time_launches(torch, fn, (), max(10, steps // 2), warmup)
    torch.cuda.synchronize()
    import oracle
    rng = np.random.default_rng(7)
    hm = [m.double().cpu().numpy() for m in mats]
    r = np.arange(n)
    sub = (r[None, None, :] + ld * r[None, :, None] + ld2 * r[:, None, None]).reshape(-1)
    num = den = 0.0
    for q in rng.integers(0, batch, 16):
        x = X[q * ldp:(q + 1) * ldp].double().cpu().numpy()[sub]
        want = oracle.kron3d(n, *hm, x, 1)
        got = Y[q * ldp:(q + 1) * ldp].double().cpu().numpy()[sub]
        num += float(np.sum((got - want) ** 2))
        den += float(np.sum(want ** 2))
    alg = 2 * batch * n ** 3 * 4
    del mats, X, Y, ws
    torch.cuda.empty_cache()
    return {"mode": f"f32 strided 3-D n=16 (ld {ld}, padded columns, beta=0)", "batch": batch, "ms": round(kmean, 4),
            "ms_min": round(kmin, 4), "wall_ms_per_step": round(wall, 4),
            "gflops": round(batch * flops_per_op(3, n) / (kmean * 1e-3) / 1e9, 1),
            "gbs": round(alg / (kmean * 1e-3) / 1e9, 1),
            "hbm_frac": round(alg / (kmean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes": alg,
            "sampled_rel_err": float(np.sqrt(num / den))}


def measure_strided2d(torch, steps, warmup, ld=17):
    """2-D n=16 FP32 through the strided entry point on padded storage:
    columns of ld elements (ldx = ldy = ld, ldxp = ld*16), beta = 0,
    262,144 arrays (1 GiB addressed in X and in Y)."""
    import paper_1304_7054_amd as kron
    import workloads
    n, batch = 16, workloads.BATCH_2D[16]
    ldp = ld * n
    g = torch.Generator(device="cuda").manual_seed(workloads.SEED_BASE + 9)
    mats = [torch.rand(n * n, generator=g, device="cuda") * 2 - 1 for _ in range(2)]
    X = torch.randn(ldp * batch, generator=g, device="cuda")
    Y = torch.empty_like(X)
    ws = torch.empty(kron.kron_ex_workspace_size(2, n, kron.MODE_F32), dtype=torch.uint8, device="cuda")
    fn = lambda stream=None: kron.kron2d_batched_strided_f32(n, "N", "N", "N", 1.0, mats[0], n, mats[1], n, X, ld,
                                                             ldp, 0.0, Y, ld, ldp, batch, ws, stream)
    wall, kmean, kmin = time_launches(torch, fn, (), max(10, steps // 2), warmup)
    torch.cuda.synchronize()
    import oracle
    rng = np.random.default_rng(9)
    hm = [m.double().cpu().numpy() for m in mats]
    r = np.arange(n)
    sub = (r[None, :] + ld * r[:, None]).reshape(-1)
    num = den = 0.0
    for q in rng.integers(0, batch, 16):
        x = X[q * ldp:(q + 1) * ldp].double().cpu().numpy()[sub]
        want = oracle.kron2d(n, *hm, x, 1)
        got = Y[q * ldp:(q + 1) * ldp].double().cpu().numpy()[sub]
        num += float(np.sum((got - want) ** 2))
        den += float(np.sum(want ** 2))
    alg = 2 * batch * n * n * 4
    del mats, X, Y, ws
    torch.cuda.empty_cache()
    return {"mode": f"f32 strided 2-D n=16 (ld {ld}, padded columns, beta=0)", "batch": batch, "ms": round(kmean, 4),
            "ms_min": round(kmin, 4), "wall_ms_per_step": round(wall, 4),
            "gflops": round(batch * flops_per_op(2, n) / (kmean * 1e-3) / 1e9, 1),
            "gbs": round(alg / (kmean * 1e-3) / 1e9, 1),
            "hbm_frac": round(alg / (kmean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes": alg,
            "sampled_rel_err": float(np.sqrt(num / den))}


def measure_tkron1(torch, steps, warmup):
    """TKRON1 (1-D), n = 16 FP32, 2^24 dense vectors (1 GiB X + 1 GiB Y),
    alpha = 1, op = N, beta = 0."""
    import paper_1304_7054_amd as kron
    import workloads
    n, batch = 16, 1 << 24
    g = torch.Generator(device="cuda").manual_seed(workloads.SEED_BASE + 8)
    A = torch.rand(n * n, generator=g, device="cuda") * 2 - 1
    X = torch.randn(batch * n, generator=g, device="cuda")
    Y = torch.empty_like(X)
    ws = torch.empty(kron.kron_ex_workspace_size(2, n, kron.MODE_F32), dtype=torch.uint8, device="cuda")
    fn = lambda stream=None: kron.kron1d_batched_f32(n, "N", 1.0, A, n, X, n, 0.0, Y, n, batch, ws, stream)
    wall, kmean, kmin = time_launches(torch, fn, (), max(10, steps // 2), warmup)
    torch.cuda.synchronize()
    Ad = A.double().cpu().numpy().reshape(n, n).T  # column-major
    rng = np.random.default_rng(8)
    idx = rng.integers(0, batch, 64)
    xs = torch.stack([X[q * n:(q + 1) * n] for q in idx]).double().cpu().numpy()
    ys = torch.stack([Y[q * n:(q + 1) * n] for q in idx]).double().cpu().numpy()
    import oracle
    want = oracle.kron1d_ex(n, "N", 1.0, A.double().cpu().numpy(), xs.reshape(-1), 0.0, np.zeros(xs.size), len(idx))
    err = float(np.linalg.norm(ys.reshape(-1) - want) / np.linalg.norm(want))
    alg = 2 * X.numel() * 4
    flops = 2 * n * n * batch
    del A, X, Y, ws
    torch.cuda.empty_cache()
    return {"mode": "f32 TKRON1 1-D n=16 (2^24 vectors)", "batch": batch, "ms": round(kmean, 4),
            "ms_min": round(kmin, 4), "wall_ms_per_step": round(wall, 4),
            "gflops": round(flops / (kmean * 1e-3) / 1e9, 1), "gbs": round(alg / (kmean * 1e-3) / 1e9, 1),
            "hbm_frac": round(alg / (kmean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes": alg,
            "sampled_rel_err": err}


def measure_backward(torch, steps, warmup):
    """dX + dA + dB + dC of the 3-D n=16 FP32 workload (reads X and dY,
    writes dX: three 1 GiB streams)."""
    import paper_1304_7054_amd as kron
    import workloads
    n, batch = 16, workloads.BATCH_3D[16]
    mats, X, _ = make_inputs(torch, 3, n, batch, "f32", 2)
    dY = torch.randn_like(X)
    dX = torch.empty_like(X)
    grads = [torch.empty(n * n, device="cuda") for _ in range(3)]
    ws = torch.empty(kron.kron_backward_workspace_size(3, n, batch, kron.MODE_F32), dtype=torch.uint8,
                     device="cuda")
    fn = lambda stream=None: kron.kron3d_backward_f32(n, *mats, X, dY, dX, *grads, batch, ws, stream)
    wall, kmean, kmin = time_launches(torch, fn, (), max(5, steps // 5), warmup)
    alg = 3 * X.numel() * 4
    del mats, X, dY, dX, grads, ws
    torch.cuda.empty_cache()
    return {"mode": "f32 backward 3-D n=16 (dX, dA, dB, dC)", "batch": batch, "ms": round(kmean, 4),
            "gbs": round(alg / (kmean * 1e-3) / 1e9, 1), "hbm_frac": round(alg / (kmean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "alg_bytes": alg}


def cpu_baseline(n=16, target_s=10.0):
    """The FP32 CPU oracle on a bounded sample of the headline workload."""
    import oracle
    import workloads
    orc = oracle.default()
    rng = workloads.rng_for(2)
    A, B, C = (workloads.uniform(rng, n * n, np.float32) for _ in range(3))
    probe = 256
    X = workloads.normal(rng, probe * n ** 3, np.float32)
    t = time.perf_counter()
    orc.kron3d(n, A, B, C, X, probe, "f32")
    dt = time.perf_counter() - t
    sample = int(min(workloads.BATCH_3D[16], max(probe, probe * target_s / max(dt, 1e-6))))
    X = workloads.normal(rng, sample * n ** 3, np.float32)
    orc.kron3d(n, A, B, C, X[: probe * n ** 3], probe, "f32")   # warm
    # whole passes over the sample until about target_s seconds have run (the
    # full workload alone takes well under a second on a many-core host)
    passes, t = 0, time.perf_counter()
    while True:
        orc.kron3d(n, A, B, C, X, sample, "f32")
        passes += 1
        dt = time.perf_counter() - t
        if dt >= target_s or passes >= 200:
            break
    return {"value": round(passes * sample * flops_per_op(3, n) / dt / 1e9, 2), "unit": "GFLOP/s",
            "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"FP32 oracle (plain C loops, OpenMP over operands) on {sample} of the 65536 "
                      f"3-D n=16 arrays, {passes} pass(es), {dt:.1f} s"}


def traffic_record(khash):
    """HBM bytes per dispatch of the headline kernel from rocprofv3 counters,
    if they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "kron3d_f32_n16_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != khash:
        return None
    return rec.get("bytes_per_dispatch")


# the FP32 n = 16 3-D kernels (which one runs depends on the launch variant)
HEADLINE_KERNELS = ("kron::kron3d_stream_kernel<kron::ModeF32,", "kron::kron3d_kernel<kron::ModeF32, 16,")
CALIBRATION_KERNEL = "__amd_rocclr_copyBuffer"


def headline_kernel_name():
    """The kernel the FP32 3-D n = 16 launch runs under the current launch table."""
    import paper_1304_7054_amd as kron
    _, v = kron.kron_get_launch(kron.MODE_F32, 3, 16)
    if v in (9, 10):
        return f"kron3d_stream_kernel<ModeF32, window {2 if v == 9 else 4}> (variant {v})"
    return f"kron3d_kernel<ModeF32, 16> (variant {v})"


def _is_headline(name):
    return any(k in name for k in HEADLINE_KERNELS)


def _csv(dirname, suffix):
    import csv
    import glob
    files = glob.glob(os.path.join(dirname, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {dirname}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def summarize_profiles(trace_dir, fetch_dir, write_dir):
    """Summary of the rocprofv3 runs of this script: the headline kernel's
    duration (kernel trace) and its HBM bytes per dispatch from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for the plain 1 GiB device copy the --copy-calibration option issues
    (1 GiB read, 1 GiB written)."""
    stats = _csv(trace_dir, "kernel_stats.csv")
    head = sorted((r for r in stats if _is_headline(r["Name"])), key=lambda r: -int(r["Calls"]))
    if not head:
        raise RuntimeError("headline kernel not in the trace")
    h = head[0]
    out = {"kernel": h["Name"], "calls": int(h["Calls"]), "avg_ns": float(h["AverageNs"]),
           "min_ns": float(h["MinNs"]), "max_ns": float(h["MaxNs"])}
    one_gib_kib = float(1 << 20)
    for tag, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = [r for r in _csv(d, "counter_collection.csv") if r["Counter_Name"] == counter]
        kern = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"] == h["Name"]]
        cal = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"] == CALIBRATION_KERNEL]
        # the calibration copies are the copyBuffer dispatches of 1 GiB: the largest ones
        cal = sorted(cal)[-3:]
        scale = one_gib_kib / (sum(cal) / len(cal))
        out[f"{tag}_kib_raw"] = sum(kern) / len(kern)
        out[f"{tag}_calibration_kib_raw"] = sum(cal) / len(cal)
        out[f"{tag}_scale"] = scale
        out[f"{tag}_bytes"] = out[f"{tag}_kib_raw"] * scale * 1024
    out["bytes_per_dispatch"] = out["fetch_bytes"] + out["write_bytes"]
    out["alg_bytes_per_dispatch"] = 2 * 65536 * 16 ** 3 * 4
    out["kernel_hash"] = kernel_hash()
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "kron3d_f32_n16_traffic.json"), "w") as f:
        json.dump(out, f, indent=1)
    with open(os.path.join(ROOT, "profiles", "kron3d_f32_n16.md"), "w") as f:
        f.write(_profile_markdown(out, stats))
    print(json.dumps(out, indent=1))
    return out


PROFILE_COMMANDS = """\
export TMPDIR=/tmp
rocprofv3 --kernel-trace --stats -d gpurun_out/prof_trace -o trace --output-format csv -- python bench.py --only-headline --no-cpu --copy-calibration --steps 20 --warmup 3
rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof_fetch -o fetch --output-format csv -- python bench.py --only-headline --no-cpu --copy-calibration --device-warm 0 --steps 3 --warmup 1
rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof_write -o write --output-format csv -- python bench.py --only-headline --no-cpu --copy-calibration --device-warm 0 --steps 3 --warmup 1
python bench.py --summarize-profiles gpurun_out/prof_trace gpurun_out/prof_fetch gpurun_out/prof_write
"""


TRACE_COMMAND = ("rocprofv3 --kernel-trace --stats -d gpurun_out/prof_all -o all --output-format csv -- "
                 "python bench.py --no-cpu --device-warm 0.2 --steps 20")


def summarize_trace(trace_dir):
    """Per-kernel durations of the library's kernels over a traced run of the
    whole benchmark (every mode, the grouped launch and the backward)."""
    stats = _csv(trace_dir, "kernel_stats.csv")
    rows = [r for r in stats if "kron" in r["Name"]]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [
        "# Kernel durations over the whole benchmark run",
        "",
        "Every `kron` kernel launched by `bench.py` (all modes, the grouped launch, the extended and strided",
        "interfaces, the backward), from one rocprofv3 kernel trace. The call counts include the untimed warm-up",
        "launches; averages are per dispatch under the profiler.",
        "",
        "```",
        "export TMPDIR=/tmp",
        TRACE_COMMAND,
        f"python bench.py --summarize-trace gpurun_out/prof_all",
        "```",
        "",
        "| kernel | calls | avg us | min us | max us |",
        "|---|---|---|---|---|",
    ]
    for r in rows:
        name = r["Name"].replace("void ", "")
        if ">(" in name:
            name = name[:name.index(">(") + 1]  # template kernel: drop the (possibly cut) parameter list
        elif name.endswith(")"):
            name = name[:name.rfind("(")]  # drop the parameter list
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} |")
    lines.append("")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "bench_kernels.md"), "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def _profile_markdown(out, stats):
    rows = sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:5]
    lines = [
        "# Headline kernel: 3-D Kronecker action, FP32, n = 16, 65,536 arrays (1 GiB X + 1 GiB Y)",
        "",
        f"Kernel: `{out['kernel']}`",
        "",
        "## Commands (repository root, on the MI355X)",
        "",
        "```",
        PROFILE_COMMANDS.rstrip(),
        "```",
        "",
        "## Kernel trace (`--stats`), top kernels of the traced run",
        "",
        "| kernel | calls | avg us | min us | max us | % |",
        "|---|---|---|---|---|---|",
    ]
    for r in rows:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    lines += [
        "",
        f"The headline kernel's {out['calls']} calls include the untimed device warm-up launches (0.5 s), "
        "3 warm-up steps and 20 timed steps; bench.py's own HIP-event average in the same run is the "
        "`kernel_ms` of its JSON line.",
        "",
        "## HBM traffic per dispatch (`--pmc`, one counter per run)",
        "",
        "FETCH_SIZE and WRITE_SIZE are KiB per dispatch.  The calibration kernel is the plain 1 GiB "
        "device-to-device copy (`__amd_rocclr_copyBuffer`, issued by `--copy-calibration`: 1 GiB read, "
        "1 GiB written); each counter is scaled by (1 GiB / its reading for that copy).",
        "",
        "| counter | headline kernel (raw KiB) | 1 GiB copy (raw KiB) | scale | headline bytes |",
        "|---|---|---|---|---|",
        f"| FETCH_SIZE | {out['fetch_kib_raw']:.0f} | {out['fetch_calibration_kib_raw']:.0f} | "
        f"{out['fetch_scale']:.4f} | {out['fetch_bytes']:.0f} |",
        f"| WRITE_SIZE | {out['write_kib_raw']:.0f} | {out['write_calibration_kib_raw']:.0f} | "
        f"{out['write_scale']:.4f} | {out['write_bytes']:.0f} |",
        "",
        f"Total {out['bytes_per_dispatch']:.0f} bytes per dispatch vs {out['alg_bytes_per_dispatch']} "
        f"algorithmic (X read once, Y written once): ratio "
        f"{out['bytes_per_dispatch'] / out['alg_bytes_per_dispatch']:.5f}.",
        "",
        f"Kernel sources hash (bench.py `kernel_hash`): `{out['kernel_hash']}`; bench.py reports "
        "`roofline.traffic` only while the sources hash to this value.",
        "",
    ]
    return "\n".join(lines)


def main():
    args = parse()
    global DEVICE_WARM_S
    DEVICE_WARM_S = max(0.0, args.device_warm)
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the batch splits into independent per-GPU shards with no communication)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    import paper_1304_7054_amd as kron
    kron.lib()  # fail loudly if the HIP library is missing
    import workloads

    if args.copy_calibration:
        src = torch.ones(1 << 28, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    head = measure(torch, "f32", 3, 16, workloads.BATCH_3D[16], args.steps, args.warmup, seed=2)
    others = []
    if not args.only_headline:
        plan = [("bf16x3", 3, 16, workloads.BATCH_3D[16], 3),
                ("bf16", 3, 16, workloads.BATCH_3D[16], 3),
                ("f32", 2, 16, workloads.BATCH_2D[16], 1),
                ("f32", 2, 10, workloads.BATCH_2D[10], 1),
                ("f32", 3, 10, workloads.BATCH_3D[10], 2),
                ("f64", 3, 16, workloads.BATCH_3D[16] // 2, 2),
                ("f64", 2, 16, workloads.BATCH_2D[16] // 2, 1),
                ("bf16x3", 2, 16, workloads.BATCH_2D[16], 3)]
        for mode, dim, n, batch, seed in plan:
            others.append(measure(torch, mode, dim, n, batch, max(10, args.steps // 2), args.warmup, seed))
            print(f"# measured {mode} {dim}-D n={n}: {others[-1]['gflops']} GFLOP/s", file=sys.stderr, flush=True)
        others.append(measure_grouped(torch, max(10, args.steps // 2), args.warmup))
        print(f"# measured grouped mixed: {others[-1]['gflops']} GFLOP/s", file=sys.stderr, flush=True)
        for beta in (0.0, 0.5):
            others.append(measure_ex(torch, args.steps, args.warmup, beta))
            print(f"# measured extended interface, beta={beta}: {others[-1]['gflops']} GFLOP/s", file=sys.stderr,
                  flush=True)
        others.append(measure_ex2d_transx(torch, args.steps, args.warmup))
        print(f"# measured extended interface 2-D op(X)=T: {others[-1]['gflops']} GFLOP/s", file=sys.stderr,
              flush=True)
        for ld in (17, 20):
            others.append(measure_strided(torch, args.steps, args.warmup, ld))
            print(f"# measured strided 3-D ld {ld}: {others[-1]['gflops']} GFLOP/s", file=sys.stderr, flush=True)
        others.append(measure_strided2d(torch, args.steps, args.warmup))
        print(f"# measured strided 2-D: {others[-1]['gflops']} GFLOP/s", file=sys.stderr, flush=True)
        others.append(measure_tkron1(torch, args.steps, args.warmup))
        print(f"# measured TKRON1: {others[-1]['gflops']} GFLOP/s", file=sys.stderr, flush=True)
        others.append(measure_backward(torch, args.steps, args.warmup))
        print(f"# measured backward: {others[-1]['ms']} ms", file=sys.stderr, flush=True)

    khash = kernel_hash()
    roof = {"bound": "hbm", "achieved": head["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(head["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic_record(khash),
            "kernel": headline_kernel_name(), "alg_bytes_per_launch": head["alg_bytes"],
            "kernel_ms": head["ms"]}
    line = {
        "metric": "Kron-action GFLOP/s + % HBM roofline, 3-D n=16 FP32: plain vs bf16x3 MFMA",
        "value": head["gflops"], "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["wall_ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3-D Kronecker action n=16 FP32, 65536 arrays 16^3 (1 GiB X + 1 GiB Y)",
                   "dim": 3, "n": 16, "batch": head["batch"]},
        "roofline": roof,
        "headline": head,
        "bf16x3": next((o for o in others if o.get("mode") == "bf16x3" and o.get("dim") == 3), None),
        "modes": others,
        "kernel_hash": khash,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
