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
# every library source and header: the counter-derived traffic of the
# headline kernel is reported only for the code and flags it was taken on
KERNEL_SOURCE_DIRS = ["paper_1304_7054_amd/csrc"]
KERNEL_HEADERS = ["include/kron.h", "paper_1304_7054_amd/tuning/gfx950.json"]


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--device-warm", type=float, default=0.5,
                   help="seconds of untimed launches before each measurement's warm-up steps (steady clocks)")
    p.add_argument("--only-headline", action="store_true", help="skip the other modes")
    p.add_argument("--only", default="", help="comma-separated names of the measurements to run after the "
                   "headline (see measurement_plan), e.g. grouped,grouped-backward")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--tune-headline", action="store_true",
                   help="autotune the headline's launch shape on this device first (default: the shipped table)")
    p.add_argument("--summarize-profiles", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                   help="read rocprofv3 outputs of this script (kernel trace, FETCH_SIZE, WRITE_SIZE runs "
                        "with --copy-calibration) and write the summary and traffic record under profiles/")
    p.add_argument("--summarize-trace", metavar="TRACE_DIR",
                   help="read a rocprofv3 --kernel-trace --stats run of the whole benchmark and write the per-kernel "
                        "summary profiles/bench_kernels.md")
    p.add_argument("--summarize-counters", nargs="+", metavar="ARG",
                   help="OUT_NAME TITLE COMMAND_FILE DIR [DIR ...]: per-kernel counter averages of rocprofv3 --pmc "
                        "runs, written to profiles/OUT_NAME.md with the commands listed in COMMAND_FILE")
    p.add_argument("--copy-calibration", action="store_true",
                   help="first run three plain 1 GiB device copies (a kernel of known traffic for "
                        "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return p.parse_args()


def kernel_sources():
    files = []
    for d in KERNEL_SOURCE_DIRS:
        files += sorted(os.path.join(d, f) for f in os.listdir(os.path.join(ROOT, d))
                        if f.endswith((".hip", ".hpp", ".h")))
    return files + KERNEL_HEADERS


def kernel_hash():
    """Hash of every library source and the device compile flags (include
    paths left out: they name the checkout's location)."""
    from paper_1304_7054_amd import build as kbuild
    h = hashlib.sha256()
    for f in kernel_sources():
        h.update(f.encode())
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(a for a in kbuild.COMMON if not a.startswith("-I")).encode())
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


LAST_TIMING = {}


def time_launches(torch, fn, args, steps, warmup):
    """Run `steps` launches bracketed by synchronisation; HIP events around
    every launch on the stream it is issued on.  Returns (wall ms/step,
    mean kernel ms, min kernel ms); the median is kept in LAST_TIMING.  The
    Python garbage collector is held off during the timed launches: a
    collection pause that outlasts the queued work would otherwise land
    inside an event interval as idle device time."""
    import gc
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
    gc_was = gc.isenabled()
    gc.disable()
    try:
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            fn(*args, stream=stream)
            b.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
    finally:
        if gc_was:
            gc.enable()
    ks = [a.elapsed_time(b) for a, b in ev]
    LAST_TIMING.update({"median_ms": float(np.median(ks)), "max_ms": float(np.max(ks))})
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
           "ms_median": round(LAST_TIMING["median_ms"], 4), "ms_max": round(LAST_TIMING["max_ms"], 4),
           "wall_ms_per_step": round(wall, 4), "gflops": round(gflops, 1), "gbs": round(gbs, 1),
           "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes": alg_bytes, "sampled_rel_err": err}
    k20 = PAPER_K20C.get((mode, dim, n))
    if k20:
        out["paper_k20c_gflops"] = k20
    del mats, X, Y
    torch.cuda.empty_cache()
    return out


def measure_copy(torch, steps, warmup):
    """Plain 1 GiB device-to-device copies (1 GiB read + 1 GiB written) timed
    like the kernels: the library's streaming copy (kron_copy_bytes, the same
    16-byte non-temporal accesses as its kernels; the reference of
    frac_of_copy) and torch's copy_ for context."""
    import paper_1304_7054_amd as kron
    src = torch.ones(1 << 28, device="cuda")
    dst = torch.empty_like(src)
    out = {"bytes": 2 * (1 << 30)}
    for tag, fn in (("stream_copy", lambda stream=None: kron.kron_copy_bytes(src, dst, stream)),
                    ("torch_copy", lambda stream=None: dst.copy_(src))):
        wall, kmean, kmin = time_launches(torch, fn, (), steps, warmup)
        gbs = 2 * (1 << 30) / (kmean * 1e-3) / 1e9
        out[tag] = {"ms": round(kmean, 4), "gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    assert bool(torch.equal(src, dst))
    out["gbs"] = out["stream_copy"]["gbs"]
    del src, dst
    torch.cuda.empty_cache()
    return out


def batch_errors(mode, n, mats_exact, X_dev, Y_dev, batch, chunk=4096):
    """Normwise relative error over the whole batch (and the largest
    per-array one) of a 3-D result against the FP64 oracle applied to
    `mats_exact` and the device operands, computed on the host in chunks.
    bf16 storage: X_dev holds the bf16 operands; the oracle sees their
    exact values."""
    import oracle
    e = n ** 3
    num = den = 0.0
    worst = 0.0
    for s0 in range(0, batch, chunk):
        b = min(chunk, batch - s0)
        x = X_dev[s0 * e:(s0 + b) * e].double().cpu().numpy()
        y = Y_dev[s0 * e:(s0 + b) * e].double().cpu().numpy()
        want = oracle.kron3d(n, *mats_exact, x, b, "f64")
        d = (y - want).reshape(b, e)
        w = want.reshape(b, e)
        dn = np.einsum("ij,ij->i", d, d)
        wn = np.einsum("ij,ij->i", w, w)
        num += float(dn.sum())
        den += float(wn.sum())
        worst = max(worst, float(np.sqrt((dn / np.maximum(wn, 1e-300)).max())))
    return float(np.sqrt(num / den)), worst


def measure_precision(torch, steps, warmup):
    """The precision workload: 3-D n = 16, 65,536 arrays, every entry of A, B,
    C and X log-uniform in magnitude on [1e-3, 1e3] with a random sign
    (factors drawn on the host, operands with a seeded device generator).
    Plain FP32, bf16x3 (FP32 I/O) and bf16 storage are timed on the same
    values, and each result is compared with the FP64 oracle over the whole
    batch.  bf16 storage rounds its inputs to bf16 (nearest even): its error
    is given against the oracle on the original FP32 values (the figure of
    merit) and on the rounded inputs (arithmetic and output rounding only)."""
    import workloads
    n, batch = 16, workloads.BATCH_3D[16]
    rng = workloads.rng_for(3)
    mats32 = [workloads.log_uniform(rng, n * n, np.float32) for _ in range(3)]
    gen = torch.Generator(device="cuda").manual_seed(workloads.SEED_BASE + 3)
    X = workloads.log_uniform_device_(torch.empty(batch * n ** 3, device="cuda"), gen)
    Y = torch.empty_like(X)
    tm = [torch.from_numpy(m).to("cuda") for m in mats32]
    exact32 = [m.astype(np.float64) for m in mats32]
    out = []
    for mode in ("f32", "bf16x3", "bf16"):
        if mode == "bf16":
            tmb = [t.to(torch.bfloat16) for t in tm]
            Xb = X.to(torch.bfloat16)
            Yb = torch.empty_like(Xb)
            args = (n, *tmb, Xb, Yb, batch)
        else:
            args = (n, *tm, X, Y, batch)
        wall, kmean, kmin = time_launches(torch, fn_for(mode, 3), args, steps, warmup)
        bytes_per = (2 if mode == "bf16" else 4) * n ** 3 * 2
        gbs = bytes_per * batch / (kmean * 1e-3) / 1e9
        rec = {"mode": mode, "dim": 3, "n": n, "batch": batch,
               "data": "log-uniform magnitudes in [1e-3, 1e3], random signs (A, B, C and X)",
               "ms": round(kmean, 4), "ms_min": round(kmin, 4), "ms_median": round(LAST_TIMING["median_ms"], 4),
               "ms_max": round(LAST_TIMING["max_ms"], 4), "wall_ms_per_step": round(wall, 4),
               "gflops": round(batch * flops_per_op(3, n) / (kmean * 1e-3) / 1e9, 1), "gbs": round(gbs, 1),
               "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes": bytes_per * batch}
        if mode == "bf16":
            # (i) against the original FP32 values; (ii) against the rounded inputs
            norm, worst = batch_errors(mode, n, exact32, X, Yb, batch)
            rounded = [t.double().cpu().numpy() for t in tmb]
            norm2, worst2 = batch_errors(mode, n, rounded, Xb, Yb, batch)
            rec.update({"rel_err_vs_fp32_inputs": norm, "max_array_rel_err_vs_fp32_inputs": worst,
                        "rel_err_vs_bf16_inputs": norm2, "max_array_rel_err_vs_bf16_inputs": worst2})
            del tmb, Xb, Yb
        else:
            norm, worst = batch_errors(mode, n, exact32, X, Y, batch)
            rec.update({"rel_err": norm, "max_array_rel_err": worst})
        rec["error_scope"] = "whole batch, normwise (Frobenius) against the FP64 oracle"
        out.append(rec)
        print(f"# measured precision workload {mode}: {rec['gflops']} GFLOP/s", file=sys.stderr, flush=True)
    del X, Y, tm
    torch.cuda.empty_cache()
    return out


_MIXED = None


def mixed_workload():
    """The 500,000-operand mixed workload (drawn once per run)."""
    global _MIXED
    if _MIXED is None:
        import workloads
        _MIXED = workloads.workload4()
    return _MIXED


def measure_grouped(torch, steps, warmup):
    """The 500,000-operand mixed workload (n in 2..16, 70/30 2-D/3-D, one
    group per (dim, n)) in one persistent launch, replayed from a HIP graph."""
    import paper_1304_7054_amd as kron
    import workloads
    probs = mixed_workload()
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


def measure_grouped_backward(torch, steps, warmup):
    """Backward over the 500,000-operand mixed workload: every group's dX and
    its batch-reduced dA, dB (, dC) from upstream gradients dY ~ N(0, 1), in
    one kron_grouped_backward call (reads X and dY, writes dX: three streams
    of the workload's operand bytes; the factor gradients are negligible)."""
    import paper_1304_7054_amd as kron
    import workloads
    probs = mixed_workload()
    groups, alg, flops = [], 0, 0
    for p in probs:
        g = {"dim": p.dim, "n": p.n, "count": p.batch, "X": torch.from_numpy(p.X).to("cuda"),
             "dY": torch.from_numpy(p.dY).to("cuda")}
        g["dX"] = torch.empty_like(g["X"])
        for k, m in zip("ABC", (p.A, p.B, p.C)):
            if m is not None:
                g[k] = torch.from_numpy(m).to("cuda")
                g["d" + k] = torch.empty(p.n * p.n, device="cuda")
        groups.append(g)
        alg += 3 * 4 * p.X.size
        flops += p.flops()
    ws = torch.empty(kron.kron_grouped_backward_workspace_size(groups), dtype=torch.uint8, device="cuda")
    wall, kmean, kmin = time_launches(torch, lambda stream=None: kron.kron_grouped_backward(groups, ws, stream), (),
                                      steps, warmup)
    torch.cuda.synchronize()
    # sampled parity: the factor gradients of the two largest-n groups against the FP64 oracle
    import oracle
    worst = 0.0
    for p, g in [(p, g) for p, g in zip(probs, groups) if p.n == 16]:
        mats = [m.astype(np.float64) for m in (p.A, p.B, p.C) if m is not None]
        grad = oracle.kron2d_grad if p.dim == 2 else oracle.kron3d_grad
        want = grad(p.n, *mats, p.X.astype(np.float64), p.dY.astype(np.float64), p.batch)
        for k, w in zip("ABC", want[1:]):
            got = g["d" + k].double().cpu().numpy()
            worst = max(worst, float(np.linalg.norm(got - w) / np.linalg.norm(w)))
    del groups, ws
    torch.cuda.empty_cache()
    return {"mode": "f32 grouped backward (500,000 mixed operands: dX, dA, dB, dC per group)",
            "operands": workloads.MIXED_COUNT, "groups": len(probs), "ms": round(kmean, 4), "ms_min": round(kmin, 4),
            "wall_ms_per_step": round(wall, 4), "gbs": round(alg / (kmean * 1e-3) / 1e9, 1),
            "hbm_frac": round(alg / (kmean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes": alg,
            "forward_gflop": round(flops / 1e9, 3), "factor_grad_rel_err_n16": worst}


def _nd_workload(torch, case):
    """The general-action workloads (1 GiB of operands each), drawn on the
    device from a seeded generator: (tag, m, n, ops, factors, ldfp, X, batch,
    flops per operand, passes)."""
    import workloads
    g = torch.Generator(device="cuda").manual_seed(workloads.SEED_BASE + 11)
    if case == "f32 4-D n=16":
        tag, dims, batch, varying = "f32", [16] * 4, 4096, False
    elif case == "c32 3-D n=16":
        tag, dims, batch, varying = "c32", [16] * 3, 32768, False
    elif case == "f32 2-D n=32":
        tag, dims, batch, varying = "f32", [32] * 2, 262144, False
    elif case == "f32 3-D varying n=16":
        tag, dims, batch, varying = "f32", [16] * 3, 65536, True
    else:
        raise KeyError(case)
    dt = {"f32": torch.float32, "c32": torch.complex64}[tag]
    d, n = len(dims), dims[0]
    count = batch if varying else 1
    fac = [(torch.rand(count * n * n, generator=g, device="cuda", dtype=torch.float64) * 2 - 1).to(dt)
           for _ in range(d)]
    if tag == "c32":
        fac = [f + 1j * (torch.rand(f.numel(), generator=g, device="cuda") * 2 - 1) for f in fac]
    X = torch.randn(batch * n ** d, generator=g, device="cuda", dtype=dt)
    ops = "NTNC"[:d] if tag == "c32" else "NTNT"[:d]
    # paper's flop model per real contraction (2 n^(d+1) per mode), x4 for complex arithmetic
    flops = d * 2 * n ** (d + 1) * (4 if tag == "c32" else 1)
    return tag, dims, dims, ops, fac, [n * n if varying else 0] * d, X, batch, flops, d


def measure_nd(torch, case, steps=10, warmup=2, check_only=False):
    """One general-action workload through kron_nd_batched_*: timed like the
    other modes, sampled operands against the oracle."""
    import paper_1304_7054_amd as kron
    import oracle
    tag, m, n, ops, fac, ldfp, X, batch, flops, passes = _nd_workload(torch, case)
    Y = torch.empty(batch * int(np.prod(m)), device="cuda", dtype=X.dtype)
    code = {"f32": kron.MODE_F32, "c32": kron.KRON_TYPE_C32}[tag]
    ws = torch.empty(max(1, kron.kron_nd_workspace_size(m, n, batch, code)), dtype=torch.uint8, device="cuda")
    fn = getattr(kron, f"kron_nd_batched_{tag}")
    call = lambda stream=None: fn(m, n, ops, 1.0, fac, X, 0.0, Y, batch, ldfp=ldfp, ws=ws, stream=stream)
    if check_only:
        call()
        kmean = kmin = wall = float("nan")
    else:
        wall, kmean, kmin = time_launches(torch, call, (), steps, warmup)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    nx, ny = int(np.prod(n)), int(np.prod(m))
    num = den = 0.0
    for q in np.unique(np.concatenate([[0, batch - 1], rng.integers(0, batch, 4)])):
        q = int(q)
        hx = X[q * nx:(q + 1) * nx].cpu().numpy()
        hf = [(f[q * s:q * s + nn * nn] if s else f).cpu().numpy() for f, s, nn in zip(fac, ldfp, n)]
        want = oracle.kron_nd(m, n, ops, 1.0, hf, hx, 0.0, np.zeros(ny), 1)
        got = Y[q * ny:(q + 1) * ny].cpu().numpy()
        num += float(np.sum(np.abs(got - want) ** 2))
        den += float(np.sum(np.abs(want) ** 2))
    finite = bool(torch.isfinite(torch.view_as_real(Y) if Y.is_complex() else Y).all())
    esz = X.element_size()
    alg = (nx + ny) * batch * esz + (sum(int(f.numel()) for f in fac) * esz if any(ldfp) else 0)
    out = {"mode": f"general action: {case}", "tag": tag, "batch": batch, "passes": passes,
           "sampled_rel_err": float(np.sqrt(num / den)) if finite else float("inf")}
    if not check_only:
        gbs = alg / (kmean * 1e-3) / 1e9
        out.update({"ms": round(kmean, 4), "ms_min": round(kmin, 4), "wall_ms_per_step": round(wall, 4),
                    "gflops": round(batch * flops / (kmean * 1e-3) / 1e9, 1), "gbs": round(gbs, 1),
                    "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes": alg,
                    "pass_bytes": passes * (nx + ny) * batch * esz,
                    "pass_traffic_frac": round(passes * (nx + ny) * batch * esz / (kmean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    del fac, X, Y, ws
    torch.cuda.empty_cache()
    return out


ND_CASES = {c: (lambda torch, check_only=False, c=c: measure_nd(torch, c, check_only=check_only))
            for c in ("f32 4-D n=16", "c32 3-D n=16", "f32 2-D n=32", "f32 3-D varying n=16")}


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


def measure_strided(torch, steps, warmup, ld=17, ldy=None):
    """3-D n=16 FP32 through the strided entry point on padded storage:
    columns of ld elements in X (ldx = ld, ldx2 = ld*16, ldxp = ld*256) and
    of ldy (default ld) in Y, beta = 0.  ld = 17 takes the element-wise
    path; strides that are multiples of 4 take the 16-byte vectors.  The
    cases with only X or only Y padded show which side limits the rate.
    Algorithmic bytes count the elements addressed (2 GiB)."""
    import paper_1304_7054_amd as kron
    import workloads
    ldy = ld if ldy is None else ldy
    n, batch = 16, workloads.BATCH_3D[16]
    ld2, ldp = ld * n, ld * n * n
    ldy2, ldyp = ldy * n, ldy * n * n
    g = torch.Generator(device="cuda").manual_seed(workloads.SEED_BASE + 7)
    mats = [torch.rand(n * n, generator=g, device="cuda") * 2 - 1 for _ in range(3)]
    X = torch.randn(ldp * batch, generator=g, device="cuda")
    Y = torch.empty(ldyp * batch, device="cuda")
    ws = torch.empty(kron.kron_ex_workspace_size(3, n, kron.MODE_F32), dtype=torch.uint8, device="cuda")
    fn = lambda stream=None: kron.kron3d_batched_strided_f32(n, "N", "N", "N", 1.0, mats[0], n, mats[1], n, mats[2],
                                                             n, X, ld, ld2, ldp, 0.0, Y, ldy, ldy2, ldyp, batch, ws,
                                                             stream)
    wall, kmean, kmin = time_launches(torch, fn, (), max(10, steps // 2), warmup)
    torch.cuda.synchronize()
    import oracle
    rng = np.random.default_rng(7)
    hm = [m.double().cpu().numpy() for m in mats]
    r = np.arange(n)
    sub = (r[None, None, :] + ld * r[None, :, None] + ld2 * r[:, None, None]).reshape(-1)
    suby = (r[None, None, :] + ldy * r[None, :, None] + ldy2 * r[:, None, None]).reshape(-1)
    num = den = 0.0
    for q in rng.integers(0, batch, 16):
        x = X[q * ldp:(q + 1) * ldp].double().cpu().numpy()[sub]
        want = oracle.kron3d(n, *hm, x, 1)
        got = Y[q * ldyp:(q + 1) * ldyp].double().cpu().numpy()[suby]
        num += float(np.sum((got - want) ** 2))
        den += float(np.sum(want ** 2))
    alg = 2 * batch * n ** 3 * 4
    del mats, X, Y, ws
    torch.cuda.empty_cache()
    lds = f"ld {ld}" if ldy == ld else f"ldx {ld}, ldy {ldy}"
    return {"mode": f"f32 strided 3-D n=16 ({lds}, padded columns, beta=0)", "batch": batch, "ms": round(kmean, 4),
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_rate(orc, call, flops, target_s, max_passes=200):
    """Whole passes of `call` until about target_s seconds have run (after
    one warm pass); returns (GFLOP/s, passes, seconds)."""
    call()
    passes, t = 0, time.perf_counter()
    while True:
        call()
        passes += 1
        dt = time.perf_counter() - t
        if dt >= target_s or passes >= max_passes:
            return passes * flops / dt / 1e9, passes, dt


def cpu_baseline(n=16, target_s=10.0):
    """The CPU oracle on a bounded sample of the headline workload: FP32 (the
    reported value) and FP64 on every host core, and the small 2-D n = 4
    workload (4096 operands) on one core."""
    import oracle
    import workloads
    orc = oracle.default()
    cores = orc.num_threads()
    rng = workloads.rng_for(2)
    A, B, C = (workloads.uniform(rng, n * n, np.float32) for _ in range(3))
    probe = 256
    X = workloads.normal(rng, probe * n ** 3, np.float32)
    t = time.perf_counter()
    orc.kron3d(n, A, B, C, X, probe, "f32")
    dt = time.perf_counter() - t
    sample = int(min(workloads.BATCH_3D[16], max(probe, probe * target_s / max(dt, 1e-6))))
    X = workloads.normal(rng, sample * n ** 3, np.float32)
    f3 = sample * flops_per_op(3, n)
    # the full workload alone takes well under a second on a many-core host
    r32, p32, t32 = _oracle_rate(orc, lambda: orc.kron3d(n, A, B, C, X, sample, "f32"), f3, target_s)
    X64 = X.astype(np.float64)
    A64, B64, C64 = (m.astype(np.float64) for m in (A, B, C))
    r64, p64, t64 = _oracle_rate(orc, lambda: orc.kron3d(n, A64, B64, C64, X64, sample, "f64"), f3, target_s / 2)
    del X, X64
    w0 = workloads.workload0(np.float32)
    f0 = w0.flops()
    one = {}
    orc.set_num_threads(1)
    try:
        for prec in ("f32", "f64"):
            dt_ = np.float32 if prec == "f32" else np.float64
            a0, b0, x0 = (np.asarray(v, dt_) for v in (w0.A, w0.B, w0.X))
            r, p, t = _oracle_rate(orc, lambda: orc.kron2d(w0.n, a0, b0, x0, w0.batch, prec), f0, 1.0, 10000)
            one[prec] = round(r, 3)
    finally:
        orc.set_num_threads(cores)
    return {"value": round(r32, 2), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"FP32 oracle (plain C loops, OpenMP over operands) on {sample} of the 65536 "
                      f"3-D n=16 arrays, {p32} pass(es), {t32:.1f} s",
            "f64": {"value": round(r64, 2), "unit": "GFLOP/s", "cores": cores,
                    "sample": f"same arrays in FP64, {p64} pass(es), {t64:.1f} s"},
            "one_core_2d_n4": {"unit": "GFLOP/s", "cores": 1, "f32": one["f32"], "f64": one["f64"],
                               "sample": "2-D n=4, 4096 operands U[-1,1], whole passes for about 1 s each"}}


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


def tune_headline(torch):
    """Autotune the headline's launch shape on this device (kron_autotune:
    every variant x workgroups-per-CU, three sweeps, lowest mean) on the
    headline workload's own buffers, before anything is timed.  Returns the
    choice."""
    import paper_1304_7054_amd as kron
    import workloads
    n, batch = 16, workloads.BATCH_3D[16]
    mats, X, Y = make_inputs(torch, 3, n, batch, "f32", 2)
    t = time.perf_counter()
    b, v, ms = kron.kron_autotune(kron.MODE_F32, 3, n, *mats, X, Y, batch, reps=10)
    out = {"variant": v, "blocks_per_cu": b, "tune_ms": round(ms, 4), "tune_s": round(time.perf_counter() - t, 1)}
    del mats, X, Y
    torch.cuda.empty_cache()
    print(f"# headline launch shape tuned on this device: {out}", file=sys.stderr, flush=True)
    return out


def launch_shape_record():
    """The launch shape the headline ran with and the autotuned table it came from."""
    import paper_1304_7054_amd as kron
    from paper_1304_7054_amd import _binding
    blocks, variant = kron.kron_get_launch(kron.MODE_F32, 3, 16)
    return {"variant": variant, "blocks_per_cu": blocks, "table": _binding.APPLIED_TABLE["path"],
            "table_entries": _binding.APPLIED_TABLE["entries"]}


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
rocprofv3 --kernel-trace --stats -d gpurun_out/prof_headline_trace -o trace --output-format csv -- python bench.py --only-headline --no-cpu --copy-calibration --steps 20 --warmup 3
rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof_headline_fetch -o fetch --output-format csv -- python bench.py --only-headline --no-cpu --copy-calibration --device-warm 0 --steps 3 --warmup 1
rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof_headline_write -o write --output-format csv -- python bench.py --only-headline --no-cpu --copy-calibration --device-warm 0 --steps 3 --warmup 1
python bench.py --summarize-profiles gpurun_out/prof_headline_trace gpurun_out/prof_headline_fetch gpurun_out/prof_headline_write
"""


TRACE_COMMAND = ("rocprofv3 --kernel-trace --stats -d gpurun_out/prof_bench_trace -o all --output-format csv -- "
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
        f"python bench.py --summarize-trace gpurun_out/prof_bench_trace",
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


def summarize_counters(out_name, title, command, dirs):
    """Per-kernel averages (per dispatch) of every counter collected in the
    rocprofv3 --pmc runs under `dirs` (library kernels only), written to
    profiles/<out_name>.md with the commands that made them."""
    import csv
    import glob
    from collections import defaultdict
    acc = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path) as f:
                for r in csv.DictReader(f):
                    name = r["Kernel_Name"]
                    if "kron" not in name and "copyBuffer" not in name:
                        continue
                    acc[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    counters = sorted({c for k in acc.values() for c in k})
    lines = [f"# {title}", "", "Counters are rocprofv3 --pmc readings averaged over the dispatches of each kernel "
             "(FETCH_SIZE / WRITE_SIZE in KiB per dispatch, raw; the others summed over the device).", "",
             "```", "export TMPDIR=/tmp", command.rstrip(), "```", "",
             "| kernel | dispatches | " + " | ".join(counters) + " |",
             "|---|---|" + "---|" * len(counters)]
    for name in sorted(acc):
        short = name.replace("void ", "")
        if ">(" in short:
            short = short[:short.index(">(") + 1]
        elif short.endswith(")"):
            short = short[:short.rfind("(")]
        n = max(len(v) for v in acc[name].values())
        vals = [f"{sum(acc[name][c]) / len(acc[name][c]):.4g}" if acc[name].get(c) else "" for c in counters]
        lines.append(f"| `{short[:110]}` | {n} | " + " | ".join(vals) + " |")
    lines.append("")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", out_name + ".md"), "w") as f:
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


def measurement_plan(torch, args):
    """Every measurement after the headline, as (name, thunk); bench.py
    --only NAME[,NAME] runs a subset (profiling runs)."""
    import workloads
    half = max(10, args.steps // 2)
    fifth = max(5, args.steps // 5)
    plan = [("precision", lambda: measure_precision(torch, half, args.warmup))]
    for mode, dim, n, batch, seed in (("f32", 2, 16, workloads.BATCH_2D[16], 1),
                                      ("f32", 2, 10, workloads.BATCH_2D[10], 1),
                                      ("f32", 3, 10, workloads.BATCH_3D[10], 2),
                                      ("f64", 3, 16, workloads.BATCH_3D[16] // 2, 2),
                                      ("f64", 2, 16, workloads.BATCH_2D[16] // 2, 1),
                                      ("bf16x3", 2, 16, workloads.BATCH_2D[16], 3)):
        plan.append((f"{mode}-{dim}d-n{n}",
                     lambda mode=mode, dim=dim, n=n, batch=batch, seed=seed:
                     measure(torch, mode, dim, n, batch, half, args.warmup, seed)))
    plan.append(("grouped", lambda: measure_grouped(torch, half, args.warmup)))
    for beta in (0.0, 0.5):
        plan.append((f"ex-beta{beta}", lambda beta=beta: measure_ex(torch, args.steps, args.warmup, beta)))
    plan.append(("ex2d-transx", lambda: measure_ex2d_transx(torch, args.steps, args.warmup)))
    for ld in (17, 20):
        plan.append((f"strided3d-ld{ld}", lambda ld=ld: measure_strided(torch, args.steps, args.warmup, ld)))
    for ldx, ldy in ((20, 16), (16, 20)):
        plan.append((f"strided3d-ldx{ldx}-ldy{ldy}",
                     lambda ldx=ldx, ldy=ldy: measure_strided(torch, args.steps, args.warmup, ldx, ldy)))
    plan.append(("strided2d", lambda: measure_strided2d(torch, args.steps, args.warmup)))
    plan.append(("tkron1", lambda: measure_tkron1(torch, args.steps, args.warmup)))
    plan.append(("backward", lambda: measure_backward(torch, args.steps, args.warmup)))
    plan.append(("grouped-backward", lambda: measure_grouped_backward(torch, fifth, args.warmup)))
    for case in ND_CASES:
        plan.append((f"nd:{case}", lambda case=case: measure_nd(torch, case, fifth, args.warmup)))
    return plan


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
    if args.summarize_counters:
        out_name, title, cmd_file, *dirs = args.summarize_counters
        with open(cmd_file) as f:
            summarize_counters(out_name, title, f.read(), dirs)
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
    tuned = None
    if args.tune_headline:
        tuned = tune_headline(torch)
    head = measure(torch, "f32", 3, 16, workloads.BATCH_3D[16], args.steps, args.warmup, seed=2)
    copy = measure_copy(torch, max(10, args.steps // 2), args.warmup)
    others = []
    if not args.only_headline:
        for name, run in measurement_plan(torch, args):
            if args.only and name not in args.only.split(","):
                continue
            got = run()
            others += got if isinstance(got, list) else [got]
            last = others[-1]
            print(f"# measured {name}: {last.get('gflops', last.get('ms'))}", file=sys.stderr, flush=True)

    khash = kernel_hash()
    roof = {"bound": "hbm", "achieved": head["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(head["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic_record(khash),
            "kernel": headline_kernel_name(), "alg_bytes_per_launch": head["alg_bytes"],
            "kernel_ms": head["ms"], "launch_shape": dict(launch_shape_record(), tuned_on_device=tuned),
            "copy_1gib": copy,
            "frac_of_copy": round(head["gbs"] / copy["gbs"], 4)}
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
        "bf16": next((o for o in others if o.get("mode") == "bf16" and o.get("dim") == 3), None),
        "modes": others,
        "kernel_hash": khash,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
