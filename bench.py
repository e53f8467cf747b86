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
                  "paper_1304_7054_amd/csrc/kron_launch.hpp"]


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--only-headline", action="store_true", help="skip the other modes")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
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


def time_launches(torch, fn, args, steps, warmup):
    """Run `steps` launches bracketed by synchronisation; HIP events around
    every launch on the stream it is issued on.  Returns (wall ms/step,
    mean kernel ms, min kernel ms)."""
    stream = torch.cuda.current_stream()
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


def cpu_baseline(n=16, target_s=12.0):
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
    t = time.perf_counter()
    orc.kron3d(n, A, B, C, X, sample, "f32")
    dt = time.perf_counter() - t
    return {"value": round(sample * flops_per_op(3, n) / dt / 1e9, 2), "unit": "GFLOP/s",
            "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"FP32 oracle (plain C loops, OpenMP over operands) on {sample} of the 65536 "
                      f"3-D n=16 arrays, {dt:.1f} s"}


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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the batch splits into independent per-GPU shards; see DESIGN.md)", file=sys.stderr)
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

    khash = kernel_hash()
    roof = {"bound": "hbm", "achieved": head["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(head["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic_record(khash),
            "kernel": "kron3d_kernel<ModeF32, 16>", "alg_bytes_per_launch": head["alg_bytes"],
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
        "modes": others,
        "kernel_hash": khash,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
