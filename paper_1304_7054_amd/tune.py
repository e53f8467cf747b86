"""Autotuner driver: measure the launch shape of each (mode, dim, n) on this
GPU with kron_autotune and persist the table as JSON.

    python -m paper_1304_7054_amd.tune --out tune.json [--cases f32:3:16,f32:2:10]

Each entry is keyed by the device architecture and the HIP runtime version,
so a table measured on one kind of GPU is never applied to another.
``load(path)`` (run at import when KRON_TUNE_CACHE names a file) applies the
entries that match the current device.
"""
import argparse
import json
import os

from . import _binding as kb

MODES = {"f32": kb.MODE_F32, "f64": kb.MODE_F64, "bf16x3": kb.MODE_BF16X3, "bf16": kb.MODE_BF16,
         "bf16x6": kb.MODE_BF16X6}


def device_key():
    import torch
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "unknown").split(":")[0]
    return f"{arch}|hip-{torch.version.hip}"


def entry_key(dev, mode, dim, n):
    return f"{dev}|{mode}|{dim}|{n}"


def tune_case(mode, dim, n, target_bytes=256 << 20, reps=10):
    """Tune one (mode, dim, n) on seeded random data of about target_bytes."""
    import torch
    dt = kb._MODE_DTYPE[MODES[mode]]
    esize = torch.tensor([], dtype=dt).element_size()
    batch = max(1, target_bytes // (esize * n ** dim))
    gen = torch.Generator(device="cuda").manual_seed(1304 + 17 * dim + n)
    X = torch.randn(batch * n ** dim, generator=gen, device="cuda").to(dt)
    Y = torch.empty_like(X)
    mats = [torch.rand(n * n, generator=gen, device="cuda").to(dt) for _ in range(3)]
    b, v, ms = kb.kron_autotune(MODES[mode], dim, n, *mats[:3], X, Y, batch, reps)
    return {"blocks_per_cu": b, "variant": v, "ms": ms, "batch": batch}


def save(table, path):
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load(path):
    """Apply the entries of a saved table that match this device; returns how many."""
    with open(path) as f:
        table = json.load(f)
    dev = device_key()
    applied = 0
    for key, e in table.items():
        parts = key.split("|")
        if len(parts) != 5 or "|".join(parts[:2]) != dev:
            continue
        mode, dim, n = parts[2], int(parts[3]), int(parts[4])
        kb.kron_set_launch(MODES[mode], dim, n, int(e["blocks_per_cu"]), int(e["variant"]))
        applied += 1
    return applied


def main(argv=None):
    p = argparse.ArgumentParser(description="tune launch shapes on this GPU")
    p.add_argument("--out", required=True)
    p.add_argument("--cases", default=",".join(f"f32:{d}:{n}" for d in (2, 3) for n in range(1, 17)))
    p.add_argument("--mib", type=int, default=256, help="operand bytes per case (MiB)")
    a = p.parse_args(argv)
    dev = device_key()
    table = {}
    if os.path.exists(a.out):
        with open(a.out) as f:
            table = json.load(f)
    for case in a.cases.split(","):
        mode, dim, n = case.split(":")
        r = tune_case(mode, int(dim), int(n), a.mib << 20)
        table[entry_key(dev, mode, int(dim), int(n))] = r
        print(f"{case}: variant {r['variant']} blocks/CU {r['blocks_per_cu']} {r['ms']:.4f} ms", flush=True)
        save(table, a.out)


if __name__ == "__main__":
    main()
