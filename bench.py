"""Benchmark of the load-balanced sample sort on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload pairs|dups|keys1m]

Default workload (the metric's configuration): 268,435,456 uniform u64 keys,
each with a u32 payload equal to its input index, P = 64 virtual processors,
512 regular samples per block, COUNT investigator.  One step = one whole
sort (steps 1-6 of Section IV) of device-resident input.  Prints one JSON line.

Measurement:
* value: keys sorted per second over K timed steps (GKeys/s), events on the
  stream the sort runs on, inputs already in HBM;
* roofline: the dominant kernel (the one with the largest share of the step)
  with its algorithmic bytes per launch divided by its average launch time,
  both taken live from per-launch HIP events; the whole pipeline's fraction
  of the byte model (K+V)(2D+2)+K per key is reported beside it;
* cpu_baseline: the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GKeys/s sorted (u64) + max/mean partition imbalance; batched vs per-instance"

WORKLOADS = {
    "pairs": dict(desc="plain sort, key-value pairs: 268,435,456 uniform u64 keys, u32 payload = input index, "
                       "P=64, 512 regular samples per block", n=1 << 28, P=64, s=512, vals=True, gen="uniform", seed=2),
    "dups": dict(desc="duplicate-heavy: 268,435,456 u64 keys, 50% one value and the rest Zipf(1.1) over 1,000 "
                      "values, P=64, 512 samples per block, keys only", n=1 << 28, P=64, s=512, vals=False,
                 gen="dups", seed=3),
    "keys1m": dict(desc="plain sort: 1,048,576 uniform u64 keys, P=8, 16 regular samples per block, keys only",
                   n=1 << 20, P=8, s=16, vals=False, gen="uniform", seed=1),
}


def kernel_bytes_per_launch(name, n, kb, vb):
    """Algorithmic bytes one launch of a bulk kernel moves (per key figure x keys)."""
    if name in ("onesweep", "merge"):
        return n * 2 * (kb + vb)          # read key+value, write key+value
    if name == "hist":
        return n * kb                     # read keys once for all digit counts
    return None


def profile_read(lib):
    need = lib.lbsort_profile_read(None, 0)
    buf = ctypes.create_string_buffer(need + 1)
    lib.lbsort_profile_read(buf, need + 1)
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


def make_input(w, device):
    import torch
    from paper_1611_00463_amd import datagen
    n = w["n"]
    if w["gen"] == "uniform":
        keys = datagen.uniform_keys_torch(n, w["seed"], device)
    else:
        keys = torch.from_numpy(datagen.duplicate_heavy_keys(n, seed=w["seed"])).to(device)
    vals = datagen.index_values_torch(n, device) if w["vals"] else None
    return keys, vals


def cpu_baseline(w, sample_n):
    """The CPU oracle as it stands, on the first sample_n keys of the workload."""
    import numpy as np
    from oracle import sample_sort as O
    from paper_1611_00463_amd import datagen
    if w["gen"] == "uniform":
        keys = datagen.uniform_keys(sample_n, seed=w["seed"])
    else:
        keys = datagen.duplicate_heavy_keys(sample_n, seed=w["seed"])
    vals = datagen.index_values(sample_n) if w["vals"] else None
    t0 = time.perf_counter()
    O.sample_sort(keys, vals, w["P"], w["s"], O.INV_COUNT)
    dt = time.perf_counter() - t0
    return {"value": round(sample_n / dt / 1e9, 6), "unit": "GKeys/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample_n} keys of the same workload (same P and s), numpy oracle, one thread, "
                      f"{dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pairs", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--cpu-sample", type=int, default=1 << 25)
    ap.add_argument("--fanin", type=int, default=0)
    ap.add_argument("--merge-tile", type=int, default=0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU exchange is not "
              f"part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1611_00463_amd import lbsort as L

    if args.copy_calibration:
        a = torch.ones(args.copy_calibration // 8, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": a.numel() * 8}))
        return

    w = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lib = L.load()
    print(f"[bench] generating {w['n']} keys ({args.workload})", file=sys.stderr, flush=True)
    keys, vals = make_input(w, dev)
    kout = torch.empty_like(keys)
    vout = torch.empty_like(vals) if vals is not None else None
    ws = L.Workspace(dev)
    kb, vb = 8, 4 if vals is not None else 0

    def step():
        if vals is None:
            return L.sort_keys(keys, w["P"], s=w["s"], fanin=args.fanin, merge_tile=args.merge_tile,
                               keys_out=kout, workspace=ws)
        return L.sort_pairs(keys, vals, w["P"], s=w["s"], fanin=args.fanin, merge_tile=args.merge_tile,
                            keys_out=kout, vals_out=vout, workspace=ws)

    for _ in range(args.warmup):
        r = step()
    torch.cuda.synchronize()
    L.check(ws.buf)
    print(f"[bench] warmup done; timing {args.steps} steps", file=sys.stderr, flush=True)
    lib.lbsort_profile_enable(1)
    profile_read(lib)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        r = step()
    e1.record(stream)
    torch.cuda.synchronize()
    lib.lbsort_profile_enable(0)
    ms = e0.elapsed_time(e1) / args.steps
    prof = profile_read(lib)
    L.check(ws.buf)

    n = w["n"]
    value = n / (ms / 1e3) / 1e9
    counts = r.part_counts.cpu().numpy()[0].astype(np.float64)
    imb = {"max_over_mean": round(float(counts.max() / counts.mean()), 6), "min": int(counts.min()),
           "max": int(counts.max()), "P": w["P"]}
    kernels = {k: {"launches_per_step": c / args.steps, "avg_ms": round(t / c, 5), "ms_per_step": round(t / args.steps, 5)}
               for k, (c, t) in prof.items()}
    dom = max(((k, t) for k, (c, t) in prof.items() if kernel_bytes_per_launch(k, n, kb, vb)), key=lambda x: x[1])[0]
    c, t = prof[dom]
    per_launch = kernel_bytes_per_launch(dom, n, kb, vb)
    achieved = per_launch / (t / c / 1e3) / 1e9
    D = kb  # one 8-bit digit pass per key byte
    model_bytes = (kb + vb) * (2 * D + 2) + kb
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_launch": per_launch, "avg_launch_ms": round(t / c, 5)}
    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "GKeys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": w["desc"], "n": n, "P": w["P"], "s": w["s"], "key": "u64",
                   "value": "u32" if vals is not None else None, "investigator": "COUNT",
                   "fanin": args.fanin or "tuned", "merge_tile": args.merge_tile or "tuned"},
        "imbalance": imb,
        "roofline": roof,
        "pipeline": {"bytes_per_key_model": model_bytes, "achieved_GBs": round(value * model_bytes, 1),
                     "frac": round(value * model_bytes / HBM_PEAK_GBS, 4)},
        "kernels": kernels,
    }
    if not args.no_cpu:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, min(args.cpu_sample, n))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
