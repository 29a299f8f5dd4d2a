"""Benchmark of the load-balanced sample sort on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload pairs|dups|keys1m|...]

Default workload (the metric's configuration): 268,435,456 uniform u64 keys,
each with a u32 payload equal to its input index, P = 64 virtual processors,
512 regular samples per block, COUNT investigator.  One step = one whole
sort (steps 1-6 of Section IV) of device-resident input.  Prints one JSON line.

Measurement:
* value: keys sorted per second over K timed steps (GKeys/s), events on the
  stream the sort runs on, inputs already in HBM, no per-launch
  instrumentation in that loop;
* kernels / roofline: a second loop of K steps with every launch bracketed by
  HIP events on the sort's stream: the dominant kernel (largest share of the
  step) with its algorithmic bytes per launch divided by its average launch
  time;
* roofline.traffic: HBM bytes one launch of that kernel moved (FETCH_SIZE +
  WRITE_SIZE, each scaled by what the same counter reads for a plain copy of
  known size), read from the committed rocprofv3 summary of this workload
  under profiles/; null when there is none or when the kernel's source file
  has changed since the counters were taken;
* pipeline: the algorithmic bytes of the kernels the step actually launched,
  per key and as a fraction of peak, beside the fixed 8-pass byte model;
* dups / batched (default run only): the duplicate-heavy configuration
  (balance and rate) and the batched configuration (one graph launch with
  autotuned settings against a per-instance loop), each checked on the device;
* cpu_baseline: the CPU oracle on a bounded sample of the same workload, on
  all host cores (steps 1 and 6 over a process pool) and on one thread.
"""
from __future__ import annotations

import argparse
import ctypes
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KEY_NAMES = {"torch.uint64": "u64", "torch.uint32": "u32", "torch.int64": "i64", "torch.int32": "i32",
             "torch.float64": "f64", "torch.float32": "f32"}
KERNEL_SOURCE = {"onesweep": "kernels_radix.hip", "merge": "kernels_merge.hip"}
METRIC = "GKeys/s sorted (u64) + max/mean partition imbalance; batched vs per-instance"

WORKLOADS = {
    "pairs": dict(desc="plain sort, key-value pairs: 268,435,456 uniform u64 keys, u32 payload = input index, "
                       "P=64, 512 regular samples per block", n=1 << 28, P=64, s=512, vals=True, gen="uniform", seed=2,
                  tag="pairs_2e28"),
    "dups": dict(desc="duplicate-heavy: 268,435,456 u64 keys, 50% one value and the rest Zipf(1.1) over 1,000 "
                      "values, P=64, 512 samples per block, keys only", n=1 << 28, P=64, s=512, vals=False,
                 gen="dups", seed=3, tag="dups_2e28"),
    "keys1m": dict(desc="plain sort: 1,048,576 uniform u64 keys, P=8, 16 regular samples per block, keys only",
                   n=1 << 20, P=8, s=16, vals=False, gen="uniform", seed=1, tag="keys1m"),
    "f64": dict(desc="float keys with provenance: 268,435,456 IEEE binary64 keys (Irwin-Hall of four uniforms, "
                     "centred, x1000; every 9973rd a NaN, infinity or signed zero), generated u32 index values, "
                     "P=64, 512 regular samples per block", n=1 << 28, P=64, s=512, vals="index", gen="typed",
                dtype="float64", seed=21, tag="f64_2e28"),
    "i64": dict(desc="signed keys with provenance: 268,435,456 uniform int64 keys, generated u32 index values, "
                     "P=64, 512 regular samples per block", n=1 << 28, P=64, s=512, vals="index", gen="typed",
                dtype="int64", seed=21, tag="i64_2e28"),
}


def kernel_bytes_per_launch(name, n, kb, vb):
    """Algorithmic bytes one launch of a bulk kernel moves over n keys (per key
    figure x keys); None for kernels whose work is metadata or depends on the
    data (the mid-size fix-up and the fallback passes, empty launches on
    uniform keys)."""
    if name in ("onesweep", "merge", "group_fix", "small_sort", "presorted"):
        return n * 2 * (kb + vb)          # read key+value, write key+value
    if name == "hist":
        return n * kb                     # read keys once for all digit counts
    return None


def executed_bytes(prof, steps, n_of, kb, vb):
    """Algorithmic bytes per step of the kernels the step launched: n_of(name)
    gives the keys one launch of that kernel covers."""
    total = 0
    for name, (cnt, _) in prof.items():
        per = kernel_bytes_per_launch(name, n_of(name), kb, vb)
        if per:
            total += per * cnt / steps
    return total


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 summaries, or None if absent or taken on other kernel source."""
    src = KERNEL_SOURCE.get(kernel)
    if src is None:
        return None
    with open(os.path.join(ROOT, "paper_1611_00463_amd", "csrc", src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic:"):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                if kv.get("kernel") == kernel and kv.get("workload") == workload and kv.get("source_sha256") == sha:
                    return {"bytes": int(kv["fetch_bytes"]) + int(kv["write_bytes"]),
                            "fetch_bytes": int(kv["fetch_bytes"]), "write_bytes": int(kv["write_bytes"]),
                            "source": os.path.relpath(path, ROOT)}
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
    import numpy as np
    import torch
    from paper_1611_00463_amd import datagen
    n = w["n"]
    if w["gen"] == "uniform":
        keys = datagen.uniform_keys_torch(n, w["seed"], device)
    elif w["gen"] == "typed":
        keys = datagen.typed_keys_torch(n, w["seed"], getattr(np, w["dtype"]), device)
    else:
        keys = torch.from_numpy(datagen.duplicate_heavy_keys(n, seed=w["seed"])).to(device)
    vals = datagen.index_values_torch(n, device) if w["vals"] is True else None
    return keys, vals


def cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_baseline(w, n_all, n_one):
    """The CPU oracle as it stands, on bounded samples of the same workload
    (the first keys, same P and s): on all host cores, with the oracle's steps
    1 and 6 over a process pool (at most 16 workers, the host share of one
    GPU), and on one thread."""
    import numpy as np
    from oracle import parallel as OP
    from oracle import sample_sort as O
    from oracle import typed as T
    from paper_1611_00463_amd import datagen
    nproc, model = cpu_info()
    workers = max(1, min(16, nproc or 1))
    if w["gen"] == "uniform":
        keys = datagen.uniform_keys(n_all, seed=w["seed"])
    elif w["gen"] == "typed":
        keys = datagen.typed_keys(n_all, seed=w["seed"], dtype=getattr(np, w["dtype"]))
    else:
        keys = datagen.duplicate_heavy_keys(n_all, seed=w["seed"])
    vals = datagen.index_values(n_all) if w["vals"] else None
    ikeys = T.total_order_int(keys) if keys.dtype.kind == "f" else keys
    t0 = time.perf_counter()
    OP.sample_sort_parallel(ikeys, vals, w["P"], w["s"], O.INV_COUNT, workers=workers)
    dt_all = time.perf_counter() - t0
    t0 = time.perf_counter()
    T.sample_sort_typed(keys[:n_one], None if vals is None else vals[:n_one], w["P"], w["s"], O.INV_COUNT)
    dt_one = time.perf_counter() - t0
    return {"value": round(n_all / dt_all / 1e9, 6), "unit": "GKeys/s", "cores": workers, "kind": "oracle",
            "nproc": nproc, "cpu_model": model,
            "sample": f"first {n_all} keys of the same workload (same P and s), numpy oracle with steps 1 and 6 "
                      f"over {workers} worker processes, {dt_all:.2f} s wall (worker start-up included)",
            "one_thread": {"value": round(n_one / dt_one / 1e9, 6), "unit": "GKeys/s", "cores": 1,
                           "sample": f"first {n_one} keys, numpy oracle, one thread, {dt_one:.2f} s"}}


def check_batch_on_device(plan, keys, seg, sizes, P):
    """Every instance of a batched sort, on the device: keys non-decreasing,
    (key, value) pairs a permutation of the instance (values are local input
    positions), equal keys in position order (stable), and each partition
    offset G_k = clamp(floor(k n / P), #keys < v_k, #keys <= v_k) for the
    instance's splitter v_k (the count-based investigator), read from the
    sorted keys themselves."""
    import numpy as np
    import torch
    total = int(sizes.sum())
    seg64 = seg.view(torch.int64)
    u = lambda t: t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    kin = u(keys)
    seen = torch.zeros(total, dtype=torch.int32, device=keys.device)
    CH = 1 << 27
    for a in range(0, total, CH):
        e = min(total, a + CH)
        idx = torch.arange(a, e, device=keys.device, dtype=torch.int64)
        seg_of = torch.searchsorted(seg64, idx, right=True) - 1
        ko, vo = u(plan.keys_out[a:e]), plan.vals_out[a:e].view(torch.int32).to(torch.int64)
        n_of = seg64[seg_of + 1] - seg64[seg_of]
        assert bool(((vo >= 0) & (vo < n_of)).all()), "batched output: value outside its instance"
        src = seg64[seg_of] + vo
        assert bool((kin[src] == ko).all()), "batched output: pairs broken"
        seen.index_add_(0, src, torch.ones_like(src, dtype=torch.int32))
        same = seg_of[1:] == seg_of[:-1]
        assert bool((ko[1:][same] >= ko[:-1][same]).all()), "batched output not sorted within instances"
        eq = same & (ko[1:] == ko[:-1])
        assert bool((vo[1:][eq] > vo[:-1][eq]).all()), "batched output not stable"
        del idx, seg_of, ko, vo, n_of, src, same, eq
    assert bool((seen == 1).all()), "batched output is not a permutation of its instances"
    del seen, kin
    ko = u(plan.keys_out)
    edges = torch.arange(CH, total, CH, device=keys.device)
    if edges.numel():
        inside = (torch.searchsorted(seg64, edges, right=True) == torch.searchsorted(seg64, edges - 1, right=True))
        assert bool((ko[edges][inside] >= ko[edges - 1][inside]).all()), "batched output not sorted"
    # partition offsets against the splitters, instance by instance
    B = seg.numel() - 1
    G = plan.part_offsets                                   # [B, P+1]
    n = torch.from_numpy(sizes.astype(np.int64)).to(keys.device)
    assert bool((G[:, 0] == 0).all() and (G[:, P] == n).all() and (G[:, 1:] >= G[:, :-1]).all()), "offsets"
    if P > 1:
        v = u(plan.splitters)                               # [B, P-1]
        k = torch.arange(1, P, device=keys.device, dtype=torch.int64)
        T_ = (k[None, :] * n[:, None]) // P
        Gk = G[:, 1:P]
        base = seg64[:B, None]
        below = torch.where(Gk > 0, ko[(base + Gk - 1).clamp(min=0, max=total - 1)], torch.full_like(Gk, -1))
        at = torch.where(Gk < n[:, None], ko[(base + Gk).clamp(max=total - 1)], torch.full_like(Gk, 1 << 40))
        # any G in [#<v, #<=v] has below <= v <= at; G above T must be #<v
        # (below < v), G below T must be #<=v (at > v)
        ok = (below <= v) & (at >= v)
        ok &= torch.where(Gk == T_, torch.ones_like(ok), torch.where(Gk > T_, below < v, at > v))
        assert bool(ok.all()), "partition offsets differ from the count-based investigator"


def presorted_keys(keys, sizes, P):
    """Keys in blocks above 4096 keys, and of those the keys in blocks that
    are already non-decreasing or non-increasing (uint32 keys, counted on the
    device)."""
    import numpy as np
    import torch
    sz = sizes.astype(np.int64)
    seg = np.concatenate([[0], np.cumsum(sz)])
    bounds = seg[:-1, None] + (np.arange(P + 1)[None, :] * sz[:, None]) // P      # [B, P+1]
    starts = np.concatenate([bounds[:, :-1].reshape(-1), [seg[-1]]])           # [NB+1]
    bsz = np.diff(starts)
    st = torch.from_numpy(starts).to(keys.device)
    NB = len(bsz)
    up_bad = torch.zeros(NB, dtype=torch.int64, device=keys.device)
    down_bad = torch.zeros_like(up_bad)
    k = keys.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    total = k.numel()
    CH = 1 << 27
    for a in range(0, max(total - 1, 0), CH):
        e = min(total - 1, a + CH)
        x = torch.arange(a, e, device=keys.device, dtype=torch.int64)
        blk = torch.searchsorted(st, x, right=True) - 1
        inside = (x + 1) < st[blk + 1]
        d = k[a + 1:e + 1] - k[a:e]
        up_bad.index_add_(0, blk[inside], (d[inside] < 0).to(torch.int64))
        down_bad.index_add_(0, blk[inside], (d[inside] > 0).to(torch.int64))
        del x, blk, inside, d
    pre = ((up_bad == 0) | (down_bad == 0)).cpu().numpy()
    large = bsz > 4096
    return int(bsz[large].sum()), int(bsz[large & pre].sum())


def run_batch(args, steps, warmup, tune=True, check=True):
    """Batched form: B uneven u32 key/value instances (sizes log-uniform in
    [1K, 4M], uniform / normal / sorted / reverse keys), P = 8, sorted by one
    lbsort_sort_batch call replayed from a HIP graph with autotuned settings,
    against a loop of B lbsort_sort_pairs calls over the same instances on
    the same stream."""
    import numpy as np
    import torch
    from paper_1611_00463_amd import datagen
    from paper_1611_00463_amd import lbsort as L
    lib = L.load()
    B, P = args.batch, 8
    print(f"[bench] generating a batch of {B} instances", file=sys.stderr, flush=True)
    keys, vals, seg, sizes = datagen.batch_u32_torch(B, 4, device="cuda")
    total = int(sizes.sum())
    tuned = None
    force = dict(fanin=args.fanin, merge_tile=args.merge_tile, radix_tile=args.radix_tile, handler=args.handler,
                 presorted=args.presorted)
    if tune and not any(force.values()):
        print("[bench] autotuning the batch", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        tuned = L.autotune(L.U32, L.VAL_U32, P, keys=keys, vals=vals, seg_offsets=seg)
        tuned["tuning_s"] = round(time.perf_counter() - t0, 2)
    used = L.resolve_params(L.U32, L.VAL_U32, P, total, B=B, **force)
    plan = L.BatchPlan(keys, seg, P, vals=vals, **force)
    for _ in range(warmup):
        plan.run()
    torch.cuda.synchronize()
    plan.check()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.run()
    e1.record()
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1) / steps
    # kernel split from one instrumented eager run
    lib.lbsort_profile_enable(1)
    profile_read(lib)
    plan.run()
    torch.cuda.synchronize()
    lib.lbsort_profile_enable(0)
    prof = profile_read(lib)
    plan.capture()
    for _ in range(warmup):
        plan.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        plan.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / steps
    plan.check()
    if check:
        check_batch_on_device(plan, keys, seg, sizes, P)
    if args.no_loop:
        return {"value": round(total / (ms_graph / 1e3) / 1e9, 4), "unit": "GKeys/s", "ms_per_step": round(ms_graph, 4),
                "config": {"workload": f"batching: {B} instances (no per-instance loop)", "total_keys": total},
                "settings": used, "graph_ms": round(ms_graph, 4),
                "kernels": {k: {"launches": c, "ms": round(t, 5)} for k, (c, t) in prof.items()}}
    # the per-instance loop
    kout = torch.empty_like(keys)
    vout = torch.empty_like(vals)
    prm = L.Params(P, 0, 0, used["fanin"], used["merge_tile"], used["radix_tile"], used["handler"],
                   used["presorted"], 0)
    offs = torch.empty((B, P + 1), dtype=torch.int64, device="cuda")
    need = ctypes.c_size_t(0)
    parts = L.Parts(offs.data_ptr(), 0, 0, 0, 0)
    L._check(lib.lbsort_sort_pairs(L.U32, L.VAL_U32, None, None, None, None, int(sizes.max()), ctypes.byref(prm),
                                   ctypes.byref(parts), None, ctypes.byref(need), None))
    wsb = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    have = ctypes.c_size_t(need.value)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    hseg = seg.cpu().numpy().astype(np.int64)
    kp, vp, kop, vop = keys.data_ptr(), vals.data_ptr(), kout.data_ptr(), vout.data_ptr()
    part_ptrs = [L.Parts(offs.data_ptr() + b * (P + 1) * 8, 0, 0, 0, 0) for b in range(B)]

    def loop():
        for b in range(B):
            a, n = int(hseg[b]), int(hseg[b + 1] - hseg[b])
            rc = lib.lbsort_sort_pairs(L.U32, L.VAL_U32, ctypes.c_void_p(kp + 4 * a), ctypes.c_void_p(vp + 4 * a),
                                       ctypes.c_void_p(kop + 4 * a), ctypes.c_void_p(vop + 4 * a), n,
                                       ctypes.byref(prm), ctypes.byref(part_ptrs[b]),
                                       ctypes.c_void_p(wsb.data_ptr()), ctypes.byref(have), stream)
            if rc:
                L._check(rc)

    loop()
    torch.cuda.synchronize()
    loops = max(1, steps // 5)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(loops):
        loop()
    e1.record()
    torch.cuda.synchronize()
    wall_loop = (time.perf_counter() - t0) * 1e3 / loops
    ms_loop = e0.elapsed_time(e1) / loops
    i32 = lambda t: t.view(torch.int32)
    assert torch.equal(i32(kout), i32(plan.keys_out)) and torch.equal(i32(vout), i32(plan.vals_out)), \
        "loop and batch differ"
    assert torch.equal(offs, plan.part_offsets), "loop and batch partition offsets differ"
    # roofline of the dominant kernel: the histogram reads the keys of blocks
    # larger than one LDS sort (4096 keys), small_sort sorts the others; of
    # the large blocks, those already in order or in reverse order are copied
    # (presorted) and the others take the radix passes (onesweep)
    n_large, n_pre = presorted_keys(keys, sizes, P)
    n_of = lambda name: {"onesweep": n_large - n_pre, "hist": n_large, "presorted": n_pre,
                         "small_sort": total - n_large}.get(name, total)
    dom = max(((k, t) for k, (c, t) in prof.items() if kernel_bytes_per_launch(k, n_of(k), 4, 4)),
              key=lambda x: x[1])[0]
    c, t = prof[dom]
    per_launch = kernel_bytes_per_launch(dom, n_of(dom), 4, 4)
    achieved = per_launch / (t / c / 1e3) / 1e9
    ex = executed_bytes(prof, 1, n_of, 4, 4)
    value = total / (ms_graph / 1e3) / 1e9
    return {
        "value": round(value, 4), "unit": "GKeys/s", "ms_per_step": round(ms_graph, 4),
        "config": {"workload": f"batching: {B} uint32 key-value instances, sizes log-uniform in [1K, 4M], "
                               f"uniform/normal/sorted/reverse keys, P=8, one HIP-graph launch, autotuned",
                   "instances": B, "total_keys": total, "P": P, "keys_in_blocks_above_4096": n_large,
                   "keys_in_presorted_blocks": n_pre},
        "settings": used, "autotuned": tuned,
        "eager_ms": round(ms_eager, 4), "graph_ms": round(ms_graph, 4),
        "loop_ms": round(ms_loop, 4), "loop_wall_ms": round(wall_loop, 2),
        "loop_GKeys_s": round(total / (ms_loop / 1e3) / 1e9, 4),
        "speedup_vs_loop": round(ms_loop / ms_graph, 3),
        "checked": "on the device: sorted, permutation, stable, offsets = count-based clamp" if check else None,
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": per_launch, "avg_launch_ms": round(t / c, 5)},
        "pipeline": {"executed_bytes_per_key": round(ex / total, 2),
                     "executed_frac": round(value * ex / total / HBM_PEAK_GBS, 4)},
        "kernels": {k: {"launches": c, "ms": round(t, 5)} for k, (c, t) in prof.items()},
    }


def bench_batch(args):
    b = run_batch(args, args.steps, args.warmup, tune=not args.no_tune)
    line = {"metric": "batched sort: GKeys/s (u32 keys + u32 values), one graph launch vs a per-instance loop",
            "value": b.pop("value"), "unit": "GKeys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": b.pop("ms_per_step"), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u32", "data": "synthetic", "config": b.pop("config")}
    line.update(b)
    print(json.dumps(line), flush=True)


def bench_balance(args):
    """Balance study (Section V: Table 2 and the sample-size figures) at the
    paper's size: N keys (10^9 by default) of each of the four input
    distributions, sorted by P = 10 virtual processors with the sample budget
    X = 256 KB / P and with 0.004X ... 1.4X, under each investigator mode at X.
    Also min/max partition sizes for P = 8 ... 52 at 0.004X, X and 1.4X on
    uniform keys, and every distribution at P = 8 ... 52 with the default
    budget (balance and sort rate: the paper's workload suite).  value = the largest max/mean share over the four
    distributions at X with the count-based investigator (Table 2's setting)."""
    import numpy as np
    import torch
    from paper_1611_00463_amd import datagen
    from paper_1611_00463_amd import lbsort as L
    n, P = args.balance_n, 10
    factors = (0.004, 0.04, 0.4, 1.0, 1.004, 1.04, 1.4)
    modes = {"COUNT": L.INV_COUNT, "NONE": L.INV_NONE, "PAPER": L.INV_PAPER}
    ws = L.Workspace("cuda")
    kout = torch.empty(n, dtype=torch.uint64, device="cuda")

    def shares(keys, P, s, mode):
        r = L.sort_keys(keys, P, s=s, investigator=mode, keys_out=kout, workspace=ws)
        L.check(ws.buf)
        c = r.part_counts.view(torch.int64).cpu().numpy()[0].astype(np.float64)
        return c

    def summary(c):
        return {"max_over_mean": round(float(c.max() / c.mean()), 6), "min_pct": round(float(100 * c.min() / c.sum()), 4),
                "max_pct": round(float(100 * c.max() / c.sum()), 4), "max_minus_min": int(c.max() - c.min())}

    table2, sweep, modes_at_x, rates, suite = {}, {}, {}, {}, {}
    X = 262144 // (P * 8)
    for dist in datagen.BALANCE_DISTS:
        print(f"[bench] balance: {dist}", file=sys.stderr, flush=True)
        keys = datagen.balance_keys_torch(dist, n, device="cuda")
        torch.cuda.synchronize()
        sweep[dist] = {}
        for f in factors:
            s = max(1, int(f * X))
            sweep[dist][f"{f}X"] = dict(s=s, **summary(shares(keys, P, s, L.INV_COUNT)))
        c = shares(keys, P, X, L.INV_COUNT)
        table2[dist] = [round(float(100 * v / c.sum()), 3) for v in c]
        modes_at_x[dist] = {m: summary(shares(keys, P, X, code)) for m, code in modes.items()}
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            L.sort_keys(keys, P, s=X, keys_out=kout, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        rates[dist] = round(n / (e0.elapsed_time(e1) / 3 / 1e3) / 1e9, 3)
        # the workload suite: every distribution at P = 8 ... 52 with the
        # default sample budget, balance and sort rate (one timed sort each)
        suite[dist] = {}
        for Pp in (8, 16, 32, 52):
            c = shares(keys, Pp, 0, L.INV_COUNT)
            e0.record()
            L.sort_keys(keys, Pp, s=0, keys_out=kout, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            suite[dist][str(Pp)] = dict(GKeys_s=round(n / (e0.elapsed_time(e1) / 1e3) / 1e9, 3), **summary(c))
        del keys
    print("[bench] balance: processor sweep", file=sys.stderr, flush=True)
    keys = datagen.balance_keys_torch("uniform", n, device="cuda")
    procs = {}
    for Pp in (8, 16, 32, 52):
        Xp = 262144 // (Pp * 8)
        procs[str(Pp)] = {f"{f}X": dict(s=max(1, int(f * Xp)), **summary(shares(keys, Pp, max(1, int(f * Xp)), L.INV_COUNT)))
                          for f in (0.004, 1.0, 1.4)}
        # X rounded down to a multiple of P: every splitter's target rank k*s/P is a whole sample
        sm = max(Pp, Xp // Pp * Pp)
        procs[str(Pp)]["X_multiple_of_P"] = dict(s=sm, **summary(shares(keys, Pp, sm, L.INV_COUNT)))
    worst = max(modes_at_x[d]["COUNT"]["max_over_mean"] for d in datagen.BALANCE_DISTS)
    line = {
        "metric": "max/mean partition share, balance study (Table 2 setting)", "value": worst, "unit": "ratio",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": round(worst / 1.0022, 4), "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"balance study: {n:,} u64 keys per distribution (uniform, normal, right-skewed, "
                               f"exponential), P=10, s = X = {X} and 0.004X..1.4X, COUNT/NONE/PAPER",
                   "n": n, "P": P, "X": X},
        "table2_shares_pct": table2, "sample_sweep": sweep, "modes_at_X": modes_at_x, "processor_sweep": procs,
        "GKeys_s_at_X": rates, "suite_P8_to_52": suite,
    }
    print(json.dumps(line), flush=True)


def bench_search(args):
    """Binary search over a sorted result (Section III, Section IV.C): 2^28
    uniform u64 keys sorted once with P = 64 (untimed), the search index built
    once (timed on its own), then K timed calls of lbsort_search_indexed for
    2^24 queries (half of them keys of the data, half random 64-bit values),
    each returning the position and the holding partition; K calls of the
    plain lbsort_search beside it, and every position compared."""
    import numpy as np
    import torch
    from paper_1611_00463_amd import datagen
    from paper_1611_00463_amd import lbsort as L
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lib = L.load()
    n, P, nq = 1 << 28, 64, 1 << 24
    print(f"[bench] search: sorting {n} keys, {nq} queries", file=sys.stderr, flush=True)
    keys = datagen.uniform_keys_torch(n, 2, dev)
    r = L.sort_keys(keys, P, s=512)
    L.check(r.workspace)
    sk, G = r.keys, r.part_offsets[0].contiguous()
    del keys
    pick = datagen.u64_torch(40, 0, nq // 2, dev).view(torch.int64).remainder(n)
    q = torch.cat([sk.view(torch.int64)[pick], datagen.u64_torch(41, 0, nq - nq // 2, dev).view(torch.int64)])
    pos = torch.empty(nq, dtype=torch.int64, device=dev)
    part = torch.empty(nq, dtype=torch.uint32, device=dev)
    pos2 = torch.empty_like(pos)
    part2 = torch.empty_like(part)
    stream = torch.cuda.current_stream()
    nbytes = int(lib.lbsort_search_index_bytes(L.U64, n))
    index = torch.empty(nbytes, dtype=torch.uint8, device=dev)

    def build():
        L._check(lib.lbsort_search_build_index(L.U64, L._ptr(sk), n, L._ptr(index), L._stream()))

    def indexed():
        L._check(lib.lbsort_search_indexed(L.U64, L._ptr(sk), n, L._ptr(index), L._ptr(q), nq, 0, L._ptr(G), P,
                                           L._ptr(pos), L._ptr(part), L._stream()))

    def plain():
        L._check(lib.lbsort_search(L.U64, L._ptr(sk), n, L._ptr(q), nq, 0, L._ptr(G), P, L._ptr(pos2),
                                   L._ptr(part2), L._stream()))

    def timed(f, steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            f()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    for _ in range(args.warmup):
        build()
        indexed()
        plain()
    torch.cuda.synchronize()
    ms_build = timed(build, args.steps)
    ms = timed(indexed, args.steps)
    ms_plain = timed(plain, args.steps)
    lib.lbsort_profile_enable(1)
    profile_read(lib)
    for _ in range(args.steps):
        indexed()
    torch.cuda.synchronize()
    lib.lbsort_profile_enable(0)
    prof = profile_read(lib)
    assert torch.equal(pos, pos2) and torch.equal(part, part2), "indexed and plain searches differ"
    # spot check against the data itself: sk[pos-1] < q <= sk[pos]
    idx = torch.arange(0, nq, 9973, device=dev)
    pp, qq = pos[idx], q[idx]
    sgn = -(1 << 63)
    sv, qv = sk.view(torch.int64) ^ sgn, qq.view(torch.int64) ^ sgn
    ok_lo = (pp == 0) | (sv[(pp - 1).clamp(min=0)] < qv)
    ok_hi = (pp == n) | (sv[pp.clamp(max=n - 1)] >= qv)
    assert bool((ok_lo & ok_hi).all()), "search positions inconsistent with the sorted data"
    c, t = prof["search_indexed"]
    per = nq * (8 + 8 + 4)                    # query in, position and partition out
    achieved = per / (t / c / 1e3) / 1e9
    line = {
        "metric": "GQueries/s, binary search over sorted u64 keys", "value": round(nq / (ms / 1e3) / 1e9, 4),
        "unit": "GQueries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "search: 16,777,216 queries (half keys of the data, half random) over 268,435,456 "
                               "sorted uniform u64 keys in 64 partitions, through the search index (built once)",
                   "n": n, "queries": nq, "P": P},
        "index": {"bytes": nbytes, "build_ms": round(ms_build, 4),
                  "GQueries_s_with_build": round(nq / ((ms + ms_build) / 1e3) / 1e9, 4)},
        "plain": {"GQueries_s": round(nq / (ms_plain / 1e3) / 1e9, 4), "ms": round(ms_plain, 4),
                  "same_positions": True},
        "roofline": {"kernel": "search_indexed", "bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": None, "bytes_per_launch": per, "avg_launch_ms": round(t / c, 5),
                     "note": "one 16-key group per index level (about 7 cache lines per query, most of them "
                             "cached): bound by memory requests, the byte figure counts only the query and its "
                             "two outputs"},
    }
    print(json.dumps(line), flush=True)


def bench_serve(args):
    """Served form: a Poisson stream of u64 sort requests (sizes log-uniform in
    [10K, 64M], uniform / Zipf(1.2) / sorted / reverse keys sliced from 64M-key
    device-resident pools), P = 64, continuous batching on 4 streams under a
    64 GB HBM budget, against serving the same stream one request at a time."""
    import torch
    from paper_1611_00463_amd import datagen
    from paper_1611_00463_amd import serve as S
    pool_n = 1 << 26
    print("[bench] generating request pools", file=sys.stderr, flush=True)
    pools = [datagen.serve_pool_u64_torch(d, pool_n, 5, "cuda") for d in range(4)]
    torch.cuda.synchronize()
    import numpy as np
    from paper_1611_00463_amd import lbsort as L
    warm = S.make_requests(64, seed=55, pool_n=pool_n, rate=args.serve_rate, lo=10_000, hi=pool_n)
    S.Server(pools, P=64, budget_bytes=64 << 30, streams=4).run(warm)
    print(f"[bench] serving {args.serve_requests} requests at {args.serve_rate} req/s", file=sys.stderr, flush=True)
    reqs = S.make_requests(args.serve_requests, seed=5, pool_n=pool_n, rate=args.serve_rate, lo=10_000, hi=pool_n)
    # a seeded sample of the requests keeps its outputs for the check below
    kept = set(int(x) for x in np.random.default_rng(5).choice(len(reqs), min(16, len(reqs)), replace=False))
    srv = S.Server(pools, P=64, budget_bytes=64 << 30, streams=4, keep_ids=kept)
    t0 = time.perf_counter()
    srv.run(reqs)
    wall = time.perf_counter() - t0
    served = S.summarize(reqs, wall)
    assert served["device_errors"] == 0, "a served batch latched a device error"
    for r in reqs:
        if r.rid in kept:
            alone = L.sort_keys(pools[r.dist][r.offset:r.offset + r.n], 64)
            L.check(alone.workspace)
            assert torch.equal(alone.keys.view(torch.int64), r.keys_out.view(torch.int64)), f"request {r.rid}"
            assert torch.equal(alone.part_offsets[0], r.part_offsets), f"request {r.rid} offsets"
            r.keys_out = r.part_offsets = None
    served["checked"] = f"{len(kept)} sampled requests equal to the same request sorted alone"
    offered = sum(r.n for r in reqs) / max(r.arrival for r in reqs) / 1e9
    print("[bench] per-request baseline", file=sys.stderr, flush=True)
    base = S.make_requests(args.serve_requests, seed=5, pool_n=pool_n, rate=args.serve_rate, lo=10_000, hi=pool_n)
    S.run_per_request(pools, base[:8], 64)
    base = S.make_requests(args.serve_requests, seed=5, pool_n=pool_n, rate=args.serve_rate, lo=10_000, hi=pool_n)
    t0 = time.perf_counter()
    S.run_per_request(pools, base, 64)
    bwall = time.perf_counter() - t0
    single = S.summarize(base, bwall)
    line = {"metric": "served sort: delivered GKeys/s (u64) with p50/p99 latency, continuous batching vs "
                      "one request at a time",
            "value": served["GKeys_s"], "unit": "GKeys/s", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": round(wall * 1e3, 2), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"serving: Poisson stream ({args.serve_rate:g} req/s) of {args.serve_requests} "
                                   "u64 sort requests, sizes log-uniform in [10K, 64M], uniform/Zipf(1.2)/sorted/"
                                   "reverse, P=64, 64 GB HBM budget, 4 streams", "P": 64},
            "offered_GKeys_s": round(offered, 4), "served": served, "one_at_a_time": single,
            "p50_ms": served["p50_ms"], "p99_ms": served["p99_ms"],
            "speedup_vs_one_at_a_time": round(served["GKeys_s"] / single["GKeys_s"], 3)}
    print(json.dumps(line), flush=True)


def measure_sort(w, args, steps, warmup, profile=True, tune=False):
    """Time one sort workload: `steps` steps without instrumentation (the
    figure), then, with profile, `steps` more with per-launch events.  With
    tune, the autotuner first picks the radix tile, handler schedule, fan-in
    and merge tile on this very input (the settings used are reported)."""
    import numpy as np
    import torch
    from paper_1611_00463_amd import lbsort as L
    dev = torch.device("cuda:0")
    lib = L.load()
    print(f"[bench] generating {w['n']} keys ({w['tag']})", file=sys.stderr, flush=True)
    keys, vals = make_input(w, dev)
    kout = torch.empty_like(keys)
    has_v = bool(w["vals"])
    vout = torch.empty(w["n"], dtype=torch.uint32, device=dev) if has_v else None
    ws = L.Workspace(dev)
    vt = (L.VAL_U32 if vals is not None else L.VAL_INDEX) if has_v else L.NOVAL
    tuned = None
    if tune and not (args.fanin or args.merge_tile or args.radix_tile or args.handler or args.presorted):
        print(f"[bench] autotuning {w['tag']}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        tuned = L.autotune(L.key_code(keys.dtype), vt, w["P"], keys=keys, vals=vals)
        tuned["tuning_s"] = round(time.perf_counter() - t0, 2)

    def step():
        if not has_v:
            return L.sort_keys(keys, w["P"], s=w["s"], fanin=args.fanin, merge_tile=args.merge_tile,
                               keys_out=kout, workspace=ws, radix_tile=args.radix_tile, handler=args.handler,
                               presorted=args.presorted)
        return L.sort_pairs(keys, vals, w["P"], s=w["s"], fanin=args.fanin, merge_tile=args.merge_tile,
                            keys_out=kout, vals_out=vout, workspace=ws, radix_tile=args.radix_tile,
                            handler=args.handler, presorted=args.presorted)

    for _ in range(warmup):
        r = step()
    torch.cuda.synchronize()
    L.check(ws.buf)
    print(f"[bench] warmup done; timing {steps} steps", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        r = step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    L.check(ws.buf)
    prof, ms_prof = None, None
    if profile:
        lib.lbsort_profile_enable(1)
        profile_read(lib)
        e0.record(stream)
        for _ in range(steps):
            r = step()
        e1.record(stream)
        torch.cuda.synchronize()
        lib.lbsort_profile_enable(0)
        prof = profile_read(lib)
        ms_prof = e0.elapsed_time(e1) / steps
        L.check(ws.buf)
    counts = r.part_counts.cpu().numpy()[0].astype(np.float64)
    imb = {"max_over_mean": round(float(counts.max() / counts.mean()), 6), "min": int(counts.min()),
           "max": int(counts.max()), "P": w["P"]}
    used = L.resolve_params(L.key_code(keys.dtype), vt, w["P"], w["n"], s=w["s"], fanin=args.fanin,
                            merge_tile=args.merge_tile, radix_tile=args.radix_tile, handler=args.handler,
                            presorted=args.presorted)
    out = dict(ms=ms, value=w["n"] / (ms / 1e3) / 1e9, prof=prof, ms_prof=ms_prof, imbalance=imb, settings=used,
               autotuned=tuned, kb=keys.element_size(), vb=4 if has_v else 0, dtype=KEY_NAMES[str(keys.dtype)])
    del keys, vals, kout, vout, ws, r
    torch.cuda.empty_cache()
    return out


def summarize_sort(w, m, steps):
    """Kernel split, the dominant kernel's roofline and the pipeline's bytes."""
    n, kb, vb, prof, value = w["n"], m["kb"], m["vb"], m["prof"], m["value"]
    kernels = {k: {"launches_per_step": c / steps, "avg_ms": round(t / c, 5), "ms_per_step": round(t / steps, 5)}
               for k, (c, t) in prof.items()}
    dom = max(((k, t) for k, (c, t) in prof.items() if kernel_bytes_per_launch(k, n, kb, vb)), key=lambda x: x[1])[0]
    c, t = prof[dom]
    per_launch = kernel_bytes_per_launch(dom, n, kb, vb)
    achieved = per_launch / (t / c / 1e3) / 1e9
    tr = measured_traffic(dom, w["tag"])
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr["bytes"] if tr else None,
            "bytes_per_launch": per_launch, "avg_launch_ms": round(t / c, 5)}
    if tr:
        roof["traffic_detail"] = tr
    ex = executed_bytes(prof, steps, lambda name: n, kb, vb) / n
    D = kb  # one 8-bit digit pass per key byte
    model_bytes = (kb + vb) * (2 * D + 2) + kb
    pipe = {"executed_bytes_per_key": round(ex, 2), "executed_GBs": round(value * ex, 1),
            "executed_frac": round(value * ex / HBM_PEAK_GBS, 4),
            "model_bytes_per_key": model_bytes, "model_frac": round(value * model_bytes / HBM_PEAK_GBS, 4),
            "note": "executed: algorithmic bytes of the kernels the step launched (histogram, radix passes, "
                    "group fix-up, merge passes); model: the fixed normalisation (K+V)(2D+2)+K of an eight-pass "
                    "LSD sort and one merge pass, which credits the radix passes the fix-up makes unnecessary"}
    return roof, pipe, kernels


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pairs", choices=sorted(WORKLOADS) + ["batch", "serve", "balance", "search"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--no-tune", action="store_true", help="run with the default settings, no autotuning")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: leave out the duplicate-heavy and batched objects")
    ap.add_argument("--cpu-sample", type=int, default=1 << 26, help="keys of the all-cores oracle sample")
    ap.add_argument("--cpu-sample-one", type=int, default=1 << 24, help="keys of the one-thread oracle sample")
    ap.add_argument("--fanin", type=int, default=0)
    ap.add_argument("--merge-tile", type=int, default=0)
    ap.add_argument("--radix-tile", type=int, default=0)
    ap.add_argument("--handler", type=int, default=0, help="1: F-way passes, 2: one pass (0: tuned)")
    ap.add_argument("--presorted", type=int, default=0,
                    help="1: detect presorted blocks, 2: ignore them (0: tuned)")
    ap.add_argument("--no-loop", action="store_true", help="batch: leave out the per-instance loop (profiling)")
    ap.add_argument("--batch", type=int, default=4096, help="instances for --workload batch")
    ap.add_argument("--serve-requests", type=int, default=10000, help="requests for --workload serve")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="mean arrivals per second (serve)")
    ap.add_argument("--balance-n", type=int, default=1_000_000_000, help="keys per distribution (balance)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU "
              f"exchange (the distributed form is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        a = torch.ones(args.copy_calibration // 8, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": a.numel() * 8}))
        return

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "balance":
        return bench_balance(args)
    if args.workload == "search":
        return bench_search(args)
    w = WORKLOADS[args.workload]
    cpu = None
    if not args.no_cpu:
        # before the GPU is touched: the oracle's worker processes start from a
        # process that has not initialised the device
        print("[bench] timing the CPU oracle on samples", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, min(args.cpu_sample, w["n"]), min(args.cpu_sample_one, w["n"]))
    torch.cuda.set_device(torch.device("cuda:0"))
    m = measure_sort(w, args, args.steps, args.warmup, tune=not args.no_tune)
    roof, pipe, kernels = summarize_sort(w, m, args.steps)
    line = {
        "metric": METRIC, "value": round(m["value"], 4), "unit": "GKeys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(m["ms"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": m["dtype"], "data": "synthetic",
        "config": {"workload": w["desc"], "n": w["n"], "P": w["P"], "s": w["s"], "key": m["dtype"],
                   "value": {True: "u32", "index": "u32 index (generated)", False: None}[w["vals"]],
                   "investigator": "COUNT", "handler": {1: "passes", 2: "one pass"}[m["settings"]["handler"]],
                   "fanin": m["settings"]["fanin"], "merge_tile": m["settings"]["merge_tile"],
                   "radix_tile": m["settings"]["radix_tile"], "autotuned": m["autotuned"]},
        "imbalance": m["imbalance"],
        "roofline": roof,
        "pipeline": pipe,
        "profiled_ms_per_step": round(m["ms_prof"], 4),
        "kernels": kernels,
    }
    if args.workload == "pairs" and not args.no_extras:
        wd = WORKLOADS["dups"]
        md = measure_sort(wd, args, max(3, args.steps // 2), 1, tune=not args.no_tune)
        rd, pd, _ = summarize_sort(wd, md, max(3, args.steps // 2))
        line["dups"] = {"workload": wd["desc"], "value": round(md["value"], 4), "unit": "GKeys/s",
                        "ms_per_step": round(md["ms"], 4), "imbalance": md["imbalance"],
                        "settings": md["settings"], "autotuned": md["autotuned"],
                        "roofline": {k: rd[k] for k in ("kernel", "achieved", "frac", "avg_launch_ms", "traffic")},
                        "pipeline": {k: pd[k] for k in ("executed_bytes_per_key", "executed_frac", "model_frac")}}
        line["batched"] = run_batch(args, max(3, args.steps // 2), 1, tune=not args.no_tune)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
