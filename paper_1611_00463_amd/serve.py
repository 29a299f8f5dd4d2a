"""Serving loop: continuous batching of sort requests on one GPU.

Requests arrive over time (each: a size, a key distribution, an offset into a
device-resident key pool of that distribution).  The scheduler

* admits waiting requests in arrival order while their memory fits the HBM
  budget (output, staging copy of the input and workspace);
* whenever one of S streams is free, launches every admitted request that is
  not yet running as ONE lbsort_sort_batch call on that stream (the batched
  form of Section IV.C), so requests that arrive while others run join the
  next batch and batches on different streams overlap on the device;
* polls completion events, records each request's latency (arrival to
  completion), releases its memory and admits more.

Keys are u64 and every request is sorted with the same P and sample budget.
Results stay on the device; a request's sorted keys and partition offsets
are identical to sorting it alone (the batch is instance-wise independent).
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import lbsort as L

KEY_BYTES = 8
BYTES_PER_KEY = 3 * KEY_BYTES + 8  # staging input, output, workspace (+ metadata slack)


@dataclass
class Request:
    rid: int
    arrival: float      # seconds from the start of the run
    n: int
    dist: int
    offset: int
    t_done: float = -1.0
    error: int = 0      # device error bits of the request's batch (0 = none)
    keys_out: torch.Tensor | None = None
    part_offsets: torch.Tensor | None = None


@dataclass
class _Batch:
    reqs: list
    stream: torch.cuda.Stream
    done: torch.cuda.Event
    bytes: int
    keep: list = field(default_factory=list)
    err: torch.Tensor | None = None   # pinned host copy of the batch's device error word


class Server:
    def __init__(self, pools: list[torch.Tensor], P: int = 64, s: int = 0, budget_bytes: int = 64 << 30,
                 streams: int = 4, max_batch_keys: int = 1 << 28, max_batch: int = 512, keep_outputs=False,
                 keep_ids=None):
        """keep_outputs: keep a copy of every request's sorted keys and
        partition offsets; keep_ids: only of the requests with these ids."""
        self.pools = pools
        self.P, self.s = P, s
        self.budget = budget_bytes
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.max_batch_keys = max_batch_keys
        self.max_batch = max_batch
        self.keep_outputs = keep_outputs
        self.keep_ids = None if keep_ids is None else set(keep_ids)
        self.lib = L.load()

    def request_bytes(self, n: int) -> int:
        return BYTES_PER_KEY * n + 64 * (self.P + 1) * 8

    def _launch(self, reqs: list[Request], stream: torch.cuda.Stream) -> _Batch:
        sizes = [r.n for r in reqs]
        offs = np.zeros(len(reqs) + 1, dtype=np.int64)
        offs[1:] = np.cumsum(sizes)
        total = int(offs[-1])
        with torch.cuda.stream(stream):
            keys = torch.empty(total, dtype=torch.uint64, device="cuda")
            for r, a in zip(reqs, offs[:-1]):
                keys[a:a + r.n].view(torch.int64).copy_(self.pools[r.dist][r.offset:r.offset + r.n].view(torch.int64),
                                                         non_blocking=True)
            seg = torch.from_numpy(offs.astype(np.uint64)).pin_memory().to("cuda", non_blocking=True)
            res = L.sort_batch(keys, seg, self.P, s=self.s)
            # the error word the sort latched (first word of its workspace),
            # copied to host memory in stream order, read once the batch is done
            err = torch.empty(1, dtype=torch.int32, pin_memory=True)
            err.copy_(res.workspace[:4].view(torch.int32), non_blocking=True)
            done = torch.cuda.Event()
            done.record(stream)
        b = _Batch(reqs, stream, done, sum(self.request_bytes(n) for n in sizes), keep=[keys, seg, res], err=err)
        b.offs = offs
        return b

    def _collect(self, b: _Batch, t: float):
        """A finished batch: latency, device errors, and the copies of the kept
        outputs.  The copies run on the batch's own stream: its buffers go back
        to that stream's pool once the batch is dropped and may be reused by its
        next batch, which is ordered after these copies."""
        err = int(b.err[0])
        with torch.cuda.stream(b.stream):
            for k, r in enumerate(b.reqs):
                r.t_done = t
                r.error = err
                if self.keep_outputs or (self.keep_ids is not None and r.rid in self.keep_ids):
                    a, e = int(b.offs[k]), int(b.offs[k + 1])
                    r.keys_out = b.keep[2].keys[a:e].clone()
                    r.part_offsets = b.keep[2].part_offsets[k].clone()

    def run(self, requests: list[Request], verbose=False):
        """Serve the requests in real time; returns them with t_done filled in."""
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting: list[Request] = []
        inflight: dict[int, _Batch] = {}
        used = 0
        i = 0
        t0 = time.perf_counter()
        free = list(range(len(self.streams)))
        n_done = 0
        while n_done < len(requests):
            now = time.perf_counter() - t0
            while i < len(pending) and pending[i].arrival <= now:
                waiting.append(pending[i])
                i += 1
            # completions
            for si in list(inflight):
                b = inflight[si]
                if b.done.query():
                    self._collect(b, time.perf_counter() - t0)
                    used -= b.bytes
                    n_done += len(b.reqs)
                    del inflight[si]
                    free.append(si)
            # admit and launch on a free stream
            if free and waiting:
                take, keys_in_batch, extra = [], 0, 0
                while waiting and len(take) < self.max_batch:
                    r = waiting[0]
                    need = self.request_bytes(r.n)
                    if used + extra + need > self.budget and (take or inflight):
                        break
                    if take and keys_in_batch + r.n > self.max_batch_keys:
                        break
                    take.append(waiting.pop(0))
                    keys_in_batch += r.n
                    extra += need
                if take:
                    si = free.pop(0)
                    inflight[si] = self._launch(take, self.streams[si])
                    used += inflight[si].bytes
                    continue
            if not inflight and i < len(pending) and not waiting:
                time.sleep(max(0.0, min(0.0005, pending[i].arrival - (time.perf_counter() - t0))))
            else:
                time.sleep(20e-6)
        torch.cuda.synchronize()
        return requests


def run_per_request(pools, requests: list[Request], P: int = 64, s: int = 0):
    """Baseline: one lbsort_sort_keys call per request, in arrival order, one
    stream, each started when it has arrived and the previous one finished."""
    ws = L.Workspace("cuda")
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: r.arrival):
        while time.perf_counter() - t0 < r.arrival:
            time.sleep(20e-6)
        res = L.sort_keys(pools[r.dist][r.offset:r.offset + r.n], P, s=s, workspace=ws)
        ev = torch.cuda.Event()
        ev.record()
        ev.synchronize()
        r.t_done = time.perf_counter() - t0
        del res
    return requests


def make_requests(n_req: int, seed: int, pool_n: int, rate: float, lo: int, hi: int) -> list[Request]:
    from . import datagen
    arr, sizes, dists = datagen.serve_requests(n_req, seed, rate, lo, hi)
    sizes = np.minimum(sizes, pool_n)
    offs = (datagen.u64_range(seed + 9, 0, n_req) % np.uint64(1 << 62)).astype(np.int64) % (pool_n - sizes + 1)
    return [Request(k, float(arr[k]), int(sizes[k]), int(dists[k]), int(offs[k])) for k in range(n_req)]


def summarize(reqs: list[Request], wall: float) -> dict:
    lat = np.array([r.t_done - r.arrival for r in reqs]) * 1e3
    keys = sum(r.n for r in reqs)
    return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3), "GKeys_s": round(keys / wall / 1e9, 4),
            "requests": len(reqs), "keys": int(keys), "wall_s": round(wall, 3),
            "device_errors": sum(1 for r in reqs if r.error)}
