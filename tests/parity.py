"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare every output with the CPU oracle, element by element."""
from __future__ import annotations

import numpy as np
import torch

from oracle import sample_sort as O
from paper_1611_00463_amd import lbsort as L


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()


def u64(t: torch.Tensor) -> np.ndarray:
    return to_host(t).view(np.uint64) if t.dtype == torch.int64 else to_host(t)


def run_gpu(keys, vals, P, s=0, mode=O.INV_COUNT, fanin=0, tile=0, ws=None, rtile=0, handler=0):
    kd = to_dev(keys)
    if vals is None:
        r = L.sort_keys(kd, P, s=s, investigator=mode, fanin=fanin, merge_tile=tile, want_send=True,
                        want_cuts=True, workspace=ws, radix_tile=rtile, handler=handler)
    else:
        r = L.sort_pairs(kd, to_dev(vals), P, s=s, investigator=mode, fanin=fanin, merge_tile=tile,
                         want_send=True, want_cuts=True, workspace=ws, radix_tile=rtile, handler=handler)
    L.check(r.workspace)
    return r


def assert_same(name, got, want):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, f"{name}: shape {got.shape} != {want.shape}"
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got.reshape(-1) != want.reshape(-1))
        raise AssertionError(f"{name}: {len(bad)} of {got.size} differ; first at {bad[:5]}: "
                             f"got {got.reshape(-1)[bad[:5]]} want {want.reshape(-1)[bad[:5]]}")


def compare(r: L.SortResult, o: O.SortResult, P: int, b: int = 0, seg=None):
    """Bit-exact comparison of one instance's outputs."""
    a, e = (0, len(o.keys)) if seg is None else seg
    assert_same("keys", to_host(r.keys)[a:e], o.keys)
    if o.vals is not None:
        assert_same("vals", to_host(r.vals)[a:e], o.vals)
    assert_same("part_offsets", u64(r.part_offsets)[b], o.part_offsets.astype(np.uint64))
    assert_same("part_counts", u64(r.part_counts)[b], o.part_counts.astype(np.uint64))
    if P > 1:
        assert_same("splitters", to_host(r.splitters)[b], o.splitters)
    if r.send_counts is not None:
        assert_same("send_counts", u64(r.send_counts)[b], o.send_counts.astype(np.uint64))
    if r.cuts is not None:
        assert_same("cuts", u64(r.cuts)[b], o.cuts.astype(np.uint64))


def check_case(keys, vals, P, s=0, mode=O.INV_COUNT, fanin=0, tile=0, ws=None, rtile=0, handler=0):
    o = O.sample_sort(keys, vals, P, s, mode)
    r = run_gpu(keys, vals, P, s, mode, fanin, tile, ws, rtile, handler)
    compare(r, o, P)
    return r, o
