"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (2^28 keys, P = 64, 512 samples per block, default fan-in and tile).

The whole oracle merge would take minutes on the CPU, so:
* the partition metadata (splitters, cut matrix, send counts, offsets) is
  computed by the oracle's own step functions and compared bit for bit;
* the sorted output is checked by properties that pin it uniquely: keys
  non-decreasing, (key, value) pairs a permutation of the input (values are
  the input indices), and equal keys in increasing index order (stable);
  for keys only, the multiset of keys is compared instead.
"""
import numpy as np
import pytest
import torch

from oracle import sample_sort as O
from paper_1611_00463_amd import datagen
from paper_1611_00463_amd import lbsort as L
from tests.parity import assert_same, u64

pytestmark = pytest.mark.gpu

N = 1 << 28
P, S = 64, 512
SIGN = -(1 << 63)


def signed(t):
    """Order-preserving view of uint64 as int64 (flip the top bit)."""
    return t.view(torch.int64) ^ SIGN


def check_metadata(r, keys_np, mode=O.INV_COUNT):
    plan = O.partition_plan(keys_np, P, S, mode)
    assert_same("splitters", r.splitters.cpu().numpy()[0], plan["splitters"])
    assert_same("cuts", u64(r.cuts)[0], plan["cuts"].astype(np.uint64))
    assert_same("send_counts", u64(r.send_counts)[0], plan["send_counts"].astype(np.uint64))
    assert_same("part_offsets", u64(r.part_offsets)[0], plan["part_offsets"].astype(np.uint64))
    return plan


def test_pairs_full_size():
    keys = datagen.uniform_keys_torch(N, 2, "cuda")
    vals = datagen.index_values_torch(N, "cuda")
    r = L.sort_pairs(keys, vals, P, s=S, want_send=True, want_cuts=True)
    L.check(r.workspace)
    ko, vo = signed(r.keys), r.vals.view(torch.int32).to(torch.int64)
    assert bool((ko[1:] >= ko[:-1]).all()), "keys not sorted"
    assert bool((torch.bincount(vo, minlength=N) == 1).all()), "values are not a permutation"
    assert bool((r.keys.view(torch.int64) == keys.view(torch.int64)[vo]).all()), "pairs broken"
    eq = ko[1:] == ko[:-1]
    assert bool((vo[1:][eq] > vo[:-1][eq]).all()), "not stable"
    del ko, vo, eq
    check_metadata(r, keys.cpu().numpy())
    counts = r.part_counts.cpu().numpy()[0]
    assert counts.max() / counts.mean() <= 1.05


def test_duplicate_heavy_full_size():
    keys_np = datagen.duplicate_heavy_keys(N, seed=3)
    keys = torch.from_numpy(keys_np).cuda()
    r = L.sort_keys(keys, P, s=S, want_send=True, want_cuts=True)
    L.check(r.workspace)
    ko = signed(r.keys)
    assert bool((ko[1:] >= ko[:-1]).all()), "keys not sorted"
    ui, ci = torch.unique(signed(keys), return_counts=True)
    uo, co = torch.unique_consecutive(ko, return_counts=True)
    assert torch.equal(ui, uo) and torch.equal(ci, co), "output is not a permutation of the input"
    plan = check_metadata(r, keys_np)
    counts = plan["part_counts"]
    assert counts.max() / counts.mean() <= 1.05, "investigator lost the balance"


def test_f64_index_values_full_size():
    """2^28 normal-like doubles with NaNs, infinities and signed zeros, and
    generated index values: the float workload of bench.py.  Most blocks take
    the mid-size group fix-up.  Partition metadata against the oracle (on the
    keys' totalOrder integers); the output by properties that pin it: keys
    in totalOrder, index values a permutation, each output key the input key
    at its index, equal keys in increasing index order."""
    from oracle import typed as T
    keys = datagen.typed_keys_torch(N, 21, np.float64, "cuda")
    r = L.sort_pairs(keys, None, P, s=S, want_send=True, want_cuts=True)
    L.check(r.workspace)
    bits = r.keys.view(torch.int64)
    # totalOrder as a signed integer: negative patterns reversed
    tko = torch.where(bits < 0, bits ^ 0x7FFFFFFFFFFFFFFF, bits)
    assert bool((tko[1:] >= tko[:-1]).all()), "keys not in totalOrder"
    vo = r.vals.view(torch.int32).to(torch.int64)
    assert bool((torch.bincount(vo, minlength=N) == 1).all()), "index values are not a permutation"
    assert bool((bits == keys.view(torch.int64)[vo]).all()), "an output key is not the input key at its index"
    eq = tko[1:] == tko[:-1]
    assert bool((vo[1:][eq] > vo[:-1][eq]).all()), "not stable"
    del tko, vo, eq, bits
    keys_np = keys.cpu().numpy()
    plan = O.partition_plan(T.total_order_int(keys_np), P, S)
    assert_same("splitters", T.total_order_int(r.splitters.cpu().numpy()[0]), plan["splitters"])
    assert_same("cuts", u64(r.cuts)[0], plan["cuts"].astype(np.uint64))
    assert_same("send_counts", u64(r.send_counts)[0], plan["send_counts"].astype(np.uint64))
    assert_same("part_offsets", u64(r.part_offsets)[0], plan["part_offsets"].astype(np.uint64))


def test_search_and_provenance_full_size():
    """Search and provenance at the benchmark's size, by properties that fix
    them: each position p satisfies sorted[p-1] < q <= sorted[p] (lower
    bound; <= and < for the upper bound), each partition index k satisfies
    G_k <= p < G_{k+1}; each source index splits into a block whose range
    holds it and the offset inside that range."""
    keys = datagen.uniform_keys_torch(N, 2, "cuda")
    r = L.sort_pairs(keys, None, P, s=S)
    L.check(r.workspace)
    sk = signed(r.keys)
    G = r.part_offsets[0].contiguous()
    nq = 1 << 22
    pick = datagen.u64_torch(40, 0, nq // 2, "cuda").view(torch.int64).remainder(N)
    q = torch.cat([r.keys.view(torch.int64)[pick], datagen.u64_torch(41, 0, nq - nq // 2, "cuda").view(torch.int64)])
    qs = q ^ SIGN
    for upper in (False, True):
        pos, part = L.search(r.keys, q.view(torch.uint64), upper, G)
        below = sk[(pos - 1).clamp(min=0)]
        at = sk[pos.clamp(max=N - 1)]
        ok_lo = (pos == 0) | ((below <= qs) if upper else (below < qs))
        ok_hi = (pos == N) | ((at > qs) if upper else (at >= qs))
        assert bool((ok_lo & ok_hi).all()), "search positions inconsistent with the sorted keys"
        k = part.view(torch.int32).to(torch.int64)
        inside = pos < N
        kk = k[inside]
        assert bool(((G[kk] <= pos[inside]) & (pos[inside] < G[kk + 1])).all()), "partition of a position"
        assert bool((k[~inside] == P).all()), "past-the-end positions belong to no partition"
    blk, off = L.provenance(r.vals, N, P)
    g = r.vals.view(torch.int32).to(torch.int64)
    b = blk.view(torch.int32).to(torch.int64)
    start = (b * N) // P
    end = ((b + 1) * N) // P
    assert bool(((start <= g) & (g < end)).all()), "source block does not hold the index"
    assert bool((off.view(torch.int32).to(torch.int64) == g - start).all()), "offset inside the block"
