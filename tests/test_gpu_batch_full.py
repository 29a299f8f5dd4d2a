"""Parity of the batched form at its configured shape, in the launch
configuration bench.py times: 4,096 uint32 key-value instances with sizes
log-uniform in [1K, 4M] (about 2.03e9 keys), keys uniform / normal / sorted /
reverse, P = 8, one lbsort_sort_batch call replayed from a HIP graph.

* every instance, on the device: keys non-decreasing, (key, value) pairs a
  permutation of the instance's input (values are local input positions),
  equal keys in increasing position order (stable), partition offsets
  monotone from 0 to the instance size;
* sampled instances (the largest among them) element by element against the
  oracle, and the partition offsets of more of them against the oracle's
  step functions.
"""
import numpy as np
import pytest
import torch

from oracle import sample_sort as O
from paper_1611_00463_amd import datagen
from paper_1611_00463_amd import lbsort as L

pytestmark = pytest.mark.gpu

B, P = 4096, 8


def test_batch_config_full_shape():
    print("[batch-full] generating 4096 instances", flush=True)
    keys, vals, seg, sizes = datagen.batch_u32_torch(B, 4, device="cuda")
    total = int(sizes.sum())
    plan = L.BatchPlan(keys, seg, P, vals=vals)
    plan.capture()
    for _ in range(2):
        plan.replay()
    torch.cuda.synchronize()
    plan.check()
    print(f"[batch-full] sorted {total} keys; checking every instance", flush=True)
    seg64 = seg.view(torch.int64)
    kin = keys.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    seen = torch.zeros(total, dtype=torch.int32, device="cuda")
    CH = 1 << 27
    for a in range(0, total, CH):
        e = min(total, a + CH)
        idx = torch.arange(a, e, device="cuda", dtype=torch.int64)
        seg_of = torch.searchsorted(seg64, idx, right=True) - 1
        ko = plan.keys_out[a:e].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        vo = plan.vals_out[a:e].view(torch.int32).to(torch.int64)
        n_of = seg64[seg_of + 1] - seg64[seg_of]
        assert bool(((vo >= 0) & (vo < n_of)).all()), "value outside its instance"
        src = seg64[seg_of] + vo
        assert bool((kin[src] == ko).all()), "pairs broken"
        seen.index_add_(0, src, torch.ones_like(src, dtype=torch.int32))
        same = seg_of[1:] == seg_of[:-1]
        assert bool((ko[1:][same] >= ko[:-1][same]).all()), "not sorted within an instance"
        eq = same & (ko[1:] == ko[:-1])
        assert bool((vo[1:][eq] > vo[:-1][eq]).all()), "not stable"
        del idx, seg_of, ko, vo, n_of, src, same, eq
    # chunk edges: the last key of a chunk and the first of the next
    edges = torch.arange(CH, total, CH, device="cuda")
    if edges.numel():
        s_of = torch.searchsorted(seg64, edges, right=True) - 1
        s_prev = torch.searchsorted(seg64, edges - 1, right=True) - 1
        ko = plan.keys_out.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        inside = s_of == s_prev
        assert bool((ko[edges][inside] >= ko[edges - 1][inside]).all())
        del ko
    assert bool((seen == 1).all()), "values are not a permutation inside their instances"
    del seen
    G = plan.part_offsets.cpu().numpy().view(np.uint64).astype(np.int64)
    assert (G[:, 0] == 0).all() and (G[:, -1] == sizes).all() and (np.diff(G, axis=1) >= 0).all()
    # sampled instances against the oracle
    offs = seg.cpu().numpy().astype(np.int64)
    rng = np.random.default_rng(4)
    order = np.argsort(sizes)
    full = sorted(set([int(order[-1]), int(order[-2]), int(order[len(order) // 2]), int(order[0])] +
                      [int(x) for x in rng.choice(B, 20, replace=False)]))
    meta = sorted(set(full) | set(int(x) for x in rng.choice(B, 40, replace=False)))
    print(f"[batch-full] {len(full)} instances against the whole oracle, {len(meta)} against its partition plan",
          flush=True)
    for b in meta:
        a, e = offs[b], offs[b + 1]
        kb = plan.keys[a:e].cpu().numpy()
        if b in full:
            o = O.sample_sort(kb, plan.vals[a:e].cpu().numpy(), P)
            np.testing.assert_array_equal(plan.keys_out[a:e].cpu().numpy(), o.keys, err_msg=f"instance {b} keys")
            np.testing.assert_array_equal(plan.vals_out[a:e].cpu().numpy(), o.vals, err_msg=f"instance {b} values")
            want = o.part_offsets
        else:
            want = O.partition_plan(kb, P)["part_offsets"]
        np.testing.assert_array_equal(G[b], want.astype(np.int64), err_msg=f"instance {b} partition offsets")
