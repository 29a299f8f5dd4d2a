"""The batched form captured into a HIP graph: every replay, with eager work
and synchronisations in between, must reproduce the eager result and the
oracle, instance by instance."""
import numpy as np
import pytest
import torch

from oracle import sample_sort as O
from paper_1611_00463_amd import datagen
from paper_1611_00463_amd import lbsort as L
from tests.parity import to_dev, to_host, u64

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager_and_oracle():
    keys, vals, seg, sizes = datagen.batch_u32_torch(24, seed=4, lo=1024, hi=200_000, device="cuda")
    plan = L.BatchPlan(keys, seg, 8, vals=vals)
    plan.run()
    torch.cuda.synchronize()
    plan.check()
    i32 = lambda t: t.view(torch.int32)
    want_k, want_v = i32(plan.keys_out).clone(), i32(plan.vals_out).clone()
    want_o = plan.part_offsets.clone()
    plan.capture()
    for i in range(4):
        i32(plan.keys_out).zero_()
        i32(plan.vals_out).zero_()
        plan.part_offsets.zero_()
        torch.cuda.synchronize()
        plan.replay()
        torch.cuda.synchronize()
        plan.check()
        assert torch.equal(i32(plan.keys_out), want_k), f"replay {i}: keys differ"
        assert torch.equal(i32(plan.vals_out), want_v), f"replay {i}: values differ"
        assert torch.equal(plan.part_offsets, want_o), f"replay {i}: offsets differ"
        _ = torch.randn(1000, device="cuda").sum().item()   # eager work between replays
    hk, hv, ho = to_host(keys), to_host(vals), to_host(seg).astype(np.int64)
    ko, vo, po = to_host(want_k).view(np.uint32), to_host(want_v).view(np.uint32), u64(want_o)
    for b in range(len(sizes)):
        a, e = int(ho[b]), int(ho[b + 1])
        o = O.sample_sort(hk[a:e], hv[a:e], 8)
        np.testing.assert_array_equal(ko[a:e], o.keys)
        np.testing.assert_array_equal(vo[a:e], o.vals)
        np.testing.assert_array_equal(po[b], o.part_offsets.astype(np.uint64))
