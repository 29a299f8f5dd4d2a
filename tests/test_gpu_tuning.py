"""The autotuner (radix tile, handler fan-in, merge tile) on the device: it
runs on a caller's batch, writes its cache (keyed by the architecture), the
chosen settings are what later calls of that shape use, and they give the
same bytes as the defaults and as the oracle."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import sample_sort as O
from paper_1611_00463_amd import datagen
from paper_1611_00463_amd import lbsort as L

pytestmark = pytest.mark.gpu


def test_autotune_on_a_batch_and_use_it(tmp_path):
    B, P = 48, 8
    keys, vals, seg, sizes = datagen.batch_u32_torch(B, 31, lo=1024, hi=300_000, device="cuda")
    total = int(sizes.sum())
    print(f"[tuning] batch of {B} instances, {total} keys", flush=True)
    path = str(tmp_path / "tune.json")
    before = L.resolve_params(L.U32, L.VAL_U32, P, total, B=B)
    chosen = L.autotune(L.U32, L.VAL_U32, P, keys=keys, vals=vals, seg_offsets=seg, cache_path=path)
    assert chosen["radix_tile"] in (4096, 8192, 16384)  # 16384 only for 32-bit keys
    assert chosen["fanin"] in (2, 4, 8) and chosen["merge_tile"] in (1024, 2048, 4096)
    # the cache file holds the entry, keyed by the device architecture
    entries = json.load(open(path))["entries"]
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    mine = [e for e in entries if e["arch"] == arch and e["P"] == P and e["batched"] == 1 and e["key_bytes"] == 4]
    assert len(mine) == 1 and mine[0]["radix_tile"] == chosen["radix_tile"]
    assert mine[0]["fanin"] == chosen["fanin"] and mine[0]["merge_tile"] == chosen["merge_tile"]
    assert L.load().lbsort_load_tuning(path.encode()) == 0
    # later calls of this shape run with the chosen settings
    after = L.resolve_params(L.U32, L.VAL_U32, P, total, B=B)
    assert {k: after[k] for k in chosen} == chosen, (before, after, chosen)
    # and give the same bytes as explicit defaults, and as the oracle
    tuned = L.BatchPlan(keys, seg, P, vals=vals)
    tuned.run()
    tuned.check()
    dflt = L.BatchPlan(keys, seg, P, vals=vals, fanin=8, merge_tile=2048, radix_tile=8192)
    dflt.run()
    dflt.check()
    i32 = lambda t: t.view(torch.int32)
    assert torch.equal(i32(tuned.keys_out), i32(dflt.keys_out))
    assert torch.equal(i32(tuned.vals_out), i32(dflt.vals_out))
    assert torch.equal(tuned.part_offsets, dflt.part_offsets)
    offs = seg.cpu().numpy().astype(np.int64)
    kin, vin = keys.cpu().numpy(), vals.cpu().numpy()
    for b in (0, 7, int(np.argmax(sizes)), B - 1):
        a, e = offs[b], offs[b + 1]
        o = O.sample_sort(kin[a:e], vin[a:e], P)
        np.testing.assert_array_equal(tuned.keys_out[a:e].cpu().numpy(), o.keys)
        np.testing.assert_array_equal(tuned.vals_out[a:e].cpu().numpy(), o.vals)
        np.testing.assert_array_equal(tuned.part_offsets[b].cpu().numpy().view(np.uint64),
                                      o.part_offsets.astype(np.uint64))


def test_autotune_synthetic_single_instance(tmp_path):
    path = str(tmp_path / "tune1.json")
    chosen = L.autotune(L.U64, L.VAL_U32, 64, total_n=1 << 21, B=1, cache_path=path)
    assert chosen["radix_tile"] in (4096, 8192) and chosen["fanin"] in (2, 4, 8, 16)
    r = L.resolve_params(L.U64, L.VAL_U32, 64, 1 << 21)
    assert {k: r[k] for k in chosen} == chosen
    # a typed key of the same width shares the entry
    r = L.resolve_params(L.F64, L.VAL_INDEX, 64, 1 << 21)
    assert {k: r[k] for k in chosen} == chosen
    assert os.path.getsize(path) > 0
