"""Serving: requests batched together while others run give the same bytes
as each request sorted alone (and as the oracle)."""
import numpy as np
import pytest
import torch

from oracle import sample_sort as O
from paper_1611_00463_amd import datagen
from paper_1611_00463_amd import lbsort as L
from paper_1611_00463_amd import serve as S

pytestmark = pytest.mark.gpu


def test_same_alone_and_in_the_mix():
    pool_n = 1 << 20
    pools = [datagen.serve_pool_u64_torch(d, pool_n, 5, "cuda") for d in range(4)]
    reqs = S.make_requests(60, seed=7, pool_n=pool_n, rate=50000.0, lo=1000, hi=300_000)
    srv = S.Server(pools, P=64, budget_bytes=64 << 20, streams=3, max_batch=16, keep_outputs=True)
    srv.run(reqs)
    assert all(r.t_done >= r.arrival for r in reqs)
    assert all(r.error == 0 for r in reqs)
    for k, r in enumerate(reqs):
        alone = L.sort_keys(pools[r.dist][r.offset:r.offset + r.n], 64)
        L.check(alone.workspace)
        assert torch.equal(alone.keys.view(torch.int64), r.keys_out.view(torch.int64)), f"request {k}: keys"
        assert torch.equal(alone.part_offsets[0], r.part_offsets), f"request {k}: partition offsets"
        # and every request against the oracle
        src = pools[r.dist][r.offset:r.offset + r.n].cpu().numpy()
        o = O.sample_sort(src, None, 64)
        np.testing.assert_array_equal(r.keys_out.cpu().numpy(), o.keys)
        np.testing.assert_array_equal(r.part_offsets.cpu().numpy().view(np.uint64), o.part_offsets.astype(np.uint64))


def test_budget_smaller_than_one_request_still_serves():
    pool_n = 1 << 16
    pools = [datagen.serve_pool_u64_torch(d, pool_n, 5, "cuda") for d in range(4)]
    reqs = S.make_requests(6, seed=8, pool_n=pool_n, rate=1000.0, lo=20_000, hi=60_000)
    srv = S.Server(pools, P=8, budget_bytes=1024, streams=2, keep_outputs=True)
    srv.run(reqs)
    for r in reqs:
        alone = L.sort_keys(pools[r.dist][r.offset:r.offset + r.n], 8)
        assert torch.equal(alone.keys.view(torch.int64), r.keys_out.view(torch.int64))


class _BusyDefaultStream(S.Server):
    """Before each finished batch is collected, the default stream is given a
    few milliseconds of unrelated work, so anything the collection enqueued
    there would run only after the next batch on the batch's own stream."""

    def __init__(self, *a, **kw):
        super().__init__(*a, **kw)
        self._x = torch.empty(64 << 20, dtype=torch.int32, device="cuda")
        self._y = torch.empty_like(self._x)

    def _collect(self, b, t):
        for _ in range(16):
            self._y.copy_(self._x)
        super()._collect(b, t)


def test_kept_outputs_survive_buffer_reuse():
    """Regression test of the kept-output copies: one stream, one request per
    batch, every request the same size, all arriving at once, so each batch
    reuses the buffers the previous one released, and the default stream is
    kept busy whenever outputs are copied.  The copies must be ordered before
    the next batch on the batch's stream and give each request's own result."""
    pool_n = 1 << 20
    pools = [datagen.serve_pool_u64_torch(d, pool_n, 5, "cuda") for d in range(4)]
    reqs = S.make_requests(12, seed=9, pool_n=pool_n, rate=1e9, lo=200_000, hi=200_001)
    for k, r in enumerate(reqs):
        r.n, r.arrival, r.dist, r.offset = 200_000, 0.0, k % 4, (k * 37_003) % (pool_n - 200_000)
    srv = _BusyDefaultStream(pools, P=16, budget_bytes=64 << 30, streams=1, max_batch=1, keep_outputs=True)
    srv.run(reqs)
    for k, r in enumerate(reqs):
        assert r.error == 0
        alone = L.sort_keys(pools[r.dist][r.offset:r.offset + r.n], 16)
        L.check(alone.workspace)
        assert torch.equal(alone.keys.view(torch.int64), r.keys_out.view(torch.int64)), f"request {k}: keys"
        assert torch.equal(alone.part_offsets[0], r.part_offsets), f"request {k}: partition offsets"
