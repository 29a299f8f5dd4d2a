"""GPU parity of the one-pass handler (all P runs of a partition merged at
once, tiles bounded by regular samples of the runs) against the oracle, bit
for bit on every output, and against the multi-pass handler: P from 2 to 64
(powers of two and not), both tile capacities, ragged and tiny inputs, heavy
duplicates in every investigator mode, all-equal, sorted and reverse inputs,
and batches of uneven instances."""
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import sample_sort as O
from paper_1611_00463_amd import datagen
from paper_1611_00463_amd import lbsort as L
from tests.parity import check_case, compare, run_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu
ONE = L.HANDLER_ONE_PASS


@pytest.fixture(scope="module")
def ws():
    return L.Workspace("cuda")


@pytest.mark.parametrize("tile", [2048, 4096])
@pytest.mark.parametrize("P", [2, 3, 8, 13, 17, 32, 37, 64])
def test_one_pass_uniform_pairs(ws, P, tile):
    n = 1_000_003
    print(f"[one-pass] P={P} tile={tile}", flush=True)
    keys = datagen.uniform_keys(n, seed=P * 7 + tile)
    check_case(keys, datagen.index_values(n), P, 0, ws=ws, tile=tile, handler=ONE)


@pytest.mark.parametrize("mode", [O.INV_COUNT, O.INV_NONE, O.INV_PAPER])
@pytest.mark.parametrize("P", [37, 64])
def test_one_pass_duplicate_heavy(ws, P, mode):
    n = 1_500_007
    keys = datagen.duplicate_heavy_keys(n, seed=3)
    check_case(keys, datagen.index_values(n), P, 512, mode=mode, ws=ws, handler=ONE)
    check_case(keys, None, P, 0, mode=mode, ws=ws, tile=2048, handler=ONE)


@pytest.mark.parametrize("n", [0, 1, 2, 63, 100, 4095, 4097, 8193, 50_000])
@pytest.mark.parametrize("P", [2, 17, 64])
def test_one_pass_small_and_ragged(ws, n, P):
    keys = datagen.uniform_keys(n, seed=n + 31 * P)
    keys[::3] = keys[0] if n else keys[::3]
    check_case(keys, datagen.index_values(n), P, 4, ws=ws, handler=ONE)


def test_one_pass_all_equal_sorted_reverse(ws):
    n = 600_001
    check_case(np.full(n, 7, dtype=np.uint64), datagen.index_values(n), 64, 0, ws=ws, handler=ONE)
    check_case(np.full(n, 7, dtype=np.uint64), datagen.index_values(n), 64, 0, mode=O.INV_NONE, ws=ws, handler=ONE)
    srt = np.sort(datagen.uniform_keys(n, seed=9))
    check_case(srt, datagen.index_values(n), 33, 8, ws=ws, handler=ONE)
    check_case(srt[::-1].copy(), datagen.index_values(n), 64, 8, ws=ws, handler=ONE)
    k32 = np.sort(datagen.uniform_keys(n, seed=10, dtype=np.uint32))[::-1].copy()
    check_case(k32, None, 40, 0, ws=ws, handler=ONE)
    check_case(datagen.normal_u32(n, seed=6), datagen.index_values(n), 64, 0, ws=ws, handler=ONE)


def test_one_pass_equals_passes(ws):
    """The same bytes from both handler schedules, on every output."""
    n = 1 << 22
    keys = datagen.uniform_keys(n, seed=77)
    vals = datagen.index_values(n)
    a = run_gpu(keys, vals, 64, 0, ws=ws, handler=ONE)
    ka, va = to_host(a.keys).copy(), to_host(a.vals).copy()
    offs, cuts = to_host(a.part_offsets).copy(), to_host(a.cuts).copy()
    for h, f in ((L.HANDLER_PASSES, 8), (L.HANDLER_PASSES, 4)):
        b = run_gpu(keys, vals, 64, 0, ws=ws, handler=h, fanin=f)
        assert np.array_equal(ka, to_host(b.keys)) and np.array_equal(va, to_host(b.vals))
        assert np.array_equal(offs, to_host(b.part_offsets)) and np.array_equal(cuts, to_host(b.cuts))


@pytest.mark.parametrize("P", [5, 8, 33, 64])
def test_one_pass_batch(ws, P):
    """Uneven instances (empty ones among them) sorted at once with the one-pass
    handler, each against its own oracle run."""
    sizes = [0, 1, 5, 4096, 4097, 10_000, 123_457, 0, 33, 250_000, 3, 65_536, 300_001]
    rng = np.random.default_rng(P)
    parts_k = []
    for i, n in enumerate(sizes):
        if i % 3 == 0:
            parts_k.append(datagen.uniform_keys(n, seed=200 + i))
        elif i % 3 == 1:
            parts_k.append(np.sort(datagen.uniform_keys(n, seed=200 + i)))
        else:
            parts_k.append(rng.integers(0, 5, size=n).astype(np.uint64))
    keys = np.concatenate(parts_k)
    vals = np.concatenate([np.arange(n, dtype=np.uint32) for n in sizes])
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    r = L.sort_batch(to_dev(keys), to_dev(seg), P, vals=to_dev(vals), s=32, want_send=True, want_cuts=True,
                     handler=ONE)
    L.check(r.workspace)
    for b in range(len(sizes)):
        a, e = int(seg[b]), int(seg[b + 1])
        o = O.sample_sort(keys[a:e], vals[a:e], P, 32)
        compare(r, o, P, b=b, seg=(a, e))


@pytest.mark.parametrize("handler", [L.HANDLER_PASSES, ONE])
def test_batch_of_many_tiny_instances(ws, handler):
    """Thousands of instances of 0 to 12 keys between a few large ones: the
    256 consecutive samples (and sample slots) a workgroup looks up span
    hundreds of blocks, many of them empty."""
    rng = np.random.default_rng(11)
    sizes = [int(x) for x in rng.integers(0, 13, size=3000)]
    sizes[100], sizes[1500], sizes[2999] = 70_000, 9_000, 130_001
    keys = np.concatenate([datagen.uniform_keys(n, seed=400 + i) if n else np.zeros(0, np.uint64)
                           for i, n in enumerate(sizes)])
    vals = np.concatenate([np.arange(n, dtype=np.uint32) for n in sizes])
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    P = 8
    r = L.sort_batch(to_dev(keys), to_dev(seg), P, vals=to_dev(vals), s=16, want_send=True, want_cuts=True,
                     handler=handler, workspace=ws)
    L.check(r.workspace)
    # host copies once, not per instance
    h = SimpleNamespace(**{f: (getattr(r, f).cpu() if getattr(r, f) is not None else None)
                           for f in ("keys", "vals", "part_offsets", "part_counts", "splitters", "send_counts",
                                     "cuts")})
    for b in range(len(sizes)):
        a, e = int(seg[b]), int(seg[b + 1])
        o = O.sample_sort(keys[a:e], vals[a:e], P, 16)
        compare(h, o, P, b=b, seg=(a, e))


@pytest.mark.parametrize("case", ["below_2_40", "medium_groups", "clustered_f64", "u32_normal", "u32_index"])
def test_one_pass_after_every_local_sort_path(ws, case):
    """The one-pass handler behind every branch of the local sort: blocks
    that fall back to the full LSD passes (keys below 2^40), groups for the
    mid-size sort (1000 top values; clustered doubles), and 32-bit keys
    (radix passes only; generated index values)."""
    n, P, vals = 1_000_000, 8, None
    if case == "below_2_40":
        keys = datagen.uniform_keys(n, seed=51) >> np.uint64(24)
    elif case == "medium_groups":
        low = datagen.uniform_keys(n, seed=52) >> np.uint64(24)
        top = np.arange(7, 7007, 7, dtype=np.uint64)[datagen.uniform_keys(n, seed=53) % np.uint64(1000)]
        keys = (top << np.uint64(40)) | low
    elif case == "clustered_f64":
        n, P = 2_000_000, 13
        x = datagen.typed_keys(n, seed=54, dtype=np.float64).view(np.uint64)
        keys = np.where(x >> np.uint64(63) == 1, ~x, x | np.uint64(1 << 63))
    elif case == "u32_normal":
        keys = datagen.normal_u32(n, seed=55)
        P = 37
    else:
        keys = datagen.uniform_keys(n, seed=56, dtype=np.uint32)
    vals = datagen.index_values(n)
    check_case(keys, vals, P, 0, ws=ws, handler=ONE)
    if case == "u32_index":
        check_case(keys, None, P, 0, ws=ws, handler=ONE)
