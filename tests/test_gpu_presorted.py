"""Blocks that are already in order, or in reverse order, skip the radix
passes (found by the histogram, copied or reversed run by run).  Parity
against the oracle, bit for bit, on inputs where some, all or none of the
blocks are presorted: distinct keys, long runs of equal keys (the reversal
must keep them in input order), runs crossing radix tiles and blocks, all
keys equal, typed keys, and a batch mixing sorted, reverse and random
instances."""
import numpy as np
import pytest

from oracle import sample_sort as O
from paper_1611_00463_amd import datagen
from paper_1611_00463_amd import lbsort as L
from tests.parity import check_case, compare, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    return L.Workspace("cuda")


def _dups(n, seed, values):
    return (datagen.uniform_keys(n, seed=seed) % np.uint64(values)) * np.uint64(0x9E3779B97F4A7C15)


@pytest.mark.parametrize("rtile", [0, 4096])
@pytest.mark.parametrize("dtype", [np.uint64, np.uint32])
def test_sorted_and_reverse_blocks(ws, dtype, rtile):
    n = 700_001
    k = datagen.uniform_keys(n, seed=51, dtype=dtype)
    s = np.sort(k)
    r = s[::-1].copy()
    print(f"[presorted] {np.dtype(dtype).name} rtile={rtile}", flush=True)
    for keys in (s, r):
        check_case(keys, datagen.index_values(n), 8, 0, ws=ws, rtile=rtile)
        check_case(keys, None, 5, 0, ws=ws, rtile=rtile)
    # reverse order with long runs of equal keys (runs across tiles and blocks)
    for values in (3, 50, 5000):
        d = np.sort(_dups(n, 52 + values, values).astype(dtype))[::-1].copy()
        check_case(d, datagen.index_values(n), 8, 0, ws=ws, rtile=rtile)
        check_case(np.sort(d), datagen.index_values(n), 8, 0, ws=ws, rtile=rtile)
    # some blocks in order, some reversed, some random (P = 4 blocks of n / 4)
    q = n // 4
    mix = np.concatenate([np.sort(k[:q]), np.sort(k[q:2 * q])[::-1], k[2 * q:3 * q], np.sort(k[3 * q:])])
    check_case(mix, datagen.index_values(n), 4, 0, ws=ws, rtile=rtile)
    check_case(mix, datagen.index_values(n), 4, 0, mode=O.INV_PAPER, ws=ws, rtile=rtile)
    # almost sorted: one pair swapped in the middle of a block
    a = s.copy()
    a[q // 2], a[q // 2 + 1] = a[q // 2 + 1], a[q // 2]
    check_case(a, datagen.index_values(n), 4, 0, ws=ws, rtile=rtile)
    b = r.copy()
    b[3 * q + 17], b[3 * q + 18] = b[3 * q + 18], b[3 * q + 17]
    check_case(b, datagen.index_values(n), 4, 0, ws=ws, rtile=rtile)


def test_all_equal_and_two_values(ws):
    n = 300_007
    check_case(np.full(n, 12345, dtype=np.uint64), datagen.index_values(n), 16, 0, ws=ws)
    two = np.where(np.arange(n) < n // 3, 9, 4).astype(np.uint64)      # 9...9 4...4: non-increasing
    check_case(two, datagen.index_values(n), 16, 0, ws=ws)
    check_case(two[::-1].copy(), datagen.index_values(n), 16, 0, ws=ws)


def test_typed_reverse_with_signed_zeros(ws):
    """Reverse-sorted doubles with -0 and +0 (different in totalOrder) and
    equal values; index values generated."""
    n = 400_003
    x = np.round(np.sort(datagen.typed_keys(n, seed=53, dtype=np.float64)), 1)[::-1].copy()
    x[::997] = 0.0
    x[1::997] = -0.0
    from oracle import typed as T
    x = x[np.argsort(T.total_order_int(x), kind="stable")[::-1]]   # non-increasing in totalOrder
    o = T.sample_sort_typed(x, np.arange(n, dtype=np.uint32), 8)
    r = L.sort_pairs(to_dev(x), None, 8)
    L.check(r.workspace)
    assert np.array_equal(r.keys.cpu().numpy().view(np.uint64), o.keys.view(np.uint64))
    assert np.array_equal(r.vals.cpu().numpy(), o.vals)


def test_batch_mixed_presorted(ws):
    sizes = [50_000, 70_001, 0, 123_457, 9000, 300_000, 4097]
    rng = np.random.default_rng(54)
    parts = []
    for i, m in enumerate(sizes):
        k = datagen.uniform_keys(m, seed=400 + i, dtype=np.uint32)
        if i % 3 == 0:
            k = np.sort(k)
        elif i % 3 == 1:
            k = np.sort(k % np.uint32(100))[::-1].copy()
        parts.append(k)
    keys = np.concatenate(parts)
    vals = np.concatenate([np.arange(m, dtype=np.uint32) for m in sizes])
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    for P in (1, 8):
        r = L.sort_batch(to_dev(keys), to_dev(seg), P, vals=to_dev(vals), s=16, want_send=True, want_cuts=True)
        L.check(r.workspace)
        for b in range(len(sizes)):
            a, e = int(seg[b]), int(seg[b + 1])
            compare(r, O.sample_sort(keys[a:e], vals[a:e], P, 16), P, b=b, seg=(a, e))


def test_presorted_detection_off_gives_the_same_bytes(ws):
    """LBSORT_PRESORTED_IGNORE (every block through the radix passes) and
    the default detection agree bit for bit, on presorted and random blocks."""
    from tests.parity import run_gpu, to_host
    n = 500_001
    k = datagen.uniform_keys(n, seed=55)
    q = n // 4
    mix = np.concatenate([np.sort(k[:q]), np.sort(k[q:2 * q])[::-1], k[2 * q:3 * q], np.sort(k[3 * q:] % np.uint64(7))[::-1]])
    vals = datagen.index_values(n)
    for keys in (mix, k):
        a = L.sort_pairs(to_dev(keys), to_dev(vals), 4, presorted=L.PRESORTED_DETECT)
        b = L.sort_pairs(to_dev(keys), to_dev(vals), 4, presorted=L.PRESORTED_IGNORE)
        L.check(a.workspace)
        L.check(b.workspace)
        assert np.array_equal(to_host(a.keys), to_host(b.keys)) and np.array_equal(to_host(a.vals), to_host(b.vals))
        assert np.array_equal(to_host(a.part_offsets), to_host(b.part_offsets))
