"""GPU parity of the generic interface (Section IV.C): signed and IEEE float
keys, generated index values (the provenance of every sorted entry), the
processor/offset split of those positions, and the binary search over a
sorted result.  Every output is compared bit for bit with the oracle in
``oracle/typed.py`` on the same seeded inputs.

Sizes span many radix tiles and merge tiles with ragged tails; the float
inputs carry NaNs of both signs, infinities and signed zeros, and the
approximately normal floats put many keys under few top-24-bit prefixes, so
the local sort's fall-back path runs as well.
"""
import numpy as np
import pytest
import torch

from oracle import sample_sort as O
from oracle import typed as T
from paper_1611_00463_amd import datagen
from paper_1611_00463_amd import lbsort as L
from tests.parity import assert_same, to_dev, to_host, u64

pytestmark = pytest.mark.gpu

TYPES = [np.int32, np.int64, np.float32, np.float64]


@pytest.fixture(scope="module")
def ws():
    return L.Workspace("cuda")


def bits(a):
    a = np.asarray(a)
    return a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint64)


def compare_typed(r, o, P, b=0, seg=None, with_vals=True):
    a, e = (0, len(o.keys)) if seg is None else seg
    assert_same("keys", bits(to_host(r.keys)[a:e]), bits(o.keys))
    if with_vals:
        assert_same("vals", to_host(r.vals)[a:e], o.vals)
    assert_same("part_offsets", u64(r.part_offsets)[b], o.part_offsets.astype(np.uint64))
    assert_same("part_counts", u64(r.part_counts)[b], o.part_counts.astype(np.uint64))
    if P > 1:
        assert_same("splitters", bits(to_host(r.splitters)[b]), bits(o.splitters))
    if r.send_counts is not None:
        assert_same("send_counts", u64(r.send_counts)[b], o.send_counts.astype(np.uint64))
    if r.cuts is not None:
        assert_same("cuts", u64(r.cuts)[b], o.cuts.astype(np.uint64))


def run_index(keys, P, s=0, mode=O.INV_COUNT, ws=None):
    r = L.sort_pairs(to_dev(keys), None, P, s=s, investigator=mode, want_send=True, want_cuts=True, workspace=ws)
    L.check(r.workspace)
    o = T.sample_sort_typed(keys, np.arange(len(keys), dtype=np.uint32), P, s, mode)
    compare_typed(r, o, P)
    return r, o


@pytest.mark.parametrize("dt", TYPES)
@pytest.mark.parametrize("n,P", [(1_500_007, 64), (300_001, 8), (50_000, 13)])
def test_typed_index_values(ws, dt, n, P):
    keys = datagen.typed_keys(n, seed=21, dtype=dt)
    run_index(keys, P, ws=ws)


@pytest.mark.parametrize("dt", TYPES)
def test_typed_keys_only_and_modes(ws, dt):
    n = 400_003
    keys = datagen.typed_keys(n, seed=22, dtype=dt)
    keys[::5] = keys[7]                               # a heavy duplicate
    for mode in (O.INV_COUNT, O.INV_NONE, O.INV_PAPER):
        r = L.sort_keys(to_dev(keys), 16, s=64, investigator=mode, want_send=True, want_cuts=True, workspace=ws)
        L.check(r.workspace)
        o = T.sample_sort_typed(keys, None, 16, 64, mode)
        compare_typed(r, o, 16, with_vals=False)


@pytest.mark.parametrize("dt", TYPES)
@pytest.mark.parametrize("n", [0, 1, 5, 4096, 4097, 20_000])
@pytest.mark.parametrize("P", [1, 3, 8])
def test_typed_small_and_ragged(ws, dt, n, P):
    keys = datagen.typed_keys(n, seed=23 + n, dtype=dt)
    run_index(keys, P, s=4, ws=ws)


@pytest.mark.parametrize("dt,udt", [(np.float64, np.uint64), (np.float32, np.uint32)])
def test_float_special_values_only(ws, dt, udt):
    """Every totalOrder corner at once, many times over, P = 1 (no merge pass:
    the keys are mapped back by the separate pass) and P = 8."""
    sp = np.array([0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000000, 0xFFF0000000000000,
                   0, 0x8000000000000000, 0x0000000000000001, 0x8000000000000001], dtype=np.uint64).view(np.float64)
    sp = sp.astype(dt) if dt == np.float32 else sp
    rng = np.random.default_rng(24)
    keys = sp[rng.integers(0, len(sp), 70_001)]
    for P in (1, 8):
        run_index(keys, P, s=16, ws=ws)


@pytest.mark.parametrize("dt", [np.int64, np.float32])
def test_typed_batch_index_values_are_instance_relative(ws, dt):
    sizes = [0, 1, 4095, 4097, 100_000, 33, 250_000]
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    keys = datagen.typed_keys(int(offs[-1]), seed=25, dtype=dt)
    P = 8
    r = L.sort_batch(to_dev(keys), to_dev(offs), P, s=32, index_values=True, want_send=True, want_cuts=True,
                     workspace=ws)
    L.check(r.workspace)
    for b in range(len(sizes)):
        a, e = int(offs[b]), int(offs[b + 1])
        o = T.sample_sort_typed(keys[a:e], np.arange(e - a, dtype=np.uint32), P, 32)
        compare_typed(r, o, P, b=b, seg=(a, e))


@pytest.mark.parametrize("dt", [np.int32, np.float64])
def test_typed_local_sort(ws, dt):
    sizes = [3, 70_000, 9000]
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    keys = datagen.typed_keys(int(offs[-1]), seed=26, dtype=dt)
    P = 4
    ko, vo, buf = L.local_sort(to_dev(keys), to_dev(offs), P, vals=to_dev(np.arange(len(keys), dtype=np.uint32)),
                               workspace=ws)
    L.check(buf)
    ko, vo = to_host(ko), to_host(vo)
    for b in range(len(sizes)):
        a, e = int(offs[b]), int(offs[b + 1])
        bounds = O.block_bounds(e - a, P)
        for i in range(P):
            x, y = a + bounds[i], a + bounds[i + 1]
            order = np.argsort(T.comparable(keys[x:y]), kind="stable")
            assert_same("keys", bits(ko[x:y]), bits(keys[x:y][order]))
            assert_same("vals", vo[x:y], (np.arange(x, y, dtype=np.uint32))[order])


def _f64_top32_groups(rng, n_target, sizes, seed, low_bits=32):
    """Doubles in groups of equal top 32 bits (sign, exponent, 20 fraction
    bits) of the given sizes, in random order: the keys of a group differ in
    their low `low_bits` bits, or (now and then) are all equal; half the
    groups negative."""
    parts, gid, total = [], 1, 0
    while total < n_target:
        g = int(sizes[rng.integers(0, len(sizes))])
        low = datagen.uniform_keys(g, seed=seed + gid) >> np.uint64(64 - low_bits)
        if rng.random() < 0.15:
            low[:] = low[0]
        top = (np.uint64(0x3FF + (gid % 7)) << np.uint64(52)) | (np.uint64((gid * 2654435761) % (1 << 20)) << np.uint64(32))
        if gid % 2:
            top |= np.uint64(1 << 63)
        parts.append(top | low)
        gid += 1
        total += g
    u = np.concatenate(parts)
    return u[rng.permutation(len(u))].view(np.float64)


@pytest.mark.parametrize("P", [1, 2])
def test_f64_groups_of_the_top_32_bits(ws, P):
    """Doubles take four top-digit passes and are grouped by their top 32
    bits: groups of every size class of the fix-up (ranked in place <= 64,
    sorted by the mid-size kernel 65..512 over the four digits below, left
    for the eight-pass sort above 512), and groups whose keys differ only in
    their low 8 bits (long runs after the mid-size kernel's first pass)."""
    rng = np.random.default_rng(90 + P)
    for sizes, low_bits in (([1, 2, 63, 64, 65, 66, 200, 511, 512, 513, 900], 32),
                            ([1, 64, 65, 100, 300, 512], 32),
                            ([70, 200, 512], 8)):
        keys = _f64_top32_groups(rng, 150_000 * P, sizes, 7000 * P + low_bits, low_bits)
        print(f"[typed] f64 top-32 groups P={P} low_bits={low_bits} n={len(keys)}", flush=True)
        run_index(keys, P, ws=ws)


@pytest.mark.parametrize("dt", [np.uint64, np.uint32] + TYPES)
def test_search_parity(ws, dt):
    n, P = 600_011, 16
    if dt in (np.uint64, np.uint32):
        keys = datagen.uniform_keys(n, seed=27, dtype=dt)
        keys[::3] = keys[1]
    else:
        keys = datagen.typed_keys(n, seed=27, dtype=dt)
    r = L.sort_keys(to_dev(keys), P, s=64, workspace=ws)
    L.check(r.workspace)
    o = T.sample_sort_typed(keys, None, P, 64)
    rng = np.random.default_rng(28)
    # queries: present keys, the duplicate, random bit patterns, the extremes
    q = np.concatenate([keys[rng.integers(0, n, 5000)], keys[1:2].repeat(7),
                        datagen.uniform_keys(5000, seed=29, dtype=np.uint64).view(np.uint8)[: 5000 * keys.itemsize]
                        .view(keys.dtype), o.keys[:1], o.keys[-1:]])
    for upper in (False, True):
        pos, part = L.search(r.keys, to_dev(q), upper, r.part_offsets[0])
        want_pos, want_part = T.search(o.keys, q, upper, o.part_offsets)
        assert_same("pos", to_host(pos).view(np.uint64), want_pos)
        assert_same("part", to_host(part), want_part)
    pos, _ = L.search(r.keys[:0], to_dev(q[:10]), False)          # empty data: every position 0
    assert not to_host(pos).any()


@pytest.mark.parametrize("dt", [np.uint64, np.uint32, np.float64, np.int32])
def test_search_indexed_parity(ws, dt):
    """The indexed search against the oracle and the plain search, bit for
    bit, at sizes around the index's level boundaries (16^k, 16^k + 1), with
    runs of equal keys that cross the 16-key groups, the extremes and keys
    outside the data."""
    rng = np.random.default_rng(31)
    for n in (0, 1, 15, 16, 17, 255, 256, 257, 4096, 4097, 65_537, 300_007):
        if dt in (np.uint64, np.uint32):
            keys = datagen.uniform_keys(n, seed=32 + n, dtype=dt)
        else:
            keys = datagen.typed_keys(n, seed=32 + n, dtype=dt)
        if n > 40:
            keys[5:40] = keys[3]          # a run of equal keys longer than a group
        sk = np.sort(keys) if dt in (np.uint64, np.uint32) else keys[np.argsort(T.comparable(keys), kind="stable")]
        P = 4
        G = np.array([i * n // P for i in range(P + 1)], dtype=np.uint64)
        qr = datagen.uniform_keys(300, seed=33, dtype=np.uint64).view(np.uint8)[: 300 * keys.itemsize].view(keys.dtype)
        q = np.concatenate([sk[rng.integers(0, n, 700)] if n else sk[:0], sk[:1], sk[-1:], sk[3:4], qr])
        dk = to_dev(sk)
        idx = L.SearchIndex(dk)
        for upper in (False, True):
            pos, part = idx.search(to_dev(q), upper, to_dev(G))
            want_pos, want_part = T.search(sk, q, upper, G)
            assert_same(f"pos n={n}", to_host(pos).view(np.uint64), want_pos)
            assert_same(f"part n={n}", to_host(part), want_part)
            p2, _ = L.search(dk, to_dev(q), upper)
            assert_same(f"plain n={n}", to_host(p2), to_host(pos))


def test_provenance_parity(ws):
    for n, P in ((1_000_003, 64), (77, 10), (5, 8)):
        keys = datagen.typed_keys(n, seed=30, dtype=np.float64)
        r = L.sort_pairs(to_dev(keys), None, P, workspace=ws)
        L.check(r.workspace)
        blk, off = L.provenance(r.vals, n, P)
        wb, wo = T.provenance(to_host(r.vals), n, P)
        assert_same("src_block", to_host(blk), wb)
        assert_same("src_offset", to_host(off), wo)
    # positions past the end
    blk, off = L.provenance(to_dev(np.array([0, 9, 10, 4000000000], dtype=np.uint32)), 10, 4)
    assert list(to_host(blk)) == [0, 3, 0xFFFFFFFF, 0xFFFFFFFF]
    assert list(to_host(off)) == [0, 9 - 7, 0xFFFFFFFF, 0xFFFFFFFF]
