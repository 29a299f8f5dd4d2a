"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit
for bit, on every output: sorted keys and values, partition offsets and
counts, splitters, send counts and the cut matrix.

Sizes span many radix tiles (4096 keys) and merge tiles with ragged tails, and
the edge cases of the method: empty input, N < P, P = 1, blocks that fit one
tile, all keys equal, heavy duplication, and every investigator mode.
"""
import numpy as np
import pytest
import torch

from oracle import sample_sort as O
from paper_1611_00463_amd import datagen
from paper_1611_00463_amd import lbsort as L
from tests.parity import check_case, compare, run_gpu, to_dev, to_host, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    return L.Workspace("cuda")


def test_config1_full_size(ws):
    """1,048,576 uniform u64 keys, P=8, 16 samples per block, keys only."""
    keys = datagen.uniform_keys(1 << 20, seed=1)
    check_case(keys, None, 8, 16, ws=ws)


@pytest.mark.parametrize("n", [3_000_017, 1 << 21])
def test_pairs_p64(ws, n):
    keys = datagen.uniform_keys(n, seed=2)
    vals = datagen.index_values(n)
    check_case(keys, vals, 64, 512, ws=ws)


@pytest.mark.parametrize("mode", [O.INV_COUNT, O.INV_NONE, O.INV_PAPER])
def test_duplicate_heavy_modes(ws, mode):
    n = 2_000_003
    keys = datagen.duplicate_heavy_keys(n, seed=3)
    vals = datagen.index_values(n)
    r, o = check_case(keys, vals, 64, 512, mode=mode, ws=ws)
    if mode == O.INV_COUNT:
        assert o.part_counts.max() / (n / 64) <= 1.05


def test_u32_pairs(ws):
    n = 1_234_567
    keys = datagen.uniform_keys(n, seed=5, dtype=np.uint32)
    check_case(keys, datagen.index_values(n), 8, 0, ws=ws)
    keys = datagen.normal_u32(n, seed=6)
    check_case(keys, datagen.index_values(n), 13, 0, ws=ws)


@pytest.mark.parametrize("n", [0, 1, 2, 7, 100, 4095, 4096, 4097, 8191, 50_000])
@pytest.mark.parametrize("P", [1, 2, 3, 8, 13])
def test_small_and_ragged(ws, n, P):
    keys = datagen.uniform_keys(n, seed=n + 17 * P)
    keys[::3] = keys[0] if n else keys[::3]          # some duplicates
    check_case(keys, datagen.index_values(n), P, 4, ws=ws)


def test_all_equal_and_sorted_inputs(ws):
    n = 300_001
    check_case(np.full(n, 7, dtype=np.uint64), datagen.index_values(n), 16, 8, ws=ws)
    srt = np.sort(datagen.uniform_keys(n, seed=9))
    check_case(srt, datagen.index_values(n), 16, 8, ws=ws)
    check_case(srt[::-1].copy(), datagen.index_values(n), 16, 8, ws=ws)
    k32 = np.sort(datagen.uniform_keys(n, seed=10, dtype=np.uint32))[::-1].copy()
    check_case(k32, None, 10, 0, ws=ws)


@pytest.mark.parametrize("rtile", [4096, 8192])
@pytest.mark.parametrize("fanin", [2, 4, 8, 16])
@pytest.mark.parametrize("tile", [1024, 2048, 4096])
def test_tuning_settings_do_not_change_bytes(ws, fanin, tile, rtile):
    n = 700_001
    keys = datagen.duplicate_heavy_keys(n, seed=11)
    check_case(keys, datagen.index_values(n), 37, 64, fanin=fanin, tile=tile, ws=ws, rtile=rtile)


def test_local_sort_stage(ws):
    """Step 1 alone: every block sorted on its own, against the oracle's blocks."""
    n, P = 1_000_003, 16
    keys = datagen.uniform_keys(n, seed=12)
    vals = datagen.index_values(n)
    seg = to_dev(np.array([0, n], dtype=np.uint64))
    k, v, buf = L.local_sort(to_dev(keys), seg, P, vals=to_dev(vals))
    L.check(buf)
    o = O.sample_sort(keys, vals, P)
    np.testing.assert_array_equal(to_host(k), np.concatenate(o.sorted_blocks))
    np.testing.assert_array_equal(to_host(v), np.concatenate(o.sorted_vals))


def test_batch_instances(ws):
    """Several data sets at once; each instance equals its own oracle run."""
    sizes = [0, 1, 5, 4096, 4097, 10_000, 123_457, 0, 33, 250_000, 3, 65_536]
    rng = np.random.default_rng(3)
    parts_k, parts_v = [], []
    for i, n in enumerate(sizes):
        if i % 3 == 0:
            k = datagen.uniform_keys(n, seed=100 + i, dtype=np.uint32)
        elif i % 3 == 1:
            k = np.sort(datagen.uniform_keys(n, seed=100 + i, dtype=np.uint32))
        else:
            k = rng.integers(0, 5, size=n).astype(np.uint32)
        parts_k.append(k)
        parts_v.append(np.arange(n, dtype=np.uint32))
    keys = np.concatenate(parts_k)
    vals = np.concatenate(parts_v)
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    for P in (1, 8, 5):
        r = L.sort_batch(to_dev(keys), to_dev(seg), P, vals=to_dev(vals), s=32, want_send=True, want_cuts=True)
        L.check(r.workspace)
        for b in range(len(sizes)):
            a, e = int(seg[b]), int(seg[b + 1])
            o = O.sample_sort(keys[a:e], vals[a:e], P, 32)
            compare(r, o, P, b=b, seg=(a, e))


def test_repeat_runs_identical(ws):
    """Same input, same workspace, five runs: identical bytes (races would show)."""
    n = 2_500_000
    keys = datagen.duplicate_heavy_keys(n, seed=13)
    kd = to_dev(keys)
    vd = to_dev(datagen.index_values(n))
    first = None
    for _ in range(5):
        r = L.sort_pairs(kd, vd, 64, s=512, workspace=ws)
        L.check(r.workspace)
        cur = (to_host(r.keys), to_host(r.vals), u64(r.part_offsets))
        if first is None:
            first = cur
        else:
            for a, b in zip(first, cur):
                np.testing.assert_array_equal(a, b)


# ---------------------------------------------------------------- local sort paths
# 64-bit keys are sorted locally by their three highest digits and a fix-up of
# the groups of equal top 24 bits; blocks with a large group of different keys
# are sorted again over all eight digits.  These inputs reach every branch.
def _top_small_keys(n, seed, top_values):
    low = datagen.uniform_keys(n, seed=seed) >> np.uint64(24)          # 40 random low bits
    pick = datagen.uniform_keys(n, seed=seed + 1) % np.uint64(len(top_values))
    return (np.asarray(top_values, dtype=np.uint64)[pick] << np.uint64(40)) | low


@pytest.mark.parametrize("rtile", [0, 4096])
@pytest.mark.parametrize("case", ["all_below_2_40", "half_blocks", "medium_groups", "small_groups", "clustered_f64"])
def test_local_sort_group_paths(ws, case, rtile):
    n, P = 1_000_000, 8
    if case == "all_below_2_40":          # one group per block with distinct keys: every block falls back
        keys = datagen.uniform_keys(n, seed=41) >> np.uint64(24)
    elif case == "half_blocks":           # blocks 0-3 fall back, blocks 4-7 take the fix-up
        keys = datagen.uniform_keys(n, seed=42)
        keys[: n // 2] >>= np.uint64(24)
    elif case == "medium_groups":         # 1000 top values: groups of ~125 keys per block (mid-size sort)
        keys = _top_small_keys(n, 43, list(range(7, 7007, 7)))
    elif case == "small_groups":          # 2^16 top values: groups of a few keys, many straddling tiles
        keys = _top_small_keys(n, 44, list(range(0, 1 << 16)))
    else:                                  # normal-like doubles as unsigned images: groups of up to ~300 keys
        n, P = 4_000_000, 2
        x = datagen.typed_keys(n, seed=47, dtype=np.float64).view(np.uint64)
        keys = np.where(x >> np.uint64(63) == 1, ~x, x | np.uint64(1 << 63))
    vals = datagen.index_values(n)
    check_case(keys, vals, P, 0, ws=ws, rtile=rtile)


def _sized_groups_block(rng, n_target, sizes, seed, low_bits=40):
    """Keys of one block made of groups (equal top 24 bits) of the given sizes,
    in random order: groups of different keys (random in their low `low_bits`
    bits), and now and then a group whose keys are all equal."""
    parts, gid, total = [], 1, 0
    while total < n_target:
        g = int(sizes[rng.integers(0, len(sizes))])
        low = datagen.uniform_keys(g, seed=seed + gid) >> np.uint64(64 - low_bits)
        if rng.random() < 0.15:
            low[:] = low[0]                       # all keys of the group equal
        parts.append((np.uint64(gid * 37 + 5) << np.uint64(40)) | low)
        gid += 1
        total += g
    keys = np.concatenate(parts)
    return keys[rng.permutation(len(keys))]


@pytest.mark.parametrize("rtile", [0, 4096])
@pytest.mark.parametrize("P", [1, 2])
def test_group_sizes_at_the_thresholds(ws, P, rtile):
    """Groups of every size class of the 64-bit fix-up at once, ranked in
    place (<= 64 keys), sorted by the mid-size kernel (65..512) or left for
    the eight-pass sort (> 512 different keys), straddling tiles and blocks."""
    rng = np.random.default_rng(46 + P)
    sizes = [1, 2, 63, 64, 65, 66, 200, 511, 512, 513, 900, 5000]
    blocks = [_sized_groups_block(rng, 300_000, sizes, 1000 * (b + 1)) for b in range(P)]
    # equal block sizes, so that block i is exactly the i-th part
    m = min(len(b) for b in blocks)
    keys = np.concatenate([b[:m] for b in blocks])
    check_case(keys, datagen.index_values(len(keys)), P, 0, ws=ws, rtile=rtile)
    # the same groups but no group above 512 keys: no block falls back
    sizes = [1, 64, 65, 100, 300, 512]
    blocks = [_sized_groups_block(rng, 300_000, sizes, 5000 * (b + 1)) for b in range(P)]
    m = min(len(b) for b in blocks)
    keys = np.concatenate([b[:m] for b in blocks])
    check_case(keys, datagen.index_values(len(keys)), P, 0, ws=ws, rtile=rtile)
    check_case(keys, None, P, 0, ws=ws, rtile=rtile)
    # groups whose keys differ only in their low 32 bits (long runs after the
    # first pass of the group sort) or only in their low 8 bits (many equal keys)
    for low_bits in (32, 8):
        blocks = [_sized_groups_block(rng, 200_000, sizes, 9000 * (b + 1), low_bits) for b in range(P)]
        m = min(len(b) for b in blocks)
        keys = np.concatenate([b[:m] for b in blocks])
        check_case(keys, datagen.index_values(len(keys)), P, 0, ws=ws, rtile=rtile)


def test_batch_with_group_paths(ws):
    """A batch of 64-bit instances whose blocks take every branch of the local
    sort's fix-up: small groups, listed mid-size groups, mixed groups above 512
    keys (the eight-pass sort), and a uniform instance; P = 3 and 4."""
    rng = np.random.default_rng(48)
    parts = [
        _sized_groups_block(rng, 200_000, [1, 64, 65, 300, 512], 11000),
        datagen.uniform_keys(150_001, seed=49),
        _sized_groups_block(rng, 120_000, [2, 100, 513, 5000], 12000),
        np.zeros(0, dtype=np.uint64),
        _sized_groups_block(rng, 90_000, [70, 200], 13000, low_bits=32),
    ]
    sizes = [len(k) for k in parts]
    keys = np.concatenate(parts)
    vals = np.concatenate([np.arange(n, dtype=np.uint32) for n in sizes])
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    for P in (3, 4):
        r = L.sort_batch(to_dev(keys), to_dev(seg), P, vals=to_dev(vals), s=64, want_send=True, want_cuts=True)
        L.check(r.workspace)
        for b in range(len(sizes)):
            a, e = int(seg[b]), int(seg[b + 1])
            o = O.sample_sort(keys[a:e], vals[a:e], P, 64)
            compare(r, o, P, b=b, seg=(a, e))


def test_local_sort_paths_agree(ws, monkeypatch):
    """The same bytes with the fix-up and with all eight radix passes."""
    keys = datagen.uniform_keys(1 << 21, seed=45)
    vals = datagen.index_values(1 << 21)
    a = check_case(keys, vals, 16, 0, ws=ws)[0]
    ka, va = to_host(a.keys).copy(), to_host(a.vals).copy()
    monkeypatch.setenv("LBSORT_LOCAL_SORT", "lsd")
    b = check_case(keys, vals, 16, 0, ws=ws)[0]
    assert np.array_equal(ka, to_host(b.keys)) and np.array_equal(va, to_host(b.vals))


@pytest.mark.parametrize("rtile", [4096, 8192])
def test_radix_tile_settings(ws, rtile):
    """Both radix tiles on the main shapes: u64 pairs at P = 64, u32 pairs,
    blocks just above one and two tiles, the duplicate-heavy input, and the
    two local-sort paths of 64-bit keys giving the same bytes."""
    n = 3_000_017
    check_case(datagen.uniform_keys(n, seed=2), datagen.index_values(n), 64, 512, ws=ws, rtile=rtile)
    n = 1_234_567
    check_case(datagen.uniform_keys(n, seed=5, dtype=np.uint32), datagen.index_values(n), 8, 0, ws=ws, rtile=rtile)
    check_case(datagen.normal_u32(n, seed=6), None, 13, 0, ws=ws, rtile=rtile)
    for n, P in ((4097, 1), (8191, 1), (8193, 1), (12_289, 3), (3 * 8192 + 5, 3), (50_000, 8)):
        check_case(datagen.uniform_keys(n, seed=n + P), datagen.index_values(n), P, 4, ws=ws, rtile=rtile)
    n = 2_000_003
    keys = datagen.duplicate_heavy_keys(n, seed=3)
    check_case(keys, datagen.index_values(n), 64, 512, ws=ws, rtile=rtile)


def test_radix_tiles_agree_on_every_local_sort_path(ws, monkeypatch):
    """Radix tiles of 4096 and 8192 keys, fix-up path and all eight passes:
    the same bytes."""
    keys = datagen.uniform_keys(1 << 21, seed=45)
    vals = datagen.index_values(1 << 21)
    ref = run_gpu(keys, vals, 16, 0, ws=ws)
    ka, va = to_host(ref.keys).copy(), to_host(ref.vals).copy()
    for lsd in (False, True):
        if lsd:
            monkeypatch.setenv("LBSORT_LOCAL_SORT", "lsd")
        for rtile in (4096, 8192):
            r = run_gpu(keys, vals, 16, 0, ws=ws, rtile=rtile)
            assert np.array_equal(ka, to_host(r.keys)) and np.array_equal(va, to_host(r.vals)), (lsd, rtile)


def test_radix_tile_16384_for_32bit_keys(ws):
    """Tiles of 16384 keys (32-bit keys only): pairs and keys, blocks just
    above one and several tiles, a batch of uneven instances."""
    n = 1_234_567
    check_case(datagen.uniform_keys(n, seed=5, dtype=np.uint32), datagen.index_values(n), 8, 0, ws=ws, rtile=16384)
    check_case(datagen.normal_u32(n, seed=6), None, 13, 0, ws=ws, rtile=16384)
    for n, P in ((16_383, 1), (16_385, 1), (3 * 16_384 + 5, 1), (100_003, 3)):
        k = datagen.uniform_keys(n, seed=n + P, dtype=np.uint32)
        check_case(k, datagen.index_values(n), P, 4, ws=ws, rtile=16384)
    sizes = [0, 5, 4097, 16_385, 70_000, 1, 250_000]
    keys = np.concatenate([datagen.uniform_keys(m, seed=300 + i, dtype=np.uint32) for i, m in enumerate(sizes)])
    vals = np.concatenate([np.arange(m, dtype=np.uint32) for m in sizes])
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    r = L.sort_batch(to_dev(keys), to_dev(seg), 8, vals=to_dev(vals), s=16, want_send=True, want_cuts=True,
                     radix_tile=16384)
    L.check(r.workspace)
    for b in range(len(sizes)):
        a, e = int(seg[b]), int(seg[b + 1])
        compare(r, O.sample_sort(keys[a:e], vals[a:e], 8, 16), 8, b=b, seg=(a, e))
