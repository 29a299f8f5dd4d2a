"""Pins of the typed-key, provenance and search oracle against things other
than itself:

* IEEE 754-2008 totalOrder (clause 5.10) on a hand-ordered list of special
  values: NaNs of both signs, infinities, signed zeros, subnormals;
* finite floats without signed zeros against numpy's own float sort (a
  library routine that agrees with totalOrder there);
* signed integers against Python's stable ``sorted`` of the numbers;
* provenance against a brute-force walk over the block boundaries;
* search against brute-force counting with Python's comparisons.
"""
import math
import struct

import numpy as np
import pytest

from oracle import sample_sort as O
from oracle import typed as T


def f64(bits):
    return struct.unpack("<d", struct.pack("<Q", bits))[0]


def f32_bits_array(bits):
    return np.array(bits, dtype=np.uint32).view(np.float32)


def f64_bits_array(bits):
    return np.array(bits, dtype=np.uint64).view(np.float64)


# Increasing in totalOrder, written out by hand from the clause: negative NaNs
# (larger payload lower), -inf, negative numbers, -0, +0, positive numbers,
# +inf, positive NaNs (signalling below quiet, then by payload).
F64_ORDERED = [
    0xFFF8000000000001,  # -qNaN, payload 1
    0xFFF8000000000000,  # -qNaN
    0xFFF0000000000001,  # -sNaN
    0xFFF0000000000000,  # -inf
    0xFFEFFFFFFFFFFFFF,  # -max
    0xBFF0000000000000,  # -1
    0x8010000000000000,  # -min normal
    0x8000000000000001,  # -min subnormal
    0x8000000000000000,  # -0
    0x0000000000000000,  # +0
    0x0000000000000001,  # +min subnormal
    0x0010000000000000,  # +min normal
    0x3FF0000000000000,  # 1
    0x7FEFFFFFFFFFFFFF,  # max
    0x7FF0000000000000,  # +inf
    0x7FF0000000000001,  # +sNaN
    0x7FF8000000000000,  # +qNaN
    0x7FF8000000000001,  # +qNaN, payload 1
]
F32_ORDERED = [0xFFC00001, 0xFFC00000, 0xFF800001, 0xFF800000, 0xFF7FFFFF, 0xBF800000, 0x80800000,
               0x80000001, 0x80000000, 0x00000000, 0x00000001, 0x00800000, 0x3F800000, 0x7F7FFFFF,
               0x7F800000, 0x7F800001, 0x7FC00000, 0x7FC00001]


@pytest.mark.parametrize("ordered,mk,udt", [(F64_ORDERED, f64_bits_array, np.uint64),
                                            (F32_ORDERED, f32_bits_array, np.uint32)])
def test_total_order_special_values(ordered, mk, udt):
    rng = np.random.default_rng(1)
    for trial in range(20):
        perm = rng.permutation(len(ordered))
        keys = mk([ordered[i] for i in perm])
        for P in (1, 3):
            r = T.sample_sort_typed(keys, np.arange(len(keys), dtype=np.uint32), P, 2)
            assert [int(b) for b in r.keys.view(udt)] == ordered
            assert list(perm[r.vals]) == list(range(len(ordered)))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_finite_floats_match_numpy_sort(dt):
    rng = np.random.default_rng(2)
    for trial in range(40):
        n = int(rng.integers(0, 300))
        keys = (rng.standard_normal(n) * 10.0 ** rng.integers(-30, 30)).astype(dt)
        keys[keys == 0] = dt(1.5)          # no signed zeros
        if trial % 3 == 0 and n:
            keys[rng.integers(0, n, n // 2)] = keys[0]   # duplicates
        P = int(rng.integers(1, 9))
        vals = np.arange(n, dtype=np.uint32)
        r = T.sample_sort_typed(keys, vals, P, int(rng.integers(1, 6)))
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(r.keys.view(np.uint8), keys[order].view(np.uint8))
        assert np.array_equal(r.vals, order.astype(np.uint32))
        # partitions: every key of partition k is <= every key of k+1
        G = r.part_offsets
        for k in range(P - 1):
            if G[k + 1] > G[k] and G[k + 2] > G[k + 1]:
                assert r.keys[G[k + 1] - 1] <= r.keys[G[k + 1]]


def test_total_order_round_trip():
    rng = np.random.default_rng(3)
    for dt, udt in ((np.float32, np.uint32), (np.float64, np.uint64)):
        bits = rng.integers(0, np.iinfo(udt).max, 5000, dtype=udt, endpoint=True)
        keys = bits.view(dt)
        back = T.from_total_order_int(T.total_order_int(keys), dt)
        assert np.array_equal(back.view(udt), bits)
        t = T.total_order_int(keys)
        # the map is monotone on numbers: compare with Python floats on finite pairs
        fin = np.isfinite(keys)
        a, b = keys[fin][:-1], keys[fin][1:]
        ta, tb = t[fin][:-1], t[fin][1:]
        for x, y, tx, ty in zip(a[:500], b[:500], ta[:500], tb[:500]):
            if float(x) < float(y):
                assert tx < ty
            elif float(x) > float(y):
                assert tx > ty


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_signed_keys_python_sorted(dt):
    rng = np.random.default_rng(4)
    info = np.iinfo(dt)
    for trial in range(200):
        n = int(rng.integers(0, 50))
        if trial % 2:
            alpha = np.array([info.min, -1, 0, 1, info.max], dtype=dt)
            keys = alpha[rng.integers(0, 5, n)]
        else:
            keys = rng.integers(info.min, info.max, n, dtype=dt, endpoint=True)
        P = int(rng.integers(1, 9))
        vals = np.arange(n, dtype=np.uint32)
        r = T.sample_sort_typed(keys, vals, P, int(rng.integers(1, 6)))
        order = sorted(range(n), key=lambda i: int(keys[i]))
        assert [int(x) for x in r.keys] == [int(keys[i]) for i in order]
        assert [int(x) for x in r.vals] == order
        # every splitter is a key and partitions are ordered as numbers
        G = [int(g) for g in r.part_offsets]
        for k in range(P - 1):
            left = [int(x) for x in r.keys[G[k]:G[k + 1]]]
            right = [int(x) for x in r.keys[G[k + 1]:]]
            if left and right:
                assert max(left) <= min(right)


def test_signed_hand_example():
    keys = np.array([3, -1, 0, -5, 2, -1], dtype=np.int64)
    r = T.sample_sort_typed(keys, np.arange(6, dtype=np.uint32), 2, 2)
    assert list(r.keys) == [-5, -1, -1, 0, 2, 3]
    assert list(r.vals) == [3, 1, 5, 2, 4, 0]


def test_provenance_brute_force():
    rng = np.random.default_rng(5)
    for trial in range(100):
        n = int(rng.integers(1, 200))
        P = int(rng.integers(1, 40))
        g = rng.integers(0, n, 50)
        blk, off = T.provenance(g, n, P)
        for x, b, o in zip(g, blk, off):
            # walk the blocks: block i is [i*n//P, (i+1)*n//P)
            i = 0
            while not (i * n // P <= x < (i + 1) * n // P):
                i += 1
            assert b == i and o == x - i * n // P


def _key_f(x):
    # Python comparison with -0 below +0 (no NaNs in these cases)
    return (float(x), math.copysign(1.0, float(x)))


@pytest.mark.parametrize("dt", [np.uint64, np.int64, np.int32, np.float64, np.float32])
def test_search_brute_force(dt):
    rng = np.random.default_rng(6)
    for trial in range(60):
        n = int(rng.integers(0, 80))
        if np.issubdtype(dt, np.floating):
            pool = np.array([-2.5, -1.0, -0.0, 0.0, 0.5, 3.0, np.inf, -np.inf], dtype=dt)
            key = _key_f
        elif np.issubdtype(dt, np.signedinteger):
            pool = np.array([np.iinfo(dt).min, -3, -1, 0, 2, 7, np.iinfo(dt).max], dtype=dt)
            key = int
        else:
            pool = np.array([0, 1, 5, 2 ** 63, 2 ** 64 - 1], dtype=dt)
            key = int
        keys = pool[rng.integers(0, len(pool), n)]
        P = int(rng.integers(1, 6))
        r = T.sample_sort_typed(keys, None, P, 2)
        q = pool[rng.integers(0, len(pool), 30)]
        for upper in (False, True):
            pos, part = T.search(r.keys, q, upper, r.part_offsets)
            G = [int(x) for x in r.part_offsets]
            for j, qq in enumerate(q):
                want = sum(1 for x in r.keys if (key(x) <= key(qq) if upper else key(x) < key(qq)))
                assert int(pos[j]) == want
                if want == n:
                    assert part[j] == P
                else:
                    assert G[part[j]] <= want < G[part[j] + 1]


def test_typed_worked_example_signed_mirrors_unsigned():
    # the worked example with every key negated and sorted as signed numbers:
    # the order reverses, so the sorted output is the mirrored key set
    keys = np.array([7, 3, 3, 9, 3, 1, 3, 3, 8, 3, 2, 3, 3, 5, 3, 3], dtype=np.int64)
    r = T.sample_sort_typed(-keys, np.arange(16, dtype=np.uint32), 4, 2)
    assert list(r.keys) == sorted((-keys).tolist())
    assert r.part_counts.sum() == 16
