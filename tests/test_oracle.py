"""Pins of the CPU oracle against things other than itself.

Each check is chosen so that a plausible slip in the oracle (a dropped term, a
wrong index or sign, a swapped operand) fails at least one of them:

* the sorted output against Python's own stable ``sorted`` (a textbook routine);
* COUNT partition offsets against the closed form clamp(floor(kN/P), #<v, #<=v)
  counted by brute force;
* COUNT cuts against "how many of the first G_k elements of the stable order
  came from block i", by brute force;
* every element sampled: the splitters must be exact order statistics;
* the hand-worked example in ``tests/golden/worked_example.txt``;
* the handler's pairing order printed in Section IV.A (Fig. 2);
* the balance guarantee max_k n_k <= N/P + N/s + O(P) on adversarial inputs,
  and Table 2's largest share (10.022% at P=10) on uniform data.
"""
import itertools
import os

import numpy as np
import pytest

from oracle import sample_sort as O
from paper_1611_00463_amd import datagen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def brute_stable_order(keys):
    return sorted(range(len(keys)), key=lambda i: int(keys[i]))


def rand_keys(rng, n, alphabet=None, dtype=np.uint64):
    if alphabet is not None:
        alpha = np.array([int(a) for a in alphabet], dtype=dtype)
        return alpha[rng.integers(0, len(alpha), size=n)]
    hi = 2 ** 64 if dtype == np.uint64 else 2 ** 32
    return np.array([int(x) for x in rng.integers(0, hi, size=n, dtype=np.uint64 if dtype == np.uint64 else np.uint32)], dtype=dtype)


ALPHA = [0, 1, 2, 2 ** 64 - 1]


# ------------------------------------------------------------------ sorted output
@pytest.mark.parametrize("mode", [O.INV_COUNT, O.INV_NONE])
def test_output_is_python_stable_sort(mode):
    rng = np.random.default_rng(11)
    for trial in range(300):
        n = int(rng.integers(0, 40))
        P = int(rng.integers(1, 9))
        s = int(rng.integers(1, 6))
        alpha = ALPHA if trial % 2 else None
        keys = rand_keys(rng, n, alpha)
        vals = np.arange(n, dtype=np.uint32)
        r = O.sample_sort(keys, vals, P, s, mode)
        order = brute_stable_order(keys)
        assert [int(x) for x in r.keys] == [int(keys[i]) for i in order]
        assert [int(x) for x in r.vals] == order


def test_exhaustive_tiny_alphabet():
    """Every key string of length <= 6 over {0, 1, 2^64-1}, P <= 4, s <= 3."""
    alpha = [0, 1, 2 ** 64 - 1]
    for n in range(0, 7):
        for tup in itertools.product(alpha, repeat=n):
            keys = np.array(tup, dtype=np.uint64)
            order = brute_stable_order(keys)
            for P in (1, 2, 3, 4):
                for s in (1, 3):
                    r = O.sample_sort(keys, np.arange(n, dtype=np.uint32), P, s, O.INV_COUNT)
                    assert [int(x) for x in r.vals] == order
                    assert int(r.part_offsets[-1]) == n
                    p = O.sample_sort(keys, np.arange(n, dtype=np.uint32), P, s, O.INV_PAPER)
                    assert [int(x) for x in p.keys] == [int(keys[i]) for i in order]
                    assert sorted(int(x) for x in p.vals) == list(range(n))


def test_paper_mode_sorted_permutation():
    rng = np.random.default_rng(5)
    for _ in range(200):
        n = int(rng.integers(0, 60))
        P = int(rng.integers(1, 9))
        keys = rand_keys(rng, n, [3, 5, 5, 5, 9])
        r = O.sample_sort(keys, np.arange(n, dtype=np.uint32), P, int(rng.integers(1, 8)), O.INV_PAPER)
        assert list(r.keys) == sorted(keys.tolist())
        assert sorted(r.vals.tolist()) == list(range(n))
        assert np.all(keys[r.vals.astype(np.int64)] == r.keys)


# ------------------------------------------------------------------ partition metadata
def brute_counts(keys, v):
    less = sum(1 for x in keys if int(x) < int(v))
    leq = sum(1 for x in keys if int(x) <= int(v))
    return less, leq


def test_count_offsets_closed_form_and_cuts_brute_force():
    rng = np.random.default_rng(7)
    for trial in range(300):
        n = int(rng.integers(0, 50))
        P = int(rng.integers(1, 9))
        s = int(rng.integers(1, 7))
        keys = rand_keys(rng, n, ALPHA if trial % 3 else [5, 5, 5, 6])
        r = O.sample_sort(keys, np.arange(n, dtype=np.uint32), P, s, O.INV_COUNT)
        G = r.part_offsets
        assert G[0] == 0 and G[P] == n
        order = brute_stable_order(keys)
        bounds = [i * n // P for i in range(P + 1)]
        block_of = [next(b for b in range(P) if bounds[b] <= j < bounds[b + 1]) for j in range(n)]
        for k in range(1, P):
            less, leq = brute_counts(keys, r.splitters[k - 1])
            assert G[k] == min(max(k * n // P, less), leq)
            for i in range(P):
                first = order[:G[k]]
                assert r.cuts[i, k] == sum(1 for j in first if block_of[j] == i)


def test_none_mode_cuts_are_lower_bounds():
    rng = np.random.default_rng(8)
    for _ in range(200):
        n = int(rng.integers(0, 40))
        P = int(rng.integers(1, 7))
        keys = rand_keys(rng, n, ALPHA)
        r = O.sample_sort(keys, None, P, int(rng.integers(1, 5)), O.INV_NONE)
        bounds = [i * n // P for i in range(P + 1)]
        for k in range(1, P):
            for i in range(P):
                blk = keys[bounds[i]:bounds[i + 1]]
                assert r.cuts[i, k] == sum(1 for x in blk if int(x) < int(r.splitters[k - 1]))


def test_every_element_sampled_gives_exact_quantiles():
    """With s >= block size every element is a sample, so the pool is the whole
    input in order and splitter k is its element of rank
    min(N-1, floor(kN/P) + floor(P/2) - 1)."""
    rng = np.random.default_rng(9)
    for _ in range(100):
        n = int(rng.integers(1, 80))
        P = int(rng.integers(1, 9))
        keys = rand_keys(rng, n)
        r = O.sample_sort(keys, None, P, n + 1)
        srt = sorted(int(x) for x in keys)
        assert sorted(int(x) for x in np.concatenate(r.samples)) == srt
        for k in range(1, P):
            assert int(r.splitters[k - 1]) == srt[min(n - 1, k * n // P + P // 2 - 1)]


def test_samples_are_block_order_statistics():
    """Sample j of a block of n keys is its element of rank floor(j n / s):
    with s = 1 the block minimum, with s = 2 the minimum and the element of
    rank floor(n/2)."""
    rng = np.random.default_rng(10)
    for _ in range(50):
        n = int(rng.integers(1, 50))
        keys = rand_keys(rng, n)
        srt = sorted(int(x) for x in keys)
        assert [int(x) for x in O.sample_sort(keys, None, 1, 1).samples[0]] == [srt[0]]
        two = [int(x) for x in O.sample_sort(keys, None, 1, 2).samples[0]]
        assert two == ([srt[0], srt[n // 2]] if n >= 2 else [srt[0]])


def test_partition_key_ranges_are_monotone():
    """Smaller keys on smaller processor ids (Section IV.C, Table 3)."""
    rng = np.random.default_rng(12)
    for mode in (O.INV_COUNT, O.INV_NONE, O.INV_PAPER):
        for _ in range(100):
            n = int(rng.integers(0, 80))
            P = int(rng.integers(1, 9))
            keys = rand_keys(rng, n, [1, 4, 4, 4, 4, 9, 2 ** 63])
            r = O.sample_sort(keys, None, P, int(rng.integers(1, 6)), mode)
            G = r.part_offsets
            v = [0] + [int(x) for x in r.splitters] + [2 ** 64 - 1]
            for k in range(P):
                part = r.keys[G[k]:G[k + 1]]
                if len(part):
                    assert v[k] <= int(part.min()) and int(part.max()) <= v[k + 1]
                if k + 1 < P and G[k + 1] > G[k] and G[k + 2] > G[k + 1]:
                    assert int(r.keys[G[k + 1] - 1]) <= int(r.keys[G[k + 1]])


# ------------------------------------------------------------------ worked example
def load_worked_example():
    common, modes, cur = {}, {}, None
    with open(os.path.join(GOLD, "worked_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, rest = line.split(None, 1)
            if name == "mode":
                cur = rest
                modes[cur] = {}
                continue
            if "|" in rest:
                val = [[int(x) for x in part.split()] for part in rest.split("|")]
            else:
                val = [int(x) for x in rest.split()]
            (modes[cur] if cur else common)[name] = val
    return common, modes


def test_worked_example():
    common, modes = load_worked_example()
    keys = np.array(common["keys"], dtype=np.uint64)
    P, s = common["P"][0], common["s"][0]
    ids = {"COUNT": O.INV_COUNT, "NONE": O.INV_NONE, "PAPER": O.INV_PAPER}
    for name, exp in modes.items():
        r = O.sample_sort(keys, np.arange(len(keys), dtype=np.uint32), P, s, ids[name])
        assert np.concatenate(r.samples).tolist() == common["samples"]
        assert r.splitters.tolist() == common["splitters"]
        assert r.lo.tolist() == common["lo"]
        assert r.hi.tolist() == common["hi"]
        assert r.keys.tolist() == common["keys_out"]
        assert r.cuts.tolist() == exp["cuts"]
        assert r.part_counts.tolist() == exp["part_counts"]
        assert r.part_offsets.tolist() == exp["part_offsets"]
        if "recv_offsets" in exp:
            assert r.recv_offsets.tolist() == exp["recv_offsets"]
        assert r.vals.tolist() == exp["vals_out"]


def test_all_keys_equal():
    keys = np.full(10, 7, dtype=np.uint64)
    assert O.sample_sort(keys, None, 4, 0, O.INV_COUNT).part_counts.tolist() == [2, 3, 2, 3]
    assert O.sample_sort(keys, None, 4, 0, O.INV_NONE).part_counts.tolist() == [0, 0, 0, 10]


def test_special_cases():
    k = np.array([5, 1, 4], dtype=np.uint64)
    r = O.sample_sort(k, None, 1, 0)
    assert r.part_offsets.tolist() == [0, 3] and r.keys.tolist() == [1, 4, 5]
    r = O.sample_sort(np.zeros(0, dtype=np.uint64), None, 4, 0)
    assert r.part_offsets.tolist() == [0, 0, 0, 0, 0] and r.splitters.tolist() == [0, 0, 0]
    r = O.sample_sort(k, np.arange(3, dtype=np.uint32), 8, 0)   # N < P: empty blocks
    assert r.keys.tolist() == [1, 4, 5] and r.vals.tolist() == [1, 2, 0]
    assert int(r.part_offsets[-1]) == 3


def test_sample_budget_is_one_read_buffer():
    """Section IV.B: each of p processors sends at most 256/p KB, one 256 KB
    buffer in all; the count is the largest multiple of p within it."""
    assert O.default_sample_count(8, 8) == 4096
    assert O.default_sample_count(64, 8) == 512
    assert O.default_sample_count(10, 8) == 3270      # 3276 rounded down to a multiple of 10
    assert O.default_sample_count(52, 8) == 624       # 630 -> 624
    assert O.default_sample_count(8, 4) == 8192
    assert O.default_sample_count(1024, 8) == 32      # budget below P: the budget itself
    for P in (3, 10, 52, 100, 1000):
        s = O.default_sample_count(P, 8)
        assert s * P * 8 <= 262144 and (s % P == 0 or s < P)


# ------------------------------------------------------------------ the handler
def test_handler_pairing_order_of_fig2():
    """Section IV.A with 8 threads: 1->0, 3->2, 5->4, 7->6; then 2->0, 6->4; then 4->0."""
    assert O.handler_schedule(8) == [[(0, 1), (2, 3), (4, 5), (6, 7)], [(0, 2), (4, 6)], [(0, 4)]]
    assert O.handler_schedule(1) == []
    assert O.handler_schedule(3) == [[(0, 1)], [(0, 2)]]


def test_merge_two_against_python_sorted():
    rng = np.random.default_rng(3)
    for _ in range(200):
        a = np.sort(rng.integers(0, 6, size=int(rng.integers(0, 12))).astype(np.uint64))
        b = np.sort(rng.integers(0, 6, size=int(rng.integers(0, 12))).astype(np.uint64))
        tags = [("a", i) for i in range(len(a))] + [("b", j) for j in range(len(b))]
        keyed = [int(x) for x in a] + [int(x) for x in b]
        want = sorted(range(len(tags)), key=lambda t: keyed[t])       # stable: a before b
        va = np.arange(len(a), dtype=np.uint32)
        vb = np.arange(len(a), len(a) + len(b), dtype=np.uint32)
        mk, mv = O.merge_two(a, va, b, vb)
        assert mv.tolist() == want
        assert mk.tolist() == [keyed[t] for t in want]


# ------------------------------------------------------------------ balance
def test_balance_guarantee_adversarial():
    """COUNT: |G_k - kN/P| <= (n/s) ceil(P/2) + P + 1 for any input (n = block
    size, blocks of at least s keys, s >= P/2), so every partition holds at
    most N/P + (N/s)(1 + 1/P) + 2P + 3 keys."""
    rng = np.random.default_rng(13)
    gens = [
        lambda n: np.full(n, 42, dtype=np.uint64),
        lambda n: np.sort(rng.integers(0, 2 ** 63, size=n).astype(np.uint64)),
        lambda n: np.sort(rng.integers(0, 2 ** 63, size=n).astype(np.uint64))[::-1].copy(),
        lambda n: np.where(rng.random(n) < 0.5, np.uint64(7), rng.integers(0, 50, size=n).astype(np.uint64)),
        lambda n: np.repeat(np.arange(n // 97 + 1, dtype=np.uint64), 97)[:n],
        lambda n: (np.arange(n, dtype=np.uint64) % np.uint64(13)) * np.uint64(2 ** 60),
    ]
    for g in gens:
        for P, s, n in [(8, 16, 20000), (16, 8, 30000), (5, 3, 9000), (64, 32, 65536)]:
            keys = g(n)
            r = O.sample_sort(keys, None, P, s, O.INV_COUNT)
            assert int(r.part_counts.max()) <= n / P + (n / s) * (1 + 1 / P) + 2 * P + 3
            assert np.all(np.diff(r.keys.astype(object)) >= 0)


def test_duplicate_heavy_needs_investigator():
    """Fig. 3b vs 3c: without the investigator the duplicates pile up."""
    keys = datagen.duplicate_heavy_keys(200000, seed=3)
    cnt = O.sample_sort(keys, None, 64, 512, O.INV_COUNT).part_counts
    non = O.sample_sort(keys, None, 64, 512, O.INV_NONE).part_counts
    mean = len(keys) / 64
    assert cnt.max() / mean <= 1.05
    assert non.max() / mean > 10


def test_table_t2_uniform_share():
    """Table 2: with P=10 and the 256 KB sample budget the largest share of
    uniform data is at most 10.022% of the total."""
    rows = {}
    with open(os.path.join(GOLD, "table_t2_balance.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, *vals = line.split()
                rows[name] = [float(x) for x in vals]
    bound = max(rows["uniform"]) / 100.0
    assert abs(bound - 0.10022) < 1e-9
    keys = datagen.uniform_keys(4_000_000, seed=21)
    r = O.sample_sort(keys, None, 10, O.default_sample_count(10, 8), O.INV_COUNT)
    share = r.part_counts / len(keys)
    assert share.max() <= bound
    assert abs(share.sum() - 1.0) < 1e-12


# ------------------------------------------------------------------ partition_plan
# partition_plan (steps 1-5 without moving data) is the reference of the
# full-size metadata checks, so it is pinned here: against the whole method
# (sample_sort, itself pinned above by Python's sorted, brute force and the
# worked example) field by field, and directly against brute force.
def _plan_vs_sample_sort(keys, P, s, mode):
    plan = O.partition_plan(keys, P, s, mode)
    r = O.sample_sort(keys, np.arange(len(keys), dtype=np.uint32), P, s, mode)
    assert [x.tolist() for x in plan["samples"]] == [x.tolist() for x in r.samples]
    assert plan["splitters"].tolist() == r.splitters.tolist()
    assert plan["lo"].tolist() == r.lo.tolist() and plan["hi"].tolist() == r.hi.tolist()
    assert plan["cuts"].tolist() == r.cuts.tolist()
    assert plan["send_counts"].tolist() == r.send_counts.tolist()
    assert plan["part_offsets"].tolist() == r.part_offsets.tolist()
    assert plan["part_counts"].tolist() == r.part_counts.tolist()
    assert plan["recv_offsets"].tolist() == r.recv_offsets.tolist()
    return plan


@pytest.mark.parametrize("mode", [O.INV_COUNT, O.INV_NONE, O.INV_PAPER])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64, np.int32, np.int64])
def test_partition_plan_matches_whole_method(mode, dtype):
    rng = np.random.default_rng(101 + mode)
    info = np.iinfo(dtype)
    for trial in range(120):
        n = int(rng.integers(0, 60))
        P = int(rng.integers(1, 12))          # includes N < P
        s = int(rng.integers(0, 7))           # 0: the default budget
        if trial % 3 == 0:                    # heavy duplicates, extremes of the type
            alpha = np.array([info.min, info.min, 0, 1, 1, 1, info.max], dtype=dtype)
            keys = alpha[rng.integers(0, len(alpha), size=n)]
        else:
            keys = rng.integers(info.min, info.max, size=n, dtype=dtype, endpoint=True)
        _plan_vs_sample_sort(keys, P, s, mode)


def test_partition_plan_typed_total_order():
    """Float keys reach partition_plan through their totalOrder integer image,
    as in the full-size float check."""
    from oracle import typed as T
    rng = np.random.default_rng(23)
    specials = np.array([np.nan, -np.nan, np.inf, -np.inf, 0.0, -0.0, 1.5, -1.5], dtype=np.float64)
    for trial in range(80):
        n = int(rng.integers(0, 50))
        P = int(rng.integers(1, 10))
        x = rng.normal(size=n)
        if n:
            x[rng.integers(0, n, size=max(1, n // 4))] = specials[rng.integers(0, len(specials), size=max(1, n // 4))]
        ti = T.total_order_int(x)
        for mode in (O.INV_COUNT, O.INV_NONE, O.INV_PAPER):
            plan = _plan_vs_sample_sort(ti, P, int(rng.integers(1, 6)), mode)
            assert plan["part_offsets"][-1] == n


def test_partition_plan_brute_force():
    """Directly: COUNT offsets are clamp(floor(kN/P), #<v, #<=v); COUNT cuts
    are the block shares of the first G_k stable-order elements; NONE cuts
    are lower bounds; PAPER cuts split each block's equal range into d+1
    pieces; send counts and receive offsets tile the output."""
    rng = np.random.default_rng(29)
    for trial in range(150):
        n = int(rng.integers(0, 45))
        P = int(rng.integers(1, 9))
        s = int(rng.integers(1, 6))
        keys = rand_keys(rng, n, ALPHA if trial % 2 else [4, 4, 4, 7, 9])
        order = brute_stable_order(keys)
        bounds = [i * n // P for i in range(P + 1)]
        blocks = [sorted(int(x) for x in keys[bounds[i]:bounds[i + 1]]) for i in range(P)]
        block_of = [next(b for b in range(P) if bounds[b] <= j < bounds[b + 1]) for j in range(n)]
        for mode in (O.INV_COUNT, O.INV_NONE, O.INV_PAPER):
            plan = O.partition_plan(keys, P, s, mode)
            G, c, C, D = plan["part_offsets"], plan["cuts"], plan["send_counts"], plan["recv_offsets"]
            v = [int(x) for x in plan["splitters"]]
            assert G[0] == 0 and G[P] == n
            for i in range(P):
                assert c[i, 0] == 0 and c[i, P] == len(blocks[i])
                for k in range(1, P):
                    less = sum(1 for x in blocks[i] if x < v[k - 1])
                    leq = sum(1 for x in blocks[i] if x <= v[k - 1])
                    assert plan["lo"][i, k - 1] == less and plan["hi"][i, k - 1] == leq
                    assert less <= c[i, k] <= leq
                    if mode == O.INV_NONE:
                        assert c[i, k] == less
            for k in range(1, P):
                less, leq = brute_counts(keys, v[k - 1])
                if mode == O.INV_COUNT:
                    assert G[k] == min(max(k * n // P, less), leq)
                    first = order[:G[k]]
                    for i in range(P):
                        assert c[i, k] == sum(1 for j in first if block_of[j] == i)
            if mode == O.INV_PAPER:
                k = 1
                while k < P:
                    d = 1
                    while k + d < P and v[k + d - 1] == v[k - 1]:
                        d += 1
                    for i in range(P):
                        lo_i = sum(1 for x in blocks[i] if x < v[k - 1])
                        m = sum(1 for x in blocks[i] if x == v[k - 1])
                        for t in range(d):
                            want = lo_i + ((t + 1) * m // (d + 1) if d > 1 else 0)
                            assert c[i, k + t] == want
                    k += d
            # send counts, offsets and receive offsets tile [0, n) exactly once
            cover = [0] * n
            for i in range(P):
                for k in range(P):
                    assert C[i, k] == c[i, k + 1] - c[i, k]
                    assert G[k] <= D[i, k] and D[i, k] + C[i, k] <= G[k + 1]
                    for j in range(int(D[i, k]), int(D[i, k] + C[i, k])):
                        cover[j] += 1
            assert cover == [1] * n
            assert plan["part_counts"].tolist() == [int(G[k + 1] - G[k]) for k in range(P)]


def test_partition_plan_worked_example():
    common, modes = load_worked_example()
    keys = np.array(common["keys"], dtype=np.uint64)
    P, s = common["P"][0], common["s"][0]
    ids = {"COUNT": O.INV_COUNT, "NONE": O.INV_NONE, "PAPER": O.INV_PAPER}
    for name, exp in modes.items():
        plan = O.partition_plan(keys, P, s, ids[name])
        assert plan["splitters"].tolist() == common["splitters"]
        assert plan["cuts"].tolist() == exp["cuts"]
        assert plan["part_offsets"].tolist() == exp["part_offsets"]
        if "recv_offsets" in exp:
            assert plan["recv_offsets"].tolist() == exp["recv_offsets"]


def test_partition_plan_default_budget():
    """s = 0 takes the default budget; blocks larger than it are sampled
    exactly that many times (512 for 64-bit keys at P = 64, 3270 at P = 10)."""
    rng = np.random.default_rng(31)
    for P, n, want in ((64, 64 * 600 + 17, 512), (10, 10 * 4000 + 3, 3270)):
        keys = rng.integers(0, 2 ** 64, size=n, dtype=np.uint64)
        keys[rng.integers(0, n, size=n // 3)] = 12345
        for mode in (O.INV_COUNT, O.INV_PAPER):
            plan = _plan_vs_sample_sort(keys, P, 0, mode)
            assert all(len(x) == want for x in plan["samples"])


def test_parallel_driver_equals_oracle():
    """The process-parallel driver (steps 1 and 6 over a pool) gives exactly
    the oracle's result."""
    import multiprocessing as mp
    from oracle.parallel import sample_sort_parallel
    rng = np.random.default_rng(37)
    with mp.get_context("spawn").Pool(2) as pool:
        for trial in range(12):
            n = int(rng.integers(0, 3000))
            P = int(rng.integers(1, 12))
            keys = rand_keys(rng, n, ALPHA if trial % 2 else None)
            vals = np.arange(n, dtype=np.uint32) if trial % 3 else None
            for mode in (O.INV_COUNT, O.INV_PAPER):
                a = O.sample_sort(keys, vals, P, 0, mode)
                b = sample_sort_parallel(keys, vals, P, 0, mode, pool=pool)
                assert a.keys.tolist() == b.keys.tolist()
                if vals is not None:
                    assert a.vals.tolist() == b.vals.tolist()
                assert a.part_offsets.tolist() == b.part_offsets.tolist()
                assert a.cuts.tolist() == b.cuts.tolist() and a.splitters.tolist() == b.splitters.tolist()
