"""CPU oracle of the load-balanced sample sort (Khatami et al., arXiv 1611.00463).

TEST INFRASTRUCTURE ONLY.  Nothing in the library may import or call this
module; only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code with the HIP path.

It is a plain, slow, step-by-step rendering of the six steps of Section IV
("Programming Model"), on one machine, with the P processors of the paper as P
virtual processors over contiguous blocks of one array.  numpy's stable sort
and ``searchsorted`` are used as library primitives; everything else is
written out in the paper's order.  Keys are 32- or 64-bit integers,
unsigned or signed, compared by numpy in their own order (floating-point keys
go through ``oracle.typed``); values are opaque uint32 payloads.

Readings where the paper is silent (each is listed with its reason in the
design notes of the repository):

* blocks: block i holds input positions [floor(i N / P), floor((i+1) N / P));
* step 1 uses a *stable* local sort (the paper's quicksort leaves the order
  of equal keys unspecified);
* step 2 takes s_i = min(s, n_i) samples at the chunk starts
  floor(j n_i / s_i), j = 0..s_i-1, the regular sampling of PSRS (Shi and
  Schaeffer 1992), the sample sort the paper builds on;
* step 3 takes splitter k (k = 1..P-1) at rank
  min(S-1, floor(k S / P) + floor(P/2) - 1) of the pooled samples (S = total
  sample count), PSRS's pivot rank: the middle of the k-th group of P pooled
  samples, which does not shift the splitters when all blocks look alike;
* step 4 bounds: partition k takes keys in [v_k, v_{k+1}) before the
  investigator moves cuts inside runs of keys equal to a splitter;
* the investigator (Section IV.B, Fig. 3c) in three modes:
  COUNT (default) divides the global range of keys equal to a duplicated
  splitter so that partition k starts at the global rank nearest
  floor(k N / P) that the splitter allows, filling blocks in block order;
  NONE is plain regular sampling (Fig. 3b); PAPER divides each block's own
  equal-key range into d+1 equal pieces for d equal splitters;
* step 6, the handler (Section IV.A, Fig. 2): rounds of pairwise merges,
  run i+r merged into run i for i = 0 mod 2r, r = 1, 2, 4, ...; ties go to
  the lower run (the left operand).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

INV_COUNT, INV_NONE, INV_PAPER = 0, 1, 2
READ_BUFFER_BYTES = 256 * 1024  # PGX.D read buffer (Section IV.B)


def default_sample_count(P: int, key_bytes: int) -> int:
    """Samples per processor within the budget of Section IV.B: all processors
    together send at most one 256 KB read buffer to Master, 256/p KB each.
    Taken as the largest multiple of P samples within that budget (the budget
    itself if it is below P): then every splitter's target rank k*s/P falls on
    a whole sample, which keeps large, alike blocks from drifting by up to half
    a sample interval per splitter."""
    b = READ_BUFFER_BYTES // (P * key_bytes)
    return b // P * P if b >= P else max(1, b)


def block_bounds(N: int, P: int) -> list[int]:
    """Equal division of the data among the P processors (Section IV.A)."""
    return [i * N // P for i in range(P + 1)]


# ---------------------------------------------------------------- step 1
def local_sort(keys: np.ndarray, vals: np.ndarray | None, bounds: list[int]):
    """Step 1: each processor sorts its own block (stable, ascending)."""
    sk, sv = [], []
    for i in range(len(bounds) - 1):
        a, b = bounds[i], bounds[i + 1]
        order = np.argsort(keys[a:b], kind="stable")
        sk.append(keys[a:b][order])
        sv.append(None if vals is None else vals[a:b][order])
    return sk, sv


# ---------------------------------------------------------------- step 2
def sample_positions(n: int, s: int) -> np.ndarray:
    si = min(s, n)
    j = np.arange(si, dtype=np.int64)
    return (j * n) // si if si > 0 else j


def regular_samples(sorted_block: np.ndarray, s: int) -> np.ndarray:
    """Step 2: regular samples of a locally sorted block."""
    return sorted_block[sample_positions(len(sorted_block), s)]


# ---------------------------------------------------------------- step 3
def select_splitters(samples: list[np.ndarray], P: int, dtype) -> tuple[np.ndarray, np.ndarray]:
    """Step 3: Master pools all samples and picks P-1 splitters."""
    pool = np.sort(np.concatenate(samples).astype(dtype), kind="stable") if samples else np.zeros(0, dtype)
    S = len(pool)
    v = np.zeros(max(P - 1, 0), dtype=dtype)
    if S > 0:
        for k in range(1, P):
            v[k - 1] = pool[min(S - 1, k * S // P + P // 2 - 1)]
    return v, pool


# ---------------------------------------------------------------- step 4
def search(sorted_blocks: list[np.ndarray], splitters: np.ndarray):
    """Step 4: binary search of every splitter in every locally sorted block.
    lo[i][k-1] = #keys < v_k, hi[i][k-1] = #keys <= v_k in block i."""
    P = len(sorted_blocks)
    lo = np.zeros((P, max(P - 1, 0)), dtype=np.int64)
    hi = np.zeros_like(lo)
    for i, blk in enumerate(sorted_blocks):
        if P > 1:
            lo[i] = np.searchsorted(blk, splitters, side="left")
            hi[i] = np.searchsorted(blk, splitters, side="right")
    return lo, hi


def investigator(lo: np.ndarray, hi: np.ndarray, sizes: list[int], splitters: np.ndarray,
                 mode: int = INV_COUNT) -> np.ndarray:
    """Step 4 continued: cut positions c[i][k], k = 0..P, in each sorted block.
    Block i sends [c[i][k], c[i][k+1]) to processor k."""
    P = len(sizes)
    N = sum(sizes)
    c = np.zeros((P, P + 1), dtype=np.int64)
    for i in range(P):
        c[i, P] = sizes[i]
    if P == 1:
        return c
    if mode == INV_NONE:
        c[:, 1:P] = lo
    elif mode == INV_COUNT:
        for k in range(1, P):
            L = int(lo[:, k - 1].sum())
            H = int(hi[:, k - 1].sum())
            G = min(max(k * N // P, L), H)
            extra = G - L
            for i in range(P):
                m = int(hi[i, k - 1] - lo[i, k - 1])
                take = min(m, max(0, extra))
                extra -= take
                c[i, k] = lo[i, k - 1] + take
    elif mode == INV_PAPER:
        k = 1
        while k < P:
            d = 1
            while k + d < P and splitters[k + d - 1] == splitters[k - 1]:
                d += 1
            for i in range(P):
                base = int(lo[i, k - 1])
                m = int(hi[i, k - 1] - lo[i, k - 1])
                if d == 1:
                    c[i, k] = base
                else:
                    for t in range(d):
                        c[i, k + t] = base + ((t + 1) * m) // (d + 1)
            k += d
    else:
        raise ValueError("unknown investigator mode")
    return c


# ---------------------------------------------------------------- step 5
def exchange(cuts: np.ndarray):
    """Step 5 bookkeeping: send counts C[i][k], partition offsets G[k] and the
    receive offsets D[i][k] at which processor k stores what block i sends
    (the ranges are broadcast, so every receiver knows its offsets; Section IV.C)."""
    P = cuts.shape[0]
    C = cuts[:, 1:] - cuts[:, :-1]
    G = np.zeros(P + 1, dtype=np.int64)
    G[1:] = np.cumsum(C.sum(axis=0))
    D = np.zeros((P, P), dtype=np.int64)
    for k in range(P):
        D[:, k] = G[k] + np.concatenate(([0], np.cumsum(C[:, k])[:-1]))
    return C, G, D


def exchange_receive(sorted_blocks, sorted_vals, cuts: np.ndarray, C: np.ndarray, D: np.ndarray, N: int):
    """Step 5 itself: every block writes its slice for processor k at the
    receive offset D[i][k]; all writes land in disjoint places, so they can
    happen at once (Section IV.C).  Returns the receive buffer(s)."""
    P = cuts.shape[0]
    dtype = sorted_blocks[0].dtype if P else np.uint64
    rk = np.zeros(N, dtype=dtype)
    rv = None if sorted_vals[0] is None else np.zeros(N, dtype=np.uint32)
    written = np.zeros(N, dtype=np.int64)
    for i in range(P):
        for k in range(P):
            a, c = int(cuts[i, k]), int(C[i, k])
            rk[D[i, k]:D[i, k] + c] = sorted_blocks[i][a:a + c]
            if rv is not None:
                rv[D[i, k]:D[i, k] + c] = sorted_vals[i][a:a + c]
            written[D[i, k]:D[i, k] + c] += 1
    assert np.all(written == 1), "receive offsets must tile the output exactly once"
    return rk, rv


# ---------------------------------------------------------------- step 6
def handler_schedule(n_runs: int) -> list[list[tuple[int, int]]]:
    """Fig. 2: round r (r = 1, 2, 4, ...) merges run i+r into run i for every
    i that is a multiple of 2r.  Returns rounds of (destination, source)."""
    rounds = []
    r = 1
    while r < n_runs:
        rounds.append([(i, i + r) for i in range(0, n_runs, 2 * r) if i + r < n_runs])
        r *= 2
    return rounds


def merge_two(ak, av, bk, bv):
    """Stable merge of two sorted runs, ties to the left run: the output
    position of a[i] is i + #(b < a[i]); that of b[j] is j + #(a <= b[j])."""
    n = len(ak) + len(bk)
    pa = np.arange(len(ak)) + np.searchsorted(bk, ak, side="left")
    pb = np.arange(len(bk)) + np.searchsorted(ak, bk, side="right")
    ok = np.empty(n, dtype=ak.dtype)
    ok[pa] = ak
    ok[pb] = bk
    ov = None
    if av is not None:
        ov = np.empty(n, dtype=av.dtype)
        ov[pa] = av
        ov[pb] = bv
    return ok, ov


def handler_merge(run_keys: list[np.ndarray], run_vals: list[np.ndarray | None]):
    """Step 6: merge the received runs with the balanced handler of Fig. 2."""
    rk = list(run_keys)
    rv = list(run_vals)
    for rnd in handler_schedule(len(rk)):
        for dst, src in rnd:
            rk[dst], rv[dst] = merge_two(rk[dst], rv[dst], rk[src], rv[src])
    return rk[0], rv[0]


@dataclass
class SortResult:
    keys: np.ndarray
    vals: np.ndarray | None
    part_offsets: np.ndarray       # G_0..G_P
    part_counts: np.ndarray        # G_{k+1} - G_k
    splitters: np.ndarray          # v_1..v_{P-1}
    send_counts: np.ndarray        # C[i][k]
    cuts: np.ndarray               # c[i][k], k = 0..P
    samples: list = field(default_factory=list)
    sorted_blocks: list = field(default_factory=list)
    sorted_vals: list = field(default_factory=list)
    lo: np.ndarray | None = None
    hi: np.ndarray | None = None
    recv_offsets: np.ndarray | None = None


def partition_plan(keys: np.ndarray, P: int, s: int = 0, mode: int = INV_COUNT) -> dict:
    """Steps 1-5 without moving any data: sorted blocks (keys only), samples,
    splitters, searches, cuts and the range table.  Used where the whole
    merge would take too long on the CPU."""
    keys = np.asarray(keys)
    N = len(keys)
    if s <= 0:
        s = default_sample_count(P, keys.dtype.itemsize)
    bounds = block_bounds(N, P)
    sizes = [bounds[i + 1] - bounds[i] for i in range(P)]
    sk, _ = local_sort(keys, None, bounds)
    samples = [regular_samples(b, s) for b in sk]
    splitters, _ = select_splitters(samples, P, keys.dtype)
    lo, hi = search(sk, splitters)
    cuts = investigator(lo, hi, sizes, splitters, mode)
    C, G, D = exchange(cuts)
    return dict(samples=samples, splitters=splitters, lo=lo, hi=hi, cuts=cuts, send_counts=C,
                part_offsets=G, part_counts=np.diff(G), recv_offsets=D)


def sample_sort(keys: np.ndarray, vals: np.ndarray | None, P: int, s: int = 0,
                mode: int = INV_COUNT) -> SortResult:
    """The whole method on one array: steps 1 to 6 of Section IV."""
    keys = np.asarray(keys)
    dtype = keys.dtype
    assert dtype in (np.uint32, np.uint64, np.int32, np.int64)
    N = len(keys)
    if s <= 0:
        s = default_sample_count(P, dtype.itemsize)
    bounds = block_bounds(N, P)
    sizes = [bounds[i + 1] - bounds[i] for i in range(P)]
    sk, sv = local_sort(keys, vals, bounds)                       # step 1
    samples = [regular_samples(b, s) for b in sk]                 # step 2
    splitters, _ = select_splitters(samples, P, dtype)            # step 3
    lo, hi = search(sk, splitters)                                # step 4
    cuts = investigator(lo, hi, sizes, splitters, mode)
    C, G, D = exchange(cuts)                                      # step 5
    recv_k, recv_v = exchange_receive(sk, sv, cuts, C, D, N)
    out_k = np.empty(N, dtype=dtype)
    out_v = None if vals is None else np.empty(N, dtype=vals.dtype)
    for k in range(P):                                            # step 6
        rk = [recv_k[D[i, k]:D[i, k] + C[i, k]] for i in range(P)]
        rv = [None if vals is None else recv_v[D[i, k]:D[i, k] + C[i, k]] for i in range(P)]
        mk, mv = handler_merge(rk, rv)
        out_k[G[k]:G[k + 1]] = mk
        if vals is not None:
            out_v[G[k]:G[k + 1]] = mv
    return SortResult(keys=out_k, vals=out_v, part_offsets=G, part_counts=np.diff(G),
                      splitters=splitters, send_counts=C, cuts=cuts, samples=samples,
                      sorted_blocks=sk, sorted_vals=sv, lo=lo, hi=hi, recv_offsets=D)

