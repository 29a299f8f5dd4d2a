"""Process-parallel driver of the CPU oracle, for timing it on all host cores.

TEST INFRASTRUCTURE ONLY.  Only the tests and the ``cpu_baseline`` leg of
``bench.py`` use it; nothing in the library may import or call it.  It shares
no code with the HIP path.

It runs the oracle's own step functions of ``oracle.sample_sort`` in the
order of Section IV, unchanged, and only spreads the two steps that are
independent per processor over a pool of worker processes: step 1 (each
processor sorts its own block) and step 6 (each processor merges the runs it
received with the handler).  Steps 2-5 (samples, splitters, search and
investigator, the exchange) run in the calling process, as the paper's Master
and range broadcast would.  The result equals ``sample_sort`` exactly.
"""
from __future__ import annotations

import multiprocessing as mp

import numpy as np

from oracle import sample_sort as O


def _step1(task):
    keys, vals = task
    sk, sv = O.local_sort(keys, vals, [0, len(keys)])
    return sk[0], sv[0]


def _step6(task):
    run_keys, run_vals = task
    return O.handler_merge(run_keys, run_vals)


def sample_sort_parallel(keys: np.ndarray, vals: np.ndarray | None, P: int, s: int = 0, mode: int = O.INV_COUNT,
                         workers: int = 1, pool=None) -> O.SortResult:
    """``oracle.sample_sort`` with steps 1 and 6 mapped over `workers`
    processes (a given `pool` is used instead of starting one)."""
    keys = np.asarray(keys)
    dtype = keys.dtype
    N = len(keys)
    if s <= 0:
        s = O.default_sample_count(P, dtype.itemsize)
    bounds = O.block_bounds(N, P)
    sizes = [bounds[i + 1] - bounds[i] for i in range(P)]
    own = pool is None
    if own:
        pool = mp.get_context("spawn").Pool(workers)
    try:
        tasks = [(keys[bounds[i]:bounds[i + 1]], None if vals is None else vals[bounds[i]:bounds[i + 1]])
                 for i in range(P)]
        res = pool.map(_step1, tasks, chunksize=1)                     # step 1
        sk = [r[0] for r in res]
        sv = [r[1] for r in res]
        samples = [O.regular_samples(b, s) for b in sk]                 # step 2
        splitters, _ = O.select_splitters(samples, P, dtype)            # step 3
        lo, hi = O.search(sk, splitters)                                # step 4
        cuts = O.investigator(lo, hi, sizes, splitters, mode)
        C, G, D = O.exchange(cuts)                                      # step 5
        recv_k, recv_v = O.exchange_receive(sk, sv, cuts, C, D, N)
        tasks = []
        for k in range(P):
            rk = [recv_k[D[i, k]:D[i, k] + C[i, k]] for i in range(P)]
            rv = [None if vals is None else recv_v[D[i, k]:D[i, k] + C[i, k]] for i in range(P)]
            tasks.append((rk, rv))
        merged = pool.map(_step6, tasks, chunksize=1)                   # step 6
    finally:
        if own:
            pool.close()
            pool.join()
    out_k = np.empty(N, dtype=dtype)
    out_v = None if vals is None else np.empty(N, dtype=vals.dtype)
    for k, (mk, mv) in enumerate(merged):
        out_k[G[k]:G[k + 1]] = mk
        if vals is not None:
            out_v[G[k]:G[k + 1]] = mv
    return O.SortResult(keys=out_k, vals=out_v, part_offsets=G, part_counts=np.diff(G), splitters=splitters,
                        send_counts=C, cuts=cuts, samples=samples, sorted_blocks=sk, sorted_vals=sv, lo=lo, hi=hi,
                        recv_offsets=D)
