"""CPU oracle of the sort library's typed keys, provenance and search
(Khatami et al., arXiv 1611.00463, Section III and Section IV.C).

TEST INFRASTRUCTURE ONLY.  Nothing in the library may import or call this
module; only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code with the HIP path.

The paper's interface is generic over the data type (Section IV.C, and the
conclusions), reports for every sorted entry the processor and the index it
came from (step 6 of Section IV and Section IV.C), and offers a binary search
over the sorted data (Section III, Section IV.C).  Here:

* signed integer keys are ordered as numbers (numpy's own comparison);
* floating-point keys are ordered by IEEE 754-2008 totalOrder (clause 5.10):
  -NaN < -inf < negative numbers < -0 < +0 < positive numbers < +inf < +NaN,
  NaNs among themselves by payload.  numpy's float sort puts NaNs last and
  treats -0 and +0 as equal, so it is not used for them; the bit patterns are
  mapped to signed integers whose numeric order is totalOrder and sorted as
  those;
* the provenance of an output entry is its position in the input before the
  sort, split into the block (processor) that held it and its offset inside
  that block;
* a search returns, per query, the number of sorted keys below it (or not
  above it) and the partition that holds that position.
"""
from __future__ import annotations

import numpy as np

from oracle import sample_sort as O

FLOAT_TYPES = {np.dtype(np.float32): (np.uint32, np.int32, 32), np.dtype(np.float64): (np.uint64, np.int64, 64)}


def total_order_int(keys: np.ndarray) -> np.ndarray:
    """Signed integers in IEEE 754 totalOrder of the float keys (binary32 or
    binary64).  An IEEE binary number with sign bit s and magnitude field m
    (exponent and fraction bits, read as an unsigned integer) has a value that
    grows with m, so totalOrder is: by m when s = 0, by -m when s = 1, every
    s = 1 pattern below every s = 0 pattern.  Mapping s = 0 to m and s = 1 to
    -1 - m realises exactly that (-0, m = 0, goes to -1, just below +0)."""
    udt, sdt, w = FLOAT_TYPES[keys.dtype]
    bits = keys.view(udt)
    mag = (bits & udt((1 << (w - 1)) - 1)).astype(sdt)
    neg = (bits >> udt(w - 1)) != 0
    return np.where(neg, -1 - mag, mag).astype(sdt)


def from_total_order_int(t: np.ndarray, float_dtype) -> np.ndarray:
    """Inverse of ``total_order_int``: the float whose bit pattern maps to t."""
    udt, sdt, w = FLOAT_TYPES[np.dtype(float_dtype)]
    t = np.asarray(t, dtype=sdt)
    neg = t < 0
    mag = np.where(neg, -1 - t, t).astype(udt)
    bits = mag | np.where(neg, udt(1 << (w - 1)), udt(0)).astype(udt)
    return bits.view(float_dtype)


def comparable(keys: np.ndarray) -> np.ndarray:
    """Keys in a form numpy compares in the key type's order."""
    if keys.dtype in FLOAT_TYPES:
        return total_order_int(keys)
    return keys


def sample_sort_typed(keys: np.ndarray, vals, P: int, s: int = 0, mode: int = O.INV_COUNT) -> O.SortResult:
    """The whole method (Section IV, steps 1-6) on keys of any of the six
    types: unsigned and signed integers as they are, floats through their
    totalOrder integers.  Sorted keys and splitters come back as the original
    type; the partition metadata does not depend on the key type."""
    keys = np.asarray(keys)
    if keys.dtype not in FLOAT_TYPES:
        return O.sample_sort(keys, vals, P, s, mode)
    if s <= 0:
        s = O.default_sample_count(P, keys.dtype.itemsize)
    r = O.sample_sort(total_order_int(keys), vals, P, s, mode)
    r.keys = from_total_order_int(r.keys, keys.dtype)
    r.splitters = from_total_order_int(r.splitters, keys.dtype)
    return r


def provenance(src_index: np.ndarray, n: int, P: int):
    """Processor (block) and offset inside the block of input position g, for
    the equal division of Section IV.A: block i holds [floor(i n/P),
    floor((i+1) n/P)); g lies in the last block whose start is <= g."""
    bounds = np.array(O.block_bounds(n, P), dtype=np.int64)
    g = np.asarray(src_index, dtype=np.int64)
    blk = np.searchsorted(bounds, g, side="right") - 1
    return blk.astype(np.uint32), (g - bounds[blk]).astype(np.uint32)


def search(sorted_keys: np.ndarray, queries: np.ndarray, upper: bool, part_offsets=None):
    """Binary search over the sorted output (Section III, Section IV.C).
    pos[j] = number of sorted keys < queries[j] (upper=False) or <= queries[j]
    (upper=True), in the key type's order.  part[j] = the partition k with
    G_k <= pos[j] < G_{k+1}, and P when pos[j] = n (past the last key)."""
    sk = comparable(np.asarray(sorted_keys))
    q = comparable(np.asarray(queries))
    pos = np.searchsorted(sk, q, side="right" if upper else "left").astype(np.uint64)
    if part_offsets is None:
        return pos, None
    G = np.asarray(part_offsets, dtype=np.uint64)
    P = len(G) - 1
    n = len(sorted_keys)
    part = (np.searchsorted(G, pos, side="right") - 1).astype(np.int64)
    part[pos == np.uint64(n)] = P
    return pos, part.astype(np.uint32)
