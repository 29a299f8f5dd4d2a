"""Seeded synthetic inputs shared by the tests, the bench and the oracle's timing.

This module only draws numbers.  It holds none of the sort's arithmetic, so the
CPU oracle and the HIP path can both be fed from it without sharing any code
of the method itself.

Every stream is counter based: ``u64(seed, i)`` is output ``i`` of a SplitMix64
generator (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) whose state starts at ``seed``:

    z  = seed + (i + 1) * 0x9E3779B97F4A7C15          (mod 2**64)
    z  = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z  = (z ^ (z >> 27)) * 0x94D049BB133111EB
    out = z ^ (z >> 31)

so any element can be recomputed on its own, on the host or on the device.

The workloads stand in for the paper's inputs (Section V: uniform, normal,
right-skewed and exponential data sets, one billion entries, and a Twitter
graph), which are not available here; the shapes below are synthetic.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= M1
        z ^= z >> np.uint64(27)
        z *= M2
        z ^= z >> np.uint64(31)
    return z


def u64(seed: int, idx) -> np.ndarray:
    """SplitMix64 output number ``idx`` (array or scalar) of the stream ``seed``."""
    i = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (i + np.uint64(1)) * GAMMA
    return _mix(z)


def u64_range(seed: int, start: int, count: int) -> np.ndarray:
    return u64(seed, np.arange(start, start + count, dtype=np.uint64))


def unit_double(bits: np.ndarray) -> np.ndarray:
    """Top 53 bits of a u64 as a double in [0, 1)."""
    return (bits >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# --------------------------------------------------------------------------
# Plain inputs
# --------------------------------------------------------------------------

def uniform_keys(n: int, seed: int, dtype=np.uint64, start: int = 0) -> np.ndarray:
    k = u64_range(seed, start, n)
    if dtype == np.uint32:
        return (k >> np.uint64(32)).astype(np.uint32)
    return k


def index_values(n: int, start: int = 0) -> np.ndarray:
    """Payload equal to the input index (so stability can be read off the output)."""
    return np.arange(start, start + n, dtype=np.uint32)


def zipf_cdf(n_ranks: int, s: float) -> np.ndarray:
    w = 1.0 / np.power(np.arange(1, n_ranks + 1, dtype=np.float64), s)
    c = np.cumsum(w)
    return c / c[-1]


def zipf_ranks(bits: np.ndarray, cdf: np.ndarray) -> np.ndarray:
    """Inverse-CDF draw of ranks 1..len(cdf) from 53-bit uniforms."""
    u = unit_double(bits)
    r = np.searchsorted(cdf, u, side="right") + 1
    return np.minimum(r, len(cdf)).astype(np.uint64)


def duplicate_heavy_keys(n: int, seed: int = 3, zipf_s: float = 1.1,
                         n_values: int = 1000, start: int = 0) -> np.ndarray:
    """Half the keys equal one value V, the rest Zipf(s) over ``n_values`` values.

    The top bit of ``u64(seed, i)`` picks V = u64(seed*11, 0); otherwise the
    remaining bits draw a Zipf rank r and the key is u64(seed*11 + 1, r).  V is
    checked to differ from every Zipf value.
    """
    u = u64_range(seed, start, n)
    heavy = np.uint64(u64(seed * 11, 0))
    cdf = zipf_cdf(n_values, zipf_s)
    ranks = zipf_ranks(u << np.uint64(1), cdf)
    table = u64(seed * 11 + 1, np.arange(0, n_values + 1, dtype=np.uint64))
    assert not np.any(table[1:] == heavy)
    keys = table[ranks]
    top = (u >> np.uint64(63)) == np.uint64(1)
    keys[top] = heavy
    return keys


def normal_u32(n: int, seed: int, start: int = 0) -> np.ndarray:
    """clamp(round(2^31 + 2^29 z)) with z ~ N(0,1) by Box-Muller on two streams."""
    a = unit_double(u64_range(seed, start, n))
    b = unit_double(u64_range(seed + 0x5bd1e995, start, n))
    z = np.sqrt(-2.0 * np.log1p(-a)) * np.cos(2.0 * math.pi * b)
    v = np.rint(2.0 ** 31 + 2.0 ** 29 * z)
    return np.clip(v, 0, 2 ** 32 - 1).astype(np.uint32)


# --------------------------------------------------------------------------
# Batched instances
# --------------------------------------------------------------------------

BATCH_DISTS = ("uniform", "normal", "sorted", "reverse")


def batch_sizes(B: int, seed: int, lo: int = 1024, hi: int = 4194304) -> np.ndarray:
    """n_b = floor(exp(U(ln lo, ln hi))), log-uniform instance sizes."""
    u = unit_double(u64_range(seed, 0, B))
    n = np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo))))
    return np.clip(n, lo, hi).astype(np.int64)


def batch_dist_ids(B: int, seed: int) -> np.ndarray:
    return (u64_range(seed + 1, 0, B) % np.uint64(4)).astype(np.int64)


def batch_instance_keys_u32(b: int, n: int, dist: int, seed: int) -> np.ndarray:
    s = (seed * 1000003 + b * 7919 + 17) & 0xFFFFFFFFFFFFFFFF
    if dist == 0:
        return uniform_keys(n, s, np.uint32)
    if dist == 1:
        return normal_u32(n, s)
    k = np.sort(uniform_keys(n, s, np.uint32))
    return k if dist == 2 else k[::-1].copy()


def batch_u32(B: int, seed: int = 4, lo: int = 1024, hi: int = 4194304):
    """Keys (u32), values (local index, u32) and seg_offsets[B+1] of a batch."""
    sizes = batch_sizes(B, seed, lo, hi)
    dists = batch_dist_ids(B, seed)
    offs = np.zeros(B + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes).astype(np.uint64)
    keys = np.empty(int(offs[-1]), dtype=np.uint32)
    vals = np.empty(int(offs[-1]), dtype=np.uint32)
    for b in range(B):
        a, e = int(offs[b]), int(offs[b + 1])
        keys[a:e] = batch_instance_keys_u32(b, e - a, int(dists[b]), seed)
        vals[a:e] = np.arange(e - a, dtype=np.uint32)
    return keys, vals, offs


# --------------------------------------------------------------------------
# Serving request stream
# --------------------------------------------------------------------------

SERVE_DISTS = ("uniform", "zipf", "sorted", "reverse")


def serve_requests(n_req: int, seed: int = 5, rate_per_s: float = 2000.0,
                   lo: int = 10000, hi: int = 67108864):
    """Poisson arrivals (exponential gaps), log-uniform sizes, distribution ids."""
    gaps = -np.log1p(-unit_double(u64_range(seed, 0, n_req))) / rate_per_s
    arrivals = np.cumsum(gaps)
    sizes = batch_sizes(n_req, seed + 2, lo, hi)
    dists = (u64_range(seed + 3, 0, n_req) % np.uint64(4)).astype(np.int64)
    return arrivals, sizes, dists


def serve_pool_u64(dist: int, n: int, seed: int = 5) -> np.ndarray:
    s = seed * 101 + dist
    if dist == 0:
        return uniform_keys(n, s)
    if dist == 1:
        cdf = zipf_cdf(1000000, 1.2)
        r = zipf_ranks(u64_range(s, 0, n), cdf)
        return u64(s + 7, r)
    k = np.sort(uniform_keys(n, s))
    return k if dist == 2 else k[::-1].copy()


# --------------------------------------------------------------------------
# Stand-ins for the four input distributions of Section V (uniform, normal,
# right-skewed, exponential; Table 2 and the sample-size study).  The paper
# gives no parameters, so these are chosen here, and built from integer
# operations only, so that the host and the device draw the same bytes:
#   uniform      U64
#   normal       Irwin-Hall: the sum of four independent 62-bit uniforms
#                (bell-shaped around 2^63)
#   right_skewed (U >> 43)^3 >> 47: a 21-bit uniform cubed and cut to 16 bits,
#                mass near zero and a long right tail, many repeated keys
#   exponential  the number of leading zero bits of a uniform u64: a discrete
#                exponential (geometric) law, P(k) = 2^-(k+1), so half of the
#                keys share one value
# --------------------------------------------------------------------------
BALANCE_DISTS = ("uniform", "normal", "right_skewed", "exponential")


def _clz64(x: np.ndarray) -> np.ndarray:
    k = np.zeros(x.shape, dtype=np.uint64)
    y = x.copy()
    for sh in (32, 16, 8, 4, 2, 1):
        m = (y >> np.uint64(64 - sh)) == 0
        k[m] += np.uint64(sh)
        y[m] <<= np.uint64(sh)
    k[x == 0] = np.uint64(64)
    return k


def balance_keys(dist: str, n: int, seed: int = 6, start: int = 0) -> np.ndarray:
    """u64 keys [start, start + n) of one of BALANCE_DISTS."""
    i = np.arange(start, start + n, dtype=np.uint64)
    if dist == "uniform":
        return u64(seed, i)
    if dist == "normal":
        acc = np.zeros(n, dtype=np.uint64)
        for j in range(4):
            acc += u64(seed + 1000 * (j + 1), i) >> np.uint64(2)
        return acc
    if dist == "right_skewed":
        u = u64(seed, i) >> np.uint64(43)
        with np.errstate(over="ignore"):
            return (u * u * u) >> np.uint64(47)
    if dist == "exponential":
        return _clz64(u64(seed, i))
    raise ValueError(dist)


# --------------------------------------------------------------------------
# The same streams generated on the device with torch int64 arithmetic
# (wrapping multiply, logical shifts by masking); bit-identical to u64().
# --------------------------------------------------------------------------

def _i64(c: int) -> int:
    c &= 0xFFFFFFFFFFFFFFFF
    return c - (1 << 64) if c >= (1 << 63) else c


def _lsr(z, s: int):
    return (z >> s) & ((1 << (64 - s)) - 1)


def u64_torch(seed: int, start: int, count: int, device="cuda"):
    import torch
    i = torch.arange(start, start + count, dtype=torch.int64, device=device)
    z = (i + 1) * _i64(0x9E3779B97F4A7C15) + _i64(seed)
    z = (z ^ _lsr(z, 30)) * _i64(0xBF58476D1CE4E5B9)
    z = (z ^ _lsr(z, 27)) * _i64(0x94D049BB133111EB)
    z = z ^ _lsr(z, 31)
    return z.view(torch.uint64)


def uniform_keys_torch(n: int, seed: int, device="cuda", chunk: int = 1 << 26):
    """uniform_keys(n, seed) as a device tensor, generated in chunks."""
    import torch
    out = torch.empty(n, dtype=torch.uint64, device=device)
    for a in range(0, n, chunk):
        e = min(n, a + chunk)
        out[a:e] = u64_torch(seed, a, e - a, device)
    return out


def index_values_torch(n: int, device="cuda"):
    import torch
    return torch.arange(n, dtype=torch.int64, device=device).to(torch.int32).view(torch.uint32)


def batch_u32_torch(B: int, seed: int = 4, lo: int = 1024, hi: int = 4194304, device="cuda"):
    """batch_u32 generated on the device: the same sizes and distribution ids;
    uniform, sorted and reverse instances are bit-identical to batch_u32, normal
    instances use the same formula in device float64 (last-bit rounding of the
    transcendental functions may differ from the host)."""
    import torch
    sizes = batch_sizes(B, seed, lo, hi)
    dists = batch_dist_ids(B, seed)
    offs = np.zeros(B + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    total = int(offs[-1])
    keys = torch.empty(total, dtype=torch.int64, device=device)
    for b in range(B):
        a, e = int(offs[b]), int(offs[b + 1])
        n = e - a
        sb = (seed * 1000003 + b * 7919 + 17) & 0xFFFFFFFFFFFFFFFF
        d = int(dists[b])
        if d == 1:
            ua = _lsr(u64_torch(sb, 0, n, device).view(torch.int64), 11).double() * (1.0 / 9007199254740992.0)
            ub = _lsr(u64_torch(sb + 0x5bd1e995, 0, n, device).view(torch.int64), 11).double() * (1.0 / 9007199254740992.0)
            z = torch.sqrt(-2.0 * torch.log1p(-ua)) * torch.cos(2.0 * math.pi * ub)
            k = torch.clamp(torch.round(2.0 ** 31 + 2.0 ** 29 * z), 0, 2 ** 32 - 1).to(torch.int64)
        else:
            k = _lsr(u64_torch(sb, 0, n, device).view(torch.int64), 32)
            if d >= 2:
                k = torch.sort(k).values
                if d == 3:
                    k = torch.flip(k, dims=[0])
        keys[a:e] = k
    keys32 = keys.to(torch.int32).view(torch.uint32)
    del keys
    local = torch.arange(total, dtype=torch.int64, device=device)
    seg_of = torch.repeat_interleave(torch.arange(B, device=device), torch.from_numpy(sizes).to(device))
    vals = (local - torch.from_numpy(offs[:-1]).to(device)[seg_of]).to(torch.int32).view(torch.uint32)
    return keys32, vals, torch.from_numpy(offs.astype(np.uint64)).to(device), sizes


def u64_torch_at(seed: int, idx):
    """u64(seed, idx) for an int64 index tensor, on idx's device."""
    import torch
    z = (idx + 1) * _i64(0x9E3779B97F4A7C15) + _i64(seed)
    z = (z ^ _lsr(z, 30)) * _i64(0xBF58476D1CE4E5B9)
    z = (z ^ _lsr(z, 27)) * _i64(0x94D049BB133111EB)
    return (z ^ _lsr(z, 31)).view(torch.uint64)


def serve_pool_u64_torch(dist: int, n: int, seed: int = 5, device="cuda"):
    """serve_pool_u64 generated on the device (same definition)."""
    import torch
    s = seed * 101 + dist
    if dist == 1:
        cdf = torch.from_numpy(zipf_cdf(1000000, 1.2)).to(device)
        u = _lsr(u64_torch(s, 0, n, device).view(torch.int64), 11).double() * (1.0 / 9007199254740992.0)
        r = torch.clamp(torch.searchsorted(cdf, u, right=True) + 1, max=len(cdf))
        return u64_torch_at(s + 7, r.to(torch.int64))
    k = uniform_keys_torch(n, s, device)
    if dist == 0:
        return k
    flip = -(1 << 63)
    srt = (torch.sort(k.view(torch.int64) ^ flip).values ^ flip).view(torch.uint64)
    return srt if dist == 2 else torch.flip(srt.view(torch.int64), dims=[0]).view(torch.uint64)


def _clz64_torch(x):
    import torch
    k = torch.zeros_like(x)
    y = x.clone()
    for sh in (32, 16, 8, 4, 2, 1):
        m = _lsr(y, 64 - sh) == 0
        k = torch.where(m, k + sh, k)
        y = torch.where(m, y << sh, y)
    return torch.where(x == 0, torch.full_like(x, 64), k)


def balance_keys_torch(dist: str, n: int, seed: int = 6, device="cuda", chunk: int = 1 << 26):
    """balance_keys(dist, n, seed) generated on the device (bit-identical)."""
    import torch
    out = torch.empty(n, dtype=torch.int64, device=device)
    for a in range(0, n, chunk):
        e = min(n, a + chunk)
        if dist == "uniform":
            v = u64_torch(seed, a, e - a, device).view(torch.int64)
        elif dist == "normal":
            v = torch.zeros(e - a, dtype=torch.int64, device=device)
            for j in range(4):
                v += _lsr(u64_torch(seed + 1000 * (j + 1), a, e - a, device).view(torch.int64), 2)
        elif dist == "right_skewed":
            u = _lsr(u64_torch(seed, a, e - a, device).view(torch.int64), 43)
            v = _lsr(u * u * u, 47)
        elif dist == "exponential":
            v = _clz64_torch(u64_torch(seed, a, e - a, device).view(torch.int64))
        else:
            raise ValueError(dist)
        out[a:e] = v
    return out.view(torch.uint64)


# --------------------------------------------------------------------------
# Signed and floating-point keys
# --------------------------------------------------------------------------
# Floats: Irwin-Hall of four uniforms (an approximately normal shape, like the
# balance study's "normal"), centred and scaled: (u1 + u2 + u3 + u4 - 2) * 1000.
# Only IEEE additions and multiplications in a fixed order, so host (numpy)
# and device (torch) produce the same bits.  Every SPECIAL_EVERY-th key is one
# of SPECIALS in turn (NaNs of both signs, infinities, signed zeros).
SPECIAL_EVERY = 9973
SPECIALS_F64 = (0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000000, 0xFFF0000000000000,
                0x0000000000000000, 0x8000000000000000)


def _specials(dtype) -> np.ndarray:
    b = np.array(SPECIALS_F64, dtype=np.uint64).view(np.float64)
    return b.astype(dtype) if dtype == np.float32 else b


def typed_keys(n: int, seed: int, dtype, start: int = 0) -> np.ndarray:
    """n keys of dtype (int32, int64, float32 or float64): signed integers are
    uniform bit patterns; floats as described above."""
    i = np.arange(start, start + n, dtype=np.uint64)
    if dtype in (np.int64, np.int32):
        k = u64(seed, i)
        return (k >> np.uint64(32)).astype(np.uint32).view(np.int32) if dtype == np.int32 else k.view(np.int64)
    acc = unit_double(u64(seed + 1000, i))
    for j in range(1, 4):
        acc = acc + unit_double(u64(seed + 1000 * (j + 1), i))
    x = ((acc - 2.0) * 1000.0).astype(dtype)
    sp = (i % np.uint64(SPECIAL_EVERY)) == 0
    x[sp] = _specials(dtype)[(i[sp] // np.uint64(SPECIAL_EVERY)) % np.uint64(6)]
    return x


def typed_keys_torch(n: int, seed: int, dtype, device="cuda", chunk: int = 1 << 25):
    """typed_keys(n, seed, dtype) generated on the device, bit for bit."""
    import torch
    tdt = {np.int32: torch.int32, np.int64: torch.int64, np.float32: torch.float32,
           np.float64: torch.float64}[dtype]
    out = torch.empty(n, dtype=tdt, device=device)
    sp64 = torch.tensor(np.array(SPECIALS_F64, dtype=np.uint64).view(np.int64), device=device).view(torch.float64)
    sp = sp64.to(tdt) if dtype == np.float32 else sp64
    scale = 1.0 / 9007199254740992.0
    for a in range(0, n, chunk):
        e = min(n, a + chunk)
        if dtype in (np.int64, np.int32):
            k = u64_torch(seed, a, e - a, device).view(torch.int64)
            out[a:e] = _lsr(k, 32).to(torch.int32) if dtype == np.int32 else k
            continue
        acc = _lsr(u64_torch(seed + 1000, a, e - a, device).view(torch.int64), 11).double() * scale
        for j in range(1, 4):
            acc = acc + _lsr(u64_torch(seed + 1000 * (j + 1), a, e - a, device).view(torch.int64), 11).double() * scale
        x = ((acc - 2.0) * 1000.0).to(tdt)
        idx = torch.arange(a, e, dtype=torch.int64, device=device)
        m = (idx % SPECIAL_EVERY) == 0
        x[m] = sp[(idx[m] // SPECIAL_EVERY) % 6]
        out[a:e] = x
    return out
