"""The allocation-free entry point (lbsort_sort_pairs_noalloc) against the
workspace entry point (lbsort_sort_pairs), through the C ABI: every output bit
for bit, on calls in a row where a later call is smaller than an earlier one
(the static scratch keeps the previous call's contents), plus the size limit,
which is checked on the host before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import sample_sort as O
from paper_1611_00463_amd import datagen
from paper_1611_00463_amd import lbsort as L
from tests.parity import assert_same, u64

SCRATCH = 64 << 20


def _parts(P, kdt):
    offs = torch.full((P + 1,), -1, dtype=torch.int64, device="cuda")
    counts = torch.full((P,), -1, dtype=torch.int64, device="cuda")
    spl = torch.zeros((max(P - 1, 1),), dtype=kdt, device="cuda")
    send = torch.full((P * P,), -1, dtype=torch.int64, device="cuda")
    cuts = torch.full((P * (P + 1),), -1, dtype=torch.int64, device="cuda")
    parts = L.Parts(offs.data_ptr(), counts.data_ptr(), spl.data_ptr() if P > 1 else None, send.data_ptr(),
                    cuts.data_ptr())
    return parts, dict(offs=offs, counts=counts, spl=spl, send=send, cuts=cuts)


def run_noalloc(keys, vals, P, val_type, s=0, mode=O.INV_COUNT):
    lib = L.load()
    n = keys.numel()
    kout = torch.empty_like(keys)
    vout = torch.empty(n, dtype=torch.uint32, device="cuda") if val_type != L.NOVAL else None
    parts, out = _parts(P, keys.dtype)
    err = torch.full((1,), 0xFFFF, dtype=torch.int32, device="cuda")
    prm = L.Params(P, s, mode, 0, 0, 0)
    rc = lib.lbsort_sort_pairs_noalloc(L.key_code(keys.dtype), val_type, L._ptr(keys), L._ptr(vals), L._ptr(kout),
                                       L._ptr(vout), n, ctypes.byref(prm), ctypes.byref(parts), L._ptr(err),
                                       L._stream())
    L._check(rc)
    torch.cuda.synchronize()
    assert int(err.item()) == 0, f"device error bits {int(err.item()):#x}"
    return kout, vout, out


def run_ws(keys, vals, P, val_type, s=0, mode=O.INV_COUNT):
    lib = L.load()
    n = keys.numel()
    kout = torch.empty_like(keys)
    vout = torch.empty(n, dtype=torch.uint32, device="cuda") if val_type != L.NOVAL else None
    parts, out = _parts(P, keys.dtype)
    prm = L.Params(P, s, mode, 0, 0, 0)
    args = (L.key_code(keys.dtype), val_type, L._ptr(keys), L._ptr(vals), L._ptr(kout), L._ptr(vout), n,
            ctypes.byref(prm), ctypes.byref(parts))
    need = ctypes.c_size_t(0)
    L._check(lib.lbsort_sort_pairs(*args, None, ctypes.byref(need), None))
    ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda")
    have = ctypes.c_size_t(ws.numel())
    L._check(lib.lbsort_sort_pairs(*args, ctypes.c_void_p(ws.data_ptr()), ctypes.byref(have), L._stream()))
    L.check(ws)
    return kout, vout, out


def same(a, b, P):
    ka, va, oa = a
    kb, vb, ob = b
    assert torch.equal(ka.view(torch.uint8), kb.view(torch.uint8)), "keys differ"
    if va is not None:
        assert torch.equal(va.view(torch.int32), vb.view(torch.int32)), "values differ"
    for name in ("offs", "counts", "send", "cuts"):
        assert torch.equal(oa[name], ob[name]), name
    if P > 1:
        assert torch.equal(oa["spl"].view(torch.uint8), ob["spl"].view(torch.uint8)), "splitters"


CASES = [
    # (key dtype, value type, n of the first call, n of the second, P)
    ("u64", L.VAL_U32, 5_000_000, 1_000_003, 64),
    ("u64", L.NOVAL, 3_000_017, 40_000, 8),
    ("u32", L.VAL_U32, 7_000_000, 4097, 13),
    ("f64", L.VAL_INDEX, 2_500_000, 300_001, 64),
]


@pytest.mark.gpu
@pytest.mark.parametrize("kt,vt,n1,n2,P", CASES)
def test_noalloc_equals_workspace_entry_point(kt, vt, n1, n2, P):
    print(f"[noalloc] {kt} vt={vt} n={n1} then {n2} P={P}", flush=True)
    for i, n in enumerate((n1, n2)):
        if kt == "u64":
            keys = datagen.uniform_keys_torch(n, 60 + i, "cuda")
        elif kt == "u32":
            keys = datagen.uniform_keys_torch(n, 70 + i, "cuda").view(torch.int64).remainder(1 << 20).to(
                torch.int32).view(torch.uint32)
        else:
            keys = datagen.typed_keys_torch(n, 80 + i, np.float64, "cuda")
        vals = datagen.index_values_torch(n, "cuda") if vt == L.VAL_U32 else None
        a = run_noalloc(keys, vals, P, vt)
        b = run_ws(keys, vals, P, vt)
        same(a, b, P)
        if i == 1 and kt == "u64":
            # the smaller call also against the oracle
            kn = keys.cpu().numpy()
            vn = vals.cpu().numpy() if vals is not None else None
            o = O.sample_sort(kn, vn, P, 0)
            assert_same("keys", a[0].cpu().numpy(), o.keys)
            if vn is not None:
                assert_same("vals", a[1].cpu().numpy(), o.vals)
            assert_same("part_offsets", u64(a[2]["offs"]), o.part_offsets.astype(np.uint64))
            assert_same("cuts", u64(a[2]["cuts"]).reshape(P, P + 1), o.cuts.astype(np.uint64))


@pytest.mark.gpu
def test_noalloc_empty_and_tiny():
    for n in (0, 1, 7):
        keys = datagen.uniform_keys_torch(max(n, 1), 90, "cuda")[:n].contiguous()
        vals = datagen.index_values_torch(n, "cuda")
        same(run_noalloc(keys, vals, 4, L.VAL_U32), run_ws(keys, vals, 4, L.VAL_U32), 4)


def test_noalloc_rejects_beyond_scratch_on_host():
    lib = L.load()
    prm = L.Params(64, 0, 0, 0, 0, 0)
    parts = L.Parts(1, 0, 0, 0, 0)
    rc = lib.lbsort_sort_pairs_noalloc(L.U64, L.VAL_U32, None, None, None, None, 1 << 28, ctypes.byref(prm),
                                       ctypes.byref(parts), None, None)
    assert rc == L.ERR_UNSUPPORTED
    assert b"scratch" in lib.lbsort_last_error()
    # a size that fits passes the size check and fails only on the null pointers
    need = ctypes.c_size_t(0)
    assert lib.lbsort_sort_pairs(L.U64, L.VAL_U32, None, None, None, None, 5_000_000, ctypes.byref(prm),
                                 ctypes.byref(parts), None, ctypes.byref(need), None) == 0
    assert need.value <= SCRATCH
