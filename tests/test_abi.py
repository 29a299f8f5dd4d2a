"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1611_00463_amd import lbsort as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbsort.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(lbsort_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_1611_00463_amd import build
        build.build()
    return L.load()


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert set(names) >= {"lbsort_sort_keys", "lbsort_sort_pairs", "lbsort_sort_batch"}
    for n in names:
        assert hasattr(lib, n), n
    assert set(L.EXPORTS) == set(names)


def test_status_strings(lib):
    assert lib.lbsort_status_string(0) == b"ok"
    assert lib.lbsort_status_string(-2) == b"workspace too small"
    assert lib.lbsort_status_string(12345) == b"unknown status"


def _size(key_type=L.U64, P=8, n=1000, **kw):
    prm = L.Params(P, kw.get("s", 0), kw.get("inv", 0), kw.get("fanin", 0), kw.get("tile", 0), kw.get("rtile", 0),
                   kw.get("handler", 0), kw.get("presorted", 0), kw.get("reserved", 0))
    parts = L.Parts(1, 0, 0, 0, 0)
    need = ctypes.c_size_t(0)
    rc = L.load().lbsort_sort_keys(key_type, None, None, n, ctypes.byref(prm), ctypes.byref(parts), None,
                                   ctypes.byref(need), None)
    return rc, need.value


def test_workspace_query_and_growth(lib):
    rc, a = _size(n=1 << 20)
    assert rc == 0 and a > 0
    rc, b = _size(n=1 << 22)
    assert rc == 0 and b > a
    rc, c = _size(n=0)
    assert rc == 0 and c > 0


@pytest.mark.parametrize("kw,code", [
    (dict(key_type=7), L.ERR_INVALID_ARG),
    (dict(P=0), L.ERR_INVALID_ARG),
    (dict(P=5000), L.ERR_INVALID_ARG),
    (dict(inv=9), L.ERR_INVALID_ARG),
    (dict(fanin=3), L.ERR_INVALID_ARG),
    (dict(tile=1000), L.ERR_INVALID_ARG),
    (dict(rtile=1000), L.ERR_INVALID_ARG),
    (dict(rtile=2048), L.ERR_INVALID_ARG),
    (dict(rtile=16384), L.ERR_INVALID_ARG),                  # 64-bit keys: no 16384-key tiles
    (dict(reserved=1), L.ERR_INVALID_ARG),
    (dict(handler=3), L.ERR_INVALID_ARG),
    (dict(presorted=3), L.ERR_INVALID_ARG),
    (dict(handler=2, P=65), L.ERR_UNSUPPORTED),
    (dict(handler=2, P=64, fanin=16), L.ERR_INVALID_ARG),
    (dict(handler=2, P=64, tile=1024), L.ERR_INVALID_ARG),
    (dict(handler=2, P=8, n=(1 << 32) + 1), L.ERR_UNSUPPORTED),
    (dict(s=(1 << 20) + 1), L.ERR_INVALID_ARG),
    (dict(n=1 << 45), L.ERR_UNSUPPORTED),
    (dict(P=1, n=1 << 33), L.ERR_UNSUPPORTED),
])
def test_rejects_bad_arguments(lib, kw, code):
    rc, _ = _size(**kw)
    assert rc == code
    assert lib.lbsort_last_error()


def test_workspace_too_small_and_misaligned(lib):
    rc, need = _size(n=1 << 16)
    assert rc == 0
    prm = L.Params(8, 0, 0, 0, 0, 0)
    parts = L.Parts(1, 0, 0, 0, 0)
    small = ctypes.c_size_t(need - 1)
    rc = lib.lbsort_sort_keys(L.U64, ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), 1 << 16, ctypes.byref(prm),
                              ctypes.byref(parts), ctypes.c_void_p(1 << 30), ctypes.byref(small), None)
    assert rc == L.ERR_WORKSPACE_TOO_SMALL
    big = ctypes.c_size_t(need)
    rc = lib.lbsort_sort_keys(L.U64, ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), 1 << 16, ctypes.byref(prm),
                              ctypes.byref(parts), ctypes.c_void_p((1 << 30) + 8), ctypes.byref(big), None)
    assert rc == L.ERR_INVALID_ARG


def test_missing_required_outputs(lib):
    rc, need = _size(n=100)
    prm = L.Params(4, 0, 0, 0, 0, 0)
    parts = L.Parts(0, 0, 0, 0, 0)
    big = ctypes.c_size_t(need)
    rc = lib.lbsort_sort_keys(L.U64, ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), 100, ctypes.byref(prm),
                              ctypes.byref(parts), ctypes.c_void_p(1 << 30), ctypes.byref(big), None)
    assert rc == L.ERR_INVALID_ARG
    rc = lib.lbsort_sort_keys(L.U64, None, None, 100, ctypes.byref(prm), None, ctypes.c_void_p(1 << 30),
                              ctypes.byref(big), None)
    assert rc == L.ERR_INVALID_ARG


@pytest.mark.parametrize("signed,unsigned", [(L.I64, L.U64), (L.F64, L.U64), (L.I32, L.U32), (L.F32, L.U32)])
def test_typed_keys_share_the_unsigned_layout(lib, signed, unsigned):
    for n in (0, 1000, 1 << 20):
        rc_a, a = _size(key_type=signed, n=n)
        rc_b, b = _size(key_type=unsigned, n=n)
        assert rc_a == 0 and rc_b == 0 and a == b


def test_index_values_need_32bit_positions(lib):
    prm = L.Params(1, 0, 0, 0, 0, 0)
    parts = L.Parts(1, 0, 0, 0, 0)
    need = ctypes.c_size_t(0)
    rc = lib.lbsort_sort_pairs(L.U64, L.VAL_INDEX, None, None, None, None, (1 << 32) + 1, ctypes.byref(prm),
                               ctypes.byref(parts), None, ctypes.byref(need), None)
    assert rc == L.ERR_UNSUPPORTED
    rc = lib.lbsort_sort_pairs(L.U64, L.VAL_INDEX, None, None, None, None, 1 << 20, ctypes.byref(prm),
                               ctypes.byref(parts), None, ctypes.byref(need), None)
    assert rc == 0 and need.value > 0
    rc = lib.lbsort_sort_pairs(L.U64, 3, None, None, None, None, 10, ctypes.byref(prm), ctypes.byref(parts), None,
                               ctypes.byref(need), None)
    assert rc == L.ERR_INVALID_ARG


def test_search_and_provenance_argument_checks(lib):
    p = ctypes.c_void_p(1 << 20)
    # nothing to do: no device work, success
    assert lib.lbsort_search(L.U64, None, 0, None, 0, 0, None, 0, None, None, None) == 0
    assert lib.lbsort_provenance(None, 0, 10, 4, None, None, None) == 0
    assert lib.lbsort_search(7, p, 10, p, 5, 0, None, 0, p, None, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_search(L.U64, p, 10, p, 5, 2, None, 0, p, None, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_search(L.U64, p, 10, None, 5, 0, None, 0, p, None, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_search(L.U64, p, 10, p, 5, 0, None, 4, p, p, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_provenance(p, 5, 10, 0, p, p, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_provenance(p, 5, (1 << 32) + 1, 4, p, p, None) == L.ERR_UNSUPPORTED
    assert lib.lbsort_provenance(p, 5, 10, 4, None, None, None) == L.ERR_INVALID_ARG


def test_search_index_sizes_and_argument_checks(lib):
    """Index bytes: levels of ceil(n_{l-1} / 16) keys up to the first of at
    most 16, each rounded up to 128 bytes (written out here from that rule);
    argument errors are found on the host before any device work."""
    def want(n, kb):
        tot, m = 0, n
        while m > 16:
            m = -(-m // 16)
            tot += -(-(m * kb) // 128) * 128
        return tot
    for n in (0, 1, 16, 17, 256, 257, 4096, 65537, 1 << 28, 10 ** 9 + 7):
        assert lib.lbsort_search_index_bytes(L.U64, n) == want(n, 8), n
        assert lib.lbsort_search_index_bytes(L.F32, n) == want(n, 4), n
    # 2^28 u64 keys: levels of 2^24, 2^20, 2^16, 2^12, 2^8 and 16 keys
    assert lib.lbsort_search_index_bytes(L.U64, 1 << 28) == 8 * (2 ** 24 + 2 ** 20 + 2 ** 16 + 2 ** 12 + 256) + 128
    assert lib.lbsort_search_index_bytes(9, 100) == 0
    p = ctypes.c_void_p(1 << 20)
    odd = ctypes.c_void_p((1 << 20) + 64)
    assert lib.lbsort_search_build_index(L.U64, None, 16, None, None) == 0        # no index needed
    assert lib.lbsort_search_build_index(9, p, 100, p, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_search_build_index(L.U64, p, 100, None, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_search_build_index(L.U64, p, 100, odd, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_search_indexed(L.U64, None, 0, None, None, 0, 0, None, 0, None, None, None) == 0
    assert lib.lbsort_search_indexed(L.U64, p, 100, None, p, 5, 0, None, 0, p, None, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_search_indexed(L.U64, p, 100, p, p, 5, 2, None, 0, p, None, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_search_indexed(L.U64, p, 100, p, p, 5, 0, None, 4, p, p, None) == L.ERR_INVALID_ARG


def test_resolve_params_defaults_and_explicit(lib):
    """Without a tuned entry (no device here) the defaults: F = 8 for P > 16,
    else the power of two reaching P (at most 16); merge tile 2048; radix tile
    8192; s = the paper's budget.  Explicit settings pass through."""
    r = L.resolve_params(L.U64, L.VAL_U32, 64, 1 << 28)
    assert r == {"P": 64, "s": 512, "investigator": 0, "fanin": 8, "merge_tile": 2048, "radix_tile": 8192,
                 "handler": L.HANDLER_PASSES, "presorted": L.PRESORTED_DETECT}
    r = L.resolve_params(L.U64, L.VAL_U32, 37, 1 << 20, handler=L.HANDLER_ONE_PASS)
    assert r["handler"] == L.HANDLER_ONE_PASS and r["fanin"] == 64 and r["merge_tile"] == 4096
    assert L.resolve_params(L.U64, L.NOVAL, 128, 1 << 20)["handler"] == L.HANDLER_PASSES
    assert L.resolve_params(L.U32, L.VAL_U32, 8, 1 << 20, B=4096)["fanin"] == 8
    assert L.resolve_params(L.U64, L.NOVAL, 5, 1000)["fanin"] == 8
    assert L.resolve_params(L.U64, L.NOVAL, 3, 1000)["fanin"] == 4
    r = L.resolve_params(L.F64, L.VAL_INDEX, 10, 10 ** 6, s=7, investigator=2, fanin=4, merge_tile=1024,
                         radix_tile=4096)
    assert r == {"P": 10, "s": 7, "investigator": 2, "fanin": 4, "merge_tile": 1024, "radix_tile": 4096,
                 "handler": L.HANDLER_PASSES, "presorted": L.PRESORTED_DETECT}
    assert L.resolve_params(L.U64, L.NOVAL, 10, 1000, presorted=L.PRESORTED_IGNORE)["presorted"] == L.PRESORTED_IGNORE
    r = L.resolve_params(L.U64, L.NOVAL, 10, 10 ** 6, handler=L.HANDLER_ONE_PASS, merge_tile=2048)
    assert r["handler"] == L.HANDLER_ONE_PASS and r["fanin"] == 16 and r["merge_tile"] == 2048
    with pytest.raises(L.LbsortError):
        L.resolve_params(L.U64, L.NOVAL, 8, 100, radix_tile=5)


def test_radix_tile_sizes_the_workspace(lib):
    """Smaller radix tiles need more look-back status words."""
    def need(rt):
        prm = L.Params(8, 0, 0, 0, 0, rt, 0, 0, 0)
        parts = L.Parts(1, 0, 0, 0, 0)
        n = ctypes.c_size_t(0)
        assert lib.lbsort_sort_keys(L.U64, None, None, 1 << 22, ctypes.byref(prm), ctypes.byref(parts), None,
                                    ctypes.byref(n), None) == 0
        return n.value
    assert need(4096) > need(8192) == need(0)
    # 32-bit keys also take tiles of 16384 keys (fewer status words)
    def need32(rt):
        prm = L.Params(8, 0, 0, 0, 0, rt, 0, 0, 0)
        parts = L.Parts(1, 0, 0, 0, 0)
        n = ctypes.c_size_t(0)
        assert lib.lbsort_sort_keys(L.F32, None, None, 1 << 22, ctypes.byref(prm), ctypes.byref(parts), None,
                                    ctypes.byref(n), None) == 0
        return n.value
    assert need32(8192) > need32(16384)


def test_autotune_argument_checks(lib):
    # rejected before any device work
    assert lib.lbsort_autotune(7, 0, None, None, None, 1, 100, 8, None, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_autotune(L.U64, 0, None, None, None, 1, 0, 8, None, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_autotune(L.U64, 0, None, None, None, 0, 100, 8, None, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_autotune(L.U64, 0, ctypes.c_void_p(256), None, None, 2, 100, 8, None, None) == L.ERR_INVALID_ARG
    assert lib.lbsort_autotune(L.U64, 1, ctypes.c_void_p(256), None, None, 1, 100, 8, None, None) == L.ERR_INVALID_ARG
