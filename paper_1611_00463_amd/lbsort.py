"""Thin Python binding of the lbsort C ABI (ctypes over ``_lib/liblbsort.so``).

Argument marshalling only: every step of the sort runs in the HIP library.
Tensors are torch CUDA (ROCm) tensors used as raw device storage; the calls
are enqueued on torch's current stream.  If the library has not been built,
every call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "liblbsort.so")

U32, U64, I32, I64, F32, F64 = 1, 2, 3, 4, 5, 6
NOVAL, VAL_U32, VAL_INDEX = 0, 1, 2
INV_COUNT, INV_NONE, INV_PAPER = 0, 1, 2
HANDLER_PASSES, HANDLER_ONE_PASS = 1, 2
PRESORTED_DETECT, PRESORTED_IGNORE = 1, 2
OK = 0
ERR_INVALID_ARG, ERR_WORKSPACE_TOO_SMALL, ERR_UNSUPPORTED, ERR_HIP, ERR_OOM, ERR_DEVICE = -1, -2, -3, -4, -5, -6

_c_u64p = ctypes.POINTER(ctypes.c_uint64)


class Params(ctypes.Structure):
    _fields_ = [("P", ctypes.c_uint32), ("s", ctypes.c_uint32), ("investigator", ctypes.c_uint32),
                ("fanin", ctypes.c_uint32), ("merge_tile", ctypes.c_uint32), ("radix_tile", ctypes.c_uint32),
                ("handler", ctypes.c_uint32), ("presorted", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Parts(ctypes.Structure):
    _fields_ = [("part_offsets", ctypes.c_void_p), ("part_counts", ctypes.c_void_p),
                ("splitters", ctypes.c_void_p), ("send_counts", ctypes.c_void_p),
                ("cuts", ctypes.c_void_p)]


EXPORTS = ("lbsort_sort_keys", "lbsort_sort_pairs", "lbsort_sort_batch", "lbsort_local_sort",
           "lbsort_check", "lbsort_status_string", "lbsort_last_error", "lbsort_autotune",
           "lbsort_load_tuning", "lbsort_profile_enable", "lbsort_profile_read", "lbsort_search",
           "lbsort_provenance", "lbsort_sort_pairs_noalloc", "lbsort_resolve_params",
           "lbsort_search_index_bytes", "lbsort_search_build_index", "lbsort_search_indexed")

_lib = None


class LbsortError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbsort error {code}: {msg}")
        self.code = code


def load():
    """Load the in-tree HIP library; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"lbsort HIP library not built ({LIB_PATH}); run paper_1611_00463_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)
    pp, pa = ctypes.POINTER(Params), ctypes.POINTER(Parts)
    lib.lbsort_sort_keys.argtypes = [i32, vp, vp, u64, pp, pa, vp, sz, vp]
    lib.lbsort_sort_pairs.argtypes = [i32, i32, vp, vp, vp, vp, u64, pp, pa, vp, sz, vp]
    lib.lbsort_sort_batch.argtypes = [i32, i32, vp, vp, vp, vp, vp, u32, u64, pp, pa, vp, sz, vp]
    lib.lbsort_local_sort.argtypes = [i32, i32, vp, vp, vp, vp, vp, u32, u64, pp, vp, sz, vp]
    lib.lbsort_check.argtypes = [vp, vp]
    lib.lbsort_status_string.argtypes = [i32]
    lib.lbsort_status_string.restype = ctypes.c_char_p
    lib.lbsort_last_error.restype = ctypes.c_char_p
    lib.lbsort_autotune.argtypes = [i32, i32, vp, vp, vp, u32, u64, u32, ctypes.c_char_p, pp]
    lib.lbsort_resolve_params.argtypes = [i32, i32, u32, u64, pp, pp]
    lib.lbsort_load_tuning.argtypes = [ctypes.c_char_p]
    lib.lbsort_profile_enable.argtypes = [i32]
    lib.lbsort_profile_read.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    lib.lbsort_search.argtypes = [i32, vp, u64, vp, u64, i32, vp, u32, vp, vp, vp]
    lib.lbsort_provenance.argtypes = [vp, u64, u64, u32, vp, vp, vp]
    lib.lbsort_search_index_bytes.argtypes = [i32, u64]
    lib.lbsort_search_index_bytes.restype = ctypes.c_uint64
    lib.lbsort_search_build_index.argtypes = [i32, vp, u64, vp, vp]
    lib.lbsort_search_indexed.argtypes = [i32, vp, u64, vp, vp, u64, i32, vp, u32, vp, vp, vp]
    lib.lbsort_sort_pairs_noalloc.argtypes = [i32, i32, vp, vp, vp, vp, u64, pp, pa, vp, vp]
    for name in EXPORTS:
        getattr(lib, name).restype = getattr(lib, name).restype or ctypes.c_int
    lib.lbsort_status_string.restype = ctypes.c_char_p
    lib.lbsort_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        lib = load()
        raise LbsortError(rc, f"{lib.lbsort_status_string(rc).decode()}: {lib.lbsort_last_error().decode()}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_KEY_CODES = {torch.uint32: U32, torch.uint64: U64, torch.int32: I32, torch.int64: I64,
              torch.float32: F32, torch.float64: F64}


def key_code(dtype) -> int:
    if dtype in _KEY_CODES:
        return _KEY_CODES[dtype]
    raise TypeError(f"keys must be 32- or 64-bit unsigned, signed or float tensors, got {dtype}")


@dataclass
class SortResult:
    keys: torch.Tensor
    vals: torch.Tensor | None
    part_offsets: torch.Tensor      # [B, P+1] (uint64 as int64 storage)
    part_counts: torch.Tensor       # [B, P]
    splitters: torch.Tensor         # [B, P-1]
    send_counts: torch.Tensor | None
    cuts: torch.Tensor | None
    workspace: torch.Tensor


class Workspace:
    """A reusable device workspace that grows on demand."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf


def _params(P, s, investigator, fanin, merge_tile, radix_tile=0, handler=0, presorted=0):
    return Params(P, s, investigator, fanin, merge_tile, radix_tile, handler, presorted, 0)


def _alloc_parts(B, P, kdt, device, want_send, want_cuts):
    offs = torch.empty((B, P + 1), dtype=torch.int64, device=device)
    counts = torch.empty((B, P), dtype=torch.int64, device=device)
    spl = torch.empty((B, max(P - 1, 0)), dtype=kdt, device=device)
    send = torch.empty((B, P, P), dtype=torch.int64, device=device) if want_send else None
    cuts = torch.empty((B, P, P + 1), dtype=torch.int64, device=device) if want_cuts else None
    parts = Parts(offs.data_ptr(), counts.data_ptr(), spl.data_ptr() if P > 1 else None,
                  send.data_ptr() if send is not None else None, cuts.data_ptr() if cuts is not None else None)
    return parts, offs, counts, spl, send, cuts


def _run(fn, args_before_ws, ws: Workspace | None, device):
    """Two-phase workspace protocol: size query, then the call."""
    lib = load()
    need = ctypes.c_size_t(0)
    _check(fn(*args_before_ws, None, ctypes.byref(need), None))
    ws = ws or Workspace(device)
    buf = ws.get(need.value)
    have = ctypes.c_size_t(buf.numel())
    _check(fn(*args_before_ws, ctypes.c_void_p(buf.data_ptr()), ctypes.byref(have), _stream()))
    return buf


def sort_batch(keys: torch.Tensor, seg_offsets: torch.Tensor, P: int, vals: torch.Tensor | None = None,
               s: int = 0, investigator: int = INV_COUNT, fanin: int = 0, merge_tile: int = 0, radix_tile: int = 0, handler: int = 0, presorted: int = 0,
               keys_out=None, vals_out=None, want_send=False, want_cuts=False,
               workspace: Workspace | None = None, index_values: bool = False) -> SortResult:
    """lbsort_sort_batch: seg_offsets is a device tensor of B+1 offsets (int64/uint64).
    index_values=True (with vals=None) sorts with LBSORT_VAL_INDEX."""
    lib = load()
    kc = key_code(keys.dtype)
    B = seg_offsets.numel() - 1
    n = keys.numel()
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    if (vals is not None or index_values) and vals_out is None:
        vals_out = torch.empty(n, dtype=torch.uint32, device=keys.device)
    vt = VAL_U32 if vals is not None else (VAL_INDEX if index_values else NOVAL)
    parts, offs, counts, spl, send, cuts = _alloc_parts(B, P, keys.dtype, keys.device, want_send, want_cuts)
    prm = _params(P, s, investigator, fanin, merge_tile, radix_tile, handler, presorted)
    args = (kc, vt, _ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out),
            _ptr(seg_offsets), B, n, ctypes.byref(prm), ctypes.byref(parts))
    buf = _run(lib.lbsort_sort_batch, args, workspace, keys.device)
    return SortResult(keys_out, vals_out, offs, counts, spl, send, cuts, buf)


def sort_keys(keys: torch.Tensor, P: int, s: int = 0, investigator: int = INV_COUNT, fanin: int = 0,
              merge_tile: int = 0, keys_out=None, want_send=False, want_cuts=False,
              workspace: Workspace | None = None, radix_tile: int = 0, handler: int = 0,
              presorted: int = 0) -> SortResult:
    """lbsort_sort_keys on one array."""
    lib = load()
    kc = key_code(keys.dtype)
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    parts, offs, counts, spl, send, cuts = _alloc_parts(1, P, keys.dtype, keys.device, want_send, want_cuts)
    prm = _params(P, s, investigator, fanin, merge_tile, radix_tile, handler, presorted)
    args = (kc, _ptr(keys), _ptr(keys_out), keys.numel(), ctypes.byref(prm), ctypes.byref(parts))
    buf = _run(lib.lbsort_sort_keys, args, workspace, keys.device)
    return SortResult(keys_out, None, offs, counts, spl, send, cuts, buf)


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor | None, P: int, s: int = 0, investigator: int = INV_COUNT,
               fanin: int = 0, merge_tile: int = 0, radix_tile: int = 0, handler: int = 0, presorted: int = 0, keys_out=None, vals_out=None, want_send=False,
               want_cuts=False, workspace: Workspace | None = None) -> SortResult:
    """lbsort_sort_pairs on one array of keys with uint32 values.  vals=None
    sorts with LBSORT_VAL_INDEX: vals_out receives every key's input position."""
    lib = load()
    kc = key_code(keys.dtype)
    if vals is not None and (vals.dtype != torch.uint32 or vals.numel() != keys.numel()):
        raise TypeError("vals must be torch.uint32 with one value per key")
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    if vals_out is None:
        vals_out = torch.empty(keys.numel(), dtype=torch.uint32, device=keys.device)
    parts, offs, counts, spl, send, cuts = _alloc_parts(1, P, keys.dtype, keys.device, want_send, want_cuts)
    prm = _params(P, s, investigator, fanin, merge_tile, radix_tile, handler, presorted)
    args = (kc, VAL_U32 if vals is not None else VAL_INDEX, _ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out),
            keys.numel(), ctypes.byref(prm), ctypes.byref(parts))
    buf = _run(lib.lbsort_sort_pairs, args, workspace, keys.device)
    return SortResult(keys_out, vals_out, offs, counts, spl, send, cuts, buf)


def local_sort(keys: torch.Tensor, seg_offsets: torch.Tensor, P: int, vals: torch.Tensor | None = None,
               workspace: Workspace | None = None):
    """lbsort_local_sort: step 1 only, every block sorted on its own."""
    lib = load()
    kc = key_code(keys.dtype)
    B = seg_offsets.numel() - 1
    keys_out = torch.empty_like(keys)
    vals_out = torch.empty_like(vals) if vals is not None else None
    prm = _params(P, 0, INV_COUNT, 0, 0)
    args = (kc, VAL_U32 if vals is not None else NOVAL, _ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out),
            _ptr(seg_offsets), B, keys.numel(), ctypes.byref(prm))
    buf = _run(lib.lbsort_local_sort, args, workspace, keys.device)
    return keys_out, vals_out, buf


def search(sorted_keys: torch.Tensor, queries: torch.Tensor, upper: bool = False,
           part_offsets: torch.Tensor | None = None):
    """lbsort_search: positions of the queries in sorted_keys (number of keys
    below, or not above, each query) and, with part_offsets ([P+1] device),
    the partition holding each position (P past the end)."""
    lib = load()
    kc = key_code(sorted_keys.dtype)
    if queries.dtype != sorted_keys.dtype:
        raise TypeError("queries must have the dtype of sorted_keys")
    nq = queries.numel()
    pos = torch.empty(nq, dtype=torch.int64, device=queries.device)
    part = None
    P = 0
    if part_offsets is not None:
        P = part_offsets.numel() - 1
        part = torch.empty(nq, dtype=torch.uint32, device=queries.device)
    _check(lib.lbsort_search(kc, _ptr(sorted_keys), sorted_keys.numel(), _ptr(queries), nq, 1 if upper else 0,
                             _ptr(part_offsets), P, _ptr(pos), _ptr(part), _stream()))
    return pos, part


class SearchIndex:
    """lbsort_search_build_index over sorted_keys (device tensor): the index
    lives in a device buffer of this object and stays valid while
    sorted_keys is unchanged; search() is lbsort_search_indexed."""

    def __init__(self, sorted_keys: torch.Tensor):
        lib = load()
        self.keys = sorted_keys
        self.kc = key_code(sorted_keys.dtype)
        nbytes = int(lib.lbsort_search_index_bytes(self.kc, sorted_keys.numel()))
        # torch's device allocations are 256-byte aligned
        self.buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=sorted_keys.device)
        self.nbytes = nbytes
        _check(lib.lbsort_search_build_index(self.kc, _ptr(sorted_keys), sorted_keys.numel(),
                                             _ptr(self.buf) if nbytes else None, _stream()))

    def search(self, queries: torch.Tensor, upper: bool = False, part_offsets: torch.Tensor | None = None):
        lib = load()
        if queries.dtype != self.keys.dtype:
            raise TypeError("queries must have the dtype of sorted_keys")
        nq = queries.numel()
        pos = torch.empty(nq, dtype=torch.int64, device=queries.device)
        part = None
        P = 0
        if part_offsets is not None:
            P = part_offsets.numel() - 1
            part = torch.empty(nq, dtype=torch.uint32, device=queries.device)
        _check(lib.lbsort_search_indexed(self.kc, _ptr(self.keys), self.keys.numel(),
                                         _ptr(self.buf) if self.nbytes else None, _ptr(queries), nq,
                                         1 if upper else 0, _ptr(part_offsets), P, _ptr(pos), _ptr(part),
                                         _stream()))
        return pos, part


def provenance(src_index: torch.Tensor, n: int, P: int):
    """lbsort_provenance: block (processor) and offset inside it of every
    input position in src_index (uint32), for n keys over P blocks."""
    lib = load()
    if src_index.dtype != torch.uint32:
        raise TypeError("src_index must be torch.uint32")
    cnt = src_index.numel()
    blk = torch.empty(cnt, dtype=torch.uint32, device=src_index.device)
    off = torch.empty(cnt, dtype=torch.uint32, device=src_index.device)
    _check(lib.lbsort_provenance(_ptr(src_index), cnt, n, P, _ptr(blk), _ptr(off), _stream()))
    return blk, off


def check(workspace_buf: torch.Tensor):
    """lbsort_check: synchronise and raise on a device-side error."""
    _check(load().lbsort_check(ctypes.c_void_p(workspace_buf.data_ptr()), _stream()))


def autotune(key_type: int, val_type: int, P: int, total_n: int = 0, B: int = 1, keys: torch.Tensor | None = None,
             vals: torch.Tensor | None = None, seg_offsets: torch.Tensor | None = None,
             cache_path: str | None = None) -> dict:
    """lbsort_autotune: tune on the given batch (keys, vals, seg_offsets
    device tensors; B and total_n taken from them) or, with keys=None, on B
    synthetic uniform instances of total_n / B keys.  Returns the chosen
    settings."""
    lib = load()
    if keys is not None:
        total_n = keys.numel()
        B = 1 if seg_offsets is None else seg_offsets.numel() - 1
    out = Params()
    _check(lib.lbsort_autotune(key_type, val_type, _ptr(keys), _ptr(vals), _ptr(seg_offsets), B, total_n, P,
                               cache_path.encode() if cache_path else None, ctypes.byref(out)))
    return {"fanin": out.fanin, "merge_tile": out.merge_tile, "radix_tile": out.radix_tile, "handler": out.handler,
            "presorted": out.presorted}


def resolve_params(key_type: int, val_type: int, P: int, total_n: int, B: int = 1, s: int = 0,
                   investigator: int = INV_COUNT, fanin: int = 0, merge_tile: int = 0, radix_tile: int = 0,
                   handler: int = 0, presorted: int = 0) -> dict:
    """lbsort_resolve_params: the settings a call of this shape would use."""
    prm = Params(P, s, investigator, fanin, merge_tile, radix_tile, handler, presorted, 0)
    out = Params()
    _check(load().lbsort_resolve_params(key_type, val_type, B, total_n, ctypes.byref(prm), ctypes.byref(out)))
    return {"P": out.P, "s": out.s, "investigator": out.investigator, "fanin": out.fanin,
            "merge_tile": out.merge_tile, "radix_tile": out.radix_tile, "handler": out.handler,
            "presorted": out.presorted}


def load_tuning(cache_path: str):
    _check(load().lbsort_load_tuning(cache_path.encode()))


class BatchPlan:
    """A batched sort of fixed shape (Section IV.C, several data sets at once):
    device buffers, workspace and partition outputs are allocated once, so the
    call can be repeated and captured into a HIP graph (torch.cuda.CUDAGraph
    records the library's launches on the capturing stream).

    keys/vals: device tensors holding every instance back to back;
    seg_offsets: device tensor of B+1 offsets.  Outputs land in self.keys_out,
    self.vals_out and self.part_offsets ([B, P+1], relative to each segment).
    """

    def __init__(self, keys: torch.Tensor, seg_offsets: torch.Tensor, P: int, vals: torch.Tensor | None = None,
                 s: int = 0, investigator: int = INV_COUNT, fanin: int = 0, merge_tile: int = 0, radix_tile: int = 0, handler: int = 0, presorted: int = 0,
                 keys_out=None, vals_out=None):
        lib = load()
        self.keys, self.vals, self.seg = keys, vals, seg_offsets
        self.B = seg_offsets.numel() - 1
        self.P = P
        self.keys_out = torch.empty_like(keys) if keys_out is None else keys_out
        self.vals_out = (torch.empty_like(vals) if vals_out is None else vals_out) if vals is not None else None
        (self._parts, self.part_offsets, self.part_counts, self.splitters, _, _) = _alloc_parts(
            self.B, P, keys.dtype, keys.device, False, False)
        self._prm = _params(P, s, investigator, fanin, merge_tile, radix_tile, handler, presorted)
        self._args = (key_code(keys.dtype), VAL_U32 if vals is not None else NOVAL, _ptr(keys), _ptr(vals),
                      _ptr(self.keys_out), _ptr(self.vals_out), _ptr(seg_offsets), self.B, keys.numel(),
                      ctypes.byref(self._prm), ctypes.byref(self._parts))
        need = ctypes.c_size_t(0)
        _check(lib.lbsort_sort_batch(*self._args, None, ctypes.byref(need), None))
        self.workspace = torch.empty(max(need.value, 256), dtype=torch.uint8, device=keys.device)
        self._have = ctypes.c_size_t(self.workspace.numel())
        self._ws = ctypes.c_void_p(self.workspace.data_ptr())
        self.graph = None

    def run(self):
        """Enqueue the whole batched sort on the current stream."""
        _check(load().lbsort_sort_batch(*self._args, self._ws, ctypes.byref(self._have), _stream()))

    def capture(self):
        """Record the sort into a HIP graph (one launch per replay)."""
        self.run()                      # first run outside the capture (warm-up)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def check(self):
        check(self.workspace)
