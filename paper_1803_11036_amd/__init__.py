"""MI355X sliding super point detector (arXiv 1803.11036), Python binding.

A thin ctypes binding of the C ABI declared in ``include/ssd.h``: the names
match the C calls without their ``ssd_`` prefix, and every function only
marshals arguments -- the hot path (scan, hot detection, candidate expansion,
verification, sort, merge) runs in the HIP kernels of ``libssd.so``.  PyTorch
provides device memory and streams.

The library must be built (``__graft_entry__.build()`` or
``python -m paper_1803_11036_amd.build``); importing this package without it
raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

__all__ = [
    "SSD_VERIFY_REHASH", "SSD_ADVANCE_ONLY", "SSDError", "Params", "make_params",
    "query_sizes", "Detector", "init_detector", "scan_slice", "scan_slice_noalloc", "close_slice", "close_begin", "close_end",
    "get_results", "merge_router_state", "read_canonical_state", "read_rk", "export_state", "import_state",
    "read_hot", "read_tuples", "get_info", "set_tuning", "destroy",
    "SSD_TUNE_SCAN_PASS_BYTES", "SSD_TUNE_SORT_BLOCK_LIMIT", "SSD_TUNE_TIMING", "read_timing",
    "SSD_TUNE_SCAN_TILE_PAIRS", "SSD_TUNE_GRAPH", "SSD_TUNE_AUTOTUNE", "PHASES",
    "SSD_TUNE_SCAN_MODE", "SSD_TUNE_SCAN_BIN_BYTES", "SSD_TUNE_SCAN_APPLY_SEGMENTS", "SSD_SCAN_PASSES",
    "SSD_SCAN_BINNED", "SSD_SCAN_AUTO", "SSD_TUNE_COUNTED", "SSD_TUNE_COUNTED_MIN_ITEMS",
    "Batch", "batch_query_sizes", "batch_init", "batch_scan", "batch_close", "batch_close_begin",
    "batch_close_end", "batch_get_results",
    "batch_set_tuning", "batch_get_tuning", "batch_read_timing", "batch_get_info", "batch_read_rk",
    "batch_read_hot", "batch_destroy",
    "Group", "group_query_sizes", "group_init", "group_scan", "group_close", "group_close_begin",
    "group_close_end", "group_destroy",
    "library_path", "RESULT_DTYPE",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libssd.so")

SSD_ABI_VERSION = 1
SSD_VERIFY_REHASH = 0x1
SSD_ADVANCE_ONLY = 0x1
SSD_E_PARAM, SSD_E_NOMEM, SSD_E_ORDER, SSD_E_OVERFLOW, SSD_E_INCOMPAT, SSD_E_TRUNC, SSD_E_DEVICE, SSD_E_STATE = \
    -1, -2, -3, -4, -5, -6, -7, -8
SSD_NOALLOC_SCRATCH_BYTES = 64 << 20
STATE_HEADER_BYTES = 80            # the checkpoint blob's header (ssd_export_state)

RESULT_DTYPE = np.dtype([("ip", "<u4"), ("rk", "<u4"), ("est", "<f8")])


class Params(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("q", C.c_uint32), ("r", C.c_uint32),
                ("delta", C.c_uint32), ("eta", C.c_uint32), ("k", C.c_uint32),
                ("theta", C.c_uint32), ("key_bits", C.c_uint32), ("flags", C.c_uint32),
                ("cell_bits", C.c_uint32), ("max_tuples", C.c_uint64), ("max_results", C.c_uint64)]


class _SuperPoint(C.Structure):
    _fields_ = [("ip", C.c_uint32), ("rk", C.c_uint32), ("est", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("open_slice", C.c_uint64), ("hot_threshold", C.c_uint32), ("r", C.c_uint32),
                ("state_bytes", C.c_uint64), ("level_counts", C.c_uint64 * 16),
                ("hot_counts", C.c_uint32 * 16), ("accepted", C.c_uint64), ("reported", C.c_uint64),
                ("counted", C.c_uint32), ("counted_bin_kib", C.c_uint32)]


assert C.sizeof(_SuperPoint) == RESULT_DTYPE.itemsize == 16


class SSDError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


def library_path() -> str:
    return _LIB_PATH


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(_LIB_PATH)
        vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
        u64p = C.POINTER(C.c_uint64)
        L.ssd_query_sizes.argtypes = [C.POINTER(Params), u64p, u64p]
        L.ssd_init_detector.argtypes = [C.POINTER(Params), C.POINTER(C.c_uint32), vp, u64, vp, u64, vp,
                                        C.POINTER(vp)]
        L.ssd_scan_slice.argtypes = [vp, vp, u64, u64]
        L.ssd_scan_slice_noalloc.argtypes = [vp, vp, u64, u64]
        L.ssd_close_slice.argtypes = [vp, u32, vp, u64, u64p]
        L.ssd_get_results.argtypes = [vp, vp, u64, u64p]
        L.ssd_close_begin.argtypes = [vp]
        L.ssd_close_end.argtypes = [vp, vp, u64, u64p]
        L.ssd_merge_router_state.argtypes = [vp, C.POINTER(vp), u32]
        L.ssd_read_canonical_state.argtypes = [vp, vp, u64]
        L.ssd_export_state.argtypes = [vp, vp, u64, u64p]
        L.ssd_import_state.argtypes = [vp, vp, u64]
        L.ssd_read_rk.argtypes = [vp, vp, u64]
        L.ssd_read_hot.argtypes = [vp, vp, vp, u64]
        L.ssd_read_tuples.argtypes = [vp, vp, u64, u64p]
        L.ssd_get_info.argtypes = [vp, C.POINTER(_Info)]
        L.ssd_set_tuning.argtypes = [vp, u32, u64]
        L.ssd_read_timing.argtypes = [vp, vp, vp, C.c_int]
        L.ssd_batch_query_sizes.argtypes = [vp, u32, u64p, u64p]
        L.ssd_batch_init.argtypes = [vp, u32, vp, vp, u64, vp, u64, vp, C.POINTER(vp)]
        L.ssd_batch_scan.argtypes = [vp, vp, vp, u64]
        L.ssd_batch_close.argtypes = [vp, vp, u64, vp, vp]
        L.ssd_batch_close_begin.argtypes = [vp]
        L.ssd_batch_close_end.argtypes = [vp, vp, u64, vp, vp]
        L.ssd_batch_get_results.argtypes = [vp, vp, u64, vp, vp]
        L.ssd_batch_set_tuning.argtypes = [vp, u32, u64]
        L.ssd_batch_get_tuning.argtypes = [vp, u32, u64p]
        L.ssd_batch_read_timing.argtypes = [vp, vp, vp, C.c_int]
        L.ssd_batch_get_info.argtypes = [vp, u32, C.POINTER(_Info)]
        L.ssd_batch_read_rk.argtypes = [vp, u32, vp, u64]
        L.ssd_batch_read_hot.argtypes = [vp, u32, vp, vp, u64]
        L.ssd_batch_destroy.argtypes = [vp]
        L.ssd_batch_destroy.restype = None
        L.ssd_group_query_sizes.argtypes = [u32, u64p]
        L.ssd_group_init.argtypes = [u32, vp, u64, vp, C.POINTER(vp)]
        L.ssd_group_scan.argtypes = [vp, C.POINTER(vp), u32, vp, vp, vp]
        L.ssd_group_close.argtypes = [vp, C.POINTER(vp), u32, vp, u64, vp, vp]
        L.ssd_group_close_begin.argtypes = [vp, C.POINTER(vp), u32]
        L.ssd_group_close_end.argtypes = [vp, vp, u64, vp, vp]
        L.ssd_group_destroy.argtypes = [vp]
        L.ssd_group_destroy.restype = None
        L.ssd_destroy.argtypes = [vp]
        L.ssd_destroy.restype = None
        L.ssd_strerror.argtypes = [C.c_int]
        L.ssd_strerror.restype = C.c_char_p
        L.ssd_last_error.argtypes = []
        L.ssd_last_error.restype = C.c_char_p
        for name in ("ssd_query_sizes", "ssd_init_detector", "ssd_scan_slice", "ssd_scan_slice_noalloc",
                     "ssd_close_slice",
                     "ssd_get_results", "ssd_merge_router_state", "ssd_read_canonical_state",
                     "ssd_read_rk", "ssd_read_hot", "ssd_read_tuples", "ssd_get_info",
                     "ssd_set_tuning", "ssd_read_timing", "ssd_batch_query_sizes", "ssd_batch_init",
                     "ssd_batch_scan", "ssd_batch_close", "ssd_batch_get_results", "ssd_batch_set_tuning",
                     "ssd_batch_get_tuning", "ssd_batch_read_timing", "ssd_batch_get_info", "ssd_batch_read_rk", "ssd_batch_read_hot",
                     "ssd_group_query_sizes",
                     "ssd_group_init", "ssd_group_scan", "ssd_group_close", "ssd_group_close_begin",
                     "ssd_group_close_end", "ssd_export_state", "ssd_import_state", "ssd_batch_close_begin",
                     "ssd_batch_close_end"):
            getattr(L, name).restype = C.c_int
        _lib_handle = L
    return _lib_handle


def _check(status: int, where: str) -> None:
    if status != 0:
        L = _lib()
        raise SSDError(status, where, L.ssd_last_error().decode() or L.ssd_strerror(status).decode())


def make_params(q: int, r: int, delta: int, eta: int, k: int, theta: int, key_bits: int = 32,
                verify_rehash: bool = False, max_tuples: int = 1 << 22, max_results: int = 1 << 20,
                cell_bits: int = 8) -> Params:
    return Params(SSD_ABI_VERSION, q, r, delta, eta, k, theta, key_bits,
                  SSD_VERIFY_REHASH if verify_rehash else 0, cell_bits, max_tuples, max_results)


def query_sizes(params: Params) -> Tuple[int, int]:
    s, t = C.c_uint64(), C.c_uint64()
    _check(_lib().ssd_query_sizes(C.byref(params), C.byref(s), C.byref(t)), "query_sizes")
    return s.value, t.value


class Detector:
    """Owns the torch device buffers of one detector and its library handle."""

    def __init__(self, params: Params, tables: np.ndarray, device=None, stream: Optional[torch.cuda.Stream] = None):
        L = _lib()
        self.params = params
        self.device = torch.device(device if device is not None else "cuda")
        state_bytes, scratch_bytes = query_sizes(params)
        # allocations from torch; 256-byte aligned
        self.state = torch.empty(state_bytes, dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(scratch_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        tabs = np.ascontiguousarray(tables, dtype=np.uint32).reshape(-1)
        if tabs.size != 2048:
            raise ValueError("tables must hold 2 x 4 x 256 words")
        self._tables = tabs
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.ssd_init_detector(C.byref(params), tabs.ctypes.data_as(C.POINTER(C.c_uint32)),
                                       self.state.data_ptr(), state_bytes, self.scratch.data_ptr(),
                                       scratch_bytes, self.stream.cuda_stream, C.byref(h)), "init_detector")
        self.handle = h

    def destroy(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib().ssd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    @property
    def r(self) -> int:
        return self.params.r

    @property
    def n_se(self) -> int:
        return self.params.r << self.params.q


def init_detector(params: Params, tables: np.ndarray, device=None, stream=None) -> Detector:
    return Detector(params, tables, device, stream)


def destroy(det: Detector) -> None:
    det.destroy()


def scan_slice(det: Detector, pairs: torch.Tensor, slice_id: int) -> None:
    """pairs: contiguous (n, 2) 32-bit tensor on the detector's device, [:,0] = cip."""
    if pairs.numel() and (pairs.device != det.state.device or pairs.element_size() != 4
                          or not pairs.is_contiguous() or pairs.dim() != 2 or pairs.shape[1] != 2):
        raise ValueError("pairs must be a contiguous (n, 2) 32-bit tensor on the detector's device")
    n = pairs.shape[0] if pairs.dim() == 2 else 0
    _check(_lib().ssd_scan_slice(det.handle, pairs.data_ptr() if n else None, n, slice_id), "scan_slice")


def scan_slice_noalloc(det: Detector, pairs: torch.Tensor, slice_id: int) -> None:
    """As scan_slice, with the binned scan's staging in the library's static
    device array instead of the detector's scratch (no allocation)."""
    if pairs.numel() and (pairs.device != det.state.device or pairs.element_size() != 4
                          or not pairs.is_contiguous() or pairs.dim() != 2 or pairs.shape[1] != 2):
        raise ValueError("pairs must be a contiguous (n, 2) 32-bit tensor on the detector's device")
    n = pairs.shape[0] if pairs.dim() == 2 else 0
    _check(_lib().ssd_scan_slice_noalloc(det.handle, pairs.data_ptr() if n else None, n, slice_id),
           "scan_slice_noalloc")


def _results(det: Detector, fn, *args) -> np.ndarray:
    L = _lib()
    n = C.c_uint64()
    cap = 4096
    while True:
        out = np.empty(cap, dtype=RESULT_DTYPE)     # only the first n entries are filled and returned
        st = fn(det.handle, *args, out.ctypes.data, cap, C.byref(n))
        if st == SSD_E_TRUNC and n.value > cap:
            cap = int(n.value)
            fn = L.ssd_get_results
            args = ()
            continue
        _check(st, fn.__name__)
        return out[:n.value].copy()


def close_slice(det: Detector, advance_only: bool = False) -> np.ndarray:
    """Close the open slice; returns the SSP list (structured array ip, rk, est)."""
    return _results(det, _lib().ssd_close_slice, SSD_ADVANCE_ONLY if advance_only else 0)


def close_begin(det: Detector) -> None:
    """Enqueue the close of the open slice and open the next one (no wait)."""
    _check(_lib().ssd_close_begin(det.handle), "close_begin")


def close_end(det: Detector) -> np.ndarray:
    """Wait for the pending close and return its SSP list."""
    return _results(det, _lib().ssd_close_end)


def get_results(det: Detector) -> np.ndarray:
    return _results(det, _lib().ssd_get_results)


def merge_router_state(global_det: Detector, routers: Sequence[Detector]) -> None:
    arr = (C.c_void_p * len(routers))(*[r.handle.value for r in routers])
    _check(_lib().ssd_merge_router_state(global_det.handle, arr, len(routers)), "merge_router_state")


def export_state(det: Detector) -> np.ndarray:
    """The detector's checkpoint blob (uint8 array in host memory)."""
    n = C.c_uint64(0)
    st = _lib().ssd_export_state(det.handle, None, 0, C.byref(n))
    if st not in (0, SSD_E_TRUNC):
        _check(st, "export_state")
    out = np.empty(n.value, dtype=np.uint8)
    _check(_lib().ssd_export_state(det.handle, out.ctypes.data, out.size, C.byref(n)), "export_state")
    return out


def import_state(det: Detector, blob: np.ndarray) -> None:
    """Continue `det` from a blob of export_state (same parameters and tables)."""
    b = np.ascontiguousarray(blob, dtype=np.uint8)
    _check(_lib().ssd_import_state(det.handle, b.ctypes.data, b.size), "import_state")


def read_canonical_state(det: Detector) -> torch.Tensor:
    """Canonical window state (int16 tensor on the device; view as uint16)."""
    n = det.n_se * det.params.eta
    out = torch.empty(n, dtype=torch.int16, device=det.state.device)
    _check(_lib().ssd_read_canonical_state(det.handle, out.data_ptr(), n), "read_canonical_state")
    return out


def read_rk(det: Detector) -> np.ndarray:
    out = np.zeros((det.params.r, 1 << det.params.q), dtype=np.uint32)
    _check(_lib().ssd_read_rk(det.handle, out.ctypes.data, out.size), "read_rk")
    return out


def read_hot(det: Detector) -> List[np.ndarray]:
    counts = np.zeros(det.params.r, dtype=np.uint32)
    flat = np.zeros(det.n_se, dtype=np.uint32)
    _check(_lib().ssd_read_hot(det.handle, counts.ctypes.data, flat.ctypes.data, flat.size), "read_hot")
    out, o = [], 0
    for c in counts.tolist():
        out.append(flat[o:o + c].copy())
        o += c
    return out


def read_tuples(det: Detector) -> np.ndarray:
    L = _lib()
    n = C.c_uint64()
    st = L.ssd_read_tuples(det.handle, None, 0, C.byref(n))
    if st not in (0, SSD_E_TRUNC):
        _check(st, "read_tuples")
    out = np.zeros((n.value, det.params.r), dtype=np.uint32)
    if n.value:
        _check(L.ssd_read_tuples(det.handle, out.ctypes.data, n.value, C.byref(n)), "read_tuples")
    return out


def get_info(det: Detector) -> Dict[str, object]:
    info = _Info()
    _check(_lib().ssd_get_info(det.handle, C.byref(info)), "get_info")
    return _info_dict(info)


def _info_dict(info) -> Dict[str, object]:
    r = info.r
    return {"open_slice": info.open_slice, "hot_threshold": info.hot_threshold,
            "state_bytes": info.state_bytes, "level_counts": list(info.level_counts)[:max(r - 2, 0)],
            "hot_counts": list(info.hot_counts)[:r], "accepted": info.accepted, "reported": info.reported,
            "counted": info.counted, "counted_bin_kib": info.counted_bin_kib}


SSD_TUNE_SCAN_PASS_BYTES = 1
SSD_TUNE_SORT_BLOCK_LIMIT = 2
SSD_TUNE_TIMING = 3
SSD_TUNE_SCAN_TILE_PAIRS = 4
SSD_TUNE_GRAPH = 5
SSD_TUNE_AUTOTUNE = 6
SSD_TUNE_SCAN_MODE = 7
SSD_TUNE_SCAN_BIN_BYTES = 8
SSD_TUNE_SCAN_APPLY_SEGMENTS = 9
SSD_TUNE_COUNTED = 10
SSD_TUNE_COUNTED_MIN_ITEMS = 11
SSD_SCAN_PASSES = 0
SSD_SCAN_BINNED = 1
SSD_SCAN_AUTO = 2
PHASES = ("scan", "hot_detect", "hot_lists", "expand", "verify", "report", "merge", "close_graph", "scan_bin",
          "count_detect", "scan_tiles")


def read_timing(det: Detector, reset: bool = False) -> Dict[str, Tuple[float, int]]:
    """Device ms and kernel launches per phase, from HIP events on the
    detector's stream (needs SSD_TUNE_TIMING on)."""
    ms = np.zeros(len(PHASES), dtype=np.float64)
    n = np.zeros(len(PHASES), dtype=np.uint64)
    _check(_lib().ssd_read_timing(det.handle, ms.ctypes.data, n.ctypes.data, int(reset)), "read_timing")
    return {name: (float(ms[i]), int(n[i])) for i, name in enumerate(PHASES)}


def set_tuning(det: Detector, knob: int, value: int) -> None:
    _check(_lib().ssd_set_tuning(det.handle, knob, value), "set_tuning")


# ---------------------------------------------------------------- batches

def batch_query_sizes(params: Sequence[Params]) -> Tuple[int, int]:
    arr = (Params * len(params))(*params)
    st, sc = C.c_uint64(), C.c_uint64()
    _check(_lib().ssd_batch_query_sizes(C.addressof(arr), len(params), C.byref(st), C.byref(sc)),
           "batch_query_sizes")
    return st.value, sc.value


class Batch:
    """n detectors ("links") scanned by one persistent launch and closed by
    one replayed graph; owns their torch device buffers."""

    def __init__(self, params: Sequence[Params], tables: Sequence[np.ndarray], device=None, stream=None):
        L = _lib()
        self.params = list(params)
        self.n = len(self.params)
        self.device = torch.device(device if device is not None else "cuda")
        self._parr = (Params * self.n)(*self.params)
        state_bytes, scratch_bytes = batch_query_sizes(self.params)
        self.state = torch.empty(state_bytes, dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(scratch_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        tabs = np.ascontiguousarray(np.stack([np.asarray(t, dtype=np.uint32).reshape(-1) for t in tables]))
        if tabs.shape != (self.n, 2048):
            raise ValueError("need one 2 x 4 x 256 table set per link")
        self._tables = tabs
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.ssd_batch_init(C.addressof(self._parr), self.n, tabs.ctypes.data, self.state.data_ptr(),
                                    state_bytes, self.scratch.data_ptr(), scratch_bytes, self.stream.cuda_stream,
                                    C.byref(h)), "batch_init")
        self.handle = h

    def destroy(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib().ssd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def batch_init(params: Sequence[Params], tables: Sequence[np.ndarray], device=None, stream=None) -> Batch:
    return Batch(params, tables, device, stream)


def batch_destroy(b: Batch) -> None:
    b.destroy()


def batch_scan(b: Batch, pairs: torch.Tensor, offsets: Sequence[int], slice_id: int) -> None:
    """pairs: contiguous (N, 2) 32-bit tensor on the batch's device holding every
    link's pairs; link l owns rows offsets[l]..offsets[l+1]."""
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    if off.shape != (b.n + 1,):
        raise ValueError("offsets needs n + 1 entries")
    if pairs.numel() and (pairs.device != b.state.device or pairs.element_size() != 4
                          or not pairs.is_contiguous() or pairs.dim() != 2 or pairs.shape[1] != 2):
        raise ValueError("pairs must be a contiguous (N, 2) 32-bit tensor on the batch's device")
    if int(off[-1]) > (pairs.shape[0] if pairs.dim() == 2 else 0):
        raise ValueError("offsets run past the pairs tensor")
    ptr = pairs.data_ptr() if pairs.numel() else None
    _check(_lib().ssd_batch_scan(b.handle, ptr, off.ctypes.data, slice_id), "batch_scan")


def _batch_lists(b: Batch, fn, *args):
    L = _lib()
    counts = np.zeros(b.n, dtype=np.uint64)
    status = np.zeros(b.n, dtype=np.int32)
    cap = 1 << 16
    while True:
        out = np.zeros(cap, dtype=RESULT_DTYPE)
        st = fn(b.handle, *args, out.ctypes.data, cap, counts.ctypes.data, status.ctypes.data)
        total = int(counts.sum())
        if st == SSD_E_TRUNC and total > cap:
            cap = total
            fn, args = L.ssd_batch_get_results, ()
            continue
        _check(st, fn.__name__)
        lists, o = [], 0
        for c in counts.tolist():
            lists.append(out[o:o + c].copy())
            o += c
        return lists, status


def batch_close(b: Batch):
    """Close the open slice of every link: (list of per-link result arrays,
    per-link status codes: 0 or -4 = capacity exceeded)."""
    return _batch_lists(b, _lib().ssd_batch_close)


def batch_close_begin(b: Batch) -> None:
    "Begin the close of every link; the next slice is open at once."
    _check(_lib().ssd_batch_close_begin(b.handle), "batch_close_begin")


def batch_close_end(b: Batch):
    "Wait for the pending batch close: as batch_close."
    return _batch_lists(b, _lib().ssd_batch_close_end)


def batch_get_results(b: Batch):
    return _batch_lists(b, _lib().ssd_batch_get_results)


def batch_set_tuning(b: Batch, knob: int, value: int) -> None:
    _check(_lib().ssd_batch_set_tuning(b.handle, knob, value), "batch_set_tuning")


def batch_get_tuning(b: Batch, knob: int) -> int:
    v = C.c_uint64()
    _check(_lib().ssd_batch_get_tuning(b.handle, knob, C.byref(v)), "batch_get_tuning")
    return v.value


def batch_read_timing(b: Batch, reset: bool = False) -> Dict[str, Tuple[float, int]]:
    ms = np.zeros(len(PHASES), dtype=np.float64)
    n = np.zeros(len(PHASES), dtype=np.uint64)
    _check(_lib().ssd_batch_read_timing(b.handle, ms.ctypes.data, n.ctypes.data, int(reset)), "batch_read_timing")
    return {name: (float(ms[i]), int(n[i])) for i, name in enumerate(PHASES)}


def batch_get_info(b: Batch, link: int) -> Dict[str, object]:
    info = _Info()
    _check(_lib().ssd_batch_get_info(b.handle, link, C.byref(info)), "batch_get_info")
    return _info_dict(info)


def batch_read_rk(b: Batch, link: int) -> np.ndarray:
    p = b.params[link]
    out = np.zeros((p.r, 1 << p.q), dtype=np.uint32)
    _check(_lib().ssd_batch_read_rk(b.handle, link, out.ctypes.data, out.size), "batch_read_rk")
    return out


def batch_read_hot(b: Batch, link: int) -> List[np.ndarray]:
    p = b.params[link]
    counts = np.zeros(p.r, dtype=np.uint32)
    flat = np.zeros(p.r << p.q, dtype=np.uint32)
    _check(_lib().ssd_batch_read_hot(b.handle, link, counts.ctypes.data, flat.ctypes.data, flat.size),
           "batch_read_hot")
    out, o = [], 0
    for c in counts.tolist():
        out.append(flat[o:o + c].copy())
        o += c
    return out


# ---------------------------------------------------------------- groups

def group_query_sizes(max_members: int) -> int:
    v = C.c_uint64()
    _check(_lib().ssd_group_query_sizes(max_members, C.byref(v)), "group_query_sizes")
    return v.value


class Group:
    """Batched scan / close over any set of single detectors, chosen per call
    (continuous batching).  Members must share its device and stream."""

    def __init__(self, max_members: int, device=None, stream=None):
        L = _lib()
        self.max_members = max_members
        self.device = torch.device(device if device is not None else "cuda")
        nbytes = group_query_sizes(max_members)
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.ssd_group_init(max_members, self.scratch.data_ptr(), nbytes, self.stream.cuda_stream,
                                    C.byref(h)), "group_init")
        self.handle = h

    def destroy(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib().ssd_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def group_init(max_members: int, device=None, stream=None) -> Group:
    return Group(max_members, device, stream)


def group_destroy(g: Group) -> None:
    g.destroy()


def _members(dets: Sequence[Detector]):
    return (C.c_void_p * len(dets))(*[d.handle.value for d in dets])


def group_scan(g: Group, dets: Sequence[Detector], pairs: torch.Tensor, offsets: Sequence[int],
               slice_ids: Sequence[int]) -> None:
    """Member i's pairs are rows offsets[i]..offsets[i+1] of `pairs`, scanned
    into its open slice slice_ids[i]."""
    n = len(dets)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    ids = np.ascontiguousarray(slice_ids, dtype=np.uint64)
    if off.shape != (n + 1,) or ids.shape != (n,):
        raise ValueError("offsets needs n + 1 entries and slice_ids n")
    if pairs.numel() and (pairs.device != g.scratch.device or pairs.element_size() != 4
                          or not pairs.is_contiguous() or pairs.dim() != 2 or pairs.shape[1] != 2):
        raise ValueError("pairs must be a contiguous (N, 2) 32-bit tensor on the group's device")
    if int(off[-1]) > (pairs.shape[0] if pairs.dim() == 2 else 0):
        raise ValueError("offsets run past the pairs tensor")
    ptr = pairs.data_ptr() if pairs.numel() else None
    _check(_lib().ssd_group_scan(g.handle, _members(dets), n, ptr, off.ctypes.data, ids.ctypes.data), "group_scan")


def group_close_begin(g: Group, dets: Sequence[Detector]) -> None:
    """Enqueue the close of every member's open slot and open the next ones
    (no wait); collect the lists with group_close_end."""
    g._pending = list(dets)
    _check(_lib().ssd_group_close_begin(g.handle, _members(dets), len(dets)), "group_close_begin")


def group_close_end(g: Group):
    """Wait for the pending group close: (per-member result arrays, status codes)."""
    dets = getattr(g, "_pending", None) or []
    n = len(dets)
    counts = np.zeros(max(n, 1), dtype=np.uint64)
    status = np.zeros(max(n, 1), dtype=np.int32)
    cap = 1 << 16
    out = np.zeros(cap, dtype=RESULT_DTYPE)
    st = _lib().ssd_group_close_end(g.handle, out.ctypes.data, cap, counts.ctypes.data, status.ctypes.data)
    g._pending = None
    if st == SSD_E_TRUNC:
        return [get_results(d) for d in dets], status[:n]
    _check(st, "group_close_end")
    lists, o = [], 0
    for c in counts[:n].tolist():
        lists.append(out[o:o + c].copy())
        o += c
    return lists, status[:n]


def group_close(g: Group, dets: Sequence[Detector]):
    """Close the open slice of every member: (per-member result arrays, status codes)."""
    n = len(dets)
    counts = np.zeros(n, dtype=np.uint64)
    status = np.zeros(n, dtype=np.int32)
    cap = 1 << 16
    arr = _members(dets)
    out = np.zeros(cap, dtype=RESULT_DTYPE)
    st = _lib().ssd_group_close(g.handle, arr, n, out.ctypes.data, cap, counts.ctypes.data, status.ctypes.data)
    if st == SSD_E_TRUNC:
        # every member keeps its own list; fetch them one by one
        return [get_results(d) for d in dets], status
    _check(st, "group_close")
    lists, o = [], 0
    for c in counts.tolist():
        lists.append(out[o:o + c].copy())
        o += c
    return lists, status
