"""CPU oracle of the sliding super point detector (test infrastructure only).

A plain, slow, literal model of the paper's method (Sec. 3, Alg. 1-5, Eq. 1-3)
in C (``rsea_oracle.c``) behind this ctypes wrapper, plus the exact "precise
algorithm" of Sec. 3.2 in ``truth.py``.  Only the tests, the smoke check and
the benchmark's CPU-baseline leg may import this package; the GPU product path
never does, and it shares no code with it.

Every function that has no independent pin says so in its docstring; the pins
live in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Sequence, Tuple

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_u32p = C.POINTER(C.c_uint32)
_u16p = C.POINTER(C.c_uint16)
_f64p = C.POINTER(C.c_double)


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_uint32] * 8 + [_u32p]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_threshold.restype = C.c_uint32
        L.orc_threshold.argtypes = [C.c_void_p]
        L.orc_dr.restype = _u16p
        L.orc_dr.argtypes = [C.c_void_p]
        L.orc_h1.restype = C.c_uint32
        L.orc_h1.argtypes = [C.c_void_p, C.c_uint32]
        L.orc_rhfg.argtypes = [C.c_void_p, C.c_uint32, _u32p]
        L.orc_scan.argtypes = [C.c_void_p, _u32p, C.c_uint64]
        L.orc_reconstruct.restype = C.c_int64
        L.orc_reconstruct.argtypes = [C.c_void_p]
        L.orc_age.argtypes = [C.c_void_p]
        L.orc_close.restype = C.c_int64
        L.orc_close.argtypes = [C.c_void_p, C.c_int]
        L.orc_results.restype = C.c_uint64
        L.orc_results.argtypes = [C.c_void_p, _u32p, _u32p, _f64p, C.c_uint64]
        L.orc_rk.argtypes = [C.c_void_p, _u32p]
        L.orc_hse.argtypes = [C.c_void_p, _u32p, _u32p]
        L.orc_tuples.restype = C.c_uint64
        L.orc_tuples.argtypes = [C.c_void_p, _u32p, C.c_uint64]
        L.orc_canonical.argtypes = [C.c_void_p, _u16p]
        L.orc_merge.restype = C.c_int
        L.orc_merge.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.c_uint32]
        L.orc_roundtrip_failures.restype = C.c_uint64
        L.orc_roundtrip_failures.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64]
        L.orc_extract.restype = C.c_uint64
        L.orc_extract.argtypes = [C.c_void_p, _u32p]
        L.orc_bruteforce.restype = C.c_uint64
        L.orc_bruteforce.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, _u32p, _u32p, C.c_uint64]
        _LIB = L
    return _LIB


def _p32(a: np.ndarray):
    return a.ctypes.data_as(_u32p)


class RSEA:
    """Reversible sliding estimator array with its RHFG (Sec. 3.3).

    ``tables`` is ``uint32[2][4][256]``: the tabulation tables of RHFG[0] and
    H1.  ``key_bits`` is the host address width (32 for IPv4); reconstructed
    values wider than it are dropped (reading R13).
    """

    def __init__(self, q: int, r: int, delta: int, eta: int, k: int, theta: int,
                 tables: np.ndarray, key_bits: int = 32, verify_rehash: bool = False):
        if not (3 <= r <= 64 and 1 <= delta < q <= 24 and (r - 2) * delta + q <= 64):
            raise ValueError("unsupported geometry")
        if (r - 2) * delta + q < key_bits:
            raise ValueError("(r-2)*delta + q must cover key_bits")
        if eta < 1 or eta & (eta - 1) or not (1 <= k <= 65534):
            raise ValueError("eta must be a power of two and 1 <= k <= 65534")
        self.q, self.r, self.delta, self.eta, self.k, self.theta = q, r, delta, eta, k, theta
        self.key_bits = key_bits
        self._tables = np.ascontiguousarray(tables, dtype=np.uint32).reshape(2, 4, 256)
        L = _lib()
        self._h = L.orc_create(q, r, delta, eta, k, theta, key_bits, int(bool(verify_rehash)),
                               _p32(self._tables))
        if not self._h:
            raise MemoryError("oracle state allocation failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib().orc_destroy(h)
            self._h = None

    @property
    def T(self) -> int:
        """Integer hot threshold ceil(eta*(1-exp(-theta/eta))) (Sec. 3.3, R5)."""
        return int(_lib().orc_threshold(self._h))

    def rhfg(self, cip: int) -> List[int]:
        out = np.zeros(self.r, dtype=np.uint32)
        _lib().orc_rhfg(self._h, cip & 0xFFFFFFFF, _p32(out))
        return [int(v) for v in out]

    def h1(self, oip: int) -> int:
        return int(_lib().orc_h1(self._h, oip & 0xFFFFFFFF))

    def dr(self) -> np.ndarray:
        """Live view of the distance recorders, uint16[r][2^q][eta]."""
        n = self.r * (1 << self.q) * self.eta
        ptr = _lib().orc_dr(self._h)
        return np.ctypeslib.as_array(ptr, shape=(n,)).reshape(self.r, 1 << self.q, self.eta)

    def scan(self, pairs: np.ndarray) -> None:
        """Alg. 2 on every (cip, oip) row of ``pairs``."""
        p = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
        _lib().orc_scan(self._h, _p32(p), p.shape[0])

    def reconstruct(self) -> int:
        n = _lib().orc_reconstruct(self._h)
        if n < 0:
            raise MemoryError("oracle reconstruction failed")
        return int(n)

    def age(self) -> None:
        _lib().orc_age(self._h)

    def close(self, advance_only: bool = False):
        """End of slot: reconstruct (unless advance_only) and age.  Returns results()."""
        n = _lib().orc_close(self._h, int(bool(advance_only)))
        if n < 0:
            raise MemoryError("oracle reconstruction failed")
        return self.results()

    def results(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """(ip, R, est) of the last reconstruction, ascending ip."""
        L = _lib()
        n = int(L.orc_results(self._h, None, None, None, 0))
        ip = np.zeros(n, np.uint32); rk = np.zeros(n, np.uint32); est = np.zeros(n, np.float64)
        if n:
            L.orc_results(self._h, _p32(ip), _p32(rk), est.ctypes.data_as(_f64p), n)
        return ip, rk, est

    def rk(self) -> np.ndarray:
        out = np.zeros((self.r, 1 << self.q), np.uint32)
        _lib().orc_rk(self._h, _p32(out))
        return out

    def hse(self) -> List[np.ndarray]:
        counts = np.zeros(self.r, np.uint32)
        flat = np.zeros(self.r << self.q, np.uint32)
        _lib().orc_hse(self._h, _p32(counts), _p32(flat))
        out, o = [], 0
        for c in counts:
            out.append(flat[o:o + int(c)].copy()); o += int(c)
        return out

    def tuples(self) -> np.ndarray:
        """Candidate tuples that reached the final test, uint32[n][r]."""
        L = _lib()
        n = int(L.orc_tuples(self._h, None, 0))
        out = np.zeros((n, self.r), np.uint32)
        if n:
            L.orc_tuples(self._h, _p32(out), n)
        return out

    def canonical(self) -> np.ndarray:
        """DR where DR < k, else 0xFFFF; uint16[r][2^q][eta]."""
        out = np.zeros((self.r, 1 << self.q, self.eta), np.uint16)
        _lib().orc_canonical(self._h, out.ctypes.data_as(_u16p))
        return out

    def merge_from(self, routers: Sequence["RSEA"]) -> None:
        """Alg. 5 with reading R3: per-DR minimum distance over the routers."""
        arr = (C.c_void_p * len(routers))(*[r._h for r in routers])
        if _lib().orc_merge(self._h, arr, len(routers)) != 0:
            raise ValueError("routers differ in geometry or hash tables")

    def roundtrip_failures(self, lo: int, hi: int, stride: int = 1) -> int:
        """Hosts in [lo, hi) (step ``stride``) whose own RHFG tuple fails the
        overlap tests or does not extract back to the host (Eq. 3)."""
        return int(_lib().orc_roundtrip_failures(self._h, lo, hi, stride))

    def extract(self, tup) -> int:
        t = np.ascontiguousarray(tup, dtype=np.uint32)
        return int(_lib().orc_extract(self._h, _p32(t)))

    def bruteforce(self, lo: int = 0, hi: int = None) -> Tuple[np.ndarray, np.ndarray]:
        """Forward enumeration of hosts in [lo, hi) on the current DRs (a pin)."""
        if hi is None:
            hi = 1 << self.key_bits
        L = _lib()
        n = int(L.orc_bruteforce(self._h, lo, hi, None, None, 0))
        if n == 2 ** 64 - 1:
            raise MemoryError
        ip = np.zeros(n, np.uint32); rk = np.zeros(n, np.uint32)
        if n:
            L.orc_bruteforce(self._h, lo, hi, _p32(ip), _p32(rk), n)
        return ip, rk


def estimate(eta: int, R: np.ndarray) -> np.ndarray:
    """Eq. 1 with z0 = eta - R, z0 at least 1 (reading R6), in float64."""
    z0 = np.maximum(eta - np.asarray(R, dtype=np.float64), 1.0)
    return -float(eta) * np.log(z0 / float(eta))
