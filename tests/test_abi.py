"""C ABI checks that need no GPU: the library loads, exports every call that
include/ssd.h declares, and validates parameters on the host."""
import ctypes as C
import os
import re

import pytest

import paper_1803_11036_amd as ssd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="ssd.h"):
    with open(os.path.join(ROOT, "include", header)) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_call():
    """Every call of every header under include/ (the detector's ABI and the
    memory-ceiling probes) is exported by the built library."""
    headers = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    assert "ssd.h" in headers and "ssd_probe.h" in headers
    lib = C.CDLL(ssd.library_path())
    total = 0
    for h in headers:
        names = _declared(h)
        total += len(names)
        for n in names:
            assert hasattr(lib, n), f"{h}: {n}"
    assert len(_declared()) >= 15 and total >= len(_declared()) + 2


def test_binding_names_match_the_abi():
    for n in _declared():
        py = n[len("ssd_"):]
        if py in ("strerror", "last_error"):
            continue
        assert hasattr(ssd, py), py


def test_binding_constants_match_the_header():
    """Every SSD_* integer the binding defines equals the header's #define,
    and the binding names one timing phase per SSD_PHASES."""
    with open(os.path.join(ROOT, "include", "ssd.h")) as f:
        defs = {m.group(1): int(m.group(2), 0)
                for m in re.finditer(r"#define\s+(SSD_[A-Z0-9_]+)\s+\(?(-?(?:0x[0-9a-fA-F]+|\d+))u?\)?", f.read())}
    shared = [n for n in defs if hasattr(ssd, n)]
    assert len(shared) >= 10
    for n in shared:
        assert getattr(ssd, n) == defs[n], n
    assert len(ssd.PHASES) == defs["SSD_PHASES"]


def _p(**kw):
    base = dict(q=12, r=6, delta=5, eta=1024, k=4, theta=1024)
    base.update(kw)
    return ssd.make_params(**base)


def test_query_sizes():
    state, scratch = ssd.query_sizes(_p())
    assert state == 6 * 4096 * 1024
    assert scratch > 6 * 4096 * 8 and scratch % 256 == 0


@pytest.mark.parametrize("bad", [
    dict(r=2), dict(r=17), dict(q=3), dict(q=21), dict(delta=0), dict(delta=12, q=12),
    dict(eta=1000), dict(eta=512), dict(eta=1 << 17), dict(k=0), dict(k=255), dict(theta=0),
    dict(key_bits=7), dict(key_bits=33), dict(q=12, r=4, delta=5),            # covers 22 < 32 bits
    dict(q=20, r=16, delta=12, key_bits=32),                                  # covers > 64 bits
    dict(max_tuples=0), dict(max_results=0), dict(max_results=1 << 29),
])
def test_invalid_params_rejected(bad):
    with pytest.raises(ssd.SSDError) as e:
        ssd.query_sizes(_p(**bad))
    assert e.value.status == -1


def test_abi_version_and_flags_checked():
    p = _p()
    p.abi_version = 2
    with pytest.raises(ssd.SSDError):
        ssd.query_sizes(p)
    p = _p()
    p.flags = 0x10
    with pytest.raises(ssd.SSDError):
        ssd.query_sizes(p)
    for bits in (1, 12, 32):
        p = _p()
        p.cell_bits = bits
        with pytest.raises(ssd.SSDError):
            ssd.query_sizes(p)


def test_paper_parameter_set_is_valid():
    """Sec. 5 runs eta = 2^11, q = 14, r = 5, delta = 6 with windows of k =
    300 slots on 16-bit recorders: valid with 16-bit cells (twice the bytes
    of 8-bit cells), refused with 8-bit cells; 16-bit cells allow k up to
    65534 (Sec. 3.2: k < 65535)."""
    cells = 5 * (1 << 14) * 2048
    state, _ = ssd.query_sizes(ssd.make_params(q=14, r=5, delta=6, eta=2048, k=300, theta=1024, cell_bits=16))
    assert state == 2 * cells
    state, _ = ssd.query_sizes(ssd.make_params(q=14, r=5, delta=6, eta=2048, k=254, theta=1024))
    assert state == cells
    for k, bits in ((300, 8), (255, 8), (65535, 16), (0, 16)):
        with pytest.raises(ssd.SSDError) as e:
            ssd.query_sizes(ssd.make_params(q=14, r=5, delta=6, eta=2048, k=k, theta=1024, cell_bits=bits))
        assert e.value.status == -1
    ssd.query_sizes(ssd.make_params(q=14, r=5, delta=6, eta=2048, k=65534, theta=1024, cell_bits=16))
    ssd.query_sizes(ssd.make_params(q=14, r=5, delta=6, eta=2048, k=200, theta=1024, cell_bits=0))


def test_batches_take_8bit_cells():
    """Batch links with 16-bit cells are refused (the batched scan and hot
    detection are written for 8-bit cells)."""
    ok = ssd.make_params(q=12, r=6, delta=5, eta=1024, k=4, theta=1024)
    wide = ssd.make_params(q=12, r=6, delta=5, eta=1024, k=300, theta=1024, cell_bits=16)
    ssd.batch_query_sizes([ok, ok])
    with pytest.raises(ssd.SSDError) as e:
        ssd.batch_query_sizes([ok, wide])
    assert e.value.status == -1


def test_init_rejects_before_touching_the_device():
    lib = C.CDLL(ssd.library_path())
    lib.ssd_init_detector.argtypes = [C.c_void_p] * 8
    lib.ssd_init_detector.restype = C.c_int
    out = C.c_void_p()
    p = _p(r=2)
    assert lib.ssd_init_detector(C.addressof(p), None, None, 0, None, 0, None, C.addressof(out)) == -1
    p = _p()
    tabs = (C.c_uint32 * 2048)()
    # NULL device buffers are rejected as too small before any HIP call
    assert lib.ssd_init_detector(C.addressof(p), C.addressof(tabs), None, 0, None, 0, None,
                                 C.addressof(out)) == -2
    assert out.value is None


def test_counter_scratch_only_for_detectors_that_can_count():
    """The per-slot counters (u32 per estimator and window slice, and a live-
    cell total per estimator) are part of
    the scratch exactly when they take at most half the state (eta >= 8 k),
    eta <= 2^14 (16-bit counters in LDS) and the cell bits and counters of a
    256 KiB bin fit a workgroup's LDS (32 KiB + 512 bytes per window slice at
    eta = 1024, within 151 KiB); the knob and the phase that use them are
    exported."""
    def scratch(k, eta=1024):
        return ssd.query_sizes(_p(k=k, eta=eta))[1]
    n_se = 6 << 12
    assert scratch(4) - scratch(129) == n_se * 5 * 4           # k = 4: counted; k = 129 > 1024 / 8: not
    assert scratch(128) - scratch(129) == n_se * 129 * 4       # the largest window that counts at eta 1024
    # eta = 4096: every 8-bit window counts (k = 254 at 256 KiB bins: 32 KiB + 254 * 128 bytes)
    assert scratch(254, 4096) - scratch(4, 4096) == n_se * 250 * 4
    # eta = 2^15: no counters, whatever the window
    assert scratch(4, 1 << 15) == scratch(5, 1 << 15)
    assert "count_detect" in ssd.PHASES and ssd.SSD_TUNE_COUNTED == 10
