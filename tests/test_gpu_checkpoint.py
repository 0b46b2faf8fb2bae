"""Checkpoint and resume: a detector exported after any close and imported
into a fresh detector with the same parameters and tables continues exactly
as the exporting one -- same lists as the oracle fed the whole stream, same
window state -- with 8- and 16-bit cells, binned and counted or pass-window
scans; blobs of other detectors or formats are refused."""
import numpy as np
import pytest

import oracle
import paper_1803_11036_amd as ssd
import tracegen as tg
from _parity import close_both, compare_state, log, make_pair, scan_both, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cell_bits,mode", [(8, "counted"), (8, "passes"), (16, "binned")])
def test_resume_from_checkpoint_equals_oracle(cell_bits, mode):
    cfg = tg.config("tiny", k=5, pairs_lo=400_000, pairs_hi=400_000, n_slices=14)
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)

    def detector():
        d = ssd.init_detector(ssd.make_params(q=cfg.q, r=cfg.r, delta=cfg.delta, eta=cfg.eta, k=cfg.k,
                                              theta=cfg.theta, cell_bits=cell_bits), tabs, device="cuda:0")
        if mode != "passes":
            ssd.set_tuning(d, ssd.SSD_TUNE_SCAN_MODE, ssd.SSD_SCAN_BINNED)
        if mode == "counted":
            ssd.set_tuning(d, ssd.SSD_TUNE_COUNTED_MIN_ITEMS, 0)
        return d

    a = detector()
    o = oracle.RSEA(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs)
    cut = 7                                   # export after slice 6's close: a full window behind it
    for t in range(cut):
        scan_both(a, o, tr.pairs(0, t), t)
        close_both(a, o, check_internals=False)
    blob = ssd.export_state(a)
    assert blob.size == ssd.STATE_HEADER_BYTES + a.state.numel()
    b = detector()
    ssd.import_state(b, blob)
    assert ssd.get_info(b)["open_slice"] == cut
    for t in range(cut, cfg.n_slices):
        p = tr.pairs(0, t)
        ssd.scan_slice(a, to_dev(p), t)
        scan_both(b, o, p, t)
        compare_state(b, o)
        ra = ssd.close_slice(a)
        rb = close_both(b, o)
        assert np.array_equal(ra, rb), f"slice {t}: resumed detector differs from the exporting one"
        log(f"resume cell_bits={cell_bits} {mode} slice {t}: {len(rb)} hosts")
    assert np.array_equal(ssd.read_rk(a), ssd.read_rk(b))
    if mode == "counted":
        # the resumed detector rebuilt its counters after its first large binned scan
        assert ssd.get_info(b)["counted"] == 1
    a.destroy()
    b.destroy()


def test_checkpoint_refusals():
    tabs = tg.hash_tables(3)
    p = ssd.make_params(q=14, r=5, delta=6, eta=1024, k=4, theta=300)
    a = ssd.init_detector(p, tabs, device="cuda:0")
    rng = np.random.default_rng(0)
    ssd.scan_slice(a, to_dev(rng.integers(0, 2 ** 32, (50_000, 2), dtype=np.uint64).astype(np.uint32)), 0)
    blob = ssd.export_state(a)
    # another window, other tables, a cut or altered blob
    for other, code in [(ssd.init_detector(ssd.make_params(q=14, r=5, delta=6, eta=1024, k=5, theta=300), tabs,
                                           device="cuda:0"), ssd.SSD_E_INCOMPAT),
                        (ssd.init_detector(p, tg.hash_tables(4), device="cuda:0"), ssd.SSD_E_INCOMPAT)]:
        with pytest.raises(ssd.SSDError) as e:
            ssd.import_state(other, blob)
        assert e.value.status == code
        other.destroy()
    b = ssd.init_detector(p, tabs, device="cuda:0")
    for bad in (blob[:-1], blob[:32], np.concatenate([np.frombuffer(b"NOTSTATE", np.uint8), blob[8:]])):
        with pytest.raises(ssd.SSDError) as e:
            ssd.import_state(b, bad)
        assert e.value.status == ssd.SSD_E_PARAM
    # no checkpoint while a close is pending
    ssd.close_begin(a)
    with pytest.raises(ssd.SSDError) as e:
        ssd.export_state(a)
    assert e.value.status == ssd.SSD_E_ORDER
    ssd.close_end(a)
    ssd.import_state(b, blob)                 # the untouched blob still imports
    assert ssd.get_info(b)["open_slice"] == 0
    a.destroy()
    b.destroy()
