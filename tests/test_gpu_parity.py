"""GPU parity: the HIP detector, called through the C ABI, against the CPU
oracle on the same seeded inputs.  Integer products (window state, R_k, hot
lists, candidate tuples, regained hosts and their R) must match bit for bit;
the f64 estimate within 1e-6 relative."""
import numpy as np
import pytest
import torch

import paper_1803_11036_amd as ssd
import tracegen as tg
from _parity import close_both, compare_state, log, make_pair, scan_both, to_dev

pytestmark = pytest.mark.gpu


def _slices_small(seed, n_slices, key_bits, theta, q, sizes=None, heavy=20, heavy_peers=None):
    """Random slices over a key_bits-wide host space: light background plus
    heavy hosts that enter and leave."""
    rng = np.random.default_rng(seed)
    hosts = rng.choice(2 ** key_bits, min(4000, 2 ** key_bits // 2), replace=False).astype(np.uint32)
    hv = rng.choice(2 ** key_bits, heavy, replace=False).astype(np.uint32)
    start = rng.integers(0, max(1, n_slices - 2), heavy)
    span = rng.integers(1, 8, heavy)
    hp = heavy_peers or 2 * theta
    out = []
    for s in range(n_slices):
        n_bg = int(sizes[s]) if sizes is not None else int(0.05 * (1 << q) * theta)
        bg = np.stack([rng.choice(hosts, n_bg),
                       rng.integers(0, 2 ** 32, n_bg, dtype=np.uint64).astype(np.uint32)], 1)
        parts = [bg]
        for h, a, b in zip(hv, start, start + span):
            if a <= s < b:
                parts.append(np.stack([np.full(hp // 2, h, np.uint32),
                                       rng.integers(0, 2 ** 32, hp // 2, dtype=np.uint64).astype(np.uint32)], 1))
        p = np.concatenate(parts).astype(np.uint32)
        out.append(p[rng.permutation(p.shape[0])])
    return out


@pytest.mark.parametrize("graph,timing", [(1, 1), (0, 0), (1, 0)])
def test_tiny_config(graph, timing):
    """1 router, 8 slices of 1M pairs, k = 4, 2^12 x 6 estimators of 1024
    cells: every product compared at every slice, full window state; the
    close replayed as a graph (with and without timing event nodes) between
    eager scans and reads, or run eagerly."""
    cfg = tg.config("tiny")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    g, o = make_pair(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs)
    ssd.set_tuning(g, ssd.SSD_TUNE_GRAPH, graph)
    ssd.set_tuning(g, ssd.SSD_TUNE_TIMING, timing)
    for t in range(cfg.n_slices):
        log(f"tiny graph={graph} timing={timing} slice {t}")
        scan_both(g, o, tr.pairs(0, t), t)
        compare_state(g, o)
        res = close_both(g, o)
    assert len(res) > 100
    assert np.all(np.isin(tr.planted_ips(), res["ip"]))
    tm = ssd.read_timing(g)
    if timing:
        assert tm["hot_detect"][1] == cfg.n_slices and tm["hot_detect"][0] > 0
        assert tm["close_graph"][1] == (cfg.n_slices if graph else 0)


@pytest.mark.parametrize("splits,mode", [(1, "passes"), (3, "passes"), (7, "passes"), (1, "binned"), (7, "binned"),
                                         (7, "binned_uncounted")])
def test_ragged_batches_and_empty_slices(splits, mode):
    """Pair counts that leave ragged tails (0, 1, 63, 64, 65, 257, odd sizes),
    several scan calls per slice, empty slices, and (binned scan) calls of
    several binning chunks -- binned with per-slot counters (two 512 KiB
    bins; the cells of one slice reach the counters through several launches,
    and calls with too few pairs store uncounted and leave them stale) and
    without."""
    q, r, delta, eta, k, theta, kb = 8, 4, 4, 1024, 3, 200, 16
    sizes = [0, 1, 63, 64, 65, 257, 10007, 0, 12345, 9999, 0, 10240]
    sl = _slices_small(5 + splits, len(sizes), kb, theta, q, sizes=sizes)
    sl = [s if sizes[i] else s[:0] for i, s in enumerate(sl)]
    sl[9] = np.resize(sl[9], (150001, 2))      # the same pairs repeated: one call of several binning chunks
    g, o = make_pair(q, r, delta, eta, k, theta, tg.hash_tables(3), key_bits=kb)
    if mode != "passes":
        ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_MODE, ssd.SSD_SCAN_BINNED)
    if mode == "binned_uncounted":
        ssd.set_tuning(g, ssd.SSD_TUNE_COUNTED, 0)
    ssd.set_tuning(g, ssd.SSD_TUNE_TIMING, 1)
    for t, p in enumerate(sl):
        log(f"ragged splits={splits} {mode} slice {t} n={p.shape[0]}")
        scan_both(g, o, p, t, splits=splits if p.shape[0] >= splits else 1)
        compare_state(g, o)
        close_both(g, o)
    tm = ssd.read_timing(g)
    # counted closes need the slice's calls large enough (256 offsets per bin on
    # average); the others read the state.  The counters are exact until the
    # first uncounted store, so a pass-scan detector's first close (an empty
    # slice here) still counts.
    if mode == "binned":
        assert tm["count_detect"][1] > 1
    else:
        assert tm["count_detect"][1] <= (1 if mode == "passes" else 0)
    assert tm["count_detect"][1] + tm["hot_detect"][1] >= len(sl)


@pytest.mark.parametrize("k,mode", [(1, "passes"), (3, "passes"), (17, "passes"), (254, "passes"),
                                    (1, "counted"), (3, "counted"), (17, "counted"), (64, "counted"),
                                    (100, "counted")])
def test_stamp_wrap_and_expiry(k, mode):
    """300 slices: the 8-bit slot stamps wrap (255 slots) and the rotating
    expiry must keep every cell's distance exact, for the discrete window
    (k = 1, Sec. 3.1), short and maximal windows -- also for R_k taken from
    the per-slot counters, whose slot of an old stamp rests on that
    distance, up to windows whose counters take 40% of the state (k = 100
    at eta = 1024, 100 KiB of counters per 256 KiB bin)."""
    q, r, delta, eta, theta, kb = 8, 4, 4, 1024, 150, 16
    n = 300
    # about 0.15 * 2^q * theta distinct background pairs per window
    per_slice = max(20, int(0.15 * (1 << q) * theta / k))
    sl = _slices_small(40 + k, n, kb, theta, q, sizes=[per_slice] * n, heavy=60 if k < 100 else 8)
    g, o = make_pair(q, r, delta, eta, k, theta, tg.hash_tables(4), key_bits=kb)
    if mode == "counted":
        ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_MODE, ssd.SSD_SCAN_BINNED)
        ssd.set_tuning(g, ssd.SSD_TUNE_COUNTED_MIN_ITEMS, 0)       # count every call, however small
        ssd.set_tuning(g, ssd.SSD_TUNE_TIMING, 1)
    for t, p in enumerate(sl):
        scan_both(g, o, p, t)
        if t % 10 == 0 or t > 250:
            compare_state(g, o)
        close_both(g, o, check_internals=(t % 25 == 0 or (mode == "counted" and t > 250)))
    if mode == "counted":
        assert ssd.read_timing(g)["count_detect"][1] == n
    log(f"wrap k={k} {mode} done")


@pytest.mark.parametrize("mode,n_slices", [("binned", 302), ("marked", 302), ("passes", 24)])
def test_paper_parameter_set_16bit_cells(mode, n_slices):
    """The paper's sliding-window parameter set (Sec. 5): windows of k = 300
    one-second slots, eta = 2^11, q = 14, r = 5, delta = 6, theta = 1024,
    which needs 16-bit cells.  A paper-shaped trace at a lighter load (300K
    background hosts, 60 planted, 30K pairs per slot; about 140 hot
    estimators per row in a full window, which keeps the oracle's literal
    enumeration within seconds per slot) runs k + 2 slots with the default
    (binned) scan, so that the first slots leave the window, the same with
    every call taking the bitmap stores (each touched chunk restamped once;
    by default only calls with 2048 offsets per bin of 2^18 cells), and 24
    slots with pass windows.  Lists at every slot; R_k, hot lists and tuples
    every 25 slots and at the last three; the whole canonical state every 60
    slots and at the end."""
    cfg = tg.config("paper", pairs_lo=30_000, pairs_hi=30_000, n_hosts=300_000, n_planted=60)
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    g, o = make_pair(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs, cell_bits=16)
    if mode == "passes":
        ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_MODE, ssd.SSD_SCAN_PASSES)
    if mode == "marked":
        ssd.set_tuning(g, ssd.SSD_TUNE_COUNTED_MIN_ITEMS, 0)
    ssd.set_tuning(g, ssd.SSD_TUNE_TIMING, 1)
    reported = 0
    for t in range(n_slices):
        scan_both(g, o, tr.pairs(0, t), t, splits=2 if t % 7 == 3 else 1)
        last = t >= n_slices - 3
        if t % 60 == 59 or t == n_slices - 1:
            log(f"paper k=300 {mode} slice {t}: comparing the whole canonical state")
            compare_state(g, o)
        elif t % 20 == 0:
            log(f"paper k=300 {mode} slice {t}")
        res = close_both(g, o, check_internals=(t % 25 == 0 or last))
        reported = len(res)
    assert reported > 0
    tm = ssd.read_timing(g)
    assert tm["hot_detect"][1] == n_slices and tm["count_detect"][1] == 0
    assert (tm["scan_bin"][1] > 0) == (mode != "passes")
    assert ssd.get_info(g)["counted_bin_kib"] == (256 if mode == "marked" else 0)
    log(f"paper k=300 {mode}: {reported} hosts at slice {n_slices - 1}")


def test_16bit_stamp_wrap_and_expiry():
    """16-bit stamps repeat after 65535 slots: scans in the first slots and
    again around slot 65535, advance-only closes in between on both sides.
    The rotating expiry (period 65535 - k) must clear every old cell before
    its stamp comes round again, so that each cell's distance stays exact
    (a cell hit in slot s must not look live at slot s + 65535)."""
    q, r, delta, eta, k, theta, kb = 6, 4, 4, 1024, 5, 150, 14
    g, o = make_pair(q, r, delta, eta, k, theta, tg.hash_tables(12), key_bits=kb, cell_bits=16)
    early, late = range(0, 12), range(65527, 65546)
    sl = _slices_small(61, len(early) + len(late), kb, theta, q, sizes=[600] * (len(early) + len(late)),
                       heavy=12)
    j = 0
    for t in range(late.stop):
        if t in early or t in late:
            scan_both(g, o, sl[j], t)
            j += 1
            if t in late or t % 4 == 0:
                compare_state(g, o)
            close_both(g, o, check_internals=(t in late))
        else:
            assert len(ssd.close_slice(g, advance_only=True)) == 0
            o.close(advance_only=True)
        if t % 10000 == 0:
            log(f"16-bit wrap: slot {t}")
        if t == 65000:
            compare_state(g, o)
            log("16-bit wrap: slot 65000 state equal")
    compare_state(g, o)


def test_many_rows_level_expansion():
    """r = 10 rows (q = 8, delta = 3): above the depth-first bound, so the
    candidates are expanded level by level (nine launches); every product
    compared with the oracle."""
    q, r, delta, eta, k, theta, kb = 8, 10, 3, 1024, 3, 200, 32
    sl = _slices_small(77, 5, kb, theta, q, sizes=[3000] * 5)
    g, o = make_pair(q, r, delta, eta, k, theta, tg.hash_tables(9), key_bits=kb)
    for t, p in enumerate(sl):
        scan_both(g, o, p, t)
        compare_state(g, o)
        res = close_both(g, o)
    assert len(res) > 0


def test_rehash_mode():
    cfg = tg.config("tiny")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    g, o = make_pair(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs, rehash=True)
    for t in range(5):
        scan_both(g, o, tr.pairs(0, t), t)
        res = close_both(g, o)
    assert np.all(np.isin(tr.planted_ips(), res["ip"]))


def test_key_width_beyond_32_bits():
    """(r-2)*delta + q = 34 > 32: tuples that would set bits 32..33 are
    dropped (R13), on both sides."""
    q, r, delta, eta, k, theta = 10, 5, 8, 1024, 3, 150
    sl = _slices_small(77, 6, 32, theta, q, heavy=40)
    g, o = make_pair(q, r, delta, eta, k, theta, tg.hash_tables(8))
    for t, p in enumerate(sl):
        scan_both(g, o, p, t)
        compare_state(g, o)
        close_both(g, o)


@pytest.mark.parametrize("k,cell_bits", [(3, 8), (300, 16)])
def test_merge_routers(k, cell_bits):
    """Alg. 5: four router detectors merged into a global one every slot;
    the global close must match the oracle's merged RSEA, and routers only
    advance their clocks (8-bit cells, and 16-bit cells with a 300-slot
    window)."""
    q, r, delta, eta, theta, kb = 8, 4, 4, 1024, 200, 16
    tabs = tg.hash_tables(9)
    nR = 4
    gpu_r, orc_r = zip(*[make_pair(q, r, delta, eta, k, theta, tabs, key_bits=kb, cell_bits=cell_bits)
                         for _ in range(nR)])
    g, o = make_pair(q, r, delta, eta, k, theta, tabs, key_bits=kb, cell_bits=cell_bits)
    rng = np.random.default_rng(10)
    for t in range(8):
        sl = _slices_small(100 + t, 1, kb, theta // 2, q, heavy=15)[0]
        parts = np.array_split(sl[rng.permutation(sl.shape[0])], nR)
        for j in range(nR):
            scan_both(gpu_r[j], orc_r[j], parts[j], t)
        ssd.merge_router_state(g, list(gpu_r))
        o.merge_from(list(orc_r))
        compare_state(g, o)
        close_both(g, o)
        for j in range(nR):
            assert len(ssd.close_slice(gpu_r[j], advance_only=True)) == 0
            orc_r[j].close(advance_only=True)
            compare_state(gpu_r[j], orc_r[j])


def test_scan_pass_windows_do_not_change_state():
    cfg = tg.config("tiny")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    g, o = make_pair(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs)
    ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_PASS_BYTES, 3 << 20)     # 8 passes, ragged last one
    for t in range(3):
        scan_both(g, o, tr.pairs(0, t), t)
        compare_state(g, o)
        close_both(g, o, check_internals=False)


@pytest.mark.parametrize("bin_kib,counted", [(256, 0), (2048, 0), (4096, 0), (1024, 1), (256, 1)])
def test_binned_scan_matches_oracle(bin_kib, counted):
    """The bin-sorted scan (96, 12 or 6 bins over the 24 MiB state; offsets
    packed three to a word up to 2 MiB bins, 4 bytes each above; with
    per-slot counters, 24 bins of 1 MiB or 96 of 256 KiB, whose marked words
    overflow the visit list) gives the oracle's state and lists, also for one
    call of 3.5M pairs (several binning chunks, the last one ragged) and for a
    slice split over five calls."""
    cfg = tg.config("tiny")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    g, o = make_pair(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs)
    ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_MODE, ssd.SSD_SCAN_BINNED)
    ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_BIN_BYTES, bin_kib << 10)
    ssd.set_tuning(g, ssd.SSD_TUNE_COUNTED, counted)
    for t in range(4):
        pairs = tr.pairs(0, t)
        if t == 1:
            pairs = np.concatenate([pairs] * 4)[:3_500_001]
        log(f"binned {bin_kib} KiB slice {t} n={pairs.shape[0]}")
        scan_both(g, o, pairs, t, splits=5 if t == 2 else 1)
        compare_state(g, o)
        close_both(g, o, check_internals=(t == 3))


@pytest.mark.parametrize("q,r,delta,counted", [(12, 4, 10, 0), (12, 4, 10, 1), (14, 5, 6, 0), (14, 5, 6, 1),
                                                (12, 6, 5, 0), (12, 6, 5, 1)])
def test_binned_scan_rows_match_oracle(q, r, delta, counted):
    """Every binning kernel against the oracle on small states with the
    binned scan forced: four rows (the general binning), five rows (the
    register binning of up to 7 pairs per thread, as in the paper's geometry
    q = 14, delta = 6) and six rows (up to 6 pairs per thread), with per-slot
    counters and without; canonical state, lists, R_k, hot lists and tuples
    every slice, one slice split over three calls."""
    eta, k, theta, kb = 1024, 3, 300, 32
    sizes = [60_000, 90_001, 45_000, 120_000, 70_000]
    sl = _slices_small(300 + r, len(sizes), kb, theta, q, sizes=sizes, heavy=24)
    g, o = make_pair(q, r, delta, eta, k, theta, tg.hash_tables(20 + r), key_bits=kb)
    ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_MODE, ssd.SSD_SCAN_BINNED)
    ssd.set_tuning(g, ssd.SSD_TUNE_COUNTED, counted)
    ssd.set_tuning(g, ssd.SSD_TUNE_TIMING, 1)
    for t, p in enumerate(sl):
        log(f"binned rows r={r} counted={counted} slice {t} n={p.shape[0]}")
        scan_both(g, o, p, t, splits=3 if t == 1 else 1)
        compare_state(g, o)
        close_both(g, o)
    tm = ssd.read_timing(g)
    assert tm["scan_bin"][1] >= len(sl)
    assert (tm["count_detect"][1] > 0) == bool(counted)


# (q, r, delta, eta, k, theta, key_bits, cell_bits): the edges of the
# parameter space the boundary accepts
_EXTREMES = {
    "r3_fewest_rows": (10, 3, 6, 1024, 2, 150, 16, 8),
    "delta1": (12, 6, 1, 1024, 3, 200, 16, 8),
    "delta12_cover38": (14, 4, 12, 1024, 3, 200, 32, 8),
    "q4_fewest_columns": (4, 4, 3, 1024, 3, 150, 8, 8),
    "eta16k_counted": (8, 4, 4, 16384, 3, 5000, 16, 8),
    "eta32k": (7, 5, 4, 32768, 2, 10000, 16, 8),
    "eta64k": (6, 4, 4, 65536, 3, 20000, 14, 8),
    "eta64k_16bit": (6, 4, 4, 65536, 4, 20000, 14, 16),
}


@pytest.mark.parametrize("mode", ["auto", "binned"])
@pytest.mark.parametrize("case", list(_EXTREMES))
def test_parameter_extremes(case, mode):
    """The edges of the accepted parameters against the oracle: the fewest
    rows (r = 3: level 0 only), the narrowest and widest overlaps (delta = 1;
    delta = 12 with (r-2)*delta + q = 38 > 32 bits), the fewest columns
    (q = 4, 8-bit keys) and the largest estimators (eta = 2^14 with per-slot
    counters, 2^15, and 2^16 with 8- and 16-bit cells), through the default
    scan and through the binned scan; canonical state, R_k, hot lists, tuples
    and lists every slice, one slice split over three calls."""
    q, r, delta, eta, k, theta, kb, cb = _EXTREMES[case]
    n_slices = k + 3
    # about ten peers per background host and slice: only the heavy hosts go hot
    bg = 10 * min(4000, 2 ** kb // 2)
    sl = _slices_small(500 + q * 7 + r, n_slices, kb, theta, q, sizes=[bg] * n_slices, heavy=12)
    g, o = make_pair(q, r, delta, eta, k, theta, tg.hash_tables(40 + q + r), key_bits=kb, cell_bits=cb)
    if mode == "binned":
        ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_MODE, ssd.SSD_SCAN_BINNED)
    ssd.set_tuning(g, ssd.SSD_TUNE_TIMING, 1)
    found = 0
    for t, p in enumerate(sl):
        log(f"extremes {case} {mode} slice {t} n={p.shape[0]}")
        scan_both(g, o, p, t, splits=3 if t == 1 else 1)
        compare_state(g, o)
        found += len(close_both(g, o))
    assert found > 0
    tm = ssd.read_timing(g)
    if mode == "binned":
        assert tm["scan_bin"][1] >= n_slices
    if case == "eta16k_counted" and mode == "binned":
        assert tm["count_detect"][1] > 0


def test_counted_detection_switches():
    """R_k from the per-slot counters through every switch of the counted
    path: counted from the first slice, stale after a pass scan (full hot
    detection), rebuilt from the state at the close after the next binned
    scan, counting switched off and on again, slices split over several
    calls, and a slice of one small call (too few offsets per bin to count:
    full hot detection, no rebuild) -- every product equals the oracle's at
    every slice."""
    cfg = tg.config("tiny")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    g, o = make_pair(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs)
    ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_MODE, ssd.SSD_SCAN_BINNED)
    ssd.set_tuning(g, ssd.SSD_TUNE_TIMING, 1)
    # (scan mode, counted knob, calls): expected detection path and launches
    plan = [(ssd.SSD_SCAN_BINNED, 1, 1, "count", 1), (ssd.SSD_SCAN_BINNED, 1, 3, "count", 1),
            (ssd.SSD_SCAN_PASSES, 1, 1, "full", 1), (ssd.SSD_SCAN_BINNED, 1, 2, "count", 2),
            (ssd.SSD_SCAN_BINNED, 1, 1, "count", 1), (ssd.SSD_SCAN_BINNED, 0, 1, "full", 1),
            (ssd.SSD_SCAN_BINNED, 1, 1, "count", 2), (ssd.SSD_SCAN_BINNED, 1, 4, "count", 1),
            (ssd.SSD_SCAN_BINNED, 1, 0, "full", 1), (ssd.SSD_SCAN_BINNED, 1, 1, "count", 2)]
    for t, (mode, counted, calls, path, launches) in enumerate(plan):
        ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_MODE, mode)
        ssd.set_tuning(g, ssd.SSD_TUNE_COUNTED, counted)
        log(f"counted switches slice {t}: mode {mode} counted {counted} calls {calls}")
        pairs = tr.pairs(0, t % cfg.n_slices)
        if calls == 0:                                  # one call of 1000 pairs: about 125 offsets per bin
            pairs, calls = pairs[:1000], 1
        scan_both(g, o, pairs, t, splits=calls)
        close_both(g, o)
        tm = ssd.read_timing(g, reset=True)
        if path == "count":
            assert tm["count_detect"][1] == launches and tm["hot_detect"][1] == 0, f"slice {t}: {tm}"
        else:
            assert tm["hot_detect"][1] == launches and tm["count_detect"][1] == 0, f"slice {t}: {tm}"
    compare_state(g, o)


def test_counted_after_advance_and_merge():
    """The per-slot counters go stale after an advance-only close and after a
    router merge into the detector (Alg. 5); the close after the detector's
    next binned scan rebuilds them from the state, a close with no scan of
    its own detects from the whole state.  Every product equals the
    oracle's, and counting cannot be switched on for a detector whose
    counters would exceed half its state (eta < 8 k)."""
    q, r, delta, eta, k, theta, kb = 8, 4, 4, 1024, 3, 200, 16
    tabs = tg.hash_tables(9)
    g, o = make_pair(q, r, delta, eta, k, theta, tabs, key_bits=kb)
    gr, orr = make_pair(q, r, delta, eta, k, theta, tabs, key_bits=kb)
    ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_MODE, ssd.SSD_SCAN_BINNED)
    ssd.set_tuning(g, ssd.SSD_TUNE_COUNTED_MIN_ITEMS, 0)           # count every call, however small
    ssd.set_tuning(g, ssd.SSD_TUNE_TIMING, 1)
    sl = _slices_small(200, 8, kb, theta // 2, q, heavy=15)
    # (own scan, router merged, advance only) -> detection path, launches
    plan = [(1, 0, 0, "count", 1), (1, 0, 0, "count", 1), (1, 0, 1, None, 0), (1, 0, 0, "count", 2),
            (1, 1, 0, "count", 2), (0, 1, 0, "full", 1), (1, 0, 0, "count", 2), (1, 0, 0, "count", 1)]
    for t, (own, merged, adv, path, launches) in enumerate(plan):
        half = sl[t].shape[0] // 2
        mine, theirs = sl[t][:half], sl[t][half:]
        scan_both(gr, orr, theirs, t)
        if merged:
            ssd.merge_router_state(g, [gr])
            o.merge_from([orr])
        if own:
            scan_both(g, o, mine, t)
        log(f"counted stale slice {t}: own {own} merged {merged} advance {adv}")
        if adv:
            assert len(ssd.close_slice(g, advance_only=True)) == 0
            o.close(advance_only=True)
        else:
            close_both(g, o)
        compare_state(g, o)
        tm = ssd.read_timing(g, reset=True)
        if path == "count":
            assert tm["count_detect"][1] == launches and tm["hot_detect"][1] == 0, f"slice {t}: {tm}"
        elif path == "full":
            assert tm["hot_detect"][1] == launches and tm["count_detect"][1] == 0, f"slice {t}: {tm}"
        assert len(ssd.close_slice(gr, advance_only=True)) == 0
        orr.close(advance_only=True)
    wide = ssd.init_detector(ssd.make_params(q=8, r=4, delta=4, eta=1024, k=254, theta=200, key_bits=16),
                             tabs, device="cuda:0")
    with pytest.raises(ssd.SSDError) as e:
        ssd.set_tuning(wide, ssd.SSD_TUNE_COUNTED, 1)
    assert e.value.status == -1
    ssd.set_tuning(wide, ssd.SSD_TUNE_COUNTED, 0)
    wide.destroy()


@pytest.mark.parametrize("mode", ["auto", "counted"])
def test_pipelined_close_matches_oracle(mode):
    """close_begin / close_end with the next slice's scans enqueued between
    them give the oracle's lists and state, also with the next slice's
    counted scan moving the counters while the close's second part runs;
    misuse is rejected."""
    cfg = tg.config("tiny")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    g, o = make_pair(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs)
    if mode == "counted":
        ssd.set_tuning(g, ssd.SSD_TUNE_SCAN_MODE, ssd.SSD_SCAN_BINNED)
    with pytest.raises(ssd.SSDError) as e:
        ssd.close_end(g)
    assert e.value.status == -3
    o.scan(tr.pairs(0, 0))
    ssd.scan_slice(g, to_dev(tr.pairs(0, 0)), 0)
    for t in range(1, 6):
        ssd.close_begin(g)
        with pytest.raises(ssd.SSDError) as e:
            ssd.close_begin(g)
        assert e.value.status == -3
        with pytest.raises(ssd.SSDError) as e:
            ssd.close_slice(g)
        assert e.value.status == -3
        ip, rk, est = o.close()                    # reconstruct, then age
        nxt = tr.pairs(0, t)
        ssd.scan_slice(g, to_dev(nxt), t)          # slice t while close t-1 is pending
        res = ssd.close_end(g)
        assert np.array_equal(res["ip"], ip) and np.array_equal(res["rk"], rk)
        assert np.all(np.abs(res["est"] - est) <= 1e-6 * np.abs(est))
        o.scan(nxt)
        compare_state(g, o)
    close_both(g, o)


def test_multi_kernel_sort_path():
    """Result lists above the single-workgroup limit go through the global
    bitonic sort; forcing that path must not change the list."""
    cfg = tg.config("tiny")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    g, o = make_pair(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs)
    ssd.set_tuning(g, ssd.SSD_TUNE_SORT_BLOCK_LIMIT, 0)
    for t in range(5):
        scan_both(g, o, tr.pairs(0, t), t)
        res = close_both(g, o, check_internals=False)
    assert len(res) > 1000


def test_errors_order_and_overflow():
    cfg = tg.config("tiny")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    p = ssd.make_params(q=cfg.q, r=cfg.r, delta=cfg.delta, eta=cfg.eta, k=cfg.k, theta=cfg.theta,
                        max_tuples=64)
    g = ssd.init_detector(p, tabs, device="cuda:0")
    pairs = to_dev(tr.pairs(0, 0))
    with pytest.raises(ssd.SSDError) as e:
        ssd.scan_slice(g, pairs, 1)
    assert e.value.status == -3
    for t in range(4):
        ssd.scan_slice(g, to_dev(tr.pairs(0, t)), t)
        if t < 3:
            ssd.close_slice(g, advance_only=True)
    with pytest.raises(ssd.SSDError) as e:
        ssd.close_slice(g)            # full window: far more than 64 candidate tuples
    assert e.value.status == -4
    assert ssd.get_info(g)["open_slice"] == 4
    # the detector stays usable after an overflow
    ssd.scan_slice(g, pairs, 4)
    with pytest.raises(ssd.SSDError):
        ssd.close_slice(g)
    g2 = ssd.init_detector(ssd.make_params(q=cfg.q, r=cfg.r, delta=cfg.delta, eta=cfg.eta, k=cfg.k,
                                           theta=cfg.theta), tabs, device="cuda:0")
    with pytest.raises(ssd.SSDError) as e:
        ssd.merge_router_state(g2, [g])
    assert e.value.status == -5
