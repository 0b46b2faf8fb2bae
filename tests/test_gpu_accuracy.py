"""Accuracy of the regained lists against exact opposite numbers (Sec. 5):
FPR = hosts reported but below theta / true super points, FNR = true super
points not reported / true super points, TFR = FPR + FNR, over full windows.
The rates are reported (the paper's 1.43% / 0.97% are on a trace that is not
available, so they are context only); the assertions are loose sanity bounds
on what the method must achieve on these synthetic traces.  Each run also
reports where its false positives come from -- hosts absent from the window
altogether (regained from hot estimators of different hosts) or present
with fewer than theta peers (estimates above the true count) -- and the
hot estimators per row at the last close."""
import numpy as np
import pytest
import torch

import paper_1803_11036_amd as ssd
import tracegen as tg
from _parity import log, to_dev
from oracle import truth

pytestmark = pytest.mark.gpu


def _origin(got, true, window_hosts):
    """False positives of one window: (absent from the window, present with
    fewer than theta peers)."""
    fp = np.setdiff1d(got, true)
    absent = np.setdiff1d(fp, window_hosts).size
    return absent, fp.size - absent


def _origin_note(absent, light, hot):
    n = absent + light
    share = f"{100 * absent / n:.1f}% absent from the window" if n else "none"
    return f"false positives {n}: {share}, {light} present below theta; hot estimators per row {hot}"


def _run(cfg, rehash=False, n_slices=None, use_device_fill=False):
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    p = ssd.make_params(q=cfg.q, r=cfg.r, delta=cfg.delta, eta=cfg.eta, k=cfg.k, theta=cfg.theta,
                        verify_rehash=rehash, max_tuples=1 << 22, max_results=1 << 20)
    det = ssd.init_detector(p, tabs, device="cuda:0")
    n_slices = n_slices or cfg.n_slices
    sl, rows = [], []
    absent = light = 0
    for t in range(n_slices):
        pairs = tr.pairs(0, t)
        sl.append(pairs)
        ssd.scan_slice(det, to_dev(pairs), t)
        res = ssd.close_slice(det)
        if t >= cfg.k - 1:                       # full windows only
            true = truth.window_super_points(sl, t, cfg.k, cfg.theta)
            got = res["ip"]
            tp = np.intersect1d(got, true).size
            fp, fn = got.size - tp, true.size - tp
            rows.append((t, true.size, got.size, fp, fn))
            hosts = np.unique(np.concatenate([s_[:, 0] for s_ in sl[t - cfg.k + 1:t + 1]]))
            a, b = _origin(got, true, hosts)
            absent, light = absent + a, light + b
        if t >= cfg.k:
            sl[t - cfg.k] = None                 # keep memory bounded
    hot = ssd.get_info(det)["hot_counts"]
    det.destroy()
    n_true = sum(r[1] for r in rows)
    fpr = sum(r[3] for r in rows) / max(1, n_true)
    fnr = sum(r[4] for r in rows) / max(1, n_true)
    log(_origin_note(absent, light, hot))
    return fpr, fnr, rows


@pytest.mark.parametrize("name,rehash,k", [("tiny", False, 4), ("tiny", True, 4), ("tiny", True, 1)])
def test_accuracy_tiny(name, rehash, k):
    cfg = tg.config(name, k=k, pairs_lo=max(1_000_000, 2_000_000 // k), pairs_hi=max(1_000_000, 2_000_000 // k))
    fpr, fnr, rows = _run(cfg, rehash=rehash)
    log(f"accuracy {name} k={k} rehash={rehash}: FPR {100 * fpr:.2f}% FNR {100 * fnr:.2f}% "
        f"TFR {100 * (fpr + fnr):.2f}% over {len(rows)} windows, true/reported per window "
        f"{[(r[1], r[2]) for r in rows]}")
    assert fnr < 0.05
    if rehash:
        assert fpr < 0.10


@pytest.mark.parametrize("rehash", [False, True])
def test_accuracy_core_link(rehash):
    cfg = tg.config("core_link")
    fpr, fnr, rows = _run(cfg, rehash=rehash, n_slices=cfg.k + 3)
    log(f"accuracy core_link rehash={rehash}: FPR {100 * fpr:.2f}% FNR {100 * fnr:.2f}% "
        f"TFR {100 * (fpr + fnr):.2f}% over {len(rows)} windows, true/reported per window "
        f"{[(r[1], r[2]) for r in rows]}")
    assert fnr < 0.05
    if rehash:
        assert fpr < 0.10


def _rates(rows):
    n_true = sum(r[1] for r in rows)
    return sum(r[3] for r in rows) / max(1, n_true), sum(r[4] for r in rows) / max(1, n_true)


def _row(t, got, true):
    tp = np.intersect1d(got, true).size
    return (t, true.size, got.size, got.size - tp, true.size - tp)


@pytest.mark.parametrize("rehash", [False, True])
def test_accuracy_paper_shape(rehash):
    """The paper's sliding-window experiment shape (Sec. 5): one-second slots,
    k = 300, eta = 2^11, q = 14, r = 5, delta = 6, theta = 1024 (16-bit
    cells), 360 slots of 6M pairs of a core-link-shaped trace: FPR, FNR and
    TFR over the 61 full windows SW(0,300) ... SW(60,300), against exact
    sliding opposite numbers."""
    cfg = tg.config("paper")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    p = ssd.make_params(q=cfg.q, r=cfg.r, delta=cfg.delta, eta=cfg.eta, k=cfg.k, theta=cfg.theta,
                        verify_rehash=rehash, max_tuples=1 << 22, max_results=1 << 20, cell_bits=16)
    det = ssd.init_detector(p, tabs, device="cuda:0")
    exact = truth.SlidingWindowTruth(cfg.k, cfg.theta)
    rows = []
    absent = light = 0
    for t in range(cfg.n_slices):
        d = tr.distinct(0, t)
        ssd.scan_slice(det, tr.pairs_device(0, t, "cuda:0", d=d), t)
        res = ssd.close_slice(det)
        true = exact.add(d)
        if t >= cfg.k - 1:
            rows.append(_row(t, res["ip"], true))
            if t % 10 == 0:                      # the origin on every tenth window (a host scan of 6M pairs)
                a, b = _origin(res["ip"], true, np.unique((exact.keys >> np.uint64(32)).astype(np.uint32)))
                absent, light = absent + a, light + b
        if t % 60 == 0:
            log(f"paper shape slot {t}: {len(res)} reported")
    log(_origin_note(absent, light, ssd.get_info(det)["hot_counts"]) + " (every tenth window)")
    det.destroy()
    fpr, fnr = _rates(rows)
    log(f"accuracy paper shape (k=300) rehash={rehash}: FPR {100 * fpr:.2f}% FNR {100 * fnr:.2f}% "
        f"TFR {100 * (fpr + fnr):.2f}% over {len(rows)} windows; true per window "
        f"{min(r[1] for r in rows)}..{max(r[1] for r in rows)}, reported {min(r[2] for r in rows)}.."
        f"{max(r[2] for r in rows)}")
    assert len(rows) == cfg.n_slices - cfg.k + 1
    assert fnr < 0.05
    if rehash:
        assert fpr < 0.10


@pytest.mark.parametrize("rehash", [False, True])
def test_accuracy_distributed_merged(rehash):
    """The distributed workload (16 routers, k = 8, theta = 2048): the global
    detector after the per-slot merge (Alg. 5) against the exact sliding
    opposite numbers of every router's pairs together, over the full
    windows of 24 slots."""
    cfg = tg.config("distributed")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    p = ssd.make_params(q=cfg.q, r=cfg.r, delta=cfg.delta, eta=cfg.eta, k=cfg.k, theta=cfg.theta,
                        verify_rehash=rehash, max_tuples=1 << 22, max_results=1 << 20)
    routers = [ssd.init_detector(p, tabs, device="cuda:0") for _ in range(cfg.n_streams)]
    glob = ssd.init_detector(p, tabs, device="cuda:0")
    exact = truth.SlidingWindowTruth(cfg.k, cfg.theta)
    rows = []
    absent = light = 0
    for t in range(cfg.n_slices):
        per = tr.distinct_all(t)
        for j, d in enumerate(routers):
            ssd.scan_slice(d, tr.pairs_device(j, t, "cuda:0", d=per[j]), t)
        ssd.merge_router_state(glob, routers)
        res = ssd.close_slice(glob)
        for d in routers:
            ssd.close_slice(d, advance_only=True)
        true = exact.add(np.concatenate(per))
        if t >= cfg.k - 1:
            rows.append(_row(t, res["ip"], true))
            a, b = _origin(res["ip"], true, np.unique((exact.keys >> np.uint64(32)).astype(np.uint32)))
            absent, light = absent + a, light + b
    log(_origin_note(absent, light, ssd.get_info(glob)["hot_counts"]))
    for d in routers + [glob]:
        d.destroy()
    fpr, fnr = _rates(rows)
    log(f"accuracy distributed merged rehash={rehash}: FPR {100 * fpr:.2f}% FNR {100 * fnr:.2f}% "
        f"TFR {100 * (fpr + fnr):.2f}% over {len(rows)} windows, true/reported per window "
        f"{[(r[1], r[2]) for r in rows]}")
    assert fnr < 0.05
    if rehash:
        assert fpr < 0.10


@pytest.mark.parametrize("rehash", [False, True])
def test_accuracy_batched_links(rehash):
    """Batched links (the 64-link workload's links with k <= 32, at their full
    rates; window distinct pairs capped at 1.5M per link so that the exact
    counts stay cheap): every link's list from the batch against its own
    exact sliding opposite numbers, over its full windows up to slot k + 7."""
    allc = tg.batch_configs(n_links=64, max_window_distinct=1.5e6)
    pick = [i for i, c in enumerate(allc) if c.k <= 32]
    cfgs = [allc[i] for i in pick]
    traces = [tg.Trace(c) for c in cfgs]
    tabs = [tg.hash_tables(c.hash_seed) for c in cfgs]
    params = [ssd.make_params(q=c.q, r=c.r, delta=c.delta, eta=c.eta, k=c.k, theta=c.theta,
                              verify_rehash=rehash, max_tuples=1 << 21, max_results=1 << 18) for c in cfgs]
    b = ssd.batch_init(params, tabs, device="cuda:0")
    exact = [truth.SlidingWindowTruth(c.k, c.theta) for c in cfgs]
    rows = [[] for _ in cfgs]
    absent = light = 0
    n_slices = max(c.k for c in cfgs) + 8
    for t in range(n_slices):
        dist = [tr.distinct(0, t % tr.cfg.n_slices) for tr in traces]
        parts = [tr.pairs_device(0, t % tr.cfg.n_slices, "cuda:0", d=dist[i]) for i, tr in enumerate(traces)]
        offs = np.zeros(len(parts) + 1, dtype=np.uint64)
        offs[1:] = np.cumsum([int(x.shape[0]) for x in parts])
        ssd.batch_scan(b, torch.cat(parts).contiguous(), offs, t)
        lists, status = ssd.batch_close(b)
        assert np.all(status == 0)
        for i, c in enumerate(cfgs):
            true = exact[i].add(dist[i])
            if c.k - 1 <= t <= c.k + 7:
                rows[i].append(_row(t, lists[i]["ip"], true))
                a, b_ = _origin(lists[i]["ip"], true, np.unique((exact[i].keys >> np.uint64(32)).astype(np.uint32)))
                absent, light = absent + a, light + b_
    hot = [sum(ssd.batch_get_info(b, i)["hot_counts"]) // cfgs[i].r for i in range(len(cfgs))]
    log(_origin_note(absent, light, f"(mean over each link's rows) {min(hot)}..{max(hot)}"))
    b.destroy()
    flat = [r for rs in rows for r in rs]
    fpr, fnr = _rates(flat)
    worst = max(_rates(rs)[1] for rs in rows)
    log(f"accuracy batched ({len(cfgs)} links, k <= 32) rehash={rehash}: FPR {100 * fpr:.2f}% "
        f"FNR {100 * fnr:.2f}% TFR {100 * (fpr + fnr):.2f}% over {len(flat)} link windows; "
        f"worst link FNR {100 * worst:.2f}%")
    assert fnr < 0.05
    if rehash:
        assert fpr < 0.10
