"""GPU parity at full workload sizes.

- The single core link (6M pairs per slice, 6 x 2^16 estimators of 4096 cells,
  k = 10) in the launch configuration that bench.py times, against the oracle
  for one full window plus a slide: regained hosts, R_k, hot lists and
  candidate tuples every slice, the window state on sampled estimators.
- The 16-router distributed workload at full size through a property that
  holds at any size: merging the routers' states gives the state, R_k and host
  list of one detector that scanned every router's pairs (Alg. 5, reading R3).
- The same 16-router topology on a smaller array against the oracle's merge.
- The 64-link batched workload at full size in the benchmark's launch
  configuration, three sampled links against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1803_11036_amd as ssd
import tracegen as tg
from _parity import close_both, compare_state, log, make_pair, scan_both, to_dev

pytestmark = pytest.mark.gpu


def test_core_link_full_size():
    cfg = tg.config("core_link")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    # same parameters as bench.py
    g, o = make_pair(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs,
                     max_tuples=1 << 22, max_results=1 << 20)
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(g.n_se, 2048, replace=False))
    for t in range(cfg.k + 2):
        scan_both(g, o, tr.pairs(0, t), t)
        if t % 4 == 3 or t == cfg.k + 1:
            compare_state(g, o, sample_se=sample)
        res = close_both(g, o)
        log(f"core_link slice {t}: {len(res)} hosts")
    assert len(res) > 500


def test_core_link_full_size_split_calls_pipelined():
    """The core link with every slice split over three counted scan calls
    (2M pairs, about 3,900 offsets per 512 KiB bin each) and the close
    pipelined behind the next slice's scans (close_begin / close_end): lists
    equal the oracle's at every slice, R_k at the last."""
    cfg = tg.config("core_link")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    g, o = make_pair(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs,
                     max_tuples=1 << 22, max_results=1 << 20)
    ssd.set_tuning(g, ssd.SSD_TUNE_TIMING, 1)
    n = 5
    scan_both(g, o, tr.pairs(0, 0), 0, splits=3)
    for t in range(1, n + 1):
        ssd.close_begin(g)
        ip, rk, est = o.close()
        if t < n:
            scan_both(g, o, tr.pairs(0, t), t, splits=3)      # slice t while close t-1 is pending
        res = ssd.close_end(g)
        assert np.array_equal(res["ip"], ip) and np.array_equal(res["rk"], rk), f"slice {t - 1}: lists differ"
        assert np.all(np.abs(res["est"] - est) <= 1e-6 * np.abs(est))
        log(f"core_link split pipelined slice {t - 1}: {len(res)} hosts")
    assert np.array_equal(ssd.read_rk(g), o.rk())
    tm = ssd.read_timing(g)
    assert tm["count_detect"][1] == n and tm["hot_detect"][1] == 0, tm


def _run_distributed(cfg, tr, tabs, n_slices, with_union=True, with_oracle=False, distinct_only=False):
    R = cfg.n_streams
    params = ssd.make_params(q=cfg.q, r=cfg.r, delta=cfg.delta, eta=cfg.eta, k=cfg.k, theta=cfg.theta,
                             max_tuples=1 << 22, max_results=1 << 20)
    routers = [ssd.init_detector(params, tabs, device="cuda:0") for _ in range(R)]
    glob = ssd.init_detector(params, tabs, device="cuda:0")
    union = ssd.init_detector(params, tabs, device="cuda:0") if with_union else None
    orc_r = [oracle.RSEA(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs) for _ in range(R)] \
        if with_oracle else None
    orc_g = oracle.RSEA(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs) if with_oracle else None
    last = None
    for t in range(n_slices):
        per = tr.distinct_all(t) if distinct_only else tr.pairs_all(t)
        for j in range(R):
            dp = to_dev(per[j])
            ssd.scan_slice(routers[j], dp, t)
            if union is not None:
                ssd.scan_slice(union, dp, t)
            if orc_r is not None:
                orc_r[j].scan(per[j])
        ssd.merge_router_state(glob, routers)
        if union is not None:
            a = ssd.read_canonical_state(glob)
            b = ssd.read_canonical_state(union)
            assert torch.equal(a, b), f"slice {t}: merged state differs from the union's"
            del a, b
        if orc_g is not None:
            orc_g.merge_from(orc_r)
            compare_state(glob, orc_g)
            res = close_both(glob, orc_g)
            for j in range(R):
                orc_r[j].close(advance_only=True)
        else:
            res = ssd.close_slice(glob)
        if union is not None:
            ru = ssd.close_slice(union)
            assert np.array_equal(res, ru), f"slice {t}: host lists differ"
            assert np.array_equal(ssd.read_rk(glob), ssd.read_rk(union))
        for j in range(R):
            ssd.close_slice(routers[j], advance_only=True)
        log(f"{cfg.name} slice {t}: {len(res)} hosts")
        last = res
    return last


def test_distributed_full_size_merge_equals_union():
    cfg = tg.config("distributed")
    tr = tg.Trace(cfg)
    res = _run_distributed(cfg, tr, tg.hash_tables(cfg.hash_seed), cfg.k + 1)
    planted = tr.planted_ips()
    # planted hosts spread over 2-8 routers, most below theta at every router
    assert np.isin(planted[tr.degree[cfg.n_hosts:] >= 2 * cfg.theta], res["ip"]).mean() > 0.9


def test_distributed_16_routers_against_oracle():
    cfg = tg.config("distributed", n_hosts=100_000, n_planted=40, q=12, r=6, delta=5, eta=1024,
                    theta=512)
    tr = tg.Trace(cfg)
    res = _run_distributed(cfg, tr, tg.hash_tables(cfg.hash_seed), cfg.k + 2, with_union=False,
                           with_oracle=True, distinct_only=True)
    assert len(res) > 20


def test_distributed_paper_geometry_against_oracle():
    """The distributed workload's geometry at full state size -- q = 14,
    r = 5, delta = 6 (the paper's), 2^14 x 5 estimators of 4096 cells, 320 MiB
    per router, so every router's scan is binned through the five-row
    register binning -- with four routers at 0.5-1M pairs per slice, merged
    into the global detector every slice (Alg. 5) and compared with the
    oracle's merge: lists, R_k, hot lists and tuples every slice, the whole
    window state every third slice, for k + 2 slices."""
    cfg = tg.config("distributed", n_streams=4, pairs_lo=500_000, pairs_hi=1_000_000)
    assert (cfg.q, cfg.r, cfg.delta, cfg.eta) == (14, 5, 6, 4096)
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    R = cfg.n_streams
    params = ssd.make_params(q=cfg.q, r=cfg.r, delta=cfg.delta, eta=cfg.eta, k=cfg.k, theta=cfg.theta,
                             max_tuples=1 << 22, max_results=1 << 20)
    routers = [ssd.init_detector(params, tabs, device="cuda:0") for _ in range(R)]
    glob = ssd.init_detector(params, tabs, device="cuda:0")
    for d in routers:
        ssd.set_tuning(d, ssd.SSD_TUNE_TIMING, 1)
    orc_r = [oracle.RSEA(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs) for _ in range(R)]
    orc_g = oracle.RSEA(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tabs)
    for t in range(cfg.k + 2):
        per = tr.pairs_all(t)
        for j in range(R):
            ssd.scan_slice(routers[j], to_dev(per[j]), t)
            orc_r[j].scan(per[j])
        ssd.merge_router_state(glob, routers)
        orc_g.merge_from(orc_r)
        if t % 3 == 2:
            compare_state(glob, orc_g)
        res = close_both(glob, orc_g)
        for j in range(R):
            assert len(ssd.close_slice(routers[j], advance_only=True)) == 0
            orc_r[j].close(advance_only=True)
        log(f"distributed paper geometry slice {t}: {len(res)} hosts")
    assert len(res) > 20
    assert all(ssd.read_timing(d)["scan_bin"][1] == cfg.k + 2 for d in routers)
    for d in routers + [glob]:
        d.destroy()


def test_batched_workload_as_benchmarked_against_oracle():
    """The 64-link batched workload at full size (152M pairs per slice, 19 GiB
    of state) in the launch configuration bench.py times -- the autotuner
    running on the first scans, one binning and one store launch for all 64
    links, the close pipelined behind the next slice's scan -- with three
    sampled links (windows up to 10 slices, states up to 1 GiB, binned and
    counted) checked against the oracle fed the same device-generated pairs,
    lists every slice, through the tuning scans and after them."""
    import torch
    cfgs = tg.batch_configs(n_links=64)
    traces = [tg.Trace(c) for c in cfgs]
    tables = [tg.hash_tables(c.hash_seed) for c in cfgs]
    pick = [i for i, c in enumerate(cfgs)
            if c.k <= 10 and c.r * (1 << c.q) * c.eta <= 1 << 30 and c.pairs_lo >= 1 << 16][:3]
    assert len(pick) == 3, pick
    params = [ssd.make_params(q=c.q, r=c.r, delta=c.delta, eta=c.eta, k=c.k, theta=c.theta,
                              max_tuples=1 << 21, max_results=1 << 18) for c in cfgs]
    b = ssd.batch_init(params, tables, device="cuda:0")
    ssd.batch_set_tuning(b, ssd.SSD_TUNE_AUTOTUNE, 1)
    orcs = {i: oracle.RSEA(cfgs[i].q, cfgs[i].r, cfgs[i].delta, cfgs[i].eta, cfgs[i].k, cfgs[i].theta, tables[i])
            for i in pick}
    # k + 2 slices of the longest sampled window, and enough for the
    # autotuner to finish (up to 11 tuning scans, collected one close late)
    # so that the tuned bin sizes are checked too
    n_slices = max(max(cfgs[i].k for i in pick) + 2, 14)
    want = None
    for t in range(n_slices):
        parts = [tr.pairs_device(0, t, "cuda:0") for tr in traces]
        offs = np.zeros(len(parts) + 1, dtype=np.uint64)
        offs[1:] = np.cumsum([int(x.shape[0]) for x in parts])
        pairs = torch.cat(parts).contiguous()
        del parts
        ssd.batch_scan(b, pairs, offs, t)                # while slice t-1's close runs
        if want is not None:
            lists, status = ssd.batch_close_end(b)
            assert np.all(status == 0)
            for i, (ip, rk, est) in want.items():
                assert np.array_equal(lists[i]["ip"], ip) and np.array_equal(lists[i]["rk"], rk), \
                    f"slice {t - 1} link {i}: lists differ from the oracle"
                assert np.all(np.abs(lists[i]["est"] - est) <= 1e-6 * np.abs(est))
            log(f"batched as benchmarked, slice {t - 1}: {sum(len(x) for x in lists)} hosts, sampled links "
                f"{[len(want[i][0]) for i in pick]}")
        ssd.batch_close_begin(b)
        want = {}
        for i in pick:
            orcs[i].scan(pairs[int(offs[i]):int(offs[i + 1])].cpu().numpy().view(np.uint32))
            want[i] = orcs[i].close()
        del pairs
    lists, status = ssd.batch_close_end(b)
    for i, (ip, rk, est) in want.items():
        assert np.array_equal(lists[i]["ip"], ip) and np.array_equal(lists[i]["rk"], rk)
    assert all(ssd.batch_get_info(b, i)["counted"] == 1 for i in pick)
    assert ssd.batch_get_tuning(b, ssd.SSD_TUNE_AUTOTUNE) == 0
    b.destroy()
