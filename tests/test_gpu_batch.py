"""Batched detectors: many links scanned by one persistent launch and closed by
one replayed HIP graph must give, link by link and slice by slice, exactly the
lists of separate detectors fed the same pairs -- and, for small links, the
oracle's lists."""
import numpy as np
import pytest
import torch

import oracle
import paper_1803_11036_amd as ssd
import tracegen as tg
from _parity import log, to_dev

pytestmark = pytest.mark.gpu


def _params(c, **kw):
    return ssd.make_params(q=c.q, r=c.r, delta=c.delta, eta=c.eta, k=c.k, theta=c.theta, **kw)


def _slice_pairs(traces, t):
    per = [tr.pairs(0, t % tr.cfg.n_slices) for tr in traces]
    offs = np.zeros(len(per) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([p.shape[0] for p in per])
    return per, offs, to_dev(np.concatenate(per))


@pytest.mark.parametrize("graph,autotune", [(1, 0), (0, 0), (1, 1)])
def test_batch_equals_separate_detectors(graph, autotune):
    cfgs = tg.batch_configs(n_links=64, pairs_scale=0.02)
    traces = [tg.Trace(c) for c in cfgs]
    tabs = [tg.hash_tables(c.hash_seed) for c in cfgs]
    b = ssd.batch_init([_params(c) for c in cfgs], tabs, device="cuda:0")
    ssd.batch_set_tuning(b, ssd.SSD_TUNE_GRAPH, graph)
    if autotune:
        ssd.batch_set_tuning(b, ssd.SSD_TUNE_AUTOTUNE, 1)
    # small windows so that 4 scans cover several tiles per link
    ssd.batch_set_tuning(b, ssd.SSD_TUNE_SCAN_PASS_BYTES, 64 << 20)
    plain = [ssd.init_detector(_params(c), tabs[i], device="cuda:0") for i, c in enumerate(cfgs)]
    small = [i for i, c in enumerate(cfgs) if c.r * (1 << c.q) * c.eta <= 64 << 20][:3]
    orcs = {i: oracle.RSEA(cfgs[i].q, cfgs[i].r, cfgs[i].delta, cfgs[i].eta, cfgs[i].k, cfgs[i].theta, tabs[i])
            for i in small}
    n_slices = 14 if autotune else 6
    total = 0
    for t in range(n_slices):
        per, offs, dev = _slice_pairs(traces, t)
        ssd.batch_scan(b, dev, offs, t)
        lists, status = ssd.batch_close(b)
        assert np.all(status == 0)
        for i in range(len(cfgs)):
            ssd.scan_slice(plain[i], dev[int(offs[i]):int(offs[i + 1])], t)
            res = ssd.close_slice(plain[i])
            assert np.array_equal(lists[i], res), f"slice {t} link {i}: batch and separate detector differ"
            total += len(res)
        for i, o in orcs.items():
            o.scan(per[i])
            ip, rk, est = o.close()
            assert np.array_equal(lists[i]["ip"], ip) and np.array_equal(lists[i]["rk"], rk)
            assert np.all(np.abs(lists[i]["est"] - est) <= 1e-6 * np.abs(est))
        log(f"batch graph={graph} autotune={autotune} slice {t}: {sum(len(x) for x in lists)} hosts")
    assert total > 100
    if autotune:
        assert ssd.batch_get_tuning(b, ssd.SSD_TUNE_AUTOTUNE) == 0        # finished, a candidate kept
        # the counted links' bin sizes: each class's fastest candidate, kept
        # after tuning (the lists above equal the separate detectors' through
        # the tuning scans' changes of bin size)
        kib = [ssd.batch_get_info(b, i)["counted_bin_kib"] for i in range(len(cfgs))]
        log(f"autotuned counted bin sizes (KiB): {kib}")
        assert any(kib) and set(kib) <= {0, 256, 512, 1024}
    b.destroy()
    for d in plain:
        d.destroy()


def test_batch_close_begin_end_pipelined():
    """The batch close in two halves with the next slice's scan enqueued
    between them: every link's list equals its separate detector's and, for
    small links, the oracle's, slice by slice; a second begin, an end with
    nothing pending and reads while a close is pending are refused."""
    cfgs = tg.batch_configs(n_links=64, pairs_scale=0.02)
    traces = [tg.Trace(c) for c in cfgs]
    tabs = [tg.hash_tables(c.hash_seed) for c in cfgs]
    b = ssd.batch_init([_params(c) for c in cfgs], tabs, device="cuda:0")
    plain = [ssd.init_detector(_params(c), tabs[i], device="cuda:0") for i, c in enumerate(cfgs)]
    small = [i for i, c in enumerate(cfgs) if c.r * (1 << c.q) * c.eta <= 64 << 20][:3]
    orcs = {i: oracle.RSEA(cfgs[i].q, cfgs[i].r, cfgs[i].delta, cfgs[i].eta, cfgs[i].k, cfgs[i].theta, tabs[i])
            for i in small}
    n_slices = 6
    want = []
    for t in range(n_slices):
        per, offs, dev = _slice_pairs(traces, t)
        ssd.batch_scan(b, dev, offs, t)                 # while slice t-1's close runs
        if t > 0:
            lists, status = ssd.batch_close_end(b)
            assert np.all(status == 0)
            for i, ref in enumerate(want):
                assert np.array_equal(lists[i], ref), f"slice {t - 1} link {i}: pipelined batch differs"
        want = []
        for i in range(len(cfgs)):
            ssd.scan_slice(plain[i], dev[int(offs[i]):int(offs[i + 1])], t)
            want.append(ssd.close_slice(plain[i]))
        for i, o in orcs.items():
            o.scan(per[i])
            ip, rk, est = o.close()
            assert np.array_equal(want[i]["ip"], ip) and np.array_equal(want[i]["rk"], rk)
        ssd.batch_close_begin(b)
        if t == 2:
            for call in (lambda: ssd.batch_close_begin(b), lambda: ssd.batch_get_results(b),
                         lambda: ssd.batch_read_rk(b, 0)):
                with pytest.raises(ssd.SSDError) as e:
                    call()
                assert e.value.status == ssd.SSD_E_ORDER
        log(f"batch pipelined slice {t}: {sum(len(x) for x in want)} hosts")
    lists, status = ssd.batch_close_end(b)
    for i, ref in enumerate(want):
        assert np.array_equal(lists[i], ref)
    with pytest.raises(ssd.SSDError) as e:
        ssd.batch_close_end(b)
    assert e.value.status == ssd.SSD_E_ORDER
    b.destroy()
    for d in plain:
        d.destroy()


def test_batch_counted_links_through_stamp_wrap():
    """300 slices, so that every link's 8-bit stamps wrap (255 slots): six
    links of 24 MiB states and 70K pairs per slice, windows k = 1, 3, 17, 64,
    100 and 254, scanned by the batch's multi-link binned stores with per-slot
    counters (k = 100 in the store launch whose LDS takes a whole compute
    unit; k = 254 cannot count) and R_k from k_count_multi, against separate
    detectors scanning pass windows and reading their whole states (pinned
    to the oracle through the wrap): every link's list equal every slice."""
    ks = [1, 3, 17, 64, 100, 254]
    q, r, delta, eta, theta, kb = 12, 6, 5, 1024, 200, 24
    params = [ssd.make_params(q=q, r=r, delta=delta, eta=eta, k=k, theta=theta, key_bits=kb) for k in ks]
    tabs = [tg.hash_tables(40 + i) for i in range(len(ks))]
    b = ssd.batch_init(params, tabs, device="cuda:0")
    ssd.batch_set_tuning(b, ssd.SSD_TUNE_TIMING, 1)
    plain = [ssd.init_detector(p, tabs[i], device="cuda:0") for i, p in enumerate(params)]
    rng = np.random.default_rng(77)
    hosts = [rng.choice(2 ** kb, 3000, replace=False).astype(np.uint32) for _ in ks]
    heavy = [rng.choice(2 ** kb, 12, replace=False).astype(np.uint32) for _ in ks]
    n_slices, total = 300, 0
    for t in range(n_slices):
        per = []
        for i, k in enumerate(ks):
            # about 2e5 distinct background pairs per window (3000 hosts, well
            # below theta each), and four heavy hosts at a time, each active
            # for 20-slice runs with about 2 theta distinct peers per window;
            # the slice filled to 70K pairs with repeats of its distinct ones
            nb = min(60_000, 200_000 // k)
            bg = np.stack([rng.choice(hosts[i], nb), rng.integers(0, 2 ** 32, nb, dtype=np.uint64).astype(np.uint32)], 1)
            act = heavy[i][(np.arange(12) + t // 20) % 3 == 0]
            m = 2 * theta // k + 2
            hv = np.stack([np.repeat(act, m), rng.integers(0, 2 ** 32, m * len(act), dtype=np.uint64).astype(np.uint32)], 1)
            d = np.concatenate([bg, hv]).astype(np.uint32)
            full = np.concatenate([d, d[rng.integers(0, d.shape[0], max(0, 70_000 - d.shape[0]))]])
            per.append(full[rng.permutation(full.shape[0])])
        offs = np.zeros(len(per) + 1, dtype=np.uint64)
        offs[1:] = np.cumsum([p.shape[0] for p in per])
        dev = to_dev(np.concatenate(per))
        ssd.batch_scan(b, dev, offs, t)
        lists, status = ssd.batch_close(b)
        assert np.all(status == 0)
        for i in range(len(ks)):
            ssd.scan_slice(plain[i], dev[int(offs[i]):int(offs[i + 1])], t)
            want = ssd.close_slice(plain[i])
            assert np.array_equal(lists[i], want), f"slice {t} link {i} (k = {ks[i]}): batch differs"
            total += len(want)
        if t % 50 == 0 or t == n_slices - 1:
            modes = [ssd.batch_get_info(b, i)["counted"] for i in range(len(ks))]
            log(f"batch wrap slice {t}: {sum(len(x) for x in lists)} hosts, detection modes {modes}")
    modes = [ssd.batch_get_info(b, i)["counted"] for i in range(len(ks))]
    assert modes[:5] == [1] * 5 and modes[5] == 0, modes
    assert total > 1000
    b.destroy()
    for d in plain:
        d.destroy()


def test_batch_binned_links_equal_separate_detectors():
    """Links with at least 2^16 pairs in the call take the binned scan inside
    the batch -- all of them together, one binning launch and one store launch
    per kind for each group of links -- keeping per-slot counters where they can
    (the rest the tile scan, with hot detection over their states).  Binned
    links that get fewer pairs in a slice are tile-scanned: their counters go
    stale, and the close after their next binned scan rebuilds them;
    counting is switched off and on.  Every link's list equals its separate
    detector's."""
    cfgs = tg.batch_configs(n_links=12, pairs_scale=0.5)
    traces = [tg.Trace(c) for c in cfgs]
    tabs = [tg.hash_tables(c.hash_seed) for c in cfgs]
    b = ssd.batch_init([_params(c) for c in cfgs], tabs, device="cuda:0")
    ssd.batch_set_tuning(b, ssd.SSD_TUNE_TIMING, 1)
    plain = [ssd.init_detector(_params(c), tabs[i], device="cuda:0") for i, c in enumerate(cfgs)]
    big = [i for i, c in enumerate(cfgs) if c.pairs_lo >= 1 << 16]
    assert len(big) >= 6, "too few links take the binned scan"
    assert ssd.batch_get_tuning(b, ssd.SSD_TUNE_COUNTED) == 1
    # slice: (binned links' pairs cut to 5000, counting knob) -> how the
    # counting links' R_k is taken at the close (1 counters, 2 counters
    # rebuilt from the state first, 0 the state read)
    plan = [(False, None, 1), (False, None, 1), (True, None, 0), (False, None, 2), (False, 0, 0), (False, 1, 2)]
    counting = None
    for t, (cut, knob, mode) in enumerate(plan):
        per = [tr.pairs(0, t % tr.cfg.n_slices) for tr in traces]
        if cut:
            per = [p[:5000] if i in big else p for i, p in enumerate(per)]
        offs = np.zeros(len(per) + 1, dtype=np.uint64)
        offs[1:] = np.cumsum([p.shape[0] for p in per])
        dev = to_dev(np.concatenate(per))
        if knob is not None:
            ssd.batch_set_tuning(b, ssd.SSD_TUNE_COUNTED, knob)
        ssd.batch_scan(b, dev, offs, t)
        lists, status = ssd.batch_close(b)
        assert np.all(status == 0)
        for i in range(len(cfgs)):
            ssd.scan_slice(plain[i], dev[int(offs[i]):int(offs[i + 1])], t)
            res = ssd.close_slice(plain[i])
            assert np.array_equal(lists[i], res), f"slice {t} link {i}: batch and separate detector differ"
        tm = ssd.batch_read_timing(b, reset=True)
        modes = [ssd.batch_get_info(b, i)["counted"] for i in range(len(cfgs))]
        log(f"batch binned slice {t}: {sum(len(x) for x in lists)} hosts, binned links {big}, detection modes "
            f"{modes}, count launches {tm['count_detect'][1]}, bin launches {tm['scan_bin'][1]}, "
            f"tile launches {tm['scan_tiles'][1]}")
        if counting is None:
            counting = [i for i, m in enumerate(modes) if m]
            assert counting and set(counting) <= set(big)
        assert [modes[i] for i in counting] == [mode] * len(counting), f"slice {t}: {modes}"
        assert all(modes[i] == 0 for i in range(len(cfgs)) if i not in counting)
        # one counted-detection launch for all counting links, plus one
        # rebuild launch per link rebuilt
        assert tm["count_detect"][1] == (0 if mode == 0 else 1 + (len(counting) if mode == 2 else 0))
        assert tm["hot_detect"][1] <= 1                        # the uncounted links' states, if any
        if cut:
            assert tm["scan_bin"][1] == 0 and tm["scan_tiles"][1] == 1
        else:
            assert 1 <= tm["scan_bin"][1] <= 3                 # one binning launch per group of links
    b.destroy()
    for d in plain:
        d.destroy()


def test_batch_overflow_is_per_link():
    """Links whose candidate capacity is exceeded report SSD_E_OVERFLOW and
    nothing else; every other link still matches its separate detector."""
    cfgs = tg.batch_configs(n_links=8, pairs_scale=0.02)
    traces = [tg.Trace(c) for c in cfgs]
    tabs = [tg.hash_tables(c.hash_seed) for c in cfgs]
    params = [_params(c) if i == 0 else _params(c, max_tuples=1) for i, c in enumerate(cfgs)]
    b = ssd.batch_init(params, tabs, device="cuda:0")
    ref = [ssd.init_detector(_params(c), tabs[i], device="cuda:0") for i, c in enumerate(cfgs)]
    overflowed = 0
    for t in range(6):
        per, offs, dev = _slice_pairs(traces, t)
        ssd.batch_scan(b, dev, offs, t)
        lists, status = ssd.batch_close(b)
        assert status[0] == 0
        for i in range(len(cfgs)):
            ssd.scan_slice(ref[i], dev[int(offs[i]):int(offs[i + 1])], t)
            res = ssd.close_slice(ref[i])
            if status[i] == 0:
                assert np.array_equal(lists[i], res), f"slice {t} link {i}"
            else:
                assert status[i] == -4 and len(lists[i]) == 0
                overflowed += 1
    assert overflowed > 0
    with pytest.raises(ssd.SSDError) as e:
        ssd.batch_scan(b, dev, offs, 99)
    assert e.value.status == -3


def test_batch_links_match_oracle():
    """Every link of a batch against the oracle, with the binned links at full
    size: two large links of the 64-link workload at full rate -- a 1.5 GiB
    (q=16, r=6, eta=4096) link and a 640 MiB (q=14, r=5, eta=8192) link,
    both scanned binned inside the batch with per-slot counters (the second
    through the five-row register binning) -- and six links at 2% of their
    rate (two of them binned with the large ones, four in the tile scan).
    Lists, R_k and hot lists of every link equal the oracle's at every
    slice, for k + 2 slices of the longest window."""
    full = tg.batch_configs(n_links=64)
    small = tg.batch_configs(n_links=64, pairs_scale=0.02)
    big_ids, small_ids = [17, 34], [9, 14, 20, 32, 44, 1]
    cfgs = [full[i] for i in big_ids] + [small[i] for i in small_ids]
    assert [c.r for c in cfgs[:2]] == [6, 5]
    assert all(c.r * (1 << c.q) * c.eta > 256 << 20 and c.pairs_lo >= 1 << 20 for c in cfgs[:2])
    traces = [tg.Trace(c) for c in cfgs]
    tabs = [tg.hash_tables(c.hash_seed) for c in cfgs]
    b = ssd.batch_init([_params(c) for c in cfgs], tabs, device="cuda:0")
    ssd.batch_set_tuning(b, ssd.SSD_TUNE_TIMING, 1)
    orcs = [oracle.RSEA(c.q, c.r, c.delta, c.eta, c.k, c.theta, tabs[i]) for i, c in enumerate(cfgs)]
    n_slices = max(c.k for c in cfgs) + 2
    total = 0
    for t in range(n_slices):
        per, offs, dev = _slice_pairs(traces, t)
        ssd.batch_scan(b, dev, offs, t)
        lists, status = ssd.batch_close(b)
        assert np.all(status == 0)
        for i, o in enumerate(orcs):
            o.scan(per[i])
            o.reconstruct()
            ip, rk, est = o.results()
            assert np.array_equal(lists[i]["ip"], ip) and np.array_equal(lists[i]["rk"], rk), \
                f"slice {t} link {i}: lists differ from the oracle"
            assert np.all(np.abs(lists[i]["est"] - est) <= 1e-6 * np.abs(est))
            assert np.array_equal(ssd.batch_read_rk(b, i), o.rk()), f"slice {t} link {i}: R_k differs"
            for row, (x, y) in enumerate(zip(ssd.batch_read_hot(b, i), o.hse())):
                assert np.array_equal(x, y), f"slice {t} link {i}: HSE({row}) differs"
            o.age()
            total += len(ip)
        tm = ssd.batch_read_timing(b, reset=True)
        log(f"batch vs oracle slice {t}: {sum(len(x) for x in lists)} hosts, bin launches {tm['scan_bin'][1]}, "
            f"count launches {tm['count_detect'][1]}")
        assert tm["scan_bin"][1] >= 1 and tm["count_detect"][1] >= 1
        assert ssd.batch_get_info(b, 0)["counted"] and ssd.batch_get_info(b, 1)["counted"]
    assert total > 0
    b.destroy()
