"""Served streams (continuous batching): every stream's list in every slot is
the same when the stream runs alone through its own detector and when it
runs in the mix, where its batches share group scans and its closes share
group closes with other streams -- also when a memory budget forces streams
to wait for admission."""
import numpy as np
import pytest

import oracle
import paper_1803_11036_amd as ssd
import tracegen as tg
from _parity import log, to_dev
from paper_1803_11036_amd import serve

pytestmark = pytest.mark.gpu


def _inputs(n_streams, n_slots, seed):
    ws = tg.served_workload(n_streams=n_streams, seed=seed, pairs_scale=0.004, n_slots=n_slots,
                            max_window_distinct=3e5)
    return serve.build_inputs(ws)


def _check_equal(inputs, rep):
    total = 0
    for i, s in enumerate(inputs):
        alone = serve.serve_alone(s)
        for o in range(s.n_slots):
            mixed = rep.results[(i, o)]
            assert mixed is not None, f"stream {i} slot {o} overflowed"
            assert np.array_equal(mixed, alone[o]), f"stream {i} slot {o}: mix differs from alone"
            total += len(mixed)
    return total


def _oracle_slots(s):
    """The oracle fed one served stream's batches slot by slot (scan every
    batch that arrived in the slot, then close): its list per slot."""
    p = s.params
    o = oracle.RSEA(p.q, p.r, p.delta, p.eta, p.k, p.theta, s.tables)
    slot_of = np.floor(s.arrivals / s.slot).astype(np.int64)
    out = []
    for t in range(s.n_slots):
        for j in np.nonzero(slot_of == t)[0]:
            o.scan(s.batch(int(j)).cpu().numpy().view(np.uint32))
        out.append(o.close())
    return out


def test_served_mix_equals_alone():
    """Every stream's list in every slot is the same alone and in the mix,
    and, for the streams with states up to 512 MiB, equal to the oracle's
    fed the same batches."""
    inputs = _inputs(8, 4, 0x5EED1)
    rep = serve.serve(inputs, budget_bytes=1 << 40, time_scale=4.0)
    log(f"served: {rep.pairs} pairs in {rep.wall_s:.2f} s, {rep.scan_calls} scans, {rep.close_calls} closes, "
        f"p50 {rep.latency(50):.2f} ms p99 {rep.latency(99):.2f} ms")
    assert rep.max_scan_members > 1          # batches of several streams shared scan launches
    assert _check_equal(inputs, rep) > 0
    checked = 0
    for i, s in enumerate(inputs):
        if serve.stream_bytes(s.params) > 512 << 20:
            continue
        for t, (ip, rk, est) in enumerate(_oracle_slots(s)):
            mixed = rep.results[(i, t)]
            assert np.array_equal(mixed["ip"], ip) and np.array_equal(mixed["rk"], rk), \
                f"stream {i} slot {t}: served list differs from the oracle"
            assert np.all(np.abs(mixed["est"] - est) <= 1e-6 * np.abs(est))
        checked += 1
    assert checked >= 2


def test_served_stream_dropped_mid_slot():
    """A stream dropped halfway through its second slot, after some of that
    slot's batches were scanned in shared group launches: its detector is
    freed without a close, its first slot's list is the one it has alone,
    and every other stream's lists are unchanged."""
    inputs = _inputs(6, 4, 0x5EED3)
    cand = [i for i, s in enumerate(inputs)
            if np.any((s.arrivals >= s.slot) & (s.arrivals < 1.5 * s.slot))]
    assert cand, "no stream has a batch in the first half of its second slot"
    d = cand[0]
    rep = serve.serve(inputs, budget_bytes=1 << 40, time_scale=1.0, drop={d: 1.5 * inputs[d].slot})
    alone = serve.serve_alone(inputs[d])
    got = sorted(o for (i, o) in rep.results if i == d)
    log(f"dropped stream {d}: slots closed {got}")
    assert set(got) <= {0}
    for o in got:
        assert np.array_equal(rep.results[(d, o)], alone[o])
    others = [s for i, s in enumerate(inputs) if i != d]
    sub = serve.ServeReport(wall_s=rep.wall_s, pairs=rep.pairs, latencies_ms=rep.latencies_ms,
                            results={(j, o): rep.results[(i, o)] for j, i in enumerate(k for k in range(len(inputs)) if k != d)
                                     for o in range(inputs[i].n_slots)},
                            max_admitted=rep.max_admitted, admit_wait_s=rep.admit_wait_s,
                            iterations=rep.iterations, scan_calls=rep.scan_calls, close_calls=rep.close_calls)
    assert _check_equal(others, sub) > 0


def test_served_admission_by_memory_budget():
    inputs = _inputs(6, 3, 0x5EED2)
    sizes = sorted(serve.stream_bytes(s.params) for s in inputs)
    budget = sum(sizes[-2:])                                        # about two streams at a time
    rep = serve.serve(inputs, budget_bytes=budget, time_scale=1.0)
    assert rep.max_admitted <= 3
    assert max(rep.admit_wait_s) > 0
    _check_equal(inputs, rep)


def test_group_binned_members_equal_separate_detectors():
    """Members with at least 2^18 pairs in the call are scanned binned inside
    the group scan, whatever their state's size (the rest share the tile scan);
    each member's list equals that of a detector of its own fed the same
    pairs, and the oracle's (lists, R_k and hot lists), slice by slice, also
    when only a subset of the members scans and closes."""
    cfgs = tg.batch_configs(n_links=12, pairs_scale=0.5)
    traces = [tg.Trace(c) for c in cfgs]
    tabs = [tg.hash_tables(c.hash_seed) for c in cfgs]

    def params(c):
        return ssd.make_params(q=c.q, r=c.r, delta=c.delta, eta=c.eta, k=c.k, theta=c.theta)

    members = [ssd.init_detector(params(c), tabs[i], device="cuda:0") for i, c in enumerate(cfgs)]
    alone = [ssd.init_detector(params(c), tabs[i], device="cuda:0") for i, c in enumerate(cfgs)]
    for d in members:
        ssd.set_tuning(d, ssd.SSD_TUNE_TIMING, 1)
    orcs = [oracle.RSEA(c.q, c.r, c.delta, c.eta, c.k, c.theta, tabs[i]) for i, c in enumerate(cfgs)]
    g = ssd.group_init(len(cfgs), device="cuda:0")
    big = [i for i, c in enumerate(cfgs) if c.pairs_lo >= 1 << 18]
    assert big, "no member takes the binned scan"
    clock = [0] * len(cfgs)           # open slice of member i and of its own detector
    for t in range(3):
        per = [tr.pairs(0, t % tr.cfg.n_slices) for tr in traces]
        offs = np.zeros(len(per) + 1, dtype=np.uint64)
        offs[1:] = np.cumsum([p.shape[0] for p in per])
        dev = to_dev(np.concatenate(per))
        # every member in the first slice; a subset (one binned, some tiled) after
        pick = list(range(len(cfgs))) if t == 0 else sorted({big[t % len(big)], 0, 1, 5})
        sub = np.concatenate([per[i] for i in pick])
        soffs = np.zeros(len(pick) + 1, dtype=np.uint64)
        soffs[1:] = np.cumsum([per[i].shape[0] for i in pick])
        sdev = to_dev(sub)
        ms = [members[i] for i in pick]
        ssd.group_scan(g, ms, sdev, soffs, [clock[i] for i in pick])
        lists, status = ssd.group_close(g, ms)
        assert np.all(status == 0)
        for j, i in enumerate(pick):
            ssd.scan_slice(alone[i], dev[int(offs[i]):int(offs[i + 1])], clock[i])
            res = ssd.close_slice(alone[i])
            clock[i] += 1
            assert np.array_equal(lists[j], res), f"slice {t} member {i}: group and own detector differ"
            o = orcs[i]
            o.scan(per[i])
            o.reconstruct()
            ip, rk, est = o.results()
            assert np.array_equal(lists[j]["ip"], ip) and np.array_equal(lists[j]["rk"], rk), \
                f"slice {t} member {i}: group and oracle differ"
            assert np.all(np.abs(lists[j]["est"] - est) <= 1e-6 * np.abs(est))
            assert np.array_equal(ssd.read_rk(members[i]), o.rk()), f"slice {t} member {i}: R_k differs"
            for row, (x, y) in enumerate(zip(ssd.read_hot(members[i]), o.hse())):
                assert np.array_equal(x, y), f"slice {t} member {i}: HSE({row}) differs"
            o.age()
        log(f"group binned slice {t}: members {pick}, {sum(len(x) for x in lists)} hosts, binned {big}")
    assert sum(ssd.read_timing(members[i])["scan_bin"][1] for i in big) >= len(big) + 2
    g.destroy()
    for d in members + alone:
        d.destroy()


def _member_slices(seed, key_bits, n_slices, n_pairs, distinct, heavy=10, heavy_peers=600):
    """Slices of n_pairs drawn with repeats from a pool of distinct pairs: a
    light background over 20000 hosts plus heavy hosts present every slice."""
    rng = np.random.default_rng(seed)
    hosts = rng.integers(0, 2 ** key_bits, 20000, dtype=np.uint64)
    hv = rng.integers(0, 2 ** key_bits, heavy, dtype=np.uint64)
    out = []
    for _ in range(n_slices):
        bg = np.stack([rng.choice(hosts, distinct), rng.integers(0, 2 ** 32, distinct, dtype=np.uint64)], 1)
        hp = np.stack([np.repeat(hv, heavy_peers), rng.integers(0, 2 ** 32, heavy * heavy_peers, dtype=np.uint64)], 1)
        pool = np.concatenate([bg, hp]).astype(np.uint32)
        out.append(pool[rng.integers(0, pool.shape[0], n_pairs)])
    return out


def test_group_binned_members_in_rounds():
    """Group scans whose binned members' calls exceed their staging: every
    round bins all of them in one launch and stores them in one launch per
    store kind.  Six rows (3.5M pairs into a 24 MiB state: several rounds),
    five rows (6M pairs into 80 MiB: two rounds), four rows (the general
    binning, 2.5M pairs into 16 MiB: several rounds) -- all three with the
    counted stores of two workgroups per compute unit --, a member whose
    counters need more LDS (k = 100), one that cannot count (k = 150 > eta / 8:
    uncounted stores), and two members with calls below 2^18 pairs (in the
    tile scan, one of them set to bin its own calls); each member's list,
    R_k, hot lists and state against a detector of its own and the oracle,
    slice by slice."""
    # (q, r, delta, key_bits, k, scan mode, pairs per call, distinct pairs per slice)
    spec = [(12, 6, 5, 32, 3, ssd.SSD_SCAN_BINNED, 3_500_000, 100_000),
            (14, 5, 6, 32, 3, ssd.SSD_SCAN_BINNED, 6_000_000, 100_000),
            (12, 4, 10, 32, 3, ssd.SSD_SCAN_BINNED, 2_500_000, 100_000),
            (12, 6, 5, 32, 100, ssd.SSD_SCAN_BINNED, 2_500_000, 100_000),
            (12, 6, 5, 32, 150, ssd.SSD_SCAN_BINNED, 2_000_000, 100_000),
            (12, 6, 5, 32, 3, ssd.SSD_SCAN_BINNED, 200_000, 60_000),
            (10, 6, 5, 30, 3, ssd.SSD_SCAN_AUTO, 200_000, 30_000)]
    n_binned = 5
    eta, theta, n_slices = 1024, 300, 4
    slices = [_member_slices(900 + i, x[3], n_slices, x[6], x[7]) for i, x in enumerate(spec)]
    tabs = [tg.hash_tables(60 + i) for i in range(len(spec))]

    def det(i):
        q, r, delta, kb, k, mode, _, _ = spec[i]
        d = ssd.init_detector(ssd.make_params(q=q, r=r, delta=delta, eta=eta, k=k, theta=theta, key_bits=kb),
                              tabs[i], device="cuda:0")
        ssd.set_tuning(d, ssd.SSD_TUNE_SCAN_MODE, mode)
        return d

    members = [det(i) for i in range(len(spec))]
    alone = [det(i) for i in range(len(spec))]
    for d in members:
        ssd.set_tuning(d, ssd.SSD_TUNE_TIMING, 1)
    orcs = [oracle.RSEA(q, r, delta, eta, k, theta, tabs[i], key_bits=kb)
            for i, (q, r, delta, kb, k, _, _, _) in enumerate(spec)]
    g = ssd.group_init(len(spec), device="cuda:0")
    for t in range(n_slices):
        per = [sl[t] for sl in slices]
        offs = np.zeros(len(per) + 1, dtype=np.uint64)
        offs[1:] = np.cumsum([p.shape[0] for p in per])
        dev = to_dev(np.concatenate(per))
        log(f"group rounds slice {t}: {offs[-1]} pairs")
        ssd.group_scan(g, members, dev, offs, [t] * len(spec))
        for i in range(len(spec)):
            orcs[i].scan(per[i])
        for i in range(n_binned):      # the binned members' window state, before the close
            got = ssd.read_canonical_state(members[i]).cpu().numpy().view(np.uint16)
            assert np.array_equal(got.reshape(orcs[i].r, -1, eta), orcs[i].canonical()), \
                f"slice {t} member {i}: state differs"
        lists, status = ssd.group_close(g, members)
        assert np.all(status == 0)
        for i in range(len(spec)):
            ssd.scan_slice(alone[i], dev[int(offs[i]):int(offs[i + 1])], t)
            res = ssd.close_slice(alone[i])
            assert np.array_equal(lists[i], res), f"slice {t} member {i}: group and own detector differ"
            o = orcs[i]
            o.reconstruct()
            ip, rk, est = o.results()
            assert np.array_equal(lists[i]["ip"], ip) and np.array_equal(lists[i]["rk"], rk), \
                f"slice {t} member {i}: group and oracle differ"
            assert np.all(np.abs(lists[i]["est"] - est) <= 1e-6 * np.abs(est))
            assert np.array_equal(ssd.read_rk(members[i]), o.rk()), f"slice {t} member {i}: R_k differs"
            for row, (x, y) in enumerate(zip(ssd.read_hot(members[i]), o.hse())):
                assert np.array_equal(x, y), f"slice {t} member {i}: HSE({row}) differs"
            o.age()
        assert sum(len(x) for x in lists) >= 10 * len(spec)
    tm = [ssd.read_timing(d)["scan_bin"][1] for d in members]
    kib = [ssd.get_info(d)["counted_bin_kib"] for d in members]
    log(f"binning launches per member: {tm}; counted bins (KiB): {kib}")
    assert tm[0] >= 2 * n_slices and tm[2] >= 2 * n_slices, "the large calls took a single round"
    assert all(x >= n_slices for x in tm[:n_binned]) and tm[n_binned:] == [0, 0]
    # counted stores for the members that keep counters, uncounted for the one that cannot
    assert all(x > 0 for x in kib[:4]) and kib[4] == 0
    g.destroy()
    for d in members + alone:
        d.destroy()


def test_group_refuses_16bit_members():
    """Groups take 8-bit members only: a detector with 16-bit cells (windows
    above 254 slots) in a group call is refused before any work."""
    p8 = ssd.make_params(q=8, r=4, delta=4, eta=1024, k=3, theta=200, key_bits=16)
    p16 = ssd.make_params(q=8, r=4, delta=4, eta=1024, k=300, theta=200, key_bits=16, cell_bits=16)
    tabs = tg.hash_tables(5)
    d8, d16 = ssd.init_detector(p8, tabs, device="cuda:0"), ssd.init_detector(p16, tabs, device="cuda:0")
    g = ssd.group_init(2, device="cuda:0")
    pairs = to_dev(np.arange(20, dtype=np.uint32).reshape(10, 2))
    with pytest.raises(ssd.SSDError) as e:
        ssd.group_scan(g, [d8, d16], pairs, [0, 5, 10], [0, 0])
    assert e.value.status == -1
    with pytest.raises(ssd.SSDError) as e:
        ssd.group_close(g, [d16])
    assert e.value.status == -1
    ssd.group_scan(g, [d8], pairs, [0, 10], [0])
    lists, status = ssd.group_close(g, [d8])
    assert status[0] == 0
    g.destroy()
    d8.destroy()
    d16.destroy()


def test_group_close_begin_end():
    """The group close in two halves: while it is pending the members' next
    slot can be scanned (group scans), but a member cannot close, merge or be
    inspected and the group cannot begin another close (SSD_E_ORDER); the
    collected lists equal those of detectors of their own, slot after slot."""
    cfgs = tg.batch_configs(n_links=4, pairs_scale=0.05)
    traces = [tg.Trace(c) for c in cfgs]
    tabs = [tg.hash_tables(c.hash_seed) for c in cfgs]

    def params(c):
        return ssd.make_params(q=c.q, r=c.r, delta=c.delta, eta=c.eta, k=c.k, theta=c.theta)

    members = [ssd.init_detector(params(c), tabs[i], device="cuda:0") for i, c in enumerate(cfgs)]
    alone = [ssd.init_detector(params(c), tabs[i], device="cuda:0") for i, c in enumerate(cfgs)]
    g = ssd.group_init(len(cfgs), device="cuda:0")

    def slot(t):
        per = [tr.pairs(0, t % tr.cfg.n_slices) for tr in traces]
        offs = np.zeros(len(per) + 1, dtype=np.uint64)
        offs[1:] = np.cumsum([p.shape[0] for p in per])
        return per, offs, to_dev(np.concatenate(per))

    per, offs, dev = slot(0)
    ssd.group_scan(g, members, dev, offs, [0] * len(cfgs))
    for t in range(1, 6):
        ssd.group_close_begin(g, members)
        for call in (lambda: ssd.group_close_begin(g, members), lambda: ssd.close_slice(members[0]),
                     lambda: ssd.close_begin(members[1]), lambda: ssd.read_rk(members[2]),
                     lambda: ssd.merge_router_state(members[3], [members[0]])):
            with pytest.raises(ssd.SSDError) as e:
                call()
            assert e.value.status == -3
        nper, noffs, ndev = slot(t)
        ssd.group_scan(g, members, ndev, noffs, [t] * len(cfgs))     # slot t while the close of t-1 is pending
        lists, status = ssd.group_close_end(g)
        assert np.all(status == 0)
        for i, d in enumerate(alone):
            ssd.scan_slice(d, dev[int(offs[i]):int(offs[i + 1])], t - 1)
            assert np.array_equal(lists[i], ssd.close_slice(d)), f"slot {t - 1} member {i}"
            assert np.array_equal(ssd.get_results(members[i]), lists[i])
        per, offs, dev = nper, noffs, ndev
        log(f"group begin/end slot {t - 1}: {sum(len(x) for x in lists)} hosts")
    with pytest.raises(ssd.SSDError) as e:
        ssd.group_close_end(g)
    assert e.value.status == -3
    g.destroy()
    for d in members + alone:
        d.destroy()
