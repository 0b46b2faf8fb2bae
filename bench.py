#!/usr/bin/env python3
"""Benchmark of the sliding super point detector's hot path on one MI355X.

A step is one pass of the whole hot path over one slice of synthetic input:
the scan of the slice's pairs (Alg. 2), then the slice close -- hot
detection, candidate expansion, final test, sort and report (Sec. 4.2) --
with the lists back in host memory.  Inputs are resident in HBM before the
timed region.

Default workload (the metric's own comparison): the batched form -- 64
independent monitored links of uneven rates (0.2M-8M pairs per slice), windows
(k 4..64) and thresholds (512..8192), about 152M pairs per slice over 19 GiB of
state -- timed as plain per-link launches (one detector per link, scan and
close per link in sequence on one stream) and as one batch (one persistent
scan launch, one graph-replayed close), on the same pairs, with the lists
checked identical for every timed slice.  `value` is the batched rate.

Prints one JSON line: pairs (packets) per second, Gb/s at an 800-byte mean
packet (also in the paper's /1024 convention), slice-close latency p50/p99,
per-phase device times from HIP events on the engine's stream, the roofline
of the dominant kernel (algorithmic bytes per launch over its event time,
against 8 TB/s), the end-to-end rate with the pairs copied from pinned host
memory, the CPU oracle's rate on a bounded sample (one thread and all host
cores), the single core link as a secondary workload and the measured memory
ceilings.  Other workloads: --workload core_link | distributed | served |
ceilings.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import ctypes as C
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
MEAN_PACKET_BYTES = 800        # the paper's assumed mean packet size (Sec. 5)
METRIC = "packets/s (and Gb/s @800B) scan + slice-close latency p50/p99, batched vs plain"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def gbps(pps: float) -> dict:
    """Gb/s at 800-byte packets: decimal, and the paper's convention
    (M pairs/s x 800 x 8 / 1024, Sec. 5)."""
    return {"gbps_at_800B": round(pps * MEAN_PACKET_BYTES * 8 / 1e9, 2),
            "gbps_at_800B_paper_convention": round(pps / 1e6 * MEAN_PACKET_BYTES * 8 / 1024, 2)}


def host_info() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_threads() -> int:
    # the GPU machine gives one GPU's process a share of 16 host cores
    return max(1, min(16, len(os.sched_getaffinity(0))))


def kernel_source_sha() -> str:
    """Hash of the kernel sources' code: comments and blank lines are left
    out, so that a comment edit does not void traffic measured on the same
    kernels."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_1803_11036_amd", "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, if they
    were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != kernel_source_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline(cands: dict, workload: str) -> dict:
    """The roofline of the kernel with the most device time per step among
    those that move algorithmic bytes (the close's chain of small launches,
    which moves none, is listed with the others).
    cands: name -> (device ms per step, algorithmic bytes per launch, ms per
    launch, launches per step, implementation bytes per launch or None)."""
    dom = max((k for k in cands if cands[k][1] > 0), key=lambda k: cands[k][0])
    _, alg, ms, per_step, impl = cands[dom]
    achieved = alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    traffic = load_traffic(dom, workload)
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
            "algorithmic_bytes_per_launch": round(alg), "ms_per_launch": round(ms, 5),
            "launches_per_step": per_step,
            "implementation_bytes_per_launch": round(impl) if impl else None,
            "traffic_gbs": round(traffic / (ms * 1e-3) / 1e9, 1) if traffic and ms > 0 else None,
            "others": {k: {"ms_per_step": round(v[0], 4), "ms_per_launch": round(v[2], 5),
                           "achieved_gbs": round(v[1] / (v[2] * 1e-3) / 1e9, 1) if v[2] > 0 else None}
                       for k, v in cands.items() if k != dom}}


def calibration_copy(dev, mib: int) -> None:
    """One plain device copy of known size: the reference against which the
    HBM counters of a profiled run are scaled."""
    import torch
    a = torch.empty(mib << 20, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


# ----------------------------------------------------------------------------
# memory ceilings (probes in the library)

def _probe_lib():
    import paper_1803_11036_amd as ssd
    L = C.CDLL(ssd.library_path())
    L.ssd_probe_stream_read.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]
    L.ssd_probe_stream_read.restype = C.c_int
    L.ssd_probe_scatter.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, C.c_void_p]
    L.ssd_probe_scatter.restype = C.c_int
    L.ssd_probe_rmw16.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint64, C.c_void_p]
    L.ssd_probe_rmw16.restype = C.c_int
    return L


RMW_BIN_BYTES, RMW_OPS_PER_BIN = 512 << 10, 2048


def ceilings(dev, sizes_mib, stores: int = 1 << 28, reps: int = 3) -> dict:
    """Stream read (GB/s), random byte scatter (G stores/s, uniform and
    XCD-local) and random 16-byte read-modify-writes in 512 KiB bins (G
    chunks/s, 2048 per bin: about the density of the counted stores' visit)
    at each working-set size, timed with events on the stream the probes run
    on (torch's current stream)."""
    import torch
    L = _probe_lib()
    s = torch.cuda.current_stream(dev)
    out = {}
    sink = torch.empty(4096, dtype=torch.uint8, device=dev)
    for mib in sizes_mib:
        nbytes = mib << 20
        buf = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        res = {}
        for name, fn in (("stream_read_gbs", lambda: L.ssd_probe_stream_read(buf.data_ptr(), nbytes, sink.data_ptr(),
                                                                             s.cuda_stream)),
                         ("scatter_uniform_gstores", lambda: L.ssd_probe_scatter(buf.data_ptr(), nbytes, stores, 7, 0,
                                                                                 s.cuda_stream)),
                         ("scatter_xcd_local_gstores", lambda: L.ssd_probe_scatter(buf.data_ptr(), nbytes, stores, 7,
                                                                                   1, s.cuda_stream)),
                         ("rmw16_bins_gchunks", lambda: L.ssd_probe_rmw16(buf.data_ptr(), nbytes, RMW_BIN_BYTES,
                                                                         RMW_OPS_PER_BIN, 7, s.cuda_stream))):
            if name == "scatter_xcd_local_gstores" and (nbytes < (16 << 20) or nbytes % (2 << 20)):
                continue
            if fn() != 0:
                raise RuntimeError(f"probe {name} failed")
            best = None
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(s)
                if fn() != 0:
                    raise RuntimeError(f"probe {name} failed")
                b.record(s)
                b.synchronize()
                ms = a.elapsed_time(b)
                best = ms if best is None else min(best, ms)
            work = {"stream_read_gbs": nbytes, "rmw16_bins_gchunks": nbytes // RMW_BIN_BYTES * RMW_OPS_PER_BIN}
            res[name] = round(work.get(name, stores) / 1e9 / (best * 1e-3), 2)
        out[f"{mib}MiB"] = res
        del buf
    torch.cuda.empty_cache()
    return out


# ----------------------------------------------------------------------------
# CPU oracle baselines

def _oracle_link_sample(cfgs, max_state=256 << 20, max_window_pairs=16_000_000, max_links=12):
    """The batched links the CPU sample takes: states up to max_state bytes
    and windows of at most max_window_pairs pairs, in link order."""
    pick = [i for i, c in enumerate(cfgs)
            if c.r * (1 << c.q) * c.eta <= max_state and c.k * c.pairs_lo <= max_window_pairs]
    return pick[:max_links]


def cpu_baseline_batched(cfgs, traces, tables) -> dict:
    """The oracle as it stands on a sample of the batched links with full
    windows: each sampled link's first k slices are scanned and aged untimed
    (its window fills), then one slice per link is timed (scan + full close)
    on one host thread, link after link, and the next slice on all host
    cores at once, one link per thread (the oracle's calls release the GIL)."""
    import oracle
    pick = _oracle_link_sample(cfgs)
    threads = min(cpu_threads(), len(pick))
    orcs = {i: oracle.RSEA(cfgs[i].q, cfgs[i].r, cfgs[i].delta, cfgs[i].eta, cfgs[i].k, cfgs[i].theta, tables[i])
            for i in pick}

    def fill(i):
        for t in range(cfgs[i].k):
            orcs[i].scan(traces[i].pairs(0, t))
            orcs[i].close(advance_only=True)
        return i

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(fill, pick))
    fill_s = time.perf_counter() - t0
    # one thread: slice k of every sampled link, one after another
    sl = {i: traces[i].pairs(0, cfgs[i].k % cfgs[i].n_slices) for i in pick}
    n1 = sum(p.shape[0] for p in sl.values())
    t0 = time.perf_counter()
    for i in pick:
        orcs[i].scan(sl[i])
        orcs[i].close()
    one_s = time.perf_counter() - t0
    # all cores: slice k+1 of every sampled link, one link per thread
    sl = {i: traces[i].pairs(0, (cfgs[i].k + 1) % cfgs[i].n_slices) for i in pick}
    nn = sum(p.shape[0] for p in sl.values())

    def step(i):
        orcs[i].scan(sl[i])
        orcs[i].close()

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(step, pick))
    all_s = time.perf_counter() - t0
    del orcs
    sample = (f"{len(pick)} of the {len(cfgs)} batched links (those with at most 256 MiB of state and 16M pairs "
              f"per window, in link order: {pick}); each link's window filled untimed ({fill_s:.1f} s), then one "
              f"slice per link timed, scan + full close with a full window: {n1} pairs in {one_s:.2f} s on one "
              f"thread, the next {nn} pairs in {all_s:.2f} s on {threads} threads (one link per thread)")
    return {"value": round(nn / all_s, 1), "unit": "packets/s", "cores": threads, "kind": "oracle",
            "sample": sample, "single_thread": {"value": round(n1 / one_s, 1), "cores": 1},
            "host": host_info()}


def cpu_baseline_link(cfg, trace, tables, n_slices: int, fill_s: float = 30.0, timed_s: float = 10.0) -> dict:
    """The oracle as it stands, one thread, on a single-link workload: the
    window filled first, untimed (k - 1 slices, or as many as fill_s seconds
    allow), then scan + full close of each following slice timed, until
    timed_s seconds or n_slices slices (at least one)."""
    import oracle
    o = oracle.RSEA(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tables)
    t = 0
    f0 = time.perf_counter()
    while t < cfg.k - 1 and time.perf_counter() - f0 < fill_s:
        o.scan(trace.pairs(0, t % cfg.n_slices))
        o.close()
        t += 1
    filled = t
    n, dt, timed = 0, 0.0, 0
    while timed < max(1, n_slices) and (timed == 0 or dt < timed_s):
        p = trace.pairs(0, t % cfg.n_slices)
        t0 = time.perf_counter()
        o.scan(p)
        o.close()
        dt += time.perf_counter() - t0
        n += p.shape[0]
        timed += 1
        t += 1
    del o
    window = "full window" if filled >= cfg.k - 1 else f"window filled to {filled + 1} of {cfg.k} slices"
    return {"value": round(n / dt, 1), "unit": "packets/s", "cores": 1, "kind": "oracle",
            "sample": f"{filled} slices filled untimed, then {timed} slices timed ({n} pairs, {window}), "
                      f"scan + full close each, {dt:.1f} s on one host thread", "host": host_info()}


def cpu_baseline_distributed(cfg, trace, tables, n_slices: int, n_routers: int = 4, fill_s: float = 30.0,
                             timed_s: float = 10.0) -> dict:
    """The oracle as it stands, one thread, on the distributed workload cut to
    its first n_routers routers (the merge's work per pair does not depend
    on the router count): per slice every router scans its pairs, the routers
    are merged into the global detector (Alg. 5), which closes, and the
    routers advance.  The window is filled untimed first, as for one link."""
    import oracle
    mk = lambda: oracle.RSEA(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tables)
    routers = [mk() for _ in range(n_routers)]
    glob = mk()

    def step(t):
        per = trace.pairs_all(t % cfg.n_slices)[:n_routers]
        t0 = time.perf_counter()
        for o, p in zip(routers, per):
            o.scan(p)
        glob.merge_from(routers)
        glob.close()
        for o in routers:
            o.close(advance_only=True)
        return time.perf_counter() - t0, sum(int(p.shape[0]) for p in per)

    t = 0
    f0 = time.perf_counter()
    while t < cfg.k - 1 and time.perf_counter() - f0 < fill_s:
        step(t)
        t += 1
    filled = t
    n, dt, timed = 0, 0.0, 0
    while timed < max(1, n_slices) and (timed == 0 or dt < timed_s):
        d, m = step(t)
        dt += d
        n += m
        timed += 1
        t += 1
    del routers, glob
    window = "full window" if filled >= cfg.k - 1 else f"window filled to {filled + 1} of {cfg.k} slices"
    return {"value": round(n / dt, 1), "unit": "packets/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_routers} of the {cfg.n_streams} routers; {filled} slices filled untimed, then {timed} "
                      f"slices timed ({n} pairs, {window}): router scans, merge, global close and router advances, "
                      f"{dt:.1f} s on one host thread", "host": host_info()}


# ----------------------------------------------------------------------------
# batched (default)

def run_batched(args) -> dict:
    """64 links of uneven rates, windows and thresholds: plain per-link
    detectors (scan + close per link, in sequence on one stream) against the
    batch (one persistent scan, one graph-replayed close), on the same pairs,
    with identical outputs checked for every timed slice."""
    import torch
    import paper_1803_11036_amd as ssd
    import tracegen as tg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ceil = None
    if not args.no_ceilings:
        log("ceilings: stream read and byte scatter at the core-link state size")
        ceil = ceilings(dev, [1536])
    cfgs = tg.batch_configs(n_links=args.links)
    log(f"batched: {len(cfgs)} links, building traces")
    traces = [tg.Trace(c) for c in cfgs]
    tables = [tg.hash_tables(c.hash_seed) for c in cfgs]
    n_var = args.variants
    slices = []
    for v in range(n_var):
        parts = [tr.pairs_device(0, v, dev) for tr in traces]
        offs = np.zeros(len(parts) + 1, dtype=np.uint64)
        offs[1:] = np.cumsum([int(x.shape[0]) for x in parts])
        slices.append((torch.cat(parts).contiguous(), offs))
        del parts
        log(f"slice variant {v}: {int(offs[-1])} pairs")
    torch.cuda.synchronize()

    def params(c):
        return ssd.make_params(q=c.q, r=c.r, delta=c.delta, eta=c.eta, k=c.k, theta=c.theta,
                               max_tuples=1 << 21, max_results=1 << 18)

    W, K = args.warmup, args.steps
    # plain: one detector per link
    plain = [ssd.init_detector(params(c), tables[i], device=dev) for i, c in enumerate(cfgs)]
    plain_lists, plain_close = [], []
    t = 0
    for i in range(W + K):
        pairs, offs = slices[i % n_var]
        if i == W:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        lists = []
        close_ms = 0.0
        for l, d in enumerate(plain):
            ssd.scan_slice(d, pairs[int(offs[l]):int(offs[l + 1])], t)
            c0 = time.perf_counter()
            lists.append(ssd.close_slice(d))
            close_ms += (time.perf_counter() - c0) * 1e3
        if i >= W:
            plain_lists.append(lists)
            plain_close.append(close_ms)
        t += 1
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    for d in plain:
        d.destroy()
    del plain
    torch.cuda.empty_cache()

    # batched: persistent scan + graph close; the autotuner times its
    # candidates on untimed scans first
    b = ssd.batch_init([params(c) for c in cfgs], tables, device=dev)
    if args.counted_min_items is not None:
        ssd.batch_set_tuning(b, ssd.SSD_TUNE_COUNTED_MIN_ITEMS, args.counted_min_items)
    t = 0
    if args.autotune:
        ssd.batch_set_tuning(b, ssd.SSD_TUNE_AUTOTUNE, 1)
        while ssd.batch_get_tuning(b, ssd.SSD_TUNE_AUTOTUNE):
            pairs, offs = slices[t % n_var]
            ssd.batch_scan(b, pairs, offs, t)
            ssd.batch_close(b)
            t += 1
        log(f"autotuned over {t} slices")
    ssd.batch_set_tuning(b, ssd.SSD_TUNE_TIMING, 1)
    for i in range(W):
        pairs, offs = slices[i % n_var]
        ssd.batch_scan(b, pairs, offs, t)
        ssd.batch_close(b)
        t += 1
    torch.cuda.synchronize()
    ssd.batch_read_timing(b, reset=True)
    batch_lists = []
    t0 = time.perf_counter()
    # pipelined: slice t+1's scan is enqueued before slice t's lists are
    # collected (ssd_batch_close_begin / _end), as for the single link
    for i in range(K):
        pairs, offs = slices[(W + i) % n_var]
        ssd.batch_scan(b, pairs, offs, t)
        if i > 0:
            batch_lists.append(ssd.batch_close_end(b))
        ssd.batch_close_begin(b)
        t += 1
    batch_lists.append(ssd.batch_close_end(b))
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t0
    timing = ssd.batch_read_timing(b, reset=True)
    # slice-close latency: scan drained first, then close call to lists in host memory
    lat = []
    for i in range(args.latency_steps):
        pairs, offs = slices[i % n_var]
        ssd.batch_scan(b, pairs, offs, t)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        ssd.batch_close(b)
        lat.append((time.perf_counter() - c0) * 1e3)
        t += 1
    same = True
    for (lists, status), ref in zip(batch_lists, plain_lists):
        same &= all(np.array_equal(x, y) for x, y in zip(lists, ref)) and not status.any()
    tuned = (ssd.batch_get_tuning(b, ssd.SSD_TUNE_SCAN_PASS_BYTES), ssd.batch_get_tuning(b, ssd.SSD_TUNE_SCAN_TILE_PAIRS))
    link_info = [ssd.batch_get_info(b, l) for l in range(len(cfgs))]

    # end to end: every step's pairs copied from pinned host memory on a copy
    # stream, the next slice's copy overlapping this slice's scan and close
    e2e = None
    if args.e2e_steps:
        host = [p.cpu().pin_memory() for p, _ in slices]
        bufs = [torch.empty_like(slices[0][0]) for _ in range(2)]
        cs = torch.cuda.Stream(dev)
        ev = [torch.cuda.Event() for _ in range(2)]
        cur = torch.cuda.current_stream(dev)

        def copy(j):
            with torch.cuda.stream(cs):
                bufs[j % 2].copy_(host[j % n_var], non_blocking=True)
                ev[j % 2].record(cs)

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        copy(0)
        n_e2e = 0
        for j in range(args.e2e_steps):
            if j + 1 < args.e2e_steps:
                copy(j + 1)             # buffer (j+1)%2 was last read by step j-1, whose close has returned
            cur.wait_event(ev[j % 2])
            offs = slices[j % n_var][1]
            ssd.batch_scan(b, bufs[j % 2], offs, t)
            ssd.batch_close(b)
            n_e2e += int(offs[-1])
            t += 1
        torch.cuda.synchronize()
        e2e_s = time.perf_counter() - t0
        e2e = {"packets_per_s": round(n_e2e / e2e_s, 1), **gbps(n_e2e / e2e_s),
               "ms_per_step": round(e2e_s * 1e3 / args.e2e_steps, 3), "steps": args.e2e_steps,
               "note": "pairs copied host->device from pinned memory each step (copy of the next slice "
                       "overlapping this slice's scan and close); bound by the host link"}
        del host, bufs
    state_bytes = b.state.numel()
    b.destroy()
    del b
    torch.cuda.empty_cache()
    if args.calibrate_copy_mib:
        calibration_copy(dev, args.calibrate_copy_mib)

    total_pairs = sum(int(slices[i % n_var][1][-1]) for i in range(W, W + K))
    pps_b, pps_p = total_pairs / batch_s, total_pairs / plain_s

    # roofline of the dominant kernel.  Algorithmic bytes (scan: 8 + r per
    # pair, the pair read and one recorder written per row; hot detection:
    # the whole state of every link it reads once per close)
    per_slice = np.diff(slices[0][1]).astype(np.int64)
    binned = [l for l in range(len(cfgs)) if per_slice[l] >= (1 << 16)]      # the library's batch rule
    tile_links = [l for l in range(len(cfgs)) if l not in binned]
    tile_alg = float(sum((8 + cfgs[l].r) * per_slice[l] for l in tile_links))
    bin_alg = float(sum((8 + cfgs[l].r) * per_slice[l] for l in binned))
    counted_links = [l for l in range(len(cfgs)) if link_info[l]["counted"]]
    cands = {}
    if timing["scan_tiles"][1]:
        ms = timing["scan_tiles"][0]
        cands["k_scan_tiles"] = (ms / K, tile_alg, ms / timing["scan_tiles"][1], timing["scan_tiles"][1] // K, None)
    if timing["scan"][1]:
        # k_apply_counted_multi / k_apply_multi: the binned links' stores,
        # one launch per group of links and kind
        ms, n_l = timing["scan"]
        per = max(1, n_l // K)
        impl = float(sum((6 if l in counted_links else 5) * cfgs[l].r * per_slice[l] for l in binned))
        n_cnt = sum(1 for l in binned if l in counted_links)
        stores = "k_apply_counted_multi" if n_cnt == len(binned) else "k_apply_multi" if n_cnt == 0 else "binned_stores"
        cands[stores] = (ms / K, bin_alg / per, ms / n_l, per, impl / per)
    if timing["scan_bin"][1]:
        ms, n_l = timing["scan_bin"]
        per = max(1, n_l // K)
        impl = float(sum((8 + 4 * cfgs[l].r) * per_slice[l] for l in binned))
        cands["k_bin_multi_rows"] = (ms / K, 8.0 * sum(per_slice[l] for l in binned) / per, ms / n_l, per, impl / per)
    if timing["hot_detect"][1]:
        ms = timing["hot_detect"][0]
        read = float(sum(c.r * (1 << c.q) * c.eta for l, c in enumerate(cfgs) if l not in counted_links))
        cands["k_hot_detect"] = (ms / K, read, ms / timing["hot_detect"][1], timing["hot_detect"][1] // K, None)
    if timing["count_detect"][1]:
        ms, n_l = timing["count_detect"]
        per = max(1, n_l // K)
        # per estimator: the live-cell total and the next slice's slot read,
        # both and R_k written (20 bytes)
        cnt = float(sum((cfgs[l].r << cfgs[l].q) * 20 for l in counted_links))
        cands["k_count_multi"] = (ms / K, cnt / per, ms / n_l, per, cnt / per)
    if timing["close_graph"][1]:
        ms = timing["close_graph"][0]
        cands["close_graph"] = (ms / K, 0.0, ms / timing["close_graph"][1], timing["close_graph"][1] // K, None)
    roof = roofline(cands, "batched")

    out = {
        "metric": METRIC,
        "value": round(pps_b, 1), "unit": "packets/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(batch_s * 1e3 / K, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"batched: {len(cfgs)} links, {total_pairs // K} pairs/slice in total, "
                               f"k 4..64, theta 512..8192, 2^12..2^16 x r estimators, {state_bytes >> 20} MiB of state",
                   "form": "batched", "links": len(cfgs), "pairs_per_slice": total_pairs // K,
                   "state_bytes": state_bytes, "slice_variants": n_var},
        **gbps(pps_b),
        "plain_packets_per_s": round(pps_p, 1),
        "batched_over_plain": round(pps_b / pps_p, 3),
        "identical_outputs": bool(same),
        "close_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                             "p99": round(float(np.percentile(lat, 99)), 4)} if lat else None,
        "plain_close_latency_ms": {"p50": round(float(np.percentile(plain_close, 50)), 4),
                                   "p99": round(float(np.percentile(plain_close, 99)), 4),
                                   "note": "sum of the 64 per-link close calls of a slice"},
        "kernels": {k: {"ms_total": round(v[0], 4), "launches": v[1]} for k, v in timing.items() if v[1]},
        "autotuned": {"pass_bytes": tuned[0], "tile_pairs": tuned[1],
                      "counted_bin_kib_links": {str(v): sum(1 for x in link_info if x["counted_bin_kib"] == v)
                                                for v in sorted({x["counted_bin_kib"] for x in link_info})}},
        "links_binned": len(binned), "links_counted": len(counted_links),
        "roofline": roof,
        "end_to_end": e2e,
        "ceilings": ceil,
    }
    if not args.no_secondary:
        log("secondary: the single core link")
        out["core_link"] = run_core(args, secondary=True)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a sample of the batched links")
        out["cpu_baseline"] = cpu_baseline_batched(cfgs, traces, tables)
    else:
        out["cpu_baseline"] = None
    return out


# ----------------------------------------------------------------------------
# single link (core link, or the tiny or paper-shaped workload)

def run_core(args, secondary: bool = False) -> dict:
    import torch
    import paper_1803_11036_amd as ssd
    import tracegen as tg

    name = "core_link" if secondary else args.workload
    cfg = tg.config(name)
    if cfg.n_streams != 1:
        raise SystemExit("this mode times a single-link workload")
    trace = tg.Trace(cfg)
    tables = tg.hash_tables(cfg.hash_seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    W, K = (10, 20) if secondary else (args.warmup, args.steps)

    n_gen = min(W + K, cfg.n_slices)
    log(f"generating {n_gen} slices of {cfg.name}")
    t0 = time.perf_counter()
    slices = [trace.pairs_device(0, t, dev) for t in range(n_gen)]
    torch.cuda.synchronize()
    log(f"generated in {time.perf_counter() - t0:.1f} s")

    cell_bits = 16 if cfg.k > 254 else 8
    params = ssd.make_params(q=cfg.q, r=cfg.r, delta=cfg.delta, eta=cfg.eta, k=cfg.k, theta=cfg.theta,
                             max_tuples=1 << 22, max_results=1 << 20, cell_bits=cell_bits)
    det = ssd.init_detector(params, tables, device=dev)
    if not secondary:
        if args.pass_mib is not None:
            ssd.set_tuning(det, ssd.SSD_TUNE_SCAN_PASS_BYTES, args.pass_mib << 20)
        if args.scan_mode is not None:
            ssd.set_tuning(det, ssd.SSD_TUNE_SCAN_MODE,
                           ssd.SSD_SCAN_BINNED if args.scan_mode == "binned" else ssd.SSD_SCAN_PASSES)
        if args.bin_kib is not None:
            ssd.set_tuning(det, ssd.SSD_TUNE_SCAN_BIN_BYTES, args.bin_kib << 10)
        if args.apply_segments is not None:
            ssd.set_tuning(det, ssd.SSD_TUNE_SCAN_APPLY_SEGMENTS, args.apply_segments)
        if args.no_counted:
            ssd.set_tuning(det, ssd.SSD_TUNE_COUNTED, 0)
    ssd.set_tuning(det, ssd.SSD_TUNE_TIMING, 1)
    state_bytes = det.state.numel()

    t = 0
    for i in range(W):
        ssd.scan_slice(det, slices[i % n_gen], t)
        ssd.close_slice(det)
        t += 1
    torch.cuda.synchronize()
    ssd.read_timing(det, reset=True)

    n_timed = 0
    torch.cuda.synchronize()
    start = time.perf_counter()
    # pipelined: slice t+1's scan is enqueued before slice t's list is
    # collected, so the host's collection overlaps device work
    for i in range(K):
        s = slices[(W + i) % n_gen]
        ssd.scan_slice(det, s, t)
        if i > 0:
            ssd.close_end(det)
        ssd.close_begin(det)
        t += 1
        n_timed += s.shape[0]
    ssd.close_end(det)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - start
    timing = ssd.read_timing(det, reset=True)
    info = ssd.get_info(det)

    # slice-close latency: scans drained first, then close_slice() call to list in host memory
    lat = []
    for i in range(args.latency_steps):
        s = slices[(W + i) % n_gen]
        ssd.scan_slice(det, s, t)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        ssd.close_slice(det)
        lat.append((time.perf_counter() - c0) * 1e3)
        t += 1
    ssd.read_timing(det, reset=True)

    # end to end: pairs from pinned host memory, the next slice's copy on a
    # copy stream overlapping this slice's scan and close
    e2e = None
    if args.e2e_steps:
        host = [s.cpu().pin_memory() for s in slices[:4]]
        bufs = [torch.empty_like(slices[0]) for _ in range(2)]
        cs = torch.cuda.Stream(dev)
        cur = torch.cuda.current_stream(dev)
        copied = [torch.cuda.Event() for _ in range(2)]
        used = [torch.cuda.Event() for _ in range(2)]

        def copy(j):
            with torch.cuda.stream(cs):
                cs.wait_event(used[j % 2])          # the scan that last read this buffer is done
                bufs[j % 2].copy_(host[j % len(host)], non_blocking=True)
                copied[j % 2].record(cs)

        for e in used:
            e.record(cur)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        copy(0)
        n_e2e = 0
        for j in range(args.e2e_steps):
            if j + 1 < args.e2e_steps:
                copy(j + 1)
            cur.wait_event(copied[j % 2])
            ssd.scan_slice(det, bufs[j % 2], t)
            used[j % 2].record(cur)
            if j > 0:
                ssd.close_end(det)
            ssd.close_begin(det)
            t += 1
            n_e2e += bufs[j % 2].shape[0]
        ssd.close_end(det)
        torch.cuda.synchronize()
        e2e_s = time.perf_counter() - t0
        e2e = {"packets_per_s": round(n_e2e / e2e_s, 1), **gbps(n_e2e / e2e_s),
               "ms_per_step": round(e2e_s * 1e3 / args.e2e_steps, 4), "steps": args.e2e_steps,
               "note": "pairs copied host->device from pinned memory each step, overlapping the previous "
                       "slice's scan and close; bound by the host link"}
        del host, bufs

    if args.calibrate_copy_mib and not secondary:
        calibration_copy(dev, args.calibrate_copy_mib)

    pps = n_timed / elapsed
    avg_pairs = n_timed / K
    kernels = {}
    for kname, (ms, launches) in timing.items():
        if launches:
            kernels[kname] = {"ms_total": round(ms, 4), "launches": launches, "ms_per_launch": round(ms / launches, 5)}
    binned = timing["scan_bin"][1] > 0
    counted = timing["count_detect"][1] > 0
    scan_ms = (timing["scan"][0] + timing["scan_bin"][0]) / K
    # algorithmic bytes (per scan call: 8 + r per pair, the pair read and one
    # recorder written per row; per close: the state read by hot detection)
    cell_b = 2 if cell_bits == 16 else 1
    alg_scan = avg_pairs * (8 + cfg.r * cell_b)
    cands = {}
    # the binned stores: counted, the bitmap stores of 16-bit cells (no
    # counters; the last call's bin size is reported), or a byte store per offset
    marked = binned and not counted and cell_bits == 16 and info["counted_bin_kib"] > 0
    stores = ("k_apply_counted" if counted else "k_apply_marked16" if marked else "k_apply") if binned else "k_scan"
    # implementation bytes: the 4-byte offsets plus the cells stored (read too
    # by the stores that read-modify-write 16-byte chunks)
    impl_scan = avg_pairs * cfg.r * (4 + cell_b * (2 if counted or marked else 1)) if binned else None
    n_scan = timing["scan"][1]
    if n_scan:
        cands[stores] = (timing["scan"][0] / K, alg_scan / max(1, n_scan // K), timing["scan"][0] / n_scan,
                         n_scan // K, impl_scan / max(1, n_scan // K) if impl_scan else None)
    if binned:
        n_bin = timing["scan_bin"][1]
        cands["k_bin"] = (timing["scan_bin"][0] / K, avg_pairs * 8.0 / max(1, n_bin // K),
                          timing["scan_bin"][0] / n_bin, n_bin // K, avg_pairs * (8 + 4 * cfg.r) / max(1, n_bin // K))
    if timing["hot_detect"][1]:
        ms = timing["hot_detect"][0]
        cands["k_hot_detect"] = (ms / K, float(state_bytes), ms / timing["hot_detect"][1], 1, None)
    if counted:
        ms = timing["count_detect"][0]
        n_se = cfg.r << cfg.q
        n_hot = sum(info["hot_counts"][:cfg.r])
        impl = n_se * 20 + n_hot * (cfg.eta + cfg.eta // 8) + n_se / (255 - cfg.k) * cfg.eta
        # R_k of every estimator from its counters instead of the state: the
        # bytes it reads and writes (counters, hot and expiring estimators'
        # cells, snapshots) stand for its work
        cands["k_count"] = (ms / K, float(impl), ms / timing["count_detect"][1], 1, impl)
    if timing["close_graph"][1]:
        ms = timing["close_graph"][0]
        cands["close_graph"] = (ms / K, 0.0, ms / timing["close_graph"][1], 1, None)
    roof = roofline(cands, cfg.name)

    out = {
        "metric": METRIC,
        "value": round(pps, 1), "unit": "packets/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(elapsed * 1e3 / K, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u16" if cell_bits == 16 else "u8", "data": "synthetic",
        "config": {"workload": f"{cfg.name}: 1 link, {cfg.pairs_lo} pairs/slice, k={cfg.k}, "
                               f"theta={cfg.theta}, {cfg.r}x2^{cfg.q} estimators x {cfg.eta} cells of {cell_bits} bits",
                   "form": "plain", "pairs_per_slice": int(avg_pairs), "k": cfg.k, "theta": cfg.theta,
                   "q": cfg.q, "r": cfg.r, "delta": cfg.delta, "eta": cfg.eta, "cell_bits": cell_bits,
                   "state_bytes": state_bytes},
        **gbps(pps),
        "scan_packets_per_s": round(avg_pairs / (scan_ms * 1e-3), 1) if scan_ms > 0 else None,
        "close_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                             "p99": round(float(np.percentile(lat, 99)), 4)} if lat else None,
        "kernels": kernels,
        "last_close": {"hot_counts": info["hot_counts"], "level_counts": info["level_counts"],
                       "reported": info["reported"]},
        "roofline": roof,
        "end_to_end": e2e,
    }
    det.destroy()
    del slices
    torch.cuda.empty_cache()
    if secondary:
        for key in ("metric", "unit", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
            out.pop(key)
        return out
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline_link(cfg, trace, tables, args.cpu_slices)
    return out


# ----------------------------------------------------------------------------
# served and distributed forms

def run_served(args) -> dict:
    """32 streams with Poisson batch arrivals (continuous batching): the
    serving loop with group scans / closes against the same schedule issued as
    plain per-stream launches; identical lists checked for every stream slot."""
    import torch
    import tracegen as tg
    from paper_1803_11036_amd import serve

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ws = tg.served_workload(n_streams=args.streams, n_slots=args.slots)
    log(f"served: {len(ws)} streams, building reservoirs")
    inputs = serve.build_inputs(ws, device=dev)
    torch.cuda.synchronize()
    budget = args.budget_gb << 30
    reps = {}
    for mode in ("plain", "batched"):
        log(f"served {mode} at time scale {args.time_scale}")
        reps[mode] = serve.serve(inputs, budget, time_scale=args.time_scale, batched=(mode == "batched"))
    b, pl = reps["batched"], reps["plain"]
    same = all((b.results.get(key) is not None and pl.results.get(key) is not None and
                np.array_equal(b.results[key], pl.results[key])) for key in pl.results)
    return {
        "metric": METRIC,
        "value": round(b.pairs_per_s, 1), "unit": "packets/s", "n_gpus": 1, "steps": len(b.latencies_ms),
        "warmup": 0, "ms_per_step": round(b.wall_s * 1e3 / max(1, len(b.latencies_ms)), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"served: {len(ws)} streams, Poisson batches of 64K-4M pairs, mean gap 5 ms / "
                               f"rate weight, slots 50-500 ms, time scale {args.time_scale}",
                   "form": "served", "streams": len(ws), "time_scale": args.time_scale,
                   "budget_bytes": budget, "pairs": b.pairs},
        **gbps(b.pairs_per_s),
        "close_latency_ms": {"p50": round(b.latency(50), 4), "p99": round(b.latency(99), 4)},
        "plain": {"packets_per_s": round(pl.pairs_per_s, 1),
                  "close_latency_ms": {"p50": round(pl.latency(50), 4), "p99": round(pl.latency(99), 4)},
                  "scan_calls": pl.scan_calls, "close_calls": pl.close_calls, "wall_s": round(pl.wall_s, 3)},
        "batched": {"scan_calls": b.scan_calls, "close_calls": b.close_calls,
                    "max_scan_members": b.max_scan_members, "max_close_members": b.max_close_members,
                    "max_admitted": b.max_admitted, "wall_s": round(b.wall_s, 3)},
        "served_over_plain": round(b.pairs_per_s / pl.pairs_per_s, 3) if pl.pairs_per_s else None,
        "identical_outputs": bool(same),
        "note": "wall-clock rate of a time-driven run: it equals the offered load when the GPU keeps up",
    }


def run_distributed(args) -> dict:
    """The distributed workload (Alg. 5): every slice, 16 router detectors scan
    their own pairs, their states are merged into the global detector, which
    closes; the routers only advance.  Throughput counts every router's pairs."""
    import torch
    import paper_1803_11036_amd as ssd
    import tracegen as tg

    cfg = tg.config("distributed")
    tr = tg.Trace(cfg)
    tabs = tg.hash_tables(cfg.hash_seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n_var = max(1, args.variants)
    log(f"generating {n_var} slices of {cfg.name} ({cfg.n_streams} routers each)")
    slices = []
    for v in range(n_var):
        per = tr.pairs_all(v)
        slices.append([torch.from_numpy(np.ascontiguousarray(p).view(np.int32)).to(dev) for p in per])
    params = ssd.make_params(q=cfg.q, r=cfg.r, delta=cfg.delta, eta=cfg.eta, k=cfg.k, theta=cfg.theta,
                             max_tuples=1 << 22, max_results=1 << 20)
    routers = [ssd.init_detector(params, tabs, device=dev) for _ in range(cfg.n_streams)]
    glob = ssd.init_detector(params, tabs, device=dev)
    for d in routers + [glob]:
        ssd.set_tuning(d, ssd.SSD_TUNE_TIMING, 1)
    if args.calibrate_copy_mib:
        calibration_copy(dev, args.calibrate_copy_mib)
    W, K = args.warmup, args.steps
    t = 0
    n_timed = 0
    reported = 0
    for i in range(W + K):
        per = slices[i % n_var]
        if i == W:
            torch.cuda.synchronize()
            for d in routers + [glob]:
                ssd.read_timing(d, reset=True)
            t0 = time.perf_counter()
        for j, d in enumerate(routers):
            ssd.scan_slice(d, per[j], t)
        ssd.merge_router_state(glob, routers)
        res = ssd.close_slice(glob)
        for d in routers:
            ssd.close_slice(d, advance_only=True)
        if i >= W:
            n_timed += sum(int(p.shape[0]) for p in per)
            reported = len(res)
        t += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tg_ = ssd.read_timing(glob, reset=True)
    rt = [ssd.read_timing(d, reset=True) for d in routers]
    # the routers' binned scans: k_bin, then the stores (the routers only
    # advance, so their counters go stale after the first close; a large call
    # still takes the counted stores, k_apply_counted, when the routers can
    # count -- the bin size of their last such call is reported -- else
    # k_apply)
    counted_routers = all(ssd.get_info(d)["counted_bin_kib"] > 0 for d in routers)
    apply_ms, apply_n = sum(x["scan"][0] for x in rt), sum(x["scan"][1] for x in rt)
    bin_ms, bin_n = sum(x["scan_bin"][0] for x in rt), sum(x["scan_bin"][1] for x in rt)
    scan_ms = apply_ms + bin_ms
    pairs_call = sum(int(p.shape[0]) for p in slices[0]) / cfg.n_streams
    state = glob.state.numel()
    merge_ms = tg_["merge"][0] / max(1, tg_["merge"][1])
    merge_bytes = (cfg.n_streams + 1) * state          # every router state read, the global written
    cands = {"k_merge": (tg_["merge"][0] / K, float(merge_bytes), merge_ms, 1, None)}
    if apply_n:
        cands["k_apply_counted" if counted_routers else "k_apply"] = (
            apply_ms / K, (8 + cfg.r) * pairs_call, apply_ms / apply_n, apply_n // K,
            (6 if counted_routers else 5) * cfg.r * pairs_call)
    if bin_n:
        cands["k_bin"] = (bin_ms / K, 8.0 * pairs_call, bin_ms / bin_n, bin_n // K, (8 + 4 * cfg.r) * pairs_call)
    if tg_["hot_detect"][1]:
        cands["k_hot_detect"] = (tg_["hot_detect"][0] / K, float(state), tg_["hot_detect"][0] / tg_["hot_detect"][1],
                                 1, None)
    roof = roofline(cands, cfg.name)
    for d in routers + [glob]:
        d.destroy()
    pps = n_timed / elapsed
    return {
        "metric": METRIC,
        "value": round(pps, 1), "unit": "packets/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(elapsed * 1e3 / K, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"distributed: {cfg.n_streams} routers, {n_timed // K} pairs/slice in total, "
                               f"k={cfg.k}, theta={cfg.theta}, {cfg.r}x2^{cfg.q} estimators x {cfg.eta} cells each",
                   "form": "distributed", "routers": cfg.n_streams, "state_bytes_per_router": state,
                   "slice_variants": n_var},
        **gbps(pps),
        "reported_last_slice": reported,
        "kernels": {"router_scans": {"ms_per_step": round(scan_ms / K, 4)},
                    "merge": {"ms_per_launch": round(merge_ms, 5), "launches": tg_["merge"][1]},
                    "global_hot_detect": {"ms_per_launch": round(tg_["hot_detect"][0] / max(1, tg_["hot_detect"][1]), 5)}},
        "roofline": roof,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_distributed(cfg, tr, tabs, args.cpu_slices),
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batched",
                    help="batched (default) | core_link | tiny | paper | distributed | served | ceilings")
    ap.add_argument("--latency-steps", type=int, default=10)
    ap.add_argument("--e2e-steps", type=int, default=12, help="steps of the pinned-host end-to-end run (0 = off)")
    ap.add_argument("--cpu-slices", type=int, default=8,
                    help="single-link workloads: oracle slices timed after the window is filled (at most, until 10 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="batched: skip the core-link secondary run")
    ap.add_argument("--no-ceilings", action="store_true", help="batched: skip the memory-ceiling probes")
    ap.add_argument("--pass-mib", type=int, default=None, help="scan pass window (MiB of state; default: library)")
    ap.add_argument("--scan-mode", choices=["passes", "binned"], default=None,
                    help="single-detector scan: pass windows or bin-sorted stores (default: library)")
    ap.add_argument("--bin-kib", type=int, default=None, help="binned scan: bin size in KiB (power of two)")
    ap.add_argument("--apply-segments", type=int, default=None, help="binned scan: segments per store workgroup")
    ap.add_argument("--no-counted", action="store_true",
                    help="hot detection scans the whole state (no per-slot counters)")
    ap.add_argument("--counted-min-items", type=int, default=None,
                    help="batched workload: offsets per bin a link's call needs to keep counters (default: library)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this size (PMC calibration)")
    ap.add_argument("--links", type=int, default=64, help="batched workload: number of links")
    ap.add_argument("--variants", type=int, default=2, help="batched workload: distinct slice contents cycled")
    ap.add_argument("--autotune", type=int, default=1, help="batched workload: autotune before the warmup")
    ap.add_argument("--streams", type=int, default=32, help="served workload: streams")
    ap.add_argument("--slots", type=int, default=6, help="served workload: slots per stream")
    ap.add_argument("--time-scale", type=float, default=0.25, help="served workload: stream time per wall second")
    ap.add_argument("--budget-gb", type=int, default=64, help="served workload: admission memory budget")
    ap.add_argument("--ceiling-mib", default="24,1536,5120", help="ceilings workload: working-set sizes in MiB")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this detector runs on one GPU; multi-GPU sharding is a design "
                                   "note only, run with --gpus 1"}), flush=True)
        return 2
    if args.workload == "batched":
        out = run_batched(args)
    elif args.workload == "served":
        out = run_served(args)
    elif args.workload == "distributed":
        out = run_distributed(args)
    elif args.workload == "ceilings":
        import torch
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        out = {"workload": "ceilings", "ceilings": ceilings(dev, [int(x) for x in args.ceiling_mib.split(",")]),
               "note": "stream read GB/s; byte scatter G stores/s (uniform over the buffer, and XCD-local: "
                       "workgroups of one XCD store into 2 MiB regions its L2 holds, every region in turn); "
                       "16-byte read-modify-writes G chunks/s (one workgroup per 512 KiB bin, 2048 hashed chunks "
                       "per bin, bins dealt to the XCDs as the counted stores deal theirs)"}
    else:
        out = run_core(args)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
