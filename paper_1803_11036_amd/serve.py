"""Serving loop: continuous batching of packet batches from many streams.

Every admitted stream owns a single detector whose state stays resident in
HBM.  Each loop iteration
  1. admits waiting streams, in arrival order, while the memory budget allows
     (state + scratch of their detectors);
  2. scans every batch that has arrived for any admitted stream's open slot,
     all in one group scan launch (streams of different geometries together);
  3. collects the lists of the group close begun in the previous iteration
     (the slice-close latency is measured from the slot's end to the list in
     host memory) and frees the detectors of finished streams, so that
     waiting streams can be admitted;
  4. begins one group close of every stream whose open slot has ended: the
     close runs on the device while the next iteration admits streams and
     enqueues their scans, and its streams' next slots are open at once.
Requests arriving while others are on the GPU simply join the next iteration.
A stream can be dropped at a given stream time (its client gone): at the
first iteration after that time with no close of it pending, its detector is
freed mid-slot; its open slot is never closed and no other stream is
touched.
All work runs in the library's kernels; this module only decides what runs
together.  Stream time advances at `time_scale` times wall time.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import (Detector, Group, get_info, group_close_begin, group_close_end, group_scan, init_detector,
               make_params, query_sizes)


@dataclasses.dataclass
class StreamInput:
    """One stream as the server sees it: detector parameters and tables, slot
    length (stream seconds), batch arrival times and sizes, and the device
    reservoir whose rows [starts[j], starts[j] + sizes[j]) (cyclic) are batch j."""
    params: object
    tables: np.ndarray
    slot: float
    n_slots: int
    arrivals: np.ndarray
    sizes: np.ndarray
    starts: np.ndarray
    reservoir: torch.Tensor

    def ranges(self, j: int) -> List[Tuple[int, int]]:
        """Batch j as (first row, rows) ranges of the reservoir: exactly
        sizes[j] rows from starts[j] on, wrapping around it as often as needed."""
        R = self.reservoir.shape[0]
        a, n = int(self.starts[j]) % R, int(self.sizes[j])
        out = []
        while n > 0:
            m = min(n, R - a)
            out.append((a, m))
            n -= m
            a = 0
        return out

    def pieces(self, j: int) -> List[torch.Tensor]:
        """Batch j as views of the reservoir."""
        return [self.reservoir[a:a + m] for a, m in self.ranges(j)]

    def run_pieces(self, j0: int, j1: int) -> List[torch.Tensor]:
        """Batches j0 .. j1 - 1 in order, as views of the reservoir, each
        covering a run of rows that the batches take one after another."""
        return [self.reservoir[a:a + m] for a, m in coalesce(r for j in range(j0, j1) for r in self.ranges(j))]

    def batch(self, j: int) -> torch.Tensor:
        """Batch j as one tensor (a view when it does not wrap, else a copy)."""
        p = self.pieces(j)
        if not p:
            return self.reservoir[:0]
        return p[0] if len(p) == 1 else torch.cat(p)


def coalesce(ranges) -> List[Tuple[int, int]]:
    """(first, count) ranges in order, each range that starts where the
    previous one ends joined to it."""
    out: List[Tuple[int, int]] = []
    for a, m in ranges:
        if m <= 0:
            continue
        if out and out[-1][0] + out[-1][1] == a:
            out[-1] = (out[-1][0], out[-1][1] + m)
        else:
            out.append((a, m))
    return out


@dataclasses.dataclass
class ServeReport:
    wall_s: float
    pairs: int
    latencies_ms: List[float]
    results: Dict[Tuple[int, int], np.ndarray]
    max_admitted: int
    admit_wait_s: List[float]
    iterations: int
    scan_calls: int
    close_calls: int
    max_scan_members: int = 0         # streams sharing one scan launch, at most
    max_close_members: int = 0        # streams sharing one close, at most

    @property
    def pairs_per_s(self) -> float:
        return self.pairs / self.wall_s if self.wall_s > 0 else 0.0

    def latency(self, pct: float) -> float:
        return float(np.percentile(self.latencies_ms, pct)) if self.latencies_ms else 0.0


def stream_bytes(params) -> int:
    a, b = query_sizes(params)
    return a + b


class _Live:
    def __init__(self, idx: int, det: Detector, nbytes: int):
        self.idx = idx
        self.det = det
        self.nbytes = nbytes
        self.slot = 0          # open slot
        self.next = 0          # next batch not yet scanned
        self.closing = False   # a close of its previous slot is pending


def serve(streams: Sequence[StreamInput], budget_bytes: int, time_scale: float = 1.0,
          max_members: int = 64, device="cuda:0", keep_results: bool = True, batched: bool = True,
          drop: Optional[Dict[int, float]] = None) -> ServeReport:
    """Run every stream to its last slot (or, for a stream in `drop`, to its
    drop time in stream seconds); returns throughput, latencies and (if
    keep_results) each stream's list per closed slot.  batched=False issues
    the same work as plain per-stream launches (one scan per batch, one close
    per stream), for comparison."""
    from . import close_slice, scan_slice
    dev = torch.device(device)
    group = Group(max_members, device=dev)
    waiting = deque(sorted(range(len(streams)),
                           key=lambda i: streams[i].arrivals[0] if streams[i].arrivals.size else 0.0))
    live: Dict[int, _Live] = {}
    used = 0
    results: Dict[Tuple[int, int], np.ndarray] = {}
    lat: List[float] = []
    waits: List[float] = []
    pairs = 0
    iters = scans = closes = 0
    max_scan_m = max_close_m = 0
    max_live = 0
    done = 0
    t0 = time.perf_counter()

    def now_tau() -> float:
        return (time.perf_counter() - t0) * time_scale

    pending = None

    def finish(closed, lists, status):
        """Lists of closed (stream, slot)s are in host memory: latencies,
        results, and the finished streams' detectors freed."""
        nonlocal used, done
        t_done = time.perf_counter()
        for (L, slot), res, st in zip(closed, lists, status):
            s = streams[L.idx]
            slot_end_wall = t0 + (slot + 1) * s.slot / time_scale
            lat.append((t_done - slot_end_wall) * 1e3)
            if keep_results:
                results[(L.idx, slot)] = res if st == 0 else None
            L.closing = False
            if L.slot >= s.n_slots:
                L.det.destroy()
                used -= L.nbytes
                del live[L.idx]
                done += 1

    drop = dict(drop or {})
    while done < len(streams):
        iters += 1
        tau = now_tau()
        # 0. dropped streams: waiting ones leave the queue, admitted ones free
        # their detector (not while a close of theirs is pending)
        for i in [i for i in waiting if drop.get(i, float("inf")) <= tau]:
            waiting.remove(i)
            done += 1
        for i in [i for i, L in live.items() if drop.get(i, float("inf")) <= tau and not L.closing]:
            L = live.pop(i)
            L.det.destroy()
            used -= L.nbytes
            done += 1
        # 1. admission in arrival order while the budget allows
        while waiting and len(live) < max_members:
            i = waiting[0]
            s = streams[i]
            first = s.arrivals[0] if s.arrivals.size else 0.0
            if first > tau:
                break
            need = stream_bytes(s.params)
            if used + need > budget_bytes and live:
                break
            waiting.popleft()
            det = init_detector(s.params, s.tables, device=dev)
            live[i] = _Live(i, det, need)
            used += need
            waits.append(max(0.0, tau - first) / time_scale)
        max_live = max(max_live, len(live))
        # 2. one scan launch over every arrived batch of every open slot
        members, parts, counts, ids = [], [], [], []
        for i, L in live.items():
            s = streams[i]
            end = (L.slot + 1) * s.slot
            j = L.next
            while j < s.arrivals.size and s.arrivals[j] <= tau and s.arrivals[j] < end:
                j += 1
            if j > L.next:
                members.append(L)
                if batched:
                    parts.extend(s.run_pieces(L.next, j))
                else:
                    parts.extend(s.batch(b) for b in range(L.next, j))
                counts.append(int(s.sizes[L.next:j].sum()))
                ids.append(L.slot)
                L.next = j
        if members and batched:
            batch = torch.cat(parts) if len(parts) > 1 else parts[0].contiguous()
            offs = np.zeros(len(members) + 1, dtype=np.uint64)
            offs[1:] = np.cumsum(counts)
            group_scan(group, [L.det for L in members], batch, offs, ids)
            pairs += int(offs[-1])
            scans += 1
            max_scan_m = max(max_scan_m, len(members))
        elif members:
            k = 0
            for L, cnt, o in zip(members, counts, ids):
                got = 0
                while got < cnt:
                    part = parts[k].contiguous()
                    scan_slice(L.det, part, o)
                    got += part.shape[0]
                    k += 1
                    scans += 1
                pairs += cnt
        # 3. the lists of the close begun in the previous iteration: its
        # kernels ran while this iteration's scans were enqueued behind them
        if pending is not None:
            closed, lists, status = pending[0], *group_close_end(group)
            finish(closed, lists, status)
            pending = None
        # 4. one close over every stream whose open slot has ended
        closing = []
        for i, L in live.items():
            s = streams[i]
            end = (L.slot + 1) * s.slot
            if L.slot < s.n_slots and end <= tau and (L.next >= s.arrivals.size or s.arrivals[L.next] >= end):
                closing.append(L)
        if closing:
            closes += 1
            max_close_m = max(max_close_m, len(closing))
            if batched:
                group_close_begin(group, [L.det for L in closing])
                pending = ([(L, L.slot) for L in closing],)
                for L in closing:
                    L.slot += 1          # the next slot is open: its batches may be scanned
                    L.closing = True
            else:
                lists = [close_slice(L.det) for L in closing]
                closed = [(L, L.slot) for L in closing]
                for L in closing:
                    L.slot += 1
                    L.closing = True
                finish(closed, lists, [0] * len(closing))
        # 5. idle until the next arrival or slot end (not while a close is
        # pending: its lists are collected next)
        if not members and not closing and pending is None:
            nxt = []
            for i, L in live.items():
                s = streams[i]
                if L.slot < s.n_slots:
                    nxt.append((L.slot + 1) * s.slot)
                if L.next < s.arrivals.size:
                    nxt.append(s.arrivals[L.next])
            if waiting:
                s = streams[waiting[0]]
                nxt.append(s.arrivals[0] if s.arrivals.size else 0.0)
            if nxt:
                gap = (min(nxt) - now_tau()) / time_scale
                if gap > 0:
                    time.sleep(min(gap, 0.002))
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    group.destroy()
    return ServeReport(wall_s=wall, pairs=pairs, latencies_ms=lat, results=results, max_admitted=max_live,
                       admit_wait_s=waits, iterations=iters, scan_calls=scans, close_calls=closes,
                       max_scan_members=max_scan_m, max_close_members=max_close_m)


def serve_alone(s: StreamInput, device="cuda:0") -> List[np.ndarray]:
    """The same stream through its own detector, slot by slot: every batch of
    slot o scanned, then the slot closed (the reference for the mix)."""
    from . import close_slice, scan_slice
    dev = torch.device(device)
    det = init_detector(s.params, s.tables, device=dev)
    slot_of = np.floor(s.arrivals / s.slot).astype(np.int64)
    out = []
    for o in range(s.n_slots):
        for j in np.nonzero(slot_of == o)[0]:
            scan_slice(det, s.batch(int(j)).contiguous(), o)
        out.append(close_slice(det))
    det.destroy()
    return out


def build_inputs(served, device="cuda:0") -> List[StreamInput]:
    """Device reservoirs (shuffled whole-window pools) for tracegen streams."""
    import tracegen as tg
    dev = torch.device(device)
    out = []
    for i, w in enumerate(served):
        c = w.cfg
        tr = tg.Trace(c)
        pool = tr.window_pool()
        g = torch.Generator(device=dev)
        g.manual_seed(0x5E7 + i)
        res = torch.from_numpy(pool.view(np.int32)).to(dev)
        res = res[torch.randperm(res.shape[0], generator=g, device=dev)].contiguous()
        params = make_params(q=c.q, r=c.r, delta=c.delta, eta=c.eta, k=c.k, theta=c.theta,
                             max_tuples=1 << 21, max_results=1 << 18)
        out.append(StreamInput(params=params, tables=tg.hash_tables(c.hash_seed), slot=w.slot,
                               n_slots=w.n_slots, arrivals=w.arrivals, sizes=w.sizes, starts=w.starts,
                               reservoir=res))
    return out
