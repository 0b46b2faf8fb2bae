"""Exact opposite numbers: the paper's "precise algorithm" (Sec. 3.2).

Test infrastructure only.  For every host the set of distinct peers seen in a
period is kept and counted (Def. 1), so the result is exact; a host is a super
point when its count is at least theta (Def. 2), and a sliding super point of
window SW(i, k) when its count over slots i..i+k-1 is (Def. 3 and 4).  This
pins the method's accuracy, not its bit-exact state.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np


def opposite_numbers(pair_sets: Iterable[np.ndarray]) -> Tuple[np.ndarray, np.ndarray]:
    """Distinct-peer counts over the union of the given pair arrays.

    Returns (hosts ascending, counts).
    """
    keys = []
    for p in pair_sets:
        p = np.asarray(p, dtype=np.uint32).reshape(-1, 2)
        keys.append((p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64))
    if not keys:
        return np.zeros(0, np.uint32), np.zeros(0, np.int64)
    u = np.unique(np.concatenate(keys))
    hosts, counts = np.unique((u >> np.uint64(32)).astype(np.uint32), return_counts=True)
    return hosts, counts


def window_super_points(slices: Sequence[np.ndarray], t: int, k: int, theta: int) -> np.ndarray:
    """SSP at the close of slot t: hosts with >= theta distinct peers over
    slots max(0, t-k+1)..t (Def. 4; early windows are the slots seen so far)."""
    lo = max(0, t - k + 1)
    hosts, counts = opposite_numbers(slices[lo:t + 1])
    return hosts[counts >= theta]


def precise_count(pairs: Sequence[Tuple[int, int]]) -> Dict[int, int]:
    """Literal sequential precise algorithm on a small list of pairs: one
    buffer of seen peers per host, a peer inserted only if not yet present."""
    buf: Dict[int, List[int]] = {}
    for cip, oip in pairs:
        seen = buf.setdefault(cip, [])
        if oip not in seen:
            seen.append(oip)
    return {h: len(v) for h, v in buf.items()}


class SlidingWindowTruth:
    """Exact sliding super points of a stream of slots, in time linear in the
    distinct pairs kept: every distinct (host, peer) pair seen remembers the
    last slot it occurred in, and a pair belongs to the window of slot t
    exactly when that slot is at least t - k + 1 (Def. 3 and 4; early
    windows are the slots seen so far).  Pairs that left the window are
    dropped (a later occurrence adds them again)."""

    def __init__(self, k: int, theta: int):
        self.k, self.theta = k, theta
        self.t = -1
        self.keys = np.zeros(0, np.uint64)       # sorted: host in the high half, peer in the low half
        self.last = np.zeros(0, np.int64)

    def add(self, pairs: np.ndarray) -> np.ndarray:
        """Feed slot t+1's pairs (any repeats); returns the SSP of its window."""
        self.t += 1
        t = self.t
        p = np.asarray(pairs, dtype=np.uint32).reshape(-1, 2)
        new = np.unique((p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64))
        keys = np.concatenate([self.keys, new])
        last = np.concatenate([self.last, np.full(new.size, t, np.int64)])
        # two sorted runs: a stable merge sort merges them in linear time, the
        # old entry of a key first, then the slot's own
        order = np.argsort(keys, kind="stable")
        keys, last = keys[order], last[order]
        # keep the latest occurrence of every key
        keep = np.ones(keys.size, bool)
        keep[:-1] = keys[:-1] != keys[1:]
        keys, last = keys[keep], last[keep]
        live = last >= t - self.k + 1
        self.keys, self.last = keys[live], last[live]
        # keys are sorted, so every host's pairs are one run
        hosts = (self.keys >> np.uint64(32)).astype(np.uint32)
        if hosts.size == 0:
            return hosts
        start = np.flatnonzero(np.concatenate([[True], hosts[1:] != hosts[:-1]]))
        counts = np.diff(np.concatenate([start, [hosts.size]]))
        return hosts[start][counts >= self.theta]
