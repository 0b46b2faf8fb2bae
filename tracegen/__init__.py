"""Seeded synthetic IP-pair traces and hash-table draws.

This module is shared test and benchmark infrastructure.  It feeds both the
GPU detector and the CPU oracle and holds none of the detector's arithmetic:
it only draws random numbers and lays out (cip, oip) pairs.

Randomness is counter based so that any (stream, slice) can be regenerated on
its own:

* ``splitmix64`` is the published SplitMix64 generator (Steele, Lea and Flood,
  "Fast splittable pseudorandom number generators", OOPSLA 2014; the constants
  are the ones in Vigna's reference ``splitmix64.c``).  Output ``i`` of the
  stream seeded with ``s`` is ``mix(s + (i + 1) * GAMMA)``.
* The tabulation hash tables that the method draws (one table set for the
  column hash RHFG[0], one for the cell hash H1; Sec. 3.2 and 3.3 cite simple
  tabulation hashing) are 2 x 4 x 256 words taken from that stream in order,
  each the high 32 bits of one output.  They are passed to both sides as input.

Trace model (the paper measures on a CAIDA core-link trace that is not
available here, so these traces stand in for it; Sec. 5):

* a host set with a heavy-tailed window degree ``d_h`` (rank-Zipf or Pareto);
* each host owns a fixed pool of ``d_h`` random peers split into ``k`` chunks
  by (index + a per-host offset) mod ``k``; slice ``s`` emits chunk ``s mod
  k``, so a host active for a whole window has exactly ``d_h`` distinct peers
  in it, and the hosts' first peers spread evenly over the slices;
* planted super points with their own pools, some active only in a slice
  range so that they enter and leave mid-window;
* each slice is filled to exactly ``N`` pairs with repeats drawn uniformly
  from its own distinct pairs, then shuffled;
* for the distributed case every host is seen at one or several routers and
  its peers are dealt round-robin over them.

Pairs are ``uint32[n][2]`` with column 0 the monitored host (cip) and column 1
its peer (oip), host byte order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

__all__ = [
    "GAMMA", "splitmix64", "splitmix64_mix", "hash_tables", "TraceConfig",
    "CONFIGS", "Trace", "config", "batch_configs", "ServedStream", "served_workload",
]

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_U64 = np.uint64


def splitmix64_mix(z: np.ndarray) -> np.ndarray:
    """The SplitMix64 output function applied elementwise (uint64, wraps)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _U64(30))) * _M1
        z = (z ^ (z >> _U64(27))) * _M2
    return z ^ (z >> _U64(31))


def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs ``start .. start+n-1`` of the SplitMix64 stream seeded with ``seed``."""
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = _U64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GAMMA
    return splitmix64_mix(state)


def hash_tables(seed: int) -> np.ndarray:
    """Tabulation tables ``uint32[2][4][256]``: [0] for RHFG[0], [1] for H1."""
    out = splitmix64(seed, 2 * 4 * 256) >> _U64(32)
    return out.astype(np.uint32).reshape(2, 4, 256)


# ----------------------------------------------------------------------------
# counter-based helpers

def _key(*parts: int) -> np.uint64:
    """Derive a 64-bit stream key from integer parts (chained SplitMix64 mix)."""
    h = _U64(0x6A09E667F3BCC909)
    for p in parts:
        with np.errstate(over="ignore"):
            h = splitmix64_mix(np.array([h ^ _U64(p & 0xFFFFFFFFFFFFFFFF)],
                                        dtype=np.uint64))[0] + GAMMA
    return _U64(h)


def _rand64(key: np.uint64, idx: np.ndarray) -> np.ndarray:
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return splitmix64_mix(key + (idx + _U64(1)) * GAMMA)


def _uniform01(key: np.uint64, idx: np.ndarray) -> np.ndarray:
    """Uniform doubles in (0, 1]."""
    return ((_rand64(key, idx) >> _U64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


def _host_ip(idx: np.ndarray, seed: int) -> np.ndarray:
    """Bijective 32-bit scramble of host indices (distinct indices -> distinct IPs)."""
    x = (np.asarray(idx, dtype=np.uint64) ^ _U64(seed & 0xFFFFFFFF)) & _U64(0xFFFFFFFF)
    with np.errstate(over="ignore"):
        x ^= x >> _U64(16)
        x = (x * _U64(0x7FEB352D)) & _U64(0xFFFFFFFF)
        x ^= x >> _U64(15)
        x = (x * _U64(0x846CA68B)) & _U64(0xFFFFFFFF)
        x ^= x >> _U64(16)
    return x.astype(np.uint32)


# ----------------------------------------------------------------------------
# configurations

@dataclasses.dataclass(frozen=True)
class TraceConfig:
    name: str
    n_streams: int            # routers (distributed) or 1
    n_slices: int
    pairs_lo: int             # pairs per slice per stream, drawn once per stream
    pairs_hi: int             # (equal bounds -> fixed)
    k: int
    theta: int
    q: int
    r: int
    delta: int
    eta: int
    n_hosts: int
    degree_law: str           # "zipf" or "pareto"
    zipf_s: float = 1.1
    zipf_d1: float = 0.0
    pareto_alpha: float = 1.2
    degree_cap: int = 1_000_000
    multi_frac: float = 0.0   # fraction of background hosts seen at several routers
    multi_lo: int = 2
    multi_hi: int = 4
    n_planted: int = 0
    planted_lo: int = 2000    # planted window degree, log-uniform in [lo, hi]
    planted_hi: int = 2000
    planted_transient: float = 0.0  # fraction active only in a slice range
    planted_routers_lo: int = 1
    planted_routers_hi: int = 1
    seed: int = 0x55D00000
    hash_seed: int = 1

    @property
    def state_cells(self) -> int:
        return self.r * (1 << self.q) * self.eta


CONFIGS: Dict[str, TraceConfig] = {
    # 1 router, 8 slices of 1M pairs, k=4, Zipf(1.1) over 50k hosts
    # (sum of degrees = 2^20 per window) + 20 planted hosts of 2000 peers.
    "tiny": TraceConfig(
        name="tiny", n_streams=1, n_slices=8, pairs_lo=1_000_000, pairs_hi=1_000_000,
        k=4, theta=1024, q=12, r=6, delta=5, eta=1024,
        n_hosts=50_000, degree_law="zipf", zipf_s=1.1, zipf_d1=145_733.0,
        n_planted=20, planted_lo=2000, planted_hi=2000, seed=0x55D00000),
    # single 40 Gb/s core link: 60 slices of 6M pairs, k=10, 2M Pareto(1.2)
    # hosts + 500 planted super points (40% transient).
    "core_link": TraceConfig(
        name="core_link", n_streams=1, n_slices=60, pairs_lo=6_000_000, pairs_hi=6_000_000,
        k=10, theta=1024, q=16, r=6, delta=4, eta=4096,
        n_hosts=2_000_000, degree_law="pareto", pareto_alpha=1.2, degree_cap=1_000_000,
        n_planted=500, planted_lo=1500, planted_hi=50_000, planted_transient=0.4,
        seed=0x55D00001),
    # 16 edge routers over a shared host space, 1-4M pairs per router slice.
    "distributed": TraceConfig(
        name="distributed", n_streams=16, n_slices=24, pairs_lo=1_000_000, pairs_hi=4_000_000,
        k=8, theta=2048, q=14, r=5, delta=6, eta=4096,
        n_hosts=1_000_000, degree_law="pareto", pareto_alpha=1.2, degree_cap=1_000_000,
        multi_frac=0.3, multi_lo=2, multi_hi=4,
        n_planted=200, planted_lo=1500, planted_hi=12_000,
        planted_routers_lo=2, planted_routers_hi=8, seed=0x55D00002),
    # the paper's sliding-window parameter set (Sec. 5: one-second slots,
    # k = 300, eta = 2^11, q = 14, r = 5, delta = 6, theta = 1024) on a
    # core-link-shaped trace of 6M pairs per slot (40 Gb/s at 800 B); a
    # window of 300 slots carries about 6M distinct pairs (background plus
    # planted).  Its cells need 16 bits (k > 254).
    "paper": TraceConfig(
        name="paper", n_streams=1, n_slices=360, pairs_lo=6_000_000, pairs_hi=6_000_000,
        k=300, theta=1024, q=14, r=5, delta=6, eta=2048,
        n_hosts=800_000, degree_law="pareto", pareto_alpha=1.2, degree_cap=100_000,
        n_planted=150, planted_lo=1500, planted_hi=50_000, planted_transient=0.4,
        seed=0x55D00005),
}


def config(name: str, **overrides) -> TraceConfig:
    """A named configuration, optionally with fields replaced (smaller test sizes)."""
    return dataclasses.replace(CONFIGS[name], **overrides)


_BATCH_GEOMETRIES = [(12, 6, 5), (13, 6, 5), (14, 5, 6), (15, 5, 6), (16, 6, 4)]
_BATCH_THETAS = [512, 1024, 2048, 4096, 8192]


def batch_configs(n_links: int = 64, seed: int = 0x55D00003, pairs_scale: float = 1.0,
                  load: float = 0.25, max_window_distinct: float = float("inf")) -> List[TraceConfig]:
    """Independent monitored links of uneven rates, windows and thresholds:
    pairs per slice log-uniform in [0.2M, 8M] (times pairs_scale), k uniform in
    4..64, theta in {512, ..., 8192}, geometry (q, r, delta) one of five sets
    covering 2^12..2^16 columns, eta = the power of two >= max(1024, theta),
    a Pareto(1.2) host population sized so that a window carries about
    load * 2^q * theta distinct pairs (and at most half the window's pairs),
    plus a few planted super points."""
    out = []
    for l in range(n_links):
        u = _uniform01(_key(seed, 0xBA7C4, l), np.arange(8))
        N = int(round(math.exp(math.log(200_000) + u[0] * math.log(40.0)) * pairs_scale))
        N = max(N, 2000)
        k = 4 + int(u[1] * 61)
        theta = _BATCH_THETAS[min(4, int(u[2] * 5))]
        q, r, delta = _BATCH_GEOMETRIES[min(4, int(u[3] * 5))]
        eta = 1024
        while eta < theta:
            eta *= 2
        window_distinct = min(load * (1 << q) * theta, 0.5 * N * k, max_window_distinct)
        hosts = max(100, int(window_distinct / 5.1))
        n_planted = 5 + int(u[4] * 46)
        n_planted = max(1, min(n_planted, int(0.2 * N * k / (2.5 * theta))))
        out.append(TraceConfig(
            name=f"batched_link{l}", n_streams=1, n_slices=k + 8, pairs_lo=N, pairs_hi=N,
            k=k, theta=theta, q=q, r=r, delta=delta, eta=eta, n_hosts=hosts, degree_law="pareto",
            pareto_alpha=1.2, degree_cap=max(1000, int(0.05 * window_distinct)),
            n_planted=n_planted, planted_lo=int(1.5 * theta), planted_hi=4 * theta,
            seed=seed ^ ((l + 1) << 20), hash_seed=1 + l))
    return out


# ----------------------------------------------------------------------------
# trace generation

_P_DEG, _P_PEER, _P_ACT, _P_ROUTE, _P_FILL, _P_PERM, _P_NPAIRS, _P_PLANT = range(1, 9)


class Trace:
    """Deterministic trace for one configuration.

    ``pairs(stream, slice)`` returns ``uint32[N][2]``; ``distinct(stream, slice)``
    the distinct pairs that slice carries (before repeats and shuffling).
    """

    def __init__(self, cfg: TraceConfig):
        self.cfg = cfg
        c = cfg
        H, P = c.n_hosts, c.n_planted
        # background degrees
        if c.degree_law == "zipf":
            rank = np.arange(1, H + 1, dtype=np.float64)
            deg = np.rint(c.zipf_d1 * rank ** (-c.zipf_s))
        elif c.degree_law == "pareto":
            u = _uniform01(_key(c.seed, _P_DEG, 0), np.arange(H))
            deg = np.floor(u ** (-1.0 / c.pareto_alpha))
        else:
            raise ValueError(c.degree_law)
        deg = np.minimum(deg, c.degree_cap).astype(np.int64)
        # planted degrees: log-uniform
        if P:
            u = _uniform01(_key(c.seed, _P_PLANT, 0), np.arange(P))
            lo, hi = math.log(c.planted_lo), math.log(c.planted_hi)
            pdeg = np.rint(np.exp(lo + (hi - lo) * (1.0 - u))).astype(np.int64)
        else:
            pdeg = np.zeros(0, dtype=np.int64)
        self.degree = np.concatenate([deg, pdeg])
        self.n_all = H + P
        self.ip = _host_ip(np.arange(self.n_all), c.seed)
        # activity: [start, end) slice range; background hosts are always active
        start = np.zeros(self.n_all, dtype=np.int64)
        end = np.full(self.n_all, c.n_slices, dtype=np.int64)
        if P and c.planted_transient > 0:
            ka = _key(c.seed, _P_ACT, 0)
            u = _uniform01(ka, np.arange(3 * P)).reshape(3, P)
            trans = u[0] < c.planted_transient
            length = np.floor(c.k / 2 + u[1] * (3 * c.k - c.k / 2 + 1)).astype(np.int64)
            length = np.clip(length, 1, None)
            st = np.floor(u[2] * c.n_slices).astype(np.int64)
            start[H:][trans] = st[trans]
            end[H:][trans] = np.minimum(st[trans] + length[trans], c.n_slices)
        self.start, self.end = start, end
        # routing: each host is seen at m_h routers (b_h + i*step_h) mod R
        R = c.n_streams
        if R > 1:
            kr = _key(c.seed, _P_ROUTE, 0)
            u = _uniform01(kr, np.arange(4 * self.n_all)).reshape(4, self.n_all)
            m = np.ones(self.n_all, dtype=np.int64)
            multi = u[0][:H] < c.multi_frac
            span = c.multi_hi - c.multi_lo + 1
            m[:H][multi] = c.multi_lo + np.floor(u[1][:H][multi] * span).astype(np.int64)
            if P:
                pspan = c.planted_routers_hi - c.planted_routers_lo + 1
                m[H:] = c.planted_routers_lo + np.floor(u[1][H:] * pspan).astype(np.int64)
            m = np.minimum(m, R)
            base = np.floor(u[2] * R).astype(np.int64)
            step = 2 * np.floor(u[3] * (R // 2)).astype(np.int64) + 1   # odd: distinct routers
            self.route_m, self.route_base, self.route_step = m, base, step
        else:
            self.route_m = np.ones(self.n_all, dtype=np.int64)
            self.route_base = np.zeros(self.n_all, dtype=np.int64)
            self.route_step = np.ones(self.n_all, dtype=np.int64)
        # pairs per slice, fixed per stream
        kn = _key(c.seed, _P_NPAIRS, 0)
        u = _uniform01(kn, np.arange(R))
        self.n_pairs = (c.pairs_lo + np.floor(u * (c.pairs_hi - c.pairs_lo + 1))).astype(np.int64)
        self.n_pairs = np.minimum(self.n_pairs, c.pairs_hi)
        self._peer_key = _key(c.seed, _P_PEER, 0)
        # per-host chunk offset: spreads every host's first peers over the k slices
        self.chunk_offset = (_rand64(_key(c.seed, _P_ACT, 1), np.arange(self.n_all))
                             % _U64(c.k)).astype(np.int64)

    # peers of host h: pool index p in [0, degree[h])
    def _peer(self, host: np.ndarray, p: np.ndarray) -> np.ndarray:
        x = (host.astype(np.uint64) << _U64(32)) | p.astype(np.uint64)
        return (_rand64(self._peer_key, x) >> _U64(32)).astype(np.uint32)

    def _chunk(self, s: int):
        """Hosts, pool indices and routers of every distinct pair of slice s."""
        c = self.cfg
        k = c.k
        # host h emits pool index p in slice s iff (p + offset_h) = s (mod k)
        s0 = (s - self.chunk_offset) % k
        act = (self.start <= s) & (s < self.end) & (self.degree > s0)
        hosts = np.nonzero(act)[0]
        cnt = (self.degree[hosts] - s0[hosts] + k - 1) // k      # p = s0_h + k*j
        tot = int(cnt.sum())
        h = np.repeat(hosts, cnt)
        first = np.cumsum(cnt) - cnt
        j = np.arange(tot, dtype=np.int64) - np.repeat(first, cnt)
        p = s0[h] + k * j
        if c.n_streams > 1:
            # deal the chunk's peers round-robin over the host's routers
            m = self.route_m[h]
            router = (self.route_base[h] + (j % m) * self.route_step[h]) % c.n_streams
        else:
            router = np.zeros(tot, dtype=np.int64)
        return h, p, router

    def _rows(self, h: np.ndarray, p: np.ndarray) -> np.ndarray:
        out = np.empty((h.size, 2), dtype=np.uint32)
        out[:, 0] = self.ip[h]
        out[:, 1] = self._peer(h, p)
        return out

    def distinct(self, stream: int, s: int) -> np.ndarray:
        """Distinct (cip, oip) pairs of slice ``s`` at stream ``stream``."""
        h, p, router = self._chunk(s)
        keep = router == stream
        return self._rows(h[keep], p[keep])

    def distinct_all(self, s: int) -> List[np.ndarray]:
        """Distinct pairs of slice ``s`` for every stream, in one pass."""
        h, p, router = self._chunk(s)
        order = np.argsort(router, kind="stable")
        bounds = np.searchsorted(router[order], np.arange(self.cfg.n_streams + 1))
        rows = self._rows(h[order], p[order])
        return [rows[bounds[i]:bounds[i + 1]] for i in range(self.cfg.n_streams)]

    def pairs(self, stream: int, s: int, n: Optional[int] = None) -> np.ndarray:
        """The slice's ``N`` pairs: distinct pairs plus uniform repeats, shuffled."""
        return self._fill(stream, s, self.distinct(stream, s), n)

    def pairs_all(self, s: int) -> List[np.ndarray]:
        """``pairs(stream, s)`` for every stream (same values, one pass)."""
        return [self._fill(i, s, d, None) for i, d in enumerate(self.distinct_all(s))]

    def _fill(self, stream: int, s: int, d: np.ndarray, n: Optional[int]) -> np.ndarray:
        c = self.cfg
        N = int(self.n_pairs[stream]) if n is None else int(n)
        D = d.shape[0]
        if D == 0 or N == 0:
            return np.zeros((0, 2), dtype=np.uint32)
        if D > N:
            raise ValueError(f"slice {s} of stream {stream} has {D} distinct pairs > {N}")
        kf = _key(c.seed, _P_FILL, stream, s)
        rep = (_rand64(kf, np.arange(N - D)) % _U64(D)).astype(np.int64)
        idx = np.concatenate([np.arange(D, dtype=np.int64), rep])
        g = np.random.Generator(np.random.Philox(key=int(_key(c.seed, _P_PERM, stream, s))))
        g.shuffle(idx)
        # gather rows as single little-endian words: low half cip, high half oip
        return np.ascontiguousarray(d).view(np.uint64)[idx, 0].view(np.uint32).reshape(N, 2)

    def planted_ips(self) -> np.ndarray:
        return self.ip[self.cfg.n_hosts:]

    def window_pool(self) -> np.ndarray:
        """Every host's whole peer pool: the distinct pairs of a full window
        (activity ranges ignored)."""
        d = self.degree
        tot = int(d.sum())
        h = np.repeat(np.arange(self.n_all), d)
        first = np.cumsum(d) - d
        p = np.arange(tot, dtype=np.int64) - np.repeat(first, d)
        return self._rows(h, p)

    def pairs_device(self, stream: int, s: int, device, n: Optional[int] = None,
                     d: Optional[np.ndarray] = None):
        """The slice's N pairs built on a torch device: the same distinct pairs
        as ``pairs``, with the repeats and the shuffle drawn by a torch Philox
        generator keyed like ``pairs`` (fast; a different but equally seeded
        arrangement).  ``d``: the slice's distinct pairs if already drawn
        (``distinct`` / ``distinct_all``).  Returns an int32 (N, 2) tensor on
        ``device``."""
        import torch
        c = self.cfg
        if d is None:
            d = self.distinct(stream, s)
        N = int(self.n_pairs[stream]) if n is None else int(n)
        D = d.shape[0]
        if D == 0 or N == 0:
            return torch.zeros((0, 2), dtype=torch.int32, device=device)
        if D > N:
            raise ValueError(f"slice {s} of stream {stream} has {D} distinct pairs > {N}")
        g = torch.Generator(device=device)
        g.manual_seed(int(_key(c.seed, _P_PERM, stream, s)) & 0x7FFFFFFFFFFFFFFF)
        dd = torch.from_numpy(d.view(np.int32)).to(device)
        rep = torch.randint(0, D, (N - D,), generator=g, device=device)
        idx = torch.cat([torch.arange(D, device=device), rep])
        perm = torch.randperm(N, generator=g, device=device)
        return dd[idx[perm]].contiguous()


# ----------------------------------------------------------------------------
# served streams

@dataclasses.dataclass
class ServedStream:
    """One stream of a serving run: detector configuration, slot length,
    Poisson batch arrivals (stream seconds) and batch sizes.  Batch j is
    rows [starts[j], starts[j] + sizes[j]) (cyclic) of the stream's reservoir,
    the shuffled distinct pairs of one full window (Trace.window_pool)."""
    cfg: TraceConfig
    slot: float
    n_slots: int
    arrivals: np.ndarray
    sizes: np.ndarray
    starts: np.ndarray
    reservoir_pairs: int

    def slot_of(self) -> np.ndarray:
        return np.floor(self.arrivals / self.slot).astype(np.int64)


def served_workload(n_streams: int = 32, seed: int = 0x55D00004, pairs_scale: float = 1.0, n_slots: int = 6,
                    mean_gap: float = 0.005, max_window_distinct: float = 4e6) -> List[ServedStream]:
    """Streams with uneven rates: slot length uniform in [50, 500] ms of stream
    time, rate weight w log-uniform in [0.2, 5], batches arriving as a Poisson
    process of mean gap mean_gap / w, batch sizes log-uniform in [64K, 4M]
    pairs (times pairs_scale); detector parameters as for batched links."""
    cfgs = batch_configs(n_streams, seed, pairs_scale=pairs_scale, max_window_distinct=max_window_distinct)
    out = []
    for i, c in enumerate(cfgs):
        key = _key(seed, 0x5E4FE, i)
        u = _uniform01(key, np.arange(2))
        slot = 0.05 + 0.45 * float(u[0])
        w = math.exp(math.log(0.2) + float(u[1]) * math.log(25.0))
        horizon = slot * n_slots
        n_max = int(horizon / (mean_gap / w) * 2 + 64)
        gaps = -np.log(_uniform01(_key(seed, 0x5E4FF, i), np.arange(n_max))) * (mean_gap / w)
        arr = np.cumsum(gaps)
        arr = arr[arr < horizon]
        lo, hi = math.log(65536 * pairs_scale), math.log(4194304 * pairs_scale)
        us = _uniform01(_key(seed, 0x5E500, i), np.arange(arr.size))
        sizes = np.maximum(64, np.exp(lo + us * (hi - lo)).astype(np.int64))
        tr_pool = int(Trace(c).degree.sum())
        starts = (np.cumsum(sizes) - sizes) % max(tr_pool, 1)
        out.append(ServedStream(cfg=c, slot=slot, n_slots=n_slots, arrivals=arr, sizes=sizes, starts=starts,
                                reservoir_pairs=tr_pool))
    return out