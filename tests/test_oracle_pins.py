"""Pins of the CPU oracle against facts that do not come from the oracle itself:
published generator vectors, the paper's worked examples, closed forms,
invariants, brute force over small key spaces and linear-counting statistics.
All run on the CPU.
"""
import itertools
import math
import os
import threading

import numpy as np
import pytest

import oracle
import tracegen as tg
from oracle import truth

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return [l.strip() for l in f if l.strip() and not l.startswith("#")]


def _tables(seed=1):
    return tg.hash_tables(seed)


# ---------------------------------------------------------------- hashing

def test_splitmix64_published_vectors():
    lines = _gold("splitmix64.txt")
    assert lines[0] == "seed 0"
    want = [int(v, 16) for v in lines[1:]]
    got = [int(v) for v in tg.splitmix64(0, len(want))]
    assert got == want


def test_table_vectors():
    t = _tables(1)
    for line in _gold("hash_vectors.txt"):
        if line.startswith("tables"):
            _, which, *vals = line.split()
            idx = 0 if which.startswith("T0") else 1
            assert [int(v) for v in t[idx, 0, :4]] == [int(v, 16) for v in vals]


def test_rhfg_h1_vectors():
    t = _tables(1)
    n = 0
    for line in _gold("hash_vectors.txt"):
        if ":" not in line:
            continue
        geo, rest = line.split(":")
        q, r, delta, eta = map(int, geo.split())
        cols, h1 = rest.split(";")
        # small estimators keep the state small: eta only masks H1
        o = oracle.RSEA(q, r, delta, 64, 4, 1024, t)
        assert o.rhfg(0xC0A80001) == [int(v) for v in cols.split()]
        o = oracle.RSEA(12, 6, 5, eta, 4, 1024, t)
        assert o.h1(0x08080808) == int(h1)
        n += 1
    assert n == 3


def _bit_window(x, start, width):
    """Bits start..start+width-1 of a 32-bit value, one bit at a time."""
    v = 0
    for b in range(width):
        pos = start + b
        if pos < 32 and (x >> pos) & 1:
            v |= 1 << b
    return v


@pytest.mark.parametrize("q,r,delta", [(12, 6, 5), (14, 5, 6), (16, 6, 4), (10, 5, 8)])
def test_B_is_a_window_of_host_bits(q, r, delta):
    """Eq. 3: RHFG[i] XOR RHFG[0] is q consecutive host bits (reading R1: from
    bit (i-1)*delta), and the windows together cover all 32 bits."""
    o = oracle.RSEA(q, r, delta, 64, 4, 64, _tables(7))
    rng = np.random.default_rng(3)
    for cip in rng.integers(0, 2 ** 32, 300, dtype=np.uint64):
        cip = int(cip)
        cols = o.rhfg(cip)
        for i in range(1, r):
            assert cols[i] ^ cols[0] == _bit_window(cip, (i - 1) * delta, q)
    covered = set()
    for i in range(1, r):
        covered |= set(range((i - 1) * delta, (i - 1) * delta + q))
    assert set(range(32)) <= covered


def test_literal_shift_reading_is_not_invertible():
    """With the shift read literally as i*delta (i = 1..r-1) the low delta bits
    never enter any B(i): two hosts differing only there are indistinguishable,
    which is why the oracle and the GPU take the (i-1)*delta reading."""
    q, r, delta = 14, 5, 6
    for cip in (0xC0A80001, 0x12345678):
        a = [(cip >> (i * delta)) & ((1 << q) - 1) for i in range(1, r)]
        b = [((cip ^ 0x3F) >> (i * delta)) & ((1 << q) - 1) for i in range(1, r)]
        assert a == b


def test_roundtrip_exhaustive_paper_geometry():
    """Every one of the 2^32 hosts passes its own overlap tests and extracts
    back to itself under the paper's geometry q=14, r=5, delta=6 (Sec. 5)."""
    o = oracle.RSEA(14, 5, 6, 64, 4, 64, _tables(1))
    nthreads = min(8, os.cpu_count() or 1)
    step = (1 << 32) // nthreads
    bad = [None] * nthreads

    def work(j):
        bad[j] = o.roundtrip_failures(j * step, (j + 1) * step if j < nthreads - 1 else 1 << 32)

    th = [threading.Thread(target=work, args=(j,)) for j in range(nthreads)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert sum(bad) == 0


@pytest.mark.parametrize("q,r,delta", [(12, 6, 5), (16, 6, 4), (10, 5, 8)])
def test_roundtrip_sampled(q, r, delta):
    o = oracle.RSEA(q, r, delta, 64, 4, 64, _tables(5))
    assert o.roundtrip_failures(0, 1 << 32, stride=4099) == 0


# ---------------------------------------------------------- worked examples

def test_precise_example():
    lines = _gold("precise_example.txt")
    pairs = [tuple(map(int, p.split(":"))) for p in lines[0].split()[1:]]
    want = int(lines[1].split()[1])
    assert truth.precise_count(pairs) == {7: want}
    hosts, counts = truth.opposite_numbers([np.array(pairs, dtype=np.uint32)])
    assert list(hosts) == [7] and list(counts) == [want]


def _parse_window_example():
    d = {}
    for line in _gold("window_example.txt"):
        key, *vals = line.split()
        d[key] = [int(v) for v in vals]
    return d


def test_window_example_truth():
    """Def. 4 example on exact counts: theta peers only in S5, k = 5."""
    ex = _parse_window_example()
    k, s5 = ex["k"][0], ex["active_slot"][0]
    theta = 50
    host = 0x0A000001
    slices = []
    for s in range(12):
        if s == s5:
            p = np.array([[host, 1000 + j] for j in range(theta)], dtype=np.uint32)
        else:
            p = np.array([[0x0B000000 + s, 5]], dtype=np.uint32)
        slices.append(p)
    reported = [t for t in range(12) if host in truth.window_super_points(slices, t, k, theta)]
    assert reported == ex["reported_at_close"]
    assert [t - k + 1 for t in reported] == ex["windows_start"]


def test_window_example_method():
    """The same example through the sliding estimators: the host is regained at
    the closes of slots 5..9 only (peers well above theta so that the
    estimate clears the threshold)."""
    ex = _parse_window_example()
    k, s5 = ex["k"][0], ex["active_slot"][0]
    o = oracle.RSEA(12, 6, 5, 1024, k, 100, _tables(2))
    host = 0x0A000001
    reported = []
    for s in range(12):
        if s == s5:
            o.scan(np.array([[host, 7000 + j] for j in range(600)], dtype=np.uint32))
        ip, rk, est = o.close()
        if host in ip:
            reported.append(s)
    assert reported == ex["reported_at_close"]


# -------------------------------------------------- threshold and estimate

@pytest.mark.parametrize("eta,theta,T", [(1024, 1024, 648), (4096, 1024, 907), (4096, 2048, 1612),
                                         (2048, 1024, 806), (1024, 512, 403), (2048, 2048, 1295),
                                         (4096, 4096, 2590), (8192, 8192, 5179)])
def test_threshold_is_the_inverse_of_eq1(eta, theta, T):
    """The hot threshold is the smallest R whose Eq. 1 estimate reaches theta:
    this ties the Sec. 3.3 threshold formula to Eq. 1 without retyping it."""
    o = oracle.RSEA(12, 6, 5, eta, 4, theta, _tables(1))
    assert o.T == T
    est = oracle.estimate(eta, np.array([T - 1, T]))
    assert est[1] >= theta - 1e-9 and est[0] < theta


def test_estimate_special_values():
    eta = 4096
    e = oracle.estimate(eta, np.array([0, 1, eta - 1, eta]))
    assert e[0] == 0.0
    assert abs(e[1] - 1.0) < 1e-3                 # one set bit ~ one peer
    assert e[2] == pytest.approx(eta * math.log(eta))
    assert e[3] == e[2]                           # saturation clamps z0 at 1 (R6)
    R = np.arange(eta + 1)
    assert np.all(np.diff(oracle.estimate(eta, R)[:-1]) > 0)


def test_linear_counting_mean():
    """One host with n distinct peers fills eta(1-(1-1/eta)^n) DRs on average
    (linear counting); statistical check over many hosts."""
    eta, n, H = 1024, 700, 300
    o = oracle.RSEA(14, 4, 9, eta, 2, 100, _tables(11), key_bits=32)
    rng = np.random.default_rng(4)
    hosts = rng.choice(2 ** 32, H, replace=False).astype(np.uint32)
    pairs = []
    for h in hosts:
        peers = rng.choice(2 ** 32, n, replace=False).astype(np.uint32)
        pairs.append(np.stack([np.full(n, h, np.uint32), peers], 1))
    o.scan(np.concatenate(pairs))
    cols = np.array([o.rhfg(int(h))[0] for h in hosts])
    uniq, cnt = np.unique(cols, return_counts=True)
    solo = np.isin(cols, uniq[cnt == 1])
    R = (o.dr()[0, cols[solo]] < o.k).sum(axis=1).astype(np.float64)
    p = (1 - 1 / eta) ** n
    mean = eta * (1 - p)
    var = eta * (eta - 1) * (1 - 2 / eta) ** n + eta * p - (eta * p) ** 2
    assert abs(R.mean() - mean) < 4 * math.sqrt(var / R.size)


# ----------------------------------------------------- state closed form

def _np_tab_hash(t, x):
    x = x.astype(np.uint32)
    return (t[0][x & 255] ^ t[1][(x >> 8) & 255] ^ t[2][(x >> 16) & 255] ^ t[3][x >> 24])


def test_state_closed_form():
    """P5: after the scans of slot t the canonical cell (i, c, d) equals
    t - (latest slot of a pair mapping to it within the window), else 0xFFFF.
    Computed here by a vectorised forward formula over the window's pairs."""
    q, r, delta, eta, k = 10, 5, 8, 64, 3
    t_all = _tables(9)
    o = oracle.RSEA(q, r, delta, eta, k, 40, t_all)
    rng = np.random.default_rng(1)
    hosts = rng.integers(0, 2 ** 32, 300, dtype=np.uint64).astype(np.uint32)
    last = np.full((r, 1 << q, eta), -1, dtype=np.int64)
    for t in range(9):
        n = int(rng.integers(0, 4000))
        p = np.stack([rng.choice(hosts, n), rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)], 1)
        o.scan(p)
        h0 = _np_tab_hash(t_all[0], p[:, 0]) & ((1 << q) - 1)
        d = _np_tab_hash(t_all[1], p[:, 1]) & (eta - 1)
        for i in range(r):
            col = h0 if i == 0 else ((p[:, 0] >> np.uint32((i - 1) * delta)) ^ h0) & ((1 << q) - 1)
            last[i, col.astype(np.int64), d.astype(np.int64)] = t
        age = np.where(last >= 0, t - last, 1 << 20)
        want = np.where(age < k, age, 0xFFFF).astype(np.uint16)
        assert np.array_equal(o.canonical(), want), f"slot {t}"
        o.close()


def test_aging_invariants():
    """Per cell: a DR set in slot s counts in R_k exactly at the closes of
    slots s..s+k-1 (an unexpired cell is never lost, an expired one never
    counts), and DRs saturate at 65535."""
    q, r, delta, eta, k = 8, 4, 4, 64, 4
    o = oracle.RSEA(q, r, delta, eta, k, 10, _tables(3), key_bits=16)
    o.scan(np.array([[0x1234, 99]], dtype=np.uint32))
    cols = o.rhfg(0x1234)
    seen = []
    for s in range(10):
        o.reconstruct()
        seen.append(int(o.rk()[0, cols[0]]))
        o.age()
    assert seen == [1] * k + [0] * (10 - k)
    dr = o.dr()
    assert dr.max() == 65535 and dr.min() == 10


# ------------------------------------------------ order, batching, merge

def _rand_slices(rng, n_slices, hosts, heavy, n_per):
    out = []
    for s in range(n_slices):
        bg = np.stack([rng.choice(hosts, n_per), rng.integers(0, 2 ** 32, n_per, dtype=np.uint64).astype(np.uint32)], 1)
        hv = np.concatenate([np.stack([np.full(400, h, np.uint32),
                                       rng.integers(0, 2 ** 32, 400, dtype=np.uint64).astype(np.uint32)], 1)
                             for h in heavy])
        out.append(np.concatenate([bg, hv]).astype(np.uint32))
    return out


def test_order_and_batching_independence():
    """P6: updates commute and are idempotent (Sec. 3.3, Sec. 4.1), so shuffled
    and re-batched pair streams give identical state and identical results."""
    q, r, delta, eta, k, theta = 12, 6, 5, 1024, 3, 300
    rng = np.random.default_rng(8)
    hosts = rng.integers(0, 2 ** 32, 2000, dtype=np.uint64).astype(np.uint32)
    slices = _rand_slices(rng, 5, hosts, hosts[:6], 20000)
    a = oracle.RSEA(q, r, delta, eta, k, theta, _tables(4))
    b = oracle.RSEA(q, r, delta, eta, k, theta, _tables(4))
    for p in slices:
        a.scan(p)
        pp = p[rng.permutation(p.shape[0])]
        pp = np.concatenate([pp, pp[:1000]])           # repeats are idempotent
        for chunk in np.array_split(pp, 7):
            b.scan(chunk)
        assert np.array_equal(a.dr(), b.dr())
        ra, rb = a.close(), b.close()
        for x, y in zip(ra, rb):
            assert np.array_equal(x, y)
    assert len(ra[0]) >= 6


def test_merge_equals_union():
    """P7 (Alg. 5 with reading R3): merging per-router states gives the state
    of one detector that scanned every router's pairs; the merge is
    commutative and idempotent; a host below theta at every router but above
    it overall is regained only after the merge."""
    q, r, delta, eta, k, theta = 12, 6, 5, 1024, 3, 300
    tabs = _tables(6)
    rng = np.random.default_rng(12)
    hosts = rng.integers(0, 2 ** 32, 3000, dtype=np.uint64).astype(np.uint32)
    split_host = np.uint32(0x0A0B0C0D)
    nR = 4
    routers = [oracle.RSEA(q, r, delta, eta, k, theta, tabs) for _ in range(nR)]
    union = oracle.RSEA(q, r, delta, eta, k, theta, tabs)
    glob = oracle.RSEA(q, r, delta, eta, k, theta, tabs)
    glob2 = oracle.RSEA(q, r, delta, eta, k, theta, tabs)
    for s in range(5):
        allp = []
        for j in range(nR):
            bg = np.stack([rng.choice(hosts, 8000),
                           rng.integers(0, 2 ** 32, 8000, dtype=np.uint64).astype(np.uint32)], 1)
            # 60 new peers per router per slot: 180 per router window (< theta),
            # 720 over the union of the routers
            sp = np.stack([np.full(60, split_host, np.uint32),
                           rng.integers(0, 2 ** 32, 60, dtype=np.uint64).astype(np.uint32)], 1)
            p = np.concatenate([bg, sp]).astype(np.uint32)
            routers[j].scan(p)
            allp.append(p)
        union.scan(np.concatenate(allp))
        glob.merge_from(routers)
        glob2.merge_from(list(reversed(routers)) + routers[:2])
        assert np.array_equal(glob.canonical(), union.canonical())
        assert np.array_equal(glob.dr(), glob2.dr())
        rg, ru = glob.close(), union.close()
        glob2.close()
        for x, y in zip(rg, ru):
            assert np.array_equal(x, y)
        per_router = [routers[j].close() for j in range(nR)]
        if s >= 2:
            assert split_host in rg[0]
            assert all(split_host not in pr[0] for pr in per_router)


# --------------------------------------------------- reconstruction

def _small_detector(key_bits, rehash, seed, n_heavy=25, n_bg=None):
    geo = {16: (8, 4, 4), 20: (10, 4, 5), 24: (12, 4, 6)}[key_bits]
    q, r, delta = geo
    if n_bg is None:
        n_bg = int(0.2 * (1 << q) * 60)     # background well below the hot load
    o = oracle.RSEA(q, r, delta, 256, 2, 60, _tables(seed), key_bits=key_bits, verify_rehash=rehash)
    rng = np.random.default_rng(seed)
    bg = np.stack([rng.integers(0, 2 ** key_bits, n_bg, dtype=np.uint64).astype(np.uint32),
                   rng.integers(0, 2 ** 32, n_bg, dtype=np.uint64).astype(np.uint32)], 1)
    heavy = rng.choice(2 ** key_bits, n_heavy, replace=False).astype(np.uint32)
    hv = np.concatenate([np.stack([np.full(150, h, np.uint32),
                                   rng.integers(0, 2 ** 32, 150, dtype=np.uint64).astype(np.uint32)], 1)
                         for h in heavy])
    o.scan(np.concatenate([bg, hv]))
    return o, heavy


@pytest.mark.parametrize("key_bits", [16, 20, 24])
def test_rehash_output_equals_bruteforce(key_bits):
    """P8: with the re-hash check the regained set equals the forward brute
    force over the whole key space (hosts whose r estimators are hot and whose
    UnionSE clears the threshold), with the same R values."""
    o, heavy = _small_detector(key_bits, True, seed=key_bits)
    o.reconstruct()
    ip, rk, _ = o.results()
    bip, brk = o.bruteforce()
    assert np.array_equal(ip, bip) and np.array_equal(rk, brk)
    assert np.isin(heavy, ip).mean() > 0.9


@pytest.mark.parametrize("key_bits", [16, 24])
def test_paper_mode_is_superset_of_bruteforce(key_bits):
    o, heavy = _small_detector(key_bits, False, seed=100 + key_bits)
    o.reconstruct()
    ip, rk, _ = o.results()
    bip, brk = o.bruteforce()
    assert np.all(np.isin(bip, ip))
    # every brute-force host is reported with at least its own tuple's R
    pos = np.searchsorted(ip, bip)
    assert np.all(rk[pos] >= brk)


def test_tuples_equal_flat_enumeration():
    """The recursive Alg. 3/4 enumeration reaches exactly the tuples of the
    flat product HSE(0) x ... x HSE(r-1) that pass every consecutive overlap
    test (reading R2) and fit the key width (R13)."""
    o, _ = _small_detector(16, False, seed=77, n_heavy=12)
    o.reconstruct()
    hs = o.hse()
    q, r, delta = o.q, o.r, o.delta
    m = (1 << (q - delta)) - 1
    want = set()
    for ct in itertools.product(*[h.tolist() for h in hs]):
        if all(((ct[0] ^ ct[i - 1]) >> delta) == ((ct[0] ^ ct[i]) & m) for i in range(2, r)):
            x = 0
            for i in range(1, r):
                x |= (ct[0] ^ ct[i]) << ((i - 1) * delta)
            if x >> 16 == 0:
                want.add(ct)
    got = set(map(tuple, o.tuples().tolist()))
    assert got == want and len(want) > 0


def test_r13_drops_wide_values():
    """With (r-2)*delta + q above the key width, tuples that would set bits
    beyond it are dropped (R13); every tuple kept extracts below 2^key_bits."""
    q, r, delta = 10, 5, 8     # covers 34 bits
    o = oracle.RSEA(q, r, delta, 256, 2, 60, _tables(21), key_bits=32)
    rng = np.random.default_rng(21)
    hv = np.concatenate([np.stack([np.full(150, h, np.uint32),
                                   rng.integers(0, 2 ** 32, 150, dtype=np.uint64).astype(np.uint32)], 1)
                         for h in rng.integers(0, 2 ** 32, 40, dtype=np.uint64).astype(np.uint32)])
    o.scan(hv)
    o.reconstruct()
    for ct in o.tuples():
        assert o.extract(ct) < 2 ** 32


# ------------------------------------------------ generator and truth

def test_generator_window_degree():
    """Always-active hosts carry exactly their planted degree in every full
    window (pool split over k chunks), up to peer collisions inside a pool."""
    cfg = tg.config("tiny")
    tr = tg.Trace(cfg)
    sl = [tr.pairs(0, s) for s in range(cfg.k + 1)]
    for t in (cfg.k - 1, cfg.k):
        hosts, counts = truth.opposite_numbers(sl[t - cfg.k + 1:t + 1])
        deg = dict(zip(tr.ip.tolist(), tr.degree.tolist()))
        for h, c in zip(hosts[:2000].tolist(), counts[:2000].tolist()):
            d = deg[h]
            assert c <= d and c >= d - max(2, d // 20000)


def test_oracle_finds_planted_super_points():
    """Accuracy sanity on the tiny trace: every planted host (2000 peers per
    window, theta 1024) is regained once the window is full."""
    cfg = tg.config("tiny")
    tr = tg.Trace(cfg)
    o = oracle.RSEA(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tg.hash_tables(cfg.hash_seed))
    for s in range(cfg.k):
        o.scan(tr.pairs(0, s))
        ip, rk, est = o.close()
    assert np.all(np.isin(tr.planted_ips(), ip))
    assert np.all(est[np.isin(ip, tr.planted_ips())] > 1024 * 0.8)


# ------------------------------------------- Eq. 1 as the C oracle reports it

def _host_with_cells(o, host, n_cells, rng):
    """Pairs (host, oip) whose cell hashes H1 cover exactly n_cells distinct
    cells (one peer per cell).  H1 is pinned by the golden vectors above."""
    seen, peers = set(), []
    while len(seen) < n_cells:
        oip = int(rng.integers(0, 2 ** 32))
        d = o.h1(oip)
        if d not in seen:
            seen.add(d)
            peers.append(oip)
    return np.array([[host, p] for p in peers], dtype=np.uint32)


def test_c_oracle_estimate_at_controlled_R():
    """A lone host whose peers fill exactly R cells: its r estimators and their
    union hold exactly those cells, so the C oracle reports R itself, and its
    Eq. 1 estimate must (i) reach theta exactly from the hot threshold T on
    (the inverse relation of Sec. 3.3), (ii) grow with R, and (iii) at
    saturation (R = eta, where Eq. 1 has ln 0) equal the estimate at
    R = eta - 1, eta * ln(eta) (reading R6: z0 at least 1)."""
    eta, theta = 1024, 700
    rng = np.random.default_rng(91)
    tabs = _tables(2)
    T = oracle.RSEA(8, 4, 4, eta, 2, theta, tabs, key_bits=16).T
    got = {}
    for R in (T - 1, T, T + 1, eta - 1, eta):
        o = oracle.RSEA(8, 4, 4, eta, 2, theta, tabs, key_bits=16, verify_rehash=True)
        o.scan(_host_with_cells(o, 0x1234, R, rng))
        ip, rk, est = o.close()
        if R < T:
            assert len(ip) == 0                      # below the hot threshold: not reported
            continue
        assert list(ip) == [0x1234] and list(rk) == [R]
        got[R] = float(est[0])
    assert got[T] >= theta and got[T] < theta + eta / (eta - T) + 1e-9
    assert got[T] < got[T + 1] < got[eta - 1]
    assert got[eta] == got[eta - 1] == pytest.approx(eta * math.log(eta), rel=1e-15)
    # the pinned Python Eq. 1 (special values, inverse of the threshold) agrees
    for R, e in got.items():
        assert e == pytest.approx(float(oracle.estimate(eta, np.array([R]))[0]), rel=4e-16)


def test_c_oracle_estimate_is_unbiased():
    """Linear counting (Sec. 3.2, Eq. 1): for hosts with n distinct peers and
    no collisions, the C oracle's estimates average n.  With eta = 4096 and
    n = 1500 one estimate has a standard deviation of about 18, so the mean of
    48 hosts lies within 15 of n; a wrong logarithm base (log10: about 650,
    log2: about 2160) or a wrong sign fails this by far."""
    eta, n, H = 4096, 1500, 48
    tabs = _tables(13)
    o = oracle.RSEA(10, 5, 8, eta, 1, 1024, tabs, verify_rehash=True)
    rng = np.random.default_rng(17)
    hosts = rng.choice(2 ** 32, H, replace=False).astype(np.uint32)
    pairs = np.concatenate([np.stack([np.full(n, h, np.uint32),
                                      rng.choice(2 ** 32, n, replace=False).astype(np.uint32)], 1)
                            for h in hosts])
    o.scan(pairs)
    ip, rk, est = o.close()
    mine = np.isin(ip, hosts)
    assert mine.sum() == H
    assert abs(est[mine].mean() - n) < 15
    # every reported estimate equals the pinned Python Eq. 1 of its R
    assert np.allclose(est, oracle.estimate(eta, rk), rtol=4e-16, atol=0)


def test_c_oracle_estimate_equals_pinned_eq1_on_trace():
    """Every host the C oracle reports on the tiny trace carries the pinned
    Eq. 1 estimate of its R."""
    cfg = tg.config("tiny")
    tr = tg.Trace(cfg)
    o = oracle.RSEA(cfg.q, cfg.r, cfg.delta, cfg.eta, cfg.k, cfg.theta, tg.hash_tables(cfg.hash_seed))
    n = 0
    for s in range(cfg.k):
        o.scan(tr.pairs(0, s))
        ip, rk, est = o.close()
        assert np.allclose(est, oracle.estimate(cfg.eta, rk), rtol=4e-16, atol=0)
        n += len(ip)
    assert n > 1000


# ------------------------------------ P8 at the paper geometry, 2^32 hosts

def _paper_geometry_state(rehash):
    """q=14, r=5, delta=6, eta=2048 (Sec. 5), theta 1024, k = 1: random
    background well below the hot load plus 40 heavy hosts of 1500 peers."""
    q, r, delta, eta, theta = 14, 5, 6, 2048, 1024
    o = oracle.RSEA(q, r, delta, eta, 1, theta, _tables(31), verify_rehash=rehash)
    rng = np.random.default_rng(31)
    n_bg = int(0.1 * (1 << q) * theta)
    bg = np.stack([rng.integers(0, 2 ** 32, n_bg, dtype=np.uint64).astype(np.uint32),
                   rng.integers(0, 2 ** 32, n_bg, dtype=np.uint64).astype(np.uint32)], 1)
    heavy = rng.choice(2 ** 32, 40, replace=False).astype(np.uint32)
    hv = np.concatenate([np.stack([np.full(1500, h, np.uint32),
                                   rng.integers(0, 2 ** 32, 1500, dtype=np.uint64).astype(np.uint32)], 1)
                         for h in heavy])
    o.scan(np.concatenate([bg, hv]))
    return o, heavy


def _bruteforce_all(o):
    """Forward brute force over all 2^32 hosts, in threads (the C routine
    releases the interpreter lock)."""
    nthreads = min(8, os.cpu_count() or 1)
    step = (1 << 32) // nthreads
    parts = [None] * nthreads

    def work(j):
        parts[j] = o.bruteforce(j * step, (j + 1) * step if j < nthreads - 1 else 1 << 32)

    th = [threading.Thread(target=work, args=(j,)) for j in range(nthreads)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


def test_rehash_output_equals_bruteforce_paper_geometry():
    """P8 at 32-bit keys and the paper's geometry: with the re-hash check the
    regained set equals the forward brute force over all 2^32 IPv4 hosts, with
    the same R values; in paper mode the regained set contains it, each
    brute-force host with at least its own R."""
    o, heavy = _paper_geometry_state(True)
    o.reconstruct()
    ip, rk, _ = o.results()
    bip, brk = _bruteforce_all(o)
    assert np.array_equal(ip, bip) and np.array_equal(rk, brk)
    assert np.isin(heavy, ip).all()
    p, _ = _paper_geometry_state(False)
    p.reconstruct()
    pip, prk, _ = p.results()
    assert np.all(np.isin(bip, pip))
    assert np.all(prk[np.searchsorted(pip, bip)] >= brk)


def test_sliding_window_truth_equals_window_recount():
    """The incremental exact truth (last slot of every distinct pair) gives,
    at every slot, the same sliding super points as counting the window's
    slots afresh (Def. 4), including early windows, pairs that leave and
    come back, and repeats."""
    rng = np.random.default_rng(3)
    for k in (1, 3, 7):
        tr = truth.SlidingWindowTruth(k, 40)
        slices = []
        for t in range(20):
            hosts = rng.integers(0, 30, 3000).astype(np.uint32)
            peers = rng.integers(0, 200, 3000).astype(np.uint32)
            p = np.stack([hosts, peers], 1)
            slices.append(p)
            got = tr.add(p)
            want = truth.window_super_points(slices, t, k, 40)
            assert np.array_equal(got, want), (k, t)
