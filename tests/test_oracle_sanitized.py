"""The CPU oracle run under AddressSanitizer and UndefinedBehaviorSanitizer.

A small C driver (tests/oracle_sanitize_driver.c) links the oracle's source
built with -fsanitize=address,undefined and drives every entry point over a
few seeded slices: scans, reconstruction, aging, the Alg. 5 merge of router
states, inspection reads, the forward brute force and the inversion round
trip.  The sanitized run must finish cleanly, its merged state must equal the
state of one detector that saw every router's pairs, and its lists must equal
those of the regular (unsanitized) oracle library on the same input.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import tracegen as tg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "oracle_sanitize_driver.c")
SRC = os.path.join(ROOT, "oracle", "rsea_oracle.c")


def _build(tmp):
    exe = os.path.join(tmp, "driver")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-o", exe, DRIVER, SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def _write_input(path, geo, tables, slices, n_routers):
    q, r, delta, eta, k, theta, key_bits, rehash = geo
    with open(path, "wb") as f:
        np.array([q, r, delta, eta, k, theta, key_bits, rehash, n_routers, len(slices)], np.uint32).tofile(f)
        np.ascontiguousarray(tables, np.uint32).tofile(f)
        for p in slices:
            np.array([p.shape[0]], np.uint64).tofile(f)
            np.ascontiguousarray(p, np.uint32).tofile(f)


def _parse(out):
    lists, equal = [], []
    lines = out.splitlines()
    i = 0
    while i < len(lines):
        _, t, n = lines[i].split()
        n = int(n)
        rows = [lines[i + 1 + j].split() for j in range(n)]
        lists.append((np.array([int(a) for a, _, _ in rows], np.uint32),
                      np.array([int(b) for _, b, _ in rows], np.uint32),
                      np.array([float(c) for _, _, c in rows], np.float64)))
        equal.append(lines[i + 1 + n] == "merged-equal 1")
        i += n + 2
    return lists, equal


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("geo,n_slices,n_per,rehash", [
    ((8, 4, 4, 256, 2, 60, 16), 4, 6000, 0),        # 16-bit keys: brute force runs every slot
    ((12, 6, 5, 1024, 3, 300, 32), 4, 40000, 0),    # IPv4 keys, paper mode
    ((10, 5, 8, 256, 2, 60, 32), 3, 8000, 1),       # (r-2)*delta + q = 34 > 32 (R13), re-hash (R14)
])
def test_oracle_under_sanitizers(tmp_path, geo, n_slices, n_per, rehash):
    q, r, delta, eta, k, theta, key_bits = geo
    tabs = tg.hash_tables(17)
    rng = np.random.default_rng(q * 100 + r)
    hosts = rng.integers(0, 2 ** key_bits, 3000, dtype=np.uint64).astype(np.uint32)
    heavy = hosts[:8]
    slices = []
    for s in range(n_slices):
        bg = np.stack([rng.choice(hosts, n_per), rng.integers(0, 2 ** 32, n_per, dtype=np.uint64).astype(np.uint32)], 1)
        hv = np.concatenate([np.stack([np.full(theta, h, np.uint32),
                                       rng.integers(0, 2 ** 32, theta, dtype=np.uint64).astype(np.uint32)], 1)
                             for h in heavy])
        p = np.concatenate([bg, hv]).astype(np.uint32)
        slices.append(p[rng.permutation(p.shape[0])])
    inp = os.path.join(tmp_path, "in.bin")
    _write_input(inp, (q, r, delta, eta, k, theta, key_bits, rehash), tabs, slices, n_routers=3)
    exe = _build(str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe, inp], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
    lists, equal = _parse(res.stdout)
    assert len(lists) == n_slices and all(equal)
    # the same lists from the regular oracle library
    o = oracle.RSEA(q, r, delta, eta, k, theta, tabs, key_bits=key_bits, verify_rehash=bool(rehash))
    reported = 0
    for p, (ip, rk, est) in zip(slices, lists):
        o.scan(p)
        wip, wrk, west = o.close()
        assert np.array_equal(ip, wip) and np.array_equal(rk, wrk)
        assert np.array_equal(est, west)
        reported += len(ip)
    assert reported > 0
