"""Shared driver of the GPU parity tests: run the HIP detector (through the C
ABI) and the CPU oracle over the same seeded slices and compare every product
the paper's method defines."""
from __future__ import annotations

import sys
from typing import Callable, List, Optional, Sequence

import numpy as np
import torch

import oracle
import paper_1803_11036_amd as ssd

EST_RTOL = 1e-6   # relative tolerance on the f64 estimate (Eq. 1)


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def make_pair(q, r, delta, eta, k, theta, tables, key_bits=32, rehash=False, max_tuples=1 << 20,
              max_results=1 << 18, cell_bits=8):
    p = ssd.make_params(q=q, r=r, delta=delta, eta=eta, k=k, theta=theta, key_bits=key_bits,
                        verify_rehash=rehash, max_tuples=max_tuples, max_results=max_results,
                        cell_bits=cell_bits)
    g = ssd.init_detector(p, tables, device="cuda:0")
    o = oracle.RSEA(q, r, delta, eta, k, theta, tables, key_bits=key_bits, verify_rehash=rehash)
    return g, o


def to_dev(pairs: np.ndarray) -> torch.Tensor:
    a = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
    return torch.from_numpy(a.view(np.int32)).to("cuda:0")


def scan_both(g, o, pairs: np.ndarray, t: int, splits: int = 1) -> None:
    o.scan(pairs)
    if pairs.shape[0] == 0:
        ssd.scan_slice(g, to_dev(pairs), t)
        return
    for chunk in np.array_split(pairs, splits):
        ssd.scan_slice(g, to_dev(chunk), t)


def compare_state(g, o, sample_se: Optional[np.ndarray] = None) -> None:
    can = ssd.read_canonical_state(g)
    eta = g.params.eta
    if sample_se is None:
        got = can.cpu().numpy().view(np.uint16).reshape(o.r, -1, eta)
        want = o.canonical()
        if not np.array_equal(got, want):
            bad = np.argwhere(got != want)
            raise AssertionError(f"canonical state differs at {len(bad)} cells, first {bad[:5].tolist()}: "
                                 f"gpu {got[tuple(bad[0])]} oracle {want[tuple(bad[0])]}")
    else:
        idx = torch.from_numpy(sample_se.astype(np.int64)).to(can.device)
        got = can.view(-1, eta).index_select(0, idx).cpu().numpy().view(np.uint16)
        dr = o.dr().reshape(-1, eta)[sample_se]
        want = np.where(dr < o.k, dr, 0xFFFF).astype(np.uint16)
        assert np.array_equal(got, want), "canonical state differs on sampled estimators"
    del can


def close_both(g, o, check_internals: bool = True):
    res = ssd.close_slice(g)
    o.reconstruct()
    ip, rk, est = o.results()
    assert np.array_equal(res["ip"], ip), f"ip lists differ: gpu {len(res)} oracle {len(ip)}"
    assert np.array_equal(res["rk"], rk), "R values differ"
    if len(ip):
        assert np.all(np.abs(res["est"] - est) <= EST_RTOL * np.abs(est)), "estimates differ"
    if check_internals:
        assert np.array_equal(ssd.read_rk(g), o.rk()), "R_k arrays differ"
        for i, (a, b) in enumerate(zip(ssd.read_hot(g), o.hse())):
            assert np.array_equal(a, b), f"HSE({i}) differs"
        gt = ssd.read_tuples(g)
        ot = o.tuples()
        gs = gt[np.lexsort(gt.T[::-1])] if len(gt) else gt
        os_ = ot[np.lexsort(ot.T[::-1])] if len(ot) else ot
        assert gs.shape == os_.shape and np.array_equal(gs, os_), \
            f"candidate tuples differ: gpu {len(gt)} oracle {len(ot)}"
    o.age()
    return res
