"""Served streams (continuous batching): every stream's list in every slot is
the same when the stream runs alone through its own detector and when it
runs in the mix, where its batches share group scans and its closes share
group closes with other streams -- also when a memory budget forces streams
to wait for admission."""
import numpy as np
import pytest

import paper_1803_11036_amd as ssd
import tracegen as tg
from _parity import log
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


def test_served_mix_equals_alone():
    inputs = _inputs(8, 4, 0x5EED1)
    rep = serve.serve(inputs, budget_bytes=1 << 40, time_scale=4.0)
    log(f"served: {rep.pairs} pairs in {rep.wall_s:.2f} s, {rep.scan_calls} scans, {rep.close_calls} closes, "
        f"p50 {rep.latency(50):.2f} ms p99 {rep.latency(99):.2f} ms")
    assert rep.max_scan_members > 1          # batches of several streams shared scan launches
    assert _check_equal(inputs, rep) > 0


def test_served_admission_by_memory_budget():
    inputs = _inputs(6, 3, 0x5EED2)
    sizes = sorted(serve.stream_bytes(s.params) for s in inputs)
    budget = sum(sizes[-2:])                                        # about two streams at a time
    rep = serve.serve(inputs, budget_bytes=budget, time_scale=1.0)
    assert rep.max_admitted <= 3
    assert max(rep.admit_wait_s) > 0
    _check_equal(inputs, rep)
