"""Host logic of the serving loop, on the CPU: a stream's batch j is the
sizes[j] reservoir rows from starts[j] on, taken cyclically."""
import numpy as np
import torch

from paper_1803_11036_amd.serve import StreamInput, coalesce


def _stream(R, starts, sizes):
    res = torch.arange(2 * R, dtype=torch.int32).reshape(R, 2)
    return StreamInput(params=None, tables=None, slot=1.0, n_slots=1, arrivals=np.zeros(len(sizes)),
                       sizes=np.asarray(sizes), starts=np.asarray(starts), reservoir=res)


def test_batch_rows_are_the_cyclic_reservoir_rows():
    R = 37
    starts = [0, 5, 30, 36, 74, 10, 3]
    sizes = [37, 10, 7, 2, 1, 100, 0]          # whole, inside, to the end, wrapping, start past R, several wraps, empty
    s = _stream(R, starts, sizes)
    for j, (a, n) in enumerate(zip(starts, sizes)):
        want = s.reservoir[(np.arange(n) + a) % R]
        pieces = s.pieces(j)
        assert all(p.data_ptr() >= s.reservoir.data_ptr() for p in pieces)     # views, no copies
        got = torch.cat(pieces) if pieces else s.reservoir[:0]
        assert torch.equal(got, want), f"batch {j}"
        assert torch.equal(s.batch(j), want), f"batch {j}"
        assert sum(p.shape[0] for p in pieces) == n


def test_runs_of_batches_are_the_concatenated_batches():
    """Several batches taken as runs of consecutive reservoir rows give the
    batches' rows in order (batches that follow one another in the reservoir
    join; a wrap or a jump starts a new run)."""
    R = 50
    sizes = [5, 7, 3, 40, 2, 0, 6, 60]
    starts = list(np.cumsum([0] + sizes[:-1]) % R)
    starts[6] = 11                                  # a jump
    s = _stream(R, starts, sizes)
    for j0 in range(len(sizes)):
        for j1 in range(j0, len(sizes) + 1):
            runs = s.run_pieces(j0, j1)
            want = [s.batch(j) for j in range(j0, j1)]
            want = torch.cat(want) if want else s.reservoir[:0]
            got = torch.cat(runs) if runs else s.reservoir[:0]
            assert torch.equal(got, want), (j0, j1)
            assert len(runs) <= sum(len(s.ranges(j)) for j in range(j0, j1))
    assert len(s.run_pieces(0, 4)) == 2                 # rows 0..54: one wrap
    assert coalesce([(0, 3), (3, 2), (9, 1), (10, 0), (10, 4), (2, 1)]) == [(0, 5), (9, 5), (2, 1)]
