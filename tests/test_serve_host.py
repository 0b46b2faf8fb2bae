"""Host logic of the serving loop, on the CPU: a stream's batch j is the
sizes[j] reservoir rows from starts[j] on, taken cyclically."""
import numpy as np
import torch

from paper_1803_11036_amd.serve import StreamInput


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
