"""The batched sweep's inputs (host only): every simulation of the 64-member sweep is a valid
cell set for the library's validator, its draws stay in their stated ranges, and the
generator is deterministic."""
import numpy as np

from paper_1503_06726_amd import lbib
from paper_1503_06726_amd import workloads as W


def test_sweep_members_valid_and_in_range():
    ws = [W.sweep_member(i) for i in range(W.SWEEP_SIMS)]
    for w in ws:
        s, msg = lbib.validate_cells(w.params_dict(), w.offsets, w.xy)
        assert s == lbib.OK, (w.name, msg)
        assert 128 <= w.nx <= 1024 and 128 <= w.ny <= 1024
        assert 10 <= w.n_cells <= min(max(500, 8 * max(w.nx, w.ny) // min(w.nx, w.ny) + 1), w.nx * w.ny // 100)
        assert 0.55 <= w.tau <= 1.2 and 0.005 <= w.k_spring <= 0.05
        assert w.bc_y == W.WALLS and w.species[0].reaction == W.REACT_SOURCE_DECAY
    sides = np.array([[w.nx, w.ny] for w in ws], float)
    # log-uniform draws: the log-sides spread over most of [log 128, log 1024]
    lg = np.log(sides)
    assert lg.min() < np.log(180) and lg.max() > np.log(700)


def test_sweep_member_deterministic():
    a, b = W.sweep_member(7), W.sweep_member(7)
    assert a.nx == b.nx and a.ny == b.ny and a.tau == b.tau and a.k_spring == b.k_spring
    assert np.array_equal(a.offsets, b.offsets) and np.array_equal(a.xy, b.xy)
