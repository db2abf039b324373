"""The FP64 lattice sums for callers that cannot allocate (lbib_reduce_device), through the C
ABI, against the sums of lbib_reduce: the same two kernels with their partials in the
library's static scratch instead of the context's buffer, so the results agree bit for bit.
Two calls in a row on two contexts, the second on a smaller lattice, check that the scratch
keeps nothing of the first call that the second would read."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1503_06726_amd import lbib
from paper_1503_06726_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_reduce_device_equals_reduce_on_two_calls():
    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    # the first lattice is the larger (200 x 130, two species), the second smaller (64 x 64)
    cases = [W.small_tissue(n_species=2, stretch=0.9, seed=5), W.tiny_cell()]
    assert cases[1].nx * cases[1].ny < cases[0].nx * cases[0].ny
    for w, steps in zip(cases, (37, 21)):
        say(f"case {w.name}: {steps} steps, then lbib_reduce_device and lbib_reduce")
        sim = lbib.from_workload(w, stream=stream)
        sim.step(steps)
        nv = 3 + w.n_species
        before = sim.device_bytes()
        out = torch.full((nv,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()                       # the fill is done before the library writes
        sim.reduce_device(out.data_ptr())
        sim.sync()
        got = out.cpu().numpy()
        assert sim.device_bytes() == before            # nothing allocated for the context
        ref = sim.reduce()
        say(f"  device {got}\n  reduce {ref}")
        assert np.array_equal(got, ref)
        o = O.from_workload(w)
        o.step(steps)
        inv = o.invariants()
        assert abs(got[0] - inv[0]) <= 1e-6 * abs(inv[0])
        # momentum: FP32 deviations round each node's momentum at about 1e-12 here
        assert np.all(np.abs(got[1:3] - inv[1:3]) <= 1e-4 * np.abs(inv[1:3]) + 1e-11 * w.nx * w.ny)
        for s in range(w.n_species):
            assert abs(got[3 + s] - inv[3 + s]) <= 1e-5 * abs(inv[3 + s])
        sim.close()


def test_reduce_device_rejects_bad_output():
    import torch
    torch.cuda.set_device(0)
    sim = lbib.from_workload(W.tiny_cell(), stream=torch.cuda.current_stream().cuda_stream)
    host = np.zeros(4)
    with pytest.raises(lbib.LbibError) as e:
        sim.reduce_device(host.ctypes.data)
    assert e.value.status == lbib.EINVAL
    with pytest.raises(lbib.LbibError) as e:
        sim.reduce_device(0)
    assert e.value.status == lbib.EINVAL
    sim.close()
