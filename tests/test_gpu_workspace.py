"""Caller-owned workspaces (lbib_workspace_size, lbib_bind_workspace) through the C ABI.

Bars:
  * binding moves the state and nothing else: a simulation kept in a torch-allocated workspace
    is bit-identical to the same simulation in library memory, through moves from one
    workspace to another and back into library memory, and the old memory is no longer read;
  * a bound context holds no library allocation, and its read-backs (fields, forces, spread
    field, reductions) come through the workspace's staging area unchanged;
  * a cell set larger than the workspace's node capacity, a short, misaligned, foreign or
    overlapping workspace are refused and leave the context as it was.
"""
import sys

import numpy as np
import pytest
import torch

from paper_1503_06726_amd import lbib
from paper_1503_06726_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def buffer(nbytes):
    """Device memory from torch's allocator, with no torch work pending on it."""
    torch.cuda.synchronize()
    t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    return t


def scribble(t):
    """Overwrite memory the library must no longer use."""
    t.fill_(0xA5)
    torch.cuda.synchronize()


def assert_same(a, b, what):
    FA, FB = a.get_fields(), b.get_fields()
    for k in ("rho", "u", "phi", "xy", "mask"):
        assert np.array_equal(FA[k], FB[k]), f"{what}: field {k} differs"


def tissue(seed=2, n_cells=10, mass=False):
    w = W.small_tissue(nx=150, ny=98, n_cells=n_cells, n_species=1, seed=seed, stretch=1.1)
    if mass:                             # mass sources keep a cell map in the lattice part
        w.mass_source, w.area_alpha = 1e-4, 1e-6
        w.rest_area = np.full(n_cells, 1.2 * 150 * 98 / n_cells)
    return w


@pytest.mark.parametrize("storage,mass", [(lbib.STORAGE_FP32, False), (lbib.STORAGE_FP16, False),
                                          (lbib.STORAGE_FP32, True)])
def test_bound_state_bit_identical_through_moves(storage, mass):
    w = tissue(mass=mass)
    d = dict(w.params_dict(), storage=storage)
    say(f"case {w.name}, storage {storage}: {w.n_nodes} nodes")
    A = lbib.from_workload(w, storage=storage)
    B = lbib.from_workload(w, storage=storage)
    A.step(5)
    B.step(5)
    need = lbib.workspace_size(d, w.n_nodes)
    t1 = buffer(need)
    B.bind_workspace(t1.data_ptr(), need, owner=t1)
    assert B.device_bytes() == 0
    assert B.workspace_nodes() >= w.n_nodes
    for n in (40, 13):                   # graph periods, direct steps, a list rebuild in between
        A.step(n)
        B.step(n)
        assert_same(A, B, f"bound, +{n} steps")
    FA, AA = A.get_forces()
    FB, AB = B.get_forces()
    assert np.array_equal(FA, FB) and np.array_equal(AA, AB)
    assert np.array_equal(A.get_spread(), B.get_spread())
    assert np.array_equal(A.reduce(), B.reduce())

    # into a second workspace (larger than needed), then back into library memory
    t2 = buffer(need + 4096)
    B.bind_workspace(t2.data_ptr(), need + 4096, owner=t2)
    scribble(t1)
    A.step(21)
    B.step(21)
    assert_same(A, B, "after the move to a second workspace")
    B.bind_workspace(None)
    assert B.workspace_nodes() == -1 and B.device_bytes() > 0
    scribble(t2)
    A.step(16)
    B.step(16)
    assert_same(A, B, "back in library memory")
    A.close()
    B.close()


def test_bind_before_cells_capacity_and_source_cells():
    w = tissue(seed=4)
    d = w.params_dict()
    A = lbib.from_workload(w)
    B = lbib.Simulation(d)
    need = lbib.workspace_size(d, w.n_nodes)
    t = buffer(need)
    B.bind_workspace(t.data_ptr(), need, owner=t)
    cap = B.workspace_nodes()
    assert cap >= w.n_nodes and lbib.workspace_size(d, cap + 1) > need
    say(f"capacity {cap} nodes for {w.n_nodes}")

    # a cell set beyond the capacity is refused and changes nothing
    big = W.small_tissue(nx=150, ny=98, n_cells=30, n_species=1, seed=4)
    assert big.n_nodes > cap
    with pytest.raises(lbib.LbibError) as e:
        B.set_cells(big.offsets, big.xy)
    assert e.value.status == lbib.ENOMEM
    assert B.get_fields()["xy"].shape == (0, 2)

    B.set_cells(w.offsets, w.xy, w.rest_len, w.rest_area)
    assert B.device_bytes() == 0
    for n in (20, 17):
        A.step(n)
        B.step(n)
        assert_same(A, B, f"bound before the cells, +{n} steps")

    # source cells use the workspace's slot; NULL restores all cells
    src = (np.arange(w.n_cells) % 3 == 0).astype(np.uint8)
    for s in (src, None, 1 - src):
        A.set_source_cells(s)
        B.set_source_cells(s)
        A.step(16)
        B.step(16)
        assert_same(A, B, f"source cells {None if s is None else s.tolist()}")
    assert B.device_bytes() == 0

    # ADE-only iterations allocate their own working set for the call and leave the state bound
    ia = A.ade_steady(1e-3, 400)
    ib = B.ade_steady(1e-3, 400)
    assert ia == ib
    assert B.device_bytes() == 0
    assert_same(A, B, "after the ADE-only iterations")
    A.close()
    B.close()


def test_workspace_errors_leave_the_context_unchanged():
    w = tissue(seed=5)
    d = w.params_dict()
    A = lbib.from_workload(w)
    B = lbib.from_workload(w)
    need = lbib.workspace_size(d, w.n_nodes)
    t = buffer(need + 1024)
    host = np.zeros(need + 1024, np.uint8)
    cases = [
        ("short", t.data_ptr(), need - 256, lbib.ENOMEM),
        ("misaligned", t.data_ptr() + 128, need, lbib.EINVAL),
        ("host memory", host.ctypes.data, need, lbib.EINVAL),
        ("past its allocation", t.data_ptr(), 1 << 50, lbib.EINVAL),
    ]
    for name, ptr, n, status in cases:
        with pytest.raises(lbib.LbibError) as e:
            B.bind_workspace(ptr, n)
        assert e.value.status == status, name
        assert B.workspace_nodes() == -1, name
    assert B.L.lbib_bind_workspace(B.h, None, 16) == lbib.EINVAL      # NULL with a size

    B.bind_workspace(t.data_ptr(), need + 1024, owner=t)
    u = buffer(2 * need)
    with pytest.raises(lbib.LbibError) as e:          # overlaps the bound workspace
        B.bind_workspace(t.data_ptr() + 512, need)
    assert e.value.status == lbib.EINVAL
    batch = lbib.Batch([B])
    with pytest.raises(lbib.LbibError) as e:          # adopted by a batch
        B.bind_workspace(u.data_ptr(), 2 * need, owner=u)
    assert e.value.status == lbib.ESTATE
    batch.step(16)
    batch.sync()
    batch.close()
    A.step(16)
    assert_same(A, B, "after the refused calls and a batched period")
    B.bind_workspace(u.data_ptr(), 2 * need, owner=u)
    A.step(9)
    B.step(9)
    assert_same(A, B, "after the move")
    A.close()
    B.close()
