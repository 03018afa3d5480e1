"""Checkpoint and resume: the state read out with get_state after k steps,
handed to a fresh context with set_state at step0 = k (the step counter
fixes the time, and with it every particle's position), continues bitwise
as the uninterrupted run does.  The deposits are summed in a fixed order
(lattice paths) or exactly (general placement), so nothing in a resumed
run depends on how the first part was run: a restart from the last
checkpoint is the recovery path after a failed check (NaN or trace drift)."""
import dataclasses

import numpy as np
import pytest

from paper_2101_02745_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.mark.parametrize("name,shape,tuning,k,n", [
    ("1d_2048x378", 1, None, 7, 20),
    ("1d_2048x378", 2, {"waves": 2, "dirs_per_wave": 5, "steps_per_graph": 3}, 5, 13),
    ("1d_32x26", 1, {"steps_per_graph": 1}, 1, 200),
])
def test_resume_1d(torch_dev, name, shape, tuning, k, n):
    from paper_2101_02745_amd.sim import Sim
    w = dataclasses.replace(I.workload(name), shape_order=shape)
    full = Sim.from_workload(w, tuning=tuning)
    full.set_state(w.state0(), 3)
    full.step(n)
    ref = full.get_state().cpu().numpy()
    assert full.step_index() == 3 + n
    first = Sim.from_workload(w, tuning=tuning)
    first.set_state(w.state0(), 3)
    first.step(k)
    ckpt, at = first.get_state().clone(), first.step_index()
    assert at == 3 + k
    resumed = Sim.from_workload(w, tuning=tuning)
    resumed.set_state(ckpt, at)
    resumed.step(n - k)
    assert resumed.step_index() == 3 + n
    assert np.array_equal(resumed.get_state().cpu().numpy(), ref)


@pytest.mark.parametrize("shape", [1, 2])
def test_resume_3d(torch_dev, shape):
    """A 48 x 40 x 36 box with 92 directions (fused linear stages, or the
    separate quadratic kernels)."""
    from paper_2101_02745_amd.sim import Sim
    w = I.Workload(name="r3", ncell=(48, 40, 36), length=(48.0, 40.0, 36.0), ndir=92, dt=0.2,
                   steps=0, f=0.1, fbar=-0.2, nbar_over_n=1.2, nhat=(0.5, 0.0, 0.8660254037844386),
                   seed=9, alpha=1e-3, shape_order=shape)
    full = Sim.from_workload(w)
    full.set_state(w.state0())
    full.step(9)
    ref = full.get_state().cpu().numpy()
    del full
    first = Sim.from_workload(w)
    first.set_state(w.state0())
    first.step(4)
    ckpt = first.get_state().clone()
    del first
    resumed = Sim.from_workload(w)
    resumed.set_state(ckpt, 4)
    resumed.step(5)
    assert np.array_equal(resumed.get_state().cpu().numpy(), ref)


def test_resume_batch(torch_dev):
    """Eight uneven boxes of the batch workload: one box resumed at step 6
    inside a fresh batch, the others restarted from their initial states at
    step 0, every box bitwise as in the uninterrupted batch."""
    from paper_2101_02745_amd.sim import Batch
    from paper_2101_02745_amd._lib import HostConfig
    ws = I.batch_workloads(nsim=8, steps=0)
    cfgs = [HostConfig.from_workload(w) for w in ws]
    tune = {"waves": 4, "dirs_per_wave": 4, "steps_per_graph": 4}
    full = Batch(cfgs, tuning=tune)
    for i, w in enumerate(ws):
        full.set_state(i, w.state0())
    full.step(6)
    mid = full.get_state(3).clone()
    full.step(6)
    ref = [full.get_state(i).cpu().numpy() for i in range(8)]
    full.close()
    # box 3 resumed from step 6; the others run their 12 steps again, but the
    # batch steps every box together, so they start 6 steps earlier
    b = Batch(cfgs, tuning=tune)
    for i, w in enumerate(ws):
        if i == 3:
            b.set_state(i, mid, 6)
        else:
            b.set_state(i, w.state0(), 0)
    b.step(6)
    assert np.array_equal(b.get_state(3).cpu().numpy(), ref[3])
    b.step(6)
    for i in range(8):
        if i != 3:
            assert np.array_equal(b.get_state(i).cpu().numpy(), ref[i]), i
    b.close()


def test_resume_general_placement(torch_dev):
    """The 3D random box (exact deposit sums): the state after 5 steps,
    handed back with the positions at t = 0 and step0 = 5, continues bitwise;
    the resumed context sorts its particles afresh, which exact sums make
    irrelevant."""
    from paper_2101_02745_amd.particles import ParticleSim
    w = I.particle_workload("3d_32x92_random")
    N, Nb = w.weights()
    pos, dirs, s0 = w.positions(), w.dirs(), w.state0()
    full = ParticleSim.from_workload(w, sort_every=3)
    full.set(pos, dirs, N, Nb, s0)
    full.step(9)
    ref = full.get_state().cpu().numpy()
    full.close()
    first = ParticleSim.from_workload(w, sort_every=3)
    first.set(pos, dirs, N, Nb, s0)
    first.step(5)
    ckpt = first.get_state().cpu().numpy()
    first.close()
    resumed = ParticleSim.from_workload(w, sort_every=3)
    resumed.set(pos, dirs, N, Nb, ckpt, 5)
    resumed.step(4)
    assert np.array_equal(resumed.get_state().cpu().numpy(), ref)
    resumed.close()
