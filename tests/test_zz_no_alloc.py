"""The allocation-free entry point fpic_step_noalloc against the workspace
path (fpic_create + set_state + step + get_state) on the same inputs: two
calls in a row, the second on a smaller box, each bitwise equal to the
workspace path (both run the same deterministic kernels)."""
import numpy as np
import pytest
import torch

from paper_2101_02745_amd import _lib, inputs as I
from paper_2101_02745_amd._lib import HostConfig
from paper_2101_02745_amd.sim import Sim, step_noalloc

pytestmark = pytest.mark.gpu


def box(ncell, ndir, shape_order, seed):
    return I.Workload(name=f"noalloc_{ncell}x{ndir}", ncell=(1, 1, ncell),
                      length=(1.0, 1.0, 0.2 * ncell), ndir=ndir, dt=0.1, steps=0,
                      f=0.1, fbar=-0.2, nbar_over_n=1.1, seed=seed, alpha=1e-3,
                      shape_order=shape_order)


def workspace_path(w, s0, step0, nsteps):
    sim = Sim.from_workload(w)
    sim.set_state(s0, step0)
    sim.step(nsteps)
    out = sim.get_state()
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("shape_order", [1, 2])
def test_noalloc_matches_workspace_path(shape_order):
    cases = [(box(700, 64, shape_order, 11), 3, 7), (box(130, 26, shape_order, 12), 0, 5)]
    for w, step0, nsteps in cases:
        print(f"noalloc case {w.name} shape {shape_order} step0 {step0} nsteps {nsteps}",
              flush=True)
        s0 = torch.from_numpy(w.state0()).cuda()
        ref = workspace_path(w, s0, step0, nsteps)
        got = s0.clone()
        step_noalloc(HostConfig.from_workload(w), got, nsteps, step0)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (w.name, (got - ref).abs().max().item())
        assert not torch.equal(got, s0)


def test_noalloc_rejects_boxes_beyond_the_scratch():
    w = box(4096, 378, 1, 13)   # ~1.5e6 particles: far beyond 64 MiB of scratch
    cfg = HostConfig.from_workload(w)
    s = torch.zeros((18, w.ndir, w.ncell_total), dtype=torch.float64, device="cuda:0")
    with pytest.raises(_lib.FpicError, match="scratch"):
        step_noalloc(cfg, s, 1)
    assert torch.count_nonzero(s).item() == 0
