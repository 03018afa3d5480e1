"""3D boxes whose x-rows are longer than a wave (nx > 64), both shape
orders, against the CPU reference.

The paper decomposes the domain into blocks of any size (Sec. II.C,
Fig. 1); on the GPU a row of more than 64 cells is cut into segments of
63 cells (linear shape) or 62 (quadratic), each wave holding its segment
plus the halo lanes that supply the neighbour in x.  The cases put
segment boundaries everywhere the x stencils can meet them: rows of one
segment and one cell (65), of whole segments (124, 126), one cell past
them (127), the 130 x 8 x 6 box from a strongly perturbed state, rows
that are the whole box (300 x 1 x 1), late start steps where every
direction's shift has wrapped the box, and direction groups split over
several workgroups."""
import dataclasses

import numpy as np
import pytest

from oracle import Problem
from paper_2101_02745_amd import inputs as I

from test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def box(ncell, ndir, shape_order, alpha=0.05, seed=5):
    return I.Workload(name="long", ncell=ncell, length=tuple(0.5 * n for n in ncell), ndir=ndir,
                      dt=0.1, steps=0, f=0.1, fbar=-0.2, nbar_over_n=1.2,
                      nhat=(0.5, 0.0, 0.8660254037844386), seed=seed, alpha=alpha,
                      shape_order=shape_order)


CASES = [
    ((130, 8, 6), 26, None, 2),
    ((130, 8, 6), 26, {"waves": 2, "dirs_per_wave": 3}, 777),
    ((65, 3, 2), 26, None, 2),
    ((124, 3, 2), 92, {"waves": 4, "dirs_per_wave": 7}, 41),
    ((126, 2, 3), 26, None, 2),
    ((127, 2, 2), 92, None, 333),
    ((200, 1, 3), 26, None, 2),     # one-cell axis in y
    ((300, 1, 1), 26, {"waves": 1, "dirs_per_wave": 2}, 5000),
]


@pytest.mark.parametrize("shape_order", [1, 2])
@pytest.mark.parametrize("ncell,ndir,tuning,step0", CASES)
def test_long_rows(torch_dev, ncell, ndir, tuning, step0, shape_order):
    from paper_2101_02745_amd.sim import Sim
    w = box(ncell, ndir, shape_order)
    s0 = w.state0()
    print(f"long rows {ncell} x {ndir}, shape {shape_order}, step0 {step0}, tuning {tuning}",
          flush=True)
    sim = Sim.from_workload(w, tuning=tuning)
    sim.set_state(s0, step0=step0)
    sim.step(4)
    got = sim.get_state().cpu().numpy()
    P = Problem.from_workload(w)
    ref = P.step(s0, 4, n0=step0)
    assert_parity(got, ref, what=f"{ncell} shape {shape_order}")
    mom = sim.moments().cpu().numpy()
    mref = P.moments(ref, (step0 + 4) * w.dt)
    assert np.abs(mom - mref).max() <= 1e-12 * np.abs(mref).max()
    tot = sim.flavor_totals()
    assert np.abs(tot - P.flavor_totals(ref)).max() <= 1e-12 * np.abs(tot).max()
    assert sim.check(1e-12) < 1e-13
    # run to run: bitwise the same
    sim2 = Sim.from_workload(w, tuning=tuning)
    sim2.set_state(s0, step0=step0)
    sim2.step(4)
    assert np.array_equal(sim2.get_state().cpu().numpy(), got)


def test_long_rows_take_the_separate_kernels(torch_dev):
    """A request for the fused linear stages on a box with nx > 64 runs the
    separate particle and deposit kernels: bitwise the same result."""
    from paper_2101_02745_amd.sim import Sim
    w = box((130, 8, 6), 26, 1)
    s0 = w.state0()
    out = []
    for fused in (1, 2):
        sim = Sim.from_workload(w, tuning={"fused": fused})
        sim.set_state(s0, step0=2)
        sim.step(3)
        out.append(sim.get_state().cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_long_rows_conserve_lepton_number(torch_dev):
    """Without the vacuum term sum_p (N rho - Nbar rhobar^*) is a linear
    invariant of the flow (Sec. II.A): 200 steps of a 257 x 4 x 4 box with
    92 directions, both shapes."""
    from paper_2101_02745_amd.sim import Sim
    for so in (1, 2):
        w = dataclasses.replace(box((257, 4, 4), 92, so, alpha=1e-3), vacuum=False)
        sim = Sim.from_workload(w)
        sim.set_state(w.state0())

        def lepton():
            t = sim.flavor_totals()
            lm = t[0].copy()
            lm[:3] -= t[1][:3]
            lm[3::2] -= t[1][3::2]
            lm[4::2] += t[1][4::2]
            return lm

        N, Nb = w.weights()
        scale = (np.abs(N).sum() + np.abs(Nb).sum()) * w.ncell_total
        l0 = lepton()
        sim.step(200)
        assert np.abs(lepton() - l0).max() <= 1e-13 * scale, so
        assert sim.check(1e-12) < 1e-13
