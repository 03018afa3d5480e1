"""The quadratic (triangular-shaped cloud) shape function of Sec. II.B.1 on
the 1D HIP path against the CPU reference: ragged and tiny boxes (where the
three-cell stencil folds onto itself), launch shapes, late times,
diagnostics, batches, the full-size 2048 x 378 box and the two-beam
instability."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import Problem
from paper_2101_02745_amd import inputs as I

from test_gpu_parity import TOL, assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def quad(w):
    return dataclasses.replace(w, shape_order=2)


def box(ncell, ndir, **kw):
    return quad(I.Workload(name="q", ncell=(1, 1, ncell), length=(1.0, 1.0, 0.2 * ncell),
                           ndir=ndir, dt=0.1, steps=0, f=kw.pop("f", 0.2),
                           fbar=kw.pop("fbar", -0.3), nbar_over_n=0.9, seed=kw.pop("seed", 7),
                           alpha=kw.pop("alpha", 1e-2), **kw))


def run_pair(w, nsteps, tuning=None, step0=0):
    from paper_2101_02745_amd.sim import Sim
    sim = Sim.from_workload(w, tuning=tuning)
    P = Problem.from_workload(w)
    s0 = w.state0()
    sim.set_state(s0, step0)
    sim.step(nsteps)
    return sim, P, sim.get_state().cpu().numpy(), P.step(s0, nsteps, n0=step0)


@pytest.mark.parametrize("ncell,ndir", [(1, 26), (2, 6), (3, 26), (5, 8), (63, 26), (64, 26),
                                        (65, 26), (66, 8), (129, 26), (130, 92), (200, 378)])
def test_quadratic_ragged_shapes(torch_dev, ncell, ndir):
    _, _, got, ref = run_pair(box(ncell, ndir), 6, step0=3)
    assert_parity(got, ref, what=f"quadratic {ncell}x{ndir}")


@pytest.mark.parametrize("tuning", [{"waves": 1, "dirs_per_wave": 1},
                                    {"waves": 2, "dirs_per_wave": 3},
                                    {"waves": 4, "dirs_per_wave": 5, "steps_per_graph": 3},
                                    {"waves": 8, "dirs_per_wave": 2, "steps_per_graph": 5}])
def test_quadratic_launch_shapes(torch_dev, tuning):
    w = quad(I.scaled(I.workload("1d_2048x378"), ncell=(1, 1, 150), ndir=92))
    _, _, got, ref = run_pair(w, 7, tuning=tuning)
    assert_parity(got, ref, what=str(tuning))


def test_quadratic_late_times_and_diagnostics(torch_dev):
    """Shifts that have wrapped the box many times; moments (72 per cell,
    deposited with the quadratic weights), flavor totals, trace check."""
    w = box(70, 26, seed=3)
    sim, P, got, ref = run_pair(w, 9, step0=12345)
    assert_parity(got, ref, what="late")
    mom = sim.moments().cpu().numpy()
    mref = P.moments(ref, (12345 + 9) * w.dt)
    assert np.abs(mom - mref).max() <= TOL * np.abs(mref).max()
    tot = sim.flavor_totals()
    tref = P.flavor_totals(ref)
    assert np.abs(tot - tref).max() <= TOL * np.abs(tref).max()
    assert sim.check(1e-12) < 1e-13


def test_quadratic_full_run_1d_32x26(torch_dev):
    w = quad(I.workload("1d_32x26"))
    from paper_2101_02745_amd.sim import Sim
    sim, P = Sim.from_workload(w), Problem.from_workload(w)
    s0 = w.state0()
    sim.set_state(s0)
    ref = s0
    for k in range(4):
        sim.step(50)
        ref = P.step(ref, 50, n0=50 * k)
        assert_parity(sim.get_state().cpu().numpy(), ref, what=f"after {50 * (k + 1)} steps")


def test_quadratic_full_size_1d_2048x378(torch_dev):
    w = quad(I.workload("1d_2048x378"))
    _, _, got, ref = run_pair(w, 2)
    assert_parity(got, ref, what="2048x378 quadratic")


def test_quadratic_batch_and_determinism(torch_dev):
    from paper_2101_02745_amd.sim import Batch, Sim
    from paper_2101_02745_amd._lib import HostConfig
    ws = [quad(I.scaled(w, ncell=(1, 1, 40 + 53 * i), ndir=w.ndir if w.ndir < 378 else 92))
          for i, w in enumerate(I.batch_workloads(nsim=4, steps=0))]
    tune = {"waves": 2, "dirs_per_wave": 4, "steps_per_graph": 4}
    b = Batch([HostConfig.from_workload(w) for w in ws], tuning=tune)
    for i, w in enumerate(ws):
        b.set_state(i, w.state0())
    b.step(10)
    for i, w in enumerate(ws):
        got = b.get_state(i).cpu().numpy()
        single = Sim.from_workload(w, tuning=tune)
        single.set_state(w.state0())
        for c in (3, 7):                  # a different graph chunking
            single.step(c)
        assert np.array_equal(got, single.get_state().cpu().numpy())
        assert_parity(got, Problem.from_workload(w).step(w.state0(), 10), what=f"batch {i}")


def test_quadratic_two_beam_growth_on_gpu(torch_dev):
    """Inhomogeneous two-beam instability (App. A.4) with the quadratic
    shape: growth rate 2 mu within the paper's 4.3e-3."""
    from paper_2101_02745_amd.sim import Sim
    from paper_2101_02745_amd._lib import HostConfig
    mu, k, n, dt = 1.0, 2.0, 64, 0.01
    L = 2 * math.pi / k
    dz = L / n
    hc = HostConfig((1, 1, n), (1.0, 1.0, dz), [[0, 0, 1.0], [0, 0, -1.0]],
                    [mu * dz, 0.0], [0.0, mu * dz], np.zeros((3, 3)), dt, shape_order=2)
    sim = Sim(hc)
    z0 = (np.arange(n) + 0.5) * dz
    st = np.zeros((18, 2, n))
    st[3] = st[12] = 1e-9 * np.sin(k * z0)
    st[1], st[10] = st[3] ** 2, st[12] ** 2
    st[0], st[9] = 1 - st[1], 1 - st[10]
    sim.set_state(st)
    amps = []
    for nsteps in (200, 400):
        sim.step(nsteps)
        s = sim.get_state().cpu().numpy()
        t = sim.step_index() * dt
        S = s[3, 0] + 1j * s[4, 0]
        amps.append(abs(np.sum(S * np.exp(-1j * k * (z0 + t)))) / n)
    rate = math.log(amps[1] / amps[0]) / (400 * dt)
    assert abs(rate - 2 * mu) / (2 * mu) < 4.3e-3, rate


@pytest.mark.parametrize("ncell,ndir,nsteps,ckpt,tuning", [
    (70, 26, 7, 3, None),
    (65, 8, 5, 5, {"waves": 2, "dirs_per_wave": 2}),
    (2, 26, 4, 2, None),
])
def test_quadratic_adjoint_matches_reference(torch_dev, ncell, ndir, nsteps, ckpt, tuning):
    from paper_2101_02745_amd.sim import Sim
    w = box(ncell, ndir, seed=11)
    rng = np.random.default_rng(ncell + 1)
    c = rng.normal(size=(18, ndir, ncell))
    s0 = w.state0()
    P = Problem.from_workload(w)
    g_ref, gN_ref, gNb_ref = P.adjoint(s0, nsteps, c, n0=2)
    sim = Sim.from_workload(w, tuning=tuning)
    sim.set_state(s0, step0=2)
    sim.adjoint_forward(nsteps, ckpt)
    g0, gN, gNb = sim.adjoint_backward(c)

    def normwise(a, b):
        return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max()
    assert normwise(g0.cpu().numpy(), g_ref) < 1e-10
    assert normwise(gN, gN_ref) < 1e-10
    assert normwise(gNb, gNb_ref) < 1e-10


@pytest.mark.parametrize("ncell,ndir,tuning,step0", [
    ((8, 6, 5), 26, None, 2),
    ((13, 7, 3), 26, {"waves": 2, "dirs_per_wave": 5}, 41),
    ((16, 1, 8), 26, None, 2),      # one-cell axis in y
    ((1, 12, 10), 6, None, 300),    # one-cell axis in x
    ((2, 2, 9), 92, None, 5),       # two-cell axes: the stencil folds
    ((64, 3, 4), 92, {"waves": 4, "dirs_per_wave": 7}, 333),
])
def test_quadratic_3d_parity(torch_dev, ncell, ndir, tuning, step0):
    from paper_2101_02745_amd.sim import Sim
    w = quad(I.Workload(name="q3", ncell=ncell, length=tuple(0.5 * n for n in ncell), ndir=ndir,
                        dt=0.1, steps=0, f=0.1, fbar=-0.2, nbar_over_n=1.2,
                        nhat=(0.5, 0.0, 0.8660254037844386), seed=3, alpha=1e-2))
    sim, P, got, ref = run_pair(w, 4, tuning=tuning, step0=step0)
    assert_parity(got, ref, what=f"quadratic 3D {ncell}")
    mom = sim.moments().cpu().numpy()
    mref = P.moments(ref, (step0 + 4) * w.dt)
    assert np.abs(mom - mref).max() <= 1e-12 * np.abs(mref).max()
    assert sim.check(1e-12) < 1e-13


def test_quadratic_3d_full_size_homogeneous(torch_dev):
    """The full 64^3 x 92 box with the quadratic shape, from a state that is
    the same in every cell: the weights sum to one, so the method reduces
    exactly to one cell holding the 92 directions (the reference computes
    it); every particle of the GPU run is compared with it."""
    import torch
    from paper_2101_02745_amd.sim import Sim
    w = quad(I.workload("3d_64x92"))
    one = quad(I.Workload(name="one", ncell=(1, 1, 1), length=w.dx, ndir=w.ndir, dt=w.dt, steps=0,
                          f=w.f, fbar=w.fbar, nbar_over_n=w.nbar_over_n, nhat=w.nhat, seed=7,
                          alpha=0.05))
    s1 = one.state0()
    ref = Problem.from_workload(one).step(s1, 4)
    sim = Sim.from_workload(w)
    sim.set_state(torch.from_numpy(s1).cuda().expand(18, w.ndir, w.ncell_total).contiguous())
    sim.step(4)
    got = sim.get_state()
    for k in range(18):
        dev = (got[k] - torch.from_numpy(ref[k]).cuda()).abs().max().item()
        assert dev <= 1e-12 * max(1.0, np.abs(ref).max()), (k, dev)
