"""Randomised GPU parity sweep of the general-placement path
(include/fpic_particles.h): seeded draws of 1D and 3D boxes, particles per
cell, random or stratified placement, direction sets, shape orders, flux
factors, matter terms, sorting intervals, starting steps and step counts,
each run on the HIP path and the CPU reference from the same inputs.
Deposits use floating-point atomics, so the comparison is at the 1e-12
normwise tolerance of every other parity test."""
import numpy as np
import pytest

from oracle import ParticleProblem
from paper_2101_02745_amd import inputs as I

from test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu

NDIRS = (6, 14, 24, 26, 92)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def draw(case):
    rng = np.random.default_rng(5000 + case)
    is3d = case % 2 == 1
    if is3d:
        ncell = tuple(int(x) for x in rng.integers(1, [7, 6, 6]))
    else:
        ncell = (1, 1, int(rng.choice([1, 2, 5, 31, 64, 97, 130])))
    dx = float(rng.uniform(0.3, 1.0))
    ndir = int(rng.choice(NDIRS))
    w = I.ParticleWorkload(
        name=f"rand{case}", ncell=ncell, length=tuple(dx * n for n in ncell),
        ppc=int(rng.integers(1, 30)), ndir=ndir, dt=float(rng.uniform(0.02, 0.4) * dx), steps=0,
        placement=str(rng.choice(["random", "stratified"])),
        nbar_over_n=float(rng.uniform(0.5, 1.5)), f=float(rng.uniform(-0.3, 0.3)),
        fbar=float(rng.uniform(-0.3, 0.3)), seed=int(rng.integers(1, 1 << 30)),
        alpha=float(10 ** rng.uniform(-4, -2)),
        vacuum=bool(rng.random() < 0.7),
        vmat=tuple(float(v) for v in rng.uniform(-0.4, 0.4, 3)) if rng.random() < 0.4 else (0.0, 0.0, 0.0),
        shape_order=int(rng.choice([1, 2])))
    return dict(w=w, sort_every=int(rng.integers(1, 6)), step0=int(rng.integers(0, 3000)),
                nsteps=int(rng.integers(1, 9)))


@pytest.mark.parametrize("case", range(24))
def test_random_particle_config(torch_dev, case):
    from paper_2101_02745_amd.particles import ParticleSim
    c = draw(case)
    w = c["w"]
    N, Nb = w.weights()
    sim = ParticleSim(w.ncell, w.dx, w.nparticles, w.hvac(), w.dt, w.shape_order, w.vmat,
                      c["sort_every"])
    P = ParticleProblem(w.ncell, w.dx, w.positions(), w.dirs(), N, Nb, w.hvac(), w.dt,
                        vmat=w.vmat, shape_order=w.shape_order)
    st = w.state0()
    sim.set_workload(w, st, c["step0"])
    sim.step(c["nsteps"])
    ref = P.step(st, c["nsteps"], n0=c["step0"])
    what = dict(ncell=w.ncell, ppc=w.ppc, ndir=w.ndir, placement=w.placement, order=w.shape_order,
                sort_every=c["sort_every"], step0=c["step0"], nsteps=c["nsteps"])
    assert_parity(sim.get_state().cpu().numpy(), ref, what=str(what))
    tot, tref = sim.flavor_totals(), P.flavor_totals(ref)
    assert np.abs(tot - tref).max() <= 1e-12 * np.abs(tref).max(), what
