"""GPU parity of the general-placement path (include/fpic_particles.h)
against the CPU reference with explicit particle positions: particles
anywhere in the box, any number per cell, sorted by cell inside the
library every `sort_every` steps.  The library sums deposits exactly (in
integer limbs) and the reference in particle order, so the comparison is at
the 1e-12 normwise tolerance of every other parity test, never bitwise
(bitwise run-to-run reproducibility has its own tests)."""
import numpy as np
import pytest

from oracle import ParticleProblem
from paper_2101_02745_amd import inputs as I

from test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def pair(w, sort_every=0, hvac=None):
    from paper_2101_02745_amd.particles import ParticleSim
    N, Nb = w.weights()
    H = w.hvac() if hvac is None else hvac
    sim = ParticleSim(w.ncell, w.dx, w.nparticles, H, w.dt, w.shape_order, w.vmat, sort_every)
    P = ParticleProblem(w.ncell, w.dx, w.positions(), w.dirs(), N, Nb, H, w.dt,
                        vmat=w.vmat, shape_order=w.shape_order)
    return sim, P


def run(w, nsteps, sort_every=0, step0=0, hvac=None, chunks=1):
    sim, P = pair(w, sort_every, hvac)
    st = w.state0()
    sim.set_workload(w, st, step0)
    ref = st
    for k in range(chunks):
        sim.step(nsteps)
        ref = P.step(ref, nsteps, n0=step0 + k * nsteps)
    return sim, P, sim.get_state().cpu().numpy(), ref


def small(ncell=(1, 1, 64), length=(1.0, 1.0, 12.8), ppc=16, ndir=26, order=1, placement="random",
          **kw):
    d = dict(name="p", ncell=ncell, length=length, ppc=ppc, ndir=ndir, dt=0.1, steps=0,
             placement=placement, f=0.1, fbar=-0.3, nbar_over_n=0.9, alpha=1e-3,
             shape_order=order, seed=12)
    d.update(kw)
    return I.ParticleWorkload(**d)


@pytest.mark.parametrize("sort_every", [1, 3, 4])
def test_one_and_several_steps(torch_dev, sort_every):
    w = I.particle_workload("1d_64x16_random")
    for n in (1, 7):
        _, _, got, ref = run(w, n, sort_every)
        assert_parity(got, ref, what=f"{n} steps, sort every {sort_every}")


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("ncell,ppc,placement", [((1, 1, 64), 16, "random"),
                                                 ((1, 1, 65), 3, "stratified"),
                                                 ((1, 1, 7), 40, "random"),
                                                 ((1, 1, 1), 50, "random"),
                                                 ((1, 1, 2), 9, "random"),
                                                 ((1, 1, 300), 1, "random")])
def test_ragged_boxes(torch_dev, order, ncell, ppc, placement):
    w = small(ncell=ncell, length=(1.0, 1.0, 0.2 * ncell[2]), ppc=ppc, order=order,
              placement=placement)
    _, _, got, ref = run(w, 5, sort_every=2)
    assert_parity(got, ref, what=f"{ncell} ppc {ppc} order {order}")


def test_sparse_particles_spread_over_many_cells(torch_dev):
    """Fewer particles than cells: a workgroup's 256 particles cover more
    cells than its LDS box holds, and it deposits straight to the grid."""
    w = I.ParticleWorkload(name="sparse", ncell=(1, 1, 5000), length=(1.0, 1.0, 1000.0),
                           ppc=1, ndir=26, dt=0.1, steps=0, f=0.1, fbar=-0.3, alpha=1e-3,
                           seed=3)
    # keep 715 of the 5000 particles: about one per seven cells
    from paper_2101_02745_amd.particles import ParticleSim
    keep = np.arange(0, w.nparticles, 7)
    pos, dirs = w.positions()[keep], w.dirs()[keep]
    N, Nb = w.weights()
    N, Nb = N[keep] * 7, Nb[keep] * 7
    st = w.state0()[:, keep]
    sim = ParticleSim(w.ncell, w.dx, keep.size, w.hvac(), w.dt)
    P = ParticleProblem(w.ncell, w.dx, pos, dirs, N, Nb, w.hvac(), w.dt)
    sim.set(pos, dirs, N, Nb, st)
    sim.step(6)
    assert_parity(sim.get_state().cpu().numpy(), P.step(st, 6), what="sparse")


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("ncell", [(4, 3, 5), (8, 8, 8), (3, 1, 6), (5, 2, 1)])
def test_3d_boxes(torch_dev, order, ncell):
    w = small(ncell=ncell, length=tuple(0.5 * n for n in ncell), ppc=6, ndir=26, order=order)
    _, _, got, ref = run(w, 4, sort_every=2)
    assert_parity(got, ref, what=f"3D {ncell} order {order}")


def test_matter_and_time_origin(torch_dev):
    w = small(vmat=(0.3, -0.1, 0.05), order=2)
    _, _, got, ref = run(w, 6, step0=12345)
    assert_parity(got, ref, what="matter, step0")


def test_long_run_with_sorting(torch_dev):
    """200 steps of the 64-cell box (the particles cross the box several
    times); the state is compared every 50 steps."""
    w = I.particle_workload("1d_64x16_random")
    sim, P = pair(w, sort_every=4)
    st = w.state0()
    sim.set_workload(w, st)
    ref = st
    for k in range(4):
        sim.step(50)
        ref = P.step(ref, 50, n0=50 * k)
        assert_parity(sim.get_state().cpu().numpy(), ref, what=f"after {50 * (k + 1)} steps")
    assert sim.step_index() == 200
    assert np.abs(ref - st).max() > 1e-4


def test_moments_totals_check(torch_dev):
    w = small(order=2)
    sim, P = pair(w)
    st = w.state0()
    sim.set_workload(w, st)
    sim.step(3)
    ref = P.step(st, 3)
    t = 3 * w.dt
    mom = sim.moments().cpu().numpy()
    mref = P.moments(ref, t)
    assert np.abs(mom - mref).max() <= 1e-12 * np.abs(mref).max()
    tot, tref = sim.flavor_totals(), P.flavor_totals(ref)
    assert np.abs(tot - tref).max() <= 1e-12 * np.abs(tref).max()
    assert sim.check() < 1e-13


def test_lepton_number_conserved(torch_dev):
    w = small(ncell=(1, 1, 32), length=(1.0, 1.0, 12.8), ppc=8, vacuum=False, alpha=1e-2)
    from paper_2101_02745_amd.particles import ParticleSim
    sim = ParticleSim.from_workload(w, sort_every=2)
    sim.set_workload(w)
    t0 = sim.flavor_totals()
    sim.step(300)
    t1 = sim.flavor_totals()
    L0 = t0[0] - t0[1] * np.array([1, 1, 1, 1, -1, 1, -1, 1, -1])
    L1 = t1[0] - t1[1] * np.array([1, 1, 1, 1, -1, 1, -1, 1, -1])
    N, _ = w.weights()
    assert np.abs(L1 - L0).max() < 1e-12 * np.abs(N).sum()
    assert np.abs(t1[0][1] - t0[0][1]) > 1e-6 * np.abs(N).sum()   # flavor moved


@pytest.mark.parametrize("sort_every,nsteps,chunks", [(1, 1, 2), (4, 4, 1)])
def test_full_size_box(torch_dev, sort_every, nsteps, chunks):
    """The 2048-cell box with 774,144 particles at random positions, every
    element against the reference: two steps sorting after each, and four
    steps sorting after the fourth as the benchmark does (three plain
    stage-4 launches, one sorting one)."""
    w = I.particle_workload("1d_2048x378_random")
    _, _, got, ref = run(w, nsteps, sort_every=sort_every, chunks=chunks)
    assert_parity(got, ref, what=f"1d_2048x378_random, sort every {sort_every}")


def test_rejects_bad_particles(torch_dev):
    from paper_2101_02745_amd._lib import FpicError
    from paper_2101_02745_amd.particles import ParticleSim
    w = small()
    sim = ParticleSim.from_workload(w)
    N, Nb = w.weights()
    dirs = w.dirs().copy()
    dirs[5] *= 1.01
    with pytest.raises(FpicError, match="unit vector"):
        sim.set(w.positions(), dirs, N, Nb, w.state0())
    pos = w.positions().copy()
    pos[3, 2] = np.nan
    with pytest.raises(FpicError):
        sim.set(pos, w.dirs(), N, Nb, w.state0())
    with pytest.raises(FpicError, match="before set"):
        sim.step(1)


@pytest.mark.parametrize("order", [1, 2])
def test_lattice_positions_match_lattice_path(torch_dev, order):
    """Particles placed at the cell centres with the direction table are the
    lattice workload; the general path (positions, atomics, sorting) and the
    lattice path (implicit positions, fixed-order deposit) then agree at the
    parity tolerance.  Both are compared with the reference as well."""
    import dataclasses
    from paper_2101_02745_amd.particles import ParticleSim
    from paper_2101_02745_amd.sim import Sim
    w = dataclasses.replace(I.scaled(I.workload("1d_512x128"), ncell=(1, 1, 96), ndir=26),
                            shape_order=order, alpha=1e-3)
    nd, nc = w.ndir, w.ncell_total
    z = (np.arange(nc) + 0.5) * w.dx[2]
    pos = np.zeros((nd * nc, 3))
    pos[:, 0] = pos[:, 1] = 0.5
    pos[:, 2] = np.tile(z, nd)
    dirs = np.repeat(w.dirs(), nc, axis=0)
    N, Nb = w.weights()
    st = w.state0()
    lat = Sim.from_workload(w)
    lat.set_state(st)
    lat.step(9)
    gen = ParticleSim(w.ncell, w.dx, nd * nc, w.hvac(), w.dt, order, sort_every=3)
    gen.set(pos, dirs, np.repeat(N, nc), np.repeat(Nb, nc), st.reshape(18, -1))
    gen.step(9)
    a = lat.get_state().cpu().numpy().reshape(18, -1)
    b = gen.get_state().cpu().numpy()
    assert_parity(b, a, what=f"general vs lattice, order {order}")
    ref = ParticleProblem(w.ncell, w.dx, pos, dirs, np.repeat(N, nc), np.repeat(Nb, nc),
                          w.hvac(), w.dt, shape_order=order).step(st.reshape(18, -1), 9)
    assert_parity(b, ref, what="general vs reference")
