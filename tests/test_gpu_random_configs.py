"""Randomised parity sweep: small boxes with random sizes (1D and 3D),
direction sets (including non-symmetric ones), weights of either sign,
time steps up to the stage limit, vacuum and matter terms, shape orders,
launch shapes and starting steps, each run on the HIP path and the CPU
reference from the same inputs.  The draws are seeded, so every case is
reproducible from its index."""
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


def draw(case):
    rng = np.random.default_rng(1000 + case)
    is3d = case % 3 == 2
    if is3d:
        ncell = tuple(int(x) for x in rng.integers(1, [9, 6, 6]))
    else:
        ncell = (1, 1, int(rng.choice([1, 2, 3, 17, 64, 65, 100, 129, 191])))
    ndir = int(rng.integers(1, 40))
    v = rng.normal(size=(ndir, 3))
    dirs = v / np.linalg.norm(v, axis=1, keepdims=True)
    dx = tuple(float(x) for x in rng.uniform(0.3, 1.5, 3))
    vmax = np.abs(dirs).max(axis=0)
    lim = min(2 * dx[a] / max(vmax[a], 1e-9) for a in range(3) if ncell[a] > 1) if max(ncell) > 1 else 1.0
    dt = float(rng.uniform(0.1, 0.95) * min(lim, 0.5))
    dV = dx[0] * dx[1] * dx[2]
    N = rng.uniform(-0.3, 1.0, ndir) * dV / ndir
    Nb = rng.uniform(-0.3, 1.0, ndir) * dV / ndir
    H = I.vacuum_hamiltonian(w21=0.1, w31=0.4, delta=0.5) if rng.random() < 0.7 else np.zeros((3, 3))
    vmat = tuple(rng.uniform(-0.5, 0.5, 3)) if rng.random() < 0.5 else None
    order = int(rng.choice([1, 2]))
    tuning = None
    if rng.random() < 0.6:
        waves = int(rng.choice([1, 2, 4] if not is3d else [1, 2, 4, 8]))
        tuning = {"waves": waves, "dirs_per_wave": int(rng.integers(1, 7)),
                  "steps_per_graph": int(rng.integers(1, 6))}
    step0 = int(rng.integers(0, 5000))
    nsteps = int(rng.integers(1, 9))
    np_ = ndir * ncell[0] * ncell[1] * ncell[2]
    st = I.state_from_seeds(0.05 * rng.uniform(-1, 1, size=(8, ndir, np_ // ndir)))
    return dict(ncell=ncell, dx=dx, dirs=dirs, N=N, Nb=Nb, H=H, vmat=vmat, order=order,
                tuning=tuning, step0=step0, nsteps=nsteps, dt=dt, st=st)


@pytest.mark.parametrize("case", range(64))
def test_random_config(torch_dev, case):
    from paper_2101_02745_amd.sim import Sim
    from paper_2101_02745_amd._lib import HostConfig
    c = draw(case)
    hc = HostConfig(c["ncell"], c["dx"], c["dirs"], c["N"], c["Nb"], c["H"], c["dt"],
                    shape_order=c["order"], vmat=c["vmat"])
    P = Problem(c["ncell"], c["dx"], c["dirs"], c["N"], c["Nb"], c["H"], c["dt"],
                vmat=c["vmat"], shape_order=c["order"])
    sim = Sim(hc, tuning=c["tuning"])
    sim.set_state(c["st"], c["step0"])
    sim.step(c["nsteps"])
    ref = P.step(c["st"], c["nsteps"], n0=c["step0"])
    what = {k: c[k] for k in ("ncell", "order", "tuning", "step0", "nsteps", "dt")}
    assert_parity(sim.get_state().cpu().numpy(), ref, what=str(what))
    tot = sim.flavor_totals()
    tref = P.flavor_totals(ref)
    assert np.abs(tot - tref).max() <= 1e-12 * max(np.abs(tref).max(), 1e-300), what


@pytest.mark.parametrize("ndir", [1, 2])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("ncell", [(7, 3, 5), (64, 2, 1)])
def test_3d_few_directions(torch_dev, ndir, order, ncell):
    """3D boxes with one or two directions: the deposit's direction loop,
    which loads each next direction while it sums the current one, runs
    with no next direction (one) or a single look-ahead (two)."""
    from paper_2101_02745_amd.sim import Sim
    from paper_2101_02745_amd._lib import HostConfig
    rng = np.random.default_rng(77 + ndir + 10 * order)
    v = rng.normal(size=(ndir, 3))
    dirs = v / np.linalg.norm(v, axis=1, keepdims=True)
    dx = (0.7, 0.9, 1.1)
    dt = 0.2
    dV = dx[0] * dx[1] * dx[2]
    N = rng.uniform(0.2, 1.0, ndir) * dV
    Nb = rng.uniform(0.2, 1.0, ndir) * dV
    H = I.vacuum_hamiltonian(w21=0.1, w31=0.4, delta=0.5)
    nc = ncell[0] * ncell[1] * ncell[2]
    st = I.state_from_seeds(0.05 * rng.uniform(-1, 1, size=(8, ndir, nc)))
    hc = HostConfig(ncell, dx, dirs, N, Nb, H, dt, shape_order=order)
    P = Problem(ncell, dx, dirs, N, Nb, H, dt, shape_order=order)
    sim = Sim(hc)
    sim.set_state(st, 31)
    sim.step(5)
    ref = P.step(st, 5, n0=31)
    assert_parity(sim.get_state().cpu().numpy(), ref, what=f"{ncell} ndir {ndir} order {order}")


def draw_batch(case):
    rng = np.random.default_rng(9000 + case)
    nsim = int(rng.integers(2, 8))
    order = int(rng.choice([1, 2]))
    sims = []
    for _ in range(nsim):
        ncell = (1, 1, int(rng.choice([1, 3, 17, 64, 65, 100, 191])))
        ndir = int(rng.integers(1, 40))
        v = rng.normal(size=(ndir, 3))
        dirs = v / np.linalg.norm(v, axis=1, keepdims=True)
        dx = (1.0, 1.0, float(rng.uniform(0.3, 1.2)))
        dt = float(rng.uniform(0.1, 0.95) * min(2 * dx[2] / max(np.abs(dirs[:, 2]).max(), 1e-9), 0.5))
        N = rng.uniform(-0.3, 1.0, ndir) * dx[2] / ndir
        Nb = rng.uniform(-0.3, 1.0, ndir) * dx[2] / ndir
        H = I.vacuum_hamiltonian(w21=0.1, w31=0.4, delta=0.5) if rng.random() < 0.7 else np.zeros((3, 3))
        vmat = tuple(rng.uniform(-0.5, 0.5, 3)) if rng.random() < 0.5 else None
        st = I.state_from_seeds(0.05 * rng.uniform(-1, 1, size=(8, ndir, ncell[2])))
        sims.append(dict(ncell=ncell, dx=dx, dirs=dirs, N=N, Nb=Nb, H=H, vmat=vmat, dt=dt, st=st,
                         step0=int(rng.integers(0, 3000))))
    tuning = {"waves": int(rng.choice([1, 2, 4])), "dirs_per_wave": int(rng.integers(1, 7)),
              "steps_per_graph": int(rng.integers(1, 6)), "cache_policy": int(rng.choice([1, 2]))}
    return sims, order, tuning, int(rng.integers(1, 9))


@pytest.mark.parametrize("case", range(6))
def test_random_batch(torch_dev, case):
    """Seeded random batches of 2-7 uneven 1D boxes (sizes, direction sets,
    weights of either sign, time steps, vacuum and matter terms, their own
    start steps; one shape order per batch) in random launch shapes and
    cache policies: every box against the reference."""
    from paper_2101_02745_amd.sim import Batch
    from paper_2101_02745_amd._lib import HostConfig
    sims, order, tuning, nsteps = draw_batch(case)
    cfgs = [HostConfig(s["ncell"], s["dx"], s["dirs"], s["N"], s["Nb"], s["H"], s["dt"],
                       shape_order=order, vmat=s["vmat"]) for s in sims]
    b = Batch(cfgs, tuning=tuning)
    for i, s in enumerate(sims):
        b.set_state(i, s["st"], s["step0"])
    b.step(nsteps)
    tots = b.flavor_totals()
    for i, s in enumerate(sims):
        P = Problem(s["ncell"], s["dx"], s["dirs"], s["N"], s["Nb"], s["H"], s["dt"],
                    vmat=s["vmat"], shape_order=order)
        ref = P.step(s["st"], nsteps, n0=s["step0"])
        what = dict(case=case, box=i, ncell=s["ncell"], ndir=len(s["dirs"]), order=order, tuning=tuning)
        assert_parity(b.get_state(i).cpu().numpy(), ref, what=str(what))
        tref = P.flavor_totals(ref)
        assert np.abs(tots[i] - tref).max() <= 1e-12 * max(np.abs(tref).max(), 1e-300), what
