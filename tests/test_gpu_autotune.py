"""The autotuner measured on the device (fpic_autotune through sim.autotune,
without the committed cache): it returns a shape from its candidate set,
writes it to the JSON cache and reads the same shape back, and a box run in
the chosen shape matches the CPU reference."""
import json

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


def tune_and_check(cfgs, cache):
    from paper_2101_02745_amd.sim import autotune
    t, ms = autotune(cfgs, cache=cache)
    assert ms > 0.0
    t2, ms2 = autotune(cfgs, cache=cache)  # from the cache: no measurement
    assert t2 == t and ms2 == ms
    rec = json.load(open(cache))
    assert any(v["launch"] == t for v in rec.values())
    return t


def test_autotune_1d_box(torch_dev, tmp_path):
    from paper_2101_02745_amd._lib import HostConfig
    from paper_2101_02745_amd.sim import Sim
    w = I.workload("1d_32x26")
    t = tune_and_check([HostConfig.from_workload(w)], str(tmp_path / "tune.json"))
    assert t["waves"] in (1, 2, 4, 8) and 1 <= t["dirs_per_wave"] <= 32
    assert t["cache_policy"] in (0, 1, 2)
    sim = Sim.from_workload(w, tuning=t)
    s0 = w.state0()
    sim.set_state(s0, 7)
    sim.step(5)
    ref = Problem.from_workload(w).step(s0, 5, n0=7)
    assert_parity(sim.get_state().cpu().numpy(), ref, what=f"1d_32x26 in {t}")


def test_autotune_batch(torch_dev, tmp_path):
    from paper_2101_02745_amd._lib import HostConfig
    from paper_2101_02745_amd.sim import Batch
    ws = I.batch_workloads(nsim=3, steps=0)
    ws = [I.scaled(w, ncell=(1, 1, 64 + 45 * i), ndir=w.ndir if w.ndir < 378 else 92)
          for i, w in enumerate(ws)]
    cfgs = [HostConfig.from_workload(w) for w in ws]
    t = tune_and_check(cfgs, str(tmp_path / "tune.json"))
    assert t["waves"] in (1, 2, 4, 8)
    b = Batch(cfgs, tuning=t)
    for i, w in enumerate(ws):
        b.set_state(i, w.state0())
    b.step(3)
    for i, w in enumerate(ws):
        ref = Problem.from_workload(w).step(w.state0(), 3)
        assert_parity(b.get_state(i).cpu().numpy(), ref, what=f"batch box {i} in {t}")
    b.close()


def test_autotune_3d_box(torch_dev, tmp_path):
    """A 3D box: the tuner also chooses between the fused linear stages and
    the separate kernels."""
    from paper_2101_02745_amd._lib import HostConfig
    from paper_2101_02745_amd.sim import Sim
    w = I.Workload(name="t3", ncell=(16, 6, 5), length=(8.0, 3.0, 2.5), ndir=26, dt=0.1, steps=0,
                   f=0.1, fbar=-0.2, nbar_over_n=1.2, nhat=(0.5, 0.0, 0.8660254037844386), seed=3,
                   alpha=1e-2)
    t = tune_and_check([HostConfig.from_workload(w)], str(tmp_path / "tune.json"))
    assert t["fused"] in (0, 1, 2)
    sim = Sim.from_workload(w, tuning=t)
    s0 = w.state0()
    sim.set_state(s0, 2)
    sim.step(3)
    ref = Problem.from_workload(w).step(s0, 3, n0=2)
    assert_parity(sim.get_state().cpu().numpy(), ref, what=f"3d in {t}")
    assert np.isfinite(sim.check(1e-12))
