"""Slopes formed again instead of stored, against the stored form
(fpic_tuning.fused 2), classical RK4 (Sec. II.C).  fused 1 forms the stage-1
slope again in stages 2 and 4, fused 0 (the default for 1D boxes and
batches) also the stage-2 slope in stages 3 and 4, with the same operations
on the same operands as the stage that first formed it (the slope path is
written with explicit fused multiply-adds): every form must agree with the
stored one bit for bit.  Agreement with the CPU reference is what the
parity tests check.  Cases: boxes smaller than the staged tile
(wrapped cells), ragged last tiles with stage-4 shifts of up to two cells,
both shape orders at the full 2048 x 378 size, and an uneven batch."""
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


def run_box(w, fused, steps, step0=0, waves=4, dpw=3):
    from paper_2101_02745_amd.sim import Sim
    t = {"waves": waves, "dirs_per_wave": dpw, "steps_per_graph": 4, "cache_policy": 0, "fused": fused}
    sim = Sim.from_workload(w, tuning=t)
    sim.set_state(w.state0(), step0)
    sim.step(steps)
    out = sim.get_state().cpu().numpy()
    del sim
    return out


def assert_bitwise(a, b, what):
    assert a.shape == b.shape
    assert np.isfinite(a).all(), what
    same = a.view(np.uint64) == b.view(np.uint64)
    assert same.all(), f"{what}: {np.count_nonzero(~same)} of {a.size} entries differ"


def assert_form(a, b, fused, what):
    assert_bitwise(a, b, what)


BOXES = [
    # (name, ncell, ndir, dt in units of the cell width, shape order)
    ("32 cells, smaller than a staged tile", 32, 26, None, 1),
    ("32 cells, quadratic", 32, 26, None, 2),
    ("100 cells, ragged tile, shifts near two cells", 100, 26, 1.8, 1),
    ("100 cells, quadratic, shifts near two cells", 100, 26, 1.8, 2),
    ("69 cells, one tile and a wrapped tail", 69, 92, 1.5, 1),
    ("71 cells, quadratic", 71, 92, 1.5, 2),
]


@pytest.mark.parametrize("name,ncell,ndir,dtc,shape", BOXES)
def test_recompute_matches_stored_small(torch_dev, name, ncell, ndir, dtc, shape):
    w = I.scaled(I.workload("1d_32x26"), ncell=(1, 1, ncell), ndir=ndir)
    if dtc is not None:
        w = dataclasses.replace(w, dt=dtc * w.dx[2])
    w = dataclasses.replace(w, shape_order=shape)
    for waves, dpw in ((4, 3), (8, 1), (1, 8)):
        b = run_box(w, 2, 6, step0=5, waves=waves, dpw=dpw)
        for fused in (0, 1):
            a = run_box(w, fused, 6, step0=5, waves=waves, dpw=dpw)
            assert_form(a, b, fused, f"{name} in {waves} x {dpw}, fused {fused}")


@pytest.mark.parametrize("shape", [1, 2])
def test_recompute_matches_stored_full_size(torch_dev, shape):
    w = dataclasses.replace(I.workload("1d_2048x378"), shape_order=shape)
    b = run_box(w, 2, 3, waves=8, dpw=6)
    for fused in (0, 1):
        a = run_box(w, fused, 3, waves=8, dpw=6)
        assert_form(a, b, fused, f"2048 x 378, shape {shape}, fused {fused}")


def test_recompute_matches_stored_batch(torch_dev):
    from paper_2101_02745_amd._lib import HostConfig
    from paper_2101_02745_amd.sim import Batch
    ws = I.batch_workloads(nsim=4, steps=0)
    ws = [I.scaled(w, ncell=(1, 1, 70 + 61 * i)) for i, w in enumerate(ws)]
    cfgs = [HostConfig.from_workload(w) for w in ws]
    outs = []
    for fused in (0, 1, 2):
        t = {"waves": 8, "dirs_per_wave": 8, "steps_per_graph": 4, "cache_policy": 0, "fused": fused}
        b = Batch(cfgs, tuning=t)
        for i, w in enumerate(ws):
            b.set_state(i, w.state0(), 2)
        b.step(5)
        outs.append([b.get_state(i).cpu().numpy() for i in range(len(ws))])
        b.close()
    for i in range(len(ws)):
        for f in (0, 1):
            assert_form(outs[f][i], outs[2][i], f, f"batch box {i}, fused {f}")
