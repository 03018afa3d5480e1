#!/usr/bin/env python3
"""Throughput of the PIC flavor hot path on one MI355X.

One step = one classical RK4 step of the whole box: four times (deposit with
the cloud-in-cell shape, interpolation, Hamiltonian, commutator, stage
update).  The workload is the 1D box of 2048 cells and 378 directions
(774,144 particles), dt = 0.1/mu, seeded synthetic initial state.

Prints one JSON line.  `value` is particle-steps per second over the timed
region (state resident in HBM, hipGraph-replayed steps).  `roofline` reports
the dominant kernel against the HBM peak, from its algorithmic bytes per
launch and its mean launch time measured with HIP events on the library's
stream; `cpu_baseline` is the CPU FP64 reference timed on a bounded sample
of the same workload on this host.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/s (deposit+gather+RK4) on 1 GPU vs roofline; adjoint/forward ratio"
STATE_B = 18 * 8        # bytes of one particle's state
SLOPE_B = 16 * 8        # bytes of one stored Runge-Kutta slope (traceless: 8 + 8 reals)
GRID_B = 36 * 8         # bytes of one cell's combined moments
SRC3_B = 8 * 8          # 3D: traceless deposit source per particle
GRID3_B = 32 * 8        # one cell's traceless combined moments (3D and general placement)
# particle bytes per stage kernel in the stage-synchronous Runge-Kutta
# schedule: stage 1 reads Y, writes k1; stages 2, 3 read Y and the previous
# slope, write their slope; stage 4 reads Y, k1, k2, k3 and writes Y
STAGE_BYTES = {1: STATE_B + SLOPE_B, 2: STATE_B + 2 * SLOPE_B, 3: STATE_B + 2 * SLOPE_B,
               4: 2 * STATE_B + 3 * SLOPE_B}
STEP_BYTES = sum(STAGE_BYTES.values())   # 1744 B per particle-step
# the same 13 passes with 18-real slopes: the stage-synchronous floor the
# throughput targets are stated against, and the per-particle figure the
# roofline blocks price a launch at (2, 3, 3 and 5 passes of 144 B)
CONTRACT_STAGE_BYTES = {1: 2 * STATE_B, 2: 3 * STATE_B, 3: 3 * STATE_B, 4: 5 * STATE_B}
CONTRACT_STEP_BYTES = 13 * STATE_B        # 1872 B per particle-step
ACCOUNTING = ("achieved: the bytes this launch form moves per launch (16-real slopes; 1D boxes and "
              "batches 144, 144, 272, 416 B per particle for stages 1-4 with the stage-1 and stage-2 "
              "slopes formed again, 144, 272, 400, 544 B with the stage-1 slope alone formed again, "
              "272, 400, 400, 672 B with every slope stored, as in 3D), plus the grid; contract_*: "
              "the same launch priced at the 13-pass stage-synchronous contract, 2, 3, 3, 5 passes "
              "of 144 B per particle, which can exceed the peak where slopes are formed again")
# 1D boxes and batches, fpic_tuning.fused 1: stage 1 stores no slope, and
# stages 2 and 4 form it again from the state and the stage-1 grid
RK1_STAGE_BYTES = {1: STATE_B, 2: STATE_B + SLOPE_B, 3: STATE_B + 2 * SLOPE_B,
                   4: 2 * STATE_B + 2 * SLOPE_B}   # 1360 B per particle-step
# fused 0 (the default): stage 2 stores none either; stages 3 and 4 form k1
# and k2 again (the stage-2 grid kept as well)
RK2_STAGE_BYTES = {1: STATE_B, 2: STATE_B, 3: STATE_B + SLOPE_B,
                   4: 2 * STATE_B + SLOPE_B}       # 976 B per particle-step


def own_stage_bytes_1d(tune):
    """Per-particle bytes of the four 1D stage kernels in this launch form."""
    fused = (tune or {}).get("fused", 0)
    return STAGE_BYTES if fused == 2 else RK1_STAGE_BYTES if fused == 1 else RK2_STAGE_BYTES
# general placement (1D): every stage also reads the particle's own z
# position at t = 0, direction and two weights; a sort reads the key inputs
# (z, Omega_z) once more, and its stage 4 also writes the particle's z,
# direction, weights and index to their sorted place (the state it writes
# anyway)
PSTATIC_B = (1 + 3 + 2) * 8
PSTAGE_BYTES = {s: b + PSTATIC_B for s, b in STAGE_BYTES.items()}
PSORT_BYTES = 16 + PSTATIC_B + 4
# 3D general placement: three position components instead of one
PSTATIC3_B = (3 + 3 + 2) * 8
PSTAGE3_BYTES = {s: b + PSTATIC3_B for s, b in STAGE_BYTES.items()}
PSORT3_BYTES = 48 + PSTATIC3_B + 4


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fpic_1d.hip", "fpic_device.h", "fpic_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2101_02745_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def particles_source_hash():
    h = hashlib.sha256()
    for f in ("fpic_particles.hip", "fpic_device.h"):
        h.update(open(os.path.join(ROOT, "paper_2101_02745_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def source_hash_3d():
    h = hashlib.sha256()
    for f in ("fpic_3d.hip", "fpic_device.h"):
        h.update(open(os.path.join(ROOT, "paper_2101_02745_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def same_launch(recorded, launch):
    """The launch shape the counters were taken at equals the timed one
    (fields the record does not name count as unset)."""
    if recorded is None or launch is None:
        return False
    keys = set(recorded) | set(launch)
    return all(int(recorded.get(k, 0)) == int(launch.get(k, 0)) for k in keys)


def measured_traffic(kernel: str, workload: str, source_hash=None, launch=None):
    """HBM bytes per launch from committed counter runs, if they were taken on
    the current kernel source and, when `launch` is given, in that launch
    shape (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    ent = rec.get(workload, {}).get(kernel)
    if not ent or ent.get("source_hash") != (source_hash or kernel_source_hash()):
        return None
    if launch is not None and not same_launch(ent.get("launch"), launch):
        return None
    return ent.get("bytes_per_launch")


def host_cpu():
    """nproc, the CPUs this process may run on, and the CPU model name."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return os.cpu_count() or 1, avail, model


def cpu_baseline(w, repeats=3):
    """The CPU reference (the oracle, as it stands) on this host: the same
    particle-steps/s of the same box, timed with one thread and with all the
    host threads this process may use (capped by OMP_NUM_THREADS when that is
    set), the median of `repeats` runs each; a bounded sample of steps."""
    import numpy as np
    from oracle import Problem, set_threads
    nproc, avail, model = host_cpu()
    allt = avail
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        allt = min(allt, int(os.environ["OMP_NUM_THREADS"]))
    P = Problem.from_workload(w)
    s = P.step(w.state0(), 1)          # warm-up (first touch of the buffers)
    out = {}
    for label, threads, steps in (("one_thread", 1, 1), ("all_threads", allt, 4)):
        used = set_threads(threads)
        rates = []
        for r in range(repeats):
            t0 = time.perf_counter()
            P.step(s, steps, n0=1 + r * steps)
            rates.append(w.nparticles * steps / (time.perf_counter() - t0))
        out[label] = {"value": float(np.median(rates)), "threads": used, "steps": steps,
                      "runs": rates}
    return {"value": out["all_threads"]["value"], "unit": "particle-steps/s",
            "cores": out["all_threads"]["threads"], "kind": "oracle",
            "sample": f"{out['all_threads']['steps']} RK4 steps of the full {w.name} box "
                      f"({w.nparticles} particles) per run, median of {repeats} runs, after a "
                      f"warm-up step; {out['all_threads']['threads']} OpenMP threads "
                      f"(one-thread figure: {out['one_thread']['steps']} step per run)",
            "one_thread": out["one_thread"], "all_threads": out["all_threads"],
            "nproc": nproc, "cpus_available": avail,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"), "cpu_model": model}


def measure_adjoint(steps=2000, ckpt=50, tune=None):
    """Reverse mode on the 512 x 128 gradient workload: time of the plain
    forward pass, of the checkpointed forward pass and of the backward pass
    (recompute + reverse sweep), all for the same number of steps."""
    import numpy as np
    import torch
    from paper_2101_02745_amd import inputs as I
    from paper_2101_02745_amd.sim import Sim
    from paper_2101_02745_amd._lib import HostConfig
    from paper_2101_02745_amd.sim import autotune
    w = I.workload("1d_512x128")
    if tune is None:
        tune, _ = autotune([HostConfig.from_workload(w)])
    sim = Sim.from_workload(w, tuning=tune)
    s0 = torch.from_numpy(w.state0()).cuda()
    N, Nb = w.weights()
    lam = np.zeros((18, w.ndir, w.ncell_total))
    lam[1] = lam[2] = (N / (N.sum() * w.ncell_total))[:, None]
    lam[10] = lam[11] = (Nb / (Nb.sum() * w.ncell_total))[:, None]
    lam = torch.from_numpy(lam).cuda()
    sim.set_state(s0)
    sim.step(20)                       # warm-up
    sim.set_state(s0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    sim.set_state(s0)
    sim.adjoint_forward(10, 5)         # warm-up of the reverse path
    sim.adjoint_backward(lam)
    sim.set_state(s0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.adjoint_forward(steps, ckpt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.adjoint_backward(lam)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return {"workload": w.name, "particles": w.nparticles, "steps": steps, "ckpt_every": ckpt,
            "launch": tune,
            "forward_s": fwd, "checkpointed_forward_s": t1 - t0, "backward_s": t2 - t1,
            "backward_over_forward": (t2 - t1) / fwd,
            "total_over_forward": (t2 - t0) / fwd}


def event_timing(reset, step, steps, runs=5):
    """Per-step time of `steps` steps from HIP events, median of `runs` runs,
    each from the same initial state (reset()) after one warm-up step.  The
    events are recorded on torch's current stream, the stream the library's
    context was created on, so they bracket its kernels."""
    import numpy as np
    import torch
    per = []
    for _ in range(runs):
        reset()
        step(1)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        step(steps)
        e1.record()
        e1.synchronize()
        per.append(e0.elapsed_time(e1) / steps)
    return {"ms_per_step_median": float(np.median(per)), "ms_per_step_runs": per,
            "steps_per_run": steps, "runs": runs,
            "timer": "HIP events on the context's stream around the steps, median of the runs, "
                     "each from the initial state after one warm-up step"}


def stage_accounting(w, tune):
    """Kernel names and algorithmic bytes per launch of the four stage
    kernels and of the kernel that follows each (reduction or deposit), at
    this implementation's slopes (own) and at the 13-pass contract, for a 1D
    box, a 3D box on the fused linear stages, or a 3D box on the separate
    kernels; and the source hash its counter records are keyed by."""
    P, nc = w.nparticles, w.ncell_total
    if w.ncell[0] == 1 and w.ncell[1] == 1:
        sb = own_stage_bytes_1d(tune)
        own = [sb[s] * P + 2 * GRID_B * nc for s in (1, 2, 3, 4)]
        contract = [CONTRACT_STAGE_BYTES[s] * P + 2 * GRID_B * nc for s in (1, 2, 3, 4)]
        return ("stage1d_kernel", "reduce1d_kernel"), own, contract, None, kernel_source_hash
    fused = (tune or {}).get("fused", 0) != 2 and w.shape_order == 1 and w.ncell[0] <= 64
    if fused:
        # stage kernel: the state passes, four staged grid rows and four
        # partial rows per workgroup (one x-row of cells); reduction: four
        # partial grids read, the grid written
        own = [STAGE_BYTES[s] * P + 2 * 4 * GRID3_B * nc for s in (1, 2, 3, 4)]
        contract = [CONTRACT_STAGE_BYTES[s] * P + 2 * 4 * GRID3_B * nc for s in (1, 2, 3, 4)]
        return ("stage3f_kernel", "reduce3f_kernel"), own, contract, 5 * GRID3_B * nc, source_hash_3d
    own = [STAGE_BYTES[s] * P + SRC3_B * P for s in (1, 2, 3, 4)]
    contract = [CONTRACT_STAGE_BYTES[s] * P + SRC3_B * P for s in (1, 2, 3, 4)]
    names = ("particle3d_kernel", "deposit3d_kernel") if w.shape_order == 1 else \
        ("particle3q_kernel", "deposit3q_kernel")
    return names, own, contract, SRC3_B * P + GRID3_B * nc, source_hash_3d


def measure_3d(steps=200, step0=0):
    """The 64^3 x 92 box (24,117,248 particles) for its 200 steps.  With the
    linear shape each stage is one fused kernel (particle update, and the
    deposit of the next stage state through per-workgroup partial rows) plus
    a reduction of those partials; the quadratic shape keeps a particle
    kernel (writing a 64-byte traceless deposit source per particle) and a
    cell-centric deposit kernel per stage."""
    import torch
    from paper_2101_02745_amd import inputs as I
    from paper_2101_02745_amd._lib import HostConfig
    from paper_2101_02745_amd.sim import Sim, autotune
    w = I.workload("3d_64x92")
    tune, _ = autotune([HostConfig.from_workload(w)])
    sim = Sim.from_workload(w, tuning=tune)
    s0 = w.state0()
    sim.set_state(s0, step0)
    sim.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = event_timing(lambda: sim.set_state(s0, step0), sim.step, steps)
    ms = sim.profile(3)
    trace = sim.check(1e-10)
    del sim
    P = w.nparticles
    stage_ms = [ms[0], ms[2], ms[4], ms[6]]
    second_ms = [ms[1], ms[3], ms[5], ms[7]]
    names, stage_bytes, contract_bytes, second_bytes, _ = stage_accounting(w, tune)
    step_bytes = sum(stage_bytes) + 4 * second_bytes
    ms_step = 1e3 * wall / steps
    dom = max(range(4), key=lambda k: stage_ms[k])
    ach = contract_bytes[dom] / (stage_ms[dom] * 1e-3) / 1e9
    own = stage_bytes[dom] / (stage_ms[dom] * 1e-3) / 1e9
    rec = {"workload": w.name, "particles": P, "steps": steps, "step0": step0 + 2,
           "launch": tune, "value": P * steps / wall, "unit": "particle-steps/s",
           "ms_per_step": ms_step,
           "kernels": list(names), "stage_kernel_ms": stage_ms, "second_kernel_ms": second_ms,
           "stage_kernel_GBs": [b / (t * 1e-3) / 1e9 for b, t in zip(stage_bytes, stage_ms)],
           "second_kernel_GBs": [second_bytes / (t * 1e-3) / 1e9 for t in second_ms],
           "alg_bytes_per_step": step_bytes,
           "step_frac_of_hbm_peak": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
           # the contract's floor: 13 passes of an 18-real particle record
           "frac_of_1872B_roofline": CONTRACT_STEP_BYTES * P / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "roofline": {"bound": "hbm", "kernel": f"{names[0]}<{dom + 1}>",
                        "achieved": own, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": own / HBM_PEAK_GBS,
                        "traffic": measured_traffic(f"stage{dom + 1}", w.name, source_hash_3d(),
                                                    launch=tune),
                        "alg_bytes_per_launch": stage_bytes[dom], "ms_per_launch": stage_ms[dom],
                        "accounting": ACCOUNTING, "contract_bytes_per_launch": contract_bytes[dom],
                        "contract_achieved": ach, "contract_frac": ach / HBM_PEAK_GBS},
           "event_timing": ev,
           "trace_error": trace}
    return rec


def measure_quadratic(steps=200):
    """The headline box with the quadratic shape function (Sec. II.B.1, the
    paper's production choice), in its own autotuned launch shape."""
    import dataclasses
    import torch
    from paper_2101_02745_amd import inputs as I
    from paper_2101_02745_amd._lib import HostConfig
    from paper_2101_02745_amd.sim import Sim, autotune
    w = dataclasses.replace(I.workload("1d_2048x378"), shape_order=2)
    tuning, _ = autotune([HostConfig.from_workload(w)])
    sim = Sim.from_workload(w, tuning=tuning)
    sim.set_state(w.state0())
    sim.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sim.profile(5)
    P = w.nparticles
    return {"workload": w.name + " (quadratic shape)", "particles": P, "steps": steps,
            "launch": tuning, "value": P * steps / wall, "unit": "particle-steps/s",
            "ms_per_step": 1e3 * wall / steps,
            "stage_ms": [ms[0], ms[2], ms[4], ms[6]], "reduce_ms": [ms[1], ms[3], ms[5], ms[7]],
            "step_frac_of_hbm_peak": sum(own_stage_bytes_1d(tuning).values()) * P / (wall / steps) / 1e9
                                     / HBM_PEAK_GBS}


def measure_batch(steps=1000, nsim=64):
    """64 uneven 1D boxes for their 1000 steps: one batched launch per stage
    vs the same boxes run one after another through the single-box path
    (each with its own captured graph)."""
    import torch
    from paper_2101_02745_amd import inputs as I
    from paper_2101_02745_amd._lib import HostConfig
    from paper_2101_02745_amd.sim import Batch, Sim
    from paper_2101_02745_amd.sim import autotune
    ws = I.batch_workloads(nsim=nsim, steps=steps)
    P = sum(w.nparticles for w in ws)
    ncell = sum(w.ncell_total for w in ws)
    cfgs = [HostConfig.from_workload(w) for w in ws]
    tune, _ = autotune(cfgs)
    b = Batch(cfgs, tuning=tune)
    for i, w in enumerate(ws):
        b.set_state(i, w.state0())
    b.step(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    s0s = [w.state0() for w in ws]

    def reset():
        for i, st in enumerate(s0s):
            b.set_state(i, st)

    ev = event_timing(reset, b.step, min(steps, 200))
    ms = b.profile(5)
    b.close()
    del b
    sims = []
    for w in ws:
        sm = Sim.from_workload(w)
        sm.set_state(w.state0())
        sm.step(5)
        sims.append(sm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sm in sims:
        sm.step(steps)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    neg = sum(1 for w in ws if min(w.weights()[0].min(), w.weights()[1].min()) < 0)
    stage_ms = [ms[0], ms[2], ms[4], ms[6]]
    sb = own_stage_bytes_1d(tune)
    stage_bytes = [sb[k] * P + 2 * GRID_B * ncell for k in (1, 2, 3, 4)]
    contract_bytes = [CONTRACT_STAGE_BYTES[k] * P + 2 * GRID_B * ncell for k in (1, 2, 3, 4)]
    dom = max(range(4), key=lambda k: stage_ms[k])
    ach = contract_bytes[dom] / (stage_ms[dom] * 1e-3) / 1e9
    own = stage_bytes[dom] / (stage_ms[dom] * 1e-3) / 1e9
    ms_step = 1e3 * tb / steps
    return {"nsim": nsim, "particles": P, "cells": ncell, "steps": steps, "batch_launch": tune,
            "batched_psteps_per_s": P * steps / tb, "sequential_psteps_per_s": P * steps / ts,
            "ratio": ts / tb, "ms_per_step": ms_step,
            "frac_of_1872B_roofline": CONTRACT_STEP_BYTES * P / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "ratio_note": "a 3x gain over the sequential runs would need "
                          f"{3 * P * steps / ts:.3g} particle-steps/s; the 1872 B "
                          f"roofline is {HBM_PEAK_GBS * 1e9 / CONTRACT_STEP_BYTES:.3g}, and at the "
                          f"{sum(sb.values())} B per particle-step this launch form moves "
                          f"{HBM_PEAK_GBS * 1e9 / sum(sb.values()):.3g}",
            "event_timing": ev,
            "stage_ms": stage_ms, "reduce_ms": [ms[1], ms[3], ms[5], ms[7]],
            "roofline": {"bound": "hbm", "kernel": f"stage1d_kernel<{dom + 1}> (batched)",
                         "achieved": own, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": own / HBM_PEAK_GBS,
                         "traffic": measured_traffic(f"stage{dom + 1}", "batch_64_uneven", launch=tune),
                         "alg_bytes_per_launch": stage_bytes[dom], "ms_per_launch": stage_ms[dom],
                         "accounting": ACCOUNTING, "contract_bytes_per_launch": contract_bytes[dom],
                         "contract_achieved": ach, "contract_frac": ach / HBM_PEAK_GBS},
            "sims_with_negative_weights": neg}


def probe_batch(tuning=None, steps=40):
    """The 64-box batch alone (no sequential runs), for kernel profiles:
    5 warm-up steps, then `steps` steps in hipGraphs."""
    import torch
    from paper_2101_02745_amd import inputs as I
    from paper_2101_02745_amd._lib import HostConfig
    from paper_2101_02745_amd.sim import Batch
    ws = I.batch_workloads(nsim=64, steps=steps)
    if not tuning:
        from paper_2101_02745_amd.sim import autotune
        tuning, _ = autotune([HostConfig.from_workload(w) for w in ws])
    P = sum(w.nparticles for w in ws)
    b = Batch([HostConfig.from_workload(w) for w in ws], tuning=tuning)
    for i, w in enumerate(ws):
        b.set_state(i, w.state0())
    b.step(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"particles": P, "steps": steps, "launch": tuning, "ms_per_step": 1e3 * wall / steps,
            "psteps_per_s": P * steps / wall}


def measure_particles(steps=200, sort_every=4, with_3d=True, exact=True):
    """General placement: the 2048-cell, 64 pi box with 774,144 particles at
    uniform random positions (378 per cell on average), sorted by cell every
    `sort_every` steps inside the timed region.  exact: deposits summed
    exactly (bitwise reproducible, the library's default); otherwise with
    floating-point atomics (reported beside it)."""
    import torch
    from paper_2101_02745_amd import inputs as I
    from paper_2101_02745_amd.particles import ParticleSim
    w = I.particle_workload("1d_2048x378_random")
    sim = ParticleSim.from_workload(w, sort_every=sort_every, exact=exact)
    sim.set_workload(w)
    sim.step(4 * sort_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sim.profile(10)
    P = w.nparticles
    grid = 2 * GRID3_B * w.ncell_total  # traceless stage grids
    stage_bytes = [PSTAGE_BYTES[s] * P + grid for s in (1, 2, 3, 4)]
    step_bytes = sum(stage_bytes) + PSORT_BYTES * P / sort_every
    # the per-kernel timings sort after every step: their stage 4 is the
    # sorting form (pstage_kernel<8>), which also moves the particles
    stage_bytes[3] += PSORT_BYTES * P
    mode = "exact" if exact else "float_atomics"
    names = [f"pstage_kernel<{m}> {mode}" for m in (1, 2, 3, 8)]
    ms_step = 1e3 * wall / steps
    dom = max(range(4), key=lambda k: ms[k])
    sim.close()
    out = {"workload": w.name, "particles": P, "steps": steps, "sort_every": sort_every,
            "deposit_sums": "exact" if exact else "float_atomics",
            "value": P * steps / wall, "unit": "particle-steps/s", "ms_per_step": ms_step,
            "stage_ms": list(ms[:4]), "sort_count_scan_ms": ms[4],
            "stage_GBs": [b / (t * 1e-3) / 1e9 for b, t in zip(stage_bytes, ms[:4])],
            "roofline": {"bound": "hbm", "kernel": names[dom],
                         "traffic": measured_traffic(names[dom], w.name, particles_source_hash()),
                         "achieved": stage_bytes[dom] / (ms[dom] * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": stage_bytes[dom] / (ms[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "alg_bytes_per_launch": stage_bytes[dom], "ms_per_launch": ms[dom]},
            "alg_bytes_per_step": step_bytes,
            "step_frac_of_hbm_peak": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if with_3d:
        out["box3d"] = measure_particles_3d(exact=exact)
    if exact:
        fast = measure_particles(steps, sort_every, with_3d, exact=False)
        out["float_atomics"] = {"value": fast["value"], "ms_per_step": fast["ms_per_step"],
                                "roofline_frac": fast["roofline"]["frac"],
                                "box3d": {k: fast["box3d"][k] for k in ("value", "ms_per_step")}
                                if with_3d else None}
    return out


def measure_particles_3d(steps=16, sort_every=4, exact=True):
    """General placement in 3D: 32^3 cells, 92 particles per cell on average
    at random positions (3,014,656 particles)."""
    import torch
    from paper_2101_02745_amd import inputs as I
    from paper_2101_02745_amd.particles import ParticleSim
    w = I.particle_workload("3d_32x92_random")
    sim = ParticleSim.from_workload(w, sort_every=sort_every, exact=exact)
    sim.set_workload(w)
    sim.step(2 * sort_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sim.profile(3)
    sim.close()
    P = w.nparticles
    grid = 2 * GRID3_B * w.ncell_total
    stage_bytes = [PSTAGE3_BYTES[s] * P + grid for s in (1, 2, 3, 4)]
    step_bytes = sum(stage_bytes) + PSORT3_BYTES * P / sort_every
    stage_bytes[3] += PSORT3_BYTES * P  # the profiled stage 4 sorts
    sums = "exact" if exact else "float_atomics"
    names = [f"pstage_kernel<{m}> {sums}" for m in (1, 2, 3, 8)]
    ms_step = 1e3 * wall / steps
    dom = max(range(4), key=lambda k: ms[k])
    return {"workload": w.name, "particles": P, "steps": steps,
            "sort_every": sort_every, "deposit_sums": "exact" if exact else "float_atomics",
            "value": P * steps / wall,
            "unit": "particle-steps/s", "ms_per_step": ms_step,
            "stage_ms": list(ms[:4]), "sort_count_scan_ms": ms[4],
            "stage_GBs": [b / (t * 1e-3) / 1e9 for b, t in zip(stage_bytes, ms[:4])],
            "roofline": {"bound": "hbm", "kernel": names[dom],
                         "traffic": measured_traffic(names[dom], w.name, particles_source_hash()),
                         "achieved": stage_bytes[dom] / (ms[dom] * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": stage_bytes[dom] / (ms[dom] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "alg_bytes_per_launch": stage_bytes[dom], "ms_per_launch": ms[dom]},
            "alg_bytes_per_step": step_bytes,
            "step_frac_of_hbm_peak": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="1d_2048x378")
    ap.add_argument("--shape", type=int, default=0, choices=[0, 1, 2],
                    help="shape-function order of the workload (0: its own; 1 linear, 2 quadratic)")
    ap.add_argument("--step0", type=int, default=0,
                    help="step number of the initial state (time step0*dt)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the adjoint and batch measurements")
    ap.add_argument("--tuning", default="",
                    help="JSON launch shape; default: autotune on the device first")
    ap.add_argument("--probe", default="", choices=["", "copy", "kernels", "adjoint", "particles",
                                                    "particles3d", "batch"],
                    help="counter-collection modes: 'copy' runs a plain 1 GiB device copy "
                         "(the reference for HBM byte counters); 'kernels' runs 5 steps "
                         "with every kernel launched on its own, then exits; 'particles' "
                         "times the general-placement box; 'batch' steps the 64-box batch "
                         "in one launch shape (--tuning, else the cached autotuned one)")
    args = ap.parse_args()
    if args.probe == "copy":
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "copy", "bytes_read": src.numel() * 8,
                          "bytes_written": dst.numel() * 8, "launches": 5}), flush=True)
        return
    if args.probe == "particles":
        r = measure_particles(steps=20, with_3d=False)
        print(json.dumps({"probe": "particles", **r}), flush=True)
        return
    if args.probe == "particles3d":
        r = measure_particles_3d(steps=8)
        f = measure_particles_3d(steps=8, exact=False)
        print(json.dumps({"probe": "particles3d", **r, "float_atomics": f}), flush=True)
        return
    if args.probe == "batch":
        r = probe_batch(json.loads(args.tuning) if args.tuning else None)
        print(json.dumps({"probe": "batch", **r}), flush=True)
        return
    if args.probe == "adjoint":
        r = measure_adjoint(steps=200, ckpt=50, tune=json.loads(args.tuning) if args.tuning else None)
        print(json.dumps({"probe": "adjoint", **r}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2101_02745_amd import inputs as I
    from paper_2101_02745_amd.sim import Sim

    w = I.workload(args.workload)
    if args.shape:
        import dataclasses
        w = dataclasses.replace(w, shape_order=args.shape)
    tune_ms = None
    if args.tuning:
        tuning = json.loads(args.tuning)
    else:
        from paper_2101_02745_amd._lib import HostConfig
        from paper_2101_02745_amd.sim import autotune
        tuning, tune_ms = autotune([HostConfig.from_workload(w)])
        print(f"[bench] autotuned launch shape {tuning} ({tune_ms:.4f} ms/step)",
              file=sys.stderr, flush=True)
    sim = Sim.from_workload(w, tuning=tuning)
    sim.set_state(w.state0(), args.step0)
    torch.cuda.synchronize()
    if args.probe == "kernels":
        ms = sim.profile(5)
        print(json.dumps({"probe": "kernels", "workload": w.name, "ms": list(ms),
                          "tuning": sim.tune.as_dict() if sim.tune else None}), flush=True)
        return
    print(f"[bench] {w.name}: {w.nparticles} particles, warmup {args.warmup} steps",
          file=sys.stderr, flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    value = w.nparticles * args.steps / wall
    print(f"[bench] timed {args.steps} steps: {ms_step:.4f} ms/step", file=sys.stderr, flush=True)
    s0 = w.state0()
    ev = event_timing(lambda: sim.set_state(s0, args.step0), sim.step, args.steps)
    print(f"[bench] HIP events: {ev['ms_per_step_median']:.4f} ms/step (median of {ev['runs']})",
          file=sys.stderr, flush=True)

    # per-kernel launch times (HIP events on the library's stream)
    ms = sim.profile(20)
    stage_ms = {s: ms[2 * (s - 1)] for s in (1, 2, 3, 4)}
    red_ms = [ms[2 * s - 1] for s in (1, 2, 3, 4)]
    dom = max(stage_ms, key=lambda s: stage_ms[s])
    launch = sim.tune.as_dict() if sim.tune else None
    names, own_b, contract_b, second_b, hashfn = stage_accounting(w, launch)
    alg_bytes = contract_b[dom - 1]
    achieved = alg_bytes / (stage_ms[dom] * 1e-3) / 1e9
    own_bytes = own_b[dom - 1]
    own = own_bytes / (stage_ms[dom] * 1e-3) / 1e9
    # the counter records are for the workloads' own (linear) shape
    traffic = (measured_traffic(f"stage{dom}", w.name, hashfn(), launch=launch)
               if w.shape_order == 1 else None)
    step_bytes = sum(contract_b) + 4 * (second_b or 0)
    own_step_bytes = sum(own_b) + 4 * (second_b or 0)
    ok = sim.check(1e-10)

    rec = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "ncell": list(w.ncell), "ndir": w.ndir,
                   "particles": w.nparticles, "dt": w.dt,
                   "shape": "cic" if w.shape_order == 1 else "tsc",
                   "integrator": "rk4", "launch": sim.tune.as_dict() if sim.tune else "default",
                   "launch_source": "explicit" if args.tuning else "autotuned"},
        "roofline": {"bound": "hbm", "achieved": own, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": own / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"{names[0]}<{dom}>",
                     "alg_bytes_per_launch": own_bytes, "ms_per_launch": stage_ms[dom],
                     "accounting": ACCOUNTING, "contract_bytes_per_launch": alg_bytes,
                     "contract_achieved": achieved, "contract_frac": achieved / HBM_PEAK_GBS},
        "step_roofline": {"alg_bytes_per_step": own_step_bytes,
                          "achieved_GBs": own_step_bytes / (ms_step * 1e-3) / 1e9,
                          "frac": own_step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          # the whole step against the 1872 B stage-synchronous floor
                          "contract_bytes_per_step": step_bytes,
                          "frac_of_1872B_roofline": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "stage_ms": [stage_ms[s] for s in (1, 2, 3, 4)],
                          "reduce_ms": red_ms},
        "event_timing": ev,
        "trace_error": ok,
    }
    if not args.no_extra:
        print("[bench] adjoint/forward on 1d_512x128", file=sys.stderr, flush=True)
        rec["adjoint"] = measure_adjoint()
        print(f"[bench] adjoint: {rec['adjoint']}", file=sys.stderr, flush=True)
        print("[bench] 3D box 64^3 x 92", file=sys.stderr, flush=True)
        rec["box3d"] = measure_3d()
        print(f"[bench] 3d: {rec['box3d']}", file=sys.stderr, flush=True)
        print("[bench] quadratic shape on the same box", file=sys.stderr, flush=True)
        rec["quadratic"] = measure_quadratic()
        print(f"[bench] quadratic: {rec['quadratic']}", file=sys.stderr, flush=True)
        print("[bench] general particle placement", file=sys.stderr, flush=True)
        rec["general_placement"] = measure_particles()
        print(f"[bench] general placement: {rec['general_placement']}", file=sys.stderr, flush=True)
        print("[bench] batched vs sequential (64 uneven 1D boxes)", file=sys.stderr, flush=True)
        rec["batch"] = measure_batch()
        print(f"[bench] batch: {rec['batch']}", file=sys.stderr, flush=True)
    if not args.no_cpu:
        print("[bench] CPU baseline (oracle)", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
