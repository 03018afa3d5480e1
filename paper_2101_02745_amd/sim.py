"""Python front end of libflavorpic: Sim (one box) and Batch (many 1D
boxes).  Torch provides the device workspace and the stream; every step of
the method runs in the HIP library."""
from __future__ import annotations

import ctypes as C
import hashlib
import json
import os
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import HostConfig, check


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev_ptr(t: torch.Tensor, n: int, device) -> int:
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    if t.device != torch.device(device):
        raise ValueError("tensor is on another device")
    return t.data_ptr()


class Sim:
    """One periodic box (1D: ncell = (1, 1, nz); 3D otherwise)."""

    def __init__(self, cfg: HostConfig, tuning: Optional[dict] = None,
                 device: str = "cuda:0"):
        lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libflavorpic needs a HIP device")
        self.device = torch.device(device)
        self.cfg = cfg
        self.tune = _lib.tuning(tuning)
        tp = C.byref(self.tune) if self.tune is not None else None
        nbytes = C.c_size_t()
        check(lib.fpic_workspace_bytes(C.byref(cfg.c), tp, C.byref(nbytes)))
        self.nbytes = nbytes.value
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib.fpic_create(C.byref(cfg.c), tp, self.ws.data_ptr(), self.nbytes,
                                  _stream_ptr(self.device), C.byref(ctx)))
        self.ctx = ctx

    @classmethod
    def from_workload(cls, w, hvac=None, tuning=None, device="cuda:0"):
        return cls(HostConfig.from_workload(w, hvac), tuning, device)

    @property
    def shape(self):
        return (18, self.cfg.ndir, self.cfg.ncell_total)

    @property
    def nparticles(self) -> int:
        return self.cfg.ndir * self.cfg.ncell_total

    def set_state(self, state, step0: int = 0):
        if isinstance(state, np.ndarray):
            state = torch.from_numpy(np.ascontiguousarray(state, dtype=np.float64)).to(self.device)
        n = int(np.prod(self.shape))
        check(_lib.load().fpic_set_state(self.ctx, _dev_ptr(state, n, self.device), int(step0)))
        self._keep = state   # stream-ordered copy: keep the source alive

    def get_state(self) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        check(_lib.load().fpic_get_state(self.ctx, out.data_ptr()))
        return out

    def step(self, nsteps: int = 1):
        check(_lib.load().fpic_step(self.ctx, int(nsteps)))

    def moments(self) -> torch.Tensor:
        out = torch.empty((72, self.cfg.ncell_total), dtype=torch.float64, device=self.device)
        check(_lib.load().fpic_moments(self.ctx, out.data_ptr()))
        return out

    def flavor_totals(self) -> np.ndarray:
        out = np.empty(18)
        check(_lib.load().fpic_flavor_totals(self.ctx, out.ctypes.data_as(_lib._dp)))
        return out.reshape(2, 9)

    def domain_averages(self, moments: Optional[torch.Tensor] = None) -> dict:
        """Domain averages of the moment magnitudes (Sec. III.B): <|n_ab|> and
        <|f^(x)_ab|> for neutrinos and antineutrinos, reduced on the device
        from `moments` ([72][ncell], default: this box's moments now)."""
        if moments is None:
            moments = self.moments()
        out = np.empty(24)
        check(_lib.load().fpic_domain_averages(
            self.ctx, _dev_ptr(moments, 72 * self.cfg.ncell_total, self.device),
            out.ctypes.data_as(_lib._dp)))
        return unpack_domain_averages(out)

    def check(self, tol: float = 1e-10) -> float:
        e = C.c_double()
        check(_lib.load().fpic_check(self.ctx, float(tol), C.byref(e)))
        return e.value

    def step_index(self) -> int:
        s = C.c_int64()
        check(_lib.load().fpic_get_step(self.ctx, C.byref(s)))
        return s.value

    def sync(self):
        check(_lib.load().fpic_sync(self.ctx))

    def profile(self, nsteps: int = 10) -> np.ndarray:
        """Mean ms per launch of [stage1, reduce1, ..., stage4, reduce4],
        measured with HIP events on the context's stream (advances the
        state by nsteps)."""
        out = np.empty(8)
        check(_lib.load().fpic_profile(self.ctx, int(nsteps), out.ctypes.data_as(_lib._dp)))
        return out

    def adjoint_forward(self, nsteps: int, ckpt_every: int = 50):
        """Advance nsteps steps, storing checkpoints for adjoint_backward."""
        lib = _lib.load()
        a = _lib.AdjointCfg(int(nsteps), int(ckpt_every), 0)
        nb = C.c_size_t()
        check(lib.fpic_adjoint_workspace_bytes(self.ctx, C.byref(a), C.byref(nb)))
        if getattr(self, "adj_ws", None) is None or self.adj_ws.numel() < nb.value:
            self.adj_ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        check(lib.fpic_adjoint_forward(self.ctx, C.byref(a), self.adj_ws.data_ptr(),
                                       self.adj_ws.numel()))

    def adjoint_backward(self, dL_dfinal):
        """Returns (dL/d(start state) [device tensor], dL/dN, dL/dNbar)."""
        if isinstance(dL_dfinal, np.ndarray):
            dL_dfinal = torch.from_numpy(np.ascontiguousarray(dL_dfinal)).to(self.device)
        n = int(np.prod(self.shape))
        g0 = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        gN = np.zeros(self.cfg.ndir)
        gNb = np.zeros(self.cfg.ndir)
        check(_lib.load().fpic_adjoint_backward(self.ctx, _dev_ptr(dL_dfinal, n, self.device),
                                                g0.data_ptr(), gN.ctypes.data_as(_lib._dp),
                                                gNb.ctypes.data_as(_lib._dp)))
        return g0, gN, gNb

    def close(self):
        if getattr(self, "ctx", None):
            _lib.load().fpic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent 1D boxes advanced together (one launch per stage)."""

    def __init__(self, cfgs: Sequence[HostConfig], tuning: Optional[dict] = None,
                 device: str = "cuda:0"):
        lib = _lib.load()
        self.device = torch.device(device)
        self.cfgs = list(cfgs)
        arr = (_lib.Config * len(self.cfgs))(*[c.c for c in self.cfgs])
        self._arr = arr
        self.tune = _lib.tuning(tuning)
        tp = C.byref(self.tune) if self.tune is not None else None
        nbytes = C.c_size_t()
        check(lib.fpic_batch_workspace_bytes(len(self.cfgs), arr, tp, C.byref(nbytes)))
        self.nbytes = nbytes.value
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        b = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib.fpic_batch_create(len(self.cfgs), arr, tp, self.ws.data_ptr(), self.nbytes,
                                        _stream_ptr(self.device), C.byref(b)))
        self.b = b
        self._keep = []

    @property
    def nsim(self):
        return len(self.cfgs)

    def shape(self, i):
        return (18, self.cfgs[i].ndir, self.cfgs[i].ncell_total)

    @property
    def nparticles(self) -> int:
        return sum(c.ndir * c.ncell_total for c in self.cfgs)

    def set_state(self, i: int, state, step0: int = 0):
        if isinstance(state, np.ndarray):
            state = torch.from_numpy(np.ascontiguousarray(state, dtype=np.float64)).to(self.device)
        n = int(np.prod(self.shape(i)))
        check(_lib.load().fpic_batch_set_state(self.b, int(i), _dev_ptr(state, n, self.device),
                                               int(step0)))
        self._keep.append(state)

    def get_state(self, i: int) -> torch.Tensor:
        out = torch.empty(self.shape(i), dtype=torch.float64, device=self.device)
        check(_lib.load().fpic_batch_get_state(self.b, int(i), out.data_ptr()))
        return out

    def step(self, nsteps: int = 1):
        check(_lib.load().fpic_batch_step(self.b, int(nsteps)))
        self._keep = []

    def flavor_totals(self) -> np.ndarray:
        out = np.empty(18 * self.nsim)
        check(_lib.load().fpic_batch_flavor_totals(self.b, out.ctypes.data_as(_lib._dp)))
        return out.reshape(self.nsim, 2, 9)

    def sync(self):
        check(_lib.load().fpic_batch_sync(self.b))

    def profile(self, nsteps: int = 10) -> np.ndarray:
        """Mean ms per launch of [stage1, reduce1, ..., stage4, reduce4] over
        all boxes, measured with HIP events on the batch's stream (advances
        every box by nsteps)."""
        out = np.empty(8)
        check(_lib.load().fpic_batch_profile(self.b, int(nsteps), out.ctypes.data_as(_lib._dp)))
        return out

    def close(self):
        if getattr(self, "b", None):
            _lib.load().fpic_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def unpack_domain_averages(out24) -> dict:
    """The 4 x 6 averages of fpic_domain_averages as 3x3 arrays (diagonal
    and upper triangle filled): keys 'n', 'fx', 'nbar', 'fxbar'."""
    out = {}
    v = np.asarray(out24).reshape(4, 6)
    for f, name in enumerate(("n", "fx", "nbar", "fxbar")):
        a = np.zeros((3, 3))
        for i in range(3):
            a[i, i] = v[f, i]
        a[0, 1], a[0, 2], a[1, 2] = v[f, 3], v[f, 4], v[f, 5]
        out[name] = a
    return out


TUNING_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def device_key(device="cuda:0") -> str:
    """The device part of a tuning-cache key: the GPU architecture and its
    compute-unit count."""
    p = torch.cuda.get_device_properties(torch.device(device))
    return f"{getattr(p, 'gcnArchName', p.name)}/{p.multi_processor_count}cu"


def shape_key(cfgs: Sequence[HostConfig]) -> str:
    """The box part of a tuning-cache key: cell counts, direction counts and
    shape orders of the boxes (a batch lists every box)."""
    desc = [[list(c.ncell), c.ndir, int(c.c.shape_order)] for c in cfgs]
    if len(desc) == 1:
        return json.dumps(desc[0], separators=(",", ""))
    h = hashlib.sha256(json.dumps(desc).encode()).hexdigest()[:16]
    return f"batch{len(desc)}:{h}"


def _read_cache(path):
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return {}


def autotune(cfgs: Sequence[HostConfig], device: str = "cuda:0", workspace_bytes=None,
             cache: Optional[str] = TUNING_CACHE, retune: bool = False):
    """Launch shape for these boxes on this device, and its ms per step.

    The shape is taken from the JSON cache (keyed by device and box shapes)
    when it holds one, else measured on the device with fpic_autotune and
    stored in the cache (cache=None: neither read nor written; retune:
    measure and overwrite)."""
    cfgs = list(cfgs)
    key = f"{device_key(device)}|{shape_key(cfgs)}"
    if cache and not retune:
        ent = _read_cache(cache).get(key)
        if ent:
            return dict(ent["launch"]), float(ent["ms_per_step"])
    tune, ms = measure_launch(cfgs, device, workspace_bytes)
    if cache:
        rec = _read_cache(cache)
        rec[key] = {"launch": tune, "ms_per_step": ms}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return tune, ms


def measure_launch(cfgs: Sequence[HostConfig], device: str = "cuda:0", workspace_bytes=None):
    """Time candidate launch shapes on the device (fpic_autotune); returns
    (tuning dict, ms per step)."""
    lib = _lib.load()
    dev = torch.device(device)
    cfgs = list(cfgs)
    arr = (_lib.Config * len(cfgs))(*[c.c for c in cfgs])
    if workspace_bytes is None:
        # the smallest shape (1 wave, 1 direction) needs the most partials
        t = _lib.Tuning()
        t.waves, t.dirs_per_wave, t.steps_per_graph = 1, 1, 8
        nb = C.c_size_t()
        if len(cfgs) == 1 and cfgs[0].ncell[0] * cfgs[0].ncell[1] > 1:
            check(lib.fpic_workspace_bytes(C.byref(cfgs[0].c), None, C.byref(nb)))
            workspace_bytes = nb.value * 2
        else:
            check(lib.fpic_batch_workspace_bytes(len(cfgs), arr, C.byref(t), C.byref(nb)))
            workspace_bytes = nb.value
    ws = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=dev)
    best = _lib.Tuning()
    ms = C.c_double()
    with torch.cuda.device(dev):
        check(lib.fpic_autotune(len(cfgs), arr, ws.data_ptr(), int(workspace_bytes),
                                _stream_ptr(dev), C.byref(best), C.byref(ms)))
    torch.cuda.synchronize(dev)
    return best.as_dict(), ms.value


def step_noalloc(cfg: HostConfig, state: torch.Tensor, nsteps: int, step0: int = 0,
                 tuning: Optional[dict] = None):
    """Advance a 1D box's state (contiguous float64 tensor [18][ndir][ncell]
    on the current device) by nsteps RK4 steps from step number step0, in
    place, through fpic_step_noalloc: no device memory is allocated, the
    library's fixed scratch array holds every other buffer."""
    lib = _lib.load()
    dev = state.device
    n = 18 * cfg.ndir * cfg.ncell_total
    t = _lib.tuning(tuning)
    with torch.cuda.device(dev):
        check(lib.fpic_step_noalloc(C.byref(cfg.c), C.byref(t) if t is not None else None,
                                    _dev_ptr(state, n, dev), int(step0), int(nsteps),
                                    _stream_ptr(dev)))
    return state
