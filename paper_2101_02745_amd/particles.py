"""Python front end of the general-placement path of libflavorpic
(include/fpic_particles.h): particles anywhere in the box, any number per
cell.  Torch provides the device workspace and the stream; every step runs
in the HIP library."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check
from .sim import _dev_ptr, _stream_ptr


def _device_array(a, shape, device) -> torch.Tensor:
    """Contiguous float64 device tensor of the given shape from a numpy
    array or a tensor."""
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
    t = a.to(device=device, dtype=torch.float64).contiguous()
    if tuple(t.shape) != tuple(shape):
        t = t.reshape(shape)
    return t


class ParticleSim:
    """One periodic box (1D: ncell = (1, 1, nz); 3D otherwise) with npart
    particles placed anywhere."""

    def __init__(self, ncell, dx, npart: int, hvac, dt: float, shape_order: int = 1,
                 vmat=None, sort_every: int = 0, device: str = "cuda:0", exact: bool = True):
        lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libflavorpic needs a HIP device")
        self.device = torch.device(device)
        self.ncell = tuple(int(x) for x in ncell)
        self.npart = int(npart)
        self.cfg = _lib.pconfig(ncell, dx, npart, hvac, dt, shape_order, vmat, sort_every, exact)
        nbytes = C.c_size_t()
        check(lib.fpic_particles_workspace_bytes(C.byref(self.cfg), C.byref(nbytes)))
        self.nbytes = nbytes.value
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib.fpic_particles_create(C.byref(self.cfg), self.ws.data_ptr(), self.nbytes,
                                            _stream_ptr(self.device), C.byref(ctx)))
        self.ctx = ctx

    @classmethod
    def from_workload(cls, w, sort_every: int = 0, device: str = "cuda:0", exact: bool = True):
        return cls(w.ncell, w.dx, w.nparticles, w.hvac(), w.dt, w.shape_order, w.vmat,
                   sort_every, device, exact)

    @property
    def ncell_total(self) -> int:
        return self.ncell[0] * self.ncell[1] * self.ncell[2]

    def set(self, pos0, dirs, N, Nbar, state, step0: int = 0):
        """pos0, dirs: [npart][3] (positions at t = 0, unit directions);
        N, Nbar: [npart]; state: [18][npart]."""
        n = self.npart
        p = _device_array(pos0, (n, 3), self.device).t().contiguous()
        d = _device_array(dirs, (n, 3), self.device).t().contiguous()
        a = _device_array(N, (n,), self.device)
        b = _device_array(Nbar, (n,), self.device)
        s = _device_array(state, (18, n), self.device)
        check(_lib.load().fpic_particles_set(self.ctx, _dev_ptr(p, 3 * n, self.device),
                                             _dev_ptr(d, 3 * n, self.device),
                                             _dev_ptr(a, n, self.device),
                                             _dev_ptr(b, n, self.device),
                                             _dev_ptr(s, 18 * n, self.device), int(step0)))

    def set_workload(self, w, state=None, step0: int = 0):
        N, Nb = w.weights()
        self.set(w.positions(), w.dirs(), N, Nb, w.state0() if state is None else state, step0)

    def get_state(self) -> torch.Tensor:
        out = torch.empty((18, self.npart), dtype=torch.float64, device=self.device)
        check(_lib.load().fpic_particles_get_state(self.ctx, out.data_ptr()))
        return out

    def step(self, nsteps: int = 1):
        check(_lib.load().fpic_particles_step(self.ctx, int(nsteps)))

    def moments(self) -> torch.Tensor:
        out = torch.empty((72, self.ncell_total), dtype=torch.float64, device=self.device)
        check(_lib.load().fpic_particles_moments(self.ctx, out.data_ptr()))
        return out

    def flavor_totals(self) -> np.ndarray:
        out = np.empty(18)
        check(_lib.load().fpic_particles_flavor_totals(self.ctx, out.ctypes.data_as(_lib._dp)))
        return out.reshape(2, 9)

    def check(self, tol: float = 1e-10) -> float:
        e = C.c_double()
        check(_lib.load().fpic_particles_check(self.ctx, float(tol), C.byref(e)))
        return e.value

    def step_index(self) -> int:
        s = C.c_int64()
        check(_lib.load().fpic_particles_get_step(self.ctx, C.byref(s)))
        return s.value

    def sync(self):
        check(_lib.load().fpic_particles_sync(self.ctx))

    def profile(self, nsteps: int = 10) -> np.ndarray:
        """Mean ms of stage 1..4, the sort and the whole step (kernels
        launched one by one, sorting after every step)."""
        ms = np.empty(6)
        check(_lib.load().fpic_particles_profile(self.ctx, int(nsteps), ms.ctypes.data_as(_lib._dp)))
        return ms

    def close(self):
        if getattr(self, "ctx", None):
            _lib.load().fpic_particles_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
