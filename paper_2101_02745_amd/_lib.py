"""ctypes binding of libflavorpic (argument marshalling only).

Every computation happens in the HIP library; this module only converts
Python/torch arguments to the C ABI declared in include/fpic.h.  It raises
if the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflavorpic.so")

FPIC_OK = 0
FPIC_EINVAL = -1
FPIC_EHIP = -2
FPIC_ESTATE = -3
FPIC_ENUMERIC = -4
FPIC_EUNSUPPORTED = -5
_NAMES = {FPIC_EINVAL: "EINVAL", FPIC_EHIP: "EHIP", FPIC_ESTATE: "ESTATE",
          FPIC_ENUMERIC: "ENUMERIC", FPIC_EUNSUPPORTED: "EUNSUPPORTED"}

_dp = C.POINTER(C.c_double)


class FpicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fpic error {_NAMES.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("ncell", C.c_int32 * 3), ("dx", C.c_double * 3),
                ("ndir", C.c_int32), ("dirs", _dp), ("N", _dp), ("Nbar", _dp),
                ("hvac", C.c_double * 18), ("vmat", C.c_double * 3), ("dt", C.c_double),
                ("shape_order", C.c_int32), ("flags", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("waves", C.c_int32), ("dirs_per_wave", C.c_int32),
                ("steps_per_graph", C.c_int32), ("cache_policy", C.c_int32),
                ("fused", C.c_int32)]

    def as_dict(self):
        return {"waves": self.waves, "dirs_per_wave": self.dirs_per_wave,
                "steps_per_graph": self.steps_per_graph, "cache_policy": self.cache_policy,
                "fused": self.fused}


class AdjointCfg(C.Structure):
    _fields_ = [("nsteps", C.c_int64), ("ckpt_every", C.c_int32), ("reserved", C.c_int32)]


class PConfig(C.Structure):
    _fields_ = [("ncell", C.c_int32 * 3), ("dx", C.c_double * 3), ("npart", C.c_int64),
                ("hvac", C.c_double * 18), ("vmat", C.c_double * 3), ("dt", C.c_double),
                ("shape_order", C.c_int32), ("sort_every", C.c_int32), ("flags", C.c_int32),
                ("reserved", C.c_int32)]


EXPORTS = {
    # name: (restype, argtypes)
    "fpic_workspace_bytes": (C.c_int, [C.POINTER(Config), C.POINTER(Tuning), C.POINTER(C.c_size_t)]),
    "fpic_create": (C.c_int, [C.POINTER(Config), C.POINTER(Tuning), C.c_void_p, C.c_size_t,
                              C.c_void_p, C.POINTER(C.c_void_p)]),
    "fpic_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "fpic_get_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fpic_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "fpic_moments": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fpic_flavor_totals": (C.c_int, [C.c_void_p, _dp]),
    "fpic_domain_averages": (C.c_int, [C.c_void_p, C.c_void_p, _dp]),
    "fpic_check": (C.c_int, [C.c_void_p, C.c_double, _dp]),
    "fpic_get_step": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "fpic_sync": (C.c_int, [C.c_void_p]),
    "fpic_destroy": (None, [C.c_void_p]),
    "fpic_last_error": (C.c_char_p, []),
    "fpic_profile": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
    "fpic_batch_workspace_bytes": (C.c_int, [C.c_int32, C.POINTER(Config), C.POINTER(Tuning),
                                             C.POINTER(C.c_size_t)]),
    "fpic_batch_create": (C.c_int, [C.c_int32, C.POINTER(Config), C.POINTER(Tuning), C.c_void_p,
                                    C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "fpic_batch_set_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]),
    "fpic_batch_get_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "fpic_batch_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "fpic_batch_flavor_totals": (C.c_int, [C.c_void_p, _dp]),
    "fpic_batch_sync": (C.c_int, [C.c_void_p]),
    "fpic_batch_destroy": (None, [C.c_void_p]),
    "fpic_batch_profile": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
    "fpic_autotune": (C.c_int, [C.c_int32, C.POINTER(Config), C.c_void_p, C.c_size_t, C.c_void_p,
                                C.POINTER(Tuning), _dp]),
    "fpic_adjoint_workspace_bytes": (C.c_int, [C.c_void_p, C.POINTER(AdjointCfg),
                                               C.POINTER(C.c_size_t)]),
    "fpic_adjoint_forward": (C.c_int, [C.c_void_p, C.POINTER(AdjointCfg), C.c_void_p, C.c_size_t]),
    "fpic_adjoint_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, _dp, _dp]),
    "fpic_step_noalloc": (C.c_int, [C.POINTER(Config), C.POINTER(Tuning), C.c_void_p, C.c_int64,
                                    C.c_int64, C.c_void_p]),
    # general particle placement (include/fpic_particles.h)
    "fpic_particles_workspace_bytes": (C.c_int, [C.POINTER(PConfig), C.POINTER(C.c_size_t)]),
    "fpic_particles_create": (C.c_int, [C.POINTER(PConfig), C.c_void_p, C.c_size_t, C.c_void_p,
                                        C.POINTER(C.c_void_p)]),
    "fpic_particles_set": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int64]),
    "fpic_particles_get_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fpic_particles_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "fpic_particles_moments": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fpic_particles_flavor_totals": (C.c_int, [C.c_void_p, _dp]),
    "fpic_particles_check": (C.c_int, [C.c_void_p, C.c_double, _dp]),
    "fpic_particles_get_step": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "fpic_particles_sync": (C.c_int, [C.c_void_p]),
    "fpic_particles_profile": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
    "fpic_particles_destroy": (None, [C.c_void_p]),
}

_lib = None


def load():
    """Load libflavorpic.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'` "
                "(or python paper_2101_02745_amd/build.py)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc: int):
    if rc != FPIC_OK:
        msg = load().fpic_last_error().decode(errors="replace")
        raise FpicError(rc, msg)


class HostConfig:
    """A Config plus the host arrays it points to (kept alive together)."""

    def __init__(self, ncell, dx, dirs, N, Nbar, hvac, dt, shape_order=1, vmat=None):
        self.dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
        nd = self.dirs.shape[0]
        self.N = np.ascontiguousarray(N, dtype=np.float64).reshape(nd)
        self.Nbar = np.ascontiguousarray(Nbar, dtype=np.float64).reshape(nd)
        H = np.asarray(hvac, dtype=np.complex128).reshape(3, 3)
        h = np.empty(18)
        h[0::2] = H.real.ravel()
        h[1::2] = H.imag.ravel()
        self.ncell = tuple(int(x) for x in ncell)
        self.c = Config()
        self.c.ncell[:] = self.ncell
        self.c.dx[:] = [float(x) for x in dx]
        self.c.ndir = nd
        self.c.dirs = self.dirs.ctypes.data_as(_dp)
        self.c.N = self.N.ctypes.data_as(_dp)
        self.c.Nbar = self.Nbar.ctypes.data_as(_dp)
        self.c.hvac[:] = h.tolist()
        self.c.vmat[:] = [0.0, 0.0, 0.0] if vmat is None else [float(x) for x in vmat]
        self.c.dt = float(dt)
        self.c.shape_order = int(shape_order)
        self.c.flags = 0

    @property
    def ndir(self):
        return self.dirs.shape[0]

    @property
    def ncell_total(self):
        return self.ncell[0] * self.ncell[1] * self.ncell[2]

    @classmethod
    def from_workload(cls, w, hvac=None):
        N, Nbar = w.weights()
        return cls(w.ncell, w.dx, w.dirs(), N, Nbar,
                   w.hvac() if hvac is None else hvac, w.dt,
                   shape_order=w.shape_order, vmat=w.vmat)


def tuning(t) -> Tuning:
    if t is None:
        return None
    if isinstance(t, Tuning):
        return t
    out = Tuning()
    out.waves = int(t.get("waves", 0))
    out.dirs_per_wave = int(t.get("dirs_per_wave", 0))
    out.steps_per_graph = int(t.get("steps_per_graph", 0))
    out.cache_policy = int(t.get("cache_policy", 0))
    out.fused = int(t.get("fused", 0))
    return out


FPIC_PFLOAT_ATOMICS = 1


def pconfig(ncell, dx, npart, hvac, dt, shape_order=1, vmat=None, sort_every=0,
            exact=True) -> PConfig:
    """PConfig for a general-placement box (hvac: 3x3 complex); exact=False
    deposits with floating-point atomics (FPIC_PFLOAT_ATOMICS)."""
    H = np.asarray(hvac, dtype=np.complex128).reshape(3, 3)
    h = np.empty(18)
    h[0::2] = H.real.ravel()
    h[1::2] = H.imag.ravel()
    c = PConfig()
    c.ncell[:] = [int(x) for x in ncell]
    c.dx[:] = [float(x) for x in dx]
    c.npart = int(npart)
    c.hvac[:] = h.tolist()
    c.vmat[:] = [0.0, 0.0, 0.0] if vmat is None else [float(x) for x in vmat]
    c.dt = float(dt)
    c.shape_order = int(shape_order)
    c.sort_every = int(sort_every)
    c.flags = 0 if exact else FPIC_PFLOAT_ATOMICS
    return c
