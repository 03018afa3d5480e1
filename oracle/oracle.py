"""ctypes binding of the CPU FP64 reference (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this module.  It wraps ``fpic_oracle.c``; see that file for what each
routine computes and which passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FPIC_ORACLE_LIB lets the mutation test load a deliberately broken build.
LIB_PATH = os.environ.get("FPIC_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)


class _Problem(C.Structure):
    _fields_ = [("ncell", C.c_int64 * 3), ("dx", C.c_double * 3),
                ("ndir", C.c_int64), ("dirs", _dp), ("N", _dp),
                ("Nbar", _dp), ("Hvac", _dp), ("dt", C.c_double), ("Vmat", _dp),
                ("shape_order", C.c_int32), ("npart", C.c_int64), ("pos0", _dp),
                ("pdirs", _dp), ("pN", _dp), ("pNbar", _dp)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        P = C.POINTER(_Problem)
        for name, args in {
            "oracle_rhs": [P, _dp, C.c_double, _dp],
            "oracle_step": [P, _dp, C.c_int64, C.c_int64],
            "oracle_moments": [P, _dp, C.c_double, _dp],
            "oracle_gather": [P, _dp, C.c_int64, C.c_double, _dp],
            "oracle_flavor_totals": [P, _dp, _dp],
            "oracle_adjoint": [P, _dp, C.c_int64, C.c_int64, _dp, _dp, _dp],
        }.items():
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = C.c_int
        _lib.oracle_set_threads.argtypes = [C.c_int]
        _lib.oracle_set_threads.restype = C.c_int
    return _lib


def set_threads(n: int) -> int:
    """Set the OpenMP thread count (n <= 0 keeps it); returns the count."""
    return lib().oracle_set_threads(int(n))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


class Problem:
    """A periodic box with one particle per direction per cell.

    ncell: (nx, ny, nz); dx: cell widths; dirs [ndir][3]; N, Nbar [ndir]
    (neutrinos per particle); hvac: 3x3 complex; dt: time step; vmat: the
    matter potentials (V_e, V_mu, V_tau) of the background charged leptons
    (eq. potentials; zero by default); shape_order: 1 linear (cloud in
    cell), 2 quadratic (Sec. II.B.1).
    """

    def __init__(self, ncell, dx, dirs, N, Nbar, hvac, dt: float, vmat=None, shape_order=1):
        self.ncell = tuple(int(n) for n in ncell)
        self.dx = tuple(float(x) for x in dx)
        self.dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
        self.ndir = self.dirs.shape[0]
        self.N = np.ascontiguousarray(N, dtype=np.float64).reshape(self.ndir)
        self.Nbar = np.ascontiguousarray(Nbar, dtype=np.float64).reshape(self.ndir)
        H = np.asarray(hvac, dtype=np.complex128).reshape(3, 3)
        h = np.empty(18)
        h[0::2] = H.real.ravel()
        h[1::2] = H.imag.ravel()
        self.hvac = h
        self.dt = float(dt)
        self.vmat = np.zeros(3) if vmat is None else np.ascontiguousarray(vmat, dtype=np.float64).reshape(3)
        self._s = _Problem((C.c_int64 * 3)(*self.ncell), (C.c_double * 3)(*self.dx),
                           self.ndir, _ptr(self.dirs), _ptr(self.N),
                           _ptr(self.Nbar), _ptr(self.hvac), self.dt, _ptr(self.vmat),
                           int(shape_order))
        self.shape_order = int(shape_order)

    @classmethod
    def from_workload(cls, w, hvac=None) -> "Problem":
        N, Nbar = w.weights()
        return cls(w.ncell, w.dx, w.dirs(), N, Nbar,
                   w.hvac() if hvac is None else hvac, w.dt, vmat=w.vmat,
                   shape_order=w.shape_order)

    @property
    def ncell_total(self) -> int:
        return self.ncell[0] * self.ncell[1] * self.ncell[2]

    def _state(self, state: np.ndarray) -> np.ndarray:
        s = np.ascontiguousarray(state, dtype=np.float64)
        if s.size != 18 * self.ndir * self.ncell_total:
            raise ValueError("state has the wrong size")
        return s

    def step(self, state: np.ndarray, nsteps: int, n0: int = 0) -> np.ndarray:
        """Return the state after nsteps RK4 steps from step number n0."""
        s = self._state(state).copy()
        if lib().oracle_step(C.byref(self._s), _ptr(s), int(n0), int(nsteps)):
            raise MemoryError("oracle_step failed")
        return s.reshape(18, self.ndir, self.ncell_total)

    def rhs(self, state: np.ndarray, t: float) -> np.ndarray:
        s = self._state(state)
        out = np.empty_like(s)
        if lib().oracle_rhs(C.byref(self._s), _ptr(s), float(t), _ptr(out)):
            raise MemoryError("oracle_rhs failed")
        return out.reshape(18, self.ndir, self.ncell_total)

    def moments(self, state: np.ndarray, t: float) -> np.ndarray:
        s = self._state(state)
        out = np.empty((72, self.ncell_total))
        if lib().oracle_moments(C.byref(self._s), _ptr(s), float(t), _ptr(out)):
            raise MemoryError("oracle_moments failed")
        return out

    def gather(self, G: np.ndarray, t: float) -> np.ndarray:
        G = np.ascontiguousarray(G, dtype=np.float64).reshape(-1, self.ncell_total)
        out = np.empty((G.shape[0], self.ndir, self.ncell_total))
        lib().oracle_gather(C.byref(self._s), _ptr(G), G.shape[0], float(t), _ptr(out))
        return out

    def adjoint(self, state0: np.ndarray, nsteps: int, dL_dfinal: np.ndarray, n0: int = 0):
        """Reference reverse mode: returns (dL/dstate0, dL/dN, dL/dNbar) for a
        loss whose gradient with respect to the state after nsteps steps is
        dL_dfinal."""
        s = self._state(state0)
        lam = self._state(dL_dfinal).copy()
        gN = np.zeros(self.ndir)
        gNb = np.zeros(self.ndir)
        if lib().oracle_adjoint(C.byref(self._s), _ptr(s), int(n0), int(nsteps), _ptr(lam),
                                _ptr(gN), _ptr(gNb)):
            raise MemoryError("oracle_adjoint failed")
        return lam.reshape(18, self.ndir, self.ncell_total), gN, gNb

    def flavor_totals(self, state: np.ndarray) -> np.ndarray:
        s = self._state(state)
        out = np.empty((2, 9))
        lib().oracle_flavor_totals(C.byref(self._s), _ptr(s), _ptr(out))
        return out


class ParticleProblem:
    """General placement: npart particles anywhere in the periodic box, with
    their own positions pos0 [npart][3] at t = 0, unit directions
    [npart][3] and weights N, Nbar [npart]; any number of particles per
    cell.  State layout [18][npart]."""

    def __init__(self, ncell, dx, pos0, dirs, N, Nbar, hvac, dt: float, vmat=None,
                 shape_order=1):
        self.ncell = tuple(int(n) for n in ncell)
        self.dx = tuple(float(x) for x in dx)
        self.pos0 = np.ascontiguousarray(pos0, dtype=np.float64).reshape(-1, 3)
        self.npart = self.pos0.shape[0]
        self.dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(self.npart, 3)
        self.N = np.ascontiguousarray(N, dtype=np.float64).reshape(self.npart)
        self.Nbar = np.ascontiguousarray(Nbar, dtype=np.float64).reshape(self.npart)
        H = np.asarray(hvac, dtype=np.complex128).reshape(3, 3)
        h = np.empty(18)
        h[0::2] = H.real.ravel()
        h[1::2] = H.imag.ravel()
        self.hvac = h
        self.dt = float(dt)
        self.vmat = np.zeros(3) if vmat is None else np.ascontiguousarray(vmat, dtype=np.float64).reshape(3)
        self.shape_order = int(shape_order)
        self._s = _Problem((C.c_int64 * 3)(*self.ncell), (C.c_double * 3)(*self.dx),
                           0, None, None, None, _ptr(self.hvac), self.dt, _ptr(self.vmat),
                           self.shape_order, self.npart, _ptr(self.pos0), _ptr(self.dirs),
                           _ptr(self.N), _ptr(self.Nbar))

    @property
    def ncell_total(self) -> int:
        return self.ncell[0] * self.ncell[1] * self.ncell[2]

    def _state(self, state: np.ndarray) -> np.ndarray:
        s = np.ascontiguousarray(state, dtype=np.float64)
        if s.size != 18 * self.npart:
            raise ValueError("state has the wrong size")
        return s

    def step(self, state: np.ndarray, nsteps: int, n0: int = 0) -> np.ndarray:
        """Return the state after nsteps RK4 steps from step number n0."""
        s = self._state(state).copy()
        if lib().oracle_step(C.byref(self._s), _ptr(s), int(n0), int(nsteps)):
            raise MemoryError("oracle_step failed")
        return s.reshape(18, self.npart)

    def rhs(self, state: np.ndarray, t: float) -> np.ndarray:
        s = self._state(state)
        out = np.empty_like(s)
        if lib().oracle_rhs(C.byref(self._s), _ptr(s), float(t), _ptr(out)):
            raise MemoryError("oracle_rhs failed")
        return out.reshape(18, self.npart)

    def moments(self, state: np.ndarray, t: float) -> np.ndarray:
        s = self._state(state)
        out = np.empty((72, self.ncell_total))
        if lib().oracle_moments(C.byref(self._s), _ptr(s), float(t), _ptr(out)):
            raise MemoryError("oracle_moments failed")
        return out

    def gather(self, G: np.ndarray, t: float) -> np.ndarray:
        G = np.ascontiguousarray(G, dtype=np.float64).reshape(-1, self.ncell_total)
        out = np.empty((G.shape[0], self.npart))
        lib().oracle_gather(C.byref(self._s), _ptr(G), G.shape[0], float(t), _ptr(out))
        return out

    def flavor_totals(self, state: np.ndarray) -> np.ndarray:
        s = self._state(state)
        out = np.empty((2, 9))
        lib().oracle_flavor_totals(C.byref(self._s), _ptr(s), _ptr(out))
        return out
