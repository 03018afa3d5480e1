"""Seeded synthetic inputs for the particle-in-cell flavor solver.

This module only *generates input arrays*; it holds none of the solver's
arithmetic (no deposit, interpolation, Hamiltonian or time stepping).  Both
the HIP library and the CPU reference consume what it produces.

Contents
--------
* Direction sets
  - ``ring_directions(C)``: latitude-ring ("polar coordinate subdivision")
    set parameterised by the number of equatorial points C (Sec. III.A and
    App. B of the paper: C = 4, 8, 16, 32, 128 give 6, 24, 92, 378, 6022
    directions per cell).
  - ``golden_antipodal_directions(n)``: an antipodally symmetric golden-angle
    spiral for direction counts the ring rule cannot produce (26, 64, 128).
* Particle weights N, Nbar from a target density and flux (Sec. III.A,
  the weight formula N_p = (n + 3 f.Omega) dV / N_ppz).
* The initial flavor state (Sec. III.A, eq. initial_flavor_state): near-pure
  electron flavor with uniform random off-diagonal seeds of amplitude alpha.
* The vacuum Hamiltonian U diag(0, w21, w31) U^dagger (Sec. II.A,
  eq. potentials), with U in the standard three-angle parameterisation.
* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) as a counter-based generator
  for the uniform draws U in [-1, 1].
* Named workloads (``workload(name)``) with the sizes used by the tests and
  the benchmark.
* General particle placement (``ParticleWorkload``, ``particle_workload``):
  particles anywhere in the box, several per cell, with their own positions,
  directions and weights.

State layout shared by every consumer: ``state[18][ndir][ncell]`` float64.
Component k of the 18 is

====  ==========================  ====  =========================
 k    neutrino rho                 k    antineutrino rhobar
====  ==========================  ====  =========================
 0    rho_ee                        9    rhobar_ee
 1    rho_mumu                     10    rhobar_mumu
 2    rho_tautau                   11    rhobar_tautau
 3,4  Re, Im rho_emu               12,13 Re, Im rhobar_emu
 5,6  Re, Im rho_etau              14,15 Re, Im rhobar_etau
 7,8  Re, Im rho_mutau             16,17 Re, Im rhobar_mutau
====  ==========================  ====  =========================

Only the diagonal and the upper triangle are stored (Sec. II.B: the lower
triangle of a Hermitian matrix follows from the upper one).  Cells are
numbered x fastest: ``cell = (z * ny + y) * nx + x``.  Particle (d, c)
starts at the centre of cell c and moves along direction d.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

NCOMP = 18  # reals per particle: 9 for rho, 9 for rhobar

# ---------------------------------------------------------------------------
# SplitMix64
# ---------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (the published finaliser)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_stream(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    """Counter-based SplitMix64: the ``index``-th output of the generator whose
    initial state is ``mix(seed) ^ mix(stream + gamma)``.

    SplitMix64 advances its state by the constant gamma and applies the
    finaliser, so output i is ``mix(state0 + (i + 1) * gamma)``; that closed
    form lets every draw be computed independently.
    """
    s0 = _mix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF)) ^ _mix64(
        np.uint64((stream + 0x632BE59BD9B4E019) & 0xFFFFFFFFFFFFFFFF))
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(s0 + (idx + np.uint64(1)) * _GAMMA)


def uniform_pm1(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    """Uniform doubles in [-1, 1): 53 high bits of the SplitMix64 output."""
    bits = splitmix64_stream(seed, stream, index) >> np.uint64(11)
    return 2.0 * bits.astype(np.float64) * (2.0 ** -53) - 1.0


# ---------------------------------------------------------------------------
# Direction sets
# ---------------------------------------------------------------------------
def ring_directions(C: int) -> np.ndarray:
    """Latitude-ring direction set with C points on the equator.

    Rings sit at latitudes 0, h, 2h, ... below 90 degrees with
    h = sqrt(3) * pi / C; the ring at latitude theta carries
    round(C cos theta) equally spaced points (every other ring is rotated by
    half a spacing); every ring above the equator is mirrored below it with
    antipodal points.  When a ring would carry one point or fewer the set is
    closed with the two poles.  This reproduces the counts printed in the
    paper (C = 4, 8, 16, 32, 128 -> 6, 24, 92, 378, 6022) and gives about
    C^2 / pi directions.
    """
    if C < 2:
        raise ValueError("need at least 2 equatorial points")
    h = math.sqrt(3.0) * math.pi / C
    pts: List[np.ndarray] = []

    def ring(theta: float, n: int, offset: float) -> np.ndarray:
        phi = 2.0 * math.pi * (np.arange(n) + offset) / n
        ct = math.cos(theta)
        return np.stack([ct * np.cos(phi), ct * np.sin(phi),
                         np.full(n, math.sin(theta))], axis=1)

    pts.append(ring(0.0, C, 0.0))
    k = 1
    while True:
        theta = k * h
        if theta >= 0.5 * math.pi:
            break
        n = int(round(C * math.cos(theta)))
        if n <= 1:
            pole = np.array([[0.0, 0.0, 1.0]])
            pts.append(pole)
            pts.append(-pole)
            break
        upper = ring(theta, n, 0.5 * (k % 2))
        pts.append(upper)
        pts.append(-upper)
        k += 1
    return np.ascontiguousarray(np.concatenate(pts, axis=0))


def golden_antipodal_directions(n: int) -> np.ndarray:
    """n (even) nearly uniform unit vectors closed under v -> -v.

    n/2 points on a golden-angle spiral over the upper hemisphere,
    z_i = 1 - (i + 1/2) / (n/2), azimuth i * pi * (3 - sqrt 5), followed by
    their exact negatives, so the set sums to zero exactly.
    """
    if n < 2 or n % 2:
        raise ValueError("golden antipodal set needs an even count >= 2")
    m = n // 2
    i = np.arange(m, dtype=np.float64)
    z = 1.0 - (i + 0.5) / m
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    up = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    return np.ascontiguousarray(np.concatenate([up, -up], axis=0))


_RING_COUNTS = {}


def ring_count(C: int) -> int:
    if C not in _RING_COUNTS:
        _RING_COUNTS[C] = ring_directions(C).shape[0]
    return _RING_COUNTS[C]


def directions(ndir: int) -> np.ndarray:
    """Ring set when ndir is one of its counts (C <= 160), otherwise the
    golden antipodal set (ndir must then be even)."""
    for C in range(2, 161):
        if ring_count(C) == ndir:
            return ring_directions(C)
    return golden_antipodal_directions(ndir)


# ---------------------------------------------------------------------------
# Weights, initial state, vacuum Hamiltonian
# ---------------------------------------------------------------------------
def particle_weights(dirs: np.ndarray, dV: float, n: float = 1.0,
                     f: float = 0.0, nbar_over_n: float = 1.0,
                     fbar: float = -1.0 / 3.0,
                     nhat: Sequence[float] = (0.0, 0.0, 1.0)):
    """Weights giving an angular distribution n (1 + 3 f Omega.nhat) from an
    isotropic particle set (Sec. III.A weight formula, with
    f_input = f n nhat and fbar_input = fbar nbar nhat).

    Returns (N, Nbar) in physical neutrinos per particle.
    """
    dirs = np.asarray(dirs, dtype=np.float64)
    nh = np.asarray(nhat, dtype=np.float64)
    nh = nh / np.linalg.norm(nh)
    ndir = dirs.shape[0]
    mu = dirs @ nh
    N = n * (1.0 + 3.0 * f * mu) * dV / ndir
    Nbar = nbar_over_n * n * (1.0 + 3.0 * fbar * mu) * dV / ndir
    return np.ascontiguousarray(N), np.ascontiguousarray(Nbar)


def seed_draws(ndir: int, ncell: int, seed: int, sim: int = 0) -> np.ndarray:
    """The eight uniform draws U in [-1, 1) of every particle,
    shape [8][ndir][ncell].  Slots 0-3: Re/Im rho_emu, Re/Im rho_etau;
    slots 4-7: the same for rhobar.  Draw (slot, d, c) is output number
    ((d * ncell + c) * 8 + slot) of stream ``sim`` of ``seed``."""
    p = np.arange(ndir * ncell, dtype=np.uint64).reshape(ndir, ncell)
    out = np.empty((8, ndir, ncell), dtype=np.float64)
    for s in range(8):
        out[s] = uniform_pm1(seed, sim, p * np.uint64(8) + np.uint64(s))
    return out


def state_from_seeds(offdiag: np.ndarray) -> np.ndarray:
    """Initial state from the off-diagonal seeds (eq. initial_flavor_state).

    ``offdiag`` is [8][ndir][ncell]: alpha*U for Re/Im rho_emu, Re/Im
    rho_etau, then the same four for rhobar.  rho_mutau = 0, and the
    diagonal is eps_mu = |rho_emu|^2, eps_tau = |rho_etau|^2,
    rho_ee = 1 - eps_mu - eps_tau (unit trace; the flavor-vector length is
    then one up to O(alpha^4)).
    """
    s = np.asarray(offdiag, dtype=np.float64)
    ndir, ncell = s.shape[1], s.shape[2]
    st = np.zeros((NCOMP, ndir, ncell), dtype=np.float64)
    for base, o in ((0, 0), (9, 4)):
        emu_r, emu_i, etau_r, etau_i = s[o], s[o + 1], s[o + 2], s[o + 3]
        eps_mu = emu_r * emu_r + emu_i * emu_i
        eps_tau = etau_r * etau_r + etau_i * etau_i
        st[base + 0] = 1.0 - eps_mu - eps_tau
        st[base + 1] = eps_mu
        st[base + 2] = eps_tau
        st[base + 3] = emu_r
        st[base + 4] = emu_i
        st[base + 5] = etau_r
        st[base + 6] = etau_i
    return st


def initial_state(ndir: int, ncell: int, seed: int, sim: int = 0,
                  alpha: float = 1e-6) -> np.ndarray:
    """Seeded near-electron-flavor initial state, [18][ndir][ncell]."""
    return state_from_seeds(alpha * seed_draws(ndir, ncell, seed, sim))


def mixing_matrix(th12: float, th13: float, th23: float,
                  delta: float = 0.0) -> np.ndarray:
    """U = R23 R13(delta) R12 (angles in radians)."""
    c12, s12 = math.cos(th12), math.sin(th12)
    c13, s13 = math.cos(th13), math.sin(th13)
    c23, s23 = math.cos(th23), math.sin(th23)
    e = complex(math.cos(delta), -math.sin(delta))
    R12 = np.array([[c12, s12, 0], [-s12, c12, 0], [0, 0, 1]], dtype=complex)
    R13 = np.array([[c13, 0, s13 * e], [0, 1, 0],
                    [-s13 * np.conj(e), 0, c13]], dtype=complex)
    R23 = np.array([[1, 0, 0], [0, c23, s23], [0, -s23, c23]], dtype=complex)
    return R23 @ R13 @ R12


def vacuum_hamiltonian(w21: float = 7.40e-5, w31: float = 2.4e-3,
                       th12_deg: float = 33.8, th13_deg: float = 8.6,
                       th23_deg: float = 48.6,
                       delta: float = 0.0) -> np.ndarray:
    """Flavor-basis vacuum Hamiltonian U diag(0, w21, w31) U^dagger
    (eq. potentials; the common |p| term drops out of the commutator).
    Returns a 3x3 complex128 Hermitian matrix."""
    U = mixing_matrix(math.radians(th12_deg), math.radians(th13_deg),
                      math.radians(th23_deg), delta)
    H = U @ np.diag([0.0, w21, w31]).astype(complex) @ U.conj().T
    return 0.5 * (H + H.conj().T)


def hvac_to_array(H: np.ndarray) -> np.ndarray:
    """3x3 complex -> 18 doubles, row-major (re, im) pairs."""
    H = np.asarray(H, dtype=np.complex128).reshape(3, 3)
    out = np.empty(18, dtype=np.float64)
    out[0::2] = H.real.ravel()
    out[1::2] = H.imag.ravel()
    return out


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    ncell: tuple            # (nx, ny, nz)
    length: tuple           # domain extent per axis, units of 1/mu
    ndir: int
    dt: float
    steps: int
    nbar_over_n: float = 1.0
    f: float = 0.0
    fbar: float = -1.0 / 3.0
    nhat: tuple = (0.0, 0.0, 1.0)
    seed: int = 1
    sim: int = 0
    alpha: float = 1e-6
    vacuum: bool = True
    # matter potentials (V_e, V_mu, V_tau) of the background charged
    # leptons; the benchmark workloads have none (comoving frame with no
    # net lepton density, as the paper's fiducial runs)
    vmat: tuple = (0.0, 0.0, 0.0)
    # shape function order: 1 linear (cloud in cell), 2 quadratic
    shape_order: int = 1

    @property
    def ncell_total(self) -> int:
        return int(self.ncell[0] * self.ncell[1] * self.ncell[2])

    @property
    def dx(self) -> tuple:
        return tuple(float(self.length[a]) / self.ncell[a] for a in range(3))

    @property
    def dV(self) -> float:
        dx = self.dx
        return dx[0] * dx[1] * dx[2]

    @property
    def nparticles(self) -> int:
        return self.ndir * self.ncell_total

    def dirs(self) -> np.ndarray:
        return directions(self.ndir)

    def weights(self):
        return particle_weights(self.dirs(), self.dV, 1.0, self.f,
                                self.nbar_over_n, self.fbar, self.nhat)

    def hvac(self) -> np.ndarray:
        if not self.vacuum:
            return np.zeros((3, 3), dtype=np.complex128)
        return vacuum_hamiltonian()

    def state0(self) -> np.ndarray:
        return initial_state(self.ndir, self.ncell_total, self.seed,
                             self.sim, self.alpha)


def _one_d(nz: int, L: float, **kw) -> dict:
    # 1D boxes run along z with unit transverse extent (the paper's
    # 1 x 1 x Nz grids).
    return dict(ncell=(1, 1, nz), length=(1.0, 1.0, L), **kw)


def workload(name: str) -> Workload:
    """Named synthetic workloads.

    * ``1d_32x26``     32 cells, L = 64, 26 directions, dt 0.2, 200 steps
    * ``1d_2048x378``  2048 cells, L = 64 pi (the paper's 64 cm at
      mu = pi/cm), 378 directions (C = 32), dt 0.1, 5000 steps
    * ``3d_64x92``     64^3 cells, L = 64 per side, 92 directions (C = 16),
      dt 0.2, 200 steps, nbar/n = 1.2, f = 0.1, fbar = -0.2, flux axis at 30
      degrees from z in the x-z plane
    * ``1d_512x128``   512 cells, L = 102.4, 128 directions, dt 0.1, 2000
      steps (the gradient workload)
    * ``1d_512x128_stable`` the same with nbar/n = 0.5, fbar = -0.2 (no
      crossing in the electron-lepton-number angular distribution)
    """
    s30 = math.sin(math.radians(30.0))
    c30 = math.cos(math.radians(30.0))
    table = {
        "1d_32x26": _one_d(32, 64.0, ndir=26, dt=0.2, steps=200, seed=1),
        "1d_2048x378": _one_d(2048, 64.0 * math.pi, ndir=378, dt=0.1,
                              steps=5000, seed=2),
        "3d_64x92": dict(ncell=(64, 64, 64), length=(64.0, 64.0, 64.0),
                         ndir=92, dt=0.2, steps=200, nbar_over_n=1.2, f=0.1,
                         fbar=-0.2, nhat=(s30, 0.0, c30), seed=3),
        "1d_512x128": _one_d(512, 102.4, ndir=128, dt=0.1, steps=2000,
                             seed=5),
        "1d_512x128_stable": _one_d(512, 102.4, ndir=128, dt=0.1, steps=2000,
                                    nbar_over_n=0.5, fbar=-0.2, seed=5),
    }
    if name not in table:
        raise KeyError(f"unknown workload {name!r}; have {sorted(table)}")
    return Workload(name=name, **table[name])


def batch_workloads(nsim: int = 64, master_seed: int = 4,
                    dt: float = 0.1, dz: float = 0.2,
                    steps: int = 1000) -> List[Workload]:
    """Uneven batch of independent 1D simulations.

    Per simulation i, draws from SplitMix64 stream (master_seed, i), in
    order: cell count uniform in {256..4096}, direction count from
    {64, 128, 378}, nbar/n ~ U[0.5, 1.5], f ~ U[-0.4, 0.4],
    fbar ~ U[-0.4, 0.4], flux-axis angle from z ~ U[0, 90] degrees in the
    x-z plane.  Cell width dz and dt are shared.
    """
    out = []
    for i in range(nsim):
        u = splitmix64_stream(master_seed, 1000 + i, np.arange(6))
        r = (u >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        nz = 256 + int(r[0] * (4096 - 256 + 1))
        ndir = (64, 128, 378)[min(2, int(r[1] * 3))]
        nbar = 0.5 + r[2]
        f = -0.4 + 0.8 * r[3]
        fbar = -0.4 + 0.8 * r[4]
        ang = math.radians(90.0 * r[5])
        out.append(Workload(name=f"batch{i}", ncell=(1, 1, nz),
                            length=(1.0, 1.0, nz * dz), ndir=ndir, dt=dt,
                            steps=steps, nbar_over_n=nbar, f=f, fbar=fbar,
                            nhat=(math.sin(ang), 0.0, math.cos(ang)),
                            seed=master_seed, sim=i + 1))
    return out


def scaled(w: Workload, ncell: Optional[tuple] = None,
           ndir: Optional[int] = None, steps: Optional[int] = None,
           **kw) -> Workload:
    """A smaller copy of a workload with the same cell width, dt and
    distribution (used where the CPU reference must finish in seconds)."""
    d = dataclasses.asdict(w)
    if ncell is not None:
        dx = w.dx
        d["ncell"] = tuple(ncell)
        d["length"] = tuple(dx[a] * ncell[a] for a in range(3))
    if ndir is not None:
        d["ndir"] = ndir
    if steps is not None:
        d["steps"] = steps
    d.update(kw)
    return Workload(**d)


# ---------------------------------------------------------------------------
# General particle placement
# ---------------------------------------------------------------------------
def uniform01(seed: int, stream: int, index: np.ndarray) -> np.ndarray:
    """Uniform draws in [0, 1): the top 53 bits of SplitMix64 output."""
    x = splitmix64_stream(seed, stream, index)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclasses.dataclass
class ParticleWorkload:
    """Particles anywhere in the periodic box (the general particle form of
    Sec. II.B), ``ppc`` per cell on average.

    placement ``"random"``: every particle uniform over the whole box;
    ``"stratified"``: exactly ``ppc`` particles per cell, each uniform within
    its cell (particle p in cell p // ppc).  Particle p moves along
    direction p mod ndir of the direction set, so every direction carries
    the same number of particles; its weights follow the same angular
    distribution as the lattice workloads, divided over ppc particles per
    cell.  Positions are given at t = 0; draws come from SplitMix64 stream
    2000 + axis of ``seed``.  State layout ``state[18][np]``.
    """
    name: str
    ncell: tuple
    length: tuple
    ppc: int
    ndir: int
    dt: float
    steps: int
    placement: str = "random"
    nbar_over_n: float = 1.0
    f: float = 0.0
    fbar: float = -1.0 / 3.0
    nhat: tuple = (0.0, 0.0, 1.0)
    seed: int = 1
    sim: int = 0
    alpha: float = 1e-6
    vacuum: bool = True
    vmat: tuple = (0.0, 0.0, 0.0)
    shape_order: int = 1

    @property
    def ncell_total(self) -> int:
        return int(self.ncell[0] * self.ncell[1] * self.ncell[2])

    @property
    def nparticles(self) -> int:
        return self.ppc * self.ncell_total

    @property
    def dx(self) -> tuple:
        return tuple(float(self.length[a]) / self.ncell[a] for a in range(3))

    @property
    def dV(self) -> float:
        dx = self.dx
        return dx[0] * dx[1] * dx[2]

    def positions(self) -> np.ndarray:
        """[np][3] positions at t = 0, each inside [0, length)."""
        n = self.nparticles
        idx = np.arange(n, dtype=np.uint64)
        out = np.empty((n, 3))
        if self.placement == "random":
            for a in range(3):
                out[:, a] = self.length[a] * uniform01(self.seed, 2000 + a, idx)
        elif self.placement == "stratified":
            nx, ny = self.ncell[0], self.ncell[1]
            c = np.arange(n) // self.ppc
            home = (c % nx, (c // nx) % ny, c // (nx * ny))
            for a in range(3):
                out[:, a] = (home[a] + uniform01(self.seed, 2000 + a, idx)) * self.dx[a]
        else:
            raise ValueError(f"unknown placement {self.placement!r}")
        return out

    def dirs(self) -> np.ndarray:
        """[np][3] unit direction of every particle."""
        table = directions(self.ndir)
        return np.ascontiguousarray(table[np.arange(self.nparticles) % self.ndir])

    def weights(self):
        """(N, Nbar), [np] each."""
        Nd, Nbd = particle_weights(directions(self.ndir), self.dV, 1.0, self.f,
                                   self.nbar_over_n, self.fbar, self.nhat)
        scale = self.ndir / self.ppc   # the table divides by ndir
        d = np.arange(self.nparticles) % self.ndir
        return np.ascontiguousarray(Nd[d] * scale), np.ascontiguousarray(Nbd[d] * scale)

    def hvac(self) -> np.ndarray:
        if not self.vacuum:
            return np.zeros((3, 3), dtype=np.complex128)
        return vacuum_hamiltonian()

    def state0(self) -> np.ndarray:
        """[18][np] seeded near-electron-flavor state."""
        st = initial_state(1, self.nparticles, self.seed, self.sim, self.alpha)
        return st.reshape(NCOMP, self.nparticles)


def particle_workload(name: str) -> ParticleWorkload:
    """Named general-placement workloads.

    * ``1d_2048x378_random``: the 2048-cell, L = 64 pi box with 774,144
      particles (378 per cell on average) at uniform random positions, one
      378-direction set shared round-robin, dt 0.1
    * ``1d_64x16_random``: 64 cells, L = 12.8, 16 particles per cell at
      random positions, 26 directions, dt 0.1 (small cases)
    * ``3d_32x92_random``: 32^3 cells, L = 32 per side, 92 particles per
      cell at random positions, 92 directions, dt 0.2, the 3D flux setup
    """
    s30 = math.sin(math.radians(30.0))
    c30 = math.cos(math.radians(30.0))
    table = {
        "1d_2048x378_random": _one_d(2048, 64.0 * math.pi, ppc=378, ndir=378, dt=0.1,
                                     steps=5000, seed=2),
        "1d_64x16_random": _one_d(64, 12.8, ppc=16, ndir=26, dt=0.1, steps=200,
                                  seed=6),
        "3d_32x92_random": dict(ncell=(32, 32, 32), length=(32.0, 32.0, 32.0), ppc=92,
                                ndir=92, dt=0.2, steps=200, nbar_over_n=1.2, f=0.1,
                                fbar=-0.2, nhat=(s30, 0.0, c30), seed=3),
    }
    if name not in table:
        raise KeyError(f"unknown workload {name!r}; have {sorted(table)}")
    return ParticleWorkload(name=name, **table[name])
