"""Property tests of the CPU reference on tiny random configurations
(hypothesis, derandomized so every run draws the same cases): box shapes
from one cell to small 3D boxes, a few directions or explicitly placed
particles, either shape function, random weights of either sign and random
Hermitian states.

* Trace: the slope of every particle is a commutator (eq. eom), whose trace
  vanishes, so Tr rho and Tr rhobar stay at their initial values.
* Lepton-number matrix (Sec. III.B): without vacuum and matter terms
  sum_p (N rho - Nbar rhobar^*) is conserved by the exact flow and, being
  linear in the state, by every Runge-Kutta step.
* Adjointness of deposit and interpolation: with the same weights W,
  <W^T x, G> = <x, W G> (the dot-product test of the interpolation against
  the deposit, both from the reference's own routines).
"""
import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import ParticleProblem, Problem

SETTINGS = dict(max_examples=25, deadline=None, derandomize=True, database=None)


def random_hermitian_states(rng, n):
    """n random Hermitian 3x3 matrices (not necessarily positive) as packed
    [9][n], trace near one."""
    out = np.empty((9, n))
    out[:3] = rng.uniform(-0.5, 1.0, (3, n))
    out[3:] = rng.uniform(-0.5, 0.5, (6, n))
    return out


def unit_vectors(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@st.composite
def configs(draw):
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    ncell = draw(st.sampled_from([(1, 1, 1), (1, 1, 2), (1, 1, 5), (2, 1, 3), (2, 2, 2), (3, 2, 1)]))
    general = draw(st.booleans())
    order = draw(st.sampled_from([1, 2]))
    dx = tuple(float(x) for x in rng.uniform(0.4, 1.3, 3))
    dt = float(rng.uniform(0.02, 0.1))
    nc = ncell[0] * ncell[1] * ncell[2]
    dV = dx[0] * dx[1] * dx[2]
    if general:
        npart = int(rng.integers(1, 12))
        L = np.array(ncell) * np.array(dx)
        pos = rng.uniform(0, 1, (npart, 3)) * L
        dirs = unit_vectors(rng, npart)
        # densities of order one: N ~ dV per particle and cell
        N = rng.uniform(-0.5, 1.0, npart) * dV * nc / npart
        Nb = rng.uniform(-0.5, 1.0, npart) * dV * nc / npart
        n_state = npart

        def make(H):
            return ParticleProblem(ncell, dx, pos, dirs, N, Nb, H, dt, shape_order=order)
        Np, Nbp = N, Nb
    else:
        ndir = int(rng.integers(1, 5))
        dirs = unit_vectors(rng, ndir)
        N = rng.uniform(-0.5, 1.0, ndir) * dV / ndir
        Nb = rng.uniform(-0.5, 1.0, ndir) * dV / ndir
        n_state = ndir * nc

        def make(H):
            return Problem(ncell, dx, dirs, N, Nb, H, dt, shape_order=order)
        Np, Nbp = np.repeat(N, nc), np.repeat(Nb, nc)
    state = np.concatenate([random_hermitian_states(rng, n_state),
                            random_hermitian_states(rng, n_state)])
    return dict(make=make, state=state, Np=Np, Nbp=Nbp, nc=nc, dV=dV,
                rng=rng, n0=int(rng.integers(0, 50)))


@settings(**SETTINGS)
@given(configs())
def test_trace_is_conserved(c):
    H = np.array([[0.1, 0.02 + 0.03j, 0.0], [0.02 - 0.03j, -0.2, 0.05j], [0.0, -0.05j, 0.3]])
    P = c["make"](H)
    s0 = c["state"]
    s1 = P.step(s0, 6, n0=c["n0"]).reshape(18, -1)
    for b in (0, 9):
        t0 = s0[b] + s0[b + 1] + s0[b + 2]
        t1 = s1[b] + s1[b + 1] + s1[b + 2]
        assert np.abs(t1 - t0).max() < 1e-13 * (1.0 + np.abs(s1).max())


@settings(**SETTINGS)
@given(configs())
def test_lepton_matrix_is_conserved_without_vacuum(c):
    P = c["make"](np.zeros((3, 3)))
    s0 = c["state"]
    s1 = P.step(s0, 6, n0=c["n0"]).reshape(18, -1)

    def lepton(s):
        nn = (c["Np"][None, :] * s[:9]).sum(1)
        nb = (c["Nbp"][None, :] * s[9:]).sum(1)
        nb[[4, 6, 8]] *= -1.0
        return nn - nb
    scale = (np.abs(c["Np"]).sum() + np.abs(c["Nbp"]).sum()) * (1.0 + np.abs(s1).max())
    assert np.abs(lepton(s1) - lepton(s0)).max() < 1e-13 * scale


@settings(**SETTINGS)
@given(configs())
def test_deposit_and_interpolation_are_adjoint(c):
    P = c["make"](np.zeros((3, 3)))
    rng = c["rng"]
    t = float(rng.uniform(-3.0, 3.0))
    s = c["state"]
    G = rng.normal(size=(1, c["nc"]))
    # <W^T (N rho_k), G> from the neutrino density moment, component k
    mom = P.moments(s, t)
    g = P.gather(G, t).reshape(-1)
    for k in range(9):
        lhs = c["dV"] * float(mom[k] @ G[0])
        rhs = float((c["Np"] * s[k]) @ g)
        assert abs(lhs - rhs) <= 1e-12 * (1.0 + abs(lhs))
