"""Two-flavor linear stability of a discrete angular distribution (the
linear analysis of Sec. III.B, for the directions a simulation actually
carries).  TEST INFRASTRUCTURE: it pins the growth rates of the
multi-angle workloads; nothing on the HIP path imports it.

Derivation, in the conventions of the CPU reference (eq. eom, eq. potentials
and the antineutrino conventions of Sec. II.A: H = H_vac + H_nunu,
Hbar = H_vac^* - H_nunu^*), for a homogeneous background in which every
particle is in the electron flavor, rho = rhobar = diag(1, 0, 0), with
neutrino and antineutrino densities n_d, nbar_d per direction d:

  background   H_ee - H_xx = Lambda_d + Delta_v,
               Lambda_d = sum_e (1 - v_d . v_e)(n_e - nbar_e),
  perturbation S_d = rho_ex, T_d = conj(rhobar_ex) of direction d,
               H_ex(d) = sum_e (1 - v_d . v_e)(n_e S_e - nbar_e T_e).

d rho/dt = -i[H, rho] linearised gives i (d/dt + v_d . grad) S_d =
(H_ee - H_xx) S_d - H_ex(d); the antineutrino equation, conjugated, is the
same equation for T_d with Delta_v -> -Delta_v (Hbar_vac = H_vac^*).  For
plane waves S_d, T_d ~ exp(i (k z - omega t)):

  omega Q_d = (k v_dz + Lambda_d + Delta_v) Q_d - sum_e G_de (n_e Q_e - nbar_e R_e)
  omega R_d = (k v_dz + Lambda_d - Delta_v) R_d - sum_e G_de (n_e Q_e - nbar_e R_e)

with G_de = 1 - v_d . v_e: an eigenvalue problem of size 2 N_dir.  Growth
rates are Im(omega).  With two opposite beams it is the 2 x 2 system of
App. A.3/A.4.  When the directions lie on rings of equal polar angle with
evenly spaced azimuths (the ring rule of Sec. III.A), modes proportional to
exp(i m phi) decouple; m = 0 preserves axial symmetry and m = 1 breaks it,
the two branches of the paper's dispersion relation (Fig. 5).
"""
from __future__ import annotations

import numpy as np


def dispersion_matrix(dirs, n, nbar, k, delta_v=0.0):
    """The 2N x 2N matrix whose eigenvalues are the mode frequencies omega
    at wavenumber k along z (densities per unit volume, units of mu)."""
    V = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    n = np.asarray(n, dtype=np.float64)
    nb = np.asarray(nbar, dtype=np.float64)
    G = 1.0 - V @ V.T
    lam = G @ (n - nb)
    Dq = np.diag(k * V[:, 2] + lam + delta_v)
    Dr = np.diag(k * V[:, 2] + lam - delta_v)
    Gn = G * n[None, :]
    Gb = G * nb[None, :]
    return np.block([[Dq - Gn, Gb], [-Gn, Dr + Gb]])


def modes(dirs, n, nbar, k, delta_v=0.0):
    """Eigenvalues and eigenvectors (columns: Q then R) at wavenumber k."""
    return np.linalg.eig(dispersion_matrix(dirs, n, nbar, k, delta_v))


def growth_rate(dirs, n, nbar, k, delta_v=0.0):
    """The largest Im(omega) at wavenumber k."""
    return float(np.linalg.eigvals(dispersion_matrix(dirs, n, nbar, k, delta_v)).imag.max())


def rings(dirs, decimals=12):
    """Group direction indices by polar angle: [(cos theta, [indices])]."""
    V = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    out = {}
    for i, z in enumerate(np.round(V[:, 2], decimals)):
        out.setdefault(float(z), []).append(i)
    return sorted(out.items())


def sector_growth_rate(dirs, n, nbar, k, m):
    """Largest Im(omega) among modes proportional to exp(i m phi) (m = 0 or
    1) for directions on rings with evenly spaced azimuths.  On a full ring
    sum_e exp(i phi_e) = 0 and sum_e cos(phi_d - phi_e) exp(i phi_e) =
    (M/2) exp(i phi_d), so the kernel 1 - v_d . v_e acts on ring amplitudes
    as 1 - c_r c_s (m = 0) or -s_r s_s / 2 per ring point (m = 1); the
    background Lambda keeps its m = 0 form."""
    rg = rings(dirs)
    n = np.asarray(n, dtype=np.float64)
    nb = np.asarray(nbar, dtype=np.float64)
    c = np.array([z for z, _ in rg])
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    nr = np.array([n[idx].sum() for _, idx in rg])
    nbr = np.array([nb[idx].sum() for _, idx in rg])
    lam = (1.0 - np.outer(c, c)) @ (nr - nbr)
    K = 1.0 - np.outer(c, c) if m == 0 else -0.5 * np.outer(s, s)
    D = np.diag(k * c + lam)
    A = np.block([[D - K * nr[None, :], K * nbr[None, :]], [-K * nr[None, :], D + K * nbr[None, :]]])
    return float(np.linalg.eigvals(A).imag.max())


def fastest(rate, kmin, kmax, nscan=64):
    """Maximise rate(k) over [kmin, kmax]: a scan, then golden-section
    refinement around the best scan point.  Returns (k, rate)."""
    ks = np.linspace(kmin, kmax, nscan)
    g = np.array([rate(k) for k in ks])
    i = int(np.argmax(g))
    a, b = ks[max(0, i - 1)], ks[min(nscan - 1, i + 1)]
    phi = (np.sqrt(5.0) - 1.0) / 2.0
    x1, x2 = b - phi * (b - a), a + phi * (b - a)
    f1, f2 = rate(x1), rate(x2)
    for _ in range(60):
        if f1 > f2:
            b, x2, f2 = x2, x1, f1
            x1 = b - phi * (b - a)
            f1 = rate(x1)
        else:
            a, x1, f1 = x1, x2, f2
            x2 = a + phi * (b - a)
            f2 = rate(x2)
    k = 0.5 * (a + b)
    return k, rate(k)
