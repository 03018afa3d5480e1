"""Differentiable flavor evolution: torch.autograd.Function over the
library's hand-written adjoint.

FlavorEvolve.apply(params, seeds, workload, nsteps, ckpt_every) runs nsteps
RK4 steps of the PIC method from the initial condition defined by
  params = (nbar/n, f, fbar)  [float64 tensor of 3; the neutrino density is
           the unit and the flux axis is the workload's],
  seeds  = the eight off-diagonal perturbations alpha*U of every particle
           [float64 tensor 8 x ndir x ncell on the device],
and returns (L_nu, L_nubar): the final number-weighted mean of
rho_mumu + rho_tautau over all neutrino particles, and the same for the
antineutrinos.  backward() runs the library's reverse mode and chains its
d/d(initial state) and d/d(N, Nbar) to params and seeds.  The loss and the
chain through the initial-condition generator (weight formula of Sec. III.A,
eq. initial_flavor_state with eps = |rho_ex|^2) are elementwise tensor
expressions; the PIC steps and their adjoint run in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import inputs as I
from .sim import Sim
from ._lib import HostConfig


def _weights(w, params):
    nbar, f, fbar = (float(x) for x in params)
    dirs = w.dirs()
    N, Nb = I.particle_weights(dirs, w.dV, 1.0, f, nbar, fbar, w.nhat)
    nh = np.asarray(w.nhat, dtype=np.float64)
    mu = dirs @ (nh / np.linalg.norm(nh))
    base = w.dV / w.ndir
    dN_df = 3.0 * mu * base
    dNb_dnbar = (1.0 + 3.0 * fbar * mu) * base
    dNb_dfbar = nbar * 3.0 * mu * base
    return dirs, N, Nb, dN_df, dNb_dnbar, dNb_dfbar


def state_from_seeds_t(seeds: torch.Tensor) -> torch.Tensor:
    """eq. initial_flavor_state on the device (same arithmetic as
    inputs.state_from_seeds)."""
    nd, nc = seeds.shape[1], seeds.shape[2]
    st = torch.zeros((18, nd, nc), dtype=torch.float64, device=seeds.device)
    for base, o in ((0, 0), (9, 4)):
        er, ei, tr, ti = seeds[o], seeds[o + 1], seeds[o + 2], seeds[o + 3]
        emu = er * er + ei * ei
        etau = tr * tr + ti * ti
        st[base + 0] = 1.0 - emu - etau
        st[base + 1] = emu
        st[base + 2] = etau
        st[base + 3], st[base + 4], st[base + 5], st[base + 6] = er, ei, tr, ti
    return st


class FlavorEvolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, seeds, workload, nsteps, ckpt_every=50, tuning=None):
        w = workload
        dirs, N, Nb, dN_df, dNb_dnbar, dNb_dfbar = _weights(w, params.detach().cpu().numpy())
        hc = HostConfig(w.ncell, w.dx, dirs, N, Nb, w.hvac(), w.dt,
                        shape_order=w.shape_order, vmat=w.vmat)
        sim = Sim(hc, tuning=tuning, device=str(seeds.device))
        st0 = state_from_seeds_t(seeds.detach())
        sim.set_state(st0, 0)
        sim.adjoint_forward(int(nsteps), int(ckpt_every))
        yT = sim.get_state()
        Nt = torch.from_numpy(N).to(seeds.device)[:, None]
        Nbt = torch.from_numpy(Nb).to(seeds.device)[:, None]
        sN = Nt.sum() * w.ncell_total
        sNb = Nbt.sum() * w.ncell_total
        Lnu = (Nt * (yT[1] + yT[2])).sum() / sN
        Lnb = (Nbt * (yT[10] + yT[11])).sum() / sNb
        ctx.sim = sim
        ctx.pdev, ctx.pdtype = params.device, params.dtype
        ctx.save_for_backward(seeds.detach(), yT)
        ctx.aux = (N, Nb, dN_df, dNb_dnbar, dNb_dfbar, float(sN), float(sNb),
                   float(Lnu), float(Lnb))
        return Lnu.detach(), Lnb.detach()

    @staticmethod
    def backward(ctx, gLnu, gLnb):
        seeds, yT = ctx.saved_tensors
        N, Nb, dN_df, dNb_dnbar, dNb_dfbar, sN, sNb, Lnu, Lnb = ctx.aux
        dev = seeds.device
        gnu = float(gLnu) if gLnu is not None else 0.0
        gnb = float(gLnb) if gLnb is not None else 0.0
        Nt = torch.from_numpy(N).to(dev)[:, None]
        Nbt = torch.from_numpy(Nb).to(dev)[:, None]
        # dL/d(final state): the loss is linear in it
        lam = torch.zeros_like(yT)
        lam[1] = lam[2] = gnu * Nt / sN
        lam[10] = lam[11] = gnb * Nbt / sNb
        g0, gN, gNb = ctx.sim.adjoint_backward(lam.contiguous())
        # explicit dependence of the loss on N, Nbar (weights and normalisation)
        nc = yT.shape[2]
        xs = (yT[1] + yT[2]).sum(dim=1).cpu().numpy()
        xsb = (yT[10] + yT[11]).sum(dim=1).cpu().numpy()
        gN = gN + gnu * (xs - Lnu * nc) / sN
        gNb = gNb + gnb * (xsb - Lnb * nc) / sNb
        gparams = torch.tensor([float(np.dot(gNb, dNb_dnbar)), float(np.dot(gN, dN_df)),
                                float(np.dot(gNb, dNb_dfbar))], dtype=ctx.pdtype,
                               device=ctx.pdev)
        # chain through eq. initial_flavor_state
        gs = torch.empty_like(seeds)
        for base, o in ((0, 0), (9, 4)):
            l0, l1, l2 = g0[base + 0], g0[base + 1], g0[base + 2]
            gs[o + 0] = g0[base + 3] + 2.0 * seeds[o + 0] * (l1 - l0)
            gs[o + 1] = g0[base + 4] + 2.0 * seeds[o + 1] * (l1 - l0)
            gs[o + 2] = g0[base + 5] + 2.0 * seeds[o + 2] * (l2 - l0)
            gs[o + 3] = g0[base + 6] + 2.0 * seeds[o + 3] * (l2 - l0)
        ctx.sim.close()
        return gparams, gs, None, None, None, None


def evolve(params, seeds, workload, nsteps, ckpt_every=50, tuning=None):
    return FlavorEvolve.apply(params, seeds, workload, nsteps, ckpt_every, tuning)
