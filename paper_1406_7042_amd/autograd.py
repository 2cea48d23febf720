"""torch.autograd wrappers of the leapfrog and its hand-written adjoint.

FDTDFunction maps per-cell (eps_r, sigma_e) to the probe waveforms of a
full-order leapfrog run; its backward is the library's reverse-time adjoint
(fdtd_adjoint) with checkpoint-every-k recomputation.  ROMFunction maps
material parameters to the probe waveforms of a reduced model stepped beyond
the CFL limit (the clamp of Sec. III-A, then eq. (reducedMNAform)); its
backward is the library's reduced adjoint (rom_adjoint), which also carries
the derivative through the clamp.  Only argument marshalling happens here.
"""
from __future__ import annotations

import numpy as np
import torch

from . import yeerom as Y


class FDTDFunction(torch.autograd.Function):
    """y = leapfrog(eps_r, sigma_e) for a fixed grid, ports, waveform and dt.

    forward(eps_r, sigma_e, geom, dt, nsteps, u, ckpt_every)
      eps_r, sigma_e: per-cell tensors ([nz, ny, nx] or [ny, nx]), any device;
      geom: dict(dim, nx, ny, nz, dx, dy, dz, mu_r, sigma_m, pec, sources, probes);
      u: CUDA tensor [nsteps, nsrc] (float32 or float64, sets the precision).
    Returns y [nsteps, nprobe] (CUDA, dtype of u).
    """

    @staticmethod
    def forward(ctx, eps_r, sigma_e, geom, dt, nsteps, u, ckpt_every=64):
        op = Y.Operator(geom["dim"], geom["nx"], geom["ny"], geom.get("nz", 1), geom["dx"],
                        geom["dy"], geom.get("dz"),
                        eps_r=eps_r.detach().double().cpu().numpy(),
                        sigma_e=sigma_e.detach().double().cpu().numpy(),
                        mu_r=geom.get("mu_r"), sigma_m=geom.get("sigma_m"), pec=geom.get("pec"))
        f = op.new_fields(u.dtype)
        y = torch.zeros((nsteps, len(geom["probes"])), dtype=u.dtype, device=u.device)
        Y.fdtd_step(op, dt, nsteps, f, geom["sources"], u, geom["probes"], y)
        ctx.op, ctx.geom, ctx.dt, ctx.nsteps, ctx.ckpt = op, geom, dt, nsteps, ckpt_every
        ctx.save_for_backward(u)
        ctx.shape, ctx.devs = eps_r.shape, (eps_r.device, sigma_e.device)
        ctx.dtypes = (eps_r.dtype, sigma_e.dtype)
        return y

    @staticmethod
    def backward(ctx, gy):
        (u,) = ctx.saved_tensors
        ge, gs = Y.fdtd_adjoint(ctx.op, ctx.dt, ctx.nsteps, ctx.geom["sources"], u,
                                ctx.geom["probes"], gy.to(u.dtype).contiguous(), ctx.ckpt)
        ge = ge.reshape(ctx.shape).to(device=ctx.devs[0], dtype=ctx.dtypes[0])
        gs = gs.reshape(ctx.shape).to(device=ctx.devs[1], dtype=ctx.dtypes[1])
        return ge, gs, None, None, None, None, None


class ROMFunction(torch.autograd.Function):
    """y = reduced leapfrog of a model whose De~ depends on parameters theta.

    forward(theta, rom, De0, dDe, dt, nsteps, u, gamma)
      theta: [nparam] tensor (any device, float);
      rom:   a Rom (from mor_reduce or Rom.from_matrices); its De~ is set to
             De0 + sum_k theta_k dDe[k] (the basis frozen: for a per-cell
             material change, dDe[k] = V1^T dD_eps V1, see
             yeerom.rom_project_cells), then rom_perturb clamps at gamma 2/dt
             and rom_step runs nsteps in FP64;
      De0:   host [q1, q1] De~ at theta = 0;  dDe: sequence of host [q1, q1];
      u:     CUDA float64 [nsteps, nsrc].
    Returns y [nsteps, nprobe] (CUDA float64).  The backward pass gives
    dL/dtheta_k = sum_n dL/dy^n . dy^n/dtheta_k through the clamp (one
    reduced adjoint sweep per parameter).
    """

    @staticmethod
    def forward(ctx, theta, rom, De0, dDe, dt, nsteps, u, gamma=0.9999):
        th = theta.detach().double().cpu().numpy().ravel()
        dDe = [np.asarray(d, dtype=np.float64) for d in dDe]
        if len(dDe) != th.size:
            raise ValueError("one direction dDe per parameter")
        De = np.array(De0, dtype=np.float64, copy=True)
        for t, d in zip(th, dDe):
            De = De + t * d
        rom.set(Y.ROM_DE, De)
        Y.rom_perturb(rom, dt, gamma, dtype="f64")
        y = Y.rom_step([rom], dt, nsteps, [u], dtype="f64")[0]
        ctx.rom, ctx.dDe, ctx.dt, ctx.nsteps, ctx.gamma = rom, dDe, dt, nsteps, gamma
        ctx.save_for_backward(u)
        ctx.tdev, ctx.tdtype, ctx.tshape = theta.device, theta.dtype, theta.shape
        return y

    @staticmethod
    def backward(ctx, gy):
        (u,) = ctx.saved_tensors
        gy = gy.to(torch.float64).contiguous()
        g = [Y.rom_adjoint(ctx.rom, ctx.dt, ctx.nsteps, u, gy, dDe=d, through_clamp=True,
                           gamma=ctx.gamma)["dJ"] for d in ctx.dDe]
        gt = torch.tensor(g, dtype=ctx.tdtype, device=ctx.tdev).reshape(ctx.tshape)
        return gt, None, None, None, None, None, None, None


def geometry_of(wl) -> dict:
    """The fixed (non-differentiated) part of a workload, for FDTDFunction."""
    return dict(dim=wl.dim, nx=wl.nx, ny=wl.ny, nz=wl.nz, dx=np.asarray(wl.dx),
                dy=np.asarray(wl.dy), dz=np.asarray(wl.dz) if wl.dim == 3 else None,
                mu_r=wl.mu_r, sigma_m=wl.sigma_m,
                pec=[list(p) for p in wl.pec] if wl.pec else None,
                sources=wl.sources, probes=wl.probes)
