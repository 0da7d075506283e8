"""PyTorch autograd of the HLBM sweep with respect to the porosity control.

``HLBMFunction`` maps a porosity field d = 1 - varpi (Sec. 3.2) to the moments
(drho, u) after ``nsteps`` sweeps from rest.  Its forward runs the HIP sweep
with a checkpoint tape; its backward runs the library's hand-written discrete
adjoint (``hlbm_adjoint_step``) and returns dJ/dd.  No PyTorch operator takes
part in either pass: torch only holds the memory and differentiates whatever
objective the caller builds on the returned moments (for instance
:func:`channel_objective`).
"""
from __future__ import annotations

import torch

from . import hlbm as _h


class HLBMFunction(torch.autograd.Function):
    """(drho, u) = F(d) for one context ``sim`` (an :class:`hlbm.HLBM`).

    d is the scalar control (nz, ny, nx), or for a tensor-control context the
    six rows xx, yy, zz, xy, xz, yz of D, (6, nz, ny, nx); the gradient has d's
    shape.

    forward(d, sim, nsteps, every): sets the porosity, resets ``sim`` to rest,
    records a tape with a checkpoint every ``every`` steps and runs ``nsteps``
    sweeps; returns FP64 device tensors drho (nz, ny, nx) and u (3, nz, ny, nx).
    backward: the reverse sweep over the same steps.  ``sim`` must not be
    stepped, reset, given a new state, tape, mask or porosity between the two
    passes: the wrapper counts every such call (``sim.generation``), and a
    backward whose forward was followed by one raises instead of
    differentiating another run's tape.
    """

    @staticmethod
    def forward(ctx, d, sim, nsteps: int, every: int):
        sim.set_porosity(d.detach().reshape(-1).to(_porosity_dtype(sim)))
        sim.reset()
        sim.set_tape(every, nsteps)
        sim.step(nsteps)
        drho, u = sim.moments("f64")
        ctx.sim = sim
        ctx.nsteps = int(nsteps)
        ctx.generation = sim.generation
        ctx.d_dtype = d.dtype
        ctx.d_shape = d.shape
        return drho, u

    @staticmethod
    def backward(ctx, g_drho, g_u):
        sim = ctx.sim
        if sim.generation != ctx.generation:
            raise RuntimeError("the lattice was changed after the forward pass (stepped, reset, "
                               "or given a new state, tape, mask or porosity); its tape no longer "
                               "matches this graph")
        if g_drho is None:
            g_drho = torch.zeros(sim.N, dtype=torch.float64, device=sim.device)
        if g_u is None:
            g_u = torch.zeros(3 * sim.N, dtype=torch.float64, device=sim.device)
        d_bar = sim.adjoint(ctx.nsteps, g_drho, g_u)
        return d_bar.reshape(ctx.d_shape).to(ctx.d_dtype), None, None, None


def _porosity_dtype(sim):
    return {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}[sim.porosity_dtype]


def moments_of_porosity(d, sim, nsteps: int, every: int = 50):
    """Differentiable (drho, u) after ``nsteps`` sweeps from rest with porosity d."""
    return HLBMFunction.apply(d, sim, nsteps, every)


CS2 = 1.0 / 3.0


def channel_objective(drho, u, d, tau: float, weight: float = 0.1):
    """Pressure drop plus weighted dissipation on a channel (torch, differentiable).

    The channel has its inlet at x = 0, outlet at x = nx - 1 and bounce-back
    walls on the first and last y and z layers.  With rho = 1 + drho (the
    pressure of the homogenized Navier-Stokes limit is c_s^2 rho):
      dp = c_s^2 (<rho>_{x=1} - <rho>_{x=nx-2}), means over the fluid cells of
           those planes;
      D  = sum over interior cells of rho [ (d/tau) |u|^2 + nu sum_ab (d_b u_a)^2 ],
           nu = (tau - 1/2)/3, central differences, interior x in [1, nx-2],
           y in [2, ny-3], z in [2, nz-3] (all neighbours fluid); the first
           term is the work of the porous drag (a fraction d/tau of the
           momentum is removed per step, Sec. 3.3), the second viscous shear;
      J  = dp + weight * D.
    drho: (nz, ny, nx); u: (3, nz, ny, nx); d: (nz, ny, nx).
    """
    nz, ny, nx = drho.shape
    rho = 1.0 + drho
    dp = CS2 * (rho[1:nz - 1, 1:ny - 1, 1].mean() - rho[1:nz - 1, 1:ny - 1, nx - 2].mean())
    nu = (tau - 0.5) / 3.0
    # central differences over the interior box; neighbours stay inside the array
    zc, yc, xc = slice(2, nz - 2), slice(2, ny - 2), slice(1, nx - 1)
    shear = torch.zeros_like(drho[zc, yc, xc])
    for a in range(3):
        ua = u[a]
        dx = 0.5 * (ua[zc, yc, 2:nx] - ua[zc, yc, 0:nx - 2])
        dy = 0.5 * (ua[zc, 3:ny - 1, xc] - ua[zc, 1:ny - 3, xc])
        dz = 0.5 * (ua[3:nz - 1, yc, xc] - ua[1:nz - 3, yc, xc])
        shear = shear + dx * dx + dy * dy + dz * dz
    uu = (u[:, zc, yc, xc] ** 2).sum(dim=0)
    D = (rho[zc, yc, xc] * ((d[zc, yc, xc] / tau) * uu + nu * shear)).sum()
    return dp + weight * D
