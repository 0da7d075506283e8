"""Diffusive-scaling refinement of the homogenized scheme.

The paper recovers its homogenized Navier-Stokes (Brinkman) equations from the
homogenized BGK equation under the diffusive scaling of Sec. 3.3 (Step 2):
the lattice spacing is eps, the time step eps^2, the relaxation time scales
with eps^2, and the porosity control scales as 1 - varpi = O(eps^2).  This
module drives the library's sweep along that limit and compares with exact
solutions of the target equations (eq:targetEBTL), so the consistency order of
the discretization can be measured.

Physical units: length H = 1, viscosity nu, permeability K, body acceleration
g.  At resolution N (eps = 1/N, dt = eps^2):
  lattice viscosity  nu (unchanged: nu dt / eps^2), tau = 3 nu + 1/2;
  porosity control   d = nu tau eps^2 / K   (Darcy drag per unit time nu/K);
  lattice force      F = g eps^3           (acceleration times dt^2 / eps);
  velocity           u_phys = u_lattice / eps.

Only host-side set-up and error norms live here; every step runs in the HIP
sweep through the C-ABI.
"""
from __future__ import annotations

import math

import numpy as np


def lattice_parameters(N: int, nu: float, K: float, g: float = 0.0) -> dict:
    eps = 1.0 / N
    tau = 3.0 * nu + 0.5
    return {"eps": eps, "tau": tau, "d": nu * tau * eps * eps / K, "force": g * eps ** 3,
            "u_scale": 1.0 / eps, "steps_per_time": N * N}


def brinkman_channel_exact(y: np.ndarray, nu: float, K: float, g: float) -> np.ndarray:
    """Steady Brinkman flow between no-slip walls at y = -1/2, 1/2:
    nu u'' - (nu/K) u + g = 0."""
    s = math.sqrt(K)
    return (g * K / nu) * (1.0 - np.cosh(y / s) / math.cosh(0.5 / s))


def brinkman_channel(hlbm, N: int, nu: float = 0.1, K: float = 0.01, g: float = 1.0,
                     decay: float = 36.0, storage: str = "f64"):
    """D2Q9 channel of N fluid rows (walls at half-cell distance) in a uniform
    porous medium, run to steady state from rest.  Returns (y, u_phys, exact,
    steps).  `decay` e-folds of the slowest transient mode are waited out."""
    p = lattice_parameters(N, nu, K, g)
    rate = nu * (math.pi ** 2 + 1.0 / K)              # slowest decay per unit time
    steps = int(math.ceil(decay / rate * p["steps_per_time"]))
    nx, ny = 4, N + 2
    sim = hlbm.HLBM(hlbm.D2Q9, storage, (nx, ny, 1), tau=p["tau"], force=(p["force"], 0.0, 0.0),
                    bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
    try:
        sim.set_porosity(np.full(nx * ny, p["d"]))
        sim.step(steps)
        _, u = sim.moments("f64")
        ux = u[0, 0, 1:ny - 1, 0].cpu().numpy() * p["u_scale"]
    finally:
        sim.close()
    y = (np.arange(1, ny - 1) - 0.5) / N - 0.5
    return y, ux, brinkman_channel_exact(y, nu, K, g), steps


def shear_wave_rate_exact(nu: float, K: float, k: float = 2.0 * math.pi) -> float:
    """Decay rate of u_x = sin(k y) under the Brinkman equation."""
    return nu * k * k + nu / K


def shear_wave_state(hlbm, N: int, amplitude_phys: float):
    """Shifted equilibrium populations of u_x = A sin(2 pi y), rho = rho0 = 1,
    on a 4 x N periodic D2Q9 box, in the library's order g[i, cell]."""
    c, w = hlbm.lattice_info(hlbm.D2Q9)
    nx, ny = 4, N
    y = (np.arange(ny) + 0.5) / N
    ux = amplitude_phys / N * np.sin(2.0 * math.pi * y)        # lattice units
    ux = np.broadcast_to(ux[:, None], (ny, nx)).ravel()
    cu = c[:, 0][:, None] * ux[None, :]
    g = w[:, None] * (3.0 * cu + 4.5 * cu * cu - 1.5 * ux[None, :] ** 2)
    return np.ascontiguousarray(g), y


def shear_wave_decay(hlbm, N: int, nu: float = 0.1, K: float = 0.05, t_end: float = 0.05,
                     amplitude: float = 0.01):
    """Measured and exact decay rates of a shear wave in a uniform porous
    medium over physical time t_end (D2Q9, FP64)."""
    import torch
    p = lattice_parameters(N, nu, K)
    steps = int(round(t_end * p["steps_per_time"]))
    g0, y = shear_wave_state(hlbm, N, amplitude)
    sim = hlbm.HLBM(hlbm.D2Q9, "f64", (4, N, 1), tau=p["tau"])
    try:
        sim.set_porosity(np.full(4 * N, p["d"]))
        sim.set_state(torch.from_numpy(g0.view(np.uint8).ravel()).to(sim.device), 0)
        _, u0 = sim.moments("f64")
        sim.step(steps)
        _, u1 = sim.moments("f64")
        s = np.sin(2.0 * math.pi * y)
        a0 = float((u0[0, 0, :, 0].cpu().numpy() * s).sum())
        a1 = float((u1[0, 0, :, 0].cpu().numpy() * s).sum())
    finally:
        sim.close()
    t = steps / p["steps_per_time"]
    return -math.log(a1 / a0) / t, shear_wave_rate_exact(nu, K), steps


def darcy_pressure_exact(x: np.ndarray, g: float, a: float) -> np.ndarray:
    """Steady 1-D flow through a periodic medium with 1/K(x) = (1 + a cos 2 pi x)/K0
    under acceleration g: continuity makes u = U uniform, periodicity of p fixes
    U = g K0 / nu, and the momentum balance dp/dx = g - nu U / K(x) gives
    p(x) = -(g a / (2 pi)) sin(2 pi x) (zero mean)."""
    return -(g * a / (2.0 * math.pi)) * np.sin(2.0 * math.pi * x)


def darcy_pressure(hlbm, N: int, nu: float = 0.1, K0: float = 0.01, g: float = 1.0, a: float = 0.5,
                   decay: float = 36.0, storage: str = "f64"):
    """Pressure of Darcy flow through a medium whose permeability varies along
    the flow (periodic in x, N cells per unit length; D2Q9 on N x 4).  The
    lattice pressure is c_s^2 drho; under the diffusive scaling the physical
    pressure is p = drho / (3 eps^2).  Returns (x, p, p_exact, U, U_exact,
    steps)."""
    eps = 1.0 / N
    tau = 3.0 * nu + 0.5
    x = (np.arange(N) + 0.5) / N
    inv_k = (1.0 + a * np.cos(2.0 * math.pi * x)) / K0
    d = nu * tau * eps * eps * inv_k                    # d = nu tau eps^2 / K(x)
    rate = nu / K0 * (1.0 - a)                          # slowest Darcy relaxation per unit time
    steps = int(math.ceil(decay / rate * N * N))
    nx, ny = N, 4
    sim = hlbm.HLBM(hlbm.D2Q9, storage, (nx, ny, 1), tau=tau, force=(g * eps ** 3, 0.0, 0.0))
    try:
        sim.set_porosity(np.ascontiguousarray(np.broadcast_to(d[None, :], (ny, nx)).ravel()))
        sim.step(steps)
        drho, u = sim.moments("f64")
        drho = drho[0, 0, :].cpu().numpy()
        ux = u[0, 0, 0, :].cpu().numpy()
    finally:
        sim.close()
    p = drho / (3.0 * eps * eps)
    U = float(((1.0 + drho) * ux).mean() / eps)          # mean mass flux, physical units
    return x, p, darcy_pressure_exact(x, g, a), U, g * K0 / nu, steps


def observed_order(errors, Ns) -> list:
    """log2 of successive error ratios for resolutions doubling."""
    return [math.log(errors[k] / errors[k + 1]) / math.log(Ns[k + 1] / Ns[k]) for k in range(len(Ns) - 1)]
