"""Objective of the differentiation workload, in numpy, with its gradient.

Test infrastructure only (see the package docstring).

On a channel with inlet at x = 0, outlet at x = nx-1 and bounce-back walls on
the first/last y and z layers, at the final time level:

  dp = c_s^2 (<rho>_{x=1} - <rho>_{x=nx-2})           (means over fluid nodes)
  D  = sum_{interior} rho [ (d/tau) |u|^2 + nu sum_{a,b} (d_b u_a)^2 ]
  J  = dp + 0.1 D

with central differences d_b u_a = (u_a(x+e_b) - u_a(x-e_b))/2 on interior
nodes x in [1, nx-2], y in [2, ny-3], z in [2, nz-3] (their neighbours are
fluid), rho = 1 + drho, nu = (tau - 1/2)/3.  The first term is the pressure
drop of the HNSE (pressure p = c_s^2 rho); the second the power dissipated by
the Darcy drag (d/tau per step, Sec. 3.3 Step 1) and by viscous shear.
"""
import numpy as np

CS2 = 1.0 / 3.0
WEIGHT = 0.1


def _interior(shape):
    nz, ny, nx = shape
    return (slice(2, nz - 2), slice(2, ny - 2), slice(1, nx - 1))


def _grad_u(u):
    """Central differences of u[a] along each lattice axis b -> g[a][b] (full arrays,
    valid where both neighbours exist)."""
    g = np.zeros((3, 3) + u.shape[1:])
    for a in range(3):
        for b in range(3):
            ax = 2 - b
            g[a, b] = 0.5 * (np.roll(u[a], -1, axis=ax) - np.roll(u[a], 1, axis=ax))
    return g


def objective(drho, u, d, tau):
    """J for fields shaped (nz, ny, nx) / (3, nz, ny, nx)."""
    drho = np.asarray(drho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    nz, ny, nx = drho.shape
    rho = 1.0 + drho
    fl = (slice(1, nz - 1), slice(1, ny - 1))
    dp = CS2 * (rho[fl + (1,)].mean() - rho[fl + (nx - 2,)].mean())
    nu = (tau - 0.5) / 3.0
    I = _interior(drho.shape)
    g = _grad_u(u)
    shear = (g ** 2).sum(axis=(0, 1))
    uu = (u ** 2).sum(axis=0)
    D = (rho * ((d / tau) * uu + nu * shear))[I].sum()
    return dp + WEIGHT * D


def objective_grad(drho, u, d, tau):
    """(dJ/d drho, dJ/du, dJ/dd explicit)."""
    drho = np.asarray(drho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    nz, ny, nx = drho.shape
    rho = 1.0 + drho
    nu = (tau - 0.5) / 3.0
    I = _interior(drho.shape)
    mask = np.zeros(drho.shape, dtype=bool)
    mask[I] = True
    g = _grad_u(u)
    shear = (g ** 2).sum(axis=(0, 1))
    uu = (u ** 2).sum(axis=0)
    gr = np.zeros_like(drho)
    fl = (slice(1, nz - 1), slice(1, ny - 1))
    n1 = (nz - 2) * (ny - 2)
    gr[fl + (1,)] += CS2 / n1
    gr[fl + (nx - 2,)] -= CS2 / n1
    gr += WEIGHT * np.where(mask, (d / tau) * uu + nu * shear, 0.0)
    gu = np.zeros_like(u)
    for a in range(3):
        gu[a] += WEIGHT * np.where(mask, 2.0 * rho * (d / tau) * u[a], 0.0)
        for b in range(3):
            ax = 2 - b
            t = WEIGHT * np.where(mask, rho * nu * 2.0 * g[a, b], 0.0) * 0.5
            gu[a] += np.roll(t, 1, axis=ax) - np.roll(t, -1, axis=ax)
    gd = WEIGHT * np.where(mask, rho * uu / tau, 0.0)
    return gr, gu, gd
