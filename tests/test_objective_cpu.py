"""The objective of the differentiation workload, pinned on fields where its
value has a closed form, and the torch objective used with autograd against
the oracle's numpy objective (value and gradient; the oracle's gradient is
itself pinned to finite differences in tests/test_oracle_adjoint.py).

The objective (pressure drop plus 0.1 x dissipation, Sec. 3.3 Step 1 for the
drag power d/tau per step; pressure c_s^2 rho of the homogenized
Navier-Stokes limit) is evaluated on
* a density linear along the channel, where the pressure drop between the
  planes x = 1 and x = nx - 2 is c_s^2 times the slope times nx - 3;
* sine velocities (one along each axis) whose central differences are exact
  cosines, over interiors that hold whole half-periods, so that the sums of
  sin^2 and cos^2 are half the cell count.
Values outside the planes and the interior (wall layers) are set to noise and
must not matter.  CPU only.
"""
import math

import numpy as np
import pytest
import torch

from oracle import objective as oobj
from paper_2310_14746_amd.autograd import channel_objective

CS2 = 1.0 / 3.0


def _torch_objective(drho, u, d, tau):
    t = [torch.tensor(v, dtype=torch.float64) for v in (drho, u, d)]
    return float(channel_objective(t[0], t[1], t[2], tau))


IMPLEMENTATIONS = {"numpy": oobj.objective, "torch": _torch_objective}


@pytest.mark.parametrize("impl", sorted(IMPLEMENTATIONS))
def test_pressure_drop_of_a_linear_density(impl):
    nz, ny, nx = 7, 8, 13
    tau, a, b = 0.7, 2e-3, -3e-5
    rng = np.random.default_rng(3)
    x = np.arange(nx)
    drho = np.broadcast_to(a + b * x, (nz, ny, nx)).copy()
    # wall layers (y or z at 0 or n-1) hold noise: the plane means run over fluid cells only
    wall = np.zeros((nz, ny, nx), dtype=bool)
    wall[[0, -1], :, :] = True
    wall[:, [0, -1], :] = True
    drho[wall] = 1e-2 * rng.standard_normal(wall.sum())
    u = np.zeros((3, nz, ny, nx))
    d = rng.random((nz, ny, nx))
    J = IMPLEMENTATIONS[impl](drho, u, d, tau)
    want = CS2 * (-b) * (nx - 3)
    # rho = 1 + drho carries the rounding of numbers near 1
    assert abs(J - want) <= 1e-15, (J, want)


@pytest.mark.parametrize("impl", sorted(IMPLEMENTATIONS))
def test_dissipation_of_sine_shear(impl):
    # interior x in [1, nx-2]: 16 cells, whole half-periods of Lx = 8;
    # interior y in [2, ny-3]: 12 cells, whole half-periods of Ly = 6;
    # interior z in [2, nz-3]: 6 cells, whole half-periods of Lz = 4
    nz, ny, nx = 10, 16, 18
    L = {"x": 8, "y": 6, "z": 4}
    tau, d0, b = 0.65, 0.37, 4e-4
    amp = {"x": 3e-3, "y": -2e-3, "z": 1.5e-3}
    nu = (tau - 0.5) / 3.0
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    drho = np.full((nz, ny, nx), b)     # uniform: no pressure drop
    u = np.zeros((3, nz, ny, nx))
    u[1] = amp["x"] * np.sin(2 * np.pi * x / L["x"])    # u_y(x): shear d_x u_y
    u[2] = amp["y"] * np.sin(2 * np.pi * y / L["y"])    # u_z(y): shear d_y u_z
    u[0] = amp["z"] * np.sin(2 * np.pi * z / L["z"])    # u_x(z): shear d_z u_x
    interior = (z >= 2) & (z <= nz - 3) & (y >= 2) & (y <= ny - 3) & (x >= 1) & (x <= nx - 2)
    rng = np.random.default_rng(5)
    d = np.where(interior, d0, rng.random((nz, ny, nx)))
    J = IMPLEMENTATIONS[impl](drho, u, d, tau)
    # central differences of A sin(2 pi s/L) are A sin(2 pi/L) cos(2 pi s/L); over
    # whole half-periods the sums of sin^2 and cos^2 are each half the cell count
    count = (nz - 4) * (ny - 4) * (nx - 2)
    per_cell = sum(amp[k] ** 2 * (d0 / tau + nu * math.sin(2 * math.pi / L[k]) ** 2) for k in L) / 2
    want = 0.1 * (1.0 + b) * count * per_cell
    assert abs(J - want) <= 1e-13 * abs(want), (J, want)


def _fields(shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    drho = 1e-3 * rng.standard_normal(shape)
    u = 1e-2 * rng.standard_normal((3,) + shape)
    d = rng.random(shape)
    return drho, u, d


def test_value_and_gradient_match_oracle():
    for shape, tau in (((7, 9, 12), 0.6), ((10, 8, 6), 0.9)):
        drho, u, d = _fields(shape, seed=shape[2])
        J_o = oobj.objective(drho, u, d, tau)
        gr, gu, gd = oobj.objective_grad(drho, u, d, tau)
        t = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in (drho, u, d)]
        J = channel_objective(t[0], t[1], t[2], tau)
        J.backward()
        assert abs(float(J.detach()) - J_o) <= 1e-13 * abs(J_o)
        for got, want in zip((t[0].grad, t[1].grad, t[2].grad), (gr, gu, gd)):
            np.testing.assert_allclose(got.numpy(), want, rtol=1e-12, atol=1e-15 * np.abs(want).max())
