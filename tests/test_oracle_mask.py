"""Pins of the oracle's resolved obstacles (a per-cell solid mask with halfway
bounce-back at every fluid-solid link, periodic box; CPU only).

* a mask of two wall rows reproduces the wall-face configuration bit for bit
  (and with it the Poiseuille pin of tests/test_oracle_pins.py);
* mass is conserved around an arbitrary obstacle;
* a sphere centred in a cube, driven along x, gives a flow mirror-symmetric in
  y and z;
* the drag on a periodic simple-cubic array of spheres agrees with Hasimoto's
  expansion F / (6 pi mu a U) = 1 / (1 - 1.7601 c^(1/3) + c - 1.5593 c^2) within
  the O(dx) uncertainty of a staircase sphere's hydrodynamic radius (10%).
"""
import math

import numpy as np

import oracle
from oracle import OracleConfig, PERIODIC, WALL
from paper_2310_14746_amd import inputs


def test_wall_rows_equal_wall_faces():
    nx, ny, nz = 7, 9, 5
    d = inputs.periodic_smooth(inputs.uniform_noise((nz, ny, nx), 4), 1.0, 3).ravel()
    walls = OracleConfig(q=19, nx=nx, ny=ny, nz=nz, tau=0.8, force=(1e-5, 0, 2e-6),
                         bc_lo=(PERIODIC, WALL, PERIODIC), bc_hi=(PERIODIC, WALL, PERIODIC))
    per = OracleConfig(q=19, nx=nx, ny=ny, nz=nz, tau=0.8, force=(1e-5, 0, 2e-6))
    mask = walls.solid_mask().ravel()
    gw = oracle.run(walls, d, 40)
    gm = oracle.run_masked(per, mask, d, 40)
    assert np.array_equal(gw, gm)


def test_mass_conserved_around_obstacle():
    n = 12
    cfg = OracleConfig(q=19, nx=n, ny=n, nz=n, tau=0.7, force=(1e-5, 3e-6, 0))
    mask = inputs.sphere_indicator(n, 3.3).ravel() > 0.5
    rng = np.random.default_rng(1)
    g = 1e-4 * rng.standard_normal((19, n ** 3))
    g[:, mask] = 0.0
    m0 = g.sum()
    g = oracle.run_masked(cfg, mask, np.zeros(n ** 3), 60, g=g)
    assert abs(g.sum() - m0) <= 1e-15 * n ** 3
    assert np.all(g[:, mask] == 0.0)


def test_centred_sphere_symmetry():
    n = 10
    cfg = OracleConfig(q=19, nx=n, ny=n, nz=n, tau=0.8, force=(1e-5, 0, 0))
    mask = inputs.sphere_indicator(n, 2.6).ravel() > 0.5
    g = oracle.run_masked(cfg, mask, np.zeros(n ** 3), 80)
    _, u = oracle.observe_masked(cfg, mask, g)
    ux = u[0].reshape(n, n, n)
    uy = u[1].reshape(n, n, n)
    scale = np.abs(ux).max()
    # the sphere's centre is at (n-1)/2: mirror y -> n-1-y and z -> n-1-z
    assert np.abs(ux - ux[:, ::-1, :]).max() <= 1e-12 * scale
    assert np.abs(ux - ux[::-1, :, :]).max() <= 1e-12 * scale
    assert np.abs(uy + uy[:, ::-1, :]).max() <= 1e-12 * scale
    assert np.all(u[:, mask] == 0.0)


def test_hasimoto_drag_of_sphere_array():
    L, a, tau = 24, 4.0, 1.0
    nu = (tau - 0.5) / 3.0
    F = 1e-6
    cfg = OracleConfig(q=19, nx=L, ny=L, nz=L, tau=tau, force=(F, 0, 0))
    mask = inputs.sphere_indicator(L, a).ravel() > 0.5
    n_fluid = int((~mask).sum())
    g = oracle.run_masked(cfg, mask, np.zeros(L ** 3), 6000, nthreads=8)
    dr, u = oracle.observe_masked(cfg, mask, g, nthreads=8)
    U = ((1.0 + dr) * u[0]).sum() / L ** 3            # superficial (cell-averaged) velocity
    drag = F * n_fluid                                # steady state: force on the fluid = drag
    c = mask.sum() / L ** 3                           # solid fraction of the staircase sphere
    a_eff = (3.0 * mask.sum() / (4.0 * math.pi)) ** (1.0 / 3.0)
    K = drag / (6.0 * math.pi * nu * a_eff * U)
    K_h = 1.0 / (1.0 - 1.7601 * c ** (1.0 / 3.0) + c - 1.5593 * c * c)
    assert abs(K / K_h - 1.0) <= 0.10, (K, K_h)


def test_masked_pull_with_tensor_collision_reduces_to_scalar():
    """The composition the GPU mask + tensor test uses as its oracle (masked
    pull, tensor collision, zeroed solid cells) equals the masked scalar run
    when D = d I."""
    nx, ny, nz = 10, 6, 5
    n = nx * ny * nz
    cfg = OracleConfig(q=19, nx=nx, ny=ny, nz=nz, tau=0.7, force=(2e-5, -7e-6, 3e-6))
    rng = np.random.default_rng(0)
    d = 0.3 * rng.random(n)
    mask = (rng.random(n) < 0.2).astype(np.uint8)
    D6 = np.zeros((6, n))
    D6[:3] = d
    g = np.zeros((19, n))
    for _ in range(20):
        g = oracle.collide_tensor(cfg, D6, oracle.stream_masked(cfg, mask, g))
        g[:, mask != 0] = 0.0
    ref = oracle.run_masked(cfg, mask, d, 20)
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()
