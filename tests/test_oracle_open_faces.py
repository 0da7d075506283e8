"""Pins of the oracle's open faces (inlet at a prescribed velocity, outlet at a
prescribed density), the boundary rule of the differentiation workload.

The paper states only the no-slip condition u = 0 on the boundary of the
porous domain (Sec. 2.4, eq:targetEBTL); the open faces are a reading of it:
a population whose pull source lies beyond an open face is the equilibrium
built from the cell's own post-collision state, f^eq(rho_b, u_in) at an
inlet, f^eq(rho_out, j_b / rho_b) at an outlet.  These tests check that
rule against things fixed outside the oracle:

* per cell, the incoming populations equal the equilibrium written out from
  the velocity set alone (and bounce-back wins on edges);
* a duct that is uniform across the flow reduces exactly to a three-velocity
  model along the flow (the five D3Q19 velocities with c_x = +1, the nine with
  c_x = 0 and the five with c_x = -1 stream together, and every moment the
  collision needs is a sum over those groups); that model, written here in a
  few lines of numpy, must follow the oracle at every step;
* its steady state is Darcy flow (Sec. 3.3 Step 1: a fraction d/tau of the
  momentum is removed per step, balanced by the pressure gradient c_s^2 d rho/dx):
  a uniform mass flux J = rho u_in through the inlet, a linear density with
  slope -3 (d/tau) J, and the outlet cell one slope above rho_out.  The
  closed form below is exact for the linearized scheme; the oracle follows it
  to O(u_in) relative.

CPU only.
"""
import numpy as np
import pytest

from oracle import OracleConfig, PERIODIC, WALL, INLET_U, OUTLET_RHO


def _feq_shifted(c, w, rho, u, rho0=1.0):
    """Second-order Maxwellian shifted by w*rho0, from the velocity set alone
    (c_s^2 = 1/3: f^eq_i = w_i rho [1 + c.u/c_s^2 + (c.u)^2/(2 c_s^4) - u.u/(2 c_s^2)])."""
    cu = c @ np.asarray(u, dtype=float)
    uu = float(np.dot(u, u))
    return w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu) - w * rho0


@pytest.mark.parametrize("q", [9, 19])
def test_open_face_populations_per_cell(orc, q):
    """Every population pulled from beyond an open face equals f^eq(rho_b, u_in)
    (inlet) or f^eq(rho_out, j_b/rho_b) (outlet) minus w rho0, with rho_b and
    j_b the cell's own post-collision mass and momentum; a source in a wall
    layer bounces back instead; every other population is the plain pull."""
    c, w = orc.lattice(q)
    opp = np.array([int(np.flatnonzero((c == -ci).all(axis=1))[0]) for ci in c])
    nz = 1 if q == 9 else 6
    nx, ny = 7, 6
    u_in = (0.031, -0.004, 0.0 if q == 9 else 0.0027)
    cfg = OracleConfig(q=q, nx=nx, ny=ny, nz=nz, tau=0.7,
                       bc_lo=(INLET_U, WALL, WALL if q == 19 else PERIODIC),
                       bc_hi=(OUTLET_RHO, WALL, WALL if q == 19 else PERIODIC),
                       inlet_u=u_in, outlet_rho=0.987)
    rng = np.random.default_rng(7)
    post = 1e-2 * rng.standard_normal((q, nz * ny * nx))
    pre = orc.stream(cfg, post)
    post4 = post.reshape(q, nz, ny, nx)
    pre4 = pre.reshape(q, nz, ny, nx)
    solid = cfg.solid_mask()
    n = (nx, ny, nz)
    checked = {"inlet": 0, "outlet": 0, "bounce": 0, "pull": 0}
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if solid[z, y, x]:
                    assert (pre4[:, z, y, x] == 0).all()
                    continue
                g = post4[:, z, y, x]
                rho_b = 1.0 + g.sum()
                j_b = c.T @ g
                for i in range(q):
                    src = [x - c[i, 0], y - c[i, 1], z - c[i, 2]]
                    for a in range(3):   # periodic axes wrap
                        if cfg.bc_lo[a] == PERIODIC:
                            src[a] %= n[a]
                    in_wall = any((cfg.bc_lo[a] == WALL and src[a] == 0) or
                                  (cfg.bc_hi[a] == WALL and src[a] == n[a] - 1) for a in range(3))
                    if in_wall:
                        want, kind = g[opp[i]], "bounce"
                    elif src[0] < 0:
                        want, kind = _feq_shifted(c, w, rho_b, u_in)[i], "inlet"
                    elif src[0] >= nx:
                        want, kind = _feq_shifted(c, w, cfg.outlet_rho, j_b / rho_b)[i], "outlet"
                    else:
                        want, kind = post4[i, src[2], src[1], src[0]], "pull"
                    assert abs(pre4[i, z, y, x] - want) <= 1e-15, (kind, i, x, y, z)
                    checked[kind] += 1
    assert min(checked.values()) > 0, checked


def _d1q3(nx, tau, d, u_in, rho_out, F, steps, rho0=1.0):
    """Three-velocity model along a duct: lumped shifted populations of the
    groups c_x = +1, 0, -1 (weights 1/6, 2/3, 1/6, the sums of the D2Q9/D3Q19
    weights over each group), with the same collision and open faces.
    Returns the moments (drho, u_x) of every time level 1..steps."""
    pref = 1.0 - 0.5 / tau

    def eq(rho, U):   # group sums of w_i[(rho - rho0) + rho(3 c.u + 9/2 (c.u)^2 - 3/2 u.u)], u = (U, 0, 0)
        return np.array([((rho - rho0) + rho * (3 * U + 3 * U * U)) / 6,
                         2 * (rho - rho0) / 3 - rho * U * U,
                         ((rho - rho0) + rho * (-3 * U + 3 * U * U)) / 6])

    P = np.zeros((3, nx))
    out = []
    for _ in range(steps + 1):
        rb = rho0 + P.sum(0)
        jb = P[0] - P[2]
        f = np.empty_like(P)
        f[0, 1:] = P[0, :-1]
        f[1] = P[1]
        f[2, :-1] = P[2, 1:]
        f[0, 0] = eq(rb[0], u_in)[0]
        f[2, -1] = eq(rho_out, jb[-1] / rb[-1])[2]
        rho = rho0 + f.sum(0)
        U = (f[0] - f[2] + F / 2) / rho
        out.append((rho - rho0, U))
        # group sums of Guo's source with u = (U, 0, 0), F along x
        S = pref * np.array([(3 * F + 6 * U * F) / 6, -2 * U * F, (-3 * F + 6 * U * F) / 6])
        P = f - (f - eq(rho, (1 - d) * U)) / tau + S
    return out[1:]


@pytest.mark.parametrize("q", [9, 19])
def test_open_duct_reduces_to_three_velocities(orc, q):
    """A duct periodic across the flow, uniform control, inlet and outlet along
    x, a force along x: the oracle's density and velocity equal the lumped
    three-velocity model at every time level, and nothing moves across."""
    nx, tau, d, u_in, rho_out, F = 24, 0.75, 0.2, 2e-3, 1.004, 3e-6
    ny, nz = (3, 1) if q == 9 else (2, 3)
    cfg = OracleConfig(q=q, nx=nx, ny=ny, nz=nz, tau=tau, force=(F, 0, 0),
                       bc_lo=(INLET_U, PERIODIC, PERIODIC), bc_hi=(OUTLET_RHO, PERIODIC, PERIODIC),
                       inlet_u=(u_in, 0, 0), outlet_rho=rho_out)
    ref = _d1q3(nx, tau, d, u_in, rho_out, F, 120)
    g = None
    for t in (1, 7, 40, 120):
        g = orc.run(cfg, np.full(cfg.ncells, d), t - (0 if g is None else prev), g=g)
        prev = t
        dr, u = orc.observe(cfg, g)
        dr = dr.reshape(nz, ny, nx)
        u = u.reshape(3, nz, ny, nx)
        dr_m, U_m = ref[t - 1]
        assert np.abs(dr - dr_m).max() <= 1e-14, t
        assert np.abs(u[0] - U_m).max() <= 1e-14, t
        assert np.abs(u[1:]).max() <= 1e-18, t


@pytest.mark.parametrize("q,nx,tau,d,u_in,rho_out", [
    (19, 32, 0.6, 0.1, 1e-4, 1.001),
    (19, 24, 0.8, 0.05, 5e-5, 0.999),
    (9, 40, 0.7, 0.3, 1e-5, 0.998),
])
def test_open_duct_darcy_steady_state(orc, q, nx, tau, d, u_in, rho_out):
    """Steady Darcy flow through a uniform duct: mass flux uniform along it
    (mass conservation) and, to first order in u_in, J = rho(0) u_in,
    drho(x) = (rho_out - 1) + s (nx - x) with s = 3 (d/tau) J, i.e.
    J = u_in rho_out / (1 - 3 d nx u_in / tau)."""
    ny, nz = (2, 1) if q == 9 else (2, 2)
    cfg = OracleConfig(q=q, nx=nx, ny=ny, nz=nz, tau=tau,
                       bc_lo=(INLET_U, PERIODIC, PERIODIC), bc_hi=(OUTLET_RHO, PERIODIC, PERIODIC),
                       inlet_u=(u_in, 0, 0), outlet_rho=rho_out)
    dfield = np.full(cfg.ncells, d)
    g = orc.run(cfg, dfield, 6000)
    for _ in range(20):   # run to a steady state (the pressure diffuses at c_s^2 tau / d per step)
        g_next = orc.run(cfg, dfield, 2000, g=g)
        change = np.abs(g_next - g).max()
        g = g_next
        if change < 1e-17:
            break
    assert change < 1e-15
    dr, u = orc.observe(cfg, g)
    dr = dr.reshape(nz, ny, nx)[0, 0]
    ux = u.reshape(3, nz, ny, nx)[0, 0, 0]
    j = (1.0 + dr) * ux
    assert np.ptp(j) <= 1e-9 * abs(j.mean())          # uniform flux
    J = u_in * rho_out / (1.0 - 3.0 * d * nx * u_in / tau)
    s = 3.0 * d * J / tau
    want = (rho_out - 1.0) + s * (nx - np.arange(nx))
    tol = 2 * u_in   # the neglected terms are O(u_in) relative (measured 0.1-0.5 u_in)
    assert abs(j.mean() / J - 1) <= tol
    assert abs(ux[0] / u_in - 1) <= tol
    assert np.abs(dr - want).max() <= tol * np.abs(want).max()
    # the slope alone, free of the boundary levels
    slope = np.polyfit(np.arange(2, nx - 2), dr[2:nx - 2], 1)[0]
    assert abs(-slope / (3.0 * d * j.mean() / tau) - 1) <= tol
