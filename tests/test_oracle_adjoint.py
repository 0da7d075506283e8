"""Pins of the oracle's discrete adjoint (CPU only).

* streaming is linear without open faces: <S v, w> = <v, S^T w> to rounding;
* every other transposed Jacobian (collision in y and d, open faces,
  moments) matches central finite differences of the forward map;
* the full gradient dJ/dd of the channel objective matches central finite
  differences (h = 1e-4) to 1e-6 and its Taylor remainder is O(h^2);
* the result does not depend on the checkpoint interval.
"""
import numpy as np
import pytest

from oracle import OracleConfig, PERIODIC, WALL, INLET_U, OUTLET_RHO
from oracle import objective as ob


def _rng(s):
    return np.random.default_rng(s)


def _channel(nx=14, ny=8, nz=8, tau=0.6):
    return OracleConfig(q=19, nx=nx, ny=ny, nz=nz, tau=tau, bc_lo=(INLET_U, WALL, WALL),
                        bc_hi=(OUTLET_RHO, WALL, WALL), inlet_u=(0.02, 0.0, 0.0), outlet_rho=1.0)


def _random_state(cfg, rng, scale=1e-3):
    g = scale * rng.standard_normal((cfg.q, cfg.ncells))
    g[:, cfg.solid_mask().ravel()] = 0.0
    return g


@pytest.mark.parametrize("bc", ["periodic", "walls"])
def test_stream_transpose_exact(orc, bc):
    if bc == "periodic":
        cfg = OracleConfig(q=19, nx=7, ny=5, nz=4)
    else:
        cfg = OracleConfig(q=19, nx=7, ny=6, nz=5, bc_lo=(PERIODIC, WALL, WALL),
                           bc_hi=(PERIODIC, WALL, WALL))
    rng = _rng(1)
    v, w = _random_state(cfg, rng), _random_state(cfg, rng)
    lhs = (orc.stream(cfg, v) * w).sum()
    rhs = (v * orc.stream_adjoint(cfg, v, w)).sum()
    assert abs(lhs - rhs) <= 1e-14 * abs(lhs)


def _fd_dir(f, x, v, h):
    return (f(x + h * v) - f(x - h * v)) / (2 * h)


def test_stream_transpose_open_faces(orc):
    cfg = _channel()
    rng = _rng(2)
    x = _random_state(cfg, rng, 1e-2)
    v, w = _random_state(cfg, rng), _random_state(cfg, rng)
    jv = _fd_dir(lambda z: orc.stream(cfg, z), x, v, 1e-4)
    lhs = (jv * w).sum()
    rhs = (v * orc.stream_adjoint(cfg, x, w)).sum()
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


@pytest.mark.parametrize("walls", [False, True])
def test_collision_transpose(orc, walls):
    cfg = _channel() if walls else OracleConfig(q=19, nx=5, ny=4, nz=3, tau=0.7,
                                                force=(1e-3, -2e-3, 5e-4))
    rng = _rng(3)
    d = rng.random(cfg.ncells)
    y = _random_state(cfg, rng, 1e-2)
    v, w = _random_state(cfg, rng), _random_state(cfg, rng)
    ybar, dbar = orc.collide_adjoint(cfg, d, y, w)
    jv = _fd_dir(lambda z: orc.collide(cfg, d, z), y, v, 1e-4)
    assert abs((jv * w).sum() - (v * ybar).sum()) <= 1e-9 * abs((jv * w).sum())
    delta = rng.standard_normal(cfg.ncells)
    jd = _fd_dir(lambda dd: orc.collide(cfg, dd, y), d, delta, 1e-4)
    assert abs((jd * w).sum() - (delta * dbar).sum()) <= 1e-8 * abs((jd * w).sum())


def test_moments_transpose(orc):
    cfg = OracleConfig(q=19, nx=5, ny=4, nz=3, force=(1e-3, 0, 2e-3))
    rng = _rng(4)
    y = _random_state(cfg, rng, 1e-2)
    v = _random_state(cfg, rng)
    rb, ub = rng.standard_normal(cfg.ncells), rng.standard_normal((3, cfg.ncells))

    def obs(z):
        r, u = orc.moments(cfg, z)
        return (r * rb).sum() + (u * ub).sum()
    fd = (obs(y + 1e-4 * v) - obs(y - 1e-4 * v)) / 2e-4
    adj = (v * orc.moments_adjoint(cfg, y, rb, ub)).sum()
    assert abs(fd - adj) <= 1e-9 * abs(fd)


STEPS = 30


def _objective(orc, cfg, d, steps=STEPS):
    g = orc.run(cfg, d, steps)
    drho, u = orc.observe(cfg, g)
    sh = (cfg.nz, cfg.ny, cfg.nx)
    return ob.objective(drho.reshape(sh), u.reshape((3,) + sh), d.reshape(sh), cfg.tau), drho, u


def _gradient(orc, cfg, d, every=7, steps=STEPS):
    J, drho, u = _objective(orc, cfg, d, steps)
    sh = (cfg.nz, cfg.ny, cfg.nx)
    gr, gu, gd = ob.objective_grad(drho.reshape(sh), u.reshape((3,) + sh), d.reshape(sh), cfg.tau)
    return J, orc.gradient(cfg, d, steps, gr.ravel(), gu.reshape(3, -1), every=every) + gd.ravel()


@pytest.fixture(scope="module")
def channel_grad(orc):
    cfg = _channel()
    d = _rng(5).random(cfg.ncells)
    J, g = _gradient(orc, cfg, d)
    return cfg, d, J, g


def test_gradient_matches_central_differences(orc, channel_grad):
    cfg, d, J, g = channel_grad
    fluid = np.nonzero(~cfg.solid_mask().ravel())[0]
    cells = _rng(6).choice(fluid, 20, replace=False)
    h = 1e-4
    scale = np.abs(g).max()
    for c in cells:
        dp, dm = d.copy(), d.copy()
        dp[c] += h
        dm[c] -= h
        fd = (_objective(orc, cfg, dp)[0] - _objective(orc, cfg, dm)[0]) / (2 * h)
        assert abs(fd - g[c]) <= 1e-6 * scale, (c, fd, g[c])
    # solid cells do not influence J
    assert np.all(g[cfg.solid_mask().ravel()] == 0.0)


def test_gradient_taylor_remainder(orc, channel_grad):
    cfg, d, J, g = channel_grad
    delta = _rng(7).standard_normal(cfg.ncells) * (~cfg.solid_mask().ravel())
    rs = []
    for h in (4e-3, 2e-3, 1e-3):
        Jh = _objective(orc, cfg, d + h * delta)[0]
        rs.append(abs(Jh - J - h * (g * delta).sum()))
    assert 3.0 < rs[0] / rs[1] < 5.0 and 3.0 < rs[1] / rs[2] < 5.0


def test_gradient_independent_of_checkpoint_interval(orc, channel_grad):
    cfg, d, J, g = channel_grad
    for every in (1, 4, 30, 100):
        _, g2 = _gradient(orc, cfg, d, every=every)
        assert np.array_equal(g2, g), every
