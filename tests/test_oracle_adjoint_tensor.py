"""Pins of the oracle's discrete adjoint with the tensor control (CPU only).

u_eq = (I - D) u with D symmetric, its six rows xx, yy, zz, xy, xz, yz; an
off-diagonal row is one variable standing at (a, b) and (b, a).

* the transposed collision Jacobian, in the populations and in each of the six
  rows, matches central finite differences of the tensor forward collision;
* at D = d I the adjoint reduces to the scalar one: the same pre_bar, and the
  scalar d_bar equals the sum of the three diagonal rows (the scalar adjoint is
  itself pinned by finite differences of the scalar forward map);
* the full gradient of a linear observation of the moments after 24 steps
  matches central differences in all six rows, with walls and open faces, and
  its Taylor remainder is O(h^2); it does not depend on the checkpoint interval.
"""
import numpy as np
import pytest

from oracle import OracleConfig, WALL, INLET_U, OUTLET_RHO


def _rng(s):
    return np.random.default_rng(s)


def _channel(nx=12, ny=7, nz=6, tau=0.6):
    return OracleConfig(q=19, nx=nx, ny=ny, nz=nz, tau=tau, bc_lo=(INLET_U, WALL, WALL),
                        bc_hi=(OUTLET_RHO, WALL, WALL), inlet_u=(0.02, 0.0, 0.0), outlet_rho=1.0)


def _periodic():
    return OracleConfig(q=19, nx=5, ny=4, nz=3, tau=0.7, force=(1e-3, -2e-3, 5e-4))


def _state(cfg, rng, scale=1e-3):
    g = scale * rng.standard_normal((cfg.q, cfg.ncells))
    g[:, cfg.solid_mask().ravel()] = 0.0
    return g


def _tensor(cfg, rng):
    D6 = np.empty((6, cfg.ncells))
    D6[:3] = 0.1 + 0.4 * rng.random((3, cfg.ncells))
    D6[3:] = 0.1 * rng.uniform(-1.0, 1.0, (3, cfg.ncells))
    return D6


def _fd(f, x, v, h):
    return (f(x + h * v) - f(x - h * v)) / (2 * h)


@pytest.mark.parametrize("walls", [False, True])
def test_tensor_collision_transpose(orc, walls):
    cfg = _channel() if walls else _periodic()
    rng = _rng(11)
    D6 = _tensor(cfg, rng)
    y = _state(cfg, rng, 1e-2)
    v, w = _state(cfg, rng), _state(cfg, rng)
    ybar, Dbar = orc.collide_adjoint_tensor(cfg, D6, y, w)
    jv = _fd(lambda z: orc.collide_tensor(cfg, D6, z), y, v, 1e-4)
    ref = (jv * w).sum()
    assert abs(ref - (v * ybar).sum()) <= 1e-9 * abs(ref)
    for r in range(6):
        delta = np.zeros_like(D6)
        delta[r] = rng.standard_normal(cfg.ncells)
        jd = _fd(lambda DD: orc.collide_tensor(cfg, DD, y), D6, delta, 1e-4)
        ref = (jd * w).sum()
        assert abs(ref - (delta * Dbar).sum()) <= 1e-8 * abs(ref), r
    solid = cfg.solid_mask().ravel()
    assert np.all(Dbar[:, solid] == 0.0) and np.all(ybar[:, solid] == 0.0)


@pytest.mark.parametrize("walls", [False, True])
def test_isotropic_tensor_reduces_to_scalar(orc, walls):
    cfg = _channel() if walls else _periodic()
    rng = _rng(12)
    d = rng.random(cfg.ncells)
    D6 = np.zeros((6, cfg.ncells))
    D6[:3] = d
    y = _state(cfg, rng, 1e-2)
    w = _state(cfg, rng)
    yb_s, db_s = orc.collide_adjoint(cfg, d, y, w)
    yb_t, Db_t = orc.collide_adjoint_tensor(cfg, D6, y, w)
    assert np.allclose(yb_t, yb_s, rtol=1e-13, atol=1e-15 * np.abs(yb_s).max())
    assert np.allclose(Db_t[:3].sum(axis=0), db_s, rtol=1e-12, atol=1e-14 * np.abs(db_s).max())


STEPS = 24


def _observation(cfg, seed):
    rng = _rng(seed)
    return rng.standard_normal(cfg.ncells), rng.standard_normal((3, cfg.ncells))


def _J(orc, cfg, D6, rb, ub):
    drho, u = orc.observe(cfg, orc.run_tensor(cfg, D6, STEPS))
    return (rb * drho).sum() + (ub * u).sum()


@pytest.fixture(scope="module")
def tensor_grad(orc):
    cfg = _channel()
    rng = _rng(13)
    D6 = _tensor(cfg, rng)
    rb, ub = _observation(cfg, 14)
    g = orc.gradient_tensor(cfg, D6, STEPS, rb, ub, every=5)
    return cfg, D6, rb, ub, g


def test_tensor_gradient_matches_central_differences(orc, tensor_grad):
    cfg, D6, rb, ub, g = tensor_grad
    fluid = np.nonzero(~cfg.solid_mask().ravel())[0]
    rng = _rng(15)
    h = 1e-4
    scale = np.abs(g).max()
    for r in range(6):
        for c in rng.choice(fluid, 3, replace=False):
            Dp, Dm = D6.copy(), D6.copy()
            Dp[r, c] += h
            Dm[r, c] -= h
            fd = (_J(orc, cfg, Dp, rb, ub) - _J(orc, cfg, Dm, rb, ub)) / (2 * h)
            assert abs(fd - g[r, c]) <= 1e-6 * scale, (r, c, fd, g[r, c])
    assert np.all(g[:, cfg.solid_mask().ravel()] == 0.0)


def test_tensor_gradient_taylor_remainder(orc, tensor_grad):
    cfg, D6, rb, ub, g = tensor_grad
    delta = _rng(16).standard_normal(D6.shape) * (~cfg.solid_mask().ravel())
    J0 = _J(orc, cfg, D6, rb, ub)
    rs = []
    for h in (4e-3, 2e-3, 1e-3):
        rs.append(abs(_J(orc, cfg, D6 + h * delta, rb, ub) - J0 - h * (g * delta).sum()))
    assert 3.0 < rs[0] / rs[1] < 5.0 and 3.0 < rs[1] / rs[2] < 5.0


def test_tensor_gradient_independent_of_checkpoint_interval(orc, tensor_grad):
    cfg, D6, rb, ub, g = tensor_grad
    for every in (1, 24, 100):
        assert np.array_equal(orc.gradient_tensor(cfg, D6, STEPS, rb, ub, every=every), g), every


def test_isotropic_tensor_gradient_is_scalar_gradient(orc):
    cfg = _channel()
    d = 0.5 * _rng(17).random(cfg.ncells)
    D6 = np.zeros((6, cfg.ncells))
    D6[:3] = d
    rb, ub = _observation(cfg, 18)
    gs = orc.gradient(cfg, d, STEPS, rb, ub, every=6)
    gt = orc.gradient_tensor(cfg, D6, STEPS, rb, ub, every=6)
    assert np.allclose(gt[:3].sum(axis=0), gs, rtol=1e-10, atol=1e-12 * np.abs(gs).max())
