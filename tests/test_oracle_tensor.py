"""Pins of the oracle's anisotropic (tensor) porosity control, u_eq = (I - D) u
with D = nu tau K^{-1} symmetric per cell (CPU only).

* D = d I reproduces the scalar oracle (to rounding);
* one collision keeps mass and changes momentum by exactly
  -(j - rho (I - D) u)/tau + (1 - 1/(2 tau)) F;
* a uniform forced periodic box follows the closed form
  u_n = u* + (I - D/tau)^n (F/2 - u*), u* = tau D^{-1} F  (tensor Darcy law
  u* = K F / nu), with off-diagonal D and an oblique force;
* permuting the axes of the problem permutes the solution (index handling of
  the off-diagonal rows).
"""
import numpy as np

import oracle
from oracle import OracleConfig
from paper_2310_14746_amd import inputs


def _spd(seed):
    rng = np.random.default_rng(seed)
    G = rng.uniform(-1, 1, (3, 3))
    M = G @ G.T
    return M / (1.0 + (G * G).sum())


def test_scalar_tensor_reduces_to_scalar():
    cfg = OracleConfig(q=19, nx=10, ny=8, nz=7, tau=0.7, force=(1e-5, -3e-6, 2e-6),
                       bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
    d = inputs.periodic_smooth(inputs.uniform_noise((7, 8, 10), 2), 1.0, 3).ravel()
    D6 = np.zeros((6, d.size))
    D6[0] = D6[1] = D6[2] = d
    gs = oracle.run(cfg, d, 30)
    gt = oracle.run_tensor(cfg, D6, 30)
    assert np.abs(gs - gt).max() <= 1e-14 * np.abs(gs).max()


def test_collision_balance_laws():
    cfg = OracleConfig(q=19, nx=1, ny=1, nz=1, tau=0.8, force=(2e-4, -1e-4, 5e-5))
    c, w = oracle.lattice(19)
    rng = np.random.default_rng(3)
    for k in range(5):
        M = _spd(k)
        D6 = inputs.tensor_rows(M)
        g = 1e-3 * rng.standard_normal(19)
        post = oracle.collide_cell_tensor(cfg, D6, g)
        rho = 1.0 + g.sum()
        j = c.T @ g
        u = (j + 0.5 * np.array(cfg.force)) / rho
        ueq = u - M @ u
        assert abs(post.sum() - g.sum()) <= 2e-16  # rounding of O(1) equilibrium terms
        want = j - (j - rho * ueq) / cfg.tau + (1 - 0.5 / cfg.tau) * np.array(cfg.force)
        np.testing.assert_allclose(c.T @ post, want, rtol=0, atol=2e-16)


def test_uniform_tensor_darcy_closed_form():
    tau = 0.7
    F = np.array([1e-5, -4e-6, 3e-6])
    M = np.array([[0.5, 0.12, -0.05], [0.12, 0.3, 0.08], [-0.05, 0.08, 0.2]])
    assert np.linalg.eigvalsh(M).min() > 0 and np.linalg.eigvalsh(M).max() < 1
    cfg = OracleConfig(q=19, nx=4, ny=3, nz=3, tau=tau, force=tuple(F))
    N = cfg.ncells
    D6 = np.repeat(inputs.tensor_rows(M)[:, None], N, axis=1)
    ustar = tau * np.linalg.solve(M, F)
    A = np.eye(3) - M / tau
    g = None
    for n in (1, 2, 5, 13, 40):
        g = oracle.run_tensor(cfg, D6, n if g is None else n - prev, g)
        prev = n
        dr, u = oracle.observe(cfg, g)
        want = ustar + np.linalg.matrix_power(A, n) @ (0.5 * F - ustar)
        assert np.abs(dr).max() <= 1e-18
        np.testing.assert_allclose(u, np.repeat(want[:, None], N, axis=1), rtol=0,
                                   atol=1e-14 * np.abs(ustar).max() * (n + 1))


def test_axis_permutation_equivariance():
    n = 6
    cfg = OracleConfig(q=19, nx=n, ny=n, nz=n, tau=0.75, force=(1e-5, 3e-6, -2e-6))
    D6 = inputs.random_tensor_field((n, n, n), seed=5)
    g = oracle.run_tensor(cfg, D6, 20)
    dr, u = oracle.observe(cfg, g)
    # cyclic permutation of the axes: new axis a' = old axis perm[a']
    perm = (1, 2, 0)
    P = np.zeros((3, 3))
    for a in range(3):
        P[a, perm[a]] = 1.0
    Mf = np.zeros((n ** 3, 3, 3))
    rows = inputs.TENSOR_ROWS
    idx = {"x": 0, "y": 1, "z": 2}
    for k, r in enumerate(rows):
        a, b = idx[r[0]], idx[r[1]]
        Mf[:, a, b] = Mf[:, b, a] = D6[k]
    Mp = P @ Mf @ P.T
    # fields are (z, y, x) arrays: numpy axis of lattice axis a is 2 - a
    def permute_field(f):
        f = f.reshape(n, n, n)
        # new(x', y', z') = old(x = ..., ...): old axis perm[a] becomes new axis a
        src_axes = [2 - perm[2 - k] for k in range(3)]
        return np.transpose(f, src_axes).ravel()
    Mp_cells = np.stack([permute_field(Mp[:, a, b]) for a in range(3) for b in range(3)]).reshape(3, 3, -1)
    D6p = np.stack([Mp_cells[idx[r[0]], idx[r[1]]] for r in rows])
    Fp = P @ np.array(cfg.force)
    cfgp = OracleConfig(q=19, nx=n, ny=n, nz=n, tau=0.75, force=tuple(Fp))
    gp = oracle.run_tensor(cfgp, D6p, 20)
    drp, up = oracle.observe(cfgp, gp)
    up_want = P @ np.stack([permute_field(u[a]) for a in range(3)])
    # drho cancels (each |g_i| >> |drho|): rounding at 1e-12 of its own size
    np.testing.assert_allclose(drp, permute_field(dr), rtol=0, atol=1e-11 * np.abs(dr).max())
    np.testing.assert_allclose(up, up_want, rtol=0, atol=1e-13 * np.abs(u).max())
