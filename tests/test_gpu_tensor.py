"""GPU parity of the anisotropic (tensor) porosity control u_eq = (I - D) u
against the FP64 oracle (same tolerances as the scalar control: FP64 1e-10,
FP32 1e-5), its reduction to the scalar control, validation of D, and the
512^3 fibre-tensor sphere array at full size (every 32^3 tile equals the
oracle's 32^3 run of the same cell)."""
import os

import numpy as np
import pytest

import oracle
from oracle import OracleConfig
from paper_2310_14746_amd import inputs
from tests._parity import rel_l2_drho, rel_l2_u
from tests.test_gpu_parity import H, say, smooth_noise  # noqa: F401

pytestmark = pytest.mark.gpu

NT = max(1, min(16, os.cpu_count() or 1))
TOL = {"f64": 1e-10, "f32": 1e-5}


def _gpu_tensor(H, storage, shape, D6, steps, **kw):
    sim = H.HLBM(19, storage, shape, porosity="tensor", **kw)
    try:
        dt = np.float64 if storage == "f64" else np.float32
        sim.set_porosity(np.ascontiguousarray(D6, dtype=dt))
        sim.step(steps)
        drho, u = sim.moments("f64")
        return drho.cpu().numpy().ravel(), u.cpu().numpy().reshape(3, -1)
    finally:
        sim.close()


@pytest.mark.parametrize("storage,shape,lo,hi,inu,F,steps", [
    ("f64", (40, 9, 8), (0, 0, 0), (0, 0, 0), (0, 0, 0), (2e-5, -7e-6, 3e-6), 60),
    ("f32", (70, 12, 10), (0, 0, 0), (0, 0, 0), (0, 0, 0), (2e-5, -7e-6, 3e-6), 100),
    ("f64", (33, 14, 12), (0, 1, 1), (0, 1, 1), (0, 0, 0), (1e-5, 0, 0), 60),
    ("f32", (30, 12, 10), (2, 1, 1), (3, 1, 1), (0.02, 0, 0), (0, 0, 0), 80),
])
def test_tensor_parity(H, storage, shape, lo, hi, inu, F, steps):
    nx, ny, nz = shape
    say(f"tensor control {storage} {shape} lo={lo} hi={hi} {steps} steps")
    D6 = inputs.random_tensor_field((nz, ny, nx), seed=nx)
    if storage == "f32":
        D6 = inputs.round_to(D6, "f32")
    kw = dict(tau=0.7, force=F, bc_lo=lo, bc_hi=hi, inlet_u=inu, outlet_rho=1.0)
    dr, u = _gpu_tensor(H, storage, shape, D6, steps, **kw)
    cfg = OracleConfig(q=19, nx=nx, ny=ny, nz=nz, **kw)
    g = oracle.run_tensor(cfg, D6, steps, nthreads=NT)
    dr_o, u_o = oracle.observe(cfg, g)
    fl = ~cfg.solid_mask().ravel()
    eu, er = rel_l2_u(u, u_o, fl), rel_l2_drho(dr, dr_o, u_o, fl)
    say(f"rel-L2 u {eu:.2e} drho {er:.2e}")
    assert eu <= TOL[storage] and er <= TOL[storage]


def test_tensor_dI_equals_scalar(H):
    shape, kw = (24, 10, 9), dict(tau=0.8, force=(1e-5, 2e-6, -1e-6), bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
    nx, ny, nz = shape
    d = smooth_noise((nz, ny, nx), seed=4).ravel()
    D6 = np.zeros((6, d.size))
    D6[0] = D6[1] = D6[2] = d
    dr_t, u_t = _gpu_tensor(H, "f64", shape, D6, 50, **kw)
    sim = H.HLBM(19, "f64", shape, **kw)
    try:
        sim.set_porosity(d)
        sim.step(50)
        dr_s, u_s = (a.cpu().numpy() for a in sim.moments("f64"))
    finally:
        sim.close()
    assert rel_l2_u(u_t, u_s.reshape(3, -1)) <= 1e-13


def test_tensor_validation(H):
    n = 4 * 4 * 4
    sim = H.HLBM(19, "f32", (4, 4, 4), porosity="tensor")
    try:
        ok = np.zeros((6, n), dtype=np.float32)
        ok[0] = ok[1] = ok[2] = 1.0               # D = I (eigenvalues exactly 1) is allowed
        sim.set_porosity(ok)
        for bad_rows in ({0: 1.2}, {1: -0.1}, {0: 0.5, 1: 0.5, 3: 0.7}, {4: float("nan")}):
            bad = np.zeros((6, n), dtype=np.float32)
            bad[:3] = 0.3
            for r, v in bad_rows.items():
                bad[r, 17] = v
            with pytest.raises(H.HLBMError, match="eigenvalues"):
                sim.set_porosity(bad)
        with pytest.raises(ValueError):
            sim.set_porosity(np.zeros(n, dtype=np.float32))   # one row only
    finally:
        sim.close()


def test_fibre_tensor_sphere_array_full_size(H):
    """512^3 FP32, 500 steps: every 32^3 tile equals the oracle's 32^3 run."""
    import torch
    n, steps = 512, 500
    say(f"fibre tensor sphere array {n}^3 f32, {steps} steps")
    tile_d = inputs.sphere_array(32)
    tile_D6 = inputs.round_to(inputs.fiber_tensor_field(tile_d), "f32")
    D6 = np.stack([np.tile(r.reshape(32, 32, 32), (n // 32,) * 3).ravel() for r in tile_D6])
    from paper_2310_14746_amd import tune
    # the launch configuration and layout bench.py times for the tensor form
    kw = dict(tau=0.6, force=(1e-6, 0, 0))
    launch = dict(block_x=tune.lookup(19, "f32", (n, n, n)), row_pad=tune.lookup_row_pad(19, "f32", (n, n, n)))
    sim = H.HLBM(19, "f32", (n, n, n), porosity="tensor", **kw, **launch)
    try:
        sim.set_porosity(torch.from_numpy(D6.astype(np.float32)).cuda())
        del D6
        sim.step(steps)
        drho, u = sim.moments("f32")
        u = u.reshape(3, n // 32, 32, n // 32, 32, n // 32, 32)
        ref = u[:, 0, :, 0, :, 0, :]
        same = bool(torch.equal(u, ref[:, None, :, None, :, None, :].expand_as(u)))
        u32 = ref.double().cpu().numpy().reshape(3, -1)
        d32 = drho.reshape(n // 32, 32, n // 32, 32, n // 32, 32)[0, :, 0, :, 0, :].double().cpu().numpy().ravel()
    finally:
        sim.close()
    cfg = OracleConfig(q=19, nx=32, ny=32, nz=32, **kw)
    g = oracle.run_tensor(cfg, tile_D6, steps, nthreads=NT)
    dr_o, u_o = oracle.observe(cfg, g)
    eu, er = rel_l2_u(u32, u_o), rel_l2_drho(d32, dr_o, u_o)
    say(f"tiles identical {same}; tile vs FP64 oracle u {eu:.2e} drho {er:.2e}")
    assert same
    assert eu <= TOL["f32"] and er <= TOL["f32"]
    # the drag is anisotropic: the flow turns toward the fibre direction
    assert abs(u_o[1].mean()) > 1e-3 * abs(u_o[0].mean())
