"""GPU parity with walls and open faces: the planar porous channel (FP64,
relative L2 1e-12), ducts with bounce-back walls and inlet/outlet faces, against
the FP64 oracle.  Collected after the periodic parity file."""
import os

import numpy as np
import pytest

import oracle
from oracle import OracleConfig
from paper_2310_14746_amd import inputs
from tests._parity import rel_l2_drho, rel_l2_u
from tests.test_gpu_parity import H, gpu_run, say, smooth_noise  # noqa: F401

pytestmark = pytest.mark.gpu

NT = max(1, min(16, os.cpu_count() or 1))
TOL = {"f64": 1e-10, "f32": 1e-5}


def test_channel_c0_f64(H):
    """D2Q9 FP64 128x64 porous channel, 2000 steps from rest."""
    say("C0 D2Q9 f64 128x64 walls y, 2000 steps")
    d = inputs.channel_2d().ravel()
    kw = dict(tau=0.8, force=(1e-6, 0, 0), bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
    dr, u, tot, _ = gpu_run(H, 9, "f64", (128, 64, 1), d, 2000, **kw)
    cfg = OracleConfig(q=9, nx=128, ny=64, nz=1, tau=0.8, force=(1e-6, 0, 0),
                       bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
    g = oracle.run(cfg, d, 2000, nthreads=NT)
    dr_o, u_o = oracle.observe(cfg, g)
    fluid = ~cfg.solid_mask().ravel()
    eu, er = rel_l2_u(u, u_o, fluid), rel_l2_drho(dr, dr_o, u_o, fluid)
    say(f"C0 rel-L2 u {eu:.2e} drho {er:.2e}")
    assert eu <= 1e-12 and er <= 1e-12
    # solid rows report zeros
    assert (dr[~fluid] == 0).all() and (u[:, ~fluid] == 0).all()
    # FP64 totals: mass excess stays at rounding level (start: 0), momentum matches
    n_fluid = fluid.sum()
    assert abs(tot[0]) / n_fluid <= 1e-12
    mom_o = ((1.0 + dr_o) * u_o)[:, fluid].sum(axis=1)
    assert np.isclose(tot[1], mom_o[0], rtol=1e-12, atol=0)
    # u_y is zero in exact arithmetic: its total is rounding noise on both sides
    assert abs(tot[2]) <= 1e-12 * abs(tot[1]) and abs(mom_o[1]) <= 1e-12 * abs(mom_o[0])
    # centreline Darcy value F tau / d and mirror symmetry through the HIP path
    U = u[0].reshape(64, 128)
    assert abs(U[31, 0] / (1e-6 * 0.8 / 0.5) - 1) < 1e-6
    assert np.abs(U[1:63] - U[62:0:-1]).max() <= 1e-12 * np.abs(U).max()



@pytest.mark.parametrize("storage,shape,lo,hi,inu,F,steps", [
    ("f64", (33, 14, 12), (0, 1, 1), (0, 1, 1), (0, 0, 0), (1e-5, 0, 0), 60),
    ("f32", (70, 10, 9), (1, 1, 0), (1, 1, 0), (0, 0, 0), (0, 1e-5, 2e-6), 80),
    ("f64", (30, 12, 10), (2, 1, 1), (3, 1, 1), (0.02, 0, 0), (0, 0, 0), 80),
    ("f32", (130, 12, 10), (2, 1, 1), (3, 1, 1), (0.02, 0, 0), (0, 0, 0), 120),
    ("f32", (20, 9, 8), (2, 0, 1), (3, 0, 1), (0.01, 0.002, 0), (0, 1e-5, 0), 40),
])
def test_walls_and_open_faces(H, storage, shape, lo, hi, inu, F, steps):
    nx, ny, nz = shape
    say(f"D3Q19 {storage} {shape} lo={lo} hi={hi} inlet={inu} {steps} steps")
    dt = "f64" if storage == "f64" else "f32"
    d = inputs.round_to(smooth_noise((nz, ny, nx), seed=nx + ny), dt).ravel()
    kw = dict(tau=0.7, force=F, bc_lo=lo, bc_hi=hi, inlet_u=inu, outlet_rho=1.0)
    dr, u, tot, _ = gpu_run(H, 19, storage, shape, d.astype(np.float64 if dt == "f64" else np.float32),
                            steps, **kw)
    cfg = OracleConfig(q=19, nx=nx, ny=ny, nz=nz, tau=0.7, force=F, bc_lo=lo, bc_hi=hi,
                       inlet_u=inu, outlet_rho=1.0)
    g = oracle.run(cfg, d, steps, nthreads=NT)
    dr_o, u_o = oracle.observe(cfg, g)
    fluid = ~cfg.solid_mask().ravel()
    eu, er = rel_l2_u(u, u_o, fluid), rel_l2_drho(dr, dr_o, u_o, fluid)
    say(f"rel-L2 u {eu:.2e} drho {er:.2e}")
    assert eu <= TOL[storage] and er <= TOL[storage]
    assert (dr[~fluid] == 0).all() and (u[:, ~fluid] == 0).all()


@pytest.mark.parametrize("storage,shape,lo,hi,inu,F,steps", [
    ("f64", (70, 20, 1), (2, 1, 0), (3, 1, 0), (0.02, 0, 0), (0, 0, 0), 80),   # D2Q9 channel with open ends
    ("f32", (66, 17, 1), (1, 2, 0), (1, 3, 0), (0, 0.01, 0), (1e-5, 0, 0), 60),  # x walls, open y faces
])
def test_d2q9_walls_and_open_faces(H, storage, shape, lo, hi, inu, F, steps):
    """D2Q9 with open faces: the plain rows' x-end fix (open x faces) and the
    x-wall bounce-back fix with open faces on the rows next to them."""
    nx, ny, nz = shape
    say(f"D2Q9 {storage} {shape} lo={lo} hi={hi} inlet={inu} {steps} steps")
    dt = "f64" if storage == "f64" else "f32"
    d = inputs.round_to(smooth_noise((nz, ny, nx), seed=nx + ny), dt).ravel()
    kw = dict(tau=0.7, force=F, bc_lo=lo, bc_hi=hi, inlet_u=inu, outlet_rho=1.0)
    dr, u, tot, _ = gpu_run(H, 9, storage, shape, d.astype(np.float64 if dt == "f64" else np.float32),
                            steps, **kw)
    cfg = OracleConfig(q=9, nx=nx, ny=ny, nz=nz, tau=0.7, force=F, bc_lo=lo, bc_hi=hi,
                       inlet_u=inu, outlet_rho=1.0)
    g = oracle.run(cfg, d, steps, nthreads=NT)
    dr_o, u_o = oracle.observe(cfg, g)
    fluid = ~cfg.solid_mask().ravel()
    eu, er = rel_l2_u(u, u_o, fluid), rel_l2_drho(dr, dr_o, u_o, fluid)
    say(f"rel-L2 u {eu:.2e} drho {er:.2e}")
    assert eu <= TOL[storage] and er <= TOL[storage]
    assert (dr[~fluid] == 0).all() and (u[:, ~fluid] == 0).all()


def test_in_sweep_diagnostics_equal_moment_totals(H):
    """Totals reduced inside the sweep equal hlbm_moments' totals at the same
    time level bit for bit; FP64 mass stays at rounding level; the log drops
    (and counts) records beyond its capacity."""
    say("in-sweep diagnostics, C0 channel f64 and a D3Q19 f32 duct")
    d = inputs.channel_2d().ravel()
    sim = H.HLBM(9, "f64", (128, 64, 1), tau=0.8, force=(1e-6, 0, 0), bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
    try:
        sim.set_porosity(d)
        sim.set_diagnostics(100, capacity=64)
        ref = {}
        for n in range(0, 2001, 100):
            ref[n] = sim.totals()
            if n < 2000:
                sim.step(100)
        steps, tot, dropped = sim.read_diagnostics()
        assert list(steps) == list(range(0, 2000, 100)) and dropped == 0
        for n, t in zip(steps, tot):
            assert np.array_equal(t, ref[n]), n
        n_fluid = 128 * 62
        assert np.abs(tot[:, 0]).max() / n_fluid <= 1e-12
    finally:
        sim.close()
    shape = (40, 12, 10)
    sim = H.HLBM(19, "f32", shape, tau=0.7, force=(1e-5, 0, 0), bc_lo=(0, 1, 1), bc_hi=(0, 1, 1))
    try:
        sim.set_porosity(inputs.round_to(smooth_noise((10, 12, 40), seed=8), "f32").astype(np.float32).ravel())
        sim.set_diagnostics(1, capacity=5)
        sim.step(3)
        t3 = sim.totals()
        sim.step(5)
        steps, tot, dropped = sim.read_diagnostics()
        assert list(steps) == [0, 1, 2, 3, 4] and dropped == 3
        assert np.array_equal(tot[3], t3)
        sim.step(2)
        steps, tot, dropped = sim.read_diagnostics()
        assert list(steps) == [8, 9] and dropped == 0
        assert np.isfinite(tot).all()
    finally:
        sim.close()


@pytest.mark.parametrize("q,storage,shape,lo,hi,porosity", [
    (19, "f32", (70, 12, 10), (2, 1, 1), (3, 1, 1), "scalar"),     # channel: inlet/outlet x, walls y, z
    (19, "f64", (33, 9, 7), (0, 1, 0), (0, 1, 0), "scalar"),       # walls in y only
    (19, "f32", (21, 8, 6), (1, 1, 1), (1, 1, 1), "tensor"),       # closed box, tensor control
    (9, "f64", (128, 64, 1), (0, 1, 0), (0, 1, 0), "scalar"),      # the D2Q9 channel
    (19, "f32", (4, 5, 9), (2, 1, 1), (3, 1, 1), "scalar"),        # every cell next to a face
])
def test_diagnostic_sweep_bitwise_with_faces(H, q, storage, shape, lo, hi, porosity):
    """With walls or open faces, the diagnostic sweep (which also reduces the
    totals) and the plain sweep write the same state bit for bit."""
    nx, ny, nz = shape
    say(f"diagnostic sweep D{'3Q19' if q == 19 else '2Q9'} {storage} {shape} faces {lo}/{hi} {porosity}")
    dt = "f64" if storage == "f64" else "f32"
    npt = np.float64 if dt == "f64" else np.float32
    if porosity == "tensor":
        d = 0.98 * inputs.random_tensor_field((nz, ny, nx), seed=3)
        d[:3] += 0.01
        d = inputs.round_to(d, dt).astype(npt)
    else:
        d = inputs.round_to(0.4 * smooth_noise((nz, ny, nx), seed=nx), dt).astype(npt).ravel()
    kw = dict(tau=0.7, force=(2e-5, -7e-6, 3e-6 if q == 19 else 0.0), bc_lo=lo, bc_hi=hi,
              inlet_u=(0.02, 0.001, 0.0), porosity=porosity)
    states = []
    for diag in (0, 1):
        sim = H.HLBM(q, storage, shape, **kw)
        try:
            sim.set_porosity(d)
            if diag:
                sim.set_diagnostics(1, capacity=64)
            sim.step(29)
            states.append(sim.get_state()[0].cpu().numpy())
        finally:
            sim.close()
    assert np.array_equal(states[0], states[1])
