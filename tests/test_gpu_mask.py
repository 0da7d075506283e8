"""Resolved obstacles (per-cell solid mask, halfway bounce-back) on the GPU:
parity with the oracle (FP64 1e-10, FP32 1e-5), two wall rows equal the wall
faces bit for bit, Hasimoto's drag of a sphere array at a finer resolution, and
the resolved unit cells of the batched workload against their homogenized
controls (reported: the homogenization error; parity unpinned)."""
import math
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


def _run(H, q, storage, shape, d, mask, steps, **kw):
    sim = H.HLBM(q, storage, shape, **kw)
    try:
        sim.set_porosity(d)
        sim.set_solid_mask(mask)
        sim.step(steps)
        drho, u, tot = sim.moments("f64", totals=True)
        return drho.cpu().numpy().ravel(), u.cpu().numpy().reshape(3, -1), tot, sim.get_state()[0].cpu().numpy()
    finally:
        sim.close()


@pytest.mark.parametrize("q,storage,shape,steps", [
    (19, "f64", (20, 9, 8), 40),
    (19, "f32", (70, 12, 10), 100),
    (9, "f64", (30, 20, 1), 60),
])
def test_masked_parity(H, q, storage, shape, steps):
    nx, ny, nz = shape
    say(f"solid mask {storage} D{'3Q19' if q == 19 else '2Q9'} {shape} {steps} steps")
    dt = "f64" if storage == "f64" else "f32"
    d = inputs.round_to(0.3 * smooth_noise((nz, ny, nx), seed=nx), dt).ravel()
    mask = (np.random.default_rng(nx).random(nx * ny * nz) < 0.2).astype(np.uint8)
    F = (2e-5, -7e-6, 3e-6 if q == 19 else 0.0)
    dr, u, tot, _ = _run(H, q, storage, shape, d.astype(np.float64 if dt == "f64" else np.float32), mask,
                         steps, tau=0.7, force=F)
    cfg = OracleConfig(q=q, nx=nx, ny=ny, nz=nz, tau=0.7, force=F)
    g = oracle.run_masked(cfg, mask, d, steps, nthreads=NT)
    dro, uo = oracle.observe_masked(cfg, mask, g)
    fl = mask == 0
    eu, er = rel_l2_u(u, uo, fl), rel_l2_drho(dr, dro, uo, fl)
    say(f"rel-L2 u {eu:.2e} drho {er:.2e}")
    assert eu <= TOL[storage] and er <= TOL[storage]
    assert (u[:, ~fl] == 0).all() and (dr[~fl] == 0).all()


def test_wall_rows_mask_equals_wall_faces(H):
    shape = (40, 12, 10)
    nx, ny, nz = shape
    d = inputs.round_to(smooth_noise((nz, ny, nx), seed=2), "f32").astype(np.float32).ravel()
    kw = dict(tau=0.8, force=(1e-5, 0, 2e-6))
    sim = H.HLBM(19, "f32", shape, bc_lo=(0, 1, 0), bc_hi=(0, 1, 0), **kw)
    try:
        sim.set_porosity(d)
        sim.step(50)
        ref = sim.get_state()[0].cpu().numpy()
    finally:
        sim.close()
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    mask[:, 0, :] = mask[:, ny - 1, :] = 1
    _, _, _, st = _run(H, 19, "f32", shape, d, mask, 50, **kw)
    assert np.array_equal(st, ref)


def test_hasimoto_drag_fine(H):
    """Sphere of radius 8 in a 48^3 periodic cell (solid fraction 0.019)."""
    L, a, tau, F = 48, 8.0, 1.0, 1e-6
    nu = (tau - 0.5) / 3.0
    mask = inputs.sphere_indicator(L, a) > 0.5
    steps = 30000
    say(f"Hasimoto sphere array {L}^3, a={a}, {steps} steps")
    dr, u, tot, _ = _run(H, 19, "f64", (L, L, L), np.zeros(L ** 3), mask.astype(np.uint8), steps,
                         tau=tau, force=(F, 0, 0))
    U = tot[1] / L ** 3
    c = mask.sum() / L ** 3
    a_eff = (3.0 * mask.sum() / (4.0 * math.pi)) ** (1.0 / 3.0)
    K = F * (L ** 3 - mask.sum()) / (6.0 * math.pi * nu * a_eff * U)
    K_h = 1.0 / (1.0 - 1.7601 * c ** (1.0 / 3.0) + c - 1.5593 * c * c)
    say(f"drag coefficient {K:.4f} vs Hasimoto {K_h:.4f} ({100 * (K / K_h - 1):+.2f}%)")
    assert abs(K / K_h - 1.0) <= 0.05


def test_resolved_vs_homogenized_unit_cells(H):
    """Unit cells resolved with a bounce-back sphere against the same cells with
    the homogenized (smoothed) control and with the sharp indicator as control,
    at steady state (five viscous diffusion times of the cell)."""
    from paper_2310_14746_amd import permeability
    spec = [(32, 0.3, 1.0), (32, 0.6, 0.8), (48, 0.45, 0.9), (48, 0.8, 1.0)]
    items = [dict(shape=(e, e, e), tau=t, force=(1e-6, 0, 0)) for e, _, t in spec]
    smooth = [inputs.round_to(inputs.batch_item_field(e, phi), "f32").astype(np.float32).ravel()
              for e, phi, _ in spec]
    sharp = [inputs.round_to(inputs.sphere_indicator(e, inputs.radius_for_porosity(e, phi)), "f32")
             .astype(np.float32).ravel() for e, phi, _ in spec]
    steps = int(5 * max(e * e / ((t - 0.5) / 3.0) for e, _, t in spec))
    say(f"resolved vs homogenized unit cells, {steps} steps")
    k_s = permeability.transient_permeability(H, items, smooth, [steps])[-1]
    k_i = permeability.transient_permeability(H, items, sharp, [steps])[-1]
    for j, ((e, phi, tau), it) in enumerate(zip(spec, items)):
        nu = (tau - 0.5) / 3.0
        mask = inputs.sphere_indicator(e, inputs.radius_for_porosity(e, phi)) > 0.5
        _, _, tot, _ = _run(H, 19, "f32", (e, e, e), np.zeros(e ** 3, dtype=np.float32),
                            mask.astype(np.uint8), steps, tau=tau, force=it["force"])
        k_r = nu * (tot[1] / e ** 3) / it["force"][0]
        say(f"cell {j}: E={e} phi={phi:.2f} tau={tau}: k resolved {k_r:.4g}, homogenized {k_s[j]:.4g} "
            f"({100 * (k_s[j] / k_r - 1):+.1f}%), sharp control {k_i[j]:.4g} ({100 * (k_i[j] / k_r - 1):+.1f}%)")
        assert k_r > 0 and np.isfinite(k_r)


def test_mask_api_rules(H):
    """Host-side rules of hlbm_set_solid_mask (no kernel runs on bad input)."""
    n = 8 ** 3
    walls = H.HLBM(19, "f32", (8, 8, 8), bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
    try:
        with pytest.raises(H.HLBMError, match="periodic"):
            walls.set_solid_mask(np.zeros(n, dtype=np.uint8))
    finally:
        walls.close()
    sim = H.HLBM(19, "f64", (8, 8, 8), force=(1e-5, 0, 0))
    try:
        sim.set_porosity(np.zeros(n))
        with pytest.raises(ValueError):
            sim.set_solid_mask(np.zeros(n - 1, dtype=np.uint8))
        sim.set_tape(2, 10)
        with pytest.raises(H.HLBMError, match="tape"):
            sim.set_solid_mask(np.zeros(n, dtype=np.uint8))
        sim.set_tape(0, 0)
        mask = np.zeros(n, dtype=np.uint8)
        mask[100] = 1
        sim.set_solid_mask(mask)
        with pytest.raises(H.HLBMError, match="solid"):
            sim.set_tape(2, 10)
        sim.step(3)
        drho, u = sim.moments("f64")
        assert float(u.reshape(3, -1)[:, 100].abs().max()) == 0.0
        sim.set_solid_mask(None)            # obstacles removed: the adjoint is available again
        sim.set_tape(2, 10)
    finally:
        sim.close()


@pytest.mark.parametrize("storage,shape,steps", [("f64", (18, 9, 7), 40), ("f32", (70, 10, 8), 80)])
def test_masked_tensor_parity(H, storage, shape, steps):
    """Resolved obstacles with the anisotropic (tensor) control in the fluid.
    The oracle composes its masked pull, its tensor collision and zeroed solid
    cells step by step."""
    nx, ny, nz = shape
    say(f"solid mask + tensor control {storage} {shape} {steps} steps")
    dt = "f64" if storage == "f64" else "f32"
    D6 = 0.98 * inputs.random_tensor_field((nz, ny, nx), seed=nx)
    D6[:3] += 0.01
    D6 = inputs.round_to(D6, dt)
    mask = (np.random.default_rng(nx + 1).random(nx * ny * nz) < 0.15).astype(np.uint8)
    F = (2e-5, -7e-6, 3e-6)
    sim = H.HLBM(19, storage, shape, tau=0.7, force=F, porosity="tensor")
    try:
        sim.set_porosity(D6.astype(np.float64 if dt == "f64" else np.float32))
        sim.set_solid_mask(mask)
        sim.step(steps)
        dr, u = sim.moments("f64")
        dr, u = dr.cpu().numpy().ravel(), u.cpu().numpy().reshape(3, -1)
    finally:
        sim.close()
    cfg = OracleConfig(q=19, nx=nx, ny=ny, nz=nz, tau=0.7, force=F)
    solid = mask != 0
    g = np.zeros((19, nx * ny * nz))
    for _ in range(steps):
        g = oracle.collide_tensor(cfg, D6, oracle.stream_masked(cfg, mask, g, nthreads=NT), nthreads=NT)
        g[:, solid] = 0.0
    dro, uo = oracle.observe_masked(cfg, mask, g)
    eu, er = rel_l2_u(u, uo, ~solid), rel_l2_drho(dr, dro, uo, ~solid)
    say(f"rel-L2 u {eu:.2e} drho {er:.2e}")
    assert eu <= TOL[storage] and er <= TOL[storage]
    assert (u[:, solid] == 0).all() and (dr[solid] == 0).all()
