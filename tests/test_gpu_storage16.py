"""16-bit shifted storage (FP16S, BF16S; FP32 arithmetic) beyond the periodic
scalar workload: walls and open faces, the tensor control, resolved obstacles,
an odd row length (one cell per thread) and D2Q9, against the FP64 oracle.

FP16S: u within 2e-3.  drho is bounded by max(2e-3, 3 x the quantization floor
of one read of the state), because one rounding of the stored populations,
whose magnitudes (~ w 3 c.u) sit far above drho, already costs that much.
BF16S (reported): u and drho within 3 x their floors.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import OracleConfig
from paper_2310_14746_amd import inputs
from tests._parity import quantization_floor, rel_l2_drho, rel_l2_u
from tests.test_gpu_parity import H, say, smooth_noise  # noqa: F401

pytestmark = pytest.mark.gpu

NT = max(1, min(16, os.cpu_count() or 1))
SCALE = 2.0 ** 16   # |g| up to ~1 after the open-face transients, still normal down to ~1e-9
FMT = {"f16s": (10, -14), "bf16s": (7, None)}   # explicit mantissa bits, minimum normal exponent


@pytest.mark.parametrize("storage,q,shape,kind", [
    ("f16s", 19, (33, 9, 7), "periodic"),      # odd row: one cell per thread
    ("f16s", 19, (70, 12, 10), "channel"),     # inlet/outlet in x, walls in y and z
    ("f16s", 19, (40, 9, 8), "tensor"),
    ("f16s", 19, (20, 9, 8), "mask"),
    ("f16s", 9, (64, 32, 1), "walls"),
    ("bf16s", 19, (70, 12, 10), "channel"),
])
def test_storage16_vs_oracle(H, storage, q, shape, kind):
    nx, ny, nz = shape
    steps = 80
    say(f"{storage} D{'3Q19' if q == 19 else '2Q9'} {shape} {kind}, {steps} steps")
    F = (4e-5, -1e-5, 5e-6 if q == 19 else 0.0)
    kw = dict(tau=0.7, force=F)
    ocfg = dict(q=q, nx=nx, ny=ny, nz=nz, tau=0.7, force=F)
    if kind == "channel":
        faces = dict(bc_lo=(2, 1, 1), bc_hi=(3, 1, 1), inlet_u=(0.02, 0.0, 0.0), outlet_rho=1.0)
        kw.update(faces)
        ocfg.update(faces)
        F = (0.0, 0.0, 0.0)
        kw["force"] = ocfg["force"] = F
    if kind == "walls":
        kw.update(bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
        ocfg.update(bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
    cfg = OracleConfig(**ocfg)
    mask = None
    if kind == "tensor":
        D6 = 0.98 * inputs.random_tensor_field((nz, ny, nx), seed=nx)
        D6[:3] += 0.01
        d = inputs.round_to(D6, "f16")
    else:
        d = inputs.round_to(0.4 * smooth_noise((nz, ny, nx), seed=nx), "f16").ravel()
    sim = H.HLBM(q, storage, shape, store_scale=SCALE, porosity="tensor" if kind == "tensor" else "scalar", **kw)
    try:
        sim.set_porosity(d.astype(np.float16))
        if kind == "mask":
            mask = (np.random.default_rng(nx).random(nx * ny * nz) < 0.15).astype(np.uint8)
            sim.set_solid_mask(mask)
        sim.step(steps)
        dr, u = sim.moments("f64")
        dr, u = dr.cpu().numpy().ravel(), u.cpu().numpy().reshape(3, -1)
    finally:
        sim.close()
    d64 = d.astype(np.float64)
    if kind == "tensor":
        g = oracle.run_tensor(cfg, d64, steps, nthreads=NT)
    elif kind == "mask":
        g = oracle.run_masked(cfg, mask, d64, steps, nthreads=NT)
    else:
        g = oracle.run(cfg, d64, steps, nthreads=NT)
    if kind == "mask":
        dro, uo = oracle.observe_masked(cfg, mask, g)
        pre = oracle.stream_masked(cfg, mask, g)
        fluid = mask == 0
    else:
        dro, uo = oracle.observe(cfg, g)
        pre = oracle.stream(cfg, g)
        fluid = ~cfg.solid_mask().ravel()
    eu, er = rel_l2_u(u, uo, fluid), rel_l2_drho(dr, dro, uo, fluid)
    c, _ = oracle.lattice(q)
    bits, emin = FMT[storage]
    fr, fu = quantization_floor(pre[:, fluid], c, SCALE, bits, emin)
    floor_u = fu / np.linalg.norm(uo[:, fluid])
    floor_r = fr / max(np.linalg.norm(dro[fluid]), np.linalg.norm(3.0 * (uo[:, fluid] ** 2).sum(axis=0)))
    say(f"rel-L2 u {eu:.2e} (floor {floor_u:.1e}), drho {er:.2e} (floor {floor_r:.1e})")
    if storage == "f16s":
        assert eu <= 2e-3
        assert er <= max(2e-3, 3.0 * floor_r)
    else:
        assert eu <= max(2e-3, 3.0 * floor_u) and er <= max(2e-3, 3.0 * floor_r)
