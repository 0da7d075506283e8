"""Padded population rows (hlbm_config.row_pad_bytes) change only where the
rows sit in memory: every observable equals the dense-row run bit for bit --
the state (snapshots are dense either way), the moments and their FP64 totals,
the in-sweep diagnostics and the adjoint gradient -- on every sweep path:
periodic (one cell and two cells per thread), walls and open faces, resolved
obstacles, the tensor control and the in-place pattern."""
import numpy as np
import pytest

from paper_2310_14746_amd import inputs
from tests.test_gpu_parity import H, say, smooth_noise  # noqa: F401

pytestmark = pytest.mark.gpu

SCALE16 = 2.0 ** 14
PADS = (256, 8448, 65536 + 256)

CASES = [
    # q, storage, shape, extra config, porosity, pattern, solid mask
    (19, "f32", (64, 9, 7), {}, "scalar", "ab", False),
    (19, "f16s", (64, 6, 5), {}, "scalar", "ab", False),        # two cells per thread
    (19, "bf16s", (33, 5, 4), {}, "scalar", "ab", False),
    (19, "f64", (40, 12, 10), dict(bc_lo=(2, 1, 1), bc_hi=(3, 1, 1), inlet_u=(0.02, 0, 0)), "scalar", "ab", False),
    (9, "f64", (48, 16, 1), dict(bc_lo=(0, 1, 0), bc_hi=(0, 1, 0)), "scalar", "ab", False),
    (19, "f32", (21, 8, 6), {}, "tensor", "ab", False),
    (19, "f32", (20, 9, 8), {}, "scalar", "ab", True),
    (19, "f32", (30, 9, 7), {}, "scalar", "aa", False),
    (19, "f16s", (24, 9, 8), dict(bc_lo=(0, 1, 1), bc_hi=(0, 1, 1)), "scalar", "aa", False),
]


def _ids(c):
    return f"q{c[0]}-{c[1]}-{c[4]}-{c[5]}-{'x'.join(map(str, c[2]))}{'-faces' if c[3] else ''}{'-mask' if c[6] else ''}"


def _state(storage, q, n, seed):
    import torch
    g = np.random.default_rng(seed).uniform(-0.01, 0.01, size=q * n)
    if storage == "bf16s":
        return torch.tensor(g * SCALE16, dtype=torch.float32).to(torch.bfloat16).view(torch.uint8)
    np_t = {"f64": np.float64, "f32": np.float32, "f16s": np.float16}[storage]
    scale = SCALE16 if storage == "f16s" else 1.0
    return torch.from_numpy(np.ascontiguousarray((g * scale).astype(np_t)).view(np.uint8))


def _run(H, q, storage, shape, extra, porosity, pattern, mask, pad, seed):
    nx, ny, nz = shape
    F = (2e-5, -7e-6, 3e-6 if q == 19 else 0.0)
    sim = H.HLBM(q, storage, shape, tau=0.7, force=F, porosity=porosity, pattern=pattern,
                 store_scale=SCALE16, row_pad=pad, **extra)
    try:
        dt = {"f64": "f64", "f32": "f32"}.get(storage, "f16")
        npt = {"f64": np.float64, "f32": np.float32, "f16": np.float16}[dt]
        if porosity == "tensor":
            D6 = 0.98 * inputs.random_tensor_field((nz, ny, nx), seed=seed)
            D6[:3] += 0.01
            sim.set_porosity(inputs.round_to(D6, dt).astype(npt))
        else:
            sim.set_porosity(inputs.round_to(0.4 * smooth_noise((nz, ny, nx), seed=seed), dt).astype(npt).ravel())
        if mask:
            sim.set_solid_mask((np.random.default_rng(seed).random(nx * ny * nz) < 0.15).astype(np.uint8))
        sim.set_state(_state(storage, q, nx * ny * nz, seed), 0)
        sim.set_diagnostics(2, capacity=16)
        out = []
        for n in (1, 1, 5):
            sim.step(n)
            snap, _ = sim.get_state()
            dr, u, tot = sim.moments("f64", totals=True)
            out.append((snap.cpu().numpy(), dr.cpu().numpy(), u.cpu().numpy(), tot))
        steps, totals, dropped = sim.read_diagnostics()
        out.append((steps, totals, dropped))
        assert sim.pop_bytes == sim.q * (sim.state_bytes // sim.q + pad)
        return out
    finally:
        sim.close()


@pytest.mark.parametrize("case", CASES, ids=[_ids(c) for c in CASES])
def test_padded_rows_bitwise_equal_dense(H, case):
    q, storage, shape, extra, porosity, pattern, mask = case
    say(f"row pad vs dense {_ids(case)}")
    ref = _run(H, q, storage, shape, extra, porosity, pattern, mask, 0, seed=sum(shape))
    for pad in PADS:
        got = _run(H, q, storage, shape, extra, porosity, pattern, mask, pad, seed=sum(shape))
        for a, b in zip(ref[:-1], got[:-1]):
            for x, y in zip(a, b):
                assert np.array_equal(x, y), pad
        assert np.array_equal(ref[-1][0], got[-1][0]) and np.array_equal(ref[-1][1], got[-1][1])


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_padded_rows_adjoint_equal_dense(H, storage):
    """The adjoint rows take the population pitch P too (P counts storage
    elements; FP16S keeps FP32 adjoint rows, so their pad is twice as many
    bytes); the tape's device bytes follow it."""
    shape = (40, 12, 10)
    nx, ny, nz = shape
    n = nx * ny * nz
    say(f"adjoint gradient with padded rows, 40x12x10 channel, {storage}")
    kw = dict(tau=0.6, bc_lo=(2, 1, 1), bc_hi=(3, 1, 1), inlet_u=(0.02, 0, 0))
    elem, dt, scale = {"f32": (4, np.float32, 1.0), "f16s": (2, np.float16, 2.0 ** 14)}[storage]
    d = smooth_noise((nz, ny, nx), seed=3).ravel()
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal(n), rng.standard_normal((3, n))
    grads = []
    for pad in (0, 8448):
        sim = H.HLBM(19, storage, shape, row_pad=pad, store_scale=scale, **kw)
        try:
            sim.set_porosity(d.astype(dt))
            sim.set_tape(6, 30)
            pitch = n + pad // elem
            # 6 checkpoints + 4 replay states, two FP32 adjoint buffers, two moment
            # records of 6 steps (4 FP32 rows of n cells each, dense)
            assert sim.tape_info()["device_bytes"] == (10 * 19 * pitch * elem + 2 * 19 * pitch * 4
                                                       + 2 * 6 * 4 * n * 4)
            sim.step(30)
            grads.append(sim.adjoint(30, a, b).cpu().numpy())
        finally:
            sim.close()
    assert np.any(grads[0])
    assert np.array_equal(grads[0], grads[1])


def test_padded_rows_tensor_adjoint_equal_dense(H):
    """The tensor control's six rows and its six gradient rows at the
    population pitch: the padded layout gives the dense gradient bit for bit,
    in all six rows."""
    shape = (40, 12, 10)
    nx, ny, nz = shape
    n = nx * ny * nz
    say("tensor-control adjoint with padded rows, 40x12x10 channel, f32")
    kw = dict(tau=0.6, bc_lo=(2, 1, 1), bc_hi=(3, 1, 1), inlet_u=(0.02, 0, 0))
    D6 = inputs.random_tensor_field((nz, ny, nx), seed=11).reshape(6, -1).astype(np.float32)
    rng = np.random.default_rng(12)
    a, b = rng.standard_normal(n), rng.standard_normal((3, n))
    grads = []
    for pad in (0, 8448):
        sim = H.HLBM(19, "f32", shape, row_pad=pad, porosity="tensor", **kw)
        try:
            sim.set_porosity(D6)
            sim.set_tape(6, 30)
            sim.step(30)
            grads.append(sim.adjoint(30, a, b).cpu().numpy())
        finally:
            sim.close()
    assert grads[0].shape == (6, nz, ny, nx)
    assert all(np.any(grads[0][r]) for r in range(6))
    assert np.array_equal(grads[0], grads[1])
