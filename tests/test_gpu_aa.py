"""In-place (AA) pattern on the GPU, through the C-ABI.

One population buffer, updated in place, with steps alternating between a
local form and a shifted form.  Each cell does the arithmetic of the
two-buffer pull sweep, so every observable must equal the two-buffer run bit
for bit: the state (exported to the two-buffer layout), the moments, their
FP64 totals and the in-sweep diagnostics, after odd and even step counts,
for every storage form, both lattices and both control kinds, at ragged sizes
and at the full 512^3 size; with wall faces (halfway bounce-back) on any set
of axes as well.  One case is also checked directly against the oracle, and
the host-side rules of the pattern are exercised.
"""
import ctypes
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
SCALE16 = 2.0 ** 14   # headroom for |g| ~ 0.05 after a step from a random state
NP_STORE = {"f64": np.float64, "f32": np.float32, "f16s": np.float16}


def _random_state(storage, q, n, seed):
    """Stored populations (bytes) of a perturbed state, |g| <= 0.01."""
    import torch
    g = np.random.default_rng(seed).uniform(-0.01, 0.01, size=q * n)
    if storage == "bf16s":
        return torch.tensor(g * SCALE16, dtype=torch.float32).to(torch.bfloat16).view(torch.uint8)
    scale = SCALE16 if storage == "f16s" else 1.0
    return torch.from_numpy(np.ascontiguousarray((g * scale).astype(NP_STORE[storage])).view(np.uint8))


def _control(storage, shape, porosity, seed):
    nx, ny, nz = shape
    dt = {"f64": "f64", "f32": "f32"}.get(storage, "f16")
    npt = {"f64": np.float64, "f32": np.float32, "f16": np.float16}[dt]
    if porosity == "tensor":
        # eigenvalues kept inside [0.01, 0.99], clear of the bounds after rounding
        D6 = 0.98 * inputs.random_tensor_field((nz, ny, nx), seed=seed)
        D6[:3] += 0.01
        return inputs.round_to(D6, dt).astype(npt)
    return inputs.round_to(0.4 * smooth_noise((nz, ny, nx), seed=seed), dt).astype(npt).ravel()


def _pair(H, q, storage, shape, porosity="scalar", diag=False, seed=0, **kw):
    sims = []
    kw = dict(dict(tau=0.7, force=(2e-5, -7e-6, 3e-6 if q == 19 else 0.0), store_scale=SCALE16), **kw)
    state = _random_state(storage, q, int(np.prod(shape)), seed)
    d = _control(storage, shape, porosity, seed + 1)
    for pattern in ("ab", "aa"):
        sim = H.HLBM(q, storage, shape, porosity=porosity, pattern=pattern, **kw)
        sim.set_porosity(d)
        sim.set_state(state, 0)
        if diag:
            sim.set_diagnostics(1, capacity=64)
        sims.append(sim)
    return sims


def _assert_same(ab, aa):
    import torch
    sa, na = ab.get_state()
    sb, nb = aa.get_state()
    assert na == nb
    assert torch.equal(sa, sb), "state differs"
    ra, ua, ta = ab.moments("f64", totals=True)
    rb, ub, tb = aa.moments("f64", totals=True)
    assert torch.equal(ra, rb) and torch.equal(ua, ub), "moments differ"
    assert np.array_equal(ta, tb), "totals differ"
    r32a, u32a = ab.moments("f32", device=False)
    r32b, u32b = aa.moments("f32", device=False)
    assert torch.equal(r32a, r32b) and torch.equal(u32a, u32b)


@pytest.mark.parametrize("q,storage,shape,porosity", [
    (19, "f64", (37, 9, 7), "scalar"),
    (19, "f32", (300, 9, 7), "scalar"),
    (19, "f16s", (64, 6, 5), "scalar"),
    (19, "bf16s", (33, 4, 3), "scalar"),
    (19, "f32", (21, 8, 6), "tensor"),
    (19, "f64", (16, 5, 4), "tensor"),
    (9, "f64", (45, 30, 1), "scalar"),
    (9, "f32", (2, 3, 1), "scalar"),
    (19, "f32", (1, 1, 1), "scalar"),
    (19, "f16s", (2, 2, 2), "scalar"),
])
def test_aa_equals_ab_bitwise(H, q, storage, shape, porosity):
    say(f"AA vs AB D{'3Q19' if q == 19 else '2Q9'} {storage} {porosity} {shape}")
    ab, aa = _pair(H, q, storage, shape, porosity, seed=sum(shape))
    try:
        for n in (1, 1, 1, 14, 7):          # time levels 1, 2, 3, 17, 24
            ab.step(n)
            aa.step(n)
            _assert_same(ab, aa)
    finally:
        ab.close()
        aa.close()


WALL_CASES = [
    # q, storage, shape, porosity, wall axes (bc_lo = bc_hi; 1 = wall, 0 = periodic)
    (9, "f64", (24, 16, 1), "scalar", (0, 1, 0)),
    (9, "f32", (17, 12, 1), "scalar", (1, 1, 0)),
    (19, "f64", (13, 9, 8), "scalar", (0, 1, 1)),
    (19, "f32", (70, 9, 7), "scalar", (1, 1, 1)),
    (19, "f16s", (40, 6, 5), "scalar", (0, 0, 1)),
    (19, "bf16s", (33, 5, 4), "scalar", (1, 0, 0)),
    (19, "f32", (21, 8, 6), "tensor", (0, 1, 1)),
    (19, "f64", (9, 8, 7), "tensor", (1, 0, 1)),
    (19, "f32", (3, 3, 3), "scalar", (1, 1, 1)),
]


@pytest.mark.parametrize("q,storage,shape,porosity,walls", WALL_CASES,
                         ids=[f"q{c[0]}-{c[1]}-{c[3]}-{c[2][0]}x{c[2][1]}x{c[2][2]}-w{''.join(map(str, c[4]))}"
                              for c in WALL_CASES])
def test_aa_walls_equal_ab_bitwise(H, q, storage, shape, porosity, walls):
    say(f"AA vs AB with walls {walls} D{'3Q19' if q == 19 else '2Q9'} {storage} {porosity} {shape}")
    ab, aa = _pair(H, q, storage, shape, porosity, seed=sum(shape) + 1, bc_lo=walls, bc_hi=walls)
    try:
        for n in (1, 1, 1, 14, 7):
            ab.step(n)
            aa.step(n)
            _assert_same(ab, aa)
    finally:
        ab.close()
        aa.close()


def test_aa_walls_channel_c0(H):
    """The D2Q9 wall channel (128 x 64, walls at y = 0 and 63, d = 0.5 on rows
    16..47), 2000 steps in place: equal to the two-buffer run bit for bit."""
    nx, ny = 128, 64
    say("AA vs AB, D2Q9 wall channel 128x64, 2000 steps")
    d = np.zeros((ny, nx))
    d[16:48] = 0.5
    sims = [H.HLBM(9, "f64", (nx, ny, 1), tau=0.8, force=(1e-6, 0, 0), bc_lo=(0, 1, 0), bc_hi=(0, 1, 0),
                   pattern=p) for p in ("ab", "aa")]
    try:
        for s in sims:
            s.set_porosity(d.ravel())
            s.step(2000)
        _assert_same(*sims)
        sims[0].step(1)
        sims[1].step(1)
        _assert_same(*sims)
    finally:
        for s in sims:
            s.close()


def test_aa_walls_state_export(H):
    """get_state from either slot order, device and host, with walls."""
    import torch
    shape = (30, 9, 8)
    say(f"AA state export with walls {shape}")
    ab, aa = _pair(H, 19, "f32", shape, seed=13, bc_lo=(1, 0, 1), bc_hi=(1, 0, 1))
    lib = H.load()
    try:
        for n in (3, 2):
            ab.step(n)
            aa.step(n)
            snap, s = aa.get_state()
            host = np.empty(aa.state_bytes, dtype=np.uint8)
            assert lib.hlbm_get_state(aa.ctx, host.ctypes.data, 0, None) == 0
            assert np.array_equal(host, snap.cpu().numpy())
            assert torch.equal(snap, ab.get_state()[0])
    finally:
        ab.close()
        aa.close()


def test_aa_diagnostics_equal_ab(H):
    for walls in ((0, 0, 0), (1, 1, 0)):
        say(f"AA vs AB in-sweep diagnostics, walls {walls}")
        ab, aa = _pair(H, 19, "f32", (70, 12, 10), diag=True, seed=5, bc_lo=walls, bc_hi=walls)
        try:
            ab.step(9)
            aa.step(9)
            sa, ta, da = ab.read_diagnostics()
            sb, tb, db = aa.read_diagnostics()
            assert np.array_equal(sa, sb) and da == db == 0
            assert np.array_equal(ta, tb)
            _assert_same(ab, aa)
        finally:
            ab.close()
            aa.close()


def test_aa_state_roundtrip_and_host_paths(H):
    """get_state from either slot order, to device and host destinations,
    equals the two-buffer state."""
    import torch
    shape = (40, 7, 6)
    say(f"AA state round trip {shape}")
    ab, aa = _pair(H, 19, "f32", shape, seed=9)
    lib = H.load()
    try:
        for n in (5, 4):                    # odd then even time level
            ab.step(n)
            aa.step(n)
            snap, s = aa.get_state()
            host = np.empty(aa.state_bytes, dtype=np.uint8)
            step = ctypes.c_longlong()
            assert lib.hlbm_get_state(aa.ctx, host.ctypes.data, 0, ctypes.byref(step)) == 0
            assert step.value == s
            assert np.array_equal(host, snap.cpu().numpy())
            assert torch.equal(snap, ab.get_state()[0])
    finally:
        ab.close()
        aa.close()


def test_aa_resume_from_snapshot(H):
    import torch
    shape = (24, 10, 5)
    say(f"AA resume from snapshot {shape}")
    d = _control("f64", shape, "scalar", 3)
    sim = H.HLBM(19, "f64", shape, tau=0.8, force=(1e-5, 2e-6, 0), pattern="aa")
    try:
        sim.set_porosity(d)
        sim.step(13)
        snap, s = sim.get_state()
        sim.step(8)
        ref = sim.get_state()[0]
        sim.reset()
        sim.set_state(snap.cpu(), s)        # host source
        sim.step(8)
        assert sim.step_count == 21
        assert torch.equal(sim.get_state()[0], ref)
        sim.set_state(snap, s)              # device source
        sim.step(8)
        assert torch.equal(sim.get_state()[0], ref)
    finally:
        sim.close()


def test_aa_oracle_parity(H):
    shape = (20, 9, 8)
    nx, ny, nz = shape
    steps = 41
    say(f"AA vs oracle f64 {shape} {steps} steps")
    d = inputs.round_to(0.3 * smooth_noise((nz, ny, nx), seed=4), "f64").ravel()
    F = (2e-5, -7e-6, 3e-6)
    sim = H.HLBM(19, "f64", shape, tau=0.7, force=F, pattern="aa")
    try:
        sim.set_porosity(d)
        sim.step(steps)
        dr, u = sim.moments("f64")
        dr, u = dr.cpu().numpy().ravel(), u.cpu().numpy().reshape(3, -1)
    finally:
        sim.close()
    cfg = OracleConfig(q=19, nx=nx, ny=ny, nz=nz, tau=0.7, force=F)
    g = oracle.run(cfg, d, steps, nthreads=NT)
    dro, uo = oracle.observe(cfg, g)
    eu, er = rel_l2_u(u, uo), rel_l2_drho(dr, dro, uo)
    say(f"rel-L2 u {eu:.2e} drho {er:.2e}")
    assert eu <= 1e-10 and er <= 1e-10


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_aa_full_size_equals_ab(H, storage):
    """The 512^3 box the throughput is quoted on, from a random state with a
    random control: three steps (the buffer then holds pulled populations) and
    a fourth, state and totals bit for bit."""
    import torch
    n = 512
    say(f"AA vs AB full size {storage} {n}^3")
    gen = torch.Generator(device="cuda").manual_seed(7)
    g = (torch.rand(19 * n ** 3, generator=gen, device="cuda") - 0.5) * 0.02
    state = (g if storage == "f32" else (g * SCALE16).half()).view(torch.uint8)
    del g
    d = (torch.rand(n ** 3, generator=gen, device="cuda") * 0.6).to(
        torch.float32 if storage == "f32" else torch.float16)
    from paper_2310_14746_amd import tune
    kw = dict(tau=0.6, force=(1e-6, -2e-7, 0), store_scale=SCALE16)
    # each pattern at the block width bench.py times it with
    sims = [H.HLBM(19, storage, (n, n, n), pattern=p, block_x=tune.lookup(19, storage, (n, n, n), p),
                   row_pad=tune.lookup_row_pad(19, storage, (n, n, n), p), **kw)
            for p in ("ab", "aa")]
    try:
        for s in sims:
            s.set_porosity(d)
            s.set_state(state, 0)
        del state
        same_bx = sims[0].cfg.block_x == sims[1].cfg.block_x
        for k in (3, 1):
            tot = []
            for s in sims:
                s.step(k)
                tot.append(s.totals())
            # the FP64 totals sum per-block partials: bitwise only at one block width
            if same_bx:
                assert np.array_equal(tot[0], tot[1])
            else:
                assert np.allclose(tot[0], tot[1], rtol=1e-10, atol=1e-8)
            a = sims[0].get_state()[0]
            b = sims[1].get_state()[0]
            assert torch.equal(a, b)
            del a, b
    finally:
        for s in sims:
            s.close()
        del d
        torch.cuda.empty_cache()


def test_aa_api_rules(H):
    import torch
    with pytest.raises(H.HLBMError, match="open faces"):
        H.HLBM(19, "f32", (8, 8, 8), bc_lo=(2, 1, 1), bc_hi=(3, 1, 1), inlet_u=(0.01, 0, 0), pattern="aa")
    sim = H.HLBM(19, "f32", (8, 8, 8), pattern="aa")
    lib = H.load()
    try:
        assert sim._pop_b is None
        sim.set_porosity(np.zeros(512, dtype=np.float32))
        with pytest.raises(H.HLBMError, match="two-buffer"):
            sim.set_solid_mask(np.zeros(512, dtype=np.uint8))
        with pytest.raises(H.HLBMError, match="two-buffer"):
            sim.set_tape(2, 10)
        # the export must not write over the buffer it reads
        rc = lib.hlbm_get_state(sim.ctx, sim._pop_a.data_ptr(), 1, None)
        assert rc == H.EINVAL
        rc = lib.hlbm_set_state(sim.ctx, sim._pop_a.data_ptr(), 1, 0)
        assert rc == H.EINVAL
        other = torch.empty(sim.pop_bytes, dtype=torch.uint8, device="cuda")
        assert lib.hlbm_bind_buffers(sim.ctx, sim._pop_a.data_ptr(), other.data_ptr(),
                                     sim._dfield.data_ptr()) == H.EINVAL
        sim.step(2)
        assert sim.step_count == 2
    finally:
        sim.close()
