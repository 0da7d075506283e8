"""hlbm_moments_noalloc, the moments entry point that allocates nothing: its
partials live in a static device array of the library.  Called through the
C-ABI and compared with hlbm_moments on the same state: the same kernel and
the same fixed-order reduction, so fields and FP64 totals agree bit for bit.
Two calls in a row, the second on a smaller box (fewer blocks of partials than
the first left in the array), and both pattern forms."""
import ctypes

import numpy as np
import pytest

from paper_2310_14746_amd import inputs
from tests.test_gpu_parity import H, say  # noqa: F401

pytestmark = pytest.mark.gpu


def _state(H, shape, pattern, seed, block_x=0, q=19, storage="f32"):
    sim = H.HLBM(q, storage, shape, tau=0.7, force=(1e-5, -3e-6, 2e-6 if q == 19 else 0.0),
                 pattern=pattern, block_x=block_x)
    nx, ny, nz = sim.shape
    d = inputs.periodic_smooth(inputs.uniform_noise((nz, ny, nx), seed), 1.0, 3)
    sim.set_porosity(inputs.round_to(d, "f64" if storage == "f64" else "f32")
                     .astype(np.float64 if storage == "f64" else np.float32).ravel())
    sim.step(7)
    return sim


def _compare(H, sim, dtype):
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    nx, ny, nz = sim.shape
    dr_ref, u_ref, tot_ref = sim.moments(dtype, totals=True)
    # caller-owned outputs, filled with garbage first
    dr = torch.full((nz, ny, nx), 7.0, dtype=tdt, device=sim.device)
    u = torch.full((3, nz, ny, nx), -7.0, dtype=tdt, device=sim.device)
    tot = torch.full((4,), 123.0, dtype=torch.float64, device=sim.device)
    lib = H.load()
    rc = lib.hlbm_moments_noalloc(sim.ctx, ctypes.c_void_p(dr.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                  H.DT_F64 if dtype == "f64" else H.DT_F32, ctypes.c_void_p(tot.data_ptr()))
    assert rc == 0, lib.hlbm_last_error()
    sim.sync()
    assert torch.equal(dr, dr_ref) and torch.equal(u, u_ref)
    assert np.array_equal(tot.cpu().numpy(), tot_ref), (tot.cpu().numpy(), tot_ref)
    # totals only
    tot2 = torch.zeros(4, dtype=torch.float64, device=sim.device)
    sim.moments_noalloc(totals=tot2)
    sim.sync()
    assert np.array_equal(tot2.cpu().numpy(), tot_ref)


@pytest.mark.parametrize("pattern", ["ab", "aa"])
def test_noalloc_matches_moments_two_calls_second_smaller(H, pattern):
    big = _state(H, (200, 40, 30), pattern, seed=1)
    try:
        say(f"noalloc moments, {pattern}, 200x40x30 then 36x20x10")
        _compare(H, big, "f64")
    finally:
        big.close()
    small = _state(H, (36, 20, 10), pattern, seed=2)
    try:
        _compare(H, small, "f64")
        _compare(H, small, "f32")
    finally:
        small.close()


def test_noalloc_d2q9_f64_and_rejections(H):
    sim = _state(H, (130, 66), "ab", seed=3, q=9, storage="f64")
    try:
        say("noalloc moments, D2Q9 f64, and its error paths")
        _compare(H, sim, "f64")
        lib = H.load()
        assert lib.hlbm_moments_noalloc(sim.ctx, None, None, 7, None) == H.EINVAL
    finally:
        sim.close()
    # a batch is not taken
    b = H.HLBMBatch([dict(shape=(16, 16, 16), tau=0.7, force=(1e-6, 0, 0))], "f32")
    try:
        assert H.load().hlbm_moments_noalloc(b.ctx, None, None, H.DT_F64, None) == H.EUNSUPPORTED
    finally:
        b.close()
    # more blocks than the static array holds: rejected before anything runs
    # (the context's memory is never bound: nothing of that size is allocated)
    lib = H.load()
    cfg = H.make_config(19, "f32", (1024, 1024, 600), block_x=64, external_memory=1)
    ctx = ctypes.c_void_p()
    assert lib.hlbm_create(ctypes.byref(cfg), ctypes.byref(ctx)) == 0, lib.hlbm_last_error()
    try:
        import torch
        tot = torch.zeros(4, dtype=torch.float64, device="cuda")
        rc = lib.hlbm_moments_noalloc(ctx, None, None, H.DT_F64, ctypes.c_void_p(tot.data_ptr()))
        assert rc == H.EINVAL and b"static scratch" in lib.hlbm_last_error()
        # without totals there is nothing to hold: only the unbound buffers stop it
        assert lib.hlbm_moments_noalloc(ctx, None, None, H.DT_F64, None) == H.ESTATE
    finally:
        assert lib.hlbm_destroy(ctx) == 0
