"""Boxes at the size limits of the library (FP32 population rows just under
4 GiB), checked by a property that holds at any size: with a uniform control
d the scheme keeps rho = rho0 and every cell follows the uniform-Darcy
transient u_n = F tau/d - (F tau/d - F/2)(1 - d/tau)^n exactly (in FP64; FP32
storage within 1e-5).  The FP64 moment fields of these boxes are larger than
4 GiB, so any 32-bit wrap of an index would leave cells unwritten or
overwritten, which the field-wide min/max comparisons catch.

* in place (AA), 1024 x 1024 x 1023 = 1,072,693,248 cells: the largest FP32
  box (19 x 4 x N bytes = 81.5 GB in one buffer), 9 steps;
* two buffers, 1024 x 1024 x 520 = 545,259,520 cells (> 2^29), 7 steps;
* the adjoint of one step on 1024 x 1024 x 513 cells (FP64 gradient rows
  above 4 GiB) against its closed form.
"""
import pytest

from tests.test_gpu_parity import H, say  # noqa: F401

pytestmark = pytest.mark.gpu

TAU, D = 0.6, 0.3
F = (1e-6, 2e-7, 0.0)


def _exact(n, d):
    return [Fa * TAU / d - (Fa * TAU / d - 0.5 * Fa) * (1.0 - d / TAU) ** n for Fa in F]


@pytest.mark.parametrize("shape,pattern,steps", [((1024, 1024, 1023), "aa", 9),
                                                 ((1024, 1024, 520), "ab", 7)])
def test_uniform_darcy_at_maximum_size(H, shape, pattern, steps):
    import torch
    nx, ny, nz = shape
    n = nx * ny * nz
    assert n * 4 < 2 ** 32 and (n > 2 ** 29)
    say(f"maximum size {shape} ({n} cells), {pattern}, {steps} steps")
    torch.cuda.empty_cache()   # memory cached by earlier tests
    sim = H.HLBM(19, "f32", shape, tau=TAU, force=F, pattern=pattern)
    try:
        d = torch.full((n,), D, dtype=torch.float32, device="cuda")
        d32 = float(d[0].item())
        sim.set_porosity(d)
        del d
        sim.step(steps)
        drho, u, tot = sim.moments("f64", totals=True)
        assert drho.numel() * 8 > 2 ** 32
        ex = _exact(steps, d32)
        say(f"drho in [{float(drho.min()):.3e}, {float(drho.max()):.3e}]; exact u {ex}")
        assert float(drho.abs().max()) <= 1e-9
        for a in range(3):
            lo, hi = float(u[a].min()), float(u[a].max())
            say(f"u[{a}] in [{lo:.9e}, {hi:.9e}]")
            scale = max(abs(ex[0]), 1e-30)
            assert abs(lo - ex[a]) <= 1e-5 * scale and abs(hi - ex[a]) <= 1e-5 * scale
        # the FP64 totals: sum rho u_x over all cells
        assert abs(tot[1] - n * ex[0]) <= 1e-5 * n * abs(ex[0])
        del drho, u
    finally:
        sim.close()
        torch.cuda.empty_cache()


def test_adjoint_gradient_rows_above_4gib(H):
    """The reverse sweep over a box of more than 2^29 cells (FP64 cotangent and
    gradient rows larger than 4 GiB), 16-bit storage so that the tape fits:
    one step from rest with a uniform control gives u_1 = 3F/2 - F d/(2 tau)
    in every cell, so for J = sum over cells of u_x every cell's dJ/dd equals
    -F_x/(2 tau) (translation invariance: the per-cell derivatives sum to
    dJ/dd of the uniform control)."""
    import torch
    shape = (1024, 1024, 513)
    nx, ny, nz = shape
    n = nx * ny * nz
    assert n * 8 > 2 ** 32
    say(f"adjoint at {shape} ({n} cells), f16s, one step")
    torch.cuda.empty_cache()   # memory cached by earlier tests
    sim = H.HLBM(19, "f16s", shape, tau=TAU, force=F, store_scale=2.0 ** 14)
    try:
        sim.set_porosity(torch.full((n,), D, dtype=torch.float16, device="cuda"))
        sim.set_tape(1, 1)
        sim.step(1)
        gr = torch.zeros(n, dtype=torch.float64, device="cuda")
        gu = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
        gu[:n] = 1.0
        g = sim.adjoint(1, gr, gu)
        del gr, gu
        ex = -F[0] / (2 * TAU)
        lo, hi = float(g.min()), float(g.max())
        say(f"dJ/dd in [{lo:.9e}, {hi:.9e}], exact {ex:.9e}")
        assert abs(lo - ex) <= 1e-6 * abs(ex) and abs(hi - ex) <= 1e-6 * abs(ex)
        del g
    finally:
        sim.close()
        torch.cuda.empty_cache()
