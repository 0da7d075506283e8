"""Refinement along the paper's diffusive scaling (Sec. 3.3 Step 2): the lattice
spacing eps = 1/N, time step eps^2, and the porosity control d = nu tau eps^2/K
(1 - varpi = O(eps^2)), against exact solutions of the target Brinkman
equations (eq:targetEBTL), on the GPU in FP64: velocity (Brinkman channel),
the decay rate of a shear wave, and pressure (Darcy flow through a medium
whose permeability varies along the flow).  The coarsest run of each study
is also compared with the oracle element by element."""
import os

import numpy as np
import pytest

import oracle
from oracle import OracleConfig
from paper_2310_14746_amd import scaling
from tests.test_gpu_parity import H, say  # noqa: F401

pytestmark = pytest.mark.gpu

NT = max(1, min(16, os.cpu_count() or 1))
NS = (16, 32, 64, 128, 256)


def test_brinkman_channel_refinement(H):
    errs = []
    for N in NS:
        y, u, ex, steps = scaling.brinkman_channel(H, N)
        errs.append(float(np.linalg.norm(u - ex) / np.linalg.norm(ex)))
        say(f"Brinkman channel N={N}: {steps} steps, rel-L2 error {errs[-1]:.3e}")
    orders = scaling.observed_order(errs, NS)
    say("observed orders " + ", ".join(f"{o:.2f}" for o in orders))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert min(orders[-2:]) >= 1.8
    # the coarsest run against the oracle
    N = NS[0]
    p = scaling.lattice_parameters(N, 0.1, 0.01, 1.0)
    y, u, _, steps = scaling.brinkman_channel(H, N)
    cfg = OracleConfig(q=9, nx=4, ny=N + 2, nz=1, tau=p["tau"], force=(p["force"], 0, 0),
                       bc_lo=(0, 1, 0), bc_hi=(0, 1, 0))
    g = oracle.run(cfg, np.full(4 * (N + 2), p["d"]), steps, nthreads=NT)
    _, uo = oracle.observe(cfg, g)
    uo = uo[0].reshape(N + 2, 4)[1:N + 1, 0] * p["u_scale"]
    assert np.linalg.norm(u - uo) <= 1e-10 * np.linalg.norm(uo)


def test_shear_wave_rate_refinement(H):
    errs = []
    for N in NS:
        rate, exact, steps = scaling.shear_wave_decay(H, N)
        errs.append(abs(rate - exact) / exact)
        say(f"shear wave N={N}: {steps} steps, rate {rate:.6f} vs {exact:.6f}, rel error {errs[-1]:.3e}")
    orders = scaling.observed_order(errs, NS)
    say("observed orders " + ", ".join(f"{o:.2f}" for o in orders))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert min(orders[-2:]) >= 1.8


def test_darcy_pressure_refinement(H):
    """Pressure along the diffusive scaling: Darcy flow through a medium whose
    permeability varies along the flow, against p(x) = -(g a / 2 pi) sin(2 pi x)
    and U = g K0 / nu; the coarsest run also against the oracle."""
    errs, uerrs = [], []
    for N in NS:
        x, p, pe, U, Ue, steps = scaling.darcy_pressure(H, N)
        errs.append(float(np.linalg.norm(p - pe) / np.linalg.norm(pe)))
        uerrs.append(abs(U - Ue) / Ue)
        say(f"Darcy pressure N={N}: {steps} steps, rel-L2 error of p {errs[-1]:.3e}, of U {uerrs[-1]:.3e}")
    orders = scaling.observed_order(errs, NS)
    say("observed orders (p) " + ", ".join(f"{o:.2f}" for o in orders))
    say("observed orders (U) " + ", ".join(f"{o:.2f}" for o in scaling.observed_order(uerrs, NS)))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert min(orders[-2:]) >= 1.8
    # the coarsest run against the oracle
    N = NS[0]
    x, p, _, _, _, steps = scaling.darcy_pressure(H, N)
    nu, K0, a, g = 0.1, 0.01, 0.5, 1.0
    eps, tau = 1.0 / N, 3.0 * nu + 0.5
    d = nu * tau * eps * eps * (1.0 + a * np.cos(2.0 * np.pi * x)) / K0
    cfg = OracleConfig(q=9, nx=N, ny=4, nz=1, tau=tau, force=(g * eps ** 3, 0, 0))
    go = oracle.run(cfg, np.broadcast_to(d[None, :], (4, N)).ravel(), steps, nthreads=NT)
    dro, _ = oracle.observe(cfg, go)
    po = dro.reshape(4, N)[0] / (3.0 * eps * eps)
    assert np.linalg.norm(p - po) <= 1e-10 * np.linalg.norm(po)
