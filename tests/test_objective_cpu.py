"""The torch channel objective used with autograd agrees with the oracle's numpy
objective (value and gradient); the oracle's gradient is itself pinned to
finite differences in tests/test_oracle_adjoint.py.  CPU only."""
import numpy as np
import torch

from oracle import objective as oobj
from paper_2310_14746_amd.autograd import channel_objective


def _fields(shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    drho = 1e-3 * rng.standard_normal(shape)
    u = 1e-2 * rng.standard_normal((3,) + shape)
    d = rng.random(shape)
    return drho, u, d


def test_value_and_gradient_match_oracle():
    for shape, tau in (((7, 9, 12), 0.6), ((10, 8, 6), 0.9)):
        drho, u, d = _fields(shape, seed=shape[2])
        J_o = oobj.objective(drho, u, d, tau)
        gr, gu, gd = oobj.objective_grad(drho, u, d, tau)
        t = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in (drho, u, d)]
        J = channel_objective(t[0], t[1], t[2], tau)
        J.backward()
        assert abs(float(J.detach()) - J_o) <= 1e-13 * abs(J_o)
        for got, want in zip((t[0].grad, t[1].grad, t[2].grad), (gr, gu, gd)):
            np.testing.assert_allclose(got.numpy(), want, rtol=1e-12, atol=1e-15 * np.abs(want).max())
