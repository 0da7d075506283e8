"""Pins of the seeded input generators (CPU only).

G1: periodic Gaussian smoothing keeps the mean and the range [0, 1].
G2: sphere of diameter equal to the cell edge gives the paper's minimum porosity
    1 - pi/6 ~= 0.4764 (Sec. 2.4, eq:porosityCalc, case (iv), C = 1) up to the
    node-count discretization.
G3: the 32^3 / r = 10 obstacle cell's solid fraction is close to (4/3) pi r^3 / 32^3.
"""
import json
import os

import numpy as np
import pytest

from paper_2310_14746_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_smoothing_preserves_mean_and_range():
    rng = np.random.default_rng(3)
    f = (rng.random((20, 24, 28)) < 0.3).astype(float)
    s = inputs.periodic_smooth(f)
    assert np.isclose(s.mean(), f.mean(), rtol=0, atol=1e-15)
    assert s.min() >= 0.0 and s.max() <= 1.0
    w = inputs.gaussian_kernel()
    assert len(w) == 17 and np.isclose(w.sum(), 1.0) and np.allclose(w, w[::-1])


def test_minimum_porosity_matches_paper():
    ref = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))["min_porosity"]
    assert abs((1.0 - np.pi / 6.0) - ref["value"]) < 0.5 * 10 ** -ref["digits"]
    errs = []
    for E in (32, 64, 96):
        phi = 1.0 - inputs.sphere_indicator(E, E / 2.0).mean()
        errs.append(abs(phi - (1.0 - np.pi / 6.0)))
    assert errs[-1] < 5e-4
    assert abs(1.0 - inputs.sphere_indicator(96, 48.0).mean() - ref["value"]) < 5e-4


def test_regular_array_solid_fraction():
    ind = inputs.sphere_indicator(32, 10.0)
    assert abs(ind.mean() / (4.0 / 3.0 * np.pi * 1000 / 32 ** 3) - 1.0) < 0.01
    d = inputs.sphere_array(64)
    assert d.shape == (64, 64, 64)
    assert np.isclose(d.mean(), ind.mean(), atol=1e-14)
    # periodic tiling == smoothing the whole box
    full = inputs.periodic_smooth(np.tile(ind, (2, 2, 2)))
    assert np.array_equal(full, d)
    # mirror symmetry about the obstacle-cell mid-planes
    t = d[:32, :32, :32]
    for m in (t[::-1], t[:, ::-1], t[:, :, ::-1]):
        assert np.abs(t - m).max() < 1e-15


def test_batch_items_and_radius():
    items = inputs.batch_items(256, seed=0)
    assert len(items) == 256
    assert {e for e, _, _ in items} <= {32, 48, 64, 80, 96}
    assert all(0.1 <= p <= 0.9 and 0.55 <= t <= 1.0 for _, p, t in items)
    assert items == inputs.batch_items(256, seed=0)
    for E, phi in [(32, 0.1), (48, 0.5), (64, 0.9)]:
        r = inputs.radius_for_porosity(E, phi)
        got = 1.0 - inputs.sphere_indicator(E, r).mean()
        assert abs(got - phi) < 3.0 / E  # one shell of nodes
        f = inputs.batch_item_field(E, phi)
        assert np.isclose(f.mean(), 1.0 - got, atol=1e-14)


def test_channel_and_noise():
    d = inputs.channel_2d()
    assert d.shape == (1, 64, 128)
    assert (d[0, 16:48] == 0.5).all() and (d[0, :16] == 0).all() and (d[0, 48:] == 0).all()
    n1 = inputs.uniform_noise((4, 5, 6), seed=5)
    assert np.array_equal(n1, inputs.uniform_noise((4, 5, 6), seed=5))
    assert n1.min() >= 0 and n1.max() < 1


@pytest.mark.parametrize("dt", ["f64", "f32", "f16"])
def test_round_to(dt):
    x = inputs.sphere_array_tile()
    r = inputs.round_to(x, dt)
    assert r.dtype == np.float64
    assert np.abs(r - x).max() <= {"f64": 0, "f32": 6e-8, "f16": 5e-4}[dt]
