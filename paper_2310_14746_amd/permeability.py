"""Unit-cell permeability workloads on the batched sweep.

The paper's Darcy law takes its permeability from the periodic unit-cell
problem (Sec. 2.2), and its nonstationary regimes from the time-dependent cell
problem, whose transient permeability Ã(t) integrates to the stationary one,
A = ∫ Ã dt (Sec. 2.3).  For a homogenized unit cell driven from rest by a body
force F, the cell-averaged velocity obeys <u>(t) = (F/nu) ∫_0^t Ã dt', so

    k(t) = nu <rho u_x>(t) / F

is the running integral of the transient permeability and tends to the
stationary permeability; Ã(t) is its time derivative.  `transient_permeability`
records k(t) for every item of a batch (one persistent launch per interval);
`sharp_fields` gives the same cells with the unsmoothed indicator as control
(d = 1 inside the sphere, 0 outside), to measure the effect of the smoothing
that the homogenized fields apply.

The permeability is a tensor (Sec. 2.2, the unit-cell tensor; Sec. 2.3, its
transient form Ã_ij and A_ij = ∫ Ã_ij dt): the force along axis j drives the
mean velocity along every axis i, k_ij(t) = nu <rho u_i>(t) / F_j.
`transient_permeability_tensor` forces every cell along x, y and z (three
items per cell, one batch) and records all nine components.  `resolved_cells`
gives the same cells with the sphere resolved instead of homogenized: a solid
mask with bounce-back links and no control in the fluid (d = 0), the geometry
of the unit-cell Stokes problem itself.

Host-side set-up and bookkeeping only; every step runs in the HIP kernels.
"""
from __future__ import annotations

import numpy as np

from . import inputs


def unit_cells(n_items: int, seed: int = 0, force: float = 1e-6, sharp: bool = False):
    """Items and FP32 control fields of the homogenized-sphere unit cells
    (edges, porosities and tau drawn as in inputs.batch_items)."""
    spec = inputs.batch_items(n_items, seed=seed)
    items = [dict(shape=(e, e, e), tau=t, force=(force, 0.0, 0.0)) for e, _, t in spec]
    fields = []
    for e, phi, _ in spec:
        if sharp:
            d = inputs.sphere_indicator(e, inputs.radius_for_porosity(e, phi))
        else:
            d = inputs.batch_item_field(e, phi)
        fields.append(inputs.round_to(d, "f32").astype(np.float32).ravel())
    return items, fields, spec


def transient_permeability(hlbm, items, fields, times, storage: str = "f32", mode: str = "graph"):
    """k(t) = nu <rho u_x>(t) / F at the given (increasing) step counts, for
    every item: array (len(times), n_items)."""
    b = hlbm.HLBMBatch(items, storage, mode=mode)
    try:
        for k, d in enumerate(fields):
            b.set_porosity(k, d)
        cells = np.array([np.prod(it["shape"]) for it in items], dtype=np.float64)
        nu = (np.array([it["tau"] for it in items]) - 0.5) / 3.0
        F = np.array([it["force"][0] for it in items])
        out = []
        done = 0
        for t in times:
            if t < done:
                raise ValueError("times must be increasing")
            b.step(int(t - done))
            done = int(t)
            tot = b.totals()
            out.append(nu * (tot[:, 1] / cells) / F)
        return np.array(out)
    finally:
        b.close()


def transient_rate(times, k) -> np.ndarray:
    """Ã at the interval midpoints: finite differences of k(t) in steps."""
    t = np.asarray(times, dtype=np.float64)
    return np.diff(k, axis=0) / np.diff(t)[:, None]


def transient_permeability_tensor(hlbm, items, fields, times, storage: str = "f32", masks=None,
                                  mode: str = "per_step", force: float = 1e-6):
    """k_ij(t) = nu <rho u_i>(t) / F_j for every item, forced along each axis j
    in turn (three copies of every item in one batch, force `force` along j):
    array (len(times), n_items, 3, 3), [t, item, i, j].  `masks`: optional
    solid masks per item (None entries: no obstacles)."""
    n = len(items)
    tri = []
    for j in range(3):
        for it in items:
            F = [0.0, 0.0, 0.0]
            F[j] = force
            tri.append(dict(shape=it["shape"], tau=it["tau"], force=tuple(F)))
    b = hlbm.HLBMBatch(tri, storage, mode=mode)
    try:
        for j in range(3):
            for k, d in enumerate(fields):
                b.set_porosity(j * n + k, d)
                if masks is not None and masks[k] is not None:
                    b.set_solid_mask(j * n + k, masks[k])
        cells = np.array([np.prod(it["shape"]) for it in items], dtype=np.float64)
        nu = (np.array([it["tau"] for it in items]) - 0.5) / 3.0
        out = []
        done = 0
        for t in times:
            if t < done:
                raise ValueError("times must be increasing")
            b.step(int(t - done))
            done = int(t)
            tot = b.totals().reshape(3, n, 4)          # [j, item, (drho, rho u_x, rho u_y, rho u_z)]
            k = np.empty((n, 3, 3))
            for j in range(3):
                for i in range(3):
                    k[:, i, j] = nu * (tot[j, :, 1 + i] / cells) / force
            out.append(k)
        return np.array(out)
    finally:
        b.close()


def resolved_cells(n_items: int, seed: int = 0, force: float = 1e-6):
    """The homogenized-sphere unit cells with the sphere resolved: items,
    zero control fields and solid masks (the sphere indicator of the radius
    that gives the cell's target porosity)."""
    spec = inputs.batch_items(n_items, seed=seed)
    items = [dict(shape=(e, e, e), tau=t, force=(force, 0.0, 0.0)) for e, _, t in spec]
    fields = [np.zeros(e ** 3, dtype=np.float32) for e, _, _ in spec]
    masks = [(inputs.sphere_indicator(e, inputs.radius_for_porosity(e, phi)) > 0.5).astype(np.uint8).ravel()
             for e, phi, _ in spec]
    return items, fields, masks, spec
