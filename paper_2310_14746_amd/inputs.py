"""Seeded synthetic inputs for the HLBM sweep (porosity-control fields).

This module holds no arithmetic of the method itself: it only builds the
per-cell field d = 1 - varpi in [0, 1] that both the HIP path and the oracle
receive.  It imports nothing else from this package, so tests can feed the same
arrays to both sides.

Geometry follows the paper's periodic obstacle array (Sec. 2.1: a periodic
array of cells of edge eps, each holding a centred sphere), homogenized by a
periodic Gaussian smoothing of the solid indicator.  Porosity phi is the void
fraction 1 - |solid|/|cell| (Sec. 2.4, eq:porosityCalc).

All fields are float64 arrays of shape (nz, ny, nx), x fastest, matching the
cell index x + nx*(y + ny*z).
"""
from __future__ import annotations

import numpy as np

SPHERE_CELL = 32          # edge of one obstacle cell in the regular arrays
SPHERE_RADIUS = 10.0      # obstacle radius in the regular arrays
SMOOTH_SIGMA = 2.0        # Gaussian smoothing width (cells)
SMOOTH_HALF = 8           # kernel support |k| <= 4 sigma


def gaussian_kernel(sigma: float = SMOOTH_SIGMA, half: int = SMOOTH_HALF) -> np.ndarray:
    """Normalized 1-D weights exp(-k^2/(2 sigma^2)) for |k| <= half."""
    k = np.arange(-half, half + 1, dtype=np.float64)
    w = np.exp(-k * k / (2.0 * sigma * sigma))
    return w / w.sum()


def periodic_smooth(field: np.ndarray, sigma: float = SMOOTH_SIGMA,
                    half: int = SMOOTH_HALF) -> np.ndarray:
    """Separable periodic Gaussian smoothing along every axis of a 3-D array.

    The weights are non-negative and sum to one, so values stay in [0, 1] and
    the mean is unchanged (up to rounding).
    """
    w = gaussian_kernel(sigma, half)
    out = np.asarray(field, dtype=np.float64)
    for ax in range(out.ndim):
        acc = np.zeros_like(out)
        for k, wk in zip(range(-half, half + 1), w):
            acc += wk * np.roll(out, k, axis=ax)
        out = acc
    return out


def sphere_indicator(edge: int, radius: float) -> np.ndarray:
    """Solid indicator of one periodic cell of edge ``edge`` with a centred sphere.

    Nodes sit at integer coordinates; the centre is at (edge-1)/2 in each axis
    and distances use the periodic minimum image, so overlapping images (radius
    above edge/2) are handled.
    """
    c = (edge - 1) / 2.0
    ax = np.arange(edge, dtype=np.float64) - c
    ax = ax - edge * np.round(ax / edge)
    r2 = ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2
    return (r2 <= radius * radius).astype(np.float64)


def sphere_distances2(edge: int) -> np.ndarray:
    c = (edge - 1) / 2.0
    ax = np.arange(edge, dtype=np.float64) - c
    ax = ax - edge * np.round(ax / edge)
    return ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2


def radius_for_porosity(edge: int, phi: float) -> float:
    """Radius whose indicator void fraction is nearest to ``phi``.

    The solid node count is a step function of the radius; the candidate radii
    are the distinct node distances, and the one whose count is nearest to
    (1 - phi)*edge^3 is returned (the smaller one on a tie).
    """
    r2 = np.sort(sphere_distances2(edge).ravel())
    target = (1.0 - phi) * edge ** 3
    vals, counts = np.unique(r2, return_counts=True)
    cum = np.cumsum(counts)
    best = int(np.argmin(np.abs(cum - target)))
    return float(np.sqrt(vals[best]))


def sphere_array_tile(edge: int = SPHERE_CELL, radius: float = SPHERE_RADIUS,
                      sigma: float = SMOOTH_SIGMA) -> np.ndarray:
    """Homogenized d on one periodic cell: smoothed sphere indicator."""
    return periodic_smooth(sphere_indicator(edge, radius), sigma)


def sphere_array(n: int, edge: int = SPHERE_CELL, radius: float = SPHERE_RADIUS,
                 sigma: float = SMOOTH_SIGMA, seed: int = 0) -> np.ndarray:
    """d on an n^3 periodic box tiled by (n/edge)^3 equal spheres.

    The array is regular (no jitter), so ``seed`` does not change the field; it
    is accepted so every workload records one.  Periodic smoothing commutes
    with periodic tiling, so the tile is smoothed once and repeated; the values
    are identical to smoothing the whole box.
    """
    del seed
    if n % edge:
        raise ValueError("box edge must be a multiple of the obstacle cell edge")
    tile = sphere_array_tile(edge, radius, sigma)
    reps = n // edge
    return np.tile(tile, (reps, reps, reps))


def channel_2d(nx: int = 128, ny: int = 64, d_core: float = 0.5,
               rows=(16, 47)) -> np.ndarray:
    """Planar channel porosity: d = d_core on rows rows[0]..rows[1], else 0.

    Shape (1, ny, nx).
    """
    d = np.zeros((1, ny, nx), dtype=np.float64)
    d[0, rows[0]:rows[1] + 1, :] = d_core
    return d


def uniform_noise(shape, seed: int = 0) -> np.ndarray:
    """d ~ U[0, 1) i.i.d. per cell from numpy's default generator."""
    rng = np.random.default_rng(seed)
    return rng.random(shape)


def batch_items(n_items: int = 256, seed: int = 0, edges=(32, 48, 64, 80, 96),
                phi_range=(0.1, 0.9), tau_range=(0.55, 1.0)):
    """Draw per-item (edge, phi, tau) in that order from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    items = []
    for _ in range(n_items):
        e = int(rng.choice(np.asarray(edges)))
        phi = float(rng.uniform(*phi_range))
        tau = float(rng.uniform(*tau_range))
        items.append((e, phi, tau))
    return items


def batch_item_field(edge: int, phi: float, sigma: float = SMOOTH_SIGMA) -> np.ndarray:
    """Homogenized d of one periodic unit cell with target porosity phi."""
    r = radius_for_porosity(edge, phi)
    return periodic_smooth(sphere_indicator(edge, r), sigma)


def round_to(d: np.ndarray, dtype: str) -> np.ndarray:
    """Round a float64 field to the storage precision ('f64', 'f32', 'f16')."""
    if dtype == "f64":
        return np.asarray(d, dtype=np.float64)
    if dtype == "f32":
        return np.asarray(d, dtype=np.float32).astype(np.float64)
    if dtype == "f16":
        return np.asarray(d, dtype=np.float16).astype(np.float64)
    raise ValueError(dtype)


# ---------------------------------------------------------------------------
# Tensor (anisotropic) porosity controls D = nu tau K^{-1}, symmetric 3x3 per
# cell with eigenvalues in [0, 1], returned as 6 rows (xx, yy, zz, xy, xz, yz).
# ---------------------------------------------------------------------------
TENSOR_ROWS = ("xx", "yy", "zz", "xy", "xz", "yz")


def tensor_rows(M: np.ndarray) -> np.ndarray:
    """(..., 3, 3) symmetric matrices -> (6, ...) rows xx, yy, zz, xy, xz, yz."""
    return np.stack([M[..., 0, 0], M[..., 1, 1], M[..., 2, 2], M[..., 0, 1], M[..., 0, 2],
                     M[..., 1, 2]])


def random_tensor_field(shape_zyx, seed: int = 0, sigma: float = 1.0, half: int = 3) -> np.ndarray:
    """D = G G^T / (1 + |G|_F^2) with G a 3x3 of smoothed noise in [-1, 1]
    per cell: symmetric positive semidefinite, eigenvalues in [0, 1)."""
    rng = np.random.default_rng(seed)
    G = np.empty(tuple(shape_zyx) + (3, 3))
    for a in range(3):
        for b in range(3):
            G[..., a, b] = 2.0 * periodic_smooth(rng.random(shape_zyx), sigma, half) - 1.0
    M = G @ np.swapaxes(G, -1, -2)
    M /= (1.0 + (G * G).sum(axis=(-1, -2)))[..., None, None]
    return tensor_rows(M).reshape(6, -1)


def fiber_tensor_field(d: np.ndarray, axis=(2.0, 1.0, 1.0), aniso: float = 0.2) -> np.ndarray:
    """D = d [aniso I + (1 - aniso) n n^T] for a scalar field d in [0, 1] and a
    fixed unit fibre direction n: full drag d along n, aniso*d across it."""
    n = np.asarray(axis, dtype=np.float64)
    n = n / np.linalg.norm(n)
    T = aniso * np.eye(3) + (1.0 - aniso) * np.outer(n, n)
    d = np.asarray(d, dtype=np.float64).ravel()
    return tensor_rows(T)[:, None] * d[None, :]
