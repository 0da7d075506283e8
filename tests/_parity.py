"""Error measures shared by the parity tests.

Per field, over fluid cells:
  * velocity: relative L2 of the vector field, ||u_a - u_b||_2 / ||u_b||_2;
  * density: relative L2 of drho = rho - rho0 with the denominator floored at
    the dynamic-pressure scale ||rho0 |u_b|^2 / c_s^2||_2.  Where drho is
    resolved (any flow with a pressure field) the floor is inactive; where the
    exact drho is zero (a straight channel) both sides hold rounding noise and
    the error is measured against the smallest pressure the flow can carry.
"""
import numpy as np

CS2 = 1.0 / 3.0


def rel_l2_u(u_a, u_b, fluid=None):
    ua = np.asarray(u_a, dtype=np.float64).reshape(3, -1)
    ub = np.asarray(u_b, dtype=np.float64).reshape(3, -1)
    if fluid is not None:
        ua, ub = ua[:, fluid], ub[:, fluid]
    return float(np.linalg.norm(ua - ub) / np.linalg.norm(ub))


def rel_l2_drho(dr_a, dr_b, u_b, fluid=None, rho0=1.0):
    a = np.asarray(dr_a, dtype=np.float64).ravel()
    b = np.asarray(dr_b, dtype=np.float64).ravel()
    ub = np.asarray(u_b, dtype=np.float64).reshape(3, -1)
    if fluid is not None:
        a, b, ub = a[fluid], b[fluid], ub[:, fluid]
    floor = np.linalg.norm(rho0 * (ub ** 2).sum(axis=0) / CS2)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor))


def max_rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.abs(a - b).max() / np.abs(b).max())


def order_map(c_from, c_to):
    """perm such that c_to[perm[i]] == c_from[i]."""
    perm = []
    for ci in c_from:
        k = int(np.nonzero((c_to == ci).all(axis=1))[0][0])
        perm.append(k)
    return np.array(perm)


def quantization_floor(pre, c, scale, mantissa_bits, min_exp=None):
    """Relative-L2 floor that storing the pulled populations `pre[q, N]` in a
    binary float format with `mantissa_bits` explicit bits (scaled by `scale`)
    puts on one read of drho and of u: RMS of the sum of per-population
    round-to-nearest errors (variance ulp^2/12 each), over the field norm.
    Returns (floor_drho_abs_norm, floor_u_abs_norm) as L2 norms."""
    v = np.abs(np.asarray(pre, dtype=np.float64) * scale)
    e = np.floor(np.log2(np.maximum(v, 1e-300)))
    if min_exp is not None:
        e = np.maximum(e, min_exp)
    ulp = np.where(v > 0, 2.0 ** (e - mantissa_bits), 0.0) / scale
    var = ulp ** 2 / 12.0
    f_rho = np.sqrt(var.sum())
    f_u = np.sqrt(sum((c[:, a:a + 1] ** 2 * var).sum() for a in range(3)))
    return f_rho, f_u
