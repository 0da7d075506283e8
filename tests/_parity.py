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
