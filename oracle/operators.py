"""Discrete Laplacians and residuals (Eqs. 1 and 2, Section 2.1).

Cartesian arrays hold every node of the vertex-centred grid including the
``g`` ghost layers ([k][j][i], x fastest); operators return values on the
unknown nodes only, shape (n-1)^3.

* 7-point, 2nd order:  (sum of the 6 neighbours - 6 u) / h^2.
* 19-point star, 6th order (radius 3, the "CG6" operator of Section 2.1.2):
  per axis the central second difference with weights
  [1/90, -3/20, 3/2, -49/18, 3/2, -3/20, 1/90] / h^2.

Log-spherical grid (Eq. 2 with s = ln r), multiplied through by r^2:
  r^2 lap u = u_ss + u_s + u_thth + cot(th) u_th + u_phph / sin^2(th),
each derivative a 2nd-order central difference; u has shape
[nph][nth][nr+2] (radial ghosts at both ends), the colatitude neighbour past a
pole is the node on the far side of the pole (phi + pi), phi is periodic.
"""
from __future__ import annotations

import math

import numpy as np

STAR6 = (-49.0 / 18.0, 1.5, -3.0 / 20.0, 1.0 / 90.0)


def _shift(u, g, n, dk, dj, di):
    e = n - 1
    return u[g + dk:g + dk + e, g + dj:g + dj + e, g + di:g + di + e]


def lap7(u: np.ndarray, n: int, h: float, g: int = 1) -> np.ndarray:
    c = _shift(u, g, n, 0, 0, 0)
    s = (_shift(u, g, n, 0, 0, 1) + _shift(u, g, n, 0, 0, -1)
         + _shift(u, g, n, 0, 1, 0) + _shift(u, g, n, 0, -1, 0)
         + _shift(u, g, n, 1, 0, 0) + _shift(u, g, n, -1, 0, 0))
    return (s - 6.0 * c) / (h * h)


def lap19(u: np.ndarray, n: int, h: float, g: int = 3) -> np.ndarray:
    assert g >= 3
    out = 3.0 * STAR6[0] * _shift(u, g, n, 0, 0, 0)
    for d in (1, 2, 3):
        out = out + STAR6[d] * (_shift(u, g, n, 0, 0, d) + _shift(u, g, n, 0, 0, -d)
                                + _shift(u, g, n, 0, d, 0) + _shift(u, g, n, 0, -d, 0)
                                + _shift(u, g, n, d, 0, 0) + _shift(u, g, n, -d, 0, 0))
    return out / (h * h)


def lap(u, n, h, order, g):
    return lap7(u, n, h, g) if order == 2 else lap19(u, n, h, g)


def residual(u, f_nodes, n, h, order, g):
    """r = f - L_h u on the unknown nodes (f = 4 pi G rho), Section 2.1."""
    s = slice(g, g + n - 1)
    return f_nodes[s, s, s] - lap(u, n, h, order, g)


def rhs_norm(u, f_nodes, n, h, order, g):
    """||r(u with its unknowns set to 0)||_2: the normaliser of the relative
    residual ||r_m|| / ||r_0|| for a cold start (Eq. rho)."""
    s = slice(g, g + n - 1)
    z = u.copy()
    z[s, s, s] = 0.0
    return float(np.linalg.norm(residual(z, f_nodes, n, h, order, g)))


# --------------------------------------------------------------------------
# log-spherical
# --------------------------------------------------------------------------
def sph_apply(u: np.ndarray, ds, th: np.ndarray) -> np.ndarray:
    """r^2-scaled Laplacian on the unknowns; u is [nph][nth][nr+2].  ds: the
    log-grid spacing, or a radial.RadialMap (radial couplings cl, cr)."""
    nph, nth, m = u.shape
    nr = m - 2
    dth = math.pi / nth
    dph = 2 * math.pi / nph
    c = u[:, :, 1:nr + 1]
    up = u[:, :, 2:nr + 2]
    um = u[:, :, 0:nr]
    if isinstance(ds, (int, float)):
        out = (up - 2 * c + um) / ds ** 2 + (up - um) / (2 * ds)
    else:
        out = ds.cr[None, None, :] * up + ds.cl[None, None, :] * um - (ds.cl + ds.cr)[None, None, :] * c
    # colatitude neighbours, reflected across the poles with phi + pi
    half = nph // 2
    flip = np.roll(c, -half, axis=0)           # value at phi + pi
    jp = np.concatenate([c[:, 1:, :], flip[:, -1:, :]], axis=1)
    jm = np.concatenate([flip[:, :1, :], c[:, :-1, :]], axis=1)
    cot = (np.cos(th) / np.sin(th))[None, :, None]
    out = out + (jp - 2 * c + jm) / dth ** 2 + cot * (jp - jm) / (2 * dth)
    kp = np.roll(c, -1, axis=0)
    km = np.roll(c, 1, axis=0)
    out = out + (kp - 2 * c + km) / (dph ** 2 * np.sin(th)[None, :, None] ** 2)
    return out


def sph_rhs(rho_nodes, r, four_pi_G=1.0):
    """b = r^2 4 pi G rho on the unknowns (r holds radii of nodes -1..nr)."""
    nr = rho_nodes.shape[2] - 2
    return four_pi_G * rho_nodes[:, :, 1:nr + 1] * (r[1:nr + 1] ** 2)[None, None, :]


def sph_residual(u, rho_nodes, r, ds, th, four_pi_G=1.0):
    """b - A u; ds as in sph_apply."""
    return sph_rhs(rho_nodes, r, four_pi_G) - sph_apply(u, ds, th)
