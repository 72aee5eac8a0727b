"""Successive overrelaxation on the log-spherical grid with a position-
dependent Chebyshev sequence of relaxation factors (Section 2.1.1:
Eqs. omega_final, omega_n and local_rjac).

Test infrastructure: imported by tests and the benchmark's CPU baseline only.

Colouring.  With the colatitude neighbour across a pole taken at phi + pi,
the parity colouring of (i + j + k) alone can put a node and its cross-pole
neighbour in the same colour (when nphi / 2 is even).  The colour used here is
(i + j + k) mod 2 plus 2 if phi lies in the second half turn (k >= nphi / 2):
no two neighbours, across a pole included, share a colour, so a colour pass
is order independent.  Colours 0 and 2 form the "red" half-sweep, 1 and 3 the
"black" one.

Local spectral radius.  Eq. local_rjac weighs cos(pi / N_d) with the inverse
squared metric spacings (dr)^-2, (r dtheta)^-2, (r sin(theta) dphi)^-2.  The
operator here is r^2 lap in s = ln r, whose diagonal couplings are
ds^-2, dtheta^-2 and (sin(theta) dphi)^-2: the same weights multiplied by
r^2 (with dr = r ds), so r cancels and r_J depends on theta only.

Relaxation sequence (Eq. omega_n started from n = 1): omega_1 = 1/(1 - rJ^2/2),
omega_{n+1} = 1/(1 - rJ^2 omega_n / 4), one term per half-sweep, per node.
"""
from __future__ import annotations

import math

import numpy as np

from . import operators as O


def local_rjac(nr: int, nth: int, nph: int, ds, th: np.ndarray) -> np.ndarray:
    """r_J, Eq. local_rjac: at every colatitude (shape nth) on the log grid
    (ds a float); on a mapped radial grid (ds a radial.RadialMap) the radial
    weight r^2 / R'^2 = (cl + cr) / 2 varies with i and r_J has shape
    [nth][nr]."""
    dth = math.pi / nth
    dph = 2.0 * math.pi / nph
    if isinstance(ds, (int, float)):
        wr = 1.0 / ds ** 2
        wt = 1.0 / dth ** 2
        wp = 1.0 / (np.sin(th) * dph) ** 2
    else:
        wr = ((ds.cl + ds.cr) / 2.0)[None, :]
        wt = 1.0 / dth ** 2
        wp = (1.0 / (np.sin(th) * dph) ** 2)[:, None]
    num = math.cos(math.pi / nr) * wr + math.cos(math.pi / nth) * wt + math.cos(math.pi / nph) * wp
    return num / (wr + wt + wp)


def omega_opt(rj):
    """Eq. omega_final."""
    return 2.0 / (1.0 + np.sqrt(1.0 - rj * rj))


def omega_next(omega, rj):
    """One step of Eq. omega_n."""
    return 1.0 / (1.0 - rj * rj * omega / 4.0)


def omega_first(rj):
    return 1.0 / (1.0 - rj * rj / 2.0)


def colours(nr: int, nth: int, nph: int) -> np.ndarray:
    """Colour of every unknown, shape [nph][nth][nr] (radial index i = 1..nr)."""
    k, j, i = np.meshgrid(np.arange(nph), np.arange(nth), np.arange(1, nr + 1), indexing="ij")
    return ((i + j + k) & 1) | ((k >= nph // 2).astype(int) << 1)


def diagonal(nr, nth, nph, ds, th) -> np.ndarray:
    """Diagonal of the r^2-scaled operator: per colatitude (shape nth) on the
    log grid, [nth][nr] on a mapped radial grid."""
    dth = math.pi / nth
    dph = 2.0 * math.pi / nph
    if isinstance(ds, (int, float)):
        return -2.0 / ds ** 2 - 2.0 / dth ** 2 - 2.0 / (np.sin(th) * dph) ** 2
    return (-(ds.cl + ds.cr)[None, :] - 2.0 / dth ** 2 - (2.0 / (np.sin(th) * dph) ** 2)[:, None])


def colour_pass(u: np.ndarray, rho_nodes: np.ndarray, r: np.ndarray, ds, th: np.ndarray, colour: int,
                omega_j: np.ndarray, four_pi_G: float = 1.0) -> np.ndarray:
    """Every unknown of `colour` becomes u + omega_j (u_GS - u), u_GS solving
    its own row of r^2 lap u = r^2 4 pi G rho for it (in place; the radial
    ghosts of u are the boundary values)."""
    nph, nth, m = u.shape
    nr = m - 2
    col = colours(nr, nth, nph)
    res = O.sph_residual(u, rho_nodes, r, ds, th, four_pi_G)
    d = diagonal(nr, nth, nph, ds, th)
    d = d[None, :, None] if d.ndim == 1 else d[None, :, :]
    # u_GS = u + res / d (the residual with u itself, divided by the diagonal);
    # omega per colatitude (log grid) or per colatitude and radius
    om = np.asarray(omega_j, dtype=np.float64)
    w = np.broadcast_to(om[None, :, None] if om.ndim == 1 else om[None, :, :], res.shape)
    upd = np.where(col == colour, w * res / d, 0.0)
    u[:, :, 1:nr + 1] += upd
    return u


def sweep(u, rho_nodes, r, ds, th, omega_red, omega_black, four_pi_G=1.0):
    """Red half-sweep (colours 0, 2) with omega_red, black (1, 3) with
    omega_black."""
    for c in (0, 2):
        colour_pass(u, rho_nodes, r, ds, th, c, omega_red, four_pi_G)
    for c in (1, 3):
        colour_pass(u, rho_nodes, r, ds, th, c, omega_black, four_pi_G)
    return u
