"""Multipole moments of the density and the open-boundary ghost potential.

Section 2.2:
* outer moments q_lm = sum over cells of w rho sqrt(4pi/(2l+1)) r'^l Y_lm
  (Eq. outer_multipole), potential at an outer point
  Phi = -G sum q_lm sqrt(4pi/(2l+1)) Y_lm / r^(l+1) (Eq. outer_expansion);
* inner moments qbar_lm = sum of w rho sqrt(4pi/(2l+1)) Y_lm / r'^(l+1)
  (Eq. inner_multipole), potential at an inner point
  Phi = -G sum qbar_lm sqrt(4pi/(2l+1)) r^l Y_lm (Eq. inner_expansion).

The integrals are sums over the unknown (interior) nodes with quadrature
weight h^3 on the Cartesian grid and r^3 ds sin(theta) dtheta dphi on the
log-spherical grid.  The expansion origin is the centre of the Cartesian box
and r = 0 on the spherical grid.  G = four_pi_G / (4 pi).

A point mass at the origin (the central sink of Section 3.3) may be added; it
contributes M to q_00 and -G M / r at inner points.
"""
from __future__ import annotations

import math

import numpy as np

from . import harmonics as H


# --------------------------------------------------------------------------
# geometry of the node arrays (written independently of the input module)
# --------------------------------------------------------------------------
def cart_coords(n: int, g: int, lo=0.0, hi=1.0) -> np.ndarray:
    h = (hi - lo) / n
    return lo + np.arange(-(g - 1), n + g, dtype=np.float64) * h


def cart_interior_points(n: int, g: int, lo=0.0, hi=1.0):
    """(points[(n-1)^3, 3] relative to the box centre, weight h^3), [k][j][i]."""
    x = cart_coords(n, g, lo, hi)[g:g + n - 1] - 0.5 * (lo + hi)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
    h = (hi - lo) / n
    return pts, h ** 3


def cart_ghost_mask(n: int, g: int) -> np.ndarray:
    m = n + 1 + 2 * (g - 1)
    mask = np.ones((m, m, m), dtype=bool)
    mask[g:g + n - 1, g:g + n - 1, g:g + n - 1] = False
    return mask


def sph_axes(nr, nth, nph, r_min=1e-3, r_max=1.0):
    ds = math.log(r_max / r_min) / (nr - 1)
    r = np.exp(math.log(r_min) + np.arange(-1, nr + 1, dtype=np.float64) * ds)
    th = (np.arange(nth, dtype=np.float64) + 0.5) * (math.pi / nth)
    ph = np.arange(nph, dtype=np.float64) * (2 * math.pi / nph)
    return r, th, ph, ds


def sph_points(r, th, ph):
    """Cartesian positions of nodes [k][j][i] for radii r, angles th, ph."""
    P, T, R = np.meshgrid(ph, th, r, indexing="ij")
    st = np.sin(T)
    return np.stack([R * st * np.cos(P), R * st * np.sin(P), R * np.cos(T)], axis=-1)


# --------------------------------------------------------------------------
# moments and ghost values
# --------------------------------------------------------------------------
def moments_outer(lmax, pts, rho_w):
    """q_lm = sum_n (w rho)_n R_lm(x_n); Eq. outer_multipole as a node sum."""
    q = np.zeros(H.n_terms(lmax))
    chunk = 1 << 18
    for s in range(0, len(rho_w), chunk):
        R = H.regular_solid(lmax, pts[s:s + chunk])
        q += R @ rho_w[s:s + chunk]
    return q


def moments_inner(lmax, pts, rho_w):
    """qbar_lm = sum_n (w rho)_n I_lm(x_n); Eq. inner_multipole as a node sum."""
    q = np.zeros(H.n_terms(lmax))
    chunk = 1 << 18
    for s in range(0, len(rho_w), chunk):
        I = H.irregular_solid(lmax, pts[s:s + chunk])
        q += I @ rho_w[s:s + chunk]
    return q


def phi_outer(q, lmax, pts, G):
    """Eq. outer_expansion at points pts[..., 3]."""
    return -G * np.tensordot(q, H.irregular_solid(lmax, pts), axes=(0, 0))


def phi_inner(qbar, lmax, pts, G):
    """Eq. inner_expansion at points pts[..., 3]."""
    return -G * np.tensordot(qbar, H.regular_solid(lmax, pts), axes=(0, 0))


def cart_moments(rho_nodes: np.ndarray, n: int, g: int, lmax: int, lo=0.0, hi=1.0):
    """Outer moments of a Cartesian node array (interior nodes, weight h^3)."""
    pts, w = cart_interior_points(n, g, lo, hi)
    s = slice(g, g + n - 1)
    rw = np.ascontiguousarray(rho_nodes[s, s, s]).ravel() * w
    return moments_outer(lmax, pts, rw)


def cart_boundary(rho_nodes: np.ndarray, n: int, g: int, lmax: int, four_pi_G=1.0,
                  lo=0.0, hi=1.0):
    """Full node array with every ghost node (faces, edges, corners, all g
    layers) set from the outer expansion and zeros at the unknowns.
    Returns (phi_ghost_array, q)."""
    G = four_pi_G / (4 * math.pi)
    q = cart_moments(rho_nodes, n, g, lmax, lo, hi)
    x = cart_coords(n, g, lo, hi) - 0.5 * (lo + hi)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    mask = cart_ghost_mask(n, g)
    pts = np.stack([X[mask], Y[mask], Z[mask]], axis=-1)
    out = np.zeros(mask.shape)
    out[mask] = phi_outer(q, lmax, pts, G)
    return out, q


def sph_boundary(rho_nodes: np.ndarray, nr, nth, nph, lmax, four_pi_G=1.0,
                 point_mass=0.0, r_min=1e-3, r_max=1.0, rmap=None):
    """Radial ghost shells of the spherical grid: outer expansion at i = nr,
    inner expansion (+ central point mass) at i = -1.  rho_nodes has shape
    [nph][nth][nr+2].  rmap: a radial.RadialMap (radii and radial volume
    weights r^2 R'), else the log grid over r_min..r_max.  Returns
    (phi_array, q, qbar)."""
    G = four_pi_G / (4 * math.pi)
    r, th, ph, ds = sph_axes(nr, nth, nph, r_min, r_max)
    dth, dph = math.pi / nth, 2 * math.pi / nph
    if rmap is not None:
        r = rmap.r
        wr = rmap.w
    else:
        wr = r[1:nr + 1] ** 3 * ds
    ri = r[1:nr + 1]
    pts = sph_points(ri, th, ph).reshape(-1, 3)
    w = wr[None, None, :] * np.sin(th)[None, :, None] * dth * dph
    rw = (rho_nodes[:, :, 1:nr + 1] * w).ravel()
    q = moments_outer(lmax, pts, rw)
    qbar = moments_inner(lmax, pts, rw)
    q[0] += point_mass
    out = np.zeros((nph, nth, nr + 2))
    pin = sph_points(r[:1], th, ph)[:, :, 0, :]
    pout = sph_points(r[-1:], th, ph)[:, :, 0, :]
    out[:, :, 0] = phi_inner(qbar, lmax, pin, G) - G * point_mass / r[0]
    out[:, :, -1] = phi_outer(q, lmax, pout, G)
    return out, q, qbar
