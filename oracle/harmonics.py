"""Real spherical harmonics and the solid harmonics of the multipole expansion.

Section 2.2: the expansion uses real spherical harmonics, cosine type for
m >= 0 and sine type for m < 0, each multiplied by sqrt(4 pi / (2l+1)).
We take them orthonormal on the unit sphere, which is the normalisation for
which the product of the two sqrt factors in the moment and in the
expansion collapses to a Legendre polynomial (addition theorem), so the
ghost potential does not depend on any further convention.  The associated
Legendre functions carry no Condon-Shortley phase.

Moments are indexed flat: ``idx(l, m) = l*l + l + m`` for ``-l <= m <= l``.
"""
from __future__ import annotations

import math

import numpy as np


def idx(l: int, m: int) -> int:
    return l * l + l + m


def n_terms(lmax: int) -> int:
    return (lmax + 1) ** 2


def assoc_legendre(lmax: int, x: np.ndarray) -> dict:
    """P_l^m(x) for 0 <= m <= l <= lmax, no Condon-Shortley phase.

    Standard recurrences: P_m^m = (2m-1)!! (1-x^2)^(m/2),
    P_{m+1}^m = (2m+1) x P_m^m,
    (l-m) P_l^m = (2l-1) x P_{l-1}^m - (l+m-1) P_{l-2}^m.
    """
    x = np.asarray(x, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    P = {}
    pmm = np.ones_like(x)
    for m in range(lmax + 1):
        if m > 0:
            pmm = pmm * (2 * m - 1) * s
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = (2 * m + 1) * x * pmm
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * x * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def real_ylm(lmax: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Orthonormal real Y_lm(theta, phi); returns array [(lmax+1)^2, ...]."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    P = assoc_legendre(lmax, np.cos(theta))
    out = np.empty((n_terms(lmax),) + np.broadcast(theta, phi).shape, dtype=np.float64)
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                             * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                out[idx(l, 0)] = norm * P[(l, 0)]
            else:
                out[idx(l, m)] = math.sqrt(2.0) * norm * P[(l, m)] * np.cos(m * phi)
                out[idx(l, -m)] = math.sqrt(2.0) * norm * P[(l, m)] * np.sin(m * phi)
    return out


def _spherical(d: np.ndarray):
    d = np.asarray(d, dtype=np.float64)
    r = np.sqrt(np.sum(d * d, axis=-1))
    safe = np.where(r > 0.0, r, 1.0)
    theta = np.arccos(np.clip(d[..., 2] / safe, -1.0, 1.0))
    phi = np.arctan2(d[..., 1], d[..., 0])
    return r, theta, phi


def regular_solid(lmax: int, d: np.ndarray) -> np.ndarray:
    """sqrt(4 pi/(2l+1)) r^l Y_lm(d/r) for points d[..., 3] (Eq. outer_multipole
    integrand without the density).  Returns [(lmax+1)^2, ...]."""
    r, theta, phi = _spherical(d)
    Y = real_ylm(lmax, theta, phi)
    for l in range(lmax + 1):
        f = math.sqrt(4 * math.pi / (2 * l + 1)) * r ** l
        for m in range(-l, l + 1):
            Y[idx(l, m)] *= f
    return Y


def irregular_solid(lmax: int, d: np.ndarray) -> np.ndarray:
    """sqrt(4 pi/(2l+1)) Y_lm(d/r) / r^(l+1) (Eq. outer_expansion term without
    the moment; also the integrand of Eq. inner_multipole)."""
    r, theta, phi = _spherical(d)
    Y = real_ylm(lmax, theta, phi)
    for l in range(lmax + 1):
        f = math.sqrt(4 * math.pi / (2 * l + 1)) / r ** (l + 1)
        for m in range(-l, l + 1):
            Y[idx(l, m)] *= f
    return Y
