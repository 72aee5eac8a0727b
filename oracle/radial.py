"""Radial node maps of the spherical grid (Section 3.3): the logarithmic grid
over r_in..r_out and its extension by padding shells, where the density is
zero and which only move the multipole boundary away from the mass.

Test infrastructure: imported by tests and the benchmark's CPU baseline only.

Map.  Radial nodes sit at integer values of a map coordinate xi; the
unknowns are i = 0 .. nr-1 with ghost (Dirichlet) nodes at i = -1 and nr.
The logarithmic core is r = r_in exp(xi ds) for xi = 0 .. nlog-1 (its first
and last nodes at r_in and r_out).  An outer pad of ext_out cells continues
the logarithmic map (its last node is the outer ghost).  An inner pad of
ext_in cells continues the grid inward with a fourth-order polynomial
Q(xi), -ext_in <= xi <= 0, that matches the logarithmic map and its first
three derivatives at r_in and ends at r_pad (the inner ghost):
    Q(xi) = r_in (1 + ds xi + (ds xi)^2/2 + (ds xi)^3/6) + c4 xi^4.
Without pads (ext = 0) the ghosts are one logarithmic step beyond r_in and
r_out, the plain log grid.

Operator.  With r = R(xi) on a uniform xi grid, r^2 lap in the radial
direction is a(xi) u_xixi + b(xi) u_xi with a = (r / R')^2 and
b = 2 r / R' - r^2 R'' / R'^3; central differences give the couplings
cl = a - b/2 (to i-1) and cr = a + b/2 (to i+1), diagonal -(cl + cr).  For
the logarithmic map a = 1/ds^2 and b = 1/ds, the s = ln r form.  The radial
part of the volume element per unit xi is r^2 R' (r^3 ds on the log map).
"""
from __future__ import annotations

import math

import numpy as np


class RadialMap:
    def __init__(self, nr: int, r_in: float, r_out: float, ext_in: int = 0, ext_out: int = 0,
                 r_pad: float | None = None):
        self.nr, self.r_in, self.r_out = nr, r_in, r_out
        self.ext_in, self.ext_out = ext_in, ext_out
        self.p = ext_in - 1 if ext_in > 0 else 0          # inner pad unknowns
        q = ext_out - 1 if ext_out > 0 else 0             # outer pad unknowns
        self.nlog = nr - self.p - q
        if self.nlog < 2:
            raise ValueError("the logarithmic core needs at least two nodes")
        self.ds = math.log(r_out / r_in) / (self.nlog - 1)
        if ext_in > 0:
            if r_pad is None or not (0.0 < r_pad < r_in):
                raise ValueError("inner pad needs 0 < r_pad < r_in")
            E, d = float(ext_in), self.ds
            cubic = 1.0 - d * E + (d * E) ** 2 / 2 - (d * E) ** 3 / 6
            self.c4 = (r_pad - r_in * cubic) / E ** 4
            t = np.linspace(-E, 0.0, 2001)
            if np.any(self._d1(t) <= 0.0):
                raise ValueError("inner pad polynomial is not monotone")
        self.r_pad = r_pad
        xi = self.xi(np.arange(-1, nr + 1))
        self.r = self.R(xi)                               # nodes -1 .. nr
        xu = xi[1:-1]
        r, r1, r2 = self.r[1:-1], self._d1(xu), self._d2(xu)
        a = (r / r1) ** 2
        b = 2.0 * r / r1 - r * r * r2 / r1 ** 3
        self.cl = a - b / 2.0
        self.cr = a + b / 2.0
        self.w = r * r * r1                               # radial volume weight per unit xi

    def level_couplings(self, level: int, n: int):
        """(cl, cr) of the operator rediscretised on multigrid level `level`,
        whose n radial unknowns pair the cells of the level below two by two:
        unknown I sits at xi = 2^level I + (2^level - 1)/2 - p (the mean of
        the nodes it pairs) with spacing h = 2^level; a = (r / (h R'))^2,
        b = 2 r / (h R') - r^2 R'' / (h R'^3)."""
        h = float(2 ** level)
        xi = h * np.arange(n) + (h - 1.0) / 2.0 - self.p
        r, r1, r2 = self.R(xi), self._d1(xi), self._d2(xi)
        a = (r / (h * r1)) ** 2
        b = 2.0 * r / (h * r1) - r * r * r2 / (h * r1 ** 3)
        return a - b / 2.0, a + b / 2.0

    def xi(self, i):
        """Map coordinate of radial index i (0 .. nr-1 unknowns, -1 and nr ghosts)."""
        return np.asarray(i, dtype=np.float64) - self.p

    def _poly(self, xi):
        return xi < 0.0 if self.ext_in > 0 else np.zeros(np.shape(xi), dtype=bool)

    def R(self, xi):
        xi = np.asarray(xi, dtype=np.float64)
        d = self.ds
        out = self.r_in * np.exp(xi * d)
        if self.ext_in > 0:
            m = self._poly(xi)
            x = xi[m]
            out[m] = self.r_in * (1 + d * x + (d * x) ** 2 / 2 + (d * x) ** 3 / 6) + self.c4 * x ** 4
        return out

    def _d1(self, xi):
        xi = np.asarray(xi, dtype=np.float64)
        d = self.ds
        out = d * self.r_in * np.exp(xi * d)
        if self.ext_in > 0:
            m = self._poly(xi)
            x = xi[m]
            out[m] = self.r_in * (d + d * d * x + d ** 3 * x * x / 2) + 4 * self.c4 * x ** 3
        return out

    def _d2(self, xi):
        xi = np.asarray(xi, dtype=np.float64)
        d = self.ds
        out = d * d * self.r_in * np.exp(xi * d)
        if self.ext_in > 0:
            m = self._poly(xi)
            x = xi[m]
            out[m] = self.r_in * (d * d + d ** 3 * x) + 12 * self.c4 * x * x
        return out
