"""Closed-form potentials of the test densities (4 pi G = four_pi_G).

* Uniform sphere of density rho0 and radius a: inside
  Phi = (4 pi G rho0 / 6)(r^2 - 3 a^2), outside Phi = -G M / r.
* Gaussian clump of mass M and width s: Phi = -G M erf(d / (sqrt(2) s)) / d.
* Smooth sphere rho_p (1 - w^2)^2 of radius a (Section 3.1):
  Phi = 4 pi G rho_p a^2 (-1/6 + w^2/6 - w^4/10 + w^6/42) inside and
  -G M_p / d outside, with M_p = (32 pi / 105) rho_p a^3.
* Truncated singular isothermal sphere rho0 / r^2 for r < R (Section 3.3):
  Phi = 4 pi G rho0 (ln(r / R) - 1) inside, -G M / r outside, M = 4 pi rho0 R.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def _dist(x, c):
    x = np.asarray(x, dtype=np.float64)
    return np.sqrt(np.sum((x - np.asarray(c, dtype=np.float64)) ** 2, axis=-1))


def uniform_sphere(x, centre, a, rho0=1.0, four_pi_G=1.0):
    G = four_pi_G / (4 * math.pi)
    r = _dist(x, centre)
    M = 4.0 / 3.0 * math.pi * a ** 3 * rho0
    inside = four_pi_G * rho0 / 6.0 * (r * r - 3 * a * a)
    outside = -G * M / np.where(r > 0, r, 1.0)
    return np.where(r < a, inside, outside)


def gaussian_clump(x, centre, sigma, mass, four_pi_G=1.0):
    G = four_pi_G / (4 * math.pi)
    d = _dist(x, centre)
    safe = np.where(d > 0, d, 1.0)
    far = -G * mass * erf(d / (math.sqrt(2.0) * sigma)) / safe
    centre_val = -G * mass * math.sqrt(2.0 / math.pi) / sigma
    return np.where(d > 0, far, centre_val)


def smooth_sphere(x, centre, a, mass, four_pi_G=1.0):
    G = four_pi_G / (4 * math.pi)
    rho_p = mass / (32.0 * math.pi / 105.0 * a ** 3)
    d = _dist(x, centre)
    w2 = (d / a) ** 2
    inside = four_pi_G * rho_p * a * a * (-1 / 6 + w2 / 6 - w2 ** 2 / 10 + w2 ** 3 / 42)
    outside = -G * mass / np.where(d > 0, d, 1.0)
    return np.where(d < a, inside, outside)


def sis(r, rho0=1.0, r_out=0.8, four_pi_G=1.0):
    G = four_pi_G / (4 * math.pi)
    r = np.asarray(r, dtype=np.float64)
    M = 4 * math.pi * rho0 * r_out
    return np.where(r < r_out, four_pi_G * rho0 * (np.log(r / r_out) - 1.0), -G * M / r)
