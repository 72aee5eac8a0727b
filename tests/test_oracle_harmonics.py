"""Pins for the oracle's spherical / solid harmonics (Section 2.2 conventions)."""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, sph_harm_y

from oracle import harmonics as H

LMAX = 8


def test_low_order_closed_forms():
    rng = np.random.default_rng(0)
    th = rng.uniform(0, np.pi, 50)
    ph = rng.uniform(-np.pi, np.pi, 50)
    Y = H.real_ylm(2, th, ph)
    c = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(Y[H.idx(0, 0)], 1 / math.sqrt(4 * math.pi), rtol=1e-15)
    np.testing.assert_allclose(Y[H.idx(1, 0)], c * np.cos(th), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(Y[H.idx(1, 1)], c * np.sin(th) * np.cos(ph), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(Y[H.idx(1, -1)], c * np.sin(th) * np.sin(ph), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(Y[H.idx(2, 0)],
                               math.sqrt(5 / (16 * math.pi)) * (3 * np.cos(th) ** 2 - 1),
                               rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(Y[H.idx(2, 2)],
                               math.sqrt(15 / (16 * math.pi)) * np.sin(th) ** 2 * np.cos(2 * ph),
                               rtol=1e-13, atol=1e-14)


def test_orthonormal_on_sphere():
    # Gauss-Legendre in cos(theta) x uniform phi integrates degree <= 2*LMAX exactly
    x, w = np.polynomial.legendre.leggauss(2 * LMAX + 2)
    nph = 4 * LMAX + 4
    ph = np.arange(nph) * 2 * np.pi / nph
    TH, PH = np.meshgrid(np.arccos(x), ph, indexing="ij")
    W = np.repeat(w[:, None], nph, axis=1) * (2 * np.pi / nph)
    Y = H.real_ylm(LMAX, TH, PH).reshape(H.n_terms(LMAX), -1)
    gram = (Y * W.ravel()) @ Y.T
    np.testing.assert_allclose(gram, np.eye(H.n_terms(LMAX)), atol=1e-13)


def test_addition_theorem():
    rng = np.random.default_rng(1)
    a = rng.normal(size=(30, 3))
    b = rng.normal(size=(30, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya = H.regular_solid(LMAX, a)
    Yb = H.regular_solid(LMAX, b)
    cosg = np.sum(a * b, axis=1)
    for l in range(LMAX + 1):
        s = sum(Ya[H.idx(l, m)] * Yb[H.idx(l, m)] for m in range(-l, l + 1))
        np.testing.assert_allclose(s, eval_legendre(l, cosg), atol=1e-13)


def test_against_scipy_complex_harmonics():
    """Real harmonics without Condon-Shortley phase from SciPy's complex ones:
    m > 0: sqrt2 (-1)^m Re Y_l^m; m < 0: sqrt2 (-1)^|m| Im Y_l^|m|."""
    rng = np.random.default_rng(2)
    th = rng.uniform(0, np.pi, 40)
    ph = rng.uniform(0, 2 * np.pi, 40)
    Y = H.real_ylm(LMAX, th, ph)
    for l in range(LMAX + 1):
        for m in range(-l, l + 1):
            z = sph_harm_y(l, abs(m), th, ph)
            if m == 0:
                ref = z.real
            elif m > 0:
                ref = math.sqrt(2) * (-1) ** m * z.real
            else:
                ref = math.sqrt(2) * (-1) ** m * z.imag
            np.testing.assert_allclose(Y[H.idx(l, m)], ref, atol=1e-12, rtol=1e-12)


def test_solid_harmonics_low_order_and_homogeneity():
    rng = np.random.default_rng(3)
    p = rng.normal(size=(20, 3))
    R = H.regular_solid(2, p)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    r2 = np.sum(p * p, axis=1)
    np.testing.assert_allclose(R[H.idx(0, 0)], 1.0, rtol=1e-15)
    np.testing.assert_allclose(R[H.idx(1, 0)], z, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(R[H.idx(1, 1)], x, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(R[H.idx(1, -1)], y, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(R[H.idx(2, 0)], (3 * z * z - r2) / 2, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(R[H.idx(2, 2)], math.sqrt(3) / 2 * (x * x - y * y), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(R[H.idx(2, -2)], math.sqrt(3) * x * y, rtol=1e-12, atol=1e-13)
    # degree-l homogeneity of r^l Y and r^-(l+1) Y
    t = 1.7
    R1 = H.regular_solid(LMAX, p)
    R2 = H.regular_solid(LMAX, t * p)
    I1 = H.irregular_solid(LMAX, p)
    I2 = H.irregular_solid(LMAX, t * p)
    for l in range(LMAX + 1):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(R2[H.idx(l, m)], t ** l * R1[H.idx(l, m)], rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(I2[H.idx(l, m)], t ** (-l - 1) * I1[H.idx(l, m)], rtol=1e-12, atol=1e-12)


def test_regular_solid_at_origin():
    R = H.regular_solid(LMAX, np.zeros((1, 3)))
    assert abs(R[0, 0] - 1.0) < 1e-15
    assert np.all(R[1:, 0] == 0.0)


@pytest.mark.parametrize("l", [1, 3, 6])
def test_regular_solid_harmonics_are_harmonic(l):
    """r^l Y_lm is a harmonic polynomial: a 4th-order finite-difference
    Laplacian at a random point vanishes to truncation level."""
    rng = np.random.default_rng(4)
    p0 = rng.normal(size=3) * 0.5
    e = 1e-2
    for m in range(-l, l + 1):
        def f(q):
            return H.regular_solid(l, q[None, :])[H.idx(l, m), 0]
        lap = 0.0
        for d in range(3):
            dv = np.zeros(3)
            dv[d] = e
            lap += (-f(p0 + 2 * dv) + 16 * f(p0 + dv) - 30 * f(p0) + 16 * f(p0 - dv) - f(p0 - 2 * dv)) / (12 * e * e)
        scale = max(1.0, abs(f(p0)))
        assert abs(lap) < 1e-6 * scale
