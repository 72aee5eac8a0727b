"""Pins for the oracle's discrete Laplacians (Eqs. 1 and 2)."""
import math

import numpy as np
import pytest

from oracle import multipole as M
from oracle import operators as O


def _cart_fields(n, g):
    x = M.cart_coords(n, g)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z


def test_lap7_exact_on_quadratics():
    n = 12
    X, Y, Z = _cart_fields(n, 1)
    u = X ** 2 + 2 * Y ** 2 - Z ** 2 + 3 * X * Y + X
    np.testing.assert_allclose(O.lap7(u, n, 1.0 / n, 1), 2.0 + 4.0 - 2.0, atol=1e-10)


@pytest.mark.parametrize("k", [(1, 1, 1), (2, 3, 5), (7, 1, 4)])
def test_lap7_dirichlet_sine_eigenmodes(k):
    n = 8
    h = 1.0 / n
    X, Y, Z = _cart_fields(n, 1)
    u = np.sin(np.pi * k[0] * X) * np.sin(np.pi * k[1] * Y) * np.sin(np.pi * k[2] * Z)
    lam = sum((2 * math.cos(math.pi * kk * h) - 2) / h ** 2 for kk in k)
    np.testing.assert_allclose(O.lap7(u, n, h, 1), lam * u[1:n, 1:n, 1:n], atol=1e-11)


def test_lap19_exact_on_degree7_polynomials():
    n = 16
    X, Y, Z = _cart_fields(n, 3)
    u = X ** 6 + Y ** 7 - 2 * Z ** 4 + X ** 3 * Y ** 2
    ref = 30 * X ** 4 + 42 * Y ** 5 - 24 * Z ** 2 + 6 * X * Y ** 2 + 2 * X ** 3
    np.testing.assert_allclose(O.lap19(u, n, 1.0 / n, 3), ref[3:3 + n - 1, 3:3 + n - 1, 3:3 + n - 1],
                               atol=1e-9)
    # and not exact at degree 8 (the leading truncation term is an 8th derivative)
    u8 = X ** 8
    err = O.lap19(u8, n, 1.0 / n, 3) - 56 * X[3:3 + n - 1, 3:3 + n - 1, 3:3 + n - 1] ** 6
    assert np.max(np.abs(err)) > 1e-8


@pytest.mark.parametrize("k", [(1, 2, 3), (5, 5, 1)])
def test_lap19_sine_modes_have_the_symbol(k):
    """Sine modes are odd about the Dirichlet planes, so with the ghosts
    holding the mode's own values the star acts by its Fourier symbol
    sum_d [c0 + 2 sum_q c_q cos(q t_d)] / h^2, t_d = pi k_d h."""
    n = 10
    h = 1.0 / n
    X, Y, Z = _cart_fields(n, 3)
    u = np.sin(np.pi * k[0] * X) * np.sin(np.pi * k[1] * Y) * np.sin(np.pi * k[2] * Z)
    c = O.STAR6
    lam = 0.0
    for kk in k:
        t = math.pi * kk * h
        lam += (c[0] + 2 * (c[1] * math.cos(t) + c[2] * math.cos(2 * t) + c[3] * math.cos(3 * t))) / h ** 2
    np.testing.assert_allclose(O.lap19(u, n, h, 3), lam * u[3:3 + n - 1, 3:3 + n - 1, 3:3 + n - 1],
                               atol=1e-10)


def test_residual_and_rhs_norm():
    n = 6
    rng = np.random.default_rng(0)
    u = rng.normal(size=(n + 1,) * 3)
    f = rng.normal(size=(n + 1,) * 3)
    r = O.residual(u, f, n, 1.0 / n, 2, 1)
    np.testing.assert_allclose(r, f[1:n, 1:n, 1:n] - O.lap7(u, n, 1.0 / n, 1))
    z = u.copy()
    z[1:n, 1:n, 1:n] = 0
    assert O.rhs_norm(u, f, n, 1.0 / n, 2, 1) == pytest.approx(
        np.linalg.norm(f[1:n, 1:n, 1:n] - O.lap7(z, n, 1.0 / n, 1)))


# ---------------------------------------------------------------- spherical
def _sph(nr=10, nth=8, nph=16):
    r, th, ph, ds = M.sph_axes(nr, nth, nph)
    return r, th, ph, ds


@pytest.mark.parametrize("p", [-1.0, 0.5, 2.0])
def test_sph_apply_on_powers_of_r(p):
    """On u = r^p = e^{ps} the angular parts vanish and the radial part is
    r^p [(2 cosh(p ds) - 2)/ds^2 + sinh(p ds)/ds] exactly."""
    r, th, ph, ds = _sph()
    u = np.broadcast_to(r[None, None, :] ** p, (len(ph), len(th), len(r))).copy()
    out = O.sph_apply(u, ds, th)
    ref = r[1:-1] ** p * ((2 * math.cosh(p * ds) - 2) / ds ** 2 + math.sinh(p * ds) / ds)
    np.testing.assert_allclose(out, np.broadcast_to(ref, out.shape), rtol=1e-10)


def test_sph_apply_on_log_r_is_one():
    """r^2 lap(ln r) = 1, and the central differences are exact on s."""
    r, th, ph, ds = _sph()
    u = np.broadcast_to(np.log(r)[None, None, :], (len(ph), len(th), len(r))).copy()
    np.testing.assert_allclose(O.sph_apply(u, ds, th), 1.0, rtol=1e-9)


@pytest.mark.parametrize("m", [2, 4])
def test_sph_apply_azimuthal_symbol(m):
    """u = cos(m phi) (even m is unchanged by the pole reflection): only the
    phi part acts, with symbol (2 cos(m dphi) - 2) / (dphi^2 sin^2 theta)."""
    r, th, ph, ds = _sph()
    dph = 2 * math.pi / len(ph)
    u = np.broadcast_to(np.cos(m * ph)[:, None, None], (len(ph), len(th), len(r))).copy()
    out = O.sph_apply(u, ds, th)
    sym = (2 * math.cos(m * dph) - 2) / (dph ** 2 * np.sin(th) ** 2)
    np.testing.assert_allclose(out, sym[None, :, None] * u[:, :, 1:-1], atol=1e-9)


def test_sph_apply_pole_reflection_on_odd_mode():
    """u = sin(theta) cos(phi) = x/r restricted to the sphere (an l = 1
    function): across the pole its value flips sign with phi + pi, which the
    reflected neighbour must reproduce; compare to the direct formula."""
    r, th, ph, ds = _sph(nr=4, nth=8, nph=16)
    P, T = np.meshgrid(ph, th, indexing="ij")
    ang = np.sin(T) * np.cos(P)
    u = np.repeat(ang[:, :, None], len(r), axis=2)
    out = O.sph_apply(u, ds, th)
    dth = math.pi / len(th)
    dph = 2 * math.pi / len(ph)
    # direct evaluation with the analytic continuation sin(-t) cos(phi) = -sin t cos phi
    tp, tm = T + dth, T - dth
    f = lambda t, p_: np.sin(t) * np.cos(p_)
    th_part = (f(tp, P) - 2 * f(T, P) + f(tm, P)) / dth ** 2 \
        + (np.cos(T) / np.sin(T)) * (f(tp, P) - f(tm, P)) / (2 * dth)
    ph_part = (f(T, P + dph) - 2 * f(T, P) + f(T, P - dph)) / (dph ** 2 * np.sin(T) ** 2)
    np.testing.assert_allclose(out, (th_part + ph_part)[:, :, None] * np.ones(len(r) - 2), atol=1e-10)
