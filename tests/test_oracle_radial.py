"""Pins of the mapped radial grid of the spherical solver (Section 3.3: the
logarithmic grid extended by padding shells, the inner one by a fourth-order
polynomial)."""
import math

import numpy as np
import pytest

from oracle import direct as D
from oracle import multipole as OM
from oracle import operators as O
from oracle import sph_sor as SS
from oracle.radial import RadialMap


def test_plain_map_is_the_log_grid():
    """Without pads the map's radii are the log grid's and its couplings the
    s = ln r form 1/ds^2 -+ 1/(2 ds)."""
    nr = 40
    m = RadialMap(nr, 1e-3, 1.0)
    r, th, ph, ds = OM.sph_axes(nr, 8, 16)
    assert m.ds == pytest.approx(ds, rel=1e-15)
    assert np.allclose(m.r, r, rtol=1e-13, atol=0)
    assert np.allclose(m.cl, 1 / ds ** 2 - 1 / (2 * ds), rtol=1e-12)
    assert np.allclose(m.cr, 1 / ds ** 2 + 1 / (2 * ds), rtol=1e-12)
    assert np.allclose(m.w, r[1:-1] ** 3 * ds, rtol=1e-12)
    u = np.random.default_rng(0).normal(size=(16, 8, nr + 2))
    a = O.sph_apply(u, ds, th)
    b = O.sph_apply(u, m, th)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_inner_pad_polynomial():
    """The pad polynomial matches the log map and its first three derivatives
    at r_in (one-sided differences agree), ends at r_pad, is monotone, and its
    spacing grows inward (the point of the extension).  The shape of the
    paper's test: 20 pad cells down to r_in / 2, log steps of about 1%."""
    m = RadialMap(100, 0.5, 1.0, ext_in=20, ext_out=10, r_pad=0.25)
    assert m.R(np.array([-20.0]))[0] == pytest.approx(0.25, rel=1e-14)
    assert m.r[0] == pytest.approx(0.25, rel=1e-14)                       # inner ghost at r_pad
    assert m.r[m.p + 1] == pytest.approx(0.5, rel=1e-14)                  # first core node at r_in
    for f in (m.R, m._d1, m._d2):
        left, right = f(np.array([-1e-7]))[0], f(np.array([1e-7]))[0]
        assert left == pytest.approx(right, rel=1e-6)
    d2l = (m._d2(np.array([-1e-6]))[0] - m._d2(np.array([0.0]))[0]) / -1e-6
    d2r = (m._d2(np.array([1e-6]))[0] - m._d2(np.array([0.0]))[0]) / 1e-6
    assert d2l == pytest.approx(d2r, rel=1e-3)                           # third derivative continuous
    assert np.all(np.diff(m.r) > 0)
    steps = np.diff(m.r)
    assert steps[0] > 3 * steps[m.p + 1]
    # outer pad continues the log map up to the outer ghost
    assert m.r[-1] == pytest.approx(1.0 * math.exp(10 * m.ds), rel=1e-13)


def test_pad_rejects_bad_parameters():
    with pytest.raises(ValueError):
        RadialMap(60, 0.01, 1.0, ext_in=20, r_pad=0.02)
    with pytest.raises(ValueError):
        RadialMap(30, 0.01, 1.0, ext_in=20, ext_out=12, r_pad=0.005)


def _radial_problem(k):
    """u = r^2 + 1/r (lap u = 6) on a padded grid refined k times."""
    nr = 40 * 2 ** k
    m = RadialMap(nr, 0.05, 1.0, ext_in=8 * 2 ** k, ext_out=4 * 2 ** k, r_pad=0.025)
    nth, nph = 4, 8
    th = (np.arange(nth) + 0.5) * math.pi / nth
    exact = m.r ** 2 + 1.0 / m.r
    ghost = np.zeros((nph, nth, nr + 2))
    ghost[:, :, 0], ghost[:, :, -1] = exact[0], exact[-1]
    rho = np.full((nph, nth, nr + 2), 6.0)
    got = D.solve_sph(ghost, rho, m.r, m, th)
    return np.max(np.abs(got[0, 0, 1:-1] - exact[1:-1])) / np.max(np.abs(exact))


def test_mapped_operator_converges_at_second_order():
    e = [_radial_problem(k) for k in range(3)]
    assert e[0] / e[1] == pytest.approx(4.0, rel=0.15)
    assert e[1] / e[2] == pytest.approx(4.0, rel=0.1)


def test_exact_solution_matches_dense_solve_on_padded_grid():
    nr, nth, nph = 14, 4, 8
    m = RadialMap(nr, 0.5, 1.0, ext_in=4, ext_out=3, r_pad=0.3)
    th = (np.arange(nth) + 0.5) * math.pi / nth
    rng = np.random.default_rng(2)
    ghost = np.zeros((nph, nth, nr + 2))
    ghost[:, :, 0], ghost[:, :, -1] = rng.normal(size=(nph, nth)), rng.normal(size=(nph, nth))
    rho = rng.normal(size=(nph, nth, nr + 2))
    a = D.solve_sph(ghost, rho, m.r, m, th)
    b = D.dense_solve_sph(ghost, rho, m.r, m, th)
    assert np.max(np.abs(a - b)) < 1e-10 * np.max(np.abs(b))


def test_radial_weights_integrate_r2():
    """sum of r^2 R' over a segment of the padded grid approaches the
    integral of r^2 at second order (trapezoid-like)."""
    errs = []
    for k in range(3):
        m = RadialMap(40 * 2 ** k, 0.05, 1.0, ext_in=8 * 2 ** k, r_pad=0.025)
        # trapezoid weights in xi between the first and last unknown
        w = m.w.copy()
        w[0] *= 0.5
        w[-1] *= 0.5
        exact = (m.r[-2] ** 3 - m.r[1] ** 3) / 3
        errs.append(abs(w.sum() - exact) / exact)
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_local_rjac_on_mapped_grid_reduces_to_colatitude_form():
    nr, nth, nph = 20, 8, 16
    m = RadialMap(nr, 1e-3, 1.0)
    th = (np.arange(nth) + 0.5) * math.pi / nth
    a = SS.local_rjac(nr, nth, nph, m.ds, th)
    b = SS.local_rjac(nr, nth, nph, m, th)
    assert b.shape == (nth, nr)
    assert np.allclose(b, a[:, None], rtol=1e-12)
    mp = RadialMap(nr, 0.05, 1.0, ext_in=3, r_pad=0.025)
    c = SS.local_rjac(nr, nth, nph, mp, th)
    assert np.all((c > 0) & (c < 1)) and np.ptp(c[0]) > 0


def test_multipole_shells_on_mapped_grid():
    """Point-like mass near the centre on a padded grid: q_00 is the
    weighted sum, the outer shell sees -G M / r, the inner shell (inside the
    mass shell's radius) a constant."""
    nr, nth, nph = 30, 8, 16
    m = RadialMap(nr, 0.05, 1.0, ext_in=6, ext_out=4, r_pad=0.025)
    rho = np.zeros((nph, nth, nr + 2))
    i0 = 12
    rho[:, :, i0] = 1.0                      # a thin spherical shell at r[i0]
    phi, q, qb = OM.sph_boundary(rho, nr, nth, nph, 4, rmap=m)
    th = (np.arange(nth) + 0.5) * math.pi / nth
    mass = m.w[i0 - 1] * np.sum(np.sin(th)) * (math.pi / nth) * (2 * math.pi / nph) * nph
    assert q[0] == pytest.approx(mass, rel=1e-12)
    G = 1.0 / (4 * math.pi)
    assert np.allclose(phi[:, :, -1], -G * q[0] / m.r[-1], rtol=1e-3)
    assert np.ptp(phi[:, :, 0]) < 1e-3 * abs(phi[0, 0, 0])


def test_level_couplings_on_the_log_map():
    """Multigrid level l of the plain log map has the s = ln r couplings of
    spacing 2^l ds."""
    m = RadialMap(64, 1e-3, 1.0)
    for level, n in ((0, 64), (1, 32), (3, 8)):
        cl, cr = m.level_couplings(level, n)
        d = m.ds * 2 ** level
        assert np.allclose(cl, 1 / d ** 2 - 1 / (2 * d), rtol=1e-12)
        assert np.allclose(cr, 1 / d ** 2 + 1 / (2 * d), rtol=1e-12)
    cl, cr = m.level_couplings(0, 64)
    assert np.allclose(cl, m.cl, rtol=1e-14) and np.allclose(cr, m.cr, rtol=1e-14)


def test_multigrid_preconditioner_cycle_on_padded_grid():
    """One V(2,2) cycle of the spherical preconditioner on a padded grid
    (levels rediscretised from the map) cuts the residual of a random right-
    hand side about as much as on the log grid (0.42 against 0.35 on this
    two-level grid)."""
    from oracle import sph_mg as SM
    nr, nth, nph = 32, 8, 16
    m = RadialMap(nr, 0.5, 1.0, ext_in=5, ext_out=5, r_pad=0.3)
    lv = SM.level0(m, nr)
    f = np.random.default_rng(3).normal(size=(nph, nth, nr))
    u = SM.vcycle(f, lv)
    red = np.linalg.norm(f - SM.apply(u, lv)) / np.linalg.norm(f)
    flog = SM.vcycle(f, m.ds)
    red_log = np.linalg.norm(f - SM.apply(flog, m.ds)) / np.linalg.norm(f)
    assert red < 0.6 and red < 1.5 * red_log, (red, red_log)
