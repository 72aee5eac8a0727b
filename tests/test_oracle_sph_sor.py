"""Pins of the spherical SOR oracle (Section 2.1.1, Eqs. omega_final,
omega_n, local_rjac)."""
import math

import numpy as np
import pytest

from oracle import direct as OD
from oracle import multipole as OM
from oracle import operators as OO
from oracle import sph_sor as SS


def _setup(nr=6, nth=4, nph=8, seed=0):
    r, th, ph, ds = OM.sph_axes(nr, nth, nph)
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((nph, nth, nr + 2))
    rho = rng.standard_normal((nph, nth, nr + 2))
    return u, rho, r, th, ds


def test_colours_separate_every_neighbour_including_across_the_poles():
    nr, nth, nph = 5, 4, 8
    col = SS.colours(nr, nth, nph)
    half = nph // 2
    for k in range(nph):
        for j in range(nth):
            for i in range(nr):
                c = col[k, j, i]
                nb = []
                if i + 1 < nr:
                    nb.append(col[k, j, i + 1])
                if i > 0:
                    nb.append(col[k, j, i - 1])
                nb.append(col[k, j + 1, i] if j + 1 < nth else col[(k + half) % nph, j, i])
                nb.append(col[k, j - 1, i] if j > 0 else col[(k + half) % nph, j, i])
                nb.append(col[(k + 1) % nph, j, i])
                nb.append(col[(k - 1) % nph, j, i])
                assert c not in nb


def test_colour_pass_equals_a_sequential_loop():
    """Updating a colour at once equals updating its nodes one by one in any
    order (brute-force loop, reversed order), with relaxation."""
    u, rho, r, th, ds = _setup()
    nph, nth, m = u.shape
    nr = m - 2
    om = 1.0 + 0.5 * np.linspace(0.1, 0.9, nth)
    for colour in range(4):
        a = u.copy()
        SS.colour_pass(a, rho, r, ds, th, colour, om)
        b = u.copy()
        col = SS.colours(nr, nth, nph)
        d = SS.diagonal(nr, nth, nph, ds, th)
        idx = [(k, j, i) for k in range(nph) for j in range(nth) for i in range(nr) if col[k, j, i] == colour]
        for k, j, i in reversed(idx):
            res = OO.sph_residual(b, rho, r, ds, th)[k, j, i]
            b[k, j, i + 1] += om[j] * res / d[j]
        assert np.allclose(a, b, rtol=0, atol=1e-12 * np.max(np.abs(a)))


def test_local_rjac_reduces_to_the_uniform_cartesian_value():
    """With equal spacings, equal counts and sin(theta) = 1 the weights are
    equal and Eq. local_rjac gives cos(pi / N) as Eq. rjac does."""
    n = 64
    ds = math.pi / n
    th = np.array([math.pi / 2])
    rj = SS.local_rjac(n, n, 2 * n, ds, th)
    # dphi = 2 pi / (2n) = pi / n: all three spacings equal; the phi count is 2n
    w = 1.0 / ds ** 2
    expect = (math.cos(math.pi / n) * 2 * w + math.cos(math.pi / (2 * n)) * w) / (3 * w)
    assert rj[0] == pytest.approx(expect, rel=1e-15)
    assert 0.0 < rj[0] < 1.0


def test_chebyshev_sequence_converges_to_omega_opt():
    """The fixed point of Eq. omega_n is Eq. omega_final's omega_opt; from
    omega_1 > omega_opt the sequence decreases monotonically onto it."""
    for rj in (0.5, 0.9, 0.999):
        w = SS.omega_first(rj)
        assert w > float(SS.omega_opt(rj)) > 1.0
        prev = w
        for _ in range(20000):
            w = SS.omega_next(w, rj)
            assert w <= prev + 1e-15
            prev = w
        assert w == pytest.approx(float(SS.omega_opt(rj)), rel=1e-6)


def test_sor_converges_to_the_exact_discrete_solution():
    nr, nth, nph = 8, 8, 8
    r, th, ph, ds = OM.sph_axes(nr, nth, nph)
    rng = np.random.default_rng(3)
    rho = np.abs(rng.standard_normal((nph, nth, nr + 2)))
    ghost = np.zeros((nph, nth, nr + 2))
    ghost[:, :, 0] = rng.standard_normal()
    ghost[:, :, -1] = -1.0
    ref = OD.solve_sph(ghost, rho, r, ds, th)
    u = ghost.copy()
    rj = SS.local_rjac(nr, nth, nph, ds, th)
    w = SS.omega_first(rj)
    for _ in range(400):
        wr = w
        w = SS.omega_next(w, rj)
        wb = w
        w = SS.omega_next(w, rj)
        SS.sweep(u, rho, r, ds, th, wr, wb)
    assert np.max(np.abs(u - ref)) < 1e-10 * np.max(np.abs(ref))
