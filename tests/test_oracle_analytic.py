"""Whole-chain pins: multipole ghosts + exact discrete solve against the
closed-form potentials of the test densities (Sections 3.1 and 3.3)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import analytic as A
from oracle import direct as D
from oracle import multipole as M
from workloads import CartGrid, Clumps, clump_density, smooth_sphere, uniform_sphere


def _solve(rho, n, g, order, lmax):
    ghost, _ = M.cart_boundary(rho, n, g, lmax)
    return D.solve_cart(ghost, rho, n, 1.0 / n, order, g)


def _interior_points(n, g):
    x = M.cart_coords(n, g)[g:g + n - 1]
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def test_uniform_sphere_potential_values():
    c = (0.5, 0.5, 0.5)
    assert A.uniform_sphere(np.array(c), c, 0.25) == pytest.approx(-0.03125)
    assert A.uniform_sphere(np.array([1.0, 0.5, 0.5]), c, 0.25) == pytest.approx(-0.25 ** 3 / 3 / 0.5)


def test_uniform_sphere_c1_against_analytic():
    """32^3, lmax = 4: relative L2 error below 5% and falling with h."""
    errs = []
    for n in (32, 64):
        grid = CartGrid(n=n, g=1)
        rho = uniform_sphere(grid).numpy()
        phi = _solve(rho, n, 1, 2, 4)
        ref = A.uniform_sphere(_interior_points(n, 1), (0.5, 0.5, 0.5), 0.25)
        s = slice(1, n)
        errs.append(np.linalg.norm(phi[s, s, s] - ref) / np.linalg.norm(ref))
    assert errs[0] < 0.05
    assert errs[1] < errs[0]


def test_gaussian_clump_second_order_7pt():
    """A centred Gaussian clump: 7-point error falls by ~4 per halving of h."""
    cl = Clumps(np.array([[0.5, 0.5, 0.5]]), np.array([0.08]), np.array([1.3]))
    errs = []
    for n in (16, 32, 64):
        grid = CartGrid(n=n, g=1)
        rho = clump_density(grid, cl).numpy()
        phi = _solve(rho, n, 1, 2, 8)
        ref = A.gaussian_clump(_interior_points(n, 1), (0.5, 0.5, 0.5), 0.08, 1.3)
        s = slice(1, n)
        errs.append(np.max(np.abs(phi[s, s, s] - ref)))
    assert 3.3 < errs[0] / errs[1] < 4.7
    assert 3.6 < errs[1] / errs[2] < 4.4


def test_gaussian_clump_high_order_19pt():
    """The 19-point star converges far faster than 2nd order."""
    cl = Clumps(np.array([[0.5, 0.5, 0.5]]), np.array([0.08]), np.array([1.0]))
    errs = []
    for n in (16, 32):
        grid = CartGrid(n=n, g=3)
        rho = clump_density(grid, cl).numpy()
        phi = _solve(rho, n, 3, 6, 8)
        ref = A.gaussian_clump(_interior_points(n, 3), (0.5, 0.5, 0.5), 0.08, 1.0)
        s = slice(3, 3 + n - 1)
        errs.append(np.max(np.abs(phi[s, s, s] - ref)))
    assert errs[0] / errs[1] > 25


def test_smooth_sphere_mass_and_radial_equation():
    """Section 3.1: M = (32 pi/105) rho_p a^3 for (1-w^2)^2, and the quoted
    potential solves (1/r^2)(r^2 Phi')' = 4 pi G rho with -GM/d outside
    (reading d = |x - x_p|)."""
    a, mass = 0.08, 2.0
    rho_p = mass / (32 * math.pi / 105 * a ** 3)
    m_int, _ = quad(lambda r: 4 * math.pi * r * r * rho_p * (1 - (r / a) ** 2) ** 2, 0, a)
    assert m_int == pytest.approx(mass, rel=1e-12)
    e = 1e-5
    for r in (0.2 * a, 0.5 * a, 0.9 * a, 1.5 * a):
        f = lambda rr: float(A.smooth_sphere(np.array([rr, 0, 0]), (0, 0, 0), a, mass))
        d1p = (f(r + e) - f(r)) / e
        d1m = (f(r) - f(r - e)) / e
        lap = ((r + e / 2) ** 2 * d1p - (r - e / 2) ** 2 * d1m) / (e * r * r)
        rho = rho_p * (1 - (r / a) ** 2) ** 2 if r < a else 0.0
        assert lap == pytest.approx(rho, rel=2e-4, abs=2e-3 * rho_p)
    # continuity at the surface
    assert float(A.smooth_sphere(np.array([a * (1 - 1e-12), 0, 0]), (0, 0, 0), a, mass)) == pytest.approx(
        -mass / (4 * math.pi * a), rel=1e-9)


def test_two_smooth_spheres_on_unit_box():
    """The paper's two-sphere test shrunk onto [0,1]^3 (centres on the z axis
    through the box centre): 2nd-order agreement with the analytic sum."""
    errs = []
    for n in (32, 64):
        grid = CartGrid(n=n, g=1)
        c1, c2 = (0.5, 0.5, 0.7), (0.5, 0.5, 0.4)
        rho = (smooth_sphere(grid, c1, 0.08, 1.0) + smooth_sphere(grid, c2, 0.08, 2.0)).numpy()
        phi = _solve(rho, n, 1, 2, 8)
        pts = _interior_points(n, 1)
        ref = A.smooth_sphere(pts, c1, 0.08, 1.0) + A.smooth_sphere(pts, c2, 0.08, 2.0)
        s = slice(1, n)
        errs.append(np.max(np.abs(phi[s, s, s] - ref)) / np.max(np.abs(ref)))
    assert errs[0] < 0.05
    assert errs[1] < errs[0] / 2.5


def test_sis_on_log_spherical_grid():
    """Truncated SIS (no perturbation): the exact discrete solution with the
    inner expansion + central point mass and the outer expansion at the
    ghost shells approaches ln(r/0.8) - 1 inside r < 0.8; the error, set by
    the density jump at r = 0.8, falls as the radial grid is refined."""
    errs = []
    for nr in (96, 192):
        nth, nph = 32, 32
        r, th, ph, ds = M.sph_axes(nr, nth, nph)
        rho = np.zeros((nph, nth, nr + 2))
        rho[:, :, 1:nr + 1] = np.where(r[1:nr + 1] < 0.8, 1.0 / r[1:nr + 1] ** 2, 0.0)[None, None, :]
        core = 4 * math.pi * r[1]   # mass of the excised core r < r_min as a central point
        ghost, q, qb = M.sph_boundary(rho, nr, nth, nph, 8, point_mass=core)
        # midpoint quadrature in theta leaves only small l > 0 moments
        assert np.max(np.abs(q[1:])) < 1e-2 * q[0]
        phi = D.solve_sph(ghost, rho, r, ds, th)
        ref = A.sis(r[1:nr + 1])
        errs.append(np.max(np.abs(phi[:, :, 1:nr + 1] - ref[None, None, :])) / np.max(np.abs(ref)))
    assert errs[0] < 5e-3
    assert errs[1] < 0.5 * errs[0]
