"""Pins for the oracle's multipole moments and ghost potential (Section 2.2)."""
import math

import numpy as np
import pytest

from oracle import harmonics as H
from oracle import multipole as M
from workloads import CartGrid, uniform_sphere

G = 1.0 / (4 * math.pi)


def _points(rng, n, rmax):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d * rmax * rng.uniform(0.1, 1.0, size=(n, 1)) ** (1 / 3)


def test_low_order_moments_are_mass_dipole_quadrupole():
    rng = np.random.default_rng(0)
    x = _points(rng, 200, 0.3)
    m = rng.uniform(0.1, 1.0, 200)
    q = M.moments_outer(4, x, m)
    assert q[H.idx(0, 0)] == pytest.approx(m.sum(), rel=1e-14)
    np.testing.assert_allclose(q[H.idx(1, 0)], np.sum(m * x[:, 2]), rtol=1e-12)
    np.testing.assert_allclose(q[H.idx(1, 1)], np.sum(m * x[:, 0]), rtol=1e-12)
    np.testing.assert_allclose(q[H.idx(1, -1)], np.sum(m * x[:, 1]), rtol=1e-12)
    r2 = np.sum(x * x, axis=1)
    np.testing.assert_allclose(q[H.idx(2, 0)], np.sum(m * (3 * x[:, 2] ** 2 - r2) / 2), rtol=1e-12)


@pytest.mark.parametrize("lmax", [0, 2, 4, 8])
def test_outer_expansion_within_legendre_tail_bound(lmax):
    """Point masses inside radius a, field points at r > a: the truncated
    expansion differs from -G sum m/|x-x'| by at most
    G sum m (r'/r)^(lmax+1) / (r - r')."""
    rng = np.random.default_rng(1)
    x = _points(rng, 50, 0.3)
    m = rng.uniform(0.1, 1.0, 50)
    q = M.moments_outer(lmax, x, m)
    d = rng.normal(size=(40, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    f = d * rng.uniform(0.5, 1.5, size=(40, 1))
    phi = M.phi_outer(q, lmax, f, G)
    exact = -G * np.sum(m[None, :] / np.linalg.norm(f[:, None, :] - x[None, :, :], axis=2), axis=1)
    r = np.linalg.norm(f, axis=1)
    rp = np.linalg.norm(x, axis=1)
    bound = G * np.sum(m[None, :] * (rp[None, :] / r[:, None]) ** (lmax + 1)
                       / (r[:, None] - rp[None, :]), axis=1)
    assert np.all(np.abs(phi - exact) <= bound * (1 + 1e-9) + 1e-15)
    if lmax == 8:
        assert np.max(np.abs(phi - exact) / np.abs(exact)) < 1e-3


@pytest.mark.parametrize("lmax", [2, 8])
def test_inner_expansion_within_tail_bound(lmax):
    rng = np.random.default_rng(2)
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    x = d * rng.uniform(0.6, 1.0, size=(50, 1))
    m = rng.uniform(0.1, 1.0, 50)
    qb = M.moments_inner(lmax, x, m)
    f = _points(rng, 30, 0.3)
    phi = M.phi_inner(qb, lmax, f, G)
    exact = -G * np.sum(m[None, :] / np.linalg.norm(f[:, None, :] - x[None, :, :], axis=2), axis=1)
    r = np.linalg.norm(f, axis=1)
    rp = np.linalg.norm(x, axis=1)
    bound = G * np.sum(m[None, :] * (r[:, None] / rp[None, :]) ** (lmax + 1)
                       / (rp[None, :] - r[:, None]), axis=1)
    assert np.all(np.abs(phi - exact) <= bound * (1 + 1e-9) + 1e-15)


def test_centred_voxel_sphere_has_cubic_symmetry():
    """A sphere sampled on a grid centred on the expansion origin has the
    cube's symmetry, so its l = 1, 2, 3 moments vanish; q_00 is its mass."""
    grid = CartGrid(n=32, g=1)
    rho = uniform_sphere(grid).numpy()
    q = M.cart_moments(rho, 32, 1, 4)
    mass = rho[1:32, 1:32, 1:32].sum() / 32 ** 3
    assert q[0] == pytest.approx(mass, rel=1e-13)
    assert np.max(np.abs(q[1:16])) < 1e-14 * mass
    assert np.max(np.abs(q[16:25])) > 1e-6 * mass   # l = 4 cubic harmonic survives


def test_cartesian_ghosts_match_point_sum_for_sparse_density():
    """Two isolated nonzero nodes: the ghost layer equals the truncated
    expansion of two point masses, checked against the direct sum within the
    tail bound (lmax = 8)."""
    n = 16
    rho = np.zeros((n + 1,) * 3)
    rho[7, 8, 9] = 3.0
    rho[9, 6, 8] = 1.0
    phi, q = M.cart_boundary(rho, n, 1, 8)
    h = 1.0 / n
    src = np.array([[9 * h, 8 * h, 7 * h], [8 * h, 6 * h, 9 * h]]) - 0.5
    mass = np.array([3.0, 1.0]) * h ** 3
    x = np.arange(n + 1) * h - 0.5
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    mask = M.cart_ghost_mask(n, 1)
    pts = np.stack([X[mask], Y[mask], Z[mask]], axis=-1)
    exact = -G * np.sum(mass[None, :] / np.linalg.norm(pts[:, None] - src[None], axis=2), axis=1)
    r = np.linalg.norm(pts, axis=1)
    rp = np.linalg.norm(src, axis=1)
    bound = G * np.sum(mass[None, :] * (rp[None, :] / r[:, None]) ** 9 / (r[:, None] - rp[None, :]), axis=1)
    assert np.all(np.abs(phi[mask] - exact) <= bound * (1 + 1e-9) + 1e-16)
    assert np.all(phi[~mask] == 0.0)


def test_spherical_boundary_point_mass_shells():
    """Spherical grid with density at a single node: the outer ghost shell is
    the outer expansion and the inner shell the inner expansion of that
    point, plus the central point mass."""
    nr, nth, nph = 12, 6, 8
    r, th, ph, ds = M.sph_axes(nr, nth, nph)
    rho = np.zeros((nph, nth, nr + 2))
    k, j, i = 3, 2, 6
    rho[k, j, 1 + i] = 5.0
    mc = 0.7
    phi, q, qb = M.sph_boundary(rho, nr, nth, nph, 8, point_mass=mc)
    w = r[1 + i] ** 3 * ds * math.sin(th[j]) * (math.pi / nth) * (2 * math.pi / nph)
    src = M.sph_points(np.array([r[1 + i]]), np.array([th[j]]), np.array([ph[k]])).reshape(1, 3)
    outer = M.sph_points(r[-1:], th, ph)[:, :, 0, :]
    inner = M.sph_points(r[:1], th, ph)[:, :, 0, :]
    d_out = np.linalg.norm(outer - src[0], axis=-1)
    d_in = np.linalg.norm(inner - src[0], axis=-1)
    exact_out = -G * (5.0 * w / d_out + mc / r[-1])
    exact_in = -G * (5.0 * w / d_in + mc / r[0])
    np.testing.assert_allclose(phi[:, :, -1], exact_out, rtol=1e-3)
    np.testing.assert_allclose(phi[:, :, 0], exact_in, rtol=1e-9)
    assert q[0] == pytest.approx(5.0 * w + mc, rel=1e-14)
