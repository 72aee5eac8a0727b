"""Pins for the oracle's exact solves and kernel-level references."""
import itertools
import math

import numpy as np
import pytest

from oracle import direct as D
from oracle import multipole as M
from oracle import operators as O
from oracle import smoothers as S


def _random_problem(n, g, seed):
    rng = np.random.default_rng(seed)
    m = n + 1 + 2 * (g - 1)
    phi = rng.normal(size=(m, m, m))
    s = slice(g, g + n - 1)
    phi[s, s, s] = 0.0
    rho = rng.normal(size=(m, m, m))
    return phi, rho


@pytest.mark.parametrize("n", [8, 9])
def test_dst_solve_equals_dense_lapack(n):
    phi, rho = _random_problem(n, 1, n)
    a = D.solve_cart(phi, rho, n, 1.0 / n, 2, 1)
    b = D.dense_solve_cart(phi, rho, n, 1.0 / n, 2, 1)
    np.testing.assert_allclose(a, b, atol=1e-12 * np.max(np.abs(b)))


def test_pcg19_equals_dense_lapack():
    n = 8
    phi, rho = _random_problem(n, 3, 5)
    a = D.solve_cart(phi, rho, n, 1.0 / n, 6, 3)
    b = D.dense_solve_cart(phi, rho, n, 1.0 / n, 6, 3)
    np.testing.assert_allclose(a, b, atol=1e-11 * np.max(np.abs(b)))


def test_pcg19_iteration_count_reflects_spectral_bound():
    n = 32
    rng = np.random.default_rng(1)
    rhs = rng.normal(size=(n - 1,) * 3)
    u, it, rel = D.pcg19(rhs, n, 1.0 / n)
    assert rel < 1e-13
    assert it <= 25


def test_dst_sine_mode_solution():
    n = 16
    h = 1.0 / n
    x = np.arange(1, n) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    k = (3, 1, 2)
    mode = np.sin(np.pi * k[0] * X) * np.sin(np.pi * k[1] * Y) * np.sin(np.pi * k[2] * Z)
    lam = sum((2 * math.cos(math.pi * kk * h) - 2) / h ** 2 for kk in k)
    np.testing.assert_allclose(D.dst_solve7(mode, n, h), mode / lam, atol=1e-14)


def test_spherical_per_mode_lu_equals_dense():
    nr, nth, nph = 5, 4, 8
    r, th, ph, ds = M.sph_axes(nr, nth, nph)
    rng = np.random.default_rng(3)
    phi = np.zeros((nph, nth, nr + 2))
    phi[:, :, 0] = rng.normal(size=(nph, nth))
    phi[:, :, -1] = rng.normal(size=(nph, nth))
    rho = rng.normal(size=(nph, nth, nr + 2))
    a = D.solve_sph(phi, rho, r, ds, th)
    b = D.dense_solve_sph(phi, rho, r, ds, th)
    np.testing.assert_allclose(a, b, atol=1e-11 * np.max(np.abs(b)))
    res = O.sph_residual(a, rho, r, ds, th)
    assert np.max(np.abs(res)) < 1e-8 * np.max(np.abs(O.sph_rhs(rho, r)))


# ------------------------------------------------------------ colour passes
def _sequential_rb(u, f, n, h, colour, omega):
    """Brute force: visit the nodes of one colour one at a time."""
    u = u.copy()
    for k, j, i in itertools.product(range(1, n), repeat=3):
        if (i + j + k) % 2 != colour:
            continue
        s = u[k, j, i + 1] + u[k, j, i - 1] + u[k, j + 1, i] + u[k, j - 1, i] + u[k + 1, j, i] + u[k - 1, j, i]
        u[k, j, i] = (1 - omega) * u[k, j, i] + omega * (s - h * h * f[k, j, i]) / 6.0
    return u


def _sequential_star(u, f, n, h, colour):
    g = 3
    c = O.STAR6
    u = u.copy()
    for k, j, i in itertools.product(range(1, n), repeat=3):
        if (i + j + k) % 4 != colour:
            continue
        K, J, I = k + g - 1, j + g - 1, i + g - 1
        s = 0.0
        for q in (1, 2, 3):
            s += c[q] * (u[K, J, I + q] + u[K, J, I - q] + u[K, J + q, I] + u[K, J - q, I]
                         + u[K + q, J, I] + u[K - q, J, I])
        u[K, J, I] = (h * h * f[K, J, I] - s) / (3 * c[0])
    return u


@pytest.mark.parametrize("colour,omega", [(0, 1.0), (1, 1.0), (0, 1.7), (1, 0.6)])
def test_rb_pass_equals_sequential_loop(colour, omega):
    n = 6
    rng = np.random.default_rng(colour)
    u = rng.normal(size=(n + 1,) * 3)
    f = rng.normal(size=(n + 1,) * 3)
    ref = _sequential_rb(u, f, n, 1.0 / n, colour, omega)
    out = S.rb_pass(u.copy(), f, n, 1.0 / n, colour, omega)
    np.testing.assert_allclose(out, ref, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("colour", [0, 1, 2, 3])
def test_star_pass_equals_sequential_loop(colour):
    n = 7
    m = n + 5
    rng = np.random.default_rng(10 + colour)
    u = rng.normal(size=(m, m, m))
    f = rng.normal(size=(m, m, m))
    ref = _sequential_star(u, f, n, 1.0 / n, colour)
    out = S.star_pass(u.copy(), f, n, 1.0 / n, colour)
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("order", [2, 6])
def test_exact_solution_is_a_fixed_point_of_the_smoother(order):
    n = 16
    g = 1 if order == 2 else 3
    phi, rho = _random_problem(n, g, 7)
    sol = D.solve_cart(phi, rho, n, 1.0 / n, order, g)
    out = S.smooth(sol.copy(), rho, n, 1.0 / n, order, g)
    assert np.max(np.abs(out - sol)) < 1e-11 * np.max(np.abs(sol))


# ------------------------------------------------------------ transfers
def test_restriction_keeps_constants_and_is_adjoint_to_prolongation():
    n = 16
    nc = n // 2
    rng = np.random.default_rng(4)
    np.testing.assert_allclose(S.restrict(np.full((n - 1,) * 3, 2.5)), 2.5, rtol=1e-15)
    u = rng.normal(size=(n - 1,) * 3)
    v = rng.normal(size=(nc - 1,) * 3)
    assert 8 * np.vdot(S.restrict(u), v) == pytest.approx(np.vdot(u, S.prolong(v)), rel=1e-13)


def test_restriction_brute_force():
    n = 8
    rng = np.random.default_rng(5)
    r = rng.normal(size=(n - 1,) * 3)
    out = S.restrict(r)
    w = {-1: 0.25, 0: 0.5, 1: 0.25}
    for K, J, I in itertools.product(range(1, n // 2), repeat=3):
        s = 0.0
        for a, b, c in itertools.product((-1, 0, 1), repeat=3):
            s += w[a] * w[b] * w[c] * r[2 * K + a - 1, 2 * J + b - 1, 2 * I + c - 1]
        assert out[K - 1, J - 1, I - 1] == pytest.approx(s, rel=1e-14, abs=1e-15)


def test_prolongation_reproduces_trilinear_functions():
    nc = 8
    n = 2 * nc
    X = np.arange(1, nc)
    Kc, Jc, Ic = np.meshgrid(X, X, X, indexing="ij")
    f = lambda i, j, k: 1.0 + 0.5 * i - 0.25 * j + 2.0 * k + 0.1 * i * j * k
    e = f(Ic * 2.0, Jc * 2.0, Kc * 2.0)
    fine = S.prolong(e)
    x = np.arange(1, n)
    K, J, I = np.meshgrid(x, x, x, indexing="ij")
    ref = f(I * 1.0, J * 1.0, K * 1.0)
    inner = slice(1, n - 2)   # fine nodes 2..n-2 never touch the coarse boundary
    np.testing.assert_allclose(fine[inner, inner, inner], ref[inner, inner, inner], rtol=1e-13)


@pytest.mark.parametrize("order", [2, 6])
def test_vcycle_fixed_point_and_contraction(order):
    n = 32
    g = 1 if order == 2 else 3
    phi, rho = _random_problem(n, g, 9)
    sol = D.solve_cart(phi, rho, n, 1.0 / n, order, g)
    u = S.vcycle(sol.copy(), rho, n, 1.0 / n, order, g)
    assert np.max(np.abs(u - sol)) < 1e-11 * np.max(np.abs(sol))
    u = phi.copy()
    r0 = np.linalg.norm(O.residual(u, rho, n, 1.0 / n, order, g))
    cache = {}
    for _ in range(6):
        S.vcycle(u, rho, n, 1.0 / n, order, g, _cache=cache)
    r6 = np.linalg.norm(O.residual(u, rho, n, 1.0 / n, order, g))
    assert (r6 / r0) ** (1 / 6) < 0.2


def test_sor_omegas():
    assert S.omega_opt(32) == pytest.approx(1.821465, abs=1e-6)
    assert S.omega_opt_a(32) == pytest.approx(1.821204, abs=1e-6)
    w = S.omega_chebyshev(32, 200)
    assert w[0] == pytest.approx(1.0 / (1.0 - math.cos(math.pi / 32) ** 2 / 2))
    assert w[-1] == pytest.approx(S.omega_opt(32), rel=1e-6)
    assert all(a > b for a, b in zip(w[1:40], w[2:41]))  # decreasing towards omega_opt
