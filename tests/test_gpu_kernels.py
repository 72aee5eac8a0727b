"""Kernel-level parity of the HIP path against the oracle's plain loops
(single operators through the C ABI, FP64, sizes spanning several tiles and
ragged tails)."""
import math

import numpy as np
import pytest
import torch

import paper_2605_03563_amd as pg
from oracle import multipole as OM
from oracle import operators as OO
from oracle import smoothers as OS
from tests.gpu_util import dev, host, random_cart, rel_l2, rel_max, say
from workloads import CartGrid, draw_clumps, clump_density, uniform_sphere

pytestmark = pytest.mark.gpu
KTOL = 1e-13   # kernel-level FP64 parity (relative to the max magnitude)


def _plan(n, order=2, method="cg", **kw):
    g = 1 if order == 2 else 3
    return pg.Plan(pg.cart_grid(n, ghost=g), pg.options(method, order=order, lmax=-1, **kw)), g


@pytest.mark.parametrize("n,order", [(16, 2), (21, 2), (70, 2), (16, 6), (23, 6), (131, 6)])
def test_apply(n, order):
    say(f"apply n={n} order={order}")
    plan, g = _plan(n, order)
    rng = np.random.default_rng(n + order)
    m = n + 1 + 2 * (g - 1)
    u = rng.normal(size=(m, m, m))
    out = torch.zeros((m, m, m), dtype=torch.float64, device="cuda:0")
    plan.apply(dev(u), out)
    ref = OO.lap(u, n, 1.0 / n, order, g)
    s = slice(g, g + n - 1)
    assert rel_max(host(out)[s, s, s], ref) < KTOL


@pytest.mark.parametrize("n,order", [(33, 2), (24, 6), (128, 6), (131, 6), (130, 2)])
def test_residual_and_norm(n, order):
    """n >= 128 takes the large-level launch shapes (eight planes per thread,
    the 19-point residual's register window); 131 and 130 end in partial
    tiles and partial plane runs."""
    say(f"residual n={n} order={order}")
    plan, g = _plan(n, order)
    phi, rho = random_cart(n, g, 3)
    rng = np.random.default_rng(5)
    s = slice(g, g + n - 1)
    phi[s, s, s] = rng.normal(size=(n - 1,) * 3)
    res = torch.zeros_like(dev(phi))
    n2 = plan.residual(dev(rho), dev(phi), res)
    ref = OO.residual(phi, rho, n, 1.0 / n, order, g)
    assert rel_max(host(res)[s, s, s], ref) < KTOL
    assert n2 == pytest.approx(float(np.sum(ref * ref)), rel=1e-12)


@pytest.mark.parametrize("n,omega,forward", [(16, 1.0, True), (16, 1.0, False), (21, 1.7, True), (66, 1.0, True)])
def test_red_black_sweep(n, omega, forward):
    say(f"rb sweep n={n} omega={omega} forward={forward}")
    plan, g = _plan(n, 2)
    phi, rho = random_cart(n, g, 7)
    t = dev(phi)
    plan.smooth(dev(rho), t, sweeps=2, forward=forward, omega=omega)
    ref = phi.copy()
    for _ in range(2):
        for c in ((0, 1) if forward else (1, 0)):
            OS.rb_pass(ref, rho, n, 1.0 / n, c, omega, g)
    assert rel_max(host(t), ref) < KTOL


@pytest.mark.parametrize("n,forward", [(16, True), (19, False), (40, True), (128, True), (131, False)])
def test_four_colour_sweep(n, forward):
    """n >= 128: eight planes per thread, as on the large multigrid levels."""
    say(f"4-colour sweep n={n} forward={forward}")
    plan, g = _plan(n, 6)
    phi, rho = random_cart(n, g, 11)
    t = dev(phi)
    plan.smooth(dev(rho), t, sweeps=1, forward=forward)
    ref = OS.smooth(phi.copy(), rho, n, 1.0 / n, 6, g, forward=forward)
    assert rel_max(host(t), ref) < KTOL


def test_four_colour_pass_and_residual_at_511():
    """The 512-interval level in the launch configuration of the benchmark
    (two FP64 compact columns per lane, 16-plane runs, in-block neighbours
    from LDS; residual blocks from compact column 1 plus the column-0 kernel):
    one forward four-colour sweep and the residual with its norm, element by
    element against the oracle."""
    n, g = 512, 3
    say(f"4-colour sweep and residual at n={n}")
    plan = pg.Plan(pg.cart_grid(n, ghost=g), pg.options("mg", order=6, lmax=-1))
    phi, rho = random_cart(n, g, 23)
    t = dev(phi)
    r = dev(rho)
    plan.smooth(r, t, sweeps=1, forward=True)
    got = host(t)
    say("  oracle sweep")
    ref = OS.smooth(phi, rho, n, 1.0 / n, 6, g, forward=True)
    assert rel_max(got, ref) < KTOL
    del phi, got
    res = torch.zeros_like(t)
    n2 = plan.residual(r, t, res)
    say("  oracle residual")
    rref = OO.residual(ref, rho, n, 1.0 / n, 6, g)
    s = slice(g, g + n - 1)
    assert rel_max(host(res)[s, s, s], rref) < KTOL
    assert n2 == pytest.approx(float(np.sum(rref * rref)), rel=1e-12)


@pytest.mark.parametrize("order,n", [(2, 64), (2, 256), (6, 64), (6, 128), (6, 192), (6, 256), (6, 512)])
def test_restricted_residual(order, n):
    """R (f - L phi) and the fine residual's sum of squares against the
    oracle's residual followed by its full weighting.  On the four-colour
    levels from 128 intervals one fused kernel forms both (n = 192: partial
    blocks along x, y and z; n = 512: the launch configuration of the 511^3
    solve's cycle head, here restricting every colour)."""
    say(f"restricted residual n={n} order={order}")
    plan, g = _plan(n, order, method="mg", **({"coarsest": 6} if n == 192 else {}))
    phi, rho = random_cart(n, g, 29)
    rng = np.random.default_rng(31)
    s = slice(g, g + n - 1)
    phi[s, s, s] = rng.normal(size=(n - 1,) * 3)
    coarse = torch.zeros((n // 2 - 1,) * 3, dtype=torch.float64, device="cuda:0")
    n2 = plan.restrict_residual(dev(rho), dev(phi), coarse)
    rref = OO.residual(phi, rho, n, 1.0 / n, order, g)
    del phi, rho
    assert n2 == pytest.approx(float(np.sum(rref * rref)), rel=1e-12)
    cref = OS.restrict(rref)
    del rref
    assert rel_max(host(coarse), cref) < KTOL


# FP32 kernels against the oracle in FP64 on the same FP32-rounded inputs:
# each residual sums up to 19 rounded terms of |c_k phi / h^2| and full
# weighting 27 more; with unit roundoff 6e-8 and terms a few times the
# result, the error stays below about 50 * 6e-8 * 3 of the largest value.
F32TOL = 1e-5


@pytest.mark.parametrize("order,n", [(2, 64), (2, 256), (6, 64), (6, 128), (6, 192), (6, 256), (6, 512)])
def test_restricted_residual_fp32(order, n):
    """The mixed plan's FP32 residual and restriction (the inner cycles'
    kernels; from 128 intervals the fused kernel, at n = 512 in the launch
    configuration of the 511^3 mixed solve) against the oracle's residual
    and full weighting of the same FP32-rounded Phi and rho, and the FP64
    sum of squares of the FP32 residuals."""
    say(f"restricted residual FP32 n={n} order={order}")
    plan, g = _plan(n, order, method="mg_ir32", **({"coarsest": 6} if n == 192 else {}))
    phi, rho = random_cart(n, g, 37)
    rng = np.random.default_rng(41)
    s = slice(g, g + n - 1)
    phi[s, s, s] = rng.normal(size=(n - 1,) * 3)
    coarse = torch.zeros((n // 2 - 1,) * 3, dtype=torch.float64, device="cuda:0")
    n2 = plan.restrict_residual(dev(rho), dev(phi), coarse)
    phi = phi.astype(np.float32).astype(np.float64)
    rho = rho.astype(np.float32).astype(np.float64)
    rref = OO.residual(phi, rho, n, 1.0 / n, order, g)
    del phi, rho
    assert n2 == pytest.approx(float(np.sum(rref * rref)), rel=F32TOL)
    cref = OS.restrict(rref)
    del rref
    assert rel_max(host(coarse), cref) < F32TOL


@pytest.mark.parametrize("order,n", [(2, 16), (2, 64), (2, 96), (6, 16), (6, 64), (6, 96), (6, 128), (6, 256)])
def test_restrict_and_prolong(order, n):
    """Full weighting and trilinear prolongation on the two-colour (7-point)
    and four-colour (19-point) level layouts; n = 96 (coarsest 6) has ragged
    tiles (on the four-colour levels a last column group with one column of
    unknowns), n = 128 and 256 the plane runs of the large levels."""
    say(f"transfers order={order} n={n}")
    g = 1 if order == 2 else 3
    plan = pg.Plan(pg.cart_grid(n, ghost=g), pg.options("mg", order=order, lmax=-1, coarsest=6 if n == 96 else 8))
    rng = np.random.default_rng(n)
    fine = rng.normal(size=(n - 1,) * 3)
    coarse = torch.zeros((n // 2 - 1,) * 3, dtype=torch.float64, device="cuda:0")
    plan.restrict(dev(fine), coarse)
    assert rel_max(host(coarse), OS.restrict(fine)) < KTOL
    ec = rng.normal(size=(n // 2 - 1,) * 3)
    tf = dev(fine)
    plan.prolong_add(dev(ec), tf)
    assert rel_max(host(tf), fine + OS.prolong(ec)) < KTOL


@pytest.mark.parametrize("order,n", [(2, 32), (2, 64), (2, 96), (2, 128), (2, 256), (6, 32), (6, 96),
                                     (6, 128), (6, 256)])
def test_one_vcycle_matches_reference_cycle(order, n):
    """One V(2,2) cycle against the oracle's cycle; n = 96 has ragged tiles,
    n = 128 and 256 take the large-level shapes of the fused residual and
    restriction (7-point) and of the four-colour passes and residual
    (19-point star, Section 2.1.2)."""
    say(f"one V(2,2) cycle order={order} n={n}")
    g = 1 if order == 2 else 3
    coarsest = 6 if n == 96 else 8
    plan = pg.Plan(pg.cart_grid(n, ghost=g), pg.options("mg", order=order, lmax=-1, coarsest=coarsest))
    phi, rho = random_cart(n, g, 13)
    t = dev(phi)
    plan.vcycle(dev(rho), t, cycles=1)
    ref = OS.vcycle(phi.copy(), rho, n, 1.0 / n, order, g, coarsest=coarsest)
    assert rel_max(host(t), ref) < 1e-12


# ------------------------------------------------------------ multipole
def _ghost_mask(n, g):
    return OM.cart_ghost_mask(n, g)


@pytest.mark.parametrize("case", ["c1_sphere_lmax4", "clumps_n64_lmax8", "clumps_g3_lmax6"])
def test_cartesian_multipole(case):
    say(f"multipole {case}")
    if case == "c1_sphere_lmax4":
        n, g, lmax = 32, 1, 4
        rho = uniform_sphere(CartGrid(n, g)).numpy()
    elif case == "clumps_n64_lmax8":
        n, g, lmax = 64, 1, 8
        rho = clump_density(CartGrid(n, g), draw_clumps(np.random.default_rng(2), 16)).numpy()
    else:
        n, g, lmax = 40, 3, 6
        rho = clump_density(CartGrid(n, g), draw_clumps(np.random.default_rng(3), 5)).numpy()
    plan = pg.Plan(pg.cart_grid(n, ghost=g), pg.options("cg", order=2 if g == 1 else 6, lmax=lmax))
    phi = torch.zeros(rho.shape, dtype=torch.float64, device="cuda:0")
    q = np.array(plan.multipole_boundary(dev(rho), phi, lmax))
    ref_phi, ref_q = OM.cart_boundary(rho, n, g, lmax)
    assert rel_max(q, ref_q) < 1e-12
    mask = _ghost_mask(n, g)
    got = host(phi)
    assert rel_max(got[mask], ref_phi[mask]) < 1e-12
    assert np.all(got[~mask] == 0.0)


def test_spherical_multipole():
    say("multipole spherical")
    nr, nth, nph, lmax = 24, 12, 16, 8
    r, th, ph, ds = OM.sph_axes(nr, nth, nph)
    rng = np.random.default_rng(4)
    rho = np.zeros((nph, nth, nr + 2))
    rho[:, :, 1:nr + 1] = rng.uniform(0, 1, size=(nph, nth, nr)) / r[1:nr + 1] ** 2
    mc = 0.3
    plan = pg.Plan(pg.sph_grid(nr, nth, nph), pg.options("bicgstab", lmax=lmax, point_mass=mc))
    phi = torch.zeros(rho.shape, dtype=torch.float64, device="cuda:0")
    q = np.array(plan.multipole_boundary(dev(rho), phi, lmax))
    ref_phi, rq, rqb = OM.sph_boundary(rho, nr, nth, nph, lmax, point_mass=mc)
    nq = (lmax + 1) ** 2
    assert rel_max(q[:nq], rq) < 1e-12
    assert rel_max(q[nq:], rqb) < 1e-12
    got = host(phi)
    assert rel_max(got[:, :, 0], ref_phi[:, :, 0]) < 1e-12
    assert rel_max(got[:, :, -1], ref_phi[:, :, -1]) < 1e-12


def test_spherical_apply():
    say("spherical apply")
    nr, nth, nph = 40, 16, 32
    r, th, ph, ds = OM.sph_axes(nr, nth, nph)
    plan = pg.Plan(pg.sph_grid(nr, nth, nph), pg.options("bicgstab", lmax=-1))
    u = np.random.default_rng(9).normal(size=(nph, nth, nr + 2))
    out = torch.zeros(u.shape, dtype=torch.float64, device="cuda:0")
    plan.apply(dev(u), out)
    assert rel_max(host(out)[:, :, 1:nr + 1], OO.sph_apply(u, ds, th)) < KTOL


@pytest.mark.parametrize("dims", [(32, 16, 32), (20, 8, 48)])
def test_spherical_preconditioner_cycle_matches_oracle(dims):
    """One FP32 V(2,2) cycle of the spherical multigrid preconditioner against
    the oracle's FP64 cycle on a random right-hand side (48 = 3 x 16: phi
    lines of three segments on the fine level; 20 x 8 x 48 coarsens twice)."""
    from oracle import sph_mg as SM
    nr, nth, nph = dims
    say(f"spherical preconditioner cycle {dims}")
    r, th, ph, ds = OM.sph_axes(nr, nth, nph)
    plan = pg.Plan(pg.sph_grid(nr, nth, nph), pg.options("bicgstab_mg32", lmax=-1))
    rng = np.random.default_rng(sum(dims))
    y = np.zeros((nph, nth, nr + 2))
    y[:, :, 1:nr + 1] = rng.standard_normal((nph, nth, nr))
    yhat = torch.zeros(y.shape, dtype=torch.float64, device="cuda:0")
    plan.precond(dev(y), yhat)
    ref = SM.vcycle(y[:, :, 1:nr + 1], ds)
    got = host(yhat)[:, :, 1:nr + 1]
    say(f"  rel L2 {rel_l2(got, ref):.2e}")
    assert rel_l2(got, ref) < 1e-5   # FP32 cycle against the FP64 oracle
