"""Converged parity of every solver path against the oracle's exact discrete
solution (relative L2 error <= 1e-10 once the residual is driven to round-off
level), error paths, and determinism."""
import functools
import math

import numpy as np
import pytest
import torch

import paper_2605_03563_amd as pg
from oracle import analytic as OA
from oracle import direct as OD
from oracle import multipole as OM
from tests.gpu_util import dev, host, rel_l2, say
import workloads as W

pytestmark = pytest.mark.gpu
CONV_TOL = 1e-10   # converged parity bar (relative L2 potential error)


def _oracle_cart(rho, n, g, order, lmax):
    ghost, _ = OM.cart_boundary(rho, n, g, lmax)
    return OD.solve_cart(ghost, rho, n, 1.0 / n, order, g)


def _solve(n, g, method, order, rho, lmax, tol, **kw):
    plan = pg.Plan(pg.cart_grid(n, ghost=g), pg.options(method, order=order, lmax=lmax, **kw))
    phi = torch.zeros(rho.shape, dtype=torch.float64, device="cuda:0")
    res = plan.solve(dev(rho), phi, tol=tol, history=4096)
    return host(phi), res


@pytest.mark.parametrize("method,kw", [("sor", {}), ("sor", {"omega_mode": pg.OMEGA_CHEBYSHEV}),
                                       ("cg", {})])
def test_c1_uniform_sphere(method, kw):
    say(f"C1 32^3 uniform sphere {method} {kw}")
    n, g, lmax = 32, 1, 4
    wl = W.config_c1()
    rho = wl.rho.numpy()
    phi, res = _solve(n, g, method, 2, rho, lmax, 1e-13, **kw)
    assert res.converged, res
    ref = _oracle_cart(rho, n, g, 2, lmax)
    s = slice(1, n)
    assert rel_l2(phi[s, s, s], ref[s, s, s]) < CONV_TOL
    mask = OM.cart_ghost_mask(n, g)
    assert np.max(np.abs(phi[mask] - ref[mask])) < 1e-12 * np.max(np.abs(ref[mask]))
    # against the analytic potential (informational bar from the staircase sphere)
    x = OM.cart_coords(n, g)[1:n]
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    ana = OA.uniform_sphere(np.stack([X, Y, Z], -1), (0.5, 0.5, 0.5), 0.25)
    assert rel_l2(phi[s, s, s], ana) < 0.05
    if method == "sor" and not kw:
        # red-black 7-point SOR at omega_opt: asymptotic rate omega_opt - 1
        hist = np.array(res.history)
        rate = (hist[-1] / hist[-41]) ** (1 / 40)
        assert rate < 0.83


def test_c1_cg_iterations_grow_and_bound():
    say("CG 1e-10 stop on C1: error bound kappa * rel")
    n = 32
    rho = W.config_c1().rho.numpy()
    phi, res = _solve(n, 1, "cg", 2, rho, 4, 1e-10)
    ref = _oracle_cart(rho, n, 1, 2, 4)
    s = slice(1, n)
    kappa = 1.0 / math.tan(math.pi / (2 * n)) ** 2
    assert rel_l2(phi[s, s, s], ref[s, s, s]) <= kappa * 1e-10
    assert 30 < res.iterations < 200


@pytest.mark.parametrize("method", ["mg", "mg_ir32"])
def test_c2_clumps_multigrid_reduced(method):
    say(f"C2 reduced 64^3 {method}")
    n, g = 64, 1
    wl = W.config_c2(n=n)
    rho = wl.rho.numpy()
    phi, res = _solve(n, g, method, 2, rho, 8, 1e-13)
    assert res.converged, res
    assert res.iterations < 25
    ref = _oracle_cart(rho, n, g, 2, 8)
    s = slice(1, n)
    assert rel_l2(phi[s, s, s], ref[s, s, s]) < CONV_TOL
    if method == "mg":
        assert res.rate < 0.15


@pytest.mark.parametrize("method", ["mg", "mg_ir32"])
def test_c3_star19_multigrid_reduced(method):
    say(f"C3 reduced 32^3 19-point {method}")
    n, g = 32, 3
    wl = W.config_c3(n=n, n_clumps=8)
    rho = wl.rho.numpy()
    phi, res = _solve(n, g, method, 6, rho, 8, 1e-13)
    assert res.converged, res
    ref = _oracle_cart(rho, n, g, 6, 8)
    s = slice(g, g + n - 1)
    assert rel_l2(phi[s, s, s], ref[s, s, s]) < CONV_TOL


@pytest.mark.parametrize("method", ["bicgstab", "bicgstab_mg32"])
def test_c4_spherical_bicgstab_reduced(method):
    say(f"C4 reduced 32x16x16 {method}")
    nr, nth, nph = 32, 16, 16
    wl = W.config_c4(nr=nr, nth=nth, nph=nph)
    rho = wl.rho.numpy()
    r, th, ph, ds = OM.sph_axes(nr, nth, nph)
    mc = 4 * math.pi * 1e-3
    plan = pg.Plan(pg.sph_grid(nr, nth, nph), pg.options(method, lmax=8, point_mass=mc, max_iter=4000))
    phi = torch.zeros(rho.shape, dtype=torch.float64, device="cuda:0")
    res = plan.solve(dev(rho), phi, tol=1e-12)
    assert res.converged, res
    ghost, _, _ = OM.sph_boundary(rho, nr, nth, nph, 8, point_mass=mc)
    ref = OD.solve_sph(ghost, rho, r, ds, th)
    got = host(phi)
    assert rel_l2(got[:, :, 1:nr + 1], ref[:, :, 1:nr + 1]) < CONV_TOL
    assert np.max(np.abs(got[:, :, [0, -1]] - ref[:, :, [0, -1]])) < 1e-12 * np.max(np.abs(ref[:, :, [0, -1]]))


def test_c4_multigrid_preconditioner_cuts_iterations():
    """64 x 32 x 64: one FP32 V(2,2) cycle as the right preconditioner needs
    well under half the BiCGSTAB iterations of the red-black Gauss-Seidel
    step, and both reach the same solution; solving twice into the same
    array (graph reuse) and into another array (re-capture) gives the same
    bits."""
    say("C4 64x32x64 preconditioners")
    nr, nth, nph = 64, 32, 64
    wl = W.config_c4(nr=nr, nth=nth, nph=nph)
    rho = dev(wl.rho.numpy())
    mc = 4 * math.pi * 1e-3
    out = {}
    for m in ("bicgstab", "bicgstab_mg32"):
        plan = pg.Plan(pg.sph_grid(nr, nth, nph), pg.options(m, lmax=8, point_mass=mc, max_iter=4000))
        phi = torch.zeros_like(rho)
        out[m] = (plan.solve(rho, phi, tol=1e-11), host(phi))
        if m == "bicgstab_mg32":
            again = torch.zeros_like(rho)
            res2 = plan.solve(rho, again, tol=1e-11)
            phi.zero_()
            res3 = plan.solve(rho, phi, tol=1e-11)
            assert torch.equal(again, phi) and res2.iterations == res3.iterations == out[m][0].iterations
    (gs, a), (mg, b) = out["bicgstab"], out["bicgstab_mg32"]
    say(f"  iterations: GS {gs.iterations}, MG {mg.iterations}")
    assert gs.converged and mg.converged
    assert mg.iterations * 2 < gs.iterations
    assert rel_l2(a[:, :, 1:-1], b[:, :, 1:-1]) < 1e-9


@functools.lru_cache(maxsize=1)
def _c2_full():
    """C2's 256^3 density and the oracle's exact solution with its multipole
    boundary (computed once for the full-size cases)."""
    rho = W.config_c2(n=256).rho.numpy()
    return rho, _oracle_cart(rho, 256, 1, 2, 8)


@pytest.mark.parametrize("method", ["mg", "mg_ir32", "cg", "pcg"])
def test_c2_full_size_multigrid(method):
    """255^3 unknowns in the benchmarks' launch configurations (the C2
    multigrid in FP64 and as FP32 cycles inside FP64 refinement; CG and PCG as
    in the 255^3 preconditioning study): converged solution against the DST
    oracle."""
    say(f"C2 full size 256^3 FP64 {method}")
    n = 256
    rho, ref = _c2_full()
    phi, res = _solve(n, 1, method, 2, rho, 8, 1e-12, max_iter=20000)
    say(f"  {res.iterations} iterations")
    assert res.converged, res
    s = slice(1, n)
    assert rel_l2(phi[s, s, s], ref[s, s, s]) < CONV_TOL


@functools.lru_cache(maxsize=1)
def _c3_256():
    """The 512^3 workload's recipe (64 clumps + turbulent floor, three ghost
    layers) at 256 intervals, its oracle ghost values (lmax 8) and the
    oracle's exact 19-point solution (about a minute of CPU)."""
    n, g = 256, 3
    rho = W.config_c3(n=n).rho.numpy()
    ghost, _ = OM.cart_boundary(rho, n, g, 8)
    return rho, ghost, OD.solve_cart(ghost, rho, n, 1.0 / n, 6, g)


@pytest.mark.parametrize("method", ["mg", "mg_ir32"])
def test_c3_star19_full_size_paths(method):
    """19-point star (sixth order, four colours, Section 2.1.2) at 256
    intervals with three ghost layers: the large-level shapes of the
    four-colour pass and the residual on the two finest levels.  FP64
    multigrid and FP32 cycles inside FP64 refinement, both driven to 1e-12,
    against the oracle's exact solution on the oracle's own multipole ghosts:
    <= 1e-10 relative L2 on the unknowns, every ghost node within 1e-12."""
    say(f"C3 recipe 256^3 19-point {method}")
    n, g = 256, 3
    rho, ghost, ref = _c3_256()
    phi, res = _solve(n, g, method, 6, rho, 8, 1e-12)
    say(f"  {res.iterations} iterations, rel residual {res.rel_residual:.2e}")
    assert res.converged, res
    s = slice(g, g + n - 1)
    assert rel_l2(phi[s, s, s], ref[s, s, s]) < CONV_TOL
    mask = OM.cart_ghost_mask(n, g)
    assert np.max(np.abs(phi[mask] - ghost[mask])) <= 1e-12 * np.max(np.abs(ghost[mask]))


def test_warm_start_and_determinism():
    say("determinism + warm start")
    n = 64
    rho = W.config_c2(n=n).rho.numpy()
    a, ra = _solve(n, 1, "mg_ir32", 2, rho, 8, 1e-8)
    b, rb = _solve(n, 1, "mg_ir32", 2, rho, 8, 1e-8)
    assert ra.iterations == rb.iterations
    assert np.array_equal(a, b)
    plan = pg.Plan(pg.cart_grid(n), pg.options("mg_ir32", lmax=8))
    phi = dev(a)
    res = plan.solve(dev(rho), phi, tol=1e-8)
    assert res.iterations <= 1


def test_error_paths():
    say("error paths")
    n = 32
    rho = W.config_c1().rho.numpy()
    phi, res = _solve(n, 1, "cg", 2, rho, 4, 1e-12, max_iter=1)
    assert res.status == pg.WARN_MAXITER and res.iterations == 1
    bad = rho.copy()
    bad[10, 10, 10] = np.nan
    with pytest.raises(pg.PoissonError) as e:
        _solve(n, 1, "mg", 2, bad, 4, 1e-8)
    assert e.value.status == -5
    plan = pg.Plan(pg.cart_grid(n), pg.options("cg", lmax=4))
    t = torch.zeros(rho.shape, dtype=torch.float64, device="cuda:0")
    with pytest.raises(pg.PoissonError) as e:
        plan.solve(dev(rho), t, tol=0.0)
    assert e.value.status == -1
    # grid differs from the plan's grid
    st = plan.lib.poisson_solve(plan.handle, pg._ptr(dev(rho)), pg._ptr(t), pg.cart_grid(16), 1e-8, None)
    assert st == -2


def test_c4_full_size_bicgstab():
    """256 x 128 x 256 log-spherical grid, BiCGSTAB with both preconditioners
    driven to 1e-12 against the per-azimuthal-mode sparse-LU oracle (about 1.5
    minutes of CPU)."""
    say("C4 full size 256x128x256 BiCGSTAB")
    wl = W.config_c4()
    rho = wl.rho.numpy()
    g = wl.grid
    mc = 4 * math.pi * g.r_min
    got = {}
    for m in ("bicgstab", "bicgstab_mg32"):
        plan = pg.Plan(pg.sph_grid(g.nr, g.nth, g.nph),
                       pg.options(m, lmax=8, point_mass=mc, max_iter=20000, check_every=10))
        phi = torch.zeros(rho.shape, dtype=torch.float64, device="cuda:0")
        res = plan.solve(dev(rho), phi, tol=1e-12)
        say(f"  {m}: {res.iterations} iterations, rel residual {res.rel_residual:.2e}")
        assert res.converged, res
        got[m] = host(phi)
        del plan, phi
    r, th, ph, ds = OM.sph_axes(g.nr, g.nth, g.nph)
    ghost, _, _ = OM.sph_boundary(rho, g.nr, g.nth, g.nph, 8, point_mass=mc)
    say("  oracle multipole done")
    ref = OD.solve_sph(ghost, rho, r, ds, th)
    for m, x in got.items():
        assert rel_l2(x[:, :, 1:-1], ref[:, :, 1:-1]) < CONV_TOL, m


def test_c3_full_size_properties():
    """511^3 unknowns, 19-point star, FP32 V-cycles inside FP64 refinement to
    1e-10: the oracle's own 19-point operator applied to the returned potential
    (with the returned ghost values) gives the stated relative residual, and the
    mass and dipole moments agree with plain sums over the density."""
    say("C3 full size 512^3 19-point mixed precision")
    n, g = 512, 3
    wl = W.config_c3(n=n, device="cuda:0")
    rho_d = wl.rho.contiguous()
    del wl
    plan = pg.Plan(pg.cart_grid(n, ghost=g), pg.options("mg_ir32", order=6, lmax=8))
    phi = torch.zeros_like(rho_d)
    res = plan.solve(rho_d, phi, tol=1e-10)
    assert res.converged, res
    say(f"  {res.iterations} refinement steps, rel residual {res.rel_residual:.2e}")
    q = np.array(plan.multipole_boundary(rho_d, torch.zeros_like(rho_d), 1))
    rho = host(rho_d)
    got = host(phi)
    del phi, rho_d
    from oracle import operators as OO
    from oracle import smoothers as OS
    h = 1.0 / n
    s = slice(g, g + n - 1)
    z = got.copy()
    z[s, s, s] = 0.0
    bn = np.linalg.norm(rho[s, s, s] - OO.lap19(z, n, h, g))
    del z
    rn = np.linalg.norm(OO.residual(got, rho, n, h, 6, g))
    assert rn / bn <= 1.0001e-10 and rn / bn == pytest.approx(res.rel_residual, rel=1e-3)
    x = (np.arange(1, n) * h - 0.5)
    w = h ** 3
    inner = rho[s, s, s]
    mass = inner.sum() * w
    assert q[0] == pytest.approx(mass, rel=1e-12)
    assert q[2] == pytest.approx((inner.sum(axis=(1, 2)) * x).sum() * w, rel=1e-9, abs=1e-12 * mass)  # z dipole
    assert q[3] == pytest.approx((inner.sum(axis=(0, 1)) * x).sum() * w, rel=1e-9, abs=1e-12 * mass)  # x dipole
    del OS


@pytest.mark.parametrize("dims", [(12, 8, 16), (13, 6, 6), (12, 8, 2)])
@pytest.mark.parametrize("mode", ["chebyshev", "opt"])
def test_spherical_sor_sweeps_match_oracle(mode, dims):
    """Three SOR sweeps on a random state with the local relaxation factors
    (Eq. local_rjac; Eq. omega_n advanced per half-sweep, or the local
    omega_opt) against the oracle's colour passes; an odd radial count and
    an odd half turn (13 x 6 x 6), and nphi = 2, where the relaxation table
    advances in its own kernel."""
    from oracle import sph_sor as SS
    say(f"spherical SOR sweeps ({mode}) {dims}")
    nr, nth, nph = dims
    r, th, ph, ds = OM.sph_axes(nr, nth, nph)
    rng = np.random.default_rng(21)
    u = rng.standard_normal((nph, nth, nr + 2))
    rho = rng.standard_normal((nph, nth, nr + 2))
    om = pg.OMEGA_CHEBYSHEV if mode == "chebyshev" else pg.OMEGA_OPT
    plan = pg.Plan(pg.sph_grid(nr, nth, nph), pg.options("sor", lmax=-1, omega_mode=om))
    x = dev(u)
    plan.smooth(dev(rho), x, sweeps=3)
    rj = SS.local_rjac(nr, nth, nph, ds, th)
    ref = u.copy()
    w = SS.omega_first(rj) if mode == "chebyshev" else SS.omega_opt(rj)
    for _ in range(3):
        wr = w
        if mode == "chebyshev":
            w = SS.omega_next(w, rj)
        wb = w
        if mode == "chebyshev":
            w = SS.omega_next(w, rj)
        SS.sweep(ref, rho, r, ds, th, wr, wb)
    got = host(x)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_spherical_sor_converges_to_the_oracle_solution():
    """C4's SIS density on 32 x 16 x 16 with the multipole boundary: SOR with
    the local Chebyshev sequence driven to 1e-12 equals the per-mode sparse
    LU solution."""
    say("spherical SOR converged")
    nr, nth, nph = 32, 16, 16
    wl = W.config_c4(nr=nr, nth=nth, nph=nph)
    rho = wl.rho.numpy()
    r, th, ph, ds = OM.sph_axes(nr, nth, nph)
    mc = 4 * math.pi * 1e-3
    plan = pg.Plan(pg.sph_grid(nr, nth, nph), pg.options("sor", lmax=8, point_mass=mc, max_iter=50000,
                                                         omega_mode=pg.OMEGA_CHEBYSHEV, check_every=10))
    phi = torch.zeros(rho.shape, dtype=torch.float64, device="cuda:0")
    res = plan.solve(dev(rho), phi, tol=1e-12)
    say(f"  {res.iterations} sweeps")
    assert res.converged, res
    ghost, _, _ = OM.sph_boundary(rho, nr, nth, nph, 8, point_mass=mc)
    ref = OD.solve_sph(ghost, rho, r, ds, th)
    assert rel_l2(host(phi)[:, :, 1:nr + 1], ref[:, :, 1:nr + 1]) < CONV_TOL


CART_METHODS = [("sor", {}), ("cg", {}), ("pcg", {}), ("mg", {}), ("mg_ir32", {}), ("mg_spai", {"order": 2}),
                ("mg_spai", {"order": 4}), ("mg_spai32", {"order": 2}), ("mg_spai", {"order": 2, "coarse_tol": 0.1})]


@pytest.mark.parametrize("method,kw", CART_METHODS)
def test_degenerate_cartesian_inputs(method, kw):
    """Zero density with the multipole boundary: converged at once, Phi stays
    zero.  Zero density with linear ghost values: the discrete solution is
    that linear function (every operator here is exact on it)."""
    say(f"degenerate inputs {method} {kw}")
    n = 32
    kw = dict(kw)
    order = kw.pop("order", 2)
    plan = pg.Plan(pg.cart_grid(n), pg.options(method, order=order, lmax=8, max_iter=20000, **kw))
    rho = torch.zeros((n + 1,) * 3, dtype=torch.float64, device="cuda:0")
    phi = torch.zeros_like(rho)
    res = plan.solve(rho, phi, tol=1e-10)
    assert res.converged and res.iterations == 0
    assert float(phi.abs().max()) == 0.0
    plan2 = pg.Plan(pg.cart_grid(n), pg.options(method, order=order, lmax=-1, max_iter=20000, **kw))
    x = np.arange(n + 1) / n
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    lin = 1.0 + 2.0 * xx - 0.5 * y + 0.25 * z
    start = lin.copy()
    start[1:n, 1:n, 1:n] = 0.0
    phi2 = dev(start)
    res2 = plan2.solve(rho, phi2, tol=1e-12)
    assert res2.converged, res2
    assert np.max(np.abs(host(phi2) - lin)) < 1e-9 * np.max(np.abs(lin))


@pytest.mark.parametrize("method", ["bicgstab", "bicgstab_mg32", "sor"])
def test_degenerate_spherical_inputs(method):
    """Zero density, no point mass: converged at once with Phi zero; zero
    density with constant radial ghosts: the solution is that constant."""
    say(f"degenerate spherical inputs {method}")
    nr, nth, nph = 16, 8, 16
    extra = {"omega_mode": pg.OMEGA_CHEBYSHEV} if method == "sor" else {}
    plan = pg.Plan(pg.sph_grid(nr, nth, nph), pg.options(method, lmax=8, max_iter=20000, **extra))
    rho = torch.zeros((nph, nth, nr + 2), dtype=torch.float64, device="cuda:0")
    phi = torch.zeros_like(rho)
    res = plan.solve(rho, phi, tol=1e-10)
    assert res.converged and res.iterations == 0
    assert float(phi.abs().max()) == 0.0
    plan2 = pg.Plan(pg.sph_grid(nr, nth, nph), pg.options(method, lmax=-1, max_iter=20000, **extra))
    phi2 = torch.zeros_like(rho)
    phi2[:, :, 0] = -3.0
    phi2[:, :, -1] = -3.0
    res2 = plan2.solve(rho, phi2, tol=1e-12)
    assert res2.converged, res2
    assert float((phi2 + 3.0).abs().max()) < 1e-9


@pytest.mark.parametrize("method,order,n,coarsest", [("mg", 2, 96, 6), ("mg_ir32", 2, 96, 6), ("mg", 6, 48, 6),
                                                     ("mg_ir32", 6, 48, 6), ("cg", 2, 33, 8), ("cg", 6, 33, 8),
                                                     ("pcg", 2, 33, 8), ("pcg", 6, 33, 8), ("sor", 2, 33, 8)])
def test_ragged_sizes_match_oracle(method, order, n, coarsest):
    """Sizes whose rows end in partial tiles (95, 47 or 32 unknowns per
    axis) and hierarchies ending at 6 intervals, against the oracle's exact
    discrete solution with its own multipole boundary."""
    say(f"ragged {method} order {order} n {n}")
    g = 1 if order == 2 else 3
    wl = W.config_c2(n=n) if g == 1 else W.config_c3(n=n, n_clumps=8)
    rho = wl.rho.numpy()
    tol = 1e-12 if method in ("sor", "cg", "pcg") else 1e-13
    phi, res = _solve(n, g, method, order, rho, 8, tol, coarsest=coarsest, max_iter=50000,
                      check_every=10 if method == "sor" else 1)
    assert res.converged, res
    ref = _oracle_cart(rho, n, g, order, 8)
    s = slice(g, g + n - 1)
    assert rel_l2(phi[s, s, s], ref[s, s, s]) < CONV_TOL
