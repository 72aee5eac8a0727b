"""SPAI multigrid on compact stencils (Section 2.1.3, Table 1) against the
oracle: residual with the compact right-hand side, Richardson steps, one
V-cycle with Galerkin coarse operators, converged solves, full size."""
import numpy as np
import pytest
import torch

import paper_2605_03563_amd as pg
from oracle import multipole as OM
from oracle import spai as SP
from tests.gpu_util import dev, host, rel_l2, rel_max, say
import workloads as W

pytestmark = pytest.mark.gpu
KERNEL_TOL = 1e-13
CYCLE_TOL = 1e-12
CONV_TOL = 1e-10


def _ghost(order):
    """Order 6 reads rho's second ghost layer."""
    return 2 if order == 6 else 1


def _random(n, seed, order=2):
    rng = np.random.default_rng(seed)
    m = n + 1 + 2 * (_ghost(order) - 1)
    phi = rng.normal(size=(m,) * 3)
    rho = rng.normal(size=(m,) * 3)
    return phi, rho


def _nodes(a, n, order):
    """Nodes 0..n of a caller array (the oracle's one-ghost node array)."""
    g = _ghost(order)
    s = slice(g - 1, g + n)
    return a[s, s, s]


def _f(rho, n, order):
    """What the oracle's right-hand side reads: nodes 0..n, order 6 one more."""
    return rho if order == 6 else _nodes(rho, n, order)


def _inner(a, n, order):
    g = _ghost(order)
    s = slice(g, g + n - 1)
    return a[s, s, s]


def _plan(n, order, coarsest=8, method="mg_spai", **kw):
    return pg.Plan(pg.cart_grid(n, ghost=_ghost(order)),
                   pg.options(method, order=order, lmax=-1, coarsest=coarsest, **kw))


@pytest.mark.parametrize("order", [2, 4, 6])
@pytest.mark.parametrize("n", [16, 48])
def test_residual_with_compact_rhs(order, n):
    say(f"SPAI residual order {order} n {n}")
    phi, rho = _random(n, 100 + n + order, order)
    plan = _plan(n, order, coarsest=n // 2 if n == 16 else 6)
    res = torch.zeros(rho.shape, dtype=torch.float64, device="cuda:0")
    n2 = plan.residual(dev(rho), dev(phi), res)
    h = 1.0 / n
    ref = SP.rhs_compact(_f(rho, n, order), n, order) - SP.apply27(_nodes(phi, n, order), n, SP.WEIGHTS[order],
                                                                   1.0 / (h * h))
    got = _inner(host(res), n, order)
    assert rel_max(got, ref) < KERNEL_TOL
    assert n2 == pytest.approx(float(np.sum(ref * ref)), rel=1e-12)


@pytest.mark.parametrize("order", [2, 4, 6])
def test_richardson_steps(order):
    n = 48
    say(f"SPAI Richardson steps order {order}")
    phi, rho = _random(n, 7 + order, order)
    plan = _plan(n, order, coarsest=6)
    x = dev(phi)
    plan.smooth(dev(rho), x, sweeps=3)
    h = 1.0 / n
    w = tuple(c / (h * h) for c in SP.WEIGHTS[order])
    f = SP.rhs_compact(_f(rho, n, order), n, order)
    ref = _nodes(phi, n, order).copy()
    for _ in range(3):
        SP.spai_step(ref, f, n, w, SP.COEFFS[order], h)
    assert rel_max(_nodes(host(x), n, order), ref) < KERNEL_TOL


def test_richardson_step_full_size_sampled():
    """511^3 unknowns (the 64 x 16 tiles and 128-plane runs of the fine
    step): one Richardson step from a random guess against the oracle's step
    evaluated around sampled nodes (r = f - A u on the 27 nodes around the
    sample, then u - omega M r there), including every tile and run seam
    and the last rows and planes."""
    n, order = 512, 2
    say("SPAI Richardson step 511^3, sampled")
    phi, rho = _random(n, 99, order)
    plan = _plan(n, order, coarsest=4)
    x = dev(phi)
    plan.smooth(dev(rho), x, sweeps=1)
    got = host(x)
    del x
    h = 1.0 / n
    w = tuple(c / (h * h) for c in SP.WEIGHTS[order])
    om, al, be, ga, de = SP.COEFFS[order][:5]
    rng = np.random.default_rng(5)
    pts = [tuple(rng.integers(2, n - 1, size=3)) for _ in range(150)]
    seams = [2, 15, 16, 17, 63, 64, 65, 127, 128, 129, 130, 256, 257, 384, 385, 509, 510]
    pts += [(a, b, c) for a in seams[::3] for b in seams[1::3] for c in seams[2::3]]
    pts += [(k, j, i) for k in (128, 129, 257, 385, 510) for j in (16, 17, 510) for i in (64, 65, 510)]
    errs, scale = [], 0.0
    for (k, j, i) in pts:
        U = phi[k - 2:k + 3, j - 2:j + 3, i - 2:i + 3]
        F = rho[k - 1:k + 2, j - 1:j + 2, i - 1:i + 2]
        r = F - SP.apply27(U, 4, w)
        ref = U[2, 2, 2] - om * SP.apply27(r, 2, (al, be, ga, de), h * h)[0, 0, 0]
        errs.append(abs(got[k, j, i] - ref))
        scale = max(scale, abs(ref))
    assert max(errs) < KERNEL_TOL * scale
    assert np.array_equal(got[0], phi[0]) and np.array_equal(got[:, :, n], phi[:, :, n])


@pytest.mark.parametrize("order,n,coarsest", [(2, 32, 8), (4, 32, 8), (6, 32, 8), (2, 48, 6), (6, 48, 6),
                                              (4, 128, 8), (6, 128, 8)])
def test_one_vcycle_matches_oracle(order, n, coarsest):
    """One V(3,3) cycle with Galerkin coarse operators from a random guess
    (n = 48: 47 unknowns per row, a ragged tile; n = 128: four levels)."""
    say(f"SPAI one V-cycle order {order} n {n}")
    phi, rho = _random(n, 11 * n + order, order)
    plan = _plan(n, order, coarsest=coarsest)
    x = dev(phi)
    plan.vcycle(dev(rho), x, 1)
    ops = SP.level_operators(order, n, coarsest)
    f = SP.rhs_compact(_f(rho, n, order), n, order)
    ref = _nodes(phi, n, order).copy()
    SP.vcycle(ref, f, n, ops, SP.COEFFS[order], 3, 3)
    assert rel_max(_nodes(host(x), n, order), ref) < CYCLE_TOL


def _clumps(n, order):
    """C2-shaped clumps at n^3 with the oracle's lmax = 8 ghosts."""
    g = _ghost(order)
    rho = W.config_c2(n=n, g=g).rho.numpy()
    ghost, _ = OM.cart_boundary(rho, n, g, 8)
    return rho, ghost


@pytest.mark.parametrize("order", [2, 4, 6])
def test_converged_solve_matches_exact_discrete_solution(order):
    """Clumps at 64^3 with the multipole boundary (lmax 8) from the oracle:
    the converged SPAI multigrid equals the DST solution of the same
    compact discretisation."""
    n = 64
    say(f"SPAI converged order {order}")
    rho, ghost = _clumps(n, order)
    plan = _plan(n, order)
    phi = dev(ghost)
    res = plan.solve(dev(rho), phi, tol=1e-13)
    assert res.converged, res
    ref = SP.solve_cart(_nodes(ghost, n, order), _f(rho, n, order), n, order)
    s = slice(1, n)
    assert rel_l2(_nodes(host(phi), n, order)[s, s, s], ref[s, s, s]) < CONV_TOL


@pytest.mark.parametrize("order", [4, 6])
def test_multipole_ghosts_and_rate_full_size(order):
    """255^3 unknowns, GPU multipole boundary: converged against the DST
    oracle on the ghosts the GPU wrote, at a V(3,3) contraction well inside
    the Table 2 regime."""
    n = 256
    say(f"SPAI full size 256^3 order {order}")
    wl = W.config_c2(n=n, device="cuda:0", g=_ghost(order))
    rho_d = wl.rho.contiguous()
    plan = pg.Plan(pg.cart_grid(n, ghost=_ghost(order)), pg.options("mg_spai", order=order, lmax=8))
    phi = torch.zeros_like(rho_d)
    res = plan.solve(rho_d, phi, tol=1e-12, history=64)
    assert res.converged, res
    say(f"  {res.iterations} cycles, rate {res.rate:.3g}")
    assert res.rate < 0.05
    got = _nodes(host(phi), n, order)
    ref = SP.solve_cart(got, _f(host(rho_d), n, order), n, order)
    s = slice(1, n)
    assert rel_l2(got[s, s, s], ref[s, s, s]) < CONV_TOL


def test_spai_plans_reject_split_layout_operators():
    plan = _plan(16, 2)
    t = torch.zeros(17 ** 3, dtype=torch.float64, device="cuda:0")
    with pytest.raises(pg.PoissonError):
        plan.apply(t, t)
    with pytest.raises(pg.PoissonError):
        plan.restrict(torch.zeros(15 ** 3, dtype=torch.float64, device="cuda:0"),
                      torch.zeros(7 ** 3, dtype=torch.float64, device="cuda:0"))


@pytest.mark.parametrize("order", [2, 4, 6])
def test_fp32_coarse_storage_vcycle(order):
    """MG_SPAI32: one V(3,3) cycle against the oracle that rounds every value
    stored on the coarse levels to FP32 (arithmetic FP64 on both sides), and
    within FP32 rounding of the all-FP64 cycle."""
    n = 64
    say(f"SPAI32 one V-cycle order {order}")
    phi, rho = _random(n, 300 + order, order)
    plan = _plan(n, order, method="mg_spai32")
    x = dev(phi)
    plan.vcycle(dev(rho), x, 1)
    ops = SP.level_operators(order, n)
    f = SP.rhs_compact(_f(rho, n, order), n, order)
    p0 = _nodes(phi, n, order)
    ref32, ref64 = p0.copy(), p0.copy()
    SP.vcycle(ref32, f, n, ops, SP.COEFFS[order], 3, 3, store32=True)
    SP.vcycle(ref64, f, n, ops, SP.COEFFS[order], 3, 3)
    got = _nodes(host(x), n, order)
    assert rel_max(got, ref32) < 1e-9
    corr = np.max(np.abs(ref64 - p0))
    assert np.max(np.abs(got - ref64)) < 1e-6 * corr


@pytest.mark.parametrize("order", [2, 6])
def test_fp32_coarse_storage_converges_to_the_fp64_solution(order):
    n = 64
    say(f"SPAI32 converged order {order}")
    rho, ghost = _clumps(n, order)
    plan = _plan(n, order, method="mg_spai32")
    phi = dev(ghost)
    res = plan.solve(dev(rho), phi, tol=1e-13)
    assert res.converged, res
    ref = SP.solve_cart(_nodes(ghost, n, order), _f(rho, n, order), n, order)
    s = slice(1, n)
    assert rel_l2(_nodes(host(phi), n, order)[s, s, s], ref[s, s, s]) < CONV_TOL


@pytest.mark.parametrize("order,coarsest", [(2, 8), (4, 4), (6, 8)])
def test_cg_coarsest_vcycle_and_solve(order, coarsest):
    """Coarsest level by CG to relative accuracy 0.013 (Section 2.1.3): one
    V-cycle against the oracle's cycle with the same CG coarsest solve, and a
    converged solve against the exact discrete solution."""
    n = 64
    say(f"SPAI CG coarsest order {order} coarsest {coarsest}")
    phi, rho = _random(n, 500 + order, order)
    plan = _plan(n, order, coarsest=coarsest, coarse_tol=0.013)
    x = dev(phi)
    plan.vcycle(dev(rho), x, 1)
    ops = SP.level_operators(order, n, coarsest)
    f = SP.rhs_compact(_f(rho, n, order), n, order)
    ref = _nodes(phi, n, order).copy()
    SP.vcycle(ref, f, n, ops, SP.COEFFS[order], 3, 3, coarse_rtol=0.013)
    assert rel_max(_nodes(host(x), n, order), ref) < 1e-10
    rho2, ghost = _clumps(n, order)
    phi2 = dev(ghost)
    res = plan.solve(dev(rho2), phi2, tol=1e-13)
    assert res.converged, res
    ref2 = SP.solve_cart(_nodes(ghost, n, order), _f(rho2, n, order), n, order)
    s = slice(1, n)
    assert rel_l2(_nodes(host(phi2), n, order)[s, s, s], ref2[s, s, s]) < CONV_TOL
