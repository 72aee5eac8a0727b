"""CG preconditioned by one symmetric multi-colour Gauss-Seidel step
(Section 2.1.2) against the oracle: iterate by iterate on the same inputs,
converged against the exact discrete solution, and beside plain CG."""
import numpy as np
import pytest
import torch

import paper_2605_03563_amd as pg
import workloads as W
from oracle import direct as OD
from oracle import krylov as OK
from oracle import multipole as OM
from tests.gpu_util import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu
ITER_TOL = 1e-10     # FP64 iterates, reduction order differs
CONV_TOL = 1e-9


def _problem(n, g, seed):
    rng = np.random.default_rng(seed)
    m = n + 1 + 2 * (g - 1)
    phi = rng.normal(size=(m, m, m))
    s = slice(g, g + n - 1)
    phi[s, s, s] = 0.0
    return phi, rng.normal(size=(m, m, m))


@pytest.mark.parametrize("order,n", [(2, 40), (6, 36)])
def test_iterates_match_oracle(order, n):
    """Ghost values read from Phi (lmax -1), random density: after 1, 2 and 7
    iterations the GPU iterate equals the oracle's (n - 1 = 39 / 35 unknowns
    per axis: partial tiles in every direction)."""
    g = 1 if order == 2 else 3
    h = 1.0 / n
    phi0, rho = _problem(n, g, n + order)
    s = slice(g, g + n - 1)
    hist = []
    OK.cg(phi0, rho, n, h, order, g, tol=0.0, max_iter=7, history=hist)
    for k in (1, 2, 7):
        say(f"PCG order {order} n {n}: {k} iterations")
        plan = pg.Plan(pg.cart_grid(n, ghost=g), pg.options("pcg", order=order, lmax=-1, max_iter=k))
        phi = dev(phi0)
        res = plan.solve(dev(rho), phi, tol=1e-30)
        assert res.iterations == k and not res.converged
        got = host(phi)
        assert rel_l2(got[s, s, s], hist[k - 1]) < ITER_TOL
        mask = OM.cart_ghost_mask(n, g)
        assert np.array_equal(got[mask], phi0[mask])


@pytest.mark.parametrize("method,n,iters", [("cg", 256, (1, 3)), ("pcg", 256, (1, 3)), ("cg", 512, (2,))])
def test_full_size_iterates_match_oracle(method, n, iters):
    """The 7-point CG and PCG at full size, where a row fills a wavefront with
    two compact columns per lane: the direction kernel marching along z
    (8-plane runs at 256 intervals, 16-plane runs at 512) and, for PCG, the
    vector colour passes that form the inner product; the GPU iterate after
    each listed count equals the oracle's."""
    order, g = 2, 1
    h = 1.0 / n
    phi0, rho = _problem(n, g, n + 7)
    s = slice(g, g + n - 1)
    hist = []
    say(f"oracle {method} n {n}: {max(iters)} iterations")
    OK.cg(phi0, rho, n, h, order, g, tol=0.0, max_iter=max(iters), precondition=(method == "pcg"), history=hist)
    for k in iters:
        say(f"{method} n {n}: {k} iterations")
        plan = pg.Plan(pg.cart_grid(n, ghost=g), pg.options(method, order=order, lmax=-1, max_iter=k))
        phi = dev(phi0)
        res = plan.solve(dev(rho), phi, tol=1e-30)
        assert res.iterations == k and not res.converged
        assert rel_l2(host(phi)[s, s, s], hist[k - 1]) < ITER_TOL
        del plan, phi


@pytest.mark.parametrize("order,n", [(2, 64), (6, 48)])
def test_converged_matches_exact_and_beats_cg(order, n):
    """Clumps (C2 / C3 shapes at reduced size) with the multipole boundary:
    the converged PCG potential equals the exact discrete solution, in fewer
    iterations than plain CG."""
    g = 1 if order == 2 else 3
    wl = W.config_c2(n=n) if g == 1 else W.config_c3(n=n, n_clumps=8)
    rho = wl.rho.numpy()
    its = {}
    out = {}
    for method in ("cg", "pcg"):
        plan = pg.Plan(pg.cart_grid(n, ghost=g), pg.options(method, order=order, lmax=8, max_iter=20000))
        phi = torch.zeros(rho.shape, dtype=torch.float64, device="cuda:0")
        res = plan.solve(dev(rho), phi, tol=1e-12)
        say(f"  {method} order {order} n {n}: {res.iterations} iterations")
        assert res.converged, res
        its[method] = res.iterations
        out[method] = host(phi)
    ghost, _ = OM.cart_boundary(rho, n, g, 8)
    ref = OD.solve_cart(ghost, rho, n, 1.0 / n, order, g)
    s = slice(g, g + n - 1)
    assert rel_l2(out["pcg"][s, s, s], ref[s, s, s]) < CONV_TOL
    assert its["pcg"] < 0.75 * its["cg"]


def test_warm_start_and_repeat_are_deterministic():
    """A converged solution as the initial guess: converged at once; two
    identical solves give identical bits."""
    n, g = 32, 1
    wl = W.config_c2(n=n)
    rho = wl.rho.to("cuda:0")
    plan = pg.Plan(pg.cart_grid(n), pg.options("pcg", lmax=8))
    a = torch.zeros_like(rho)
    b = torch.zeros_like(rho)
    plan.solve(rho, a, tol=1e-11)
    plan.solve(rho, b, tol=1e-11)
    assert torch.equal(a, b)
    res = plan.solve(rho, a, tol=1e-10)
    assert res.converged and res.iterations == 0
