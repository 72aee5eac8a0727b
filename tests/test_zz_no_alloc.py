"""The allocation-free multipole boundary (fixed per-device scratch array)
against the plan-based multipole_boundary and the oracle, on two calls in a
row, the second with a smaller grid, through the C ABI."""
import numpy as np
import pytest
import torch

import paper_2605_03563_amd as pg
from oracle import multipole as OM
from tests.gpu_util import dev, host, rel_max, say
from workloads import CartGrid, clump_density, draw_clumps, embed

pytestmark = pytest.mark.gpu


def _case(n, g, lmax, nclumps, seed, pitch_pad):
    rho = clump_density(CartGrid(n, g), draw_clumps(np.random.default_rng(seed), nclumps)).numpy()
    m = rho.shape[0]
    px = m + pitch_pad
    grid = pg.cart_grid(n, ghost=g, pitch_x=px)
    rho_d = embed(dev(rho), px).contiguous()
    return rho, grid, rho_d, px


@pytest.mark.parametrize("first,second", [((128, 3, 8, 24, 21, 0), (40, 1, 6, 5, 22, 7))])
def test_noalloc_multipole_matches_plan_and_oracle(first, second):
    for (n, g, lmax, nc, seed, pad) in (first, second):
        say(f"noalloc multipole n={n} g={g} lmax={lmax} pitch_pad={pad}")
        rho, grid, rho_d, px = _case(n, g, lmax, nc, seed, pad)
        m = rho.shape[0]
        sentinel = 7.25
        phi_a = torch.full((m, m, px), sentinel, dtype=torch.float64, device="cuda:0")
        phi_b = phi_a.clone()
        q_a = np.array(pg.multipole_boundary_noalloc(grid, rho_d, phi_a, lmax))
        plan = pg.Plan(grid, pg.options("cg", order=2 if g == 1 else 6, lmax=lmax))
        q_b = np.array(plan.multipole_boundary(rho_d, phi_b, lmax))
        torch.cuda.synchronize()
        plan.close()
        a, b = host(phi_a), host(phi_b)
        # same kernels and summation order: identical to the plan's result
        assert np.array_equal(q_a, q_b)
        assert np.array_equal(a, b)
        # and within the kernel-level bar of the oracle
        ref_phi, ref_q = OM.cart_boundary(rho, n, g, lmax)
        assert rel_max(q_a, ref_q) < 1e-12
        mask = OM.cart_ghost_mask(n, g)
        got = a[:, :, :m]
        assert rel_max(got[mask], ref_phi[mask]) < 1e-12
        # the unknowns and the row padding are left untouched
        assert np.all(got[~mask] == sentinel)
        assert np.all(a[:, :, m:] == sentinel)

