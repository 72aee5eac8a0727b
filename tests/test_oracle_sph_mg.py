"""Pins of the spherical multigrid preconditioner oracle (the construction
chosen for the right-preconditioned BiCGSTAB; Sections 2.1.2-2.1.3)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import multipole as OM
from oracle import operators as OO
from oracle import sph_mg as SM


def test_level_rule():
    assert SM.levels(256, 128, 256)[-1] == (8, 4, 8)
    assert len(SM.levels(256, 128, 256)) == 6
    assert SM.levels(9, 8, 8) == [(9, 8, 8)]


def test_operator_matches_the_oracle_spherical_operator():
    """With zero radial ghosts the level operator is the oracle's r^2-scaled
    operator of the fine grid."""
    nr, nth, nph = 6, 4, 8
    r, th, ph, ds = OM.sph_axes(nr, nth, nph)
    rng = np.random.default_rng(0)
    u = rng.standard_normal((nph, nth, nr))
    full = np.zeros((nph, nth, nr + 2))
    full[:, :, 1:nr + 1] = u
    assert np.allclose(SM.apply(u, ds), OO.sph_apply(full, ds, th), rtol=0, atol=1e-10)


def test_line_pass_solves_its_lines():
    """After a pass of colour c, the residual vanishes on the lines of colour
    c except for the lagged cross-pole term on the pole lines."""
    nr, nth, nph = 6, 4, 8
    rng = np.random.default_rng(1)
    ds = 0.1
    u = rng.standard_normal((nph, nth, nr))
    f = rng.standard_normal((nph, nth, nr))
    for c in (0, 1):
        v = u.copy()
        SM.line_pass(v, f, ds, c)
        res = f - SM.apply(v, ds)
        mask = np.zeros((nph, nth, nr), bool)
        for j in range(1, nth - 1):
            for i in range(nr):
                if (i + j) % 2 == c:
                    mask[:, j, i] = True
        assert np.max(np.abs(res[mask])) < 1e-9 * np.max(np.abs(f))
        assert np.max(np.abs(res[~mask])) > 1e-3


def test_transfers_are_adjoint_up_to_the_volume_factor():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((8, 4, 6))
    b = rng.standard_normal((4, 2, 3))
    assert np.sum(SM.restrict(a) * b) == pytest.approx(np.sum(a * SM.prolong(b)) / 8.0, rel=1e-12)


def test_cycle_is_linear_and_cuts_bicgstab_iterations():
    """The cycle is a linear map (a fixed preconditioner), and as the right
    preconditioner of BiCGSTAB on the SIS workload it needs far fewer
    iterations than no preconditioner."""
    import workloads as W
    nr, nth, nph = 32, 16, 32
    r, th, ph, ds = OM.sph_axes(nr, nth, nph)
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal((2, nph, nth, nr))
    cache = {}
    lin = SM.vcycle(2.0 * x - 0.5 * y, ds, _cache=cache)
    assert np.allclose(lin, 2.0 * SM.vcycle(x, ds, _cache=cache) - 0.5 * SM.vcycle(y, ds, _cache=cache),
                       rtol=0, atol=1e-10 * np.max(np.abs(lin)))
    wl = W.config_c4(nr=nr, nth=nth, nph=nph)
    ghost, _, _ = OM.sph_boundary(wl.rho.numpy(), nr, nth, nph, 8, point_mass=4 * np.pi * 1e-3)
    z = ghost.copy()
    z[:, :, 1:nr + 1] = 0.0
    b = OO.sph_residual(z, wl.rho.numpy(), r, ds, th).ravel()
    N = b.size
    A = spla.LinearOperator((N, N), matvec=lambda v: SM.apply(np.asarray(v).reshape(nph, nth, nr), ds).ravel(),
                            dtype=np.float64)
    M = spla.LinearOperator((N, N), matvec=lambda v: SM.vcycle(np.asarray(v).reshape(nph, nth, nr), ds,
                                                               _cache=cache).ravel(), dtype=np.float64)
    counts = []
    for prec in (None, M):
        it = [0]
        _, info = spla.bicgstab(A, b, rtol=1e-8, maxiter=5000, M=prec, callback=lambda _x: it.__setitem__(0, it[0] + 1))
        assert info == 0
        counts.append(it[0])
    assert counts[1] * 10 < counts[0], counts
