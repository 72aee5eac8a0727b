"""Kernel-level references: colour passes, grid transfers, a V-cycle.

* Red-black SOR/Gauss-Seidel (Section 2.1.1): the colour of node (i, j, k)
  (global node indices, unknowns 1..n-1) is (i+j+k) mod 2, colour 0 ("red")
  first.  One colour pass replaces every unknown u of that colour by
  (1 - w) u + w * (sum of its 6 neighbours - h^2 f) / 6; w = 1 is Gauss-Seidel.
  No two nodes of a colour are neighbours, so updating them all from the
  array as it was before the pass is the same as updating them one by one.
* Four-colour Gauss-Seidel for the 19-point star (Section 2.1.2, four colours
  for 6th order): colour (i+j+k) mod 4; a pass solves each node's own row of
  the star operator for that node, i.e. u = (h^2 f - sum of neighbour terms)
  / (3 c0).  Offsets 1, 2, 3 along an axis change the colour, so the pass is
  again order-independent.
* Full-weighting restriction R = R1 x R1 x R1, R1 = [1 2 1]/4, onto the
  coarse unknowns at fine nodes 2I, and prolongation P = 8 R^T, which keeps
  constants (trilinear interpolation) (Section 2.1.3).
* One V-cycle with nu1 pre- and nu2 post-smoothing sweeps, coarse operators
  rediscretised at spacing 2h, homogeneous Dirichlet corrections and an exact
  solve on the coarsest level (E_N = A_N^-1).
"""
from __future__ import annotations

import numpy as np

from . import operators as O

STAR6 = O.STAR6


def colour_mask(n: int, g: int, ncol: int, colour: int) -> np.ndarray:
    """Boolean mask over the full node array: unknown nodes of `colour`."""
    m = n + 1 + 2 * (g - 1)
    i = np.arange(m) - (g - 1)
    s = i[:, None, None] + i[None, :, None] + i[None, None, :]
    mask = (s % ncol) == colour
    inner = np.zeros((m, m, m), dtype=bool)
    inner[g:g + n - 1, g:g + n - 1, g:g + n - 1] = True
    return mask & inner


def _neigh_sum7(u, g, n):
    """sum of the 6 neighbours, on the unknowns."""
    return O.lap7(u, n, 1.0, g) + 6.0 * O._shift(u, g, n, 0, 0, 0)


def _neigh_sum19(u, g, n):
    """sum over the 18 off-centre star coefficients (h = 1)."""
    return O.lap19(u, n, 1.0, g) - 3.0 * STAR6[0] * O._shift(u, g, n, 0, 0, 0)


def rb_pass(u, f, n, h, colour, omega=1.0, g=1):
    """One red-black SOR colour pass, in place on u; returns u."""
    s = slice(g, g + n - 1)
    gs = (_neigh_sum7(u, g, n) - h * h * f[s, s, s]) / 6.0
    mask = colour_mask(n, g, 2, colour)[s, s, s]
    inner = u[s, s, s]
    inner[mask] = (1.0 - omega) * inner[mask] + omega * gs[mask]
    return u


def star_pass(u, f, n, h, colour, g=3):
    """One four-colour Gauss-Seidel pass of the 19-point star, in place."""
    s = slice(g, g + n - 1)
    gs = (h * h * f[s, s, s] - _neigh_sum19(u, g, n)) / (3.0 * STAR6[0])
    mask = colour_mask(n, g, 4, colour)[s, s, s]
    inner = u[s, s, s]
    inner[mask] = gs[mask]
    return u


def smooth(u, f, n, h, order, g, forward=True, omega=1.0):
    """One full sweep: colours in increasing order (forward) or reversed."""
    ncol = 2 if order == 2 else 4
    cols = range(ncol) if forward else range(ncol - 1, -1, -1)
    for c in cols:
        if order == 2:
            rb_pass(u, f, n, h, c, omega, g)
        else:
            star_pass(u, f, n, h, c, g)
    return u


def restrict(r_int: np.ndarray) -> np.ndarray:
    """Full weighting of an interior residual (n-1)^3 -> (n/2-1)^3."""
    n = r_int.shape[0] + 1
    nc = n // 2
    w = {-1: 0.25, 0: 0.5, 1: 0.25}
    out = np.zeros((nc - 1,) * 3)
    # fine interior index (0-based) of coarse unknown I (1..nc-1) is 2I-1
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                out += w[a] * w[b] * w[c] * r_int[
                    slice(1 + a, 1 + a + 2 * (nc - 1), 2),
                    slice(1 + b, 1 + b + 2 * (nc - 1), 2),
                    slice(1 + c, 1 + c + 2 * (nc - 1), 2)]
    return out


def prolong(e_int: np.ndarray) -> np.ndarray:
    """P = 8 R^T: coarse interior (nc-1)^3 -> fine interior (2nc-1)^3 with
    zero coarse boundary (trilinear interpolation)."""
    nc = e_int.shape[0] + 1
    ec = np.zeros((nc + 1,) * 3)
    ec[1:nc, 1:nc, 1:nc] = e_int
    n = 2 * nc
    full = np.zeros((n + 1,) * 3)
    # 1-D linear interpolation along each axis in turn
    tmp = np.zeros((nc + 1, nc + 1, n + 1))
    tmp[:, :, 0::2] = ec
    tmp[:, :, 1::2] = 0.5 * (ec[:, :, :-1] + ec[:, :, 1:])
    tmp2 = np.zeros((nc + 1, n + 1, n + 1))
    tmp2[:, 0::2, :] = tmp
    tmp2[:, 1::2, :] = 0.5 * (tmp[:, :-1, :] + tmp[:, 1:, :])
    full[0::2] = tmp2
    full[1::2] = 0.5 * (tmp2[:-1] + tmp2[1:])
    return full[1:n, 1:n, 1:n]


def coarse_matrix(n: int, order: int, h: float) -> np.ndarray:
    """Dense matrix of L_h on the (n-1)^3 unknowns with zero ghosts, built
    column by column by applying the operator to unit vectors."""
    g = 1 if order == 2 else 3
    e = n - 1
    m = n + 1 + 2 * (g - 1)
    A = np.zeros((e ** 3, e ** 3))
    u = np.zeros((m, m, m))
    for col in range(e ** 3):
        k, rem = divmod(col, e * e)
        j, i = divmod(rem, e)
        u[g + k, g + j, g + i] = 1.0
        A[:, col] = O.lap(u, n, h, order, g).ravel()
        u[g + k, g + j, g + i] = 0.0
    return A


def vcycle(u, f, n, h, order, g, nu1=2, nu2=2, coarsest=8, _cache=None):
    """One V(nu1, nu2) cycle on u (full node array, ghosts fixed), in place.

    Pre-smoothing sweeps colours forward, post-smoothing backward, so the
    cycle is symmetric.  Coarse problems L_{2h} e = R r with zero Dirichlet
    ghosts; the coarsest (`coarsest` intervals) is solved exactly.
    """
    if _cache is None:
        _cache = {}
    if n == coarsest:
        key = (n, order, h)
        if key not in _cache:
            _cache[key] = np.linalg.inv(coarse_matrix(n, order, h))
        s = slice(g, g + n - 1)
        z = u.copy()
        z[s, s, s] = 0.0
        rhs = f[s, s, s] - O.lap(z, n, h, order, g)
        u[s, s, s] = (_cache[key] @ rhs.ravel()).reshape(rhs.shape)
        return u
    for _ in range(nu1):
        smooth(u, f, n, h, order, g, forward=True)
    r = O.residual(u, f, n, h, order, g)
    rc = restrict(r)
    nc = n // 2
    mc = nc + 1 + 2 * (g - 1)
    ec = np.zeros((mc,) * 3)
    fc = np.zeros((mc,) * 3)
    sc = slice(g, g + nc - 1)
    fc[sc, sc, sc] = rc
    vcycle(ec, fc, nc, 2 * h, order, g, nu1, nu2, coarsest, _cache)
    s = slice(g, g + n - 1)
    u[s, s, s] += prolong(ec[sc, sc, sc])
    for _ in range(nu2):
        smooth(u, f, n, h, order, g, forward=False)
    return u


def omega_opt(n: int) -> float:
    """Eq. omega_final with r_J = cos(pi/N) (Eq. rjac, isotropic grid)."""
    return 2.0 / (1.0 + np.sin(np.pi / n))


def omega_opt_a(n: int) -> float:
    """Large-N approximation 2 / (1 + pi/N) (Section 2.1.1)."""
    return 2.0 / (1.0 + np.pi / n)


def omega_chebyshev(n: int, count: int):
    """Chebyshev sequence of Eq. omega_n started from n = 1:
    w1 = 1/(1 - rJ^2/2), w_{k+1} = 1/(1 - rJ^2 w_k / 4)."""
    rj = np.cos(np.pi / n)
    w = [1.0 / (1.0 - rj * rj / 2.0)]
    while len(w) < count:
        w.append(1.0 / (1.0 - rj * rj * w[-1] / 4.0))
    return w
