"""The multigrid preconditioner of the log-spherical BiCGSTAB, as one
V(nu1, nu2) cycle from a zero guess (Section 2.1.2: right-preconditioned
BiCGSTAB; Section 2.1.3: multigrid).  The paper gives no spherical
multigrid; this follows the construction chosen for it:

* levels pair the nodes two by two along every axis while nr, ntheta, nphi
  stay even (ntheta >= 4, nphi >= 8, nr >= 4) and the level holds more than
  512 unknowns; level l has spacings ds 2^l, pi / ntheta_l, 2 pi / nphi_l and
  colatitudes (j + 1/2) pi / ntheta_l; its operator is the r^2-scaled
  Laplacian rediscretised on it with zero radial ghosts;
* smoother: zebra phi-line Gauss-Seidel -- the lines (i, j) with
  (i + j) mod 2 = colour are solved exactly along the periodic phi direction
  with the r- and theta-neighbours (the other colour) held fixed; across a
  pole a line meets itself half a turn away, and that term is taken from the
  values before the pass; pre-smoothing colours 0, 1, post-smoothing 1, 0;
* restriction: mean of the 8 fine residuals a coarse node pairs; prolongation:
  injection of the coarse correction into its 8 fine nodes; coarsest level:
  a dense solve.

On a padded radial grid (radial.RadialMap in place of ds) every level takes
the radial couplings of the map rediscretised on it (RadialMap.level_couplings:
unknowns at the means of the nodes they pair, spacing doubled per level).

Test infrastructure: imported by tests only.  FP64 throughout (the GPU cycle
runs in FP32; the tests state the tolerance).
"""
from __future__ import annotations

import math

import numpy as np


def levels(nr: int, nth: int, nph: int):
    out = []
    while True:
        out.append((nr, nth, nph))
        if nr * nth * nph <= 512 or nr % 2 or nth % 2 or nph % 2 or nth < 4 or nph < 8 or nr < 4:
            break
        nr //= 2
        nth //= 2
        nph //= 2
    return out


def coefs(nth: int, nph: int, ds: float):
    dth = math.pi / nth
    dph = 2.0 * math.pi / nph
    th = (np.arange(nth) + 0.5) * dth
    cot2 = np.cos(th) / np.sin(th) / (2.0 * dth)
    aphi = 1.0 / (np.sin(th) ** 2 * dph ** 2)
    diag = -2.0 / ds ** 2 - 2.0 / dth ** 2 - 2.0 * aphi
    return dth, cot2, aphi, diag


class _Level:
    """Radial couplings of one level of a mapped radial grid."""
    def __init__(self, rmap, level, nr):
        self.rmap, self.level = rmap, level
        self.cl, self.cr = rmap.level_couplings(level, nr)

    def coarser(self, nr):
        return _Level(self.rmap, self.level + 1, nr)


def _radial(ds, nr):
    """(cl, cr) per radial unknown: from a float spacing (log grid) or a level
    of a mapped grid."""
    if isinstance(ds, (int, float)):
        return (np.full(nr, 1 / ds ** 2 - 1 / (2 * ds)), np.full(nr, 1 / ds ** 2 + 1 / (2 * ds)))
    return ds.cl, ds.cr


def level0(rmap, nr):
    """The finest level of the mapped grid rmap, to pass in place of ds."""
    return _Level(rmap, 0, nr)


def apply(u: np.ndarray, ds: float) -> np.ndarray:
    """r^2 lap u on the unknowns of u [nph][nth][nr] (zero radial ghosts)."""
    nph, nth, nr = u.shape
    dth, cot2, aphi, diag = coefs(nth, nph, ds if isinstance(ds, (int, float)) else 1.0)
    z = np.zeros((nph, nth, 1))
    up = np.concatenate([u[:, :, 1:], z], axis=2)
    um = np.concatenate([z, u[:, :, :-1]], axis=2)
    half = nph // 2
    flip = np.roll(u, -half, axis=0)
    jp = np.concatenate([u[:, 1:, :], flip[:, -1:, :]], axis=1)
    jm = np.concatenate([flip[:, :1, :], u[:, :-1, :]], axis=1)
    kp = np.roll(u, -1, axis=0)
    km = np.roll(u, 1, axis=0)
    c2 = cot2[None, :, None]
    ap = aphi[None, :, None]
    if isinstance(ds, (int, float)):
        return ((1 / ds ** 2 + 1 / (2 * ds)) * up + (1 / ds ** 2 - 1 / (2 * ds)) * um + (1 / dth ** 2 + c2) * jp
                + (1 / dth ** 2 - c2) * jm + ap * (kp + km) + diag[None, :, None] * u)
    cl, cr = ds.cl[None, None, :], ds.cr[None, None, :]
    dang = (-2.0 / dth ** 2 - 2.0 * aphi)[None, :, None]
    return (cr * up + cl * um + (1 / dth ** 2 + c2) * jp + (1 / dth ** 2 - c2) * jm + ap * (kp + km)
            + (dang - (cl + cr)) * u)


def line_pass(u: np.ndarray, f: np.ndarray, ds: float, colour: int) -> np.ndarray:
    """Solve every line (i, j) of the colour exactly along phi, in place."""
    nph, nth, nr = u.shape
    dth, cot2, aphi, _ = coefs(nth, nph, 1.0)
    cl, cr = _radial(ds, nr)
    half = nph // 2
    old = u.copy()
    for j in range(nth):
        for i in range(nr):
            if (i + j) % 2 != colour:
                continue
            C = np.zeros((nph, nph))
            for k in range(nph):
                C[k, k] = -(cl[i] + cr[i]) - 2.0 / dth ** 2 - 2.0 * aphi[j]
                C[k, (k + 1) % nph] += aphi[j]
                C[k, (k - 1) % nph] += aphi[j]
            ip = old[:, j, i + 1] if i + 1 < nr else np.zeros(nph)
            im = old[:, j, i - 1] if i > 0 else np.zeros(nph)
            jp = old[:, j + 1, i] if j + 1 < nth else np.roll(old[:, j, i], -half)
            jm = old[:, j - 1, i] if j > 0 else np.roll(old[:, j, i], -half)
            rhs = f[:, j, i] - (cr[i] * ip + cl[i] * im
                                + (1 / dth ** 2 + cot2[j]) * jp + (1 / dth ** 2 - cot2[j]) * jm)
            u[:, j, i] = np.linalg.solve(C, rhs)
    return u


def restrict(r: np.ndarray) -> np.ndarray:
    return 0.125 * sum(r[a::2, b::2, c::2] for a in (0, 1) for b in (0, 1) for c in (0, 1))


def prolong(e: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(np.repeat(e, 2, 0), 2, 1), 2, 2)


def dense_matrix(nr: int, nth: int, nph: int, ds: float) -> np.ndarray:
    N = nr * nth * nph
    A = np.zeros((N, N))
    for col in range(N):
        x = np.zeros(N)
        x[col] = 1.0
        A[:, col] = apply(x.reshape(nph, nth, nr), ds).ravel()
    return A


def vcycle(f: np.ndarray, ds: float, nu1: int = 2, nu2: int = 2, _lv=None, _cache=None) -> np.ndarray:
    """One V(nu1, nu2) cycle for r^2 lap u = f from u = 0; f is [nph][nth][nr]."""
    nph, nth, nr = f.shape
    if _lv is None:
        _lv = levels(nr, nth, nph)
    if _cache is None:
        _cache = {}
    if len(_lv) == 1:
        key = (nr, nth, nph, ds if isinstance(ds, (int, float)) else (id(ds.rmap), ds.level))
        if key not in _cache:
            _cache[key] = np.linalg.inv(dense_matrix(nr, nth, nph, ds))
        return (_cache[key] @ f.ravel()).reshape(f.shape)
    u = np.zeros_like(f)
    for _ in range(nu1):
        for c in (0, 1):
            line_pass(u, f, ds, c)
    r = f - apply(u, ds)
    coarse = 2.0 * ds if isinstance(ds, (int, float)) else ds.coarser(_lv[1][0])
    e = vcycle(restrict(r), coarse, nu1, nu2, _lv[1:], _cache)
    u += prolong(e)
    for _ in range(nu2):
        for c in (1, 0):
            line_pass(u, f, ds, c)
    return u
