"""The exact discrete solution every iterative solver converges to.

For a Dirichlet problem the iterative methods of Section 2.1 (SOR, CG,
BiCGSTAB, multigrid) all approach the unique solution of A u = b, where A is
the discrete Laplacian restricted to the unknowns and b is 4 pi G rho minus
the couplings to the known ghost values (Section 2.2).  The oracle computes
that solution directly:

* 7-point Cartesian: the DST-I diagonalises A (eigenvalues
  sum_d (2 cos(pi k_d / n) - 2) / h^2) -- a textbook exact solve.
* 19-point star: conjugate gradients on -A preconditioned by the 7-point
  DST solve, run to a relative residual of 1e-14 (the spectrum of the
  preconditioned operator lies in [1, 1.52], so this takes ~15 steps).
* log-spherical: an FFT in phi separates azimuthal modes m; the pole
  reflection (phi + pi) becomes a factor (-1)^m; each mode is a real sparse
  2-D system in (theta, s) solved by sparse LU.
* dense: brute-force assembly of A by applying the operator to unit vectors
  and a LAPACK solve, for small grids; used to pin the three above.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import operators as O
from . import smoothers as S


def _workers():
    import os
    return os.cpu_count() or 1


def dst_solve7(rhs: np.ndarray, n: int, h: float) -> np.ndarray:
    """Solve L7 u = rhs on (n-1)^3 unknowns with zero Dirichlet ghosts."""
    k = np.arange(1, n, dtype=np.float64)
    lam = (2.0 * np.cos(np.pi * k / n) - 2.0) / (h * h)
    hat = sfft.dstn(rhs, type=1, norm="ortho", workers=_workers())
    hat /= lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    return sfft.idstn(hat, type=1, norm="ortho", workers=_workers())


def _ghost_rhs(phi_ghost, f_nodes, n, h, order, g):
    s = slice(g, g + n - 1)
    z = phi_ghost.copy()
    z[s, s, s] = 0.0
    return f_nodes[s, s, s] - O.lap(z, n, h, order, g)


def pcg19(rhs, n, h, tol=1e-14, maxit=200):
    """Solve L19 u = rhs (zero ghosts) by CG on -L19, preconditioned by the
    7-point DST solve.  Returns (u, iterations, final relative residual)."""
    g = 3
    m = n + 1 + 2 * (g - 1)
    s = slice(g, g + n - 1)
    work = np.zeros((m, m, m))

    def A(v):  # -L19 v with zero ghosts
        work[s, s, s] = v
        return -O.lap19(work, n, h, g)

    def Minv(v):  # (-L7)^-1 v
        return -dst_solve7(v, n, h)

    b = -rhs
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, 0.0
    z = Minv(r)
    p = z.copy()
    rz = np.vdot(r, z)
    it = 0
    rel = 1.0
    while it < maxit:
        q = A(p)
        alpha = rz / np.vdot(p, q)
        x += alpha * p
        r -= alpha * q
        it += 1
        rel = np.linalg.norm(r) / bn
        if rel <= tol:
            break
        z = Minv(r)
        rz_new = np.vdot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    # report the true residual of the returned iterate
    rel = np.linalg.norm(b - A(x)) / bn
    return x, it, rel


def solve_cart(phi_ghost, rho_nodes, n, h, order, g, four_pi_G=1.0):
    """Exact Cartesian solution; phi_ghost holds the Dirichlet ghost values.
    Returns the full node array (ghosts kept, unknowns solved)."""
    f = four_pi_G * rho_nodes
    rhs = _ghost_rhs(phi_ghost, f, n, h, order, g)
    if order == 2:
        u = dst_solve7(rhs, n, h)
    else:
        u, _, _ = pcg19(rhs, n, h)
    out = phi_ghost.copy()
    s = slice(g, g + n - 1)
    out[s, s, s] = u
    return out


def dense_solve_cart(phi_ghost, rho_nodes, n, h, order, g, four_pi_G=1.0):
    """Brute force: assemble A from unit vectors, LAPACK solve.  Small n."""
    f = four_pi_G * rho_nodes
    rhs = _ghost_rhs(phi_ghost, f, n, h, order, g)
    A = S.coarse_matrix(n, order, h)
    u = np.linalg.solve(A, rhs.ravel()).reshape(rhs.shape)
    out = phi_ghost.copy()
    s = slice(g, g + n - 1)
    out[s, s, s] = u
    return out


# --------------------------------------------------------------------------
# log-spherical
# --------------------------------------------------------------------------
def _sph_mode_matrix(m, nph, nth, nr, ds, th):
    dth = math.pi / nth
    dph = 2 * math.pi / nph
    cot = np.cos(th) / np.sin(th)
    sgn = -1.0 if (m % 2) else 1.0
    N = nth * nr
    rows, cols, vals = [], [], []

    def add(a, b, v):
        rows.append(a)
        cols.append(b)
        vals.append(v)

    for j in range(nth):
        sphi = (2.0 * math.cos(2 * math.pi * m / nph) - 2.0) / (dph ** 2 * math.sin(th[j]) ** 2)
        cjm = 1.0 / dth ** 2 - cot[j] / (2 * dth)
        cjp = 1.0 / dth ** 2 + cot[j] / (2 * dth)
        for i in range(nr):
            row = j * nr + i
            if isinstance(ds, (int, float)):
                cl, cr = 1.0 / ds ** 2 - 1.0 / (2 * ds), 1.0 / ds ** 2 + 1.0 / (2 * ds)
            else:
                cl, cr = ds.cl[i], ds.cr[i]
            diag = -(cl + cr) - 2.0 / dth ** 2 + sphi
            if i + 1 < nr:
                add(row, row + 1, cr)
            if i - 1 >= 0:
                add(row, row - 1, cl)
            if j + 1 < nth:
                add(row, row + nr, cjp)
            else:
                diag += sgn * cjp
            if j - 1 >= 0:
                add(row, row - nr, cjm)
            else:
                diag += sgn * cjm
            add(row, row, diag)
    return sp.csc_matrix((vals, (rows, cols)), shape=(N, N))


def solve_sph(phi_ghost, rho_nodes, r, ds, th, four_pi_G=1.0):
    """Exact solution on the spherical grid (ds: log spacing or a
    radial.RadialMap); phi_ghost [nph][nth][nr+2] carries the radial ghost
    values.  Returns the full array."""
    nph, nth, m2 = phi_ghost.shape
    nr = m2 - 2
    z = phi_ghost.copy()
    z[:, :, 1:nr + 1] = 0.0
    rhs = O.sph_residual(z, rho_nodes, r, ds, th, four_pi_G)
    hat = np.fft.rfft(rhs, axis=0)
    sol = np.empty_like(hat)
    for m in range(hat.shape[0]):
        lu = spla.splu(_sph_mode_matrix(m, nph, nth, nr, ds, th))
        b = hat[m].reshape(-1)
        sol[m] = (lu.solve(np.ascontiguousarray(b.real))
                  + 1j * lu.solve(np.ascontiguousarray(b.imag))).reshape(nth, nr)
    out = phi_ghost.copy()
    out[:, :, 1:nr + 1] = np.fft.irfft(sol, n=nph, axis=0)
    return out


def dense_solve_sph(phi_ghost, rho_nodes, r, ds, th, four_pi_G=1.0):
    """Brute force on a small spherical grid: assemble from unit vectors."""
    nph, nth, m2 = phi_ghost.shape
    nr = m2 - 2
    N = nph * nth * nr
    z = phi_ghost.copy()
    z[:, :, 1:nr + 1] = 0.0
    rhs = O.sph_residual(z, rho_nodes, r, ds, th, four_pi_G)
    A = np.zeros((N, N))
    u = np.zeros_like(phi_ghost)
    for col in range(N):
        k, rem = divmod(col, nth * nr)
        j, i = divmod(rem, nr)
        u[k, j, 1 + i] = 1.0
        A[:, col] = O.sph_apply(u, ds, th).ravel()
        u[k, j, 1 + i] = 0.0
    x = np.linalg.solve(A, rhs.ravel()).reshape(nph, nth, nr)
    out = phi_ghost.copy()
    out[:, :, 1:nr + 1] = x
    return out
