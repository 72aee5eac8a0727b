"""Conjugate gradients on the Cartesian operators, plain and preconditioned by
multi-colour Gauss-Seidel (Section 2.1.2).

Test infrastructure: imported by tests only.  FP64 throughout.

System.  The unknowns u of the vertex-centred grid solve L u = f with the
ghost layers fixed; with A = -L (symmetric positive definite on the
unknowns) and b = -(f - L u0) for the ghost-only part, CG runs on A in the
textbook form: residual rho = b - A x = -(f - L u), so rho is the negative of
operators.residual.

Preconditioner.  The grid is coloured so that no node couples to a node of
its own colour (two colours for the 7-point operator, four for the 19-point
star).  In colour order A has diagonal blocks D_c and couplings N_cd; the
section's preconditioner is the block lower triangle B (D_c on the
diagonal, N_cd below it), applied by one forward sweep over the colours from
a zero guess.  CG needs a symmetric positive definite preconditioner, so the
sweep is symmetrised: forward over the colours, then backward (the textbook
symmetric Gauss-Seidel M = B D^-1 B^T).  The backward sweep's first colour
would recompute the forward sweep's last colour from unchanged neighbours,
so it is left out: colours 0 .. C-1, then C-2 .. 0.
"""
from __future__ import annotations

import numpy as np

from . import operators as O
from . import smoothers as S


def ncolours(order: int) -> int:
    return 2 if order == 2 else 4


def colour_sweeps(order: int):
    """Colour order of one symmetric multi-colour Gauss-Seidel step."""
    c = ncolours(order)
    return list(range(c)) + list(range(c - 2, -1, -1))


def _pass(z, f, n, h, order, g, colour):
    if order == 2:
        return S.rb_pass(z, f, n, h, colour, 1.0, g)
    return S.star_pass(z, f, n, h, colour, g)


def sgs(res: np.ndarray, n: int, h: float, order: int, g: int) -> np.ndarray:
    """One symmetric multi-colour Gauss-Seidel step for L z = res from z = 0
    with zero ghosts; res holds the (n-1)^3 unknowns.  Returns z on the
    unknowns: z = M^-1 rho for rho = -res, the CG residual."""
    m = n + 1 + 2 * (g - 1)
    s = slice(g, g + n - 1)
    f = np.zeros((m, m, m))
    f[s, s, s] = res
    z = np.zeros((m, m, m))
    for c in colour_sweeps(order):
        _pass(z, f, n, h, order, g, c)
    return z[s, s, s].copy()


def forward_sweep(res: np.ndarray, n: int, h: float, order: int, g: int) -> np.ndarray:
    """The section's B: one forward multi-colour sweep from z = 0 (z = B^-1 rho)."""
    m = n + 1 + 2 * (g - 1)
    s = slice(g, g + n - 1)
    f = np.zeros((m, m, m))
    f[s, s, s] = res
    z = np.zeros((m, m, m))
    for c in range(ncolours(order)):
        _pass(z, f, n, h, order, g, c)
    return z[s, s, s].copy()


def _apply_A(p: np.ndarray, n: int, h: float, order: int, g: int) -> np.ndarray:
    """A p = -L p on the unknowns, zero ghosts."""
    m = n + 1 + 2 * (g - 1)
    s = slice(g, g + n - 1)
    u = np.zeros((m, m, m))
    u[s, s, s] = p
    return -O.lap(u, n, h, order, g)


def cg(phi, f_nodes, n, h, order, g, tol=1e-12, max_iter=10000, precondition=True, history=None):
    """(P)CG from the initial guess phi (ghosts hold the boundary values);
    stops when ||rho|| <= tol ||rho(unknowns = 0)|| or after max_iter
    iterations.  Returns (phi, iterations, relative residual); history, if a
    list, receives each iterate's unknowns."""
    s = slice(g, g + n - 1)
    x = phi.copy()
    bnorm = O.rhs_norm(x, f_nodes, n, h, order, g)
    rho = -O.residual(x, f_nodes, n, h, order, g)
    zeta = sgs(-rho, n, h, order, g) if precondition else rho.copy()
    gamma = float(np.sum(rho * zeta))
    p = zeta.copy()
    rel = float(np.linalg.norm(rho)) / bnorm if bnorm > 0 else 0.0
    it = 0
    while it < max_iter and rel > tol:
        q = _apply_A(p, n, h, order, g)
        alpha = gamma / float(np.sum(p * q))
        x[s, s, s] += alpha * p
        rho = rho - alpha * q
        it += 1
        if history is not None:
            history.append(x[s, s, s].copy())
        rel = float(np.linalg.norm(rho)) / bnorm
        zeta = sgs(-rho, n, h, order, g) if precondition else rho.copy()
        gamma_new = float(np.sum(rho * zeta))
        p = zeta + (gamma_new / gamma) * p
        gamma = gamma_new
    return x, it, rel
