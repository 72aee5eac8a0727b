"""Pins of the oracle's conjugate gradients with the multi-colour
Gauss-Seidel preconditioner (Section 2.1.2)."""
import numpy as np
import pytest

from oracle import direct as D
from oracle import krylov as K

CASES = [(2, 6, 1), (6, 8, 3)]   # (order, n, ghost layers)


def _dense_A(n, h, order, g):
    e = n - 1
    N = e ** 3
    A = np.zeros((N, N))
    for col in range(N):
        x = np.zeros(N)
        x[col] = 1.0
        A[:, col] = K._apply_A(x.reshape(e, e, e), n, h, order, g).ravel()
    return A


def _colours(n, order):
    """(i + j + k) mod C over the unknowns, global node indices 1..n-1."""
    i = np.arange(1, n)
    s = i[:, None, None] + i[None, :, None] + i[None, None, :]
    return (s % K.ncolours(order)).ravel()


@pytest.mark.parametrize("order,n,g", CASES)
def test_sweeps_are_the_block_triangular_preconditioners(order, n, g):
    """The forward sweep applies B^-1 and the symmetric step (B D^-1 B^T)^-1,
    with B the block lower triangle of A in colour order (diagonal blocks
    plus the couplings to lower colours), assembled here from the dense A."""
    h = 1.0 / n
    A = _dense_A(n, h, order, g)
    col = _colours(n, order)
    assert np.all(A[col[:, None] == col[None, :]] * (1 - np.eye(len(col)))[col[:, None] == col[None, :]] == 0.0)
    B = np.where(col[:, None] > col[None, :], A, 0.0) + np.diag(np.diag(A))
    M = B @ np.diag(1.0 / np.diag(A)) @ B.T
    res = np.random.default_rng(order).normal(size=(n - 1,) * 3)
    rho = -res.ravel()
    zf = K.forward_sweep(res, n, h, order, g).ravel()
    zs = K.sgs(res, n, h, order, g).ravel()
    assert np.max(np.abs(zf - np.linalg.solve(B, rho))) < 1e-12 * np.max(np.abs(zf))
    assert np.max(np.abs(zs - np.linalg.solve(M, rho))) < 1e-12 * np.max(np.abs(zs))


@pytest.mark.parametrize("order,n,g", CASES)
def test_symmetric_step_is_spd_and_forward_sweep_is_not_symmetric(order, n, g):
    """Column by column from unit vectors: the symmetric step's matrix is
    symmetric and positive definite (as CG requires); the forward sweep's is
    not symmetric."""
    h = 1.0 / n
    e = n - 1
    N = e ** 3
    Zs = np.zeros((N, N))
    Zf = np.zeros((N, N))
    for c in range(N):
        x = np.zeros(N)
        x[c] = -1.0                       # rho = e_c
        Zs[:, c] = K.sgs(x.reshape(e, e, e), n, h, order, g).ravel()
        Zf[:, c] = K.forward_sweep(x.reshape(e, e, e), n, h, order, g).ravel()
    scale = np.max(np.abs(Zs))
    assert np.max(np.abs(Zs - Zs.T)) < 1e-13 * scale
    assert np.min(np.linalg.eigvalsh(0.5 * (Zs + Zs.T))) > 0.0
    assert np.max(np.abs(Zf - Zf.T)) > 1e-3 * np.max(np.abs(Zf))


def _problem(n, g, seed):
    rng = np.random.default_rng(seed)
    m = n + 1 + 2 * (g - 1)
    phi = rng.normal(size=(m, m, m))
    s = slice(g, g + n - 1)
    phi[s, s, s] = 0.0
    rho = rng.normal(size=(m, m, m))
    return phi, rho


@pytest.mark.parametrize("order,g", [(2, 1), (6, 3)])
def test_pcg_reaches_the_exact_solution_with_fewer_iterations(order, g):
    n = 16
    h = 1.0 / n
    phi, rho = _problem(n, g, 7 + order)
    exact = D.solve_cart(phi, rho, n, h, order, g)
    x, it, rel = K.cg(phi, rho, n, h, order, g, tol=1e-12)
    x0, it0, rel0 = K.cg(phi, rho, n, h, order, g, tol=1e-12, precondition=False)
    s = slice(g, g + n - 1)
    scale = np.max(np.abs(exact[s, s, s]))
    assert rel <= 1e-12 and rel0 <= 1e-12
    assert np.max(np.abs(x[s, s, s] - exact[s, s, s])) < 1e-10 * scale
    assert np.max(np.abs(x0[s, s, s] - exact[s, s, s])) < 1e-10 * scale
    assert it < 0.75 * it0, (it, it0)


@pytest.mark.parametrize("order,g", [(2, 1), (6, 3)])
def test_pcg_error_decreases_in_the_energy_norm(order, g):
    """CG minimises ||x* - x_m||_A over its Krylov space, which grows each
    iteration: the energy norm of the error cannot increase."""
    n = 10
    h = 1.0 / n
    phi, rho = _problem(n, g, 3)
    exact = D.solve_cart(phi, rho, n, h, order, g)
    s = slice(g, g + n - 1)
    hist = []
    K.cg(phi, rho, n, h, order, g, tol=1e-13, history=hist)
    en = []
    for xm in hist:
        e = exact[s, s, s] - xm
        en.append(float(np.sum(e * K._apply_A(e, n, h, order, g))))
    en = np.sqrt(np.maximum(en, 0.0))
    assert len(en) > 5
    assert np.all(np.diff(en) <= 1e-12 * en[0])
