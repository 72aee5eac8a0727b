"""SPAI-smoothed multigrid on compact radius-1 stencils with Galerkin coarse
operators, and the local Fourier analysis of the smoother (Section 2.1.3:
Eq. richardson, Eq. Smoother, Table 1, the Galerkin operator A_{i+1} =
R A_i R^T, the compact stencils of Section 2.1.3's last paragraphs).

Test infrastructure: imported by tests and the benchmark's CPU baseline only.

Conventions.  A cubically symmetric radius-1 stencil is four weights
(centre, face, edge, corner): applied to u at node n it gives
w0 u_n + wf (6 face neighbours) + we (12 edge neighbours) + wc (8 corners).
Operators here approximate the Laplacian L_h (negative definite); the paper's
SPD operator is A = -L_h.  With r = f - L_h u the Richardson step
u <- (I - w M A) u + w M b (b = -f) reads u <- u - w M r.

Compact discretisations (weights times 1/h^2, right-hand side operator B):
  order 2: 7-point  (-6, 1, 0, 0),           B f = f;
  order 4: 19-point (-24, 2, 1, 0) / 6,      B f = (6 f_n + sum of 6 faces) / 12
           (the Mehrstellen scheme; L u = B (lap u) is exact for
           polynomials of degree <= 5);
  order 6: 27-point (-128, 14, 3, 1) / 30 (the isotropic compact sixth-order
           scheme the paper cites for Section 2.1.3).  Its truncation error
           for lap u = f is (h^2/12) lap f + (h^4/360) (sum_d f_dddd +
           4 sum_{d<e} f_ddee) + O(h^6), so B adds exactly that:
           B f = f + (1/12) sum_d D_d f - (1/240) sum_d D_d D_d f
                   + (1/90) sum_{d<e} D_d D_e f,
           D_d the unit-spacing second difference along axis d.  The paper
           does not give its right-hand side; this one reads f two nodes
           beyond the unknowns (the density's second ghost layer) and makes
           L u = B (lap u) exact for polynomials of degree <= 7.

M(alpha, beta, gamma, delta) = h^2 * stencil (alpha, beta, gamma, delta)
(Eq. Smoother); every level uses its own spacing h_l and the same
coefficients.  With store32 the levels below the finest keep their data in
FP32 and compute in FP64 (the paper's mixed precision): every stored value
is rounded to FP32 where it is written.  Coarse operators are Galerkin products R A_l P with full
weighting R and P = 8 R^T (trilinear), which for the stencils here stay
radius 1 and cubically symmetric.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import smoothers as S

# Table 1: order -> (omega, alpha, beta, gamma, delta, mu) as printed
TABLE1 = {
    2: (1.3699, 0.1432, 0.0284, 0.0081, 0.0025, 0.1888),
    4: (0.9363, 0.2807, 0.0329, 0.0166, 0.0044, 0.0828),
    6: (0.3543, 0.7064, 0.1005, 0.0363, 0.0909, 0.0909),
}

# compact Laplacians, weights times 1/h^2
WEIGHTS = {
    2: (-6.0, 1.0, 0.0, 0.0),
    4: (-24.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0, 0.0),
    6: (-128.0 / 30.0, 14.0 / 30.0, 3.0 / 30.0, 1.0 / 30.0),
}

# Smoother coefficients (omega, alpha, beta, gamma, delta) used by the
# method.  Orders 2 and 4: Table 1 as printed.  Order 6: the printed delta
# cell repeats mu and makes the smoother diverge; delta = 0.0151 is the value
# that minimises the smoothing factor with the other four printed
# coefficients kept (mu = 0.0912 against the printed 0.0909).
COEFFS = {
    2: TABLE1[2][:5],
    4: TABLE1[4][:5],
    6: TABLE1[6][:4] + (0.0151,),
}

OFFSETS = [d for d in itertools.product((-1, 0, 1), repeat=3)]


def weight_of(w, d):
    """Weight of offset d = (dk, dj, di) in the stencil w."""
    return w[sum(1 for x in d if x != 0)]


def apply27(u: np.ndarray, n: int, w, scale: float = 1.0) -> np.ndarray:
    """Stencil w (times scale) applied at the unknown nodes of a node array
    with one ghost layer; returns shape (n-1)^3."""
    e = n - 1
    out = np.zeros((e, e, e))
    for d in OFFSETS:
        c = weight_of(w, d)
        if c != 0.0:
            out += c * u[1 + d[0]:1 + d[0] + e, 1 + d[1]:1 + d[1] + e, 1 + d[2]:1 + d[2] + e]
    return scale * out


def embed(x_int: np.ndarray) -> np.ndarray:
    """Interior values -> node array with zero ghosts."""
    e = x_int.shape[0]
    u = np.zeros((e + 2,) * 3)
    u[1:-1, 1:-1, 1:-1] = x_int
    return u


def rhs_compact(f_nodes: np.ndarray, n: int, order: int) -> np.ndarray:
    """B f at the unknown nodes.  Orders 2 and 4: f_nodes holds nodes 0..n
    (shape (n+1)^3); order 6: nodes -1..n+1 (shape (n+3)^3)."""
    if order == 2:
        return f_nodes[1:n, 1:n, 1:n].copy()
    if order == 4:
        return apply27(f_nodes, n, (6.0 / 12.0, 1.0 / 12.0, 0.0, 0.0))
    if order != 6:
        raise ValueError("compact orders are 2, 4 and 6")
    if f_nodes.shape != (n + 3,) * 3:
        raise ValueError("order 6 needs f on nodes -1..n+1")

    def sh(dk, dj, di):
        # f shifted by (dk, dj, di) nodes, at the unknowns 1..n-1
        return f_nodes[2 + dk:n + 1 + dk, 2 + dj:n + 1 + dj, 2 + di:n + 1 + di]

    axes = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]

    def along(e, s):
        return sh(e[0] * s, e[1] * s, e[2] * s)

    f0 = sh(0, 0, 0)
    d2 = [along(e, 1) - 2.0 * f0 + along(e, -1) for e in axes]
    d4 = [along(e, 2) - 4.0 * along(e, 1) + 6.0 * f0 - 4.0 * along(e, -1) + along(e, -2) for e in axes]
    mixed = 0.0
    for a in range(3):
        for b in range(a + 1, 3):
            ea, eb = axes[a], axes[b]
            corners = sum(sh(sa * ea[0] + sb * eb[0], sa * ea[1] + sb * eb[1], sa * ea[2] + sb * eb[2])
                          for sa in (-1, 1) for sb in (-1, 1))
            # D_a D_b f: the 3 x 3 tensor product of (1, -2, 1) in the (a, b) plane
            mixed = mixed + corners - 2.0 * (along(ea, 1) + along(ea, -1) + along(eb, 1) + along(eb, -1)) + 4.0 * f0
    return f0 + sum(d2) / 12.0 - sum(d4) / 240.0 + mixed / 90.0


def symbol(w, kx, ky, kz):
    """Fourier symbol of the stencil w (h = 1) at frequencies (kx, ky, kz)."""
    cx, cy, cz = np.cos(kx), np.cos(ky), np.cos(kz)
    return (w[0] + 2.0 * w[1] * (cx + cy + cz) + 4.0 * w[2] * (cx * cy + cy * cz + cz * cx)
            + 8.0 * w[3] * cx * cy * cz)


def smoother_symbol(order_w, coef, kx, ky, kz):
    """S~(k) = 1 - omega M~(k) A~(k) with A = -L (Eq. richardson)."""
    omega, alpha, beta, gamma, delta = coef[:5]
    return 1.0 - omega * symbol((alpha, beta, gamma, delta), kx, ky, kz) * (-symbol(order_w, kx, ky, kz))


def smoothing_factor(order_w, coef, N: int = 64) -> float:
    """mu = max of |S~(k)| over the high frequencies of an N-periodic grid:
    theta_j = 2 pi j / N with at least one |theta| > pi/2, i.e. the discrete
    version of T = [-pi, pi]^3 minus [-pi/2, pi/2]^3.  (The supremum over the
    continuous set is approached at the inner edge (pi/2, 0, 0) and is larger.)"""
    k = 2.0 * np.pi * np.arange(-(N // 2), N // 2 + 1) / N
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    high = (np.abs(kx) > np.pi / 2) | (np.abs(ky) > np.pi / 2) | (np.abs(kz) > np.pi / 2)
    return float(np.abs(smoother_symbol(order_w, coef, kx, ky, kz))[high].max())


def galerkin(w):
    """Weights of R A P for the operator A = stencil w (absolute weights) on
    the fine level: A is applied to the prolongation of a unit coarse vector
    at the centre of a 16-interval fine grid (the stencil has constant
    coefficients, so the grid size does not matter), the result restricted,
    and the coarse stencil read off around the centre."""
    n = 16
    nc = n // 2
    ec = np.zeros((nc - 1,) * 3)
    cI = nc // 2 - 1
    ec[cI, cI, cI] = 1.0
    fine = S.prolong(ec)
    a = apply27(embed(fine), n, w)
    col = S.restrict(a)
    out = {}
    for d in OFFSETS:
        out[d] = col[cI + d[0], cI + d[1], cI + d[2]]
    mask = np.ones_like(col, dtype=bool)
    mask[cI - 1:cI + 2, cI - 1:cI + 2, cI - 1:cI + 2] = False
    if np.max(np.abs(col[mask])) > 1e-12 * np.max(np.abs(col)):
        raise AssertionError("Galerkin operator is not radius 1")
    wc = [None] * 4
    for d, v in out.items():
        cls = sum(1 for x in d if x != 0)
        if wc[cls] is None:
            wc[cls] = v
        elif abs(wc[cls] - v) > 1e-12 * abs(out[(0, 0, 0)]):
            raise AssertionError("Galerkin operator is not cubically symmetric")
    return tuple(float(x) for x in wc)


def level_operators(order: int, n: int, coarsest: int = 8):
    """Per level l (n, n/2, ..., coarsest): the operator weights as absolute
    values (fine: WEIGHTS/h^2; coarse: Galerkin products)."""
    h = 1.0 / n
    ops = [tuple(x / (h * h) for x in WEIGHTS[order])]
    m = n
    while m > coarsest:
        ops.append(galerkin(ops[-1]))
        m //= 2
    return ops


def _stored(x, store32: bool):
    """Value as stored: rounded to FP32 when the level keeps FP32 data."""
    return x.astype(np.float32).astype(np.float64) if store32 else x


def spai_step(u: np.ndarray, f_int: np.ndarray, n: int, w_abs, coef, h: float, store32: bool = False) -> np.ndarray:
    """One Richardson step u <- u - omega M r, r = f - A_L u, in place on the
    unknowns of the node array u (ghosts fixed); M acts on r extended by zero.
    store32: the level stores r and u in FP32 (arithmetic stays FP64)."""
    omega, alpha, beta, gamma, delta = coef[:5]
    r = _stored(f_int - apply27(u, n, w_abs), store32)
    u[1:n, 1:n, 1:n] = _stored(u[1:n, 1:n, 1:n] - omega * apply27(embed(r), n, (alpha, beta, gamma, delta), h * h),
                               store32)
    return u


def coarse_dense(w_abs, n: int) -> np.ndarray:
    """Dense matrix of the stencil on the (n-1)^3 unknowns, zero ghosts."""
    e = n - 1
    A = np.zeros((e ** 3, e ** 3))
    for col in range(e ** 3):
        x = np.zeros(e ** 3)
        x[col] = 1.0
        A[:, col] = apply27(embed(x.reshape(e, e, e)), n, w_abs).ravel()
    return A


def cg_coarse(w_abs, b: np.ndarray, n: int, rtol: float, maxit: int = 10000):
    """Conjugate gradients on A = -stencil (SPD) from a zero guess, stopped
    once ||b - L x|| <= rtol ||b|| (Section 2.1.2's CG, used as the coarsest
    solve of Section 2.1.3).  Returns (x, iterations)."""
    x = np.zeros_like(b)
    r = b.copy()            # residual of L x = b with x = 0
    p = r.copy()
    rr = float(np.sum(r * r))
    stop = rtol * rtol * rr
    it = 0
    while rr > stop and it < maxit:
        q = -apply27(embed(p), n, w_abs)      # A p with A = -L
        alpha = rr / float(np.sum(p * q))
        x = x - alpha * p                     # L x = b  <=>  A x = -b
        r = r - alpha * q
        rr_new = float(np.sum(r * r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def vcycle(u, f_int, n, ops, coef, nu1=3, nu2=3, level=0, _cache=None, store32=False, coarse_rtol=0.0):
    """One V(nu1, nu2) cycle with SPAI smoothing and Galerkin coarse
    operators on the node array u (one ghost layer, ghosts fixed); f_int is
    the right-hand side at the unknowns.  The coarsest level is solved
    exactly (dense), or by CG to relative accuracy coarse_rtol when that is
    positive.  store32: every level below the finest stores its data
    (u, f, r) in FP32 while all arithmetic stays FP64 (Section 2.1.3's mixed
    precision)."""
    if _cache is None:
        _cache = {}
    h = 1.0 / n
    w = ops[level]
    s32 = store32 and level > 0
    if level == len(ops) - 1:
        z = u.copy()
        z[1:n, 1:n, 1:n] = 0.0
        rhs = f_int - apply27(z, n, w)
        if coarse_rtol > 0.0:
            x, _ = cg_coarse(w, rhs, n, coarse_rtol)
            u[1:n, 1:n, 1:n] = _stored(x, s32)
            return u
        key = (n, w)
        if key not in _cache:
            _cache[key] = np.linalg.inv(coarse_dense(w, n))
        u[1:n, 1:n, 1:n] = _stored((_cache[key] @ rhs.ravel()).reshape(rhs.shape), s32)
        return u
    for _ in range(nu1):
        spai_step(u, f_int, n, w, coef, h, s32)
    r = _stored(f_int - apply27(u, n, w), s32)
    nc = n // 2
    rc = _stored(S.restrict(r), store32)
    ec = np.zeros((nc + 1,) * 3)
    vcycle(ec, rc, nc, ops, coef, nu1, nu2, level + 1, _cache, store32, coarse_rtol)
    u[1:n, 1:n, 1:n] = _stored(u[1:n, 1:n, 1:n] + S.prolong(ec[1:nc, 1:nc, 1:nc]), s32)
    for _ in range(nu2):
        spai_step(u, f_int, n, w, coef, h, s32)
    return u


def dst_solve(w_abs, rhs: np.ndarray, n: int) -> np.ndarray:
    """Exact solve of a cubically symmetric radius-1 stencil with zero
    Dirichlet ghosts: sine modes are its eigenvectors (DST-I)."""
    import scipy.fft as sfft
    k = np.arange(1, n, dtype=np.float64) * np.pi / n
    lam = symbol(w_abs, k[:, None, None], k[None, :, None], k[None, None, :])
    hat = sfft.dstn(rhs, type=1, norm="ortho")
    return sfft.idstn(hat / lam, type=1, norm="ortho")


def solve_cart(phi_ghost, f_nodes, n, order):
    """Exact discrete solution of L u = B f with the ghost values of
    phi_ghost (one layer) and f = 4 pi G rho at every node (order 6: one
    more layer of f, see rhs_compact)."""
    h = 1.0 / n
    w = tuple(x / (h * h) for x in WEIGHTS[order])
    z = phi_ghost.copy()
    z[1:n, 1:n, 1:n] = 0.0
    rhs = rhs_compact(f_nodes, n, order) - apply27(z, n, w)
    out = phi_ghost.copy()
    out[1:n, 1:n, 1:n] = dst_solve(w, rhs, n)
    return out
