"""Seeded synthetic inputs shaped like the paper's self-gravity workloads.

This module only *generates inputs*: node coordinates of the grids and density
fields sampled at those nodes.  It contains none of the solver's arithmetic
(no Laplacian, no multipole, no iteration) and is the only code shared by the
CPU oracle and the GPU path.

Grid convention (vertex-centred): a Cartesian grid of ``n`` intervals per axis
on the box ``[lo, hi]^3`` has nodes ``i = -(g-1) .. n+(g-1)`` at
``x_i = lo + i*h`` with ``h = (hi-lo)/n``.  Nodes ``1..n-1`` are unknowns,
nodes ``<= 0`` and ``>= n`` hold Dirichlet (ghost) values; ``g`` is the stencil
radius (1 for the 7-point, 3 for the 19-point star).  Arrays are indexed
``[k][j][i]`` (x fastest).

The log-spherical grid (Section 3.3, Eq. 2) has ``nr`` radial unknowns at
``s_i = ln(r_min) + i*ds`` (``i = 0..nr-1``, ``ds = ln(r_max/r_min)/(nr-1)``)
plus one radial ghost on each side, ``nth`` colatitudes
``theta_j = (j+1/2)*pi/nth`` and ``nph`` periodic longitudes
``phi_k = 2*pi*k/nph``.  Arrays are ``[k][j][i]`` with i over ``-1..nr``.

Random numbers come from ``numpy.random.default_rng(seed)`` in a fixed draw
order (centres, widths, masses, floor field, phase); field evaluation can run
on any torch device in float64, so that both sides of a comparison can be fed
the very same array.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Iterator, List, Optional

import numpy as np
import torch

FOUR_PI_G = 1.0  # 4*pi*G = 1 in every workload


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class CartGrid:
    n: int                 # intervals per axis
    g: int = 1             # ghost layers (stencil radius)
    lo: float = 0.0
    hi: float = 1.0

    @property
    def h(self) -> float:
        return (self.hi - self.lo) / self.n

    @property
    def nodes(self) -> int:  # nodes per axis including ghosts
        return self.n + 1 + 2 * (self.g - 1)

    @property
    def unknowns(self) -> int:
        return (self.n - 1) ** 3

    def axis(self) -> np.ndarray:
        idx = np.arange(-(self.g - 1), self.n + self.g, dtype=np.float64)
        return self.lo + idx * self.h

    def interior(self) -> tuple:
        """Slice selecting the unknown nodes 1..n-1 in a full node array."""
        s = slice(self.g, self.g + self.n - 1)
        return (s, s, s)


@dataclass(frozen=True)
class SphGrid:
    nr: int = 256
    nth: int = 128
    nph: int = 256
    r_min: float = 1e-3
    r_max: float = 1.0

    @property
    def ds(self) -> float:
        return math.log(self.r_max / self.r_min) / (self.nr - 1)

    @property
    def dth(self) -> float:
        return math.pi / self.nth

    @property
    def dph(self) -> float:
        return 2.0 * math.pi / self.nph

    @property
    def unknowns(self) -> int:
        return self.nr * self.nth * self.nph

    def r_axis(self) -> np.ndarray:
        """Radii of nodes i = -1 .. nr (radial ghosts included)."""
        i = np.arange(-1, self.nr + 1, dtype=np.float64)
        return np.exp(math.log(self.r_min) + i * self.ds)

    def th_axis(self) -> np.ndarray:
        return (np.arange(self.nth, dtype=np.float64) + 0.5) * self.dth

    def ph_axis(self) -> np.ndarray:
        return np.arange(self.nph, dtype=np.float64) * self.dph


# --------------------------------------------------------------------------
# density fields
# --------------------------------------------------------------------------
@dataclass
class Clumps:
    centres: np.ndarray    # (n, 3)
    widths: np.ndarray     # (n,)   Gaussian sigma
    masses: np.ndarray     # (n,)

    def copy(self) -> "Clumps":
        return Clumps(self.centres.copy(), self.widths.copy(), self.masses.copy())


def draw_clumps(rng: np.random.Generator, n: int, lo=0.2, hi=0.8,
                wmin=0.02, wmax=0.08) -> Clumps:
    centres = rng.uniform(lo, hi, size=(n, 3))
    widths = rng.uniform(wmin, wmax, size=n)
    masses = rng.lognormal(mean=0.0, sigma=0.5, size=n)
    return Clumps(centres, widths, masses)


def clump_density(grid: CartGrid, clumps: Clumps, device="cpu") -> torch.Tensor:
    """rho(x) = sum_c M_c (2 pi s_c^2)^(-3/2) exp(-|x-x_c|^2 / (2 s_c^2)).

    Evaluated separably (outer product of three 1-D Gaussians) in float64.
    """
    ax = torch.as_tensor(grid.axis(), dtype=torch.float64, device=device)
    m = ax.numel()
    rho = torch.zeros((m, m, m), dtype=torch.float64, device=device)
    for c in range(len(clumps.masses)):
        s = float(clumps.widths[c])
        amp = float(clumps.masses[c]) * (2.0 * math.pi * s * s) ** -1.5
        gx = torch.exp(-(ax - float(clumps.centres[c, 0])) ** 2 / (2 * s * s))
        gy = torch.exp(-(ax - float(clumps.centres[c, 1])) ** 2 / (2 * s * s))
        gz = torch.exp(-(ax - float(clumps.centres[c, 2])) ** 2 / (2 * s * s))
        rho.add_((amp * gz)[:, None, None] * gy[None, :, None] * gx[None, None, :])
    return rho


def uniform_sphere(grid: CartGrid, radius=0.25, centre=(0.5, 0.5, 0.5),
                   rho0=1.0, device="cpu") -> torch.Tensor:
    """rho = rho0 for |x - c| < radius (strict), 0 otherwise."""
    ax = torch.as_tensor(grid.axis(), dtype=torch.float64, device=device)
    d2 = ((ax - centre[2]) ** 2)[:, None, None] + ((ax - centre[1]) ** 2)[None, :, None] \
        + ((ax - centre[0]) ** 2)[None, None, :]
    return torch.where(d2 < radius * radius, rho0, 0.0).to(torch.float64)


def smooth_sphere(grid: CartGrid, centre, radius, mass, n=2, device="cpu") -> torch.Tensor:
    """rho_p (1 - w^2)^n inside radius a (w = d/a); Section 3.1 test density.
    rho_p is set from the sphere's mass M = (32 pi / 105) rho_p a^3 (n = 2)."""
    assert n == 2
    rho_p = mass / (32.0 * math.pi / 105.0 * radius ** 3)
    ax = torch.as_tensor(grid.axis(), dtype=torch.float64, device=device)
    d2 = ((ax - centre[2]) ** 2)[:, None, None] + ((ax - centre[1]) ** 2)[None, :, None] \
        + ((ax - centre[0]) ** 2)[None, None, :]
    w2 = d2 / (radius * radius)
    return torch.where(w2 < 1.0, rho_p * (1.0 - w2) ** 2, 0.0).to(torch.float64)


def turbulent_floor(grid: CartGrid, rng: np.random.Generator, mean_density: float,
                    frac=0.05, device="cpu") -> torch.Tensor:
    """Lognormal floor frac * mean * exp(g - 1/2), g a unit-variance Gaussian
    random field with power spectrum |k|^-2 on integer wave-vectors
    1 <= |k| <= n/2 of an n^3 periodic grid laid over the nodes."""
    n = grid.n
    white = rng.standard_normal(size=(n, n, n))
    w = torch.as_tensor(white, dtype=torch.float64, device=device)
    del white
    wk = torch.fft.rfftn(w)
    del w
    kz = torch.fft.fftfreq(n, d=1.0 / n, device=device, dtype=torch.float64)
    kx = torch.fft.rfftfreq(n, d=1.0 / n, device=device, dtype=torch.float64)
    k2 = kz[:, None, None] ** 2 + kz[None, :, None] ** 2 + kx[None, None, :] ** 2
    amp = torch.where((k2 >= 1.0) & (k2 <= (n / 2) ** 2), k2.clamp(min=1.0) ** -0.5, 0.0)
    wk.mul_(amp)
    del amp, k2
    gfield = torch.fft.irfftn(wk, s=(n, n, n))
    del wk
    gfield -= gfield.mean()
    gfield /= gfield.std()
    m = grid.nodes
    idx = (torch.arange(m, device=device) - (grid.g - 1)) % n
    g_nodes = gfield[idx][:, idx][:, :, idx]
    return frac * mean_density * torch.exp(g_nodes - 0.5)


def sis_density(grid: SphGrid, phase: float, r_out=0.8, amp=0.1, rho0=1.0,
                device="cpu") -> torch.Tensor:
    """rho = rho0 r^-2 [1 + amp sin^2(theta) cos(2(phi - phase))] for r < r_out.
    Radial ghost nodes carry zero density."""
    r = torch.as_tensor(grid.r_axis(), dtype=torch.float64, device=device)
    th = torch.as_tensor(grid.th_axis(), dtype=torch.float64, device=device)
    ph = torch.as_tensor(grid.ph_axis(), dtype=torch.float64, device=device)
    ang = 1.0 + amp * torch.sin(th)[None, :] ** 2 * torch.cos(2.0 * (ph[:, None] - phase))
    radial = torch.where(r < r_out, rho0 / (r * r), 0.0)
    radial[0] = 0.0
    radial[-1] = 0.0
    return ang[:, :, None] * radial[None, None, :]


# --------------------------------------------------------------------------
# the five workload configurations
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    grid: object
    rho: torch.Tensor
    lmax: int
    meta: dict = field(default_factory=dict)


def config_c1(n=32, device="cpu") -> Workload:
    """Uniform sphere r = 0.25 at the box centre, 32^3 cells, lmax = 4."""
    grid = CartGrid(n=n, g=1)
    return Workload("c1_uniform_sphere", grid, uniform_sphere(grid, device=device), 4,
                    {"radius": 0.25, "centre": (0.5, 0.5, 0.5), "rho0": 1.0})


def config_c2(n=256, n_clumps=16, seed=2, device="cpu", g=1) -> Workload:
    """Sum of Gaussian clumps, centres U[0.2,0.8]^3, sigma U[0.02,0.08],
    masses lognormal(0, 0.5); 256^3 cells, lmax = 8 (g ghost layers)."""
    grid = CartGrid(n=n, g=g)
    rng = np.random.default_rng(seed)
    cl = draw_clumps(rng, n_clumps)
    return Workload(f"c2_clumps{n_clumps}_n{n}", grid, clump_density(grid, cl, device), 8,
                    {"clumps": cl, "seed": seed})


def config_c3(n=512, n_clumps=64, seed=3, device="cpu", g=3) -> Workload:
    """64 Gaussian clumps plus a 5% lognormal |k|^-2 floor; 512^3 cells,
    19-point star (3 ghost layers), lmax = 8."""
    grid = CartGrid(n=n, g=g)
    rng = np.random.default_rng(seed)
    cl = draw_clumps(rng, n_clumps)
    rho = clump_density(grid, cl, device)
    mean = float(cl.masses.sum()) / (grid.hi - grid.lo) ** 3
    rho += turbulent_floor(grid, rng, mean, device=device)
    return Workload(f"c3_clumps{n_clumps}_floor_n{n}", grid, rho, 8,
                    {"clumps": cl, "seed": seed})


def config_c4(nr=256, nth=128, nph=256, seed=4, device="cpu") -> Workload:
    """Truncated singular isothermal sphere with a 10% m = 2 perturbation on
    the log-spherical grid r in [1e-3, 1]; lmax = 8."""
    grid = SphGrid(nr=nr, nth=nth, nph=nph)
    rng = np.random.default_rng(seed)
    phase = float(rng.uniform(0.0, math.pi))
    return Workload(f"c4_sis_m2_{nr}x{nth}x{nph}", grid,
                    sis_density(grid, phase, device=device), 8, {"phase": phase})


# --------------------------------------------------------------------------
# serving stream
# --------------------------------------------------------------------------
SERVE_SIZES = (32, 64, 128, 256)
SERVE_WEIGHTS = (0.4, 0.3, 0.2, 0.1)


@dataclass
class Request:
    index: int
    arrival: float         # seconds since stream start
    stream_id: int
    n: int
    clumps: Clumps
    version: int           # 0 for the stream's first request (cold start)

    def density(self, device="cpu") -> torch.Tensor:
        return clump_density(CartGrid(n=self.n, g=1), self.clumps, device)


def serving_stream(n_requests=2000, rate=100.0, n_streams=64, seed=5,
                   sizes=SERVE_SIZES, weights=SERVE_WEIGHTS) -> List[Request]:
    """Poisson arrivals at `rate` per second over `n_streams` stream ids.

    Per stream: grid size drawn once with `weights`, clump count once from
    U{1..32}; every later request of a stream moves each centre by
    N(0, 0.002^2) per axis and scales each mass by exp(N(0, 0.02^2)).
    """
    ss = np.random.SeedSequence(seed)
    master = np.random.default_rng(ss)
    children = ss.spawn(n_streams)
    stream_rngs = [np.random.default_rng(c) for c in children]
    state = []
    for s in range(n_streams):
        r = stream_rngs[s]
        n = int(r.choice(np.asarray(sizes), p=np.asarray(weights)))
        nc = int(r.integers(1, 33))
        state.append({"n": n, "clumps": draw_clumps(r, nc), "version": -1})
    t = 0.0
    out = []
    for q in range(n_requests):
        t += float(master.exponential(1.0 / rate))
        s = int(master.integers(0, n_streams))
        st = state[s]
        r = stream_rngs[s]
        if st["version"] >= 0:
            cl = st["clumps"]
            cl.centres = cl.centres + r.normal(0.0, 0.002, size=cl.centres.shape)
            cl.masses = cl.masses * np.exp(r.normal(0.0, 0.02, size=cl.masses.shape))
        st["version"] += 1
        out.append(Request(q, t, s, st["n"], st["clumps"].copy(), st["version"]))
    return out


def embed(rho_nodes: torch.Tensor, pitch_x: int) -> torch.Tensor:
    """Copy a dense [k][j][i] node array into a zero-padded one whose rows
    have `pitch_x` elements (the layout the library reads)."""
    nz, ny, nx = rho_nodes.shape
    out = torch.zeros((nz, ny, pitch_x), dtype=rho_nodes.dtype, device=rho_nodes.device)
    out[:, :, :nx] = rho_nodes
    return out
