"""MI355X (gfx950) iterative Poisson solvers for self-gravity.

Thin Python binding of the C ABI in ``include/poisson.h``: it only marshals
torch device tensors (as raw pointers) and structures; every step of the
solve runs in the HIP library ``libpoisson_mi355x.so``.  There is no CPU
fallback: when the library is missing every call raises.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib as L
from ._lib import (BICGSTAB, BICGSTAB_MG32, CARTESIAN, CG, ETIMEOUT, MG, MG_IR32, MG_SPAI, MG_SPAI32, OMEGA_CHEBYSHEV,
                   OMEGA_FIXED, OMEGA_OPT, OMEGA_OPT_A, PCG, SOR, SPHERICAL_LOG, WARN_MAXITER)

METHODS = {"sor": SOR, "cg": CG, "bicgstab": BICGSTAB, "mg": MG, "mg_ir32": MG_IR32,
           "bicgstab_mg32": BICGSTAB_MG32, "mg_spai": MG_SPAI, "mg_spai32": MG_SPAI32, "pcg": PCG}


class PoissonError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = L.load()
        msg = lib.poisson_strerror(status).decode()
        detail = lib.poisson_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}): {detail}")
        self.status = status


def _check(status: int, where: str) -> int:
    if status < 0:
        raise PoissonError(status, where)
    return status


def _ptr(t: Optional[torch.Tensor], need: int = 0):
    """Raw device pointer of a float64 device tensor holding >= need elements."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("contiguous float64 tensor expected")
    if t.numel() < need:
        raise ValueError(f"tensor holds {t.numel()} elements, {need} needed")
    return C.c_void_p(t.data_ptr())


def cart_grid(n: int, ghost: int = 1, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), pitch_x: Optional[int] = None):
    m = n + 1 + 2 * (ghost - 1)
    px = m if pitch_x is None else pitch_x
    g = L.Grid()
    g.coord = CARTESIAN
    g.n[:] = [n, n, n]
    g.lo[:] = list(lo)
    g.hi[:] = list(hi)
    g.ghost = ghost
    g.pitch[:] = [px, px * m]
    return g


def sph_grid(nr: int, nth: int, nph: int, r_min=1e-3, r_max=1.0, pitch_r: Optional[int] = None,
             ext_in: int = 0, ext_out: int = 0, r_pad: float = 0.0):
    """Spherical grid: nr radial unknowns (pads included), the log core from
    r_min to r_max; ext_in / ext_out pad cells inside / outside it (the inner
    pad ends at r_pad)."""
    pr = nr + 2 if pitch_r is None else pitch_r
    g = L.Grid()
    g.coord = SPHERICAL_LOG
    g.n[:] = [nr, nth, nph]
    g.lo[:] = [r_min, 0.0, 0.0]
    g.hi[:] = [r_max, math.pi, 2 * math.pi]
    g.ghost = 1
    g.pitch[:] = [pr, pr * nth]
    g.ext_in, g.ext_out, g.r_pad = ext_in, ext_out, r_pad
    return g


def array_shape(grid) -> tuple:
    """Shape (planes, rows, pitch) of a caller array for `grid`."""
    if grid.coord == CARTESIAN:
        m = grid.n[0] + 1 + 2 * (grid.ghost - 1)
        return (m, m, grid.pitch[0])
    return (grid.n[2], grid.n[1], grid.pitch[0])


def options(method="mg", order=2, lmax=8, nu1=None, nu2=None, coarsest=8, omega_mode=OMEGA_OPT, omega=1.0,
            max_iter=10000, check_every=1, four_pi_G=1.0, point_mass=0.0, coarse_tol=0.0):
    """Solver options; nu1 / nu2 default to the library's per-method values
    (V(2,2), V(3,3) for the SPAI multigrid)."""
    o = L.Opts()
    L.load().poisson_default_opts(C.byref(o), METHODS[method] if isinstance(method, str) else method)
    o.order, o.lmax, o.coarsest = order, lmax, coarsest
    if nu1 is not None:
        o.nu1 = nu1
    if nu2 is not None:
        o.nu2 = nu2
    o.omega_mode, o.omega, o.max_iter, o.check_every = omega_mode, omega, max_iter, check_every
    o.four_pi_G, o.point_mass, o.coarse_tol = four_pi_G, point_mass, coarse_tol
    return o


def workspace_bytes(grid, opts) -> int:
    nbytes = L.load().poisson_workspace_bytes(C.byref(grid), C.byref(opts))
    if nbytes == 0:
        raise PoissonError(L.EINVAL, "poisson_workspace_bytes")
    return int(nbytes)


@dataclass
class SolveResult:
    status: int
    iterations: int
    rel_residual: float
    b_norm: float
    rate: float
    t_multipole_ms: float
    t_iter_ms: float
    history: list

    @property
    def converged(self) -> bool:
        return self.status == 0


class Plan:
    """A solver plan with its device workspace (a torch uint8 tensor), run on
    `stream` (default: torch's current stream); a second torch stream, on
    which nothing runs, records the plan's graphs."""

    def __init__(self, grid, opts, device="cuda:0", stream: Optional[torch.cuda.Stream] = None):
        self.lib = L.load()
        self.grid, self.opts = grid, opts
        self.device = torch.device(device)
        nbytes = workspace_bytes(grid, opts)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.capture_stream = torch.cuda.Stream(self.device)
        handle = C.c_void_p()
        _check(self.lib.poisson_plan(C.byref(handle), C.byref(grid), C.byref(opts),
                                     C.c_void_p(self._ws_ptr), nbytes, C.c_void_p(self.stream.cuda_stream)),
               "poisson_plan")
        self.handle = handle
        _check(self.lib.poisson_plan_set_capture_stream(handle, C.c_void_p(self.capture_stream.cuda_stream)),
               "poisson_plan_set_capture_stream")

    @property
    def node_elems(self) -> int:
        """Elements a caller rho / phi array must hold."""
        p, r, _ = array_shape(self.grid)
        return int(p * self.grid.pitch[1])

    def _dense_elems(self, level: int) -> int:
        e = self.grid.n[0] // (2 ** level) - 1
        return e ** 3

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.poisson_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ hot path
    def solve(self, rho: torch.Tensor, phi: torch.Tensor, tol: float = 1e-8, history: int = 0) -> SolveResult:
        st = L.Stats()
        buf = None
        if history > 0:
            buf = (C.c_double * history)()
            st.residual_history = C.cast(buf, C.POINTER(C.c_double))
            st.history_cap = history
        ne = self.node_elems
        status = _check(self.lib.poisson_solve(self.handle, _ptr(rho, ne), _ptr(phi, ne), C.byref(self.grid), tol,
                                               C.byref(st)), "poisson_solve")
        hist = [buf[i] for i in range(st.history_len)] if buf is not None else []
        return SolveResult(status, st.iterations, st.rel_residual, st.b_norm, st.rate, st.t_multipole_ms,
                           st.t_iter_ms, hist)

    def multipole_boundary(self, rho: torch.Tensor, phi: torch.Tensor, lmax: int):
        nq = (lmax + 1) ** 2 * (2 if self.grid.coord == SPHERICAL_LOG else 1)
        q = (C.c_double * nq)()
        ne = self.node_elems
        _check(self.lib.multipole_boundary(self.handle, _ptr(rho, ne), _ptr(phi, ne), lmax, q), "multipole_boundary")
        return [q[i] for i in range(nq)]

    # ------------------------------------------------------------ single operators
    def apply(self, phi: torch.Tensor, out: torch.Tensor):
        ne = self.node_elems
        _check(self.lib.poisson_op_apply(self.handle, _ptr(phi, ne), _ptr(out, ne)), "poisson_op_apply")

    def residual(self, rho, phi, res) -> float:
        n2 = C.c_double()
        ne = self.node_elems
        _check(self.lib.poisson_op_residual(self.handle, _ptr(rho, ne), _ptr(phi, ne), _ptr(res, ne), C.byref(n2)),
               "poisson_op_residual")
        return n2.value

    def smooth(self, rho, phi, sweeps=1, forward=True, omega=1.0):
        ne = self.node_elems
        _check(self.lib.poisson_op_smooth(self.handle, _ptr(rho, ne), _ptr(phi, ne), sweeps, 1 if forward else 0,
                                          omega),
               "poisson_op_smooth")

    def restrict(self, fine, coarse):
        _check(self.lib.poisson_op_restrict(self.handle, _ptr(fine, self._dense_elems(0)),
                                            _ptr(coarse, self._dense_elems(1))), "poisson_op_restrict")

    def restrict_residual(self, rho, phi, coarse) -> float:
        """coarse = R (4 pi G rho - L phi) (dense coarse unknowns); returns the
        fine residual's sum of squares."""
        n2 = C.c_double()
        ne = self.node_elems
        _check(self.lib.poisson_op_restrict_residual(self.handle, _ptr(rho, ne), _ptr(phi, ne),
                                                     _ptr(coarse, self._dense_elems(1)), C.byref(n2)),
               "poisson_op_restrict_residual")
        return n2.value

    def prolong_add(self, coarse, fine):
        _check(self.lib.poisson_op_prolong_add(self.handle, _ptr(coarse, self._dense_elems(1)),
                                               _ptr(fine, self._dense_elems(0))), "poisson_op_prolong_add")

    def precond(self, y, yhat):
        """yhat = M^-1 y, one FP32 multigrid cycle of a bicgstab_mg32 plan."""
        ne = self.node_elems
        _check(self.lib.poisson_op_precond(self.handle, _ptr(y, ne), _ptr(yhat, ne)), "poisson_op_precond")

    def vcycle(self, rho, phi, cycles=1):
        ne = self.node_elems
        _check(self.lib.poisson_op_vcycle(self.handle, _ptr(rho, ne), _ptr(phi, ne), cycles), "poisson_op_vcycle")


class Server:
    """Continuous-batching solve server (a persistent loop in the library).
    Its device memory is one torch uint8 arena of budget_bytes and its slots
    are max_slots torch streams; the library carves plans and cached
    potentials from the arena and launches on those streams."""

    def __init__(self, budget_bytes: int, max_slots=8, mixed=True, lmax=8, nu=2, tol=1e-8, warm_start=True,
                 use_graphs=True, device="cuda:0"):
        self.lib = L.load()
        self.device = torch.device(device)
        budget = int(budget_bytes)
        self.arena = torch.empty(budget + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.arena.data_ptr() + 255) & ~255
        self.streams = [torch.cuda.Stream(self.device) for _ in range(max_slots)]
        handles = (C.c_void_p * max_slots)(*[s.cuda_stream for s in self.streams])
        self._held = {}   # ticket -> (rho, phi): kept alive until the request is done
        h = C.c_void_p()
        _check(self.lib.poisson_server_create(C.byref(h), C.c_void_p(ptr), budget, max_slots, handles, int(mixed),
                                              lmax, nu, tol, int(warm_start), int(use_graphs)),
               "poisson_server_create")
        self.handle = h

    def submit(self, stream_id: int, n: int, rho: torch.Tensor, phi: torch.Tensor,
               stream: Optional[torch.cuda.Stream] = None) -> int:
        """Queue a solve; it starts after the work already queued on `stream`
        (default: torch's current stream), which produced rho and phi."""
        t = C.c_int64()
        need = (n + 1) ** 3
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(self.lib.poisson_server_submit(self.handle, stream_id, n, _ptr(rho, need), _ptr(phi, need),
                                              C.c_void_p(st.cuda_stream), C.byref(t)), "poisson_server_submit")
        self._held[t.value] = (rho, phi)
        return t.value

    def poll(self, ticket: int):
        done = C.c_int32()
        st = L.Stats()
        lat = C.c_double()
        status = self.lib.poisson_server_poll(self.handle, ticket, C.byref(done), C.byref(st), C.byref(lat))
        if not done.value:
            _check(status, "poisson_server_poll")
            return None
        self._held.pop(ticket, None)
        return SolveResult(status, st.iterations, st.rel_residual, st.b_norm, st.rate, 0.0, st.t_iter_ms, []), \
            lat.value

    def wait(self, ticket: int, timeout_ms: float = 120000.0) -> int:
        """The request's status once done, or ETIMEOUT (-7) if timeout_ms ran
        out first."""
        return self.lib.poisson_server_wait(self.handle, ticket, timeout_ms)

    def reserve(self, n: int, count: int):
        _check(self.lib.poisson_server_reserve(self.handle, n, count), "poisson_server_reserve")

    def footprint(self, n: int) -> int:
        b = C.c_size_t()
        _check(self.lib.poisson_server_footprint(self.handle, n, C.byref(b)), "poisson_server_footprint")
        return b.value

    def usage(self):
        used = C.c_size_t()
        q = C.c_int32()
        a = C.c_int32()
        _check(self.lib.poisson_server_usage(self.handle, C.byref(used), C.byref(q), C.byref(a)),
               "poisson_server_usage")
        return used.value, q.value, a.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.poisson_server_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_SCRATCH_BYTES = 80 * 1024 * 1024


def multipole_boundary_noalloc(grid, rho: torch.Tensor, phi: torch.Tensor, lmax: int, four_pi_G: float = 1.0,
                               point_mass: float = 0.0, stream: Optional[torch.cuda.Stream] = None):
    """Cartesian multipole boundary without a plan or any device allocation
    (the library's fixed per-device scratch array); returns q_lm."""
    lib = L.load()
    p, r, _ = array_shape(grid)
    ne = int(p * grid.pitch[1])
    q = (C.c_double * ((lmax + 1) ** 2))()
    st = stream if stream is not None else torch.cuda.current_stream(rho.device)
    _check(lib.multipole_boundary_noalloc(C.byref(grid), _ptr(rho, ne), _ptr(phi, ne), lmax, four_pi_G, point_mass,
                                          q, C.c_void_p(st.cuda_stream)), "multipole_boundary_noalloc")
    return [q[i] for i in range(len(q))]


def sweep_resident(plan: "Plan", sweeps: int):
    _check(plan.lib.poisson_op_sweep_resident(plan.handle, sweeps), "poisson_op_sweep_resident")


def library_path() -> str:
    return L.LIB_PATH
