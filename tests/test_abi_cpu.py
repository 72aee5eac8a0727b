"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and validates grids / options on the host (no GPU work)."""
import ctypes as C
import os
import re

import pytest

import paper_2605_03563_amd as pg
from paper_2605_03563_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_function():
    lib = L.load()
    declared = _declared_functions()
    assert "poisson_solve" in declared and "multipole_boundary" in declared and "poisson_plan" in declared
    for name in declared:
        assert hasattr(lib, name), f"{name} declared but not exported"
        assert name in L.SIGNATURES, f"{name} has no ctypes signature"


def test_struct_layouts_match_header_sizes():
    assert C.sizeof(L.Grid) == 4 + 12 + 24 + 24 + 4 + 4 + 16 + 4 + 4 + 8
    assert C.sizeof(L.Opts) == 10 * 4 + 4 * 8
    assert C.sizeof(L.Stats) == 8 + 5 * 8 + 8 + 8


def test_default_options_and_strerror():
    o = pg.options("mg")
    assert (o.order, o.lmax, o.nu1, o.nu2, o.coarsest) == (2, 8, 2, 2, 8)
    lib = L.load()
    assert lib.poisson_strerror(0) == b"converged"
    assert b"max_iter" in lib.poisson_strerror(1)


@pytest.mark.parametrize("n,ok", [(256, True), (64, True), (8, True), (96, False), (250, False)])
def test_multigrid_grid_rule(n, ok):
    """Multigrid needs n = 2^L * coarsest intervals (Section 2.1.3)."""
    grid = pg.cart_grid(n)
    opts = pg.options("mg")
    nbytes = L.load().poisson_workspace_bytes(C.byref(grid), C.byref(opts))
    assert (nbytes > 0) == ok
    if not ok:
        assert b"2^L" in L.load().poisson_last_error()


def test_workspace_sizes_are_sane():
    grid = pg.cart_grid(256)
    nb = pg.workspace_bytes(grid, pg.options("mg"))
    # three FP64 colour-split fine arrays dominate: ~3 * 257^2 * 2 * 160 * 8 bytes
    assert 3 * 257 * 257 * 320 * 8 < nb < 5 * 257 * 257 * 320 * 8
    nb32 = pg.workspace_bytes(grid, pg.options("mg_ir32"))
    assert nb32 < 1.6 * nb
    g19 = pg.cart_grid(512, ghost=3)
    nb19 = pg.workspace_bytes(g19, pg.options("mg_ir32", order=6))
    assert nb19 < 12e9


@pytest.mark.parametrize("kw,err", [
    (dict(order=4), "order"),
    (dict(lmax=9), "lmax"),
    (dict(max_iter=0), "max_iter"),
    (dict(four_pi_G=0.0), "four_pi_G"),
])
def test_invalid_options_rejected(kw, err):
    grid = pg.cart_grid(32)
    opts = pg.options("cg", **kw)
    assert L.load().poisson_workspace_bytes(C.byref(grid), C.byref(opts)) == 0
    assert err.encode() in L.load().poisson_last_error()


def test_ghost_layers_must_match_order():
    assert L.load().poisson_workspace_bytes(C.byref(pg.cart_grid(32, ghost=1)),
                                            C.byref(pg.options("cg", order=6))) == 0
    assert L.load().poisson_workspace_bytes(C.byref(pg.cart_grid(32, ghost=3)),
                                            C.byref(pg.options("cg", order=6))) > 0


def test_pitch_and_spherical_checks():
    g = pg.cart_grid(32, pitch_x=20)
    assert L.load().poisson_workspace_bytes(C.byref(g), C.byref(pg.options("cg"))) == 0
    s = pg.sph_grid(64, 32, 32)
    assert L.load().poisson_workspace_bytes(C.byref(s), C.byref(pg.options("bicgstab"))) > 0
    assert L.load().poisson_workspace_bytes(C.byref(s), C.byref(pg.options("mg"))) == 0
    s_odd = pg.sph_grid(64, 31, 32)
    assert L.load().poisson_workspace_bytes(C.byref(s_odd), C.byref(pg.options("bicgstab"))) == 0


def test_spherical_multigrid_preconditioner_sizes():
    lib = L.load()
    s = pg.sph_grid(64, 32, 32)
    gs = lib.poisson_workspace_bytes(C.byref(s), C.byref(pg.options("bicgstab")))
    mg = lib.poisson_workspace_bytes(C.byref(s), C.byref(pg.options("bicgstab_mg32")))
    # FP32 u, f, r on the fine level (with radial ghosts) and the coarser levels
    assert mg > gs + 3 * 4 * 66 * 32 * 32
    # 96 x 48 x 48 halves three times, to 12 x 6 x 6 (432 unknowns)
    assert lib.poisson_workspace_bytes(C.byref(pg.sph_grid(96, 48, 48)),
                                       C.byref(pg.options("bicgstab_mg32"))) > 0
    # odd radial count: no coarsening, 33 x 32 x 32 unknowns is too many for the dense level
    assert lib.poisson_workspace_bytes(C.byref(pg.sph_grid(33, 32, 32)),
                                       C.byref(pg.options("bicgstab_mg32"))) == 0
    assert b"coarsen" in lib.poisson_last_error()
    # a small odd grid is its own coarsest level
    assert lib.poisson_workspace_bytes(C.byref(pg.sph_grid(9, 8, 8)),
                                       C.byref(pg.options("bicgstab_mg32"))) > 0
    assert lib.poisson_workspace_bytes(C.byref(s), C.byref(pg.options("bicgstab_mg32", nu1=0))) == 0


def test_plan_rejects_small_or_misaligned_workspace_before_any_device_call():
    lib = L.load()
    grid = pg.cart_grid(32)
    opts = pg.options("cg")
    h = C.c_void_p()
    need = lib.poisson_workspace_bytes(C.byref(grid), C.byref(opts))
    st = lib.poisson_plan(C.byref(h), C.byref(grid), C.byref(opts), C.c_void_p(0x100000), need - 1, None)
    assert st == L.EWORKSPACE
    st = lib.poisson_plan(C.byref(h), C.byref(grid), C.byref(opts), C.c_void_p(0x100010), need, None)
    assert st == L.EWORKSPACE
    st = lib.poisson_plan(C.byref(h), C.byref(grid), C.byref(opts), None, need, None)
    assert st == L.EWORKSPACE
    assert h.value is None


def test_coarse_tol_validation():
    lib = L.load()
    g = pg.cart_grid(32)
    assert lib.poisson_workspace_bytes(C.byref(g), C.byref(pg.options("mg_spai", coarse_tol=0.013))) > 0
    assert lib.poisson_workspace_bytes(C.byref(g), C.byref(pg.options("mg", coarse_tol=0.013))) == 0
    assert lib.poisson_workspace_bytes(C.byref(g), C.byref(pg.options("mg_spai", coarse_tol=1.5))) == 0
    assert lib.poisson_workspace_bytes(C.byref(pg.cart_grid(64)),
                                       C.byref(pg.options("mg_spai", coarse_tol=0.1, coarsest=16))) == 0
    s = pg.sph_grid(32, 16, 16)
    assert lib.poisson_workspace_bytes(C.byref(s), C.byref(pg.options("bicgstab", coarse_tol=0.1))) == 0


def test_spherical_sor_options():
    lib = L.load()
    s = pg.sph_grid(32, 16, 16)
    assert lib.poisson_workspace_bytes(C.byref(s), C.byref(pg.options("sor", omega_mode=pg.OMEGA_CHEBYSHEV))) > 0
    assert lib.poisson_workspace_bytes(C.byref(s), C.byref(pg.options("sor", omega_mode=pg.OMEGA_OPT))) > 0
    assert lib.poisson_workspace_bytes(C.byref(s), C.byref(pg.options("sor", omega_mode=pg.OMEGA_OPT_A))) == 0
    assert lib.poisson_workspace_bytes(C.byref(s), C.byref(pg.options("sor", omega_mode=pg.OMEGA_FIXED,
                                                                      omega=2.5))) == 0
    assert lib.poisson_workspace_bytes(C.byref(s), C.byref(pg.options("cg"))) == 0


def test_spai_order_and_ghost_validation():
    """Compact orders 2, 4 and 6; order 6 reads rho's second ghost layer and
    needs ghost = 2, while the 19-point star (order 6 of the other methods)
    keeps ghost = 3."""
    lib = L.load()
    for order in (2, 4):
        assert lib.poisson_workspace_bytes(C.byref(pg.cart_grid(32)),
                                           C.byref(pg.options("mg_spai", order=order))) > 0
    assert lib.poisson_workspace_bytes(C.byref(pg.cart_grid(32, ghost=2)),
                                       C.byref(pg.options("mg_spai", order=6))) > 0
    assert lib.poisson_workspace_bytes(C.byref(pg.cart_grid(32, ghost=2)),
                                       C.byref(pg.options("mg_spai32", order=6))) > 0
    assert lib.poisson_workspace_bytes(C.byref(pg.cart_grid(32)),
                                       C.byref(pg.options("mg_spai", order=6))) == 0
    assert b"ghost = 2" in lib.poisson_last_error()
    assert lib.poisson_workspace_bytes(C.byref(pg.cart_grid(32, ghost=3)),
                                       C.byref(pg.options("mg_spai", order=6))) == 0
    assert lib.poisson_workspace_bytes(C.byref(pg.cart_grid(32, ghost=2)),
                                       C.byref(pg.options("mg", order=6))) == 0
    assert lib.poisson_workspace_bytes(C.byref(pg.cart_grid(32, ghost=3)),
                                       C.byref(pg.options("mg", order=6))) > 0
    assert lib.poisson_workspace_bytes(C.byref(pg.cart_grid(32)),
                                       C.byref(pg.options("mg_spai", order=8))) == 0


def test_radial_pad_validation():
    """Pads belong to spherical grids; the inner pad needs 0 < r_pad < r_in and
    a monotone quartic; at least two log-core unknowns remain; the FP32
    FP32 multigrid preconditioner keeps one line-smoother table per radius
    and colatitude inside an inner pad (where the map bends), one per
    colatitude for the rest and on log grids."""
    lib = L.load()
    ok = pg.sph_grid(60, 8, 16, 0.5, 1.0, ext_in=8, ext_out=6, r_pad=0.3)
    assert lib.poisson_workspace_bytes(C.byref(ok), C.byref(pg.options("bicgstab"))) > 0
    assert lib.poisson_workspace_bytes(C.byref(ok), C.byref(pg.options("sor"))) > 0
    padded = lib.poisson_workspace_bytes(C.byref(ok), C.byref(pg.options("bicgstab_mg32")))
    outer = lib.poisson_workspace_bytes(C.byref(pg.sph_grid(60, 8, 16, 0.5, 1.0, ext_out=6)),
                                        C.byref(pg.options("bicgstab_mg32")))
    plain = lib.poisson_workspace_bytes(C.byref(pg.sph_grid(60, 8, 16, 0.5, 1.0)),
                                        C.byref(pg.options("bicgstab_mg32")))
    assert padded > outer == plain > 0
    bad_pad = pg.sph_grid(60, 8, 16, 0.5, 1.0, ext_in=8, r_pad=0.6)
    assert lib.poisson_workspace_bytes(C.byref(bad_pad), C.byref(pg.options("bicgstab"))) == 0
    assert b"r_pad" in lib.poisson_last_error()
    too_few = pg.sph_grid(12, 8, 16, 0.5, 1.0, ext_in=8, ext_out=6, r_pad=0.3)
    assert lib.poisson_workspace_bytes(C.byref(too_few), C.byref(pg.options("bicgstab"))) == 0
    # a pad of many cells over a large log step cannot be monotone
    non_mono = pg.sph_grid(40, 8, 16, 0.01, 1.0, ext_in=20, r_pad=0.009)
    assert lib.poisson_workspace_bytes(C.byref(non_mono), C.byref(pg.options("bicgstab"))) == 0
    cart = pg.cart_grid(32)
    cart.ext_in = 2
    assert lib.poisson_workspace_bytes(C.byref(cart), C.byref(pg.options("mg"))) == 0


def test_pcg_workspace_and_validation():
    """PCG keeps one more FP64 array than CG (the preconditioned residual),
    takes both Cartesian orders, and is not a spherical method."""
    lib = L.load()
    g = pg.cart_grid(64)
    cg = lib.poisson_workspace_bytes(C.byref(g), C.byref(pg.options("cg")))
    pcg = lib.poisson_workspace_bytes(C.byref(g), C.byref(pg.options("pcg")))
    assert pcg > cg > 0
    g3 = pg.cart_grid(64, ghost=3)
    assert lib.poisson_workspace_bytes(C.byref(g3), C.byref(pg.options("pcg", order=6))) > 0
    assert lib.poisson_workspace_bytes(C.byref(pg.sph_grid(16, 8, 16)), C.byref(pg.options("pcg"))) == 0


def test_server_and_capture_stream_validation_before_any_device_call():
    """The serving loop takes the caller's arena and streams: a missing arena,
    a misaligned one or a NULL slot stream is refused on the host, and so is
    a NULL capture stream; a wait that runs out of time has its own status."""
    lib = L.load()
    h = C.c_void_p()
    streams = (C.c_void_p * 2)(C.c_void_p(0x1000), C.c_void_p(0x2000))
    assert lib.poisson_server_create(C.byref(h), None, 1 << 20, 2, streams, 1, 8, 2, 1e-8, 1, 1) == L.EINVAL
    assert lib.poisson_server_create(C.byref(h), C.c_void_p(0x10080), 1 << 20, 2, streams, 1, 8, 2, 1e-8, 1,
                                     1) == L.EWORKSPACE
    nulls = (C.c_void_p * 2)(C.c_void_p(0x1000), None)
    assert lib.poisson_server_create(C.byref(h), C.c_void_p(0x10000), 1 << 20, 2, nulls, 1, 8, 2, 1e-8, 1,
                                     1) == L.EINVAL
    assert b"NULL stream" in lib.poisson_last_error()
    assert lib.poisson_server_create(C.byref(h), C.c_void_p(0x10000), 1 << 20, 17, streams, 1, 8, 2, 1e-8, 1,
                                     1) == L.EINVAL
    assert lib.poisson_plan_set_capture_stream(None, C.c_void_p(0x1000)) == L.EINVAL
    assert lib.poisson_strerror(L.ETIMEOUT) != lib.poisson_strerror(L.WARN_MAXITER)
    assert b"timed out" in lib.poisson_strerror(L.ETIMEOUT)


def test_noalloc_multipole_validation_before_any_device_call():
    """The allocation-free multipole boundary rejects, on the host, grids its
    fixed scratch array cannot hold and everything but Cartesian grids."""
    lib = L.load()
    fake = C.c_void_p(1 << 20)   # never dereferenced: validation fails first

    def call(grid, lmax=8, four_pi_g=1.0, rho=fake):
        return lib.multipole_boundary_noalloc(C.byref(grid), rho, fake, lmax, four_pi_g, 0.0, None, None)

    assert call(pg.cart_grid(1024)) == L.EINVAL
    assert b"scratch" in lib.poisson_last_error()
    assert call(pg.sph_grid(16, 8, 8)) == L.EINVAL
    assert call(pg.cart_grid(32), lmax=9) == L.EINVAL
    assert call(pg.cart_grid(32), lmax=-1) == L.EINVAL
    assert call(pg.cart_grid(32), four_pi_g=0.0) == L.EINVAL
    assert call(pg.cart_grid(32), rho=None) == L.EINVAL
    assert call(pg.cart_grid(32, pitch_x=20)) == L.EINVAL
    g = pg.cart_grid(32)
    g.ghost = 4
    assert call(g) == L.EGRID
    assert pg.NOALLOC_SCRATCH_BYTES == 80 * 1024 * 1024


def test_operator_calls_reject_a_null_plan_before_any_device_call():
    """Every operator entry point checks its plan on the host: a NULL plan is
    an argument error, reported before any kernel is launched."""
    lib = L.load()
    p = C.c_void_p(0x1000)
    calls = [
        lambda: lib.poisson_op_apply(None, p, p),
        lambda: lib.poisson_op_residual(None, p, p, p, None),
        lambda: lib.poisson_op_restrict(None, p, p),
        lambda: lib.poisson_op_restrict_residual(None, p, p, p, None),
        lambda: lib.poisson_op_prolong_add(None, p, p),
        lambda: lib.poisson_op_vcycle(None, p, p, 1),
    ]
    for call in calls:
        assert call() == L.EINVAL
        assert lib.poisson_last_error() in (b"null plan", b"null argument")
