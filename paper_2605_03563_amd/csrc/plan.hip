// Host side of the gfx950 Poisson library: workspace layout, plan
// construction, the solver drivers (red-black SOR, CG, geometric multigrid,
// FP32 multigrid inside FP64 iterative refinement, BiCGSTAB on the
// log-spherical grid) and the C ABI declared in include/poisson.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"
#include "plan_impl.h"
#include "reduce.h"

using namespace psn;

// ============================================================ error state
static thread_local char g_err[512] = "";

void psn::set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));                      \
      return POISSON_EHIP;                                                           \
    }                                                                                \
  } while (0)

#define CHK(expr)                      \
  do {                                 \
    int s_ = (expr);                   \
    if (s_ < 0) return s_;             \
  } while (0)

int psn::launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("kernel launch in %s failed: %s", what, hipGetErrorString(e));
    return POISSON_EHIP;
  }
  return POISSON_OK;
}

// ============================================================ plan
namespace {

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  void* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Level sizes of the spherical FP32 multigrid preconditioner: halve every axis
// while all three stay even (ntheta >= 4, nphi >= 8, nr >= 4) and the level
// has more than 512 unknowns.
std::vector<std::array<int, 3>> sph_levels(int nr, int nth, int nph) {
  std::vector<std::array<int, 3>> out;
  while (true) {
    out.push_back({nr, nth, nph});
    if ((long long)nr * nth * nph <= 512 || (nr & 1) || (nth & 1) || (nph & 1) || nth < 4 || nph < 8 || nr < 4) break;
    nr /= 2;
    nth /= 2;
    nph /= 2;
  }
  return out;
}

// Split of a phi line of nph nodes for the line smoother: when nph is a
// multiple of 16 and at most 256, sixteen segments (eight below 32 nodes),
// since the pass is bound by the latency of its sequential recurrences
// (at 256 x 128 x 256 sixteen segments of 16 nodes take the C4 solve from
// 11.1 to 9.7 ms against eight of 32; 32 segments of 8 gain nothing more);
// else segments of the largest divisor of nph up to 32; nseg = nph / seg of
// them, nl lines per block (a power of two, <= 64 lines, <= 1024 threads
// and the LDS of Y plus the interface values within 64 KiB).  False if no
// split fits.
bool line_split(int nph, int* seg, int* nseg, int* nl) {
  int L = 1;
  if (nph % 16 == 0 && nph <= 256) {
    L = nph >= 32 ? nph / 16 : nph / 8;
  } else {
    for (int d = 2; d <= 32 && d <= nph; ++d)
      if (nph % d == 0) L = d;
  }
  const int P = nph / L;
  if (L < 2 || P > 64) return false;
  int n = 64;
  while (n > 1 && (n * P > 1024 || (long long)n * (nph + 2 * P) * 4 > 65536)) n >>= 1;
  if ((long long)n * (nph + 2 * P) * 4 > 65536 || n * P > 1024) return false;
  *seg = L;
  *nseg = P;
  *nl = n;
  return true;
}

// Radial map of the spherical grid (Section 3.3).  Radial index a = 0 ..
// nr+1 (a = 0 and nr+1 the ghosts) sits at map coordinate xi = a - 1 - p,
// p = max(ext_in - 1, 0) inner pad unknowns; the log core r_in e^(xi ds)
// covers xi = 0 .. nlog-1 and continues outward; with an inner pad, xi < 0
// follows the quartic Q(xi) that matches the log map's value and first
// three derivatives at xi = 0 and reaches r_pad at xi = -ext_in.
struct RadialFn {
  double rin = 0.0, ds = 0.0, c4 = 0.0;
  int ein = 0, p = 0;
  void eval(double xi, double& R, double& R1, double& R2) const {
    if (ein > 0 && xi < 0.0) {
      const double d = ds, x = d * xi;
      R = rin * (1.0 + x + x * x / 2.0 + x * x * x / 6.0) + c4 * xi * xi * xi * xi;
      R1 = rin * d * (1.0 + x + x * x / 2.0) + 4.0 * c4 * xi * xi * xi;
      R2 = rin * d * d * (1.0 + x) + 12.0 * c4 * xi * xi;
    } else {
      R = rin * exp(xi * ds);
      R1 = ds * R;
      R2 = ds * ds * R;
    }
  }
  // The operator on the map coordinate is a u_xixi + b u_xi with
  // a = (r/R')^2, b = 2r/R' - r^2 R''/R'^3; central differences of spacing h
  // give the couplings cl = a/h^2 - b/(2h) (to xi - h), cr = a/h^2 + b/(2h).
  void couple(double xi, double h, double& cl, double& cr) const {
    double R, R1, R2;
    eval(xi, R, R1, R2);
    const double q = R / (h * R1);
    const double bb = 2.0 * q - R * R * R2 / (h * R1 * R1 * R1);
    cl = q * q - 0.5 * bb;
    cr = q * q + 0.5 * bb;
  }
};

bool radial_fn(const poisson_grid_t& g, RadialFn& f) {
  const int nr = g.n[0];
  const int ein = g.ext_in, eout = g.ext_out;
  const int p = ein > 0 ? ein - 1 : 0, q = eout > 0 ? eout - 1 : 0;
  const int nlog = nr - p - q;
  if (nlog < 2 || ein < 0 || eout < 0) return false;
  f.rin = g.lo[0];
  f.ein = ein;
  f.p = p;
  f.ds = log(g.hi[0] / f.rin) / (nlog - 1);
  f.c4 = 0.0;
  if (ein > 0) {
    const double E = ein, x = f.ds * E;
    f.c4 = (g.r_pad - f.rin * (1.0 - x + x * x / 2.0 - x * x * x / 6.0)) / (E * E * E * E);
    // the pad must map monotonically (R' > 0 on [-ext_in, 0])
    for (int t = 0; t <= 2000; ++t) {
      double R, R1, R2;
      f.eval(-ein + ein * (t / 2000.0), R, R1, R2);
      if (!(R1 > 0.0) || !(R > 0.0)) return false;
    }
  }
  return true;
}

// Radii, couplings (spacing 1 in xi) and radial volume weights r^2 R' per
// radial index of the finest grid.
bool sph_radial_map(const poisson_grid_t& g, std::vector<double>& r, std::vector<double>& cl,
                    std::vector<double>& cr, std::vector<double>& w, double& ds) {
  RadialFn f;
  if (!radial_fn(g, f)) return false;
  const int nr = g.n[0];
  ds = f.ds;
  r.assign(nr + 2, 0.0);
  cl.assign(nr + 2, 0.0);
  cr.assign(nr + 2, 0.0);
  w.assign(nr + 2, 0.0);
  for (int a = 0; a < nr + 2; ++a) {
    const double xi = (double)(a - 1 - f.p);
    double R, R1, R2;
    f.eval(xi, R, R1, R2);
    r[a] = R;
    if (a >= 1 && a <= nr) {
      f.couple(xi, 1.0, cl[a], cr[a]);
      w[a] = R * R * R1;
    }
  }
  return true;
}

// Radial couplings of multigrid level `level` with n radial unknowns: level
// unknown I pairs two nodes of the level below and sits at their mean,
// xi = 2^level I + (2^level - 1)/2 - p, with spacing h = 2^level.
void sph_level_couplings(const poisson_grid_t& g, int level, int n, std::vector<double>& cl,
                         std::vector<double>& cr) {
  RadialFn f;
  radial_fn(g, f);
  const double h = (double)(1 << level);
  cl.assign(n, 0.0);
  cr.assign(n, 0.0);
  for (int I = 0; I < n; ++I) f.couple(h * I + 0.5 * (h - 1.0) - f.p, h, cl[I], cr[I]);
}

int validate(const poisson_grid_t* g, const poisson_opts_t* o) {
  if (!g || !o) {
    set_error("null grid or options");
    return POISSON_EINVAL;
  }
  if (o->lmax < -1 || o->lmax > kLmaxMax) {
    set_error("lmax must be in -1..%d", kLmaxMax);
    return POISSON_EINVAL;
  }
  if (o->max_iter < 1 || o->check_every < 1) {
    set_error("max_iter and check_every must be >= 1");
    return POISSON_EINVAL;
  }
  if (!(o->coarse_tol >= 0.0 && o->coarse_tol < 1.0)) {
    set_error("coarse_tol must lie in [0, 1)");
    return POISSON_EINVAL;
  }
  if (o->coarse_tol != 0.0 && o->method != POISSON_MG_SPAI && o->method != POISSON_MG_SPAI32) {
    set_error("coarse_tol applies to the SPAI multigrid only");
    return POISSON_EINVAL;
  }
  if (!(o->four_pi_G > 0.0)) {
    set_error("four_pi_G must be positive");
    return POISSON_EINVAL;
  }
  if (g->coord == POISSON_SPHERICAL_LOG) {
    if (o->method != POISSON_BICGSTAB && o->method != POISSON_BICGSTAB_MG32 && o->method != POISSON_SOR) {
      set_error("the log-spherical grid is solved by BiCGSTAB or SOR");
      return POISSON_EINVAL;
    }
    if (o->method == POISSON_SOR && o->omega_mode != POISSON_OMEGA_OPT && o->omega_mode != POISSON_OMEGA_CHEBYSHEV &&
        o->omega_mode != POISSON_OMEGA_FIXED) {
      set_error("spherical SOR takes the local omega_opt, the local Chebyshev sequence or a fixed omega");
      return POISSON_EINVAL;
    }
    if (o->method == POISSON_SOR && o->omega_mode == POISSON_OMEGA_FIXED && !(o->omega > 0.0 && o->omega < 2.0)) {
      set_error("SOR needs 0 < omega < 2");
      return POISSON_EINVAL;
    }
    if (o->method == POISSON_BICGSTAB_MG32) {
      if (o->nu1 < 1 || o->nu2 < 1) {
        set_error("the multigrid preconditioner needs nu1, nu2 >= 1");
        return POISSON_EINVAL;
      }
      const auto lv = sph_levels(g->n[0], g->n[1], g->n[2]);
      const auto& c = lv.back();
      if ((long long)c[0] * c[1] * c[2] > 4096) {
        set_error("spherical grid does not coarsen to <= 4096 unknowns (sizes must keep halving evenly)");
        return POISSON_EGRID;
      }
      int sg, ns, nl;
      for (size_t l = 0; l + 1 < lv.size(); ++l)
        if (!line_split(lv[l][2], &sg, &ns, &nl)) {
          set_error("nphi = %d has no segment split for the phi-line smoother", lv[l][2]);
          return POISSON_EGRID;
        }
    }
    if (g->n[0] < 3 || g->n[1] < 2 || g->n[2] < 2 || (g->n[1] & 1) || (g->n[2] & 1)) {
      set_error("spherical grid needs nr >= 3 and even ntheta, nphi");
      return POISSON_EGRID;
    }
    if (!(g->lo[0] > 0.0) || !(g->hi[0] > g->lo[0])) {
      set_error("spherical grid needs 0 < r_min < r_max");
      return POISSON_EGRID;
    }
    if (g->ext_in < 0 || g->ext_out < 0) {
      set_error("radial pads need ext_in, ext_out >= 0");
      return POISSON_EGRID;
    }
    if (g->ext_in > 0 && !(g->r_pad > 0.0 && g->r_pad < g->lo[0])) {
      set_error("an inner pad needs 0 < r_pad < r_in");
      return POISSON_EGRID;
    }
    {
      std::vector<double> r, cl, cr, w;
      double ds;
      if (!sph_radial_map(*g, r, cl, cr, w, ds)) {
        set_error("radial pads leave fewer than two log-core unknowns or a non-monotone inner pad");
        return POISSON_EGRID;
      }
    }
    if (g->pitch[0] < g->n[0] + 2 || g->pitch[1] < (int64_t)g->n[1] * g->pitch[0]) {
      set_error("pitch too small for the spherical grid");
      return POISSON_EINVAL;
    }
    if (o->order != 2) {
      set_error("the spherical operator is 2nd order");
      return POISSON_EINVAL;
    }
    SGeom S{};
    S.nr = g->n[0];
    S.nth = g->n[1];
    S.nph = g->n[2];
    if (sph_blocks(S) > kPartialCap) {
      set_error("grid too large for the reduction buffers");
      return POISSON_EGRID;
    }
    return POISSON_OK;
  }
  if (g->coord != POISSON_CARTESIAN) {
    set_error("unknown coordinate system %d", g->coord);
    return POISSON_EINVAL;
  }
  const int n = g->n[0];
  if (g->n[1] != n || g->n[2] != n) {
    set_error("Cartesian grids must have the same interval count on every axis");
    return POISSON_EGRID;
  }
  if (n < 2) {
    set_error("need at least 2 intervals");
    return POISSON_EGRID;
  }
  if (g->ext_in != 0 || g->ext_out != 0) {
    set_error("radial pads belong to spherical grids");
    return POISSON_EGRID;
  }
  const double h = (g->hi[0] - g->lo[0]) / n;
  for (int d = 0; d < 3; ++d) {
    const double hd = (g->hi[d] - g->lo[d]) / n;
    if (!(hd > 0.0) || fabs(hd - h) > 1e-12 * h) {
      set_error("Cartesian grids must be isotropic (equal spacing on all axes)");
      return POISSON_EGRID;
    }
  }
  if (o->method == POISSON_MG_SPAI || o->method == POISSON_MG_SPAI32) {
    if (o->order != 2 && o->order != 4 && o->order != 6) {
      set_error("the SPAI multigrid takes the compact stencils of order 2, 4 or 6");
      return POISSON_EINVAL;
    }
    if (o->coarse_tol > 0.0 && o->coarsest > 12) {
      set_error("the CG coarsest solve keeps its level in LDS: coarsest <= 12 intervals");
      return POISSON_EINVAL;
    }
  } else if (o->order != 2 && o->order != 6) {
    set_error("order must be 2 (7-point) or 6 (19-point star)");
    return POISSON_EINVAL;
  }
  // the 19-point star reads three ghost layers of Phi; the compact
  // sixth-order right-hand side reads two layers of rho
  const bool spai = o->method == POISSON_MG_SPAI || o->method == POISSON_MG_SPAI32;
  const int need_g = o->order != 6 ? 1 : spai ? 2 : 3;
  if (g->ghost != need_g) {
    set_error("order %d needs ghost = %d", o->order, need_g);
    return POISSON_EGRID;
  }
  const int M = n + 1 + 2 * (g->ghost - 1);
  if ((!spai && residual_blocks(make_geom(n, g->ghost, o->order == 6 ? 4 : 2, 1.0)) > kPartialCap) ||
      (spai && n27_blocks(make_ngeom(n, 1.0)) > kPartialCap)) {
    set_error("grid too large for the reduction buffers");
    return POISSON_EGRID;
  }
  if (g->pitch[0] < M || g->pitch[1] < (int64_t)M * g->pitch[0]) {
    set_error("pitch too small: need pitch[0] >= %d and pitch[1] >= %d*pitch[0]", M, M);
    return POISSON_EINVAL;
  }
  switch (o->method) {
    case POISSON_SOR:
      if (o->order != 2) {
        set_error("red-black SOR is defined for the 7-point operator");
        return POISSON_EINVAL;
      }
      break;
    case POISSON_CG:
    case POISSON_PCG:
      break;
    case POISSON_MG:
    case POISSON_MG_IR32:
    case POISSON_MG_SPAI:
    case POISSON_MG_SPAI32: {
      if (o->coarsest < 2 || o->nu1 < 0 || o->nu2 < 0) {
        set_error("multigrid needs coarsest >= 2, nu >= 0");
        return POISSON_EINVAL;
      }
      if (n % o->coarsest != 0 || !is_pow2(n / o->coarsest)) {
        set_error("multigrid needs n = 2^L * coarsest (n = %d, coarsest = %d)", n, o->coarsest);
        return POISSON_EGRID;
      }
      const int Nc = (o->coarsest - 1) * (o->coarsest - 1) * (o->coarsest - 1);
      if (Nc > 4096) {
        set_error("coarsest level too large for the dense solve (%d unknowns)", Nc);
        return POISSON_EGRID;
      }
      break;
    }
    default:
      set_error("method %d is not available on Cartesian grids", o->method);
      return POISSON_EINVAL;
  }
  return POISSON_OK;
}

// Lay out (or measure, when base == nullptr) the workspace of a plan.
void carve(poisson_plan_s* P, Carver& cv) {
  const poisson_grid_t& g = P->grid;
  const poisson_opts_t& o = P->opts;
  P->partial = (double*)cv.take(sizeof(double) * 2 * kPartialCap);
  P->scal = (Scalars*)cv.take(sizeof(Scalars));
  P->qlm = (double*)cv.take(sizeof(double) * 2 * kNqMax);
  if (!P->sph) {
    P->mom_mono = (int*)cv.take(sizeof(int) * kMonoMax);
    P->mom_toff = (int*)cv.take(sizeof(int) * (kNqMax + 1));
    P->mom_tmono = (int*)cv.take(sizeof(int) * kTermMax);
    P->mom_tcoef = (double*)cv.take(sizeof(double) * kTermMax);
    P->mom_scratch = (double*)cv.take(cart_moment_scratch(g.n[0]));
  }
  if (P->sph) {
    P->mom_scratch = (double*)cv.take(sph_moment_scratch(g.n[1], g.n[2]));
    const long long elems = g.pitch[1] * (long long)g.n[2];
    const size_t vb = sizeof(double) * elems;
    P->sc.cot = (const double*)cv.take(sizeof(double) * g.n[1]);
    P->sc.isin2 = (const double*)cv.take(sizeof(double) * g.n[1]);
    P->sc.r2 = (const double*)cv.take(sizeof(double) * (g.n[0] + 2));
    P->sc.rcl = (const double*)cv.take(sizeof(double) * (g.n[0] + 2));
    P->sc.rcr = (const double*)cv.take(sizeof(double) * (g.n[0] + 2));
    P->S.rr = (const double*)cv.take(sizeof(double) * (g.n[0] + 2));
    P->S.rw = (const double*)cv.take(sizeof(double) * (g.n[0] + 2));
    P->sr = (double*)cv.take(vb);
    P->srh = (double*)cv.take(vb);
    for (int i = 0; i < 2; ++i) {
      P->sp[i] = (double*)cv.take(vb);
      P->sv[i] = (double*)cv.take(vb);
    }
    P->ss = (double*)cv.take(vb);
    P->stt = (double*)cv.take(vb);
    if (o.method == POISSON_SOR) {
      // relaxation factors and local spectral radii per colatitude and radial index
      const size_t nrel = (size_t)g.n[1] * (g.n[0] + 2);
      P->somega = (double*)cv.take(sizeof(double) * nrel);
      P->somega2 = (double*)cv.take(sizeof(double) * nrel);
      P->srj = (double*)cv.take(sizeof(double) * nrel);
    }
    P->slv.clear();
    if (o.method == POISSON_BICGSTAB_MG32) {
      int lev = 0;
      for (const auto& d : sph_levels(g.n[0], g.n[1], g.n[2])) {
        SLev L{};
        L.nr = d[0];
        L.nth = d[1];
        L.nph = d[2];
        L.hp = (L.nr + 3) / 2;  // radial array indices 0 .. nr+1 split by parity
        L.p0 = 2 * L.hp;
        L.p1 = (long long)L.nth * L.p0;
        const double dth = M_PI / L.nth, dph = 2.0 * M_PI / L.nph;
        L.idt2 = (float)(1.0 / (dth * dth));
        L.idp2 = (float)(1.0 / (dph * dph));
        const size_t fb = sizeof(float) * (size_t)L.count();
        L.u = (float*)cv.take(fb);
        L.f = (float*)cv.take(fb);
        L.r = (float*)cv.take(fb);
        L.rcl = (const float*)cv.take(sizeof(float) * L.nr);
        L.rcr = (const float*)cv.take(sizeof(float) * L.nr);
        L.cot2 = (const float*)cv.take(sizeof(float) * L.nth);
        L.isin2 = (const float*)cv.take(sizeof(float) * L.nth);
        // unknown I of level `lev` sits at xi = 2^lev I + (2^lev - 1)/2 - p;
        // from the first I with xi >= 0 on, the map is the log map and the
        // couplings (so the line tables) are the same
        {
          const int p = g.ext_in > 0 ? g.ext_in - 1 : 0;
          const double h = (double)(1 << lev);
          const int i0 = (int)ceil((p - 0.5 * (h - 1.0)) / h);
          L.ntab = 1 + std::min(std::max(i0, 0), L.nr - 1);
        }
        if (line_split(L.nph, &L.seg, &L.nseg, &L.nl)) {
          L.tstride = 4 * L.seg + 4 * L.nseg * L.nseg;
          const size_t nlines = (size_t)L.nth * L.ntab;
          L.ltab = (const float*)cv.take(sizeof(float) * (size_t)L.tstride * nlines);
        }
        P->slv.push_back(L);
        ++lev;
      }
      const SLev& C = P->slv.back();
      P->sncoarse = C.nr * C.nth * C.nph;
      P->scinv = (double*)cv.take(sizeof(double) * (size_t)P->sncoarse * P->sncoarse);
    }
    return;
  }
  const int n = g.n[0];
  const double h = (g.hi[0] - g.lo[0]) / n;
  if (o.method == POISSON_MG_SPAI || o.method == POISSON_MG_SPAI32) {
    P->nlv.clear();
    for (int nl = n;; nl /= 2) {
      NLevel L;
      L.G = make_ngeom(nl, h * (n / nl));
      L.f32 = o.method == POISSON_MG_SPAI32 && nl != n;
      const size_t b = (L.f32 ? sizeof(float) : sizeof(double)) * L.G.total();
      const bool dense_only = nl == o.coarsest && nl != n;  // coarsest below the finest: solved densely
      L.u = cv.take(b);
      L.u2 = dense_only ? nullptr : cv.take(b);
      L.f = cv.take(b);
      L.r = dense_only ? nullptr : cv.take(b);
      P->nlv.push_back(L);
      if (nl == o.coarsest) break;
    }
    const int E = o.coarsest - 1;
    P->ncoarse = E * E * E;
    P->cinv = (double*)cv.take(sizeof(double) * (size_t)P->ncoarse * P->ncoarse);
    return;
  }
  P->G0 = make_geom(n, g.ghost, P->C, h);
  const size_t b64 = sizeof(double) * P->G0.total();
  P->phi64 = (double*)cv.take(b64);
  P->f64 = (double*)cv.take(b64);
  P->t64 = (double*)cv.take(b64);
  if (o.method == POISSON_CG || o.method == POISSON_PCG) {
    P->cr = (double*)cv.take(b64);
    P->cp0 = (double*)cv.take(b64);
    P->cp1 = (double*)cv.take(b64);
    P->cq = (double*)cv.take(b64);
    if (o.method == POISSON_PCG) P->cz = (double*)cv.take(b64);
  }
  if (o.method == POISSON_MG || o.method == POISSON_MG_IR32) {
    P->mg32 = o.method == POISSON_MG_IR32;
    const size_t es = P->mg32 ? sizeof(float) : sizeof(double);
    P->lv.clear();
    int nl = n;
    double hl = h;
    bool first = true;
    while (true) {
      Level L;
      L.G = make_geom(nl, g.ghost, P->C, hl);
      if (first && !P->mg32) {
        L.phi = P->phi64;
        L.f = P->f64;
        L.tmp = P->t64;
      } else {
        L.phi = cv.take(es * L.G.total());
        L.f = cv.take(es * L.G.total());
        L.tmp = (nl == o.coarsest) ? nullptr : cv.take(es * L.G.total());
      }
      P->lv.push_back(L);
      first = false;
      if (nl == o.coarsest) break;
      nl /= 2;
      hl *= 2.0;
    }
    const int E = o.coarsest - 1;
    P->ncoarse = E * E * E;
    P->cinv = (double*)cv.take(sizeof(double) * (size_t)P->ncoarse * P->ncoarse);
  }
}

// Dense matrix of L_h on the (E)^3 unknowns of a level with zero ghosts
// (7-point or 19-point star), inverted through a Cholesky factorisation of
// the SPD matrix -L_h.  Returns false if the factorisation fails.
bool coarse_inverse_compute(int nc, double h, int order, std::vector<double>& inv) {
  const int E = nc - 1;
  const int N = E * E * E;
  std::vector<double> A((size_t)N * N, 0.0);
  const double ih2 = 1.0 / (h * h);
  const double w[4] = {-49.0 / 18.0, 1.5, -3.0 / 20.0, 1.0 / 90.0};
  auto id = [&](int i, int j, int k) { return (k * E + j) * E + i; };
  for (int k = 0; k < E; ++k)
    for (int j = 0; j < E; ++j)
      for (int i = 0; i < E; ++i) {
        const int row = id(i, j, k);
        // -L: SPD
        if (order == 2) {
          A[(size_t)row * N + row] = 6.0 * ih2;
          const int di[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
          for (auto& d : di) {
            const int a = i + d[0], b = j + d[1], c = k + d[2];
            if (a >= 0 && a < E && b >= 0 && b < E && c >= 0 && c < E) A[(size_t)row * N + id(a, b, c)] -= ih2;
          }
        } else {
          A[(size_t)row * N + row] = -3.0 * w[0] * ih2;
          for (int q = 1; q <= 3; ++q) {
            const int di[6][3] = {{q, 0, 0}, {-q, 0, 0}, {0, q, 0}, {0, -q, 0}, {0, 0, q}, {0, 0, -q}};
            for (auto& d : di) {
              const int a = i + d[0], b = j + d[1], c = k + d[2];
              if (a >= 0 && a < E && b >= 0 && b < E && c >= 0 && c < E)
                A[(size_t)row * N + id(a, b, c)] -= w[q] * ih2;
            }
          }
        }
      }
  // Cholesky A = U^T U (upper), in place
  std::vector<double> U = A;
  for (int i = 0; i < N; ++i) {
    for (int k = 0; k < i; ++k) {
      const double f = U[(size_t)k * N + i];
      if (f == 0.0) continue;
      for (int j = i; j < N; ++j) U[(size_t)i * N + j] -= f * U[(size_t)k * N + j];
    }
    const double d = U[(size_t)i * N + i];
    if (!(d > 0.0)) return false;
    const double s = 1.0 / sqrt(d);
    for (int j = i; j < N; ++j) U[(size_t)i * N + j] *= s;
  }
  // inverse of -L: solve U^T U x = e_c for every column, then negate
  inv.assign((size_t)N * N, 0.0);
  std::vector<double> y(N);
  for (int c = 0; c < N; ++c) {
    for (int i = 0; i < N; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= U[(size_t)k * N + i] * y[k];
      y[i] = s / U[(size_t)i * N + i];
    }
    for (int i = N - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < N; ++k) s -= U[(size_t)i * N + k] * y[k];
      y[i] = s / U[(size_t)i * N + i];
    }
    for (int r = 0; r < N; ++r) inv[(size_t)r * N + c] = -y[r];
  }
  return true;
}

// The exact coarsest inverse depends only on (intervals, spacing, stencil);
// plans of the same shape share one host copy instead of refactorising.
bool coarse_inverse(int nc, double h, int order, std::vector<double>& inv) {
  static std::mutex mu;
  static std::map<std::tuple<int, double, int>, std::vector<double>> cache;
  const auto key = std::make_tuple(nc, h, order);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      inv = it->second;
      return true;
    }
  }
  if (!coarse_inverse_compute(nc, h, order, inv)) return false;
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = inv;
  return true;
}

// Inverse of a general dense matrix by Gauss-Jordan elimination with partial
// pivoting (the spherical operator is not symmetric).
bool invert_general(int N, std::vector<double>& A, std::vector<double>& inv) {
  inv.assign((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i) inv[(size_t)i * N + i] = 1.0;
  for (int c = 0; c < N; ++c) {
    int piv = c;
    for (int r = c + 1; r < N; ++r)
      if (fabs(A[(size_t)r * N + c]) > fabs(A[(size_t)piv * N + c])) piv = r;
    if (!(fabs(A[(size_t)piv * N + c]) > 0.0)) return false;
    if (piv != c)
      for (int k = 0; k < N; ++k) {
        std::swap(A[(size_t)c * N + k], A[(size_t)piv * N + k]);
        std::swap(inv[(size_t)c * N + k], inv[(size_t)piv * N + k]);
      }
    const double d = 1.0 / A[(size_t)c * N + c];
    for (int k = 0; k < N; ++k) {
      A[(size_t)c * N + k] *= d;
      inv[(size_t)c * N + k] *= d;
    }
    for (int r = 0; r < N; ++r) {
      if (r == c) continue;
      const double f = A[(size_t)r * N + c];
      if (f == 0.0) continue;
      for (int k = 0; k < N; ++k) {
        A[(size_t)r * N + k] -= f * A[(size_t)c * N + k];
        inv[(size_t)r * N + k] -= f * inv[(size_t)c * N + k];
      }
    }
  }
  return true;
}

// Dense operator of a spherical multigrid level (zero radial ghosts, pole
// reflection, periodic phi), in the same coefficients as the level kernels;
// cl, cr: radial couplings per radial unknown.
void sph_level_matrix(int nr, int nth, int nph, const std::vector<double>& cl, const std::vector<double>& cr,
                      std::vector<double>& A) {
  const int N = nr * nth * nph;
  A.assign((size_t)N * N, 0.0);
  const double dth = M_PI / nth, dph = 2.0 * M_PI / nph;
  const int half = nph / 2;
  auto id = [&](int i, int j, int k) { return (k * nth + j) * nr + i; };
  for (int k = 0; k < nph; ++k)
    for (int j = 0; j < nth; ++j) {
      const double th = (j + 0.5) * dth;
      const double cot2 = cos(th) / sin(th) / (2.0 * dth), is2 = 1.0 / (sin(th) * sin(th));
      for (int i = 0; i < nr; ++i) {
        double* row = &A[(size_t)id(i, j, k) * N];
        row[id(i, j, k)] += -(cl[i] + cr[i]) - 2.0 / (dth * dth) - 2.0 * is2 / (dph * dph);
        if (i + 1 < nr) row[id(i + 1, j, k)] += cr[i];
        if (i > 0) row[id(i - 1, j, k)] += cl[i];
        row[(j + 1 < nth) ? id(i, j + 1, k) : id(i, nth - 1, (k + half) % nph)] += 1.0 / (dth * dth) + cot2;
        row[(j > 0) ? id(i, j - 1, k) : id(i, 0, (k + half) % nph)] += 1.0 / (dth * dth) - cot2;
        row[id(i, j, (k + 1) % nph)] += is2 / (dph * dph);
        row[id(i, j, (k + nph - 1) % nph)] += is2 / (dph * dph);
      }
    }
}

// Tables of the phi-line smoother for one level (layout in SLev): line
// (i, j) is the periodic tridiagonal system a x[k-1] + b x[k] + a x[k+1]
// with a = 1 / (sin^2 theta_j dphi^2) and b the level diagonal
// -(cl_i + cr_i) - 2/dtheta^2 - 2a (one table per j when the radial
// couplings are constant, per (i, j) otherwise); computed in FP64, stored
// FP32.
bool line_tables(const SLev& L, const std::vector<double>& cl, const std::vector<double>& cr,
                 std::vector<float>& tab) {
  const int SL = L.seg, Pn = L.nseg;
  const int ni = L.ntab;
  tab.assign((size_t)L.tstride * L.nth * ni, 0.0f);
  const double dth = M_PI / L.nth, dph = 2.0 * M_PI / L.nph;
  std::vector<double> m(SL), cp(SL), v(SL), w(SL), K, G;
  for (int it = 0; it < ni; ++it)
  for (int j = 0; j < L.nth; ++j) {
    const double th = (j + 0.5) * dth;
    const double a = 1.0 / (sin(th) * sin(th) * dph * dph);
    const double b = -(cl[it] + cr[it]) - 2.0 / (dth * dth) - 2.0 * a;
    m[0] = 1.0 / b;
    cp[0] = a / b;
    for (int q = 1; q < SL; ++q) {
      const double den = b - a * cp[q - 1];
      m[q] = 1.0 / den;
      cp[q] = a / den;
    }
    auto tsolve = [&](int unit, std::vector<double>& y) {
      double d = 0.0;
      for (int q = 0; q < SL; ++q) {
        d = ((q == unit ? 1.0 : 0.0) - a * d) * m[q];
        y[q] = d;
      }
      for (int q = SL - 2; q >= 0; --q) y[q] -= cp[q] * y[q + 1];
    };
    tsolve(0, v);
    tsolve(SL - 1, w);
    // interface system: X[2s] = x at the first node of segment s, X[2s+1] at
    // its last; X + a (v X_left + w X_right) = E
    const int n2 = 2 * Pn;
    K.assign((size_t)n2 * n2, 0.0);
    for (int q = 0; q < n2; ++q) K[(size_t)q * n2 + q] = 1.0;
    for (int sgi = 0; sgi < Pn; ++sgi) {
      const int xl = 2 * ((sgi + Pn - 1) % Pn) + 1, xr = 2 * ((sgi + 1) % Pn);
      K[(size_t)(2 * sgi) * n2 + xl] += a * v[0];
      K[(size_t)(2 * sgi) * n2 + xr] += a * w[0];
      K[(size_t)(2 * sgi + 1) * n2 + xl] += a * v[SL - 1];
      K[(size_t)(2 * sgi + 1) * n2 + xr] += a * w[SL - 1];
    }
    if (!invert_general(n2, K, G)) return false;
    float* t = &tab[((size_t)it * L.nth + j) * L.tstride];
    for (int q = 0; q < SL; ++q) {
      t[q] = (float)m[q];
      t[SL + q] = (float)cp[q];
      t[2 * SL + q] = (float)v[q];
      t[3 * SL + q] = (float)w[q];
    }
    for (int q = 0; q < n2 * n2; ++q) t[4 * SL + q] = (float)G[q];
  }
  return true;
}

// Table 1: SPAI smoother coefficients (omega, alpha, beta, gamma, delta) of
// the compact stencils of order 2, 4 and 6.  The printed order-6 delta cell
// repeats mu and makes the smoother diverge; 0.0151 minimises the smoothing
// factor with the other four printed values (mu 0.0912 against 0.0909).
const double kSpai[3][5] = {{1.3699, 0.1432, 0.0284, 0.0081, 0.0025},
                            {0.9363, 0.2807, 0.0329, 0.0166, 0.0044},
                            {0.3543, 0.7064, 0.1005, 0.0363, 0.0151}};

// Galerkin product R A P of a cubically symmetric radius-1 stencil with full
// weighting and trilinear prolongation.  Per axis, R shift(d) P is the coarse
// 1-D stencil s_d: s_0 = (1/8, 3/4, 1/8), s_+1 = (1/2, 1/2, 0),
// s_-1 = (0, 1/2, 1/2) (entries for coarse offsets -1, 0, +1), and the 3-D
// product factorises, so W(D) = sum_d w(d) s_dx(Dx) s_dy(Dy) s_dz(Dz).
W4 galerkin_w4(const W4& w) {
  const double s[3][3] = {{0.0, 0.5, 0.5}, {0.125, 0.75, 0.125}, {0.5, 0.5, 0.0}};  // [d+1][D+1]
  const double cls[4] = {w.c, w.f, w.e, w.k};
  double out[4] = {0, 0, 0, 0};
  // read each class at one representative offset D: (0,0,0), (1,0,0), (1,1,0), (1,1,1)
  const int rep[4][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {1, 1, 1}};
  for (int c = 0; c < 4; ++c)
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int nz = (dx != 0) + (dy != 0) + (dz != 0);
          out[c] += cls[nz] * s[dx + 1][rep[c][0] + 1] * s[dy + 1][rep[c][1] + 1] * s[dz + 1][rep[c][2] + 1];
        }
  return W4{out[0], out[1], out[2], out[3]};
}

// dense matrix of a W4 stencil on the (n-1)^3 unknowns with zero ghosts
void w4_matrix(const W4& w, int n, std::vector<double>& A) {
  const int E = n - 1;
  const int N = E * E * E;
  A.assign((size_t)N * N, 0.0);
  const double cls[4] = {w.c, w.f, w.e, w.k};
  for (int k = 0; k < E; ++k)
    for (int j = 0; j < E; ++j)
      for (int i = 0; i < E; ++i)
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int a = i + dx, b = j + dy, c = k + dz;
              if (a < 0 || a >= E || b < 0 || b >= E || c < 0 || c >= E) continue;
              A[(size_t)((k * E + j) * E + i) * N + (c * E + b) * E + a] += cls[(dx != 0) + (dy != 0) + (dz != 0)];
            }
}

// ------------------------------------------------------------ solver pieces
// One V(nu1, nu2) cycle from level l down.  zero_guess: the level's
// unknowns start at zero (every coarse correction, and the FP32 correction of
// a refinement step), so the first forward sweep reads colours it has not yet
// updated as zero instead of clearing the array first.  On two-colour levels
// a Gauss-Seidel pass leaves its colour's residual at zero: after the
// pre-smoothing (last colour 1) only colour-0 residuals are restricted.  On
// every level the correction skips the last colour, since the first
// post-smoothing pass (that colour) reads none of its values and overwrites
// them all.
void vcycle(poisson_plan_s* P, int l, bool zero_guess, hipStream_t st) {
  Level& L = P->lv[l];
  const bool f32 = P->mg32;
  const poisson_opts_t& o = P->opts;
  const int C = P->C;
  if (l + 1 == (int)P->lv.size()) {
    coarse_solve(P->cinv, L.f, L.phi, f32, L.G, st);
    return;
  }
  if (zero_guess && o.nu1 == 0) zero_unknowns(L.phi, f32, L.G, st);
  for (int s = 0; s < o.nu1; ++s)
    for (int c = 0; c < C; ++c) {
      int zmask = 0;
      if (zero_guess && s == 0) zmask = ((1 << C) - 1) & ~((1 << (c + 1)) - 1);  // colours > c
      colour_pass(L.phi, L.f, f32, L.G, P->order, c, 1.0, st, zmask);
    }
  Level& Lc = P->lv[l + 1];
  if (P->order == 2 && resrestrict_ok(L.G)) {
    resrestrict(L.phi, L.f, f32, L.G, Lc.f, Lc.G, st, o.nu1 > 0);
  } else if (resrestrict19_ok(L.G)) {
    resrestrict19(L.phi, L.f, f32, L.G, Lc.f, Lc.G, nullptr, o.nu1 > 0, st);
  } else {
    // after a forward pre-smoothing sweep the residuals of the last colour
    // vanish; on four-colour levels the restriction does not read them
    residual(L.phi, L.f, f32, L.tmp, f32, L.G, P->order, false, nullptr, st);
    restrict_fw(L.tmp, L.G, Lc.f, Lc.G, f32, st, C == 4 && o.nu1 > 0);
  }
  vcycle(P, l + 1, true, st);
  prolong_add(Lc.phi, Lc.G, L.phi, L.G, f32, st, o.nu2 > 0);
  for (int s = 0; s < o.nu2; ++s)
    for (int c = C - 1; c >= 0; --c) colour_pass(L.phi, L.f, f32, L.G, P->order, c, 1.0, st);
}

// One FP32 V(nu1, nu2) cycle of the spherical preconditioner from level l on a
// zero initial guess (colours forward before, backward after the correction).
void svcycle(poisson_plan_s* P, int l, hipStream_t st) {
  const SLev& L = P->slv[l];
  if (l + 1 == (int)P->slv.size()) {
    sph_coarse32(P->scinv, L, st);
    return;
  }
  // zero guess: the first colour-0 pass sees u = 0 and writes every colour-0
  // line; the colour-1 pass then reads colour-0 values and, across a pole,
  // its own (still zero) lines; radial ghosts stay zero from plan creation,
  // so u needs no clearing
  for (int s = 0; s < P->opts.nu1; ++s)
    for (int c = 0; c < 2; ++c) sph_line_pass(L, c, s == 0 ? (c == 0 ? 1 : 2) : 0, st);
  sph_residual32(L, st);
  sph_restrict32(L, P->slv[l + 1], st);
  svcycle(P, l + 1, st);
  sph_prolong_add32(P->slv[l + 1], L, st);
  for (int s = 0; s < P->opts.nu2; ++s)
    for (int c = 1; c >= 0; --c) sph_line_pass(L, c, 0, st);
}

// yhat = M^-1 y with M^-1 one FP32 V-cycle (inputs / outputs FP64)
void sph_precond(poisson_plan_s* P, const double* y, double* yhat, hipStream_t st) {
  sph_cast_in(y, P->S, P->slv[0], st);
  svcycle(P, 0, st);
  sph_cast_out(P->slv[0], yhat, P->S, st);
}

// one right-preconditioned BiCGSTAB iteration with the multigrid preconditioner
void sph_mg_iteration(poisson_plan_s* P, double* phi, hipStream_t st) {
  const SGeom& S = P->S;
  const int nb = sph_blocks(S);
  double* p = P->sp[0];
  double* phat = P->sp[1];
  double* v = P->sv[0];
  double* shat = P->sv[1];
  pbicg_update_p(P->sr, p, v, S, P->sc, P->scal, st);
  sph_precond(P, p, phat, st);
  pbicg_apply(phat, v, P->srh, 0, S, P->sc, P->partial, st);
  bicg_scalars(P->partial, nb, P->scal, 0, st);
  pbicg_update_s(P->sr, v, P->ss, S, P->sc, P->scal, st);
  sph_precond(P, P->ss, shat, st);
  pbicg_apply(shat, P->stt, P->ss, 1, S, P->sc, P->partial, st);
  bicg_scalars(P->partial, nb, P->scal, 1, st);
  pbicg_xr(phi, P->sr, phat, shat, P->ss, P->stt, P->srh, S, P->scal, P->partial, st);
  bicg_scalars(P->partial, nb, P->scal, 2, st);
}

// Stream on which the plan's graphs are recorded: the caller's capture
// stream when one was given, else the plan's own stream; the NULL stream
// cannot be captured, so with neither the steps run kernel by kernel.
hipStream_t capture_stream(const poisson_plan_s* P) { return P->cap ? P->cap : P->st; }

int capture_sph_iteration(poisson_plan_s* P, double* phi) {
  if (P->iter_exec && P->iter_phi == phi) return POISSON_OK;
  if (P->iter_exec) {
    hipGraphExecDestroy(P->iter_exec);
    P->iter_exec = nullptr;
  }
  hipGraph_t graph = nullptr;
  hipStream_t cs = capture_stream(P);
  HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  sph_mg_iteration(P, phi, cs);
  hipError_t e = hipStreamEndCapture(cs, &graph);
  if (e != hipSuccess) {
    set_error("graph capture failed: %s", hipGetErrorString(e));
    return POISSON_EHIP;
  }
  e = hipGraphInstantiate(&P->iter_exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) {
    P->iter_exec = nullptr;
    set_error("graph instantiation failed: %s", hipGetErrorString(e));
    return POISSON_EHIP;
  }
  P->iter_phi = phi;
  return POISSON_OK;
}

// `steps` fused Richardson steps on level L, alternating between u and u2;
// returns the array holding the result.
void* spai_smooth(NLevel& L, void* cur, int steps, hipStream_t st) {
  for (int s = 0; s < steps; ++s) {
    void* nxt = (cur == L.u) ? L.u2 : L.u;
    n_spai_step(cur, L.f, nxt, L.f32, L.G, L.A, L.M, st);
    cur = nxt;
  }
  return cur;
}

// One SPAI V(nu1, nu2) cycle from level l: Richardson steps u <- u - M (f - A u)
// (Eq. richardson), Galerkin coarse problems on a zero initial guess.  The
// result is left in L.u (copied back when the step count is odd).
void spai_vcycle(poisson_plan_s* P, int l, hipStream_t st) {
  NLevel& L = P->nlv[l];
  if (l + 1 == (int)P->nlv.size()) {
    if (P->opts.coarse_tol > 0.0)
      n_coarse_cg(L.f, L.u, L.f32, L.G, L.A, P->opts.coarse_tol, st);
    else
      n_coarse(P->cinv, L.f, L.u, L.f32, L.G, st);
    return;
  }
  void* cur = spai_smooth(L, L.u, P->opts.nu1, st);
  n27_residual(cur, L.f, L.r, L.f32, L.G, L.A, false, nullptr, st);
  NLevel& C = P->nlv[l + 1];
  n_restrict(L.r, L.f32, L.G, C.f, C.f32, C.G, st);
  fill_zero(C.u, C.f32, C.G.total(), st);
  spai_vcycle(P, l + 1, st);
  n_prolong_add(C.u, C.f32, C.G, cur, L.f32, L.G, st);
  cur = spai_smooth(L, cur, P->opts.nu2, st);
  if (cur != L.u) n_copy(cur, L.u, L.f32, L.G, st);
}

void spai_step(poisson_plan_s* P, hipStream_t st) {
  NLevel& L = P->nlv[0];
  spai_vcycle(P, 0, st);
  n27_residual(L.u, L.f, nullptr, false, L.G, L.A, true, P->partial, st);
  finish_sum(P->partial, (int)n27_blocks(L.G), 1, P->scal, kRes2, st);
}

// One multigrid iteration followed by the fine residual norm into
// scal->v[kRes2].  MG: a V-cycle on (phi64; f64).  MG_IR32: the FP32
// V-cycle for the correction e of the current FP32 residual r32, phi64 += e,
// and the new FP64 residual, stored as FP32 for the next step.
void mg_step(poisson_plan_s* P, hipStream_t st) {
  const int nb = residual_blocks(P->G0);
  if (P->mg32) {
    Level& L0 = P->lv[0];
    vcycle(P, 0, true, st);
    add_correction(P->phi64, L0.phi, true, P->G0, st);
    residual(P->phi64, P->f64, false, L0.f, true, P->G0, P->order, false, P->partial, st);
  } else {
    vcycle(P, 0, false, st);
    // the cycle ends with a Gauss-Seidel pass over colour 0 on two-colour
    // grids: only colour 1 carries a residual
    const int col = (P->C == 2 && P->opts.nu2 > 0 && P->lv.size() > 1) ? 1 : -1;
    residual(P->phi64, P->f64, false, nullptr, false, P->G0, P->order, false, P->partial, st, col);
  }
  finish_sum(P->partial, nb, 1, P->scal, kRes2, st);
}

// Record what fn enqueues on the capture stream into *exec (once).
template <typename Fn>
int capture_into(poisson_plan_s* P, hipGraphExec_t* exec, Fn fn) {
  if (*exec) return POISSON_OK;
  hipGraph_t graph = nullptr;
  hipStream_t cs = capture_stream(P);
  HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  fn(cs);
  hipError_t e = hipStreamEndCapture(cs, &graph);
  if (e != hipSuccess) {
    set_error("graph capture failed: %s", hipGetErrorString(e));
    return POISSON_EHIP;
  }
  e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) {
    *exec = nullptr;
    set_error("graph instantiation failed: %s", hipGetErrorString(e));
    return POISSON_EHIP;
  }
  return POISSON_OK;
}

int capture_step(poisson_plan_s* P) {
  return capture_into(P, &P->step_exec, [P](hipStream_t cs) {
    if (!P->nlv.empty())
      spai_step(P, cs);
    else
      mg_step(P, cs);
  });
}

// FP64 multigrid whose finest level stores its residual for the restriction
// (four-colour levels; two-colour levels too large for the fused residual and
// restriction): a solve stops on that residual, formed after the
// pre-smoothing of every cycle, instead of forming another one after the
// cycle.  The iterate it returns is the one after that pre-smoothing.
bool split_cycle(const poisson_plan_s* P) {
  return !P->mg32 && P->lv.size() > 1 && P->opts.nu1 > 0 && !(P->order == 2 && resrestrict_ok(P->G0));
}

// head of a cycle: pre-smoothing of the finest level, its residual (kept for
// the restriction) and the residual's norm^2 into scal->v[kRes2]
void cycle_head(poisson_plan_s* P, hipStream_t st) {
  Level& L = P->lv[0];
  for (int s = 0; s < P->opts.nu1; ++s)
    for (int c = 0; c < P->C; ++c) colour_pass(L.phi, L.f, false, L.G, P->order, c, 1.0, st);
  int nb = residual_blocks(L.G);
  if (resrestrict19_ok(L.G)) {
    // the coarse right-hand side is formed here, with the norm
    Level& Lc = P->lv[1];
    nb = resrestrict19(L.phi, L.f, false, L.G, Lc.f, Lc.G, P->partial, true, st);
  } else {
    residual(L.phi, L.f, false, L.tmp, false, L.G, P->order, false, P->partial, st);
  }
  finish_sum(P->partial, nb, 1, P->scal, kRes2, st);
}

// tail of a cycle: restriction of the head's residual (the last colour's
// vanish on four-colour levels) unless the head restricted it already, the
// coarse cycle, prolongation and post-smoothing
void cycle_tail(poisson_plan_s* P, hipStream_t st) {
  Level& L = P->lv[0];
  Level& Lc = P->lv[1];
  const poisson_opts_t& o = P->opts;
  if (!resrestrict19_ok(L.G)) restrict_fw(L.tmp, L.G, Lc.f, Lc.G, false, st, P->C == 4);
  vcycle(P, 1, true, st);
  prolong_add(Lc.phi, Lc.G, L.phi, L.G, false, st, o.nu2 > 0);
  for (int s = 0; s < o.nu2; ++s)
    for (int c = P->C - 1; c >= 0; --c) colour_pass(L.phi, L.f, false, L.G, P->order, c, 1.0, st);
}

// first == true: the head of the first cycle; else the tail of the current
// cycle and the head of the next
int launch_split(poisson_plan_s* P, bool first) {
  if (!capture_stream(P)) {
    if (!first) cycle_tail(P, P->st);
    cycle_head(P, P->st);
    return launch_check("multigrid step");
  }
  if (first) {
    CHK(capture_into(P, &P->head_exec, [P](hipStream_t cs) { cycle_head(P, cs); }));
    HIPCHK(hipGraphLaunch(P->head_exec, P->st));
  } else {
    CHK(capture_into(P, &P->cont_exec, [P](hipStream_t cs) {
      cycle_tail(P, cs);
      cycle_head(P, cs);
    }));
    HIPCHK(hipGraphLaunch(P->cont_exec, P->st));
  }
  return POISSON_OK;
}

// One multigrid iteration on the plan's stream: the captured graph when the
// plan has a stream to record it on, else its kernels one by one.
int launch_step(poisson_plan_s* P) {
  if (!capture_stream(P)) {
    if (!P->nlv.empty())
      spai_step(P, P->st);
    else
      mg_step(P, P->st);
    return launch_check("multigrid step");
  }
  CHK(capture_step(P));
  HIPCHK(hipGraphLaunch(P->step_exec, P->st));
  return POISSON_OK;
}

int read_scalars(poisson_plan_s* P, int first, int count) {
  HIPCHK(hipMemcpyAsync(P->host, &P->scal->v[first], sizeof(double) * count, hipMemcpyDeviceToHost, P->st));
  HIPCHK(hipStreamSynchronize(P->st));
  return POISSON_OK;
}

double rjac(const poisson_plan_s* P) { return cos(M_PI / P->grid.n[0]); }

int do_multipole(poisson_plan_s* P, const double* rho, double* phi, int lmax, double* h_q) {
  const poisson_grid_t& g = P->grid;
  const int nq = (lmax + 1) * (lmax + 1);
  const double G = P->opts.four_pi_G / (4.0 * M_PI);
  hipStream_t st = P->st;
  if (!P->sph) {
    const int n = g.n[0];
    const double h = (g.hi[0] - g.lo[0]) / n;
    const double cx = 0.5 * (g.lo[0] + g.hi[0]), cy = 0.5 * (g.lo[1] + g.hi[1]), cz = 0.5 * (g.lo[2] + g.hi[2]);
    const MomTables tab{P->mom_mono, P->mom_toff, P->mom_tmono, P->mom_tcoef};
    cart_moments(rho, g.pitch[0], g.pitch[1], n, g.ghost, h, cx, cy, cz, lmax, tab, P->opts.point_mass,
                 P->mom_scratch, P->qlm, st);
    cart_ghosts(phi, g.pitch[0], g.pitch[1], n, g.ghost, h, g.lo[0], cx, cy, cz, lmax, P->qlm, G, st);
  } else {
    sph_moments(rho, P->S, lmax, P->opts.point_mass, P->mom_scratch, P->qlm, P->qlm + kNqMax, st);
    sph_ghosts(phi, P->S, lmax, P->qlm, P->qlm + kNqMax, P->opts.point_mass, G, st);
  }
  CHK(launch_check("multipole_boundary"));
  if (h_q) {
    HIPCHK(hipMemcpyAsync(h_q, P->qlm, sizeof(double) * nq, hipMemcpyDeviceToHost, st));
    if (P->sph) HIPCHK(hipMemcpyAsync(h_q + nq, P->qlm + kNqMax, sizeof(double) * nq, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return POISSON_OK;
}

struct Tracker {
  poisson_stats_t* stats;
  double bnorm = 0.0;
  void push(double rel) {
    if (stats && stats->residual_history && stats->history_len < stats->history_cap)
      stats->residual_history[stats->history_len++] = rel;
  }
};

int finish_status(poisson_plan_s* P, Tracker& T, int it, double rel, bool converged, float t_mp, float t_it) {
  const int status = converged ? POISSON_OK : POISSON_WARN_MAXITER;
  if (T.stats) {
    T.stats->iterations = it;
    T.stats->status = status;
    T.stats->rel_residual = rel;
    T.stats->b_norm = T.bnorm;
    T.stats->rate = (it > 0 && rel > 0.0) ? pow(rel, 1.0 / it) : 0.0;
    T.stats->t_multipole_ms = t_mp;
    T.stats->t_iter_ms = t_it;
  }
  (void)P;
  return status;
}

double rel_of(double r2, double bnorm) {
  const double r = sqrt(std::max(r2, 0.0));
  return bnorm > 0.0 ? r / bnorm : r;
}

// One symmetric multi-colour Gauss-Seidel step for L z = r from z = 0 with
// zero ghosts (Section 2.1.2): colours 0 .. C-1 forward, each reading only
// the colours already updated (the later ones are still zero), then
// C-2 .. 0 backward; the backward sweep's first colour would repeat the
// forward sweep's last from unchanged neighbours and is left out.
// Then partial[0 .. nb) holds the partial sums of -(r . z), nb returned.
// On two-colour grids the passes that finish colours 1 and 0 form them
// (one partial per block of each); on four-colour grids a separate
// inner-product kernel.
int pcg_precondition(poisson_plan_s* P, hipStream_t st) {
  const Geom& G = P->G0;
  const int cb = cg_blocks(G);
  if (P->order == 2) {
    colour_pass(P->cz, P->cr, false, G, 2, 0, 1.0, st, 2);  // colour 1 still zero
    const int nb1 = colour_pass_dot(P->cz, P->cr, G, 1, P->partial, st);
    const int nb0 = colour_pass_dot(P->cz, P->cr, G, 0, P->partial + nb1, st);
    return nb1 + nb0;
  }
  const int C = 4;
  for (int c = 0; c < C; ++c) {
    const int zmask = ((1 << C) - 1) & ~((2 << c) - 1);  // colours above c
    colour_pass(P->cz, P->cr, false, G, P->order, c, 1.0, st, zmask);
  }
  for (int c = C - 2; c >= 0; --c) colour_pass(P->cz, P->cr, false, G, P->order, c, 1.0, st);
  pcg_dot(P->cr, P->cz, G, P->partial, st);
  return cb;
}

// ------------------------------------------------------------ Cartesian solve
int cart_setup_impl(poisson_plan_s* P, const double* rho, double* phi) {
  const poisson_grid_t& g = P->grid;
  const poisson_opts_t& o = P->opts;
  hipStream_t st = P->st;
  HIPCHK(hipEventRecord(P->ev[0], st));
  if (o.lmax >= 0) CHK(do_multipole(P, rho, phi, o.lmax, nullptr));
  HIPCHK(hipEventRecord(P->ev[1], st));
  const Geom& G = P->G0;
  split_from_natural(phi, g.pitch[0], g.pitch[1], P->phi64, false, G, 1.0, st);
  split_from_natural(rho, g.pitch[0], g.pitch[1], P->f64, false, G, o.four_pi_G, st);
  const int nb = residual_blocks(G);
  residual(P->phi64, P->f64, false, nullptr, false, G, P->order, true, P->partial, st);
  finish_sum(P->partial, nb, 1, P->scal, kBnorm2, st);
  // initial residual (MG_IR32 keeps it as the FP32 right-hand side; CG keeps it)
  void* rout = nullptr;
  bool rout32 = false;
  if (o.method == POISSON_MG_IR32) {
    rout = P->lv[0].f;
    rout32 = true;
  } else if (o.method == POISSON_CG || o.method == POISSON_PCG) {
    rout = P->cr;
  }
  residual(P->phi64, P->f64, false, rout, rout32, G, P->order, false, P->partial, st);
  finish_sum(P->partial, nb, 1, P->scal, kRes2, st);
  return launch_check("solve setup");
}

int solve_spai(poisson_plan_s* P, const double* rho, double* phi, double tol, poisson_stats_t* stats) {
  const poisson_grid_t& g = P->grid;
  const poisson_opts_t& o = P->opts;
  hipStream_t st = P->st;
  Tracker T{stats};
  if (stats) stats->history_len = 0;
  NLevel& L = P->nlv[0];
  const int nb = (int)n27_blocks(L.G);
  HIPCHK(hipEventRecord(P->ev[0], st));
  if (o.lmax >= 0) CHK(do_multipole(P, rho, phi, o.lmax, nullptr));
  HIPCHK(hipEventRecord(P->ev[1], st));
  n_rhs(rho, g.pitch[0], g.pitch[1], g.ghost, (double*)L.f, L.G, o.order, o.four_pi_G, st);
  n_from_caller(phi, g.pitch[0], g.pitch[1], g.ghost, (double*)L.u, L.G, true, st);
  n27_residual(L.u, L.f, nullptr, false, L.G, L.A, true, P->partial, st);
  finish_sum(P->partial, nb, 1, P->scal, kBnorm2, st);
  n_from_caller(phi, g.pitch[0], g.pitch[1], g.ghost, (double*)L.u, L.G, false, st);
  if (L.u2) n_from_caller(phi, g.pitch[0], g.pitch[1], g.ghost, (double*)L.u2, L.G, false, st);
  n27_residual(L.u, L.f, nullptr, false, L.G, L.A, true, P->partial, st);
  finish_sum(P->partial, nb, 1, P->scal, kRes2, st);
  CHK(launch_check("SPAI setup"));
  CHK(read_scalars(P, kBnorm2, 2));
  T.bnorm = sqrt(P->host[0]);
  double rel = rel_of(P->host[1], T.bnorm);
  T.push(rel);
  if (!isfinite(rel)) {
    set_error("non-finite initial residual (NaN/Inf in rho or phi)");
    return POISSON_ENUMERIC;
  }
  int it = 0;
  bool conv = rel <= tol;
  while (!conv && it < o.max_iter) {
    CHK(launch_step(P));
    ++it;
    if (it % o.check_every == 0 || it == o.max_iter) {
      CHK(read_scalars(P, kRes2, 1));
      rel = rel_of(P->host[0], T.bnorm);
      T.push(rel);
      if (!isfinite(rel)) {
        set_error("multigrid diverged (non-finite residual)");
        return POISSON_ENUMERIC;
      }
      conv = rel <= tol;
    }
  }
  n_to_caller((const double*)L.u, L.G, phi, g.pitch[0], g.pitch[1], g.ghost, st);
  HIPCHK(hipEventRecord(P->ev[2], st));
  HIPCHK(hipEventSynchronize(P->ev[2]));
  CHK(launch_check("SPAI multigrid"));
  float t_mp = 0.f, t_it = 0.f;
  HIPCHK(hipEventElapsedTime(&t_mp, P->ev[0], P->ev[1]));
  HIPCHK(hipEventElapsedTime(&t_it, P->ev[1], P->ev[2]));
  return finish_status(P, T, it, rel, conv, t_mp, t_it);
}

int solve_cart(poisson_plan_s* P, const double* rho, double* phi, double tol, poisson_stats_t* stats) {
  const poisson_grid_t& g = P->grid;
  const poisson_opts_t& o = P->opts;
  hipStream_t st = P->st;
  Tracker T{stats};
  if (stats) stats->history_len = 0;
  const Geom& G = P->G0;
  const int nb = residual_blocks(G);
  CHK(cart_setup_impl(P, rho, phi));
  CHK(read_scalars(P, kBnorm2, 2));
  T.bnorm = sqrt(P->host[0]);
  double rel = rel_of(P->host[1], T.bnorm);
  T.push(rel);
  if (!isfinite(rel)) {
    set_error("non-finite initial residual (NaN/Inf in rho or phi)");
    return POISSON_ENUMERIC;
  }
  int it = 0;
  bool conv = rel <= tol;
  if (o.method == POISSON_SOR) {
    const double rj = rjac(P);
    double w_opt = 2.0 / (1.0 + sqrt(1.0 - rj * rj));
    if (o.omega_mode == POISSON_OMEGA_OPT_A) w_opt = 2.0 / (1.0 + M_PI / g.n[0]);
    if (o.omega_mode == POISSON_OMEGA_FIXED) w_opt = o.omega;
    double wc = 1.0 / (1.0 - rj * rj / 2.0);  // Chebyshev sequence from n = 1
    while (!conv && it < o.max_iter) {
      for (int c = 0; c < 2; ++c) {
        double w = w_opt;
        if (o.omega_mode == POISSON_OMEGA_CHEBYSHEV) {
          w = wc;
          wc = 1.0 / (1.0 - rj * rj * wc / 4.0);
        }
        colour_pass(P->phi64, P->f64, false, G, 2, c, w, st);
      }
      ++it;
      if (it % o.check_every == 0 || it == o.max_iter) {
        residual(P->phi64, P->f64, false, nullptr, false, G, 2, false, P->partial, st);
        finish_sum(P->partial, nb, 1, P->scal, kRes2, st);
        CHK(launch_check("SOR"));
        CHK(read_scalars(P, kRes2, 1));
        rel = rel_of(P->host[0], T.bnorm);
        T.push(rel);
        if (!isfinite(rel)) {
          set_error("SOR diverged (non-finite residual)");
          return POISSON_ENUMERIC;
        }
        conv = rel <= tol;
      }
    }
  } else if (o.method == POISSON_PCG) {
    // z = M^-1 rho by one symmetric multi-colour Gauss-Seidel step on
    // L z = r (r = -rho) from z = 0; the direction is built from -z so the
    // CG kernels keep their signs (x -= alpha p, r -= alpha q); the inner
    // product rho . zeta = -(r . z) sits in v[kRR], ||r||^2 in v[kRes2].
    const int cb = cg_blocks(G);
    finish_sum(P->partial, pcg_precondition(P, st), 1, P->scal, kRR, st);
    const double zero = 0.0;
    HIPCHK(hipMemcpyAsync(&P->scal->v[2], &zero, sizeof(double), hipMemcpyHostToDevice, st));
    fill_zero(P->cp0, false, G.total(), st);
    double* pold = P->cp0;
    double* pnew = P->cp1;
    while (!conv && it < o.max_iter) {
      cg_direction_apply(P->cz, pold, pnew, P->cq, G, P->order, P->scal, P->partial, st, -1.0);
      cg_scalars(P->partial, cg_dir_blocks(G, P->order), P->scal, 0, st);
      cg_update(P->phi64, P->cr, pnew, P->cq, G, P->scal, P->partial, st);
      finish_sum(P->partial, cb, 1, P->scal, kRes2, st);
      cg_scalars(P->partial, pcg_precondition(P, st), P->scal, 1, st);
      std::swap(pold, pnew);
      ++it;
      if (it % o.check_every == 0 || it == o.max_iter) {
        CHK(launch_check("PCG"));
        CHK(read_scalars(P, kRes2, 1));
        rel = rel_of(P->host[0], T.bnorm);
        T.push(rel);
        if (!isfinite(rel)) {
          set_error("PCG breakdown (non-finite residual)");
          return POISSON_ENUMERIC;
        }
        conv = rel <= tol;
      }
    }
  } else if (o.method == POISSON_CG) {
    const int cb = cg_blocks(G);
    // rr = r.r ; beta = 0 ; p_old = 0
    finish_sum(P->partial, nb, 1, P->scal, kRR, st);
    const double zero = 0.0;
    HIPCHK(hipMemcpyAsync(&P->scal->v[2], &zero, sizeof(double), hipMemcpyHostToDevice, st));
    fill_zero(P->cp0, false, G.total(), st);
    double* pold = P->cp0;
    double* pnew = P->cp1;
    while (!conv && it < o.max_iter) {
      cg_direction_apply(P->cr, pold, pnew, P->cq, G, P->order, P->scal, P->partial, st);
      cg_scalars(P->partial, cg_dir_blocks(G, P->order), P->scal, 0, st);
      cg_update(P->phi64, P->cr, pnew, P->cq, G, P->scal, P->partial, st);
      cg_scalars(P->partial, cb, P->scal, 1, st);
      std::swap(pold, pnew);
      ++it;
      if (it % o.check_every == 0 || it == o.max_iter) {
        CHK(launch_check("CG"));
        CHK(read_scalars(P, kRR, 1));
        rel = rel_of(P->host[0], T.bnorm);
        T.push(rel);
        if (!isfinite(rel)) {
          set_error("CG breakdown (non-finite residual)");
          return POISSON_ENUMERIC;
        }
        conv = rel <= tol;
      }
    }
  } else {  // multigrid
    const bool split = split_cycle(P);
    while (!conv && it < o.max_iter) {
      CHK(split ? launch_split(P, it == 0) : launch_step(P));
      ++it;
      if (it % o.check_every == 0 || it == o.max_iter) {
        CHK(read_scalars(P, kRes2, 1));
        rel = rel_of(P->host[0], T.bnorm);
        T.push(rel);
        if (!isfinite(rel)) {
          set_error("multigrid diverged (non-finite residual)");
          return POISSON_ENUMERIC;
        }
        conv = rel <= tol;
      }
    }
  }
  merge_to_natural(P->phi64, phi, g.pitch[0], g.pitch[1], G, true, 1.0, st);
  HIPCHK(hipEventRecord(P->ev[2], st));
  CHK(launch_check("solve"));
  HIPCHK(hipEventSynchronize(P->ev[2]));
  float t_mp = 0.f, t_it = 0.f;
  HIPCHK(hipEventElapsedTime(&t_mp, P->ev[0], P->ev[1]));
  HIPCHK(hipEventElapsedTime(&t_it, P->ev[1], P->ev[2]));
  return finish_status(P, T, it, rel, conv, t_mp, t_it);
}

// ------------------------------------------------------------ spherical solve
// SOR on the spherical grid (Section 2.1.1): red half-sweep (colours 0,
// 2), then black (1, 3); the relaxation factors are per colatitude and radius -- the
// local omega_opt of Eqs. omega_final and local_rjac, the local Chebyshev
// sequence of Eq. omega_n from n = 1 advanced after every half-sweep, or a
// fixed omega.
// relaxation factors at the start of a solve
int sph_sor_init(poisson_plan_s* P) {
  const poisson_opts_t& o = P->opts;
  const std::vector<double>& rj = P->srj_host;
  std::vector<double> w(rj.size());
  for (size_t j = 0; j < rj.size(); ++j) {
    if (o.omega_mode == POISSON_OMEGA_FIXED)
      w[j] = o.omega;
    else if (o.omega_mode == POISSON_OMEGA_OPT)
      w[j] = 2.0 / (1.0 + sqrt(1.0 - rj[j] * rj[j]));
    else
      w[j] = 1.0 / (1.0 - rj[j] * rj[j] / 2.0);
  }
  HIPCHK(hipMemcpyAsync(P->somega, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice, P->st));
  HIPCHK(hipStreamSynchronize(P->st));
  return POISSON_OK;
}

// one SOR sweep: red half (colours 0, 2), then black (1, 3).  With the
// Chebyshev sequence the second pass of each half also writes the next term
// into the other table (one writer per colatitude and radius), and the
// tables swap; with nphi = 2 that pass has no writer for every entry and a
// separate kernel advances the table.
void sph_sor_sweep(poisson_plan_s* P, const double* rho, double* phi, hipStream_t st) {
  const bool cheb = P->opts.omega_mode == POISSON_OMEGA_CHEBYSHEV;
  const bool fused = cheb && P->S.nph >= 4;
  for (int half = 0; half < 2; ++half) {
    sph_sor_pass(phi, rho, P->S, P->sc, P->opts.four_pi_G, P->somega, half, st);
    if (fused) {
      sph_sor_pass(phi, rho, P->S, P->sc, P->opts.four_pi_G, P->somega, half + 2, st, P->srj, P->somega2);
      std::swap(P->somega, P->somega2);
    } else {
      sph_sor_pass(phi, rho, P->S, P->sc, P->opts.four_pi_G, P->somega, half + 2, st);
      if (cheb) sph_omega_next(P->somega, P->srj, P->S.nth * (P->S.nr + 2), st);
    }
  }
}

int solve_sph_sor(poisson_plan_s* P, const double* rho, double* phi, double tol, Tracker& T, double rel) {
  const poisson_opts_t& o = P->opts;
  hipStream_t st = P->st;
  const SGeom& S = P->S;
  const int nb = sph_blocks(S);
  CHK(sph_sor_init(P));
  int it = 0;
  bool conv = rel <= tol;
  while (!conv && it < o.max_iter) {
    sph_sor_sweep(P, rho, phi, st);
    ++it;
    if (it % o.check_every == 0 || it == o.max_iter) {
      sph_residual(phi, rho, nullptr, S, P->sc, o.four_pi_G, false, P->partial, st);
      finish_sum(P->partial, nb, 1, P->scal, kRes2, st);
      CHK(launch_check("spherical SOR"));
      CHK(read_scalars(P, kRes2, 1));
      rel = rel_of(P->host[0], T.bnorm);
      T.push(rel);
      if (!isfinite(rel)) {
        set_error("SOR diverged (non-finite residual)");
        return POISSON_ENUMERIC;
      }
      conv = rel <= tol;
    }
  }
  HIPCHK(hipEventRecord(P->ev[2], st));
  HIPCHK(hipEventSynchronize(P->ev[2]));
  float t_mp = 0.f, t_it = 0.f;
  HIPCHK(hipEventElapsedTime(&t_mp, P->ev[0], P->ev[1]));
  HIPCHK(hipEventElapsedTime(&t_it, P->ev[1], P->ev[2]));
  return finish_status(P, T, it, rel, conv, t_mp, t_it);
}

int solve_sph(poisson_plan_s* P, const double* rho, double* phi, double tol, poisson_stats_t* stats) {
  const poisson_opts_t& o = P->opts;
  hipStream_t st = P->st;
  const SGeom& S = P->S;
  Tracker T{stats};
  if (stats) stats->history_len = 0;
  HIPCHK(hipEventRecord(P->ev[0], st));
  if (o.lmax >= 0) CHK(do_multipole(P, rho, phi, o.lmax, nullptr));
  HIPCHK(hipEventRecord(P->ev[1], st));
  const int nb = sph_blocks(S);
  sph_residual(phi, rho, nullptr, S, P->sc, o.four_pi_G, true, P->partial, st);
  finish_sum(P->partial, nb, 1, P->scal, kBnorm2, st);
  sph_residual(phi, rho, P->sr, S, P->sc, o.four_pi_G, false, P->partial, st);
  finish_sum(P->partial, nb, 1, P->scal, kRes2, st);
  CHK(launch_check("spherical setup"));
  CHK(read_scalars(P, kBnorm2, 2));
  T.bnorm = sqrt(P->host[0]);
  double rel = rel_of(P->host[1], T.bnorm);
  T.push(rel);
  if (!isfinite(rel)) {
    set_error("non-finite initial residual (NaN/Inf in rho or phi)");
    return POISSON_ENUMERIC;
  }
  int it = 0;
  bool conv = rel <= tol;
  int restarts = 0;
  auto restart = [&]() -> int {
    // rhat = r, rho = r.r, alpha = omega = 1, beta = 0, p = v = 0
    sph_copy(P->sr, P->srh, S, st);
    sph_fill_zero(P->sp[0], S, st);
    sph_fill_zero(P->sv[0], S, st);
    double init[4] = {P->host[0], 1.0, 1.0, 0.0};
    HIPCHK(hipMemcpyAsync(P->scal->v, init, sizeof init, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return POISSON_OK;
  };
  if (o.method == POISSON_SOR) return solve_sph_sor(P, rho, phi, tol, T, rel);
  if (!conv) {
    P->host[0] = P->host[1];
    CHK(restart());
  }
  // right-preconditioned BiCGSTAB (p, v, phat, shat, s, t) with either the
  // red-black Gauss-Seidel preconditioner or one FP32 multigrid V-cycle; the
  // latter runs as one captured graph per iteration
  double* p = P->sp[0];
  double* phat = P->sp[1];
  double* v = P->sv[0];
  double* shat = P->sv[1];
  const bool mg = o.method == POISSON_BICGSTAB_MG32;
  const bool mg_graph = mg && capture_stream(P) != nullptr;
  if (mg_graph) CHK(capture_sph_iteration(P, phi));
  while (!conv && it < o.max_iter) {
    if (mg_graph) {
      HIPCHK(hipGraphLaunch(P->iter_exec, st));
    } else if (mg) {
      sph_mg_iteration(P, phi, st);
    } else {
      pbicg_direction(P->sr, p, v, phat, S, P->sc, P->scal, st);
      pbicg_apply(phat, v, P->srh, 0, S, P->sc, P->partial, st);
      bicg_scalars(P->partial, nb, P->scal, 0, st);
      pbicg_s(P->sr, v, P->ss, shat, S, P->sc, P->scal, st);
      pbicg_apply(shat, P->stt, P->ss, 1, S, P->sc, P->partial, st);
      bicg_scalars(P->partial, nb, P->scal, 1, st);
      pbicg_xr(phi, P->sr, phat, shat, P->ss, P->stt, P->srh, S, P->scal, P->partial, st);
      bicg_scalars(P->partial, nb, P->scal, 2, st);
    }
    ++it;
    if (!(it % o.check_every == 0 || it == o.max_iter)) continue;
    {
      CHK(launch_check("BiCGSTAB"));
      CHK(read_scalars(P, 0, 8));
      const double rr = P->host[7];
      rel = rel_of(rr, T.bnorm);
      T.push(rel);
      if (!isfinite(rel)) {
        set_error("BiCGSTAB breakdown (non-finite residual)");
        return POISSON_ENUMERIC;
      }
      conv = rel <= tol;
      // breakdown: rho or omega vanishing relative to the residual
      const double rho_ = P->host[0], om = P->host[2];
      if (!conv && (fabs(rho_) < 1e-30 * rr || om == 0.0)) {
        if (++restarts > 8) {
          set_error("BiCGSTAB breakdown persisted after restarts");
          return POISSON_ENUMERIC;
        }
        P->host[0] = rr;
        CHK(restart());
      }
    }
  }
  HIPCHK(hipEventRecord(P->ev[2], st));
  HIPCHK(hipEventSynchronize(P->ev[2]));
  float t_mp = 0.f, t_it = 0.f;
  HIPCHK(hipEventElapsedTime(&t_mp, P->ev[0], P->ev[1]));
  HIPCHK(hipEventElapsedTime(&t_it, P->ev[1], P->ev[2]));
  return finish_status(P, T, it, rel, conv, t_mp, t_it);
}

bool same_grid(const poisson_grid_t* a, const poisson_grid_t* b) {
  if (a->coord != b->coord || a->ghost != b->ghost) return false;
  for (int d = 0; d < 3; ++d)
    if (a->n[d] != b->n[d] || a->lo[d] != b->lo[d] || a->hi[d] != b->hi[d]) return false;
  return a->pitch[0] == b->pitch[0] && a->pitch[1] == b->pitch[1];
}

}  // namespace

int psn::cart_setup(poisson_plan_s* P, const double* rho, double* phi) { return cart_setup_impl(P, rho, phi); }

int psn::cart_step(poisson_plan_s* P, bool use_graph) {
  if (P->lv.empty()) {
    set_error("multigrid plan expected");
    return POISSON_EINVAL;
  }
  if (use_graph) return launch_step(P);
  mg_step(P, P->st);
  return launch_check("multigrid step");
}

int psn::cart_prepare_graph(poisson_plan_s* P) {
  if (P->lv.empty()) {
    set_error("multigrid plan expected");
    return POISSON_EINVAL;
  }
  return capture_stream(P) ? capture_step(P) : POISSON_OK;
}

int psn::cart_finish(poisson_plan_s* P, double* phi) {
  const poisson_grid_t& g = P->grid;
  merge_to_natural(P->phi64, phi, g.pitch[0], g.pitch[1], P->G0, true, 1.0, P->st);
  return launch_check("solve finish");
}

// ============================================================ C ABI
extern "C" {

void poisson_default_opts(poisson_opts_t* o, int32_t method) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->method = method;
  o->order = 2;
  o->lmax = 8;
  o->nu1 = (method == POISSON_MG_SPAI || method == POISSON_MG_SPAI32) ? 3 : 2;
  o->nu2 = o->nu1;
  o->coarsest = 8;
  o->omega_mode = POISSON_OMEGA_OPT;
  o->max_iter = 10000;
  o->check_every = 1;
  o->omega = 1.0;
  o->four_pi_G = 1.0;
  o->point_mass = 0.0;
}

size_t poisson_workspace_bytes(const poisson_grid_t* grid, const poisson_opts_t* opts) {
  if (validate(grid, opts) != POISSON_OK) return 0;
  poisson_plan_s P;
  P.grid = *grid;
  P.opts = *opts;
  P.sph = grid->coord == POISSON_SPHERICAL_LOG;
  P.order = opts->order;
  P.C = opts->order == 6 ? 4 : 2;
  Carver cv(nullptr);
  carve(&P, cv);
  return cv.off + 256;
}

int poisson_plan(poisson_plan_t* out, const poisson_grid_t* grid, const poisson_opts_t* opts, void* d_workspace,
                 size_t ws_bytes, void* stream) {
  if (!out) {
    set_error("null plan output");
    return POISSON_EINVAL;
  }
  CHK(validate(grid, opts));
  const size_t need = poisson_workspace_bytes(grid, opts);
  if (!d_workspace || ws_bytes < need) {
    set_error("workspace of %zu bytes given, %zu needed", ws_bytes, need);
    return POISSON_EWORKSPACE;
  }
  if (((uintptr_t)d_workspace & 255u) != 0) {
    set_error("workspace must be 256-byte aligned");
    return POISSON_EWORKSPACE;
  }
  poisson_plan_s* P = new poisson_plan_s();
  P->grid = *grid;
  P->opts = *opts;
  P->st = (hipStream_t)stream;
  P->sph = grid->coord == POISSON_SPHERICAL_LOG;
  P->order = opts->order;
  P->C = opts->order == 6 ? 4 : 2;
  Carver cv(d_workspace);
  carve(P, cv);
  int status = POISSON_OK;
  auto fail = [&](int s) {
    poisson_plan_destroy(P);
    return s;
  };
  if (hipHostMalloc((void**)&P->host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    set_error("pinned host allocation failed");
    P->host = nullptr;
    return fail(POISSON_EHIP);
  }
  for (int i = 0; i < 3; ++i)
    if (hipEventCreate(&P->ev[i]) != hipSuccess) {
      set_error("event creation failed");
      return fail(POISSON_EHIP);
    }
  hipStream_t st = P->st;
  // zero the whole workspace once: ghosts of correction and direction
  // vectors must stay zero and are never written afterwards
  fill_zero(d_workspace, false, (long long)(need / sizeof(double)), st);
  if (!P->sph) {
    // monomial tables of the Cartesian multipole moments
    std::vector<int> mono, toff, tmono;
    std::vector<double> tcoef;
    if (!build_mom_tables(mono, toff, tmono, tcoef)) {
      set_error("multipole term table exceeds its bound");
      return fail(POISSON_ENUMERIC);
    }
    if (hipMemcpyAsync(P->mom_mono, mono.data(), sizeof(int) * mono.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(P->mom_toff, toff.data(), sizeof(int) * toff.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(P->mom_tmono, tmono.data(), sizeof(int) * tmono.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(P->mom_tcoef, tcoef.data(), sizeof(double) * tcoef.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("upload of the multipole tables failed");
      return fail(POISSON_EHIP);
    }
  }
  if (P->sph) {
    const poisson_grid_t& g = *grid;
    SGeom& S = P->S;
    S.nr = g.n[0];
    S.nth = g.n[1];
    S.nph = g.n[2];
    S.p0 = g.pitch[0];
    S.p1 = g.pitch[1];
    std::vector<double> rr, rcl, rcr, rw;
    if (!sph_radial_map(g, rr, rcl, rcr, rw, S.ds)) {
      set_error("invalid radial map");
      return fail(POISSON_EGRID);
    }
    S.r_min = rr[1];
    S.dth = M_PI / S.nth;
    S.dph = 2.0 * M_PI / S.nph;
    std::vector<double> cot(S.nth), isin2(S.nth), r2(S.nr + 2);
    for (int j = 0; j < S.nth; ++j) {
      const double th = (j + 0.5) * S.dth;
      cot[j] = cos(th) / sin(th) / (2.0 * S.dth);
      isin2[j] = 1.0 / (sin(th) * sin(th));
    }
    for (int i = 0; i < S.nr + 2; ++i) r2[i] = rr[i] * rr[i];
    const size_t rb = sizeof(double) * (S.nr + 2);
    if (hipMemcpyAsync((void*)P->sc.rcl, rcl.data(), rb, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync((void*)P->sc.rcr, rcr.data(), rb, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync((void*)S.rr, rr.data(), rb, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync((void*)S.rw, rw.data(), rb, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("upload of the radial tables failed");
      return fail(POISSON_EHIP);
    }
    if (hipMemcpyAsync((void*)P->sc.cot, cot.data(), sizeof(double) * S.nth, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync((void*)P->sc.isin2, isin2.data(), sizeof(double) * S.nth, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync((void*)P->sc.r2, r2.data(), sizeof(double) * (S.nr + 2), hipMemcpyHostToDevice, st) !=
            hipSuccess) {
      set_error("upload of spherical coefficients failed");
      return fail(POISSON_EHIP);
    }
    if (P->srj) {
      // Eq. local_rjac: the weights (dr)^-2, (r dtheta)^-2, (r sin(theta)
      // dphi)^-2 times r^2 are the operator's diagonal couplings a_i =
      // (cl + cr)/2 (ds^-2 on the log grid, where r_J depends on theta only),
      // dtheta^-2 and (sin(theta) dphi)^-2; one entry per (j, radial index)
      const int ni = S.nr + 2;
      std::vector<double> rj((size_t)S.nth * ni, 0.0);
      for (int j = 0; j < S.nth; ++j) {
        const double th = (j + 0.5) * S.dth;
        const double wt = 1.0 / (S.dth * S.dth);
        const double wp = 1.0 / (sin(th) * sin(th) * S.dph * S.dph);
        for (int i = 1; i <= S.nr; ++i) {
          const double wr = 0.5 * (rcl[i] + rcr[i]);
          rj[(size_t)j * ni + i] =
              (cos(M_PI / S.nr) * wr + cos(M_PI / S.nth) * wt + cos(M_PI / S.nph) * wp) / (wr + wt + wp);
        }
      }
      if (hipMemcpyAsync(P->srj, rj.data(), sizeof(double) * rj.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        set_error("upload of the local spectral radii failed");
        return fail(POISSON_EHIP);
      }
      P->srj_host = rj;
    }
    std::vector<double> lcl, lcr;
    for (size_t l = 0; l < P->slv.size(); ++l) {
      const SLev& L = P->slv[l];
      std::vector<float> c2(L.nth), is2(L.nth), tab;
      sph_level_couplings(g, (int)l, L.nr, lcl, lcr);
      std::vector<float> fcl(lcl.begin(), lcl.end()), fcr(lcr.begin(), lcr.end());
      if (hipMemcpyAsync((void*)L.rcl, fcl.data(), sizeof(float) * L.nr, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync((void*)L.rcr, fcr.data(), sizeof(float) * L.nr, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        set_error("upload of preconditioner radial couplings failed");
        return fail(POISSON_EHIP);
      }
      if (L.ltab) {
        if (!line_tables(L, lcl, lcr, tab)) {
          set_error("phi-line interface system is singular");
          return fail(POISSON_ENUMERIC);
        }
        if (hipMemcpyAsync((void*)L.ltab, tab.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice, st) !=
            hipSuccess) {
          set_error("upload of line-smoother tables failed");
          return fail(POISSON_EHIP);
        }
      }
      const double dth = M_PI / L.nth;
      for (int j = 0; j < L.nth; ++j) {
        const double th = (j + 0.5) * dth;
        c2[j] = (float)(cos(th) / sin(th) / (2.0 * dth));
        is2[j] = (float)(1.0 / (sin(th) * sin(th)));
      }
      if (hipMemcpyAsync((void*)L.cot2, c2.data(), sizeof(float) * L.nth, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync((void*)L.isin2, is2.data(), sizeof(float) * L.nth, hipMemcpyHostToDevice, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        set_error("upload of preconditioner coefficients failed");
        return fail(POISSON_EHIP);
      }
    }
    if (!P->slv.empty()) {
      const SLev& C = P->slv.back();
      std::vector<double> A, inv;
      sph_level_couplings(g, (int)P->slv.size() - 1, C.nr, lcl, lcr);
      sph_level_matrix(C.nr, C.nth, C.nph, lcl, lcr, A);
      if (!invert_general(P->sncoarse, A, inv)) {
        set_error("coarsest preconditioner level is singular");
        return fail(POISSON_ENUMERIC);
      }
      if (hipMemcpyAsync(P->scinv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        set_error("upload of the coarsest inverse failed");
        return fail(POISSON_EHIP);
      }
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
      set_error("stream synchronisation failed");
      return fail(POISSON_EHIP);
    }
  } else if (!P->nlv.empty()) {
    const double* sp = kSpai[P->order / 2 - 1];
    for (size_t l = 0; l < P->nlv.size(); ++l) {
      NLevel& L = P->nlv[l];
      const double h2 = L.G.h * L.G.h;
      if (l == 0) {
        // compact Laplacians: 7-point, 19-point Mehrstellen (-24, 2, 1, 0)/6,
        // 27-point sixth order (-128, 14, 3, 1)/30
        if (P->order == 6)
          L.A = W4{-128.0 / (30.0 * h2), 14.0 / (30.0 * h2), 3.0 / (30.0 * h2), 1.0 / (30.0 * h2)};
        else if (P->order == 4)
          L.A = W4{-4.0 / h2, 1.0 / (3.0 * h2), 1.0 / (6.0 * h2), 0.0};
        else
          L.A = W4{-6.0 / h2, 1.0 / h2, 0.0, 0.0};
      } else {
        L.A = galerkin_w4(P->nlv[l - 1].A);
      }
      const double s = sp[0] * h2;
      L.M = W4{s * sp[1], s * sp[2], s * sp[3], s * sp[4]};
    }
    const NLevel& Lc = P->nlv.back();
    std::vector<double> A, inv;
    w4_matrix(Lc.A, Lc.G.n, A);
    if (!invert_general(P->ncoarse, A, inv)) {
      set_error("coarsest Galerkin operator is singular");
      return fail(POISSON_ENUMERIC);
    }
    if (hipMemcpyAsync(P->cinv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("upload of the coarsest inverse failed");
      return fail(POISSON_EHIP);
    }
  } else if (!P->lv.empty()) {
    const Level& Lc = P->lv.back();
    std::vector<double> inv;
    if (!coarse_inverse(Lc.G.n, Lc.G.h, P->order, inv)) {
      set_error("coarsest-level factorisation failed");
      return fail(POISSON_ENUMERIC);
    }
    if (hipMemcpyAsync(P->cinv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("upload of the coarsest inverse failed");
      return fail(POISSON_EHIP);
    }
  }
  status = launch_check("poisson_plan");
  if (status == POISSON_OK && hipStreamSynchronize(st) != hipSuccess) {
    set_error("stream synchronisation failed");
    status = POISSON_EHIP;
  }
  if (status != POISSON_OK) return fail(status);
  *out = P;
  return POISSON_OK;
}

void poisson_plan_destroy(poisson_plan_t P) {
  if (!P) return;
  if (P->step_exec) hipGraphExecDestroy(P->step_exec);
  if (P->head_exec) hipGraphExecDestroy(P->head_exec);
  if (P->cont_exec) hipGraphExecDestroy(P->cont_exec);
  if (P->iter_exec) hipGraphExecDestroy(P->iter_exec);
  for (int i = 0; i < 3; ++i)
    if (P->ev[i]) hipEventDestroy(P->ev[i]);
  if (P->host) hipHostFree(P->host);
  delete P;
}

int poisson_plan_set_capture_stream(poisson_plan_t P, void* stream) {
  if (!P || !stream) {
    set_error("a plan and a non-NULL capture stream are needed");
    return POISSON_EINVAL;
  }
  // graphs recorded before stay valid: a graph does not depend on the stream
  // it was recorded on
  P->cap = (hipStream_t)stream;
  return POISSON_OK;
}

int multipole_boundary(poisson_plan_t P, const double* d_rho, double* d_phi, int32_t lmax, double* h_q) {
  if (!P || !d_rho || !d_phi) {
    set_error("null argument");
    return POISSON_EINVAL;
  }
  if (lmax < 0 || lmax > kLmaxMax) {
    set_error("lmax must be in 0..%d", kLmaxMax);
    return POISSON_EINVAL;
  }
  return do_multipole(P, d_rho, d_phi, lmax, h_q);
}

int poisson_solve(poisson_plan_t P, const double* d_rho, double* d_phi, const poisson_grid_t* grid, double tol,
                  poisson_stats_t* stats) {
  if (!P || !d_rho || !d_phi || !grid) {
    set_error("null argument");
    return POISSON_EINVAL;
  }
  if (!(tol > 0.0)) {
    set_error("tol must be positive");
    return POISSON_EINVAL;
  }
  if (!same_grid(grid, &P->grid)) {
    set_error("grid differs from the plan's grid");
    return POISSON_EGRID;
  }
  int s = P->sph                               ? solve_sph(P, d_rho, d_phi, tol, stats)
          : !P->nlv.empty()                   ? solve_spai(P, d_rho, d_phi, tol, stats)
                                               : solve_cart(P, d_rho, d_phi, tol, stats);
  if (stats && s < 0) stats->status = s;
  return s;
}

const char* poisson_strerror(int s) {
  switch (s) {
    case POISSON_OK: return "converged";
    case POISSON_WARN_MAXITER: return "tolerance not reached within max_iter";
    case POISSON_EINVAL: return "invalid argument";
    case POISSON_EGRID: return "grid unsuited to the method";
    case POISSON_EWORKSPACE: return "workspace missing, too small or misaligned";
    case POISSON_EHIP: return "HIP runtime error";
    case POISSON_ENUMERIC: return "non-finite residual or breakdown";
    case POISSON_EADMIT: return "request exceeds the memory budget";
    case POISSON_ETIMEOUT: return "timed out waiting for a request";
    default: return "unknown status";
  }
}

const char* poisson_last_error(void) { return g_err; }

// ------------------------------------------------------------ single operators
static int need_cart(poisson_plan_t P) {
  if (!P) {
    set_error("null plan");
    return POISSON_EINVAL;
  }
  if (P->sph) {
    set_error("operation defined on Cartesian plans only");
    return POISSON_EINVAL;
  }
  return POISSON_OK;
}

int poisson_op_apply(poisson_plan_t P, const double* d_phi, double* d_out) {
  if (!P || !d_phi || !d_out) {
    set_error("null argument");
    return POISSON_EINVAL;
  }
  hipStream_t st = P->st;
  if (P->sph) {
    sph_apply(d_phi, d_out, P->S, P->sc, st);
    return launch_check("poisson_op_apply");
  }
  if (!P->nlv.empty()) {
    set_error("poisson_op_apply is not defined for SPAI plans (use poisson_op_residual)");
    return POISSON_EINVAL;
  }
  const poisson_grid_t& g = P->grid;
  split_from_natural(d_phi, g.pitch[0], g.pitch[1], P->phi64, false, P->G0, 1.0, st);
  fill_zero(P->f64, false, P->G0.total(), st);
  residual(P->phi64, P->f64, false, P->t64, false, P->G0, P->order, false, nullptr, st);
  merge_to_natural(P->t64, d_out, g.pitch[0], g.pitch[1], P->G0, true, -1.0, st);
  return launch_check("poisson_op_apply");
}

int poisson_op_residual(poisson_plan_t P, const double* d_rho, const double* d_phi, double* d_res,
                        double* h_norm2) {
  if (!P || !d_rho || !d_phi || !d_res) {
    set_error("null argument");
    return POISSON_EINVAL;
  }
  hipStream_t st = P->st;
  if (P->sph) {
    sph_residual(d_phi, d_rho, d_res, P->S, P->sc, P->opts.four_pi_G, false, P->partial, st);
    finish_sum(P->partial, sph_blocks(P->S), 1, P->scal, kRes2, st);
  } else if (!P->nlv.empty()) {
    const poisson_grid_t& g = P->grid;
    NLevel& L = P->nlv[0];
    n_rhs(d_rho, g.pitch[0], g.pitch[1], g.ghost, (double*)L.f, L.G, P->order, P->opts.four_pi_G, st);
    n_from_caller(d_phi, g.pitch[0], g.pitch[1], g.ghost, (double*)L.u, L.G, false, st);
    n27_residual(L.u, L.f, L.r, false, L.G, L.A, true, P->partial, st);
    finish_sum(P->partial, (int)n27_blocks(L.G), 1, P->scal, kRes2, st);
    n_to_caller((const double*)L.r, L.G, d_res, g.pitch[0], g.pitch[1], g.ghost, st);
  } else {
    const poisson_grid_t& g = P->grid;
    split_from_natural(d_phi, g.pitch[0], g.pitch[1], P->phi64, false, P->G0, 1.0, st);
    split_from_natural(d_rho, g.pitch[0], g.pitch[1], P->f64, false, P->G0, P->opts.four_pi_G, st);
    residual(P->phi64, P->f64, false, P->t64, false, P->G0, P->order, false, P->partial, st);
    finish_sum(P->partial, residual_blocks(P->G0), 1, P->scal, kRes2, st);
    merge_to_natural(P->t64, d_res, g.pitch[0], g.pitch[1], P->G0, true, 1.0, st);
  }
  CHK(launch_check("poisson_op_residual"));
  if (h_norm2) {
    CHK(read_scalars(P, kRes2, 1));
    *h_norm2 = P->host[0];
  }
  return POISSON_OK;
}

int poisson_op_smooth(poisson_plan_t P, const double* d_rho, double* d_phi, int32_t sweeps, int32_t forward,
                      double omega) {
  if (P && P->sph && P->opts.method == POISSON_SOR) {
    // spherical SOR plans: `sweeps` sweeps with the plan's relaxation factors
    // from the start of their sequence (forward and omega do not apply)
    if (!d_rho || !d_phi || sweeps < 0) {
      set_error("bad argument");
      return POISSON_EINVAL;
    }
    CHK(sph_sor_init(P));
    for (int s = 0; s < sweeps; ++s) sph_sor_sweep(P, d_rho, d_phi, P->st);
    return launch_check("poisson_op_smooth");
  }
  CHK(need_cart(P));
  if (!d_rho || !d_phi || sweeps < 0) {
    set_error("bad argument");
    return POISSON_EINVAL;
  }
  if (P->order == 6 && P->nlv.empty() && omega != 1.0) {
    set_error("the four-colour sweep is plain Gauss-Seidel (omega = 1)");
    return POISSON_EINVAL;
  }
  hipStream_t st = P->st;
  const poisson_grid_t& g = P->grid;
  if (!P->nlv.empty()) {
    // SPAI plans: `sweeps` Richardson steps with the plan's smoother
    // (the sweep direction and omega do not apply)
    NLevel& L = P->nlv[0];
    n_rhs(d_rho, g.pitch[0], g.pitch[1], g.ghost, (double*)L.f, L.G, P->order, P->opts.four_pi_G, st);
    n_from_caller(d_phi, g.pitch[0], g.pitch[1], g.ghost, (double*)L.u, L.G, false, st);
    if (L.u2) n_from_caller(d_phi, g.pitch[0], g.pitch[1], g.ghost, (double*)L.u2, L.G, false, st);
    const void* cur = spai_smooth(L, L.u, sweeps, st);
    n_to_caller((const double*)cur, L.G, d_phi, g.pitch[0], g.pitch[1], g.ghost, st);
    return launch_check("poisson_op_smooth");
  }
  split_from_natural(d_phi, g.pitch[0], g.pitch[1], P->phi64, false, P->G0, 1.0, st);
  split_from_natural(d_rho, g.pitch[0], g.pitch[1], P->f64, false, P->G0, P->opts.four_pi_G, st);
  for (int s = 0; s < sweeps; ++s)
    for (int i = 0; i < P->C; ++i) {
      const int c = forward ? i : P->C - 1 - i;
      colour_pass(P->phi64, P->f64, false, P->G0, P->order, c, omega, st);
    }
  merge_to_natural(P->phi64, d_phi, g.pitch[0], g.pitch[1], P->G0, true, 1.0, st);
  return launch_check("poisson_op_smooth");
}

int poisson_op_restrict(poisson_plan_t P, const double* d_fine, double* d_coarse) {
  CHK(need_cart(P));
  if (P->lv.size() < 2 || P->mg32) {
    set_error("restriction needs an FP64 multigrid plan with at least two levels");
    return POISSON_EINVAL;
  }
  hipStream_t st = P->st;
  Level& L1 = P->lv[1];
  dense_to_split(d_fine, P->t64, false, P->G0, st);
  restrict_fw(P->t64, P->G0, L1.f, L1.G, false, st);
  split_to_dense(L1.f, false, d_coarse, L1.G, st);
  return launch_check("poisson_op_restrict");
}

int poisson_op_restrict_residual(poisson_plan_t P, const double* d_rho, const double* d_phi, double* d_coarse,
                                 double* h_norm2) {
  CHK(need_cart(P));
  if (!d_rho || !d_phi || !d_coarse) {
    set_error("null argument");
    return POISSON_EINVAL;
  }
  if (P->lv.size() < 2) {
    set_error("the restricted residual needs a multigrid plan (MG or MG_IR32) with at least two levels");
    return POISSON_EINVAL;
  }
  hipStream_t st = P->st;
  const poisson_grid_t& g = P->grid;
  // MG_IR32 plans: the FP32 cycle's finest arrays and kernels
  const bool f32 = P->mg32;
  Level& L0 = P->lv[0];
  Level& L1 = P->lv[1];
  void* x = f32 ? L0.phi : (void*)P->phi64;
  void* f = f32 ? L0.f : (void*)P->f64;
  void* r = f32 ? L0.tmp : (void*)P->t64;
  split_from_natural(d_phi, g.pitch[0], g.pitch[1], x, f32, P->G0, 1.0, st);
  split_from_natural(d_rho, g.pitch[0], g.pitch[1], f, f32, P->G0, P->opts.four_pi_G, st);
  int nb = residual_blocks(P->G0);
  if (resrestrict19_ok(P->G0)) {
    nb = resrestrict19(x, f, f32, P->G0, L1.f, L1.G, P->partial, false, st);
  } else {
    residual(x, f, f32, r, f32, P->G0, P->order, false, P->partial, st);
    restrict_fw(r, P->G0, L1.f, L1.G, f32, st);
  }
  finish_sum(P->partial, nb, 1, P->scal, kRes2, st);
  split_to_dense(L1.f, f32, d_coarse, L1.G, st);
  CHK(launch_check("poisson_op_restrict_residual"));
  if (h_norm2) {
    CHK(read_scalars(P, kRes2, 1));
    *h_norm2 = P->host[0];
  }
  return POISSON_OK;
}

int poisson_op_prolong_add(poisson_plan_t P, const double* d_coarse, double* d_fine) {
  CHK(need_cart(P));
  if (P->lv.size() < 2 || P->mg32) {
    set_error("prolongation needs an FP64 multigrid plan with at least two levels");
    return POISSON_EINVAL;
  }
  hipStream_t st = P->st;
  Level& L1 = P->lv[1];
  dense_to_split(d_coarse, L1.phi, false, L1.G, st);
  dense_to_split(d_fine, P->t64, false, P->G0, st);
  prolong_add(L1.phi, L1.G, P->t64, P->G0, false, st);
  split_to_dense(P->t64, false, d_fine, P->G0, st);
  return launch_check("poisson_op_prolong_add");
}

int poisson_op_vcycle(poisson_plan_t P, const double* d_rho, double* d_phi, int32_t cycles) {
  CHK(need_cart(P));
  if ((P->lv.empty() && P->nlv.empty()) || !d_rho || !d_phi || cycles < 0) {
    set_error("V-cycles need a multigrid plan");
    return POISSON_EINVAL;
  }
  hipStream_t st = P->st;
  const poisson_grid_t& g = P->grid;
  if (!P->nlv.empty()) {
    NLevel& L = P->nlv[0];
    n_rhs(d_rho, g.pitch[0], g.pitch[1], g.ghost, (double*)L.f, L.G, P->order, P->opts.four_pi_G, st);
    n_from_caller(d_phi, g.pitch[0], g.pitch[1], g.ghost, (double*)L.u, L.G, false, st);
    if (L.u2) n_from_caller(d_phi, g.pitch[0], g.pitch[1], g.ghost, (double*)L.u2, L.G, false, st);
    for (int c = 0; c < cycles; ++c) spai_step(P, st);
    n_to_caller((const double*)L.u, L.G, d_phi, g.pitch[0], g.pitch[1], g.ghost, st);
    return launch_check("poisson_op_vcycle");
  }
  split_from_natural(d_phi, g.pitch[0], g.pitch[1], P->phi64, false, P->G0, 1.0, st);
  split_from_natural(d_rho, g.pitch[0], g.pitch[1], P->f64, false, P->G0, P->opts.four_pi_G, st);
  if (P->mg32) residual(P->phi64, P->f64, false, P->lv[0].f, true, P->G0, P->order, false, nullptr, st);
  for (int c = 0; c < cycles; ++c) mg_step(P, st);
  merge_to_natural(P->phi64, d_phi, g.pitch[0], g.pitch[1], P->G0, true, 1.0, st);
  return launch_check("poisson_op_vcycle");
}

int poisson_op_precond(poisson_plan_t P, const double* d_y, double* d_yhat) {
  if (!P || !d_y || !d_yhat) {
    set_error("null argument");
    return POISSON_EINVAL;
  }
  if (!P->sph || P->slv.empty()) {
    set_error("poisson_op_precond needs a POISSON_BICGSTAB_MG32 plan");
    return POISSON_EINVAL;
  }
  sph_precond(P, d_y, d_yhat, P->st);
  return launch_check("poisson_op_precond");
}

int poisson_op_sweep_resident(poisson_plan_t P, int32_t sweeps) {
  CHK(need_cart(P));
  if (sweeps < 0) {
    set_error("sweeps must be >= 0");
    return POISSON_EINVAL;
  }
  if (!P->nlv.empty()) {
    // an even number of out-of-place steps leaves the result where it started
    NLevel& L = P->nlv[0];
    if (L.u2) spai_smooth(L, L.u, 2 * sweeps, P->st);
    return launch_check("poisson_op_sweep_resident");
  }
  void* phi = P->phi64;
  const void* f = P->f64;
  bool f32 = false;
  if (!P->lv.empty()) {
    phi = P->lv[0].phi;
    f = P->lv[0].f;
    f32 = P->mg32;
  }
  for (int s = 0; s < sweeps; ++s)
    for (int c = 0; c < P->C; ++c) colour_pass(phi, f, f32, P->G0, P->order, c, 1.0, P->st);
  return launch_check("poisson_op_sweep_resident");
}

}  // extern "C"
