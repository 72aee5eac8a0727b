// Multipole boundary of a Cartesian grid without any device allocation: the
// same moment and ghost kernels as multipole_boundary (Section 2.2, Eqs.
// outer_multipole and outer_expansion), with their scratch (monomial tables,
// moments, partial sums) in a fixed device array of this file instead of a
// plan workspace.  For callers that cannot allocate device memory.
#include <math.h>
#include <mutex>
#include <vector>

#include "plan_impl.h"

// Device-resident scratch, one copy per GPU for the life of the process.  In
// host code this name is not a device address: kernels receive the address
// that hipGetSymbolAddress returns for the current device (dev_scratch).
static __device__ __align__(256) unsigned char scratch[POISSON_NOALLOC_SCRATCH_BYTES];

namespace psn {
namespace {

constexpr size_t kStaticBytes = POISSON_NOALLOC_SCRATCH_BYTES;
constexpr size_t kAlignS = 256;
constexpr int kMaxDevices = 64;

size_t up(size_t b) { return (b + kAlignS - 1) & ~(kAlignS - 1); }

// Layout inside the array: the four monomial tables, the moments q_lm, then
// the separable moment sums.
constexpr size_t kOffMono = 0;
constexpr size_t kOffToff = kOffMono + ((sizeof(int) * kMonoMax + kAlignS - 1) & ~(kAlignS - 1));
constexpr size_t kOffTmono = kOffToff + ((sizeof(int) * (kNqMax + 1) + kAlignS - 1) & ~(kAlignS - 1));
constexpr size_t kOffTcoef = kOffTmono + ((sizeof(int) * kTermMax + kAlignS - 1) & ~(kAlignS - 1));
constexpr size_t kOffQ = kOffTcoef + ((sizeof(double) * kTermMax + kAlignS - 1) & ~(kAlignS - 1));
constexpr size_t kOffSums = kOffQ + ((sizeof(double) * kNqMax + kAlignS - 1) & ~(kAlignS - 1));

// Host copies of the tables, filled once when the library is loaded.
struct HostTables {
  int mono[kMonoMax];
  int toff[kNqMax + 1];
  int tmono[kTermMax];
  double tcoef[kTermMax];
  int nterms = 0;
  bool ok = false;
  HostTables() {
    std::vector<int> m, t, tm;
    std::vector<double> tc;
    ok = build_mom_tables(m, t, tm, tc) && (int)m.size() == kMonoMax && (int)t.size() == kNqMax + 1;
    if (!ok) return;
    for (int i = 0; i < kMonoMax; ++i) mono[i] = m[i];
    for (int i = 0; i <= kNqMax; ++i) toff[i] = t[i];
    nterms = (int)tm.size();
    for (int i = 0; i < nterms; ++i) {
      tmono[i] = tm[i];
      tcoef[i] = tc[i];
    }
  }
};
const HostTables g_tables;

std::mutex g_mu;
unsigned char* g_dev[kMaxDevices];  // address of `scratch` on each device, nullptr until set up

// Once per device, with that device current: look up the array's device
// address and upload the tables into it.
int dev_scratch(unsigned char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error("no current HIP device (or device index >= %d)", kMaxDevices);
    return POISSON_EHIP;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_dev[dev]) {
    *out = g_dev[dev];
    return POISSON_OK;
  }
  if (!g_tables.ok) {
    set_error("multipole term table exceeds its bound");
    return POISSON_ENUMERIC;
  }
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    set_error("hipGetSymbolAddress of the static scratch array failed");
    return POISSON_EHIP;
  }
  unsigned char* base = (unsigned char*)p;
  if (hipMemcpy(base + kOffMono, g_tables.mono, sizeof(int) * kMonoMax, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + kOffToff, g_tables.toff, sizeof(int) * (kNqMax + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + kOffTmono, g_tables.tmono, sizeof(int) * g_tables.nterms, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(base + kOffTcoef, g_tables.tcoef, sizeof(double) * g_tables.nterms, hipMemcpyHostToDevice) !=
          hipSuccess) {
    set_error("upload of the multipole tables into the static scratch failed");
    return POISSON_EHIP;
  }
  g_dev[dev] = base;
  *out = base;
  return POISSON_OK;
}

}  // namespace
}  // namespace psn

using namespace psn;

int multipole_boundary_noalloc(const poisson_grid_t* g, const double* d_rho, double* d_phi, int32_t lmax,
                               double four_pi_G, double point_mass, double* h_q, void* stream) {
  if (!g || !d_rho || !d_phi) {
    set_error("null argument");
    return POISSON_EINVAL;
  }
  if (g->coord != POISSON_CARTESIAN) {
    set_error("the allocation-free multipole boundary takes Cartesian grids only");
    return POISSON_EINVAL;
  }
  if (lmax < 0 || lmax > kLmaxMax) {
    set_error("lmax must be in 0..%d", kLmaxMax);
    return POISSON_EINVAL;
  }
  if (!(four_pi_G > 0.0)) {
    set_error("four_pi_G must be positive");
    return POISSON_EINVAL;
  }
  const int n = g->n[0];
  if (n < 2 || g->n[1] != n || g->n[2] != n) {
    set_error("Cartesian grids need the same interval count (>= 2) on every axis");
    return POISSON_EGRID;
  }
  if (g->ghost < 1 || g->ghost > 3) {
    set_error("ghost must be 1, 2 or 3");
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
  const int M = n + 1 + 2 * (g->ghost - 1);
  if (g->pitch[0] < M || g->pitch[1] < (int64_t)M * g->pitch[0]) {
    set_error("pitch too small: need pitch[0] >= %d and pitch[1] >= %d*pitch[0]", M, M);
    return POISSON_EINVAL;
  }
  const size_t need = kOffSums + up(cart_moment_scratch(n));
  if (need > kStaticBytes) {
    set_error("n = %d needs %zu bytes of scratch; the static array holds %zu (n <= 512)", n, need,
              kStaticBytes);
    return POISSON_EINVAL;
  }
  unsigned char* base = nullptr;
  const int s = dev_scratch(&base);
  if (s != POISSON_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const MomTables tab{(const int*)(base + kOffMono), (const int*)(base + kOffToff),
                      (const int*)(base + kOffTmono), (const double*)(base + kOffTcoef)};
  double* q = (double*)(base + kOffQ);
  const double cx = 0.5 * (g->lo[0] + g->hi[0]), cy = 0.5 * (g->lo[1] + g->hi[1]), cz = 0.5 * (g->lo[2] + g->hi[2]);
  cart_moments(d_rho, g->pitch[0], g->pitch[1], n, g->ghost, h, cx, cy, cz, lmax, tab, point_mass,
               (double*)(base + kOffSums), q, st);
  cart_ghosts(d_phi, g->pitch[0], g->pitch[1], n, g->ghost, h, g->lo[0], cx, cy, cz, lmax, q,
              four_pi_G / (4.0 * M_PI), st);
  const int lc = launch_check("multipole_boundary_noalloc");
  if (lc != POISSON_OK) return lc;
  if (h_q) {
    const int nq = (lmax + 1) * (lmax + 1);
    if (hipMemcpyAsync(h_q, q, sizeof(double) * nq, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("copy of the moments to the host failed");
      return POISSON_EHIP;
    }
  }
  return POISSON_OK;
}
