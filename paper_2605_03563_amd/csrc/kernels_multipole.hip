// Multipole open boundary (Section 2.2) for gfx950, all in FP64.
//
// Regular solid harmonics R_lm(x) = sqrt(4 pi/(2l+1)) r^l Y_lm(x/r) with
// orthonormal real Y_lm (cosine m >= 0, sine m < 0, no Condon-Shortley
// phase) are generated in Cartesian form from the complex quantities
// Q_lm = sqrt((l-m)!/(l+m)!) r^l P_l^m(cos theta) e^{i m phi}:
//   Q_00 = 1,  Q_mm = Q_{m-1,m-1} (x + i y) sqrt((2m-1)/(2m)),
//   Q_lm = [(2l-1) z Q_{l-1,m} - r^2 sqrt((l+m-1)(l-m-1)) Q_{l-2,m}]
//          / sqrt((l+m)(l-m)),
// R_l0 = Q_l0, R_lm = sqrt2 Re Q_lm, R_l,-m = sqrt2 Im Q_lm (m > 0).
// The irregular harmonics of the expansion, I_lm(x) = R_lm(x) / r^(2l+1),
// are evaluated as R_lm(x / r^2) / r.  The moment sums are the per-node
// quadrature of Eqs. outer_multipole / inner_multipole; each thread keeps all
// (lmax+1)^2 accumulators in registers over a grid-stride loop, then a
// fixed-order block and grid reduction makes the result deterministic.
#include "internal.h"
#include "reduce.h"

namespace psn {

namespace {

constexpr int kMomThreads = 256;

template <int LMAX>
__device__ inline void regular_solid(double x, double y, double z, double w, double* __restrict__ acc) {
  const double r2 = x * x + y * y + z * z;
  double qr = 1.0, qi = 0.0;
#pragma unroll
  for (int m = 0; m <= LMAX; ++m) {
    if (m > 0) {
      const double f = sqrt((2.0 * m - 1.0) / (2.0 * m));
      const double nr = (qr * x - qi * y) * f;
      const double ni = (qr * y + qi * x) * f;
      qr = nr;
      qi = ni;
    }
    double pr = qr, pi = qi, ppr = 0.0, ppi = 0.0;
#pragma unroll
    for (int l = m; l <= LMAX; ++l) {
      if (l > m) {
        const double ca = (2.0 * l - 1.0) / sqrt((double)(l + m) * (double)(l - m));
        const double cb = sqrt((double)(l + m - 1) * (double)(l - m - 1)) / sqrt((double)(l + m) * (double)(l - m));
        const double cr = ca * z * pr - cb * r2 * ppr;
        const double ci = ca * z * pi - cb * r2 * ppi;
        ppr = pr;
        ppi = pi;
        pr = cr;
        pi = ci;
      }
      if (m == 0) {
        acc[l * l + l] += w * pr;
      } else {
        const double s2 = 1.4142135623730951 * w;
        acc[l * l + l + m] += s2 * pr;
        acc[l * l + l - m] += s2 * pi;
      }
    }
  }
}

// sum_lm q_lm R_lm(x)
template <int LMAX>
__device__ inline double dot_regular(double x, double y, double z, const double* __restrict__ q) {
  const double r2 = x * x + y * y + z * z;
  double qr = 1.0, qi = 0.0, out = 0.0;
#pragma unroll
  for (int m = 0; m <= LMAX; ++m) {
    if (m > 0) {
      const double f = sqrt((2.0 * m - 1.0) / (2.0 * m));
      const double nr = (qr * x - qi * y) * f;
      const double ni = (qr * y + qi * x) * f;
      qr = nr;
      qi = ni;
    }
    double pr = qr, pi = qi, ppr = 0.0, ppi = 0.0;
#pragma unroll
    for (int l = m; l <= LMAX; ++l) {
      if (l > m) {
        const double ca = (2.0 * l - 1.0) / sqrt((double)(l + m) * (double)(l - m));
        const double cb = sqrt((double)(l + m - 1) * (double)(l - m - 1)) / sqrt((double)(l + m) * (double)(l - m));
        const double cr = ca * z * pr - cb * r2 * ppr;
        const double ci = ca * z * pi - cb * r2 * ppi;
        ppr = pr;
        ppi = pi;
        pr = cr;
        pi = ci;
      }
      if (m == 0) {
        out += q[l * l + l] * pr;
      } else {
        out += 1.4142135623730951 * (q[l * l + l + m] * pr + q[l * l + l - m] * pi);
      }
    }
  }
  return out;
}

// sum_lm q_lm I_lm(x),  I_lm(x) = R_lm(x/r^2)/r
template <int LMAX>
__device__ inline double dot_irregular(double x, double y, double z, const double* __restrict__ q) {
  const double r2 = x * x + y * y + z * z;
  const double ir2 = 1.0 / r2;
  return dot_regular<LMAX>(x * ir2, y * ir2, z * ir2, q) * sqrt(ir2);
}

template <int LMAX>
__device__ inline void store_partials(double* acc, double* __restrict__ partial) {
  constexpr int NQ = (LMAX + 1) * (LMAX + 1);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double s = block_sum(acc[q]);
    if (threadIdx.x == 0) partial[(long long)q * kMomBlocks + blockIdx.x] = s;
  }
}

template <int LMAX>
__global__ __launch_bounds__(kMomThreads) void k_cart_moments(const double* __restrict__ rho, long long p0,
                                                              long long p1, int n, int g, double h, double cx,
                                                              double cy, double cz, double lo,
                                                              double* __restrict__ partial) {
  constexpr int NQ = (LMAX + 1) * (LMAX + 1);
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  const int E = n - 1;
  const long long total = (long long)E * E * E;
  const double w = h * h * h;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t % E);
    const int j = (int)((t / E) % E);
    const int k = (int)(t / ((long long)E * E));
    const double v = rho[(long long)(k + g) * p1 + (long long)(j + g) * p0 + (i + g)];
    if (v == 0.0) continue;
    const double x = lo + (i + 1) * h - cx;
    const double y = lo + (j + 1) * h - cy;
    const double z = lo + (k + 1) * h - cz;
    regular_solid<LMAX>(x, y, z, w * v, acc);
  }
  store_partials<LMAX>(acc, partial);
}

template <int LMAX, bool INNER>
__global__ __launch_bounds__(kMomThreads) void k_sph_moments(const double* __restrict__ rho, SGeom S,
                                                             double* __restrict__ partial) {
  constexpr int NQ = (LMAX + 1) * (LMAX + 1);
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  const long long total = (long long)S.nr * S.nth * S.nph;
  const double wang = S.ds * S.dth * S.dph;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t % S.nr);
    const int j = (int)((t / S.nr) % S.nth);
    const int k = (int)(t / ((long long)S.nr * S.nth));
    const double v = rho[S.at(i + 1, j, k)];
    if (v == 0.0) continue;
    const double r = S.r_min * exp(i * S.ds);
    const double th = (j + 0.5) * S.dth;
    const double ph = k * S.dph;
    const double st = sin(th);
    const double w = r * r * r * st * wang * v;
    const double x = r * st * cos(ph), y = r * st * sin(ph), z = r * cos(th);
    if (INNER) {
      const double ir2 = 1.0 / (r * r);
      regular_solid<LMAX>(x * ir2, y * ir2, z * ir2, w / r, acc);
    } else {
      regular_solid<LMAX>(x, y, z, w, acc);
    }
  }
  store_partials<LMAX>(acc, partial);
}

// one block per moment: fixed-order sum of its kMomBlocks partials
__global__ __launch_bounds__(256) void k_finish_moments(const double* __restrict__ partial, double point_mass,
                                                        double* __restrict__ q) {
  const int c = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < kMomBlocks; b += blockDim.x) s += partial[(long long)c * kMomBlocks + b];
  s = block_sum(s);
  if (threadIdx.x == 0) q[c] = s + (c == 0 ? point_mass : 0.0);
}

// Every ghost node of the Cartesian node array: z ghost planes, then y ghost
// rows of the interior planes, then x ghost ends of the interior rows.
template <int LMAX>
__global__ __launch_bounds__(256) void k_cart_ghosts(double* __restrict__ phi, long long p0, long long p1, int n,
                                                     int g, double h, double lo, double cx, double cy, double cz,
                                                     const double* __restrict__ q, double G) {
  const int E = n - 1;
  const int M = E + 2 * g;
  const long long nA = 2LL * g * M * M;
  const long long nB = (long long)E * 2 * g * M;
  const long long nC = (long long)E * E * 2 * g;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= nA + nB + nC) return;
  int a, b, k;
  if (t < nA) {
    const int p = (int)(t / ((long long)M * M));
    const int rem = (int)(t % ((long long)M * M));
    k = p < g ? p : g + E + (p - g);
    b = rem / M;
    a = rem % M;
  } else if (t < nA + nB) {
    const long long u = t - nA;
    k = g + (int)(u / (2LL * g * M));
    const int rem = (int)(u % (2LL * g * M));
    const int qq = rem / M;
    b = qq < g ? qq : g + E + (qq - g);
    a = rem % M;
  } else {
    const long long u = t - nA - nB;
    k = g + (int)(u / ((long long)E * 2 * g));
    const int rem = (int)(u % ((long long)E * 2 * g));
    b = g + rem / (2 * g);
    const int qq = rem % (2 * g);
    a = qq < g ? qq : g + E + (qq - g);
  }
  const int sh = g - 1;
  const double x = lo + (a - sh) * h - cx;
  const double y = lo + (b - sh) * h - cy;
  const double z = lo + (k - sh) * h - cz;
  phi[(long long)k * p1 + (long long)b * p0 + a] = -G * dot_irregular<LMAX>(x, y, z, q);
}

template <int LMAX>
__global__ __launch_bounds__(256) void k_sph_ghosts(double* __restrict__ phi, SGeom S, const double* __restrict__ q,
                                                    const double* __restrict__ qbar, double point_mass, double G) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = S.nth * S.nph;
  if (t >= 2 * per) return;
  const bool outer = t >= per;
  const int u = outer ? t - per : t;
  const int j = u % S.nth, k = u / S.nth;
  const int i = outer ? S.nr + 1 : 0;
  const double r = S.r_min * exp((i - 1) * S.ds);
  const double th = (j + 0.5) * S.dth, ph = k * S.dph;
  const double st = sin(th);
  const double x = r * st * cos(ph), y = r * st * sin(ph), z = r * cos(th);
  double v;
  if (outer)
    v = -G * dot_irregular<LMAX>(x, y, z, q);
  else
    v = -G * dot_regular<LMAX>(x, y, z, qbar) - G * point_mass / r;
  phi[S.at(i, j, k)] = v;
}

}  // namespace

#define PSN_LMAX_SWITCH(L, CALL) \
  switch (L) {                   \
    case 0: CALL(0); break;      \
    case 1: CALL(1); break;      \
    case 2: CALL(2); break;      \
    case 3: CALL(3); break;      \
    case 4: CALL(4); break;      \
    case 5: CALL(5); break;      \
    case 6: CALL(6); break;      \
    case 7: CALL(7); break;      \
    default: CALL(8); break;     \
  }

void cart_moments(const double* rho, long long p0, long long p1, int n, int g, double h, double cx, double cy,
                  double cz, int lmax, double* partial, hipStream_t st) {
  // lo is recovered from the centre: node array index a has position
  // lo + (a - (g-1)) h; the kernel uses unknown index i (node i+1) directly.
  const double lo = cx - 0.5 * n * h;
#define PSN_CALL(L) \
  k_cart_moments<L><<<kMomBlocks, kMomThreads, 0, st>>>(rho, p0, p1, n, g, h, cx, cy, cz, lo, partial)
  PSN_LMAX_SWITCH(lmax, PSN_CALL)
#undef PSN_CALL
}

void sph_moments(const double* rho, const SGeom& S, int lmax, bool inner, double* partial, hipStream_t st) {
#define PSN_CALL(L)                                                                      \
  if (inner)                                                                             \
    k_sph_moments<L, true><<<kMomBlocks, kMomThreads, 0, st>>>(rho, S, partial);         \
  else                                                                                   \
    k_sph_moments<L, false><<<kMomBlocks, kMomThreads, 0, st>>>(rho, S, partial)
  PSN_LMAX_SWITCH(lmax, PSN_CALL)
#undef PSN_CALL
}

void finish_moments(const double* partial, int nq, double point_mass, double* q, hipStream_t st) {
  k_finish_moments<<<nq, 256, 0, st>>>(partial, point_mass, q);
}

void cart_ghosts(double* phi, long long p0, long long p1, int n, int g, double h, double lo, double cx, double cy,
                 double cz, int lmax, const double* q, double G, hipStream_t st) {
  const int E = n - 1, M = E + 2 * g;
  const long long total = 2LL * g * M * M + (long long)E * 2 * g * M + (long long)E * E * 2 * g;
  const unsigned blocks = (unsigned)((total + 255) / 256);
#define PSN_CALL(L) \
  k_cart_ghosts<L><<<blocks, 256, 0, st>>>(phi, p0, p1, n, g, h, lo, cx, cy, cz, q, G)
  PSN_LMAX_SWITCH(lmax, PSN_CALL)
#undef PSN_CALL
}

void sph_ghosts(double* phi, const SGeom& S, int lmax, const double* q, const double* qbar, double point_mass,
                double G, hipStream_t st) {
  const int total = 2 * S.nth * S.nph;
  const unsigned blocks = (unsigned)((total + 255) / 256);
#define PSN_CALL(L) k_sph_ghosts<L><<<blocks, 256, 0, st>>>(phi, S, q, qbar, point_mass, G)
  PSN_LMAX_SWITCH(lmax, PSN_CALL)
#undef PSN_CALL
}

}  // namespace psn
