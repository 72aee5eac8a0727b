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
// quadrature of Eqs. outer_multipole / inner_multipole, computed by
// separable sums (Cartesian: monomial moments; spherical: radial sums per
// ray, then phi and theta), each in a fixed order.
#include "internal.h"
#include "reduce.h"

namespace psn {

namespace {

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

// ------------------------------------------------- Cartesian moments, separable
// R_lm is a homogeneous polynomial of degree l, so the Cartesian moments are
// fixed combinations of the monomial moments
//   M_abc = h^3 sum_nodes rho x^a y^b z^c,   a + b + c <= lmax,
// which factor along the axes: T_b(i,k) = sum_j rho y_j^b (threads along x
// march y), V_ab(k) = sum_i x_i^a T_b(i,k) (one block per plane), M_abc =
// sum_k z_k^c V_ab(k) (one block per monomial), and q_lm = sum C_lm^abc M_abc with the
// monomial coefficients of R_lm (host table from the same recurrence as
// regular_solid).  Every sum runs in a fixed order.

// Stage 1: thread (i, k) of chunk c sums rows j = c, c + kMomChunks, ... < E
// (interleaved chunks); T[c][k][b][i] with row pitch TP.
constexpr int kMomChunks = 4;
template <int LMAX>
__global__ __launch_bounds__(256) void k_mom_rows(const double* __restrict__ rho, long long p0, long long p1, int n,
                                                  int g, double h, double y0, double* __restrict__ T, int TP) {
  const int E = n - 1;
  const int i = blockIdx.x * 64 + (int)threadIdx.x;
  const int k = blockIdx.y * 4 + (int)threadIdx.y;
  const int c = blockIdx.z;
  if (i >= E || k >= E) return;
  const double* __restrict__ col = rho + (long long)(k + g) * p1 + (long long)g * p0 + (i + g);
  double acc[LMAX + 1];
#pragma unroll
  for (int b = 0; b <= LMAX; ++b) acc[b] = 0.0;
  int j = c;
  // eight rows per round, loads first
  for (; j + 7 * kMomChunks < E; j += 8 * kMomChunks) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = col[(long long)(j + u * kMomChunks) * p0];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double y = y0 + (j + u * kMomChunks) * h;
      double t = v[u];
#pragma unroll
      for (int b = 0; b <= LMAX; ++b) {
        acc[b] += t;
        t *= y;
      }
    }
  }
  for (; j < E; j += kMomChunks) {
    const double y = y0 + j * h;
    double t = col[(long long)j * p0];
#pragma unroll
    for (int b = 0; b <= LMAX; ++b) {
      acc[b] += t;
      t *= y;
    }
  }
  double* __restrict__ out = T + ((long long)(c * E + k) * (LMAX + 1)) * TP + i;
#pragma unroll
  for (int b = 0; b <= LMAX; ++b) out[(long long)b * TP] = acc[b];
}

// Stage 2: one block per plane k; V[k][ab] for the (a, b) pairs with
// a + b <= LMAX in the order a = 0.., b = 0..LMAX-a.  Each wave reduces its
// products with shuffles, the waves' sums meet in LDS.
template <int LMAX>
__global__ __launch_bounds__(256) void k_mom_cols(const double* __restrict__ T, int TP, int n, double h, double x0,
                                                  double* __restrict__ V) {
  constexpr int NAB = (LMAX + 1) * (LMAX + 2) / 2;
  __shared__ double red[NAB][4];
  const int E = n - 1;
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  double acc[NAB];
#pragma unroll
  for (int q = 0; q < NAB; ++q) acc[q] = 0.0;
  for (int i = tid; i < E; i += 256) {
    double tb[LMAX + 1];
#pragma unroll
    for (int b = 0; b <= LMAX; ++b) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < kMomChunks; ++c) s += T[((long long)(c * E + k) * (LMAX + 1) + b) * TP + i];
      tb[b] = s;
    }
    const double x = x0 + i * h;
    double xa = 1.0;
    int q = 0;
#pragma unroll
    for (int a = 0; a <= LMAX; ++a) {
#pragma unroll
      for (int b = 0; b + a <= LMAX; ++b) acc[q++] += xa * tb[b];
      xa *= x;
    }
  }
#pragma unroll
  for (int q = 0; q < NAB; ++q) {
    const double w = wave_sum(acc[q]);
    if ((tid & 63) == 0) red[q][tid >> 6] = w;
  }
  __syncthreads();
  if (tid < NAB) V[(long long)k * NAB + tid] = (red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]);
}

// Stage 3: one block per monomial u = (a, b, c) (packed a | b << 4 | c << 8
// in mono[u]): M_u = h^3 sum_k z_k^c V_ab(k), fixed-order block sum.
template <int LMAX>
__global__ __launch_bounds__(256) void k_mom_z(const double* __restrict__ V, int n, double h, double z0,
                                               const int* __restrict__ mono, double* __restrict__ M) {
  constexpr int NAB = (LMAX + 1) * (LMAX + 2) / 2;
  const int E = n - 1;
  const int u = blockIdx.x;
  const int a = mono[u] & 15, b = (mono[u] >> 4) & 15, c = (mono[u] >> 8) & 15;
  const int ab = a * (LMAX + 1) - a * (a - 1) / 2 + b;  // index of (a, b) in V's pair order
  double s = 0.0;
  for (int k = threadIdx.x; k < E; k += 256) {
    const double z = z0 + k * h;
    double zc = 1.0;
    for (int e = 0; e < c; ++e) zc *= z;
    s += zc * V[(long long)k * NAB + ab];
  }
  s = block_sum(s);
  if (threadIdx.x == 0) M[u] = s * (h * h * h);
}

// Stage 4: thread q < nq forms q_lm = sum of its terms coef * M[monomial]
// (+ point mass on q_00).
__global__ __launch_bounds__(128) void k_mom_q(const double* __restrict__ M, int nq, const int* __restrict__ toff,
                                               const int* __restrict__ tmono, const double* __restrict__ tcoef,
                                               double point_mass, double* __restrict__ q) {
  const int t = threadIdx.x;
  if (t >= nq) return;
  double s = 0.0;
  for (int e = toff[t]; e < toff[t + 1]; ++e) s += tcoef[e] * M[tmono[e]];
  q[t] = s + (t == 0 ? point_mass : 0.0);
}

// ------------------------------------------------- spherical moments by rays
// On a ray of direction n(theta_j, phi_k), R_lm(r n) = r^l R_lm(n), and with
// the volume weight w_i sin(theta) dtheta dphi (w_i = r^2 R' per unit of the
// radial map coordinate; r^3 ds on the log grid) the moments are
//   q_lm  = dA sum_j sin(theta_j) sum_k R_lm(n_jk) sum_i rho_ijk w_i r_i^l,
//   qb_lm = dA sum_j sin(theta_j) sum_k R_lm(n_jk) sum_i rho_ijk w_i r_i^(-l-1)
// (inner: R_lm(x / r^2) / r), dA = dtheta dphi.  R_lm(n) = A_l|m|(theta) c_m(phi) with c_m =
// cos(m phi) (m >= 0) or sin(|m| phi) (m < 0) and A_l|m| = R_l|m| at phi = 0.
// Stage 1: one wavefront per ray sums the 2 (lmax+1) radial powers (both
// expansions in one read of rho); stage 2: one block per theta_j sums over
// phi with c_m and applies sin(theta_j) A(theta_j); stage 3: one block per
// moment sums over theta.  All sums in a fixed order.

// Stage 1: S[ray][0..L] outer, S[ray][L+1..2L+1] inner, ray = k * nth + j.
template <int LMAX>
__global__ __launch_bounds__(256) void k_sph_rays(const double* __restrict__ rho, SGeom S, double* __restrict__ R) {
  constexpr int NS = 2 * (LMAX + 1);
  const int lane = threadIdx.x & 63;
  const int ray = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (ray >= S.nth * S.nph) return;  // whole wavefronts leave together
  const int j = ray % S.nth, k = ray / S.nth;
  const double* __restrict__ row = rho + S.at(1, j, k);
  double acc[NS];
#pragma unroll
  for (int e = 0; e < NS; ++e) acc[e] = 0.0;
  for (int i = lane; i < S.nr; i += 64) {
    const double v = row[i] * S.rw[i + 1];
    const double r = S.rr[i + 1];
    const double ir = 1.0 / r;
    double po = v, pi = v * ir;  // rho w, rho w / r
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) {
      acc[l] += po;
      acc[LMAX + 1 + l] += pi;
      po *= r;
      pi *= ir;
    }
  }
#pragma unroll
  for (int e = 0; e < NS; ++e) {
    const double t = wave_sum(acc[e]);
    if (lane == 0) R[(long long)ray * NS + e] = t;
  }
}

// Stage 2: block j; thread t takes phi_k for k = t, t + 256, ...; G[j][2 NQ]
// (outer then inner, index l^2 + l + m).
template <int LMAX>
__global__ __launch_bounds__(256) void k_sph_phi(const double* __restrict__ R, SGeom S, double* __restrict__ G) {
  constexpr int NS = 2 * (LMAX + 1);
  constexpr int NQ = (LMAX + 1) * (LMAX + 1);
  __shared__ double red[2 * NQ][4];
  __shared__ double A[NQ];
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  const double th = (j + 0.5) * S.dth;
  if (tid == 0) {
    // R_lm at phi = 0: A_l|m| in the m >= 0 entries (the m < 0 entries vanish)
    double a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] = 0.0;
    regular_solid<LMAX>(sin(th), 0.0, cos(th), 1.0, a);
#pragma unroll
    for (int q = 0; q < NQ; ++q) A[q] = a[q];
  }
  // one m at a time keeps the live partial sums to 4 (lmax + 1)
#pragma unroll
  for (int m = 0; m <= LMAX; ++m) {
    double co[LMAX + 1], ci[LMAX + 1], so[LMAX + 1], si[LMAX + 1];
#pragma unroll
    for (int l = 0; l <= LMAX; ++l) co[l] = ci[l] = so[l] = si[l] = 0.0;
    for (int k = tid; k < S.nph; k += 256) {
      const double* __restrict__ s = R + ((long long)k * S.nth + j) * NS;
      double sm, cm;
      sincos(m * (k * S.dph), &sm, &cm);
#pragma unroll
      for (int l = m; l <= LMAX; ++l) {
        const double vo = s[l], vi = s[LMAX + 1 + l];
        co[l] += cm * vo;
        ci[l] += cm * vi;
        so[l] += sm * vo;
        si[l] += sm * vi;
      }
    }
#pragma unroll
    for (int l = m; l <= LMAX; ++l) {
      const int qc = l * l + l + m, qs = l * l + l - m;
      const double a = wave_sum(co[l]), b = wave_sum(ci[l]);
      if ((tid & 63) == 0) {
        red[qc][tid >> 6] = a;
        red[NQ + qc][tid >> 6] = b;
      }
      if (m > 0) {
        const double c = wave_sum(so[l]), d = wave_sum(si[l]);
        if ((tid & 63) == 0) {
          red[qs][tid >> 6] = c;
          red[NQ + qs][tid >> 6] = d;
        }
      }
    }
  }
  __syncthreads();
  const double st = sin(th);
  for (int q = tid; q < 2 * NQ; q += 256) {
    const int qq = q % NQ;
    const int l = (int)sqrt((double)qq + 0.5);
    const int m = qq - l * l - l;
    const double a = A[l * l + l + (m < 0 ? -m : m)];
    G[(long long)j * 2 * NQ + q] = st * a * ((red[q][0] + red[q][1]) + (red[q][2] + red[q][3]));
  }
}

// Stage 3: block q sums G[j][q] over theta; q < NQ outer (+ point mass on
// q_00), q >= NQ inner.
__global__ __launch_bounds__(256) void k_sph_theta(const double* __restrict__ G, int nth, int nq, double dA,
                                                   double point_mass, double* __restrict__ q_out,
                                                   double* __restrict__ qb_out) {
  const int q = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < nth; j += 256) s += G[(long long)j * 2 * nq + q];
  s = block_sum(s);
  if (threadIdx.x == 0) {
    if (q < nq)
      q_out[q] = dA * s + (q == 0 ? point_mass : 0.0);
    else
      qb_out[q - nq] = dA * s;
  }
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
  const double r = S.rr[i];
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

// Host: the recurrence of regular_solid carried out on polynomials (dense
// complex coefficient arrays over x^a y^b z^c, a, b, c <= kLmaxMax).
namespace {
constexpr int kP = kLmaxMax + 1;
struct Poly {
  double re[kP][kP][kP] = {};
  double im[kP][kP][kP] = {};
};
}  // namespace

bool build_mom_tables(std::vector<int>& mono, std::vector<int>& toff, std::vector<int>& tmono,
                      std::vector<double>& tcoef) {
  const int L = kLmaxMax;
  // monomials ordered by total degree
  int index[kP][kP][kP];
  mono.clear();
  for (int d = 0; d <= L; ++d)
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b) {
        const int c = d - a - b;
        index[a][b][c] = (int)mono.size();
        mono.push_back(a | (b << 4) | (c << 8));
      }
  std::vector<std::vector<std::pair<int, double>>> terms(kNqMax);
  auto emit = [&](int qi, const double (&p)[kP][kP][kP], double scale) {
    for (int a = 0; a < kP; ++a)
      for (int b = 0; b < kP; ++b)
        for (int c = 0; c < kP; ++c)
          if (p[a][b][c] != 0.0) terms[qi].push_back({index[a][b][c], scale * p[a][b][c]});
  };
  Poly q;  // Q_mm
  q.re[0][0][0] = 1.0;
  for (int m = 0; m <= L; ++m) {
    if (m > 0) {
      // Q_mm = Q_{m-1,m-1} (x + i y) sqrt((2m-1)/(2m))
      const double f = sqrt((2.0 * m - 1.0) / (2.0 * m));
      Poly nq;
      for (int a = 0; a < kP; ++a)
        for (int b = 0; b < kP; ++b)
          for (int c = 0; c < kP; ++c) {
            const double r = q.re[a][b][c], i = q.im[a][b][c];
            if (r == 0.0 && i == 0.0) continue;
            if (a + 1 < kP) {  // times x
              nq.re[a + 1][b][c] += f * r;
              nq.im[a + 1][b][c] += f * i;
            }
            if (b + 1 < kP) {  // times i y
              nq.re[a][b + 1][c] -= f * i;
              nq.im[a][b + 1][c] += f * r;
            }
          }
      q = nq;
    }
    Poly p = q, pp;
    for (int l = m; l <= L; ++l) {
      if (l > m) {
        // Q_lm = [(2l-1) z Q_{l-1,m} - r^2 sqrt((l+m-1)(l-m-1)) Q_{l-2,m}] / sqrt((l+m)(l-m))
        const double ca = (2.0 * l - 1.0) / sqrt((double)(l + m) * (double)(l - m));
        const double cb = sqrt((double)(l + m - 1) * (double)(l - m - 1)) / sqrt((double)(l + m) * (double)(l - m));
        Poly np;
        for (int a = 0; a < kP; ++a)
          for (int b = 0; b < kP; ++b)
            for (int c = 0; c < kP; ++c) {
              if (c + 1 < kP) {
                np.re[a][b][c + 1] += ca * p.re[a][b][c];
                np.im[a][b][c + 1] += ca * p.im[a][b][c];
              }
              const double r = pp.re[a][b][c], i = pp.im[a][b][c];
              if (r == 0.0 && i == 0.0) continue;
              if (a + 2 < kP) {
                np.re[a + 2][b][c] -= cb * r;
                np.im[a + 2][b][c] -= cb * i;
              }
              if (b + 2 < kP) {
                np.re[a][b + 2][c] -= cb * r;
                np.im[a][b + 2][c] -= cb * i;
              }
              if (c + 2 < kP) {
                np.re[a][b][c + 2] -= cb * r;
                np.im[a][b][c + 2] -= cb * i;
              }
            }
        pp = p;
        p = np;
      }
      if (m == 0) {
        emit(l * l + l, p.re, 1.0);
      } else {
        emit(l * l + l + m, p.re, 1.4142135623730951);
        emit(l * l + l - m, p.im, 1.4142135623730951);
      }
    }
  }
  toff.assign(1, 0);
  tmono.clear();
  tcoef.clear();
  for (int qi = 0; qi < kNqMax; ++qi) {
    for (const auto& t : terms[qi]) {
      tmono.push_back(t.first);
      tcoef.push_back(t.second);
    }
    toff.push_back((int)tmono.size());
  }
  return (int)tmono.size() <= kTermMax;
}

size_t cart_moment_scratch(int n) {
  const int E = n - 1;
  const long long TP = (E + 63) / 64 * 64;
  return sizeof(double) * ((long long)kMomChunks * E * (kLmaxMax + 1) * TP +
                           (long long)E * ((kLmaxMax + 1) * (kLmaxMax + 2) / 2) + kMonoMax);
}

void cart_moments(const double* rho, long long p0, long long p1, int n, int g, double h, double cx, double cy,
                  double cz, int lmax, const MomTables& tab, double point_mass, double* scratch, double* q,
                  hipStream_t st) {
  // unknown i (node i + 1) sits at lo + (i + 1) h; lo = centre - n h / 2
  const double lo = cx - 0.5 * n * h;
  const double x0 = lo + h - cx, y0 = (cy - 0.5 * n * h) + h - cy, z0 = (cz - 0.5 * n * h) + h - cz;
  const int E = n - 1;
  const int TP = (E + 63) / 64 * 64;
  double* T = scratch;
  double* V = scratch + (long long)kMomChunks * E * (kLmaxMax + 1) * TP;
  double* M = V + (long long)E * ((kLmaxMax + 1) * (kLmaxMax + 2) / 2);
  const int nq = (lmax + 1) * (lmax + 1);
  const int nm = (lmax + 1) * (lmax + 2) * (lmax + 3) / 6;
  const dim3 g1((E + 63) / 64, (E + 3) / 4, kMomChunks), b1(64, 4);
#define PSN_CALL(L)                                                                                     \
  k_mom_rows<L><<<g1, b1, 0, st>>>(rho, p0, p1, n, g, h, y0, T, TP);                                    \
  k_mom_cols<L><<<E, 256, 0, st>>>(T, TP, n, h, x0, V);                                                 \
  k_mom_z<L><<<nm, 256, 0, st>>>(V, n, h, z0, tab.mono, M);                                            \
  k_mom_q<<<1, 128, 0, st>>>(M, nq, tab.toff, tab.tmono, tab.tcoef, point_mass, q)
  PSN_LMAX_SWITCH(lmax, PSN_CALL)
#undef PSN_CALL
}

size_t sph_moment_scratch(int nth, int nph) {
  return sizeof(double) * ((long long)nth * nph * 2 * (kLmaxMax + 1) + (long long)nth * 2 * kNqMax);
}

void sph_moments(const double* rho, const SGeom& S, int lmax, double point_mass, double* scratch, double* q,
                 double* qbar, hipStream_t st) {
  const int nq = (lmax + 1) * (lmax + 1);
  double* R = scratch;
  double* G = scratch + (long long)S.nth * S.nph * 2 * (kLmaxMax + 1);
  const unsigned rays = (unsigned)S.nth * S.nph;
  const double dA = S.dth * S.dph;
#define PSN_CALL(L)                                                      \
  k_sph_rays<L><<<(rays + 3) / 4, 256, 0, st>>>(rho, S, R);             \
  k_sph_phi<L><<<S.nth, 256, 0, st>>>(R, S, G);                          \
  k_sph_theta<<<2 * nq, 256, 0, st>>>(G, S.nth, nq, dA, point_mass, q, qbar)
  PSN_LMAX_SWITCH(lmax, PSN_CALL)
#undef PSN_CALL
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
