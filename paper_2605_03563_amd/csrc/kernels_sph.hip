// Spherical Poisson operator (Eq. 2 multiplied by r^2) and the fused
// BiCGSTAB kernels (Section 2.1.2: BiCGSTAB for the non-symmetric direct
// finite-difference spherical Laplacian) for gfx950, FP64.
//   r^2 lap u = a u_xixi + b u_xi + u_tt + cot(t) u_t + u_pp / sin^2(t)
// on the radial map coordinate xi (a = 1/ds^2, b = 1/ds on the log grid,
// i.e. u_ss + u_s), with 2nd-order central differences: the radial couplings
// cl = a - b/2, cr = a + b/2 come per radial index from tables; radial ghosts hold Dirichlet values,
// the colatitude neighbour past a pole is the node at phi + pi, phi is
// periodic.  Direction vectors keep zero radial ghosts.
#include "internal.h"
#include "reduce.h"

namespace psn {

namespace {

constexpr int BX = 64, BY = 4;

struct Coef {
  double idt2, idp2;
  const double* rcl;  // radial couplings per radial index
  const double* rcr;
};

inline dim3 sgrid(const SGeom& S) { return dim3((S.nr + BX - 1) / BX, (S.nth + BY - 1) / BY, S.nph); }

// value of the operator at unknown (i, j, k) for a vector given by functor V
template <typename F>
__device__ inline double sph_op(const F& V, const SGeom& S, const Coef& c, const double* __restrict__ cot2,
                                const double* __restrict__ isin2, int i, int j, int k) {
  const int half = S.nph >> 1;
  const double u = V(i, j, k);
  const double ip = V(i + 1, j, k), im = V(i - 1, j, k);
  const double jp = (j + 1 < S.nth) ? V(i, j + 1, k) : V(i, S.nth - 1, (k + half) % S.nph);
  const double jm = (j > 0) ? V(i, j - 1, k) : V(i, 0, (k + half) % S.nph);
  const double kp = V(i, j, (k + 1) % S.nph), km = V(i, j, (k + S.nph - 1) % S.nph);
  return c.rcr[i] * ip + c.rcl[i] * im - (c.rcl[i] + c.rcr[i]) * u + (jp - 2.0 * u + jm) * c.idt2 +
         cot2[j] * (jp - jm) + (kp - 2.0 * u + km) * isin2[j] * c.idp2;
}

// one thread per pair of radial indices (the kernels that visit one colour)
inline dim3 black_grid(const SGeom& S) {
  return dim3((S.nr + 2 * BX - 1) / (2 * BX), (S.nth + BY - 1) / BY, S.nph);
}

__device__ inline bool active(const SGeom& S, int i, int j, int k) {
  return i >= 1 && i <= S.nr && j < S.nth && k < S.nph;
}

template <bool ZU>
__global__ __launch_bounds__(256) void k_sph_residual(const double* __restrict__ U, const double* __restrict__ rho,
                                                      double* __restrict__ R, SGeom S, Coef c,
                                                      const double* __restrict__ cot2,
                                                      const double* __restrict__ isin2,
                                                      const double* __restrict__ r2, double fpg,
                                                      double* __restrict__ partial) {
  const int i = 1 + blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  double acc = 0.0;
  if (active(S, i, j, k)) {
    auto V = [&](int ii, int jj, int kk) -> double {
      if (ZU && ii >= 1 && ii <= S.nr) return 0.0;
      return U[S.at(ii, jj, kk)];
    };
    const long long idx = S.at(i, j, k);
    const double res = fpg * r2[i] * rho[idx] - sph_op(V, S, c, cot2, isin2, i, j, k);
    if (R) R[idx] = res;
    acc = res * res;
  }
  if (partial) {
    const double s = block_sum(acc);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = s;
  }
}

__global__ __launch_bounds__(256) void k_sph_apply(const double* __restrict__ U, double* __restrict__ out, SGeom S,
                                                   Coef c, const double* __restrict__ cot2,
                                                   const double* __restrict__ isin2) {
  const int i = 1 + blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (!active(S, i, j, k)) return;
  auto V = [&](int ii, int jj, int kk) -> double { return U[S.at(ii, jj, kk)]; };
  out[S.at(i, j, k)] = sph_op(V, S, c, cot2, isin2, i, j, k);
}

// One colour of SOR (Section 2.1.1) on the log-spherical grid.  Colour =
// parity of (i + j + k) plus 2 for phi in the second half turn, so no two
// neighbours -- across a pole included -- share a colour; the grid covers the
// colour's half turn only.  u += omega_j (u_GS - u), u_GS solving the node's
// own row: u_GS - u = residual / diagonal.
__global__ __launch_bounds__(256) void k_sph_sor(double* __restrict__ U, const double* __restrict__ rho, SGeom S,
                                                 Coef c, const double* __restrict__ cot2,
                                                 const double* __restrict__ isin2, const double* __restrict__ r2,
                                                 double fpg, const double* __restrict__ omega, int colour,
                                                 const double* __restrict__ rj, double* __restrict__ omega_out) {
  // thread t of the row takes the node of the pass's parity among radial
  // indices 1 + 2t and 2 + 2t, so every lane has work
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z + ((colour >> 1) ? (S.nph >> 1) : 0);
  const int i0 = 1 + 2 * (int)(blockIdx.x * BX + threadIdx.x);
  const int i = i0 + ((colour + i0 + j + k) & 1);
  if (!active(S, i, j, k)) return;
  auto V = [&](int ii, int jj, int kk) -> double { return U[S.at(ii, jj, kk)]; };
  const long long idx = S.at(i, j, k);
  const double res = fpg * r2[i] * rho[idx] - sph_op(V, S, c, cot2, isin2, i, j, k);
  const double d = -(c.rcl[i] + c.rcr[i]) - 2.0 * c.idt2 - 2.0 * isin2[j] * c.idp2;
  const long long t = (long long)j * (S.nr + 2) + i;
  const double w = omega[t];
  U[idx] += w * res / d;
  // next term of the sequence (Eq. omega_n), written by the one thread of
  // (i, j) that is active in the first two planes of the half turn
  if (omega_out && (int)blockIdx.z == ((colour + i + j + (S.nph >> 1)) & 1))
    omega_out[t] = 1.0 / (1.0 - rj[t] * rj[t] * w / 4.0);
}

// next term of the relaxation sequence at every node of the table (Eq. omega_n)
__global__ void k_sph_omega(double* __restrict__ omega, const double* __restrict__ rj, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) omega[e] = 1.0 / (1.0 - rj[e] * rj[e] * omega[e] / 4.0);
}

// Right-preconditioned BiCGSTAB (Section 2.1.2: a multi-colour Gauss-Seidel
// preconditioner B, the block lower triangle of A in red-black order, applied
// by block substitution).  Red nodes (i + j + k even) solve with their
// diagonal, black nodes subtract their red neighbours' values first;
// couplings between nodes of one colour (only across a pole, when nphi/2 is
// even) are left out of B.  scal->v: 0 rho, 1 alpha, 2 omega, 3 beta,
// 4 rhat.v, 5 t.s, 6 t.t, 7 r.r.

__device__ inline double sph_diag(const Coef& c, const double* __restrict__ isin2, int i, int j) {
  return -(c.rcl[i] + c.rcr[i]) - 2.0 * c.idt2 - 2.0 * isin2[j] * c.idp2;
}

__device__ inline bool is_red(int i, int j, int k) { return ((i + j + k) & 1) == 0; }

// p = r + beta (p - omega v)   (in place);   phat = p / D on red nodes
__global__ __launch_bounds__(256) void k_pbicg_p(const double* __restrict__ R, double* __restrict__ P,
                                                 const double* __restrict__ Vv, double* __restrict__ Ph, SGeom S,
                                                 Coef c, const double* __restrict__ isin2,
                                                 const Scalars* __restrict__ scal) {
  const int i = 1 + blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (!active(S, i, j, k)) return;
  const double beta = scal->v[3], omega = scal->v[2];
  const long long idx = S.at(i, j, k);
  const double pv = R[idx] + beta * (P[idx] - omega * Vv[idx]);
  P[idx] = pv;
  if (Ph && is_red(i, j, k)) Ph[idx] = pv / sph_diag(c, isin2, i, j);
}

// s = r - alpha v;   shat = s / D on red nodes
__global__ __launch_bounds__(256) void k_pbicg_s(const double* __restrict__ R, const double* __restrict__ Vv,
                                                 double* __restrict__ Sv, double* __restrict__ Sh, SGeom S, Coef c,
                                                 const double* __restrict__ isin2,
                                                 const Scalars* __restrict__ scal) {
  const int i = 1 + blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (!active(S, i, j, k)) return;
  const long long idx = S.at(i, j, k);
  const double sv = R[idx] - scal->v[1] * Vv[idx];
  Sv[idx] = sv;
  if (Sh && is_red(i, j, k)) Sh[idx] = sv / sph_diag(c, isin2, i, j);
}

// black nodes of xhat = B^-1 y: (y - sum over red neighbours of a_n xhat_n) / D
__global__ __launch_bounds__(256) void k_gs_black(const double* __restrict__ Y, double* __restrict__ Xh, SGeom S,
                                                  Coef c, const double* __restrict__ cot2,
                                                  const double* __restrict__ isin2) {
  // thread t of the row takes the black node among radial indices 1 + 2t
  // and 2 + 2t
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  const int i0 = 1 + 2 * (int)(blockIdx.x * BX + threadIdx.x);
  const int i = i0 + ((1 + i0 + j + k) & 1);
  if (!active(S, i, j, k)) return;
  const int half = S.nph >> 1;
  // value of a neighbour if it is red, else 0 (radial ghosts of xhat are 0)
  auto red = [&](int ii, int jj, int kk) -> double { return is_red(ii, jj, kk) ? Xh[S.at(ii, jj, kk)] : 0.0; };
  double s = c.rcr[i] * red(i + 1, j, k) + c.rcl[i] * red(i - 1, j, k);
  const double cjp = c.idt2 + cot2[j], cjm = c.idt2 - cot2[j];
  s += cjp * ((j + 1 < S.nth) ? red(i, j + 1, k) : red(i, S.nth - 1, (k + half) % S.nph));
  s += cjm * ((j > 0) ? red(i, j - 1, k) : red(i, 0, (k + half) % S.nph));
  const double cp = isin2[j] * c.idp2;
  s += cp * (red(i, j, (k + 1) % S.nph) + red(i, j, (k + S.nph - 1) % S.nph));
  const long long idx = S.at(i, j, k);
  Xh[idx] = (Y[idx] - s) / sph_diag(c, isin2, i, j);
}

// out = A xhat with dots: mode 0: partial0 += a.out (a = rhat);
// mode 1: partial0 += out.a, partial1 += out.out (a = s)
template <int MODE>
__global__ __launch_bounds__(256) void k_apply_dot(const double* __restrict__ Xh, double* __restrict__ Out,
                                                   const double* __restrict__ Aw, SGeom S, Coef c,
                                                   const double* __restrict__ cot2, const double* __restrict__ isin2,
                                                   double* __restrict__ partial) {
  const int i = 1 + blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  double a0 = 0.0, a1 = 0.0;
  if (active(S, i, j, k)) {
    auto V = [&](int ii, int jj, int kk) -> double { return Xh[S.at(ii, jj, kk)]; };
    const long long idx = S.at(i, j, k);
    const double o = sph_op(V, S, c, cot2, isin2, i, j, k);
    Out[idx] = o;
    a0 = Aw[idx] * o;
    if (MODE == 1) a1 = o * o;
  }
  const double s0 = block_sum(a0);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = s0;
  if (MODE == 1) {
    const double s1 = block_sum(a1);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[kPartialCap + linear_block()] = s1;
  }
}

// x += alpha phat + omega shat;  r = s - omega t;  partial0 += rhat.r, partial1 += r.r
__global__ __launch_bounds__(256) void k_pbicg_xr(double* __restrict__ X, double* __restrict__ R,
                                                  const double* __restrict__ Ph, const double* __restrict__ Sh,
                                                  const double* __restrict__ Sv, const double* __restrict__ T,
                                                  const double* __restrict__ Rhat, SGeom S,
                                                  const Scalars* __restrict__ scal, double* __restrict__ partial) {
  const int i = 1 + blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  const double alpha = scal->v[1], omega = scal->v[2];
  double a0 = 0.0, a1 = 0.0;
  if (active(S, i, j, k)) {
    const long long idx = S.at(i, j, k);
    X[idx] += alpha * Ph[idx] + omega * Sh[idx];
    const double rn = Sv[idx] - omega * T[idx];
    R[idx] = rn;
    a0 = Rhat[idx] * rn;
    a1 = rn * rn;
  }
  const double s0 = block_sum(a0);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = s0;
  const double s1 = block_sum(a1);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[kPartialCap + linear_block()] = s1;
}

// stage 0: alpha = rho / (rhat.v); stage 1: omega = (t.s)/(t.t);
// stage 2: beta = (rho_new/rho)(alpha/omega), rho = rho_new, v[7] = r.r
__global__ __launch_bounds__(kFinishThreads) void k_bicg_scalars(const double* __restrict__ partial, int nb,
                                                                 Scalars* __restrict__ scal, int stage) {
  const double s0 = sum_partials(partial, nb);
  __syncthreads();
  const double s1 = stage > 0 ? sum_partials(partial + kPartialCap, nb) : 0.0;
  if (threadIdx.x == 0) {
    double* v = scal->v;
    if (stage == 0) {
      v[4] = s0;
      v[1] = (s0 != 0.0) ? v[0] / s0 : 0.0;
    } else if (stage == 1) {
      v[5] = s0;
      v[6] = s1;
      v[2] = (s1 != 0.0) ? s0 / s1 : 0.0;
    } else {
      v[3] = (v[0] != 0.0 && v[2] != 0.0) ? (s0 / v[0]) * (v[1] / v[2]) : 0.0;
      v[0] = s0;
      v[7] = s1;
    }
  }
}

__global__ __launch_bounds__(256) void k_sph_fill(double* __restrict__ x, SGeom S) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= S.p0 || j >= S.nth) return;
  x[S.at(i, j, k)] = 0.0;
}

__global__ __launch_bounds__(256) void k_sph_copy(const double* __restrict__ a, double* __restrict__ b, SGeom S) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= S.nr + 2 || j >= S.nth) return;
  b[S.at(i, j, k)] = a[S.at(i, j, k)];
}

// ---------------------------------------------------------------- FP32 multigrid preconditioner
// off-diagonal part of the level operator at unknown (i, j, k) (array index i+1)
__device__ inline float slev_off(const SLev& L, int i, int j, int k) {
  const int half = L.nph >> 1;
  const int a = i + 1;
  auto u = [&](int aa, int jj, int kk) -> float { return L.u[L.at(aa, jj, kk)]; };
  const float jp = (j + 1 < L.nth) ? u(a, j + 1, k) : u(a, L.nth - 1, (k + half) % L.nph);
  const float jm = (j > 0) ? u(a, j - 1, k) : u(a, 0, (k + half) % L.nph);
  const float kp = u(a, j, (k + 1) % L.nph), km = u(a, j, (k + L.nph - 1) % L.nph);
  return L.rcr[i] * u(a + 1, j, k) + L.rcl[i] * u(a - 1, j, k) + (L.idt2 + L.cot2[j]) * jp +
         (L.idt2 - L.cot2[j]) * jm + L.isin2[j] * L.idp2 * (kp + km);
}

__device__ inline float slev_diag(const SLev& L, int i, int j) {
  return -(L.rcl[i] + L.rcr[i]) - 2.0f * L.idt2 - 2.0f * L.isin2[j] * L.idp2;
}

// One zebra colour of phi-line Gauss-Seidel.  Block (x, j) takes nl lines
// i = 2 (x nl + line) + ((j + colour) & 1) at colatitude j; thread
// (line, segment) eliminates its segment of seg nodes with the tabulated
// factors (y = T^-1 d, T the segment's tridiagonal block), the segment ends
// meet in the interface system X = G E (X: line values at segment ends,
// E: the y values there), and each segment then adds the end loads:
// x = y - a (x_left v + x_right w).  Y lives in LDS as [seg][thread].
__global__ __launch_bounds__(1024) void k_sline(SLev L, int colour, int zero_guess) {
  extern __shared__ float lds[];
  const int nt = blockDim.x;
  const int t = threadIdx.x;
  const int line = t % L.nl, sgi = t / L.nl;
  const int j = blockIdx.y;
  const int i = 2 * (blockIdx.x * L.nl + line) + ((j + colour) & 1);
  const int SL = L.seg, P = L.nseg;
  float* Y = lds;
  float* E = lds + (size_t)SL * nt;
  const int it = min(i, L.ntab - 1);
  const float* tb = L.ltab + ((size_t)it * L.nth + j) * L.tstride;
  const float* m = tb;
  const float* cp = tb + SL;
  const float* v = tb + 2 * SL;
  const float* w = tb + 3 * SL;
  const float* G = tb + 4 * SL;
  const bool act = i < L.nr;
  const float aphi = L.isin2[j] * L.idp2;
  const int k0 = sgi * SL;
  if (act) {
    const int a = i + 1, half = L.nph >> 1;
    const float cr = L.rcr[i], cl = L.rcl[i];
    const float cjp = L.idt2 + L.cot2[j], cjm = L.idt2 - L.cot2[j];
    float d = 0.0f;
#pragma unroll 8
    for (int q = 0; q < SL; ++q) {
      const int k = k0 + q;
      const long long idx = L.at(a, j, k);
      // zero_guess 1: u is zero everywhere; 2: this colour's lines are still
      // zero (the cross-pole term, which reads the line itself, is zero)
      float rhs = L.f[idx];
      if (zero_guess != 1) {
        const float pole = (zero_guess == 2) ? 0.0f : L.u[L.at(a, j, (k + half) % L.nph)];
        const float up = (j + 1 < L.nth) ? L.u[idx + L.p0] : pole;
        const float um = (j > 0) ? L.u[idx - L.p0] : pole;
        rhs -= cr * L.u[L.at(a + 1, j, k)] + cl * L.u[L.at(a - 1, j, k)] + cjp * up + cjm * um;
      }
      d = (rhs - aphi * d) * m[q];
      Y[(size_t)q * nt + t] = d;
    }
    float y = d;
    for (int q = SL - 2; q >= 0; --q) {
      y = Y[(size_t)q * nt + t] - cp[q] * y;
      Y[(size_t)q * nt + t] = y;
    }
    E[(size_t)(2 * sgi) * L.nl + line] = y;
    E[(size_t)(2 * sgi + 1) * L.nl + line] = d;
  }
  __syncthreads();
  if (!act) return;
  const int rl = 2 * ((sgi + P - 1) % P) + 1, rr = 2 * ((sgi + 1) % P);
  float xl = 0.0f, xr = 0.0f;
  for (int q = 0; q < 2 * P; ++q) {
    const float e = E[(size_t)q * L.nl + line];
    xl += G[rl * 2 * P + q] * e;
    xr += G[rr * 2 * P + q] * e;
  }
  xl *= aphi;
  xr *= aphi;
  const int a = i + 1;
  for (int q = 0; q < SL; ++q)
    L.u[L.at(a, j, k0 + q)] = Y[(size_t)q * nt + t] - (xl * v[q] + xr * w[q]);
}

// Thread x of a level row takes radial array index a in the row's storage
// order (even a first, then odd), so a wavefront's accesses are contiguous;
// returns the unknown index a - 1 (outside 0 .. nr-1 for ghosts and padding).
__device__ inline int slev_unknown(const SLev& L, int x) { return (x < L.hp ? 2 * x : 2 * (x - L.hp) + 1) - 1; }

__global__ __launch_bounds__(256) void k_sres32(SLev L) {
  const int i = slev_unknown(L, blockIdx.x * BX + threadIdx.x);
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i < 0 || i >= L.nr || j >= L.nth) return;
  const long long idx = L.at(i + 1, j, k);
  L.r[idx] = L.f[idx] - (slev_off(L, i, j, k) + slev_diag(L, i, j) * L.u[idx]);
}

// coarse f = mean of the 8 fine residuals it pairs
__global__ __launch_bounds__(256) void k_srestrict(SLev Lf, SLev Lc) {
  const int I = slev_unknown(Lc, blockIdx.x * BX + threadIdx.x);
  const int J = blockIdx.y * BY + threadIdx.y;
  const int K = blockIdx.z;
  if (I < 0 || I >= Lc.nr || J >= Lc.nth) return;
  float s = 0.0f;
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) s += Lf.r[Lf.at(2 * I + a + 1, 2 * J + b, 2 * K + c)];
  Lc.f[Lc.at(I + 1, J, K)] = 0.125f * s;
}

__global__ __launch_bounds__(256) void k_sprolong(SLev Lc, SLev Lf) {
  const int i = slev_unknown(Lf, blockIdx.x * BX + threadIdx.x);
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i < 0 || i >= Lf.nr || j >= Lf.nth) return;
  Lf.u[Lf.at(i + 1, j, k)] += Lc.u[Lc.at((i >> 1) + 1, j >> 1, k >> 1)];
}

// coarsest level: u = A^-1 f with the dense FP64 inverse, one wavefront per row
__global__ __launch_bounds__(256) void k_scoarse(const double* __restrict__ inv, SLev L) {
  const int N = L.nr * L.nth * L.nph;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= N) return;
  double acc = 0.0;
  for (int col = lane; col < N; col += 64) {
    const int i = col % L.nr, j = (col / L.nr) % L.nth, k = col / (L.nr * L.nth);
    acc += inv[(long long)row * N + col] * (double)L.f[L.at(i + 1, j, k)];
  }
  acc = wave_sum(acc);
  if (lane == 0) {
    const int i = row % L.nr, j = (row / L.nr) % L.nth, k = row / (L.nr * L.nth);
    L.u[L.at(i + 1, j, k)] = (float)acc;
  }
}

__global__ __launch_bounds__(256) void k_scast_in(const double* __restrict__ x, SGeom S, SLev L) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= S.nr || j >= S.nth) return;
  L.f[L.at(i + 1, j, k)] = (float)x[S.at(i + 1, j, k)];
}

__global__ __launch_bounds__(256) void k_scast_out(SLev L, double* __restrict__ x, SGeom S) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= S.nr || j >= S.nth) return;
  x[S.at(i + 1, j, k)] = (double)L.u[L.at(i + 1, j, k)];
}

// one thread per stored entry of a level row (p0 = 2 hp), for the kernels
// indexed through slev_unknown
inline dim3 lgrid_split(const SLev& L) { return dim3((L.p0 + BX - 1) / BX, (L.nth + BY - 1) / BY, L.nph); }

Coef make_coef(const SGeom& S, const SphCoef& sc) {
  Coef c;
  c.idt2 = 1.0 / (S.dth * S.dth);
  c.idp2 = 1.0 / (S.dph * S.dph);
  c.rcl = sc.rcl;
  c.rcr = sc.rcr;
  return c;
}

}  // namespace

int sph_blocks(const SGeom& S) {
  const dim3 g = sgrid(S);
  return (int)(g.x * g.y * g.z);
}

void sph_residual(const double* u, const double* rho, double* r, const SGeom& S, const SphCoef& c,
                  double four_pi_G, bool zu, double* partial, hipStream_t st) {
  const Coef cf = make_coef(S, c);
  if (zu)
    k_sph_residual<true><<<sgrid(S), dim3(BX, BY), 0, st>>>(u, rho, r, S, cf, c.cot, c.isin2, c.r2, four_pi_G,
                                                           partial);
  else
    k_sph_residual<false><<<sgrid(S), dim3(BX, BY), 0, st>>>(u, rho, r, S, cf, c.cot, c.isin2, c.r2, four_pi_G,
                                                            partial);
}

void sph_apply(const double* u, double* out, const SGeom& S, const SphCoef& c, hipStream_t st) {
  k_sph_apply<<<sgrid(S), dim3(BX, BY), 0, st>>>(u, out, S, make_coef(S, c), c.cot, c.isin2);
}

void pbicg_direction(const double* r, double* p, const double* v, double* phat, const SGeom& S, const SphCoef& c,
                     const Scalars* scal, hipStream_t st) {
  const Coef cf = make_coef(S, c);
  k_pbicg_p<<<sgrid(S), dim3(BX, BY), 0, st>>>(r, p, v, phat, S, cf, c.isin2, scal);
  k_gs_black<<<black_grid(S), dim3(BX, BY), 0, st>>>(p, phat, S, cf, c.cot, c.isin2);
}

void pbicg_update_p(const double* r, double* p, const double* v, const SGeom& S, const SphCoef& c,
                    const Scalars* scal, hipStream_t st) {
  k_pbicg_p<<<sgrid(S), dim3(BX, BY), 0, st>>>(r, p, v, nullptr, S, make_coef(S, c), c.isin2, scal);
}

void pbicg_update_s(const double* r, const double* v, double* s, const SGeom& S, const SphCoef& c,
                    const Scalars* scal, hipStream_t st) {
  k_pbicg_s<<<sgrid(S), dim3(BX, BY), 0, st>>>(r, v, s, nullptr, S, make_coef(S, c), c.isin2, scal);
}

void pbicg_s(const double* r, const double* v, double* s, double* shat, const SGeom& S, const SphCoef& c,
             const Scalars* scal, hipStream_t st) {
  const Coef cf = make_coef(S, c);
  k_pbicg_s<<<sgrid(S), dim3(BX, BY), 0, st>>>(r, v, s, shat, S, cf, c.isin2, scal);
  k_gs_black<<<black_grid(S), dim3(BX, BY), 0, st>>>(s, shat, S, cf, c.cot, c.isin2);
}

void pbicg_apply(const double* xhat, double* out, const double* w, int mode, const SGeom& S, const SphCoef& c,
                 double* partial, hipStream_t st) {
  const Coef cf = make_coef(S, c);
  if (mode == 0)
    k_apply_dot<0><<<sgrid(S), dim3(BX, BY), 0, st>>>(xhat, out, w, S, cf, c.cot, c.isin2, partial);
  else
    k_apply_dot<1><<<sgrid(S), dim3(BX, BY), 0, st>>>(xhat, out, w, S, cf, c.cot, c.isin2, partial);
}

void pbicg_xr(double* x, double* r, const double* phat, const double* shat, const double* s, const double* t,
              const double* rhat, const SGeom& S, const Scalars* scal, double* partial, hipStream_t st) {
  k_pbicg_xr<<<sgrid(S), dim3(BX, BY), 0, st>>>(x, r, phat, shat, s, t, rhat, S, scal, partial);
}

void bicg_scalars(const double* partial, int nb, Scalars* scal, int stage, hipStream_t st) {
  k_bicg_scalars<<<1, kFinishThreads, 0, st>>>(partial, nb, scal, stage);
}

void sph_line_pass(const SLev& L, int colour, int zero_guess, hipStream_t st) {
  const int nt = L.nl * L.nseg;
  const size_t lds = sizeof(float) * ((size_t)L.seg * nt + (size_t)2 * L.nseg * L.nl);
  const int lines = (L.nr + 1) / 2;
  k_sline<<<dim3((lines + L.nl - 1) / L.nl, L.nth), nt, lds, st>>>(L, colour, zero_guess);
}
void sph_residual32(const SLev& L, hipStream_t st) { k_sres32<<<lgrid_split(L), dim3(BX, BY), 0, st>>>(L); }
void sph_restrict32(const SLev& Lf, const SLev& Lc, hipStream_t st) {
  k_srestrict<<<lgrid_split(Lc), dim3(BX, BY), 0, st>>>(Lf, Lc);
}
void sph_prolong_add32(const SLev& Lc, const SLev& Lf, hipStream_t st) {
  k_sprolong<<<lgrid_split(Lf), dim3(BX, BY), 0, st>>>(Lc, Lf);
}
void sph_coarse32(const double* inv, const SLev& L, hipStream_t st) {
  const int N = L.nr * L.nth * L.nph;
  k_scoarse<<<(N + 3) / 4, 256, 0, st>>>(inv, L);
}
void sph_cast_in(const double* x, const SGeom& S, const SLev& L0, hipStream_t st) {
  k_scast_in<<<sgrid(S), dim3(BX, BY), 0, st>>>(x, S, L0);
}
void sph_cast_out(const SLev& L0, double* x, const SGeom& S, hipStream_t st) {
  k_scast_out<<<sgrid(S), dim3(BX, BY), 0, st>>>(L0, x, S);
}

void sph_sor_pass(double* u, const double* rho, const SGeom& S, const SphCoef& c, double four_pi_G,
                  const double* omega, int colour, hipStream_t st, const double* rj, double* omega_out) {
  const dim3 g((S.nr + 2 * BX - 1) / (2 * BX), (S.nth + BY - 1) / BY, S.nph / 2);
  k_sph_sor<<<g, dim3(BX, BY), 0, st>>>(u, rho, S, make_coef(S, c), c.cot, c.isin2, c.r2, four_pi_G, omega, colour,
                                        rj, omega_out);
}

void sph_omega_next(double* omega, const double* rj, int n, hipStream_t st) {
  k_sph_omega<<<(n + 255) / 256, 256, 0, st>>>(omega, rj, n);
}

void sph_fill_zero(double* x, const SGeom& S, hipStream_t st) {
  k_sph_fill<<<dim3((unsigned)((S.p0 + BX - 1) / BX), (S.nth + BY - 1) / BY, S.nph), dim3(BX, BY), 0, st>>>(x, S);
}

void sph_copy(const double* src, double* dst, const SGeom& S, hipStream_t st) {
  k_sph_copy<<<dim3((S.nr + 2 + BX - 1) / BX, (S.nth + BY - 1) / BY, S.nph), dim3(BX, BY), 0, st>>>(src, dst, S);
}

}  // namespace psn
