// Log-spherical Poisson operator (Eq. 2 multiplied by r^2, s = ln r) and the
// fused BiCGSTAB kernels (Section 2.1.2: BiCGSTAB for the non-symmetric
// direct finite-difference spherical Laplacian) for gfx950, FP64.
//   r^2 lap u = u_ss + u_s + u_tt + cot(t) u_t + u_pp / sin^2(t)
// with 2nd-order central differences; radial ghosts hold Dirichlet values,
// the colatitude neighbour past a pole is the node at phi + pi, phi is
// periodic.  Direction vectors keep zero radial ghosts.
#include "internal.h"
#include "reduce.h"

namespace psn {

namespace {

constexpr int BX = 64, BY = 4;

struct Coef {
  double ids2, i2ds, idt2, idp2;
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
  return (ip - 2.0 * u + im) * c.ids2 + (ip - im) * c.i2ds + (jp - 2.0 * u + jm) * c.idt2 + cot2[j] * (jp - jm) +
         (kp - 2.0 * u + km) * isin2[j] * c.idp2;
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

// Right-preconditioned BiCGSTAB (Section 2.1.2: a multi-colour Gauss-Seidel
// preconditioner B, the block lower triangle of A in red-black order, applied
// by block substitution).  Red nodes (i + j + k even) solve with their
// diagonal, black nodes subtract their red neighbours' values first;
// couplings between nodes of one colour (only across a pole, when nphi/2 is
// even) are left out of B.  scal->v: 0 rho, 1 alpha, 2 omega, 3 beta,
// 4 rhat.v, 5 t.s, 6 t.t, 7 r.r.

__device__ inline double sph_diag(const SGeom& S, const Coef& c, const double* __restrict__ isin2, int j) {
  return -2.0 * c.ids2 - 2.0 * c.idt2 - 2.0 * isin2[j] * c.idp2;
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
  if (is_red(i, j, k)) Ph[idx] = pv / sph_diag(S, c, isin2, j);
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
  if (is_red(i, j, k)) Sh[idx] = sv / sph_diag(S, c, isin2, j);
}

// black nodes of xhat = B^-1 y: (y - sum over red neighbours of a_n xhat_n) / D
__global__ __launch_bounds__(256) void k_gs_black(const double* __restrict__ Y, double* __restrict__ Xh, SGeom S,
                                                  Coef c, const double* __restrict__ cot2,
                                                  const double* __restrict__ isin2) {
  const int i = 1 + blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (!active(S, i, j, k) || is_red(i, j, k)) return;
  const int half = S.nph >> 1;
  // value of a neighbour if it is red, else 0 (radial ghosts of xhat are 0)
  auto red = [&](int ii, int jj, int kk) -> double { return is_red(ii, jj, kk) ? Xh[S.at(ii, jj, kk)] : 0.0; };
  const double cr = c.ids2 + c.i2ds, cl = c.ids2 - c.i2ds;
  double s = cr * red(i + 1, j, k) + cl * red(i - 1, j, k);
  const double cjp = c.idt2 + cot2[j], cjm = c.idt2 - cot2[j];
  s += cjp * ((j + 1 < S.nth) ? red(i, j + 1, k) : red(i, S.nth - 1, (k + half) % S.nph));
  s += cjm * ((j > 0) ? red(i, j - 1, k) : red(i, 0, (k + half) % S.nph));
  const double cp = isin2[j] * c.idp2;
  s += cp * (red(i, j, (k + 1) % S.nph) + red(i, j, (k + S.nph - 1) % S.nph));
  const long long idx = S.at(i, j, k);
  Xh[idx] = (Y[idx] - s) / sph_diag(S, c, isin2, j);
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
__global__ void k_bicg_scalars(const double* __restrict__ partial, int nb, Scalars* __restrict__ scal, int stage) {
  double s0 = 0.0, s1 = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    s0 += partial[b];
    if (stage > 0) s1 += partial[kPartialCap + b];
  }
  s0 = block_sum(s0);
  __syncthreads();
  s1 = block_sum(s1);
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

Coef make_coef(const SGeom& S) {
  Coef c;
  c.ids2 = 1.0 / (S.ds * S.ds);
  c.i2ds = 1.0 / (2.0 * S.ds);
  c.idt2 = 1.0 / (S.dth * S.dth);
  c.idp2 = 1.0 / (S.dph * S.dph);
  return c;
}

}  // namespace

int sph_blocks(const SGeom& S) {
  const dim3 g = sgrid(S);
  return (int)(g.x * g.y * g.z);
}

void sph_residual(const double* u, const double* rho, double* r, const SGeom& S, const SphCoef& c,
                  double four_pi_G, bool zu, double* partial, hipStream_t st) {
  const Coef cf = make_coef(S);
  if (zu)
    k_sph_residual<true><<<sgrid(S), dim3(BX, BY), 0, st>>>(u, rho, r, S, cf, c.cot, c.isin2, c.r2, four_pi_G,
                                                           partial);
  else
    k_sph_residual<false><<<sgrid(S), dim3(BX, BY), 0, st>>>(u, rho, r, S, cf, c.cot, c.isin2, c.r2, four_pi_G,
                                                            partial);
}

void sph_apply(const double* u, double* out, const SGeom& S, const SphCoef& c, hipStream_t st) {
  k_sph_apply<<<sgrid(S), dim3(BX, BY), 0, st>>>(u, out, S, make_coef(S), c.cot, c.isin2);
}

void pbicg_direction(const double* r, double* p, const double* v, double* phat, const SGeom& S, const SphCoef& c,
                     const Scalars* scal, hipStream_t st) {
  const Coef cf = make_coef(S);
  k_pbicg_p<<<sgrid(S), dim3(BX, BY), 0, st>>>(r, p, v, phat, S, cf, c.isin2, scal);
  k_gs_black<<<sgrid(S), dim3(BX, BY), 0, st>>>(p, phat, S, cf, c.cot, c.isin2);
}

void pbicg_s(const double* r, const double* v, double* s, double* shat, const SGeom& S, const SphCoef& c,
             const Scalars* scal, hipStream_t st) {
  const Coef cf = make_coef(S);
  k_pbicg_s<<<sgrid(S), dim3(BX, BY), 0, st>>>(r, v, s, shat, S, cf, c.isin2, scal);
  k_gs_black<<<sgrid(S), dim3(BX, BY), 0, st>>>(s, shat, S, cf, c.cot, c.isin2);
}

void pbicg_apply(const double* xhat, double* out, const double* w, int mode, const SGeom& S, const SphCoef& c,
                 double* partial, hipStream_t st) {
  const Coef cf = make_coef(S);
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
  k_bicg_scalars<<<1, 256, 0, st>>>(partial, nb, scal, stage);
}

void sph_fill_zero(double* x, const SGeom& S, hipStream_t st) {
  k_sph_fill<<<dim3((unsigned)((S.p0 + BX - 1) / BX), (S.nth + BY - 1) / BY, S.nph), dim3(BX, BY), 0, st>>>(x, S);
}

void sph_copy(const double* src, double* dst, const SGeom& S, hipStream_t st) {
  k_sph_copy<<<dim3((S.nr + 2 + BX - 1) / BX, (S.nth + BY - 1) / BY, S.nph), dim3(BX, BY), 0, st>>>(src, dst, S);
}

}  // namespace psn
