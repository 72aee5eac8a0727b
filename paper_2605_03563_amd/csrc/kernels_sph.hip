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

// scal->v: 0 rho, 1 alpha, 2 omega, 3 beta, 4 rhat.v, 5 t.s, 6 t.t, 7 r.r
// p = r + beta (p_old - omega v_old);  v = A p;  partial0 += rhat . v
__global__ __launch_bounds__(256) void k_bicg_pv(const double* __restrict__ R, const double* __restrict__ Pold,
                                                 const double* __restrict__ Vold, double* __restrict__ P,
                                                 double* __restrict__ Vn, const double* __restrict__ Rhat, SGeom S,
                                                 Coef c, const double* __restrict__ cot2,
                                                 const double* __restrict__ isin2,
                                                 const Scalars* __restrict__ scal, double* __restrict__ partial) {
  const int i = 1 + blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  const double beta = scal->v[3], omega = scal->v[2];
  double acc = 0.0;
  if (active(S, i, j, k)) {
    auto V = [&](int ii, int jj, int kk) -> double {
      const long long q = S.at(ii, jj, kk);
      return R[q] + beta * (Pold[q] - omega * Vold[q]);
    };
    const long long idx = S.at(i, j, k);
    const double av = sph_op(V, S, c, cot2, isin2, i, j, k);
    P[idx] = V(i, j, k);
    Vn[idx] = av;
    acc = Rhat[idx] * av;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = s;
}

// s = r - alpha v;  t = A s;  partial0 += t.s, partial1 += t.t
__global__ __launch_bounds__(256) void k_bicg_st(const double* __restrict__ R, const double* __restrict__ Vv,
                                                 double* __restrict__ Sv, double* __restrict__ T, SGeom S, Coef c,
                                                 const double* __restrict__ cot2, const double* __restrict__ isin2,
                                                 const Scalars* __restrict__ scal, double* __restrict__ partial) {
  const int i = 1 + blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  const double alpha = scal->v[1];
  double a0 = 0.0, a1 = 0.0;
  if (active(S, i, j, k)) {
    auto V = [&](int ii, int jj, int kk) -> double {
      const long long q = S.at(ii, jj, kk);
      return R[q] - alpha * Vv[q];
    };
    const long long idx = S.at(i, j, k);
    const double sv = V(i, j, k);
    const double tv = sph_op(V, S, c, cot2, isin2, i, j, k);
    Sv[idx] = sv;
    T[idx] = tv;
    a0 = tv * sv;
    a1 = tv * tv;
  }
  const double s0 = block_sum(a0);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = s0;
  const double s1 = block_sum(a1);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[kPartialCap + linear_block()] = s1;
}

// x += alpha p + omega s;  r = s - omega t;  partial0 += rhat.r, partial1 += r.r
__global__ __launch_bounds__(256) void k_bicg_xr(double* __restrict__ X, double* __restrict__ R,
                                                 const double* __restrict__ P, const double* __restrict__ Sv,
                                                 const double* __restrict__ T, const double* __restrict__ Rhat,
                                                 SGeom S, const Scalars* __restrict__ scal,
                                                 double* __restrict__ partial) {
  const int i = 1 + blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  const double alpha = scal->v[1], omega = scal->v[2];
  double a0 = 0.0, a1 = 0.0;
  if (active(S, i, j, k)) {
    const long long idx = S.at(i, j, k);
    const double sv = Sv[idx];
    X[idx] += alpha * P[idx] + omega * sv;
    const double rn = sv - omega * T[idx];
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

void bicg_p_v(const double* r, const double* p_old, const double* v_old, double* p, double* v, const double* rhat,
              const SGeom& S, const SphCoef& c, const Scalars* scal, double* partial, hipStream_t st) {
  k_bicg_pv<<<sgrid(S), dim3(BX, BY), 0, st>>>(r, p_old, v_old, p, v, rhat, S, make_coef(S), c.cot, c.isin2, scal,
                                               partial);
}

void bicg_s_t(const double* r, const double* v, double* s, double* t, const SGeom& S, const SphCoef& c,
              const Scalars* scal, double* partial, hipStream_t st) {
  k_bicg_st<<<sgrid(S), dim3(BX, BY), 0, st>>>(r, v, s, t, S, make_coef(S), c.cot, c.isin2, scal, partial);
}

void bicg_xr(double* x, double* r, const double* p, const double* s, const double* t, const double* rhat,
             const SGeom& S, const Scalars* scal, double* partial, hipStream_t st) {
  k_bicg_xr<<<sgrid(S), dim3(BX, BY), 0, st>>>(x, r, p, s, t, rhat, S, scal, partial);
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
