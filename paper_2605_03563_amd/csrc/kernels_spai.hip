// Multigrid with sparse-approximate-inverse (SPAI) smoothing on compact
// radius-1 stencils and Galerkin coarse operators (Section 2.1.3: the
// preconditioned Richardson iteration, the radius-1 smoother stencil M, the
// Galerkin operator R A P), on natural-layout level arrays.
//
// Every operator here is a cubically symmetric 27-point stencil given by its
// centre, face, edge and corner weights.  A thread owns one (i, j) column and
// marches k; for each plane it forms the in-plane sums c = u(i, j),
// f4 = the 4 in-plane face neighbours, e4 = the 4 in-plane corners, and keeps
// them for planes k-1, k, k+1 in registers, so
//   (S u)(i,j,k) = w_c c_k + w_f (f4_k + c_{k-1} + c_{k+1})
//                + w_e (e4_k + f4_{k-1} + f4_{k+1}) + w_k (e4_{k-1} + e4_{k+1}).
#include "internal.h"
#include "reduce.h"

namespace psn {
namespace {

constexpr int BX = 64, BY = 4, KZ = 8;

inline int nkz(const NGeom& G) { return G.n >= 128 ? KZ : 1; }
inline dim3 ngrid(const NGeom& G) {
  const int e = G.n - 1;
  const int kz = nkz(G);
  return dim3((e + BX - 1) / BX, (e + BY - 1) / BY, (e + kz - 1) / kz);
}

struct Plane {
  double c, f, e;
};

// in-plane sums in FP64 whatever the storage type
template <typename T>
__device__ inline Plane plane_sums(const T* __restrict__ u, long long idx, int W) {
  auto v = [&](long long q) { return (double)u[q]; };
  Plane p;
  p.c = v(idx);
  p.f = (v(idx - 1) + v(idx + 1)) + (v(idx - W) + v(idx + W));
  p.e = (v(idx - W - 1) + v(idx - W + 1)) + (v(idx + W - 1) + v(idx + W + 1));
  return p;
}

__device__ inline double apply_sums(const W4& w, const Plane& m, const Plane& z, const Plane& p) {
  return w.c * z.c + w.f * (z.f + m.c + p.c) + w.e * (z.e + m.f + p.f) + w.k * (m.e + p.e);
}

// MODE 0: r = f - A u (r stored unless r == nullptr; with NORM the squares
// summed into one partial per block).  MODE 1: u -= M r (M already holds
// omega h^2): reads the stencil of r, writes u at the centre only.  T is the
// storage type of the level (FP64, or FP32 on coarse levels); all arithmetic
// is FP64.
template <int MODE, bool NORM, typename T>
__global__ __launch_bounds__(BX* BY) void k_n27(const T* __restrict__ src, const T* __restrict__ f,
                                                T* __restrict__ dst, NGeom G, W4 w, double* __restrict__ partial) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int i = 1 + bx * BX + (int)threadIdx.x;
  const int j = 1 + by * BY + (int)threadIdx.y;
  const int kz = (G.n - 1 + (int)gridDim.z - 1) / (int)gridDim.z;
  const int k0 = 1 + bz * kz;
  const int k1 = min(k0 + kz - 1, G.n - 1);
  double acc = 0.0;
  if (i < G.n && j < G.n && k0 <= k1) {
    Plane m = plane_sums(src, G.at(i, j, k0 - 1), G.W);
    Plane z = plane_sums(src, G.at(i, j, k0), G.W);
    for (int k = k0; k <= k1; ++k) {
      const long long idx = G.at(i, j, k);
      const Plane p = plane_sums(src, idx + G.P, G.W);
      const double s = apply_sums(w, m, z, p);
      if (MODE == 0) {
        const double r = (double)f[idx] - s;
        if (dst) dst[idx] = (T)r;
        if (NORM) acc += r * r;
      } else {
        dst[idx] = (T)((double)dst[idx] - s);
      }
      m = z;
      z = p;
    }
  }
  if (NORM) {
    const double b = block_sum(acc);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = b;
  }
}

// coarse f(I,J,K) = full weighting of the fine residual around (2I,2J,2K)
template <typename TF, typename TC>
__global__ __launch_bounds__(BX* BY) void k_nrestrict(const TF* __restrict__ r, NGeom Gf, TC* __restrict__ fc,
                                                      NGeom Gc) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int I = 1 + bx * BX + (int)threadIdx.x;
  const int J = 1 + by * BY + (int)threadIdx.y;
  const int K = 1 + bz;
  if (I >= Gc.n || J >= Gc.n || K >= Gc.n) return;
  const long long c = Gf.at(2 * I, 2 * J, 2 * K);
  auto v = [&](long long q) { return (double)r[q]; };
  auto plane = [&](long long q) {
    const double a = v(q - 1) + 2.0 * v(q) + v(q + 1);
    const double b = v(q - Gf.W - 1) + 2.0 * v(q - Gf.W) + v(q - Gf.W + 1);
    const double d = v(q + Gf.W - 1) + 2.0 * v(q + Gf.W) + v(q + Gf.W + 1);
    return b + 2.0 * a + d;
  };
  fc[Gc.at(I, J, K)] = (TC)((plane(c - Gf.P) + 2.0 * plane(c) + plane(c + Gf.P)) * (1.0 / 64.0));
}

// fine u += trilinear interpolation of the coarse correction (P = 8 R^T)
template <typename TC, typename TF>
__global__ __launch_bounds__(BX* BY) void k_nprolong(const TC* __restrict__ uc, NGeom Gc, TF* __restrict__ uf,
                                                     NGeom Gf) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int i = 1 + bx * BX + (int)threadIdx.x;
  const int j = 1 + by * BY + (int)threadIdx.y;
  const int k = 1 + bz;
  if (i >= Gf.n || j >= Gf.n || k >= Gf.n) return;
  const int i0 = i >> 1, j0 = j >> 1, k0 = k >> 1;
  const int i1 = i0 + (i & 1), j1 = j0 + (j & 1), k1 = k0 + (k & 1);
  auto line = [&](int jj, int kk) { return (double)uc[Gc.at(i0, jj, kk)] + (double)uc[Gc.at(i1, jj, kk)]; };
  const double s = (line(j0, k0) + line(j1, k0)) + (line(j0, k1) + line(j1, k1));
  const long long q = Gf.at(i, j, k);
  uf[q] = (TF)((double)uf[q] + 0.125 * s);
}

// coarsest level: u = A^-1 f with the dense inverse, one wavefront per row
template <typename T>
__global__ __launch_bounds__(256) void k_ncoarse(const double* __restrict__ inv, const T* __restrict__ f,
                                                 T* __restrict__ u, NGeom G) {
  const int E = G.n - 1;
  const int N = E * E * E;
  const int row = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= N) return;
  double acc = 0.0;
  for (int col = lane; col < N; col += 64) {
    const int i = col % E, j = (col / E) % E, k = col / (E * E);
    acc += inv[(long long)row * N + col] * (double)f[G.at(i + 1, j + 1, k + 1)];
  }
  acc = wave_sum(acc);
  if (lane == 0) {
    const int i = row % E, j = (row / E) % E, k = row / (E * E);
    u[G.at(i + 1, j + 1, k + 1)] = (T)acc;
  }
}

// caller node array (one ghost layer, pitches p0, p1) -> level array;
// interior zeroed when zero_inner
__global__ __launch_bounds__(BX* BY) void k_nin(const double* __restrict__ src, long long p0, long long p1,
                                                double* __restrict__ u, NGeom G, int zero_inner) {
  const int i = blockIdx.x * BX + (int)threadIdx.x;
  const int j = blockIdx.y * BY + (int)threadIdx.y;
  const int k = blockIdx.z;
  if (i > G.n || j > G.n || k > G.n) return;
  const bool inner = i > 0 && i < G.n && j > 0 && j < G.n && k > 0 && k < G.n;
  u[G.at(i, j, k)] = (zero_inner && inner) ? 0.0 : src[k * p1 + j * p0 + i];
}

// right-hand side at the unknowns: scale * B rho, B = identity (order 2) or
// (6 rho_n + sum of the 6 face neighbours) / 12 (order 4)
__global__ __launch_bounds__(BX* BY) void k_nrhs(const double* __restrict__ rho, long long p0, long long p1,
                                                 double* __restrict__ f, NGeom G, int order, double scale) {
  const int i = 1 + blockIdx.x * BX + (int)threadIdx.x;
  const int j = 1 + blockIdx.y * BY + (int)threadIdx.y;
  const int k = 1 + blockIdx.z;
  if (i >= G.n || j >= G.n || k >= G.n) return;
  const long long q = k * p1 + j * p0 + i;
  double v = rho[q];
  if (order == 4)
    v = (6.0 * v + ((rho[q - 1] + rho[q + 1]) + (rho[q - p0] + rho[q + p0]) + (rho[q - p1] + rho[q + p1]))) *
        (1.0 / 12.0);
  f[G.at(i, j, k)] = scale * v;
}

__global__ __launch_bounds__(BX* BY) void k_nout(const double* __restrict__ u, NGeom G, double* __restrict__ dst,
                                                 long long p0, long long p1) {
  const int i = 1 + blockIdx.x * BX + (int)threadIdx.x;
  const int j = 1 + blockIdx.y * BY + (int)threadIdx.y;
  const int k = 1 + blockIdx.z;
  if (i >= G.n || j >= G.n || k >= G.n) return;
  dst[k * p1 + j * p0 + i] = u[G.at(i, j, k)];
}

inline dim3 inner_grid(const NGeom& G) { return dim3((G.n - 1 + BX - 1) / BX, (G.n - 1 + BY - 1) / BY, G.n - 1); }

}  // namespace

NGeom make_ngeom(int n, double h) {
  NGeom G{};
  G.n = n;
  G.W = (n + 1 + 31) / 32 * 32;
  G.P = (long long)(n + 1) * G.W;
  G.h = h;
  return G;
}

long long n27_blocks(const NGeom& G) {
  const dim3 g = ngrid(G);
  return (long long)g.x * g.y * g.z;
}

void n27_residual(const void* u, const void* f, void* r, bool f32, const NGeom& G, const W4& A, bool norm,
                  double* partial, hipStream_t st) {
  const dim3 gr = ngrid(G), bl(BX, BY);
  if (f32) {
    if (norm)
      k_n27<0, true, float><<<gr, bl, 0, st>>>((const float*)u, (const float*)f, (float*)r, G, A, partial);
    else
      k_n27<0, false, float><<<gr, bl, 0, st>>>((const float*)u, (const float*)f, (float*)r, G, A, nullptr);
  } else {
    if (norm)
      k_n27<0, true, double><<<gr, bl, 0, st>>>((const double*)u, (const double*)f, (double*)r, G, A, partial);
    else
      k_n27<0, false, double><<<gr, bl, 0, st>>>((const double*)u, (const double*)f, (double*)r, G, A, nullptr);
  }
}

void n27_update(const void* r, void* u, bool f32, const NGeom& G, const W4& M, hipStream_t st) {
  if (f32)
    k_n27<1, false, float><<<ngrid(G), dim3(BX, BY), 0, st>>>((const float*)r, nullptr, (float*)u, G, M, nullptr);
  else
    k_n27<1, false, double><<<ngrid(G), dim3(BX, BY), 0, st>>>((const double*)r, nullptr, (double*)u, G, M,
                                                                nullptr);
}

void n_restrict(const void* r, bool f32_fine, const NGeom& Gf, void* fc, bool f32_coarse, const NGeom& Gc,
                hipStream_t st) {
  const dim3 gr = inner_grid(Gc), bl(BX, BY);
  if (f32_fine && f32_coarse)
    k_nrestrict<float, float><<<gr, bl, 0, st>>>((const float*)r, Gf, (float*)fc, Gc);
  else if (!f32_fine && f32_coarse)
    k_nrestrict<double, float><<<gr, bl, 0, st>>>((const double*)r, Gf, (float*)fc, Gc);
  else if (!f32_fine && !f32_coarse)
    k_nrestrict<double, double><<<gr, bl, 0, st>>>((const double*)r, Gf, (double*)fc, Gc);
  else
    k_nrestrict<float, double><<<gr, bl, 0, st>>>((const float*)r, Gf, (double*)fc, Gc);
}

void n_prolong_add(const void* uc, bool f32_coarse, const NGeom& Gc, void* uf, bool f32_fine, const NGeom& Gf,
                   hipStream_t st) {
  const dim3 gr = inner_grid(Gf), bl(BX, BY);
  if (f32_coarse && f32_fine)
    k_nprolong<float, float><<<gr, bl, 0, st>>>((const float*)uc, Gc, (float*)uf, Gf);
  else if (f32_coarse && !f32_fine)
    k_nprolong<float, double><<<gr, bl, 0, st>>>((const float*)uc, Gc, (double*)uf, Gf);
  else if (!f32_coarse && !f32_fine)
    k_nprolong<double, double><<<gr, bl, 0, st>>>((const double*)uc, Gc, (double*)uf, Gf);
  else
    k_nprolong<double, float><<<gr, bl, 0, st>>>((const double*)uc, Gc, (float*)uf, Gf);
}

void n_coarse(const double* inv, const void* f, void* u, bool f32, const NGeom& G, hipStream_t st) {
  const int E = G.n - 1;
  const int N = E * E * E;
  if (f32)
    k_ncoarse<float><<<(N + 3) / 4, 256, 0, st>>>(inv, (const float*)f, (float*)u, G);
  else
    k_ncoarse<double><<<(N + 3) / 4, 256, 0, st>>>(inv, (const double*)f, (double*)u, G);
}

void n_from_caller(const double* src, long long p0, long long p1, double* u, const NGeom& G, bool zero_inner,
                   hipStream_t st) {
  k_nin<<<dim3((G.n + 1 + BX - 1) / BX, (G.n + 1 + BY - 1) / BY, G.n + 1), dim3(BX, BY), 0, st>>>(
      src, p0, p1, u, G, zero_inner ? 1 : 0);
}

void n_rhs(const double* rho, long long p0, long long p1, double* f, const NGeom& G, int order, double scale,
           hipStream_t st) {
  k_nrhs<<<inner_grid(G), dim3(BX, BY), 0, st>>>(rho, p0, p1, f, G, order, scale);
}

void n_to_caller(const double* u, const NGeom& G, double* dst, long long p0, long long p1, hipStream_t st) {
  k_nout<<<inner_grid(G), dim3(BX, BY), 0, st>>>(u, G, dst, p0, p1);
}

}  // namespace psn
