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
#include <algorithm>

#include "internal.h"
#include "reduce.h"

namespace psn {
namespace {

constexpr int BX = 64, BY = 4, KZ = 8;

// planes per block of the 27-point kernels: 32 on the 511^3 level (2-4% less
// time per SPAI cycle than 8: fewer plane pipelines to start), 8 from 127^3
inline int nkz(const NGeom& G) { return G.n >= 512 ? 32 : G.n >= 128 ? KZ : 1; }
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

// r = f - A u (r stored unless r == nullptr; with NORM the squares summed
// into one partial per block).  T is the storage type of the level (FP64, or
// FP32 on coarse levels); all arithmetic is FP64.
template <bool NORM, typename T>
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
      const double r = (double)f[idx] - s;
      if (dst) dst[idx] = (T)r;
      if (NORM) acc += r * r;
      m = z;
      z = p;
    }
  }
  if (NORM) {
    const double b = block_sum(acc);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = b;
  }
}

// One fused Richardson step out of place: out = u - M (f - A u) at the
// unknowns (Eq. richardson), reading u and f once and writing out once.
// A block owns a 64 x FY output tile and a run of planes.  Per plane q it
// loads u on the tile plus a 2-node halo into LDS, every thread forms the
// in-plane sums (c, f4, e4) of u for its points of the 66 x (FY+2) residual tile
// (tile plus a 1-node halo) and keeps the last three planes of them in
// registers, which gives r at plane q-1 (zero off the unknowns, so M acts on
// r extended by zero); r goes to LDS, and the in-plane sums of r at the
// thread's own column, again kept for three planes, give the output at plane
// q-2.  Out of place because neighbouring tiles read the old u in their halos.
constexpr int FX = 64;
template <typename T, int FY>
__global__ __launch_bounds__(FX* FY) void k_nspai(const T* __restrict__ u, const T* __restrict__ f,
                                                  T* __restrict__ out, NGeom G, W4 A, W4 M) {
  constexpr int UX = FX + 4, UY = FY + 4, RX = FX + 2, RY = FY + 2, NT = FX * FY;
  static_assert(RX * RY <= 2 * NT, "at most two residual-tile points per thread");
  __shared__ double Us[UY][UX];
  __shared__ double Rs[RY][RX];
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int n = G.n;
  const int tid = (int)threadIdx.x + FX * (int)threadIdx.y;
  const int i0 = 1 + bx * FX, j0 = 1 + by * FY;
  const int kz = (n - 1 + (int)gridDim.z - 1) / (int)gridDim.z;
  const int kb = 1 + bz * kz;
  const int ke = min(kb + kz - 1, n - 1);
  if (kb > ke) return;  // uniform over the block
  // residual-tile points of this thread: tid and tid + NT
  int rx[2], ry[2];
  bool rin[2];
  const int np = (tid + NT < RX * RY) ? 2 : 1;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int idx = tid + p * NT;
    rx[p] = idx % RX;
    ry[p] = idx / RX;
    const int gi = i0 - 1 + rx[p], gj = j0 - 1 + ry[p];
    rin[p] = p < np && gi >= 1 && gi <= n - 1 && gj >= 1 && gj <= n - 1;
  }
  const int oi = (int)threadIdx.x, oj = (int)threadIdx.y;
  const int gi = i0 + oi, gj = j0 + oj;
  const bool oin = gi <= n - 1 && gj <= n - 1;
  auto lds_sums = [](const double* b, int pitch) {
    Plane s;
    s.c = b[0];
    s.f = (b[-1] + b[1]) + (b[-pitch] + b[pitch]);
    s.e = (b[-pitch - 1] + b[-pitch + 1]) + (b[pitch - 1] + b[pitch + 1]);
    return s;
  };
  Plane us[2][3] = {};
  Plane rs[3] = {};
  double uown[3] = {0.0, 0.0, 0.0};
  // software pipeline: the u plane for the next iteration and the f values
  // of the next residual plane are loaded while this plane is computed
  constexpr int NL = (UX * UY + NT - 1) / NT;  // u-tile entries per thread (2)
  // per-thread tile offsets, fixed over the planes
  long long uoff[NL];
  bool uok[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    const int idx = tid + l * NT;
    const int x = idx % UX, y = idx / UX;
    const int gx = i0 - 2 + x, gy = j0 - 2 + y;
    uok[l] = idx < UX * UY && gx >= 0 && gx <= n && gy >= 0 && gy <= n;
    uoff[l] = uok[l] ? (long long)gy * G.W + gx : 0;
  }
  long long foff[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) foff[p] = rin[p] ? (long long)(j0 - 1 + ry[p]) * G.W + (i0 - 1 + rx[p]) : 0;
  double ureg[NL];
  auto load_u = [&](int q) {
    const bool qok = q >= 0 && q <= n;
    const long long base = (long long)q * G.P;
#pragma unroll
    for (int l = 0; l < NL; ++l) ureg[l] = (qok && uok[l]) ? (double)u[base + uoff[l]] : 0.0;
  };
  double freg[2] = {0.0, 0.0};
  auto load_f = [&](int pr) {
    const bool pok = pr >= 1 && pr <= n - 1;
    const long long base = (long long)pr * G.P;
#pragma unroll
    for (int p = 0; p < 2; ++p) freg[p] = (pok && rin[p]) ? (double)f[base + foff[p]] : 0.0;
  };
  load_u(kb - 2);
  load_f(kb - 1);
  for (int q = kb - 2; q <= ke + 2; ++q) {
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int idx = tid + l * NT;
      if (idx < UX * UY) (&Us[0][0])[idx] = ureg[l];
    }
    __syncthreads();
    if (q + 1 <= ke + 2) load_u(q + 1);
    const double fcur0 = freg[0], fcur1 = freg[1];
    if (q >= kb && q <= ke + 1) load_f(q);
    uown[0] = uown[1];
    uown[1] = uown[2];
    uown[2] = Us[oj + 2][oi + 2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (p < np) {
        us[p][0] = us[p][1];
        us[p][1] = us[p][2];
        us[p][2] = lds_sums(&Us[ry[p] + 1][rx[p] + 1], UX);
        if (q >= kb) {
          const int pr = q - 1;
          double r = 0.0;
          if (rin[p] && pr >= 1 && pr <= n - 1)
            r = (p == 0 ? fcur0 : fcur1) - apply_sums(A, us[p][0], us[p][1], us[p][2]);
          Rs[ry[p]][rx[p]] = r;
        }
      }
    }
    __syncthreads();
    if (q >= kb) {
      rs[0] = rs[1];
      rs[1] = rs[2];
      rs[2] = lds_sums(&Rs[oj + 1][oi + 1], RX);
      if (q >= kb + 2 && oin)
        __builtin_nontemporal_store((T)(uown[0] - apply_sums(M, rs[0], rs[1], rs[2])), out + G.at(gi, gj, q - 2));
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_ncopy(const T* __restrict__ a, T* __restrict__ b, long long count) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < count; i += (long long)gridDim.x * 256) b[i] = a[i];
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

// fine u += trilinear interpolation of the coarse correction (P = 8 R^T).
// A thread owns a fine (i, j) column and marches k: b_K, the sum of the four
// coarse values around (i, j) on coarse plane K (each counted twice when i or
// j is even), is formed once per coarse plane; fine plane 2K takes 2 b_K,
// plane 2K+1 takes b_K + b_{K+1}, both times 1/8.
template <typename TC, typename TF>
__global__ __launch_bounds__(BX* BY) void k_nprolong(const TC* __restrict__ uc, NGeom Gc, TF* __restrict__ uf,
                                                     NGeom Gf) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int i = 1 + bx * BX + (int)threadIdx.x;
  const int j = 1 + by * BY + (int)threadIdx.y;
  const int kz = (Gf.n - 1 + (int)gridDim.z - 1) / (int)gridDim.z;
  const int k0 = 1 + bz * kz;
  const int k1 = min(k0 + kz - 1, Gf.n - 1);
  if (i >= Gf.n || j >= Gf.n || k0 > k1) return;
  const int i0 = i >> 1, j0 = j >> 1;
  const int i1 = i0 + (i & 1), j1 = j0 + (j & 1);
  auto bsum = [&](int K) {
    return ((double)uc[Gc.at(i0, j0, K)] + (double)uc[Gc.at(i1, j0, K)]) +
           ((double)uc[Gc.at(i0, j1, K)] + (double)uc[Gc.at(i1, j1, K)]);
  };
  int Kc = k0 >> 1;
  double bc = bsum(Kc), bn = bsum(Kc + 1);
  for (int k = k0; k <= k1; ++k) {
    if ((k >> 1) != Kc) {
      Kc = k >> 1;
      bc = bn;
      bn = bsum(Kc + 1);
    }
    const double s = (k & 1) ? (bc + bn) : 2.0 * bc;
    const long long q = Gf.at(i, j, k);
    uf[q] = (TF)((double)uf[q] + 0.125 * s);
  }
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

// coarsest level by conjugate gradients on A = -L (SPD) from a zero guess,
// one block, everything in LDS: p with a zero ghost layer, x, r, q.  Stops
// once ||r|| <= rtol ||f|| or after maxit steps (Section 2.1.2's CG as the
// coarsest solve of Section 2.1.3).  Sums are block reductions in a fixed
// order.
template <typename T>
__global__ __launch_bounds__(1024) void k_ncg(const T* __restrict__ f, T* __restrict__ u, NGeom G, W4 A,
                                              double rtol, int maxit) {
  extern __shared__ double sh[];
  __shared__ double bc;
  const int E = G.n - 1, EP = E + 2, N = E * E * E;
  double* pp = sh;
  double* x = pp + EP * EP * EP;
  double* r = x + N;
  double* q = r + N;
  const int tid = threadIdx.x, nt = blockDim.x;
  auto pad = [&](int c) {
    const int i = c % E, j = (c / E) % E, k = c / (E * E);
    return ((k + 1) * EP + (j + 1)) * EP + (i + 1);
  };
  auto at = [&](int c) {
    const int i = c % E, j = (c / E) % E, k = c / (E * E);
    return G.at(i + 1, j + 1, k + 1);
  };
  for (int c = tid; c < EP * EP * EP; c += nt) pp[c] = 0.0;
  __syncthreads();
  double part = 0.0;
  for (int c = tid; c < N; c += nt) {
    const double v = (double)f[at(c)];
    x[c] = 0.0;
    r[c] = v;
    pp[pad(c)] = v;
    part += v * v;
  }
  auto allsum = [&](double v) {
    const double s = block_sum(v);
    if (tid == 0) bc = s;
    __syncthreads();
    const double out = bc;
    __syncthreads();
    return out;
  };
  double rr = allsum(part);
  const double stop = rtol * rtol * rr;
  for (int it = 0; it < maxit && rr > stop; ++it) {
    part = 0.0;
    for (int c = tid; c < N; c += nt) {
      const int o = pad(c);
      const double* b = pp + o;
      double fc = 0.0, ec = 0.0, kc = 0.0;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int nz = (dx != 0) + (dy != 0) + (dz != 0);
            const double v = b[(dz * EP + dy) * EP + dx];
            if (nz == 1) fc += v;
            else if (nz == 2) ec += v;
            else if (nz == 3) kc += v;
          }
      const double qv = -(A.c * b[0] + A.f * fc + A.e * ec + A.k * kc);
      q[c] = qv;
      part += b[0] * qv;
    }
    const double alpha = rr / allsum(part);
    part = 0.0;
    for (int c = tid; c < N; c += nt) {
      x[c] -= alpha * pp[pad(c)];
      r[c] -= alpha * q[c];
      part += r[c] * r[c];
    }
    const double rr_new = allsum(part);
    const double beta = rr_new / rr;
    for (int c = tid; c < N; c += nt) pp[pad(c)] = r[c] + beta * pp[pad(c)];
    __syncthreads();
    rr = rr_new;
  }
  for (int c = tid; c < N; c += nt) u[at(c)] = (T)x[c];
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

// right-hand side at the unknowns: scale * B rho, with B
//   order 2: the identity;
//   order 4: (6 rho_n + sum of the 6 face neighbours) / 12;
//   order 6: (402 rho_n + 40 (6 face neighbours) - 3 (6 axis nodes at
//            distance 2) + 8 (12 in-plane diagonals)) / 720, i.e.
//            rho + D/12 - D^2/240 + (mixed D_d D_e)/90 collected per node
//            (D the unit-spacing second differences); reads rho two nodes
//            beyond the unknowns.
__global__ __launch_bounds__(BX* BY) void k_nrhs(const double* __restrict__ rho, long long p0, long long p1,
                                                 double* __restrict__ f, NGeom G, int order, double scale) {
  const int i = 1 + blockIdx.x * BX + (int)threadIdx.x;
  const int j = 1 + blockIdx.y * BY + (int)threadIdx.y;
  const int k = 1 + blockIdx.z;
  if (i >= G.n || j >= G.n || k >= G.n) return;
  const long long q = k * p1 + j * p0 + i;
  double v = rho[q];
  if (order == 4) {
    v = (6.0 * v + ((rho[q - 1] + rho[q + 1]) + (rho[q - p0] + rho[q + p0]) + (rho[q - p1] + rho[q + p1]))) *
        (1.0 / 12.0);
  } else if (order == 6) {
    const double f1 = (rho[q - 1] + rho[q + 1]) + (rho[q - p0] + rho[q + p0]) + (rho[q - p1] + rho[q + p1]);
    const double f2 =
        (rho[q - 2] + rho[q + 2]) + (rho[q - 2 * p0] + rho[q + 2 * p0]) + (rho[q - 2 * p1] + rho[q + 2 * p1]);
    const double exy = (rho[q - p0 - 1] + rho[q - p0 + 1]) + (rho[q + p0 - 1] + rho[q + p0 + 1]);
    const double exz = (rho[q - p1 - 1] + rho[q - p1 + 1]) + (rho[q + p1 - 1] + rho[q + p1 + 1]);
    const double eyz = (rho[q - p1 - p0] + rho[q - p1 + p0]) + (rho[q + p1 - p0] + rho[q + p1 + p0]);
    v = (402.0 * v + 40.0 * f1 - 3.0 * f2 + 8.0 * (exy + exz + eyz)) * (1.0 / 720.0);
  }
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
      k_n27<true, float><<<gr, bl, 0, st>>>((const float*)u, (const float*)f, (float*)r, G, A, partial);
    else
      k_n27<false, float><<<gr, bl, 0, st>>>((const float*)u, (const float*)f, (float*)r, G, A, nullptr);
  } else {
    if (norm)
      k_n27<true, double><<<gr, bl, 0, st>>>((const double*)u, (const double*)f, (double*)r, G, A, partial);
    else
      k_n27<false, double><<<gr, bl, 0, st>>>((const double*)u, (const double*)f, (double*)r, G, A, nullptr);
  }
}

// Tile rows FY and planes per block kz: on the 511^3 level 64 x 16 tiles
// and runs of 128 planes (1024 blocks of 1024 threads) take 0.98 ms per
// step against 1.11 ms with 64 x 8 tiles and 32 planes (less recomputed
// halo, fewer pipeline start-ups); smaller levels keep 64 x 8 and shorter
// runs so that they still spread over the compute units.
template <int FY>
inline dim3 fgrid(const NGeom& G, int kz) {
  const int e = G.n - 1;
  return dim3((e + FX - 1) / FX, (e + FY - 1) / FY, (e + kz - 1) / kz);
}

template <typename T>
static void spai_step_t(const T* u, const T* f, T* out, const NGeom& G, const W4& A, const W4& M, hipStream_t st) {
  if (G.n >= 512) {
    k_nspai<T, 16><<<fgrid<16>(G, 128), dim3(FX, 16), 0, st>>>(u, f, out, G, A, M);
  } else {
    const int kz = G.n >= 256 ? 32 : G.n >= 128 ? 16 : 4;
    k_nspai<T, 8><<<fgrid<8>(G, kz), dim3(FX, 8), 0, st>>>(u, f, out, G, A, M);
  }
}

void n_spai_step(const void* u, const void* f, void* out, bool f32, const NGeom& G, const W4& A, const W4& M,
                 hipStream_t st) {
  if (f32)
    spai_step_t<float>((const float*)u, (const float*)f, (float*)out, G, A, M, st);
  else
    spai_step_t<double>((const double*)u, (const double*)f, (double*)out, G, A, M, st);
}

void n_copy(const void* a, void* b, bool f32, const NGeom& G, hipStream_t st) {
  const long long count = G.total();
  const long long blocks = std::min<long long>((count + 255) / 256, 65536);
  if (f32)
    k_ncopy<float><<<(unsigned)blocks, 256, 0, st>>>((const float*)a, (float*)b, count);
  else
    k_ncopy<double><<<(unsigned)blocks, 256, 0, st>>>((const double*)a, (double*)b, count);
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
  const dim3 gr = ngrid(Gf), bl(BX, BY);
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

size_t n_cg_lds_bytes(const NGeom& G) {
  const size_t E = G.n - 1, EP = E + 2;
  return sizeof(double) * (EP * EP * EP + 3 * E * E * E);
}

void n_coarse_cg(const void* f, void* u, bool f32, const NGeom& G, const W4& A, double rtol, hipStream_t st) {
  const int E = G.n - 1;
  const int maxit = 2 * E * E * E;
  const size_t lds = n_cg_lds_bytes(G);
  if (f32)
    k_ncg<float><<<1, 1024, lds, st>>>((const float*)f, (float*)u, G, A, rtol, maxit);
  else
    k_ncg<double><<<1, 1024, lds, st>>>((const double*)f, (double*)u, G, A, rtol, maxit);
}

// Caller arrays hold `ghost` layers; node 0 of the level (the first ghost
// layer) sits ghost - 1 nodes in along every axis.
static long long node0(int ghost, long long p0, long long p1) { return (long long)(ghost - 1) * (p1 + p0 + 1); }

void n_from_caller(const double* src, long long p0, long long p1, int ghost, double* u, const NGeom& G,
                   bool zero_inner, hipStream_t st) {
  k_nin<<<dim3((G.n + 1 + BX - 1) / BX, (G.n + 1 + BY - 1) / BY, G.n + 1), dim3(BX, BY), 0, st>>>(
      src + node0(ghost, p0, p1), p0, p1, u, G, zero_inner ? 1 : 0);
}

void n_rhs(const double* rho, long long p0, long long p1, int ghost, double* f, const NGeom& G, int order,
           double scale, hipStream_t st) {
  k_nrhs<<<inner_grid(G), dim3(BX, BY), 0, st>>>(rho + node0(ghost, p0, p1), p0, p1, f, G, order, scale);
}

void n_to_caller(const double* u, const NGeom& G, double* dst, long long p0, long long p1, int ghost,
                 hipStream_t st) {
  k_nout<<<inner_grid(G), dim3(BX, BY), 0, st>>>(u, G, dst + node0(ghost, p0, p1), p0, p1);
}

}  // namespace psn
