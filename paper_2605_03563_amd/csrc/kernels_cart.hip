// Cartesian hot-path kernels for gfx950 on the colour-split layout:
// Gauss-Seidel/SOR colour passes (Section 2.1.1, 7-point; Section 2.1.2,
// four-colour 19-point star), residual with fused norm, full-weighting
// restriction and trilinear prolongation (Section 2.1.3), the exact
// coarsest-level solve (E_N = A_N^-1), conjugate-gradient vector kernels
// (Section 2.1.2) and layout conversions.  All stencil work is bound by HBM
// bandwidth: one thread owns one compact column position and marches along
// z; wavefronts read 64 consecutive elements of a colour row.
#include "internal.h"
#include "reduce.h"

namespace psn {

namespace {

constexpr int BX = 64;   // threads along a compact row
constexpr int BY = 4;    // rows per block
constexpr int KZ = 8;    // planes marched per thread

// 19-point star weights (6th-order central second difference per axis)
constexpr double kC0 = -49.0 / 18.0, kC1 = 1.5, kC2 = -3.0 / 20.0, kC3 = 1.0 / 90.0;

inline dim3 col_grid(const Geom& G) {
  const int mc = G.mhi() - G.mlo() + 1;
  const int E = G.n - 1;
  return dim3((mc + BX - 1) / BX, (E + BY - 1) / BY, (E + KZ - 1) / KZ);
}

inline dim3 node_grid(int M) { return dim3((M + BX - 1) / BX, (M + BY - 1) / BY, M); }

inline unsigned nblocks(dim3 g) { return g.x * g.y * g.z; }

template <typename T>
__device__ inline T ld(const T* p) { return *p; }

// L_h u at node (a, b, k); zu: treat the unknowns of u as zero.
template <typename T, int ORDER, bool ZU>
__device__ inline T lap_at(const T* __restrict__ X, const Geom& G, int a, int b, int k, T ih2) {
  auto v = [&](int aa, int bb, int kk) -> T {
    if (ZU && G.inner(aa) && G.inner(bb) && G.inner(kk)) return (T)0;
    return X[G.at(aa, bb, kk)];
  };
  if (ORDER == 2) {
    const T s = v(a - 1, b, k) + v(a + 1, b, k) + v(a, b - 1, k) + v(a, b + 1, k) + v(a, b, k - 1) +
                v(a, b, k + 1);
    return (s - (T)6 * v(a, b, k)) * ih2;
  } else {
    const T s1 = v(a - 1, b, k) + v(a + 1, b, k) + v(a, b - 1, k) + v(a, b + 1, k) + v(a, b, k - 1) +
                 v(a, b, k + 1);
    const T s2 = v(a - 2, b, k) + v(a + 2, b, k) + v(a, b - 2, k) + v(a, b + 2, k) + v(a, b, k - 2) +
                 v(a, b, k + 2);
    const T s3 = v(a - 3, b, k) + v(a + 3, b, k) + v(a, b - 3, k) + v(a, b + 3, k) + v(a, b, k - 3) +
                 v(a, b, k + 3);
    return ((T)(3.0 * kC0) * v(a, b, k) + (T)kC1 * s1 + (T)kC2 * s2 + (T)kC3 * s3) * ih2;
  }
}

// ---------------------------------------------------------------- colour passes
template <typename T, bool SOR>
__global__ __launch_bounds__(256) void k_pass7(T* __restrict__ X, const T* __restrict__ F, Geom G, int c,
                                               T omega, T h2) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  if (m > G.mhi() || b > last) return;
  const int k0 = G.g + bz * KZ;
  const int k1 = min(k0 + KZ - 1, last);
  T* __restrict__ Xc = X + (long long)c * G.cs;
  const T* __restrict__ Xo = X + (long long)(c ^ 1) * G.cs;
  const T* __restrict__ Fc = F + (long long)c * G.cs;
  const T sixth = (T)(1.0 / 6.0);
  for (int k = k0; k <= k1; ++k) {
    const int a = 2 * m + ((c - b - k - G.off) & 1);
    if (!G.inner(a)) continue;
    const long long row = G.row(b, k);
    const T s = Xo[row + ((a - 1) >> 1)] + Xo[row + ((a + 1) >> 1)] + Xo[G.row(b - 1, k) + m] +
                Xo[G.row(b + 1, k) + m] + Xo[G.row(b, k - 1) + m] + Xo[G.row(b, k + 1) + m];
    const T gs = (s - h2 * Fc[row + m]) * sixth;
    if (SOR)
      Xc[row + m] = ((T)1 - omega) * Xc[row + m] + omega * gs;
    else
      Xc[row + m] = gs;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_pass19(T* __restrict__ X, const T* __restrict__ F, Geom G, int c,
                                                T h2) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  if (m > G.mhi() || b > last) return;
  const int k0 = G.g + bz * KZ;
  const int k1 = min(k0 + KZ - 1, last);
  const T* __restrict__ X1 = X + (long long)((c + 1) & 3) * G.cs;  // colour c+1 (= c-3)
  const T* __restrict__ X2 = X + (long long)((c + 2) & 3) * G.cs;  // colour c+2 (= c-2)
  const T* __restrict__ X3 = X + (long long)((c + 3) & 3) * G.cs;  // colour c+3 (= c-1)
  T* __restrict__ Xc = X + (long long)c * G.cs;
  const T* __restrict__ Fc = F + (long long)c * G.cs;
  const T inv = (T)(1.0 / (3.0 * kC0));
  for (int k = k0; k <= k1; ++k) {
    const int a = 4 * m + ((c - b - k - G.off) & 3);
    if (!G.inner(a)) continue;
    const long long row = G.row(b, k);
    const T s1 = X1[row + ((a + 1) >> 2)] + X3[row + ((a - 1) >> 2)] + X1[G.row(b + 1, k) + m] +
                 X3[G.row(b - 1, k) + m] + X1[G.row(b, k + 1) + m] + X3[G.row(b, k - 1) + m];
    const T s2 = X2[row + ((a + 2) >> 2)] + X2[row + ((a - 2) >> 2)] + X2[G.row(b + 2, k) + m] +
                 X2[G.row(b - 2, k) + m] + X2[G.row(b, k + 2) + m] + X2[G.row(b, k - 2) + m];
    const T s3 = X3[row + ((a + 3) >> 2)] + X1[row + ((a - 3) >> 2)] + X3[G.row(b + 3, k) + m] +
                 X1[G.row(b - 3, k) + m] + X3[G.row(b, k + 3) + m] + X1[G.row(b, k - 3) + m];
    const T s = (T)kC1 * s1 + (T)kC2 * s2 + (T)kC3 * s3;
    Xc[row + m] = (h2 * Fc[row + m] - s) * inv;
  }
}

// ---------------------------------------------------------------- residual
// r = f - L u for every unknown; one thread handles the C nodes of a compact
// column position in a row and marches KZ planes.  Partial sums of r^2 (in
// FP64) per block when partial != nullptr.
template <typename T, typename TO, int ORDER, bool ZU>
__global__ __launch_bounds__(256) void k_residual(const T* __restrict__ X, const T* __restrict__ F,
                                                  TO* __restrict__ R, Geom G, T ih2,
                                                  double* __restrict__ partial) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  double acc = 0.0;
  if (m <= G.mhi() && b <= last) {
    const int k0 = G.g + bz * KZ;
    const int k1 = min(k0 + KZ - 1, last);
    for (int k = k0; k <= k1; ++k) {
      for (int r = 0; r < G.C; ++r) {
        const int a = (m << G.lc) + r;
        if (!G.inner(a)) continue;
        const long long idx = G.at(a, b, k);
        const T res = F[idx] - lap_at<T, ORDER, ZU>(X, G, a, b, k, ih2);
        if (R) R[idx] = (TO)res;
        acc += (double)res * (double)res;
      }
    }
  }
  if (partial) {
    const double s = block_sum(acc);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = s;
  }
}

// ---------------------------------------------------------------- transfers
// coarse f(A,B,K) = sum over the 27 fine nodes around fine node 2I of
// (1/4)[1 2 1] weights per axis; fine array index of coarse array index A is
// 2A - (g-1).
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(const T* __restrict__ Rf, Geom Gf, T* __restrict__ Fc,
                                                  Geom Gc) {
  const int A = blockIdx.x * BX + threadIdx.x;
  const int B = blockIdx.y * BY + threadIdx.y;
  const int K = blockIdx.z;
  if (A >= Gc.M || B >= Gc.M || !Gc.inner(A) || !Gc.inner(B) || !Gc.inner(K)) return;
  const int sh = Gf.g - 1;
  const int a0 = 2 * A - sh, b0 = 2 * B - sh, k0 = 2 * K - sh;
  const T w[3] = {(T)0.25, (T)0.5, (T)0.25};
  T s = (T)0;
  for (int dk = -1; dk <= 1; ++dk)
    for (int db = -1; db <= 1; ++db)
      for (int da = -1; da <= 1; ++da)
        s += w[dk + 1] * w[db + 1] * w[da + 1] * Rf[Gf.at(a0 + da, b0 + db, k0 + dk)];
  Fc[Gc.at(A, B, K)] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add(const T* __restrict__ Ec, Geom Gc, T* __restrict__ Xf,
                                                     Geom Gf) {
  const int a = blockIdx.x * BX + threadIdx.x;
  const int b = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (a >= Gf.M || b >= Gf.M || !Gf.inner(a) || !Gf.inner(b) || !Gf.inner(k)) return;
  const int sh = Gf.g - 1;
  const int i = a - sh, j = b - sh, l = k - sh;       // global fine node indices
  const int I = (i >> 1) + sh, J = (j >> 1) + sh, L = (l >> 1) + sh;  // coarse array indices
  const int oi = i & 1, oj = j & 1, ol = l & 1;
  const T half = (T)0.5;
  T s = (T)0;
  for (int dk = 0; dk <= ol; ++dk)
    for (int db = 0; db <= oj; ++db)
      for (int da = 0; da <= oi; ++da) {
        const T w = (oi ? half : (T)1) * (oj ? half : (T)1) * (ol ? half : (T)1);
        s += w * Ec[Gc.at(I + da, J + db, L + dk)];
      }
  Xf[Gf.at(a, b, k)] += s;
}

// e = A_c^{-1} f on the coarsest level: one wavefront per row of the dense
// FP64 inverse; FP32 levels are cast in and out (the solve itself is FP64).
template <typename T>
__global__ __launch_bounds__(256) void k_coarse(const double* __restrict__ inv, const T* __restrict__ F,
                                                T* __restrict__ X, Geom G) {
  const int E = G.n - 1;
  const int N = E * E * E;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= N) return;
  double acc = 0.0;
  for (int col = lane; col < N; col += 64) {
    const int ii = col % E, jj = (col / E) % E, kk = col / (E * E);
    acc += inv[(long long)row * N + col] * (double)F[G.at(ii + G.g, jj + G.g, kk + G.g)];
  }
  acc = wave_sum(acc);
  if (lane == 0) {
    const int ii = row % E, jj = (row / E) % E, kk = row / (E * E);
    X[G.at(ii + G.g, jj + G.g, kk + G.g)] = (T)acc;
  }
}

// ---------------------------------------------------------------- conversions
template <typename T>
__global__ __launch_bounds__(256) void k_split(const double* __restrict__ src, long long p0, long long p1,
                                               T* __restrict__ dst, Geom G, double scale) {
  const int a = blockIdx.x * BX + threadIdx.x;
  const int b = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (a >= G.M || b >= G.M) return;
  dst[G.at(a, b, k)] = (T)(scale * src[(long long)k * p1 + (long long)b * p0 + a]);
}

__global__ __launch_bounds__(256) void k_merge(const double* __restrict__ src, double* __restrict__ dst,
                                               long long p0, long long p1, Geom G, int unknowns_only,
                                               double scale) {
  const int a = blockIdx.x * BX + threadIdx.x;
  const int b = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (a >= G.M || b >= G.M) return;
  if (unknowns_only && !(G.inner(a) && G.inner(b) && G.inner(k))) return;
  dst[(long long)k * p1 + (long long)b * p0 + a] = scale * src[G.at(a, b, k)];
}

template <typename T>
__global__ __launch_bounds__(256) void k_ghost_copy(const double* __restrict__ src, T* __restrict__ dst,
                                                    Geom G) {
  const int a = blockIdx.x * BX + threadIdx.x;
  const int b = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (a >= G.M || b >= G.M) return;
  if (G.inner(a) && G.inner(b) && G.inner(k)) return;
  const long long i = G.at(a, b, k);
  dst[i] = (T)src[i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ x, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = (T)0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero_unknowns(T* __restrict__ X, Geom G) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  if (m > G.mhi() || b > last) return;
  const int k1 = min(G.g + bz * KZ + KZ - 1, last);
  for (int k = G.g + bz * KZ; k <= k1; ++k)
    for (int r = 0; r < G.C; ++r) {
      const int a = (m << G.lc) + r;
      if (G.inner(a)) X[G.at(a, b, k)] = (T)0;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_add_corr(double* __restrict__ X, const T* __restrict__ E, Geom G) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  if (m > G.mhi() || b > last) return;
  const int k1 = min(G.g + bz * KZ + KZ - 1, last);
  for (int k = G.g + bz * KZ; k <= k1; ++k)
    for (int r = 0; r < G.C; ++r) {
      const int a = (m << G.lc) + r;
      if (G.inner(a)) {
        const long long i = G.at(a, b, k);
        X[i] += (double)E[i];
      }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dense_split(const double* __restrict__ dense, T* __restrict__ split,
                                                     Geom G, int to_split) {
  const int E = G.n - 1;
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int l = blockIdx.z;
  if (i >= E || j >= E) return;
  const long long d = ((long long)l * E + j) * E + i;
  const long long s = G.at(i + G.g, j + G.g, l + G.g);
  if (to_split)
    split[s] = (T)dense[d];
  else
    const_cast<double*>(dense)[d] = (double)split[s];
}

// ---------------------------------------------------------------- reductions
__global__ __launch_bounds__(256) void k_finish(const double* __restrict__ partial, int nb, int nslots,
                                                Scalars* __restrict__ scal, int dst) {
  for (int slot = 0; slot < nslots; ++slot) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[slot * kPartialCap + i];
    s = block_sum(s);
    if (threadIdx.x == 0) scal->v[dst + slot] = s;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- CG (A = -L)
// p_new = r + beta p_old;  q = A p_new;  partial (p_new . q).
// scal: v[0] = rr (current r.r), v[2] = beta, v[3] = alpha.
template <int ORDER>
__global__ __launch_bounds__(256) void k_cg_dir(const double* __restrict__ R, const double* __restrict__ Pold,
                                                double* __restrict__ Pnew, double* __restrict__ Q, Geom G,
                                                double ih2, const Scalars* __restrict__ scal,
                                                double* __restrict__ partial) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  const double beta = scal->v[2];
  double acc = 0.0;
  if (m <= G.mhi() && b <= last) {
    const int k1 = min(G.g + bz * KZ + KZ - 1, last);
    auto pv = [&](int aa, int bb, int kk) -> double {
      const long long i = G.at(aa, bb, kk);
      return R[i] + beta * Pold[i];  // ghosts of R and Pold are zero
    };
    for (int k = G.g + bz * KZ; k <= k1; ++k)
      for (int r = 0; r < G.C; ++r) {
        const int a = (m << G.lc) + r;
        if (!G.inner(a)) continue;
        const double pc = pv(a, b, k);
        double lap;
        if (ORDER == 2) {
          const double s = pv(a - 1, b, k) + pv(a + 1, b, k) + pv(a, b - 1, k) + pv(a, b + 1, k) +
                           pv(a, b, k - 1) + pv(a, b, k + 1);
          lap = (s - 6.0 * pc) * ih2;
        } else {
          double s[3];
          for (int d = 1; d <= 3; ++d)
            s[d - 1] = pv(a - d, b, k) + pv(a + d, b, k) + pv(a, b - d, k) + pv(a, b + d, k) +
                       pv(a, b, k - d) + pv(a, b, k + d);
          lap = (3.0 * kC0 * pc + kC1 * s[0] + kC2 * s[1] + kC3 * s[2]) * ih2;
        }
        const long long i = G.at(a, b, k);
        Pnew[i] = pc;
        Q[i] = -lap;
        acc += pc * (-lap);
      }
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = s;
}

// x -= alpha p; r -= alpha q; partial (r . r).  The vectors follow the
// residual r = f - L x (the negative of the residual of the SPD system
// -L x = -f), so the direction enters x with a minus sign.
__global__ __launch_bounds__(256) void k_cg_upd(double* __restrict__ X, double* __restrict__ R,
                                                const double* __restrict__ P, const double* __restrict__ Q,
                                                Geom G, const Scalars* __restrict__ scal,
                                                double* __restrict__ partial) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  const double alpha = scal->v[3];
  double acc = 0.0;
  if (m <= G.mhi() && b <= last) {
    const int k1 = min(G.g + bz * KZ + KZ - 1, last);
    for (int k = G.g + bz * KZ; k <= k1; ++k)
      for (int r = 0; r < G.C; ++r) {
        const int a = (m << G.lc) + r;
        if (!G.inner(a)) continue;
        const long long i = G.at(a, b, k);
        X[i] -= alpha * P[i];
        const double rn = R[i] - alpha * Q[i];
        R[i] = rn;
        acc += rn * rn;
      }
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = s;
}

// stage 0: v[4] = p.q (summed) -> alpha = rr / pq
// stage 1: v[5] = new rr (summed) -> beta = rr_new / rr; rr = rr_new
__global__ void k_cg_scalars(const double* __restrict__ partial, int nb, Scalars* __restrict__ scal,
                             int stage) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
  s = block_sum(s);
  if (threadIdx.x == 0) {
    if (stage == 0) {
      scal->v[4] = s;
      scal->v[3] = (s != 0.0) ? scal->v[0] / s : 0.0;
    } else {
      scal->v[5] = s;
      scal->v[2] = (scal->v[0] != 0.0) ? s / scal->v[0] : 0.0;
      scal->v[0] = s;
    }
  }
}

template <typename T>
inline void launch_fill(T* x, long long count, hipStream_t st) {
  if (count <= 0) return;
  long long blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_fill<T><<<(unsigned)blocks, 256, 0, st>>>(x, count);
}

}  // namespace

// ============================================================== wrappers
Geom make_geom(int n, int g, int C, double h) {
  Geom G{};
  G.n = n;
  G.g = g;
  G.C = C;
  G.lc = (C == 2) ? 1 : 2;
  G.M = n + 1 + 2 * (g - 1);
  const int wc = (G.M + C - 1) / C;
  G.W = (wc + kRowAlign - 1) / kRowAlign * kRowAlign;
  G.off = ((-3 * (g - 1)) % C + C) % C;
  G.cs = (long long)G.M * G.M * G.W;
  G.h = h;
  return G;
}

void split_from_natural(const double* src, long long p0, long long p1, void* dst, bool dst_f32,
                        const Geom& G, double scale, hipStream_t st) {
  const dim3 grid = node_grid(G.M), blk(BX, BY);
  if (dst_f32)
    k_split<float><<<grid, blk, 0, st>>>(src, p0, p1, (float*)dst, G, scale);
  else
    k_split<double><<<grid, blk, 0, st>>>(src, p0, p1, (double*)dst, G, scale);
}

void merge_to_natural(const double* src, double* dst, long long p0, long long p1, const Geom& G,
                      bool unknowns_only, double scale, hipStream_t st) {
  k_merge<<<node_grid(G.M), dim3(BX, BY), 0, st>>>(src, dst, p0, p1, G, unknowns_only ? 1 : 0, scale);
}

void fill_zero(void* x, bool f32, long long count, hipStream_t st) {
  if (f32)
    launch_fill<float>((float*)x, count, st);
  else
    launch_fill<double>((double*)x, count, st);
}

void zero_unknowns(void* x, bool f32, const Geom& G, hipStream_t st) {
  if (f32)
    k_zero_unknowns<float><<<col_grid(G), dim3(BX, BY), 0, st>>>((float*)x, G);
  else
    k_zero_unknowns<double><<<col_grid(G), dim3(BX, BY), 0, st>>>((double*)x, G);
}

void copy_ghosts_split(const double* src, void* dst, bool dst_f32, const Geom& G, hipStream_t st) {
  if (dst_f32)
    k_ghost_copy<float><<<node_grid(G.M), dim3(BX, BY), 0, st>>>(src, (float*)dst, G);
  else
    k_ghost_copy<double><<<node_grid(G.M), dim3(BX, BY), 0, st>>>(src, (double*)dst, G);
}

void colour_pass(void* phi, const void* f, bool f32, const Geom& G, int order, int colour, double omega,
                 hipStream_t st) {
  const dim3 grid = col_grid(G), blk(BX, BY);
  const double h2 = G.h * G.h;
  if (order == 2) {
    const bool sor = omega != 1.0;
    if (f32) {
      if (sor)
        k_pass7<float, true><<<grid, blk, 0, st>>>((float*)phi, (const float*)f, G, colour, (float)omega,
                                                   (float)h2);
      else
        k_pass7<float, false><<<grid, blk, 0, st>>>((float*)phi, (const float*)f, G, colour, 1.0f,
                                                    (float)h2);
    } else {
      if (sor)
        k_pass7<double, true><<<grid, blk, 0, st>>>((double*)phi, (const double*)f, G, colour, omega, h2);
      else
        k_pass7<double, false><<<grid, blk, 0, st>>>((double*)phi, (const double*)f, G, colour, 1.0, h2);
    }
  } else {
    if (f32)
      k_pass19<float><<<grid, blk, 0, st>>>((float*)phi, (const float*)f, G, colour, (float)h2);
    else
      k_pass19<double><<<grid, blk, 0, st>>>((double*)phi, (const double*)f, G, colour, h2);
  }
}

template <typename T, typename TO>
static void residual_t(const T* phi, const T* f, TO* r, const Geom& G, int order, bool zu, double* partial,
                       hipStream_t st) {
  const dim3 grid = col_grid(G), blk(BX, BY);
  const T ih2 = (T)(1.0 / (G.h * G.h));
  if (order == 2) {
    if (zu)
      k_residual<T, TO, 2, true><<<grid, blk, 0, st>>>(phi, f, r, G, ih2, partial);
    else
      k_residual<T, TO, 2, false><<<grid, blk, 0, st>>>(phi, f, r, G, ih2, partial);
  } else {
    if (zu)
      k_residual<T, TO, 6, true><<<grid, blk, 0, st>>>(phi, f, r, G, ih2, partial);
    else
      k_residual<T, TO, 6, false><<<grid, blk, 0, st>>>(phi, f, r, G, ih2, partial);
  }
}

int residual_blocks(const Geom& G) { return (int)nblocks(col_grid(G)); }

void residual(const void* phi, const void* f, bool in_f32, void* r_out, bool out_f32, const Geom& G, int order,
              bool zu, double* partial, hipStream_t st) {
  if (in_f32) {
    residual_t<float, float>((const float*)phi, (const float*)f, (float*)r_out, G, order, zu, partial, st);
  } else if (out_f32) {
    residual_t<double, float>((const double*)phi, (const double*)f, (float*)r_out, G, order, zu, partial, st);
  } else {
    residual_t<double, double>((const double*)phi, (const double*)f, (double*)r_out, G, order, zu, partial,
                               st);
  }
}

void restrict_fw(const void* r_fine, const Geom& Gf, void* f_coarse, const Geom& Gc, bool f32, hipStream_t st) {
  const dim3 grid = node_grid(Gc.M), blk(BX, BY);
  if (f32)
    k_restrict<float><<<grid, blk, 0, st>>>((const float*)r_fine, Gf, (float*)f_coarse, Gc);
  else
    k_restrict<double><<<grid, blk, 0, st>>>((const double*)r_fine, Gf, (double*)f_coarse, Gc);
}

void prolong_add(const void* e_coarse, const Geom& Gc, void* phi_fine, const Geom& Gf, bool f32,
                 hipStream_t st) {
  const dim3 grid = node_grid(Gf.M), blk(BX, BY);
  if (f32)
    k_prolong_add<float><<<grid, blk, 0, st>>>((const float*)e_coarse, Gc, (float*)phi_fine, Gf);
  else
    k_prolong_add<double><<<grid, blk, 0, st>>>((const double*)e_coarse, Gc, (double*)phi_fine, Gf);
}

void coarse_solve(const double* inv, const void* f, void* phi, bool f32, const Geom& G, hipStream_t st) {
  const int E = G.n - 1;
  const int N = E * E * E;
  const dim3 grid((N + 3) / 4);
  if (f32)
    k_coarse<float><<<grid, 256, 0, st>>>(inv, (const float*)f, (float*)phi, G);
  else
    k_coarse<double><<<grid, 256, 0, st>>>(inv, (const double*)f, (double*)phi, G);
}

void add_correction(double* phi, const void* e, bool e_f32, const Geom& G, hipStream_t st) {
  if (e_f32)
    k_add_corr<float><<<col_grid(G), dim3(BX, BY), 0, st>>>(phi, (const float*)e, G);
  else
    k_add_corr<double><<<col_grid(G), dim3(BX, BY), 0, st>>>(phi, (const double*)e, G);
}

void dense_to_split(const double* dense, void* split, bool f32, const Geom& G, hipStream_t st) {
  const int E = G.n - 1;
  const dim3 grid((E + BX - 1) / BX, (E + BY - 1) / BY, E);
  if (f32)
    k_dense_split<float><<<grid, dim3(BX, BY), 0, st>>>(dense, (float*)split, G, 1);
  else
    k_dense_split<double><<<grid, dim3(BX, BY), 0, st>>>(dense, (double*)split, G, 1);
}

void split_to_dense(const void* split, bool f32, double* dense, const Geom& G, hipStream_t st) {
  const int E = G.n - 1;
  const dim3 grid((E + BX - 1) / BX, (E + BY - 1) / BY, E);
  if (f32)
    k_dense_split<float><<<grid, dim3(BX, BY), 0, st>>>(dense, (float*)split, G, 0);
  else
    k_dense_split<double><<<grid, dim3(BX, BY), 0, st>>>(dense, (double*)split, G, 0);
}

void finish_sum(const double* partial, int nb, int nslots, Scalars* scal, int dst, hipStream_t st) {
  k_finish<<<1, 256, 0, st>>>(partial, nb, nslots, scal, dst);
}

int cg_blocks(const Geom& G) { return (int)nblocks(col_grid(G)); }

void cg_direction_apply(const double* r, const double* p_old, double* p_new, double* q, const Geom& G, int order,
                        const Scalars* scal, double* partial, hipStream_t st) {
  const double ih2 = 1.0 / (G.h * G.h);
  if (order == 2)
    k_cg_dir<2><<<col_grid(G), dim3(BX, BY), 0, st>>>(r, p_old, p_new, q, G, ih2, scal, partial);
  else
    k_cg_dir<6><<<col_grid(G), dim3(BX, BY), 0, st>>>(r, p_old, p_new, q, G, ih2, scal, partial);
}

void cg_update(double* x, double* r, const double* p, const double* q, const Geom& G, const Scalars* scal,
               double* partial, hipStream_t st) {
  k_cg_upd<<<col_grid(G), dim3(BX, BY), 0, st>>>(x, r, p, q, G, scal, partial);
}

void cg_scalars(const double* partial, int nb, Scalars* scal, int stage, hipStream_t st) {
  k_cg_scalars<<<1, 256, 0, st>>>(partial, nb, scal, stage);
}

}  // namespace psn
