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
constexpr int TBY = 8;   // rows per block of the LDS-staged 19-point kernels

// 19-point star weights (6th-order central second difference per axis)
constexpr double kC0 = -49.0 / 18.0, kC1 = 1.5, kC2 = -3.0 / 20.0, kC3 = 1.0 / 90.0;

// Planes marched per thread: KZ on large levels; one on small levels, where
// parallelism rather than reuse along z hides the latency.
inline int kz_for(const Geom& G) { return G.n >= 128 ? KZ : 1; }

inline dim3 col_grid(const Geom& G) {
  const int mc = G.mhi() - G.mlo() + 1;
  const int E = G.n - 1;
  const int kz = kz_for(G);
  return dim3((mc + BX - 1) / BX, (E + BY - 1) / BY, (E + kz - 1) / kz);
}

// First compact column of the LDS-staged 19-point kernels' blocks.  On
// four-colour levels compact column 0 holds a single unknown per row (node 3
// of the first three ghost layers), and the unknowns span mhi + 1 = n/4 + 1
// columns: starting the blocks at column 1 lets n/4 columns fill whole
// wavefronts, and a small kernel forms the residuals of column 0.
inline int staged_mbase(const Geom& G) { return (G.C == 4 && G.mlo() == 0 && G.g == 3) ? 1 : G.mlo(); }
inline bool staged_col0(const Geom& G) { return staged_mbase(G) > G.mlo(); }
inline unsigned col0_blocks(const Geom& G) {
  const long long E = G.n - 1;
  return staged_col0(G) ? (unsigned)((E * E + 255) / 256) : 0u;
}

// 256-thread blocks numbered over the (compact column, row) pairs of the
// unknowns, z-runs as col_grid
inline dim3 flat_grid(const Geom& G) {
  const int mc = G.mhi() - G.mlo() + 1;
  const int E = G.n - 1;
  const int kz = kz_for(G);
  return dim3((unsigned)(((long long)mc * E + 255) / 256), 1, (E + kz - 1) / kz);
}

// grid of the LDS-staged 19-point kernels (64 x 8 threads per block); runs of
// 32 planes from 255^3 up, 8 on the 127^3 level, one below
inline dim3 staged_grid(const Geom& G) {
  const int mc = G.mhi() - staged_mbase(G) + 1;
  const int E = G.n - 1;
  const int kz = G.n >= 256 ? 32 : kz_for(G);
  return dim3((mc + BX - 1) / BX, (E + TBY - 1) / TBY, (E + kz - 1) / kz);
}

__device__ inline int planes_per_block(const Geom& G) { return (G.n - 1 + (int)gridDim.z - 1) / (int)gridDim.z; }

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
template <typename T>
__device__ inline void store_stream(T* p, T v) { __builtin_nontemporal_store(v, p); }

// 7-point red-black pass of colour c.  The thread owns compact column m of
// row b and KZP consecutive planes k0..k1 (k1 - k0 < KZP).  The other
// colour's value at compact m of plane k is, for the node updated on plane
// k, one x-neighbour, and the z-neighbour of the nodes updated on planes k-1
// and k+1, so it is loaded once per plane (z[]).  Every load of the thread's
// planes is issued before the first update: the loop is unrolled at compile
// time, plane indices past k1 are clamped to planes inside the array, and
// only the stores are predicated, so a wavefront keeps all of its planes'
// loads in flight at once.  ZG: zero initial guess -- the other colour is
// taken as 0 (first pass of a cycle on a zeroed correction).  DOT: also the
// block's partial sum of -(f . x_new) over the updated nodes (the PCG inner
// product when F holds the CG residual and X the preconditioned one).
template <typename T, bool SOR, bool ZG, int KZP, bool DOT>
__global__ __launch_bounds__(256) void k_pass7(T* __restrict__ X, const T* __restrict__ F, Geom G, int c,
                                               T omega, T h2, double* __restrict__ partial) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  const bool live = m <= G.mhi() && b <= last;
  if constexpr (!DOT) {
    if (!live) return;
  }
  double acc = 0.0;
  if (live) {
    const int kz = planes_per_block(G);
    const int k0 = G.g + bz * kz;
    const int k1 = min(k0 + kz - 1, last);
    const long long plane = (long long)G.M * G.W;
    const long long W = G.W;
    const long long q0 = G.row(b, 0) + m;  // (m, b) on plane 0
    T* __restrict__ xc = X + (long long)c * G.cs + q0;
    const T* __restrict__ xo = X + (long long)(c ^ 1) * G.cs + q0;
    const T* __restrict__ fc = F + (long long)c * G.cs + q0;
    const T sixth = (T)(1.0 / 6.0);
    T z[KZP + 2];
#pragma unroll
    for (int t = 0; t < KZP + 2; ++t) z[t] = ZG ? (T)0 : xo[(long long)min(k0 - 1 + t, k1 + 1) * plane];
    T xs[KZP], ym[KZP], yp[KZP], fv[KZP], old[KZP];
#pragma unroll
    for (int t = 0; t < KZP; ++t) {
      const int k = min(k0 + t, k1);
      const long long o = (long long)k * plane;
      const int r = (c - b - k - G.off) & 1;  // node a = 2m + r of plane k has colour c
      if (!ZG) {
        xs[t] = xo[o + 2 * r - 1];
        ym[t] = xo[o - W];
        yp[t] = xo[o + W];
      }
      fv[t] = fc[o];
      if (SOR) old[t] = xc[o];
    }
#pragma unroll
    for (int t = 0; t < KZP; ++t) {
      const int k = k0 + t;
      const int r = (c - b - k - G.off) & 1;
      if (k <= k1 && G.inner(2 * m + r)) {
        T s = (T)0;
        if (!ZG) s = z[t + 1] + xs[t] + ym[t] + yp[t] + z[t] + z[t + 2];
        const T gs = (s - h2 * fv[t]) * sixth;
        T* __restrict__ dst = xc + (long long)k * plane;
        if (SOR)
          *dst = ((T)1 - omega) * old[t] + omega * gs;
        else
          store_stream(dst, gs);
        if constexpr (DOT) acc += (double)fv[t] * (double)gs;
      }
    }
  }
  if constexpr (DOT) {
    const double sum = block_sum(acc);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = -sum;
  }
}

// Vector types of CPL consecutive compact columns (16-byte loads for two
// FP64 or four FP32 values, 8-byte for two FP32).
template <typename T, int N> struct VecOf;
template <> struct VecOf<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct VecOf<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };

// 7-point red-black Gauss-Seidel pass (omega = 1) of colour c with CPL
// consecutive compact columns m0 .. m0+CPL-1 per lane, read and written as
// vectors; otherwise as k_pass7 (other colour's plane window z[], every load
// of the lane's KZP planes issued before the first update).  In a row of
// colour shift r the node of column m is a = 2m + r: its x-neighbours are the
// other colour at columns m and m - 1 (r = 0) or m + 1 (r = 1), from the
// lane's own vector except at its ends, where the neighbouring lanes supply
// them (the wavefront's edge lanes load theirs).  ZG: the other colour is
// taken as zero.  DOT: also the block's partial sum of -(f . x_new) over the
// updated nodes, as k_pass7.
template <typename T, int CPL, bool ZG, int KZP, bool DOT>
__global__ __launch_bounds__(256) void k_pass7v(T* __restrict__ X, const T* __restrict__ F, Geom G, int c, T h2,
                                                double* __restrict__ partial) {
  typedef typename VecOf<T, CPL>::type V;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int lane = threadIdx.x;
  const int m0 = G.mlo() + CPL * (bx * BX + lane);
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  const bool live = m0 <= G.mhi() && b <= last;
  const int mm = live ? m0 : G.mlo();  // idle lanes load a valid group (they still shuffle)
  const int bb = min(b, last);
  const int kz = planes_per_block(G);
  const int k0 = G.g + bz * kz;
  const int k1 = min(k0 + kz - 1, last);
  const long long plane = (long long)G.M * G.W;
  const long long W = G.W;
  const long long q0 = G.row(bb, 0) + mm;
  T* __restrict__ xc = X + (long long)c * G.cs + q0;
  const T* __restrict__ xo = X + (long long)(c ^ 1) * G.cs + q0;
  const T* __restrict__ fc = F + (long long)c * G.cs + q0;
  auto ld = [](const T* p) -> V { return *reinterpret_cast<const V*>(p); };
  V z[KZP + 2];
#pragma unroll
  for (int t = 0; t < KZP + 2; ++t) z[t] = ZG ? V{} : ld(xo + (long long)min(k0 - 1 + t, k1 + 1) * plane);
  V ym[KZP], yp[KZP], fv[KZP];
  T xe[KZP];
  const bool needl = lane == 0 && mm >= 1;
  const bool needr = lane == BX - 1 && mm + CPL < G.W;
#pragma unroll
  for (int t = 0; t < KZP; ++t) {
    const int k = min(k0 + t, k1);
    const long long o = (long long)k * plane;
    const int r = (c - bb - k - G.off) & 1;
    if (!ZG) {
      ym[t] = ld(xo + o - W);
      yp[t] = ld(xo + o + W);
      xe[t] = (T)0;
      if (r == 0 && needl) xe[t] = xo[o - 1];
      if (r == 1 && needr) xe[t] = xo[o + CPL];
    }
    fv[t] = ld(fc + o);
  }
  const T sixth = (T)(1.0 / 6.0);
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < KZP; ++t) {
    const int k = k0 + t;
    const int r = (c - bb - k - G.off) & 1;
    V o;
    if (ZG) {
#pragma unroll
      for (int i = 0; i < CPL; ++i) o[i] = ((T)0 - h2 * fv[t][i]) * sixth;
    } else {
      T lft = __shfl_up(z[t + 1][CPL - 1], 1, 64);
      T rgt = __shfl_down(z[t + 1][0], 1, 64);
      if (lane == 0) lft = xe[t];
      if (lane == BX - 1) rgt = xe[t];
#pragma unroll
      for (int i = 0; i < CPL; ++i) {
        const T xs = r == 0 ? (i == 0 ? lft : z[t + 1][i - 1]) : (i == CPL - 1 ? rgt : z[t + 1][i + 1]);
        const T sum = z[t + 1][i] + xs + ym[t][i] + yp[t][i] + z[t][i] + z[t + 2][i];
        o[i] = (sum - h2 * fv[t][i]) * sixth;
      }
    }
    bool ok[CPL];
    bool all = live && k <= k1;
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      ok[i] = live && k <= k1 && mm + i <= G.mhi() && G.inner(2 * (mm + i) + r);
      all = all && ok[i];
    }
    T* __restrict__ dst = xc + (long long)k * plane;
    if (all) {
      __builtin_nontemporal_store(o, reinterpret_cast<V*>(dst));
    } else {
#pragma unroll
      for (int i = 0; i < CPL; ++i)
        if (ok[i]) store_stream(dst + i, o[i]);
    }
    if constexpr (DOT) {
#pragma unroll
      for (int i = 0; i < CPL; ++i)
        if (ok[i]) acc += (double)fv[t][i] * (double)o[i];
    }
  }
  if constexpr (DOT) {
    const double sum = block_sum(acc);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = -sum;
  }
}

// ---------------------------------------------------------------- 19-point star
// Both kernels keep a register window along z: the values at the thread's own
// compact columns of row b for planes k-3..k+3, so each plane costs one new
// load per colour.  The residual kernel stages the window's centre plane, three
// halo rows above and below and one halo column on each side in an LDS tile
// (64 x TBY threads march planes in lock step) and reads x- and y-neighbours
// from it; the pass kernel takes x-neighbours from its own vector or the
// adjacent lanes and needs no barrier.
constexpr int TROWS = TBY + 6;
static_assert(TBY >= 6, "the six halo rows of a plane tile are loaded by the first six thread rows");
static_assert(BX * TBY >= 8 * TROWS, "one halo-column cell per thread");
constexpr int TCOLS = BX + 2;

// Four-colour pass.  A lane owns CPL consecutive compact columns
// m0 .. m0+CPL-1 of one row (16-byte vector loads: two FP64 or four FP32
// columns) and marches the planes of its run; lanes are numbered over (column
// group, row) pairs of the level, so every lane of a wavefront has work
// whatever the row length, and a block of 256 lanes holds about 256 / groups
// consecutive rows.  The register window along z holds the three other
// colours at the lane's columns for planes k-3..k+3 (one new vector load per
// colour and plane).  Each plane the lanes put their window's centre vectors
// in LDS (double-buffered, one barrier per plane); x-neighbours in the
// adjacent compact columns and y-neighbours in rows b +- 1..3 come from there
// when the lane holding them is in the block, and are loaded otherwise.  ZM:
// colours whose bit is set in zmask are read as zero (the first sweep on a
// zero initial guess).  The node at position q of a compact column in a row
// with colour shift s has colour (q + s) mod 4.
// column groups of CPL compact columns covering the columns 0 .. mhi (the
// four-colour levels have mlo = 0); loads of a group stay below the row pitch
// because W is a multiple of 32 and W >= mhi + 1
template <int CPL>
__host__ __device__ inline int col_groups(const Geom& G) { return (G.mhi() + CPL) / CPL; }

template <typename T, int CPL, bool ZM>
__global__ __launch_bounds__(256) void k_pass19v(T* __restrict__ X, const T* __restrict__ F, Geom G, int c, T h2,
                                                 int zmask) {
  typedef typename VecOf<T, CPL>::type V;
  constexpr int BT = 256;
  __shared__ V cen[2][3][BT];
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int ngr = col_groups<CPL>(G);
  const int E = G.n - 1;
  const int tid = threadIdx.x;
  const int fi = bx * BT + tid;
  const int nfl = ngr * E;
  const bool live = fi < nfl;
  const int fl = live ? fi : nfl - 1;  // idle lanes mirror the last pair (loads stay in the array)
  const int gp = fl % ngr;
  const int m0 = gp * CPL;
  const int b = G.g + fl / ngr;
  const int last = G.g + G.n - 2;
  const int kz = planes_per_block(G);
  const int k0 = G.g + bz * kz;
  const int k1 = min(k0 + kz - 1, last);
  // x-neighbour groups of the same row held by the adjacent lanes of the block
  const bool lds_l = gp > 0 && tid > 0;
  const bool lds_r = gp < ngr - 1 && tid < BT - 1;
  const bool needl = !lds_l && m0 >= 1;
  const bool needr = !lds_r && m0 + CPL < G.W;
  const T* P[3];
  bool zero[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int col = (c + e + 1) & 3;
    P[e] = X + (long long)col * G.cs;
    zero[e] = ZM && ((zmask >> col) & 1);
  }
  const long long plane = (long long)G.M * G.W;
  const long long cb = (long long)b * G.W + m0;
  auto ldv = [&](int e, long long off) -> V {
    if (ZM && zero[e]) return V{};
    return *reinterpret_cast<const V*>(P[e] + off);
  };
  // y-neighbours: colour c+d (slot d-1) at row b+d, colour c-d (slot 3-d) at
  // row b-d, d = 1, 2, 3; lane tid + dy ngr holds row b+dy of the same group
  constexpr int dy[6] = {1, -1, 2, -2, 3, -3};
  constexpr int ey[6] = {0, 2, 1, 1, 2, 0};
  bool ylds[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const int t = tid + dy[i] * ngr;
    ylds[i] = t >= 0 && t < BT && fi + dy[i] * ngr < nfl;
  }
  V win[7][3];
#pragma unroll
  for (int d = -3; d <= 2; ++d)
#pragma unroll
    for (int e = 0; e < 3; ++e) win[d + 3][e] = ldv(e, (k0 + d) * plane + cb);
  T* __restrict__ Xc = X + (long long)c * G.cs;
  const T* __restrict__ Fc = F + (long long)c * G.cs;
  const T inv = (T)(1.0 / (3.0 * kC0));
  for (int k = k0; k <= k1; ++k) {
    const int buf = k & 1;
    const long long row = k * plane + cb;
#pragma unroll
    for (int e = 0; e < 3; ++e) cen[buf][e][tid] = win[3][e];
#pragma unroll
    for (int e = 0; e < 3; ++e) win[6][e] = ldv(e, row + 3 * plane);
    V yv[6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
      if (!ylds[i]) yv[i] = ldv(ey[i], row + dy[i] * (long long)G.W);
    const V fv = *reinterpret_cast<const V*>(Fc + row);
    T lft[3], rgt[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      lft[e] = (needl && !(ZM && zero[e])) ? P[e][row - 1] : (T)0;
      rgt[e] = (needr && !(ZM && zero[e])) ? P[e][row + CPL] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 6; ++i)
      if (ylds[i]) yv[i] = cen[buf][ey[i]][tid + dy[i] * ngr];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      if (lds_l) lft[e] = cen[buf][e][tid - 1][CPL - 1];
      if (lds_r) rgt[e] = cen[buf][e][tid + 1][0];
    }
    const int q = (c - b - k - G.off) & 3;  // position of the colour-c node in each compact column
    T out[CPL];
    bool ok[CPL];
    bool all = live;
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      const int a = 4 * (m0 + i) + q;
      ok[i] = live && G.inner(a);
      all = all && ok[i];
      // slot e at compact column m0 + j (j = -1 .. CPL)
      auto colv = [&](int j, int e) -> T { return j < 0 ? lft[e] : (j >= CPL ? rgt[e] : win[3][e][j]); };
      auto xval = [&](int d, int e) -> T { return colv(((a + d) >> 2) - m0, e); };
      const T s1 = xval(1, 0) + xval(-1, 2) + yv[0][i] + yv[1][i] + win[4][0][i] + win[2][2][i];
      const T s2 = xval(2, 1) + xval(-2, 1) + yv[2][i] + yv[3][i] + win[5][1][i] + win[1][1][i];
      const T s3 = xval(3, 2) + xval(-3, 0) + yv[4][i] + yv[5][i] + win[6][2][i] + win[0][0][i];
      const T sum = (T)kC1 * s1 + (T)kC2 * s2 + (T)kC3 * s3;
      out[i] = (h2 * fv[i] - sum) * inv;
    }
    if (all) {
      V o;
#pragma unroll
      for (int i = 0; i < CPL; ++i) o[i] = out[i];
      __builtin_nontemporal_store(o, reinterpret_cast<V*>(Xc + row));
    } else {
#pragma unroll
      for (int i = 0; i < CPL; ++i)
        if (ok[i]) store_stream(Xc + row + i, out[i]);
    }
    // the next plane writes the other buffer; the plane after it waits at
    // that plane's barrier, which every lane passes only after these reads
#pragma unroll
    for (int d = 0; d < 6; ++d)
#pragma unroll
      for (int e = 0; e < 3; ++e) win[d][e] = win[d + 1][e];
  }
}

// Residual of the 19-point star for all four nodes of a compact column.  The
// register window and the LDS tile are indexed by the node's position q in
// its compact column (colour (q + shift) mod 4 of that row), so every register
// index is a compile-time constant; the colour rotation goes into the load
// and store addresses.  The tile of a plane is the window's centre plane of
// the block's rows, three halo rows above and below (loaded by the first six
// thread rows) and one halo column on each side (one cell per thread for the
// first 8 TROWS threads).  Those halo values, the right-hand sides and the
// window's next plane are loaded one plane ahead, while the current plane is
// computed from the other tile buffer, so each plane's loads are in flight
// across the barrier and the compute of the plane before.
template <typename T, typename TO>
__global__ __launch_bounds__(BX * TBY) void k_residual19s(const T* __restrict__ X, const T* __restrict__ F,
                                                          TO* __restrict__ R, Geom G, T ih2,
                                                          double* __restrict__ partial, int mbase) {
  __shared__ T tile[2][TROWS][4][TCOLS];  // double-buffered by plane parity
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * BX + tx;
  const int m0 = mbase + bx * BX;
  const int m = m0 + tx;
  const int b0 = G.g + by * TBY;
  const int b = b0 + ty;
  const int last = G.g + G.n - 2;
  const int kz = planes_per_block(G);
  const int k0 = G.g + bz * kz;
  const int k1 = min(k0 + kz - 1, last);
  const bool colok = m < G.W;
  const bool rowok = b < G.M;
  const long long plane = (long long)G.M * G.W;
  const long long cb = (long long)b * G.W + m;
  // value at position q of compact column mm in row bb of plane kk
  auto load = [&](int bb, int kk, int mm, int q) -> T {
    const int col = (q + bb + kk + G.off) & 3;
    return X[(long long)col * G.cs + kk * plane + (long long)bb * G.W + mm];
  };
  // this thread's halo row (thread rows 0..5) and halo-column cell (threads
  // 0 .. 8 TROWS - 1: position, side, tile row)
  const int hb = ty < 3 ? b0 - 3 + ty : b0 + TBY + (ty - 3);
  const int htr = ty < 3 ? ty : TBY + ty;
  const bool hrow = ty < 6 && hb >= 0 && hb < G.M && colok;
  const int cq = tid & 3, cside = (tid >> 2) & 1, ctr = tid >> 3;
  const int chb = b0 - 3 + ctr, chm = cside ? m0 + BX : m0 - 1;
  const int ctc = cside ? BX + 1 : 0;
  const bool hcell = tid < 8 * TROWS;
  const bool hcol = hcell && chb >= 0 && chb < G.M && chm >= 0 && chm < G.W;
  T win[7][4];  // win[d + 3][q] at (m, b, k + d)
#pragma unroll
  for (int d = -3; d <= 2; ++d)
#pragma unroll
    for (int q = 0; q < 4; ++q) win[d + 3][q] = (colok && rowok) ? load(b, k0 + d, m, q) : (T)0;
  const bool live = m <= G.mhi() && b <= last;
  T hr[4], hc, fq[4], wn[4];
  auto fetch = [&](int k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) hr[q] = hrow ? load(hb, k, m, q) : (T)0;
    hc = hcol ? load(chb, k, chm, cq) : (T)0;
    const int s = (b + k + G.off) & 3;
#pragma unroll
    for (int q = 0; q < 4; ++q) fq[q] = live ? F[(long long)((q + s) & 3) * G.cs + k * plane + cb] : (T)0;
#pragma unroll
    for (int q = 0; q < 4; ++q) wn[q] = (colok && rowok) ? load(b, k + 3, m, q) : (T)0;
  };
  fetch(k0);
  double acc = 0.0;
  for (int k = k0; k <= k1; ++k) {
    const int buf = k & 1;
    T fc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      win[6][q] = wn[q];
      fc[q] = fq[q];
      tile[buf][ty + 3][q][tx + 1] = win[3][q];
    }
    if (ty < 6) {
#pragma unroll
      for (int q = 0; q < 4; ++q) tile[buf][htr][q][tx + 1] = hr[q];
    }
    if (hcell) tile[buf][ctr][cq][ctc] = hc;
    __syncthreads();
    if (k < k1) fetch(k + 1);
    const int s = (b + k + G.off) & 3;
    if (live) {
      const int r0 = ty + 3;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = 4 * m + q;
        if (!G.inner(a)) continue;
        T sd[3];
#pragma unroll
        for (int d = 1; d <= 3; ++d) {
          // x: positions q +- d, possibly in the neighbouring compact column
          const int qp = q + d, qm = q - d;
          const T xp = tile[buf][r0][qp & 3][tx + 1 + (qp >> 2)];
          const T xm = tile[buf][r0][qm & 3][tx + 1 + (qm >> 2)];
          sd[d - 1] = xp + xm + tile[buf][r0 + d][q][tx + 1] + tile[buf][r0 - d][q][tx + 1] + win[3 + d][q] +
                      win[3 - d][q];
        }
        const T lap = ((T)(3.0 * kC0) * win[3][q] + (T)kC1 * sd[0] + (T)kC2 * sd[1] + (T)kC3 * sd[2]) * ih2;
        const long long idx = (long long)((q + s) & 3) * G.cs + k * plane + cb;
        const T res = fc[q] - lap;
        if (R) R[idx] = (TO)res;
        acc += (double)res * (double)res;
      }
    }
    // the next plane writes the other buffer; the plane after it waits at
    // that plane's barrier, which every thread passes only after this compute
#pragma unroll
    for (int d = 0; d < 6; ++d)
#pragma unroll
      for (int q = 0; q < 4; ++q) win[d][q] = win[d + 1][q];
  }
  if (partial) {
    const double sum = block_sum(acc);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = sum;
  }
}

// The same residual with two positions of two adjacent compact columns per
// thread: a block of 32 x 2 x TBY threads covers 64 compact columns from
// mbase (lanes of thread-y 0 own positions 0 and 1, of thread-y 1 positions 2
// and 3), so the window, right-hand side and result are moved with 16-byte
// (FP64) or 8-byte (FP32) accesses, half as many instructions as one column
// per thread.  The pair of a lane starts at an odd compact column (mbase 1),
// so the vector accesses are aligned to the element size only.  Tile and
// window as in k_residual19s, the tile's columns shifted by one so that a
// lane's pair is aligned in LDS.  Same blocks per level as the staged grid.
constexpr int VX2 = 32;                // lanes along x, two compact columns each
constexpr int TCOLS2 = 2 * VX2 + 4;    // 64 columns, one halo column each side, alignment pad
template <typename T, typename TO>
__global__ __launch_bounds__(VX2 * 2 * TBY) void k_residual19v(const T* __restrict__ X, const T* __restrict__ F,
                                                       TO* __restrict__ R, Geom G, T ih2,
                                                       double* __restrict__ partial, int mbase) {
  typedef T V __attribute__((ext_vector_type(2), aligned(sizeof(T))));
  typedef TO VO __attribute__((ext_vector_type(2), aligned(sizeof(TO))));
  __shared__ T tile[2][TROWS][4][TCOLS2];
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int tx = threadIdx.x, pp = threadIdx.y, ty = threadIdx.z;
  const int tid = tx + VX2 * (pp + 2 * ty);
  const int c0 = mbase + bx * 2 * VX2;
  const int m0 = c0 + 2 * tx;
  const int b0 = G.g + by * TBY;
  const int b = b0 + ty;
  const int last = G.g + G.n - 2;
  const int kz = planes_per_block(G);
  const int k0 = G.g + bz * kz;
  const int k1 = min(k0 + kz - 1, last);
  const bool colok = m0 + 1 < G.W;
  const bool rowok = b < G.M;
  const long long plane = (long long)G.M * G.W;
  const long long cb = (long long)b * G.W + m0;
  auto loadv = [&](int bb, int kk, int mm, int q) -> V {
    const int col = (q + bb + kk + G.off) & 3;
    return *reinterpret_cast<const V*>(X + (long long)col * G.cs + kk * plane + (long long)bb * G.W + mm);
  };
  auto load1 = [&](int bb, int kk, int mm, int q) -> T {
    const int col = (q + bb + kk + G.off) & 3;
    return X[(long long)col * G.cs + kk * plane + (long long)bb * G.W + mm];
  };
  const int q0 = 2 * pp;
  const int hb = ty < 3 ? b0 - 3 + ty : b0 + TBY + (ty - 3);
  const int htr = ty < 3 ? ty : TBY + ty;
  const bool hrow = ty < 6 && hb >= 0 && hb < G.M && colok;
  const int cq = tid & 3, cside = (tid >> 2) & 1, ctr = tid >> 3;
  const int chb = b0 - 3 + ctr, chm = cside ? c0 + 2 * VX2 : c0 - 1;
  const int ctc = cside ? 2 * VX2 + 2 : 1;
  const bool hcell = tid < 8 * TROWS;
  const bool hcol = hcell && chb >= 0 && chb < G.M && chm >= 0 && chm < G.W;
  V win[7][2];
#pragma unroll
  for (int d = -3; d <= 2; ++d)
#pragma unroll
    for (int j = 0; j < 2; ++j) win[d + 3][j] = (colok && rowok) ? loadv(b, k0 + d, m0, q0 + j) : V{};
  const bool live = b <= last && colok;
  V hr[2], fq[2], wn[2];
  T hc;
  auto fetch = [&](int k) {
#pragma unroll
    for (int j = 0; j < 2; ++j) hr[j] = hrow ? loadv(hb, k, m0, q0 + j) : V{};
    hc = hcol ? load1(chb, k, chm, cq) : (T)0;
    const int s = (b + k + G.off) & 3;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      fq[j] = live ? *reinterpret_cast<const V*>(F + (long long)((q0 + j + s) & 3) * G.cs + k * plane + cb) : V{};
#pragma unroll
    for (int j = 0; j < 2; ++j) wn[j] = (colok && rowok) ? loadv(b, k + 3, m0, q0 + j) : V{};
  };
  fetch(k0);
  double acc = 0.0;
  for (int k = k0; k <= k1; ++k) {
    const int buf = k & 1;
    V fc[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      win[6][j] = wn[j];
      fc[j] = fq[j];
      tile[buf][ty + 3][q0 + j][2 * tx + 2] = win[3][j][0];
      tile[buf][ty + 3][q0 + j][2 * tx + 3] = win[3][j][1];
    }
    if (ty < 6) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        tile[buf][htr][q0 + j][2 * tx + 2] = hr[j][0];
        tile[buf][htr][q0 + j][2 * tx + 3] = hr[j][1];
      }
    }
    if (hcell) tile[buf][ctr][cq][ctc] = hc;
    __syncthreads();
    if (k < k1) fetch(k + 1);
    const int s = (b + k + G.off) & 3;
    if (live) {
      const int r0 = ty + 3;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int q = q0 + j;
        T res[2];
        bool ok[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int a = 4 * (m0 + i) + q;
          const int tc = 2 * tx + 2 + i;
          ok[i] = G.inner(a);
          T sd[3];
#pragma unroll
          for (int d = 1; d <= 3; ++d) {
            const int qp = q + d, qm = q - d;
            const T xp = tile[buf][r0][qp & 3][tc + (qp >> 2)];
            const T xm = tile[buf][r0][qm & 3][tc + (qm >> 2)];
            sd[d - 1] = xp + xm + tile[buf][r0 + d][q][tc] + tile[buf][r0 - d][q][tc] + win[3 + d][j][i] +
                        win[3 - d][j][i];
          }
          const T lap = ((T)(3.0 * kC0) * win[3][j][i] + (T)kC1 * sd[0] + (T)kC2 * sd[1] + (T)kC3 * sd[2]) * ih2;
          res[i] = fc[j][i] - lap;
        }
        const long long idx = (long long)((q + s) & 3) * G.cs + k * plane + cb;
        if (R) {
          if (ok[0] && ok[1]) {
            VO o;
            o[0] = (TO)res[0];
            o[1] = (TO)res[1];
            *reinterpret_cast<VO*>(R + idx) = o;
          } else {
            if (ok[0]) R[idx] = (TO)res[0];
            if (ok[1]) R[idx + 1] = (TO)res[1];
          }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
          if (ok[i]) acc += (double)res[i] * (double)res[i];
      }
    }
#pragma unroll
    for (int d = 0; d < 6; ++d)
#pragma unroll
      for (int j = 0; j < 2; ++j) win[d][j] = win[d + 1][j];
  }
  if (partial) {
    const double sum = block_sum(acc);
    if (tid == 0) partial[linear_block()] = sum;
  }
}

// Residual of the 19-point star fused with full weighting onto the next
// coarser four-colour level: the coarse right-hand side without storing the
// fine residual, the squares of the fine residuals summed per block as in
// k_residual19s.  The block, tile and register window are those of
// k_residual19s, TR own rows and one more thread row: rows b0 .. b0+TR-1 are
// the block's own (their residuals enter the norm) and row b0+TR, the next
// block's first, completes the three fine rows of the block's last coarse
// row; likewise the run marches one plane past its own (b0 and the first
// plane of a run are odd, so the block's coarse centres, on even fine rows
// and planes, lie inside it).  Coarse node A sits on fine node 2A-2: per
// fine row and plane a thread restricts along x at its compact column's
// positions 0 and 2, the value left of position 0 coming from the previous
// lane.  For the first lane that value is the residual at position 3 of the
// compact column before the block: one more wavefront forms it for all the
// block's rows (lane r for row b0 + r, a window along z in registers, the
// tile's halo column) and adds compact column 0's one unknown per row and
// plane to the norm in the blocks of the first column group.  The x sums go
// to LDS and are combined along y by the threads of the even rows one plane
// later (after that plane's barrier; the first lane adds the halo residual
// there), and along z in registers.  SKIPLAST: the residuals of colour 3 are
// zero after a Gauss-Seidel pass over colour 3 and are restricted as zero
// (they still enter the norm).  Requires runs of an even number of planes
// (levels from 128 intervals).  FP64 or FP32 levels.
// TR: the block's own rows (even, so that its coarse rows are whole).
template <typename T, bool SKIPLAST, int TR>
__global__ __launch_bounds__(BX*(TR + 2)) void k_resrestrict19(const T* __restrict__ X, const T* __restrict__ F,
                                                               Geom G, T ih2, T* __restrict__ Fc, Geom Gc,
                                                               double* __restrict__ partial, int mbase) {
  constexpr int RRY = TR + 1;  // thread rows over fine rows; thread row RRY forms the halo residuals
  constexpr int RTROWS = RRY + 6;
  static_assert(TR % 2 == 0, "coarse rows whole within a block");
  static_assert(BX * RRY >= 8 * RTROWS, "one halo-column cell per thread");
  static_assert(RRY <= BX, "one halo-wavefront lane per row");
  static_assert(RRY >= 6, "thread rows 0-5 load the six halo rows");
  __shared__ T tile[2][RTROWS][4][TCOLS];
  __shared__ T srx[2][RRY][2][BX];
  __shared__ T hres[2][RRY];  // residual at position 3 of compact column m0-1, per row
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * BX + tx;
  const bool hw = ty == RRY;  // the halo wavefront
  const int m0 = mbase + bx * BX;
  const int mh = m0 - 1;
  const int m = hw ? mh : m0 + tx;
  const int b0 = G.g + by * TR;
  const int b = b0 + (hw ? tx : ty);
  const int last = G.g + G.n - 2;
  const int kz = planes_per_block(G);
  const int k0 = G.g + bz * kz;
  const int k1 = min(k0 + kz - 1, last);
  const int kend = min(k1 + 1, last);
  const bool colok = m < G.W;
  const bool rowok = b < G.M && (!hw || tx < RRY);
  const long long plane = (long long)G.M * G.W;
  const long long cb = (long long)b * G.W + m;
  auto load = [&](int bb, int kk, int mm, int q) -> T {
    const int col = (q + bb + kk + G.off) & 3;
    return X[(long long)col * G.cs + kk * plane + (long long)bb * G.W + mm];
  };
  const int hb = ty < 3 ? b0 - 3 + ty : b0 + RRY + (ty - 3);
  const int htr = ty < 3 ? ty : RRY + ty;
  const bool hrow = ty < 6 && hb >= 0 && hb < G.M && colok;
  const int cq = tid & 3, cside = (tid >> 2) & 1, ctr = tid >> 3;
  const int chb = b0 - 3 + ctr, chm = cside ? m0 + BX : m0 - 1;
  const int ctc = cside ? BX + 1 : 0;
  const bool hcell = tid < 8 * RTROWS;
  const bool hcol = hcell && chb >= 0 && chb < G.M && chm >= 0 && chm < G.W;
  // the window: four positions of the lane's compact column (the halo
  // wavefront: position 3 only, of column m0-1)
  T win[7][4];
#pragma unroll
  for (int d = -3; d <= 2; ++d)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      win[d + 3][q] = (colok && rowok && (!hw || q == 3)) ? load(b, k0 + d, m, q) : (T)0;
  const bool live = m <= G.mhi() && b <= last && rowok;
  const bool own = live && !hw && ty < TR;  // the block's own rows: their residuals enter the norm
  const bool col0 = hw && live && tx < TR && mh == 0 && G.inner(3);  // compact column 0's unknown
  const bool hlive = hw && live && G.inner(4 * mh + 3);
  T hr[4], hc, fq[4], wn[4];
  auto fetch = [&](int k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) hr[q] = hrow ? load(hb, k, m, q) : (T)0;
    hc = hcol ? load(chb, k, chm, cq) : (T)0;
    const int s = (b + k + G.off) & 3;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      fq[q] = (live && (!hw || q == 3)) ? F[(long long)((q + s) & 3) * G.cs + k * plane + cb] : (T)0;
#pragma unroll
    for (int q = 0; q < 4; ++q) wn[q] = (colok && rowok && (!hw || q == 3)) ? load(b, k + 3, m, q) : (T)0;
  };
  fetch(k0);
  const T q4 = (T)0.25, h2 = (T)0.5;
  const int Alo = Gc.g, Ahi = Gc.g + Gc.n - 2;
  const bool centre = !hw && ((b & 1) == 0) && ty > 0 && ty < RRY - 1;  // fine row 2B-2 of coarse row B
  const int B = (b + 2) >> 1;
  T acc0 = (T)0, acc2 = (T)0;
  double nrm = 0.0;
  // y weights of plane p's x sums (buffer p & 1), then z weights; a coarse
  // plane is written at its last (odd) fine plane
  auto ycombine = [&](int p) {
    if (!centre) return;
    const int pb = p & 1;
    auto sx0 = [&](int row) -> T {
      return tx == 0 ? q4 * hres[pb][row] + srx[pb][row][0][0] : srx[pb][row][0][tx];
    };
    const T ry0 = q4 * sx0(ty - 1) + h2 * sx0(ty) + q4 * sx0(ty + 1);
    const T ry2 = q4 * srx[pb][ty - 1][1][tx] + h2 * srx[pb][ty][1][tx] + q4 * srx[pb][ty + 1][1][tx];
    if (p & 1) {
      if (p > k0) {
        acc0 += q4 * ry0;
        acc2 += q4 * ry2;
        const int K = (p + 1) >> 1;
        const int A0 = 2 * m + 1, A2 = 2 * m + 2;
        if (m <= G.mhi() && B >= Alo && B <= Ahi && K >= Alo && K <= Ahi) {
          if (A0 >= Alo && A0 <= Ahi) Fc[Gc.at(A0, B, K)] = acc0;
          if (A2 >= Alo && A2 <= Ahi) Fc[Gc.at(A2, B, K)] = acc2;
        }
      }
      acc0 = q4 * ry0;
      acc2 = q4 * ry2;
    } else {
      acc0 += h2 * ry0;
      acc2 += h2 * ry2;
    }
  };
  for (int k = k0; k <= kend; ++k) {
    const int buf = k & 1;
    T fc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      win[6][q] = wn[q];
      fc[q] = fq[q];
    }
    if (!hw) {
#pragma unroll
      for (int q = 0; q < 4; ++q) tile[buf][ty + 3][q][tx + 1] = win[3][q];
    }
    if (ty < 6) {
#pragma unroll
      for (int q = 0; q < 4; ++q) tile[buf][htr][q][tx + 1] = hr[q];
    }
    if (hcell) tile[buf][ctr][cq][ctc] = hc;
    __syncthreads();
    if (k < kend) fetch(k + 1);
    if (k > k0) ycombine(k - 1);
    const int s = (b + k + G.off) & 3;
    // staged-order 19-point residual at position q of the tile column tc, row r0
    auto res_at = [&](int r0, int q, int tc, const T* w, T f) -> T {
      T sd[3];
#pragma unroll
      for (int d = 1; d <= 3; ++d) {
        const int qp = q + d, qm = q - d;
        const T xp = tile[buf][r0][qp & 3][tc + (qp >> 2)];
        const T xm = tile[buf][r0][qm & 3][tc + (qm >> 2)];
        sd[d - 1] = xp + xm + tile[buf][r0 + d][q][tc] + tile[buf][r0 - d][q][tc] + w[3 + d] + w[3 - d];
      }
      const T lap = ((T)(3.0 * kC0) * w[3] + (T)kC1 * sd[0] + (T)kC2 * sd[1] + (T)kC3 * sd[2]) * ih2;
      return f - lap;
    };
    if (hw) {
      if (tx < RRY) {
        T rh = (T)0;
        if (hlive) {
          T w[7];
#pragma unroll
          for (int d = 0; d < 7; ++d) w[d] = win[d][3];
          rh = res_at(tx + 3, 3, 0, w, fc[3]);
          if (col0 && k <= k1) nrm += (double)rh * (double)rh;
          if (SKIPLAST && ((3 + s) & 3) == 3) rh = (T)0;
        }
        hres[buf][tx] = rh;
      }
    } else {
      T r[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        r[q] = (T)0;
        if (live && G.inner(4 * m + q)) {
          T w[7];
#pragma unroll
          for (int d = 0; d < 7; ++d) w[d] = win[d][q];
          r[q] = res_at(ty + 3, q, tx + 1, w, fc[q]);
          if (own && k <= k1) nrm += (double)r[q] * (double)r[q];
        }
        if (SKIPLAST && ((q + s) & 3) == 3) r[q] = (T)0;
      }
      const T left = __shfl_up(r[3], 1, 64);
      // the first lane's halo term is added when its rows are combined
      srx[buf][ty][0][tx] = tx == 0 ? h2 * r[0] + q4 * r[1] : q4 * left + h2 * r[0] + q4 * r[1];
      srx[buf][ty][1][tx] = q4 * r[1] + h2 * r[2] + q4 * r[3];
    }
#pragma unroll
    for (int d = 0; d < 6; ++d)
#pragma unroll
      for (int q = 0; q < 4; ++q) win[d][q] = win[d + 1][q];
  }
  __syncthreads();
  ycombine(kend);
  if (partial) {
    const double sum = block_sum(nrm);
    if (tid == 0) partial[linear_block()] = sum;
  }
}

// Residuals of the unknowns in compact column 0 of a four-colour level (node
// a = 3, the blocks of the staged kernels start at column 1): one thread per
// (row, plane); partial sums of r^2 per block go to partial[pbase + block].
// ZU: the unknowns of u are taken as zero.
template <typename T, typename TO, bool ZU>
__global__ __launch_bounds__(256) void k_res19_col0(const T* __restrict__ X, const T* __restrict__ F,
                                                    TO* __restrict__ R, Geom G, T ih2, double* __restrict__ partial,
                                                    unsigned pbase) {
  const int E = G.n - 1;
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (t < (long long)E * E) {
    const int b = G.g + (int)(t % E);
    const int k = G.g + (int)(t / E);
    const int a = 3;  // the only unknown of column 0 (three ghost layers)
    const long long idx = G.at(a, b, k);
    // the staged kernels' order of terms: x+d, x-d, y+d, y-d, z+d, z-d
    auto v = [&](int aa, int bb, int kk) -> T {
      if (ZU && G.inner(aa) && G.inner(bb) && G.inner(kk)) return (T)0;
      return X[G.at(aa, bb, kk)];
    };
    T sd[3];
#pragma unroll
    for (int d = 1; d <= 3; ++d)
      sd[d - 1] = v(a + d, b, k) + v(a - d, b, k) + v(a, b + d, k) + v(a, b - d, k) + v(a, b, k + d) + v(a, b, k - d);
    const T lap = ((T)(3.0 * kC0) * v(a, b, k) + (T)kC1 * sd[0] + (T)kC2 * sd[1] + (T)kC3 * sd[2]) * ih2;
    const T res = F[idx] - lap;
    if (R) R[idx] = (TO)res;
    acc = (double)res * (double)res;
  }
  if (partial) {
    const double sum = block_sum(acc);
    if (threadIdx.x == 0) partial[pbase + blockIdx.x] = sum;
  }
}

// ---------------------------------------------------------------- residual
// r = f - L u for every unknown.  One thread handles the C consecutive nodes
// a = C*m .. C*m+C-1 of row (b, k) and marches KZ planes.  In a row whose
// colour shift is s = (b + k + off) mod C, the node at position q of any
// compact column has colour (q + s) mod C, so per row the thread builds the
// C colour pointers rotated by s once and then indexes them with compile-time
// positions.  Partial sums of r^2 (in FP64) per block when partial != nullptr;
// ZU treats the unknowns of u as zero (norm of b).
template <typename T, typename TO, int ORDER, bool ZU>
__global__ __launch_bounds__(512) void k_residual(const T* __restrict__ X, const T* __restrict__ F,
                                                  TO* __restrict__ R, Geom G, T ih2,
                                                  double* __restrict__ partial, int mbase) {
  constexpr int C = ORDER == 2 ? 2 : 4;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = mbase + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * (int)blockDim.y + (int)threadIdx.y;  // launched with 4 or 8 rows per block
  const int last = G.g + G.n - 2;
  double acc = 0.0;
  if (m <= G.mhi() && b <= last) {
    const int kz = planes_per_block(G);
    const int k0 = G.g + bz * kz;
    const int k1 = min(k0 + kz - 1, last);
    const bool bin = G.inner(b);
    for (int k = k0; k <= k1; ++k) {
      const int s = (b + k + G.off) & (C - 1);
      const T* P[C];
#pragma unroll
      for (int q = 0; q < C; ++q) P[q] = X + (long long)((q + s) & (C - 1)) * G.cs;
      const long long row = G.row(b, k);
      // centre row: positions a' = C*(m+t) + q for t = -1, 0, 1
      T ext[3 * C];
#pragma unroll
      for (int t = -1; t <= 1; ++t)
#pragma unroll
        for (int q = 0; q < C; ++q) {
          const int a2 = C * (m + t) + q;
          T v = (T)0;
          if (a2 >= 0 && a2 < G.M && !(ZU && G.inner(a2) && bin && G.inner(k))) v = P[q][row + m + t];
          ext[(t + 1) * C + q] = v;
        }
#pragma unroll
      for (int q = 0; q < C; ++q) {
        const int a = C * m + q;
        if (!G.inner(a)) continue;
        const int e = C + q;
        T lap;
        if (ORDER == 2) {
          // y / z neighbours sit at the same a with colour (q + s + 1) mod 2;
          // with ZU only those that are ghost nodes contribute
          const T* Po = P[(q + 1) & 1];
          T sy = (T)0;
          if (!ZU || !G.inner(b - 1)) sy += Po[G.row(b - 1, k) + m];
          if (!ZU || !G.inner(b + 1)) sy += Po[G.row(b + 1, k) + m];
          if (!ZU || !G.inner(k - 1)) sy += Po[G.row(b, k - 1) + m];
          if (!ZU || !G.inner(k + 1)) sy += Po[G.row(b, k + 1) + m];
          const T sx = ext[e - 1] + ext[e + 1];
          lap = ((sx + sy) - (T)6 * ext[e]) * ih2;
        } else {
          T sd[3];
#pragma unroll
          for (int d = 1; d <= 3; ++d) {
            const T* Pp = P[(q + d) & 3];
            const T* Pm = P[(q - d) & 3];
            T v = ext[e - d] + ext[e + d];
            const bool gy_m = !G.inner(b - d), gy_p = !G.inner(b + d);
            const bool gz_m = !G.inner(k - d), gz_p = !G.inner(k + d);
            if (!ZU || gy_p) v += Pp[G.row(b + d, k) + m];
            if (!ZU || gy_m) v += Pm[G.row(b - d, k) + m];
            if (!ZU || gz_p) v += Pp[G.row(b, k + d) + m];
            if (!ZU || gz_m) v += Pm[G.row(b, k - d) + m];
            sd[d - 1] = v;
          }
          lap = ((T)(3.0 * kC0) * ext[e] + (T)kC1 * sd[0] + (T)kC2 * sd[1] + (T)kC3 * sd[2]) * ih2;
        }
        const long long idx = (long long)((q + s) & (C - 1)) * G.cs + row + m;
        const T res = F[idx] - lap;
        if (R) R[idx] = (TO)res;
        acc += (double)res * (double)res;
      }
    }
  }
  if (partial) {
    const double sum = block_sum(acc);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = sum;
  }
}

// 7-point residual (no zero-unknown option): the thread owns the two nodes
// a = 2m (colour s) and a = 2m+1 (colour 1-s) of row (b, k) for KZP
// consecutive planes.  Both colours' values at compact m are loaded once per
// plane (z0, z1: centre values and z-neighbours); each plane adds two
// x-neighbour loads, four y-neighbour loads and the two right-hand sides.  As
// in the colour pass, the loop is unrolled at compile time, load indices past
// k1 are clamped into the array and only the stores and sums are predicated,
// so the loads of all planes can be in flight together.  COL >= 0: only the
// nodes of colour COL (the other colour's residual is known to vanish, e.g.
// right after a Gauss-Seidel pass over it), with only their neighbour and
// right-hand-side loads.
template <typename T, typename TO, int KZP, int COL>
__global__ __launch_bounds__(256) void k_residual7(const T* __restrict__ X, const T* __restrict__ F,
                                                   TO* __restrict__ R, Geom G, T ih2,
                                                   double* __restrict__ partial) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  double acc = 0.0;
  if (m <= G.mhi() && b <= last) {
    const int kz = planes_per_block(G);
    const int k0 = G.g + bz * kz;
    const int k1 = min(k0 + kz - 1, last);
    const long long plane = (long long)G.M * G.W;
    const long long W = G.W;
    const long long q0 = G.row(b, 0) + m;  // (m, b) on plane 0
    const T* __restrict__ x0 = X + q0;
    const T* __restrict__ x1 = X + G.cs + q0;
    // planes in chunks of CH: a chunk's loads are issued together (FP64:
    // four planes, so that the values in flight stay within the registers)
    constexpr int CH = sizeof(T) == 8 ? (KZP < 4 ? KZP : 4) : KZP;
    T z0[KZP + 2], z1[KZP + 2];
    T xl[KZP], xr[KZP], ya0[KZP], ya1[KZP], yb0[KZP], yb1[KZP], fa[KZP], fb[KZP];
    const bool inA = G.inner(2 * m), inB = G.inner(2 * m + 1);
#pragma unroll
    for (int c0 = 0; c0 < KZP; c0 += CH) {
#pragma unroll
      for (int t = (c0 == 0 ? 0 : c0 + 2); t < c0 + CH + 2; ++t) {
        const long long o = (long long)min(k0 - 1 + t, k1 + 1) * plane;
        z0[t] = x0[o];
        z1[t] = x1[o];
      }
#pragma unroll
      for (int t = c0; t < c0 + CH; ++t) {
        const int k = min(k0 + t, k1);
        const long long o = (long long)k * plane;
        const long long sa = (long long)((b + k + G.off) & 1) * G.cs;  // colour of A = 2m
        const long long sb = G.cs - sa;                                 // colour of B = 2m+1
        const bool doA = COL < 0 || ((b + k + G.off) & 1) == COL;
        if (doA) {
          xl[t] = X[sb + q0 + o - 1];  // A's left neighbour (B's colour)
          yb0[t] = X[sb + q0 + o - W];
          yb1[t] = X[sb + q0 + o + W];
          fa[t] = F[sa + q0 + o];
        }
        if (COL < 0 || !doA) {
          xr[t] = X[sa + q0 + o + 1];  // B's right neighbour (A's colour)
          ya0[t] = X[sa + q0 + o - W];
          ya1[t] = X[sa + q0 + o + W];
          fb[t] = F[sb + q0 + o];
        }
      }
#pragma unroll
      for (int t = c0; t < c0 + CH; ++t) {
        const int k = k0 + t;
        if (k <= k1) {
          const int s = (b + k + G.off) & 1;
          const long long o = (long long)k * plane;
          const T uA = s ? z1[t + 1] : z0[t + 1], uB = s ? z0[t + 1] : z1[t + 1];
          // z-neighbours of A have B's colour and vice versa
          const T zbA = s ? z0[t] + z0[t + 2] : z1[t] + z1[t + 2];
          const T zbB = s ? z1[t] + z1[t + 2] : z0[t] + z0[t + 2];
          if (inA && (COL < 0 || s == COL)) {
            const T sx = xl[t] + uB;
            const T sy = yb0[t] + yb1[t] + zbA;
            const T res = fa[t] - ((sx + sy) - (T)6 * uA) * ih2;
            if (R) R[(long long)s * G.cs + q0 + o] = (TO)res;
            acc += (double)res * (double)res;
          }
          if (inB && (COL < 0 || s != COL)) {
            const T sx = uA + xr[t];
            const T sy = ya0[t] + ya1[t] + zbB;
            const T res = fb[t] - ((sx + sy) - (T)6 * uB) * ih2;
            if (R) R[(long long)(s ^ 1) * G.cs + q0 + o] = (TO)res;
            acc += (double)res * (double)res;
          }
        }
      }
    }
  }
  if (partial) {
    const double sum = block_sum(acc);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = sum;
  }
}

// ---------------------------------------------------------------- transfers
// Full weighting on the two-colour layout, marching along z.  A thread
// owns one fine compact column m of the fine rows 2B-sh-1 .. 2B-sh+1 of one
// coarse row B (sh = g - 1; coarse node A sits on fine node 2A - sh) and the
// coarse planes of its run.  Per fine row and plane it loads the C values of
// its column (position q lives in colour array (q + row + plane + off) mod C)
// and forms the x-weighted sums at the coarse positions of the column (q even)
// with the left column's last value from the neighbouring lane; the y weights
// combine its three rows, and the z weights combine consecutive fine planes,
// the last of one coarse plane being the first of the next.
template <typename T, int C>
__global__ __launch_bounds__(256) void k_restrict_z(const T* __restrict__ Rf, Geom Gf, T* __restrict__ Fc, Geom Gc) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int sh = Gf.g - 1;
  const int gc = Gc.g, nc = Gc.n;
  const int Alo = gc, Ahi = gc + nc - 2;  // inner coarse nodes per axis
  const int m_first = (2 * Alo - sh) / C, m_last = (2 * Ahi - sh) / C;
  const int lane = threadIdx.x;
  const int m = m_first + bx * 64 + lane;
  const int B = Alo + by * 4 + (int)threadIdx.y;
  const int kz = (nc - 1 + (int)gridDim.z - 1) / (int)gridDim.z;
  const int K0 = Alo + bz * kz;
  const int K1 = min(K0 + kz - 1, Ahi);
  const bool live = m <= m_last && B <= Ahi;
  const int mm = min(m, m_last);  // idle lanes of a partial wavefront load a valid column
  const int Bc = min(B, Ahi);
  const long long fplane = (long long)Gf.M * Gf.W;
  const int b = 2 * Bc - sh;
  const T q4 = (T)0.25, h2 = (T)0.5;
  // x-weighted sums at the column's coarse positions (q = 0, 2, ... < C) of
  // fine row j, plane p
  auto xrow = [&](int j, int p, T* rx) {
    const int sft = (j + p + Gf.off) & (C - 1);
    const long long ro = (long long)p * fplane + (long long)j * Gf.W;
    T v[C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
      const int col = (q + sft) & (C - 1);
      v[q] = Rf[(long long)col * Gf.cs + ro + mm];
    }
    T left = __shfl_up(v[C - 1], 1, 64);
    if (lane == 0) {
      const int col = (C - 1 + sft) & (C - 1);
      left = Rf[(long long)col * Gf.cs + ro + mm - 1];
    }
#pragma unroll
    for (int q = 0; q < C; q += 2) rx[q / 2] = q4 * (q == 0 ? left : v[q - 1]) + h2 * v[q] + q4 * v[q + 1];
  };
  constexpr int NQ = C / 2;
  auto yplane = [&](int p, T* ry) {
    T r0[NQ], r1[NQ], r2[NQ];
    xrow(b - 1, p, r0);
    xrow(b, p, r1);
    xrow(b + 1, p, r2);
#pragma unroll
    for (int i = 0; i < NQ; ++i) ry[i] = q4 * r0[i] + h2 * r1[i] + q4 * r2[i];
  };
  if (K0 > K1) return;
  T prev[NQ];
  yplane(2 * K0 - sh - 1, prev);
  for (int K = K0; K <= K1; ++K) {
    T mid[NQ], nxt[NQ];
    yplane(2 * K - sh, mid);
    yplane(2 * K - sh + 1, nxt);
    if (live) {
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const int A = (C * m + 2 * i + sh) / 2;
        if (A >= Alo && A <= Ahi) Fc[Gc.at(A, B, K)] = q4 * prev[i] + h2 * mid[i] + q4 * nxt[i];
      }
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) prev[i] = nxt[i];
  }
}

// Full weighting on the four-colour levels (three ghost layers).  A lane
// owns CPL consecutive compact columns m0 .. m0+CPL-1 (groups aligned to
// CPL, 16-byte loads) of the fine rows 2B-3 .. 2B-1 of one coarse row B, and
// the coarse planes of its run; lanes are numbered over (column group, coarse
// row) pairs.  Per fine row and plane it loads the four positions of its
// columns (position q of a row with colour shift s lives in colour array
// (q + s) mod 4) and forms the x-weighted sums at the coarse positions q = 0
// and 2 of each column, the value left of the first column coming from the
// previous lane when it holds the previous group of the same row, and loaded
// otherwise; y and z weights as in the two-colour kernel.  SKIPLAST: the
// residuals of colour 3 vanish (a Gauss-Seidel pass over that colour came
// last) and are not loaded.
template <typename T, int CPL, bool SKIPLAST>
__global__ __launch_bounds__(256) void k_restrict4(const T* __restrict__ Rf, Geom Gf, T* __restrict__ Fc, Geom Gc) {
  typedef typename VecOf<T, CPL>::type V;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  constexpr int sh = 2;
  constexpr int NO = 2 * CPL;  // coarse positions per lane
  const int Alo = Gc.g, Ahi = Gc.g + Gc.n - 2;
  const int gf = ((2 * Alo - sh) >> 2) / CPL;
  const int ngr = ((2 * Ahi - sh) >> 2) / CPL - gf + 1;
  const int nB = Ahi - Alo + 1;
  const int fi = bx * 256 + (int)threadIdx.x;
  const bool live = fi < ngr * nB;
  const int fl = live ? fi : ngr * nB - 1;  // idle lanes mirror the last pair (loads stay in the array)
  const int gp = fl % ngr;
  const int B = Alo + fl / ngr;
  const int m0 = (gf + gp) * CPL;
  const int kz = (Gc.n - 1 + (int)gridDim.z - 1) / (int)gridDim.z;
  const int K0 = Alo + bz * kz;
  const int K1 = min(K0 + kz - 1, Ahi);
  const long long fplane = (long long)Gf.M * Gf.W;
  const int b = 2 * B - sh;
  const T q4 = (T)0.25, h2 = (T)0.5;
  const bool left_lane = gp > 0 && (threadIdx.x & 63) > 0;
  const bool left_load = !left_lane && m0 >= 1;
  // x-weighted sums at the lane's coarse positions of fine row j, plane p
  auto xrow = [&](int j, int p, T* rx) {
    const int sft = (j + p + Gf.off) & 3;
    const long long ro = (long long)p * fplane + (long long)j * Gf.W + m0;
    V v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = (q + sft) & 3;
      v[q] = (SKIPLAST && col == 3) ? V{} : *reinterpret_cast<const V*>(Rf + (long long)col * Gf.cs + ro);
    }
    T left = __shfl_up(v[3][CPL - 1], 1, 64);
    if (!left_lane) {
      const int col = (3 + sft) & 3;
      left = (left_load && !(SKIPLAST && col == 3)) ? Rf[(long long)col * Gf.cs + ro - 1] : (T)0;
    }
#pragma unroll
    for (int jj = 0; jj < CPL; ++jj) {
      const T l = jj == 0 ? left : v[3][jj - 1];
      rx[2 * jj] = q4 * l + h2 * v[0][jj] + q4 * v[1][jj];
      rx[2 * jj + 1] = q4 * v[1][jj] + h2 * v[2][jj] + q4 * v[3][jj];
    }
  };
  auto yplane = [&](int p, T* ry) {
    T r0[NO], r1[NO], r2[NO];
    xrow(b - 1, p, r0);
    xrow(b, p, r1);
    xrow(b + 1, p, r2);
#pragma unroll
    for (int i = 0; i < NO; ++i) ry[i] = q4 * r0[i] + h2 * r1[i] + q4 * r2[i];
  };
  if (K0 > K1) return;
  T prev[NO];
  yplane(2 * K0 - sh - 1, prev);
  for (int K = K0; K <= K1; ++K) {
    T mid[NO], nxt[NO];
    yplane(2 * K - sh, mid);
    yplane(2 * K - sh + 1, nxt);
    if (live) {
#pragma unroll
      for (int i = 0; i < NO; ++i) {
        const int A = (4 * m0 + 2 * i + sh) / 2;
        if (A >= Alo && A <= Ahi) Fc[Gc.at(A, B, K)] = q4 * prev[i] + h2 * mid[i] + q4 * nxt[i];
      }
    }
#pragma unroll
    for (int i = 0; i < NO; ++i) prev[i] = nxt[i];
  }
}

// Residual of the 7-point operator fused with full-weighting restriction:
// f_c = R (f - L phi) on the inner coarse nodes, without storing the fine
// residual.  Only for one ghost layer and two colours (fine node a of compact
// column m is 2m or 2m+1, coarse node A sits on fine node 2A).
//
// A block spans every compact column of the level (blockDim.x = BXR >= n/2,
// so levels up to 256 intervals)
// and 2 TYC + 1 fine rows 2 B0 - 1 + ty, i.e. the rows of TYC coarse rows
// B0 .. B0 + TYC - 1 (the last fine row is recomputed by the next block), and
// marches fine planes 2 K0 - 1 .. 2 K1 + 1 for KZC coarse planes.  Per fine
// plane each thread forms the residuals of its two nodes 2m, 2m+1 (as in the
// residual kernel) and restricts along x with its left neighbour's odd
// residual from LDS, rx = r(2m)/2 + (r(2m-1) + r(2m+1))/4; the centre fine row
// of each coarse row then restricts along y from the rows above and below,
// and the z weights 1/4, 1/2, 1/4 accumulate in registers; a coarse plane is
// written when its last fine plane is done.  The loads of the next fine plane
// are issued before the current one's LDS stages, all loads are clamped into
// the array, and rows or nodes outside the unknowns contribute zero.  R0:
// the colour-1 residuals are known to vanish (the level was just swept by a
// Gauss-Seidel pass over colour 1), so only colour-0 residuals are formed and
// only their neighbours and right-hand sides are loaded.
template <typename T, int BXR, int TYC, int KZC, bool R0>
__global__ __launch_bounds__(BXR*(2 * TYC + 1)) void k_resrestrict7(const T* __restrict__ X,
                                                                    const T* __restrict__ F, Geom Gf,
                                                                    T* __restrict__ Fc, Geom Gc, T ih2) {
  constexpr int TYF = 2 * TYC + 1;
  __shared__ T s_odd[2][TYF][BXR];
  __shared__ T s_rx[2][TYF][BXR];
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int n = Gf.n;            // fine intervals; unknowns 1..n-1 (g = 1)
  const int nc = Gc.n;           // coarse intervals
  const int B0 = 1 + by * TYC;
  const int K0 = 1 + bz * KZC;
  const int K1 = min(K0 + KZC - 1, nc - 1);
  const int m = tx;                            // compact column (mlo = 0 for g = 1)
  const int b = 2 * B0 - 1 + ty;               // fine row
  const bool rowok = b <= n - 1 && m <= Gf.mhi();
  const int bl = min(b, n - 1);                // row used for (discarded) loads
  const int ml = min(m, Gf.mhi());
  const long long plane = (long long)Gf.M * Gf.W;
  const long long W = Gf.W;
  const long long q0 = (long long)bl * W + ml;  // (m, b) on plane 0
  const T* __restrict__ x0 = X + q0;
  const T* __restrict__ x1 = X + Gf.cs + q0;
  const bool inA = rowok && Gf.inner(2 * m), inB = rowok && Gf.inner(2 * m + 1);
  const int kf0 = 2 * K0 - 1, kf1 = 2 * K1 + 1;
  // loads of plane k: the z-window's next centre values (plane k+1) and the
  // neighbours / right-hand sides of plane k
  struct Ld {
    T hi0, hi1, xl, xr, ya0, ya1, yb0, yb1, fa, fb;
  };
  auto load = [&](int k) {
    Ld v{};
    const long long oz = (long long)min(k + 1, n) * plane;
    v.hi0 = x0[oz];
    v.hi1 = x1[oz];
    const long long o = (long long)k * plane;
    const long long sa = (long long)((bl + k + Gf.off) & 1) * Gf.cs;  // colour of node 2m
    const long long sb = Gf.cs - sa;
    if (!R0 || sa == 0) {
      v.xl = X[sb + q0 + o - 1];
      v.yb0 = X[sb + q0 + o - W];
      v.yb1 = X[sb + q0 + o + W];
      v.fa = F[sa + q0 + o];
    }
    if (!R0 || sa != 0) {
      v.xr = X[sa + q0 + o + 1];
      v.ya0 = X[sa + q0 + o - W];
      v.ya1 = X[sa + q0 + o + W];
      v.fb = F[sb + q0 + o];
    }
    return v;
  };
  T lo0 = x0[(long long)(kf0 - 1) * plane], lo1 = x1[(long long)(kf0 - 1) * plane];
  T cu0 = x0[(long long)kf0 * plane], cu1 = x1[(long long)kf0 * plane];
  Ld cur = load(kf0);
  T acc = (T)0;
  const bool centre = (ty & 1) && (B0 + (ty >> 1)) <= nc - 1;  // fine row 2B of coarse row B
  const bool outx = m >= 1 && m <= nc - 1;                      // coarse column A = m inner
  const T q = (T)0.25, hf = (T)0.5;
  for (int k = kf0; k <= kf1; ++k) {
    const Ld nxt = load(min(k + 1, kf1));
    const int s = (bl + k + Gf.off) & 1;
    const T uA = s ? cu1 : cu0, uB = s ? cu0 : cu1;
    T rA = (T)0, rB = (T)0;
    if (inA && (!R0 || s == 0)) {
      const T sx = cur.xl + uB;
      const T sy = cur.yb0 + cur.yb1 + (s ? lo0 + cur.hi0 : lo1 + cur.hi1);
      rA = cur.fa - ((sx + sy) - (T)6 * uA) * ih2;
    }
    if (inB && (!R0 || s != 0)) {
      const T sx = uA + cur.xr;
      const T sy = cur.ya0 + cur.ya1 + (s ? lo1 + cur.hi1 : lo0 + cur.hi0);
      rB = cur.fb - ((sx + sy) - (T)6 * uB) * ih2;
    }
    const int buf = k & 1;
    s_odd[buf][ty][tx] = rB;
    __syncthreads();
    const T left = tx > 0 ? s_odd[buf][ty][tx - 1] : (T)0;
    s_rx[buf][ty][tx] = hf * rA + q * (left + rB);
    __syncthreads();
    if (centre) {
      const T ry = hf * s_rx[buf][ty][tx] + q * (s_rx[buf][ty - 1][tx] + s_rx[buf][ty + 1][tx]);
      if (k & 1) {
        // odd fine plane 2K+1: closes coarse plane K (unless k = kf0) and opens K+1
        acc += q * ry;
        const int K = (k - 1) >> 1;
        if (k > kf0 && outx) Fc[Gc.at(m, B0 + (ty >> 1), K)] = acc;
        acc = q * ry;
      } else {
        acc += hf * ry;
      }
    }
    lo0 = cu0;
    lo1 = cu1;
    cu0 = cur.hi0;
    cu1 = cur.hi1;
    cur = nxt;
  }
}

template <typename T, int BXR, int TYC, int KZC>
static void resrestrict7_go(const T* phi, const T* f, const Geom& Gf, T* fc, const Geom& Gc, bool r0,
                            hipStream_t st) {
  const int nc = Gc.n;
  const T ih2 = (T)(1.0 / (Gf.h * Gf.h));
  const dim3 grid(1, (nc - 1 + TYC - 1) / TYC, (nc - 1 + KZC - 1) / KZC), blk(BXR, 2 * TYC + 1);
  if (r0)
    k_resrestrict7<T, BXR, TYC, KZC, true><<<grid, blk, 0, st>>>(phi, f, Gf, fc, Gc, ih2);
  else
    k_resrestrict7<T, BXR, TYC, KZC, false><<<grid, blk, 0, st>>>(phi, f, Gf, fc, Gc, ih2);
}

// Large levels: several coarse rows and planes per block (little recomputed
// halo); small levels: one coarse row and plane per block (short dependent
// chains, many blocks).
template <typename T>
static void resrestrict7_t(const T* phi, const T* f, const Geom& Gf, T* fc, const Geom& Gc, bool r0,
                           hipStream_t st) {
  const int mc = Gf.mhi() + 1;
  if (mc <= 32)
    resrestrict7_go<T, 64, 1, 1>(phi, f, Gf, fc, Gc, r0, st);
  else if (mc <= 64)
    resrestrict7_go<T, 64, 1, 4>(phi, f, Gf, fc, Gc, r0, st);
  else
    resrestrict7_go<T, 128, 2, 4>(phi, f, Gf, fc, Gc, r0, st);
}

// Four-colour (19-point hierarchy, three ghost layers) prolongation: a lane
// owns CPL consecutive compact columns m0 .. m0+CPL-1 of one fine row (groups
// aligned to CPL over the columns 0 .. mhi, lanes numbered over (group, row)
// pairs) and marches fine planes.  Its 4 CPL fine nodes 4 m0 + p sit at
// coarse x-index 2 m0 + ((p - 2) >> 1) + 2, halfway to the next coarse node
// when p is odd, so one coarse row of a coarse plane contributes the 2 CPL + 1
// consecutive coarse nodes from 2 m0 + 1; the interpolated values of a coarse
// plane (along x, and along y when the fine row is odd) are formed once and
// kept for the two or three fine planes that use them.  The correction is a
// 16-byte read-modify-write per colour array; nodes outside the unknowns are
// written back unchanged.  SKIP3: colour 3 is not corrected (the following
// Gauss-Seidel pass over colour 3 reads no colour-3 value and overwrites it).
template <typename T, int CPL, bool SKIP3>
__global__ __launch_bounds__(256) void k_prolong4(const T* __restrict__ Ec, Geom Gc, T* __restrict__ Xf, Geom Gf) {
  typedef typename VecOf<T, CPL>::type V;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  constexpr int sh = 2;
  constexpr int NP = 4 * CPL;      // fine nodes of the lane's columns
  constexpr int NC = 2 * CPL + 1;  // coarse nodes of one coarse row they use
  const int ngr = col_groups<CPL>(Gf);
  const int E = Gf.n - 1;
  const int fi = bx * 256 + (int)threadIdx.x;
  if (fi >= ngr * E) return;
  const int m0 = (fi % ngr) * CPL;
  const int b = Gf.g + fi / ngr;
  const int last = Gf.g + Gf.n - 2;
  const int kz = planes_per_block(Gf);
  const int k0 = Gf.g + bz * kz;
  const int k1 = min(k0 + kz - 1, last);
  const int j = b - sh;
  const int J = (j >> 1) + sh, oj = j & 1;
  const T half = (T)0.5;
  bool in[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) in[p] = Gf.inner(4 * m0 + p);
  const int I0 = 2 * m0 + ((0 - sh) >> 1) + sh;
  auto plane_vals = [&](int L, T* v) {
#pragma unroll
    for (int p = 0; p < NP; ++p) v[p] = (T)0;
    for (int db = 0; db <= oj; ++db) {
      const int Bc = J + db;
      const int sc = Bc + L + Gc.off;
      const long long crow = Gc.row(Bc, L);
      const T wy = oj ? half : (T)1;
      T c[NC];
#pragma unroll
      for (int t = 0; t < NC; ++t) {
        const int I = min(I0 + t, Gc.M - 1);  // nodes past the array only feed non-unknowns
        c[t] = Ec[(long long)((I + sc) & 3) * Gc.cs + crow + (I >> 2)];
      }
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int t = ((p - sh) >> 1) - ((0 - sh) >> 1);
        T x = c[t];
        if ((p - sh) & 1) x = half * (x + c[t + 1]);
        v[p] += wy * x;
      }
    }
  };
  int Lc = ((k0 - sh) >> 1) + sh;
  T cv[NP], nv[NP];
  plane_vals(Lc, cv);
  plane_vals(Lc + 1, nv);
  for (int k = k0; k <= k1; ++k) {
    const int l = k - sh;
    const int L = (l >> 1) + sh;
    if (L != Lc) {  // one coarse plane further
#pragma unroll
      for (int p = 0; p < NP; ++p) cv[p] = nv[p];
      Lc = L;
      plane_vals(L + 1, nv);
    }
    const int s = (b + k + Gf.off) & 3;
    const long long row = Gf.row(b, k) + m0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = (q + s) & 3;
      if (SKIP3 && col == 3) continue;
      V* x = reinterpret_cast<V*>(Xf + (long long)col * Gf.cs + row);
      V v = *x;
#pragma unroll
      for (int jj = 0; jj < CPL; ++jj) {
        const int p = 4 * jj + q;
        if (in[p]) v[jj] += (l & 1) ? half * (cv[p] + nv[p]) : cv[p];
      }
      *x = v;
    }
  }
}

// Two-colour (7-point hierarchy, one ghost layer) prolongation: the fine
// nodes 2m and 2m+1 of a row need the coarse values at coarse columns m and
// m+1 of one or two coarse rows on one or two coarse planes; the coarse plane
// values are cached in registers while the thread marches fine planes.  C0:
// only colour-0 nodes are corrected (a Gauss-Seidel pass over colour 1,
// which reads no colour-1 value, follows and overwrites the rest).
template <typename T, bool C0>
__global__ __launch_bounds__(256) void k_prolong2(const T* __restrict__ Ec, Geom Gc, T* __restrict__ Xf, Geom Gf) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = Gf.mlo() + bx * BX + (int)threadIdx.x;
  const int b = Gf.g + by * BY + (int)threadIdx.y;
  const int last = Gf.g + Gf.n - 2;
  if (m > Gf.mhi() || b > last) return;
  const int kz = planes_per_block(Gf);
  const int k0 = Gf.g + bz * kz;
  const int k1 = min(k0 + kz - 1, last);
  const int J = b >> 1, oj = b & 1;
  const T half = (T)0.5;
  const bool inA = Gf.inner(2 * m), inB = Gf.inner(2 * m + 1);
  // coarse value pair (column m, column m+1) of coarse row Bc on plane K,
  // already interpolated along y when oj = 1
  auto plane_vals = [&](int K, T& vm, T& vp) {
    T am, ap;
    {
      const int sc = (m + J + K + Gc.off) & 1;
      const long long crow = Gc.row(J, K);
      am = Ec[(long long)sc * Gc.cs + crow + (m >> 1)];
      ap = Ec[(long long)(sc ^ 1) * Gc.cs + crow + ((m + 1) >> 1)];
    }
    if (oj) {
      const int sc = (m + J + 1 + K + Gc.off) & 1;
      const long long crow = Gc.row(J + 1, K);
      am = half * (am + Ec[(long long)sc * Gc.cs + crow + (m >> 1)]);
      ap = half * (ap + Ec[(long long)(sc ^ 1) * Gc.cs + crow + ((m + 1) >> 1)]);
    }
    vm = am;
    vp = ap;
  };
  int Kc = k0 >> 1;
  T cm, cp, nm = (T)0, np = (T)0;
  bool have_next = false;
  plane_vals(Kc, cm, cp);
  for (int k = k0; k <= k1; ++k) {
    const int L = k >> 1;
    if (L != Kc) {  // advanced one coarse plane
      if (have_next) {
        cm = nm;
        cp = np;
      } else {
        plane_vals(L, cm, cp);
      }
      Kc = L;
      have_next = false;
    }
    T em = cm, ep = cp;
    if (k & 1) {
      if (!have_next) {
        plane_vals(L + 1, nm, np);
        have_next = true;
      }
      em = half * (cm + nm);
      ep = half * (cp + np);
    }
    const int s = (b + k + Gf.off) & 1;  // colour of fine node 2m
    const long long row = Gf.row(b, k);
    if (inA && (!C0 || s == 0)) Xf[(long long)s * Gf.cs + row + m] += em;
    if (inB && (!C0 || s != 0)) Xf[(long long)(s ^ 1) * Gf.cs + row + m] += half * (em + ep);
  }
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
  const int kz = planes_per_block(G);
  const int k1 = min(G.g + bz * kz + kz - 1, last);
  for (int k = G.g + bz * kz; k <= k1; ++k)
    for (int r = 0; r < G.C; ++r) {
      const int a = (m << G.lc) + r;
      if (G.inner(a)) X[G.at(a, b, k)] = (T)0;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_add_corr(double* __restrict__ X, const T* __restrict__ E, Geom G) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  // threads numbered over the level's (compact column, row) pairs
  const int mc = G.mhi() - G.mlo() + 1;
  const int fi = bx * 256 + (int)threadIdx.x;
  if (fi >= mc * (G.n - 1)) return;
  const int m = G.mlo() + fi % mc;
  const int b = G.g + fi / mc;
  const int last = G.g + G.n - 2;
  const int kz = planes_per_block(G);
  const int k1 = min(G.g + bz * kz + kz - 1, last);
  for (int k = G.g + bz * kz; k <= k1; ++k)
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
__global__ __launch_bounds__(kFinishThreads) void k_finish(const double* __restrict__ partial, int nb, int nslots,
                                                           Scalars* __restrict__ scal, int dst) {
  for (int slot = 0; slot < nslots; ++slot) {
    const double s = sum_partials(partial + slot * kPartialCap, nb);
    if (threadIdx.x == 0) scal->v[dst + slot] = s;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- CG (A = -L)
// p_new = sr r + beta p_old;  q = A p_new;  partial (p_new . q), for the
// 19-point star (node by node, p formed at every stencil point).
// scal: v[0] = rr (current r.r, or the PCG inner product), v[2] = beta,
// v[3] = alpha.
__global__ __launch_bounds__(256) void k_cg_dir19(const double* __restrict__ R, const double* __restrict__ Pold,
                                                double* __restrict__ Pnew, double* __restrict__ Q, Geom G,
                                                double ih2, double sr, const Scalars* __restrict__ scal,
                                                double* __restrict__ partial) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  const double beta = scal->v[2];
  double acc = 0.0;
  if (m <= G.mhi() && b <= last) {
    const int kz = planes_per_block(G);
    const int k1 = min(G.g + bz * kz + kz - 1, last);
    auto pv = [&](int aa, int bb, int kk) -> double {
      const long long i = G.at(aa, bb, kk);
      return sr * R[i] + beta * Pold[i];  // ghosts of R and Pold are zero
    };
    for (int k = G.g + bz * kz; k <= k1; ++k)
      for (int r = 0; r < G.C; ++r) {
        const int a = (m << G.lc) + r;
        if (!G.inner(a)) continue;
        const double pc = pv(a, b, k);
        double s[3];
        for (int d = 1; d <= 3; ++d)
          s[d - 1] = pv(a - d, b, k) + pv(a + d, b, k) + pv(a, b - d, k) + pv(a, b + d, k) + pv(a, b, k - d) +
                     pv(a, b, k + d);
        const double lap = (3.0 * kC0 * pc + kC1 * s[0] + kC2 * s[1] + kC3 * s[2]) * ih2;
        const long long i = G.at(a, b, k);
        Pnew[i] = pc;
        Q[i] = -lap;
        acc += pc * (-lap);
      }
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = s;
}

// The same for the 7-point operator, with a register window along z as in
// the residual kernel: the thread owns nodes A = 2m and B = 2m+1 of row
// (b, k) for KZP planes, forms p = sr r + beta p_old at every position it
// loads (both colours at compact m for the z-window, x- and y-neighbours per
// plane; ghosts of r and p_old are zero), issues a chunk's loads before its
// updates, then stores p_new and q = -L p and sums p . q.
template <int KZP>
__global__ __launch_bounds__(256) void k_cg_dir7(const double* __restrict__ Rr, const double* __restrict__ Pold,
                                                 double* __restrict__ Pnew, double* __restrict__ Q, Geom G,
                                                 double ih2, double sr, const Scalars* __restrict__ scal,
                                                 double* __restrict__ partial) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  const double beta = scal->v[2];
  double acc = 0.0;
  if (m <= G.mhi() && b <= last) {
    const int kz = planes_per_block(G);
    const int k0 = G.g + bz * kz;
    const int k1 = min(k0 + kz - 1, last);
    const long long plane = (long long)G.M * G.W;
    const long long W = G.W;
    const long long q0 = G.row(b, 0) + m;
    auto pv = [&](long long i) -> double { return sr * Rr[i] + beta * Pold[i]; };
    constexpr int CH = KZP < 4 ? KZP : 4;
    double z0[KZP + 2], z1[KZP + 2];
    double xl[KZP], xr[KZP], ya0[KZP], ya1[KZP], yb0[KZP], yb1[KZP];
    const bool inA = G.inner(2 * m), inB = G.inner(2 * m + 1);
#pragma unroll
    for (int c0 = 0; c0 < KZP; c0 += CH) {
#pragma unroll
      for (int t = (c0 == 0 ? 0 : c0 + 2); t < c0 + CH + 2; ++t) {
        const long long o = (long long)min(k0 - 1 + t, k1 + 1) * plane;
        z0[t] = pv(q0 + o);
        z1[t] = pv(G.cs + q0 + o);
      }
#pragma unroll
      for (int t = c0; t < c0 + CH; ++t) {
        const int k = min(k0 + t, k1);
        const long long o = (long long)k * plane;
        const long long sa = (long long)((b + k + G.off) & 1) * G.cs;  // colour of A = 2m
        const long long sb = G.cs - sa;                                 // colour of B = 2m+1
        xl[t] = pv(sb + q0 + o - 1);
        xr[t] = pv(sa + q0 + o + 1);
        yb0[t] = pv(sb + q0 + o - W);
        yb1[t] = pv(sb + q0 + o + W);
        ya0[t] = pv(sa + q0 + o - W);
        ya1[t] = pv(sa + q0 + o + W);
      }
#pragma unroll
      for (int t = c0; t < c0 + CH; ++t) {
        const int k = k0 + t;
        if (k <= k1) {
          const int s = (b + k + G.off) & 1;
          const long long o = (long long)k * plane;
          const double pA = s ? z1[t + 1] : z0[t + 1], pB = s ? z0[t + 1] : z1[t + 1];
          const double zbA = s ? z0[t] + z0[t + 2] : z1[t] + z1[t + 2];
          const double zbB = s ? z1[t] + z1[t + 2] : z0[t] + z0[t + 2];
          if (inA) {
            const double lap = ((xl[t] + pB) + (yb0[t] + yb1[t] + zbA) - 6.0 * pA) * ih2;
            const long long i = (long long)s * G.cs + q0 + o;
            Pnew[i] = pA;
            Q[i] = -lap;
            acc += pA * (-lap);
          }
          if (inB) {
            const double lap = ((pA + xr[t]) + (ya0[t] + ya1[t] + zbB) - 6.0 * pB) * ih2;
            const long long i = (long long)(s ^ 1) * G.cs + q0 + o;
            Pnew[i] = pB;
            Q[i] = -lap;
            acc += pB * (-lap);
          }
        }
      }
    }
  }
  const double sum = block_sum(acc);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = sum;
}

// CG direction and operator, 7-point, with two compact columns m0, m0+1 per
// lane read and written as 16-byte vectors: p_new = sr r + beta p_old and
// q = -L p_new at the four nodes 2m0 .. 2m0+3, plus the block's partial sum of
// p_new . q.  The lane marches KZR planes keeping p for both colour arrays at
// its columns on planes k-1 .. k+1, and loads plane k+2 (r and p_old) one
// step ahead; the centre plane goes to LDS (double-buffered, one barrier per
// plane), so the y-neighbours inside the block's BY rows come from there and
// only the first and last thread rows load theirs (also one plane ahead);
// x-neighbours come from the lane's own vectors or the adjacent lanes (edge
// lanes load theirs).
template <int KZR>
__global__ __launch_bounds__(BX* BY) void k_cg_dir7z(const double* __restrict__ Rr, const double* __restrict__ Pold,
                                                     double* __restrict__ Pnew, double* __restrict__ Q, Geom G,
                                                     double ih2, double sr, const Scalars* __restrict__ scal,
                                                     double* __restrict__ partial) {
  typedef VecOf<double, 2>::type V;
  __shared__ V cen[2][2][BY][BX];
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int lane = threadIdx.x, ty = threadIdx.y;
  const int m0 = G.mlo() + 2 * (bx * BX + lane);
  const int b = G.g + by * BY + ty;
  const int last = G.g + G.n - 2;
  const double beta = scal->v[2];
  const bool live = m0 <= G.mhi() && b <= last;
  const int mm = live ? m0 : G.mlo();
  const int bb = min(b, last);
  const int k0 = G.g + bz * KZR;
  const int k1 = min(k0 + KZR - 1, last);
  const long long plane = (long long)G.M * G.W;
  const long long W = G.W;
  const long long q0 = G.row(bb, 0) + mm;
  auto ld = [](const double* p) -> V { return *reinterpret_cast<const V*>(p); };
  auto pv = [&](long long i) -> V { return sr * ld(Rr + i) + beta * ld(Pold + i); };
  auto ps = [&](long long i) -> double { return sr * Rr[i] + beta * Pold[i]; };
  // rows above and below the block's: loaded by its first and last thread rows
  const bool ylo = ty == 0 || bb - 1 < G.g + by * BY;   // b - 1 outside the block's rows
  const bool yhi = ty == BY - 1 || bb + 1 > min(G.g + by * BY + BY - 1, last);
  const bool needl = lane == 0 && mm >= 1;
  const bool needr = lane == BX - 1 && mm + 2 < G.W;
  // window: p of colour arrays 0 and 1 on planes k-1, k, k+1
  V z0[3], z1[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const long long o = (long long)min(k0 - 1 + t, k1 + 1) * plane;
    z0[t] = pv(q0 + o);
    z1[t] = pv(G.cs + q0 + o);
  }
  // one step ahead: plane k+2 of the window, rows b -+ 1 and the x edges of plane k+1
  V n0, n1, ym0, ym1, yp0, yp1;
  double el, er;
  auto side = [&](int k) {  // rows b -+ 1 and x edges of plane k
    const long long o = (long long)k * plane;
    if (ylo) {
      ym0 = pv(q0 + o - W);
      ym1 = pv(G.cs + q0 + o - W);
    }
    if (yhi) {
      yp0 = pv(q0 + o + W);
      yp1 = pv(G.cs + q0 + o + W);
    }
    const long long sa = (long long)((bb + k + G.off) & 1) * G.cs;
    const long long sb = G.cs - sa;
    el = needl ? ps(sb + q0 + o - 1) : 0.0;
    er = needr ? ps(sa + q0 + o + 2) : 0.0;
  };
  side(k0);
  double acc = 0.0;
  for (int k = k0; k <= k1; ++k) {
    const int buf = k & 1;
    cen[buf][0][ty][lane] = z0[1];
    cen[buf][1][ty][lane] = z1[1];
    V cym0 = ym0, cym1 = ym1, cyp0 = yp0, cyp1 = yp1;
    const double cel = el, cer = er;
    if (k < k1) {
      const long long o = (long long)min(k + 2, k1 + 1) * plane;
      n0 = pv(q0 + o);
      n1 = pv(G.cs + q0 + o);
      side(k + 1);
    }
    __syncthreads();
    if (!ylo) {
      cym0 = cen[buf][0][ty - 1][lane];
      cym1 = cen[buf][1][ty - 1][lane];
    }
    if (!yhi) {
      cyp0 = cen[buf][0][ty + 1][lane];
      cyp1 = cen[buf][1][ty + 1][lane];
    }
    const int s = (bb + k + G.off) & 1;  // colour of the even nodes
    const V pE = s ? z1[1] : z0[1], pO = s ? z0[1] : z1[1];
    const V zE = s ? z0[0] + z0[2] : z1[0] + z1[2];
    const V zO = s ? z1[0] + z1[2] : z0[0] + z0[2];
    const V yE = s ? cym0 + cyp0 : cym1 + cyp1;
    const V yO = s ? cym1 + cyp1 : cym0 + cyp0;
    double lftO = __shfl_up(pO[1], 1, 64);
    double rgtE = __shfl_down(pE[0], 1, 64);
    if (lane == 0) lftO = cel;
    if (lane == BX - 1) rgtE = cer;
    V qE, qO;
    qE[0] = -(((lftO + pO[0]) + (yE[0] + zE[0]) - 6.0 * pE[0]) * ih2);
    qE[1] = -(((pO[0] + pO[1]) + (yE[1] + zE[1]) - 6.0 * pE[1]) * ih2);
    qO[0] = -(((pE[0] + pE[1]) + (yO[0] + zO[0]) - 6.0 * pO[0]) * ih2);
    qO[1] = -(((pE[1] + rgtE) + (yO[1] + zO[1]) - 6.0 * pO[1]) * ih2);
    if (live) {
      const long long o = (long long)k * plane;
      const long long iE = (long long)s * G.cs + q0 + o, iO = (long long)(s ^ 1) * G.cs + q0 + o;
      bool inE[2], inO[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        inE[i] = mm + i <= G.mhi() && G.inner(2 * (mm + i));
        inO[i] = mm + i <= G.mhi() && G.inner(2 * (mm + i) + 1);
      }
      if (inE[0] && inE[1]) {
        *reinterpret_cast<V*>(Pnew + iE) = pE;
        *reinterpret_cast<V*>(Q + iE) = qE;
      } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
          if (inE[i]) {
            Pnew[iE + i] = pE[i];
            Q[iE + i] = qE[i];
          }
      }
      if (inO[0] && inO[1]) {
        *reinterpret_cast<V*>(Pnew + iO) = pO;
        *reinterpret_cast<V*>(Q + iO) = qO;
      } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
          if (inO[i]) {
            Pnew[iO + i] = pO[i];
            Q[iO + i] = qO[i];
          }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (inE[i]) acc += pE[i] * qE[i];
        if (inO[i]) acc += pO[i] * qO[i];
      }
    }
    z0[0] = z0[1];
    z0[1] = z0[2];
    z0[2] = n0;
    z1[0] = z1[1];
    z1[1] = z1[2];
    z1[2] = n1;
  }
  const double sum = block_sum(acc);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = sum;
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
    const int kz = planes_per_block(G);
    const int k1 = min(G.g + bz * kz + kz - 1, last);
    for (int k = G.g + bz * kz; k <= k1; ++k)
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

// partial sums of -(r . z): with the CG residual rho = -r and the
// preconditioned residual zeta = z, the inner product rho . zeta.
__global__ __launch_bounds__(256) void k_pcg_dot(const double* __restrict__ R, const double* __restrict__ Z, Geom G,
                                                 double* __restrict__ partial) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int m = G.mlo() + bx * BX + (int)threadIdx.x;
  const int b = G.g + by * BY + (int)threadIdx.y;
  const int last = G.g + G.n - 2;
  double acc = 0.0;
  if (m <= G.mhi() && b <= last) {
    const int kz = planes_per_block(G);
    const int k1 = min(G.g + bz * kz + kz - 1, last);
    for (int k = G.g + bz * kz; k <= k1; ++k)
      for (int r = 0; r < G.C; ++r) {
        const int a = (m << G.lc) + r;
        if (!G.inner(a)) continue;
        const long long i = G.at(a, b, k);
        acc += R[i] * Z[i];
      }
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[linear_block()] = -s;
}

// stage 0: v[4] = p.q (summed) -> alpha = rr / pq
// stage 1: v[5] = new rr (summed) -> beta = rr_new / rr; rr = rr_new
__global__ __launch_bounds__(kFinishThreads) void k_cg_scalars(const double* __restrict__ partial, int nb,
                                                               Scalars* __restrict__ scal, int stage) {
  const double s = sum_partials(partial, nb);
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

// planes per thread fixed at compile time: KZ on large levels, one on small
template <typename T, bool SOR, bool ZG>
static void pass7_kz(T* x, const T* f, const Geom& G, int colour, T omega, T h2, dim3 grid, dim3 blk,
                     hipStream_t st) {
  if (kz_for(G) == KZ)
    k_pass7<T, SOR, ZG, KZ, false><<<grid, blk, 0, st>>>(x, f, G, colour, omega, h2, nullptr);
  else
    k_pass7<T, SOR, ZG, 1, false><<<grid, blk, 0, st>>>(x, f, G, colour, omega, h2, nullptr);
}

// columns per lane of the vector 7-point pass: as many as make one 16-byte
// load while a row still fills a wavefront, and the last group stays inside
// the row pitch; 1 selects the one-column kernel
template <typename T>
static int pass7_cpl(const Geom& G) {
  const int mc = G.mhi() - G.mlo() + 1;
  for (int cpl = (int)(16 / sizeof(T)); cpl >= 2; cpl /= 2)
    if (mc >= BX * cpl && G.mhi() + cpl - 1 < G.W && G.mlo() % cpl == 0) return cpl;
  return 1;
}

constexpr int kPass7vKz = 4;  // planes per lane of the vector 7-point pass
template <int CPL>
static dim3 pass7v_grid(const Geom& G) {
  const int mc = G.mhi() - G.mlo() + 1, E = G.n - 1;
  return dim3((mc + BX * CPL - 1) / (BX * CPL), (E + BY - 1) / BY, (E + kPass7vKz - 1) / kPass7vKz);
}
template <typename T, int CPL>
static void pass7v_launch(T* x, const T* f, const Geom& G, int colour, bool zg, T h2, hipStream_t st) {
  const dim3 grid = pass7v_grid<CPL>(G), blk(BX, BY);
  if (zg)
    k_pass7v<T, CPL, true, kPass7vKz, false><<<grid, blk, 0, st>>>(x, f, G, colour, h2, nullptr);
  else
    k_pass7v<T, CPL, false, kPass7vKz, false><<<grid, blk, 0, st>>>(x, f, G, colour, h2, nullptr);
}

template <typename T>
static void pass7_launch(T* x, const T* f, const Geom& G, int colour, bool sor, bool zg, T omega, T h2, dim3 grid,
                         dim3 blk, hipStream_t st) {
  if (!sor) {
    const int cpl = pass7_cpl<T>(G);
    if (cpl == 4) {
      if constexpr (sizeof(T) == 4) return pass7v_launch<T, 4>(x, f, G, colour, zg, h2, st);
    } else if (cpl == 2) {
      return pass7v_launch<T, 2>(x, f, G, colour, zg, h2, st);
    }
  }
  if (sor)
    pass7_kz<T, true, false>(x, f, G, colour, omega, h2, grid, blk, st);
  else if (zg)
    pass7_kz<T, false, true>(x, f, G, colour, (T)1, h2, grid, blk, st);
  else
    pass7_kz<T, false, false>(x, f, G, colour, (T)1, h2, grid, blk, st);
}

void colour_pass(void* phi, const void* f, bool f32, const Geom& G, int order, int colour, double omega,
                 hipStream_t st, int zmask) {
  const dim3 grid = col_grid(G), blk(BX, BY);
  const double h2 = G.h * G.h;
  if (order == 2) {
    const bool sor = omega != 1.0;
    const bool zg = (zmask >> (colour ^ 1)) & 1;
    if (f32) {
      pass7_launch<float>((float*)phi, (const float*)f, G, colour, sor, zg, (float)omega, (float)h2, grid, blk,
                          st);
    } else {
      pass7_launch<double>((double*)phi, (const double*)f, G, colour, sor, zg, omega, h2, grid, blk, st);
    }
  } else {
    // planes per run: long runs on the 511^3 level, where the window's reload
    // at each run start costs bandwidth; shorter ones below, where the
    // blocks of a pass must still fill the chip
    const int E = G.n - 1;
    if (f32) {
      const int kz = G.n >= 512 ? 8 : G.n >= 128 ? 2 : 1;
      const dim3 g4((col_groups<4>(G) * E + 255) / 256, 1, (E + kz - 1) / kz);
      if (zmask)
        k_pass19v<float, 4, true><<<g4, 256, 0, st>>>((float*)phi, (const float*)f, G, colour, (float)h2, zmask);
      else
        k_pass19v<float, 4, false><<<g4, 256, 0, st>>>((float*)phi, (const float*)f, G, colour, (float)h2, 0);
    } else {
      const int kz = G.n >= 512 ? 16 : G.n >= 256 ? 4 : G.n >= 128 ? 2 : 1;
      const dim3 g2((col_groups<2>(G) * E + 255) / 256, 1, (E + kz - 1) / kz);
      if (zmask)
        k_pass19v<double, 2, true><<<g2, 256, 0, st>>>((double*)phi, (const double*)f, G, colour, h2, zmask);
      else
        k_pass19v<double, 2, false><<<g2, 256, 0, st>>>((double*)phi, (const double*)f, G, colour, h2, 0);
    }
  }
}

int colour_pass_dot(double* phi, const double* f, const Geom& G, int colour, double* partial, hipStream_t st) {
  const dim3 grid = col_grid(G), blk(BX, BY);
  const double h2 = G.h * G.h;
  // the vector pass where it applies and writes no more partial sums than
  // the one-column pass (the callers size their partial arrays for those)
  if (pass7_cpl<double>(G) == 2 && nblocks(pass7v_grid<2>(G)) <= nblocks(grid)) {
    const dim3 gv = pass7v_grid<2>(G);
    k_pass7v<double, 2, false, kPass7vKz, true><<<gv, blk, 0, st>>>(phi, f, G, colour, h2, partial);
    return (int)nblocks(gv);
  }
  if (kz_for(G) == KZ)
    k_pass7<double, false, false, KZ, true><<<grid, blk, 0, st>>>(phi, f, G, colour, 1.0, h2, partial);
  else
    k_pass7<double, false, false, 1, true><<<grid, blk, 0, st>>>(phi, f, G, colour, 1.0, h2, partial);
  return (int)nblocks(grid);
}

template <typename T, typename TO, int COL>
static void residual7_col(const T* phi, const T* f, TO* r, const Geom& G, T ih2, double* partial, hipStream_t st) {
  const dim3 grid = col_grid(G), blk(BX, BY);
  if (kz_for(G) == KZ)
    k_residual7<T, TO, KZ, COL><<<grid, blk, 0, st>>>(phi, f, r, G, ih2, partial);
  else
    k_residual7<T, TO, 1, COL><<<grid, blk, 0, st>>>(phi, f, r, G, ih2, partial);
}

template <typename T, typename TO>
static void residual_t(const T* phi, const T* f, TO* r, const Geom& G, int order, bool zu, double* partial,
                       int colour, hipStream_t st) {
  const dim3 grid = col_grid(G), blk(BX, BY);
  const T ih2 = (T)(1.0 / (G.h * G.h));
  if (order == 2) {
    if (zu)
      k_residual<T, TO, 2, true><<<grid, blk, 0, st>>>(phi, f, r, G, ih2, partial, G.mlo());
    else if (colour == 0)
      residual7_col<T, TO, 0>(phi, f, r, G, ih2, partial, st);
    else if (colour == 1)
      residual7_col<T, TO, 1>(phi, f, r, G, ih2, partial, st);
    else
      residual7_col<T, TO, -1>(phi, f, r, G, ih2, partial, st);
  } else {
    // both variants launch on the staged grid (and the column-0 kernel) so
    // that partial-sum counts agree
    const dim3 sg = staged_grid(G), sb(BX, TBY);
    const int mb = staged_mbase(G);
    // FP32 results on the large levels: two columns per thread (the FP64
    // form needs 194 registers and gains nothing); BX = 2 VX2, so the block
    // count equals the staged grid's
    bool two_col = false;
    if constexpr (sizeof(TO) == 4) two_col = !zu && G.n >= 256 && mb == 1;
    if (zu)
      k_residual<T, TO, 6, true><<<sg, sb, 0, st>>>(phi, f, r, G, ih2, partial, mb);
    else if (two_col) {
      if constexpr (sizeof(TO) == 4)
        k_residual19v<T, TO><<<sg, dim3(VX2, 2, TBY), 0, st>>>(phi, f, r, G, ih2, partial, mb);
    } else
      k_residual19s<T, TO><<<sg, sb, 0, st>>>(phi, f, r, G, ih2, partial, mb);
    if (staged_col0(G)) {
      const unsigned nb0 = col0_blocks(G);
      if (zu)
        k_res19_col0<T, TO, true><<<nb0, 256, 0, st>>>(phi, f, r, G, ih2, partial, nblocks(sg));
      else
        k_res19_col0<T, TO, false><<<nb0, 256, 0, st>>>(phi, f, r, G, ih2, partial, nblocks(sg));
    }
  }
}

int residual_blocks(const Geom& G) {
  return G.C == 4 ? (int)(nblocks(staged_grid(G)) + col0_blocks(G)) : (int)nblocks(col_grid(G));
}

void residual(const void* phi, const void* f, bool in_f32, void* r_out, bool out_f32, const Geom& G, int order,
              bool zu, double* partial, hipStream_t st, int colour) {
  if (in_f32) {
    residual_t<float, float>((const float*)phi, (const float*)f, (float*)r_out, G, order, zu, partial, colour, st);
  } else if (out_f32) {
    residual_t<double, float>((const double*)phi, (const double*)f, (float*)r_out, G, order, zu, partial, colour,
                              st);
  } else {
    residual_t<double, double>((const double*)phi, (const double*)f, (double*)r_out, G, order, zu, partial,
                               colour, st);
  }
}

bool resrestrict_ok(const Geom& Gf) { return Gf.C == 2 && Gf.g == 1 && Gf.n >= 4 && Gf.mhi() + 1 <= 128; }

void resrestrict(const void* phi, const void* f, bool f32, const Geom& Gf, void* f_coarse, const Geom& Gc,
                 hipStream_t st, bool r0only) {
  if (f32)
    resrestrict7_t<float>((const float*)phi, (const float*)f, Gf, (float*)f_coarse, Gc, r0only, st);
  else
    resrestrict7_t<double>((const double*)phi, (const double*)f, Gf, (double*)f_coarse, Gc, r0only, st);
}

bool resrestrict19_ok(const Geom& Gf) {
  // runs of an even number of planes from odd first planes: the staged grid's
  // 32-plane runs from 256 intervals, 8-plane runs at 128
  return Gf.C == 4 && Gf.g == 3 && Gf.n >= 128 && staged_mbase(Gf) == 1 && (Gf.n % 2) == 0;
}

// Own rows per block of the fused kernel: the residual kernel's 8, or 6 on
// FP32 levels from 512 intervals, where two blocks of eight wavefronts fill
// a CU's 16 wave slots (503 against 577 us at 511^3).  Taller blocks (FP32:
// 12 or 14 rows; FP64: 10) were slower.
template <typename T, int TR>
static int resrestrict19_tr(const T* phi, const T* f, const Geom& Gf, T* f_coarse, const Geom& Gc, double* partial,
                            bool last_zero, hipStream_t st) {
  const dim3 sg0 = staged_grid(Gf);
  const dim3 sg(sg0.x, (Gf.n - 1 + TR - 1) / TR, sg0.z), blk(BX, TR + 2);
  const T ih2 = (T)(1.0 / (Gf.h * Gf.h));
  const int mb = staged_mbase(Gf);
  if (last_zero)
    k_resrestrict19<T, true, TR><<<sg, blk, 0, st>>>(phi, f, Gf, ih2, f_coarse, Gc, partial, mb);
  else
    k_resrestrict19<T, false, TR><<<sg, blk, 0, st>>>(phi, f, Gf, ih2, f_coarse, Gc, partial, mb);
  return (int)nblocks(sg);
}

int resrestrict19(const void* phi, const void* f, bool f32, const Geom& Gf, void* f_coarse, const Geom& Gc,
                  double* partial, bool last_zero, hipStream_t st) {
  if (f32) {
    auto x = (const float*)phi, y = (const float*)f;
    auto c = (float*)f_coarse;
    // 6-row blocks write 4/3 as many partial sums as the 8-row grid, for
    // which the plan checked the partial-sum capacity
    const dim3 sg0 = staged_grid(Gf);
    const bool six = Gf.n >= 512 && (!partial || (long long)sg0.x * ((Gf.n - 1 + 5) / 6) * sg0.z <= kPartialCap);
    return six ? resrestrict19_tr<float, 6>(x, y, Gf, c, Gc, partial, last_zero, st)
               : resrestrict19_tr<float, TBY>(x, y, Gf, c, Gc, partial, last_zero, st);
  }
  return resrestrict19_tr<double, TBY>((const double*)phi, (const double*)f, Gf, (double*)f_coarse, Gc, partial,
                                       last_zero, st);
}

void restrict_fw(const void* r_fine, const Geom& Gf, void* f_coarse, const Geom& Gc, bool f32, hipStream_t st,
                 bool last_zero) {
  const int sh = Gf.g - 1, nc = Gc.n, C = Gf.C;
  if (C == 4) {  // four colours, three ghost layers
    const int kzc = nc >= 32 ? 4 : 1;
    auto grid = [&](int cpl) {
      const long long groups = ((2 * (Gc.g + nc - 2) - sh) >> 2) / cpl - ((2 * Gc.g - sh) >> 2) / cpl + 1;
      return dim3((unsigned)((groups * (nc - 1) + 255) / 256), 1, (nc - 1 + kzc - 1) / kzc);
    };
#define PSN_R4(T, CPL, SK) \
  k_restrict4<T, CPL, SK><<<grid(CPL), 256, 0, st>>>((const T*)r_fine, Gf, (T*)f_coarse, Gc)
    if (f32) {
      if (last_zero) PSN_R4(float, 4, true); else PSN_R4(float, 4, false);
    } else {
      if (last_zero) PSN_R4(double, 2, true); else PSN_R4(double, 2, false);
    }
#undef PSN_R4
    return;
  }
  // two colours: every residual is read
  const int mcols = (2 * (Gc.g + nc - 2) - sh) / C - (2 * Gc.g - sh) / C + 1;
  const int kzc = nc >= 128 ? 8 : (nc >= 32 ? 4 : 1);
  const dim3 grid((mcols + 63) / 64, (nc - 1 + 3) / 4, (nc - 1 + kzc - 1) / kzc), blk(64, 4);
  if (f32)
    k_restrict_z<float, 2><<<grid, blk, 0, st>>>((const float*)r_fine, Gf, (float*)f_coarse, Gc);
  else
    k_restrict_z<double, 2><<<grid, blk, 0, st>>>((const double*)r_fine, Gf, (double*)f_coarse, Gc);
}

void prolong_add(const void* e_coarse, const Geom& Gc, void* phi_fine, const Geom& Gf, bool f32,
                 hipStream_t st, bool c0only) {
  // c0only: the last colour's correction is dead (see the declaration).
  // Plans create two layouts only: two colours with one ghost layer (7-point)
  // and four colours with three (19-point star).
  const dim3 grid = col_grid(Gf), blk(BX, BY);
  if (Gf.C == 2 && Gf.g == 1) {
    if (f32) {
      if (c0only)
        k_prolong2<float, true><<<grid, blk, 0, st>>>((const float*)e_coarse, Gc, (float*)phi_fine, Gf);
      else
        k_prolong2<float, false><<<grid, blk, 0, st>>>((const float*)e_coarse, Gc, (float*)phi_fine, Gf);
    } else {
      if (c0only)
        k_prolong2<double, true><<<grid, blk, 0, st>>>((const double*)e_coarse, Gc, (double*)phi_fine, Gf);
      else
        k_prolong2<double, false><<<grid, blk, 0, st>>>((const double*)e_coarse, Gc, (double*)phi_fine, Gf);
    }
    return;
  }
  if (Gf.C == 4) {  // four colours, three ghost layers
    const int E = Gf.n - 1;
    const int kz = Gf.n >= 128 ? 4 : 1;
    auto grid = [&](int groups) { return dim3((unsigned)(((long long)groups * E + 255) / 256), 1, (E + kz - 1) / kz); };
    if (f32) {
      const dim3 g4 = grid(col_groups<4>(Gf));
      if (c0only)
        k_prolong4<float, 4, true><<<g4, 256, 0, st>>>((const float*)e_coarse, Gc, (float*)phi_fine, Gf);
      else
        k_prolong4<float, 4, false><<<g4, 256, 0, st>>>((const float*)e_coarse, Gc, (float*)phi_fine, Gf);
    } else {
      const dim3 g4 = grid(col_groups<2>(Gf));
      if (c0only)
        k_prolong4<double, 2, true><<<g4, 256, 0, st>>>((const double*)e_coarse, Gc, (double*)phi_fine, Gf);
      else
        k_prolong4<double, 2, false><<<g4, 256, 0, st>>>((const double*)e_coarse, Gc, (double*)phi_fine, Gf);
    }
    return;
  }
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
    k_add_corr<float><<<flat_grid(G), 256, 0, st>>>(phi, (const float*)e, G);
  else
    k_add_corr<double><<<flat_grid(G), 256, 0, st>>>(phi, (const double*)e, G);
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
  k_finish<<<1, kFinishThreads, 0, st>>>(partial, nb, nslots, scal, dst);
}

int cg_blocks(const Geom& G) { return (int)nblocks(col_grid(G)); }

// the 7-point direction kernel with two columns per lane where a row fills a
// wavefront at that width (and the last pair stays inside the row pitch)
static bool cg_dir_vec(const Geom& G, int order) {
  return order == 2 && G.mhi() - G.mlo() + 1 >= 2 * BX && G.mlo() % 2 == 0 && G.mhi() + 1 < G.W;
}
// planes per block of the z-marching direction kernel
static int cg_dir_kz(const Geom& G) { return G.n > 256 ? 16 : 8; }
static dim3 cg_dir_vec_grid(const Geom& G) {
  const int mc = G.mhi() - G.mlo() + 1, E = G.n - 1, kz = cg_dir_kz(G);
  return dim3((mc + 2 * BX - 1) / (2 * BX), (E + BY - 1) / BY, (E + kz - 1) / kz);
}

int cg_dir_blocks(const Geom& G, int order) {
  return (int)nblocks(cg_dir_vec(G, order) ? cg_dir_vec_grid(G) : col_grid(G));
}

void cg_direction_apply(const double* r, const double* p_old, double* p_new, double* q, const Geom& G, int order,
                        const Scalars* scal, double* partial, hipStream_t st, double sr) {
  const double ih2 = 1.0 / (G.h * G.h);
  if (cg_dir_vec(G, order)) {
    if (cg_dir_kz(G) == 16)
      k_cg_dir7z<16><<<cg_dir_vec_grid(G), dim3(BX, BY), 0, st>>>(r, p_old, p_new, q, G, ih2, sr, scal, partial);
    else
      k_cg_dir7z<8><<<cg_dir_vec_grid(G), dim3(BX, BY), 0, st>>>(r, p_old, p_new, q, G, ih2, sr, scal, partial);
  }
  else if (order == 2 && kz_for(G) == KZ)
    k_cg_dir7<KZ><<<col_grid(G), dim3(BX, BY), 0, st>>>(r, p_old, p_new, q, G, ih2, sr, scal, partial);
  else if (order == 2)
    k_cg_dir7<1><<<col_grid(G), dim3(BX, BY), 0, st>>>(r, p_old, p_new, q, G, ih2, sr, scal, partial);
  else
    k_cg_dir19<<<col_grid(G), dim3(BX, BY), 0, st>>>(r, p_old, p_new, q, G, ih2, sr, scal, partial);
}

void pcg_dot(const double* r, const double* z, const Geom& G, double* partial, hipStream_t st) {
  k_pcg_dot<<<col_grid(G), dim3(BX, BY), 0, st>>>(r, z, G, partial);
}

void cg_update(double* x, double* r, const double* p, const double* q, const Geom& G, const Scalars* scal,
               double* partial, hipStream_t st) {
  k_cg_upd<<<col_grid(G), dim3(BX, BY), 0, st>>>(x, r, p, q, G, scal, partial);
}

void cg_scalars(const double* partial, int nb, Scalars* scal, int stage, hipStream_t st) {
  k_cg_scalars<<<1, kFinishThreads, 0, st>>>(partial, nb, scal, stage);
}

}  // namespace psn
