// Internal declarations of the gfx950 Poisson library: level geometry,
// device helpers and the host-side launch wrappers of every kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>
#include <stdint.h>
#include <stddef.h>

#include "../../include/poisson.h"

namespace psn {

constexpr int kLmaxMax = 8;
constexpr int kNqMax = (kLmaxMax + 1) * (kLmaxMax + 1);  // 81 real moments
constexpr int kRowAlign = 32;       // compact rows padded to 32 elements

// ---------------------------------------------------------------------------
// Colour-split level layout.
//
// A level with n intervals and g ghost layers has M = n + 1 + 2(g-1) nodes
// per axis, node array indices a, b, k in [0, M) (x, y, z).  The node's
// colour is (a + b + k + off) mod C with off chosen so that the colour equals
// (i + j + k) mod C in global node indices i = a - (g-1) (Sections 2.1.1 and
// 2.1.2: two colours for the 7-point operator, four for the 19-point star).
// Nodes are stored per colour, compacted along x: node (a, b, k) lives in
// colour array c = colour(a,b,k) at row (k*M + b) and column a / C.  A pass
// over one colour therefore streams whole rows of that colour and reads the
// other colours at the same or adjacent columns.
// ---------------------------------------------------------------------------
struct Geom {
  int n;      // intervals per axis
  int g;      // ghost layers (stencil radius)
  int C;      // colours (power of two: 2 or 4)
  int lc;     // log2(C)
  int M;      // nodes per axis
  int W;      // row pitch of a colour array (elements)
  int off;    // colour offset
  int pad_;
  long long cs;  // elements per colour array (M*M*W)
  double h;

  __host__ __device__ long long row(int b, int k) const { return ((long long)k * M + b) * W; }
  __host__ __device__ int colour(int a, int b, int k) const { return (a + b + k + off) & (C - 1); }
  __host__ __device__ long long at(int a, int b, int k) const {
    return (long long)colour(a, b, k) * cs + row(b, k) + (a >> lc);
  }
  __host__ __device__ bool inner(int a) const { return a >= g && a <= g + n - 2; }
  __host__ __device__ long long total() const { return cs * C; }
  // number of compact columns that can hold an unknown
  __host__ __device__ int mlo() const { return g >> lc; }
  __host__ __device__ int mhi() const { return (g + n - 2) >> lc; }
};

Geom make_geom(int n, int g, int C, double h);

// ---------------------------------------------------------------------------
// Log-spherical natural layout (radius fastest, one ghost at each end).
// ---------------------------------------------------------------------------
struct SGeom {
  int nr, nth, nph;
  int pad_;
  long long p0, p1;   // row pitch (>= nr + 2), plane pitch (>= nth * p0)
  double ds, dth, dph, r_min;  // ds: log-core step in ln r; r_min: first unknown's radius
  const double* rr;   // radius per radial index 0 .. nr+1 (ghosts at 0 and nr+1)
  const double* rw;   // radial volume weight r^2 R' per radial index (unknowns)
  __host__ __device__ long long at(int i, int j, int k) const { return (long long)k * p1 + (long long)j * p0 + i; }
};

// One level of the FP32 multigrid preconditioner on the spherical grid:
// nr x nth x nph unknowns in [phi][theta][r] layout with one zero radial
// ghost on each side; level l pairs the nodes of level l-1 two by two along
// each axis (spacings doubled, colatitudes (j + 1/2) pi / nth).  The radial
// couplings rcl[i], rcr[i] (to unknowns i-1, i+1; diagonal -(rcl + rcr))
// are the radial map's operator rediscretised on the level: constant on the
// log grid, varying with i where an inner pad bends the map.  A row holds
// the even radial array indices a (ghost a = 0 included) in its first hp
// entries and the odd ones in the next hp, so the lines of one zebra colour
// at a colatitude are contiguous.
struct SLev {
  int nr, nth, nph, p0;  // unknowns, row pitch (2 hp)
  int hp;                // entries per parity half of a row
  long long p1;          // plane pitch
  float idt2, idp2;
  float* u;
  float* f;
  float* r;
  const float* rcl;    // per radial unknown i
  const float* rcr;
  const float* cot2;   // cot(theta_j) / (2 dtheta)
  const float* isin2;  // 1 / sin^2(theta_j)
  // phi-line solver: each line splits into nseg segments of seg nodes; a
  // block holds nl lines; the table of line (i, j) at ltab + (it nth + j)
  // tstride, it = min(i, ntab - 1): the radial couplings vary only on the
  // unknowns inside an inner pad (the first ntab - 1), every other radius
  // has the log map's and shares the last table (ntab = 1 on a log grid);
  // it holds
  // the segment elimination factors m[seg], c'[seg], the responses v[seg],
  // w[seg] to unit end loads and the 2nseg x 2nseg interface inverse
  int seg, nseg, nl, tstride, ntab;
  const float* ltab;
  __host__ __device__ long long at(int a, int j, int k) const {
    return (long long)k * p1 + (long long)j * p0 + (long long)(a & 1) * hp + (a >> 1);
  }
  __host__ __device__ long long count() const { return p1 * nph; }
};

// Natural-layout level of the SPAI multigrid: nodes 0..n per axis (one
// ghost layer), x pitch W (a multiple of 32), plane pitch P = (n + 1) W.
struct NGeom {
  int n, W;
  long long P;
  double h;
  __host__ __device__ long long at(int i, int j, int k) const { return (long long)k * P + (long long)j * W + i; }
  __host__ __device__ long long total() const { return (long long)(n + 1) * P; }
};

// Cubically symmetric 27-point stencil: centre, face, edge, corner weights.
struct W4 {
  double c, f, e, k;
};

// Per-plan device scalars used by the Krylov solvers and reductions.
struct Scalars {
  double v[32];
};

// ---------------------------------------------------------------------------
// Launch wrappers (all asynchronous on `st`).
// ---------------------------------------------------------------------------
// natural <-> split conversions; scale multiplies the values (4 pi G for rho).
void split_from_natural(const double* src, long long p0, long long p1, void* dst, bool dst_f32,
                        const Geom& G, double scale, hipStream_t st);
void merge_to_natural(const double* src_split, double* dst, long long p0, long long p1, const Geom& G,
                      bool unknowns_only, double scale, hipStream_t st);
void fill_zero(void* x, bool f32, long long count, hipStream_t st);
void zero_unknowns(void* x, bool f32, const Geom& G, hipStream_t st);

// one colour pass of Gauss-Seidel / SOR in place (order 2: 7-point, order 6:
// star); colours whose bit is set in zmask are read as zero (first sweep on a
// zero initial guess, which then needs no separate clearing pass)
void colour_pass(void* phi, const void* f, bool f32, const Geom& G, int order, int colour,
                 double omega, hipStream_t st, int zmask = 0);

// Four-colour levels from 128 intervals (FP64, or FP32 when f32): the
// 19-point residual fused with full weighting into f_coarse, without storing
// the fine residual; partial (when not null) receives partial sums of r^2,
// as many as the call returns (at most residual_blocks(Gf)); last_zero as
// restrict_fw.
bool resrestrict19_ok(const Geom& Gf);
int resrestrict19(const void* phi, const void* f, bool f32, const Geom& Gf, void* f_coarse, const Geom& Gc,
                  double* partial, bool last_zero, hipStream_t st);

// r = f - L phi on the unknowns (split in, split out or nullptr); partial sums
// of r^2 go to partial[kReduceBlocks].  zero_unknowns_in treats the unknowns of
// phi as 0 (norm of b).  out_f32 selects the output precision.  colour 0 / 1
// (7-point only): only that colour's residual, the other one being known to
// vanish (right after a Gauss-Seidel pass over it).
void residual(const void* phi, const void* f, bool in_f32, void* r_out, bool out_f32, const Geom& G,
              int order, bool zero_unknowns_in, double* partial, hipStream_t st, int colour = -1);
int residual_blocks(const Geom& G);   // partials written by residual()
// f_coarse = R (f - L phi) for the 7-point operator without storing the fine
// residual; resrestrict_ok tells whether the level's shape is supported
// (two colours, one ghost layer, at most 256 intervals)
bool resrestrict_ok(const Geom& Gf);
// r0only: the colour-1 residuals vanish (a Gauss-Seidel pass over colour 1
// came last) and only the colour-0 ones are formed.
void resrestrict(const void* phi, const void* f, bool f32, const Geom& Gf, void* f_coarse, const Geom& Gc,
                 hipStream_t st, bool r0only = false);
// last_zero (four colours): the residuals of colour 3 vanish (a Gauss-Seidel
// pass over it came last) and are not read
void restrict_fw(const void* r_fine, const Geom& Gf, void* f_coarse, const Geom& Gc, bool f32,
                 hipStream_t st, bool last_zero = false);
// c0only: leave the last colour (1 of two, 3 of four) uncorrected, when a
// Gauss-Seidel pass over that colour follows, which reads no value of its
// own colour and overwrites them all.
void prolong_add(const void* e_coarse, const Geom& Gc, void* phi_fine, const Geom& Gf, bool f32,
                 hipStream_t st, bool c0only = false);
void coarse_solve(const double* inv, const void* f, void* phi, bool f32, const Geom& G, hipStream_t st);
// phi64 (unknowns) += e (f32 or f64)
void add_correction(double* phi, const void* e, bool e_f32, const Geom& G, hipStream_t st);

// dense interior (n-1)^3 <-> split helpers for the single-operator entry points
void dense_to_split(const double* dense, void* split, bool f32, const Geom& G, hipStream_t st);
void split_to_dense(const void* split, bool f32, double* dense, const Geom& G, hipStream_t st);

// reductions: sum nb partials of each of nslots slots (stride kPartialCap)
// into scal->v[dst + slot]
void finish_sum(const double* partial, int nb, int nslots, Scalars* scal, int dst, hipStream_t st);

// CG (A = -L, zero-ghost direction vectors, split layout, FP64).  The
// direction is p_new = sr r + beta p_old (sr = 1: CG on r; sr = -1: PCG on
// the preconditioned residual z, which has the opposite sign).
void cg_direction_apply(const double* r, const double* p_old, double* p_new, double* q, const Geom& G,
                        int order, const Scalars* scal, double* partial, hipStream_t st, double sr = 1.0);
// partial sums cg_direction_apply writes
int cg_dir_blocks(const Geom& G, int order);
// partial sums of -(r . z) over the unknowns (the PCG inner product)
void pcg_dot(const double* r, const double* z, const Geom& G, double* partial, hipStream_t st);
// 7-point FP64 Gauss-Seidel pass of one colour that also writes the blocks'
// partial sums of -(f . phi_new) over the nodes it updates at partial;
// returns how many (at most cg_blocks(G))
int colour_pass_dot(double* phi, const double* f, const Geom& G, int colour, double* partial, hipStream_t st);
void cg_update(double* x, double* r, const double* p, const double* q, const Geom& G, const Scalars* scal,
               double* partial, hipStream_t st);
void cg_scalars(const double* partial, int nb, Scalars* scal, int stage, hipStream_t st);
int cg_blocks(const Geom& G);

// multipole (Section 2.2)
// Monomial form of the regular solid harmonics (device copies): monomial t
// (degree-ordered, all a + b + c <= kLmaxMax) is mono[t] = a | b << 4 | c << 8;
// R_q (q = l^2 + l + m) = sum over e in [toff[q], toff[q+1]) of
// tcoef[e] x^a y^b z^c with (a, b, c) = monomial tmono[e].
struct MomTables {
  const int* mono;
  const int* toff;
  const int* tmono;
  const double* tcoef;
};
constexpr int kMonoMax = (kLmaxMax + 1) * (kLmaxMax + 2) * (kLmaxMax + 3) / 6;  // 165
constexpr int kTermMax = 1024;  // bound on the number of terms (415 at lmax 8)
// host construction of the tables from the recurrence; returns false if the
// term count exceeds kTermMax
bool build_mom_tables(std::vector<int>& mono, std::vector<int>& toff, std::vector<int>& tmono,
                      std::vector<double>& tcoef);
// scratch of the separable Cartesian moments (bytes) for n intervals
size_t cart_moment_scratch(int n);
// q (nq = (lmax+1)^2 values, point_mass added to q_00) of the Cartesian node
// array rho by separable monomial sums
void cart_moments(const double* rho, long long p0, long long p1, int n, int g, double h, double cx, double cy,
                  double cz, int lmax, const MomTables& tab, double point_mass, double* scratch, double* q,
                  hipStream_t st);
// q (outer, + point_mass on q_00) and qbar (inner) of the log-spherical
// array rho by ray sums; scratch of sph_moment_scratch(nth, nph) bytes
size_t sph_moment_scratch(int nth, int nph);
void sph_moments(const double* rho, const SGeom& S, int lmax, double point_mass, double* scratch, double* q,
                 double* qbar, hipStream_t st);
void cart_ghosts(double* phi, long long p0, long long p1, int n, int g, double h, double lo, double cx,
                 double cy, double cz, int lmax, const double* q, double G, hipStream_t st);
void sph_ghosts(double* phi, const SGeom& S, int lmax, const double* q, const double* qbar,
                double point_mass, double G, hipStream_t st);

// spherical operator and BiCGSTAB building blocks (FP64, natural layout)
// cot: cot(theta_j)/(2 dtheta); isin2: 1/sin^2(theta_j); r2: r^2 per radial
// index; rcl, rcr: radial couplings to i-1 and i+1 per radial index
struct SphCoef { const double* cot; const double* isin2; const double* r2; const double* rcl; const double* rcr; };

void sph_residual(const double* u, const double* rho, double* r, const SGeom& S, const SphCoef& c,
                  double four_pi_G, bool zero_unknowns_in, double* partial, hipStream_t st);
void sph_apply(const double* u, double* out, const SGeom& S, const SphCoef& c, hipStream_t st);
// one SOR colour pass (colours 0..3: parity + 2 in the second half turn) with
// relaxation factor omega[j (nr+2) + i] per colatitude and radial index, and
// one step of the Chebyshev sequence omega <- 1 / (1 - rj^2 omega / 4) over
// n entries
// omega_out (with rj): also write the next Chebyshev term per (j, i) there
// (nphi >= 4 and colour >= 2, the second pass of a half-sweep)
void sph_sor_pass(double* u, const double* rho, const SGeom& S, const SphCoef& c, double four_pi_G,
                  const double* omega, int colour, hipStream_t st, const double* rj = nullptr,
                  double* omega_out = nullptr);
void sph_omega_next(double* omega, const double* rj, int n, hipStream_t st);
// right-preconditioned BiCGSTAB: p = r + beta (p - omega v), phat = B^-1 p;
// s = r - alpha v, shat = B^-1 s (B: red-black block lower triangle);
// out = A xhat with dots (mode 0: w.out; mode 1: w.out and out.out);
// x += alpha phat + omega shat, r = s - omega t with dots rhat.r and r.r
void pbicg_direction(const double* r, double* p, const double* v, double* phat, const SGeom& S,
                     const SphCoef& c, const Scalars* scal, hipStream_t st);
void pbicg_s(const double* r, const double* v, double* s, double* shat, const SGeom& S, const SphCoef& c,
             const Scalars* scal, hipStream_t st);
// the same vector updates without the Gauss-Seidel preconditioner
void pbicg_update_p(const double* r, double* p, const double* v, const SGeom& S, const SphCoef& c,
                    const Scalars* scal, hipStream_t st);
void pbicg_update_s(const double* r, const double* v, double* s, const SGeom& S, const SphCoef& c,
                    const Scalars* scal, hipStream_t st);
void pbicg_apply(const double* xhat, double* out, const double* w, int mode, const SGeom& S,
                 const SphCoef& c, double* partial, hipStream_t st);
void pbicg_xr(double* x, double* r, const double* phat, const double* shat, const double* s, const double* t,
              const double* rhat, const SGeom& S, const Scalars* scal, double* partial, hipStream_t st);
// FP32 multigrid preconditioner on the spherical grid.  The smoother is
// zebra phi-line Gauss-Seidel: the lines (i, j) with (i + j) & 1 == colour
// are solved exactly along phi (a periodic tridiagonal system), with the
// neighbours in r and theta -- the other colour -- held fixed; across a pole
// a line meets itself half a turn away, and that coupling is taken from the
// values before the pass.
// zero_guess (first sweep of a cycle from a zero guess, so u needs no
// clearing): 1 = u is taken as zero (first colour), 2 = the pass's own lines
// are taken as zero (second colour: only its cross-pole term reads them)
void sph_line_pass(const SLev& L, int colour, int zero_guess, hipStream_t st);
void sph_residual32(const SLev& L, hipStream_t st);
void sph_restrict32(const SLev& Lf, const SLev& Lc, hipStream_t st);
void sph_prolong_add32(const SLev& Lc, const SLev& Lf, hipStream_t st);
void sph_coarse32(const double* inv, const SLev& L, hipStream_t st);
void sph_cast_in(const double* x, const SGeom& S, const SLev& L0, hipStream_t st);
void sph_cast_out(const SLev& L0, double* x, const SGeom& S, hipStream_t st);
void bicg_scalars(const double* partial, int nb, Scalars* scal, int stage, hipStream_t st);
// SPAI multigrid on natural-layout levels (27-point stencils).
NGeom make_ngeom(int n, double h);
long long n27_blocks(const NGeom& G);
// r = f - A u at the unknowns (r may be nullptr with norm); norm: one partial
// sum of r^2 per block.  f32: the level is stored in FP32 (arithmetic FP64).
void n27_residual(const void* u, const void* f, void* r, bool f32, const NGeom& G, const W4& A, bool norm,
                  double* partial, hipStream_t st);
// fused Richardson step out of place: out = u - M (f - A u) at the unknowns
// (ghost entries of out are not written)
void n_spai_step(const void* u, const void* f, void* out, bool f32, const NGeom& G, const W4& A, const W4& M,
                 hipStream_t st);
void n_copy(const void* a, void* b, bool f32, const NGeom& G, hipStream_t st);
void n_restrict(const void* r, bool f32_fine, const NGeom& Gf, void* fc, bool f32_coarse, const NGeom& Gc,
                hipStream_t st);
void n_prolong_add(const void* uc, bool f32_coarse, const NGeom& Gc, void* uf, bool f32_fine, const NGeom& Gf,
                   hipStream_t st);
void n_coarse(const double* inv, const void* f, void* u, bool f32, const NGeom& G, hipStream_t st);
// coarsest level by CG to relative residual rtol (one block, LDS resident)
size_t n_cg_lds_bytes(const NGeom& G);
void n_coarse_cg(const void* f, void* u, bool f32, const NGeom& G, const W4& A, double rtol, hipStream_t st);
// caller arrays (pitches p0, p1; `ghost` layers) <-> level arrays
void n_from_caller(const double* src, long long p0, long long p1, int ghost, double* u, const NGeom& G,
                   bool zero_inner, hipStream_t st);
void n_rhs(const double* rho, long long p0, long long p1, int ghost, double* f, const NGeom& G, int order,
           double scale, hipStream_t st);
void n_to_caller(const double* u, const NGeom& G, double* dst, long long p0, long long p1, int ghost,
                 hipStream_t st);
int sph_blocks(const SGeom& S);
void sph_fill_zero(double* x, const SGeom& S, hipStream_t st);
void sph_copy(const double* src, double* dst, const SGeom& S, hipStream_t st);

}  // namespace psn
