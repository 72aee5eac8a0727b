/*
 * poisson.h -- C ABI of the MI355X (gfx950) self-gravity Poisson library.
 *
 * Problem (Sections 2 and 2.1 of Krasnopolsky et al., "Iterative Poisson
 * Solvers for Self-gravity with the GPU Code Astaroth"): given the mass
 * density rho on a 3-D structured grid, find the potential Phi with
 *     lap Phi = 4 pi G rho                                   (Eqs. 1, 2)
 * under Dirichlet ghost values, iterating until the residual falls below a
 * tolerance and warning when a maximum iteration count is reached
 * (Section 2.1).  The ghost values come from the multipole expansion of rho
 * with a user-chosen lmax (Section 2.2, Eqs. outer_expansion ..
 * inner_multipole) or are supplied by the caller (analytic test mode).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All device pointers are HIP device memory owned by the caller (the
 *   library never allocates or frees caller buffers).  The caller also owns
 *   the workspace handed to poisson_plan; a plan keeps non-owning views into
 *   it and must be destroyed before the workspace is released.
 * - Every call is ordered on the plan's stream.  A plan is not thread-safe;
 *   distinct plans (with distinct workspaces) are independent.
 * - Cartesian arrays (rho, Phi) are vertex-centred node arrays in natural
 *   layout, x fastest: element (i, j, k) of node array indices
 *   0 <= i, j, k < n + 1 + 2(ghost - 1) lives at  k*pitch[1] + j*pitch[0] + i.
 *   Nodes ghost..ghost+n-2 along every axis are unknowns; the others hold the
 *   Dirichlet (ghost) values.  The box is [lo, hi]^3, h = (hi-lo)/n.
 * - Log-spherical arrays are [phi][theta][r]: element (i, j, k) with
 *   0 <= i < nr + 2 (radial ghosts at i = 0 and i = nr + 1),
 *   0 <= j < ntheta, 0 <= k < nphi lives at k*pitch[1] + j*pitch[0] + i.
 *   Radii r_i = r_min * exp((i-1) ds), ds = ln(r_max/r_min)/(nr-1);
 *   theta_j = (j + 1/2) pi / ntheta; phi_k = 2 pi k / nphi (periodic).  The
 *   colatitude neighbour past a pole is the node at phi + pi.
 * - Functions return a status (POISSON_OK or a negative error); no exception
 *   crosses the boundary.  poisson_last_error() gives the detail of the most
 *   recent failure on the calling thread.
 */
#ifndef POISSON_MI355X_H
#define POISSON_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define POISSON_OK            0   /* converged / done */
#define POISSON_WARN_MAXITER  1   /* tolerance not met within max_iter (Section 2.1); Phi holds the last iterate */
#define POISSON_EINVAL       -1   /* null pointer, bad option, tol <= 0, pitch too small */
#define POISSON_EGRID        -2   /* grid unsuited to the method (multigrid needs n = 2^L * coarsest, Section 2.1.3) */
#define POISSON_EWORKSPACE   -3   /* workspace missing, too small or misaligned */
#define POISSON_EHIP         -4   /* a HIP runtime call failed */
#define POISSON_ENUMERIC     -5   /* NaN/Inf residual or Krylov breakdown */
#define POISSON_EADMIT       -6   /* serving: request larger than the whole memory budget */
#define POISSON_ETIMEOUT     -7   /* serving: poisson_server_wait ran out of time (the request goes on) */

/* ---- enumerations ---------------------------------------------------- */
#define POISSON_CARTESIAN      0
#define POISSON_SPHERICAL_LOG  1

#define POISSON_SOR            0  /* red-black SOR (Section 2.1.1); on spherical grids four
                                     colours (parity, half turn) and relaxation factors per
                                     colatitude and radius from Eq. local_rjac: omega_mode OPT (local
                                     omega_opt), CHEBYSHEV (local Eq. omega_n from n = 1) or
                                     FIXED */
#define POISSON_CG             1  /* conjugate gradients (Section 2.1.2) */
#define POISSON_BICGSTAB       2  /* BiCGSTAB, spherical grids (Section 2.1.2), right-preconditioned
                                     by one red-black Gauss-Seidel step (Section 2.1.1) */
#define POISSON_MG             3  /* FP64 geometric multigrid V-cycles (Section 2.1.3); where the
                                     finest level stores its residual for the restriction
                                     (19-point star; 7-point grids above 256 intervals) the
                                     stopping test reads that residual, formed after each
                                     cycle's pre-smoothing, and the iterate returned is the one
                                     after the last cycle's pre-smoothing (iterations counts the
                                     cycles begun) */
#define POISSON_MG_IR32        4  /* FP32 V-cycles inside FP64 iterative refinement */
#define POISSON_BICGSTAB_MG32  5  /* spherical grids: BiCGSTAB right-preconditioned by one FP32
                                     V(nu1, nu2) cycle (four-colour Gauss-Seidel, cell-pair
                                     coarsening); every axis must halve evenly down to a
                                     level of <= 4096 unknowns, solved by a dense inverse */
#define POISSON_MG_SPAI        6  /* Cartesian FP64 V(nu1, nu2) cycles with the SPAI Richardson
                                     smoother of Table 1 (Eqs. richardson, Smoother), Galerkin
                                     coarse operators R A P and compact radius-1 stencils:
                                     order 2 (7-point), 4 (19-point Mehrstellen, right-hand
                                     side (6 f + face sum) / 12) or 6 (27-point
                                     (-128, 14, 3, 1)/30h^2, right-hand side
                                     (402 f + 40 faces - 3 axis nodes at distance 2 + 8 in-plane
                                     diagonals) / 720, which reads rho's second ghost layer:
                                     grid.ghost = 2; Table 1's order-6 delta taken as 0.0151);
                                     coarsest level solved by a dense inverse, or by CG with
                                     opts.coarse_tol (Section 2.1.3) */
#define POISSON_MG_SPAI32      7  /* POISSON_MG_SPAI with every level below the finest stored in
                                     FP32 and all arithmetic in FP64 (the paper's mixed
                                     precision, Section 2.1.3) */
#define POISSON_PCG            8  /* Cartesian CG preconditioned by one symmetric multi-colour
                                     Gauss-Seidel step from a zero guess (Section 2.1.2: two
                                     colours for order 2, four for the 19-point star): the
                                     section's block lower triangle B applied forward over the
                                     colours, then backward (B D^-1 B^T, symmetric positive
                                     definite as CG needs) */

#define POISSON_OMEGA_OPT       0 /* 2/(1+sqrt(1-rJ^2)), rJ from Eq. rjac */
#define POISSON_OMEGA_OPT_A     1 /* 2/(1+pi/N) */
#define POISSON_OMEGA_CHEBYSHEV 2 /* Eq. omega_n started from n = 1, one term per colour pass */
#define POISSON_OMEGA_FIXED     3 /* opts.omega */

typedef struct poisson_plan_s* poisson_plan_t;   /* opaque */

typedef struct {
    int32_t coord;      /* POISSON_CARTESIAN or POISSON_SPHERICAL_LOG */
    int32_t n[3];       /* Cartesian: intervals per axis (all three equal);
                           spherical: nr, ntheta, nphi unknowns (ntheta, nphi even) */
    double  lo[3];      /* Cartesian box corner; spherical: lo[0] = r_min */
    double  hi[3];      /* Cartesian box corner; spherical: hi[0] = r_max */
    int32_t ghost;      /* Cartesian ghost layers: 1 (7-point and compact orders 2, 4), 2 (compact
                           order 6) or 3 (19-point star); spherical: 1 */
    int32_t pad_;
    int64_t pitch[2];   /* elements per row, elements per plane of caller arrays */
    /* Spherical radial padding (Section 3.3; zero on Cartesian grids).  The
       log core runs from r_in = lo[0] (first core unknown) to r_out = hi[0]
       (last core unknown) with equal steps ds in ln r.  ext_out > 0: ext_out
       more cells continue the log map outward (the last node is the outer
       ghost).  ext_in > 0: ext_in cells continue inward along the quartic
       Q(xi) = r_in (1 + ds xi + (ds xi)^2/2 + (ds xi)^3/6) + c4 xi^4 of the
       map coordinate xi (xi = 0 at r_in), which matches the log map and its
       first three derivatives at r_in and reaches r_pad at xi = -ext_in (the
       inner ghost); it must increase monotonically.  n[0] counts every radial
       unknown, pads included: n[0] = nlog + max(ext_in-1, 0) +
       max(ext_out-1, 0) with nlog >= 2 core unknowns.  The operator is
       discretised on the map coordinate (a u_xixi + b u_xi, a = (r/R')^2,
       b = 2r/R' - r^2 R''/R'^3), the s = ln r form on the plain log grid. */
    int32_t ext_in;
    int32_t ext_out;
    double  r_pad;
} poisson_grid_t;

typedef struct {
    int32_t method;      /* POISSON_SOR .. POISSON_PCG */
    int32_t order;       /* Cartesian: 2 (7-point) or 6 (19-point star); POISSON_MG_SPAI(32):
                            2, 4 or 6 (compact); spherical: 2 */
    int32_t lmax;        /* >= 0: multipole boundary of this order (<= 8);
                            -1: ghost values are read from Phi as given (Section 2.2 test mode) */
    int32_t nu1, nu2;    /* multigrid pre/post smoothing sweeps */
    int32_t coarsest;    /* multigrid coarsest intervals per axis (solved exactly) */
    int32_t omega_mode;  /* SOR: POISSON_OMEGA_* */
    int32_t max_iter;    /* iteration / cycle cap */
    int32_t check_every; /* iterations between residual checks (>= 1) */
    int32_t pad_;
    double  omega;       /* SOR with POISSON_OMEGA_FIXED */
    double  four_pi_G;   /* 4 pi G */
    double  point_mass;  /* mass of a point at the expansion origin (central sink), 0 for none */
    double  coarse_tol;  /* POISSON_MG_SPAI(32): 0 = coarsest level by its dense inverse; in (0, 1):
                            by CG from a zero guess to this relative residual (Section 2.1.3
                            takes the cycle's rate), coarsest <= 12 intervals */
} poisson_opts_t;

typedef struct {
    int32_t iterations;       /* sweeps / Krylov steps / V-cycles / refinement steps done */
    int32_t status;           /* same as the return value */
    double  rel_residual;     /* ||b - A Phi|| / ||b|| at exit (2-norm over unknowns) */
    double  b_norm;           /* ||b||: residual of Phi with zero unknowns */
    double  rate;             /* mean convergence rate (rel_residual)^(1/iterations) (Eq. rho) */
    double  t_multipole_ms;   /* time of the multipole boundary phase */
    double  t_iter_ms;        /* time of the iteration phase */
    double* residual_history; /* optional caller-owned host array, rel residual per check */
    int32_t history_cap;      /* its capacity */
    int32_t history_len;      /* entries written */
} poisson_stats_t;

/* Default options for a method (order 2, lmax 8, V(2,2) to 8 intervals --
   V(3,3) for POISSON_MG_SPAI(32), the paper's choice --, max_iter 10000,
   check_every 1, four_pi_G 1). */
void poisson_default_opts(poisson_opts_t* opts, int32_t method);

/* Bytes of device workspace a plan for (grid, opts) needs.  Returns 0 and
   sets the last error when the combination is invalid. */
size_t poisson_workspace_bytes(const poisson_grid_t* grid, const poisson_opts_t* opts);

/* Build a plan: validate the grid (multigrid: n = 2^L * coarsest,
   Section 2.1.3), carve d_workspace (256-byte aligned, >= the size above)
   into level arrays, precompute omega (Eqs. omega_final, rjac, omega_n) and
   the exact inverse of the coarsest operator, and record the stream
   (a hipStream_t; NULL = default stream).  *out is set only on success. */
int poisson_plan(poisson_plan_t* out, const poisson_grid_t* grid, const poisson_opts_t* opts,
                 void* d_workspace, size_t ws_bytes, void* stream);

/* Multigrid plans (and the multigrid-preconditioned BiCGSTAB) launch each
   iteration as one recorded HIP graph.  The graph is recorded on `stream`, a
   caller-owned hipStream_t other than the NULL stream that must outlive the
   plan and carry no other work while a poisson_* call of this plan runs;
   nothing is executed on it.  Without a capture stream the graph is recorded
   on the plan's own stream, and when that is the NULL stream (which cannot be
   recorded) every iteration is launched kernel by kernel instead, with the
   same results.  The library creates no stream.  POISSON_EINVAL for a NULL
   plan or stream. */
int poisson_plan_set_capture_stream(poisson_plan_t plan, void* stream);

/* Section 2.2: compute the multipole moments of d_rho (sums over the
   unknown nodes with weight h^3, or r^3 ds sin(theta) dtheta dphi on the
   spherical grid; expansion origin at the box centre / r = 0) and overwrite
   every ghost node of d_phi with the expansion's potential (Cartesian: all
   faces, edges and corners of every ghost layer; spherical: the outer shell
   from the outer expansion, the inner shell from the inner expansion plus
   the central point mass).  lmax in 0..8.  If h_q is not NULL it receives
   (lmax+1)^2 outer moments (index l*l + l + m; m < 0 sine, m >= 0 cosine
   real harmonics, orthonormal, no Condon-Shortley phase) followed, on the
   spherical grid, by (lmax+1)^2 inner moments; it is written after a
   stream synchronisation. */
int multipole_boundary(poisson_plan_t plan, const double* d_rho, double* d_phi, int32_t lmax,
                       double* h_q);

/* Allocation-free multipole boundary, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc): the Cartesian case of
   multipole_boundary without a plan.  The moment sums, the monomial tables
   and q_lm live in a fixed device array of POISSON_NOALLOC_SCRATCH_BYTES that
   the library holds on each GPU it runs on until the process ends (enough for
   n <= 512 at any lmax <= 8); nothing is allocated or freed per call, and the
   first call on a device uploads the tables into that device's array with
   hipMemcpy.  grid: Cartesian, ghost 1..3, pitches as for poisson_plan;
   d_rho is read at the unknowns, every ghost node of d_phi is overwritten
   (the unknowns are left untouched); four_pi_G > 0; point_mass is added to
   q_00; h_q as for multipole_boundary (NULL to skip; synchronises).  Work is
   queued on `stream` (a hipStream_t, NULL = default stream).  Every call on
   one GPU shares that GPU's array, so calls that overlap on one GPU (other
   threads or streams) race; calls queued on one stream are ordered.
   POISSON_EINVAL for a spherical grid, bad arguments, or an n whose scratch
   exceeds the array; POISSON_EHIP when the array's address cannot be
   obtained. */
#define POISSON_NOALLOC_SCRATCH_BYTES (80u * 1024u * 1024u)
int multipole_boundary_noalloc(const poisson_grid_t* grid, const double* d_rho, double* d_phi,
                               int32_t lmax, double four_pi_G, double point_mass, double* h_q,
                               void* stream);

/* Solve lap Phi = 4 pi G rho (Cartesian) or r^2 lap Phi = r^2 4 pi G rho
   (spherical, Eq. 2 in s = ln r) for the unknowns of d_phi.  On entry the
   unknowns are the initial guess (warm start, Section 2.1); with
   opts.lmax >= 0 the ghosts are first set by multipole_boundary, otherwise
   read as given.  Stops when ||b - A Phi|| <= tol ||b|| (checked every
   check_every iterations) or after max_iter; returns POISSON_OK or
   POISSON_WARN_MAXITER.  grid must equal the plan's grid.  stats may be
   NULL. */
int poisson_solve(poisson_plan_t plan, const double* d_rho, double* d_phi,
                  const poisson_grid_t* grid, double tol, poisson_stats_t* stats);

void poisson_plan_destroy(poisson_plan_t plan);

const char* poisson_strerror(int status);
const char* poisson_last_error(void);

/* ---- single-operator entry points (same plan, same layouts) ------------
   These expose the individual hot-path operations for verification and
   profiling; all are asynchronous on the plan stream unless a host output
   is requested. */

/* d_out[unknowns] = (L_h Phi) on the unknown nodes (Cartesian: 7-point or
   19-point star by opts.order; spherical: the r^2-scaled operator).  Other
   entries of d_out are left untouched.  POISSON_EINVAL for POISSON_MG_SPAI
   plans, whose operator is exposed through poisson_op_residual. */
int poisson_op_apply(poisson_plan_t plan, const double* d_phi, double* d_out);

/* d_res[unknowns] = 4 pi G rho - L_h Phi (spherical: r^2-scaled;
   POISSON_MG_SPAI: 4 pi G B rho - L_h Phi with the compact stencil and its
   right-hand side operator B), and *h_norm2 = sum of squares over the
   unknowns (NULL to skip; synchronises). */
int poisson_op_residual(poisson_plan_t plan, const double* d_rho, const double* d_phi,
                        double* d_res, double* h_norm2);

/* `sweeps` full Gauss-Seidel/SOR sweeps in place on the unknowns of d_phi
   (Cartesian): colours in increasing order when forward != 0, reversed
   otherwise; red-black with relaxation omega for order 2 (Section 2.1.1),
   four colours with omega = 1 for order 6 (Section 2.1.2).  POISSON_MG_SPAI
   plans: `sweeps` steps of the SPAI Richardson smoother (Eq. richardson;
   forward and omega are ignored).  Spherical POISSON_SOR plans: `sweeps`
   SOR sweeps (colours 0, 2 then 1, 3) with the plan's relaxation factors
   per colatitude and radius from the start of their sequence (forward and
   omega are ignored). */
int poisson_op_smooth(poisson_plan_t plan, const double* d_rho, double* d_phi, int32_t sweeps,
                      int32_t forward, double omega);

/* Full-weighting restriction (Section 2.1.3) of a dense (n-1)^3 array of
   unknown values to a dense (n/2-1)^3 array (both x fastest, no ghosts). */
int poisson_op_restrict(poisson_plan_t plan, const double* d_fine, double* d_coarse);

/* Restricted residual (Section 2.1.3): d_coarse = R (4 pi G rho - L_h Phi),
   the right-hand side a V-cycle hands to the next coarser level, as a dense
   (n/2-1)^3 array (x fastest, no ghosts); rho and Phi as in
   poisson_op_residual (caller layout, Phi's ghosts used as given); and
   *h_norm2 = sum of squares of the fine residual over the unknowns (NULL to
   skip; synchronises).  Multigrid plans with at least two levels
   (POISSON_EINVAL otherwise): POISSON_MG in FP64; POISSON_MG_IR32 rounds Phi
   and 4 pi G rho to FP32 and works in FP32 as its inner cycles do (the
   squares still summed in FP64).  On four-colour levels from 128 intervals
   one fused kernel forms both without storing the fine residual. */
int poisson_op_restrict_residual(poisson_plan_t plan, const double* d_rho, const double* d_phi,
                                 double* d_coarse, double* h_norm2);

/* d_fine += P d_coarse, P = 8 R^T (trilinear), dense interior arrays as above. */
int poisson_op_prolong_add(poisson_plan_t plan, const double* d_coarse, double* d_fine);

/* `cycles` V(nu1,nu2) cycles (MG, MG_IR32 or MG_SPAI plans, each in its own
   precision; for MG_IR32 one cycle = one refinement step) on d_phi with the
   ghosts as given, no convergence test. */
int poisson_op_vcycle(poisson_plan_t plan, const double* d_rho, double* d_phi, int32_t cycles);

/* `sweeps` forward Gauss-Seidel sweeps (omega = 1) on the plan's resident
   fine-level arrays exactly as the last poisson_solve / poisson_op_* call
   left them, with no layout conversion: the smoother kernel alone, for
   timing it in its solver launch configuration.  MG / MG_IR32 plans sweep
   their cycle's finest level (FP64 or FP32); MG_SPAI plans take 2 * sweeps
   fused SPAI steps (out of place, so the result returns to where it
   started) on theirs; other Cartesian plans sweep the FP64 potential. */
int poisson_op_sweep_resident(poisson_plan_t plan, int32_t sweeps);

/* POISSON_BICGSTAB_MG32 plans: d_yhat = M^-1 d_y, M^-1 being one FP32
   V(nu1, nu2) cycle of the spherical multigrid preconditioner from a zero
   guess (the right preconditioner of the BiCGSTAB iteration, Sections
   2.1.2-2.1.3).  Both arrays in the plan's spherical layout (FP64); the
   unknowns of d_y are read, the unknowns of d_yhat written, radial ghosts of
   either are not accessed.  POISSON_EINVAL for other plans. */
int poisson_op_precond(poisson_plan_t plan, const double* d_y, double* d_yhat);

/* ---- serving loop: continuous batching of independent solves -----------
   A persistent worker thread advances every admitted request by one
   multigrid iteration at a time on its own stream slot, so requests of
   different sizes overlap on the device; requests that arrive while others
   run are admitted as slots and memory free up.  The caller owns every
   device resource: plan workspaces and one cached potential per stream id
   are ranges of the caller's arena, handed out first fit and returned to a
   free list (merged with free neighbours) when idle plans and cached
   potentials are released, least recently used first; the slot streams are
   the caller's.  The server allocates no device memory and creates no
   stream.  Each stream id's last potential is the initial guess of its next
   request (Section 2.1: the previous potential as initial estimate).  A
   result depends only on its density and its stream's history, not on what
   else is running. */
typedef struct poisson_server_s* poisson_server_t;

/* d_arena: caller-owned device memory of arena_bytes (256-byte aligned) that
   the server uses, and nothing else, until poisson_server_destroy returns;
   arena_bytes is the memory budget.  slot_streams: max_slots (1..16)
   caller-owned hipStream_t, none the NULL stream, that must outlive the
   server; the server launches on them and records its graphs on them.
   mixed != 0: FP32 V-cycles inside FP64 refinement (7-point), else FP64
   V-cycles; lmax: multipole order of the open boundary; nu: smoothing sweeps
   nu1 = nu2; tol: relative residual target; warm_start: reuse each stream's
   previous potential; use_graphs: launch each iteration as one recorded
   graph.  Uses the current device. */
int poisson_server_create(poisson_server_t* out, void* d_arena, size_t arena_bytes, int32_t max_slots,
                          void* const* slot_streams, int32_t mixed, int32_t lmax, int32_t nu, double tol,
                          int32_t warm_start, int32_t use_graphs);
/* Queue a solve on the unit box with n = 8 * 2^L intervals per axis.
   d_rho and d_phi are caller-owned device arrays in natural layout with
   pitch (n+1, (n+1)^2) elements; both must stay valid until the request is
   done; the potential is written into d_phi.  The request reads d_rho and
   writes d_phi only after the work queued on caller_stream (a hipStream_t;
   NULL = the NULL stream) before this call: an event recorded on it here is
   waited for on the request's slot.  Once poisson_server_poll reports the
   request done, d_phi holds the result on the device; it is not ordered with
   any stream.  Returns POISSON_EADMIT when the request alone exceeds the
   arena, POISSON_EGRID for other sizes. */
int poisson_server_submit(poisson_server_t srv, int32_t stream_id, int32_t n, const double* d_rho,
                          double* d_phi, void* caller_stream, int64_t* ticket);
/* *done = 1 once the request has finished; then returns its status
   (POISSON_OK, POISSON_WARN_MAXITER or an error) and fills stats (NULL
   allowed; t_iter_ms = start-to-finish time on the device) and the latency
   from submission to completion in milliseconds. */
int poisson_server_poll(poisson_server_t srv, int64_t ticket, int32_t* done, poisson_stats_t* stats,
                        double* latency_ms);
/* Block up to timeout_ms for a ticket; returns its status, or
   POISSON_ETIMEOUT when the time ran out first (the request is not
   cancelled). */
int poisson_server_wait(poisson_server_t srv, int64_t ticket, double timeout_ms);
/* Build `count` (<= 16) plans of size n with their captured graphs ahead of
   traffic, within the budget, so that no request pays for plan construction;
   blocks until done.  Returns POISSON_EADMIT if they do not fit. */
int poisson_server_reserve(poisson_server_t srv, int32_t n, int32_t count);
/* Arena bytes one request of size n occupies (plan workspace + cached
   potential, each rounded up to 256 bytes). */
int poisson_server_footprint(poisson_server_t srv, int32_t n, size_t* bytes);
/* Arena bytes in use, queued and running request counts (any may be NULL). */
int poisson_server_usage(poisson_server_t srv, size_t* used_bytes, int32_t* queued, int32_t* active);
/* Waits for every queued and running request, then releases the server;
   the arena and the slot streams return to the caller. */
void poisson_server_destroy(poisson_server_t srv);

#ifdef __cplusplus
}
#endif
#endif /* POISSON_MI355X_H */
