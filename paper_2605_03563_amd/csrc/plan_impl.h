// Internal definition of a solver plan, shared by the solver drivers and the
// serving loop (not part of the C ABI).
#pragma once

#include <vector>

#include "internal.h"

namespace psn {

void set_error(const char* fmt, ...);
int launch_check(const char* what);

struct Level {
  Geom G;
  void* phi = nullptr;
  void* f = nullptr;
  void* tmp = nullptr;
};
// level of the SPAI multigrid: natural layout, operator A (Galerkin on coarse
// levels) and smoother M = omega h^2 (alpha, beta, gamma, delta)
struct NLevel {
  NGeom G{};
  void* u = nullptr;
  void* u2 = nullptr;  // partner of u for the out-of-place smoothing steps (same ghosts)
  void* f = nullptr;
  void* r = nullptr;
  bool f32 = false;  // stored in FP32 (coarse levels of MG_SPAI32); arithmetic FP64
  W4 A{};
  W4 M{};
};

}  // namespace psn

struct poisson_plan_s {
  poisson_grid_t grid{};
  poisson_opts_t opts{};
  hipStream_t st = nullptr;
  hipStream_t cap = nullptr;  // caller's stream for recording graphs (nullptr: the plan's stream)
  bool sph = false;
  int order = 2;
  int C = 2;
  // Cartesian level 0 (FP64, colour split)
  psn::Geom G0{};
  double* phi64 = nullptr;
  double* f64 = nullptr;
  double* t64 = nullptr;
  // multigrid hierarchy: lv[0] is the finest level of the cycle
  std::vector<psn::Level> lv;
  bool mg32 = false;
  double* cinv = nullptr;
  int ncoarse = 0;
  // SPAI multigrid (natural layout)
  std::vector<psn::NLevel> nlv;
  // CG
  double *cr = nullptr, *cp0 = nullptr, *cp1 = nullptr, *cq = nullptr;
  double* cz = nullptr;  // PCG: preconditioned residual
  // spherical
  psn::SGeom S{};
  psn::SphCoef sc{};
  double *sr = nullptr, *srh = nullptr, *sp[2] = {nullptr, nullptr}, *sv[2] = {nullptr, nullptr};
  double *ss = nullptr, *stt = nullptr;
  double* somega = nullptr;            // SOR: relaxation factor per colatitude
  double* somega2 = nullptr;           // SOR, Chebyshev sequence: the next term
  double* srj = nullptr;               // SOR: local Jacobi spectral radius per colatitude
  std::vector<double> srj_host;        // the same on the host
  std::vector<psn::SLev> slv;          // FP32 multigrid preconditioner levels (BICGSTAB_MG32)
  double* scinv = nullptr;             // dense inverse of its coarsest level
  int sncoarse = 0;
  hipGraphExec_t iter_exec = nullptr;  // captured preconditioned BiCGSTAB iteration
  const double* iter_phi = nullptr;    // caller array the captured iteration updates
  // reductions and moments
  double* partial = nullptr;
  psn::Scalars* scal = nullptr;
  double* qlm = nullptr;  // 2 * kNqMax
  // multipole moments: monomial tables (Cartesian) and the scratch of the
  // separable (Cartesian) or ray (spherical) sums
  int* mom_mono = nullptr;
  int* mom_toff = nullptr;
  int* mom_tmono = nullptr;
  double* mom_tcoef = nullptr;
  double* mom_scratch = nullptr;
  double* host = nullptr; // pinned scalars
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  hipGraphExec_t step_exec = nullptr;
  // FP64 multigrid solves whose fine level stores its residual: the first
  // cycle head, and the tail of a cycle followed by the next head
  hipGraphExec_t head_exec = nullptr;
  hipGraphExec_t cont_exec = nullptr;
};

namespace psn {

enum ScalarSlot { kRR = 0, kBnorm2 = 8, kRes2 = 9 };

// Asynchronous phases of a Cartesian multigrid solve on the plan's stream
// (no host synchronisation): setup = multipole boundary (when lmax >= 0),
// layout split, ||b||^2 into scal->v[kBnorm2] and the initial residual norm^2
// into scal->v[kRes2]; step = one multigrid iteration (graph launch when
// use_graph) leaving the new residual norm^2 in scal->v[kRes2]; finish =
// write the unknowns back to the caller's array.
int cart_setup(poisson_plan_s* P, const double* rho, double* phi);
int cart_step(poisson_plan_s* P, bool use_graph);
int cart_finish(poisson_plan_s* P, double* phi);
// capture the step graph now (done lazily by the first graph step otherwise)
int cart_prepare_graph(poisson_plan_s* P);

}  // namespace psn
