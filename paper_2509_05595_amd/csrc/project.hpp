// The safe projection stage (Sec. 6): the simplified mesh's vertices move
// towards the input mesh by projected Newton on the augmented energy of
// Sec. 6.2, along a piecewise-linear path that additive CCD keeps free of
// self-intersections (Alg. 2).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace pamo {

// the mesh to project is not a closed, consistently oriented manifold
struct ProjectMeshError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// Uniform samples on the triangle mesh (V, F): sample s takes the first
// triangle whose inclusive cumulative area exceeds U[s][0] times the total,
// and the point (1 - r) a + r (1 - U[s][2]) b + r U[s][2] c, r = sqrt(U[s][1]).
// Returns the total area (synchronises).
double project_sample(Workspace& ws, hipStream_t s, const double* V, int nv, const int* F, int nf, const double* U,
                      int64_t m, double* Y);

// Closest-feature targets: targets[i] = the point of (Vin, Fin) closest to
// X[i]; tri[s] = the triangle of (X, F) closest to Y[s].  Ties: the smallest
// triangle index whose squared distance is within a relative 1e-9 (plus
// 1e-24) of the smallest.
void project_targets(Workspace& ws, hipStream_t s, const double* X, int nv, const int* F, int nf, const double* Vin,
                     int nvin, const int* Fin, int nfin, const double* Y, int m, double* targets, int* tri);

// One evaluation at X of the pieces of an iteration (fixed targets): the five
// energy terms (unweighted) and B, the contact counts; optionally the
// gradient of B, the projected Hessian times v, the CG direction and the
// ACCD step along it.  X0 is the rest shape.
struct ProjectEvalOut {
  double parts[6];  // s2m, m2s, elastic, bend, barrier, B
  int64_t npt, nee;
  double* grad = nullptr;     // device [nv][3] or null
  const double* v = nullptr;  // device [nv][3] or null
  double* Hv = nullptr;       // device [nv][3] or null
  double* dir = nullptr;      // device [nv][3] or null
  int cg_iters = 0;
  bool want_step = false;
  double step = 0.0;
};
void project_eval(Workspace& ws, hipStream_t s, const double* X0, const double* X, int nv, const int* F, int nf,
                  const double* targets, const double* Y, const int* tri, int m, double area_in,
                  const pamo_project_options& o, ProjectEvalOut& out);

// Alg. 2 from (X0, F) towards (Vin, Fin) with the samples Y (m of them, on the
// input mesh); the result in Xout.  log: host [iterations][8] or null (B at
// the iteration's start, ACCD step, step taken, halvings, CG iterations,
// point-triangle and edge-edge contacts, gradient norm).
void project_run(Workspace& ws, hipStream_t s, const double* X0, int nv, const int* F, int nf, const double* Vin,
                 int nvin, const int* Fin, int nfin, const double* Y, int m, const pamo_project_options& o,
                 double* Xout, double* log, pamo_project_stats* stats);

}  // namespace pamo
