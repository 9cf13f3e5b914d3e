// Reverse-mode step with frozen events (internal).
#pragma once
#include "launch.h"

namespace tf {

// One recorded step: the state entering it and the sort/field of the step.
struct TrajStep {
  PState st;          // state entering the step (slot order of the previous sort)
  int* perm;          // new slot -> old slot
  int* skey;          // cell of each new slot
  int* start;         // cell runs [c_tot + 1]
  double* phi;        // potential
  signed char* wall;  // wall impact of each new slot (-1 none, 0 lower, 1 upper)
};

struct AdjLam {
  double *x, *y, *z, *vx, *vy, *vz, *q;
};

struct AdjWork {
  bool enabled;
  AdjLam lamA, lamB, lamP;  // cotangents: two state buffers and the per-slot local part
  double* lamE;             // [3][n_tot] per-slot field cotangent ke * lambda_a
  double* lamS;             // [3][n_tot] per-slot cotangent of the same-cell Coulomb sum
  double* dth;              // [3][n_tot] per-slot d/d(k_c, dU, e), summed over a segment's steps
  double* lamEc;            // [3][c_tot] field cotangent per cell
  double* radj;             // [c_tot]    -G^T lambda_E (right-hand side of the adjoint Poisson problem)
  double* lamQ;             // [c_tot]    cotangent of the cell charge
  double* part;             // [n_ens][nch][3] chunk sums of d/dtheta
  int nch;                  // chunks of kAdjChunk slots in the largest ensemble
  double* wwall;            // [n_ens][2] cotangent of the wall charge accumulators (copied from the caller)
};

constexpr int kAdjChunk = 2048;  // slots per block of the d/dtheta reduction

AdjWork carve_adjoint(Carver& cv, long long n_tot, long long c_tot, long long s_tot, int n_ens, long long np_max,
                      bool enabled);

hipError_t run_adjoint(const Ctx& C, const LaunchGeo& G, const AdjWork& W, int n_ens, const Ens* eh,
                       const long long* p_off, const long long* c_off, const TrajStep* steps, int n_steps,
                       const double* const* lambda, const double* w_wall, double* dtheta, hipStream_t st);

}  // namespace tf
