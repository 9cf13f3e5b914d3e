// Reverse-mode step with frozen events (internal).
#pragma once
#include "launch.h"

namespace tf {

struct TrajStep {
  PState st;   // state entering the step (slot order of the previous sort)
  int* perm;   // new slot -> old slot of this step
  double* phi; // potential of this step
};

struct AdjWork {
  bool enabled;
};

AdjWork carve_adjoint(Carver& cv, long long n_tot, long long c_tot, long long s_tot, int n_ens, bool enabled);

hipError_t run_adjoint(const Ctx& C, const LaunchGeo& G, const AdjWork& W, int n_ens, const Ens* eh,
                       const long long* p_off, const TrajStep* steps, int n_steps, const double* const* lambda,
                       const double* w_wall, double* dtheta, hipStream_t st);

}  // namespace tf
