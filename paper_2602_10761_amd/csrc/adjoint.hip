// Reverse-mode step (placeholder until the adjoint kernels land).
#include "adjoint.h"

namespace tf {

AdjWork carve_adjoint(Carver&, long long, long long, long long, int, bool enabled) {
  AdjWork w;
  w.enabled = enabled;
  return w;
}

hipError_t run_adjoint(const Ctx&, const LaunchGeo&, const AdjWork&, int, const Ens*, const long long*,
                       const TrajStep*, int, const double* const*, const double*, double*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace tf
