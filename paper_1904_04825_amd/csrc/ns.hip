// Navier-Stokes (BR1) residual and element-Jacobi assembly.
#include "internal.h"

namespace frjf {

hipError_t launch_ns_residual(const fr_disc*, int, const ResArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_ns_ejacobi_assemble(const fr_disc*, const double*, double, void*, int, int, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace frjf
