// Discrete adjoint of the fused BBK step (placeholder until the reverse kernels land).
#include "../../include/xyl.h"
#include "xyl_internal.hpp"

struct xyl_lattice;

namespace xyl {
void adjoint_release(xyl_lattice*) {}
}  // namespace xyl

extern "C" {
int xyl_adjoint_forward(xyl_lattice*, uint64_t, uint64_t, uint64_t, double*) { return XYL_EUNSUPPORTED; }
int xyl_adjoint_backward(xyl_lattice*, double*, double*, double*) { return XYL_EUNSUPPORTED; }
}
