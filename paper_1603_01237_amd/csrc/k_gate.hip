// Dense gate path (evolution operators): placeholder until the MFMA kernels land.
#include "ism_paths.h"

namespace ism {
int gate_create(ism_problem*, const double*, int, const double*, const double*, const double*) {
    return ISM_E_UNSUPPORTED;
}
int gate_boundary_pass(ism_problem*, double*, double, bool) { return ISM_E_UNSUPPORTED; }
int gate_slice_pass(ism_problem*, int, double, double*, bool) { return ISM_E_UNSUPPORTED; }
int gate_copy_state(ism_problem*, double*, int) { return ISM_E_UNSUPPORTED; }
size_t gate_footprint_extra(int, int, int, int, int, int) { return 0; }
}  // namespace ism
