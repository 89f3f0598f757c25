// Gross-Pitaevskii path: placeholder until the split-step kernels land.
#include "ism_paths.h"

namespace ism {
int gpe_create(ism_problem*, int, double, double, const double*, const double*, double,
               const double*, const double*) {
    return ISM_E_UNSUPPORTED;
}
int gpe_boundary_pass(ism_problem*, double*, double, bool) { return ISM_E_UNSUPPORTED; }
int gpe_slice_pass(ism_problem*, int, double, double*, bool) { return ISM_E_UNSUPPORTED; }
int gpe_copy_state(ism_problem*, double*, int) { return ISM_E_UNSUPPORTED; }
size_t gpe_footprint_extra(size_t, int, int, int, int) { return 0; }
}  // namespace ism

extern "C" int ism_problem_create_gpe(ism_problem** out, int n_grid, double L, double g,
                                      const double* V0, const double* V1, double V2,
                                      const double* psi0, const double* target, double T, int K,
                                      int N, const ism_options* opt) {
    (void)out; (void)n_grid; (void)L; (void)g; (void)V0; (void)V1; (void)V2; (void)psi0;
    (void)target; (void)T; (void)K; (void)N; (void)opt;
    return ISM_E_UNSUPPORTED;
}
