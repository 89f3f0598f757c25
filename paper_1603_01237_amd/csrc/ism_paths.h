// Per-path entry points used by the host runtime (ism_api.cpp).
#pragma once

#include "ism_internal.h"

namespace ism {

// shared host helpers (ism_api.cpp)
int dev_alloc(ism_problem* p, void** ptr, size_t bytes);
int dev_upload(ism_problem* p, void** ptr, const void* host, size_t bytes);
int copy_out(ism_problem* p, void* dst, const void* src, size_t bytes);
int copy_rows_out(ism_problem* p, void* dst, const void* src, size_t row_bytes, size_t src_pitch,
                  int rows);
int read_flags(ism_problem* p, int* host_flags);
int common_setup(ism_problem* p, int d, int C, double T, int K, int N, const ism_options* o);
int validate_common(int d, int C, double T, int K, int N, const ism_options* o);

// per-step data at the current controls without a boundary rebuild (ism_api.cpp)
int refresh_steps(ism_problem* p);

// the iteration loop of ism_iterate_inner on caller-provided history buffers (ism_api.cpp);
// `fills` clears flags with launch_fill_i32 instead of host copies and hipMemsetAsync
int iterate_loop(ism_problem* p, int n_iter, int n_inner, double rho, double fid_stop,
                 double err_stop, double* jbuf, double* ebuf, bool fills, int* done_out);
// x[0..n) = v by a kernel (ism_static.hip)
hipError_t launch_fill_i32(int* x, int v, int n, hipStream_t st);

// serving (ism_api.cpp): enqueue-only iteration steps, no host synchronisation
int serve_begin(ism_problem* p, double fid_stop);
int serve_chunk(ism_problem* p, int n, double rho, double fid_stop);

// dense gate path (k_gate.hip)
int gate_create(ism_problem* p, const double* H0, int h0_batched, const double* Hc,
                const double* psi0, const double* target);
int gate_boundary_pass(ism_problem* p, double* Jhist_k, double fid_stop, bool use_active);
int gate_slice_pass(ism_problem* p, int update, double rho, double* grad, bool use_active);
// per-step propagators and in-slice products at the current controls (no boundary rebuild)
int gate_refresh_pass(ism_problem* p);
int gate_copy_state(ism_problem* p, double* out, int which_end);
size_t gate_footprint_extra(int d, int C, int K, int N, int batch, int precision);

// Gross-Pitaevskii path (k_gpe.hip)
int gpe_create(ism_problem* p, int n_grid, double L, double g, const double* V0, const double* V1,
               double V2, const double* psi0, const double* target);
int gpe_boundary_pass(ism_problem* p, double* Jhist_k, double fid_stop, bool use_active);
int gpe_slice_pass(ism_problem* p, int update, double rho, double* grad, bool use_active);
int gpe_copy_state(ism_problem* p, double* out, int which_end);
size_t gpe_footprint_extra(size_t n, int K, int N, int batch, int precision);

}  // namespace ism
