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
// the path's boundary pass (steps (a)-(b), J row at Jhist_k) and slice pass (gradients into
// grad, the update u += rho g when `update`), ism_api.cpp
int boundary_pass(ism_problem* p, double* Jhist_k, double fid_stop, bool use_active);
int slice_pass(ism_problem* p, int update, double rho, double* grad, bool use_active);

// the iteration loop of ism_iterate_inner on caller-provided history buffers (ism_api.cpp);
// `fills` clears flags with launch_fill_i32 instead of host copies and hipMemsetAsync
int iterate_loop(ism_problem* p, int n_iter, int n_inner, double rho, double fid_stop,
                 double err_stop, double* jbuf, double* ebuf, bool fills, int* done_out);
// x[0..n) = v by a kernel (ism_static.hip)
hipError_t launch_fill_i32(int* x, int v, int n, hipStream_t st);
// count[b] += (active[b] != 0), b < n (ism_static.hip)
hipError_t launch_count_active(int* count, const int* active, int n, hipStream_t st);

// serving (ism_api.cpp): enqueue-only iteration steps, no host synchronisation
int serve_begin(ism_problem* p, double fid_stop);
int serve_chunk(ism_problem* p, int n, double rho, double fid_stop, int* count = nullptr);

// one-launch solve of small FP64 state problems (k_small.hip): every iteration of every
// instance in one launch, one workgroup per instance
bool small_eligible(const ism_problem* p);
size_t small_workspace_bytes(int d, int C, int K, int N, int B);
int small_setup(ism_problem* p, const double* H0, int h0_batched, const double* Hc);
// first_boundary: B_0 (J row 0) then n x (slice pass with update, boundary; J row k+1 while
// k+1 < n); otherwise n x (slice pass, boundary) after a boundary of an earlier launch.
// count (device, nullable) accumulates the updates per instance.
// use_active: frozen instances skip the launch, freezes at fid_stop are recorded and flags[1]
// counts the instances still active; otherwise every instance runs and the flags stay as they are.
int small_run(ism_problem* p, int n_iter, double rho, double fid_stop, double* jhist,
              int* count, bool first_boundary, bool use_active);
// flags[2] = max over instances of the handle's update counters (sm_count)
hipError_t small_launch_done(ism_problem* p);
// ism_iterate on the one-launch solve (ism_api.cpp)
int small_iterate(ism_problem* p, int n_iter, double rho, double fid_stop, double* jbuf,
                  int* done_out);

// per-slice vector operations of the Newton slice solver (k_newton.hip); vectors laid out as
// the controls (B x K x C), one reduction per (instance, slice) in a fixed order
hipError_t nw_dot(const double* x, const double* y, const int* s, int B, int K, int N, int C,
                  double* out, int ostride, hipStream_t st);
hipError_t nw_sub(double* y, const double* x, const int* s, int B, int K, int N, int C,
                  const double* coef, int cstride, hipStream_t st);
hipError_t nw_normalize(double* y, const double* x, const int* s, int B, int K, int N, int C,
                        const double* nn, double* nrm, int nstride, const double* ref,
                        double sign, int* kdim, int it, hipStream_t st);
hipError_t nw_lincomb(double* u, const double* u0, const double* v, double a, size_t n,
                      hipStream_t st);
hipError_t nw_diff(double* w, const double* gp, const double* gm, double h, size_t n,
                   hipStream_t st);
hipError_t nw_lsq(double* H, const double* beta, const int* kdim, int m, int nslices, double* y,
                  hipStream_t st);
hipError_t nw_apply(double* u, const double* V, size_t vstride, const int* s, int B, int K,
                    int N, int C, const double* y, int m, const int* active, hipStream_t st);

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
// boundaries by frozen-density propagator assembling, densities of the last slice pass
int gpe_boundary_frozen_pass(ism_problem* p, double* Jhist_k, double fid_stop, bool use_active);
size_t gpe_frozen_bytes(size_t n, int N, int batch);
int gpe_slice_pass(ism_problem* p, int update, double rho, double* grad, bool use_active);
int gpe_copy_state(ism_problem* p, double* out, int which_end);
size_t gpe_footprint_extra(size_t n, int K, int N, int batch, int precision);

}  // namespace ism
