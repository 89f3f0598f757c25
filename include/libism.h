/*
 * libism -- Intermediate State Method (ISM) hot path on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only; no C++ types, no PyTorch types.
 *
 * Method (Riahi, Salomon, Glaser, Sugny, "A fully efficient time-parallelized
 * quantum optimal control algorithm"):
 *   dynamics   i d/dt psi = H(u) psi,  H(u) = H0 + sum_c u_c H_c        (Sec. 2, Eq. (dir))
 *   objective  J[u] = Re<psi(T)|psi_f> - alpha/2 int u^2                 (Sec. 2)
 *   K steps of length tau = T/K, control u_j constant on step j; the step map is
 *   the exact exponential exp(-i tau H(u_j)) (finite dimension) or Strang
 *   splitting (Gross-Pitaevskii, Sec. 3 Eq. (OS)).
 *   ISM (Algorithm 1): N time slices s_n = floor(n K / N); intermediate states
 *   phi_n = (T - t_n)/T psi(t_n) + t_n/T chi(t_n) (Eq. (cible)); every slice
 *   runs a forward sweep from phi_n and an adjoint sweep from phi_{n+1}, forms
 *   beta_n grad J_n = grad J (Theorem 2) and takes one constant-step gradient
 *   step (Eq. (gradStep), ascent); the boundary states psi(t_n), chi(t_n) are
 *   rebuilt from assembled slice propagators M_n by 2N matrix-vector products
 *   (propagator assembling, Sec. 3).  Gross-Pitaevskii uses the BEC variant of
 *   Sec. 4.C (slice starts on the forward trajectory, slice targets on the
 *   adjoint trajectory, boundaries by sequential sweeps).
 *
 * Conventions for every function below:
 *   - Complex numbers are interleaved pairs of doubles (re, im), C99
 *     "double _Complex" compatible; matrices are row-major.
 *   - The return value is an ism_status.  On error no output argument is written.
 *     No C++ exception crosses this interface.
 *   - A handle is not thread-safe; distinct handles may be used concurrently.
 *   - All device work is issued on the handle's stream in call order.  A call that
 *     writes a host pointer synchronises that stream before returning; with
 *     io_device = 1 the pointers are device pointers and the call does not
 *     synchronise (the result is ready in stream order).
 *   - The library allocates its own device memory at create time (and for the
 *     J history of ism_iterate); the caller keeps ownership of every buffer it
 *     passes in; inputs are copied.
 */
#ifndef LIBISM_H
#define LIBISM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ism_problem ism_problem;

typedef enum ism_status {
    ISM_OK = 0,
    ISM_E_ARG = 1,          /* invalid argument: shape, NULL pointer, non-Hermitian H, N > K ... */
    ISM_E_NOMEM = 2,        /* device or host allocation failed */
    ISM_E_DEVICE = 3,       /* a HIP runtime call failed */
    ISM_E_STATE = 4,        /* call order: e.g. a result requested that was never computed */
    ISM_E_NUMERIC = 5,      /* NaN or Inf in J or in the gradient */
    ISM_E_UNSUPPORTED = 6,  /* valid request this build does not handle (e.g. d too large) */
    ISM_E_BUDGET = 7        /* serving: request does not fit the memory budget */
} ism_status;

typedef enum ism_precision {
    ISM_FP64 = 0,           /* plain path: every step in FP64 */
    ISM_FP32_MIXED = 1      /* FP32 complex propagation with FP32 accumulate; per-step
                               generator data and all overlaps, gradients, boundary states,
                               J and F formed in FP64 (small state problems on the one-launch
                               solve compute in FP64 throughout; see launch_per_pass) */
} ism_precision;

typedef enum ism_kind {
    ISM_STATE = 0,          /* psi0, target are d-vectors; <a|b> = sum conj(a) b */
    ISM_GATE = 1,           /* psi0, target are d x d matrices (evolution operators, Sec. 2
                               remark); <A|B> = Tr(A^dagger B)/d */
    ISM_DENSITY = 2         /* psi0, target are Hermitian d x d operators evolving as
                               i d/dt rho = [H, rho] (the density-matrix formalism of the
                               five-spin run, Sec. 4.A): one step is rho <- U_j rho U_j^dagger,
                               <A|B> = Tr(A^dagger B), J = Re<rho(T)|rho_f> - penalty,
                               F = |<rho(T)|rho_f>|^2 / (<rho_0|rho_0><rho_f|rho_f>), gradient
                               Im Tr(Hhat_{c,j} [rho_j, lambda_j]).  Dense (MFMA) path, batch 1,
                               exponential step map only.  On the dense path (ISM_GATE and
                               ISM_DENSITY) the exact gradient's series is bounded: steps with
                               2 tau ||H_j - s||_inf above 1.46 (FP64) or 2.0 (FP32 mixed) make
                               ism_gradient / ism_iterate return ISM_E_UNSUPPORTED (s: the
                               midpoint of the diagonal of H0). */
} ism_kind;

typedef enum ism_step_map {
    ISM_STEP_EXP = 0,       /* psi_{j+1} = exp(-i tau H_j) psi_j, exact exponential */
    ISM_STEP_CN = 1         /* Crank-Nicolson (Sec. 3): (I + L_j) psi_{j+1} = (I - L_j) psi_j,
                               L_j = (i tau/2) H_j, with its exact gradient
                               1/2 Im<chi_j|H_c|psi_j + psi_{j+1}>, (I - L_j) chi_j = lambda_{j+1}.
                               State problems of the sparse path only; the inverse is applied as
                               a Neumann series, so tau ||H_j||_inf / 2 must stay below 0.25
                               (FP64) or 0.45 (FP32 mixed): steps beyond that make
                               ism_gradient / ism_iterate return ISM_E_UNSUPPORTED. */
} ism_step_map;

typedef struct ism_options {
    int precision;          /* ism_precision (default ISM_FP64) */
    int kind;               /* ism_kind (default ISM_STATE) */
    int batch;              /* number of independent instances B >= 1 (default 1) */
    int h0_batched;         /* 1: H0 holds B matrices (B x d x d), 0: one shared H0 (default 0) */
    const double* alpha;    /* penalty weight: NULL => alpha = 0; else alpha_len doubles */
    int alpha_len;          /* 1 (constant alpha) or K (alpha_j per step, e.g. a time-dependent
                               weight as in Sec. 4.B) */
    int device;             /* HIP device ordinal (default 0) */
    void* stream;           /* hipStream_t to issue work on; NULL => library-owned stream */
    int io_device;          /* 1: pointers of set/get_controls, forward, adjoint, gradient,
                               fidelity and the J history are device pointers (default 0) */
    int alloc_async;        /* 1: the handle's device memory is allocated and freed
                               stream-ordered on its stream (hipMallocAsync / hipFreeAsync), so
                               creating and destroying the handle never synchronises the whole
                               device (default 0: hipMalloc / hipFree) */
    int step_map;           /* ism_step_map of a state problem (default ISM_STEP_EXP) */
    int launch_per_pass;    /* 0 (default): small state problems (d <= 4, at most 4 controls
                               and 64 slices, exponential map) run ism_iterate and their served
                               iterations as one persistent launch, one workgroup per instance
                               holding every phase of Algorithm 1, in FP64 for both precisions
                               (the solve is bound by the serial chains of its slices, so an
                               FP32 mixed handle gains nothing from FP32 there); 1: always the
                               sequence of per-pass launches.  In FP64 both give the iterates
                               of Algorithm 1 to FP64 rounding (not bitwise the same). */
    int gpe_frozen;         /* condensate (ism_problem_create_gpe, n_grid 64 or 1024): 1 builds
                               the boundaries of every iteration after the first by
                               propagator assembling with the density frozen at the last
                               slice pass's trajectories (the reading of Sec. 4.C): per slice
                               the linear step maps S_j psi = Kh e^{-i tau (V(u_j)+g|a_j|^2)} Kh psi
                               and the exact adjoint steps linearised at those a_j, assembled
                               on basis vectors (n and 2n columns), then 2N matrix-vector
                               products.  The iterates then differ from the plain gradient
                               method's and share its fixed points; J^(k), F^(k) come from the
                               assembled Psi_N.  Holds 3 B N n^2 complex doubles on the device
                               from creation.  Default 0: exact sequential sweeps. */
} ism_options;

/* Fill *opt with the defaults listed above.  opt must not be NULL. */
void ism_default_options(ism_options* opt);

/*
 * Create a finite-dimensional problem (Sec. 2 statement of the problem; partition
 * of Sec. 2; time grid of Sec. 3).
 *   out     : receives the new handle.
 *   d       : Hilbert-space dimension, 1 <= d <= 256 for state problems (ISM_STATE),
 *             d <= 256 for gate (ISM_GATE) and density-matrix (ISM_DENSITY) problems.
 *   n_ctrl  : number of controls C >= 1.
 *   H0      : d x d complex (or B x d x d if opt->h0_batched), Hermitian to 1e-12 relative.
 *   Hc      : C x d x d complex, contiguous, each Hermitian.
 *   psi0    : initial state: d complex (ISM_STATE) or d x d (ISM_GATE, ISM_DENSITY; Hermitian
 *             for ISM_DENSITY); shared by all instances.
 *   target  : target psi_f, same shape as psi0.
 *   T       : final time > 0.
 *   K       : number of time steps >= 1 (tau = T/K).
 *   N       : number of ISM slices, 1 <= N <= K.
 *   opt     : options (NULL => defaults).
 * The initial controls are zero; set them with ism_set_controls.
 * Errors: ISM_E_ARG for NULL/invalid sizes/non-Hermitian input, ISM_E_UNSUPPORTED for
 * sizes outside the limits, ISM_E_NOMEM, ISM_E_DEVICE.
 */
int ism_problem_create(ism_problem** out, int d, int n_ctrl, const double* H0, const double* Hc,
                       const double* psi0, const double* target, double T, int K, int N,
                       const ism_options* opt);

/*
 * Create a 1-D Gross-Pitaevskii problem (Sec. 4.C; step map Eq. (OS)):
 *   i d/dt psi = (-1/2 d_xx + V(x,u) + g |psi|^2) psi,   V(x,u) = V0(x) + u V1(x) + u^2 V2,
 * on the periodic grid x_m = -L/2 + m L/n_grid, with one scalar control (C = 1).
 *   n_grid  : 64, 1024 or 4096 (LDS-resident FFT; 64 is the scale of the paper's own
 *             50-point grid).
 *   L       : box length > 0.   g : nonlinearity.
 *   V0, V1  : n_grid doubles each.   V2 : scalar.
 *   psi0, target : n_grid complex, normalised with <a|b> = dx sum conj(a) b.
 *   T, K, N : as above.   opt : precision, batch, device, stream, io_device and gpe_frozen
 *             are used (gpe_frozen with n_grid 4096: ISM_E_UNSUPPORTED).
 */
int ism_problem_create_gpe(ism_problem** out, int n_grid, double L, double g, const double* V0,
                           const double* V1, double V2, const double* psi0, const double* target,
                           double T, int K, int N, const ism_options* opt);

/* Free all device memory of the handle (NULL-safe). */
void ism_problem_destroy(ism_problem* p);

/* Controls u[B][K][C] (FP64), host or device pointer per io_device.  Setting the
 * controls invalidates the boundary states. */
int ism_set_controls(ism_problem* p, const double* u);
int ism_get_controls(ism_problem* p, double* u);

/*
 * Forward pass at the current controls: per-step propagator data, slice propagators
 * M_n (propagator assembling), boundary rebuild (2N products) and intermediate states
 * (Eq. (cible)), J and F.  psi_T (nullable) receives psi(T) per instance:
 * B x d complex (state), B x d x d (gate) or B x n_grid (GPE).
 */
int ism_forward(ism_problem* p, double* psi_T);

/* Adjoint at t = 0 (Eq. (adj) with chi(T) = psi_f): chi_0 (nullable) receives chi(0)
 * per instance, same shape as psi_T.  Runs ism_forward first if the boundaries are stale. */
int ism_adjoint(ism_problem* p, double* chi_0);

/*
 * Gradient g = (1/tau) dJ_tau/du (function-space gradient of Eq. (gradJ), exact for the
 * discrete step map), computed slice-parallel through Theorem 2:
 *   g_{j,c} = beta_n [ Im<chi^n_j|Hhat_{c,j}|psi^n_j> - alpha_{n,j} u_{j,c} ],
 * with Hhat the step average of H_c.  grad receives B x K x C doubles.
 * ISM_E_NUMERIC if any entry is NaN/Inf.
 */
int ism_gradient(ism_problem* p, double* grad);

/*
 * n_iter ISM iterations (Algorithm 1 with one constant-step gradient step per slice,
 * u <- u + rho g).  Iteration k records J^(k) (at u^k, before its update) in
 * J_hist[k*B + b] (nullable; n_iter*B doubles).  An instance whose fidelity
 * F = |<psi(T)|psi_f>|^2 reaches fid_stop is frozen (pass fid_stop > 1 to disable);
 * the loop ends early once every instance is frozen.  *iters_done (nullable) receives
 * the number of iterations the loop ran.  ISM_E_NUMERIC if J becomes NaN/Inf.
 */
int ism_iterate(ism_problem* p, int n_iter, double rho, double fid_stop, double* J_hist,
                int* iters_done);

/*
 * Allocation-free ism_iterate, for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.  Same arguments,
 * stopping rule, kernels and results as ism_iterate (bitwise, for the same handle state);
 * the J history the boundary kernels write lives in a fixed device array of the library,
 * ISM_STATIC_HIST_MAX doubles (1 MiB) on each GPU it runs on, held until the process ends,
 * instead of a buffer grown per handle; flags are cleared by a kernel, not a host copy.
 * The call allocates no device or host memory (the handle's buffers come from create).
 *   - ISM_E_BUDGET if max(n_iter, 1) * batch > ISM_STATIC_HIST_MAX; nothing runs.
 *   - J_hist receives the rows the loop wrote, J^(k) for k < *iters_done and the row of the
 *     iteration that stopped the loop early; later rows are left untouched.
 *   - Every call on one GPU shares that GPU's array: calls that overlap on a GPU (from
 *     several host threads, or on streams whose work runs concurrently) race.  Each call
 *     writes its rows before it reads them, so nothing from an earlier call is read.
 */
#define ISM_STATIC_HIST_MAX 131072
int ism_iterate_static(ism_problem* p, int n_iter, double rho, double fid_stop, double* J_hist,
                       int* iters_done);

/*
 * ISM iterations with several gradient steps per slice problem and the Err stopping rule
 * (Algorithm 1, steps (c) and (e); Eq. (gradStep) iterated).  Iteration k rebuilds the
 * boundaries and intermediate states phi^(k) at u^(k) (steps (a)-(b)), then every slice n
 * takes n_inner constant steps on its own problem max J_n[., phi^(k)] with phi^(k) held:
 *     u_n <- u_n + rho beta_n grad J_n[u_n, phi^(k)]                      (n_inner times)
 * (scaled by beta_n so that n_inner = 1 is exactly ism_iterate), and finally
 *     Err^(k) = sum_n tau sum_{j in slice n} || grad J_n[u^(k+1), phi^(k)]_j ||_2
 * (Euclidean norm over the controls of step j).  Gross-Pitaevskii problems use the slice
 * problems of the BEC variant (Sec. 4.C), whose gradients carry no beta_n.
 *   n_inner   >= 1 (else ISM_E_ARG).
 *   err_stop  eta > 0: an instance whose Err^(k) <= eta is frozen after iteration k, and
 *             the loop ends once every instance is frozen; <= 0: no Err rule.
 *   fid_stop, J_hist, iters_done: as ism_iterate.
 *   Err_hist  nullable; receives Err^(k) in Err_hist[k*B + b] for the *iters_done
 *             iterations run (entries past that are not written).  Err costs one more
 *             slice pass per iteration and is only computed when err_stop > 0 or
 *             Err_hist is non-NULL.
 * ISM_E_NUMERIC if J or Err becomes NaN/Inf; ISM_E_UNSUPPORTED as ism_iterate.
 */
int ism_iterate_inner(ism_problem* p, int n_iter, int n_inner, double rho, double fid_stop,
                      double err_stop, double* J_hist, double* Err_hist, int* iters_done);

/*
 * ISM iterations whose Step (c) is one Newton step per slice problem (Sec. 4.B: the
 * matrix-free Newton method with a GMRES solver, the paper's second slice solver for the
 * molecular-orientation runs).  Iteration k rebuilds the boundaries and intermediate states
 * phi^(k) at u^(k) (steps (a)-(b)); then every slice n solves
 *     A_n delta_n = -G_n,   G_n = beta_n grad J_n[u_n, phi^(k)],
 * A_n the Jacobian of G_n applied matrix-free as (G_n(u + eps v) - G_n(u - eps v)) / (2 eps),
 * by gmres_m steps of GMRES from delta_n = 0 (Euclidean inner product over the slice's
 * controls, modified Gram-Schmidt, no restart; a breakdown, h_{i+1,i} <= 1e-14 ||A v_i||,
 * ends that slice's Arnoldi early), and takes the full step u_n <- u_n + delta_n (no damping).
 * One Newton step costs 2 gmres_m + 1 slice passes.
 *   gmres_m   1 <= gmres_m <= 32 (else ISM_E_ARG).
 *   fd_eps    > 0, the difference step along unit vectors (1e-5 suits O(1) controls).
 *   fid_stop, J_hist, iters_done: as ism_iterate (J_hist rows past *iters_done + 1 are not
 *             written).
 * FP64 handles of the state, gate and density paths only (ISM_E_UNSUPPORTED otherwise: the
 * difference quotient needs FP64 gradients).  Device memory: (gmres_m + 6) B K C doubles and
 * B N (gmres_m + 2)^2 doubles, allocated on the first call with a larger gmres_m and held
 * by the handle.  ISM_E_NUMERIC if J becomes NaN/Inf.
 */
int ism_iterate_newton(ism_problem* p, int n_iter, int gmres_m, double fd_eps, double fid_stop,
                       double* J_hist, int* iters_done);

/* J = Re<psi(T)|psi_f> - tau/2 sum_j alpha_j |u_j|^2 and F = |<psi(T)|psi_f>|^2 per instance
 * (gate: Re Tr(W^+ U)/d and |Tr(W^+ U)|^2/d^2), B doubles each (either may be NULL).
 * Recomputes the boundaries if the controls changed since the last forward pass. */
int ism_fidelity(ism_problem* p, double* J, double* F);

/* Read-only description of a handle. */
typedef struct ism_info {
    int path;           /* 0 sparse state path, 1 dense gate path (MFMA), 2 GPE split-step */
    int d, n_ctrl, K, N, batch, precision, kind;
    int ell_width;      /* sparse path: stored nonzeros per row of H */
    size_t device_bytes;/* device memory held by the handle */
    int taylor_m;       /* sparse path: largest Taylor term count over instances at the last
                           forward pass (0 if none yet; reading it synchronises the stream) */
    int taylor_S;       /* sparse path: largest sub-step count, same convention */
} ism_info;
int ism_problem_info(const ism_problem* p, ism_info* info);

/* Sparse path: the series parameters of every instance at the last forward pass, Taylor
 * terms m[b] and sub-steps S[b] per step (exponential map) or Neumann terms m[b] and S[b] = 1
 * (Crank-Nicolson), b < batch; host arrays of batch ints, written after a synchronisation
 * of the handle's stream.  ISM_E_STATE before the first forward pass and on handles whose
 * boundaries come from the one-launch solve of small problems (which picks its series per
 * step; see launch_per_pass), ISM_E_UNSUPPORTED on the dense and Gross-Pitaevskii paths. */
int ism_taylor_params(const ism_problem* p, int* m, int* S);

/*
 * Per-kernel timing (tracing).  With timing enabled, every kernel launch of the handle is
 * bracketed by two HIP events recorded on the handle's stream.  ism_kernel_times
 * synchronises the stream, sums the event intervals per kernel name into
 * out[0..*n_entries) (at most max_entries; names are static strings) and clears the
 * record.  Timing adds two event records per launch and no synchronisation.
 */
typedef struct ism_kernel_time {
    const char* name;
    int launches;
    double total_ms;
} ism_kernel_time;
int ism_set_timing(ism_problem* p, int enable);
int ism_kernel_times(ism_problem* p, ism_kernel_time* out, int max_entries, int* n_entries);

/* Human-readable name of a status code (static storage). */
const char* ism_status_string(int status);

/* Device memory (bytes) a problem of this shape would hold; used for admission by
 * memory budget.  kind/precision as in ism_options; path chosen as ism_problem_create
 * would.  Returns 0 on invalid input. */
size_t ism_problem_footprint(int d, int n_ctrl, int K, int N, int batch, int kind, int precision,
                             int gpe_grid);

/*
 * Serving: many independent solves on one device.
 *
 * A solve request is a problem (the arguments of ism_problem_create or
 * ism_problem_create_gpe), initial controls and a stopping rule: run ISM iterations
 * (ism_iterate semantics, u <- u + rho g) until F = |<psi(T)|psi_f>|^2 >= fid_stop or
 * max_iter updates.  The server copies every input at submit time.  Requests are
 * admitted in arrival order while the device memory they would hold
 * (ism_problem_footprint, or the handle's actual bytes if larger) fits in hbm_budget.
 * The head of the queue is admitted together with every queued request that differs from
 * it only in the diagonal of H0 and the initial controls (finite state problems with the
 * same d, controls, psi0, target, off-diagonal H0, T, K, N, precision, rho, fid_stop and
 * max_iter), or, for a condensate request, only in the initial controls (same n_grid, L,
 * g, V0, V1, V2, psi0, target, T, K, N, precision, rho, fid_stop and max_iter); at most
 * 256: they run as the instances of one batched handle, so one set of launches serves them
 * all, and each instance freezes on its own.  Each such group has its own handle and HIP stream,
 * so the kernels of different groups overlap on the device.  Work is issued in chunks of
 * iters_per_round iterations with no host synchronisation; ism_server_progress polls the
 * chunks' events, finishes requests (copying their controls out), retires finished groups
 * (freeing their memory), admits waiting ones and issues the next chunks.  It never blocks
 * on device work, except inside handle creation and when a finished request's controls are
 * copied out.  A request's result does not depend on what else is being served: the
 * kernels compute every instance of a batch independently, with the arithmetic of its lone
 * run, so a merged request returns bitwise what it would alone.  An error inside a group
 * (a non-finite value, a device failure) fails all its running requests.
 *
 * A server is not thread-safe.  Time stamps are seconds on a monotonic clock
 * (ism_server_clock).
 */
typedef struct ism_server ism_server;

typedef enum ism_request_model {
    ISM_REQ_FINITE = 0,     /* finite-dimensional state or gate problem (ism_problem_create) */
    ISM_REQ_GPE = 1         /* Gross-Pitaevskii problem (ism_problem_create_gpe) */
} ism_request_model;

typedef struct ism_request {
    int model;              /* ism_request_model */
    int kind;               /* ism_kind (finite model) */
    int precision;          /* ism_precision */
    /* finite model: ism_problem_create arguments (d x d complex matrices, C of them in Hc) */
    int d, n_ctrl;
    const double* H0;
    const double* Hc;
    /* GPE model: ism_problem_create_gpe arguments */
    int n_grid;
    double L, g, V2;
    const double* V0;
    const double* V1;
    /* both: psi0 and target (d, d x d or n_grid complex), time grid and partition */
    const double* psi0;
    const double* target;
    double T;
    int K, N;
    const double* u0;       /* initial controls [K][C] (C = 1 for GPE) */
    int max_iter;           /* >= 0 updates at most */
    double rho;             /* gradient step (Eq. (gradStep), ascent) */
    double fid_stop;        /* stop once F >= fid_stop (> 1 disables) */
} ism_request;

typedef enum ism_request_state {
    ISM_REQ_QUEUED = 0,
    ISM_REQ_RUNNING = 1,
    ISM_REQ_DONE = 2,
    ISM_REQ_FAILED = 3
} ism_request_state;

typedef struct ism_result {
    int state;              /* ism_request_state */
    int status;             /* ism_status of a failed request (ISM_OK otherwise) */
    int iters;              /* updates performed so far */
    double J, F;            /* at the current controls (valid once DONE) */
    double t_arrival;       /* as passed to ism_server_submit */
    double t_admit;         /* handle created (0 while queued) */
    double t_done;          /* result available (0 before) */
    size_t device_bytes;    /* memory charged against the budget */
} ism_result;

typedef struct ism_server_stats {
    uint64_t submitted, completed, failed;
    int queued, running;    /* requests waiting / admitted and not finished */
    size_t bytes_in_use, bytes_peak;
    double busy_s;          /* time with at least one request running */
    uint64_t groups;        /* handles admitted so far (one per group of merged requests) */
    uint64_t merged;        /* requests admitted into another request's handle */
} ism_server_stats;

/* Monotonic clock in seconds, the time base of all server time stamps. */
double ism_server_clock(void);

/*
 * Create a server on `device` with a device-memory budget of hbm_budget bytes for the
 * admitted requests, iters_per_round iterations per issued chunk (>= 1) and at most
 * max_running requests in flight at once (>= 1).  Errors: ISM_E_ARG, ISM_E_NOMEM,
 * ISM_E_DEVICE.
 */
int ism_server_create(ism_server** out, int device, size_t hbm_budget, int iters_per_round,
                      int max_running);

/*
 * Queue a request; its inputs are copied before return.  t_arrival < 0 stamps it with
 * ism_server_clock().  *ticket receives its id.  ISM_E_ARG for missing or inconsistent
 * fields, ISM_E_BUDGET if its footprint exceeds the whole budget (it could never be
 * admitted).  Problems that are well-formed here but rejected by handle creation end
 * in state ISM_REQ_FAILED with that status.
 */
int ism_server_submit(ism_server* s, const ism_request* req, double t_arrival, uint64_t* ticket);

/* Poll the device, retire finished requests, admit and issue work (non-blocking, see
 * above).  n_queued / n_running (nullable) receive the counts after the call. */
int ism_server_progress(ism_server* s, int* n_queued, int* n_running);

/* State of a request (ISM_E_ARG for an unknown ticket). */
int ism_server_poll(ism_server* s, uint64_t ticket, ism_result* res);

/* Take a finished (DONE or FAILED) request: *res as ism_server_poll, u_out (nullable)
 * receives its final controls [K][C]; the server then forgets the ticket.
 * ISM_E_STATE if the request is still queued or running. */
int ism_server_take(ism_server* s, uint64_t ticket, ism_result* res, double* u_out);

int ism_server_stats_get(ism_server* s, ism_server_stats* st);

/* Wait for every running request's issued work, free everything (NULL-safe). */
void ism_server_destroy(ism_server* s);

#ifdef __cplusplus
}
#endif
#endif /* LIBISM_H */
