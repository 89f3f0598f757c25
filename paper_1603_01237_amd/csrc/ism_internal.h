// Internal definitions shared by the libism host runtime and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "libism.h"

namespace ism {

struct dcx { double re, im; };   // interleaved complex, same layout as the ABI's double pairs

// largest Taylor degree of the tridiagonal kernels, whose Horner series are unrolled
constexpr int kTriMaxTerms = 12;
// limits of the one-launch solve of small FP64 state problems (k_small.hip)
constexpr int kSmallD = 4, kSmallC = 4, kSmallN = 64;
// most GMRES steps of the Newton slice solver (ism_newton.cpp)
constexpr int kNewtonMaxM = 32;

// device buffers of the Newton slice solver, kept by the handle for the GMRES size m
struct NewtonBufs {
    int m = 0;
    double* V = nullptr;     // (m + 1) x BKC Arnoldi vectors
    double* G = nullptr;     // BKC: slice gradients at u^(k)
    double* Gp = nullptr;    // BKC
    double* Gm = nullptr;    // BKC
    double* W = nullptr;     // BKC
    double* u0 = nullptr;    // BKC
    double* H = nullptr;     // B N (m + 1) m Hessenberg matrices, column-major per slice
    double* beta = nullptr;  // B N
    double* wn = nullptr;    // B N: ||A v_i||^2 before the orthogonalisation
    double* nn = nullptr;    // B N
    double* y = nullptr;     // B N m
    int* kdim = nullptr;     // B N: Krylov dimension at a breakdown, -1 otherwise
};
struct fcx { float re, im; };

enum Path { PATH_SPARSE = 0, PATH_GATE = 1, PATH_GPE = 2 };

// Per-instance parameters of the Taylor action of exp(-i tau (H - s)):
// S sub-steps of length tau_sub = tau/S, m terms each.
struct TaylorP {
    int m;
    int S;
    double tau_sub;
};

// Arguments of the sparse-path kernels (one item = the rows of one d-vector held by
// d consecutive lanes of a wavefront; P items per wavefront).
struct SpArgs {
    int B, d, K, N, C, CG, WC;
    int P;                 // items per wavefront
    int waves_per_inst;    // wavefronts per instance
    int items_per_inst;    // N (slice kernel) or N*d (assembly kernel)
    int LMAX;              // longest slice (ceil(K/N))
    int has_offdiag;       // generator CG-1 is the off-diagonal part of H0 (control value 1)
    const int* s;          // N+1 slice starts
    double* u;             // B*K*C controls (read; updated in place when update != 0)
    const double* alpha;   // K penalty weights (nullptr => 0)
    const double* h0diag;  // diagonal of H0: B*d (h0diag_stride = d) or d (stride 0)
    int h0diag_stride;
    const int* gcol;       // CG*d*WC column of each stored entry (ELL)
    const dcx* gval;       // CG*d*WC value of each stored entry (0 for padding)
    const double* shift;   // B scalar shift s_b
    const TaylorP* tp;     // B
    const dcx* phi;        // B*(N+1)*d intermediate states
    void* M;               // B*N*d*d slice propagators, column-major per matrix, precision of the path
    double* grad;          // B*K*C (nullable)
    const int* active;     // B (nullable): 0 => instance frozen, no update
    double rho;
    int update;            // 1 => u += rho * g in place
    int cn;                // 1 => Crank-Nicolson step map (tp.m = Neumann terms, S = 1)
    int mmax;              // largest Taylor degree the kernels accept (more sub-steps beyond)
    double tau, T;
};

struct BndArgs {
    int B, d, K, N, C;
    const int* s;
    const void* M;         // phase-less slice propagators (column-major)
    int m_fp32;            // 1 if M holds float pairs
    const double* shift;   // B
    const dcx* psi0;       // d
    const dcx* target;     // d
    dcx* Psi;              // B*(N+1)*d
    dcx* Lam;              // B*(N+1)*d
    dcx* phi;              // B*(N+1)*d
    const double* u;       // B*K*C
    const double* alpha;   // K (nullable)
    double tau, T;
    double* J;             // B
    double* F;             // B
    double* Jhist;         // nullable: B values written at Jhist[0..B)
    int* active;           // nullable
    double fid_stop;
    int* flags;            // [0]: numeric error flag, [1]: number of active instances
};

// kernel classes for per-kernel timing
enum KernelId {
    KID_SP_PARAMS = 0, KID_SP_ASSEMBLE, KID_SP_BOUNDARY, KID_SP_SLICE, KID_CHECK,
    KID_GATE_BUILD, KID_GATE_GEMM, KID_GATE_GRAD, KID_GATE_BOUNDARY,
    KID_GPE_SWEEP, KID_GPE_SLICE, KID_GPE_BOUNDARY, KID_SP_SWEEP, KID_ERR, KID_SMALL_SOLVE,
    KID_GPE_ASSEMBLE, KID_COUNT
};
extern const char* const kKernelNames[KID_COUNT];

// Records HIP events around the launches issued in its scope when timing is enabled.
struct TimeScope {
    ism_problem* p;
    int kid;
    hipEvent_t e1 = nullptr;
    TimeScope(ism_problem* prob, int k);
    ~TimeScope();
};

// kernel launchers (k_sparse.hip)
int sp_variant_index(int CG, int WC, int realh, int d);
bool sp_variant_cn(int variant);     // variant compiled with the Crank-Nicolson map
hipError_t sp_launch_params(const SpArgs& a, const double* h0norm, const double* gnorm,
                            int precision, hipStream_t st, int* flags);
hipError_t sp_launch_assemble(const SpArgs& a, int variant, int precision, hipStream_t st);
// assembly for one real tridiagonal control operator and a diagonal H0 (several rows per lane)
hipError_t sp_launch_assemble_tri(const SpArgs& a, int precision, hipStream_t st);
hipError_t sp_launch_slice_tri(const SpArgs& a, int precision, hipStream_t st);
bool sp_tri_supported(int d);
hipError_t sp_launch_slice(const SpArgs& a, int variant, int precision, hipStream_t st);
hipError_t sp_launch_boundary(const BndArgs& a, hipStream_t st);
hipError_t launch_check_finite(const double* x, size_t n, int* flag, hipStream_t st);
// Err[b] of Algorithm 1 step (e) from the slice gradients g (B x K x C), which hold
// beta_n grad J_n (beta_scaled = 1) or grad J_n (0); freezes active instances with
// Err <= eta when eta > 0 and active is non-null
hipError_t launch_err(const double* grad, const int* s, int B, int K, int N, int C, double tau,
                      int beta_scaled, double* err, int* active, double eta, int* flags,
                      hipStream_t st);

}  // namespace ism

// The handle.  Fields are used by the host runtime only.
struct ism_problem {
    int path = 0, precision = 0, kind = 0;
    int d = 0, C = 0, K = 0, N = 0, B = 0;
    double T = 0, tau = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool async_alloc = false;   // stream-ordered allocation on `stream`
    int io_device = 0;
    size_t bytes = 0;
    std::vector<void*> allocs;

    // common device state
    double* u = nullptr;
    double* alpha = nullptr;
    int* s = nullptr;
    double* grad = nullptr;
    double* J = nullptr;
    double* F = nullptr;
    int* active = nullptr;
    int* flags = nullptr;
    double* Jhist = nullptr;
    int Jhist_cap = 0;
    double* Errhist = nullptr;
    int Errhist_cap = 0;
    bool bvalid = false;
    bool tp_valid = false;   // Taylor parameters computed at least once

    // sparse path
    int CG = 0, WC = 0, has_offdiag = 0, realh = 0, variant = -1;
    int tri = 0;               // generator is one real operator coupling rows r, r +- 1 only
    int step_cn = 0;           // Crank-Nicolson step map instead of the exponential
    double* h0diag = nullptr;
    int h0diag_stride = 0;
    int* gcol = nullptr;
    ism::dcx* gval = nullptr;
    double* shift = nullptr;
    double* h0norm = nullptr;
    double* gnorm = nullptr;
    ism::TaylorP* tp = nullptr;
    ism::dcx* psi0 = nullptr;
    ism::dcx* target = nullptr;
    ism::dcx* Psi = nullptr;
    ism::dcx* Lam = nullptr;
    ism::dcx* phi = nullptr;
    void* M = nullptr;

    // condensate: boundaries of iterations after the first by frozen-density assembling
    int gpe_frozen = 0;

    // one-launch solve of small FP64 state problems (k_small.hip)
    int launch_per_pass = 0;   // option: never use it
    bool small = false;        // set up at create (d, C, N within its limits)
    ism::dcx* sm_h = nullptr;  // (1 + C) padded generators per H0 instance, H0 shifted
    long long sm_hstride = 0;
    double* sm_shift = nullptr;
    double* sm_xnorm = nullptr;
    double* sm_cnorm = nullptr;
    ism::dcx* sm_work = nullptr;
    int* sm_count = nullptr;

    // Newton slice solver (ism_newton.cpp)
    ism::NewtonBufs nw;

    // per-kernel timing
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> timed;
    std::vector<hipEvent_t> event_pool;

    // path-specific extension (gate / GPE), owned by the respective module
    void* ext = nullptr;
    void (*ext_free)(ism_problem*) = nullptr;
};
