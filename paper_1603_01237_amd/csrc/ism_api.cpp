// libism host runtime: argument validation, problem set-up, device memory, launch
// sequencing of the ISM iteration (Algorithm 1), status codes.  No C++ exception
// leaves this file.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <new>
#include <vector>

#include "ism_internal.h"
#include "ism_paths.h"

using ism::dcx;

namespace {

int hip_status(hipError_t e) {
    if (e == hipSuccess) return ISM_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return ISM_E_NOMEM;
    return ISM_E_DEVICE;
}

#define ISM_TRY_HIP(expr)                            \
    do {                                             \
        const hipError_t e__ = (expr);               \
        if (e__ != hipSuccess) return hip_status(e__); \
    } while (0)

bool finite_all(const double* x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

// Hermitian to 1e-12 relative to the largest entry.
bool hermitian(const double* H, int d) {
    double mx = 0.0;
    for (int i = 0; i < 2 * d * d; ++i) mx = std::max(mx, fabs(H[i]));
    const double tol = 1e-12 * std::max(1.0, mx);
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            const double ar = H[2 * (r * d + c)], ai = H[2 * (r * d + c) + 1];
            const double br = H[2 * (c * d + r)], bi = H[2 * (c * d + r) + 1];
            if (fabs(ar - br) > tol || fabs(ai + bi) > tol) return false;
        }
    return true;
}

}  // namespace

namespace ism {

const char* const kKernelNames[KID_COUNT] = {
    "sp_params", "sp_assemble", "sp_boundary", "sp_slice", "check_finite",
    "gate_build", "gate_gemm", "gate_grad", "gate_boundary",
    "gpe_sweep", "gpe_slice", "gpe_boundary", "sp_sweep", "err", "small_solve", "gpe_assemble"};

static hipEvent_t pool_get(ism_problem* p) {
    if (!p->event_pool.empty()) {
        hipEvent_t e = p->event_pool.back();
        p->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

TimeScope::TimeScope(ism_problem* prob, int k) : p(prob), kid(k) {
    if (!p->timing) return;
    e1 = pool_get(p);
    if (e1) hipEventRecord(e1, p->stream);
}

TimeScope::~TimeScope() {
    if (!p->timing || !e1) return;
    hipEvent_t e2 = pool_get(p);
    if (!e2) return;
    hipEventRecord(e2, p->stream);
    p->timed.push_back({kid, {e1, e2}});
}

int dev_alloc(ism_problem* p, void** ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) bytes = 16;
    const hipError_t e = p->async_alloc ? hipMallocAsync(ptr, bytes, p->stream) : hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        return hip_status(e);
    }
    p->allocs.push_back(*ptr);
    p->bytes += bytes;
    return ISM_OK;
}

int dev_upload(ism_problem* p, void** ptr, const void* host, size_t bytes) {
    int st = dev_alloc(p, ptr, bytes);
    if (st) return st;
    const hipError_t e = hipMemcpyAsync(*ptr, host, bytes, hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return hip_status(e);
    return hipStreamSynchronize(p->stream) == hipSuccess ? ISM_OK : ISM_E_DEVICE;
}

int copy_out(ism_problem* p, void* dst, const void* src, size_t bytes) {
    const hipMemcpyKind kind = p->io_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    ISM_TRY_HIP(hipMemcpyAsync(dst, src, bytes, kind, p->stream));
    if (!p->io_device) ISM_TRY_HIP(hipStreamSynchronize(p->stream));
    return ISM_OK;
}

// strided gather of B rows of `row` elements from a pitched device array
int copy_rows_out(ism_problem* p, void* dst, const void* src, size_t row_bytes, size_t src_pitch,
                  int rows) {
    const hipMemcpyKind kind = p->io_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    ISM_TRY_HIP(hipMemcpy2DAsync(dst, row_bytes, src, src_pitch, row_bytes, rows, kind, p->stream));
    if (!p->io_device) ISM_TRY_HIP(hipStreamSynchronize(p->stream));
    return ISM_OK;
}

int read_flags(ism_problem* p, int* host_flags) {
    ISM_TRY_HIP(hipMemcpyAsync(host_flags, p->flags, 4 * sizeof(int), hipMemcpyDeviceToHost,
                               p->stream));
    ISM_TRY_HIP(hipStreamSynchronize(p->stream));
    return ISM_OK;
}

int common_setup(ism_problem* p, int d, int C, double T, int K, int N, const ism_options* o) {
    p->precision = o->precision;
    p->kind = o->kind;
    p->step_cn = o->step_map == ISM_STEP_CN ? 1 : 0;
    p->B = o->batch;
    p->d = d;
    p->C = C;
    p->T = T;
    p->K = K;
    p->N = N;
    p->tau = T / K;
    p->device = o->device;
    p->io_device = o->io_device;
    p->async_alloc = o->alloc_async != 0;
    p->launch_per_pass = o->launch_per_pass != 0;
    p->gpe_frozen = o->gpe_frozen != 0;
    ISM_TRY_HIP(hipSetDevice(o->device));
    if (o->stream) {
        p->stream = (hipStream_t)o->stream;
    } else {
        ISM_TRY_HIP(hipStreamCreate(&p->stream));
        p->own_stream = true;
    }
    int st;
    std::vector<int> s(N + 1);
    for (int n = 0; n <= N; ++n) s[n] = (int)(((long long)n * K) / N);
    if ((st = dev_upload(p, (void**)&p->s, s.data(), s.size() * sizeof(int)))) return st;
    // controls, plus zero padding: a kernel that prefetches the control of the step after a
    // slice's last may read one element past the end
    std::vector<double> u0((size_t)p->B * K * C + 8, 0.0);
    if ((st = dev_upload(p, (void**)&p->u, u0.data(), u0.size() * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&p->grad, (u0.size() - 8) * sizeof(double)))) return st;
    if (o->alpha) {
        std::vector<double> al(K);
        for (int j = 0; j < K; ++j) al[j] = o->alpha_len == 1 ? o->alpha[0] : o->alpha[j];
        bool any = false;
        for (double x : al) any |= (x != 0.0);
        if (any && (st = dev_upload(p, (void**)&p->alpha, al.data(), K * sizeof(double)))) return st;
    }
    if ((st = dev_alloc(p, (void**)&p->J, p->B * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&p->F, p->B * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&p->active, p->B * sizeof(int)))) return st;
    if ((st = dev_alloc(p, (void**)&p->flags, 4 * sizeof(int)))) return st;
    ISM_TRY_HIP(hipMemsetAsync(p->flags, 0, 4 * sizeof(int), p->stream));
    return ISM_OK;
}

int validate_common(int d, int C, double T, int K, int N, const ism_options* o) {
    if (d < 1 || C < 1 || K < 1 || N < 1 || N > K) return ISM_E_ARG;
    if (!(T > 0.0) || !std::isfinite(T)) return ISM_E_ARG;
    if (o->batch < 1 || (o->precision != ISM_FP64 && o->precision != ISM_FP32_MIXED)) return ISM_E_ARG;
    if (o->kind != ISM_STATE && o->kind != ISM_GATE && o->kind != ISM_DENSITY) return ISM_E_ARG;
    if (o->step_map != ISM_STEP_EXP && o->step_map != ISM_STEP_CN) return ISM_E_ARG;
    if (o->alpha) {
        if (o->alpha_len != 1 && o->alpha_len != K) return ISM_E_ARG;
        if (!finite_all(o->alpha, o->alpha_len)) return ISM_E_ARG;
    }
    return ISM_OK;
}

// ------------------------------------------------------------------------------
// sparse state path
// ------------------------------------------------------------------------------

static SpArgs sp_args(ism_problem* p, int assemble) {
    SpArgs a{};
    a.B = p->B;
    a.d = p->d;
    a.K = p->K;
    a.N = p->N;
    a.C = p->C;
    a.CG = p->CG;
    a.WC = p->WC;
    a.P = p->d <= 64 ? 64 / p->d : 1;     // items per wavefront (one item per workgroup beyond 64 rows)
    a.items_per_inst = assemble ? p->N * p->d : p->N;
    a.waves_per_inst = (a.items_per_inst + a.P - 1) / a.P;
    a.LMAX = (p->K + p->N - 1) / p->N;
    a.has_offdiag = p->has_offdiag;
    a.s = p->s;
    a.u = p->u;
    a.alpha = p->alpha;
    a.h0diag = p->h0diag;
    a.h0diag_stride = p->h0diag_stride;
    a.gcol = p->gcol;
    a.gval = p->gval;
    a.shift = p->shift;
    a.tp = p->tp;
    a.phi = p->phi;
    a.M = p->M;
    a.grad = nullptr;
    a.active = nullptr;
    a.rho = 0.0;
    a.update = 0;
    a.tau = p->tau;
    a.T = p->T;
    a.cn = p->step_cn;
    a.mmax = p->tri ? kTriMaxTerms : 0;
    return a;
}

static int sp_boundary_pass(ism_problem* p, double* Jhist_k, double fid_stop, bool use_active) {
    SpArgs a = sp_args(p, 1);
    {
        TimeScope ts(p, KID_SP_PARAMS);
        ISM_TRY_HIP(sp_launch_params(a, p->h0norm, p->gnorm, p->precision, p->stream, p->flags));
    }
    {
        TimeScope ts(p, KID_SP_ASSEMBLE);
        if (p->tri)
            ISM_TRY_HIP(sp_launch_assemble_tri(a, p->precision, p->stream));
        else
            ISM_TRY_HIP(sp_launch_assemble(a, p->variant, p->precision, p->stream));
    }
    BndArgs bnd{};
    bnd.B = p->B;
    bnd.d = p->d;
    bnd.K = p->K;
    bnd.N = p->N;
    bnd.C = p->C;
    bnd.s = p->s;
    bnd.M = p->M;
    bnd.m_fp32 = p->precision == ISM_FP32_MIXED;
    bnd.shift = p->shift;
    bnd.psi0 = p->psi0;
    bnd.target = p->target;
    bnd.Psi = p->Psi;
    bnd.Lam = p->Lam;
    bnd.phi = p->phi;
    bnd.u = p->u;
    bnd.alpha = p->alpha;
    bnd.tau = p->tau;
    bnd.T = p->T;
    bnd.J = p->J;
    bnd.F = p->F;
    bnd.Jhist = Jhist_k;
    bnd.active = use_active ? p->active : nullptr;
    bnd.fid_stop = fid_stop;
    bnd.flags = p->flags;
    {
        TimeScope ts(p, KID_SP_BOUNDARY);
        ISM_TRY_HIP(sp_launch_boundary(bnd, p->stream));
    }
    p->bvalid = true;
    p->tp_valid = true;
    return ISM_OK;
}

static int sp_slice_pass(ism_problem* p, int update, double rho, double* grad, bool use_active) {
    if (!p->tp_valid) {        // boundaries from the one-launch solve: no Taylor parameters yet
        SpArgs ap = sp_args(p, 1);
        TimeScope ts(p, KID_SP_PARAMS);
        ISM_TRY_HIP(sp_launch_params(ap, p->h0norm, p->gnorm, p->precision, p->stream, p->flags));
        p->tp_valid = true;
    }
    SpArgs a = sp_args(p, 0);
    a.update = update;
    a.rho = rho;
    a.grad = grad;
    a.active = use_active ? p->active : nullptr;
    {
        TimeScope ts(p, KID_SP_SLICE);
        if (p->tri)
            ISM_TRY_HIP(sp_launch_slice_tri(a, p->precision, p->stream));
        else
            ISM_TRY_HIP(sp_launch_slice(a, p->variant, p->precision, p->stream));
    }
    if (update) p->bvalid = false;
    return ISM_OK;
}

static int sp_create(ism_problem* p, const double* H0, int h0_batched, const double* Hc,
                     const double* psi0, const double* target) {
    const int d = p->d, C = p->C, B = p->B;
    const int nH0 = h0_batched ? B : 1;
    // diagonal of H0 per instance; off-diagonal part must be shared
    std::vector<double> diag((size_t)nH0 * d);
    bool offdiag = false;
    for (int b = 0; b < nH0; ++b) {
        const double* H = H0 + (size_t)b * 2 * d * d;
        for (int r = 0; r < d; ++r) {
            diag[(size_t)b * d + r] = H[2 * (r * d + r)];
            for (int c = 0; c < d; ++c) {
                if (c == r) continue;
                const double* e = H + 2 * (r * d + c);
                const double* e0 = H0 + 2 * (r * d + c);
                if (e[0] != 0.0 || e[1] != 0.0) offdiag = true;
                if (e[0] != e0[0] || e[1] != e0[1]) return ISM_E_UNSUPPORTED;
            }
        }
    }
    const int CG = C + (offdiag ? 1 : 0);
    // generators in ELL form (entries per row up to WC)
    std::vector<std::vector<std::vector<std::pair<int, dcx>>>> rows(
        CG, std::vector<std::vector<std::pair<int, dcx>>>(d));
    bool realh = true;
    int WC = 1;
    for (int g = 0; g < CG; ++g) {
        const double* G = g < C ? Hc + (size_t)g * 2 * d * d : H0;
        for (int r = 0; r < d; ++r) {
            for (int c = 0; c < d; ++c) {
                if (g == C && c == r) continue;  // H0 diagonal is handled separately
                const double re = G[2 * (r * d + c)], im = G[2 * (r * d + c) + 1];
                if (re != 0.0 || im != 0.0) {
                    rows[g][r].push_back({c, dcx{re, im}});
                    if (im != 0.0) realh = false;
                }
            }
            WC = std::max<int>(WC, (int)rows[g][r].size());
        }
    }
    const int vi = sp_variant_index(CG, WC, realh ? 1 : 0, d);
    if (vi < 0) return ISM_E_UNSUPPORTED;
    if (p->step_cn && !sp_variant_cn(vi)) return ISM_E_UNSUPPORTED;
    // one real control operator with entries only at (r, r +- 1) and a diagonal H0
    bool tri = CG == 1 && realh && !offdiag && WC <= 2 && sp_tri_supported(d);
    for (int r = 0; tri && r < d; ++r)
        for (const auto& e : rows[0][r])
            if (e.first != r - 1 && e.first != r + 1) tri = false;
    p->tri = tri ? 1 : 0;
    p->CG = CG;
    p->WC = WC;
    p->has_offdiag = offdiag ? 1 : 0;
    p->realh = realh ? 1 : 0;
    p->variant = vi;
    std::vector<int> gcol((size_t)CG * d * WC, 0);
    std::vector<dcx> gval((size_t)CG * d * WC, dcx{0.0, 0.0});
    std::vector<double> gnorm(CG, 0.0);
    for (int g = 0; g < CG; ++g)
        for (int r = 0; r < d; ++r) {
            double rs = 0.0;
            for (size_t w = 0; w < rows[g][r].size(); ++w) {
                gcol[((size_t)g * d + r) * WC + w] = rows[g][r][w].first;
                gval[((size_t)g * d + r) * WC + w] = rows[g][r][w].second;
                rs += std::hypot(rows[g][r][w].second.re, rows[g][r][w].second.im);
            }
            for (size_t w = rows[g][r].size(); w < (size_t)WC; ++w) gcol[((size_t)g * d + r) * WC + w] = r;
            gnorm[g] = std::max(gnorm[g], rs);
        }
    std::vector<double> shift(B), h0norm(B);
    for (int b = 0; b < B; ++b) {
        const double* dg = diag.data() + (size_t)(h0_batched ? b : 0) * d;
        const double mx = *std::max_element(dg, dg + d), mn = *std::min_element(dg, dg + d);
        if (p->step_cn) {              // the Cayley map takes no spectral shift
            shift[b] = 0.0;
            h0norm[b] = std::max(fabs(mx), fabs(mn));
        } else {
            shift[b] = 0.5 * (mx + mn);
            h0norm[b] = 0.5 * (mx - mn);
        }
    }
    int st;
    if ((st = dev_upload(p, (void**)&p->h0diag, diag.data(), diag.size() * sizeof(double)))) return st;
    p->h0diag_stride = h0_batched ? d : 0;
    if ((st = dev_upload(p, (void**)&p->gcol, gcol.data(), gcol.size() * sizeof(int)))) return st;
    if ((st = dev_upload(p, (void**)&p->gval, gval.data(), gval.size() * sizeof(dcx)))) return st;
    if ((st = dev_upload(p, (void**)&p->gnorm, gnorm.data(), CG * sizeof(double)))) return st;
    if ((st = dev_upload(p, (void**)&p->shift, shift.data(), B * sizeof(double)))) return st;
    if ((st = dev_upload(p, (void**)&p->h0norm, h0norm.data(), B * sizeof(double)))) return st;
    if ((st = dev_upload(p, (void**)&p->psi0, psi0, d * sizeof(dcx)))) return st;
    if ((st = dev_upload(p, (void**)&p->target, target, d * sizeof(dcx)))) return st;
    if ((st = dev_alloc(p, (void**)&p->tp, B * sizeof(TaylorP)))) return st;
    const size_t nb = (size_t)B * (p->N + 1) * d * sizeof(dcx);
    if ((st = dev_alloc(p, (void**)&p->Psi, nb))) return st;
    if ((st = dev_alloc(p, (void**)&p->Lam, nb))) return st;
    if ((st = dev_alloc(p, (void**)&p->phi, nb))) return st;
    const size_t msz = (size_t)B * p->N * d * d * 2 *
                       (p->precision == ISM_FP64 ? sizeof(double) : sizeof(float));
    if ((st = dev_alloc(p, &p->M, msz))) return st;
    // small state problems take the one-launch solve in both precisions: it computes in
    // FP64, and its time is set by the serial chains of the slices, not by arithmetic
    if (!p->step_cn && d <= kSmallD && C <= kSmallC && p->N <= kSmallN) {
        if ((st = small_setup(p, H0, h0_batched, Hc))) return st;
        p->small = true;
    }
    return ISM_OK;
}

// ------------------------------------------------------------------------------
// path dispatch
// ------------------------------------------------------------------------------

int boundary_pass(ism_problem* p, double* Jhist_k, double fid_stop, bool use_active) {
    switch (p->path) {
        case PATH_SPARSE:
            // small FP64 problems: the boundaries of the one-launch solve, so that every entry
            // point sees the same J, F and intermediate states as its iterations
            if (small_eligible(p))
                return small_run(p, 0, 0.0, fid_stop, Jhist_k, nullptr, true, use_active);
            return sp_boundary_pass(p, Jhist_k, fid_stop, use_active);
        case PATH_GATE: return gate_boundary_pass(p, Jhist_k, fid_stop, use_active);
        case PATH_GPE: return gpe_boundary_pass(p, Jhist_k, fid_stop, use_active);
    }
    return ISM_E_STATE;
}

int slice_pass(ism_problem* p, int update, double rho, double* grad, bool use_active) {
    switch (p->path) {
        case PATH_SPARSE: return sp_slice_pass(p, update, rho, grad, use_active);
        case PATH_GATE: return gate_slice_pass(p, update, rho, grad, use_active);
        case PATH_GPE: return gpe_slice_pass(p, update, rho, grad, use_active);
    }
    return ISM_E_STATE;
}

// Per-step data at the current controls, for a slice pass that follows an update without a
// boundary rebuild in between: Taylor / Neumann parameters (sparse path), step propagators and
// in-slice products (gate path); the GPE slice kernel builds its steps from u itself.
int refresh_steps(ism_problem* p) {
    switch (p->path) {
        case PATH_SPARSE: {
            SpArgs a = sp_args(p, 0);
            TimeScope ts(p, KID_SP_PARAMS);
            ISM_TRY_HIP(sp_launch_params(a, p->h0norm, p->gnorm, p->precision, p->stream, p->flags));
            return ISM_OK;
        }
        case PATH_GATE: return gate_refresh_pass(p);
        case PATH_GPE: return ISM_OK;
    }
    return ISM_E_STATE;
}

// number of complex entries of one state (psi(T), chi(0)) per instance
size_t state_elems(const ism_problem* p) {
    if (p->path == PATH_GATE) return (size_t)p->d * p->d;
    return (size_t)p->d;
}

int copy_boundary_state(ism_problem* p, double* out, int which_end) {
    if (p->path == PATH_GATE) return gate_copy_state(p, out, which_end);
    if (p->path == PATH_GPE) return gpe_copy_state(p, out, which_end);
    const size_t e = state_elems(p);
    const dcx* base = which_end == 0 ? p->Psi + (size_t)p->N * e : p->Lam;
    return copy_rows_out(p, out, base, e * sizeof(dcx), (size_t)(p->N + 1) * e * sizeof(dcx), p->B);
}

// Start of a served solve: every instance active, flags cleared, boundary pass at the
// initial controls (J, F and the freeze decision for the first update).
int serve_begin(ism_problem* p, double fid_stop) {
    std::vector<int> ones(p->B, 1);
    ISM_TRY_HIP(hipMemcpyAsync(p->active, ones.data(), p->B * sizeof(int), hipMemcpyHostToDevice,
                               p->stream));
    ISM_TRY_HIP(hipStreamSynchronize(p->stream));      // `ones` is pageable and goes out of scope
    ISM_TRY_HIP(hipMemsetAsync(p->flags, 0, 4 * sizeof(int), p->stream));
    return boundary_pass(p, nullptr, fid_stop, true);
}

// n more iterations, enqueued with no host synchronisation: each is the slice pass with
// the update u += rho g (skipped by frozen instances) followed by the boundary pass at the
// new controls, so after the chunk J and F belong to the current u.  flags[1] counts the
// instances still active after each of the n boundary passes; count (device, nullable)
// accumulates per instance the updates it took.
int serve_chunk(ism_problem* p, int n, double rho, double fid_stop, int* count) {
    int st;
    ISM_TRY_HIP(hipMemsetAsync(p->flags, 0, 4 * sizeof(int), p->stream));
    if (small_eligible(p)) return small_run(p, n, rho, fid_stop, nullptr, count, false, true);
    for (int k = 0; k < n; ++k) {
        if ((st = slice_pass(p, 1, rho, nullptr, true))) return st;
        // the instances active in this slice pass took an update
        if (count) ISM_TRY_HIP(launch_count_active(count, p->active, p->B, p->stream));
        if ((st = boundary_pass(p, nullptr, fid_stop, true))) return st;
    }
    return ISM_OK;
}

}  // namespace ism

using namespace ism;

extern "C" {

void ism_default_options(ism_options* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->precision = ISM_FP64;
    o->kind = ISM_STATE;
    o->batch = 1;
    o->h0_batched = 0;
    o->alpha = nullptr;
    o->alpha_len = 0;
    o->device = 0;
    o->stream = nullptr;
    o->io_device = 0;
    o->alloc_async = 0;
    o->step_map = ISM_STEP_EXP;
    o->launch_per_pass = 0;
    o->gpe_frozen = 0;
}

const char* ism_status_string(int s) {
    switch (s) {
        case ISM_OK: return "ok";
        case ISM_E_ARG: return "invalid argument";
        case ISM_E_NOMEM: return "out of memory";
        case ISM_E_DEVICE: return "device error";
        case ISM_E_STATE: return "invalid call order";
        case ISM_E_NUMERIC: return "NaN or Inf in J or gradient";
        case ISM_E_UNSUPPORTED: return "unsupported problem";
        case ISM_E_BUDGET: return "memory budget exceeded";
    }
    return "unknown status";
}

void ism_problem_destroy(ism_problem* p) {
    if (!p) return;
    hipSetDevice(p->device);
    if (p->stream) hipStreamSynchronize(p->stream);
    if (p->ext_free) p->ext_free(p);
    for (auto& t : p->timed) {
        hipEventDestroy(t.second.first);
        hipEventDestroy(t.second.second);
    }
    for (hipEvent_t e : p->event_pool) hipEventDestroy(e);
    for (void* a : p->allocs) {
        if (p->async_alloc)
            (void)hipFreeAsync(a, p->stream);
        else
            (void)hipFree(a);
    }
    if (p->async_alloc && p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

int ism_problem_create(ism_problem** out, int d, int n_ctrl, const double* H0, const double* Hc,
                       const double* psi0, const double* target, double T, int K, int N,
                       const ism_options* opt) {
    if (!out || !H0 || !Hc || !psi0 || !target) return ISM_E_ARG;
    ism_options o;
    ism_default_options(&o);
    if (opt) o = *opt;
    int st = validate_common(d, n_ctrl, T, K, N, &o);
    if (st) return st;
    if (d > 256) return ISM_E_UNSUPPORTED;
    const int nH0 = o.h0_batched ? o.batch : 1;
    for (int b = 0; b < nH0; ++b)
        if (!finite_all(H0 + (size_t)b * 2 * d * d, (size_t)2 * d * d) ||
            !hermitian(H0 + (size_t)b * 2 * d * d, d))
            return ISM_E_ARG;
    for (int c = 0; c < n_ctrl; ++c)
        if (!finite_all(Hc + (size_t)c * 2 * d * d, (size_t)2 * d * d) ||
            !hermitian(Hc + (size_t)c * 2 * d * d, d))
            return ISM_E_ARG;
    const bool dense = o.kind == ISM_GATE || o.kind == ISM_DENSITY;
    const size_t se = dense ? (size_t)d * d : (size_t)d;
    if (!finite_all(psi0, 2 * se) || !finite_all(target, 2 * se)) return ISM_E_ARG;
    if (o.kind == ISM_DENSITY && (!hermitian(psi0, d) || !hermitian(target, d))) return ISM_E_ARG;

    ism_problem* p = new (std::nothrow) ism_problem();
    if (!p) return ISM_E_NOMEM;
    st = common_setup(p, d, n_ctrl, T, K, N, &o);
    if (!st) {
        if (dense) {
            p->path = PATH_GATE;
            st = gate_create(p, H0, o.h0_batched, Hc, psi0, target);
        } else {
            p->path = PATH_SPARSE;
            st = sp_create(p, H0, o.h0_batched, Hc, psi0, target);
        }
    }
    if (st) {
        ism_problem_destroy(p);
        return st;
    }
    *out = p;
    return ISM_OK;
}

int ism_set_controls(ism_problem* p, const double* u) {
    if (!p || !u) return ISM_E_ARG;
    ISM_TRY_HIP(hipSetDevice(p->device));
    const size_t bytes = (size_t)p->B * p->K * p->C * sizeof(double);
    if (!p->io_device) {
        if (!finite_all(u, bytes / sizeof(double))) return ISM_E_ARG;
        ISM_TRY_HIP(hipMemcpyAsync(p->u, u, bytes, hipMemcpyHostToDevice, p->stream));
        ISM_TRY_HIP(hipStreamSynchronize(p->stream));
    } else {
        ISM_TRY_HIP(hipMemcpyAsync(p->u, u, bytes, hipMemcpyDeviceToDevice, p->stream));
    }
    p->bvalid = false;
    return ISM_OK;
}

int ism_get_controls(ism_problem* p, double* u) {
    if (!p || !u) return ISM_E_ARG;
    ISM_TRY_HIP(hipSetDevice(p->device));
    return copy_out(p, u, p->u, (size_t)p->B * p->K * p->C * sizeof(double));
}

int ism_forward(ism_problem* p, double* psi_T) {
    if (!p) return ISM_E_ARG;
    ISM_TRY_HIP(hipSetDevice(p->device));
    int st = boundary_pass(p, nullptr, 2.0, false);
    if (st) return st;
    if (psi_T) return copy_boundary_state(p, psi_T, 0);
    return ISM_OK;
}

int ism_adjoint(ism_problem* p, double* chi_0) {
    if (!p) return ISM_E_ARG;
    ISM_TRY_HIP(hipSetDevice(p->device));
    if (!p->bvalid) {
        int st = boundary_pass(p, nullptr, 2.0, false);
        if (st) return st;
    }
    if (chi_0) return copy_boundary_state(p, chi_0, 1);
    return ISM_OK;
}

int ism_gradient(ism_problem* p, double* grad) {
    if (!p || !grad) return ISM_E_ARG;
    ISM_TRY_HIP(hipSetDevice(p->device));
    int st;
    ISM_TRY_HIP(hipMemsetAsync(p->flags, 0, 4 * sizeof(int), p->stream));
    if (!p->bvalid && (st = boundary_pass(p, nullptr, 2.0, false))) return st;
    if ((st = slice_pass(p, 0, 0.0, p->grad, false))) return st;
    const size_t n = (size_t)p->B * p->K * p->C;
    {
        TimeScope ts(p, KID_CHECK);
        ISM_TRY_HIP(launch_check_finite(p->grad, n, p->flags, p->stream));
    }
    int fl[4];
    if ((st = read_flags(p, fl))) return st;
    if (fl[0] & 2) return ISM_E_UNSUPPORTED;
    if (fl[0]) return ISM_E_NUMERIC;
    return copy_out(p, grad, p->grad, n * sizeof(double));
}

int ism_iterate(ism_problem* p, int n_iter, double rho, double fid_stop, double* J_hist,
                int* iters_done) {
    return ism_iterate_inner(p, n_iter, 1, rho, fid_stop, 0.0, J_hist, nullptr, iters_done);
}

int ism_iterate_inner(ism_problem* p, int n_iter, int n_inner, double rho, double fid_stop,
                      double err_stop, double* J_hist, double* Err_hist, int* iters_done) {
    if (!p || n_iter < 0 || n_inner < 1 || !std::isfinite(rho) || std::isnan(err_stop) ||
        std::isnan(fid_stop))
        return ISM_E_ARG;
    ISM_TRY_HIP(hipSetDevice(p->device));
    int st;
    const size_t need = (size_t)std::max(n_iter, 1) * p->B;
    if ((size_t)p->Jhist_cap < need) {
        double* nh = nullptr;
        if ((st = dev_alloc(p, (void**)&nh, need * sizeof(double)))) return st;
        p->Jhist = nh;
        p->Jhist_cap = (int)need;
    }
    const bool want_err = err_stop > 0.0 || Err_hist != nullptr;
    if (want_err && (size_t)p->Errhist_cap < need) {
        double* nh = nullptr;
        if ((st = dev_alloc(p, (void**)&nh, need * sizeof(double)))) return st;
        p->Errhist = nh;
        p->Errhist_cap = (int)need;
    }
    int done = 0;
    if (n_inner == 1 && !want_err && small_eligible(p)) {
        if ((st = small_iterate(p, n_iter, rho, fid_stop, p->Jhist, &done))) return st;
    } else if ((st = iterate_loop(p, n_iter, n_inner, rho, fid_stop, err_stop, p->Jhist,
                                  want_err ? p->Errhist : nullptr, false, &done))) {
        return st;
    }
    if (J_hist && n_iter > 0) {
        if ((st = copy_out(p, J_hist, p->Jhist, (size_t)n_iter * p->B * sizeof(double)))) return st;
    }
    if (Err_hist && done > 0) {
        if ((st = copy_out(p, Err_hist, p->Errhist, (size_t)done * p->B * sizeof(double)))) return st;
    }
    if (iters_done) *iters_done = done;
    return ISM_OK;
}

}  // extern "C"

namespace ism {

// ism_iterate as one launch (small FP64 state problems): active flags, flags and update
// counters cleared by fills, n_iter iterations, one host wait; done = the most updates any
// instance took, which is the iteration at which the per-pass loop ends.  Allocates nothing
// (ism_iterate_static uses it with its fixed history array).
int small_iterate(ism_problem* p, int n_iter, double rho, double fid_stop, double* jbuf,
                  int* done_out) {
    int st;
    *done_out = 0;
    if (n_iter == 0) return ISM_OK;
    ISM_TRY_HIP(launch_fill_i32(p->active, 1, p->B, p->stream));
    ISM_TRY_HIP(launch_fill_i32(p->flags, 0, 4, p->stream));
    ISM_TRY_HIP(launch_fill_i32(p->sm_count, 0, p->B, p->stream));
    if ((st = small_run(p, n_iter, rho, fid_stop, jbuf, p->sm_count, true, true))) return st;
    ISM_TRY_HIP(small_launch_done(p));
    int fl[4];
    if ((st = read_flags(p, fl))) return st;
    if (fl[0] & 2) return ISM_E_UNSUPPORTED;
    if (fl[0]) return ISM_E_NUMERIC;
    *done_out = fl[2];
    return ISM_OK;
}

// The iteration loop of Algorithm 1 (steps (a)-(e)) on history buffers the caller provides:
// jbuf holds n_iter * B doubles, ebuf (null unless Err is wanted) as many.  With `fills` the
// active flags and counters are set by a fill kernel rather than a host copy and
// hipMemsetAsync, so the loop touches no host memory besides the flags it reads back.
int iterate_loop(ism_problem* p, int n_iter, int n_inner, double rho, double fid_stop,
                 double err_stop, double* jbuf, double* ebuf, bool fills, int* done_out) {
    int st;
    const bool err_rule = err_stop > 0.0;
    if (fills) {
        ISM_TRY_HIP(launch_fill_i32(p->active, 1, p->B, p->stream));
        ISM_TRY_HIP(launch_fill_i32(p->flags, 0, 4, p->stream));
    } else {
        std::vector<int> ones(p->B, 1);
        ISM_TRY_HIP(hipMemcpyAsync(p->active, ones.data(), p->B * sizeof(int),
                                   hipMemcpyHostToDevice, p->stream));
        ISM_TRY_HIP(hipStreamSynchronize(p->stream));      // `ones` is pageable and goes out of scope
        ISM_TRY_HIP(hipMemsetAsync(p->flags, 0, 4 * sizeof(int), p->stream));
    }
    const bool check_stop = fid_stop <= 1.0 || err_rule;
    int done = 0;
    for (int k = 0; k < n_iter; ++k) {
        if (check_stop) {
            if (fills) ISM_TRY_HIP(launch_fill_i32(p->flags + 1, 0, 1, p->stream));
            else ISM_TRY_HIP(hipMemsetAsync(p->flags + 1, 0, sizeof(int), p->stream));
        }
        // steps (a)-(b): boundaries and intermediate states at u^(k); the condensate's
        // frozen-density mode assembles them from the last slice pass's trajectories
        if (p->path == PATH_GPE && p->gpe_frozen && k > 0)
            st = gpe_boundary_frozen_pass(p, jbuf + (size_t)k * p->B, fid_stop, true);
        else
            st = boundary_pass(p, jbuf + (size_t)k * p->B, fid_stop, true);
        if (st) return st;
        if (check_stop) {
            int fl[4];
            if ((st = read_flags(p, fl))) return st;
            if (fl[0] & 2) return ISM_E_UNSUPPORTED;
            if (fl[0]) return ISM_E_NUMERIC;
            if (fl[1] == 0) break;
        }
        // steps (c)-(d): n_inner gradient steps on every slice problem, phi^(k) held
        for (int l = 0; l < n_inner; ++l) {
            if (l > 0 && (st = refresh_steps(p))) return st;
            if ((st = slice_pass(p, 1, rho, nullptr, true))) return st;
        }
        // step (e): Err from the slice gradients at u^(k+1), phi^(k)
        if (ebuf) {
            if ((st = refresh_steps(p))) return st;
            if ((st = slice_pass(p, 0, 0.0, p->grad, true))) return st;
            TimeScope ts(p, KID_ERR);
            ISM_TRY_HIP(launch_err(p->grad, p->s, p->B, p->K, p->N, p->C, p->tau,
                                   p->path != PATH_GPE, ebuf + (size_t)k * p->B,
                                   err_rule ? p->active : nullptr, err_stop, p->flags, p->stream));
        }
        done = k + 1;
    }
    int fl[4];
    if ((st = read_flags(p, fl))) return st;
    if (fl[0] & 2) return ISM_E_UNSUPPORTED;
    if (fl[0]) return ISM_E_NUMERIC;
    *done_out = done;
    return ISM_OK;
}

}  // namespace ism

extern "C" {

int ism_fidelity(ism_problem* p, double* J, double* F) {
    if (!p) return ISM_E_ARG;
    ISM_TRY_HIP(hipSetDevice(p->device));
    int st;
    if (!p->bvalid && (st = boundary_pass(p, nullptr, 2.0, false))) return st;
    if (J && (st = copy_out(p, J, p->J, p->B * sizeof(double)))) return st;
    if (F && (st = copy_out(p, F, p->F, p->B * sizeof(double)))) return st;
    return ISM_OK;
}

int ism_problem_info(const ism_problem* p, ism_info* info) {
    if (!p || !info) return ISM_E_ARG;
    info->path = p->path;
    info->d = p->d;
    info->n_ctrl = p->C;
    info->K = p->K;
    info->N = p->N;
    info->batch = p->B;
    info->precision = p->precision;
    info->kind = p->kind;
    info->ell_width = p->WC;
    info->device_bytes = p->bytes;
    info->taylor_m = 0;
    info->taylor_S = 0;
    if (p->path == PATH_SPARSE && p->tp && p->tp_valid) {
        std::vector<TaylorP> tp(p->B);
        if (hipMemcpyAsync(tp.data(), p->tp, p->B * sizeof(TaylorP), hipMemcpyDeviceToHost,
                           p->stream) != hipSuccess ||
            hipStreamSynchronize(p->stream) != hipSuccess)
            return ISM_E_DEVICE;
        for (const TaylorP& t : tp) {
            info->taylor_m = std::max(info->taylor_m, t.m);
            info->taylor_S = std::max(info->taylor_S, t.S);
        }
    }
    return ISM_OK;
}

int ism_taylor_params(const ism_problem* p, int* m, int* S) {
    if (!p || !m || !S) return ISM_E_ARG;
    if (p->path != PATH_SPARSE) return ISM_E_UNSUPPORTED;
    if (!p->tp || !p->tp_valid) return ISM_E_STATE;
    std::vector<TaylorP> tp(p->B);
    if (hipSetDevice(p->device) != hipSuccess ||
        hipMemcpyAsync(tp.data(), p->tp, p->B * sizeof(TaylorP), hipMemcpyDeviceToHost,
                       p->stream) != hipSuccess ||
        hipStreamSynchronize(p->stream) != hipSuccess)
        return ISM_E_DEVICE;
    for (int b = 0; b < p->B; ++b) {
        m[b] = tp[b].m;
        S[b] = tp[b].S;
    }
    return ISM_OK;
}

int ism_set_timing(ism_problem* p, int enable) {
    if (!p) return ISM_E_ARG;
    p->timing = enable != 0;
    return ISM_OK;
}

int ism_kernel_times(ism_problem* p, ism_kernel_time* out, int max_entries, int* n_entries) {
    if (!p || (max_entries > 0 && !out)) return ISM_E_ARG;
    ISM_TRY_HIP(hipSetDevice(p->device));
    ISM_TRY_HIP(hipStreamSynchronize(p->stream));
    int launches[KID_COUNT] = {0};
    double ms[KID_COUNT] = {0.0};
    for (auto& t : p->timed) {
        float dt = 0.0f;
        if (hipEventElapsedTime(&dt, t.second.first, t.second.second) == hipSuccess) {
            launches[t.first] += 1;
            ms[t.first] += dt;
        }
        p->event_pool.push_back(t.second.first);
        p->event_pool.push_back(t.second.second);
    }
    p->timed.clear();
    int n = 0;
    for (int k = 0; k < KID_COUNT; ++k) {
        if (!launches[k]) continue;
        if (n < max_entries) {
            out[n].name = kKernelNames[k];
            out[n].launches = launches[k];
            out[n].total_ms = ms[k];
        }
        ++n;
    }
    if (n_entries) *n_entries = n < max_entries ? n : max_entries;
    return ISM_OK;
}

size_t ism_problem_footprint(int d, int n_ctrl, int K, int N, int batch, int kind, int precision,
                             int gpe_grid) {
    if (d < 1 || n_ctrl < 1 || K < 1 || N < 1 || N > K || batch < 1) return 0;
    const size_t B = batch, KC = (size_t)K * n_ctrl;
    const size_t rs = precision == ISM_FP64 ? 8 : 4;
    size_t bytes = B * KC * 8 * 2 + K * 8 + (N + 1) * 4 + B * 64;   // u, grad, alpha, s, J/F/flags
    if (gpe_grid > 0) {      // (frozen-density mode: gpe_frozen_bytes more)
        const size_t n = gpe_grid;
        return bytes + 4 * n * 8 + 2 * n * 16 +
               gpe_footprint_extra(n, K, N, batch, precision);
    }
    if (kind == ISM_GATE || kind == ISM_DENSITY)
        return bytes + gate_footprint_extra(d, n_ctrl, K, N, batch, precision);
    const size_t dd = d;
    bytes += 3 * B * (N + 1) * dd * 16;              // Psi, Lam, phi
    bytes += B * N * dd * dd * 2 * rs;               // slice propagators
    bytes += (size_t)(n_ctrl + 1) * dd * 8 * 24 + B * 64;   // generators, params
    // one-launch solve of small problems (either precision)
    if (small_workspace_bytes(d, n_ctrl, K, N, batch))
        bytes += small_workspace_bytes(d, n_ctrl, K, N, batch) + B * 32 +
                 (size_t)batch * (n_ctrl + 1) * kSmallD * kSmallD * 16;
    return bytes;
}

}  // extern "C"
