// ism_iterate_newton: Algorithm 1 with Step (c) done by one Newton step per slice problem
// (Sec. 4.B), matrix-free, the Newton system A_n delta_n = -G_n of every slice solved by m
// steps of GMRES (Arnoldi with modified Gram-Schmidt from delta_n = 0, no restart, a
// breakdown ending a slice's Arnoldi early).  G_n = beta_n grad J_n[u_n, phi^(k)] are the
// path's slice gradients; A_n v = (G_n(u + eps v) - G_n(u - eps v)) / (2 eps) with the
// intermediate states phi^(k) held, each product being two slice passes at perturbed
// controls.  All slices of all instances advance together; the Arnoldi coefficients and the
// least-squares solves stay on the device (k_newton.hip), so an iteration synchronises with
// the host only to read the stop flags.
#include <math.h>

#include <algorithm>
#include <vector>

#include "ism_internal.h"
#include "ism_paths.h"

#define ISM_NW_TRY(expr)                               \
    do {                                               \
        const hipError_t e__ = (expr);                 \
        if (e__ != hipSuccess) return ISM_E_DEVICE;    \
    } while (0)

namespace ism {

namespace {

// the handle's buffers for GMRES size m (allocated once per larger m, freed with the handle)
int newton_alloc(ism_problem* p, int m) {
    NewtonBufs& w = p->nw;
    if (w.m >= m) return ISM_OK;
    const size_t bkc = (size_t)p->B * p->K * p->C, bn = (size_t)p->B * p->N;
    int st;
    w = NewtonBufs{};
    if ((st = dev_alloc(p, (void**)&w.V, (m + 1) * bkc * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&w.G, bkc * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&w.Gp, bkc * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&w.Gm, bkc * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&w.W, bkc * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&w.u0, bkc * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&w.H, bn * (m + 1) * m * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&w.beta, bn * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&w.wn, bn * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&w.nn, bn * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&w.y, bn * m * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&w.kdim, bn * sizeof(int)))) return st;
    w.m = m;
    return ISM_OK;
}

// slice gradients at u = u0 + a v (a = 0: at u0 itself)
int grad_at(ism_problem* p, const NewtonBufs& w, const double* v, double a, double* out) {
    const size_t bkc = (size_t)p->B * p->K * p->C;
    int st;
    ISM_NW_TRY(nw_lincomb(p->u, w.u0, v, a, bkc, p->stream));
    if ((st = refresh_steps(p))) return st;
    return slice_pass(p, 0, 0.0, out, false);
}

// one Newton step on every slice problem at phi^(k) (boundaries valid at u^(k))
int newton_step(ism_problem* p, int m, double eps) {
    const NewtonBufs& w = p->nw;
    const int B = p->B, K = p->K, N = p->N, C = p->C;
    const size_t bkc = (size_t)B * K * C;
    const int hs = (m + 1) * m;
    hipStream_t st = p->stream;
    int rc;
    ISM_NW_TRY(hipMemcpyAsync(w.u0, p->u, bkc * sizeof(double), hipMemcpyDeviceToDevice, st));
    if ((rc = slice_pass(p, 0, 0.0, w.G, false))) return rc;
    ISM_NW_TRY(launch_fill_i32(w.kdim, -1, B * N, st));
    // v_0 = -G / ||G||, beta = ||G||
    ISM_NW_TRY(nw_dot(w.G, w.G, p->s, B, K, N, C, w.nn, 1, st));
    ISM_NW_TRY(nw_normalize(w.V, w.G, p->s, B, K, N, C, w.nn, w.beta, 1, nullptr, -1.0, w.kdim, 0,
                            st));
    for (int i = 0; i < m; ++i) {
        const double* vi = w.V + (size_t)i * bkc;
        // w = A v_i by the central difference of slice gradients
        if ((rc = grad_at(p, w, vi, eps, w.Gp))) return rc;
        if ((rc = grad_at(p, w, vi, -eps, w.Gm))) return rc;
        ISM_NW_TRY(nw_diff(w.W, w.Gp, w.Gm, 0.5 / eps, bkc, st));
        ISM_NW_TRY(nw_dot(w.W, w.W, p->s, B, K, N, C, w.wn, 1, st));
        // modified Gram-Schmidt: h_{l,i} = <v_l, w>, w -= h_{l,i} v_l
        for (int l = 0; l <= i; ++l) {
            const double* vl = w.V + (size_t)l * bkc;
            double* h = w.H + (size_t)i * (m + 1) + l;
            ISM_NW_TRY(nw_dot(vl, w.W, p->s, B, K, N, C, h, hs, st));
            ISM_NW_TRY(nw_sub(w.W, vl, p->s, B, K, N, C, h, hs, st));
        }
        // h_{i+1,i} = ||w||, v_{i+1} = w / h_{i+1,i} (a breakdown sets the slice's kdim)
        ISM_NW_TRY(nw_dot(w.W, w.W, p->s, B, K, N, C, w.nn, 1, st));
        ISM_NW_TRY(nw_normalize(w.V + (size_t)(i + 1) * bkc, w.W, p->s, B, K, N, C, w.nn,
                                w.H + (size_t)i * (m + 1) + i + 1, hs, w.wn, 1.0, w.kdim, i + 1,
                                st));
    }
    ISM_NW_TRY(hipMemcpyAsync(p->u, w.u0, bkc * sizeof(double), hipMemcpyDeviceToDevice, st));
    ISM_NW_TRY(nw_lsq(w.H, w.beta, w.kdim, m, B * N, w.y, st));
    ISM_NW_TRY(nw_apply(p->u, w.V, bkc, p->s, B, K, N, C, w.y, m, p->active, st));
    p->bvalid = false;
    return ISM_OK;
}

}  // namespace

}  // namespace ism

using namespace ism;

extern "C" int ism_iterate_newton(ism_problem* p, int n_iter, int gmres_m, double fd_eps,
                                  double fid_stop, double* J_hist, int* iters_done) {
    if (!p || n_iter < 0 || gmres_m < 1 || gmres_m > kNewtonMaxM || !(fd_eps > 0.0) ||
        !std::isfinite(fd_eps) || std::isnan(fid_stop))
        return ISM_E_ARG;
    if (p->precision != ISM_FP64 || p->path == PATH_GPE) return ISM_E_UNSUPPORTED;
    if (hipSetDevice(p->device) != hipSuccess) return ISM_E_DEVICE;
    int st;
    const size_t need = (size_t)std::max(n_iter, 1) * p->B;
    if ((size_t)p->Jhist_cap < need) {
        double* nh = nullptr;
        if ((st = dev_alloc(p, (void**)&nh, need * sizeof(double)))) return st;
        p->Jhist = nh;
        p->Jhist_cap = (int)need;
    }
    if ((st = newton_alloc(p, gmres_m))) return st;
    ISM_NW_TRY(launch_fill_i32(p->active, 1, p->B, p->stream));
    ISM_NW_TRY(launch_fill_i32(p->flags, 0, 4, p->stream));
    const bool check_stop = fid_stop <= 1.0;
    int done = 0;
    for (int k = 0; k < n_iter; ++k) {
        if (check_stop) ISM_NW_TRY(launch_fill_i32(p->flags + 1, 0, 1, p->stream));
        // steps (a)-(b): boundaries and intermediate states at u^(k)
        if ((st = boundary_pass(p, p->Jhist + (size_t)k * p->B, fid_stop, true))) return st;
        int fl[4];
        if ((st = read_flags(p, fl))) return st;
        if (fl[0] & 2) return ISM_E_UNSUPPORTED;
        if (fl[0]) return ISM_E_NUMERIC;
        if (check_stop && fl[1] == 0) break;
        // steps (c)-(d): one Newton-GMRES step per slice problem, phi^(k) held
        if ((st = newton_step(p, gmres_m, fd_eps))) return st;
        done = k + 1;
    }
    int fl[4];
    if ((st = read_flags(p, fl))) return st;
    if (fl[0] & 2) return ISM_E_UNSUPPORTED;
    if (fl[0]) return ISM_E_NUMERIC;
    if (J_hist && n_iter > 0) {
        const int rows = std::min(n_iter, done + 1);
        if ((st = copy_out(p, J_hist, p->Jhist, (size_t)rows * p->B * sizeof(double)))) return st;
    }
    if (iters_done) *iters_done = done;
    return ISM_OK;
}
