// Sparse / small-dimension state problems on gfx950 (one d-vector per item,
// rows of the item on consecutive lanes of a 64-wide wavefront, several items
// packed per wavefront).
//
// What is computed (Sec. 2 and Sec. 3 of the paper, exponential step map):
//   per step j:  U_j = exp(-i tau H_j),  H_j = H0 + sum_c u_{j,c} H_c
//   slice n   :  forward  psi^n from phi_n over steps s_n..s_{n+1}-1   (Eq. (dirpara))
//                adjoint  chi^n from phi_{n+1} backwards               (proof of Theorem 2)
//                gradient beta_n [ Im<chi^n_j|Hhat_{c,j}|psi^n_j> - alpha_{n,j} u_{j,c} ]
//                update   u_{j,c} += rho g_{j,c}                         (Eq. (gradStep), ascent)
//   assembly  :  M_n = U_{s_{n+1}-1} ... U_{s_n}  (propagator assembling, Sec. 3)
//   boundary  :  Psi_{n+1} = M_n Psi_n, Lambda_n = M_n^+ Lambda_{n+1}, phi_n (Eq. (cible)), J, F.
//
// Step map.  exp(-i tau H) = e^{-i tau s} exp(-i tau (H - s)) with a scalar shift s per
// instance (midpoint of the diagonal of H0).  The kernels apply only the shifted
// factor, as a truncated Taylor series of its action on the vector (S sub-steps of
// tau/S, m terms each, m and S per instance from a norm bound so that the truncation
// is below rounding).  The scalar phase e^{-i tau s L_n} of a whole slice is put back
// once, in FP64: on the slice propagator in the boundary kernel and on the gradient
// overlaps in the slice kernel.  Unitarity is therefore never broken by a rounded
// per-step phase.
//
// Exact gradient.  dU_j/du_c = e^{-i tau s} L(A, E_c) (Frechet derivative of exp at
// A = -i tau (H - s) in the direction E_c = -i tau H_c).  The backward sweep applies
// the block exponential exp([[A^+, E_c^+], [0, A^+]]) to (0, chi_{j+1}), which yields
// chi_j and y_c = L(A^+, E_c^+) chi_{j+1} in one series; then
//   (1/tau) dJ/du_{j,c} = (1/tau) Re( e^{-i tau s L_n} <y_c | psi_j> ),
// which equals Im<chi_j|Hhat_c|psi_j> of the step-averaged operator.  The forward slice
// states are recovered in the backward sweep by applying U_j^+ (reversal), so no
// per-step trajectory is stored.
//
// Precision.  Real = double for ISM_FP64; Real = float for ISM_FP32_MIXED, where the
// per-step generator data (tau(H0 - s), tau H_c, u_j) are formed in FP64 and rounded
// once, the series runs in FP32 with FP32 accumulation, and every overlap, gradient,
// control update and boundary quantity is formed in FP64.
#include <math.h>

#include "ism_internal.h"

namespace ism {
namespace {

constexpr int WAVE = 64;
constexpr int WPB = 4;        // wavefronts per block
constexpr int MMAX = 28;      // largest Taylor term count

__constant__ double RK_D[MMAX] = {
    1.0, 1.0 / 2, 1.0 / 3, 1.0 / 4, 1.0 / 5, 1.0 / 6, 1.0 / 7, 1.0 / 8, 1.0 / 9, 1.0 / 10,
    1.0 / 11, 1.0 / 12, 1.0 / 13, 1.0 / 14, 1.0 / 15, 1.0 / 16, 1.0 / 17, 1.0 / 18, 1.0 / 19,
    1.0 / 20, 1.0 / 21, 1.0 / 22, 1.0 / 23, 1.0 / 24, 1.0 / 25, 1.0 / 26, 1.0 / 27, 1.0 / 28};
__constant__ float RK_F[MMAX] = {
    1.0f, 1.0f / 2, 1.0f / 3, 1.0f / 4, 1.0f / 5, 1.0f / 6, 1.0f / 7, 1.0f / 8, 1.0f / 9,
    1.0f / 10, 1.0f / 11, 1.0f / 12, 1.0f / 13, 1.0f / 14, 1.0f / 15, 1.0f / 16, 1.0f / 17,
    1.0f / 18, 1.0f / 19, 1.0f / 20, 1.0f / 21, 1.0f / 22, 1.0f / 23, 1.0f / 24, 1.0f / 25,
    1.0f / 26, 1.0f / 27, 1.0f / 28};

__device__ __forceinline__ float rk_of(float, int k) { return RK_F[k]; }
__device__ __forceinline__ double rk_of(double, int k) { return RK_D[k]; }

// value of v held by the lane whose byte address (lane * 4) is addr
__device__ __forceinline__ float lane_fetch(int addr, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_fetch(int addr, double v) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(bits & 0xffffffffull));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(bits >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned long long)(unsigned)lo));
}

// Generator terms of one row: H - s = diag + sum_g v_g G_g, G_g stored as WCM entries
// per row (lane address of the column, pre-scaled value).
template <typename R, int CGM, int WCM, bool RH>
struct Gen {
    int addr[CGM][WCM];
    R vre[CGM][WCM];
    R vim[CGM][WCM];
};

template <typename R, int CGM, int WCM, bool RH>
__device__ __forceinline__ void gen_apply(const Gen<R, CGM, WCM, RH>& G, R xr, R xi, R (&tr)[CGM],
                                          R (&ti)[CGM]) {
#pragma unroll
    for (int g = 0; g < CGM; ++g) {
        R ar = 0, ai = 0;
#pragma unroll
        for (int w = 0; w < WCM; ++w) {
            const R nr = lane_fetch(G.addr[g][w], xr);
            const R ni = lane_fetch(G.addr[g][w], xi);
            if (RH) {
                ar = fma(G.vre[g][w], nr, ar);
                ai = fma(G.vre[g][w], ni, ai);
            } else {
                ar = fma(G.vre[g][w], nr, fma(-G.vim[g][w], ni, ar));
                ai = fma(G.vre[g][w], ni, fma(G.vim[g][w], nr, ai));
            }
        }
        tr[g] = ar;
        ti[g] = ai;
    }
}

// x <- exp(-i (H - s) tau_sub) x by m Taylor terms (generator pre-scaled by tau_sub).
template <typename R, int CGM, int WCM, bool RH>
__device__ __forceinline__ void fwd_substep(R& xr, R& xi, R d0, const R (&v)[CGM],
                                            const Gen<R, CGM, WCM, RH>& G, int m) {
    R ar = xr, ai = xi, tr = xr, ti = xi;
#pragma unroll 1
    for (int k = 0; k < m; ++k) {
        R gr[CGM], gi[CGM];
        gen_apply(G, tr, ti, gr, gi);
        R hr = d0 * tr, hi = d0 * ti;
#pragma unroll
        for (int g = 0; g < CGM; ++g) {
            hr = fma(v[g], gr[g], hr);
            hi = fma(v[g], gi[g], hi);
        }
        const R rk = rk_of(R(0), k);
        tr = hi * rk;        // t <- -i h / (k+1)
        ti = -hr * rk;
        ar += tr;
        ai += ti;
    }
    xr = ar;
    xi = ai;
}

// One sub-step of the block exponential exp([[A^+, E^+],[0, A^+]]) with
// A^+ = +i tau_sub (H - s), E_c^+ = +i tau_sub G_c, applied to (y_c, chi), and of
// exp(A^+) applied to psi (reversal of the forward slice trajectory).
template <typename R, int CGM, int WCM, bool RH>
__device__ __forceinline__ void adj_substep(R& cr, R& ci, R& pr, R& pi, R (&yr)[CGM], R (&yi)[CGM],
                                            R d0, const R (&v)[CGM],
                                            const Gen<R, CGM, WCM, RH>& G, int m) {
    R acr = cr, aci = ci, tcr = cr, tci = ci;
    R apr = pr, api = pi, tpr = pr, tpi = pi;
    R ayr[CGM], ayi[CGM], tyr[CGM], tyi[CGM];
#pragma unroll
    for (int c = 0; c < CGM; ++c) {
        ayr[c] = tyr[c] = yr[c];
        ayi[c] = tyi[c] = yi[c];
    }
#pragma unroll 1
    for (int k = 0; k < m; ++k) {
        const R rk = rk_of(R(0), k);
        R gcr[CGM], gci[CGM];
        gen_apply(G, tcr, tci, gcr, gci);
        R gpr[CGM], gpi[CGM];
        gen_apply(G, tpr, tpi, gpr, gpi);
        R hcr = d0 * tcr, hci = d0 * tci, hpr = d0 * tpr, hpi = d0 * tpi;
#pragma unroll
        for (int g = 0; g < CGM; ++g) {
            hcr = fma(v[g], gcr[g], hcr);
            hci = fma(v[g], gci[g], hci);
            hpr = fma(v[g], gpr[g], hpr);
            hpi = fma(v[g], gpi[g], hpi);
        }
#pragma unroll
        for (int c = 0; c < CGM; ++c) {
            R gyr[CGM], gyi[CGM];
            gen_apply(G, tyr[c], tyi[c], gyr, gyi);
            R hyr = fma(d0, tyr[c], gcr[c]), hyi = fma(d0, tyi[c], gci[c]);
#pragma unroll
            for (int g = 0; g < CGM; ++g) {
                hyr = fma(v[g], gyr[g], hyr);
                hyi = fma(v[g], gyi[g], hyi);
            }
            tyr[c] = -hyi * rk;  // t <- +i h / (k+1)
            tyi[c] = hyr * rk;
            ayr[c] += tyr[c];
            ayi[c] += tyi[c];
        }
        tcr = -hci * rk;
        tci = hcr * rk;
        acr += tcr;
        aci += tci;
        tpr = -hpi * rk;
        tpi = hpr * rk;
        apr += tpr;
        api += tpi;
    }
    cr = acr;
    ci = aci;
    pr = apr;
    pi = api;
#pragma unroll
    for (int c = 0; c < CGM; ++c) {
        yr[c] = ayr[c];
        yi[c] = ayi[c];
    }
}

// Sum of v over the d lanes of this item; the result is valid on the item's row 0.
__device__ __forceinline__ double item_sum(double v, int lane, int r, int d) {
    for (int off = 1; off < d; off <<= 1) {
        const int src = lane + off < WAVE ? lane + off : WAVE - 1;
        const double o = lane_fetch(src * 4, v);
        if (r + off < d) v += o;
    }
    return v;
}

struct ItemMap {
    int b, lane, p, r, item, base;
    bool valid;
};

__device__ __forceinline__ bool map_item(const SpArgs& a, ItemMap& im) {
    im.lane = threadIdx.x & (WAVE - 1);
    int gw = blockIdx.x * WPB + (threadIdx.x >> 6);
    gw = __builtin_amdgcn_readfirstlane(gw);
    im.b = gw / a.waves_per_inst;
    if (im.b >= a.B) return false;
    const int wi = gw - im.b * a.waves_per_inst;
    im.p = im.lane / a.d;
    im.r = im.lane - im.p * a.d;
    im.item = wi * a.P + im.p;
    im.valid = (im.p < a.P) && (im.item < a.items_per_inst);
    im.base = im.p * a.d;
    return true;
}

template <typename R, int CGM, int WCM, bool RH>
__device__ __forceinline__ void load_gen(const SpArgs& a, const ItemMap& im, double ts,
                                         Gen<R, CGM, WCM, RH>& G) {
#pragma unroll
    for (int g = 0; g < CGM; ++g) {
#pragma unroll
        for (int w = 0; w < WCM; ++w) {
            if (im.valid && g < a.CG && w < a.WC) {
                const int idx = (g * a.d + im.r) * a.WC + w;
                G.addr[g][w] = (im.base + a.gcol[idx]) * 4;
                const dcx gv = a.gval[idx];
                G.vre[g][w] = (R)(gv.re * ts);
                G.vim[g][w] = (R)(gv.im * ts);
            } else {
                G.addr[g][w] = im.lane * 4;
                G.vre[g][w] = 0;
                G.vim[g][w] = 0;
            }
        }
    }
}

// control values of step j: v_g = u_{j,g} (g < C), 1 for the off-diagonal part of H0
template <typename R, int CGM>
__device__ __forceinline__ void load_controls(const SpArgs& a, int b, int j, R (&v)[CGM],
                                              double (&ud)[CGM]) {
    const double* uj = a.u + ((size_t)b * a.K + j) * a.C;
#pragma unroll
    for (int g = 0; g < CGM; ++g) {
        double x = 0.0;
        if (g < a.C) x = uj[g];
        else if (g < a.CG && a.has_offdiag) x = 1.0;
        ud[g] = x;
        v[g] = (R)x;
    }
}

template <typename R, int CGM, int WCM, bool RH>
__global__ __launch_bounds__(WAVE * WPB) void k_sp_assemble(SpArgs a) {
    ItemMap im;
    if (!map_item(a, im)) return;
    const TaylorP tp = a.tp[im.b];
    const int m = __builtin_amdgcn_readfirstlane(tp.m);
    const int S = __builtin_amdgcn_readfirstlane(tp.S);
    Gen<R, CGM, WCM, RH> G;
    load_gen(a, im, tp.tau_sub, G);
    const double sh = a.shift[im.b];
    const R d0 = im.valid ? (R)((a.h0diag[(size_t)im.b * a.h0diag_stride + im.r] - sh) * tp.tau_sub)
                          : R(0);
    const int n = im.valid ? im.item / a.d : 0;
    const int col = im.valid ? im.item - n * a.d : 0;
    const int sn = a.s[n], L = a.s[n + 1] - sn;
    R xr = (im.valid && im.r == col) ? R(1) : R(0), xi = 0;
    for (int jl = 0; jl < a.LMAX; ++jl) {
        const bool act = im.valid && jl < L;
        const int j = sn + (jl < L ? jl : L - 1);
        R v[CGM];
        double ud[CGM];
        load_controls(a, im.b, j, v, ud);
        R nr = xr, ni = xi;
        for (int sub = 0; sub < S; ++sub) fwd_substep(nr, ni, d0, v, G, m);
        if (act) {
            xr = nr;
            xi = ni;
        }
    }
    if (im.valid) {
        R* M = reinterpret_cast<R*>(a.M);
        const size_t o = ((((size_t)im.b * a.N + n) * a.d + col) * a.d + im.r) * 2;
        M[o] = xr;
        M[o + 1] = xi;
    }
}

template <typename R, int CGM, int WCM, bool RH>
__global__ __launch_bounds__(WAVE * WPB) void k_sp_slice(SpArgs a) {
    ItemMap im;
    if (!map_item(a, im)) return;
    const TaylorP tp = a.tp[im.b];
    const int m = __builtin_amdgcn_readfirstlane(tp.m);
    const int S = __builtin_amdgcn_readfirstlane(tp.S);
    Gen<R, CGM, WCM, RH> G;
    load_gen(a, im, tp.tau_sub, G);
    const double sh = a.shift[im.b];
    const R d0 = im.valid ? (R)((a.h0diag[(size_t)im.b * a.h0diag_stride + im.r] - sh) * tp.tau_sub)
                          : R(0);
    const int n = im.valid ? im.item : 0;
    const int sn = a.s[n], L = a.s[n + 1] - sn;
    const size_t pb = ((size_t)im.b * (a.N + 1)) * a.d;
    R xr = 0, xi = 0;
    if (im.valid) {
        const dcx ph = a.phi[pb + (size_t)n * a.d + im.r];
        xr = (R)ph.re;
        xi = (R)ph.im;
    }
    // forward sweep from phi_n (phase-less factor of the step map)
    for (int jl = 0; jl < a.LMAX; ++jl) {
        const bool act = im.valid && jl < L;
        const int j = sn + (jl < L ? jl : L - 1);
        R v[CGM];
        double ud[CGM];
        load_controls(a, im.b, j, v, ud);
        R nr = xr, ni = xi;
        for (int sub = 0; sub < S; ++sub) fwd_substep(nr, ni, d0, v, G, m);
        if (act) {
            xr = nr;
            xi = ni;
        }
    }
    // adjoint sweep from phi_{n+1}, reversal of the forward sweep, gradient, update
    R cr = 0, ci = 0;
    if (im.valid) {
        const dcx ph = a.phi[pb + (size_t)(n + 1) * a.d + im.r];
        cr = (R)ph.re;
        ci = (R)ph.im;
    }
    R pr = xr, pi = xi;
    const double theta = a.tau * sh * (double)L;
    const double cph = cos(theta), sph = sin(theta);   // e^{-i theta} = cph - i sph
    const double beta_over_tau = ((double)a.K / (double)L) / a.tau;
    const bool upd = a.update && (a.active == nullptr || a.active[im.b] != 0);
    for (int jl = a.LMAX - 1; jl >= 0; --jl) {
        const bool act = im.valid && jl < L;
        const int j = sn + (jl < L ? jl : L - 1);
        R v[CGM];
        double ud[CGM];
        load_controls(a, im.b, j, v, ud);
        R yr[CGM], yi[CGM];
#pragma unroll
        for (int c = 0; c < CGM; ++c) yr[c] = yi[c] = 0;
        R ncr = cr, nci = ci, npr = pr, npi = pi;
        for (int sub = 0; sub < S; ++sub) adj_substep(ncr, nci, npr, npi, yr, yi, d0, v, G, m);
        if (act) {
            cr = ncr;
            ci = nci;
            pr = npr;
            pi = npi;
        }
        const double al = a.alpha ? a.alpha[j] : 0.0;
#pragma unroll
        for (int c = 0; c < CGM; ++c) {
            if (c >= a.C) break;
            // <y_c | psi_j> in FP64
            const double yre = (double)yr[c], yim = (double)yi[c];
            const double qre = (double)pr, qim = (double)pi;
            double ore = fma(yre, qre, yim * qim);
            double oim = fma(yre, qim, -yim * qre);
            ore = item_sum(ore, im.lane, im.r, a.d);
            oim = item_sum(oim, im.lane, im.r, a.d);
            if (act && im.r == 0) {
                const double g = beta_over_tau * fma(cph, ore, sph * oim) - al * ud[c];
                const size_t ui = ((size_t)im.b * a.K + j) * a.C + c;
                if (a.grad) a.grad[ui] = g;
                if (upd) a.u[ui] = fma(a.rho, g, ud[c]);
            }
        }
    }
}

// Per-instance Taylor parameters from the infinity-norm bound
//   || tau (H_j - s) || <= tau ( max_r |H0_rr - s| + sum_g max_j |v_g| ||G_g||_inf ).
template <int PREC>
__global__ __launch_bounds__(256) void k_sp_params(SpArgs a, const double* h0norm,
                                                   const double* gnorm, int* flags) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    double bound = h0norm[b];
    for (int g = 0; g < a.CG; ++g) {
        double mx = 0.0;
        if (g < a.C) {
            for (int j = threadIdx.x; j < a.K; j += blockDim.x) {
                const double x = fabs(a.u[((size_t)b * a.K + j) * a.C + g]);
                mx = (x > mx || x != x) ? x : mx;
            }
        } else {
            mx = 1.0;
        }
        red[threadIdx.x] = mx;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                const double o = red[threadIdx.x + w];
                const double me = red[threadIdx.x];
                red[threadIdx.x] = (o > me || o != o) ? o : me;
            }
            __syncthreads();
        }
        bound += red[0] * gnorm[g];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double theta = a.tau * bound;
        const double cap = 1.5;
        const double tol = PREC == 0 ? 1e-17 : 1e-10;
        TaylorP tp;
        if (!(theta < 1e4)) {          // NaN / Inf / absurd controls: keep the loops bounded
            tp.S = 1;
            tp.m = 1;
            flags[0] = 1;
        } else {
            int S = (int)ceil(theta / cap);
            if (S < 1) S = 1;
            const double ts = theta / S;
            int m = 1;
            double term = ts;          // ts^{m} / m! for the current m
            const double ex = exp(ts);
            while (m < MMAX) {
                const double next = term * ts / (m + 1);
                if (next * ex <= tol) break;
                term = next;
                ++m;
            }
            tp.S = S;
            tp.m = m;
        }
        tp.tau_sub = a.tau / tp.S;
        const_cast<TaylorP*>(a.tp)[b] = tp;
    }
}

// --------------------------------------------------------------------------------
// boundary rebuild: 2N products with the assembled slice propagators (FP64)
// --------------------------------------------------------------------------------
template <typename RM>
__global__ __launch_bounds__(512) void k_sp_boundary(BndArgs a) {
    extern __shared__ double smem[];
    dcx* xs = reinterpret_cast<dcx*>(smem);             // 2*d
    double* red = smem + 4 * a.d;                        // blockDim
    const int b = blockIdx.x, tid = threadIdx.x;
    const int DP = blockDim.x / 2;
    const int grp = tid / DP, r = tid - grp * DP;
    const int d = a.d, N = a.N;
    const double sh = a.shift[b];
    const size_t pb = (size_t)b * (N + 1) * d;
    const RM* Mb = reinterpret_cast<const RM*>(a.M) + (size_t)b * N * d * d * 2;
    if (r < d) {
        const dcx v = grp == 0 ? a.psi0[r] : a.target[r];
        xs[grp * d + r] = v;
        if (grp == 0) a.Psi[pb + r] = v;
        else a.Lam[pb + (size_t)N * d + r] = v;
    }
    __syncthreads();
    for (int it = 0; it < N; ++it) {
        dcx y = {0.0, 0.0};
        const int n = grp == 0 ? it : N - 1 - it;
        if (r < d) {
            const RM* Mn = Mb + (size_t)n * d * d * 2;
            double yr = 0.0, yi = 0.0;
            if (grp == 0) {
                for (int c = 0; c < d; ++c) {         // (M' x)_r, M' column-major
                    const double mr = (double)Mn[(c * d + r) * 2], mi = (double)Mn[(c * d + r) * 2 + 1];
                    const dcx x = xs[c];
                    yr = fma(mr, x.re, fma(-mi, x.im, yr));
                    yi = fma(mr, x.im, fma(mi, x.re, yi));
                }
            } else {
                for (int c = 0; c < d; ++c) {         // (M'^+ x)_r = sum_c conj(M'_{c r}) x_c
                    const double mr = (double)Mn[(r * d + c) * 2], mi = (double)Mn[(r * d + c) * 2 + 1];
                    const dcx x = xs[d + c];
                    yr = fma(mr, x.re, fma(mi, x.im, yr));
                    yi = fma(mr, x.im, fma(-mi, x.re, yi));
                }
            }
            // slice phase e^{-i theta_n} (forward) or e^{+i theta_n} (adjoint)
            const double th = a.tau * sh * (double)(a.s[n + 1] - a.s[n]);
            const double c0 = cos(th), s0 = grp == 0 ? -sin(th) : sin(th);
            y.re = c0 * yr - s0 * yi;
            y.im = c0 * yi + s0 * yr;
        }
        __syncthreads();
        if (r < d) {
            xs[grp * d + r] = y;
            if (grp == 0) a.Psi[pb + (size_t)(it + 1) * d + r] = y;
            else a.Lam[pb + (size_t)n * d + r] = y;
        }
        __syncthreads();
    }
    // intermediate states (Eq. (cible)), t_n / T = s_n / K
    for (int idx = tid; idx < (N + 1) * d; idx += blockDim.x) {
        const int n = idx / d;
        const double w = (double)a.s[n] / (double)a.K;
        const dcx P = a.Psi[pb + idx], Lm = a.Lam[pb + idx];
        dcx f;
        f.re = (1.0 - w) * P.re + w * Lm.re;
        f.im = (1.0 - w) * P.im + w * Lm.im;
        if (n == 0) f = a.psi0[idx];
        if (n == N) f = a.target[idx - N * d];
        a.phi[pb + idx] = f;
    }
    // z = <Psi_N | psi_f>, penalty tau/2 sum alpha_j u^2 (deterministic tree reductions)
    double zr = 0.0, zi = 0.0;
    if (tid < d) {
        const dcx P = a.Psi[pb + (size_t)N * d + tid], t = a.target[tid];
        zr = P.re * t.re + P.im * t.im;
        zi = P.re * t.im - P.im * t.re;
    }
    double pen = 0.0;
    if (a.alpha) {
        const size_t KC = (size_t)a.K * a.C;
        for (size_t i = tid; i < KC; i += blockDim.x) {
            const double uu = a.u[(size_t)b * KC + i];
            pen += a.alpha[i / a.C] * uu * uu;
        }
    }
    double vals[3] = {zr, zi, pen};
    double outv[3];
    for (int q = 0; q < 3; ++q) {
        red[tid] = vals[q];
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        outv[q] = red[0];
        __syncthreads();
    }
    if (tid == 0) {
        const double J = outv[0] - 0.5 * a.tau * outv[2];
        const double F = outv[0] * outv[0] + outv[1] * outv[1];
        a.J[b] = J;
        a.F[b] = F;
        if (a.Jhist) a.Jhist[b] = J;
        if (!(fabs(J) < 1e300)) atomicOr(&a.flags[0], 1);
        if (a.active) {
            if (a.active[b] && F >= a.fid_stop) a.active[b] = 0;
            if (a.active[b]) atomicAdd(&a.flags[1], 1);
        }
    }
}

__global__ void k_check_finite(const double* x, size_t n, int* flag) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (; i < n; i += stride) bad |= !(fabs(x[i]) < 1e300);
    if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------------
// variant table: (generators, entries per generator row, real generators)
// ---------------------------------------------------------------------------------
struct Variant {
    int CG, WC, realh;
};
constexpr Variant kVariants[] = {
    {1, 2, 1},     // tridiagonal real generator (rigid rotor)
    {1, 2, 0},
    {2, 2, 0},     // two controls, two entries per row (two coupled spins)
    {4, 1, 0},     // spin chains: one flip per control
    {8, 1, 0},
    {12, 1, 0},
    {16, 1, 0},
    {4, 4, 0},     // small dense problems (d <= 4) with up to 3 controls + H0 off-diagonal
    {3, 8, 0},     // d <= 8 dense, up to 2 controls + H0 off-diagonal
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

#define ISM_SP_DISPATCH(KERNEL, R, VI, GRID, BLOCK, SHMEM, ST, ARGS)                      \
    switch (VI) {                                                                        \
        case 0: hipLaunchKernelGGL((KERNEL<R, 1, 2, true>), GRID, BLOCK, SHMEM, ST, ARGS); break;  \
        case 1: hipLaunchKernelGGL((KERNEL<R, 1, 2, false>), GRID, BLOCK, SHMEM, ST, ARGS); break; \
        case 2: hipLaunchKernelGGL((KERNEL<R, 2, 2, false>), GRID, BLOCK, SHMEM, ST, ARGS); break; \
        case 3: hipLaunchKernelGGL((KERNEL<R, 4, 1, false>), GRID, BLOCK, SHMEM, ST, ARGS); break; \
        case 4: hipLaunchKernelGGL((KERNEL<R, 8, 1, false>), GRID, BLOCK, SHMEM, ST, ARGS); break; \
        case 5: hipLaunchKernelGGL((KERNEL<R, 12, 1, false>), GRID, BLOCK, SHMEM, ST, ARGS); break;\
        case 6: hipLaunchKernelGGL((KERNEL<R, 16, 1, false>), GRID, BLOCK, SHMEM, ST, ARGS); break;\
        case 7: hipLaunchKernelGGL((KERNEL<R, 4, 4, false>), GRID, BLOCK, SHMEM, ST, ARGS); break; \
        case 8: hipLaunchKernelGGL((KERNEL<R, 3, 8, false>), GRID, BLOCK, SHMEM, ST, ARGS); break; \
        default: return hipErrorInvalidValue;                                            \
    }

}  // namespace

int sp_variant_index(int CG, int WC, int realh, int d) {
    if (d < 1 || d > WAVE) return -1;
    int best = -1;
    long best_cost = 0;
    for (int i = 0; i < kNumVariants; ++i) {
        const Variant& v = kVariants[i];
        if (v.CG < CG || v.WC < WC) continue;
        if (v.realh && !realh) continue;
        const long cost = (long)v.CG * v.CG * v.WC * (v.realh ? 1 : 2);
        if (best < 0 || cost < best_cost) {
            best = i;
            best_cost = cost;
        }
    }
    return best;
}

hipError_t sp_launch_params(const SpArgs& a, const double* h0norm, const double* gnorm,
                            int precision, hipStream_t st, int* flags) {
    if (precision == ISM_FP64)
        hipLaunchKernelGGL(k_sp_params<0>, dim3(a.B), dim3(256), 0, st, a, h0norm, gnorm, flags);
    else
        hipLaunchKernelGGL(k_sp_params<1>, dim3(a.B), dim3(256), 0, st, a, h0norm, gnorm, flags);
    return hipGetLastError();
}

hipError_t sp_launch_assemble(const SpArgs& a, int vi, int precision, hipStream_t st) {
    const long waves = (long)a.B * a.waves_per_inst;
    const dim3 grid((unsigned)((waves + WPB - 1) / WPB)), block(WAVE * WPB);
    if (precision == ISM_FP64) {
        ISM_SP_DISPATCH(k_sp_assemble, double, vi, grid, block, 0, st, a);
    } else {
        ISM_SP_DISPATCH(k_sp_assemble, float, vi, grid, block, 0, st, a);
    }
    return hipGetLastError();
}

hipError_t sp_launch_slice(const SpArgs& a, int vi, int precision, hipStream_t st) {
    const long waves = (long)a.B * a.waves_per_inst;
    const dim3 grid((unsigned)((waves + WPB - 1) / WPB)), block(WAVE * WPB);
    if (precision == ISM_FP64) {
        ISM_SP_DISPATCH(k_sp_slice, double, vi, grid, block, 0, st, a);
    } else {
        ISM_SP_DISPATCH(k_sp_slice, float, vi, grid, block, 0, st, a);
    }
    return hipGetLastError();
}

hipError_t sp_launch_boundary(const BndArgs& a, hipStream_t st) {
    int DP = ((a.d + 63) / 64) * 64;
    const int threads = 2 * DP;
    const size_t shmem = (size_t)4 * a.d * sizeof(double) + (size_t)threads * sizeof(double);
    if (a.m_fp32)
        hipLaunchKernelGGL(k_sp_boundary<float>, dim3(a.B), dim3(threads), shmem, st, a);
    else
        hipLaunchKernelGGL(k_sp_boundary<double>, dim3(a.B), dim3(threads), shmem, st, a);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double* x, size_t n, int* flag, hipStream_t st) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, st, x, n, flag);
    return hipGetLastError();
}

}  // namespace ism
