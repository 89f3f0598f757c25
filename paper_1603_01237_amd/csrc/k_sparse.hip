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
// factor, as a truncated Taylor polynomial of its action on the vector evaluated by
// Horner's rule (S sub-steps of tau/S, degree m, m and S per instance from a norm bound
// so that the truncation is below rounding).  The scalar phase e^{-i tau s L_n} of a whole slice is put back
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

// Workgroup barrier that orders LDS only.  __syncthreads() also orders global memory, so it
// waits for every global load in flight (a prefetch issued before it is then no prefetch);
// this one waits for the LDS operations alone.  For loops whose threads exchange data
// through LDS only, with every prefetched value consumed before the next barrier.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

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

// (cos theta, sin theta) of the slice phase theta = tau s L.  The angle is carried as an
// unevaluated sum hi + lo: tau s and its product with L are formed together with their exact
// rounding errors (fma), so the angle is exact to ~1e-31 relative before cos and sin see it.
// A plain tau * s * L is off by up to an ulp of theta (4e-15 at theta ~ 20 on the rotor),
// the same for every slice of equal length, and those errors add up over the slices into
// the global phase of psi(T) (2.7e-13 on the rotor batch at K = 20000).
__device__ __forceinline__ void slice_phase(double tau, double s, int L, double* c, double* sn) {
    const double p = tau * s;
    const double pe = fma(tau, s, -p);                  // tau s = p + pe
    const double h = p * (double)L;
    const double he = fma(p, (double)L, -h);            // p L = h + he
    const double lo = he + pe * (double)L;
    double sh, ch;
    sincos(h, &sh, &ch);
    *c = fma(-sh, lo, ch);
    *sn = fma(ch, lo, sh);
}

// Row exchange between the lanes that hold one item.
//  XWave : d <= 64, several items per wavefront; a neighbour row is read straight from the
//          other lane's register (ds_bpermute), so publish/sync are no-ops and `addr` is the
//          lane's byte address.
//  XBlock: 64 < d <= 256, one item per workgroup; rows are published to LDS slots, the
//          workgroup synchronises, and `addr` is the row index.
template <typename R>
struct XWave {
    static constexpr bool kBlock = false;
    __device__ __forceinline__ void publish(int, int, R) const {}
    __device__ __forceinline__ void sync() const {}
    __device__ __forceinline__ R fetch(int, int addr, R v) const { return lane_fetch(addr, v); }
};
template <typename R>
struct XBlock {
    static constexpr bool kBlock = true;
    R* lds;
    int ld;
    __device__ __forceinline__ void publish(int slot, int r, R v) const { lds[slot * ld + r] = v; }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
    __device__ __forceinline__ R fetch(int slot, int addr, R) const { return lds[slot * ld + addr]; }
};

// Diagonal entry tau_sub (H0_rr - s) of the generator.  In FP32 it is carried as a pair
// hi + lo: the rounding of a single FP32 value would be the same at every step and shift
// the phase of that row coherently over a sweep (about 1e-8 per step, 1.5e-4 after 20000
// steps of the rotor); the pair keeps the product accurate to ~1e-14 relative.
template <typename R>
struct Diag {
    R h, l;
    __device__ __forceinline__ static Diag make(double x) {
        Diag d;
        d.h = (R)x;
        d.l = (R)(x - (double)d.h);
        return d;
    }
    __device__ __forceinline__ R mul(R t) const {
        if (sizeof(R) == 8) return h * t;
        return fma(l, t, h * t);
    }
};

// Generator terms of one row: H - s = diag + sum_g v_g G_g, G_g stored as WCM entries
// per row (exchange address of the column, pre-scaled value).
template <typename R, int CGM, int WCM, bool RH>
struct Gen {
    int addr[CGM][WCM];
    R vre[CGM][WCM];
    R vim[CGM][WCM];
};

template <typename R, int CGM, int WCM, bool RH, class X>
__device__ __forceinline__ void gen_apply(const Gen<R, CGM, WCM, RH>& G, const X& ex, int slot,
                                          R xr, R xi, R (&tr)[CGM], R (&ti)[CGM]) {
#pragma unroll
    for (int g = 0; g < CGM; ++g) {
        R ar = 0, ai = 0;
#pragma unroll
        for (int w = 0; w < WCM; ++w) {
            const R nr = ex.fetch(slot, G.addr[g][w], xr);
            const R ni = ex.fetch(slot + 1, G.addr[g][w], xi);
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

// Generator terms with the step's control values folded in (v_g G_g), formed once per step
// so that a Taylor term costs no separate control multiplication.
template <typename R, int CGM, int WCM, bool RH>
__device__ __forceinline__ Gen<R, CGM, WCM, RH> scaled(const Gen<R, CGM, WCM, RH>& G,
                                                       const R (&v)[CGM]) {
    Gen<R, CGM, WCM, RH> S;
#pragma unroll
    for (int g = 0; g < CGM; ++g)
#pragma unroll
        for (int w = 0; w < WCM; ++w) {
            S.addr[g][w] = G.addr[g][w];
            S.vre[g][w] = v[g] * G.vre[g][w];
            S.vim[g][w] = RH ? R(0) : v[g] * G.vim[g][w];
        }
    return S;
}

// x <- exp(-i (H - s) tau_sub) x, degree-m Taylor polynomial evaluated by Horner's rule
// p <- x + A p / k (k = m..1): the small high-order terms are combined before they meet x,
// so they are not lost to the rounding of x (which in FP32 would shorten the series the same
// way at every step).  Gs holds the generator of the step, pre-scaled by tau_sub and by the
// controls (see scaled()).
template <typename R, int CGM, int WCM, bool RH, class X>
__device__ __forceinline__ void fwd_substep(R& xr, R& xi, Diag<R> d0,
                                            const Gen<R, CGM, WCM, RH>& Gs, const X& ex, int r,
                                            int m) {
    R pr = xr, pi = xi;
#pragma unroll 1
    for (int k = m; k >= 1; --k) {
        ex.publish(0, r, pr);
        ex.publish(1, r, pi);
        ex.sync();
        R hr = d0.mul(pr), hi = d0.mul(pi);
#pragma unroll
        for (int g = 0; g < CGM; ++g)
#pragma unroll
            for (int w = 0; w < WCM; ++w) {
                const R nr = ex.fetch(0, Gs.addr[g][w], pr);
                const R ni = ex.fetch(1, Gs.addr[g][w], pi);
                if (RH) {
                    hr = fma(Gs.vre[g][w], nr, hr);
                    hi = fma(Gs.vre[g][w], ni, hi);
                } else {
                    hr = fma(Gs.vre[g][w], nr, fma(-Gs.vim[g][w], ni, hr));
                    hi = fma(Gs.vre[g][w], ni, fma(Gs.vim[g][w], nr, hi));
                }
            }
        ex.sync();
        const R rk = rk_of(R(0), k - 1);     // 1/k
        pr = fma(hi, rk, xr);                // p <- x - i h / k
        pi = fma(-hr, rk, xi);
    }
    xr = pr;
    xi = pi;
}

// h = (D + sum_g Gs_g) p on this lane's row (generator pre-scaled, controls folded in)
template <typename R, int CGM, int WCM, bool RH, class X>
__device__ __forceinline__ void gen_h(R pr, R pi, Diag<R> d0, const Gen<R, CGM, WCM, RH>& Gs,
                                      const X& ex, int r, R& hr, R& hi) {
    ex.publish(0, r, pr);
    ex.publish(1, r, pi);
    ex.sync();
    hr = d0.mul(pr);
    hi = d0.mul(pi);
#pragma unroll
    for (int g = 0; g < CGM; ++g)
#pragma unroll
        for (int w = 0; w < WCM; ++w) {
            const R nr = ex.fetch(0, Gs.addr[g][w], pr);
            const R ni = ex.fetch(1, Gs.addr[g][w], pi);
            if (RH) {
                hr = fma(Gs.vre[g][w], nr, hr);
                hi = fma(Gs.vre[g][w], ni, hi);
            } else {
                hr = fma(Gs.vre[g][w], nr, fma(-Gs.vim[g][w], ni, hr));
                hi = fma(Gs.vre[g][w], ni, fma(Gs.vim[g][w], nr, hi));
            }
        }
    ex.sync();
}

// The Crank-Nicolson map is compiled into the variants with at most four generators (the
// larger ones are register-bound already); handles with more generators reject it.
template <int CGM>
constexpr bool kCnVariant = CGM <= 4;

// Crank-Nicolson step (Sec. 3): x <- (I + L)^{-1} (I - L) x with L = i h, h = (tau/2) H (the
// generator is pre-scaled by tau/2).  y = (I - L) x, then the Neumann series
// z <- y - L z (nt times) for (I + L)^{-1} y, convergent since ||L|| < 1.
template <typename R, int CGM, int WCM, bool RH, class X>
__device__ __forceinline__ void fwd_cn(R& xr, R& xi, Diag<R> d0, const Gen<R, CGM, WCM, RH>& Gs,
                                       const X& ex, int r, int nt) {
    R hr, hi;
    gen_h(xr, xi, d0, Gs, ex, r, hr, hi);
    const R yr = xr + hi, yi = xi - hr;              // y = x - i h
    R zr = yr, zi = yi;
#pragma unroll 1
    for (int k = 0; k < nt; ++k) {
        gen_h(zr, zi, d0, Gs, ex, r, hr, hi);
        zr = yr + hi;                                // z <- y - i h(z)
        zi = yi - hr;
    }
    xr = zr;
    xi = zi;
}

// One sub-step of the block exponential exp([[A^+, E^+],[0, A^+]]) with
// A^+ = +i tau_sub (H - s), E_c^+ = +i tau_sub G_c, applied to (y_c, chi), and of
// exp(A^+) applied to psi (reversal of the forward slice trajectory); Horner's rule on the
// block matrix: (p_y, p_x) <- (y, x) + (A^+ p_y + E^+ p_x, A^+ p_x) / k.
template <typename R, int CGM, int WCM, bool RH, class X>
__device__ __forceinline__ void adj_substep(R& cr, R& ci, R& pr, R& pi, R (&yr)[CGM], R (&yi)[CGM],
                                            Diag<R> d0, const R (&v)[CGM],
                                            const Gen<R, CGM, WCM, RH>& G, const X& ex, int r,
                                            int m) {
    R qcr = cr, qci = ci, qpr = pr, qpi = pi;
    R qyr[CGM], qyi[CGM];
#pragma unroll
    for (int c = 0; c < CGM; ++c) {
        qyr[c] = yr[c];
        qyi[c] = yi[c];
    }
#pragma unroll 1
    for (int k = m; k >= 1; --k) {
        const R rk = rk_of(R(0), k - 1);
        ex.publish(0, r, qcr);
        ex.publish(1, r, qci);
        ex.publish(2, r, qpr);
        ex.publish(3, r, qpi);
#pragma unroll
        for (int c = 0; c < CGM; ++c) {
            ex.publish(4 + 2 * c, r, qyr[c]);
            ex.publish(5 + 2 * c, r, qyi[c]);
        }
        ex.sync();
        R gcr[CGM], gci[CGM];
        gen_apply(G, ex, 0, qcr, qci, gcr, gci);
        R gpr[CGM], gpi[CGM];
        gen_apply(G, ex, 2, qpr, qpi, gpr, gpi);
        R hcr = d0.mul(qcr), hci = d0.mul(qci), hpr = d0.mul(qpr), hpi = d0.mul(qpi);
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
            gen_apply(G, ex, 4 + 2 * c, qyr[c], qyi[c], gyr, gyi);
            R hyr = d0.mul(qyr[c]) + gcr[c], hyi = d0.mul(qyi[c]) + gci[c];
#pragma unroll
            for (int g = 0; g < CGM; ++g) {
                hyr = fma(v[g], gyr[g], hyr);
                hyi = fma(v[g], gyi[g], hyi);
            }
            qyr[c] = fma(-hyi, rk, yr[c]);   // q <- y + i h / k
            qyi[c] = fma(hyr, rk, yi[c]);
        }
        ex.sync();
        qcr = fma(-hci, rk, cr);
        qci = fma(hcr, rk, ci);
        qpr = fma(-hpi, rk, pr);
        qpi = fma(hpr, rk, pi);
    }
    cr = qcr;
    ci = qci;
    pr = qpr;
    pi = qpi;
#pragma unroll
    for (int c = 0; c < CGM; ++c) {
        yr[c] = qyr[c];
        yi[c] = qyi[c];
    }
}

// Sum of v over the rows of this item; the result is valid on the item's row 0.
__device__ __forceinline__ double item_sum(double v, int lane, int r, int d, const XWave<float>&) {
    for (int off = 1; off < d; off <<= 1) {
        const int src = lane + off < WAVE ? lane + off : WAVE - 1;
        const double o = lane_fetch(src * 4, v);
        if (r + off < d) v += o;
    }
    return v;
}
__device__ __forceinline__ double item_sum(double v, int lane, int r, int d, const XWave<double>& x) {
    return item_sum(v, lane, r, d, XWave<float>());
}
template <typename R>
__device__ __forceinline__ double item_sum(double v, int lane, int r, int d, const XBlock<R>&) {
    __shared__ double red[4];
    (void)r;
    (void)d;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if (lane == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

struct ItemMap {
    int b, lane, p, r, item, base;
    bool valid;
};

template <class X>
__device__ __forceinline__ bool map_item(const SpArgs& a, ItemMap& im) {
    im.lane = threadIdx.x & (WAVE - 1);
    if (X::kBlock) {                      // one item per workgroup, rows on threads
        im.b = blockIdx.y;
        im.p = 0;
        im.r = threadIdx.x;
        im.item = blockIdx.x;
        im.valid = im.r < a.d;
        im.base = 0;
        return true;
    }
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

template <typename R, int CGM, int WCM, bool RH, class X>
__device__ __forceinline__ void load_gen(const SpArgs& a, const ItemMap& im, double ts,
                                         Gen<R, CGM, WCM, RH>& G) {
#pragma unroll
    for (int g = 0; g < CGM; ++g) {
#pragma unroll
        for (int w = 0; w < WCM; ++w) {
            if (im.valid && g < a.CG && w < a.WC) {
                const int idx = (g * a.d + im.r) * a.WC + w;
                const int col = a.gcol[idx];
                G.addr[g][w] = X::kBlock ? col : (im.base + col) * 4;
                const dcx gv = a.gval[idx];
                G.vre[g][w] = (R)(gv.re * ts);
                G.vim[g][w] = (R)(gv.im * ts);
            } else {
                G.addr[g][w] = X::kBlock ? 0 : im.lane * 4;
                G.vre[g][w] = 0;
                G.vim[g][w] = 0;
            }
        }
    }
}

// control values of step j: v_g = u_{j,g} (g < C), 1 for the off-diagonal part of H0
template <int CGM>
__device__ __forceinline__ void fetch_controls(const SpArgs& a, int b, int j, double (&ud)[CGM]) {
    const double* uj = a.u + ((size_t)b * a.K + j) * a.C;
#pragma unroll
    for (int g = 0; g < CGM; ++g) {
        double x = 0.0;
        if (g < a.C) x = uj[g];
        else if (g < a.CG && a.has_offdiag) x = 1.0;
        ud[g] = x;
    }
}

template <typename R, class X>
__device__ __forceinline__ X make_exchange(unsigned char* smem);
template <>
__device__ __forceinline__ XWave<float> make_exchange<float, XWave<float>>(unsigned char*) {
    return XWave<float>();
}
template <>
__device__ __forceinline__ XWave<double> make_exchange<double, XWave<double>>(unsigned char*) {
    return XWave<double>();
}
template <>
__device__ __forceinline__ XBlock<float> make_exchange<float, XBlock<float>>(unsigned char* s) {
    return XBlock<float>{reinterpret_cast<float*>(s), (int)blockDim.x};
}
template <>
__device__ __forceinline__ XBlock<double> make_exchange<double, XBlock<double>>(unsigned char* s) {
    return XBlock<double>{reinterpret_cast<double*>(s), (int)blockDim.x};
}

template <typename R, int CGM, int WCM, bool RH, class X>
__global__ __launch_bounds__(256) void k_sp_assemble(SpArgs a) {
    extern __shared__ unsigned char sp_smem[];
    ItemMap im;
    if (!map_item<X>(a, im)) return;
    const X ex = make_exchange<R, X>(sp_smem);
    const TaylorP tp = a.tp[im.b];
    const int m = __builtin_amdgcn_readfirstlane(tp.m);
    const int S = __builtin_amdgcn_readfirstlane(tp.S);
    Gen<R, CGM, WCM, RH> G;
    load_gen<R, CGM, WCM, RH, X>(a, im, tp.tau_sub, G);
    const double sh = a.shift[im.b];
    const Diag<R> d0 = Diag<R>::make(
        im.valid ? (a.h0diag[(size_t)im.b * a.h0diag_stride + im.r] - sh) * tp.tau_sub : 0.0);
    const bool item_ok = X::kBlock ? true : im.valid;
    const int n = item_ok ? im.item / a.d : 0;
    const int col = item_ok ? im.item - n * a.d : 0;
    const int sn = a.s[n], L = a.s[n + 1] - sn;
    R xr = (im.valid && im.r == col) ? R(1) : R(0), xi = 0;
    double unext[CGM];
    fetch_controls<CGM>(a, im.b, sn, unext);
    for (int jl = 0; jl < a.LMAX; ++jl) {
        const bool act = im.valid && jl < L;
        R v[CGM];
#pragma unroll
        for (int g = 0; g < CGM; ++g) v[g] = (R)unext[g];
        // the next step's controls are requested before this step's series
        const int jn = sn + (jl + 1 < L ? jl + 1 : L - 1);
        fetch_controls<CGM>(a, im.b, jn, unext);
        const Gen<R, CGM, WCM, RH> Gs = scaled(G, v);
        R nr = xr, ni = xi;
        if (kCnVariant<CGM> && a.cn)
            fwd_cn(nr, ni, d0, Gs, ex, im.r, m);
        else
            for (int sub = 0; sub < S; ++sub) fwd_substep(nr, ni, d0, Gs, ex, im.r, m);
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

template <typename R, int CGM, int WCM, bool RH, class X>
__global__ __launch_bounds__(256) void k_sp_slice(SpArgs a) {
    extern __shared__ unsigned char sp_smem[];
    ItemMap im;
    if (!map_item<X>(a, im)) return;
    const X ex = make_exchange<R, X>(sp_smem);
    const TaylorP tp = a.tp[im.b];
    const int m = __builtin_amdgcn_readfirstlane(tp.m);
    const int S = __builtin_amdgcn_readfirstlane(tp.S);
    Gen<R, CGM, WCM, RH> G;
    load_gen<R, CGM, WCM, RH, X>(a, im, tp.tau_sub, G);
    const double sh = a.shift[im.b];
    const Diag<R> d0 = Diag<R>::make(
        im.valid ? (a.h0diag[(size_t)im.b * a.h0diag_stride + im.r] - sh) * tp.tau_sub : 0.0);
    const bool item_ok = X::kBlock ? true : im.valid;
    const int n = item_ok ? im.item : 0;
    const int sn = a.s[n], L = a.s[n + 1] - sn;
    const size_t pb = ((size_t)im.b * (a.N + 1)) * a.d;
    R xr = 0, xi = 0;
    if (im.valid) {
        const dcx ph = a.phi[pb + (size_t)n * a.d + im.r];
        xr = (R)ph.re;
        xi = (R)ph.im;
    }
    // forward sweep from phi_n (phase-less factor of the step map)
    double unext[CGM];
    fetch_controls<CGM>(a, im.b, sn, unext);
    for (int jl = 0; jl < a.LMAX; ++jl) {
        const bool act = im.valid && jl < L;
        R v[CGM];
#pragma unroll
        for (int g = 0; g < CGM; ++g) v[g] = (R)unext[g];
        const int jn = sn + (jl + 1 < L ? jl + 1 : L - 1);
        fetch_controls<CGM>(a, im.b, jn, unext);
        const Gen<R, CGM, WCM, RH> Gs = scaled(G, v);
        R nr = xr, ni = xi;
        if (kCnVariant<CGM> && a.cn)
            fwd_cn(nr, ni, d0, Gs, ex, im.r, m);
        else
            for (int sub = 0; sub < S; ++sub) fwd_substep(nr, ni, d0, Gs, ex, im.r, m);
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
    double cph, sph;                                   // e^{-i theta} = cph - i sph
    slice_phase(a.tau, sh, L, &cph, &sph);
    const double beta_over_tau = ((double)a.K / (double)L) / a.tau;
    const bool upd = a.update && (a.active == nullptr || a.active[im.b] != 0);
    fetch_controls<CGM>(a, im.b, sn + (a.LMAX - 1 < L ? a.LMAX - 1 : L - 1), unext);
    for (int jl = a.LMAX - 1; jl >= 0; --jl) {
        const bool act = im.valid && jl < L;
        const int j = sn + (jl < L ? jl : L - 1);
        R v[CGM];
        double ud[CGM];
#pragma unroll
        for (int g = 0; g < CGM; ++g) {
            ud[g] = unext[g];
            v[g] = (R)ud[g];
        }
        // the previous step's controls (not yet updated: step j-1 is updated in the next
        // pass of this loop) are requested before this step's series
        if (jl > 0) fetch_controls<CGM>(a, im.b, sn + (jl - 1 < L ? jl - 1 : L - 1), unext);
        const double al = a.alpha ? a.alpha[j] : 0.0;
        if constexpr (kCnVariant<CGM>) if (a.cn) {
            // Crank-Nicolson adjoint step: with L = i h(.), chi~ = (I - L)^{-1} chi_{j+1} and
            // psi~ = (I - L)^{-1} psi_{j+1} (Neumann series z <- b + L z), then
            // chi_j = (I + L) chi~, psi_j = (I + L) psi~, and the gradient
            // beta_n Im<chi~|H_c|psi~> (psi_j + psi_{j+1} = 2 psi~).
            const Gen<R, CGM, WCM, RH> Gs = scaled(G, v);
            R zcr = cr, zci = ci, zpr = pr, zpi = pi, hr, hi;
#pragma unroll 1
            for (int k = 0; k < m; ++k) {
                gen_h(zcr, zci, d0, Gs, ex, im.r, hr, hi);
                const R ncr = cr - hi, nci = ci + hr;    // b + i h(z)
                gen_h(zpr, zpi, d0, Gs, ex, im.r, hr, hi);
                zpr = pr - hi;
                zpi = pi + hr;
                zcr = ncr;
                zci = nci;
            }
            // G_c psi~ (unscaled control operators, pre-scaled by tau/2) for the overlaps
            ex.publish(0, im.r, zpr);
            ex.publish(1, im.r, zpi);
            ex.sync();
            R gpr[CGM], gpi[CGM];
            gen_apply(G, ex, 0, zpr, zpi, gpr, gpi);
            ex.sync();
            R hcr, hci, hpr, hpi;
            gen_h(zcr, zci, d0, Gs, ex, im.r, hcr, hci);
            gen_h(zpr, zpi, d0, Gs, ex, im.r, hpr, hpi);
            if (act) {
                cr = zcr - hci;                          // (I + L) z = z + i h(z)
                ci = zci + hcr;
                pr = zpr - hpi;
                pi = zpi + hpr;
            }
            const double two_over_tau = 2.0 / a.tau;
#pragma unroll
            for (int c = 0; c < CGM; ++c) {
                if (c >= a.C) break;
                // Im <chi~ | G_c psi~> in FP64 (rows beyond d hold zeros)
                const double xre = (double)zcr, xim = (double)zci;
                const double yre = (double)gpr[c], yim = (double)gpi[c];
                double oim = fma(xre, yim, -xim * yre);
                oim = item_sum(oim, im.lane, im.r, a.d, ex);
                if (act && im.r == 0) {
                    const double g = ((double)a.K / (double)L) * two_over_tau * oim - al * ud[c];
                    const size_t ui = ((size_t)im.b * a.K + j) * a.C + c;
                    if (a.grad) a.grad[ui] = g;
                    if (upd) a.u[ui] = fma(a.rho, g, ud[c]);
                }
            }
            continue;
        }
        R yr[CGM], yi[CGM];
#pragma unroll
        for (int c = 0; c < CGM; ++c) yr[c] = yi[c] = 0;
        R ncr = cr, nci = ci, npr = pr, npi = pi;
        for (int sub = 0; sub < S; ++sub)
            adj_substep(ncr, nci, npr, npi, yr, yi, d0, v, G, ex, im.r, m);
        if (act) {
            cr = ncr;
            ci = nci;
            pr = npr;
            pi = npi;
        }
#pragma unroll
        for (int c = 0; c < CGM; ++c) {
            if (c >= a.C) break;
            // <y_c | psi_j> in FP64 (rows beyond d hold zeros)
            const double yre = (double)yr[c], yim = (double)yi[c];
            const double qre = (double)pr, qim = (double)pi;
            double ore = fma(yre, qre, yim * qim);
            double oim = fma(yre, qim, -yim * qre);
            ore = item_sum(ore, im.lane, im.r, a.d, ex);
            oim = item_sum(oim, im.lane, im.r, a.d, ex);
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
// Series truncation per step.  FP64: below its rounding.  FP32 mixed: the truncation summed
// over all K steps stays below 1e-5 (a tenth of the 1e-4 bar on the state; FP32 rounding
// contributes about 1e-5 at K = 20000), and never above 1e-8 per step.
__device__ __forceinline__ double fp32_step_tol(int K) {
    return fmin(1e-8, 1e-5 / (double)K);
}

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
    if (threadIdx.x == 0 && a.cn) {
        // Crank-Nicolson: terms of the Neumann series of (I + L)^{-1}, ||L|| <= theta; steps
        // outside the series' useful range are flagged (bit 2) and run one term
        const double theta = 0.5 * a.tau * bound;
        const double tol = PREC == 0 ? 1e-17 : fp32_step_tol(a.K);
        TaylorP tp;
        tp.S = 1;
        tp.m = 1;
        tp.tau_sub = 0.5 * a.tau;
        if (!(theta < 0.9)) {
            atomicOr(&flags[0], theta == theta ? 2 : 1);
        } else {
            int nt = 1;
            double t = theta * theta / (1.0 - theta);     // remainder after nt terms
            while (nt < MMAX && t > tol) {
                ++nt;
                t *= theta;
            }
            if (t > tol) atomicOr(&flags[0], 2);
            tp.m = nt;
        }
        const_cast<TaylorP*>(a.tp)[b] = tp;
        return;
    }
    if (threadIdx.x == 0) {
        const double theta = a.tau * bound;
        const double cap = 1.5;
        const double tol = PREC == 0 ? 1e-17 : fp32_step_tol(a.K);
        TaylorP tp;
        if (!(theta < 1e4)) {          // NaN / Inf / absurd controls: keep the loops bounded
            tp.S = 1;
            tp.m = 1;
            atomicOr(&flags[0], 1);
        } else {
            const int mcap = a.mmax > 0 ? a.mmax : MMAX;
            int S = (int)ceil(theta / cap);
            if (S < 1) S = 1;
            int m = 1;
            for (;;) {                 // more sub-steps until the degree fits the kernels
                const double ts = theta / S;
                double term = ts;      // ts^{m} / m! for the current m
                const double ex = exp(ts);
                m = 1;
                while (m < MMAX) {
                    const double next = term * ts / (m + 1);
                    if (next * ex * S <= tol) break;      // S sub-steps per step
                    term = next;
                    ++m;
                }
                if (m <= mcap) break;
                ++S;
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
template <typename RM, bool STAGED>
__global__ __launch_bounds__(512) void k_sp_boundary(BndArgs a) {
    // LDS: the two current vectors, the reduction slots and (STAGED, small d) a double buffer
    // holding the forward and adjoint slice propagators of the current product while those
    // of the next one are on their way from HBM
    extern __shared__ double smem[];
    dcx* xs = reinterpret_cast<dcx*>(smem);             // 2*d
    double* red = smem + 4 * a.d;                        // blockDim
    const int d = a.d, N = a.N, dd = d * d;
    RM* ms = reinterpret_cast<RM*>(red + blockDim.x);    // 2 buffers x 2 matrices x dd pairs
    const int b = blockIdx.x, tid = threadIdx.x;
    const int DP = blockDim.x / 2;
    const int grp = tid / DP, r = tid - grp * DP;
    const double sh = a.shift[b];
    const size_t pb = (size_t)b * (N + 1) * d;
    const RM* Mb = reinterpret_cast<const RM*>(a.M) + (size_t)b * N * dd * 2;
    // this thread's share of the 2 dd complex entries of one product's pair of propagators
    constexpr int PER = 4;
    RM pre[PER][2];
    auto fetch = [&](int it) {
        if (!STAGED) return;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + q * (int)blockDim.x;
            if (idx < 2 * dd) {
                const int which = idx >= dd, e = idx - which * dd;
                const int n = which == 0 ? it : N - 1 - it;
                pre[q][0] = Mb[((size_t)n * dd + e) * 2];
                pre[q][1] = Mb[((size_t)n * dd + e) * 2 + 1];
            }
        }
    };
    auto stage = [&](int it) {
        if (!STAGED) return;
        RM* dst = ms + (size_t)(it & 1) * 4 * dd;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + q * (int)blockDim.x;
            if (idx < 2 * dd) {
                dst[idx * 2] = pre[q][0];
                dst[idx * 2 + 1] = pre[q][1];
            }
        }
    };
    if (r < d) {
        const dcx v = grp == 0 ? a.psi0[r] : a.target[r];
        xs[grp * d + r] = v;
        if (grp == 0) a.Psi[pb + r] = v;
        else a.Lam[pb + (size_t)N * d + r] = v;
    }
    // slice phases: the slice starts are floor(n K / N), so slice n holds K/N or K/N + 1 steps
    const int Llo = a.K / N;
    double clo, slo, chi, shi;
    slice_phase(a.tau, sh, Llo, &clo, &slo);
    slice_phase(a.tau, sh, Llo + 1, &chi, &shi);
    fetch(0);
    // the loop's threads exchange the vectors through LDS only (Psi and Lambda are read back
    // after the loop, past a full barrier), so its barriers leave the prefetch in flight
    for (int it = 0; it < N; ++it) {
        stage(it);
        lds_barrier();                                   // staged matrices and xs visible
        if (it + 1 < N) fetch(it + 1);                  // next pair, consumed a step later
        const RM* Mf = STAGED ? ms + (size_t)(it & 1) * 4 * dd : Mb + (size_t)it * dd * 2;
        const RM* Ma = STAGED ? Mf + 2 * dd : Mb + (size_t)(N - 1 - it) * dd * 2;
        dcx y = {0.0, 0.0};
        const int n = grp == 0 ? it : N - 1 - it;
        if (r < d) {
            double yr = 0.0, yi = 0.0;
            if (grp == 0) {
                for (int c = 0; c < d; ++c) {         // (M' x)_r, M' column-major
                    const double mr = (double)Mf[(c * d + r) * 2], mi = (double)Mf[(c * d + r) * 2 + 1];
                    const dcx x = xs[c];
                    yr = fma(mr, x.re, fma(-mi, x.im, yr));
                    yi = fma(mr, x.im, fma(mi, x.re, yi));
                }
            } else {
                for (int c = 0; c < d; ++c) {         // (M'^+ x)_r = sum_c conj(M'_{c r}) x_c
                    const double mr = (double)Ma[(r * d + c) * 2], mi = (double)Ma[(r * d + c) * 2 + 1];
                    const dcx x = xs[d + c];
                    yr = fma(mr, x.re, fma(mi, x.im, yr));
                    yi = fma(mr, x.im, fma(-mi, x.re, yi));
                }
            }
            // slice phase e^{-i theta_n} (forward) or e^{+i theta_n} (adjoint)
            const int Ln = (int)(((long long)(n + 1) * a.K) / N - ((long long)n * a.K) / N);
            const double c0 = Ln == Llo ? clo : chi, sv = Ln == Llo ? slo : shi;
            const double s0 = grp == 0 ? -sv : sv;
            y.re = c0 * yr - s0 * yi;
            y.im = c0 * yi + s0 * yr;
        }
        lds_barrier();                                   // every product has read xs
        if (r < d) {
            xs[grp * d + r] = y;
            if (grp == 0) a.Psi[pb + (size_t)(it + 1) * d + r] = y;
            else a.Lam[pb + (size_t)n * d + r] = y;
        }
    }
    __syncthreads();
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

// Err of Algorithm 1, step (e), for instance blockIdx.x:
//   Err = sum_n tau sum_{j in slice n} ||grad J_n|_j||_2,  grad J_n = g / beta_n,
// g = beta_n grad J_n being what the slice kernels write (B x K x C, FP64) and
// beta_n = K / (s_{n+1} - s_n); with beta_scaled == 0 the slice gradients are grad J_n
// themselves (the BEC variant's slice problems carry no beta_n).  Each thread sums a fixed subset of steps in a fixed order
// and the workgroup reduces in a fixed tree, so the result does not depend on timing.  An
// active instance whose Err is <= eta (eta > 0) is frozen.
__global__ __launch_bounds__(256) void k_err(const double* g, const int* s, int K, int N, int C,
                                              double tau, int beta_scaled, double* err,
                                              int* active, double eta, int* flags) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    const double* gb = g + (size_t)b * K * C;
    double acc = 0.0;
    for (int n = 0; n < N; ++n) {
        const int j0 = s[n], j1 = s[n + 1];
        const double w = beta_scaled ? tau * (double)(j1 - j0) / (double)K : tau;   // tau / beta_n
        double part = 0.0;
        for (int j = j0 + (int)threadIdx.x; j < j1; j += 256) {
            double q = 0.0;
            for (int c = 0; c < C; ++c) {
                const double x = gb[(size_t)j * C + c];
                q += x * x;
            }
            part += sqrt(q);
        }
        acc += w * part;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double e = red[0];
        err[b] = e;
        if (!(e < 1e300)) atomicOr(&flags[0], 1);
        if (active && eta > 0.0 && active[b] && e <= eta) active[b] = 0;
    }
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

// Tridiagonal generators: one real symmetric control operator that couples row r only to
// rows r-1 and r+1, and a diagonal H0 (the rotor's cos(theta) in the m = 0 basis).  Each
// lane holds RPL consecutive rows, so only the two band edges of a lane cross lanes: a third
// of the lane exchanges of the one-row-per-lane layout, whose assembly is bound by the LDS
// crossbar that carries them.  In FP32 the diagonal tau_sub (H0_rr - s) is a single rounded
// coefficient and its rounding residual delta_r is put back once per sub-step as the phase
// e^{-i delta_r} (delta_r ~ 1e-9, so the commutator it leaves out is ~1e-10 per step).
constexpr int RPL = 3;
constexpr bool kTriDpp64 = true;       // FP64 lane edges by DPP shifts (tri_edges)

// Per-lane coefficients of the tridiagonal layout: rows r0 .. r0+RPL-1 of instance b,
// scaled by tau_sub; dg the (rounded) diagonal, dl its FP32 rounding residual, Lc / Rc the
// couplings to rows r-1 / r+1 (zero where absent or beyond d).
template <typename R>
__device__ __forceinline__ void tri_coeffs(const SpArgs& a, int b, int r0, bool valid, double ts,
                                           R (&dg)[RPL], R (&dl)[RPL], R (&Lc)[RPL],
                                           R (&Rc)[RPL]) {
    const double sh = a.shift[b];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int r = r0 + q;
        const bool ok = valid && r < a.d;
        const double hv = ok ? a.h0diag[(size_t)b * a.h0diag_stride + r] : sh;
        const double df = hv - sh;
        const double dd = df * ts;
        dg[q] = (R)dd;
        if (sizeof(R) == 4) {
            dl[q] = (R)(dd - (double)dg[q]);
        } else {
            // FP64: the residual of the exact (h - s) tau / nsub against dd, from the exact
            // rounding errors of the difference (two-sum), of the product (fma) and of the
            // sub-step length ts = tau / nsub
            const double bv = df - hv, av = df - bv;
            const double e1 = (hv - av) + (-sh - bv);
            const double e2 = fma(df, ts, -dd);
            const double ns = rint(a.tau / ts);
            const double rts = fma(-ns, ts, a.tau) / ns;
            dl[q] = (R)(e2 + e1 * ts + df * rts);
        }
        double lv = 0.0, rv = 0.0;
        if (ok) {
            for (int w = 0; w < a.WC; ++w) {
                const int idx = r * a.WC + w;
                const int c = a.gcol[idx];
                const double v = a.gval[idx].re * ts;
                if (c == r - 1) lv = v;
                else if (c == r + 1) rv = v;
            }
        }
        Lc[q] = (R)lv;
        Rc[q] = (R)rv;
    }
}

// Neighbour rows across the lane edges: the row below this lane's first row and the row
// above its last row.
// FP64: the neighbours are lanes lane - 1 and lane + 1 (lane 0 and lane 63 their own), so
// the values move by whole-wavefront DPP shifts (wave_shr:1, wave_shl:1), VALU moves
// without the LDS round trip of ds_bpermute; the FP64 Horner chain waits on these fetches
// at every term, with half the wavefronts per SIMD of the FP32 kernels to hide them.
// FP32 keeps ds_bpermute: those kernels are bound by VALU issue, which the moves would add to.
__device__ __forceinline__ int dpp_shift(int v, bool prev) {
    return prev ? __builtin_amdgcn_update_dpp(v, v, 0x138, 0xF, 0xF, false)     // wave_shr:1
                : __builtin_amdgcn_update_dpp(v, v, 0x130, 0xF, 0xF, false);    // wave_shl:1
}
__device__ __forceinline__ double lane_shift(double v, bool prev) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    const int lo = dpp_shift((int)(unsigned)(bits & 0xffffffffull), prev);
    const int hi = dpp_shift((int)(unsigned)(bits >> 32), prev);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned long long)(unsigned)lo));
}

__device__ __forceinline__ float lane_shift(float v, bool prev) {
    return __int_as_float(dpp_shift(__float_as_int(v), prev));
}

template <typename R>
__device__ __forceinline__ void tri_edges(const R (&xr)[RPL], const R (&xi)[RPL], int left,
                                          int right, R& lr, R& li, R& rr, R& ri) {
    if constexpr (sizeof(R) == 8 && kTriDpp64) {
        lr = lane_shift(xr[RPL - 1], true);
        li = lane_shift(xi[RPL - 1], true);
        rr = lane_shift(xr[0], false);
        ri = lane_shift(xi[0], false);
    } else {
        lr = lane_fetch(left, xr[RPL - 1]);
        li = lane_fetch(left, xi[RPL - 1]);
        rr = lane_fetch(right, xr[0]);
        ri = lane_fetch(right, xi[0]);
    }
}

// h = (D + L shift_down + R shift_up) x on this lane's rows
template <typename R>
__device__ __forceinline__ void tri_apply(const R (&xr)[RPL], const R (&xi)[RPL], R lr, R li, R rr,
                                          R ri, const R (&dg)[RPL], const R (&Ls)[RPL],
                                          const R (&Rs)[RPL], R (&hr)[RPL], R (&hi)[RPL]) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const R pvr = q > 0 ? xr[q - 1] : lr, pvi = q > 0 ? xi[q - 1] : li;
        const R nxr = q < RPL - 1 ? xr[q + 1] : rr, nxi = q < RPL - 1 ? xi[q + 1] : ri;
        hr[q] = fma(Rs[q], nxr, fma(Ls[q], pvr, dg[q] * xr[q]));
        hi[q] = fma(Rs[q], nxi, fma(Ls[q], pvi, dg[q] * xi[q]));
    }
}

// Horner terms up to this order are unrolled with 1/k as an instruction constant (terms
// above the instance's m are skipped by a wavefront-uniform branch); larger m loop.
constexpr int MU_TRI = kTriMaxTerms;

// One Horner term: p <- x - i (D + V) p / k
template <typename R>
__device__ __forceinline__ void tri_fwd_term(R (&pr)[RPL], R (&pi)[RPL], const R (&nr)[RPL],
                                             const R (&ni)[RPL], const R (&dg)[RPL],
                                             const R (&Ls)[RPL], const R (&Rs)[RPL], int left,
                                             int right, R rk) {
    R lr, li, rr, ri, hr[RPL], hi[RPL];
    tri_edges(pr, pi, left, right, lr, li, rr, ri);
    tri_apply(pr, pi, lr, li, rr, ri, dg, Ls, Rs, hr, hi);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        pr[q] = fma(hi[q], rk, nr[q]);
        pi[q] = fma(-hr[q], rk, ni[q]);
    }
}

// x <- e^{-i k delta} x to first order (k delta ~ 1e-8)
template <typename R>
__device__ __forceinline__ void tri_phase(R (&nr)[RPL], R (&ni)[RPL], const R (&dl)[RPL], R k) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const R th = k * dl[q], t = nr[q];
        nr[q] = fma(th, ni[q], nr[q]);
        ni[q] = fma(-th, t, ni[q]);
    }
}

// x <- T_M(-i (D + V)) x by Horner, M fixed: the first term is applied to x itself, so no
// copy of x is made and every 1/k is an instruction constant.
template <int M, typename R>
__device__ __forceinline__ void tri_horner(R (&nr)[RPL], R (&ni)[RPL], const R (&dg)[RPL],
                                           const R (&Ls)[RPL], const R (&Rs)[RPL], int left,
                                           int right) {
    R pr[RPL], pi[RPL];
    {
        R lr, li, rr, ri, hr[RPL], hi[RPL];
        tri_edges(nr, ni, left, right, lr, li, rr, ri);
        tri_apply(nr, ni, lr, li, rr, ri, dg, Ls, Rs, hr, hi);
        const R rk = R(1) / R(M);
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            pr[q] = fma(hi[q], rk, nr[q]);
            pi[q] = fma(-hr[q], rk, ni[q]);
        }
    }
#pragma unroll
    for (int k = M - 1; k >= 1; --k) tri_fwd_term(pr, pi, nr, ni, dg, Ls, Rs, left, right, R(1) / R(k));
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        nr[q] = pr[q];
        ni[q] = pi[q];
    }
}

// the degree is wavefront-uniform: a chain of scalar branches selects the unrolled series
template <int M, typename R>
__device__ __forceinline__ void tri_horner_dispatch(int m, R (&nr)[RPL], R (&ni)[RPL],
                                                    const R (&dg)[RPL], const R (&Ls)[RPL],
                                                    const R (&Rs)[RPL], int left, int right) {
    if (m == M) {
        tri_horner<M>(nr, ni, dg, Ls, Rs, left, right);
    } else {
        if constexpr (M > 1) tri_horner_dispatch<M - 1>(m, nr, ni, dg, Ls, Rs, left, right);
    }
}

// x <- e^{-i delta} T_m(-i (D + V)) x for one sub-step (Horner, as fwd_substep; m is at most
// MU_TRI, which the series parameters guarantee for the tridiagonal kernels)
template <typename R, bool PHASE = true>
__device__ __forceinline__ void tri_fwd_substep(R (&nr)[RPL], R (&ni)[RPL], const R (&dg)[RPL],
                                                const R (&dl)[RPL], const R (&Ls)[RPL],
                                                const R (&Rs)[RPL], int left, int right, int m) {
    tri_horner_dispatch<MU_TRI>(m, nr, ni, dg, Ls, Rs, left, right);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        if (PHASE && sizeof(R) == 4) {                    // e^{-i delta}
            const R t = nr[q];
            nr[q] = fma(dl[q], ni[q], nr[q]);
            ni[q] = fma(-dl[q], t, ni[q]);
        }
    }
}

// Crank-Nicolson step in the tridiagonal layout: x <- (I + L)^{-1} (I - L) x, L = i h, by
// y = (I - L) x and the Neumann series z <- y - L z (nt terms); in FP32 the rounding residual
// of the diagonal enters as e^{-2 i delta} (the Cayley map's first-order response to a
// diagonal shift), applied once per step.
template <typename R>
__device__ __forceinline__ void tri_fwd_cn(R (&nr)[RPL], R (&ni)[RPL], const R (&dg)[RPL],
                                           const R (&dl)[RPL], const R (&Ls)[RPL],
                                           const R (&Rs)[RPL], int left, int right, int nt) {
    R lr, li, rr, ri, hr[RPL], hi[RPL], yr[RPL], yi[RPL];
    tri_edges(nr, ni, left, right, lr, li, rr, ri);
    tri_apply(nr, ni, lr, li, rr, ri, dg, Ls, Rs, hr, hi);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        yr[q] = nr[q] + hi[q];                            // y = x - i h
        yi[q] = ni[q] - hr[q];
        nr[q] = yr[q];
        ni[q] = yi[q];
    }
#pragma unroll 1
    for (int k = 0; k < nt; ++k) {
        tri_edges(nr, ni, left, right, lr, li, rr, ri);
        tri_apply(nr, ni, lr, li, rr, ri, dg, Ls, Rs, hr, hi);
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            nr[q] = yr[q] + hi[q];                        // z <- y - i h(z)
            ni[q] = yi[q] - hr[q];
        }
    }
    if (sizeof(R) == 4) {
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const R t = nr[q], d2 = 2 * dl[q];
            nr[q] = fma(d2, ni[q], nr[q]);
            ni[q] = fma(-d2, t, ni[q]);
        }
    }
}

// Crank-Nicolson adjoint step in the tridiagonal layout: with L = i h, chi~ = (I - L)^{-1} chi
// and psi~ = (I - L)^{-1} psi (Neumann series z <- b + L z), then chi <- (I + L) chi~,
// psi <- (I + L) psi~ (and e^{+2 i delta} in FP32).  Leaves chi~ in (zcr, zci) and the
// unscaled control operator applied to psi~ in (gr, gi).
template <typename R>
__device__ __forceinline__ void tri_adj_cn(R (&cr)[RPL], R (&ci)[RPL], R (&pr)[RPL], R (&pi)[RPL],
                                           R (&zcr)[RPL], R (&zci)[RPL], R (&gr)[RPL],
                                           R (&gi)[RPL], const R (&dg)[RPL], const R (&dl)[RPL],
                                           const R (&Lc)[RPL], const R (&Rc)[RPL],
                                           const R (&Ls)[RPL], const R (&Rs)[RPL], int left,
                                           int right, int nt) {
    R zpr[RPL], zpi[RPL], lr, li, rr, ri, hr[RPL], hi[RPL];
    const R zero[RPL] = {};
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        zcr[q] = cr[q];
        zci[q] = ci[q];
        zpr[q] = pr[q];
        zpi[q] = pi[q];
    }
#pragma unroll 1
    for (int k = 0; k < nt; ++k) {
        tri_edges(zcr, zci, left, right, lr, li, rr, ri);
        tri_apply(zcr, zci, lr, li, rr, ri, dg, Ls, Rs, hr, hi);
        R ncr[RPL], nci[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            ncr[q] = cr[q] - hi[q];                       // b + i h(z)
            nci[q] = ci[q] + hr[q];
        }
        tri_edges(zpr, zpi, left, right, lr, li, rr, ri);
        tri_apply(zpr, zpi, lr, li, rr, ri, dg, Ls, Rs, hr, hi);
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            zpr[q] = pr[q] - hi[q];
            zpi[q] = pi[q] + hr[q];
            zcr[q] = ncr[q];
            zci[q] = nci[q];
        }
    }
    tri_edges(zpr, zpi, left, right, lr, li, rr, ri);
    tri_apply(zpr, zpi, lr, li, rr, ri, zero, Lc, Rc, gr, gi);      // G psi~
    tri_apply(zpr, zpi, lr, li, rr, ri, dg, Ls, Rs, hr, hi);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        pr[q] = zpr[q] - hi[q];                           // (I + L) psi~
        pi[q] = zpi[q] + hr[q];
    }
    tri_edges(zcr, zci, left, right, lr, li, rr, ri);
    tri_apply(zcr, zci, lr, li, rr, ri, dg, Ls, Rs, hr, hi);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        cr[q] = zcr[q] - hi[q];                           // (I + L) chi~
        ci[q] = zci[q] + hr[q];
        if (sizeof(R) == 4) {
            const R d2 = 2 * dl[q];
            R t = cr[q];
            cr[q] = fma(-d2, ci[q], cr[q]);
            ci[q] = fma(d2, t, ci[q]);
            t = pr[q];
            pr[q] = fma(-d2, pi[q], pr[q]);
            pi[q] = fma(d2, t, pi[q]);
        }
    }
}

// One Horner term of the adjoint block series: sources s* (the current terms, or the
// sub-step's input for the first term) to outputs q*, around the input (c, p, y).
template <typename R>
__device__ __forceinline__ void tri_adj_term(const R (&scr)[RPL], const R (&sci)[RPL],
                                             const R (&spr)[RPL], const R (&spi)[RPL],
                                             const R (&syr)[RPL], const R (&syi)[RPL],
                                             R (&qcr)[RPL], R (&qci)[RPL], R (&qpr)[RPL],
                                             R (&qpi)[RPL], R (&qyr)[RPL], R (&qyi)[RPL],
                                             const R (&cr)[RPL], const R (&ci)[RPL],
                                             const R (&pr)[RPL], const R (&pi)[RPL],
                                             const R (&yr)[RPL], const R (&yi)[RPL],
                                             const R (&dg)[RPL], const R (&Lc)[RPL],
                                             const R (&Rc)[RPL], const R (&Ls)[RPL],
                                             const R (&Rs)[RPL], R v, int left, int right, R rk) {
    const R zero[RPL] = {};
    R clr, cli, crr, cri, plr, pli, prr, pri, ylr, yli, yrr, yri;
    tri_edges(scr, sci, left, right, clr, cli, crr, cri);
    tri_edges(spr, spi, left, right, plr, pli, prr, pri);
    tri_edges(syr, syi, left, right, ylr, yli, yrr, yri);
    R gcr[RPL], gci[RPL], hpr[RPL], hpi[RPL], hyr[RPL], hyi[RPL];
    tri_apply(scr, sci, clr, cli, crr, cri, zero, Lc, Rc, gcr, gci);   // G chi
    tri_apply(spr, spi, plr, pli, prr, pri, dg, Ls, Rs, hpr, hpi);
    tri_apply(syr, syi, ylr, yli, yrr, yri, dg, Ls, Rs, hyr, hyi);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const R hcr = fma(v, gcr[q], dg[q] * scr[q]), hci = fma(v, gci[q], dg[q] * sci[q]);
        hyr[q] += gcr[q];                             // E^+ chi enters the y block
        hyi[q] += gci[q];
        qcr[q] = fma(-hci, rk, cr[q]);                // q <- x + i h / k
        qci[q] = fma(hcr, rk, ci[q]);
        qpr[q] = fma(-hpi[q], rk, pr[q]);
        qpi[q] = fma(hpr[q], rk, pi[q]);
        qyr[q] = fma(-hyi[q], rk, yr[q]);
        qyi[q] = fma(hyr[q], rk, yi[q]);
    }
}

// The adjoint block series of fixed degree M by Horner: the first term reads the input
// itself, every 1/k is an instruction constant, and the result replaces the input.
template <int M, typename R>
__device__ __forceinline__ void tri_adj_horner(R (&cr)[RPL], R (&ci)[RPL], R (&pr)[RPL],
                                               R (&pi)[RPL], R (&yr)[RPL], R (&yi)[RPL],
                                               const R (&dg)[RPL], const R (&Lc)[RPL],
                                               const R (&Rc)[RPL], const R (&Ls)[RPL],
                                               const R (&Rs)[RPL], R v, int left, int right) {
    R qcr[RPL], qci[RPL], qpr[RPL], qpi[RPL], qyr[RPL], qyi[RPL];
    tri_adj_term(cr, ci, pr, pi, yr, yi, qcr, qci, qpr, qpi, qyr, qyi, cr, ci, pr, pi, yr, yi,
                 dg, Lc, Rc, Ls, Rs, v, left, right, R(1) / R(M));
#pragma unroll
    for (int k = M - 1; k >= 1; --k)
        tri_adj_term(qcr, qci, qpr, qpi, qyr, qyi, qcr, qci, qpr, qpi, qyr, qyi, cr, ci, pr, pi,
                     yr, yi, dg, Lc, Rc, Ls, Rs, v, left, right, R(1) / R(k));
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        cr[q] = qcr[q];
        ci[q] = qci[q];
        pr[q] = qpr[q];
        pi[q] = qpi[q];
        yr[q] = qyr[q];
        yi[q] = qyi[q];
    }
}

template <int M, typename R>
__device__ __forceinline__ void tri_adj_dispatch(int m, R (&cr)[RPL], R (&ci)[RPL],
                                                 R (&pr)[RPL], R (&pi)[RPL], R (&yr)[RPL],
                                                 R (&yi)[RPL], const R (&dg)[RPL],
                                                 const R (&Lc)[RPL], const R (&Rc)[RPL],
                                                 const R (&Ls)[RPL], const R (&Rs)[RPL], R v,
                                                 int left, int right) {
    if (m == M) {
        tri_adj_horner<M>(cr, ci, pr, pi, yr, yi, dg, Lc, Rc, Ls, Rs, v, left, right);
    } else {
        if constexpr (M > 1)
            tri_adj_dispatch<M - 1>(m, cr, ci, pr, pi, yr, yi, dg, Lc, Rc, Ls, Rs, v, left, right);
    }
}

// One sub-step of the block exponential of adj_substep in the tridiagonal layout:
// (y, chi) <- exp([[A^+, E^+], [0, A^+]]) (y, chi) and psi <- exp(A^+) psi, with
// A^+ = +i (D + v G), E^+ = +i G (G the unscaled control operator), then e^{+i delta} on
// all three (FP32).  m is at most MU_TRI.
template <typename R>
__device__ __forceinline__ void tri_adj_substep(R (&cr)[RPL], R (&ci)[RPL], R (&pr)[RPL],
                                                R (&pi)[RPL], R (&yr)[RPL], R (&yi)[RPL],
                                                const R (&dg)[RPL], const R (&dl)[RPL],
                                                const R (&Lc)[RPL], const R (&Rc)[RPL],
                                                const R (&Ls)[RPL], const R (&Rs)[RPL], R v,
                                                int left, int right, int m) {
    tri_adj_dispatch<MU_TRI>(m, cr, ci, pr, pi, yr, yi, dg, Lc, Rc, Ls, Rs, v, left, right);
    if (sizeof(R) == 4) {
#pragma unroll
        for (int q = 0; q < RPL; ++q) {                   // e^{+i delta} on all three
            R t = cr[q];
            cr[q] = fma(-dl[q], ci[q], cr[q]);
            ci[q] = fma(dl[q], t, ci[q]);
            t = pr[q];
            pr[q] = fma(-dl[q], pi[q], pr[q]);
            pi[q] = fma(dl[q], t, pi[q]);
            t = yr[q];
            yr[q] = fma(-dl[q], yi[q], yr[q]);
            yi[q] = fma(dl[q], t, yi[q]);
        }
    }
}

// Sum over the LPI lanes of one item; valid on the item's first lane.
__device__ __forceinline__ double lanes_sum(double v, int lane, int li, int LPI) {
    for (int off = 1; off < LPI; off <<= 1) {
        const int src = lane + off < WAVE ? lane + off : WAVE - 1;
        const double o = lane_fetch(src * 4, v);
        if (li + off < LPI) v += o;
    }
    return v;
}

template <typename R>
__global__ __launch_bounds__(256) void k_sp_assemble_tri(SpArgs a) {
    const int lane = threadIdx.x & (WAVE - 1);
    int gw = blockIdx.x * WPB + (threadIdx.x >> 6);
    gw = __builtin_amdgcn_readfirstlane(gw);
    const int b = gw / a.waves_per_inst;
    if (b >= a.B) return;
    const int wi = gw - b * a.waves_per_inst;
    const int d = a.d, LPI = (d + RPL - 1) / RPL;
    const int p = lane / LPI, li = lane - p * LPI;
    const int item = wi * a.P + p;
    const bool valid = p < a.P && item < a.items_per_inst;
    const int n = valid ? item / d : 0;
    const int col = valid ? item - n * d : 0;
    const int r0 = li * RPL;
    const TaylorP tp = a.tp[b];
    const int m = __builtin_amdgcn_readfirstlane(tp.m);
    const int S = __builtin_amdgcn_readfirstlane(tp.S);
    R dg[RPL], dl[RPL], Lc[RPL], Rc[RPL], xr[RPL], xi[RPL];
    tri_coeffs(a, b, r0, valid, tp.tau_sub, dg, dl, Lc, Rc);
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        xr[q] = (valid && r0 + q < d && r0 + q == col) ? R(1) : R(0);
        xi[q] = 0;
    }
    const int sn = a.s[n], L = a.s[n + 1] - sn;
    const int left = (lane > 0 ? lane - 1 : 0) * 4, right = (lane < WAVE - 1 ? lane + 1 : lane) * 4;
    // this item's controls (one control); the element after the slice's last is readable
    // (the next slice's first, or the allocation's padding)
    const double* up = a.u + (size_t)b * a.K + sn;
    double unext = up[0];
    // FP32: the residual phase e^{-i delta} of each sub-step is applied as e^{-i k delta}
    // once k >= 4 sub-steps have accumulated (delta ~ 1e-8: deferring it past the coupling
    // part changes a step by ~1e-12)
    int pend = 0;
    // each item runs its own slice length; the lanes of an item share it, so a lane whose
    // item has finished only ever lends its (finite) state to an edge coupling that is zero
    for (int jl = 0; jl < L; ++jl) {
        const R v = (R)unext;
        unext = up[jl + 1];
        R Ls[RPL], Rs[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            Ls[q] = v * Lc[q];
            Rs[q] = v * Rc[q];
        }
        if (a.cn) {
            tri_fwd_cn(xr, xi, dg, dl, Ls, Rs, left, right, m);
        } else {
            for (int sub = 0; sub < S; ++sub)
                tri_fwd_substep<R, false>(xr, xi, dg, dl, Ls, Rs, left, right, m);
            if (sizeof(R) == 4) {
                pend += S;
                if (pend >= 4) {
                    tri_phase(xr, xi, dl, (R)pend);
                    pend = 0;
                }
            }
        }
    }
    if (sizeof(R) == 4 && pend > 0) tri_phase(xr, xi, dl, (R)pend);
    // FP64: the diagonal's residual is the same at every sub-step; the phase it builds up over
    // the slice (twice the residual per step for the Cayley map) is applied once here, where it
    // is large enough to survive rounding (~1e-15 against ~1e-17 per step)
    if (sizeof(R) == 8) tri_phase(xr, xi, dl, (R)(a.cn ? 2 * L : L * S));
    if (valid) {
        R* M = reinterpret_cast<R*>(a.M);
        const size_t o = (((size_t)b * a.N + n) * d + col) * d;
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int r = r0 + q;
            if (r < d) {
                M[(o + r) * 2] = xr[q];
                M[(o + r) * 2 + 1] = xi[q];
            }
        }
    }
}


// Slice kernel for the tridiagonal layout (see k_sp_slice for what is computed).
template <typename R>
__global__ __launch_bounds__(256) void k_sp_slice_tri(SpArgs a) {
    const int lane = threadIdx.x & (WAVE - 1);
    int gw = blockIdx.x * WPB + (threadIdx.x >> 6);
    gw = __builtin_amdgcn_readfirstlane(gw);
    const int b = gw / a.waves_per_inst;
    if (b >= a.B) return;
    const int wi = gw - b * a.waves_per_inst;
    const int d = a.d, LPI = (d + RPL - 1) / RPL;
    const int p = lane / LPI, li = lane - p * LPI;
    const int item = wi * a.P + p;
    const bool valid = p < a.P && item < a.items_per_inst;
    const int n = valid ? item : 0;
    const int r0 = li * RPL;
    const TaylorP tp = a.tp[b];
    const int m = __builtin_amdgcn_readfirstlane(tp.m);
    const int S = __builtin_amdgcn_readfirstlane(tp.S);
    R dg[RPL], dl[RPL], Lc[RPL], Rc[RPL];
    tri_coeffs(a, b, r0, valid, tp.tau_sub, dg, dl, Lc, Rc);
    const int sn = a.s[n], L = a.s[n + 1] - sn;
    const size_t pb = ((size_t)b * (a.N + 1)) * d;
    const int left = (lane > 0 ? lane - 1 : 0) * 4, right = (lane < WAVE - 1 ? lane + 1 : lane) * 4;
    R xr[RPL], xi[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int r = r0 + q;
        xr[q] = xi[q] = 0;
        if (valid && r < d) {
            const dcx ph = a.phi[pb + (size_t)n * d + r];
            xr[q] = (R)ph.re;
            xi[q] = (R)ph.im;
        }
    }
    // forward sweep from phi_n (phase-less factor of the step map)
    const double* ub = a.u + (size_t)b * a.K;
    double unext = ub[sn];
    for (int jl = 0; jl < a.LMAX; ++jl) {
        const bool act = valid && jl < L;
        const R v = (R)unext;
        unext = ub[sn + (jl + 1 < L ? jl + 1 : L - 1)];
        R Ls[RPL], Rs[RPL], nr[RPL], ni[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            Ls[q] = v * Lc[q];
            Rs[q] = v * Rc[q];
            nr[q] = xr[q];
            ni[q] = xi[q];
        }
        if (a.cn)
            tri_fwd_cn(nr, ni, dg, dl, Ls, Rs, left, right, m);
        else
            for (int sub = 0; sub < S; ++sub) tri_fwd_substep(nr, ni, dg, dl, Ls, Rs, left, right, m);
        if (act) {
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                xr[q] = nr[q];
                xi[q] = ni[q];
            }
        }
    }
    // adjoint sweep from phi_{n+1}, reversal of the forward sweep, gradient, update
    R cr[RPL], ci[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int r = r0 + q;
        cr[q] = ci[q] = 0;
        if (valid && r < d) {
            const dcx ph = a.phi[pb + (size_t)(n + 1) * d + r];
            cr[q] = (R)ph.re;
            ci[q] = (R)ph.im;
        }
    }
    double cph, sph;                                   // e^{-i theta} = cph - i sph
    slice_phase(a.tau, a.shift[b], L, &cph, &sph);
    const double beta_over_tau = ((double)a.K / (double)L) / a.tau;
    const bool upd = a.update && (a.active == nullptr || a.active[b] != 0);
    unext = ub[sn + (a.LMAX - 1 < L ? a.LMAX - 1 : L - 1)];
    for (int jl = a.LMAX - 1; jl >= 0; --jl) {
        const bool act = valid && jl < L;
        const int j = sn + (jl < L ? jl : L - 1);
        const double ud = unext;
        const R v = (R)ud;
        // step j-1 is updated only in the next pass of this loop
        if (jl > 0) unext = ub[sn + (jl - 1 < L ? jl - 1 : L - 1)];
        R Ls[RPL], Rs[RPL], ncr[RPL], nci[RPL], npr[RPL], npi[RPL], yr[RPL], yi[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            Ls[q] = v * Lc[q];
            Rs[q] = v * Rc[q];
            ncr[q] = cr[q];
            nci[q] = ci[q];
            npr[q] = xr[q];
            npi[q] = xi[q];
            yr[q] = yi[q] = 0;
        }
        if (a.cn) {
            // chi~ in (yr, yi) and G psi~ in (zgr, zgi): the gradient is
            // beta_n (2/tau) Im<chi~|G psi~> (G pre-scaled by tau/2)
            R zgr[RPL], zgi[RPL];
            tri_adj_cn(ncr, nci, npr, npi, yr, yi, zgr, zgi, dg, dl, Lc, Rc, Ls, Rs, left, right, m);
            double oim = 0.0;
#pragma unroll
            for (int q = 0; q < RPL; ++q)
                oim += fma((double)yr[q], (double)zgi[q], -(double)yi[q] * (double)zgr[q]);
            oim = lanes_sum(oim, lane, li, LPI);
            if (act) {
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    cr[q] = ncr[q];
                    ci[q] = nci[q];
                    xr[q] = npr[q];
                    xi[q] = npi[q];
                }
            }
            if (act && li == 0) {
                const double al = a.alpha ? a.alpha[j] : 0.0;
                const double g = ((double)a.K / (double)L) * (2.0 / a.tau) * oim - al * ud;
                const size_t ui = (size_t)b * a.K + j;
                if (a.grad) a.grad[ui] = g;
                if (upd) a.u[ui] = fma(a.rho, g, ud);
            }
            continue;
        }
        for (int sub = 0; sub < S; ++sub)
            tri_adj_substep(ncr, nci, npr, npi, yr, yi, dg, dl, Lc, Rc, Ls, Rs, v, left, right, m);
        if (act) {
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                cr[q] = ncr[q];
                ci[q] = nci[q];
                xr[q] = npr[q];
                xi[q] = npi[q];
            }
        }
        // <y | psi_j> in FP64 (rows beyond d hold zeros)
        double ore = 0.0, oim = 0.0;
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const double yre = (double)yr[q], yim = (double)yi[q];
            const double qre = (double)xr[q], qim = (double)xi[q];
            ore += fma(yre, qre, yim * qim);
            oim += fma(yre, qim, -yim * qre);
        }
        ore = lanes_sum(ore, lane, li, LPI);
        oim = lanes_sum(oim, lane, li, LPI);
        if (act && li == 0) {
            const double al = a.alpha ? a.alpha[j] : 0.0;
            const double g = beta_over_tau * fma(cph, ore, sph * oim) - al * ud;
            const size_t ui = (size_t)b * a.K + j;
            if (a.grad) a.grad[ui] = g;
            if (upd) a.u[ui] = fma(a.rho, g, ud);
        }
    }
}

#define ISM_SP_DISPATCH(KERNEL, R, X, VI, GRID, BLOCK, SHMEM, ST, ARGS)                            \
    switch (VI) {                                                                                \
        case 0: launch_with_shm(KERNEL<R, 1, 2, true, X<R>>, GRID, BLOCK, SHMEM, ST, ARGS); break;  \
        case 1: launch_with_shm(KERNEL<R, 1, 2, false, X<R>>, GRID, BLOCK, SHMEM, ST, ARGS); break; \
        case 2: launch_with_shm(KERNEL<R, 2, 2, false, X<R>>, GRID, BLOCK, SHMEM, ST, ARGS); break; \
        case 3: launch_with_shm(KERNEL<R, 4, 1, false, X<R>>, GRID, BLOCK, SHMEM, ST, ARGS); break; \
        case 4: launch_with_shm(KERNEL<R, 8, 1, false, X<R>>, GRID, BLOCK, SHMEM, ST, ARGS); break; \
        case 5: launch_with_shm(KERNEL<R, 12, 1, false, X<R>>, GRID, BLOCK, SHMEM, ST, ARGS); break;\
        case 6: launch_with_shm(KERNEL<R, 16, 1, false, X<R>>, GRID, BLOCK, SHMEM, ST, ARGS); break;\
        case 7: launch_with_shm(KERNEL<R, 4, 4, false, X<R>>, GRID, BLOCK, SHMEM, ST, ARGS); break; \
        case 8: launch_with_shm(KERNEL<R, 3, 8, false, X<R>>, GRID, BLOCK, SHMEM, ST, ARGS); break; \
        default: return hipErrorInvalidValue;                                                    \
    }

template <typename Kern, typename Args>
static void launch_with_shm(Kern kf, dim3 grid, dim3 block, size_t shm, hipStream_t st,
                            const Args& a) {
    if (shm > 65536)
        hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(kf, grid, block, shm, st, a);
}

// LDS bytes of the block exchange: (4 + 2 CG) row slots of DP values
static size_t sp_block_shmem(int vi, int dp, int precision) {
    const int cg = kVariants[vi].CG;
    return (size_t)(4 + 2 * cg) * dp * (precision == ISM_FP64 ? 8 : 4);
}

}  // namespace

bool sp_variant_cn(int vi) { return vi >= 0 && vi < kNumVariants && kVariants[vi].CG <= 4; }

int sp_variant_index(int CG, int WC, int realh, int d) {
    if (d < 1 || d > 256) return -1;
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

template <template <typename> class X>
static hipError_t sp_launch_kernel(const SpArgs& a, int vi, int precision, hipStream_t st,
                                   bool assemble) {
    dim3 grid, block;
    size_t shm = 0;
    if (!X<float>::kBlock) {
        const long waves = (long)a.B * a.waves_per_inst;
        grid = dim3((unsigned)((waves + WPB - 1) / WPB));
        block = dim3(WAVE * WPB);
    } else {
        const int dp = (a.d + WAVE - 1) / WAVE * WAVE;
        grid = dim3((unsigned)a.items_per_inst, (unsigned)a.B);
        block = dim3(dp);
        shm = sp_block_shmem(vi, dp, precision);
    }
    if (assemble) {
        if (precision == ISM_FP64) { ISM_SP_DISPATCH(k_sp_assemble, double, X, vi, grid, block, shm, st, a); }
        else { ISM_SP_DISPATCH(k_sp_assemble, float, X, vi, grid, block, shm, st, a); }
    } else {
        if (precision == ISM_FP64) { ISM_SP_DISPATCH(k_sp_slice, double, X, vi, grid, block, shm, st, a); }
        else { ISM_SP_DISPATCH(k_sp_slice, float, X, vi, grid, block, shm, st, a); }
    }
    return hipGetLastError();
}

hipError_t sp_launch_assemble_tri(const SpArgs& a0, int precision, hipStream_t st) {
    SpArgs a = a0;
    const int LPI = (a.d + RPL - 1) / RPL;
    a.P = WAVE / LPI;
    a.items_per_inst = a.N * a.d;
    a.waves_per_inst = (a.items_per_inst + a.P - 1) / a.P;
    const long waves = (long)a.B * a.waves_per_inst;
    const dim3 grid((unsigned)((waves + WPB - 1) / WPB)), block(WAVE * WPB);
    if (precision == ISM_FP64)
        hipLaunchKernelGGL(k_sp_assemble_tri<double>, grid, block, 0, st, a);
    else
        hipLaunchKernelGGL(k_sp_assemble_tri<float>, grid, block, 0, st, a);
    return hipGetLastError();
}

hipError_t sp_launch_slice_tri(const SpArgs& a0, int precision, hipStream_t st) {
    SpArgs a = a0;
    const int LPI = (a.d + RPL - 1) / RPL;
    a.P = WAVE / LPI;
    a.items_per_inst = a.N;
    a.waves_per_inst = (a.items_per_inst + a.P - 1) / a.P;
    const long waves = (long)a.B * a.waves_per_inst;
    const dim3 grid((unsigned)((waves + WPB - 1) / WPB)), block(WAVE * WPB);
    if (precision == ISM_FP64)
        hipLaunchKernelGGL(k_sp_slice_tri<double>, grid, block, 0, st, a);
    else
        hipLaunchKernelGGL(k_sp_slice_tri<float>, grid, block, 0, st, a);
    return hipGetLastError();
}

bool sp_tri_supported(int d) { return d >= 1 && d <= RPL * WAVE; }

hipError_t sp_launch_assemble(const SpArgs& a, int vi, int precision, hipStream_t st) {
    return a.d <= WAVE ? sp_launch_kernel<XWave>(a, vi, precision, st, true)
                       : sp_launch_kernel<XBlock>(a, vi, precision, st, true);
}

hipError_t sp_launch_slice(const SpArgs& a, int vi, int precision, hipStream_t st) {
    return a.d <= WAVE ? sp_launch_kernel<XWave>(a, vi, precision, st, false)
                       : sp_launch_kernel<XBlock>(a, vi, precision, st, false);
}

hipError_t sp_launch_boundary(const BndArgs& a, hipStream_t st) {
    // staged (double-buffered propagators in LDS) when one product's pair of propagators,
    // 2 d^2 entries, fits 4 per thread of a 512-thread workgroup
    const bool staged = 2 * a.d * a.d <= 4 * 512;
    const int DP = staged ? 256 : ((a.d + 63) / 64) * 64;
    const int threads = 2 * DP;
    const size_t rs = a.m_fp32 ? sizeof(float) : sizeof(double);
    const size_t shmem = (size_t)4 * a.d * sizeof(double) + (size_t)threads * sizeof(double) +
                         (staged ? (size_t)8 * a.d * a.d * rs : 0);
    if (a.m_fp32) {
        if (staged) launch_with_shm(k_sp_boundary<float, true>, dim3(a.B), dim3(threads), shmem, st, a);
        else launch_with_shm(k_sp_boundary<float, false>, dim3(a.B), dim3(threads), shmem, st, a);
    } else {
        if (staged) launch_with_shm(k_sp_boundary<double, true>, dim3(a.B), dim3(threads), shmem, st, a);
        else launch_with_shm(k_sp_boundary<double, false>, dim3(a.B), dim3(threads), shmem, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_err(const double* grad, const int* s, int B, int K, int N, int C, double tau,
                      int beta_scaled, double* err, int* active, double eta, int* flags,
                      hipStream_t st) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_err, dim3(B), dim3(256), 0, st, grad, s, K, N, C, tau, beta_scaled, err,
                       active, eta, flags);
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
