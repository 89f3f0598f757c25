// One-launch solve of small state problems (d <= 4, FP64, exponential step map).
//
// For a two-spin problem one ISM iteration (Algorithm 1 with one gradient step per slice) is
// a few thousand 4 x 4 products, far too little work to fill a launch; run as the usual
// sequence of per-pass launches it costs launch latency and the serial chains of each pass.
// Here one workgroup runs every iteration of one instance (grid = B instances) with the state
// of the whole solve in LDS and in a per-instance workspace, and the host waits once.
//
// One iteration, each phase separated by a workgroup barrier:
//  A  step propagators U'_j = exp(-i tau (H_j - s)) for all j, one thread per (step, column),
//     by a Taylor series (sub-steps when tau ||H_j - s|| > 1/2), stored row-major in the
//     workspace (the spectral shift s is the same as on the per-pass path; the phase
//     e^{-i tau s L_n} of slice n is restored once per slice, in FP64)
//  B  slice propagators M'_n = U'_{s_{n+1}-1} ... U'_{s_n} (Sec. 3, propagator assembling):
//     one chain of matrix-vector products per (slice, column), four lanes per vector
//  C  boundaries (Algorithm 1 steps (a)-(b)): Psi_{n+1} = M_n Psi_n, Lambda_n = M_n^+ Lambda_{n+1}
//     on one wavefront, the intermediate states of Eq. (cible), J and F, freezing at fid_stop
//  D  slice trajectories: psi'_j forward from phi_n and lambda'_{j+1} backward from
//     phi_{n+1}, one chain per slice and direction, stored in the workspace
//  E  gradient and update (Theorem 2, Eq. (gradStep)), one thread per step:
//        g_{j,c} = beta_n Re(e^{-i tau s L_n} <lambda'_{j+1}| L(-i X_j, -i tau H_c) psi'_j>) / tau
//                  - alpha_j u_{j,c},
//     X_j = tau (H_j - s), L the Frechet derivative of the exponential, evaluated as the
//     upper block of exp([[-i X, -i tau H_c], [0, -i X]]) applied to (0, psi'_j) by a Taylor
//     series; this is (1/tau) dJ/du_{j,c} exactly (the step average of H_c sandwiched
//     between lambda_j and psi_j), and u <- u + rho g on active instances.
// A launch runs n iterations: with first_boundary the sequence is B_0 (S B)^n, otherwise
// (S B)^n after a boundary of an earlier launch, whose intermediate states and active flags
// it reads back from the handle's arrays.  An instance frozen at a boundary takes no further
// update; J rows after it repeat its last J.
#include <math.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ism_internal.h"
#include "ism_paths.h"

namespace ism {
namespace {

constexpr int SD = kSmallD;     // padded dimension
constexpr int SC = kSmallC;     // most controls
constexpr int SN = kSmallN;     // most slices
constexpr int NT = 256;         // threads per workgroup
constexpr int MAXM = 24;        // most Taylor terms per sub-step
constexpr double kTol = 1e-17;  // truncation per series, below FP64 rounding

struct SmallArgs {
    int B, d, K, N, C;
    const int* s;          // N+1 slice starts
    double* u;             // B*K*C controls, updated in place
    const double* alpha;   // K (nullable)
    const dcx* H;          // (1 + C) padded SD x SD matrices per H0 instance: H0 - s_b, H_c
    long long h_stride;    // elements between instances (0: shared H0)
    const double* shift;   // B
    const double* xnorm;   // B: ||H0 - s_b||_inf
    const double* cnorm;   // C: ||H_c||_inf
    const dcx* psi0;       // d
    const dcx* target;     // d
    dcx* Psi;              // B*(N+1)*d
    dcx* Lam;              // B*(N+1)*d
    dcx* phi;              // B*(N+1)*d
    double* J;             // B
    double* F;             // B
    int* active;           // B
    int* flags;            // [0]: bit 0 NaN/Inf, bit 1 series range; [1]: active instances
                           // after the launch (use_active)
    double* jhist;         // nullable: row k at jhist[k*B + b]
    int* count;            // nullable: updates taken per instance, accumulated
    dcx* work;             // B * K * (SD*SD + 2 SD)
    double tau, rho, fid_stop;
    int n_iter, first_boundary;
    int use_active;        // 0: every instance runs, the active flags are neither read nor written
};

// slice phase e^{i tau s L} = c + i sn with the product tau s L carried in two parts
__device__ __forceinline__ void small_phase(double tau, double s, int L, double* c, double* sn) {
    const double p = tau * s;
    const double pe = fma(tau, s, -p);
    const double h = p * (double)L;
    const double he = fma(p, (double)L, -h);
    const double lo = he + pe * (double)L;
    double sh, ch;
    sincos(h, &sh, &ch);
    *c = fma(-sh, lo, ch);
    *sn = fma(ch, lo, sh);
}

// sub-steps S and terms m of a Taylor series of exp(A), ||A|| <= theta, each sub-step's
// remainder theta_s^(m+1)/(m+1)! below kTol; m = -1 when theta is not finite or beyond 512
// (more than 1024 sub-steps: reported, never truncated)
__device__ __forceinline__ void taylor_plan(double theta, int& S, int& m) {
    if (!(theta <= 512.0)) {
        S = 1;
        m = -1;
        return;
    }
    S = theta > 0.5 ? (int)ceil(theta / 0.5) : 1;
    const double ts = theta / S;
    m = 0;
    double rem = ts;             // ts^(m+1)/(m+1)!
    while (rem > kTol && m < MAXM) {
        ++m;
        rem *= ts / (m + 1);
    }
    if (rem > kTol) m = -1;
}

// X = tau (H0 - s + sum_c u_c H_c), padded SD x SD, from the LDS copies of the generators
__device__ __forceinline__ void form_x(const dcx* Hs, const double* uj, int C, double tau,
                                       dcx X[SD][SD]) {
#pragma unroll
    for (int r = 0; r < SD; ++r)
#pragma unroll
        for (int c = 0; c < SD; ++c) {
            double xr = Hs[r * SD + c].re, xi = Hs[r * SD + c].im;
            for (int q = 0; q < C; ++q) {
                const dcx h = Hs[(1 + q) * SD * SD + r * SD + c];
                xr = fma(uj[q], h.re, xr);
                xi = fma(uj[q], h.im, xi);
            }
            X[r][c].re = tau * xr;
            X[r][c].im = tau * xi;
        }
}

// y = -i (A v) * w
__device__ __forceinline__ void mv_mi(const dcx A[SD][SD], const dcx v[SD], double w, dcx y[SD]) {
#pragma unroll
    for (int r = 0; r < SD; ++r) {
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int c = 0; c < SD; ++c) {
            ar = fma(A[r][c].re, v[c].re, fma(-A[r][c].im, v[c].im, ar));
            ai = fma(A[r][c].re, v[c].im, fma(A[r][c].im, v[c].re, ai));
        }
        y[r].re = ai * w;
        y[r].im = -ar * w;
    }
}

// y += -i (tau H v) * w, H read from LDS (every lane reads the same entry: a broadcast)
__device__ __forceinline__ void mv_mi_lds_add(const dcx* H, const dcx v[SD], double w, dcx y[SD]) {
#pragma unroll
    for (int r = 0; r < SD; ++r) {
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int c = 0; c < SD; ++c) {
            const dcx h = H[r * SD + c];
            ar = fma(h.re, v[c].re, fma(-h.im, v[c].im, ar));
            ai = fma(h.re, v[c].im, fma(h.im, v[c].re, ai));
        }
        y[r].re = fma(ai, w, y[r].re);
        y[r].im = fma(-ar, w, y[r].im);
    }
}

__device__ __forceinline__ dcx shfl_cx(dcx v, int src) {
    return dcx{__shfl(v.re, src, 64), __shfl(v.im, src, 64)};
}

__global__ __launch_bounds__(NT) void k_small_solve(SmallArgs a) {
    __shared__ dcx Hs[(1 + SC) * SD * SD];
    __shared__ dcx Ms[SN * SD * SD];
    __shared__ dcx Ps[(SN + 1) * SD], Ls[(SN + 1) * SD], Fs[(SN + 1) * SD];
    __shared__ double phc[SN], phs[SN];      // e^{-i tau s L_n}: cos, -sin
    __shared__ int sl[SN + 1];
    __shared__ double red[NT];
    __shared__ double jf[2];
    __shared__ int act_s, stop_s;
    const int b = blockIdx.x, t = threadIdx.x;
    const int d = a.d, K = a.K, N = a.N, C = a.C;
    const double tau = a.tau, sh = a.shift[b];
    double* ub = a.u + (size_t)b * K * C;
    dcx* Uw = a.work + (size_t)b * K * (SD * SD + 2 * SD);
    dcx* Pw = Uw + (size_t)K * SD * SD;
    dcx* Lw = Pw + (size_t)K * SD;
    const size_t pb = (size_t)b * (N + 1) * d;
    const dcx* Hb = a.H + (size_t)b * a.h_stride;
    for (int i = t; i < (1 + C) * SD * SD; i += NT) Hs[i] = Hb[i];
    for (int i = t; i <= N; i += NT) sl[i] = a.s[i];
    if (t == 0) {
        act_s = a.use_active ? a.active[b] : 1;
        stop_s = 0;
        jf[0] = a.J[b];
    }
    if (!a.first_boundary) {      // intermediate states of the boundary that ended the last launch
        for (int i = t; i < (N + 1) * SD; i += NT) {
            const int n = i / SD, r = i - n * SD;
            Fs[i] = r < d ? a.phi[pb + (size_t)n * d + r] : dcx{0.0, 0.0};
        }
    }
    __syncthreads();
    for (int n = t; n < N; n += NT) {
        double c, sn;
        small_phase(tau, sh, sl[n + 1] - sl[n], &c, &sn);
        phc[n] = c;
        phs[n] = -sn;
    }
    double cmax = 0.0;
    for (int q = 0; q < C; ++q) cmax = fmax(cmax, a.cnorm[q]);
    const double xn = a.xnorm[b];
    int bad = 0;

    // ---- phases A-C: U'_j, M'_n, boundaries, J and F at the current controls
    auto boundary = [&](int row) {
        // A: column k of U'_j for task (j, k)
        for (int task = t; task < K * SD; task += NT) {
            const int j = task / SD, k = task - j * SD;
            const double* uj = ub + (size_t)j * C;
            double theta = xn;
            for (int q = 0; q < C; ++q) theta += fabs(uj[q]) * a.cnorm[q];
            theta *= tau;
            int S, m;
            taylor_plan(theta, S, m);
            if (m < 0) {
                bad |= theta == theta ? 2 : 1;
                S = 1;
                m = 1;
            }
            dcx X[SD][SD];
            form_x(Hs, uj, C, tau, X);
            dcx v[SD];
#pragma unroll
            for (int r = 0; r < SD; ++r) v[r] = dcx{r == k ? 1.0 : 0.0, 0.0};
            const double iS = 1.0 / S;
            for (int sub = 0; sub < S; ++sub) {
                dcx tr[SD], acc[SD];
#pragma unroll
                for (int r = 0; r < SD; ++r) tr[r] = acc[r] = v[r];
                for (int i = 1; i <= m; ++i) {
                    dcx y[SD];
                    mv_mi(X, tr, iS / i, y);
#pragma unroll
                    for (int r = 0; r < SD; ++r) {
                        tr[r] = y[r];
                        acc[r].re += y[r].re;
                        acc[r].im += y[r].im;
                    }
                }
#pragma unroll
                for (int r = 0; r < SD; ++r) v[r] = acc[r];
            }
#pragma unroll
            for (int r = 0; r < SD; ++r) Uw[(size_t)j * SD * SD + r * SD + k] = v[r];
        }
        __syncthreads();
        // B: column k of M'_n, lane r of the four lanes of task (n, k) holds row r
        for (int task = t; task < N * SD * SD; task += NT) {
            const int r = task & (SD - 1), k = (task / SD) & (SD - 1), n = task / (SD * SD);
            const int g0 = (t & 63) & ~(SD - 1);
            dcx x = dcx{r == k ? 1.0 : 0.0, 0.0};
            for (int j = sl[n]; j < sl[n + 1]; ++j) {     // same trip count in the four lanes
                const dcx* Ur = Uw + (size_t)j * SD * SD + r * SD;
                double yr = 0.0, yi = 0.0;
#pragma unroll
                for (int c = 0; c < SD; ++c) {
                    const dcx xc = shfl_cx(x, g0 + c);
                    const dcx uc = Ur[c];
                    yr = fma(uc.re, xc.re, fma(-uc.im, xc.im, yr));
                    yi = fma(uc.re, xc.im, fma(uc.im, xc.re, yi));
                }
                x = dcx{yr, yi};
            }
            Ms[n * SD * SD + r * SD + k] = x;
        }
        __syncthreads();
        // C: boundaries on wavefront 0, lanes 0-3 forward, 4-7 adjoint
        if (t < 2 * SD) {
            const int grp = t / SD, r = t & (SD - 1);
            dcx x = {0.0, 0.0};
            if (r < d) x = grp == 0 ? a.psi0[r] : a.target[r];
            if (grp == 0) Ps[r] = x;
            else Ls[N * SD + r] = x;
            for (int it = 0; it < N; ++it) {
                const int n = grp == 0 ? it : N - 1 - it;
                const dcx* M = Ms + n * SD * SD;
                double yr = 0.0, yi = 0.0;
#pragma unroll
                for (int c = 0; c < SD; ++c) {
                    const dcx xc = shfl_cx(x, grp * SD + c);
                    if (grp == 0) {          // (M' x)_r
                        const dcx m = M[r * SD + c];
                        yr = fma(m.re, xc.re, fma(-m.im, xc.im, yr));
                        yi = fma(m.re, xc.im, fma(m.im, xc.re, yi));
                    } else {                 // (M'^+ x)_r = sum_c conj(M'_{c r}) x_c
                        const dcx m = M[c * SD + r];
                        yr = fma(m.re, xc.re, fma(m.im, xc.im, yr));
                        yi = fma(m.re, xc.im, fma(-m.im, xc.re, yi));
                    }
                }
                // slice phase e^{-i theta_n} forward, e^{+i theta_n} adjoint
                const double c0 = phc[n], s0 = grp == 0 ? phs[n] : -phs[n];
                x = dcx{c0 * yr - s0 * yi, c0 * yi + s0 * yr};
                if (grp == 0) Ps[(n + 1) * SD + r] = x;
                else Ls[n * SD + r] = x;
            }
        }
        __syncthreads();
        // intermediate states (Eq. (cible)), t_n / T = s_n / K
        for (int i = t; i < (N + 1) * SD; i += NT) {
            const int n = i / SD, r = i - n * SD;
            const double w = (double)sl[n] / (double)K;
            dcx f;
            f.re = (1.0 - w) * Ps[i].re + w * Ls[i].re;
            f.im = (1.0 - w) * Ps[i].im + w * Ls[i].im;
            if (n == 0) f = Ps[i];
            if (n == N) f = Ls[i];
            Fs[i] = f;
            if (r < d) {
                a.Psi[pb + (size_t)n * d + r] = Ps[i];
                a.Lam[pb + (size_t)n * d + r] = Ls[i];
                a.phi[pb + (size_t)n * d + r] = f;
            }
        }
        // z = <Psi_N | psi_f>, penalty tau/2 sum alpha_j u^2 (fixed-order tree reductions)
        double vals[3] = {0.0, 0.0, 0.0};
        if (t < d) {
            const dcx P = Ps[N * SD + t], g = a.target[t];
            vals[0] = P.re * g.re + P.im * g.im;
            vals[1] = P.re * g.im - P.im * g.re;
        }
        if (a.alpha) {
            for (int i = t; i < K * C; i += NT) {
                const double x = ub[i];
                vals[2] += a.alpha[i / C] * x * x;
            }
        }
        double outv[3];
        for (int q = 0; q < 3; ++q) {
            red[t] = vals[q];
            __syncthreads();
            for (int w = NT / 2; w > 0; w >>= 1) {
                if (t < w) red[t] += red[t + w];
                __syncthreads();
            }
            outv[q] = red[0];
            __syncthreads();
        }
        if (t == 0) {
            const double J = outv[0] - 0.5 * tau * outv[2];
            const double F = outv[0] * outv[0] + outv[1] * outv[1];
            a.J[b] = J;
            a.F[b] = F;
            jf[0] = J;
            if (row >= 0 && a.jhist) a.jhist[(size_t)row * a.B + b] = J;
            if (!(fabs(J) < 1e300)) {
                atomicOr(&a.flags[0], 1);
                stop_s = 1;
            }
            if (act_s && F >= a.fid_stop) act_s = 0;
        }
        __syncthreads();
    };

    if (a.first_boundary && act_s) boundary(0);
    const int rows = a.first_boundary ? a.n_iter : 0;
    int done = 0;
    for (int k = 0; k < a.n_iter; ++k) {
        if (!act_s || stop_s) break;
        // D: slice trajectories; threads [0, NT/2) forward, [NT/2, NT) backward
        {
            const int half = t >= NT / 2, lt = t - half * (NT / 2);
            const int g0 = (t & 63) & ~(SD - 1);
            for (int task = lt; task < N * SD; task += NT / 2) {
                const int n = task / SD, r = task & (SD - 1);
                if (!half) {
                    dcx x = Fs[n * SD + r];
                    for (int j = sl[n]; j < sl[n + 1]; ++j) {
                        Pw[(size_t)j * SD + r] = x;
                        const dcx* Ur = Uw + (size_t)j * SD * SD + r * SD;
                        double yr = 0.0, yi = 0.0;
#pragma unroll
                        for (int c = 0; c < SD; ++c) {
                            const dcx xc = shfl_cx(x, g0 + c);
                            const dcx uc = Ur[c];
                            yr = fma(uc.re, xc.re, fma(-uc.im, xc.im, yr));
                            yi = fma(uc.re, xc.im, fma(uc.im, xc.re, yi));
                        }
                        x = dcx{yr, yi};
                    }
                } else {
                    dcx x = Fs[(n + 1) * SD + r];
                    for (int j = sl[n + 1] - 1; j >= sl[n]; --j) {
                        Lw[(size_t)j * SD + r] = x;
                        const dcx* Uc = Uw + (size_t)j * SD * SD + r;
                        double yr = 0.0, yi = 0.0;
#pragma unroll
                        for (int c = 0; c < SD; ++c) {
                            const dcx xc = shfl_cx(x, g0 + c);
                            const dcx uc = Uc[c * SD];       // conj(U'_{c r}) x_c
                            yr = fma(uc.re, xc.re, fma(uc.im, xc.im, yr));
                            yi = fma(uc.re, xc.im, fma(-uc.im, xc.re, yi));
                        }
                        x = dcx{yr, yi};
                    }
                }
            }
        }
        __syncthreads();
        // E: gradient and update, one thread per step
        for (int j = t; j < K; j += NT) {
            int n = (int)(((long long)(j + 1) * N + K - 1) / K) - 1;
            while (n > 0 && j < sl[n]) --n;
            while (n < N - 1 && j >= sl[n + 1]) ++n;
            const int L = sl[n + 1] - sl[n];
            const double beta = (double)K / (double)L;
            double* uj = ub + (size_t)j * C;
            double ucur[SC];
            for (int q = 0; q < C; ++q) ucur[q] = uj[q];
            dcx X[SD][SD];
            form_x(Hs, ucur, C, tau, X);
            double theta = xn;
            for (int q = 0; q < C; ++q) theta += fabs(ucur[q]) * a.cnorm[q];
            theta = tau * (theta + cmax);
            int S, m;
            taylor_plan(theta, S, m);
            if (m < 0) {
                bad |= theta == theta ? 2 : 1;
                S = 1;
                m = 1;
            }
            // the Frechet block's term k is bounded by theta^(k-1) tau ||H_c|| / (k-1)!: one
            // more term keeps its tail below kTol relative to the derivative itself
            ++m;
            dcx psi[SD], lam[SD];
#pragma unroll
            for (int r = 0; r < SD; ++r) {
                psi[r] = Pw[(size_t)j * SD + r];
                lam[r] = Lw[(size_t)j * SD + r];
            }
            const double iS = 1.0 / S;
            const double al = a.alpha ? a.alpha[j] : 0.0;
            double g[SC];
            for (int q = 0; q < C; ++q) {
                const dcx* Hq = Hs + (1 + q) * SD * SD;
                dcx v[SD], w[SD];
#pragma unroll
                for (int r = 0; r < SD; ++r) {
                    v[r] = psi[r];
                    w[r] = dcx{0.0, 0.0};
                }
                // (w, v) <- exp([[-iX, -i tau H_q], [0, -iX]] / S) (w, v), S times
                for (int sub = 0; sub < S; ++sub) {
                    dcx tv[SD], tw[SD], av[SD], aw[SD];
#pragma unroll
                    for (int r = 0; r < SD; ++r) {
                        tv[r] = av[r] = v[r];
                        tw[r] = aw[r] = w[r];
                    }
                    for (int i = 1; i <= m; ++i) {
                        const double c = iS / i;
                        dcx nw[SD], nv[SD];
                        mv_mi(X, tw, c, nw);
                        mv_mi_lds_add(Hq, tv, c * tau, nw);
                        mv_mi(X, tv, c, nv);
#pragma unroll
                        for (int r = 0; r < SD; ++r) {
                            tv[r] = nv[r];
                            tw[r] = nw[r];
                            av[r].re += nv[r].re;
                            av[r].im += nv[r].im;
                            aw[r].re += nw[r].re;
                            aw[r].im += nw[r].im;
                        }
                    }
#pragma unroll
                    for (int r = 0; r < SD; ++r) {
                        v[r] = av[r];
                        w[r] = aw[r];
                    }
                }
                // Re(e^{-i theta_n} <lambda'|w>)
                double zr = 0.0, zi = 0.0;
#pragma unroll
                for (int r = 0; r < SD; ++r) {
                    zr = fma(lam[r].re, w[r].re, fma(lam[r].im, w[r].im, zr));
                    zi = fma(lam[r].re, w[r].im, fma(-lam[r].im, w[r].re, zi));
                }
                const double ov = phc[n] * zr - phs[n] * zi;
                g[q] = beta * ov / tau - al * ucur[q];
            }
            for (int q = 0; q < C; ++q) uj[q] = fma(a.rho, g[q], ucur[q]);
        }
        __syncthreads();
        ++done;
        boundary(k + 1 < rows ? k + 1 : -1);
    }
    if (bad) atomicOr(&a.flags[0], bad);
    if (t == 0) {
        // rows after a freeze (or the stop) repeat the last J
        if (a.jhist && a.first_boundary)
            for (int k = done + 1; k < rows; ++k) a.jhist[(size_t)k * a.B + b] = jf[0];
        if (a.use_active) {
            a.active[b] = act_s;
            if (act_s) atomicAdd(&a.flags[1], 1);
        }
        if (a.count) a.count[b] += done;
    }
}

// flags[2] = the most updates any instance took (the iteration at which the per-pass loop
// would have ended), one workgroup
__global__ __launch_bounds__(256) void k_small_done(const int* count, int B, int* flags) {
    __shared__ int red[256];
    int m = 0;
    for (int b = threadIdx.x; b < B; b += 256) m = max(m, count[b]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) flags[2] = red[0];
}

}  // namespace

bool small_eligible(const ism_problem* p) {
    return p->small && !p->launch_per_pass;
}

size_t small_workspace_bytes(int d, int C, int K, int N, int B) {
    if (d > SD || C > SC || N > SN) return 0;
    return (size_t)B * K * (SD * SD + 2 * SD) * sizeof(dcx);
}

int small_setup(ism_problem* p, const double* H0, int h0_batched, const double* Hc) {
    const int d = p->d, C = p->C, B = p->B;
    const int nH = h0_batched ? B : 1;
    const size_t per = (size_t)(1 + C) * SD * SD;
    std::vector<dcx> H(per * nH, dcx{0.0, 0.0});
    std::vector<double> shift(B), xnorm(B), cnorm(C, 0.0);
    std::vector<double> sh_h(nH), xn_h(nH);
    for (int h = 0; h < nH; ++h) {
        const double* A = H0 + (size_t)h * 2 * d * d;
        double mx = -1e300, mn = 1e300;
        for (int r = 0; r < d; ++r) {
            mx = std::max(mx, A[2 * (r * d + r)]);
            mn = std::min(mn, A[2 * (r * d + r)]);
        }
        const double s = 0.5 * (mx + mn);     // same shift as the per-pass path
        double nrm = 0.0;
        for (int r = 0; r < d; ++r) {
            double rs = 0.0;
            for (int c = 0; c < d; ++c) {
                dcx v{A[2 * (r * d + c)], A[2 * (r * d + c) + 1]};
                if (r == c) v.re -= s;
                H[per * h + r * SD + c] = v;
                rs += std::hypot(v.re, v.im);
            }
            nrm = std::max(nrm, rs);
        }
        sh_h[h] = s;
        xn_h[h] = nrm;
        for (int q = 0; q < C; ++q) {
            const double* G = Hc + (size_t)q * 2 * d * d;
            for (int r = 0; r < d; ++r)
                for (int c = 0; c < d; ++c)
                    H[per * h + (1 + q) * SD * SD + r * SD + c] =
                        dcx{G[2 * (r * d + c)], G[2 * (r * d + c) + 1]};
        }
    }
    for (int q = 0; q < C; ++q) {
        const double* G = Hc + (size_t)q * 2 * d * d;
        for (int r = 0; r < d; ++r) {
            double rs = 0.0;
            for (int c = 0; c < d; ++c) rs += std::hypot(G[2 * (r * d + c)], G[2 * (r * d + c) + 1]);
            cnorm[q] = std::max(cnorm[q], rs);
        }
    }
    for (int b = 0; b < B; ++b) {
        shift[b] = sh_h[h0_batched ? b : 0];
        xnorm[b] = xn_h[h0_batched ? b : 0];
    }
    int st;
    if ((st = dev_upload(p, (void**)&p->sm_h, H.data(), H.size() * sizeof(dcx)))) return st;
    p->sm_hstride = h0_batched ? (long long)per : 0;
    if ((st = dev_upload(p, (void**)&p->sm_shift, shift.data(), B * sizeof(double)))) return st;
    if ((st = dev_upload(p, (void**)&p->sm_xnorm, xnorm.data(), B * sizeof(double)))) return st;
    if ((st = dev_upload(p, (void**)&p->sm_cnorm, cnorm.data(), C * sizeof(double)))) return st;
    if ((st = dev_alloc(p, (void**)&p->sm_work, small_workspace_bytes(d, C, p->K, p->N, B))))
        return st;
    if ((st = dev_alloc(p, (void**)&p->sm_count, B * sizeof(int)))) return st;
    return ISM_OK;
}

int small_run(ism_problem* p, int n_iter, double rho, double fid_stop, double* jhist,
              int* count, bool first_boundary, bool use_active) {
    SmallArgs a{};
    a.B = p->B;
    a.d = p->d;
    a.K = p->K;
    a.N = p->N;
    a.C = p->C;
    a.s = p->s;
    a.u = p->u;
    a.alpha = p->alpha;
    a.H = p->sm_h;
    a.h_stride = p->sm_hstride;
    a.shift = p->sm_shift;
    a.xnorm = p->sm_xnorm;
    a.cnorm = p->sm_cnorm;
    a.psi0 = p->psi0;
    a.target = p->target;
    a.Psi = p->Psi;
    a.Lam = p->Lam;
    a.phi = p->phi;
    a.J = p->J;
    a.F = p->F;
    a.active = p->active;
    a.flags = p->flags;
    a.jhist = jhist;
    a.count = count;
    a.work = p->sm_work;
    a.tau = p->tau;
    a.rho = rho;
    a.fid_stop = fid_stop;
    a.n_iter = n_iter;
    a.first_boundary = first_boundary ? 1 : 0;
    a.use_active = use_active ? 1 : 0;
    {
        TimeScope ts(p, KID_SMALL_SOLVE);
        hipLaunchKernelGGL(k_small_solve, dim3(p->B), dim3(NT), 0, p->stream, a);
        if (hipGetLastError() != hipSuccess) return ISM_E_DEVICE;
    }
    // J, F, the boundaries and intermediate states belong to the current controls; the
    // per-pass path's Taylor parameters do not
    p->bvalid = true;
    p->tp_valid = false;
    return ISM_OK;
}

hipError_t small_launch_done(ism_problem* p) {
    hipLaunchKernelGGL(k_small_done, dim3(1), dim3(256), 0, p->stream, p->sm_count, p->B,
                       p->flags);
    return hipGetLastError();
}

}  // namespace ism
