// Gross-Pitaevskii path (Sec. 4.C): i d/dt psi = (-1/2 d_xx + V(x,u) + g|psi|^2) psi on a
// periodic grid of n = 1024 or 4096 points, V(x,u) = V0(x) + u V1(x) + u^2 V2, one control.
//
// Step map: Strang splitting (Eq. (OS)) with exact kinetic half steps in Fourier space,
//   a_j = F^-1 Kh F psi_j,  b_j = e^{-i theta_j} a_j,  theta_j = tau (V(x,u_j) + g |a_j|^2),
//   psi_{j+1} = F^-1 Kh F b_j,  Kh = e^{-i tau k^2/4}.
// Consecutive kinetic half steps are fused: a_{j+1} = F^-1 Kh^2 F b_j, so a step costs one
// forward and one inverse FFT; psi itself is formed only at slice boundaries.
//
// Exact discrete adjoint (real inner product Re<.|.>), fused the same way:
//   nu'_j = F^-1 conj(Kh) F nu_{j+1};  g_j = dx sum_m dV/du Im(conj(nu'_j) b_j);
//   w = e^{+i theta_j} nu'_j;  mu_j = w + 2 tau g Im(conj(w) a_j) a_j;
//   nu_j = F^-1 conj(Kh) F mu_j  (nu'_{j-1} = F^-1 conj(Kh)^2 F mu_j).
//
// ISM, BEC variant (Sec. 4.C): slice n starts from psi(t_n) on the forward trajectory and
// its adjoint ends on nu(t_{n+1}) of the adjoint trajectory; both boundary sequences come
// from one sequential forward and one sequential adjoint sweep (the map is nonlinear, so
// no slice propagator exists to assemble).  The slice gradient equals the plain gradient
// on the slice (weight 1).
//
// FFT: radix-4 Stockham, natural order in and out, ping-pong buffers in LDS, one
// butterfly per thread per pass (n/4 threads), twiddles from a table built in FP64.
// The whole state stays in LDS for the entire sweep.
#include <math.h>

#include <algorithm>
#include <vector>

#include "ism_paths.h"

namespace ism {
namespace {

template <typename R> struct Cx { R re, im; };

template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
    return Cx<R>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b) {    // a * conj(b)
    return Cx<R>{a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

__device__ __forceinline__ void sincos_r(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_r(double x, double* s, double* c) { sincos(x, s, c); }

// Radix-4 Stockham FFT of n points held in LDS buffer `a` (scratch `b`), n/4 threads.
// SIGN = -1: forward e^{-2 pi i jk/n}; SIGN = +1: inverse without the 1/n factor.
// Returns the buffer holding the result.
template <typename R>
__device__ __forceinline__ Cx<double> up(Cx<R> v) {
    return Cx<double>{(double)v.re, (double)v.im};
}
template <typename R>
__device__ __forceinline__ Cx<R> down(Cx<double> v) {
    return Cx<R>{(R)v.re, (R)v.im};
}

// The butterflies run in FP64 with FP64 twiddles whatever the storage precision R: with
// FP32-rounded twiddles every transform is non-unitary in the same way at every step and
// the error grows linearly over a sweep; rounding only the stored values keeps it a random
// walk.
template <typename R, int SIGN>
__device__ Cx<R>* fft_lds(Cx<R>* a, Cx<R>* b, const Cx<double>* __restrict__ tw, int n) {
    const int j = threadIdx.x, q = n >> 2;
    for (int Ns = 1; Ns < n; Ns <<= 2) {
        Cx<double> v0 = up(a[j]), v1 = up(a[j + q]), v2 = up(a[j + 2 * q]), v3 = up(a[j + 3 * q]);
        const int k = j & (Ns - 1);
        const int stride = n / (4 * Ns);
        if (Ns > 1) {
            Cx<double> w1 = tw[k * stride], w2 = tw[2 * k * stride], w3 = tw[3 * k * stride];
            if (SIGN > 0) {
                w1.im = -w1.im;
                w2.im = -w2.im;
                w3.im = -w3.im;
            }
            v1 = cmul(v1, w1);
            v2 = cmul(v2, w2);
            v3 = cmul(v3, w3);
        }
        const Cx<double> a0{v0.re + v2.re, v0.im + v2.im}, a1{v0.re - v2.re, v0.im - v2.im};
        const Cx<double> a2{v1.re + v3.re, v1.im + v3.im};
        // (v1 - v3) times -i (forward) or +i (inverse)
        const Cx<double> a3 = SIGN < 0 ? Cx<double>{v1.im - v3.im, -(v1.re - v3.re)}
                                       : Cx<double>{-(v1.im - v3.im), v1.re - v3.re};
        const int idx = (j / Ns) * Ns * 4 + k;
        __syncthreads();                      // every thread has read a[]
        b[idx] = down<R>(Cx<double>{a0.re + a2.re, a0.im + a2.im});
        b[idx + Ns] = down<R>(Cx<double>{a1.re + a3.re, a1.im + a3.im});
        b[idx + 2 * Ns] = down<R>(Cx<double>{a0.re - a2.re, a0.im - a2.im});
        b[idx + 3 * Ns] = down<R>(Cx<double>{a1.re - a3.re, a1.im - a3.im});
        __syncthreads();
        Cx<R>* t = a;
        a = b;
        b = t;
    }
    return a;
}

struct GpeArgs {
    int B, n, K, N;
    const int* s;
    double tau, dx, g;
    const double* V0;
    const double* V1;
    double V2;
    const void* tw;        // n twiddles e^{-2 pi i t/n} (FP64)
    const void* Kh;        // n: e^{-i tau k^2/4} / n (FP64)
    const void* Kf;        // n: e^{-i tau k^2/2} / n (FP64)
    double* u;             // B*K
    const double* alpha;   // unused by the model (alpha = 0 in Sec. 4.C), kept for uniformity
    dcx* Psi;              // B*(N+1)*n  psi(t_n)
    dcx* Lam;              // B*(N+1)*n  nu(t_n)
    const dcx* psi0;       // n
    const dcx* target;     // n
    void* traj;            // B*K*n  a_j (FP32 in the mixed path, FP64 in the plain path)
    double* J;
    double* F;
    double* Jhist;
    int* active;
    double fid_stop;
    int* flags;
    double* grad;          // B*K or null
    double rho;
    int update;
};

template <typename R>
__device__ __forceinline__ double block_sum(double v, double* red) {
    // wave reduction, then across wavefronts (deterministic order)
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// theta_j and b_j = e^{-i theta} a_j for this thread's four points; V formed in FP64.
template <typename R>
__device__ __forceinline__ void potential_phase(const GpeArgs& A, const double (&v0)[4],
                                                const double (&v1)[4], double u,
                                                const Cx<double> (&a)[4], Cx<R> (&e)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double V = v0[r] + u * v1[r] + u * u * A.V2;
        const R th = (R)(A.tau * (V + A.g * (a[r].re * a[r].re + a[r].im * a[r].im)));
        R sn, cs;
        sincos_r(th, &sn, &cs);
        e[r] = Cx<R>{cs, -sn};   // e^{-i theta}
    }
}

// Forward steps j = j0 .. j1-1 starting from a_{j0} held in buf (LDS, natural order).
// Stores a_j in traj; if psi_out is given, psi_{j1} = F^-1 Kh F b_{j1-1} is written there.
// On return buf holds a_{j1} (if want_next) — used by the sequential sweep.
template <typename R>
__device__ Cx<double>* forward_steps(const GpeArgs& A, int b, int j0, int j1, Cx<double>* buf,
                                     Cx<double>* scr,
                                const double (&v0)[4], const double (&v1)[4], Cx<R>* traj_b,
                                dcx* psi_out, bool want_next) {
    const int n = A.n, q = n >> 2, t = threadIdx.x;
    const Cx<double>* tw = reinterpret_cast<const Cx<double>*>(A.tw);
    const Cx<double>* Kh = reinterpret_cast<const Cx<double>*>(A.Kh);
    const Cx<double>* Kf = reinterpret_cast<const Cx<double>*>(A.Kf);
    for (int j = j0; j < j1; ++j) {
        Cx<double> a[4];
        Cx<R> e[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = buf[t + r * q];
#pragma unroll
        for (int r = 0; r < 4; ++r) traj_b[(size_t)j * n + t + r * q] = down<R>(a[r]);
        if (j == j1 - 1 && !psi_out && !want_next) return buf;   // trajectory complete
        const double u = A.u[(size_t)b * A.K + j];
        potential_phase<R>(A, v0, v1, u, a, e);
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[t + r * q] = cmul(a[r], up(e[r]));   // b_j
        __syncthreads();
        Cx<double>* fb = fft_lds<double, -1>(buf, scr, tw, n);                      // F b_j
        Cx<double>* other = fb == buf ? scr : buf;
        const bool last = (j == j1 - 1);
        if (last && psi_out) {
            // psi_{j1} = F^-1 Kh F b_j into `other`, then back to fb's data for a_{j+1}
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = t + r * q;
                other[m] = cmul(fb[m], Kh[m]);
            }
            __syncthreads();
            // keep F b_j: transform a copy
            Cx<double> keep[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) keep[r] = fb[t + r * q];
            __syncthreads();
            Cx<double>* pr = fft_lds<double, 1>(other, fb, tw, n);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = t + r * q;
                psi_out[m] = dcx{(double)pr[m].re, (double)pr[m].im};
            }
            __syncthreads();
            if (!want_next) return pr;
            Cx<double>* dst = pr == buf ? scr : buf;
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[t + r * q] = keep[r];
            __syncthreads();
            fb = dst;
            other = dst == buf ? scr : buf;
        } else if (last && !want_next) {
            return fb;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = t + r * q;
            fb[m] = cmul(fb[m], Kf[m]);
        }
        __syncthreads();
        Cx<double>* an = fft_lds<double, 1>(fb, other, tw, n);                      // a_{j+1}
        if (an != buf) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = t + r * q;
                const Cx<double> v = an[m];
                __syncthreads();
                buf[m] = v;
            }
            __syncthreads();
        }
    }
    return buf;
}

// nu'_{j} from nu_{j+1} held in buf:  F^-1 conj(Kh) F nu
template <typename R>
__device__ Cx<double>* adj_half_kick(const GpeArgs& A, Cx<double>* buf, Cx<double>* scr, bool full) {
    const int n = A.n, q = n >> 2, t = threadIdx.x;
    const Cx<double>* tw = reinterpret_cast<const Cx<double>*>(A.tw);
    const Cx<double>* Kt = reinterpret_cast<const Cx<double>*>(full ? A.Kf : A.Kh);
    Cx<double>* f = fft_lds<double, -1>(buf, scr, tw, n);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = t + r * q;
        f[m] = cmulc(f[m], Kt[m]);
    }
    __syncthreads();
    Cx<double>* o = f == buf ? scr : buf;
    return fft_lds<double, 1>(f, o, tw, n);
}

// Adjoint steps j = j1-1 down to j0, starting from nu'_{j1-1} in buf; a_j read from traj.
// Every step but the last continues with the fused kick (nu'_{j-1} in buf); after the last
// step final_kick selects: 0 nothing, 1 the half kick nu_{j0} (written to nu_out),
// 2 the fused kick nu'_{j0-1}.  Computes the gradient of each step if grad_on.
template <typename R>
__device__ void adjoint_steps(const GpeArgs& A, int b, int j0, int j1, Cx<double>* buf,
                              Cx<double>* scr,
                              const double (&v0)[4], const double (&v1)[4], const Cx<R>* traj_b,
                              dcx* nu_out, int final_kick, bool grad_on, bool upd, double* red) {
    const int n = A.n, q = n >> 2, t = threadIdx.x;
    for (int j = j1 - 1; j >= j0; --j) {
        Cx<double> a[4], nup[4];
        Cx<R> e[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a[r] = up(traj_b[(size_t)j * n + t + r * q]);
            nup[r] = buf[t + r * q];
        }
        const double u = A.u[(size_t)b * A.K + j];
        potential_phase<R>(A, v0, v1, u, a, e);
        if (grad_on) {
            double part = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const Cx<double> bb = cmul(a[r], up(e[r]));
                const double dV = v1[r] + 2.0 * u * A.V2;
                // Im(conj(nu') b)
                part += dV * ((double)nup[r].re * (double)bb.im - (double)nup[r].im * (double)bb.re);
            }
            const double gj = A.dx * block_sum<R>(part, red);
            if (t == 0) {
                const size_t ui = (size_t)b * A.K + j;
                if (A.grad) A.grad[ui] = gj;
                if (upd) A.u[ui] = fma(A.rho, gj, u);
                if (!(fabs(gj) < 1e300)) atomicOr(&A.flags[0], 1);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // w = e^{+i theta} nu' = nu' * conj(e);  mu = w + 2 tau g Im(conj(w) a) a
            const Cx<double> w = cmulc(nup[r], up(e[r]));
            const Cx<double> ad = a[r];
            const double f = 2.0 * A.tau * A.g * (w.re * ad.im - w.im * ad.re);
            buf[t + r * q] = Cx<double>{w.re + f * ad.re, w.im + f * ad.im};
        }
        __syncthreads();
        const bool last = (j == j0);
        if (last && final_kick == 0) break;
        Cx<double>* res = adj_half_kick<R>(A, buf, scr, !(last && final_kick == 1));
        if (last && nu_out && final_kick == 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = t + r * q;
                nu_out[m] = dcx{(double)res[m].re, (double)res[m].im};
            }
        }
        if (res != buf) {
            Cx<double> v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = res[t + r * q];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) buf[t + r * q] = v[r];
        }
        __syncthreads();
    }
}

template <typename R>
__device__ __forceinline__ void load_pot(const GpeArgs& A, double (&v0)[4], double (&v1)[4]) {
    const int q = A.n >> 2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        v0[r] = A.V0[threadIdx.x + r * q];
        v1[r] = A.V1[threadIdx.x + r * q];
    }
}

// a_{j0} = F^-1 Kh F psi with psi (FP64) read from src
template <typename R>
__device__ Cx<double>* first_half_kick(const GpeArgs& A, const dcx* src, Cx<double>* buf,
                                       Cx<double>* scr) {
    const int n = A.n, q = n >> 2, t = threadIdx.x;
    const Cx<double>* tw = reinterpret_cast<const Cx<double>*>(A.tw);
    const Cx<double>* Kh = reinterpret_cast<const Cx<double>*>(A.Kh);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const dcx v = src[t + r * q];
        buf[t + r * q] = Cx<double>{v.re, v.im};
    }
    __syncthreads();
    Cx<double>* f = fft_lds<double, -1>(buf, scr, tw, n);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = t + r * q;
        f[m] = cmul(f[m], Kh[m]);
    }
    __syncthreads();
    Cx<double>* o = f == buf ? scr : buf;
    Cx<double>* res = fft_lds<double, 1>(f, o, tw, n);
    if (res != buf) {
        Cx<double> v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = res[t + r * q];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[t + r * q] = v[r];
        __syncthreads();
    }
    return buf;
}

// Sequential forward sweep of one instance: psi(t_n) for every n, a_j for every step,
// J and F at T.
template <typename R>
__global__ __launch_bounds__(1024) void k_gpe_fwd_sweep(GpeArgs A) {
    extern __shared__ unsigned char smem_raw[];
    Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem_raw);
    Cx<double>* scr = buf + A.n;
    double* red = reinterpret_cast<double*>(scr + A.n);
    const int b = blockIdx.x, n = A.n, q = n >> 2, t = threadIdx.x;
    double v0[4], v1[4];
    load_pot<R>(A, v0, v1);
    dcx* Psi_b = A.Psi + (size_t)b * (A.N + 1) * n;
    Cx<R>* traj_b = reinterpret_cast<Cx<R>*>(A.traj) + (size_t)b * A.K * n;
#pragma unroll
    for (int r = 0; r < 4; ++r) Psi_b[t + r * q] = A.psi0[t + r * q];
    first_half_kick<R>(A, A.psi0, buf, scr);
    for (int nn = 0; nn < A.N; ++nn) {
        forward_steps<R>(A, b, A.s[nn], A.s[nn + 1], buf, scr, v0, v1, traj_b,
                         Psi_b + (size_t)(nn + 1) * n, nn + 1 < A.N);
        __syncthreads();
    }
    // J = Re <psi_K|psi_f> dx, F = |<psi_K|psi_f> dx|^2
    const dcx* pK = Psi_b + (size_t)A.N * n;
    double zr = 0.0, zi = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const dcx p = pK[t + r * q], f = A.target[t + r * q];
        zr += p.re * f.re + p.im * f.im;
        zi += p.re * f.im - p.im * f.re;
    }
    zr = A.dx * block_sum<R>(zr, red);
    zi = A.dx * block_sum<R>(zi, red);
    if (t == 0) {
        const double F = zr * zr + zi * zi;
        A.J[b] = zr;
        A.F[b] = F;
        if (A.Jhist) A.Jhist[b] = zr;
        if (!(fabs(zr) < 1e300)) atomicOr(&A.flags[0], 1);
        if (A.active) {
            if (A.active[b] && F >= A.fid_stop) A.active[b] = 0;
            if (A.active[b]) atomicAdd(&A.flags[1], 1);
        }
    }
}

// Sequential adjoint sweep of one instance: nu(t_n) for every n.
template <typename R>
__global__ __launch_bounds__(1024) void k_gpe_adj_sweep(GpeArgs A) {
    extern __shared__ unsigned char smem_raw[];
    Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem_raw);
    Cx<double>* scr = buf + A.n;
    double* red = reinterpret_cast<double*>(scr + A.n);
    const int b = blockIdx.x, n = A.n, q = n >> 2, t = threadIdx.x;
    double v0[4], v1[4];
    load_pot<R>(A, v0, v1);
    dcx* Lam_b = A.Lam + (size_t)b * (A.N + 1) * n;
    const Cx<R>* traj_b = reinterpret_cast<const Cx<R>*>(A.traj) + (size_t)b * A.K * n;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const dcx v = A.target[t + r * q];
        Lam_b[(size_t)A.N * n + t + r * q] = v;
        buf[t + r * q] = Cx<double>{v.re, v.im};
    }
    __syncthreads();
    Cx<double>* res = adj_half_kick<R>(A, buf, scr, false);         // nu'_{K-1}
    if (res != buf) {
        Cx<double> v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = res[t + r * q];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[t + r * q] = v[r];
        __syncthreads();
    }
    for (int nn = A.N - 1; nn >= 0; --nn) {
        // steps of slice nn; at its first step nu_{s_nn} is stored and nu'_{s_nn - 1} kept
        const int j0 = A.s[nn], j1 = A.s[nn + 1];
        adjoint_steps<R>(A, b, j0 + 1, j1, buf, scr, v0, v1, traj_b, nullptr, 2, false, false, red);
        // step j0: store nu_{j0}, continue with nu'_{j0-1}
        Cx<double> a[4], nup[4];
        Cx<R> e[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a[r] = up(traj_b[(size_t)j0 * n + t + r * q]);
            nup[r] = buf[t + r * q];
        }
        potential_phase<R>(A, v0, v1, A.u[(size_t)b * A.K + j0], a, e);
        Cx<double> mu[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const Cx<double> w = cmulc(nup[r], up(e[r]));
            const Cx<double> ad = a[r];
            const double f = 2.0 * A.tau * A.g * (w.re * ad.im - w.im * ad.re);
            mu[r] = Cx<double>{w.re + f * ad.re, w.im + f * ad.im};
            buf[t + r * q] = mu[r];
        }
        __syncthreads();
        Cx<double>* nu = adj_half_kick<R>(A, buf, scr, false);         // nu_{j0}
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = t + r * q;
            Lam_b[(size_t)nn * n + m] = dcx{(double)nu[m].re, (double)nu[m].im};
        }
        __syncthreads();
        if (nn == 0) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[t + r * q] = mu[r];
        __syncthreads();
        res = adj_half_kick<R>(A, buf, scr, true);               // nu'_{j0-1}
        if (res != buf) {
            Cx<double> v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = res[t + r * q];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) buf[t + r * q] = v[r];
        }
        __syncthreads();
    }
}

// Slice n of instance b: forward from psi(t_n), adjoint from nu(t_{n+1}), gradient, update.
template <typename R>
__global__ __launch_bounds__(1024) void k_gpe_slice(GpeArgs A) {
    extern __shared__ unsigned char smem_raw[];
    Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem_raw);
    Cx<double>* scr = buf + A.n;
    double* red = reinterpret_cast<double*>(scr + A.n);
    const int nn = blockIdx.x, b = blockIdx.y, n = A.n, q = n >> 2, t = threadIdx.x;
    double v0[4], v1[4];
    load_pot<R>(A, v0, v1);
    const int j0 = A.s[nn], j1 = A.s[nn + 1];
    Cx<R>* traj_b = reinterpret_cast<Cx<R>*>(A.traj) + (size_t)b * A.K * n;
    const dcx* Psi_b = A.Psi + (size_t)b * (A.N + 1) * n;
    const dcx* Lam_b = A.Lam + (size_t)b * (A.N + 1) * n;
    first_half_kick<R>(A, Psi_b + (size_t)nn * n, buf, scr);
    forward_steps<R>(A, b, j0, j1, buf, scr, v0, v1, traj_b, nullptr, false);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const dcx v = Lam_b[(size_t)(nn + 1) * n + t + r * q];
        buf[t + r * q] = Cx<double>{v.re, v.im};
    }
    __syncthreads();
    Cx<double>* res = adj_half_kick<R>(A, buf, scr, false);            // nu'_{j1-1}
    if (res != buf) {
        Cx<double> v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = res[t + r * q];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[t + r * q] = v[r];
        __syncthreads();
    }
    const bool upd = A.update && (A.active == nullptr || A.active[b] != 0);
    adjoint_steps<R>(A, b, j0, j1, buf, scr, v0, v1, traj_b, nullptr, 0, true, upd, red);
}

}  // namespace

struct GpeExt {
    int n = 0;
    double L = 0, g = 0, V2 = 0, dx = 0;
    double* V0 = nullptr;
    double* V1 = nullptr;
    void* tw = nullptr;
    void* Kh = nullptr;
    void* Kf = nullptr;
    dcx* Psi = nullptr;
    dcx* Lam = nullptr;
    dcx* psi0 = nullptr;
    dcx* target = nullptr;
    void* traj = nullptr;
};

static void gpe_free(ism_problem* p) {
    delete reinterpret_cast<GpeExt*>(p->ext);
    p->ext = nullptr;
}

size_t gpe_footprint_extra(size_t n, int K, int N, int batch, int precision) {
    const size_t rs = precision == ISM_FP64 ? 16 : 8;
    return (size_t)batch * K * n * rs + 2 * (size_t)batch * (N + 1) * n * 16 + 3 * n * rs;
}

static GpeArgs gpe_args(ism_problem* p) {
    GpeExt* x = reinterpret_cast<GpeExt*>(p->ext);
    GpeArgs A{};
    A.B = p->B;
    A.n = x->n;
    A.K = p->K;
    A.N = p->N;
    A.s = p->s;
    A.tau = p->tau;
    A.dx = x->dx;
    A.g = x->g;
    A.V0 = x->V0;
    A.V1 = x->V1;
    A.V2 = x->V2;
    A.tw = x->tw;
    A.Kh = x->Kh;
    A.Kf = x->Kf;
    A.u = p->u;
    A.alpha = p->alpha;
    A.Psi = x->Psi;
    A.Lam = x->Lam;
    A.psi0 = x->psi0;
    A.target = x->target;
    A.traj = x->traj;
    A.J = p->J;
    A.F = p->F;
    A.flags = p->flags;
    return A;
}

static size_t gpe_shmem(int n, int prec) {
    (void)prec;   // the LDS-resident state is FP64 in both precisions
    return 2 * (size_t)n * 16 + 16 * sizeof(double);
}

template <typename R>
static int gpe_boundary_t(ism_problem* p, double* Jhist_k, double fid_stop, bool use_active) {
    GpeArgs A = gpe_args(p);
    A.Jhist = Jhist_k;
    A.active = use_active ? p->active : nullptr;
    A.fid_stop = fid_stop;
    const size_t shm = gpe_shmem(A.n, p->precision);
    {
        TimeScope ts(p, KID_GPE_SWEEP);
        hipLaunchKernelGGL(k_gpe_fwd_sweep<R>, dim3(p->B), dim3(A.n / 4), shm, p->stream, A);
        hipLaunchKernelGGL(k_gpe_adj_sweep<R>, dim3(p->B), dim3(A.n / 4), shm, p->stream, A);
    }
    if (hipGetLastError() != hipSuccess) return ISM_E_DEVICE;
    p->bvalid = true;
    return ISM_OK;
}

template <typename R>
static int gpe_slice_t(ism_problem* p, int update, double rho, double* grad, bool use_active) {
    GpeArgs A = gpe_args(p);
    A.grad = grad;
    A.rho = rho;
    A.update = update;
    A.active = use_active ? p->active : nullptr;
    const size_t shm = gpe_shmem(A.n, p->precision);
    {
        TimeScope ts(p, KID_GPE_SLICE);
        hipLaunchKernelGGL(k_gpe_slice<R>, dim3(p->N, p->B), dim3(A.n / 4), shm, p->stream, A);
    }
    if (hipGetLastError() != hipSuccess) return ISM_E_DEVICE;
    if (update) p->bvalid = false;
    return ISM_OK;
}

int gpe_boundary_pass(ism_problem* p, double* Jhist_k, double fid_stop, bool use_active) {
    return p->precision == ISM_FP64 ? gpe_boundary_t<double>(p, Jhist_k, fid_stop, use_active)
                                    : gpe_boundary_t<float>(p, Jhist_k, fid_stop, use_active);
}

int gpe_slice_pass(ism_problem* p, int update, double rho, double* grad, bool use_active) {
    return p->precision == ISM_FP64 ? gpe_slice_t<double>(p, update, rho, grad, use_active)
                                    : gpe_slice_t<float>(p, update, rho, grad, use_active);
}

int gpe_copy_state(ism_problem* p, double* out, int which_end) {
    GpeExt* x = reinterpret_cast<GpeExt*>(p->ext);
    const size_t n = x->n;
    const dcx* base = which_end == 0 ? x->Psi + (size_t)p->N * n : x->Lam;
    return copy_rows_out(p, out, base, n * sizeof(dcx), (size_t)(p->N + 1) * n * sizeof(dcx), p->B);
}

template <typename R>
static int upload_cx(ism_problem* p, void** dst, const std::vector<dcx>& v) {
    std::vector<R> h(2 * v.size());
    for (size_t i = 0; i < v.size(); ++i) {
        h[2 * i] = (R)v[i].re;
        h[2 * i + 1] = (R)v[i].im;
    }
    return dev_upload(p, dst, h.data(), h.size() * sizeof(R));
}

int gpe_create(ism_problem* p, int n, double L, double g, const double* V0, const double* V1,
               double V2, const double* psi0, const double* target) {
    GpeExt* x = new (std::nothrow) GpeExt();
    if (!x) return ISM_E_NOMEM;
    p->ext = x;
    p->ext_free = gpe_free;
    x->n = n;
    x->L = L;
    x->g = g;
    x->V2 = V2;
    x->dx = L / n;
    int st;
    if ((st = dev_upload(p, (void**)&x->V0, V0, n * sizeof(double)))) return st;
    if ((st = dev_upload(p, (void**)&x->V1, V1, n * sizeof(double)))) return st;
    if ((st = dev_upload(p, (void**)&x->psi0, psi0, n * sizeof(dcx)))) return st;
    if ((st = dev_upload(p, (void**)&x->target, target, n * sizeof(dcx)))) return st;
    const double PI = 3.14159265358979323846;
    std::vector<dcx> tw(n), kh(n), kf(n);
    for (int t = 0; t < n; ++t) tw[t] = dcx{cos(2 * PI * t / n), -sin(2 * PI * t / n)};
    for (int m = 0; m < n; ++m) {
        const int f = m < n / 2 ? m : m - n;            // fftfreq ordering
        const double k = 2 * PI * f / L;
        const double ph = -p->tau * k * k / 4;
        kh[m] = dcx{cos(ph) / n, sin(ph) / n};
        kf[m] = dcx{cos(2 * ph) / n, sin(2 * ph) / n};
    }
    const bool f64 = p->precision == ISM_FP64;
    if ((st = upload_cx<double>(p, &x->tw, tw))) return st;       // tables stay FP64
    if ((st = upload_cx<double>(p, &x->Kh, kh))) return st;
    if ((st = upload_cx<double>(p, &x->Kf, kf))) return st;
    const size_t nb = (size_t)p->B * (p->N + 1) * n * sizeof(dcx);
    if ((st = dev_alloc(p, (void**)&x->Psi, nb))) return st;
    if ((st = dev_alloc(p, (void**)&x->Lam, nb))) return st;
    if ((st = dev_alloc(p, &x->traj, (size_t)p->B * p->K * n * (f64 ? 16 : 8)))) return st;
    const size_t shm = gpe_shmem(n, p->precision);
    const hipError_t e1 = f64 ? hipFuncSetAttribute((const void*)k_gpe_fwd_sweep<double>,
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm)
                              : hipFuncSetAttribute((const void*)k_gpe_fwd_sweep<float>,
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    const hipError_t e2 = f64 ? hipFuncSetAttribute((const void*)k_gpe_adj_sweep<double>,
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm)
                              : hipFuncSetAttribute((const void*)k_gpe_adj_sweep<float>,
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    const hipError_t e3 = f64 ? hipFuncSetAttribute((const void*)k_gpe_slice<double>,
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm)
                              : hipFuncSetAttribute((const void*)k_gpe_slice<float>,
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return ISM_E_DEVICE;
    return ISM_OK;
}

}  // namespace ism

extern "C" int ism_problem_create_gpe(ism_problem** out, int n_grid, double L, double g,
                                      const double* V0, const double* V1, double V2,
                                      const double* psi0, const double* target, double T, int K,
                                      int N, const ism_options* opt) {
    using namespace ism;
    if (!out || !V0 || !V1 || !psi0 || !target) return ISM_E_ARG;
    ism_options o;
    ism_default_options(&o);
    if (opt) o = *opt;
    o.kind = ISM_STATE;
    if (n_grid != 1024 && n_grid != 4096) return n_grid > 0 ? ISM_E_UNSUPPORTED : ISM_E_ARG;
    if (!(L > 0.0) || !std::isfinite(L) || !std::isfinite(g) || !std::isfinite(V2)) return ISM_E_ARG;
    int st = validate_common(n_grid, 1, T, K, N, &o);
    if (st) return st;
    if (o.alpha) {          // the condensate problem carries no control penalty (Sec. 4.C)
        for (int i = 0; i < o.alpha_len; ++i)
            if (o.alpha[i] != 0.0) return ISM_E_UNSUPPORTED;
    }
    for (int i = 0; i < n_grid; ++i)
        if (!std::isfinite(V0[i]) || !std::isfinite(V1[i])) return ISM_E_ARG;
    for (int i = 0; i < 2 * n_grid; ++i)
        if (!std::isfinite(psi0[i]) || !std::isfinite(target[i])) return ISM_E_ARG;
    ism_problem* p = new (std::nothrow) ism_problem();
    if (!p) return ISM_E_NOMEM;
    st = common_setup(p, n_grid, 1, T, K, N, &o);
    if (!st) {
        p->path = PATH_GPE;
        st = gpe_create(p, n_grid, L, g, V0, V1, V2, psi0, target);
    }
    if (st) {
        ism_problem_destroy(p);
        return st;
    }
    *out = p;
    return ISM_OK;
}
