// Dense gate path (evolution operators, the remark of Sec. 2): the propagated object
// is the d x d evolution operator, psi0 = I, target W, <A|B> = Tr(A^+ B)/d.
//
// One ISM iteration (Algorithm 1, one gradient step per slice):
//   build     U_j = exp(-i tau H_j) for every step, in FP64 (row r of U_j is the
//             action of exp(-i tau conj(H_j)) on e_r, a truncated Taylor series of a
//             sparse generator), stored in the path's precision, re/im planes split;
//   assemble  P_j = U_j U_{j-1} ... U_{s_n} for every step of slice n (d <= 64: a chunked
//             scan of 32 x 32 or 64 x 64 products; larger d: a chain of batched complex
//             GEMMs over the slices); M_n = P_{s_{n+1}-1}  (propagator assembling, Sec. 3);
//   boundary  Psi_{n+1} = M_n Psi_n, Lambda_n = M_n^+ Lambda_{n+1} (FP64 GEMMs),
//             phi_n (Eq. (cible)), J and F;
//   sweeps    the slice trajectories from phi_n (forward) and phi_{n+1} (adjoint) are
//             X_j = P_{j-1} phi_n and Y_j = P_{j-1} (M_n^+ phi_{n+1}), one batched GEMM
//             [X_j | Y_j] = P_{j-1} [phi_n | M_n^+ phi_{n+1}] over every step at once
//             (d <= 32: on the leading 32 x 32 blocks only);
//   gradient  g_{j,c} = beta_n Im Tr(Y_j^+ Hhat_{c,j} X_j)/d - alpha_j u_{j,c} (Theorem 2),
//             with the step average Hhat of H_c evaluated column by column through
//               <y|Hhat_c|x> = sum_{a+b<=m} w_ab <(tau H')^a y | H_c | (tau H')^b x>,
//               w_ab = i^{a+b} (-1)^b / ((a+b+1) a! b!),  H' = H_j - s,
//             which is the series of (1/tau) int_0^tau e^{isH} H_c e^{-isH} ds written with
//             Krylov vectors of the two states (no extra dense product);
//   update    u += rho g (Eq. (gradStep), ascent).
//
// Complex GEMM: C = op(A) op(B), op in {N, conjugate transpose}, on MFMA
// (v_mfma_*_16x16x4) with the real and imaginary tiles staged separately in LDS;
// 64 x 64 output tile per workgroup of four wavefronts, 32 x 32 per wavefront,
// Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.  FP32 operands with FP32 accumulation
// (mixed path) or FP64 throughout (plain path; the boundary products are FP64 in both).
#include <math.h>

#include <cmath>

#include <algorithm>
#include <vector>

#include "ism_paths.h"

namespace ism {
namespace {

constexpr int GT = 64;        // output tile (rows and columns)
constexpr int MMAX_G = 24;    // largest Taylor / Krylov order
constexpr int RB = 8;         // rows of U built per workgroup
constexpr int CBW = 128;      // columns per workgroup in the gradient kernel
constexpr int CMAX_G = 32;    // largest number of controls in the gate path
constexpr int WMAX_G = 16;    // largest union-pattern width

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// complex LDS slot of the gradient's Krylov buffers (real and imaginary part side by side)
template <typename R> struct alignas(2 * sizeof(R)) Cx { R re, im; };

template <typename R> struct Acc;
template <> struct Acc<float> { typedef f4 T; };
template <> struct Acc<double> { typedef d4 T; };

// Workgroup barrier that orders LDS only.  __syncthreads() also orders global memory, so it
// waits for every global load in flight (a prefetch issued before it is then no prefetch);
// this one waits for the LDS operations alone.  For loops whose threads exchange data
// through LDS only, with every prefetched value consumed before the next barrier.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One batched complex GEMM entry: element offsets of the real planes of A, B, C and
// op flags (bit 0: A conjugate-transposed, bit 1: B conjugate-transposed).
struct GemmEntry {
    long long a, b, c;
    int flags;
    int pad;
};

struct GemmArgs {
    int M, N, Kd;
    int lda, ldb, ldc;            // row strides (elements)
    long long pa, pb, pc;         // offset of the imaginary plane from the real plane
    const void* A;
    const void* B;
    void* C;
    const GemmEntry* e;
};

template <typename R, int KC>
__global__ __launch_bounds__(256, sizeof(R) == 4 ? 4 : 2) void k_zgemm(GemmArgs g) {
    __shared__ R As[2][KC][GT + 1];   // [re/im][k][i]
    __shared__ R Bs[2][KC][GT + 1];   // [re/im][k][j]
    // XCD-aware placement.  Workgroups go to the 8 XCDs round-robin by linear id, so in the
    // plain (tile, entry) order the tiles of one product land on every XCD and each XCD's
    // L2 fetches both of its operands.  Here linear id L of the first nt * ne8 workgroups
    // (ne8: the entry count rounded down to a multiple of 8) runs tile (L / 8) % nt of entry
    // ((L / 8) / nt) * 8 + L % 8: every tile of an entry on one XCD.  The remaining entries
    // keep the plain order.  Both parts are bijections, so each tile is computed as before.
    int tile, ent;
    {
        const int nt = gridDim.x, ne8 = gridDim.y & ~7;
        const int L = blockIdx.y * nt + blockIdx.x;
        if (L < nt * ne8) {
            const int s = L >> 3;
            ent = (s / nt) * 8 + (L & 7);
            tile = s % nt;
        } else {
            const int q = L - nt * ne8;
            ent = ne8 + q / nt;
            tile = q % nt;
        }
    }
    const GemmEntry e = g.e[ent];
    const R* A = reinterpret_cast<const R*>(g.A) + e.a;
    const R* Bm = reinterpret_cast<const R*>(g.B) + e.b;
    R* Cm = reinterpret_cast<R*>(g.C) + e.c;
    const int tilesN = g.N / GT;
    const int i0 = (tile / tilesN) * GT, j0 = (tile % tilesN) * GT;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const bool hA = e.flags & 1, hB = e.flags & 2, addB = e.flags & 4;
    typename Acc<R>::T cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) cr[a][b][v] = ci[a][b][v] = 0;
    // op(A)[i0:i0+64, k0:k0+KC] is staged as As[k][i] and op(B)[k0:k0+KC, j0:j0+64] as
    // Bs[k][j]; element q of a chunk (PQ per thread) is fetched into registers while the
    // previous chunk runs on MFMA, and the loop's barriers order LDS only (the kernel's
    // threads share nothing else: C never overlaps A or B), so the fetch stays in flight
    constexpr int PQ = GT * KC / 256;
    R far[PQ], fai[PQ], fbr[PQ], fbi[PQ];
    auto a_ik = [&](int q, int& i, int& k) {
        if (!hA) { i = q / KC; k = q % KC; } else { k = q / GT; i = q % GT; }
    };
    auto b_kj = [&](int q, int& kk, int& jj) {
        if (!hB) { kk = q / GT; jj = q % GT; } else { jj = q / KC; kk = q % KC; }
    };
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < PQ; ++u) {
            const int q = t + 256 * u;
            int i, k, kk, jj;
            a_ik(q, i, k);
            b_kj(q, kk, jj);
            const long long off = !hA ? (long long)(i0 + i) * g.lda + (k0 + k)
                                      : (long long)(k0 + k) * g.lda + (i0 + i);
            const long long offb = !hB ? (long long)(k0 + kk) * g.ldb + (j0 + jj)
                                       : (long long)(j0 + jj) * g.ldb + (k0 + kk);
            far[u] = A[off];
            fai[u] = A[off + g.pa];
            fbr[u] = Bm[offb];
            fbi[u] = Bm[offb + g.pb];
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < g.Kd; k0 += KC) {
#pragma unroll
        for (int u = 0; u < PQ; ++u) {
            const int q = t + 256 * u;
            int i, k, kk, jj;
            a_ik(q, i, k);
            b_kj(q, kk, jj);
            As[0][k][i] = far[u];
            As[1][k][i] = hA ? -fai[u] : fai[u];
            Bs[0][kk][jj] = fbr[u];
            Bs[1][kk][jj] = hB ? -fbi[u] : fbi[u];
        }
        lds_barrier();
        if (k0 + KC < g.Kd) fetch(k0 + KC);
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            const int kr = kk + (lane >> 4), li = lane & 15;
            R ar[2], ai[2], br[2], bi[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                ar[a] = As[0][kr][wr + a * 16 + li];
                ai[a] = As[1][kr][wr + a * 16 + li];
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                br[b] = Bs[0][kr][wc + b * 16 + li];
                bi[b] = Bs[1][kr][wc + b * 16 + li];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    cr[a][b] = mfma16(ar[a], br[b], cr[a][b]);
                    cr[a][b] = mfma16(-ai[a], bi[b], cr[a][b]);
                    ci[a][b] = mfma16(ar[a], bi[b], ci[a][b]);
                    ci[a][b] = mfma16(ai[a], br[b], ci[a][b]);
                }
        }
        lds_barrier();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // output lane layout of the 16x16x4 MFMA: f32 holds rows 4(l/16)+v,
                // f64 holds rows l/16 + 4v (columns l%16 in both)
                const int i = i0 + wr + a * 16 +
                              (sizeof(R) == 8 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
                const int j = j0 + wc + b * 16 + (lane & 15);
                const long long o = (long long)i * g.ldc + j;
                if (addB) {                       // C = A B + B (square, B not transposed)
                    const long long ob = (long long)i * g.ldb + j;
                    Cm[o] = cr[a][b][v] + Bm[ob];
                    Cm[o + g.pc] = ci[a][b][v] + Bm[ob + g.pb];
                } else {
                    Cm[o] = cr[a][b][v];
                    Cm[o + g.pc] = ci[a][b][v];
                }
            }
}

// ---------------------------------------------------------------------------------
// data of the generator on the union sparsity pattern of H0 and all H_c (ELL, width W)
// ---------------------------------------------------------------------------------
struct GateGen {
    int d, dp, W, C, K;
    const int* col;          // d*W column of each stored entry (padding: own row)
    const dcx* h0v;          // d*W  values of H0 - s I
    const dcx* hcu;          // C*d*W values of H_c on the union pattern
    const int* wq;           // d*W*CW: the controls with an entry at position w of row r's
                             // union pattern (padding: control 0 with value 0)
    const dcx* wv;           // d*W*CW: those entries of H_c
    int CW;
    const double* u;         // K*C
    double tau, shift;
    double h0norm;           // || H0 - s ||_inf
    const double* cnorm;     // C  || H_c ||_inf
    int cn;                  // 1: Crank-Nicolson (Cayley) step map, no spectral shift (s = 0)
};

__device__ __forceinline__ int taylor_terms(double theta, double tol, int& S) {
    S = 1;
    if (!(theta < 1e4)) return -1;
    S = (int)ceil(theta / 1.0);
    if (S < 1) S = 1;
    const double ts = theta / S, ex = exp(ts);
    int m = 1;
    double term = ts;
    while (m < MMAX_G) {
        const double next = term * ts / (m + 1);
        if (next * ex <= tol) break;
        term = next;
        ++m;
    }
    return m;
}

// Terms of the Neumann series sum_k (-L)^k of (I + L)^{-1}, ||L|| <= theta, until the
// remainder theta^(n+1) / (1 - theta) is below tol; -1 beyond the useful range (theta at
// least `lim`: 0.25 in FP64, 0.45 in FP32), which is reported, never truncated.
__device__ __forceinline__ int neumann_terms(double theta, double tol, double lim) {
    if (!(theta < lim)) return -1;
    int n = 1;
    double rem = theta * theta / (1.0 - theta);
    while (n < 64 && rem > tol) {
        ++n;
        rem *= theta;
    }
    return rem > tol ? -1 : n;
}

// Krylov order of the gradient series at step j (at most cap): the dropped terms
// (2 theta)^n / (n+1)!, n > m, theta = tau (||H_0 - s|| + sum_c |u_c| ||H_c||), are below
// the path's tolerance; rem is the first dropped term.
template <typename R>
__device__ __forceinline__ int grad_order(const GateGen& gg, int j, int cap, double& rem) {
    const double* uj = gg.u + (size_t)j * gg.C;
    double bound = gg.h0norm;
    for (int q = 0; q < gg.C; ++q) bound += fabs(uj[q]) * gg.cnorm[q];
    const double x = 2.0 * gg.tau * bound;
    const double tol = sizeof(R) == 8 ? 1e-17 : fmin(1e-8, 1e-5 / (double)gg.K);
    int m = 1;
    rem = x * x / 6.0;
    while (m < cap && rem > tol) {
        ++m;
        rem = rem * x / (m + 2);
    }
    return m;
}

// Rows r0..r0+RB-1 of U_j = e^{-i tau s} exp(-i tau (H_j - s)) (FP64), stored as R; the
// largest Krylov order the gradient needs at these controls goes to kmax (cleared before).
// Thread t holds component c = t mod lpc of the rows of row block t / lpc: lpc = dp unless
// d <= 32, where lpc is the least power of two >= d and a workgroup of dp = 64 threads takes
// 64 / lpc row blocks at once.  Entries of D_j outside the problem's rows and columns are
// zero from the clear at create and are not written.
// VS: row stride of the LDS vectors, dp rounded up to 64 or 256 (a 256-wide array at dp = 64
// would hold 32 KB per one-wavefront workgroup and cap the residency at 5 per CU).
template <typename R, int WT, int VS>
__global__ __launch_bounds__(256) void k_gate_build(GateGen gg, R* U, long long plane, int* flags,
                                                    int* kmax) {
    __shared__ dcx vs[RB * VS];
    const int j = blockIdx.x, t = threadIdx.x;
    const int d = gg.d, dp = gg.dp;
    int lpc = dp;
    if (d <= 32) {
        lpc = 1;
        while (lpc < d) lpc <<= 1;
    }
    // lpc is dp (a multiple of 64, not always a power of two) or a power of two up to 32
    const int c = t % lpc, base = t - c, grp = t / lpc, ngrp = dp / lpc;
    const double* uj = gg.u + (size_t)j * gg.C;
    // row c of conj(H_j - s) on the union pattern
    dcx hv[WT];
    int hc[WT];
    double theta = gg.h0norm;
    for (int q = 0; q < gg.C; ++q) theta += fabs(uj[q]) * gg.cnorm[q];
    theta *= gg.tau;
    int S;
    // FP64 path: truncation below FP64 rounding.  FP32 path (U_j stored in FP32): the
    // truncation summed over the K steps below 1e-5, never above 1e-8 per step
    const double tol = sizeof(R) == 8 ? 1e-17 : fmin(1e-8, 1e-5 / (double)gg.K);
    int m;
    if (gg.cn) {
        // Crank-Nicolson: D_j = U_j - I = -2 (I + L_j)^{-1} L_j = 2 sum_{k >= 1} (-L_j)^k,
        // L_j = (i tau/2) H_j, as a Neumann series (row r of D_j is that series of L_j^T on e_r)
        S = 1;
        m = neumann_terms(0.5 * theta, tol, sizeof(R) == 8 ? 0.25 : 0.45);
        if (m < 0) {
            if (t == 0 && blockIdx.y == 0) atomicOr(flags, theta == theta ? 2 : 1);
            m = 1;
        }
    } else {
        m = taylor_terms(theta, tol, S);
        if (m < 0) {
            if (t == 0 && blockIdx.y == 0) atomicOr(flags, 1);
            m = 1;
        }
    }
    const double ts = gg.cn ? 0.5 * gg.tau : gg.tau / S;
#pragma unroll
    for (int w = 0; w < WT; ++w) {
        dcx h = {0.0, 0.0};
        int cc = c;
        if (c < d && w < gg.W) {
            const size_t idx = (size_t)c * gg.W + w;
            h = gg.h0v[idx];
            for (int q = 0; q < gg.C; ++q) {
                const dcx x = gg.hcu[(size_t)q * d * gg.W + idx];
                h.re += uj[q] * x.re;
                h.im += uj[q] * x.im;
            }
            cc = gg.col[idx];
        }
        hv[w].re = ts * h.re;        // tau_sub * conj(H - s)
        hv[w].im = -ts * h.im;
        hc[w] = cc;
    }
    // the generator row above is set up once and serves every row block of this workgroup
    const int nrb = (d + RB - 1) / RB;
    for (int rbb = blockIdx.y * ngrp; rbb < nrb; rbb += gridDim.y * ngrp) {   // uniform
        const int rb = rbb + grp;
        const int r0 = rb * RB;
        // acc holds x - e_r, the series terms of order >= 1 only: D_j = U_j - I is formed
        // without ever holding U_j, whose entries near 1 would carry an absolute rounding
        // error of ~1e-16 that is the same at every step (it added up to 2.7e-12 over the
        // 2^15 steps of the five-spin density run)
        dcx acc[RB], tr[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[q] = dcx{0.0, 0.0};
        for (int sub = 0; sub < S; ++sub) {
#pragma unroll
            for (int q = 0; q < RB; ++q) tr[q] = dcx{acc[q].re + ((c == r0 + q) ? 1.0 : 0.0), acc[q].im};
            for (int k = 0; k < m; ++k) {
#pragma unroll
                for (int q = 0; q < RB; ++q) vs[q * VS + t] = tr[q];
                __syncthreads();
                // Taylor: -i (h x) / (k+1), all terms summed; Neumann: -i (h x), summed twice
                const double rk = gg.cn ? 1.0 : 1.0 / (k + 1);
                const double wk = gg.cn ? 2.0 : 1.0;
#pragma unroll
                for (int q = 0; q < RB; ++q) {
                    double ar = 0.0, ai = 0.0;
#pragma unroll
                    for (int w = 0; w < WT; ++w) {
                        const dcx x = vs[q * VS + base + hc[w]];
                        ar = fma(hv[w].re, x.re, fma(-hv[w].im, x.im, ar));
                        ai = fma(hv[w].re, x.im, fma(hv[w].im, x.re, ai));
                    }
                    tr[q].re = ai * rk;
                    tr[q].im = -ar * rk;
                    acc[q].re = fma(wk, tr[q].re, acc[q].re);
                    acc[q].im = fma(wk, tr[q].im, acc[q].im);
                }
                __syncthreads();
            }
        }
        // U_j = e^{i ph} (I + acc), so D_j = (e^{i ph} - 1) I + e^{i ph} acc, with
        // e^{i ph} - 1 = -2 sin^2(ph/2) + i sin(ph) formed without cancellation
        const double ph = -gg.tau * gg.shift;
        const double sh2 = sin(0.5 * ph);
        const double em1r = -2.0 * sh2 * sh2, em1i = sin(ph);
        const double cp = 1.0 + em1r, sp = em1i;
        if (rb < nrb) {
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int r = r0 + q;
                if (r >= dp) break;
                const long long o = (long long)j * plane * 2 + (long long)r * dp + c;
                double xr = 0.0, xi = 0.0;         // padded block: D = 0 (identity in U)
                if (r < d && c < d) {
                    xr = cp * acc[q].re - sp * acc[q].im;
                    xi = cp * acc[q].im + sp * acc[q].re;
                    if (r == c) {
                        xr += em1r;
                        xi += em1i;
                    }
                }
                // stored as D_j = U_j - I: at small tau U_j is close to I, and rounding I + delta
                // to FP32 would make the same error at every step of a slice
                U[o] = (R)xr;
                U[o + plane] = (R)xi;
            }
        }
    }
    if (!gg.cn && t == 0 && blockIdx.y == 0) {   // the gradient's Krylov order at this step
        double rem;
        const int mj = grad_order<R>(gg, j, MMAX_G + 1, rem);
        // most steps need the same order: update only when it is above the value seen so far
        if (mj > __hip_atomic_load(kmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(kmax, mj);
    }
}

__global__ void k_gate_set_int(int* v, int x) { *v = x; }

// Identity outside the leading 32 x 32 block of each of the K planar 64 x 64 matrices P_j.
template <typename R>
__global__ void k_gate_pad_identity(R* P, long long K) {
    constexpr long long plane = (long long)GT * GT;
    const long long total = K * 2 * plane;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long x = e % (2 * plane);
        const int pl = (int)(x / plane), r = (int)((x % plane) / GT), c = (int)(x % GT);
        if (r < 32 && c < 32) continue;
        P[e] = (pl == 0 && r == c) ? R(1) : R(0);
    }
}

// Chunked assembly scan (d <= 64).  The prefix products of a slice form a scan over its
// steps; run as one chain it keeps one workgroup busy per slice.  The steps are cut into
// chunks of consecutive steps inside the slices, and
//  1. k_gate_chain runs every chunk from the identity (one workgroup per chunk), giving
//     the local prefixes Q_j = U_j ... U_{first step of the chunk};
//  2. k_gate_carry (one workgroup per slice) turns the last local prefix of each chunk into
//     the true prefix, chunk after chunk: P_e(c) = Q_e(c) P_e(c-1) (e(c) the last step of
//     chunk c; the first chunk of a slice already holds true prefixes);
//  3. k_gate_apply (one workgroup per chunk after the first of a slice) multiplies the
//     other local prefixes by the true prefix that ends the previous chunk:
//     P_j = Q_j P_e(c-1).
// The dependent chain shrinks from the slice length L to about 2 Lc + L / Lc products.
// Local prefixes are kept as E_j = Q_j - I (a chunk's Q_j stays close to I, and rounding
// I + small to the path's precision at every step would lose the small part); steps 2 and 3
// form P = B + E B, each rounding like one addition.
// BS is the block formed: the leading 32 x 32 block (d <= 32, the rest of each P_j is the
// identity) or the whole 64 x 64 matrix.  Blocks live in LDS as A^T (left factor) and
// row-major (right factor), rows padded to BS + 1.
template <int BS>
__device__ __forceinline__ long long blk_gidx(int e) {
    constexpr long long plane = (long long)GT * GT;
    return (long long)(e / (BS * BS)) * plane + ((e / BS) % BS) * GT + (e % BS);
}

template <typename R, int BS>
static size_t gate_scan_shmem() {
    return (size_t)4 * BS * (BS + 1) * sizeof(R);
}

// C = A B for the two BS x BS blocks in LDS (At[p][k][i] = A[i][k], Bs[p][k][c] = B[k][c]);
// each wavefront owns a (BS/2) x (BS/2) quarter of C as (BS/32)^2 16 x 16 MFMA tiles.
template <typename R, int BS>
__device__ __forceinline__ void blk_mm(const R* At, const R* Bs, typename Acc<R>::T (&cr)[BS / 32][BS / 32],
                                       typename Acc<R>::T (&ci)[BS / 32][BS / 32]) {
    constexpr int LD = BS + 1, PL = BS * LD, NT = BS / 32;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * (BS / 2), wc = (w & 1) * (BS / 2);
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) cr[a][b][v] = ci[a][b][v] = 0;
#pragma unroll 4
    for (int kk = 0; kk < BS; kk += 4) {
        const int kr = kk + (lane >> 4), li = lane & 15;
        R ar[NT], ai[NT], br[NT], bi[NT];
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            ar[a] = At[kr * LD + wr + a * 16 + li];
            ai[a] = At[PL + kr * LD + wr + a * 16 + li];
        }
#pragma unroll
        for (int b = 0; b < NT; ++b) {
            br[b] = Bs[kr * LD + wc + b * 16 + li];
            bi[b] = Bs[PL + kr * LD + wc + b * 16 + li];
        }
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                cr[a][b] = mfma16(ar[a], br[b], cr[a][b]);
                cr[a][b] = mfma16(-ai[a], bi[b], cr[a][b]);
                ci[a][b] = mfma16(ar[a], bi[b], ci[a][b]);
                ci[a][b] = mfma16(ai[a], br[b], ci[a][b]);
            }
    }
}

// Row and column of accumulator element v of tile (a, b) of this lane's wavefront.
template <typename R, int BS>
__device__ __forceinline__ void blk_rc(int a, int b, int v, int& i, int& c) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    i = (w >> 1) * (BS / 2) + a * 16 + (sizeof(R) == 8 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
    c = (w & 1) * (BS / 2) + b * 16 + (lane & 15);
}

// Step 1 of the scan, blockIdx.x = chunk c (steps cb[c] .. cb[c+1]-1):
// E_first = D_first, E_j = E_{j-1} + (D_j + D_j E_{j-1}) with D_j = U_j - I.  The sum is
// compensated (Kahan) by the lane that owns the entry: the increments of neighbouring steps
// are alike, so their roundings would otherwise add up instead of cancelling.  E_{j-1} stays
// in LDS and D_{j+1} is fetched while step j runs on MFMA.  The first chunk of a slice
// stores I + E_j (true prefixes), the others E_j.
template <typename R, int BS>
__global__ __launch_bounds__(256) void k_gate_chain(const R* D, R* P, const int* cb, const int* s, int N) {
    extern __shared__ unsigned char smem_raw[];
    constexpr int LD = BS + 1, PL = BS * LD, NT = BS / 32, PER = 2 * BS * BS / 256;
    constexpr long long mat = 2LL * GT * GT;
    R* Dt = reinterpret_cast<R*>(smem_raw);   // Dt[p][k][i] = D_j[i][k]
    R* Es = Dt + 2 * PL;                       // Es[p][k][c] = E_{j-1}[k][c]
    const int ch = blockIdx.x, j0 = cb[ch], j1 = cb[ch + 1], t = threadIdx.x;
    int lo = 0, hi = N;                        // the chunk is the first of its slice when
    while (hi - lo > 1) {                      // it starts at a slice start
        const int mid = (lo + hi) >> 1;
        if (s[mid] <= j0) lo = mid; else hi = mid;
    }
    const R one = s[lo] == j0 ? R(1) : R(0);
    R pre[PER];
    {
        const R* src = D + (long long)j0 * mat;
#pragma unroll
        for (int q = 0; q < PER; ++q) pre[q] = src[blk_gidx<BS>(t + 256 * q)];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = t + 256 * q, p = e / (BS * BS), r = (e / BS) % BS, c = e % BS;
        Es[p * PL + r * LD + c] = pre[q];
        P[(long long)j0 * mat + blk_gidx<BS>(e)] = pre[q] + ((p == 0 && r == c) ? one : R(0));
    }
    if (j0 + 1 < j1) {
        const R* src = D + (long long)(j0 + 1) * mat;
#pragma unroll
        for (int q = 0; q < PER; ++q) pre[q] = src[blk_gidx<BS>(t + 256 * q)];
    }
    R kr[NT][NT][4], ki[NT][NT][4];           // compensation of the owned entries
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) kr[a][b][v] = ki[a][b][v] = 0;
    lds_barrier();
    for (int j = j0 + 1; j < j1; ++j) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q, p = e / (BS * BS), r = (e / BS) % BS, c = e % BS;
            Dt[p * PL + c * LD + r] = pre[q];
        }
        lds_barrier();                  // D_j complete in LDS
        if (j + 1 < j1) {
            const R* src = D + (long long)(j + 1) * mat;
#pragma unroll
            for (int q = 0; q < PER; ++q) pre[q] = src[blk_gidx<BS>(t + 256 * q)];
        }
        typename Acc<R>::T cr[NT][NT], ci[NT][NT];
        blk_mm<R, BS>(Dt, Es, cr, ci);
        lds_barrier();                  // every wavefront is done with Es
        R* dst = P + (long long)j * mat;
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int i, c;
                    blk_rc<R, BS>(a, b, v, i, c);
                    const int o = i * LD + c;
                    const R yr = (cr[a][b][v] + Dt[c * LD + i]) - kr[a][b][v];
                    const R yi = (ci[a][b][v] + Dt[PL + c * LD + i]) - ki[a][b][v];
                    const R er = Es[o], ei = Es[PL + o];
                    const R tr = er + yr, ti = ei + yi;
                    kr[a][b][v] = (tr - er) - yr;
                    ki[a][b][v] = (ti - ei) - yi;
                    Es[o] = tr;
                    Es[PL + o] = ti;
                    dst[i * GT + c] = tr + (i == c ? one : R(0));
                    dst[GT * GT + i * GT + c] = ti;
                }
        lds_barrier();                  // E_j complete in LDS, Dt free for the next step
    }
}

// Step 2 of the scan, blockIdx.x = slice n: chunks cfirst[n] .. cfirst[n+1]-1 with step
// bounds cb (chunk c covers steps cb[c] .. cb[c+1]-1); P_e(c) = P_e(c-1) + E_e(c) P_e(c-1).
template <typename R, int BS>
__global__ __launch_bounds__(256) void k_gate_carry(R* P, const int* cb, const int* cfirst) {
    extern __shared__ unsigned char smem_raw[];
    constexpr int LD = BS + 1, PL = BS * LD, NT = BS / 32, PER = 2 * BS * BS / 256;
    constexpr long long mat = 2LL * GT * GT;
    R* At = reinterpret_cast<R*>(smem_raw);
    R* Bs = At + 2 * PL;
    const int n = blockIdx.x, c0 = cfirst[n], c1 = cfirst[n + 1];
    if (c1 - c0 < 2) return;
    const int t = threadIdx.x;
    R pre[PER];
    {
        const R* src = P + (long long)(cb[c0 + 1] - 1) * mat;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q, p = e / (BS * BS), r = (e / BS) % BS, c = e % BS;
            Bs[p * PL + r * LD + c] = src[blk_gidx<BS>(e)];
        }
        const R* nxt = P + (long long)(cb[c0 + 2] - 1) * mat;
#pragma unroll
        for (int q = 0; q < PER; ++q) pre[q] = nxt[blk_gidx<BS>(t + 256 * q)];
    }
    for (int ch = c0 + 1; ch < c1; ++ch) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q, p = e / (BS * BS), r = (e / BS) % BS, c = e % BS;
            At[p * PL + c * LD + r] = pre[q];
        }
        lds_barrier();                  // A and B complete in LDS
        if (ch + 1 < c1) {
            const R* nxt = P + (long long)(cb[ch + 2] - 1) * mat;
#pragma unroll
            for (int q = 0; q < PER; ++q) pre[q] = nxt[blk_gidx<BS>(t + 256 * q)];
        }
        typename Acc<R>::T cr[NT][NT], ci[NT][NT];
        blk_mm<R, BS>(At, Bs, cr, ci);
        lds_barrier();                  // every wavefront is done with At and Bs
        R* dst = P + (long long)(cb[ch + 1] - 1) * mat;
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int i, c;
                    blk_rc<R, BS>(a, b, v, i, c);
                    const R nr = cr[a][b][v] + Bs[i * LD + c];
                    const R ni = ci[a][b][v] + Bs[PL + i * LD + c];
                    Bs[i * LD + c] = nr;
                    Bs[PL + i * LD + c] = ni;
                    dst[i * GT + c] = nr;
                    dst[GT * GT + i * GT + c] = ni;
                }
    }
}

// Step 3 of the scan, blockIdx.x = entry of capply: a chunk c that is not the first of its
// slice.  Its last product was made true by step 2; the others become
// P_{cb[c]-1} + E_j P_{cb[c]-1}.
template <typename R, int BS>
__global__ __launch_bounds__(256) void k_gate_apply(R* P, const int* cb, const int* capply) {
    extern __shared__ unsigned char smem_raw[];
    constexpr int LD = BS + 1, PL = BS * LD, NT = BS / 32, PER = 2 * BS * BS / 256;
    constexpr long long mat = 2LL * GT * GT;
    R* At = reinterpret_cast<R*>(smem_raw);
    R* Bs = At + 2 * PL;
    const int ch = capply[blockIdx.x];
    const int j0 = cb[ch], j1 = cb[ch + 1] - 1;
    if (j0 >= j1) return;
    const int t = threadIdx.x;
    R pre[PER];
    {
        const R* src = P + (long long)(j0 - 1) * mat;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q, p = e / (BS * BS), r = (e / BS) % BS, c = e % BS;
            Bs[p * PL + r * LD + c] = src[blk_gidx<BS>(e)];
        }
        const R* nxt = P + (long long)j0 * mat;
#pragma unroll
        for (int q = 0; q < PER; ++q) pre[q] = nxt[blk_gidx<BS>(t + 256 * q)];
    }
    for (int j = j0; j < j1; ++j) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q, p = e / (BS * BS), r = (e / BS) % BS, c = e % BS;
            At[p * PL + c * LD + r] = pre[q];
        }
        lds_barrier();                  // Q_j complete in LDS
        if (j + 1 < j1) {
            const R* nxt = P + (long long)(j + 1) * mat;
#pragma unroll
            for (int q = 0; q < PER; ++q) pre[q] = nxt[blk_gidx<BS>(t + 256 * q)];
        }
        typename Acc<R>::T cr[NT][NT], ci[NT][NT];
        blk_mm<R, BS>(At, Bs, cr, ci);
        R* dst = P + (long long)j * mat;
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int i, c;
                    blk_rc<R, BS>(a, b, v, i, c);
                    dst[i * GT + c] = cr[a][b][v] + Bs[i * LD + c];
                    dst[GT * GT + i * GT + c] = ci[a][b][v] + Bs[PL + i * LD + c];
                }
        lds_barrier();                  // every wavefront is done with At
    }
}

// Slice products for d <= 32, blockIdx.x = step j: [X_j | Y_j] = P_{j-1} [phi_n | B_n] on
// the leading 32 x 32 blocks only (P_{j-1}, phi_n and B_n are block diagonal in the padded
// layout and the gradient reads no other entry), written as [X_j | Y_j]^+ (2dp x dp planar,
// dp = 64).  The first step of a slice is left to k_gate_rhs_adj.
template <typename R>
__global__ __launch_bounds__(256) void k_gate_xy32(const R* RHS, const R* P, R* XY, const int* s, int N) {
    constexpr int BS = 32, LD = BS + 1, PL = BS * LD, PER = 2 * BS * BS / 256;
    constexpr long long plane = (long long)GT * GT, mat = 2 * plane;
    constexpr long long rplane = 2 * plane, rmat = 2 * rplane;   // dp x 2dp and 2dp x dp
    __shared__ R At[2 * PL], Bx[2 * PL], By[2 * PL];
    const int j = blockIdx.x, t = threadIdx.x;
    int lo = 0, hi = N;                   // slice n: s[n] <= j < s[n+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s[mid] <= j) lo = mid; else hi = mid;
    }
    const int n = lo;
    if (j == s[n]) return;
    const R* Pm = P + (long long)(j - 1) * mat;
    const R* Rn = RHS + (long long)n * rmat;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = t + 256 * q, p = e / (BS * BS), r = (e / BS) % BS, c = e % BS;
        At[p * PL + c * LD + r] = Pm[p * plane + r * GT + c];
        Bx[p * PL + r * LD + c] = Rn[p * rplane + r * 2 * GT + c];
        By[p * PL + r * LD + c] = Rn[p * rplane + r * 2 * GT + GT + c];
    }
    __syncthreads();
    typename Acc<R>::T xr[1][1], xi[1][1], yr[1][1], yi[1][1];
    blk_mm<R, BS>(At, Bx, xr, xi);
    blk_mm<R, BS>(At, By, yr, yi);
    R* out = XY + (long long)j * rmat;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        int i, c;
        blk_rc<R, BS>(0, 0, v, i, c);
        // row c of X^+ holds conj(X[i][c]) at column i; Y^+ starts at row dp
        out[(long long)c * GT + i] = xr[0][0][v];
        out[rplane + (long long)c * GT + i] = -xi[0][0][v];
        out[(long long)(GT + c) * GT + i] = yr[0][0][v];
        out[rplane + (long long)(GT + c) * GT + i] = -yi[0][0][v];
    }
}

// FP64 boundaries of density matrices for d <= 32, in one launch: workgroup 0 runs
// Psi_{n+1} = W_n Psi_n W_n^+ for n = 0..N-1, workgroup 1 runs Lambda_n = W_n^+ Lambda_{n+1} W_n
// for n = N-1..0 (PL = [Psi_0..Psi_N | Lambda_0..Lambda_N], W_n = M64 slot n).  The states are
// zero outside their leading 32 x 32 block and the W_n the identity there, so the products
// are formed on the blocks and every slot is written whole.  W for the next step is fetched
// while the current sandwich runs on MFMA; the threads share data through LDS only.
__global__ __launch_bounds__(256) void k_gate_dchain32(const double* M64, double* PL, int N) {
    constexpr int BS = 32, LD = BS + 1, BP = BS * LD, PER = 2 * BS * BS / 256;
    constexpr long long plane = (long long)GT * GT, mat = 2 * plane;
    __shared__ double At[2 * BP], Bs[2 * BP], Ws[2 * BP];
    const bool fwd = blockIdx.x == 0;
    const int t = threadIdx.x;
    const long long lam0 = (long long)(N + 1) * mat;
    {
        const double* S0 = PL + (fwd ? 0 : lam0 + (long long)N * mat);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q, p = e / (BS * BS), r = (e / BS) % BS, c = e % BS;
            Bs[p * BP + r * LD + c] = S0[blk_gidx<BS>(e)];
        }
    }
    double pre[PER];
    auto fetch = [&](int n) {
        const double* W = M64 + (long long)n * mat;
#pragma unroll
        for (int q = 0; q < PER; ++q) pre[q] = W[blk_gidx<BS>(t + 256 * q)];
    };
    fetch(fwd ? 0 : N - 1);
    for (int it = 0; it < N; ++it) {
        const int n = fwd ? it : N - 1 - it;
        // W_n row-major into Ws; the first product's left factor into At (At[k][i] = A[i][k]):
        // A = W_n (forward) or W_n^+ (backward)
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q, p = e / (BS * BS), r = (e / BS) % BS, c = e % BS;
            const double v = pre[q];                       // W_n[r][c], plane p
            Ws[p * BP + r * LD + c] = v;
            if (fwd) At[p * BP + c * LD + r] = v;
            else At[p * BP + r * LD + c] = p ? -v : v;
        }
        lds_barrier();                                     // W_n, At and the state in LDS
        if (it + 1 < N) fetch(fwd ? it + 1 : N - 2 - it);
        Acc<double>::T cr[1][1], ci[1][1];
        blk_mm<double, BS>(At, Bs, cr, ci);                // T = A S
        lds_barrier();                                     // every wavefront is done with At, Bs
        // second product S' = T B2, B2 = W_n^+ (forward) or W_n (backward)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int i, c;
            blk_rc<double, BS>(0, 0, v, i, c);
            At[c * LD + i] = cr[0][0][v];
            At[BP + c * LD + i] = ci[0][0][v];
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + 256 * q, p = e / (BS * BS), r = (e / BS) % BS, c = e % BS;
            double v = fwd ? Ws[p * BP + c * LD + r] : Ws[p * BP + r * LD + c];
            if (fwd && p) v = -v;
            Bs[p * BP + r * LD + c] = v;
        }
        lds_barrier();                                     // T and B2 in LDS
        blk_mm<double, BS>(At, Bs, cr, ci);
        lds_barrier();                                     // every wavefront is done with At, Bs
        double* dst = PL + (fwd ? (long long)(n + 1) * mat : lam0 + (long long)n * mat);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int i, c;
            blk_rc<double, BS>(0, 0, v, i, c);
            Bs[i * LD + c] = cr[0][0][v];
            Bs[BP + i * LD + c] = ci[0][0][v];
            dst[i * GT + c] = cr[0][0][v];
            dst[plane + i * GT + c] = ci[0][0][v];
        }
        for (int e = t; e < (int)mat; e += 256) {          // zero outside the leading block
            const int rc = e % (int)plane, r = rc / GT, c = rc % GT;
            if (r >= BS || c >= BS) dst[e] = 0.0;
        }
        lds_barrier();                                     // the new state complete in Bs
    }
}

// First step of every slice (blockIdx.y = n): [X | Y]^+ at step s_n is RHS_n^+ (RHS_n is
// dp x 2dp planar, the output 2dp x dp planar).
template <typename R>
__global__ void k_gate_rhs_adj(const R* RHS, R* XY, const int* s, int dp) {
    const long long rplane = 2LL * dp * dp;
    const R* src = RHS + (long long)blockIdx.y * 2 * rplane;
    R* dst = XY + (long long)s[blockIdx.y] * 2 * rplane;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < rplane;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / dp), c = (int)(e % dp);     // output row i < 2dp, column c < dp
        const long long o = (long long)c * 2 * dp + i;       // RHS_n[c][i]
        dst[e] = src[o];
        dst[e + rplane] = -src[o + rplane];
    }
}

// First propagator of every slice: P_{s_n} = I + D_{s_n} (blockIdx.y = n).
template <typename R>
__global__ void k_gate_first(const R* D, R* P, const int* s, int dp) {
    const long long plane = (long long)dp * dp;
    const long long base = (long long)s[blockIdx.y] * 2 * plane;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < 2 * plane;
         e += (long long)gridDim.x * blockDim.x) {
        R v = D[base + e];
        if (e < plane && e / dp == e % dp) v += R(1);
        P[base + e] = v;
    }
}

// w_ab = i^{a+b} (-1)^b / ((a+b+1) a! b!) as a real magnitude; the phase i^{a+b}(-1)^b is
// applied in the kernel.
struct WabTable {
    double v[MMAX_G + 1][MMAX_G + 1];
};
// |w_ab| = 1 / ((a+b+1) a! b!), evaluated by the compiler so that the unrolled series
// take the weights as instruction constants
constexpr WabTable make_wab() {
    WabTable t{};
    double f[2 * MMAX_G + 2] = {};
    f[0] = 1.0;
    for (int i = 1; i < 2 * MMAX_G + 2; ++i) f[i] = f[i - 1] * i;
    for (int a = 0; a <= MMAX_G; ++a)
        for (int b = 0; a + b <= MMAX_G; ++b) t.v[a][b] = 1.0 / ((a + b + 1) * f[a] * f[b]);
    return t;
}
__device__ constexpr WabTable kWab = make_wab();

// Per (step, block of CBW columns): partial sums over rows and columns of
// Im <y_k| Hhat_c |x_k> for every control c, in FP64.  MK bounds the Krylov order.
// Thread t works on row r = t mod lpc of column group t / lpc: lpc = dp (one column at a
// time) unless d <= 32, where lpc is the least power of two >= d and a workgroup of dp = 64
// threads takes 64 / lpc columns at once (rows d..dp-1 of the padded layout are never
// worked on).  Slot t of every LDS vector belongs to thread t.
//
// With Hhat_c = sum_{a,b} w_ab (i tau H')^a H_c (-i tau H')^b / tau^0 (the series of the step
// average, H' = H_j - s), <y|Hhat_c|x> = sum_b <t_b| H_c r_b> with p_a = (tau H')^a y,
// r_b = (tau H')^b x and t_b = sum_a conj(w_ab) p_a.  Two Krylov phases per column, each
// through one double-buffered LDS vector (one barrier per Krylov step):
//   (1) p_a, a = 0..m, folded into the t_b (registers) as they are produced;
//   (2) r_b, b = 0..m: the gathers that form r_{b+1} read r_b at every column w of this
//       row's union pattern, which is where the controls' entries lie; they are folded into
//       S_w = sum_b conj(t_b) r_b(col_w) at once.
// Then Im <t|H_c r> over this row is Im sum h_{c,w} S_w over the control's entries of the
// row (wq, wv list them per position of the union pattern).  Neither phase keeps a Krylov
// sequence in LDS.
//
// A step whose series, cut at MK terms, leaves a remainder bound above 1e-13 (FP64) or 1e-7
// (FP32) sets bit 1 of flags[0] (reported as unsupported, never truncated silently):
// 2 tau ||H_j - s||_inf above 1.46 in FP64 or 2.0 in FP32.
// Two bounds MK are launched: the one with MK = mks runs when every step's order is at
// most mks (kmax, from the step build at the same controls; then the order of every step is
// the same as with the larger bound, and so is the result), the other one otherwise.  The
// smaller bound holds fewer registers.  Two wavefronts per SIMD, except FP64 at d <= 64:
// at d = 256 three FP64 wavefronts (168 registers) spilled and took 18.0 ms against 12.5;
// at d = 32, whose workgroups are one wavefront, the third wavefront hides more latency
// than its spill costs (1.91 against 2.06 ms for the five-spin density gradient).
template <typename R, int MK, int WT, int VS, int NC>
__global__ __launch_bounds__(256, sizeof(R) == 8 && VS == 64 ? 3 : 2) void k_gate_grad(GateGen gg, const R* XY, long long xy_plane,
                                                   double* gpart, int ncb, int* flags,
                                                   const int* kmax, int mks) {
    if ((*kmax <= mks) != (MK == mks)) return;      // the other bound's launch does this work
    // LDS: per-row gradient accumulators of every control (FP64, thread t's slots only) and,
    // for each of the NC columns a thread works on at once, a Krylov double buffer (2 x re/im
    // planes), at a compile-time plane stride VS >= dp so that every gather of a row needs
    // one address and immediate offsets
    extern __shared__ unsigned char smem_raw[];
    double* gacc = reinterpret_cast<double*>(smem_raw);          // C VS
    R* vb = reinterpret_cast<R*>(gacc + (size_t)gg.C * VS);     // 4 NC VS
    __shared__ double red[4][CMAX_G];
    const int j = blockIdx.x, cb = blockIdx.y, t = threadIdx.x;
    const int d = gg.d, dp = gg.dp;
    int lpc = dp;
    if (d <= 32) {
        lpc = 1;
        while (lpc < d) lpc <<= 1;
    }
    // lpc is dp (a multiple of 64, not always a power of two) or a power of two up to 32
    const int r = t % lpc, base = t - r, grp = t / lpc, ngrp = dp / lpc;
    const double* uj = gg.u + (size_t)j * gg.C;
    int m;
    {
        double rem;
        m = grad_order<R>(gg, j, MK, rem);
        if (rem > (sizeof(R) == 8 ? 1e-13 : 1e-7) && t == 0 && cb == 0) atomicOr(flags, 2);
    }
    // row r of tau (H_j - s) on the union pattern
    R hvr[WT], hvi[WT];
    int hcol[WT];
#pragma unroll
    for (int w = 0; w < WT; ++w) {
        double hr = 0.0, hi = 0.0;
        int cc = r;
        if (r < d && w < gg.W) {
            const size_t idx = (size_t)r * gg.W + w;
            hr = gg.h0v[idx].re;
            hi = gg.h0v[idx].im;
            for (int q = 0; q < gg.C; ++q) {
                const dcx x = gg.hcu[(size_t)q * d * gg.W + idx];
                hr += uj[q] * x.re;
                hi += uj[q] * x.im;
            }
            cc = gg.col[idx];
        }
        hvr[w] = (R)(gg.tau * hr);
        hvi[w] = (R)(gg.tau * hi);
        hcol[w] = cc;
    }
    for (int q = 0; q < gg.C; ++q) gacc[q * VS + t] = 0.0;     // own slots only
    // Krylov buffer `buf` (0/1) of column slot `c`, 2 VS reals.  FP32 keeps (re, im) of a
    // slot side by side, so that a gather is one 8-byte LDS read; FP64 keeps two planes
    // (16-byte reads at the gathered slots run slower than two 8-byte ones).
    constexpr bool kIl = sizeof(R) == 4;
    auto vbp = [&](int c, int buf) { return vb + (c * 2 + buf) * 2 * VS; };
    auto ld = [&](const R* p, int i) {
        if constexpr (kIl) return reinterpret_cast<const Cx<R>*>(p)[i];
        else return Cx<R>{p[i], p[VS + i]};
    };
    auto st = [&](R* p, int i, R re, R im) {
        if constexpr (kIl) {
            reinterpret_cast<Cx<R>*>(p)[i] = Cx<R>{re, im};
        } else {
            p[i] = re;
            p[VS + i] = im;
        }
    };
    // S_w of this row, summed over every column the thread works on (only the sum enters
    // the gradient, and a dead column adds exact zeros); contracted with the controls once,
    // after the last column
    R swr[WT], swi[WT];
#pragma unroll
    for (int w = 0; w < WT; ++w) swr[w] = swi[w] = 0;
    for (int kk = 0; kk < CBW; kk += ngrp * NC) {
        if (cb * CBW + kk >= d) break;        // uniform over the workgroup
        // columns k_c of X_j (x) and Y_j (y) for this thread's group, c < NC
        // stored as [X_j | Y_j]^+: column k of X_j is row k, conjugated; of Y_j row dp + k
        R xr[NC], xi[NC], yr[NC], yi[NC];
        bool live[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int kc = kk + c * ngrp + grp;
            const int k = cb * CBW + kc;
            live[c] = r < d && k < d && kc < CBW;
            const long long ox = (long long)j * xy_plane * 2 + (long long)k * dp + r;
            const long long oy = ox + (long long)dp * dp;
            xr[c] = live[c] ? XY[ox] : R(0);
            xi[c] = live[c] ? -XY[ox + xy_plane] : R(0);
            yr[c] = live[c] ? XY[oy] : R(0);
            yi[c] = live[c] ? -XY[oy + xy_plane] : R(0);
        }
        // phase 1: p_a = (tau H')^a y; t_b += conj(w_ab) p_a, conj(w_ab) = (-i)^{a+b} (-1)^b |w_ab|
        R ttr[NC][MK + 1], tti[NC][MK + 1];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int b = 0; b <= MK; ++b) ttr[c][b] = tti[c][b] = 0;
        __syncthreads();                      // the previous columns' readers of vb are done
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            st(vbp(c, 0), t, yr[c], yi[c]);
        }
#pragma unroll
        for (int a = 0; a <= MK; ++a) {
            if (a <= m) {                     // m is uniform over the workgroup
                if (a > 0) {
                    __syncthreads();          // p_{a-1} is in buffer (a-1) & 1
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const R* ys = vbp(c, (a - 1) & 1);
                        R nyr = 0, nyi = 0;
#pragma unroll
                        for (int w = 0; w < WT; ++w) {
                            const int cc = hcol[w];
                            const Cx<R> v = ld(ys, base + cc);
                            const R vr = v.re, vi = v.im;
                            nyr = fma(hvr[w], vr, fma(-hvi[w], vi, nyr));
                            nyi = fma(hvr[w], vi, fma(hvi[w], vr, nyi));
                        }
                        if (a < m) {          // p_m is read by nobody
                            st(vbp(c, a & 1), t, nyr, nyi);
                        }
                        yr[c] = nyr;
                        yi[c] = nyi;
                    }
                }
#pragma unroll
                for (int b = 0; b + a <= MK; ++b) {
                    if (a + b <= m) {
                        R wr = (R)kWab.v[a][b];
                        if (b & 1) wr = -wr;
                        const int ph = (a + b) & 3;
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            const R qr = ph == 0 ? yr[c] : ph == 1 ? yi[c] : ph == 2 ? -yr[c] : -yi[c];
                            const R qi = ph == 0 ? yi[c] : ph == 1 ? -yr[c] : ph == 2 ? -yi[c] : yr[c];
                            ttr[c][b] = fma(wr, qr, ttr[c][b]);
                            tti[c][b] = fma(wr, qi, tti[c][b]);
                        }
                    }
                }
            }
        }
        // phase 2: r_b = (tau H')^b x; S_w += conj(t_b) r_b(col_w)
        __syncthreads();                      // phase 1's readers of vb are done
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            st(vbp(c, 0), t, xr[c], xi[c]);
        }
#pragma unroll
        for (int b = 0; b <= MK; ++b) {
            if (b <= m) {
                __syncthreads();              // r_b is in buffer b & 1
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const R* xs = vbp(c, b & 1);
                    const R cr = ttr[c][b], ci = tti[c][b];
                    R nxr = 0, nxi = 0;
#pragma unroll
                    for (int w = 0; w < WT; ++w) {
                        const int cc = hcol[w];
                        const Cx<R> v = ld(xs, base + cc);
                        const R ur = v.re, ui = v.im;
                        swr[w] = fma(cr, ur, fma(ci, ui, swr[w]));
                        swi[w] = fma(cr, ui, fma(-ci, ur, swi[w]));
                        nxr = fma(hvr[w], ur, fma(-hvi[w], ui, nxr));
                        nxi = fma(hvr[w], ui, fma(hvi[w], ur, nxi));
                    }
                    if (b < m) {
                        st(vbp(c, (b + 1) & 1), t, nxr, nxi);
                    }
                }
            }
        }
    }
    // per control: Im(h S_w) summed over the control's entries of this row, in FP64
#pragma unroll
    for (int w = 0; w < WT; ++w) {
        if (w < gg.W && r < d) {
            const double sr = swr[w], si = swi[w];
            const size_t e0 = ((size_t)r * gg.W + w) * gg.CW;
            for (int e = 0; e < gg.CW; ++e) {
                const int q = gg.wq[e0 + e];
                const dcx hv = gg.wv[e0 + e];
                gacc[q * VS + t] += hv.re * si + hv.im * sr;
            }
        }
    }
    // reduction over rows: wavefront tree, then the partials of the wavefronts in order
    const int wv = t >> 6, lane = t & 63;
    for (int q = 0; q < gg.C; ++q) {
        double v = gacc[q * VS + t];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    if (t < gg.C) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w][t];
        gpart[((size_t)j * ncb + cb) * gg.C + t] = s;
    }
}
// Crank-Nicolson gradient on the dense path (Sec. 3 with the reading of the discrete
// gradient): per step j and column k of X_j (x) and Y_j (y), Im <A y| H_c |A x> with
// A = (I + L_j)^{-1}, L_j = (i tau/2) H_j; with psi_j + psi_{j+1} = 2 A psi_j and
// chi_j = (I - L_j)^{-1} lambda_{j+1} = A lambda_j this is the exact gradient
// 1/2 Im <chi_j|H_c|psi_j + psi_{j+1}> (density matrices: 2 Im Tr((A Y)^+ H_c (A X)), the
// factor applied by k_gate_grad_finish).  A v = sum_a (-L)^a v is a Neumann series whose
// terms run through one double-buffered LDS vector (one barrier per term); the sum of y's
// stays in registers, the sum of x's goes to LDS once for the gathers of H_c.  Same layout,
// column blocking and partial sums as k_gate_grad.
template <typename R, int WT, int VS>
__global__ __launch_bounds__(256) void k_gate_grad_cn(GateGen gg, const R* XY, long long xy_plane,
                                                      double* gpart, int ncb, int* flags) {
    extern __shared__ unsigned char smem_raw[];
    double* gacc = reinterpret_cast<double*>(smem_raw);          // C VS
    R* vb = reinterpret_cast<R*>(gacc + (size_t)gg.C * VS);     // 6 VS: 2 buffers + the sum of x
    __shared__ double red[4][CMAX_G];
    const int j = blockIdx.x, cb = blockIdx.y, t = threadIdx.x;
    const int d = gg.d, dp = gg.dp;
    int lpc = dp;
    if (d <= 32) {
        lpc = 1;
        while (lpc < d) lpc <<= 1;
    }
    // lpc is dp (a multiple of 64, not always a power of two) or a power of two up to 32
    const int r = t % lpc, base = t - r, grp = t / lpc, ngrp = dp / lpc;
    const double* uj = gg.u + (size_t)j * gg.C;
    int nt;
    {
        double bound = gg.h0norm;
        for (int q = 0; q < gg.C; ++q) bound += fabs(uj[q]) * gg.cnorm[q];
        const double tol = sizeof(R) == 8 ? 1e-17 : fmin(1e-8, 1e-5 / (double)gg.K);
        nt = neumann_terms(0.5 * gg.tau * bound, tol, sizeof(R) == 8 ? 0.25 : 0.45);
        if (nt < 0) {
            if (t == 0 && cb == 0) atomicOr(flags, 2);
            nt = 1;
        }
    }
    // row r of (tau/2) H_j on the union pattern
    R hvr[WT], hvi[WT];
    int hcol[WT];
#pragma unroll
    for (int w = 0; w < WT; ++w) {
        double hr = 0.0, hi = 0.0;
        int cc = r;
        if (r < d && w < gg.W) {
            const size_t idx = (size_t)r * gg.W + w;
            hr = gg.h0v[idx].re;
            hi = gg.h0v[idx].im;
            for (int q = 0; q < gg.C; ++q) {
                const dcx x = gg.hcu[(size_t)q * d * gg.W + idx];
                hr += uj[q] * x.re;
                hi += uj[q] * x.im;
            }
            cc = gg.col[idx];
        }
        hvr[w] = (R)(0.5 * gg.tau * hr);
        hvi[w] = (R)(0.5 * gg.tau * hi);
        hcol[w] = cc;
    }
    for (int q = 0; q < gg.C; ++q) gacc[q * VS + t] = 0.0;     // own slots only
    // v <- A v = sum_a (-L)^a v through the double buffer; returns the sum
    auto neumann = [&](R vr, R vi, R& sr, R& si) {
        sr = vr;
        si = vi;
        vb[t] = vr;
        vb[VS + t] = vi;
        for (int a = 1; a <= nt; ++a) {          // nt is uniform over the workgroup
            __syncthreads();                     // term a-1 is in buffer (a-1) & 1
            const R* pr = vb + 2 * ((a - 1) & 1) * VS + base;
            R hr = 0, hi = 0;
#pragma unroll
            for (int w = 0; w < WT; ++w) {
                const int cc = hcol[w];
                const R xr = pr[cc], xi = pr[VS + cc];
                hr = fma(hvr[w], xr, fma(-hvi[w], xi, hr));
                hi = fma(hvr[w], xi, fma(hvi[w], xr, hi));
            }
            // -L v = -i (tau/2) H v
            const R nr = hi, ni = -hr;
            sr += nr;
            si += ni;
            if (a < nt) {
                vb[2 * (a & 1) * VS + t] = nr;
                vb[(2 * (a & 1) + 1) * VS + t] = ni;
            }
        }
    };
    // S_w = sum over the thread's columns of conj(A y)_r (A x)_{col_w}, in FP64, contracted
    // with the controls once after the last column
    double swr[WT], swi[WT];
#pragma unroll
    for (int w = 0; w < WT; ++w) swr[w] = swi[w] = 0.0;
    for (int kk = 0; kk < CBW; kk += ngrp) {
        if (cb * CBW + kk >= d) break;        // uniform over the workgroup
        const int k = cb * CBW + kk + grp;
        const bool live = r < d && k < d && kk + grp < CBW;
        const long long ox = (long long)j * xy_plane * 2 + (long long)k * dp + r;
        const long long oy = ox + (long long)dp * dp;
        const R xr = live ? XY[ox] : R(0), xi = live ? -XY[ox + xy_plane] : R(0);
        const R yr = live ? XY[oy] : R(0), yi = live ? -XY[oy + xy_plane] : R(0);
        R ayr, ayi, axr, axi;
        __syncthreads();                      // the previous column's readers of vb are done
        neumann(yr, yi, ayr, ayi);
        __syncthreads();                      // readers of the y terms are done
        neumann(xr, xi, axr, axi);
        vb[4 * VS + t] = axr;                 // A x, for the gathers of H_c
        vb[5 * VS + t] = axi;
        __syncthreads();
        if (live) {
            const R* ax = vb + 4 * VS + base;
#pragma unroll
            for (int w = 0; w < WT; ++w) {
                if (w < gg.W) {
                    const int cc = hcol[w];
                    const R ur = ax[cc], ui = ax[VS + cc];
                    swr[w] += (double)ayr * ur + (double)ayi * ui;
                    swi[w] += (double)ayr * ui - (double)ayi * ur;
                }
            }
        }
    }
    // per control: Im(h S_w) summed over the control's entries of this row
#pragma unroll
    for (int w = 0; w < WT; ++w) {
        if (w < gg.W && r < d) {
            const size_t e0 = ((size_t)r * gg.W + w) * gg.CW;
            for (int e = 0; e < gg.CW; ++e) {
                const int q = gg.wq[e0 + e];
                const dcx hv = gg.wv[e0 + e];
                gacc[q * VS + t] += hv.re * swi[w] + hv.im * swr[w];
            }
        }
    }
    const int wv = t >> 6, lane = t & 63;
    for (int q = 0; q < gg.C; ++q) {
        double v = gacc[q * VS + t];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    if (t < gg.C) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w][t];
        gpart[((size_t)j * ncb + cb) * gg.C + t] = s;
    }
}

// g_{j,c} = beta_n (1/d) sum_cb gpart - alpha_j u_{j,c}; update or write the gradient.
// gscale: 1/d for evolution operators (<A|B> = Tr(A^+ B)/d); 2 for density matrices, where
// Im Tr(Hhat [rho_j, lambda_j]) = 2 Im Tr(Y_j^+ Hhat X_j) with X_j = P_{j-1} phi_n and
// Y_j = P_{j-1} M_n^+ phi_{n+1} M_n.
__global__ void k_gate_grad_finish(const double* gpart, int ncb, int K, int N, int C,
                                   double gscale, const int* s, double* u, const double* alpha,
                                   double* grad, double rho, int update, const int* active) {
    if (active && active[0] == 0) update = 0;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= K * C) return;
    const int j = idx / C, c = idx - j * C;
    int lo = 0, hi = N;                         // slice of step j: s[n] <= j < s[n+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (s[mid] <= j) lo = mid;
        else hi = mid;
    }
    const double beta = (double)K / (double)(s[lo + 1] - s[lo]);
    double acc = 0.0;
    for (int cb = 0; cb < ncb; ++cb) acc += gpart[((size_t)j * ncb + cb) * C + c];
    const double uu = u[idx];
    const double g = beta * acc * gscale - (alpha ? alpha[j] : 0.0) * uu;
    if (grad) grad[idx] = g;
    if (update) u[idx] = fma(rho, g, uu);
}

// Slice propagators M_n = P_{s_{n+1}-1} to FP64, blockIdx.y = n.
template <typename R>
__global__ void k_slice_ends_f64(const R* P, double* M64, const int* s, long long mat) {
    const R* src = P + (long long)(s[blockIdx.y + 1] - 1) * mat;
    double* dst = M64 + (long long)blockIdx.y * mat;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < mat; i += stride)
        dst[i] = (double)src[i];
}

template <typename R>
__global__ void k_from_f64(const double* src, R* dst, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = (R)src[i];
}

// phi_n = (1 - w_n) Psi_n + w_n Lambda_n (planar FP64), w_n = s_n / K; and the right-hand
// operand [phi_n | .] of the slice sweeps (columns 0..dp-1 of RHS_n) in precision R.
template <typename R>
__global__ void k_gate_phi(const double* Psi, const double* Lam, double* phi, R* rhs, const int* s,
                           int N, int K, int dp, const double* psi0, const double* target) {
    const long long per = 2LL * dp * dp;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n_all = (long long)(N + 1) * per;
    for (; i < n_all; i += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(i / per);
        const long long e = i - n * per;
        const double w = (double)s[n] / (double)K;
        double f = (1.0 - w) * Psi[i] + w * Lam[i];
        if (n == 0) f = psi0[e];
        if (n == N) f = target[e];
        phi[i] = f;
        if (n < N) {
            const long long plane = (long long)dp * dp;
            const int p = (int)(e / plane);
            const long long rc = e - p * plane;
            const int rr = (int)(rc / dp), cc = (int)(rc - (long long)rr * dp);
            rhs[(long long)n * 2 * dp * 2 * dp + p * (long long)dp * 2 * dp + (long long)rr * 2 * dp + cc] = (R)f;
        }
    }
}

// z = js Tr(W^+ Psi_N): J = Re z - penalty, F = fs |z|^2 (one block).  Evolution operators:
// js = 1/d, fs = 1; density matrices: js = 1, fs = 1/(<rho_0|rho_0><rho_f|rho_f>).
__global__ void k_gate_fid(const double* PsiN, const double* W, int d, int dp, double js,
                           double fs, const double* u, const double* alpha, int K, int C,
                           double tau, double* J, double* F, double* Jhist, int* active,
                           double fid_stop, int* flags) {
    __shared__ double red[3][256];
    const int t = threadIdx.x;
    const long long plane = (long long)dp * dp;
    double zr = 0.0, zi = 0.0, pen = 0.0;
    for (long long e = t; e < (long long)d * dp; e += blockDim.x) {
        const int r = (int)(e / dp), c = (int)(e % dp);
        if (c >= d) continue;
        const long long o = (long long)r * dp + c;
        const double wr = W[o], wi = W[o + plane], pr = PsiN[o], pi = PsiN[o + plane];
        zr += wr * pr + wi * pi;
        zi += wr * pi - wi * pr;
    }
    if (alpha)
        for (int i = t; i < K * C; i += blockDim.x) pen += alpha[i / C] * u[i] * u[i];
    red[0][t] = zr;
    red[1][t] = zi;
    red[2][t] = pen;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int q = 0; q < 3; ++q) red[q][t] += red[q][t + w];
        __syncthreads();
    }
    if (t == 0) {
        const double a = red[0][0] * js, b = red[1][0] * js;
        const double Jv = a - 0.5 * tau * red[2][0];
        const double Fv = (a * a + b * b) * fs;
        J[0] = Jv;
        F[0] = Fv;
        if (Jhist) Jhist[0] = Jv;
        if (!(fabs(Jv) < 1e300)) atomicOr(&flags[0], 1);
        if (active) {
            if (active[0] && Fv >= fid_stop) active[0] = 0;
            if (active[0]) atomicAdd(&flags[1], 1);
        }
    }
}

// Planar FP64 matrix from interleaved complex d x d, zero padded to dp.
__global__ void k_planar_from_interleaved(const dcx* src, double* dst, int d, int dp) {
    const long long plane = (long long)dp * dp;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < plane;
         e += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(e / dp), c = (int)(e % dp);
        dcx v = {0.0, 0.0};
        if (r < d && c < d) v = src[(long long)r * d + c];
        dst[e] = v.re;
        dst[e + plane] = v.im;
    }
}

__global__ void k_interleaved_from_planar(const double* src, dcx* dst, int d, int dp) {
    const long long plane = (long long)dp * dp;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)d * d;
         e += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(e / d), c = (int)(e % d);
        const long long o = (long long)r * dp + c;
        dst[e].re = src[o];
        dst[e].im = src[o + plane];
    }
}

template <typename R>
__global__ void k_copy_identity_or(R* dst, const R* src, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (long long)gridDim.x * blockDim.x) dst[i] = src[i];
}

}  // namespace

#include "k_gate_host.inc"

}  // namespace ism
