// Gross-Pitaevskii path (Sec. 4.C): i d/dt psi = (-1/2 d_xx + V(x,u) + g|psi|^2) psi on a
// periodic grid of n = 64, 1024 or 4096 points, V(x,u) = V0(x) + u V1(x) + u^2 V2, one control.
//
// Step map: Strang splitting (Eq. (OS)) with exact kinetic half steps in Fourier space,
//   a_j = F^-1 Kh F psi_j,  b_j = e^{-i theta_j} a_j,  theta_j = tau (V(x,u_j) + g |a_j|^2),
//   psi_{j+1} = F^-1 Kh F b_j,  Kh = e^{-i tau k^2/4}.
// Inside a slice consecutive kinetic half steps are fused, a_{j+1} = F^-1 Kh^2 F b_j, so a
// step costs one forward and one inverse FFT; at a slice end psi_{j1} = F^-1 Kh F b is
// formed and the next slice restarts from it with a half step, exactly as a slice kernel
// that starts from the stored psi(t_n) does.
//
// Exact discrete adjoint (real inner product Re<.|.>), fused the same way:
//   nu'_j = F^-1 conj(Kh) F nu_{j+1};  g_j = dx sum_m dV/du Im(conj(nu'_j) b_j);
//   w = e^{+i theta_j} nu'_j;  mu_j = w + 2 tau g Im(conj(w) a_j) a_j;
//   nu_j = F^-1 conj(Kh) F mu_j  (inside a slice nu'_{j-1} = F^-1 conj(Kh)^2 F mu_j).
//
// ISM, BEC variant (Sec. 4.C): slice n starts from psi(t_n) on the forward trajectory and
// its adjoint ends on nu(t_{n+1}) of the adjoint trajectory; both boundary sequences come
// from one sequential forward and one sequential adjoint sweep (the map is nonlinear, so
// no slice propagator exists to assemble).  The slice gradient equals the plain gradient
// on the slice (weight 1).
//
// Data layout: a workgroup of T = n/P threads holds the state in registers, thread t
// owning the points t + T i, i = 0..P-1.  The FFT is a Stockham transform whose first pass
// reads its inputs from registers and whose last pass leaves its outputs in registers in the
// same ownership pattern, so the pointwise potential phase, the kinetic factors, the
// trajectory and the gradient terms are formed in registers and only the exchanges between
// passes go through LDS, as 16-byte complex slots.
//  * n = 4096: P = 8, 512 threads (two wavefronts per SIMD), radices 8, 8, 8, 8.  The
//    pass-3 twiddles and the kinetic factors at the owned frequencies stay in registers for
//    the whole launch, the pass-2 twiddles in an LDS table, and the pass-1 twiddles, uniform
//    over a wavefront, are applied by pass 0 from scalar registers; the three exchanges of a
//    transform alternate between two LDS buffers of 16-byte complex slots, so each needs
//    one barrier (a buffer is written again only after the barrier that follows its last
//    reads), and each exchange has its own padding, which makes all its accesses
//    bank-conflict free and each a per-thread base plus a compile-time offset.
//  * n = 1024 and 64: P = 4, 256 and 16 threads, radix-4 passes (5 and 3); twiddles and
//    kinetic factors in registers, the exchanges alternating between two LDS slot buffers,
//    again one barrier and one conflict-free padding per exchange.
// Butterflies, twiddles and the LDS state are FP64 in both precisions; the FP32 mixed path
// stores the trajectory a_j and forms the phase e^{-i theta} in FP32.
#include <math.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "ism_paths.h"

namespace ism {
namespace {

template <typename R> struct Cx { R re, im; };
using Cd = Cx<double>;

constexpr int kSlots8 = 4608;     // slots of an exchange buffer of the radix-8 engine

// points per thread and threads per workgroup of the FFT engine for grid size NN
template <int NN> struct Lay {
    static constexpr int P = NN == 4096 ? 8 : 4;
    static constexpr int T = NN / P;
};

// Workgroup barrier that orders LDS only: the FFT exchanges go through LDS alone, and a
// full barrier would also wait for the trajectory stores and read-ahead loads in flight.
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ Cd cmul(Cd a, Cd b) {
    return Cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ Cd cmulc(Cd a, Cd b) {      // a * conj(b)
    return Cd{a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// multiplication by a forward root (SIGN = -1) or by its conjugate (SIGN = +1)
template <int SIGN>
__device__ __forceinline__ Cd cmul_s(Cd a, Cd w) { return SIGN < 0 ? cmul(a, w) : cmulc(a, w); }

template <typename R>
__device__ __forceinline__ Cd up(Cx<R> v) { return Cd{(double)v.re, (double)v.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> down(Cd v) { return Cx<R>{(R)v.re, (R)v.im}; }

__device__ __forceinline__ void sincos_r(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_r(double x, double* s, double* c) { sincos(x, s, c); }

// 4-point DFT in place, roots e^{SIGN 2 pi i/4}
template <int SIGN>
__device__ __forceinline__ void dft4(Cd& a, Cd& b, Cd& c, Cd& d) {
    const Cd t0{a.re + c.re, a.im + c.im}, t1{a.re - c.re, a.im - c.im};
    const Cd t2{b.re + d.re, b.im + d.im};
    const Cd bd{b.re - d.re, b.im - d.im};
    const Cd t3 = SIGN < 0 ? Cd{bd.im, -bd.re} : Cd{-bd.im, bd.re};     // (b - d) * SIGN i
    a = Cd{t0.re + t2.re, t0.im + t2.im};
    b = Cd{t1.re + t3.re, t1.im + t3.im};
    c = Cd{t0.re - t2.re, t0.im - t2.im};
    d = Cd{t1.re - t3.re, t1.im - t3.im};
}

// 8-point DFT in place (x[c] <- sum_r x[r] e^{SIGN 2 pi i r c/8}): 4-point DFTs of the even
// and odd inputs, then x[c] = E_c + W^c O_c, x[c+4] = E_c - W^c O_c with W = e^{SIGN 2 pi i/8}
template <int SIGN>
__device__ __forceinline__ void dft8(Cd (&x)[8]) {
    dft4<SIGN>(x[0], x[2], x[4], x[6]);           // E_0..E_3
    dft4<SIGN>(x[1], x[3], x[5], x[7]);           // O_0..O_3
    constexpr double h = 0.70710678118654752440;  // cos(pi/4)
    const Cd o0 = x[1];
    const Cd o1{h * (x[3].re - SIGN * x[3].im), h * (x[3].im + SIGN * x[3].re)};
    const Cd o2{-SIGN * x[5].im, SIGN * x[5].re};
    const Cd o3{h * (-x[7].re - SIGN * x[7].im), h * (-x[7].im + SIGN * x[7].re)};
    const Cd e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
    x[0] = Cd{e0.re + o0.re, e0.im + o0.im};
    x[4] = Cd{e0.re - o0.re, e0.im - o0.im};
    x[1] = Cd{e1.re + o1.re, e1.im + o1.im};
    x[5] = Cd{e1.re - o1.re, e1.im - o1.im};
    x[2] = Cd{e2.re + o2.re, e2.im + o2.im};
    x[6] = Cd{e2.re - o2.re, e2.im - o2.im};
    x[3] = Cd{e3.re + o3.re, e3.im + o3.im};
    x[7] = Cd{e3.re - o3.re, e3.im - o3.im};
}

// 16-byte complex slot of the radix-8 exchanges (one ds_read_b128 / ds_write_b128 each)
struct alignas(16) Cl {
    double re, im;
};

// Slot of element i in the three exchanges of a transform (A after pass 0, B after pass 1,
// C after pass 2): A: i + (i >> 4), B: i + 2 (i >> 4), C: i.  Every access is then a
// per-thread base plus a compile-time offset, and the 16 lanes served together by the LDS
// hit 16 distinct slots modulo 16 (distinct banks) in every pattern:
//   A: writes 8t + c at 8t + (t >> 1) + c;  reads t + 512 r at t + (t >> 4) + 544 r
//   B: writes 64 (t >> 3) + 8c + (t & 7) at 72 (t >> 3) + (t & 7) + 8c + 2 (c >> 1);
//      reads at t + 2 (t >> 4) + 576 r
//   C: writes 512 (t >> 6) + 64c + (t & 63) at the same slot; reads at t + 512 r

// LDS carve-up of a workgroup: two exchange buffers of 16-byte slots, the radix-8 engine's
// pass-2 twiddle table, and the slots of the workgroup reductions.
struct Lds {
    Cl* x0;            // exchange buffers (radix 8: 4608 slots each; radix 4: n + n/4)
    Cl* x1;
    Cl* tw;            // radix 8: twiddles of pass 2, W_512^{r k} at (r-1) 64 + k
    double* red;       // 16
};

template <int NN>
__device__ __forceinline__ Lds lds_carve(unsigned char* raw) {
    constexpr int NS = Lay<NN>::P == 8 ? kSlots8 : NN + NN / 4;
    Lds L{};
    L.x0 = reinterpret_cast<Cl*>(raw);
    L.x1 = L.x0 + NS;
    L.tw = L.x1 + NS;
    L.red = reinterpret_cast<double*>(L.tw + (Lay<NN>::P == 8 ? 448 : 0));
    return L;
}

// Constants of the radix-8 engine (n = 4096, thread t), loaded once per launch:
//   w1[c-1] = W_64^{w c}, w = t >> 6 the thread's wavefront: the pass-1 twiddle of element
//   8t + c, which pass 0 applies before its write (pass 1 reads that element as input
//   r = w of its sub-transform position c); uniform over the wavefront (scalar registers);
//   tw[r-1] = W_4096^{r t}, the twiddles of pass 3 (r = 1..7; pass 2 reads its twiddles
//   W_512^{r (t mod 64)} from an LDS table);
//   kf[c] + kl[c] = e^{-i tau k^2/2} / n at the owned frequency t + 512 c (rounded value and
//   its rounding residual, the residual kept in FP32).
struct Eng8 {
    Cd w1[7];
    Cd tw[7];
    Cd kf[8];
    Cx<float> kl[8];
};
// Constants of the radix-4 engine (n = 4^NP, T = n/4 threads, thread t): tw[p-1][r-1] =
// W_{4S}^{r (t mod S)}, S = 4^p, the twiddles of pass p = 1..NP-1 (r = 1..3); kf, kl as
// for the radix-8 engine at the owned frequencies t + T c.
template <int NP>
struct Eng4 {
    Cd tw[NP - 1][3];
    Cd kf[4];
    Cx<float> kl[4];
};
template <int NN> struct Log4 { static constexpr int v = NN == 64 ? 3 : NN == 1024 ? 5 : 0; };
template <int NN>
using Eng = std::conditional_t<Lay<NN>::P == 8, Eng8, Eng4<Log4<NN>::v>>;

// Radix-8 Stockham pass p = 1, 2, 3 over sub-transforms of size S = 8^p: thread t reads
// x_r = A[t + 512 r] (exchange A, B or C), multiplies by W_{8S}^{r (t mod S)} (pass 1: done
// by pass 0 before its write) and forms the 8-point DFT; passes 1 and 2 write y_c to
// B[8S (t / S) + S c + (t mod S)] (exchange B or C), pass 3 keeps X[t + 512 c] = y_c.
template <int SIGN, int PASS>
__device__ __forceinline__ void pass8(Cd (&x)[8], const Cl* a, Cl* b, const Lds& L,
                                      const Eng8& E) {
    const int t = threadIdx.x;
    const Cl* pa = a + (PASS == 1 ? t + (t >> 4) : PASS == 2 ? t + 2 * (t >> 4) : t);
    constexpr int RS = PASS == 1 ? 544 : PASS == 2 ? 576 : 512;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const Cl v = pa[RS * r];
        x[r] = Cd{v.re, v.im};
    }
    if constexpr (PASS != 1) {                  // pass 0 applies the pass-1 twiddles
#pragma unroll
        for (int r = 1; r < 8; ++r) {
            Cl w;
            if constexpr (PASS == 2) w = L.tw[(r - 1) * 64 + (t & 63)];
            else w = Cl{E.tw[r - 1].re, E.tw[r - 1].im};
            x[r] = cmul_s<SIGN>(x[r], Cd{w.re, w.im});
        }
    }
    dft8<SIGN>(x);
    if constexpr (PASS == 1) {
        Cl* pb = b + 72 * (t >> 3) + (t & 7);
#pragma unroll
        for (int c = 0; c < 8; ++c) pb[8 * c + 2 * (c >> 1)] = Cl{x[c].re, x[c].im};
    } else if constexpr (PASS == 2) {
        Cl* pb = b + 512 * (t >> 6) + (t & 63);
#pragma unroll
        for (int c = 0; c < 8; ++c) pb[64 * c] = Cl{x[c].re, x[c].im};
    }
}

// radix-8 engine (n = 4096): forward transforms exchange through buffers 0, 1, 0 and
// inverse ones through 1, 0, 1; they only occur in forward-inverse pairs, so consecutive
// exchanges always alternate.  `hook` runs after the last exchange, before the last pass:
// loads issued there have that pass to arrive in.
template <int SIGN, typename Hook>
__device__ __forceinline__ void fft8e(Cd (&x)[8], const Lds& L, const Eng8& E, Hook&& hook) {
    Cl* u = SIGN < 0 ? L.x0 : L.x1;
    Cl* v = SIGN < 0 ? L.x1 : L.x0;
    const int t = threadIdx.x;
    dft8<SIGN>(x);                               // pass 0: sub-transform size 1
#pragma unroll
    for (int c = 1; c < 8; ++c) x[c] = cmul_s<SIGN>(x[c], E.w1[c - 1]);
    Cl* pu = u + 8 * t + (t >> 1);               // exchange A
#pragma unroll
    for (int c = 0; c < 8; ++c) pu[c] = Cl{x[c].re, x[c].im};
    lds_sync();
    pass8<SIGN, 1>(x, u, v, L, E);               // A -> B
    lds_sync();
    pass8<SIGN, 2>(x, v, u, L, E);               // B -> C
    lds_sync();
    hook();
    pass8<SIGN, 3>(x, u, nullptr, L, E);         // C -> registers
}

// Radix-4 engine (n = 4^NP, T = n/4 threads): pass p = 0..NP-1 over sub-transforms of size
// S = 4^p; thread t reads x_r = A[t + T r] (pass 0: its registers), multiplies by
// W_{4S}^{r (t mod S)} and forms the 4-point DFT; passes p < NP-1 write y_c to
// B[4S (t / S) + S c + (t mod S)] (exchange p, buffer p mod 2), the last pass keeps
// X[t + T c] = y_c.  Slot of element i in exchange p: i + (i >> 4) (p = 0), i + 4 (i >> 4)
// (p = 1), i (p >= 2): every access is a per-thread base plus a compile-time offset, and
// the 16 lanes served together by the LDS hit distinct slots modulo 16 in every pattern.
// A transform has an even number of exchanges (2 or 4), so each restarts on buffer 0, and
// a buffer is written again only after the barrier that follows its last reads.
template <int NN, int SIGN, int PASS>
__device__ __forceinline__ void pass4(Cd (&x)[4], const Lds& L, const Eng<NN>& E) {
    constexpr int T = NN / 4, NP = Log4<NN>::v, S = 1 << (2 * PASS);
    const int t = threadIdx.x;
    const Cl* a = (PASS - 1) % 2 ? L.x1 : L.x0;
    // reads of exchange PASS-1: slot(t + T r) = base + r (T + pad per T elements)
    const Cl* pa = a + (PASS == 1 ? t + (t >> 4) : PASS == 2 ? t + 4 * (t >> 4) : t);
    constexpr int RS = PASS == 1 ? T + T / 16 : PASS == 2 ? T + T / 4 : T;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const Cl v = pa[RS * r];
        x[r] = r ? cmul_s<SIGN>(Cd{v.re, v.im}, E.tw[PASS - 1][r - 1]) : Cd{v.re, v.im};
    }
    dft4<SIGN>(x[0], x[1], x[2], x[3]);
    if constexpr (PASS < NP - 1) {
        Cl* b = PASS % 2 ? L.x1 : L.x0;
        // writes of exchange PASS: element 4S (t / S) + S c + (t mod S)
        Cl* pb = b + (PASS == 1 ? 20 * (t >> 2) + (t & 3) : 4 * S * (t / S) + (t & (S - 1)));
#pragma unroll
        for (int c = 0; c < 4; ++c) pb[S * c] = Cl{x[c].re, x[c].im};
    }
}

template <int NN, int SIGN, typename Hook>
__device__ __forceinline__ void fft4e(Cd (&x)[4], const Lds& L, const Eng<NN>& E, Hook&& hook) {
    constexpr int NP = Log4<NN>::v;
    static_assert(NP == 3 || NP == 5, "radix-4 engine: n = 64 or 1024");
    const int t = threadIdx.x;
    dft4<SIGN>(x[0], x[1], x[2], x[3]);          // pass 0
    Cl* pu = L.x0 + 4 * t + (t >> 2);            // slot(4t + c) = 4t + (t >> 2) + c
#pragma unroll
    for (int c = 0; c < 4; ++c) pu[c] = Cl{x[c].re, x[c].im};
    lds_sync();
    pass4<NN, SIGN, 1>(x, L, E);
    lds_sync();
    if constexpr (NP == 5) {
        pass4<NN, SIGN, 2>(x, L, E);
        lds_sync();
        pass4<NN, SIGN, 3>(x, L, E);
        lds_sync();
        hook();
        pass4<NN, SIGN, 4>(x, L, E);
    } else {
        hook();
        pass4<NN, SIGN, 2>(x, L, E);
    }
}

// FFT of the register-resident state (natural order, thread t owns t + T i), result in the
// same layout.  SIGN = -1 forward e^{-2 pi i jk/n}; +1 inverse without 1/n.
template <int NN, int SIGN, typename Hook>
__device__ __forceinline__ void fft(Cd (&x)[Lay<NN>::P], const Lds& L, const Eng<NN>& E,
                                    Hook&& hook) {
    if constexpr (Lay<NN>::P == 8)
        fft8e<SIGN>(x, L, E, hook);
    else
        fft4e<NN, SIGN>(x, L, E, hook);
}

struct NoHook {
    __device__ __forceinline__ void operator()() const {}
};

struct GpeArgs {
    int B, n, K, N;
    const int* s;
    double tau, dx, g;
    const double* V0;
    const double* V1;
    double V2;
    const dcx* tab;        // FFT twiddles W_n^m, m < n (FP64)
    const dcx* Kh;         // n: e^{-i tau k^2/4} / n (FP64)
    const dcx* Kf;         // n/2 + 1: e^{-i tau k^2/2} / n at |frequency| 0..n/2 (FP64)
    const dcx* Kfl;        // n/2 + 1: rounding residual of Kf (FP64)
    double* u;             // B*K
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

// engine constants into registers (the radix-8 pass-2 twiddles into LDS); potentials into
// registers
template <int NN>
__device__ __forceinline__ void setup(const GpeArgs& A, const Lds& L, Eng<NN>& E,
                                      double (&v0)[Lay<NN>::P], double (&v1)[Lay<NN>::P]) {
    constexpr int T = Lay<NN>::T, P = Lay<NN>::P;
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        v0[i] = A.V0[t + T * i];
        v1[i] = A.V1[t + T * i];
    }
    if constexpr (P == 8) {
        // W_512^{r k} = W_4096^{8 r k}
        for (int i = t; i < 448; i += T) {
            const int m = 8 * (i / 64 + 1) * (i & 63);
            L.tw[i] = Cl{A.tab[m].re, A.tab[m].im};
        }
        const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
#pragma unroll
        for (int r = 1; r < 8; ++r) {
            const dcx w = A.tab[(r * t) & (NN - 1)];
            E.tw[r - 1] = Cd{w.re, w.im};
            const dcx w1 = A.tab[(64 * wv * r) & (NN - 1)];
            E.w1[r - 1] = Cd{w1.re, w1.im};
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int m = t + T * c, mf = m <= NN / 2 ? m : NN - m;
            const dcx k = A.Kf[mf], kl = A.Kfl[mf];
            E.kf[c] = Cd{k.re, k.im};
            E.kl[c] = Cx<float>{(float)kl.re, (float)kl.im};
        }
        __syncthreads();
        return;
    } else {
        constexpr int NP = Log4<NN>::v;
#pragma unroll
        for (int q = 1; q < NP; ++q) {            // W_{4S}^{m} = W_n^{(n / 4S) m}, S = 4^q
            const int S = 1 << (2 * q);
#pragma unroll
            for (int r = 1; r < 4; ++r) {
                const dcx w = A.tab[((NN / (4 * S)) * r * (t & (S - 1))) & (NN - 1)];
                E.tw[q - 1][r - 1] = Cd{w.re, w.im};
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int m = t + T * c, mf = m <= NN / 2 ? m : NN - m;
            const dcx k = A.Kf[mf], kl = A.Kfl[mf];
            E.kf[c] = Cd{k.re, k.im};
            E.kl[c] = Cx<float>{(float)kl.re, (float)kl.im};
        }
    }
}

// deterministic workgroup sum (wave tree, then the wavefront partials in order)
template <int NN>
__device__ __forceinline__ double block_sum(double v, const Lds& L) {
    constexpr int T = Lay<NN>::T;
    constexpr int TT = T < 64 ? T : 64;                    // lanes of the (first) wavefront
    constexpr int NW = T / 64;
    for (int off = TT / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, TT);
    if constexpr (NW <= 1) return v;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) L.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += L.red[i];
    return s;
}

// x <- F^-1 diag(k) F x, k at the owned frequencies: the fused kinetic factor held in
// registers (kt == nullptr) or a table in global memory; CONJ uses conj(k) (adjoint kicks).
// The fused factor is applied as its rounded value plus the rounding residual: a rounded
// factor alone makes the same relative error at every one of the K steps of a sweep, which
// adds up coherently (about 5e-13 over 10^4 steps).
template <int NN, bool CONJ, typename Hook>
__device__ __forceinline__ void kick(Cd (&x)[Lay<NN>::P], const Lds& L, const Eng<NN>& E,
                                     const Cd* kt, Hook&& hook) {
    constexpr int T = Lay<NN>::T, P = Lay<NN>::P;
    fft<NN, -1>(x, L, E, NoHook{});
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int m = threadIdx.x + T * i;
        if (kt) {
            const Cd k = kt[m];
            x[i] = CONJ ? cmulc(x[i], k) : cmul(x[i], k);
        } else {
            const Cd k = E.kf[i], kl = up<float>(E.kl[i]);
            const Cd lo = CONJ ? cmulc(x[i], kl) : cmul(x[i], kl);
            const Cd v = x[i];
            if (CONJ)
                x[i] = Cd{fma(v.re, k.re, fma(v.im, k.im, lo.re)),
                          fma(v.im, k.re, fma(-v.re, k.im, lo.im))};
            else
                x[i] = Cd{fma(v.re, k.re, fma(-v.im, k.im, lo.re)),
                          fma(v.im, k.re, fma(v.re, k.im, lo.im))};
        }
    }
    fft<NN, 1>(x, L, E, hook);
}
template <int NN, bool CONJ>
__device__ __forceinline__ void kick(Cd (&x)[Lay<NN>::P], const Lds& L, const Eng<NN>& E,
                                     const Cd* kt) {
    kick<NN, CONJ>(x, L, E, kt, NoHook{});
}

template <int NN>
__device__ __forceinline__ void load_state(Cd (&x)[Lay<NN>::P], const dcx* src) {
    constexpr int T = Lay<NN>::T;
#pragma unroll
    for (int i = 0; i < Lay<NN>::P; ++i) {
        const dcx v = src[threadIdx.x + T * i];
        x[i] = Cd{v.re, v.im};
    }
}

template <int NN>
__device__ __forceinline__ void store_state(dcx* dst, const Cd (&x)[Lay<NN>::P]) {
    constexpr int T = Lay<NN>::T;
#pragma unroll
    for (int i = 0; i < Lay<NN>::P; ++i) dst[threadIdx.x + T * i] = dcx{x[i].re, x[i].im};
}

// e^{-i theta} at the owned points, theta = tau (V(x,u) + g |a|^2) (V in FP64)
template <typename R>
__device__ __forceinline__ Cd phase(const GpeArgs& A, double v0, double v1, double u, Cd a) {
    const double V = v0 + u * v1 + u * u * A.V2;
    const R th = (R)(A.tau * (V + A.g * (a.re * a.re + a.im * a.im)));
    R sn, cs;
    sincos_r(th, &sn, &cs);
    return Cd{(double)cs, -(double)sn};
}

// The radix-8 engine has no registers to spare for the potentials across a transform: they
// are loaded again inside the last pass of every inverse transform (`reload_pot`, called
// from the kick's hook), through a pointer the compiler cannot prove unchanged, so the loads
// stay where they are issued instead of being hoisted out of the step loop (which turns
// them into spills).  The radix-16 engine keeps them in registers.
template <typename T>
__device__ __forceinline__ const T* opaque(const T* p) {
    __asm__ volatile("" : "+s"(p));
    return p;
}
template <int NN>
__device__ __forceinline__ void reload_pot(const GpeArgs& A, double (&v0)[Lay<NN>::P],
                                           double (&v1)[Lay<NN>::P]) {
    if constexpr (Lay<NN>::P == 8) {
        constexpr int T = Lay<NN>::T;
        const double* V0 = opaque(A.V0) + threadIdx.x;
        const double* V1 = opaque(A.V1) + threadIdx.x;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            v0[i] = V0[T * i];
            v1[i] = V1[T * i];
        }
    }
}

// Forward steps j0 .. j1-1 from x = a_{j0}, storing a_j in traj_b.  After the last step:
// psi_{j1} = F^-1 Kh F b_{j1-1} is formed (and written to psi_out if given) when psi_out or
// cont is set, and with cont x = a_{j1} = F^-1 Kh F psi_{j1} on return.
template <int NN, typename R>
__device__ void fwd_run(const GpeArgs& A, const Lds& L, const Eng<NN>& E, int b, int j0,
                        int j1, Cd (&x)[Lay<NN>::P], double (&v0)[Lay<NN>::P],
                        double (&v1)[Lay<NN>::P], Cx<R>* traj_b, dcx* psi_out, bool cont) {
    constexpr int T = Lay<NN>::T, P = Lay<NN>::P;
    const int t = threadIdx.x;
    const auto reload = [&] { reload_pot<NN>(A, v0, v1); };
    const double* ub = A.u + (size_t)b * A.K;
    double un = ub[j0];
    for (int j = j0; j < j1; ++j) {
        Cx<R>* tj = traj_b + (size_t)j * NN;
#pragma unroll
        for (int i = 0; i < P; ++i) tj[t + T * i] = down<R>(x[i]);
        const bool last = j == j1 - 1;
        if (last && !psi_out && !cont) return;
        const double u = un;
        if (!last) un = ub[j + 1];                        // next step's control, ahead of use
#pragma unroll
        for (int i = 0; i < P; ++i) x[i] = cmul(x[i], phase<R>(A, v0[i], v1[i], u, x[i]));
        if (!last) {
            kick<NN, false>(x, L, E, nullptr, reload);
        } else {
            kick<NN, false>(x, L, E, reinterpret_cast<const Cd*>(A.Kh), reload);
            if (psi_out) store_state<NN>(psi_out, x);
            if (cont) kick<NN, false>(x, L, E, reinterpret_cast<const Cd*>(A.Kh), reload);
        }
    }
}

// Adjoint steps j1-1 down to j0 from x = nu'_{j1-1}, reading a_j from traj_b.  After step
// j0 (mu_{j0} in x): final 0 stops; 1 forms nu_{j0} (written to nu_out); 2 forms nu_{j0},
// writes it, and continues to x = nu'_{j0-1}.  With grad_on every step's gradient is formed
// and, with upd, the update u_j += rho g_j applied (u_j is not read again here).
template <int NN, typename R>
__device__ void adj_run(const GpeArgs& A, const Lds& L, const Eng<NN>& E, int b, int j0,
                        int j1, Cd (&x)[Lay<NN>::P], double (&v0)[Lay<NN>::P],
                        double (&v1)[Lay<NN>::P], const Cx<R>* traj_b, dcx* nu_out,
                        int final_kick, bool grad_on, bool upd) {
    constexpr int T = Lay<NN>::T, P = Lay<NN>::P;
    const int t = threadIdx.x;
    const Cd* conjKh = reinterpret_cast<const Cd*>(A.Kh);
    double* ub = A.u + (size_t)b * A.K;
    // u_j of the next step down is requested one step ahead (u_{j-1} is read before this
    // loop updates it); so is a_j in the FP32 path, whose copy costs half the registers,
    // and in both paths of the radix-8 engine, whose kick requests it in its last pass
    constexpr bool kHook = P == 8;
    constexpr bool kAhead = kHook || sizeof(R) == 4;
    Cx<R> an[P];
    int jn = j1 - 1;                  // row requested by the next kick's hook
    const auto reload = [&] { reload_pot<NN>(A, v0, v1); };
    const auto reload_ahead = [&] {
        reload_pot<NN>(A, v0, v1);
        if constexpr (kHook) {
            const Cx<R>* row = opaque(traj_b) + (size_t)jn * NN + t;
#pragma unroll
            for (int i = 0; i < P; ++i) an[i] = row[T * i];
        }
    };
    double un = ub[j1 - 1];
    if (kAhead) {
#pragma unroll
        for (int i = 0; i < P; ++i) an[i] = traj_b[(size_t)(j1 - 1) * NN + t + T * i];
    }
    for (int j = j1 - 1; j >= j0; --j) {
        const double u = un;
        Cd av[P];
#pragma unroll
        for (int i = 0; i < P; ++i)
            av[i] = up<R>(kAhead ? an[i] : traj_b[(size_t)j * NN + t + T * i]);
        if (j > j0) {
            un = ub[j - 1];
            jn = j - 1;
            if (kAhead && !kHook) {
#pragma unroll
                for (int i = 0; i < P; ++i) an[i] = traj_b[(size_t)(j - 1) * NN + t + T * i];
            }
        }
        double part = 0.0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const Cd a = av[i];
            const Cd e = phase<R>(A, v0[i], v1[i], u, a);
            if (grad_on) {
                const Cd bb = cmul(a, e);
                const double dV = v1[i] + 2.0 * u * A.V2;
                part += dV * (x[i].re * bb.im - x[i].im * bb.re);      // Im(conj(nu') b)
            }
            const Cd w = cmulc(x[i], e);                               // e^{+i theta} nu'
            const double f = 2.0 * A.tau * A.g * (w.re * a.im - w.im * a.re);
            x[i] = Cd{w.re + f * a.re, w.im + f * a.im};
        }
        if (grad_on) {
            const double gj = A.dx * block_sum<NN>(part, L);
            if (t == 0) {
                const size_t ui = (size_t)b * A.K + j;
                if (A.grad) A.grad[ui] = gj;
                if (upd) ub[j] = fma(A.rho, gj, u);
                if (!(fabs(gj) < 1e300)) atomicOr(&A.flags[0], 1);
            }
        }
        if (j > j0) {
            kick<NN, true>(x, L, E, nullptr, reload_ahead);
        } else if (final_kick > 0) {
            kick<NN, true>(x, L, E, conjKh, reload);
            if (nu_out) store_state<NN>(nu_out, x);
            if (final_kick == 2) kick<NN, true>(x, L, E, conjKh, reload);
        }
    }
}

// Sequential forward sweep of one instance: psi(t_n) for every n, a_j for every step,
// J and F at T.
template <int NN, typename R>
__global__ __launch_bounds__(Lay<NN>::T) void k_gpe_fwd_sweep(GpeArgs A) {
    extern __shared__ unsigned char smem_raw[];
    const Lds L = lds_carve<NN>(smem_raw);
    const int b = blockIdx.x;
    constexpr int P = Lay<NN>::P;
    double v0[P], v1[P];
    Eng<NN> E;
    setup<NN>(A, L, E, v0, v1);
    dcx* Psi_b = A.Psi + (size_t)b * (A.N + 1) * NN;
    Cx<R>* traj_b = reinterpret_cast<Cx<R>*>(A.traj) + (size_t)b * A.K * NN;
    Cd x[P];
    load_state<NN>(x, A.psi0);
    store_state<NN>(Psi_b, x);
    kick<NN, false>(x, L, E, reinterpret_cast<const Cd*>(A.Kh));      // a_0
    for (int nn = 0; nn < A.N; ++nn)
        fwd_run<NN, R>(A, L, E, b, A.s[nn], A.s[nn + 1], x, v0, v1, traj_b,
                       Psi_b + (size_t)(nn + 1) * NN, nn + 1 < A.N);
    // x = psi_K:  J = Re <psi_K|psi_f> dx,  F = |<psi_K|psi_f> dx|^2
    constexpr int T = Lay<NN>::T;
    double zr = 0.0, zi = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const dcx f = A.target[threadIdx.x + T * i];
        zr += x[i].re * f.re + x[i].im * f.im;
        zi += x[i].re * f.im - x[i].im * f.re;
    }
    zr = A.dx * block_sum<NN>(zr, L);
    zi = A.dx * block_sum<NN>(zi, L);
    if (threadIdx.x == 0) {
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
template <int NN, typename R>
__global__ __launch_bounds__(Lay<NN>::T) void k_gpe_adj_sweep(GpeArgs A) {
    extern __shared__ unsigned char smem_raw[];
    const Lds L = lds_carve<NN>(smem_raw);
    const int b = blockIdx.x;
    constexpr int P = Lay<NN>::P;
    double v0[P], v1[P];
    Eng<NN> E;
    setup<NN>(A, L, E, v0, v1);
    dcx* Lam_b = A.Lam + (size_t)b * (A.N + 1) * NN;
    const Cx<R>* traj_b = reinterpret_cast<const Cx<R>*>(A.traj) + (size_t)b * A.K * NN;
    Cd x[P];
    load_state<NN>(x, A.target);
    store_state<NN>(Lam_b + (size_t)A.N * NN, x);
    kick<NN, true>(x, L, E, reinterpret_cast<const Cd*>(A.Kh));       // nu'_{K-1}
    for (int nn = A.N - 1; nn >= 0; --nn)
        adj_run<NN, R>(A, L, E, b, A.s[nn], A.s[nn + 1], x, v0, v1, traj_b,
                       Lam_b + (size_t)nn * NN, nn > 0 ? 2 : 1, false, false);
}

// Slice n of instance b: forward from psi(t_n), adjoint from nu(t_{n+1}), gradient, update.
template <int NN, typename R>
__global__ __launch_bounds__(Lay<NN>::T) void k_gpe_slice(GpeArgs A) {
    extern __shared__ unsigned char smem_raw[];
    const Lds L = lds_carve<NN>(smem_raw);
    const int nn = blockIdx.x, b = blockIdx.y;
    constexpr int P = Lay<NN>::P;
    double v0[P], v1[P];
    Eng<NN> E;
    setup<NN>(A, L, E, v0, v1);
    const int j0 = A.s[nn], j1 = A.s[nn + 1];
    Cx<R>* traj_b = reinterpret_cast<Cx<R>*>(A.traj) + (size_t)b * A.K * NN;
    const dcx* Psi_b = A.Psi + (size_t)b * (A.N + 1) * NN;
    const dcx* Lam_b = A.Lam + (size_t)b * (A.N + 1) * NN;
    Cd x[P];
    load_state<NN>(x, Psi_b + (size_t)nn * NN);
    kick<NN, false>(x, L, E, reinterpret_cast<const Cd*>(A.Kh));      // a_{j0}
    fwd_run<NN, R>(A, L, E, b, j0, j1, x, v0, v1, traj_b, nullptr, false);
    load_state<NN>(x, Lam_b + (size_t)(nn + 1) * NN);
    kick<NN, true>(x, L, E, reinterpret_cast<const Cd*>(A.Kh));       // nu'_{j1-1}
    const bool upd = A.update && (A.active == nullptr || A.active[b] != 0);
    adj_run<NN, R>(A, L, E, b, j0, j1, x, v0, v1, traj_b, nullptr, 0, true, upd);
}

// ---------------------------------------------------------------------------------------
// Frozen-density propagator assembling (the reading of Sec. 4.C's propagator assembling for
// the condensate).  With a_j frozen at the last slice pass's trajectories (traj), one Strang
// step is the linear unitary map S_j psi = Kh e^{-i tau (V(u_j) + g |a_j|^2)} Kh psi and the
// exact adjoint step linearised there is the real-linear map R_j of adj_run.  The slice maps
// are formed on basis vectors (one workgroup per vector, slice and instance), and the
// boundaries follow from 2N matrix-vector products:
//   Psi_0 = psi0, Psi_{n+1} = M_n Psi_n;  Lambda_N = psi_f,
//   Lambda_n = sum_m Re(Lambda_{n+1,m}) A_n(e_m) + Im(Lambda_{n+1,m}) A_n(i e_m).
// Column v of M_n (and of A_n) is stored contiguously: M[((b N + n) ncol + v) n_grid + r].

// column v of M_n: S_{j1-1} ... S_{j0} e_v (kinetic half steps fused inside the slice)
template <int NN, typename R>
__global__ __launch_bounds__(Lay<NN>::T) void k_gpe_frozen_fwd(GpeArgs A, dcx* M) {
    extern __shared__ unsigned char smem_raw[];
    const Lds L = lds_carve<NN>(smem_raw);
    const int v = blockIdx.x, nn = blockIdx.y, b = blockIdx.z;
    constexpr int T = Lay<NN>::T, P = Lay<NN>::P;
    const int t = threadIdx.x;
    double v0[P], v1[P];
    Eng<NN> E;
    setup<NN>(A, L, E, v0, v1);
    const int j0 = A.s[nn], j1 = A.s[nn + 1];
    const Cx<R>* traj_b = reinterpret_cast<const Cx<R>*>(A.traj) + (size_t)b * A.K * NN;
    const double* ub = A.u + (size_t)b * A.K;
    Cd x[P];
#pragma unroll
    for (int i = 0; i < P; ++i) x[i] = Cd{t + T * i == v ? 1.0 : 0.0, 0.0};
    kick<NN, false>(x, L, E, reinterpret_cast<const Cd*>(A.Kh));
    for (int j = j0; j < j1; ++j) {
        const double u = ub[j];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const Cd af = up<R>(traj_b[(size_t)j * NN + t + T * i]);     // frozen a_j
            x[i] = cmul(x[i], phase<R>(A, v0[i], v1[i], u, af));
        }
        kick<NN, false>(x, L, E, j + 1 < j1 ? nullptr : reinterpret_cast<const Cd*>(A.Kh));
    }
    store_state<NN>(M + (((size_t)b * A.N + nn) * NN + v) * NN, x);
}

// column c of A_n: R_{j0} ... R_{j1-1} applied to e_c (c < n) or i e_{c-n}
template <int NN, typename R>
__global__ __launch_bounds__(Lay<NN>::T) void k_gpe_frozen_adj(GpeArgs A, dcx* Aj) {
    extern __shared__ unsigned char smem_raw[];
    const Lds L = lds_carve<NN>(smem_raw);
    const int c = blockIdx.x, nn = blockIdx.y, b = blockIdx.z;
    constexpr int T = Lay<NN>::T, P = Lay<NN>::P;
    const int t = threadIdx.x;
    double v0[P], v1[P];
    Eng<NN> E;
    setup<NN>(A, L, E, v0, v1);
    const int j0 = A.s[nn], j1 = A.s[nn + 1];
    const Cx<R>* traj_b = reinterpret_cast<const Cx<R>*>(A.traj) + (size_t)b * A.K * NN;
    const int m = c < NN ? c : c - NN;
    Cd x[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const bool on = t + T * i == m;
        x[i] = c < NN ? Cd{on ? 1.0 : 0.0, 0.0} : Cd{0.0, on ? 1.0 : 0.0};
    }
    kick<NN, true>(x, L, E, reinterpret_cast<const Cd*>(A.Kh));
    adj_run<NN, R>(A, L, E, b, j0, j1, x, v0, v1, traj_b,
                   Aj + (((size_t)b * A.N + nn) * 2 * NN + c) * NN, 1, false, false);
}

// y = sum_c w_c col_c over ncol columns of n_grid entries (one thread per entry, instances on
// blockIdx.y): complex weights w_c = x_c (ncol = n_grid), or real weights Re x_c, Im x_c
// for the columns c and n_grid + c (ncol = 2 n_grid)
__global__ __launch_bounds__(256) void k_gpe_gemv(const dcx* cols, size_t cstride, int ng,
                                                  int realw, const dcx* x, size_t xstride,
                                                  dcx* y, size_t ystride) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    if (r >= ng) return;
    const dcx* C = cols + (size_t)b * cstride;
    const dcx* xb = x + (size_t)b * xstride;
    double ar = 0.0, ai = 0.0;
    if (!realw) {
        for (int c = 0; c < ng; ++c) {
            const dcx m = C[(size_t)c * ng + r], w = xb[c];
            ar = fma(m.re, w.re, fma(-m.im, w.im, ar));
            ai = fma(m.re, w.im, fma(m.im, w.re, ai));
        }
    } else {
        for (int c = 0; c < ng; ++c) {
            const dcx m1 = C[(size_t)c * ng + r], m2 = C[(size_t)(ng + c) * ng + r];
            const dcx w = xb[c];
            ar = fma(m1.re, w.re, fma(m2.re, w.im, ar));
            ai = fma(m1.im, w.re, fma(m2.im, w.im, ai));
        }
    }
    y[(size_t)b * ystride + r] = dcx{ar, ai};
}

// Psi_0 = psi0 and Lambda_N = psi_f for every instance
__global__ void k_gpe_bnd_ends(GpeArgs A) {
    const int b = blockIdx.y;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < A.n; r += gridDim.x * blockDim.x) {
        A.Psi[(size_t)b * (A.N + 1) * A.n + r] = A.psi0[r];
        A.Lam[((size_t)b * (A.N + 1) + A.N) * A.n + r] = A.target[r];
    }
}

// J, F from Psi_N (fixed-order reduction), freezing at fid_stop, numeric flag
__global__ __launch_bounds__(256) void k_gpe_bnd_finish(GpeArgs A) {
    __shared__ double rr[256], ri[256];
    const int b = blockIdx.x, t = threadIdx.x;
    const dcx* P = A.Psi + ((size_t)b * (A.N + 1) + A.N) * A.n;
    double zr = 0.0, zi = 0.0;
    for (int r = t; r < A.n; r += 256) {
        const dcx p = P[r], f = A.target[r];
        zr += p.re * f.re + p.im * f.im;
        zi += p.re * f.im - p.im * f.re;
    }
    rr[t] = zr;
    ri[t] = zi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            rr[t] += rr[t + w];
            ri[t] += ri[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double J = A.dx * rr[0], Zi = A.dx * ri[0];
        const double F = J * J + Zi * Zi;
        A.J[b] = J;
        A.F[b] = F;
        if (A.Jhist) A.Jhist[b] = J;
        if (!(fabs(J) < 1e300)) atomicOr(&A.flags[0], 1);
        if (A.active) {
            if (A.active[b] && F >= A.fid_stop) A.active[b] = 0;
            if (A.active[b]) atomicAdd(&A.flags[1], 1);
        }
    }
}

}  // namespace

struct GpeExt {
    int n = 0;
    double L = 0, g = 0, V2 = 0, dx = 0;
    double* V0 = nullptr;
    double* V1 = nullptr;
    dcx* tab = nullptr;
    dcx* Kh = nullptr;
    dcx* Kf = nullptr;
    dcx* Kfl = nullptr;
    dcx* Psi = nullptr;
    dcx* Lam = nullptr;
    dcx* psi0 = nullptr;
    dcx* target = nullptr;
    void* traj = nullptr;
    dcx* fM = nullptr;     // frozen-density slice maps: B N n columns of n (forward)
    dcx* fA = nullptr;     //                            B N 2n columns of n (adjoint)
};

static void gpe_free(ism_problem* p) {
    delete reinterpret_cast<GpeExt*>(p->ext);
    p->ext = nullptr;
}

size_t gpe_footprint_extra(size_t n, int K, int N, int batch, int precision) {
    const size_t rs = precision == ISM_FP64 ? 16 : 8;
    return (size_t)batch * K * n * rs + 2 * (size_t)batch * (N + 1) * n * 16 + (3 * n + 2) * 16;
}

size_t gpe_frozen_bytes(size_t n, int N, int batch) {
    return (size_t)batch * N * 3 * n * n * sizeof(dcx);
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
    A.tab = x->tab;
    A.Kh = x->Kh;
    A.Kf = x->Kf;
    A.Kfl = x->Kfl;
    A.u = p->u;
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

// two exchange buffers of 16-byte slots, the radix-8 engine's pass-2 twiddle table and the
// reduction slots (FP64 in both precisions)
static size_t gpe_shmem(int n) {
    if (n == 4096) return (2 * (size_t)kSlots8 + 448) * 16 + 16 * sizeof(double);
    return 2 * ((size_t)n + n / 4) * 16 + 16 * sizeof(double);
}

template <int NN, typename R>
static void gpe_launch_sweeps_n(const GpeArgs& A, hipStream_t st, size_t shm) {
    hipLaunchKernelGGL((k_gpe_fwd_sweep<NN, R>), dim3(A.B), dim3(Lay<NN>::T), shm, st, A);
    hipLaunchKernelGGL((k_gpe_adj_sweep<NN, R>), dim3(A.B), dim3(Lay<NN>::T), shm, st, A);
}

template <typename R>
static void gpe_launch_sweeps(const GpeArgs& A, hipStream_t st, size_t shm) {
    if (A.n == 4096) gpe_launch_sweeps_n<4096, R>(A, st, shm);
    else if (A.n == 1024) gpe_launch_sweeps_n<1024, R>(A, st, shm);
    else gpe_launch_sweeps_n<64, R>(A, st, shm);
}

template <typename R>
static void gpe_launch_slice(const GpeArgs& A, hipStream_t st, size_t shm) {
    if (A.n == 4096)
        hipLaunchKernelGGL((k_gpe_slice<4096, R>), dim3(A.N, A.B), dim3(Lay<4096>::T), shm, st, A);
    else if (A.n == 1024)
        hipLaunchKernelGGL((k_gpe_slice<1024, R>), dim3(A.N, A.B), dim3(Lay<1024>::T), shm, st, A);
    else
        hipLaunchKernelGGL((k_gpe_slice<64, R>), dim3(A.N, A.B), dim3(Lay<64>::T), shm, st, A);
}

template <int NN, typename R>
static hipError_t gpe_set_shmem(int shm) {
    const void* ks[] = {(const void*)k_gpe_fwd_sweep<NN, R>, (const void*)k_gpe_adj_sweep<NN, R>,
                        (const void*)k_gpe_slice<NN, R>, (const void*)k_gpe_frozen_fwd<NN, R>,
                        (const void*)k_gpe_frozen_adj<NN, R>};
    hipError_t e = hipSuccess;
    for (const void* k : ks)
        if (e == hipSuccess) e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, shm);
    return e;
}

// slice maps at the current controls with the densities of the last slice pass, then the
// 2N boundary products, J and F
template <int NN, typename R>
static void gpe_launch_frozen(ism_problem* p, const GpeArgs& A, GpeExt* x, size_t shm) {
    const int B = A.B, N = A.N;
    {
        TimeScope ts(p, KID_GPE_ASSEMBLE);
        hipLaunchKernelGGL((k_gpe_frozen_fwd<NN, R>), dim3(NN, N, B), dim3(Lay<NN>::T), shm,
                           p->stream, A, x->fM);
        hipLaunchKernelGGL((k_gpe_frozen_adj<NN, R>), dim3(2 * NN, N, B), dim3(Lay<NN>::T), shm,
                           p->stream, A, x->fA);
    }
    TimeScope ts(p, KID_GPE_BOUNDARY);
    const dim3 g((NN + 255) / 256, B), blk(NN < 256 ? NN : 256);
    const size_t nb = (size_t)(N + 1) * NN;
    hipLaunchKernelGGL(k_gpe_bnd_ends, g, blk, 0, p->stream, A);
    for (int n = 0; n < N; ++n)
        hipLaunchKernelGGL(k_gpe_gemv, g, blk, 0, p->stream, x->fM + (size_t)n * NN * NN,
                           (size_t)N * NN * NN, NN, 0, x->Psi + (size_t)n * NN, nb,
                           x->Psi + (size_t)(n + 1) * NN, nb);
    for (int n = N - 1; n >= 0; --n)
        hipLaunchKernelGGL(k_gpe_gemv, g, blk, 0, p->stream, x->fA + (size_t)n * 2 * NN * NN,
                           (size_t)N * 2 * NN * NN, NN, 1, x->Lam + (size_t)(n + 1) * NN, nb,
                           x->Lam + (size_t)n * NN, nb);
    hipLaunchKernelGGL(k_gpe_bnd_finish, dim3(B), dim3(256), 0, p->stream, A);
}

template <typename R>
static int gpe_boundary_t(ism_problem* p, double* Jhist_k, double fid_stop, bool use_active) {
    GpeArgs A = gpe_args(p);
    A.Jhist = Jhist_k;
    A.active = use_active ? p->active : nullptr;
    A.fid_stop = fid_stop;
    {
        TimeScope ts(p, KID_GPE_SWEEP);
        gpe_launch_sweeps<R>(A, p->stream, gpe_shmem(A.n));
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
    {
        TimeScope ts(p, KID_GPE_SLICE);
        gpe_launch_slice<R>(A, p->stream, gpe_shmem(A.n));
    }
    if (hipGetLastError() != hipSuccess) return ISM_E_DEVICE;
    if (update) p->bvalid = false;
    return ISM_OK;
}

template <typename R>
static int gpe_boundary_frozen_t(ism_problem* p, double* Jhist_k, double fid_stop, bool use_active) {
    GpeExt* x = reinterpret_cast<GpeExt*>(p->ext);
    if (!x->fM || !x->fA) return ISM_E_STATE;
    GpeArgs A = gpe_args(p);
    A.Jhist = Jhist_k;
    A.active = use_active ? p->active : nullptr;
    A.fid_stop = fid_stop;
    const size_t shm = gpe_shmem(A.n);
    if (A.n == 1024) gpe_launch_frozen<1024, R>(p, A, x, shm);
    else gpe_launch_frozen<64, R>(p, A, x, shm);
    if (hipGetLastError() != hipSuccess) return ISM_E_DEVICE;
    p->bvalid = true;
    return ISM_OK;
}

int gpe_boundary_frozen_pass(ism_problem* p, double* Jhist_k, double fid_stop, bool use_active) {
    return p->precision == ISM_FP64
               ? gpe_boundary_frozen_t<double>(p, Jhist_k, fid_stop, use_active)
               : gpe_boundary_frozen_t<float>(p, Jhist_k, fid_stop, use_active);
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
    // Tables, each entry computed in extended precision (x87 long double) and rounded once
    // to FP64.  Twiddles e^{-2 pi i e/m} with the exponent reduced exactly.
    const long double PIL = 3.141592653589793238462643383279502884L;
    auto root = [&](long long e, long long m) {
        e %= m;
        const long double a = 2.0L * PIL * (long double)e / (long double)m;
        return dcx{(double)cosl(a), (double)-sinl(a)};
    };
    std::vector<dcx> tab(n), kh(n), kf(n / 2 + 1), kfl(n / 2 + 1);
    for (int m = 0; m < n; ++m) tab[m] = root(m, n);          // every root W_n^m
    // wavenumbers k_f = 2 pi f / (n dx) in FP64, formed as (2 pi) (f (1 / (n dx))) with
    // dx = L / n (the grid's frequencies in the usual fftfreq order); the kinetic phase
    // -tau k^2 / 4 and its exponential are then evaluated in extended precision
    const double dxd = L / n, fscale = 1.0 / (n * dxd), twopi = 2 * 3.141592653589793;
    auto phase_of = [&](int f) {
        const double k = twopi * ((double)f * fscale);
        return -(long double)p->tau * (long double)k * (long double)k / 4.0L;
    };
    for (int m = 0; m < n; ++m) {
        const int f = m < n / 2 ? m : m - n;            // fftfreq ordering
        const long double ph = phase_of(f);
        kh[m] = dcx{(double)(cosl(ph) / n), (double)(sinl(ph) / n)};
    }
    for (int m = 0; m <= n / 2; ++m) {                  // |frequency| m (the factor is even)
        const long double ph = 2.0L * phase_of(m == n / 2 ? -m : m);
        const long double cr = cosl(ph) / n, ci = sinl(ph) / n;
        kf[m] = dcx{(double)cr, (double)ci};
        kfl[m] = dcx{(double)(cr - (long double)kf[m].re), (double)(ci - (long double)kf[m].im)};
    }
    const bool f64 = p->precision == ISM_FP64;
    if ((st = dev_upload(p, (void**)&x->tab, tab.data(), tab.size() * sizeof(dcx)))) return st;
    if ((st = dev_upload(p, (void**)&x->Kh, kh.data(), kh.size() * sizeof(dcx)))) return st;
    if ((st = dev_upload(p, (void**)&x->Kf, kf.data(), kf.size() * sizeof(dcx)))) return st;
    if ((st = dev_upload(p, (void**)&x->Kfl, kfl.data(), kfl.size() * sizeof(dcx)))) return st;
    const size_t nb = (size_t)p->B * (p->N + 1) * n * sizeof(dcx);
    if ((st = dev_alloc(p, (void**)&x->Psi, nb))) return st;
    if ((st = dev_alloc(p, (void**)&x->Lam, nb))) return st;
    if ((st = dev_alloc(p, &x->traj, (size_t)p->B * p->K * n * (f64 ? 16 : 8)))) return st;
    if (p->gpe_frozen) {      // slice maps of the frozen-density boundaries, held from the start
        if (n > 1024) return ISM_E_UNSUPPORTED;
        const size_t m = (size_t)p->B * p->N * n * n * sizeof(dcx);
        if ((st = dev_alloc(p, (void**)&x->fM, m))) return st;
        if ((st = dev_alloc(p, (void**)&x->fA, 2 * m))) return st;
    }
    const int shm = (int)gpe_shmem(n);
    hipError_t e;
    if (n == 4096)
        e = f64 ? gpe_set_shmem<4096, double>(shm) : gpe_set_shmem<4096, float>(shm);
    else if (n == 1024)
        e = f64 ? gpe_set_shmem<1024, double>(shm) : gpe_set_shmem<1024, float>(shm);
    else
        e = f64 ? gpe_set_shmem<64, double>(shm) : gpe_set_shmem<64, float>(shm);
    if (e != hipSuccess) return ISM_E_DEVICE;
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
    if (o.step_map != ISM_STEP_EXP) return ISM_E_UNSUPPORTED;   // the condensate uses Eq. (OS)
    if (n_grid != 64 && n_grid != 1024 && n_grid != 4096)
        return n_grid > 0 ? ISM_E_UNSUPPORTED : ISM_E_ARG;
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
