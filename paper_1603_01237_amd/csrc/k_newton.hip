// Newton slice solver (Sec. 4.B): Step (c) of Algorithm 1 as one Newton step per slice
// problem, the Newton system A_n delta_n = -G_n solved matrix-free by m GMRES steps, with
// A_n v the central difference of slice gradients (G_n(u + eps v) - G_n(u - eps v)) / 2 eps
// at the held intermediate states.  Every slice of every instance runs its own GMRES in
// lockstep: the vectors are laid out as the controls (B x K x C, FP64), and the slice
// reductions (one workgroup per (instance, slice), fixed-order tree) give the per-slice
// Arnoldi coefficients, which stay on the device.  The host sequences the launches
// (ism_newton.cpp); the gradients come from the path's own slice kernels.
#include <math.h>

#include <algorithm>

#include "ism_internal.h"
#include "ism_paths.h"

namespace ism {
namespace {

constexpr int NWT = 256;

// out[(b N + n) * ostride] = sum over slice n of instance b of x * y
__global__ __launch_bounds__(NWT) void k_nw_dot(const double* x, const double* y, const int* s,
                                                int K, int N, int C, double* out, int ostride) {
    __shared__ double red[NWT];
    const int n = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    const size_t off = ((size_t)b * K + s[n]) * C;
    const int len = (s[n + 1] - s[n]) * C;
    double acc = 0.0;
    for (int i = t; i < len; i += NWT) acc = fma(x[off + i], y[off + i], acc);
    red[t] = acc;
    __syncthreads();
    for (int w = NWT / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[((size_t)b * N + n) * ostride] = red[0];
}

// y -= coef[(b N + n) * cstride] x on slice n of instance b
__global__ __launch_bounds__(NWT) void k_nw_sub(double* y, const double* x, const int* s, int K,
                                                int N, int C, const double* coef, int cstride) {
    const int n = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    const size_t off = ((size_t)b * K + s[n]) * C;
    const int len = (s[n + 1] - s[n]) * C;
    const double a = coef[((size_t)b * N + n) * cstride];
    for (int i = t; i < len; i += NWT) y[off + i] = fma(-a, x[off + i], y[off + i]);
}

// y = sign x / sqrt(nn) on every slice; nrm[(b N + n) * nstride] = sqrt(nn).  A slice whose
// norm is at most 1e-14 of the reference norm (ref, nullable) has broken down: its kdim is
// set to `it` (if not set before) and y is zero there.
__global__ __launch_bounds__(NWT) void k_nw_normalize(double* y, const double* x, const int* s,
                                                      int K, int N, int C, const double* nn,
                                                      double* nrm, int nstride, const double* ref,
                                                      double sign, int* kdim, int it) {
    const int n = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    const size_t sl = (size_t)b * N + n;
    const size_t off = ((size_t)b * K + s[n]) * C;
    const int len = (s[n + 1] - s[n]) * C;
    const double v = sqrt(fmax(nn[sl], 0.0));
    bool broken = kdim[sl] >= 0 || !(v > 0.0);
    if (ref && !(v > 1e-14 * sqrt(fmax(ref[sl], 0.0)))) broken = true;
    const double sc = broken ? 0.0 : sign / v;
    for (int i = t; i < len; i += NWT) y[off + i] = sc * x[off + i];
    if (t == 0) {
        nrm[sl * nstride] = v;
        if (broken && kdim[sl] < 0) kdim[sl] = it;
    }
}

// u = u0 + a v (every entry)
__global__ void k_nw_lincomb(double* u, const double* u0, const double* v, double a, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        u[i] = fma(a, v[i], u0[i]);
}

// w = (gp - gm) * h (every entry)
__global__ void k_nw_diff(double* w, const double* gp, const double* gm, double h, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        w[i] = (gp[i] - gm[i]) * h;
}

// Per slice (one thread each): the least-squares problem min || beta e1 - H y || of the
// (k+1) x k Hessenberg matrix (k = kdim, or m without a breakdown), by Givens rotations and
// back substitution, in place on the slice's H (column-major, leading dimension m + 1).
__global__ void k_nw_lsq(double* Hs, const double* beta, const int* kdim, int m, int nslices,
                         double* y) {
    const int sl = blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= nslices) return;
    double g[kNewtonMaxM + 1];
    const int k = kdim[sl] >= 0 ? kdim[sl] : m;
    double* H = Hs + (size_t)sl * (m + 1) * m;
    auto R = [&](int r, int c) -> double& { return H[(size_t)c * (m + 1) + r]; };
    for (int r = 0; r <= m; ++r) g[r] = 0.0;
    g[0] = beta[sl];
    for (int c = 0; c < k; ++c) {
        const double a = R(c, c), bb = R(c + 1, c);
        const double rr = hypot(a, bb);
        const double cs = rr > 0.0 ? a / rr : 1.0, sn = rr > 0.0 ? bb / rr : 0.0;
        for (int cc = c; cc < k; ++cc) {
            const double x0 = R(c, cc), x1 = R(c + 1, cc);
            R(c, cc) = cs * x0 + sn * x1;
            R(c + 1, cc) = -sn * x0 + cs * x1;
        }
        const double g0 = g[c], g1 = g[c + 1];
        g[c] = cs * g0 + sn * g1;
        g[c + 1] = -sn * g0 + cs * g1;
    }
    double* yo = y + (size_t)sl * m;
    for (int c = k - 1; c >= 0; --c) {
        double acc = g[c];
        for (int cc = c + 1; cc < k; ++cc) acc -= R(c, cc) * yo[cc];
        yo[c] = R(c, c) != 0.0 ? acc / R(c, c) : 0.0;
    }
    for (int c = k; c < m; ++c) yo[c] = 0.0;
}

// u += sum_l y_l V_l on every slice of the active instances (delta_n = V y)
__global__ __launch_bounds__(NWT) void k_nw_apply(double* u, const double* V, size_t vstride,
                                                  const int* s, int K, int N, int C,
                                                  const double* y, int m, const int* active) {
    const int n = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
    if (active && !active[b]) return;
    const size_t sl = (size_t)b * N + n;
    const size_t off = ((size_t)b * K + s[n]) * C;
    const int len = (s[n + 1] - s[n]) * C;
    for (int i = t; i < len; i += NWT) {
        double d = 0.0;
        for (int l = 0; l < m; ++l) d = fma(y[sl * m + l], V[l * vstride + off + i], d);
        u[off + i] += d;
    }
}

inline dim3 grid1(size_t n) { return dim3((unsigned)std::min<size_t>((n + 255) / 256, 65535)); }

}  // namespace

hipError_t nw_dot(const double* x, const double* y, const int* s, int B, int K, int N, int C,
                  double* out, int ostride, hipStream_t st) {
    hipLaunchKernelGGL(k_nw_dot, dim3(N, B), dim3(NWT), 0, st, x, y, s, K, N, C, out, ostride);
    return hipGetLastError();
}

hipError_t nw_sub(double* y, const double* x, const int* s, int B, int K, int N, int C,
                  const double* coef, int cstride, hipStream_t st) {
    hipLaunchKernelGGL(k_nw_sub, dim3(N, B), dim3(NWT), 0, st, y, x, s, K, N, C, coef, cstride);
    return hipGetLastError();
}

hipError_t nw_normalize(double* y, const double* x, const int* s, int B, int K, int N, int C,
                        const double* nn, double* nrm, int nstride, const double* ref,
                        double sign, int* kdim, int it, hipStream_t st) {
    hipLaunchKernelGGL(k_nw_normalize, dim3(N, B), dim3(NWT), 0, st, y, x, s, K, N, C, nn, nrm,
                       nstride, ref, sign, kdim, it);
    return hipGetLastError();
}

hipError_t nw_lincomb(double* u, const double* u0, const double* v, double a, size_t n,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_nw_lincomb, grid1(n), dim3(256), 0, st, u, u0, v, a, n);
    return hipGetLastError();
}

hipError_t nw_diff(double* w, const double* gp, const double* gm, double h, size_t n,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_nw_diff, grid1(n), dim3(256), 0, st, w, gp, gm, h, n);
    return hipGetLastError();
}

hipError_t nw_lsq(double* H, const double* beta, const int* kdim, int m, int nslices, double* y,
                  hipStream_t st) {
    hipLaunchKernelGGL(k_nw_lsq, dim3((nslices + 63) / 64), dim3(64), 0, st, H, beta, kdim, m,
                       nslices, y);
    return hipGetLastError();
}

hipError_t nw_apply(double* u, const double* V, size_t vstride, const int* s, int B, int K,
                    int N, int C, const double* y, int m, const int* active, hipStream_t st) {
    hipLaunchKernelGGL(k_nw_apply, dim3(N, B), dim3(NWT), 0, st, u, V, vstride, s, K, N, C, y, m,
                       active);
    return hipGetLastError();
}

}  // namespace ism
