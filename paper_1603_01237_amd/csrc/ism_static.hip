// Allocation-free iteration entry point (ism_iterate_static), and two small utility kernels:
// a fill (flags and counters) and a per-instance update counter (serving).
//
// ism_iterate keeps the per-iteration J history that the boundary kernels write in a device
// buffer it grows per handle.  ism_iterate_static runs the same launch sequence with that
// history in `scratch`, a fixed device array of the library: the call itself allocates
// nothing, neither device nor host memory.  Every call on a GPU shares that GPU's copy of the
// array, so calls that overlap on one GPU (different host threads, or streams whose work
// runs concurrently) race on it.
#include <math.h>

#include <algorithm>
#include <mutex>

#include "ism_internal.h"
#include "ism_paths.h"

namespace ism {
namespace {

// the J history of ism_iterate_static: n_iter * batch doubles of the current call
static __device__ __align__(256) double scratch[ISM_STATIC_HIST_MAX];

// Device address of `scratch` on each GPU, taken once per device with that device current.
// In host code `scratch` names a host-side stand-in, not a device address, so the kernels get
// this pointer and never the array's name.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

int scratch_on(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return ISM_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return ISM_E_DEVICE;
        g_scratch[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch[dev];
    return ISM_OK;
}

__global__ void k_fill_i32(int* x, int v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void k_count_active(int* count, const int* active, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) count[i] += active[i] != 0;
}

}  // namespace

hipError_t launch_fill_i32(int* x, int v, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, x, v, n);
    return hipGetLastError();
}

hipError_t launch_count_active(int* count, const int* active, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_active, dim3((n + 255) / 256), dim3(256), 0, st, count, active, n);
    return hipGetLastError();
}

}  // namespace ism

extern "C" int ism_iterate_static(ism_problem* p, int n_iter, double rho, double fid_stop,
                                  double* J_hist, int* iters_done) {
    using namespace ism;
    if (!p || n_iter < 0 || !std::isfinite(rho) || std::isnan(fid_stop)) return ISM_E_ARG;
    if ((size_t)std::max(n_iter, 1) * (size_t)p->B > (size_t)ISM_STATIC_HIST_MAX)
        return ISM_E_BUDGET;
    if (hipSetDevice(p->device) != hipSuccess) return ISM_E_DEVICE;
    double* jbuf = nullptr;
    int st = scratch_on(p->device, &jbuf);
    if (st) return st;
    int done = 0;
    if (small_eligible(p)) {
        if ((st = small_iterate(p, n_iter, rho, fid_stop, jbuf, &done))) return st;
    } else if ((st = iterate_loop(p, n_iter, 1, rho, fid_stop, 0.0, jbuf, nullptr, true, &done))) {
        return st;
    }
    // the rows the loop wrote: J^(k) for k < done, and J^(done) when it stopped early
    const int rows = std::min(n_iter, done + 1);
    if (J_hist && rows > 0) {
        if ((st = copy_out(p, J_hist, jbuf, (size_t)rows * p->B * sizeof(double)))) return st;
    }
    if (iters_done) *iters_done = done;
    return ISM_OK;
}
