// Stand-alone batched Hines solve of caller-given tree systems on the
// device: the cable system of Eq. 4 (Sec. 2.4) of many cells at once, each
// cell's matrix symmetric with one off-diagonal entry per CV coupling it to
// its parent (Hines 1989).  Two entry points share one kernel: one takes its
// elimination workspace from hipMalloc for the call, the other from a
// file-scope device array, for callers that cannot allocate.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "../../include/plasticarbor.h"

namespace pa {
namespace {

// Largest n_cv of one call of the variant without allocation: its workspace
// (the eliminated diagonal and right-hand side, 16 bytes per CV) is this
// array, 16 MiB per device.
constexpr uint64_t NOALLOC_MAX_CV = 1ull << 20;

__device__ __align__(256) double scratch[2 * NOALLOC_MAX_CV];

// One lane per cell.  The cell's CVs are cv_off[c] .. cv_off[c+1]-1 with
// cell-local parents (parent of the first CV -1, else 0 <= parent[i] < i).
// Elimination from the last CV towards the root, then substitution from the
// root, in the order of the sequential algorithm; the eliminated diagonal
// and right-hand side live in the workspace ws (D at [0, n_cv), b at
// [n_cv, 2 n_cv)), the inputs stay untouched.  A cell whose CV range or
// parents break these rules gets NaN in every x it owns within [0, n_cv).
__global__ void k_tree_solve(uint32_t n_cells, uint64_t n_cv, const int64_t *__restrict__ cv_off,
                             const int32_t *__restrict__ parent, const double *__restrict__ diag,
                             const double *__restrict__ off, const double *__restrict__ rhs,
                             double *__restrict__ x, double *__restrict__ ws) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int64_t a = cv_off[c], b = cv_off[c + 1];
    const bool range_ok = a >= 0 && b >= a && (uint64_t)b <= n_cv;
    if (!range_ok) {
        // write the NaNs only where the cell's range meets [0, n_cv)
        const int64_t lo = a < 0 ? 0 : a;
        const int64_t hi = (b < 0) ? 0 : ((uint64_t)b > n_cv ? (int64_t)n_cv : b);
        for (int64_t i = lo; i < hi; ++i) x[i] = NAN;
        return;
    }
    const int64_t n = b - a;
    if (n == 0) return;
    bool ok = parent[a] == -1;
    for (int64_t i = 1; ok && i < n; ++i) {
        const int32_t p = parent[a + i];
        ok = p >= 0 && p < i;
    }
    if (!ok) {
        for (int64_t i = a; i < b; ++i) x[i] = NAN;
        return;
    }
    double *D = ws + a, *B = ws + n_cv + a;
    for (int64_t i = 0; i < n; ++i) {
        D[i] = diag[a + i];
        B[i] = rhs[a + i];
    }
    const int32_t *par = parent + a;
    const double *U = off + a;
    for (int64_t i = n - 1; i > 0; --i) {
        const int32_t p = par[i];
        const double f = U[i] / D[i];
        D[p] -= f * U[i];
        B[p] -= f * B[i];
    }
    double *X = x + a;
    X[0] = B[0] / D[0];
    for (int64_t i = 1; i < n; ++i) X[i] = (B[i] - U[i] * X[par[i]]) / D[i];
}

pa_status check_args(uint32_t n_cells, uint64_t n_cv, const void *cv_off, const void *parent,
                     const void *diag, const void *off, const void *rhs, const void *x) {
    if (n_cells == 0) return PA_OK;
    if (!cv_off || !parent) return PA_EINVAL;
    if (n_cv > 0 && (!diag || !off || !rhs || !x)) return PA_EINVAL;
    return PA_OK;
}

pa_status launch(uint32_t n_cells, uint64_t n_cv, const int64_t *cv_off, const int32_t *parent,
                 const double *diag, const double *off, const double *rhs, double *x, double *ws,
                 hipStream_t st) {
    const uint32_t bs = 64;
    const uint32_t grid = (uint32_t)(((uint64_t)n_cells + bs - 1) / bs);
    hipLaunchKernelGGL(k_tree_solve, dim3(grid), dim3(bs), 0, st, n_cells, n_cv, cv_off, parent, diag,
                       off, rhs, x, ws);
    return hipGetLastError() == hipSuccess ? PA_OK : PA_EDEVICE;
}

// Device address of `scratch` on each device, taken once per device with
// that device current.
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_ptr[MAX_DEVICES] = {};

pa_status scratch_of_current_device(double **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return PA_EDEVICE;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PA_EDEVICE;
        scratch_ptr[dev] = (double *)p;
    }
    *out = scratch_ptr[dev];
    return PA_OK;
}

}  // namespace
}  // namespace pa

extern "C" pa_status pa_tree_solve(uint32_t n_cells, uint64_t n_cv, const int64_t *cv_off,
                                   const int32_t *parent, const double *diag, const double *off,
                                   const double *rhs, double *x, void *hip_stream) {
    pa_status st = pa::check_args(n_cells, n_cv, cv_off, parent, diag, off, rhs, x);
    if (st != PA_OK || n_cells == 0) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    void *ws = nullptr;
    if (hipMalloc(&ws, 16 * (n_cv > 0 ? n_cv : 1)) != hipSuccess) return PA_ENOMEM;
    st = pa::launch(n_cells, n_cv, cv_off, parent, diag, off, rhs, x, (double *)ws, s);
    // the workspace is released once the solve has run
    const hipError_t e = hipStreamSynchronize(s);
    (void)hipFree(ws);
    if (st == PA_OK && e != hipSuccess) st = PA_EDEVICE;
    return st;
}

extern "C" pa_status pa_tree_solve_noalloc(uint32_t n_cells, uint64_t n_cv, const int64_t *cv_off,
                                           const int32_t *parent, const double *diag, const double *off,
                                           const double *rhs, double *x, void *hip_stream) {
    pa_status st = pa::check_args(n_cells, n_cv, cv_off, parent, diag, off, rhs, x);
    if (st != PA_OK || n_cells == 0) return st;
    if (n_cv > pa::NOALLOC_MAX_CV) return PA_ERANGE;
    double *ws = nullptr;
    st = pa::scratch_of_current_device(&ws);
    if (st != PA_OK) return st;
    return pa::launch(n_cells, n_cv, cv_off, parent, diag, off, rhs, x, ws, (hipStream_t)hip_stream);
}
