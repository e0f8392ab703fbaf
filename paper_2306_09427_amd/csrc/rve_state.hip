// Export and import of a batch's relaxation state (checkpoint and restart,
// warm starts carried across batches): the free-node fluctuation h moves
// between the packed free-first order of the device and the caller's node
// order through a per-node map (packed global free index, or -1 for a
// boundary node), and imported per-RVE statuses are re-checked against F
// (Algorithm "Dynamic Relaxation" starts an increment from the last
// converged state; Algorithm 1 keeps that state per integration point).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rve_internal.h"

namespace rve {

namespace {

constexpr int kStateThreads = 256;
constexpr int ST_NONFINITE = 2, ST_BAD_F = 3, ST_STAGNATED = 8;

__global__ __launch_bounds__(kStateThreads) void export_h_kernel(const double* __restrict__ dh,
                                                                  const int32_t* __restrict__ map, int64_t nn,
                                                                  double* __restrict__ out)
{
    const int64_t n = (int64_t)blockIdx.x * kStateThreads + threadIdx.x;
    if (n >= nn) return;
    const int32_t q = map[n];
    for (int c = 0; c < 3; ++c) out[3 * n + c] = q >= 0 ? dh[3 * (int64_t)q + c] : 0.0;
}

__global__ __launch_bounds__(kStateThreads) void import_h_kernel(const double* __restrict__ in,
                                                                  const int32_t* __restrict__ map, int64_t nn,
                                                                  double* __restrict__ dh)
{
    const int64_t n = (int64_t)blockIdx.x * kStateThreads + threadIdx.x;
    if (n >= nn) return;
    const int32_t q = map[n];
    if (q < 0) return;
    for (int c = 0; c < 3; ++c) dh[3 * (int64_t)q + c] = in[3 * n + c];
}

// Imported statuses: codes other than CONVERGED..BAD_F and STAGNATED become
// NONFINITE (no usable state); a non-finite F or det F <= 0 becomes BAD_F.  st_in may be
// st itself (each thread reads its entry before writing it).  The stored
// diagnostics of the imported state are unknown: iterations 0, norms NaN.
__global__ __launch_bounds__(kStateThreads) void import_status_kernel(const double* __restrict__ F,
                                                                       const int32_t* st_in, int64_t R,
                                                                       int32_t* st, int64_t* iters, double* Rn,
                                                                       double* Dn, double* Bn)
{
    const int64_t r = (int64_t)blockIdx.x * kStateThreads + threadIdx.x;
    if (r >= R) return;
    int s = st_in[r];
    if (!((s >= 0 && s <= ST_BAD_F) || s == ST_STAGNATED)) s = ST_NONFINITE;
    const double* f = F + 9 * r;
    bool finite = true;
    for (int k = 0; k < 9; ++k) finite = finite && isfinite(f[k]);
    const double J = f[0] * (f[4] * f[8] - f[5] * f[7]) - f[1] * (f[3] * f[8] - f[5] * f[6]) +
                     f[2] * (f[3] * f[7] - f[4] * f[6]);
    if (!finite || !(J > 0.0)) s = ST_BAD_F;
    st[r] = s;
    iters[r] = 0;
    Rn[r] = NAN;
    Dn[r] = NAN;
    Bn[r] = NAN;
}

// Reference start (RVE_INIT_REFERENCE): free node a of RVE r at its
// reference position Xm_a, i.e. the fluctuation h_a = Xm_a - F Xm_a; one
// workgroup per RVE.
__global__ __launch_bounds__(kStateThreads) void reference_h_kernel(const double* __restrict__ F,
                                                                     const int64_t* __restrict__ free_off,
                                                                     const double* __restrict__ xm, double* dh)
{
    const int64_t r = blockIdx.x;
    const int64_t a0 = free_off[r], nf = free_off[r + 1] - a0;
    const double* Fr = F + 9 * r;
    for (int64_t a = threadIdx.x; a < nf; a += kStateThreads) {
        const double* X = xm + 3 * (a0 + a);
        double* h = dh + 3 * (a0 + a);
        for (int i = 0; i < 3; ++i) {
            const double y = Fr[3 * i] * X[0] + Fr[3 * i + 1] * X[1] + Fr[3 * i + 2] * X[2];
            h[i] = isfinite(y) ? X[i] - y : 0.0;
        }
    }
}

inline unsigned grid_of(int64_t n)
{
    return (unsigned)((n + kStateThreads - 1) / kStateThreads);
}

}  // namespace

hipError_t launch_export_h(const double* dh, const int32_t* map, int64_t nn, double* out, hipStream_t s)
{
    if (nn <= 0) return hipSuccess;
    hipLaunchKernelGGL(export_h_kernel, dim3(grid_of(nn)), dim3(kStateThreads), 0, s, dh, map, nn, out);
    return hipGetLastError();
}

hipError_t launch_import_h(const double* in, const int32_t* map, int64_t nn, double* dh, hipStream_t s)
{
    if (nn <= 0) return hipSuccess;
    hipLaunchKernelGGL(import_h_kernel, dim3(grid_of(nn)), dim3(kStateThreads), 0, s, in, map, nn, dh);
    return hipGetLastError();
}

hipError_t launch_import_status(const double* F, const int32_t* st_in, int64_t R, int32_t* st, int64_t* iters,
                                double* Rn, double* Dn, double* Bn, hipStream_t s)
{
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL(import_status_kernel, dim3(grid_of(R)), dim3(kStateThreads), 0, s, F, st_in, R, st, iters, Rn,
                       Dn, Bn);
    return hipGetLastError();
}

hipError_t launch_reference_h(const double* F, const int64_t* free_off, const double* xm, int64_t R, double* dh,
                              hipStream_t s)
{
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL(reference_h_kernel, dim3((unsigned)R), dim3(kStateThreads), 0, s, F, free_off, xm, dh);
    return hipGetLastError();
}

hipError_t state_fixed_private(size_t* bytes)
{
    return max_private_bytes({(const void*)export_h_kernel, (const void*)import_h_kernel, (const void*)reference_h_kernel,
                              (const void*)import_status_kernel},
                             bytes);
}

}  // namespace rve
