// Fiber-orientation outputs of each RVE at the state of the last solve: the
// orientation tensor <n n^T> and the degree of alignment <(3 (n.e)^2 - 1)/2>
// (second Legendre polynomial of the angle to the reference direction e),
// averages over the fibers of the unit current direction n (Section 6,
// degree of alignment; Section 4, orientation data sent to the macroscale).
// One workgroup per RVE, FP64, fixed summation order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rve_internal.h"

namespace rve {

namespace {

constexpr int kOrientThreads = 256;
constexpr int ST_NONFINITE = 2, ST_BAD_F = 3;

template <typename T>
__device__ __forceinline__ T wave_sum64(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(kOrientThreads) void orientation_kernel(OrientArgs A)
{
    __shared__ double part[7][kOrientThreads / 64];
    const int r = blockIdx.x;
    const DevNet& net = A.net;
    const int64_t f0 = net.fib_off[r], nfib = net.fib_off[r + 1] - f0;
    const int64_t a0 = net.free_off[r], nf = net.free_off[r + 1] - a0;
    const int st = A.status[r];
    if (st == ST_NONFINITE || st == ST_BAD_F || nfib == 0) {
        if (threadIdx.x < 9) A.omega[9 * r + threadIdx.x] = NAN;
        if (threadIdx.x == 0) A.p2[r] = NAN;
        return;
    }
    double F[9];
    for (int k = 0; k < 9; ++k) F[k] = A.F[9 * r + k];
    // xx, xy, xz, yy, yz, zz, P2
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (int64_t k = threadIdx.x; k < nfib; k += kOrientThreads) {
        const double* d0 = net.d0 + 3 * (f0 + k);
        const uint32_t e = net.ends[f0 + k];
        const int64_t i = e & 0xffff, j = e >> 16;
        double d[3];
        for (int p = 0; p < 3; ++p) {
            d[p] = F[3 * p] * d0[0] + F[3 * p + 1] * d0[1] + F[3 * p + 2] * d0[2];
            if (j < nf) d[p] += A.h_state[3 * (a0 + j) + p];
            if (i < nf) d[p] -= A.h_state[3 * (a0 + i) + p];
        }
        const double il = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double n0 = d[0] * il, n1 = d[1] * il, n2 = d[2] * il;
        s[0] += n0 * n0;
        s[1] += n0 * n1;
        s[2] += n0 * n2;
        s[3] += n1 * n1;
        s[4] += n1 * n2;
        s[5] += n2 * n2;
        const double c = n0 * A.e[0] + n1 * A.e[1] + n2 * A.e[2];
        s[6] += 0.5 * (3.0 * c * c - 1.0);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const double w = wave_sum64(s[q]);
        if (lane == 0) part[q][wave] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[7];
        for (int q = 0; q < 7; ++q) {
            t[q] = 0.0;
            for (int w = 0; w < kOrientThreads / 64; ++w) t[q] += part[q][w];
            t[q] /= (double)nfib;
        }
        double* o = A.omega + 9 * r;
        o[0] = t[0]; o[1] = t[1]; o[2] = t[2];
        o[3] = t[1]; o[4] = t[3]; o[5] = t[4];
        o[6] = t[2]; o[7] = t[4]; o[8] = t[5];
        A.p2[r] = t[6];
    }
}

}  // namespace

hipError_t launch_orientation(const OrientArgs& a, int64_t n_rve, hipStream_t s)
{
    if (n_rve <= 0) return hipSuccess;
    hipLaunchKernelGGL(orientation_kernel, dim3((unsigned)n_rve), dim3(kOrientThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t orient_fixed_private(size_t* bytes)
{
    return max_private_bytes({(const void*)orientation_kernel}, bytes);
}

}  // namespace rve
