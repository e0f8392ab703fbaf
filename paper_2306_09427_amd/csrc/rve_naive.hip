// Plain FP64 one-RVE-at-a-time engine (the "naive" GPU approach of
// Section 4.2): the RVEs of a batch are relaxed one after another; every
// relaxation iteration is a sequence of separate launches (half-step update,
// zero the force vector, scatter fiber forces to nodes with atomics, node
// update with block reductions, boundary reaction norm), and the host reads
// the reduced scalars back after every iteration to take the time step and
// the convergence decision.  Same mathematics as the persistent kernels, in
// double precision; it is the baseline the batched engines are measured
// against.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rve_batch.h"
#include "rve_internal.h"

namespace rve {
namespace naive {

constexpr int NT = 256;

__device__ inline void law(int lw, double EA, double B, double eps, double& T, double& kt)
{
    if (lw != 0 && eps >= 0.0) {
        double em1 = expm1(B * eps);
        T = EA * em1 / B;
        kt = EA * (em1 + 1.0);
    } else {
        T = EA * eps;
        kt = EA;
    }
}

__global__ void prep(SolveArgs A, int r, double* D0q, double* h, double* v, double* M)
{
    const DevNet& n = A.net;
    const int64_t f0 = n.fib_off[r], nfib = n.fib_off[r + 1] - f0;
    const int64_t a0 = n.free_off[r], nf = n.free_off[r + 1] - a0;
    const double* F = A.F + 9 * r;
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < nfib) {
        const double* d0 = n.d0 + 3 * (f0 + t);
        double L0 = n.L0[f0 + t];
        double Dx = F[0] * d0[0] + F[1] * d0[1] + F[2] * d0[2];
        double Dy = F[3] * d0[0] + F[4] * d0[1] + F[5] * d0[2];
        double Dz = F[6] * d0[0] + F[7] * d0[1] + F[8] * d0[2];
        D0q[4 * t] = Dx;
        D0q[4 * t + 1] = Dy;
        D0q[4 * t + 2] = Dz;
        D0q[4 * t + 3] = (Dx * Dx + Dy * Dy + Dz * Dz) - L0 * L0;
    }
    if (t <= nf) {
        for (int c = 0; c < 3; ++c) {
            h[3 * t + c] = (t < nf && A.init == 2) ? A.h_state[3 * (a0 + t) + c] : 0.0;
            if (t < nf) v[3 * t + c] = 0.0;
        }
        if (t < nf) M[t] = n.mass[a0 + t] * A.rhoA;
    }
}

__global__ void zero(double* f, double* G, int64_t nn)
{
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < nn) {
        f[3 * t] = f[3 * t + 1] = f[3 * t + 2] = 0.0;
        G[t] = 0.0;
    }
}

__global__ void fibers(SolveArgs A, int r, const double* D0q, const double* h, double* f, double* G)
{
    const DevNet& n = A.net;
    const int64_t f0 = n.fib_off[r], nfib = n.fib_off[r + 1] - f0;
    const int64_t nf = n.free_off[r + 1] - n.free_off[r];
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nfib) return;
    uint32_t e = n.ends[f0 + k];
    int i = e & 0xffff, j = e >> 16;
    int hi = i < nf ? i : (int)nf, hj = j < nf ? j : (int)nf;
    double dh[3] = {h[3 * hj] - h[3 * hi], h[3 * hj + 1] - h[3 * hi + 1], h[3 * hj + 2] - h[3 * hi + 2]};
    const double* D = D0q + 4 * k;
    double L0 = n.L0[f0 + k];
    double d[3] = {D[0] + dh[0], D[1] + dh[1], D[2] + dh[2]};
    double q = D[3] + (2.0 * (D[0] * dh[0] + D[1] * dh[1] + D[2] * dh[2]) + (dh[0] * dh[0] + dh[1] * dh[1] + dh[2] * dh[2]));
    double l = sqrt(L0 * L0 + q);
    double eps = q / (L0 * (l + L0));
    double T, kt;
    law(A.law, A.EA, A.B, eps, T, kt);
    double g = T / l;
    double b = fmax(kt / L0, fabs(g));
    for (int c = 0; c < 3; ++c) {
        atomicAdd(&f[3 * j + c], g * d[c]);
        atomicAdd(&f[3 * i + c], -g * d[c]);
    }
    atomicAdd(&G[i], 2.0 * b);
    atomicAdd(&G[j], 2.0 * b);
}

__device__ inline double block_sum(double v, double* sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    __syncthreads();
    return s;
}

__device__ inline double block_max(double v, double* sh)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = fmax(s, sh[w]);
    __syncthreads();
    return s;
}

// red: [0] max G/M (as ordered bits), [1] |f_free|^2, [2] |c M v|^2, [3] |f_bnd|^2
__global__ void nodes(SolveArgs A, int r, const double* f, const double* G, double* v, double* a, double* M,
                      double hdt, int first, int check, double* red)
{
    __shared__ double sh[16];
    const DevNet& n = A.net;
    const int64_t nf = n.free_off[r + 1] - n.free_off[r];
    const double c = A.c[r];
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double gm = 0.0, r2 = 0.0, d2 = 0.0;
    if (t < nf) {
        if (first && A.mass_mode == 1) M[t] = G[t] > 0.0 ? G[t] / 4.0 : 1.0;
        double m = M[t];
        for (int k = 0; k < 3; ++k) {
            double ak = first ? -f[3 * t + k] / m : -f[3 * t + k] / m - c * v[3 * t + k];
            a[3 * t + k] = ak;
            if (!first) v[3 * t + k] += hdt * ak;
            r2 += f[3 * t + k] * f[3 * t + k];
            double p = c * m * v[3 * t + k];
            d2 += p * p;
        }
        gm = G[t] / m;
    }
    gm = block_max(gm, sh);
    if (check) {
        r2 = block_sum(r2, sh);
        d2 = block_sum(d2, sh);
    }
    if (threadIdx.x == 0) {
        atomicMax(reinterpret_cast<unsigned long long*>(&red[0]), (unsigned long long)__double_as_longlong(gm));
        if (check) {
            atomicAdd(&red[1], r2);
            atomicAdd(&red[2], d2);
        }
    }
}

__global__ void bnorm(SolveArgs A, int r, const double* f, double* red)
{
    __shared__ double sh[16];
    const DevNet& n = A.net;
    const int64_t nf = n.free_off[r + 1] - n.free_off[r], nb = n.bnd_off[r + 1] - n.bnd_off[r];
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double s = 0.0;
    if (t < nb) {
        const double* fb = f + 3 * (nf + t);
        s = fb[0] * fb[0] + fb[1] * fb[1] + fb[2] * fb[2];
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) atomicAdd(&red[3], s);
}

__global__ void step(double* h, double* v, const double* a, double dt, int64_t nf)
{
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < 3 * nf) {
        v[t] += 0.5 * dt * a[t];
        h[t] += dt * v[t];
    }
}

// sigma = 1/(J V0) sum_b f_b x_b^T, one block, compensated per-thread sums
__global__ void stress(SolveArgs A, int r, const double* f, double J)
{
    __shared__ double sh[16];
    const DevNet& n = A.net;
    const int64_t nf = n.free_off[r + 1] - n.free_off[r], b0 = n.bnd_off[r], nb = n.bnd_off[r + 1] - b0;
    const double* F = A.F + 9 * r;
    double s[9] = {0}, cc[9] = {0};
    for (int64_t t = threadIdx.x; t < nb; t += blockDim.x) {
        const double* Xm = n.Xb + 3 * (b0 + t);
        const double* fb = f + 3 * (nf + t);
        double x[3] = {F[0] * Xm[0] + F[1] * Xm[1] + F[2] * Xm[2], F[3] * Xm[0] + F[4] * Xm[1] + F[5] * Xm[2],
                       F[6] * Xm[0] + F[7] * Xm[1] + F[8] * Xm[2]};
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
                double y = fb[p] * x[q], u = s[3 * p + q] + y;
                cc[3 * p + q] += fabs(s[3 * p + q]) >= fabs(y) ? (s[3 * p + q] - u) + y : (y - u) + s[3 * p + q];
                s[3 * p + q] = u;
            }
    }
    for (int p = 0; p < 9; ++p) {
        double tot = block_sum(s[p], sh) + block_sum(cc[p], sh);
        if (threadIdx.x == 0) A.sigma[9 * r + p] = tot / (J * n.V0[r]);
    }
}

__global__ void finish(SolveArgs A, int r, const double* h, int status, int64_t it, double R, double D, double Bn)
{
    const DevNet& n = A.net;
    const int64_t a0 = n.free_off[r], nf = n.free_off[r + 1] - a0;
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < 3 * nf && status != 3) A.h_state[3 * a0 + t] = h[t];
    if (t == 0) {
        A.status[r] = status;
        A.iters[r] = it;
        A.Rres[r] = R;
        A.Dres[r] = D;
        A.Bres[r] = Bn;
        if (status == 2 || status == 3)
            for (int k = 0; k < 9; ++k) A.sigma[9 * r + k] = NAN;
    }
}

static inline int blocks(int64_t n) { return (int)((n + NT - 1) / NT); }

}  // namespace naive
hipError_t naive_fixed_private(size_t* bytes)
{
    return max_private_bytes({(const void*)naive::prep, (const void*)naive::zero, (const void*)naive::fibers,
                              (const void*)naive::nodes, (const void*)naive::bnorm, (const void*)naive::step,
                              (const void*)naive::stress, (const void*)naive::finish},
                             bytes);
}

}  // namespace rve

using namespace rve;

int rve_naive_run(const SolveArgs& A, const std::vector<int64_t>& fib_off,
                               const std::vector<int64_t>& free_off, const std::vector<int64_t>& bnd_off,
                               const std::vector<double>& F, const std::vector<double>& c, hipStream_t s,
                               std::string* err)
{
    using namespace rve::naive;
    const int64_t R = (int64_t)fib_off.size() - 1;
    int64_t mfib = 1, mnn = 1, mnf = 1;
    for (int64_t r = 0; r < R; ++r) {
        int64_t nfib = fib_off[r + 1] - fib_off[r], nf = free_off[r + 1] - free_off[r];
        int64_t nn = nf + bnd_off[r + 1] - bnd_off[r];
        mfib = std::max(mfib, nfib);
        mnn = std::max(mnn, nn);
        mnf = std::max(mnf, nf);
    }
    double *D0q = nullptr, *h = nullptr, *v = nullptr, *a = nullptr, *f = nullptr, *G = nullptr, *M = nullptr,
           *red = nullptr, *hred = nullptr;
    size_t bytes = 8 * (4 * mfib + 3 * (mnf + 1) + 3 * mnf + 3 * mnf + 3 * mnn + mnn + mnf + 8);
    char* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) {
        *err = "naive engine: device allocation failed";
        return RVE_ENOMEM;
    }
    if (hipHostMalloc(&hred, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(mem);
        *err = "naive engine: pinned allocation failed";
        return RVE_ENOMEM;
    }
    double* p = reinterpret_cast<double*>(mem);
    D0q = p; p += 4 * mfib;
    h = p; p += 3 * (mnf + 1);
    v = p; p += 3 * mnf;
    a = p; p += 3 * mnf;
    f = p; p += 3 * mnn;
    G = p; p += mnn;
    M = p; p += mnf;
    red = p;
    int rc = RVE_OK;
    auto chk = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == RVE_OK) {
            rc = RVE_EDEVICE;
            *err = std::string("naive engine: ") + what + ": " + hipGetErrorString(e);
        }
        return e == hipSuccess;
    };
    auto fetch = [&](bool check) -> bool {
        if (!chk(hipMemcpyAsync(hred, red, 4 * sizeof(double), hipMemcpyDeviceToHost, s), "readback")) return false;
            (void)check;
        return chk(hipStreamSynchronize(s), "sync");
    };
    for (int64_t r = 0; r < R && rc == RVE_OK; ++r) {
        const double* Fr = &F[9 * r];
        double J = Fr[0] * (Fr[4] * Fr[8] - Fr[5] * Fr[7]) - Fr[1] * (Fr[3] * Fr[8] - Fr[5] * Fr[6]) +
                   Fr[2] * (Fr[3] * Fr[7] - Fr[4] * Fr[6]);
        bool finite = true;
        for (int k = 0; k < 9; ++k) finite = finite && std::isfinite(Fr[k]);
        const int64_t nfib = fib_off[r + 1] - fib_off[r], nf = free_off[r + 1] - free_off[r];
        const int64_t nb = bnd_off[r + 1] - bnd_off[r], nn = nf + nb;
        if (!finite || !(J > 0)) {
            hipLaunchKernelGGL(finish, dim3(1), dim3(NT), 0, s, A, (int)r, h, 3, (int64_t)0, NAN, NAN, NAN);
            chk(hipGetLastError(), "finish");
            continue;
        }
        hipLaunchKernelGGL(prep, dim3(blocks(std::max(nfib, nf + 1))), dim3(NT), 0, s, A, (int)r, D0q, h, v, M);
        auto force_and_reduce = [&](bool first, bool check, double hdt) {
            hipLaunchKernelGGL(zero, dim3(blocks(nn)), dim3(NT), 0, s, f, G, nn);
            if (nfib) hipLaunchKernelGGL(fibers, dim3(blocks(nfib)), dim3(NT), 0, s, A, (int)r, D0q, h, f, G);
            chk(hipMemsetAsync(red, 0, 4 * sizeof(double), s), "memset");
            hipLaunchKernelGGL(nodes, dim3(blocks(std::max<int64_t>(nf, 1))), dim3(NT), 0, s, A, (int)r, f, G, v, a,
                               M, hdt, first ? 1 : 0, check ? 1 : 0, red);
            if (check) hipLaunchKernelGGL(bnorm, dim3(blocks(std::max<int64_t>(nb, 1))), dim3(NT), 0, s, A, (int)r, f, red);
            chk(hipGetLastError(), "launch");
        };
        force_and_reduce(true, true, 0.0);
        if (!fetch(true)) break;
        double gmax = hred[0], Rn = std::sqrt(hred[1]), Dn = 0.0, Bn = std::sqrt(hred[3]);
        double tol = std::max(A.tol_abs, A.tol_rel * Bn);
        int64_t n = 0;
        int status = 0;
        const int ce = A.check_every > 0 ? A.check_every : 1;
        bool done = Rn <= tol;
        if (!std::isfinite(Rn)) {
            status = 2;
            done = true;
        }
        if (!done && n >= A.n_max) {
            status = 1;
            done = true;
        }
        while (!done && rc == RVE_OK) {
            double dt = A.alpha * 2.0 / std::sqrt(gmax);
            hipLaunchKernelGGL(step, dim3(blocks(3 * std::max<int64_t>(nf, 1))), dim3(NT), 0, s, h, v, a, dt, nf);
            ++n;
            const bool check = (n % ce) == 0;
            force_and_reduce(false, check, 0.5 * dt);
            if (!fetch(check)) break;
            gmax = hred[0];
            if (check) {
                Rn = std::sqrt(hred[1]);
                Dn = std::sqrt(hred[2]);
                Bn = std::sqrt(hred[3]);
                tol = std::max(A.tol_abs, A.tol_rel * Bn);
                if (!std::isfinite(Rn) || !std::isfinite(Dn)) {
                    status = 2;
                    break;
                }
                if (Rn <= tol && Dn <= tol) break;
            }
            if (!(gmax > 0) || !std::isfinite(gmax)) {
                status = 2;
                break;
            }
            if (n >= A.n_max) {
                status = 1;
                break;
            }
        }
        if (rc != RVE_OK) break;
        if (status != 2) hipLaunchKernelGGL(stress, dim3(1), dim3(NT), 0, s, A, (int)r, f, J);
        hipLaunchKernelGGL(finish, dim3(blocks(3 * std::max<int64_t>(nf, 1))), dim3(NT), 0, s, A, (int)r, h, status, n,
                           Rn, Dn, Bn);
        chk(hipGetLastError(), "stress/finish");
    }
    chk(hipStreamSynchronize(s), "final sync");
    (void)hipFree(mem);
    (void)hipHostFree(hred);
    (void)c;
    return rc;
}
