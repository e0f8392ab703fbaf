// Dynamic relaxation with the alternatives to constant viscous damping that
// the paper names (Section 3.2): kinetic damping (no viscous force, every
// velocity set to zero once the kinetic energy has passed a peak), a damping
// coefficient re-estimated each step as the critical damping of the
// Rayleigh quotient of the displacement since the start (c = 2 sqrt(u.Ku /
// u.Mu), K the tangent stiffness at the current positions), and the
// optional energy-balance check of the two-step central difference (stored
// energy W, kinetic energy KE and damping work Wd add up to the starting
// stored energy when the boundary is held fixed; a violation beyond
// energy_tol of the largest of them ends the RVE with RVE_ST_ENERGY).
//
// FP64 throughout, one 256-thread workgroup per RVE, state in a global
// workspace (per free node h, v, a, f, h_start, M, G; per fiber the force
// vector, the Gershgorin term and the stored energy).  Convergence and the
// kinetic-energy peak are tested every iteration; the stress is left to the
// stress kernel of the ordinary solve, which reads the final state.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rve_internal.h"

namespace rve {

namespace {

constexpr int kVT = 256;
constexpr int kWaves = kVT / 64;
constexpr int ST_CONVERGED = 0, ST_MAXITER = 1, ST_NONFINITE = 2, ST_BAD_F = 3, ST_ENERGY = 7;
constexpr int LAW_EXP = 1, MASS_SCALED = 1, INIT_WARM = 2;
constexpr int DAMP_KINETIC = 1, DAMP_ADAPTIVE = 2;
constexpr int kNodeDoubles = 17;   // h 3, v 3, a 3, f 3, h_start 3, M, G
constexpr int kFibDoubles = 5;     // force vector 3, Gershgorin term, stored energy

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Sums of N values over the workgroup (value k of every thread), and one
// maximum, in a fixed order: wave sums, then the waves in order.  Every
// thread receives the results.
template <int N>
__device__ __forceinline__ void block_reduce(double (&v)[N], double& mx, double (*lds)[kWaves], double* lds_max)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
    mx = wave_max(mx);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) lds[k][w] = v[k];
        lds_max[w] = mx;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double t = 0.0;
        for (int q = 0; q < kWaves; ++q) t += lds[k][q];
        v[k] = t;
    }
    double m = lds_max[0];
    for (int q = 1; q < kWaves; ++q) m = fmax(m, lds_max[q]);
    mx = m;
    __syncthreads();
}

struct Law {
    int law;
    double EA, B;
    // axial force, its strain derivative and the stored energy L0 * int T
    __device__ void eval(double eps, double L0, double& T, double& kt, double& W) const
    {
        if (law == LAW_EXP && eps >= 0.0) {
            const double e = exp(B * eps);
            T = EA * (e - 1.0) / B;
            kt = EA * e;
            W = L0 * EA * ((e - 1.0) / B - eps) / B;
        } else {
            T = EA * eps;
            kt = EA;
            W = 0.5 * L0 * EA * eps * eps;
        }
    }
};

struct VarCtx {
    const VariantArgs& A;
    int64_t f0, nfib, a0, nf, b0, nb;
    double F[9];
    double* node;   // [nf][kNodeDoubles] of this RVE
    double* fibw;   // [nfib][kFibDoubles] of this RVE
};

// Fiber pass: force vector, Gershgorin term and stored energy of every fiber
// at the current fluctuation h; returns this thread's share of the energy
// and, when want_rq is set, adds its share of u.K u to rq (u = h - h_start, K the
// tangent stiffness: (k_t/L0) (n.du)^2 + (T/l) (|du|^2 - (n.du)^2) per fiber).
__device__ __forceinline__ double fiber_pass(const VarCtx& C, const Law& law, bool want_rq, double& rq)
{
    const DevNet& net = C.A.s.net;
    double Wsum = 0.0;
    for (int64_t k = threadIdx.x; k < C.nfib; k += kVT) {
        const uint32_t e = net.ends[C.f0 + k];
        const int i = e & 0xffff, j = e >> 16;
        const double* d0 = net.d0 + 3 * (C.f0 + k);
        const double L0 = net.L0[C.f0 + k];
        double D[3], dh[3];
        for (int c = 0; c < 3; ++c) {
            D[c] = C.F[3 * c] * d0[0] + C.F[3 * c + 1] * d0[1] + C.F[3 * c + 2] * d0[2];
            dh[c] = (j < C.nf ? C.node[kNodeDoubles * j + c] : 0.0) - (i < C.nf ? C.node[kNodeDoubles * i + c] : 0.0);
        }
        // l^2 - L0^2 formed without cancellation: (|D|^2 - L0^2) + 2 D.dh + |dh|^2
        const double q0 = (D[0] * D[0] + D[1] * D[1] + D[2] * D[2]) - L0 * L0;
        const double q = q0 + 2.0 * (D[0] * dh[0] + D[1] * dh[1] + D[2] * dh[2]) +
                         (dh[0] * dh[0] + dh[1] * dh[1] + dh[2] * dh[2]);
        const double d[3] = {D[0] + dh[0], D[1] + dh[1], D[2] + dh[2]};
        const double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double eps = q / (L0 * (l + L0));
        double T, kt, W;
        law.eval(eps, L0, T, kt, W);
        double* o = C.fibw + kFibDoubles * k;
        for (int c = 0; c < 3; ++c) o[c] = T * d[c] / l;
        o[3] = fmax(kt / L0, fabs(T) / l);
        o[4] = W;
        Wsum += W;
        if (want_rq) {
            double du[3];
            for (int c = 0; c < 3; ++c)
                du[c] = (j < C.nf ? C.node[kNodeDoubles * j + c] - C.node[kNodeDoubles * j + 12 + c] : 0.0) -
                        (i < C.nf ? C.node[kNodeDoubles * i + c] - C.node[kNodeDoubles * i + 12 + c] : 0.0);
            const double nd = (d[0] * du[0] + d[1] * du[1] + d[2] * du[2]) / l;
            const double du2 = du[0] * du[0] + du[1] * du[1] + du[2] * du[2];
            rq += kt / L0 * nd * nd + T / l * (du2 - nd * nd);
        }
    }
    return Wsum;
}

// Internal force and Gershgorin sum of free node a from the fiber pass.
__device__ __forceinline__ void gather_free(const VarCtx& C, int64_t a, double (&f)[3], double& G)
{
    const DevNet& net = C.A.s.net;
    f[0] = f[1] = f[2] = 0.0;
    G = 0.0;
    for (int64_t q = net.inc_off[C.a0 + a]; q < net.inc_off[C.a0 + a + 1]; ++q) {
        const uint32_t e = net.inc[q];
        const double* o = C.fibw + kFibDoubles * (int64_t)(e & 0x7fffffffu);
        const double sg = (e >> 31) ? -1.0 : 1.0;   // end i receives -T d/l
        for (int c = 0; c < 3; ++c) f[c] += sg * o[c];
        G += 2.0 * o[3];
    }
}

// Squared norm of the boundary-node internal forces (this thread's share).
__device__ __forceinline__ double boundary_norm2(const VarCtx& C)
{
    const DevNet& net = C.A.s.net;
    double s = 0.0;
    for (int64_t bq = threadIdx.x; bq < C.nb; bq += kVT) {
        double f[3] = {0.0, 0.0, 0.0};
        for (int64_t q = net.binc_off[C.b0 + bq]; q < net.binc_off[C.b0 + bq + 1]; ++q) {
            const uint32_t e = net.binc[q];
            const double* o = C.fibw + kFibDoubles * (int64_t)(e & 0x7fffffffu);
            const double sg = (e >> 31) ? -1.0 : 1.0;
            for (int c = 0; c < 3; ++c) f[c] += sg * o[c];
        }
        s += f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
    }
    return s;
}

__global__ __launch_bounds__(kVT) void dr_variant_kernel(VariantArgs A)
{
    __shared__ double red[8][kWaves];
    __shared__ double red_max[kWaves];
    const int64_t r = blockIdx.x;
    const SolveArgs& S = A.s;
    const DevNet& net = S.net;
    VarCtx C{A, net.fib_off[r], net.fib_off[r + 1] - net.fib_off[r], net.free_off[r],
             net.free_off[r + 1] - net.free_off[r], net.bnd_off[r], net.bnd_off[r + 1] - net.bnd_off[r], {},
             A.ws_node + kNodeDoubles * net.free_off[r], A.ws_fib + kFibDoubles * net.fib_off[r]};
    bool fin = true;
    for (int k = 0; k < 9; ++k) {
        C.F[k] = S.F[9 * r + k];
        fin = fin && isfinite(C.F[k]);
    }
    const double J = C.F[0] * (C.F[4] * C.F[8] - C.F[5] * C.F[7]) - C.F[1] * (C.F[3] * C.F[8] - C.F[5] * C.F[6]) +
                     C.F[2] * (C.F[3] * C.F[7] - C.F[4] * C.F[6]);
    if (!fin || !(J > 0.0)) {
        if (threadIdx.x == 0) {
            S.status[r] = ST_BAD_F;
            S.iters[r] = 0;
            S.Rres[r] = S.Dres[r] = S.Bres[r] = NAN;
            A.c_final[r] = A.energy[r] = NAN;
        }
        return;
    }
    const Law law{S.law, S.EA, S.B};
    const int damping = A.damping;
    // start: fluctuation (warm or affine), v = 0
    for (int64_t a = threadIdx.x; a < C.nf; a += kVT) {
        double* nd = C.node + kNodeDoubles * a;
        for (int c = 0; c < 3; ++c) {
            const double h = S.init == INIT_WARM ? S.h_state[3 * (C.a0 + a) + c] : 0.0;
            nd[c] = h;          // h
            nd[3 + c] = 0.0;    // v
            nd[12 + c] = h;     // h_start
        }
    }
    __syncthreads();
    double unused_rq = 0.0;
    double W = fiber_pass(C, law, false, unused_rq);
    __syncthreads();
    double R2 = 0.0, gmax = 0.0;
    for (int64_t a = threadIdx.x; a < C.nf; a += kVT) {
        double* nd = C.node + kNodeDoubles * a;
        double f[3], G;
        gather_free(C, a, f, G);
        const double M = S.mass_mode == MASS_SCALED ? (G > 0.0 ? G / 4.0 : 1.0) : net.mass[C.a0 + a] * S.rhoA;
        for (int c = 0; c < 3; ++c) {
            nd[9 + c] = f[c];
            nd[6 + c] = -f[c] / M;
        }
        nd[15] = M;
        nd[16] = G;
        R2 += f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
        gmax = fmax(gmax, G / M);
    }
    {
        double v[3] = {R2, boundary_norm2(C), W};
        block_reduce<3>(v, gmax, red, red_max);
        R2 = v[0];
        double B2 = v[1];
        W = v[2];
        double R = sqrt(R2), D = 0.0, tol = fmax(S.tol_abs, S.tol_rel * sqrt(B2));
        const double W0 = W;
        double cc = damping == DAMP_KINETIC ? 0.0 : S.c[r];
        double KE = 0.0, KE_prev = 0.0, Wd = 0.0, ebal = 0.0;
        int64_t n = 0;
        int status = ST_CONVERGED;
        while (!(R <= tol && D <= tol)) {
            if (!isfinite(R)) {
                status = ST_NONFINITE;
                break;
            }
            if (n >= S.n_max) {
                status = ST_MAXITER;
                break;
            }
            const double dt = S.alpha * 2.0 / sqrt(gmax);
            // half-step velocity and position of the free nodes; keep f^n
            for (int64_t a = threadIdx.x; a < C.nf; a += kVT) {
                double* nd = C.node + kNodeDoubles * a;
                for (int c = 0; c < 3; ++c) {
                    nd[3 + c] += 0.5 * dt * nd[6 + c];
                    nd[c] += dt * nd[3 + c];
                }
            }
            __syncthreads();
            double num = 0.0, den = 0.0;
            W = fiber_pass(C, law, damping == DAMP_ADAPTIVE, num);
            __syncthreads();
            // forces at the new positions; adaptive Rayleigh-quotient sums
            for (int64_t a = threadIdx.x; a < C.nf; a += kVT) {
                double* nd = C.node + kNodeDoubles * a;
                double f[3], G;
                gather_free(C, a, f, G);
                if (damping == DAMP_ADAPTIVE)
                    for (int c = 0; c < 3; ++c) {
                        const double u = nd[c] - nd[12 + c];
                        den += nd[15] * u * u;
                    }
                for (int c = 0; c < 3; ++c) nd[9 + c] = f[c];
                nd[16] = G;
            }
            if (damping == DAMP_ADAPTIVE) {
                double v2[2] = {num, den};
                double dummy = 0.0;
                block_reduce<2>(v2, dummy, red, red_max);
                cc = (v2[0] > 0.0 && v2[1] > 0.0) ? 2.0 * sqrt(v2[0] / v2[1]) : 0.0;
            }
            // damping work over the step, accelerations, second half step, sums
            double wd = 0.0, r2 = 0.0, mv2 = 0.0, ke = 0.0, gm = 0.0;
            for (int64_t a = threadIdx.x; a < C.nf; a += kVT) {
                double* nd = C.node + kNodeDoubles * a;
                const double M = nd[15];
                if (damping != DAMP_KINETIC)
                    for (int c = 0; c < 3; ++c) wd += cc * M * nd[3 + c] * nd[3 + c] * dt;
                for (int c = 0; c < 3; ++c) {
                    const double fc = nd[9 + c];
                    r2 += fc * fc;
                    nd[6 + c] = -(fc + cc * M * nd[3 + c]) / M;
                    nd[3 + c] += 0.5 * dt * nd[6 + c];
                    const double mv = M * nd[3 + c];
                    mv2 += mv * mv;
                    ke += 0.5 * M * nd[3 + c] * nd[3 + c];
                }
                gm = fmax(gm, nd[16] / M);
            }
            double v5[6] = {r2, mv2, ke, wd, boundary_norm2(C), W};
            block_reduce<6>(v5, gm, red, red_max);
            R2 = v5[0];
            double MV2 = v5[1];
            KE = v5[2];
            Wd += v5[3];
            B2 = v5[4];
            W = v5[5];
            gmax = gm;
            if (damping == DAMP_KINETIC) {
                if (KE < KE_prev) {
                    Wd += KE;
                    KE = 0.0;
                    MV2 = 0.0;
                    for (int64_t a = threadIdx.x; a < C.nf; a += kVT) {
                        double* nd = C.node + kNodeDoubles * a;
                        for (int c = 0; c < 3; ++c) {
                            nd[3 + c] = 0.0;
                            nd[6 + c] = -nd[9 + c] / nd[15];
                        }
                    }
                }
                KE_prev = KE;
            }
            const double scale = fmax(fmax(W0, W), fmax(KE, Wd));
            ebal = scale > 0.0 ? fabs(W + KE + Wd - W0) / scale : 0.0;
            R = sqrt(R2);
            D = (damping == DAMP_KINETIC ? S.c[r] : cc) * sqrt(MV2);
            tol = fmax(S.tol_abs, S.tol_rel * sqrt(B2));
            ++n;
            __syncthreads();
            if (A.energy_check && ebal > A.energy_tol) {
                status = ST_ENERGY;
                break;
            }
        }
        if (status == ST_CONVERGED && !isfinite(R)) status = ST_NONFINITE;
        // final fluctuation for the stress kernel, tangent and warm starts
        for (int64_t a = threadIdx.x; a < C.nf; a += kVT)
            for (int c = 0; c < 3; ++c) S.h_state[3 * (C.a0 + a) + c] = C.node[kNodeDoubles * a + c];
        if (threadIdx.x == 0) {
            S.status[r] = status;
            S.iters[r] = n;
            S.Rres[r] = R;
            S.Dres[r] = D;
            S.Bres[r] = sqrt(B2);
            A.c_final[r] = cc;
            A.energy[r] = ebal;
        }
    }
}

}  // namespace

hipError_t launch_variant(const VariantArgs& a, int64_t n_rve, hipStream_t s)
{
    if (n_rve <= 0) return hipSuccess;
    hipLaunchKernelGGL(dr_variant_kernel, dim3((unsigned)n_rve), dim3(kVT), 0, s, a);
    return hipGetLastError();
}

size_t variant_ws_bytes(int64_t n_free, int64_t n_fib)
{
    return 8 * ((size_t)kNodeDoubles * (size_t)n_free + (size_t)kFibDoubles * (size_t)n_fib);
}

hipError_t variant_fixed_private(size_t* bytes)
{
    return max_private_bytes({(const void*)dr_variant_kernel}, bytes);
}

}  // namespace rve
