// Material tangent dsigma/dF and its vector-Jacobian product on the state of
// the last relaxation, by matrix-free conjugate gradients on the free-node
// stiffness K_ff (the paper differentiates the stress by finite differences
// of extra relaxations, Section 3.2; here the same linearisation is solved
// directly at the converged network).
//
// Per fiber, K contributes B_f = a n n^T + g (I - n n^T) with n = d/l,
// a = k_t/L0, g = T/l, so (K u)_a = sum_{fibers at a} B_f (u_a - u_other).
//
// Tangent (9 right-hand sides, one per F_kl): the boundary moves by E Xm_b,
// E = e_k e_l, so K_ff dx = -[K (E Xm)]_f with [K (E Xm)]_a =
// sum s_af B_f (E d0_f); then df_b = sum s_bf B_f (E d0_f + dx_j - dx_i) and
// dsigma = (sum_b df_b x_b^T + f_b (E Xm_b)^T) / (J V0) - sigma (F^-1)_lk.
//
// VJP (1 right-hand side): with y_b = G x_b on boundary nodes (G = dL/dsigma)
// and u = [0; y], solve K_ff lambda = (K u)_f, then z_b = (K [-lambda; y])_b
// and dL/dF_kl = sum_b (z_b + G^T f_b)_k Xm_b,l / (J V0) - (G:sigma) F^-T_kl.
//
// Products are FP32 (fiber operators and vectors), dot products and the
// residual norms FP64, the final assembly FP64 from an FP64 re-evaluation of
// the boundary fibers.  One workgroup per RVE, persistent over a work queue.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rve_internal.h"

namespace rve {

namespace {

constexpr int ST_CONVERGED = 0, ST_NO_STATE = 4, ST_CG_MAXITER = 5, ST_CG_INDEFINITE = 6;

__device__ inline double det3(const double* F)
{
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
}

// FP64 fiber state: unit vector n, a = k_t/L0, g = T/l, axial force T.
struct FiberOp {
    double nx, ny, nz, a, g, T;
};

__device__ inline FiberOp fiber_op(const TangentArgs& A, const double* F, int64_t f0, int64_t a0, int64_t nf,
                                   int64_t k)
{
    const DevNet& net = A.net;
    const double* d0 = net.d0 + 3 * (f0 + k);
    const double L0 = net.L0[f0 + k];
    uint32_t e = net.ends[f0 + k];
    int i = e & 0xffff, j = e >> 16;
    double D[3];
    for (int p = 0; p < 3; ++p) D[p] = F[3 * p] * d0[0] + F[3 * p + 1] * d0[1] + F[3 * p + 2] * d0[2];
    double q0 = (D[0] * D[0] + D[1] * D[1] + D[2] * D[2]) - L0 * L0;
    double dh[3] = {0, 0, 0};
    for (int p = 0; p < 3; ++p) {
        if (j < nf) dh[p] += A.h_state[3 * (a0 + j) + p];
        if (i < nf) dh[p] -= A.h_state[3 * (a0 + i) + p];
    }
    double d[3] = {D[0] + dh[0], D[1] + dh[1], D[2] + dh[2]};
    double q = q0 + (2.0 * (D[0] * dh[0] + D[1] * dh[1] + D[2] * dh[2]) + (dh[0] * dh[0] + dh[1] * dh[1] + dh[2] * dh[2]));
    double l = sqrt(L0 * L0 + q);
    double eps = q / (L0 * (l + L0));
    double T, kt;
    if (A.law != 0 && eps >= 0.0) {
        double em1 = expm1(A.B * eps);
        T = A.EA * em1 / A.B;
        kt = A.EA * (em1 + 1.0);
    } else {
        T = A.EA * eps;
        kt = A.EA;
    }
    FiberOp o;
    o.nx = d[0] / l;
    o.ny = d[1] / l;
    o.nz = d[2] / l;
    o.a = kt / L0;
    o.g = T / l;
    o.T = T;
    return o;
}

template <typename T>
__device__ inline T wsum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum NR doubles over the workgroup; every thread gets the totals.
template <int NR, int NT>
__device__ inline void block_sum(double* v, double (*sh)[NT / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        double s = wsum(v[k]);
        if (lane == 0) sh[k][wave] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += sh[k][w];
        v[k] = s;
    }
    __syncthreads();
}

// Apply B_f (FP32 parameters) to a vector.
__device__ inline void apply_B(const float4 nA, float g, float dx, float dy, float dz, float& wx, float& wy, float& wz)
{
    float dn = nA.x * dx + nA.y * dy + nA.z * dz;
    float c = (nA.w - g) * dn;
    wx = g * dx + c * nA.x;
    wy = g * dy + c * nA.y;
    wz = g * dz + c * nA.z;
}

template <int NR, int NT>
__device__ void cg_one(const TangentArgs& A, int r, double (*sh)[NT / 64])
{
    const DevNet& net = A.net;
    const int tid = threadIdx.x;
    const int64_t f0 = net.fib_off[r], nfib = net.fib_off[r + 1] - f0;
    const int64_t a0 = net.free_off[r], nf = net.free_off[r + 1] - a0;
    const int64_t b0 = net.bnd_off[r];
    constexpr int W = NR * 3;
    double* out = A.out + (int64_t)r * (NR == 9 ? 81 : 9);
    if (A.solve_status[r] != 0) {
        if (tid == 0) A.status[r] = ST_NO_STATE;
        for (int k = tid; k < (NR == 9 ? 81 : 9); k += NT) out[k] = NAN;
        return;
    }
    double F[9], G[9];
    for (int k = 0; k < 9; ++k) F[k] = A.F[9 * r + k];
    if (NR == 1)
        for (int k = 0; k < 9; ++k) G[k] = A.gsigma[9 * r + k];
    const double J = det3(F);
    float4* par = reinterpret_cast<float4*>(A.ws_par) + 2 * (f0 + r);   // [nfib][2]: (n, a), (g, -, -, -)
    float* vx = A.ws_vec + (a0 + r) * (int64_t)W;                       // x
    float* vr = vx + (A.n_free_total + A.n_rve) * (int64_t)W;            // r
    float* vp = vr + (A.n_free_total + A.n_rve) * (int64_t)W;            // p (entry nf = 0)
    float* vq = vp + (A.n_free_total + A.n_rve) * (int64_t)W;            // Ap

    // fiber operators
#pragma unroll 1
    for (int64_t k = tid; k < nfib; k += NT) {
        FiberOp o = fiber_op(A, F, f0, a0, nf, k);
        par[2 * k] = make_float4((float)o.nx, (float)o.ny, (float)o.nz, (float)o.a);
        par[2 * k + 1] = make_float4((float)o.g, 0.f, 0.f, 0.f);
    }
    if (tid < W) vp[nf * W + tid] = 0.f;
    __syncthreads();

    // right-hand sides
    double rr[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) rr[k] = 0.0;
#pragma unroll 1
    for (int64_t a = tid; a < nf; a += NT) {
        float b[W];
#pragma unroll
        for (int k = 0; k < W; ++k) b[k] = 0.f;
#pragma unroll 1
        for (int64_t e = net.inc_off[a0 + a]; e < net.inc_off[a0 + a + 1]; ++e) {
            uint32_t w = net.inc[e];
            int64_t k = w & 0x7fffffffu;
            float sgn = (w >> 31) ? -1.f : 1.f;     // end i: -1, end j: +1
            float4 nA = par[2 * k];
            float g = par[2 * k + 1].x;
            if (NR == 9) {
                // -s B_f (e_kk d0_l) for direction (kk, l)
                const double* d0 = net.d0 + 3 * (f0 + k);
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    float ex = kk == 0, ey = kk == 1, ez = kk == 2;
                    float wx, wy, wz;
                    apply_B(nA, g, ex, ey, ez, wx, wy, wz);
#pragma unroll
                    for (int l = 0; l < 3; ++l) {
                        float s = -sgn * (float)d0[l];
                        int col = 3 * kk + l;
                        b[3 * col] += s * wx;
                        b[3 * col + 1] += s * wy;
                        b[3 * col + 2] += s * wz;
                    }
                }
            } else {
                // (K u)_a with u = y on boundary ends: B_f (0 - y_other)
                uint32_t en = net.ends[f0 + k];
                int o = (w >> 31) ? (int)(en >> 16) : (int)(en & 0xffff);
                if (o >= nf) {
                    const double* Xm = net.Xb + 3 * (b0 + (o - nf));
                    double x[3], y[3];
                    for (int p = 0; p < 3; ++p) x[p] = F[3 * p] * Xm[0] + F[3 * p + 1] * Xm[1] + F[3 * p + 2] * Xm[2];
                    for (int p = 0; p < 3; ++p) y[p] = G[3 * p] * x[0] + G[3 * p + 1] * x[1] + G[3 * p + 2] * x[2];
                    float wx, wy, wz;
                    apply_B(nA, g, (float)-y[0], (float)-y[1], (float)-y[2], wx, wy, wz);
                    b[0] += wx;
                    b[1] += wy;
                    b[2] += wz;
                }
            }
        }
        float* X = vx + a * W;
        float* R = vr + a * W;
        float* P = vp + a * W;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            X[k] = 0.f;
            R[k] = b[k];
            P[k] = b[k];
        }
#pragma unroll
        for (int k = 0; k < NR; ++k)
            rr[k] += (double)b[3 * k] * b[3 * k] + (double)b[3 * k + 1] * b[3 * k + 1] + (double)b[3 * k + 2] * b[3 * k + 2];
    }
    block_sum<NR, NT>(rr, sh);
    double bb[NR];
    bool active[NR];
    int status = ST_CONVERGED;
    const double tol2 = A.cg_tol * A.cg_tol;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        bb[k] = rr[k];
        active[k] = rr[k] > 0.0;
    }
    const int64_t maxit = A.cg_max > 0 ? A.cg_max : 6 * nf + 100;
    int64_t it = 0;
    for (;;) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < NR; ++k) any = any || active[k];
        if (!any) break;
        if (it >= maxit) {
            status = ST_CG_MAXITER;
            break;
        }
        ++it;
        // q = K p and p.q
        double pq[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) pq[k] = 0.0;
#pragma unroll 1
        for (int64_t a = tid; a < nf; a += NT) {
            const float* Pa = vp + a * W;
            float pa[W], q[W];
#pragma unroll
            for (int k = 0; k < W; ++k) {
                pa[k] = Pa[k];
                q[k] = 0.f;
            }
#pragma unroll 1
            for (int64_t e = net.inc_off[a0 + a]; e < net.inc_off[a0 + a + 1]; ++e) {
                uint32_t w = net.inc[e];
                int64_t k = w & 0x7fffffffu;
                uint32_t en = net.ends[f0 + k];
                int o = (w >> 31) ? (int)(en >> 16) : (int)(en & 0xffff);
                const float* Po = vp + (o < nf ? o : nf) * (int64_t)W;
                float4 nA = par[2 * k];
                float g = par[2 * k + 1].x;
#pragma unroll
                for (int c = 0; c < NR; ++c) {
                    float wx, wy, wz;
                    apply_B(nA, g, pa[3 * c] - Po[3 * c], pa[3 * c + 1] - Po[3 * c + 1], pa[3 * c + 2] - Po[3 * c + 2],
                            wx, wy, wz);
                    q[3 * c] += wx;
                    q[3 * c + 1] += wy;
                    q[3 * c + 2] += wz;
                }
            }
            float* Q = vq + a * W;
#pragma unroll
            for (int k = 0; k < W; ++k) Q[k] = q[k];
#pragma unroll
            for (int c = 0; c < NR; ++c)
                pq[c] += (double)pa[3 * c] * q[3 * c] + (double)pa[3 * c + 1] * q[3 * c + 1] + (double)pa[3 * c + 2] * q[3 * c + 2];
        }
        block_sum<NR, NT>(pq, sh);
        float alpha[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            alpha[k] = 0.f;
            if (active[k]) {
                if (!(pq[k] > 0.0)) {
                    active[k] = false;
                    status = ST_CG_INDEFINITE;
                } else {
                    alpha[k] = (float)(rr[k] / pq[k]);
                }
            }
        }
        double rn[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) rn[k] = 0.0;
#pragma unroll 1
        for (int64_t a = tid; a < nf; a += NT) {
            float* X = vx + a * W;
            float* R = vr + a * W;
            const float* P = vp + a * W;
            const float* Q = vq + a * W;
#pragma unroll
            for (int c = 0; c < NR; ++c)
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    int k = 3 * c + p;
                    X[k] += alpha[c] * P[k];
                    float rk = R[k] - alpha[c] * Q[k];
                    R[k] = rk;
                    rn[c] += (double)rk * rk;
                }
        }
        block_sum<NR, NT>(rn, sh);
        float beta[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            beta[k] = active[k] ? (float)(rn[k] / rr[k]) : 0.f;
            if (active[k]) {
                rr[k] = rn[k];
                if (rn[k] <= tol2 * bb[k]) active[k] = false;
            }
        }
#pragma unroll 1
        for (int64_t a = tid; a < nf; a += NT) {
            float* P = vp + a * W;
            const float* R = vr + a * W;
#pragma unroll
            for (int c = 0; c < NR; ++c)
#pragma unroll
                for (int p = 0; p < 3; ++p) P[3 * c + p] = R[3 * c + p] + beta[c] * P[3 * c + p];
        }
        __syncthreads();
    }

    // assembly over fibers with a boundary end (FP64 operators)
    const double V0 = net.V0[r];
    double Finv[9];
    {
        double id = 1.0 / J;
        Finv[0] = (F[4] * F[8] - F[5] * F[7]) * id;
        Finv[1] = (F[2] * F[7] - F[1] * F[8]) * id;
        Finv[2] = (F[1] * F[5] - F[2] * F[4]) * id;
        Finv[3] = (F[5] * F[6] - F[3] * F[8]) * id;
        Finv[4] = (F[0] * F[8] - F[2] * F[6]) * id;
        Finv[5] = (F[2] * F[3] - F[0] * F[5]) * id;
        Finv[6] = (F[3] * F[7] - F[4] * F[6]) * id;
        Finv[7] = (F[1] * F[6] - F[0] * F[7]) * id;
        Finv[8] = (F[0] * F[4] - F[1] * F[3]) * id;
    }
    double sig[9];
    for (int k = 0; k < 9; ++k) sig[k] = A.sigma[9 * r + k];
    if (NR == 9) {
        for (int col = 0; col < 9; ++col) {
            const int kk = col / 3, l = col % 3;
            double acc[9];
#pragma unroll
            for (int p = 0; p < 9; ++p) acc[p] = 0.0;
#pragma unroll 1
            for (int64_t k = tid; k < nfib; k += NT) {
                uint32_t en = net.ends[f0 + k];
                int i = en & 0xffff, j = en >> 16;
                if (i < nf && j < nf) continue;
                FiberOp o = fiber_op(A, F, f0, a0, nf, k);
                const double* d0 = net.d0 + 3 * (f0 + k);
                double u[3] = {0, 0, 0};
                u[kk] = d0[l];
                for (int p = 0; p < 3; ++p) {
                    if (j < nf) u[p] += vx[j * W + 3 * col + p];
                    if (i < nf) u[p] -= vx[i * W + 3 * col + p];
                }
                double dn = o.nx * u[0] + o.ny * u[1] + o.nz * u[2];
                double cc = (o.a - o.g) * dn;
                double w[3] = {o.g * u[0] + cc * o.nx, o.g * u[1] + cc * o.ny, o.g * u[2] + cc * o.nz};
                double fv[3] = {o.T * o.nx, o.T * o.ny, o.T * o.nz};
                for (int end = 0; end < 2; ++end) {
                    int node = end ? j : i;
                    if (node < nf) continue;
                    double s = end ? 1.0 : -1.0;
                    const double* Xm = net.Xb + 3 * (b0 + (node - nf));
                    double x[3];
                    for (int p = 0; p < 3; ++p) x[p] = F[3 * p] * Xm[0] + F[3 * p + 1] * Xm[1] + F[3 * p + 2] * Xm[2];
                    // df_b x_b^T + f_b (E Xm_b)^T, (E Xm_b) = e_kk Xm_b,l
                    for (int p = 0; p < 3; ++p) {
                        for (int q = 0; q < 3; ++q) acc[3 * p + q] += s * w[p] * x[q];
                        acc[3 * p + kk] += s * fv[p] * Xm[l];
                    }
                }
            }
            block_sum<9, NT>(acc, sh);
            if (tid < 9) out[9 * tid + col] = acc[tid] / (J * V0) - sig[tid] * Finv[3 * l + kk];
        }
    } else {
        double gs = 0.0;
        for (int k = 0; k < 9; ++k) gs += G[k] * sig[k];
        double acc[9];
#pragma unroll
        for (int p = 0; p < 9; ++p) acc[p] = 0.0;
#pragma unroll 1
        for (int64_t k = tid; k < nfib; k += NT) {
            uint32_t en = net.ends[f0 + k];
            int i = en & 0xffff, j = en >> 16;
            if (i < nf && j < nf) continue;
            FiberOp o = fiber_op(A, F, f0, a0, nf, k);
            // u = [-lambda; y]
            double ui[3], uj[3];
            for (int end = 0; end < 2; ++end) {
                int node = end ? j : i;
                double* u = end ? uj : ui;
                if (node < nf) {
                    for (int p = 0; p < 3; ++p) u[p] = -(double)vx[node * W + p];
                } else {
                    const double* Xm = net.Xb + 3 * (b0 + (node - nf));
                    double x[3];
                    for (int p = 0; p < 3; ++p) x[p] = F[3 * p] * Xm[0] + F[3 * p + 1] * Xm[1] + F[3 * p + 2] * Xm[2];
                    for (int p = 0; p < 3; ++p) u[p] = G[3 * p] * x[0] + G[3 * p + 1] * x[1] + G[3 * p + 2] * x[2];
                }
            }
            double du[3] = {uj[0] - ui[0], uj[1] - ui[1], uj[2] - ui[2]};
            double dn = o.nx * du[0] + o.ny * du[1] + o.nz * du[2];
            double cc = (o.a - o.g) * dn;
            double w[3] = {o.g * du[0] + cc * o.nx, o.g * du[1] + cc * o.ny, o.g * du[2] + cc * o.nz};
            double fv[3] = {o.T * o.nx, o.T * o.ny, o.T * o.nz};
            double gtf[3];
            for (int p = 0; p < 3; ++p) gtf[p] = G[p] * fv[0] + G[3 + p] * fv[1] + G[6 + p] * fv[2];
            for (int end = 0; end < 2; ++end) {
                int node = end ? j : i;
                if (node < nf) continue;
                double s = end ? 1.0 : -1.0;
                const double* Xm = net.Xb + 3 * (b0 + (node - nf));
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) acc[3 * p + q] += s * (w[p] + gtf[p]) * Xm[q];
            }
        }
        block_sum<9, NT>(acc, sh);
        if (tid < 9) {
            int kk = tid / 3, l = tid % 3;
            out[tid] = acc[tid] / (J * V0) - gs * Finv[3 * l + kk];
        }
    }
    if (tid == 0) A.status[r] = status;
    __syncthreads();
}

template <int NR, int NT>
__global__ __launch_bounds__(NT) void cg_kernel(TangentArgs A)
{
    __shared__ double sh[9][NT / 64];
    __shared__ int task;
    for (;;) {
        if (threadIdx.x == 0) task = atomicAdd(A.queue, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(task);
        __syncthreads();
        if (t >= A.n_rve) break;
        cg_one<NR, NT>(A, t, sh);
    }
}

}  // namespace

hipError_t launch_tangent(const TangentArgs& a, int grid, hipStream_t s)
{
    if (a.mode == 0)
        hipLaunchKernelGGL((cg_kernel<9, 256>), dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((cg_kernel<1, 256>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace rve
