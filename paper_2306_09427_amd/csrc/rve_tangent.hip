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
// Precision: iterative refinement.  The outer loop keeps the solution, the
// right-hand side and the residual r = b - K x in FP64 (FP64 fiber operators);
// each inner solve K d = r is conjugate gradients with FP32 products and FP64
// dot products, stopped after a 1e-6 reduction of its residual; x += d.
// Plain FP32 CG stalls near eps_32 cond(K_ff), about 1e-3 on these networks,
// which refinement removes.  The final assembly is FP64 from an FP64
// re-evaluation of the boundary fibers.  One workgroup per RVE, persistent
// over a work queue.
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
    const int64_t NV = (A.n_free_total + A.n_rve) * (int64_t)W;   // length of one vector over the batch
    // fiber operators: FP32 copy for the inner solves, FP64 copy for residuals
    float4* par = reinterpret_cast<float4*>(A.ws_par) + 2 * (f0 + r);   // [nfib][2]: (n, a), (g, -, -, -)
    double* par64 = A.ws_par64 + 5 * (f0 + r);                          // [nfib][5]: n, a, g
    float* vx = A.ws_vec + (a0 + r) * (int64_t)W;     // inner solution d
    float* vr = vx + NV;                              // inner residual
    float* vp = vr + NV;                              // search direction (entry nf = 0)
    float* vq = vp + NV;                              // K p
    double* xb = A.ws_vec64 + (a0 + r) * (int64_t)W;  // FP64 solution (entry nf = 0)
    double* bb64 = xb + NV;                           // FP64 right-hand side

#pragma unroll 1
    for (int64_t k = tid; k < nfib; k += NT) {
        FiberOp o = fiber_op(A, F, f0, a0, nf, k);
        par[2 * k] = make_float4((float)o.nx, (float)o.ny, (float)o.nz, (float)o.a);
        par[2 * k + 1] = make_float4((float)o.g, 0.f, 0.f, 0.f);
        double* q = par64 + 5 * k;
        q[0] = o.nx; q[1] = o.ny; q[2] = o.nz; q[3] = o.a; q[4] = o.g;
    }
    if (tid < W) {
        vp[nf * W + tid] = 0.f;
        xb[nf * W + tid] = 0.0;
    }
    __syncthreads();

    // right-hand sides (FP64)
    double bnorm2[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) bnorm2[k] = 0.0;
#pragma unroll 1
    for (int64_t a = tid; a < nf; a += NT) {
        double b[W];
#pragma unroll
        for (int k = 0; k < W; ++k) b[k] = 0.0;
#pragma unroll 1
        for (int64_t e = net.inc_off[a0 + a]; e < net.inc_off[a0 + a + 1]; ++e) {
            uint32_t w = net.inc[e];
            int64_t k = w & 0x7fffffffu;
            double sgn = (w >> 31) ? -1.0 : 1.0;     // end i: -1, end j: +1
            const double* q = par64 + 5 * k;
            if (NR == 9) {
                // -s B_f (e_kk d0_l) for direction (kk, l)
                const double* d0 = net.d0 + 3 * (f0 + k);
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    double n_k = q[kk], c = (q[3] - q[4]) * n_k;
                    double wv[3] = {c * q[0], c * q[1], c * q[2]};
                    wv[kk] += q[4];
#pragma unroll
                    for (int l = 0; l < 3; ++l) {
                        double s = -sgn * d0[l];
                        int col = 3 * kk + l;
                        b[3 * col] += s * wv[0];
                        b[3 * col + 1] += s * wv[1];
                        b[3 * col + 2] += s * wv[2];
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
                    for (int p = 0; p < 3; ++p) y[p] = -(G[3 * p] * x[0] + G[3 * p + 1] * x[1] + G[3 * p + 2] * x[2]);
                    double dn = q[0] * y[0] + q[1] * y[1] + q[2] * y[2];
                    double c = (q[3] - q[4]) * dn;
                    for (int p = 0; p < 3; ++p) b[p] += q[4] * y[p] + c * q[p];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < W; ++k) {
            bb64[a * W + k] = b[k];
            xb[a * W + k] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) bnorm2[k] += b[3 * k] * b[3 * k] + b[3 * k + 1] * b[3 * k + 1] + b[3 * k + 2] * b[3 * k + 2];
    }
    block_sum<NR, NT>(bnorm2, sh);

    int status = ST_CONVERGED;
    const double tol2 = A.cg_tol * A.cg_tol;
    const int64_t maxit = A.cg_max > 0 ? A.cg_max : 6 * nf + 100;
    int64_t it_total = 0;
    bool done[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) done[k] = !(bnorm2[k] > 0.0);

    // Outer loop: FP64 residual r = b - K x of the FP64 solution, inner CG with
    // FP32 products on K d = r, x += d (iterative refinement).
    for (int outer = 0; outer < 8; ++outer) {
        double rr[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) rr[k] = 0.0;
#pragma unroll 1
        for (int64_t a = tid; a < nf; a += NT) {
            double ra[W];
#pragma unroll
            for (int k = 0; k < W; ++k) ra[k] = bb64[a * W + k];
            if (outer > 0) {
                double xa[W];
#pragma unroll
                for (int k = 0; k < W; ++k) xa[k] = xb[a * W + k];
#pragma unroll 1
                for (int64_t e = net.inc_off[a0 + a]; e < net.inc_off[a0 + a + 1]; ++e) {
                    uint32_t w = net.inc[e];
                    int64_t k = w & 0x7fffffffu;
                    uint32_t en = net.ends[f0 + k];
                    int o = (w >> 31) ? (int)(en >> 16) : (int)(en & 0xffff);
                    const double* xo = xb + (o < nf ? o : nf) * (int64_t)W;
                    const double* q = par64 + 5 * k;
#pragma unroll
                    for (int c = 0; c < NR; ++c) {
                        double dx = xa[3 * c] - xo[3 * c], dy = xa[3 * c + 1] - xo[3 * c + 1],
                               dz = xa[3 * c + 2] - xo[3 * c + 2];
                        double dn = q[0] * dx + q[1] * dy + q[2] * dz;
                        double cc = (q[3] - q[4]) * dn;
                        ra[3 * c] -= q[4] * dx + cc * q[0];
                        ra[3 * c + 1] -= q[4] * dy + cc * q[1];
                        ra[3 * c + 2] -= q[4] * dz + cc * q[2];
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < W; ++k) {
                vr[a * W + k] = (float)ra[k];
                vp[a * W + k] = (float)ra[k];
                vx[a * W + k] = 0.f;
            }
#pragma unroll
            for (int c = 0; c < NR; ++c)
                rr[c] += ra[3 * c] * ra[3 * c] + ra[3 * c + 1] * ra[3 * c + 1] + ra[3 * c + 2] * ra[3 * c + 2];
        }
        block_sum<NR, NT>(rr, sh);
        bool active[NR];
        bool any = false;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (!done[k] && rr[k] <= tol2 * bnorm2[k]) done[k] = true;
            active[k] = !done[k];
            any = any || active[k];
        }
        if (!any) break;
        if (it_total >= maxit) {
            status = ST_CG_MAXITER;
            break;
        }
        // inner CG: reduce the FP32 residual by 1e-3 (or to the final tolerance)
        double rr0[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) rr0[k] = rr[k];
        for (;;) {
            bool anyi = false;
#pragma unroll
            for (int k = 0; k < NR; ++k) anyi = anyi || active[k];
            if (!anyi) break;
            if (it_total >= maxit) break;
            ++it_total;
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
                        apply_B(nA, g, pa[3 * c] - Po[3 * c], pa[3 * c + 1] - Po[3 * c + 1],
                                pa[3 * c + 2] - Po[3 * c + 2], wx, wy, wz);
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
                    pq[c] += (double)pa[3 * c] * q[3 * c] + (double)pa[3 * c + 1] * q[3 * c + 1] +
                             (double)pa[3 * c + 2] * q[3 * c + 2];
            }
            block_sum<NR, NT>(pq, sh);
            float alpha[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                alpha[k] = 0.f;
                if (active[k]) {
                    if (!(pq[k] > 0.0)) {
                        active[k] = false;
                        done[k] = true;
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
                    if (rn[k] <= 1e-6 * rr0[k] || rn[k] <= 0.25 * tol2 * bnorm2[k]) active[k] = false;
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
        // x += d
#pragma unroll 1
        for (int64_t a = tid; a < nf; a += NT)
#pragma unroll
            for (int k = 0; k < W; ++k) xb[a * W + k] += (double)vx[a * W + k];
        __syncthreads();
        if (outer == 7) {
            bool left = false;
#pragma unroll
            for (int k = 0; k < NR; ++k) left = left || !done[k];
            if (left && status == ST_CONVERGED) status = ST_CG_MAXITER;
        }
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
                    if (j < nf) u[p] += xb[j * W + 3 * col + p];
                    if (i < nf) u[p] -= xb[i * W + 3 * col + p];
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
                    for (int p = 0; p < 3; ++p) u[p] = -xb[node * W + p];
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
