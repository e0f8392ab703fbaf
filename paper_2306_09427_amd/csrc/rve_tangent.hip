// Material tangent dsigma/dF and its vector-Jacobian product on the state of
// the last relaxation, by matrix-free conjugate gradients on the free-node
// stiffness K_ff (the paper differentiates the stress by finite differences
// of extra relaxations, Section 3.2; here the same linearisation is solved
// directly at the converged network).
//
// Per fiber, K contributes B_f = a n n^T + g (I - n n^T) with n = d/l,
// a = k_t/L0, g = T/l, so (K u)_a = sum_{fibers at a} B_f (u_a - u_other).
//
// Tangent (one right-hand side per F_kl): the boundary moves by E Xm_b,
// E = e_k e_l, so K_ff dx = -[K (E Xm)]_f with [K (E Xm)]_a =
// sum s_af B_f (E d0_f); then df_b = sum s_bf B_f (E d0_f + dx_j - dx_i) and
// dsigma = (sum_b df_b x_b^T + f_b (E Xm_b)^T) / (J V0) - sigma (F^-1)_lk.
//
// VJP (one right-hand side): with y_b = G x_b on boundary nodes (G = dL/dsigma)
// and u = [0; y], solve K_ff lambda = (K u)_f, then z_b = (K [-lambda; y])_b
// and dL/dF_kl = sum_b (z_b + G^T f_b)_k Xm_b,l / (J V0) - (G:sigma) F^-T_kl.
//
// Work decomposition: one wavefront per (RVE, right-hand side) task, pulled
// from a work counter in longest-first order of the RVEs, so the nine solves
// of one RVE's tangent run as nine independent wavefronts with no workgroup
// synchronisation.  A first kernel
// forms, once per call, the fiber operators (FP64 per fiber, FP32 per
// incidence record) and the block-Jacobi preconditioner.  The incidence of
// the free nodes is stored in ELL chunks of 64 nodes (record s of the chunk's
// lane-th node at s*64 + lane), so the lanes of a wavefront read their
// records with unit stride.
//
// Precision: iterative refinement.  The outer loop keeps the solution, the
// right-hand side and the residual r = b - K x in FP64 (FP64 fiber
// operators); each inner solve K d = r is conjugate gradients preconditioned
// by the inverse 3x3 diagonal blocks of K_ff, with FP32 products and FP64 dot
// products, stopped after a 1e-6 reduction of its residual; x += d.  Plain
// FP32 CG stalls near eps_32 cond(K_ff), about 1e-3 on these networks, which
// refinement removes.  The final assembly is FP64.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rve_internal.h"

namespace rve {

namespace {

constexpr int ST_CONVERGED = 0, ST_NO_STATE = 4, ST_CG_MAXITER = 5, ST_CG_INDEFINITE = 6;
constexpr int kOpsThreads = 256;

__device__ inline double det3(const double* F)
{
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
}

// ------------------------------------------------------------------ static records
// Fills (fiber, other end) of every ELL record of RVE blockIdx.x from the CSR
// incidence; padding records are (-1, nf).
__global__ __launch_bounds__(kOpsThreads) void ell_build_kernel(TangentArgs A)
{
    const int r = blockIdx.x;
    const DevNet& net = A.net;
    const int64_t f0 = net.fib_off[r];
    const int64_t a0 = net.free_off[r], nf = net.free_off[r + 1] - a0;
    const int64_t cf = A.chunk_first[r], nch = A.chunk_first[r + 1] - cf;
#pragma unroll 1
    for (int64_t a = threadIdx.x; a < 64 * nch; a += kOpsThreads) {
        const int64_t c = cf + (a >> 6);
        const int64_t base = A.chunk_rec[c] + (a & 63), w = (A.chunk_rec[c + 1] - A.chunk_rec[c]) >> 6;
        const int64_t e0 = a < nf ? net.inc_off[a0 + a] : 0, deg = a < nf ? net.inc_off[a0 + a + 1] - e0 : 0;
#pragma unroll 1
        for (int64_t s = 0; s < w; ++s) {
            int2 v = make_int2(-1, (int)nf);
            if (s < deg) {
                const uint32_t e = net.inc[e0 + s];
                const int64_t k = e & 0x7fffffffu;
                const uint32_t en = net.ends[f0 + k];
                const int64_t o = (e >> 31) ? (int64_t)(en >> 16) : (int64_t)(en & 0xffff);
                v = make_int2((int)k, (int)(o < nf ? o : nf));
            }
            A.rec_static[base + 64 * s] = v;
        }
    }
}

// ------------------------------------------------------------------ fiber operators
// One workgroup per RVE: n, a = k_t/L0, g = T/l and T of every fiber at the
// last solve's state (FP64), then the FP32 record operators and the inverse
// diagonal blocks of K_ff.
__global__ __launch_bounds__(kOpsThreads) void fiber_ops_kernel(TangentArgs A)
{
    const int r = blockIdx.x;
    if (A.solve_status[r] != 0) return;
    const DevNet& net = A.net;
    const int64_t f0 = net.fib_off[r], nfib = net.fib_off[r + 1] - f0;
    const int64_t a0 = net.free_off[r], nf = net.free_off[r + 1] - a0;
    double F[9];
    for (int k = 0; k < 9; ++k) F[k] = A.F[9 * r + k];
#pragma unroll 1
    for (int64_t k = threadIdx.x; k < nfib; k += kOpsThreads) {
        const double* d0 = net.d0 + 3 * (f0 + k);
        const double L0 = net.L0[f0 + k];
        uint32_t e = net.ends[f0 + k];
        int i = e & 0xffff, j = e >> 16;
        double D[3], dh[3] = {0, 0, 0};
        for (int p = 0; p < 3; ++p) D[p] = F[3 * p] * d0[0] + F[3 * p + 1] * d0[1] + F[3 * p + 2] * d0[2];
        for (int p = 0; p < 3; ++p) {
            if (j < nf) dh[p] += A.h_state[3 * (a0 + j) + p];
            if (i < nf) dh[p] -= A.h_state[3 * (a0 + i) + p];
        }
        double q0 = (D[0] * D[0] + D[1] * D[1] + D[2] * D[2]) - L0 * L0;
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
        double* q64 = A.par64 + 6 * (f0 + k);
        q64[0] = (D[0] + dh[0]) / l;
        q64[1] = (D[1] + dh[1]) / l;
        q64[2] = (D[2] + dh[2]) / l;
        q64[3] = kt / L0;
        q64[4] = T / l;
        q64[5] = T;
    }
    __syncthreads();
    const double* par64 = A.par64 + 6 * f0;
    const int64_t cf = A.chunk_first[r], nch = A.chunk_first[r + 1] - cf;
#pragma unroll 1
    for (int64_t a = threadIdx.x; a < 64 * nch; a += kOpsThreads) {
        const int64_t c = cf + (a >> 6);
        const int64_t base = A.chunk_rec[c] + (a & 63), w = (A.chunk_rec[c + 1] - A.chunk_rec[c]) >> 6;
        double Dg[6] = {0, 0, 0, 0, 0, 0};   // 00 01 02 11 12 22
#pragma unroll 1
        for (int64_t s = 0; s < w; ++s) {
            const int2 st = A.rec_static[base + 64 * s];
            float4 ra = make_float4(0.f, 0.f, 0.f, 0.f);
            int2 rb = make_int2(st.y, 0);
            if (st.x >= 0) {
                const double* q = par64 + 6 * st.x;
                ra = make_float4((float)q[0], (float)q[1], (float)q[2], (float)q[3]);
                rb.y = __float_as_int((float)q[4]);
                const double c2 = q[3] - q[4];
                Dg[0] += q[4] + c2 * q[0] * q[0];
                Dg[1] += c2 * q[0] * q[1];
                Dg[2] += c2 * q[0] * q[2];
                Dg[3] += q[4] + c2 * q[1] * q[1];
                Dg[4] += c2 * q[1] * q[2];
                Dg[5] += q[4] + c2 * q[2] * q[2];
            }
            A.recA[base + 64 * s] = ra;
            A.recB[base + 64 * s] = rb;
        }
        if (a < nf) {
            // inverse by cofactors when the block is positive definite
            // (leading minors), else a scalar 1/max diagonal
            const double m1 = Dg[0], m2 = Dg[0] * Dg[3] - Dg[1] * Dg[1];
            const double c00 = Dg[3] * Dg[5] - Dg[4] * Dg[4], c01 = Dg[2] * Dg[4] - Dg[1] * Dg[5],
                         c02 = Dg[1] * Dg[4] - Dg[2] * Dg[3], c11 = Dg[0] * Dg[5] - Dg[2] * Dg[2],
                         c12 = Dg[1] * Dg[2] - Dg[0] * Dg[4], c22 = m2;
            const double det = Dg[0] * c00 + Dg[1] * c01 + Dg[2] * c02;
            const double tr = Dg[0] + Dg[3] + Dg[5];
            float4 p0, p1;
            if (m1 > 0.0 && m2 > 0.0 && det > 1e-9 * tr * tr * tr) {
                const double id = 1.0 / det;
                p0 = make_float4((float)(c00 * id), (float)(c01 * id), (float)(c02 * id), (float)(c11 * id));
                p1 = make_float4((float)(c12 * id), (float)(c22 * id), 0.f, 0.f);
            } else {
                const double dm = fmax(fmax(fabs(Dg[0]), fabs(Dg[3])), fabs(Dg[5]));
                const float s = dm > 0.0 ? (float)(1.0 / dm) : 1.f;
                p0 = make_float4(s, 0.f, 0.f, s);
                p1 = make_float4(0.f, s, 0.f, 0.f);
            }
            A.precond[2 * (a0 + a)] = p0;
            A.precond[2 * (a0 + a) + 1] = p1;
        }
    }
}

// ------------------------------------------------------------------ wave helpers
template <typename T>
__device__ __forceinline__ T wsum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Values the whole wavefront shares (loaded through vector memory) moved to
// scalar registers.
__device__ __forceinline__ int64_t uni64(int64_t x)
{
    int lo = __builtin_amdgcn_readfirstlane((int)(x & 0xffffffff));
    int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double uniformd(double x)
{
    int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
    int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ void apply_B64(const double* q, double dx, double dy, double dz, double& wx, double& wy,
                                          double& wz)
{
    double dn = q[0] * dx + q[1] * dy + q[2] * dz;
    double c = (q[3] - q[4]) * dn;
    wx = q[4] * dx + c * q[0];
    wy = q[4] * dy + c * q[1];
    wz = q[4] * dz + c * q[2];
}

// z = P v with P the symmetric inverse block (00, 01, 02, 11), (12, 22, -, -)
__device__ __forceinline__ float4 precond_apply(const float4* P, float4 v)
{
    const float4 p0 = P[0], p1 = P[1];
    return make_float4(p0.x * v.x + p0.y * v.y + p0.z * v.z, p0.y * v.x + p0.w * v.y + p1.x * v.z,
                       p0.z * v.x + p1.x * v.y + p1.y * v.z, 0.f);
}

__device__ __forceinline__ double dot3(float4 a, float4 b)
{
    return (double)a.x * b.x + (double)a.y * b.y + (double)a.z * b.z;
}

// ------------------------------------------------------------------ per-RVE context
struct Ctx {
    int64_t f0, nfib, a0, nf, b0;
    const double* par64;
    const int64_t* incoff;
    const uint32_t* ends;
};

__device__ __forceinline__ Ctx make_ctx(const TangentArgs& A, int r)
{
    const DevNet& net = A.net;
    Ctx c;
    c.f0 = uni64(net.fib_off[r]);
    c.nfib = uni64(net.fib_off[r + 1]) - c.f0;
    c.a0 = uni64(net.free_off[r]);
    c.nf = uni64(net.free_off[r + 1]) - c.a0;
    c.b0 = uni64(net.bnd_off[r]);
    c.par64 = A.par64 + 6 * c.f0;
    c.incoff = net.inc_off + c.a0;
    c.ends = net.ends + c.f0;
    return c;
}

// Outputs of a task whose RVE has no converged state.  tid: the caller's
// thread id (opaque in the persistent kernels); the NaN is produced at the
// store so that no constant is kept live across tasks.
template <bool TAN>
__device__ void no_state(const TangentArgs& A, int r, int col, int tid)
{
    if (tid == 0) atomicMax(&A.status[r], ST_NO_STATE);
    if (tid < 9) {
        double nanv = NAN;
        asm volatile("" : "+v"(nanv));
        if (TAN)
            A.out[(int64_t)r * 81 + 9 * tid + col] = nanv;
        else
            A.out[(int64_t)r * 9 + tid] = nanv;
    }
}

// Right-hand side at free node a (FP64).  Tangent: -sum s B_f (e_k d0_l),
// s = +1 at end j, -1 at end i.  VJP: (K u)_a with u = -G x_b on fixed ends.
template <bool TAN>
__device__ __forceinline__ void rhs_node(const TangentArgs& A, const Ctx& c, int64_t a, int kk, int ll,
                                         const double* F, const double* G, double* b)
{
    const DevNet& net = A.net;
    b[0] = b[1] = b[2] = 0.0;
#pragma unroll 1
    for (int64_t e = c.incoff[a]; e < c.incoff[a + 1]; ++e) {
        const uint32_t w = net.inc[e];
        const int64_t k = w & 0x7fffffffu;
        const double* q = c.par64 + 6 * k;
        if (TAN) {
            const double s = ((w >> 31) ? 1.0 : -1.0) * net.d0[3 * (c.f0 + k) + ll];
            const double nk = kk == 0 ? q[0] : (kk == 1 ? q[1] : q[2]);
            const double cc = (q[3] - q[4]) * nk;
            for (int p = 0; p < 3; ++p) b[p] += s * (cc * q[p] + (p == kk ? q[4] : 0.0));
        } else {
            const uint32_t en = c.ends[k];
            const int64_t o = (w >> 31) ? (int64_t)(en >> 16) : (int64_t)(en & 0xffff);
            if (o >= c.nf) {
                const double* Xm = net.Xb + 3 * (c.b0 + (o - c.nf));
                double x[3], y[3];
                for (int p = 0; p < 3; ++p) x[p] = F[3 * p] * Xm[0] + F[3 * p + 1] * Xm[1] + F[3 * p + 2] * Xm[2];
                for (int p = 0; p < 3; ++p) y[p] = -(G[3 * p] * x[0] + G[3 * p + 1] * x[1] + G[3 * p + 2] * x[2]);
                double w3[3];
                apply_B64(q, y[0], y[1], y[2], w3[0], w3[1], w3[2]);
                for (int p = 0; p < 3; ++p) b[p] += w3[p];
            }
        }
    }
}

// FP64 residual b - K x at free node a; x64 holds the solution (entry nf = 0).
__device__ __forceinline__ void residual_node(const TangentArgs& A, const Ctx& c, int64_t a, const double* x64,
                                              const double* b64, bool first, double* ra)
{
    for (int p = 0; p < 3; ++p) ra[p] = b64[3 * a + p];
    if (first) return;
    const double xa[3] = {x64[3 * a], x64[3 * a + 1], x64[3 * a + 2]};
#pragma unroll 1
    for (int64_t e = c.incoff[a]; e < c.incoff[a + 1]; ++e) {
        const uint32_t w = A.net.inc[e];
        const uint32_t en = c.ends[w & 0x7fffffffu];
        int64_t o = (w >> 31) ? (int64_t)(en >> 16) : (int64_t)(en & 0xffff);
        o = o < c.nf ? o : c.nf;
        const double* xo = x64 + 3 * o;
        double w3[3];
        apply_B64(c.par64 + 6 * (w & 0x7fffffffu), xa[0] - xo[0], xa[1] - xo[1], xa[2] - xo[2], w3[0], w3[1], w3[2]);
        for (int p = 0; p < 3; ++p) ra[p] -= w3[p];
    }
}

// Partial sums of the assembly over fibers k0, k0 + stride, ... that have a
// fixed end (FP64).  acc[3p + c] collects sum_b df_b,p x_b,c + f_b,p (E Xm_b)_c
// (tangent) or sum_b (z_b + G^T f_b)_p Xm_b,c (VJP).
template <bool TAN>
__device__ __forceinline__ void assembly_partial(const TangentArgs& A, const Ctx& c, int r, int kk, int ll,
                                                 const double* x64, int64_t k0, int stride, double* acc)
{
    const DevNet& net = A.net;
    double F[9], G[9];
    for (int k = 0; k < 9; ++k) F[k] = A.F[9 * r + k];
    if (!TAN)
        for (int k = 0; k < 9; ++k) G[k] = A.gsigma[9 * r + k];
#pragma unroll
    for (int p = 0; p < 9; ++p) acc[p] = 0.0;
#pragma unroll 1
    for (int64_t k = k0; k < c.nfib; k += stride) {
        const uint32_t en = c.ends[k];
        const int64_t i = en & 0xffff, j = en >> 16;
        if (i < c.nf && j < c.nf) continue;
        const double* q = c.par64 + 6 * k;
        double u[3] = {0.0, 0.0, 0.0};
        if (TAN) {
            const double d0l = net.d0[3 * (c.f0 + k) + ll];
            for (int p = 0; p < 3; ++p) {
                u[p] = p == kk ? d0l : 0.0;
                if (j < c.nf) u[p] += x64[3 * j + p];
                if (i < c.nf) u[p] -= x64[3 * i + p];
            }
        } else {
            // u = [-lambda; y] at the two ends, difference j - i
            for (int end = 0; end < 2; ++end) {
                const int64_t node = end ? j : i;
                const double s = end ? 1.0 : -1.0;
                if (node < c.nf) {
                    for (int p = 0; p < 3; ++p) u[p] -= s * x64[3 * node + p];
                } else {
                    const double* Xm = net.Xb + 3 * (c.b0 + (node - c.nf));
                    double x[3];
                    for (int p = 0; p < 3; ++p) x[p] = F[3 * p] * Xm[0] + F[3 * p + 1] * Xm[1] + F[3 * p + 2] * Xm[2];
                    for (int p = 0; p < 3; ++p) u[p] += s * (G[3 * p] * x[0] + G[3 * p + 1] * x[1] + G[3 * p + 2] * x[2]);
                }
            }
        }
        double w[3];
        apply_B64(q, u[0], u[1], u[2], w[0], w[1], w[2]);
        const double fv[3] = {q[5] * q[0], q[5] * q[1], q[5] * q[2]};
        for (int end = 0; end < 2; ++end) {
            const int64_t node = end ? j : i;
            if (node < c.nf) continue;
            const double s = end ? 1.0 : -1.0;
            const double* Xm = net.Xb + 3 * (c.b0 + (node - c.nf));
            if (TAN) {
                double x[3];
                for (int p = 0; p < 3; ++p) x[p] = F[3 * p] * Xm[0] + F[3 * p + 1] * Xm[1] + F[3 * p + 2] * Xm[2];
                const double xl = ll == 0 ? Xm[0] : (ll == 1 ? Xm[1] : Xm[2]);
                for (int p = 0; p < 3; ++p)
                    for (int cc = 0; cc < 3; ++cc) acc[3 * p + cc] += s * (w[p] * x[cc] + (cc == kk ? fv[p] * xl : 0.0));
            } else {
                double gtf[3];
                for (int p = 0; p < 3; ++p) gtf[p] = G[p] * fv[0] + G[3 + p] * fv[1] + G[6 + p] * fv[2];
                for (int p = 0; p < 3; ++p)
                    for (int cc = 0; cc < 3; ++cc) acc[3 * p + cc] += s * (w[p] + gtf[p]) * Xm[cc];
            }
        }
    }
}

// Final outputs of a task from the summed assembly (one thread).
template <bool TAN>
__device__ void assembly_write(const TangentArgs& A, int r, int col, const double* acc, int status, int64_t iters)
{
    double F[9];
    for (int k = 0; k < 9; ++k) F[k] = A.F[9 * r + k];
    const double J = det3(F);
    const double V0 = A.net.V0[r];
    const double id = 1.0 / J;
    // F^-1 by cofactors
    const double Fi[9] = {(F[4] * F[8] - F[5] * F[7]) * id, (F[2] * F[7] - F[1] * F[8]) * id,
                          (F[1] * F[5] - F[2] * F[4]) * id, (F[5] * F[6] - F[3] * F[8]) * id,
                          (F[0] * F[8] - F[2] * F[6]) * id, (F[2] * F[3] - F[0] * F[5]) * id,
                          (F[3] * F[7] - F[4] * F[6]) * id, (F[1] * F[6] - F[0] * F[7]) * id,
                          (F[0] * F[4] - F[1] * F[3]) * id};
    if (TAN) {
        const int kk = col / 3, ll = col % 3;
        double fi = 0.0;   // (F^-1)_{l k}
        for (int m = 0; m < 9; ++m) fi = m == 3 * ll + kk ? Fi[m] : fi;
        for (int p = 0; p < 9; ++p)
            A.out[(int64_t)r * 81 + 9 * p + col] = acc[p] / (J * V0) - A.sigma[9 * r + p] * fi;
    } else {
        double gs = 0.0;
        for (int p = 0; p < 9; ++p) gs += A.gsigma[9 * r + p] * A.sigma[9 * r + p];
        for (int p = 0; p < 9; ++p) {
            const int k2 = p / 3, l2 = p % 3;
            A.out[(int64_t)r * 9 + p] = acc[p] / (J * V0) - gs * Fi[3 * l2 + k2];
        }
    }
    if (status != ST_CONVERGED) atomicMax(&A.status[r], status);
    atomicAdd(&A.iters[r], (unsigned long long)iters);
}

// ------------------------------------------------------------------ workgroup sums
struct CgRed {
    double s[2][3][16];   // per-wavefront partial sums, alternating buffers
};

template <int NW>
__device__ __forceinline__ void block_sum3(CgRed& red, int parity, double& a, double& b, double& c)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    a = wsum(a);
    b = wsum(b);
    c = wsum(c);
    if (lane == 0) {
        red.s[parity][0][wave] = a;
        red.s[parity][1][wave] = b;
        red.s[parity][2][wave] = c;
    }
    __syncthreads();
    double x = 0.0, y = 0.0, z = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        x += red.s[parity][0][i];
        y += red.s[parity][1][i];
        z += red.s[parity][2][i];
    }
    a = uniformd(x);
    b = uniformd(y);
    c = uniformd(z);
}

// ------------------------------------------------------------------ streamed tasks
// A task is (RVE r, right-hand side col): col = 3k + l for the tangent, 0 for
// the VJP.  One workgroup of T threads (T = 64: one wavefront); wavefront w
// takes ELL chunks w, w + T/64, ... and lane = node within its chunk.
// Solver vectors live in the workgroup's global slot (any RVE size).
template <bool TAN, int T>
__device__ void cg_stream_task(const TangentArgs& A, int r, int col, CgRed& red)
{
    constexpr int NW = T / 64;
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int parity = 0;
    // sums over the workgroup (every thread gets the same totals)
    auto sum2 = [&](double& x, double& y) __attribute__((always_inline)) {
        if (T == 64) {
            x = uniformd(wsum(x));
            y = uniformd(wsum(y));
        } else {
            double z = 0.0;
            block_sum3<NW>(red, parity, x, y, z);
            parity ^= 1;
        }
    };
    if (__builtin_amdgcn_readfirstlane(A.solve_status[r]) != 0) {
        no_state<TAN>(A, r, col, tid);
        return;
    }
    const Ctx c = make_ctx(A, r);
    const int64_t nf = c.nf;
    const int kk = col / 3, ll = col % 3;
    const float4* Pc = A.precond + 2 * c.a0;
    const int64_t cf = uni64(A.chunk_first[r]), nch = uni64(A.chunk_first[r + 1]) - cf;
    const float4* recA = A.recA;
    const int2* recB = A.recB;

    // slot workspace: FP64 x and b (3 per node), FP32 p, q, r, d, z (float4
    // per node); entry nf of p and x is the zero vector of fixed ends
    const int64_t S = A.slot_nodes;
    double* x64 = A.slot_ws64 + (int64_t)blockIdx.x * 6 * S;
    double* b64 = x64 + 3 * S;
    float4* vp = A.slot_ws32 + (int64_t)blockIdx.x * 5 * S;
    float4* vq = vp + S;
    float4* vr = vq + S;
    float4* vd = vr + S;
    float4* vz = vd + S;
    if (tid == 0) vp[nf] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (tid < 3) x64[3 * nf + tid] = 0.0;

    double bb = 0.0;
    {
        double F[9], G[9];
        for (int k = 0; k < 9; ++k) F[k] = A.F[9 * r + k];
        if (!TAN)
            for (int k = 0; k < 9; ++k) G[k] = A.gsigma[9 * r + k];
#pragma unroll 1
        for (int64_t a = tid; a < nf; a += T) {
            double b[3];
            rhs_node<TAN>(A, c, a, kk, ll, F, G, b);
            for (int p = 0; p < 3; ++p) {
                b64[3 * a + p] = b[p];
                x64[3 * a + p] = 0.0;
            }
            bb += b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
        }
    }
    {
        double u = 0.0;
        sum2(bb, u);
    }
    __syncthreads();

    int status = ST_CONVERGED;
    const double tol2 = A.cg_tol * A.cg_tol;
    const int64_t maxit = A.cg_max > 0 ? A.cg_max : 6 * nf + 100;
    int64_t it_total = 0;
    bool done = !(bb > 0.0);
    for (int outer = 0; outer < 8 && !done; ++outer) {
        // FP64 residual r = b - K x of the FP64 solution; z = P r, p = z
        double rr = 0.0, rz = 0.0;
#pragma unroll 1
        for (int64_t a = tid; a < nf; a += T) {
            double ra[3];
            residual_node(A, c, a, x64, b64, outer == 0, ra);
            const float4 r4 = make_float4((float)ra[0], (float)ra[1], (float)ra[2], 0.f);
            const float4 z4 = precond_apply(Pc + 2 * a, r4);
            vr[a] = r4;
            vz[a] = z4;
            vp[a] = z4;
            vd[a] = make_float4(0.f, 0.f, 0.f, 0.f);
            rr += ra[0] * ra[0] + ra[1] * ra[1] + ra[2] * ra[2];
            rz += dot3(r4, z4);
        }
        sum2(rr, rz);
        __syncthreads();
        if (rr <= tol2 * bb) {
            done = true;
            break;
        }
        if (it_total >= maxit) {
            status = ST_CG_MAXITER;
            break;
        }
        // inner preconditioned CG with FP32 products
        const double rr0 = rr;
        for (;;) {
            if (it_total >= maxit) break;
            ++it_total;
            // q = K p over the ELL records of each chunk
            double pq = 0.0;
#pragma unroll 1
            for (int64_t ch = wave; ch < nch; ch += NW) {
                const int64_t a = 64 * ch + lane;
                const int64_t c0 = uni64(A.chunk_rec[cf + ch]), w = (uni64(A.chunk_rec[cf + ch + 1]) - c0) >> 6;
                const int64_t rb = c0 + lane;
                if (a < nf) {
                    const float4 pa = vp[a];
                    float qx = 0.f, qy = 0.f, qz = 0.f;
                    // w is a multiple of 4: issue 4 records' loads, then their gathers
#pragma unroll 1
                    for (int64_t s0 = 0; s0 < w; s0 += 4) {
                        float4 nA[4];
                        int2 ob[4];
                        float4 po[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            nA[u] = recA[rb + 64 * (s0 + u)];
                            ob[u] = recB[rb + 64 * (s0 + u)];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) po[u] = vp[ob[u].x];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const float g = __int_as_float(ob[u].y);
                            const float dx = pa.x - po[u].x, dy = pa.y - po[u].y, dz = pa.z - po[u].z;
                            const float cn = (nA[u].w - g) * (nA[u].x * dx + nA[u].y * dy + nA[u].z * dz);
                            qx += fmaf(g, dx, cn * nA[u].x);
                            qy += fmaf(g, dy, cn * nA[u].y);
                            qz += fmaf(g, dz, cn * nA[u].z);
                        }
                    }
                    vq[a] = make_float4(qx, qy, qz, 0.f);
                    pq += (double)pa.x * qx + (double)pa.y * qy + (double)pa.z * qz;
                }
            }
            {
                double u = 0.0;
                sum2(pq, u);
            }
            if (!(pq > 0.0)) {
                status = ST_CG_INDEFINITE;
                done = true;
                break;
            }
            const float alpha = (float)(rz / pq);
            double rn = 0.0, rzn = 0.0;
#pragma unroll 1
            for (int64_t a = tid; a < nf; a += T) {
                const float4 pa = vp[a], qa = vq[a];
                float4 da = vd[a], ra = vr[a];
                da.x = fmaf(alpha, pa.x, da.x);
                da.y = fmaf(alpha, pa.y, da.y);
                da.z = fmaf(alpha, pa.z, da.z);
                ra.x = fmaf(-alpha, qa.x, ra.x);
                ra.y = fmaf(-alpha, qa.y, ra.y);
                ra.z = fmaf(-alpha, qa.z, ra.z);
                const float4 za = precond_apply(Pc + 2 * a, ra);
                vd[a] = da;
                vr[a] = ra;
                vz[a] = za;
                rn += dot3(ra, ra);
                rzn += dot3(ra, za);
            }
            sum2(rn, rzn);
            if (rn <= 1e-6 * rr0 || rn <= 0.25 * tol2 * bb) break;
            const float beta = (float)(rzn / rz);
            rz = rzn;
#pragma unroll 1
            for (int64_t a = tid; a < nf; a += T) {
                const float4 za = vz[a];
                float4 pa = vp[a];
                pa.x = fmaf(beta, pa.x, za.x);
                pa.y = fmaf(beta, pa.y, za.y);
                pa.z = fmaf(beta, pa.z, za.z);
                vp[a] = pa;
            }
            __syncthreads();
        }
        // x += d
        __syncthreads();
#pragma unroll 1
        for (int64_t a = tid; a < nf; a += T) {
            const float4 da = vd[a];
            x64[3 * a] += (double)da.x;
            x64[3 * a + 1] += (double)da.y;
            x64[3 * a + 2] += (double)da.z;
        }
        __syncthreads();
        if (outer == 7 && !done && status == ST_CONVERGED) status = ST_CG_MAXITER;
    }

    double acc[9];
    assembly_partial<TAN>(A, c, r, kk, ll, x64, tid, T, acc);
    if (T == 64) {
#pragma unroll
        for (int p = 0; p < 9; ++p) acc[p] = wsum(acc[p]);
    } else {
#pragma unroll
        for (int p = 0; p < 9; p += 3) {
            block_sum3<NW>(red, parity, acc[p], acc[p + 1], acc[p + 2]);
            parity ^= 1;
        }
    }
    if (tid == 0) assembly_write<TAN>(A, r, col, acc, status, it_total);
    __syncthreads();
}

template <bool TAN, int T>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(4))) void cg_stream_kernel(TangentArgs A)
{
    __shared__ CgRed red;
    __shared__ int task;
    constexpr int per = TAN ? 9 : 1;
    const int64_t n_tasks = A.n_order * per;
    for (;;) {
        if (threadIdx.x == 0) task = atomicAdd(A.queue, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(task);
        __syncthreads();
        if (t >= n_tasks) break;
        cg_stream_task<TAN, T>(A, __builtin_amdgcn_readfirstlane(A.order[t / per]), t % per, red);
    }
}

// ------------------------------------------------------------------ resident tasks
// One workgroup of T threads per task; thread tid owns free nodes
// tid + T k (k < SN), so wavefront w owns ELL chunks w + (T/64) k.  The
// solver vectors of the inner solve stay in registers, the vector the
// matrix-free product gathers is exchanged through LDS.
//
// The inner solve is plain preconditioned CG with a fresh product q = K p
// every iteration: three workgroup barriers per iteration (p exchanged, p.q
// summed, (r,r) and (r,z) summed).  Recurrence forms with one reduction (the
// Chronopoulos-Gear update of q) lose the sign of p.Kp to FP32 cancellation
// on these ill-conditioned systems.
template <bool TAN, int T, int SN, bool PL>
__device__ void cg_res_task(const TangentArgs& A, int r, int col, float4* zl, CgRed& red)
{
    constexpr int NW = T / 64;
    // thread id made opaque per task: otherwise the compiler hoists every
    // per-thread address of every slot out of the persistent task loop and
    // keeps them live (spilled) across the whole kernel
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (__builtin_amdgcn_readfirstlane(A.solve_status[r]) != 0) {
        no_state<TAN>(A, r, col, tid);
        return;
    }
    const Ctx c = make_ctx(A, r);
    const int64_t nf = c.nf;
    const int kk = col / 3, ll = col % 3;
    const float4* Pc = A.precond + 2 * c.a0;
    const int64_t cf = uni64(A.chunk_first[r]);
    const int64_t S = A.slot_nodes;
    double* x64 = A.slot_ws64 + (int64_t)blockIdx.x * 8 * S;   // x, b (3 S each), d32 (S float4)
    double* b64 = x64 + 3 * S;

    // ELL chunk of each slot (uniform over the wavefront); width 0 past the
    // end.  Record offsets are 32-bit, relative to the RVE's first record.
    const int64_t rec0 = uni64(A.chunk_rec[cf]);
    const float4* recA = A.recA + rec0;
    const int2* recB = A.recB + rec0;
    int rb[SN];
    int wd[SN];
#pragma unroll
    for (int k = 0; k < SN; ++k) {
        const int64_t ch = wave + NW * k;
        rb[k] = 0;
        wd[k] = 0;
        if (64 * ch < nf) {
            const int64_t c0 = uni64(A.chunk_rec[cf + ch]);
            wd[k] = (int)((uni64(A.chunk_rec[cf + ch + 1]) - c0) >> 6);
            rb[k] = (int)(c0 - rec0) + lane;
        }
    }
    int parity = 0;

    // right-hand side (FP64)
    double bb = 0.0;
    {
        double F[9], G[9];
        for (int k = 0; k < 9; ++k) F[k] = A.F[9 * r + k];
        if (!TAN)
            for (int k = 0; k < 9; ++k) G[k] = A.gsigma[9 * r + k];
#pragma unroll 1
        for (int k = 0; k < SN; ++k) {
            const int64_t a = tid + T * k;
            if (a < nf) {
                double b[3];
                rhs_node<TAN>(A, c, a, kk, ll, F, G, b);
                for (int p = 0; p < 3; ++p) {
                    b64[3 * a + p] = b[p];
                    x64[3 * a + p] = 0.0;
                }
                bb += b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
            }
        }
        if (tid < 3) x64[3 * nf + tid] = 0.0;
    }
    {
        double u0 = 0.0, u1 = 0.0;
        block_sum3<NW>(red, parity, bb, u0, u1);
        parity ^= 1;
    }

    // Register state per node slot: r and q; unless PL also z, p and d.
    // PL (lean, for large SN): p lives only in LDS, the correction d in the
    // workgroup's global slot (d32), and z = P r is recomputed where needed.
    float R[SN][3], Q[SN][3];
    float Z[PL ? 1 : SN][3], P[PL ? 1 : SN][3], D[PL ? 1 : SN][3];
    float4* d32 = reinterpret_cast<float4*>(b64 + 3 * S);   // [S] (PL only)
    auto own_p = [&](int k) __attribute__((always_inline)) -> float4 {
        return PL ? zl[tid + T * k] : make_float4(P[k][0], P[k][1], P[k][2], 0.f);
    };
    // z = P_a r for slot k (block reloaded every time: keeping the blocks of
    // all slots live across the loop costs 8 registers per slot)
    auto precond_r = [&](int k) __attribute__((always_inline)) -> float4 {
        const int64_t a = tid + T * k;
        float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f), p1 = p0;
        if (a < nf) {
            const float4* pp = Pc + 2 * a;
            asm volatile("" : "+v"(pp));
            p0 = pp[0];
            p1 = pp[1];
        }
        return make_float4(p0.x * R[k][0] + p0.y * R[k][1] + p0.z * R[k][2],
                           p0.y * R[k][0] + p0.w * R[k][1] + p1.x * R[k][2],
                           p0.z * R[k][0] + p1.x * R[k][1] + p1.y * R[k][2], 0.f);
    };
    int status = ST_CONVERGED;
    // per-task copy: a kernel-lifetime value would be kept live across tasks
    double cgt = A.cg_tol;
    asm volatile("" : "+v"(cgt));
    const double tol2 = uniformd(cgt * cgt);
    const int64_t maxit = A.cg_max > 0 ? A.cg_max : 6 * nf + 100;
    int64_t it_total = 0;
    bool done = !(bb > 0.0);
    for (int outer = 0; outer < 8 && !done; ++outer) {
        // thread id opaque per phase: no per-thread address is hoisted out of
        // the loops and kept live across them
        asm volatile("" : "+v"(tid));
        // FP64 residual of the FP64 solution (x64 complete: barrier above);
        // d = 0, p = z = P r
        double rr = 0.0, rz = 0.0;
#pragma unroll
        for (int k = 0; k < SN; ++k) {
            const int64_t a = tid + T * k;
            double ra[3] = {0.0, 0.0, 0.0};
            if (a < nf) residual_node(A, c, a, x64, b64, outer == 0, ra);
            for (int p = 0; p < 3; ++p) {
                R[k][p] = (float)ra[p];
                Q[k][p] = 0.f;
            }
            rr += ra[0] * ra[0] + ra[1] * ra[1] + ra[2] * ra[2];
            const float4 z = precond_r(k);
            rz += (double)R[k][0] * z.x + (double)R[k][1] * z.y + (double)R[k][2] * z.z;
            if (PL) {
                zl[tid + T * k] = z;
                if (a < nf) d32[a] = make_float4(0.f, 0.f, 0.f, 0.f);
            } else {
                Z[k][0] = P[k][0] = z.x;
                Z[k][1] = P[k][1] = z.y;
                Z[k][2] = P[k][2] = z.z;
                D[k][0] = D[k][1] = D[k][2] = 0.f;
            }
        }
        {
            double u0 = 0.0;
            block_sum3<NW>(red, parity, rr, rz, u0);
            parity ^= 1;
        }
        if (rr <= tol2 * bb) {
            done = true;
            break;
        }
        if (it_total >= maxit) {
            status = ST_CG_MAXITER;
            break;
        }
        // inner preconditioned CG (FP32 vectors, p exchanged through LDS):
        // q = K p, alpha = rz / p.q, d += alpha p, r -= alpha q, z = P r,
        // beta = r.z / rz, p = z + beta p
        const double rr0 = rr;
        for (;;) {
            if (it_total >= maxit) break;
            ++it_total;
            asm volatile("" : "+v"(tid));
            if (!PL) {
#pragma unroll
                for (int k = 0; k < SN; ++k) zl[tid + T * k] = make_float4(P[k][0], P[k][1], P[k][2], 0.f);
            }
            __syncthreads();
            double pq = 0.0;
#pragma unroll
            for (int k = 0; k < SN; ++k) {
                const float4 pk = own_p(k);
                float sx = 0.f, sy = 0.f, sz = 0.f;
                // records in groups of RB (chunk widths are multiples of 4)
                constexpr int RB = SN > 2 ? 2 : 4;
#pragma unroll 1
                for (int s0 = 0; s0 < wd[k]; s0 += RB) {
                    float4 nA[RB];
                    int2 ob[RB];
#pragma unroll
                    for (int u = 0; u < RB; ++u) {
                        nA[u] = recA[rb[k] + 64 * (s0 + u)];
                        ob[u] = recB[rb[k] + 64 * (s0 + u)];
                    }
#pragma unroll
                    for (int u = 0; u < RB; ++u) {
                        const float4 po = zl[ob[u].x];
                        const float g = __int_as_float(ob[u].y);
                        const float dx = pk.x - po.x, dy = pk.y - po.y, dz = pk.z - po.z;
                        const float cn = (nA[u].w - g) * (nA[u].x * dx + nA[u].y * dy + nA[u].z * dz);
                        sx += fmaf(g, dx, cn * nA[u].x);
                        sy += fmaf(g, dy, cn * nA[u].y);
                        sz += fmaf(g, dz, cn * nA[u].z);
                    }
                }
                Q[k][0] = sx;
                Q[k][1] = sy;
                Q[k][2] = sz;
                pq += (double)pk.x * sx + (double)pk.y * sy + (double)pk.z * sz;
            }
            {
                double u0 = 0.0, u1 = 0.0;
                block_sum3<NW>(red, parity, pq, u0, u1);
                parity ^= 1;
            }
            if (!(pq > 0.0)) {
                status = ST_CG_INDEFINITE;
                done = true;
                break;
            }
            const float af = (float)(rz / pq);
            double rn = 0.0, rzn = 0.0;
#pragma unroll
            for (int k = 0; k < SN; ++k) {
                const float4 pk = own_p(k);
                if (PL) {
                    const int64_t a = tid + T * k;
                    if (a < nf) {
                        float4 d = d32[a];
                        d.x = fmaf(af, pk.x, d.x);
                        d.y = fmaf(af, pk.y, d.y);
                        d.z = fmaf(af, pk.z, d.z);
                        d32[a] = d;
                    }
                } else {
                    D[k][0] = fmaf(af, pk.x, D[k][0]);
                    D[k][1] = fmaf(af, pk.y, D[k][1]);
                    D[k][2] = fmaf(af, pk.z, D[k][2]);
                }
                for (int p = 0; p < 3; ++p) R[k][p] = fmaf(-af, Q[k][p], R[k][p]);
                const float4 z = precond_r(k);
                if (!PL) {
                    Z[k][0] = z.x;
                    Z[k][1] = z.y;
                    Z[k][2] = z.z;
                }
                rn += (double)R[k][0] * R[k][0] + (double)R[k][1] * R[k][1] + (double)R[k][2] * R[k][2];
                rzn += (double)R[k][0] * z.x + (double)R[k][1] * z.y + (double)R[k][2] * z.z;
            }
            {
                double u0 = 0.0;
                block_sum3<NW>(red, parity, rn, rzn, u0);
                parity ^= 1;
            }
            if (rn <= 1e-6 * rr0 || rn <= 0.25 * tol2 * bb) break;
            const float bf = (float)(rzn / rz);
            rz = rzn;
#pragma unroll
            for (int k = 0; k < SN; ++k) {
                if (PL) {
                    const float4 z = precond_r(k);
                    const float4 pk = zl[tid + T * k];
                    zl[tid + T * k] = make_float4(fmaf(bf, pk.x, z.x), fmaf(bf, pk.y, z.y), fmaf(bf, pk.z, z.z), 0.f);
                } else {
                    for (int p = 0; p < 3; ++p) P[k][p] = fmaf(bf, P[k][p], Z[k][p]);
                }
            }
        }
        // x += d
        asm volatile("" : "+v"(tid));
#pragma unroll
        for (int k = 0; k < SN; ++k) {
            const int64_t a = tid + T * k;
            if (a < nf) {
                if (PL) {
                    const float4 d = d32[a];
                    x64[3 * a] += (double)d.x;
                    x64[3 * a + 1] += (double)d.y;
                    x64[3 * a + 2] += (double)d.z;
                } else {
                    for (int p = 0; p < 3; ++p) x64[3 * a + p] += (double)D[k][p];
                }
            }
        }
        __syncthreads();
        if (outer == 7 && !done && status == ST_CONVERGED) status = ST_CG_MAXITER;
    }

    // assembly (x64 complete: barrier above, or no update since the RHS sum)
    double acc[9];
    assembly_partial<TAN>(A, c, r, kk, ll, x64, tid, T, acc);
    double tot[9];
#pragma unroll
    for (int p = 0; p < 9; p += 3) {
        double a1 = acc[p], a2 = acc[p + 1], a3 = acc[p + 2];
        block_sum3<NW>(red, parity, a1, a2, a3);
        parity ^= 1;
        tot[p] = a1;
        tot[p + 1] = a2;
        tot[p + 2] = a3;
    }
    if (tid == 0) assembly_write<TAN>(A, r, col, tot, status, it_total);
    __syncthreads();
}

template <bool TAN, int T, int SN, bool PL>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(4))) void cg_res_kernel(TangentArgs A)
{
    extern __shared__ float4 zl[];   // [T * SN + 1]; the last entry stays zero
    __shared__ CgRed red;
    __shared__ int task;
    if (threadIdx.x == 0) zl[T * SN] = make_float4(0.f, 0.f, 0.f, 0.f);
    constexpr int per = TAN ? 9 : 1;
    const int64_t n_tasks = A.n_order * per;
    for (;;) {
        if (threadIdx.x == 0) task = atomicAdd(A.queue, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(task);
        __syncthreads();
        if (t >= n_tasks) break;
        cg_res_task<TAN, T, SN, PL>(A, __builtin_amdgcn_readfirstlane(A.order[t / per]), t % per, zl, red);
    }
}

// ------------------------------------------------------------------ blocked tangent tasks
// Tangent only: one workgroup solves the three right-hand sides F_k0, F_k1,
// F_k2 of one column group k together.  Every ELL record is read once per
// iteration for the three products, and every workgroup reduction carries
// the three columns' sums, so one record read and one barrier serve three
// solves.  Per column the arithmetic is that of cg_res_task, in the same
// order and with the same workgroup sums, so each column's result equals
// the per-column kernel's bitwise.  A column whose inner solve has met its
// criterion (or has ended) makes no further update while the others finish
// theirs; then the columns of the round take the refinement step x += d
// together.  p of each column lives in LDS, its correction d in the
// workgroup's global slot, z = P r is recomputed where needed.
constexpr int kBlk = kTanBlkRhs;

struct BlkRed {
    double s[2][2 * kBlk][16];   // per-wavefront partial sums, alternating buffers
};

// Workgroup sums of N values; each value is summed exactly as block_sum3
// sums it (wavefront sum, then the wavefronts in order).
template <int NW, int N>
__device__ __forceinline__ void block_sum_n(BlkRed& red, int parity, double (&v)[N])
{
    static_assert(N <= 2 * kBlk, "too many values");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double w = wsum(v[i]);
        if (lane == 0) red.s[parity][i][wave] = w;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double x = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) x += red.s[parity][i][q];
        v[i] = uniformd(x);
    }
}

template <int T, int SN, int BLK_RB>
__device__ void cg_blk_task(const TangentArgs& A, int r, int grp, float4* zl, BlkRed& red)
{
    constexpr int NW = T / 64;
    constexpr int ZS = T * SN + 1;   // LDS entries of one column's p
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (__builtin_amdgcn_readfirstlane(A.solve_status[r]) != 0) {
        // as no_state, with the opaque thread id (nothing kept live across tasks)
        if (tid == 0) atomicMax(&A.status[r], ST_NO_STATE);
        if (tid < 9) {
            // one double per store (a vector store would keep a NaN tuple live)
#pragma unroll 1
            for (int j = 0; j < kBlk; ++j) {
                double nanv = NAN;
                asm volatile("" : "+v"(nanv));
                A.out[(int64_t)r * 81 + 9 * tid + kBlk * grp + j] = nanv;
            }
        }
        return;
    }
    const Ctx c = make_ctx(A, r);
    const int64_t nf = c.nf;
    const int kk = grp;
    const float4* Pc = A.precond + 2 * c.a0;
    const int64_t cf = uni64(A.chunk_first[r]);
    const int64_t S = A.slot_nodes;
    // slot: x, b (FP64, 3 S each), then d and q = K p (FP32 float4, S each)
    // per column
    double* ws = A.slot_ws64 + (int64_t)blockIdx.x * 10 * kBlk * S;
    auto x64 = [&](int j) __attribute__((always_inline)) { return ws + 6 * S * j; };
    auto b64 = [&](int j) __attribute__((always_inline)) { return ws + 6 * S * j + 3 * S; };
    float4* d32 = reinterpret_cast<float4*>(ws + 6 * S * kBlk);
    float4* q32 = d32 + S * kBlk;
    const int64_t rec0 = uni64(A.chunk_rec[cf]);
    const float4* recA = A.recA + rec0;
    const int2* recB = A.recB + rec0;
    int rb[SN];
    int wd[SN];
#pragma unroll
    for (int k = 0; k < SN; ++k) {
        const int64_t ch = wave + NW * k;
        rb[k] = 0;
        wd[k] = 0;
        if (64 * ch < nf) {
            const int64_t c0 = uni64(A.chunk_rec[cf + ch]);
            wd[k] = (int)((uni64(A.chunk_rec[cf + ch + 1]) - c0) >> 6);
            rb[k] = (int)(c0 - rec0) + lane;
        }
    }
    int parity = 0;

    // right-hand sides (FP64)
    double bb[kBlk];
    {
        double F[9], G[9];
        for (int k = 0; k < 9; ++k) F[k] = A.F[9 * r + k];
#pragma unroll
        for (int j = 0; j < kBlk; ++j) bb[j] = 0.0;
#pragma unroll 1
        for (int k = 0; k < SN; ++k) {
            const int64_t a = tid + T * k;
            if (a < nf) {
#pragma unroll 1
                for (int j = 0; j < kBlk; ++j) {
                    double b[3];
                    rhs_node<true>(A, c, a, kk, j, F, G, b);
                    for (int p = 0; p < 3; ++p) {
                        b64(j)[3 * a + p] = b[p];
                        x64(j)[3 * a + p] = 0.0;
                    }
                    bb[j] += b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
                }
            }
        }
        if (tid < 3)
            for (int j = 0; j < kBlk; ++j) x64(j)[3 * nf + tid] = 0.0;
    }
    block_sum_n<NW>(red, parity, bb);
    parity ^= 1;

    float R[kBlk][SN][3];
    auto own_p = [&](int j, int k) __attribute__((always_inline)) -> float4 { return zl[ZS * j + tid + T * k]; };
    // inverse block of slot k (reloaded where needed, as in cg_res_task)
    auto pblock = [&](int k, float4& p0, float4& p1) __attribute__((always_inline)) {
        const int64_t a = tid + T * k;
        p0 = make_float4(0.f, 0.f, 0.f, 0.f);
        p1 = p0;
        if (a < nf) {
            const float4* pp = Pc + 2 * a;
            asm volatile("" : "+v"(pp));
            p0 = pp[0];
            p1 = pp[1];
        }
    };
    auto papply = [&](const float4& p0, const float4& p1, const float* v) __attribute__((always_inline)) -> float4 {
        return make_float4(p0.x * v[0] + p0.y * v[1] + p0.z * v[2], p0.y * v[0] + p0.w * v[1] + p1.x * v[2],
                           p0.z * v[0] + p1.x * v[1] + p1.y * v[2], 0.f);
    };
    int status[kBlk];
    int it_total[kBlk];
    // bit j: column j's solve has ended (converged, cap, indefinite) / is in
    // this round's inner solve / took part in this round
    unsigned fin = 0u, act = 0u, in_round = 0u;
    // per-task copy: a kernel-lifetime value would be kept live across tasks
    double cgt = A.cg_tol;
    asm volatile("" : "+v"(cgt));
    const double tol2 = uniformd(cgt * cgt);
    const int64_t maxit = A.cg_max > 0 ? A.cg_max : 6 * nf + 100;
#pragma unroll
    for (int j = 0; j < kBlk; ++j) {
        status[j] = ST_CONVERGED;
        it_total[j] = 0;
        if (!(bb[j] > 0.0)) fin |= 1u << j;
    }
    for (int outer = 0; outer < 8; ++outer) {
        // thread id opaque per phase: no per-thread address of any column is
        // hoisted out of the loops and kept live
        asm volatile("" : "+v"(tid));
        if (fin == (1u << kBlk) - 1u) break;
        // FP64 residuals of the columns still running; d = 0, p = z = P r
        double sums[2 * kBlk];
#pragma unroll
        for (int i = 0; i < 2 * kBlk; ++i) sums[i] = 0.0;
#pragma unroll
        for (int k = 0; k < SN; ++k) {
            const int64_t a = tid + T * k;
            float4 p0, p1;
            pblock(k, p0, p1);
#pragma unroll
            for (int j = 0; j < kBlk; ++j) {
                if (fin & (1u << j)) continue;
                double ra[3] = {0.0, 0.0, 0.0};
                if (a < nf) residual_node(A, c, a, x64(j), b64(j), outer == 0, ra);
                for (int p = 0; p < 3; ++p) R[j][k][p] = (float)ra[p];
                sums[j] += ra[0] * ra[0] + ra[1] * ra[1] + ra[2] * ra[2];
                const float4 z = papply(p0, p1, R[j][k]);
                sums[kBlk + j] += (double)R[j][k][0] * z.x + (double)R[j][k][1] * z.y + (double)R[j][k][2] * z.z;
                zl[ZS * j + tid + T * k] = z;
                if (a < nf) d32[S * j + a] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        block_sum_n<NW>(red, parity, sums);
        parity ^= 1;
        double rz[kBlk], rr0[kBlk];
        act = 0u;
#pragma unroll
        for (int j = 0; j < kBlk; ++j) {
            rz[j] = sums[kBlk + j];
            rr0[j] = sums[j];
            if (fin & (1u << j)) continue;
            if (sums[j] <= tol2 * bb[j]) {
                fin |= 1u << j;   // converged
                continue;
            }
            if (it_total[j] >= maxit) {
                status[j] = ST_CG_MAXITER;
                fin |= 1u << j;
                continue;
            }
            act |= 1u << j;
        }
        in_round = act;
        for (;;) {
#pragma unroll
            for (int j = 0; j < kBlk; ++j) {
                if ((act & (1u << j)) && it_total[j] >= maxit) act &= ~(1u << j);
                if (act & (1u << j)) ++it_total[j];
            }
            if (!act) break;
            asm volatile("" : "+v"(tid));
            __syncthreads();
            // q = K p for the active columns: each record read once
            double pq[kBlk];
#pragma unroll
            for (int i = 0; i < kBlk; ++i) pq[i] = 0.0;
#pragma unroll
            for (int k = 0; k < SN; ++k) {
                float sx[kBlk], sy[kBlk], sz[kBlk];
                float px[kBlk], py[kBlk], pz[kBlk];
#pragma unroll
                for (int j = 0; j < kBlk; ++j) {
                    sx[j] = sy[j] = sz[j] = 0.f;
                    const float4 q = (act & (1u << j)) ? own_p(j, k) : make_float4(0.f, 0.f, 0.f, 0.f);
                    px[j] = q.x;
                    py[j] = q.y;
                    pz[j] = q.z;
                }
                constexpr int RB = BLK_RB;
#pragma unroll 1
                for (int s0 = 0; s0 < wd[k]; s0 += RB) {
                    float4 nA[RB];
                    int2 ob[RB];
#pragma unroll
                    for (int u = 0; u < RB; ++u) {
                        nA[u] = recA[rb[k] + 64 * (s0 + u)];
                        ob[u] = recB[rb[k] + 64 * (s0 + u)];
                    }
#pragma unroll
                    for (int j = 0; j < kBlk; ++j) {
                        if (!(act & (1u << j))) continue;
#pragma unroll
                        for (int u = 0; u < RB; ++u) {
                            const float4 po = zl[ZS * j + ob[u].x];
                            const float g = __int_as_float(ob[u].y);
                            const float dx = px[j] - po.x, dy = py[j] - po.y, dz = pz[j] - po.z;
                            const float cn = (nA[u].w - g) * (nA[u].x * dx + nA[u].y * dy + nA[u].z * dz);
                            sx[j] += fmaf(g, dx, cn * nA[u].x);
                            sy[j] += fmaf(g, dy, cn * nA[u].y);
                            sz[j] += fmaf(g, dz, cn * nA[u].z);
                        }
                    }
                }
                const int64_t a = tid + T * k;
#pragma unroll
                for (int j = 0; j < kBlk; ++j) {
                    if (!(act & (1u << j))) continue;
                    if (a < nf) q32[S * j + a] = make_float4(sx[j], sy[j], sz[j], 0.f);
                    pq[j] += (double)px[j] * sx[j] + (double)py[j] * sy[j] + (double)pz[j] * sz[j];
                }
            }
            block_sum_n<NW>(red, parity, pq);
            parity ^= 1;
            float af[kBlk];
#pragma unroll
            for (int j = 0; j < kBlk; ++j) {
                af[j] = 0.f;
                if (!(act & (1u << j))) continue;
                if (!(pq[j] > 0.0)) {
                    status[j] = ST_CG_INDEFINITE;
                    fin |= 1u << j;
                    act &= ~(1u << j);
                    continue;
                }
                af[j] = (float)(rz[j] / pq[j]);
            }
            double rs[2 * kBlk];
#pragma unroll
            for (int i = 0; i < 2 * kBlk; ++i) rs[i] = 0.0;
#pragma unroll
            for (int k = 0; k < SN; ++k) {
                const int64_t a = tid + T * k;
                float4 p0, p1;
                pblock(k, p0, p1);
#pragma unroll
                for (int j = 0; j < kBlk; ++j) {
                    if (!(act & (1u << j))) continue;
                    const float4 pk = own_p(j, k);
                    if (a < nf) {
                        float4 d = d32[S * j + a];
                        d.x = fmaf(af[j], pk.x, d.x);
                        d.y = fmaf(af[j], pk.y, d.y);
                        d.z = fmaf(af[j], pk.z, d.z);
                        d32[S * j + a] = d;
                    }
                    const float4 qa = a < nf ? q32[S * j + a] : make_float4(0.f, 0.f, 0.f, 0.f);
                    R[j][k][0] = fmaf(-af[j], qa.x, R[j][k][0]);
                    R[j][k][1] = fmaf(-af[j], qa.y, R[j][k][1]);
                    R[j][k][2] = fmaf(-af[j], qa.z, R[j][k][2]);
                    const float4 z = papply(p0, p1, R[j][k]);
                    rs[j] += (double)R[j][k][0] * R[j][k][0] + (double)R[j][k][1] * R[j][k][1] +
                             (double)R[j][k][2] * R[j][k][2];
                    rs[kBlk + j] += (double)R[j][k][0] * z.x + (double)R[j][k][1] * z.y + (double)R[j][k][2] * z.z;
                }
            }
            block_sum_n<NW>(red, parity, rs);
            parity ^= 1;
            float bf[kBlk];
#pragma unroll
            for (int j = 0; j < kBlk; ++j) {
                bf[j] = 0.f;
                if (!(act & (1u << j))) continue;
                if (rs[j] <= 1e-6 * rr0[j] || rs[j] <= 0.25 * tol2 * bb[j]) {
                    act &= ~(1u << j);   // inner solve of this round done
                    continue;
                }
                bf[j] = (float)(rs[kBlk + j] / rz[j]);
                rz[j] = rs[kBlk + j];
            }
#pragma unroll
            for (int k = 0; k < SN; ++k) {
                float4 p0, p1;
                if (!act) break;
                pblock(k, p0, p1);
#pragma unroll
                for (int j = 0; j < kBlk; ++j) {
                    if (!(act & (1u << j))) continue;
                    const float4 z = papply(p0, p1, R[j][k]);
                    const float4 pk = own_p(j, k);
                    zl[ZS * j + tid + T * k] =
                        make_float4(fmaf(bf[j], pk.x, z.x), fmaf(bf[j], pk.y, z.y), fmaf(bf[j], pk.z, z.z), 0.f);
                }
            }
        }
        // x += d for the columns of this round
        asm volatile("" : "+v"(tid));
#pragma unroll
        for (int k = 0; k < SN; ++k) {
            const int64_t a = tid + T * k;
            if (a < nf) {
#pragma unroll
                for (int j = 0; j < kBlk; ++j) {
                    if (!(in_round & (1u << j))) continue;
                    const float4 d = d32[S * j + a];
                    x64(j)[3 * a] += (double)d.x;
                    x64(j)[3 * a + 1] += (double)d.y;
                    x64(j)[3 * a + 2] += (double)d.z;
                }
            }
        }
        __syncthreads();
        if (outer == 7)
#pragma unroll
            for (int j = 0; j < kBlk; ++j)
                if (!(fin & (1u << j)) && status[j] == ST_CONVERGED) status[j] = ST_CG_MAXITER;
    }

    // assembly of each column
#pragma unroll 1
    for (int j = 0; j < kBlk; ++j) {
        asm volatile("" : "+v"(tid));
        double acc[9];
        assembly_partial<true>(A, c, r, kk, j, x64(j), tid, T, acc);
        double tot[9];
#pragma unroll
        for (int p = 0; p < 9; p += 3) {
            double v3[3] = {acc[p], acc[p + 1], acc[p + 2]};
            block_sum_n<NW>(red, parity, v3);
            parity ^= 1;
            tot[p] = v3[0];
            tot[p + 1] = v3[1];
            tot[p + 2] = v3[2];
        }
        if (tid == 0) assembly_write<true>(A, r, kBlk * grp + j, tot, status[j], it_total[j]);
    }
    __syncthreads();
}

// Waves per SIMD WPE (registers 512 / WPE): the three columns' residuals
// stay in registers.
template <int T, int SN, int WPE>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(WPE))) void cg_blk_kernel(TangentArgs A)
{
    extern __shared__ float4 zl[];   // [kBlk][T * SN + 1]; entries past an RVE's nodes stay zero
    __shared__ BlkRed red;
    __shared__ int task;
    constexpr int ZS = T * SN + 1;
    if (threadIdx.x < kBlk) zl[ZS * threadIdx.x + T * SN] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t n_tasks = A.n_order * kBlk;
    for (;;) {
        if (threadIdx.x == 0) task = atomicAdd(A.queue, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(task);
        __syncthreads();
        if (t >= n_tasks) break;
        cg_blk_task<T, SN, WPE >= 4 ? 1 : 2>(A, __builtin_amdgcn_readfirstlane(A.order[t / kBlk]), t % kBlk, zl, red);
    }
}

__global__ void zero_status(int32_t* st, unsigned long long* it, int64_t n)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        st[i] = 0;
        it[i] = 0;
    }
}

template <bool TAN, int T, int SN, bool PL>
const void* res_fn()
{
    return (const void*)cg_res_kernel<TAN, T, SN, PL>;
}

const void* res_kernel(int v, bool vjp)
{
    switch (v) {
    case 0: return vjp ? res_fn<false, 256, 2, false>() : res_fn<true, 256, 2, false>();
    case 1: return vjp ? res_fn<false, 512, 2, false>() : res_fn<true, 512, 2, false>();
    case 2: return vjp ? res_fn<false, 1024, 2, false>() : res_fn<true, 1024, 2, false>();
    case 3: return vjp ? res_fn<false, 1024, 4, true>() : res_fn<true, 1024, 4, true>();
    default: return vjp ? res_fn<false, 1024, 8, true>() : res_fn<true, 1024, 8, true>();
    }
}

}  // namespace

const TangentVariant kTanRes[kNumTanRes] = {{256, 2}, {512, 2}, {1024, 2}, {1024, 4}, {1024, 8}};

hipError_t launch_tangent_prep(const TangentArgs& a, hipStream_t s)
{
    if (a.n_rve <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_status, dim3((unsigned)((a.n_rve + 255) / 256)), dim3(256), 0, s, a.status, a.iters, a.n_rve);
    if (a.build_static) hipLaunchKernelGGL(ell_build_kernel, dim3((unsigned)a.n_rve), dim3(kOpsThreads), 0, s, a);
    hipLaunchKernelGGL(fiber_ops_kernel, dim3((unsigned)a.n_rve), dim3(kOpsThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tangent_stream(const TangentArgs& a, int threads, int grid, hipStream_t s)
{
    if (a.n_order <= 0) return hipSuccess;
    if (threads == 64) {
        if (a.mode == 0)
            hipLaunchKernelGGL((cg_stream_kernel<true, 64>), dim3(grid), dim3(64), 0, s, a);
        else
            hipLaunchKernelGGL((cg_stream_kernel<false, 64>), dim3(grid), dim3(64), 0, s, a);
    } else if (threads == 1024) {
        if (a.mode == 0)
            hipLaunchKernelGGL((cg_stream_kernel<true, 1024>), dim3(grid), dim3(1024), 0, s, a);
        else
            hipLaunchKernelGGL((cg_stream_kernel<false, 1024>), dim3(grid), dim3(1024), 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static size_t res_lds(int v)
{
    return 16 * ((size_t)kTanRes[v].threads * kTanRes[v].sn + 1);
}

hipError_t tangent_res_blocks(int v, bool vjp, int* blocks_per_cu)
{
    if (v < 0 || v >= kNumTanRes) return hipErrorInvalidValue;
    const void* k = res_kernel(v, vjp);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)res_lds(v));
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, kTanRes[v].threads, res_lds(v));
}

hipError_t launch_tangent_res(int v, const TangentArgs& a, int grid, hipStream_t s)
{
    if (v < 0 || v >= kNumTanRes) return hipErrorInvalidValue;
    if (a.n_order <= 0) return hipSuccess;
    const void* k = res_kernel(v, a.mode != 0);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)res_lds(v));
    if (e != hipSuccess) return e;
    void* args[] = {const_cast<TangentArgs*>(&a)};
    return hipLaunchKernel(k, dim3(grid), dim3(kTanRes[v].threads), args, res_lds(v), s);
}

hipError_t tangent_res_scratch_bytes(int v, bool vjp, size_t* bytes)
{
    if (v < 0 || v >= kNumTanRes) return hipErrorInvalidValue;
    return max_private_bytes({res_kernel(v, vjp)}, bytes);
}

// Blocked tangent tasks (three right-hand sides per workgroup) with the
// node capacity of the per-column variants 0-2 (512, 1024, 2048 free nodes).
const TangentVariant kTanBlk[kNumTanBlk] = {{256, 2}, {512, 2}, {1024, 2}};

static const void* blk_kernel(int v)
{
    switch (v) {
    case 0: return (const void*)cg_blk_kernel<256, 2, 4>;
    case 1: return (const void*)cg_blk_kernel<512, 2, 4>;
    default: return (const void*)cg_blk_kernel<1024, 2, 4>;
    }
}

static size_t blk_lds(int v)
{
    return 16 * (size_t)kBlk * ((size_t)kTanBlk[v].threads * kTanBlk[v].sn + 1);
}

hipError_t tangent_blk_blocks(int v, int* blocks_per_cu)
{
    if (v < 0 || v >= kNumTanBlk) return hipErrorInvalidValue;
    const void* k = blk_kernel(v);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)blk_lds(v));
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, kTanBlk[v].threads, blk_lds(v));
}

hipError_t launch_tangent_blk(int v, const TangentArgs& a, int grid, hipStream_t s)
{
    if (v < 0 || v >= kNumTanBlk) return hipErrorInvalidValue;
    if (a.n_order <= 0) return hipSuccess;
    const void* k = blk_kernel(v);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)blk_lds(v));
    if (e != hipSuccess) return e;
    void* args[] = {const_cast<TangentArgs*>(&a)};
    return hipLaunchKernel(k, dim3(grid), dim3(kTanBlk[v].threads), args, blk_lds(v), s);
}

hipError_t tangent_blk_scratch_bytes(int v, size_t* bytes)
{
    if (v < 0 || v >= kNumTanBlk) return hipErrorInvalidValue;
    return max_private_bytes({blk_kernel(v)}, bytes);
}

hipError_t tangent_fixed_private(size_t* bytes)
{
    return max_private_bytes({(const void*)ell_build_kernel, (const void*)fiber_ops_kernel,
                              (const void*)cg_stream_kernel<true, 64>, (const void*)cg_stream_kernel<false, 64>,
                              (const void*)cg_stream_kernel<true, 1024>, (const void*)cg_stream_kernel<false, 1024>,
                              (const void*)zero_status},
                             bytes);
}

}  // namespace rve
