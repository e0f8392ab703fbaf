// Team engine: k workgroups relax one RVE together (Section 4.3: one team per
// sub-problem, sized to the problem), for RVEs whose state does not fit one
// CU.  The RVE's free nodes are split into k parts of contiguous
// breadth-first ranges (host, rve_host.hip); part p owns its nodes and
// evaluates every fiber with a free end among them (a fiber cut by the
// partition is evaluated by both parts, so no part needs another's forces),
// and keeps its fibers, its owned nodes and the positions of the foreign
// free ends of its fibers (its halo) on chip exactly as the register-
// resident kernel does for a whole RVE.
//
// Per iteration each part publishes, for its owned nodes that lie in other
// parts' halos, the state (h, v, a) after its force gather, and its partial
// time-step maximum and norms, then meets the other parts at one team
// barrier in global memory.  After it every part combines the k partials in
// the same fixed order (so all parts take the same time step and the same
// stopping decision) and advances its halo nodes itself with the owners'
// (h, v, a) and the common time step -- the same two half-step operations
// the owner applies to its own nodes -- so the positions of the next fiber
// pass need no second exchange.
//
// The k workgroups of a team are mapped to one XCD (workgroup ids that are
// equal modulo 8), so the exchange stays in that XCD's L2.  The launch is
// cooperative (every workgroup resident at once); every team barrier is a
// bounded wait: a team that waits longer than the spin limit sets the
// launch's error word, and every workgroup then leaves at its next barrier,
// so no kernel can hang.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rve_internal.h"

namespace rve {

namespace {

constexpr int ST_CONVERGED = 0, ST_MAXITER = 1, ST_NONFINITE = 2, ST_BAD_F = 3, ST_STAGNATED = 8;
constexpr int kLawLinear = 0, kMassScaled = 1, kInitWarm = 2;

__device__ __forceinline__ int opaque(int t)
{
    asm volatile("" : "+v"(t));
    return t;
}
__device__ __forceinline__ double uni(double x)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float uni(float x) { return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x))); }
__device__ __forceinline__ int uni32(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni64(int64_t x)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ inline float t_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline float t_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double t_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ inline double t_rcp(double x) { return 1.0 / x; }

// e^x - 1 in FP32 for x >= 0: the Taylor series to x^6 below 1/4, the
// hardware 2^x minus one above (the resident kernel's formula)
__device__ inline float t_expm1(float x)
{
    float t = x * (1.f / 720.f) + (1.f / 120.f);
    t = t * x + (1.f / 24.f);
    t = t * x + (1.f / 6.f);
    t = t * x + 0.5f;
    t = t * x + 1.f;
    const float taylor = t * x;
    const float big = __builtin_amdgcn_exp2f(x * 1.44269504088896341f) - 1.f;
    return x < 0.25f ? taylor : big;
}
__device__ inline double t_expm1(double x) { return expm1(x); }

template <typename Real>
struct Fv {
    Real x, y, z, b;
};

// The fiber law in the scaled form of the resident kernel (constants
// Dn = F d0 / L0, Qn = (|F d0|^2 - L0^2) / L0^2, iL = 1 / L0).
template <typename Real>
__device__ __forceinline__ Fv<Real> fiber_scaled(bool linear, Real EA, Real B, Real EAoB, Real Dx, Real Dy, Real Dz,
                                                 Real Qn, Real iL, Real dhx, Real dhy, Real dhz)
{
    const Real ux = dhx * iL, uy = dhy * iL, uz = dhz * iL;
    const Real qn = Qn + (Real(2) * (Dx * ux + Dy * uy + Dz * uz) + (ux * ux + uy * uy + uz * uz));
    const Real m = Real(1) + qn;
    const Real rs = t_rsqrt(m);
    Real s;
    if constexpr (sizeof(Real) == 4)
        s = m * rs;
    else
        s = sqrt(m);
    const Real eps = qn * t_rcp(s + Real(1));
    Real T, kt;
    const Real Tl = EA * eps;
    if (linear) {
        T = Tl;
        kt = EA;
    } else {
        const bool pos = eps >= Real(0);
        const Real Te = EAoB * t_expm1(B * fmax(eps, Real(0)));
        T = pos ? Te : Tl;
        kt = pos ? fma(B, Te, EA) : EA;
    }
    const Real g = T * rs;
    Fv<Real> o;
    o.x = g * (Dx + ux);
    o.y = g * (Dy + uy);
    o.z = g * (Dz + uz);
    o.b = iL * fmax(kt, fabs(g));
    return o;
}

// One half-step velocity update and the position update that follows it;
// the owner of a node and every part that holds it in its halo apply exactly
// these operations, so their copies of the position agree bitwise.
template <typename Real>
__device__ __forceinline__ void advance(Real& v, Real& h, Real a, Real hdt, Real rdt)
{
    v = fma(hdt, a, v);
    h = fma(rdt, v, h);
}

// LDS exchange arrays of a part: positions of owned + halo nodes and the zero
// slot, fiber forces of its fibers and the zero slot.
template <typename Real>
struct TLds;
template <>
struct TLds<float> {
    float4* h;
    float4* fv;
    __device__ void init(char* base, int nh, int nfib)
    {
        h = reinterpret_cast<float4*>(base);
        fv = h + (nh + 1);
        (void)nfib;
    }
    __device__ void put_h(int a, float x, float y, float z) { h[a] = make_float4(x, y, z, 0.f); }
    __device__ void get_h(int a, float& x, float& y, float& z) const
    {
        const float4 q = h[a];
        x = q.x; y = q.y; z = q.z;
    }
    __device__ void put_fv(int k, const Fv<float>& o) { fv[k] = make_float4(o.x, o.y, o.z, o.b); }
    __device__ void get_fv(int k, float& x, float& y, float& z, float& b) const
    {
        const float4 q = fv[k];
        x = q.x; y = q.y; z = q.z; b = q.w;
    }
};
template <>
struct TLds<double> {
    double *hx, *hy, *hz, *fx, *fy, *fz;
    float* fb;
    __device__ void init(char* base, int nh, int nfib)
    {
        hx = reinterpret_cast<double*>(base);
        hy = hx + (nh + 1);
        hz = hy + (nh + 1);
        fx = hz + (nh + 1);
        fy = fx + (nfib + 1);
        fz = fy + (nfib + 1);
        fb = reinterpret_cast<float*>(fz + (nfib + 1));
    }
    __device__ void put_h(int a, double x, double y, double z)
    {
        hx[a] = x; hy[a] = y; hz[a] = z;
    }
    __device__ void get_h(int a, double& x, double& y, double& z) const
    {
        x = hx[a]; y = hy[a]; z = hz[a];
    }
    __device__ void put_fv(int k, const Fv<double>& o)
    {
        fx[k] = o.x; fy[k] = o.y; fz[k] = o.z; fb[k] = (float)o.b;
    }
    __device__ void get_fv(int k, double& x, double& y, double& z, double& b) const
    {
        x = fx[k]; y = fy[k]; z = fz[k]; b = (double)fb[k];
    }
};

__device__ __forceinline__ void t_two_sum(double a, double b, double& s, double& e)
{
    s = a + b;
    const double z = s - a;
    e = (a - (s - z)) + (b - z);
}

template <typename T>
__device__ inline T t_wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ inline double t_wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Shared scalars of a team workgroup.
struct TeamShared {
    double w[16][6];    // per-wave partials: gmax, |f_free|^2, |cMv|^2, |f_bnd|^2, KE
    double tot[6];      // this workgroup's totals (compensated over waves)
    int task;
    int ok;
};

// Workgroup totals of the per-thread partials (wave sums pairwise, waves in
// order with an exact two-sum), left in S.tot by thread 0 (no barrier at the
// end: the team barrier that follows provides it).
template <int NW>
__device__ __forceinline__ void wg_partials(TeamShared& S, int tid, double g, double r2, double d2, double b2,
                                            double ke)
{
    const int lane = tid & 63, wave = tid >> 6;
    g = t_wave_max(g);
    r2 = t_wave_sum(r2);
    d2 = t_wave_sum(d2);
    b2 = t_wave_sum(b2);
    ke = t_wave_sum(ke);
    if (lane == 0) {
        S.w[wave][0] = g; S.w[wave][1] = r2; S.w[wave][2] = d2; S.w[wave][3] = b2; S.w[wave][4] = ke;
    }
    __syncthreads();
    if (tid == 0) {
        double gm = 0.0;
        for (int q = 1; q < 5; ++q) {
            double s = 0.0, c = 0.0;
            for (int w = 0; w < NW; ++w) {
                double t, e;
                t_two_sum(s, S.w[w][q], t, e);
                s = t;
                c += e;
            }
            S.tot[q] = s + c;
        }
        for (int w = 0; w < NW; ++w) gm = fmax(gm, S.w[w][0]);
        S.tot[0] = gm;
    }
}

// Team barrier: every workgroup of the team adds one to the team's counter
// after its writes, then waits until the counter reaches `target` (k times
// the number of barriers passed so far).  Thread 0 publishes with an
// agent-scope release fence and reads with an acquire fence after the wait,
// the workgroup barriers on either side carry the other threads' accesses.
// The wait is bounded: after spin_limit polls, or when another team has
// given up, the launch's error word is set and false is returned to every
// thread of the workgroup.
__device__ __forceinline__ bool team_barrier(TeamShared& S, unsigned* ctr, unsigned target, int64_t spin_limit,
                                             int32_t* error)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __threadfence();
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int64_t spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > spin_limit || __hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __hip_atomic_store(error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        S.ok = ok;
    }
    __syncthreads();
    return S.ok != 0;
}

template <typename Real, int T, int SF, int SN, bool KIN>
__device__ __forceinline__ bool team_solve(const TeamArgs& A, int r, int team, int rank, char* smem, TeamShared& S,
                                           unsigned& seq)
{
    constexpr int NW = T / 64;
    const SolveArgs& P = A.s;
    const DevNet& net = P.net;
    const int k = A.k;
    const TeamPart part = A.parts[(int64_t)A.part_first[r] + rank];
    const int nfib = uni32(part.nfib), nown = uni32(part.nown), nhalo = uni32(part.nhalo), nbnd = uni32(part.nbnd);
    const int64_t fib0 = uni64(part.fib0), own0 = uni64(part.own0), halo0 = uni64(part.halo0), bnd0 = uni64(part.bnd0);
    const int zs = nown + nhalo;   // zero position slot
    unsigned* ctr = A.bar + team;
    Real* xb = reinterpret_cast<Real*>(A.xchg) + (size_t)team * 2 * 9 * (size_t)A.max_xslots;
    double* pt = A.partials + (size_t)team * 2 * 8 * (size_t)k;
    int tid = opaque((int)threadIdx.x);

    double F[9];
    bool finite = true;
    for (int q = 0; q < 9; ++q) {
        F[q] = P.F[9 * r + q];
        finite = finite && isfinite(F[q]);
    }
    const double J = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
                     F[2] * (F[3] * F[7] - F[4] * F[6]);
    if (!finite || !(J > 0.0)) {
        if (rank == 0 && tid == 0) {
            P.status[r] = ST_BAD_F;
            P.iters[r] = 0;
            P.Rres[r] = NAN; P.Dres[r] = NAN; P.Bres[r] = NAN;
            for (int q = 0; q < 9; ++q) P.sigma[9 * r + q] = NAN;
        }
        return true;
    }
    const bool linear = P.law == kLawLinear;
    const Real EA = uni((Real)P.EA), Bc = uni((Real)P.B), EAoB = uni((Real)(P.EA / P.B));
    const double cr = uni(P.c[r]);
    const Real c = KIN ? Real(0) : uni((Real)cr);
    const Real cg = uni((Real)cr);

    TLds<Real> L;
    L.init(smem, zs, nfib);

    // ---- fibers of the part into registers
    Real Dx[SF], Dy[SF], Dz[SF], Qn[SF], iL[SF];
    uint32_t E[SF];
#pragma unroll
    for (int s = 0; s < SF; ++s) {
        const int q = s * T + tid;
        Dx[s] = Dy[s] = Dz[s] = Qn[s] = Real(0);
        iL[s] = Real(1);
        E[s] = 0;
        if (q < nfib) {
            const int64_t g = A.fib_gid[fib0 + q];
            const double* d0 = net.d0 + 3 * g;
            const double L0 = net.L0[g], il = 1.0 / L0;
            const double dx = F[0] * d0[0] + F[1] * d0[1] + F[2] * d0[2];
            const double dy = F[3] * d0[0] + F[4] * d0[1] + F[5] * d0[2];
            const double dz = F[6] * d0[0] + F[7] * d0[1] + F[8] * d0[2];
            Dx[s] = (Real)(dx * il); Dy[s] = (Real)(dy * il); Dz[s] = (Real)(dz * il);
            Qn[s] = (Real)((((dx * dx + dy * dy + dz * dz) - L0 * L0) * il) * il);
            iL[s] = (Real)il;
            E[s] = A.fib_ends[fib0 + q];
        }
    }
    // ---- owned nodes: velocity, acceleration, inverse mass, incidence codes
    Real vx[SN], vy[SN], vz[SN], iM[SN];
    uint32_t inc[SN][kResIncRegs / 2];
    int degw[SN];
#pragma unroll
    for (int s = 0; s < SN; ++s) {
        const int a = s * T + tid;
        vx[s] = vy[s] = vz[s] = Real(0);
        iM[s] = Real(0);
        int deg = 0;
#pragma unroll
        for (int q = 0; q < kResIncRegs / 2; ++q) inc[s][q] = (uint32_t)nfib | ((uint32_t)nfib << 16);
        if (a < nown) {
            const int64_t g = A.own_gid[own0 + a];
            iM[s] = (Real)(1.0 / (net.mass[g] * P.rhoA));
            const int64_t e0 = A.own_inc_off[own0 + a];
            deg = (int)(A.own_inc_off[own0 + a + 1] - e0);
#pragma unroll
            for (int q = 0; q < kResIncRegs; ++q) {
                if (q < deg) {
                    const uint32_t code = A.own_inc[e0 + q];
                    if (q & 1)
                        inc[s][q >> 1] = (inc[s][q >> 1] & 0xffffu) | (code << 16);
                    else
                        inc[s][q >> 1] = (inc[s][q >> 1] & 0xffff0000u) | code;
                }
            }
            Real hx = Real(0), hy = Real(0), hz = Real(0);
            if (P.init == kInitWarm) {
                const double* h = P.h_state + 3 * g;
                hx = (Real)h[0]; hy = (Real)h[1]; hz = (Real)h[2];
            }
            L.put_h(a, hx, hy, hz);
        }
        int dm = deg;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) dm = max(dm, __shfl_xor(dm, off, 64));
        degw[s] = uni32(dm);
    }
    // halo positions of the start (the owners start from the same state)
    for (int q = tid; q < nhalo; q += T) {
        Real hx = Real(0), hy = Real(0), hz = Real(0);
        if (P.init == kInitWarm) {
            const double* h = P.h_state + 3 * A.halo_gid[halo0 + q];
            hx = (Real)h[0]; hy = (Real)h[1]; hz = (Real)h[2];
        }
        L.put_h(nown + q, hx, hy, hz);
    }
    if (tid == 0) {
        L.put_h(zs, Real(0), Real(0), Real(0));
        Fv<Real> z{Real(0), Real(0), Real(0), Real(0)};
        L.put_fv(nfib, z);
    }
    __syncthreads();

    auto fiber_pass = [&](int t) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < SF; ++s) {
            const int q = s * T + t;
            if (q < nfib) {
                Real ix, iy, iz, jx, jy, jz;
                L.get_h((int)res_end_i(E[s]), ix, iy, iz);
                L.get_h((int)res_end_j(E[s]), jx, jy, jz);
                L.put_fv(q, fiber_scaled<Real>(linear, EA, Bc, EAoB, Dx[s], Dy[s], Dz[s], Qn[s], iL[s], jx - ix,
                                               jy - iy, jz - iz));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    auto gather = [&](int t, int s, Real& fx, Real& fy, Real& fz, Real& G) __attribute__((always_inline)) {
        fx = fy = fz = G = Real(0);
#pragma unroll
        for (int q = 0; q < kResIncRegs; ++q) {
            const uint32_t code = (q & 1) ? (inc[s][q >> 1] >> 16) : (inc[s][q >> 1] & 0xffffu);
            Real x, y, z, b;
            L.get_fv((int)res_code_fiber(code), x, y, z, b);
            const Real sg = res_code_neg(code) ? Real(-1) : Real(1);
            fx = fma(sg, x, fx); fy = fma(sg, y, fy); fz = fma(sg, z, fz); G += b;
        }
        if (degw[s] > kResIncRegs) {
            const int a = s * T + t;
            if (a < nown) {
                const int64_t e1 = A.own_inc_off[own0 + a + 1];
#pragma unroll 1
                for (int64_t e = A.own_inc_off[own0 + a] + kResIncRegs; e < e1; ++e) {
                    const uint32_t code = A.own_inc[e];
                    Real x, y, z, b;
                    L.get_fv((int)res_code_fiber(code), x, y, z, b);
                    const Real sg = res_code_neg(code) ? Real(-1) : Real(1);
                    fx = fma(sg, x, fx); fy = fma(sg, y, fy); fz = fma(sg, z, fz); G += b;
                }
            }
        }
        G *= Real(2);
    };
    // |f_b|^2 of the boundary nodes assigned to this part (all their fibers are its fibers)
    auto bnorm = [&](int t) __attribute__((always_inline)) -> double {
        double acc = 0.0;
#pragma unroll 1
        for (int q = t; q < nbnd; q += T) {
            double x = 0.0, y = 0.0, z = 0.0;
#pragma unroll 1
            for (int64_t e = A.bnd_inc_off[bnd0 + q]; e < A.bnd_inc_off[bnd0 + q + 1]; ++e) {
                const uint32_t code = A.bnd_inc[e];
                Real fx, fy, fz, fb;
                L.get_fv((int)res_code_fiber(code), fx, fy, fz, fb);
                const double sg = res_code_neg(code) ? -1.0 : 1.0;
                x += sg * (double)fx; y += sg * (double)fy; z += sg * (double)fz;
            }
            acc += x * x + y * y + z * z;
        }
        return acc;
    };
    // export the state of owned nodes that other parts hold in their halo
    auto publish = [&](int t, int buf, const Real* ax, const Real* ay, const Real* az) __attribute__((always_inline)) {
        Real* xo = xb + (size_t)buf * 9 * A.max_xslots;
#pragma unroll
        for (int s = 0; s < SN; ++s) {
            const int a = s * T + t;
            if (a < nown) {
                const int x = A.own_xslot[own0 + a];
                if (x >= 0) {
                    Real hx, hy, hz;
                    L.get_h(a, hx, hy, hz);
                    Real* o = xo + 9 * (size_t)x;
                    o[0] = hx; o[1] = hy; o[2] = hz;
                    o[3] = vx[s]; o[4] = vy[s]; o[5] = vz[s];
                    o[6] = ax[s]; o[7] = ay[s]; o[8] = az[s];
                }
            }
        }
    };
    // combine the k partials of a buffer in part order (every part alike)
    auto combine = [&](int buf, double& gm, double& r2, double& d2, double& b2, double& ke) __attribute__((always_inline)) {
        const double* src = pt + (size_t)buf * 8 * k;
        gm = 0.0;
        double s[4] = {0.0, 0.0, 0.0, 0.0}, cc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int p = 0; p < k; ++p) {
            gm = fmax(gm, src[8 * p]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double t, e;
                t_two_sum(s[q], src[8 * p + 1 + q], t, e);
                s[q] = t;
                cc[q] += e;
            }
        }
        gm = uni(gm);
        r2 = uni(s[0] + cc[0]);
        d2 = uni(s[1] + cc[1]);
        b2 = uni(s[2] + cc[2]);
        ke = uni(s[3] + cc[3]);
    };

    // ---- initial forces, accelerations and norms
    fiber_pass(tid);
    __syncthreads();
    Real ax[SN], ay[SN], az[SN];
    {
        Real gpart = Real(0);
        double r2p = 0.0;
#pragma unroll
        for (int s = 0; s < SN; ++s) {
            const int a = s * T + tid;
            ax[s] = ay[s] = az[s] = Real(0);
            if (a < nown) {
                Real fx, fy, fz, G;
                gather(tid, s, fx, fy, fz, G);
                if (P.mass_mode == kMassScaled) iM[s] = G > Real(0) ? Real(4) / G : Real(1);
                ax[s] = -fx * iM[s];
                ay[s] = -fy * iM[s];
                az[s] = -fz * iM[s];
                gpart = fmax(gpart, G * iM[s]);
                r2p += (double)fx * fx + (double)fy * fy + (double)fz * fz;
            }
        }
        wg_partials<NW>(S, tid, (double)gpart, r2p, 0.0, bnorm(tid), 0.0);
    }
    publish(tid, 0, ax, ay, az);
    if (tid == 0)
        for (int q = 0; q < 5; ++q) pt[8 * rank + q] = S.tot[q];
    if (!team_barrier(S, ctr, k * ++seq, A.spin_limit, A.error)) return false;
    double gmax, R2, D2, B2, KE;
    combine(0, gmax, R2, D2, B2, KE);
    D2 = 0.0;

    int64_t n = 0;
    int status = ST_CONVERGED;
    const int ce = P.check_every > 0 ? P.check_every : 1;
    int countdown = ce;
    bool done = sqrt(R2) <= fmax(P.tol_abs, P.tol_rel * sqrt(B2));
    double Rref = uni(sqrt(R2));
    int stall = 0;
    if (!isfinite(R2)) {
        status = ST_NONFINITE;
        done = true;
    }
    if (!done && n >= P.n_max) {
        status = ST_MAXITER;
        done = true;
    }
    auto time_step = [&](double g) __attribute__((always_inline)) -> double {
        if constexpr (sizeof(Real) == 4)
            return uni((double)(uni((float)(2.0 * P.alpha)) * __builtin_amdgcn_rsqf((float)g)));
        else
            return uni(P.alpha * 2.0 / sqrt(g));
    };
    double dt = time_step(gmax);
    double ke_prev = 0.0;
    bool reset = false;   // kinetic damping: the last reduction restarted every node from rest

    while (!done) {
        const int t = opaque((int)threadIdx.x);
#pragma unroll
        for (int s = 0; s < SF; ++s) asm volatile("" : "+v"(E[s]));
#pragma unroll
        for (int s = 0; s < SN; ++s) {
#pragma unroll
            for (int q = 0; q < kResIncRegs / 2; ++q) asm volatile("" : "+v"(inc[s][q]));
        }
        const Real hdt = (Real)(0.5 * dt), rdt = (Real)dt;
        // owned nodes
#pragma unroll
        for (int s = 0; s < SN; ++s) {
            const int a = s * T + t;
            if (a < nown) {
                Real hx, hy, hz;
                L.get_h(a, hx, hy, hz);
                advance(vx[s], hx, ax[s], hdt, rdt);
                advance(vy[s], hy, ay[s], hdt, rdt);
                advance(vz[s], hz, az[s], hdt, rdt);
                L.put_h(a, hx, hy, hz);
            }
        }
        // halo nodes, from their owners' published state of the last iteration
        {
            const Real* xi = xb + (size_t)(n & 1) * 9 * A.max_xslots;
#pragma unroll 1
            for (int q = t; q < nhalo; q += T) {
                const Real* o = xi + 9 * (size_t)A.halo_xslot[halo0 + q];
                Real hx = o[0], hy = o[1], hz = o[2];
                Real ux = o[3], uy = o[4], uz = o[5];
                if (KIN && reset) ux = uy = uz = Real(0);
                advance(ux, hx, o[6], hdt, rdt);
                advance(uy, hy, o[7], hdt, rdt);
                advance(uz, hz, o[8], hdt, rdt);
                L.put_h(nown + q, hx, hy, hz);
            }
        }
        __syncthreads();
        fiber_pass(t);
        __syncthreads();
        ++n;
        const bool check = --countdown == 0;
        if (check) countdown = ce;
        Real gpart = Real(0);
        double r2p = 0.0, d2p = 0.0, kep = 0.0;
#pragma unroll
        for (int s = 0; s < SN; ++s) {
            const int a = s * T + t;
            if (a < nown) {
                Real fx, fy, fz, G;
                gather(t, s, fx, fy, fz, G);
                ax[s] = -fx * iM[s] - c * vx[s];
                ay[s] = -fy * iM[s] - c * vy[s];
                az[s] = -fz * iM[s] - c * vz[s];
                vx[s] = fma(hdt, ax[s], vx[s]);
                vy[s] = fma(hdt, ay[s], vy[s]);
                vz[s] = fma(hdt, az[s], vz[s]);
                gpart = fmax(gpart, G * iM[s]);
                if constexpr (KIN)
                    kep += 0.5 * (double)((vx[s] * vx[s] + vy[s] * vy[s] + vz[s] * vz[s]) * t_rcp(iM[s]));
                if (check) {
                    r2p += (double)fx * fx + (double)fy * fy + (double)fz * fz;
                    const Real cm = cg * t_rcp(iM[s]);
                    const double px = (double)(cm * vx[s]), py = (double)(cm * vy[s]), pz = (double)(cm * vz[s]);
                    d2p += px * px + py * py + pz * pz;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        const double b2p = check ? bnorm(t) : 0.0;
        wg_partials<NW>(S, t, (double)gpart, r2p, d2p, b2p, kep);
        const int buf = (int)(n & 1);
        publish(t, buf, ax, ay, az);
        if (t == 0)
            for (int q = 0; q < 5; ++q) pt[(size_t)buf * 8 * k + 8 * rank + q] = S.tot[q];
        if (!team_barrier(S, ctr, k * ++seq, A.spin_limit, A.error)) return false;
        double r2n, d2n, b2n, ke;
        combine(buf, gmax, r2n, d2n, b2n, ke);
        reset = false;
        if constexpr (KIN) {
            if (ke < ke_prev) {
#pragma unroll
                for (int s = 0; s < SN; ++s) vx[s] = vy[s] = vz[s] = Real(0);
                ke = 0.0;
                d2n = 0.0;
                reset = true;
            }
            ke_prev = ke;
        }
        if (check) {
            R2 = r2n;
            D2 = d2n;
            B2 = b2n;
            if (!isfinite(R2) || !isfinite(D2)) {
                status = ST_NONFINITE;
                break;
            }
            const double Rn = sqrt(R2), Dn = sqrt(D2), Bn = sqrt(B2);
            const double tol = fmax(P.tol_abs, P.tol_rel * Bn);
            if (Rn <= tol && Dn <= tol) break;
            if (P.floor_tol_rel > 0.0) {
                if (Rn < 0.5 * Rref) {
                    Rref = uni(Rn);
                    stall = 0;
                } else {
                    if (stall < P.stall_checks) ++stall;
                    const double ftol = P.floor_tol_rel * Bn;
                    if (stall >= P.stall_checks && Rn <= ftol && Dn <= ftol) {
                        status = ST_STAGNATED;
                        break;
                    }
                }
            }
        }
        if (!(gmax > 0.0) || !isfinite(gmax)) {
            status = ST_NONFINITE;
            break;
        }
        if (n >= P.n_max) {
            status = ST_MAXITER;
            break;
        }
        dt = time_step(gmax);
    }

    const int te = opaque((int)threadIdx.x);
#pragma unroll
    for (int s = 0; s < SN; ++s) {
        const int a = s * T + te;
        if (a < nown) {
            Real hx, hy, hz;
            L.get_h(a, hx, hy, hz);
            double* h = P.h_state + 3 * A.own_gid[own0 + a];
            h[0] = (double)hx; h[1] = (double)hy; h[2] = (double)hz;
        }
    }
    if (rank == 0 && te == 0) {
        P.status[r] = status;
        P.iters[r] = n;
        P.Rres[r] = sqrt(R2);
        P.Dres[r] = sqrt(D2);
        P.Bres[r] = sqrt(B2);
    }
    return true;
}

// Teams of k workgroups: workgroup w belongs to team (w % 8) + 8 ((w / 8) / k)
// with rank (w / 8) % k, so the workgroups of a team share w % 8 (one XCD).
// The team's rank-0 workgroup takes the next RVE from the launch's work
// counter and hands it to the others through the team's task slot.
template <typename Real, int T, int SF, int SN, bool KIN>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 && T == 1024 ? 4 : (sizeof(Real) == 4 ? 3 : 2))))
void dr_team_kernel(TeamArgs A)
{
    extern __shared__ char smem[];
    __shared__ TeamShared S;
    const int w = blockIdx.x, k = A.k;
    const int team = (w & 7) + 8 * ((w >> 3) / k);
    const int rank = (w >> 3) % k;
    unsigned seq = 0;
    for (;;) {
        if (rank == 0 && threadIdx.x == 0) {
            const int t = atomicAdd(A.s.queue, 1);
            A.team_task[2 * team + (seq & 1)] = t;
        }
        if (!team_barrier(S, A.bar + team, k * ++seq, A.spin_limit, A.error)) return;
        if (threadIdx.x == 0) S.task = A.team_task[2 * team + ((seq - 1) & 1)];
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(S.task);
        __syncthreads();
        if (t >= A.s.n_list) return;
        const int r = __builtin_amdgcn_readfirstlane(A.s.list[t]);
        if (!team_solve<Real, T, SF, SN, KIN>(A, r, team, rank, smem, S, seq)) return;
    }
}

}  // namespace

// Team builds: FP32 with 4 fiber and 2 node slots per thread of 768 (168
// VGPRs), FP64 with 6 and 3 per thread of 512 (256 VGPRs); both fit their
// register budgets without private memory.
template <typename Real, int T, int SF, int SN>
static hipError_t launch_team_t(const TeamArgs& a, size_t lds, int grid, hipStream_t s)
{
    const void* k = a.kinetic ? (const void*)dr_team_kernel<Real, T, SF, SN, true>
                              : (const void*)dr_team_kernel<Real, T, SF, SN, false>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    void* args[] = {const_cast<TeamArgs*>(&a)};
    return hipLaunchCooperativeKernel(k, dim3(grid), dim3(T), args, (unsigned)lds, s);
}

template <typename Real, int T, int SF, int SN>
static hipError_t team_info_t(bool kin, size_t lds, int* blocks, size_t* priv)
{
    const void* k = kin ? (const void*)dr_team_kernel<Real, T, SF, SN, true>
                        : (const void*)dr_team_kernel<Real, T, SF, SN, false>;
    hipFuncAttributes at;
    hipError_t e = hipFuncGetAttributes(&at, k);
    if (e != hipSuccess) return e;
    *priv = at.localSizeBytes;
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k, T, lds);
}

const TeamUnit kTeamUnit[2] = {{768, 4, 2}, {512, 6, 3}};   // [fp64]

hipError_t launch_team(bool fp64, const TeamArgs& a, size_t lds, int grid, hipStream_t s)
{
    return fp64 ? launch_team_t<double, 512, 6, 3>(a, lds, grid, s) : launch_team_t<float, 768, 4, 2>(a, lds, grid, s);
}

hipError_t team_info(bool fp64, bool kin, size_t lds, int* blocks_per_cu, size_t* private_bytes)
{
    return fp64 ? team_info_t<double, 512, 6, 3>(kin, lds, blocks_per_cu, private_bytes)
                : team_info_t<float, 768, 4, 2>(kin, lds, blocks_per_cu, private_bytes);
}

size_t team_lds_bytes(bool fp64, int64_t n_pos, int64_t nfib)
{
    return fp64 ? 24 * (size_t)(n_pos + 1) + 28 * (size_t)(nfib + 1) + 16 : 16 * (size_t)(n_pos + 1) + 16 * (size_t)(nfib + 1);
}

}  // namespace rve
