// Persistent batched dynamic-relaxation kernels for gfx950 (MI355X).
//
// One workgroup relaxes one RVE at a time and pulls the next RVE id from a
// device work counter (longest-first order), so thousands of uneven RVEs go
// through one launch (the whole relaxation loop inside a single kernel,
// Section 4.3).  Per iteration (Algorithm "Dynamic Relaxation"):
//
//   fiber pass   every fiber: d = F d0 + h_j - h_i, strain, axial force T,
//                force vector fv = T d / l and Gershgorin term
//                b = max(k_t/L0, |T|/l)                       -> LDS
//   node pass    every free node gathers +-fv of its fibers (no atomics:
//                a fixed incidence list, so results are bitwise repeatable),
//                forms the damped acceleration and the velocity update,
//                G = 2 sum b, and partial reductions
//   reduction    max G/M (time step) every iteration; |f_free|^2,
//                |c M v|^2 and |f_bnd|^2 in FP64 on test iterations
//   update       half-step velocity and position of the free nodes -> LDS
//
// The state is the fluctuation h of the free nodes (x = F Xm + h, Section 2,
// Taylor expansion of the micro coordinates); boundary nodes have h = 0 by
// the affine boundary condition, so they read a zero slot.  With
// l^2 - L0^2 = q0 + 2 D0.dh + dh.dh, q0 = |F d0|^2 - L0^2 formed once per
// solve in FP64, the strain carries no cancellation in FP32.
//
// Resident variant: the RVE's fibers and free nodes are dealt round-robin to
// the threads and kept in VGPRs for the whole solve (the register file of a
// CU is 512 KB, three times its LDS); LDS only holds the two exchange arrays
// (positions and fiber forces).  Streamed variant: the same loop with every
// array in global memory, for RVEs too large for one CU's LDS.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rve_internal.h"

namespace rve {

const ResidentVariant kResident[kNumResident] = {
    {256, 4, 2}, {512, 4, 2}, {768, 4, 2}, {512, 6, 3}, {1024, 4, 2}, {1024, 6, 3},
};

constexpr int kLawLinear = 0;
constexpr int kMassScaled = 1;
constexpr int kInitWarm = 2;

constexpr int ST_CONVERGED = 0, ST_MAXITER = 1, ST_NONFINITE = 2, ST_BAD_F = 3, ST_STAGNATED = 8;

// Stagnation stop, evaluated at a convergence test that did not converge
// (floor_tol_rel > 0): Rref is the residual of the start, replaced by R
// whenever R falls below half of it, and stall counts the tests since (it
// saturates at stall_checks).  The run stops once stall_checks tests have
// passed without a halving while R and the damping-force norm D are both
// within floor_tol_rel |f_bnd|.
__device__ __forceinline__ bool stagnated(const SolveArgs& A, double R, double D, double B, double& Rref,
                                          int& stall)
{
    if (!(A.floor_tol_rel > 0.0)) return false;
    if (R < 0.5 * Rref) {
        Rref = R;
        stall = 0;
        return false;
    }
    if (stall < A.stall_checks) ++stall;
    const double ftol = A.floor_tol_rel * B;
    return stall >= A.stall_checks && R <= ftol && D <= ftol;
}

// ------------------------------------------------------------------ helpers
template <typename Real>
struct Vec4;
template <>
struct Vec4<float> {
    using T = float4;
};
template <>
struct Vec4<double> {
    using T = double4;
};

__device__ inline float dev_sqrt(float x) { return __builtin_sqrtf(x); }
__device__ inline double dev_sqrt(double x) { return sqrt(x); }
// exp(x) - 1 for the exponential fiber law in FP32: degree-8 Taylor series
// below 0.5 (relative truncation error < 2e-8 there), the hardware 2^x
// above (relative error < 2e-7 of e^x - 1 at the switch, falling with x).
// e^x - 1 for x >= 0 (the law's argument B max(eps, 0)): below 1/4 the
// Taylor series to x^6 (truncation x^6/5040 relative, under half an FP32
// ulp); above, the hardware exp2 minus one (cancellation at most a factor
// e^x / (e^x - 1) <= 4.6 on its error).
__device__ inline float dev_expm1(float x)
{
    float t = x * (1.f / 720.f) + (1.f / 120.f);
    t = t * x + (1.f / 24.f);
    t = t * x + (1.f / 6.f);
    t = t * x + 0.5f;
    t = t * x + 1.f;
    float taylor = t * x;
    float big = __builtin_amdgcn_exp2f(x * 1.44269504088896341f) - 1.f;
    return x < 0.25f ? taylor : big;
}
__device__ inline double dev_expm1(double x) { return expm1(x); }

// Axial force T(eps) and k_t = dT/deps (truss law); EAoB = EA / B.
template <typename Real>
__device__ inline void fiber_law(int law, Real EA, Real B, Real EAoB, Real eps, Real& T, Real& kt)
{
    if (law != kLawLinear && eps >= Real(0)) {
        Real em1 = dev_expm1(B * eps);
        T = EAoB * em1;
        kt = EA * (em1 + Real(1));
    } else {
        T = EA * eps;
        kt = EA;
    }
}

template <typename Real>
struct FiberOut {
    Real fx, fy, fz, b;
};

// Force vector on end j (= -force on end i) and Gershgorin term of one fiber.
// iL0 = 1/L0.  FP32 uses the hardware reciprocal square root and reciprocal
// (about 1 ulp); FP64 uses correctly rounded sqrt and division.
__device__ inline float dev_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline float dev_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double dev_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ inline double dev_rcp(double x) { return 1.0 / x; }

template <typename Real>
__device__ __forceinline__ FiberOut<Real> fiber_eval(int law, Real EA, Real B, Real EAoB, Real D0x, Real D0y,
                                                     Real D0z, Real q0, Real L0, Real iL0, Real dhx, Real dhy,
                                                     Real dhz)
{
    Real dx = D0x + dhx, dy = D0y + dhy, dz = D0z + dhz;
    // l^2 - L0^2 without cancellation
    Real q = q0 + (Real(2) * (D0x * dhx + D0y * dhy + D0z * dhz) + (dhx * dhx + dhy * dhy + dhz * dhz));
    Real l2 = L0 * L0 + q;
    Real il = dev_rsqrt(l2);
    Real l = l2 * il;
    Real eps = q * iL0 * dev_rcp(l + L0);
    Real T, kt;
    fiber_law<Real>(law, EA, B, EAoB, eps, T, kt);
    Real g = T * il;
    FiberOut<Real> o;
    o.fx = g * dx;
    o.fy = g * dy;
    o.fz = g * dz;
    o.b = fmax(kt * iL0, fabs(g));
    return o;
}

// Exact-arithmetic fiber evaluation in FP64 (stress recompute).
__device__ __forceinline__ FiberOut<double> fiber_eval_exact(int law, double EA, double B, double D0x, double D0y,
                                                             double D0z, double q0, double L0, double dhx, double dhy,
                                                             double dhz)
{
    double dx = D0x + dhx, dy = D0y + dhy, dz = D0z + dhz;
    double q = q0 + (2.0 * (D0x * dhx + D0y * dhy + D0z * dhz) + (dhx * dhx + dhy * dhy + dhz * dhz));
    double l = sqrt(L0 * L0 + q);
    double eps = q / (L0 * (l + L0));
    double T, kt;
    if (law != kLawLinear && eps >= 0.0) {
        double em1 = expm1(B * eps);
        T = EA * em1 / B;
        kt = EA * (em1 + 1.0);
    } else {
        T = EA * eps;
        kt = EA;
    }
    double g = T / l;
    FiberOut<double> o;
    o.fx = g * dx;
    o.fy = g * dy;
    o.fz = g * dz;
    o.b = fmax(kt / L0, fabs(g));
    return o;
}

// The thread id as a value the compiler cannot see through: indices derived
// from it are recomputed where used instead of being hoisted and kept live.
__device__ __forceinline__ int opaque_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Broadcast helpers: values every lane holds identically (read back from LDS
// after a barrier) are moved to scalar registers.
__device__ __forceinline__ double uniform(double x)
{
    int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
    int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float uniform(float x)
{
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x)));
}
__device__ __forceinline__ int uniform32(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uniform64(int64_t x)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <typename T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Maximum over the 64 lanes of a non-negative float (bit patterns of
// non-negative floats order like unsigned integers), by DPP butterflies
// inside each row of 16 lanes and row broadcasts across rows; the result of
// lane 63 is returned in a scalar register.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned dpp_max_step(unsigned v)
{
    unsigned o = (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, ROW_MASK, 0xf, false);
    return o > v ? o : v;
}
__device__ __forceinline__ float wave_max_nonneg(float x)
{
    unsigned v = __float_as_uint(x);
    v = dpp_max_step<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v = dpp_max_step<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v = dpp_max_step<0x141, 0xf>(v);   // row_half_mirror
    v = dpp_max_step<0x140, 0xf>(v);   // row_mirror
    v = dpp_max_step<0x142, 0xa>(v);   // row_bcast:15
    v = dpp_max_step<0x143, 0xc>(v);   // row_bcast:31
    return __uint_as_float(__builtin_amdgcn_readlane(v, 63));
}

// Neumaier-compensated accumulation (sum, compensation).
__device__ inline void neumaier_add(double& s, double& c, double x)
{
    double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

__device__ inline double det3(const double* F)
{
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
}

// ------------------------------------------------------------------ LDS layouts
// FP32: positions and fiber forces as float4 (one 16-byte LDS access each).
// FP64: structure-of-arrays doubles, fiber Gershgorin term as float, so an
// RVE of ~1900 free nodes and ~4000 fibers still fits one CU's 160 KB.
template <typename Real>
struct Lds;

template <>
struct Lds<float> {
    float4* h;
    float4* fv;
    static __host__ __device__ size_t bytes(int64_t nf, int64_t nfib)
    {
        return 16 * (size_t)(nf + 1) + 16 * (size_t)(nfib + 1);
    }
    __device__ void init(char* base, int64_t nf, int64_t nfib)
    {
        h = reinterpret_cast<float4*>(base);
        fv = h + (nf + 1);
    }
    __device__ void put_h(int a, float x, float y, float z) { h[a] = make_float4(x, y, z, 0.f); }
    __device__ void get_h(int a, float& x, float& y, float& z) const
    {
        float4 q = h[a];
        x = q.x; y = q.y; z = q.z;
    }
    // position record with a per-node word in .w (the resident kernel keeps
    // the inverse mass there instead of in a register)
    __device__ void put_hw(int a, float x, float y, float z, float w) { h[a] = make_float4(x, y, z, w); }
    __device__ float4 get_hw(int a) const { return h[a]; }
    __device__ float get_w(int a) const { return h[a].w; }
    __device__ void put_w(int a, float w) { h[a].w = w; }
    __device__ void put_fv(int k, const FiberOut<float>& o) { fv[k] = make_float4(o.fx, o.fy, o.fz, o.b); }
    __device__ void get_fv(int k, float& x, float& y, float& z, float& b) const
    {
        float4 q = fv[k];
        x = q.x; y = q.y; z = q.z; b = q.w;
    }
};

template <>
struct Lds<double> {
    double *hx, *hy, *hz, *fx, *fy, *fz;
    float* fb;
    static __host__ __device__ size_t bytes(int64_t nf, int64_t nfib)
    {
        return 24 * (size_t)(nf + 1) + 24 * (size_t)(nfib + 1) + 4 * (size_t)(nfib + 1) + 16;
    }
    __device__ void init(char* base, int64_t nf, int64_t nfib)
    {
        hx = reinterpret_cast<double*>(base);
        hy = hx + (nf + 1);
        hz = hy + (nf + 1);
        fx = hz + (nf + 1);
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
    __device__ void put_fv(int k, const FiberOut<double>& o)
    {
        fx[k] = o.fx; fy[k] = o.fy; fz[k] = o.fz; fb[k] = (float)o.b;
    }
    __device__ void get_fv(int k, double& x, double& y, double& z, double& b) const
    {
        x = fx[k]; y = fy[k]; z = fz[k]; b = (double)fb[k];
    }
};

size_t resident_lds_bytes(bool fp64, int64_t nf, int64_t nfib, int /*threads*/)
{
    return fp64 ? Lds<double>::bytes(nf, nfib) : Lds<float>::bytes(nf, nfib);
}

// Reduction slots of a workgroup: per-wave partial sums of |f_free|^2,
// |c M v|^2, |f_bnd|^2 and (kinetic damping) the kinetic energy, and two
// alternating slots for the time-step maximum (LDS atomic max on the bit
// pattern of a non-negative number).

__device__ __forceinline__ void reset_gslots(RedSlots& red)
{
    if (threadIdx.x < 2) {
        red.g64[threadIdx.x] = 0ull;
        red.g32[threadIdx.x] = 0u;
    }
}

__device__ __forceinline__ double readlane_d(double x, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// Error-free sum of two doubles: s + e == a + b exactly (Knuth's two-sum;
// symmetric in a and b).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e)
{
    s = a + b;
    const double z = s - a;
    e = (a - (s - z)) + (b - z);
}

// Workgroup reduction: max of gpart (>= 0) every call, and the three norms
// when `full` (the kinetic energy too in the kinetic builds).  Inside a wave
// the partials are added pairwise; across waves the sums are compensated:
// lane 16 p + w of every wave loads partial w of quantity p, and a butterfly
// over each row of 16 lanes combines (sum, error) pairs with an exact
// two-sum, so every wave ends with the same totals in a fixed order.  One
// barrier; the max slot alternates with `parity`, the other slot is cleared
// for the next call (at least two barriers separate a clear from the next
// atomic on that slot).
template <typename Real, int NW, bool KE = false>
__device__ __forceinline__ void block_reduce(RedSlots& red, int tid, int parity, Real gpart, double r2, double d2,
                                             double b2, bool full, double& gmax_o, double& r2_o, double& d2_o,
                                             double& b2_o, double ke = 0.0, double* ke_o = nullptr)
{
    static_assert(NW <= 16, "at most 16 waves per workgroup");
    const int lane = tid & 63, wave = tid >> 6;
    if constexpr (KE) {
        ke = wave_sum(ke);
        if (lane == 0) red.v[3][wave] = ke;
    }
    if constexpr (sizeof(Real) == 4) {
        float g = wave_max_nonneg((float)gpart);
        if (lane == 0) atomicMax(&red.g32[parity], __float_as_uint(g));
    } else {
        double g = wave_max((double)gpart);
        if (lane == 0) atomicMax(&red.g64[parity], (unsigned long long)__double_as_longlong(g));
    }
    if (full) {
        r2 = wave_sum(r2);
        d2 = wave_sum(d2);
        b2 = wave_sum(b2);
        if (lane == 0) {
            red.v[0][wave] = r2;
            red.v[1][wave] = d2;
            red.v[2][wave] = b2;
        }
    }
    __syncthreads();
    if constexpr (sizeof(Real) == 4)
        gmax_o = (double)__uint_as_float(__builtin_amdgcn_readfirstlane(red.g32[parity]));
    else
        gmax_o = uniform(__longlong_as_double((long long)red.g64[parity]));
    if (tid == 0) {
        red.g32[parity ^ 1] = 0u;
        if constexpr (sizeof(Real) == 8) red.g64[parity ^ 1] = 0ull;   // FP32 builds use the 32-bit slots only
    }
    if (full || KE) {
        const int p = lane >> 4, w = lane & 15;
        const bool use = w < NW && (p == 3 ? KE : full);
        double s = use ? red.v[p][w] : 0.0, c = 0.0;
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            const double so = __shfl_xor(s, off, 16), co = __shfl_xor(c, off, 16);
            double t, e;
            two_sum(s, so, t, e);
            s = t;
            c = (c + co) + e;
        }
        const double tot = s + c;
        if (full) {
            r2_o = readlane_d(tot, 0);
            d2_o = readlane_d(tot, 16);
            b2_o = readlane_d(tot, 32);
        }
        if constexpr (KE) *ke_o = readlane_d(tot, 48);
    }
}

// Boundary reaction norm^2 partial of this thread (test iterations only).
template <typename Real, int T>
__device__ __forceinline__ double boundary_norm2_partial(const DevNet& net, const Lds<Real>& L, int64_t b0, int nb,
                                                         int tid)
{
    double acc = 0.0;
#pragma unroll 1
    for (int q = tid; q < nb; q += T) {
        double x = 0, y = 0, z = 0;
#pragma unroll 1
        for (int64_t e = net.binc_off[b0 + q]; e < net.binc_off[b0 + q + 1]; ++e) {
            uint32_t w = net.binc[e];
            int k = (int)(w & 0x7fffffffu);
            Real fx, fy, fz, bb;
            L.get_fv(k, fx, fy, fz, bb);
            double s = (w >> 31) ? -1.0 : 1.0;
            x += s * (double)fx; y += s * (double)fy; z += s * (double)fz;
        }
        acc += x * x + y * y + z * z;
    }
    return acc;
}

// Block-reduce the 9 per-thread stress sums and write sigma = tau / (J V0):
// pairwise (tree) sums inside each wave, then Neumaier-compensated
// accumulation of the per-wave partials in a fixed order.
template <int NW>
__device__ __forceinline__ void stress_finish(double* s, double J, double V0, double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ double xs[9][16];
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        double a = wave_sum(s[p]);
        if (lane == 0) xs[p][wave] = a;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        const int p = threadIdx.x;
        double a = 0.0, ca = 0.0;
        for (int w = 0; w < NW; ++w) neumaier_add(a, ca, xs[p][w]);
        out[p] = (a + ca) / (J * V0);
    }
    __syncthreads();
}

// ------------------------------------------------------------------ resident kernel
// Fiber evaluation in the scaled form of the register-resident engine.  Per
// fiber the engine keeps Dn = F d0 / L0, Qn = (|F d0|^2 - L0^2) / L0^2 and
// iL = 1/L0 (formed in FP64 once per solve); with u = dh / L0
//   qn  = (l^2 - L0^2) / L0^2 = Qn + 2 Dn.u + u.u      (no cancellation)
//   l/L0 = sqrt(1 + qn),  eps = qn / (l/L0 + 1)
//   force on end j = T d / l = (T L0 / l) (Dn + u)
//   Gershgorin term max(k_t / L0, |T| / l) = iL max(k_t, |T L0 / l|).
template <typename Real>
__device__ __forceinline__ FiberOut<Real> fiber_eval_scaled(bool linear, Real EA, Real B, Real EAoB, Real Dx, Real Dy,
                                                            Real Dz, Real Qn, Real iL, Real dhx, Real dhy, Real dhz)
{
    const Real ux = dhx * iL, uy = dhy * iL, uz = dhz * iL;
    const Real qn = Qn + (Real(2) * (Dx * ux + Dy * uy + Dz * uz) + (ux * ux + uy * uy + uz * uz));
    const Real m = Real(1) + qn;
    const Real rs = dev_rsqrt(m);   // L0 / l
    Real s;                          // l / L0
    if constexpr (sizeof(Real) == 4)
        s = m * rs;
    else
        s = sqrt(m);
    const Real eps = qn * dev_rcp(s + Real(1));
    Real T, kt;
    const Real Tl = EA * eps;   // linear law (and the exponential law in compression)
    if (linear) {
        T = Tl;
        kt = EA;
    } else {
        // both branches of the exponential law without divergence; in
        // tension k_t = EA e^{B eps} = EA + B T
        const bool pos = eps >= Real(0);
        const Real Te = EAoB * dev_expm1(B * fmax(eps, Real(0)));
        T = pos ? Te : Tl;
        kt = pos ? fma(B, Te, EA) : EA;
    }
    const Real g = T * rs;
    FiberOut<Real> o;
    o.fx = g * (Dx + ux);
    o.fy = g * (Dy + uy);
    o.fz = g * (Dz + uz);
    o.b = iL * fmax(kt, fabs(g));
    return o;
}

// One RVE on one workgroup, state in registers.  Index arithmetic (replayed
// on the host by rve_check_indexing): fiber k lives in slot k / T of thread
// k % T, free node a in slot a / T of thread a % T; fiber ends are packed
// by res_pack_ends (boundary ends read the zero position slot nf), the first
// kResIncRegs incidences of a node are 16-bit codes from res_inc_code
// (padding reads the zero force slot nfib), further incidences are read from
// the CSR in global memory.
template <typename Real, int T, int SF, int SN, bool KIN>
__device__ __forceinline__ void resident_solve(const SolveArgs& A, int r, char* smem, RedSlots& red)
{
    constexpr int NW = T / 64;
    // incidences gathered per batch of LDS reads (all four where the
    // registers allow, else two)
    constexpr int GB = (SF + SN > 6 && sizeof(Real) == 4) ? 2 : kResIncRegs;
    // Opaque per RVE: slot indices derived from the thread id are recomputed
    // for each RVE instead of being held live across the persistent loop.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const DevNet& net = A.net;
    // per-RVE sizes and offsets are the same in every lane: scalar registers
    const int64_t f0 = uniform64(net.fib_off[r]), a0 = uniform64(net.free_off[r]), b0 = uniform64(net.bnd_off[r]);
    const int nfib = uniform32((int)(net.fib_off[r + 1] - f0));
    const int nf = uniform32((int)(net.free_off[r + 1] - a0));
    const int nb = uniform32((int)(net.bnd_off[r + 1] - b0));
    const double* d0b = net.d0 + 3 * f0;
    const double* L0b = net.L0 + f0;
    const uint32_t* endb = net.ends + f0;
    const double* massb = net.mass + a0;
    const int64_t* incoffb = net.inc_off + a0;
    double* hsb = A.h_state + 3 * a0;

    double F[9];
    bool finite = true;
    for (int k = 0; k < 9; ++k) {
        F[k] = A.F[9 * r + k];
        finite = finite && isfinite(F[k]);
    }
    const double J = det3(F);
    if (!finite || !(J > 0.0)) {
        if (tid == 0) {
            A.status[r] = ST_BAD_F;
            A.iters[r] = 0;
            A.Rres[r] = NAN; A.Dres[r] = NAN; A.Bres[r] = NAN;
            for (int k = 0; k < 9; ++k) A.sigma[9 * r + k] = NAN;
        }
        return;
    }
    const bool linear = A.law == kLawLinear;
    const Real EA = uniform((Real)A.EA), Bc = uniform((Real)A.B), EAoB = uniform((Real)(A.EA / A.B));
    // kinetic damping: no viscous force (c = 0); velocities are zeroed at
    // kinetic-energy peaks below
    const double cr = uniform(A.c[r]);
    const Real c = KIN ? Real(0) : uniform((Real)cr);
    const Real cg = uniform((Real)cr);   // scale of the damping-force test

    Lds<Real> L;
    L.init(smem, nf, nfib);

    // ---- fibers into registers (scaled form, see fiber_eval_scaled)
    Real Dx[SF], Dy[SF], Dz[SF], Qn[SF], iL[SF];
    uint32_t E[SF];
#pragma unroll
    for (int s = 0; s < SF; ++s) {
        const int k = s * T + tid;
        Dx[s] = Dy[s] = Dz[s] = Qn[s] = Real(0);
        iL[s] = Real(1);
        E[s] = 0;
        if (k < nfib) {
            const double* d0 = d0b + 3 * k;
            const double L0 = L0b[k], il = 1.0 / L0;
            const double Dxd = F[0] * d0[0] + F[1] * d0[1] + F[2] * d0[2];
            const double Dyd = F[3] * d0[0] + F[4] * d0[1] + F[5] * d0[2];
            const double Dzd = F[6] * d0[0] + F[7] * d0[1] + F[8] * d0[2];
            Dx[s] = (Real)(Dxd * il); Dy[s] = (Real)(Dyd * il); Dz[s] = (Real)(Dzd * il);
            Qn[s] = (Real)((((Dxd * Dxd + Dyd * Dyd + Dzd * Dzd) - L0 * L0) * il) * il);
            iL[s] = (Real)il;
            E[s] = res_pack_ends(endb[k], (uint32_t)nf);
        }
    }
    // ---- free nodes: velocity, acceleration, inverse mass and incidence in
    // registers; the positions live only in the LDS exchange array
    // FP32: the inverse mass of a free node lives in the .w word of its LDS
    // position record (read once per iteration by the node's own thread),
    // which frees one register per node slot; FP64 keeps it in registers.
    constexpr bool IML = sizeof(Real) == 4;
    Real vx[SN], vy[SN], vz[SN], iMr[IML ? 1 : SN];
    auto iM_get = [&](int s, int a) __attribute__((always_inline)) -> Real {
        if constexpr (IML)
            return L.get_w(a);
        else
            return iMr[s];
    };
    auto iM_set = [&](int s, int a, Real v) __attribute__((always_inline)) {
        if constexpr (IML)
            L.put_w(a, v);
        else
            iMr[s] = v;
    };
    uint32_t inc[SN][kResIncRegs / 2];
    int degw[SN];   // largest degree in this wave's node slot (scalar)
#pragma unroll
    for (int s = 0; s < SN; ++s) {
        const int a = s * T + tid;
        vx[s] = vy[s] = vz[s] = Real(0);
        if constexpr (!IML) iMr[s] = Real(0);
        int deg = 0;
#pragma unroll
        for (int q = 0; q < kResIncRegs / 2; ++q) inc[s][q] = (uint32_t)nfib | ((uint32_t)nfib << 16);
        if (a < nf) {
            const Real im0 = (Real)(1.0 / (massb[a] * A.rhoA));
            const int64_t e0 = incoffb[a];
            deg = (int)(incoffb[a + 1] - e0);
#pragma unroll
            for (int q = 0; q < kResIncRegs; ++q) {
                if (q < deg) {
                    const uint32_t code = res_inc_code(net.inc[e0 + q]);
                    if (q & 1)
                        inc[s][q >> 1] = (inc[s][q >> 1] & 0xffffu) | (code << 16);
                    else
                        inc[s][q >> 1] = (inc[s][q >> 1] & 0xffff0000u) | code;
                }
            }
            Real hx = Real(0), hy = Real(0), hz = Real(0);
            if (A.init == kInitWarm) {
                const double* h = hsb + 3 * a;
                hx = (Real)h[0]; hy = (Real)h[1]; hz = (Real)h[2];
            }
            if constexpr (IML) {
                L.put_hw(a, hx, hy, hz, im0);
            } else {
                iMr[s] = im0;
                L.put_h(a, hx, hy, hz);
            }
        }
        degw[s] = (int)__builtin_amdgcn_readfirstlane(
            __float_as_uint(wave_max_nonneg(__uint_as_float((unsigned)deg))));
    }
    reset_gslots(red);
    if (tid == 0) {
        L.put_h(nf, Real(0), Real(0), Real(0));
        FiberOut<Real> z{Real(0), Real(0), Real(0), Real(0)};
        L.put_fv(nfib, z);
    }
    __syncthreads();

    // The loop bodies take the thread id as an argument that is made opaque
    // once per iteration (opaque_tid), so nothing derived from it is hoisted
    // out of the relaxation loop and held in registers for the whole solve.
    auto fiber_pass = [&](int t) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < SF; ++s) {
            const int k = s * T + t;
            if (k < nfib) {
                Real ix, iy, iz, jx, jy, jz;
                L.get_h((int)res_end_i(E[s]), ix, iy, iz);
                L.get_h((int)res_end_j(E[s]), jx, jy, jz);
                const FiberOut<Real> o = fiber_eval_scaled<Real>(linear, EA, Bc, EAoB, Dx[s], Dy[s], Dz[s], Qn[s],
                                                                 iL[s], jx - ix, jy - iy, jz - iz);
                L.put_fv(k, o);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // forces and Gershgorin sum of node slot s: the register-held incidences
    // are read back to back (padding reads the zero slot); a wave whose node
    // slot holds a node of higher degree (a wave-uniform test) reads the rest
    // from the CSR
    auto gather = [&](int t, int s, Real& fx, Real& fy, Real& fz, Real& G) __attribute__((always_inline)) {
        fx = fy = fz = G = Real(0);
#pragma unroll
        for (int h = 0; h < kResIncRegs / GB; ++h) {
            Real x[GB], y[GB], z[GB], b[GB];
            uint32_t code[GB];
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                const int q = h * GB + u;
                code[u] = (q & 1) ? (inc[s][q >> 1] >> 16) : (inc[s][q >> 1] & 0xffffu);
                L.get_fv((int)res_code_fiber(code[u]), x[u], y[u], z[u], b[u]);
            }
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                const Real sg = res_code_neg(code[u]) ? Real(-1) : Real(1);
                fx = fma(sg, x[u], fx); fy = fma(sg, y[u], fy); fz = fma(sg, z[u], fz); G += b[u];
            }
        }
        if (degw[s] > kResIncRegs) {
            const int a = s * T + t;
            if (a < nf) {
                const int64_t e1 = incoffb[a + 1];
#pragma unroll 1
                for (int64_t e = incoffb[a] + kResIncRegs; e < e1; ++e) {
                    const uint32_t w = net.inc[e];
                    Real xx, yy, zz, bb;
                    L.get_fv((int)(w & 0x7fffffffu), xx, yy, zz, bb);
                    const Real sg = (w >> 31) ? Real(-1) : Real(1);
                    fx = fma(sg, xx, fx); fy = fma(sg, yy, fy); fz = fma(sg, zz, fz); G += bb;
                }
            }
        }
        G *= Real(2);
    };

    // ---- initial force, residual and (optionally) stiffness-scaled mass
    fiber_pass(tid);
    __syncthreads();
    Real ax[SN], ay[SN], az[SN];
    Real gpart = Real(0);
    double r2p = 0.0, b2p = 0.0;
#pragma unroll
    for (int s = 0; s < SN; ++s) {
        const int a = s * T + tid;
        ax[s] = ay[s] = az[s] = Real(0);
        if (a < nf) {
            Real fx, fy, fz, G;
            gather(tid, s, fx, fy, fz, G);
            Real im = iM_get(s, a);
            if (A.mass_mode == kMassScaled) {
                im = G > Real(0) ? Real(4) / G : Real(1);
                iM_set(s, a, im);
            }
            ax[s] = -fx * im;
            ay[s] = -fy * im;
            az[s] = -fz * im;
            gpart = fmax(gpart, G * im);
            r2p += (double)fx * fx + (double)fy * fy + (double)fz * fz;
        }
    }
    b2p = boundary_norm2_partial<Real, T>(net, L, b0, nb, tid);
    double gmax;
    double R2 = 0.0, D2 = 0.0, B2 = 0.0;
    int parity = 0;
    block_reduce<Real, NW>(red, tid, parity, gpart, r2p, 0.0, b2p, true, gmax, R2, D2, B2);

    int64_t n = 0;
    int status = ST_CONVERGED;
    const int ce = A.check_every > 0 ? A.check_every : 1;
    int countdown = ce;   // iterations to the next convergence test
    // R2, D2, B2 hold the norms of the last test (reported at the end); every
    // loop-carried scalar is uniform and kept in scalar registers
    bool done = sqrt(R2) <= fmax(A.tol_abs, A.tol_rel * sqrt(B2));   // v = 0: damping norm is 0
    double Rref = uniform(sqrt(R2));   // stagnation stop: reference residual
    int stall = 0;                     // stagnation stop: tests since R last halved
    if (!isfinite(R2)) {
        status = ST_NONFINITE;
        done = true;
    }
    if (!done && n >= A.n_max) {
        status = ST_MAXITER;
        done = true;
    }
    // time step: FP64 in FP64 mode; FP32 (hardware rsqrt) in mixed mode, where
    // the state it advances is FP32 anyway
    auto time_step = [&](double g) __attribute__((always_inline)) -> double {
        if constexpr (sizeof(Real) == 4)
            return uniform((double)(uniform((float)(2.0 * A.alpha)) * __builtin_amdgcn_rsqf((float)g)));
        else
            return uniform(A.alpha * 2.0 / sqrt(g));
    };
    double dt = time_step(gmax);
    double ke_prev = 0.0;   // kinetic damping: kinetic energy at the previous full step

    while (!done) {
        const int t = opaque_tid();
        // Keep the packed fiber ends and incidence codes packed: without this
        // the compiler hoists their unpacked LDS addresses and sign masks out
        // of the loop, which multiplies the registers they occupy.
#pragma unroll
        for (int s = 0; s < SF; ++s) asm volatile("" : "+v"(E[s]));
#pragma unroll
        for (int s = 0; s < SN; ++s) {
#pragma unroll
            for (int q = 0; q < kResIncRegs / 2; ++q) asm volatile("" : "+v"(inc[s][q]));
        }
        // half-step velocity and position update with the time step of this state
        const Real hdt = (Real)(0.5 * dt), rdt = (Real)dt;
#pragma unroll
        for (int s = 0; s < SN; ++s) {
            const int a = s * T + t;
            if (a < nf) {
                vx[s] += hdt * ax[s]; vy[s] += hdt * ay[s]; vz[s] += hdt * az[s];
                if constexpr (IML) {
                    float4 q = L.get_hw(a);
                    q.x += rdt * vx[s]; q.y += rdt * vy[s]; q.z += rdt * vz[s];
                    L.put_hw(a, q.x, q.y, q.z, q.w);
                } else {
                    Real hx, hy, hz;
                    L.get_h(a, hx, hy, hz);
                    hx += rdt * vx[s]; hy += rdt * vy[s]; hz += rdt * vz[s];
                    L.put_h(a, hx, hy, hz);
                }
            }
        }
        __syncthreads();
        fiber_pass(t);
        __syncthreads();
        ++n;
        const bool check = --countdown == 0;
        if (check) countdown = ce;
        gpart = Real(0);
        r2p = 0.0;
        double d2p = 0.0, kep = 0.0;
#pragma unroll
        for (int s = 0; s < SN; ++s) {
            const int a = s * T + t;
            if (a < nf) {
                Real fx, fy, fz, G;
                const Real im = iM_get(s, a);
                gather(t, s, fx, fy, fz, G);
                // damped acceleration with the half-step velocity, then second half step
                ax[s] = -fx * im - c * vx[s];
                ay[s] = -fy * im - c * vy[s];
                az[s] = -fz * im - c * vz[s];
                vx[s] += hdt * ax[s]; vy[s] += hdt * ay[s]; vz[s] += hdt * az[s];
                gpart = fmax(gpart, G * im);
                if constexpr (KIN)
                    kep += 0.5 * (double)((vx[s] * vx[s] + vy[s] * vy[s] + vz[s] * vz[s]) * dev_rcp(im));
                if (check) {
                    r2p += (double)fx * fx + (double)fy * fy + (double)fz * fz;
                    // damping-force norm c |M v| of this node (kinetic damping
                    // applies no viscous force but keeps c as the test's scale)
                    const Real cm = cg * dev_rcp(im);
                    const double px = (double)(cm * vx[s]), py = (double)(cm * vy[s]), pz = (double)(cm * vz[s]);
                    d2p += px * px + py * py + pz * pz;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if (check) b2p = boundary_norm2_partial<Real, T>(net, L, b0, nb, t);
        parity ^= 1;
        double r2n = R2, d2n = D2, b2n = B2, ke = 0.0;
        block_reduce<Real, NW, KIN>(red, t, parity, gpart, r2p, d2p, b2p, check, gmax, r2n, d2n, b2n, kep, &ke);
        if constexpr (KIN) {
            // a kinetic-energy peak was passed: restart every node from rest
            // (the acceleration is already -f/M)
            if (ke < ke_prev) {
#pragma unroll
                for (int s = 0; s < SN; ++s) vx[s] = vy[s] = vz[s] = Real(0);
                ke = 0.0;
                if (check) d2n = 0.0;
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
            const double tol = fmax(A.tol_abs, A.tol_rel * Bn);
            if (Rn <= tol && Dn <= tol) break;
            if (stagnated(A, Rn, Dn, Bn, Rref, stall)) {
                status = ST_STAGNATED;
                break;
            }
            Rref = uniform(Rref);
        }
        if (!(gmax > 0.0) || !isfinite(gmax)) {
            status = ST_NONFINITE;
            break;
        }
        if (n >= A.n_max) {
            status = ST_MAXITER;
            break;
        }
        dt = time_step(gmax);
    }

    // ---- fluctuation state for warm starts, positions and the tangent
    const int te = opaque_tid();
#pragma unroll
    for (int s = 0; s < SN; ++s) {
        const int a = s * T + te;
        if (a < nf) {
            Real hx, hy, hz;
            L.get_h(a, hx, hy, hz);
            double* h = hsb + 3 * a;
            h[0] = (double)hx; h[1] = (double)hy; h[2] = (double)hz;
        }
    }
    if (te == 0) {
        A.status[r] = status;
        A.iters[r] = n;
        A.Rres[r] = sqrt(R2);
        A.Dres[r] = sqrt(D2);
        A.Bres[r] = sqrt(B2);
    }
    __syncthreads();
}

// Register budget (waves per SIMD the build must allow): FP32 builds of 4
// fiber and 2 node slots per thread are held to 128 VGPRs (four waves per
// SIMD, so two 512-thread or four 256-thread workgroups share a CU), the
// 768-thread and 6/3-slot FP32 builds to 168 (three waves per SIMD), FP64
// builds to 256 (two).  A build that does not fit its budget without private
// memory is never launched (the host checks every build's private segment
// size before the first launch).
template <typename Real, int T, int SF, int SN>
constexpr int resident_waves_per_eu()
{
    return sizeof(Real) == 8 ? 2 : (T == 768 ? 3 : 4);
}

template <typename Real, int T, int SF, int SN, bool KIN>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(resident_waves_per_eu<Real, T, SF, SN>())))
void dr_resident_kernel(SolveArgs A)
{
    extern __shared__ char smem[];
    __shared__ RedSlots red;
    __shared__ int task;
    for (;;) {
        if (threadIdx.x == 0) task = atomicAdd(A.queue, 1);
        __syncthreads();
        // the task id is the same for every lane: keep everything derived from it in SGPRs
        const int t = __builtin_amdgcn_readfirstlane(task);
        __syncthreads();
        if (t >= A.n_list) break;
        resident_solve<Real, T, SF, SN, KIN>(A, __builtin_amdgcn_readfirstlane(A.list[t]), smem, red);
    }
}

// ------------------------------------------------------------------ streamed kernel
// Same iteration for RVEs too large for the register-resident variants: one
// workgroup per RVE, fibers and node state in per-RVE regions of the global
// workspace, every loop strided over the workgroup.  HL: the positions h live
// in LDS (structure of arrays, A.lds_h_nodes entries per component) instead of
// the workspace, so the fiber pass gathers them from LDS.  Per-fiber constants
// (F d0, q0, L0, 1/L0) are formed once per solve; the inverse mass is kept
// next to the velocity; the loops issue the loads of two fibers, or of up to
// four incidences, before using them.
template <typename Real, int T, bool HL, bool KIN>
__device__ __forceinline__ void streamed_solve(const SolveArgs& A, int r, RedSlots& red, char* smem)
{
    using R4 = typename Vec4<Real>::T;
    constexpr int NW = T / 64;
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const DevNet& net = A.net;
    // per-RVE sizes and offsets are the same in every lane: scalar registers
    const int64_t f0 = uniform64(net.fib_off[r]), nfib = uniform64(net.fib_off[r + 1] - f0);
    const int64_t a0 = uniform64(net.free_off[r]), nf = uniform64(net.free_off[r + 1] - a0);
    const int64_t b0 = uniform64(net.bnd_off[r]), nb = uniform64(net.bnd_off[r + 1] - b0);
    const int64_t NF = uniform64(net.fib_off[net.n_rve]), NFREE = uniform64(net.free_off[net.n_rve]);

    R4* wsD = reinterpret_cast<R4*>(A.ws_fib) + (f0 + r);                             // [nfib+1] (D0, q0)
    R4* wsFv = reinterpret_cast<R4*>(A.ws_fib) + (NF + net.n_rve) + (f0 + r);         // [nfib+1] (fv, b)
    R4* wsL = reinterpret_cast<R4*>(A.ws_fib) + 2 * (NF + net.n_rve) + (f0 + r);      // [nfib] (L0, 1/L0, ends)
    R4* wsH = reinterpret_cast<R4*>(A.ws_node) + (a0 + r);                            // [nf+1]
    R4* wsV = reinterpret_cast<R4*>(A.ws_node) + (NFREE + net.n_rve) + a0;            // [nf] (v, 1/M)
    Real* wsM = reinterpret_cast<Real*>(reinterpret_cast<R4*>(A.ws_node) + (NFREE + net.n_rve) + NFREE) + a0;
    R4* wsA = reinterpret_cast<R4*>(A.ws_node) + 2 * (NFREE + net.n_rve) + NFREE + a0;   // [nf] accel
    const int64_t nh = A.lds_h_nodes;
    Real* lhx = reinterpret_cast<Real*>(smem);
    Real* lhy = lhx + nh;
    Real* lhz = lhy + nh;

    auto get_h = [&](int64_t i, Real& x, Real& y, Real& z) __attribute__((always_inline)) {
        if constexpr (HL) {
            x = lhx[i];
            y = lhy[i];
            z = lhz[i];
        } else {
            R4 h = wsH[i];
            x = h.x;
            y = h.y;
            z = h.z;
        }
    };
    auto put_h = [&](int64_t i, Real x, Real y, Real z) __attribute__((always_inline)) {
        if constexpr (HL) {
            lhx[i] = x;
            lhy[i] = y;
            lhz[i] = z;
        } else {
            R4 h;
            h.x = x; h.y = y; h.z = z; h.w = Real(0);
            wsH[i] = h;
        }
    };

    double F[9];
    bool finite = true;
    for (int k = 0; k < 9; ++k) {
        F[k] = A.F[9 * r + k];
        finite = finite && isfinite(F[k]);
    }
    const double J = det3(F);
    if (!finite || !(J > 0.0)) {
        if (tid == 0) {
            A.status[r] = ST_BAD_F;
            A.iters[r] = 0;
            A.Rres[r] = NAN; A.Dres[r] = NAN; A.Bres[r] = NAN;
            for (int k = 0; k < 9; ++k) A.sigma[9 * r + k] = NAN;
        }
        return;
    }
    const Real EA = (Real)A.EA, Bc = (Real)A.B, EAoB = (Real)(A.EA / A.B);
    const double cd = KIN ? 0.0 : A.c[r];   // kinetic damping: no viscous force
    const Real c = (Real)cd;
    const double cgd = KIN ? A.c[r] : cd;     // scale of the damping-force test

#pragma unroll 1
    for (int64_t k = tid; k < nfib; k += T) {
        const double* d0 = net.d0 + 3 * (f0 + k);
        double L0 = net.L0[f0 + k];
        double Dx = F[0] * d0[0] + F[1] * d0[1] + F[2] * d0[2];
        double Dy = F[3] * d0[0] + F[4] * d0[1] + F[5] * d0[2];
        double Dz = F[6] * d0[0] + F[7] * d0[1] + F[8] * d0[2];
        R4 q;
        q.x = (Real)Dx; q.y = (Real)Dy; q.z = (Real)Dz;
        q.w = (Real)((Dx * Dx + Dy * Dy + Dz * Dz) - L0 * L0);
        wsD[k] = q;
        // boundary ends read the zero slot nf
        uint32_t e = net.ends[f0 + k];
        uint32_t i = e & 0xffffu, j = e >> 16;
        i = i < (uint32_t)nf ? i : (uint32_t)nf;
        j = j < (uint32_t)nf ? j : (uint32_t)nf;
        R4 l;
        l.x = (Real)L0;
        l.y = (Real)(1.0 / L0);
        l.z = (Real)i;
        l.w = (Real)j;
        wsL[k] = l;
    }
#pragma unroll 1
    for (int64_t a = tid; a < nf; a += T) {
        Real hx = Real(0), hy = Real(0), hz = Real(0);
        if (A.init == kInitWarm) {
            const double* hs = A.h_state + 3 * (a0 + a);
            hx = (Real)hs[0]; hy = (Real)hs[1]; hz = (Real)hs[2];
        }
        put_h(a, hx, hy, hz);
        R4 z;
        z.x = z.y = z.z = z.w = Real(0);
        wsV[a] = z;
        wsM[a] = (Real)(net.mass[a0 + a] * A.rhoA);
    }
    if (tid == 0) {
        R4 z;
        z.x = z.y = z.z = z.w = Real(0);
        put_h(nf, Real(0), Real(0), Real(0));
        wsFv[nfib] = z;
    }
    __syncthreads();

    auto fiber_one = [&](const R4& D, const R4& l) __attribute__((always_inline)) -> R4 {
        const int64_t i = (int64_t)l.z, j = (int64_t)l.w;
        Real ix, iy, iz, jx, jy, jz;
        get_h(i, ix, iy, iz);
        get_h(j, jx, jy, jz);
        FiberOut<Real> o = fiber_eval<Real>(A.law, EA, Bc, EAoB, D.x, D.y, D.z, D.w, l.x, l.y, jx - ix, jy - iy,
                                            jz - iz);
        R4 w;
        w.x = o.fx; w.y = o.fy; w.z = o.fz; w.w = o.b;
        return w;
    };
    auto fiber_pass = [&]() __attribute__((always_inline)) {
#pragma unroll 1
        for (int64_t k = tid; k < nfib; k += 2 * T) {
            const int64_t k2 = k + T;
            const bool two = k2 < nfib;
            const R4 Da = wsD[k], la = wsL[k];
            R4 Db = Da, lb = la;
            if (two) {
                Db = wsD[k2];
                lb = wsL[k2];
            }
            const R4 wa = fiber_one(Da, la);
            if (two) {
                const R4 wb = fiber_one(Db, lb);
                wsFv[k2] = wb;
            }
            wsFv[k] = wa;
        }
    };
    // forces and Gershgorin sum at free node a: up to four incidences loaded
    // together, the rest (high-degree nodes) one by one
    auto gather = [&](int64_t a, Real& fx, Real& fy, Real& fz, Real& G) __attribute__((always_inline)) {
        fx = fy = fz = G = Real(0);
        const int64_t e0 = net.inc_off[a0 + a], e1 = net.inc_off[a0 + a + 1];
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = e0 + q < e1 ? net.inc[e0 + q] : (uint32_t)nfib;
        R4 f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) f[q] = wsFv[w[q] & 0x7fffffffu];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const Real sg = (w[q] >> 31) ? Real(-1) : Real(1);
            fx += sg * f[q].x; fy += sg * f[q].y; fz += sg * f[q].z; G += f[q].w;
        }
#pragma unroll 1
        for (int64_t e = e0 + 4; e < e1; ++e) {
            uint32_t we = net.inc[e];
            R4 q = wsFv[we & 0x7fffffffu];
            if (we >> 31) {
                q.x = -q.x; q.y = -q.y; q.z = -q.z;
            }
            fx += q.x; fy += q.y; fz += q.z; G += q.w;
        }
        G *= Real(2);
    };
    auto bnorm2 = [&]() __attribute__((always_inline)) {
        double acc = 0.0;
#pragma unroll 1
        for (int64_t q = tid; q < nb; q += T) {
            double x = 0, y = 0, z = 0;
#pragma unroll 1
            for (int64_t e = net.binc_off[b0 + q]; e < net.binc_off[b0 + q + 1]; ++e) {
                uint32_t w = net.binc[e];
                R4 f = wsFv[w & 0x7fffffffu];
                double s = (w >> 31) ? -1.0 : 1.0;
                x += s * (double)f.x; y += s * (double)f.y; z += s * (double)f.z;
            }
            acc += x * x + y * y + z * z;
        }
        return acc;
    };

    reset_gslots(red);
    fiber_pass();
    __syncthreads();
    Real gpart = Real(0);
    double r2p = 0.0;
#pragma unroll 1
    for (int64_t a = tid; a < nf; a += T) {
        Real fx, fy, fz, G;
        gather(a, fx, fy, fz, G);
        Real m = wsM[a];
        if (A.mass_mode == kMassScaled) {
            m = G > Real(0) ? G / Real(4) : Real(1);
            wsM[a] = m;
        }
        Real im = Real(1) / m;
        R4 acc;
        acc.x = -fx * im; acc.y = -fy * im; acc.z = -fz * im; acc.w = Real(0);
        wsA[a] = acc;
        R4 v = wsV[a];
        v.w = im;
        wsV[a] = v;
        gpart = fmax(gpart, G * im);
        r2p += (double)fx * fx + (double)fy * fy + (double)fz * fz;
    }
    double b2p = bnorm2();
    double gmax;
    double R2 = 0.0, D2 = 0.0, B2 = 0.0;
    int parity = 0;
    block_reduce<Real, NW>(red, tid, parity, gpart, r2p, 0.0, b2p, true, gmax, R2, D2, B2);

    int64_t n = 0;
    int status = ST_CONVERGED;
    const int ce = A.check_every > 0 ? A.check_every : 1;
    double tol = fmax(A.tol_abs, A.tol_rel * sqrt(B2));
    bool done = (sqrt(R2) <= tol);
    double Rlast = sqrt(R2), Dlast = 0.0, Blast = sqrt(B2);
    double Rref = Rlast;   // stagnation stop: reference residual
    int stall = 0;         // stagnation stop: tests since R last halved
    if (!isfinite(R2)) {
        status = ST_NONFINITE;
        done = true;
    }
    if (!done && n >= A.n_max) {
        status = ST_MAXITER;
        done = true;
    }
    double dt = A.alpha * 2.0 / sqrt(gmax);
    double ke_prev = 0.0;   // kinetic damping: kinetic energy at the previous full step
    while (!done) {
        const Real hdt = (Real)(0.5 * dt), rdt = (Real)dt;
#pragma unroll 1
        for (int64_t a = tid; a < nf; a += T) {
            R4 v = wsV[a], acc = wsA[a];
            Real hx, hy, hz;
            get_h(a, hx, hy, hz);
            v.x += hdt * acc.x; v.y += hdt * acc.y; v.z += hdt * acc.z;
            hx += rdt * v.x; hy += rdt * v.y; hz += rdt * v.z;
            wsV[a] = v;
            put_h(a, hx, hy, hz);
        }
        __syncthreads();
        fiber_pass();
        __syncthreads();
        ++n;
        // every ce-th iteration (32-bit remainder: a 64-bit one expands to
        // dozens of scalar instructions per iteration)
        const bool check = ((uint32_t)n % (uint32_t)ce) == 0;
        gpart = Real(0);
        r2p = 0.0;
        double d2p = 0.0, kep = 0.0;
        // damping-force norm of the convergence test, c |M v| (kinetic
        // damping applies no viscous force but keeps c as the guard's scale)
        const double dfac = cgd;
#pragma unroll 1
        for (int64_t a = tid; a < nf; a += T) {
            Real fx, fy, fz, G;
            gather(a, fx, fy, fz, G);
            R4 v = wsV[a], acc;
            const Real im = v.w;
            acc.x = -fx * im - c * v.x;
            acc.y = -fy * im - c * v.y;
            acc.z = -fz * im - c * v.z;
            acc.w = Real(0);
            v.x += hdt * acc.x; v.y += hdt * acc.y; v.z += hdt * acc.z;
            wsV[a] = v;
            wsA[a] = acc;
            gpart = fmax(gpart, G * im);
            if constexpr (KIN)
                kep += 0.5 * (double)wsM[a] * ((double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z);
            if (check) {
                r2p += (double)fx * fx + (double)fy * fy + (double)fz * fz;
                double md = (double)wsM[a] * dfac;
                double px = md * (double)v.x, py = md * (double)v.y, pz = md * (double)v.z;
                d2p += px * px + py * py + pz * pz;
            }
        }
        if (check) b2p = bnorm2();
        parity ^= 1;
        double ke = 0.0;
        block_reduce<Real, NW, KIN>(red, tid, parity, gpart, r2p, d2p, b2p, check, gmax, R2, D2, B2, kep, &ke);
        if constexpr (KIN) {
            // a kinetic-energy peak was passed: restart every node from rest
            // (the stored acceleration is already -f/M)
            if (ke < ke_prev) {
#pragma unroll 1
                for (int64_t a = tid; a < nf; a += T) {
                    R4 v = wsV[a];
                    v.x = v.y = v.z = Real(0);
                    wsV[a] = v;
                }
                ke = 0.0;
                D2 = 0.0;
            }
            ke_prev = ke;
        }
        if (check) {
            Rlast = sqrt(R2);
            Dlast = sqrt(D2);
            Blast = sqrt(B2);
            tol = fmax(A.tol_abs, A.tol_rel * Blast);
            if (!isfinite(R2) || !isfinite(D2)) {
                status = ST_NONFINITE;
                break;
            }
            if (Rlast <= tol && Dlast <= tol) break;
            if (stagnated(A, Rlast, Dlast, Blast, Rref, stall)) {
                status = ST_STAGNATED;
                break;
            }
        }
        if (!(gmax > 0.0) || !isfinite(gmax)) {
            status = ST_NONFINITE;
            break;
        }
        if (n >= A.n_max) {
            status = ST_MAXITER;
            break;
        }
        dt = A.alpha * 2.0 / sqrt(gmax);
    }

#pragma unroll 1
    for (int64_t a = tid; a < nf; a += T) {
        Real hx, hy, hz;
        get_h(a, hx, hy, hz);
        double* hs = A.h_state + 3 * (a0 + a);
        hs[0] = (double)hx; hs[1] = (double)hy; hs[2] = (double)hz;
    }
    if (tid == 0) {
        A.status[r] = status;
        A.iters[r] = n;
        A.Rres[r] = Rlast;
        A.Dres[r] = Dlast;
        A.Bres[r] = Blast;
    }
    __syncthreads();
}

// RVEs whose positions fit the launch's LDS copy (nf + 1 <= lds_h_nodes) run
// the LDS form, the others the workspace form, in one persistent launch.
template <typename Real, int T, bool KIN>
__global__ __launch_bounds__(T) void dr_streamed_kernel(SolveArgs A)
{
    extern __shared__ char smem_h[];
    __shared__ RedSlots red;
    __shared__ int task;
    for (;;) {
        if (threadIdx.x == 0) task = atomicAdd(A.queue, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(task);
        __syncthreads();
        if (t >= A.n_list) break;
        const int r = __builtin_amdgcn_readfirstlane(A.list[t]);
        const int64_t nf = A.net.free_off[r + 1] - A.net.free_off[r];
        if (nf + 1 <= A.lds_h_nodes)
            streamed_solve<Real, T, true, KIN>(A, r, red, smem_h);
        else
            streamed_solve<Real, T, false, KIN>(A, r, red, smem_h);
    }
}

// ------------------------------------------------------------------ incidence kernel
// RVEs beyond the register-resident capacity whose free nodes fit one
// workgroup's registers and LDS (layout in rve_internal.h).  Per iteration
// the network is read once from global memory as per-incidence records, the
// node state never leaves the CU, and no fiber force goes through memory:
// each fiber is evaluated at both of its ends (twice the fiber arithmetic of
// the other engines, which this memory-bound regime has to spare).
const IncVariant kInc[kNumInc] = {{768, 16}};

// Record of one incidence under F: the scaled form (Dn, Qn) of the fiber
// oriented so that the node is its end j (rve_internal.h), formed in FP64.
__device__ __forceinline__ float4 inc_record(const double* F, const DevNet& net, int64_t f0, uint32_t w)
{
    const int64_t k = f0 + (int64_t)(w & 0x7fffffffu);
    const double* d0 = net.d0 + 3 * k;
    const double L0 = net.L0[k], il = 1.0 / L0;
    const double Dx = F[0] * d0[0] + F[1] * d0[1] + F[2] * d0[2];
    const double Dy = F[3] * d0[0] + F[4] * d0[1] + F[5] * d0[2];
    const double Dz = F[6] * d0[0] + F[7] * d0[1] + F[8] * d0[2];
    const double sg = (w >> 31) ? -il : il;
    return make_float4((float)(Dx * sg), (float)(Dy * sg), (float)(Dz * sg),
                       (float)((((Dx * Dx + Dy * Dy + Dz * Dz) - L0 * L0) * il) * il));
}

// One RVE on one workgroup of T threads with S node slots per thread: the
// velocity and acceleration of every node slot stay in registers, the
// inverse masses are read from a global float array (rank order; in
// registers they would exceed the build's budget).  The first QU rounds of
// a slot are unrolled and their records loaded QR rounds at a time: all
// four in the viscous build (one memory round trip per node slot), two in
// the kinetic build, whose kinetic-energy sum leaves fewer registers.
template <int T, int S, int QR, bool KIN>
__device__ __forceinline__ void incidence_solve(const SolveArgs& A, const IncArgs& I, int r, char* smem,
                                                RedSlots& red)
{
    constexpr int NW = T / 64;
    constexpr int QU = 4;
    static_assert(QU % QR == 0, "record batches tile the unrolled rounds");
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const DevNet& net = A.net;
    const int64_t f0 = uniform64(net.fib_off[r]), a0 = uniform64(net.free_off[r]), b0 = uniform64(net.bnd_off[r]);
    const int nf = uniform32((int)(net.free_off[r + 1] - a0));
    const int nb = uniform32((int)(net.bnd_off[r + 1] - b0));
    const int64_t rb = uniform64(I.rec_first[r]);
    const int32_t* rq = I.round_first + (int64_t)r * (kIncMaxDeg + 1);
    int Rq[QU + 1];
#pragma unroll
    for (int q = 0; q <= QU; ++q) Rq[q] = uniform32(rq[q]);
    const int nrec = uniform32(rq[kIncMaxDeg]);
    const float4* recb = I.rec + rb;
    const uint2* stb = I.rec_st + rb;
    const int32_t* permb = I.perm + a0;
    float* imb = I.imass + a0;
    double* hsb = A.h_state + 3 * a0;

    double F[9];
    bool finite = true;
    for (int k = 0; k < 9; ++k) {
        F[k] = A.F[9 * r + k];
        finite = finite && isfinite(F[k]);
    }
    const double J = det3(F);
    if (!finite || !(J > 0.0)) {
        if (tid == 0) {
            A.status[r] = ST_BAD_F;
            // an opaque zero: no 64-bit zero register pair is held across RVEs for it
            int64_t zero = 0;
            asm volatile("" : "+s"(zero));
            A.iters[r] = zero;
            A.Rres[r] = NAN; A.Dres[r] = NAN; A.Bres[r] = NAN;
            for (int k = 0; k < 9; ++k) A.sigma[9 * r + k] = NAN;
        }
        return;
    }
    const bool linear = A.law == kLawLinear;
    // law constants from opaque per-RVE copies: nothing derived from them is
    // held in vector registers across RVEs of the persistent loop
    double EAd = A.EA, Bd = A.B;
    asm volatile("" : "+s"(EAd), "+s"(Bd));
    const float EA = uniform((float)EAd), Bc = uniform((float)Bd), EAoB = uniform((float)(EAd / Bd));
    const double cr = uniform(A.c[r]);
    const float c = KIN ? 0.f : uniform((float)cr);
    const float cg = uniform((float)cr);   // scale of the damping-force test

    float* lhx = reinterpret_cast<float*>(smem);
    float* lhy = lhx + (nf + 1);
    float* lhz = lhy + (nf + 1);

    // ---- records of this F (free and boundary incidences)
#pragma unroll 1
    for (int j = tid; j < nrec; j += T) I.rec[rb + j] = inc_record(F, net, f0, I.rec_fib[rb + j]);
    const int64_t be0 = uniform64(net.binc_off[b0]), be1 = uniform64(net.binc_off[b0 + nb]);
#pragma unroll 1
    for (int64_t e = be0 + tid; e < be1; e += T) I.brec[e] = inc_record(F, net, f0, net.binc[e]);

    // ---- node state: velocity and acceleration in registers, positions in LDS
    float vx[S], vy[S], vz[S], ax[S], ay[S], az[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int p = s * T + tid;
        vx[s] = vy[s] = vz[s] = ax[s] = ay[s] = az[s] = 0.f;
        if (p < nf) {
            const int a = permb[p];
            imb[p] = (float)(1.0 / (net.mass[a0 + a] * A.rhoA));
            float hx = 0.f, hy = 0.f, hz = 0.f;
            if (A.init == kInitWarm) {
                const double* h = hsb + 3 * a;
                hx = (float)h[0]; hy = (float)h[1]; hz = (float)h[2];
            }
            lhx[p] = hx; lhy[p] = hy; lhz[p] = hz;
        }
    }
    if (tid < 2) red.g32[tid] = 0u;   // FP32: only the 32-bit time-step slots are used
    if (tid == 0) lhx[nf] = lhy[nf] = lhz[nf] = 0.f;
    __syncthreads();

    // records of the first QU rounds of slot s (a lane past a round's nodes
    // keeps a null record that reads the zero slot; its result is discarded)
    struct Recs {
        float4 rc[QU];
        uint2 st[QU];
    };
    auto load_recs = [&](int t, int s, Recs& R, int qlo, int qhi) __attribute__((always_inline)) {
        const int p = s * T + t;
#pragma unroll
        for (int q = 0; q < QU; ++q) {
            if (q < qlo || q >= qhi) continue;
            const int Pq = Rq[q + 1] - Rq[q];
            R.rc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            R.st[q] = make_uint2(0u, (uint32_t)nf);
            if (s * T < Pq && p < Pq) {
                R.rc[q] = recb[Rq[q] + p];
                R.st[q] = stb[Rq[q] + p];
            }
        }
    };
    // internal force and Gershgorin sum at the node of slot s: rounds
    // [qlo, qhi) from its loaded records; node_tail adds the rounds beyond
    // QU (nodes of higher degree, the first ranks), read one at a time.  The
    // node's own position is read from LDS in every round rather than held
    // (three registers fewer across the rounds; lanes past nf read the zero
    // slot)
    auto node_rounds = [&](int t, int s, const Recs& R, int qlo, int qhi, float& fx, float& fy, float& fz, float& G)
                           __attribute__((always_inline)) {
        const int p = s * T + t, pp = p < nf ? p : nf;
#pragma unroll
        for (int q = 0; q < QU; ++q) {
            if (q < qlo || q >= qhi) continue;
            const int Pq = Rq[q + 1] - Rq[q];
            if (s * T < Pq) {
                const int o = (int)R.st[q].y;
                const FiberOut<float> f = fiber_eval_scaled<float>(linear, EA, Bc, EAoB, R.rc[q].x, R.rc[q].y,
                                                                   R.rc[q].z, R.rc[q].w, __uint_as_float(R.st[q].x),
                                                                   lhx[pp] - lhx[o], lhy[pp] - lhy[o], lhz[pp] - lhz[o]);
                if (p < Pq) {
                    fx += f.fx; fy += f.fy; fz += f.fz; G += f.b;
                }
            }
            // one fiber evaluation at a time (their temporaries do not overlap)
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    auto node_tail = [&](int t, int s, float& fx, float& fy, float& fz, float& G) __attribute__((always_inline)) {
        const int p = s * T + t, pp = p < nf ? p : nf;
#pragma unroll 1
        for (int q = QU; q < kIncMaxDeg; ++q) {
            const int R0 = uniform32(rq[q]), Pq = uniform32(rq[q + 1]) - R0;
            if (s * T >= Pq) break;
            if (p < Pq) {
                const float4 x = recb[R0 + p];
                const uint2 y = stb[R0 + p];
                const int o = (int)y.y;
                const FiberOut<float> f = fiber_eval_scaled<float>(linear, EA, Bc, EAoB, x.x, x.y, x.z, x.w,
                                                                   __uint_as_float(y.x), lhx[pp] - lhx[o],
                                                                   lhy[pp] - lhy[o], lhz[pp] - lhz[o]);
                fx += f.fx; fy += f.fy; fz += f.fz; G += f.b;
            }
        }
        G *= 2.f;
    };
    // boundary reaction norm^2 partial of this thread (test iterations)
    auto bnorm2 = [&](int t) __attribute__((always_inline)) -> double {
        double acc = 0.0;
#pragma unroll 1
        for (int q = t; q < nb; q += T) {
            double x = 0.0, y = 0.0, z = 0.0;
            const int64_t e1 = net.binc_off[b0 + q + 1];
#pragma unroll 1
            for (int64_t e = net.binc_off[b0 + q]; e < e1; ++e) {
                const float4 rc = I.brec[e];
                const uint2 st = I.brec_st[e];
                const int o = (int)st.y;
                const FiberOut<float> f = fiber_eval_scaled<float>(linear, EA, Bc, EAoB, rc.x, rc.y, rc.z, rc.w,
                                                                   __uint_as_float(st.x), 0.f - lhx[o], 0.f - lhy[o],
                                                                   0.f - lhz[o]);
                x += (double)f.fx; y += (double)f.fy; z += (double)f.fz;
            }
            acc += x * x + y * y + z * z;
        }
        return acc;
    };
    // the force pass over every slot: slot_body(s, p, fx, fy, fz, G) runs on
    // the lanes that hold a node
    auto force_pass = [&](int t, auto&& slot_body) __attribute__((always_inline)) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s * T < nf) {
                const int p = s * T + t;
                float fx = 0.f, fy = 0.f, fz = 0.f, G = 0.f;
#pragma unroll
                for (int q0 = 0; q0 < QU; q0 += QR) {
                    Recs R;
                    load_recs(t, s, R, q0, q0 + QR);
                    node_rounds(t, s, R, q0, q0 + QR, fx, fy, fz, G);
                }
                node_tail(t, s, fx, fy, fz, G);
                if (p < nf) slot_body(s, p, fx, fy, fz, G);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // ---- initial force, residual and (optionally) stiffness-scaled mass
    float gpart = 0.f;
    double r2p = 0.0, b2p = 0.0;
    force_pass(tid, [&](int s, int p, float fx, float fy, float fz, float G) __attribute__((always_inline)) {
        float im = imb[p];
        if (A.mass_mode == kMassScaled) {
            im = G > 0.f ? 4.f / G : 1.f;
            imb[p] = im;
        }
        ax[s] = -fx * im;
        ay[s] = -fy * im;
        az[s] = -fz * im;
        gpart = fmax(gpart, G * im);
        r2p += (double)fx * fx + (double)fy * fy + (double)fz * fz;
    });
    b2p = bnorm2(tid);
    double gmax;
    double R2 = 0.0, D2 = 0.0, B2 = 0.0;
    int parity = 0;
    block_reduce<float, NW>(red, tid, parity, gpart, r2p, 0.0, b2p, true, gmax, R2, D2, B2);

    int64_t n = 0;
    int status = ST_CONVERGED;
    const int ce = A.check_every > 0 ? A.check_every : 1;
    int countdown = ce;
    bool done = sqrt(R2) <= fmax(A.tol_abs, A.tol_rel * sqrt(B2));   // v = 0: damping norm is 0
    double Rref = uniform(sqrt(R2));
    int stall = 0;
    if (!isfinite(R2)) {
        status = ST_NONFINITE;
        done = true;
    }
    if (!done && n >= A.n_max) {
        status = ST_MAXITER;
        done = true;
    }
    auto time_step = [&](double g) __attribute__((always_inline)) -> double {
        return uniform((double)(uniform((float)(2.0 * A.alpha)) * __builtin_amdgcn_rsqf((float)g)));
    };
    double dt = time_step(gmax);
    double ke_prev = 0.0;

    while (!done) {
        const int t = opaque_tid();
        // round starts opaque per iteration: the record addresses of every
        // (slot, round) are formed where used, not hoisted and held in SGPRs
#pragma unroll
        for (int q = 0; q <= QU; ++q) asm volatile("" : "+s"(Rq[q]));
        const float hdt = (float)(0.5 * dt), rdt = (float)dt;
        // half-step velocity and position update
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int p = s * T + t;
            if (s * T < nf && p < nf) {
                vx[s] += hdt * ax[s]; vy[s] += hdt * ay[s]; vz[s] += hdt * az[s];
                lhx[p] += rdt * vx[s]; lhy[p] += rdt * vy[s]; lhz[p] += rdt * vz[s];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
        // a new opaque thread id for the force phase: the lane masks and LDS
        // addresses of the update phase are not kept live across the barrier
        const int tb = opaque_tid();
        ++n;
        const bool check = --countdown == 0;
        if (check) countdown = ce;
        gpart = 0.f;
        r2p = 0.0;
        double d2p = 0.0, kep = 0.0;
        force_pass(tb, [&](int s, int p, float fx, float fy, float fz, float G) __attribute__((always_inline)) {
            const float im = imb[p];
            // damped acceleration with the half-step velocity, then second half step
            ax[s] = -fx * im - c * vx[s];
            ay[s] = -fy * im - c * vy[s];
            az[s] = -fz * im - c * vz[s];
            vx[s] += hdt * ax[s]; vy[s] += hdt * ay[s]; vz[s] += hdt * az[s];
            gpart = fmax(gpart, G * im);
            if constexpr (KIN)
                kep += 0.5 * (double)((vx[s] * vx[s] + vy[s] * vy[s] + vz[s] * vz[s]) * dev_rcp(im));
            if (check) {
                r2p += (double)fx * fx + (double)fy * fy + (double)fz * fz;
                const float cm = cg * dev_rcp(im);
                const double px = (double)(cm * vx[s]), py = (double)(cm * vy[s]), pz = (double)(cm * vz[s]);
                d2p += px * px + py * py + pz * pz;
            }
        });
        if (check) b2p = bnorm2(tb);
        parity ^= 1;
        double r2n = R2, d2n = D2, b2n = B2, ke = 0.0;
        block_reduce<float, NW, KIN>(red, tb, parity, gpart, r2p, d2p, b2p, check, gmax, r2n, d2n, b2n, kep, &ke);
        if constexpr (KIN) {
            // a kinetic-energy peak was passed: restart every node from rest
            // (the acceleration is already -f/M)
            if (ke < ke_prev) {
#pragma unroll
                for (int s = 0; s < S; ++s) vx[s] = vy[s] = vz[s] = 0.f;
                ke = 0.0;
                if (check) d2n = 0.0;
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
            const double tol = fmax(A.tol_abs, A.tol_rel * Bn);
            if (Rn <= tol && Dn <= tol) break;
            if (stagnated(A, Rn, Dn, Bn, Rref, stall)) {
                status = ST_STAGNATED;
                break;
            }
            Rref = uniform(Rref);
        }
        if (!(gmax > 0.0) || !isfinite(gmax)) {
            status = ST_NONFINITE;
            break;
        }
        if (n >= A.n_max) {
            status = ST_MAXITER;
            break;
        }
        dt = time_step(gmax);
    }

    // ---- fluctuation state in the packed order
    const int te = opaque_tid();
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int p = s * T + te;
        if (s * T < nf && p < nf) {
            double* h = hsb + 3 * permb[p];
            h[0] = (double)lhx[p]; h[1] = (double)lhy[p]; h[2] = (double)lhz[p];
        }
    }
    if (te == 0) {
        A.status[r] = status;
        A.iters[r] = n;
        A.Rres[r] = sqrt(R2);
        A.Dres[r] = sqrt(D2);
        A.Bres[r] = sqrt(B2);
    }
    __syncthreads();
}

template <int T, int S, int QR, bool KIN>
__global__ __launch_bounds__(T) void dr_incidence_kernel(SolveArgs A, IncArgs I)
{
    extern __shared__ char smem_i[];
    __shared__ RedSlots red;
    __shared__ int task;
    for (;;) {
        if (threadIdx.x == 0) task = atomicAdd(A.queue, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(task);
        __syncthreads();
        if (t >= A.n_list) break;
        incidence_solve<T, S, QR, KIN>(A, I, __builtin_amdgcn_readfirstlane(A.list[t]), smem_i, red);
    }
}

// Global mode of the incidence engine, for RVEs whose positions do not fit
// LDS (more than kIncMaxNodes free nodes): the same records and rounds, the
// node state (h with 1/M, v, a) in global arrays in rank order, each thread
// taking ranks tid, tid + T, ...  Per iteration every record is read once,
// the other end's position is gathered from global memory (the RVE's
// positions, 16 B per node, stay in L2), and no fiber force is written.
// The force pass takes NP nodes of a thread at once and loads the records
// of QU rounds of all of them before the gathers and the arithmetic, so
// each thread has NP x QU record loads, then gathers, in flight: the pass
// is a chain of dependent loads, and their number per iteration sets its
// time.
template <int T, int NP, int QU, bool KIN>
__device__ __forceinline__ void incidence_global_solve(const SolveArgs& A, const IncArgs& I, int r, RedSlots& red)
{
    constexpr int NW = T / 64;
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const DevNet& net = A.net;
    const int64_t f0 = uniform64(net.fib_off[r]), a0 = uniform64(net.free_off[r]), b0 = uniform64(net.bnd_off[r]);
    const int nf = uniform32((int)(net.free_off[r + 1] - a0));
    const int nb = uniform32((int)(net.bnd_off[r + 1] - b0));
    const int64_t rb = uniform64(I.rec_first[r]);
    const int32_t* rq = I.round_first + (int64_t)r * (kIncMaxDeg + 1);
    const int nrec = uniform32(rq[kIncMaxDeg]);
    const float4* recb = I.rec + rb;
    const uint2* stb = I.rec_st + rb;
    const int32_t* permb = I.perm + a0;
    const int64_t gb = uniform64(I.g_first[r]);
    float4* hg = I.hg + gb;
    float4* vg = I.vg + gb;
    float4* ag = I.ag + gb;
    double* hsb = A.h_state + 3 * a0;

    double F[9];
    bool finite = true;
    for (int k = 0; k < 9; ++k) {
        F[k] = A.F[9 * r + k];
        finite = finite && isfinite(F[k]);
    }
    const double J = det3(F);
    if (!finite || !(J > 0.0)) {
        if (tid == 0) {
            A.status[r] = ST_BAD_F;
            A.iters[r] = 0;
            A.Rres[r] = NAN; A.Dres[r] = NAN; A.Bres[r] = NAN;
            for (int k = 0; k < 9; ++k) A.sigma[9 * r + k] = NAN;
        }
        return;
    }
    const bool linear = A.law == kLawLinear;
    double EAd = A.EA, Bd = A.B;
    asm volatile("" : "+s"(EAd), "+s"(Bd));
    const float EA = uniform((float)EAd), Bc = uniform((float)Bd), EAoB = uniform((float)(EAd / Bd));
    const double cr = uniform(A.c[r]);
    const float c = KIN ? 0.f : uniform((float)cr);
    const float cg = uniform((float)cr);

    // ---- records of this F, node state
#pragma unroll 1
    for (int j = tid; j < nrec; j += T) I.rec[rb + j] = inc_record(F, net, f0, I.rec_fib[rb + j]);
    const int64_t be0 = uniform64(net.binc_off[b0]), be1 = uniform64(net.binc_off[b0 + nb]);
#pragma unroll 1
    for (int64_t e = be0 + tid; e < be1; e += T) I.brec[e] = inc_record(F, net, f0, net.binc[e]);
#pragma unroll 1
    for (int p = tid; p < nf; p += T) {
        const int a = permb[p];
        float hx = 0.f, hy = 0.f, hz = 0.f;
        if (A.init == kInitWarm) {
            const double* h = hsb + 3 * a;
            hx = (float)h[0]; hy = (float)h[1]; hz = (float)h[2];
        }
        hg[p] = make_float4(hx, hy, hz, (float)(1.0 / (net.mass[a0 + a] * A.rhoA)));
        vg[p] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (tid < 2) red.g32[tid] = 0u;   // FP32: only the 32-bit time-step slots are used
    if (tid == 0) hg[nf] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();

    // internal force and Gershgorin sum at ranks pp[0 .. NP) (pp ascending,
    // own positions ho; act: the rank is a node)
    auto node_force = [&](const int (&pp)[NP], const bool (&act)[NP], const float4 (&ho)[NP], float (&fx)[NP],
                          float (&fy)[NP], float (&fz)[NP], float (&G)[NP]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < NP; ++i) fx[i] = fy[i] = fz[i] = G[i] = 0.f;
        // a wave's ranks are consecutive, its first lane's node 0 the
        // smallest: the wave stops at the first batch of rounds none of its
        // nodes has
        const int pw = __builtin_amdgcn_readfirstlane(pp[0]);
#pragma unroll 1
        for (int q0 = 0; q0 < kIncMaxDeg; q0 += QU) {
            if (pw >= uniform32(rq[q0 + 1]) - uniform32(rq[q0])) break;
            float4 rc[NP][QU], oh[NP][QU];
            uint2 st[NP][QU];
            bool on[NP][QU];
#pragma unroll
            for (int u = 0; u < QU; ++u) {
                const int R0 = uniform32(rq[q0 + u]), Pq = uniform32(rq[q0 + u + 1]) - R0;
#pragma unroll
                for (int i = 0; i < NP; ++i) {
                    on[i][u] = act[i] && pp[i] < Pq;
                    rc[i][u] = make_float4(0.f, 0.f, 0.f, 0.f);
                    st[i][u] = make_uint2(0u, (uint32_t)nf);
                    if (on[i][u]) {
                        rc[i][u] = recb[R0 + pp[i]];
                        st[i][u] = stb[R0 + pp[i]];
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < NP; ++i)
#pragma unroll
                for (int u = 0; u < QU; ++u) oh[i][u] = hg[st[i][u].y];
#pragma unroll
            for (int i = 0; i < NP; ++i)
#pragma unroll
                for (int u = 0; u < QU; ++u) {
                    const FiberOut<float> f = fiber_eval_scaled<float>(
                        linear, EA, Bc, EAoB, rc[i][u].x, rc[i][u].y, rc[i][u].z, rc[i][u].w,
                        __uint_as_float(st[i][u].x), ho[i].x - oh[i][u].x, ho[i].y - oh[i][u].y,
                        ho[i].z - oh[i][u].z);
                    if (on[i][u]) {
                        fx[i] += f.fx; fy[i] += f.fy; fz[i] += f.fz; G[i] += f.b;
                    }
                }
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) G[i] *= 2.f;
    };
    auto bnorm2 = [&](int t) __attribute__((always_inline)) -> double {
        double acc = 0.0;
#pragma unroll 1
        for (int q = t; q < nb; q += T) {
            double x = 0.0, y = 0.0, z = 0.0;
            const int64_t e1 = net.binc_off[b0 + q + 1];
#pragma unroll 1
            for (int64_t e = net.binc_off[b0 + q]; e < e1; ++e) {
                const float4 rc = I.brec[e];
                const uint2 st = I.brec_st[e];
                const float4 oh = hg[st.y];
                const FiberOut<float> f = fiber_eval_scaled<float>(linear, EA, Bc, EAoB, rc.x, rc.y, rc.z, rc.w,
                                                                   __uint_as_float(st.x), 0.f - oh.x, 0.f - oh.y,
                                                                   0.f - oh.z);
                x += (double)f.fx; y += (double)f.fy; z += (double)f.fz;
            }
            acc += x * x + y * y + z * z;
        }
        return acc;
    };

    // the force pass over the thread's nodes, NP at a time: body(p, ho, v,
    // fx, fy, fz, G) for each node (its position record ho and velocity v)
    auto force_pass = [&](int t, auto&& body) __attribute__((always_inline)) {
#pragma unroll 1
        for (int p0 = t; p0 < nf; p0 += NP * T) {
            int pp[NP];
            bool act[NP];
            float4 ho[NP], v[NP];
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                pp[i] = p0 + i * T;
                act[i] = pp[i] < nf;
                ho[i] = act[i] ? hg[pp[i]] : make_float4(0.f, 0.f, 0.f, 1.f);
                v[i] = act[i] ? vg[pp[i]] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
            float fx[NP], fy[NP], fz[NP], G[NP];
            node_force(pp, act, ho, fx, fy, fz, G);
#pragma unroll
            for (int i = 0; i < NP; ++i)
                if (act[i]) body(pp[i], ho[i], v[i], fx[i], fy[i], fz[i], G[i]);
        }
    };

    // ---- initial force, residual and (optionally) stiffness-scaled mass
    float gpart = 0.f;
    double r2p = 0.0, b2p = 0.0;
    force_pass(tid, [&](int p, float4 ho, float4, float fx, float fy, float fz, float G) __attribute__((always_inline)) {
        float im = ho.w;
        if (A.mass_mode == kMassScaled) {
            im = G > 0.f ? 4.f / G : 1.f;
            ho.w = im;
            hg[p] = ho;
        }
        ag[p] = make_float4(-fx * im, -fy * im, -fz * im, 0.f);
        gpart = fmax(gpart, G * im);
        r2p += (double)fx * fx + (double)fy * fy + (double)fz * fz;
    });
    b2p = bnorm2(tid);
    double gmax;
    double R2 = 0.0, D2 = 0.0, B2 = 0.0;
    int parity = 0;
    block_reduce<float, NW>(red, tid, parity, gpart, r2p, 0.0, b2p, true, gmax, R2, D2, B2);

    int64_t n = 0;
    int status = ST_CONVERGED;
    const int ce = A.check_every > 0 ? A.check_every : 1;
    int countdown = ce;
    bool done = sqrt(R2) <= fmax(A.tol_abs, A.tol_rel * sqrt(B2));   // v = 0: damping norm is 0
    double Rref = uniform(sqrt(R2));
    int stall = 0;
    if (!isfinite(R2)) {
        status = ST_NONFINITE;
        done = true;
    }
    if (!done && n >= A.n_max) {
        status = ST_MAXITER;
        done = true;
    }
    auto time_step = [&](double g) __attribute__((always_inline)) -> double {
        return uniform((double)(uniform((float)(2.0 * A.alpha)) * __builtin_amdgcn_rsqf((float)g)));
    };
    double dt = time_step(gmax);
    double ke_prev = 0.0;

    while (!done) {
        const int t = opaque_tid();
        const float hdt = (float)(0.5 * dt), rdt = (float)dt;
        // half-step velocity and position update
#pragma unroll 1
        for (int p = t; p < nf; p += T) {
            float4 v = vg[p], h = hg[p];
            const float4 a = ag[p];
            v.x += hdt * a.x; v.y += hdt * a.y; v.z += hdt * a.z;
            h.x += rdt * v.x; h.y += rdt * v.y; h.z += rdt * v.z;
            vg[p] = v;
            hg[p] = h;
        }
        __syncthreads();
        const int tb = opaque_tid();
        ++n;
        const bool check = --countdown == 0;
        if (check) countdown = ce;
        gpart = 0.f;
        r2p = 0.0;
        double d2p = 0.0, kep = 0.0;
        force_pass(tb, [&](int p, float4 ho, float4 v, float fx, float fy, float fz, float G) __attribute__((always_inline)) {
            const float im = ho.w;
            float4 a;
            a.x = -fx * im - c * v.x;
            a.y = -fy * im - c * v.y;
            a.z = -fz * im - c * v.z;
            a.w = 0.f;
            v.x += hdt * a.x; v.y += hdt * a.y; v.z += hdt * a.z;
            ag[p] = a;
            vg[p] = v;
            gpart = fmax(gpart, G * im);
            if constexpr (KIN) kep += 0.5 * (double)((v.x * v.x + v.y * v.y + v.z * v.z) * dev_rcp(im));
            if (check) {
                r2p += (double)fx * fx + (double)fy * fy + (double)fz * fz;
                const float cm = cg * dev_rcp(im);
                const double px = (double)(cm * v.x), py = (double)(cm * v.y), pz = (double)(cm * v.z);
                d2p += px * px + py * py + pz * pz;
            }
        });
        if (check) b2p = bnorm2(tb);
        parity ^= 1;
        double r2n = R2, d2n = D2, b2n = B2, ke = 0.0;
        block_reduce<float, NW, KIN>(red, tb, parity, gpart, r2p, d2p, b2p, check, gmax, r2n, d2n, b2n, kep, &ke);
        if constexpr (KIN) {
            // a kinetic-energy peak was passed: restart every node from rest
            // (the stored acceleration is already -f/M); the velocities are
            // read by their own threads only, so no barrier is needed
            if (ke < ke_prev) {
#pragma unroll 1
                for (int p = tb; p < nf; p += T) vg[p] = make_float4(0.f, 0.f, 0.f, 0.f);
                ke = 0.0;
                if (check) d2n = 0.0;
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
            const double tol = fmax(A.tol_abs, A.tol_rel * Bn);
            if (Rn <= tol && Dn <= tol) break;
            if (stagnated(A, Rn, Dn, Bn, Rref, stall)) {
                status = ST_STAGNATED;
                break;
            }
            Rref = uniform(Rref);
        }
        if (!(gmax > 0.0) || !isfinite(gmax)) {
            status = ST_NONFINITE;
            break;
        }
        if (n >= A.n_max) {
            status = ST_MAXITER;
            break;
        }
        dt = time_step(gmax);
    }

    // ---- fluctuation state in the packed order
    const int te = opaque_tid();
    __syncthreads();
#pragma unroll 1
    for (int p = te; p < nf; p += T) {
        const float4 h = hg[p];
        double* hs = hsb + 3 * permb[p];
        hs[0] = (double)h.x; hs[1] = (double)h.y; hs[2] = (double)h.z;
    }
    if (te == 0) {
        A.status[r] = status;
        A.iters[r] = n;
        A.Rres[r] = sqrt(R2);
        A.Dres[r] = sqrt(D2);
        A.Bres[r] = sqrt(B2);
    }
    __syncthreads();
}

template <int T, int NP, int QU, bool KIN>
__global__ __launch_bounds__(T) void dr_incidence_global_kernel(SolveArgs A, IncArgs I)
{
    __shared__ RedSlots red;
    __shared__ int task;
    for (;;) {
        if (threadIdx.x == 0) task = atomicAdd(A.queue, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(task);
        __syncthreads();
        if (t >= A.n_list) break;
        incidence_global_solve<T, NP, QU, KIN>(A, I, __builtin_amdgcn_readfirstlane(A.list[t]), red);
    }
}

// ------------------------------------------------------------------ stress kernel
// Homogenized stress of every RVE from its final fluctuation state, one
// workgroup per RVE: each fiber with a boundary end is re-evaluated in FP64
// and f_b (x) x_b is accumulated at that end (x_b = F Xm_b); per-thread sums,
// pairwise wave sums and a compensated sum over waves, then / (det F V0).
// RVEs whose status is NONFINITE or BAD_F get NaN (a stagnated RVE gets its
// stress like a converged one).
constexpr int kStressThreads = 256;

__global__ __launch_bounds__(kStressThreads) void stress_kernel(SolveArgs A)
{
    const int r = blockIdx.x;
    const DevNet& net = A.net;
    const int st = A.status[r];
    if (st == ST_NONFINITE || st == ST_BAD_F) {
        if (threadIdx.x < 9) A.sigma[9 * r + threadIdx.x] = NAN;
        return;
    }
    const int64_t f0 = net.fib_off[r], nfib = net.fib_off[r + 1] - f0;
    const int64_t a0 = net.free_off[r], nf = net.free_off[r + 1] - a0;
    const int64_t b0 = net.bnd_off[r];
    double F[9];
    for (int k = 0; k < 9; ++k) F[k] = A.F[9 * r + k];
    const double J = det3(F);
    double s9[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) s9[p] = 0.0;
#pragma unroll 1
    for (int64_t k = threadIdx.x; k < nfib; k += kStressThreads) {
        uint32_t e = net.ends[f0 + k];
        int i = e & 0xffff, j = e >> 16;
        if (i < nf && j < nf) continue;
        const double* d0 = net.d0 + 3 * (f0 + k);
        double L0 = net.L0[f0 + k];
        double Dx = F[0] * d0[0] + F[1] * d0[1] + F[2] * d0[2];
        double Dy = F[3] * d0[0] + F[4] * d0[1] + F[5] * d0[2];
        double Dz = F[6] * d0[0] + F[7] * d0[1] + F[8] * d0[2];
        double q0 = (Dx * Dx + Dy * Dy + Dz * Dz) - L0 * L0;
        double dh[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 3; ++c) {
            if (j < nf) dh[c] += A.h_state[3 * (a0 + j) + c];
            if (i < nf) dh[c] -= A.h_state[3 * (a0 + i) + c];
        }
        FiberOut<double> o = fiber_eval_exact(A.law, A.EA, A.B, Dx, Dy, Dz, q0, L0, dh[0], dh[1], dh[2]);
        const double fvv[3] = {o.fx, o.fy, o.fz};
        for (int end = 0; end < 2; ++end) {
            int node = end ? j : i;
            if (node < nf) continue;
            const double* Xm = net.Xb + 3 * (b0 + (node - nf));
            double xb[3] = {F[0] * Xm[0] + F[1] * Xm[1] + F[2] * Xm[2], F[3] * Xm[0] + F[4] * Xm[1] + F[5] * Xm[2],
                            F[6] * Xm[0] + F[7] * Xm[1] + F[8] * Xm[2]};
            double sg = end ? 1.0 : -1.0;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) s9[3 * p + q] += sg * fvv[p] * xb[q];
        }
    }
    stress_finish<kStressThreads / 64>(s9, J, net.V0[r], A.sigma + 9 * r);
}

// Zero n work counters (a kernel rather than a memset node, so that a
// solve can be captured in a HIP graph and replayed).
__global__ void reset_counters(int32_t* c, int n)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

// Fill n words with zero (graph-capturable, unlike a memset node).
__global__ void zero_words(int32_t* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Before a team launch: every RVE of its list starts as non-finite, so an RVE
// that a launch which gave up never reached reports it.
__global__ void mark_unfinished(const int32_t* list, int n, int32_t* status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) status[list[i]] = ST_NONFINITE;
}

hipError_t launch_zero32(int32_t* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(zero_words, dim3(grid), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_mark_unfinished(const int32_t* list, int n, int32_t* status, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mark_unfinished, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, list, n, status);
    return hipGetLastError();
}

// Longest-processing-time order of the work lists: one workgroup per launch
// group sorts the group's RVE ids by the estimated cost iters[r] * fibers(r)
// of the previous solve, largest first, ties in the present order (a stable
// sort: the key carries the position), with a bitonic sort of packed 64-bit
// keys (cost << 14 | (16383 - position)) in LDS.  Groups of more than
// kOrderMax RVEs keep their order.  Only the order in which the persistent
// workgroups take RVEs changes; every RVE's arithmetic is the same.
constexpr int kOrderThreads = 1024;

__global__ __launch_bounds__(kOrderThreads) void order_by_cost_kernel(OrderArgs o)
{
    __shared__ unsigned long long key[kOrderMax];
    __shared__ int32_t id[kOrderMax];
    const int g = blockIdx.x;
    const int n = o.count[g];
    if (n < 2 || n > kOrderMax) return;
    int32_t* list = o.list + o.first[g];
    int m = 2;
    while (m < n) m <<= 1;
    for (int i = threadIdx.x; i < m; i += kOrderThreads) {
        unsigned long long k = 0ull;   // padding sorts last
        if (i < n) {
            const int32_t r = list[i];
            id[i] = r;
            const int64_t it = o.iters[r] > 0 ? o.iters[r] : 0;
            const int64_t nf = o.fib_off[r + 1] - o.fib_off[r];
            unsigned long long cost = (unsigned long long)it * (unsigned long long)(nf > 0 ? nf : 0);
            cost = cost < (1ull << 48) ? cost : (1ull << 48) - 1ull;
            k = ((cost + 1ull) << 14) | (unsigned long long)(kOrderMax - 1 - i);
        }
        key[i] = k;
    }
    __syncthreads();
    // bitonic sort, descending
    for (int size = 2; size <= m; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < (m >> 1); t += kOrderThreads) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool desc = (lo & size) == 0;
                const unsigned long long a = key[lo], b = key[hi];
                if ((a < b) == desc) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += kOrderThreads)
        list[i] = id[kOrderMax - 1 - (int)(key[i] & (unsigned long long)(kOrderMax - 1))];
}

hipError_t launch_order_by_cost(const OrderArgs& o, int n_groups, hipStream_t s)
{
    if (n_groups <= 0) return hipSuccess;
    if (n_groups > kOrderGroups) return hipErrorInvalidValue;
    hipLaunchKernelGGL(order_by_cost_kernel, dim3((unsigned)n_groups), dim3(kOrderThreads), 0, s, o);
    return hipGetLastError();
}

hipError_t launch_reset(int32_t* counters, int n, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, counters, n);
    return hipGetLastError();
}

hipError_t launch_stress(const SolveArgs& a, int n_rve, hipStream_t s)
{
    if (n_rve <= 0) return hipSuccess;
    hipLaunchKernelGGL(stress_kernel, dim3(n_rve), dim3(kStressThreads), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launch helpers
template <typename Real, int T, int SF, int SN, bool KIN>
static hipError_t launch_res(const SolveArgs& a, size_t lds, int grid, hipStream_t s)
{
    auto k = dr_resident_kernel<Real, T, SF, SN, KIN>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(T), lds, s, a);
    return hipGetLastError();
}

template <typename Real, int T, int SF, int SN, bool KIN>
static hipError_t spill_res(size_t* bytes)
{
    hipFuncAttributes at;
    hipError_t e = hipFuncGetAttributes(&at, (const void*)dr_resident_kernel<Real, T, SF, SN, KIN>);
    *bytes = at.localSizeBytes;
    return e;
}

template <typename Real, int T, int SF, int SN, bool KIN>
static hipError_t occ_res(size_t lds, int* blocks)
{
    auto k = dr_resident_kernel<Real, T, SF, SN, KIN>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void*)k, T, lds);
}

// precision x damping (viscous or kinetic) for one resident variant
#define RVE_RES_PK(FN, T, SF, SN, ...)                                                                \
    (kin ? (fp64 ? FN<double, T, SF, SN, true>(__VA_ARGS__) : FN<float, T, SF, SN, true>(__VA_ARGS__))  \
         : (fp64 ? FN<double, T, SF, SN, false>(__VA_ARGS__) : FN<float, T, SF, SN, false>(__VA_ARGS__)))
#define RVE_RES_DISPATCH(FN, ...)                                                                     \
    switch (variant) {                                                                                \
    case 0: return RVE_RES_PK(FN, 256, 4, 2, __VA_ARGS__);                                            \
    case 1: return RVE_RES_PK(FN, 512, 4, 2, __VA_ARGS__);                                            \
    case 2: return RVE_RES_PK(FN, 768, 4, 2, __VA_ARGS__);                                            \
    case 3: return RVE_RES_PK(FN, 512, 6, 3, __VA_ARGS__);                                            \
    case 4: return RVE_RES_PK(FN, 1024, 4, 2, __VA_ARGS__);                                           \
    case 5: return RVE_RES_PK(FN, 1024, 6, 3, __VA_ARGS__);                                           \
    default: return hipErrorInvalidValue;                                                             \
    }

hipError_t launch_resident(int variant, bool fp64, const SolveArgs& a, size_t lds, int grid, hipStream_t s)
{
    const bool kin = a.kinetic != 0;
    RVE_RES_DISPATCH(launch_res, a, lds, grid, s)
}

hipError_t max_resident_blocks(int variant, bool fp64, bool kin, size_t lds, int* blocks)
{
    RVE_RES_DISPATCH(occ_res, lds, blocks)
}

hipError_t resident_scratch_bytes(int variant, bool fp64, bool kin, size_t* bytes)
{
    RVE_RES_DISPATCH(spill_res, bytes)
}

template <typename Real, int T>
static hipError_t launch_streamed_t(const SolveArgs& a, int grid, hipStream_t s)
{
    const size_t lds = 3 * sizeof(Real) * (size_t)a.lds_h_nodes;
    const void* k = a.kinetic ? (const void*)dr_streamed_kernel<Real, T, true> : (const void*)dr_streamed_kernel<Real, T, false>;
    if (lds > 0) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    void* args[] = {const_cast<SolveArgs*>(&a)};
    return hipLaunchKernel(k, dim3(grid), dim3(T), args, lds, s);
}

hipError_t launch_streamed(bool fp64, const SolveArgs& a, int grid, int threads, hipStream_t s)
{
    if (threads == 256) return fp64 ? launch_streamed_t<double, 256>(a, grid, s) : launch_streamed_t<float, 256>(a, grid, s);
    return fp64 ? launch_streamed_t<double, 1024>(a, grid, s) : launch_streamed_t<float, 1024>(a, grid, s);
}

size_t streamed_lds_cap() { return 150 * 1024; }

template <typename Real, int T>
static hipError_t streamed_private_t(bool kin, size_t* bytes)
{
    return max_private_bytes({kin ? (const void*)dr_streamed_kernel<Real, T, true> : (const void*)dr_streamed_kernel<Real, T, false>},
                             bytes);
}

hipError_t streamed_scratch_bytes(bool fp64, bool kin, int threads, size_t* bytes)
{
    if (threads == 256) return fp64 ? streamed_private_t<double, 256>(kin, bytes) : streamed_private_t<float, 256>(kin, bytes);
    if (threads == 1024)
        return fp64 ? streamed_private_t<double, 1024>(kin, bytes) : streamed_private_t<float, 1024>(kin, bytes);
    return hipErrorInvalidValue;
}

template <int T, int S, int QR, bool KIN>
static hipError_t launch_inc_t(const SolveArgs& a, const IncArgs& inc, size_t lds, int grid, hipStream_t s)
{
    auto k = dr_incidence_kernel<T, S, QR, KIN>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(T), lds, s, a, inc);
    return hipGetLastError();
}

template <int T, int S, int QR, bool KIN>
static hipError_t occ_inc_t(size_t lds, int* blocks)
{
    auto k = dr_incidence_kernel<T, S, QR, KIN>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void*)k, T, lds);
}

template <int T, int S, int QR, bool KIN>
static hipError_t spill_inc_t(size_t* bytes)
{
    return max_private_bytes({(const void*)dr_incidence_kernel<T, S, QR, KIN>}, bytes);
}

#define RVE_INC_DISPATCH(FN, ...)                                                                      \
    switch (variant) {                                                                                \
    case 0: return kin ? FN<768, 16, 2, true>(__VA_ARGS__) : FN<768, 16, 4, false>(__VA_ARGS__);       \
    default: return hipErrorInvalidValue;                                                             \
    }

hipError_t launch_incidence(int variant, const SolveArgs& a, const IncArgs& inc, size_t lds, int grid, hipStream_t s)
{
    const bool kin = a.kinetic != 0;
    RVE_INC_DISPATCH(launch_inc_t, a, inc, lds, grid, s)
}

hipError_t incidence_blocks(int variant, bool kin, size_t lds, int* blocks)
{
    RVE_INC_DISPATCH(occ_inc_t, lds, blocks)
}

hipError_t incidence_scratch_bytes(int variant, bool kin, size_t* bytes)
{
    RVE_INC_DISPATCH(spill_inc_t, bytes)
}

// global-mode build: nodes per thread taken together and rounds per load batch
constexpr int kIncGNP = 2, kIncGQU = 2;

static const void* incg_kernel(bool kin)
{
    constexpr int T = kIncGlobalThreads;
    return kin ? (const void*)dr_incidence_global_kernel<T, kIncGNP, kIncGQU, true>
               : (const void*)dr_incidence_global_kernel<T, kIncGNP, kIncGQU, false>;
}

hipError_t launch_incidence_global(const SolveArgs& a, const IncArgs& inc, int grid, hipStream_t s)
{
    void* args[] = {const_cast<SolveArgs*>(&a), const_cast<IncArgs*>(&inc)};
    return hipLaunchKernel(incg_kernel(a.kinetic != 0), dim3(grid), dim3(kIncGlobalThreads), args, 0, s);
}

hipError_t incidence_global_blocks(bool kin, int* blocks)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, incg_kernel(kin), kIncGlobalThreads, 0);
}

hipError_t incidence_global_scratch_bytes(bool kin, size_t* bytes)
{
    return max_private_bytes({incg_kernel(kin)}, bytes);
}

hipError_t kernels_fixed_private(size_t* bytes)
{
    return max_private_bytes({(const void*)stress_kernel, (const void*)reset_counters, (const void*)zero_words,
                              (const void*)mark_unfinished, (const void*)order_by_cost_kernel},
                             bytes);
}

}  // namespace rve
