// The paper's finite-difference material tangent (Section 3.2, material
// stiffness): per RVE, six probe relaxations under the right stretch U plus
// h times each probing direction, forward differences of the second
// Piola-Kirchhoff stress, the Mandel solve for A = dPi/dE and the
// push-forward to the spatial tangent C.  The probe relaxations run as one
// batched solve (rve_host.hip); this file holds the per-RVE 3x3 / 6x6
// algebra (host) and the kernel that seeds each probe with the base state
// rotated back to the stretch frame.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rve_internal.h"

namespace rve {

namespace {

const double kS2 = 1.41421356237309504880;

// Mandel order 11, 22, 33, 23, 13, 12
const int kMi[6] = {0, 1, 2, 1, 0, 0};
const int kMj[6] = {0, 1, 2, 2, 2, 1};

void mandel_vec(const double* S, double* v)
{
    for (int I = 0; I < 6; ++I) v[I] = (I < 3 ? 1.0 : kS2) * S[3 * kMi[I] + kMj[I]];
}

void from_mandel_vec(const double* v, double* S)
{
    for (int I = 0; I < 6; ++I) {
        const double s = v[I] / (I < 3 ? 1.0 : kS2);
        S[3 * kMi[I] + kMj[I]] = s;
        S[3 * kMj[I] + kMi[I]] = s;
    }
}

void mat3_mul(const double* A, const double* B, double* C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

double det3h(const double* F)
{
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
}

void inv3(const double* F, double* G)
{
    const double id = 1.0 / det3h(F);
    G[0] = (F[4] * F[8] - F[5] * F[7]) * id;
    G[1] = (F[2] * F[7] - F[1] * F[8]) * id;
    G[2] = (F[1] * F[5] - F[2] * F[4]) * id;
    G[3] = (F[5] * F[6] - F[3] * F[8]) * id;
    G[4] = (F[0] * F[8] - F[2] * F[6]) * id;
    G[5] = (F[2] * F[3] - F[0] * F[5]) * id;
    G[6] = (F[3] * F[7] - F[4] * F[6]) * id;
    G[7] = (F[1] * F[6] - F[0] * F[7]) * id;
    G[8] = (F[0] * F[4] - F[1] * F[3]) * id;
}

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations:
// S = V diag(w) V^T (columns of V are the eigenvectors).
void sym3_eig(const double* S, double* w, double* V)
{
    double a[9];
    for (int k = 0; k < 9; ++k) {
        a[k] = S[k];
        V[k] = (k % 4 == 0) ? 1.0 : 0.0;
    }
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
        const double tot = off + a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = a[3 * p + q];
                if (apq == 0.0) continue;
                const double theta = (a[3 * q + q] - a[3 * p + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                // a <- J^T a J with J the rotation in the (p, q) plane
                for (int k = 0; k < 3; ++k) {
                    const double akp = a[3 * k + p], akq = a[3 * k + q];
                    a[3 * k + p] = c * akp - s * akq;
                    a[3 * k + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = a[3 * p + k], aqk = a[3 * q + k];
                    a[3 * p + k] = c * apk - s * aqk;
                    a[3 * q + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[3 * k + p], vkq = V[3 * k + q];
                    V[3 * k + p] = c * vkp - s * vkq;
                    V[3 * k + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int k = 0; k < 3; ++k) w[k] = a[4 * k];
}

// F = R U: U = sqrt(F^T F), R = F U^-1.
void polar3(const double* F, double* R, double* U)
{
    double C[9], w[3], V[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
    sym3_eig(C, w, V);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += V[3 * i + k] * sqrt(w[k]) * V[3 * j + k];
            U[3 * i + j] = s;
        }
    double Ui[9];
    inv3(U, Ui);
    mat3_mul(F, Ui, R);
}

// Mandel vector of Pi = J F^-1 sigma F^-T.
void pk2_mandel(const double* F, const double* sigma, double* v)
{
    double Fi[9], t[9], P[9], FiT[9];
    inv3(F, Fi);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) FiT[3 * i + j] = Fi[3 * j + i];
    mat3_mul(Fi, sigma, t);
    mat3_mul(t, FiT, P);
    const double J = det3h(F);
    for (int k = 0; k < 9; ++k) P[k] *= J;
    mandel_vec(P, v);
}

// The probing directions (columns, Mandel form) printed in Section 3.2.
void probe_T(double T[6][6])
{
    const double h2 = 0.5 * kS2;
    const double t[6][6] = {{0.5, 0, 0, 0, h2, h2}, {0, 0.5, 0, h2, 0, h2}, {0, 0, 0.5, h2, h2, 0},
                            {0, 0, 0, 1, 0, 0},     {0, 0, 0, 0, 1, 0},     {0, 0, 0, 0, 0, 1}};
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) T[i][j] = t[i][j];
}

// [dE/dU] of the stretch U in Mandel form, as printed in Section 3.2.
void mandel_M(const double* U, double M[6][6])
{
    const double u11 = U[0], u22 = U[4], u33 = U[8], u12 = U[1], u13 = U[2], u23 = U[5];
    const double s = kS2;
    const double m[6][6] = {{2 * u11, 0, 0, 0, s * u13, s * u12},
                            {0, 2 * u22, 0, s * u23, 0, s * u12},
                            {0, 0, 2 * u33, s * u23, s * u13, 0},
                            {0, s * u23, s * u23, u22 + u33, u12, u13},
                            {s * u13, 0, s * u13, u12, u11 + u33, u23},
                            {s * u12, s * u12, 0, u13, u23, u11 + u22}};
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) M[i][j] = 0.5 * m[i][j];
}

// Solve X B = P for X (6x6) by Gauss-Jordan on B^T X^T = P^T with partial
// pivoting.  Returns false when B is singular.
bool right_solve6(double B[6][6], double P[6][6], double X[6][6])
{
    double a[6][12];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            a[i][j] = B[j][i];
            a[i][6 + j] = P[j][i];
        }
    for (int c = 0; c < 6; ++c) {
        int piv = c;
        for (int i = c + 1; i < 6; ++i)
            if (fabs(a[i][c]) > fabs(a[piv][c])) piv = i;
        if (!(fabs(a[piv][c]) > 0.0)) return false;
        if (piv != c)
            for (int j = 0; j < 12; ++j) {
                double t = a[c][j];
                a[c][j] = a[piv][j];
                a[piv][j] = t;
            }
        const double d = a[c][c];
        for (int j = 0; j < 12; ++j) a[c][j] /= d;
        for (int i = 0; i < 6; ++i)
            if (i != c) {
                const double f = a[i][c];
                for (int j = 0; j < 12; ++j) a[i][j] -= f * a[c][j];
            }
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) X[j][i] = a[i][6 + j];   // X^T = solution
    return true;
}

// Rotate the base fluctuation state into the stretch frame for every probe
// copy: h_probe = R^T h_base (copy c of RVE r is probe RVE 6 r + c).
__global__ void probe_state_kernel(ProbeStateArgs A)
{
    const int64_t p = blockIdx.x;
    const int64_t r = p / 6;
    double Rm[9];
    for (int k = 0; k < 9; ++k) Rm[k] = A.Rm[9 * r + k];
    const int64_t a0 = A.probe_free_off[p], a1 = A.probe_free_off[p + 1];
#pragma unroll 1
    for (int64_t a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
        const double* hb = A.h_base + 3 * A.map[a];
        const double x = hb[0], y = hb[1], z = hb[2];
        double* hp = A.h_probe + 3 * a;
        hp[0] = Rm[0] * x + Rm[3] * y + Rm[6] * z;
        hp[1] = Rm[1] * x + Rm[4] * y + Rm[7] * z;
        hp[2] = Rm[2] * x + Rm[5] * y + Rm[8] * z;
    }
}

}  // namespace

void fd_prepare(const double* F, double h, double* Fprobe, double* Rm)
{
    double U[9];
    polar3(F, Rm, U);
    double T[6][6];
    probe_T(T);
    for (int c = 0; c < 6; ++c) {
        double v[6], S[9];
        for (int I = 0; I < 6; ++I) v[I] = T[I][c];
        from_mandel_vec(v, S);
        for (int k = 0; k < 9; ++k) Fprobe[9 * c + k] = U[k] + h * S[k];
    }
}

bool fd_finish(const double* F, const double* sigma, const double* sigma_probe, const double* Fprobe, double h,
               double* C, double* A)
{
    double Rm[9], U[9];
    polar3(F, Rm, U);
    double M[6][6], T[6][6], MT[6][6], P[6][6], A6[6][6];
    mandel_M(U, M);
    probe_T(T);
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += M[i][k] * T[k][j];
            MT[i][j] = s;
        }
    double pi0[6];
    pk2_mandel(F, sigma, pi0);
    for (int c = 0; c < 6; ++c) {
        double pic[6];
        pk2_mandel(Fprobe + 9 * c, sigma_probe + 9 * c, pic);
        for (int I = 0; I < 6; ++I) P[I][c] = (pic[I] - pi0[I]) / h;
    }
    if (!right_solve6(MT, P, A6)) return false;
    // C = Q A Q^T / J with Q the Mandel matrix of S -> F S F^T
    double Q[6][6];
    for (int J = 0; J < 6; ++J) {
        double e[6] = {0, 0, 0, 0, 0, 0}, S[9], t[9], FS[9], Ft[9], v[6];
        e[J] = 1.0;
        from_mandel_vec(e, S);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Ft[3 * i + j] = F[3 * j + i];
        mat3_mul(F, S, t);
        mat3_mul(t, Ft, FS);
        mandel_vec(FS, v);
        for (int I = 0; I < 6; ++I) Q[I][J] = v[I];
    }
    const double Jd = det3h(F);
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k)
                for (int l = 0; l < 6; ++l) s += Q[i][k] * A6[k][l] * Q[j][l];
            C[6 * i + j] = s / Jd;
            if (A) A[6 * i + j] = A6[i][j];
        }
    return true;
}

hipError_t launch_probe_state(const ProbeStateArgs& a, int64_t n_probe, hipStream_t s)
{
    if (n_probe <= 0) return hipSuccess;
    hipLaunchKernelGGL(probe_state_kernel, dim3((unsigned)n_probe), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t fd_fixed_private(size_t* bytes)
{
    return max_private_bytes({(const void*)probe_state_kernel}, bytes);
}

}  // namespace rve
