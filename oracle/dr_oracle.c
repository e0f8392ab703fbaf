/*
 * FP64 CPU oracle for the batched fiber-network RVE solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header or constant with the HIP
 * path: it is a plain, slow, obviously-correct restatement of the method.
 *
 * What it computes (paper: Section 2, eqs. micro_coords, affine-bc and the
 * boundary-traction form of the homogenized stress; Section 3.2, Algorithm
 * "Dynamic Relaxation"):
 *
 *   O1  Reference coordinates are centred on the RVE centre, Xm = X - c0
 *       (the RVE centroid coincides with the macroscale material point).
 *   O2  Boundary nodes follow the affine map x_b = F Xm_b (affine BC).
 *   O3  Free nodes start at x_a = F Xm_a (affine start) or x_a = Xm_a
 *       (reference start) or a caller-given state.
 *   O4  Lumped (diagonal) mass M_a = 1/2 rhoA sum_{fibers f at a} L0_f, or,
 *       since the inertial parameters of the relaxation are fictitious
 *       (Section 3.2), the stiffness-scaled mass M_a = G_a(x0)/4 of the
 *       classical dynamic-relaxation literature the paper cites, with G_a the
 *       Gershgorin row sum of O6 at the starting state (so dt = alpha there).
 *   O5  Truss fibers: d = x_j - x_i, l = |d|, eps = l/L0 - 1, axial force
 *       T(eps) (linear: EA eps; exponential: EA (exp(B eps) - 1)/B for
 *       eps >= 0 and EA eps below), internal force +T d/l on node j and
 *       -T d/l on node i.
 *   O6  Time step from a block-Gershgorin bound on the largest eigenvalue of
 *       M^-1 K: per fiber b_f = max(k_t/L0, |T|/l) with k_t = dT/deps; per
 *       node G_a = 2 sum b_f; dt = alpha * 2 / sqrt(max_a G_a / M_a).
 *   O7  Mass-proportional viscous damping force c M v at the half step.
 *   O8  Two-step central difference, stopped on the free-DOF residual
 *       R = |f_free|_2 (external force is zero) and on the damping-force
 *       norm c |M v|_2, both against max(tol_abs, tol_rel |f_bnd|_2).
 *       Optional stagnation stop (floor_tol_rel > 0): after
 *       stall_checks consecutive tests in which R did not fall below half
 *       of a reference value (R of the start, replaced by R each time R
 *       falls below half of it), with R and c |M v|_2 both within
 *       floor_tol_rel |f_bnd|_2, the run stops as stagnated at the
 *       precision floor; the stress is evaluated as for a converged run.
 *   O9  Homogenized Cauchy stress from the boundary reactions:
 *       sigma_ij = 1/(det F V0) sum_b f_b,i x_b,j.
 *
 * All arithmetic is double precision, one RVE at a time; the batch entry
 * point spreads whole RVEs over POSIX threads.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_LINEAR 0
#define OR_EXP 1

#define OR_INIT_AFFINE 0
#define OR_INIT_REFERENCE 1
#define OR_INIT_GIVEN 2

#define OR_MASS_LUMPED 0
#define OR_MASS_SCALED 1

#define OR_CONVERGED 0
#define OR_MAXITER 1
#define OR_NONFINITE 2
#define OR_BAD_F 3
#define OR_STAGNATED 8

typedef struct {
    int32_t law;
    int32_t init;
    int32_t mass;
    int32_t pad_;
    double EA, B, rhoA, alpha;
    double tol_abs, tol_rel;
    int64_t n_max;
    double floor_tol_rel;   /* stagnation stop; 0 = off */
    int32_t stall_checks;
    int32_t pad2_;
} or_opts;

/* ---------------------------------------------------------------- fiber law */
/* Axial force T and its strain derivative k_t = dT/deps (O5). */
static void fiber_law(const or_opts* o, double eps, double* T, double* kt)
{
    if (o->law == OR_EXP && eps >= 0.0) {
        double e = exp(o->B * eps);
        *T = o->EA * (e - 1.0) / o->B;
        *kt = o->EA * e;
    } else {
        *T = o->EA * eps;
        *kt = o->EA;
    }
}

/* Stored energy of one fiber, W = L0 * integral_0^eps T(e) de. */
static double fiber_energy(const or_opts* o, double eps, double L0)
{
    if (o->law == OR_EXP && eps >= 0.0) {
        double Bb = o->B;
        return L0 * o->EA * ((exp(Bb * eps) - 1.0) / Bb - eps) / Bb;
    }
    return L0 * o->EA * eps * eps / 2.0;
}

static double det3(const double* F)
{
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
}

static void matvec3(const double* F, const double* X, double* y)
{
    for (int i = 0; i < 3; ++i)
        y[i] = F[3 * i + 0] * X[0] + F[3 * i + 1] * X[1] + F[3 * i + 2] * X[2];
}

/*
 * Internal forces at every node (O5), the per-node Gershgorin sums G (O6)
 * and the total stored energy.  f and G are overwritten.  G may be NULL.
 */
void or_forces(int64_t n_nodes, int64_t n_fib, const double* x, const int32_t* fib,
               const double* L0, const or_opts* o, double* f, double* G, double* W)
{
    memset(f, 0, sizeof(double) * 3 * (size_t)n_nodes);
    if (G) memset(G, 0, sizeof(double) * (size_t)n_nodes);
    double energy = 0.0;
    for (int64_t k = 0; k < n_fib; ++k) {
        int32_t i = fib[2 * k], j = fib[2 * k + 1];
        double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
        double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double eps = l / L0[k] - 1.0;
        double T, kt;
        fiber_law(o, eps, &T, &kt);
        energy += fiber_energy(o, eps, L0[k]);
        for (int c = 0; c < 3; ++c) {
            double fc = T * d[c] / l;
            f[3 * j + c] += fc;
            f[3 * i + c] -= fc;
        }
        if (G) {
            double b1 = kt / L0[k], b2 = fabs(T) / l;
            double b = b1 > b2 ? b1 : b2;
            G[i] += 2.0 * b;
            G[j] += 2.0 * b;
        }
    }
    if (W) *W = energy;
}

/*
 * Dense stiffness K = d f_int / d x (3 n_nodes square, row-major) for tiny
 * networks.  Each fiber contributes the 3x3 block
 *   Kf = (k_t/L0) n n^T + (T/l) (I - n n^T)
 * to (j,j) and (i,i) and -Kf to (i,j) and (j,i).
 */
void or_stiffness_dense(int64_t n_nodes, int64_t n_fib, const double* x, const int32_t* fib,
                        const double* L0, const or_opts* o, double* K)
{
    int64_t N = 3 * n_nodes;
    memset(K, 0, sizeof(double) * (size_t)(N * N));
    for (int64_t k = 0; k < n_fib; ++k) {
        int32_t i = fib[2 * k], j = fib[2 * k + 1];
        double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
        double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double n[3] = {d[0] / l, d[1] / l, d[2] / l};
        double T, kt;
        fiber_law(o, l / L0[k] - 1.0, &T, &kt);
        double a = kt / L0[k], g = T / l;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double blk = a * n[r] * n[c] + g * ((r == c ? 1.0 : 0.0) - n[r] * n[c]);
                K[(3 * j + r) * N + 3 * j + c] += blk;
                K[(3 * i + r) * N + 3 * i + c] += blk;
                K[(3 * i + r) * N + 3 * j + c] -= blk;
                K[(3 * j + r) * N + 3 * i + c] -= blk;
            }
    }
}

/* sigma = 1/(det F V0) sum_b f_b (x) x_b   (O9) */
void or_stress(int64_t n_nodes, const double* x, const double* f, const uint8_t* is_bnd,
               const double* F, double V0, double* sigma)
{
    double tau[9] = {0};
    for (int64_t a = 0; a < n_nodes; ++a) {
        if (!is_bnd[a]) continue;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) tau[3 * i + j] += f[3 * a + i] * x[3 * a + j];
    }
    double J = det3(F);
    for (int k = 0; k < 9; ++k) sigma[k] = tau[k] / (J * V0);
}

/* Reference rest lengths L0_f = |X_j - X_i|. */
void or_rest_lengths(int64_t n_fib, const double* X, const int32_t* fib, double* L0)
{
    for (int64_t k = 0; k < n_fib; ++k) {
        int32_t i = fib[2 * k], j = fib[2 * k + 1];
        double d0 = X[3 * j] - X[3 * i], d1 = X[3 * j + 1] - X[3 * i + 1], d2 = X[3 * j + 2] - X[3 * i + 2];
        L0[k] = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    }
}

/*
 * Dynamic relaxation of one RVE (O1-O10).
 *
 * X, is_bnd, fib: reference network.  L0: rest lengths (NULL: |X_j - X_i|).
 * F: 3x3 row-major.  c: damping constant.  x (3 n_nodes): output positions;
 * when o->init == OR_INIT_GIVEN it also holds the starting free positions
 * (boundary entries are overwritten by F Xm).  Outputs sigma[9], iteration
 * count, final R, final damping-force norm.  Returns the status code.
 */
int or_solve(int64_t n_nodes, int64_t n_fib, const double* X, const uint8_t* is_bnd,
             const int32_t* fib, const double* L0_in, double V0, const double* F, double c,
             const or_opts* o, double* x, double* sigma, int64_t* iters, double* R_out,
             double* D_out)
{
    for (int k = 0; k < 9; ++k) sigma[k] = NAN;
    *iters = 0;
    *R_out = NAN;
    *D_out = NAN;
    double J = det3(F);
    int finite = 1;
    for (int k = 0; k < 9; ++k) finite &= isfinite(F[k]);
    if (!finite || !(J > 0.0)) return OR_BAD_F;

    size_t nn = (size_t)n_nodes;
    double* L0 = malloc(sizeof(double) * (size_t)(n_fib > 0 ? n_fib : 1));
    double* M = calloc(nn ? nn : 1, sizeof(double));
    double* v = calloc(3 * nn + 1, sizeof(double));
    double* a = calloc(3 * nn + 1, sizeof(double));
    double* f = calloc(3 * nn + 1, sizeof(double));
    double* G = calloc(nn + 1, sizeof(double));

    if (L0_in) memcpy(L0, L0_in, sizeof(double) * (size_t)n_fib);
    else or_rest_lengths(n_fib, X, fib, L0);

    /* O4 lumped mass */
    for (int64_t k = 0; k < n_fib; ++k) {
        M[fib[2 * k]] += 0.5 * o->rhoA * L0[k];
        M[fib[2 * k + 1]] += 0.5 * o->rhoA * L0[k];
    }
    /* O1-O3 positions */
    for (int64_t p = 0; p < n_nodes; ++p) {
        double Xm[3] = {X[3 * p] - 0.5, X[3 * p + 1] - 0.5, X[3 * p + 2] - 0.5};
        if (is_bnd[p] || o->init == OR_INIT_AFFINE) {
            matvec3(F, Xm, &x[3 * p]);
        } else if (o->init == OR_INIT_REFERENCE) {
            x[3 * p] = Xm[0]; x[3 * p + 1] = Xm[1]; x[3 * p + 2] = Xm[2];
        }
    }

    /* initial force, acceleration and residual */
    or_forces(n_nodes, n_fib, x, fib, L0, o, f, G, NULL);
    if (o->mass == OR_MASS_SCALED)
        for (int64_t p = 0; p < n_nodes; ++p) M[p] = G[p] > 0.0 ? G[p] / 4.0 : 1.0;
    double R2 = 0.0, B2 = 0.0;
    for (int64_t p = 0; p < n_nodes; ++p) {
        double s = f[3 * p] * f[3 * p] + f[3 * p + 1] * f[3 * p + 1] + f[3 * p + 2] * f[3 * p + 2];
        if (is_bnd[p]) { B2 += s; continue; }
        R2 += s;
        for (int k = 0; k < 3; ++k) a[3 * p + k] = -f[3 * p + k] / M[p];
    }
    double R = sqrt(R2), D = 0.0;
    double tol = fmax(o->tol_abs, o->tol_rel * sqrt(B2));
    int64_t n = 0;
    int status = OR_CONVERGED;
    /* stagnation stop (O8): reference residual and the tests since R last
       fell below half of it */
    double Rref = R;
    int64_t stall = 0;

    while (!(R <= tol && D <= tol)) {
        if (!isfinite(R)) { status = OR_NONFINITE; break; }
        if (n > 0 && o->floor_tol_rel > 0.0) {
            double ftol = o->floor_tol_rel * sqrt(B2);
            if (R < 0.5 * Rref) {
                Rref = R;
                stall = 0;
            } else if (++stall >= o->stall_checks && R <= ftol && D <= ftol) {
                status = OR_STAGNATED;
                break;
            }
        }
        if (n >= o->n_max) { status = OR_MAXITER; break; }
        /* O6 time step from the current state */
        double gmax = 0.0;
        for (int64_t p = 0; p < n_nodes; ++p)
            if (!is_bnd[p] && G[p] / M[p] > gmax) gmax = G[p] / M[p];
        double dt = o->alpha * 2.0 / sqrt(gmax);
        /* half-step velocity and position update of the free nodes */
        for (int64_t p = 0; p < n_nodes; ++p) {
            if (is_bnd[p]) continue;
            for (int k = 0; k < 3; ++k) {
                v[3 * p + k] += 0.5 * dt * a[3 * p + k];
                x[3 * p + k] += dt * v[3 * p + k];
            }
        }
        or_forces(n_nodes, n_fib, x, fib, L0, o, f, G, NULL);
        /* damped acceleration, second half-step, residual and damping norm */
        R2 = 0.0; B2 = 0.0;
        double D2 = 0.0;
        for (int64_t p = 0; p < n_nodes; ++p) {
            double s = f[3 * p] * f[3 * p] + f[3 * p + 1] * f[3 * p + 1] + f[3 * p + 2] * f[3 * p + 2];
            if (is_bnd[p]) { B2 += s; continue; }
            R2 += s;
            for (int k = 0; k < 3; ++k) {
                a[3 * p + k] = -(f[3 * p + k] + c * M[p] * v[3 * p + k]) / M[p];
                v[3 * p + k] += 0.5 * dt * a[3 * p + k];
                double dk = c * M[p] * v[3 * p + k];
                D2 += dk * dk;
            }
        }
        R = sqrt(R2);
        D = sqrt(D2);
        tol = fmax(o->tol_abs, o->tol_rel * sqrt(B2));
        ++n;
    }
    if (status == OR_CONVERGED && !isfinite(R)) status = OR_NONFINITE;
    *iters = n;
    *R_out = R;
    *D_out = D;
    if (status != OR_NONFINITE) or_stress(n_nodes, x, f, is_bnd, F, V0, sigma);

    free(L0); free(M); free(v); free(a); free(f); free(G);
    return status;
}

/*
 * Dynamic relaxation with the alternatives the paper lists beside its
 * constant viscous damping (Section 3.2: kinetic damping, an automatically
 * updated damping coefficient, and the optional energy-balance check of
 * the two-step central difference, three whole-state reductions per step).
 *
 *   damping 0  viscous, constant c (the same iteration as or_solve);
 *   damping 1  kinetic: no viscous force; when the kinetic energy
 *              KE = 1/2 sum M |v|^2 at the full step has dropped below its
 *              value at the previous full step (a peak was passed), every
 *              velocity is set to zero and the acceleration to -f/M;
 *   damping 2  adaptive viscous: after each force evaluation the
 *              coefficient becomes c = 2 sqrt(u.K u / u.M u), the critical
 *              damping of the Rayleigh quotient of the displacement since
 *              the start, u = x - x_start, with K the tangent stiffness at
 *              the new positions (per fiber (k_t/L0) (n.du)^2 +
 *              (T/l) (|du|^2 - (n.du)^2), du the difference of u over the
 *              fiber); c = 0 when u.K u <= 0 or u = 0; the new c enters
 *              the damping force of the same step.
 *
 *   Energy balance (energy_check != 0): with the boundary fixed during the
 *   relaxation no external work is done, so the stored energy W, the
 *   kinetic energy KE and the work removed by damping Wd (viscous: the sum
 *   over steps of c M v^{n+1/2}.(x^{n+1} - x^n); kinetic: the kinetic
 *   energy dropped at each reset) satisfy W + KE + Wd = W(x_start).  A
 *   violation |W + KE + Wd - W0| > energy_tol * max(W0, W, KE, Wd) ends the
 *   relaxation with OR_ENERGY (an unstable or unphysical trajectory).
 *
 * Convergence as in or_solve with the damping-force norm D = c |M v|_2 (for
 * kinetic damping c is not applied as a force, only as the scale of this
 * velocity guard, so that the test is the viscous one).  Outputs as or_solve plus the final
 * coefficient (c_out; 0 for kinetic damping) and the final relative energy
 * balance |W + KE + Wd - W0| / max(W0, W, KE, Wd) (e_out; evaluated whether
 * or not the check is enabled).
 */
#define OR_ENERGY 7

int or_solve_variant(int64_t n_nodes, int64_t n_fib, const double* X, const uint8_t* is_bnd,
                     const int32_t* fib, double V0, const double* F, double c, const or_opts* o,
                     int32_t damping, int32_t energy_check, double energy_tol, double* x, double* sigma,
                     int64_t* iters, double* R_out, double* D_out, double* c_out, double* e_out)
{
    for (int k = 0; k < 9; ++k) sigma[k] = NAN;
    *iters = 0;
    *R_out = NAN;
    *D_out = NAN;
    *c_out = NAN;
    *e_out = NAN;
    double J = det3(F);
    int finite = 1;
    for (int k = 0; k < 9; ++k) finite &= isfinite(F[k]);
    if (!finite || !(J > 0.0)) return OR_BAD_F;

    size_t nn = (size_t)n_nodes;
    double* L0 = malloc(sizeof(double) * (size_t)(n_fib > 0 ? n_fib : 1));
    double* M = calloc(nn ? nn : 1, sizeof(double));
    double* v = calloc(3 * nn + 1, sizeof(double));
    double* a = calloc(3 * nn + 1, sizeof(double));
    double* f = calloc(3 * nn + 1, sizeof(double));
    double* x0 = calloc(3 * nn + 1, sizeof(double));
    double* G = calloc(nn + 1, sizeof(double));

    or_rest_lengths(n_fib, X, fib, L0);
    for (int64_t k = 0; k < n_fib; ++k) {
        M[fib[2 * k]] += 0.5 * o->rhoA * L0[k];
        M[fib[2 * k + 1]] += 0.5 * o->rhoA * L0[k];
    }
    for (int64_t p = 0; p < n_nodes; ++p) {
        double Xm[3] = {X[3 * p] - 0.5, X[3 * p + 1] - 0.5, X[3 * p + 2] - 0.5};
        if (is_bnd[p] || o->init == OR_INIT_AFFINE) {
            matvec3(F, Xm, &x[3 * p]);
        } else if (o->init == OR_INIT_REFERENCE) {
            x[3 * p] = Xm[0]; x[3 * p + 1] = Xm[1]; x[3 * p + 2] = Xm[2];
        }
    }
    memcpy(x0, x, sizeof(double) * 3 * nn);

    double W0 = 0.0, W = 0.0;
    or_forces(n_nodes, n_fib, x, fib, L0, o, f, G, &W0);
    W = W0;
    if (o->mass == OR_MASS_SCALED)
        for (int64_t p = 0; p < n_nodes; ++p) M[p] = G[p] > 0.0 ? G[p] / 4.0 : 1.0;
    double R2 = 0.0, B2 = 0.0;
    for (int64_t p = 0; p < n_nodes; ++p) {
        double s = f[3 * p] * f[3 * p] + f[3 * p + 1] * f[3 * p + 1] + f[3 * p + 2] * f[3 * p + 2];
        if (is_bnd[p]) { B2 += s; continue; }
        R2 += s;
        for (int k = 0; k < 3; ++k) a[3 * p + k] = -f[3 * p + k] / M[p];
    }
    double cc = damping == 1 ? 0.0 : c;
    double R = sqrt(R2), D = 0.0, KE = 0.0, KE_prev = 0.0, Wd = 0.0, ebal = 0.0;
    double tol = fmax(o->tol_abs, o->tol_rel * sqrt(B2));
    int64_t n = 0;
    int status = OR_CONVERGED;

    while (!(R <= tol && D <= tol)) {
        if (!isfinite(R)) { status = OR_NONFINITE; break; }
        if (n >= o->n_max) { status = OR_MAXITER; break; }
        double gmax = 0.0;
        for (int64_t p = 0; p < n_nodes; ++p)
            if (!is_bnd[p] && G[p] / M[p] > gmax) gmax = G[p] / M[p];
        double dt = o->alpha * 2.0 / sqrt(gmax);
        for (int64_t p = 0; p < n_nodes; ++p) {
            if (is_bnd[p]) continue;
            for (int k = 0; k < 3; ++k) {
                v[3 * p + k] += 0.5 * dt * a[3 * p + k];
                x[3 * p + k] += dt * v[3 * p + k];
            }
        }
        or_forces(n_nodes, n_fib, x, fib, L0, o, f, G, &W);
        if (damping == 2) {
            double num = 0.0, den = 0.0;
            for (int64_t k = 0; k < n_fib; ++k) {
                int32_t i = fib[2 * k], j = fib[2 * k + 1];
                double d[3], du[3];
                for (int q = 0; q < 3; ++q) {
                    d[q] = x[3 * j + q] - x[3 * i + q];
                    du[q] = (x[3 * j + q] - x0[3 * j + q]) - (x[3 * i + q] - x0[3 * i + q]);
                }
                double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                double T, kt;
                fiber_law(o, l / L0[k] - 1.0, &T, &kt);
                double nd = (d[0] * du[0] + d[1] * du[1] + d[2] * du[2]) / l;
                double du2 = du[0] * du[0] + du[1] * du[1] + du[2] * du[2];
                num += kt / L0[k] * nd * nd + T / l * (du2 - nd * nd);
            }
            for (int64_t p = 0; p < n_nodes; ++p) {
                if (is_bnd[p]) continue;
                for (int q = 0; q < 3; ++q) {
                    double u = x[3 * p + q] - x0[3 * p + q];
                    den += M[p] * u * u;
                }
            }
            cc = (num > 0.0 && den > 0.0) ? 2.0 * sqrt(num / den) : 0.0;
        }
        /* work of the damping force over the step, with the half-step velocity */
        if (damping != 1)
            for (int64_t p = 0; p < n_nodes; ++p) {
                if (is_bnd[p]) continue;
                for (int k = 0; k < 3; ++k) Wd += cc * M[p] * v[3 * p + k] * v[3 * p + k] * dt;
            }
        R2 = 0.0; B2 = 0.0;
        double MV2 = 0.0;
        KE = 0.0;
        for (int64_t p = 0; p < n_nodes; ++p) {
            double s = f[3 * p] * f[3 * p] + f[3 * p + 1] * f[3 * p + 1] + f[3 * p + 2] * f[3 * p + 2];
            if (is_bnd[p]) { B2 += s; continue; }
            R2 += s;
            for (int k = 0; k < 3; ++k) {
                a[3 * p + k] = -(f[3 * p + k] + cc * M[p] * v[3 * p + k]) / M[p];
                v[3 * p + k] += 0.5 * dt * a[3 * p + k];
                double mv = M[p] * v[3 * p + k];
                MV2 += mv * mv;
                KE += 0.5 * M[p] * v[3 * p + k] * v[3 * p + k];
            }
        }
        if (damping == 1) {
            if (KE < KE_prev) {
                Wd += KE;
                KE = 0.0;
                MV2 = 0.0;
                for (int64_t p = 0; p < n_nodes; ++p) {
                    if (is_bnd[p]) continue;
                    for (int k = 0; k < 3; ++k) {
                        v[3 * p + k] = 0.0;
                        a[3 * p + k] = -f[3 * p + k] / M[p];
                    }
                }
            }
            KE_prev = KE;
        }
        double scale = fmax(fmax(W0, W), fmax(KE, Wd));
        ebal = scale > 0.0 ? fabs(W + KE + Wd - W0) / scale : 0.0;
        R = sqrt(R2);
        D = (damping == 1 ? c : cc) * sqrt(MV2);
        tol = fmax(o->tol_abs, o->tol_rel * sqrt(B2));
        ++n;
        if (energy_check && ebal > energy_tol) { status = OR_ENERGY; break; }
    }
    if (status == OR_CONVERGED && !isfinite(R)) status = OR_NONFINITE;
    *iters = n;
    *R_out = R;
    *D_out = D;
    *c_out = cc;
    *e_out = ebal;
    if (status != OR_NONFINITE) or_stress(n_nodes, x, f, is_bnd, F, V0, sigma);

    free(L0); free(M); free(v); free(a); free(f); free(x0); free(G);
    return status;
}

/* ------------------------------------------------------------ batch driver */
typedef struct {
    int64_t n_rve;
    const int64_t *node_off, *fib_off;
    const double* X;
    const uint8_t* is_bnd;
    const int32_t* fib;
    const double* V0;   /* nullable: 1 */
    const double* F;
    const double* c;
    const or_opts* o;
    double *x, *sigma, *R, *D;
    int64_t* iters;
    int32_t* status;
    int64_t next;
    pthread_mutex_t mu;
} batch_job;

static void* batch_worker(void* arg)
{
    batch_job* b = (batch_job*)arg;
    for (;;) {
        pthread_mutex_lock(&b->mu);
        int64_t r = b->next++;
        pthread_mutex_unlock(&b->mu);
        if (r >= b->n_rve) break;
        int64_t n0 = b->node_off[r], n1 = b->node_off[r + 1];
        int64_t f0 = b->fib_off[r], f1 = b->fib_off[r + 1];
        double* xr = b->x + 3 * n0;
        b->status[r] = or_solve(n1 - n0, f1 - f0, b->X + 3 * n0, b->is_bnd + n0, b->fib + 2 * f0, NULL,
                                b->V0 ? b->V0[r] : 1.0, b->F + 9 * r, b->c[r], b->o, xr,
                                b->sigma + 9 * r, b->iters + r, b->R + r, b->D + r);
    }
    return NULL;
}

/* Solve every RVE of a packed batch on n_threads POSIX threads. */
void or_solve_batch(int64_t n_rve, const int64_t* node_off, const int64_t* fib_off, const double* X,
                    const uint8_t* is_bnd, const int32_t* fib, const double* V0, const double* F,
                    const double* c, const or_opts* o, int32_t n_threads, double* x, double* sigma,
                    int64_t* iters, double* R, double* D, int32_t* status)
{
    batch_job b = {n_rve, node_off, fib_off, X, is_bnd, fib, V0, F, c, o, x, sigma, R, D, iters, status, 0,
                   PTHREAD_MUTEX_INITIALIZER};
    if (n_threads < 1) n_threads = 1;
    pthread_t* th = malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, batch_worker, &b);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    free(th);
}
