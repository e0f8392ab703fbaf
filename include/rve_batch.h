/*
 * rve_batch.h - C ABI of the MI355X batched fiber-network RVE solver.
 *
 * The library is the microscale side of an FE^2 computation (paper:
 * Section 4, "batched" microscale routines that take a set of deformation
 * states and return stresses and material stiffnesses for the whole set at
 * once; Section 4.3, one independent sub-problem per RVE).  Each RVE is a
 * truss network in the unit cube; its boundary nodes follow the affine map
 * x = F Xm (Section 2, affine boundary condition), its free nodes are
 * relaxed to static equilibrium by damped explicit dynamic relaxation
 * (Section 3.2, Algorithm "Dynamic Relaxation"), and the homogenized Cauchy
 * stress is the boundary-traction integral sigma_ij = 1/V sum_b f_b,i x_b,j
 * (Section 2, stress as the surface integral of traction times position).
 *
 * Conventions shared by every entry point
 *  - Return value: RVE_OK (0) on success, a negative RVE_E* code otherwise.
 *    No entry point throws, aborts or exits; rve_last_error() returns a
 *    thread-local message for the last failure on the calling thread.
 *  - Matrices are row-major doubles: F[r][i][j] = F_ij of RVE r, sigma the
 *    same, dsdF[r][3i+j][3k+l] = d sigma_ij / d F_kl.
 *  - ptr_kind says whether the caller's output/input arrays live in host
 *    memory (RVE_PTR_HOST: the call is synchronous) or device memory
 *    (RVE_PTR_DEVICE: the call is stream-ordered on opts.stream and returns
 *    before the work finishes).
 *  - A batch object is not thread-safe: one call at a time per object.
 *    Distinct objects may be used from distinct threads.
 *  - Per-RVE outcomes are written to status[r] (RVE_ST_*); the outputs of an
 *    RVE that did not converge hold the last state's values (MAXITER,
 *    STAGNATED, ENERGY) or NaN (NONFINITE, BAD_F).
 */
#ifndef RVE_BATCH_H
#define RVE_BATCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RVE_API_VERSION 1

/* return codes */
#define RVE_OK 0
#define RVE_EINVAL (-22)       /* malformed argument, topology or option */
#define RVE_ENOMEM (-12)       /* host or device allocation failed */
#define RVE_EDEVICE (-5)       /* HIP runtime error or no usable gfx950 device */
#define RVE_ESTATE (-3)        /* call order: e.g. tangent before any solve */
#define RVE_EWORKSPACE (-28)   /* workspace: a caller-bound workspace that is too
                                  small, misaligned or not device memory, or a
                                  request beyond a fixed workspace's limit */

/* per-RVE status codes */
#define RVE_ST_CONVERGED 0     /* R <= tol and damping-force norm <= tol */
#define RVE_ST_MAXITER 1       /* n_max iterations reached first */
#define RVE_ST_NONFINITE 2     /* the relaxation produced Inf/NaN */
#define RVE_ST_BAD_F 3         /* F non-finite or det F <= 0: RVE skipped */
#define RVE_ST_NO_STATE 4      /* tangent: RVE has no converged state */
#define RVE_ST_CG_MAXITER 5    /* tangent: CG stopped at its iteration cap */
#define RVE_ST_CG_INDEFINITE 6 /* tangent: K_ff not positive (unstable state) */
#define RVE_ST_ENERGY 7        /* energy-balance check failed (opts.energy_check) */
#define RVE_ST_STAGNATED 8     /* stopped at the precision floor (opts.floor_tol_rel) */

/* options */
#define RVE_FP64 0             /* all arithmetic in double */
#define RVE_MIXED 1            /* fibers and state in float; residual, damping
                                  test, time-step scalar and stress in double */
#define RVE_LAW_LINEAR 0       /* T = EA eps */
#define RVE_LAW_EXP 1          /* T = EA (exp(B eps) - 1)/B, eps >= 0; EA eps below */
#define RVE_MASS_LUMPED 0      /* M_a = rhoA/2 sum L0 over fibers at a */
#define RVE_MASS_SCALED 1      /* M_a = G_a(x0)/4, Gershgorin sum at the start */
#define RVE_INIT_AFFINE 0      /* free nodes start at F Xm */
#define RVE_INIT_REFERENCE 1   /* free nodes start at their reference position Xm
                                  (free displacements zero, as Algorithm "Dynamic
                                  Relaxation" prints it for an increment from the
                                  undeformed state); the boundary is at F Xm */
#define RVE_INIT_WARM 2        /* free nodes start at F Xm + h, h = fluctuation
                                  left by the previous solve of this batch */
#define RVE_ENGINE_AUTO 0      /* register-resident persistent kernel where an
                                  RVE fits; beyond it the incidence kernel
                                  (RVE_MIXED, free nodes of degree <= 16),
                                  else the streamed persistent kernel */
#define RVE_ENGINE_STREAMED 1  /* persistent kernel, state in global memory */
#define RVE_ENGINE_NAIVE 2     /* one RVE at a time, one launch per step of
                                  every iteration, atomics, FP64 only */
#define RVE_ENGINE_TEAM 3      /* as AUTO, but RVEs no resident build holds run
                                  on the team engine (k workgroups per RVE)
                                  wherever a partition fits, else as AUTO;
                                  AUTO runs them on the team engine only where
                                  rve_batch_autotune measured it faster than
                                  the streamed kernel */
#define RVE_ENGINE_INCIDENCE 4 /* every RVE within the incidence kernel's
                                  limits runs on it (RVE_MIXED only; free
                                  nodes of degree <= 16): one record per
                                  node-fiber incidence read from global
                                  memory each iteration, node state in
                                  registers and positions in LDS up to 12288
                                  free nodes, node state in global arrays
                                  above (global mode); the rest as AUTO.  Its
                                  tables (about 56 bytes per fiber) are built
                                  at rve_batch_create: for every RVE that
                                  fits when the batch is created with this
                                  engine, else only for the RVEs no resident
                                  build holds */
#define RVE_DAMP_VISCOUS 0     /* constant mass-proportional damping c M v */
#define RVE_DAMP_KINETIC 1     /* kinetic damping: v = 0 at kinetic-energy peaks */
#define RVE_DAMP_ADAPTIVE 2    /* c re-estimated each step (Rayleigh quotient) */

/* opts.work_order: the order in which a persistent launch takes its RVEs */
#define RVE_ORDER_AUTO 0       /* library choice per engine (below) */
#define RVE_ORDER_HOST 1       /* most fibers first, every solve */
#define RVE_ORDER_COST 2       /* after a first solve: longest previous solve first */
#define RVE_PTR_HOST 0
#define RVE_PTR_DEVICE 1

typedef struct rve_batch rve_batch;

/*
 * Network description: a ragged batch in row-offset + value layout.
 * All pointers are host pointers; create() copies what it needs and the
 * caller keeps ownership.
 *   node_off[n_rve+1], fib_off[n_rve+1]: offsets of each RVE's nodes/fibers.
 *   X[node_off[n_rve]][3]: reference coordinates in the unit cube [0,1]^3
 *     (the RVE centre 0.5,0.5,0.5 is the macroscale material point).
 *   is_bnd[node_off[n_rve]]: 1 for a boundary node (prescribed x = F Xm).
 *   fib[fib_off[n_rve]][2]: fiber end nodes as ids local to the RVE.
 *   V0[n_rve]: reference RVE volume (NULL: 1, the unit cube).
 *   L0[fib_off[n_rve]]: rest length of every fiber (NULL: the reference
 *     chord |X_j - X_i|, a network stress-free at F = I; given values make
 *     a pre-stressed network).  Must be positive and finite.
 * Rejected with RVE_EINVAL: ids out of range, a fiber joining a node to
 * itself, a zero-length fiber, an RVE without a boundary node, an RVE with
 * 65535 nodes or more, non-finite coordinates.
 */
typedef struct {
    int64_t n_rve;
    const int64_t* node_off;
    const int64_t* fib_off;
    const double* X;
    const uint8_t* is_bnd;
    const int32_t* fib;
    const double* V0;
    const double* L0;
} rve_net_desc;

/*
 * Solver options (copied at create; change later with rve_batch_set_opts).
 *   EA, B: fiber law constants.  rhoA: lumped-mass density (RVE_MASS_LUMPED).
 *   alpha: time-step safety factor, dt = alpha * 2 / sqrt(max_a G_a / M_a)
 *     with G_a = 2 sum_{fibers at a} max(k_t/L0, |T|/l).
 *   c: mass-proportional damping constant (c_per_rve, if non-NULL, is a host
 *     array of n_rve values that overrides it; copied).
 *   Convergence: R = |f_free|_2 <= tol and c |M v|_2 <= tol with
 *     tol = max(tol_abs, tol_rel |f_bnd|_2), tested every check_every
 *     iterations (>= 1); n_max caps the iterations.
 *   engine: RVE_ENGINE_*.  threads_per_rve: 0 = automatic (default or
 *     autotuned variant per size tier), else 256/512/768/1024: only
 *     resident builds of that workgroup size; RVEs none of them holds run
 *     on the streamed kernel (256 threads when 256 is asked for, else 1024
 *     where that build uses no private memory).  A kernel build that uses
 *     private (scratch) memory is never launched.
 *   cg_tol, cg_max_iter: conjugate-gradient controls of rve_batch_tangent and
 *     rve_batch_vjp.
 *   stream: hipStream_t for every launch and copy (NULL: the null stream).
 *   damping, energy_check, energy_tol: the alternatives the paper lists
 *     beside constant viscous damping (Section 3.2).  RVE_DAMP_KINETIC: no
 *     viscous force; whenever the kinetic energy 1/2 sum M |v|^2 at a full
 *     step is below its value at the previous full step, every velocity is
 *     set to zero (c is applied as no force, only as the scale of the
 *     damping-force test c |M v|_2).  RVE_DAMP_ADAPTIVE: after each force
 *     evaluation c = 2 sqrt(u.K u / u.M u), the critical damping of the Rayleigh
 *     quotient of u, the displacement since the start of the solve, with K
 *     the tangent stiffness at the current positions (0 when u.K u <= 0);
 *     c of the opts is only the value before the first step.
 *     energy_check = 1: after every step the stored energy W, kinetic energy
 *     KE and the work Wd removed by damping must satisfy
 *     |W + KE + Wd - W_start| <= energy_tol max(W_start, W, KE, Wd), else the
 *     RVE stops with RVE_ST_ENERGY (an unstable trajectory).  Kinetic
 *     damping alone runs on the ordinary engines (kinetic builds of the
 *     resident and streamed kernels, either precision; the kinetic-energy
 *     peak is tested every iteration).  Adaptive damping or the energy
 *     check run every RVE on an FP64 engine with one workgroup per RVE and
 *     a convergence test every iteration (precision must be RVE_FP64);
 *     check_every and threads_per_rve do not apply there.  None of them
 *     with RVE_ENGINE_NAIVE.
 *   floor_tol_rel, stall_checks: stagnation stop for a tol below what the
 *     arithmetic can reach (float positions put a floor under R, about
 *     1e-5 |f_bnd|_2 on Voronoi networks in RVE_MIXED).  With
 *     floor_tol_rel > 0 (0 = off, the default) a convergence test that
 *     does not converge also compares R with a reference value: R of the
 *     start, replaced by R whenever R falls below half of it.  After
 *     stall_checks (>= 1) consecutive tests without such a halving, with R
 *     and c |M v|_2 both <= floor_tol_rel |f_bnd|_2, the RVE stops with
 *     RVE_ST_STAGNATED; its stress is evaluated as for a converged RVE.
 *     The tangent and VJP treat it as an RVE without a converged state.
 *     Constant viscous damping on the resident and streamed engines only
 *     (RVE_EINVAL with kinetic or adaptive damping, the energy check or
 *     RVE_ENGINE_NAIVE).
 *   work_order: the order in which the workgroups of a persistent resident
 *     or streamed launch take its RVEs.  RVE_ORDER_HOST: most fibers first.
 *     RVE_ORDER_COST: from the second solve of the batch on, descending
 *     cost of the previous solve (iterations x fibers, longest processing
 *     time first; ties and the first solve in host order).  RVE_ORDER_AUTO:
 *     cost order for resident and incidence launches, host order for
 *     streamed and global-mode incidence ones.  Team launches keep host
 *     order.  Results do not depend on the order.
 */
typedef struct {
    int32_t precision;
    int32_t law;
    int32_t mass;
    int32_t init;
    double EA, B, rhoA;
    double alpha;
    double c;
    const double* c_per_rve;
    double tol_abs, tol_rel;
    int64_t n_max;
    int32_t check_every;
    int32_t engine;
    int32_t threads_per_rve;
    double cg_tol;          /* tangent/vjp CG: stop at |r_k| <= cg_tol |b_k| */
    int64_t cg_max_iter;    /* tangent/vjp CG iteration cap per right-hand side (0: 2 x free DOFs + 100) */
    void* stream;
    int32_t damping;        /* RVE_DAMP_* */
    int32_t energy_check;   /* 0 or 1 */
    double energy_tol;      /* relative energy-balance tolerance (> 0) */
    double floor_tol_rel;   /* stagnation stop (0: off) */
    int32_t stall_checks;   /* tests without R halving before the stop (>= 1) */
    int32_t tangent_rhs;    /* right-hand sides per tangent task: 0 library choice (one per task,
                               the faster on MI355X), 1 one per task, 3 three per task where a
                               blocked build holds the RVE (at most 2048 free nodes) */
    int32_t work_order;     /* RVE_ORDER_*: order of the RVEs in a resident or streamed launch */
} rve_opts;

/* Optional per-RVE diagnostics of a solve (each pointer may be NULL; same
 * ptr_kind as the solve call). */
typedef struct {
    int64_t* iters;   /* iterations taken */
    double* R;        /* final |f_free|_2 */
    double* D;        /* final damping-force norm c |M v|_2 */
    double* Fb;       /* final |f_bnd|_2 (reaction scale of tol_rel) */
} rve_stats;

int rve_version(void);
const char* rve_last_error(void);

/* Fill *o with defaults: FP64, linear law, EA 1, B 10, rhoA 1, alpha 0.9,
 * c 2, tol_abs 1e-10, tol_rel 0, n_max 1e6, check_every 1, auto engine,
 * cg_tol 1e-6, cg_max_iter 0, viscous damping, no energy check,
 * energy_tol 0.05. */
void rve_default_opts(rve_opts* o);

/*
 * Build a batch: validate and copy the networks, reorder each RVE's nodes
 * (free nodes first in a locality order, boundary nodes last), compute rest
 * lengths and lumped masses, build node->fiber incidence, pick a kernel
 * variant per RVE, and upload everything to the current HIP device
 * (Algorithm "Dynamic Relaxation": connectivity and mass prepared on the
 * host once and transferred to the device).  *out is NULL on failure.
 */
int rve_batch_create(const rve_net_desc* net, const rve_opts* opts, rve_batch** out);

/* Replace the options of an existing batch (same validation as create). */
int rve_batch_set_opts(rve_batch* b, const rve_opts* opts);

/* Replace only the stream of the batch (hipStream_t; NULL = null stream). */
int rve_batch_set_stream(rve_batch* b, void* stream);

/*
 * Kernel timing: after rve_batch_profile(b, 1), every solve records HIP
 * events around each relaxation launch (on the stream that launch runs on:
 * the batch's stream or, for concurrent launch groups, an auxiliary stream
 * joined back to it) and around the stress launch.  rve_batch_kernel_ms then
 * returns, for the last solve, the span of the relaxation from the earliest
 * launch's start to the join of all launches (*relax_ms) and the duration of
 * the stress kernel (*stress_ms) in milliseconds (it synchronises the
 * stream); rve_batch_groups gives each launch's own duration.
 */
int rve_batch_profile(rve_batch* b, int enable);
int rve_batch_kernel_ms(rve_batch* b, double* relax_ms, double* stress_ms);

/*
 * Kernel groups of the last solve: group_of_rve[R] receives the launch group
 * of every RVE, variant[g] its resident variant index (-1 streamed, -1 - k
 * a team of k workgroups per RVE, -100 the incidence kernel, -101 its
 * global mode) and, if
 * the solve was profiled, ms[g] the duration of that group's relaxation
 * launch (NaN otherwise).  Arrays are host memory of max_groups entries;
 * *n_groups receives the number of groups.
 */
int rve_batch_groups(rve_batch* b, int32_t* group_of_rve, int32_t* variant, double* ms, int32_t max_groups,
                     int32_t* n_groups);

/*
 * Autotuner: for every size tier of the batch (RVEs grouped by the smallest
 * register-resident variant that holds them), run each eligible kernel
 * variant (threads per RVE x fiber/node slots per thread, and the streamed
 * kernel) on a sample of that tier's largest RVEs for n_iter relaxation
 * iterations under F (host or device pointer per ptr_kind), time it with HIP
 * events, and keep the fastest per fiber evaluation for the batch's current
 * precision; for the RVEs beyond every resident build that the incidence
 * kernel does not take, the team engine of each team size k against the
 * streamed kernel, kept only where it takes less CU-time (k times its time
 * below the streamed kernel's: a team holds k CUs per RVE, and team
 * launches run alone, before the other groups).  Later solves use the
 * choice.  The trial runs overwrite the state of the last solve.
 */
int rve_batch_autotune(rve_batch* b, const double* F, int32_t ptr_kind, int32_t n_iter);

/*
 * After a solve that used adaptive damping or the energy check: the
 * damping coefficient at the end of each RVE's relaxation (c_final[n_rve];
 * 0 for kinetic damping, the constant c for viscous damping) and the final
 * relative energy balance |W + KE + Wd - W_start| / max(W_start, W, KE, Wd)
 * (energy[n_rve]); either pointer may be NULL.  RVE_ESTATE otherwise.
 */
int rve_batch_damping_stats(rve_batch* b, double* c_final, double* energy, int32_t ptr_kind);

/* Describe the kernel groups of the next solve ("variant:count;...") into
 * buf (NUL-terminated, truncated to n bytes). */
int rve_batch_describe(const rve_batch* b, char* buf, size_t n);

/*
 * Caller-owned workspace.  rve_batch_workspace_size reports the bytes of
 * device memory that cover every work area the batch would otherwise
 * allocate on demand: the streamed relaxation workspace (sized for FP64, so
 * any later precision or engine fits), the tangent/VJP arena (per-fiber
 * operators, incidence records, preconditioner, task tables, outputs) and
 * solver slots (the larger of tangent and VJP, both engines), the
 * orientation outputs and the state-export map.  rve_batch_bind_workspace
 * makes the batch carve those areas from [ptr, ptr + bytes): ptr must be
 * device memory of the batch's device, 256-byte aligned, and bytes at least
 * the reported size (RVE_EINVAL otherwise).  The caller keeps ownership
 * (e.g. a torch tensor) and must keep the memory alive until the batch is
 * destroyed or another workspace (or NULL) is bound.  Binding waits for the
 * batch's stream, releases the areas the library had allocated, and
 * discards what was built in them: the next tangent or VJP call rebuilds its
 * tables, and rve_batch_tangent_iters reports RVE_ESTATE until then.  With
 * a workspace bound, solve, tangent, vjp, orientation and state export or
 * import allocate no device memory.  Binding NULL returns to library-owned
 * areas.  Not covered: the network and state arrays allocated by create,
 * the probe batch of rve_batch_fd_tangent and the autotuner's task list.
 */
int rve_batch_workspace_size(const rve_batch* b, size_t* bytes);
int rve_batch_bind_workspace(rve_batch* b, void* ptr, size_t bytes);

/* Number of RVEs, nodes and fibers of the batch. */
int rve_batch_sizes(const rve_batch* b, int64_t* n_rve, int64_t* n_nodes, int64_t* n_fib);

/*
 * Relax every RVE under its F and return the homogenized Cauchy stress.
 *   F[n_rve][3][3] (input), sigma[n_rve][3][3] (output), status[n_rve].
 *   sigma_ij = 1/(det F V0) sum_b f_b,i x_b,j, f_b the internal force at
 *   boundary node b (its reaction), x_b = F Xm_b.
 * The converged fluctuation state stays on the device for rve_batch_tangent,
 * rve_batch_vjp, rve_batch_positions and warm starts.
 * Scheduling: the RVEs of a launch group are taken most-fibers-first on the
 * batch's first solve and, after it, in decreasing order of the previous
 * solve's iterations times fibers (a device-side sort on the batch's
 * stream); every RVE's arithmetic and results are independent of the order.
 */
int rve_batch_solve(rve_batch* b, const double* F, double* sigma, int32_t* status,
                    rve_stats* stats, int32_t ptr_kind);

/*
 * Material tangent dsigma/dF at the state left by the last solve, by an
 * adjoint (the paper obtains the same linearisation by finite differences of
 * extra relaxations, Section 3.2): for each of the 9 directions E = e_k e_l
 * the free nodes follow K_ff dx_f = -K_fb (E Xm)_b, the reactions change by
 * df_b = (K dx)_b, and dsigma = (sum_b df_b x_b^T + f_b (E Xm_b)^T)/(J V0)
 * - sigma (F^-1)_lk.  K_ff is applied matrix-free (per-fiber Hessian
 * blocks); each right-hand side is an independent block-Jacobi
 * preconditioned CG with FP32 products inside FP64 iterative refinement,
 * stopped at |r| <= cg_tol |b| (FP64 residual).  With opts.tangent_rhs 3
 * the three right-hand sides of one k (columns 3k, 3k+1, 3k+2) of an RVE of
 * at most 2048 free nodes share one workgroup, each record read and each
 * reduction; every column still follows its own CG, and the results agree
 * with one task per right-hand side to rounding.
 * dsdF[n_rve][9][9] (row 3i+j = sigma_ij, column 3k+l = F_kl); status per
 * RVE: 0, RVE_ST_NO_STATE if the solve did not converge (outputs NaN),
 * RVE_ST_CG_MAXITER, RVE_ST_CG_INDEFINITE (p.Kp <= 0 met: K_ff not
 * positive definite at this state).  The first tangent or VJP call on a
 * batch allocates its workspace, so it cannot be captured in a graph; later
 * calls allocate only when the task grid grows.
 */
int rve_batch_tangent(rve_batch* b, double* dsdF, int32_t* status, int32_t ptr_kind);

/*
 * Vector-Jacobian product of the last solve: gF_kl = sum_ij g_ij dsigma_ij/dF_kl
 * with one adjoint CG per RVE.  gsigma[n_rve][9] in, gF[n_rve][9] out.
 */
int rve_batch_vjp(rve_batch* b, const double* gsigma, double* gF, int32_t* status, int32_t ptr_kind);

/*
 * The paper's material tangent by finite differences (Section 3.2, material
 * stiffness), at the state of the last solve: with F = R U (polar
 * decomposition), six probe relaxations under U + h T_c (T_c the six
 * probing directions the paper prints, in Mandel form), each warm-started
 * from the base state rotated back by R^T, give forward differences
 * [P] = (Pi(U + h T_c) - Pi(F)) / h of the second Piola-Kirchhoff stress
 * Pi = J F^-1 sigma F^-T; then [A] = [P] ([M][T])^-1 with [M] = [dE/dU]
 * (A = dPi/dE) and C = F F A F F / J (push-forward, the updated-Lagrangian
 * spatial tangent).  Mandel order 11, 22, 33, 23, 13, 12 with sqrt(2) on
 * shear components.  C[n_rve][36] and A[n_rve][36] (A may be NULL) are
 * row-major 6x6 Mandel matrices; status per RVE: 0, RVE_ST_NO_STATE when
 * the base solve did not converge, else the worst probe status (outputs
 * NaN when not 0).  h > 0 (e.g. 1e-4).  The first call builds an internal
 * batch of six copies of every RVE (six times the device memory of the
 * batch); every call runs one batched solve of it.  Host pointers or device
 * pointers per ptr_kind; the call returns after the outputs are written.
 */
int rve_batch_fd_tangent(rve_batch* b, double h, double* C, double* A, int32_t* status, int32_t ptr_kind);

/*
 * Fiber orientation at the state of the last solve (Section 6, degree of
 * alignment; Section 4, orientation data sent to the macroscale): per RVE
 * the orientation tensor omega_ab = <n_a n_b> (row-major 3x3, symmetric,
 * trace 1) and the degree of alignment p2 = <(3 (n.e)^2 - 1)/2> in
 * [-1/2, 1], averages over the RVE's fibers of the unit current direction n
 * of each fiber; e (host pointer, 3 doubles, normalised here) is the
 * reference direction, typically the loading direction.  omega[n_rve][9] and
 * p2[n_rve] follow ptr_kind.  RVEs whose solve ended non-finite or with a bad
 * F, and RVEs without fibers, get NaN.  RVE_EINVAL for a zero or non-finite
 * e, RVE_ESTATE before the first solve.
 */
int rve_batch_orientation(rve_batch* b, const double* e, double* omega, double* p2, int32_t ptr_kind);

/*
 * Inner CG iterations of the last rve_batch_tangent or rve_batch_vjp call,
 * summed over each RVE's right-hand sides: iters[n_rve].  RVE_ESTATE before
 * the first such call.
 */
int rve_batch_tangent_iters(rve_batch* b, int64_t* iters, int32_t ptr_kind);

/*
 * State export and import (checkpoint and restart; moving RVE states between
 * batches built from the same networks): the microscale state of an
 * integration point is its converged fluctuation, from which the next
 * increment starts (Algorithm "Dynamic Relaxation": free displacements of
 * an increment start from the last state; Algorithm 1: one RVE state per
 * macroscale integration point).
 *   F[n_rve][9]: F of the last solve (or import).
 *   h[n_nodes][3]: fluctuation x - F Xm of every node, in the caller's node
 *     numbering of create() (node_off layout); rows of boundary nodes are 0
 *     on export and ignored on import.
 *   status[n_rve]: RVE_ST_* of the last solve.
 * export writes them (RVE_ESTATE before any solve or import).  import
 * replaces the batch's state with them: statuses other than 0..3 and
 * RVE_ST_STAGNATED become RVE_ST_NONFINITE, a non-finite F or det F <= 0 gives RVE_ST_BAD_F; the
 * stress is re-evaluated from the imported state (the stress kernel of
 * rve_batch_solve, FP64) and written to sigma[n_rve][9] unless sigma is
 * NULL; the stored diagnostics become iterations 0 and NaN norms.  Afterwards the batch behaves as after a solve that ended in
 * that state: rve_batch_tangent, rve_batch_vjp, rve_batch_fd_tangent,
 * rve_batch_orientation, rve_batch_positions and RVE_INIT_WARM solves use
 * it.  The caller vouches that an imported "converged" state is one (an
 * exported state is).  Host pointers (synchronous) or device pointers
 * (stream-ordered; the first device-pointer call uploads a 4-byte-per-node
 * map and synchronises).  RVE_EINVAL for batches of 2^31 or more free nodes.
 */
int rve_batch_export_state(rve_batch* b, double* F, double* h, int32_t* status, int32_t ptr_kind);
int rve_batch_import_state(rve_batch* b, const double* F, const double* h, const int32_t* status,
                           double* sigma, int32_t ptr_kind);

/* Positions x[n_nodes_r][3] of RVE r after the last solve, in the caller's
 * original node order (host pointer; synchronous). */
int rve_batch_positions(rve_batch* b, int64_t r, double* x);

/*
 * Team engine (RVEs too large for one CU run on k workgroups that exchange
 * partition-boundary state through global memory once per iteration and
 * meet at a barrier): the number of polls a workgroup makes at a team
 * barrier before it gives up (default 2^24, about a second).  A launch whose
 * team gave up leaves its unfinished RVEs with status RVE_ST_NONFINITE and
 * NaN stress, and a host-pointer solve returns RVE_EDEVICE.  Mainly for
 * tests of that path (a limit of 1 poll forces it); polls >= 1.
 */
int rve_batch_team_spin_limit(rve_batch* b, int64_t polls);

/*
 * Generation of the batch's state: a counter that every successful
 * rve_batch_solve, rve_batch_import_state and rve_batch_set_opts increments.
 * A caller that computes a VJP or tangent for a state it solved earlier (an
 * autograd backward pass) records the generation after its solve and
 * compares it before the VJP: a different value means the state or the
 * options changed in between.
 */
int rve_batch_generation(const rve_batch* b, uint64_t* gen);

/*
 * Host replay of the kernels' index arithmetic (no device needed): packs the
 * networks as rve_batch_create does and, for every RVE and every
 * register-resident kernel build whose slots hold it, bounds every index the
 * build forms (packed fiber ends against the LDS position array, incidence
 * codes and overflow reads against the LDS force array, the code's end sign,
 * LDS bytes against 160 KB), the streamed engine's workspace offsets, the
 * team engine's partition and halo tables for the RVEs it would take, the
 * incidence engine's rank permutation, rounds and records (each record's
 * fiber, orientation and other end), and the packing's incidence lists.
 * precision: RVE_FP64 or RVE_MIXED (LDS layout).
 * plant: 0; 1 makes the replay assume one LDS position entry fewer, 2
 * corrupts the other end of one incidence record (deliberate mistakes that
 * the replay must report; tests only).
 * RVE_OK, or RVE_EINVAL with the first violation in rve_last_error().
 */
int rve_check_indexing(const rve_net_desc* net, int32_t precision, int32_t plant);

/*
 * Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same launches and results as rve_batch_solve (resident,
 * team and streamed engines, constant viscous or kinetic damping, affine or
 * warm start), but the work areas those launches need -- the launch work
 * counters, the team engine's exchange buffers, partials and barriers, and
 * the streamed engine's per-fiber and per-node workspace -- are carved from
 * a fixed device array of 256 MiB that the library holds on each device
 * until the process ends, instead of being allocated.  The call itself
 * makes no device allocation (the array is located once per device by
 * rve_batch_create).  F[n_rve][9] in, sigma[n_rve][9] and status[n_rve] out
 * (host: synchronous; device: stream-ordered).  RVE_EWORKSPACE when the
 * batch's work areas exceed the array; RVE_EINVAL for the naive engine,
 * adaptive damping, the energy check or the reference start.  Every call on
 * one device shares that device's array: calls that overlap in time on one
 * device (other streams, other threads, other batches) race and must be
 * serialised by the caller.  No per-RVE diagnostics and no profiling.
 */
int rve_batch_solve_static(rve_batch* b, const double* F, double* sigma, int32_t* status, int32_t ptr_kind);

/* Free every host and device resource of the batch (NULL is a no-op). */
void rve_batch_destroy(rve_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* RVE_BATCH_H */
