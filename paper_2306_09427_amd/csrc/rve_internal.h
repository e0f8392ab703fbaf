// Internal layout shared by the host runtime (rve_host.hip) and the kernels
// (rve_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <initializer_list>

namespace rve {

// Packed, reordered batch on the device.  Within an RVE the nodes are
// renumbered free-first (ids 0..nf-1, locality ordered) and boundary-last
// (ids nf..nn-1), so an operation over the free DOFs is a contiguous range
// and boundary nodes never need their positions recomputed inside the loop
// (the grouping of free and fixed DOFs of Section 3.2).
struct DevNet {
    int64_t n_rve;
    const int64_t* fib_off;   // [R+1] fibers of RVE r: fib_off[r] .. fib_off[r+1]
    const int64_t* free_off;  // [R+1] free nodes
    const int64_t* bnd_off;   // [R+1] boundary nodes
    const double* d0;         // [NF][3] reference fiber vector Xm_j - Xm_i
    const double* L0;         // [NF] rest length |d0|
    const uint32_t* ends;     // [NF] local ids i | (j << 16), free-first numbering
    const double* mass;       // [NFREE] lumped mass rhoA/2 sum L0
    const int64_t* inc_off;   // [NFREE+1] CSR node -> fiber incidence of free nodes
    const uint32_t* inc;      // local fiber id | (1u << 31 if the node is end i)
    const int64_t* binc_off;  // [NBND+1] same for boundary nodes
    const uint32_t* binc;
    const double* Xb;         // [NBND][3] centred reference coordinates of boundary nodes
    const double* V0;         // [R] reference volume
};

struct SolveArgs {
    DevNet net;
    const double* F;          // [R][9]
    const double* c;          // [R] damping
    const int32_t* list;      // RVE ids handled by this launch, in work order
    int32_t n_list;
    int32_t* queue;           // work counter, zero at launch
    int32_t law, mass_mode, init, check_every;
    double EA, B, rhoA, alpha, tol_abs, tol_rel;
    int64_t n_max;
    double* sigma;            // [R][9]
    int32_t* status;          // [R]
    int64_t* iters;           // [R]
    double* Rres;             // [R]
    double* Dres;             // [R]
    double* Bres;             // [R]
    double* h_state;          // [NFREE][3] fluctuation h (warm-start input, output)
    // workspace of the streamed engine (indexed with fib_off / free_off + r)
    void* ws_fib;             // [NF + R] Real4 (D0, q0), [NF + R] Real4 (fv, b), [NF + R] Real4 (L0, 1/L0, ends)
    void* ws_node;            // [NFREE + R] Real4 h, [NFREE] Real4 (v, 1/M), [NFREE] Real mass, [NFREE] Real4 accel
    int64_t lds_h_nodes;      // streamed engine: > 0 keeps h in LDS (this many entries per component)
    int32_t kinetic;          // 1: kinetic damping (c ignored; v = 0 at kinetic-energy peaks)
    int32_t stall_checks;     // stagnation stop: tests without R halving
    double floor_tol_rel;     // stagnation stop: floor relative to |f_bnd| (0: off)
};

struct TangentArgs {
    DevNet net;
    const double* F;             // [R][9]
    const double* sigma;         // [R][9] stress of the last solve
    const int32_t* solve_status; // [R]
    const double* h_state;       // [NFREE][3]
    const double* gsigma;        // [R][9] (vjp)
    double* out;                 // [R][81] (tangent) or [R][9] (vjp)
    int32_t* status;             // [R]
    unsigned long long* iters;   // [R] inner CG iterations summed over the RVE's right-hand sides
    int32_t* queue;              // work counter of the launch
    const int32_t* order;        // RVE ids of the launch, most free nodes first
    int64_t n_order;
    int32_t mode;                // 0 tangent, 1 vjp
    int32_t law;
    double EA, B, cg_tol;
    int64_t cg_max;
    int64_t n_free_total;
    int64_t n_rve;
    // free-node incidence in ELL chunks of 64 nodes (records s*64 + lane)
    const int64_t* chunk_first;  // [R+1] first chunk of each RVE
    const int64_t* chunk_rec;    // [NCH+1] first record of each chunk; width = records / 64
    int2* rec_static;            // [NREC] (local fiber id or -1, other end; nf if fixed or padding)
    float4* recA;                // [NREC] FP32 operator of the record's fiber: (n, k_t/L0)
    int2* recB;                  // [NREC] (other end, bits of FP32 T/l)
    float4* precond;             // [NFREE][2] inverse 3x3 diagonal block: (00, 01, 02, 11), (12, 22, -, -)
    double* par64;               // [NF][6] FP64 fiber operators: n, k_t/L0, T/l, T
    double* slot_ws64;           // per workgroup: FP64 x and b [3 slot_nodes] each (resident
                                 // kernels: then FP32 d [slot_nodes] float4)
    float4* slot_ws32;           // [grid][5][slot_nodes] per-wavefront FP32 p, q, r, d, z (wave kernel)
    int64_t slot_nodes;          // free-node capacity of a slot + 1
    int32_t build_static;        // 1: fill rec_static from the incidence first
};

// Fiber-orientation outputs at the state of the last solve.
struct OrientArgs {
    DevNet net;
    const double* F;             // [R][9]
    const double* h_state;       // [NFREE][3]
    const int32_t* status;       // [R] of the last solve
    double e[3];                 // unit reference direction
    double* omega;               // [R][9] orientation tensor <n n^T>
    double* p2;                  // [R] degree of alignment <(3 (n.e)^2 - 1)/2>
};
hipError_t launch_orientation(const OrientArgs& a, int64_t n_rve, hipStream_t s);

// Finite-difference tangent (rve_fd.hip): per-RVE host algebra and the
// kernel that seeds the probe batch (copy c of RVE r = probe RVE 6 r + c).
struct ProbeStateArgs {
    const int64_t* probe_free_off;   // [6R+1]
    const int64_t* map;              // [NFREE_probe] global base free-node index
    const double* Rm;                // [R][9] rotation of the polar decomposition
    const double* h_base;            // [NFREE][3]
    double* h_probe;                 // [NFREE_probe][3]
};
hipError_t launch_probe_state(const ProbeStateArgs& a, int64_t n_probe, hipStream_t s);
// Fprobe[6][9] = U + h T_c and the rotation Rm[9] of F = R U.
void fd_prepare(const double* F, double h, double* Fprobe, double* Rm);
// C[36] (spatial tangent, Mandel 6x6) and A[36] (dPi/dE; may be NULL) from the
// base stress and the six probe stresses; false when [M][T] is singular.
bool fd_finish(const double* F, const double* sigma, const double* sigma_probe, const double* Fprobe, double h,
               double* C, double* A);

// State export/import (rve_state.hip).  map[n] = packed global free index of
// caller node n, -1 for a boundary node; h arrays are [nodes][3] doubles.
hipError_t launch_export_h(const double* dh, const int32_t* map, int64_t nn, double* out, hipStream_t s);
hipError_t launch_import_h(const double* in, const int32_t* map, int64_t nn, double* dh, hipStream_t s);
// dh = Xm - F Xm for every free node (reference start); xm[NFREE][3] in the
// packed free-first order.
hipError_t launch_reference_h(const double* F, const int64_t* free_off, const double* xm, int64_t R, double* dh,
                              hipStream_t s);
// st[r] = st_in[r] checked against F (BAD_F, codes out of range -> NONFINITE);
// iterations 0 and norms NaN.
hipError_t launch_import_status(const double* F, const int32_t* st_in, int64_t R, int32_t* st, int64_t* iters,
                                double* Rn, double* Dn, double* Bn, hipStream_t s);

// Relaxation with the damping alternatives and the energy-balance check
// (rve_variants.hip): FP64, one workgroup per RVE (grid = n_rve, RVE r =
// block r), state in ws_node / ws_fib.  Writes h_state, status, iters and
// the residual norms; the stress kernel runs afterwards as for any solve.
struct VariantArgs {
    SolveArgs s;
    int32_t damping;        // 0 viscous, 1 kinetic, 2 adaptive
    int32_t energy_check;   // 1: stop with status 7 on an energy-balance violation
    double energy_tol;
    double* ws_node;        // [NFREE][17]
    double* ws_fib;         // [NF][5]
    double* c_final;        // [R] damping coefficient at the end
    double* energy;         // [R] final relative energy balance
};
hipError_t launch_variant(const VariantArgs& a, int64_t n_rve, hipStream_t s);
size_t variant_ws_bytes(int64_t n_free, int64_t n_fib);

// Index arithmetic of the register-resident engine, shared by the kernels
// and the host replay that bounds every index (rve_check_indexing).
// Fiber ends: two 16-bit local node ids, free-first numbering; a boundary
// end (id >= nf) reads the zero position slot nf.
__host__ __device__ inline uint32_t res_pack_ends(uint32_t ends, uint32_t nf)
{
    uint32_t i = ends & 0xffffu, j = ends >> 16;
    i = i < nf ? i : nf;
    j = j < nf ? j : nf;
    return i | (j << 16);
}
__host__ __device__ inline uint32_t res_end_i(uint32_t E) { return E & 0xffffu; }
__host__ __device__ inline uint32_t res_end_j(uint32_t E) { return E >> 16; }
// Incidence codes: fiber id in 15 bits, bit 15 set when the node is end i
// (its force enters with a minus sign).  The padding code nfib reads the zero
// force slot, so fiber ids stay below 0x7fff.
__host__ __device__ inline uint32_t res_inc_code(uint32_t w) { return (w & 0x7fffu) | ((w >> 31) << 15); }
__host__ __device__ inline uint32_t res_code_fiber(uint32_t code) { return code & 0x7fffu; }
__host__ __device__ inline bool res_code_neg(uint32_t code) { return (code & 0x8000u) != 0; }
constexpr int kResIncRegs = 4;          // incidences per node held in registers (two codes per word)
constexpr int kResMaxFibers = 0x7fff;   // fiber ids and the zero slot fit the 15-bit code

// Reduction slots of a relaxation workgroup (static LDS of the resident and
// streamed kernels): per-wave partial sums of |f_free|^2, |c M v|^2,
// |f_bnd|^2 and the kinetic energy, and two alternating slots for the
// time-step maximum.
struct RedSlots {
    double v[4][16];
    unsigned long long g64[2];
    unsigned g32[2];
};
// Static LDS of a resident workgroup: the reduction slots and the task id.
constexpr size_t kResStaticLds = sizeof(RedSlots) + 16;

// Team engine (rve_team.hip): k workgroups per RVE.  Part p of an RVE owns a
// range of its free nodes and evaluates every fiber with a free end among
// them; its local position slots are [owned | halo | zero slot].
struct TeamPart {
    int64_t fib0;    // first entry of the part in fib_gid / fib_ends
    int64_t own0;    // first entry in own_gid / own_xslot / own_inc_off
    int64_t halo0;   // first entry in halo_gid / halo_xslot
    int64_t bnd0;    // first entry in bnd_inc_off
    int32_t nfib, nown, nhalo, nbnd;
};
struct TeamArgs {
    SolveArgs s;                  // network, options, outputs, work list and counter
    const TeamPart* parts;        // [sum k] part records
    const int64_t* part_first;    // [R] first part record of each RVE (-1: not a team RVE)
    const int32_t* fib_gid;       // packed global fiber id of each part fiber
    const uint32_t* fib_ends;     // local ends i | (j << 16) (zero slot for boundary ends)
    const int32_t* own_gid;       // packed global free-node id of each owned node
    const int32_t* own_xslot;     // its exchange slot, -1 when no other part needs it
    const int64_t* own_inc_off;   // [per part: nown + 1] incidence of owned nodes (codes below)
    const uint16_t* own_inc;      // local fiber id (15 bits) | 0x8000 when the node is end i
    const int32_t* halo_gid;      // packed global free-node id of each halo node
    const int32_t* halo_xslot;    // its exchange slot
    const int64_t* bnd_inc_off;   // [per part: nbnd + 1] incidence of the boundary nodes the part reduces
    const uint16_t* bnd_inc;
    int32_t k;                    // workgroups per RVE
    int32_t kinetic;
    void* xchg;                   // [teams][2][max_xslots][9] Real: h, v, a of exported nodes
    int64_t max_xslots;
    double* partials;             // [teams][2][k][8]
    unsigned* bar;                // [teams] barrier counters, zero at launch
    int32_t* team_task;           // [teams][2]
    int32_t* error;               // set when a team barrier gave up
    int64_t spin_limit;
};
struct TeamUnit {
    int threads, sf, sn;
};
extern const TeamUnit kTeamUnit[2];   // [fp64]
constexpr int kTeamMax = 16;          // largest team
hipError_t launch_team(bool fp64, const TeamArgs& a, size_t lds_bytes, int grid, hipStream_t s);
// occupancy (workgroups per CU) and private bytes of the team build
hipError_t team_info(bool fp64, bool kin, size_t lds_bytes, int* blocks_per_cu, size_t* private_bytes);
size_t team_lds_bytes(bool fp64, int64_t n_pos, int64_t nfib);   // n_pos: owned + halo nodes

// Incidence engine (rve_kernels.hip): one workgroup per RVE; the velocity,
// acceleration and inverse mass of the free nodes stay in registers (node
// rank p in slot p / T of thread p % T), the positions in LDS (one float
// array per component, the zero slot at nf), and every iteration reads one
// record per (node, incident fiber) from global memory and evaluates the
// fiber at that end, so no fiber force is written or gathered.  Ranks order
// the free nodes by descending degree; round q holds the q-th incidence of
// the ranks 0 .. P_q - 1 (the nodes of degree > q), rank p at record
// rec_first + round_first[q] + p, so the lanes of a wave read consecutive
// records.  Record orientation: the node plays the fiber's end j, i.e. (Dn,
// Qn, 1/L0) of the scaled form with Dn = F (X_node - X_other) / L0 and the
// position difference h_node - h_other; the force it yields is the
// internal force at the node.
constexpr int kIncMaxDeg = 16;    // free-node degree limit of the tables
constexpr int kIncMaxNodes = 12288;
struct IncArgs {
    const int64_t* rec_first;     // [R] first record of the RVE, -1 when it has no tables
    const int32_t* round_first;   // [R][kIncMaxDeg + 1] start of round q relative to rec_first ([kIncMaxDeg]: total)
    const int32_t* perm;          // [NFREE] local free-node id of rank p, at free_off[r] + p
    const uint32_t* rec_fib;      // [NREC] local fiber id | (1u << 31 when the node is the fiber's end i)
    const uint2* rec_st;          // [NREC] (bits of FP32 1/L0, rank of the other end or nf for a boundary end)
    float4* rec;                  // [NREC] (Dn, Qn) under the solve's F, written at the start of the solve
    const uint2* brec_st;         // [NBINC] the same for each boundary incidence (DevNet::binc order)
    float4* brec;                 // [NBINC]
    float* imass;                 // [NFREE] inverse mass of rank p
    // global mode (RVEs whose positions do not fit LDS): node state of rank p
    // at g_first[r] + p, the zero slot at g_first[r] + nf (nf + 1 entries per
    // global-mode RVE)
    const int64_t* g_first;       // [R] first entry of the RVE's node state, -1 when it has none
    float4* hg;                   // (h, 1/M)
    float4* vg;                   // velocity
    float4* ag;                   // acceleration
};
struct IncVariant {
    int threads, slots;
};
constexpr int kNumInc = 1;
extern const IncVariant kInc[kNumInc];
inline size_t incidence_lds_bytes(int64_t nf) { return 12 * (size_t)(nf + 1); }
hipError_t launch_incidence(int variant, const SolveArgs& a, const IncArgs& inc, size_t lds_bytes, int grid,
                            hipStream_t s);
hipError_t incidence_blocks(int variant, bool kin, size_t lds_bytes, int* blocks_per_cu);
hipError_t incidence_scratch_bytes(int variant, bool kin, size_t* bytes);
// Global mode of the incidence engine: the same records, the node state in
// the global arrays above (one 1024-thread workgroup per RVE, any size).
constexpr int kIncGlobalThreads = 1024;
hipError_t launch_incidence_global(const SolveArgs& a, const IncArgs& inc, int grid, hipStream_t s);
hipError_t incidence_global_blocks(bool kin, int* blocks_per_cu);
hipError_t incidence_global_scratch_bytes(bool kin, size_t* bytes);
// whether an RVE of nf free nodes runs the LDS form (else the global mode)
inline bool incidence_lds_mode(int64_t nf) { return nf <= kIncMaxNodes; }

// Which register-resident variants exist (threads per RVE, fiber slots per
// thread, free-node slots per thread).
struct ResidentVariant {
    int threads, sf, sn;
};

constexpr int kNumResident = 6;
extern const ResidentVariant kResident[kNumResident];

// LDS bytes a resident variant needs for an RVE of nf free nodes and nfib fibers.
size_t resident_lds_bytes(bool fp64, int64_t nf, int64_t nfib, int threads);

hipError_t launch_resident(int variant, bool fp64, const SolveArgs& a, size_t lds_bytes, int grid,
                           hipStream_t s);
hipError_t launch_streamed(bool fp64, const SolveArgs& a, int grid, int threads, hipStream_t s);
size_t streamed_lds_cap();   // bytes of LDS the streamed engine may use for h
hipError_t launch_stress(const SolveArgs& a, int n_rve, hipStream_t s);
hipError_t launch_reset(int32_t* counters, int n, hipStream_t s);   // n <= 64

// Work-list order by the previous solve's cost (iterations x fibers), one
// sort per launch group; groups of more than kOrderMax RVEs keep their order.
constexpr int kOrderMax = 8192;     // positions fit the key's 14 low bits
constexpr int kOrderGroups = 32;
struct OrderArgs {
    int32_t* list;                  // device work lists of all groups
    const int64_t* iters;           // [R] iterations of the previous solve
    const int64_t* fib_off;         // [R+1]
    int32_t first[kOrderGroups];    // offset of group g's ids in list
    int32_t count[kOrderGroups];    // RVEs of group g (0: leave alone)
};
hipError_t launch_order_by_cost(const OrderArgs& o, int n_groups, hipStream_t s);
hipError_t launch_zero32(int32_t* p, int64_t n, hipStream_t s);
hipError_t launch_mark_unfinished(const int32_t* list, int n, int32_t* status, hipStream_t s);
// Tangent / VJP.  prep: statuses, ELL records (first call), fiber operators
// and preconditioner for every RVE.  Then the tasks of the RVEs in a.order:
// register/LDS-resident workgroups (variant v, RVEs with at most
// threads * sn free nodes) or streamed workgroups of 64 or 1024 threads with
// the vectors in global slots (any size).
struct TangentVariant {
    int threads, sn;
};
constexpr int kNumTanRes = 5;
extern const TangentVariant kTanRes[kNumTanRes];
hipError_t launch_tangent_prep(const TangentArgs& a, hipStream_t s);
hipError_t launch_tangent_res(int variant, const TangentArgs& a, int grid, hipStream_t s);
hipError_t launch_tangent_stream(const TangentArgs& a, int threads, int grid, hipStream_t s);
hipError_t tangent_res_blocks(int variant, bool vjp, int* blocks_per_cu);
// kin: the kinetic-damping build of the variant (launch_resident reads a.kinetic).
hipError_t max_resident_blocks(int variant, bool fp64, bool kin, size_t lds_bytes, int* blocks_per_cu);
// Private (spill) bytes per lane of a resident variant; > 0 means it spills.
hipError_t resident_scratch_bytes(int variant, bool fp64, bool kin, size_t* bytes);
// Same for a streamed build (256 or 1024 threads) and a resident tangent build.
hipError_t streamed_scratch_bytes(bool fp64, bool kin, int threads, size_t* bytes);
hipError_t tangent_res_scratch_bytes(int variant, bool vjp, size_t* bytes);
// Blocked tangent tasks (three right-hand sides of one RVE per workgroup) for
// the RVEs of the per-column variants 0 .. kNumTanBlk-1 (same node capacity);
// slot: FP64 x and b (3 slot_nodes each) and FP32 d and q (slot_nodes float4
// each) per right-hand side, 240 slot_nodes bytes per workgroup.
constexpr int kNumTanBlk = 3;
constexpr int kTanBlkRhs = 3;
extern const TangentVariant kTanBlk[kNumTanBlk];   // threads * sn = that of kTanRes[v]
hipError_t tangent_blk_blocks(int variant, int* blocks_per_cu);
hipError_t launch_tangent_blk(int variant, const TangentArgs& a, int grid, hipStream_t s);
hipError_t tangent_blk_scratch_bytes(int variant, size_t* bytes);
// Largest private segment over the kernels that have a single build (stress,
// counters, naive engine, orientation, state, tangent preparation and
// streamed tangent, variant engine, probe seeding): must be 0.
hipError_t fixed_kernels_scratch_bytes(size_t* bytes);
hipError_t kernels_fixed_private(size_t* bytes);
hipError_t naive_fixed_private(size_t* bytes);
hipError_t orient_fixed_private(size_t* bytes);
hipError_t state_fixed_private(size_t* bytes);
hipError_t tangent_fixed_private(size_t* bytes);
hipError_t variant_fixed_private(size_t* bytes);
hipError_t fd_fixed_private(size_t* bytes);

// Largest private segment (bytes per lane) over a list of kernels.
inline hipError_t max_private_bytes(std::initializer_list<const void*> kernels, size_t* bytes)
{
    size_t m = 0;
    for (const void* k : kernels) {
        hipFuncAttributes at;
        const hipError_t e = hipFuncGetAttributes(&at, k);
        if (e != hipSuccess) return e;
        m = std::max(m, (size_t)at.localSizeBytes);
    }
    *bytes = m;
    return hipSuccess;
}


}  // namespace rve
