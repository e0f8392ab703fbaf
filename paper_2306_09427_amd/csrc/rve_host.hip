// Host runtime and C ABI of the batched RVE solver (the "RVE batch manager"
// of Section 4.3: data marshalling on the CPU, solver selection, launches).
//
// rve_batch_create validates the networks on the host before touching the
// device, so malformed input is rejected (RVE_EINVAL) even where no GPU is
// present.  Packing per RVE: free nodes first in breadth-first locality
// order, boundary nodes last; fibers sorted by their lower end; reference
// fiber vectors, rest lengths and lumped masses in FP64; CSR node->fiber
// incidence with the end sign.  All RVEs of a batch share one device
// allocation in row-offset + value layout (the packed-view layout of
// Section 4.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rve_batch.h"
#include "rve_internal.h"

using namespace rve;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(RVE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

struct DeviceArena {
    char* base = nullptr;
    size_t used = 0, cap = 0;
    size_t reserve(size_t bytes)
    {
        size_t off = (used + 255) & ~size_t(255);
        used = off + bytes;
        return off;
    }
};

}  // namespace

struct rve_batch {
    int64_t R = 0, NN = 0, NF = 0, NFREE = 0, NBND = 0;
    std::vector<int64_t> node_off, fib_off, free_off, bnd_off;
    std::vector<int32_t> newid;        // [NN] original node -> reordered local id
    std::vector<double> Xm;            // [NN][3] centred reference coordinates (original order)
    std::vector<int64_t> nf_of, nfib_of;
    std::vector<int32_t> maxdeg_of;
    // tangent incidence in ELL chunks of 64 free nodes: first chunk of each
    // RVE, and the first record of each chunk (width = records / 64, a
    // multiple of 4)
    std::vector<int64_t> chunk_first, chunk_rec;
    rve_opts opts{};
    std::vector<double> c_host;
    int device = 0, n_cu = 0;
    // device memory
    char* dmem = nullptr;
    DevNet net{};
    double *dF = nullptr, *dc = nullptr, *dsigma = nullptr, *dR = nullptr, *dD = nullptr, *dB = nullptr;
    double *dh = nullptr, *dV0 = nullptr;
    int32_t *dstatus = nullptr, *dqueue = nullptr, *dlist = nullptr;
    int64_t* diters = nullptr;
    bool cost_order = false;   // diters holds a previous solve's iterations: order the work lists by cost
    void *ws_fib = nullptr, *ws_node = nullptr;
    size_t ws_fib_bytes = 0, ws_node_bytes = 0;
    // engine assignment: RVE ids per launch group, in longest-first order
    std::vector<int32_t> group_variant;        // resident variant per group, -1 = streamed
    std::vector<std::vector<int32_t>> groups;  // RVE ids
    std::vector<int32_t> group_first;          // offset of each group's ids in dlist
    std::vector<size_t> group_lds;
    bool have_state = false;
    // [kinetic][fp64][variant]: the build uses private (scratch) memory and is never launched
    bool variant_spills[2][2][kNumResident] = {};
    bool streamed_private[2][2][2] = {};            // [kinetic][fp64][1024 threads]: same for the streamed builds
    bool tangent_private[2][kNumTanRes] = {};        // [vjp][variant]: same for the resident tangent builds
    bool tangent_blk_private[kNumTanBlk] = {};       // same for the blocked tangent builds
    // tangent / vjp workspace
    char* t_mem = nullptr;             // operators, records, preconditioner, chunk tables, I/O
    bool t_static_built = false;       // records' (fiber, other end) filled
    double* t_par64 = nullptr;
    int2 *t_rec_static = nullptr, *t_recB = nullptr;
    float4 *t_recA = nullptr, *t_precond = nullptr;
    int64_t *t_chunk_first = nullptr, *t_chunk_rec = nullptr;
    double* t_out = nullptr;
    double* t_in = nullptr;
    int32_t* t_status = nullptr;
    int64_t* t_iters = nullptr;
    int32_t* t_order = nullptr;
    std::vector<int64_t> t_group_first;   // [kNumTanRes + 2] offsets of the task groups in t_order
    std::vector<int32_t> t_order_host;    // host copy of t_order
    std::vector<int64_t> t_max_nf;        // per launch of the last call: largest free-node count
    char* t_slots = nullptr;           // per-wavefront solver vectors
    double* o_mem = nullptr;           // orientation outputs [R][9] + [R]
    // finite-difference tangent: the probe batch (six copies of every RVE),
    // the probe-to-base free-node map and the per-call rotations
    rve_batch* probe = nullptr;
    int64_t* d_probe_map = nullptr;
    double* d_fd_rot = nullptr;
    size_t t_slot_bytes = 0;
    // profiling events: [group][start, stop], then the stress kernel
    bool profile = false;
    std::vector<hipEvent_t> ev;
    int ev_used = 0;
    // autotuner choice per [fp64][tier]: -2 untuned, -1 streamed, else a resident variant
    int tuned[2][8] = {{-2, -2, -2, -2, -2, -2, -2, -2}, {-2, -2, -2, -2, -2, -2, -2, -2}};
    int32_t* dtune_list = nullptr;
    int32_t* d_state_map = nullptr;    // [NN] packed global free index of each caller node, -1 boundary
    bool state_map_ready = false;
    bool t_tables = false;             // tangent arena carved, task tables uploaded
    // caller-provided workspace (rve_batch_bind_workspace): the streamed
    // workspace, tangent arena and slots, orientation outputs and state map
    // point into it and are never freed by the library
    char* ws_user = nullptr;
    size_t ws_user_bytes = 0;
    // damping alternatives / energy check: node and fiber state, then
    // c_final [R] and the energy balance [R]; whether the last solve used them
    double* v_ws = nullptr;
    bool last_variant = false;
    uint64_t generation = 0;           // bumped by solve, import_state, set_opts
    // team engine (k workgroups per RVE): per-RVE team size (0: no partition),
    // its largest exchange-slot count, LDS bytes of its largest part per
    // precision; the tables on the device; the team work area
    std::vector<int32_t> team_k;
    std::vector<int64_t> team_xslots;
    std::vector<size_t> team_lds[2];
    char* team_mem = nullptr;
    TeamArgs team_tab{};               // table pointers (carved from team_mem)
    char* team_ws = nullptr;           // library-owned team work area
    size_t team_ws_bytes = 0;
    std::vector<int32_t> group_team;   // team size of each group, 0 = not a team group
    int64_t team_spin_limit = int64_t(1) << 24;   // polls of a team barrier before it gives up
    // autotuner's choice for RVEs partitioned into k parts: [fp64][k] 1 team, 0 streamed, -1 untuned
    int tuned_team[2][kTeamMax + 1];
    // concurrent launch groups: auxiliary streams (default priority) and the
    // events that fork them from and join them to the batch's stream
    hipStream_t aux[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork_ev = nullptr, join_ev[3] = {nullptr, nullptr, nullptr};
    double* d_xm_free = nullptr;       // [NFREE][3] reference coordinates of free nodes (RVE_INIT_REFERENCE)
    // incidence engine: per-RVE first record (-1: no tables), the tables on
    // the device, and which builds use private memory ([kinetic][variant])
    std::vector<int64_t> inc_first;
    char* inc_mem = nullptr;
    IncArgs inc_tab{};
    bool inc_private[2][kNumInc] = {};
    bool incg_private[2] = {};         // [kinetic]: the global-mode build uses private memory
};

// Launch-group codes beside the resident variants (>= 0): the streamed
// kernel, teams of k workgroups per RVE (-1 - k, k >= 2) and the incidence
// kernel.
constexpr int kStreamedGroup = -1;
constexpr int kIncGroup = -100;
constexpr int kIncGlobalGroup = -101;
static bool team_group(int v) { return v <= -3 && v >= -1 - kTeamMax; }

// Adaptive damping and the energy check run on the FP64 variant engine;
// kinetic damping alone runs on the ordinary engines (their kinetic builds).
static bool variant_mode(const rve_opts& o)
{
    return o.damping == RVE_DAMP_ADAPTIVE || o.energy_check != 0;
}

static bool kinetic_mode(const rve_opts& o)
{
    return o.damping == RVE_DAMP_KINETIC && !variant_mode(o);
}

static bool spills(const rve_batch* b, int v, bool fp64)
{
    return b->variant_spills[kinetic_mode(b->opts) ? 1 : 0][fp64 ? 1 : 0][v];
}

// Size tiers: distinct (fiber, node) capacities of the resident variants, ascending.
static std::vector<std::pair<int64_t, int64_t>> tier_caps()
{
    std::vector<std::pair<int64_t, int64_t>> caps;
    for (int v = 0; v < kNumResident; ++v)
        caps.push_back({(int64_t)kResident[v].threads * kResident[v].sf, (int64_t)kResident[v].threads * kResident[v].sn});
    std::sort(caps.begin(), caps.end());
    caps.erase(std::unique(caps.begin(), caps.end()), caps.end());
    return caps;
}

// Tier of an RVE (index into tier_caps) or -1 when only the streamed kernel can take it.
static int tier_of(const rve_batch* b, int64_t r, bool fp64)
{
    size_t lds_cap = 160 * 1024 - 4096;
    if (b->nfib_of[r] >= kResMaxFibers || resident_lds_bytes(fp64, b->nf_of[r], b->nfib_of[r], 0) > lds_cap) return -1;
    auto caps = tier_caps();
    for (size_t t = 0; t < caps.size(); ++t)
        if (b->nfib_of[r] <= caps[t].first && b->nf_of[r] <= caps[t].second) return (int)t;
    return -1;
}

static bool variant_fits_tier(int v, int tier)
{
    auto caps = tier_caps();
    return (int64_t)kResident[v].threads * kResident[v].sf >= caps[tier].first &&
           (int64_t)kResident[v].threads * kResident[v].sn >= caps[tier].second;
}

static int ensure_events(rve_batch* b, int n)
{
    while ((int)b->ev.size() < n) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        b->ev.push_back(e);
    }
    return RVE_OK;
}

// ------------------------------------------------------------------ helpers
static int validate_opts(const rve_opts* o, int64_t R)
{
    if (!o) return fail(RVE_EINVAL, "opts is NULL");
    if (o->precision != RVE_FP64 && o->precision != RVE_MIXED) return fail(RVE_EINVAL, "bad precision");
    if (o->law != RVE_LAW_LINEAR && o->law != RVE_LAW_EXP) return fail(RVE_EINVAL, "bad law");
    if (o->mass != RVE_MASS_LUMPED && o->mass != RVE_MASS_SCALED) return fail(RVE_EINVAL, "bad mass mode");
    if (o->init != RVE_INIT_AFFINE && o->init != RVE_INIT_REFERENCE && o->init != RVE_INIT_WARM)
        return fail(RVE_EINVAL, "bad init");
    if (!(o->EA > 0) || !std::isfinite(o->EA)) return fail(RVE_EINVAL, "EA must be positive");
    if (o->law == RVE_LAW_EXP && (!(o->B > 0) || !std::isfinite(o->B))) return fail(RVE_EINVAL, "B must be positive");
    if (!(o->rhoA > 0) || !std::isfinite(o->rhoA)) return fail(RVE_EINVAL, "rhoA must be positive");
    if (!(o->alpha > 0) || !(o->alpha <= 1.0)) return fail(RVE_EINVAL, "alpha must be in (0, 1]");
    if (!o->c_per_rve && (!(o->c >= 0) || !std::isfinite(o->c))) return fail(RVE_EINVAL, "c must be >= 0");
    if (o->c_per_rve)
        for (int64_t r = 0; r < R; ++r)
            if (!(o->c_per_rve[r] >= 0) || !std::isfinite(o->c_per_rve[r]))
                return fail(RVE_EINVAL, "c_per_rve[" + std::to_string(r) + "] must be >= 0");
    if (!(o->tol_abs >= 0) || !(o->tol_rel >= 0)) return fail(RVE_EINVAL, "tolerances must be >= 0");
    if (o->n_max < 0) return fail(RVE_EINVAL, "n_max must be >= 0");
    if (o->check_every < 1) return fail(RVE_EINVAL, "check_every must be >= 1");
    if (o->engine != RVE_ENGINE_AUTO && o->engine != RVE_ENGINE_STREAMED && o->engine != RVE_ENGINE_NAIVE &&
        o->engine != RVE_ENGINE_TEAM && o->engine != RVE_ENGINE_INCIDENCE)
        return fail(RVE_EINVAL, "bad engine");
    if (o->engine == RVE_ENGINE_NAIVE && o->precision != RVE_FP64)
        return fail(RVE_EINVAL, "the naive engine is FP64 only");
    if (o->engine == RVE_ENGINE_INCIDENCE && o->precision != RVE_MIXED)
        return fail(RVE_EINVAL, "the incidence engine is RVE_MIXED only");
    if (!(o->cg_tol > 0) || o->cg_max_iter < 0) return fail(RVE_EINVAL, "cg_tol must be > 0, cg_max_iter >= 0");
    if (o->threads_per_rve != 0 && o->threads_per_rve != 256 && o->threads_per_rve != 512 &&
        o->threads_per_rve != 768 && o->threads_per_rve != 1024)
        return fail(RVE_EINVAL, "threads_per_rve must be 0, 256, 512, 768 or 1024");
    if (o->damping != RVE_DAMP_VISCOUS && o->damping != RVE_DAMP_KINETIC && o->damping != RVE_DAMP_ADAPTIVE)
        return fail(RVE_EINVAL, "bad damping mode");
    if (!(o->energy_tol > 0) || !std::isfinite(o->energy_tol)) return fail(RVE_EINVAL, "energy_tol must be > 0");
    if (o->damping != RVE_DAMP_VISCOUS || o->energy_check) {
        if (o->engine == RVE_ENGINE_NAIVE)
            return fail(RVE_EINVAL, "the naive engine has constant viscous damping only");
        if ((o->damping == RVE_DAMP_ADAPTIVE || o->energy_check) && o->precision != RVE_FP64)
            return fail(RVE_EINVAL, "adaptive damping and the energy check are FP64 only");
    }
    if (o->tangent_rhs != 0 && o->tangent_rhs != 1 && o->tangent_rhs != 3)
        return fail(RVE_EINVAL, "tangent_rhs must be 0, 1 or 3");
    if (o->work_order != RVE_ORDER_AUTO && o->work_order != RVE_ORDER_HOST && o->work_order != RVE_ORDER_COST)
        return fail(RVE_EINVAL, "work_order must be RVE_ORDER_AUTO, RVE_ORDER_HOST or RVE_ORDER_COST");
    if (!(o->floor_tol_rel >= 0) || !std::isfinite(o->floor_tol_rel))
        return fail(RVE_EINVAL, "floor_tol_rel must be >= 0 and finite");
    if (o->floor_tol_rel > 0) {
        if (o->stall_checks < 1) return fail(RVE_EINVAL, "stall_checks must be >= 1");
        if (o->engine == RVE_ENGINE_NAIVE || o->damping != RVE_DAMP_VISCOUS || o->energy_check)
            return fail(RVE_EINVAL,
                        "the stagnation stop needs constant viscous damping on the resident or streamed engine");
    }
    return RVE_OK;
}

static int validate_net(const rve_net_desc* d)
{
    if (!d) return fail(RVE_EINVAL, "net is NULL");
    if (d->n_rve < 0) return fail(RVE_EINVAL, "n_rve < 0");
    if (d->n_rve == 0) return RVE_OK;
    if (!d->node_off || !d->fib_off || !d->X || !d->is_bnd || !d->fib)
        return fail(RVE_EINVAL, "NULL array in net");
    if (d->node_off[0] != 0 || d->fib_off[0] != 0) return fail(RVE_EINVAL, "offsets must start at 0");
    for (int64_t r = 0; r < d->n_rve; ++r) {
        int64_t n0 = d->node_off[r], n1 = d->node_off[r + 1], f0 = d->fib_off[r], f1 = d->fib_off[r + 1];
        std::string rs = "RVE " + std::to_string(r) + ": ";
        if (n1 < n0 || f1 < f0) return fail(RVE_EINVAL, rs + "offsets decrease");
        int64_t nn = n1 - n0;
        if (nn >= 65535) return fail(RVE_EINVAL, rs + "65535 or more nodes");
        bool anyb = false;
        for (int64_t p = n0; p < n1; ++p) {
            if (d->is_bnd[p] > 1) return fail(RVE_EINVAL, rs + "is_bnd must be 0 or 1");
            anyb |= d->is_bnd[p] != 0;
            for (int k = 0; k < 3; ++k)
                if (!std::isfinite(d->X[3 * p + k])) return fail(RVE_EINVAL, rs + "non-finite coordinate");
        }
        if (!anyb) return fail(RVE_EINVAL, rs + "no boundary node");
        for (int64_t k = f0; k < f1; ++k) {
            int32_t i = d->fib[2 * k], j = d->fib[2 * k + 1];
            if (i < 0 || j < 0 || i >= nn || j >= nn)
                return fail(RVE_EINVAL, rs + "fiber " + std::to_string(k - f0) + " has a node id out of range");
            if (i == j) return fail(RVE_EINVAL, rs + "fiber " + std::to_string(k - f0) + " joins a node to itself");
            const double* a = d->X + 3 * (n0 + i);
            const double* b = d->X + 3 * (n0 + j);
            double L = std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) +
                                 (b[2] - a[2]) * (b[2] - a[2]));
            if (!(L > 0)) return fail(RVE_EINVAL, rs + "fiber " + std::to_string(k - f0) + " has zero length");
        }
        if (d->V0 && !(d->V0[r] > 0)) return fail(RVE_EINVAL, rs + "V0 must be positive");
        if (d->L0)
            for (int64_t k = f0; k < f1; ++k)
                if (!(d->L0[k] > 0) || !std::isfinite(d->L0[k]))
                    return fail(RVE_EINVAL, rs + "fiber " + std::to_string(k - f0) + ": L0 must be positive and finite");
    }
    return RVE_OK;
}

// Host packing of one batch (everything except the upload).
struct HostPack {
    std::vector<int64_t> fib_off, free_off, bnd_off;
    std::vector<double> d0, L0, mass, Xb;
    std::vector<uint32_t> ends, inc, binc;
    std::vector<int64_t> inc_off, binc_off;
    std::vector<int32_t> newid;
    std::vector<int64_t> nf, nfib;
    std::vector<int32_t> maxdeg;
};

static void pack_batch(const rve_net_desc* d, HostPack& P)
{
    const int64_t R = d->n_rve;
    P.fib_off.assign(R + 1, 0);
    P.free_off.assign(R + 1, 0);
    P.bnd_off.assign(R + 1, 0);
    const int64_t NN = R ? d->node_off[R] : 0, NF = R ? d->fib_off[R] : 0;
    P.newid.assign(NN, -1);
    P.d0.resize(3 * NF);
    P.L0.resize(NF);
    P.ends.resize(NF);
    P.nf.assign(R, 0);
    P.nfib.assign(R, 0);
    P.maxdeg.assign(R, 0);
    P.inc_off.push_back(0);
    P.binc_off.push_back(0);
    std::vector<std::vector<std::pair<int32_t, int32_t>>> adj;
    for (int64_t r = 0; r < R; ++r) {
        const int64_t n0 = d->node_off[r], nn = d->node_off[r + 1] - n0;
        const int64_t f0 = d->fib_off[r], nfib = d->fib_off[r + 1] - f0;
        const uint8_t* ib = d->is_bnd + n0;
        const int32_t* fb = d->fib + 2 * f0;
        adj.assign(nn, {});
        for (int64_t k = 0; k < nfib; ++k) {
            adj[fb[2 * k]].push_back({fb[2 * k + 1], (int32_t)k});
            adj[fb[2 * k + 1]].push_back({fb[2 * k], (int32_t)k});
        }
        // breadth-first order of the free nodes (locality), seeded at the
        // lowest-degree unvisited free node of each component
        std::vector<int32_t> order;
        order.reserve(nn);
        std::vector<char> seen(nn, 0);
        std::vector<int32_t> seeds;
        for (int32_t p = 0; p < nn; ++p)
            if (!ib[p]) seeds.push_back(p);
        std::stable_sort(seeds.begin(), seeds.end(),
                         [&](int32_t a, int32_t b) { return adj[a].size() < adj[b].size(); });
        for (int32_t s : seeds) {
            if (seen[s]) continue;
            size_t head = order.size();
            order.push_back(s);
            seen[s] = 1;
            while (head < order.size()) {
                int32_t u = order[head++];
                for (auto& e : adj[u])
                    if (!ib[e.first] && !seen[e.first]) {
                        seen[e.first] = 1;
                        order.push_back(e.first);
                    }
            }
        }
        const int64_t nf = (int64_t)order.size();
        // Nodes of degree above 4 go to the end of the free range (stable, so
        // the locality order is kept inside each class): most waves then see
        // only degree <= 4 nodes and skip the extra gathers entirely.
        std::stable_partition(order.begin(), order.end(), [&](int32_t p) { return adj[p].size() <= 4; });
        for (int32_t p = 0; p < nn; ++p)
            if (ib[p]) order.push_back(p);
        std::vector<int32_t> nid(nn);
        for (int64_t q = 0; q < nn; ++q) nid[order[q]] = (int32_t)q;
        for (int64_t q = 0; q < nn; ++q) P.newid[n0 + q] = nid[q];
        P.nf[r] = nf;
        P.nfib[r] = nfib;
        P.fib_off[r + 1] = P.fib_off[r] + nfib;
        P.free_off[r + 1] = P.free_off[r] + nf;
        P.bnd_off[r + 1] = P.bnd_off[r] + (nn - nf);
        // fibers sorted by their lower reordered end
        std::vector<int32_t> fo(nfib);
        for (int64_t k = 0; k < nfib; ++k) fo[k] = (int32_t)k;
        std::stable_sort(fo.begin(), fo.end(), [&](int32_t a, int32_t b) {
            int32_t la = std::min(nid[fb[2 * a]], nid[fb[2 * a + 1]]), lb = std::min(nid[fb[2 * b]], nid[fb[2 * b + 1]]);
            if (la != lb) return la < lb;
            return std::max(nid[fb[2 * a]], nid[fb[2 * a + 1]]) < std::max(nid[fb[2 * b]], nid[fb[2 * b + 1]]);
        });
        std::vector<int32_t> fpos(nfib);
        std::vector<std::vector<uint32_t>> inc_of(nn);
        for (int64_t q = 0; q < nfib; ++q) {
            int32_t k = fo[q];
            fpos[k] = (int32_t)q;
            int32_t i = fb[2 * k], j = fb[2 * k + 1];
            const double* Xi = d->X + 3 * (n0 + i);
            const double* Xj = d->X + 3 * (n0 + j);
            int64_t g = P.fib_off[r] + q;
            double dx = Xj[0] - Xi[0], dy = Xj[1] - Xi[1], dz = Xj[2] - Xi[2];
            P.d0[3 * g] = dx;
            P.d0[3 * g + 1] = dy;
            P.d0[3 * g + 2] = dz;
            P.L0[g] = d->L0 ? d->L0[f0 + k] : std::sqrt(dx * dx + dy * dy + dz * dz);
            P.ends[g] = (uint32_t)nid[i] | ((uint32_t)nid[j] << 16);
            inc_of[nid[i]].push_back((uint32_t)q | (1u << 31));
            inc_of[nid[j]].push_back((uint32_t)q);
        }
        for (int64_t q = 0; q < nn; ++q)
            std::sort(inc_of[q].begin(), inc_of[q].end(),
                      [](uint32_t a, uint32_t b) { return (a & 0x7fffffffu) < (b & 0x7fffffffu); });
        int32_t md = 0;
        for (int64_t q = 0; q < nf; ++q) {
            double m = 0.0;
            for (uint32_t w : inc_of[q]) {
                m += 0.5 * P.L0[P.fib_off[r] + (w & 0x7fffffffu)];
                P.inc.push_back(w);
            }
            P.mass.push_back(m);
            P.inc_off.push_back((int64_t)P.inc.size());
            md = std::max<int32_t>(md, (int32_t)inc_of[q].size());
        }
        P.maxdeg[r] = md;
        for (int64_t q = nf; q < nn; ++q) {
            for (uint32_t w : inc_of[q]) P.binc.push_back(w);
            P.binc_off.push_back((int64_t)P.binc.size());
            const double* X = d->X + 3 * (n0 + order[q]);
            P.Xb.push_back(X[0] - 0.5);
            P.Xb.push_back(X[1] - 0.5);
            P.Xb.push_back(X[2] - 0.5);
        }
    }
}



template <typename T>
static T* carve(char* base, size_t off)
{
    return reinterpret_cast<T*>(base + off);
}

// ------------------------------------------------------------------ team partition
// Partition of one RVE for the team engine (k workgroups): free nodes split
// into k contiguous ranges of a breadth-first order over the free-free
// fibers; part p owns its range and takes every fiber with a free end in it
// (fibers with no free end go to part 0), every boundary node whose fibers
// it holds all of (the first fiber's part, completed with the others), and
// holds the foreign free ends of its fibers as halo.  Returns false when a
// part exceeds the team build's capacity (fibers, owned nodes, LDS).
struct TeamHost {
    std::vector<TeamPart> parts;
    std::vector<int64_t> part_first;
    std::vector<int32_t> fib_gid, own_gid, own_xslot, halo_gid, halo_xslot;
    std::vector<uint32_t> fib_ends;
    std::vector<int64_t> own_inc_off, bnd_inc_off;
    std::vector<uint16_t> own_inc, bnd_inc;
};

static bool team_partition(const HostPack& P, int64_t r, int k, TeamHost& T, int64_t* xslots, size_t lds_out[2])
{
    const int64_t f0 = P.fib_off[r], nfib = P.fib_off[r + 1] - f0;
    const int64_t a0 = P.free_off[r], nf = P.free_off[r + 1] - a0;
    const int64_t b0 = P.bnd_off[r], nb = P.bnd_off[r + 1] - b0;
    const int cap_f = kTeamUnit[0].threads * kTeamUnit[0].sf, cap_n = kTeamUnit[0].threads * kTeamUnit[0].sn;
    if (nf < k) return false;
    // breadth-first order over free-free fibers
    std::vector<std::vector<int32_t>> adj(nf);
    for (int64_t q = 0; q < nfib; ++q) {
        const uint32_t e = P.ends[f0 + q];
        const int64_t i = e & 0xffffu, j = e >> 16;
        if (i < nf && j < nf) {
            adj[i].push_back((int32_t)j);
            adj[j].push_back((int32_t)i);
        }
    }
    std::vector<int32_t> order;
    order.reserve(nf);
    std::vector<char> seen(nf, 0);
    for (int64_t s0 = 0; s0 < nf; ++s0) {
        if (seen[s0]) continue;
        size_t head = order.size();
        order.push_back((int32_t)s0);
        seen[s0] = 1;
        while (head < order.size()) {
            const int32_t u = order[head++];
            for (int32_t w : adj[u])
                if (!seen[w]) {
                    seen[w] = 1;
                    order.push_back(w);
                }
        }
    }
    std::vector<int32_t> part_of(nf);
    for (int64_t q = 0; q < nf; ++q) part_of[order[q]] = (int32_t)std::min<int64_t>(k - 1, q * k / nf);
    std::vector<std::vector<int32_t>> fibs(k), bnds(k);
    auto parts_of_fiber = [&](int64_t q, int32_t* out) {
        const uint32_t e = P.ends[f0 + q];
        const int64_t i = e & 0xffffu, j = e >> 16;
        int n = 0;
        if (i < nf) out[n++] = part_of[i];
        if (j < nf && (n == 0 || part_of[j] != out[0])) out[n++] = part_of[j];
        if (n == 0) out[n++] = 0;
        return n;
    };
    for (int64_t q = 0; q < nfib; ++q) {
        int32_t ps[2];
        const int n = parts_of_fiber(q, ps);
        for (int t = 0; t < n; ++t) fibs[ps[t]].push_back((int32_t)q);
    }
    for (int64_t bq = 0; bq < nb; ++bq) {
        const int64_t e0 = P.binc_off[b0 + bq], e1 = P.binc_off[b0 + bq + 1];
        if (e0 == e1) continue;
        int32_t ps[2];
        parts_of_fiber(P.binc[e0] & 0x7fffffffu, ps);
        const int32_t pb = ps[0];
        for (int64_t e = e0; e < e1; ++e) fibs[pb].push_back((int32_t)(P.binc[e] & 0x7fffffffu));
        bnds[pb].push_back((int32_t)(nf + bq));
    }
    for (auto& f : fibs) {
        std::sort(f.begin(), f.end());
        f.erase(std::unique(f.begin(), f.end()), f.end());
    }
    // halo sets and exchange slots
    std::vector<std::vector<int32_t>> owned(k), halo(k);
    for (int64_t a = 0; a < nf; ++a) owned[part_of[a]].push_back((int32_t)a);
    std::vector<int32_t> xslot(nf, -1);
    int64_t nx = 0;
    for (int p = 0; p < k; ++p) {
        std::vector<int32_t>& h = halo[p];
        for (int32_t q : fibs[p]) {
            const uint32_t e = P.ends[f0 + q];
            const int64_t i = e & 0xffffu, j = e >> 16;
            if (i < nf && part_of[i] != p) h.push_back((int32_t)i);
            if (j < nf && part_of[j] != p) h.push_back((int32_t)j);
        }
        std::sort(h.begin(), h.end());
        h.erase(std::unique(h.begin(), h.end()), h.end());
        for (int32_t a : h)
            if (xslot[a] < 0) xslot[a] = (int32_t)nx++;
    }
    size_t lds[2] = {0, 0};
    for (int p = 0; p < k; ++p) {
        const int64_t npos = (int64_t)owned[p].size() + (int64_t)halo[p].size();
        if ((int64_t)fibs[p].size() > cap_f || (int64_t)owned[p].size() > cap_n || npos + 1 >= 65535) return false;
        for (int fp = 0; fp < 2; ++fp) {
            const size_t l = team_lds_bytes(fp == 1, npos, (int64_t)fibs[p].size());
            if (l + 4096 > 160 * 1024) return false;
            lds[fp] = std::max(lds[fp], l);
        }
    }
    // append the tables
    T.part_first[r] = (int64_t)T.parts.size();
    for (int p = 0; p < k; ++p) {
        TeamPart tp{};
        tp.fib0 = (int64_t)T.fib_gid.size();
        tp.own0 = (int64_t)T.own_gid.size();
        tp.halo0 = (int64_t)T.halo_gid.size();
        tp.bnd0 = (int64_t)T.bnd_inc_off.size() - 1;
        tp.nfib = (int32_t)fibs[p].size();
        tp.nown = (int32_t)owned[p].size();
        tp.nhalo = (int32_t)halo[p].size();
        tp.nbnd = (int32_t)bnds[p].size();
        const uint32_t zs = (uint32_t)(tp.nown + tp.nhalo);
        // local position slot of a packed node id (owned, halo, else the zero slot)
        auto local = [&](int64_t id) -> uint32_t {
            if (id >= nf) return zs;
            if (part_of[id] == p) return (uint32_t)(std::lower_bound(owned[p].begin(), owned[p].end(), (int32_t)id) -
                                                    owned[p].begin());
            return (uint32_t)tp.nown +
                   (uint32_t)(std::lower_bound(halo[p].begin(), halo[p].end(), (int32_t)id) - halo[p].begin());
        };
        auto code_of = [&](uint32_t w) -> uint16_t {
            const int32_t q = (int32_t)(w & 0x7fffffffu);
            const uint16_t lf = (uint16_t)(std::lower_bound(fibs[p].begin(), fibs[p].end(), q) - fibs[p].begin());
            return (uint16_t)(lf | ((w >> 31) ? 0x8000u : 0u));
        };
        for (int32_t q : fibs[p]) {
            const uint32_t e = P.ends[f0 + q];
            T.fib_gid.push_back((int32_t)(f0 + q));
            T.fib_ends.push_back(local(e & 0xffffu) | (local(e >> 16) << 16));
        }
        for (int32_t a : owned[p]) {
            T.own_gid.push_back((int32_t)(a0 + a));
            T.own_xslot.push_back(xslot[a]);
            for (int64_t e = P.inc_off[a0 + a]; e < P.inc_off[a0 + a + 1]; ++e) T.own_inc.push_back(code_of(P.inc[e]));
            T.own_inc_off.push_back((int64_t)T.own_inc.size());
        }
        for (int32_t a : halo[p]) {
            T.halo_gid.push_back((int32_t)(a0 + a));
            T.halo_xslot.push_back(xslot[a]);
        }
        for (int32_t bn : bnds[p]) {
            const int64_t bq = bn - nf;
            for (int64_t e = P.binc_off[b0 + bq]; e < P.binc_off[b0 + bq + 1]; ++e) T.bnd_inc.push_back(code_of(P.binc[e]));
            T.bnd_inc_off.push_back((int64_t)T.bnd_inc.size());
        }
        T.parts.push_back(tp);
    }
    *xslots = nx;
    lds_out[0] = lds[0];
    lds_out[1] = lds[1];
    return true;
}


// Team partitions of every RVE that no resident build holds in FP64 (more
// than 3072 fibers or 1536 free nodes): the smallest team size, from the
// part capacity up to kTeamMax, whose parts fit the team build; RVEs without
// one run on the streamed kernel.  Tables for all of them in one device
// allocation.
static int build_team_tables(rve_batch* b, const HostPack& P)
{
    const int64_t R = b->R;
    b->team_k.assign(R, 0);
    b->team_xslots.assign(R, 0);
    b->team_lds[0].assign(R, 0);
    b->team_lds[1].assign(R, 0);
    const int cap_f = kTeamUnit[0].threads * kTeamUnit[0].sf, cap_n = kTeamUnit[0].threads * kTeamUnit[0].sn;
    TeamHost T;
    T.part_first.assign(R, -1);
    T.own_inc_off.assign(1, 0);
    T.bnd_inc_off.assign(1, 0);
    bool any = false;
    try {
        for (int64_t r = 0; r < R; ++r) {
            const int64_t nfib = b->nfib_of[r], nf = b->nf_of[r];
            if (nfib <= cap_f && nf <= cap_n) continue;
            int k0 = (int)std::max<int64_t>(2, std::max((nfib * 11 + 10 * cap_f - 1) / (10 * cap_f),
                                                        (nf * 11 + 10 * cap_n - 1) / (10 * cap_n)));
            for (int k = k0; k <= kTeamMax; ++k) {
                TeamHost save_sizes;   // roll back on failure: remember the table lengths
                const size_t s_parts = T.parts.size(), s_fib = T.fib_gid.size(), s_own = T.own_gid.size(),
                             s_inc = T.own_inc.size(), s_ioff = T.own_inc_off.size(), s_halo = T.halo_gid.size(),
                             s_binc = T.bnd_inc.size(), s_boff = T.bnd_inc_off.size();
                int64_t xs = 0;
                size_t lds[2];
                if (team_partition(P, r, k, T, &xs, lds)) {
                    b->team_k[r] = k;
                    b->team_xslots[r] = xs;
                    b->team_lds[0][r] = lds[0];
                    b->team_lds[1][r] = lds[1];
                    any = true;
                    break;
                }
                T.parts.resize(s_parts);
                T.fib_gid.resize(s_fib);
                T.fib_ends.resize(s_fib);
                T.own_gid.resize(s_own);
                T.own_xslot.resize(s_own);
                T.own_inc.resize(s_inc);
                T.own_inc_off.resize(s_ioff);
                T.halo_gid.resize(s_halo);
                T.halo_xslot.resize(s_halo);
                T.bnd_inc.resize(s_binc);
                T.bnd_inc_off.resize(s_boff);
                T.part_first[r] = -1;
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(RVE_ENOMEM, "host allocation failed while partitioning RVEs for the team engine");
    }
    if (!any) return RVE_OK;
    DeviceArena A;
    const size_t o_parts = A.reserve(sizeof(TeamPart) * T.parts.size()), o_first = A.reserve(8 * (size_t)R),
                 o_fg = A.reserve(4 * T.fib_gid.size()), o_fe = A.reserve(4 * T.fib_ends.size()),
                 o_og = A.reserve(4 * T.own_gid.size()), o_ox = A.reserve(4 * T.own_xslot.size()),
                 o_oi = A.reserve(8 * T.own_inc_off.size()), o_oc = A.reserve(2 * T.own_inc.size() + 2),
                 o_hg = A.reserve(4 * T.halo_gid.size() + 4), o_hx = A.reserve(4 * T.halo_xslot.size() + 4),
                 o_bi = A.reserve(8 * T.bnd_inc_off.size()), o_bc = A.reserve(2 * T.bnd_inc.size() + 2);
    if (hipMalloc((void**)&b->team_mem, A.used + 256) != hipSuccess) {
        b->team_mem = nullptr;
        return fail(RVE_ENOMEM, "device allocation of the team tables failed");
    }
    char* m = b->team_mem;
    auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpy(m + off, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    hipError_t e = hipSuccess;
    e = e ? e : up(o_parts, T.parts.data(), sizeof(TeamPart) * T.parts.size());
    e = e ? e : up(o_first, T.part_first.data(), 8 * (size_t)R);
    e = e ? e : up(o_fg, T.fib_gid.data(), 4 * T.fib_gid.size());
    e = e ? e : up(o_fe, T.fib_ends.data(), 4 * T.fib_ends.size());
    e = e ? e : up(o_og, T.own_gid.data(), 4 * T.own_gid.size());
    e = e ? e : up(o_ox, T.own_xslot.data(), 4 * T.own_xslot.size());
    e = e ? e : up(o_oi, T.own_inc_off.data(), 8 * T.own_inc_off.size());
    e = e ? e : up(o_oc, T.own_inc.data(), 2 * T.own_inc.size());
    e = e ? e : up(o_hg, T.halo_gid.data(), 4 * T.halo_gid.size());
    e = e ? e : up(o_hx, T.halo_xslot.data(), 4 * T.halo_xslot.size());
    e = e ? e : up(o_bi, T.bnd_inc_off.data(), 8 * T.bnd_inc_off.size());
    e = e ? e : up(o_bc, T.bnd_inc.data(), 2 * T.bnd_inc.size());
    if (e != hipSuccess) return fail(RVE_EDEVICE, std::string("team table upload failed: ") + hipGetErrorString(e));
    TeamArgs& t = b->team_tab;
    t.parts = carve<TeamPart>(m, o_parts);
    t.part_first = carve<int64_t>(m, o_first);
    t.fib_gid = carve<int32_t>(m, o_fg);
    t.fib_ends = carve<uint32_t>(m, o_fe);
    t.own_gid = carve<int32_t>(m, o_og);
    t.own_xslot = carve<int32_t>(m, o_ox);
    t.own_inc_off = carve<int64_t>(m, o_oi);
    t.own_inc = carve<uint16_t>(m, o_oc);
    t.halo_gid = carve<int32_t>(m, o_hg);
    t.halo_xslot = carve<int32_t>(m, o_hx);
    t.bnd_inc_off = carve<int64_t>(m, o_bi);
    t.bnd_inc = carve<uint16_t>(m, o_bc);
    return RVE_OK;
}

// ------------------------------------------------------------------ incidence tables
// Host tables of the incidence engine (layout in rve_internal.h).  An RVE
// gets tables when no free node has more than kIncMaxDeg fibers; it runs the
// LDS form up to kIncMaxNodes free nodes, the global mode above.
struct IncHost {
    std::vector<int64_t> rec_first;     // [R]
    std::vector<int32_t> round_first;   // [R][kIncMaxDeg + 1]
    std::vector<int32_t> perm;          // [NFREE]
    std::vector<uint32_t> rec_fib;
    std::vector<uint2> rec_st;
    std::vector<uint2> brec_st;         // [NBINC]
};

static size_t inc_lds_cap() { return 160 * 1024 - kResStaticLds; }

static bool inc_fits(const HostPack& P, int64_t r)
{
    const int64_t nf = P.free_off[r + 1] - P.free_off[r];
    return nf >= 1 && P.maxdeg[r] <= kIncMaxDeg && (!incidence_lds_mode(nf) || incidence_lds_bytes(nf) <= inc_lds_cap());
}

static uint32_t f32_bits(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    return u;
}

// Tables of RVE r: ranks by descending degree (ties in the packed order),
// then round q lists the q-th incidence of ranks 0 .. P_q - 1.  Each record
// keeps the incidence word (fiber and which end the node is), 1/L0 in FP32
// and the rank of the fiber's other end (nf, the zero slot, for a boundary
// end).  Boundary incidences get the same static part in DevNet::binc order.
static void inc_build(const HostPack& P, int64_t r, IncHost& H)
{
    const int64_t f0 = P.fib_off[r], a0 = P.free_off[r], b0 = P.bnd_off[r];
    const int64_t nf = P.free_off[r + 1] - a0, nb = P.bnd_off[r + 1] - b0;
    auto deg = [&](int64_t a) { return P.inc_off[a0 + a + 1] - P.inc_off[a0 + a]; };
    std::vector<int32_t> order(nf), rank(nf);
    for (int64_t a = 0; a < nf; ++a) order[a] = (int32_t)a;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return deg(x) > deg(y); });
    for (int64_t p = 0; p < nf; ++p) {
        rank[order[p]] = (int32_t)p;
        H.perm[a0 + p] = order[p];
    }
    auto other_rank = [&](uint32_t w) -> uint32_t {
        const uint32_t e = P.ends[f0 + (w & 0x7fffffffu)];
        const int64_t o = (w >> 31) ? (e >> 16) : (e & 0xffffu);   // the node is end i: the other is end j
        return o < nf ? (uint32_t)rank[o] : (uint32_t)nf;
    };
    auto inv_len = [&](uint32_t w) { return f32_bits((float)(1.0 / P.L0[f0 + (w & 0x7fffffffu)])); };
    H.rec_first[r] = (int64_t)H.rec_fib.size();
    int32_t* rf = &H.round_first[(size_t)r * (kIncMaxDeg + 1)];
    int32_t cur = 0;
    for (int q = 0; q < kIncMaxDeg; ++q) {
        rf[q] = cur;
        for (int64_t p = 0; p < nf && deg(order[p]) > q; ++p) {
            const uint32_t w = P.inc[P.inc_off[a0 + order[p]] + q];
            H.rec_fib.push_back(w);
            H.rec_st.push_back(make_uint2(inv_len(w), other_rank(w)));
            ++cur;
        }
    }
    rf[kIncMaxDeg] = cur;
    for (int64_t e = P.binc_off[b0]; e < P.binc_off[b0 + nb]; ++e)
        H.brec_st[e] = make_uint2(inv_len(P.binc[e]), other_rank(P.binc[e]));
}

// want(r): whether RVE r gets tables (every RVE that fits when null).
template <typename Want>
static void inc_build_all(const HostPack& P, int64_t R, IncHost& H, Want want)
{
    H.rec_first.assign(R, -1);
    H.round_first.assign((size_t)R * (kIncMaxDeg + 1), 0);
    H.perm.assign(P.free_off[R], 0);
    H.brec_st.assign(P.binc.size(), make_uint2(0u, 0u));
    for (int64_t r = 0; r < R; ++r)
        if (inc_fits(P, r) && want(r)) inc_build(P, r, H);
}

// Tables for the RVEs AUTO sends to the incidence kernel (those no FP32
// resident build holds), or for every RVE that fits when the batch is
// created with RVE_ENGINE_INCIDENCE: about 56 B per fiber of device memory.
static int build_inc_tables(rve_batch* b, const HostPack& P)
{
    IncHost H;
    const bool all = b->opts.engine == RVE_ENGINE_INCIDENCE;
    try {
        inc_build_all(P, b->R, H, [&](int64_t r) { return all || tier_of(b, r, false) < 0; });
    } catch (const std::bad_alloc&) {
        return fail(RVE_ENOMEM, "host allocation failed while building the incidence tables");
    }
    b->inc_first = H.rec_first;
    if (H.rec_fib.empty()) return RVE_OK;
    const size_t NREC = H.rec_fib.size(), NB = std::max<size_t>(H.brec_st.size(), 1);
    // node-state entries of the global-mode RVEs (nf + 1 each)
    std::vector<int64_t> g_first(b->R, -1);
    size_t NG = 0;
    for (int64_t r = 0; r < b->R; ++r)
        if (H.rec_first[r] >= 0 && !incidence_lds_mode(b->nf_of[r])) {
            g_first[r] = (int64_t)NG;
            NG += (size_t)b->nf_of[r] + 1;
        }
    NG = std::max<size_t>(NG, 1);
    DeviceArena A;
    const size_t o_first = A.reserve(8 * (size_t)b->R), o_round = A.reserve(4 * H.round_first.size()),
                 o_perm = A.reserve(4 * H.perm.size() + 4), o_fib = A.reserve(4 * NREC), o_st = A.reserve(8 * NREC),
                 o_rec = A.reserve(16 * NREC), o_bst = A.reserve(8 * NB), o_brec = A.reserve(16 * NB),
                 o_im = A.reserve(4 * H.perm.size() + 4), o_gf = A.reserve(8 * (size_t)b->R),
                 o_hg = A.reserve(16 * NG), o_vg = A.reserve(16 * NG), o_ag = A.reserve(16 * NG);
    if (hipMalloc((void**)&b->inc_mem, A.used + 256) != hipSuccess) {
        b->inc_mem = nullptr;
        b->inc_first.assign(b->R, -1);
        return fail(RVE_ENOMEM, "device allocation of the incidence tables failed");
    }
    char* m = b->inc_mem;
    auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpy(m + off, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    hipError_t e = hipSuccess;
    e = e ? e : up(o_first, H.rec_first.data(), 8 * (size_t)b->R);
    e = e ? e : up(o_round, H.round_first.data(), 4 * H.round_first.size());
    e = e ? e : up(o_perm, H.perm.data(), 4 * H.perm.size());
    e = e ? e : up(o_fib, H.rec_fib.data(), 4 * NREC);
    e = e ? e : up(o_st, H.rec_st.data(), 8 * NREC);
    e = e ? e : up(o_bst, H.brec_st.data(), 8 * H.brec_st.size());
    e = e ? e : up(o_gf, g_first.data(), 8 * (size_t)b->R);
    if (e != hipSuccess) return fail(RVE_EDEVICE, std::string("incidence table upload failed: ") + hipGetErrorString(e));
    IncArgs& t = b->inc_tab;
    t.rec_first = carve<int64_t>(m, o_first);
    t.round_first = carve<int32_t>(m, o_round);
    t.perm = carve<int32_t>(m, o_perm);
    t.rec_fib = carve<uint32_t>(m, o_fib);
    t.rec_st = carve<uint2>(m, o_st);
    t.rec = carve<float4>(m, o_rec);
    t.brec_st = carve<uint2>(m, o_bst);
    t.brec = carve<float4>(m, o_brec);
    t.imass = carve<float>(m, o_im);
    t.g_first = carve<int64_t>(m, o_gf);
    t.hg = carve<float4>(m, o_hg);
    t.vg = carve<float4>(m, o_vg);
    t.ag = carve<float4>(m, o_ag);
    return RVE_OK;
}

// Team launches: workgroups per CU of the team build at this LDS size, and
// the number of teams (a multiple of 8, so every team lies on one XCD).
static int team_grid(const rve_batch* b, bool fp64, bool kin, size_t lds, int k, int* n_teams)
{
    int per_cu = 0;
    size_t priv = 1;
    HIP_TRY(team_info(fp64, kin, lds, &per_cu, &priv));
    if (priv > 0) return fail(RVE_EDEVICE, "internal: the team kernel build uses private memory");
    const int64_t total = (int64_t)per_cu * b->n_cu;
    *n_teams = (int)(total / (8 * k)) * 8;
    if (*n_teams < 8) return fail(RVE_EDEVICE, "a team of " + std::to_string(k) + " workgroups does not fit the device");
    return RVE_OK;
}

// Work area of the largest team launch of the batch: per team two exchange
// buffers of max_xslots (h, v, a) records and two sets of k partials, then
// the barrier counters, task slots and the error word.
struct TeamWs {
    size_t xchg, partials, words, total;
};
static TeamWs team_ws_layout(const rve_batch* b, int k, int n_teams, int64_t max_xslots, bool fp64)
{
    TeamWs L;
    L.xchg = ((size_t)n_teams * 2 * 9 * (size_t)std::max<int64_t>(max_xslots, 1) * (fp64 ? 8 : 4) + 255) & ~size_t(255);
    L.partials = ((size_t)n_teams * 2 * 8 * (size_t)k * 8 + 255) & ~size_t(255);
    L.words = 4 * (size_t)(3 * n_teams + 1);
    L.total = L.xchg + L.partials + ((L.words + 255) & ~size_t(255));
    return L;
}

// Teams a launch can hold at most (team builds run one workgroup per CU).
static int team_bound(const rve_batch* b, int k) { return 8 * ((b->n_cu + 8 * k - 1) / (8 * k)) + 8; }

// Bytes of the team work area: the largest over every team size the batch's
// partitions use (whichever precision or option puts them on the team
// engine; FP64 records, so either precision fits), after 256 bytes of
// per-group error words.
static size_t team_ws_bytes(const rve_batch* b)
{
    size_t m = 0;
    for (int k = 2; k <= kTeamMax; ++k) {
        int64_t mx = -1;
        for (int64_t r = 0; r < b->R; ++r)
            if (!b->team_k.empty() && b->team_k[r] == k) mx = std::max(mx, b->team_xslots[r]);
        if (mx >= 0) m = std::max(m, team_ws_layout(b, k, team_bound(b, k), mx, true).total);
    }
    return m ? m + 256 : 0;
}

// ------------------------------------------------------------------ index replay
// Host replay of the index arithmetic of the relaxation kernels over a
// packed batch, with every index bounded against the array it addresses.
// Register-resident engine, for every RVE and every resident build whose
// slots hold it: each fiber slot's packed ends (res_pack_ends) against the
// nf + 1 LDS positions, each node slot's register-held incidence codes
// (res_inc_code) and CSR overflow reads against the nfib + 1 LDS forces, the
// code's sign against the incidence, the LDS bytes (dynamic + static)
// against a CU's 160 KB.  Streamed engine: the workspace offsets of every
// fiber, node and zero slot against the workspace sizes.  The packing itself:
// every fiber appears in the incidence of each of its ends with the sign of
// that end.  Incidence engine: the rank permutation, the rounds and every
// record (node, fiber, orientation, other end) of the tables the batch
// builds.  `plant` (tests only) 1 shrinks the LDS position array by one
// entry, 2 corrupts the other-end rank of one incidence record: mistakes the
// replay must report.
static int check_indexing(const rve_net_desc* net, bool fp64, int plant)
{
    HostPack P;
    try {
        pack_batch(net, P);
    } catch (const std::bad_alloc&) {
        return fail(RVE_ENOMEM, "host allocation failed while packing");
    }
    const int64_t R = net->n_rve;
    const int64_t NF = P.fib_off[R], NFREE = P.free_off[R];
    auto bad = [&](int64_t r, const std::string& what) {
        return fail(RVE_EINVAL, "index replay, RVE " + std::to_string(r) + ": " + what);
    };
    IncHost H;
    try {
        inc_build_all(P, R, H, [](int64_t) { return true; });
    } catch (const std::bad_alloc&) {
        return fail(RVE_ENOMEM, "host allocation failed while building the incidence tables");
    }
    if (plant == 2 && !H.rec_st.empty()) H.rec_st[H.rec_st.size() / 2].y ^= 1u;
    // node-state entries of the global-mode RVEs, as build_inc_tables lays them out
    std::vector<int64_t> gfirst(R, -1);
    int64_t gtotal = 0;
    for (int64_t r = 0; r < R; ++r)
        if (H.rec_first[r] >= 0 && !incidence_lds_mode(P.free_off[r + 1] - P.free_off[r])) {
            gfirst[r] = gtotal;
            gtotal += P.free_off[r + 1] - P.free_off[r] + 1;
        }
    for (int64_t r = 0; r < R; ++r) {
        const int64_t f0 = P.fib_off[r], a0 = P.free_off[r], b0 = P.bnd_off[r];
        const int64_t nfib = P.fib_off[r + 1] - f0, nf = P.free_off[r + 1] - a0, nb = P.bnd_off[r + 1] - b0;
        const int64_t nn = nf + nb;
        // packing: incidence of every fiber end, with its sign
        std::vector<int> seen(2 * nfib, 0);
        for (int64_t a = 0; a < nn; ++a) {
            const bool fr = a < nf;
            const int64_t e0 = fr ? P.inc_off[a0 + a] : P.binc_off[b0 + a - nf];
            const int64_t e1 = fr ? P.inc_off[a0 + a + 1] : P.binc_off[b0 + a - nf + 1];
            for (int64_t e = e0; e < e1; ++e) {
                const uint32_t w = fr ? P.inc[e] : P.binc[e];
                const int64_t k = w & 0x7fffffffu;
                if (k >= nfib) return bad(r, "incidence names fiber " + std::to_string(k) + " of " + std::to_string(nfib));
                const uint32_t ends = P.ends[f0 + k];
                const int64_t end = (w >> 31) ? (ends & 0xffffu) : (ends >> 16);
                if (end != a) return bad(r, "incidence of node " + std::to_string(a) + " names a fiber it is not an end of");
                seen[2 * k + ((w >> 31) ? 0 : 1)] += 1;
            }
        }
        for (int64_t q = 0; q < 2 * nfib; ++q)
            if (seen[q] != 1) return bad(r, "fiber " + std::to_string(q / 2) + " end " + std::to_string(q % 2) + " listed " +
                                                std::to_string(seen[q]) + " times");
        // register-resident builds that hold this RVE
        const int64_t h_entries = nf + 1 - (plant == 1 ? 1 : 0);
        const int64_t fv_entries = nfib + 1;
        for (int v = 0; v < kNumResident; ++v) {
            const ResidentVariant& rv = kResident[v];
            if (nfib > (int64_t)rv.threads * rv.sf || nf > (int64_t)rv.threads * rv.sn) continue;
            if (nfib >= kResMaxFibers) continue;   // such RVEs only run streamed (tier_of)
            const size_t dyn = resident_lds_bytes(fp64, nf, nfib, rv.threads);
            if (dyn > 160 * 1024 - 4096) continue;   // tier_of sends these to the streamed engine
            if (dyn + kResStaticLds > 160 * 1024) return bad(r, "LDS of a resident workgroup exceeds 160 KB");
            for (int tid = 0; tid < rv.threads; ++tid) {
                for (int sl = 0; sl < rv.sf; ++sl) {
                    const int64_t k = (int64_t)sl * rv.threads + tid;
                    if (k >= nfib) continue;
                    const uint32_t E = res_pack_ends(P.ends[f0 + k], (uint32_t)nf);
                    if ((int64_t)res_end_i(E) >= h_entries || (int64_t)res_end_j(E) >= h_entries)
                        return bad(r, "build " + std::to_string(v) + ": fiber " + std::to_string(k) +
                                          " reads a position outside the LDS array");
                }
                for (int sl = 0; sl < rv.sn; ++sl) {
                    const int64_t a = (int64_t)sl * rv.threads + tid;
                    if (a >= nf) continue;   // lanes past nf only read the zero slot (padding codes)
                    const int64_t e0 = P.inc_off[a0 + a], deg = P.inc_off[a0 + a + 1] - e0;
                    for (int q = 0; q < kResIncRegs; ++q) {
                        const uint32_t code = q < deg ? res_inc_code(P.inc[e0 + q]) : (uint32_t)nfib;
                        if ((int64_t)res_code_fiber(code) >= fv_entries)
                            return bad(r, "build " + std::to_string(v) + ": node " + std::to_string(a) +
                                              " reads a force outside the LDS array");
                        if (q < deg && res_code_neg(code) != ((P.inc[e0 + q] >> 31) != 0))
                            return bad(r, "incidence code loses the end sign");
                        if (q < deg && (int64_t)res_code_fiber(code) != (int64_t)(P.inc[e0 + q] & 0x7fffffffu))
                            return bad(r, "incidence code loses fiber id bits");
                    }
                    for (int64_t e = e0 + kResIncRegs; e < e0 + deg; ++e)
                        if ((int64_t)(P.inc[e] & 0x7fffffffu) >= fv_entries)
                            return bad(r, "overflow incidence reads a force outside the LDS array");
                }
            }
            if (nfib > 0x7fff) return bad(r, "the zero force slot does not fit the 15-bit code");
        }
        // streamed engine: workspace entries [NF + R] per fiber array, [NFREE + R] positions
        if (f0 + r + nfib >= NF + R) return bad(r, "streamed fiber zero slot outside the workspace");
        if (a0 + r + nf >= NFREE + R) return bad(r, "streamed position zero slot outside the workspace");
        // incidence engine: ranks, rounds and records against the node slots,
        // the LDS positions (nf + 1) and the record arrays; each record names
        // its node's fiber, the node as the end its sign says, and the rank of
        // the other end (the zero slot nf for a boundary end)
        if (H.rec_first[r] >= 0) {
            const int64_t rb0 = H.rec_first[r];
            const int32_t* rf = &H.round_first[(size_t)r * (kIncMaxDeg + 1)];
            if (incidence_lds_mode(nf)) {
                for (int v = 0; v < kNumInc; ++v)
                    if ((int64_t)kInc[v].threads * kInc[v].slots < nf) return bad(r, "incidence: node slots below nf");
                if (incidence_lds_bytes(nf) + kResStaticLds > 160 * 1024) return bad(r, "incidence: LDS beyond 160 KB");
            } else if (gfirst[r] < 0 || gfirst[r] + nf >= gtotal) {
                return bad(r, "incidence (global mode): zero slot outside the node-state arrays");
            }
            std::vector<int> hit(nf, 0);
            for (int64_t p = 0; p < nf; ++p) {
                const int32_t a = H.perm[a0 + p];
                if (a < 0 || a >= nf || hit[a]++) return bad(r, "incidence: ranks are not a permutation");
            }
            if (rf[0] != 0) return bad(r, "incidence: round 0 does not start the records");
            int64_t count = 0;
            for (int q = 0; q < kIncMaxDeg; ++q) {
                const int64_t Pq = rf[q + 1] - rf[q];
                if (Pq < 0 || Pq > nf || (q > 0 && Pq > rf[q] - rf[q - 1]))
                    return bad(r, "incidence: rounds are not shrinking prefixes of the ranks");
                for (int64_t p = 0; p < Pq; ++p) {
                    const int64_t j = rb0 + rf[q] + p;
                    if (j < 0 || j >= (int64_t)H.rec_fib.size()) return bad(r, "incidence: record outside the arrays");
                    const int32_t a = H.perm[a0 + p];
                    const int64_t deg = P.inc_off[a0 + a + 1] - P.inc_off[a0 + a];
                    if (deg <= q || H.rec_fib[j] != P.inc[P.inc_off[a0 + a] + q])
                        return bad(r, "incidence: record is not the node's incidence of its round");
                    const uint32_t w = H.rec_fib[j], e = P.ends[f0 + (w & 0x7fffffffu)];
                    if ((int64_t)(w & 0x7fffffffu) >= nfib) return bad(r, "incidence: fiber outside the RVE");
                    const int64_t self = (w >> 31) ? (e & 0xffffu) : (e >> 16);
                    const int64_t other = (w >> 31) ? (e >> 16) : (e & 0xffffu);
                    if (self != a) return bad(r, "incidence: record oriented from another node");
                    const uint32_t o = H.rec_st[j].y;
                    if (o > (uint32_t)nf || (other < nf ? (o == (uint32_t)nf || H.perm[a0 + o] != other) : o != (uint32_t)nf))
                        return bad(r, "incidence: record names a wrong other end");
                    ++count;
                }
            }
            if (count != P.inc_off[a0 + nf] - P.inc_off[a0] || rf[kIncMaxDeg] != count)
                return bad(r, "incidence: rounds do not hold every incidence once");
            for (int64_t e = P.binc_off[b0]; e < P.binc_off[b0 + nb]; ++e) {
                const uint32_t w = P.binc[e], ee = P.ends[f0 + (w & 0x7fffffffu)];
                const int64_t other = (w >> 31) ? (ee >> 16) : (ee & 0xffffu);
                const uint32_t o = H.brec_st[e].y;
                if (o > (uint32_t)nf || (other < nf ? (o == (uint32_t)nf || H.perm[a0 + o] != other) : o != (uint32_t)nf))
                    return bad(r, "incidence: boundary record names a wrong other end");
            }
        }
        // team engine: the partition of an RVE no FP64 resident build holds
        const int cap_f = kTeamUnit[0].threads * kTeamUnit[0].sf, cap_n = kTeamUnit[0].threads * kTeamUnit[0].sn;
        if (nfib <= cap_f && nf <= cap_n) continue;
        TeamHost T;
        T.part_first.assign(R, -1);
        T.own_inc_off.assign(1, 0);
        T.bnd_inc_off.assign(1, 0);
        int k = 0;
        int64_t xs = 0;
        size_t lds[2];
        for (int kk = 2; kk <= kTeamMax && !k; ++kk)
            if (team_partition(P, r, kk, T, &xs, lds)) k = kk;
            else {
                T = TeamHost();
                T.part_first.assign(R, -1);
                T.own_inc_off.assign(1, 0);
                T.bnd_inc_off.assign(1, 0);
            }
        if (!k) continue;   // runs streamed
        std::vector<int> owner(nf, -1), owned_seen(nf, 0);
        std::vector<int32_t> slot_of(nf, -1);
        for (int p = 0; p < k; ++p) {
            const TeamPart& tp = T.parts[p];
            for (int32_t a = 0; a < tp.nown; ++a) {
                const int64_t g = T.own_gid[tp.own0 + a] - a0;
                if (g < 0 || g >= nf) return bad(r, "team: owned node outside the RVE");
                owner[g] = p;
                owned_seen[g] += 1;
                slot_of[g] = T.own_xslot[tp.own0 + a];
            }
        }
        for (int64_t a = 0; a < nf; ++a)
            if (owned_seen[a] != 1) return bad(r, "team: free node " + std::to_string(a) + " owned " +
                                                       std::to_string(owned_seen[a]) + " times");
        for (int p = 0; p < k; ++p) {
            const TeamPart& tp = T.parts[p];
            const int zs = tp.nown + tp.nhalo;
            const int cap_fib = kTeamUnit[fp64 ? 1 : 0].threads * kTeamUnit[fp64 ? 1 : 0].sf;
            const int cap_own = kTeamUnit[fp64 ? 1 : 0].threads * kTeamUnit[fp64 ? 1 : 0].sn;
            if (tp.nfib > cap_fib || tp.nown > cap_own) return bad(r, "team: a part exceeds the build's slots");
            if (team_lds_bytes(fp64, zs, tp.nfib) + 4096 > 160 * 1024) return bad(r, "team: part LDS beyond 160 KB");
            std::vector<int> has(nfib, 0);
            for (int32_t q = 0; q < tp.nfib; ++q) {
                const int64_t g = T.fib_gid[tp.fib0 + q] - f0;
                if (g < 0 || g >= nfib) return bad(r, "team: fiber outside the RVE");
                has[g] = 1;
                const uint32_t E = T.fib_ends[tp.fib0 + q];
                if ((int)res_end_i(E) > zs || (int)res_end_j(E) > zs)
                    return bad(r, "team: fiber end outside the part's position slots");
                // local ends name the fiber's true ends
                const uint32_t e = P.ends[f0 + g];
                for (int end = 0; end < 2; ++end) {
                    const int64_t id = end ? (e >> 16) : (e & 0xffffu);
                    const int loc = (int)(end ? res_end_j(E) : res_end_i(E));
                    int64_t back = -1;
                    if (loc < tp.nown) back = T.own_gid[tp.own0 + loc] - a0;
                    else if (loc < zs) back = T.halo_gid[tp.halo0 + (loc - tp.nown)] - a0;
                    if (id < nf ? back != id : loc != zs) return bad(r, "team: a fiber end maps to another node");
                }
            }
            for (int32_t a = 0; a < tp.nown; ++a) {
                const int64_t g = T.own_gid[tp.own0 + a] - a0;
                for (int64_t e = P.inc_off[a0 + g]; e < P.inc_off[a0 + g + 1]; ++e)
                    if (!has[P.inc[e] & 0x7fffffffu]) return bad(r, "team: an owned node's fiber is not in its part");
                const int64_t e0 = T.own_inc_off[tp.own0 + a], e1 = T.own_inc_off[tp.own0 + a + 1];
                if (e1 - e0 != P.inc_off[a0 + g + 1] - P.inc_off[a0 + g]) return bad(r, "team: owned degree differs");
                for (int64_t e = e0; e < e1; ++e) {
                    const uint32_t c = T.own_inc[e];
                    if ((int)res_code_fiber(c) >= tp.nfib) return bad(r, "team: incidence code outside the part's fibers");
                    const int64_t g2 = T.fib_gid[tp.fib0 + res_code_fiber(c)] - f0;
                    const uint32_t ee = P.ends[f0 + g2];
                    const int64_t end = res_code_neg(c) ? (ee & 0xffffu) : (ee >> 16);
                    if (end != g) return bad(r, "team: incidence code names a fiber of another node or end");
                }
            }
            for (int32_t q = 0; q < tp.nhalo; ++q) {
                const int64_t g = T.halo_gid[tp.halo0 + q] - a0;
                if (g < 0 || g >= nf || owner[g] == p) return bad(r, "team: halo node is not foreign");
                const int32_t x = T.halo_xslot[tp.halo0 + q];
                if (x < 0 || x >= xs || x != slot_of[g]) return bad(r, "team: halo slot differs from its owner's");
            }
            for (int32_t q = 0; q < tp.nbnd; ++q)
                for (int64_t e = T.bnd_inc_off[tp.bnd0 + q]; e < T.bnd_inc_off[tp.bnd0 + q + 1]; ++e)
                    if ((int)res_code_fiber(T.bnd_inc[e]) >= tp.nfib)
                        return bad(r, "team: boundary code outside the part's fibers");
        }
    }
    return RVE_OK;
}


// Assign every RVE to an engine/variant group, longest-first inside a group.
// Resident variants are chosen per size tier: the autotuner's choice if one
// exists, else, among the builds without private memory that hold the tier,
// the one that places the most workgroups (RVEs) on a compute unit at the
// tier's largest LDS footprint, then the one of smallest capacity, then more
// threads.  Several RVEs per CU overlap one RVE's barrier waits with the
// others' arithmetic: on 512 RVEs of at most 2048 fibers, two 512-thread
// workgroups per CU relax 1.47x the fiber-iterations per second of one
// 1024-thread workgroup.
static int default_variant(const rve_batch* b, int tier, bool fp64)
{
    const int T = b->opts.threads_per_rve;
    const bool kin = kinetic_mode(b->opts);
    const auto caps = tier_caps();
    const size_t lds = resident_lds_bytes(fp64, caps[tier].second, caps[tier].first, 0);
    int chosen = -1, best_blocks = 0;
    int64_t best = 0;
    for (int v = 0; v < kNumResident; ++v) {
        const ResidentVariant& rv = kResident[v];
        if (T && rv.threads != T) continue;
        if (spills(b, v, fp64)) continue;   // never launched
        if (!variant_fits_tier(v, tier)) continue;
        int per_cu = 0;
        if (max_resident_blocks(v, fp64, kin, lds, &per_cu) != hipSuccess || per_cu < 1) continue;
        const int64_t key = (int64_t)rv.threads * rv.sf * 4096 - rv.threads;
        if (chosen < 0 || per_cu > best_blocks || (per_cu == best_blocks && key < best)) {
            chosen = v;
            best = key;
            best_blocks = per_cu;
        }
    }
    return chosen;
}

// Incidence build for the batch's options: the first of kInc without
// private memory (of threads_per_rve threads when that is set), -1 when
// none or the options rule the engine out.
static bool inc_options(const rve_batch* b)
{
    return b->opts.precision == RVE_MIXED && b->opts.damping != RVE_DAMP_ADAPTIVE && !b->opts.energy_check &&
           b->opts.engine != RVE_ENGINE_STREAMED && b->opts.engine != RVE_ENGINE_NAIVE && !b->inc_first.empty();
}

static int inc_variant(const rve_batch* b)
{
    if (!inc_options(b)) return -1;
    const int k = b->opts.damping == RVE_DAMP_KINETIC ? 1 : 0;
    for (int v = 0; v < kNumInc; ++v)
        if (!b->inc_private[k][v] && (!b->opts.threads_per_rve || b->opts.threads_per_rve == kInc[v].threads))
            return v;
    return -1;
}

// whether the global-mode build may run for the batch's options
static bool incg_ok(const rve_batch* b)
{
    return inc_options(b) && !b->incg_private[b->opts.damping == RVE_DAMP_KINETIC ? 1 : 0] &&
           (!b->opts.threads_per_rve || b->opts.threads_per_rve == kIncGlobalThreads);
}

// whether RVE r can take the incidence engine (its tables exist and the
// build of its form may run)
static bool inc_rve(const rve_batch* b, int64_t r)
{
    if (b->inc_first.empty() || b->inc_first[r] < 0) return false;
    return incidence_lds_mode(b->nf_of[r]) ? inc_variant(b) >= 0 : incg_ok(b);
}

static void assign_groups(rve_batch* b)
{
    b->groups.clear();
    b->group_variant.clear();
    b->group_lds.clear();
    b->group_team.clear();
    const bool fp64 = b->opts.precision == RVE_FP64;
    // [resident variants..., streamed, teams of 2..kTeamMax, incidence]
    const int inc_slot = kNumResident + kTeamMax + 1, incg_slot = inc_slot + 1;
    std::vector<std::vector<int32_t>> per(incg_slot + 1);
    const int eng = b->opts.engine;
    for (int64_t r = 0; r < b->R; ++r) {
        int slot = kNumResident;   // streamed
        const bool inc = inc_rve(b, r);
        const int islot = incidence_lds_mode(b->nf_of[r]) ? inc_slot : incg_slot;
        if (eng == RVE_ENGINE_INCIDENCE && inc) {
            slot = islot;
        } else if (eng == RVE_ENGINE_AUTO || eng == RVE_ENGINE_TEAM || eng == RVE_ENGINE_INCIDENCE) {
            int t = tier_of(b, r, fp64);
            int chosen = -1;
            if (t >= 0) {
                int tv = b->tuned[fp64 ? 1 : 0][t];
                if (tv >= 0 && spills(b, tv, fp64)) tv = -2;   // tuned for the other damping build
                chosen = (tv != -2 && !b->opts.threads_per_rve) ? tv : default_variant(b, t, fp64);
            }
            // the autotuner's team choice was measured against the streamed
            // kernel: it applies to the RVEs the incidence kernel does not take
            const int k = b->team_k.empty() ? 0 : b->team_k[r];
            const bool team = k > 0 && !b->opts.threads_per_rve &&
                              (eng == RVE_ENGINE_TEAM || (b->tuned_team[fp64 ? 1 : 0][k] == 1 && !inc));
            if (chosen >= 0)
                slot = chosen;
            else if (team)
                slot = kNumResident + k;
            else if (inc)
                slot = islot;
        }
        per[slot].push_back((int32_t)r);
    }
    for (size_t v = 0; v < per.size(); ++v) {
        std::vector<int32_t>& members = per[v];
        if (members.empty()) continue;
        std::stable_sort(members.begin(), members.end(),
                         [&](int32_t a, int32_t c) { return b->nfib_of[a] > b->nfib_of[c]; });
        size_t lds = 0;
        int team = 0, code = kStreamedGroup;
        if (v < (size_t)kNumResident) {
            for (int32_t r : members) lds = std::max(lds, resident_lds_bytes(fp64, b->nf_of[r], b->nfib_of[r], 0));
            code = (int)v;
        } else if (v == (size_t)inc_slot) {
            for (int32_t r : members) lds = std::max(lds, incidence_lds_bytes(b->nf_of[r]));
            code = kIncGroup;
        } else if (v == (size_t)incg_slot) {
            code = kIncGlobalGroup;
        } else if (v > (size_t)kNumResident) {
            team = (int)(v - kNumResident);
            for (int32_t r : members) lds = std::max(lds, b->team_lds[fp64 ? 1 : 0][r]);
            code = -1 - team;
        }
        b->groups.push_back(members);
        b->group_variant.push_back(code);
        b->group_lds.push_back(lds);
        b->group_team.push_back(team);
    }
}

static int upload_groups(rve_batch* b)
{
    std::vector<int32_t> flat;
    b->group_first.clear();
    for (auto& g : b->groups) {
        b->group_first.push_back((int32_t)flat.size());
        flat.insert(flat.end(), g.begin(), g.end());
    }
    if (!flat.empty()) HIP_TRY(hipMemcpy(b->dlist, flat.data(), flat.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    return RVE_OK;
}

// Streamed engine: entries per component of the LDS copy of h for a launch
// over `rves`: the largest nf + 1 that fits the LDS budget (RVEs above it keep
// h in the workspace), 0 when none fits; and workgroups per CU.
static int64_t streamed_lds_nodes(const rve_batch* b, const int32_t* rves, size_t n, bool fp64)
{
    int64_t m = 0;
    for (size_t q = 0; q < n; ++q) {
        const int64_t need = b->nf_of[rves[q]] + 1;
        if (3 * (fp64 ? 8 : 4) * (size_t)need <= streamed_lds_cap()) m = std::max<int64_t>(m, need);
    }
    return m;
}

static int streamed_blocks_per_cu(int threads, int64_t lds_nodes, bool fp64)
{
    const int base = threads == 256 ? 4 : 2;
    if (lds_nodes <= 0) return base;
    const size_t lds = 3 * (fp64 ? 8 : 4) * (size_t)lds_nodes + 1024;
    return (int)std::max<size_t>(1, std::min<size_t>(base, (160 * 1024) / lds));
}

// Workgroup size of the streamed engine: 1024 threads unless 256 are asked
// for or the 1024-thread build of this precision and damping uses private
// memory (the FP64 builds do); 0 when neither build may be launched.
static int streamed_threads(const rve_batch* b, bool fp64)
{
    const int k = kinetic_mode(b->opts) ? 1 : 0, p = fp64 ? 1 : 0;
    if (b->opts.threads_per_rve != 256 && !b->streamed_private[k][p][1]) return 1024;
    return b->streamed_private[k][p][0] ? 0 : 256;
}

static int ensure_workspace(rve_batch* b)
{
    const size_t tw = team_ws_bytes(b);
    if (tw > b->team_ws_bytes) {
        if (b->ws_user) return fail(RVE_EWORKSPACE, "internal: bound workspace smaller than the team work area");
        if (b->team_ws) (void)hipFree(b->team_ws);
        b->team_ws = nullptr;
        b->team_ws_bytes = 0;
        if (hipMalloc((void**)&b->team_ws, tw) != hipSuccess) return fail(RVE_ENOMEM, "team work area allocation failed");
        b->team_ws_bytes = tw;
    }
    bool need = false;
    for (int v : b->group_variant) need |= (v == -1);
    if (!need) return RVE_OK;
    const size_t r4 = b->opts.precision == RVE_FP64 ? 32 : 16;
    size_t fb = r4 * 3 * (size_t)(b->NF + b->R);
    size_t nb = r4 * (2 * (size_t)(b->NFREE + b->R) + 2 * (size_t)b->NFREE + 1);
    if ((fb > b->ws_fib_bytes || nb > b->ws_node_bytes) && b->ws_user)
        return fail(RVE_EWORKSPACE, "internal: bound workspace smaller than the streamed workspace");
    if (fb > b->ws_fib_bytes) {
        if (b->ws_fib) (void)hipFree(b->ws_fib);
        b->ws_fib = nullptr;
        b->ws_fib_bytes = 0;
        if (hipMalloc(&b->ws_fib, fb) != hipSuccess) return fail(RVE_ENOMEM, "workspace allocation failed");
        b->ws_fib_bytes = fb;
    }
    if (nb > b->ws_node_bytes) {
        if (b->ws_node) (void)hipFree(b->ws_node);
        b->ws_node = nullptr;
        b->ws_node_bytes = 0;
        if (hipMalloc(&b->ws_node, nb) != hipSuccess) return fail(RVE_ENOMEM, "workspace allocation failed");
        b->ws_node_bytes = nb;
    }
    return RVE_OK;
}

int rve_naive_run(const SolveArgs& A, const std::vector<int64_t>& fib_off, const std::vector<int64_t>& free_off,
                  const std::vector<int64_t>& bnd_off, const std::vector<double>& F, const std::vector<double>& c,
                  hipStream_t s, std::string* err);

namespace rve {
hipError_t fixed_kernels_scratch_bytes(size_t* bytes)
{
    size_t m = 0;
    for (auto fn : {kernels_fixed_private, naive_fixed_private, orient_fixed_private, state_fixed_private,
                    tangent_fixed_private, variant_fixed_private, fd_fixed_private}) {
        size_t b = 0;
        const hipError_t e = fn(&b);
        if (e != hipSuccess) return e;
        m = std::max(m, b);
    }
    *bytes = m;
    return hipSuccess;
}
}  // namespace rve

// ------------------------------------------------------------------ ABI
extern "C" {

int rve_version(void) { return RVE_API_VERSION; }

const char* rve_last_error(void) { return g_last_error.c_str(); }

void rve_default_opts(rve_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = RVE_FP64;
    o->law = RVE_LAW_LINEAR;
    o->mass = RVE_MASS_LUMPED;
    o->init = RVE_INIT_AFFINE;
    o->EA = 1.0;
    o->B = 10.0;
    o->rhoA = 1.0;
    o->alpha = 0.9;
    o->c = 2.0;
    o->tol_abs = 1e-10;
    o->tol_rel = 0.0;
    o->n_max = 1000000;
    o->check_every = 1;
    o->engine = RVE_ENGINE_AUTO;
    o->cg_tol = 1e-6;
    o->cg_max_iter = 0;
    o->damping = RVE_DAMP_VISCOUS;
    o->energy_check = 0;
    o->energy_tol = 0.05;
    o->floor_tol_rel = 0.0;
    o->stall_checks = 16;
    o->tangent_rhs = 0;
    o->work_order = RVE_ORDER_AUTO;
}

// Address of the allocation-free solve's scratch array on device dev, taken
// once per device (definition at the end of this file).
static int device_scratch(int dev, void** out);

int rve_check_indexing(const rve_net_desc* net, int32_t precision, int32_t plant)
{
    int rc = validate_net(net);
    if (rc) return rc;
    if (precision != RVE_FP64 && precision != RVE_MIXED) return fail(RVE_EINVAL, "bad precision");
    return check_indexing(net, precision == RVE_FP64, plant);
}

int rve_batch_create(const rve_net_desc* net, const rve_opts* opts, rve_batch** out)
{
    if (!out) return fail(RVE_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_net(net);
    if (rc) return rc;
    rc = validate_opts(opts, net->n_rve);
    if (rc) return rc;

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(RVE_EDEVICE, "no HIP device");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(RVE_EDEVICE, std::string("device is ") + prop.gcnArchName + ", the kernels are built for gfx950");

    {
        // set-up of the allocation-free solve: the device copy of its scratch
        // array is located (and so made resident) once per device, here
        void* sp = nullptr;
        int rc_s = device_scratch(dev, &sp);
        if (rc_s) return rc_s;
    }
    rve_batch* b = new (std::nothrow) rve_batch();
    if (!b) return fail(RVE_ENOMEM, "host allocation failed");
    b->device = dev;
    b->n_cu = prop.multiProcessorCount;
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k <= kTeamMax; ++k) b->tuned_team[p][k] = -1;
    // Admission: a kernel build that uses private (scratch) memory is never
    // launched.  Every GPU fault and wrong result seen while developing these
    // kernels came from builds at or over their register budget, so the rule
    // is strict: any private segment at all (spilled registers, stack arrays)
    // excludes the build; the RVEs it would take go to the next build that
    // holds them, else to the streamed kernel.
    for (int k = 0; k < 2; ++k)
        for (int p = 0; p < 2; ++p) {
            for (int v = 0; v < kNumResident; ++v) {
                size_t sb = 1;
                if (resident_scratch_bytes(v, p == 1, k == 1, &sb) != hipSuccess) sb = 1;
                b->variant_spills[k][p][v] = sb > 0;
            }
            for (int w = 0; w < 2; ++w) {
                size_t sb = 1;
                if (streamed_scratch_bytes(p == 1, k == 1, w ? 1024 : 256, &sb) != hipSuccess) sb = 1;
                b->streamed_private[k][p][w] = sb > 0;
            }
        }
    for (int k = 0; k < 2; ++k) {
        for (int v = 0; v < kNumInc; ++v) {
            size_t sb = 1;
            if (incidence_scratch_bytes(v, k == 1, &sb) != hipSuccess) sb = 1;
            b->inc_private[k][v] = sb > 0;
        }
        size_t sb = 1;
        if (incidence_global_scratch_bytes(k == 1, &sb) != hipSuccess) sb = 1;
        b->incg_private[k] = sb > 0;
    }
    for (int m = 0; m < 2; ++m)
        for (int v = 0; v < kNumTanRes; ++v) {
            size_t sb = 1;
            if (tangent_res_scratch_bytes(v, m == 1, &sb) != hipSuccess) sb = 1;
            b->tangent_private[m][v] = sb > 0;
        }
    for (int v = 0; v < kNumTanBlk; ++v) {
        size_t sb = 1;
        if (tangent_blk_scratch_bytes(v, &sb) != hipSuccess) sb = 1;
        b->tangent_blk_private[v] = sb > 0;
    }
    {
        size_t sb = 1;
        if (fixed_kernels_scratch_bytes(&sb) != hipSuccess || sb > 0) {
            delete b;
            return fail(RVE_EDEVICE, "internal: a fixed kernel of the library uses private memory");
        }
    }
    b->R = net->n_rve;
    b->opts = *opts;
    b->c_host.assign(b->R, opts->c);
    if (opts->c_per_rve) std::copy(opts->c_per_rve, opts->c_per_rve + b->R, b->c_host.begin());
    b->opts.c_per_rve = nullptr;

    HostPack P;
    try {
        pack_batch(net, P);
    } catch (const std::bad_alloc&) {
        delete b;
        return fail(RVE_ENOMEM, "host allocation failed while packing");
    }
    const int64_t R = b->R;
    b->NN = R ? net->node_off[R] : 0;
    b->NF = R ? net->fib_off[R] : 0;
    b->NFREE = P.free_off[R];
    b->NBND = P.bnd_off[R];
    b->node_off.assign(net->node_off, net->node_off + R + 1);
    b->fib_off = P.fib_off;
    b->free_off = P.free_off;
    b->bnd_off = P.bnd_off;
    b->newid = P.newid;
    b->nf_of = P.nf;
    b->nfib_of = P.nfib;
    b->maxdeg_of = P.maxdeg;
    b->chunk_first.assign(1, 0);
    b->chunk_rec.assign(1, 0);
    for (int64_t r = 0; r < R; ++r) {
        const int64_t a0 = P.free_off[r], nf = P.free_off[r + 1] - a0;
        for (int64_t c0 = 0; c0 < nf; c0 += 64) {
            int64_t w = 0;
            for (int64_t a = c0; a < std::min<int64_t>(c0 + 64, nf); ++a)
                w = std::max<int64_t>(w, P.inc_off[a0 + a + 1] - P.inc_off[a0 + a]);
            w = (w + 3) & ~int64_t(3);   // whole groups of 4 records per lane
            b->chunk_rec.push_back(b->chunk_rec.back() + 64 * w);
        }
        b->chunk_first.push_back((int64_t)b->chunk_rec.size() - 1);
    }
    b->Xm.resize(3 * b->NN);
    for (int64_t p = 0; p < 3 * b->NN; ++p) b->Xm[p] = net->X[p] - 0.5;

    // one device allocation for the network, per-RVE inputs/outputs and state
    DeviceArena A;
    size_t o_fib_off = A.reserve(8 * (R + 1)), o_free_off = A.reserve(8 * (R + 1)), o_bnd_off = A.reserve(8 * (R + 1));
    size_t o_d0 = A.reserve(24 * b->NF), o_L0 = A.reserve(8 * b->NF), o_ends = A.reserve(4 * b->NF);
    size_t o_mass = A.reserve(8 * b->NFREE), o_inc_off = A.reserve(8 * (b->NFREE + 1)),
           o_inc = A.reserve(4 * P.inc.size() + 4);
    size_t o_binc_off = A.reserve(8 * (b->NBND + 1)), o_binc = A.reserve(4 * P.binc.size() + 4);
    size_t o_Xb = A.reserve(24 * b->NBND), o_V0 = A.reserve(8 * R);
    size_t o_F = A.reserve(72 * R), o_c = A.reserve(8 * R), o_sig = A.reserve(72 * R), o_R = A.reserve(8 * R),
           o_D = A.reserve(8 * R), o_B = A.reserve(8 * R), o_h = A.reserve(24 * b->NFREE + 8),
           o_st = A.reserve(4 * R), o_it = A.reserve(8 * R), o_q = A.reserve(256), o_list = A.reserve(4 * R + 4);
    if (hipMalloc(&b->dmem, A.used + 256) != hipSuccess) {
        delete b;
        return fail(RVE_ENOMEM, "device allocation of " + std::to_string(A.used) + " bytes failed");
    }
    char* m = b->dmem;
    auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpy(m + off, src, bytes, hipMemcpyHostToDevice);
    };
    std::vector<double> V0(R, 1.0);
    if (net->V0) std::copy(net->V0, net->V0 + R, V0.begin());
    hipError_t e = hipSuccess;
    e = e ? e : up(o_fib_off, P.fib_off.data(), 8 * (R + 1));
    e = e ? e : up(o_free_off, P.free_off.data(), 8 * (R + 1));
    e = e ? e : up(o_bnd_off, P.bnd_off.data(), 8 * (R + 1));
    e = e ? e : up(o_d0, P.d0.data(), 24 * b->NF);
    e = e ? e : up(o_L0, P.L0.data(), 8 * b->NF);
    e = e ? e : up(o_ends, P.ends.data(), 4 * b->NF);
    e = e ? e : up(o_mass, P.mass.data(), 8 * b->NFREE);
    e = e ? e : up(o_inc_off, P.inc_off.data(), 8 * (b->NFREE + 1));
    e = e ? e : up(o_inc, P.inc.data(), 4 * P.inc.size());
    e = e ? e : up(o_binc_off, P.binc_off.data(), 8 * (b->NBND + 1));
    e = e ? e : up(o_binc, P.binc.data(), 4 * P.binc.size());
    e = e ? e : up(o_Xb, P.Xb.data(), 24 * b->NBND);
    e = e ? e : up(o_V0, V0.data(), 8 * R);
    e = e ? e : up(o_c, b->c_host.data(), 8 * R);
    e = e ? e : hipMemset(m + o_h, 0, 24 * b->NFREE + 8);
    if (e != hipSuccess) {
        (void)hipFree(b->dmem);
        delete b;
        return fail(RVE_EDEVICE, std::string("upload failed: ") + hipGetErrorString(e));
    }
    DevNet& n = b->net;
    n.n_rve = R;
    n.fib_off = carve<int64_t>(m, o_fib_off);
    n.free_off = carve<int64_t>(m, o_free_off);
    n.bnd_off = carve<int64_t>(m, o_bnd_off);
    n.d0 = carve<double>(m, o_d0);
    n.L0 = carve<double>(m, o_L0);
    n.ends = carve<uint32_t>(m, o_ends);
    n.mass = carve<double>(m, o_mass);
    n.inc_off = carve<int64_t>(m, o_inc_off);
    n.inc = carve<uint32_t>(m, o_inc);
    n.binc_off = carve<int64_t>(m, o_binc_off);
    n.binc = carve<uint32_t>(m, o_binc);
    n.Xb = carve<double>(m, o_Xb);
    n.V0 = carve<double>(m, o_V0);
    b->dV0 = carve<double>(m, o_V0);
    b->dF = carve<double>(m, o_F);
    b->dc = carve<double>(m, o_c);
    b->dsigma = carve<double>(m, o_sig);
    b->dR = carve<double>(m, o_R);
    b->dD = carve<double>(m, o_D);
    b->dB = carve<double>(m, o_B);
    b->dh = carve<double>(m, o_h);
    b->dstatus = carve<int32_t>(m, o_st);
    b->diters = carve<int64_t>(m, o_it);
    b->dqueue = carve<int32_t>(m, o_q);
    b->dlist = carve<int32_t>(m, o_list);

    rc = build_team_tables(b, P);
    if (!rc) rc = build_inc_tables(b, P);
    if (rc) {
        rve_batch_destroy(b);
        return rc;
    }
    assign_groups(b);
    rc = upload_groups(b);
    if (rc) {
        rve_batch_destroy(b);
        return rc;
    }
    *out = b;
    return RVE_OK;
}

int rve_batch_set_opts(rve_batch* b, const rve_opts* opts)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    int rc = validate_opts(opts, b->R);
    if (rc) return rc;
    b->opts = *opts;
    b->c_host.assign(b->R, opts->c);
    if (opts->c_per_rve) std::copy(opts->c_per_rve, opts->c_per_rve + b->R, b->c_host.begin());
    b->opts.c_per_rve = nullptr;
    if (b->R) HIP_TRY(hipMemcpy(b->dc, b->c_host.data(), 8 * b->R, hipMemcpyHostToDevice));
    ++b->generation;
    assign_groups(b);
    return upload_groups(b);
}

int rve_batch_team_spin_limit(rve_batch* b, int64_t polls)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    if (polls < 1) return fail(RVE_EINVAL, "the spin limit must be at least 1 poll");
    b->team_spin_limit = polls;
    return RVE_OK;
}

int rve_batch_generation(const rve_batch* b, uint64_t* gen)
{
    if (!b || !gen) return fail(RVE_EINVAL, "NULL argument");
    *gen = b->generation;
    return RVE_OK;
}

int rve_batch_set_stream(rve_batch* b, void* stream)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    b->opts.stream = stream;
    return RVE_OK;
}

int rve_batch_profile(rve_batch* b, int enable)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    b->profile = enable != 0;
    return RVE_OK;
}

int rve_batch_kernel_ms(rve_batch* b, double* relax_ms, double* stress_ms)
{
    if (!b || !relax_ms || !stress_ms) return fail(RVE_EINVAL, "NULL argument");
    if (b->ev_used < 2) return fail(RVE_ESTATE, "no profiled solve");
    HIP_TRY(hipEventSynchronize(b->ev[b->ev_used - 1]));
    // relaxation span: from the earliest group start to the join of all
    // groups (the groups may run concurrently on several streams)
    double relax = 0.0;
    for (int g = 0; g + 2 < b->ev_used; g += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, b->ev[g], b->ev[b->ev_used - 2]));
        relax = std::max(relax, (double)ms);
    }
    float st = 0.f;
    HIP_TRY(hipEventElapsedTime(&st, b->ev[b->ev_used - 2], b->ev[b->ev_used - 1]));
    *relax_ms = relax;
    *stress_ms = st;
    return RVE_OK;
}

int rve_batch_groups(rve_batch* b, int32_t* group_of_rve, int32_t* variant, double* ms, int32_t max_groups,
                     int32_t* n_groups)
{
    if (!b || !n_groups) return fail(RVE_EINVAL, "NULL argument");
    const int G = (int)b->groups.size();
    *n_groups = G;
    if (group_of_rve)
        for (int g = 0; g < G; ++g)
            for (int32_t r : b->groups[g]) group_of_rve[r] = g;
    const bool timed = b->ev_used == 2 * G + 2;
    for (int g = 0; g < G && g < max_groups; ++g) {
        if (variant) variant[g] = b->group_variant[g];
        if (ms) {
            float t = NAN;
            if (timed) {
                HIP_TRY(hipEventSynchronize(b->ev[2 * g + 1]));
                HIP_TRY(hipEventElapsedTime(&t, b->ev[2 * g], b->ev[2 * g + 1]));
            }
            ms[g] = t;
        }
    }
    return RVE_OK;
}

int rve_batch_sizes(const rve_batch* b, int64_t* n_rve, int64_t* n_nodes, int64_t* n_fib)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    if (n_rve) *n_rve = b->R;
    if (n_nodes) *n_nodes = b->NN;
    if (n_fib) *n_fib = b->NF;
    return RVE_OK;
}


// The relaxation launches of a solve on the resident, team and streamed
// engines: one persistent launch per kernel group (work counters queues[2 g]),
// then the stress kernel; with `profile`, HIP events around each launch.
// team_ws: the team work area (error words first, one per group, cleared
// here; then the work area of one team launch, reused by the next).
static int launch_groups(rve_batch* b, SolveArgs& a, int32_t* queues, void* ws_fib, void* ws_node, char* team_ws,
                         hipStream_t s, bool profile, bool concurrent)
{
    const bool fp64 = b->opts.precision == RVE_FP64;
    a.ws_fib = ws_fib;
    a.ws_node = ws_node;
    b->ev_used = 0;
    if (profile) {
        int rc = ensure_events(b, 2 * (int)b->groups.size() + 2);
        if (rc) return rc;
    }
    // Work order (opts.work_order).  In cost order a group takes its RVEs in
    // longest-processing-time order of the previous solve's cost (iterations
    // x fibers), so the RVEs that ran longest start first and the launch's
    // tail (its last, long RVEs on few CUs) shrinks; in host order, most
    // fibers first.  The sort is in place and stable (ties keep host order);
    // rve_batch_set_opts uploads the host order again, so a change of
    // work_order starts from it.  Team groups keep host order.
    if ((int)b->groups.size() <= kOrderGroups) {
        OrderArgs o{};
        o.list = b->dlist;
        o.iters = b->diters;
        o.fib_off = b->net.fib_off;
        bool any = false;
        for (size_t g = 0; g < b->groups.size(); ++g) {
            const int v = b->group_variant[g];
            bool by_cost = b->cost_order && !team_group(v);
            if (b->opts.work_order == RVE_ORDER_HOST) by_cost = false;
            if (b->opts.work_order == RVE_ORDER_AUTO && (v == kStreamedGroup || v == kIncGlobalGroup)) by_cost = false;
            o.first[g] = b->group_first[g];
            o.count[g] = by_cost ? (int32_t)b->groups[g].size() : 0;
            any = any || by_cost;
        }
        if (any) HIP_TRY(launch_order_by_cost(o, (int)b->groups.size(), s));
    }
    HIP_TRY(launch_reset(queues, 2 * (int)b->groups.size(), s));
    int32_t* team_err = reinterpret_cast<int32_t*>(team_ws);
    char* team_area = team_ws ? team_ws + 256 : nullptr;
    if (team_ws) HIP_TRY(launch_zero32(team_err, (int64_t)b->groups.size(), s));
    // Launch order: team groups first, alone on the batch's stream (their
    // workgroups must all be resident at once); then the other groups, the
    // heaviest (most fibers) first, each on its own stream when `concurrent`,
    // so the tail of one group (its last, longest RVEs) overlaps the others.
    std::vector<size_t> order;
    for (size_t g = 0; g < b->groups.size(); ++g)
        if (team_group(b->group_variant[g])) order.push_back(g);
    const size_t n_team = order.size();
    std::vector<std::pair<int64_t, size_t>> rest;
    for (size_t g = 0; g < b->groups.size(); ++g)
        if (!team_group(b->group_variant[g])) {
            int64_t w = 0;
            for (int32_t r : b->groups[g]) w += b->nfib_of[r];
            rest.push_back({-w, g});
        }
    std::sort(rest.begin(), rest.end());
    for (auto& pr : rest) order.push_back(pr.second);
    const bool fork = concurrent && rest.size() > 1;
    if (fork) {
        for (int q = 0; q < 3; ++q) {
            if (!b->aux[q]) HIP_TRY(hipStreamCreateWithFlags(&b->aux[q], hipStreamNonBlocking));
            if (!b->join_ev[q]) HIP_TRY(hipEventCreateWithFlags(&b->join_ev[q], hipEventDisableTiming));
        }
        if (!b->fork_ev) HIP_TRY(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
    }
    for (size_t oi = 0; oi < order.size(); ++oi) {
        const size_t g = order[oi];
        hipStream_t gs_ = s;
        if (fork && oi == n_team) {
            HIP_TRY(hipEventRecord(b->fork_ev, s));
            for (int q = 0; q < 3; ++q) HIP_TRY(hipStreamWaitEvent(b->aux[q], b->fork_ev, 0));
        }
        if (fork && oi > n_team) gs_ = b->aux[(oi - n_team - 1) % 3];
        a.list = b->dlist + b->group_first[g];
        a.n_list = (int32_t)b->groups[g].size();
        a.queue = queues + 2 * g;
        const int v = b->group_variant[g];
        if (profile) HIP_TRY(hipEventRecord(b->ev[2 * g], gs_));
        if (v >= 0) {
            int per_cu = 1;
            HIP_TRY(max_resident_blocks(v, fp64, a.kinetic != 0, b->group_lds[g], &per_cu));
            if (per_cu < 1) return fail(RVE_EDEVICE, "resident kernel variant does not fit a CU");
            int grid = std::min<int64_t>((int64_t)per_cu * b->n_cu, a.n_list);
            HIP_TRY(launch_resident(v, fp64, a, b->group_lds[g], grid, gs_));
        } else if (v == kIncGroup) {
            const int iv = inc_variant(b);
            if (iv < 0) return fail(RVE_EDEVICE, "internal: no incidence build for these options");
            int per_cu = 1;
            HIP_TRY(incidence_blocks(iv, a.kinetic != 0, b->group_lds[g], &per_cu));
            if (per_cu < 1) return fail(RVE_EDEVICE, "incidence kernel does not fit a CU");
            int grid = std::min<int64_t>((int64_t)per_cu * b->n_cu, a.n_list);
            HIP_TRY(launch_incidence(iv, a, b->inc_tab, b->group_lds[g], grid, gs_));
        } else if (v == kIncGlobalGroup) {
            if (!incg_ok(b)) return fail(RVE_EDEVICE, "internal: no global-mode incidence build for these options");
            int per_cu = 1;
            HIP_TRY(incidence_global_blocks(a.kinetic != 0, &per_cu));
            if (per_cu < 1) return fail(RVE_EDEVICE, "incidence kernel (global mode) does not fit a CU");
            int grid = std::min<int64_t>((int64_t)per_cu * b->n_cu, a.n_list);
            HIP_TRY(launch_incidence_global(a, b->inc_tab, grid, gs_));
        } else if (team_group(v)) {
            const int k = b->group_team[g];
            if (!team_ws) return fail(RVE_EWORKSPACE, "internal: no team work area");
            int n_teams = 0;
            int rc = team_grid(b, fp64, a.kinetic != 0, b->group_lds[g], k, &n_teams);
            if (rc) return rc;
            // no more teams than RVEs (rounded up to whole XCD sets)
            n_teams = std::min(n_teams, 8 * (int)((a.n_list + 7) / 8));
            int64_t mx = 0;
            for (int32_t r : b->groups[g]) mx = std::max(mx, b->team_xslots[r]);
            const TeamWs L = team_ws_layout(b, k, n_teams, mx, fp64);
            TeamArgs ta = b->team_tab;
            ta.s = a;
            ta.k = k;
            ta.kinetic = a.kinetic;
            ta.xchg = team_area;
            ta.max_xslots = std::max<int64_t>(mx, 1);
            ta.partials = reinterpret_cast<double*>(team_area + L.xchg);
            int32_t* words = reinterpret_cast<int32_t*>(team_area + L.xchg + L.partials);
            ta.bar = reinterpret_cast<unsigned*>(words);
            ta.team_task = words + n_teams;
            ta.error = team_err + g;
            ta.spin_limit = b->team_spin_limit;
            HIP_TRY(launch_zero32(words, 3 * (int64_t)n_teams, gs_));
            HIP_TRY(launch_mark_unfinished(a.list, a.n_list, a.status, gs_));
            HIP_TRY(launch_team(fp64, ta, b->group_lds[g], n_teams * k, gs_));
        } else {
            int threads = streamed_threads(b, fp64);
            if (!threads) return fail(RVE_EDEVICE, "internal: every streamed kernel build uses private memory");
            a.lds_h_nodes = streamed_lds_nodes(b, b->groups[g].data(), b->groups[g].size(), fp64);
            int grid = std::min<int64_t>((int64_t)b->n_cu * streamed_blocks_per_cu(threads, a.lds_h_nodes, fp64),
                                         a.n_list);
            HIP_TRY(launch_streamed(fp64, a, grid, threads, gs_));
            a.lds_h_nodes = 0;
        }
        if (profile) HIP_TRY(hipEventRecord(b->ev[2 * g + 1], gs_));
    }
    if (fork)
        for (int q = 0; q < 3; ++q) {
            HIP_TRY(hipEventRecord(b->join_ev[q], b->aux[q]));
            HIP_TRY(hipStreamWaitEvent(s, b->join_ev[q], 0));
        }
    const size_t gs = b->groups.size();
    if (profile) HIP_TRY(hipEventRecord(b->ev[2 * gs], s));
    HIP_TRY(launch_stress(a, (int)b->R, s));
    if (profile) {
        HIP_TRY(hipEventRecord(b->ev[2 * gs + 1], s));
        b->ev_used = 2 * (int)gs + 2;
    }
    return RVE_OK;
}

// After a synchronous solve: did a team launch give up at a barrier?
static int team_errors(rve_batch* b, const char* team_ws)
{
    if (!team_ws || b->groups.empty()) return RVE_OK;
    std::vector<int32_t> e(b->groups.size(), 0);
    HIP_TRY(hipMemcpy(e.data(), team_ws, 4 * e.size(), hipMemcpyDeviceToHost));
    for (size_t g = 0; g < e.size(); ++g)
        if (e[g])
            return fail(RVE_EDEVICE, "a team of " + std::to_string(b->group_team[g]) +
                                         " workgroups waited beyond its limit at a barrier (workgroups not co-resident?); "
                                         "its RVEs are reported non-finite");
    return RVE_OK;
}

int rve_batch_solve(rve_batch* b, const double* F, double* sigma, int32_t* status, rve_stats* stats,
                    int32_t ptr_kind)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    if (ptr_kind != RVE_PTR_HOST && ptr_kind != RVE_PTR_DEVICE) return fail(RVE_EINVAL, "bad ptr_kind");
    if (b->R == 0) return RVE_OK;
    if (!F || !sigma || !status) return fail(RVE_EINVAL, "F, sigma and status are required");
    if (b->opts.init == RVE_INIT_WARM && !b->have_state)
        return fail(RVE_ESTATE, "warm start requested before any solve");
    hipStream_t s = (hipStream_t)b->opts.stream;
    const hipMemcpyKind in_kind = ptr_kind == RVE_PTR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const hipMemcpyKind out_kind = ptr_kind == RVE_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    HIP_TRY(hipMemcpyAsync(b->dF, F, 72 * b->R, in_kind, s));
    int rc = ensure_workspace(b);
    if (rc) return rc;
    int32_t init = b->opts.init;
    if (init == RVE_INIT_REFERENCE) {
        // free nodes at Xm: the fluctuation (I - F) Xm, then a warm start from it
        if (!b->d_xm_free) {
            std::vector<double> xf(3 * (size_t)b->NFREE + 3);
            for (int64_t r = 0; r < b->R; ++r) {
                const int64_t n0 = b->node_off[r], nn = b->node_off[r + 1] - n0, nf = b->nf_of[r];
                for (int64_t q = 0; q < nn; ++q) {
                    const int64_t id = b->newid[n0 + q];
                    if (id < nf)
                        for (int k = 0; k < 3; ++k) xf[3 * (b->free_off[r] + id) + k] = b->Xm[3 * (n0 + q) + k];
                }
            }
            if (hipMalloc((void**)&b->d_xm_free, xf.size() * 8) != hipSuccess) {
                b->d_xm_free = nullptr;
                return fail(RVE_ENOMEM, "reference-coordinate allocation failed");
            }
            HIP_TRY(hipMemcpy(b->d_xm_free, xf.data(), xf.size() * 8, hipMemcpyHostToDevice));
        }
        HIP_TRY(launch_reference_h(b->dF, b->net.free_off, b->d_xm_free, b->R, b->dh, s));
        init = RVE_INIT_WARM;
    }

    SolveArgs a{};
    a.net = b->net;
    a.F = b->dF;
    a.c = b->dc;
    a.queue = b->dqueue;
    a.law = b->opts.law;
    a.mass_mode = b->opts.mass;
    a.init = init;
    a.check_every = b->opts.check_every;
    a.EA = b->opts.EA;
    a.B = b->opts.B;
    a.rhoA = b->opts.rhoA;
    a.alpha = b->opts.alpha;
    a.tol_abs = b->opts.tol_abs;
    a.tol_rel = b->opts.tol_rel;
    a.n_max = b->opts.n_max;
    a.sigma = b->dsigma;
    a.status = b->dstatus;
    a.iters = b->diters;
    a.Rres = b->dR;
    a.Dres = b->dD;
    a.Bres = b->dB;
    a.h_state = b->dh;
    a.ws_fib = b->ws_fib;
    a.ws_node = b->ws_node;
    a.kinetic = kinetic_mode(b->opts) ? 1 : 0;
    a.floor_tol_rel = b->opts.floor_tol_rel;
    a.stall_checks = b->opts.stall_checks;

    b->last_variant = false;
    if (variant_mode(b->opts)) {
        if (!b->v_ws) {
            if (b->ws_user) return fail(RVE_EWORKSPACE, "internal: bound workspace has no variant area");
            if (hipMalloc((void**)&b->v_ws, variant_ws_bytes(b->NFREE, b->NF) + 16 * (size_t)b->R) != hipSuccess) {
                b->v_ws = nullptr;
                return fail(RVE_ENOMEM, "variant workspace allocation failed");
            }
        }
        VariantArgs va{};
        va.s = a;
        va.damping = b->opts.damping;
        va.energy_check = b->opts.energy_check;
        va.energy_tol = b->opts.energy_tol;
        va.ws_node = b->v_ws;
        va.ws_fib = b->v_ws + 17 * (size_t)b->NFREE;
        va.c_final = reinterpret_cast<double*>(reinterpret_cast<char*>(b->v_ws) + variant_ws_bytes(b->NFREE, b->NF));
        va.energy = va.c_final + b->R;
        b->ev_used = 0;
        if (b->profile) {
            rc = ensure_events(b, 4);
            if (rc) return rc;
            HIP_TRY(hipEventRecord(b->ev[0], s));
        }
        HIP_TRY(launch_variant(va, b->R, s));
        if (b->profile) {
            HIP_TRY(hipEventRecord(b->ev[1], s));
            HIP_TRY(hipEventRecord(b->ev[2], s));
        }
        HIP_TRY(launch_stress(a, (int)b->R, s));
        if (b->profile) {
            HIP_TRY(hipEventRecord(b->ev[3], s));
            b->ev_used = 4;
        }
        b->last_variant = true;
    } else if (b->opts.engine == RVE_ENGINE_NAIVE) {
        std::vector<double> Fh(9 * b->R);
        HIP_TRY(hipMemcpyAsync(Fh.data(), b->dF, 72 * b->R, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        std::string err;
        rc = rve_naive_run(a, b->fib_off, b->free_off, b->bnd_off, Fh, b->c_host, s, &err);
        if (rc) return fail(rc, err);
    } else {
        rc = launch_groups(b, a, b->dqueue, b->ws_fib, b->ws_node, b->team_ws, s, b->profile, true);
        if (rc) return rc;
        b->cost_order = true;
    }
    HIP_TRY(hipMemcpyAsync(sigma, b->dsigma, 72 * b->R, out_kind, s));
    HIP_TRY(hipMemcpyAsync(status, b->dstatus, 4 * b->R, out_kind, s));
    if (stats) {
        if (stats->iters) HIP_TRY(hipMemcpyAsync(stats->iters, b->diters, 8 * b->R, out_kind, s));
        if (stats->R) HIP_TRY(hipMemcpyAsync(stats->R, b->dR, 8 * b->R, out_kind, s));
        if (stats->D) HIP_TRY(hipMemcpyAsync(stats->D, b->dD, 8 * b->R, out_kind, s));
        if (stats->Fb) HIP_TRY(hipMemcpyAsync(stats->Fb, b->dB, 8 * b->R, out_kind, s));
    }
    if (ptr_kind == RVE_PTR_HOST) {
        HIP_TRY(hipStreamSynchronize(s));
        b->have_state = true;
        ++b->generation;
        return team_errors(b, b->team_ws);
    }
    b->have_state = true;
    ++b->generation;
    return RVE_OK;
}

static void fill_solve_args(rve_batch* b, SolveArgs& a)
{
    a = SolveArgs{};
    a.net = b->net;
    a.F = b->dF;
    a.c = b->dc;
    a.law = b->opts.law;
    a.mass_mode = b->opts.mass;
    a.init = RVE_INIT_AFFINE;
    a.check_every = b->opts.check_every;
    a.EA = b->opts.EA;
    a.B = b->opts.B;
    a.rhoA = b->opts.rhoA;
    a.alpha = b->opts.alpha;
    a.tol_abs = b->opts.tol_abs;
    a.tol_rel = b->opts.tol_rel;
    a.n_max = b->opts.n_max;
    a.sigma = b->dsigma;
    a.status = b->dstatus;
    a.iters = b->diters;
    a.Rres = b->dR;
    a.Dres = b->dD;
    a.Bres = b->dB;
    a.h_state = b->dh;
    a.ws_fib = b->ws_fib;
    a.ws_node = b->ws_node;
    a.kinetic = kinetic_mode(b->opts) ? 1 : 0;
    a.floor_tol_rel = b->opts.floor_tol_rel;
    a.stall_checks = b->opts.stall_checks;
}

int rve_batch_autotune(rve_batch* b, const double* F, int32_t ptr_kind, int32_t n_iter)
{
    if (!b || !F) return fail(RVE_EINVAL, "NULL argument");
    if (ptr_kind != RVE_PTR_HOST && ptr_kind != RVE_PTR_DEVICE) return fail(RVE_EINVAL, "bad ptr_kind");
    if (n_iter < 1) return fail(RVE_EINVAL, "n_iter must be >= 1");
    if (b->R == 0 || (b->opts.engine != RVE_ENGINE_AUTO && b->opts.engine != RVE_ENGINE_TEAM) || variant_mode(b->opts))
        return RVE_OK;
    hipStream_t s = (hipStream_t)b->opts.stream;
    const bool fp64 = b->opts.precision == RVE_FP64;
    HIP_TRY(hipMemcpyAsync(b->dF, F, 72 * b->R, ptr_kind == RVE_PTR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    if (!b->dtune_list && hipMalloc((void**)&b->dtune_list, 4 * (size_t)b->R + 4) != hipSuccess)
        return fail(RVE_ENOMEM, "autotune list allocation failed");
    // the streamed candidate needs its workspace
    std::vector<int> saved_variant = b->group_variant;
    b->group_variant.assign(1, -1);
    int rc = ensure_workspace(b);
    b->group_variant = saved_variant;
    if (rc) return rc;
    int rc_ev = ensure_events(b, 2);
    if (rc_ev) return rc_ev;
    auto caps = tier_caps();
    for (size_t t = 0; t < caps.size(); ++t) {
        std::vector<int32_t> members;
        for (int64_t r = 0; r < b->R; ++r)
            if (tier_of(b, r, fp64) == (int)t) members.push_back((int32_t)r);
        if (members.empty()) continue;
        std::stable_sort(members.begin(), members.end(),
                         [&](int32_t x, int32_t y) { return b->nfib_of[x] > b->nfib_of[y]; });
        members.resize(std::min<size_t>(members.size(), (size_t)b->n_cu * 2));
        double fibs = 0.0;
        size_t lds = 0;
        for (int32_t r : members) {
            fibs += (double)b->nfib_of[r];
            lds = std::max(lds, resident_lds_bytes(fp64, b->nf_of[r], b->nfib_of[r], 0));
        }
        HIP_TRY(hipMemcpy(b->dtune_list, members.data(), 4 * members.size(), hipMemcpyHostToDevice));
        SolveArgs a;
        fill_solve_args(b, a);
        a.n_max = n_iter;
        a.tol_abs = 0.0;
        a.tol_rel = 0.0;
        a.list = b->dtune_list;
        a.n_list = (int32_t)members.size();
        a.queue = b->dqueue + 62;
        double best = 1e300;
        int best_v = -1;
        std::vector<double> href;   // final states, statuses and iterations of the streamed run
        std::vector<int32_t> sref;
        std::vector<int64_t> iref;
        for (int v = -1; v < kNumResident; ++v) {
            // Variants that spill registers are not candidates: the FP64
            // (1024, 4, 2) build returned wrong final states after an unrelated
            // edit changed its spill code, and a later build of it faulted.
            // Each remaining candidate's final states must also stay close to
            // those of the streamed kernel (timed first) on the tuning RVEs.
            if (v >= 0 && (!variant_fits_tier(v, (int)t) || spills(b, v, fp64))) continue;
            if (v < 0 && !streamed_threads(b, fp64)) continue;
            int grid = 0;
            if (v >= 0) {
                int per_cu = 0;
                if (max_resident_blocks(v, fp64, a.kinetic != 0, lds, &per_cu) != hipSuccess || per_cu < 1) continue;
                grid = (int)std::min<int64_t>((int64_t)per_cu * b->n_cu, a.n_list);
            } else {
                a.lds_h_nodes = streamed_lds_nodes(b, members.data(), members.size(), fp64);
                grid = (int)std::min<int64_t>((int64_t)b->n_cu * streamed_blocks_per_cu(streamed_threads(b, fp64),
                                                                                          a.lds_h_nodes, fp64),
                                              a.n_list);
            }
            for (int rep = 0; rep < 2; ++rep) {   // first run warms up
                HIP_TRY(launch_reset(a.queue, 1, s));
                HIP_TRY(hipEventRecord(b->ev[0], s));
                if (v >= 0)
                    HIP_TRY(launch_resident(v, fp64, a, lds, grid, s));
                else
                    HIP_TRY(launch_streamed(fp64, a, grid, streamed_threads(b, fp64), s));
                HIP_TRY(hipEventRecord(b->ev[1], s));
            }
            HIP_TRY(hipEventSynchronize(b->ev[1]));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
            double per = ms / (fibs * n_iter);
            // A candidate counts only if every tuning RVE that the streamed run
            // (timed first) took through all n_iter iterations (tol = 0) also
            // runs them all here, to a final state close to the streamed one.  A variant that stops early on a non-finite state
            // would otherwise look fast.
            {
                std::vector<int32_t> stv(b->R);
                std::vector<int64_t> itv(b->R);
                std::vector<double> hv(3 * (size_t)b->NFREE);
                HIP_TRY(hipMemcpy(stv.data(), b->dstatus, 4 * (size_t)b->R, hipMemcpyDeviceToHost));
                HIP_TRY(hipMemcpy(itv.data(), b->diters, 8 * (size_t)b->R, hipMemcpyDeviceToHost));
                if (b->NFREE) HIP_TRY(hipMemcpy(hv.data(), b->dh, 24 * (size_t)b->NFREE, hipMemcpyDeviceToHost));
                bool valid = true;
                if (v < 0) {
                    href = hv;
                    sref = stv;
                    iref = itv;
                } else if (!href.empty()) {
                    // a coarse check for corrupted states: the trajectories of
                    // the variants differ in rounding (e.g. 4/G against
                    // 1/(G/4)), which floppy RVEs amplify over n_iter steps
                    const double tolh = 0.05;
                    for (int32_t r : members) {
                        // RVEs the streamed run lost to a non-finite state say
                        // nothing about the candidate
                        if (sref[r] != RVE_ST_MAXITER) continue;
                        valid = valid && stv[r] == RVE_ST_MAXITER && itv[r] == iref[r];
                        double dmax = 0.0, hmax = 0.0;
                        for (int64_t q = 3 * b->free_off[r]; q < 3 * b->free_off[r + 1]; ++q) {
                            dmax = std::max(dmax, std::fabs(hv[q] - href[q]));
                            hmax = std::max(hmax, std::fabs(href[q]));
                        }
                        valid = valid && std::isfinite(dmax) && dmax <= tolh * std::max(hmax, 1e-30);
                    }
                }
                if (!valid) continue;
            }
            if (per < best) {
                best = per;
                best_v = v;
            }
        }
        b->tuned[fp64 ? 1 : 0][t] = best_v;
    }
    // RVEs no resident build holds and the incidence kernel does not take:
    // the team engine (per team size k) against the streamed kernel on the
    // same RVEs, both from the affine start for n_iter iterations, compared
    // per CU-time; the team counts only if it takes every RVE the streamed
    // run took through all iterations through the same count to a final
    // state within 5% of the streamed one
    for (int k = 2; k <= kTeamMax; ++k) {
        std::vector<int32_t> members;
        for (int64_t r = 0; r < b->R; ++r)
            if (tier_of(b, r, fp64) < 0 && b->team_k[r] == k && !inc_rve(b, r)) members.push_back((int32_t)r);
        if (members.empty()) continue;
        std::stable_sort(members.begin(), members.end(),
                         [&](int32_t x, int32_t y) { return b->nfib_of[x] > b->nfib_of[y]; });
        members.resize(std::min<size_t>(members.size(), (size_t)std::max(8, (b->n_cu / k) / 8 * 8)));
        double ms_c[2] = {0.0, 0.0};
        std::vector<double> href;
        std::vector<int32_t> sref;
        std::vector<int64_t> iref;
        bool team_valid = true;
        const std::vector<std::vector<int32_t>> saved_groups = b->groups;
        const std::vector<int32_t> saved_v = b->group_variant, saved_team = b->group_team, saved_first = b->group_first;
        const std::vector<size_t> saved_lds = b->group_lds;
        for (int cand = 0; cand < 2; ++cand) {   // 0 streamed, 1 team
            size_t lds = 0;
            for (int32_t r : members) lds = std::max(lds, b->team_lds[fp64 ? 1 : 0][r]);
            b->groups.assign(1, members);
            b->group_variant.assign(1, cand ? -1 - k : -1);
            b->group_team.assign(1, cand ? k : 0);
            b->group_lds.assign(1, cand ? lds : 0);
            b->group_first.assign(1, 0);
            HIP_TRY(hipMemcpy(b->dlist, members.data(), 4 * members.size(), hipMemcpyHostToDevice));
            rc = ensure_workspace(b);
            if (rc) break;
            SolveArgs a;
            fill_solve_args(b, a);
            a.n_max = n_iter;
            a.tol_abs = 0.0;
            a.tol_rel = 0.0;
            for (int rep = 0; rep < 2 && !rc; ++rep) {
                HIP_TRY(hipEventRecord(b->ev[0], s));
                rc = launch_groups(b, a, b->dqueue, b->ws_fib, b->ws_node, b->team_ws, s, false, false);
                HIP_TRY(hipEventRecord(b->ev[1], s));
            }
            if (rc) break;
            HIP_TRY(hipEventSynchronize(b->ev[1]));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
            ms_c[cand] = ms;
            std::vector<int32_t> stv(b->R);
            std::vector<int64_t> itv(b->R);
            std::vector<double> hv(3 * (size_t)b->NFREE);
            HIP_TRY(hipMemcpy(stv.data(), b->dstatus, 4 * (size_t)b->R, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(itv.data(), b->diters, 8 * (size_t)b->R, hipMemcpyDeviceToHost));
            if (b->NFREE) HIP_TRY(hipMemcpy(hv.data(), b->dh, 24 * (size_t)b->NFREE, hipMemcpyDeviceToHost));
            if (!cand) {
                href = hv;
                sref = stv;
                iref = itv;
            } else {
                if (team_errors(b, b->team_ws)) team_valid = false;
                for (int32_t r : members) {
                    if (sref[r] != RVE_ST_MAXITER) continue;
                    team_valid = team_valid && stv[r] == RVE_ST_MAXITER && itv[r] == iref[r];
                    double dmax = 0.0, hmax = 0.0;
                    for (int64_t q = 3 * b->free_off[r]; q < 3 * b->free_off[r + 1]; ++q) {
                        dmax = std::max(dmax, std::fabs(hv[q] - href[q]));
                        hmax = std::max(hmax, std::fabs(href[q]));
                    }
                    team_valid = team_valid && std::isfinite(dmax) && dmax <= 0.05 * std::max(hmax, 1e-30);
                }
            }
        }
        b->groups = saved_groups;
        b->group_variant = saved_v;
        b->group_team = saved_team;
        b->group_first = saved_first;
        b->group_lds = saved_lds;
        if (rc) return rc;
        // per CU-time: a team holds k CUs per RVE where the streamed kernel
        // holds one (and team launches run alone), so the team must relax
        // its RVEs k times faster to give the batch more throughput
        b->tuned_team[fp64 ? 1 : 0][k] = (team_valid && (double)k * ms_c[1] < ms_c[0]) ? 1 : 0;
    }
    b->have_state = false;
    b->cost_order = false;   // the iterations of the timing runs are no cost estimate
    assign_groups(b);
    return upload_groups(b);
}

int rve_batch_damping_stats(rve_batch* b, double* c_final, double* energy, int32_t ptr_kind)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    if (ptr_kind != RVE_PTR_HOST && ptr_kind != RVE_PTR_DEVICE) return fail(RVE_EINVAL, "bad ptr_kind");
    if (!b->last_variant) return fail(RVE_ESTATE, "the last solve did not use a damping alternative or the energy check");
    if (b->R == 0) return RVE_OK;
    hipStream_t s = (hipStream_t)b->opts.stream;
    const hipMemcpyKind k = ptr_kind == RVE_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    const double* cf = reinterpret_cast<const double*>(reinterpret_cast<const char*>(b->v_ws) +
                                                       variant_ws_bytes(b->NFREE, b->NF));
    if (c_final) HIP_TRY(hipMemcpyAsync(c_final, cf, 8 * (size_t)b->R, k, s));
    if (energy) HIP_TRY(hipMemcpyAsync(energy, cf + b->R, 8 * (size_t)b->R, k, s));
    if (ptr_kind == RVE_PTR_HOST) HIP_TRY(hipStreamSynchronize(s));
    return RVE_OK;
}

int rve_batch_describe(const rve_batch* b, char* buf, size_t n)
{
    if (!b || !buf || n == 0) return fail(RVE_EINVAL, "NULL argument");
    std::string d;
    if (variant_mode(b->opts)) {
        std::snprintf(buf, n, "variants(fp64):%lld;", (long long)b->R);
        return RVE_OK;
    }
    for (size_t g = 0; g < b->groups.size(); ++g) {
        int v = b->group_variant[g];
        if (v >= 0)
            d += "resident(" + std::to_string(kResident[v].threads) + "," + std::to_string(kResident[v].sf) + "," +
                 std::to_string(kResident[v].sn) + ")";
        else if (v == kIncGroup) {
            const int iv = std::max(inc_variant(b), 0);
            d += "incidence(" + std::to_string(kInc[iv].threads) + "," + std::to_string(kInc[iv].slots) + ")";
        } else if (v == kIncGlobalGroup) {
            d += "incidence(global," + std::to_string(kIncGlobalThreads) + ")";
        } else if (team_group(v))
            d += "team(" + std::to_string(-1 - v) + "x" + std::to_string(kTeamUnit[b->opts.precision == RVE_FP64].threads) + ")";
        else
            d += streamed_lds_nodes(b, b->groups[g].data(), b->groups[g].size(), b->opts.precision == RVE_FP64) > 0
                     ? "streamed(lds)"
                     : "streamed";
        d += ":" + std::to_string(b->groups[g].size()) + ";";
    }
    std::snprintf(buf, n, "%s", d.c_str());
    return RVE_OK;
}

int rve_batch_positions(rve_batch* b, int64_t r, double* x)
{
    if (!b || !x) return fail(RVE_EINVAL, "NULL argument");
    if (r < 0 || r >= b->R) return fail(RVE_EINVAL, "RVE index out of range");
    if (!b->have_state) return fail(RVE_ESTATE, "no solve yet");
    hipStream_t s = (hipStream_t)b->opts.stream;
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t nf = b->nf_of[r], a0 = b->free_off[r];
    std::vector<double> h(3 * nf), F(9);
    if (nf) HIP_TRY(hipMemcpy(h.data(), b->dh + 3 * a0, 24 * nf, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(F.data(), b->dF + 9 * r, 72, hipMemcpyDeviceToHost));
    const int64_t n0 = b->node_off[r], nn = b->node_off[r + 1] - n0;
    for (int64_t p = 0; p < nn; ++p) {
        const double* X = &b->Xm[3 * (n0 + p)];
        int32_t q = b->newid[n0 + p];
        for (int i = 0; i < 3; ++i) {
            double v = F[3 * i] * X[0] + F[3 * i + 1] * X[1] + F[3 * i + 2] * X[2];
            if (q < nf) v += h[3 * q + i];
            x[3 * p + i] = v;
        }
    }
    return RVE_OK;
}

// Packed global free index of caller node n of the batch (-1: boundary node).
static std::vector<int32_t> state_map_host(const rve_batch* b)
{
    std::vector<int32_t> map(b->NN);
    for (int64_t r = 0; r < b->R; ++r) {
        const int64_t n0 = b->node_off[r], nn = b->node_off[r + 1] - n0, nf = b->nf_of[r];
        for (int64_t p = 0; p < nn; ++p) {
            const int64_t q = b->newid[n0 + p];
            map[n0 + p] = q < nf ? (int32_t)(b->free_off[r] + q) : -1;
        }
    }
    return map;
}

static int ensure_state_map(rve_batch* b)
{
    if (b->state_map_ready) return RVE_OK;
    if (b->NFREE >= INT32_MAX) return fail(RVE_EINVAL, "state export/import supports fewer than 2^31 free nodes");
    std::vector<int32_t> map;
    try {
        map = state_map_host(b);
    } catch (const std::bad_alloc&) {
        return fail(RVE_ENOMEM, "host allocation failed for the state map");
    }
    if (!b->d_state_map && hipMalloc((void**)&b->d_state_map, 4 * (size_t)b->NN + 4) != hipSuccess) {
        b->d_state_map = nullptr;
        return fail(RVE_ENOMEM, "state map allocation failed");
    }
    HIP_TRY(hipMemcpy(b->d_state_map, map.data(), 4 * (size_t)b->NN, hipMemcpyHostToDevice));
    b->state_map_ready = true;
    return RVE_OK;
}

int rve_batch_export_state(rve_batch* b, double* F, double* h, int32_t* status, int32_t ptr_kind)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    if (ptr_kind != RVE_PTR_HOST && ptr_kind != RVE_PTR_DEVICE) return fail(RVE_EINVAL, "bad ptr_kind");
    if (!b->have_state) return fail(RVE_ESTATE, "no solve or import yet");
    if (b->R == 0) return RVE_OK;
    if (!F || !h || !status) return fail(RVE_EINVAL, "F, h and status are required");
    hipStream_t s = (hipStream_t)b->opts.stream;
    if (ptr_kind == RVE_PTR_DEVICE) {
        int rc = ensure_state_map(b);
        if (rc) return rc;
        HIP_TRY(launch_export_h(b->dh, b->d_state_map, b->NN, h, s));
        HIP_TRY(hipMemcpyAsync(F, b->dF, 72 * (size_t)b->R, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(status, b->dstatus, 4 * (size_t)b->R, hipMemcpyDeviceToDevice, s));
        return RVE_OK;
    }
    std::vector<double> hp;
    std::vector<int32_t> map;
    try {
        hp.resize(3 * (size_t)b->NFREE);
        map = state_map_host(b);
    } catch (const std::bad_alloc&) {
        return fail(RVE_ENOMEM, "host allocation failed for the state export");
    }
    if (b->NFREE) HIP_TRY(hipMemcpyAsync(hp.data(), b->dh, 24 * (size_t)b->NFREE, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(F, b->dF, 72 * (size_t)b->R, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(status, b->dstatus, 4 * (size_t)b->R, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t n = 0; n < b->NN; ++n)
        for (int c = 0; c < 3; ++c) h[3 * n + c] = map[n] >= 0 ? hp[3 * (size_t)map[n] + c] : 0.0;
    return RVE_OK;
}

int rve_batch_import_state(rve_batch* b, const double* F, const double* h, const int32_t* status, double* sigma,
                           int32_t ptr_kind)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    if (ptr_kind != RVE_PTR_HOST && ptr_kind != RVE_PTR_DEVICE) return fail(RVE_EINVAL, "bad ptr_kind");
    if (b->R == 0) return RVE_OK;
    if (!F || !h || !status) return fail(RVE_EINVAL, "F, h and status are required");
    hipStream_t s = (hipStream_t)b->opts.stream;
    if (ptr_kind == RVE_PTR_DEVICE) {
        int rc = ensure_state_map(b);
        if (rc) return rc;
        HIP_TRY(launch_import_h(h, b->d_state_map, b->NN, b->dh, s));
        HIP_TRY(hipMemcpyAsync(b->dF, F, 72 * (size_t)b->R, hipMemcpyDeviceToDevice, s));
        HIP_TRY(launch_import_status(b->dF, status, b->R, b->dstatus, b->diters, b->dR, b->dD, b->dB, s));
    } else {
        std::vector<double> hp;
        std::vector<int32_t> map;
        try {
            hp.resize(3 * (size_t)b->NFREE);
            map = state_map_host(b);
        } catch (const std::bad_alloc&) {
            return fail(RVE_ENOMEM, "host allocation failed for the state import");
        }
        for (int64_t n = 0; n < b->NN; ++n)
            if (map[n] >= 0)
                for (int c = 0; c < 3; ++c) hp[3 * (size_t)map[n] + c] = h[3 * n + c];
        // the status input goes through the device copy of the last statuses
        // (the kernel reads it before writing the checked value in place)
        if (b->NFREE) HIP_TRY(hipMemcpyAsync(b->dh, hp.data(), 24 * (size_t)b->NFREE, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b->dF, F, 72 * (size_t)b->R, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b->dstatus, status, 4 * (size_t)b->R, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_import_status(b->dF, b->dstatus, b->R, b->dstatus, b->diters, b->dR, b->dD, b->dB, s));
    }
    SolveArgs a;
    fill_solve_args(b, a);
    HIP_TRY(launch_stress(a, (int)b->R, s));
    if (sigma)
        HIP_TRY(hipMemcpyAsync(sigma, b->dsigma, 72 * (size_t)b->R,
                               ptr_kind == RVE_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
    if (ptr_kind == RVE_PTR_HOST) HIP_TRY(hipStreamSynchronize(s));
    b->have_state = true;
    ++b->generation;
    return RVE_OK;
}

// Tangent workspace: fiber operators, ELL records, preconditioner, chunk
// tables and task groups for the whole batch (allocated once), and the
// per-workgroup solver slots (`slot_bytes`, grown on demand).
// Offsets of the tangent arena: fiber operators, ELL records,
// preconditioner, chunk tables, outputs/inputs, statuses, iterations, order.
struct TanArena {
    size_t par, rs, ra, rb, pc, cf, cr, out, in, st, it, ord, bytes;
};

static TanArena tangent_arena(const rve_batch* b)
{
    const int64_t nch = (int64_t)b->chunk_rec.size() - 1, nrec = b->chunk_rec.back();
    DeviceArena A;
    TanArena t;
    t.par = A.reserve(48 * (size_t)b->NF);
    t.rs = A.reserve(8 * (size_t)nrec);
    t.ra = A.reserve(16 * (size_t)nrec);
    t.rb = A.reserve(8 * (size_t)nrec);
    t.pc = A.reserve(32 * (size_t)b->NFREE);
    t.cf = A.reserve(8 * (size_t)(b->R + 1));
    t.cr = A.reserve(8 * (size_t)(nch + 1));
    t.out = A.reserve(8 * 81 * (size_t)b->R);
    t.in = A.reserve(8 * 9 * (size_t)b->R);
    t.st = A.reserve(4 * (size_t)b->R);
    t.it = A.reserve(8 * (size_t)b->R);
    t.ord = A.reserve(4 * (size_t)b->R);
    t.bytes = A.used + 256;
    return t;
}

// Task groups of the tangent (host tables, computed once): RVEs for each
// resident variant (smallest that holds the RVE), then the rest for the
// streamed kernel; longest first in each.
static void tangent_groups(rve_batch* b)
{
    if (!b->t_group_first.empty()) return;
    std::vector<int32_t> lpt(b->R);
    for (int64_t r = 0; r < b->R; ++r) lpt[r] = (int32_t)r;
    std::stable_sort(lpt.begin(), lpt.end(), [&](int32_t x, int32_t y) { return b->nf_of[x] > b->nf_of[y]; });
    std::vector<int32_t> order;
    order.reserve(b->R);
    std::vector<int64_t> first(kNumTanRes + 2, 0);
    for (int v = 0; v <= kNumTanRes; ++v) {
        first[v] = (int64_t)order.size();
        for (int32_t r : lpt) {
            int g = kNumTanRes;
            for (int u = 0; u < kNumTanRes; ++u) {
                if (b->tangent_private[0][u] || b->tangent_private[1][u]) continue;   // never launched
                if (b->nf_of[r] <= (int64_t)kTanRes[u].threads * kTanRes[u].sn) {
                    g = u;
                    break;
                }
            }
            if (g == v) order.push_back(r);
        }
    }
    first[kNumTanRes + 1] = (int64_t)order.size();
    b->t_order_host = order;
    b->t_group_first = first;
}

// Tangent workspace: the arena (carved once, from the caller's workspace when
// one is bound) with its task tables uploaded, and the per-workgroup solver
// slots (`slot_bytes`, grown on demand unless the workspace is bound).
static int ensure_tangent_ws(rve_batch* b, size_t slot_bytes)
{
    if (!b->t_tables) {
        const TanArena t = tangent_arena(b);
        const int64_t nch = (int64_t)b->chunk_rec.size() - 1;
        if (!b->t_mem) {
            if (b->ws_user) return fail(RVE_EINVAL, "internal: bound workspace has no tangent arena");
            if (hipMalloc((void**)&b->t_mem, t.bytes) != hipSuccess) {
                b->t_mem = nullptr;
                return fail(RVE_ENOMEM, "tangent workspace allocation failed");
            }
        }
        char* m = b->t_mem;
        b->t_par64 = carve<double>(m, t.par);
        b->t_rec_static = carve<int2>(m, t.rs);
        b->t_recA = carve<float4>(m, t.ra);
        b->t_recB = carve<int2>(m, t.rb);
        b->t_precond = carve<float4>(m, t.pc);
        b->t_chunk_first = carve<int64_t>(m, t.cf);
        b->t_chunk_rec = carve<int64_t>(m, t.cr);
        b->t_out = carve<double>(m, t.out);
        b->t_in = carve<double>(m, t.in);
        b->t_status = carve<int32_t>(m, t.st);
        b->t_iters = carve<int64_t>(m, t.it);
        b->t_order = carve<int32_t>(m, t.ord);
        tangent_groups(b);
        hipError_t e = hipMemcpy(b->t_order, b->t_order_host.data(), 4 * (size_t)b->R, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(b->t_chunk_first, b->chunk_first.data(), 8 * (size_t)(b->R + 1), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(b->t_chunk_rec, b->chunk_rec.data(), 8 * (size_t)(nch + 1), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (!b->ws_user) {
                (void)hipFree(b->t_mem);
                b->t_mem = nullptr;
            }
            return fail(RVE_EDEVICE, std::string("tangent table upload: ") + hipGetErrorString(e));
        }
        b->t_static_built = false;
        b->t_tables = true;
    }
    if (slot_bytes > b->t_slot_bytes) {
        if (b->ws_user) return fail(RVE_EINVAL, "internal: bound workspace smaller than the tangent slots");
        if (b->t_slots) (void)hipFree(b->t_slots);
        b->t_slots = nullptr;
        b->t_slot_bytes = 0;
        if (hipMalloc((void**)&b->t_slots, slot_bytes) != hipSuccess) {
            b->t_slots = nullptr;
            return fail(RVE_ENOMEM, "tangent workspace allocation failed");
        }
        b->t_slot_bytes = slot_bytes;
    }
    return RVE_OK;
}

// Launch plan of a tangent (mode 0, nine right-hand sides per RVE) or VJP
// (mode 1) call: task ranges per kernel variant in the task order, grid and
// slot length S per launch, and the slot bytes the plan needs.  Engines other
// than AUTO run every task on the 64-thread streamed kernel.  blk[v]: the
// launch of variant v runs the blocked build (three right-hand sides per
// task; tangent, AUTO engine, tangent_rhs 3, a build without private memory).
// The library's own choice (tangent_rhs 0) is one task per right-hand side:
// on the 4096-RVE workload the blocked tasks take 303 ms per tangent call
// against 190 ms (the per-column task keeps p, q, r, z and d in registers,
// the blocked one keeps three columns' q and d in global memory and waits
// for its slowest column).
static int tangent_plan(rve_batch* b, int mode, int engine, int rhs_opt, std::vector<int64_t>& gf, int* grid,
                        int64_t* S, bool* blk, size_t* slot_bytes)
{
    tangent_groups(b);
    const int per = mode == 0 ? 9 : 1;
    for (int v = 0; v <= kNumTanRes; ++v)
        blk[v] = mode == 0 && engine == RVE_ENGINE_AUTO && rhs_opt == 3 && v < kNumTanBlk &&
                 !b->tangent_blk_private[v];
    gf = b->t_group_first;
    if (engine != RVE_ENGINE_AUTO) {
        for (int v = 0; v <= kNumTanRes; ++v) gf[v] = 0;
        gf[kNumTanRes + 1] = b->R;
    }
    *slot_bytes = 0;
    const int stream_threads = engine == RVE_ENGINE_AUTO ? 1024 : 64;
    for (int v = 0; v <= kNumTanRes; ++v) {
        const int64_t tasks = (gf[v + 1] - gf[v]) * per;
        grid[v] = 0;
        S[v] = 1;
        if (tasks == 0) continue;
        if (v < kNumTanRes && blk[v]) {
            int bpc = 0;
            HIP_TRY(tangent_blk_blocks(v, &bpc));
            if (bpc < 1) return fail(RVE_EDEVICE, "blocked tangent kernel does not fit a compute unit");
            const int64_t btasks = (gf[v + 1] - gf[v]) * (9 / kTanBlkRhs);
            grid[v] = (int)std::min<int64_t>((int64_t)bpc * b->n_cu, btasks);
            S[v] = (int64_t)kTanRes[v].threads * kTanRes[v].sn + 1;
            *slot_bytes = std::max(*slot_bytes, 80 * (size_t)kTanBlkRhs * (size_t)S[v] * (size_t)grid[v]);
        } else if (v < kNumTanRes) {
            int bpc = 0;
            HIP_TRY(tangent_res_blocks(v, mode != 0, &bpc));
            if (bpc < 1) return fail(RVE_EDEVICE, "tangent kernel does not fit a compute unit");
            grid[v] = (int)std::min<int64_t>((int64_t)bpc * b->n_cu, tasks);
            S[v] = (int64_t)kTanRes[v].threads * kTanRes[v].sn + 1;
            *slot_bytes = std::max(*slot_bytes, 64 * (size_t)S[v] * (size_t)grid[v]);
        } else {
            // streamed: one 1024-thread workgroup per CU for the RVEs too large
            // for LDS, or one wavefront per task (8 per CU) on the STREAMED engine
            grid[v] = (int)std::min<int64_t>((int64_t)b->n_cu * (stream_threads == 64 ? 8 : 1), tasks);
            for (int64_t r = 0; r < b->R; ++r) S[v] = std::max<int64_t>(S[v], b->nf_of[r] + 1);
            *slot_bytes = std::max(*slot_bytes, 128 * (size_t)S[v] * (size_t)grid[v]);
        }
    }
    return RVE_OK;
}

// Caller-provided workspace: the streamed workspace (sized for FP64, so a
// change of precision never outgrows it), the tangent arena, the largest
// tangent/VJP slot area over both engines, the orientation outputs and the
// state map, each at a 256-byte aligned offset.
struct WsLayout {
    size_t fib, node, tmem, slots, omem, smap, var, team;
    size_t o_fib, o_node, o_tmem, o_slots, o_omem, o_smap, o_var, o_team, total;
};

static int ws_layout(rve_batch* b, WsLayout& L)
{
    L.fib = 32 * 3 * (size_t)(b->NF + b->R);
    L.node = 32 * (2 * (size_t)(b->NFREE + b->R) + 2 * (size_t)b->NFREE + 1);
    L.tmem = tangent_arena(b).bytes;
    L.slots = 0;
    for (int mode = 0; mode < 2; ++mode)
        for (int engine : {(int)RVE_ENGINE_AUTO, (int)RVE_ENGINE_STREAMED}) {
            std::vector<int64_t> gf;
            int grid[kNumTanRes + 1];
            int64_t S[kNumTanRes + 1];
            size_t sb = 0;
            for (int rhs : {0, 3}) {
                bool blk[kNumTanRes + 1];
                int rc = tangent_plan(b, mode, engine, rhs, gf, grid, S, blk, &sb);
                if (rc) return rc;
                L.slots = std::max(L.slots, sb);
            }
        }
    L.omem = 80 * (size_t)b->R;
    L.smap = 4 * (size_t)b->NN + 4;
    L.var = variant_ws_bytes(b->NFREE, b->NF) + 16 * (size_t)b->R;
    L.team = team_ws_bytes(b);
    DeviceArena A;
    L.o_fib = A.reserve(L.fib);
    L.o_node = A.reserve(L.node);
    L.o_tmem = A.reserve(L.tmem);
    L.o_slots = A.reserve(L.slots);
    L.o_omem = A.reserve(L.omem);
    L.o_smap = A.reserve(L.smap);
    L.o_var = A.reserve(L.var);
    L.o_team = A.reserve(L.team);
    L.total = A.used;
    return RVE_OK;
}

int rve_batch_workspace_size(const rve_batch* cb, size_t* bytes)
{
    if (!cb || !bytes) return fail(RVE_EINVAL, "NULL argument");
    // the layout caches the tangent's host task tables in the batch
    rve_batch* b = const_cast<rve_batch*>(cb);
    WsLayout L;
    int rc = ws_layout(b, L);
    if (rc) return rc;
    *bytes = L.total;
    return RVE_OK;
}

// Free the library-owned workspace regions (when no caller workspace is
// bound) and forget every region pointer; tables built in them are rebuilt.
static void drop_workspace(rve_batch* b)
{
    if (!b->ws_user) {
        if (b->ws_fib) (void)hipFree(b->ws_fib);
        if (b->ws_node) (void)hipFree(b->ws_node);
        if (b->t_mem) (void)hipFree(b->t_mem);
        if (b->t_slots) (void)hipFree(b->t_slots);
        if (b->o_mem) (void)hipFree(b->o_mem);
        if (b->d_state_map) (void)hipFree(b->d_state_map);
        if (b->v_ws) (void)hipFree(b->v_ws);
        if (b->team_ws) (void)hipFree(b->team_ws);
    }
    b->team_ws = nullptr;
    b->team_ws_bytes = 0;
    b->ws_fib = b->ws_node = nullptr;
    b->ws_fib_bytes = b->ws_node_bytes = 0;
    b->t_mem = nullptr;
    b->t_slots = nullptr;
    b->t_slot_bytes = 0;
    b->o_mem = nullptr;
    b->d_state_map = nullptr;
    b->v_ws = nullptr;
    b->last_variant = false;
    b->t_tables = false;
    b->t_static_built = false;
    b->state_map_ready = false;
    b->ws_user = nullptr;
    b->ws_user_bytes = 0;
}

int rve_batch_bind_workspace(rve_batch* b, void* ptr, size_t bytes)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    WsLayout L;
    int rc = ws_layout(b, L);
    if (rc) return rc;
    if (ptr) {
        if (reinterpret_cast<uintptr_t>(ptr) & 255) return fail(RVE_EWORKSPACE, "workspace must be 256-byte aligned");
        if (bytes < L.total)
            return fail(RVE_EWORKSPACE, "workspace too small: " + std::to_string(L.total) + " bytes needed");
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, ptr) != hipSuccess || at.type != hipMemoryTypeDevice ||
            at.device != b->device) {
            (void)hipGetLastError();
            return fail(RVE_EWORKSPACE, "workspace must be device memory of the batch's device");
        }
    }
    // work already queued may still use the current regions
    HIP_TRY(hipStreamSynchronize((hipStream_t)b->opts.stream));
    drop_workspace(b);
    if (!ptr) return RVE_OK;
    char* m = static_cast<char*>(ptr);
    b->ws_user = m;
    b->ws_user_bytes = bytes;
    b->ws_fib = m + L.o_fib;
    b->ws_fib_bytes = L.fib;
    b->ws_node = m + L.o_node;
    b->ws_node_bytes = L.node;
    b->t_mem = m + L.o_tmem;
    b->t_slots = m + L.o_slots;
    b->t_slot_bytes = L.slots;
    b->o_mem = reinterpret_cast<double*>(m + L.o_omem);
    b->d_state_map = reinterpret_cast<int32_t*>(m + L.o_smap);
    b->v_ws = reinterpret_cast<double*>(m + L.o_var);
    b->team_ws = L.team ? m + L.o_team : nullptr;
    b->team_ws_bytes = L.team;
    return RVE_OK;
}

static int run_cg(rve_batch* b, int mode, const double* gsigma, double* out, int32_t* status, int32_t ptr_kind)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    if (ptr_kind != RVE_PTR_HOST && ptr_kind != RVE_PTR_DEVICE) return fail(RVE_EINVAL, "bad ptr_kind");
    if (b->R == 0) return RVE_OK;
    if (!out || !status || (mode == 1 && !gsigma)) return fail(RVE_EINVAL, "NULL output or input");
    if (!b->have_state) return fail(RVE_ESTATE, "no solve yet");
    // allocate the batch tables first (task groups), then size the slots
    int rc = ensure_tangent_ws(b, 0);
    if (rc) return rc;
    const int stream_threads = b->opts.engine == RVE_ENGINE_AUTO ? 1024 : 64;
    std::vector<int64_t> gf;
    int grid[kNumTanRes + 1];
    int64_t S[kNumTanRes + 1];
    size_t slot_bytes = 0;
    bool blk[kNumTanRes + 1];
    rc = tangent_plan(b, mode, b->opts.engine, b->opts.tangent_rhs, gf, grid, S, blk, &slot_bytes);
    if (rc) return rc;
    // largest free-node count of each launch's RVEs
    b->t_max_nf.assign(kNumTanRes + 1, 0);
    for (int v = 0; v <= kNumTanRes; ++v)
        for (int64_t q = gf[v]; q < gf[v + 1]; ++q)
            b->t_max_nf[v] = std::max<int64_t>(b->t_max_nf[v], b->nf_of[b->t_order_host[q]]);
    rc = ensure_tangent_ws(b, slot_bytes);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)b->opts.stream;
    const hipMemcpyKind in_kind = ptr_kind == RVE_PTR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const hipMemcpyKind out_kind = ptr_kind == RVE_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (mode == 1) HIP_TRY(hipMemcpyAsync(b->t_in, gsigma, 72 * b->R, in_kind, s));
    TangentArgs a{};
    a.net = b->net;
    a.F = b->dF;
    a.sigma = b->dsigma;
    a.solve_status = b->dstatus;
    a.h_state = b->dh;
    a.gsigma = b->t_in;
    a.out = b->t_out;
    a.status = b->t_status;
    a.iters = reinterpret_cast<unsigned long long*>(b->t_iters);
    a.queue = b->dqueue + 60;
    a.mode = mode;
    a.law = b->opts.law;
    a.EA = b->opts.EA;
    a.B = b->opts.B;
    a.cg_tol = b->opts.cg_tol;
    a.cg_max = b->opts.cg_max_iter;
    a.n_free_total = b->NFREE;
    a.n_rve = b->R;
    a.chunk_first = b->t_chunk_first;
    a.chunk_rec = b->t_chunk_rec;
    a.rec_static = b->t_rec_static;
    a.recA = b->t_recA;
    a.recB = b->t_recB;
    a.precond = b->t_precond;
    a.par64 = b->t_par64;
    a.slot_ws64 = reinterpret_cast<double*>(b->t_slots);
    a.build_static = b->t_static_built ? 0 : 1;
    HIP_TRY(launch_tangent_prep(a, s));
    b->t_static_built = true;
    for (int v = 0; v <= kNumTanRes; ++v) {
        if (grid[v] == 0) continue;
        // every RVE of the launch must fit its slot (and, resident, its LDS)
        const size_t need =
            (v < kNumTanRes ? (blk[v] ? 80 * (size_t)kTanBlkRhs : 64) : 128) * (size_t)S[v] * (size_t)grid[v];
        if (need > b->t_slot_bytes || b->t_max_nf[v] >= S[v])
            return fail(RVE_EINVAL, "internal: tangent slot smaller than an RVE of its group");
        a.order = b->t_order + gf[v];
        a.n_order = gf[v + 1] - gf[v];
        a.slot_nodes = S[v];
        a.slot_ws32 = reinterpret_cast<float4*>(b->t_slots + 48 * (size_t)S[v] * (size_t)grid[v]);
        HIP_TRY(launch_reset(a.queue, 1, s));
        if (v < kNumTanRes && blk[v])
            HIP_TRY(launch_tangent_blk(v, a, grid[v], s));
        else if (v < kNumTanRes)
            HIP_TRY(launch_tangent_res(v, a, grid[v], s));
        else
            HIP_TRY(launch_tangent_stream(a, stream_threads, grid[v], s));
    }
    HIP_TRY(hipMemcpyAsync(out, b->t_out, (mode == 0 ? 648 : 72) * b->R, out_kind, s));
    HIP_TRY(hipMemcpyAsync(status, b->t_status, 4 * b->R, out_kind, s));
    if (ptr_kind == RVE_PTR_HOST) HIP_TRY(hipStreamSynchronize(s));
    return RVE_OK;
}

int rve_batch_tangent(rve_batch* b, double* dsdF, int32_t* status, int32_t ptr_kind)
{
    return run_cg(b, 0, nullptr, dsdF, status, ptr_kind);
}

int rve_batch_vjp(rve_batch* b, const double* gsigma, double* gF, int32_t* status, int32_t ptr_kind)
{
    return run_cg(b, 1, gsigma, gF, status, ptr_kind);
}

int rve_batch_orientation(rve_batch* b, const double* e, double* omega, double* p2, int32_t ptr_kind)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    if (ptr_kind != RVE_PTR_HOST && ptr_kind != RVE_PTR_DEVICE) return fail(RVE_EINVAL, "bad ptr_kind");
    if (!e) return fail(RVE_EINVAL, "reference direction is NULL");
    const double en = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    if (!std::isfinite(en) || !(en > 0.0)) return fail(RVE_EINVAL, "reference direction must be finite and nonzero");
    if (b->R == 0) return RVE_OK;
    if (!omega || !p2) return fail(RVE_EINVAL, "NULL output");
    if (!b->have_state) return fail(RVE_ESTATE, "no solve yet");
    if (!b->o_mem && hipMalloc((void**)&b->o_mem, 80 * (size_t)b->R) != hipSuccess) {
        b->o_mem = nullptr;
        return fail(RVE_ENOMEM, "orientation output allocation failed");
    }
    hipStream_t s = (hipStream_t)b->opts.stream;
    OrientArgs a{};
    a.net = b->net;
    a.F = b->dF;
    a.h_state = b->dh;
    a.status = b->dstatus;
    for (int k = 0; k < 3; ++k) a.e[k] = e[k] / en;
    a.omega = b->o_mem;
    a.p2 = b->o_mem + 9 * b->R;
    HIP_TRY(launch_orientation(a, b->R, s));
    const hipMemcpyKind k = ptr_kind == RVE_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    HIP_TRY(hipMemcpyAsync(omega, a.omega, 72 * b->R, k, s));
    HIP_TRY(hipMemcpyAsync(p2, a.p2, 8 * b->R, k, s));
    if (ptr_kind == RVE_PTR_HOST) HIP_TRY(hipStreamSynchronize(s));
    return RVE_OK;
}

// The probe batch of the finite-difference tangent: the same networks, six
// copies of each (copy c of RVE r is probe RVE 6 r + c), rebuilt in the
// caller's original node order from the packed batch, and the map from each
// probe free node to the base free node of the same original node.
static int ensure_probe(rve_batch* b)
{
    if (b->probe) return RVE_OK;
    const int64_t R = b->R;
    std::vector<uint32_t> ends(b->NF);
    std::vector<double> V0(R), L0(b->NF), L0p;
    if (b->NF) HIP_TRY(hipMemcpy(ends.data(), b->net.ends, 4 * (size_t)b->NF, hipMemcpyDeviceToHost));
    if (b->NF) HIP_TRY(hipMemcpy(L0.data(), b->net.L0, 8 * (size_t)b->NF, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(V0.data(), b->dV0, 8 * (size_t)R, hipMemcpyDeviceToHost));
    std::vector<int64_t> node_off(1, 0), fib_off(1, 0);
    std::vector<double> X, V0p, cp;
    std::vector<uint8_t> isb;
    std::vector<int32_t> fib;
    try {
        X.reserve(18 * (size_t)b->NN);
        isb.reserve(6 * (size_t)b->NN);
        fib.reserve(12 * (size_t)b->NF);
        L0p.reserve(6 * (size_t)b->NF);
        for (int64_t r = 0; r < R; ++r) {
            const int64_t n0 = b->node_off[r], nn = b->node_off[r + 1] - n0;
            const int64_t f0 = b->fib_off[r], nfib = b->fib_off[r + 1] - f0, nf = b->nf_of[r];
            std::vector<int32_t> inv(nn);
            for (int64_t q = 0; q < nn; ++q) inv[b->newid[n0 + q]] = (int32_t)q;
            for (int c = 0; c < 6; ++c) {
                for (int64_t q = 0; q < nn; ++q) {
                    for (int k = 0; k < 3; ++k) X.push_back(b->Xm[3 * (n0 + q) + k] + 0.5);
                    isb.push_back(b->newid[n0 + q] >= nf ? 1 : 0);
                }
                for (int64_t k = 0; k < nfib; ++k) {
                    const uint32_t e = ends[f0 + k];
                    fib.push_back(inv[e & 0xffffu]);
                    fib.push_back(inv[e >> 16]);
                    L0p.push_back(L0[f0 + k]);
                }
                node_off.push_back(node_off.back() + nn);
                fib_off.push_back(fib_off.back() + nfib);
                V0p.push_back(V0[r]);
                cp.push_back(b->c_host[r]);
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(RVE_ENOMEM, "host allocation failed while building the probe batch");
    }
    rve_net_desc d{};
    d.n_rve = 6 * R;
    d.node_off = node_off.data();
    d.fib_off = fib_off.data();
    d.X = X.data();
    d.is_bnd = isb.data();
    d.fib = fib.data();
    d.V0 = V0p.data();
    d.L0 = L0p.data();
    rve_opts o = b->opts;
    o.init = RVE_INIT_WARM;
    o.c_per_rve = cp.data();
    rve_batch* pb = nullptr;
    int rc = rve_batch_create(&d, &o, &pb);
    if (rc) return rc;
    std::vector<int64_t> map(pb->NFREE);
    for (int64_t r = 0; r < R; ++r) {
        const int64_t n0 = b->node_off[r], nn = b->node_off[r + 1] - n0, nf = b->nf_of[r];
        for (int c = 0; c < 6; ++c) {
            const int64_t p = 6 * r + c, pn0 = pb->node_off[p];
            for (int64_t q = 0; q < nn; ++q) {
                const int64_t np_ = pb->newid[pn0 + q];
                if (np_ < nf) map[pb->free_off[p] + np_] = b->free_off[r] + b->newid[n0 + q];
            }
        }
    }
    if (hipMalloc((void**)&b->d_probe_map, 8 * (size_t)pb->NFREE + 8) != hipSuccess ||
        hipMalloc((void**)&b->d_fd_rot, 72 * (size_t)R) != hipSuccess) {
        rve_batch_destroy(pb);
        return fail(RVE_ENOMEM, "probe map allocation failed");
    }
    if (pb->NFREE) HIP_TRY(hipMemcpy(b->d_probe_map, map.data(), 8 * (size_t)pb->NFREE, hipMemcpyHostToDevice));
    b->probe = pb;
    return RVE_OK;
}

int rve_batch_fd_tangent(rve_batch* b, double h, double* C, double* A, int32_t* status, int32_t ptr_kind)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    if (ptr_kind != RVE_PTR_HOST && ptr_kind != RVE_PTR_DEVICE) return fail(RVE_EINVAL, "bad ptr_kind");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(RVE_EINVAL, "h must be positive and finite");
    if (b->R == 0) return RVE_OK;
    if (!C || !status) return fail(RVE_EINVAL, "NULL output");
    if (!b->have_state) return fail(RVE_ESTATE, "no solve yet");
    int rc = ensure_probe(b);
    if (rc) return rc;
    const int64_t R = b->R;
    rve_batch* pb = b->probe;
    hipStream_t s = (hipStream_t)b->opts.stream;
    // probe options follow the base batch (warm start, same stream)
    {
        rve_opts o = b->opts;
        o.init = RVE_INIT_WARM;
        std::vector<double> cp(6 * R);
        for (int64_t r = 0; r < R; ++r)
            for (int c = 0; c < 6; ++c) cp[6 * r + c] = b->c_host[r];
        o.c_per_rve = cp.data();
        rc = rve_batch_set_opts(pb, &o);
        if (rc) return rc;
    }
    std::vector<double> F(9 * R), sig(9 * R), Fp(54 * R), Rm(9 * R), sp(54 * R);
    std::vector<int32_t> st(R), stp(6 * R);
    HIP_TRY(hipMemcpyAsync(F.data(), b->dF, 72 * R, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(sig.data(), b->dsigma, 72 * R, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(st.data(), b->dstatus, 4 * R, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t r = 0; r < R; ++r) fd_prepare(&F[9 * r], h, &Fp[54 * r], &Rm[9 * r]);
    HIP_TRY(hipMemcpyAsync(b->d_fd_rot, Rm.data(), 72 * R, hipMemcpyHostToDevice, s));
    ProbeStateArgs pa{};
    pa.probe_free_off = pb->net.free_off;
    pa.map = b->d_probe_map;
    pa.Rm = b->d_fd_rot;
    pa.h_base = b->dh;
    pa.h_probe = pb->dh;
    HIP_TRY(launch_probe_state(pa, 6 * R, s));
    pb->have_state = true;
    rc = rve_batch_solve(pb, Fp.data(), sp.data(), stp.data(), nullptr, RVE_PTR_HOST);
    if (rc) return rc;
    std::vector<double> Cout(36 * R), Aout(36 * R);
    std::vector<int32_t> sout(R);
    for (int64_t r = 0; r < R; ++r) {
        int worst = 0;
        for (int c = 0; c < 6; ++c) worst = std::max(worst, (int)stp[6 * r + c]);
        bool ok = st[r] == 0 && worst == 0 &&
                  fd_finish(&F[9 * r], &sig[9 * r], &sp[54 * r], &Fp[54 * r], h, &Cout[36 * r], &Aout[36 * r]);
        sout[r] = st[r] != 0 ? RVE_ST_NO_STATE : worst;
        if (!ok) {
            if (sout[r] == 0) sout[r] = RVE_ST_NONFINITE;
            for (int k = 0; k < 36; ++k) Cout[36 * r + k] = Aout[36 * r + k] = NAN;
        }
    }
    const hipMemcpyKind k = ptr_kind == RVE_PTR_HOST ? hipMemcpyHostToHost : hipMemcpyHostToDevice;
    HIP_TRY(hipMemcpyAsync(C, Cout.data(), 288 * R, k, s));
    if (A) HIP_TRY(hipMemcpyAsync(A, Aout.data(), 288 * R, k, s));
    HIP_TRY(hipMemcpyAsync(status, sout.data(), 4 * R, k, s));
    HIP_TRY(hipStreamSynchronize(s));
    return RVE_OK;
}

int rve_batch_tangent_iters(rve_batch* b, int64_t* iters, int32_t ptr_kind)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    if (ptr_kind != RVE_PTR_HOST && ptr_kind != RVE_PTR_DEVICE) return fail(RVE_EINVAL, "bad ptr_kind");
    if (b->R == 0) return RVE_OK;
    if (!iters) return fail(RVE_EINVAL, "iters is NULL");
    if (!b->t_iters || !b->t_static_built) return fail(RVE_ESTATE, "no tangent or vjp call yet");
    hipStream_t s = (hipStream_t)b->opts.stream;
    HIP_TRY(hipMemcpyAsync(iters, b->t_iters, 8 * b->R,
                           ptr_kind == RVE_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
    if (ptr_kind == RVE_PTR_HOST) HIP_TRY(hipStreamSynchronize(s));
    return RVE_OK;
}

void rve_batch_destroy(rve_batch* b)
{
    if (!b) return;
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    for (int q = 0; q < 3; ++q) {
        if (b->aux[q]) (void)hipStreamDestroy(b->aux[q]);
        if (b->join_ev[q]) (void)hipEventDestroy(b->join_ev[q]);
    }
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    drop_workspace(b);
    if (b->probe) rve_batch_destroy(b->probe);
    if (b->d_probe_map) (void)hipFree(b->d_probe_map);
    if (b->d_fd_rot) (void)hipFree(b->d_fd_rot);
    if (b->dtune_list) (void)hipFree(b->dtune_list);
    if (b->d_xm_free) (void)hipFree(b->d_xm_free);
    if (b->team_mem) (void)hipFree(b->team_mem);
    if (b->inc_mem) (void)hipFree(b->inc_mem);
    if (b->dmem) (void)hipFree(b->dmem);
    delete b;
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free solve
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation):
// rve_batch_solve_static runs the solve's resident, team and streamed
// launches with their work areas -- the launch work counters, the team work
// area and the streamed engine's per-fiber and per-node workspace -- carved
// from this file-scope device array (256 MiB) instead of from allocations.  Each device that runs the
// library holds its own copy until the process ends; its address is taken
// once per device with hipGetSymbolAddress and kept (the array's name in
// host code is a host-side stand-in, never a device address).
constexpr size_t kStaticScratchBytes = size_t(256) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

static int device_scratch(int dev, void** out)
{
    if (dev < 0 || dev >= 64) return fail(RVE_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(RVE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RVE_OK;
}

extern "C" int rve_batch_solve_static(rve_batch* b, const double* F, double* sigma, int32_t* status,
                                      int32_t ptr_kind)
{
    if (!b) return fail(RVE_EINVAL, "batch is NULL");
    if (ptr_kind != RVE_PTR_HOST && ptr_kind != RVE_PTR_DEVICE) return fail(RVE_EINVAL, "bad ptr_kind");
    if (b->R == 0) return RVE_OK;
    if (!F || !sigma || !status) return fail(RVE_EINVAL, "F, sigma and status are required");
    if (b->opts.engine == RVE_ENGINE_NAIVE || variant_mode(b->opts))
        return fail(RVE_EINVAL, "the allocation-free solve runs the resident, incidence, team and streamed engines only");
    if (b->opts.init == RVE_INIT_REFERENCE)
        return fail(RVE_EINVAL, "the allocation-free solve takes the affine or warm start");
    if (b->opts.init == RVE_INIT_WARM && !b->have_state)
        return fail(RVE_ESTATE, "warm start requested before any solve");
    const bool fp64 = b->opts.precision == RVE_FP64;
    bool streamed = false, team = false;
    for (int v : b->group_variant) {
        streamed |= (v == kStreamedGroup);
        team |= team_group(v);
    }
    // layout: work counters (two per launch group), the team work area, then
    // the streamed workspace of this batch's precision
    const size_t counters = 256 * ((8 * b->groups.size() + 255) / 256 + 1);
    const size_t tw = team ? (team_ws_bytes(b) + 255) & ~size_t(255) : 0;
    const size_t r4 = fp64 ? 32 : 16;
    const size_t fb = streamed ? r4 * 3 * (size_t)(b->NF + b->R) : 0;
    const size_t nb = streamed ? r4 * (2 * (size_t)(b->NFREE + b->R) + 2 * (size_t)b->NFREE + 1) : 0;
    const size_t fb_al = (fb + 255) & ~size_t(255);
    if (counters + tw + fb_al + nb > kStaticScratchBytes)
        return fail(RVE_EWORKSPACE, "the batch needs " + std::to_string(counters + tw + fb_al + nb) +
                                        " bytes of work area, beyond the " + std::to_string(kStaticScratchBytes) +
                                        " of the allocation-free solve");
    void* base = nullptr;
    int rc = device_scratch(b->device, &base);
    if (rc) return rc;
    char* sp = static_cast<char*>(base);
    int32_t* queues = reinterpret_cast<int32_t*>(sp);
    char* team_ws = team ? sp + counters : nullptr;
    void* ws_fib = streamed ? sp + counters + tw : nullptr;
    void* ws_node = streamed ? sp + counters + tw + fb_al : nullptr;

    hipStream_t s = (hipStream_t)b->opts.stream;
    const hipMemcpyKind in_kind = ptr_kind == RVE_PTR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const hipMemcpyKind out_kind = ptr_kind == RVE_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    HIP_TRY(hipMemcpyAsync(b->dF, F, 72 * b->R, in_kind, s));
    SolveArgs a{};
    fill_solve_args(b, a);
    a.init = b->opts.init;
    rc = launch_groups(b, a, queues, ws_fib, ws_node, team_ws, s, false, false);
    if (rc) return rc;
    b->cost_order = true;
    HIP_TRY(hipMemcpyAsync(sigma, b->dsigma, 72 * b->R, out_kind, s));
    HIP_TRY(hipMemcpyAsync(status, b->dstatus, 4 * b->R, out_kind, s));
    b->have_state = true;
    b->last_variant = false;
    ++b->generation;
    if (ptr_kind == RVE_PTR_HOST) {
        HIP_TRY(hipStreamSynchronize(s));
        return team_errors(b, team_ws);
    }
    return RVE_OK;
}
