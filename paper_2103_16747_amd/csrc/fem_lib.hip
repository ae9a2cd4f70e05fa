// libfem host side: mesh layout construction, the batch engine and the C ABI
// (include/fem.h).
//
// The host builds each mesh's tiled layout once, owns device memory, and
// enqueues rounds of kernels; every arithmetic step of the solve and every
// solver decision (Newton test, CG stop, line-search acceptance, next load
// step) is taken on the device by the kernels in fem_kernels.h. A single mesh
// handle is a batch holding one job.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <bitset>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fem.h"
#include "fem_kernels.h"
#include "layout.h"

using namespace fem;
using namespace fem_layout;

// Staging of fem_batch_get_contact_patch_noalloc: the resultant (4 doubles),
// the contact count, then per contact node its force (3 doubles), phi and
// device node id, for at most FEM_NOALLOC_MAX_CONTACT contact-eligible
// nodes. Each device holds its own copy for the life of the process.
constexpr size_t kNoAllocBytes = 64 + (size_t)FEM_NOALLOC_MAX_CONTACT * (4 * sizeof(double) + sizeof(int));
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

thread_local std::string g_last_error;

// Device address of `scratch` per device ordinal, resolved once per device
// by fem_batch_create with that device current (the host-side symbol is not
// a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return fail(e_ == hipErrorOutOfMemory ? FEM_E_OOM : FEM_E_DEVICE,                       \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                        \
    } while (0)

#define TRY(expr)               \
    do {                        \
        int rc_ = (expr);       \
        if (rc_) return rc_;    \
    } while (0)

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }
inline int pad8(int x) { return (x + 7) & ~7; }
bool is_finite(double x) { return std::isfinite(x); }

int launch_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FEM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return FEM_OK;
}

// Sub-allocations of one device allocation, 256-byte aligned.
struct Arena {
    size_t off = 0;
    template <typename T>
    size_t take(size_t count) {
        size_t at = (off + 255) & ~size_t(255);
        off = at + std::max<size_t>(count, 1) * sizeof(T);
        return at;
    }
};

// Start/stop HIP events attached to every launch of every `every`-th round
// (hipExtLaunchKernel; the other rounds replay captured graphs), harvested
// after stream synchronisations.
struct KernelTimer {
    static constexpr int kKinds = 3, kPool = 1024;
    int every = 0;
    long long rounds = 0;                     // rounds launched since timing was set
    long long seen[kKinds] = {0, 0, 0};       // launches of each kernel kind
    long long count[kKinds] = {0, 0, 0};
    double total_ms[kKinds] = {0, 0, 0};
    hipEvent_t ev[kPool][2] = {};
    int kind_of[kPool] = {};
    int used = 0;
    bool created = false;
};

// A captured round of kernels for one CG chunk length.
struct RoundGraph {
    int chunk = 0;
    int variant = 0;        // kernel instances captured (see kernel_variant)
    int groups = 1;         // job groups (streams) captured
    hipGraphExec_t exec = nullptr;
};

// One group of running jobs: its slices of the tile and node work tables and
// of the live list. A round runs each group's solver steps on a stream of its
// own (see enqueue_round).
struct JobGroup {
    int tile_off = 0, tile_n = 0, node_off = 0, node_n = 0, live_off = 0, live_n = 0;
};

// Events for the cross-stream order of one captured or launched round.
constexpr int kRoundEvents = 2 * 64 + 2;

struct TopoRec {
    int n = 0, n_free = 0, m = 0, ntile = 0, nent = 0, nc = 0, ncb = 0;
    std::vector<int> perm;     // device node id -> caller's node id (node_order())
    // order of the mesh's tile-pass and node-pass blocks in the work tables
    // (spread_order())
    std::vector<int> tile_cols, node_cols;
    void *arena = nullptr;
    uint8_t *elig = nullptr;   // device, n
    Topo<float> v32{};
    Topo<double> v64{};
};

struct InstRec {
    bool live = false;
    bool in_tables = false;   // has blocks in the current work tables
    int topo = -1;
    void *arena = nullptr;
    InstBufs<float> b32{};
    InstBufs<double> b64{};
};

}  // namespace

struct fem_batch {
    int precision = FEM_PREC_FP64;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t stream2 = nullptr;          // the second job group's stream (library-owned)
    hipEvent_t xev[kRoundEvents] = {};      // cross-stream order within a round
    bool xev_created = false;
    JobGroup grp[2];
    int ngroups = 1;
    int groups_opt = 0;                     // 2: two job groups per round; 0 or 1: one
    bool deterministic = false;             // tile partials summed in a fixed order
    int capacity = 0;
    std::vector<TopoRec> topos;
    std::vector<InstRec> insts;     // size capacity
    InstState *d_states = nullptr;
    InstState *h_states = nullptr;  // pinned mirror
    void *d_topos = nullptr, *d_bufs = nullptr;
    int2 *d_work_tile = nullptr, *d_work_node = nullptr;
    int nwork_tile = 0, nwork_node = 0, cap_work_tile = 0, cap_work_node = 0;
    int *d_live = nullptr;
    int nlive = 0;
    int n_law[2] = {0, 0};                  // running jobs per constitutive law
    int n_fric = 0;                         // running jobs with friction
    SolveParams *d_params = nullptr;
    SolveParams *h_params = nullptr;
    bool tables_dirty = true;
    void *patch = nullptr;
    size_t patch_bytes = 0;
    void *outbuf = nullptr;                 // stress / statistics outputs
    size_t outbuf_bytes = 0;
    void *h_stage = nullptr;
    size_t h_stage_bytes = 0;
    KernelTimer timer;
    bool use_graphs = true;
    int chunk = 0;                          // CG iterations per round (0 = automatic)
    int tile_tets = kTileTets, tile_nodes = kTileNodes;   // layout limits for meshes added next
    std::vector<RoundGraph> graphs;
    size_t elem() const { return precision == FEM_PREC_FP32 ? sizeof(float) : sizeof(double); }
};

// Friction settings of a job: coefficient, smoothing length and its lag state
// (lag_ok = 0: none, so the first step has no friction).
struct FrictionInit {
    double mu_f = 0.0, eps_f = 1e-5;
    int lag_ok = 0;
    double c_lag[3] = {0.0, 0.0, 0.0};
};

struct fem_mesh {
    fem_batch *batch = nullptr;
    int n = 0, m = 0;
    bool have_material = false, have_indenter = false;
    double E = 0, nu = 0, density = 0;
    double dt = 0;                  // implicit time step; 0 = quasi-static
    int model = FEM_MODEL_NEOHOOKEAN;
    FrictionInit friction;          // coefficient, slip length and lag state of the next step
    Indenter ind{};
};

namespace {

int set_device(const fem_batch *B) {
    HIP_TRY(hipSetDevice(B->device));
    return FEM_OK;
}

// With `device` current: the device address of `scratch` on it, once.
int resolve_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(FEM_E_INVALID, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return FEM_OK;
    void *ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(FEM_E_DEVICE, "no device address for the static scratch");
    g_scratch_ptr[device] = ptr;
    return FEM_OK;
}

int stage(fem_batch *B, size_t bytes) {
    if (B->h_stage_bytes >= bytes) return FEM_OK;
    if (B->h_stage) (void)hipHostFree(B->h_stage);
    B->h_stage = nullptr;
    B->h_stage_bytes = 0;
    HIP_TRY(hipHostMalloc(&B->h_stage, bytes));
    B->h_stage_bytes = bytes;
    return FEM_OK;
}

// Sampling: in a sampled round every launch gets a timer slot; the launch
// then goes through hipExtLaunchKernel with the slot's events, which take the
// dispatch's own start and end timestamps (no marker packets or cache
// maintenance of separate event records inside the measured span).
int timer_slot(fem_batch *B, int kind, bool sample) {
    KernelTimer &t = B->timer;
    if (!sample || t.used >= KernelTimer::kPool) return -1;
    const int slot = t.used++;
    t.kind_of[slot] = kind;
    return slot;
}

// Launches `kernel` plainly, or with the timer slot's start (first) and stop
// (last) events when sampled.
template <typename K, typename... Args>
void launch_timed(fem_batch *B, hipStream_t st, int slot, bool first, bool last, K kernel, dim3 grid, dim3 block,
                  Args... args) {
    if (slot < 0) {
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
        return;
    }
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, first ? B->timer.ev[slot][0] : nullptr,
                          last ? B->timer.ev[slot][1] : nullptr, 0, args...);
}

void timer_harvest(fem_batch *B) {
    KernelTimer &t = B->timer;
    for (int i = 0; i < t.used; i++) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, t.ev[i][0], t.ev[i][1]) == hipSuccess) {
            t.count[t.kind_of[i]]++;
            t.total_ms[t.kind_of[i]] += ms;
        }
    }
    t.used = 0;
}

int sync(fem_batch *B) {
    HIP_TRY(hipStreamSynchronize(B->stream));
    if (B->timer.used) timer_harvest(B);
    return FEM_OK;
}

void drop_graphs(fem_batch *B) {
    for (RoundGraph &G : B->graphs)
        if (G.exec) (void)hipGraphExecDestroy(G.exec);
    B->graphs.clear();
}

// ---------------------------------------------------------------------------
// Mesh upload: layout, rest volume check, contact-eligible nodes.
// ---------------------------------------------------------------------------
template <typename T> Topo<T> &topo_view(TopoRec &R);
template <> Topo<float> &topo_view<float>(TopoRec &R) { return R.v32; }
template <> Topo<double> &topo_view<double>(TopoRec &R) { return R.v64; }

template <typename T>
int add_topology(fem_batch *B, const double *X_in, int n, const int32_t *tets_in, int m, const uint8_t *fixed_in,
                 int *id) {
    // Everything on the device uses the node numbering of node_order(), with
    // the fixed nodes moved after the free ones (in the same order), so a CG
    // update skips whole blocks of fixed nodes.
    TopoRec R;
    R.perm = node_order(X_in, n, tets_in, m);
    std::stable_partition(R.perm.begin(), R.perm.end(), [&](int v) { return fixed_in[v] == 0; });
    int n_free = 0;
    for (int i = 0; i < n; i++) n_free += fixed_in[i] == 0;
    std::vector<int> inv(n);
    for (int i = 0; i < n; i++) inv[R.perm[i]] = i;
    std::vector<double> Xv(3 * (size_t)n);
    std::vector<uint8_t> fv(n);
    std::vector<int32_t> tv(4 * (size_t)m);
    for (int i = 0; i < n; i++) {
        for (int d = 0; d < 3; d++) Xv[3 * (size_t)i + d] = X_in[3 * (size_t)R.perm[i] + d];
        fv[i] = fixed_in[R.perm[i]];
    }
    for (size_t q = 0; q < 4 * (size_t)m; q++) tv[q] = inv[tets_in[q]];
    const double *X = Xv.data();
    const int32_t *tets = tv.data();
    const uint8_t *fixed = fv.data();
    HostLayout L;
    build_layout(X, n, tets, m, B->tile_tets, B->tile_nodes, L);
    R.n = n;
    R.m = m;
    R.ntile = L.ntile;
    R.nent = L.nent;
    Arena A;
    const size_t o_tile_tet = A.take<int>(L.ntile + 1), o_tile_ent = A.take<int>(L.ntile + 1);
    const size_t o_ent_node = A.take<int>(L.nent), o_rec = A.take<TetRec<T>>(m);
    const size_t o_neo = A.take<int>(n + 1), o_ne = A.take<int>(L.nent);
    const size_t o_fixed = A.take<uint8_t>(n), o_cn = A.take<int>(n), o_cidx = A.take<int>(n);
    const size_t o_X = A.take<double>(3 * (size_t)n), o_elig = A.take<uint8_t>(n);
    const size_t o_nvol = A.take<T>(n), o_owner = A.take<uint8_t>(L.nent), o_tid = A.take<int>(m);
    const size_t o_ent_slot = A.take<uint8_t>(L.nent), o_ne4 = A.take<int4>(n);
    std::vector<int4> ne4(n);
    for (int i = 0; i < n; i++) {
        int e[kGather];
        for (int k = 0; k < kGather; k++) {
            const int q = L.node_ent_off[i] + k;
            e[k] = q < L.node_ent_off[i + 1] ? L.node_ent[q] : -1;
        }
        ne4[i] = make_int4(e[0], e[1], e[2], e[3]);
    }
    std::vector<int> inc_off;
    std::vector<uint16_t> inc;
    build_incidence(L, inc_off, inc);
    const size_t o_inc_off = A.take<int>(L.nent + 1), o_inc = A.take<uint16_t>(4 * (size_t)m);
    // Lumped volume share per node (sum over its tets of V_e / 4, FP64 on the
    // host) and each node's first tile entry.
    std::vector<T> nvol(n, (T)0);
    {
        std::vector<double> acc(n, 0.0);
        for (int e = 0; e < m; e++) {
            const int32_t *t = tets + 4 * (size_t)e;
            double D[9];
            for (int a = 0; a < 3; a++)
                for (int i = 0; i < 3; i++) D[3 * i + a] = X[3 * (size_t)t[a + 1] + i] - X[3 * (size_t)t[0] + i];
            const double det = D[0] * (D[4] * D[8] - D[5] * D[7]) - D[1] * (D[3] * D[8] - D[5] * D[6]) +
                               D[2] * (D[3] * D[7] - D[4] * D[6]);
            for (int a = 0; a < 4; a++) acc[t[a]] += std::fabs(det) / 24.0;
        }
        for (int i = 0; i < n; i++) nvol[i] = (T)acc[i];
    }
    std::vector<uint8_t> owner(std::max(L.nent, 1), 0);
    for (int i = 0; i < n; i++)
        if (L.node_ent_off[i + 1] > L.node_ent_off[i]) owner[L.node_ent[L.node_ent_off[i]]] = 1;
    HIP_TRY(hipMalloc(&R.arena, A.off));
    char *base = (char *)R.arena;
    auto up = [&](size_t off, const void *src, size_t bytes) -> int {
        HIP_TRY(hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, B->stream));
        return FEM_OK;
    };
    int rc = FEM_OK;
    if (!rc) rc = up(o_tile_tet, L.tile_tet.data(), L.tile_tet.size() * sizeof(int));
    if (!rc) rc = up(o_tile_ent, L.tile_ent.data(), L.tile_ent.size() * sizeof(int));
    if (!rc) rc = up(o_ent_node, L.ent_node.data(), L.ent_node.size() * sizeof(int));
    if (!rc) rc = up(o_ent_slot, L.ent_slot.data(), L.ent_slot.size());
    if (!rc) rc = up(o_ne4, ne4.data(), ne4.size() * sizeof(int4));
    if (!rc) rc = up(o_neo, L.node_ent_off.data(), L.node_ent_off.size() * sizeof(int));
    if (!rc) rc = up(o_ne, L.node_ent.data(), L.node_ent.size() * sizeof(int));
    if (!rc) rc = up(o_fixed, fixed, n);
    if (!rc) rc = up(o_X, X, 3 * (size_t)n * sizeof(double));
    if (!rc) rc = up(o_nvol, nvol.data(), (size_t)n * sizeof(T));
    if (!rc) rc = up(o_owner, owner.data(), (size_t)L.nent);
    if (!rc) rc = up(o_tid, L.order.data(), (size_t)m * sizeof(int));
    if (!rc) rc = up(o_inc_off, inc_off.data(), inc_off.size() * sizeof(int));
    if (!rc) rc = up(o_inc, inc.data(), inc.size() * sizeof(uint16_t));
    // Rest volumes and boundary faces from the original connectivity.
    unsigned slots = 1;
    while (slots < 8u * (unsigned)m) slots <<= 1;
    int *d_tets = nullptr, *d_scalar = nullptr, *d_tnodes = nullptr;
    uint32_t *d_loc = nullptr;
    unsigned long long *keys = nullptr;
    unsigned *cnt = nullptr;
    uint8_t *surf = nullptr;
    const int big = 0x7fffffff;
    if (!rc && (hipMalloc(&d_tets, 4 * (size_t)m * sizeof(int)) != hipSuccess || hipMalloc(&d_scalar, 2 * sizeof(int)) != hipSuccess ||
                hipMalloc(&d_tnodes, 4 * (size_t)m * sizeof(int)) != hipSuccess ||
                hipMalloc(&d_loc, (size_t)m * sizeof(uint32_t)) != hipSuccess ||
                hipMalloc(&keys, slots * sizeof(unsigned long long)) != hipSuccess ||
                hipMalloc(&cnt, slots * sizeof(unsigned)) != hipSuccess || hipMalloc(&surf, n) != hipSuccess))
        rc = fail(FEM_E_OOM, "set-up scratch allocation failed");
    if (!rc && (hipMemcpyAsync(d_tets, tets, 4 * (size_t)m * sizeof(int), hipMemcpyHostToDevice, B->stream) != hipSuccess ||
                hipMemcpyAsync(d_tnodes, L.tet_nodes.data(), 4 * (size_t)m * sizeof(int), hipMemcpyHostToDevice, B->stream) != hipSuccess ||
                hipMemcpyAsync(d_loc, L.tet_loc.data(), (size_t)m * sizeof(uint32_t), hipMemcpyHostToDevice, B->stream) != hipSuccess ||
                hipMemcpyAsync(d_scalar, &big, sizeof(int), hipMemcpyHostToDevice, B->stream) != hipSuccess ||
                hipMemsetAsync(keys, 0xff, slots * sizeof(unsigned long long), B->stream) != hipSuccess ||
                hipMemsetAsync(cnt, 0, slots * sizeof(unsigned), B->stream) != hipSuccess ||
                hipMemsetAsync(surf, 0, n, B->stream) != hipSuccess))
        rc = fail(FEM_E_DEVICE, "set-up copies failed");
    int host[2] = {0, 0};
    if (!rc) {
        k_check_volumes<<<ceil_div(m, kBlock), kBlock, 0, B->stream>>>((const double *)(base + o_X), d_tets, m, d_scalar);
        k_rest_constants<T><<<ceil_div(m, kBlock), kBlock, 0, B->stream>>>((const double *)(base + o_X), d_tnodes, d_loc,
                                                                           m, (TetRec<T> *)(base + o_rec));
        k_faces_insert<<<ceil_div(4LL * m, kBlock), kBlock, 0, B->stream>>>(d_tets, m, keys, cnt, slots - 1);
        k_faces_mark<<<ceil_div(4LL * m, kBlock), kBlock, 0, B->stream>>>(d_tets, m, keys, cnt, slots - 1, surf);
        k_compact_eligible<<<1, 1024, 0, B->stream>>>(surf, (const uint8_t *)(base + o_fixed), n,
                                                      (uint8_t *)(base + o_elig), (int *)(base + o_cn),
                                                      (int *)(base + o_cidx), d_scalar + 1);
        rc = launch_check("mesh set-up");
    }
    if (!rc && hipMemcpyAsync(host, d_scalar, sizeof host, hipMemcpyDeviceToHost, B->stream) != hipSuccess)
        rc = fail(FEM_E_DEVICE, "copy");
    if (!rc && hipStreamSynchronize(B->stream) != hipSuccess) rc = fail(FEM_E_DEVICE, "mesh set-up failed");
    (void)hipStreamSynchronize(B->stream);
    if (d_tets) (void)hipFree(d_tets);
    if (d_tnodes) (void)hipFree(d_tnodes);
    if (d_loc) (void)hipFree(d_loc);
    if (d_scalar) (void)hipFree(d_scalar);
    if (keys) (void)hipFree(keys);
    if (cnt) (void)hipFree(cnt);
    if (surf) (void)hipFree(surf);
    if (!rc && host[0] != big) rc = fail(FEM_E_DEGENERATE, "tet " + std::to_string(host[0]) + " has rest volume <= 0");
    if (rc) {
        (void)hipFree(R.arena);
        return rc;
    }
    R.nc = host[1];
    R.ncb = ceil_div(R.nc, kBlock);
    R.n_free = n_free;
    R.tile_cols = spread_order(R.ntile, R.ncb);
    {
        // node blocks with free nodes (block 0 always runs a CG update)
        const int nb = ceil_div(n, kBlock), ncg = n_free > kBlock ? ceil_div(n_free, kBlock) : 1;
        R.node_cols = spread_order(ncg, nb - ncg);
    }
    R.elig = (uint8_t *)(base + o_elig);
    Topo<T> &v = topo_view<T>(R);
    v.n = n;
    v.n_free = n_free;
    v.m = m;
    v.ntile = L.ntile;
    v.nent = L.nent;
    v.nc = R.nc;
    v.ncb = R.ncb;
    v.tile_tet = (const int *)(base + o_tile_tet);
    v.tile_ent = (const int *)(base + o_tile_ent);
    v.ent_node = (const int *)(base + o_ent_node);
    v.ent_slot = (const uint8_t *)(base + o_ent_slot);
    v.rec = (const TetRec<T> *)(base + o_rec);
    v.node_ent_off = (const int *)(base + o_neo);
    v.node_ent = (const int *)(base + o_ne);
    v.node_ent4 = (const int4 *)(base + o_ne4);
    v.inc_off = (const int *)(base + o_inc_off);
    v.inc = (const uint16_t *)(base + o_inc);
    v.fixed = (const uint8_t *)(base + o_fixed);
    v.cnodes = (const int *)(base + o_cn);
    v.cidx = (const int *)(base + o_cidx);
    v.X = (const double *)(base + o_X);
    v.nvol = (const T *)(base + o_nvol);
    v.owner = (const uint8_t *)(base + o_owner);
    v.tet_id = (const int *)(base + o_tid);
    B->topos.push_back(R);
    B->tables_dirty = true;
    *id = (int)B->topos.size() - 1;
    return FEM_OK;
}

// ---------------------------------------------------------------------------
// Instances
// ---------------------------------------------------------------------------
template <typename T> InstBufs<T> &inst_view(InstRec &R);
template <> InstBufs<float> &inst_view<float>(InstRec &R) { return R.b32; }
template <> InstBufs<double> &inst_view<double>(InstRec &R) { return R.b64; }

template <typename T>
int alloc_instance(fem_batch *B, int slot, int topo) {
    const TopoRec &tp = B->topos[topo];
    const int n = tp.n;
    const int stride = std::max(tp.ntile + tp.ncb, kWaves * ceil_div(n, kBlock));   // node pass: partials per wavefront
    Arena A;
    size_t o[7];
    for (int k = 0; k < 6; k++) o[k] = A.take<T>(3 * (size_t)n);
    o[6] = A.take<T>(6 * (size_t)n);
    const size_t o_pg = A.take<T>(9 * (size_t)tp.nent), o_pq = A.take<T>(3 * (size_t)tp.nent);
    const size_t o_cp = A.take<T>(9 * (size_t)std::max(tp.nc, 1)), o_q = A.take<T>(3 * (size_t)n);
    const size_t o_red = A.take<double>(RS_COUNT * (size_t)stride);
    const size_t o_v = A.take<T>(3 * (size_t)n), o_ut = A.take<T>(3 * (size_t)n);
    const size_t o_fr = A.take<double>(8 * (size_t)std::max(tp.nc, 1));
    const size_t o_hist = A.take<signed char>(kHistSteps);
    const size_t o_cact = A.take<uint8_t>(std::max(tp.nc, 1));
    InstRec &R = B->insts[slot];
    HIP_TRY(hipMalloc(&R.arena, A.off));
    HIP_TRY(hipMemsetAsync(R.arena, 0, A.off, B->stream));
    char *base = (char *)R.arena;
    InstBufs<T> &b = inst_view<T>(R);
    b.topo = topo;
    b.red_stride = stride;
    T **vec[6] = {&b.u, &b.dx, &b.g, &b.r, &b.z, &b.p};
    for (int k = 0; k < 6; k++) *vec[k] = (T *)(base + o[k]);
    b.dinv = (T *)(base + o[6]);
    b.pg = (T *)(base + o_pg);
    b.pq = (T *)(base + o_pq);
    b.cp = (T *)(base + o_cp);
    b.qout = (T *)(base + o_q);
    b.red = (double *)(base + o_red);
    b.v = (T *)(base + o_v);
    b.ut = (T *)(base + o_ut);
    b.fr = (double *)(base + o_fr);
    b.hist = (signed char *)(base + o_hist);
    b.cact = (uint8_t *)(base + o_cact);
    b.s = B->d_states + slot;
    R.topo = topo;
    R.live = true;
    B->tables_dirty = true;
    return FEM_OK;
}

void free_instance(fem_batch *B, int slot) {
    InstRec &R = B->insts[slot];
    if (R.arena) (void)hipFree(R.arena);
    R = InstRec();
    B->tables_dirty = true;
}

inline bool running_phase(int ph) { return ph != PH_IDLE && ph != PH_DONE; }

// Work tables: tile (+ contact) blocks and node blocks of every running
// instance (as of the host's last view of the states), ordered tile-major so
// one tile of consecutive instances is processed back to back (on one XCD,
// see logical_block()), the tiles of each mesh taken in spread_order(), so
// that every XCD's share holds its share of the heavy blocks. Finished instances are left out, so their blocks
// cost nothing; one made to run again (restart) is put back by the next run.
// Mesh and buffer descriptors are uploaded again only after a structural
// change (mesh or job added or removed).
template <typename T>
int rebuild_tables(fem_batch *B) {
    std::vector<int2> wt, wn;
    std::vector<int> live;
    std::vector<int> members[2];
    for (int i = 0; i < B->capacity; i++) {
        InstRec &R = B->insts[i];
        R.in_tables = R.live && running_phase(B->h_states[i].phase);
        if (!R.in_tables) continue;
        live.push_back(i);
    }
    // Two groups only on request (on the 256-job fingertip batch they run
    // within the run-to-run spread of one group, the node pass of one group
    // taking wave slots from the other's tile pass): jobs dealt to the group
    // with fewer tile blocks so far.
    const int ng = B->groups_opt == 2 && live.size() >= 2 ? 2 : 1;
    long long load[2] = {0, 0};
    for (int i : live) {
        const TopoRec &tp = B->topos[B->insts[i].topo];
        const int g = ng == 2 && load[1] < load[0] ? 1 : 0;
        members[g].push_back(i);
        load[g] += tp.ntile + tp.ncb;
    }
    live.clear();
    for (int g = 0; g < ng; g++) {
        JobGroup &G = B->grp[g];
        int max_t = 0, max_nb = 0;
        for (int i : members[g]) {
            const TopoRec &tp = B->topos[B->insts[i].topo];
            max_t = std::max(max_t, tp.ntile + tp.ncb);
            max_nb = std::max(max_nb, ceil_div(tp.n, kBlock));
        }
        G.tile_off = (int)wt.size();
        for (int c = 0; c < max_t; c++)
            for (int i : members[g]) {
                const TopoRec &tp = B->topos[B->insts[i].topo];
                if (c < tp.ntile + tp.ncb) wt.push_back(make_int2(i, tp.tile_cols[c]));
            }
        G.tile_n = (int)wt.size() - G.tile_off;
        G.node_off = (int)wn.size();
        for (int c = 0; c < max_nb; c++)
            for (int i : members[g]) {
                const TopoRec &tp = B->topos[B->insts[i].topo];
                if (c < ceil_div(tp.n, kBlock)) wn.push_back(make_int2(i, tp.node_cols[c]));
            }
        G.node_n = (int)wn.size() - G.node_off;
        G.live_off = (int)live.size();
        live.insert(live.end(), members[g].begin(), members[g].end());
        G.live_n = (int)members[g].size();
    }
    B->ngroups = ng;
    auto upload = [&](const std::vector<int2> &v, int2 *&d, int &cap, int &count) -> int {
        if ((int)v.size() > cap) {
            if (d) (void)hipFree(d);
            d = nullptr;
            cap = std::max<int>((int)v.size(), 64);
            HIP_TRY(hipMalloc(&d, cap * sizeof(int2)));
        }
        if (!v.empty()) HIP_TRY(hipMemcpyAsync(d, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice, B->stream));
        count = (int)v.size();
        return FEM_OK;
    };
    drop_graphs(B);
    TRY(upload(wt, B->d_work_tile, B->cap_work_tile, B->nwork_tile));
    TRY(upload(wn, B->d_work_node, B->cap_work_node, B->nwork_node));
    B->nlive = (int)live.size();
    if (!live.empty())
        HIP_TRY(hipMemcpyAsync(B->d_live, live.data(), live.size() * sizeof(int), hipMemcpyHostToDevice, B->stream));
    if (B->tables_dirty) {
        std::vector<Topo<T>> tv;
        for (TopoRec &R : B->topos) tv.push_back(topo_view<T>(R));
        TRY(sync(B));
        if (B->d_topos) (void)hipFree(B->d_topos);
        B->d_topos = nullptr;
        HIP_TRY(hipMalloc(&B->d_topos, std::max<size_t>(tv.size(), 1) * sizeof(Topo<T>)));
        if (!tv.empty())
            HIP_TRY(hipMemcpyAsync(B->d_topos, tv.data(), tv.size() * sizeof(Topo<T>), hipMemcpyHostToDevice, B->stream));
        std::vector<InstBufs<T>> bv(B->capacity);
        for (int i = 0; i < B->capacity; i++) bv[i] = inst_view<T>(B->insts[i]);
        HIP_TRY(hipMemcpyAsync(B->d_bufs, bv.data(), bv.size() * sizeof(InstBufs<T>), hipMemcpyHostToDevice, B->stream));
        TRY(sync(B));
    } else {
        TRY(sync(B));
    }
    B->tables_dirty = false;
    return FEM_OK;
}

int params_to_device(fem_batch *B, const fem_solve_params &P) {
    SolveParams &d = *B->h_params;
    d.newton_rtol = P.newton_rtol;
    d.newton_atol = P.newton_atol;
    d.cg_rtol = P.cg_rtol;
    d.cg_eta_max = P.cg_eta_max;
    d.eta_power = P.cg_eta_power;
    d.c1 = P.c1;
    d.floor_rtol = P.newton_floor_rtol;
    d.noise_eps = 16.0 * (B->precision == FEM_PREC_FP32 ? (double)std::numeric_limits<float>::epsilon()
                                                        : std::numeric_limits<double>::epsilon());
    d.max_newton = P.max_newton;
    d.max_cg = P.max_cg;
    d.block_jacobi = P.precond == FEM_PRECOND_BLOCK ? 1 : 0;
    d.contact_full = P.contact_hessian ? 1 : 0;
    d.max_halvings = P.max_halvings;
    HIP_TRY(hipMemcpyAsync(B->d_params, B->h_params, sizeof(SolveParams), hipMemcpyHostToDevice, B->stream));
    return sync(B);
}

int read_states(fem_batch *B) {
    HIP_TRY(hipMemcpyAsync(B->h_states, B->d_states, B->capacity * sizeof(InstState), hipMemcpyDeviceToHost, B->stream));
    return sync(B);
}

int write_state(fem_batch *B, int slot) {
    HIP_TRY(hipMemcpyAsync(B->d_states + slot, B->h_states + slot, sizeof(InstState), hipMemcpyHostToDevice, B->stream));
    return sync(B);
}

// One solver step of one job group on stream st: a tile pass (one launch per
// constitutive law present; blocks of jobs on the other law return at once),
// a node pass (the friction instance only when a job needs it) and a
// finalize. Returns after enqueueing the tile pass through `after_tile`, so
// the caller can order the other group's tile pass behind it.
template <typename T>
void enqueue_step(fem_batch *B, const JobGroup &G, hipStream_t st, bool sample, hipEvent_t after_tile) {
    const Topo<T> *tp = (const Topo<T> *)B->d_topos;
    const InstBufs<T> *bf = (const InstBufs<T> *)B->d_bufs;
    const int2 *wt = (const int2 *)B->d_work_tile + G.tile_off, *wn = (const int2 *)B->d_work_node + G.node_off;
    const int *lv = (const int *)B->d_live + G.live_off;
    const SolveParams *P = (const SolveParams *)B->d_params;
    const int gt = pad8(G.tile_n), gn = pad8(G.node_n), nl = G.live_n;
    const bool nh = B->n_law[0] > 0, cr = B->n_law[1] > 0, fric = B->n_fric > 0;
    int slot = timer_slot(B, FEM_KERNEL_TILE, sample);
    if (B->deterministic) {
        if (nh) launch_timed(B, st, slot, true, !cr, k_tile<T, LAW_NH, true>, dim3(gt), dim3(kBlock), tp, bf, wt, G.tile_n, P);
        if (cr) launch_timed(B, st, slot, !nh, true, k_tile<T, LAW_CR, true>, dim3(gt), dim3(kBlock), tp, bf, wt, G.tile_n, P);
    } else {
        if (nh) launch_timed(B, st, slot, true, !cr, k_tile<T, LAW_NH, false>, dim3(gt), dim3(kBlock), tp, bf, wt, G.tile_n, P);
        if (cr) launch_timed(B, st, slot, !nh, true, k_tile<T, LAW_CR, false>, dim3(gt), dim3(kBlock), tp, bf, wt, G.tile_n, P);
    }
    if (after_tile) (void)hipEventRecord(after_tile, st);
    slot = timer_slot(B, FEM_KERNEL_NODE, sample);
    if (fric)
        launch_timed(B, st, slot, true, true, k_node<T, true>, dim3(gn), dim3(kBlock), tp, bf, wn, G.node_n, P);
    else
        launch_timed(B, st, slot, true, true, k_node<T, false>, dim3(gn), dim3(kBlock), tp, bf, wn, G.node_n, P);
    slot = timer_slot(B, FEM_KERNEL_FINALIZE, sample);
    launch_timed(B, st, slot, true, true, k_finalize<T>, dim3(nl), dim3(64), tp, bf, lv, nl, P);
}

// One round: C solver steps of every job group. With one group the steps run
// on the batch stream. With two, group 0 runs on the batch stream and group 1
// on the second stream, each group's steps in order, and the tile passes of
// the two groups alternate (group 1's step c after group 0's tile pass c,
// group 0's step c + 1 after group 1's tile pass c): a group's node pass,
// bound by memory bandwidth, then overlaps the other group's tile pass, bound
// by vector arithmetic. The round ends with the second stream joined back.
template <typename T>
int enqueue_round(fem_batch *B, int chunk, bool sample) {
    if (B->ngroups == 1) {
        for (int c = 0; c < chunk; c++) enqueue_step<T>(B, B->grp[0], B->stream, sample, nullptr);
        return launch_check("round");
    }
    hipStream_t s0 = B->stream, s1 = B->stream2;
    hipEvent_t *ev = B->xev;   // [0] fork, [1] join, then two per step
    HIP_TRY(hipEventRecord(ev[0], s0));
    HIP_TRY(hipStreamWaitEvent(s1, ev[0], 0));
    for (int c = 0; c < chunk; c++) {
        hipEvent_t tile0 = ev[2 + 2 * c], tile1 = ev[3 + 2 * c];
        if (c > 0) HIP_TRY(hipStreamWaitEvent(s0, ev[3 + 2 * (c - 1)], 0));
        enqueue_step<T>(B, B->grp[0], s0, sample, tile0);
        HIP_TRY(hipStreamWaitEvent(s1, tile0, 0));
        enqueue_step<T>(B, B->grp[1], s1, sample, tile1);
    }
    HIP_TRY(hipEventRecord(ev[1], s1));
    HIP_TRY(hipStreamWaitEvent(s0, ev[1], 0));
    return launch_check("round");
}

// Kernel instances a round needs, from the host's view of the running jobs
// (laws present, friction present), as bits 1 (Neo-Hookean), 2
// (co-rotational), 4 (friction). A job's law and friction are set with its
// state by the host, so this view is current at every round.
int kernel_variant(fem_batch *B) {
    B->n_law[0] = B->n_law[1] = 0;
    B->n_fric = 0;
    for (int i = 0; i < B->capacity; i++) {
        if (!B->insts[i].live || !B->insts[i].in_tables || !running_phase(B->h_states[i].phase)) continue;
        B->n_law[B->h_states[i].model == LAW_CR ? 1 : 0]++;
        if (B->h_states[i].mu_f > 0.0) B->n_fric++;
    }
    return (B->n_law[0] > 0 ? 1 : 0) | (B->n_law[1] > 0 ? 2 : 0) | (B->n_fric > 0 ? 4 : 0) |
           (B->deterministic ? 8 : 0);
}

// Launches a round, replaying a captured graph for its length when graphs are
// on (lengths rounded up to a multiple of 4, of 8 above 32; at most 64 solver
// steps). With kernel timing on, every `every`-th round is launched kernel by
// kernel so its launches can carry events (event records cannot be captured
// into the graph here); the others replay graphs as without timing.
template <typename T>
int launch_round(fem_batch *B, int chunk) {
    if (pad8(B->nwork_tile) == 0 || pad8(B->nwork_node) == 0 || B->nlive == 0) return FEM_OK;
    const int variant = kernel_variant(B);
    KernelTimer &tm = B->timer;
    const bool timing = tm.every > 0;
    const bool sample = timing && (tm.rounds++ % tm.every) == 0;
    if (!B->use_graphs || sample) {
        const int c = std::max(1, std::min(64, chunk));
        TRY(enqueue_round<T>(B, c, sample));
        if (timing)
            for (int k = 0; k < KernelTimer::kKinds; k++) tm.seen[k] += (long long)c * B->ngroups;
        return FEM_OK;
    }
    // graph lengths: multiples of 4 up to 32, of 8 up to 64
    int c = std::max(4, std::min(64, chunk));
    c = c <= 32 ? (c + 3) / 4 * 4 : (c + 7) / 8 * 8;
    int gi = -1;
    for (int i = 0; i < (int)B->graphs.size(); i++)
        if (B->graphs[i].chunk == c && B->graphs[i].variant == variant && B->graphs[i].groups == B->ngroups) gi = i;
    if (gi < 0) {
        RoundGraph G;
        G.chunk = c;
        G.variant = variant;
        G.groups = B->ngroups;
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_round<T>(B, c, false);
        const hipError_t ec = hipStreamEndCapture(B->stream, &graph);
        if (rc) return rc;
        if (ec != hipSuccess) return fail(FEM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
        const hipError_t ei = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(FEM_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
        B->graphs.push_back(G);
        gi = (int)B->graphs.size() - 1;
    }
    HIP_TRY(hipGraphLaunch(B->graphs[gi].exec, B->stream));
    if (timing)
        for (int k = 0; k < KernelTimer::kKinds; k++) tm.seen[k] += (long long)c * B->ngroups;
    return FEM_OK;
}

// Advances every running job until all are done or max_rounds rounds ran.
template <typename T>
int run_impl(fem_batch *B, int max_rounds, int *n_running) {
    int rounds = 0, running = 0;
    TRY(read_states(B));
    for (;;) {
        running = 0;
        int single = -1, dead = 0;
        bool missing = false;
        for (int i = 0; i < B->capacity; i++) {
            const InstRec &R = B->insts[i];
            if (!R.live) continue;
            if (running_phase(B->h_states[i].phase)) {
                running++;
                single = i;
                missing = missing || !R.in_tables;
            } else if (R.in_tables) {
                dead += B->topos[R.topo].ntile + B->topos[R.topo].ncb;
            }
        }
        if (running == 0 || (max_rounds > 0 && rounds >= max_rounds)) break;
        // Finished jobs leave the tables once they hold a quarter of the tile
        // blocks (a geometric number of rebuilds over a batch's tail).
        if (B->tables_dirty || missing || 4 * dead > B->nwork_tile) TRY(rebuild_tables<T>(B));
        // Solver steps per round: a fixed 16 for batches; for one job, what
        // its current Newton iteration is expected to need (CG iterations of
        // the previous solve, plus the line-search trial and the init).
        int chunk = B->chunk > 0 ? B->chunk : 16;
        if (running == 1 && B->chunk <= 0) {
            const InstState &s = B->h_states[single];
            const int expect = s.last_cg > 0 ? s.last_cg : 16;
            chunk = s.phase == PH_CG ? expect - s.cg_it + 2 : expect + 3;
        }
        TRY(launch_round<T>(B, chunk));
        TRY(read_states(B));
        rounds++;
    }
    if (n_running) *n_running = running;
    return FEM_OK;
}

int run(fem_batch *B, int max_rounds, int *n_running) {
    return B->precision == FEM_PREC_FP32 ? run_impl<float>(B, max_rounds, n_running)
                                         : run_impl<double>(B, max_rounds, n_running);
}

// ---------------------------------------------------------------------------
// Host <-> device node vectors in the batch precision
// ---------------------------------------------------------------------------
// Node vectors (n x 3) between the caller's numbering and the device's
// (perm[device id] = caller id), converted to the batch precision.
int upload_nodes(fem_batch *B, const std::vector<int> &perm, void *dst, const double *src) {
    const size_t n = perm.size();
    TRY(stage(B, std::max<size_t>(3 * n * 8, 64)));
    if (B->precision == FEM_PREC_FP32) {
        float *h = (float *)B->h_stage;
        for (size_t i = 0; i < n; i++)
            for (int d = 0; d < 3; d++) h[3 * i + d] = (float)src[3 * (size_t)perm[i] + d];
    } else {
        double *h = (double *)B->h_stage;
        for (size_t i = 0; i < n; i++)
            for (int d = 0; d < 3; d++) h[3 * i + d] = src[3 * (size_t)perm[i] + d];
    }
    HIP_TRY(hipMemcpyAsync(dst, B->h_stage, 3 * n * B->elem(), hipMemcpyHostToDevice, B->stream));
    return sync(B);
}

int download_nodes(fem_batch *B, const std::vector<int> &perm, double *dst, const void *src) {
    const size_t n = perm.size();
    TRY(stage(B, std::max<size_t>(3 * n * 8, 64)));
    HIP_TRY(hipMemcpyAsync(B->h_stage, src, 3 * n * B->elem(), hipMemcpyDeviceToHost, B->stream));
    TRY(sync(B));
    if (B->precision == FEM_PREC_FP32) {
        const float *h = (const float *)B->h_stage;
        for (size_t i = 0; i < n; i++)
            for (int d = 0; d < 3; d++) dst[3 * (size_t)perm[i] + d] = (double)h[3 * i + d];
    } else {
        const double *h = (const double *)B->h_stage;
        for (size_t i = 0; i < n; i++)
            for (int d = 0; d < 3; d++) dst[3 * (size_t)perm[i] + d] = h[3 * i + d];
    }
    return FEM_OK;
}

enum { V_U = 0, V_G, V_Z, V_P, V_Q, V_V, V_UT };

void *inst_ptr(fem_batch *B, int slot, int which) {
    InstRec &R = B->insts[slot];
    if (B->precision == FEM_PREC_FP32) {
        InstBufs<float> &b = R.b32;
        float *p[] = {b.u, b.g, b.z, b.p, b.qout, b.v, b.ut};
        return p[which];
    }
    InstBufs<double> &b = R.b64;
    double *p[] = {b.u, b.g, b.z, b.p, b.qout, b.v, b.ut};
    return p[which];
}

// Velocity of a job at the end of its last completed step, in the caller's
// numbering: the stored velocity plus the update the next step would make,
// v + (u - ut) / dt (zero for quasi-static jobs).
int download_velocity(fem_batch *B, int slot, double *v) {
    const std::vector<int> &perm = B->topos[B->insts[slot].topo].perm;
    const size_t n = perm.size();
    const double dt = B->h_states[slot].dt;
    if (!(dt > 0.0)) {
        std::fill(v, v + 3 * n, 0.0);
        return FEM_OK;
    }
    std::vector<double> u(3 * n), ut(3 * n);
    TRY(download_nodes(B, perm, v, inst_ptr(B, slot, V_V)));
    TRY(download_nodes(B, perm, u.data(), inst_ptr(B, slot, V_U)));
    TRY(download_nodes(B, perm, ut.data(), inst_ptr(B, slot, V_UT)));
    for (size_t q = 0; q < 3 * n; q++) v[q] += (u[q] - ut[q]) / dt;
    return FEM_OK;
}

// ---------------------------------------------------------------------------
// Batch life cycle
// ---------------------------------------------------------------------------
void batch_release(fem_batch *B) {
    if (!B) return;
    (void)hipSetDevice(B->device);
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    drop_graphs(B);
    for (int i = 0; i < (int)B->insts.size(); i++) free_instance(B, i);
    for (TopoRec &R : B->topos)
        if (R.arena) (void)hipFree(R.arena);
    if (B->timer.created)
        for (int i = 0; i < KernelTimer::kPool; i++) {
            (void)hipEventDestroy(B->timer.ev[i][0]);
            (void)hipEventDestroy(B->timer.ev[i][1]);
        }
    void *dev[] = {B->d_states, B->d_topos, B->d_bufs, B->d_work_tile, B->d_work_node, B->d_live, B->d_params,
                   B->patch, B->outbuf};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    if (B->h_states) (void)hipHostFree(B->h_states);
    if (B->h_params) (void)hipHostFree(B->h_params);
    if (B->h_stage) (void)hipHostFree(B->h_stage);
    if (B->own_stream && B->stream) (void)hipStreamDestroy(B->stream);
    if (B->stream2) (void)hipStreamDestroy(B->stream2);
    if (B->xev_created)
        for (hipEvent_t e : B->xev) (void)hipEventDestroy(e);
    delete B;
}

int batch_create(const fem_config *cfg, int capacity, fem_batch **out) {
    *out = nullptr;
    fem_config c = {FEM_PREC_FP64, 0, nullptr};
    if (cfg) c = *cfg;
    if (c.precision != FEM_PREC_FP64 && c.precision != FEM_PREC_FP32) return fail(FEM_E_INVALID, "bad precision");
    if (capacity < 1 || capacity > 65536) return fail(FEM_E_INVALID, "max_jobs must be in 1..65536");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(FEM_E_DEVICE, "no HIP device");
    if (c.device < 0 || c.device >= ndev) return fail(FEM_E_INVALID, "bad device ordinal");
    fem_batch *B = new (std::nothrow) fem_batch();
    if (!B) return fail(FEM_E_OOM, "host allocation failed");
    B->precision = c.precision;
    B->device = c.device;
    B->capacity = capacity;
    B->insts.resize(capacity);
    int rc = set_device(B);
    if (!rc) rc = resolve_scratch(B->device);
    if (!rc) {
        if (c.stream) {
            B->stream = (hipStream_t)c.stream;
        } else if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) == hipSuccess) {
            B->own_stream = true;
        } else {
            rc = fail(FEM_E_DEVICE, "stream creation failed");
        }
    }
    if (!rc && hipStreamCreateWithFlags(&B->stream2, hipStreamNonBlocking) != hipSuccess)
        rc = fail(FEM_E_DEVICE, "stream creation failed");
    if (!rc) {
        for (hipEvent_t &e : B->xev)
            if (!rc && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                rc = fail(FEM_E_DEVICE, "event creation failed");
        B->xev_created = true;
    }
    const size_t bufs_bytes = (size_t)capacity * std::max(sizeof(InstBufs<float>), sizeof(InstBufs<double>));
    if (!rc && hipMalloc(&B->d_states, capacity * sizeof(InstState)) != hipSuccess) rc = fail(FEM_E_OOM, "states");
    if (!rc && hipMemset(B->d_states, 0, capacity * sizeof(InstState)) != hipSuccess) rc = fail(FEM_E_DEVICE, "memset");
    if (!rc && hipMalloc(&B->d_bufs, bufs_bytes) != hipSuccess) rc = fail(FEM_E_OOM, "views");
    if (!rc && hipMalloc(&B->d_params, sizeof(SolveParams)) != hipSuccess) rc = fail(FEM_E_OOM, "params");
    if (!rc && hipMalloc(&B->d_live, capacity * sizeof(int)) != hipSuccess) rc = fail(FEM_E_OOM, "live list");
    if (!rc && hipHostMalloc(&B->h_states, capacity * sizeof(InstState)) != hipSuccess) rc = fail(FEM_E_OOM, "pinned");
    if (!rc && hipHostMalloc(&B->h_params, sizeof(SolveParams)) != hipSuccess) rc = fail(FEM_E_OOM, "pinned");
    if (!rc) {
        std::memset(B->h_states, 0, capacity * sizeof(InstState));
        std::memset(B->h_params, 0, sizeof(SolveParams));
        rc = stage(B, 4096);
    }
    if (rc) {
        std::string msg = g_last_error;
        batch_release(B);
        g_last_error = msg;
        return rc;
    }
    *out = B;
    return FEM_OK;
}

int check_mesh_args(const double *X, int32_t n_nodes, const int32_t *tets, int32_t n_tets, const uint8_t *fixed) {
    if (!X || !tets || !fixed) return fail(FEM_E_INVALID, "null input array");
    if (n_nodes <= 0 || n_tets <= 0) return fail(FEM_E_INVALID, "empty mesh");
    if (n_nodes >= (1 << 21)) return fail(FEM_E_INVALID, "n_nodes must be below 2^21");
    if (n_tets >= (1 << 28)) return fail(FEM_E_INVALID, "too many tets");
    for (long long i = 0; i < 3LL * n_nodes; i++)
        if (!is_finite(X[i])) return fail(FEM_E_INVALID, "non-finite node coordinate");
    for (long long i = 0; i < 4LL * n_tets; i++)
        if (tets[i] < 0 || tets[i] >= n_nodes) return fail(FEM_E_INVALID, "tet index out of range");
    for (long long e = 0; e < n_tets; e++)
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < a; b++)
                if (tets[4 * e + a] == tets[4 * e + b]) return fail(FEM_E_DEGENERATE, "tet with a repeated node");
    return FEM_OK;
}

int check_indenter(int32_t kind, const double *shape, int32_t n_shape, const double *R, const double *c, double k,
                   Indenter *out) {
    if (!shape || !R || !c) return fail(FEM_E_INVALID, "null argument");
    static const int need[4] = {1, 2, 3, 2};
    if (kind < 0 || kind > 3) return fail(FEM_E_INVALID, "bad indenter kind");
    if (n_shape < need[kind]) return fail(FEM_E_INVALID, "too few shape values");
    for (int i = 0; i < need[kind]; i++)
        if (!is_finite(shape[i]) || !(shape[i] > 0)) return fail(FEM_E_INVALID, "shape values must be positive");
    if (kind == FEM_RING && !(shape[1] < shape[0])) return fail(FEM_E_INVALID, "ring needs minor < major radius");
    for (int i = 0; i < 9; i++)
        if (!is_finite(R[i])) return fail(FEM_E_INVALID, "non-finite rotation");
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            const double s = R[i] * R[j] + R[3 + i] * R[3 + j] + R[6 + i] * R[6 + j];
            if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-9) return fail(FEM_E_INVALID, "R is not orthonormal");
        }
    const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                       R[2] * (R[3] * R[7] - R[4] * R[6]);
    if (det < 0) return fail(FEM_E_INVALID, "R is a reflection");
    if (!is_finite(c[0]) || !is_finite(c[1]) || !is_finite(c[2]) || !is_finite(k) || k < 0)
        return fail(FEM_E_INVALID, "bad centre or penalty");
    Indenter ind{};
    ind.kind = kind;
    for (int i = 0; i < 4; i++) ind.shape[i] = i < need[kind] ? shape[i] : 0.0;
    for (int i = 0; i < 9; i++) ind.R[i] = R[i];
    for (int i = 0; i < 3; i++) ind.c[i] = c[i];
    ind.k = k;
    *out = ind;
    return FEM_OK;
}

int check_friction(double mu_f, double eps) {
    if (!is_finite(mu_f) || mu_f < 0.0) return fail(FEM_E_INVALID, "friction coefficient must be finite and >= 0");
    if (mu_f > 0.0 && !(is_finite(eps) && eps > 0.0)) return fail(FEM_E_INVALID, "friction needs a slip length > 0");
    return FEM_OK;
}

int check_material(double E, double nu, double density) {
    if (!is_finite(E) || !is_finite(nu) || !is_finite(density) || !(E > 0) || !(nu > -1.0) || !(nu < 0.5) ||
        density < 0)
        return fail(FEM_E_INVALID, "need E > 0, -1 < nu < 0.5, density >= 0");
    return FEM_OK;
}

int check_params(const fem_solve_params &P) {
    if (!(P.newton_rtol >= 0) || !(P.newton_atol >= 0) || P.max_newton < 0 || !(P.cg_rtol > 0) ||
        !(P.cg_eta_max >= P.cg_rtol) || !(P.cg_eta_power > 0.0 && P.cg_eta_power <= 1.0) || P.max_cg < 1 || (P.precond != 0 && P.precond != 1) || !(P.c1 >= 0) ||
        !(P.c1 < 1) || P.max_halvings < 0 || P.max_halvings > 200 || !(P.newton_floor_rtol >= 0) ||
        !(P.newton_floor_rtol < 1))
        return fail(FEM_E_INVALID, "invalid solve parameters");
    return FEM_OK;
}

// A job's initial state: material, pose schedule, counters, phase GRAD.
// A batch job's friction: its lag state at the start is u = 0 with the
// indenter at c0.
FrictionInit job_friction(const fem_indentation *job) {
    FrictionInit f;
    f.mu_f = job->friction;
    f.eps_f = job->friction > 0.0 ? job->friction_eps : 1e-5;
    f.lag_ok = 1;
    for (int d = 0; d < 3; d++) f.c_lag[d] = job->c0[d];
    return f;
}

void init_job_state(InstState &s, double E, double nu, const Indenter &ind, const double c0[3], const double dir[3],
                    double depth, int steps, double dt, double rho, int model, const FrictionInit &fr) {
    std::memset(&s, 0, sizeof s);
    s.model = model;
    s.mu_f = fr.mu_f;
    s.eps_f = fr.eps_f;
    s.lag_ok = fr.lag_ok;
    for (int d = 0; d < 3; d++) s.c_lag[d] = fr.c_lag[d];
    s.dt = dt;
    s.rho = rho;
    s.mdt2 = dt > 0.0 ? rho / (dt * dt) : 0.0;
    s.mu = E / (2.0 * (1.0 + nu));
    s.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    s.ind = ind;
    for (int d = 0; d < 3; d++) {
        s.c0[d] = c0[d];
        s.dir[d] = dir[d];
    }
    s.depth = depth;
    s.steps = steps;
    s.step = 1;
    const double f = depth / (double)steps;
    for (int d = 0; d < 3; d++) s.ind.c[d] = c0[d] + f * dir[d];
    s.step_started = 1;
    s.after_lag = PH_GRAD;
    s.phase = s.mu_f > 0.0 ? PH_LAG : PH_GRAD;
}

void fill_step_info(const InstState &s, int m, fem_step_info *info) {
    info->status = s.last_status;
    info->newton_iters = s.st_newton;
    info->cg_iters = s.st_cg;
    info->ls_trials = s.st_ls;
    info->grad_passes = s.st_grad;
    info->hv_products = s.st_hv;
    info->g0_norm = s.st_g0;
    info->g_norm = s.st_g;
    info->energy = s.E;
    info->min_J = s.minJ;
    info->tet_updates = (int64_t)m * (int64_t)(s.st_grad + s.st_hv);
}

// Staging of the contact patch kernel in a buffer of `cap` contact slots:
// resultant (4 doubles), count, then forces (3 cap doubles), phi (cap
// doubles) and device node ids (cap ints).
struct PatchStage {
    double *F, *f, *phi;
    int *count, *ids;
    PatchStage(void *base, size_t cap) {
        char *b = (char *)base;
        F = (double *)b;
        count = (int *)(b + 32);
        f = (double *)(b + 64);
        phi = f + 3 * cap;
        ids = (int *)(phi + cap);
    }
};

// Runs the contact patch kernel of one instance into `st` and reads the
// count and resultant back (the kernel writes every slot it reports and
// clears the count and resultant itself).
int contact_patch_launch(fem_batch *B, int slot, const PatchStage &st, int *count, double Ft[3]) {
    if (B->precision == FEM_PREC_FP32)
        k_contact_patch<float><<<1, 1024, 0, B->stream>>>((const Topo<float> *)B->d_topos,
                                                            (const InstBufs<float> *)B->d_bufs, slot, st.ids, st.f,
                                                            st.phi, st.count, st.F);
    else
        k_contact_patch<double><<<1, 1024, 0, B->stream>>>((const Topo<double> *)B->d_topos,
                                                             (const InstBufs<double> *)B->d_bufs, slot, st.ids, st.f,
                                                             st.phi, st.count, st.F);
    TRY(launch_check("k_contact_patch"));
    HIP_TRY(hipMemcpyAsync(count, st.count, sizeof(int), hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipMemcpyAsync(Ft, st.F, 3 * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    return sync(B);
}

int contact_patch_impl(fem_batch *B, int slot, int32_t *ids, double *f, double *phi, int32_t capacity,
                       int32_t *n_contact, double F_total[3]) {
    const int n = B->topos[B->insts[slot].topo].n;
    const size_t need = 64 + (size_t)n * (sizeof(int) + 4 * sizeof(double)) + 256;
    if (B->patch_bytes < need) {
        if (B->patch) (void)hipFree(B->patch);
        B->patch = nullptr;
        B->patch_bytes = 0;
        HIP_TRY(hipMalloc(&B->patch, need));
        B->patch_bytes = need;
    }
    if (B->tables_dirty) TRY(B->precision == FEM_PREC_FP32 ? rebuild_tables<float>(B) : rebuild_tables<double>(B));
    const PatchStage st(B->patch, (size_t)n);
    double *d_f = st.f, *d_phi = st.phi;
    int *d_ids = st.ids;
    int count = 0;
    double Ft[3];
    TRY(contact_patch_launch(B, slot, st, &count, Ft));
    *n_contact = count;
    if (F_total) std::memcpy(F_total, Ft, sizeof Ft);
    if (capacity < count) return fail(FEM_E_BUFFER, "capacity below the contact count");
    if (count > 0 && (ids || f || phi)) {
        // Device node ids -> caller ids, listed in ascending caller order.
        std::vector<int> hid(count);
        std::vector<double> hf(3 * (size_t)count), hphi(count);
        HIP_TRY(hipMemcpyAsync(hid.data(), d_ids, count * sizeof(int), hipMemcpyDeviceToHost, B->stream));
        HIP_TRY(hipMemcpyAsync(hf.data(), d_f, 3 * (size_t)count * sizeof(double), hipMemcpyDeviceToHost, B->stream));
        HIP_TRY(hipMemcpyAsync(hphi.data(), d_phi, count * sizeof(double), hipMemcpyDeviceToHost, B->stream));
        TRY(sync(B));
        const std::vector<int> &perm = B->topos[B->insts[slot].topo].perm;
        std::vector<int> idx(count);
        for (int k = 0; k < count; k++) idx[k] = k;
        std::sort(idx.begin(), idx.end(), [&](int a, int b) { return perm[hid[a]] < perm[hid[b]]; });
        for (int k = 0; k < count; k++) {
            const int src = idx[k];
            if (ids) ids[k] = perm[hid[src]];
            if (f)
                for (int d = 0; d < 3; d++) f[3 * (size_t)k + d] = hf[3 * (size_t)src + d];
            if (phi) phi[k] = hphi[src];
        }
    }
    return FEM_OK;
}

// The contact patch staged in the device's static scratch: the same kernel
// and the same caller-visible result as contact_patch_impl, with the caller's
// arrays as the only host storage (the device ids are mapped to caller ids
// and the entries ordered by a heap sort in place).
int contact_patch_noalloc_impl(fem_batch *B, int slot, int32_t *ids, double *f, double *phi, int32_t capacity,
                               int32_t *n_contact, double F_total[3]) {
    const TopoRec &tp = B->topos[B->insts[slot].topo];
    if (tp.nc > FEM_NOALLOC_MAX_CONTACT)
        return fail(FEM_E_INVALID, "mesh has " + std::to_string(tp.nc) + " contact-eligible nodes, above the " +
                                       std::to_string(FEM_NOALLOC_MAX_CONTACT) + " the static scratch holds");
    if (B->tables_dirty) return fail(FEM_E_STATE, "jobs changed since the last fem_batch_run (run the batch first)");
    if ((f || phi) && !ids) return fail(FEM_E_INVALID, "ids is needed to order f and phi");
    void *base = g_scratch_ptr[B->device];
    if (!base) return fail(FEM_E_STATE, "static scratch not resolved on this device");
    const PatchStage st(base, (size_t)FEM_NOALLOC_MAX_CONTACT);
    int count = 0;
    double Ft[3];
    TRY(contact_patch_launch(B, slot, st, &count, Ft));
    *n_contact = count;
    if (F_total) std::memcpy(F_total, Ft, sizeof Ft);
    if (capacity < count) return fail(FEM_E_BUFFER, "capacity below the contact count");
    if (count == 0 || !ids) return FEM_OK;
    HIP_TRY(hipMemcpyAsync(ids, st.ids, count * sizeof(int), hipMemcpyDeviceToHost, B->stream));
    if (f) HIP_TRY(hipMemcpyAsync(f, st.f, 3 * (size_t)count * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    if (phi) HIP_TRY(hipMemcpyAsync(phi, st.phi, count * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    TRY(sync(B));
    for (int k = 0; k < count; k++) ids[k] = tp.perm[ids[k]];
    auto swap_entries = [&](int a, int b) {
        std::swap(ids[a], ids[b]);
        if (f)
            for (int d = 0; d < 3; d++) std::swap(f[3 * (size_t)a + d], f[3 * (size_t)b + d]);
        if (phi) std::swap(phi[a], phi[b]);
    };
    auto sift_down = [&](int root, int end) {
        for (;;) {
            int child = 2 * root + 1;
            if (child >= end) return;
            if (child + 1 < end && ids[child + 1] > ids[child]) child++;
            if (ids[root] >= ids[child]) return;
            swap_entries(root, child);
            root = child;
        }
    };
    for (int k = count / 2 - 1; k >= 0; k--) sift_down(k, count);
    for (int end = count - 1; end > 0; end--) {
        swap_entries(0, end);
        sift_down(0, end);
    }
    return FEM_OK;
}

bool job_ok(const fem_batch *B, int job) { return B && job >= 0 && job < B->capacity && B->insts[job].live; }

int outbuf(fem_batch *B, size_t bytes) {
    if (B->outbuf_bytes >= bytes) return FEM_OK;
    if (B->outbuf) (void)hipFree(B->outbuf);
    B->outbuf = nullptr;
    B->outbuf_bytes = 0;
    HIP_TRY(hipMalloc(&B->outbuf, bytes));
    B->outbuf_bytes = bytes;
    return FEM_OK;
}

// Per-tet Cauchy and von Mises stress of one instance at its current state,
// staged in d_out (7 m doubles of device memory: sigma, then von Mises) and
// copied to the caller's host arrays.
int tet_stress_into(fem_batch *B, int slot, double *d_out, double *sigma, double *vm) {
    const TopoRec &tp = B->topos[B->insts[slot].topo];
    double *d_sig = d_out, *d_vm = d_out + 6 * (size_t)tp.m;
    if (B->precision == FEM_PREC_FP32)
        k_tet_stress<float><<<tp.ntile, kBlock, 0, B->stream>>>((const Topo<float> *)B->d_topos,
                                                                (const InstBufs<float> *)B->d_bufs, slot, d_sig, d_vm);
    else
        k_tet_stress<double><<<tp.ntile, kBlock, 0, B->stream>>>((const Topo<double> *)B->d_topos,
                                                                 (const InstBufs<double> *)B->d_bufs, slot, d_sig, d_vm);
    TRY(launch_check("k_tet_stress"));
    if (sigma) HIP_TRY(hipMemcpyAsync(sigma, d_sig, 6 * (size_t)tp.m * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    if (vm) HIP_TRY(hipMemcpyAsync(vm, d_vm, (size_t)tp.m * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    return sync(B);
}

int tet_stress_impl(fem_batch *B, int slot, double *sigma, double *vm, int64_t capacity) {
    const TopoRec &tp = B->topos[B->insts[slot].topo];
    if (capacity < tp.m) return fail(FEM_E_BUFFER, "capacity below the tet count");
    if (!sigma && !vm) return FEM_OK;
    if (B->tables_dirty) TRY(B->precision == FEM_PREC_FP32 ? rebuild_tables<float>(B) : rebuild_tables<double>(B));
    TRY(outbuf(B, 7 * (size_t)tp.m * sizeof(double)));
    return tet_stress_into(B, slot, (double *)B->outbuf, sigma, vm);
}

int disp_stats_impl(fem_batch *B, int slot, double *max_norm, double *mean_norm) {
    if (B->tables_dirty) TRY(B->precision == FEM_PREC_FP32 ? rebuild_tables<float>(B) : rebuild_tables<double>(B));
    TRY(outbuf(B, 2 * sizeof(double)));
    double *d = (double *)B->outbuf, h[2];
    if (B->precision == FEM_PREC_FP32)
        k_disp_stats<float><<<1, 1024, 0, B->stream>>>((const Topo<float> *)B->d_topos,
                                                       (const InstBufs<float> *)B->d_bufs, slot, d);
    else
        k_disp_stats<double><<<1, 1024, 0, B->stream>>>((const Topo<double> *)B->d_topos,
                                                        (const InstBufs<double> *)B->d_bufs, slot, d);
    TRY(launch_check("k_disp_stats"));
    HIP_TRY(hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, B->stream));
    TRY(sync(B));
    if (max_norm) *max_norm = h[0];
    if (mean_norm) *mean_norm = h[1];
    return FEM_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *fem_status_string(int status) {
    switch (status) {
    case FEM_OK: return "ok";
    case FEM_W_FLOOR: return "stopped at the rounding floor";
    case FEM_E_INVALID: return "invalid argument";
    case FEM_E_DEGENERATE: return "degenerate tetrahedron";
    case FEM_E_OOM: return "out of device memory";
    case FEM_E_DEVICE: return "device error";
    case FEM_E_STATE: return "material or indenter not set";
    case FEM_E_NOT_CONVERGED: return "not converged";
    case FEM_E_INVERSION: return "element inversion";
    case FEM_E_BUFFER: return "buffer too small";
    default: return "unknown status";
    }
}

const char *fem_last_error(void) { return g_last_error.c_str(); }

void fem_default_params(fem_solve_params *P, int32_t precision) {
    if (!P) return;
    P->newton_rtol = precision == FEM_PREC_FP32 ? 3e-6 : 1e-8;
    P->newton_atol = precision == FEM_PREC_FP32 ? 1e-9 : 1e-14;
    P->max_newton = 50;
    P->cg_rtol = precision == FEM_PREC_FP32 ? 1e-5 : 1e-8;
    P->cg_eta_max = 0.1;
    P->cg_eta_power = precision == FEM_PREC_FP32 ? 0.75 : 1.0;
    P->max_cg = 100000;
    P->precond = FEM_PRECOND_BLOCK;
    P->contact_hessian = 1;
    P->c1 = 1e-4;
    P->max_halvings = 40;
    P->newton_floor_rtol = precision == FEM_PREC_FP32 ? 1e-3 : 1e-6;
}

// ---- single mesh ----------------------------------------------------------
int fem_create_mesh(const double *X, int32_t n_nodes, const int32_t *tets, int32_t n_tets, const uint8_t *fixed,
                    const fem_config *cfg, fem_mesh **out) {
    g_last_error.clear();
    if (!out) return fail(FEM_E_INVALID, "out is null");
    *out = nullptr;
    TRY(check_mesh_args(X, n_nodes, tets, n_tets, fixed));
    fem_mesh *M = new (std::nothrow) fem_mesh();
    if (!M) return fail(FEM_E_OOM, "host allocation failed");
    M->n = n_nodes;
    M->m = n_tets;
    int rc = batch_create(cfg, 1, &M->batch);
    int topo = -1;
    if (!rc)
        rc = M->batch->precision == FEM_PREC_FP32 ? add_topology<float>(M->batch, X, n_nodes, tets, n_tets, fixed, &topo)
                                                  : add_topology<double>(M->batch, X, n_nodes, tets, n_tets, fixed, &topo);
    if (!rc)
        rc = M->batch->precision == FEM_PREC_FP32 ? alloc_instance<float>(M->batch, 0, topo)
                                                  : alloc_instance<double>(M->batch, 0, topo);
    if (!rc) rc = sync(M->batch);
    if (rc) {
        std::string msg = g_last_error;
        if (M->batch) batch_release(M->batch);
        delete M;
        g_last_error = msg;
        return rc;
    }
    *out = M;
    return FEM_OK;
}

void fem_destroy_mesh(fem_mesh *M) {
    if (!M) return;
    batch_release(M->batch);
    delete M;
}

int fem_set_material(fem_mesh *M, double E, double nu, double density) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    TRY(check_material(E, nu, density));
    M->E = E;
    M->nu = nu;
    M->density = density;
    M->have_material = true;
    return FEM_OK;
}

int fem_set_indenter(fem_mesh *M, int32_t kind, const double *shape, int32_t n_shape, const double R[9],
                     const double c[3], double k_penalty) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    Indenter ind;
    TRY(check_indenter(kind, shape, n_shape, R, c, k_penalty, &ind));
    M->ind = ind;
    M->have_indenter = true;
    return FEM_OK;
}

int fem_step(fem_mesh *M, const fem_solve_params *params, fem_step_info *info) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    if (!M->have_material || !M->have_indenter) return fail(FEM_E_STATE, "set material and indenter first");
    fem_solve_params P;
    if (params)
        P = *params;
    else
        fem_default_params(&P, M->batch->precision);
    TRY(check_params(P));
    fem_batch *B = M->batch;
    TRY(set_device(B));
    TRY(params_to_device(B, P));
    const double zero[3] = {0.0, 0.0, 0.0};
    const int hint = B->h_states[0].last_cg;
    init_job_state(B->h_states[0], M->E, M->nu, M->ind, M->ind.c, zero, 0.0, 1, M->dt, M->density, M->model,
                   M->friction);
    B->h_states[0].last_cg = hint;
    TRY(write_state(B, 0));
    TRY(run(B, 0, nullptr));
    // the state reached is the next step's friction lag state
    M->friction.lag_ok = 1;
    for (int d = 0; d < 3; d++) M->friction.c_lag[d] = M->ind.c[d];
    fem_step_info local{};
    fill_step_info(B->h_states[0], M->m, &local);
    if (info) *info = local;
    if (local.status == FEM_E_NOT_CONVERGED) g_last_error = "Newton did not converge";
    if (local.status == FEM_E_INVERSION) g_last_error = "line search could not keep det F > 0";
    return local.status;
}

int fem_get_displacements(const fem_mesh *M, double *u, int64_t capacity) {
    g_last_error.clear();
    if (!M || !u) return fail(FEM_E_INVALID, "null argument");
    if (capacity < 3LL * M->n) return fail(FEM_E_BUFFER, "capacity below 3 n");
    TRY(set_device(M->batch));
    return download_nodes(M->batch, M->batch->topos[0].perm, u, inst_ptr(M->batch, 0, V_U));
}

int fem_set_displacements(fem_mesh *M, const double *u, int64_t count) {
    g_last_error.clear();
    if (!M || !u) return fail(FEM_E_INVALID, "null argument");
    if (count != 3LL * M->n) return fail(FEM_E_INVALID, "count must be 3 n");
    for (int64_t i = 0; i < count; i++)
        if (!is_finite(u[i])) return fail(FEM_E_INVALID, "non-finite displacement");
    TRY(set_device(M->batch));
    TRY(upload_nodes(M->batch, M->batch->topos[0].perm, inst_ptr(M->batch, 0, V_U), u));
    // The predictor follows, so the stored velocity is kept as it is.
    HIP_TRY(hipMemcpyAsync(inst_ptr(M->batch, 0, V_UT), inst_ptr(M->batch, 0, V_U), 3 * (size_t)M->n * M->batch->elem(),
                           hipMemcpyDeviceToDevice, M->batch->stream));
    // u at the current indenter pose becomes the friction lag state
    M->friction.lag_ok = M->have_indenter ? 1 : 0;
    for (int d = 0; d < 3; d++) M->friction.c_lag[d] = M->ind.c[d];
    return sync(M->batch);
}

int fem_set_friction(fem_mesh *M, double mu_f, double eps) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    TRY(check_friction(mu_f, eps));
    M->friction.mu_f = mu_f;
    M->friction.eps_f = mu_f > 0.0 ? eps : 1e-5;
    return FEM_OK;
}

int fem_set_model(fem_mesh *M, int32_t model) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    if (model != FEM_MODEL_NEOHOOKEAN && model != FEM_MODEL_COROTATIONAL) return fail(FEM_E_INVALID, "unknown model");
    M->model = model;
    return FEM_OK;
}

int fem_set_dynamics(fem_mesh *M, double dt) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    if (!is_finite(dt) || dt < 0) return fail(FEM_E_INVALID, "dt must be >= 0");
    if (dt > 0 && !(M->have_material && M->density > 0)) return fail(FEM_E_STATE, "set a material with density > 0 first");
    M->dt = dt;
    return FEM_OK;
}

int fem_get_velocities(const fem_mesh *Mc, double *v, int64_t capacity) {
    g_last_error.clear();
    if (!Mc || !v) return fail(FEM_E_INVALID, "null argument");
    if (capacity < 3LL * Mc->n) return fail(FEM_E_BUFFER, "capacity below 3 n");
    fem_mesh *M = const_cast<fem_mesh *>(Mc);
    TRY(set_device(M->batch));
    M->batch->h_states[0].dt = M->dt;
    return download_velocity(M->batch, 0, v);
}

int fem_set_velocities(fem_mesh *M, const double *v, int64_t count) {
    g_last_error.clear();
    if (!M || !v) return fail(FEM_E_INVALID, "null argument");
    if (count != 3LL * M->n) return fail(FEM_E_INVALID, "count must be 3 n");
    for (int64_t i = 0; i < count; i++)
        if (!is_finite(v[i])) return fail(FEM_E_INVALID, "non-finite velocity");
    TRY(set_device(M->batch));
    TRY(upload_nodes(M->batch, M->batch->topos[0].perm, inst_ptr(M->batch, 0, V_V), v));
    HIP_TRY(hipMemcpyAsync(inst_ptr(M->batch, 0, V_UT), inst_ptr(M->batch, 0, V_U), 3 * (size_t)M->n * M->batch->elem(),
                           hipMemcpyDeviceToDevice, M->batch->stream));
    return sync(M->batch);
}

int fem_get_contact_patch(const fem_mesh *Mc, int32_t *ids, double *f, double *phi, int32_t capacity,
                          int32_t *n_contact, double F_total[3]) {
    g_last_error.clear();
    if (!Mc || !n_contact) return fail(FEM_E_INVALID, "null argument");
    fem_mesh *M = const_cast<fem_mesh *>(Mc);
    if (!M->have_indenter) return fail(FEM_E_STATE, "no indenter");
    fem_batch *B = M->batch;
    TRY(set_device(B));
    // The patch is evaluated at the handle's current indenter pose.
    TRY(read_states(B));
    B->h_states[0].ind = M->ind;
    TRY(write_state(B, 0));
    return contact_patch_impl(B, 0, ids, f, phi, capacity, n_contact, F_total);
}

int fem_get_mesh_info(const fem_mesh *M, int32_t *n_nodes, int32_t *n_tets, int32_t *n_eligible, uint8_t *eligible,
                      int32_t capacity) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    const TopoRec &tp = M->batch->topos[0];
    if (n_nodes) *n_nodes = M->n;
    if (n_tets) *n_tets = M->m;
    if (n_eligible) *n_eligible = tp.nc;
    if (eligible) {
        if (capacity < M->n) return fail(FEM_E_BUFFER, "capacity below n");
        TRY(set_device(M->batch));
        std::vector<uint8_t> dev(M->n);
        HIP_TRY(hipMemcpyAsync(dev.data(), tp.elig, M->n, hipMemcpyDeviceToHost, M->batch->stream));
        TRY(sync(M->batch));
        for (int i = 0; i < M->n; i++) eligible[tp.perm[i]] = dev[i];
    }
    return FEM_OK;
}

int fem_eval_gradient(fem_mesh *M, double *g, int64_t capacity, double *energy, double *min_J) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    if (!M->have_material || !M->have_indenter) return fail(FEM_E_STATE, "set material and indenter first");
    if (g && capacity < 3LL * M->n) return fail(FEM_E_BUFFER, "capacity below 3 n");
    fem_batch *B = M->batch;
    TRY(set_device(B));
    fem_solve_params P;
    fem_default_params(&P, B->precision);
    TRY(params_to_device(B, P));
    const double zero[3] = {0.0, 0.0, 0.0};
    init_job_state(B->h_states[0], M->E, M->nu, M->ind, M->ind.c, zero, 0.0, 1, M->dt, M->density, M->model,
                   M->friction);
    // with friction, the node pass forms the lag data first
    B->h_states[0].after_lag = PH_EVAL_GRAD;
    B->h_states[0].phase = M->friction.mu_f > 0.0 ? PH_LAG : PH_EVAL_GRAD;
    TRY(write_state(B, 0));
    TRY(run(B, 2, nullptr));
    if (energy) *energy = B->h_states[0].E;
    if (min_J) *min_J = B->h_states[0].minJ;
    if (g) return download_nodes(B, B->topos[0].perm, g, inst_ptr(B, 0, V_G));
    return FEM_OK;
}

int fem_eval_hessvec(fem_mesh *M, const fem_solve_params *params, const double *v, double *q, int64_t capacity) {
    g_last_error.clear();
    if (!M || !v || !q) return fail(FEM_E_INVALID, "null argument");
    if (!M->have_material || !M->have_indenter) return fail(FEM_E_STATE, "set material and indenter first");
    if (capacity < 3LL * M->n) return fail(FEM_E_BUFFER, "capacity below 3 n");
    fem_batch *B = M->batch;
    fem_solve_params P;
    if (params)
        P = *params;
    else
        fem_default_params(&P, B->precision);
    TRY(check_params(P));
    TRY(set_device(B));
    TRY(params_to_device(B, P));
    const double zero[3] = {0.0, 0.0, 0.0};
    init_job_state(B->h_states[0], M->E, M->nu, M->ind, M->ind.c, zero, 0.0, 1, M->dt, M->density, M->model,
                   M->friction);
    // with friction, the node pass forms the lag data first
    B->h_states[0].after_lag = PH_EVAL_GRAD;
    B->h_states[0].phase = M->friction.mu_f > 0.0 ? PH_LAG : PH_EVAL_GRAD;
    TRY(write_state(B, 0));
    TRY(run(B, 2, nullptr));
    // q = H v through the CG kernels with z = v, p_prev = 0, beta = 0.
    std::vector<double> zeros(3 * (size_t)M->n, 0.0);
    TRY(upload_nodes(B, B->topos[0].perm, inst_ptr(B, 0, V_Z), v));
    TRY(upload_nodes(B, B->topos[0].perm, inst_ptr(B, 0, V_P), zeros.data()));
    TRY(read_states(B));
    B->h_states[0].beta = 0.0;
    B->h_states[0].phase = PH_EVAL_HV;
    TRY(write_state(B, 0));
    TRY(run(B, 2, nullptr));
    return download_nodes(B, B->topos[0].perm, q, inst_ptr(B, 0, V_Q));
}

int fem_set_kernel_timing(fem_mesh *M, int32_t every) {
    return fem_batch_set_kernel_timing(M ? M->batch : nullptr, every);
}

int fem_get_kernel_timing(const fem_mesh *M, int32_t kernel, int64_t *count, double *total_ms) {
    return fem_batch_get_kernel_timing(M ? M->batch : nullptr, kernel, count, total_ms);
}

// ---- batches --------------------------------------------------------------
int fem_batch_create(const fem_config *cfg, int32_t max_jobs, fem_batch **out) {
    g_last_error.clear();
    if (!out) return fail(FEM_E_INVALID, "out is null");
    return batch_create(cfg, max_jobs, out);
}

void fem_batch_destroy(fem_batch *B) { batch_release(B); }

int fem_batch_add_mesh(fem_batch *B, const double *X, int32_t n_nodes, const int32_t *tets, int32_t n_tets,
                       const uint8_t *fixed, int32_t *mesh_id) {
    g_last_error.clear();
    if (!B || !mesh_id) return fail(FEM_E_INVALID, "null argument");
    TRY(check_mesh_args(X, n_nodes, tets, n_tets, fixed));
    TRY(set_device(B));
    int id = -1;
    TRY(B->precision == FEM_PREC_FP32 ? add_topology<float>(B, X, n_nodes, tets, n_tets, fixed, &id)
                                     : add_topology<double>(B, X, n_nodes, tets, n_tets, fixed, &id));
    *mesh_id = id;
    return FEM_OK;
}

int fem_batch_add_job(fem_batch *B, int32_t mesh_id, double E, double nu, const fem_indentation *job,
                      int32_t *job_id) {
    g_last_error.clear();
    if (!B || !job || !job_id) return fail(FEM_E_INVALID, "null argument");
    if (mesh_id < 0 || mesh_id >= (int)B->topos.size()) return fail(FEM_E_INVALID, "unknown mesh id");
    TRY(check_material(E, nu, 0.0));
    Indenter ind;
    TRY(check_indenter(job->kind, job->shape, 4, job->R, job->c0, job->k_penalty, &ind));
    if (job->steps < 1 || !is_finite(job->depth) || job->depth < 0) return fail(FEM_E_INVALID, "bad schedule");
    for (int d = 0; d < 3; d++)
        if (!is_finite(job->direction[d])) return fail(FEM_E_INVALID, "bad direction");
    if (!is_finite(job->dt) || job->dt < 0 || (job->dt > 0 && !(job->density > 0 && is_finite(job->density))))
        return fail(FEM_E_INVALID, "implicit steps need dt >= 0 and density > 0");
    if (job->model != FEM_MODEL_NEOHOOKEAN && job->model != FEM_MODEL_COROTATIONAL)
        return fail(FEM_E_INVALID, "unknown constitutive model");
    TRY(check_friction(job->friction, job->friction_eps));
    int slot = -1;
    for (int i = 0; i < B->capacity; i++)
        if (!B->insts[i].live) {
            slot = i;
            break;
        }
    if (slot < 0) return fail(FEM_E_BUFFER, "batch is full");
    TRY(set_device(B));
    TRY(B->precision == FEM_PREC_FP32 ? alloc_instance<float>(B, slot, mesh_id)
                                     : alloc_instance<double>(B, slot, mesh_id));
    init_job_state(B->h_states[slot], E, nu, ind, job->c0, job->direction, job->depth, job->steps, job->dt,
                   job->density, job->model, job_friction(job));
    TRY(write_state(B, slot));
    *job_id = slot;
    return FEM_OK;
}

int fem_batch_restart_job(fem_batch *B, int32_t job_id, double E, double nu, const fem_indentation *job) {
    g_last_error.clear();
    if (!job || !job_ok(B, job_id)) return fail(FEM_E_INVALID, "unknown job");
    TRY(check_material(E, nu, 0.0));
    Indenter ind;
    TRY(check_indenter(job->kind, job->shape, 4, job->R, job->c0, job->k_penalty, &ind));
    if (job->steps < 1 || !is_finite(job->depth) || job->depth < 0) return fail(FEM_E_INVALID, "bad schedule");
    for (int d = 0; d < 3; d++)
        if (!is_finite(job->direction[d])) return fail(FEM_E_INVALID, "bad direction");
    if (!is_finite(job->dt) || job->dt < 0 || (job->dt > 0 && !(job->density > 0 && is_finite(job->density))))
        return fail(FEM_E_INVALID, "implicit steps need dt >= 0 and density > 0");
    if (job->model != FEM_MODEL_NEOHOOKEAN && job->model != FEM_MODEL_COROTATIONAL)
        return fail(FEM_E_INVALID, "unknown constitutive model");
    TRY(check_friction(job->friction, job->friction_eps));
    TRY(set_device(B));
    const int n = B->topos[B->insts[job_id].topo].n;
    for (int which : {V_U, V_V, V_UT})
        HIP_TRY(hipMemsetAsync(inst_ptr(B, job_id, which), 0, 3 * (size_t)n * B->elem(), B->stream));
    const int hint = B->h_states[job_id].last_cg;
    init_job_state(B->h_states[job_id], E, nu, ind, job->c0, job->direction, job->depth, job->steps, job->dt,
                   job->density, job->model, job_friction(job));
    B->h_states[job_id].last_cg = hint;
    // Stream-ordered before any later kernel or state read; the pinned source
    // slot is not written again until the host has synchronised.
    HIP_TRY(hipMemcpyAsync(B->d_states + job_id, B->h_states + job_id, sizeof(InstState), hipMemcpyHostToDevice,
                           B->stream));
    return FEM_OK;
}

int fem_batch_remove_job(fem_batch *B, int32_t job) {
    g_last_error.clear();
    if (!job_ok(B, job)) return fail(FEM_E_INVALID, "unknown job");
    TRY(set_device(B));
    TRY(sync(B));
    free_instance(B, job);
    std::memset(B->h_states + job, 0, sizeof(InstState));
    return write_state(B, job);
}

int fem_batch_run(fem_batch *B, const fem_solve_params *params, int32_t max_rounds, int32_t *n_running) {
    g_last_error.clear();
    if (!B) return fail(FEM_E_INVALID, "null batch");
    fem_solve_params P;
    if (params)
        P = *params;
    else
        fem_default_params(&P, B->precision);
    TRY(check_params(P));
    TRY(set_device(B));
    TRY(params_to_device(B, P));
    int running = 0;
    TRY(run(B, max_rounds, &running));
    if (n_running) *n_running = running;
    return FEM_OK;
}

int fem_batch_job_info(const fem_batch *B, int32_t job, fem_job_info *info) {
    g_last_error.clear();
    if (!info || !job_ok(B, job)) return fail(FEM_E_INVALID, "unknown job");
    const InstState &s = B->h_states[job];
    const int m = B->topos[B->insts[job].topo].m;
    const bool done = s.phase == PH_DONE;
    fem_job_info J{};
    J.done = done ? 1 : 0;
    J.status = s.first_fail;
    J.step = s.step;
    J.steps_ok = s.steps_ok;
    J.steps_failed = s.steps_failed;
    J.steps_floor = s.steps_floor;
    J.newton_iters = s.tot_newton + (done ? 0 : s.st_newton);
    J.cg_iters = s.tot_cg + (done ? 0 : s.st_cg);
    J.hv_products = s.tot_hv + (done ? 0 : s.st_hv);
    J.grad_passes = s.tot_grad + (done ? 0 : s.st_grad);
    J.ls_trials = s.tot_ls + (done ? 0 : s.st_ls);
    J.tet_updates = (int64_t)m * (J.grad_passes + J.hv_products);
    J.energy = s.E;
    J.min_J = s.minJ;
    J.g_norm = s.st_g;
    *info = J;
    return FEM_OK;
}

int fem_batch_job_step_status(const fem_batch *B, int32_t job, int32_t *status, int32_t capacity, int32_t *n_steps) {
    g_last_error.clear();
    if (!n_steps || !job_ok(B, job)) return fail(FEM_E_INVALID, "unknown job");
    const InstState &s = B->h_states[job];
    const int taken = std::min(s.steps_ok + s.steps_failed, kHistSteps);
    *n_steps = taken;
    if (!status) return FEM_OK;   // count query
    if (capacity < taken) return fail(FEM_E_BUFFER, "capacity below the number of load steps taken");
    if (taken == 0) return FEM_OK;
    fem_batch *W = const_cast<fem_batch *>(B);
    TRY(set_device(W));
    const InstRec &R = B->insts[job];
    const signed char *src = B->precision == FEM_PREC_FP32 ? R.b32.hist : R.b64.hist;
    signed char h[kHistSteps];
    HIP_TRY(hipMemcpyAsync(h, src, (size_t)taken, hipMemcpyDeviceToHost, W->stream));
    TRY(sync(W));
    for (int k = 0; k < taken; k++) status[k] = h[k];
    return FEM_OK;
}

int fem_get_tet_stress(const fem_mesh *M, double *sigma, double *von_mises, int64_t capacity) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    if (!M->have_material) return fail(FEM_E_STATE, "set the material first");
    TRY(set_device(M->batch));
    // the material and law of the handle, as the next step would use them
    TRY(read_states(M->batch));
    InstState &s = M->batch->h_states[0];
    s.mu = M->E / (2.0 * (1.0 + M->nu));
    s.lam = M->E * M->nu / ((1.0 + M->nu) * (1.0 - 2.0 * M->nu));
    s.model = M->model;
    TRY(write_state(M->batch, 0));
    return tet_stress_impl(M->batch, 0, sigma, von_mises, capacity);
}

int fem_get_displacement_stats(const fem_mesh *M, double *max_norm, double *mean_norm) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    TRY(set_device(M->batch));
    return disp_stats_impl(M->batch, 0, max_norm, mean_norm);
}

int fem_batch_get_tet_stress(fem_batch *B, int32_t job, double *sigma, double *von_mises, int64_t capacity) {
    g_last_error.clear();
    if (!job_ok(B, job)) return fail(FEM_E_INVALID, "unknown job");
    TRY(set_device(B));
    return tet_stress_impl(B, job, sigma, von_mises, capacity);
}

int fem_batch_get_displacement_stats(fem_batch *B, int32_t job, double *max_norm, double *mean_norm) {
    g_last_error.clear();
    if (!job_ok(B, job)) return fail(FEM_E_INVALID, "unknown job");
    TRY(set_device(B));
    return disp_stats_impl(B, job, max_norm, mean_norm);
}

int fem_batch_get_velocities(fem_batch *B, int32_t job, double *v, int64_t capacity) {
    g_last_error.clear();
    if (!v || !job_ok(B, job)) return fail(FEM_E_INVALID, "unknown job");
    const int n = B->topos[B->insts[job].topo].n;
    if (capacity < 3LL * n) return fail(FEM_E_BUFFER, "capacity below 3 n");
    TRY(set_device(B));
    return download_velocity(B, job, v);
}

int fem_batch_get_displacements(fem_batch *B, int32_t job, double *u, int64_t capacity) {
    g_last_error.clear();
    if (!u || !job_ok(B, job)) return fail(FEM_E_INVALID, "unknown job");
    const int n = B->topos[B->insts[job].topo].n;
    if (capacity < 3LL * n) return fail(FEM_E_BUFFER, "capacity below 3 n");
    TRY(set_device(B));
    return download_nodes(B, B->topos[B->insts[job].topo].perm, u, inst_ptr(B, job, V_U));
}

int fem_batch_get_contact_patch(fem_batch *B, int32_t job, int32_t *ids, double *f, double *phi, int32_t capacity,
                                int32_t *n_contact, double F_total[3]) {
    g_last_error.clear();
    if (!n_contact || !job_ok(B, job)) return fail(FEM_E_INVALID, "unknown job");
    TRY(set_device(B));
    return contact_patch_impl(B, job, ids, f, phi, capacity, n_contact, F_total);
}

int fem_batch_get_contact_patch_noalloc(fem_batch *B, int32_t job, int32_t *ids, double *f, double *phi,
                                        int32_t capacity, int32_t *n_contact, double F_total[3]) {
    g_last_error.clear();
    if (!n_contact || !job_ok(B, job)) return fail(FEM_E_INVALID, "unknown job");
    TRY(set_device(B));
    return contact_patch_noalloc_impl(B, job, ids, f, phi, capacity, n_contact, F_total);
}

int fem_batch_set_kernel_timing(fem_batch *B, int32_t every) {
    g_last_error.clear();
    if (!B || every < 0) return fail(FEM_E_INVALID, "bad argument");
    TRY(set_device(B));
    KernelTimer &t = B->timer;
    if (every > 0 && !t.created) {
        for (int i = 0; i < KernelTimer::kPool; i++) {
            HIP_TRY(hipEventCreate(&t.ev[i][0]));
            HIP_TRY(hipEventCreate(&t.ev[i][1]));
        }
        t.created = true;
    }
    TRY(sync(B));
    t.used = 0;
    t.every = every;
    t.rounds = 0;
    for (int k = 0; k < KernelTimer::kKinds; k++) {
        t.seen[k] = 0;
        t.count[k] = 0;
        t.total_ms[k] = 0.0;
    }
    return FEM_OK;
}

int fem_batch_get_kernel_timing(const fem_batch *B, int32_t kernel, int64_t *count, double *total_ms) {
    g_last_error.clear();
    if (!B || kernel < 0 || kernel >= KernelTimer::kKinds) return fail(FEM_E_INVALID, "bad argument");
    if (count) *count = B->timer.count[kernel];
    if (total_ms) *total_ms = B->timer.total_ms[kernel];
    return FEM_OK;
}

int fem_batch_get_kernel_launches(const fem_batch *B, int32_t kernel, int64_t *launches) {
    g_last_error.clear();
    if (!B || !launches || kernel < 0 || kernel >= KernelTimer::kKinds) return fail(FEM_E_INVALID, "bad argument");
    *launches = B->timer.seen[kernel];
    return FEM_OK;
}

int fem_batch_set_graphs(fem_batch *B, int32_t enable) {
    g_last_error.clear();
    if (!B) return fail(FEM_E_INVALID, "null batch");
    TRY(set_device(B));
    TRY(sync(B));
    drop_graphs(B);
    B->use_graphs = enable != 0;
    return FEM_OK;
}

int fem_set_graphs(fem_mesh *M, int32_t enable) { return fem_batch_set_graphs(M ? M->batch : nullptr, enable); }

int fem_batch_set_option(fem_batch *B, int32_t option, int32_t value) {
    g_last_error.clear();
    if (!B) return fail(FEM_E_INVALID, "null batch");
    switch (option) {
    case FEM_OPT_ROUND_STEPS:
        if (value < 0 || value > 64) return fail(FEM_E_INVALID, "chunk must be 0..64");
        B->chunk = value;
        return FEM_OK;
    case FEM_OPT_TILE_TETS:
        if (value < 64 || value > kTileTets) return fail(FEM_E_INVALID, "tile tets must be 64..512");
        B->tile_tets = value;
        return FEM_OK;
    case FEM_OPT_DETERMINISTIC:
        if (value < 0 || value > 1) return fail(FEM_E_INVALID, "deterministic must be 0 or 1");
        TRY(set_device(B));
        TRY(sync(B));
        drop_graphs(B);
        B->deterministic = value != 0;
        return FEM_OK;
    case FEM_OPT_GROUPS:
        if (value < 0 || value > 2) return fail(FEM_E_INVALID, "groups must be 0, 1 or 2");
        B->groups_opt = value;
        B->tables_dirty = true;
        return FEM_OK;
    case FEM_OPT_TILE_NODES:
        if (value < 16 || value > kTileNodes) return fail(FEM_E_INVALID, "tile nodes must be 16..256");
        B->tile_nodes = value;
        return FEM_OK;
    default:
        return fail(FEM_E_INVALID, "unknown option");
    }
}

int fem_batch_job_footprint(const fem_batch *B, int32_t mesh_id, int64_t *bytes) {
    g_last_error.clear();
    if (!B || !bytes || mesh_id < 0 || mesh_id >= (int)B->topos.size()) return fail(FEM_E_INVALID, "unknown mesh");
    const TopoRec &tp = B->topos[mesh_id];
    const size_t w = B->elem();
    const size_t stride = std::max(tp.ntile + tp.ncb, kWaves * ceil_div(tp.n, kBlock));
    // the arena of alloc_instance, with its 256-byte alignment padding
    size_t total = 0;
    auto add = [&](size_t b) { total += (b + 255) & ~size_t(255); };
    for (int k = 0; k < 7; k++) add(3 * (size_t)tp.n * w);
    add(6 * (size_t)tp.n * w);
    add(9 * (size_t)tp.nent * w);
    add(3 * (size_t)tp.nent * w);
    add(9 * (size_t)std::max(tp.nc, 1) * w);
    add(RS_COUNT * stride * sizeof(double));
    add(3 * (size_t)tp.n * w);
    add(3 * (size_t)tp.n * w);
    add(8 * (size_t)std::max(tp.nc, 1) * sizeof(double));
    add(kHistSteps);
    add(std::max(tp.nc, 1));   // contact-block flags
    *bytes = (int64_t)total;
    return FEM_OK;
}

int fem_batch_mesh_info(const fem_batch *B, int32_t mesh_id, fem_mesh_layout *info) {
    g_last_error.clear();
    if (!B || !info || mesh_id < 0 || mesh_id >= (int)B->topos.size()) return fail(FEM_E_INVALID, "unknown mesh");
    const TopoRec &tp = B->topos[mesh_id];
    info->n_nodes = tp.n;
    info->n_tets = tp.m;
    info->n_tiles = tp.ntile;
    info->n_entries = tp.nent;
    info->n_eligible = tp.nc;
    return FEM_OK;
}

}  // extern "C"
