// libfem host driver and C ABI (declared in include/fem.h).
//
// The host owns control flow only: argument checks, device memory, kernel
// launches and the Newton / line-search decisions that need the FP64 scalars
// the kernels reduce. Every arithmetic step of the solve runs in the kernels
// of fem_kernels.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "../../include/fem.h"
#include "fem_kernels.h"

using namespace fem;

namespace {

thread_local std::string g_last_error;

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

inline int nblocks(long long work, int block = kBlock) { return (int)((work + block - 1) / block); }

// Carves sub-buffers out of one device allocation, 256-byte aligned.
struct Arena {
    size_t off = 0;
    template <typename T>
    size_t take(size_t count) {
        size_t at = (off + 255) & ~size_t(255);
        off = at + count * sizeof(T);
        return at;
    }
};

}  // namespace

struct fem_mesh {
    int device = 0;
    int precision = FEM_PREC_FP64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n = 0, m = 0, nc = 0;
    void *arena = nullptr;
    size_t arena_bytes = 0;
    // typed views into the arena (the element type is the precision's)
    int *tet = nullptr;
    void *B = nullptr, *vol = nullptr;
    double *X = nullptr;
    uint8_t *fixed = nullptr, *eligible = nullptr;
    int *cnodes = nullptr;
    void *u = nullptr, *dx = nullptr, *g = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    void *diag = nullptr, *dinv = nullptr, *finv = nullptr, *c1 = nullptr, *chess = nullptr;
    double *partial = nullptr;
    unsigned *ticket = nullptr;
    Scalars *s = nullptr;
    // patch outputs
    int *patch_ids = nullptr, *patch_count = nullptr;
    double *patch_f = nullptr, *patch_phi = nullptr, *patch_F = nullptr;
    // pinned staging
    Scalars *h_s = nullptr;
    void *h_stage = nullptr;
    size_t h_stage_bytes = 0;
    // problem data
    bool have_material = false, have_indenter = false;
    double E = 0, nu = 0, density = 0, mu = 0, lam = 0;
    Indenter ind{};
    int last_cg = 0;
    size_t elem() const { return precision == FEM_PREC_FP32 ? sizeof(float) : sizeof(double); }
};

namespace {

template <typename T>
Buffers<T> views(const fem_mesh *M) {
    Buffers<T> b;
    b.n = M->n;
    b.m = M->m;
    b.nc = M->nc;
    b.tet = M->tet;
    b.B = (const T *)M->B;
    b.vol = (const T *)M->vol;
    b.X = M->X;
    b.fixed = M->fixed;
    b.cnodes = M->cnodes;
    b.u = (T *)M->u;
    b.dx = (T *)M->dx;
    b.g = (T *)M->g;
    b.r = (T *)M->r;
    b.z = (T *)M->z;
    b.p = (T *)M->p;
    b.q = (T *)M->q;
    b.diag = (T *)M->diag;
    b.dinv = (T *)M->dinv;
    b.finv = (T *)M->finv;
    b.c1 = (T *)M->c1;
    b.chess = (T *)M->chess;
    b.partial = M->partial;
    b.ticket = M->ticket;
    b.s = M->s;
    b.mu = M->mu;
    b.lam = M->lam;
    b.ind = M->ind;
    return b;
}

int set_device(const fem_mesh *M) {
    HIP_TRY(hipSetDevice(M->device));
    return FEM_OK;
}

int fetch_scalars(fem_mesh *M) {
    HIP_TRY(hipMemcpyAsync(M->h_s, M->s, sizeof(Scalars), hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
    return FEM_OK;
}

int launch_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FEM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return FEM_OK;
}

// Element + contact pass at u + alpha dx; with_grad also rebuilds g, the node
// diagonal blocks and the Hessian caches.
template <typename T>
int element_pass(fem_mesh *M, T alpha, bool with_grad, int contact_full) {
    Buffers<T> b = views<T>(M);
    if (with_grad) {
        HIP_TRY(hipMemsetAsync(M->g, 0, 3 * (size_t)M->n * sizeof(T), M->stream));
        HIP_TRY(hipMemsetAsync(M->diag, 0, 6 * (size_t)M->n * sizeof(T), M->stream));
    }
    const int tb = nblocks(M->m), cb = nblocks(M->nc);
    k_element_pass<T><<<tb + cb, kBlock, 0, M->stream>>>(b, alpha, with_grad ? 1 : 0, contact_full, tb);
    return launch_check("k_element_pass");
}

template <typename T>
int newton_init(fem_mesh *M, int block_jacobi) {
    k_newton_init<T><<<nblocks(M->n), kBlock, 0, M->stream>>>(views<T>(M), block_jacobi);
    return launch_check("k_newton_init");
}

struct Control {
    double tol2;
    int max_it;
};

// Runs CG on H dx = -g from dx = 0 until its device-side state leaves
// kRunning. Iterations are enqueued in chunks sized from the previous solve;
// a chunk whose iterations find the state already stopped exits at once.
template <typename T>
int run_cg(fem_mesh *M, double tol2, int max_it, int *iters, int *hv) {
    Buffers<T> b = views<T>(M);
    // Host-written CG controls (tolerance, cap) live in Scalars.
    Control *ctl = (Control *)M->h_stage;
    ctl->tol2 = tol2;
    ctl->max_it = max_it;
    HIP_TRY(hipMemcpyAsync(&M->s->tol2, &ctl->tol2, sizeof(double), hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipMemcpyAsync(&M->s->max_it, &ctl->max_it, sizeof(int), hipMemcpyHostToDevice, M->stream));
    const int tb = nblocks(M->m), cb = nblocks(M->nc), nb = nblocks(M->n);
    int launched = 0;
    int chunk = std::max(8, (M->last_cg * 3) / 4);
    for (;;) {
        const int todo = std::min(chunk, max_it + 1 - launched);
        for (int k = 0; k < todo; k++) {
            k_cg_hv<T><<<tb + cb, kBlock, 0, M->stream>>>(b, tb, 0);
            k_cg_update<T><<<nb, kBlock, 0, M->stream>>>(b);
        }
        launched += todo;
        int rc = launch_check("cg");
        if (rc) return rc;
        rc = fetch_scalars(M);
        if (rc) return rc;
        if (M->h_s->state != kRunning || launched > max_it) break;
        chunk = 16;
    }
    *iters = M->h_s->it;
    *hv = M->h_s->nhv;
    M->last_cg = M->h_s->it;
    return FEM_OK;
}

template <typename T>
int step_impl(fem_mesh *M, const fem_solve_params &P, fem_step_info &info) {
    const double eps = std::numeric_limits<T>::epsilon();
    const int contact_full = P.contact_hessian ? 1 : 0;
    int rc;
    if ((rc = element_pass<T>(M, (T)0, true, contact_full))) return rc;
    if ((rc = newton_init<T>(M, P.precond == FEM_PRECOND_BLOCK))) return rc;
    if ((rc = fetch_scalars(M))) return rc;
    info.grad_passes = 1;
    double E = M->h_s->energy, mag = M->h_s->emag, minJ = M->h_s->minJ;
    double gn = std::sqrt(M->h_s->gg);
    const double r0 = gn;
    info.g0_norm = gn;
    int status = FEM_E_NOT_CONVERGED;
    for (int it = 0;; it++) {
        if (gn <= std::max(P.newton_rtol * r0, P.newton_atol)) {
            status = FEM_OK;
            break;
        }
        if (it == P.max_newton) {
            status = FEM_E_NOT_CONVERGED;
            break;
        }
        double eta = std::min(P.cg_eta_max, std::max(P.cg_rtol, gn / r0));
        int cg_it = 0, hv = 0;
        if ((rc = run_cg<T>(M, eta * eta * gn * gn, P.max_cg, &cg_it, &hv))) return rc;
        info.cg_iters += cg_it;
        info.hv_products += hv;
        k_dot_gdx<T><<<nblocks(M->n), kBlock, 0, M->stream>>>(views<T>(M));
        if ((rc = launch_check("k_dot_gdx"))) return rc;
        double gd = 0.0;
        bool accepted = false, have_gd = false;
        double alpha = 1.0;
        double Et = 0.0, magt = 0.0, mjt = 0.0;
        for (int h = 0; h <= P.max_halvings; h++) {
            if ((rc = element_pass<T>(M, (T)alpha, true, contact_full))) return rc;
            if ((rc = fetch_scalars(M))) return rc;
            if (!have_gd) {
                gd = M->h_s->gd;
                have_gd = true;
            }
            info.grad_passes++;
            info.ls_trials++;
            Et = M->h_s->energy;
            magt = M->h_s->emag;
            mjt = M->h_s->minJ;
            const double noise = 16.0 * eps * mag;
            if (mjt > 0.0 && Et <= E + P.c1 * alpha * gd + noise) {
                accepted = true;
                break;
            }
            alpha *= 0.5;
        }
        if (!accepted) {
            status = mjt > 0.0 ? FEM_E_NOT_CONVERGED : FEM_E_INVERSION;
            break;
        }
        k_axpy<T><<<nblocks(3LL * M->n), kBlock, 0, M->stream>>>((T *)M->u, (const T *)M->dx, (T)alpha, 3 * M->n);
        if ((rc = launch_check("k_axpy"))) return rc;
        if ((rc = newton_init<T>(M, P.precond == FEM_PRECOND_BLOCK))) return rc;
        if ((rc = fetch_scalars(M))) return rc;
        E = Et;
        mag = magt;
        minJ = mjt;
        gn = std::sqrt(M->h_s->gg);
        info.newton_iters++;
    }
    info.status = status;
    info.g_norm = gn;
    info.energy = E;
    info.min_J = minJ;
    info.tet_updates = (int64_t)M->m * (int64_t)(info.grad_passes + info.hv_products);
    if (status == FEM_E_NOT_CONVERGED) g_last_error = "Newton did not converge";
    if (status == FEM_E_INVERSION) g_last_error = "line search could not keep det F > 0";
    return status;
}

bool is_finite(double x) { return std::isfinite(x); }

int stage(fem_mesh *M, size_t bytes) {
    if (M->h_stage_bytes >= bytes) return FEM_OK;
    if (M->h_stage) (void)hipHostFree(M->h_stage);
    M->h_stage = nullptr;
    M->h_stage_bytes = 0;
    HIP_TRY(hipHostMalloc(&M->h_stage, bytes));
    M->h_stage_bytes = bytes;
    return FEM_OK;
}

// Copies a host double array of len values into a device array of the mesh's
// precision (through the pinned staging buffer).
int upload_real(fem_mesh *M, void *dst, const double *src, size_t len) {
    int rc = stage(M, std::max<size_t>(len * 8, 64));
    if (rc) return rc;
    if (M->precision == FEM_PREC_FP32) {
        float *h = (float *)M->h_stage;
        for (size_t i = 0; i < len; i++) h[i] = (float)src[i];
    } else {
        std::memcpy(M->h_stage, src, len * sizeof(double));
    }
    HIP_TRY(hipMemcpyAsync(dst, M->h_stage, len * M->elem(), hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
    return FEM_OK;
}

int download_real(const fem_mesh *Mc, double *dst, const void *src, size_t len) {
    fem_mesh *M = const_cast<fem_mesh *>(Mc);
    int rc = stage(M, std::max<size_t>(len * 8, 64));
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(M->h_stage, src, len * M->elem(), hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
    if (M->precision == FEM_PREC_FP32) {
        const float *h = (const float *)M->h_stage;
        for (size_t i = 0; i < len; i++) dst[i] = (double)h[i];
    } else {
        std::memcpy(dst, M->h_stage, len * sizeof(double));
    }
    return FEM_OK;
}

template <typename T>
int create_impl(fem_mesh *M, const double *X, const int32_t *tets, const uint8_t *fixed) {
    const int n = M->n, m = M->m;
    // Hash table for boundary faces: power of two >= 8 m slots.
    unsigned slots = 1;
    while (slots < 8u * (unsigned)m) slots <<= 1;
    Arena A;
    const size_t o_tet = A.take<int>(4 * (size_t)m);
    const size_t o_B = A.take<T>(9 * (size_t)m);
    const size_t o_vol = A.take<T>(m);
    const size_t o_X = A.take<double>(3 * (size_t)n);
    const size_t o_fixed = A.take<uint8_t>(n);
    const size_t o_elig = A.take<uint8_t>(n);
    const size_t o_cn = A.take<int>(n);
    size_t o_vec[7];
    for (int k = 0; k < 7; k++) o_vec[k] = A.take<T>(3 * (size_t)n);
    const size_t o_diag = A.take<T>(6 * (size_t)n);
    const size_t o_dinv = A.take<T>(6 * (size_t)n);
    const size_t o_finv = A.take<T>(9 * (size_t)m);
    const size_t o_c1 = A.take<T>(m);
    const size_t o_chess = A.take<T>(6 * (size_t)n);
    const size_t o_part = A.take<double>(4 * (size_t)kMaxPartials);
    const size_t o_ticket = A.take<unsigned>(kTicketCount + 8);
    const size_t o_s = A.take<Scalars>(1);
    const size_t o_pid = A.take<int>(n);
    const size_t o_pcount = A.take<int>(1);
    const size_t o_pf = A.take<double>(3 * (size_t)n);
    const size_t o_pphi = A.take<double>(n);
    const size_t o_pF = A.take<double>(3);
    const size_t o_bad = A.take<int>(1);
    M->arena_bytes = A.off;
    HIP_TRY(hipMalloc(&M->arena, M->arena_bytes));
    char *base = (char *)M->arena;
    HIP_TRY(hipMemsetAsync(M->arena, 0, M->arena_bytes, M->stream));
    M->tet = (int *)(base + o_tet);
    M->B = base + o_B;
    M->vol = base + o_vol;
    M->X = (double *)(base + o_X);
    M->fixed = (uint8_t *)(base + o_fixed);
    M->eligible = (uint8_t *)(base + o_elig);
    M->cnodes = (int *)(base + o_cn);
    void **vecs[7] = {&M->u, &M->dx, &M->g, &M->r, &M->z, &M->p, &M->q};
    for (int k = 0; k < 7; k++) *vecs[k] = base + o_vec[k];
    M->diag = base + o_diag;
    M->dinv = base + o_dinv;
    M->finv = base + o_finv;
    M->c1 = base + o_c1;
    M->chess = base + o_chess;
    M->partial = (double *)(base + o_part);
    M->ticket = (unsigned *)(base + o_ticket);
    M->s = (Scalars *)(base + o_s);
    M->patch_ids = (int *)(base + o_pid);
    M->patch_count = (int *)(base + o_pcount);
    M->patch_f = (double *)(base + o_pf);
    M->patch_phi = (double *)(base + o_pphi);
    M->patch_F = (double *)(base + o_pF);
    int *bad = (int *)(base + o_bad);

    // Upload: X as is; tets transposed to field-major; fixed flags.
    std::vector<int> tT(4 * (size_t)m);
    for (int e = 0; e < m; e++)
        for (int a = 0; a < 4; a++) tT[(size_t)a * m + e] = tets[4 * (size_t)e + a];
    HIP_TRY(hipMemcpyAsync(M->X, X, 3 * (size_t)n * sizeof(double), hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipMemcpyAsync(M->tet, tT.data(), tT.size() * sizeof(int), hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipMemcpyAsync(M->fixed, fixed, n, hipMemcpyHostToDevice, M->stream));
    const int big = 0x7fffffff;
    HIP_TRY(hipMemcpyAsync(bad, &big, sizeof(int), hipMemcpyHostToDevice, M->stream));
    k_precompute<T><<<nblocks(m), kBlock, 0, M->stream>>>(M->X, M->tet, m, (T *)M->B, (T *)M->vol, bad);
    int rc = launch_check("k_precompute");
    if (rc) return rc;
    // Boundary faces -> surface nodes -> contact-eligible list.
    unsigned long long *keys = nullptr;
    unsigned *cnt = nullptr;
    uint8_t *surf = nullptr;
    HIP_TRY(hipMalloc(&keys, slots * sizeof(unsigned long long)));
    HIP_TRY(hipMalloc(&cnt, slots * sizeof(unsigned)));
    HIP_TRY(hipMalloc(&surf, n));
    HIP_TRY(hipMemsetAsync(keys, 0xff, slots * sizeof(unsigned long long), M->stream));
    HIP_TRY(hipMemsetAsync(cnt, 0, slots * sizeof(unsigned), M->stream));
    HIP_TRY(hipMemsetAsync(surf, 0, n, M->stream));
    k_faces_insert<<<nblocks(4LL * m), kBlock, 0, M->stream>>>(M->tet, m, keys, cnt, slots - 1);
    k_faces_mark<<<nblocks(4LL * m), kBlock, 0, M->stream>>>(M->tet, m, keys, cnt, slots - 1, surf);
    k_compact_eligible<<<1, 1024, 0, M->stream>>>(surf, M->fixed, n, M->eligible, M->cnodes, M->patch_count);
    rc = launch_check("mesh topology");
    if (rc) return rc;
    int host[2];
    HIP_TRY(hipMemcpyAsync(&host[0], bad, sizeof(int), hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipMemcpyAsync(&host[1], M->patch_count, sizeof(int), hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
    (void)hipFree(keys);
    (void)hipFree(cnt);
    (void)hipFree(surf);
    if (host[0] != big) return fail(FEM_E_DEGENERATE, "tet " + std::to_string(host[0]) + " has rest volume <= 0");
    M->nc = host[1];
    return FEM_OK;
}

void release(fem_mesh *M) {
    if (!M) return;
    (void)hipSetDevice(M->device);
    if (M->stream) (void)hipStreamSynchronize(M->stream);
    if (M->arena) (void)hipFree(M->arena);
    if (M->h_s) (void)hipHostFree(M->h_s);
    if (M->h_stage) (void)hipHostFree(M->h_stage);
    if (M->own_stream && M->stream) (void)hipStreamDestroy(M->stream);
    delete M;
}

int check_params(const fem_solve_params &P) {
    if (!(P.newton_rtol >= 0) || !(P.newton_atol >= 0) || P.max_newton < 0 || !(P.cg_rtol > 0) ||
        !(P.cg_eta_max >= P.cg_rtol) || P.max_cg < 1 || (P.precond != 0 && P.precond != 1) || !(P.c1 >= 0) ||
        !(P.c1 < 1) || P.max_halvings < 0)
        return fail(FEM_E_INVALID, "invalid solve parameters");
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
    P->newton_rtol = precision == FEM_PREC_FP32 ? 1e-5 : 1e-8;
    P->newton_atol = precision == FEM_PREC_FP32 ? 1e-9 : 1e-14;
    P->max_newton = 50;
    P->cg_rtol = precision == FEM_PREC_FP32 ? 1e-5 : 1e-8;
    P->cg_eta_max = 0.1;
    P->max_cg = 100000;
    P->precond = FEM_PRECOND_BLOCK;
    P->contact_hessian = 1;
    P->c1 = 1e-4;
    P->max_halvings = 40;
}

int fem_create_mesh(const double *X, int32_t n_nodes, const int32_t *tets, int32_t n_tets, const uint8_t *fixed,
                    const fem_config *cfg, fem_mesh **out) {
    g_last_error.clear();
    if (!out) return fail(FEM_E_INVALID, "out is null");
    *out = nullptr;
    if (!X || !tets || !fixed) return fail(FEM_E_INVALID, "null input array");
    if (n_nodes <= 0 || n_tets <= 0) return fail(FEM_E_INVALID, "empty mesh");
    if (n_nodes >= (1 << 21)) return fail(FEM_E_INVALID, "n_nodes must be below 2^21");
    if ((long long)n_tets * 4 >= (1LL << 31) / 2) return fail(FEM_E_INVALID, "too many tets");
    if (nblocks(n_tets) + nblocks(n_nodes) > kMaxPartials) return fail(FEM_E_INVALID, "mesh too large for one launch");
    for (long long i = 0; i < 3LL * n_nodes; i++)
        if (!is_finite(X[i])) return fail(FEM_E_INVALID, "non-finite node coordinate");
    for (long long i = 0; i < 4LL * n_tets; i++)
        if (tets[i] < 0 || tets[i] >= n_nodes) return fail(FEM_E_INVALID, "tet index out of range");
    fem_config c = {FEM_PREC_FP64, 0, nullptr};
    if (cfg) c = *cfg;
    if (c.precision != FEM_PREC_FP64 && c.precision != FEM_PREC_FP32) return fail(FEM_E_INVALID, "bad precision");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(FEM_E_DEVICE, "no HIP device");
    if (c.device < 0 || c.device >= ndev) return fail(FEM_E_INVALID, "bad device ordinal");
    fem_mesh *M = new (std::nothrow) fem_mesh();
    if (!M) return fail(FEM_E_OOM, "host allocation failed");
    M->device = c.device;
    M->precision = c.precision;
    M->n = n_nodes;
    M->m = n_tets;
    int rc = set_device(M);
    if (!rc) {
        if (c.stream) {
            M->stream = (hipStream_t)c.stream;
        } else if (hipStreamCreateWithFlags(&M->stream, hipStreamNonBlocking) == hipSuccess) {
            M->own_stream = true;
        } else {
            rc = fail(FEM_E_DEVICE, "stream creation failed");
        }
    }
    if (!rc && hipHostMalloc(&M->h_s, sizeof(Scalars)) != hipSuccess) rc = fail(FEM_E_OOM, "pinned allocation failed");
    if (!rc) rc = stage(M, 4096);
    if (!rc)
        rc = M->precision == FEM_PREC_FP32 ? create_impl<float>(M, X, tets, fixed)
                                           : create_impl<double>(M, X, tets, fixed);
    if (rc) {
        std::string msg = g_last_error;
        release(M);
        g_last_error = msg;
        return rc;
    }
    *out = M;
    return FEM_OK;
}

void fem_destroy_mesh(fem_mesh *mesh) { release(mesh); }

int fem_set_material(fem_mesh *M, double E, double nu, double density) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    if (!is_finite(E) || !is_finite(nu) || !is_finite(density) || !(E > 0) || !(nu > -1.0) || !(nu < 0.5) || density < 0)
        return fail(FEM_E_INVALID, "need E > 0, -1 < nu < 0.5, density >= 0");
    M->E = E;
    M->nu = nu;
    M->density = density;
    M->mu = E / (2.0 * (1.0 + nu));
    M->lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    M->have_material = true;
    return FEM_OK;
}

int fem_set_indenter(fem_mesh *M, int32_t kind, const double *shape, int32_t n_shape, const double R[9],
                     const double c[3], double k_penalty) {
    g_last_error.clear();
    if (!M || !shape || !R || !c) return fail(FEM_E_INVALID, "null argument");
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
            double s = R[i] * R[j] + R[3 + i] * R[3 + j] + R[6 + i] * R[6 + j];
            if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-9) return fail(FEM_E_INVALID, "R is not orthonormal");
        }
    const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                       R[2] * (R[3] * R[7] - R[4] * R[6]);
    if (det < 0) return fail(FEM_E_INVALID, "R is a reflection");
    if (!is_finite(c[0]) || !is_finite(c[1]) || !is_finite(c[2]) || !is_finite(k_penalty) || k_penalty < 0)
        return fail(FEM_E_INVALID, "bad centre or penalty");
    Indenter ind{};
    ind.kind = kind;
    for (int i = 0; i < 4; i++) ind.shape[i] = i < need[kind] ? shape[i] : 0.0;
    for (int i = 0; i < 9; i++) ind.R[i] = R[i];
    for (int i = 0; i < 3; i++) ind.c[i] = c[i];
    ind.k = k_penalty;
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
        fem_default_params(&P, M->precision);
    int rc = check_params(P);
    if (rc) return rc;
    if ((rc = set_device(M))) return rc;
    fem_step_info local{};
    rc = M->precision == FEM_PREC_FP32 ? step_impl<float>(M, P, local) : step_impl<double>(M, P, local);
    local.status = rc;
    if (info) *info = local;
    return rc;
}

int fem_get_displacements(const fem_mesh *M, double *u, int64_t capacity) {
    g_last_error.clear();
    if (!M || !u) return fail(FEM_E_INVALID, "null argument");
    if (capacity < 3LL * M->n) return fail(FEM_E_BUFFER, "capacity below 3 n");
    int rc = set_device(M);
    if (rc) return rc;
    return download_real(M, u, M->u, 3 * (size_t)M->n);
}

int fem_set_displacements(fem_mesh *M, const double *u, int64_t count) {
    g_last_error.clear();
    if (!M || !u) return fail(FEM_E_INVALID, "null argument");
    if (count != 3LL * M->n) return fail(FEM_E_INVALID, "count must be 3 n");
    for (int64_t i = 0; i < count; i++)
        if (!is_finite(u[i])) return fail(FEM_E_INVALID, "non-finite displacement");
    int rc = set_device(M);
    if (rc) return rc;
    return upload_real(M, M->u, u, (size_t)count);
}

int fem_get_contact_patch(const fem_mesh *Mc, int32_t *ids, double *f, double *phi, int32_t capacity,
                          int32_t *n_contact, double F_total[3]) {
    g_last_error.clear();
    if (!Mc || !n_contact) return fail(FEM_E_INVALID, "null argument");
    fem_mesh *M = const_cast<fem_mesh *>(Mc);
    if (!M->have_indenter) return fail(FEM_E_STATE, "no indenter");
    int rc = set_device(M);
    if (rc) return rc;
    if (M->precision == FEM_PREC_FP32)
        k_contact_patch<float><<<1, 1024, 0, M->stream>>>(views<float>(M), M->patch_ids, M->patch_f, M->patch_phi,
                                                            M->patch_count, M->patch_F);
    else
        k_contact_patch<double><<<1, 1024, 0, M->stream>>>(views<double>(M), M->patch_ids, M->patch_f, M->patch_phi,
                                                             M->patch_count, M->patch_F);
    if ((rc = launch_check("k_contact_patch"))) return rc;
    int count = 0;
    double Ft[3];
    HIP_TRY(hipMemcpyAsync(&count, M->patch_count, sizeof(int), hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipMemcpyAsync(Ft, M->patch_F, sizeof Ft, hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
    *n_contact = count;
    if (F_total) std::memcpy(F_total, Ft, sizeof Ft);
    if (capacity < count) return fail(FEM_E_BUFFER, "capacity below the contact count");
    if (count > 0) {
        if (ids) HIP_TRY(hipMemcpyAsync(ids, M->patch_ids, count * sizeof(int), hipMemcpyDeviceToHost, M->stream));
        if (f) HIP_TRY(hipMemcpyAsync(f, M->patch_f, 3 * (size_t)count * sizeof(double), hipMemcpyDeviceToHost, M->stream));
        if (phi) HIP_TRY(hipMemcpyAsync(phi, M->patch_phi, count * sizeof(double), hipMemcpyDeviceToHost, M->stream));
        HIP_TRY(hipStreamSynchronize(M->stream));
    }
    return FEM_OK;
}

int fem_get_mesh_info(const fem_mesh *M, int32_t *n_nodes, int32_t *n_tets, int32_t *n_eligible, uint8_t *eligible,
                      int32_t capacity) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    if (n_nodes) *n_nodes = M->n;
    if (n_tets) *n_tets = M->m;
    if (n_eligible) *n_eligible = M->nc;
    if (eligible) {
        if (capacity < M->n) return fail(FEM_E_BUFFER, "capacity below n");
        int rc = set_device(M);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(eligible, M->eligible, M->n, hipMemcpyDeviceToHost, M->stream));
        HIP_TRY(hipStreamSynchronize(M->stream));
    }
    return FEM_OK;
}

int fem_eval_gradient(fem_mesh *M, double *g, int64_t capacity, double *energy, double *min_J) {
    g_last_error.clear();
    if (!M) return fail(FEM_E_INVALID, "null mesh");
    if (!M->have_material || !M->have_indenter) return fail(FEM_E_STATE, "set material and indenter first");
    if (g && capacity < 3LL * M->n) return fail(FEM_E_BUFFER, "capacity below 3 n");
    int rc = set_device(M);
    if (rc) return rc;
    rc = M->precision == FEM_PREC_FP32 ? element_pass<float>(M, 0.0f, true, 1) : element_pass<double>(M, 0.0, true, 1);
    if (rc) return rc;
    if ((rc = fetch_scalars(M))) return rc;
    if (energy) *energy = M->h_s->energy;
    if (min_J) *min_J = M->h_s->minJ;
    if (g) return download_real(M, g, M->g, 3 * (size_t)M->n);
    return FEM_OK;
}

int fem_eval_hessvec(fem_mesh *M, const fem_solve_params *params, const double *v, double *q, int64_t capacity) {
    g_last_error.clear();
    if (!M || !v || !q) return fail(FEM_E_INVALID, "null argument");
    if (!M->have_material || !M->have_indenter) return fail(FEM_E_STATE, "set material and indenter first");
    if (capacity < 3LL * M->n) return fail(FEM_E_BUFFER, "capacity below 3 n");
    fem_solve_params P;
    if (params)
        P = *params;
    else
        fem_default_params(&P, M->precision);
    int rc = set_device(M);
    if (rc) return rc;
    const bool f32 = M->precision == FEM_PREC_FP32;
    const int cf = P.contact_hessian ? 1 : 0;
    rc = f32 ? element_pass<float>(M, 0.0f, true, cf) : element_pass<double>(M, 0.0, true, cf);
    if (rc) return rc;
    // q = H v with p = z + beta p_prev: z = v, p_prev = 0, beta = 0.
    if ((rc = upload_real(M, M->z, v, 3 * (size_t)M->n))) return rc;
    HIP_TRY(hipMemsetAsync(M->p, 0, 3 * (size_t)M->n * M->elem(), M->stream));
    HIP_TRY(hipMemsetAsync(M->q, 0, 3 * (size_t)M->n * M->elem(), M->stream));
    HIP_TRY(hipMemsetAsync(&M->s->beta, 0, sizeof(double), M->stream));
    const int tb = nblocks(M->m), cb = nblocks(M->nc);
    if (f32)
        k_cg_hv<float><<<tb + cb, kBlock, 0, M->stream>>>(views<float>(M), tb, 1);
    else
        k_cg_hv<double><<<tb + cb, kBlock, 0, M->stream>>>(views<double>(M), tb, 1);
    if ((rc = launch_check("k_cg_hv"))) return rc;
    return download_real(M, q, M->q, 3 * (size_t)M->n);
}

}  // extern "C"
