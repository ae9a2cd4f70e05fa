// Device kernels of the indentation solve for gfx950 (CDNA4, wave64).
//
// Data layout in HBM.
//   Topology (shared by every instance of one mesh): nodes numbered by first
//   touch along the tets' Morton order; tets in Morton order, cut into tiles
//   of at most kTileTets tets that touch at most kTileNodes distinct nodes.
//   Per tile: its node list ("entries", global ids). Per tet, in tile order,
//   one record of D_m^-1, V (computed once in FP64) and four 8-bit local node
//   slots. Node -> entry CSR lists for the deterministic gather of tile
//   partial sums.
//   Instance state: node vectors packed xyz (n x 3), tile partial sums per
//   entry, contact blocks per contact-eligible node, FP64 solver scalars.
//
// Per pass a tile block stages its entries' state vectors in LDS, reads each
// tet's record (shared by every job on the mesh, so a tile's records are
// fetched once per XCD and reused from L2 by the other jobs), recomputes F
// from u, accumulates nodal contributions with FP64 LDS atomics and writes
// one partial per entry; node kernels gather those partials. Global memory
// sees no atomics in the solve kernels.
//
// Control: each instance runs a Newton / PCG / line-search state machine on
// the device. Work kernels write one FP64 partial per block and per reduced
// quantity; a finalize kernel (one wavefront per instance) sums them in a
// fixed order and takes the transition, so no kernel needs cross-block
// synchronisation (an agent-scope fence per block costs an L2 write-back on
// this part). A solver step is a tile pass, a node pass and a finalize over
// every running instance; each instance advances by one phase per step
// (a CG iteration, a line-search trial, a Newton init), whatever phase the
// others are in.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace fem {

constexpr int kBlock = 256;       // 4 wavefronts of 64
constexpr int kWaves = kBlock / 64;
constexpr int kGather = 4;        // node pass: tile entries per node held with the node (node_ent4)
static_assert(kGather == 4, "node_ent4 holds four entries");
constexpr int kTileTets = 512;    // tets per tile (2 per thread)
constexpr int kTileNodes = 256;   // distinct nodes per tile (8-bit local ids)
static_assert(kTileNodes <= kBlock, "the tile passes stage one entry per thread");
constexpr int kDetElemChunk = 128; // deterministic element pass: tets per chunk of contributions
constexpr int kHistSteps = 1024;  // load steps whose status a job records

enum Phase : int {
    PH_IDLE = 0,
    PH_GRAD = 1,      // element pass at u, then Newton init (start of a load step)
    PH_INIT = 2,      // Newton init after an accepted line-search trial
    PH_CG = 3,        // CG iterations
    PH_TRIAL = 4,     // line-search trial: element pass at u + alpha dx
    PH_DONE = 5,      // all load steps taken
    PH_EVAL_GRAD = 6, // diagnostics: gradient at u, then idle
    PH_EVAL_HV = 7,   // diagnostics: q = H z, then idle
    PH_LAG = 8        // node pass forms the friction lag data, then after_lag
};

// Status codes (same values as the C ABI).
enum : int { ST_OK = 0, ST_FLOOR = 1, ST_NOT_CONVERGED = -6, ST_INVERSION = -7 };

// Partial-sum streams of an instance (each red_stride doubles).
// RS_EN: inertial energy of implicit time steps (node blocks). RS_PQN: slot 0
// holds p.q as every node block summed it (written by node block 0), which the
// finalize takes, so the CG decision and the update applied always agree.
enum : int { RS_PQ = 0, RS_RZ, RS_RR, RS_GD, RS_E, RS_MAG, RS_MINJ, RS_GG, RS_IRZ, RS_EN, RS_PQN, RS_COUNT };

struct Indenter {
    int kind;            // 0 sphere, 1 cylinder, 2 box, 3 ring
    double shape[4];
    double R[9];         // row-major, local -> world
    double c[3];
    double k;
};

struct SolveParams {
    double newton_rtol, newton_atol, cg_rtol, cg_eta_max, c1, noise_eps, floor_rtol, eta_power;
    int max_newton, max_cg, block_jacobi, contact_full, max_halvings, pad;
};

// Dynamic state of one instance (device-resident; the host reads it).
struct InstState {
    int phase, step, steps, step_started;
    int newton_it, cg_it, halvings, apply;
    int status, last_status, last_cg, need_gd;   // last_cg: length of the previous CG solve
    double rz, rr, pq, alpha, beta, tol2;
    double E, emag, minJ, gg, r0, gd, alpha_ls;
    double mu, lam, depth;
    double dt, rho;                           // implicit time step (0: quasi-static), density
    double mdt2;                              // rho / dt^2 (0: quasi-static)
    double gbest;                             // smallest |g_free| of the load step so far
    int stall, steps_floor;                   // accepted iterations without halving gbest
    int model, pad3;                          // constitutive law (LAW_NH, LAW_CR)
    double mu_f, eps_f;                       // Coulomb friction coefficient (0: none), slip smoothing length
    double c_lag[3];                          // indenter centre of the friction lag state
    int lag_ok, after_lag;                    // 1: a lag state exists (u at the step start, c_lag);
                                              // the phase that follows PH_LAG
    double c0[3], dir[3];
    Indenter ind;
    // current load step
    int st_newton, st_cg, st_hv, st_grad, st_ls, pad1;
    double st_g0, st_g;
    // whole job
    long long tot_newton, tot_cg, tot_hv, tot_grad, tot_ls;
    int steps_ok, steps_failed, first_fail, pad2;
};

// Per-tet record in tile order: D_m^-1 (row a = shape gradient of local node
// a+1), rest volume and the four 8-bit local node slots, padded to a multiple
// of 16 bytes so a lane fetches its tet with 16-byte loads from one address.
template <typename T> struct TetRec;
template <> struct alignas(16) TetRec<float> {
    float Bm[9];
    float V;
    uint32_t loc;
    uint32_t pad;
};
template <> struct alignas(16) TetRec<double> {
    double Bm[9];
    double V;
    uint32_t loc;
    uint32_t pad[3];
};
static_assert(sizeof(TetRec<float>) == 48 && sizeof(TetRec<double>) == 96, "tet record layout");

// Buffer pointers of the descriptors below. The host fills them as plain
// pointers; kernels read them through a device view (DEV = true, same
// layout) whose pointers are in the global address space, so accesses
// compile to global memory instructions instead of flat ones (a flat
// instruction also counts against the LDS counter, which makes every wait
// for an LDS result wait for the outstanding memory loads as well).
#ifdef __HIP_DEVICE_COMPILE__
template <class U> using glob_ptr = U __attribute__((address_space(1))) *;
#else
template <class U> using glob_ptr = U *;
#endif
template <class U, bool DEV> using buf_ptr = std::conditional_t<DEV, glob_ptr<U>, U *>;

template <typename T, bool DEV = false>
struct Topo {
    int n, m, ntile, nent, nc, ncb;                 // ncb = contact blocks
    int n_free, pad0;                               // nodes 0 .. n_free-1 are free, the rest fixed
    buf_ptr<const int, DEV> tile_tet;               // ntile + 1
    buf_ptr<const int, DEV> tile_ent;               // ntile + 1
    buf_ptr<const int, DEV> ent_node;               // nent: node of each entry (ascending within a tile)
    buf_ptr<const uint8_t, DEV> ent_slot;           // nent: LDS slot of each entry (local id in the tet records)
    buf_ptr<const TetRec<T>, DEV> rec;              // m, tile order
    buf_ptr<const int, DEV> node_ent_off;           // n + 1
    buf_ptr<const int, DEV> node_ent;               // nent
    buf_ptr<const int4, DEV> node_ent4;             // n: each node's first kGather entries (-1 past its last)
    buf_ptr<const int, DEV> inc_off;                // nent + 1: each tile entry's incident (tet, slot) pairs
    buf_ptr<const uint16_t, DEV> inc;               // 4 m: (local tet << 2 | slot), ascending tet per entry
    buf_ptr<const uint8_t, DEV> fixed;              // n
    buf_ptr<const int, DEV> cnodes;                 // nc
    buf_ptr<const int, DEV> cidx;                   // n: contact slot or -1
    buf_ptr<const double, DEV> X;                   // n x 3
    buf_ptr<const T, DEV> nvol;                     // n: lumped volume share sum_e V_e / 4
    buf_ptr<const uint8_t, DEV> owner;              // nent: 1 on each node's first entry
    buf_ptr<const int, DEV> tet_id;                 // m: input index of the tet at each tile position
};

template <typename T, bool DEV = false>
struct InstBufs {
    int topo;
    int red_stride;                                 // partial slots per reduction stream
    buf_ptr<T, DEV> u, dx, g, r, z, p, dinv;        // dinv n x 6, others n x 3
    buf_ptr<T, DEV> pg;                             // nent x 9: gradient (3) + node block (6) partials
    buf_ptr<T, DEV> pq;                             // nent x 3: Hv partials
    buf_ptr<T, DEV> cp;                             // nc x 9: contact gradient (3) + block (6)
    buf_ptr<uint8_t, DEV> cact;                     // nc: 1 where that block is nonzero
    buf_ptr<T, DEV> qout;                           // n x 3 (diagnostics)
    buf_ptr<T, DEV> v, ut;                          // n x 3: velocity of the last completed step, inertial predictor
    buf_ptr<double, DEV> fr;                        // nc x 8: friction lag data (w, normal, displacement
                                                    // relative to the indenter since the lag state, pad)
    buf_ptr<double, DEV> red;                       // RS_COUNT x red_stride
    buf_ptr<signed char, DEV> hist;                 // kHistSteps: status of each load step taken (ST_*)
    buf_ptr<InstState, DEV> s;
};

// Device views of descriptors read from device memory.
template <typename T> using TopoD = Topo<T, true>;
template <typename T> using BufsD = InstBufs<T, true>;
template <typename T> __device__ __forceinline__ TopoD<T> dev_view(const Topo<T> &t) {
    return __builtin_bit_cast(TopoD<T>, t);
}
template <typename T> __device__ __forceinline__ BufsD<T> dev_view(const InstBufs<T> &b) {
    return __builtin_bit_cast(BufsD<T>, b);
}

// ---------------------------------------------------------------------------
// Work mapping: blocks are dealt to the 8 XCDs round-robin, so logical work
// item L is given to hardware block (L % per) * 8 + L / per; consecutive work
// items (same tile of consecutive instances) then share an XCD and its L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int logical_block() {
    const int per = gridDim.x >> 3;
    const int b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
// Wavefront reductions with DPP lane moves (vector ALU, no LDS traffic): a
// prefix sum within each row of 16 lanes (row_shr 1, 2, 4, 8), then the row
// totals carried across rows (row_bcast 15 and 31), so lane 63 holds the
// result, which is broadcast. The order is fixed: every wavefront that
// reduces the same values gets the same bits. Lanes without a source take
// the identity (`empty`, as two 32-bit halves).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v, int empty_lo, int empty_hi) {
    const int lo = __builtin_amdgcn_update_dpp(empty_lo, __double2loint(v), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(empty_hi, __double2hiint(v), CTRL, ROWMASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane63(double v) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0x111, 0xf>(v, 0, 0);   // row_shr:1
    v += dpp_move<0x112, 0xf>(v, 0, 0);   // row_shr:2
    v += dpp_move<0x114, 0xf>(v, 0, 0);   // row_shr:4
    v += dpp_move<0x118, 0xf>(v, 0, 0);   // row_shr:8
    v += dpp_move<0x142, 0xa>(v, 0, 0);   // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v, 0, 0);   // row_bcast:31 into rows 2 and 3
    return lane63(v);
}

__device__ __forceinline__ double wave_min(double v) {
    const int ilo = 0, ihi = 0x7ff00000;  // +inf
    v = fmin(v, dpp_move<0x111, 0xf>(v, ilo, ihi));
    v = fmin(v, dpp_move<0x112, 0xf>(v, ilo, ihi));
    v = fmin(v, dpp_move<0x114, 0xf>(v, ilo, ihi));
    v = fmin(v, dpp_move<0x118, 0xf>(v, ilo, ihi));
    v = fmin(v, dpp_move<0x142, 0xa>(v, ilo, ihi));
    v = fmin(v, dpp_move<0x143, 0xc>(v, ilo, ihi));
    return lane63(v);
}

template <int NS, bool MIN>
__device__ __forceinline__ void block_reduce(double (&v)[NS], double &mn) {
    __shared__ double lds[kWaves][NS + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NS; i++) v[i] = wave_sum(v[i]);
    if (MIN) mn = wave_min(mn);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NS; i++) lds[w][i] = v[i];
        if (MIN) lds[w][NS] = mn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NS; i++) {
            double t = lds[0][i];
            for (int k = 1; k < kWaves; k++) t += lds[k][i];
            v[i] = t;
        }
        if (MIN) {
            double t = lds[0][NS];
            for (int k = 1; k < kWaves; k++) t = fmin(t, lds[k][NS]);
            mn = t;
        }
    }
    __syncthreads();
}

// Wavefront sum / min of nb partials in a fixed order: lane l adds partials
// l, l + 64, ..., then the wavefront tree. Every wavefront that calls it gets
// the same value (finalize kernel; the node pass's p.q, formed by each of its
// wavefronts without a block barrier).
__device__ __forceinline__ double wave_sum_partials(const double *part, int nb) {
    double v = 0.0;
    for (int b = threadIdx.x & 63; b < nb; b += 64) v += part[b];
    return wave_sum(v);
}

__device__ __forceinline__ double wave_min_partials(const double *part, int nb) {
    double v = INFINITY;
    for (int b = threadIdx.x; b < nb; b += 64) v = fmin(v, part[b]);
    return wave_min(v);
}

// ---------------------------------------------------------------------------
// Scalar helpers
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T fma_t(T a, T b, T c);
template <> __device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> __device__ __forceinline__ T log1p_t(T x);
template <> __device__ __forceinline__ float log1p_t<float>(float x) { return log1pf(x); }
template <> __device__ __forceinline__ double log1p_t<double>(double x) { return log1p(x); }

template <typename T> __device__ __forceinline__ T abs_t(T x) { return x < (T)0 ? -x : x; }

template <typename T> __device__ __forceinline__ T safe_recip(T d) {
    return d > (T)0 ? (T)1 / d : (d < (T)0 ? (T)1 / -d : (T)1);
}

// ---------------------------------------------------------------------------
// Element kinematics from LDS-staged tile data.
// ---------------------------------------------------------------------------
template <typename T>
struct ElemGeo {
    T Bm[9];   // D_m^-1, row a = shape gradient of local node a+1
    T V;
};

__device__ __forceinline__ void unpack_loc(uint32_t w, int l[4]) {
    l[0] = w & 0xff;
    l[1] = (w >> 8) & 0xff;
    l[2] = (w >> 16) & 0xff;
    l[3] = w >> 24;
}

// Rest constants and local node slots of tet k (tile order) from the per-mesh
// records, fetched as whole 16-byte words (fetch_tet) and unpacked once they
// are needed (unpack_tet), so a fetch can be issued ahead of its use.
template <typename T> struct TetWords {
    uint4 w[sizeof(TetRec<T>) / 16];
};

template <typename T>
__device__ __forceinline__ void fetch_tet(const TopoD<T> &tp, int k, TetWords<T> &tw) {
    const uint4 *src = reinterpret_cast<const uint4 *>(tp.rec + k);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(TetRec<T>) / 16); i++) tw.w[i] = src[i];
}

template <typename T>
__device__ __forceinline__ ElemGeo<T> unpack_tet(const TetWords<T> &tw, int l[4]) {
    TetRec<T> r;
    __builtin_memcpy(&r, tw.w, sizeof r);
    ElemGeo<T> g;
#pragma unroll
    for (int c = 0; c < 9; c++) g.Bm[c] = r.Bm[c];
    g.V = r.V;
    unpack_loc(r.loc, l);
    return g;
}

// Hessian-path helpers: the Hessian only steers the Newton direction (the
// solution is fixed by the gradient), so the tangent's ln J and 1/J use a
// short series and the hardware reciprocal instead of the correctly rounded
// library routines; ~1e-7 relative in FP32, ~1e-13 in FP64 for |J - 1| < 1/2.
template <typename T> __device__ __forceinline__ T fast_rcp(T x);
template <> __device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double fast_rcp<double>(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return r;
}

// ln(1 + x) = 2 atanh(s), s = x / (2 + x); |s| <= 0.2 for |x| <= 1/2.
template <typename T>
__device__ __forceinline__ T fast_log1p(T x) {
    if (!(x > (T)-0.5 && x < (T)0.5)) return log1p_t(x);
    const T s = x * fast_rcp((T)2 + x);
    const T s2 = s * s;
    T p;
    if (sizeof(T) == 4) {
        p = fma_t(s2, (T)(1.0 / 9.0), (T)(1.0 / 7.0));
        p = fma_t(s2, p, (T)(1.0 / 5.0));
    } else {
        p = fma_t(s2, (T)(1.0 / 21.0), (T)(1.0 / 19.0));
        p = fma_t(s2, p, (T)(1.0 / 17.0));
        p = fma_t(s2, p, (T)(1.0 / 15.0));
        p = fma_t(s2, p, (T)(1.0 / 13.0));
        p = fma_t(s2, p, (T)(1.0 / 11.0));
        p = fma_t(s2, p, (T)(1.0 / 9.0));
        p = fma_t(s2, p, (T)(1.0 / 7.0));
        p = fma_t(s2, p, (T)(1.0 / 5.0));
    }
    p = fma_t(s2, p, (T)(1.0 / 3.0));
    p = fma_t(s2, p, (T)1);
    return (T)2 * s * p;
}

// Staged node vectors in LDS: kSw values per entry (x, y, z, unused), so a
// node is one aligned 4-vector read.
constexpr int kSw = 4;
template <typename T> using vec4_t = T __attribute__((ext_vector_type(4)));

// The four nodes' staged vectors of one tet, read once into registers.
template <typename T>
__device__ __forceinline__ void load_nodes(const T *sw, const int l[4], T w[4][3]) {
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const vec4_t<T> v = *reinterpret_cast<const vec4_t<T> *>(sw + kSw * l[a]);
        w[a][0] = v.x;
        w[a][1] = v.y;
        w[a][2] = v.z;
    }
}

// G = sum_a (w_{a+1} - w_0) (x) row_a(D_m^-1).
template <typename T>
__device__ __forceinline__ void edge_gradient(const T w[4][3], const T Bm[9], T G[9]) {
    T d[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int i = 0; i < 3; i++) d[a][i] = w[a + 1][i] - w[0][i];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) G[3 * i + j] = d[0][i] * Bm[j] + d[1][i] * Bm[3 + j] + d[2][i] * Bm[6 + j];
}

// J - 1 = tr G + (sum of principal 2x2 minors of G) + det G, free of the
// cancellation of det(I + G) - 1.
template <typename T>
__device__ __forceinline__ T det_minus_one(const T G[9]) {
    const T trG = G[0] + G[4] + G[8];
    const T m2 = (G[0] * G[4] - G[1] * G[3]) + (G[0] * G[8] - G[2] * G[6]) + (G[4] * G[8] - G[5] * G[7]);
    const T dG = G[0] * (G[4] * G[8] - G[5] * G[7]) - G[1] * (G[3] * G[8] - G[5] * G[6]) + G[2] * (G[3] * G[7] - G[4] * G[6]);
    return trG + m2 + dG;
}

// F^-T = cof(F) / J (FAST: hardware reciprocal, Hessian path only).
template <typename T, bool FAST = false>
__device__ __forceinline__ void inverse_transpose(const T G[9], T J, T FiT[9]) {
    T F[9];
#pragma unroll
    for (int k = 0; k < 9; k++) F[k] = G[k];
    F[0] += (T)1; F[4] += (T)1; F[8] += (T)1;
    const T iJ = FAST ? fast_rcp(J) : (T)1 / J;
    FiT[0] = (F[4] * F[8] - F[5] * F[7]) * iJ;
    FiT[1] = (F[5] * F[6] - F[3] * F[8]) * iJ;
    FiT[2] = (F[3] * F[7] - F[4] * F[6]) * iJ;
    FiT[3] = (F[2] * F[7] - F[1] * F[8]) * iJ;
    FiT[4] = (F[0] * F[8] - F[2] * F[6]) * iJ;
    FiT[5] = (F[1] * F[6] - F[0] * F[7]) * iJ;
    FiT[6] = (F[1] * F[5] - F[2] * F[4]) * iJ;
    FiT[7] = (F[2] * F[3] - F[0] * F[5]) * iJ;
    FiT[8] = (F[0] * F[4] - F[1] * F[3]) * iJ;
}

// ---------------------------------------------------------------------------
// Constitutive laws, per tet from G = F - I (J - 1 and J given).
//   element(): energy density (sum and rounding magnitude of its terms), the
//     first Piola-Kirchhoff stress P, and the node diagonal block of the
//     element's Hessian (or its fixed-rotation part) in the form
//     V (alpha |b|^2 I + beta c c^T), c = Mb b.
//   hessvec(): dP for the perturbation dG.
// LAW_NH, compressible Neo-Hookean: Psi = mu/2 (tr F^T F - 3) - mu ln J +
//   lam/2 ln^2 J. LAW_CR, co-rotational linear elasticity (F = R S):
//   Psi = mu |F - R|^2 + lam/2 (tr S - 3)^2, P = 2 mu (F - R) + lam (tr S - 3) R.
// ---------------------------------------------------------------------------
enum : int { LAW_NH = 0, LAW_CR = 1 };

template <typename T, int LAW> struct Law;

template <typename T> struct Law<T, LAW_NH> {
    __device__ static __forceinline__ void element(const T G[9], T Jm1, T J, T mu, T lam, T &psi, T &mag, T P[9],
                                                   T Mb[9], T &alpha, T &beta) {
        const T lnJ = log1p_t(Jm1);
        const T trG = G[0] + G[4] + G[8];
        T G2 = (T)0;
#pragma unroll
        for (int c = 0; c < 9; c++) G2 += G[c] * G[c];
        const T t1 = (T)0.5 * mu * ((T)2 * trG + G2), t2 = -mu * lnJ, t3 = (T)0.5 * lam * lnJ * lnJ;
        psi = t1 + t2 + t3;
        mag = abs_t(t1) + abs_t(t2) + abs_t(t3);
        inverse_transpose(G, J, Mb);
        // P = mu (F - F^-T) + lam ln J F^-T with F - F^-T = G + F^-T G^T, which
        // keeps full relative precision at small strain.
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const T FG = Mb[3 * i] * G[3 * j] + Mb[3 * i + 1] * G[3 * j + 1] + Mb[3 * i + 2] * G[3 * j + 2];
                P[3 * i + j] = mu * (G[3 * i + j] + FG) + lam * lnJ * Mb[3 * i + j];
            }
        alpha = mu;
        beta = mu + lam - lam * lnJ;
    }

    // dP = mu dG + (mu - lam ln J) (F^-1 dG F^-1)^T + lam tr(F^-1 dG) F^-T
    __device__ static __forceinline__ void hessvec(const T G[9], T Jm1, T J, const T dG[9], T mu, T lam, T dP[9]) {
        const T cc = mu - lam * fast_log1p(Jm1);
        T FiT[9];
        inverse_transpose<T, true>(G, J, FiT);
        // A = F^-1 dG (F^-1 = FiT^T)
        T A[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) A[3 * i + j] = FiT[i] * dG[j] + FiT[3 + i] * dG[3 + j] + FiT[6 + i] * dG[6 + j];
        const T tr = A[0] + A[4] + A[8];
        // (A F^-1)^T_ij = sum_k A_jk FiT_ik
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                const T Mt = A[3 * j] * FiT[3 * i] + A[3 * j + 1] * FiT[3 * i + 1] + A[3 * j + 2] * FiT[3 * i + 2];
                dP[3 * i + j] = mu * dG[3 * i + j] + cc * Mt + lam * tr * FiT[3 * i + j];
            }
    }
};

// Rotation factor of F = I + G (det F > 0) by Newton's iteration for the
// polar decomposition with determinant scaling, X <- (g X + X^-T / g) / 2,
// g = |det X|^(-1/3), to convergence at the working precision.
template <typename T>
__device__ __forceinline__ void polar_rotation(const T G[9], T R[9]) {
#pragma unroll
    for (int c = 0; c < 9; c++) R[c] = G[c];
    R[0] += (T)1;
    R[4] += (T)1;
    R[8] += (T)1;
    const T tol = sizeof(T) == 4 ? (T)8e-7 : (T)4e-15;
    for (int it = 0; it < 12; it++) {
        T C[9];   // cofactors: X^-T = C / det
        C[0] = R[4] * R[8] - R[5] * R[7];
        C[1] = R[5] * R[6] - R[3] * R[8];
        C[2] = R[3] * R[7] - R[4] * R[6];
        C[3] = R[2] * R[7] - R[1] * R[8];
        C[4] = R[0] * R[8] - R[2] * R[6];
        C[5] = R[1] * R[6] - R[0] * R[7];
        C[6] = R[1] * R[5] - R[2] * R[4];
        C[7] = R[2] * R[3] - R[0] * R[5];
        C[8] = R[0] * R[4] - R[1] * R[3];
        const T det = R[0] * C[0] + R[1] * C[1] + R[2] * C[2];
        const float g = exp2f(-log2f((float)abs_t(det)) * (1.0f / 3.0f));
        const T a = (T)0.5 * (T)g, b = (T)0.5 / ((T)g * det);
        T diff = (T)0;
#pragma unroll
        for (int c = 0; c < 9; c++) {
            const T x = a * R[c] + b * C[c];
            diff = fmax(diff, abs_t(x - R[c]));
            R[c] = x;
        }
        if (diff <= tol) break;
    }
}

template <typename T> struct Law<T, LAW_CR> {
    // R, and E = S - I formed without cancellation as (C - I)(S + I)^-1 with
    // C - I = G + G^T + G^T G (C = F^T F, S = R^T F, S + I near 2 I).
    __device__ static __forceinline__ void rotation_strain(const T G[9], T R[9], T E[9]) {
        polar_rotation(G, R);
        T S[9], E2[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                // S = R^T (I + G)
                S[3 * i + j] = R[3 * 0 + i] * G[3 * 0 + j] + R[3 * 1 + i] * G[3 * 1 + j] + R[3 * 2 + i] * G[3 * 2 + j] +
                               R[3 * j + i];
                E2[3 * i + j] = G[3 * i + j] + G[3 * j + i] +
                                (G[3 * 0 + i] * G[3 * 0 + j] + G[3 * 1 + i] * G[3 * 1 + j] + G[3 * 2 + i] * G[3 * 2 + j]);
            }
        // (S + I)^-1, S symmetrised
        T A[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) A[3 * i + j] = (T)0.5 * (S[3 * i + j] + S[3 * j + i]) + (i == j ? (T)1 : (T)0);
        T Ai[9];
        Ai[0] = A[4] * A[8] - A[5] * A[7];
        Ai[1] = A[2] * A[7] - A[1] * A[8];
        Ai[2] = A[1] * A[5] - A[2] * A[4];
        Ai[3] = A[5] * A[6] - A[3] * A[8];
        Ai[4] = A[0] * A[8] - A[2] * A[6];
        Ai[5] = A[2] * A[3] - A[0] * A[5];
        Ai[6] = A[3] * A[7] - A[4] * A[6];
        Ai[7] = A[1] * A[6] - A[0] * A[7];
        Ai[8] = A[0] * A[4] - A[1] * A[3];
        const T id = (T)1 / (A[0] * Ai[0] + A[1] * Ai[3] + A[2] * Ai[6]);
        T Q[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++)
                Q[3 * i + j] = (E2[3 * i] * Ai[j] + E2[3 * i + 1] * Ai[3 + j] + E2[3 * i + 2] * Ai[6 + j]) * id;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) E[3 * i + j] = (T)0.5 * (Q[3 * i + j] + Q[3 * j + i]);
    }

    __device__ static __forceinline__ void element(const T G[9], T Jm1, T J, T mu, T lam, T &psi, T &mag, T P[9],
                                                   T Mb[9], T &alpha, T &beta) {
        T E[9];
        rotation_strain(G, Mb, E);
        const T trE = E[0] + E[4] + E[8];
        T E2 = (T)0;
#pragma unroll
        for (int c = 0; c < 9; c++) E2 += E[c] * E[c];
        psi = mu * E2 + (T)0.5 * lam * trE * trE;   // |F - R| = |R (S - I)| = |E|
        mag = psi;
        // P = R (2 mu E + lam tr E I)
        T X[9];
#pragma unroll
        for (int c = 0; c < 9; c++) X[c] = (T)2 * mu * E[c];
        X[0] += lam * trE;
        X[4] += lam * trE;
        X[8] += lam * trE;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++)
                P[3 * i + j] = Mb[3 * i] * X[j] + Mb[3 * i + 1] * X[3 + j] + Mb[3 * i + 2] * X[6 + j];
        alpha = (T)2 * mu;
        beta = lam;
    }

    // R and E = sym(R^T F) - I formed directly: in the tangent E only enters
    // through tr S I - S = (2 + tr E) I - E and lam tr E dR, where its
    // rounding (absolute, about the working precision) is negligible.
    __device__ static __forceinline__ void rotation_strain_direct(const T G[9], T R[9], T E[9]) {
        polar_rotation(G, R);
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = i; j < 3; j++) {
                // S_ij = (R^T (I + G))_ij, symmetrised
                const T sij = R[3 * 0 + i] * G[3 * 0 + j] + R[3 * 1 + i] * G[3 * 1 + j] + R[3 * 2 + i] * G[3 * 2 + j] +
                              R[3 * j + i];
                const T sji = R[3 * 0 + j] * G[3 * 0 + i] + R[3 * 1 + j] * G[3 * 1 + i] + R[3 * 2 + j] * G[3 * 2 + i] +
                              R[3 * i + j];
                const T e = (T)0.5 * (sij + sji) - (i == j ? (T)1 : (T)0);
                E[3 * i + j] = e;
                E[3 * j + i] = e;
            }
    }

    // dP = 2 mu (dG - dR) + lam tr(R^T dG) R + lam tr E dR, dR = R [w]x with
    // (tr S I - S) w = axial(R^T dG - dG^T R).
    __device__ static __forceinline__ void hessvec(const T G[9], T Jm1, T J, const T dG[9], T mu, T lam, T dP[9]) {
        T R[9], E[9];
        rotation_strain_direct(G, R, E);
        T M[9];   // R^T dG
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) M[3 * i + j] = R[i] * dG[j] + R[3 + i] * dG[3 + j] + R[6 + i] * dG[6 + j];
        const T ax[3] = {M[7] - M[5], M[2] - M[6], M[3] - M[1]};
        const T trE = E[0] + E[4] + E[8];
        // K = tr S I - S = (2 + tr E) I - E (symmetric)
        const T k00 = (T)2 + trE - E[0], k11 = (T)2 + trE - E[4], k22 = (T)2 + trE - E[8];
        const T k01 = -E[1], k02 = -E[2], k12 = -E[5];
        const T c00 = k11 * k22 - k12 * k12, c01 = k02 * k12 - k01 * k22, c02 = k01 * k12 - k02 * k11;
        const T c11 = k00 * k22 - k02 * k02, c12 = k01 * k02 - k00 * k12, c22 = k00 * k11 - k01 * k01;
        const T kid = (T)1 / (k00 * c00 + k01 * c01 + k02 * c02);
        const T w0 = (c00 * ax[0] + c01 * ax[1] + c02 * ax[2]) * kid;
        const T w1 = (c01 * ax[0] + c11 * ax[1] + c12 * ax[2]) * kid;
        const T w2 = (c02 * ax[0] + c12 * ax[1] + c22 * ax[2]) * kid;
        const T trM = M[0] + M[4] + M[8];
        // dR = R W, W = [[0, -w2, w1], [w2, 0, -w0], [-w1, w0, 0]]
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const T r0 = R[3 * i], r1 = R[3 * i + 1], r2 = R[3 * i + 2];
            const T dR0 = r1 * w2 - r2 * w1, dR1 = r2 * w0 - r0 * w2, dR2 = r0 * w1 - r1 * w0;
            dP[3 * i + 0] = (T)2 * mu * (dG[3 * i + 0] - dR0) + lam * trM * r0 + lam * trE * dR0;
            dP[3 * i + 1] = (T)2 * mu * (dG[3 * i + 1] - dR1) + lam * trM * r1 + lam * trE * dR1;
            dP[3 * i + 2] = (T)2 * mu * (dG[3 * i + 2] - dR2) + lam * trM * r2 + lam * trE * dR2;
        }
    }
};

// Nodal vectors V S row_a(D_m^-1)^T for nodes a+1; node 0 gets minus the sum.
template <typename T>
__device__ __forceinline__ void element_nodal(const T S[9], const T Bm[9], T V, T f[4][3]) {
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int i = 0; i < 3; i++)
            f[a + 1][i] = V * (S[3 * i] * Bm[3 * a] + S[3 * i + 1] * Bm[3 * a + 1] + S[3 * i + 2] * Bm[3 * a + 2]);
#pragma unroll
    for (int i = 0; i < 3; i++) f[0][i] = -(f[1][i] + f[2][i] + f[3][i]);
}

// ---------------------------------------------------------------------------
// Indenter signed distance in double precision: value, unit world gradient
// and, inside the indenter, the world Hessian (xx yy zz xy xz yz). Medial
// ties go to the lower axis (x, y, z) and to the radial branch before the
// axial one.
// ---------------------------------------------------------------------------
__device__ inline void sdf_eval(const Indenter &ind, const double x[3], bool want_h, double &phi, double n[3],
                                double Hw[6]) {
    const double *R = ind.R;
    const double d0 = x[0] - ind.c[0], d1 = x[1] - ind.c[1], d2 = x[2] - ind.c[2];
    double q[3];
#pragma unroll
    for (int k = 0; k < 3; k++) q[k] = R[k] * d0 + R[3 + k] * d1 + R[6 + k] * d2;
    double gq[3] = {0.0, 0.0, 0.0};
    double Hq[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    switch (ind.kind) {
    case 0: {
        const double L = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        phi = L - ind.shape[0];
        if (L > 0.0) {
            const double iL = 1.0 / L;
            gq[0] = q[0] * iL; gq[1] = q[1] * iL; gq[2] = q[2] * iL;
            if (want_h) {
                Hq[0] = (1.0 - gq[0] * gq[0]) * iL; Hq[1] = (1.0 - gq[1] * gq[1]) * iL;
                Hq[2] = (1.0 - gq[2] * gq[2]) * iL; Hq[3] = -gq[0] * gq[1] * iL;
                Hq[4] = -gq[0] * gq[2] * iL; Hq[5] = -gq[1] * gq[2] * iL;
            }
        } else {
            gq[2] = 1.0;
        }
        break;
    }
    case 1: {
        const double a = ind.shape[0], hh = 0.5 * ind.shape[1];
        const double rho = sqrt(q[0] * q[0] + q[1] * q[1]);
        const double ex = rho > 0.0 ? q[0] / rho : 1.0, ey = rho > 0.0 ? q[1] / rho : 0.0;
        const double sz = q[2] >= 0.0 ? 1.0 : -1.0;
        const double dr = rho - a, dz = fabs(q[2]) - hh;
        if (dr > 0.0 && dz > 0.0) {
            phi = sqrt(dr * dr + dz * dz);
            gq[0] = ex * dr / phi; gq[1] = ey * dr / phi; gq[2] = sz * dz / phi;
        } else if (dr > 0.0 || (dz <= 0.0 && dr >= dz)) {
            phi = dr;
            gq[0] = ex; gq[1] = ey;
            if (want_h && phi < 0.0 && rho > 0.0) {
                const double tx = -ey, ty = ex, ir = 1.0 / rho;
                Hq[0] = tx * tx * ir; Hq[1] = ty * ty * ir; Hq[3] = tx * ty * ir;
            }
        } else {
            phi = dz;
            gq[2] = sz;
        }
        break;
    }
    case 2: {
        double o2 = 0.0, dd[3];
        bool outside = false;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            dd[i] = fabs(q[i]) - ind.shape[i];
            if (dd[i] > 0.0) { outside = true; o2 += dd[i] * dd[i]; }
        }
        if (outside) {
            phi = sqrt(o2);
#pragma unroll
            for (int i = 0; i < 3; i++) gq[i] = dd[i] > 0.0 ? (q[i] >= 0.0 ? dd[i] : -dd[i]) / phi : 0.0;
        } else {
            int j = 0;
            if (dd[1] > dd[j]) j = 1;
            if (dd[2] > dd[j]) j = 2;
            phi = dd[j];
            gq[j] = q[j] >= 0.0 ? 1.0 : -1.0;
        }
        break;
    }
    default: {
        const double Rm = ind.shape[0], rm = ind.shape[1];
        const double rho = sqrt(q[0] * q[0] + q[1] * q[1]);
        const double ex = rho > 0.0 ? q[0] / rho : 1.0, ey = rho > 0.0 ? q[1] / rho : 0.0;
        const double wr = rho - Rm, wz = q[2];
        const double L = sqrt(wr * wr + wz * wz);
        phi = L - rm;
        if (L > 0.0) {
            const double cr = wr / L, cz = wz / L;
            gq[0] = cr * ex; gq[1] = cr * ey; gq[2] = cz;
            if (want_h && rho > 0.0) {
                // meridian tangent (curvature 1/L) and hoop direction (cr / rho)
                const double tx = -cz * ex, ty = -cz * ey, tz = cr;
                const double iL = 1.0 / L, kh = cr / rho;
                Hq[0] = tx * tx * iL + ey * ey * kh; Hq[1] = ty * ty * iL + ex * ex * kh;
                Hq[2] = tz * tz * iL; Hq[3] = tx * ty * iL - ex * ey * kh;
                Hq[4] = tx * tz * iL; Hq[5] = ty * tz * iL;
            }
        } else {
            gq[2] = 1.0;
        }
        break;
    }
    }
#pragma unroll
    for (int i = 0; i < 3; i++) n[i] = R[3 * i] * gq[0] + R[3 * i + 1] * gq[1] + R[3 * i + 2] * gq[2];
    if (want_h) {
        const double Hf[9] = {Hq[0], Hq[3], Hq[4], Hq[3], Hq[1], Hq[5], Hq[4], Hq[5], Hq[2]};
        double RH[9], W[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) RH[3 * i + j] = R[3 * i] * Hf[j] + R[3 * i + 1] * Hf[3 + j] + R[3 * i + 2] * Hf[6 + j];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) W[3 * i + j] = RH[3 * i] * R[3 * j] + RH[3 * i + 1] * R[3 * j + 1] + RH[3 * i + 2] * R[3 * j + 2];
        Hw[0] = W[0]; Hw[1] = W[4]; Hw[2] = W[8]; Hw[3] = W[1]; Hw[4] = W[2]; Hw[5] = W[5];
    }
}

// ---------------------------------------------------------------------------
// End of a load step (called by the finalising thread): bookkeeping, then the
// next load step's pose c = c0 + depth * step / steps * dir, or done.
// ---------------------------------------------------------------------------
__device__ inline void end_step(InstState *s, signed char *hist, int status) {
    s->last_status = status;
    if (s->step >= 1 && s->step <= kHistSteps) hist[s->step - 1] = (signed char)status;
    s->st_g = sqrt(s->gg);
    s->tot_newton += s->st_newton;
    s->tot_cg += s->st_cg;
    s->tot_hv += s->st_hv;
    s->tot_grad += s->st_grad;
    s->tot_ls += s->st_ls;
    if (status >= ST_OK) {
        s->steps_ok++;
        if (status == ST_FLOOR) s->steps_floor++;
    } else {
        s->steps_failed++;
        if (s->first_fail == 0) s->first_fail = status;
    }
    // the state just reached is the next step's friction lag state
    for (int d = 0; d < 3; d++) s->c_lag[d] = s->ind.c[d];
    s->lag_ok = 1;
    if (s->step >= s->steps) {
        s->phase = PH_DONE;
        return;
    }
    s->step++;
    const double f = s->depth * (double)s->step / (double)s->steps;
    for (int d = 0; d < 3; d++) s->ind.c[d] = s->c0[d] + f * s->dir[d];
    s->phase = s->mu_f > 0.0 ? PH_LAG : PH_GRAD;
    s->after_lag = PH_GRAD;
    s->step_started = 1;
    s->newton_it = 0;
    s->st_newton = s->st_cg = s->st_hv = s->st_grad = s->st_ls = 0;
}

// Block-level partial sums of a work kernel: thread 0 stores them.
template <int NS>
__device__ __forceinline__ void store_partials(double *red, int stride, const int (&streams)[NS], int slot,
                                               double (&v)[NS]) {
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NS; i++) red[streams[i] * stride + slot] = v[i];
}

// LDS of a tile block, shared by the two tile paths (doubles): the element
// path keeps 9 FP64 accumulators and one staged vector per entry, the
// Hessian path 3 accumulators and two staged vectors.
// In the deterministic mode (DET) the accumulators are replaced by a buffer of
// one chunk of tets' contributions in the path precision: 9 values per node
// and tet (element path, chunks of kDetElemChunk tets) or 3 (Hessian path,
// chunks of kBlock tets).
template <typename T, bool DET = false>
struct TileLds {
    static constexpr int kVec = kSw * kTileNodes * (int)sizeof(T) / 8;
    static constexpr int kElem = DET ? kVec + kDetElemChunk * 36 * (int)sizeof(T) / 8 : 9 * kTileNodes + kVec;
    static constexpr int kHv = DET ? 2 * kVec + kBlock * 12 * (int)sizeof(T) / 8 : 3 * kTileNodes + 2 * kVec;
    static constexpr int kDoubles = kElem > kHv ? kElem : kHv;
};

// ---------------------------------------------------------------------------
// Lagged, smoothed Coulomb friction at one contact node, in FP64. The lag
// data fr: w = mu_f k (-phi) and the unit normal n at the lag state, then the
// node's displacement relative to the indenter since the lag state, dd: it
// starts at minus the indenter's translation and accumulates the applied
// Newton increments in FP64 (so the slip keeps full precision on the FP32
// path, where it would otherwise be a difference of two rounded positions).
// With the tangential slip s = (I - n n^T) dd and y = |s|: energy
// w f0(y), f0 = y^2/eps - y^3/(3 eps^2) + eps/3 below y = eps and y above
// (C1), gradient w (f1/y) s, and the node block
// w [(f1/y)(I - n n^T) + (f1' - f1/y)/y^2 s s^T] (xx yy zz xy xz yz), which
// is positive semidefinite; f1 = f0'.
// ---------------------------------------------------------------------------
__device__ inline double friction_eval(const double fr[8], const double dd[3], double eps, double g[3], double H[6]) {
    const double w = fr[0];
    const double nl[3] = {fr[1], fr[2], fr[3]};
    const double dn = dd[0] * nl[0] + dd[1] * nl[1] + dd[2] * nl[2];
    double sv[3];
#pragma unroll
    for (int d = 0; d < 3; d++) sv[d] = dd[d] - dn * nl[d];
    const double y = sqrt(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2]);
    double f0, a, b;
    if (y < eps) {
        const double ie = 1.0 / eps;
        f0 = y * y * ie - y * y * y * ie * ie * (1.0 / 3.0) + eps * (1.0 / 3.0);
        a = 2.0 * ie - y * ie * ie;              // f1 / y
        b = y > 0.0 ? -ie * ie / y : 0.0;         // (f1' - f1 / y) / y^2
    } else {
        f0 = y;
        a = 1.0 / y;
        b = -a * a * a;
    }
#pragma unroll
    for (int d = 0; d < 3; d++) g[d] = w * a * sv[d];
    H[0] = w * (a * (1.0 - nl[0] * nl[0]) + b * sv[0] * sv[0]);
    H[1] = w * (a * (1.0 - nl[1] * nl[1]) + b * sv[1] * sv[1]);
    H[2] = w * (a * (1.0 - nl[2] * nl[2]) + b * sv[2] * sv[2]);
    H[3] = w * (-a * nl[0] * nl[1] + b * sv[0] * sv[1]);
    H[4] = w * (-a * nl[0] * nl[2] + b * sv[0] * sv[2]);
    H[5] = w * (-a * nl[1] * nl[2] + b * sv[1] * sv[2]);
    return w * f0;
}

// Friction lag data of one contact node at the start of a load step (node
// pass, phase PH_LAG): the penetration and normal at the current
// displacement u (the previous step's result) against the indenter at its
// previous centre c_lag; the relative displacement starts at minus the
// indenter's translation since, c_lag - c.
__device__ inline void friction_lag(const InstState *s, const double x[3], double fr[8]) {
#pragma unroll
    for (int c = 0; c < 8; c++) fr[c] = 0.0;
    if (s->lag_ok) {
        Indenter il = s->ind;
#pragma unroll
        for (int d = 0; d < 3; d++) il.c[d] = s->c_lag[d];
        double phl, nl[3], Hn[6];
        sdf_eval(il, x, false, phl, nl, Hn);
        if (phl < 0.0) {
            fr[0] = s->mu_f * s->ind.k * (-phl);
#pragma unroll
            for (int d = 0; d < 3; d++) fr[1 + d] = nl[d];
        }
    }
#pragma unroll
    for (int d = 0; d < 3; d++) fr[4 + d] = s->c_lag[d] - s->ind.c[d];
}

// Relative displacement of a contact node for friction, with a trial
// increment.
__device__ inline void friction_rel(const double fr[8], const double inc[3], double dd[3]) {
#pragma unroll
    for (int d = 0; d < 3; d++) dd[d] = fr[4 + d] + inc[d];
}

// ---------------------------------------------------------------------------
// Element + contact pass of one tile block (phases GRAD, EVAL_GRAD, TRIAL at
// u + alpha dx). Tile blocks: energy, magnitude, min J, and per entry
// partials of the gradient and of the 3x3 node diagonal blocks
// V (mu |b|^2 I + (mu + lam - lam ln J) c c^T), c = F^-T b. Contact blocks:
// penalty energy, gradient k phi n and block k n n^T (+ k phi Hess(phi) with
// the exact contact Hessian) per eligible node.
// ---------------------------------------------------------------------------
template <typename T, int LAW, bool DET>
__device__ __forceinline__ void tile_element(const TopoD<T> &tp, const BufsD<T> &B, const InstState *s, int blk,
                                             T alpha, int contact_full, double *pool) {
    const T mu = (T)s->mu, lam = (T)s->lam;
    double acc[3] = {0.0, 0.0, INFINITY};   // energy, magnitude, min J
    if (blk < tp.ntile) {
        double *sa = pool;                                    // 9 per entry, FP64 in both precisions
        T *su = (T *)(pool + (DET ? 0 : 9 * kTileNodes));     // kSw per entry
        T *cf = su + kSw * kTileNodes;                        // DET: 36 per tet of a chunk
        const int t = blk;
        const int e0 = tp.tile_ent[t], ne = tp.tile_ent[t + 1] - e0;
        const int k0 = tp.tile_tet[t], nk = tp.tile_tet[t + 1] - k0;
        // This thread's first tet record is fetched before the staging
        // barrier, so its latency overlaps the staging loads.
        TetWords<T> tw;
        if ((int)threadIdx.x < nk) fetch_tet(tp, k0 + (int)threadIdx.x, tw);
        // entry threadIdx.x (ne <= kTileNodes <= kBlock), staged at its slot
        const int sl = (int)threadIdx.x < ne ? tp.ent_slot[e0 + threadIdx.x] : 0;
        if ((int)threadIdx.x < ne) {
            const int gid = tp.ent_node[e0 + threadIdx.x];
#pragma unroll
            for (int d = 0; d < 3; d++) {
                T uu = B.u[3 * gid + d];
                if (alpha != (T)0) uu = fma_t(alpha, B.dx[3 * gid + d], uu);
                su[kSw * sl + d] = uu;
            }
            su[kSw * sl + 3] = (T)0;
            if (!DET)
#pragma unroll
                for (int c = 0; c < 9; c++) sa[9 * sl + c] = 0.0;
        }
        __syncthreads();
        // One tet: its energy into acc, and per node a the gradient (c = 0..2)
        // and diagonal block (c = 3..8) contributions to put(l, a, c, value).
        auto tet = [&](int k, auto &&put) {
            int l[4];
            if (k != (int)threadIdx.x) fetch_tet(tp, k0 + k, tw);
            const ElemGeo<T> geo = unpack_tet(tw, l);
            T wu[4][3];
            load_nodes(su, l, wu);
            T G[9];
            edge_gradient(wu, geo.Bm, G);
            const T Jm1 = det_minus_one(G);
            const T J = (T)1 + Jm1;
            acc[2] = fmin(acc[2], (double)J);
            if (!(J > (T)0)) {
                acc[0] = INFINITY;
                return;
            }
            T psi, mag, Pk[9], FiT[9], kI, kc;   // FiT: the block's c = Mb b
            Law<T, LAW>::element(G, Jm1, J, mu, lam, psi, mag, Pk, FiT, kI, kc);
            acc[0] += (double)(geo.V * psi);
            acc[1] += (double)(geo.V * mag);
            T f[4][3];
            element_nodal(Pk, geo.Bm, geo.V, f);
#pragma unroll
            for (int a = 0; a < 4; a++) {
                put(l, a, 0, f[a][0]);
                put(l, a, 1, f[a][1]);
                put(l, a, 2, f[a][2]);
                T bb[3];
                if (a == 0) {
                    bb[0] = -(geo.Bm[0] + geo.Bm[3] + geo.Bm[6]);
                    bb[1] = -(geo.Bm[1] + geo.Bm[4] + geo.Bm[7]);
                    bb[2] = -(geo.Bm[2] + geo.Bm[5] + geo.Bm[8]);
                } else {
                    bb[0] = geo.Bm[3 * (a - 1)];
                    bb[1] = geo.Bm[3 * (a - 1) + 1];
                    bb[2] = geo.Bm[3 * (a - 1) + 2];
                }
                const T cx = FiT[0] * bb[0] + FiT[1] * bb[1] + FiT[2] * bb[2];
                const T cy = FiT[3] * bb[0] + FiT[4] * bb[1] + FiT[5] * bb[2];
                const T cz = FiT[6] * bb[0] + FiT[7] * bb[1] + FiT[8] * bb[2];
                const T sI = geo.V * kI * (bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2]);
                const T Vk = geo.V * kc;
                put(l, a, 3, sI + Vk * cx * cx);
                put(l, a, 4, sI + Vk * cy * cy);
                put(l, a, 5, sI + Vk * cz * cz);
                put(l, a, 6, Vk * cx * cy);
                put(l, a, 7, Vk * cx * cz);
                put(l, a, 8, Vk * cy * cz);
            }
        };
        if constexpr (!DET) {
            for (int k = threadIdx.x; k < nk; k += kBlock)
                tet(k, [&](const int *l, int a, int c, T v) { atomicAdd(sa + 9 * l[a] + c, (double)v); });
            __syncthreads();
            if ((int)threadIdx.x < ne)
#pragma unroll
                for (int c = 0; c < 9; c++) B.pg[9 * (e0 + threadIdx.x) + c] = (T)sa[9 * sl + c];
        } else {
            // Deterministic: a chunk of tets stores its contributions, then
            // each entry sums its incident ones in ascending tet order.
            double ga[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            const bool mine = (int)threadIdx.x < ne;
            int ip = mine ? tp.inc_off[e0 + threadIdx.x] : 0;
            const int ie = mine ? tp.inc_off[e0 + threadIdx.x + 1] : 0;
            for (int c0 = 0; c0 < nk; c0 += kDetElemChunk) {
                const int k = c0 + (int)threadIdx.x;
                if ((int)threadIdx.x < kDetElemChunk && k < nk) {
                    T *dst = cf + 36 * threadIdx.x;
#pragma unroll
                    for (int q = 0; q < 36; q++) dst[q] = (T)0;
                    tet(k, [&](const int *, int a, int c, T v) { dst[9 * a + c] = v; });
                }
                __syncthreads();
                for (; ip < ie; ip++) {
                    const int code = tp.inc[ip];
                    if ((code >> 2) >= c0 + kDetElemChunk) break;
                    const T *src = cf + 36 * ((code >> 2) - c0) + 9 * (code & 3);
#pragma unroll
                    for (int c = 0; c < 9; c++) ga[c] += (double)src[c];
                }
                __syncthreads();
            }
            if (mine)
#pragma unroll
                for (int c = 0; c < 9; c++) B.pg[9 * (e0 + threadIdx.x) + c] = (T)ga[c];
        }
    } else {
        const int j = (blk - tp.ntile) * kBlock + threadIdx.x;
        if (j < tp.nc) {
            const int i = tp.cnodes[j];
            double x[3];
#pragma unroll
            for (int d = 0; d < 3; d++) {
                T ui = B.u[3 * i + d];
                if (alpha != (T)0) ui = fma_t(alpha, B.dx[3 * i + d], ui);
                x[d] = tp.X[3 * i + d] + (double)ui;
            }
            double phi, nv[3], Hs[6];
            sdf_eval(s->ind, x, contact_full != 0, phi, nv, Hs);
            double od[9];
#pragma unroll
            for (int c = 0; c < 9; c++) od[c] = 0.0;
            if (phi < 0.0) {
                const double kp = s->ind.k;
                const double ec = 0.5 * kp * phi * phi;
                acc[0] += ec;
                acc[1] += ec;
#pragma unroll
                for (int d = 0; d < 3; d++) od[d] = kp * phi * nv[d];
                const double nn[6] = {nv[0] * nv[0], nv[1] * nv[1], nv[2] * nv[2], nv[0] * nv[1], nv[0] * nv[2], nv[1] * nv[2]};
#pragma unroll
                for (int c = 0; c < 6; c++) od[3 + c] = kp * (nn[c] + (contact_full ? phi * Hs[c] : 0.0));
            }
            if (s->mu_f > 0.0) {
                double fl[8];
#pragma unroll
                for (int c = 0; c < 8; c++) fl[c] = B.fr[8 * j + c];
                if (fl[0] > 0.0) {
                    double inc[3], dd[3], gf[3], Hf[6];
#pragma unroll
                    for (int d = 0; d < 3; d++)
                        inc[d] = alpha != (T)0 ? (double)alpha * (double)B.dx[3 * i + d] : 0.0;
                    friction_rel(fl, inc, dd);
                    const double ef = friction_eval(fl, dd, s->eps_f, gf, Hf);
                    acc[0] += ef;
                    acc[1] += ef;
#pragma unroll
                    for (int d = 0; d < 3; d++) od[d] += gf[d];
#pragma unroll
                    for (int c = 0; c < 6; c++) od[3 + c] += Hf[c];
                }
            }
            // the Hessian-vector passes read a node's contact block only
            // where it is nonzero (most eligible nodes are out of contact)
            bool act = false;
#pragma unroll
            for (int c = 0; c < 9; c++) {
                B.cp[9 * j + c] = (T)od[c];
                if (c >= 3) act = act || (T)od[c] != (T)0;
            }
            B.cact[j] = act ? 1 : 0;
        }
    }
    double sums[2] = {acc[0], acc[1]};
    double mn = acc[2];
    block_reduce<2, true>(sums, mn);
    double v[3] = {sums[0], sums[1], mn};
    const int streams[3] = {RS_E, RS_MAG, RS_MINJ};
    store_partials<3>(B.red, B.red_stride, streams, blk, v);
}

// ---------------------------------------------------------------------------
// Hessian-vector product of one tile block (phases CG, EVAL_HV): q = H p with
// p = z + beta p_prev formed while staging (the node pass forms the same
// value). Per tet, with F recomputed from the staged u:
//   dP = mu dG + (mu - lam ln J) (F^-1 dG F^-1)^T + lam tr(F^-1 dG) F^-T.
// p.q is accumulated element by element (and over contact blocks), so alpha
// is known to the node pass without a pass over q.
// ---------------------------------------------------------------------------
template <typename T, int LAW, bool DET>
__device__ __forceinline__ void tile_hessvec(const TopoD<T> &tp, const BufsD<T> &B, const InstState *s, int blk,
                                             double *pool) {
    const T beta = (T)s->beta;
    const T mu = (T)s->mu, lam = (T)s->lam;
    double acc[1] = {0.0};
    double unused = 0.0;
    if (blk < tp.ntile) {
        double *sa = pool;                                    // 3 per entry, FP64 in both precisions
        T *su = (T *)(pool + (DET ? 0 : 3 * kTileNodes));     // kSw per entry
        T *sp = su + kSw * kTileNodes;                        // kSw per entry
        T *cf = sp + kSw * kTileNodes;                        // DET: 12 per tet of a chunk
        const int t = blk;
        const int e0 = tp.tile_ent[t], ne = tp.tile_ent[t + 1] - e0;
        const int k0 = tp.tile_tet[t], nk = tp.tile_tet[t + 1] - k0;
        // Implicit steps add (m_i / dt^2) |p_i|^2 to p.q, taken once per node
        // (on its first entry).
        const double cm = s->mdt2;
        double pq = 0.0;
        // This thread's first tet record is fetched before the staging
        // barrier, so its latency overlaps the staging loads.
        TetWords<T> tw;
        if ((int)threadIdx.x < nk) fetch_tet(tp, k0 + (int)threadIdx.x, tw);
        // entry threadIdx.x (ne <= kTileNodes <= kBlock), staged at its slot
        const int sl = (int)threadIdx.x < ne ? tp.ent_slot[e0 + threadIdx.x] : 0;
        if ((int)threadIdx.x < ne) {
            const int gid = tp.ent_node[e0 + threadIdx.x];
            T pv[3];
#pragma unroll
            for (int d = 0; d < 3; d++) {
                su[kSw * sl + d] = B.u[3 * gid + d];
                pv[d] = fma_t(beta, B.p[3 * gid + d], B.z[3 * gid + d]);
                sp[kSw * sl + d] = pv[d];
                if (!DET) sa[3 * sl + d] = 0.0;
            }
            su[kSw * sl + 3] = (T)0;
            sp[kSw * sl + 3] = (T)0;
            if (cm > 0.0 && tp.owner[e0 + threadIdx.x])
                pq += cm * (double)tp.nvol[gid] *
                      ((double)pv[0] * (double)pv[0] + (double)pv[1] * (double)pv[1] + (double)pv[2] * (double)pv[2]);
        }
        __syncthreads();
        // One tet: its p.q into pq and its nodal vectors to put(l, a, d, value).
        auto tet = [&](int k, auto &&put) {
            int l[4];
            if (k != (int)threadIdx.x) fetch_tet(tp, k0 + k, tw);
            const ElemGeo<T> geo = unpack_tet(tw, l);
            T wu[4][3], wp[4][3];
            load_nodes(su, l, wu);
            load_nodes(sp, l, wp);
            T G[9];
            edge_gradient(wu, geo.Bm, G);
            const T Jm1 = det_minus_one(G);
            const T J = (T)1 + Jm1;
            if (!(J > (T)0)) return;
            T dG[9];
            edge_gradient(wp, geo.Bm, dG);
            T dP[9];
            Law<T, LAW>::hessvec(G, Jm1, J, dG, mu, lam, dP);
            T f[4][3];
            element_nodal(dP, geo.Bm, geo.V, f);
            T e_pq = (T)0;
#pragma unroll
            for (int a = 0; a < 4; a++) {
                put(l, a, 0, f[a][0]);
                put(l, a, 1, f[a][1]);
                put(l, a, 2, f[a][2]);
                e_pq += wp[a][0] * f[a][0] + wp[a][1] * f[a][1] + wp[a][2] * f[a][2];
            }
            pq += (double)e_pq;
        };
        if constexpr (!DET) {
            for (int k = threadIdx.x; k < nk; k += kBlock)
                tet(k, [&](const int *l, int a, int d, T v) { atomicAdd(sa + 3 * l[a] + d, (double)v); });
            acc[0] = pq;
            __syncthreads();
            if ((int)threadIdx.x < ne)
#pragma unroll
                for (int d = 0; d < 3; d++) B.pq[3 * (e0 + threadIdx.x) + d] = (T)sa[3 * sl + d];
        } else {
            // Deterministic: each chunk of kBlock tets stores its nodal
            // vectors, then each entry sums its incident ones in ascending
            // tet order.
            double qa[3] = {0.0, 0.0, 0.0};
            const bool mine = (int)threadIdx.x < ne;
            int ip = mine ? tp.inc_off[e0 + threadIdx.x] : 0;
            const int ie = mine ? tp.inc_off[e0 + threadIdx.x + 1] : 0;
            for (int c0 = 0; c0 < nk; c0 += kBlock) {
                const int k = c0 + (int)threadIdx.x;
                if (k < nk) {
                    T *dst = cf + 12 * threadIdx.x;
#pragma unroll
                    for (int q = 0; q < 12; q++) dst[q] = (T)0;
                    tet(k, [&](const int *, int a, int d, T v) { dst[3 * a + d] = v; });
                }
                __syncthreads();
                for (; ip < ie; ip++) {
                    const int code = tp.inc[ip];
                    if ((code >> 2) >= c0 + kBlock) break;
                    const T *src = cf + 12 * ((code >> 2) - c0) + 3 * (code & 3);
#pragma unroll
                    for (int d = 0; d < 3; d++) qa[d] += (double)src[d];
                }
                __syncthreads();
            }
            acc[0] = pq;
            if (mine)
#pragma unroll
                for (int d = 0; d < 3; d++) B.pq[3 * (e0 + threadIdx.x) + d] = (T)qa[d];
        }
    } else {
        const int j = (blk - tp.ntile) * kBlock + threadIdx.x;
        if (j < tp.nc && B.cact[j]) {
            const T *H = B.cp + 9 * j + 3;
            const int i = tp.cnodes[j];
            T pv[3];
#pragma unroll
            for (int d = 0; d < 3; d++) pv[d] = fma_t(beta, B.p[3 * i + d], B.z[3 * i + d]);
            const T q0 = H[0] * pv[0] + H[3] * pv[1] + H[4] * pv[2];
            const T q1 = H[3] * pv[0] + H[1] * pv[1] + H[5] * pv[2];
            const T q2 = H[4] * pv[0] + H[5] * pv[1] + H[2] * pv[2];
            acc[0] = (double)(pv[0] * q0 + pv[1] * q1 + pv[2] * q2);
        }
    }
    block_reduce<1, false>(acc, unused);
    const int streams[1] = {RS_PQ};
    store_partials<1>(B.red, B.red_stride, streams, blk, acc);
}

// ---------------------------------------------------------------------------
// Tile pass: one block per (instance, tile or contact block). Each instance's
// blocks take the Hessian-vector path while it is in CG (or EVAL_HV), the
// element path in GRAD, EVAL_GRAD and TRIAL, and return otherwise. The two
// paths share one LDS pool (their register needs are alike, so the union
// does not lower occupancy).
// ---------------------------------------------------------------------------
template <typename T, int LAW, bool DET>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 1 : 3))) void k_tile(const Topo<T> *topos, const InstBufs<T> *bufs, const int2 *work,
                                                 int nwork, const SolveParams *P) {
    __shared__ __attribute__((aligned(32))) double pool[TileLds<T, DET>::kDoubles];
    const int L = logical_block();
    if (L >= nwork) return;
    const int2 w = work[L];
    // Descriptors copied up front, before any store of the kernel, so they
    // are fetched once as uniform (scalar) loads.
    const BufsD<T> B = dev_view(bufs[w.x]);
    const TopoD<T> tp = dev_view(topos[B.topo]);
    const int contact_full = P->contact_full;
    const InstState *s = B.s;
    const int phase = s->phase;
    if (s->model != LAW) return;   // served by the other law's launch
    if (phase == PH_CG || phase == PH_EVAL_HV) {
        tile_hessvec<T, LAW, DET>(tp, B, s, w.y, pool);
    } else if (phase == PH_GRAD || phase == PH_EVAL_GRAD || phase == PH_TRIAL) {
        const T alpha = phase == PH_TRIAL ? (T)s->alpha_ls : (T)0;
        tile_element<T, LAW, DET>(tp, B, s, w.y, alpha, contact_full, pool);
    }
}

// ---------------------------------------------------------------------------
// Newton init of one node block (phases GRAD, EVAL_GRAD after the element
// path of the same pass; INIT after an accepted line-search trial). Applies
// an accepted step u += alpha dx, gathers g and the node block from the tile
// and contact partials, forms the block (or scalar) Jacobi inverse, r = -g and
// z = M^-1 r on free nodes; partial sums of |g_free|^2 and r.z.
// Implicit steps (dt > 0): at the start of a time step (step_start) the
// velocity of the step just completed, v += (u - ut) / dt, and the new
// predictor ut = u + dt v are formed first; every init then adds the inertial
// gradient (m/dt^2)(u - ut), (m/dt^2) I to the node block, and the inertial
// energy (m/2dt^2)|u - ut|^2 to its own partial sum.
// ---------------------------------------------------------------------------
template <typename T, bool FRIC>
__device__ __forceinline__ void node_init(const TopoD<T> &tp, const BufsD<T> &B, const InstState *s, int blk,
                                          bool apply, bool step_start, int block_jacobi) {
    const T alpha = (T)s->alpha_ls;
    const double dt = s->dt, mdt2 = s->mdt2;
    const bool dyn = dt > 0.0;
    double acc[3] = {0.0, 0.0, 0.0};   // |g_free|^2, r.z, inertial energy
    double unused = 0.0;
    const int i = blk * kBlock + threadIdx.x;
    if (i < tp.n) {
        if (apply) {
#pragma unroll
            for (int d = 0; d < 3; d++) B.u[3 * i + d] = fma_t(alpha, B.dx[3 * i + d], B.u[3 * i + d]);
            // contact nodes with friction also accumulate the increment in FP64
            if (FRIC && s->mu_f > 0.0) {
                const int jc = tp.cidx[i];
                if (jc >= 0)
#pragma unroll
                    for (int d = 0; d < 3; d++) B.fr[8 * jc + 4 + d] += (double)alpha * (double)B.dx[3 * i + d];
            }
        }
        T gsum[9];
#pragma unroll
        for (int c = 0; c < 9; c++) gsum[c] = (T)0;
        for (int q = tp.node_ent_off[i]; q < tp.node_ent_off[i + 1]; q++) {
            const T *src = B.pg + 9 * tp.node_ent[q];
#pragma unroll
            for (int c = 0; c < 9; c++) gsum[c] += src[c];
        }
        const int j = tp.cidx[i];
        if (j >= 0)
#pragma unroll
            for (int c = 0; c < 9; c++) gsum[c] += B.cp[9 * j + c];
        if (dyn && !tp.fixed[i]) {
            const T h = (T)dt;
            const T cm = (T)mdt2 * tp.nvol[i];
            double en = 0.0;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                const T ui = B.u[3 * i + d];
                T ti = B.ut[3 * i + d];
                if (step_start) {
                    const T vv = B.v[3 * i + d] + (ui - ti) / h;
                    B.v[3 * i + d] = vv;
                    ti = fma_t(h, vv, ui);
                    B.ut[3 * i + d] = ti;
                }
                const T w = ui - ti;
                gsum[d] = fma_t(cm, w, gsum[d]);
                en += (double)w * (double)w;
            }
            acc[2] = 0.5 * (double)cm * en;
            gsum[3] += cm;
            gsum[4] += cm;
            gsum[5] += cm;
        }
#pragma unroll
        for (int d = 0; d < 3; d++) B.g[3 * i + d] = gsum[d];
        T M[6] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
        T rr[3] = {(T)0, (T)0, (T)0}, zz[3] = {(T)0, (T)0, (T)0};
        if (!tp.fixed[i]) {
            const T a = gsum[3], bb = gsum[4], c = gsum[5], d = gsum[6], e = gsum[7], f = gsum[8];
            const T m2 = a * bb - d * d;
            const T c00 = bb * c - f * f, c01 = e * f - d * c, c02 = d * f - bb * e;
            const T det = a * c00 + d * c01 + e * c02;
            if (block_jacobi && a > (T)0 && m2 > (T)0 && det > (T)0) {
                const T id = (T)1 / det;
                M[0] = c00 * id;
                M[1] = (a * c - e * e) * id;
                M[2] = m2 * id;
                M[3] = c01 * id;
                M[4] = c02 * id;
                M[5] = (d * e - a * f) * id;
            } else {
                M[0] = safe_recip(a);
                M[1] = safe_recip(bb);
                M[2] = safe_recip(c);
            }
#pragma unroll
            for (int d2 = 0; d2 < 3; d2++) rr[d2] = -gsum[d2];
            zz[0] = M[0] * rr[0] + M[3] * rr[1] + M[4] * rr[2];
            zz[1] = M[3] * rr[0] + M[1] * rr[1] + M[5] * rr[2];
            zz[2] = M[4] * rr[0] + M[5] * rr[1] + M[2] * rr[2];
#pragma unroll
            for (int d2 = 0; d2 < 3; d2++) {
                acc[0] += (double)rr[d2] * (double)rr[d2];
                acc[1] += (double)rr[d2] * (double)zz[d2];
            }
        }
#pragma unroll
        for (int c = 0; c < 6; c++) B.dinv[6 * i + c] = M[c];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            B.r[3 * i + d] = rr[d];
            B.z[3 * i + d] = zz[d];
            B.p[3 * i + d] = (T)0;
            B.dx[3 * i + d] = (T)0;
        }
    }
    block_reduce<3, false>(acc, unused);
    const int streams[3] = {RS_GG, RS_IRZ, RS_EN};
    store_partials<3>(B.red, B.red_stride, streams, blk, acc);
}

// ---------------------------------------------------------------------------
// CG update of one node block (phases CG, EVAL_HV). Every block sums the tile
// pass's p.q partials (fixed order, so all blocks agree; block 0 records the
// sum for the finalize) and forms
// alpha = r.z / p.q; then it gathers q from the tile partials plus the contact
// block times p (read only where the element pass flagged the block nonzero)
// and, on free nodes, sets p = z + beta p_prev, dx += alpha p,
// r -= alpha q, z = M^-1 r, with partial sums of r.z and r.r. At p.q <= 0 CG
// stops (on its first iteration the preconditioned residual becomes the
// Newton direction). EVAL_HV writes q instead.
// ---------------------------------------------------------------------------
template <typename T, bool DYN>
__device__ __forceinline__ void node_update(const TopoD<T> &tp, const BufsD<T> &B, const InstState *s, int blk,
                                            bool eval) {
    // solver scalars and this thread's node data first: their loads are in
    // flight while the block sums the p.q partials
    const double rz = s->rz;
    const T beta = (T)s->beta;
    const int cg_first = s->cg_it == 0;
    const int i = blk * kBlock + threadIdx.x;
    const bool live = i < tp.n;
    T pv[3] = {(T)0, (T)0, (T)0}, qv[3] = {(T)0, (T)0, (T)0}, rv[3] = {(T)0, (T)0, (T)0}, dxv[3] = {(T)0, (T)0, (T)0};
    T M[6] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
    bool fixed = true;
    if (live) {
        // every load that depends only on i is issued first (r, dx and the
        // block inverse after the fixed flag: fixed nodes are numbered last,
        // so the test is uniform across almost every wavefront)
        const int4 e4 = tp.node_ent4[i];
        const int j = tp.cidx[i];
        fixed = tp.fixed[i] != 0;
#pragma unroll
        for (int d = 0; d < 3; d++) pv[d] = fma_t(beta, B.p[3 * i + d], B.z[3 * i + d]);
        if (!eval && !fixed) {
#pragma unroll
            for (int d = 0; d < 3; d++) {
                rv[d] = B.r[3 * i + d];
                dxv[d] = B.dx[3 * i + d];
            }
#pragma unroll
            for (int c = 0; c < 6; c++) M[c] = B.dinv[6 * i + c];
        }
        // the node's tile partials, summed in entry order: the first kGather
        // entries come with the node (their loads are in flight together; an
        // absent entry, -1, reads entry 0 and is dropped), the rest from the
        // node -> entry lists (1.92 entries per node on the 50k fingertip)
        const int ent[kGather] = {e4.x, e4.y, e4.z, e4.w};
        T part[kGather][3];
#pragma unroll
        for (int k = 0; k < kGather; k++)
#pragma unroll
            for (int d = 0; d < 3; d++) {
                const T v = B.pq[3 * (ent[k] >= 0 ? ent[k] : 0) + d];
                part[k][d] = ent[k] >= 0 ? v : (T)0;
            }
#pragma unroll
        for (int k = 0; k < kGather; k++)
#pragma unroll
            for (int d = 0; d < 3; d++) qv[d] += part[k][d];
        if (e4.w >= 0)
            for (int q = tp.node_ent_off[i] + kGather; q < tp.node_ent_off[i + 1]; q++)
#pragma unroll
                for (int d = 0; d < 3; d++) qv[d] += B.pq[3 * tp.node_ent[q] + d];
        if (j >= 0 && B.cact[j]) {
            const T *H = B.cp + 9 * j + 3;
            qv[0] += H[0] * pv[0] + H[3] * pv[1] + H[4] * pv[2];
            qv[1] += H[3] * pv[0] + H[1] * pv[1] + H[5] * pv[2];
            qv[2] += H[4] * pv[0] + H[5] * pv[1] + H[2] * pv[2];
        }
        if (DYN && !fixed) {
            const T cm = (T)s->mdt2 * tp.nvol[i];
#pragma unroll
            for (int d = 0; d < 3; d++) qv[d] = fma_t(cm, pv[d], qv[d]);
        }
    }
    const double pq = wave_sum_partials(B.red + RS_PQ * B.red_stride, tp.ntile + tp.ncb);
    if (blk == 0 && threadIdx.x == 0) B.red[RS_PQN * B.red_stride] = pq;
    const bool negcurv = !(pq > 0.0);
    const T alpha = negcurv ? (T)0 : (T)(rz / pq);
    double acc[2] = {0.0, 0.0};   // r.z, r.r
    if (live) {
        if (eval) {
#pragma unroll
            for (int d = 0; d < 3; d++) B.qout[3 * i + d] = qv[d];
        } else if (!negcurv) {
            if (!fixed) {
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    B.p[3 * i + d] = pv[d];
                    B.dx[3 * i + d] = fma_t(alpha, pv[d], dxv[d]);
                    rv[d] = fma_t(-alpha, qv[d], rv[d]);
                    B.r[3 * i + d] = rv[d];
                }
                const T z0 = M[0] * rv[0] + M[3] * rv[1] + M[4] * rv[2];
                const T z1 = M[3] * rv[0] + M[1] * rv[1] + M[5] * rv[2];
                const T z2 = M[4] * rv[0] + M[5] * rv[1] + M[2] * rv[2];
                B.z[3 * i] = z0;
                B.z[3 * i + 1] = z1;
                B.z[3 * i + 2] = z2;
                acc[0] = (double)rv[0] * (double)z0 + (double)rv[1] * (double)z1 + (double)rv[2] * (double)z2;
                acc[1] = (double)rv[0] * (double)rv[0] + (double)rv[1] * (double)rv[1] + (double)rv[2] * (double)rv[2];
            }
        } else if (cg_first) {
#pragma unroll
            for (int d = 0; d < 3; d++) B.dx[3 * i + d] = pv[d];
        }
    }
    // per-wavefront partials (kWaves per block), summed by the finalize
    acc[0] = wave_sum(acc[0]);
    acc[1] = wave_sum(acc[1]);
    if ((threadIdx.x & 63) == 0) {
        const int slot = kWaves * blk + (int)(threadIdx.x >> 6);
        B.red[RS_RZ * B.red_stride + slot] = acc[0];
        B.red[RS_RR * B.red_stride + slot] = acc[1];
    }
}

// Line-search trial, node part: partial sums of g . dx (first trial of a
// line search) and, for implicit steps, of the inertial energy
// (m/2dt^2)|u + alpha dx - ut|^2 at the trial point.
template <typename T>
__device__ __forceinline__ void node_trial(const TopoD<T> &tp, const BufsD<T> &B, const InstState *s, int blk) {
    double acc[2] = {0.0, 0.0};
    double unused = 0.0;
    const int i = blk * kBlock + threadIdx.x;
    if (i < tp.n) {
        if (s->need_gd)
#pragma unroll
            for (int d = 0; d < 3; d++) acc[0] += (double)B.g[3 * i + d] * (double)B.dx[3 * i + d];
        if (s->dt > 0.0 && !tp.fixed[i]) {
            const T alpha = (T)s->alpha_ls;
            double en = 0.0;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                const T w = fma_t(alpha, B.dx[3 * i + d], B.u[3 * i + d]) - B.ut[3 * i + d];
                en += (double)w * (double)w;
            }
            acc[1] = 0.5 * s->mdt2 * (double)tp.nvol[i] * en;
        }
    }
    block_reduce<2, false>(acc, unused);
    const int streams[2] = {RS_GD, RS_EN};
    store_partials<2>(B.red, B.red_stride, streams, blk, acc);
}

// ---------------------------------------------------------------------------
// Node pass: one block per (instance, 256 nodes), after the tile pass of the
// same step. CG -> update; GRAD, EVAL_GRAD, INIT -> Newton init; TRIAL ->
// g . dx on the first trial of a line search and the inertial energy of
// implicit steps; other phases return.
// ---------------------------------------------------------------------------
// Friction lag data of the contact-eligible nodes of one node block.
template <typename T>
__device__ __forceinline__ void node_lag(const TopoD<T> &tp, const BufsD<T> &B, const InstState *s, int blk) {
    const int i = blk * kBlock + threadIdx.x;
    if (i >= tp.n) return;
    const int j = tp.cidx[i];
    if (j < 0) return;
    double x[3], fl[8];
#pragma unroll
    for (int d = 0; d < 3; d++) x[d] = tp.X[3 * i + d] + (double)B.u[3 * i + d];
    friction_lag(s, x, fl);
#pragma unroll
    for (int c = 0; c < 8; c++) B.fr[8 * j + c] = fl[c];
}

template <typename T, bool FRIC>
__global__ __launch_bounds__(kBlock) void k_node(const Topo<T> *topos, const InstBufs<T> *bufs, const int2 *work,
                                                 int nwork, const SolveParams *P) {
    const int L = logical_block();
    if (L >= nwork) return;
    const int2 w = work[L];
    // Descriptors copied up front, before any store of the kernel, so they
    // are fetched once as uniform (scalar) loads.
    const BufsD<T> B = dev_view(bufs[w.x]);
    const TopoD<T> tp = dev_view(topos[B.topo]);
    const InstState *s = B.s;
    const int phase = s->phase;
    if (phase == PH_CG || phase == PH_EVAL_HV) {
        // a CG update changes free nodes only: blocks of fixed nodes (numbered
        // last) have nothing to do; block 0 always runs (it records p.q)
        if (phase == PH_CG && w.y > 0 && w.y * kBlock >= tp.n_free) return;
        // the inertial term as a separate instance keeps it out of the
        // quasi-static CG update
        if (s->mdt2 > 0.0)
            node_update<T, true>(tp, B, s, w.y, phase == PH_EVAL_HV);
        else
            node_update<T, false>(tp, B, s, w.y, phase == PH_EVAL_HV);
    }
    else if (phase == PH_GRAD || phase == PH_EVAL_GRAD || phase == PH_INIT)
        node_init<T, FRIC>(tp, B, s, w.y, phase == PH_INIT && s->apply != 0, phase == PH_GRAD, P->block_jacobi);
    else if (phase == PH_TRIAL && (s->need_gd || s->dt > 0.0))
        node_trial(tp, B, s, w.y);
    else if (FRIC && phase == PH_LAG)
        node_lag(tp, B, s, w.y);
}

// Newton test on |g_free| against the load step's first residual, then CG
// set-up with the inexact-Newton tolerance (finalising thread). Rounding
// floor: once the residual sits below floor_rtol * r0 and two accepted steps
// in a row whose predicted energy change lies within rounding have not halved
// the smallest residual of the step, the working precision cannot take it
// lower and the step ends with ST_FLOOR.
template <class StatePtr, class HistPtr>   // global-address-space pointers on the device
__device__ inline void newton_test(StatePtr s, HistPtr hist, const SolveParams *P, double gg, double rz) {
    s->gg = gg;
    const double gn = sqrt(gg);
    if (s->step_started) {
        s->r0 = gn;
        s->st_g0 = gn;
        s->step_started = 0;
        s->gbest = gn;
        s->stall = 0;
    } else if (s->apply) {
        // At the rounding floor the search direction is noise: accepted steps
        // do not reduce the residual, and the energy change they predict,
        // g.dx, lies within the energy's rounding noise. A step that predicts
        // a resolvable decrease means the iteration is still limited by
        // nonlinearity (stick-slip transitions of friction, large
        // rotations), so it does not count.
        const bool at_noise = fabs(s->gd) <= P->noise_eps * s->emag;
        if (gn <= 0.5 * s->gbest || !at_noise) {
            s->stall = 0;
        } else {
            s->stall++;
        }
        s->gbest = fmin(s->gbest, gn);
    }
    if (s->apply) {
        s->newton_it++;
        s->st_newton++;
        s->apply = 0;
    }
    if (gn <= fmax(P->newton_rtol * s->r0, P->newton_atol)) {
        end_step(s, hist, ST_OK);
    } else if (s->stall >= 2 && gn <= P->floor_rtol * s->r0) {
        end_step(s, hist, ST_FLOOR);
    } else if (s->newton_it >= P->max_newton) {
        end_step(s, hist, ST_NOT_CONVERGED);
    } else {
        // inexact Newton: forcing term (|g| / |g_start|)^p, p = 1/2 by default
        // (superlinear of order 1 + p, without tight solves late in a step)
        const double rel = gn / s->r0;
        const double eta = fmin(P->cg_eta_max, fmax(P->cg_rtol, P->eta_power == 1.0 ? rel : pow(rel, P->eta_power)));
        s->tol2 = eta * eta * gg;
        s->rz = rz;
        s->rr = gg;
        s->beta = 0.0;
        s->alpha = 0.0;
        s->cg_it = 0;
        s->phase = PH_CG;
    }
}

// End of a CG solve: the first line-search trial at alpha = 1 follows, with
// g . dx taken by its node pass.
__device__ inline void start_line_search(InstState *s) {
    s->last_cg = s->cg_it;
    s->alpha_ls = 1.0;
    s->halvings = 0;
    s->need_gd = 1;
    s->phase = PH_TRIAL;
}

// ---------------------------------------------------------------------------
// Finalize: one wavefront per live instance sums, in a fixed order, the
// partials its blocks wrote in this step's tile and node passes and takes the
// state-machine transition.
//   CG         alpha, beta, r.z; CG stop (tolerance, iteration cap, p.q <= 0)
//              -> TRIAL at alpha = 1.
//   GRAD       energy of the load step's start, then the Newton test.
//   TRIAL      Armijo test with the rounding floor noise_eps * sum of
//              energy-term magnitudes: accept -> INIT, else halve alpha or
//              end the load step.
//   INIT       Newton test.
//   EVAL_GRAD, EVAL_HV -> IDLE.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_finalize(const Topo<T> *topos, const InstBufs<T> *bufs, const int *live,
                                                 int nlive, const SolveParams *P) {
    if ((int)blockIdx.x >= nlive) return;
    const BufsD<T> B = dev_view(bufs[live[blockIdx.x]]);
    const TopoD<T> tp = dev_view(topos[B.topo]);
    const auto s = B.s;   // global-address-space pointer on the device
    const int phase = s->phase;
    const int S = B.red_stride;
    const int nt = tp.ntile + tp.ncb, nn = (tp.n + kBlock - 1) / kBlock;
    if (phase == PH_LAG) {
        if (threadIdx.x == 0) s->phase = s->after_lag;
        return;
    }
    if (phase == PH_CG || phase == PH_EVAL_HV) {
        const double pq = B.red[RS_PQN * S];   // the node pass's sum, as it applied it
        // the node pass's per-wavefront partials of its blocks with free nodes
        const int ncg = tp.n_free > kBlock ? (tp.n_free + kBlock - 1) / kBlock : 1;
        const double rz = wave_sum_partials(B.red + RS_RZ * S, kWaves * ncg);
        const double rr = wave_sum_partials(B.red + RS_RR * S, kWaves * ncg);
        if (threadIdx.x != 0) return;
        s->pq = pq;
        if (phase == PH_EVAL_HV) {
            s->phase = PH_IDLE;
            return;
        }
        s->st_hv++;
        if (!(pq > 0.0)) {
            start_line_search(s);
            return;
        }
        s->alpha = s->rz / pq;
        s->cg_it++;
        s->st_cg++;
        s->beta = rz / s->rz;
        s->rz = rz;
        s->rr = rr;
        if (rr <= s->tol2 || s->cg_it >= P->max_cg) start_line_search(s);
    } else if (phase == PH_GRAD || phase == PH_EVAL_GRAD || phase == PH_TRIAL) {
        // tile partials, plus the nodes' inertial energy of implicit steps
        const double en = s->dt > 0.0 ? wave_sum_partials(B.red + RS_EN * S, nn) : 0.0;
        const double E = wave_sum_partials(B.red + RS_E * S, nt) + en;
        const double mag = wave_sum_partials(B.red + RS_MAG * S, nt) + en;
        const double mn = wave_min_partials(B.red + RS_MINJ * S, nt);
        double gg = 0.0, rz = 0.0, gd = 0.0;
        if (phase != PH_TRIAL) {
            gg = wave_sum_partials(B.red + RS_GG * S, nn);
            rz = wave_sum_partials(B.red + RS_IRZ * S, nn);
        } else if (s->need_gd) {
            gd = wave_sum_partials(B.red + RS_GD * S, nn);
        }
        if (threadIdx.x != 0) return;
        const double Et = mn > 0.0 ? E : INFINITY;
        s->st_grad++;
        if (phase != PH_TRIAL) {
            s->E = Et;
            s->emag = mag;
            s->minJ = mn;
            s->apply = 0;
            if (phase == PH_EVAL_GRAD) {
                s->gg = gg;
                s->phase = PH_IDLE;
            } else {
                newton_test(s, B.hist, P, gg, rz);
            }
            return;
        }
        if (s->need_gd) {
            s->gd = gd;
            s->need_gd = 0;
        }
        s->st_ls++;
        const double noise = P->noise_eps * s->emag;
        if (mn > 0.0 && Et <= s->E + P->c1 * s->alpha_ls * s->gd + noise) {
            s->E = Et;
            s->emag = mag;
            s->minJ = mn;
            s->apply = 1;
            s->phase = PH_INIT;
        } else if (s->halvings >= P->max_halvings) {
            end_step(s, B.hist, mn > 0.0 ? ST_NOT_CONVERGED : ST_INVERSION);
        } else {
            s->halvings++;
            s->alpha_ls *= 0.5;
        }
    } else if (phase == PH_INIT) {
        const double gg = wave_sum_partials(B.red + RS_GG * S, nn);
        const double rz = wave_sum_partials(B.red + RS_IRZ * S, nn);
        if (threadIdx.x != 0) return;
        newton_test(s, B.hist, P, gg, rz);
    }
}

// ---------------------------------------------------------------------------
// Contact patch of one instance at its current state: one block walks the
// eligible nodes in ascending order and compacts those that carry a contact
// force, phi < 0 or friction from the lag state (ordered scan): ids, forces
// on the skin -k min(0, phi) n minus the friction gradient, phi, count and
// FP64 resultant.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void k_contact_patch(const Topo<T> *topos, const InstBufs<T> *bufs, int inst,
                                                          int *ids, double *f, double *phi_out, int *count,
                                                          double *Ftot) {
    __shared__ int wave_cnt[16];
    __shared__ double wave_f[16][3];
    __shared__ int base_s;
    __shared__ double F_s[3];
    const BufsD<T> B = dev_view(bufs[inst]);
    const TopoD<T> tp = dev_view(topos[B.topo]);
    const Indenter ind = B.s->ind;
    const bool fric = B.s->mu_f > 0.0;
    const double eps_f = B.s->eps_f;
    if (threadIdx.x == 0) {
        base_s = 0;
        F_s[0] = F_s[1] = F_s[2] = 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int start = 0; start < tp.nc; start += 1024) {
        const int j = start + threadIdx.x;
        double phi = 0.0, nv[3] = {0.0, 0.0, 0.0}, Hs[6], gf[3] = {0.0, 0.0, 0.0};
        int i = -1;
        bool act = false;
        if (j < tp.nc) {
            i = tp.cnodes[j];
            double x[3];
#pragma unroll
            for (int d = 0; d < 3; d++) x[d] = tp.X[3 * i + d] + (double)B.u[3 * i + d];
            sdf_eval(ind, x, false, phi, nv, Hs);
            act = phi < 0.0;
            if (fric) {
                double fl[8], Hf[6], dd[3];
                const double zero[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 8; c++) fl[c] = B.fr[8 * j + c];
                if (fl[0] > 0.0) {
                    friction_rel(fl, zero, dd);
                    friction_eval(fl, dd, eps_f, gf, Hf);
                    act = true;
                }
            }
        }
        double fv[3];
#pragma unroll
        for (int d = 0; d < 3; d++) fv[d] = act ? (phi < 0.0 ? -ind.k * phi * nv[d] : 0.0) - gf[d] : 0.0;
        const unsigned long long mask = __ballot(act);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        double sf[3];
#pragma unroll
        for (int d = 0; d < 3; d++) sf[d] = wave_sum(fv[d]);
        if (lane == 0) {
            wave_cnt[w] = __popcll(mask);
#pragma unroll
            for (int d = 0; d < 3; d++) wave_f[w][d] = sf[d];
        }
        __syncthreads();
        int off = base_s;
        for (int k = 0; k < w; k++) off += wave_cnt[k];
        if (act) {
            const int slot = off + before;
            ids[slot] = i;
            phi_out[slot] = phi;
#pragma unroll
            for (int d = 0; d < 3; d++) f[3 * slot + d] = fv[d];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int k = 0; k < 16; k++) {
                tot += wave_cnt[k];
#pragma unroll
                for (int d = 0; d < 3; d++) F_s[d] += wave_f[k][d];
            }
            base_s += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *count = base_s;
#pragma unroll
        for (int d = 0; d < 3; d++) Ftot[d] = F_s[d];
    }
}

// ---------------------------------------------------------------------------
// Outputs for data generation (one instance at its current state).
// k_tet_stress: one block per tile stages the tile's displacements in LDS;
// per tet F = I + G, the first Piola-Kirchhoff stress as in the element
// pass, the Cauchy stress sigma = P F^T / J (symmetrised; xx yy zz xy xz yz)
// and its von Mises value, written in FP64 at the tet's input index.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tet_stress(const Topo<T> *topos, const InstBufs<T> *bufs, int inst,
                                                       double *sigma, double *vm) {
    __shared__ __attribute__((aligned(32))) T su[kSw * kTileNodes];
    const BufsD<T> B = dev_view(bufs[inst]);
    const TopoD<T> tp = dev_view(topos[B.topo]);
    const int t = blockIdx.x;
    if (t >= tp.ntile) return;
    const T mu = (T)B.s->mu, lam = (T)B.s->lam;
    const int model = B.s->model;
    const int e0 = tp.tile_ent[t], ne = tp.tile_ent[t + 1] - e0;
    const int k0 = tp.tile_tet[t], nk = tp.tile_tet[t + 1] - k0;
    for (int l = threadIdx.x; l < ne; l += kBlock) {
        const int gid = tp.ent_node[e0 + l], sl = tp.ent_slot[e0 + l];
#pragma unroll
        for (int d = 0; d < 3; d++) su[kSw * sl + d] = B.u[3 * gid + d];
        su[kSw * sl + 3] = (T)0;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nk; k += kBlock) {
        int l[4];
        TetWords<T> tw;
        fetch_tet(tp, k0 + k, tw);
        const ElemGeo<T> geo = unpack_tet(tw, l);
        T wu[4][3];
        load_nodes(su, l, wu);
        T G[9];
        edge_gradient(wu, geo.Bm, G);
        const T Jm1 = det_minus_one(G);
        const T J = (T)1 + Jm1;
        const int id = tp.tet_id[k0 + k];
        double out[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        double v = 0.0;
        if (J > (T)0) {
            T psi, mag, Pk[9], Mb[9], ka, kb, F[9];
            if (model == LAW_CR)
                Law<T, LAW_CR>::element(G, Jm1, J, mu, lam, psi, mag, Pk, Mb, ka, kb);
            else
                Law<T, LAW_NH>::element(G, Jm1, J, mu, lam, psi, mag, Pk, Mb, ka, kb);
#pragma unroll
            for (int c = 0; c < 9; c++) F[c] = G[c] + (c % 4 == 0 ? (T)1 : (T)0);
            double S[9];
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++)
                    S[3 * i + j] = ((double)Pk[3 * i] * F[3 * j] + (double)Pk[3 * i + 1] * F[3 * j + 1] +
                                    (double)Pk[3 * i + 2] * F[3 * j + 2]) / (double)J;
            out[0] = S[0];
            out[1] = S[4];
            out[2] = S[8];
            out[3] = 0.5 * (S[1] + S[3]);
            out[4] = 0.5 * (S[2] + S[6]);
            out[5] = 0.5 * (S[5] + S[7]);
            const double a = out[0] - out[1], b = out[1] - out[2], c = out[2] - out[0];
            v = sqrt(0.5 * (a * a + b * b + c * c) + 3.0 * (out[3] * out[3] + out[4] * out[4] + out[5] * out[5]));
        } else {
            v = NAN;
#pragma unroll
            for (int c = 0; c < 6; c++) out[c] = NAN;
        }
        if (sigma)
#pragma unroll
            for (int c = 0; c < 6; c++) sigma[6 * (size_t)id + c] = out[c];
        if (vm) vm[id] = v;
    }
}

// max_i |u_i| and mean_i |u_i| of one instance (one block, FP64 sums).
template <typename T>
__global__ __launch_bounds__(1024) void k_disp_stats(const Topo<T> *topos, const InstBufs<T> *bufs, int inst,
                                                     double *out) {
    __shared__ double smax[16], ssum[16];
    const BufsD<T> B = dev_view(bufs[inst]);
    const int n = topos[B.topo].n;
    double mx = 0.0, sum = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double x = B.u[3 * i], y = B.u[3 * i + 1], z = B.u[3 * i + 2];
        const double a = sqrt(x * x + y * y + z * z);
        mx = fmax(mx, a);
        sum += a;
    }
    sum = wave_sum(sum);
    mx = -wave_min(-mx);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        smax[wv] = mx;
        ssum[wv] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m2 = 0.0, s2 = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); k++) {
            m2 = fmax(m2, smax[k]);
            s2 += ssum[k];
        }
        out[0] = m2;
        out[1] = n > 0 ? s2 / n : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Mesh set-up kernels.
// ---------------------------------------------------------------------------
// Rest volume check (FP64): records the first tet with det D_m <= 0.
__global__ __launch_bounds__(kBlock) void k_check_volumes(const double *X, const int *tet, int m, int *bad) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const int v0 = tet[4 * e];
    double D[9];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int va = tet[4 * e + a + 1];
#pragma unroll
        for (int i = 0; i < 3; i++) D[3 * i + a] = X[3 * va + i] - X[3 * v0 + i];
    }
    const double det = D[0] * (D[4] * D[8] - D[5] * D[7]) - D[1] * (D[3] * D[8] - D[5] * D[6]) +
                       D[2] * (D[3] * D[7] - D[4] * D[6]);
    if (!(det > 0.0)) atomicMin(bad, e);
}

// Rest constants per tet in tile order (FP64, stored in the path precision):
// D_m = [X1-X0, X2-X0, X3-X0], D_m^-1 by cofactors, V = |det D_m| / 6, from
// the tet's nodes in device vertex order (tnodes, 4 per tet in tile order;
// any reordering of the input's vertices: F = D_s D_m^-1 does not depend on
// it, and the input orientation is checked by k_check_volumes); with the
// tet's packed local node slots.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rest_constants(const double *X, const int *tnodes, const uint32_t *loc,
                                                           int m, TetRec<T> *rec) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= m) return;
    const int *tet = tnodes + 4 * (size_t)k;
    const int v0 = tet[0];
    double D[9];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int va = tet[a + 1];
#pragma unroll
        for (int i = 0; i < 3; i++) D[3 * i + a] = X[3 * va + i] - X[3 * v0 + i];
    }
    const double c00 = D[4] * D[8] - D[5] * D[7], c01 = D[5] * D[6] - D[3] * D[8], c02 = D[3] * D[7] - D[4] * D[6];
    const double det = D[0] * c00 + D[1] * c01 + D[2] * c02;
    const double id = 1.0 / det;
    const double inv[9] = {c00 * id, (D[2] * D[7] - D[1] * D[8]) * id, (D[1] * D[5] - D[2] * D[4]) * id,
                           c01 * id, (D[0] * D[8] - D[2] * D[6]) * id, (D[2] * D[3] - D[0] * D[5]) * id,
                           c02 * id, (D[1] * D[6] - D[0] * D[7]) * id, (D[0] * D[4] - D[1] * D[3]) * id};
    TetRec<T> r{};
#pragma unroll
    for (int c = 0; c < 9; c++) r.Bm[c] = (T)inv[c];
    r.V = (T)(fabs(det) / 6.0);
    r.loc = loc[k];
    rec[k] = r;
}

// Boundary faces by hashing the sorted node triple (21 bits per id) of each
// of the 4m faces into an open-addressing table; faces seen once are on the
// boundary.
__device__ __forceinline__ unsigned long long face_key(const int *tet, int e, int f) {
    int a = tet[4 * e + ((f + 1) & 3)], b = tet[4 * e + ((f + 2) & 3)], c = tet[4 * e + ((f + 3) & 3)];
    int t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    return ((unsigned long long)a << 42) | ((unsigned long long)b << 21) | (unsigned long long)c;
}

// Slot hash of a face key: the 64-bit finaliser (fmix64) of Austin Appleby's
// public-domain MurmurHash3, with its published shift and multiplier constants.
__device__ __forceinline__ unsigned face_hash(unsigned long long k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return (unsigned)k;
}

__global__ __launch_bounds__(kBlock) void k_faces_insert(const int *tet, int m, unsigned long long *keys,
                                                         unsigned *cnt, unsigned mask) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= 4 * m) return;
    const unsigned long long k = face_key(tet, t >> 2, t & 3);
    unsigned h = face_hash(k) & mask;
    for (;;) {   // load factor <= 1/2: a free or matching slot is always found
        const unsigned long long prev = atomicCAS(keys + h, ~0ull, k);
        if (prev == ~0ull || prev == k) {
            atomicAdd(cnt + h, 1u);
            return;
        }
        h = (h + 1) & mask;
    }
}

__global__ __launch_bounds__(kBlock) void k_faces_mark(const int *tet, int m, const unsigned long long *keys,
                                                       const unsigned *cnt, unsigned mask, uint8_t *surf) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= 4 * m) return;
    const int e = t >> 2, f = t & 3;
    const unsigned long long k = face_key(tet, e, f);
    unsigned h = face_hash(k) & mask;
    while (keys[h] != k) h = (h + 1) & mask;   // the key was inserted
    if (cnt[h] == 1u) {
        surf[tet[4 * e + ((f + 1) & 3)]] = 1;
        surf[tet[4 * e + ((f + 2) & 3)]] = 1;
        surf[tet[4 * e + ((f + 3) & 3)]] = 1;
    }
}

// One block: eligible = surface and not fixed; ascending compaction and the
// node -> contact slot map.
__global__ __launch_bounds__(1024) void k_compact_eligible(const uint8_t *surf, const uint8_t *fixed, int n,
                                                           uint8_t *elig, int *list, int *cidx, int *count) {
    __shared__ int wave_cnt[16];
    __shared__ int base_s;
    if (threadIdx.x == 0) base_s = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int start = 0; start < n; start += 1024) {
        const int i = start + threadIdx.x;
        const bool act = i < n && surf[i] && !fixed[i];
        const unsigned long long mask = __ballot(act);
        if (lane == 0) wave_cnt[w] = __popcll(mask);
        __syncthreads();
        int off = base_s;
        for (int k = 0; k < w; k++) off += wave_cnt[k];
        if (i < n) {
            elig[i] = act ? 1 : 0;
            const int slot = off + __popcll(mask & ((1ull << lane) - 1ull));
            cidx[i] = act ? slot : -1;
            if (act) list[slot] = i;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int k = 0; k < 16; k++) tot += wave_cnt[k];
            base_s += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base_s;
}

}  // namespace fem
