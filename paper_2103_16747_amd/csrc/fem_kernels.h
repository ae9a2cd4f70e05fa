// Device kernels of the indentation solve for gfx950 (CDNA4, wave64).
//
// Layout in HBM (per instance): tet connectivity and per-tet constants are
// SoA (field-major, one coalesced stream per field); node vectors are packed
// xyz (n x 3) so a tet's four-node gather is four 12- or 24-byte loads. All
// kernels are bandwidth-bound: the element and Hessian-vector kernels stream
// per-tet constants once per pass and gather/scatter node data that stays in
// L2/MALL; the node kernels stream the CG vectors. Reductions are FP64 in
// both precision modes: per-wave shuffles, per-block LDS, one partial per
// block, and the last block to finish (ticket counter) sums the partials in a
// fixed order, so every reduction is deterministic for a given grid.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fem {

constexpr int kBlock = 256;               // 4 wavefronts of 64
constexpr int kWaves = kBlock / 64;

// CG state codes kept in Scalars::state.
enum : int { kRunning = 0, kConverged = 1, kNegCurv = 2, kMaxIter = 3 };

struct Indenter {
    int kind;            // 0 sphere, 1 cylinder, 2 box, 3 ring
    double shape[4];
    double R[9];         // row-major, local -> world
    double c[3];
    double k;
};

// Device-resident scalars of one solve.
struct Scalars {
    double energy, emag, minJ;   // last element pass
    double gg;                   // |g_free|^2 at the last Newton init
    double rz, rr, pq, alpha, beta;
    double tol2;                 // CG stops when |r|^2 <= tol2
    double gd;                   // g . dx
    int it, max_it, state, nhv;  // CG iteration, cap, state, Hv products
};

template <typename T>
struct Buffers {
    int n, m, nc;
    const int *tet;       // 4 x m
    const T *B;           // 9 x m  (row-major D_m^-1 entries, field-major)
    const T *vol;         // m
    const double *X;      // n x 3
    const uint8_t *fixed; // n
    const int *cnodes;    // nc contact-eligible node ids, ascending
    T *u, *dx, *g, *r, *z, *p, *q;   // n x 3
    T *diag;              // n x 6 symmetric node blocks (xx yy zz xy xz yz)
    T *dinv;              // n x 6
    T *finv;              // 9 x m cached F^-1 (row-major entries)
    T *c1;                // m cached mu - lam ln J
    T *chess;             // nc x 6 contact Hessian blocks
    double *partial;      // 4 x kMaxPartials
    unsigned *ticket;     // one counter per reduction kernel
    Scalars *s;
    double mu, lam;
    Indenter ind;
};

constexpr int kMaxPartials = 1 << 16;
enum : int { kTicketGrad = 0, kTicketInit, kTicketHv, kTicketUpd, kTicketDot, kTicketCount };

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
    return v;
}

// Reduces NS sums and (optionally) one min over the block; thread 0 gets them.
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

// After thread 0 has written this block's partials: returns true in every
// thread of the last block to arrive. Release/acquire at agent scope so the
// partials written on other XCDs are visible to the last block.
__device__ __forceinline__ bool last_block(unsigned *ticket) {
    __shared__ unsigned s_last;
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (t == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    const bool last = s_last != 0;
    if (last) __threadfence();
    return last;
}

__device__ __forceinline__ double load_partial(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sums NS partial streams (stride kMaxPartials) over nb blocks in a fixed
// order; valid in thread 0. Optionally also the min of stream NS.
template <int NS, bool MIN>
__device__ __forceinline__ void sum_partials(const double *partial, int nb, double (&out)[NS], double &mn) {
#pragma unroll
    for (int i = 0; i < NS; i++) out[i] = 0.0;
    mn = INFINITY;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
#pragma unroll
        for (int i = 0; i < NS; i++) out[i] += load_partial(partial + i * kMaxPartials + b);
        if (MIN) mn = fmin(mn, load_partial(partial + NS * kMaxPartials + b));
    }
    block_reduce<NS, MIN>(out, mn);
}

// ---------------------------------------------------------------------------
// Small dense helpers
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c);
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ T log1p_t(T x);
template <>
__device__ __forceinline__ float log1p_t<float>(float x) { return log1pf(x); }
template <>
__device__ __forceinline__ double log1p_t<double>(double x) { return log1p(x); }

template <typename T>
__device__ __forceinline__ T abs_t(T x) { return x < (T)0 ? -x : x; }

template <typename T>
__device__ __forceinline__ void load3(const T *a, int i, T v[3]) {
    v[0] = a[3 * i]; v[1] = a[3 * i + 1]; v[2] = a[3 * i + 2];
}

template <typename T>
__device__ __forceinline__ void atomic_add3(T *a, int i, T x, T y, T z) {
    atomicAdd(a + 3 * i, x);
    atomicAdd(a + 3 * i + 1, y);
    atomicAdd(a + 3 * i + 2, z);
}

// Shape-function gradient of local node a (a = 0..3) from the SoA rows of
// D_m^-1: b_{a} = row a-1 for a >= 1, b_0 = -(b_1 + b_2 + b_3).
template <typename T>
__device__ __forceinline__ void shape_grad(const T Bm[9], int a, T b[3]) {
    if (a == 0) {
        b[0] = -(Bm[0] + Bm[3] + Bm[6]);
        b[1] = -(Bm[1] + Bm[4] + Bm[7]);
        b[2] = -(Bm[2] + Bm[5] + Bm[8]);
    } else {
        b[0] = Bm[3 * (a - 1)];
        b[1] = Bm[3 * (a - 1) + 1];
        b[2] = Bm[3 * (a - 1) + 2];
    }
}

// Edge-difference gradient: G = sum_a (w_{a+1} - w_0) (x) row_a(D_m^-1).
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

// Nodal vectors of an element first-Piola field: node a+1 receives
// V * S * row_a(D_m^-1)^T, node 0 the negated sum (the four sum to zero).
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
// and (for points inside) the world Hessian. Medial-axis ties go to the lower
// axis (x, y, z) and to the radial branch before the axial one.
// ---------------------------------------------------------------------------
__device__ inline void sdf_eval(const Indenter &ind, const double x[3], bool want_h, double &phi, double n[3],
                                double Hw[6]) {
    const double *R = ind.R;
    const double d0 = x[0] - ind.c[0], d1 = x[1] - ind.c[1], d2 = x[2] - ind.c[2];
    // q = R^T (x - c)
    double q[3];
#pragma unroll
    for (int k = 0; k < 3; k++) q[k] = R[k] * d0 + R[3 + k] * d1 + R[6 + k] * d2;
    double gq[3] = {0.0, 0.0, 0.0};
    double Hq[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // xx yy zz xy xz yz
    switch (ind.kind) {
    case 0: {   // sphere
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
    case 1: {   // capped cylinder about local z
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
            if (want_h && phi < 0.0 && rho > 0.0) {   // hoop curvature of the side wall
                const double tx = -ey, ty = ex, ir = 1.0 / rho;
                Hq[0] = tx * tx * ir; Hq[1] = ty * ty * ir; Hq[3] = tx * ty * ir;
            }
        } else {
            phi = dz;
            gq[2] = sz;
        }
        break;
    }
    case 2: {   // box
        double o2 = 0.0;
        double dd[3];
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
    default: {  // ring: torus about local z
        const double Rm = ind.shape[0], rm = ind.shape[1];
        const double rho = sqrt(q[0] * q[0] + q[1] * q[1]);
        const double ex = rho > 0.0 ? q[0] / rho : 1.0, ey = rho > 0.0 ? q[1] / rho : 0.0;
        const double wr = rho - Rm, wz = q[2];
        const double L = sqrt(wr * wr + wz * wz);
        phi = L - rm;
        if (L > 0.0) {
            const double cr = wr / L, cz = wz / L;   // gradient in the meridian plane
            gq[0] = cr * ex; gq[1] = cr * ey; gq[2] = cz;
            if (want_h && rho > 0.0) {
                // meridian tangent t = (-cz e_r + cr e_z), curvature 1/L; hoop
                // direction e_t = (-ey, ex, 0), curvature cr / rho.
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
    // n = R gq ; Hw = R Hq R^T
#pragma unroll
    for (int i = 0; i < 3; i++) n[i] = R[3 * i] * gq[0] + R[3 * i + 1] * gq[1] + R[3 * i + 2] * gq[2];
    if (want_h) {
        double Hf[9] = {Hq[0], Hq[3], Hq[4], Hq[3], Hq[1], Hq[5], Hq[4], Hq[5], Hq[2]};
        double RH[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) RH[3 * i + j] = R[3 * i] * Hf[j] + R[3 * i + 1] * Hf[3 + j] + R[3 * i + 2] * Hf[6 + j];
        double W[9];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) W[3 * i + j] = RH[3 * i] * R[3 * j] + RH[3 * i + 1] * R[3 * j + 1] + RH[3 * i + 2] * R[3 * j + 2];
        Hw[0] = W[0]; Hw[1] = W[4]; Hw[2] = W[8]; Hw[3] = W[1]; Hw[4] = W[2]; Hw[5] = W[5];
    }
}

// ---------------------------------------------------------------------------
// Element + contact pass. Blocks [0, tet_blocks) take one tet per thread,
// blocks after that one contact-eligible node per thread. Evaluates the state
// u + alpha dx (alpha = 0: the current state). Accumulates the energy, the
// energy-term magnitudes and min det F; with with_grad also scatters the
// gradient and the 3x3 node diagonal blocks, and caches F^-1, mu - lam ln J
// and the contact Hessian blocks for the Hessian-vector kernel.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_element_pass(Buffers<T> b, T alpha, int with_grad, int contact_full,
                                                          int tet_blocks) {
    double acc[2] = {0.0, 0.0};   // energy, magnitude
    double mnJ = INFINITY;
    const T mu = (T)b.mu, lam = (T)b.lam;
    if ((int)blockIdx.x < tet_blocks) {
        const int e = blockIdx.x * kBlock + threadIdx.x;
        if (e < b.m) {
            int v[4];
            T w[4][3];
#pragma unroll
            for (int a = 0; a < 4; a++) {
                v[a] = b.tet[a * b.m + e];
                T uu[3], dd[3];
                load3(b.u, v[a], uu);
                if (alpha != (T)0) {
                    load3(b.dx, v[a], dd);
#pragma unroll
                    for (int i = 0; i < 3; i++) uu[i] = fma_t(alpha, dd[i], uu[i]);
                }
#pragma unroll
                for (int i = 0; i < 3; i++) w[a][i] = uu[i];
            }
            T Bm[9];
#pragma unroll
            for (int k = 0; k < 9; k++) Bm[k] = b.B[k * b.m + e];
            const T V = b.vol[e];
            T G[9];
            edge_gradient(w, Bm, G);
            // J - 1 = tr G + (sum of principal 2x2 minors of G) + det G, without cancellation.
            const T trG = G[0] + G[4] + G[8];
            const T m2 = (G[0] * G[4] - G[1] * G[3]) + (G[0] * G[8] - G[2] * G[6]) + (G[4] * G[8] - G[5] * G[7]);
            const T dG = G[0] * (G[4] * G[8] - G[5] * G[7]) - G[1] * (G[3] * G[8] - G[5] * G[6]) +
                         G[2] * (G[3] * G[7] - G[4] * G[6]);
            const T Jm1 = trG + m2 + dG;
            const T J = (T)1 + Jm1;
            mnJ = (double)J;
            if (J > (T)0) {
                const T lnJ = log1p_t(Jm1);
                T G2 = (T)0;
#pragma unroll
                for (int k = 0; k < 9; k++) G2 += G[k] * G[k];
                // tr(F^T F) - 3 = 2 tr G + |G|^2
                const T t1 = (T)0.5 * mu * ((T)2 * trG + G2), t2 = -mu * lnJ, t3 = (T)0.5 * lam * lnJ * lnJ;
                acc[0] = (double)(V * (t1 + t2 + t3));
                acc[1] = (double)(V * (abs_t(t1) + abs_t(t2) + abs_t(t3)));
                if (with_grad) {
                    T F[9];
#pragma unroll
                    for (int k = 0; k < 9; k++) F[k] = G[k];
                    F[0] += (T)1; F[4] += (T)1; F[8] += (T)1;
                    // cofactor matrix C = J F^-T
                    T C[9];
                    C[0] = F[4] * F[8] - F[5] * F[7]; C[1] = F[5] * F[6] - F[3] * F[8]; C[2] = F[3] * F[7] - F[4] * F[6];
                    C[3] = F[2] * F[7] - F[1] * F[8]; C[4] = F[0] * F[8] - F[2] * F[6]; C[5] = F[1] * F[6] - F[0] * F[7];
                    C[6] = F[1] * F[5] - F[2] * F[4]; C[7] = F[2] * F[3] - F[0] * F[5]; C[8] = F[0] * F[4] - F[1] * F[3];
                    const T iJ = (T)1 / J;
                    T FiT[9];
#pragma unroll
                    for (int k = 0; k < 9; k++) FiT[k] = C[k] * iJ;
                    // P = mu (F - F^-T) + lam ln J F^-T
                    T P[9];
#pragma unroll
                    for (int k = 0; k < 9; k++) P[k] = mu * (F[k] - FiT[k]) + lam * lnJ * FiT[k];
                    T f[4][3];
                    element_nodal(P, Bm, V, f);
#pragma unroll
                    for (int a = 0; a < 4; a++) atomic_add3(b.g, v[a], f[a][0], f[a][1], f[a][2]);
                    // node diagonal blocks V (mu |b|^2 I + (mu + lam - lam ln J) c c^T), c = F^-T b
                    const T kc = mu + lam - lam * lnJ;
#pragma unroll
                    for (int a = 0; a < 4; a++) {
                        T bb[3];
                        shape_grad(Bm, a, bb);
                        const T c0 = FiT[0] * bb[0] + FiT[1] * bb[1] + FiT[2] * bb[2];
                        const T c1v = FiT[3] * bb[0] + FiT[4] * bb[1] + FiT[5] * bb[2];
                        const T c2 = FiT[6] * bb[0] + FiT[7] * bb[1] + FiT[8] * bb[2];
                        const T s = V * mu * (bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2]);
                        const T Vk = V * kc;
                        T *dg = b.diag + 6 * v[a];
                        atomicAdd(dg + 0, s + Vk * c0 * c0);
                        atomicAdd(dg + 1, s + Vk * c1v * c1v);
                        atomicAdd(dg + 2, s + Vk * c2 * c2);
                        atomicAdd(dg + 3, Vk * c0 * c1v);
                        atomicAdd(dg + 4, Vk * c0 * c2);
                        atomicAdd(dg + 5, Vk * c1v * c2);
                    }
                    // cache F^-1 (transpose of F^-T) and mu - lam ln J
#pragma unroll
                    for (int i = 0; i < 3; i++)
#pragma unroll
                        for (int j = 0; j < 3; j++) b.finv[(3 * i + j) * b.m + e] = FiT[3 * j + i];
                    b.c1[e] = mu - lam * lnJ;
                }
            } else {
                acc[0] = INFINITY;
            }
        }
    } else {
        const int j = (blockIdx.x - tet_blocks) * kBlock + threadIdx.x;
        if (j < b.nc) {
            const int i = b.cnodes[j];
            double x[3];
#pragma unroll
            for (int d = 0; d < 3; d++) {
                T ui = b.u[3 * i + d];
                if (alpha != (T)0) ui = fma_t(alpha, b.dx[3 * i + d], ui);
                x[d] = b.X[3 * i + d] + (double)ui;
            }
            double phi, nv[3], Hs[6];
            sdf_eval(b.ind, x, with_grad && contact_full, phi, nv, Hs);
            T blk[6] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
            if (phi < 0.0) {
                const double kp = b.ind.k;
                const double ec = 0.5 * kp * phi * phi;
                acc[0] = ec;
                acc[1] = ec;
                if (with_grad) {
                    atomic_add3(b.g, i, (T)(kp * phi * nv[0]), (T)(kp * phi * nv[1]), (T)(kp * phi * nv[2]));
                    const double hs = contact_full ? phi : 0.0;
                    double h6[6] = {nv[0] * nv[0], nv[1] * nv[1], nv[2] * nv[2], nv[0] * nv[1], nv[0] * nv[2], nv[1] * nv[2]};
#pragma unroll
                    for (int k = 0; k < 6; k++) {
                        blk[k] = (T)(kp * (h6[k] + (contact_full ? hs * Hs[k] : 0.0)));
                        atomicAdd(b.diag + 6 * i + k, blk[k]);
                    }
                }
            }
            if (with_grad) {
#pragma unroll
                for (int k = 0; k < 6; k++) b.chess[6 * j + k] = blk[k];
            }
        }
    }
    block_reduce<2, true>(acc, mnJ);
    if (threadIdx.x == 0) {
        b.partial[blockIdx.x] = acc[0];
        b.partial[kMaxPartials + blockIdx.x] = acc[1];
        b.partial[2 * kMaxPartials + blockIdx.x] = mnJ;
    }
    if (last_block(b.ticket + kTicketGrad)) {
        double tot[2], mn;
        sum_partials<2, true>(b.partial, gridDim.x, tot, mn);
        if (threadIdx.x == 0) {
            b.s->energy = mn > 0.0 ? tot[0] : INFINITY;
            b.s->emag = tot[1];
            b.s->minJ = mn;
            b.ticket[kTicketGrad] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Newton init: r = -g and z = M^-1 r on free nodes, block or scalar Jacobi
// from the node diagonal blocks; clears dx, p, q; reduces |g_free|^2 and r.z.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T safe_recip(T d) {
    return d > (T)0 ? (T)1 / d : (d < (T)0 ? (T)1 / -d : (T)1);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_newton_init(Buffers<T> b, int block_jacobi) {
    double acc[2] = {0.0, 0.0};   // g.g, r.z
    double unused = 0.0;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < b.n) {
        T M[6] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
        T rr[3] = {(T)0, (T)0, (T)0}, zz[3] = {(T)0, (T)0, (T)0};
        if (!b.fixed[i]) {
            const T *D = b.diag + 6 * i;
            const T a = D[0], bb = D[1], c = D[2], d = D[3], e = D[4], f = D[5];
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
            for (int k = 0; k < 3; k++) rr[k] = -b.g[3 * i + k];
            zz[0] = M[0] * rr[0] + M[3] * rr[1] + M[4] * rr[2];
            zz[1] = M[3] * rr[0] + M[1] * rr[1] + M[5] * rr[2];
            zz[2] = M[4] * rr[0] + M[5] * rr[1] + M[2] * rr[2];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                acc[0] += (double)rr[k] * (double)rr[k];
                acc[1] += (double)rr[k] * (double)zz[k];
            }
        }
#pragma unroll
        for (int k = 0; k < 6; k++) b.dinv[6 * i + k] = M[k];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            b.r[3 * i + k] = rr[k];
            b.z[3 * i + k] = zz[k];
            b.dx[3 * i + k] = (T)0;
            b.p[3 * i + k] = (T)0;
            b.q[3 * i + k] = (T)0;
        }
    }
    block_reduce<2, false>(acc, unused);
    if (threadIdx.x == 0) {
        b.partial[blockIdx.x] = acc[0];
        b.partial[kMaxPartials + blockIdx.x] = acc[1];
    }
    if (last_block(b.ticket + kTicketInit)) {
        double tot[2], mn;
        sum_partials<2, false>(b.partial, gridDim.x, tot, mn);
        if (threadIdx.x == 0) {
            Scalars *s = b.s;
            s->gg = tot[0];
            s->rr = tot[0];
            s->rz = tot[1];
            s->beta = 0.0;
            s->alpha = 0.0;
            s->it = 0;
            s->nhv = 0;
            s->state = kRunning;
            b.ticket[kTicketInit] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// CG, Hessian-vector half: q = H p with p = z + beta p_prev formed on the fly
// (the update kernel forms the identical value), element part from the cached
// F^-1 and mu - lam ln J:
//   dP = mu dG + (mu - lam ln J) (F^-1 dG F^-1)^T + lam tr(F^-1 dG) F^-T,
// plus the contact blocks; p.q is accumulated element by element, so no
// second pass over q is needed. force = 1 ignores the CG state (diagnostics).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_hv(Buffers<T> b, int tet_blocks, int force) {
    if (!force && b.s->state != kRunning) return;
    const T beta = (T)b.s->beta;
    const T mu = (T)b.mu, lam = (T)b.lam;
    double acc[1] = {0.0};
    double unused = 0.0;
    if ((int)blockIdx.x < tet_blocks) {
        const int e = blockIdx.x * kBlock + threadIdx.x;
        if (e < b.m) {
            int v[4];
            T w[4][3];
#pragma unroll
            for (int a = 0; a < 4; a++) {
                v[a] = b.tet[a * b.m + e];
#pragma unroll
                for (int i = 0; i < 3; i++) w[a][i] = fma_t(beta, b.p[3 * v[a] + i], b.z[3 * v[a] + i]);
            }
            T Bm[9], Fi[9];
#pragma unroll
            for (int k = 0; k < 9; k++) {
                Bm[k] = b.B[k * b.m + e];
                Fi[k] = b.finv[k * b.m + e];
            }
            const T V = b.vol[e], cc = b.c1[e];
            T dG[9];
            edge_gradient(w, Bm, dG);
            T A[9];   // F^-1 dG
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) A[3 * i + j] = Fi[3 * i] * dG[j] + Fi[3 * i + 1] * dG[3 + j] + Fi[3 * i + 2] * dG[6 + j];
            const T tr = A[0] + A[4] + A[8];
            T Mm[9];  // F^-1 dG F^-1
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) Mm[3 * i + j] = A[3 * i] * Fi[j] + A[3 * i + 1] * Fi[3 + j] + A[3 * i + 2] * Fi[6 + j];
            T dP[9];
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++)
                    dP[3 * i + j] = mu * dG[3 * i + j] + cc * Mm[3 * j + i] + lam * tr * Fi[3 * j + i];
            T f[4][3];
            element_nodal(dP, Bm, V, f);
            double pq = 0.0;
#pragma unroll
            for (int a = 0; a < 4; a++) {
                atomic_add3(b.q, v[a], f[a][0], f[a][1], f[a][2]);
                pq += (double)(w[a][0] * f[a][0] + w[a][1] * f[a][1] + w[a][2] * f[a][2]);
            }
            acc[0] = pq;
        }
    } else {
        const int j = (blockIdx.x - tet_blocks) * kBlock + threadIdx.x;
        if (j < b.nc) {
            const T *H = b.chess + 6 * j;
            if (H[0] != (T)0 || H[1] != (T)0 || H[2] != (T)0 || H[3] != (T)0 || H[4] != (T)0 || H[5] != (T)0) {
                const int i = b.cnodes[j];
                T pv[3];
#pragma unroll
                for (int d = 0; d < 3; d++) pv[d] = fma_t(beta, b.p[3 * i + d], b.z[3 * i + d]);
                const T q0 = H[0] * pv[0] + H[3] * pv[1] + H[4] * pv[2];
                const T q1 = H[3] * pv[0] + H[1] * pv[1] + H[5] * pv[2];
                const T q2 = H[4] * pv[0] + H[5] * pv[1] + H[2] * pv[2];
                atomic_add3(b.q, i, q0, q1, q2);
                acc[0] = (double)(pv[0] * q0 + pv[1] * q1 + pv[2] * q2);
            }
        }
    }
    block_reduce<1, false>(acc, unused);
    if (threadIdx.x == 0) b.partial[3 * kMaxPartials + blockIdx.x] = acc[0];
    if (last_block(b.ticket + kTicketHv)) {
        double tot[1], mn;
        sum_partials<1, false>(b.partial + 3 * kMaxPartials, gridDim.x, tot, mn);
        if (threadIdx.x == 0) {
            Scalars *s = b.s;
            s->pq = tot[0];
            if (!force) {
                s->nhv += 1;
                if (tot[0] > 0.0)
                    s->alpha = s->rz / tot[0];
                else
                    s->state = kNegCurv;
            }
            b.ticket[kTicketHv] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// CG, update half (free nodes): p = z + beta p_prev; dx += alpha p;
// r -= alpha q; q = 0; z = M^-1 r; reduces r.z and r.r, then beta and the
// stopping test. On non-positive curvature at the first iteration the
// preconditioned residual becomes the Newton direction.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update(Buffers<T> b) {
    const int state = b.s->state;
    if (state == kConverged || state == kMaxIter) return;
    const bool negcurv = state == kNegCurv;
    const T alpha = (T)b.s->alpha, beta = (T)b.s->beta;
    double acc[2] = {0.0, 0.0};   // r.z, r.r
    double unused = 0.0;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < b.n) {
        if (negcurv) {
            if (b.s->it == 0)
#pragma unroll
                for (int k = 0; k < 3; k++) b.dx[3 * i + k] = fma_t(beta, b.p[3 * i + k], b.z[3 * i + k]);
        } else if (!b.fixed[i]) {
            T pv[3], rv[3];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                pv[k] = fma_t(beta, b.p[3 * i + k], b.z[3 * i + k]);
                b.p[3 * i + k] = pv[k];
                b.dx[3 * i + k] = fma_t(alpha, pv[k], b.dx[3 * i + k]);
                rv[k] = fma_t(-alpha, b.q[3 * i + k], b.r[3 * i + k]);
                b.r[3 * i + k] = rv[k];
                b.q[3 * i + k] = (T)0;
            }
            const T *M = b.dinv + 6 * i;
            const T z0 = M[0] * rv[0] + M[3] * rv[1] + M[4] * rv[2];
            const T z1 = M[3] * rv[0] + M[1] * rv[1] + M[5] * rv[2];
            const T z2 = M[4] * rv[0] + M[5] * rv[1] + M[2] * rv[2];
            b.z[3 * i] = z0;
            b.z[3 * i + 1] = z1;
            b.z[3 * i + 2] = z2;
            acc[0] = (double)rv[0] * (double)z0 + (double)rv[1] * (double)z1 + (double)rv[2] * (double)z2;
            acc[1] = (double)rv[0] * (double)rv[0] + (double)rv[1] * (double)rv[1] + (double)rv[2] * (double)rv[2];
        } else {
#pragma unroll
            for (int k = 0; k < 3; k++) b.q[3 * i + k] = (T)0;
        }
    }
    block_reduce<2, false>(acc, unused);
    if (threadIdx.x == 0) {
        b.partial[blockIdx.x] = acc[0];
        b.partial[kMaxPartials + blockIdx.x] = acc[1];
    }
    if (last_block(b.ticket + kTicketUpd)) {
        double tot[2], mn;
        sum_partials<2, false>(b.partial, gridDim.x, tot, mn);
        if (threadIdx.x == 0) {
            Scalars *s = b.s;
            if (negcurv) {
                s->state = kConverged;
            } else {
                s->it += 1;
                s->beta = tot[0] / s->rz;
                s->rz = tot[0];
                s->rr = tot[1];
                if (tot[1] <= s->tol2)
                    s->state = kConverged;
                else if (s->it >= s->max_it)
                    s->state = kMaxIter;
            }
            b.ticket[kTicketUpd] = 0;
        }
    }
}

// g . dx over all nodes (dx is zero on fixed nodes).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot_gdx(Buffers<T> b) {
    double acc[1] = {0.0};
    double unused = 0.0;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < b.n)
#pragma unroll
        for (int k = 0; k < 3; k++) acc[0] += (double)b.g[3 * i + k] * (double)b.dx[3 * i + k];
    block_reduce<1, false>(acc, unused);
    if (threadIdx.x == 0) b.partial[blockIdx.x] = acc[0];
    if (last_block(b.ticket + kTicketDot)) {
        double tot[1], mn;
        sum_partials<1, false>(b.partial, gridDim.x, tot, mn);
        if (threadIdx.x == 0) {
            b.s->gd = tot[0];
            b.ticket[kTicketDot] = 0;
        }
    }
}

// u = u + alpha dx, with the same rounding as the trial evaluation.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy(T *u, const T *dx, T alpha, int len) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < len) u[i] = fma_t(alpha, dx[i], u[i]);
}

// ---------------------------------------------------------------------------
// Contact patch at the current state: one block walks the eligible nodes in
// ascending order and compacts those with phi < 0 (ordered scan), writing
// ids, forces on the skin -k phi n, phi, the count and the FP64 resultant.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void k_contact_patch(Buffers<T> b, int *ids, double *f, double *phi_out,
                                                          int *count, double *Ftot) {
    __shared__ int wave_cnt[16];
    __shared__ double wave_f[16][3];
    __shared__ int base_s;
    __shared__ double F_s[3];
    if (threadIdx.x == 0) {
        base_s = 0;
        F_s[0] = F_s[1] = F_s[2] = 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int start = 0; start < b.nc; start += 1024) {
        const int j = start + threadIdx.x;
        double phi = 0.0, nv[3] = {0.0, 0.0, 0.0}, Hs[6];
        int i = -1;
        bool act = false;
        if (j < b.nc) {
            i = b.cnodes[j];
            double x[3];
#pragma unroll
            for (int d = 0; d < 3; d++) x[d] = b.X[3 * i + d] + (double)b.u[3 * i + d];
            sdf_eval(b.ind, x, false, phi, nv, Hs);
            act = phi < 0.0;
        }
        double fv[3];
#pragma unroll
        for (int d = 0; d < 3; d++) fv[d] = act ? -b.ind.k * phi * nv[d] : 0.0;
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
// Mesh precompute (FP64): D_m = [X1-X0, X2-X0, X3-X0], V = det D_m / 6,
// D_m^-1 by cofactors; the first tet with V <= 0 is recorded.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_precompute(const double *X, const int *tet, int m, T *B, T *vol,
                                                        int *bad) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const int v0 = tet[e];
    double D[9];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int va = tet[(a + 1) * m + e];
#pragma unroll
        for (int i = 0; i < 3; i++) D[3 * i + a] = X[3 * va + i] - X[3 * v0 + i];
    }
    const double c00 = D[4] * D[8] - D[5] * D[7], c01 = D[5] * D[6] - D[3] * D[8], c02 = D[3] * D[7] - D[4] * D[6];
    const double det = D[0] * c00 + D[1] * c01 + D[2] * c02;
    const double V = det / 6.0;
    if (!(V > 0.0)) {
        atomicMin(bad, e);
        return;
    }
    const double id = 1.0 / det;
    // inverse = adj(D) / det, adj = cofactor^T
    double inv[9];
    inv[0] = c00 * id;
    inv[1] = (D[2] * D[7] - D[1] * D[8]) * id;
    inv[2] = (D[1] * D[5] - D[2] * D[4]) * id;
    inv[3] = c01 * id;
    inv[4] = (D[0] * D[8] - D[2] * D[6]) * id;
    inv[5] = (D[2] * D[3] - D[0] * D[5]) * id;
    inv[6] = c02 * id;
    inv[7] = (D[1] * D[6] - D[0] * D[7]) * id;
    inv[8] = (D[0] * D[4] - D[1] * D[3]) * id;
#pragma unroll
    for (int k = 0; k < 9; k++) B[k * m + e] = (T)inv[k];
    vol[e] = (T)V;
}

// Boundary faces by hashing: each of the 4m faces is keyed by its sorted node
// triple (21 bits per id) and counted in an open-addressing table; faces seen
// once are boundary faces.
__device__ __forceinline__ unsigned long long face_key(const int *tet, int m, int e, int f) {
    int a = tet[((f + 1) & 3) * m + e], b = tet[((f + 2) & 3) * m + e], c = tet[((f + 3) & 3) * m + e];
    int t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    return ((unsigned long long)a << 42) | ((unsigned long long)b << 21) | (unsigned long long)c;
}

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
    const unsigned long long k = face_key(tet, m, t >> 2, t & 3);
    unsigned h = face_hash(k) & mask;
    for (;;) {   // load factor <= 1/2, so a free or matching slot is always found
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
    const unsigned long long k = face_key(tet, m, e, f);
    unsigned h = face_hash(k) & mask;
    while (keys[h] != k) h = (h + 1) & mask;   // the key was inserted
    if (cnt[h] == 1u) {
        surf[tet[((f + 1) & 3) * m + e]] = 1;
        surf[tet[((f + 2) & 3) * m + e]] = 1;
        surf[tet[((f + 3) & 3) * m + e]] = 1;
    }
}

// One block: eligible = surface and not fixed; ascending compaction.
__global__ __launch_bounds__(1024) void k_compact_eligible(const uint8_t *surf, const uint8_t *fixed, int n,
                                                           uint8_t *elig, int *list, int *count) {
    __shared__ int wave_cnt[16];
    __shared__ int base_s;
    if (threadIdx.x == 0) base_s = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int start = 0; start < n; start += 1024) {
        const int i = start + threadIdx.x;
        const bool act = i < n && surf[i] && !fixed[i];
        if (i < n) elig[i] = act ? 1 : 0;
        const unsigned long long mask = __ballot(act);
        if (lane == 0) wave_cnt[w] = __popcll(mask);
        __syncthreads();
        int off = base_s;
        for (int k = 0; k < w; k++) off += wave_cnt[k];
        if (act) list[off + __popcll(mask & ((1ull << lane) - 1ull))] = i;
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
