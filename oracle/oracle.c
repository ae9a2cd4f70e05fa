/*
 * FP64 CPU oracle for the quasi-static Neo-Hookean indentation solve.
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow, obviously-correct reference that
 * the device path is checked against. Only tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.
 *
 * What it computes follows paper Sec. III-A (linear tetrahedral FEM of the
 * skin, Neo-Hookean material as in the validated model, fixed boundary nodes,
 * rigid indenters driven into the skin, outputs = nodal positions and nodal
 * contact forces). The paper prints no equations; where it is silent the
 * following readings are taken:
 *   - Neo-Hookean: the compressible form
 *       Psi(F) = mu/2 (tr F^T F - 3) - mu ln J + lam/2 (ln J)^2,  J = det F,
 *     whose linearisation at F = I is isotropic Hooke with Lame (mu, lam);
 *   - contact: per-node penalty k/2 min(0, phi)^2 against the indenter's
 *     signed distance phi, on surface nodes that are not fixed; optionally
 *     with lagged, smoothed Coulomb friction (see oracle.h);
 *   - quasi-static load steps solved by Newton, with the linear systems solved
 *     by Jacobi-preconditioned CG (truncated at non-positive curvature) and an
 *     Armijo backtracking line search that also rejects inverted tets;
 *   - the Newton matrix is the exact Neo-Hookean tangent plus the contact
 *     block, either Gauss-Newton k n n^T or the exact k (n n^T + phi Hess(phi)).
 * The oracle assembles the Hessian explicitly in a 3x3 block-sparse format,
 * which the device path never does.
 *
 * Rounding: IEEE double, compiled without fast-math and without FMA
 * contraction.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* 3x3 helpers (row-major)                                                  */
/* ------------------------------------------------------------------------ */
static double det3(const double A[9]) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* Inverse by the adjugate; returns the determinant. */
static double inv3(const double A[9], double Ai[9]) {
    double d = det3(A);
    Ai[0] = (A[4] * A[8] - A[5] * A[7]) / d;
    Ai[1] = (A[2] * A[7] - A[1] * A[8]) / d;
    Ai[2] = (A[1] * A[5] - A[2] * A[4]) / d;
    Ai[3] = (A[5] * A[6] - A[3] * A[8]) / d;
    Ai[4] = (A[0] * A[8] - A[2] * A[6]) / d;
    Ai[5] = (A[2] * A[3] - A[0] * A[5]) / d;
    Ai[6] = (A[3] * A[7] - A[4] * A[6]) / d;
    Ai[7] = (A[1] * A[6] - A[0] * A[7]) / d;
    Ai[8] = (A[0] * A[4] - A[1] * A[3]) / d;
    return d;
}

static void matmul3(const double A[9], const double B[9], double C[9]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

static void transpose3(const double A[9], double At[9]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) At[3 * j + i] = A[3 * i + j];
}

static double dot(int len, const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < len; i++) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------------ */
/* Material (paper Sec. III-A: E and nu are the skin's free parameters)      */
/* ------------------------------------------------------------------------ */
void orc_lame(double E, double nu, double *mu, double *lam) {
    *mu = E / (2.0 * (1.0 + nu));
    *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

/* Neo-Hookean strain energy density (the law of the paper's validated skin
 * model, Sec. III-A; compressible form). +inf when J <= 0. */
double orc_psi(const double F[9], double mu, double lam) {
    double J = det3(F);
    if (!(J > 0.0)) return INFINITY;
    double I1 = 0.0;
    for (int i = 0; i < 9; i++) I1 += F[i] * F[i];
    double lnJ = log(J);
    return 0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
}

/* First Piola-Kirchhoff stress P = dPsi/dF = mu (F - F^-T) + lam ln J F^-T. */
void orc_pk1(const double F[9], double mu, double lam, double P[9]) {
    double Fi[9], FiT[9];
    double J = inv3(F, Fi);
    transpose3(Fi, FiT);
    double lnJ = log(J);
    for (int i = 0; i < 9; i++) P[i] = mu * (F[i] - FiT[i]) + lam * lnJ * FiT[i];
}

/* Directional derivative of P:
 * dP = mu dF + (mu - lam ln J) F^-T dF^T F^-T + lam tr(F^-1 dF) F^-T. */
void orc_dpk1(const double F[9], const double dF[9], double mu, double lam, double dP[9]) {
    double Fi[9], FiT[9], dFT[9], t1[9], t2[9], t3[9];
    double J = inv3(F, Fi);
    transpose3(Fi, FiT);
    transpose3(dF, dFT);
    double lnJ = log(J);
    matmul3(FiT, dFT, t1);
    matmul3(t1, FiT, t2);
    matmul3(Fi, dF, t3);
    double tr = t3[0] + t3[4] + t3[8];
    for (int i = 0; i < 9; i++)
        dP[i] = mu * dF[i] + (mu - lam * lnJ) * t2[i] + lam * tr * FiT[i];
}

/* ------------------------------------------------------------------------ */
/* Co-rotational linear elasticity (the constitutive model of the paper's    */
/* own simulator, Sec. III-A): with the polar decomposition F = R S,          */
/*   Psi = mu |F - R|^2 + lam/2 (tr S - 3)^2,                                 */
/*   P = 2 mu (F - R) + lam (tr S - 3) R.                                     */
/* ------------------------------------------------------------------------ */

/* Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations:
 * A = V diag(w) V^T, V's columns the eigenvectors. */
static void sym_eig3(const double A[9], double w[3], double V[9]) {
    double a[9];
    memcpy(a, A, sizeof a);
    for (int i = 0; i < 9; i++) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
        double dia = a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
        if (off <= 1e-34 * dia) break;
        static const int PQ[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (int r = 0; r < 3; r++) {
            int p = PQ[r][0], q = PQ[r][1];
            double apq = a[3 * p + q];
            if (apq == 0.0) continue;
            double theta = (a[3 * q + q] - a[3 * p + p]) / (2.0 * apq);
            double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
            /* a <- J^T a J with J the rotation in the (p, q) plane */
            for (int k = 0; k < 3; k++) {
                double akp = a[3 * k + p], akq = a[3 * k + q];
                a[3 * k + p] = c * akp - sn * akq;
                a[3 * k + q] = sn * akp + c * akq;
            }
            for (int k = 0; k < 3; k++) {
                double apk = a[3 * p + k], aqk = a[3 * q + k];
                a[3 * p + k] = c * apk - sn * aqk;
                a[3 * q + k] = sn * apk + c * aqk;
            }
            for (int k = 0; k < 3; k++) {
                double vkp = V[3 * k + p], vkq = V[3 * k + q];
                V[3 * k + p] = c * vkp - sn * vkq;
                V[3 * k + q] = sn * vkp + c * vkq;
            }
        }
    }
    w[0] = a[0];
    w[1] = a[4];
    w[2] = a[8];
}

int orc_polar(const double F[9], double R[9], double S[9]) {
    double C[9], w[3], V[9], Si[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) C[3 * i + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
    sym_eig3(C, w, V);
    if (!(w[0] > 0.0 && w[1] > 0.0 && w[2] > 0.0)) return -1;
    double sq[3] = {sqrt(w[0]), sqrt(w[1]), sqrt(w[2])};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0, si = 0.0;
            for (int k = 0; k < 3; k++) {
                s += V[3 * i + k] * sq[k] * V[3 * j + k];
                si += V[3 * i + k] / sq[k] * V[3 * j + k];
            }
            S[3 * i + j] = s;
            Si[3 * i + j] = si;
        }
    matmul3(F, Si, R);
    return det3(F) > 0.0 ? 0 : -1;
}

double orc_psi_cr(const double F[9], double mu, double lam) {
    double R[9], S[9];
    if (orc_polar(F, R, S) != 0) return INFINITY;
    double d2 = 0.0;
    for (int i = 0; i < 9; i++) d2 += (F[i] - R[i]) * (F[i] - R[i]);
    double e = S[0] + S[4] + S[8] - 3.0;
    return mu * d2 + 0.5 * lam * e * e;
}

void orc_pk1_cr(const double F[9], double mu, double lam, double P[9]) {
    double R[9], S[9];
    orc_polar(F, R, S);
    double e = S[0] + S[4] + S[8] - 3.0;
    for (int i = 0; i < 9; i++) P[i] = 2.0 * mu * (F[i] - R[i]) + lam * e * R[i];
}

/* dR = R W with W = [w]x skew: symmetry of d(R^T F) gives
 * (tr S I - S) w = axial(R^T dF - dF^T R), axial(K) = (K_21, K_02, K_10). */
void orc_dpk1_cr(const double F[9], const double dF[9], double mu, double lam, double dP[9]) {
    double R[9], S[9], RT[9], M[9], K[9], Ki[9], dR[9];
    orc_polar(F, R, S);
    transpose3(R, RT);
    matmul3(RT, dF, M);
    double a[3] = {M[7] - M[5], M[2] - M[6], M[3] - M[1]};
    double trS = S[0] + S[4] + S[8];
    for (int i = 0; i < 9; i++) K[i] = -S[i];
    K[0] += trS;
    K[4] += trS;
    K[8] += trS;
    inv3(K, Ki);
    double w[3];
    for (int i = 0; i < 3; i++) w[i] = Ki[3 * i] * a[0] + Ki[3 * i + 1] * a[1] + Ki[3 * i + 2] * a[2];
    double W[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    matmul3(R, W, dR);
    double trM = M[0] + M[4] + M[8];
    for (int i = 0; i < 9; i++)
        dP[i] = 2.0 * mu * (dF[i] - dR[i]) + lam * trM * R[i] + lam * (trS - 3.0) * dR[i];
}

/* 9x9 tangent A[(i,j),(k,l)] = dP_ij / dF_kl, column by column from dP, for
 * the problem's law. */
static void dpdf_law(int model, const double F[9], double mu, double lam, double A[81]) {
    for (int kl = 0; kl < 9; kl++) {
        double dF[9] = {0}, dP[9];
        dF[kl] = 1.0;
        if (model == ORC_COROTATIONAL)
            orc_dpk1_cr(F, dF, mu, lam, dP);
        else
            orc_dpk1(F, dF, mu, lam, dP);
        for (int ij = 0; ij < 9; ij++) A[ij * 9 + kl] = dP[ij];
    }
}

/* ------------------------------------------------------------------------ */
/* Indenter signed distances (rigid indenters driven into the skin, Sec.     */
/* III-A; sphere, cylinder, box and ring families as in Sec. IV-A).          */
/* Tie-breaks at the medial axis: the largest face distance wins, equal      */
/* distances go to the lower axis (x < y < z; radial before axial).          */
/* ------------------------------------------------------------------------ */
double orc_sdf(const orc_indenter *ind, const double x[3], double grad[3]) {
    const double *R = ind->R;
    double d[3] = {x[0] - ind->c[0], x[1] - ind->c[1], x[2] - ind->c[2]};
    double q[3];
    for (int i = 0; i < 3; i++) q[i] = R[0 + i] * d[0] + R[3 + i] * d[1] + R[6 + i] * d[2];
    double gq[3] = {0.0, 0.0, 0.0};
    double phi;
    if (ind->kind == ORC_SPHERE) {
        double L = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        phi = L - ind->shape[0];
        if (L > 0.0) {
            gq[0] = q[0] / L; gq[1] = q[1] / L; gq[2] = q[2] / L;
        } else {
            gq[2] = 1.0;
        }
    } else if (ind->kind == ORC_CYLINDER) {
        double a = ind->shape[0], hh = 0.5 * ind->shape[1];
        double rho = sqrt(q[0] * q[0] + q[1] * q[1]);
        double er[3] = {1.0, 0.0, 0.0};
        if (rho > 0.0) { er[0] = q[0] / rho; er[1] = q[1] / rho; }
        double sz = q[2] >= 0.0 ? 1.0 : -1.0;
        double dr = rho - a, dz = fabs(q[2]) - hh;
        if (dr > 0.0 && dz > 0.0) {
            phi = sqrt(dr * dr + dz * dz);
            gq[0] = dr * er[0] / phi; gq[1] = dr * er[1] / phi; gq[2] = dz * sz / phi;
        } else if (dr > 0.0) {
            phi = dr; gq[0] = er[0]; gq[1] = er[1];
        } else if (dz > 0.0) {
            phi = dz; gq[2] = sz;
        } else if (dr >= dz) {
            phi = dr; gq[0] = er[0]; gq[1] = er[1];
        } else {
            phi = dz; gq[2] = sz;
        }
    } else if (ind->kind == ORC_BOX) {
        double dd[3], s[3], o[3], on = 0.0;
        int outside = 0;
        for (int i = 0; i < 3; i++) {
            s[i] = q[i] >= 0.0 ? 1.0 : -1.0;
            dd[i] = fabs(q[i]) - ind->shape[i];
            o[i] = dd[i] > 0.0 ? dd[i] : 0.0;
            if (dd[i] > 0.0) outside = 1;
            on += o[i] * o[i];
        }
        if (outside) {
            phi = sqrt(on);
            for (int i = 0; i < 3; i++) gq[i] = s[i] * o[i] / phi;
        } else {
            int j = 0;
            for (int i = 1; i < 3; i++) if (dd[i] > dd[j]) j = i;
            phi = dd[j];
            gq[j] = s[j];
        }
    } else { /* ORC_RING: torus around the local z axis */
        double Rm = ind->shape[0], rm = ind->shape[1];
        double rho = sqrt(q[0] * q[0] + q[1] * q[1]);
        double er[3] = {1.0, 0.0, 0.0};
        if (rho > 0.0) { er[0] = q[0] / rho; er[1] = q[1] / rho; }
        double w[3] = {(rho - Rm) * er[0], (rho - Rm) * er[1], q[2]};
        double L = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        phi = L - rm;
        if (L > 0.0) {
            gq[0] = w[0] / L; gq[1] = w[1] / L; gq[2] = w[2] / L;
        } else {
            gq[2] = 1.0;
        }
    }
    for (int i = 0; i < 3; i++) grad[i] = R[3 * i + 0] * gq[0] + R[3 * i + 1] * gq[1] + R[3 * i + 2] * gq[2];
    return phi;
}


/* Hessian of the signed distance in the world frame, needed only where
 * phi < 0 (inside the indenter): sphere (I - n n^T)/|q|; cylinder side
 * e_t e_t^T / rho (flat faces: 0); box 0; ring t t^T/|w| + (n_rho/rho) e_t e_t^T
 * with t the in-meridian tangent and e_t the hoop direction. */
static void sdf_hessian(const orc_indenter *ind, const double x[3], double Hw[9]) {
    const double *R = ind->R;
    double d[3] = {x[0] - ind->c[0], x[1] - ind->c[1], x[2] - ind->c[2]};
    double q[3];
    for (int i = 0; i < 3; i++) q[i] = R[0 + i] * d[0] + R[3 + i] * d[1] + R[6 + i] * d[2];
    double Hq[9] = {0};
    if (ind->kind == ORC_SPHERE) {
        double L = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        if (L > 0.0)
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) Hq[3 * i + j] = ((i == j ? 1.0 : 0.0) - q[i] * q[j] / (L * L)) / L;
    } else if (ind->kind == ORC_CYLINDER) {
        double a = ind->shape[0], hh = 0.5 * ind->shape[1];
        double rho = sqrt(q[0] * q[0] + q[1] * q[1]);
        double dr = rho - a, dz = fabs(q[2]) - hh;
        if (rho > 0.0 && dr <= 0.0 && dz <= 0.0 && dr >= dz) {
            double et[3] = {-q[1] / rho, q[0] / rho, 0.0};
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) Hq[3 * i + j] = et[i] * et[j] / rho;
        }
    } else if (ind->kind == ORC_RING) {
        double Rm = ind->shape[0];
        double rho = sqrt(q[0] * q[0] + q[1] * q[1]);
        if (rho > 0.0) {
            double er[3] = {q[0] / rho, q[1] / rho, 0.0}, et[3] = {-q[1] / rho, q[0] / rho, 0.0};
            double wr = rho - Rm, wz = q[2];
            double L = sqrt(wr * wr + wz * wz);
            if (L > 0.0) {
                double t[3] = {-wz / L * er[0], -wz / L * er[1], wr / L};
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) Hq[3 * i + j] = t[i] * t[j] / L + (wr / L) / rho * et[i] * et[j];
            }
        }
    }
    /* Hw = R Hq R^T */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) s += R[3 * i + a] * Hq[3 * a + b] * R[3 * j + b];
            Hw[3 * i + j] = s;
        }
}

/* ------------------------------------------------------------------------ */
/* Mesh precompute                                                          */
/* ------------------------------------------------------------------------ */
int orc_precompute(int n, const double *X, int m, const int *T, double *B, double *V) {
    (void)n;
    for (int e = 0; e < m; e++) {
        const double *x0 = X + 3 * T[4 * e];
        double Dm[9];
        for (int a = 0; a < 3; a++) {
            const double *xa = X + 3 * T[4 * e + 1 + a];
            for (int i = 0; i < 3; i++) Dm[3 * i + a] = xa[i] - x0[i];
        }
        double det = inv3(Dm, B + 9 * e);
        V[e] = det / 6.0;
        if (!(V[e] > 0.0)) return -(1 + e);
    }
    return 0;
}

static int cmp_face(const void *a, const void *b) {
    const int *x = (const int *)a, *y = (const int *)b;
    for (int i = 0; i < 3; i++)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

int orc_surface_nodes(int n, int m, const int *T, unsigned char *surf) {
    static const int fv[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    int *faces = (int *)malloc(sizeof(int) * 12 * (size_t)m);
    for (int e = 0; e < m; e++)
        for (int f = 0; f < 4; f++) {
            int v[3] = {T[4 * e + fv[f][0]], T[4 * e + fv[f][1]], T[4 * e + fv[f][2]]};
            /* sort the three ids */
            for (int i = 0; i < 2; i++)
                for (int j = 0; j < 2 - i; j++)
                    if (v[j] > v[j + 1]) { int t = v[j]; v[j] = v[j + 1]; v[j + 1] = t; }
            memcpy(faces + 3 * (4 * (size_t)e + f), v, sizeof v);
        }
    qsort(faces, 4 * (size_t)m, 3 * sizeof(int), cmp_face);
    memset(surf, 0, (size_t)n);
    int nb = 0;
    for (size_t i = 0; i < 4 * (size_t)m;) {
        size_t j = i + 1;
        while (j < 4 * (size_t)m && cmp_face(faces + 3 * i, faces + 3 * j) == 0) j++;
        if (j - i == 1) {
            nb++;
            for (int k = 0; k < 3; k++) surf[faces[3 * i + k]] = 1;
        }
        i = j;
    }
    free(faces);
    return nb;
}

/* ------------------------------------------------------------------------ */
/* Element kinematics: F = D_s D_m^-1 with D_s the deformed edge matrix.     */
/* ------------------------------------------------------------------------ */
void orc_deformation_gradient(const orc_problem *p, const double *u, int e, double F[9]) {
    const int *t = p->T + 4 * e;
    double Ds[9];
    double x0[3];
    for (int i = 0; i < 3; i++) x0[i] = p->X[3 * t[0] + i] + u[3 * t[0] + i];
    for (int a = 0; a < 3; a++)
        for (int i = 0; i < 3; i++)
            Ds[3 * i + a] = (p->X[3 * t[1 + a] + i] + u[3 * t[1 + a] + i]) - x0[i];
    matmul3(Ds, p->B + 9 * e, F);
}

/* Shape-function gradients b_a (rows of D_m^-1 for a = 1..3, b_0 = -sum). */
static void shape_grads(const double *B, double b[4][3]) {
    for (int a = 0; a < 3; a++)
        for (int j = 0; j < 3; j++) b[a + 1][j] = B[3 * a + j];
    for (int j = 0; j < 3; j++) b[0][j] = -(b[1][j] + b[2][j] + b[3][j]);
}

/* Backward Euler's inertial term is present (dt > 0 with masses and predictor). */
static int dynamic(const orc_problem *p) { return p->dt > 0.0 && p->mass && p->utilde; }

void orc_lumped_mass(int n, int m, const int *T, const double *V, double rho, double *mass) {
    memset(mass, 0, sizeof(double) * (size_t)n);
    for (int e = 0; e < m; e++)
        for (int a = 0; a < 4; a++) mass[T[4 * e + a]] += rho * V[e] / 4.0;
}

static double contact_phi(const orc_problem *p, const double *u, int i, double nrm[3]) {
    double x[3] = {p->X[3 * i] + u[3 * i], p->X[3 * i + 1] + u[3 * i + 1], p->X[3 * i + 2] + u[3 * i + 2]};
    return orc_sdf(&p->ind, x, nrm);
}

/* ------------------------------------------------------------------------ */
/* Lagged, smoothed Coulomb friction                                         */
/* ------------------------------------------------------------------------ */
void orc_friction_f0(double y, double eps, double *f0, double *f1, double *df1) {
    if (y < eps) {
        *f0 = y * y / eps - y * y * y / (3.0 * eps * eps) + eps / 3.0;
        *f1 = 2.0 * y / eps - y * y / (eps * eps);
        *df1 = 2.0 / eps - 2.0 * y / (eps * eps);
    } else {
        *f0 = y;
        *f1 = 1.0;
        *df1 = 0.0;
    }
}

/* Friction data of node i at u: returns 1 when the node carries friction
 * (eligible, lag state present, in contact at the lag state), with its
 * weight w = mu_f k (-phi_lag), lag normal and tangential slip s. */
static int friction_at(const orc_problem *p, const double *u, int i, double *w, double nrm[3], double s[3]) {
    if (!(p->mu_f > 0.0) || !p->u_lag || !p->eligible[i]) return 0;
    orc_indenter lag = p->ind;
    for (int d = 0; d < 3; d++) lag.c[d] = p->c_lag[d];
    double xl[3];
    for (int d = 0; d < 3; d++) xl[d] = p->X[3 * i + d] + p->u_lag[3 * i + d];
    double phl = orc_sdf(&lag, xl, nrm);
    if (!(phl < 0.0)) return 0;
    *w = p->mu_f * p->ind.k * (-phl);
    double dd[3];
    for (int d = 0; d < 3; d++) dd[d] = u[3 * i + d] - p->u_lag[3 * i + d] - (p->ind.c[d] - p->c_lag[d]);
    double dn = dd[0] * nrm[0] + dd[1] * nrm[1] + dd[2] * nrm[2];
    for (int d = 0; d < 3; d++) s[d] = dd[d] - dn * nrm[d];
    return 1;
}

/* Friction energy of node i and its gradient (either may be NULL). */
static double friction_energy_grad(const orc_problem *p, const double *u, int i, double g[3]) {
    double w, nrm[3], s[3];
    if (g) g[0] = g[1] = g[2] = 0.0;
    if (!friction_at(p, u, i, &w, nrm, s)) return 0.0;
    double y = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]), f0, f1, df1;
    orc_friction_f0(y, p->eps_f, &f0, &f1, &df1);
    if (g && y > 0.0)
        for (int d = 0; d < 3; d++) g[d] = w * f1 / y * s[d];
    return w * f0;
}

/* Friction block of node i: w [ (f1/y) P + (f1' - f1/y) s s^T / y^2 ] with
 * P = I - n n^T (the limit 2w/eps P at y = 0). */
static void friction_block(const orc_problem *p, const double *u, int i, double Hb[9]) {
    double w, nrm[3], s[3];
    for (int c = 0; c < 9; c++) Hb[c] = 0.0;
    if (!friction_at(p, u, i, &w, nrm, s)) return;
    double y = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]), f0, f1, df1;
    orc_friction_f0(y, p->eps_f, &f0, &f1, &df1);
    double a = y > 0.0 ? f1 / y : 2.0 / p->eps_f;
    double b = y > 0.0 ? (df1 - f1 / y) / (y * y) : 0.0;
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            Hb[3 * r + c] = w * (a * ((r == c ? 1.0 : 0.0) - nrm[r] * nrm[c]) + b * s[r] * s[c]);
}

/* Energy, with the sum of the magnitudes of its terms (for the line search's
 * rounding floor) and the smallest J. */
static double energy_terms(const orc_problem *p, const double *u, double *mag, double *min_J) {
    double E = 0.0, M = 0.0, mj = INFINITY;
    for (int e = 0; e < p->m; e++) {
        double F[9];
        orc_deformation_gradient(p, u, e, F);
        double J = det3(F);
        if (J < mj) mj = J;
        if (!(J > 0.0)) {
            E = INFINITY;
            continue;
        }
        double I1 = 0.0;
        for (int i = 0; i < 9; i++) I1 += F[i] * F[i];
        if (p->model == ORC_COROTATIONAL) {
            double R[9], S[9];
            orc_polar(F, R, S);
            double d2 = 0.0;
            for (int i = 0; i < 9; i++) d2 += (F[i] - R[i]) * (F[i] - R[i]);
            double trS = S[0] + S[4] + S[8];
            E += p->V[e] * (p->mu * d2 + 0.5 * p->lam * (trS - 3.0) * (trS - 3.0));
            /* rounding scale: the operands of F - R and tr S - 3 */
            M += p->V[e] * (p->mu * (I1 + 3.0) + 0.5 * p->lam * (trS + 3.0) * (trS + 3.0));
            continue;
        }
        double lnJ = log(J);
        double t1 = 0.5 * p->mu * (I1 - 3.0), t2 = -p->mu * lnJ, t3 = 0.5 * p->lam * lnJ * lnJ;
        E += p->V[e] * (t1 + t2 + t3);
        /* Rounding scale of the three terms: I1 - 3 and ln J are formed by
         * cancellation, so their error follows the operands (I1 + 3, and 1
         * for ln J near J = 1), not the terms' own size. */
        M += p->V[e] * (0.5 * p->mu * (I1 + 3.0) + (p->mu + p->lam * fabs(lnJ)) * (1.0 + fabs(lnJ)));
    }
    for (int i = 0; i < p->n; i++) {
        if (!p->eligible[i]) continue;
        double nrm[3];
        double phi = contact_phi(p, u, i, nrm);
        if (phi < 0.0) {
            double c = 0.5 * p->ind.k * phi * phi;
            E += c;
            M += c;
        }
    }
    for (int i = 0; i < p->n; i++) {
        double c = friction_energy_grad(p, u, i, NULL);
        E += c;
        M += c;
    }
    if (dynamic(p)) {
        for (int i = 0; i < p->n; i++) {
            if (p->fixed[i]) continue;
            double d2 = 0.0;
            for (int d = 0; d < 3; d++) {
                double w = u[3 * i + d] - p->utilde[3 * i + d];
                d2 += w * w;
            }
            double c = 0.5 * p->mass[i] / (p->dt * p->dt) * d2;
            E += c;
            M += c;
        }
    }
    if (mag) *mag = M;
    if (min_J) *min_J = mj;
    return E;
}

double orc_energy(const orc_problem *p, const double *u, double *min_J) {
    return energy_terms(p, u, NULL, min_J);
}

void orc_gradient(const orc_problem *p, const double *u, double *g) {
    memset(g, 0, sizeof(double) * 3 * (size_t)p->n);
    for (int e = 0; e < p->m; e++) {
        double F[9], P[9], b[4][3];
        orc_deformation_gradient(p, u, e, F);
        if (p->model == ORC_COROTATIONAL)
            orc_pk1_cr(F, p->mu, p->lam, P);
        else
            orc_pk1(F, p->mu, p->lam, P);
        shape_grads(p->B + 9 * e, b);
        const int *t = p->T + 4 * e;
        /* dE/dx_a = V P b_a */
        for (int a = 0; a < 4; a++)
            for (int i = 0; i < 3; i++) {
                double s = 0.0;
                for (int j = 0; j < 3; j++) s += P[3 * i + j] * b[a][j];
                g[3 * t[a] + i] += p->V[e] * s;
            }
    }
    for (int i = 0; i < p->n; i++) {
        if (!p->eligible[i]) continue;
        double nrm[3];
        double phi = contact_phi(p, u, i, nrm);
        if (phi < 0.0)
            for (int d = 0; d < 3; d++) g[3 * i + d] += p->ind.k * phi * nrm[d];
        double gf[3];
        friction_energy_grad(p, u, i, gf);
        for (int d = 0; d < 3; d++) g[3 * i + d] += gf[d];
    }
    if (dynamic(p))
        for (int i = 0; i < p->n; i++) {
            if (p->fixed[i]) continue;
            for (int d = 0; d < 3; d++) g[3 * i + d] += p->mass[i] / (p->dt * p->dt) * (u[3 * i + d] - p->utilde[3 * i + d]);
        }
}

/* Element stiffness K_e[(a,i),(c,k)] = V sum_{j,l} b_a,j A[(i,j),(k,l)] b_c,l. */
static void element_hessian(const orc_problem *p, const double *u, int e, double K[144]) {
    double F[9], A[81], b[4][3];
    orc_deformation_gradient(p, u, e, F);
    dpdf_law(p->model, F, p->mu, p->lam, A);
    shape_grads(p->B + 9 * e, b);
    for (int a = 0; a < 4; a++)
        for (int i = 0; i < 3; i++)
            for (int c = 0; c < 4; c++)
                for (int k = 0; k < 3; k++) {
                    double s = 0.0;
                    for (int j = 0; j < 3; j++)
                        for (int l = 0; l < 3; l++) s += b[a][j] * A[(3 * i + j) * 9 + 3 * k + l] * b[c][l];
                    K[(3 * a + i) * 12 + 3 * c + k] = p->V[e] * s;
                }
}

/* ------------------------------------------------------------------------ */
/* Block-sparse (3x3) Hessian                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    int *rowptr; /* n+1 */
    int *col;    /* nnzb */
    double *val; /* 9 * nnzb */
} bsr;

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

static void bsr_pattern(const orc_problem *p, bsr *H) {
    int n = p->n, m = p->m;
    /* node -> incident tets */
    int *cnt = (int *)calloc((size_t)n + 1, sizeof(int));
    for (int e = 0; e < m; e++)
        for (int a = 0; a < 4; a++) cnt[p->T[4 * e + a] + 1]++;
    for (int i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    int *inc = (int *)malloc(sizeof(int) * 4 * (size_t)m);
    int *fill = (int *)calloc((size_t)n, sizeof(int));
    for (int e = 0; e < m; e++)
        for (int a = 0; a < 4; a++) {
            int v = p->T[4 * e + a];
            inc[cnt[v] + fill[v]++] = e;
        }
    H->n = n;
    H->rowptr = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int cap = 16 * n + 16, nnz = 0;
    H->col = (int *)malloc(sizeof(int) * (size_t)cap);
    int *tmp = (int *)malloc(sizeof(int) * 4 * 256);
    H->rowptr[0] = 0;
    for (int i = 0; i < n; i++) {
        int deg = cnt[i + 1] - cnt[i], k = 0;
        if (4 * deg > 4 * 256) tmp = (int *)realloc(tmp, sizeof(int) * 4 * (size_t)deg);
        for (int s = cnt[i]; s < cnt[i + 1]; s++)
            for (int a = 0; a < 4; a++) tmp[k++] = p->T[4 * inc[s] + a];
        if (deg == 0) tmp[k++] = i;
        qsort(tmp, (size_t)k, sizeof(int), cmp_int);
        for (int s = 0; s < k; s++) {
            if (s > 0 && tmp[s] == tmp[s - 1]) continue;
            if (nnz == cap) {
                cap *= 2;
                H->col = (int *)realloc(H->col, sizeof(int) * (size_t)cap);
            }
            H->col[nnz++] = tmp[s];
        }
        H->rowptr[i + 1] = nnz;
    }
    H->val = (double *)calloc(9 * (size_t)nnz, sizeof(double));
    free(tmp);
    free(fill);
    free(inc);
    free(cnt);
}

static double *bsr_block(bsr *H, int i, int j) {
    int lo = H->rowptr[i], hi = H->rowptr[i + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (H->col[mid] == j) return H->val + 9 * (size_t)mid;
        if (H->col[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return NULL;
}

static void bsr_free(bsr *H) {
    free(H->rowptr);
    free(H->col);
    free(H->val);
}

/* Exact Neo-Hookean tangent plus the contact block: Gauss-Newton k n n^T, or
 * with contact_full the exact k (n n^T + phi d2(phi)/dx2). */
static void bsr_assemble(const orc_problem *p, const double *u, bsr *H, int contact_full) {
    memset(H->val, 0, sizeof(double) * 9 * (size_t)H->rowptr[H->n]);
    for (int e = 0; e < p->m; e++) {
        double K[144];
        element_hessian(p, u, e, K);
        const int *t = p->T + 4 * e;
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 4; c++) {
                double *blk = bsr_block(H, t[a], t[c]);
                for (int i = 0; i < 3; i++)
                    for (int k = 0; k < 3; k++) blk[3 * i + k] += K[(3 * a + i) * 12 + 3 * c + k];
            }
    }
    for (int i = 0; i < p->n; i++) {
        if (!p->eligible[i]) continue;
        double nrm[3];
        double phi = contact_phi(p, u, i, nrm);
        if (phi < 0.0) {
            double *blk = bsr_block(H, i, i), Hs[9] = {0};
            if (contact_full) {
                double x[3] = {p->X[3 * i] + u[3 * i], p->X[3 * i + 1] + u[3 * i + 1], p->X[3 * i + 2] + u[3 * i + 2]};
                sdf_hessian(&p->ind, x, Hs);
            }
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) blk[3 * a + b] += p->ind.k * (nrm[a] * nrm[b] + phi * Hs[3 * a + b]);
        }
        double Hf[9];
        friction_block(p, u, i, Hf);
        double *blk = bsr_block(H, i, i);
        for (int c = 0; c < 9; c++) blk[c] += Hf[c];
    }
    if (dynamic(p))
        for (int i = 0; i < p->n; i++) {
            if (p->fixed[i]) continue;
            double *blk = bsr_block(H, i, i);
            for (int a = 0; a < 3; a++) blk[4 * a] += p->mass[i] / (p->dt * p->dt);
        }
}

static void bsr_mul(const bsr *H, const double *v, double *q) {
    for (int i = 0; i < H->n; i++) {
        double s[3] = {0.0, 0.0, 0.0};
        for (int k = H->rowptr[i]; k < H->rowptr[i + 1]; k++) {
            const double *blk = H->val + 9 * (size_t)k;
            const double *vj = v + 3 * (size_t)H->col[k];
            for (int a = 0; a < 3; a++) s[a] += blk[3 * a] * vj[0] + blk[3 * a + 1] * vj[1] + blk[3 * a + 2] * vj[2];
        }
        q[3 * i] = s[0]; q[3 * i + 1] = s[1]; q[3 * i + 2] = s[2];
    }
}

void orc_hessvec(const orc_problem *p, const double *u, const double *v, double *q, int contact_full) {
    bsr H;
    bsr_pattern(p, &H);
    bsr_assemble(p, u, &H, contact_full);
    bsr_mul(&H, v, q);
    bsr_free(&H);
}

void orc_hessian_dense(const orc_problem *p, const double *u, double *Hd, int contact_full) {
    int N = 3 * p->n;
    memset(Hd, 0, sizeof(double) * (size_t)N * (size_t)N);
    bsr H;
    bsr_pattern(p, &H);
    bsr_assemble(p, u, &H, contact_full);
    for (int i = 0; i < p->n; i++)
        for (int k = H.rowptr[i]; k < H.rowptr[i + 1]; k++)
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    Hd[(size_t)(3 * i + a) * N + 3 * H.col[k] + b] = H.val[9 * (size_t)k + 3 * a + b];
    bsr_free(&H);
}

/* ------------------------------------------------------------------------ */
/* Jacobi preconditioners                                                   */
/* ------------------------------------------------------------------------ */
static double safe_recip(double d) {
    if (d > 0.0) return 1.0 / d;
    if (d < 0.0) return 1.0 / -d;
    return 1.0;
}

/* Minv: n x 9. Block Jacobi inverts each free node's 3x3 diagonal block when
 * it is positive definite (leading minors > 0); otherwise, and for scalar
 * Jacobi, it is diag(1/|d_ii|). Fixed nodes get 0. */
static void build_precond(const orc_problem *p, bsr *H, int block, double *Minv) {
    for (int i = 0; i < p->n; i++) {
        double *M = Minv + 9 * (size_t)i;
        memset(M, 0, 9 * sizeof(double));
        if (p->fixed[i]) continue;
        const double *D = bsr_block(H, i, i);
        double m1 = D[0], m2 = D[0] * D[4] - D[1] * D[3], m3 = det3(D);
        if (block && m1 > 0.0 && m2 > 0.0 && m3 > 0.0) {
            inv3(D, M);
        } else {
            M[0] = safe_recip(D[0]);
            M[4] = safe_recip(D[4]);
            M[8] = safe_recip(D[8]);
        }
    }
}

static void apply_precond(int n, const double *Minv, const double *r, double *z) {
    for (int i = 0; i < n; i++) {
        const double *M = Minv + 9 * (size_t)i;
        const double *ri = r + 3 * (size_t)i;
        for (int a = 0; a < 3; a++) z[3 * i + a] = M[3 * a] * ri[0] + M[3 * a + 1] * ri[1] + M[3 * a + 2] * ri[2];
    }
}

static void mask_fixed(const orc_problem *p, double *v) {
    for (int i = 0; i < p->n; i++)
        if (p->fixed[i]) v[3 * i] = v[3 * i + 1] = v[3 * i + 2] = 0.0;
}

/* ------------------------------------------------------------------------ */
/* Linear solves on the free nodes                                          */
/* ------------------------------------------------------------------------ */
/* Preconditioned CG, textbook form, stopped when |r| <= rtol |r_0|, or at the
 * first direction with p^T H p <= 0 (then the current iterate is returned, or
 * the preconditioned residual if that happens on the first iteration). */
static int pcg(const orc_problem *p, bsr *H, const double *b, double *x, const orc_params *prm, double rtol,
               int *hv) {
    int N = 3 * p->n;
    double *r = (double *)malloc(sizeof(double) * N), *z = (double *)malloc(sizeof(double) * N);
    double *d = (double *)malloc(sizeof(double) * N), *q = (double *)malloc(sizeof(double) * N);
    double *Minv = (double *)malloc(sizeof(double) * 9 * (size_t)p->n);
    build_precond(p, H, prm->precond, Minv);
    memset(x, 0, sizeof(double) * N);
    memcpy(r, b, sizeof(double) * N);
    mask_fixed(p, r);
    apply_precond(p->n, Minv, r, z);
    memcpy(d, z, sizeof(double) * N);
    double rz = dot(N, r, z);
    double r0 = sqrt(dot(N, r, r));
    int it = 0;
    if (r0 > 0.0) {
        for (it = 0; it < prm->max_cg;) {
            bsr_mul(H, d, q);
            mask_fixed(p, q);
            (*hv)++;
            double dq = dot(N, d, q);
            if (!(dq > 0.0)) {
                if (it == 0) memcpy(x, d, sizeof(double) * N);
                break;
            }
            double alpha = rz / dq;
            for (int k = 0; k < N; k++) {
                x[k] += alpha * d[k];
                r[k] -= alpha * q[k];
            }
            it++;
            if (sqrt(dot(N, r, r)) <= rtol * r0) break;
            apply_precond(p->n, Minv, r, z);
            double rz_new = dot(N, r, z);
            double beta = rz_new / rz;
            rz = rz_new;
            for (int k = 0; k < N; k++) d[k] = z[k] + beta * d[k];
        }
    }
    free(r); free(z); free(d); free(q); free(Minv);
    return it;
}

/* Dense Cholesky of the free-node block (tiny meshes only). */
static int dense_solve(const orc_problem *p, bsr *H, const double *b, double *x) {
    int n = p->n;
    int *map = (int *)malloc(sizeof(int) * 3 * (size_t)n);
    int N = 0;
    for (int i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) map[3 * i + a] = p->fixed[i] ? -1 : N++;
    double *A = (double *)calloc((size_t)N * N, sizeof(double));
    double *y = (double *)malloc(sizeof(double) * (N > 0 ? N : 1));
    for (int i = 0; i < n; i++)
        for (int k = H->rowptr[i]; k < H->rowptr[i + 1]; k++)
            for (int a = 0; a < 3; a++)
                for (int c = 0; c < 3; c++) {
                    int r = map[3 * i + a], s = map[3 * H->col[k] + c];
                    if (r >= 0 && s >= 0) A[(size_t)r * N + s] = H->val[9 * (size_t)k + 3 * a + c];
                }
    int ok = 1;
    for (int j = 0; j < N && ok; j++) {
        double s = A[(size_t)j * N + j];
        for (int k = 0; k < j; k++) s -= A[(size_t)j * N + k] * A[(size_t)j * N + k];
        if (!(s > 0.0)) { ok = 0; break; }
        double L = sqrt(s);
        A[(size_t)j * N + j] = L;
        for (int i = j + 1; i < N; i++) {
            double t = A[(size_t)i * N + j];
            for (int k = 0; k < j; k++) t -= A[(size_t)i * N + k] * A[(size_t)j * N + k];
            A[(size_t)i * N + j] = t / L;
        }
    }
    if (ok) {
        for (int i = 0; i < n; i++)
            for (int a = 0; a < 3; a++)
                if (map[3 * i + a] >= 0) y[map[3 * i + a]] = b[3 * i + a];
        for (int i = 0; i < N; i++) {
            double t = y[i];
            for (int k = 0; k < i; k++) t -= A[(size_t)i * N + k] * y[k];
            y[i] = t / A[(size_t)i * N + i];
        }
        for (int i = N - 1; i >= 0; i--) {
            double t = y[i];
            for (int k = i + 1; k < N; k++) t -= A[(size_t)k * N + i] * y[k];
            y[i] = t / A[(size_t)i * N + i];
        }
        for (int i = 0; i < 3 * n; i++) x[i] = map[i] >= 0 ? y[map[i]] : 0.0;
    }
    free(map); free(A); free(y);
    return ok ? 0 : ORC_NOT_SPD;
}

int orc_linear_solve(const orc_problem *p, const double *u, const double *b, double *x, const orc_params *prm,
                     double rtol) {
    bsr H;
    bsr_pattern(p, &H);
    bsr_assemble(p, u, &H, prm->contact_hessian);
    int hv = 0, ret;
    if (prm->dense)
        ret = dense_solve(p, &H, b, x);
    else
        ret = pcg(p, &H, b, x, prm, rtol, &hv);
    bsr_free(&H);
    return ret;
}

/* ------------------------------------------------------------------------ */
/* One quasi-static load step                                               */
/* ------------------------------------------------------------------------ */
int orc_step(const orc_problem *p, const orc_params *prm, double *u, orc_info *info) {
    int N = 3 * p->n;
    double *g = (double *)malloc(sizeof(double) * N), *b = (double *)malloc(sizeof(double) * N);
    double *dx = (double *)malloc(sizeof(double) * N), *ut = (double *)malloc(sizeof(double) * N);
    bsr H;
    bsr_pattern(p, &H);
    memset(info, 0, sizeof *info);
    int status = ORC_NOT_CONVERGED;
    double r0 = 0.0, mag, minJ;
    double E = energy_terms(p, u, &mag, &minJ);
    info->energy_passes++;
    for (int it = 0;; it++) {
        orc_gradient(p, u, g);
        info->grad_passes++;
        mask_fixed(p, g);
        double gn = sqrt(dot(N, g, g));
        if (it == 0) { r0 = gn; info->g0_norm = gn; }
        info->g_norm = gn;
        if (gn <= fmax(prm->newton_rtol * r0, prm->newton_atol)) { status = ORC_OK; break; }
        if (it == prm->max_newton) { status = ORC_NOT_CONVERGED; break; }
        /* Inexact Newton: CG tolerance follows the residual reduction. */
        double eta = gn / r0;
        if (eta > prm->cg_eta_max) eta = prm->cg_eta_max;
        if (eta < prm->cg_rtol) eta = prm->cg_rtol;
        bsr_assemble(p, u, &H, prm->contact_hessian);
        for (int k = 0; k < N; k++) b[k] = -g[k];
        int hv = 0;
        if (prm->dense) {
            if (dense_solve(p, &H, b, dx) != 0) { status = ORC_NOT_SPD; break; }
        } else {
            info->cg_iters += pcg(p, &H, b, dx, prm, eta, &hv);
            info->hv_products += hv;
        }
        double gd = dot(N, g, dx);
        double noise = 16.0 * DBL_EPSILON * mag;
        double alpha = 1.0, Et = 0.0, magt = 0.0, mjt = 0.0;
        int accepted = 0;
        for (int h = 0; h <= prm->max_halvings; h++) {
            for (int k = 0; k < N; k++) ut[k] = u[k] + alpha * dx[k];
            Et = energy_terms(p, ut, &magt, &mjt);
            info->energy_passes++;
            info->ls_trials++;
            if (mjt > 0.0 && Et <= E + prm->c1 * alpha * gd + noise) { accepted = 1; break; }
            alpha *= 0.5;
        }
        if (!accepted) { status = mjt > 0.0 ? ORC_NOT_CONVERGED : ORC_INVERSION; break; }
        memcpy(u, ut, sizeof(double) * N);
        E = Et; mag = magt; minJ = mjt;
        info->newton_iters++;
    }
    info->status = status;
    info->energy = E;
    info->min_J = minJ;
    bsr_free(&H);
    free(g); free(b); free(dx); free(ut);
    return status;
}

int orc_contact_patch(const orc_problem *p, const double *u, int *ids, double *f, double *phi, double F_total[3]) {
    int count = 0;
    double Ft[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < p->n; i++) {
        if (!p->eligible[i]) continue;
        double nrm[3], wf, nf[3], sf[3], gf[3];
        double ph = contact_phi(p, u, i, nrm);
        int fr = friction_at(p, u, i, &wf, nf, sf);
        if (!(ph < 0.0) && !fr) continue;
        friction_energy_grad(p, u, i, gf);
        double fi[3];
        for (int d = 0; d < 3; d++) {
            fi[d] = (ph < 0.0 ? -p->ind.k * ph * nrm[d] : 0.0) - gf[d];
            Ft[d] += fi[d];
        }
        if (ids) ids[count] = i;
        if (f) memcpy(f + 3 * (size_t)count, fi, sizeof fi);
        if (phi) phi[count] = ph;
        count++;
    }
    if (F_total) memcpy(F_total, Ft, sizeof Ft);
    return count;
}

/* ------------------------------------------------------------------------ */
/* Outputs for data generation: per-tet Cauchy stress and von Mises stress,
 * and the displacement-norm statistics the paper reports per indentation. */
static void cauchy_from_pk1(const double F[9], const double P[9], double sigma[6], double *vm) {
    double S[9];
    double J = det3(F);
    /* sigma = P F^T / J */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += P[3 * i + k] * F[3 * j + k];
            S[3 * i + j] = s / J;
        }
    sigma[0] = S[0];
    sigma[1] = S[4];
    sigma[2] = S[8];
    sigma[3] = 0.5 * (S[1] + S[3]);
    sigma[4] = 0.5 * (S[2] + S[6]);
    sigma[5] = 0.5 * (S[5] + S[7]);
    if (vm) {
        double a = sigma[0] - sigma[1], b = sigma[1] - sigma[2], c = sigma[2] - sigma[0];
        *vm = sqrt(0.5 * (a * a + b * b + c * c) + 3.0 * (sigma[3] * sigma[3] + sigma[4] * sigma[4] + sigma[5] * sigma[5]));
    }
}

void orc_cauchy(const double F[9], double mu, double lam, double sigma[6], double *vm) {
    double P[9];
    orc_pk1(F, mu, lam, P);
    cauchy_from_pk1(F, P, sigma, vm);
}

void orc_tet_stress(const orc_problem *p, const double *u, double *sigma, double *vm) {
    for (int e = 0; e < p->m; e++) {
        double F[9], s[6], v;
        orc_deformation_gradient(p, u, e, F);
        if (p->model == ORC_COROTATIONAL) {
            double P[9];
            orc_pk1_cr(F, p->mu, p->lam, P);
            cauchy_from_pk1(F, P, s, &v);
        } else {
            orc_cauchy(F, p->mu, p->lam, s, &v);
        }
        if (sigma)
            for (int c = 0; c < 6; c++) sigma[6 * (size_t)e + c] = s[c];
        if (vm) vm[e] = v;
    }
}

void orc_displacement_stats(int n, const double *u, double *max_norm, double *mean_norm) {
    double mx = 0.0, sum = 0.0;
    for (int i = 0; i < n; i++) {
        double a = sqrt(u[3 * i] * u[3 * i] + u[3 * i + 1] * u[3 * i + 1] + u[3 * i + 2] * u[3 * i + 2]);
        if (a > mx) mx = a;
        sum += a;
    }
    *max_norm = mx;
    *mean_norm = n > 0 ? sum / n : 0.0;
}
