/*
 * FP64 CPU oracle for the quasi-static Neo-Hookean indentation solve.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, plain reference that the
 * device path is checked against. It shares no code, header, table or helper
 * with the device library and must never be linked into, or called by, the
 * product path; only tests, the smoke check and the CPU-baseline timing of the
 * benchmark use it.
 *
 * Problem (paper Sec. III-A, with readings where the paper is silent):
 * linear tetrahedral FEM of a hyperelastic skin (the compressible Neo-Hookean
 * law that the paper's validated model uses), fixed boundary nodes, and rigid
 * indenters pushed into the skin; contact is a frictionless node-vs-signed-
 * distance penalty. Each load step finds a stationary point of
 *   Pi(u) = sum_e V_e Psi(F_e(u)) + sum_{i eligible} k/2 min(0, phi(X_i+u_i))^2
 * with the displacement of fixed nodes held at its current value.
 *
 * Implicit dynamics (the paper's simulator integrates the skin in time,
 * Sec. III-A): with a time step dt > 0 and lumped nodal masses m_i, a step
 * of backward Euler minimises the incremental potential
 *   Phi(u) = Pi(u) + sum_{i free} m_i / (2 dt^2) |u_i - ut_i|^2,
 * ut = u^n + dt v^n, and then v^{n+1} = (u^{n+1} - u^n) / dt.
 *
 * Coulomb friction (the paper's simulator uses friction coefficient 0.783,
 * Sec. III-A), lagged and smoothed so that each step stays a minimisation:
 * the normal force and normal of every contact node are taken from a lag
 * state (u_lag at indenter centre c_lag, normally the previous step's
 * result), w_i = mu_f k max(0, -phi_lag_i); the node's slip relative to the
 * indenter's translation since the lag state is s_i = (I - n_i n_i^T)
 * (u_i - u_lag_i - (c - c_lag)), and the step adds
 *   D(u) = sum_i w_i f0(|s_i|),
 * f0(y) = y^2/eps - y^3/(3 eps^2) + eps/3 for y < eps and y beyond: a C1
 * smoothing of |s| whose derivative rises from 0 to 1 over a slip of eps
 * (the smoothing of Li et al., "Incremental Potential Contact", 2020). The
 * friction force on a node is then at most w_i, and exactly w_i against the
 * slip once |s_i| >= eps.
 *
 * All arrays are row-major, caller-owned, double precision unless stated.
 */
#ifndef FEM_ORACLE_H
#define FEM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_SPHERE = 0, ORC_CYLINDER = 1, ORC_BOX = 2, ORC_RING = 3 };

/* Constitutive law: compressible Neo-Hookean (the paper's validated skin
 * model) or co-rotational linear elasticity (its simulator's model). */
enum { ORC_NEOHOOKEAN = 0, ORC_COROTATIONAL = 1 };

enum {
    ORC_OK = 0,
    ORC_NOT_CONVERGED = -6,
    ORC_INVERSION = -7,
    ORC_BAD_INPUT = -1,
    ORC_DEGENERATE = -2,
    ORC_NOT_SPD = -9
};

typedef struct {
    int kind;          /* ORC_SPHERE .. ORC_RING */
    double shape[4];   /* sphere: r; cylinder: radius, height; box: hx,hy,hz; ring: Rmaj, rmin */
    double R[9];       /* rotation, row-major; local frame -> world: x = R q + c */
    double c[3];       /* centre */
    double k;          /* penalty stiffness, N/m per node */
} orc_indenter;

typedef struct {
    int n, m;
    const double *X;              /* n x 3 rest positions */
    const int *T;                 /* m x 4 node ids */
    const unsigned char *fixed;   /* n: 1 = displacement prescribed */
    const unsigned char *eligible;/* n: 1 = contact-eligible (surface, not fixed) */
    const double *B;              /* m x 9: inverse rest edge matrix, row-major */
    const double *V;              /* m: rest volumes */
    double mu, lam;               /* Lame parameters */
    orc_indenter ind;
    double dt;                    /* time step (s); 0 = quasi-static */
    const double *mass;           /* n lumped nodal masses (kg), or NULL */
    const double *utilde;         /* n x 3 inertial predictor u^n + dt v^n, or NULL */
    int model;                    /* ORC_NEOHOOKEAN or ORC_COROTATIONAL */
    double mu_f;                  /* Coulomb friction coefficient; 0 = frictionless */
    double eps_f;                 /* slip smoothing length (m), > 0 when mu_f > 0 */
    const double *u_lag;          /* n x 3 displacement of the lag state, or NULL (no friction) */
    double c_lag[3];              /* indenter centre of the lag state */
} orc_problem;

typedef struct {
    double newton_rtol;   /* stop when |g_free| <= max(newton_rtol*r0, newton_atol) */
    double newton_atol;
    int max_newton;
    double cg_rtol;       /* lower bound of the CG forcing term */
    double cg_eta_max;    /* upper bound of the CG forcing term */
    int max_cg;
    int precond;          /* 0 = scalar Jacobi, 1 = 3x3 block Jacobi */
    double c1;            /* Armijo constant */
    int max_halvings;
    int dense;            /* 1: dense Cholesky instead of PCG (tiny meshes) */
    int contact_hessian;  /* 0: Gauss-Newton k n n^T; 1: exact k (n n^T + phi Hess(phi)) */
} orc_params;

typedef struct {
    int status;
    int newton_iters;
    int cg_iters;
    int ls_trials;
    int grad_passes;      /* gradient evaluations */
    int energy_passes;    /* energy-only evaluations (line-search trials) */
    int hv_products;      /* Hessian-vector products */
    double g0_norm, g_norm, energy, min_J;
} orc_info;

/* Lame parameters from Young's modulus and Poisson's ratio. */
void orc_lame(double E, double nu, double *mu, double *lam);

/* Constitutive law at one deformation gradient F (3x3 row-major). */
double orc_psi(const double F[9], double mu, double lam);
void orc_pk1(const double F[9], double mu, double lam, double P[9]);
void orc_dpk1(const double F[9], const double dF[9], double mu, double lam, double dP[9]);

/* Co-rotational law: polar decomposition F = R S (R proper rotation, S
 * symmetric positive definite; returns 0, or -1 when det F <= 0), energy
 * Psi = mu |F - R|^2 + lam/2 (tr S - 3)^2, P = 2 mu (F - R) + lam (tr S - 3) R
 * and its exact directional derivative (with dR). */
int orc_polar(const double F[9], double R[9], double S[9]);
double orc_psi_cr(const double F[9], double mu, double lam);
void orc_pk1_cr(const double F[9], double mu, double lam, double P[9]);
void orc_dpk1_cr(const double F[9], const double dF[9], double mu, double lam, double dP[9]);

/* Friction smoothing: f0(y), f1(y) = f0'(y) and f1'(y) for slip y >= 0. */
void orc_friction_f0(double y, double eps, double *f0, double *f1, double *df1);

/* Signed distance of world point x to the indenter and its world gradient. */
double orc_sdf(const orc_indenter *ind, const double x[3], double grad[3]);

/* Mesh precompute: B and V per tet. Returns 0, or -(1+e) for the first tet e
 * with V <= 0. */
int orc_precompute(int n, const double *X, int m, const int *T, double *B, double *V);

/* Lumped nodal masses: each tet gives rho V_e / 4 to each of its nodes. */
void orc_lumped_mass(int n, int m, const int *T, const double *V, double rho, double *mass);

/* Marks nodes on boundary faces (faces of exactly one tet); returns the number
 * of boundary faces. */
int orc_surface_nodes(int n, int m, const int *T, unsigned char *surf);

/* Deformation gradient of tet e at displacement u. */
void orc_deformation_gradient(const orc_problem *p, const double *u, int e, double F[9]);

/* Total energy; min_J receives the smallest det F (may be NULL). Tets with
 * det F <= 0 contribute +inf. */
double orc_energy(const orc_problem *p, const double *u, double *min_J);

/* Full gradient dPi/du (n x 3), fixed nodes included (not masked). */
void orc_gradient(const orc_problem *p, const double *u, double *g);

/* Dense Hessian (3n x 3n): exact Neo-Hookean tangent plus the contact block on
 * active contact nodes (Gauss-Newton, or exact when contact_full). Small meshes only. */
void orc_hessian_dense(const orc_problem *p, const double *u, double *H, int contact_full);

/* q = H(u) v using the assembled block-sparse Hessian (not masked). */
void orc_hessvec(const orc_problem *p, const double *u, const double *v, double *q, int contact_full);

/* Solves H(u) x = b on the free nodes (fixed rows and columns removed) by PCG
 * (or dense Cholesky when prm->dense). Returns CG iterations or ORC_NOT_SPD. */
int orc_linear_solve(const orc_problem *p, const double *u, const double *b, double *x,
                     const orc_params *prm, double rtol);

/* One load step: Newton from u (in/out) at the problem's indenter pose. */
int orc_step(const orc_problem *p, const orc_params *prm, double *u, orc_info *info);

/* Contact patch at u: ascending ids of nodes that carry a contact force
 * (phi < 0, or a lagged friction weight w > 0), forces on the skin
 * -k min(0, phi) n - dD/du_i, phi and the resultant. Returns the count
 * (arrays may be NULL to query it). */
int orc_contact_patch(const orc_problem *p, const double *u, int *ids, double *f, double *phi,
                      double F_total[3]);

/* Cauchy stress sigma = P F^T / J of one deformation gradient, as
 * (xx, yy, zz, xy, xz, yz), and its von Mises value (vm may be NULL). */
void orc_cauchy(const double F[9], double mu, double lam, double sigma[6], double *vm);

/* Per-tet Cauchy stress (m x 6) and von Mises stress (m) at u (either output
 * may be NULL). */
void orc_tet_stress(const orc_problem *p, const double *u, double *sigma, double *vm);

/* max_i |u_i| and mean_i |u_i| over all n nodes (paper Sec. IV's per-
 * indentation displacement statistics). */
void orc_displacement_stats(int n, const double *u, double *max_norm, double *mean_norm);

#ifdef __cplusplus
}
#endif
#endif
