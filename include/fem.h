/*
 * libfem: indentation of a tetrahedral skin mesh on one AMD Instinct MI355X
 * (gfx950).
 *
 * The problem is the finite-element contact simulation of paper Sec. III-A: a
 * volumetric mesh of linear tetrahedra (a soft skin), fixed boundary nodes
 * (bonded to a rigid core / clamped), rigid indenters driven into the skin,
 * and, per step, the nodal positions (displacements) and nodal contact forces
 * with their resultant. By default the skin is the compressible Neo-Hookean
 * solid that the paper's validated model uses,
 *     Psi(F) = mu/2 (tr F^T F - 3) - mu ln J + lam/2 (ln J)^2,
 * or, per mesh handle or job, the co-rotational law of the paper's own
 * simulator (fem_set_model). Contact is a per-node penalty k/2 min(0, phi)^2
 * against the indenter's signed distance phi, optionally with lagged,
 * smoothed Coulomb friction (fem_set_friction). Each step, quasi-static or a
 * backward-Euler time step (fem_set_dynamics), is solved to a stationary
 * point of its energy by Newton's method with matrix-free
 * Jacobi-preconditioned CG and a backtracking line search.
 *
 * Conventions for every call:
 *   - SI units; all floating-point arguments are double whatever the
 *     internal precision; all pointers are HOST pointers;
 *   - node-vector arrays are n x 3, row-major (x, y, z per node);
 *   - inputs are copied, the caller keeps ownership of its buffers;
 *   - return value 0 = FEM_OK, negative = error (no exception crosses the
 *     ABI); fem_last_error() then describes the failure (thread-local);
 *     positive = a usable result with a warning (FEM_W_FLOOR);
 *   - a handle is not thread-safe; distinct handles are independent.
 */
#ifndef LIBFEM_FEM_H
#define LIBFEM_FEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define FEM_OK 0
#define FEM_W_FLOOR 1             /* step ended at the rounding floor of the working
                                     precision: |g_free| stopped falling, below
                                     newton_floor_rtol * |g_free(start)| but above
                                     the newton_rtol target; the iterate is usable */
#define FEM_E_INVALID (-1)        /* bad argument: null, size, index, non-finite */
#define FEM_E_DEGENERATE (-2)     /* a tet has rest volume <= 0 */
#define FEM_E_OOM (-3)            /* device allocation failed */
#define FEM_E_DEVICE (-4)         /* HIP runtime error, or no usable device */
#define FEM_E_STATE (-5)          /* call order: material or indenter not set */
#define FEM_E_NOT_CONVERGED (-6)  /* Newton cap or line-search stall; state kept */
#define FEM_E_INVERSION (-7)      /* line search could not keep every det F > 0 */
#define FEM_E_BUFFER (-8)         /* caller buffer too small */

/* ---- enums -------------------------------------------------------------- */
#define FEM_PREC_FP64 0           /* all arithmetic in double */
#define FEM_PREC_FP32 1           /* element math and CG vectors in float;
                                     dot products, norms, energies, the Newton
                                     test and contact geometry in double */

/* Indenter families (paper Sec. IV-A names spherical, cylindrical and ring
 * indenters; a box stands for the flat-faced pegs of Fig. 3). The indenter's
 * local frame q maps to the world as x = R q + c. */
#define FEM_SPHERE 0              /* shape = {radius} */
#define FEM_CYLINDER 1            /* shape = {radius, height}; axis = local z, centred */
#define FEM_BOX 2                 /* shape = {hx, hy, hz} half extents */
#define FEM_RING 3                /* shape = {major radius, minor radius}; torus about local z */

/* Constitutive laws (paper Sec. III-A): the compressible Neo-Hookean law of
 * the validated skin model, Psi = mu/2 (tr F^T F - 3) - mu ln J + lam/2 ln^2 J,
 * and the co-rotational linear elasticity of the paper's own simulator,
 * Psi = mu |F - R|^2 + lam/2 (tr S - 3)^2 with the polar decomposition
 * F = R S (Newton's method uses its exact tangent, rotation derivative
 * included). mu and lam follow from (E, nu) for both. */
#define FEM_MODEL_NEOHOOKEAN 0
#define FEM_MODEL_COROTATIONAL 1

#define FEM_PRECOND_JACOBI 0      /* scalar Jacobi */
#define FEM_PRECOND_BLOCK 1       /* 3x3 node-block Jacobi */

typedef struct fem_mesh fem_mesh;

typedef struct {
    int32_t precision;   /* FEM_PREC_FP64 or FEM_PREC_FP32 */
    int32_t device;      /* HIP device ordinal */
    void *stream;        /* hipStream_t to run on; NULL = the library's own stream */
} fem_config;

typedef struct {
    double newton_rtol;  /* converged when |g_free| <= max(newton_rtol * |g_free(start)|, newton_atol) */
    double newton_atol;  /* newtons */
    int32_t max_newton;
    double cg_rtol;      /* floor of the CG forcing term
                            eta = clamp((|g|/|g_start|)^cg_eta_power, cg_rtol, cg_eta_max) */
    double cg_eta_max;
    int32_t max_cg;      /* per Newton iteration */
    int32_t precond;     /* FEM_PRECOND_* */
    int32_t contact_hessian; /* 0: Gauss-Newton k n n^T; 1: exact k (n n^T + phi Hess(phi)) */
    double c1;           /* Armijo constant */
    int32_t max_halvings;
    double newton_floor_rtol; /* rounding-floor exit: after two accepted Newton
                                 iterations in a row that fail to halve the
                                 step's smallest |g_free|, the step ends with
                                 FEM_W_FLOOR if |g_free| <= newton_floor_rtol *
                                 |g_free(start)|; 0 disables the exit */
    double cg_eta_power; /* exponent p of the forcing term, in (0, 1]: 1 keeps
                            Newton's quadratic convergence with tight late
                            solves; p < 1 gives order 1 + p with fewer CG
                            iterations per Newton iteration (default 0.75 on
                            the FP32 path, 1 on FP64) */
} fem_solve_params;

typedef struct {
    int32_t status;      /* same value fem_step returned */
    int32_t newton_iters;
    int32_t cg_iters;    /* summed over Newton iterations */
    int32_t ls_trials;   /* line-search energy/gradient evaluations */
    int32_t grad_passes; /* element passes (gradient or trial), line-search trials included */
    int32_t hv_products; /* Hessian-vector products */
    double g0_norm;      /* |g_free| at the start of the step */
    double g_norm;       /* |g_free| at the end */
    double energy;       /* total energy at the end */
    double min_J;        /* smallest det F at the end */
    int64_t tet_updates; /* m * (grad_passes + hv_products) */
} fem_step_info;

/* Creates a mesh handle (paper Sec. III-A: volumetric tet mesh with fixed
 * boundary conditions on some nodes).
 *   X      n_nodes x 3 rest positions (m);
 *   tets   n_tets x 4 node ids, 0-based; each tet must have det[X1-X0, X2-X0, X3-X0] > 0;
 *   fixed  n_nodes flags, 1 = the node's displacement is prescribed (it keeps
 *          its current value, 0 after creation);
 *   cfg    precision, device and stream (NULL = FP64 on device 0).
 * Computes per-tet inverse rest edge matrices and volumes and the
 * contact-eligible nodes (nodes on boundary faces that are not fixed) on the
 * device. *out receives the handle, which owns all device memory.
 * Errors: FEM_E_INVALID (null pointer, n_nodes <= 0, n_tets <= 0,
 * n_nodes >= 2^21, index out of range, non-finite X), FEM_E_DEGENERATE,
 * FEM_E_OOM, FEM_E_DEVICE. */
int fem_create_mesh(const double *X, int32_t n_nodes, const int32_t *tets, int32_t n_tets,
                    const uint8_t *fixed, const fem_config *cfg, fem_mesh **out);

/* Releases the handle and its device memory; NULL is ignored. */
void fem_destroy_mesh(fem_mesh *mesh);

/* Sets the skin material (paper Sec. III-A: elastic modulus E and Poisson's
 * ratio nu are the free material parameters). mu = E / (2 (1 + nu)),
 * lam = E nu / ((1 + nu)(1 - 2 nu)). density is stored and unused by the
 * quasi-static solve. Errors: FEM_E_INVALID (E <= 0, nu outside (-1, 0.5),
 * density < 0, non-finite). */
int fem_set_material(fem_mesh *mesh, double E, double nu, double density);

/* Sets the rigid indenter pose for the next fem_step (paper Sec. III-A:
 * rigid objects driven into the skin; here moved kinematically per load step).
 *   kind     FEM_SPHERE .. FEM_RING; shape/n_shape as listed with the kinds;
 *   R        3x3 row-major rotation (orthonormal to 1e-9, det +1);
 *   c        centre; k_penalty  contact stiffness per node (N/m), >= 0.
 * Errors: FEM_E_INVALID (bad kind, too few or non-positive shape values,
 * R not a rotation, non-finite values). */
int fem_set_indenter(fem_mesh *mesh, int32_t kind, const double *shape, int32_t n_shape, const double R[9],
                     const double c[3], double k_penalty);

/* Selects the constitutive law for the following steps (default
 * FEM_MODEL_NEOHOOKEAN). Errors: FEM_E_INVALID (unknown model). */
int fem_set_model(fem_mesh *mesh, int32_t model);

/* Coulomb friction between skin and indenter (paper Sec. III-A: the
 * simulator's contact is frictional, coefficient 0.783), lagged and smoothed
 * so that every step stays a minimisation with a symmetric Newton matrix.
 * The normal force and normal of each contact node come from the lag state
 * (the displacement at the start of the step, with the indenter where it was
 * when that state was reached): w = mu_f k max(0, -phi_lag). Its slip is the
 * tangential part of its displacement relative to the indenter's translation
 * since, s = (I - n n^T)(u - u_lag - (c - c_lag)), and the step adds
 * w f0(|s|) to the potential, f0 a C1 smoothing of |s| that is exact beyond
 * a slip of eps: the friction force is at most w, and exactly w against the
 * slip once |s| >= eps. The lag state is the result of the previous fem_step
 * at its indenter pose, or the displacements of fem_set_displacements at the
 * indenter pose set then; before either there is none and the step carries no
 * friction. mu_f = 0 turns friction off (the default). eps = 1e-5 m suits
 * millimetre indentations in steps of tens of micrometres; smaller values
 * sharpen the stick-slip transition at the cost of Newton iterations.
 * Errors: FEM_E_INVALID (mu_f < 0, or eps <= 0 with mu_f > 0, non-finite). */
int fem_set_friction(fem_mesh *mesh, double mu_f, double eps);

/* Fills the default solve parameters for a precision mode. */
void fem_default_params(fem_solve_params *params, int32_t precision);

/* Solves one quasi-static load step at the current indenter pose, warm-
 * started from the current displacement: Newton on the total energy
 * (elastic + contact penalty) over the free nodes. Synchronous: returns when
 * the step is done. params NULL = defaults; info may be NULL.
 * Returns FEM_OK, or FEM_W_FLOOR when Newton stopped at the rounding floor
 * (see newton_floor_rtol). Errors: FEM_E_STATE (no material or indenter),
 * FEM_E_NOT_CONVERGED (the last accepted iterate is kept and usable),
 * FEM_E_INVERSION, FEM_E_DEVICE. */
int fem_step(fem_mesh *mesh, const fem_solve_params *params, fem_step_info *info);

/* Copies the nodal displacements (paper Sec. III-A: nodal positions / the
 * deformation field are the simulator's output) into u (capacity doubles,
 * at least 3 n). Errors: FEM_E_INVALID, FEM_E_BUFFER. */
int fem_get_displacements(const fem_mesh *mesh, double *u, int64_t capacity);

/* Replaces the nodal displacements (warm start, resume, or prescribed
 * displacements on fixed nodes); count must equal 3 n. Velocities are kept.
 * With an indenter set, u at its current pose becomes the friction lag state
 * of the next step. Errors: FEM_E_INVALID. */
int fem_set_displacements(fem_mesh *mesh, const double *u, int64_t count);

/* Implicit time stepping (paper Sec. III-A: the simulator integrates the
 * skin in time). With dt > 0 every fem_step is one backward-Euler step of
 * length dt: Newton on the incremental potential
 *   Pi(u) + sum_{i free} m_i / (2 dt^2) |u_i - ut_i|^2,  ut = u^n + dt v^n,
 * with lumped masses m_i = density * sum_{tets at i} V_e / 4 (density from
 * fem_set_material), then v^{n+1} = (u^{n+1} - u^n) / dt. dt = 0 returns to
 * quasi-static load steps. Velocities start at zero.
 * Errors: FEM_E_INVALID (dt < 0 or non-finite), FEM_E_STATE (dt > 0 without
 * a material of positive density). */
int fem_set_dynamics(fem_mesh *mesh, double dt);

/* Nodal velocities after the last step (n x 3, capacity >= 3 n; zero for
 * quasi-static steps), and their replacement (count = 3 n, e.g. an initial
 * velocity field). Errors: FEM_E_INVALID, FEM_E_BUFFER. */
int fem_get_velocities(const fem_mesh *mesh, double *v, int64_t capacity);
int fem_set_velocities(fem_mesh *mesh, const double *v, int64_t count);

/* Contact patch at the current state (paper Sec. III-A: nodal contact forces,
 * summed into resultant forces): ids of the eligible nodes that carry a
 * contact force (phi < 0, or friction from the lag state) in ascending order,
 * the force each exerts on the skin f = -k min(0, phi) grad(phi) plus the
 * friction force (n_contact x 3), the penetrations phi, and F_total = sum f. Any output
 * pointer may be NULL except n_contact. If capacity < count, returns
 * FEM_E_BUFFER with *n_contact = the count needed (F_total still filled). */
int fem_get_contact_patch(const fem_mesh *mesh, int32_t *ids, double *f, double *phi, int32_t capacity,
                          int32_t *n_contact, double F_total[3]);

/* Per-tet stress at the current displacement (paper Sec. III-A: the
 * simulator's deformation field, here reduced to the stress a data-generation
 * pipeline records): Cauchy stress sigma = P F^T / J of the Neo-Hookean law,
 * 6 values per tet (xx, yy, zz, xy, xz, yz, Pa) in the caller's tet order,
 * and its von Mises value sqrt(3/2 s:s) with s the deviator. Computed in the
 * handle's precision, returned as double; a tet with det F <= 0 gives NaN.
 * Either output may be NULL; capacity is in tets (>= n_tets).
 * Errors: FEM_E_INVALID, FEM_E_STATE (no material), FEM_E_BUFFER. */
int fem_get_tet_stress(const fem_mesh *mesh, double *sigma, double *von_mises, int64_t capacity);

/* max_i |u_i| and mean_i |u_i| over all nodes at the current displacement
 * (the per-indentation displacement statistics of paper Sec. IV). Either
 * output may be NULL. Errors: FEM_E_INVALID. */
int fem_get_displacement_stats(const fem_mesh *mesh, double *max_norm, double *mean_norm);

/* Mesh facts computed at creation: node and tet counts, number of
 * contact-eligible nodes, and (if eligible != NULL, capacity >= n) the
 * per-node eligibility flags. */
int fem_get_mesh_info(const fem_mesh *mesh, int32_t *n_nodes, int32_t *n_tets, int32_t *n_eligible,
                      uint8_t *eligible, int32_t capacity);

/* Evaluates, at the current displacement, the unmasked energy gradient
 * g = dPi/du (n x 3, fixed nodes included), the total energy and the smallest
 * det F, running the same element and contact kernels as fem_step. Any output
 * may be NULL. Errors: FEM_E_STATE, FEM_E_BUFFER (capacity < 3 n). */
int fem_eval_gradient(fem_mesh *mesh, double *g, int64_t capacity, double *energy, double *min_J);

/* q = H(u) v at the current displacement with the matrix-free Hessian-vector
 * kernels of fem_step (unmasked; contact block per params->contact_hessian,
 * params NULL = defaults). v and q are n x 3. Errors: FEM_E_STATE, FEM_E_BUFFER. */
int fem_eval_hessvec(fem_mesh *mesh, const fem_solve_params *params, const double *v, double *q, int64_t capacity);

/* Kernel timing (measurement aid, not part of the solve). A solver step is
 * three kernels over every live job: the tile pass (per job the matrix-free
 * Hessian-vector product during CG, the element + contact pass of a gradient
 * or line-search trial otherwise), the node pass (CG update, Newton init,
 * line-search directional derivative) and the finalize. With every > 0,
 * every every-th round of solver steps is launched kernel by kernel, each
 * launch with a start and a stop HIP event (hipExtLaunchKernel on the job
 * group's stream: the dispatch's own start and end); the other rounds
 * replay captured graphs as without timing. every = 0 turns timing off.
 * Counters are cleared on each call. */
#define FEM_KERNEL_TILE 0
#define FEM_KERNEL_NODE 1
#define FEM_KERNEL_FINALIZE 2
int fem_set_kernel_timing(fem_mesh *mesh, int32_t every);

/* Sampled launches of one timed kernel so far and their summed event-to-event
 * milliseconds. Errors: FEM_E_INVALID (null, unknown kernel). */
int fem_get_kernel_timing(const fem_mesh *mesh, int32_t kernel, int64_t *count, double *total_ms);

/* ---- batches of indentation jobs ------------------------------------------
 * A batch holds meshes (shared, read-only) and up to max_jobs indentation
 * jobs, each with its own displacement and solver state resident on the
 * device. fem_batch_run advances every unfinished job concurrently: one
 * launch sequence serves all jobs, whichever solver phase each is in, so jobs
 * of different meshes, indenters and depths progress together and a job
 * added between runs joins the next round (continuous batching). The
 * indenters are driven in as in paper Sec. III-A: kinematically, load step s
 * of S placing the indenter at c0 + depth * s / S * direction.
 */
typedef struct fem_batch fem_batch;

typedef struct {
    int32_t kind;        /* FEM_SPHERE .. FEM_RING */
    double shape[4];     /* as listed with the kinds; unused entries ignored */
    double R[9];         /* rotation, row-major */
    double c0[3];        /* centre at depth 0 (initial contact) */
    double direction[3]; /* press direction (unit) */
    double depth;        /* total indentation depth (m) */
    int32_t steps;       /* quasi-static load steps */
    double k_penalty;    /* N/m per node */
    double dt;           /* > 0: each step is a backward-Euler time step of
                            this length (see fem_set_dynamics); 0: quasi-static */
    double density;      /* kg/m^3, for the lumped masses when dt > 0 */
    int32_t model;       /* FEM_MODEL_NEOHOOKEAN or FEM_MODEL_COROTATIONAL */
    double friction;     /* Coulomb coefficient, 0 = frictionless (see fem_set_friction);
                            the lag state of the first step is u = 0 at c0 */
    double friction_eps; /* slip smoothing length (m), > 0 when friction > 0;
                            1e-5 suits millimetre indentations in 100 steps */
} fem_indentation;

typedef struct {
    int32_t done;        /* 1 when every load step has been taken */
    int32_t status;      /* FEM_OK, or the status of the first failed load step */
    int32_t step;        /* current (or last) load step, 1-based */
    int32_t steps_ok, steps_failed; /* steps_ok counts FEM_W_FLOOR steps too */
    int32_t steps_floor; /* load steps that ended with FEM_W_FLOOR */
    int64_t newton_iters, cg_iters, hv_products, grad_passes, ls_trials;
    int64_t tet_updates; /* n_tets * (grad_passes + hv_products) */
    double energy, min_J, g_norm;
} fem_job_info;

typedef struct {
    int32_t n_nodes, n_tets, n_tiles, n_entries, n_eligible;
} fem_mesh_layout;

/* Creates an empty batch for at most max_jobs (1..65536) concurrent jobs.
 * Errors: FEM_E_INVALID, FEM_E_OOM, FEM_E_DEVICE. */
int fem_batch_create(const fem_config *cfg, int32_t max_jobs, fem_batch **out);
void fem_batch_destroy(fem_batch *batch);

/* Adds a mesh (arguments and errors as fem_create_mesh); *mesh_id names it. */
int fem_batch_add_mesh(fem_batch *batch, const double *X, int32_t n_nodes, const int32_t *tets, int32_t n_tets,
                       const uint8_t *fixed, int32_t *mesh_id);

/* Layout facts of a mesh: nodes, tets, tiles, tile entries, contact-eligible nodes. */
int fem_batch_mesh_info(const fem_batch *batch, int32_t mesh_id, fem_mesh_layout *info);

/* Adds an indentation job on a mesh, starting from rest (u = 0) with material
 * (E, nu); its device state is allocated now. Errors: FEM_E_INVALID (bad
 * mesh id, material, indenter or schedule), FEM_E_BUFFER (batch full), FEM_E_OOM. */
int fem_batch_add_job(fem_batch *batch, int32_t mesh_id, double E, double nu, const fem_indentation *job,
                      int32_t *job_id);

/* Restarts a job in its existing slot from rest with a new material and
 * schedule, allocating nothing (arguments and errors as fem_batch_add_job). */
int fem_batch_restart_job(fem_batch *batch, int32_t job_id, double E, double nu, const fem_indentation *job);

/* Frees a job's slot and device state. */
int fem_batch_remove_job(fem_batch *batch, int32_t job_id);

/* Advances all unfinished jobs: until every job is done (max_rounds <= 0) or
 * for max_rounds rounds. *n_running (may be NULL) receives the number of jobs
 * still running. Errors: FEM_E_INVALID, FEM_E_DEVICE. */
int fem_batch_run(fem_batch *batch, const fem_solve_params *params, int32_t max_rounds, int32_t *n_running);

/* Progress and counters of a job (as of the end of the last run). */
int fem_batch_job_info(const fem_batch *batch, int32_t job_id, fem_job_info *info);

/* Status of each load step the job has taken so far (as of the end of the
 * last run), in order: status[k] is the outcome of load step k + 1 (paper
 * Sec. III-A: the indenter is driven in step by step), FEM_OK, FEM_W_FLOOR,
 * FEM_E_NOT_CONVERGED or FEM_E_INVERSION. *n_steps receives the number of
 * steps taken; the first 1024 load steps of a job are recorded. status may be
 * NULL to query the count. Errors: FEM_E_INVALID (null n_steps, unknown job),
 * FEM_E_BUFFER (capacity < *n_steps). */
int fem_batch_job_step_status(const fem_batch *batch, int32_t job_id, int32_t *status, int32_t capacity,
                              int32_t *n_steps);

/* A job's per-tet stress and displacement statistics, as the single-mesh calls. */
int fem_batch_get_tet_stress(fem_batch *batch, int32_t job_id, double *sigma, double *von_mises, int64_t capacity);
int fem_batch_get_displacement_stats(fem_batch *batch, int32_t job_id, double *max_norm, double *mean_norm);

/* A job's velocities (n x 3, zero for quasi-static jobs), as fem_get_velocities. */
int fem_batch_get_velocities(fem_batch *batch, int32_t job_id, double *v, int64_t capacity);

/* A job's displacements (n x 3) and contact patch, as the single-mesh calls. */
int fem_batch_get_displacements(fem_batch *batch, int32_t job_id, double *u, int64_t capacity);
int fem_batch_get_contact_patch(fem_batch *batch, int32_t job_id, int32_t *ids, double *f, double *phi,
                                int32_t capacity, int32_t *n_contact, double F_total[3]);

/* fem_batch_get_contact_patch for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result in the same caller arrays, with the kernel's
 * staging in a static device array of the library (about 1.2 MB per device,
 * held until the process ends) instead of a buffer the batch allocates. It
 * calls no hipMalloc or hipFree and allocates no host memory either: the
 * entries are ordered in the caller's arrays. Every call on one device shares
 * that array, so calls that overlap on one device (from several threads or
 * batches) race and must be serialised by the caller. Limits and errors, in
 * addition to those of fem_batch_get_contact_patch: FEM_E_INVALID if the
 * job's mesh has more than FEM_NOALLOC_MAX_CONTACT contact-eligible nodes, or
 * if f or phi is requested without ids (the ids order the entries);
 * FEM_E_STATE if jobs were added, restarted or removed since the last
 * fem_batch_run (updating the launch tables would allocate). */
#define FEM_NOALLOC_MAX_CONTACT 32768
int fem_batch_get_contact_patch_noalloc(fem_batch *batch, int32_t job_id, int32_t *ids, double *f, double *phi,
                                        int32_t capacity, int32_t *n_contact, double F_total[3]);

/* Kernel timing for a batch (as fem_set_kernel_timing). */
int fem_batch_set_kernel_timing(fem_batch *batch, int32_t every);
int fem_batch_get_kernel_timing(const fem_batch *batch, int32_t kernel, int64_t *count, double *total_ms);

/* Launches of one timed kernel since timing was turned on (sampled or not). */
int fem_batch_get_kernel_launches(const fem_batch *batch, int32_t kernel, int64_t *launches);

/* Launch mode: with enable != 0 (the default) each round of kernels is
 * captured once per round length into a HIP graph and replayed; 0 launches
 * the kernels one by one. Results are the same either way. */
int fem_set_graphs(fem_mesh *mesh, int32_t enable);
int fem_batch_set_graphs(fem_batch *batch, int32_t enable);

/* Batch tuning options (set before fem_batch_run; tile limits apply to meshes
 * added afterwards):
 *   FEM_OPT_ROUND_STEPS solver steps per round between host polls, 1..64
 *                      (0 = automatic: 16 for batches, the expected length
 *                      of the Newton iteration for a single job);
 *   FEM_OPT_TILE_TETS  tets per tile, 64..512 (default 512);
 *   FEM_OPT_TILE_NODES distinct nodes per tile, 16..256 (default 256);
 *   FEM_OPT_DETERMINISTIC 0 (default) or 1: the tile passes sum element
 *                      contributions into the tile partials in a fixed
 *                      order (each chunk of tets stores its contributions,
 *                      then every tile entry adds its incident ones in
 *                      ascending tet order) instead of with LDS atomics, so
 *                      a job's result is bitwise independent of the other
 *                      jobs in the batch and of the launch configuration;
 *                      slower, a cross-check of the default mode, whose
 *                      atomic sums depend on the order of wavefronts;
 *   FEM_OPT_GROUPS     job groups per round: 0 or 1 (default) one, 2 two.
 *                      With two groups each group's solver steps run on a
 *                      stream of its own and the groups' tile passes
 *                      alternate, so one group's node pass (memory-bound)
 *                      overlaps the other's tile pass (arithmetic-bound);
 *                      every job computes the same steps either way.
 * Errors: FEM_E_INVALID (unknown option, value out of range). */
#define FEM_OPT_ROUND_STEPS 0
#define FEM_OPT_TILE_TETS 1
#define FEM_OPT_TILE_NODES 2
#define FEM_OPT_GROUPS 3
#define FEM_OPT_DETERMINISTIC 4
int fem_batch_set_option(fem_batch *batch, int32_t option, int32_t value);

/* Device bytes one job on mesh mesh_id allocates (for admission by HBM
 * footprint); the mesh itself is shared and not included. */
int fem_batch_job_footprint(const fem_batch *batch, int32_t mesh_id, int64_t *bytes);

/* Static text for a status code. */
const char *fem_status_string(int status);

/* Message for the last failed call on this thread ("" if none). */
const char *fem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
