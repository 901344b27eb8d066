/*
 * t2r.h — C ABI of the MI355X PNCG-IPC visuotactile gel solver.
 *
 * The library computes, per environment and per load step, the quasi-static
 * equilibrium of a tetrahedral neo-Hookean gel pad pressed by a rigid
 * indenter, and the displacement of markers embedded in its top face.
 *
 *   Step energy (Tac2Real, Supp. A, eq. ipc_energy, without the inertia term):
 *     Pi_s(x) = sum_e V_e psi(F_e) + kappa sum_{k in C(x)} b(d_k(x)) + D_s(x)
 *   minimised by preconditioned Dai-Kou nonlinear CG (Supp. A,
 *   eqs. dk_direction, step_size) with a Jacobi preconditioner, the
 *   analytic step bound dhat / (2 |p|_inf), a conservative CCD bound and
 *   backtracking. Markers follow Sec. 3.2 (interpolated from mesh nodes).
 *
 * Conventions
 *   units      mm, N, MPa (N/mm^2), energy N*mm
 *   floats     double (IEEE binary64) unless stated
 *   indices    int32, zero-based
 *   arrays     row-major; "[n][3]" means n consecutive xyz triples
 *   poses      7 doubles (tx, ty, tz, qw, qx, qy, qz): indenter-local point y
 *              maps to R(q) y + t; q need not be normalised
 *   host ptr   readable by the CPU; borrowed for the duration of the call
 *   device ptr HIP device memory on the context's device; borrowed until the
 *              work enqueued on the context's stream has completed
 *
 * Errors
 *   Every entry point returns t2r_status: T2R_OK (0) or a negative code. On a
 *   negative code the call had no effect on the context; t2r_last_error()
 *   describes it. Nothing is thrown across the ABI. Per-environment solve
 *   outcomes are not call errors: they are written as T2R_ENV_* bit masks.
 *   A context is not thread-safe: one host thread at a time.
 *
 * Lifetime
 *   t2r_create performs no HIP call. Classes and environments are described
 *   on the host; device memory is allocated and filled on the first call that
 *   needs the GPU (t2r_step, t2r_eval, t2r_get_state, ...), after which no
 *   more classes or environments can be added (T2R_E_STATE).
 */
#ifndef T2R_H
#define T2R_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct t2r_ctx t2r_ctx;
typedef int32_t t2r_status;

enum {
  T2R_OK = 0,
  T2R_E_ARG = -1,          /* invalid argument, size or mesh */
  T2R_E_NOMEM = -2,        /* device allocation failed */
  T2R_E_HIP = -3,          /* HIP runtime error (no device, launch failure, ...) */
  T2R_E_STATE = -4,        /* call not valid in the context's current state */
  T2R_E_UNSUPPORTED = -5   /* feature not available in the library as compiled */
};

/* Per-environment outcome bits written by t2r_step (d_status). */
enum {
  T2R_ENV_CONVERGED = 1,      /* every solve of the step reached its tolerance */
  T2R_ENV_MAXITER = 2,        /* some solve stopped at max_iters */
  T2R_ENV_INFEASIBLE = 4,     /* the step started from an intersecting state */
  T2R_ENV_NONFINITE = 8,      /* NaN/Inf pose or state; the env was not advanced */
  T2R_ENV_PAIR_OVERFLOW = 16, /* contact pair list overflowed; env rolled back */
  T2R_ENV_LINESEARCH = 32,    /* 30 halvings found no acceptable step */
  T2R_ENV_SUBSTEPS = 64,      /* continuation hit max_substeps before the target pose: the
                                 env keeps the equilibrium of the last pose it reached, which
                                 becomes its pose (t2r_get_state) */
  T2R_ENV_SKIPPED = 128,      /* masked out by the caller; state unchanged */
  T2R_ENV_BUDGET = 256        /* the env used up max_evals in this launch: the load step is
                                 rolled back (with T2R_ENV_MAXITER), the env keeps its last
                                 completed step's state and pose for the rest of the launch */
};

/* Material and contact parameters of one environment.
 *   E, nu   Young's modulus (MPa) and Poisson ratio of the gel, 0 < nu < 0.5
 *   mu_f    friction coefficient (0 disables friction)
 *   eps_v   friction mollifier width, mm per step (Supp. A, eq. friction_mollifier)
 *   dhat    barrier activation distance, mm
 *   kappa   barrier stiffness, N/mm */
typedef struct { double E, nu, mu_f, eps_v, dhat, kappa; } t2r_material;

/* Solver options.
 *   tol           stop a solve when |P g|_inf <= tol (mm), P = diag(H)^-1 (each
 *                 contact pair's contribution to an entry clamped at zero)
 *   substep_tol   tolerance of intermediate continuation solves (<= 0: use tol)
 *   max_iters     PNCG iterations per solve
 *   max_substeps  continuation solves per load step
 *   precision     0: all FP64; 1: FP32 element terms, FP64 elsewhere
 *   pair_capacity contact candidate pairs per env (0: automatic, 3x the gel's
 *                 surface vertices + edges + faces, at least 8192); the coarse
 *                 list holds 4x and the friction list 1/2 of it
 *   armijo        1: require sufficient decrease of Pi in the line search
 *   block_size    threads per env workgroup: 256 (two envs per CU) or 512 (one env
 *                 per CU, for few large envs); 0 = automatic: 512 while the envs
 *                 do not outnumber the compute units, else 256
 *   warm_start    1: when a load step continues the previous step's indenter
 *                 motion, start from x_{s-1} + f (x_{s-1} - x_{s-2}) if that point
 *                 is feasible (f = this step's motion over the previous one's,
 *                 less the gap it closed when it started out of contact), and
 *                 solve directly at the final pose when that start is clear of
 *                 the indenter there; 0: start from x_{s-1}
 *   dynamic       1: implicit-Euler form (Supp. A, eq. ipc_energy with its
 *                 inertia term): each load step is one time step dt and adds
 *                 1/2 sum_v m_v / dt^2 |x_v - xhat_v|^2, m_v = density x the
 *                 vertex's share sum V_e / 4 of its tets' rest volumes,
 *                 xhat = x^t + dt v^t; after the step v = (x - x^t) / dt (v = 0
 *                 after t2r_create, t2r_reset_envs and t2r_set_state). 0: the
 *                 quasi-static form. The adjoint and t2r_eval cover the
 *                 quasi-static form only.
 *   dt, density   time step (s) and mass density (t/mm^3, so that forces are in
 *                 N: 1,100 kg/m^3 = 1.1e-9) of the dynamic form
 *   max_evals     work budget of one env in one launch: energy (line-search trial)
 *                 plus curvature evaluation passes over its mesh and contact list;
 *                 0 = no limit. Every loop of a solve is bounded (max_iters, 30
 *                 halvings, max_substeps), but those bounds multiply; this one caps
 *                 the product, so a launch ends after at most about max_evals passes
 *                 of its slowest env (T2R_ENV_BUDGET)
 *   ee_mollifier  1: weight each gel-edge / indenter-edge barrier by IPC's
 *                 parallel-edge mollifier m(c) (the contact model of Supp. A
 *                 follows IPC), c = |a x b|^2 of the two edge vectors,
 *                 m(c) = (c/e)(2 - c/e) below e = 1e-3 |a_rest|^2 |b_rest|^2 and
 *                 1 above, so the edge-edge potential stays smooth as two edges
 *                 turn parallel; the friction lag keeps the unweighted barrier
 *                 force. 0: the plain barrier on every pair
 *   outer_radius  margin of the coarse candidate list beyond dhat, in multiples
 *                 of dhat (0: 6; else >= 2, at most 64). The inner list keeps a
 *                 margin of one dhat; the coarse list is rebuilt from the
 *                 indenter grids once the surface and the indenter have moved by
 *                 the difference of the margins since its last build. A wider
 *                 margin rebuilds less often and filters more pairs each time;
 *                 results do not depend on it
 *   deterministic 1: every sum of per-element and per-pair terms into per-vertex
 *                 totals, and every candidate and friction list, is built in a
 *                 fixed order (those passes run on one thread of the env's
 *                 workgroup, in index order; the lists are rebuilt at the start
 *                 of every load step), so a step's results depend only on its
 *                 inputs and its starting state (t2r_save_checkpoint) and repeat
 *                 bit for bit, also after t2r_load_checkpoint and in any batch,
 *                 at equal block_size. Much slower: for tests and debugging.
 *                 The adjoint entry points keep their atomic sums. 0: sums in
 *                 LDS / global atomics, whose order varies from run to run in
 *                 the last bits
 *   self_contact  1: the barrier also acts between gel surface primitives that
 *                 share no vertex (vertex / triangle and edge / edge pairs of the
 *                 gel; Supp. A places it between all surface primitives), without
 *                 friction. Such pairs are searched where the gel can deform:
 *                 among the surface primitives whose vertices all lie within the
 *                 coarse list's margin of the indenter (at most 512 vertices;
 *                 beyond that the env reports T2R_ENV_PAIR_OVERFLOW). The step
 *                 bound and the list margins count both sides' motion.
 *                 0: gel / indenter pairs only */
typedef struct {
  double tol;
  double substep_tol;
  int32_t max_iters;
  int32_t max_substeps;
  int32_t precision;
  int32_t pair_capacity;
  int32_t armijo;
  int32_t block_size;
  int32_t warm_start;
  int32_t dynamic;
  double dt;
  double density;
  int32_t max_evals;
  int32_t ee_mollifier;
  double outer_radius;
  int32_t deterministic;
  int32_t self_contact;
} t2r_solver_opts;

/* Per-environment counters of the last launch (t2r_step or t2r_step_sequence;
 * t2r_get_stats). Counts are summed over the launch's load steps; status,
 * n_candidates, n_active, n_friction, d_min, residual and energy are those of
 * its last load step. */
typedef struct {
  int32_t status;        /* T2R_ENV_* bits of the last load step */
  int32_t iters;         /* PNCG iterations, all solves of all load steps */
  int32_t substeps;      /* continuation solves */
  int32_t restarts;      /* direction resets to -P g */
  int32_t halvings;      /* line-search halvings */
  int32_t reculls;       /* candidate-list refreshes (filter of the outer list) */
  int32_t n_candidates;  /* candidate pairs at the last cull */
  int32_t n_active;      /* pairs closer than dhat at the end */
  int32_t n_friction;    /* lagged friction pairs of the last load step */
  int32_t max_solve_iters;
  int32_t outer_builds;  /* grid traversals building the outer candidate list */
  int32_t n_outer;       /* coarse (outer) candidate pairs at the end */
  double d_min;          /* smallest gel/indenter distance at the end (mm), inf if none < dhat */
  double residual;       /* final |P g|_inf (mm) */
  double energy;         /* final Pi (N mm) */
  double phase_ms[10];   /* ms spent by this env's workgroup in: [0] coarse (grid) culls,
                            [1] candidate filtering, [2] curvature elements, [3] curvature
                            pairs, [4] CCD, [5] evaluation elements, [6] evaluation pairs
                            and friction, [7] vector passes, [8] the whole launch, [9] friction lag */
  double list_fill;      /* largest (list length / capacity) of the inner, outer and friction
                            lists during the launch; > 1 means a list overflowed */
  int32_t evals;         /* energy and curvature evaluation passes of the launch (see max_evals) */
  int32_t reserved;
} t2r_env_stats;

/* Fills *o with the defaults: tol 1e-6, substep_tol 1e-4, max_iters 20000,
 * max_substeps 1000, precision 0, pair_capacity 0, armijo 1, block_size 0, warm_start 1,
 * dynamic 0, dt 1/60, density 1.1e-9, max_evals 200000, ee_mollifier 0, outer_radius 0,
 * deterministic 0, self_contact 0. */
void t2r_default_opts(t2r_solver_opts* o);

/* Creates a context bound to `hip_stream` (a hipStream_t, or NULL for the null
 * stream) of the device current at the first GPU call. `opts` may be NULL for
 * the defaults; it is copied. No HIP call is made. */
t2r_status t2r_create(t2r_ctx** out, const t2r_solver_opts* opts, void* hip_stream);

/* Releases every device allocation (synchronising the stream first) and the context. */
void t2r_destroy(t2r_ctx* ctx);

/* Message of the last failed call on ctx (empty if none); valid until the next call. */
const char* t2r_last_error(const t2r_ctx* ctx);

/* Optional device allocator used instead of hipMalloc/hipFree, e.g. a caching
 * allocator owned by the caller. Must be set before the first GPU call. */
typedef void* (*t2r_alloc_fn)(size_t bytes, void* user);
typedef void (*t2r_free_fn)(void* ptr, void* user);
t2r_status t2r_set_allocator(t2r_ctx* ctx, t2r_alloc_fn alloc, t2r_free_fn free_fn, void* user);

/* Adds a gel mesh class (host copy; validated here, no GPU use).
 *   n_v, X[n_v][3]     rest positions (mm)
 *   n_t, tets[n_t][4]  vertex ids; every tet must have a positive rest volume
 *                      and every vertex must belong to some tet
 *   fixed[n_v]         1 = vertex held at rest (Dirichlet), 0 = free
 *   n_m, markers[n_m][2] marker rest xy; each must lie inside the top face
 *                      (boundary triangles at the maximal z), where it is
 *                      embedded barycentrically (Sec. 3.2)
 * Surface primitives (boundary triangles, their edges and vertices) are
 * extracted; primitives whose vertices are all fixed are dropped.
 * T2R_E_ARG on inverted/degenerate tets, out-of-range ids, unreferenced
 * vertices, markers outside the top face, or sizes beyond 2^24 vertices. */
t2r_status t2r_add_gel(t2r_ctx* ctx, int32_t n_v, const double* X, int32_t n_t,
                       const int32_t* tets, const uint8_t* fixed, int32_t n_m,
                       const double* markers, int32_t* gel_id);

/* Counts of a gel class: out[0..9] = n_v, n_t, surface vertices, surface edges,
 * surface triangles, markers, tiles, top-face triangles, fixed vertices, and the
 * inner pair-list capacity its envs get under the current options. Host only. */
t2r_status t2r_gel_info(const t2r_ctx* ctx, int32_t gel_id, int32_t* out10);

/* Host copy of a gel class's embedding: marker_tri[n_m][3] vertex ids and
 * marker_w[n_m][3] barycentric weights (either pointer may be NULL). */
t2r_status t2r_gel_markers(const t2r_ctx* ctx, int32_t gel_id, int32_t* marker_tri,
                           double* marker_w);

/* Replaces a gel class's marker map with any linear one: marker m's
 * displacement is sum_k weight[m][k] (x - X) at vertex[m][k], k < 3 (host
 * arrays [n_m][3]; e.g. the k-nearest-neighbour map of Sec. 3.2 with k <= 3).
 * Before the first GPU call only (T2R_E_STATE after). Errors: T2R_E_ARG for a
 * bad gel id, n_m < 0, vertex ids out of range or non-finite weights. Host
 * only. */
t2r_status t2r_set_gel_markers(t2r_ctx* ctx, int32_t gel_id, int32_t n_m, const int32_t* vertex,
                               const double* weight);

/* Replaces a gel class's marker map with the k-nearest-neighbour map of
 * Sec. 3.2 (Tactile Representation: marker displacements interpolated from the
 * k nearest mesh nodes of each marker in the initial mesh, with weights; the
 * paper gives neither k nor the weights). Read here as: the k <= 3 top-face
 * vertices (vertices of the top-face triangles) nearest to the marker's rest xy
 * position, ties by vertex id, weighted by 1 / distance^power normalised to sum
 * 1; a marker within 1e-12 mm of a vertex takes that vertex alone (weight 1).
 * Unused slots repeat the nearest vertex with weight 0.
 *   n_m, markers_xy[n_m][2] marker rest xy (host, mm)
 *   k                   1, 2 or 3;  power > 0 (1: inverse distance)
 * Before the first GPU call only (T2R_E_STATE after). Errors: T2R_E_ARG for a
 * bad gel id, k, power or non-finite markers. Host only; the map is read back
 * with t2r_gel_markers. */
t2r_status t2r_set_gel_markers_knn(t2r_ctx* ctx, int32_t gel_id, int32_t n_m, const double* markers_xy,
                                   int32_t k, double power);

/* Adds a rigid indenter class: n_v local vertices Y[n_v][3] (mm) and n_f
 * triangles tris[n_f][3] of a closed surface. Edges are derived. Host only. */
t2r_status t2r_add_indenter(t2r_ctx* ctx, int32_t n_v, const double* Y, int32_t n_f,
                            const int32_t* tris, int32_t* ind_id);

/* Adds n environments; env i uses gel_ids[i], ind_ids[i], mats[i] and starts
 * at rest (x = X) with the indenter at pose0[i][7], which must leave every
 * gel/indenter distance > 0 (checked at the first step). Ids of the new envs
 * are first_env .. first_env + n - 1. Host only. */
t2r_status t2r_add_envs(t2r_ctx* ctx, int32_t n, const int32_t* gel_ids,
                        const int32_t* ind_ids, const t2r_material* mats,
                        const double* pose0, int32_t* first_env);

/* Replaces the material of the listed envs (host env ids, host materials,
 * validated as in t2r_add_envs). Takes effect from the next launch; changed
 * envs rebuild their contact lists. Synchronises the context's stream. */
t2r_status t2r_set_materials(t2r_ctx* ctx, int32_t n, const int32_t* env_ids, const t2r_material* mats);

/* Number of environments and total vertices over all envs. */
t2r_status t2r_env_count(const t2r_ctx* ctx, int32_t* n_env, int64_t* total_verts);

/* Advances every environment by one load step: the indenter moves from the
 * env's previous pose to d_pose[env][7] (device), with friction lagged at the
 * previous equilibrium, and the new equilibrium is solved.
 *   d_pose     device [n_env][7]
 *   d_env_mask device [n_env] int32 or NULL; envs with 0 are skipped (status
 *              T2R_ENV_SKIPPED, state unchanged)
 *   d_markers  device [sum n_m][3] or NULL: marker displacements, envs in order
 *   d_x        device [sum n_v][3] or NULL: equilibrium positions, envs in order
 *   d_status   device [n_env] int32 or NULL: T2R_ENV_* bits
 * All work is enqueued on the context's stream; the call does not wait. */
t2r_status t2r_step(t2r_ctx* ctx, const double* d_pose, const int32_t* d_env_mask,
                    double* d_markers, double* d_x, int32_t* d_status);

/* Advances every environment through n_steps consecutive load steps in one
 * launch (a scripted indenter trajectory, Sec. 4.2: the simulator replays the
 * recorded press and shear poses): load step k moves the indenter to
 * d_poses[k][env][7], exactly as n_steps calls of t2r_step would. Each env's
 * workgroup keeps its env for all steps, so the uneven cost of individual
 * solves averages out over the trajectory; envs whose previous launch took
 * longest start first.
 *   n_steps    >= 1
 *   d_poses    device [n_steps][n_env][7]
 *   d_env_mask device [n_env] int32 or NULL; envs with 0 skip every step
 *   d_markers  device [n_steps][sum n_m][3] or NULL: marker displacements after
 *              each load step
 *   d_x        device [sum n_v][3] or NULL: positions after the last step
 *   d_status   device [n_steps][n_env] int32 or NULL: T2R_ENV_* bits per step
 * A step that overflows or becomes infeasible is rolled back (the env keeps its
 * previous pose) and the next step starts from there. Asynchronous like
 * t2r_step; t2r_step is this call with n_steps = 1. */
t2r_status t2r_step_sequence(t2r_ctx* ctx, int32_t n_steps, const double* d_poses,
                             const int32_t* d_env_mask, double* d_markers, double* d_x,
                             int32_t* d_status);

/* Load steps driven by the indenter's motion instead of target poses (the
 * physics-engine input of Sec. 3.3: per engine step the object's pose relative
 * to the sensor, or its velocity, drives the tactile simulation). Every env
 * starts from its current pose q_0 = (t_0, r_0) and moves at a constant linear
 * velocity v and world-frame angular velocity w over one engine step of length
 * dt, cut into n_steps load steps: load step k (1-based) targets
 *   t = t_0 + v dt k / n_steps,   r = exp([w dt k / n_steps]x) r_0,
 * all in one persistent launch (otherwise as t2r_step_sequence: markers, x,
 * status and the tape as there; pose offsets do not apply, the motion is
 * relative to the env's own pose).
 *   t2r_step_velocity: d_vel device [n_env][6] = (v, w) in mm/s and rad/s;
 *                      dt > 0 in s.
 *   t2r_step_relative: d_rel0, d_rel1 device [n_env][7] = the object's pose
 *                      relative to the sensor at the start and at the end of
 *                      the engine step; the motion is (t_1 - t_0) and the
 *                      shortest rotation r_1 r_0^-1 (dt cancels).
 * Errors: T2R_E_ARG for NULL inputs, n_steps < 1 or dt <= 0. Asynchronous. */
t2r_status t2r_step_velocity(t2r_ctx* ctx, int32_t n_steps, double dt, const double* d_vel,
                             const int32_t* d_env_mask, double* d_markers, double* d_x, int32_t* d_status);
t2r_status t2r_step_relative(t2r_ctx* ctx, int32_t n_steps, const double* d_rel0, const double* d_rel1,
                             const int32_t* d_env_mask, double* d_markers, double* d_x, int32_t* d_status);

/* Sets each listed env's own mass density of the dynamic form (host arrays;
 * t/mm^3, e.g. 1.1e-9 = 1,100 kg/m^3), replacing the option `density` for it;
 * 0 returns the env to the option's density. Used by calibrations that fit
 * density per candidate (theta = [E, nu, rho, mu], Sec. 4.2, eq.
 * optimization_problem). Only the dynamic form reads it. Errors: T2R_E_ARG for
 * bad ids or negative / non-finite densities. Synchronises the stream. */
t2r_status t2r_set_densities(t2r_ctx* ctx, int32_t n, const int32_t* env_ids, const double* density);

/* Sets a rigid offset per env (host arrays; offsets[n][6] = translation dt in
 * mm and rotation vector dw in rad): from now on every target pose the env
 * receives from t2r_step / t2r_step_sequence, and its start pose at
 * t2r_reset_envs (and at the first GPU call), is moved so that each indenter
 * point R y + t becomes exp([dw]x) R y + t + dt. The current state is not
 * changed (reset to start from the offset start pose). The adjoints
 * (t2r_backward, t2r_backward_sequence) then report the pose part of dL/dtheta
 * with respect to this offset, dL/d(dt) and dL/d(dw) (through the left
 * Jacobian of SO(3)); with no offset set they are the derivatives at zero.
 * Zero offsets clear it. Errors: T2R_E_ARG for bad ids or non-finite values.
 * Synchronises the context's stream. */
t2r_status t2r_set_pose_offsets(t2r_ctx* ctx, int32_t n, const int32_t* env_ids, const double* offsets);

/* Diagnostic evaluation of one env's step energy at given positions, without
 * touching its state: the friction lag is taken at (d_x_lag, pose_lag) when
 * d_x_lag is not NULL, and the energy is evaluated at (d_x, pose).
 *   d_x, d_x_lag, d_p    device [n_v][3]; d_p may be NULL (curvature then 0)
 *   pose, pose_lag       host [7]
 *   d_grad, d_diag       device [n_v][3] or NULL: gradient, and the diagonal of the
 *                        Hessian with each contact pair's contribution clamped at
 *                        zero (the Jacobi preconditioner's; fixed vertices: 0 and 1)
 *   d_scalars            device [8] or NULL: Pi, p^T H p, d_min, active pairs,
 *                        feasible (1/0), candidate pairs, friction pairs, Pi_elastic
 * Synchronises the stream before returning. Returns T2R_E_NOMEM (outputs not
 * written) when the env's contact pair lists exceed their capacity. */
t2r_status t2r_eval(t2r_ctx* ctx, int32_t env, const double* d_x, const double* d_p,
                    const double* d_x_lag, const double* pose, const double* pose_lag,
                    double* d_grad, double* d_diag, double* d_scalars);

/* Copies the per-env counters of the last step into host_out (an array of
 * n_env t2r_env_stats; bytes must be >= n_env * sizeof). Synchronises. */
t2r_status t2r_get_stats(t2r_ctx* ctx, void* host_out, size_t bytes);

/* Device copies of the resumable state: per env its positions [n_v][3]
 * followed by its previous pose [7], envs in order (t2r_state_size doubles). */
t2r_status t2r_state_size(const t2r_ctx* ctx, int64_t* n_doubles);
t2r_status t2r_get_state(t2r_ctx* ctx, double* d_state);
t2r_status t2r_set_state(t2r_ctx* ctx, const double* d_state);

/* Checkpoint of everything a later load step reads besides its inputs: per
 * env its positions x_s and x_{s-1}, velocities (dynamic form), poses q_s and
 * q_{s-1}, and the smallest distance at the start of its last load step (the
 * warm start's motion estimate). The buffer (device, t2r_checkpoint_size
 * doubles, caller-owned) is opaque: the library's own array order, valid for
 * contexts built with the same meshes and envs. t2r_load_checkpoint restores
 * it, clears the neighbour lists (rebuilt at the next step) and restarts a
 * recording as t2r_set_state does. In deterministic mode the steps after a
 * load repeat those after the save bit for bit; in atomic mode they agree to
 * the last bits of the atomic sums. Both are asynchronous on the context's
 * stream. Errors: T2R_E_ARG for NULL. */
t2r_status t2r_checkpoint_size(const t2r_ctx* ctx, int64_t* n_doubles);
t2r_status t2r_save_checkpoint(t2r_ctx* ctx, double* d_buf);
t2r_status t2r_load_checkpoint(t2r_ctx* ctx, const double* d_buf);

/* Puts the listed envs (host ids) back at rest with their initial pose. */
t2r_status t2r_reset_envs(t2r_ctx* ctx, const int32_t* env_ids, int32_t n);

/* Sets the contact pair capacity per env (0: automatic). After the first GPU
 * call this reallocates the pair lists (positions and poses are kept; the lists
 * are rebuilt on the next step). T2R_E_NOMEM leaves the old capacity. */
t2r_status t2r_set_pair_capacity(t2r_ctx* ctx, int32_t capacity);

/* Generation counter of the context's launch layout: it changes whenever the
 * parameters or device buffers a launch captures change (the first GPU call,
 * t2r_set_pair_capacity, t2r_set_opts, t2r_set_materials, t2r_record). A
 * caller that replays a captured t2r_step (a HIP graph) must capture again
 * after it changes: the old capture may refer to freed buffers or stale
 * options. Host only. */
t2r_status t2r_layout_generation(const t2r_ctx* ctx, int64_t* gen);

/* Reads / replaces the solver options. Every field may change between steps
 * (block_size picks the workgroup shape of the next launch; a new
 * pair_capacity reallocates as t2r_set_pair_capacity). Invalid options:
 * T2R_E_ARG and no change. */
t2r_status t2r_get_opts(const t2r_ctx* ctx, t2r_solver_opts* out);
t2r_status t2r_set_opts(t2r_ctx* ctx, const t2r_solver_opts* opts);

/* Gradient of a loss L on the marker displacements of the current equilibrium
 * (the result of the last load step) with respect to each env's parameters
 * theta = (E, nu, mu_f, dt_x, dt_y, dt_z, dw_x, dw_y, dw_z): material, friction
 * coefficient and a rigid offset of the indenter that moves every indenter
 * point y to exp([dw]x)(y - t) + t + dt (t the indenter origin at the current
 * pose), taken at dt = dw = 0. Implicit differentiation at the equilibrium
 * (the paper itself calibrates without gradients):
 *   H lambda = dL/dx  (exact Hessian of the step energy, free DOFs; Jacobi-
 *                      preconditioned CG to a relative residual of 1e-10, at
 *                      most max_iters iterations, matrix-free on the GPU),
 *   dL/dtheta = -lambda^T dg/dtheta.
 * Covers frictionless equilibria (every env mu_f = 0): the last step then does
 * not depend on earlier steps, and dL/dmu_f is the derivative at mu_f = 0
 * (friction lagged at the previous equilibrium, with unit coefficient).
 *   d_dL_du  device [sum n_m][3]: dL/du, envs in order
 *   d_grad   device [n_env][9]: dL/dtheta
 * Per-env CG iterations, relative residual and status (T2R_ENV_CONVERGED,
 * T2R_ENV_MAXITER, T2R_ENV_NONFINITE for a Hessian that is not positive on
 * the CG directions) are reported by t2r_get_stats. Errors: T2R_E_UNSUPPORTED
 * if an env has mu_f != 0 (use t2r_backward_sequence), T2R_E_STATE before the
 * first load step. Asynchronous; positions and poses are not changed. */
t2r_status t2r_backward(t2r_ctx* ctx, const double* d_dL_du, double* d_grad);

/* t2r_backward without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving or training loops,
 * harnesses that forbid hipMalloc). Same arguments, results and errors as
 * t2r_backward, from the same kernel; the two-entry tape it needs (x_{s-1},
 * x_s and both poses of every env: 2 x (total 3 n_v + 7 n_env) doubles) is
 * copied into a static workspace of 2^21 doubles (16 MiB) that the library
 * holds on each GPU it runs on until the process ends, instead of a
 * context-owned buffer. T2R_E_ARG (checked before any GPU use) when the tape
 * does not fit, e.g. beyond about 700 envs of the 484-vertex gel or 70 of the
 * 4,914-vertex gel. All calls on one GPU share that workspace: calls that
 * overlap on one GPU (different streams or threads) race and must be ordered
 * by the caller. No hipMalloc/hipFree or allocating library call is made; the
 * context must already have stepped (its own buffers exist since then). */
t2r_status t2r_backward_static(t2r_ctx* ctx, const double* d_dL_du, double* d_grad);

/* Starts recording a trajectory tape of at most max_steps load steps (device
 * memory: (max_steps + 1) x (sum 3 n_v + 7 n_env) doubles, owned by the
 * context). Entry 0 is the current state of every env; each later t2r_step /
 * t2r_step_sequence appends every env's positions and pose after each of its
 * load steps. t2r_reset_envs and t2r_set_state restart the recording from the
 * new state. max_steps = 0 stops recording and frees the tape. A launch that
 * would exceed the tape returns T2R_E_STATE without stepping.
 * Errors: T2R_E_ARG (max_steps < 0), T2R_E_NOMEM (tape not allocated,
 * recording off). */
t2r_status t2r_record(t2r_ctx* ctx, int32_t max_steps);

/* Load steps on the tape (-1: not recording). */
t2r_status t2r_tape_length(const t2r_ctx* ctx, int32_t* n_steps);

/* Copies tape entry `entry` (0: the state when recording started; k: after
 * the k-th recorded load step) into d_state, device [t2r_state_size] in the
 * layout of t2r_get_state (per env: positions [n_v][3], then the pose [7]).
 * Errors: T2R_E_STATE without a tape, T2R_E_ARG for an entry outside
 * [0, t2r_tape_length]. Asynchronous. */
t2r_status t2r_tape_read(t2r_ctx* ctx, int32_t entry, double* d_state);

/* Gradient of a loss L on the marker displacements of the last n_steps
 * recorded load steps with respect to each env's theta (as t2r_backward; the
 * pose offset applies to every pose of the window, including the lag pose of
 * its first step). With lagged friction (Supp. A, eq. friction_energy) step s
 * depends on (x_{s-1}, q_{s-1}) through lambda_k, the closest points and the
 * normal of its friction pairs, so the solve runs backwards through the
 * window, last step first:
 *   H_s lambda_s = W^T dL/du_s - (d g_{s+1}/d x_s)^T lambda_{s+1},
 *   dL/dtheta = -sum_s lambda_s^T d g_s/d theta,
 * H_s the exact Hessian of step s with its friction term (Jacobi-PCG to the
 * relative residual 1e-10, at most max_iters iterations per step). The state
 * before the window's first step is taken as given (record from rest to
 * differentiate a whole trajectory). Every state is read from the tape.
 *   d_dL_du  device [n_steps][sum n_m][3]: dL/du of each step, oldest first
 *   d_grad   device [n_env][9]: dL/dtheta
 * Stats as t2r_backward (iterations summed over the steps, the largest
 * relative residual, substeps = n_steps). Errors: T2R_E_STATE without a tape,
 * T2R_E_ARG for n_steps outside [1, t2r_tape_length]. Asynchronous; positions,
 * poses and the tape are not changed. */
t2r_status t2r_backward_sequence(t2r_ctx* ctx, int32_t n_steps, const double* d_dL_du, double* d_grad);

#ifdef __cplusplus
}
#endif
#endif /* T2R_H */
