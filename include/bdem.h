/*
 * bdem.h -- C ABI of the MI355X implicit bonded-DEM library.
 *
 * One implicit time step of bonded DEM with manifold optimization (Lu, Cao,
 * Li, Hu, "Implicit Bonded Discrete Element Method with Manifold
 * Optimization"): minimise the incremental potential of Section 3.1
 * (implicit-Euler form, equation "eq:optimization form") over particle
 * positions p in R^3 and unit quaternions q in S^3 by the manifold Newton
 * method of Section 4.2 / Algorithm 2, inside the stable integrator of
 * Algorithm 3 (SPD-projected Hessian, PCG with relative tolerance
 * eps_r = min(0.5, sqrt|grad f|), exp-map line search, projection, velocity
 * update, bond update).  Bond potentials: Section 3.2 (stretch, shear,
 * bend/twist).  Fracture: Section 3.3.  Ground repulsion: Section 5.4.
 *
 * Conventions
 *   - quaternions are (x, y, z, w), scalar last (Appendix A); the rest
 *     orientation of every particle is the identity, rest bond data (l0, d0)
 *     come from the positions passed to bdem_create;
 *   - reduced tangent coordinates: 6 per particle, (dp, y) with
 *     dq = G_l(q)^T y, G_l the nullspace operator of Appendix A;
 *   - all host arrays are row-major, tightly packed, in the caller's particle
 *     and bond order.
 *
 * Ownership and streams
 *   - bdem_create copies every host input; the caller may free them on return.
 *   - device memory comes from the caller's workspace (workspace_dev, sized by
 *     bdem_workspace_bytes, >= 256-byte aligned) or, if workspace_dev is NULL,
 *     from hipMalloc inside the library (freed by bdem_destroy).
 *   - all work is enqueued on hip_stream (a hipStream_t; NULL = the null
 *     stream).  Calls that return host data synchronise that stream.
 *   - calls on one handle are not thread safe; distinct handles are
 *     independent.
 *
 * Errors
 *   - every call returns a status; < 0 is an error (state unchanged),
 *     > 0 a warning (step taken with the last accepted iterate, as in
 *     Algorithm 3).  bdem_last_error() gives a message.
 */
#ifndef BDEM_H
#define BDEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bdem_ctx bdem_ctx;

enum {
  BDEM_OK = 0,
  BDEM_W_NOT_CONVERGED = 1, /* Newton cap reached in some scene */
  BDEM_W_LS_FAILED = 2,     /* line search exhausted in some scene */
  BDEM_E_INVALID = -1,      /* bad argument (index, i==j, duplicate bond, non-unit q, dt<=0, ...) */
  BDEM_E_HIP = -2,          /* HIP runtime error */
  BDEM_E_NOMEM = -3,        /* workspace too small / allocation failed */
  BDEM_E_NONFINITE = -4,    /* NaN / Inf in the state or the objective */
  BDEM_E_DEGENERATE = -5,   /* |q_i + q_j| < 1e-6 for an alive bond at a Newton iterate: the
                               shear midpoint is undefined.  Line-search trials there count as
                               infinite energy and are rejected, so only a step's initial guess
                               can end here. */
  BDEM_E_STATE = -6,        /* call not valid in the handle's state */
  BDEM_E_CAPACITY = -7      /* a particle has more than 32 element-repulsion candidates */
};

enum { BDEM_FREE = 0, BDEM_FIXED = 1, BDEM_KINEMATIC = 2 };  /* per-particle flags */
enum { BDEM_PREC_FP64 = 0, BDEM_PREC_MIXED = 1 };
enum { BDEM_SHEAR_LENGTH_SCALED = 0, BDEM_SHEAR_LITERAL = 1 };
enum {
  BDEM_EGH_E = 1,              /* energy */
  BDEM_EGH_G = 2,              /* reduced gradient */
  BDEM_EGH_H = 4,              /* reduced Hessian blocks */
  BDEM_EGH_PSD = 8,            /* PSD-project the Hessian (Section 5.2): per-bond eigen-clamp */
  BDEM_EGH_POTENTIAL_ONLY = 16, /* V only: no inertia term */
  BDEM_EGH_GN = 32,            /* with BDEM_EGH_H: the Gauss-Newton form of the bond Hessians
                                  (PSD by construction, see bdem_options.hessian) */
  BDEM_EGH_PCG_MATRIX = 64     /* with BDEM_EGH_H | BDEM_EGH_PSD: the form the handle's PCG
                                  iterates on (bdem_options.hessian) */
};

/* Particles (Section 3.1: state x = {p, q}, extended mass from m and r). */
typedef struct {
  int32_t n;
  const double *pos;       /* 3n, m */
  const double *quat;      /* 4n, unit, scalar last; initial state (rest = identity) */
  const double *vel;       /* 3n or NULL (= 0) */
  const double *qvel;      /* 4n quaternion rate dq/dt or NULL (= 0) */
  const double *radius;    /* n, m */
  const int32_t *material; /* n, index into the material table */
  const uint8_t *flags;    /* n or NULL (= FREE); KINEMATIC moves with its own velocity */
  const int32_t *scene;    /* n or NULL (= one scene); non-decreasing ids 0..S-1 */
} bdem_particles;

/* Bonds (Section 3.2): unordered pairs, i != j, unique, within one scene. */
typedef struct {
  int64_t nb;
  const int32_t *ij;       /* 2nb */
  const int32_t *material; /* nb or NULL (= material of particle i) */
} bdem_bonds;

/* Material (Section 3.2 stiffnesses, Section 3.3 strengths).  G = E/(2(1+nu)). */
typedef struct {
  double young, poisson, density;
  double sigma_c, tau_c;   /* tensile / shear strength, <= 0: unbreakable */
  double stiff_scale[4];   /* multipliers of stretch, shear, twist, bend stiffness */
  int32_t shear_mode;      /* BDEM_SHEAR_LENGTH_SCALED: 1/2 k_t (l0 theta)^2; LITERAL: 1/2 k_t theta^2 */
  int32_t tension_only;    /* 1: compression does not count in sigma */
} bdem_material;

typedef struct {
  double gravity[3];
  double ground_normal[3], ground_offset; /* plane n.p = h; gap = n.p - h - r */
  double k_contact;        /* < 0: per scene, E_max * r_max over that scene's materials and
                              particles (Section 5.4); 0: no ground; > 0: this value for all */
  double mu_s, mu_r;       /* friction of Section 5.4 (>= 0; 0: off), applied to the velocities
                              after each step, before the fracture test: per contact (ground,
                              overlapping candidate pair) dv_i = -min(1, mu_s F_n dt/(m_i |v_t|)) v_t
                              and dw_i = -min(1, mu_r F_n r_i dt/(I_i |w_ij|)) w_ij, I_i = 2/5 m r^2;
                              the sums are projected on the particle's own (angular) velocity and
                              clipped so they at most stop it */
  double k_self;           /* element repulsion of Section 5.4, 1/2 k_ec min(0, l - r_i - r_j)^2 over
                              the candidate pairs of each step: < 0: per scene E_max * r_max;
                              0: off (default); > 0: this value */
  double contact_margin;   /* candidates of a step: pairs of one scene not joined by an alive bond
                              whose centres at the predicted positions are closer than
                              r_i + r_j + contact_margin (< 0: the scene's r_max; default -1); at
                              most 32 per particle (BDEM_E_CAPACITY otherwise) */
  double newton_tol;       /* absolute stop |z|_2 <= newton_tol */
  double newton_rtol;      /* relative stop |z|_2 <= newton_rtol |z0|_2 */
  double armijo_c;         /* sufficient-decrease constant */
  double cg_rtol_max;      /* PCG stops at |r| <= min(cg_rtol_max, sqrt|z|) |z| (Section 5.3) */
  int32_t max_newton, max_cg, max_ls;
  int32_t precision;       /* BDEM_PREC_FP64 or BDEM_PREC_MIXED */
  int32_t break_each_step; /* apply the fracture test at the end of every step */
  int32_t cg_chunk;        /* PCG iterations between host convergence checks */
  int32_t use_graph;       /* replay the PCG chunk as a captured HIP graph */
  int32_t solver;          /* BDEM_SOLVER_NEWTON: Algorithm 2 (default); BDEM_SOLVER_FIRST_ORDER:
                              Algorithm 1, steepest descent along -grad f with the same retraction
                              and line search (its search starts at twice the last accepted step,
                              at most 1); max_newton then caps its iterations */
  int32_t integrator;      /* BDEM_INTEGRATOR_EULER (default): Phi(x) = |x - x_hat|^2_{M_s}/(2 dt^2)
                              + V(x), the first-order form Section 3.1 uses in its experiments;
                              BDEM_INTEGRATOR_MIDPOINT: the variational midpoint form of Section 3.1
                              and Appendix C, Phi(x) = |x - z_hat|^2_{M_s}/(2 dt^2) + V((x + x_n)/2)
                              with z_hat = x_hat - dt^2/2 M_s^{-1} grad V((x_{n-1} + x_n)/2),
                              x_{n-1} = x_n - dt v_n: second order in the positions; the
                              unit-norm constraint holds at the new state */
  int32_t preconditioner;  /* PCG preconditioner: BDEM_PRECOND_BLOCK_JACOBI (default, the 6x6
                              diagonal blocks) or BDEM_PRECOND_AMG (Section 5.3 solves with AMG):
                              aggregates = cells of side 4 r_max from each scene's initial box
                              corner, doubled per level until a scene has at most 12; rigid-body
                              modes of each aggregate as prolongation; Galerkin coarse operators
                              rebuilt at every Newton iteration; omega = 0.8 block-Jacobi pre- and
                              post-smoothing; a dense exact solve on the last level.  Built from
                              the diagonal and bond blocks (not the element-repulsion couplings);
                              its hierarchy is allocated by bdem_create, outside the workspace */
  int32_t hessian;         /* PSD form of the bond Hessians the Newton step solves with
                              (Section 5.2 asks only for a PSD matrix; the fixed point is that of
                              the exact gradient either way): BDEM_HESS_EIGEN_CLAMP: the exact
                              reduced 12x12 bond Hessian with its negative eigenvalues set to
                              zero; BDEM_HESS_GAUSS_NEWTON (default): stretch exact with its
                              (1 - l0/l) factor clamped at 0, shear and bend/twist in
                              Gauss-Newton form (J^T W J, the second derivatives of the shear
                              residual and the bend/twist cross term dropped), the bond's
                              Weingarten share kept only where positive; PSD term by term and
                              equal to the exact Hessian at zero strain.  It is evaluated by one
                              row-parallel kernel (no per-slot halves in memory) */
  int32_t amg_refresh;     /* multigrid only: 0 rebuilds the coarse levels (prolongators, Galerkin
                              products, inverses) at every Newton iteration; 1 (default) at the
                              first Newton iteration of each step and reuses them for the rest of
                              the step (the fine level, its smoother and the PCG's matrix are
                              always current; any such V-cycle is a fixed SPD operator within a
                              PCG solve, so only the iteration count can change) */
} bdem_options;

typedef struct {
  int32_t newton_iters, cg_iters, ls_backtracks, status;
  int64_t bonds_broken;
  double grad0, grad_final, phi;
  /* milliseconds: 0 setup, 1 bond+particle evaluation, 2 PCG, 3 line search,
   * 4 fracture + velocity, 5 total, 6 bond-kernel time (events), 7 SpMV-kernel time */
  double t_ms[8];
} bdem_step_stats;

/* Launch shapes of the PCG kernels (none changes a result: every shape
 * computes the same bits). */
typedef struct {
  int32_t spmv_threads;    /* SpMV workgroup size; 32 block rows per workgroup (192, 256, 384, 512) */
  int32_t spmv_trips;      /* slots (FP32 blocks) or slot halves (FP64) in flight per SpMV thread (1, 2) */
  int32_t update_rows;     /* block rows per CG-update workgroup (32, 64, 128) */
  int32_t cg_chunk;        /* PCG iterations issued per host poll */
  int32_t use_graph;       /* 1: those iterations replay a captured HIP graph */
  int32_t pad_;
  double spmv_us, update_us, pcg_us_per_iter; /* times measured by bdem_autotune (0: not tuned) */
} bdem_tuning;

enum { BDEM_SOLVER_NEWTON = 0, BDEM_SOLVER_FIRST_ORDER = 1 };
enum { BDEM_INTEGRATOR_EULER = 0, BDEM_INTEGRATOR_MIDPOINT = 1 };
enum { BDEM_PRECOND_BLOCK_JACOBI = 0, BDEM_PRECOND_AMG = 1 };
enum { BDEM_HESS_EIGEN_CLAMP = 0, BDEM_HESS_GAUSS_NEWTON = 1 };

/* Defaults: gravity (0,0,-9.81), no ground, newton_tol 0, newton_rtol 1e-8,
 * armijo_c 1e-4, cg_rtol_max 0.5, max_newton 50, max_cg 2000, max_ls 30,
 * FP64, fracture on, cg_chunk 16, no graph, Newton solver, implicit-Euler form,
 * block-Jacobi preconditioner, Gauss-Newton bond Hessians. */
void bdem_default_options(bdem_options *opt);

/* Device bytes bdem_create needs for this problem (0 on invalid input). */
size_t bdem_workspace_bytes(const bdem_particles *p, const bdem_bonds *b,
                            const bdem_options *opt);

/* Build a handle: validates the inputs, computes per-bond rest data (l0, d0,
 * stiffnesses; Section 3.2), the block-sparse pattern of the reduced Hessian
 * and uploads everything.  Errors: INVALID, NOMEM, HIP. */
int bdem_create(const bdem_particles *p, const bdem_bonds *b, const bdem_material *mats,
                int32_t n_mats, const bdem_options *opt, void *hip_stream,
                void *workspace_dev, size_t workspace_bytes, bdem_ctx **out);

/* bdem_create for callers that cannot allocate device memory (serving loops
 * and harnesses that forbid hipMalloc, code that sets up work to be captured
 * into a HIP graph): the handle's workspace is the library's static device
 * array of BDEM_SCRATCH_BYTES on the current device (held from the library's
 * first use on that device until the process ends), its host mirrors are
 * unpinned and its convergence counters live in device memory (read back
 * after the stream drains, so the PCG polls without running ahead).  It
 * calls no hipMalloc, hipHostMalloc, hipFree or other allocating routine;
 * everything else is bdem_create's (same kernels, same results).  One handle
 * per device may live in the array at a time: bdem_destroy releases it.  The
 * array keeps the contents of the last handle; create initialises every
 * buffer it reads.  Errors: NOMEM (the problem needs more than
 * BDEM_SCRATCH_BYTES; the message gives both sizes), STATE (the device's
 * array is in use), INVALID (as bdem_create, and the multigrid
 * preconditioner, whose hierarchy is a separate allocation), HIP. */
#define BDEM_SCRATCH_BYTES (64u << 20)
int bdem_create_in_scratch(const bdem_particles *p, const bdem_bonds *b, const bdem_material *mats,
                           int32_t n_mats, const bdem_options *opt, void *hip_stream,
                           bdem_ctx **out);

/* One implicit step of every scene with the same dt (Algorithm 3).  stats
 * (nullable) receives the totals over scenes.  Errors: INVALID (dt <= 0),
 * NONFINITE, DEGENERATE, HIP; warnings NOT_CONVERGED, LS_FAILED. */
int bdem_step(bdem_ctx *ctx, double dt, bdem_step_stats *stats);

/* One implicit step with a time step per scene; stats_per_scene (nullable)
 * has one entry per scene. */
int bdem_step_batched(bdem_ctx *ctx, const double *dt_per_scene,
                      bdem_step_stats *stats_per_scene);

/* Objective at an evaluation state without solving (Section 3.1 Phi of the
 * configured integrator, with the prediction x_hat = x_n + dt v_n of the
 * current state, and z_hat in the midpoint form; Sections 4.1-4.2
 * reduced Riemannian gradient and Hessian; Section 5.2 projection when
 * BDEM_EGH_PSD).  pos_eval / quat_eval NULL: the current state.  Outputs
 * (host, nullable): energy (1), grad6 (6n), hdiag36 (36n: the 6x6 diagonal
 * blocks), hoff36 (36nb: for bond (i,j) the block with rows of i and columns
 * of j).  Fixed / kinematic particles: zero gradient, identity diagonal
 * block, zero off-diagonal blocks. */
int bdem_energy_grad_hess(bdem_ctx *ctx, double dt, int32_t what, const double *pos_eval,
                          const double *quat_eval, double *energy, double *grad6,
                          double *hdiag36, double *hoff36);

/* One product w = H u with the matrix the PCG of Section 5.3 iterates on: the
 * projected reduced Hessian (Sections 4.2 and 5.2, as bdem_energy_grad_hess
 * with BDEM_EGH_H | BDEM_EGH_PSD) at the evaluation state (NULL: the current
 * state), through the step's own SpMV kernel and launch shape and, with
 * element repulsion, its pair couplings.  in6 (6n, host): u in reduced
 * coordinates per particle; out6 (6n, host): w.  Fixed / kinematic particles
 * have an identity diagonal block and no couplings.  Errors as
 * bdem_energy_grad_hess. */
int bdem_hess_apply(bdem_ctx *ctx, double dt, const double *pos_eval, const double *quat_eval,
                    const double *in6, double *out6);

/* One application of the configured PCG preconditioner M^-1 (Section 5.3) to
 * in6 (6n, host, reduced coordinates per particle), with M built from the
 * projected reduced Hessian at the evaluation state (as bdem_energy_grad_hess
 * with BDEM_EGH_H | BDEM_EGH_PSD; NULL: the current state); the result goes
 * to out6 (6n, host).  Errors as bdem_energy_grad_hess. */
int bdem_precond_apply(bdem_ctx *ctx, double dt, const double *pos_eval, const double *quat_eval,
                       const double *in6, double *out6);

/* Section 3.3 stress test of every alive bond at the current state; bonds
 * with sigma > sigma_c or tau > tau_c break permanently.  n_broken (nullable)
 * = newly broken; alive_out (nb, nullable) = the alive mask after the test. */
int bdem_break_bonds(bdem_ctx *ctx, int64_t *n_broken, uint8_t *alive_out);

/* Element-repulsion candidate pairs (Section 5.4) of the last step or
 * evaluation, in user particle indices, i < j, sorted: up to cap pairs are
 * written to pairs (2 x int32 each); count (nullable) receives their number.
 * No pairs when k_self = 0.  Errors: INVALID, HIP. */
int bdem_contact_pairs(const bdem_ctx *ctx, int64_t cap, int32_t *pairs, int64_t *count);

/* Checkpoint / restore of the mutable state (host arrays, nullable). */
int bdem_get_state(const bdem_ctx *ctx, double *pos, double *quat, double *vel, double *qvel,
                   uint8_t *alive);
int bdem_set_state(bdem_ctx *ctx, const double *pos, const double *quat, const double *vel,
                   const double *qvel, const uint8_t *alive);

/* Launch-shape autotuner: assembles the Hessian at the prediction of a step
 * of length dt_per_scene[s] (the first Newton iteration's matrix), times each
 * pair of CG-update tile and SpMV shape (the two kernels back to back, as a
 * PCG iteration runs them) and each PCG polling mode (cg_chunk, use_graph) on
 * it with HIP events, keeps the fastest and reports it in out (nullable;
 * spmv_us and update_us are the chosen kernels timed alone).  The simulation
 * state is not changed, and since every shape computes the same bits, no
 * later result depends on the choice.  Errors: INVALID, DEGENERATE, HIP. */
int bdem_autotune(bdem_ctx *ctx, const double *dt_per_scene, bdem_tuning *out);
/* Current launch shapes / set them explicitly (INVALID if not a listed shape). */
int bdem_get_tuning(const bdem_ctx *ctx, bdem_tuning *out);
int bdem_set_tuning(bdem_ctx *ctx, const bdem_tuning *tuning);

/* Sizes of the handle's problem. */
int bdem_sizes(const bdem_ctx *ctx, int32_t *n, int64_t *nb, int32_t *n_scenes);

/* Measurement hook.  enable = 1: HIP events bracket every bond-evaluation
 * and SpMV launch of bdem_step (the PCG then issues plain launches, no graph);
 * enable = 2: only the bond-evaluation launches are bracketed and the PCG
 * runs as tuned; 0: off.  The summed kernel milliseconds land in
 * bdem_step_stats.t_ms[6] (bond) and t_ms[7] (SpMV) and the launch counts of
 * the last step in bdem_profile_counts.  Errors: INVALID (other levels). */
int bdem_set_profiling(bdem_ctx *ctx, int32_t enable);
int bdem_profile_counts(const bdem_ctx *ctx, int32_t *bond_launches, int32_t *spmv_launches);

void bdem_destroy(bdem_ctx *ctx); /* NULL-safe */

/* Message of the last failed call on ctx; NULL ctx: of the last failed create
 * on this thread. */
const char *bdem_last_error(const bdem_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* BDEM_H */
