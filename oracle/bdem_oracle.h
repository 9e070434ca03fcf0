/*
 * FP64 CPU oracle for implicit bonded DEM with manifold Newton
 * (Lu, Cao, Li, Hu: "Implicit Bonded Discrete Element Method with Manifold
 * Optimization").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the GPU path is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code with the
 * GPU library.
 *
 * Conventions: quaternions (x, y, z, w), scalar last (Appendix A).
 * Per-particle flags: 0 free, 1 fixed, 2 kinematic.
 * Reduced coordinates: 6 per particle, (dp, y) with dq = G_l(q)^T y
 * (Section 4.2 nullspace reduction).
 */
#ifndef BDEM_ORACLE_H
#define BDEM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_sys orc_sys;

/* material row: young, poisson, density, sigma_c, tau_c, s_stretch, s_shear,
 * s_twist, s_bend, shear_mode (0: length scaled, 1: literal), tension_only */
#define ORC_MAT_STRIDE 11
/* env: gravity[3], ground_normal[3], ground_offset, k_contact,
 * k_self, contact_margin, mu_s, mu_r
 * (k_contact, k_self < 0: E_max * r_max, 0: off; contact_margin < 0: r_max) */
#define ORC_ENV_LEN 12

orc_sys *orc_create(int32_t n, const double *pos, const double *quat, const double *vel,
                    const double *qvel, const double *radius, const int32_t *pmat,
                    const uint8_t *flags, int64_t nb, const int32_t *ij,
                    const int32_t *bmat, int32_t nmat, const double *mat, const double *env);
void orc_destroy(orc_sys *s);
const char *orc_last_error(void);

int orc_get_state(const orc_sys *s, double *pos, double *quat, double *vel, double *qvel,
                  uint8_t *alive);
int orc_set_state(orc_sys *s, const double *pos, const double *quat, const double *vel,
                  const double *qvel, const uint8_t *alive);

/* Euclidean energy / gradient (14) / Hessian (14x14 row-major) of one bond at
 * the given endpoint states; variable order (p_i, q_i, p_j, q_j). */
int orc_bond_eval(const orc_sys *s, int64_t b, const double *pi, const double *qi,
                  const double *pj, const double *qj, double *energy, double *g14,
                  double *h14);
/* the three energy parts (stretch, shear, bend/twist) of one bond */
int orc_bond_energy_parts(const orc_sys *s, int64_t b, const double *pi, const double *qi,
                          const double *pj, const double *qj, double *parts3);
/* reduced Riemannian gradient (12) and Hessian (12x12) of one bond, PSD
 * projected when psd != 0; order (p_i, y_i, p_j, y_j). */
int orc_bond_reduced(const orc_sys *s, int64_t b, const double *pi, const double *qi,
                     const double *pj, const double *qj, int psd, double *g12, double *h12);
/* stresses of one bond (Section 3.3) at the given state arrays */
int orc_bond_stress(const orc_sys *s, int64_t b, const double *pos, const double *quat,
                    double *sigma, double *tau);

/* stresses of every bond (alive or not) at the given state */
int orc_stresses(const orc_sys *s, const double *pos, const double *quat, double *sigma,
                 double *tau);

/* predicted state of a step: p_hat (3n), q_hat (4n) */
int orc_predict(const orc_sys *s, double dt, double *p_hat, double *q_hat);

/* Phi at (pos, quat) with the prediction of the current state and dt.
 * potential_only != 0: V only (bonds + gravity + ground, no inertia). */
int orc_energy(orc_sys *s, double dt, const double *pos, const double *quat,
               int potential_only, double *phi);

/* z_hat = x_hat - 1/2 M_s^{-1} dt^2 grad V((x_{i-1} + x_i)/2) of the
 * variational midpoint form (Section 3.1, Appendix C), with x_i the current
 * state, x_hat its prediction and x_{i-1} = 2 x_i - x_hat; grad V is the
 * Euclidean gradient over (p, q).  Particles that are not unknowns keep
 * z_hat = x_hat.  zp (3n), zq (4n). */
int orc_midpoint_target(const orc_sys *s, double dt, double *zp, double *zq);

/* The objective of a step: midpoint = 0 is orc_energy / orc_energy_grad_hess;
 * midpoint = 1: Phi(x) = 1/(2 dt^2)|x - z_hat|^2_{M_s} + V((x + x_i)/2), whose
 * Euclidean gradient and Hessian carry V's at the midpoint times 1/2 and 1/4,
 * reduced at the quaternions of x. */
int orc_objective(orc_sys *s, double dt, int midpoint, const double *pos,
                  const double *quat, int potential_only, double *phi);
int orc_objective_grad_hess(orc_sys *s, double dt, int midpoint, const double *pos,
                            const double *quat, int psd, double *phi, double *z, double *hdiag,
                            double *hoff);

/* Phi, reduced gradient z (6n) and reduced Hessian: diagonal blocks hdiag
 * (36n, row-major 6x6) and one off-diagonal block per bond hoff (36nb, the
 * (i,j) block, rows of i, columns of j).  Any output may be NULL.  Broken
 * bonds contribute nothing.  Fixed / kinematic particles: z = 0, diagonal
 * block = identity, off-diagonal blocks touching them = 0. */
int orc_energy_grad_hess(orc_sys *s, double dt, const double *pos, const double *quat,
                         int psd, double *phi, double *z, double *hdiag, double *hoff);

/* Element repulsion (Section 5.4): the candidate pairs of a step are every
 * pair i < j not joined by an alive bond whose centres at the positions p
 * are closer than r_i + r_j + margin; the step takes them at its predicted
 * positions, and orc_energy / orc_objective* rebuild them from the prediction
 * of the current state.  Returns their number.  orc_contacts copies up to
 * cap pairs (2 x int32 each) and returns the number.  The couplings of the
 * last Hessian evaluation enter orc_hess_apply and orc_pcg. */
int64_t orc_contact_candidates(orc_sys *s, const double *p);
int64_t orc_contacts(const orc_sys *s, int32_t *pairs, int64_t cap);
/* friction of Section 5.4 applied to the current velocities */
void orc_friction(orc_sys *s, double dt);

/* One V-cycle of the aggregation multigrid preconditioner on b (6n): x (6n)
 * ~ H^-1 b with H the diagonal (hdiag) and bond (hoff) blocks of
 * orc_energy_grad_hess at the state (pos, quat) the prolongation is built
 * from.  Aggregates: cells of side 4 r_max from the initial box corner
 * (doubled per level); rigid-body-mode prolongation; Galerkin coarse
 * operators; omega = 0.8 block-Jacobi pre- and post-smoothing; exact solve
 * on the first level with <= 12 nodes.  Returns the number of coarse levels,
 * -1 if the coarsest operator is singular. */
int orc_amg_apply(const orc_sys *s, const double *pos, const double *quat, const double *hdiag,
                  const double *hoff, const double *b, double *x);

/* y = H x with the blocks of orc_energy_grad_hess */
void orc_hess_apply(const orc_sys *s, const double *hdiag, const double *hoff,
                    const double *x, double *y);

/* block-Jacobi PCG on H y = b; returns iterations (negative on breakdown) */
int orc_pcg(const orc_sys *s, const double *hdiag, const double *hoff, const double *b,
            double rtol, int max_iter, double *y, double *res_out);

/* symmetric k x k: negative eigenvalues set to zero (cyclic Jacobi) */
int orc_psd_project(int k, const double *a, double *out);

/* Appendix A operators: Q_l (4x4), Q_r (4x4), G_l (3x4), product, rotation */
void orc_quat_matrices(const double *q, double *Ql, double *Qr, double *Gl);
void orc_quat_mul(const double *a, const double *b, double *c);
void orc_quat_rotate(const double *q, const double *d0, double *d);

/* exp map on S^3 followed by normalisation (Section 4.1) */
void orc_quat_exp_step(const double *q, const double *dq, double alpha, double *out);

typedef struct {
  double tol_abs, tol_rel;   /* Newton stop: |z| <= max(tol_abs, tol_rel |z0|) */
  double cg_rtol;            /* linear solve relative tolerance */
  double armijo_c;
  int32_t max_newton, max_cg, max_ls, break_bonds;
  int32_t first_order;       /* 1: Algorithm 1 (Riemannian gradient descent) instead of Algorithm 2 */
  int32_t midpoint;          /* 1: the variational midpoint objective of Section 3.1 */
  int32_t cg_forcing;        /* 1: each linear solve stops at the relative residual
                                min(cg_rtol, sqrt|z|) of Section 5.3 instead of cg_rtol */
} orc_options;

typedef struct {
  int32_t newton_iters, cg_iters, ls_backtracks, status;
  int64_t bonds_broken;
  double grad0, grad_final, phi;
} orc_stats;

void orc_default_options(orc_options *o);
/* one implicit time step (Algorithm 3 with Algorithm 2 inside, or with
 * Algorithm 1 when first_order is set) */
int orc_step(orc_sys *s, double dt, const orc_options *o, orc_stats *st);
/* stress test of every alive bond at the current state; breaks are permanent */
int orc_break_bonds(orc_sys *s, int64_t *n_broken);

#ifdef __cplusplus
}
#endif
#endif
