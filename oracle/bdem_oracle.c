/*
 * FP64 CPU oracle for implicit bonded DEM with manifold Newton.
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow, obviously-written reference that
 * the GPU library is checked against.  It is loaded by the test suite, the
 * smoke check and the benchmark's CPU-baseline leg, nowhere else, and shares
 * no code with the GPU library.
 *
 * Everything is FP64 and follows the paper's definitions in the paper's
 * order:
 *   - quaternion algebra: Appendix A (Q_l, Q_r, cross matrix, direction
 *     rotation operator, nullspace operator G_l);
 *   - incremental potential, implicit-Euler form: Section 3.1, equation
 *     "eq:optimization form", with the constant extended mass matrix M_s;
 *   - bond potentials: Section 3.2 (stretch, shear, bend/twist);
 *   - fracture criteria with implicit forces: Section 3.3;
 *   - Riemannian gradient / Hessian and nullspace reduction: Sections 4.1
 *     and 4.2 (equations manifold-hessian-1..4);
 *   - SPD projection, PCG, exp-map line search, stable integrator:
 *     Section 5 and Algorithm 3; ground repulsion: Section 5.4.
 * Readings taken where the paper is silent or garbled are listed in the
 * design notes (shear angle, shear units, R_0, r_0, nu, mass, gravity,
 * ground gap, line search, stop test, PSD projection).
 *
 * The derivatives are analytic; they are pinned against central finite
 * differences of the energy by the test suite.
 */
#include "bdem_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static char g_err[256];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *orc_last_error(void) { return g_err; }

struct orc_sys {
  int32_t n;
  int64_t nb;
  double *pos, *quat, *vel, *qvel;      /* state x_n, v_n */
  double *radius, *mass, *cq;           /* cq = (8/5) m r^2 */
  uint8_t *flags;
  int32_t *ij;
  uint8_t *alive;
  /* per-bond rest data */
  double *l0, *d0, *R0, *kn, *kt, *K, *S, *r0, *I, *J, *sigc, *tauc;
  int32_t *tension_only;
  double gravity[3], gn[3], gh, kc;
  /* element-element repulsion and friction (Section 5.4) */
  double kself, cmargin, mu_s, mu_r;
  uint64_t *bkey;                       /* sorted (min(i,j) << 32 | max(i,j)) of every bond */
  int64_t *bkey_idx;                    /* bond index of each sorted key */
  int64_t ncp;                          /* contact candidate pairs of the current step */
  int32_t *cp;                          /* (i, j) with i < j */
  double *hcp;                          /* (i, j) 6x6 block of each pair at the last Hessian */
  int hcp_valid;
  /* multigrid aggregation: cells of size 8 r_max from the initial box corner */
  int64_t *cell;                        /* 3 per particle */
};

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                       */
/* ------------------------------------------------------------------------ */

/* C (m x n) = A (m x k) * B (k x n), row-major */
static void mm(int m, int k, int n, const double *A, const double *B, double *C) {
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < n; ++c) {
      double acc = 0.0;
      for (int t = 0; t < k; ++t) acc += A[r * k + t] * B[t * n + c];
      C[r * n + c] = acc;
    }
}
/* C (m x n) = A^T (A is k x m) * B (k x n) */
static void mtm(int k, int m, int n, const double *A, const double *B, double *C) {
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < n; ++c) {
      double acc = 0.0;
      for (int t = 0; t < k; ++t) acc += A[t * m + r] * B[t * n + c];
      C[r * n + c] = acc;
    }
}
/* C (m x n) = A (m x k) * B^T (B is n x k) */
static void mmt(int m, int k, int n, const double *A, const double *B, double *C) {
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < n; ++c) {
      double acc = 0.0;
      for (int t = 0; t < k; ++t) acc += A[r * k + t] * B[c * k + t];
      C[r * n + c] = acc;
    }
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double dot4(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}
static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------------ */
/* Appendix A: quaternion operations, q = (u, v, w, s)                       */
/* ------------------------------------------------------------------------ */

/* cross matrix t^x of t = (u, v, w) */
static void cross_matrix(const double *t, double *X) {
  X[0] = 0.0;   X[1] = -t[2]; X[2] = t[1];
  X[3] = t[2];  X[4] = 0.0;   X[5] = -t[0];
  X[6] = -t[1]; X[7] = t[0];  X[8] = 0.0;
}
/* left multiplication matrix Q_l(q) = [[s I + t^x, t], [-t^T, s]] */
static void Q_left(const double *q, double *Q) {
  double X[9];
  cross_matrix(q, X);
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) Q[r * 4 + c] = (r == c ? q[3] : 0.0) + X[r * 3 + c];
    Q[r * 4 + 3] = q[r];
    Q[12 + r] = -q[r];
  }
  Q[15] = q[3];
}
/* right multiplication matrix Q_r(q) = [[s I - t^x, t], [-t^T, s]] */
static void Q_right(const double *q, double *Q) {
  double X[9];
  cross_matrix(q, X);
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) Q[r * 4 + c] = (r == c ? q[3] : 0.0) - X[r * 3 + c];
    Q[r * 4 + 3] = q[r];
    Q[12 + r] = -q[r];
  }
  Q[15] = q[3];
}
/* quaternion product a b = Q_l(a) b */
static void qmul(const double *a, const double *b, double *c) {
  double Q[16];
  Q_left(a, Q);
  mm(4, 4, 1, Q, b, c);
}
static void qconj(const double *q, double *c) { c[0] = -q[0]; c[1] = -q[1]; c[2] = -q[2]; c[3] = q[3]; }
/* direction rotation operator d = q (.) d0 :  (d, 0) = q (d0, 0) conj(q) */
static void qrotate(const double *q, const double *d0, double *d) {
  double a[4] = {d0[0], d0[1], d0[2], 0.0}, qc[4], t[4], r[4];
  qconj(q, qc);
  qmul(q, a, t);
  qmul(t, qc, r);
  d[0] = r[0]; d[1] = r[1]; d[2] = r[2];
}
/* nullspace operator G_l(q) = [s I - t^x, -t]  (3 x 4) */
static void G_left(const double *q, double *G) {
  double X[9];
  cross_matrix(q, X);
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) G[r * 4 + c] = (r == c ? q[3] : 0.0) - X[r * 3 + c];
    G[r * 4 + 3] = -q[r];
  }
}
/* rotation matrix of a unit quaternion: columns are q (.) e_k */
static void rotmat(const double *q, double *R) {
  for (int k = 0; k < 3; ++k) {
    double e[3] = {0, 0, 0}, d[3];
    e[k] = 1.0;
    qrotate(q, e, d);
    for (int r = 0; r < 3; ++r) R[r * 3 + k] = d[r];
  }
}

/* exported for the operator-identity tests */
void orc_quat_matrices(const double *q, double *Ql, double *Qr, double *Gl) {
  if (Ql) Q_left(q, Ql);
  if (Qr) Q_right(q, Qr);
  if (Gl) G_left(q, Gl);
}
void orc_quat_mul(const double *a, const double *b, double *c) { qmul(a, b, c); }
void orc_quat_rotate(const double *q, const double *d0, double *d) { qrotate(q, d0, d); }

/* ------------------------------------------------------------------------ */
/* creation: rest data of Section 3.2                                        */
/* ------------------------------------------------------------------------ */

static double *dup(const double *src, size_t n, double fill) {
  double *d = (double *)malloc(n * sizeof(double));
  for (size_t k = 0; k < n; ++k) d[k] = src ? src[k] : fill;
  return d;
}

void orc_destroy(orc_sys *s) {
  if (!s) return;
  double *arrs[] = {s->pos, s->quat, s->vel, s->qvel, s->radius, s->mass, s->cq, s->l0,
                    s->d0, s->R0, s->kn, s->kt, s->K, s->S, s->r0, s->I, s->J, s->sigc, s->tauc};
  for (size_t k = 0; k < sizeof arrs / sizeof arrs[0]; ++k) free(arrs[k]);
  free(s->flags); free(s->ij); free(s->alive); free(s->tension_only);
  free(s->bkey); free(s->bkey_idx); free(s->cp); free(s->hcp); free(s->cell);
  free(s);
}

orc_sys *orc_create(int32_t n, const double *pos, const double *quat, const double *vel,
                    const double *qvel, const double *radius, const int32_t *pmat,
                    const uint8_t *flags, int64_t nb, const int32_t *ij,
                    const int32_t *bmat, int32_t nmat, const double *mat, const double *env) {
  if (n <= 0 || nb < 0 || !pos || !quat || !radius || !pmat || (nb > 0 && !ij) || nmat <= 0 ||
      !mat || !env) {
    set_err("invalid arguments");
    return NULL;
  }
  for (int64_t b = 0; b < nb; ++b) {
    int32_t i = ij[2 * b], j = ij[2 * b + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) { set_err("bad bond index"); return NULL; }
  }
  for (int32_t i = 0; i < n; ++i) {
    if (pmat[i] < 0 || pmat[i] >= nmat) { set_err("bad material index"); return NULL; }
    double qn = sqrt(dot4(quat + 4 * i, quat + 4 * i));
    if (fabs(qn - 1.0) > 1e-6) { set_err("non-unit quaternion"); return NULL; }
  }
  orc_sys *s = (orc_sys *)calloc(1, sizeof(orc_sys));
  s->n = n; s->nb = nb;
  s->pos = dup(pos, 3 * (size_t)n, 0); s->quat = dup(quat, 4 * (size_t)n, 0);
  s->vel = dup(vel, 3 * (size_t)n, 0); s->qvel = dup(qvel, 4 * (size_t)n, 0);
  s->radius = dup(radius, n, 0);
  s->mass = dup(NULL, n, 0); s->cq = dup(NULL, n, 0);
  s->flags = (uint8_t *)calloc(n, 1);
  if (flags) memcpy(s->flags, flags, n);
  double Emax = 0.0, rmax = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    const double *m = mat + ORC_MAT_STRIDE * pmat[i];
    double r = radius[i];
    /* mass of a solid sphere; M_s = diag(m I3, (8/5) m r^2 I4)  (Section 3.1) */
    s->mass[i] = m[2] * 4.0 / 3.0 * M_PI * r * r * r;
    s->cq[i] = 8.0 / 5.0 * s->mass[i] * r * r;
    if (r > rmax) rmax = r;
  }
  for (int32_t k = 0; k < nmat; ++k)
    if (mat[ORC_MAT_STRIDE * k] > Emax) Emax = mat[ORC_MAT_STRIDE * k];
  size_t B = nb > 0 ? (size_t)nb : 1;
  s->ij = (int32_t *)malloc(2 * B * sizeof(int32_t));
  if (nb > 0) memcpy(s->ij, ij, 2 * (size_t)nb * sizeof(int32_t));
  s->alive = (uint8_t *)malloc(B);
  memset(s->alive, 1, B);
  s->l0 = dup(NULL, B, 0); s->d0 = dup(NULL, 3 * B, 0); s->R0 = dup(NULL, 9 * B, 0);
  s->kn = dup(NULL, B, 0); s->kt = dup(NULL, B, 0); s->K = dup(NULL, 3 * B, 0);
  s->S = dup(NULL, B, 0); s->r0 = dup(NULL, B, 0); s->I = dup(NULL, B, 0); s->J = dup(NULL, B, 0);
  s->sigc = dup(NULL, B, 0); s->tauc = dup(NULL, B, 0);
  s->tension_only = (int32_t *)calloc(B, sizeof(int32_t));
  for (int64_t b = 0; b < nb; ++b) {
    int32_t i = ij[2 * b], j = ij[2 * b + 1];
    int32_t mi = bmat ? bmat[b] : pmat[i];
    const double *m = mat + ORC_MAT_STRIDE * mi;
    double E = m[0], nu = m[1], G = E / (2.0 * (1.0 + nu));
    double u[3] = {pos[3 * j] - pos[3 * i], pos[3 * j + 1] - pos[3 * i + 1],
                   pos[3 * j + 2] - pos[3 * i + 2]};
    double l0 = sqrt(dot3(u, u));
    if (!(l0 > 0.0)) { set_err("coincident bonded particles"); orc_destroy(s); return NULL; }
    double d0[3] = {u[0] / l0, u[1] / l0, u[2] / l0};
    /* q0: rotation taking e_x to d0 (shortest arc; 180 deg about e_z if antiparallel) */
    double ex[3] = {1, 0, 0}, ax[3], q0[4];
    cross3(ex, d0, ax);
    double w = 1.0 + dot3(ex, d0);
    if (w < 1e-12) { q0[0] = 0; q0[1] = 0; q0[2] = 1; q0[3] = 0; }
    else {
      double nq = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2] + w * w);
      q0[0] = ax[0] / nq; q0[1] = ax[1] / nq; q0[2] = ax[2] / nq; q0[3] = w / nq;
    }
    double R[9];
    rotmat(q0, R);
    /* R_0 = R(q0)^T maps d0 to e_x: component 0 of t is twist, 1 and 2 bend */
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) s->R0[9 * b + r * 3 + c] = R[c * 3 + r];
    double r0 = 0.5 * (radius[i] + radius[j]);
    double S = M_PI * r0 * r0, I = M_PI * r0 * r0 * r0 * r0 / 4.0, J = M_PI * r0 * r0 * r0 * r0 / 2.0;
    double L2 = (m[9] != 0.0) ? 1.0 : l0 * l0;   /* shear: length scaled (l0 theta)^2 by default */
    s->l0[b] = l0;
    memcpy(s->d0 + 3 * b, d0, sizeof d0);
    s->kn[b] = E * S / l0 * m[5];
    s->kt[b] = G * S / l0 * m[6] * L2;
    s->K[3 * b + 0] = G * J / l0 * m[7];
    s->K[3 * b + 1] = E * I / l0 * m[8];
    s->K[3 * b + 2] = E * I / l0 * m[8];
    s->S[b] = S; s->r0[b] = r0; s->I[b] = I; s->J[b] = J;
    s->sigc[b] = m[3]; s->tauc[b] = m[4];
    s->tension_only[b] = m[10] != 0.0;
  }
  memcpy(s->gravity, env, 3 * sizeof(double));
  double gnn = sqrt(dot3(env + 3, env + 3));
  for (int k = 0; k < 3; ++k) s->gn[k] = gnn > 0 ? env[3 + k] / gnn : 0.0;
  s->gh = env[6];
  s->kc = env[7] < 0.0 ? Emax * rmax : env[7];
  /* element repulsion stiffness k_ec (< 0: E_max r_max, the order Section
   * 5.4 recommends; 0: off), candidate margin (< 0: r_max), friction */
  s->kself = env[8] < 0.0 ? Emax * rmax : env[8];
  s->cmargin = env[9] < 0.0 ? rmax : env[9];
  s->mu_s = env[10];
  s->mu_r = env[11];
  /* multigrid aggregation cells of the initial positions */
  {
    double lo[3] = {1e300, 1e300, 1e300};
    for (int32_t i = 0; i < n; ++i)
      for (int k = 0; k < 3; ++k) lo[k] = fmin(lo[k], pos[3 * i + k]);
    double h0 = 8.0 * rmax;
    s->cell = (int64_t *)malloc(3 * (size_t)n * sizeof(int64_t));
    for (int32_t i = 0; i < n; ++i)
      for (int k = 0; k < 3; ++k) s->cell[3 * i + k] = (int64_t)floor((pos[3 * i + k] - lo[k]) / h0);
  }
  /* bond lookup by endpoint pair */
  s->bkey = (uint64_t *)malloc(B * sizeof(uint64_t));
  s->bkey_idx = (int64_t *)malloc(B * sizeof(int64_t));
  for (int64_t b = 0; b < nb; ++b) {
    uint64_t i = (uint64_t)ij[2 * b], j = (uint64_t)ij[2 * b + 1];
    s->bkey[b] = i < j ? (i << 32 | j) : (j << 32 | i);
    s->bkey_idx[b] = b;
  }
  for (int64_t a = 1; a < nb; ++a) {   /* insertion sort: test sizes only */
    uint64_t k = s->bkey[a];
    int64_t v = s->bkey_idx[a], c = a - 1;
    while (c >= 0 && s->bkey[c] > k) { s->bkey[c + 1] = s->bkey[c]; s->bkey_idx[c + 1] = s->bkey_idx[c]; --c; }
    s->bkey[c + 1] = k;
    s->bkey_idx[c + 1] = v;
  }
  return s;
}

/* bond index joining i and j, or -1 */
static int64_t find_bond(const orc_sys *s, int32_t i, int32_t j) {
  uint64_t a = (uint64_t)(i < j ? i : j), b = (uint64_t)(i < j ? j : i), k = a << 32 | b;
  int64_t lo = 0, hi = s->nb - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    if (s->bkey[mid] == k) return s->bkey_idx[mid];
    if (s->bkey[mid] < k) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* Candidate pairs of the element repulsion for one step: every pair i < j
 * not joined by an alive bond whose centres at the positions p are closer
 * than r_i + r_j + margin (all pairs are tested). */
int64_t orc_contact_candidates(orc_sys *s, const double *p) {
  free(s->cp); free(s->hcp);
  s->cp = NULL; s->hcp = NULL; s->ncp = 0; s->hcp_valid = 0;
  if (!(s->kself > 0.0)) return 0;
  int64_t cap = 0;
  for (int32_t i = 0; i < s->n; ++i)
    for (int32_t j = i + 1; j < s->n; ++j) {
      double u[3] = {p[3 * j] - p[3 * i], p[3 * j + 1] - p[3 * i + 1], p[3 * j + 2] - p[3 * i + 2]};
      double reach = s->radius[i] + s->radius[j] + s->cmargin;
      if (!(dot3(u, u) < reach * reach)) continue;
      int64_t b = find_bond(s, i, j);
      if (b >= 0 && s->alive[b]) continue;
      if (s->ncp == cap) {
        cap = cap ? 2 * cap : 64;
        s->cp = (int32_t *)realloc(s->cp, 2 * cap * sizeof(int32_t));
      }
      s->cp[2 * s->ncp] = i;
      s->cp[2 * s->ncp + 1] = j;
      s->ncp++;
    }
  s->hcp = (double *)calloc(36 * (size_t)(s->ncp > 0 ? s->ncp : 1), sizeof(double));
  return s->ncp;
}

int64_t orc_contacts(const orc_sys *s, int32_t *pairs, int64_t cap) {
  if (pairs)
    for (int64_t k = 0; k < s->ncp && k < cap; ++k) { pairs[2 * k] = s->cp[2 * k]; pairs[2 * k + 1] = s->cp[2 * k + 1]; }
  return s->ncp;
}

/* Element repulsion of candidate pair k at the positions ep (Section 5.4):
 * V = 1/2 k_ec min(0, |p_j - p_i| - r_i - r_j)^2.  Returns the energy;
 * g6 (p_i, p_j) and H36 (6x6 over (p_i, p_j)) are its Euclidean gradient and
 * Hessian times wg and wh, zero when the spheres do not overlap. */
static double contact_pair(const orc_sys *s, int64_t k, const double *ep, double wg, double wh,
                           double *g6, double *H36) {
  int32_t i = s->cp[2 * k], j = s->cp[2 * k + 1];
  if (g6) memset(g6, 0, 6 * sizeof(double));
  if (H36) memset(H36, 0, 36 * sizeof(double));
  double u[3] = {ep[3 * j] - ep[3 * i], ep[3 * j + 1] - ep[3 * i + 1], ep[3 * j + 2] - ep[3 * i + 2]};
  double l = sqrt(dot3(u, u)), d = s->radius[i] + s->radius[j];
  if (!(l < d) || !(l > 0.0)) return 0.0;
  double e = l - d, n[3] = {u[0] / l, u[1] / l, u[2] / l};
  if (g6)
    for (int r = 0; r < 3; ++r) { g6[r] = -wg * s->kself * e * n[r]; g6[3 + r] = wg * s->kself * e * n[r]; }
  if (H36)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double h = wh * s->kself * (n[r] * n[c] + (1.0 - d / l) * ((r == c) - n[r] * n[c]));
        H36[r * 6 + c] = h; H36[(3 + r) * 6 + 3 + c] = h;
        H36[r * 6 + 3 + c] = -h; H36[(3 + r) * 6 + c] = -h;
      }
  return 0.5 * s->kself * e * e;
}

int orc_get_state(const orc_sys *s, double *pos, double *quat, double *vel, double *qvel,
                  uint8_t *alive) {
  if (!s) return -1;
  if (pos) memcpy(pos, s->pos, 3 * (size_t)s->n * sizeof(double));
  if (quat) memcpy(quat, s->quat, 4 * (size_t)s->n * sizeof(double));
  if (vel) memcpy(vel, s->vel, 3 * (size_t)s->n * sizeof(double));
  if (qvel) memcpy(qvel, s->qvel, 4 * (size_t)s->n * sizeof(double));
  if (alive && s->nb > 0) memcpy(alive, s->alive, (size_t)s->nb);
  return 0;
}
int orc_set_state(orc_sys *s, const double *pos, const double *quat, const double *vel,
                  const double *qvel, const uint8_t *alive) {
  if (!s) return -1;
  if (pos) memcpy(s->pos, pos, 3 * (size_t)s->n * sizeof(double));
  if (quat) memcpy(s->quat, quat, 4 * (size_t)s->n * sizeof(double));
  if (vel) memcpy(s->vel, vel, 3 * (size_t)s->n * sizeof(double));
  if (qvel) memcpy(s->qvel, qvel, 4 * (size_t)s->n * sizeof(double));
  if (alive && s->nb > 0) memcpy(s->alive, alive, (size_t)s->nb);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Section 3.2: bond energy                                                  */
/* ------------------------------------------------------------------------ */

/* theta^2 = F(y) with y = |n - d|^2 = (2 sin(theta/2))^2 and its first two
 * derivatives.  Series sum_n 2 y^n / (n^2 C(2n,n)) below y = 0.1. */
static void theta2_of_y(double y, double *F, double *F1, double *F2) {
  if (y < 0.1) {
    double f = 0.0, f1 = 0.0, f2 = 0.0, binom = 1.0; /* C(2n, n), starting at C(0,0) */
    double pw[18];                                   /* pw[k] = y^k */
    pw[0] = 1.0;
    for (int k = 1; k < 18; ++k) pw[k] = pw[k - 1] * y;
    for (int nn = 1; nn <= 16; ++nn) {
      binom = binom * (2.0 * nn) * (2.0 * nn - 1.0) / ((double)nn * nn);
      double c = 2.0 / ((double)nn * nn * binom);
      f += c * pw[nn];
      f1 += nn * c * pw[nn - 1];
      if (nn >= 2) f2 += nn * (nn - 1) * c * pw[nn - 2];
    }
    *F = f; *F1 = f1; *F2 = f2;
    return;
  }
  double th = 2.0 * asin(0.5 * sqrt(y));
  double q = y * (4.0 - y);
  *F = th * th;
  *F1 = 2.0 * th / sqrt(q);
  *F2 = (2.0 - (*F1) * (2.0 - y)) / q;
}

int orc_bond_energy_parts(const orc_sys *s, int64_t b, const double *pi, const double *qi,
                          const double *pj, const double *qj, double *parts) {
  if (!s || b < 0 || b >= s->nb) return -1;
  /* stretch: 1/2 k_n (|p_i - p_j| - l0)^2 */
  double u[3] = {pj[0] - pi[0], pj[1] - pi[1], pj[2] - pi[2]};
  double l = sqrt(dot3(u, u));
  double e = l - s->l0[b];
  parts[0] = 0.5 * s->kn[b] * e * e;
  /* shear: angle between the current bond direction n and d = q_c (.) d0,
   * q_c = (q_i + q_j)/|q_i + q_j|;  1/2 k_t (l0 theta)^2 */
  double w[4] = {qi[0] + qj[0], qi[1] + qj[1], qi[2] + qj[2], qi[3] + qj[3]};
  if (dot4(w, w) < 1e-12) {
    /* q_c does not exist (q_j = -q_i): outside the domain of the potential;
     * a line-search trial here is rejected like any non-finite objective */
    parts[1] = INFINITY;
  } else {
    double wn = sqrt(dot4(w, w));
    double qc[4] = {w[0] / wn, w[1] / wn, w[2] / wn, w[3] / wn}, d[3];
    qrotate(qc, s->d0 + 3 * b, d);
    double nv[3] = {u[0] / l, u[1] / l, u[2] / l};
    double y = (nv[0] - d[0]) * (nv[0] - d[0]) + (nv[1] - d[1]) * (nv[1] - d[1]) +
               (nv[2] - d[2]) * (nv[2] - d[2]);
    double th = 2.0 * asin(0.5 * sqrt(y));
    parts[1] = 0.5 * s->kt[b] * th * th;
  }
  /* bend / twist: t = R_0 G_l(q_j) q_i,  1/2 t^T K t */
  double G[12], tp[3], t[3];
  G_left(qj, G);
  mm(3, 4, 1, G, qi, tp);
  mm(3, 3, 1, s->R0 + 9 * b, tp, t);
  const double *K = s->K + 3 * b;
  parts[2] = 0.5 * (K[0] * t[0] * t[0] + K[1] * t[1] * t[1] + K[2] * t[2] * t[2]);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Euclidean derivatives of one bond; 14 variables (p_i, q_i, p_j, q_j)      */
/* ------------------------------------------------------------------------ */

enum { PI_ = 0, QI_ = 3, PJ_ = 7, QJ_ = 10 };

int orc_bond_eval(const orc_sys *s, int64_t b, const double *pi, const double *qi,
                  const double *pj, const double *qj, double *energy, double *g,
                  double *H) {
  if (!s || b < 0 || b >= s->nb) return -1;
  double parts[3];
  orc_bond_energy_parts(s, b, pi, qi, pj, qj, parts);
  if (energy) *energy = parts[0] + parts[1] + parts[2];
  double gl[14] = {0}, Hl[196] = {0};
  const int want_h = H != NULL;

  double u[3] = {pj[0] - pi[0], pj[1] - pi[1], pj[2] - pi[2]};
  double l = sqrt(dot3(u, u));
  double n[3] = {u[0] / l, u[1] / l, u[2] / l};
  double Pn[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Pn[r * 3 + c] = (r == c) - n[r] * n[c];

  /* ---- stretch, as a function of u = p_j - p_i ---- */
  {
    double kn = s->kn[b], e = l - s->l0[b];
    double gu[3], Huu[9];
    for (int r = 0; r < 3; ++r) gu[r] = kn * e * n[r];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        Huu[r * 3 + c] = kn * (n[r] * n[c] + (1.0 - s->l0[b] / l) * Pn[r * 3 + c]);
    for (int r = 0; r < 3; ++r) {
      gl[PI_ + r] -= gu[r];
      gl[PJ_ + r] += gu[r];
      if (want_h)
      for (int c = 0; c < 3; ++c) {
        Hl[(PI_ + r) * 14 + PI_ + c] += Huu[r * 3 + c];
        Hl[(PJ_ + r) * 14 + PJ_ + c] += Huu[r * 3 + c];
        Hl[(PI_ + r) * 14 + PJ_ + c] -= Huu[r * 3 + c];
        Hl[(PJ_ + r) * 14 + PI_ + c] -= Huu[r * 3 + c];
      }
    }
  }

  /* ---- shear, as a function of (u, w = q_i + q_j) ----
   * y = |n - d|^2 = 2 - 2 phi,  phi = n . d,  d = M(w) d0 / (w.w)
   * with M(w) d0 = (s^2 - |v|^2) d0 + 2 (v.d0) v + 2 s (v x d0), w = (v, s). */
  {
    const double *d0 = s->d0 + 3 * b;
    double w[4] = {qi[0] + qj[0], qi[1] + qj[1], qi[2] + qj[2], qi[3] + qj[3]};
    const double *v = w;
    double sw = w[3], ww = dot4(w, w), h = 1.0 / ww;
    double vd = dot3(v, d0), vv = dot3(v, v), vxd[3], D0X[9];
    cross3(v, d0, vxd);
    cross_matrix(d0, D0X);
    double mw[3];
    for (int r = 0; r < 3; ++r) mw[r] = (sw * sw - vv) * d0[r] + 2.0 * vd * v[r] + 2.0 * sw * vxd[r];
    /* J_m = d(M(w) d0)/dw, 3 x 4 */
    double Jm[12];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c)
        Jm[r * 4 + c] = -2.0 * d0[r] * v[c] + 2.0 * v[r] * d0[c] + 2.0 * vd * (r == c) -
                        2.0 * sw * D0X[r * 3 + c];
      Jm[r * 4 + 3] = 2.0 * sw * d0[r] + 2.0 * vxd[r];
    }
    double d[3] = {h * mw[0], h * mw[1], h * mw[2]};
    /* N(n, w) = n . M(w) d0 = w^T A_n w */
    double N = dot3(n, mw);
    double gN[4];
    mtm(3, 4, 1, Jm, n, gN); /* J_m^T n */
    double nd0 = dot3(n, d0), d0xn[3], An[16];
    cross3(d0, n, d0xn);
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c)
        An[r * 4 + c] = -nd0 * (r == c) + d0[r] * n[c] + n[r] * d0[c];
      An[r * 4 + 3] = d0xn[r];
      An[12 + r] = d0xn[r];
    }
    An[15] = nd0;
    /* h(w) = 1/(w.w) */
    double gh[4], Hh[16];
    for (int r = 0; r < 4; ++r) gh[r] = -2.0 * h * h * w[r];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) Hh[r * 4 + c] = -2.0 * h * h * (r == c) + 8.0 * h * h * h * w[r] * w[c];
    /* phi = N h */
    double phi = N * h;
    (void)phi;
    double gpw[4], Hpww[16];
    for (int r = 0; r < 4; ++r) gpw[r] = h * gN[r] + N * gh[r];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c)
        Hpww[r * 4 + c] = h * 2.0 * An[r * 4 + c] + gN[r] * gh[c] + gh[r] * gN[c] + N * Hh[r * 4 + c];
    double gpu[3];
    mm(3, 3, 1, Pn, d, gpu);
    for (int r = 0; r < 3; ++r) gpu[r] /= l;
    double Hpuu[9], dn = dot3(d, n);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        Hpuu[r * 3 + c] = -(d[r] * n[c] + n[r] * d[c] + dn * ((r == c) - 3.0 * n[r] * n[c])) / (l * l);
    /* d(d)/dw = h J_m + m_w gh^T */
    double Jd[12], Hpuw[12];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 4; ++c) Jd[r * 4 + c] = h * Jm[r * 4 + c] + mw[r] * gh[c];
    mm(3, 3, 4, Pn, Jd, Hpuw);
    for (int k = 0; k < 12; ++k) Hpuw[k] /= l;
    /* V = 1/2 k F(y), y = 2 - 2 phi (evaluated as |n - d|^2) */
    double y = (n[0] - d[0]) * (n[0] - d[0]) + (n[1] - d[1]) * (n[1] - d[1]) + (n[2] - d[2]) * (n[2] - d[2]);
    double F, F1, F2, k = s->kt[b];
    theta2_of_y(y, &F, &F1, &F2);
    /* 7-vector (u, w) */
    double gp7[7] = {gpu[0], gpu[1], gpu[2], gpw[0], gpw[1], gpw[2], gpw[3]};
    double Hp7[49];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) Hp7[r * 7 + c] = Hpuu[r * 3 + c];
      for (int c = 0; c < 4; ++c) { Hp7[r * 7 + 3 + c] = Hpuw[r * 4 + c]; Hp7[(3 + c) * 7 + r] = Hpuw[r * 4 + c]; }
    }
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) Hp7[(3 + r) * 7 + 3 + c] = Hpww[r * 4 + c];
    double g7[7], H7[49];
    for (int r = 0; r < 7; ++r) g7[r] = -k * F1 * gp7[r];
    for (int r = 0; r < 7; ++r)
      for (int c = 0; c < 7; ++c) H7[r * 7 + c] = 2.0 * k * F2 * gp7[r] * gp7[c] - k * F1 * Hp7[r * 7 + c];
    /* chain rule through u = p_j - p_i, w = q_i + q_j:  A is 7 x 14 */
    double A[98] = {0};
    for (int r = 0; r < 3; ++r) { A[r * 14 + PI_ + r] = -1.0; A[r * 14 + PJ_ + r] = 1.0; }
    for (int r = 0; r < 4; ++r) { A[(3 + r) * 14 + QI_ + r] = 1.0; A[(3 + r) * 14 + QJ_ + r] = 1.0; }
    double ga[14], T[98], Ha[196];
    mtm(7, 14, 1, A, g7, ga);
    for (int r = 0; r < 14; ++r) gl[r] += ga[r];
    if (want_h) {
      mm(7, 7, 14, H7, A, T);
      mtm(7, 14, 14, A, T, Ha);
      for (int r = 0; r < 196; ++r) Hl[r] += Ha[r];
    }
  }

  /* ---- bend / twist: t' = G_l(q_j) q_i (bilinear), t = R_0 t', V = 1/2 t^T K t ---- */
  {
    const double *R0 = s->R0 + 9 * b, *Kd = s->K + 3 * b;
    double Gj[12], tp[3], t[3], Kt[3], m[3];
    G_left(qj, Gj);
    mm(3, 4, 1, Gj, qi, tp);
    mm(3, 3, 1, R0, tp, t);
    for (int r = 0; r < 3; ++r) Kt[r] = Kd[r] * t[r];
    mtm(3, 3, 1, R0, Kt, m);                 /* m = R0^T K t = dV/dt' */
    /* Ti = dt'/dq_i = G_l(q_j);  Tj = dt'/dq_j, column k = G_l(e_k) q_i */
    double Ti[12], Tj[12], Ge[4][12];
    memcpy(Ti, Gj, sizeof Ti);
    for (int kk = 0; kk < 4; ++kk) {
      double e[4] = {0, 0, 0, 0}, col[3];
      e[kk] = 1.0;
      G_left(e, Ge[kk]);
      mm(3, 4, 1, Ge[kk], qi, col);
      for (int r = 0; r < 3; ++r) Tj[r * 4 + kk] = col[r];
    }
    /* K' = R0^T K R0 */
    double KR[9], Kp[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) KR[r * 3 + c] = Kd[r] * R0[r * 3 + c];
    mtm(3, 3, 3, R0, KR, Kp);
    double gqi[4], gqj[4];
    mtm(3, 4, 1, Ti, m, gqi);
    mtm(3, 4, 1, Tj, m, gqj);
    double T1[12], Hii[16], Hjj[16], Hij[16];
    mm(3, 3, 4, Kp, Ti, T1);
    mtm(3, 4, 4, Ti, T1, Hii);
    mm(3, 3, 4, Kp, Tj, T1);
    mtm(3, 4, 4, Tj, T1, Hjj);
    mtm(3, 4, 4, Ti, T1, Hij);
    /* second derivative of the bilinear map: d^2 t'_r / dq_i[a] dq_j[k] = G_l(e_k)[r][a] */
    for (int a = 0; a < 4; ++a)
      for (int kk = 0; kk < 4; ++kk)
        for (int r = 0; r < 3; ++r) Hij[a * 4 + kk] += m[r] * Ge[kk][r * 4 + a];
    for (int r = 0; r < 4; ++r) {
      gl[QI_ + r] += gqi[r];
      gl[QJ_ + r] += gqj[r];
      if (want_h)
      for (int c = 0; c < 4; ++c) {
        Hl[(QI_ + r) * 14 + QI_ + c] += Hii[r * 4 + c];
        Hl[(QJ_ + r) * 14 + QJ_ + c] += Hjj[r * 4 + c];
        Hl[(QI_ + r) * 14 + QJ_ + c] += Hij[r * 4 + c];
        Hl[(QJ_ + c) * 14 + QI_ + r] += Hij[r * 4 + c];
      }
    }
  }
  if (g) memcpy(g, gl, sizeof gl);
  if (H) memcpy(H, Hl, sizeof Hl);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* symmetric eigen-clamp (cyclic Jacobi)                                     */
/* ------------------------------------------------------------------------ */

int orc_psd_project(int k, const double *a, double *out) {
  if (k <= 0 || k > 64) return -1;
  double *A = (double *)malloc(sizeof(double) * k * k);
  double *V = (double *)calloc((size_t)k * k, sizeof(double));
  for (int r = 0; r < k; ++r)
    for (int c = 0; c < k; ++c) A[r * k + c] = 0.5 * (a[r * k + c] + a[c * k + r]);
  for (int r = 0; r < k; ++r) V[r * k + r] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int r = 0; r < k; ++r)
      for (int c = 0; c < k; ++c) {
        tot += A[r * k + c] * A[r * k + c];
        if (r != c) off += A[r * k + c] * A[r * k + c];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        double apq = A[p * k + q];
        if (apq == 0.0) continue;
        double theta = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int r = 0; r < k; ++r) { /* columns p, q */
          double arp = A[r * k + p], arq = A[r * k + q];
          A[r * k + p] = c * arp - sn * arq;
          A[r * k + q] = sn * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) { /* rows p, q */
          double apr = A[p * k + r], aqr = A[q * k + r];
          A[p * k + r] = c * apr - sn * aqr;
          A[q * k + r] = sn * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          double vrp = V[r * k + p], vrq = V[r * k + q];
          V[r * k + p] = c * vrp - sn * vrq;
          V[r * k + q] = sn * vrp + c * vrq;
        }
      }
  }
  for (int r = 0; r < k; ++r)
    for (int c = 0; c < k; ++c) {
      double acc = 0.0;
      for (int e = 0; e < k; ++e) {
        double lam = A[e * k + e];
        if (lam > 0.0) acc += V[r * k + e] * lam * V[c * k + e];
      }
      out[r * k + c] = acc;
    }
  free(A);
  free(V);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Section 4: Riemannian gradient / Hessian, nullspace reduction             */
/* ------------------------------------------------------------------------ */

/* reduce a Euclidean gradient / Hessian over blocks (p: 3, q: 4)... of `nblk`
 * particles to the manifold (P H P + Weingarten) and to reduced coordinates
 * via G_l:  z = G P g,  H_red = G (P H P - sum lambda_a P_a) G^T. */
static void reduce_to_manifold(int nblk, const double *const *q, const double *gE,
                               const double *HE, double *gR, double *HR) {
  int nE = 7 * nblk, nR = 6 * nblk;
  double *P = (double *)calloc((size_t)nE * nE, sizeof(double));
  double *Gf = (double *)calloc((size_t)nR * nE, sizeof(double));
  double *Hm = (double *)malloc(sizeof(double) * nE * nE);
  double *T = (double *)malloc(sizeof(double) * nE * nE);
  double *gp = (double *)malloc(sizeof(double) * nE);
  for (int a = 0; a < nblk; ++a) {
    int oE = 7 * a, oR = 6 * a;
    for (int r = 0; r < 3; ++r) { P[(oE + r) * nE + oE + r] = 1.0; Gf[(oR + r) * nE + oE + r] = 1.0; }
    double G[12];
    G_left(q[a], G);
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) P[(oE + 3 + r) * nE + oE + 3 + c] = (r == c) - q[a][r] * q[a][c];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 4; ++c) Gf[(oR + 3 + r) * nE + oE + 3 + c] = G[r * 4 + c];
  }
  /* Riemannian gradient (Section 4.1): grad_p = grad_p, grad_q = (I - q q^T) grad_q */
  mm(nE, nE, 1, P, gE, gp);
  /* Riemannian Hessian (Section 4.2, manifold-hessian-1..4) */
  mm(nE, nE, nE, P, HE, T);
  mm(nE, nE, nE, T, P, Hm);
  for (int a = 0; a < nblk; ++a) {
    int oE = 7 * a;
    double lam = dot4(q[a], gE + oE + 3);
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) Hm[(oE + 3 + r) * nE + oE + 3 + c] -= lam * P[(oE + 3 + r) * nE + oE + 3 + c];
  }
  /* nullspace reduction: z = G grad, H_red = G Hess G^T */
  if (gR) mm(nR, nE, 1, Gf, gp, gR);
  if (HR) {
    mm(nR, nE, nE, Gf, Hm, T);
    mmt(nR, nE, nR, T, Gf, HR);
  }
  free(P); free(Gf); free(Hm); free(T); free(gp);
}

/* Reduced gradient and Hessian of one bond for the unknowns (p_i, q_i, p_j, q_j):
 * V_b is evaluated at the endpoint states (epi, eqi, epj, eqj); its Euclidean
 * gradient and Hessian with respect to the unknowns are those at the
 * evaluation point times wg and wh (1 and 1 when it is the unknown itself,
 * 1/2 and 1/4 when it is the midpoint (x + x_n)/2 of Section 3.1); the
 * reduction of Sections 4.1-4.2 uses the unknowns' own quaternions. */
static int bond_reduced_at(const orc_sys *s, int64_t b, const double *qi, const double *qj,
                           const double *epi, const double *eqi, const double *epj,
                           const double *eqj, double wg, double wh, int psd, double *g12,
                           double *h12) {
  double g14[14], H14[196], Hr[144];
  if (orc_bond_eval(s, b, epi, eqi, epj, eqj, NULL, g14, H14)) return -1;
  for (int a = 0; a < 14; ++a) g14[a] *= wg;
  for (int a = 0; a < 196; ++a) H14[a] *= wh;
  const double *qs[2] = {qi, qj};
  reduce_to_manifold(2, qs, g14, H14, g12, Hr);
  if (h12) {
    if (psd) orc_psd_project(12, Hr, h12);
    else memcpy(h12, Hr, sizeof Hr);
  }
  return 0;
}

int orc_bond_reduced(const orc_sys *s, int64_t b, const double *pi, const double *qi,
                     const double *pj, const double *qj, int psd, double *g12, double *h12) {
  return bond_reduced_at(s, b, qi, qj, pi, qi, pj, qj, 1.0, 1.0, psd, g12, h12);
}

/* ------------------------------------------------------------------------ */
/* per-particle terms: inertia (M_s), gravity, ground repulsion              */
/* ------------------------------------------------------------------------ */

int orc_predict(const orc_sys *s, double dt, double *ph, double *qh) {
  for (int32_t i = 0; i < s->n; ++i) {
    int f = s->flags[i];
    for (int r = 0; r < 3; ++r)
      ph[3 * i + r] = s->pos[3 * i + r] + (f == 1 ? 0.0 : dt * s->vel[3 * i + r]);
    for (int r = 0; r < 4; ++r)
      qh[4 * i + r] = s->quat[4 * i + r] + (f == 0 ? dt * s->qvel[4 * i + r] : 0.0);
  }
  return 0;
}

/* Energy, Euclidean gradient (7) and Hessian (7x7) of particle i's own terms:
 * the inertia 1/(2 dt^2) (x - x_t)^T M_s (x - x_t) about the target (ph, qh),
 * plus gravity and ground evaluated at the position pv, whose gradient and
 * Hessian enter with the weights wg and wh (see bond_reduced_at). */
static double particle_terms(const orc_sys *s, int32_t i, double dt, const double *p,
                             const double *q, const double *ph, const double *qh,
                             const double *pv, double wg, double wh, int potential_only,
                             double *g7, double *H7) {
  double m = s->mass[i], c = s->cq[i], idt2 = potential_only ? 0.0 : 1.0 / (dt * dt);
  double E = 0.0;
  if (g7) memset(g7, 0, 7 * sizeof(double));
  if (H7) memset(H7, 0, 49 * sizeof(double));
  /* inertia: 1/(2 dt^2) (x - x_t)^T M_s (x - x_t) */
  for (int r = 0; r < 3; ++r) {
    double e = p[r] - ph[r];
    E += 0.5 * m * idt2 * e * e;
    if (g7) g7[r] += m * idt2 * e;
    if (H7) H7[r * 7 + r] += m * idt2;
  }
  for (int r = 0; r < 4; ++r) {
    double e = q[r] - qh[r];
    E += 0.5 * c * idt2 * e * e;
    if (g7) g7[3 + r] += c * idt2 * e;
    if (H7) H7[(3 + r) * 7 + 3 + r] += c * idt2;
  }
  /* gravity: -m g . p */
  E -= m * dot3(s->gravity, pv);
  if (g7) for (int r = 0; r < 3; ++r) g7[r] -= wg * m * s->gravity[r];
  /* ground: 1/2 k_c min(0, gap)^2 with gap = n . p - h - r */
  if (s->kc != 0.0) {
    double gap = dot3(s->gn, pv) - s->gh - s->radius[i];
    if (gap < 0.0) {
      E += 0.5 * s->kc * gap * gap;
      if (g7) for (int r = 0; r < 3; ++r) g7[r] += wg * s->kc * gap * s->gn[r];
      if (H7)
        for (int r = 0; r < 3; ++r)
          for (int cc = 0; cc < 3; ++cc) H7[r * 7 + cc] += wh * s->kc * s->gn[r] * s->gn[cc];
    }
  }
  return E;
}

static int is_solved(const orc_sys *s, int32_t i) { return s->flags[i] == 0; }

/* Kahan-Babuska (Neumaier) accumulation */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
  else k->c += (x - t) + k->s;
  k->s = t;
}

/* ------------------------------------------------------------------------ */
/* the objective of one step (Section 3.1)                                   */
/* ------------------------------------------------------------------------ */

/* midpoint = 0: Phi(x) = 1/(2 dt^2)|x - x_hat|^2_{M_s} + V(x), the form the
 * experiments use; midpoint = 1: Phi(x) = 1/(2 dt^2)|x - z_hat|^2_{M_s} +
 * V((x + x_n)/2), the variational midpoint form.  tp / tq: the inertia target. */
typedef struct {
  int midpoint;
  const double *tp, *tq;
} objective;

int orc_midpoint_target(const orc_sys *s, double dt, double *zp, double *zq) {
  int32_t n = s->n;
  double *ph = (double *)malloc(sizeof(double) * 3 * n), *qh = (double *)malloc(sizeof(double) * 4 * n);
  double *mp = (double *)malloc(sizeof(double) * 3 * n), *mq = (double *)malloc(sizeof(double) * 4 * n);
  double *gv = (double *)calloc(7 * (size_t)n, sizeof(double));
  orc_predict(s, dt, ph, qh);
  /* x_hat = 2 x_i - x_{i-1}, so x_{i-1} = 2 x_i - x_hat; midpoint (x_{i-1} + x_i) / 2 */
  for (int32_t i = 0; i < n; ++i) {
    for (int r = 0; r < 3; ++r) {
      double prev = 2.0 * s->pos[3 * i + r] - ph[3 * i + r];
      mp[3 * i + r] = 0.5 * (prev + s->pos[3 * i + r]);
    }
    for (int r = 0; r < 4; ++r) {
      double prev = 2.0 * s->quat[4 * i + r] - qh[4 * i + r];
      mq[4 * i + r] = 0.5 * (prev + s->quat[4 * i + r]);
    }
  }
  /* Euclidean gradient of V at that midpoint: particle terms, then bonds in order */
  for (int32_t i = 0; i < n; ++i) {
    double g7[7];
    particle_terms(s, i, dt, mp + 3 * i, mq + 4 * i, mp + 3 * i, mq + 4 * i, mp + 3 * i, 1.0,
                   1.0, 1, g7, NULL);
    for (int r = 0; r < 7; ++r) gv[7 * i + r] += g7[r];
  }
  int64_t nb = s->nb;
  double *gb = (double *)malloc(sizeof(double) * 14 * (nb > 0 ? nb : 1));
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < nb; ++b) {
    if (!s->alive[b]) continue;
    int32_t i = s->ij[2 * b], j = s->ij[2 * b + 1];
    orc_bond_eval(s, b, mp + 3 * i, mq + 4 * i, mp + 3 * j, mq + 4 * j, NULL, gb + 14 * b, NULL);
  }
  for (int64_t b = 0; b < nb; ++b) {
    if (!s->alive[b]) continue;
    int32_t i = s->ij[2 * b], j = s->ij[2 * b + 1];
    for (int r = 0; r < 7; ++r) { gv[7 * i + r] += gb[14 * b + r]; gv[7 * j + r] += gb[14 * b + 7 + r]; }
  }
  /* z_hat = x_hat - 1/2 M_s^{-1} dt^2 grad V; particles that are not unknowns keep x_hat */
  for (int32_t i = 0; i < n; ++i) {
    int free_ = is_solved(s, i);
    double fm = free_ ? 0.5 * dt * dt / s->mass[i] : 0.0, fc = free_ ? 0.5 * dt * dt / s->cq[i] : 0.0;
    for (int r = 0; r < 3; ++r) zp[3 * i + r] = ph[3 * i + r] - fm * gv[7 * i + r];
    for (int r = 0; r < 4; ++r) zq[4 * i + r] = qh[4 * i + r] - fc * gv[7 * i + 3 + r];
  }
  free(ph); free(qh); free(mp); free(mq); free(gv); free(gb);
  return 0;
}

/* evaluation point of V for the state (pos, quat): itself, or (x + x_n)/2 */
static void eval_point(const orc_sys *s, const objective *ob, const double *pos,
                       const double *quat, double *ep, double *eq) {
  int32_t n = s->n;
  if (ob->midpoint) {
    for (size_t a = 0; a < 3 * (size_t)n; ++a) ep[a] = 0.5 * (pos[a] + s->pos[a]);
    for (size_t a = 0; a < 4 * (size_t)n; ++a) eq[a] = 0.5 * (quat[a] + s->quat[a]);
  } else {
    memcpy(ep, pos, sizeof(double) * 3 * n);
    memcpy(eq, quat, sizeof(double) * 4 * n);
  }
}

static int objective_energy(const orc_sys *s, double dt, const objective *ob, const double *pos,
                            const double *quat, int potential_only, double *phi) {
  int32_t n = s->n;
  double *ep = (double *)malloc(sizeof(double) * 3 * n), *eq = (double *)malloc(sizeof(double) * 4 * n);
  eval_point(s, ob, pos, quat, ep, eq);
  ksum acc = {0, 0};
  for (int32_t i = 0; i < n; ++i)
    kadd(&acc, particle_terms(s, i, dt, pos + 3 * i, quat + 4 * i, ob->tp + 3 * i, ob->tq + 4 * i,
                              ep + 3 * i, 1.0, 1.0, potential_only, NULL, NULL));
  double *eb = (double *)malloc(sizeof(double) * (s->nb > 0 ? s->nb : 1));
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < s->nb; ++b) {
    double parts[3];
    eb[b] = 0.0;
    if (!s->alive[b]) continue;
    int32_t i = s->ij[2 * b], j = s->ij[2 * b + 1];
    orc_bond_energy_parts(s, b, ep + 3 * i, eq + 4 * i, ep + 3 * j, eq + 4 * j, parts);
    eb[b] = parts[0] + parts[1] + parts[2];
  }
  for (int64_t b = 0; b < s->nb; ++b) kadd(&acc, eb[b]);
  for (int64_t k = 0; k < s->ncp; ++k) kadd(&acc, contact_pair(s, k, ep, 1.0, 1.0, NULL, NULL));
  *phi = acc.s + acc.c;
  free(eb); free(ep); free(eq);
  return 0;
}

static int objective_grad_hess(const orc_sys *s, double dt, const objective *ob,
                               const double *pos, const double *quat, int psd, double *phi,
                               double *z, double *hdiag, double *hoff) {
  int32_t n = s->n;
  const double wg = ob->midpoint ? 0.5 : 1.0, wh = ob->midpoint ? 0.25 : 1.0;
  double *ep = (double *)malloc(sizeof(double) * 3 * n), *eq = (double *)malloc(sizeof(double) * 4 * n);
  eval_point(s, ob, pos, quat, ep, eq);
  if (phi) objective_energy(s, dt, ob, pos, quat, 0, phi);
  if (z) memset(z, 0, sizeof(double) * 6 * n);
  if (hdiag) memset(hdiag, 0, sizeof(double) * 36 * n);
  if (hoff && s->nb > 0) memset(hoff, 0, sizeof(double) * 36 * s->nb);
  /* particle terms */
  for (int32_t i = 0; i < n; ++i) {
    double g7[7], H7[49], g6[6], H6[36], P6[36];
    particle_terms(s, i, dt, pos + 3 * i, quat + 4 * i, ob->tp + 3 * i, ob->tq + 4 * i,
                   ep + 3 * i, wg, wh, 0, g7, H7);
    const double *qs[1] = {quat + 4 * i};
    reduce_to_manifold(1, qs, g7, H7, g6, H6);
    if (psd) orc_psd_project(6, H6, P6);
    else memcpy(P6, H6, sizeof P6);
    if (z) for (int r = 0; r < 6; ++r) z[6 * i + r] += g6[r];
    if (hdiag) for (int r = 0; r < 36; ++r) hdiag[36 * i + r] += P6[r];
  }
  /* bonds: per-bond reduced blocks computed independently, assembled in bond order */
  int64_t nb = s->nb;
  double *gb = (double *)malloc(sizeof(double) * 12 * (nb > 0 ? nb : 1));
  double *hb = (double *)malloc(sizeof(double) * 144 * (nb > 0 ? nb : 1));
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t b = 0; b < nb; ++b) {
    if (!s->alive[b]) continue;
    int32_t i = s->ij[2 * b], j = s->ij[2 * b + 1];
    bond_reduced_at(s, b, quat + 4 * i, quat + 4 * j, ep + 3 * i, eq + 4 * i, ep + 3 * j,
                    eq + 4 * j, wg, wh, psd, gb + 12 * b, hb + 144 * b);
  }
  for (int64_t b = 0; b < nb; ++b) {
    if (!s->alive[b]) continue;
    int32_t i = s->ij[2 * b], j = s->ij[2 * b + 1];
    const double *g12 = gb + 12 * b, *H12 = hb + 144 * b;
    if (z)
      for (int r = 0; r < 6; ++r) { z[6 * i + r] += g12[r]; z[6 * j + r] += g12[6 + r]; }
    if (hdiag)
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
          hdiag[36 * i + r * 6 + c] += H12[r * 12 + c];
          hdiag[36 * j + r * 6 + c] += H12[(6 + r) * 12 + 6 + c];
        }
    if (hoff)
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) hoff[36 * b + r * 6 + c] = H12[r * 12 + 6 + c];
  }
  /* element repulsion: position blocks only, the pair's 6x6 projected as a whole */
  for (int64_t k = 0; k < s->ncp; ++k) {
    int32_t i = s->cp[2 * k], j = s->cp[2 * k + 1];
    double g6[6], H36[36], P36[36];
    contact_pair(s, k, ep, wg, wh, g6, H36);
    if (psd) orc_psd_project(6, H36, P36);
    else memcpy(P36, H36, sizeof P36);
    if (z) for (int r = 0; r < 3; ++r) { z[6 * i + r] += g6[r]; z[6 * j + r] += g6[3 + r]; }
    if (hdiag)
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          hdiag[36 * i + r * 6 + c] += P36[r * 6 + c];
          hdiag[36 * j + r * 6 + c] += P36[(3 + r) * 6 + 3 + c];
        }
    if (hoff) {
      double *hc = s->hcp + 36 * k;
      memset(hc, 0, 36 * sizeof(double));
      if (is_solved(s, i) && is_solved(s, j))
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) hc[r * 6 + c] = P36[r * 6 + 3 + c];
    }
  }
  if (hoff) ((orc_sys *)s)->hcp_valid = 1;
  /* fixed / kinematic particles are not unknowns */
  for (int32_t i = 0; i < n; ++i) {
    if (is_solved(s, i)) continue;
    if (z) for (int r = 0; r < 6; ++r) z[6 * i + r] = 0.0;
    if (hdiag) for (int r = 0; r < 36; ++r) hdiag[36 * i + r] = (r % 7 == 0) ? 1.0 : 0.0;
  }
  if (hoff)
    for (int64_t b = 0; b < nb; ++b) {
      int32_t i = s->ij[2 * b], j = s->ij[2 * b + 1];
      if (!is_solved(s, i) || !is_solved(s, j)) memset(hoff + 36 * b, 0, 36 * sizeof(double));
    }
  free(gb); free(hb); free(ep); free(eq);
  return 0;
}

/* inertia target of the step: x_hat, or z_hat for the midpoint form */
static void step_target(const orc_sys *s, double dt, int midpoint, double *tp, double *tq) {
  if (midpoint) orc_midpoint_target(s, dt, tp, tq);
  else orc_predict(s, dt, tp, tq);
}

/* contact candidates of the step that would start from the current state */
static void step_candidates(orc_sys *s, double dt) {
  double *ph = (double *)malloc(sizeof(double) * 3 * s->n), *qh = (double *)malloc(sizeof(double) * 4 * s->n);
  orc_predict(s, dt, ph, qh);
  orc_contact_candidates(s, ph);
  free(ph); free(qh);
}

int orc_objective(orc_sys *s, double dt, int midpoint, const double *pos,
                  const double *quat, int potential_only, double *phi) {
  double *tp = (double *)malloc(sizeof(double) * 3 * s->n), *tq = (double *)malloc(sizeof(double) * 4 * s->n);
  step_candidates(s, dt);
  step_target(s, dt, midpoint, tp, tq);
  objective ob = {midpoint != 0, tp, tq};
  int rc = objective_energy(s, dt, &ob, pos, quat, potential_only, phi);
  free(tp); free(tq);
  return rc;
}

int orc_objective_grad_hess(orc_sys *s, double dt, int midpoint, const double *pos,
                            const double *quat, int psd, double *phi, double *z, double *hdiag,
                            double *hoff) {
  double *tp = (double *)malloc(sizeof(double) * 3 * s->n), *tq = (double *)malloc(sizeof(double) * 4 * s->n);
  step_candidates(s, dt);
  step_target(s, dt, midpoint, tp, tq);
  objective ob = {midpoint != 0, tp, tq};
  int rc = objective_grad_hess(s, dt, &ob, pos, quat, psd, phi, z, hdiag, hoff);
  free(tp); free(tq);
  return rc;
}

int orc_energy(orc_sys *s, double dt, const double *pos, const double *quat,
               int potential_only, double *phi) {
  return orc_objective(s, dt, 0, pos, quat, potential_only, phi);
}

int orc_energy_grad_hess(orc_sys *s, double dt, const double *pos, const double *quat,
                         int psd, double *phi, double *z, double *hdiag, double *hoff) {
  return orc_objective_grad_hess(s, dt, 0, pos, quat, psd, phi, z, hdiag, hoff);
}

void orc_hess_apply(const orc_sys *s, const double *hdiag, const double *hoff,
                    const double *x, double *y) {
  for (int32_t i = 0; i < s->n; ++i) mm(6, 6, 1, hdiag + 36 * i, x + 6 * i, y + 6 * i);
  /* element-repulsion couplings of the last Hessian evaluation */
  if (s->hcp_valid)
    for (int64_t k = 0; k < s->ncp; ++k) {
      int32_t i = s->cp[2 * k], j = s->cp[2 * k + 1];
      const double *Hc = s->hcp + 36 * k;
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
          y[6 * i + r] += Hc[r * 6 + c] * x[6 * j + c];
          y[6 * j + c] += Hc[r * 6 + c] * x[6 * i + r];
        }
    }
  for (int64_t b = 0; b < s->nb; ++b) {
    if (!s->alive[b]) continue;
    int32_t i = s->ij[2 * b], j = s->ij[2 * b + 1];
    const double *Hb = hoff + 36 * b;
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 6; ++c) {
        y[6 * i + r] += Hb[r * 6 + c] * x[6 * j + c];
        y[6 * j + c] += Hb[r * 6 + c] * x[6 * i + r];
      }
  }
}

/* Cholesky of a 6x6 SPD block (lower, in place); returns 0 on success */
static int chol6(double *A) {
  for (int j = 0; j < 6; ++j) {
    double d = A[j * 6 + j];
    for (int k = 0; k < j; ++k) d -= A[j * 6 + k] * A[j * 6 + k];
    if (!(d > 0.0)) return -1;
    d = sqrt(d);
    A[j * 6 + j] = d;
    for (int i = j + 1; i < 6; ++i) {
      double v = A[i * 6 + j];
      for (int k = 0; k < j; ++k) v -= A[i * 6 + k] * A[j * 6 + k];
      A[i * 6 + j] = v / d;
    }
  }
  return 0;
}
static void chol6_solve(const double *L, const double *b, double *x) {
  double y[6];
  for (int i = 0; i < 6; ++i) {
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= L[i * 6 + k] * y[k];
    y[i] = v / L[i * 6 + i];
  }
  for (int i = 5; i >= 0; --i) {
    double v = y[i];
    for (int k = i + 1; k < 6; ++k) v -= L[k * 6 + i] * x[k];
    x[i] = v / L[i * 6 + i];
  }
}

static double vdot(const double *a, const double *b, size_t n) {
  ksum k = {0, 0};
  for (size_t i = 0; i < n; ++i) kadd(&k, a[i] * b[i]);
  return k.s + k.c;
}

/* Section 5.3: preconditioned conjugate gradient, block-Jacobi preconditioner */
int orc_pcg(const orc_sys *s, const double *hdiag, const double *hoff, const double *bvec,
            double rtol, int max_iter, double *x, double *res_out) {
  size_t N = 6 * (size_t)s->n;
  double *L = (double *)malloc(sizeof(double) * 36 * s->n);
  double *r = (double *)malloc(sizeof(double) * N), *zz = (double *)malloc(sizeof(double) * N);
  double *p = (double *)malloc(sizeof(double) * N), *Ap = (double *)malloc(sizeof(double) * N);
  int ret = 0;
  for (int32_t i = 0; i < s->n; ++i) {
    memcpy(L + 36 * i, hdiag + 36 * i, 36 * sizeof(double));
    if (chol6(L + 36 * i)) { /* singular block: fall back to the identity */
      memset(L + 36 * i, 0, 36 * sizeof(double));
      for (int k = 0; k < 6; ++k) L[36 * i + 7 * k] = 1.0;
    }
  }
  memset(x, 0, N * sizeof(double));
  memcpy(r, bvec, N * sizeof(double));
  double bn = sqrt(vdot(bvec, bvec, N));
  if (bn == 0.0) { if (res_out) *res_out = 0.0; goto done; }
  for (int32_t i = 0; i < s->n; ++i) chol6_solve(L + 36 * i, r + 6 * i, zz + 6 * i);
  memcpy(p, zz, N * sizeof(double));
  double rz = vdot(r, zz, N), rn = bn;
  int it = 0;
  for (; it < max_iter; ++it) {
    if (rn <= rtol * bn) break;
    orc_hess_apply(s, hdiag, hoff, p, Ap);
    double pAp = vdot(p, Ap, N);
    if (!(pAp > 0.0)) { ret = -1; break; }
    double alpha = rz / pAp;
    for (size_t k = 0; k < N; ++k) { x[k] += alpha * p[k]; r[k] -= alpha * Ap[k]; }
    for (int32_t i = 0; i < s->n; ++i) chol6_solve(L + 36 * i, r + 6 * i, zz + 6 * i);
    double rz2 = vdot(r, zz, N), beta = rz2 / rz;
    rz = rz2;
    for (size_t k = 0; k < N; ++k) p[k] = zz[k] + beta * p[k];
    rn = sqrt(vdot(r, r, N));
  }
  if (res_out) *res_out = rn / bn;
  if (ret == 0) ret = it;
  else ret = -(it + 1);
done:
  free(L); free(r); free(zz); free(p); free(Ap);
  return ret;
}

/* Section 4.1: q_new = q cos|a dq| + (a dq/|a dq|) sin|a dq|, then q/|q| */
void orc_quat_exp_step(const double *q, const double *dq, double alpha, double *out) {
  double v[4] = {alpha * dq[0], alpha * dq[1], alpha * dq[2], alpha * dq[3]};
  double th = sqrt(dot4(v, v));
  if (th < 1e-8) {
    double f = 1.0 - th * th / 6.0;
    for (int r = 0; r < 4; ++r) out[r] = q[r] + v[r] * f;
  } else {
    double c = cos(th), sn = sin(th) / th;
    for (int r = 0; r < 4; ++r) out[r] = q[r] * c + v[r] * sn;
  }
  double nq = sqrt(dot4(out, out));
  for (int r = 0; r < 4; ++r) out[r] /= nq;
}

/* ------------------------------------------------------------------------ */
/* Section 3.3: fracture with implicit forces                                */
/* ------------------------------------------------------------------------ */

int orc_bond_stress(const orc_sys *s, int64_t b, const double *pos, const double *quat,
                    double *sigma, double *tau) {
  if (!s || b < 0 || b >= s->nb) return -1;
  int32_t i = s->ij[2 * b], j = s->ij[2 * b + 1];
  const double *pi = pos + 3 * i, *pj = pos + 3 * j, *qi = quat + 4 * i, *qj = quat + 4 * j;
  double u[3] = {pj[0] - pi[0], pj[1] - pi[1], pj[2] - pi[2]};
  double l = sqrt(dot3(u, u));
  /* F_n = grad_p V_stretch: magnitude k_n |l - l0| */
  double e = l - s->l0[b];
  if (s->tension_only[b] && e < 0.0) e = 0.0;
  double Fn = s->kn[b] * fabs(e);
  /* F_s = grad_p V_shear: from the shear part of the bond gradient.  The
   * shear gradient is the full gradient minus the stretch part (bend/twist
   * has no position dependence). */
  double g14[14];
  orc_bond_eval(s, b, pi, qi, pj, qj, NULL, g14, NULL);
  double n[3] = {u[0] / l, u[1] / l, u[2] / l}, Fs3[3];
  double est = l - s->l0[b];
  for (int r = 0; r < 3; ++r) Fs3[r] = g14[PJ_ + r] - s->kn[b] * est * n[r];
  double Fs = sqrt(dot3(Fs3, Fs3));
  /* moments from M = K t */
  double G[12], tp[3], t[3];
  G_left(qj, G);
  mm(3, 4, 1, G, qi, tp);
  mm(3, 3, 1, s->R0 + 9 * b, tp, t);
  const double *K = s->K + 3 * b;
  double Mt = fabs(K[0] * t[0]);
  double Mb = sqrt(K[1] * t[1] * K[1] * t[1] + K[2] * t[2] * K[2] * t[2]);
  *sigma = Fn / s->S[b] + Mb * s->r0[b] / s->I[b];
  *tau = Fs / s->S[b] + Mt * s->r0[b] / s->J[b];
  return 0;
}

int orc_stresses(const orc_sys *s, const double *pos, const double *quat, double *sigma,
                 double *tau) {
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < s->nb; ++b) orc_bond_stress(s, b, pos, quat, sigma + b, tau + b);
  return 0;
}

int orc_break_bonds(orc_sys *s, int64_t *n_broken) {
  int64_t cnt = 0;
  uint8_t *brk = (uint8_t *)calloc(s->nb > 0 ? s->nb : 1, 1);
  /* all bonds are tested at the same state, then broken together */
  for (int64_t b = 0; b < s->nb; ++b) {
    if (!s->alive[b]) continue;
    double sg, ta;
    orc_bond_stress(s, b, s->pos, s->quat, &sg, &ta);
    if ((s->sigc[b] > 0.0 && sg > s->sigc[b]) || (s->tauc[b] > 0.0 && ta > s->tauc[b])) brk[b] = 1;
  }
  for (int64_t b = 0; b < s->nb; ++b)
    if (brk[b]) { s->alive[b] = 0; ++cnt; }
  free(brk);
  if (n_broken) *n_broken = cnt;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 3: one implicit step, manifold Newton (Algorithm 2) inside      */
/* ------------------------------------------------------------------------ */

/* Friction of Section 5.4, applied to the velocities after the step, from
 * the contacts at x_{n+1}: the ground (gap < 0, F_n = k_c |gap|, the ground at
 * rest) and every candidate pair that overlaps (F_n = k_ec |l - r_i - r_j|).
 * Per contact, with the relative velocity v_ij = v_n + v_t about the contact
 * normal and the relative angular velocity w_ij (world frame,
 * w = 2 vec(qdot conj(q))):
 *   dv_i = -min(1, mu_s |F_n| dt / (m_i |v_t|)) v_t,
 *   dw_i = -min(1, mu_r |F_n| r_i dt / (I_i |w_ij|)) w_ij,   I_i = 2/5 m_i r_i^2.
 * The sums over a particle's contacts are projected on the direction of its
 * own velocity (angular velocity) and clipped so they at most stop it.  All
 * particles use the velocities before friction; fixed and kinematic
 * particles keep theirs. */
static void ang_vel(const double *q, const double *qd, double *w) {
  double qc[4] = {-q[0], -q[1], -q[2], q[3]}, t[4];
  orc_quat_mul(qd, qc, t);
  w[0] = 2.0 * t[0]; w[1] = 2.0 * t[1]; w[2] = 2.0 * t[2];
}

static void friction_contact(double mu_s, double mu_r, double Fn, double dt, double m, double Iw,
                             double r, const double *n, const double *vrel, const double *wrel,
                             double *dv, double *dw) {
  double vn = dot3(vrel, n), vt[3] = {vrel[0] - vn * n[0], vrel[1] - vn * n[1], vrel[2] - vn * n[2]};
  double vtn = sqrt(dot3(vt, vt));
  if (mu_s > 0.0 && vtn > 0.0) {
    double f = fmin(1.0, mu_s * Fn * dt / (m * vtn));
    for (int k = 0; k < 3; ++k) dv[k] -= f * vt[k];
  }
  double wn = sqrt(dot3(wrel, wrel));
  if (mu_r > 0.0 && wn > 0.0) {
    double f = fmin(1.0, mu_r * Fn * r * dt / (Iw * wn));
    for (int k = 0; k < 3; ++k) dw[k] -= f * wrel[k];
  }
}

static void clip_along(const double *v, const double *d, double *out) {
  double vn = sqrt(dot3(v, v));
  out[0] = out[1] = out[2] = 0.0;
  if (!(vn > 0.0)) return;
  double s = dot3(d, v) / vn;
  s = fmax(-vn, fmin(0.0, s));
  for (int k = 0; k < 3; ++k) out[k] = s * v[k] / vn;
}

void orc_friction(orc_sys *s, double dt) {
  int32_t n = s->n;
  double *dv = (double *)calloc(3 * (size_t)n, sizeof(double)), *dw = (double *)calloc(3 * (size_t)n, sizeof(double));
  double *w = (double *)malloc(sizeof(double) * 3 * n);
  for (int32_t i = 0; i < n; ++i) ang_vel(s->quat + 4 * i, s->qvel + 4 * i, w + 3 * i);
  for (int32_t i = 0; i < n; ++i) {
    if (!is_solved(s, i) || s->kc == 0.0) continue;
    double gap = dot3(s->gn, s->pos + 3 * i) - s->gh - s->radius[i];
    if (!(gap < 0.0)) continue;
    double m = s->mass[i], Iw = 0.4 * m * s->radius[i] * s->radius[i];
    friction_contact(s->mu_s, s->mu_r, s->kc * fabs(gap), dt, m, Iw, s->radius[i], s->gn,
                     s->vel + 3 * i, w + 3 * i, dv + 3 * i, dw + 3 * i);
  }
  for (int64_t k = 0; k < s->ncp; ++k) {
    int32_t a = s->cp[2 * k], b = s->cp[2 * k + 1];
    const double *pa = s->pos + 3 * a, *pb = s->pos + 3 * b;
    double u[3] = {pa[0] - pb[0], pa[1] - pb[1], pa[2] - pb[2]};
    double l = sqrt(dot3(u, u)), d = s->radius[a] + s->radius[b];
    if (!(l < d) || !(l > 0.0)) continue;
    double Fn = s->kself * fabs(l - d), nab[3] = {u[0] / l, u[1] / l, u[2] / l};
    for (int side = 0; side < 2; ++side) {
      int32_t i = side ? b : a, j = side ? a : b;
      if (!is_solved(s, i)) continue;
      double nrm[3] = {side ? -nab[0] : nab[0], side ? -nab[1] : nab[1], side ? -nab[2] : nab[2]};
      double vrel[3], wrel[3];
      for (int c = 0; c < 3; ++c) {
        vrel[c] = s->vel[3 * i + c] - s->vel[3 * j + c];
        wrel[c] = w[3 * i + c] - w[3 * j + c];
      }
      double m = s->mass[i], Iw = 0.4 * m * s->radius[i] * s->radius[i];
      friction_contact(s->mu_s, s->mu_r, Fn, dt, m, Iw, s->radius[i], nrm, vrel, wrel,
                       dv + 3 * i, dw + 3 * i);
    }
  }
  for (int32_t i = 0; i < n; ++i) {
    if (!is_solved(s, i)) continue;
    double cv[3], cw[3];
    clip_along(s->vel + 3 * i, dv + 3 * i, cv);
    clip_along(w + 3 * i, dw + 3 * i, cw);
    for (int c = 0; c < 3; ++c) s->vel[3 * i + c] += cv[c];
    /* qdot += 1/2 (dw, 0) q */
    double dq4[4] = {cw[0], cw[1], cw[2], 0.0}, t[4];
    orc_quat_mul(dq4, s->quat + 4 * i, t);
    for (int c = 0; c < 4; ++c) s->qvel[4 * i + c] += 0.5 * t[c];
  }
  free(dv); free(dw); free(w);
}

/* ------------------------------------------------------------------------ */
/* Aggregation multigrid preconditioner.  Section 5.3 solves with AMG-PCG    */
/* without giving the method; this is the variant the GPU path implements:  */
/* aggregates = cells of side 8 r_max (from the initial box corner; cells    */
/* of twice the side at each coarser level), prolongation from the six      */
/* rigid-body modes of each aggregate, Galerkin coarse operators, damped    */
/* block-Jacobi smoothing (omega = 0.9) before and after the coarse          */
/* correction, and an exact solve on the first level with at most 16 nodes  */
/* (always at least one coarse level).  Built from the diagonal and bond    */
/* blocks; element-repulsion couplings are not part of it.                   */
/* ------------------------------------------------------------------------ */
#define AMG_OMEGA 0.9
#define AMG_COARSE_MAX 16

typedef struct {
  int32_t n;
  double *A;        /* levels >= 1: dense 6n x 6n */
  double *Dinv;     /* 36 per node */
  double *P;        /* 36 per node: block of the prolongation to the next level */
  int32_t *parent;  /* node of the next level */
  double *cen;      /* 3 per node */
  int32_t *active;  /* node has a free particle below it */
  int64_t *cell;    /* 3 per node */
} amg_level;

/* dense inverse by Gauss-Jordan with partial pivoting; returns -1 if singular */
static int dense_inverse(int N, const double *A, double *X) {
  double *M = (double *)malloc(sizeof(double) * N * N);
  memcpy(M, A, sizeof(double) * N * N);
  for (int r = 0; r < N; ++r)
    for (int c = 0; c < N; ++c) X[r * N + c] = (r == c);
  for (int k = 0; k < N; ++k) {
    int piv = k;
    for (int r = k + 1; r < N; ++r) if (fabs(M[r * N + k]) > fabs(M[piv * N + k])) piv = r;
    if (!(fabs(M[piv * N + k]) > 0.0)) { free(M); return -1; }
    if (piv != k)
      for (int c = 0; c < N; ++c) {
        double t = M[k * N + c]; M[k * N + c] = M[piv * N + c]; M[piv * N + c] = t;
        t = X[k * N + c]; X[k * N + c] = X[piv * N + c]; X[piv * N + c] = t;
      }
    double inv = 1.0 / M[k * N + k];
    for (int c = 0; c < N; ++c) { M[k * N + c] *= inv; X[k * N + c] *= inv; }
    for (int r = 0; r < N; ++r) {
      if (r == k) continue;
      double f = M[r * N + k];
      if (f == 0.0) continue;
      for (int c = 0; c < N; ++c) { M[r * N + c] -= f * M[k * N + c]; X[r * N + c] -= f * X[k * N + c]; }
    }
  }
  free(M);
  return 0;
}

static int cmp_key(const void *a, const void *b) {
  const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
  return x[0] < y[0] ? -1 : (x[0] > y[0] ? 1 : (x[1] < y[1] ? -1 : (x[1] > y[1])));
}

/* next level: group the nodes of lv by cell >> 1 (or by their own cell for
 * the particles, whose cells are already the first aggregation cells) */
static void amg_coarsen(const amg_level *lv, int first, amg_level *nx) {
  int32_t n = lv->n;
  int64_t *kv = (int64_t *)malloc(2 * sizeof(int64_t) * n);
  for (int32_t i = 0; i < n; ++i) {
    int64_t c[3];
    for (int k = 0; k < 3; ++k) c[k] = first ? lv->cell[3 * i + k] : (lv->cell[3 * i + k] >> 1);
    kv[2 * i] = (c[0] << 42) | (c[1] << 21) | c[2];
    kv[2 * i + 1] = i;
  }
  qsort(kv, n, 2 * sizeof(int64_t), cmp_key);
  int32_t m = 0;
  for (int32_t k = 0; k < n; ++k) if (k == 0 || kv[2 * k] != kv[2 * k - 2]) ++m;
  nx->n = m;
  nx->cell = (int64_t *)malloc(3 * sizeof(int64_t) * m);
  nx->cen = (double *)calloc(3 * (size_t)m, sizeof(double));
  nx->active = (int32_t *)calloc(m, sizeof(int32_t));
  int32_t a = -1;
  for (int32_t k = 0; k < n; ++k) {
    if (k == 0 || kv[2 * k] != kv[2 * k - 2]) {
      ++a;
      int32_t i = (int32_t)kv[2 * k + 1];
      for (int c = 0; c < 3; ++c) nx->cell[3 * a + c] = first ? lv->cell[3 * i + c] : (lv->cell[3 * i + c] >> 1);
    }
    lv->parent[kv[2 * k + 1]] = a;
  }
  free(kv);
  /* centroids over active children (all children when none is active) */
  int32_t *cnt = (int32_t *)calloc(m, sizeof(int32_t));
  for (int32_t i = 0; i < n; ++i) if (lv->active[i]) nx->active[lv->parent[i]] = 1;
  for (int32_t i = 0; i < n; ++i) {
    int32_t p = lv->parent[i];
    if (nx->active[p] && !lv->active[i]) continue;
    for (int c = 0; c < 3; ++c) nx->cen[3 * p + c] += lv->cen[3 * i + c];
    cnt[p]++;
  }
  for (int32_t p = 0; p < m; ++p)
    for (int c = 0; c < 3; ++c) nx->cen[3 * p + c] /= cnt[p];
  free(cnt);
}

/* P block of node i of lv (already coarsened into nx): rows (dp, y) of the
 * node, columns (t, w) of the parent: dp = t + w x (x_i - c), y = S w */
static void amg_prolong_blocks(amg_level *lv, const amg_level *nx, const double *quat, int fine) {
  lv->P = (double *)calloc(36 * (size_t)lv->n, sizeof(double));
  for (int32_t i = 0; i < lv->n; ++i) {
    if (!lv->active[i]) continue;
    double *P = lv->P + 36 * i;
    const double *c = nx->cen + 3 * lv->parent[i];
    double d[3] = {lv->cen[3 * i] - c[0], lv->cen[3 * i + 1] - c[1], lv->cen[3 * i + 2] - c[2]};
    double X[9];
    cross_matrix(d, X);   /* w x d = -d x w = -[d]x w */
    for (int r = 0; r < 3; ++r) {
      P[r * 6 + r] = 1.0;
      for (int k = 0; k < 3; ++k) P[r * 6 + 3 + k] = -X[r * 3 + k];
    }
    double S[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (fine) {   /* y = 1/2 R(q)^T w: dq = G_l(q)^T y = q (y, 0) equals 1/2 (w, 0) q */
      double R[9];
      rotmat(quat + 4 * i, R);
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) S[r * 3 + k] = 0.5 * R[k * 3 + r];
    }
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) P[(3 + r) * 6 + 3 + k] = S[r * 3 + k];
  }
}

/* C += P_a^T B P_b for 6x6 blocks */
static void ptbp_add(const double *Pa, const double *Bm, const double *Pb, double *C, int ldc) {
  double T[36], U[36];
  mm(6, 6, 6, Bm, Pb, T);
  mtm(6, 6, 6, Pa, T, U);
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) C[r * ldc + c] += U[r * 6 + c];
}

static void amg_diag_inverse(amg_level *lv, const double *hdiag) {
  lv->Dinv = (double *)malloc(36 * sizeof(double) * lv->n);
  int32_t N = 6 * lv->n;
  for (int32_t i = 0; i < lv->n; ++i) {
    double B[36];
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 6; ++c) B[r * 6 + c] = hdiag ? hdiag[36 * i + r * 6 + c] : lv->A[(6 * i + r) * N + 6 * i + c];
    if (dense_inverse(6, B, lv->Dinv + 36 * i)) memset(lv->Dinv + 36 * i, 0, 36 * sizeof(double));
  }
}

/* y = A x on level l (level 0: diagonal and bond blocks) */
static void amg_apply_A(const orc_sys *s, const amg_level *lv, int l, const double *hdiag,
                        const double *hoff, const double *x, double *y) {
  if (l == 0) {
    for (int32_t i = 0; i < s->n; ++i) mm(6, 6, 1, hdiag + 36 * i, x + 6 * i, y + 6 * i);
    for (int64_t b = 0; b < s->nb; ++b) {
      if (!s->alive[b]) continue;
      int32_t i = s->ij[2 * b], j = s->ij[2 * b + 1];
      const double *Hb = hoff + 36 * b;
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
          y[6 * i + r] += Hb[r * 6 + c] * x[6 * j + c];
          y[6 * j + c] += Hb[r * 6 + c] * x[6 * i + r];
        }
    }
  } else {
    int32_t N = 6 * lv[l].n;
    mm(N, N, 1, lv[l].A, x, y);
  }
}

static void amg_vcycle(const orc_sys *s, const amg_level *lv, int l, int L, const double *Ainv,
                       const double *hdiag, const double *hoff, const double *b, double *x) {
  int32_t n = lv[l].n, N = 6 * n;
  if (l == L) { mm(N, N, 1, Ainv, b, x); return; }
  double *t = (double *)calloc(N, sizeof(double)), *r = (double *)calloc(N, sizeof(double));
  int32_t nc = lv[l + 1].n;
  double *bc = (double *)calloc(6 * (size_t)nc, sizeof(double)), *ec = (double *)malloc(sizeof(double) * 6 * nc);
  /* pre-smoothing from zero */
  for (int32_t i = 0; i < n; ++i) {
    mm(6, 6, 1, lv[l].Dinv + 36 * i, b + 6 * i, t + 6 * i);
    for (int k = 0; k < 6; ++k) t[6 * i + k] *= AMG_OMEGA;
  }
  /* restricted residual */
  amg_apply_A(s, lv, l, hdiag, hoff, t, r);
  for (int32_t k = 0; k < N; ++k) r[k] = b[k] - r[k];
  for (int32_t i = 0; i < n; ++i) {
    double u[6];
    mtm(6, 6, 1, lv[l].P + 36 * i, r + 6 * i, u);
    for (int k = 0; k < 6; ++k) bc[6 * lv[l].parent[i] + k] += u[k];
  }
  amg_vcycle(s, lv, l + 1, L, Ainv, hdiag, hoff, bc, ec);
  /* coarse correction */
  for (int32_t i = 0; i < n; ++i) {
    double u[6];
    mm(6, 6, 1, lv[l].P + 36 * i, ec + 6 * lv[l].parent[i], u);
    for (int k = 0; k < 6; ++k) t[6 * i + k] += u[k];
  }
  /* post-smoothing */
  amg_apply_A(s, lv, l, hdiag, hoff, t, r);
  for (int32_t i = 0; i < n; ++i) {
    double e[6], u[6];
    for (int k = 0; k < 6; ++k) e[k] = b[6 * i + k] - r[6 * i + k];
    mm(6, 6, 1, lv[l].Dinv + 36 * i, e, u);
    for (int k = 0; k < 6; ++k) x[6 * i + k] = t[6 * i + k] + AMG_OMEGA * u[k];
  }
  free(t); free(r); free(bc); free(ec);
}

int orc_amg_apply(const orc_sys *s, const double *pos, const double *quat, const double *hdiag,
                  const double *hoff, const double *b, double *x) {
  enum { MAXL = 24 };
  amg_level lv[MAXL];
  memset(lv, 0, sizeof lv);
  int32_t n = s->n;
  lv[0].n = n;
  lv[0].cell = (int64_t *)malloc(3 * sizeof(int64_t) * n);
  memcpy(lv[0].cell, s->cell, 3 * sizeof(int64_t) * n);
  lv[0].cen = (double *)malloc(3 * sizeof(double) * n);
  memcpy(lv[0].cen, pos, 3 * sizeof(double) * n);
  lv[0].active = (int32_t *)malloc(sizeof(int32_t) * n);
  for (int32_t i = 0; i < n; ++i) lv[0].active[i] = s->flags[i] == 0;
  amg_diag_inverse(&lv[0], hdiag);
  int L = 0;
  do {
    amg_level *f = &lv[L], *c = &lv[L + 1];
    f->parent = (int32_t *)malloc(sizeof(int32_t) * f->n);
    amg_coarsen(f, L == 0, c);
    amg_prolong_blocks(f, c, quat, L == 0);
    /* Galerkin product */
    int32_t Nc = 6 * c->n;
    c->A = (double *)calloc((size_t)Nc * Nc, sizeof(double));
    if (L == 0) {
      for (int32_t i = 0; i < n; ++i) {
        int32_t a = f->parent[i];
        ptbp_add(f->P + 36 * i, hdiag + 36 * i, f->P + 36 * i, c->A + (size_t)(6 * a) * Nc + 6 * a, Nc);
      }
      for (int64_t bb = 0; bb < s->nb; ++bb) {
        if (!s->alive[bb]) continue;
        int32_t i = s->ij[2 * bb], j = s->ij[2 * bb + 1], a = f->parent[i], cc = f->parent[j];
        double Ht[36];
        for (int r = 0; r < 6; ++r)
          for (int q = 0; q < 6; ++q) Ht[r * 6 + q] = hoff[36 * bb + q * 6 + r];
        ptbp_add(f->P + 36 * i, hoff + 36 * bb, f->P + 36 * j, c->A + (size_t)(6 * a) * Nc + 6 * cc, Nc);
        ptbp_add(f->P + 36 * j, Ht, f->P + 36 * i, c->A + (size_t)(6 * cc) * Nc + 6 * a, Nc);
      }
    } else {
      int32_t Nf = 6 * f->n;
      for (int32_t i = 0; i < f->n; ++i)
        for (int32_t j = 0; j < f->n; ++j) {
          double B[36];
          int nz = 0;
          for (int r = 0; r < 6; ++r)
            for (int q = 0; q < 6; ++q) {
              B[r * 6 + q] = f->A[(size_t)(6 * i + r) * Nf + 6 * j + q];
              nz |= B[r * 6 + q] != 0.0;
            }
          if (!nz) continue;
          int32_t a = f->parent[i], cc = f->parent[j];
          ptbp_add(f->P + 36 * i, B, f->P + 36 * j, c->A + (size_t)(6 * a) * Nc + 6 * cc, Nc);
        }
    }
    for (int32_t a = 0; a < c->n; ++a)
      if (!c->active[a])
        for (int r = 0; r < 6; ++r) c->A[(size_t)(6 * a + r) * Nc + 6 * a + r] = 1.0;
    amg_diag_inverse(c, NULL);
    ++L;
  } while (lv[L].n > AMG_COARSE_MAX && L < MAXL - 1);
  int32_t NL = 6 * lv[L].n;
  double *Ainv = (double *)malloc(sizeof(double) * NL * NL);
  int rc = dense_inverse(NL, lv[L].A, Ainv) ? -1 : L;
  if (rc >= 0) amg_vcycle(s, lv, 0, L, Ainv, hdiag, hoff, b, x);
  free(Ainv);
  for (int l = 0; l <= L; ++l) {
    free(lv[l].A); free(lv[l].Dinv); free(lv[l].P); free(lv[l].parent); free(lv[l].cen);
    free(lv[l].active); free(lv[l].cell);
  }
  return rc;
}

void orc_default_options(orc_options *o) {
  o->tol_abs = 0.0;
  o->tol_rel = 1e-12;
  o->cg_rtol = 1e-12;
  o->armijo_c = 1e-4;
  o->max_newton = 200;
  o->max_cg = 0; /* 0: 20 * 6n */
  o->max_ls = 30;
  o->break_bonds = 1;
  o->first_order = 0;
  o->midpoint = 0;
  o->cg_forcing = 0;
}

int orc_step(orc_sys *s, double dt, const orc_options *o, orc_stats *st) {
  if (!s || !(dt > 0.0)) { set_err("invalid step"); return -1; }
  orc_options def;
  if (!o) { orc_default_options(&def); o = &def; }
  int32_t n = s->n;
  size_t N6 = 6 * (size_t)n;
  double *ph = (double *)malloc(sizeof(double) * 3 * n), *qh = (double *)malloc(sizeof(double) * 4 * n);
  double *x_p = (double *)malloc(sizeof(double) * 3 * n), *x_q = (double *)malloc(sizeof(double) * 4 * n);
  double *t_p = (double *)malloc(sizeof(double) * 3 * n), *t_q = (double *)malloc(sizeof(double) * 4 * n);
  double *z = (double *)malloc(sizeof(double) * N6), *rhs = (double *)malloc(sizeof(double) * N6);
  double *y = (double *)malloc(sizeof(double) * N6);
  double *hdiag = (double *)malloc(sizeof(double) * 36 * n);
  double *hoff = (double *)malloc(sizeof(double) * 36 * (s->nb > 0 ? s->nb : 1));
  double *dq = (double *)malloc(sizeof(double) * 4 * n);
  orc_stats S = {0};
  int status = 0;
  /* initial guess x0 = x_n + v_n dt, quaternion normalised */
  orc_predict(s, dt, ph, qh);
  memcpy(x_p, ph, sizeof(double) * 3 * n);
  for (int32_t i = 0; i < n; ++i) {
    double nq = sqrt(dot4(qh + 4 * i, qh + 4 * i));
    for (int r = 0; r < 4; ++r) x_q[4 * i + r] = qh[4 * i + r] / nq;
  }
  /* element-repulsion candidates of this step, at the predicted positions */
  orc_contact_candidates(s, ph);
  /* inertia target: x_hat, or z_hat of the midpoint form (Section 3.1) */
  if (o->midpoint) orc_midpoint_target(s, dt, ph, qh);
  const objective ob = {o->midpoint != 0, ph, qh};
  /* an initial guess outside the domain of the potential (an alive bond with
   * q_j = -q_i at the point V is evaluated, where the shear midpoint does not
   * exist) is replaced by the state x_n for the free particles */
  {
    int outside = 0;
    for (int64_t b = 0; b < s->nb && !outside; ++b) {
      if (!s->alive[b]) continue;
      int32_t i = s->ij[2 * b], j = s->ij[2 * b + 1];
      const double *qa = x_q + 4 * i, *qb = x_q + 4 * j;
      double w[4];
      for (int r = 0; r < 4; ++r)
        w[r] = o->midpoint ? 0.5 * (qa[r] + s->quat[4 * i + r]) + 0.5 * (qb[r] + s->quat[4 * j + r])
                           : qa[r] + qb[r];
      if (dot4(w, w) < 1e-12) outside = 1;
    }
    if (outside)
      for (int32_t i = 0; i < n; ++i)
        if (s->flags[i] == 0) {
          memcpy(x_p + 3 * i, s->pos + 3 * i, sizeof(double) * 3);
          memcpy(x_q + 4 * i, s->quat + 4 * i, sizeof(double) * 4);
        }
  }
  int max_cg = o->max_cg > 0 ? o->max_cg : (int)(20 * N6);
  double phi = 0.0, z0 = -1.0, last_move = 0.0, xmax = 0.0, z_prev = 0.0;
  double alpha_prev = 0.5;   /* first-order: the first search starts at alpha = 1 */
  int unresolved = 0, stall = 0;
  for (int k = 0;; ++k) {
    if (o->first_order)
      objective_grad_hess(s, dt, &ob, x_p, x_q, 1, &phi, z, NULL, NULL);
    else
      objective_grad_hess(s, dt, &ob, x_p, x_q, 1, &phi, z, hdiag, hoff);
    double zn = sqrt(vdot(z, z, N6));
    if (k == 0) { z0 = zn; S.grad0 = zn; }
    S.grad_final = zn;
    S.phi = phi;
    double tol = o->tol_abs > o->tol_rel * z0 ? o->tol_abs : o->tol_rel * z0;
    if (zn <= tol) break;
    /* rounding floor: the last accepted step no longer moved the state */
    if (k > 0 && last_move <= 1e-14 * (1.0 + xmax)) break;
    /* rounding floor: three accepted steps in a row whose predicted decrease
     * the objective cannot resolve, without halving the gradient */
    if (k > 0) {
      stall = (unresolved && zn > 0.5 * z_prev) ? stall + 1 : 0;
      if (stall >= 3) break;
    }
    z_prev = zn;
    if (k >= o->max_newton) { status = 1; break; }
    if (o->first_order) {
      /* Algorithm 1: descend along -grad f.  In the reduced coordinates
       * (dp, y) with dq = G_l(q)^T y the rows of G_l are orthonormal, so
       * -grad f is y = -z (Section 4.1) */
      for (size_t a = 0; a < N6; ++a) y[a] = -z[a];
    } else {
      /* solve (Hess' f) dx = -grad f in the reduced tangent space */
      for (size_t a = 0; a < N6; ++a) rhs[a] = -z[a];
      double res, rt = o->cg_rtol;
      /* Section 5.3: relative tolerance min(eps, sqrt|grad f|) when asked for */
      if (o->cg_forcing && sqrt(zn) < rt) rt = sqrt(zn);
      int it = orc_pcg(s, hdiag, hoff, rhs, rt, max_cg, y, &res);
      S.cg_iters += it >= 0 ? it : -it;
    }
    double slope = vdot(z, y, N6);
    if (!(slope < 0.0)) { status = 2; break; }
    /* direction: dp = y_p, dq = G_l(q)^T y_q */
    for (int32_t i = 0; i < n; ++i) {
      double G[12];
      G_left(x_q + 4 * i, G);
      mtm(3, 4, 1, G, y + 6 * i + 3, dq + 4 * i);
    }
    /* backtracking Armijo line search along the manifold; the first-order
     * search starts at twice the last accepted step (at most 1) */
    double alpha = o->first_order ? fmin(1.0, 2.0 * alpha_prev) : 1.0;
    int accepted = 0;
    double max_move = 0.0;
    for (int ls = 0; ls <= o->max_ls; ++ls) {
      for (int32_t i = 0; i < n; ++i) {
        for (int r = 0; r < 3; ++r) t_p[3 * i + r] = x_p[3 * i + r] + alpha * y[6 * i + r];
        orc_quat_exp_step(x_q + 4 * i, dq + 4 * i, alpha, t_q + 4 * i);
      }
      double phit;
      objective_energy(s, dt, &ob, t_p, t_q, 0, &phit);
      if (phit <= phi + o->armijo_c * alpha * slope) { accepted = 1; break; }
      alpha *= 0.5;
      S.ls_backtracks++;
    }
    if (!accepted) { status = 2; break; }
    alpha_prev = alpha;
    unresolved = -alpha * slope <= 1e-15 * fabs(phi);
    xmax = 0.0;
    for (size_t a = 0; a < 3 * (size_t)n; ++a) {
      double m = fabs(t_p[a] - x_p[a]);
      if (m > max_move) max_move = m;
      if (fabs(t_p[a]) > xmax) xmax = fabs(t_p[a]);
    }
    for (size_t a = 0; a < 4 * (size_t)n; ++a) {
      double m = fabs(t_q[a] - x_q[a]);
      if (m > max_move) max_move = m;
    }
    last_move = max_move;
    memcpy(x_p, t_p, sizeof(double) * 3 * n);
    memcpy(x_q, t_q, sizeof(double) * 4 * n);
    S.newton_iters++;
  }
  if (status == 2 && S.grad_final <= 1e-6 * (z0 > 0 ? z0 : 1.0)) status = 0; /* at the rounding floor */
  /* v_{n+1} = (x_{n+1} - x_n) / dt ; friction hook: off */
  for (int32_t i = 0; i < n; ++i) {
    for (int r = 0; r < 3; ++r) {
      s->vel[3 * i + r] = (x_p[3 * i + r] - s->pos[3 * i + r]) / dt;
      s->pos[3 * i + r] = x_p[3 * i + r];
    }
    for (int r = 0; r < 4; ++r) {
      s->qvel[4 * i + r] = (x_q[4 * i + r] - s->quat[4 * i + r]) / dt;
      s->quat[4 * i + r] = x_q[4 * i + r];
    }
  }
  /* friction: explicit velocity change (Section 5.4, Algorithm 3) */
  if (s->mu_s > 0.0 || s->mu_r > 0.0) orc_friction(s, dt);
  /* update bond state with x_{n+1} */
  if (o->break_bonds) orc_break_bonds(s, &S.bonds_broken);
  S.status = status;
  if (st) *st = S;
  free(ph); free(qh); free(x_p); free(x_q); free(t_p); free(t_q); free(z); free(rhs); free(y);
  free(hdiag); free(hoff); free(dq);
  return status;
}
