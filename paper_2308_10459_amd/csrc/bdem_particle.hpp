// Per-particle terms of the incremental potential (Section 3.1 inertia with
// the extended mass M_s, gravity, the ground penalty and element repulsion of
// Section 5.4) and the finish of a particle row of the reduced system (its
// diagonal block, block-Jacobi inverse and gradient), shared by the
// particle-parallel and the row-parallel evaluation kernels.
#pragma once
#include "bdem_contact.hpp"
#include "bdem_math.hpp"

namespace bdem {

// energy and Euclidean derivatives of the particle's own terms
struct PTerms {
  double E;
  double gp[3], gr[3];
  double kgap;   // weight * k_c if the ground penalty is active
};

// inertia of (p, q) about the target (ph, qh), plus gravity and ground at the
// position pv where V is evaluated; their gradient and Hessian with respect
// to p enter with the weights 1, 1 (pv = p) or 1/2, 1/4 (pv = (p + p_n)/2)
__device__ __forceinline__ void particle_terms(const Params &P, double kc, double idt2, double4 pc,
                                               double4 p, double4 q, double4 ph, double4 qh,
                                               double4 pv, double wg, double wh, PTerms &t) {
  const double m = pc.x, c = pc.y, rad = pc.z;
  const double ep[3] = {p.x - ph.x, p.y - ph.y, p.z - ph.z};
  const double eq[4] = {q.x - qh.x, q.y - qh.y, q.z - qh.z, q.w - qh.w};
  t.E = 0.5 * m * idt2 * (ep[0] * ep[0] + ep[1] * ep[1] + ep[2] * ep[2]) +
        0.5 * c * idt2 * (eq[0] * eq[0] + eq[1] * eq[1] + eq[2] * eq[2] + eq[3] * eq[3]) -
        m * (P.gx * pv.x + P.gy * pv.y + P.gz * pv.z);
  t.gp[0] = m * idt2 * ep[0] - wg * m * P.gx;
  t.gp[1] = m * idt2 * ep[1] - wg * m * P.gy;
  t.gp[2] = m * idt2 * ep[2] - wg * m * P.gz;
  t.kgap = 0.0;
  if (kc != 0.0) {
    const double gap = P.gnx * pv.x + P.gny * pv.y + P.gnz * pv.z - P.gh - rad;
    if (gap < 0.0) {
      t.E += 0.5 * kc * gap * gap;
      t.gp[0] += wg * kc * gap * P.gnx;
      t.gp[1] += wg * kc * gap * P.gny;
      t.gp[2] += wg * kc * gap * P.gnz;
      t.kgap = wh * kc;
    }
  }
  // reduced rotational gradient G_l(q) c/dt^2 (q - q_hat) = vec(conj(q) (c/dt^2)(q - q_hat))
  const double qc[4] = {-q.x, -q.y, -q.z, q.w};
  const double g4[4] = {c * idt2 * eq[0], c * idt2 * eq[1], c * idt2 * eq[2], c * idt2 * eq[3]};
  double rr[4];
  qmul(qc, g4, rr);
  t.gr[0] = rr[0]; t.gr[1] = rr[1]; t.gr[2] = rr[2];
}

// symmetric 6x6 (packed upper, double) -> inverse via Cholesky; false if not PD
__device__ __forceinline__ bool spd_inverse6(const double (&A)[21], double (&Ainv)[21]) {
  double L[6][6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double dj = A[up6(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= L[j][k] * L[j][k];
    if (!(dj > 0.0)) return false;
    dj = sqrt(dj);
    L[j][j] = dj;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double v = A[up6(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / dj;
    }
  }
  // X = L^-1 (lower)
  double X[6][6];
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      if (i < c) { X[i][c] = 0.0; continue; }
      double v = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k)
        if (k >= c) v -= L[i][k] * X[k][c];
      X[i][c] = v / L[i][i];
    }
  // A^-1 = X^T X
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r; c < 6; ++c) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) v += X[k][r] * X[k][c];
      Ainv[up6(r, c)] = v;
    }
  return true;
}

// Everything a particle row adds once the bond halves of its row are summed
// into z (reduced gradient) and D (diagonal block, packed upper): the
// particle's own terms (inertia about the target, gravity, ground penalty,
// element repulsion), the PSD clamp of its own rotational block, the
// fixed / kinematic masking and the block-Jacobi inverse; writes z, the
// diagonal block and its inverse, and adds the row's energy and |z|^2 to
// e and g2.  Padding rows (flag 255) get an identity block.
template <typename T, bool HESS>
__device__ __forceinline__ void particle_row_finish(const DevPtrs &d, const Params &P,
                                                    const SceneCtl &ctl, int r, uint8_t f,
                                                    int potential_only, double (&z)[6],
                                                    double (&D)[21], KSum &e, KSum &g2) {
  if (f != 255) {
    const double idt2 = potential_only ? 0.0 : ctl.inv_dt2;
    const double4 p = d.px[r], q = d.qx[r], qh = d.qh[r];
    const double4 pv = P.midpoint ? mid4(p, d.pn[r]) : p;
    PTerms t;
    particle_terms(P, ctl.kc, idt2, d.pconst[r], p, q, d.ph[r], qh, pv, P.midpoint ? 0.5 : 1.0,
                   P.midpoint ? 0.25 : 1.0, t);
    kadd(e, t.E);
    z[0] += t.gp[0]; z[1] += t.gp[1]; z[2] += t.gp[2];
    z[3] += t.gr[0]; z[4] += t.gr[1]; z[5] += t.gr[2];
    if (ctl.kself > 0.0) {
      // element repulsion (Section 5.4): half of each overlapping candidate
      // pair's energy, this row's gradient and projected diagonal share
      // (k n n^T), and the overlapping free partners for the Hessian product
      const int nc = d.ncand[r];
      const double rr = d.pconst[r].z, kc = ctl.kself;
      const double wg = P.midpoint ? 0.5 : 1.0, wh = P.midpoint ? 0.25 : 1.0;
      int na = 0;
      for (int m = 0; m < nc; ++m) {
        const int j = d.cand[(size_t)r * CMAXC + m];
        double n[3], g;
        if (!contact_overlap(pv, contact_point(d, d.px, j, P.midpoint), rr, d.pconst[j].z, n, g)) continue;
        kadd(e, 0.25 * kc * g * g);
        z[0] -= wg * kc * g * n[0]; z[1] -= wg * kc * g * n[1]; z[2] -= wg * kc * g * n[2];
        if (HESS) {
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = a; b < 3; ++b) D[up6(a, b)] += wh * kc * n[a] * n[b];
        }
        if (f == 0 && d.flags[j] == 0) d.cact[(size_t)r * CMAXC + na++] = j;
      }
      d.nact[r] = na;
    } else if (P.contact) {
      d.nact[r] = 0;
    }
    if (HESS) {
      const double m = d.pconst[r].x, c = d.pconst[r].y;
      const double n[3] = {P.gnx, P.gny, P.gnz};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) D[up6(a, b)] += (a == b ? m * idt2 : 0.0) + t.kgap * n[a] * n[b];
      const double rot = c * idt2 * (q.x * qh.x + q.y * qh.y + q.z * qh.z + q.w * qh.w);
      const double rotc = rot > 0.0 ? rot : 0.0;   // PSD clamp of the particle's own block
      D[up6(3, 3)] += rotc; D[up6(4, 4)] += rotc; D[up6(5, 5)] += rotc;
    }
    if (f != 0) {   // fixed / kinematic: not an unknown
#pragma unroll
      for (int c = 0; c < 6; ++c) z[c] = 0.0;
#pragma unroll
      for (int k = 0; k < 21; ++k) D[k] = 0.0;
      D[up6(0, 0)] = D[up6(1, 1)] = D[up6(2, 2)] = D[up6(3, 3)] = D[up6(4, 4)] = D[up6(5, 5)] = 1.0;
    }
  } else {
    D[up6(0, 0)] = D[up6(1, 1)] = D[up6(2, 2)] = D[up6(3, 3)] = D[up6(4, 4)] = D[up6(5, 5)] = 1.0;
    if (P.contact) d.nact[r] = 0;
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    d.z[(size_t)r * 6 + c] = z[c];
    kadd(g2, z[c] * z[c]);
  }
  if (HESS) {
    T *hd = reinterpret_cast<T *>(d.hdiag) + (size_t)r * 21;
    T *di = reinterpret_cast<T *>(d.dinv) + (size_t)r * 21;
    double Di[21];
    if (!spd_inverse6(D, Di)) {
#pragma unroll
      for (int k = 0; k < 21; ++k) Di[k] = 0.0;
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        const double v = D[up6(a, a)];
        Di[up6(a, a)] = v > 0.0 ? 1.0 / v : 1.0;
      }
    }
#pragma unroll
    for (int k = 0; k < 21; ++k) { hd[k] = T(D[k]); di[k] = T(Di[k]); }
  }
}

}  // namespace bdem
