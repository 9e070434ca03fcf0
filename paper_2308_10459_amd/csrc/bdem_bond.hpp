// Per-bond geometry of the potentials of Section 3.2 in FP64, shared by the
// bond-parallel kernels and the row-parallel evaluation: stretch
// (l, l0), shear (the angle between the bond direction n and the rotated
// rest direction d = R(q_c) d0, q_c = (q_i + q_j)/|q_i + q_j|, through
// theta^2 = F(|n - d|^2)) and bend / twist (t' = vec(conj(q_j) q_i),
// m = K' t').
#pragma once
#include "bdem_internal.hpp"
#include "bdem_math.hpp"

namespace bdem {

struct BondGeom {
  // FP64 quantities shared by energy, gradient and Hessian
  double n[3], d[3], d0[3], w[4], Aw[4];
  double l, l0, e, h, phi, y, F, F1, F2;
  double gphi_u[3], gphi_w[4];
  double tp[3], m[3];   // t' = vec(conj(q_j) q_i), m = K' t'
  double kn, kts, ktw, kb;
};

__device__ __forceinline__ void bond_geometry(const double4 Pi, const double4 Qi,
                                              const double4 Pj, const double4 Qj,
                                              const double4 ra, const double4 rb, BondGeom &g) {
  g.d0[0] = ra.x; g.d0[1] = ra.y; g.d0[2] = ra.z; g.l0 = ra.w;
  g.kn = rb.x; g.kts = rb.y; g.ktw = rb.z; g.kb = rb.w;
  const double u[3] = {Pj.x - Pi.x, Pj.y - Pi.y, Pj.z - Pi.z};
  g.l = sqrt(dot3(u, u));
  const double il = 1.0 / g.l;
  g.n[0] = u[0] * il; g.n[1] = u[1] * il; g.n[2] = u[2] * il;
  g.e = g.l - g.l0;
  // shear: phi(u, w) = n . d(w), d(w) = R(w/|w|) d0, as the Rayleigh quotient
  // w^T A_n w / w^T w with A_n = [[-(n.d0) I + d0 n^T + n d0^T, d0 x n], [(d0 x n)^T, n.d0]]
  g.w[0] = Qi.x + Qj.x; g.w[1] = Qi.y + Qj.y; g.w[2] = Qi.z + Qj.z; g.w[3] = Qi.w + Qj.w;
  const double *v = g.w;
  const double sw = g.w[3];
  g.h = 1.0 / dot4(g.w, g.w);
  const double nd0 = dot3(g.n, g.d0), vn = dot3(v, g.n), vd = dot3(v, g.d0);
  double d0xn[3];
  cross3(g.d0, g.n, d0xn);
#pragma unroll
  for (int k = 0; k < 3; ++k) g.Aw[k] = -nd0 * v[k] + g.d0[k] * vn + g.n[k] * vd + sw * d0xn[k];
  g.Aw[3] = dot3(d0xn, v) + nd0 * sw;
  g.phi = g.h * dot4(g.w, g.Aw);
  double vxd0[3];
  cross3(v, g.d0, vxd0);
  const double vv = dot3(v, v);
#pragma unroll
  for (int k = 0; k < 3; ++k) g.d[k] = g.h * ((sw * sw - vv) * g.d0[k] + 2.0 * vd * v[k] + 2.0 * sw * vxd0[k]);
  const double dx = g.n[0] - g.d[0], dy = g.n[1] - g.d[1], dz = g.n[2] - g.d[2];
  g.y = dx * dx + dy * dy + dz * dz;
  theta2_fn(g.y, g.F, g.F1, g.F2);
#pragma unroll
  for (int k = 0; k < 4; ++k) g.gphi_w[k] = 2.0 * g.h * (g.Aw[k] - g.phi * g.w[k]);
  const double nd = dot3(g.n, g.d);
#pragma unroll
  for (int k = 0; k < 3; ++k) g.gphi_u[k] = (g.d[k] - nd * g.n[k]) * il;
  // bend / twist: t' = vec(conj(q_j) q_i); K' = EI/l0 I + (GJ - EI)/l0 d0 d0^T
  const double qjc[4] = {-Qj.x, -Qj.y, -Qj.z, Qj.w}, qi[4] = {Qi.x, Qi.y, Qi.z, Qi.w};
  double r[4];
  qmul(qjc, qi, r);
  g.tp[0] = r[0]; g.tp[1] = r[1]; g.tp[2] = r[2];
  const double td = dot3(g.tp, g.d0);
#pragma unroll
  for (int k = 0; k < 3; ++k) g.m[k] = g.kb * g.tp[k] + (g.ktw - g.kb) * td * g.d0[k];
}

__device__ __forceinline__ double bond_energy_of(const BondGeom &g) {
  return 0.5 * g.kn * g.e * g.e + 0.5 * g.kts * g.F + 0.5 * dot3(g.tp, g.m);
}

}  // namespace bdem
