// Particle-parallel kernels of one implicit step (Algorithm 3):
//   prediction and initial guess, per-particle terms of the incremental
//   potential (inertia with the constant extended mass matrix M_s of
//   Section 3.1, gravity, ground repulsion of Section 5.4), fixed-order
//   assembly of the bond halves into the diagonal block and the reduced
//   gradient, the block-Jacobi inverse, the exp-map retraction of Section 4.1
//   with the trial energy, and the velocity update.
// One thread per particle, TILE particles per workgroup, one scene per tile.
#include "bdem_particle.hpp"

namespace bdem {

// initial guess x0 = x_n + v_n dt, q normalised; kinematic particles move
// with their own velocity, fixed particles stay (their q is held).
__global__ __launch_bounds__(TILE) void k_predict(DevPtrs d, int write_iterate) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const uint8_t f = d.flags[r];
  if (f == 255) return;
  const double dt = d.ctl[d.psid[r]].dt;
  const double4 p = d.pn[r], q = d.qn[r], v = d.vn[r], w = d.wn[r];
  double4 ph = p, qh = q;
  if (f != 1) { ph.x += dt * v.x; ph.y += dt * v.y; ph.z += dt * v.z; }
  if (f == 0) { qh.x += dt * w.x; qh.y += dt * w.y; qh.z += dt * w.z; qh.w += dt * w.w; }
  d.ph[r] = ph;
  d.qh[r] = qh;
  if (!write_iterate) return;
  d.px[r] = ph;
  const double inv = 1.0 / sqrt(qh.x * qh.x + qh.y * qh.y + qh.z * qh.z + qh.w * qh.w);
  d.qx[r] = (f == 0) ? make_double4(qh.x * inv, qh.y * inv, qh.z * inv, qh.w * inv) : q;
}

// Initial guess outside the potential's domain (an alive bond with
// q_j = -q_i at the prediction): the free particles of that scene start the
// Newton iteration from x_n instead; kinematic and fixed particles keep
// their prescribed positions.
__global__ __launch_bounds__(TILE) void k_restart_from_state(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  if (d.ctl[d.psid[blockIdx.x * TILE]].ndegen == 0) return;   // uniform over the tile
  if (d.flags[r] != 0) return;
  d.px[r] = d.pn[r];
  d.qx[r] = d.qn[r];
}

__global__ __launch_bounds__(TILE) void k_copy_state(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  d.px[r] = d.pn[r];
  d.qx[r] = d.qn[r];
}

template <typename T, bool HESS>
__global__ __launch_bounds__(TILE) void k_particle_eval(DevPtrs d, Params P, int potential_only) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const int scene = d.psid[blockIdx.x * TILE];
  const SceneCtl &ctl = d.ctl[scene];
  if (!ctl.newton_active) return;
  const uint8_t f = d.flags[r];
  KSum e = {0.0, 0.0}, g2 = {0.0, 0.0};
  double z[6] = {0, 0, 0, 0, 0, 0};
  double D[21];
#pragma unroll
  for (int k = 0; k < 21; ++k) D[k] = 0.0;
  if (f != 255) {
    const int beg = d.row_ptr[r], end = d.row_ptr[r + 1];
    const T *hh = reinterpret_cast<const T *>(d.hhalf);
    for (int k = beg; k < end; ++k) {
      const double *gh = d.ghalf + (size_t)k * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) z[c] += gh[c];
      if (HESS) {
#pragma unroll
        for (int c = 0; c < 21; ++c) D[c] += double(hh[(size_t)k * 21 + c]);
      }
    }
  }
  particle_row_finish<T, HESS>(d, P, ctl, r, f, potential_only, z, D, e, g2);
  const KSum te = block_ksum(e);
  const KSum tg = block_ksum(g2);
  if (threadIdx.x == 0) {
    d.part_b[blockIdx.x] = make_double2(te.s, te.c);
    d.part_c[blockIdx.x] = make_double2(tg.s, tg.c);
  }
}

// z_hat = x_hat - 1/2 M_s^{-1} dt^2 grad V((x_{n-1} + x_n)/2) of the variational
// midpoint form (Section 3.1), written over the prediction (ph, qh) of the
// free particles: the bond gradients that k_bond_force left in the row's
// slots are summed in slot order, then gravity and ground at the previous
// midpoint are added.  Fixed and kinematic particles keep x_hat.
__global__ __launch_bounds__(TILE) void k_midpoint_target(DevPtrs d, Params P) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const SceneCtl &ctl = d.ctl[d.psid[blockIdx.x * TILE]];
  if (!ctl.newton_active) return;
  if (d.flags[r] != 0) return;
  const double *fh = reinterpret_cast<const double *>(d.hoff);
  double g[7] = {0, 0, 0, 0, 0, 0, 0};
  const int beg = d.row_ptr[r], end = d.row_ptr[r + 1];
  for (int k = beg; k < end; ++k) {
#pragma unroll
    for (int c = 0; c < 7; ++c) g[c] += fh[(size_t)k * 8 + c];
  }
  const double4 pc = d.pconst[r], pn = d.pn[r], ph = d.ph[r], qh = d.qh[r];
  const double m = pc.x, c = pc.y, rad = pc.z;
  g[0] -= m * P.gx; g[1] -= m * P.gy; g[2] -= m * P.gz;
  if (ctl.kc != 0.0) {
    const double mp[3] = {0.5 * ((2.0 * pn.x - ph.x) + pn.x), 0.5 * ((2.0 * pn.y - ph.y) + pn.y),
                          0.5 * ((2.0 * pn.z - ph.z) + pn.z)};
    const double gap = P.gnx * mp[0] + P.gny * mp[1] + P.gnz * mp[2] - P.gh - rad;
    if (gap < 0.0) {
      g[0] += ctl.kc * gap * P.gnx;
      g[1] += ctl.kc * gap * P.gny;
      g[2] += ctl.kc * gap * P.gnz;
    }
  }
  const double dt2 = ctl.dt * ctl.dt, fm = 0.5 * dt2 / m, fc = 0.5 * dt2 / c;
  d.ph[r] = make_double4(ph.x - fm * g[0], ph.y - fm * g[1], ph.z - fm * g[2], ph.w);
  d.qh[r] = make_double4(qh.x - fc * g[3], qh.y - fc * g[4], qh.z - fc * g[5], qh.w - fc * g[6]);
}

// trial state of the line search: p + a dp, q (x) exp(a y) renormalised in
// FP64 (Section 4.1, manifold-update-1/2; dq = G_l(q)^T y = q (y, 0) so the
// geodesic step is a right multiplication by (sin|a y| y/|y|, cos|a y|)),
// plus the particle part of the trial energy and the step size maxima.
__global__ __launch_bounds__(TILE) void k_ls_trial(DevPtrs d, Params P) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const int scene = d.psid[blockIdx.x * TILE];
  const SceneCtl &ctl = d.ctl[scene];
  if (!ctl.ls_active) return;
  const uint8_t f = d.flags[r];
  KSum e = {0.0, 0.0};
  double mv = 0.0, xm = 0.0;
  if (f != 255) {
    const double a = ctl.alpha_ls;
    const double4 p = d.px[r], q = d.qx[r];
    const double *x = d.cx + (size_t)r * 6;
    double4 pt = p, qt = q;
    if (f == 0) {
      pt = make_double4(p.x + a * x[0], p.y + a * x[1], p.z + a * x[2], 0.0);
      const double y[3] = {a * x[3], a * x[4], a * x[5]};
      const double th = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
      double sc, cc;
      if (th < 1e-8) { sc = 1.0 - th * th / 6.0; cc = 1.0 - 0.5 * th * th; }
      else { sc = sin(th) / th; cc = cos(th); }
      const double e4[4] = {sc * y[0], sc * y[1], sc * y[2], cc};
      const double q4[4] = {q.x, q.y, q.z, q.w};
      double o[4];
      qmul(q4, e4, o);
      const double inv = 1.0 / sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2] + o[3] * o[3]);
      qt = make_double4(o[0] * inv, o[1] * inv, o[2] * inv, o[3] * inv);
    }
    d.pt[r] = pt;
    d.qt[r] = qt;
    PTerms t;
    const double4 pv = P.midpoint ? mid4(pt, d.pn[r]) : pt;
    particle_terms(P, ctl.kc, ctl.inv_dt2, d.pconst[r], pt, qt, d.ph[r], d.qh[r], pv, 1.0, 1.0, t);
    kadd(e, t.E);
    mv = fmax(fmax(fabs(pt.x - p.x), fabs(pt.y - p.y)), fabs(pt.z - p.z));
    mv = fmax(mv, fmax(fmax(fabs(qt.x - q.x), fabs(qt.y - q.y)), fmax(fabs(qt.z - q.z), fabs(qt.w - q.w))));
    xm = fmax(fmax(fabs(pt.x), fabs(pt.y)), fabs(pt.z));
  }
  const KSum te = block_ksum(e);
  mv = block_max(mv);
  xm = block_max(xm);
  if (threadIdx.x == 0) {
    d.part_b[blockIdx.x] = make_double2(te.s, te.c);
    d.part_max[2 * blockIdx.x] = mv;
    d.part_max[2 * blockIdx.x + 1] = xm;
  }
}

__global__ __launch_bounds__(TILE) void k_ls_accept(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const int scene = d.psid[blockIdx.x * TILE];
  if (!d.ctl[scene].ls_accept) return;
  d.px[r] = d.pt[r];
  d.qx[r] = d.qt[r];
}

// v_{n+1} = (x_{n+1} - x_n) / dt, then x_n <- x_{n+1} (Algorithm 3).
// Friction hook of Algorithm 3: off.
__global__ __launch_bounds__(TILE) void k_finish(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  if (d.flags[r] == 255) return;
  const double idt = 1.0 / d.ctl[d.psid[r]].dt;
  const double4 p = d.px[r], q = d.qx[r], p0 = d.pn[r], q0 = d.qn[r];
  d.vn[r] = make_double4((p.x - p0.x) * idt, (p.y - p0.y) * idt, (p.z - p0.z) * idt, 0.0);
  d.wn[r] = make_double4((q.x - q0.x) * idt, (q.y - q0.y) * idt, (q.z - q0.z) * idt,
                         (q.w - q0.w) * idt);
  d.pn[r] = p;
  d.qn[r] = q;
}

void launch_predict(const DevPtrs &d, bool write_iterate, hipStream_t s) {
  k_predict<<<d.n_pad / TILE, TILE, 0, s>>>(d, write_iterate ? 1 : 0);
}
void launch_restart_from_state(const DevPtrs &d, hipStream_t s) {
  k_restart_from_state<<<d.n_pad / TILE, TILE, 0, s>>>(d);
}

void launch_copy_state_to_iterate(const DevPtrs &d, hipStream_t s) {
  k_copy_state<<<d.n_pad / TILE, TILE, 0, s>>>(d);
}
void launch_particle_eval(const DevPtrs &d, const Params &P, bool mixed, bool hess,
                          bool potential_only, hipStream_t s) {
  const int nb = d.n_pad / TILE, po = potential_only ? 1 : 0;
  if (mixed) {
    if (hess) k_particle_eval<float, true><<<nb, TILE, 0, s>>>(d, P, po);
    else k_particle_eval<float, false><<<nb, TILE, 0, s>>>(d, P, po);
  } else {
    if (hess) k_particle_eval<double, true><<<nb, TILE, 0, s>>>(d, P, po);
    else k_particle_eval<double, false><<<nb, TILE, 0, s>>>(d, P, po);
  }
}
void launch_midpoint_target(const DevPtrs &d, const Params &P, hipStream_t s) {
  k_midpoint_target<<<d.n_pad / TILE, TILE, 0, s>>>(d, P);
}
void launch_ls_trial(const DevPtrs &d, const Params &P, hipStream_t s) {
  k_ls_trial<<<d.n_pad / TILE, TILE, 0, s>>>(d, P);
}
void launch_ls_accept(const DevPtrs &d, hipStream_t s) {
  k_ls_accept<<<d.n_pad / TILE, TILE, 0, s>>>(d);
}
void launch_finish_step(const DevPtrs &d, hipStream_t s) {
  k_finish<<<d.n_pad / TILE, TILE, 0, s>>>(d);
}

}  // namespace bdem
