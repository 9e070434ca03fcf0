// Row-parallel evaluation of the reduced system with the Gauss-Newton form
// of the bond Hessian (one kernel per Newton iteration instead of the bond
// evaluation, the eigen-clamp and the particle assembly).
//
// Section 5.2 (and Algorithm 3) only asks that the Hessian handed to the
// linear solver be positive semi-definite: any SPD matrix keeps the Newton
// fixed point (the gradient is exact), only the path changes.  The
// Gauss-Newton form is PSD term by term without an eigen-decomposition:
//   stretch     1/2 k_n (l - l0)^2: exact Hessian over u = p_j - p_i,
//               k_n [n n^T + (1 - l0/l)(I - n n^T)], with the factor
//               (1 - l0/l) clamped at 0 (its exact per-term projection);
//   shear       1/2 k_t L^2 F(y), y = |e|^2, e = n - d:
//               k_t L^2 [2 F'' grad(phi) grad(phi)^T + F' J^T J], J = de/dx,
//               i.e. the second derivatives of e itself dropped (F', F'' > 0);
//   bend/twist  1/2 t'^T K' t':  J_t^T K' J_t with J_t = dt'/dx (the bilinear
//               cross term B(K' t') dropped);
//   Weingarten  the bond's share -lambda I_3 of the sphere's curvature term
//               (Section 4.2) kept only where it is positive: max(0, -lambda) I_3.
// Every dropped term vanishes with the strain, so at small strain the form
// equals the exact reduced Hessian.  In reduced coordinates
// (p_i, y_i, p_j, y_j), dq = G_l(q)^T y, the Jacobians of a bond are
//   de/dp_i = -Ju, de/dp_j = Ju, Ju = (I - n n^T)/l;  de/dy = -D,  D = Jd G_l(q)^T,
//   dphi/dp_i = -a, dphi/dp_j = a, a = (d - (n.d) n)/l;  dphi/dy = b = G_l(q) dphi/dw,
//   dt'/dy_i = A_i = G_l(q_j) G_l(q_i)^T,  dt'/dy_j = A_j = -G_l(q_i) G_l(q_j)^T,
// with Jd = dd/dw (w = q_i + q_j) as in the bond-parallel kernel.
//
// One workgroup owns ROWS_RT consecutive block rows of one scene.  Its
// threads walk the rows' block-CSR slots (one slot = one bond seen from one
// of its ends), ROWS_NT slots per pass: each evaluates its bond (FP64
// geometry and reduced gradient, Hessian blocks in T) and stages its row's
// diagonal half and gradient half in LDS; the bond's first end also writes
// the bond's off-diagonal block.  The halves are summed per row in slot
// order (deterministic, no atomics), then one thread per row adds the
// particle's own terms and forms the diagonal block's inverse.  Nothing per
// slot goes through HBM: each bond's geometry is evaluated at both ends
// instead.
#include "bdem_bond.hpp"
#include "bdem_particle.hpp"

namespace bdem {

constexpr int ROWS_NT = 256;   // threads = slots per pass

// C = Ga Gb^T (3x4 by 4x3)
template <typename T> __device__ __forceinline__ void ggt(const T *Ga, const T *Gb, T *C) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      C[r * 3 + c] = Ga[r * 4] * Gb[c * 4] + Ga[r * 4 + 1] * Gb[c * 4 + 1] + Ga[r * 4 + 2] * Gb[c * 4 + 2] +
                     Ga[r * 4 + 3] * Gb[c * 4 + 3];
}

// One slot: the bond seen from one of its rows (its first end when !tr, its
// second end when tr).  Writes that row's diagonal half (21 packed T) and
// gradient half (6 FP64) into column `col` of the LDS staging arrays sh_h /
// sh_g; the first end also writes the bond's block (rows of i, columns of
// j) into hoff.  Quantities of the row's own end carry the suffix s, those
// of the other end o.
template <typename T, bool MID>
__device__ __forceinline__ void rows_slot(const DevPtrs &d, int b, bool tr, int scene,
                                          T (*sh_h)[ROWS_NT], double (*sh_g)[ROWS_NT], int col) {
  const int2 ij = d.bij[b];
  const int i = ij.x, j = ij.y;
  const double4 Qi = d.qx[i], Qj = d.qx[j];
  double4 Pi = d.px[i], Pj = d.px[j], Ei = Qi, Ej = Qj;   // evaluation point of V
  if (MID) {
    Pi = mid4(Pi, d.pn[i]); Pj = mid4(Pj, d.pn[j]);
    Ei = mid4(Qi, d.qn[i]); Ej = mid4(Qj, d.qn[j]);
  }
  BondGeom g;
  bond_geometry(Pi, Ei, Pj, Ej, d.brest_a[b], d.brest_b[b], g);
  if (!tr && dot4(g.w, g.w) < 1e-12) {   // counted once per bond
    atomicAdd(d.degenerate, 1);
    atomicAdd(&d.ctl[scene].ndegen, 1);
  }
  const double4 Qs = tr ? Qj : Qi, Qo = tr ? Qi : Qj, Es = tr ? Ej : Ei, Eo = tr ? Ei : Ej;
  // ---------------- reduced gradient of this end (FP64) ----------------
  double lam;
  {
    const double wg = MID ? 0.5 : 1.0;
    const double sg = tr ? 1.0 : -1.0;     // dV/dp_i = -dV/du, dV/dp_j = dV/du
    // grad_{q_i} V = grad_w V + q_j (m, 0);  grad_{q_j} V = grad_w V - q_i (m, 0)
    const double eo[4] = {Eo.x, Eo.y, Eo.z, Eo.w}, qs[4] = {Qs.x, Qs.y, Qs.z, Qs.w};
    const double m4[4] = {wg * g.m[0], wg * g.m[1], wg * g.m[2], 0.0};
    double bq[4];
    qmul(eo, m4, bq);
    double gq[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) gq[k] = -wg * g.kts * g.F1 * g.gphi_w[k] - sg * bq[k];
    const double qsc[4] = {-qs[0], -qs[1], -qs[2], qs[3]};
    double rs[4];
    qmul(qsc, gq, rs);   // G_l(q) grad_q = vec(conj(q) grad_q)
    lam = dot4(qs, gq);
#pragma unroll
    for (int k = 0; k < 3; ++k) sh_g[k][col] = sg * wg * (g.kn * g.e * g.n[k] - g.kts * g.F1 * g.gphi_u[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) sh_g[3 + k][col] = rs[k];
  }
  // ---------------- Gauss-Newton Hessian blocks (precision T) ----------------
  const T wh = T(MID ? 0.25 : 1.0);
  const T il = T(1.0 / g.l), kn = T(g.kn), lat = T(fmax(0.0, 1.0 - g.l0 / g.l));
  const T al = T(2.0 * g.kts * g.F2), be = T(g.kts * g.F1);
  const T kb = T(g.kb), ktb = T(g.ktw - g.kb);
  T n[3], a[3], d0[3], gpw[4];
#pragma unroll
  for (int k = 0; k < 3; ++k) { n[k] = T(g.n[k]); a[k] = T(g.gphi_u[k]); d0[k] = T(g.d0[k]); }
#pragma unroll
  for (int k = 0; k < 4; ++k) gpw[k] = T(g.gphi_w[k]);
  // Jd = dd/dw (3x4): row k = 2h (A_{e_k} w - d_k w)
  T Jd[12];
  {
    const T hh = T(g.h);
    const T w[4] = {T(g.w[0]), T(g.w[1]), T(g.w[2]), T(g.w[3])};
    const T dd[3] = {T(g.d[0]), T(g.d[1]), T(g.d[2])};
    const T v[3] = {w[0], w[1], w[2]}, sw = w[3];
    const T vd = dot3(v, d0);
    T vxd0[3];
    cross3(v, d0, vxd0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T ek[3] = {T(0), T(0), T(0)};
      ek[k] = T(1);
      T d0xe[3];
      cross3(d0, ek, d0xe);
      T a4[4];
#pragma unroll
      for (int c = 0; c < 3; ++c) a4[c] = -d0[k] * v[c] + d0[c] * v[k] + ek[c] * vd + sw * d0xe[c];
      a4[3] = vxd0[k] + d0[k] * sw;
#pragma unroll
      for (int c = 0; c < 4; ++c) Jd[k * 4 + c] = T(2) * hh * (a4[c] - dd[k] * w[c]);
    }
  }
  // Ju = (I - n n^T)/l;  P0 = k_n [n n^T + c (I - n n^T)] + al a a^T + be Ju / l
  T Ju[9], P0[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T pr = (r == c ? T(1) : T(0)) - n[r] * n[c];
      Ju[r * 3 + c] = pr * il;
      P0[r * 3 + c] = kn * (n[r] * n[c] + lat * pr) + al * a[r] * a[c] + be * pr * il * il;
    }
  // K' X = kb X + (ktw - kb) d0 (d0^T X)
  auto kmul = [&](const T *X, T *Y) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T s = d0[0] * X[c] + d0[1] * X[3 + c] + d0[2] * X[6 + c];
#pragma unroll
      for (int r = 0; r < 3; ++r) Y[r * 3 + c] = kb * X[r * 3 + c] + ktb * d0[r] * s;
    }
  };
  // this end: D_s = Jd G_l(q_s)^T, b_s = G_l(q_s) dphi/dw,
  // A_s = +-G_l(E_o) G_l(q_s)^T (+ for the first end, - for the second)
  T Ds[9], bs[3], As[9];
  {
    T Gs[12], GEo[12];
    const T tqs[4] = {T(Qs.x), T(Qs.y), T(Qs.z), T(Qs.w)};
    const T teo[4] = {T(Eo.x), T(Eo.y), T(Eo.z), T(Eo.w)};
    gleft(tqs, Gs);
    gleft(teo, GEo);
    ggt(Jd, Gs, Ds);
    ggt(GEo, Gs, As);
    const T sa = tr ? T(-1) : T(1);
#pragma unroll
    for (int k = 0; k < 9; ++k) As[k] *= sa;
#pragma unroll
    for (int r = 0; r < 3; ++r)
      bs[r] = Gs[r * 4] * gpw[0] + Gs[r * 4 + 1] * gpw[1] + Gs[r * 4 + 2] * gpw[2] + Gs[r * 4 + 3] * gpw[3];
  }
  // ---- this end's diagonal half: [[P0, sgn(be Ju D_s - al a b_s^T)],
  //      [., al b_s b_s^T + be D_s^T D_s + A_s^T K' A_s + max(0, -lambda) I]] ----
  {
    const T sgn = tr ? T(-1) : T(1);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = r; c < 3; ++c) sh_h[up6(r, c)][col] = wh * P0[r * 3 + c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T jd = Ju[r * 3] * Ds[c] + Ju[r * 3 + 1] * Ds[3 + c] + Ju[r * 3 + 2] * Ds[6 + c];
        sh_h[up6(r, 3 + c)][col] = wh * sgn * (be * jd - al * a[r] * bs[c]);
      }
    T KA[9];
    kmul(As, KA);
    const T wl = T(fmax(0.0, -lam));
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = r; c < 3; ++c) {
        const T dd = Ds[r] * Ds[c] + Ds[3 + r] * Ds[3 + c] + Ds[6 + r] * Ds[6 + c];
        const T aka = As[r] * KA[c] + As[3 + r] * KA[3 + c] + As[6 + r] * KA[6 + c];
        sh_h[up6(3 + r, 3 + c)][col] = wh * (al * bs[r] * bs[c] + be * dd + aka) + (r == c ? wl : T(0));
      }
  }
  // ---- the bond's off-diagonal block, from its first end (s = i, o = j):
  //   [[-P0, be Ju D_j - al a b_j^T], [al b_i a^T - be D_i^T Ju, al b_i b_j^T + be D_i^T D_j + A_i^T K' A_j]] ----
  if (!tr) {
    T *o = reinterpret_cast<T *>(d.hoff) + (size_t)b * 36;
    const bool couple = d.flags[i] == 0 && d.flags[j] == 0;
    const T cw = couple ? wh : T(0);
    T Do[9], bo[3], KAo[9];
    {
      T Go[12], GEs[12];
      const T tqo[4] = {T(Qo.x), T(Qo.y), T(Qo.z), T(Qo.w)};
      const T tes[4] = {T(Es.x), T(Es.y), T(Es.z), T(Es.w)};
      gleft(tqo, Go);
      gleft(tes, GEs);
      ggt(Jd, Go, Do);
      T Ao[9];
      ggt(GEs, Go, Ao);   // A_j = -G_l(E_i) G_l(q_j)^T
#pragma unroll
      for (int k = 0; k < 9; ++k) Ao[k] = -Ao[k];
      kmul(Ao, KAo);
#pragma unroll
      for (int r = 0; r < 3; ++r)
        bo[r] = Go[r * 4] * gpw[0] + Go[r * 4 + 1] * gpw[1] + Go[r * 4 + 2] * gpw[2] + Go[r * 4 + 3] * gpw[3];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c) o[r * 6 + c] = -cw * P0[r * 3 + c];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T jd = Ju[r * 3] * Do[c] + Ju[r * 3 + 1] * Do[3 + c] + Ju[r * 3 + 2] * Do[6 + c];
        o[r * 6 + 3 + c] = cw * (be * jd - al * a[r] * bo[c]);
      }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        // (D_i^T Ju)[r][c] = (Ju D_i)[c][r]
        const T dj = Ju[c * 3] * Ds[r] + Ju[c * 3 + 1] * Ds[3 + r] + Ju[c * 3 + 2] * Ds[6 + r];
        o[(3 + r) * 6 + c] = cw * (al * bs[r] * a[c] - be * dj);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T dd = Ds[r] * Do[c] + Ds[3 + r] * Do[3 + c] + Ds[6 + r] * Do[6 + c];
        const T aka = As[r] * KAo[c] + As[3 + r] * KAo[3 + c] + As[6 + r] * KAo[6 + c];
        o[(3 + r) * 6 + 3 + c] = cw * (al * bs[r] * bo[c] + be * dd + aka);
      }
    }
  }
}

template <typename T, bool MID>
__global__ __launch_bounds__(ROWS_NT) void k_rows_eval(DevPtrs d, Params P, int potential_only) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int r0 = lb * ROWS_RT;
  const int scene = d.psid[r0];
  const SceneCtl &ctl = d.ctl[scene];
  if (!ctl.newton_active) return;   // uniform over the workgroup
  __shared__ T sh_h[21][ROWS_NT];
  __shared__ double sh_g[6][ROWS_NT];
  __shared__ double sh_acc[ROWS_RT][28];
  __shared__ int sh_rp[ROWS_RT + 1];
  const int tid = threadIdx.x;
  if (tid <= ROWS_RT) sh_rp[tid] = d.row_ptr[r0 + tid];
  __syncthreads();
  const int sbeg = sh_rp[0], send = sh_rp[ROWS_RT];
  // summation role: row ar, part ap (0..2: seven packed diagonal values; 3: the gradient)
  const int ar = tid >> 2, ap = tid & 3;
  const int rb = sh_rp[ar], re = sh_rp[ar + 1];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int cb = sbeg; cb < send; cb += ROWS_NT) {
    const int s = cb + tid;
    if (s < send) {
      const int sb = d.sblk[s];
      const int b = sb >> 1;
      const bool tr = (sb & 1) != 0;
      if (d.alive[b]) {
        rows_slot<T, MID>(d, b, tr, scene, sh_h, sh_g, tid);
      } else {
#pragma unroll
        for (int k = 0; k < 21; ++k) sh_h[k][tid] = T(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) sh_g[k][tid] = 0.0;
        if (!tr) {
          T *o = reinterpret_cast<T *>(d.hoff) + (size_t)b * 36;
#pragma unroll
          for (int k = 0; k < 36; ++k) o[k] = T(0);
        }
      }
    }
    __syncthreads();
    const int lo = max(rb, cb) - cb, hi = min(re, cb + ROWS_NT) - cb;
    if (ap < 3) {
      for (int k = lo; k < hi; ++k)
#pragma unroll
        for (int c = 0; c < 7; ++c) acc[c] += double(sh_h[ap * 7 + c][k]);
    } else {
      for (int k = lo; k < hi; ++k)
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += sh_g[c][k];
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 7; ++c) sh_acc[ar][ap * 7 + c] = acc[c];
  __syncthreads();
  KSum e = {0.0, 0.0}, g2 = {0.0, 0.0};
  if (tid < ROWS_RT) {
    const int r = r0 + tid;
    double z[6], D[21];
#pragma unroll
    for (int c = 0; c < 21; ++c) D[c] = sh_acc[tid][c];
#pragma unroll
    for (int c = 0; c < 6; ++c) z[c] = sh_acc[tid][21 + c];
    particle_row_finish<T, true>(d, P, ctl, r, d.flags[r], potential_only, z, D, e, g2);
  }
  // one |z|^2 partial per workgroup (the energy comes from the energy pass)
  const KSum tg = block_ksum(g2);
  if (tid == 0) d.part_c[lb] = make_double2(tg.s, tg.c);
}

// Particle part of the objective at the Newton iterate (inertia about the
// target, gravity, ground, half of each overlapping candidate pair's
// repulsion), one compensated partial per TILE particles, in the same form as
// the line-search trial pass evaluates it; with k_bond_energy at the iterate
// it gives Phi of the first iterate of a step.
__global__ __launch_bounds__(TILE) void k_particle_energy(DevPtrs d, Params P, int potential_only) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const int scene = d.psid[blockIdx.x * TILE];
  const SceneCtl &ctl = d.ctl[scene];
  if (!ctl.newton_active) return;
  KSum e = {0.0, 0.0};
  if (d.flags[r] != 255) {
    const double4 p = d.px[r], q = d.qx[r];
    const double4 pv = P.midpoint ? mid4(p, d.pn[r]) : p;
    PTerms t;
    particle_terms(P, ctl.kc, potential_only ? 0.0 : ctl.inv_dt2, d.pconst[r], p, q, d.ph[r], d.qh[r], pv,
                   1.0, 1.0, t);
    kadd(e, t.E);
  }
  const KSum te = block_ksum(e);
  KSum ec = {0.0, 0.0};
  if (ctl.kself > 0.0) {
    const int nc = d.ncand[r];
    if (nc > 0) {
      const double4 pr = contact_point(d, d.px, r, P.midpoint);
      const double rr = d.pconst[r].z;
      for (int k = 0; k < nc; ++k) {
        const int j = d.cand[(size_t)r * CMAXC + k];
        double n[3], g;
        if (contact_overlap(pr, contact_point(d, d.px, j, P.midpoint), rr, d.pconst[j].z, n, g))
          kadd(ec, 0.25 * ctl.kself * g * g);
      }
    }
  }
  const KSum tc = block_ksum(ec);
  if (threadIdx.x == 0) {
    const KSum m = kmerge(te, tc);
    d.part_b[blockIdx.x] = make_double2(m.s, m.c);
  }
}

void launch_rows_eval(const DevPtrs &d, const Params &P, bool mixed, bool midpoint,
                      bool potential_only, hipStream_t s) {
  static_assert(TILE % ROWS_RT == 0, "row tiles nest in the scene tiles");
  static_assert(ROWS_NT == 4 * ROWS_RT, "four summation threads per row");
  const int nblk = d.n_pad / ROWS_RT, po = potential_only ? 1 : 0;
  if (nblk == 0) return;
  if (mixed) {
    if (midpoint) k_rows_eval<float, true><<<nblk, ROWS_NT, 0, s>>>(d, P, po);
    else k_rows_eval<float, false><<<nblk, ROWS_NT, 0, s>>>(d, P, po);
  } else {
    if (midpoint) k_rows_eval<double, true><<<nblk, ROWS_NT, 0, s>>>(d, P, po);
    else k_rows_eval<double, false><<<nblk, ROWS_NT, 0, s>>>(d, P, po);
  }
}

void launch_particle_energy(const DevPtrs &d, const Params &P, bool potential_only, hipStream_t s) {
  k_particle_energy<<<d.n_pad / TILE, TILE, 0, s>>>(d, P, potential_only ? 1 : 0);
}

}  // namespace bdem
