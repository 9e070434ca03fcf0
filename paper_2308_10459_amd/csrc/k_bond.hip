// Bond-parallel kernels: per-bond energy / reduced Riemannian gradient /
// reduced Riemannian Hessian (Sections 3.2, 4.1, 4.2), the SPD projection of
// Section 5.2, the line-search energy pass and the fracture test of
// Section 3.3.
//
// One thread per bond.  Bonds are tiled TILE per workgroup and every tile
// belongs to a single scene.  The bond writes its off-diagonal 6x6 blocks
// into the two block-CSR slots it owns (row i and row j) and its shares of
// the two diagonal blocks and of the reduced gradient into per-slot halves,
// which the particle kernel sums in a fixed order: no atomics, bitwise
// deterministic.
//
// Reduced coordinates per bond: the energy depends on p_i, p_j only through
// u = p_j - p_i, so its 12x12 reduced Hessian equals T^T H9 T with T the
// orthonormal-row map (p_i, y_i, p_j, y_j) -> ((p_j - p_i)/sqrt2, y_i, y_j).
// The eigen-clamp of the 12x12 therefore equals T^T clamp(H9) T exactly and
// is computed on the 9x9 H9.
#include "bdem_bond.hpp"

namespace bdem {

// MID = false: V and its derivatives at the unknowns x (the implicit-Euler
// form of Section 3.1).  MID = true: the variational midpoint form, V at
// (x + x_n)/2, so the Euclidean gradient and Hessian with respect to x are
// V's at the midpoint times 1/2 and 1/4; the reduction to the tangent space
// always uses the unknowns' own quaternions.
template <typename T, bool HESS, bool MID>
__global__ __launch_bounds__(TILE) void k_bond_eval(DevPtrs d) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int b = lb * TILE + threadIdx.x;
  const int scene = d.bsid[lb * TILE];
  if (!d.ctl[scene].newton_active) return;   // uniform over the block
  const int2 ij = d.bij[b];
  const int2 sl = d.bslot[b];
  const bool real = sl.x >= 0;
  const bool alive = real && d.alive[b];
  KSum esum = {0.0, 0.0};
  if (alive) {
    const int i = ij.x, j = ij.y;
    BondGeom g;
    const double4 Qi = d.qx[i], Qj = d.qx[j];
    double4 Pi = d.px[i], Pj = d.px[j], Ei = Qi, Ej = Qj;   // evaluation point of V
    if (MID) {
      Pi = mid4(Pi, d.pn[i]); Pj = mid4(Pj, d.pn[j]);
      Ei = mid4(Qi, d.qn[i]); Ej = mid4(Qj, d.qn[j]);
    }
    bond_geometry(Pi, Ei, Pj, Ej, d.brest_a[b], d.brest_b[b], g);
    // |q_i + q_j| < 1e-6: the shear midpoint is undefined.  A non-finite state
    // is not counted here; the Newton check reports it as non-finite.
    if (dot4(g.w, g.w) < 1e-12) {
      atomicAdd(d.degenerate, 1);
      atomicAdd(&d.ctl[scene].ndegen, 1);
    }
    kadd(esum, bond_energy_of(g));
    // ---------------- reduced gradient (FP64) ----------------
    const double wg = MID ? 0.5 : 1.0;
    const double qi[4] = {Qi.x, Qi.y, Qi.z, Qi.w}, qj[4] = {Qj.x, Qj.y, Qj.z, Qj.w};
    const double ei[4] = {Ei.x, Ei.y, Ei.z, Ei.w}, ej[4] = {Ej.x, Ej.y, Ej.z, Ej.w};
    double gu[3], gw[4];
#pragma unroll
    for (int k = 0; k < 3; ++k) gu[k] = wg * (g.kn * g.e * g.n[k] - g.kts * g.F1 * g.gphi_u[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) gw[k] = -wg * g.kts * g.F1 * g.gphi_w[k];
    // bend: grad_{q_i} = G_l(q_j)^T m = q_j (m, 0); grad_{q_j} = -G_l(q_i)^T m = -q_i (m, 0)
    const double m4[4] = {wg * g.m[0], wg * g.m[1], wg * g.m[2], 0.0};
    double bqi[4], bqj[4];
    qmul(ej, m4, bqi);
    qmul(ei, m4, bqj);
    double gqi[4], gqj[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) { gqi[k] = gw[k] + bqi[k]; gqj[k] = gw[k] - bqj[k]; }
    // reduce: z_r = G_l(q) grad_q = vec(conj(q) grad_q)
    const double qic[4] = {-qi[0], -qi[1], -qi[2], qi[3]}, qjc[4] = {-qj[0], -qj[1], -qj[2], qj[3]};
    double ri[4], rj[4];
    qmul(qic, gqi, ri);
    qmul(qjc, gqj, rj);
    const double lam_i = dot4(qi, gqi), lam_j = dot4(qj, gqj);
    double *gi = d.ghalf + (size_t)sl.x * 6, *gj = d.ghalf + (size_t)sl.y * 6;
    gi[0] = -gu[0]; gi[1] = -gu[1]; gi[2] = -gu[2]; gi[3] = ri[0]; gi[4] = ri[1]; gi[5] = ri[2];
    gj[0] = gu[0];  gj[1] = gu[1];  gj[2] = gu[2];  gj[3] = rj[0]; gj[4] = rj[1]; gj[5] = rj[2];
    if (HESS) {
      // ---------------- reduced Hessian (precision T) ----------------
      const T kts = T(g.kts), F1 = T(g.F1), F2 = T(g.F2), h = T(g.h), phi = T(g.phi);
      const T il = T(1.0 / g.l);
      T n[3], dd[3], d0[3], gpu[3], gpw[4], w[4], Aw[4];
#pragma unroll
      for (int k = 0; k < 3; ++k) { n[k] = T(g.n[k]); dd[k] = T(g.d[k]); d0[k] = T(g.d0[k]); gpu[k] = T(g.gphi_u[k]); }
#pragma unroll
      for (int k = 0; k < 4; ++k) { gpw[k] = T(g.gphi_w[k]); w[k] = T(g.w[k]); Aw[k] = T(g.Aw[k]); }
      const T nd = dot3(n, dd);
      // stretch: k_n [n n^T + (1 - l0/l)(I - n n^T)]
      const T kn = T(g.kn), lat = T(1.0 - g.l0 / g.l);
      T Huu[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T nn = n[r] * n[c];
          const T hphi = -(dd[r] * n[c] + n[r] * dd[c] + nd * ((r == c ? T(1) : T(0)) - T(3) * nn)) * il * il;
          Huu[r * 3 + c] = kn * (nn + lat * ((r == c ? T(1) : T(0)) - nn)) +
                           T(2) * kts * F2 * gpu[r] * gpu[c] - kts * F1 * hphi;
        }
      // shear, mixed block: d(phi)/du dw = (P_n / l) J_d, J_d row k = 2h (A_{e_k} w - d_k w)
      const T v[3] = {w[0], w[1], w[2]}, sw = w[3];
      const T vd = dot3(v, d0);
      T vxd0[3];
      cross3(v, d0, vxd0);
      T Jd[12];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        // A_{e_k} w = (-d0_k v + d0 v_k + e_k (d0.v) + s (d0 x e_k), (v x d0)_k + d0_k s)
        T ek[3] = {T(0), T(0), T(0)};
        ek[k] = T(1);
        T d0xe[3];
        cross3(d0, ek, d0xe);
        T a4[4];
#pragma unroll
        for (int c = 0; c < 3; ++c) a4[c] = -d0[k] * v[c] + d0[c] * v[k] + ek[c] * vd + sw * d0xe[c];
        a4[3] = vxd0[k] + d0[k] * sw;
#pragma unroll
        for (int c = 0; c < 4; ++c) Jd[k * 4 + c] = T(2) * h * (a4[c] - dd[k] * w[c]);
      }
      T Huw[12];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          T pj = T(0);
#pragma unroll
          for (int k = 0; k < 3; ++k) pj += ((r == k ? T(1) : T(0)) - n[r] * n[k]) * Jd[k * 4 + c];
          Huw[r * 4 + c] = T(2) * kts * F2 * gpu[r] * gpw[c] - kts * F1 * pj * il;
        }
      // shear, w block: 2h (A_n - phi I) - 2h (w gphi^T + gphi w^T)
      T An[16];
      {
        const T nd0 = dot3(n, d0);
        T d0xn[3];
        cross3(d0, n, d0xn);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
          for (int c = 0; c < 3; ++c) An[r * 4 + c] = (r == c ? -nd0 : T(0)) + d0[r] * n[c] + n[r] * d0[c];
          An[r * 4 + 3] = d0xn[r];
          An[12 + r] = d0xn[r];
        }
        An[15] = nd0;
      }
      T Hww[16];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const T hp = T(2) * h * (An[r * 4 + c] - (r == c ? phi : T(0))) -
                       T(2) * h * (w[r] * gpw[c] + gpw[r] * w[c]);
          Hww[r * 4 + c] = T(2) * kts * F2 * gpw[r] * gpw[c] - kts * F1 * hp;
        }
      (void)Aw;
      // bend / twist 4x4 blocks: G_j^T K' G_j, G_i^T K' G_i, -G_j^T K' G_i + B(m),
      // with G_l of the quaternions V is evaluated at
      T Mii[16], Mjj[16], Mij[16];
      {
        T Bi[12], Bj[12];
        const T tei[4] = {T(ei[0]), T(ei[1]), T(ei[2]), T(ei[3])};
        const T tej[4] = {T(ej[0]), T(ej[1]), T(ej[2]), T(ej[3])};
        gleft(tei, Bi);
        gleft(tej, Bj);
        const T kb = T(g.kb), ktw = T(g.ktw);
        T KGi[12], KGj[12];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const T di = d0[0] * Bi[c] + d0[1] * Bi[4 + c] + d0[2] * Bi[8 + c];
          const T dj = d0[0] * Bj[c] + d0[1] * Bj[4 + c] + d0[2] * Bj[8 + c];
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            KGi[r * 4 + c] = kb * Bi[r * 4 + c] + (ktw - kb) * d0[r] * di;
            KGj[r * 4 + c] = kb * Bj[r * 4 + c] + (ktw - kb) * d0[r] * dj;
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            T aii = T(0), ajj = T(0), aij = T(0);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              aii += Bj[k * 4 + r] * KGj[k * 4 + c];
              ajj += Bi[k * 4 + r] * KGi[k * 4 + c];
              aij -= Bj[k * 4 + r] * KGi[k * 4 + c];
            }
            Mii[r * 4 + c] = Hww[r * 4 + c] + aii;
            Mjj[r * 4 + c] = Hww[r * 4 + c] + ajj;
            Mij[r * 4 + c] = Hww[r * 4 + c] + aij;
          }
      }
      const T m[3] = {T(g.m[0]), T(g.m[1]), T(g.m[2])};
      // B(m) = [[-m^x, m], [-m^T, 0]]  (rows q_i, columns q_j)
      Mij[0 * 4 + 1] += m[2];  Mij[0 * 4 + 2] -= m[1];
      Mij[1 * 4 + 0] -= m[2];  Mij[1 * 4 + 2] += m[0];
      Mij[2 * 4 + 0] += m[1];  Mij[2 * 4 + 1] -= m[0];
      Mij[0 * 4 + 3] += m[0];  Mij[1 * 4 + 3] += m[1];  Mij[2 * 4 + 3] += m[2];
      Mij[3 * 4 + 0] -= m[0];  Mij[3 * 4 + 1] -= m[1];  Mij[3 * 4 + 2] -= m[2];
      // reduction with G_l of the unknowns; assemble the scaled 9x9
      // (u/sqrt2, y_i, y_j), packed upper triangle
      T Gi[12], Gj[12];
      {
        const T tqi[4] = {T(qi[0]), T(qi[1]), T(qi[2]), T(qi[3])};
        const T tqj[4] = {T(qj[0]), T(qj[1]), T(qj[2]), T(qj[3])};
        gleft(tqi, Gi);
        gleft(tqj, Gj);
      }
      T Rii[9], Rjj[9], Rij[9];
      gmgt(Gi, Mii, Gi, Rii);
      gmgt(Gj, Mjj, Gj, Rjj);
      gmgt(Gi, Mij, Gj, Rij);
      const T li = T(lam_i), lj = T(lam_j);
      T Uri[9], Urj[9];   // H_uw G^T
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T ai = T(0), aj = T(0);
#pragma unroll
          for (int k = 0; k < 4; ++k) { ai += Huw[r * 4 + k] * Gi[c * 4 + k]; aj += Huw[r * 4 + k] * Gj[c * 4 + k]; }
          Uri[r * 3 + c] = ai;
          Urj[r * 3 + c] = aj;
        }
      // the Euclidean Hessian enters with weight wh (1/4 at the midpoint); the
      // lambda terms already carry the gradient's weight
      const T wh = T(MID ? 0.25 : 1.0);
      const T s2 = T(1.4142135623730950488), s2h = s2 * wh;
      T *A = reinterpret_cast<T *>(d.h9) + (size_t)b * 45;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (c >= r) {
            A[up9(r, c)] = T(2) * wh * Huu[r * 3 + c];
            A[up9(3 + r, 3 + c)] = wh * Rii[r * 3 + c] - (r == c ? li : T(0));
            A[up9(6 + r, 6 + c)] = wh * Rjj[r * 3 + c] - (r == c ? lj : T(0));
          }
          A[up9(r, 3 + c)] = s2h * Uri[r * 3 + c];
          A[up9(r, 6 + c)] = s2h * Urj[r * 3 + c];
          A[up9(3 + r, 6 + c)] = wh * Rij[r * 3 + c];
        }
    }
  } else if (real) {
    // broken bond: its slots contribute nothing
    double *gi = d.ghalf + (size_t)sl.x * 6, *gj = d.ghalf + (size_t)sl.y * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) { gi[k] = 0.0; gj[k] = 0.0; }
  }
  const KSum tot = block_ksum(esum);
  if (threadIdx.x == 0) d.part_a[lb] = make_double2(tot.s, tot.c);
}

// Eigen-clamp of the per-bond 9x9 (Section 5.2, per bond); writes the bond's
// off-diagonal block (i, j) (row j of the matrix reads it transposed) and its
// two diagonal halves.  Reads the packed 9x9 written by k_bond_eval; holds
// only the Jacobi state in registers.
template <typename T, bool PSD>
__global__ __launch_bounds__(TILE) void k_bond_project(DevPtrs d) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int b = lb * TILE + threadIdx.x;
  const int scene = d.bsid[lb * TILE];
  if (!d.ctl[scene].newton_active) return;
  const int2 sl = d.bslot[b];
  if (sl.x < 0) return;
  T *hoff = reinterpret_cast<T *>(d.hoff);
  T *hhalf = reinterpret_cast<T *>(d.hhalf);
  T *oi = hoff + (size_t)b * 36;
  T *hi = hhalf + (size_t)sl.x * 21, *hj = hhalf + (size_t)sl.y * 21;
  if (!d.alive[b]) {
#pragma unroll
    for (int k = 0; k < 36; ++k) oi[k] = T(0);
#pragma unroll
    for (int k = 0; k < 21; ++k) { hi[k] = T(0); hj[k] = T(0); }
    return;
  }
  T A[45];
  const T *src = reinterpret_cast<const T *>(d.h9) + (size_t)b * 45;
#pragma unroll
  for (int k = 0; k < 45; ++k) A[k] = src[k];
  if (PSD) psd_clamp9<T>(A);
  // unscale: P_uu = A_uu / 2, P_ur = A_ur / sqrt2, P_rr = A_rr
  const T is2 = T(0.70710678118654752440), hf = T(0.5);
  const int2 ij = d.bij[b];
  const bool couple = d.flags[ij.x] == 0 && d.flags[ij.y] == 0;
  const T cpl = couple ? T(1) : T(0);
  // block (i, j): rows (p_i, y_i), cols (p_j, y_j) = [[-P_uu, -P_u,rj], [P_ri,u, P_ri,rj]]
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T uu = -hf * A[up9(r, c)] * cpl;
      const T uj = -is2 * A[up9(r, 6 + c)] * cpl;
      const T iu = is2 * A[up9(c, 3 + r)] * cpl;
      const T ij_ = A[up9(3 + r, 6 + c)] * cpl;
      oi[r * 6 + c] = uu;
      oi[r * 6 + 3 + c] = uj;
      oi[(3 + r) * 6 + c] = iu;
      oi[(3 + r) * 6 + 3 + c] = ij_;
    }
  // diagonal halves: i: [[P_uu, -P_u,ri], [., P_ri,ri]],  j: [[P_uu, P_u,rj], [., P_rj,rj]]
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r; c < 6; ++c) {
      T vi, vj;
      if (r < 3 && c < 3) { vi = hf * A[up9(r, c)]; vj = vi; }
      else if (r < 3) { vi = -is2 * A[up9(r, c)]; vj = is2 * A[up9(r, c + 3)]; }
      else { vi = A[up9(r, c)]; vj = A[up9(r + 3, c + 3)]; }
      hi[up6(r, c)] = vi;
      hj[up6(r, c)] = vj;
    }
}

// Energy of every alive bond at the iterate (trial = false) or the line-search
// trial state (trial = true), FP64; one compensated partial per tile.  mid:
// V at the midpoint (x + x_n)/2 of that state.
__global__ __launch_bounds__(TILE) void k_bond_energy(DevPtrs d, int trial, int mid) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int b = lb * TILE + threadIdx.x;
  const int scene = d.bsid[lb * TILE];
  const SceneCtl &c = d.ctl[scene];
  if (trial ? !c.ls_active : !c.newton_active) return;
  const double4 *P = trial ? d.pt : d.px;
  const double4 *Q = trial ? d.qt : d.qx;
  KSum esum = {0.0, 0.0};
  const int2 sl = d.bslot[b];
  if (sl.x >= 0 && d.alive[b]) {
    const int2 ij = d.bij[b];
    BondGeom g;
    double4 Pi = P[ij.x], Qi = Q[ij.x], Pj = P[ij.y], Qj = Q[ij.y];
    if (mid) {
      Pi = mid4(Pi, d.pn[ij.x]); Qi = mid4(Qi, d.qn[ij.x]);
      Pj = mid4(Pj, d.pn[ij.y]); Qj = mid4(Qj, d.qn[ij.y]);
    }
    bond_geometry(Pi, Qi, Pj, Qj, d.brest_a[b], d.brest_b[b], g);
    // q_j = -q_i leaves the shear midpoint undefined: outside the potential's
    // domain, so the objective is infinite and the line search backtracks
    kadd(esum, dot4(g.w, g.w) < 1e-12 ? INFINITY : bond_energy_of(g));
  }
  // bond tiles report in part_a, particle tiles in part_b (read together by
  // the line-search decision)
  const KSum tot = block_ksum(esum);
  if (threadIdx.x == 0) d.part_a[lb] = make_double2(tot.s, tot.c);
}

// Euclidean gradient of V_b over (p_i, q_i, p_j, q_j) at the previous
// midpoint (x_{n-1} + x_n)/2, x_{n-1} = 2 x_n - x_hat, of every bond, for the
// constant term z_hat of the variational midpoint form (Section 3.1).  The
// bond writes its two 7-vectors into its slots of row i and row j (8 doubles
// per slot, in the off-diagonal block buffer, which holds at least 64 bytes
// per slot and is free until the first Hessian of the step).
__global__ __launch_bounds__(TILE) void k_bond_force(DevPtrs d) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int b = lb * TILE + threadIdx.x;
  const int scene = d.bsid[lb * TILE];
  if (!d.ctl[scene].newton_active) return;
  const int2 sl = d.bslot[b];
  if (sl.x < 0) return;
  double *fi = reinterpret_cast<double *>(d.hoff) + (size_t)sl.x * 8;
  double *fj = reinterpret_cast<double *>(d.hoff) + (size_t)sl.y * 8;
  double gi[7] = {0, 0, 0, 0, 0, 0, 0}, gj[7] = {0, 0, 0, 0, 0, 0, 0};
  if (d.alive[b]) {
    const int2 ij = d.bij[b];
    auto prev_mid = [&](int r, double4 &p, double4 &q) {
      const double4 pn = d.pn[r], qn = d.qn[r], ph = d.ph[r], qh = d.qh[r];
      // x_{n-1} = 2 x_n - x_hat
      p = make_double4(0.5 * ((2.0 * pn.x - ph.x) + pn.x), 0.5 * ((2.0 * pn.y - ph.y) + pn.y),
                       0.5 * ((2.0 * pn.z - ph.z) + pn.z), 0.0);
      q = make_double4(0.5 * ((2.0 * qn.x - qh.x) + qn.x), 0.5 * ((2.0 * qn.y - qh.y) + qn.y),
                       0.5 * ((2.0 * qn.z - qh.z) + qn.z), 0.5 * ((2.0 * qn.w - qh.w) + qn.w));
    };
    double4 Pi, Qi, Pj, Qj;
    prev_mid(ij.x, Pi, Qi);
    prev_mid(ij.y, Pj, Qj);
    BondGeom g;
    bond_geometry(Pi, Qi, Pj, Qj, d.brest_a[b], d.brest_b[b], g);
    const double ei[4] = {Qi.x, Qi.y, Qi.z, Qi.w}, ej[4] = {Qj.x, Qj.y, Qj.z, Qj.w};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double gu = g.kn * g.e * g.n[k] - g.kts * g.F1 * g.gphi_u[k];
      gi[k] = -gu;
      gj[k] = gu;
    }
    const double m4[4] = {g.m[0], g.m[1], g.m[2], 0.0};
    double bqi[4], bqj[4];
    qmul(ej, m4, bqi);
    qmul(ei, m4, bqj);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double gw = -g.kts * g.F1 * g.gphi_w[k];
      gi[3 + k] = gw + bqi[k];
      gj[3 + k] = gw - bqj[k];
    }
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) { fi[k] = gi[k]; fj[k] = gj[k]; }
}

// Section 3.3 with implicit forces, at the state x_n (after the step):
//   sigma = |F_n| / S + |M_b| r0 / I,  tau = |F_s| / S + |M_t| r0 / J,
//   |F_n| = k_n |l - l0|,  |F_s| = k_t L^2 theta / l  (|d theta / d p| = 1/l),
//   M = K t: |M_t| = GJ/l0 |d0 . t'|,  |M_b| = EI/l0 |t' - (d0 . t') d0|.
// All bonds are tested at the same state; breaks are permanent.
__global__ __launch_bounds__(TILE) void k_bond_fracture(DevPtrs d) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int b = lb * TILE + threadIdx.x;
  int broke = 0;
  const int2 sl = d.bslot[b];
  if (sl.x >= 0 && d.alive[b]) {
    const double2 st = d.bstrength[b];
    if (st.x > 0.0 || st.y > 0.0) {
      const int2 ij = d.bij[b];
      BondGeom g;
      bond_geometry(d.pn[ij.x], d.qn[ij.x], d.pn[ij.y], d.qn[ij.y], d.brest_a[b], d.brest_b[b], g);
      const double4 rc = d.brest_c[b];   // (S, r0/I, r0/J, tension_only)
      double e = g.e;
      if (rc.w != 0.0 && e < 0.0) e = 0.0;
      const double Fn = g.kn * fabs(e);
      const double theta = 2.0 * asin(fmin(1.0, 0.5 * sqrt(g.y)));
      const double Fs = g.kts * theta / g.l;
      const double td = dot3(g.tp, g.d0);
      const double b0 = g.tp[0] - td * g.d0[0], b1 = g.tp[1] - td * g.d0[1], b2 = g.tp[2] - td * g.d0[2];
      const double Mt = g.ktw * fabs(td);
      const double Mb = g.kb * sqrt(b0 * b0 + b1 * b1 + b2 * b2);
      const double sigma = Fn / rc.x + Mb * rc.y;
      const double tau = Fs / rc.x + Mt * rc.z;
      if ((st.x > 0.0 && sigma > st.x) || (st.y > 0.0 && tau > st.y)) {
        d.alive[b] = 0;
        broke = 1;
      }
    }
  }
  // deterministic per-tile count
  __shared__ int cnt[TILE / 64];
  unsigned long long bal = __ballot(broke);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int k = 0; k < TILE / 64; ++k) s += cnt[k];
    d.part_cnt[lb] = s;
  }
}

template <bool MID>
static void launch_bond_eval_t(const DevPtrs &d, bool mixed, bool hess, int nblk, hipStream_t s) {
  if (mixed) {
    if (hess) k_bond_eval<float, true, MID><<<nblk, TILE, 0, s>>>(d);
    else k_bond_eval<float, false, MID><<<nblk, TILE, 0, s>>>(d);
  } else {
    if (hess) k_bond_eval<double, true, MID><<<nblk, TILE, 0, s>>>(d);
    else k_bond_eval<double, false, MID><<<nblk, TILE, 0, s>>>(d);
  }
}

void launch_bond_eval(const DevPtrs &d, bool mixed, bool psd, bool hess, bool midpoint,
                      hipStream_t s) {
  const int nblk = d.nb_pad / TILE;
  if (nblk == 0) return;
  if (midpoint) launch_bond_eval_t<true>(d, mixed, hess, nblk, s);
  else launch_bond_eval_t<false>(d, mixed, hess, nblk, s);
  if (!hess) return;
  if (mixed) {
    if (psd) k_bond_project<float, true><<<nblk, TILE, 0, s>>>(d);
    else k_bond_project<float, false><<<nblk, TILE, 0, s>>>(d);
  } else {
    if (psd) k_bond_project<double, true><<<nblk, TILE, 0, s>>>(d);
    else k_bond_project<double, false><<<nblk, TILE, 0, s>>>(d);
  }
}

void launch_bond_energy(const DevPtrs &d, bool trial, bool midpoint, hipStream_t s) {
  const int nblk = d.nb_pad / TILE;
  if (nblk == 0) return;
  k_bond_energy<<<nblk, TILE, 0, s>>>(d, trial ? 1 : 0, midpoint ? 1 : 0);
}

void launch_bond_force(const DevPtrs &d, hipStream_t s) {
  const int nblk = d.nb_pad / TILE;
  if (nblk == 0) return;
  k_bond_force<<<nblk, TILE, 0, s>>>(d);
}

void launch_bond_fracture(const DevPtrs &d, hipStream_t s) {
  const int nblk = d.nb_pad / TILE;
  if (nblk == 0) return;
  k_bond_fracture<<<nblk, TILE, 0, s>>>(d);
}

}  // namespace bdem
