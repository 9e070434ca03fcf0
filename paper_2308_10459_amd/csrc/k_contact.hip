// Element repulsion and friction (Section 5.4).
//
// Candidates.  At the start of a step every particle lists the particles of
// its scene that no alive bond joins to it and whose centres at the predicted
// positions are closer than r_i + r_j + margin: at most CMAXC, sorted by
// index.  A hash grid with cells of at least 2 r_max + margin finds them in
// the 27 cells around the particle's own.  Counting and filling the grid use
// integer atomics only and every list is sorted afterwards, so candidate sets
// and all sums over them are deterministic.
//
// Objective.  Each overlapping candidate pair adds 1/2 k_ec (l - r_i - r_j)^2.
// On (p_i, p_j) its Hessian is [[H, -H], [-H, H]] with
// H = k_ec (n n^T + (1 - d/l)(I - n n^T)); while the spheres overlap the
// transverse curvature k_ec (1 - d/l) is negative, so the projected block is
// k_ec n n^T exactly.  Rows keep their own lists: each pair appears in both
// rows and each row carries half its energy.  The particle kernel adds the
// diagonal share and records the overlapping free partners; the PCG adds the
// off-diagonal couplings -k_ec n (n . u_j) to H u after the bond SpMV.
#include "bdem_contact.hpp"
#include "bdem_math.hpp"

namespace bdem {

__device__ __forceinline__ long long cell_of(double x, double h) { return (long long)floor(x / h); }

__device__ __forceinline__ int bucket_of(long long cx, long long cy, long long cz, int scene,
                                         int nbucket) {
  unsigned long long h = (unsigned long long)cx * 0x9E3779B97F4A7C15ull;
  h ^= (unsigned long long)cy * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
  h ^= (unsigned long long)cz * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
  h ^= (unsigned long long)scene * 0x27D4EB2F165667C5ull + (h << 6) + (h >> 2);
  h ^= h >> 29;
  return (int)(h & (unsigned long long)(nbucket - 1));
}

// a real particle of a scene whose repulsion is on
__device__ __forceinline__ bool in_grid(const DevPtrs &d, int r) {
  return d.flags[r] != 255 && d.ctl[d.psid[r]].kself > 0.0;
}

__device__ __forceinline__ int grid_bucket(const DevPtrs &d, int r) {
  const double h = d.ctl[d.psid[r]].ccell;
  const double4 p = d.ph[r];
  return bucket_of(cell_of(p.x, h), cell_of(p.y, h), cell_of(p.z, h), d.psid[r], d.n_bucket);
}

__global__ __launch_bounds__(TILE) void k_grid_clear(DevPtrs d) {
  const int b = blockIdx.x * TILE + threadIdx.x;
  if (b < d.n_bucket) d.gcnt[b] = 0;
  if (b == 0) *d.cand_over = 0;
}

__global__ __launch_bounds__(TILE) void k_grid_count(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  if (!in_grid(d, r)) return;
  atomicAdd(&d.gcnt[grid_bucket(d, r)], 1);
}

// exclusive scan of the bucket counts into gbeg (one workgroup of 1024
// threads, n_bucket a power of two >= 1024); the counts are reset to serve as
// fill cursors
__global__ __launch_bounds__(1024) void k_grid_scan(DevPtrs d) {
  __shared__ int part[1024];
  const int t = threadIdx.x, per = d.n_bucket / 1024, b0 = t * per;
  int sum = 0;
  for (int k = 0; k < per; ++k) sum += d.gcnt[b0 + k];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - sum;
  for (int k = 0; k < per; ++k) {
    const int c = d.gcnt[b0 + k];
    d.gbeg[b0 + k] = run;
    d.gcnt[b0 + k] = 0;
    run += c;
  }
  if (t == 1023) d.gbeg[d.n_bucket] = run;
}

__global__ __launch_bounds__(TILE) void k_grid_fill(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  if (!in_grid(d, r)) return;
  const int b = grid_bucket(d, r);
  const int pos = atomicAdd(&d.gcnt[b], 1);
  d.gitem[d.gbeg[b] + pos] = r;
}

__global__ __launch_bounds__(TILE) void k_contact_candidates(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  if (!in_grid(d, r)) {
    d.ncand[r] = 0;
    return;
  }
  const int scene = d.psid[r];
  const SceneCtl &c = d.ctl[scene];
  const double4 p = d.ph[r];
  const double ri = d.pconst[r].z;
  const long long cx = cell_of(p.x, c.ccell), cy = cell_of(p.y, c.ccell), cz = cell_of(p.z, c.ccell);
  const int rb = d.row_ptr[r], re = d.row_ptr[r + 1];
  int seen[27], nseen = 0;
  int list[CMAXC], cnt = 0;
  bool over = false;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int b = bucket_of(cx + dx, cy + dy, cz + dz, scene, d.n_bucket);
        bool dup = false;
        for (int k = 0; k < nseen; ++k) dup |= seen[k] == b;
        if (dup) continue;
        seen[nseen++] = b;
        const int kb = d.gbeg[b], ke = d.gbeg[b + 1];
        for (int k = kb; k < ke; ++k) {
          const int j = d.gitem[k];
          if (j == r || d.psid[j] != scene) continue;
          const double4 q = d.ph[j];
          const double reach = ri + d.pconst[j].z + c.cmargin;
          const double ux = q.x - p.x, uy = q.y - p.y, uz = q.z - p.z;
          if (!(ux * ux + uy * uy + uz * uz < reach * reach)) continue;
          // an alive bond joins r and j: row r's neighbour columns are sorted
          int lo = rb, hi = re - 1;
          bool bonded = false;
          while (lo <= hi) {
            const int m = (lo + hi) >> 1, cm = d.col[m];
            if (cm == j) { bonded = d.alive[d.sblk[m] >> 1] != 0; break; }
            if (cm < j) lo = m + 1; else hi = m - 1;
          }
          if (bonded) continue;
          if (cnt == CMAXC) { over = true; continue; }
          int pos = cnt++;
          while (pos > 0 && list[pos - 1] > j) { list[pos] = list[pos - 1]; --pos; }
          list[pos] = j;
        }
      }
  if (over) atomicAdd(d.cand_over, 1);
  d.ncand[r] = cnt;
  for (int k = 0; k < cnt; ++k) d.cand[(size_t)r * CMAXC + k] = list[k];
}

// PCG: w_r += sum over overlapping free partners of -k n (n . u_j) (position
// rows), and the tile's partial of (that addition) . u.  Runs after the bond
// SpMV on the same w.
__global__ __launch_bounds__(TILE) void k_contact_spmv(DevPtrs d, Params P) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const int scene = d.psid[blockIdx.x * TILE];
  const SceneCtl &c = d.ctl[scene];
  if (!c.cg_active) return;
  KSum wu = {0.0, 0.0};
  const int na = d.nact[r];
  if (na > 0) {
    const double wh = (P.midpoint ? 0.25 : 1.0) * c.kself;
    const double4 pr = contact_point(d, d.px, r, P.midpoint);
    const double rr = d.pconst[r].z;
    double w[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < na; ++k) {
      const int j = d.cact[(size_t)r * CMAXC + k];
      double n[3], e;
      if (!contact_overlap(pr, contact_point(d, d.px, j, P.midpoint), rr, d.pconst[j].z, n, e)) continue;
      const double *uj = d.cs + (size_t)j * 6;
      const double s = wh * (n[0] * uj[0] + n[1] * uj[1] + n[2] * uj[2]);
      w[0] -= s * n[0]; w[1] -= s * n[1]; w[2] -= s * n[2];
    }
    double *wr = d.cAp + (size_t)r * 6;
    const double *ur = d.cs + (size_t)r * 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      wr[k] += w[k];
      kadd(wu, w[k] * ur[k]);
    }
  }
  const KSum t = block_ksum(wu);
  if (threadIdx.x == 0) d.part_d[blockIdx.x] = make_double2(t.s, t.c);
}

// line search: half of each overlapping candidate pair's energy at the trial
// state, merged into the particle tile's trial energy
__global__ __launch_bounds__(TILE) void k_contact_trial_energy(DevPtrs d, Params P) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const int scene = d.psid[blockIdx.x * TILE];
  const SceneCtl &c = d.ctl[scene];
  if (!c.ls_active) return;
  KSum e = {0.0, 0.0};
  const int nc = d.ncand[r];
  if (nc > 0) {
    const double4 pr = contact_point(d, d.pt, r, P.midpoint);
    const double rr = d.pconst[r].z;
    for (int k = 0; k < nc; ++k) {
      const int j = d.cand[(size_t)r * CMAXC + k];
      double n[3], g;
      if (contact_overlap(pr, contact_point(d, d.pt, j, P.midpoint), rr, d.pconst[j].z, n, g))
        kadd(e, 0.25 * c.kself * g * g);
    }
  }
  const KSum t = block_ksum(e);
  if (threadIdx.x == 0) {
    const double2 pb = d.part_b[blockIdx.x];
    const KSum m = kmerge(KSum{pb.x, pb.y}, t);
    d.part_b[blockIdx.x] = make_double2(m.s, m.c);
  }
}

// ---------------------------------------------------------------------------
// friction (Section 5.4), after the velocity update and before the fracture
// test, from the contacts at x_{n+1}: the ground (F_n = k_c |gap|) and every
// overlapping candidate (F_n = k_ec |l - r_i - r_j|).  Per contact, with the
// relative velocity v_ij = v_n + v_t and relative angular velocity w_ij
// (world frame, w = 2 vec(qdot conj(q))):
//   dv_i = -min(1, mu_s F_n dt / (m_i |v_t|)) v_t,
//   dw_i = -min(1, mu_r F_n r_i dt / (I_i |w_ij|)) w_ij,  I_i = 2/5 m_i r_i^2;
// the sums are projected on the particle's own velocity (angular velocity)
// and clipped so they at most stop it.  Every particle reads the velocities
// before friction (results go to the trial buffers first).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ang_vel(double4 q, double4 qd, double (&w)[3]) {
  // 2 vec(qd conj(q))
  const double a[4] = {qd.x, qd.y, qd.z, qd.w}, b[4] = {-q.x, -q.y, -q.z, q.w};
  double t[4];
  qmul(a, b, t);
  w[0] = 2.0 * t[0]; w[1] = 2.0 * t[1]; w[2] = 2.0 * t[2];
}

__device__ __forceinline__ void friction_contact(const Params &P, double Fn, double dt, double m,
                                                 double Iw, double rad, const double (&n)[3],
                                                 const double (&vrel)[3], const double (&wrel)[3],
                                                 double (&dv)[3], double (&dw)[3]) {
  const double vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
  const double vt[3] = {vrel[0] - vn * n[0], vrel[1] - vn * n[1], vrel[2] - vn * n[2]};
  const double vtn = sqrt(vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
  if (P.mu_s > 0.0 && vtn > 0.0) {
    const double f = fmin(1.0, P.mu_s * Fn * dt / (m * vtn));
    dv[0] -= f * vt[0]; dv[1] -= f * vt[1]; dv[2] -= f * vt[2];
  }
  const double wn = sqrt(wrel[0] * wrel[0] + wrel[1] * wrel[1] + wrel[2] * wrel[2]);
  if (P.mu_r > 0.0 && wn > 0.0) {
    const double f = fmin(1.0, P.mu_r * Fn * rad * dt / (Iw * wn));
    dw[0] -= f * wrel[0]; dw[1] -= f * wrel[1]; dw[2] -= f * wrel[2];
  }
}

__device__ __forceinline__ void clip_along(const double (&v)[3], const double (&dv)[3], double (&out)[3]) {
  const double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  out[0] = out[1] = out[2] = 0.0;
  if (!(vn > 0.0)) return;
  double s = (dv[0] * v[0] + dv[1] * v[1] + dv[2] * v[2]) / vn;
  s = fmax(-vn, fmin(0.0, s));
  out[0] = s * v[0] / vn; out[1] = s * v[1] / vn; out[2] = s * v[2] / vn;
}

__global__ __launch_bounds__(TILE) void k_friction(DevPtrs d, Params P) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  if (d.flags[r] != 0) return;
  const SceneCtl &c = d.ctl[d.psid[r]];
  const double dt = c.dt;
  const double4 pr = d.pn[r], qr = d.qn[r], vr4 = d.vn[r], wr4 = d.wn[r], pc = d.pconst[r];
  const double m = pc.x, rad = pc.z, Iw = 0.4 * m * rad * rad;
  const double v[3] = {vr4.x, vr4.y, vr4.z};
  double w[3];
  ang_vel(qr, wr4, w);
  double dv[3] = {0.0, 0.0, 0.0}, dw[3] = {0.0, 0.0, 0.0};
  if (c.kc != 0.0) {
    const double gap = P.gnx * pr.x + P.gny * pr.y + P.gnz * pr.z - P.gh - rad;
    if (gap < 0.0) {
      const double n[3] = {P.gnx, P.gny, P.gnz};
      friction_contact(P, c.kc * fabs(gap), dt, m, Iw, rad, n, v, w, dv, dw);
    }
  }
  const int nc = c.kself > 0.0 ? d.ncand[r] : 0;
  for (int k = 0; k < nc; ++k) {
    const int j = d.cand[(size_t)r * CMAXC + k];
    double nrj[3], e;
    if (!contact_overlap(pr, d.pn[j], rad, d.pconst[j].z, nrj, e)) continue;
    const double n[3] = {-nrj[0], -nrj[1], -nrj[2]};   // from j to r
    const double4 vj = d.vn[j];
    double wj[3];
    ang_vel(d.qn[j], d.wn[j], wj);
    const double vrel[3] = {v[0] - vj.x, v[1] - vj.y, v[2] - vj.z};
    const double wrel[3] = {w[0] - wj[0], w[1] - wj[1], w[2] - wj[2]};
    friction_contact(P, c.kself * fabs(e), dt, m, Iw, rad, n, vrel, wrel, dv, dw);
  }
  double cv[3], cw[3];
  clip_along(v, dv, cv);
  clip_along(w, dw, cw);
  // qdot += 1/2 (dw, 0) q
  const double dq4[4] = {cw[0], cw[1], cw[2], 0.0}, q4[4] = {qr.x, qr.y, qr.z, qr.w};
  double t[4];
  qmul(dq4, q4, t);
  d.pt[r] = make_double4(v[0] + cv[0], v[1] + cv[1], v[2] + cv[2], 0.0);
  d.qt[r] = make_double4(wr4.x + 0.5 * t[0], wr4.y + 0.5 * t[1], wr4.z + 0.5 * t[2], wr4.w + 0.5 * t[3]);
}

__global__ __launch_bounds__(TILE) void k_friction_apply(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  if (d.flags[r] != 0) return;
  d.vn[r] = d.pt[r];
  d.wn[r] = d.qt[r];
}

void launch_contact_broad_phase(const DevPtrs &d, hipStream_t s) {
  const int np = d.n_pad / TILE;
  k_grid_clear<<<(d.n_bucket + TILE - 1) / TILE, TILE, 0, s>>>(d);
  k_grid_count<<<np, TILE, 0, s>>>(d);
  k_grid_scan<<<1, 1024, 0, s>>>(d);
  k_grid_fill<<<np, TILE, 0, s>>>(d);
  k_contact_candidates<<<np, TILE, 0, s>>>(d);
}
void launch_contact_spmv(const DevPtrs &d, const Params &P, hipStream_t s) {
  k_contact_spmv<<<d.n_pad / TILE, TILE, 0, s>>>(d, P);
}
void launch_contact_trial_energy(const DevPtrs &d, const Params &P, hipStream_t s) {
  k_contact_trial_energy<<<d.n_pad / TILE, TILE, 0, s>>>(d, P);
}
void launch_friction(const DevPtrs &d, const Params &P, hipStream_t s) {
  k_friction<<<d.n_pad / TILE, TILE, 0, s>>>(d, P);
  k_friction_apply<<<d.n_pad / TILE, TILE, 0, s>>>(d);
}

}  // namespace bdem
