// Block-Jacobi preconditioned CG on the reduced Hessian (Section 5.3,
// Algorithm 3) and the per-scene decision kernels of the Newton loop.
//
// Matrix: diagonal blocks (21 packed values per particle) plus off-diagonal
// 6x6 blocks in full block-CSR, precision T (float on the mixed path,
// double on the FP64 path).  Vectors and every dot product are FP64 with
// compensated (TwoSum) accumulation in a fixed order: results are bitwise
// reproducible run to run.
//
// All scalars (alpha, beta, tolerances, stop flags) live in the per-scene
// control blocks on the device, so one CG iteration is a fixed sequence of
// launches that can be replayed from a captured graph; the host only polls
// the number of scenes still iterating.
#include "bdem_internal.hpp"
#include "bdem_math.hpp"

namespace bdem {

__device__ __forceinline__ KSum range_ksum(const double2 *part, int beg, int end) {
  KSum acc = {0.0, 0.0};
  for (int k = beg + (int)threadIdx.x; k < end; k += blockDim.x) acc = kmerge(acc, KSum{part[k].x, part[k].y});
  return block_ksum(acc);
}
__device__ __forceinline__ double range_max(const double *part, int stride, int off, int beg, int end) {
  double m = 0.0;
  for (int k = beg + (int)threadIdx.x; k < end; k += blockDim.x) m = fmax(m, part[k * stride + off]);
  return block_max(m);
}

// ---------------------------------------------------------------------------
// Newton stop test (Algorithm 2 / 3: |grad f| < eps), CG tolerance
// eps_r = min(0.5, sqrt|grad f|) (Section 5.3).  One workgroup per scene.
// ---------------------------------------------------------------------------
__global__ void k_newton_check(DevPtrs d, Params P, int first) {
  const int s = blockIdx.x;
  SceneCtl &c = d.ctl[s];
  if (!c.newton_active) return;
  const int pb = d.scene_pbeg[s] / TILE, pe = d.scene_pbeg[s + 1] / TILE;
  const int bb = d.scene_bbeg[s] / TILE, be = d.scene_bbeg[s + 1] / TILE;
  const KSum eb = range_ksum(d.part_a, bb, be);
  const KSum ep = range_ksum(d.part_b, pb, pe);
  const KSum g2 = range_ksum(d.part_c, pb, pe);
  if (threadIdx.x != 0) return;
  const KSum et = kmerge(eb, ep);
  const double phi = et.s + et.c;
  const double gn = sqrt(g2.s + g2.c);
  c.phi = phi;
  c.gnorm = gn;
  c.ls_accept = 0;
  if (first) { c.gnorm0 = gn; c.newton_it = 0; c.cg_total = 0; c.ls_total = 0; c.status = ST_OK; }
  if (!isfinite(phi) || !isfinite(gn)) {
    c.status = ST_NONFINITE; c.nonfinite = 1; c.newton_active = 0; c.cg_active = 0;
    return;
  }
  const double tol = fmax(P.newton_tol, P.newton_rtol * c.gnorm0);
  bool stop = gn <= tol;
  // rounding floor: the last accepted step no longer moved the state
  if (!first && c.last_move <= 1e-14 * (1.0 + c.xmax)) stop = true;
  if (!stop && c.newton_it >= P.max_newton) { stop = true; c.status = ST_NOT_CONVERGED; }
  if (stop) { c.newton_active = 0; c.cg_active = 0; return; }
  c.cg_tol = fmin(P.cg_rtol_max, sqrt(gn)) * gn;
  c.cg_active = 1;
  c.cg_it = 0;
}

__global__ void k_count_active(DevPtrs d, int n_scenes) {
  __shared__ int a[3];
  if (threadIdx.x < 3) a[threadIdx.x] = 0;
  __syncthreads();
  int na = 0, nc = 0, nl = 0;
  for (int s = threadIdx.x; s < n_scenes; s += blockDim.x) {
    na += d.ctl[s].newton_active;
    nc += d.ctl[s].cg_active;
    nl += d.ctl[s].ls_active;
  }
  atomicAdd(&a[0], na);
  atomicAdd(&a[1], nc);
  atomicAdd(&a[2], nl);
  __syncthreads();
  if (threadIdx.x == 0) {
    d.counters[0] = a[0]; d.counters[1] = a[1]; d.counters[2] = a[2];
    d.counters[3] = *d.degenerate;
  }
}

// ---------------------------------------------------------------------------
// PCG vectors: one thread per particle (6 FP64 components)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void sym6_apply(const T *A, const double (&x)[6], double (&y)[6]) {
  double a[21];
#pragma unroll
  for (int k = 0; k < 21; ++k) a[k] = double(A[k]);
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) acc += a[up6(r, c)] * x[c];
    y[r] = acc;
  }
}

__device__ __forceinline__ void load6(const double *p, double (&v)[6]) {
  const double2 *q = reinterpret_cast<const double2 *>(p);
  const double2 a = q[0], b = q[1], c = q[2];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y; v[4] = c.x; v[5] = c.y;
}
__device__ __forceinline__ void store6(double *p, const double (&v)[6]) {
  double2 *q = reinterpret_cast<double2 *>(p);
  q[0] = make_double2(v[0], v[1]);
  q[1] = make_double2(v[2], v[3]);
  q[2] = make_double2(v[4], v[5]);
}

// r = -z, x = 0, s = M^-1 r, p = s ; partials r.s, r.r
template <typename T> __global__ __launch_bounds__(TILE) void k_cg_init(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const int scene = d.psid[blockIdx.x * TILE];
  if (!d.ctl[scene].cg_active) return;
  double z[6], rv[6], sv[6];
  load6(d.z + (size_t)r * 6, z);
#pragma unroll
  for (int k = 0; k < 6; ++k) rv[k] = -z[k];
  sym6_apply(reinterpret_cast<const T *>(d.dinv) + (size_t)r * 21, rv, sv);
  const double zero[6] = {0, 0, 0, 0, 0, 0};
  store6(d.cx + (size_t)r * 6, zero);
  store6(d.cr + (size_t)r * 6, rv);
  store6(d.cs + (size_t)r * 6, sv);
  store6(d.cp + (size_t)r * 6, sv);
  KSum rs = {0.0, 0.0}, rr = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 6; ++k) { kadd(rs, rv[k] * sv[k]); kadd(rr, rv[k] * rv[k]); }
  const KSum a = block_ksum(rs), b = block_ksum(rr);
  if (threadIdx.x == 0) {
    d.part_a[blockIdx.x] = make_double2(a.s, a.c);
    d.part_b[blockIdx.x] = make_double2(b.s, b.c);
  }
}

__global__ void k_cg_start(DevPtrs d) {
  const int s = blockIdx.x;
  SceneCtl &c = d.ctl[s];
  if (!c.cg_active) return;
  const int pb = d.scene_pbeg[s] / TILE, pe = d.scene_pbeg[s + 1] / TILE;
  const KSum rs = range_ksum(d.part_a, pb, pe);
  const KSum rr = range_ksum(d.part_b, pb, pe);
  if (threadIdx.x != 0) return;
  c.rz = rs.s + rs.c;
  c.rr = rr.s + rr.c;
  if (!(sqrt(c.rr) > c.cg_tol) || !(c.rz > 0.0)) c.cg_active = 0;
}

// Ap = H p: lane (row, component); 64 block rows per workgroup; partial p.Ap
template <typename T> __global__ __launch_bounds__(6 * SPMV_ROWS) void k_spmv(DevPtrs d) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int row0 = lb * SPMV_ROWS;
  const int scene = d.psid[row0];
  if (!d.ctl[scene].cg_active) return;
  const int t = threadIdx.x;
  const int row = row0 + t / 6, c = t - (t / 6) * 6;
  const T *D = reinterpret_cast<const T *>(d.hdiag) + (size_t)row * 21;
  const double *p = d.cp;
  double pr[6];
  load6(p + (size_t)row * 6, pr);
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) acc += double(D[up6(c, k)]) * pr[k];
  const int beg = d.row_ptr[row], end = d.row_ptr[row + 1];
  const T *H = reinterpret_cast<const T *>(d.hoff);
  for (int k = beg; k < end; ++k) {
    const int j = d.col[k];
    double pj[6];
    load6(p + (size_t)j * 6, pj);
    const T *h = H + (size_t)k * 36 + c * 6;
#pragma unroll
    for (int e = 0; e < 6; ++e) acc += double(h[e]) * pj[e];
  }
  d.cAp[(size_t)row * 6 + c] = acc;
  KSum pap = {0.0, 0.0};
  kadd(pap, p[(size_t)row * 6 + c] * acc);
  const KSum tot = block_ksum(pap);
  if (t == 0) d.part_c[lb] = make_double2(tot.s, tot.c);
}

__global__ void k_cg_alpha(DevPtrs d) {
  const int s = blockIdx.x;
  SceneCtl &c = d.ctl[s];
  if (!c.cg_active) return;
  const int b0 = d.scene_pbeg[s] / SPMV_ROWS, b1 = d.scene_pbeg[s + 1] / SPMV_ROWS;
  const KSum pap = range_ksum(d.part_c, b0, b1);
  if (threadIdx.x != 0) return;
  c.pAp = pap.s + pap.c;
  if (!(c.pAp > 0.0) || !isfinite(c.pAp)) {   // breakdown: keep the current x
    c.cg_active = 0;
    c.alpha = 0.0;
    return;
  }
  c.alpha = c.rz / c.pAp;
}

// x += alpha p ; r -= alpha Ap ; s = M^-1 r ; partials r.s, r.r
template <typename T> __global__ __launch_bounds__(TILE) void k_cg_update(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const int scene = d.psid[blockIdx.x * TILE];
  const SceneCtl &c = d.ctl[scene];
  if (!c.cg_active) return;
  const double a = c.alpha;
  double x[6], rv[6], p[6], ap[6], sv[6];
  load6(d.cx + (size_t)r * 6, x);
  load6(d.cr + (size_t)r * 6, rv);
  load6(d.cp + (size_t)r * 6, p);
  load6(d.cAp + (size_t)r * 6, ap);
#pragma unroll
  for (int k = 0; k < 6; ++k) { x[k] += a * p[k]; rv[k] -= a * ap[k]; }
  sym6_apply(reinterpret_cast<const T *>(d.dinv) + (size_t)r * 21, rv, sv);
  store6(d.cx + (size_t)r * 6, x);
  store6(d.cr + (size_t)r * 6, rv);
  store6(d.cs + (size_t)r * 6, sv);
  KSum rs = {0.0, 0.0}, rr = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 6; ++k) { kadd(rs, rv[k] * sv[k]); kadd(rr, rv[k] * rv[k]); }
  const KSum ta = block_ksum(rs), tb = block_ksum(rr);
  if (threadIdx.x == 0) {
    d.part_a[blockIdx.x] = make_double2(ta.s, ta.c);
    d.part_b[blockIdx.x] = make_double2(tb.s, tb.c);
  }
}

// beta = r.s_new / r.s ; stop at |r| <= eps_r |z| or max_cg
__global__ void k_cg_beta(DevPtrs d, Params P) {
  const int s = blockIdx.x;
  SceneCtl &c = d.ctl[s];
  if (!c.cg_active) return;
  const int pb = d.scene_pbeg[s] / TILE, pe = d.scene_pbeg[s + 1] / TILE;
  const KSum rs = range_ksum(d.part_a, pb, pe);
  const KSum rr = range_ksum(d.part_b, pb, pe);
  if (threadIdx.x != 0) return;
  const double rz_new = rs.s + rs.c;
  c.rr = rr.s + rr.c;
  c.beta = rz_new / c.rz;
  c.rz = rz_new;
  c.cg_it += 1;
  c.cg_total += 1;
  if (!(sqrt(c.rr) > c.cg_tol) || c.cg_it >= P.max_cg || !(rz_new > 0.0)) c.cg_active = 0;
}

// p = s + beta p
__global__ __launch_bounds__(TILE) void k_cg_pupdate(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const int scene = d.psid[blockIdx.x * TILE];
  const SceneCtl &c = d.ctl[scene];
  if (!c.cg_active) return;
  const double b = c.beta;
  double p[6], sv[6];
  load6(d.cp + (size_t)r * 6, p);
  load6(d.cs + (size_t)r * 6, sv);
#pragma unroll
  for (int k = 0; k < 6; ++k) p[k] = sv[k] + b * p[k];
  store6(d.cp + (size_t)r * 6, p);
}

// ---------------------------------------------------------------------------
// line search (Armijo, backtracking by halves)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_slope_part(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const int scene = d.psid[blockIdx.x * TILE];
  if (!d.ctl[scene].newton_active) return;
  double z[6], x[6];
  load6(d.z + (size_t)r * 6, z);
  load6(d.cx + (size_t)r * 6, x);
  KSum a = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 6; ++k) kadd(a, z[k] * x[k]);
  const KSum t = block_ksum(a);
  if (threadIdx.x == 0) d.part_a[blockIdx.x] = make_double2(t.s, t.c);
}

__global__ void k_slope(DevPtrs d) {
  const int s = blockIdx.x;
  SceneCtl &c = d.ctl[s];
  if (!c.newton_active) return;
  const int pb = d.scene_pbeg[s] / TILE, pe = d.scene_pbeg[s + 1] / TILE;
  const KSum a = range_ksum(d.part_a, pb, pe);
  if (threadIdx.x != 0) return;
  c.slope = a.s + a.c;
  c.alpha_ls = 1.0;
  c.ls_it = 0;
  c.ls_accept = 0;
  if (!(c.slope < 0.0)) {   // not a descent direction: nothing more to gain
    c.newton_active = 0;
    c.ls_active = 0;
    if (c.gnorm > 1e-6 * c.gnorm0) c.status = ST_LS_FAILED;
    return;
  }
  c.ls_active = 1;
}

__global__ void k_ls_decide(DevPtrs d, Params P) {
  const int s = blockIdx.x;
  SceneCtl &c = d.ctl[s];
  if (!c.ls_active) return;
  const int pb = d.scene_pbeg[s] / TILE, pe = d.scene_pbeg[s + 1] / TILE;
  const int bb = d.scene_bbeg[s] / TILE, be = d.scene_bbeg[s + 1] / TILE;
  const KSum eb = range_ksum(d.part_a, bb, be);
  const KSum ep = range_ksum(d.part_b, pb, pe);
  const double mv = range_max(d.part_max, 2, 0, pb, pe);
  const double xm = range_max(d.part_max, 2, 1, pb, pe);
  if (threadIdx.x != 0) return;
  const KSum et = kmerge(eb, ep);
  const double phit = et.s + et.c;
  c.phi_trial = phit;
  if (isfinite(phit) && phit <= c.phi + P.armijo_c * c.alpha_ls * c.slope) {
    c.ls_accept = 1;
    c.ls_active = 0;
    c.newton_it += 1;
    c.last_move = mv;
    c.xmax = xm;
    return;
  }
  c.ls_it += 1;
  c.ls_total += 1;
  if (c.ls_it > P.max_ls) {
    c.ls_active = 0;
    c.newton_active = 0;
    if (c.gnorm > 1e-6 * c.gnorm0) c.status = ST_LS_FAILED;   // else: at the rounding floor
    return;
  }
  c.alpha_ls *= 0.5;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_newton_check(const DevPtrs &d, const Params &P, int first, hipStream_t s) {
  k_newton_check<<<P.n_scenes, 256, 0, s>>>(d, P, first);
}
void launch_count_active(const DevPtrs &d, int n_scenes, hipStream_t s) {
  k_count_active<<<1, 256, 0, s>>>(d, n_scenes);
}
void launch_cg_init(const DevPtrs &d, bool mixed, hipStream_t s) {
  const int nb = d.n_pad / TILE;
  if (mixed) k_cg_init<float><<<nb, TILE, 0, s>>>(d);
  else k_cg_init<double><<<nb, TILE, 0, s>>>(d);
}
void launch_cg_start(const DevPtrs &d, int n_scenes, hipStream_t s) {
  k_cg_start<<<n_scenes, 256, 0, s>>>(d);
}
void launch_spmv(const DevPtrs &d, bool mixed, hipStream_t s) {
  const int nsp = d.n_pad / SPMV_ROWS;
  if (mixed) k_spmv<float><<<nsp, 6 * SPMV_ROWS, 0, s>>>(d);
  else k_spmv<double><<<nsp, 6 * SPMV_ROWS, 0, s>>>(d);
}
void launch_cg_rest(const DevPtrs &d, const Params &P, bool mixed, hipStream_t s) {
  const int nb = d.n_pad / TILE;
  k_cg_alpha<<<P.n_scenes, 256, 0, s>>>(d);
  if (mixed) k_cg_update<float><<<nb, TILE, 0, s>>>(d);
  else k_cg_update<double><<<nb, TILE, 0, s>>>(d);
  k_cg_beta<<<P.n_scenes, 256, 0, s>>>(d, P);
  k_cg_pupdate<<<nb, TILE, 0, s>>>(d);
}
void launch_cg_slope(const DevPtrs &d, int n_scenes, hipStream_t s) {
  k_slope_part<<<d.n_pad / TILE, TILE, 0, s>>>(d);
  k_slope<<<n_scenes, 256, 0, s>>>(d);
}
void launch_ls_decide(const DevPtrs &d, const Params &P, hipStream_t s) {
  k_ls_decide<<<P.n_scenes, 256, 0, s>>>(d, P);
}

}  // namespace bdem
