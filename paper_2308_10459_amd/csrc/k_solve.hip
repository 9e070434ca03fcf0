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
#include "bdem_amg.hpp"
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
// rows: the reduced gradient came from the row-parallel evaluation (one |z|^2
// partial per ROWS_RT rows), which forms no energy: Phi of the first iterate
// comes from the energy pass at the iterate, Phi of a later one is that of
// the line-search trial it accepted (the same kernels, the same state).
__global__ void k_newton_check(DevPtrs d, Params P, int first, int rows) {
  const int s = blockIdx.x;
  SceneCtl &c = d.ctl[s];
  if (!c.newton_active) return;
  const int pb = d.scene_pbeg[s] / TILE, pe = d.scene_pbeg[s + 1] / TILE;
  const int bb = d.scene_bbeg[s] / TILE, be = d.scene_bbeg[s + 1] / TILE;
  const int zg = rows ? ROWS_RT : TILE;
  const KSum eb = range_ksum(d.part_a, bb, be);
  const KSum ep = range_ksum(d.part_b, pb, pe);
  const KSum g2 = range_ksum(d.part_c, d.scene_pbeg[s] / zg, d.scene_pbeg[s + 1] / zg);
  if (threadIdx.x != 0) return;
  const KSum et = kmerge(eb, ep);
  const double phi = (rows && !first) ? c.phi_trial : et.s + et.c;
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
  // rounding floor: three accepted steps in a row whose predicted decrease
  // the objective cannot resolve, without halving the gradient
  if (!first) {
    c.stall = (c.unresolved && gn > 0.5 * c.gnorm_prev) ? c.stall + 1 : 0;
    if (c.stall >= 3) stop = true;
  }
  c.gnorm_prev = gn;
  if (!stop && c.newton_it >= P.max_newton) { stop = true; c.status = ST_NOT_CONVERGED; }
  if (stop) { c.newton_active = 0; c.cg_active = 0; return; }
  c.cg_tol = fmin(P.cg_rtol_max, sqrt(gn)) * gn;
  c.cg_active = 1;
  c.cg_it = 0;
}

// active-scene counts into counter slot `slot` (mapped host memory, read by
// the host after the stream or an event has passed this kernel)
__global__ void k_count_active(DevPtrs d, int n_scenes, int slot) {
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
    int *c = d.counters + 4 * slot;
    c[0] = a[0]; c[1] = a[1]; c[2] = a[2];
    c[3] = *d.degenerate;
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

// Preconditioned CG in the Chronopoulos-Gear arrangement: the same Krylov
// iterates as textbook PCG with one reduction phase per iteration.  With
// u = M^-1 r, w = H u:
//   gamma = (r, u), delta = (w, u);  beta = gamma / gamma_prev;
//   alpha = gamma / (delta - beta gamma / alpha_prev);
//   p = u + beta p;  q = w + beta q;  x += alpha p;  r -= alpha q;  u = M^-1 r.
// One iteration = k_cg_update (also the dots r.u and r.r of the u it
// writes), k_spmv (w = H u and the dot w.u, and it merges the update's dot
// partials in groups; all three dots after k_cg_init and with multigrid) and
// k_cg_scalars (per scene).  Buffers: cx = x, cr = r, cs = u, cAp = w,
// cp = p, cq = q.

// r = -z, x = 0, u = M^-1 r, p = q = 0
template <typename T> __global__ __launch_bounds__(TILE) void k_cg_init(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  const int scene = row_scene(d, blockIdx.x * TILE);
  if (!d.ctl[scene].cg_active) return;
  double z[6], rv[6], uv[6];
  load6(d.z + (size_t)r * 6, z);
#pragma unroll
  for (int k = 0; k < 6; ++k) rv[k] = -z[k];
  sym6_apply(reinterpret_cast<const T *>(d.dinv) + (size_t)r * 21, rv, uv);
  const double zero[6] = {0, 0, 0, 0, 0, 0};
  store6(d.cx + (size_t)r * 6, zero);
  store6(d.cr + (size_t)r * 6, rv);
  store6(d.cs + (size_t)r * 6, uv);
  store6(d.cp + (size_t)r * 6, zero);
  store6(d.cq + (size_t)r * 6, zero);
}

// w = H u plus the partial dots (r, u), (w, u), (r, r) of the workgroup.
// Workgroup = SPMV_ROWS consecutive block rows of one scene; their slots are
// one contiguous range of the block-CSR arrays, taken in passes of SPMV_CAP
// slots.  Each bond's block is stored once: the row of the bond's i end uses
// it as stored, the row of its j end uses the transpose.  Rows follow a
// Morton order and bonds their first row, so a block read for one row is
// usually still in cache when the other row reads it.
// Phase 1 is slot-parallel, every load of a trip issued before any use.
// FP32 blocks: one lane per slot loads the slot's whole block (nine 16-byte
// pieces) and u_j, U slots in flight, and writes the six components of
// H_slot u_j to LDS; waves take 64-slot chunks and load the next chunks'
// indices while the current blocks are in flight.  FP64 blocks (twice the
// registers per block): two adjacent lanes per slot, lane h loading rows
// 3h .. 3h + 2 as stored (nine 16-byte pieces) and u_j, U slot halves in
// flight.  For the block as stored each lane forms components 3h .. 3h + 2;
// for the transpose each forms, over its three rows, partial sums of all
// six components and takes its partner's for its own three, so that every
// component is the sum over rows 0-2 plus the sum over rows 3-5 in both
// lanes.
// Phase 2: thread (row, c) adds the diagonal block times u_row and its row's
// slot products in slot order, so the sum order is fixed and the launch
// shape (NT, U) does not change a bit: threads past 6 * SPMV_ROWS add zeros
// to the dots after the row threads' waves.  With rdots = SPMV_DOTS_WU the
// kernel leaves (r, u) and (r, r) to the kernel that produced u (the CG
// update, or the multigrid cycle's last kernel) and does not read r; their
// partials are then that kernel's, and every DOT_GROUP-th
// workgroup of a scene merges them for the scalars step: wavefront 0 takes
// the partials of its own block and the next DOT_GROUP - 1 (one butterfly
// tree per group, whatever the launch shape).  The merging workgroups are
// spread over the scene, and so over all XCDs.  SPMV_DOTS_NONE (the product
// inside the multigrid cycle) writes w and nothing else.
template <typename T, int NT, int U> __global__ __launch_bounds__(NT) void k_spmv(DevPtrs d, int rdots, int rev) {
  static_assert(NT >= 6 * SPMV_ROWS, "one thread per (row, component)");
  constexpr int NQ = 36 * (int)sizeof(T) / 16;       // 16-byte pieces per block
  __shared__ double2 prod2[SPMV_CAP * 3];
  const double *prod = reinterpret_cast<const double *>(prod2);
  const int lb = rev ? xcd_block_rev(blockIdx.x, gridDim.x) : xcd_block(blockIdx.x, gridDim.x);
  const int r0 = lb * SPMV_ROWS;
  const int scene = row_scene(d, r0);
  if (!d.ctl[scene].cg_active) return;
  const int t = threadIdx.x;
  const int s0 = d.row_ptr[r0], s1 = d.row_ptr[r0 + SPMV_ROWS];
  const int rl = t / 6, c_out = t - (t / 6) * 6;
  const bool rowthr = t < 6 * SPMV_ROWS;
  const int row = r0 + (rowthr ? rl : 0);
  const float4 *H4 = reinterpret_cast<const float4 *>(d.hoff);
  const double *u = d.cs;
  // the workgroup's diagonal blocks (SPMV_ROWS x 21 T) and its rows' u
  // (SPMV_ROWS x 6 doubles), both contiguous, staged in LDS with 16-byte
  // loads issued first and read after the first barrier (read directly,
  // each row thread would issue six scattered loads of its block)
  typedef float v4f __attribute__((ext_vector_type(4)));
  constexpr int NDG = SPMV_ROWS * 21 * (int)sizeof(T) / 16, NUR = SPMV_ROWS * 6 * 8 / 16;
  static_assert(SPMV_ROWS * 21 * sizeof(T) % 16 == 0, "16-byte pieces");
  __shared__ v4f dg4[NDG + NUR];
  {
    const v4f *sd = reinterpret_cast<const v4f *>(reinterpret_cast<const T *>(d.hdiag) + (size_t)r0 * 21);
    const v4f *su = reinterpret_cast<const v4f *>(u + (size_t)r0 * 6);
    for (int k = t; k < NDG; k += NT) dg4[k] = sd[k];
    for (int k = t; k < NUR; k += NT) dg4[NDG + k] = su[k];
  }
  double acc = 0.0, uc = 0.0, rc = 0.0;
  int rbeg = 0, rend = 0;
  if (rowthr) {
    rbeg = d.row_ptr[row];
    rend = d.row_ptr[row + 1];
    if (rdots == SPMV_DOTS_ALL) rc = d.cr[(size_t)row * 6 + c_out];
  }
  // the diagonal block times u_row, added before any slot product
  auto add_diag = [&]() {
    if (rowthr) {
      const T *D = reinterpret_cast<const T *>(dg4) + rl * 21;
      const double *ur = reinterpret_cast<const double *>(dg4 + NDG) + rl * 6;
#pragma unroll
      for (int k = 0; k < 6; ++k) acc += double(D[up6(c_out, k)]) * ur[k];
      uc = ur[c_out];
    }
  };
  if (s1 == s0) {   // no slots: uniform over the workgroup
    __syncthreads();
    add_diag();
  }
  for (int cb = s0; cb < s1; cb += SPMV_CAP) {
    const int ns = min(SPMV_CAP, s1 - cb);
    if constexpr (sizeof(T) == 4) {
      // wave w takes the pass's 64-slot chunks w, w + NW, ... (U at a time);
      // the indices of its next chunks are loaded while the current ones'
      // blocks are in flight
      constexpr int NW = NT / 64;
      const int w = t >> 6, lane = t & 63;
      int sb[U], jj[U];
#pragma unroll
      for (int m = 0; m < U; ++m) {   // lanes past the pass repeat its last slot
        const int sl = min((w + m * NW) * 64 + lane, ns - 1);
        sb[m] = d.sblk[cb + sl];
        jj[m] = d.col[cb + sl];
      }
      for (int ch = w; ch * 64 < ns; ch += NW * U) {
        float4 hq[U][NQ];
        double uj[U][6];
        int tr[U], sbn[U], jjn[U];
#pragma unroll
        for (int m = 0; m < U; ++m) {
          tr[m] = sb[m] & 1;
          const float4 *b = H4 + (size_t)(sb[m] >> 1) * NQ;
#pragma unroll
          for (int q = 0; q < NQ; ++q) hq[m][q] = b[q];
          load6(u + (size_t)jj[m] * 6, uj[m]);
        }
#pragma unroll
        for (int m = 0; m < U; ++m) {
          const int sl = min((ch + (U + m) * NW) * 64 + lane, ns - 1);
          sbn[m] = d.sblk[cb + sl];
          jjn[m] = d.col[cb + sl];
        }
#pragma unroll
        for (int m = 0; m < U; ++m) {
          const int sl = (ch + m * NW) * 64 + lane;
          const T *h = reinterpret_cast<const T *>(hq[m]);
          double o[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            double a = 0.0;
#pragma unroll
            for (int e = 0; e < 6; ++e) a += double(tr[m] ? h[e * 6 + c] : h[c * 6 + e]) * uj[m][e];
            o[c] = a;
          }
          if (sl < ns) {
            double2 *pp = prod2 + sl * 3;
            pp[0] = make_double2(o[0], o[1]);
            pp[1] = make_double2(o[2], o[3]);
            pp[2] = make_double2(o[4], o[5]);
          }
          sb[m] = sbn[m];
          jj[m] = jjn[m];
        }
      }
    } else {
      const double2 *H2 = reinterpret_cast<const double2 *>(d.hoff);
      double *prodw = reinterpret_cast<double *>(prod2);
      const int ni = ns * 2;   // (slot, half) items; a pair of adjacent lanes per slot
      for (int base = 0; base < ni; base += NT * U) {
        double2 hq[U][9];
        double uj[U][6];
        int id[U], tr[U];
#pragma unroll
        for (int m = 0; m < U; ++m) {   // lanes past the pass repeat its last item
          id[m] = min(base + m * NT + t, ni - 1);
          const int sl = id[m] >> 1;
          const int sb = d.sblk[cb + sl];
          const int jj = d.col[cb + sl];
          tr[m] = sb & 1;
          const double2 *b = H2 + (size_t)(sb >> 1) * 18 + (id[m] & 1) * 9;
#pragma unroll
          for (int q = 0; q < 9; ++q) hq[m][q] = b[q];
          load6(u + (size_t)jj * 6, uj[m]);
        }
#pragma unroll
        for (int m = 0; m < U; ++m) {
          const bool h = (id[m] & 1) != 0;
          const double *hr = reinterpret_cast<const double *>(hq[m]);   // rows 3h .. 3h + 2 as stored
          double own[3], give[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            double a = 0.0, g = 0.0;
            if (!tr[m]) {
#pragma unroll
              for (int e = 0; e < 6; ++e) a += hr[k * 6 + e] * uj[m][e];
            } else {
#pragma unroll
              for (int e = 0; e < 3; ++e) {
                const double ue = h ? uj[m][3 + e] : uj[m][e];
                a += (h ? hr[e * 6 + 3 + k] : hr[e * 6 + k]) * ue;
                g += (h ? hr[e * 6 + k] : hr[e * 6 + 3 + k]) * ue;
              }
            }
            own[k] = a;
            give[k] = g;
          }
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const double rx = __shfl_xor(give[k], 1);
            if (tr[m]) own[k] += rx;
          }
          if (base + m * NT + t < ni) {
            double *pw = prodw + (id[m] >> 1) * 6 + (h ? 3 : 0);
#pragma unroll
            for (int k = 0; k < 3; ++k) pw[k] = own[k];
          }
        }
      }
    }
    __syncthreads();
    if (cb == s0) add_diag();
    if (rowthr) {
      const int lo = max(rbeg, cb), hi = min(rend, cb + ns);
      for (int k = lo; k < hi; ++k) acc += prod[(k - cb) * 6 + c_out];
    }
    __syncthreads();
  }
  if (rdots == SPMV_DOTS_NONE) {   // uniform over the launch
    // the cycle's product, read twice more in the same cycle: streamed out
    // so that it does not take the matrix's place in the Infinity Cache
    if (rowthr) __builtin_nontemporal_store(acc, d.cAp + (size_t)row * 6 + c_out);
    return;
  }
  if (rowthr) d.cAp[(size_t)row * 6 + c_out] = acc;
  KSum ru = {0.0, 0.0}, wu = {0.0, 0.0}, rr = {0.0, 0.0};
  if (rowthr) {
    kadd(ru, rc * uc);
    kadd(wu, acc * uc);
    kadd(rr, rc * rc);
  }
  block_ksum3(ru, wu, rr);
  if (t == 0) {
    d.part_b[lb] = make_double2(wu.s, wu.c);
    if (rdots == SPMV_DOTS_ALL) {
      d.part_a[lb] = make_double2(ru.s, ru.c);
      d.part_c[lb] = make_double2(rr.s, rr.c);
    }
  }
  // the update's dot partials this workgroup merges, if any (at the end, so
  // that their loads do not sit ahead of the block loads)
  const int sb0 = d.scene_pbeg[scene] / SPMV_ROWS, sb1 = d.scene_pbeg[scene + 1] / SPMV_ROWS, gl = lb - sb0;
  if (rdots == SPMV_DOTS_WU && gl % DOT_GROUP == 0 && t < 64) {   // all of wavefront 0
    double2 ga = make_double2(0.0, 0.0), gc = make_double2(0.0, 0.0);
    const int k = lb + t;
    if (t < DOT_GROUP && k < sb1) {
      ga = d.part_a[k];
      gc = d.part_c[k];
    }
    const KSum a = wave_ksum(KSum{ga.x, ga.y}), c = wave_ksum(KSum{gc.x, gc.y});
    if (t == 0) {
      const int slot = sb0 / (TILE / SPMV_ROWS) + gl / DOT_GROUP;
      d.part_ag[slot] = make_double2(a.s, a.c);
      d.part_cg[slot] = make_double2(c.s, c.c);
    }
  }
}

// per-scene scalars of one iteration and the stop test |r| <= eps_r |z|.
// The partial loads do not wait for the activity flag: everything the block
// reads is issued at once, then the three sums share one LDS round.
// GROUPED: (r, u) and (r, r) arrive merged per DOT_GROUP blocks by the SpMV
// (one slot per TILE rows of the scene, the first ceil(blocks / DOT_GROUP)
// used) and (w, u) per block; otherwise all three per block.  One workgroup
// of SCAL_THREADS per scene: a narrow workgroup starts and reduces sooner,
// and U loads per thread cover the plate's 6,845 blocks in two trips.
constexpr int SCAL_THREADS = 256;
template <bool GROUPED> __global__ __launch_bounds__(SCAL_THREADS) void k_cg_scalars(DevPtrs d, Params P) {
  static_assert(DOT_GROUP >= TILE / SPMV_ROWS && TILE % SPMV_ROWS == 0, "one grouped slot per tile at most");
  const int s = blockIdx.x;
  SceneCtl &c = d.ctl[s];
  const int b0 = d.scene_pbeg[s] / SPMV_ROWS, b1 = d.scene_pbeg[s + 1] / SPMV_ROWS;
  const int active = c.cg_active;
  // the scalars the decision needs, fetched with the partials
  const double rz_prev = c.rz, alpha_prev = c.alpha, cg_tol = c.cg_tol;
  const int cg_it = c.cg_it;
  const int t = threadIdx.x;
  KSum ru = {0.0, 0.0}, wu = {0.0, 0.0}, rr = {0.0, 0.0};
  if constexpr (GROUPED) {
    constexpr int U = 14;
    const int g0 = b0 / (TILE / SPMV_ROWS), g1 = g0 + (b1 - b0 + DOT_GROUP - 1) / DOT_GROUP;
    for (int k = g0 + t; k < g1; k += SCAL_THREADS) {
      const double2 pa = d.part_ag[k], pc = d.part_cg[k];
      ru = kmerge(ru, KSum{pa.x, pa.y});
      rr = kmerge(rr, KSum{pc.x, pc.y});
    }
    for (int k0 = b0; k0 < b1; k0 += U * SCAL_THREADS) {
      double2 pb[U];
#pragma unroll
      for (int m = 0; m < U; ++m) pb[m] = d.part_b[min(k0 + m * SCAL_THREADS + t, b1 - 1)];
#pragma unroll
      for (int m = 0; m < U; ++m)
        if (k0 + m * SCAL_THREADS + t < b1) wu = kmerge(wu, KSum{pb[m].x, pb[m].y});
    }
  } else {
    constexpr int U = 14;
    for (int k0 = b0; k0 < b1; k0 += U * SCAL_THREADS) {
      double2 pa[U], pb[U], pc[U];
#pragma unroll
      for (int m = 0; m < U; ++m) {
        const int k = min(k0 + m * SCAL_THREADS + t, b1 - 1);
        pa[m] = d.part_a[k];
        pb[m] = d.part_b[k];
        pc[m] = d.part_c[k];
      }
#pragma unroll
      for (int m = 0; m < U; ++m) {
        if (k0 + m * SCAL_THREADS + t >= b1) continue;
        ru = kmerge(ru, KSum{pa[m].x, pa[m].y});
        wu = kmerge(wu, KSum{pb[m].x, pb[m].y});
        rr = kmerge(rr, KSum{pc[m].x, pc[m].y});
      }
    }
  }
  // the element repulsion's share of (w, u), added after the bond SpMV
  if (P.contact) {
    const int t0 = d.scene_pbeg[s] / TILE, t1 = d.scene_pbeg[s + 1] / TILE;
    for (int k = t0 + (int)threadIdx.x; k < t1; k += blockDim.x) wu = kmerge(wu, KSum{d.part_d[k].x, d.part_d[k].y});
  }
  // the host's poll slot holds 1 while the solve runs (set when it starts);
  // it is written only when this scene stops
  if (!active) return;
  block_ksum3(ru, wu, rr);
  if (threadIdx.x != 0) return;
  const double gamma = ru.s + ru.c, delta = wu.s + wu.c;
  c.rr = rr.s + rr.c;
  c.rz_new = gamma;   // kept for the trace
  c.pAp = delta;
  bool stop = !(sqrt(c.rr) > cg_tol) || cg_it >= P.max_cg || !(gamma > 0.0);
  double alpha = 0.0, beta = 0.0;
  if (!stop) {
    if (cg_it == 0) {
      beta = 0.0;
      alpha = gamma / delta;
      if (!(delta > 0.0)) stop = true;
    } else {
      beta = gamma / rz_prev;
      const double den = delta - beta * gamma / alpha_prev;
      alpha = gamma / den;
      if (!(den > 0.0)) stop = true;
    }
  }
  if (stop || !isfinite(alpha) || !isfinite(beta)) {   // x holds the solution of this solve
    c.cg_active = 0;
    if (gridDim.x == 1) {
      d.counters[1] = 0;
      d.counters[5] = 0;
    }
  } else {
    c.rz = gamma;
    c.alpha = alpha;
    c.beta = beta;
    c.cg_it = cg_it + 1;
    c.cg_total += 1;
  }
}

// p = u + beta p ; q = w + beta q ; x += alpha p ; r -= alpha q ; u = M^-1 r
// (with multigrid t0 = omega D^-1 r, the first step of the V-cycle, in place
// of u).  Thread (row, component): every vector is read and written with unit
// stride; the new residual of the row is shared through LDS for M^-1 r, and
// the rows' Jacobi inverses are staged there with 16-byte loads (read
// directly, each thread would issue six scattered 4-byte loads).
// With rdots the kernel also writes the (r, u) and (r, r) partials of each
// SPMV_ROWS-row block (the SpMV then skips them): thread (row, c) adds its
// product, each wavefront reduces, and the block's three wavefronts merge in
// order, the tree the SpMV uses, so the partials are bit-identical to the
// SpMV's.
template <typename T, int ROWS> __global__ __launch_bounds__(6 * ROWS) void k_cg_update(DevPtrs d, int rdots) {
  static_assert(ROWS % SPMV_ROWS == 0 && 6 * SPMV_ROWS == 192, "dot blocks of three wavefronts");
  __shared__ double rs[6 * ROWS];
  const int r0 = blockIdx.x * ROWS;
  const int scene = row_scene(d, r0);
  const SceneCtl &c = d.ctl[scene];
  if (!c.cg_active) return;
  const double a = c.alpha, b = c.beta;
  const int t = threadIdx.x;
  const size_t o = (size_t)r0 * 6 + t;
  // With FP32 blocks (the mixed path) x, r, p, q, w and the Jacobi inverse
  // are loaded and stored non-temporally: the SpMV reads none of them (it
  // leaves the r dots to this kernel; with multigrid it reads r once), and
  // keeping them out of the caches leaves room there for the SpMV's matrix
  // and u (about 255 MB against the 256 MB Infinity Cache) between
  // iterations.  u, which the SpMV gathers, is stored normally.  The FP64
  // matrix does not fit either way and keeps plain accesses (non-temporal
  // ones there cost the update more than they gain the SpMV).
  constexpr bool NT = sizeof(T) == 4;
  auto ld = [](const auto *q) { if constexpr (NT) return __builtin_nontemporal_load(q); else return *q; };
  auto stn = [](double v, double *q) { if constexpr (NT) __builtin_nontemporal_store(v, q); else *q = v; };
  // the block's Jacobi inverses (ROWS x 21 T, contiguous) staged in LDS
  // with 16-byte loads
  typedef float v4f __attribute__((ext_vector_type(4)));
  constexpr int NPC = ROWS * 21 * (int)sizeof(T) / 16;
  static_assert(ROWS * 21 * sizeof(T) % 16 == 0, "16-byte pieces");
  __shared__ v4f dl4[NPC];
  {
    const v4f *src = reinterpret_cast<const v4f *>(reinterpret_cast<const T *>(d.dinv) + (size_t)r0 * 21);
    for (int k = t; k < NPC; k += 6 * ROWS) dl4[k] = ld(src + k);
  }
  const double x = ld(d.cx + o), rv = ld(d.cr + o), u = ld(d.cs + o), w = ld(d.cAp + o);
  const double p = ld(d.cp + o), q = ld(d.cq + o);
  const double pn = u + b * p, qn = w + b * q;
  const double xn = x + a * pn, rn = rv - a * qn;
  rs[t] = rn;
  stn(pn, d.cp + o);
  stn(qn, d.cq + o);
  stn(xn, d.cx + o);
  stn(rn, d.cr + o);
  __syncthreads();
  const int rl = t / 6, cc = t - rl * 6;
  const T *Di = reinterpret_cast<const T *>(dl4) + rl * 21;
  double un = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) un += double(Di[up6(cc, k)]) * rs[rl * 6 + k];
  if (d.amg_t0) {   // multigrid (uniform over the launch): the cycle's pre-smoothed
                    // start; the cycle's last kernel writes u and the r dots
    d.amg_t0[o] = AMG_OMEGA * un;
    return;
  }
  d.cs[o] = un;
  if (!rdots) return;   // uniform over the launch
  constexpr int NWV = 6 * ROWS / 64;
  __shared__ double wd[4][NWV];
  KSum ru = {0.0, 0.0}, rr = {0.0, 0.0};
  kadd(ru, rn * un);
  kadd(rr, rn * rn);
  ru = wave_ksum(ru);
  rr = wave_ksum(rr);
  const int wv = t >> 6;
  if ((t & 63) == 0) { wd[0][wv] = ru.s; wd[1][wv] = ru.c; wd[2][wv] = rr.s; wd[3][wv] = rr.c; }
  __syncthreads();
  if (t < ROWS / SPMV_ROWS) {
    KSum a = {0.0, 0.0}, c2 = {0.0, 0.0};
    for (int k = 3 * t; k < 3 * t + 3; ++k) {
      a = kmerge(a, KSum{wd[0][k], wd[1][k]});
      c2 = kmerge(c2, KSum{wd[2][k], wd[3][k]});
    }
    const int blk = r0 / SPMV_ROWS + t;
    d.part_a[blk] = make_double2(a.s, a.c);
    d.part_c[blk] = make_double2(c2.s, c2.c);
  }
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

// Algorithm 1 direction: -grad f.  In the reduced coordinates (dp, y) with
// dq = G_l(q)^T y the rows of G_l are orthonormal, so -grad f is x = -z.
__global__ __launch_bounds__(TILE) void k_steepest(DevPtrs d) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  if (!d.ctl[d.psid[blockIdx.x * TILE]].newton_active) return;
  double z[6];
  load6(d.z + (size_t)r * 6, z);
#pragma unroll
  for (int k = 0; k < 6; ++k) z[k] = -z[k];
  store6(d.cx + (size_t)r * 6, z);
}

__global__ void k_slope(DevPtrs d, Params P) {
  const int s = blockIdx.x;
  SceneCtl &c = d.ctl[s];
  if (!c.newton_active) return;
  const int pb = d.scene_pbeg[s] / TILE, pe = d.scene_pbeg[s + 1] / TILE;
  const KSum a = range_ksum(d.part_a, pb, pe);
  if (threadIdx.x != 0) return;
  c.slope = a.s + a.c;
  // first-order search: from twice the last accepted step (1 on the first)
  c.alpha_ls = P.first_order ? fmin(1.0, 2.0 * (c.newton_it == 0 ? 0.5 : c.alpha_prev)) : 1.0;
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
  // Armijo test.  When the predicted decrease -alpha * slope is below the
  // objective's FP64 resolution (1e-15 |Phi|), the comparison of two sums of
  // that size is decided by rounding: there a trial is accepted unless it
  // raises Phi by more than that resolution, so that the Newton step near
  // the fixed point is not cut down by rounding noise
  const double res = 1e-15 * fabs(c.phi);
  const double slack = (-c.alpha_ls * c.slope <= res) ? res : 0.0;
  if (isfinite(phit) && phit <= c.phi + P.armijo_c * c.alpha_ls * c.slope + slack) {
    c.ls_accept = 1;
    c.ls_active = 0;
    c.unresolved = -c.alpha_ls * c.slope <= 1e-15 * fabs(c.phi);
    c.alpha_prev = c.alpha_ls;
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
void launch_newton_check(const DevPtrs &d, const Params &P, int first, bool rows, hipStream_t s) {
  k_newton_check<<<P.n_scenes, 256, 0, s>>>(d, P, first, rows ? 1 : 0);
}
void launch_count_active(const DevPtrs &d, int n_scenes, int slot, hipStream_t s) {
  k_count_active<<<1, 256, 0, s>>>(d, n_scenes, slot);
}
void launch_cg_init(const DevPtrs &d, bool mixed, hipStream_t s) {
  const int nb = d.n_pad / TILE;
  if (mixed) k_cg_init<float><<<nb, TILE, 0, s>>>(d);
  else k_cg_init<double><<<nb, TILE, 0, s>>>(d);
}
// launch shapes the autotuner chooses from (bitwise-identical results)
static const int kSpmvShape[][2] = {{256, 1}, {192, 1}, {256, 2}, {512, 1}, {192, 2}, {384, 1}, {384, 2}};
static const int kUpdateRows[] = {64, 32, 128};
int spmv_variants() { return (int)(sizeof(kSpmvShape) / sizeof(kSpmvShape[0])); }
int update_variants() { return (int)(sizeof(kUpdateRows) / sizeof(kUpdateRows[0])); }
void spmv_shape(int v, int *threads, int *trips) { *threads = kSpmvShape[v][0]; *trips = kSpmvShape[v][1]; }
int update_rows(int v) { return kUpdateRows[v]; }

template <typename T> static void spmv_dispatch(const DevPtrs &d, int v, int rd, int rev, hipStream_t s) {
  static_assert(TILE % SPMV_ROWS == 0, "SpMV tiling");
  const int nsp = d.n_pad / SPMV_ROWS;
  switch (v) {
    case 1: k_spmv<T, 192, 1><<<nsp, 192, 0, s>>>(d, rd, rev); break;
    case 2: k_spmv<T, 256, 2><<<nsp, 256, 0, s>>>(d, rd, rev); break;
    case 3: k_spmv<T, 512, 1><<<nsp, 512, 0, s>>>(d, rd, rev); break;
    case 4: k_spmv<T, 192, 2><<<nsp, 192, 0, s>>>(d, rd, rev); break;
    case 5: k_spmv<T, 384, 1><<<nsp, 384, 0, s>>>(d, rd, rev); break;
    case 6: k_spmv<T, 384, 2><<<nsp, 384, 0, s>>>(d, rd, rev); break;
    default: k_spmv<T, 256, 1><<<nsp, 256, 0, s>>>(d, rd, rev); break;
  }
}
void launch_spmv(const DevPtrs &d, bool mixed, int variant, hipStream_t s, int dots, bool reverse) {
  if (mixed) spmv_dispatch<float>(d, variant, dots, reverse ? 1 : 0, s);
  else spmv_dispatch<double>(d, variant, dots, reverse ? 1 : 0, s);
}
void launch_cg_scalars(const DevPtrs &d, const Params &P, hipStream_t s, bool grouped) {
  if (grouped) k_cg_scalars<true><<<P.n_scenes, SCAL_THREADS, 0, s>>>(d, P);
  else k_cg_scalars<false><<<P.n_scenes, SCAL_THREADS, 0, s>>>(d, P);
}
template <typename T> static void update_dispatch(const DevPtrs &d, int v, int rd, hipStream_t s) {
  static_assert(TILE % 128 == 0, "update tiling");
  switch (v) {
    case 1: k_cg_update<T, 32><<<d.n_pad / 32, 6 * 32, 0, s>>>(d, rd); break;
    case 2: k_cg_update<T, 128><<<d.n_pad / 128, 6 * 128, 0, s>>>(d, rd); break;
    default: k_cg_update<T, 64><<<d.n_pad / 64, 6 * 64, 0, s>>>(d, rd); break;
  }
}
void launch_cg_update(const DevPtrs &d, bool mixed, int variant, hipStream_t s, bool rdots) {
  if (mixed) update_dispatch<float>(d, variant, rdots ? 1 : 0, s);
  else update_dispatch<double>(d, variant, rdots ? 1 : 0, s);
}
void launch_cg_slope(const DevPtrs &d, const Params &P, hipStream_t s) {
  k_slope_part<<<d.n_pad / TILE, TILE, 0, s>>>(d);
  k_slope<<<P.n_scenes, 256, 0, s>>>(d, P);
}
void launch_steepest(const DevPtrs &d, hipStream_t s) {
  k_steepest<<<d.n_pad / TILE, TILE, 0, s>>>(d);
}
void launch_ls_decide(const DevPtrs &d, const Params &P, hipStream_t s) {
  k_ls_decide<<<P.n_scenes, 256, 0, s>>>(d, P);
}

}  // namespace bdem
