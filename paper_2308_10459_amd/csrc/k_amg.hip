// Aggregation multigrid preconditioner: numeric setup at the first Newton
// iteration of a step, or at every one (rigid-body-mode prolongation,
// Galerkin coarse operators, block-Jacobi inverses, dense inverse of the
// last level and the tail matrix per scene), the fine coupling H P after
// every Hessian evaluation, and the V-cycle applied to the PCG residual.
// The symbolic hierarchy and its definitions are described in
// bdem_amg.hpp.  All sums run in a fixed order (contribution and child
// lists are sorted at create), so results are reproducible run to run.
#include <algorithm>

#include "bdem_amg.hpp"
#include "bdem_math.hpp"

namespace bdem {

// ---------------------------------------------------------------------------
// small dense helpers (FP64)
// ---------------------------------------------------------------------------

// y = P x for P = [[I, -[d]x], [0, S]]: (t - d x w, S w)
__device__ __forceinline__ void p_apply(const double (&dd)[3], const double (&S)[9], const double (&x)[6],
                                        double (&y)[6]) {
  const double w[3] = {x[3], x[4], x[5]};
  y[0] = x[0] - (dd[1] * w[2] - dd[2] * w[1]);
  y[1] = x[1] - (dd[2] * w[0] - dd[0] * w[2]);
  y[2] = x[2] - (dd[0] * w[1] - dd[1] * w[0]);
#pragma unroll
  for (int r = 0; r < 3; ++r) y[3 + r] = S[r * 3] * w[0] + S[r * 3 + 1] * w[1] + S[r * 3 + 2] * w[2];
}
// y = P^T x: (x_p, d x x_p + S^T x_y)
__device__ __forceinline__ void pt_apply(const double (&dd)[3], const double (&S)[9], const double (&x)[6],
                                         double (&y)[6]) {
  y[0] = x[0]; y[1] = x[1]; y[2] = x[2];
  y[3] = (dd[1] * x[2] - dd[2] * x[1]) + S[0] * x[3] + S[3] * x[4] + S[6] * x[5];
  y[4] = (dd[2] * x[0] - dd[0] * x[2]) + S[1] * x[3] + S[4] * x[4] + S[7] * x[5];
  y[5] = (dd[0] * x[1] - dd[1] * x[0]) + S[2] * x[3] + S[5] * x[4] + S[8] * x[5];
}

__device__ __forceinline__ void ident3(double (&S)[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) S[k] = (k % 4 == 0) ? 1.0 : 0.0;
}

// 6x6 SPD inverse (full storage) by Cholesky; false if not positive definite
__device__ __forceinline__ bool spd_inv36(const double (&A)[36], double (&X)[36]) {
  double L[6][6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double dj = A[j * 6 + j];
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= L[j][k] * L[j][k];
    if (!(dj > 0.0)) return false;
    dj = sqrt(dj);
    L[j][j] = dj;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double v = A[i * 6 + j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / dj;
    }
  }
  double Y[6][6];   // L^-1
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      if (i < c) { Y[i][c] = 0.0; continue; }
      double v = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k)
        if (k >= c) v -= L[i][k] * Y[k][c];
      Y[i][c] = v / L[i][i];
    }
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) v += Y[k][r] * Y[k][c];
      X[r * 6 + c] = v;
    }
  return true;
}

template <typename T>
__device__ __forceinline__ void mat36_apply(const T *M, const double (&x)[6], double (&y)[6]) {
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    double a = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) a += double(M[r * 6 + c]) * x[c];
    y[r] = a;
  }
}
template <typename T>
__device__ __forceinline__ void sym21_apply(const T *M, const double (&x)[6], double (&y)[6]) {
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    double a = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) a += double(M[up6(r, c)]) * x[c];
    y[r] = a;
  }
}
__device__ __forceinline__ void ld6(const double *p, double (&v)[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = p[k];
}
__device__ __forceinline__ void st6(double *p, const double (&v)[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) p[k] = v[k];
}
// a particle's prolongator block (x_i - c_a, S_i), stored in T: 12 values
template <typename T>
__device__ __forceinline__ void load_pd0(const AmgDev &a, int i, double (&dd)[3], double (&S)[9]) {
  const T *p = reinterpret_cast<const T *>(a.pd0) + (size_t)i * 12;
#pragma unroll
  for (int m = 0; m < 3; ++m) dd[m] = double(p[m]);
#pragma unroll
  for (int m = 0; m < 9; ++m) S[m] = double(p[3 + m]);
}


// ---------------------------------------------------------------------------
// numeric setup
// ---------------------------------------------------------------------------

// level 1: centroids of the aggregates (iterate positions of their free
// particles), and each particle's (x_i - c_a, S_i = 1/2 R(q_i)^T).  One
// wavefront per aggregate: lane k takes members k, k + 64, ...; the lanes'
// sums meet in a fixed butterfly.
template <typename T> __global__ __launch_bounds__(256) void k_amg_geom1(DevPtrs d, AmgDev a) {
  const AmgLevel &L = a.lv[1];
  const int A = (blockIdx.x * 256 + (int)threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (A >= L.n) return;   // uniform over the wavefront
  const int mb = L.mbeg[A], me = L.mbeg[A + 1];
  const bool act = L.active[A] != 0;
  double c[4] = {0.0, 0.0, 0.0, 0.0};   // position sum, count
  for (int k = mb + lane; k < me; k += 64) {
    const int i = L.mlist[k];
    if (act && d.flags[i] != 0) continue;
    const double4 p = d.px[i];
    c[0] += p.x; c[1] += p.y; c[2] += p.z; c[3] += 1.0;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int m = 0; m < 4; ++m) c[m] += __shfl_xor(c[m], off, 64);
  c[0] /= c[3]; c[1] /= c[3]; c[2] /= c[3];
  if (lane == 0) { L.cen[3 * A] = c[0]; L.cen[3 * A + 1] = c[1]; L.cen[3 * A + 2] = c[2]; }
  for (int k = mb + lane; k < me; k += 64) {
    const int i = L.mlist[k];
    const double4 p = d.px[i], q = d.qx[i];
    T *o = reinterpret_cast<T *>(a.pd0) + (size_t)i * 12;
    o[0] = T(p.x - c[0]); o[1] = T(p.y - c[1]); o[2] = T(p.z - c[2]);
    // R(q) for q = (x, y, z, w); S = 1/2 R^T
    const double x = q.x, y = q.y, z = q.z, w = q.w;
    const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                         2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                         2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) o[3 + r * 3 + cc] = T(0.5 * R[cc * 3 + r]);
  }
}

// level l >= 2: centroids of the active children's centroids, children's offsets
__global__ __launch_bounds__(256) void k_amg_geom(AmgDev a, int l) {
  const AmgLevel &L = a.lv[l], &F = a.lv[l - 1];
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= L.n) return;
  const int mb = L.mbeg[A], me = L.mbeg[A + 1];
  const bool act = L.active[A] != 0;
  double c[3] = {0.0, 0.0, 0.0};
  int cnt = 0;
  for (int k = mb; k < me; ++k) {
    const int i = L.mlist[k];
    if (act && !F.active[i]) continue;
    c[0] += F.cen[3 * i]; c[1] += F.cen[3 * i + 1]; c[2] += F.cen[3 * i + 2];
    ++cnt;
  }
  c[0] /= cnt; c[1] /= cnt; c[2] /= cnt;
  L.cen[3 * A] = c[0]; L.cen[3 * A + 1] = c[1]; L.cen[3 * A + 2] = c[2];
  for (int k = mb; k < me; ++k) {
    const int i = L.mlist[k];
    F.pd[3 * i] = F.cen[3 * i] - c[0];
    F.pd[3 * i + 1] = F.cen[3 * i + 1] - c[1];
    F.pd[3 * i + 2] = F.cen[3 * i + 2] - c[2];
  }
}

// acc += P_r^T H P_c, column by column (H: 36 values, row-major, the
// transpose of such a block, or the packed upper triangle of a symmetric
// block), the block read once
enum BlockForm { BLK_FULL = 0, BLK_TRANSPOSED = 1, BLK_SYM21 = 2 };
template <typename T>
__device__ __forceinline__ void add_ptap(double (&acc)[36], const T *H, int form, const double (&dr)[3],
                                         const double (&Sr)[9], const double (&dc)[3], const double (&Sc)[9]) {
  double Hm[36];
  if (form == BLK_SYM21) {
    T h[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) h[k] = H[k];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) Hm[r * 6 + c] = double(h[up6(r, c)]);
  } else {
    const bool tr = form == BLK_TRANSPOSED;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) Hm[r * 6 + c] = double(H[tr ? c * 6 + r : r * 6 + c]);
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double e[6] = {0, 0, 0, 0, 0, 0};
    e[c] = 1.0;
    double v[6], w[6], o[6];
    p_apply(dc, Sc, e, v);
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) t += Hm[r * 6 + k] * v[k];
      w[r] = t;
    }
    pt_apply(dr, Sr, w, o);
#pragma unroll
    for (int r = 0; r < 6; ++r) acc[r * 6 + c] += o[r];
  }
}

// Galerkin block of every level-1 slot from the fine diagonal (packed) and
// off-diagonal blocks of its contribution list.  One wavefront per slot (an
// aggregate of ~60-90 particles has ~1,000 contributions on its diagonal
// slot): lane k takes contributions k, k + 64, ...; the lanes' 36 sums are
// then added in lane order through LDS.
template <typename T> __global__ __launch_bounds__(64) void k_amg_galerkin1(DevPtrs d, AmgDev a) {
  __shared__ double part[64][37];
  const AmgLevel &L = a.lv[1];
  const int s = blockIdx.x, lane = threadIdx.x;
  double acc[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) acc[k] = 0.0;
  const T *hd = reinterpret_cast<const T *>(d.hdiag), *ho = reinterpret_cast<const T *>(d.hoff);
  for (int k = L.gptr[s] + lane; k < L.gptr[s + 1]; k += 64) {
    const int src = L.gsrc[k];
    const bool diag = src < 0;
    const int i = diag ? -1 - src : a.slot_row0[src];
    const int j = diag ? i : d.col[src];
    if (d.flags[i] != 0 || d.flags[j] != 0) continue;   // P is zero on non-unknowns
    double dr[3], Sr[9], dc[3], Sc[9];
    load_pd0<T>(a, i, dr, Sr);
    load_pd0<T>(a, j, dc, Sc);
    if (diag) {
      add_ptap<T>(acc, hd + (size_t)i * 21, BLK_SYM21, dr, Sr, dc, Sc);
    } else {
      const int sb = d.sblk[src];
      add_ptap<T>(acc, ho + (size_t)(sb >> 1) * 36, (sb & 1) ? BLK_TRANSPOSED : BLK_FULL, dr, Sr, dc, Sc);
    }
  }
#pragma unroll
  for (int k = 0; k < 36; ++k) part[lane][k] = acc[k];
  __syncthreads();
  if (lane >= 36) return;
  double v = 0.0;
  for (int m = 0; m < 64; ++m) v += part[m][lane];
  const int A = L.slot_row[s];
  if (!L.active[A] && L.dslot[A] == s) v = (lane % 7 == 0) ? 1.0 : 0.0;
  reinterpret_cast<T *>(L.val)[(size_t)s * 36 + lane] = T(v);
}

template <typename T> __global__ __launch_bounds__(128) void k_amg_galerkin(AmgDev a, int l) {
  const AmgLevel &L = a.lv[l], &F = a.lv[l - 1];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= L.nslots) return;
  double acc[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) acc[k] = 0.0;
  double S[9];
  ident3(S);
  const T *fv = reinterpret_cast<const T *>(F.val);
  for (int k = L.gptr[s]; k < L.gptr[s + 1]; ++k) {
    const int src = L.gsrc[k];
    const int i = F.slot_row[src], j = F.col[src];
    if (!F.active[i] || !F.active[j]) continue;
    const double dr[3] = {F.pd[3 * i], F.pd[3 * i + 1], F.pd[3 * i + 2]};
    const double dc[3] = {F.pd[3 * j], F.pd[3 * j + 1], F.pd[3 * j + 2]};
    add_ptap<T>(acc, fv + (size_t)src * 36, BLK_FULL, dr, S, dc, S);
  }
  const int A = L.slot_row[s];
  if (!L.active[A] && L.dslot[A] == s) {
#pragma unroll
    for (int k = 0; k < 36; ++k) acc[k] = (k % 7 == 0) ? 1.0 : 0.0;
  }
  T *o = reinterpret_cast<T *>(L.val) + (size_t)s * 36;
#pragma unroll
  for (int k = 0; k < 36; ++k) o[k] = T(acc[k]);
}

// block-Jacobi inverse of every node of a coarse level
template <typename T> __global__ __launch_bounds__(128) void k_amg_dinv(AmgDev a, int l) {
  const AmgLevel &L = a.lv[l];
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= L.n) return;
  const T *B = reinterpret_cast<const T *>(L.val) + (size_t)L.dslot[A] * 36;
  double M[36], X[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) M[k] = double(B[k]);
  // symmetrise: FP32 Galerkin sums are symmetric only to rounding
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r + 1; c < 6; ++c) { const double v = 0.5 * (M[r * 6 + c] + M[c * 6 + r]); M[r * 6 + c] = v; M[c * 6 + r] = v; }
  if (!spd_inv36(M, X)) {
#pragma unroll
    for (int k = 0; k < 36; ++k) X[k] = 0.0;
#pragma unroll
    for (int r = 0; r < 6; ++r) X[r * 7] = M[r * 7] > 0.0 ? 1.0 / M[r * 7] : 1.0;
  }
  T *o = reinterpret_cast<T *>(L.dinv) + (size_t)A * 36;
#pragma unroll
  for (int k = 0; k < 36; ++k) o[k] = T(X[k]);
}

// dense inverse of the last level of each scene (one workgroup per scene):
// Gauss-Jordan without pivoting on the symmetric positive definite operator,
// in LDS (at most 6 * AMG_COARSE_MAX rows); the inverse goes to cwork
template <typename T> __global__ __launch_bounds__(1024) void k_amg_coarse_inverse(AmgDev a) {
  constexpr int NMAX = 6 * AMG_COARSE_MAX;
  __shared__ double M[NMAX * NMAX], X[NMAX * NMAX], fcol[NMAX];
  const int sc = blockIdx.x;
  const AmgLevel &L = a.lv[a.L];
  const int nb = a.cbeg[sc], ne = a.cbeg[sc + 1], m = ne - nb, N = 6 * m;
  if (m == 0) return;
  const T *v = reinterpret_cast<const T *>(L.val);
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) { M[e] = 0.0; X[e] = (e / N == e % N) ? 1.0 : 0.0; }
  __syncthreads();
  for (int A = nb; A < ne; ++A)
    for (int s = L.row_ptr[A]; s < L.row_ptr[A + 1]; ++s) {
      const int B = L.col[s];
      for (int e = threadIdx.x; e < 36; e += blockDim.x)
        M[(6 * (A - nb) + e / 6) * N + 6 * (B - nb) + e % 6] = double(v[(size_t)s * 36 + e]);
    }
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    const double piv = M[k * N + k];
    __syncthreads();
    for (int c = threadIdx.x; c < N; c += blockDim.x) { M[k * N + c] /= piv; X[k * N + c] /= piv; }
    __syncthreads();
    for (int r = threadIdx.x; r < N; r += blockDim.x) fcol[r] = M[r * N + k];
    __syncthreads();
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
      const int r = e / N, c = e - (e / N) * N;
      if (r == k) continue;
      const double f = fcol[r];
      M[r * N + c] -= f * M[k * N + c];
      X[r * N + c] -= f * X[k * N + c];
    }
    __syncthreads();
  }
  double *out = a.cwork + a.coff[sc];
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) out[e] = X[e];
}

// ---------------------------------------------------------------------------
// V-cycle
// ---------------------------------------------------------------------------

// fine pre-smoothing from zero: t0 = omega D^-1 r
template <typename T> __global__ __launch_bounds__(TILE) void k_amg_fine_pre(DevPtrs d, AmgDev a) {
  const int r = blockIdx.x * TILE + threadIdx.x;
  if (!d.ctl[row_scene(d, blockIdx.x * TILE)].cg_active) return;
  double x[6], y[6];
  ld6(d.cr + (size_t)r * 6, x);
  sym21_apply(reinterpret_cast<const T *>(d.dinv) + (size_t)r * 21, x, y);
#pragma unroll
  for (int k = 0; k < 6; ++k) y[k] *= AMG_OMEGA;
  st6(a.t0 + (size_t)r * 6, y);
}

// b of level 1 from the fine residual r - H t0 (r0 holds H t0), and with
// `smooth` (level 1 is not the coarsest) its pre-smoothing t = omega D^-1 b.
// R1_LANES lanes per level-1 node: lane k takes the node's particles k,
// k + R1_LANES, ...; the lanes' sums then meet in a fixed butterfly, and six
// of them write b and t.
constexpr int R1_LANES = 64;   // a cell of side 8 r_max holds 60-90 close-packed particles

template <int G> __device__ __forceinline__ void lanes_sum6(double (&v)[6]) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1)
#pragma unroll
    for (int m = 0; m < 6; ++m) v[m] += __shfl_xor(v[m], off, 64);
}

// row c (c < 6; clamped, so that every lane may load one) of node A's
// block-Jacobi inverse, loaded at a kernel's start, ahead of the sums it
// multiplies
template <typename T>
__device__ __forceinline__ void load_dinv_row(const AmgLevel &L, int A, int c, T (&di)[6]) {
  const T *Di = reinterpret_cast<const T *>(L.dinv) + (size_t)A * 36 + min(c, 5) * 6;
#pragma unroll
  for (int m = 0; m < 6; ++m) di[m] = Di[m];
}
// lane c < 6 of a node's group: b_c, and with `smooth` t_c = omega (D^-1 b)_c
// (di: row c of the node's inverse)
template <typename T>
__device__ __forceinline__ void store_b_and_smooth(const AmgLevel &L, int A, int c, const double (&acc)[6],
                                                   int smooth, const T (&di)[6]) {
  double bc = 0.0;
#pragma unroll
  for (int m = 0; m < 6; ++m)
    if (m == c) bc = acc[m];
  L.b[(size_t)A * 6 + c] = bc;
  if (!smooth) return;
  double y = 0.0;
#pragma unroll
  for (int m = 0; m < 6; ++m) y += double(di[m]) * acc[m];
  L.t[(size_t)A * 6 + c] = AMG_OMEGA * y;
}

typedef double nt_v2d __attribute__((ext_vector_type(2)));
typedef float nt_v4f __attribute__((ext_vector_type(4)));

// The members of a level-1 aggregate are consecutive rows (the internal
// order sorts particles by their aggregation cell; checked at create), so
// a wavefront stages its members' r - H t0 and prolongator records through
// LDS, R1_CHUNK members at a time: contiguous 16-byte pieces, every load of
// a chunk issued before the first store, read non-temporally (they are not
// read again in the cycle; the matrix the PCG's product reads next stays in
// the Infinity Cache).  Lane k then takes members k, k + 64, ... as before.
constexpr int R1_CHUNK = 128;   // an interior cell of 8 r_max holds ~90 close-packed particles
template <typename T>
__global__ __launch_bounds__(256) void k_amg_restrict1(DevPtrs d, AmgDev a, int smooth) {
  static_assert(R1_LANES == 64, "one wavefront per aggregate");
  constexpr int RW = 3;                            // 16-byte pieces of six doubles
  constexpr int PW = 12 * (int)sizeof(T) / 16;     // of a prolongator record
  constexpr int NX = R1_CHUNK * RW / 64, NPC = R1_CHUNK * PW / 64;   // pieces per lane
  __shared__ nt_v2d sx[4][R1_CHUNK * RW];
  __shared__ nt_v4f sp[4][R1_CHUNK * PW];
  const AmgLevel &L = a.lv[1];
  const int w = threadIdx.x >> 6, k0 = threadIdx.x & 63;
  const int A = blockIdx.x * 4 + w;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  T di[6];
  if (A < L.n) {   // uniform over the wavefront
    load_dinv_row<T>(L, A, k0, di);
    const int mb = L.mbeg[A], nm = L.mbeg[A + 1] - mb;
    const int row0 = L.mlist[mb];
    const nt_v2d *R2 = reinterpret_cast<const nt_v2d *>(d.cr + (size_t)row0 * 6);
    const nt_v2d *H2 = reinterpret_cast<const nt_v2d *>(a.r0 + (size_t)row0 * 6);
    const nt_v4f *P4 = reinterpret_cast<const nt_v4f *>(reinterpret_cast<const T *>(a.pd0) + (size_t)row0 * 12);
    for (int c0 = 0; c0 < nm; c0 += R1_CHUNK) {
      const int cnt = min(R1_CHUNK, nm - c0), nx = cnt * RW, np = cnt * PW;
      nt_v2d rv[NX], hv[NX];
      nt_v4f pv[NPC];
#pragma unroll
      for (int m = 0; m < NX; ++m) {   // pieces past the chunk repeat its last one
        const int q = min(k0 + 64 * m, nx - 1);
        rv[m] = __builtin_nontemporal_load(R2 + c0 * RW + q);
        hv[m] = __builtin_nontemporal_load(H2 + c0 * RW + q);
      }
#pragma unroll
      for (int m = 0; m < NPC; ++m) pv[m] = __builtin_nontemporal_load(P4 + c0 * PW + min(k0 + 64 * m, np - 1));
#pragma unroll
      for (int m = 0; m < NX; ++m)
        if (k0 + 64 * m < nx) sx[w][k0 + 64 * m] = rv[m] - hv[m];
#pragma unroll
      for (int m = 0; m < NPC; ++m)
        if (k0 + 64 * m < np) sp[w][k0 + 64 * m] = pv[m];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int k = k0; k < cnt; k += 64) {
        if (d.flags[row0 + c0 + k] != 0) continue;
        const double *xs = reinterpret_cast<const double *>(&sx[w][k * RW]);
        const T *ps = reinterpret_cast<const T *>(&sp[w][k * PW]);
        double dd[3], S[9], x[6], y[6];
#pragma unroll
        for (int m = 0; m < 3; ++m) dd[m] = double(ps[m]);
#pragma unroll
        for (int m = 0; m < 9; ++m) S[m] = double(ps[3 + m]);
#pragma unroll
        for (int m = 0; m < 6; ++m) x[m] = xs[m];
        pt_apply(dd, S, x, y);
#pragma unroll
        for (int m = 0; m < 6; ++m) acc[m] += y[m];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();   // every lane has read before the next pieces land
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  lanes_sum6<R1_LANES>(acc);
  if (A < L.n && k0 < 6) store_b_and_smooth<T>(L, A, k0, acc, smooth, di);
}

// r = b - A t on a level above the tail, one wavefront per row
// component (lane mod 6) of A_row x by one wavefront: lane (g, c) with
// g = lane / 6 < 10 takes the row's slots g, g + 10, ... for output
// component c; the ten partials of a component are then added in lane order
template <typename T>
__device__ __forceinline__ double wave_row_apply(const AmgLevel &L, int A, const double *x, int lane) {
  const T *val = reinterpret_cast<const T *>(L.val);
  const int s0 = L.row_ptr[A], s1 = L.row_ptr[A + 1];
  const int g = lane / 6, c = lane - g * 6;
  double part = 0.0;
  // four of the lane's slots at a time, all their loads issued before the
  // first product (a row of up to 40 blocks in one round)
  if (lane < 60)
    for (int sb = s0 + g; sb < s1; sb += 40) {
      int sl[4], cj[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        sl[m] = sb + 10 * m < s1 ? sb + 10 * m : sb;
        cj[m] = L.col[sl[m]];
      }
      T bv[4][6];
      double xv[4][6];
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int e = 0; e < 6; ++e) {
          bv[m][e] = val[(size_t)sl[m] * 36 + c * 6 + e];
          xv[m][e] = x[(size_t)cj[m] * 6 + e];
        }
#pragma unroll
      for (int m = 0; m < 4; ++m) {   // branch-free, so that no load sinks into a branch
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < 6; ++e) acc += double(bv[m][e]) * xv[m][e];
        part += (sb + 10 * m < s1) ? acc : 0.0;
      }
    }
  double y = 0.0;
  for (int k = 0; k < 10; ++k) y += __shfl(part, k * 6 + (lane % 6), 64);
  return y;
}

// Residual and restriction in one launch: for each node of level l + 1,
// r_A = b_A - (A_l t_l)_A on each of its children A (at most 8, a cell of
// twice the side), then b = sum over the active children of P_A^T r_A
// (S = I above the particles) and, with `smooth` (level l + 1 is not the
// coarsest), its pre-smoothing.  RR_THREADS threads per node: thread
// (g, h) takes child g and its row's slots h, h + 16, ..., all six
// components of each slot's product, with every load of a row of up to
// 16 RR_U slots issued at once; the sixteen lanes of a child meet in a
// fixed butterfly, the eight children in LDS in child order.
constexpr int RR_THREADS = 128;
template <typename T>
__global__ __launch_bounds__(256) void k_amg_resid_restrict(AmgDev a, int l, int smooth) {
  constexpr int U = sizeof(T) == 4 ? 2 : 1;      // slots in flight per thread (registers)
  constexpr int NQ = 36 * (int)sizeof(T) / 16;   // 16-byte pieces per block
  constexpr int NPB = 256 / RR_THREADS;           // nodes per workgroup
  __shared__ double zs[NPB][8][6];
  const AmgLevel &C = a.lv[l + 1], &F = a.lv[l];
  const int nl = threadIdx.x / RR_THREADS, tid = threadIdx.x % RR_THREADS;
  const int node = blockIdx.x * NPB + nl;
  const bool live = node < C.n;
  const int g = tid >> 4, h = tid & 15;
  double z[6] = {0, 0, 0, 0, 0, 0};
  T di[6];
  if (live) {   // uniform over each wavefront (two per node)
    load_dinv_row<T>(C, node, tid, di);
    const int mb = C.mbeg[node], me = C.mbeg[node + 1];
    const bool has = mb + g < me;
    const int A = C.mlist[has ? mb + g : mb];   // threads without a child repeat the first (dropped below)
    const bool act = has && F.active[A] != 0;
    const double dd[3] = {F.pd[3 * A], F.pd[3 * A + 1], F.pd[3 * A + 2]};
    double bA[6];
    ld6(F.b + (size_t)A * 6, bA);
    const int s0 = F.row_ptr[A], s1 = F.row_ptr[A + 1];
    const float4 *V4 = reinterpret_cast<const float4 *>(F.val);
    double y[6] = {0, 0, 0, 0, 0, 0};
    for (int sb = s0 + h; sb < s1; sb += 16 * U) {
      int sl[U];
      float4 bq[U][NQ];
      double xv[U][6];
#pragma unroll
      for (int m = 0; m < U; ++m) sl[m] = (sb + 16 * m < s1) ? sb + 16 * m : sb;
#pragma unroll
      for (int m = 0; m < U; ++m) {
        const float4 *b4 = V4 + (size_t)sl[m] * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q) bq[m][q] = b4[q];
        ld6(F.t + (size_t)F.col[sl[m]] * 6, xv[m]);
      }
#pragma unroll
      for (int m = 0; m < U; ++m) {   // branch-free, so that no load sinks into a branch
        const T *bv = reinterpret_cast<const T *>(bq[m]);
        const bool in = sb + 16 * m < s1;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          double acc = 0.0;
#pragma unroll
          for (int e = 0; e < 6; ++e) acc += double(bv[c * 6 + e]) * xv[m][e];
          y[c] += in ? acc : 0.0;
        }
      }
    }
    // the child's row sum over its sixteen lanes, r_A, and P_A^T r_A
#pragma unroll
    for (int off = 1; off < 16; off <<= 1)
#pragma unroll
      for (int c = 0; c < 6; ++c) y[c] += __shfl_xor(y[c], off, 64);
    double r[6], S[9];
#pragma unroll
    for (int c = 0; c < 6; ++c) r[c] = bA[c] - y[c];
    ident3(S);
    pt_apply(dd, S, r, z);
#pragma unroll
    for (int c = 0; c < 6; ++c) z[c] = act ? z[c] : 0.0;
  }
  if (h == 0)
#pragma unroll
    for (int c = 0; c < 6; ++c) zs[nl][g][c] = z[c];
  __syncthreads();
  if (live && tid < 6) {
    double acc[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) v += zs[nl][k][c];
      acc[c] = v;
    }
    store_b_and_smooth<T>(C, node, tid, acc, smooth, di);
  }
}

// t_f += P_f e for one member f of a level-l node, l >= 2 (a level l - 1
// node; S = I above the particles).  Level 1's correction is not prolonged
// here: the cycle's last kernel applies it to the particles.
__device__ __forceinline__ void prolong_one(const AmgDev &a, int l, int i, const double (&e)[6]) {
  const AmgLevel &F = a.lv[l - 1];
  if (!F.active[i]) return;
  const double dd[3] = {F.pd[3 * i], F.pd[3 * i + 1], F.pd[3 * i + 2]};
  double S[9], y[6];
  ident3(S);
  double *t = F.t + (size_t)i * 6;
  p_apply(dd, S, e, y);
#pragma unroll
  for (int m = 0; m < 6; ++m) t[m] += y[m];
}

// on each level going up: e_l = t_l + omega D^-1 (b_l - A t_l) (t_l already
// holds the prolonged correction), prolonged into the members of each node
// (level 1 keeps e_1 for the cycle's last kernel).  One wavefront per row;
// its lanes then take the row's members.
template <typename T> __global__ __launch_bounds__(256) void k_amg_post(AmgDev a, int l) {
  const AmgLevel &L = a.lv[l];
  const int A = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (A >= L.n) return;   // uniform over the wavefront
  // the row's b, t and inverse, loaded ahead of the row's product
  const int c6 = min(lane, 5);
  const double bl = L.b[(size_t)A * 6 + c6], tl = L.t[(size_t)A * 6 + c6];
  T di[6];
  load_dinv_row<T>(L, A, lane, di);
  const double y = wave_row_apply<T>(L, A, L.t, lane);
  const double rb = (lane < 6) ? bl - y : 0.0;
  double rv[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) rv[k] = __shfl(rb, k, 64);
  double ev = 0.0;
  if (lane < 6) {
    double u = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) u += double(di[k]) * rv[k];
    ev = tl + AMG_OMEGA * u;
    if (l == 1) L.e[(size_t)A * 6 + lane] = ev;
  }
  if (l == 1) return;   // uniform over the launch
  double e[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) e[k] = __shfl(ev, k, 64);
  for (int k = L.mbeg[A] + lane; k < L.mbeg[A + 1]; k += 64) prolong_one(a, l, L.mlist[k], e);
}

// ---------------------------------------------------------------------------
// The tail (levels Lt..L): one symmetric matrix N per scene (bdem_amg.hpp),
// formed at setup in FP64 from the coarsest level up, in four work slots
// per scene of (6 n_Lt)^2: slot 0 holds N of the level above, slot 1
// W = I - A S, slot 2 Q = P N P^T, slot 3 T = S + Q W; then N = S + W^T T
// goes to slot 0.  S = omega D^-1 of the level; P = [[I, -[d]x], [0, I]]
// for an active node (d its offset from its parent's centroid), zero for
// an inactive one.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void tail_range(const AmgDev &a, int l, int sc, int &nb, int &ne) {
  const int *tb = a.tbeg + (size_t)(l - a.Lt) * (gridDim.y + 1);
  nb = tb[sc];
  ne = tb[sc + 1];
}
__device__ __forceinline__ double *tail_slot(const AmgDev &a, int sc, int k) {
  return a.nwork + 4 * a.noff[sc] + (size_t)k * (size_t)(a.noff[sc + 1] - a.noff[sc]);
}

// slot 0 = the coarsest level's dense inverse
__global__ __launch_bounds__(256) void k_tail_init(AmgDev a) {
  const int sc = blockIdx.y;
  const int64_t m = 6 * (int64_t)(a.cbeg[sc + 1] - a.cbeg[sc]);
  const double *X = a.cwork + a.coff[sc];
  double *o = tail_slot(a, sc, 0);
  for (int64_t q = blockIdx.x * 256 + threadIdx.x; q < m * m; q += (int64_t)gridDim.x * 256) o[q] = X[q];
}

// slot 1 = W = I - A S of level l (dense, the scene's nodes): zeros first
// (node pairs without a block), then every block of the level's pattern
// (the diagonal ones included) from its slot
__global__ __launch_bounds__(256) void k_tail_zero_w(AmgDev a, int l) {
  const int sc = blockIdx.y;
  int nb, ne;
  tail_range(a, l, sc, nb, ne);
  const int N6 = 6 * (ne - nb);
  double *W = tail_slot(a, sc, 1);
  for (int q = blockIdx.x * 256 + threadIdx.x; q < N6 * N6; q += gridDim.x * 256) W[q] = 0.0;
}
template <typename T> __global__ __launch_bounds__(256) void k_tail_fill_w(AmgDev a, int l) {
  const int sc = blockIdx.y;
  const AmgLevel &L = a.lv[l];
  int nb, ne;
  tail_range(a, l, sc, nb, ne);
  const int N6 = 6 * (ne - nb);
  double *W = tail_slot(a, sc, 1);
  const T *val = reinterpret_cast<const T *>(L.val), *dinv = reinterpret_cast<const T *>(L.dinv);
  const int s0 = L.row_ptr[nb], s1 = L.row_ptr[ne];
  for (int q = blockIdx.x * 256 + threadIdx.x; q < 36 * (s1 - s0); q += gridDim.x * 256) {
    const int sl = s0 + q / 36, e = q - (q / 36) * 36, r = e / 6, c = e - (e / 6) * 6;
    const int i = L.slot_row[sl], j = L.col[sl];
    const T *Ab = val + (size_t)sl * 36 + r * 6, *Sj = dinv + (size_t)j * 36 + c;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) v += double(Ab[k]) * double(Sj[k * 6]);
    W[(size_t)(6 * (i - nb) + r) * N6 + 6 * (j - nb) + c] = (i == j && r == c ? 1.0 : 0.0) - AMG_OMEGA * v;
  }
}

// slot 2 = Q = P N P^T of level l, N (slot 0) of level l + 1
__device__ __forceinline__ void tail_p(const AmgLevel &L, int i, double (&Pm)[36]) {
#pragma unroll
  for (int k = 0; k < 36; ++k) Pm[k] = (k % 7 == 0) ? 1.0 : 0.0;
  if (!L.active[i]) {
#pragma unroll
    for (int k = 0; k < 36; ++k) Pm[k] = 0.0;
    return;
  }
  const double d0 = L.pd[3 * i], d1 = L.pd[3 * i + 1], d2 = L.pd[3 * i + 2];
  // -[d]x in rows 0-2, columns 3-5
  Pm[0 * 6 + 4] = d2;  Pm[0 * 6 + 5] = -d1;
  Pm[1 * 6 + 3] = -d2; Pm[1 * 6 + 5] = d0;
  Pm[2 * 6 + 3] = d1;  Pm[2 * 6 + 4] = -d0;
}
__global__ __launch_bounds__(256) void k_tail_form_q(AmgDev a, int l) {
  const int sc = blockIdx.y;
  const AmgLevel &L = a.lv[l];
  int nb, ne, cb, ce;
  tail_range(a, l, sc, nb, ne);
  tail_range(a, l + 1, sc, cb, ce);
  const int n = ne - nb, N6 = 6 * n, M6 = 6 * (ce - cb);
  const double *Nc = tail_slot(a, sc, 0);
  double *Q = tail_slot(a, sc, 2);
  for (int q = blockIdx.x * 256 + threadIdx.x; q < n * n; q += gridDim.x * 256) {   // one 6x6 block each
    const int i = nb + q / n, j = nb + q % n;
    double Pi[36], Pj[36];
    tail_p(L, i, Pi);
    tail_p(L, j, Pj);
    const int pi = L.parent[i] - cb, pj = L.parent[j] - cb;
    double B[36];   // N_{pi pj} P_j^T
#pragma unroll
    for (int x = 0; x < 6; ++x)
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        double v = 0.0;
#pragma unroll
        for (int y = 0; y < 6; ++y) v += Nc[(size_t)(6 * pi + x) * M6 + 6 * pj + y] * Pj[b * 6 + y];
        B[x * 6 + b] = v;
      }
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        double v = 0.0;
#pragma unroll
        for (int x = 0; x < 6; ++x) v += Pi[r * 6 + x] * B[x * 6 + b];
        Q[(size_t)(6 * (i - nb) + r) * N6 + 6 * (j - nb) + b] = v;
      }
  }
}

// MODE 0: slot 3 = S + Q W (slots 2, 1); MODE 1: slot 0 = S + W^T T (slots
// 1, 3).  32 x 32 output tiles, the k range in 32-wide steps through LDS;
// thread (ty, tx) forms outputs (ty + 16 u, tx + 16 v).
template <typename T, int MODE> __global__ __launch_bounds__(256) void k_tail_gemm(AmgDev a, int l) {
  __shared__ double As[32][33], Bs[32][33];
  const int sc = blockIdx.y;
  const AmgLevel &L = a.lv[l];
  int nb, ne;
  tail_range(a, l, sc, nb, ne);
  const int N6 = 6 * (ne - nb), nt = (N6 + 31) / 32;
  if ((int)blockIdx.x >= nt * nt) return;   // uniform over the workgroup
  const int R0 = 32 * (blockIdx.x / nt), C0 = 32 * (blockIdx.x % nt);
  const double *Am = tail_slot(a, sc, MODE == 0 ? 2 : 1), *Bm = tail_slot(a, sc, MODE == 0 ? 1 : 3);
  double *Cm = tail_slot(a, sc, MODE == 0 ? 3 : 0);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int k0 = 0; k0 < N6; k0 += 32) {
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
      const int r = e >> 5, c = e & 31;
      const int gr = R0 + r, gk = k0 + c;   // As[r][c] = A(gr, gk)
      double av = 0.0;
      if (gr < N6 && gk < N6) av = MODE == 0 ? Am[(size_t)gr * N6 + gk] : Am[(size_t)gk * N6 + gr];
      As[r][c] = av;
      const int bk = k0 + r, bc = C0 + c;   // Bs[r][c] = B(bk, bc)
      Bs[r][c] = (bk < N6 && bc < N6) ? Bm[(size_t)bk * N6 + bc] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < 32; ++k)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] += As[ty + 16 * u][k] * Bs[k][tx + 16 * v];
    __syncthreads();
  }
  const T *dinv = reinterpret_cast<const T *>(L.dinv);
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int r = R0 + ty + 16 * u, c = C0 + tx + 16 * v;
      if (r >= N6 || c >= N6) continue;
      double o = acc[u][v];
      if (r / 6 == c / 6) o += AMG_OMEGA * double(dinv[(size_t)(nb + r / 6) * 36 + (r % 6) * 6 + c % 6]);
      Cm[(size_t)r * N6 + c] = o;
    }
}

// N of the tail level (slot 0) into the cycle's matrix (T)
template <typename T> __global__ __launch_bounds__(256) void k_tail_store(AmgDev a) {
  const int sc = blockIdx.y;
  const int64_t m = a.noff[sc + 1] - a.noff[sc];
  const double *src = tail_slot(a, sc, 0);
  T *o = reinterpret_cast<T *>(a.nmat) + a.noff[sc];
  for (int64_t q = blockIdx.x * 256 + threadIdx.x; q < m; q += (int64_t)gridDim.x * 256) o[q] = T(src[q]);
}

// Per PCG iteration: e = N b on AMG_DENSE_NODES tail nodes of one scene
// (each row by 16 lanes in a fixed butterfly, b staged in LDS), prolonged
// into their members one level down (on level 1 kept for the cycle's last
// kernel).
constexpr int TAIL_THREADS = 6 * AMG_DENSE_NODES * 16;
template <typename T> __global__ __launch_bounds__(TAIL_THREADS) void k_amg_tail(DevPtrs d, AmgDev a) {
  __shared__ double bs[6 * AMG_DENSE_MAX];
  __shared__ double ev[6 * AMG_DENSE_NODES];
  const int sc = blockIdx.y;
  if (!d.ctl[sc].cg_active) return;   // uniform over the workgroup
  int nb, ne;
  tail_range(a, a.Lt, sc, nb, ne);
  const int node0 = nb + AMG_DENSE_NODES * (int)blockIdx.x;
  if (node0 >= ne) return;   // uniform over the workgroup
  const int nn = min(AMG_DENSE_NODES, ne - node0), N6 = 6 * (ne - nb);
  const AmgLevel &L = a.lv[a.Lt];
  for (int q = threadIdx.x; q < N6; q += TAIL_THREADS) bs[q] = L.b[(size_t)6 * nb + q];
  __syncthreads();
  const int r = threadIdx.x >> 4, h = threadIdx.x & 15;   // row of the chunk, its lane
  const int rr = min(r, 6 * nn - 1);
  const T *Nr = reinterpret_cast<const T *>(a.nmat) + a.noff[sc] + (size_t)(6 * (node0 - nb) + rr) * N6;
  double acc = 0.0;
#pragma unroll 4
  for (int k = h; k < N6; k += 16) acc += double(Nr[k]) * bs[k];
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) acc += __shfl_xor(acc, off, 64);
  if (h == 0 && r < 6 * nn) ev[r] = acc;
  __syncthreads();
  if (a.Lt == 1) {
    for (int q = threadIdx.x; q < 6 * nn; q += TAIL_THREADS) L.e[(size_t)6 * node0 + q] = ev[q];
  } else {
    const int *parent = a.lv[a.Lt - 1].parent;
    for (int k = L.mbeg[node0] + (int)threadIdx.x; k < L.mbeg[node0 + nn]; k += TAIL_THREADS) {
      const int i = L.mlist[k];
      const double *ep = ev + (parent[i] - node0) * 6;
      const double e[6] = {ep[0], ep[1], ep[2], ep[3], ep[4], ep[5]};
      prolong_one(a, a.Lt, i, e);
    }
  }
}

// ---------------------------------------------------------------------------
// The fine level's end of the cycle
// ---------------------------------------------------------------------------

// fine coupling (H P)_{i,a} = sum of H_ij P_j over the blocks of row i whose
// column j is an unknown of aggregate a, the diagonal block first, then the
// off-diagonal ones in slot order.  Row r of H_ij P_j, with h = row r of H_ij
// split into (h_t, h_w): columns 0-2 are h_t, columns 3-5 are
// d_j x h_t + S_j^T h_w.  A workgroup takes HP_ROWS fine rows, whose
// entries and sources are contiguous ranges: phase 1 gives each thread a
// source (its whole block and the column's prolongator record, every load
// issued at once) and writes the 36 values of its product to LDS, the rows'
// diagonal products too; phase 2 gives each thread entry values (entry,
// element), summed from LDS in the fixed order.  Sources beyond HP_CAP are
// taken in further passes, their sums added to the entry's values.
constexpr int HP_ROWS = 8, HP_THREADS = 128, HP_CAP = 128;   // ~100 off-diagonal sources per 8 rows
template <typename T>
__device__ __forceinline__ void hp_product(const T (&H)[36], const T (&pr)[12], T *out) {
  const double dd[3] = {double(pr[0]), double(pr[1]), double(pr[2])};
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    const double h0 = double(H[r * 6]), h1 = double(H[r * 6 + 1]), h2 = double(H[r * 6 + 2]);
    const double h3 = double(H[r * 6 + 3]), h4 = double(H[r * 6 + 4]), h5 = double(H[r * 6 + 5]);
    out[r * 6] = T(h0);
    out[r * 6 + 1] = T(h1);
    out[r * 6 + 2] = T(h2);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const double cr = m == 0 ? dd[1] * h2 - dd[2] * h1 : (m == 1 ? dd[2] * h0 - dd[0] * h2 : dd[0] * h1 - dd[1] * h0);
      out[r * 6 + 3 + m] = T(cr + double(pr[3 + m]) * h3 + double(pr[6 + m]) * h4 + double(pr[9 + m]) * h5);
    }
  }
}
template <typename T> __global__ __launch_bounds__(HP_THREADS) void k_amg_hp(DevPtrs d, AmgDev a) {
  constexpr int NQ = 36 * (int)sizeof(T) / 16, NP4 = 12 * (int)sizeof(T) / 16;   // 16-byte pieces
  constexpr int U = (HP_CAP + HP_THREADS - 1) / HP_THREADS;
  __shared__ T prod[HP_CAP * 36];
  __shared__ T dprod[HP_ROWS * 36];
  __shared__ int sh_ptr[HP_ROWS + 1], sh_self[HP_ROWS];
  const int r0 = blockIdx.x * HP_ROWS, t = threadIdx.x;
  if (t <= HP_ROWS) sh_ptr[t] = a.hp_ptr[r0 + t];
  if (t < HP_ROWS) sh_self[t] = a.hp_self[r0 + t];
  const T *hd = reinterpret_cast<const T *>(d.hdiag);
  const float4 *HO = reinterpret_cast<const float4 *>(d.hoff);
  const float4 *PD = reinterpret_cast<const float4 *>(a.pd0);
  // the rows' diagonal products (rows without a self entry skip theirs)
  if (t < HP_ROWS) {
    const int i = r0 + t;
    T H[36], pr[12];
    const T *D = hd + (size_t)i * 21;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) H[r * 6 + c] = D[up6(r, c)];
    float4 *pp = reinterpret_cast<float4 *>(pr);
#pragma unroll
    for (int x = 0; x < NP4; ++x) pp[x] = PD[(size_t)i * NP4 + x];
    hp_product<T>(H, pr, dprod + t * 36);
  }
  __syncthreads();
  const int e0 = sh_ptr[0], e1 = sh_ptr[HP_ROWS];
  if (e0 == e1) return;   // uniform over the workgroup
  const int g0 = a.hp_gptr[e0], g1 = a.hp_gptr[e1];
  T *hv = reinterpret_cast<T *>(a.hp_val);
  const int nitems = 36 * (e1 - e0);
  for (int pb = g0; pb == g0 || pb < g1; pb += HP_CAP) {   // at least once: the diagonal-only entries
    const int ns = max(0, min(HP_CAP, g1 - pb));
    {
      int src[U], j[U];
#pragma unroll
      for (int m = 0; m < U; ++m) {   // threads past the pass repeat its last source
        const int q = pb + min(m * HP_THREADS + t, max(ns - 1, 0));
        src[m] = ns > 0 ? a.hp_src[q] : 0;
        j[m] = ns > 0 ? a.hp_col[q] : r0;
      }
      float4 bq[U][NQ], pq[U][NP4];
#pragma unroll
      for (int m = 0; m < U; ++m) {
        if (ns > 0) {
#pragma unroll
          for (int x = 0; x < NQ; ++x) bq[m][x] = HO[(size_t)(src[m] >> 1) * NQ + x];
        }
#pragma unroll
        for (int x = 0; x < NP4; ++x) pq[m][x] = PD[(size_t)j[m] * NP4 + x];
      }
#pragma unroll
      for (int m = 0; m < U; ++m) {
        const int q = m * HP_THREADS + t;
        if (q >= ns) continue;
        const T *b = reinterpret_cast<const T *>(bq[m]);
        const bool tr = (src[m] & 1) != 0;   // H_ij is the transpose of the stored block
        // the transpose as register swaps at fixed indices: a select between
        // b[c * 6 + r] and b[r * 6 + c] became an indexed private array (scratch) in FP64
        T H[36];
#pragma unroll
        for (int k = 0; k < 36; ++k) H[k] = b[k];
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int c = r + 1; c < 6; ++c) {
            const T x = H[r * 6 + c], y = H[c * 6 + r];
            H[r * 6 + c] = tr ? y : x;
            H[c * 6 + r] = tr ? x : y;
          }
        hp_product<T>(H, reinterpret_cast<const T(&)[12]>(pq[m]), prod + q * 36);
      }
    }
    __syncthreads();
    for (int it = t; it < nitems; it += HP_THREADS) {
      const int k = e0 + it / 36, q = it - (it / 36) * 36;
      int rl = 0;
      while (rl + 1 < HP_ROWS && sh_ptr[rl + 1] <= k) ++rl;
      const int s0 = a.hp_gptr[k], s1 = a.hp_gptr[k + 1];
      const int lo = max(s0, pb), hi = min(s1, pb + ns);
      const bool first = pb == g0 || s0 >= pb;   // no value written for this entry yet
      if (!first && lo >= hi) continue;
      double acc = first ? 0.0 : double(hv[(size_t)k * 36 + q]);
      if (first && sh_self[rl] == k) acc += double(dprod[rl * 36 + q]);
      for (int m = lo; m < hi; ++m) acc += double(prod[(m - pb) * 36 + q]);
      hv[(size_t)k * 36 + q] = T(acc);
    }
    __syncthreads();
    if (pb >= g1 - HP_CAP) break;   // uniform: the last pass
  }
}

// six values of an array the cycle reads once, with non-temporal loads.
// The cycle's last kernel reads all its operands this way: measured on the
// 219K plate, the PCG's product that follows then finds more of the Hessian
// in the Infinity Cache (67.8 against 72.3 us with ordinary loads).
__device__ __forceinline__ void ld6_stream(const float *p, float (&v)[6]) {
  typedef float v2f __attribute__((ext_vector_type(2)));
  const v2f *q = reinterpret_cast<const v2f *>(p);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const v2f x = __builtin_nontemporal_load(q + k);
    v[2 * k] = x.x;
    v[2 * k + 1] = x.y;
  }
}
__device__ __forceinline__ void ld6_stream(const double *p, double (&v)[6]) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  const v2d *q = reinterpret_cast<const v2d *>(p);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const v2d x = __builtin_nontemporal_load(q + k);
    v[2 * k] = x.x;
    v[2 * k + 1] = x.y;
  }
}

// The cycle's result u = t + omega D^-1 (r - H t) for t = t0 + P e_1, with
// H t = H t0 + (H P) e_1 (r0 holds H t0, the cycle's fine product), written
// to the PCG's u, and the (r, u) and (r, r) partials of each SPMV_ROWS-row
// block for the scalars step.  The block's coupling entries are one
// contiguous range: phase 1 gives each lane a row of an entry (six
// consecutive values, so that a wavefront reads one contiguous stretch) and
// e_1 of the entry's aggregate, FINAL_U rows in flight, and writes the
// product to LDS; phase 2 is thread (row, component), which adds its row's
// products in entry order after H t0.
constexpr int FINAL_U = 3;
constexpr int FINAL_CAP = FINAL_U * SPMV_ROWS;   // entries per pass: FINAL_U per row on average
template <typename T> __global__ __launch_bounds__(6 * SPMV_ROWS) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 4))) void k_amg_final(DevPtrs d, AmgDev a) {
  constexpr int NT = 6 * SPMV_ROWS;
  static_assert(6 * FINAL_CAP == NT * FINAL_U, "one round of every lane's rows per pass");
  // the block's Jacobi inverses and prolongator records: contiguous 16-byte
  // pieces loaded (non-temporally) with the row operands, held over the
  // entries' pass and read back through LDS by the row threads
  constexpr int NSD = SPMV_ROWS * 21 * (int)sizeof(T) / 16, NSP = SPMV_ROWS * 12 * (int)sizeof(T) / 16;
  constexpr int NSTG = (NSD + NSP + NT - 1) / NT;
  static_assert(SPMV_ROWS * 21 * sizeof(T) % 16 == 0 && SPMV_ROWS * 12 * sizeof(T) % 16 == 0, "16-byte pieces");
  __shared__ double prod[FINAL_CAP * 6];
  __shared__ double ys[NT];
  __shared__ nt_v4f stg[NSD + NSP];
  const int lb = blockIdx.x, r0 = lb * SPMV_ROWS;
  if (!d.ctl[row_scene(d, r0)].cg_active) return;   // uniform over the workgroup
  const int t = threadIdx.x, rl = t / 6, c = t - (t / 6) * 6, row = r0 + rl;
  const size_t o = (size_t)row * 6 + c;
  const double *e1 = a.lv[1].e;
  // the row thread's own operands (non-temporal): its r, t0 and H t0; its
  // aggregate (component c of P_row e_p is added when the row is an unknown
  // of one), and the staged pieces
  const double rc = __builtin_nontemporal_load(d.cr + o);
  double tc = __builtin_nontemporal_load(a.t0 + o), hc = __builtin_nontemporal_load(a.r0 + o);
  const int kr0 = a.hp_ptr[row], kr1 = a.hp_ptr[row + 1];
  const int eb = a.hp_ptr[r0], ee = a.hp_ptr[r0 + SPMV_ROWS];
  const int p = a.parent0[row];
  const bool use = p >= 0 && d.flags[row] == 0;
  nt_v4f sv[NSTG];
  {
    const nt_v4f *gd = reinterpret_cast<const nt_v4f *>(reinterpret_cast<const T *>(d.dinv) + (size_t)r0 * 21);
    const nt_v4f *gp = reinterpret_cast<const nt_v4f *>(reinterpret_cast<const T *>(a.pd0) + (size_t)r0 * 12);
#pragma unroll
    for (int m = 0; m < NSTG; ++m) {
      const int q = m * NT + t;
      if (q < NSD) sv[m] = __builtin_nontemporal_load(gd + q);
      else if (q < NSD + NSP) sv[m] = __builtin_nontemporal_load(gp + (q - NSD));
    }
  }
  double ep[6];
  ld6(e1 + (size_t)max(p, 0) * 6, ep);
  const T *hv = reinterpret_cast<const T *>(a.hp_val);
  for (int cb = eb; cb < ee; cb += FINAL_CAP) {
    const int nw = 6 * min(FINAL_CAP, ee - cb);   // (entry, row) items of the pass
    T h[FINAL_U][6];
    double ev[FINAL_U][6];
#pragma unroll
    for (int m = 0; m < FINAL_U; ++m) {   // lanes past the pass repeat its last item
      const int q = min(m * NT + t, nw - 1);
      const int k = cb + q / 6;
      ld6_stream(hv + (size_t)k * 36 + (q - (q / 6) * 6) * 6, h[m]);
      const double *e = e1 + (size_t)a.hp_agg[k] * 6;
#pragma unroll
      for (int x = 0; x < 6; ++x) ev[m][x] = e[x];
    }
#pragma unroll
    for (int m = 0; m < FINAL_U; ++m) {
      double y = 0.0;
#pragma unroll
      for (int x = 0; x < 6; ++x) y += double(h[m][x]) * ev[m][x];
      if (m * NT + t < nw) prod[m * NT + t] = y;
    }
    __syncthreads();
    const int lo = max(kr0, cb), hi = min(kr1, cb + nw / 6);
    for (int k = lo; k < hi; ++k) hc += prod[(k - cb) * 6 + c];
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < NSTG; ++m)
    if (m * NT + t < NSD + NSP) stg[m * NT + t] = sv[m];
  ys[t] = rc - hc;
  __syncthreads();
  const T *Di = reinterpret_cast<const T *>(stg) + rl * 21;
  const T *pp = reinterpret_cast<const T *>(stg + NSD) + rl * 12;
  {   // component c of P_row e_p
    double dd[3], S[9], y[6];
#pragma unroll
    for (int m = 0; m < 3; ++m) dd[m] = double(pp[m]);
#pragma unroll
    for (int m = 0; m < 9; ++m) S[m] = double(pp[3 + m]);
    p_apply(dd, S, ep, y);
    double pe = y[0];
#pragma unroll
    for (int k = 1; k < 6; ++k) pe = (c == k) ? y[k] : pe;
    tc += use ? pe : 0.0;
  }
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) v += double(Di[up6(c, k)]) * ys[rl * 6 + k];
  const double un = tc + AMG_OMEGA * v;
  d.cs[o] = un;
  KSum ru = {0.0, 0.0}, none = {0.0, 0.0}, rr = {0.0, 0.0};
  kadd(ru, rc * un);
  kadd(rr, rc * rc);
  block_ksum3(ru, none, rr);
  if (t == 0) {
    d.part_a[lb] = make_double2(ru.s, ru.c);
    d.part_c[lb] = make_double2(rr.s, rr.c);
  }
}

// ---------------------------------------------------------------------------

static inline int nblk(int n, int b) { return (n + b - 1) / b; }

template <typename T>
static void setup_t(const DevPtrs &d, const AmgDev &a, const AmgLevel *hl, int n_scenes, hipStream_t s) {
  k_amg_geom1<T><<<nblk(hl[1].n * 64, 256), 256, 0, s>>>(d, a);
  for (int l = 2; l <= a.L; ++l) k_amg_geom<<<nblk(hl[l].n, 256), 256, 0, s>>>(a, l);
  if (hl[1].nslots > 0) k_amg_galerkin1<T><<<hl[1].nslots, 64, 0, s>>>(d, a);
  k_amg_dinv<T><<<nblk(hl[1].n, 128), 128, 0, s>>>(a, 1);
  for (int l = 2; l <= a.L; ++l) {
    k_amg_galerkin<T><<<nblk(hl[l].nslots, 128), 128, 0, s>>>(a, l);
    k_amg_dinv<T><<<nblk(hl[l].n, 128), 128, 0, s>>>(a, l);
  }
  k_amg_coarse_inverse<T><<<n_scenes, 1024, 0, s>>>(a);
  // the tail matrices, from the coarsest level up to Lt
  auto grid = [&](int64_t work) { return dim3((unsigned)std::min<int64_t>(std::max<int64_t>((work + 255) / 256, 1), 256), n_scenes); };
  const int64_t mL = 6 * (int64_t)a.tmax[a.L];
  k_tail_init<<<grid(mL * mL), 256, 0, s>>>(a);
  for (int l = a.L - 1; l >= a.Lt; --l) {
    const int64_t n6 = 6 * (int64_t)a.tmax[l], nt = (n6 + 31) / 32;
    k_tail_zero_w<<<grid(n6 * n6), 256, 0, s>>>(a, l);
    k_tail_fill_w<T><<<grid(n6 * n6), 256, 0, s>>>(a, l);
    k_tail_form_q<<<grid(n6 * n6 / 36), 256, 0, s>>>(a, l);
    k_tail_gemm<T, 0><<<dim3((unsigned)(nt * nt), n_scenes), 256, 0, s>>>(a, l);
    k_tail_gemm<T, 1><<<dim3((unsigned)(nt * nt), n_scenes), 256, 0, s>>>(a, l);
  }
  const int64_t mt = 6 * (int64_t)a.tmax[a.Lt];
  k_tail_store<T><<<grid(mt * mt), 256, 0, s>>>(a);
}

template <typename T>
static void vcycle_t(const DevPtrs &d, const AmgDev &a, const AmgLevel *hl, int n_scenes, bool mixed,
                     int spmv_variant, bool t0_ready, bool rev, hipStream_t s, SpmvMark mark) {
  // the fine product H t0 runs through the PCG's own SpMV kernel, without
  // its dots, into r0
  DevPtrs dt = d;
  dt.cs = a.t0;
  dt.cAp = a.r0;
  if (!t0_ready) k_amg_fine_pre<T><<<d.n_pad / TILE, TILE, 0, s>>>(d, a);
  if (mark.fn) mark.fn(mark.arg, true);
  launch_spmv(dt, mixed, spmv_variant, s, SPMV_DOTS_NONE, rev);
  if (mark.fn) mark.fn(mark.arg, false);
  // each restriction also pre-smooths the level it fills, above the tail
  k_amg_restrict1<T><<<nblk(hl[1].n, 4), 256, 0, s>>>(d, a, a.Lt > 1 ? 1 : 0);
  for (int l = 1; l < a.Lt; ++l)
    k_amg_resid_restrict<T><<<nblk(hl[l + 1].n, 256 / RR_THREADS), 256, 0, s>>>(a, l, l + 1 < a.Lt ? 1 : 0);
  // the tail: e = N b on level Lt, prolonged into level Lt - 1 (or kept as e_1)
  k_amg_tail<T><<<dim3(nblk(a.tmax[a.Lt], AMG_DENSE_NODES), n_scenes), TAIL_THREADS, 0, s>>>(d, a);
  // each level's kernel also prolongs its correction one level down (level
  // 1 keeps e_1)
  for (int l = a.Lt - 1; l >= 1; --l) k_amg_post<T><<<nblk(hl[l].n, 4), 256, 0, s>>>(a, l);
  // t = t0 + P e_1 and the post-smoothing u = t + omega D^-1 (r - H t),
  // H t from H t0 and the fine coupling, with the PCG's r dots
  k_amg_final<T><<<d.n_pad / SPMV_ROWS, 6 * SPMV_ROWS, 0, s>>>(d, a);
}

void launch_amg_couple(const DevPtrs &d, const AmgDev &a, bool mixed, hipStream_t s) {
  if (a.nhp == 0) return;
  static_assert(TILE % HP_ROWS == 0, "coupling row blocks nest in the tiles");
  if (mixed) k_amg_hp<float><<<d.n_pad / HP_ROWS, HP_THREADS, 0, s>>>(d, a);
  else k_amg_hp<double><<<d.n_pad / HP_ROWS, HP_THREADS, 0, s>>>(d, a);
}

void launch_amg_setup(const DevPtrs &d, const AmgDev &a, const AmgLevel *hl, int n_scenes, bool mixed,
                      hipStream_t s) {
  if (mixed) setup_t<float>(d, a, hl, n_scenes, s);
  else setup_t<double>(d, a, hl, n_scenes, s);
}
void launch_amg_vcycle(const DevPtrs &d, const AmgDev &a, const AmgLevel *hl, int n_scenes, bool mixed,
                       int spmv_variant, bool t0_ready, bool rev, hipStream_t s, SpmvMark mark) {
  if (mixed) vcycle_t<float>(d, a, hl, n_scenes, true, spmv_variant, t0_ready, rev, s, mark);
  else vcycle_t<double>(d, a, hl, n_scenes, false, spmv_variant, t0_ready, rev, s, mark);
}

}  // namespace bdem
