// Device-side math for the bonded-DEM kernels (gfx950, wave64).
//
// Quaternions are (x, y, z, w) with the scalar last, stored in double4.
#pragma once
#include <hip/hip_runtime.h>

namespace bdem {

// ---------------------------------------------------------------------------
// small vector helpers
// ---------------------------------------------------------------------------
template <typename T> struct V3 { T x, y, z; };

template <typename T> __device__ __forceinline__ T dot3(const T *a, const T *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
template <typename T> __device__ __forceinline__ T dot4(const T *a, const T *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}
template <typename T> __device__ __forceinline__ void cross3(const T *a, const T *b, T *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Hamilton product c = a * b, scalar last.
template <typename T> __device__ __forceinline__ void qmul(const T *a, const T *b, T *c) {
  c[0] = a[3] * b[0] + b[3] * a[0] + a[1] * b[2] - a[2] * b[1];
  c[1] = a[3] * b[1] + b[3] * a[1] + a[2] * b[0] - a[0] * b[2];
  c[2] = a[3] * b[2] + b[3] * a[2] + a[0] * b[1] - a[1] * b[0];
  c[3] = a[3] * b[3] - a[0] * b[0] - a[1] * b[1] - a[2] * b[2];
}

// componentwise midpoint (a + b)/2
__device__ __forceinline__ double4 mid4(double4 a, double4 b) {
  return make_double4(0.5 * (a.x + b.x), 0.5 * (a.y + b.y), 0.5 * (a.z + b.z), 0.5 * (a.w + b.w));
}

// G_l(q) = [s I - v^x, -v] as a 3x4 row-major matrix.
template <typename T> __device__ __forceinline__ void gleft(const T *q, T *G) {
  const T x = q[0], y = q[1], z = q[2], s = q[3];
  G[0] = s;  G[1] = z;  G[2] = -y; G[3] = -x;
  G[4] = -z; G[5] = s;  G[6] = x;  G[7] = -y;
  G[8] = y;  G[9] = -x; G[10] = s; G[11] = -z;
}

// C (3x3) = G_a M G_b^T with G_* 3x4 and M 4x4 (all row-major).
template <typename T>
__device__ __forceinline__ void gmgt(const T *Ga, const T *M, const T *Gb, T *C) {
  T GM[12];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      T acc = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) acc += Ga[r * 4 + k] * M[k * 4 + c];
      GM[r * 4 + c] = acc;
    }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T acc = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) acc += GM[r * 4 + k] * Gb[c * 4 + k];
      C[r * 3 + c] = acc;
    }
}

// ---------------------------------------------------------------------------
// theta^2 = F(y), y = |n - d|^2 = (2 sin(theta/2))^2 and derivatives.
// Series 2 y^n / (n^2 C(2n,n)) for small y, closed form otherwise.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void theta2_fn(double y, double &F, double &F1, double &F2) {
  if (y < 0.05) {
    // coefficients c_n = 2 / (n^2 C(2n, n)), n = 1..12
    const double c[12] = {1.0,
                          1.0 / 12.0,
                          1.0 / 90.0,
                          1.0 / 560.0,
                          1.0 / 3150.0,
                          1.0 / 16632.0,
                          1.0 / 84084.0,
                          1.0 / 411840.0,
                          1.0 / 1969110.0,
                          1.0 / 9237800.0,
                          1.0 / 42678636.0,
                          1.0 / 194699232.0};
    double f = 0.0, f1 = 0.0, f2 = 0.0;
#pragma unroll
    for (int k = 11; k >= 0; --k) {  // Horner in y
      const double n = k + 1;
      f = f * y + c[k];
      f1 = f1 * y + n * c[k];
      if (k >= 1) f2 = f2 * y + n * (n - 1.0) * c[k];
    }
    F = f * y;
    F1 = f1;
    F2 = f2;
  } else {
    const double th = 2.0 * asin(0.5 * sqrt(y));
    const double q = y * (4.0 - y);
    F = th * th;
    F1 = 2.0 * th / sqrt(q);
    F2 = (2.0 - F1 * (2.0 - y)) / q;
  }
}

// ---------------------------------------------------------------------------
// compensated (TwoSum / Neumaier) accumulation, deterministic reductions
// ---------------------------------------------------------------------------
struct KSum {
  double s, c;
};
__device__ __forceinline__ void kadd(KSum &k, double x) {
  const double t = k.s + x;
  const double bp = t - k.s;
  k.c += (k.s - (t - bp)) + (x - bp);  // TwoSum error
  k.s = t;
}
__device__ __forceinline__ KSum kmerge(KSum a, KSum b) {
  KSum r;
  r.s = a.s + b.s;
  const double bp = r.s - a.s;
  r.c = a.c + b.c + ((a.s - (r.s - bp)) + (b.s - bp));
  return r;
}
__device__ __forceinline__ KSum wave_ksum(KSum v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    KSum o;
    o.s = __shfl_xor(v.s, off, 64);
    o.c = __shfl_xor(v.c, off, 64);
    // fixed combination order: lower lane first, identical on both partners
    const bool lower = (threadIdx.x & off) == 0;
    v = lower ? kmerge(v, o) : kmerge(o, v);
  }
  return v;
}
// Block-wide compensated sum; every thread gets the result.  blockDim.x must
// be a multiple of 64 and <= 1024.
__device__ __forceinline__ KSum block_ksum(KSum v) {
  __shared__ double ls[16], lc[16];
  v = wave_ksum(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) { ls[w] = v.s; lc[w] = v.c; }
  __syncthreads();
  KSum r = {0.0, 0.0};
  for (int k = 0; k < nw; ++k) r = kmerge(r, KSum{ls[k], lc[k]});
  __syncthreads();
  return r;
}
// three block-wide compensated sums in one LDS round (same combination
// order as three block_ksum calls); every thread gets the results
__device__ __forceinline__ void block_ksum3(KSum &a, KSum &b, KSum &c) {
  __shared__ double l3[6][16];
  a = wave_ksum(a);
  b = wave_ksum(b);
  c = wave_ksum(c);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    l3[0][w] = a.s; l3[1][w] = a.c; l3[2][w] = b.s; l3[3][w] = b.c; l3[4][w] = c.s; l3[5][w] = c.c;
  }
  __syncthreads();
  KSum ra = {0.0, 0.0}, rb = {0.0, 0.0}, rc = {0.0, 0.0};
  for (int k = 0; k < nw; ++k) {
    ra = kmerge(ra, KSum{l3[0][k], l3[1][k]});
    rb = kmerge(rb, KSum{l3[2][k], l3[3][k]});
    rc = kmerge(rc, KSum{l3[4][k], l3[5][k]});
  }
  __syncthreads();
  a = ra; b = rb; c = rc;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double block_max(double v) {
  __shared__ double lm[16];
  v = wave_max(v);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) lm[w] = v;
  __syncthreads();
  double r = lm[0];
  for (int k = 1; k < nw; ++k) r = fmax(r, lm[k]);
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// XCD-aware block order: consecutive logical blocks land on the same XCD so
// neighbouring rows / bonds share that XCD's L2.  Hardware dispatches
// workgroup b to XCD b % 8.  Bijective for any grid size.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_block(int b, int nblk) {
  const int q = nblk >> 3, rem = nblk & 7;
  const int xcd = b & 7, k = b >> 3;
  return (xcd < rem) ? xcd * (q + 1) + k : rem * (q + 1) + (xcd - rem) * q + k;
}
// the same ranges per XCD, each walked from its end
__device__ __forceinline__ int xcd_block_rev(int b, int nblk) {
  const int q = nblk >> 3, rem = nblk & 7;
  const int xcd = b & 7, k = b >> 3;
  return (xcd < rem) ? xcd * (q + 1) + (q - k) : rem * (q + 1) + (xcd - rem) * q + (q - 1 - k);
}

// ---------------------------------------------------------------------------
// Symmetric 9x9 eigen-clamp by cyclic Jacobi, register resident.
// A holds the upper triangle (45 entries, row-major upper packing); on
// return A holds the projection onto the PSD cone (negative eigenvalues
// set to zero).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int up9(int r, int c) {
  return r <= c ? r * 9 - (r * (r - 1)) / 2 + (c - r) : c * 9 - (c * (c - 1)) / 2 + (r - c);
}

template <typename T> struct JacobiTol;
template <> struct JacobiTol<float> {
  static constexpr float rel = 1e-14f;  // squared relative off-diagonal threshold
  static constexpr int max_sweeps = 10;
};
template <> struct JacobiTol<double> {
  static constexpr double rel = 1e-30;
  static constexpr int max_sweeps = 16;
};

// Rotation angle of one Jacobi step: any (c, s) with c^2 + s^2 = 1 to
// rounding is an exact orthogonal similarity, so the FP32 path takes the
// hardware reciprocal and reciprocal square root (1 ulp) instead of the
// correctly rounded divide and square root; FP64 keeps IEEE operations.
template <typename T> struct JacobiAngle;
template <> struct JacobiAngle<float> {
  __device__ static __forceinline__ void cs(float app, float aqq, float apq, float &t, float &c) {
    // rotate only where the hardware reciprocal of 2 apq is finite: for a
    // denormal apq it overflows, and with aqq == app (symmetric, unstrained
    // bonds) theta would be 0 * inf; such an off-diagonal is left in place
    const bool act = fabsf(apq) >= 1e-30f;
    const float theta = (aqq - app) * __builtin_amdgcn_rcpf(act ? 2.0f * apq : 1.0f);
    const float at = fabsf(theta);
    const float x = fmaf(theta, theta, 1.0f);
    // 1 / (|theta| + sqrt(theta^2 + 1)); about 1 / (2 |theta|) once theta^2 overflows
    const float t0 = at < 1e18f ? __builtin_amdgcn_rcpf(at + x * __builtin_amdgcn_rsqf(x))
                                : 0.5f * __builtin_amdgcn_rcpf(at);
    t = act ? (theta >= 0.0f ? t0 : -t0) : 0.0f;
    c = __builtin_amdgcn_rsqf(fmaf(t, t, 1.0f));
  }
};
template <> struct JacobiAngle<double> {
  __device__ static __forceinline__ void cs(double app, double aqq, double apq, double &t, double &c) {
    const bool act = apq != 0.0;
    const double den = act ? 2.0 * apq : 1.0;
    const double theta = (aqq - app) / den;
    const double at = fabs(theta);
    const double t0 = 1.0 / (at + sqrt(theta * theta + 1.0));
    t = act ? (theta >= 0.0 ? t0 : -t0) : 0.0;
    c = 1.0 / sqrt(t * t + 1.0);
  }
};

template <typename T>
__device__ __forceinline__ void jacobi_rot(T (&A)[45], T (&V)[81], const int p, const int q) {
  const T apq = A[up9(p, q)];
  const T app = A[up9(p, p)], aqq = A[up9(q, q)];
  T t, c;
  JacobiAngle<T>::cs(app, aqq, apq, t, c);
  const T s = t * c;
  A[up9(p, p)] = app - t * apq;
  A[up9(q, q)] = aqq + t * apq;
  A[up9(p, q)] = T(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k == p || k == q) continue;
    const T akp = A[up9(k, p)], akq = A[up9(k, q)];
    A[up9(k, p)] = c * akp - s * akq;
    A[up9(k, q)] = s * akp + c * akq;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const T vkp = V[k * 9 + p], vkq = V[k * 9 + q];
    V[k * 9 + p] = c * vkp - s * vkq;
    V[k * 9 + q] = s * vkp + c * vkq;
  }
}

template <typename T> __device__ __forceinline__ void psd_clamp9(T (&A)[45]) {
  T V[81];
#pragma unroll
  for (int k = 0; k < 81; ++k) V[k] = (k % 10 == 0) ? T(1) : T(0);
  for (int sweep = 0; sweep < JacobiTol<T>::max_sweeps; ++sweep) {
    T off = 0, dia = 0;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      dia += A[up9(r, r)] * A[up9(r, r)];
#pragma unroll
      for (int c = r + 1; c < 9; ++c) off += A[up9(r, c)] * A[up9(r, c)];
    }
    if (off <= JacobiTol<T>::rel * dia) break;
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
      for (int q = p + 1; q < 9; ++q) jacobi_rot<T>(A, V, p, q);
  }
  T lam[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) lam[k] = A[up9(k, k)] > T(0) ? A[up9(k, k)] : T(0);
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int c = r; c < 9; ++c) {
      T acc = 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) acc += V[r * 9 + k] * lam[k] * V[c * 9 + k];
      A[up9(r, c)] = acc;
    }
}

// index of (r, c) in the packed upper triangle of a symmetric 6x6
__host__ __device__ constexpr int up6(int r, int c) {
  return r <= c ? r * 6 - (r * (r - 1)) / 2 + (c - r) : c * 6 - (c * (c - 1)) / 2 + (r - c);
}

}  // namespace bdem
