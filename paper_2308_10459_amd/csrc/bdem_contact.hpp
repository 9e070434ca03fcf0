// Device helpers shared by the element-repulsion kernels (Section 5.4).
#pragma once
#include "bdem_internal.hpp"

namespace bdem {

// Position at which V is evaluated for particle j of the state X (iterate or
// line-search trial): X itself, or the midpoint (X + x_n)/2.
__device__ __forceinline__ double4 contact_point(const DevPtrs &d, const double4 *X, int j,
                                                 int midpoint) {
  const double4 x = X[j];
  if (!midpoint) return x;
  const double4 n = d.pn[j];
  return make_double4(0.5 * (x.x + n.x), 0.5 * (x.y + n.y), 0.5 * (x.z + n.z), 0.0);
}

// Overlap of the spheres (r, j) at the centres pr, pj: false unless
// 0 < l < rr + rj; then n is the unit vector from r to j and e = l - rr - rj.
__device__ __forceinline__ bool contact_overlap(double4 pr, double4 pj, double rr, double rj,
                                                double (&n)[3], double &e) {
  const double ux = pj.x - pr.x, uy = pj.y - pr.y, uz = pj.z - pr.z;
  const double l = sqrt(ux * ux + uy * uy + uz * uz), dd = rr + rj;
  if (!(l < dd) || !(l > 0.0)) return false;
  n[0] = ux / l; n[1] = uy / l; n[2] = uz / l;
  e = l - dd;
  return true;
}

}  // namespace bdem
