// Trilinear box element (hex8) bookkeeping shared by the 3D RVE kernel and
// the setup kernel that builds its reference tables.
#pragma once

#include "elem2d.hpp"

namespace fe2 {

// coordinate bit of local corner m along axis f (corners ordered as the
// bottom face counter-clockwise, then the top face)
__host__ __device__ constexpr int hbit(int m, int f) {
  return f == 0 ? cxo(m & 3) : (f == 1 ? cyo(m & 3) : (m >> 2));
}
__host__ __device__ constexpr int hsg(int m, int f) { return 2 * hbit(m, f) - 1; }
__host__ __device__ constexpr int hcorner(int bx, int by, int bz) { return (by ? (bx ? 2 : 3) : (bx ? 1 : 0)) + 4 * bz; }

// Distinct entries of the hex8 box-element stiffness of an isotropic phase
// (cube of side h, lambda/mu = rho, mu = 1).  Entry K[3a+d][3b+e] equals
// kref3_sign * kv[kref3_id].  With 1D integrals of the linear shape
// functions, equal-component entries (d = e) are sums of products of
// stiffness and mass factors that depend only on whether a and b differ
// along axis d and on how many of the other two axes they differ along
// (ids 0..5); mixed entries (d != e) are
//   h/4 * m_g * (lambda s_a,d s_b,e + mu s_a,e s_b,d),
// with corner signs s and the mass factor m_g of the third axis g, i.e.
// +-(lambda + mu) or +-(lambda - mu) times one of two mass factors (ids 6..9).
__host__ __device__ constexpr int kref3_id(int r, int c) {
  return (r % 3 == c % 3)
             ? ((hbit(r / 3, r % 3) == hbit(c / 3, r % 3)) ? 0 : 3) +
                   (hbit(r / 3, (r % 3 + 1) % 3) != hbit(c / 3, (r % 3 + 1) % 3)) +
                   (hbit(r / 3, (r % 3 + 2) % 3) != hbit(c / 3, (r % 3 + 2) % 3))
             : 6 +
                   ((hsg(r / 3, r % 3) * hsg(c / 3, c % 3) == hsg(r / 3, c % 3) * hsg(c / 3, r % 3)) ? 0 : 2) +
                   ((hbit(r / 3, 3 - r % 3 - c % 3) == hbit(c / 3, 3 - r % 3 - c % 3)) ? 0 : 1);
}
__host__ __device__ constexpr int kref3_sign(int r, int c) {
  return (r % 3 == c % 3) ? 1 : hsg(r / 3, r % 3) * hsg(c / 3, c % 3);
}

}  // namespace fe2
