// Bilinear box element (Q4) bookkeeping shared by the 2D RVE kernels and the
// setup kernel that builds the reference tables.
#pragma once

namespace fe2 {

// local corner m of a Q4 element, counter-clockwise from the lower-left node
__host__ __device__ constexpr int cxo(int m) { return (m == 1 || m == 2) ? 1 : 0; }
__host__ __device__ constexpr int cyo(int m) { return m >= 2 ? 1 : 0; }
__host__ __device__ constexpr int sgn_x(int m) { return 2 * cxo(m) - 1; }
__host__ __device__ constexpr int sgn_y(int m) { return 2 * cyo(m) - 1; }

// Distinct entries of the bilinear box-element stiffness for an isotropic
// phase (lambda/mu = rho, mu = 1).  Entry K[2a+d][2b+e] (nodes a, b;
// components d, e) equals kref_sign * kv[kref_id].  Equal-component entries
// depend only on how nodes a and b are placed (same, across x, across y,
// diagonal); mixed-component entries are (rho s_a s_b' + s_a' s_b)/4 with
// corner signs s = +-1, i.e. +-(rho+1)/4 or +-(rho-1)/4.
__host__ __device__ constexpr int kref_rel(int a, int b) {
  return (a == b) ? 0 : (cyo(a) == cyo(b) ? 1 : (cxo(a) == cxo(b) ? 2 : 3));
}
__host__ __device__ constexpr int kref_id(int r, int c) {
  return ((r & 1) == (c & 1))
             ? 4 * (r & 1) + kref_rel(r >> 1, c >> 1)
             : (((r & 1) == 0 ? sgn_x(r >> 1) * sgn_y(c >> 1) : sgn_y(r >> 1) * sgn_x(c >> 1)) ==
                        ((r & 1) == 0 ? sgn_y(r >> 1) * sgn_x(c >> 1) : sgn_x(r >> 1) * sgn_y(c >> 1))
                    ? 8
                    : 9);
}
__host__ __device__ constexpr int kref_sign(int r, int c) {
  return ((r & 1) == (c & 1)) ? 1
                              : ((r & 1) == 0 ? sgn_x(r >> 1) * sgn_y(c >> 1) : sgn_y(r >> 1) * sgn_x(c >> 1));
}

}  // namespace fe2
