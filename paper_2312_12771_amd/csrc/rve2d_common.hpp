// Device helpers shared by the 2D RVE kernels: Q4 neighbourhood
// bookkeeping, the padded periodic LDS layout and work-group sums.
#pragma once

#include "elem2d.hpp"
#include "fe2_internal.hpp"

namespace fe2 {
namespace rve2d {

// Element q (0..3) around an owned node (di, dj): position of the element's
// lower-left node in the 3x3 element neighbourhood and the local corner the
// node occupies in it.
__host__ __device__ constexpr int elem_ea(int di, int q) { return di + ((q == 1 || q == 2) ? 1 : 0); }
__host__ __device__ constexpr int elem_ec(int dj, int q) { return dj + (q >= 2 ? 1 : 0); }
__host__ __device__ constexpr int elem_cc(int q) { return (q + 2) & 3; }

// Padded (halo) layout of a periodic N1 x N2 nodal or element field:
// entry (i, j), i in [-1, N1], j in [-1, N2], at (j+1)*PW + (i+1).  Odd
// sizes get one more unused column/row so that the 4x4 window of the last,
// partial 2x2 block stays inside the array.
__host__ __device__ constexpr int pad_w(int n) { return n + 2 + (n & 1); }
template <int N1, int N2>
struct Pad {
  static constexpr int PW = pad_w(N1);
  static constexpr int PN = pad_w(N1) * pad_w(N2);
  static __host__ __device__ constexpr int at(int i, int j) { return (j + 1) * PW + (i + 1); }
};

// Write value v of real node/element (i, j) and its halo images.
template <int N1, int N2, typename V>
__device__ __forceinline__ void put_halo(V* f, int i, int j, V v) {
  using P = Pad<N1, N2>;
  f[P::at(i, j)] = v;
  const int ig = (i == 0) ? N1 : ((i == N1 - 1) ? -1 : -2);
  const int jg = (j == 0) ? N2 : ((j == N2 - 1) ? -1 : -2);
  if (ig != -2) f[P::at(ig, j)] = v;
  if (jg != -2) f[P::at(i, jg)] = v;
  if (ig != -2 && jg != -2) f[P::at(ig, jg)] = v;
}

// Work-group sum with two alternating reduction buffers (one barrier each).
template <int NV, int NW>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double* s_red, int& parity) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  double* buf = s_red + parity * (NW * NV);
  parity ^= 1;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) buf[wid * NV + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += buf[w * NV + i];
    v[i] = t;
  }
}

}  // namespace rve2d
}  // namespace fe2
