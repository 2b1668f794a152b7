// Device helpers shared by the 2D RVE kernels: Q4 neighbourhood
// bookkeeping, the padded periodic LDS layout and work-group sums.
#pragma once

#include "elem2d.hpp"
#include "fe2_internal.hpp"

namespace fe2 {

// LDS writes of this wave visible to its other lanes (no work-group barrier)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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
// Each buffer holds NW * MAXNV doubles at a fixed offset, so a reduction of
// any width never overlaps the buffer that the previous one is still being
// read from (s_red: 2 * NW * MAXNV doubles).
template <int NV, int NW, int MAXNV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double* s_red, int& parity) {
  static_assert(NV <= MAXNV, "reduction wider than its buffer");
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  double* buf = s_red + parity * (NW * MAXNV);
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

// Wave sum with DPP cross-lane moves (no LDS traffic): quad butterflies,
// half-row and row mirrors give every lane its 16-lane row sum; the two row
// broadcasts accumulate the rows upwards, so lane 63 holds the wave total.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf,
                                                               false));
}
__device__ __forceinline__ float wave_sum_to_last(float v) {
  v += dpp_f<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_f<0x4E>(v);         // quad_perm [2,3,0,1]
  v += dpp_f<0x141>(v);        // row_half_mirror
  v += dpp_f<0x140>(v);        // row_mirror
  v += dpp_f<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_f<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// Work-group sum of FP32 per-lane partials: wave totals by DPP, the
// cross-wave sum in FP32 (the totals feed FP32 scalar recurrences).  Buffers
// as wg_sum.
template <int NV, int NW, int MAXNV>
__device__ __forceinline__ void wg_sum_f32(const float (&v)[NV], float (&out)[NV], double* s_red, int& parity) {
  static_assert(NV <= MAXNV, "reduction wider than its buffer");
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  float* buf = reinterpret_cast<float*>(s_red + parity * (NW * MAXNV));
  parity ^= 1;
  float w[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) w[i] = wave_sum_to_last(v[i]);
  if (lane == 63) {
#pragma unroll
    for (int i = 0; i < NV; ++i) buf[wid * NV + i] = w[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < NW; ++k) t += buf[k * NV + i];
    out[i] = t;
  }
}

}  // namespace rve2d
}  // namespace fe2
