// Dense direct solve of small RVEs (2D small strain): the reduced stiffness
// K_ww (Eq. (42)'s RVE block after the periodic reduction and the corner
// pin) assembled densely in LDS in FP32, factored K = L L^T by a blocked
// right-looking Cholesky whose panel and trailing tile products run on the
// FP32 matrix cores (v_mfma_f32_16x16x4f32), and applied by blocked forward
// and backward substitution with the inverted 16 x 16 diagonal tiles.  The
// caller refines in FP64 around it (the factor's error, about
// cond(K_ww) * 2^-24, sets the refinement's contraction per sweep).
//
// Storage: row-major [MD][MD + 4] floats (MD = the unknowns rounded up to
// 16, identity on the padding); the row pitch MD + 4 spreads the sixteen
// rows a matrix-core operand reads over the LDS banks.  After the
// factorization the tiles below the diagonal hold L and each diagonal tile
// holds the inverse of its L tile (lower triangular, zeros above).
#pragma once

#include "rve2d_common.hpp"

namespace fe2 {
namespace dense2d {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int dense_md(int n1, int n2) { return ((2 * n1 * n2 - 2 + 15) / 16) * 16; }
constexpr int dense_pitch(int md) { return md + 4; }
// LDS floats: matrix, one vector, reduction scratch [16][16]
constexpr size_t dense_floats(int md) { return static_cast<size_t>(md) * dense_pitch(md) + md + 256; }

// Unknown index of node n = j n1 + i, component d (node 0 is pinned: -1).
__device__ __forceinline__ int dof_of(int n, int d) { return n == 0 ? -1 : 2 * n + d - 2; }

// Dense K_ww: node n's rows gather the element stiffnesses mu_e K_ref of
// the (up to four) elements it shares with each of its nine periodic
// neighbours; one thread per node, so every entry has one writer.  sc:
// padded FP64 element scales (Pad<N1, N2> layout), kv: the ten distinct
// entries of K_ref (mu = 1).  Needs n1, n2 >= 3 (distinct neighbours).
template <int N1, int N2>
__device__ __forceinline__ void dense_assemble(float* __restrict__ A, const double* __restrict__ sc, const double (&kv)[10]) {
  constexpr int MD = dense_md(N1, N2), LD = dense_pitch(MD), NN = N1 * N2, NU = 2 * NN - 2;
  using P = rve2d::Pad<N1, N2>;
  for (int t = threadIdx.x; t < MD * LD; t += blockDim.x) {
    const int r = t / LD, c = t % LD;
    A[t] = (r == c && r >= NU) ? 1.0f : 0.0f;
  }
  __syncthreads();
  for (int n = threadIdx.x; n < NN; n += blockDim.x) {
    if (n == 0) continue;
    const int i = n % N1, j = n / N1;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int mi = (i + di + N1) % N1, mj = (j + dj + N2) % N2, m = mj * N1 + mi;
        if (m == 0) continue;
        double k[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        // elements (ei, ej) = (i - 1 .. i, j - 1 .. j) around n that also hold m
#pragma unroll
        for (int ey = -1; ey <= 0; ++ey)
#pragma unroll
          for (int ex = -1; ex <= 0; ++ex) {
            const int ax = -ex, ay = -ey;               // n's offset inside the element
            const int bx = ax + di, by = ay + dj;        // m's offset
            if (bx < 0 || bx > 1 || by < 0 || by > 1) continue;
            const int ca = ay ? (ax ? 2 : 3) : (ax ? 1 : 0);   // corners counter-clockwise
            const int cb = by ? (bx ? 2 : 3) : (bx ? 1 : 0);
            const double mu = sc[P::at(i + ex, j + ey)];
#pragma unroll
            for (int d = 0; d < 2; ++d)
#pragma unroll
              for (int e = 0; e < 2; ++e) {
                const int rr = 2 * ca + d, cc = 2 * cb + e;
                k[d][e] += mu * kref_sign(rr, cc) * kv[kref_id(rr, cc)];
              }
          }
#pragma unroll
        for (int d = 0; d < 2; ++d)
#pragma unroll
          for (int e = 0; e < 2; ++e) A[dof_of(n, d) * LD + dof_of(m, e)] = static_cast<float>(k[d][e]);
      }
  }
  __syncthreads();
}

// Value v of lane src (ds_bpermute: any lane pattern, no LDS storage).
__device__ __forceinline__ float wave_take(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(4 * src, __builtin_bit_cast(int, v)));
}

// C += A_tile * B_tile^T on the matrix cores, A and B 16 x 16 tiles at
// (base + row * ld + col); every lane of the wave calls it.  Lane l supplies
// row l % 16, k = 4 q + l / 16 of both operands (chunk q of four), and holds
// C[4 (l / 16) + j][l % 16] in acc[j].
__device__ __forceinline__ void mma_abt(const float* __restrict__ a, const float* __restrict__ b, int ld, f4v& acc) {
  const int l = threadIdx.x & 63, r = l & 15, kq = l >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r * ld + 4 * q + kq], b[r * ld + 4 * q + kq], acc, 0, 0, 0);
}

// In-place blocked Cholesky of A (MD x MD): L below the diagonal tiles,
// the inverse of each diagonal L tile in its place.  Every thread of the
// work-group calls it.  Returns (work-group uniform) false when a pivot is
// not positive.
template <int MD>
__device__ __forceinline__ bool dense_potrf(float* __restrict__ A, int* s_flag) {
  constexpr int LD = dense_pitch(MD), T = MD / 16;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  if (tid == 0) *s_flag = 0;
  __syncthreads();
  for (int k = 0; k < T; ++k) {
    float* Akk = A + 16 * k * LD + 16 * k;
    if (wid == 0) {
      // The 16 x 16 diagonal tile in the registers of one wave: lane l holds
      // column s = l % 16, rows 4 g .. 4 g + 3 (g = l / 16).  Right-looking
      // Cholesky of the symmetric tile, fused with the forward substitution
      // L X = I that gives its inverse: step c takes the pivot, the scaled
      // column c (entries moved between lanes by ds_bpermute), the rank-one
      // update of the trailing tile and the elimination of row c in X.
      const int s = lane & 15, g = lane >> 4;
      float t4[4], x4[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        t4[t] = Akk[(4 * g + t) * LD + s];
        x4[t] = (4 * g + t == s) ? 1.0f : 0.0f;
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int gc = c >> 2, tc = c & 3;
        const float piv = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, t4[tc]),
                                                                               c + 16 * gc));
        if (!(piv > 0.0f) && lane == 0) *s_flag = 1;
        const float rd = 1.0f / sqrtf(piv > 0.0f ? piv : 1.0f);
        // A[c][s] (= A[s][c]) from lane (s, c / 4); A[r][c] of own rows from lane (c, g)
        const float lsc = wave_take(t4[tc], s + 16 * gc) * rd;
        const float xc = wave_take(x4[tc], s + 16 * gc) * rd;
        float lrc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) lrc[t] = wave_take(t4[t], c + 16 * g) * rd;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int r = 4 * g + t;
          if (r > c && s > c) t4[t] -= lrc[t] * lsc;
          if (r > c) x4[t] -= lrc[t] * xc;
          if (r == c) x4[t] = xc;
        }
      }
      // the inverse replaces the tile (every lane has read its entries)
#pragma unroll
      for (int t = 0; t < 4; ++t) Akk[(4 * g + t) * LD + s] = x4[t];
    }
    __syncthreads();
    // panel: L_ik = A_ik Dinv_k^T, one tile per wave at a time (in place
    // through registers: the wave reads its tile, then overwrites it)
    for (int i = k + 1 + wid; i < T; i += nw) {
      float* Aik = A + 16 * i * LD + 16 * k;
      f4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
      {
        const int r = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Aik[r * LD + 4 * q + kq], Akk[r * LD + 4 * q + kq], acc, 0, 0, 0);
      }
      wave_sync();
#pragma unroll
      for (int j = 0; j < 4; ++j) Aik[(4 * (lane >> 4) + j) * LD + (lane & 15)] = acc[j];
    }
    __syncthreads();
    // trailing update A_ij -= L_ik L_jk^T, k < j <= i
    const int nt = T - k - 1;
    for (int t = wid; t < nt * (nt + 1) / 2; t += nw) {
      int i = 0, rem = t;
      while (rem > i) rem -= ++i;   // t -> (i, j) with j <= i in the trailing triangle
      const int ti = k + 1 + i, tj = k + 1 + rem;
      f4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
      mma_abt(A + 16 * ti * LD + 16 * k, A + 16 * tj * LD + 16 * k, LD, acc);
      float* Aij = A + 16 * ti * LD + 16 * tj;
#pragma unroll
      for (int j = 0; j < 4; ++j) Aij[(4 * (lane >> 4) + j) * LD + (lane & 15)] -= acc[j];
    }
    __syncthreads();
  }
  return *s_flag == 0;
}

// v <- A^-1 v with A = L L^T from dense_potrf (v: MD floats in LDS;
// scratch: 256 floats).  Blocked substitution: per diagonal tile, the
// products with the finished tiles are summed by 16 partial sums per row,
// then the tile's inverse is applied.  Every thread calls it.
template <int MD>
__device__ __forceinline__ void dense_solve(const float* __restrict__ A, float* __restrict__ v, float* __restrict__ scratch) {
  constexpr int LD = dense_pitch(MD), T = MD / 16;
  const int tid = threadIdx.x;
  const int r = tid & 15, part = (tid >> 4) & 15;   // 256 threads: row of the tile, partial sum
  const bool act = tid < 256;
  // forward: L y = v
  for (int k = 0; k < T; ++k) {
    float s = 0.0f;
    if (act)
      for (int c = part; c < 16 * k; c += 16) s += A[(16 * k + r) * LD + c] * v[c];
    if (act) scratch[part * 16 + r] = s;
    __syncthreads();
    if (tid < 16) {
      float t = v[16 * k + tid];
#pragma unroll
      for (int p = 0; p < 16; ++p) t -= scratch[p * 16 + tid];
      v[16 * k + tid] = t;   // right-hand side of the tile
    }
    __syncthreads();
    if (tid < 16) {
      float y = 0.0f;
#pragma unroll
      for (int c = 0; c < 16; ++c) y += A[(16 * k + tid) * LD + 16 * k + c] * v[16 * k + c];
      scratch[tid] = y;
    }
    __syncthreads();
    if (tid < 16) v[16 * k + tid] = scratch[tid];
    __syncthreads();
  }
  // backward: L^T x = y
  for (int k = T - 1; k >= 0; --k) {
    float s = 0.0f;
    if (act)
      for (int c = 16 * (k + 1) + part; c < MD; c += 16) s += A[c * LD + 16 * k + r] * v[c];
    if (act) scratch[part * 16 + r] = s;
    __syncthreads();
    if (tid < 16) {
      float t = v[16 * k + tid];
#pragma unroll
      for (int p = 0; p < 16; ++p) t -= scratch[p * 16 + tid];
      v[16 * k + tid] = t;
    }
    __syncthreads();
    if (tid < 16) {
      float y = 0.0f;   // Dinv_k^T applied: y_r = sum_c Dinv_k[c][r] t_c
#pragma unroll
      for (int c = 0; c < 16; ++c) y += A[(16 * k + c) * LD + 16 * k + tid] * v[16 * k + c];
      scratch[tid] = y;
    }
    __syncthreads();
    if (tid < 16) v[16 * k + tid] = scratch[tid];
    __syncthreads();
  }
}

}  // namespace dense2d
}  // namespace fe2
