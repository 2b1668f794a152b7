// FP64 direct solve of the banded SPD macro system (row a8) by block cyclic
// reduction.
//
// A symmetric matrix of half bandwidth bw is block tridiagonal once it is cut
// into blocks of bs >= bw rows: block i couples only to i-1 and i+1.  Block
// cyclic reduction eliminates the odd blocks of the active set in parallel,
// leaving a block tridiagonal Schur complement on the even blocks, and
// recurses; log2(nb) levels instead of the n sequential column steps of a
// banded Cholesky factorisation.  For an SPD matrix every Schur complement is
// SPD (the scheme is Cholesky factorisation in a nested-dissection order of
// the blocks), so no pivoting is needed and a non-positive pivot means the
// matrix is not SPD.
//
// Per level (stride h; active blocks are the multiples of h; odd ones j =
// h, 3h, ... are eliminated, with left neighbour j-h and right neighbour j+h):
//   potrf : D_j = L_j L_j^T (in place), inverses of its 16x16 diagonal tiles;
//   trsm  : [G_l | G_r | L_j^-1 | g] = L_j^-1 [A_{j,j-h} | A_{j+h,j}^T | I | f_j];
//   schur : for even i:  D_i -= G_r(i-h)^T G_r(i-h) + G_l(i+h)^T G_l(i+h),
//           f_i -= G_r(i-h)^T g(i-h) + G_l(i+h)^T g(i+h),
//           A_{i,i-2h} = -G_r(i-h)^T G_l(i-h).
// Block 0 is left; back substitution runs the levels in reverse:
//   x_j = L_j^-T (g_j - G_l x_{j-h} - G_r x_{j+h}).
//
// Storage (device, FP64): D and C [nb][bs][bs] column-major (C_i couples
// block i to its left active neighbour), G [nb][bs][2 bs] column-major
// ([G_l | G_r]), invL [nb][bs/16][16][16] column-major inverses of the
// diagonal tiles, Linv [nb][bs][bs] column-major L_j^-1, F [nb*bs] the padded
// right-hand side, overwritten by g and then by the solution, T [nb*bs] the
// back-substitution right sides.  Rows beyond n are padded with the identity.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fe2_internal.hpp"
#include "macro.hpp"

namespace fe2 {

namespace {

constexpr int BT = 16;   // tile size

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane-uniform read of lane src's value (two v_readlane) and a per-lane read
// of lane src's value (two ds_bpermute) for FP64 data.
__device__ __forceinline__ double lane_read(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffu), src);
  const unsigned hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), src);
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

// -- extraction of the blocks from lower band storage ------------------------
__global__ void k_bcr_extract(const double* __restrict__ band, int n, int bw, int bs, int nb,
                              double* __restrict__ D, double* __restrict__ C) {
  const size_t per = static_cast<size_t>(bs) * bs;
  const size_t total = per * nb;
  for (size_t t = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int b = static_cast<int>(t / per);
    const int rem = static_cast<int>(t - b * per);
    const int c = rem / bs, r = rem - c * bs;
    const int i = b * bs + r, j = b * bs + c;
    double dv;
    if (i < n && j < n) {
      const int lo = i > j ? i : j, hi = i > j ? j : i;
      dv = (lo - hi <= bw) ? band[static_cast<size_t>(hi) * (bw + 1) + (lo - hi)] : 0.0;
    } else {
      dv = (r == c) ? 1.0 : 0.0;
    }
    D[t] = dv;
    double cv = 0.0;
    if (b > 0 && i < n) {
      const int jj = (b - 1) * bs + c;   // i - jj = bs + r - c >= 1
      if (i - jj <= bw) cv = band[static_cast<size_t>(jj) * (bw + 1) + (i - jj)];
    }
    C[t] = cv;
  }
}

__global__ void k_bcr_copy_in(const double* __restrict__ y, int n, int np, double* __restrict__ F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) F[i] = i < n ? y[i] : 0.0;
}

__global__ void k_bcr_copy_out(const double* __restrict__ F, int n, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = F[i];
}

// -- potrf: one work-group per eliminated block -------------------------------
// Right-looking Cholesky in 16-column panels.  When the lower triangle of the
// block fits in LDS (tile-packed 16x16 column-major tiles) it is factored
// there and written back once; for larger blocks the first steps run in
// place in global memory until the trailing triangle fits, which is then
// factored in LDS.  Wave 0 factors the diagonal tile and inverts it (the tile
// in its registers, exchanges between lanes); all waves form the panel below
// with the inverse and apply the trailing update in 16x16 MFMA tiles.  With
// lookahead: during the trailing update of step p wave 0 updates diagonal
// tile p + 1 first and factors it while the other waves update the rest, so
// the diagonal factor leaves the critical path and a step needs two barriers.
constexpr int PO_WG = 1024;
typedef double v4d __attribute__((ext_vector_type(4)));

struct GlobalTiles {
  double* base;
  int ld;
  __device__ double* tile(int ti, int tk) const { return base + static_cast<size_t>(tk) * BT * ld + ti * BT; }
};
// Lower-triangle tiles in LDS, column-major with a column pitch of BT + 1:
// the sixteen columns a wave's tile access touches then fall on different
// banks (with a pitch of BT they shared eight).
constexpr int LDS_TILE = BT * (BT + 1);
struct LdsTiles {
  double* base;
  int o = 0;   // the tiles held: o <= tk <= ti (the trailing triangle from step o on)
  static constexpr int ld = BT + 1;
  __device__ double* tile(int ti, int tk) const {
    const int a = ti - o, c = tk - o;
    return base + (a * (a + 1) / 2 + c) * LDS_TILE;
  }
};

__device__ __forceinline__ int tri_row(int q) {   // largest a with a(a+1)/2 <= q
  int a = static_cast<int>((sqrtf(8.0f * q + 1.0f) - 1.0f) * 0.5f);
  while (a * (a + 1) / 2 > q) --a;
  while ((a + 1) * (a + 2) / 2 <= q) ++a;
  return a;
}

// Cross-lane moves of the diagonal factor, register to register (no LDS
// trip).  Lanes form four rows of 16; lane (s, g) = s + 16 g.
// From lane (N, g) of the same row: DPP row_newbcast.
template <int N>
__device__ __forceinline__ double from_row_lane(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  // every lane of every row is a valid source: no old value to keep
  const unsigned lo = __builtin_amdgcn_mov_dpp(static_cast<int>(u & 0xffffffffu), 0x150 + N, 0xf, 0xf, true);
  const unsigned hi = __builtin_amdgcn_mov_dpp(static_cast<int>(u >> 32), 0x150 + N, 0xf, 0xf, true);
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}
// From lane src, any row: ds_bpermute (through the LDS crossbar; its latency
// overlaps the pivot's reciprocal square root).
__device__ __forceinline__ double lane_take(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_ds_bpermute(4 * src, static_cast<int>(u & 0xffffffffu));
  const unsigned hi = __builtin_amdgcn_ds_bpermute(4 * src, static_cast<int>(u >> 32));
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

// Column step C of the diagonal factor (below): pivot, scaled column C of L,
// rank-one update of the trailing entries, elimination of row C in X.  A
// pivot that is not positive records C in fail_c (uniform); from then on the
// pivots are taken as 1 and the tile is discarded.  Each wave64 VALU
// instruction takes four cycles on the 16-lane SIMD and the steps are
// serial, so the step is written for few instructions: the multipliers are
// masked once (an update with a zero multiplier leaves the entry as it is),
// and lane column C keeps its entries unscaled: nothing changes or reads them
// after this step, so the factor's write-back scales them by the rd kept in
// dsc (the same products).
template <int C>
__device__ __forceinline__ void diag_cols(double (&t4)[4], double (&x4)[4], double& dsc, int s, int g, int& fail_c) {
  constexpr int GC = C >> 2, TC = C & 3;
  double piv = lane_read(t4[TC], C + 16 * GC);
  if (!(piv > 0.0) && fail_c < 0) fail_c = C;
  if (fail_c >= 0) piv = 1.0;
  // A[C][s] (= A[s][C]) and X[C][s] from lane (s, C / 4); A[r][C] of own rows from lane (C, g)
  const double asc = lane_take(t4[TC], s + 16 * GC);
  const double xsc = lane_take(x4[TC], s + 16 * GC);
  const double rd = rsqrt(piv);
  const double lsc = s > C ? asc * rd : 0.0;
  const double xc = xsc * rd;
  // rd masked to the rows below row C: for t > C % 4 those of g >= C / 4, else g > C / 4
  const double rd_gt = g > GC ? rd : 0.0, rd_ge = g >= GC ? rd : 0.0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double lrc = from_row_lane<C>(t4[t]) * (t > TC ? rd_ge : rd_gt);
    t4[t] = fma(-lrc, lsc, t4[t]);
    x4[t] = fma(-lrc, xc, x4[t]);
  }
  if (s == C) dsc = rd;   // column C of L: the column times rd (its diagonal piv * rd)
  if (g == GC) x4[TC] = xc;
  if constexpr (C + 1 < BT) diag_cols<C + 1>(t4, x4, dsc, s, g, fail_c);
}

// Factor diagonal tile p in place and write its inverse to s_inv; wave 0
// only.  The tile sits in the registers of the wave: lane (s, g) holds
// column s, rows 4 g .. 4 g + 3, read from the lower triangle (the upper
// entries mirrored).  Right-looking Cholesky fused with the forward
// substitution L X = I that gives invL_pp.  A pivot that is not positive sets
// *s_fail and info (the caller checks *s_fail after its next barrier).
template <class M>
__device__ __forceinline__ void potrf_diag(const M& A, int p, int col0, double* s_inv, int* s_fail,
                                           int* __restrict__ info) {
  const int ld = A.ld;
  const int ln = threadIdx.x, s = ln & 15, g = ln >> 4;
  double* Tpp = A.tile(p, p);
  double t4[4], x4[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = 4 * g + t;
    t4[t] = r >= s ? Tpp[s * ld + r] : Tpp[r * ld + s];
    x4[t] = (r == s) ? 1.0 : 0.0;
  }
  int fail_c = -1;
  double dsc = 1.0;
  diag_cols<0>(t4, x4, dsc, s, g, fail_c);
  if (fail_c >= 0) {
    if (ln == 0) {
      *s_fail = 1;
      atomicCAS(info, 0, col0 + p * BT + fail_c + 1);
    }
    return;
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = 4 * g + t;
    if (r >= s) Tpp[s * ld + r] = t4[t] * dsc;
    s_inv[s * BT + r] = x4[t];   // column-major; zero above the diagonal
  }
}

// Returns false when a pivot is not positive (info set, every thread returns).
// diag_done: tile p_begin was already factored (and s_inv holds its inverse)
// by the lookahead of an earlier call.
template <class M>
__device__ __forceinline__ bool potrf_core(const M& A, double* __restrict__ Ij, int nt, int p_begin, int p_end,
                                           int col0, double* s_panel, double* s_inv, int* s_fail,
                                           int* __restrict__ info, bool diag_done) {
  const int tid = threadIdx.x;
  const int ld = A.ld;
  if (!diag_done && p_begin < p_end) {
    if (tid < 64) potrf_diag(A, p_begin, col0, s_inv, s_fail, info);
    __syncthreads();
    if (*s_fail) return false;
  }
  for (int p = p_begin; p < p_end; ++p) {
    // the inverse tile goes out after the barrier (its stores complete
    // during the panel phase instead of delaying wave 0)
    static_assert(PO_WG >= BT * BT && PO_WG % (BT * BT) == 0, "one inverse entry per thread");
    if (tid < BT * BT) Ij[p * BT * BT + tid] = s_inv[tid];
    // panel below: L_ip = A_ip invL_pp^T, one 16x16 tile per wave at a time
    // as four 16x16x4 FP64 MFMAs (s_inv is column-major: s_inv[k*16 + n] =
    // (invL_pp)_nk, the (k, n) entry of invL_pp^T)
    {
      const int wv = tid >> 6, ln = tid & 63;
      const int lr = ln & 15, lk = ln >> 4;
      for (int t = wv; t < nt - p - 1; t += PO_WG / 64) {
        double* Tip = A.tile(p + 1 + t, p);
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < BT; kk += 4)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Tip[(kk + lk) * ld + lr], s_inv[(kk + lk) * BT + lr], acc, 0,
                                                     0, 0);
        // every lane has read its operands of this tile before any lane
        // overwrites it: the MFMAs consume them in order within the wave
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = lk + 4 * j;
          Tip[lr * ld + row] = acc[j];
          s_panel[(t * BT + row) * (BT + 1) + lr] = acc[j];
        }
      }
    }
    __syncthreads();
    // trailing update of the lower tiles (ti, tk), p < tk <= ti < nt, one
    // 16x16 tile per wave at a time on the FP64 matrix cores:
    // T_ab -= P_a P_b^T as four 16x16x4 products over the panel's columns.
    // Operand layout of the 16x16x4 FP64 MFMA: lane l supplies row l%16 and
    // k = l/16 of both operands; result register j of lane l is entry
    // (l/16 + 4j, l%16).
    const int m = nt - p - 1;
    const int ntiles = m * (m + 1) / 2;
    const int wv = tid >> 6, ln = tid & 63;
    const int lr = ln & 15, lk = ln >> 4;
    auto update = [&](int q) {
      const int ta = tri_row(q), tb = q - ta * (ta + 1) / 2;
      const double* pa = s_panel + (ta * BT + lr) * (BT + 1) + lk;
      const double* pb = s_panel + (tb * BT + lr) * (BT + 1) + lk;
      v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < BT; kk += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[kk], pb[kk], acc, 0, 0, 0);
      double* Tab = A.tile(p + 1 + ta, p + 1 + tb);
#pragma unroll
      for (int j = 0; j < 4; ++j) Tab[lr * ld + lk + 4 * j] -= acc[j];
    };
    // lookahead: wave 0 updates the next diagonal tile (q = 0) and factors
    // it while the other waves update the rest of the trailing triangle
    if (wv == 0) {
      if (m > 0) {
        update(0);
        __threadfence_block();   // the tile's new entries, written by other lanes, before the wave reads them
        potrf_diag(A, p + 1, col0, s_inv, s_fail, info);
      }
    } else {
      for (int q = wv; q < ntiles; q += PO_WG / 64 - 1) update(q);
    }
    __syncthreads();
    if (*s_fail) return false;
  }
  return true;
}

// LDS bytes of the two variants
__host__ __device__ constexpr size_t potrf_lds_global(int bs) { return static_cast<size_t>(bs) * (BT + 1) * 8; }
// with the trailing triangle of m tile rows in LDS
__host__ __device__ constexpr size_t potrf_lds_resident(int bs, int m) {
  return potrf_lds_global(bs) + static_cast<size_t>(m * (m + 1) / 2) * LDS_TILE * 8;
}

// RESIDENT: steps p < p0 run on the tiles in global memory, then the
// trailing triangle (tiles p0 <= tk <= ti) is loaded into LDS, factored there
// and written back once (p0 = 0 when the whole lower triangle fits).
template <bool RESIDENT>
__global__ void __launch_bounds__(PO_WG) k_bcr_potrf(double* __restrict__ D, double* __restrict__ invL, int bs,
                                                     int first, int stride, int p0, int* __restrict__ info) {
  extern __shared__ __align__(16) double smem[];
  __shared__ double s_inv[BT * BT];   // column-major
  __shared__ int s_fail;
  const int j = first + stride * static_cast<int>(blockIdx.x);
  const int nt = bs / BT;
  double* Dj = D + static_cast<size_t>(j) * bs * bs;
  double* Ij = invL + static_cast<size_t>(j) * nt * BT * BT;
  const int tid = threadIdx.x;
  double* s_panel = smem;   // [bs][BT + 1] (padded rows)
  if (tid == 0) s_fail = 0;
  if constexpr (RESIDENT) {
    if (p0 > 0) {
      __syncthreads();
      const GlobalTiles G{Dj, bs};
      if (!potrf_core(G, Ij, nt, 0, p0, j * bs, s_panel, s_inv, &s_fail, info, false)) return;
    }
    double* s_tiles = smem + bs * (BT + 1);
    const int m = nt - p0;
    const int ntri = m * (m + 1) / 2;
    // With the whole triangle resident, wave 0 copies tile 0 and factors it
    // while waves 4.. load the other tiles (the factor of the first tile
    // then overlaps the load instead of following it).
    const bool early = p0 == 0;
    if (early && tid < 64) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e2 = tid + 64 * u, cc = e2 >> 4, rr = e2 & 15;
        s_tiles[cc * (BT + 1) + rr] = Dj[static_cast<size_t>(cc) * bs + rr];
      }
      __threadfence_block();
      potrf_diag(LdsTiles{s_tiles, 0}, 0, j * bs, s_inv, &s_fail, info);
    }
    // one element of a tile per thread, one tile per 256 threads and pass
    constexpr int TPP = PO_WG / (BT * BT);
    const int el = tid % (BT * BT), c = el >> 4, r = el & 15;
    const int grp = tid / (BT * BT) - (early ? 1 : 0), ngrp = TPP - (early ? 1 : 0), q_first = early ? 1 : 0;
    // the loads of a batch of tiles are all issued before the first is
    // stored, so their latencies overlap
    constexpr int LB = 16;
    if (grp >= 0) {
      for (int q0 = q_first + grp; q0 < ntri; q0 += LB * ngrp) {
        double v[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int q = q0 + u * ngrp;
          if (q < ntri) {
            const int ti = tri_row(q), tk = q - ti * (ti + 1) / 2;
            v[u] = Dj[static_cast<size_t>((tk + p0) * BT + c) * bs + (ti + p0) * BT + r];
          }
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int q = q0 + u * ngrp;
          if (q < ntri) s_tiles[q * LDS_TILE + c * (BT + 1) + r] = v[u];
        }
      }
    }
    __syncthreads();
    if (s_fail) return;
    const LdsTiles A{s_tiles, p0};
    if (!potrf_core(A, Ij, nt, p0, nt, j * bs, s_panel, s_inv, &s_fail, info, true)) return;
#pragma unroll 2
    for (int q = tid / (BT * BT); q < ntri; q += TPP) {
      const int ti = tri_row(q), tk = q - ti * (ti + 1) / 2;
      Dj[static_cast<size_t>((tk + p0) * BT + c) * bs + (ti + p0) * BT + r] = s_tiles[q * LDS_TILE + c * (BT + 1) + r];
    }
  } else {
    __syncthreads();
    const GlobalTiles A{Dj, bs};
    potrf_core(A, Ij, nt, 0, nt, j * bs, s_panel, s_inv, &s_fail, info, false);
  }
}

// -- trsm: one wave per (16-column tile, eliminated block) ---------------------
// Forward substitution L_j X = R on one tile of R = [C_j | C_{j+h}^T | I | f_j]
// (the identity tiles give L_j^-1 for the back substitution), 16 rows at a
// time: S_i = R_i - sum_{k<i} L_ik X_k, X_i = invL_ii S_i, both products as
// 16x16x4 FP64 MFMAs (lane l supplies row l%16 and k = l/16 of both
// operands; result register j of lane l is entry (l/16 + 4j, l%16)).  Tiles:
// [0, nt) left coupling, [nt, 2nt) right coupling, [2nt, 3nt) identity, 3nt
// right-hand side (one column; the other 15 stay zero); a block with no
// neighbours (the last one left) runs only the last nt + 1.
constexpr int TR_WG = 64;
constexpr int TR_UNROLL = 16;   // MFMAs whose L operand loads are issued together (four tiles)

__global__ void __launch_bounds__(TR_WG) k_bcr_trsm(const double* __restrict__ D, const double* __restrict__ invL,
                                                    const double* __restrict__ C, double* __restrict__ G,
                                                    double* __restrict__ Linv, double* __restrict__ F, int bs,
                                                    int nb, int first, int stride, int h, int alone) {
  extern __shared__ __align__(16) double s_x[];   // [bs][BT] row-major: R, overwritten by X
  __shared__ double s_s[BT * BT];                 // [row][col]
  const int j = first + stride * static_cast<int>(blockIdx.y);
  const int nt = bs / BT;
  const int ct = alone ? 2 * nt + static_cast<int>(blockIdx.x) : static_cast<int>(blockIdx.x);
  const size_t per = static_cast<size_t>(bs) * bs;
  const double* src = nullptr;
  double* out;
  int ld_r = 0, ld_c = 0, ncol = BT, ident = -1, i0 = 0;
  // R(r, c) = src[r * ld_r + c * ld_c], or (r == ident + c) for identity tiles;
  // out(r, c) = out[c * bs + r]
  if (ct < nt) {
    src = C + j * per + static_cast<size_t>(ct) * BT * bs;
    ld_r = 1;
    ld_c = bs;
    out = G + j * 2 * per + static_cast<size_t>(ct) * BT * bs;
  } else if (ct < 2 * nt) {
    if (j + h >= nb) return;
    src = C + (j + h) * per + (ct - nt) * BT;
    ld_r = bs;
    ld_c = 1;
    out = G + j * 2 * per + static_cast<size_t>(bs + (ct - nt) * BT) * bs;
  } else if (ct < 3 * nt) {
    i0 = ct - 2 * nt;   // rows above the tile's diagonal stay zero
    ident = i0 * BT;
    out = Linv + j * per + static_cast<size_t>(i0) * BT * bs;
  } else {
    src = F + static_cast<size_t>(j) * bs;
    ld_r = 1;
    ld_c = 0;
    out = F + static_cast<size_t>(j) * bs;
    ncol = 1;
  }
  const double* Lj = D + j * per;
  const double* Ij = invL + static_cast<size_t>(j) * nt * BT * BT;
  const int ln = threadIdx.x, lr = ln & 15, lk = ln >> 4;
  // R into LDS: lane (lr, lk) covers column lr, rows lk, lk + 4, ...
  for (int row = lk; row < bs; row += 4) {
    double v;
    if (ident >= 0) v = (row == ident + lr) ? 1.0 : 0.0;
    else v = (lr < ncol) ? src[static_cast<size_t>(row) * ld_r + static_cast<size_t>(lr) * ld_c] : 0.0;
    s_x[row * BT + lr] = v;
  }
  wave_sync();
  for (int i = i0; i < nt; ++i) {
    // invL_ii (column-major: entry (r, c) at Ij[i*256 + c*16 + r]) depends on
    // nothing computed here: its loads go out first and land during the
    // product below
    double il[BT / 4];
#pragma unroll
    for (int kk = 0; kk < BT; kk += 4) il[kk / 4] = Ij[i * BT * BT + (kk + lk) * BT + lr];
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    // sum_{k<i} L_ik X_k: L is column-major (entry (r, k) at Lj[k * bs + r])
    const double* lcol = Lj + static_cast<size_t>(lk) * bs + i * BT + lr;
    for (int k0 = i0 * BT; k0 < i * BT; k0 += 4 * TR_UNROLL) {
      double xl[TR_UNROLL];
#pragma unroll
      for (int u = 0; u < TR_UNROLL; ++u) {
        const int k = k0 + 4 * u;
        xl[u] = k < i * BT ? lcol[static_cast<size_t>(k) * bs] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < TR_UNROLL; ++u) {
        const int k = k0 + 4 * u;
        if (k < i * BT) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xl[u], s_x[(k + lk) * BT + lr], acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = lk + 4 * q;
      s_s[rr * BT + lr] = s_x[(i * BT + rr) * BT + lr] - acc[q];
    }
    wave_sync();
    // X_i = invL_ii S_i
    v4d x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < BT; kk += 4)
      x = __builtin_amdgcn_mfma_f64_16x16x4f64(il[kk / 4], s_s[(kk + lk) * BT + lr], x, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) s_x[(i * BT + lk + 4 * q) * BT + lr] = x[q];
    wave_sync();
  }
  if (lr < ncol)
    for (int row = lk; row < bs; row += 4) out[static_cast<size_t>(lr) * bs + row] = row < i0 * BT ? 0.0 : s_x[row * BT + lr];
}

// -- schur: one wave per (output tile, even block) -----------------------------
// Output tiles of block i: lower tiles of D_i, all tiles of the new coupling
// C_i, and the 16-row pieces of f_i.  Each is a sum of at most two products
// A^T B with K = bs, formed on the FP64 matrix cores as 16x16x4 MFMAs
// (lane l supplies row l%16 and k = l/16 of both operands; result register
// j of lane l is entry (l/16 + 4j, l%16)).  A right-hand-side piece is the
// product with a single column: the other 15 columns of the B operand are
// zero.
constexpr int SC_WG = 64;
constexpr int SC_UNROLL = 8;   // MFMAs whose operand loads are issued together

__global__ void __launch_bounds__(SC_WG) k_bcr_schur(const double* __restrict__ G, double* __restrict__ D,
                                                     double* __restrict__ C, double* __restrict__ F, int bs, int nb,
                                                     int h) {
  const int i = 2 * h * static_cast<int>(blockIdx.y);
  const int nt = bs / BT;
  const int ntri = nt * (nt + 1) / 2;
  const int q = blockIdx.x;
  const size_t per = static_cast<size_t>(bs) * bs;
  const int jl = i - h, jr = i + h;
  const bool has_l = i > 0, has_r = jr < nb;
  int kind, ta, tb;
  if (q < ntri) {
    kind = 0;
    ta = static_cast<int>((sqrtf(8.0f * q + 1.0f) - 1.0f) * 0.5f);
    while (ta * (ta + 1) / 2 > q) --ta;
    while ((ta + 1) * (ta + 2) / 2 <= q) ++ta;
    tb = q - ta * (ta + 1) / 2;
  } else if (q < ntri + nt * nt) {
    kind = 1;
    ta = (q - ntri) / nt;
    tb = (q - ntri) - ta * nt;
    if (!has_l || i < 2 * h) return;
  } else {
    kind = 2;
    ta = q - ntri - nt * nt;
    tb = 0;
  }
  // contributions: (A columns, B columns or vector), at most two
  const double *A0 = nullptr, *B0 = nullptr, *A1 = nullptr, *B1 = nullptr;
  int ncon = 0;
  if (has_l) {   // G_r(i-h) on the left
    const double* Gl = G + static_cast<size_t>(jl) * 2 * per;
    A0 = Gl + per + static_cast<size_t>(ta) * BT * bs;
    B0 = kind == 0 ? Gl + per + static_cast<size_t>(tb) * BT * bs
       : kind == 1 ? Gl + static_cast<size_t>(tb) * BT * bs
                   : F + static_cast<size_t>(jl) * bs;
    ncon = 1;
  }
  if (has_r && kind != 1) {   // G_l(i+h)
    const double* Gr = G + static_cast<size_t>(jr) * 2 * per;
    const double* a = Gr + static_cast<size_t>(ta) * BT * bs;
    const double* bb = kind == 0 ? Gr + static_cast<size_t>(tb) * BT * bs : F + static_cast<size_t>(jr) * bs;
    if (ncon == 0) {
      A0 = a;
      B0 = bb;
    } else {
      A1 = a;
      B1 = bb;
    }
    ++ncon;
  }
  if (ncon == 0) return;
  const int ln = threadIdx.x, lr = ln & 15, lk = ln >> 4;
  const bool vec = kind == 2;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  // Within each 16-wide slab of the summation index, lane (lr, lk) supplies
  // entries 4 lk .. 4 lk + 3 of column lr of the A block and of the B block,
  // one per MFMA of the slab: the four MFMAs together still contract the
  // slab's 16 entries once, and each lane reads its four as one 32-byte
  // load (four lanes cover a 128-byte line) instead of four strided ones.
  // bs is a multiple of 16.  A vector B is read by the lr = 0 lanes.
  constexpr int SU = SC_UNROLL / 4;   // slabs per batch of loads
#pragma unroll
  for (int cn = 0; cn < 2; ++cn) {
    if (cn >= ncon) break;
    const double* Aq = cn == 0 ? A0 : A1;
    const double* Bq = cn == 0 ? B0 : B1;
    const double* pa = Aq + static_cast<size_t>(lr) * bs + 4 * lk;
    const double* pb = vec ? Bq + 4 * lk : Bq + static_cast<size_t>(lr) * bs + 4 * lk;
    const bool bload = !vec || lr == 0;
    for (int k0 = 0; k0 < bs; k0 += BT * SU) {
      double2 xa[SU][2], xb[SU][2];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        // a slab past the end reads slab 0 (a valid address) and is zeroed
        const int k = k0 + BT * u;
        const bool in = k < bs;
        const int kc = in ? k : 0;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const double2 va = reinterpret_cast<const double2*>(pa + kc)[hh];
          const double2 vb = reinterpret_cast<const double2*>(pb + kc)[hh];
          xa[u][hh] = make_double2(in ? va.x : 0.0, in ? va.y : 0.0);
          xb[u][hh] = make_double2(in && bload ? vb.x : 0.0, in && bload ? vb.y : 0.0);
        }
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u][0].x, xb[u][0].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u][0].y, xb[u][0].y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u][1].x, xb[u][1].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u][1].y, xb[u][1].y, acc, 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = ta * BT + lk + 4 * j;   // entry (lk + 4j, lr) of the tile
    if (kind == 0) {
      D[i * per + static_cast<size_t>(tb * BT + lr) * bs + row] -= acc[j];
    } else if (kind == 1) {
      C[i * per + static_cast<size_t>(tb * BT + lr) * bs + row] = -acc[j];
    } else if (lr == 0) {
      F[static_cast<size_t>(i) * bs + row] -= acc[j];
    }
  }
}

// -- back substitution: two passes per level, one work-group per (16-row tile,
// eliminated block) --------------------------------------------------------
//   back_t: t_j = g_j - G_l x_{j-h} - G_r x_{j+h}   (into T)
//   back_x: x_j = L_j^-T t_j = sum_k Linv(k, .) t_k  (into F)
// 256 threads = 16 rows x 16 slices of the summation index, reduced in LDS.
constexpr int BK_WG = 256;

__global__ void __launch_bounds__(BK_WG) k_bcr_back_t(const double* __restrict__ G, const double* __restrict__ F,
                                                      double* __restrict__ T, int bs, int nb, int first, int stride,
                                                      int h, int alone) {
  __shared__ double s_red[BT][BT + 1];
  const int j = first + stride * static_cast<int>(blockIdx.y);
  const int rr = threadIdx.x & 15, sl = threadIdx.x >> 4;   // 16 consecutive rows per slice
  const int row = blockIdx.x * BT + rr;
  const size_t per = static_cast<size_t>(bs) * bs;
  const bool has_l = !alone && j >= h, has_r = !alone && j + h < nb;
  const double* Gj = G + j * 2 * per;
  const double* xl = F + static_cast<size_t>(has_l ? j - h : j) * bs;
  const double* xr = F + static_cast<size_t>(has_r ? j + h : j) * bs;
  double a0 = 0.0, a1 = 0.0;
  if (has_l)
#pragma unroll 4
    for (int c = sl; c < bs; c += BT) a0 = fma(Gj[static_cast<size_t>(c) * bs + row], xl[c], a0);
  if (has_r)
#pragma unroll 4
    for (int c = sl; c < bs; c += BT) a1 = fma(Gj[per + static_cast<size_t>(c) * bs + row], xr[c], a1);
  s_red[rr][sl] = a0 + a1;
  __syncthreads();
  if (threadIdx.x < BT) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < BT; ++q) t += s_red[threadIdx.x][q];
    const size_t o = static_cast<size_t>(j) * bs + blockIdx.x * BT + threadIdx.x;
    T[o] = F[o] - t;
  }
}

__global__ void __launch_bounds__(BK_WG) k_bcr_back_x(const double* __restrict__ Linv, const double* __restrict__ T,
                                                      double* __restrict__ F, int bs, int first, int stride) {
  __shared__ double s_red[BT][BT + 1];
  const int j = first + stride * static_cast<int>(blockIdx.y);
  const int rr = threadIdx.x >> 4, sl = threadIdx.x & 15;
  const int row = blockIdx.x * BT + rr;
  const double* li = Linv + static_cast<size_t>(j) * bs * bs + static_cast<size_t>(row) * bs;   // column `row` of L^-1
  const double* tj = T + static_cast<size_t>(j) * bs;
  double a0 = 0.0, a1 = 0.0;
  int k = blockIdx.x * BT + sl;   // L^-1(k, row) = 0 for k < row
  for (; k + BT < bs; k += 2 * BT) {
    a0 = fma(li[k], tj[k], a0);
    a1 = fma(li[k + BT], tj[k + BT], a1);
  }
  if (k < bs) a0 = fma(li[k], tj[k], a0);
  s_red[rr][sl] = a0 + a1;
  __syncthreads();
  if (threadIdx.x < BT) {
    double x = 0.0;
#pragma unroll
    for (int q = 0; q < BT; ++q) x += s_red[threadIdx.x][q];
    F[static_cast<size_t>(j) * bs + blockIdx.x * BT + threadIdx.x] = x;
  }
}

}  // namespace

BcrPlan bcr_plan(int n, int bw) {
  BcrPlan p;
  p.n = n;
  p.bw = bw;
  p.bs = std::max(BT, ((bw + BT - 1) / BT) * BT);
  p.nb = (n + p.bs - 1) / p.bs;
  const size_t per = static_cast<size_t>(p.bs) * p.bs;
  p.d_len = per * p.nb;
  p.g_len = 2 * per * p.nb;
  p.inv_len = static_cast<size_t>(p.nb) * p.bs * BT;
  p.f_len = static_cast<size_t>(p.nb) * p.bs;
  return p;
}

int bcr_max_bandwidth() { return 1120; }   // trsm right-hand sides + staging within 160 KiB of LDS

size_t bcr_workspace_doubles(const BcrPlan& p) { return 3 * p.d_len + p.g_len + p.inv_len + 2 * p.f_len; }

int bcr_solve(const BcrPlan& p, double* ws, const double* band, double* y, int* info, hipStream_t s) {
  double* D = ws;
  double* C = D + p.d_len;
  double* G = C + p.d_len;
  double* IL = G + p.g_len;
  double* F = IL + p.inv_len;
  double* LI = F + p.f_len;
  double* T = LI + p.d_len;
  const int bs = p.bs, nb = p.nb, nt = bs / BT;
  const unsigned eg = static_cast<unsigned>(std::min<size_t>(8192, (p.d_len + 255) / 256));
  hipLaunchKernelGGL(k_bcr_extract, dim3(eg), dim3(256), 0, s, band, p.n, p.bw, bs, nb, D, C);
  const int np = nb * bs;
  hipLaunchKernelGGL(k_bcr_copy_in, dim3((np + 255) / 256), dim3(256), 0, s, y, p.n, np, F);
  const size_t lds_tr = static_cast<size_t>(bs) * BT * sizeof(double);
  // factor in LDS the trailing triangle of as many tile rows as fit next to
  // the panel (all nt when the block's whole lower triangle does; the steps
  // before it run on the tiles in global memory)
  int m_lds = nt;
  while (m_lds > 0 && potrf_lds_resident(bs, m_lds) + 8 * 1024 > 160 * 1024) --m_lds;
  const bool resident = m_lds >= 2;
  const int p0 = resident ? nt - m_lds : 0;
  const size_t lds_po = resident ? potrf_lds_resident(bs, m_lds) : potrf_lds_global(bs);
  auto potrf = resident ? k_bcr_potrf<true> : k_bcr_potrf<false>;
  if (lds_po + 8 * 1024 > 64 * 1024)
    FE2_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(potrf), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      static_cast<int>(lds_po)));
  if (lds_tr + 12 * 1024 > 64 * 1024)
    FE2_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bcr_trsm),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_tr)));
  const int ntri = nt * (nt + 1) / 2;
  int h = 1;
  for (;;) {
    const int nact = (nb - 1) / h + 1;
    if (nact == 1) break;
    const int nodd = nact / 2, neven = (nact + 1) / 2;
    hipLaunchKernelGGL(potrf, dim3(nodd), dim3(PO_WG), lds_po, s, D, IL, bs, h, 2 * h, p0, info);
    hipLaunchKernelGGL(k_bcr_trsm, dim3(3 * nt + 1, nodd), dim3(TR_WG), lds_tr, s, D, IL, C, G, LI, F, bs, nb, h,
                       2 * h, h, 0);
    hipLaunchKernelGGL(k_bcr_schur, dim3(ntri + nt * nt + nt, neven), dim3(SC_WG), 0, s, G, D, C, F, bs, nb, h);
    h *= 2;
  }
  const int htop = h;
  hipLaunchKernelGGL(potrf, dim3(1), dim3(PO_WG), lds_po, s, D, IL, bs, 0, 0, p0, info);
  hipLaunchKernelGGL(k_bcr_trsm, dim3(nt + 1, 1), dim3(TR_WG), lds_tr, s, D, IL, C, G, LI, F, bs, nb, 0, 0, 0, 1);
  hipLaunchKernelGGL(k_bcr_back_t, dim3(nt, 1), dim3(BK_WG), 0, s, G, F, T, bs, nb, 0, 0, 0, 1);
  hipLaunchKernelGGL(k_bcr_back_x, dim3(nt, 1), dim3(BK_WG), 0, s, LI, T, F, bs, 0, 0);
  for (h = htop / 2; h >= 1; h /= 2) {
    const int nact = (nb - 1) / h + 1;
    const int nodd = nact / 2;
    hipLaunchKernelGGL(k_bcr_back_t, dim3(nt, nodd), dim3(BK_WG), 0, s, G, F, T, bs, nb, h, 2 * h, h, 0);
    hipLaunchKernelGGL(k_bcr_back_x, dim3(nt, nodd), dim3(BK_WG), 0, s, LI, T, F, bs, h, 2 * h);
  }
  hipLaunchKernelGGL(k_bcr_copy_out, dim3((p.n + 255) / 256), dim3(256), 0, s, F, p.n, y);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

}  // namespace fe2
