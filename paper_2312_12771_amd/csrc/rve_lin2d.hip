// RVE element integration, periodic null-space solve and condensation for
// two-dimensional small-strain RVEs (Q4, plane strain, linear isotropic
// phases), one work-group per RVE.
//
// Method (Hesch, Schmidt, Schuss, arXiv:2312.12771):
//   * micro residual r_b = K_wF eps_b + K_ww w_b and stress integral
//     int sigma~ = K_FF eps_b + K_wF^T w_b (Eqs. (34)-(35), (17));
//   * solve K_ww [X_F | x_r] = [K_wF | r_b] (the RVE block of L in Eq. (42))
//     with the periodic null space of condition (iii) in Eq. (15): periodic
//     node identification and a pinned corner node;
//   * condensation Cbar = (K_FF - K_wF^T X_F)/|Omega|,
//     Phat = (int sigma~ - K_wF^T x_r)/|Omega| (Eqs. (46)-(48)).
//
// GPU design
//   * Every RVE element has stiffness mu_e * K_ref (all phases of a
//     resolution class share lambda/mu).  K_ref of the bilinear box element
//     has ten distinct entries; the operator is applied matrix-free from those
//     ten scalars (held in scalar registers) and one scale per element in LDS.
//   * Each thread owns a 2x2 block of nodes and gathers the 4x4 neighbourhood
//     of the search direction.  Vectors live in LDS with a one-node periodic
//     halo, so the neighbourhood is a contiguous window addressed from one
//     base register with immediate offsets; node-centric gather, no scatter,
//     no atomics, deterministic.
//   * RVE sizes are compile-time template parameters.
//   * PCG state lives in registers and LDS; HBM is touched only for phase ids,
//     the state w and the outputs.
//   * Preconditioner: Jacobi, or (square 8/16/32/48 RVEs) the inverse of the
//     periodic operator of a homogeneous reference medium, applied by a 2D
//     FFT in LDS (48 = 3 x 16: one radix-3 x 3 stage, then radix-2 x 2
//     stages); the latter with the standard two-reduction PCG loop.
//   * Precision: the inner PCG runs in TI (float for the FP32_IR form, double
//     for plain FP64).  An outer refinement loop forms the true residual in
//     FP64 from the FP64 solution kept in the output buffer; the condensation
//     uses the FP64 residual to correct the Schur product (energy form, error
//     quadratic in the solve error).
#include <cmath>
#include <type_traits>

#include "rve2d_common.hpp"

namespace fe2 {

using namespace rve2d;

namespace {

constexpr int NF = 3;

template <typename V>
__device__ __forceinline__ V kfma(const V (&kv)[10], int r, int c, V x, V acc) {
  return kref_sign(r, c) > 0 ? fma(kv[kref_id(r, c)], x, acc) : fma(-kv[kref_id(r, c)], x, acc);
}

// a <- b * a + c in a's own register (a loop-carried multiplicand would
// otherwise be recomputed into c's register and copied back every iteration)
__device__ __forceinline__ float fma_keep(float a, float b, float c) {
  asm("v_fma_f32 %0, %1, %0, %2" : "+v"(a) : "v"(b), "v"(c));
  return a;
}
__device__ __forceinline__ double fma_keep(double a, double b, double c) {
  asm("v_fma_f64 %0, %1, %0, %2" : "+v"(a) : "v"(b), "v"(c));
  return a;
}

// y = K v for the four nodes of the owned block.  pb points at the padded
// entry of node (i0-1, j0-1) of component x (component y follows at +PN);
// eb at the padded element (i0-1, j0-1).
template <int N1, int N2, typename V>
__device__ __forceinline__ void mv_block(const V* __restrict__ pb, const V* __restrict__ eb,
                                         const V (&kv)[10], V (&y)[4][2]) {
  using P = Pad<N1, N2>;
  V ux[4][4], uy[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      ux[c][a] = pb[c * P::PW + a];
      uy[c][a] = pb[P::PN + c * P::PW + a];
    }
  V se[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) se[c][a] = eb[c * P::PW + a];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int di = k & 1, dj = k >> 1;
    V acc0 = V(0), acc1 = V(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ea = elem_ea(di, q), ec = elem_ec(dj, q), cc = elem_cc(q);
      V t0 = V(0), t1 = V(0);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const V vx = ux[ec + cyo(m)][ea + cxo(m)];
        const V vy = uy[ec + cyo(m)][ea + cxo(m)];
        t0 = kfma(kv, 2 * cc, 2 * m, vx, t0);
        t0 = kfma(kv, 2 * cc, 2 * m + 1, vy, t0);
        t1 = kfma(kv, 2 * cc + 1, 2 * m, vx, t1);
        t1 = kfma(kv, 2 * cc + 1, 2 * m + 1, vy, t1);
      }
      acc0 = fma(se[ec][ea], t0, acc0);
      acc1 = fma(se[ec][ea], t1, acc1);
    }
    y[k][0] = acc0;
    y[k][1] = acc1;
  }
}

// Block-major vectors of the even-size operator: block (I, J) holds its
// nodes (2I + a, 2J + c) at [4 * (J * NB1 + I) + a + 2c], one array per
// component; periodic neighbours are plain block indices, no halo.
template <typename V>
__device__ __forceinline__ void ld4(const V* p, V (&o)[4]) {
  if constexpr (sizeof(V) == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    o[0] = t.x, o[1] = t.y, o[2] = t.z, o[3] = t.w;
  } else {
    const double2 t0 = reinterpret_cast<const double2*>(p)[0], t1 = reinterpret_cast<const double2*>(p)[1];
    o[0] = t0.x, o[1] = t0.y, o[2] = t1.x, o[3] = t1.y;
  }
}
template <typename V>
__device__ __forceinline__ void st4(V* p, V a0, V a1, V a2, V a3) {
  if constexpr (sizeof(V) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(a0, a1, a2, a3);
  } else {
    reinterpret_cast<double2*>(p)[0] = make_double2(a0, a1);
    reinterpret_cast<double2*>(p)[1] = make_double2(a2, a3);
  }
}

// y = K v at the four owned nodes (even sizes), element by element through
// the mode form of the box-element stiffness: per element the projections of
// (v_x, v_y) on the corner patterns bx, by, g (from the edge differences of
// the patch) give six generalized forces G1..G6 (mode constants mc, element
// scale m), which go back to the corners as f_x = bx G1 + by G3 + g G5,
// f_y = bx G4 + by G2 + g G6.  The thread's 2x2 elements cover its 3x3 node
// patch; the partial sums of the five patch nodes owned by the right, top
// and diagonal neighbours pass through LDS (three lane-contiguous quad slots
// [3][WG][4], one barrier).  vb: block-major vector (component x, y at
// +NBT*4); es: scales of the elements (i0 + a, j0 + c) as es[c][a];
// blk/br/bt/bd: own, right,
// top and top-right blocks; tl, tb, td: threads owning the blocks to the
// left, below and below-left.
template <int N1, int N2, int WG, typename V>
__device__ __forceinline__ void mv_modes_post(const V* __restrict__ vb, const V (&es)[2][2], const V (&mc)[10],
                                              V* __restrict__ sx, int blk, int br, int bt, int bd, int tid,
                                              V (&own)[2][2][2]) {
  constexpr int NBT = (N1 / 2) * (N2 / 2);
  V ux[3][3], uy[3][3];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    V(&u)[3][3] = d ? uy : ux;
    const V* v = vb + d * NBT * 4;
    V q[4], r[4], t[4], g[4];   // 16-byte reads: lane-contiguous, no bank conflicts
    ld4(v + 4 * blk, q);
    ld4(v + 4 * br, r);
    ld4(v + 4 * bt, t);
    ld4(v + 4 * bd, g);
    u[0][0] = q[0], u[0][1] = q[1], u[1][0] = q[2], u[1][1] = q[3];
    u[0][2] = r[0], u[1][2] = r[2];
    u[2][0] = t[0], u[2][1] = t[1];
    u[2][2] = g[0];
  }
  V hx[3][2], hy[3][2], vx[2][3], vy[2][3];   // horizontal / vertical edge differences
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      hx[c][a] = ux[c][a + 1] - ux[c][a];
      hy[c][a] = uy[c][a + 1] - uy[c][a];
    }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vx[c][a] = ux[c + 1][a] - ux[c][a];
      vy[c][a] = uy[c + 1][a] - uy[c][a];
    }
  V fx[3][3], fy[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) fx[c][a] = fy[c][a] = V(0);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const V m = es[c][a];
      const V mX = m * (hx[c][a] + hx[c + 1][a]);   // m bx.ux
      const V mY = m * (vy[c][a] + vy[c][a + 1]);   // m by.uy
      const V mSx = m * (vx[c][a] + vx[c][a + 1]);  // m by.ux
      const V mSy = m * (hy[c][a] + hy[c + 1][a]);  // m bx.uy
      const V G1 = fma(mc[0], mX, mc[1] * mY);
      const V G2 = fma(mc[2], mX, mc[3] * mY);
      const V G3 = fma(mc[4], mSx, mc[5] * mSy);
      const V G4 = fma(mc[6], mSx, mc[7] * mSy);
      const V G5 = mc[8] * (m * (hx[c + 1][a] - hx[c][a]));   // g.ux
      const V G6 = mc[9] * (m * (vy[c][a + 1] - vy[c][a]));   // g.uy
      const V P1 = G1 + G3, Q1 = G1 - G3, P2 = G4 + G2, Q2 = G4 - G2;
      fx[c][a] += G5 - P1;
      fx[c][a + 1] += Q1 - G5;
      fx[c + 1][a + 1] += P1 + G5;
      fx[c + 1][a] -= Q1 + G5;
      fy[c][a] += G6 - P2;
      fy[c][a + 1] += Q2 - G6;
      fy[c + 1][a + 1] += P2 + G6;
      fy[c + 1][a] -= Q2 + G6;
    }
  // slot 0: nodes (i0+2, j0), (i0+2, j0+1) -> right neighbour's (0, 0), (0, 1)
  // slot 1: nodes (i0, j0+2), (i0+1, j0+2) -> top neighbour's (0, 0), (1, 0)
  // slot 2: node (i0+2, j0+2)              -> diagonal neighbour's (0, 0)
  st4(sx + 4 * (0 * WG + tid), fx[0][2], fy[0][2], fx[1][2], fy[1][2]);
  st4(sx + 4 * (1 * WG + tid), fx[2][0], fy[2][0], fx[2][1], fy[2][1]);
  st4(sx + 4 * (2 * WG + tid), fx[2][2], fy[2][2], V(0), V(0));
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      own[c][a][0] = fx[c][a];
      own[c][a][1] = fy[c][a];
    }
}

// Second half after the work-group barrier: add the neighbours' partial sums.
template <int WG, typename V>
__device__ __forceinline__ void mv_modes_gather(const V* __restrict__ sx, const V (&own)[2][2][2], int tl, int tb,
                                                int td, V (&y)[4][2]) {
  V gl[4], gb[4], gd[4];
  ld4(sx + 4 * (0 * WG + tl), gl);
  ld4(sx + 4 * (1 * WG + tb), gb);
  ld4(sx + 4 * (2 * WG + td), gd);
  y[0][0] = own[0][0][0] + gl[0] + gb[0] + gd[0];
  y[0][1] = own[0][0][1] + gl[1] + gb[1] + gd[1];
  y[1][0] = own[0][1][0] + gb[2];
  y[1][1] = own[0][1][1] + gb[3];
  y[2][0] = own[1][0][0] + gl[2];
  y[2][1] = own[1][0][1] + gl[3];
  y[3][0] = own[1][1][0];
  y[3][1] = own[1][1][1];
}

// y = K v at the four owned nodes, exchange barrier included.
template <int N1, int N2, int WG, typename V>
__device__ __forceinline__ void mv_modes(const V* __restrict__ vb, const V (&es)[2][2], const V (&mc)[10],
                                         V* __restrict__ sx, int blk, int br, int bt, int bd, int tid, int tl, int tb,
                                         int td, V (&y)[4][2]) {
  V own[2][2][2];
  mv_modes_post<N1, N2, WG, V>(vb, es, mc, sx, blk, br, bt, bd, tid, own);
  __syncthreads();
  mv_modes_gather<WG, V>(sx, own, tl, tb, td, y);
}

// y = K v (FP64) at one owned node (di, dj) of the block, element by
// element; used by the FP64 passes (residuals, assembly, condensation),
// which run a few times per column.  The empty asm after each element
// consumes its contribution and keeps the next element's loads behind it,
// so only one element's corner values are live (the FP64 window of the
// whole block would otherwise set the kernel's register budget).
template <int N1, int N2>
__device__ __forceinline__ void mv_node64(const double* __restrict__ pb, const double* __restrict__ eb,
                                          const double (&kv)[10], int di, int dj, double (&y)[2]) {
  using P = Pad<N1, N2>;
  y[0] = y[1] = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ea = elem_ea(di, q), ec = elem_ec(dj, q), cc = elem_cc(q);
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int o = (ec + cyo(m)) * P::PW + ea + cxo(m);
      const double vx = pb[o], vy = pb[P::PN + o];
      t0 = kfma(kv, 2 * cc, 2 * m, vx, t0);
      t0 = kfma(kv, 2 * cc, 2 * m + 1, vy, t0);
      t1 = kfma(kv, 2 * cc + 1, 2 * m, vx, t1);
      t1 = kfma(kv, 2 * cc + 1, 2 * m + 1, vy, t1);
    }
    const double sc = eb[ec * P::PW + ea];
    y[0] = fma(sc, t0, y[0]);
    y[1] = fma(sc, t1, y[1]);
    asm volatile("" : "+v"(y[0]), "+v"(y[1]) : : "memory");
  }
}

template <int N1, int N2>
__device__ __forceinline__ double elem_scale(const double* __restrict__ eb, int di, int dj, int q) {
  return eb[elem_ec(dj, q) * Pad<N1, N2>::PW + elem_ea(di, q)];
}

// Column j of K_wF at owned node (di, dj), component d; KwF is the uniform
// [8][NF] element table in global memory (read through scalar loads).
template <int N1, int N2>
__device__ __forceinline__ double bF_entry(const double* __restrict__ eb, const double* __restrict__ KwF,
                                           int di, int dj, int d, int j) {
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) s += elem_scale<N1, N2>(eb, di, dj, q) * KwF[(2 * elem_cc(q) + d) * NF + j];
  return s;
}

}  // namespace

// ---------------------------------------------------------------------------
// Spectral preconditioner of the homogeneous reference medium
// ---------------------------------------------------------------------------
// Every element of a resolution class has stiffness mu_e K_ref, so the
// periodic operator of a uniform medium (mu = 1) is block-circulant and the
// Fourier transform diagonalises it into a real symmetric 2x2 symbol S(k).
// M^-1 r = R K_0^+ R^T r (R drops the pinned corner, K_0^+ the inverse on
// the non-constant modes) is applied in three steps on one complex field
// z = r_x + i r_y of N x N nodes in LDS:
//   * forward DFT by vector-radix 2x2 decimation in frequency (in place,
//     one 2x2 butterfly group per thread and stage, output in bit-reversed
//     order along both axes);
//   * per bit-reversed position: W(k) = alpha(k) Z(k) + beta(k) conj Z(-k),
//     the symbol inverse [a b; b c] applied to the two real fields packed in
//     Z (alpha = (a + c)/2, beta = (a - c)/2 + i b; alpha = beta = 0 at k = 0);
//   * inverse DFT by vector-radix 2x2 decimation in time (bit-reversed in,
//     natural order out, unscaled: PCG is invariant to the preconditioner's
//     scale), whose last stage writes u_x, u_y into the block-major search
//     direction directly.
// Table tab (per class): [N*N][4] (alpha, Re beta, Im beta, 0) by position
// q*N + p, then [N/2][2] twiddles (cos, -sin)(2 pi t / N).
template <typename TI>
struct Cx {
  TI re, im;
};
template <typename TI>
__device__ __forceinline__ Cx<TI> cadd(Cx<TI> a, Cx<TI> b) { return {a.re + b.re, a.im + b.im}; }
template <typename TI>
__device__ __forceinline__ Cx<TI> csub(Cx<TI> a, Cx<TI> b) { return {a.re - b.re, a.im - b.im}; }
template <typename TI>
__device__ __forceinline__ Cx<TI> cmul(Cx<TI> a, Cx<TI> w) {
  return {a.re * w.re - a.im * w.im, a.re * w.im + a.im * w.re};
}
template <typename TI>
__device__ __forceinline__ Cx<TI> cmulc(Cx<TI> a, Cx<TI> w) {   // a * conj(w)
  return {a.re * w.re + a.im * w.im, a.im * w.re - a.re * w.im};
}
template <typename TI>
__device__ __forceinline__ Cx<TI> zld(const TI* z, int i, int j, int n) {
  const TI* q = z + 2 * (j * n + i);
  return {q[0], q[1]};
}
template <typename TI>
__device__ __forceinline__ void zst(TI* z, int i, int j, int n, Cx<TI> v) {
  TI* q = z + 2 * (j * n + i);
  q[0] = v.re;
  q[1] = v.im;
}
__device__ __forceinline__ int bitrev(int x, int m) { return static_cast<int>(__brev(static_cast<unsigned>(x)) >> (32 - m)); }

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

// Per-thread constants of the preconditioner, loaded once per RVE: the
// symbol coefficients of the thread's four positions, and pointers to the
// LDS tables (twiddles, partner positions).
template <int N, typename TI>
struct SpectralRegs {
  static constexpr int M = (N == 8) ? 3 : (N == 16 || N == 48) ? 4 : 5;   // log2 of the radix-2 extent
  static_assert((1 << M) == N || (N == 48 && (3 << M) == N), "spectral preconditioner: N must be 8, 16, 32 or 48");
  static constexpr bool HOLD = N != 48;   // symbol coefficients in registers (N = 48: read at use)
  const TI* tw;              // LDS copy of the twiddles
  const unsigned char* pm;   // LDS: position of -k along one axis, per position
  const TI* tab;             // the class table (N = 48)
  TI al[HOLD ? 4 : 1], br[HOLD ? 4 : 1], bi[HOLD ? 4 : 1];
};

// Position that holds the frequency -k when position p holds k (along one
// axis): bit reversal for powers of two; for N = 48, sub-block s = p / 16
// holds the frequencies s + 3 k, k bit-reversed within the block.
template <int N>
__device__ __forceinline__ int spectral_partner(int p) {
  constexpr int M = (N == 8) ? 3 : (N == 16 || N == 48) ? 4 : 5;
  if constexpr (N == 48) {
    const int k = 3 * bitrev(p % 16, M) + p / 16;
    const int n = (N - k) % N;
    return 16 * (n % 3) + bitrev(n / 3, M);
  } else {
    return bitrev((N - bitrev(p, M)) & (N - 1), M);
  }
}

// s_tw: LDS table [t][2] of twiddles followed by the partner map [N] bytes,
// filled here (visible after the caller's next barrier).
template <int N, typename TI>
__device__ __forceinline__ void spectral_setup(SpectralRegs<N, TI>& g, const TI* __restrict__ tab, TI* s_tw, bool own,
                                               int I, int J) {
  constexpr int T = lin2d_spectral_twiddles(N);
  const TI* tw = tab + 4 * N * N;
  if (threadIdx.x < 2 * T) s_tw[threadIdx.x] = tw[threadIdx.x];
  unsigned char* pm = reinterpret_cast<unsigned char*>(s_tw + 2 * T);
  if (threadIdx.x < N) pm[threadIdx.x] = static_cast<unsigned char>(spectral_partner<N>(threadIdx.x));
  g.tw = s_tw;
  g.pm = pm;
  g.tab = tab;
  if constexpr (SpectralRegs<N, TI>::HOLD)
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int p = own ? 2 * I + (k & 1) : 0, q = own ? 2 * J + (k >> 1) : 0;
    const TI* t = tab + 4 * (q * N + p);
    g.al[k] = t[0];
    g.br[k] = t[1];
    g.bi[k] = t[2];
  }
}

// Work-group layout of the spectral instantiations: every wave owns a tile
// of TW x TW blocks (2TW x 2TW nodes), so the transform stages whose
// butterflies stay inside one such window (h <= TW) exchange data within a
// wave and need no work-group barrier.  Blocks are stored in the same order
// (storage index of block (I, J) = its owner's thread id): the four-node
// reads of a wave are contiguous.
template <int NB>
struct Tiles {
  static constexpr int TW = NB < 8 ? NB : 8;
  static constexpr int NT = NB / TW;
  static_assert(NB % TW == 0, "block grid not a multiple of the wave tile");
  static __host__ __device__ constexpr int bix(int I, int J) {
    return ((J / TW) * NT + I / TW) * (TW * TW) + (J % TW) * TW + I % TW;
  }
  static __device__ __forceinline__ int I_of(int t) { return ((t / (TW * TW)) % NT) * TW + t % TW; }
  static __device__ __forceinline__ int J_of(int t) { return ((t / (TW * TW)) / NT) * TW + (t % (TW * TW)) / TW; }
};

// LDS writes of this wave visible to its other lanes (no work-group barrier)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work-group sum of per-lane partials split around a barrier that the
// caller places (so that it can share it): wsum_post writes the wave totals
// into one of the two alternating reduction buffers, wsum_collect adds them
// after the barrier.
template <int NW, typename TI>
__device__ __forceinline__ TI wsum_collect(const TI* buf) {
  TI t = TI(0);
#pragma unroll
  for (int w = 0; w < NW; ++w) t += buf[w];
  return t;
}

// Radix-2 x 2 butterfly group at distance H of the thread with block
// coordinates (I, J): points (i, j), (i + H, j), (i, j + H), (i + H, j + H)
// with i = I + (I & ~(H - 1)) (the (I / H) * 2H + I mod H of an in-place
// transform), j likewise; twiddle index (I mod H) * TS along x, (J mod H) *
// TS along y.  DIF forward (INV = false) or DIT inverse with conjugate
// twiddles (INV = true); in place.  One base address per call, the four
// points at constant offsets.
template <int N, int H, int TS, bool INV, typename TI>
__device__ __forceinline__ void vr2(TI* __restrict__ z, const TI* __restrict__ tw, unsigned I, unsigned J) {
  const unsigned i = I + (I & ~(H - 1u)), j = J + (J & ~(H - 1u));
  TI* zb = z + 2 * (j * N + i);
  const TI* tx = tw + 2 * ((I & (H - 1u)) * TS);
  const TI* ty = tw + 2 * ((J & (H - 1u)) * TS);
  const Cx<TI> wx = {tx[0], tx[1]}, wy = {ty[0], ty[1]};
  constexpr int DX = 2 * H, DY = 2 * H * N;
  const Cx<TI> a0 = {zb[0], zb[1]}, b0 = {zb[DX], zb[DX + 1]};
  const Cx<TI> c0 = {zb[DY], zb[DY + 1]}, d0 = {zb[DX + DY], zb[DX + DY + 1]};
  Cx<TI> o00, o10, o01, o11;
  if constexpr (!INV) {
    const Cx<TI> A = cadd(a0, b0), B = cmul(csub(a0, b0), wx), C = cadd(c0, d0), D = cmul(csub(c0, d0), wx);
    o00 = cadd(A, C);
    o01 = cmul(csub(A, C), wy);
    o10 = cadd(B, D);
    o11 = cmul(csub(B, D), wy);
  } else {
    const Cx<TI> b = cmulc(b0, wx), d = cmulc(d0, wx);
    const Cx<TI> A = cadd(a0, b), B = csub(a0, b), C = cmulc(cadd(c0, d), wy), D = cmulc(csub(c0, d), wy);
    o00 = cadd(A, C);
    o10 = cadd(B, D);
    o01 = csub(A, C);
    o11 = csub(B, D);
  }
  zb[0] = o00.re, zb[1] = o00.im;
  zb[DX] = o10.re, zb[DX + 1] = o10.im;
  zb[DY] = o01.re, zb[DY + 1] = o01.im;
  zb[DX + DY] = o11.re, zb[DX + DY + 1] = o11.im;
}

// Block-major position of node (x, y) in the search direction.
template <int N>
__host__ __device__ constexpr int sp_at(int x, int y) {
  return 4 * Tiles<N / 2>::bix(x >> 1, y >> 1) + (x & 1) + 2 * (y & 1);
}

// The owned block's four points (2I + a, 2J + c) of a complex field: base
// pointer (a = c = 0), the others at +2 and +2N.
template <int N, typename TI>
__device__ __forceinline__ TI* own_pts(TI* z, unsigned I, unsigned J) {
  return z + 4 * (J * N + I);
}

// Last forward stage (h = 1, unit twiddles) on the owned block: v and z
// at the owned positions.  The caller's barrier then makes z readable for
// the symbol's partner reads (spectral_symbol).
template <int N, typename TI>
__device__ __forceinline__ void spectral_fwd1(Cx<TI> (&v)[4], TI* __restrict__ z, unsigned I, unsigned J) {
  TI* zo = own_pts<N>(z, I, J);
  // h = 1 (unit twiddles) on the owned block
  {
    const Cx<TI> a = {zo[0], zo[1]}, b = {zo[2], zo[3]};
    const Cx<TI> c = {zo[2 * N], zo[2 * N + 1]}, d = {zo[2 * N + 2], zo[2 * N + 3]};
    const Cx<TI> A = cadd(a, b), B = csub(a, b), C = cadd(c, d), D = csub(c, d);
    v[0] = cadd(A, C);
    v[2] = csub(A, C);
    v[1] = cadd(B, D);
    v[3] = csub(B, D);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) zo[(k & 1) * 2 + (k >> 1) * 2 * N] = v[k].re, zo[(k & 1) * 2 + (k >> 1) * 2 * N + 1] = v[k].im;
}

// The symbol at the owned positions: W = alpha Z + beta conj Z(-k).  Shared
// by every size (the transform stages differ: radix-2 only, or radix-3
// first for N = 48).
template <int N, typename TI>
__device__ __forceinline__ void spectral_symbol(Cx<TI> (&v)[4], const TI* __restrict__ z, const SpectralRegs<N, TI>& g,
                                                unsigned I, unsigned J) {
  // partner positions of the owned block from the LDS map (one 16-bit read
  // per axis: the entries of 2I and 2I + 1)
  const unsigned px = *reinterpret_cast<const unsigned short*>(g.pm + 2 * I);
  const unsigned py = *reinterpret_cast<const unsigned short*>(g.pm + 2 * J);
  const unsigned ppx[2] = {px & 0xffu, px >> 8}, ppy[2] = {py & 0xffu, py >> 8};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const TI* zp = z + 2 * (ppy[k >> 1] * N + ppx[k & 1]);
    const TI zr = zp[0], zi = zp[1];
    TI al, br, bi;
    if constexpr (SpectralRegs<N, TI>::HOLD) {
      al = g.al[k], br = g.br[k], bi = g.bi[k];
    } else {
      const TI* t = g.tab + 4 * ((2 * J + (k >> 1)) * N + 2 * I + (k & 1));
      al = t[0], br = t[1], bi = t[2];
    }
    // alpha Z + beta conj(Zp)
    v[k] = {al * v[k].re + br * zr + bi * zi, al * v[k].im + bi * zr - br * zi};
  }
}

// Inverse h = 1 of the owned block into z2.
template <int N, typename TI>
__device__ __forceinline__ void spectral_inv1(const Cx<TI> (&v)[4], TI* __restrict__ z2, unsigned I, unsigned J) {
  TI* zo = own_pts<N>(z2, I, J);
  const Cx<TI> A = cadd(v[0], v[1]), B = csub(v[0], v[1]), C = cadd(v[2], v[3]), D = csub(v[2], v[3]);
  const Cx<TI> o[4] = {cadd(A, C), cadd(B, D), csub(A, C), csub(B, D)};   // (0,0) (1,0) (0,1) (1,1)
#pragma unroll
  for (int k = 0; k < 4; ++k) zo[(k & 1) * 2 + (k >> 1) * 2 * N] = o[k].re, zo[(k & 1) * 2 + (k >> 1) * 2 * N + 1] = o[k].im;
}

template <int N, typename TI, int S>
__device__ __forceinline__ void fwd_stages(TI* z, const TI* tw, bool own, unsigned I, unsigned J) {
  // forward radix-2 stages h = N/2 .. 2 (S = stage index), powers of two
  constexpr int M = ilog2c(N);
  if constexpr (S < M - 1) {
    constexpr int H = N >> (S + 1);
    constexpr int TW = Tiles<N / 2>::TW;
    if (own) vr2<N, H, N / (2 * H), false, TI>(z, tw, I, J);
    if constexpr (H > TW) __syncthreads();
    else wave_sync();
    fwd_stages<N, TI, S + 1>(z, tw, own, I, J);
  }
}
template <int N, typename TI, int S>
__device__ __forceinline__ void inv_stages(TI* z2, const TI* tw, bool own, unsigned I, unsigned J) {
  // inverse radix-2 stages h = 2 .. N/4 (the last, h = N/2, writes the
  // search direction and is done by the caller); S counts down
  constexpr int TW = Tiles<N / 2>::TW;
  if constexpr (S >= 1) {
    constexpr int H = N >> (S + 1);
    if constexpr (H > TW) __syncthreads();
    else wave_sync();
    if (own) vr2<N, H, N / (2 * H), true, TI>(z2, tw, I, J);
    inv_stages<N, TI, S - 1>(z2, tw, own, I, J);
  }
}

// u = M^-1 r for the owned 2x2 block (I, J) (every thread of the work-group
// must call it: it holds barriers; all threads own a block for N >= 16,
// the first 16 for N = 8).  r: inner residual of the owned nodes, pinned
// node masked by the caller; z, z2: two complex LDS buffers [N*N][2]
// (forward transform in z, inverse in z2, so the symbol's partner reads
// need no barrier behind them); sp: block-major search direction (x at 0,
// y at +N*N), written with u (pinned node zero).  Ends without a barrier:
// the caller's next barrier makes sp visible.
template <int N, typename TI>
__device__ __forceinline__ void spectral_precond(const TI (&r)[4][2], TI* __restrict__ z, TI* __restrict__ z2,
                                                 TI* __restrict__ sp, const SpectralRegs<N, TI>& g, bool own, int Ii,
                                                 int Ji) {
  constexpr int M = SpectralRegs<N, TI>::M;
  constexpr int H = N / 2;   // last inverse stage
  constexpr int TW = Tiles<N / 2>::TW;
  // I and J opaque per call: the stage addresses (integer arithmetic on
  // them) are formed here rather than hoisted out of the PCG loop, where
  // they would hold some forty registers across the whole solve
  asm volatile("" : "+v"(Ii), "+v"(Ji));
  const unsigned I = static_cast<unsigned>(Ii), J = static_cast<unsigned>(Ji);
  if (own) {
    TI* zo = own_pts<N>(z, I, J);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      zo[(k & 1) * 2 + (k >> 1) * 2 * N] = r[k][0], zo[(k & 1) * 2 + (k >> 1) * 2 * N + 1] = r[k][1];
  }
  __syncthreads();
  // forward: decimation in frequency; a stage that combines points of
  // different wave windows (h > TW) is followed by a work-group barrier, the
  // others by a wave sync
  fwd_stages<N, TI, 0>(z, g.tw, own, I, J);
  Cx<TI> v[4];
  if (own) spectral_fwd1<N, TI>(v, z, I, J);
  __syncthreads();
  if (own) {
    spectral_symbol<N, TI>(v, z, g, I, J);
    spectral_inv1<N, TI>(v, z2, I, J);
  }
  inv_stages<N, TI, M - 2>(z2, g.tw, own, I, J);
  if constexpr (H > TW) __syncthreads();
  else wave_sync();
  if (own) {   // last inverse stage, h = N/2: i = I, j = J, output into the search direction
    TI* zb = z2 + 2 * (J * N + I);
    const TI* tx = g.tw + 2 * I;
    const TI* ty = g.tw + 2 * J;
    const Cx<TI> wx = {tx[0], tx[1]}, wy = {ty[0], ty[1]};
    constexpr int DX = 2 * H, DY = 2 * H * N;
    const Cx<TI> a = {zb[0], zb[1]}, b = cmulc(Cx<TI>{zb[DX], zb[DX + 1]}, wx);
    const Cx<TI> c = {zb[DY], zb[DY + 1]}, d = cmulc(Cx<TI>{zb[DX + DY], zb[DX + DY + 1]}, wx);
    const Cx<TI> A = cadd(a, b), B = csub(a, b), C = cmulc(cadd(c, d), wy), D = cmulc(csub(c, d), wy);
    const Cx<TI> o00 = cadd(A, C), o10 = cadd(B, D), o01 = csub(A, C), o11 = csub(B, D);
    // node (x, y) -> block-major slot; +H along x or y is a constant offset
    TI* sb = sp + 4 * Tiles<N / 2>::bix(I >> 1, J >> 1) + (I & 1) + 2 * (J & 1);
    constexpr int OX = sp_at<N>(H, 0) - sp_at<N>(0, 0), OY = sp_at<N>(0, H) - sp_at<N>(0, 0);
    const bool pin = (I | J) == 0;
    sb[0] = pin ? TI(0) : o00.re;
    sb[N * N] = pin ? TI(0) : o00.im;
    sb[OX] = o10.re, sb[N * N + OX] = o10.im;
    sb[OY] = o01.re, sb[N * N + OY] = o01.im;
    sb[OX + OY] = o11.re, sb[N * N + OX + OY] = o11.im;
  }
}

// N = 48 = 3 x 16: the forward transform starts with a radix-3 x 3 stage
// (one group of nine points (x + 16a, y + 16b), x, y < 16, per lane for the
// first 256 lanes: the 3 x 3 DFT, then the twiddles W48^(x mx) W48^(y my)),
// which leaves the nine residue classes of the frequency mod 3 in the nine
// 16 x 16 sub-blocks; vector-radix 2 x 2 stages inside every sub-block
// follow, each sub-block on the wave that owns its 8 x 8 blocks (no
// work-group barriers).  Sub-block s holds frequencies s + 3 k, k
// bit-reversed within the block.  The inverse mirrors it: radix-2 stages by
// decimation in time (in z2), then the radix-3 combination, which writes the
// search direction.  Twiddle table: W48^t, t < 32.
template <typename TI>
__device__ __forceinline__ void spectral_precond48(const TI (&r)[4][2], TI* __restrict__ z, TI* __restrict__ z2,
                                                   TI* __restrict__ sp, const SpectralRegs<48, TI>& g, bool own,
                                                   int Ii, int Ji) {
  constexpr int N = 48, NS = 16;
  asm volatile("" : "+v"(Ii), "+v"(Ji));
  const unsigned I = static_cast<unsigned>(Ii), J = static_cast<unsigned>(Ji);
  const int tid = threadIdx.x;
  const TI c3 = TI(-0.5), s3 = TI(0.86602540378443864676);   // W3 = c3 - i s3
  auto w48 = [&](int t) -> Cx<TI> { return {g.tw[2 * t], g.tw[2 * t + 1]}; };
  // 3-point DFT of (v0, v1, v2): out_m = sum_a v_a W3^(a m)
  auto dft3 = [&](Cx<TI> v0, Cx<TI> v1, Cx<TI> v2, Cx<TI>* o, bool inverse) {
    const Cx<TI> sum = cadd(v1, v2), dif = csub(v1, v2);
    const Cx<TI> base = {v0.re + c3 * sum.re, v0.im + c3 * sum.im};
    // W3^m (v1) + W3^2m (v2): the +-i s3 (v1 - v2) part, sign by direction
    const TI sg = inverse ? TI(-1) : TI(1);
    const Cx<TI> rot = {sg * s3 * dif.im, -sg * s3 * dif.re};
    o[0] = cadd(v0, sum);
    o[1] = cadd(base, rot);
    o[2] = csub(base, rot);
  };
  (void)own;
  {
    TI* zo = own_pts<N>(z, I, J);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      zo[(k & 1) * 2 + (k >> 1) * 2 * N] = r[k][0], zo[(k & 1) * 2 + (k >> 1) * 2 * N + 1] = r[k][1];
  }
  __syncthreads();
  if (tid < NS * NS) {   // radix-3 x 3, forward: the lane's nine points, in place, one axis at a time
    const int x = tid % NS, y = tid / NS;
#pragma unroll 1
    for (int b = 0; b < 3; ++b) {   // along x
      Cx<TI> o[3];
      dft3(zld<TI>(z, x, y + NS * b, N), zld<TI>(z, x + NS, y + NS * b, N), zld<TI>(z, x + 2 * NS, y + NS * b, N), o,
           false);
#pragma unroll
      for (int mx = 0; mx < 3; ++mx) zst<TI>(z, x + NS * mx, y + NS * b, N, o[mx]);
    }
#pragma unroll 1
    for (int mx = 0; mx < 3; ++mx) {   // along y, then the twiddles
      Cx<TI> o[3];
      dft3(zld<TI>(z, x + NS * mx, y, N), zld<TI>(z, x + NS * mx, y + NS, N), zld<TI>(z, x + NS * mx, y + 2 * NS, N), o,
           false);
#pragma unroll
      for (int my = 0; my < 3; ++my) zst<TI>(z, x + NS * mx, y + NS * my, N, cmul(o[my], cmul(w48(x * mx), w48(y * my))));
    }
  }
  __syncthreads();
  // radix-2 x 2 DIF, h = 8, 4, 2 inside the sub-block (one wave); twiddle
  // W16^(t) = W48^(3t): index step 3 * 16 / (2h)
  // (every lane owns a block: 24 x 24 blocks on 576 lanes)
  vr2<N, 8, 3, false, TI>(z, g.tw, I, J);
  wave_sync();
  vr2<N, 4, 6, false, TI>(z, g.tw, I, J);
  wave_sync();
  vr2<N, 2, 12, false, TI>(z, g.tw, I, J);
  wave_sync();
  Cx<TI> v[4];
  spectral_fwd1<N, TI>(v, z, I, J);
  __syncthreads();
  spectral_symbol<N, TI>(v, z, g, I, J);
  spectral_inv1<N, TI>(v, z2, I, J);
  wave_sync();
  vr2<N, 2, 12, true, TI>(z2, g.tw, I, J);
  wave_sync();
  vr2<N, 4, 6, true, TI>(z2, g.tw, I, J);
  wave_sync();
  vr2<N, 8, 3, true, TI>(z2, g.tw, I, J);
  __syncthreads();
  if (tid < NS * NS) {   // radix-3 x 3 combination (inverse), in place along x, then along y into sp
    const int x = tid % NS, y = tid / NS;
#pragma unroll 1
    for (int my = 0; my < 3; ++my) {
      Cx<TI> vv[3], o[3];
#pragma unroll
      for (int mx = 0; mx < 3; ++mx)
        vv[mx] = cmulc(zld<TI>(z2, x + NS * mx, y + NS * my, N), cmul(w48(x * mx), w48(y * my)));
      dft3(vv[0], vv[1], vv[2], o, true);
#pragma unroll
      for (int a = 0; a < 3; ++a) zst<TI>(z2, x + NS * a, y + NS * my, N, o[a]);
    }
#pragma unroll 1
    for (int a = 0; a < 3; ++a) {
      Cx<TI> o[3];
      dft3(zld<TI>(z2, x + NS * a, y, N), zld<TI>(z2, x + NS * a, y + NS, N), zld<TI>(z2, x + NS * a, y + 2 * NS, N),
           o, true);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int xx = x + NS * a, yy = y + NS * b;
        const int at = sp_at<N>(xx, yy);
        const bool pin = (xx | yy) == 0;
        sp[at] = pin ? TI(0) : o[b].re;
        sp[N * N + at] = pin ? TI(0) : o[b].im;
      }
    }
  }
}

// LDS layout: reduction buffers | element scales FP64 [PN] | FP32 [PN] |
// one search direction [2][PN] in TI aliased with the FP64 staging [2][PN] |
// exchange slots of the element-wise operator [3][WG][4] in TI (even sizes;
// the spectral preconditioner's two complex fields [2][N*N][2] alias them,
// the region growing to hold both) | twiddle table [n/2][2] in TI (spectral
// preconditioner).
constexpr int RED_NV = 2 * NF > 5 ? 2 * NF : 5;   // widest work-group reduction
template <int NW, typename TI>
__device__ __forceinline__ const TI* wsum_post(TI v, double* s_red, int& parity) {
  TI* buf = reinterpret_cast<TI*>(s_red + parity * (NW * RED_NV));
  parity ^= 1;
  if constexpr (sizeof(TI) == 4) {
    const float w = wave_sum_to_last(v);
    if ((threadIdx.x & 63) == 63) buf[threadIdx.x >> 6] = w;
  } else {
    const double w = wave_sum(v);
    if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = w;
  }
  return buf;
}
__host__ __device__ constexpr size_t lin2d_red_doubles(int nw, int nrhs) {
  return 2 * static_cast<size_t>(nw) * RED_NV + 0 * nrhs;
}
__host__ __device__ constexpr size_t lin2d_vec_offset(int n1, int n2, int wg, int nrhs) {
  return ((lin2d_red_doubles(wg / 64, nrhs) * 8 + static_cast<size_t>(pad_w(n1)) * pad_w(n2) * 12) + 15) &
         ~static_cast<size_t>(15);
}
__host__ __device__ constexpr size_t lin2d_xch_offset(int n1, int n2, int wg, int nrhs) {
  return lin2d_vec_offset(n1, n2, wg, nrhs) + 2 * static_cast<size_t>(pad_w(n1)) * pad_w(n2) * 8;
}
// exchange region in elements of the inner precision
__host__ __device__ constexpr size_t lin2d_xch_len(int n1, int n2, int wg, bool spectral) {
  return spectral && 4 * static_cast<size_t>(n1) * n2 > 12 * static_cast<size_t>(wg) ? 4 * static_cast<size_t>(n1) * n2
                                                                                     : 12 * static_cast<size_t>(wg);
}
__host__ __device__ constexpr size_t lin2d_lds_bytes_t(int n1, int n2, int wg, int nrhs, int ti_bytes,
                                                       bool spectral = false) {
  return lin2d_xch_offset(n1, n2, wg, nrhs) +
         (((n1 | n2) & 1) == 0 && nrhs > 0 ? lin2d_xch_len(n1, n2, wg, spectral) * ti_bytes : 0) +
         (spectral ? 2 * static_cast<size_t>(lin2d_spectral_twiddles(n1)) * ti_bytes + n1 + 2 : 0);   // twiddles, partner map
}

// The spectral FP32 form is held to three work-groups of 256 lanes per CU
// (at most 168 VGPRs), the occupancy of the Jacobi form.
template <typename TI, bool FFT, int WG>
constexpr int kLin2dMinBlocks = (sizeof(TI) == 4 && FFT && WG == 256) ? 3 : (FFT && WG == 256) ? 2 : 1;

template <typename TI, int NRHS, int N1, int N2, int WG, bool FFT>
__global__ void __launch_bounds__(WG, (kLin2dMinBlocks<TI, FFT, WG>)) k_lin2d(const Lin2DArgs a) {
  using P = Pad<N1, N2>;
  constexpr int NW = WG / 64;
  constexpr int NN = N1 * N2;
  constexpr int NB1 = (N1 + 1) / 2, NB2 = (N2 + 1) / 2;
  static_assert(NB1 * NB2 <= WG, "work-group too small for the RVE");
  const int tid = threadIdx.x;
  const int b = a.rve_list[blockIdx.x];
  if (a.skip && a.skip[b]) return;   // handled elsewhere (whole work-group)

  extern __shared__ __align__(16) unsigned char smem[];
  double* s_red = reinterpret_cast<double*>(smem);
  double* s_sc = s_red + lin2d_red_doubles(NW, NRHS);                    // [PN] FP64
  float* s_sc32 = reinterpret_cast<float*>(s_sc + P::PN);                 // [PN] FP32
  unsigned char* s_vec = smem + lin2d_vec_offset(N1, N2, WG, NRHS);
  TI* s_p = reinterpret_cast<TI*>(s_vec);          // [2][PN] search direction
  double* s_st = reinterpret_cast<double*>(s_vec);  // [2][PN] FP64 staging (aliases s_p)
  TI* s_x = reinterpret_cast<TI*>(smem + lin2d_xch_offset(N1, N2, WG, NRHS));   // [3][WG][4] (even sizes)
  constexpr bool EVEN = ((N1 | N2) & 1) == 0;
  static_assert(!FFT || (EVEN && N1 == N2), "spectral preconditioner needs square power-of-two RVEs");
  const TI* ftab = nullptr;
  if constexpr (FFT) {
    if constexpr (sizeof(TI) == 4) ftab = reinterpret_cast<const TI*>(a.fft_tab);
    else ftab = reinterpret_cast<const TI*>(a.fft_tab64);
  }
  struct NoSpectral {};
  using SpecRegs = typename std::conditional<FFT, SpectralRegs<FFT ? N1 : 8, TI>, NoSpectral>::type;
  SpecRegs sreg;
  int parity = 0;

  // ---- reference element scalars (uniform: scalar registers) -------------
  double kv64[10];
  TI kvI[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) {
    kv64[t] = a.kv64[t];
    kvI[t] = static_cast<TI>(kv64[t]);
  }
  const double* KwF = a.KwF64;   // [8][NF], uniform
  TI mcI[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) mcI[t] = EVEN ? static_cast<TI>(a.modes64[t]) : TI(0);

  // ---- ownership of a 2x2 node block -------------------------------------
  // (spectral form: wave tiles of blocks, see Tiles; else row by row)
  const bool own = tid < NB1 * NB2;
  auto bix = [](int I_, int J_) {
    if constexpr (FFT) return Tiles<NB1>::bix(I_, J_);
    else return J_ * NB1 + I_;
  };
  int I = 0, J = 0;
  if (own) {
    if constexpr (FFT) {
      I = Tiles<NB1>::I_of(tid);
      J = Tiles<NB1>::J_of(tid);
    } else {
      I = tid % NB1;
      J = tid / NB1;
    }
  }
  const int i0 = 2 * I, j0 = 2 * J;
  bool exists[4], dof[4];
  int pidx[4];   // padded index of each owned node
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = i0 + (k & 1), j = j0 + (k >> 1);
    exists[k] = own && i < N1 && j < N2;
    dof[k] = exists[k] && (i | j) != 0;   // corner node 0 is pinned
    pidx[k] = P::at(i, j);
  }
  const int base = P::at(i0 - 1, j0 - 1);
  auto node_of = [&](int k) { return (j0 + (k >> 1)) * N1 + i0 + (k & 1); };
  // threads owning the blocks to the left, below and below-left (periodic)
  const int Il = (I + NB1 - 1) % NB1, Jb = (J + NB2 - 1) % NB2;
  const int t_l = bix(Il, J), t_b = bix(I, Jb), t_d = bix(Il, Jb);
  const int Ir = (I + 1) % NB1, Jt = (J + 1) % NB2;
  const int b_own = bix(I, J), b_r = bix(Ir, J), b_t = bix(I, Jt), b_d = bix(Ir, Jt);

  // ---- element scales (mu of the phase), padded --------------------------
  const double* par = a.params + static_cast<size_t>(b) * 4;
  const double mu0 = par[1], mu1 = par[3];
  const uint8_t* ph = a.phase + a.phase_off[b];
  double ssum = 0.0;
  // every load of the thread in flight at once, then the LDS writes (a loop
  // that waits for each load before the next would serialise the latencies)
  constexpr int PE = (NN + WG - 1) / WG;   // elements (and nodes) per thread
  uint8_t phv[PE];
#pragma unroll
  for (int q = 0; q < PE; ++q) {
    const int e = tid + q * WG;
    phv[q] = e < NN ? ph[e] : uint8_t(0);
  }
#pragma unroll
  for (int q = 0; q < PE; ++q) {
    const int e = tid + q * WG;
    if (e >= NN) continue;
    const double s = phv[q] ? mu1 : mu0;
    const int i = e % N1, j = e / N1;
    put_halo<N1, N2>(s_sc, i, j, s);
    put_halo<N1, N2>(s_sc32, i, j, static_cast<float>(s));
    ssum += s;
  }
  __syncthreads();
  const double* eb = s_sc + base;
  const TI* ebI;
  if constexpr (sizeof(TI) == 4) ebI = reinterpret_cast<const TI*>(s_sc32 + base);
  else ebI = reinterpret_cast<const TI*>(s_sc + base);

  const int64_t fo = a.foff[b];
  constexpr int64_t flen = 2 * NN;
  double* Xb = a.X + fo * (NF + 1);
  const double V = a.volume;
  double eps[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) eps[j] = a.macro[static_cast<size_t>(b) * NF + j];

  auto stage = [&](const double* src) {   // periodic field -> padded FP64 staging
    if constexpr (NRHS == 0) {
      // assembly only: one 16-byte load per node (fields start at even
      // offsets), all in flight before the LDS writes.  The solve
      // instantiations keep the plain loop, whose registers do not add to
      // the PCG's.
      double2 v[PE];
#pragma unroll
      for (int q = 0; q < PE; ++q) {
        const int n = tid + q * WG;
        if (n < NN) v[q] = reinterpret_cast<const double2*>(src)[n];
      }
#pragma unroll
      for (int q = 0; q < PE; ++q) {
        const int n = tid + q * WG;
        if (n >= NN) continue;
        const int i = n % N1, j = n / N1;
        put_halo<N1, N2>(s_st, i, j, v[q].x);
        put_halo<N1, N2>(s_st + P::PN, i, j, v[q].y);
      }
    } else {
      for (int n = tid; n < NN; n += WG) {
        const int i = n % N1, j = n / N1;
        put_halo<N1, N2>(s_st, i, j, src[2 * n]);
        put_halo<N1, N2>(s_st + P::PN, i, j, src[2 * n + 1]);
      }
    }
  };

  // ---- a3: residual and stress integral at (eps_b, w_b) ------------------
  double Pint[NF];
  if (a.flags & RVE_ASSEMBLE) {
    stage(a.w + fo);
    __syncthreads();
    double y[4][2];
    #pragma unroll
    for (int k = 0; k < 4; ++k) mv_node64<N1, N2>(s_st + base, eb, kv64, k & 1, k >> 1, y[k]);
    double red[5] = {0.0, 0.0, 0.0, 0.0, ssum};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!exists[k]) continue;
      const int di = k & 1, dj = k >> 1;
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        double rv = 0.0;
        if (dof[k]) {
          rv = y[k][d];
#pragma unroll
          for (int j = 0; j < NF; ++j) rv += bF_entry<N1, N2>(eb, KwF, di, dj, d, j) * eps[j];
        }
        a.r[fo + 2 * node_of(k) + d] = rv;
        red[0] += rv * rv;
        const double wv = s_st[d * P::PN + pidx[k]];
#pragma unroll
        for (int j = 0; j < NF; ++j) red[1 + j] += bF_entry<N1, N2>(eb, KwF, di, dj, d, j) * wv;
      }
    }
    wg_sum<5, NW, RED_NV>(red, s_red, parity);
    ssum = red[4];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      double kf = 0.0;
#pragma unroll
      for (int j = 0; j < NF; ++j) kf += a.KFF64[i * NF + j] * eps[j];
      Pint[i] = ssum * kf + red[1 + i];
    }
    if (tid == 0) {
#pragma unroll
      for (int i = 0; i < NF; ++i) a.Pbar[static_cast<size_t>(b) * NF + i] = Pint[i] / V;
      a.rnorm2[b] = red[0];
    }
  } else {
    double red[1] = {ssum};
    wg_sum<1, NW, RED_NV>(red, s_red, parity);
    ssum = red[0];
#pragma unroll
    for (int i = 0; i < NF; ++i) Pint[i] = a.Pbar[static_cast<size_t>(b) * NF + i] * V;
  }
  if constexpr (NRHS == 0) {   // assemble-only instantiation
    return;
  } else {
  if (!(a.flags & RVE_SOLVE)) return;
  const bool ronly = (a.flags & RVE_RONLY) != 0;
  if (ronly && a.rnorm2[b] <= a.thr2[b]) {   // already in equilibrium: x_r = 0
    double* xc = Xb + NF * flen;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (exists[k]) {
        xc[2 * node_of(k)] = 0.0;
        xc[2 * node_of(k) + 1] = 0.0;
      }
    if (tid == 0) {
      a.relres[b] = 0.0;
      a.iters[b] = 0.0;
      a.mv64[b] = 0.0;
    }
    return;
  }

  // ---- a5: per column, FP64 refinement around the inner PCG --------------
  TI dinv[4][2];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int di = k & 1, dj = k >> 1;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      double dg = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 2 * elem_cc(q) + d;
        dg += elem_scale<N1, N2>(eb, di, dj, q) * kv64[kref_id(r, r)];
      }
      dinv[k][d] = dof[k] ? static_cast<TI>(1.0 / dg) : TI(0);
    }
  }
  if constexpr (FFT) spectral_setup<N1, TI>(sreg, ftab, s_x + lin2d_xch_len(N1, N2, WG, true), own, I, J);
  const bool warm = (a.flags & RVE_WARM) != 0;
  const double tin2 = a.tol_in * a.tol_in;
  const double tol2 = a.tol * a.tol;
  int iters = 0, nmv64 = 0;
  bool all_ok = true;
  double worst = 0.0;

#pragma unroll 1
  for (int kc = ronly ? NF : 0; kc < NRHS; ++kc) {
    double* xc = Xb + kc * flen;
    bool xzero = !warm || kc >= NF;   // warm start: previous X_F; x_r from zero
    if (xzero) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (exists[k]) {
          xc[2 * node_of(k)] = 0.0;
          xc[2 * node_of(k) + 1] = 0.0;
        }
    }
#pragma unroll 1
    for (int sweep = 0;; ++sweep) {
      // FP64 residual r = b - K x of this column
      double y[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
      if (!xzero) {
        __syncthreads();   // earlier readers of the staging buffer are done
        stage(xc);
        __syncthreads();
        #pragma unroll
    for (int k = 0; k < 4; ++k) mv_node64<N1, N2>(s_st + base, eb, kv64, k & 1, k >> 1, y[k]);
        ++nmv64;
      }
      double r64[4][2];
      double red[2] = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int di = k & 1, dj = k >> 1;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          r64[k][d] = 0.0;
          if (dof[k]) {
            const double bk = (kc < NF) ? bF_entry<N1, N2>(eb, KwF, di, dj, d, kc)
                                        : a.r[fo + 2 * node_of(k) + d];
            r64[k][d] = bk - y[k][d];
            red[0] += r64[k][d] * r64[k][d];
            red[1] += bk * bk;
          }
        }
      }
      wg_sum<2, NW, RED_NV>(red, s_red, parity);
      // the inner solve runs on r / ||r|| (no FP32 underflow for the small
      // corrections of late sweeps); its result is scaled back in FP64
      const double rnrm = sqrt(red[0]);
      const double rinv = red[0] > 0.0 ? 1.0 / rnrm : 0.0;
      TI ri[4][2];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 2; ++d) ri[k][d] = static_cast<TI>(r64[k][d] * rinv);
      const double rel = red[1] > 0.0 ? sqrt(red[0] / red[1]) : 0.0;
      if (red[1] == 0.0 || red[0] <= tol2 * red[1]) {
        worst = rel > worst ? rel : worst;
        break;
      }
      if (sweep >= a.max_ir) {
        worst = rel > worst ? rel : worst;
        all_ok = false;
        break;
      }
      // ---- inner PCG on K d = r (precision TI, Jacobi preconditioner) -----
      // Chronopoulos-Gear form of CG: u = M^-1 r and w = K u are formed
      // every iteration and both inner products (r.u, w.u) go through one
      // fused work-group reduction; p and s = K p follow by recurrence, with
      // den_i = (w.u)_i - beta_i^2 den_{i-1} (= gamma_i / alpha_i).  Two
      // barriers per iteration (u visible, reduction; even sizes add the
      // operator's exchange barrier).  Scalars are kept in
      // TI.  The pinned node has M^-1 = 0, so its u, p and x stay zero and
      // its residual entry (which is left to drift) never enters r.u or w.u;
      // nodes of a block beyond the grid (odd sizes) get w = 0.  Convergence
      // is measured in the M^-1 norm, r.u <= tol_in^2 (r.u)_0.
      __syncthreads();   // staging reads finished before s_p is written
      TI xi[4][2], uv[4][2], pv[4][2], sv[4][2];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          xi[k][d] = pv[k][d] = sv[k][d] = TI(0);
          uv[k][d] = dinv[k][d] * ri[k][d];
          if constexpr (!EVEN)
            if (exists[k]) put_halo<N1, N2>(s_p + d * P::PN, i0 + (k & 1), j0 + (k >> 1), uv[k][d]);
        }
      if constexpr (EVEN && !FFT)
        if (own)
#pragma unroll
          for (int d = 0; d < 2; ++d) st4(s_p + d * NB1 * NB2 * 4 + 4 * b_own, uv[0][d], uv[1][d], uv[2][d], uv[3][d]);
      const TI tinI = static_cast<TI>(tin2);
      TI gam0 = TI(0), gam_old = TI(1), den_old = TI(1);
      TI esc[2][2];   // scales of the thread's four elements (even sizes)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2) esc[c][a2] = EVEN ? ebI[(c + 1) * P::PW + a2 + 1] : TI(0);
      if constexpr (FFT) {
        // Standard PCG with the spectral preconditioner, ordered so that the
        // operator acts on u = M^-1 r as soon as the preconditioner has
        // written it to LDS, and q = K p follows by q = K u + beta q.  Per
        // iteration: one preconditioner application, one operator
        // application, the reduction of r.u (it shares the operator's
        // exchange barrier) and that of p.q.  The single-reduction
        // recurrence for p.Kp used by the Jacobi form loses definiteness in
        // FP32 under this strong preconditioner; p.q formed from p and q
        // does not.  Each thread keeps its own x, r, p, q in registers; only
        // u passes through LDS.
        TI qv[4][2];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) qv[k][d] = TI(0);
#pragma unroll 1
        for (int it = 0;; ++it) {
          TI rm[4][2];
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int d = 0; d < 2; ++d) rm[k][d] = dof[k] ? ri[k][d] : TI(0);
          if constexpr (N1 == 48) spectral_precond48<TI>(rm, s_x, s_x + 2 * N1 * N2, s_p, sreg, own, I, J);
          else spectral_precond<N1, TI>(rm, s_x, s_x + 2 * N1 * N2, s_p, sreg, own, I, J);
          __syncthreads();   // u visible (and every read of the transform buffers done)
          // u of the owned block is read from LDS where it is used (it stays
          // there until the next preconditioner application) rather than
          // held across the operator
          auto load_u = [&]() {
            if (own) {
              TI o[4];
#pragma unroll
              for (int d = 0; d < 2; ++d) {
                ld4(s_p + d * NB1 * NB2 * 4 + 4 * b_own, o);
#pragma unroll
                for (int k = 0; k < 4; ++k) uv[k][d] = o[k];
              }
            }
          };
          load_u();
          TI gpart = TI(0);
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int d = 0; d < 2; ++d) gpart = fma(ri[k][d], uv[k][d], gpart);
          TI fo[2][2][2];
          mv_modes_post<N1, N2, WG, TI>(s_p, esc, mcI, s_x, b_own, b_r, b_t, b_d, tid, fo);
          const TI* rb = wsum_post<NW, TI>(gpart, s_red, parity);
          __syncthreads();   // exchange slots and the r.u wave totals visible
          TI wv[4][2];
          mv_modes_gather<WG, TI>(s_x, fo, t_l, t_b, t_d, wv);
          const TI gam = wsum_collect<NW, TI>(rb);
          if (it == 0) gam0 = gam;
          if (it >= a.max_it || !(gam > tinI * gam0) || !(gam > TI(0))) break;
          const TI beta = (it == 0) ? TI(0) : gam / gam_old;
          load_u();
          TI qpart = TI(0);
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int d = 0; d < 2; ++d) {
              pv[k][d] = fma_keep(pv[k][d], beta, uv[k][d]);
              qv[k][d] = fma_keep(qv[k][d], beta, wv[k][d]);
              qpart = fma(pv[k][d], qv[k][d], qpart);
            }
          const TI* qb = wsum_post<NW, TI>(qpart, s_red, parity);
          __syncthreads();
          const TI pq = wsum_collect<NW, TI>(qb);
          if (!(pq > TI(0))) break;   // exact solution or loss of definiteness
          const TI alpha = gam / pq;
          ++iters;
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int d = 0; d < 2; ++d) {
              xi[k][d] = fma(alpha, pv[k][d], xi[k][d]);
              ri[k][d] = fma(-alpha, qv[k][d], ri[k][d]);
            }
          gam_old = gam;
        }
      } else {
#pragma unroll 1
      for (int it = 0; it < a.max_it; ++it) {
        __syncthreads();   // u visible
        TI wv[4][2];
        if constexpr (EVEN) {
          mv_modes<N1, N2, WG, TI>(s_p, esc, mcI, s_x, b_own, b_r, b_t, b_d, tid, t_l, t_b, t_d, wv);
        } else {
          mv_block<N1, N2, TI>(s_p + base, ebI, kvI, wv);
#pragma unroll
          for (int k = 0; k < 4; ++k)   // blocks reaching past the grid: keep s, r finite there
#pragma unroll
            for (int d = 0; d < 2; ++d)
              if (!exists[k]) wv[k][d] = TI(0);
        }
        TI red[2] = {TI(0), TI(0)};
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            red[0] = fma(ri[k][d], uv[k][d], red[0]);
            red[1] = fma(wv[k][d], uv[k][d], red[1]);
          }
        if constexpr (sizeof(TI) == 4) {
          const float v2[2] = {red[0], red[1]};
          wg_sum_f32<2, NW, RED_NV>(v2, red, s_red, parity);
        } else {
          wg_sum<2, NW, RED_NV>(red, s_red, parity);
        }
        const TI gam = red[0], del = red[1];
        if (it == 0) gam0 = gam;
        if (!(gam > tinI * gam0) || !(gam > TI(0))) break;
        const TI beta = (it == 0) ? TI(0) : gam / gam_old;
        const TI den = del - beta * beta * den_old;
        if (!(den > TI(0))) break;   // breakdown (exact solution or loss of definiteness)
        const TI alpha = gam / den;
        ++iters;
        // every read of s_p in this iteration precedes the reduction's barrier
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            pv[k][d] = fma_keep(pv[k][d], beta, uv[k][d]);
            sv[k][d] = fma_keep(sv[k][d], beta, wv[k][d]);
            xi[k][d] = fma(alpha, pv[k][d], xi[k][d]);
            ri[k][d] = fma(-alpha, sv[k][d], ri[k][d]);
            uv[k][d] = dinv[k][d] * ri[k][d];
            if constexpr (!EVEN)
              if (exists[k]) put_halo<N1, N2>(s_p + d * P::PN, i0 + (k & 1), j0 + (k >> 1), uv[k][d]);
          }
        if constexpr (EVEN)
          if (own)
#pragma unroll
            for (int d = 0; d < 2; ++d)
              st4(s_p + d * NB1 * NB2 * 4 + 4 * b_own, uv[0][d], uv[1][d], uv[2][d], uv[3][d]);
        gam_old = gam;
        den_old = den;
      }
      }
      // x64 += x_inner (FP64 accumulation in the output column)
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 2; ++d)
          if (exists[k]) xc[2 * node_of(k) + d] += rnrm * static_cast<double>(xi[k][d]);
      xzero = false;
    }
  }
  if constexpr (NRHS == NF) {   // residual column not solved: x_r = 0
    double* xc = Xb + NF * flen;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (exists[k]) {
        xc[2 * node_of(k)] = 0.0;
        xc[2 * node_of(k) + 1] = 0.0;
      }
  }

  if (ronly) {
    if (tid == 0) {
      a.relres[b] = worst;
      a.iters[b] = static_cast<double>(iters);
      a.mv64[b] = static_cast<double>(nmv64);
      if (!all_ok) atomicAdd(a.fail_count, 1);
    }
    return;
  }

  // ---- a6: condensation (energy form) from a final FP64 pass -------------
  //   G1[i][j] = b_i . x_j,  G2[i][j] = x_i . (b_j - K x_j), one column j
  //   at a time; thread 0 writes Cbar column j (or Phat for j = NF)
  double* Cb = a.Cbar + static_cast<size_t>(b) * NF * NF;
#pragma unroll 1
  for (int jc = 0; jc < NRHS; ++jc) {
    const double* xc = Xb + jc * flen;
    __syncthreads();   // global writes of X visible, staging free
    stage(xc);
    __syncthreads();
    double y[4][2];
#pragma unroll
    for (int k = 0; k < 4; ++k) mv_node64<N1, N2>(s_st + base, eb, kv64, k & 1, k >> 1, y[k]);
    ++nmv64;
    double g[2 * NF] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!dof[k]) continue;
      const int di = k & 1, dj = k >> 1;
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const double bj = (jc < NF) ? bF_entry<N1, N2>(eb, KwF, di, dj, d, jc)
                                    : a.r[fo + 2 * node_of(k) + d];
        const double xj = s_st[d * P::PN + pidx[k]];
        const double res = bj - y[k][d];
#pragma unroll
        for (int i = 0; i < NF; ++i) {
          g[i] += bF_entry<N1, N2>(eb, KwF, di, dj, d, i) * xj;
          g[NF + i] += Xb[i * flen + 2 * node_of(k) + d] * res;
        }
      }
    }
    wg_sum<2 * NF, NW, RED_NV>(g, s_red, parity);
    if (tid == 0) {
      if (jc < NF) {
#pragma unroll
        for (int i = 0; i < NF; ++i) Cb[i * NF + jc] = (ssum * a.KFF64[i * NF + jc] - g[i] - g[NF + i]) / V;
      } else {
#pragma unroll
        for (int i = 0; i < NF; ++i) a.Phat[static_cast<size_t>(b) * NF + i] = (Pint[i] - g[i] - g[NF + i]) / V;
      }
    }
  }
  if (tid == 0) {
    a.relres[b] = worst;
    a.iters[b] = static_cast<double>(iters);
    a.mv64[b] = static_cast<double>(nmv64);
    if (!all_ok) atomicAdd(a.fail_count, 1);
    if constexpr (NRHS == NF) {
#pragma unroll
      for (int i = 0; i < NF; ++i) a.Phat[static_cast<size_t>(b) * NF + i] = Pint[i] / V;
    }
  }
  }
}


// Host: the spectral table of one class (mu = 1, lambda = rho, square
// elements; the element size cancels in 2D).  The Q4 element stiffness by
// 2x2 Gauss quadrature, its periodic symbol S(k) = sum_ab K_e[a][b]
// cos(k . (x_b - x_a)) (real: the stencil is centro-symmetric), the inverse
// of S at every k != 0 and the packing coefficients of the two real fields.
void lin2d_spectral_table(int n, double rho, double* out) {
  const bool r3 = n == 48;   // 3 x 16: a radix-3 stage, then radix-2 inside 16-wide sub-blocks
  const int ns = r3 ? 16 : n;
  int m = 0;
  while ((1 << m) < ns) ++m;
  const double xa[4] = {-1, 1, 1, -1}, ya[4] = {-1, -1, 1, 1};
  const int ox[4] = {0, 1, 1, 0}, oy[4] = {0, 0, 1, 1};
  const double C[3][3] = {{rho + 2.0, rho, 0.0}, {rho, rho + 2.0, 0.0}, {0.0, 0.0, 1.0}};
  double K[8][8] = {};
  const double g = 1.0 / std::sqrt(3.0);
  for (int gp = 0; gp < 4; ++gp) {
    const double xi = (gp & 1) ? g : -g, eta = (gp & 2) ? g : -g;
    double B[3][8] = {};
    for (int a = 0; a < 4; ++a) {
      const double dx = 0.5 * xa[a] * (1.0 + ya[a] * eta), dy = 0.5 * ya[a] * (1.0 + xa[a] * xi);   // x in [0, 1]
      B[0][2 * a] = dx;
      B[1][2 * a + 1] = dy;
      B[2][2 * a] = dy;
      B[2][2 * a + 1] = dx;
    }
    for (int r = 0; r < 8; ++r)
      for (int c = 0; c < 8; ++c) {
        double v = 0.0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) v += B[i][r] * C[i][j] * B[j][c];
        K[r][c] += 0.25 * v;   // det J = 1/4, unit weights
      }
  }
  auto rev = [m](int x) {
    int y = 0;
    for (int t = 0; t < m; ++t) y |= ((x >> t) & 1) << (m - 1 - t);
    return y;
  };
  // frequency held at position p after the forward transform: bit reversal
  // (powers of two); sub-block s = p / 16 holds frequencies s + 3 k (n = 48)
  auto freq = [&](int p) { return r3 ? 3 * rev(p % ns) + p / ns : rev(p); };
  const double two_pi = 6.283185307179586476925;
  for (int q = 0; q < n; ++q)
    for (int p = 0; p < n; ++p) {
      const int kx = freq(p), ky = freq(q);
      double S[2][2] = {};
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          const double cs = std::cos(two_pi * (kx * (ox[b] - ox[a]) + ky * (oy[b] - oy[a])) / n);
          for (int c = 0; c < 2; ++c)
            for (int e = 0; e < 2; ++e) S[c][e] += K[2 * a + c][2 * b + e] * cs;
        }
      double* t = out + 4 * (q * n + p);
      t[0] = t[1] = t[2] = t[3] = 0.0;
      if (kx == 0 && ky == 0) continue;   // translations: projected out
      const double det = S[0][0] * S[1][1] - S[0][1] * S[1][0];
      const double ia = S[1][1] / det, ic = S[0][0] / det, ib = -0.5 * (S[0][1] + S[1][0]) / det;
      t[0] = 0.5 * (ia + ic);
      t[1] = 0.5 * (ia - ic);
      t[2] = ib;
    }
  for (int k = 0; k < lin2d_spectral_twiddles(n); ++k) {
    out[4 * n * n + 2 * k] = std::cos(two_pi * k / n);
    out[4 * n * n + 2 * k + 1] = -std::sin(two_pi * k / n);
  }
}

// ---------------------------------------------------------------------------
// launch: dispatch on the compile-time RVE size
// ---------------------------------------------------------------------------
static constexpr int wg_for(int n1, int n2) {
  return 64 * ((((n1 + 1) / 2) * ((n2 + 1) / 2) + 63) / 64);
}

template <typename TI, int NRHS, int N1, int N2, bool FFT = false>
static int launch_t(const Lin2DArgs& a, int n_launch, hipStream_t s) {
  constexpr int WG = wg_for(N1, N2);
  constexpr size_t lds = lin2d_lds_bytes_t(N1, N2, WG, NRHS, static_cast<int>(sizeof(TI)), FFT);
  static_assert(lds <= 160 * 1024, "RVE too large for the LDS-resident solver");
  // the spectral preconditioner's complex field [N*N][2] aliases the exchange slots [3][WG][4]
  static_assert(!FFT || 2 * N1 * N2 <= 12 * WG, "exchange slots too small for the spectral field");
  static_assert(!FFT || N1 != 48 || WG == 576, "the 48-element transform assumes one block per lane");
  auto kern = &k_lin2d<TI, NRHS, N1, N2, WG, FFT>;
  if (lds > 64 * 1024)
    FE2_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  hipLaunchKernelGGL(kern, dim3(n_launch), dim3(WG), lds, s, a);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

template <int N1, int N2>
static int launch_n(const Lin2DArgs& a, int n_launch, int precision, int nrhs, hipStream_t s) {
  if (nrhs == 0) return launch_t<double, 0, N1, N2>(a, n_launch, s);   // assemble only (FP64)
  if constexpr (lin2d_spectral_size(N1, N2)) {
    if (a.flags & RVE_FFT) {
      if (!a.fft_tab || !a.fft_tab64) return set_error("spectral preconditioner table missing"), FE2_EINVAL;
      if (precision == FE2_PREC_FP64)
        return nrhs == 3 ? launch_t<double, 3, N1, N2, true>(a, n_launch, s)
                         : launch_t<double, 4, N1, N2, true>(a, n_launch, s);
      return nrhs == 3 ? launch_t<float, 3, N1, N2, true>(a, n_launch, s) : launch_t<float, 4, N1, N2, true>(a, n_launch, s);
    }
  } else {
    if (a.flags & RVE_FFT) return set_error("no spectral preconditioner for this RVE size"), FE2_ENOTSUP;
  }
  if (precision == FE2_PREC_FP64)
    return nrhs == 3 ? launch_t<double, 3, N1, N2>(a, n_launch, s) : launch_t<double, 4, N1, N2>(a, n_launch, s);
  return nrhs == 3 ? launch_t<float, 3, N1, N2>(a, n_launch, s) : launch_t<float, 4, N1, N2>(a, n_launch, s);
}

#define FE2_LIN2D_SIZES(X) X(4, 4) X(6, 10) X(8, 8) X(10, 10) X(15, 15) X(16, 16) X(17, 17) X(30, 30) X(32, 32) X(48, 48)

bool lin2d_supported(int n1, int n2) {
#define FE2_CASE(A, B) if (n1 == A && n2 == B) return true;
  FE2_LIN2D_SIZES(FE2_CASE)
#undef FE2_CASE
  return false;
}

int launch_lin2d(const Lin2DArgs& a, int n_launch, int precision, int nrhs, hipStream_t s) {
  if (n_launch <= 0) return FE2_OK;
#define FE2_CASE(A, B) \
  if (a.n1 == A && a.n2 == B) return launch_n<A, B>(a, n_launch, precision, nrhs, s);
  FE2_LIN2D_SIZES(FE2_CASE)
#undef FE2_CASE
  set_error("RVE resolution has no compiled 2D kernel");
  return FE2_ENOTSUP;
}

}  // namespace fe2
