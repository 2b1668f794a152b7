// Spectral preconditioner of the RVE PCG (2D): the inverse of the periodic
// Q4 operator of a homogeneous reference medium, applied by a vector-radix
// FFT in LDS.  Shared by the small-strain and the finite-strain kernels.
#pragma once

#include "rve2d_common.hpp"

namespace fe2 {

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

// Row pitch (complex elements) of the transform fields in LDS.  A wave
// works on an 8 x 8 tile of butterfly groups whose rows lie a power-of-two
// apart; with a pitch of N the eight rows fall on the same LDS banks
// (eight-way conflicts in every stage).  These pitches spread them, the
// worst stage staying at three-way for 32 (two to four for the others).
__host__ __device__ constexpr int spectral_pitch(int n) { return n == 32 ? 38 : n + 2; }

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
  constexpr int ZP = spectral_pitch(N);
  const unsigned i = I + (I & ~(H - 1u)), j = J + (J & ~(H - 1u));
  TI* zb = z + 2 * (j * ZP + i);
  const TI* tx = tw + 2 * ((I & (H - 1u)) * TS);
  const TI* ty = tw + 2 * ((J & (H - 1u)) * TS);
  const Cx<TI> wx = {tx[0], tx[1]}, wy = {ty[0], ty[1]};
  constexpr int DX = 2 * H, DY = 2 * H * ZP;
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
  return z + 4 * (J * spectral_pitch(N) + I);
}

// Last forward stage (h = 1, unit twiddles) on the owned block: v and z
// at the owned positions.  The caller's barrier then makes z readable for
// the symbol's partner reads (spectral_symbol).
template <int N, typename TI>
__device__ __forceinline__ void spectral_fwd1(Cx<TI> (&v)[4], TI* __restrict__ z, unsigned I, unsigned J) {
  constexpr int ZP = spectral_pitch(N);
  TI* zo = own_pts<N>(z, I, J);
  // h = 1 (unit twiddles) on the owned block
  {
    const Cx<TI> a = {zo[0], zo[1]}, b = {zo[2], zo[3]};
    const Cx<TI> c = {zo[2 * ZP], zo[2 * ZP + 1]}, d = {zo[2 * ZP + 2], zo[2 * ZP + 3]};
    const Cx<TI> A = cadd(a, b), B = csub(a, b), C = cadd(c, d), D = csub(c, d);
    v[0] = cadd(A, C);
    v[2] = csub(A, C);
    v[1] = cadd(B, D);
    v[3] = csub(B, D);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) zo[(k & 1) * 2 + (k >> 1) * 2 * ZP] = v[k].re, zo[(k & 1) * 2 + (k >> 1) * 2 * ZP + 1] = v[k].im;
}

// The symbol at the owned positions: W = alpha Z + beta conj Z(-k).  Shared
// by every size (the transform stages differ: radix-2 only, or radix-3
// first for N = 48).
template <int N, typename TI>
__device__ __forceinline__ void spectral_symbol(Cx<TI> (&v)[4], const TI* __restrict__ z, const SpectralRegs<N, TI>& g,
                                                unsigned I, unsigned J) {
  constexpr int ZP = spectral_pitch(N);
  // partner positions of the owned block from the LDS map (one 16-bit read
  // per axis: the entries of 2I and 2I + 1)
  const unsigned px = *reinterpret_cast<const unsigned short*>(g.pm + 2 * I);
  const unsigned py = *reinterpret_cast<const unsigned short*>(g.pm + 2 * J);
  const unsigned ppx[2] = {px & 0xffu, px >> 8}, ppy[2] = {py & 0xffu, py >> 8};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const TI* zp = z + 2 * (ppy[k >> 1] * ZP + ppx[k & 1]);
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
  constexpr int ZP = spectral_pitch(N);
  TI* zo = own_pts<N>(z2, I, J);
  const Cx<TI> A = cadd(v[0], v[1]), B = csub(v[0], v[1]), C = cadd(v[2], v[3]), D = csub(v[2], v[3]);
  const Cx<TI> o[4] = {cadd(A, C), cadd(B, D), csub(A, C), csub(B, D)};   // (0,0) (1,0) (0,1) (1,1)
#pragma unroll
  for (int k = 0; k < 4; ++k) zo[(k & 1) * 2 + (k >> 1) * 2 * ZP] = o[k].re, zo[(k & 1) * 2 + (k >> 1) * 2 * ZP + 1] = o[k].im;
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
// y at +N*N), written with u (pinned node zero); with NAT, sp is instead a
// complex field in natural order (row pitch spectral_pitch(N), u_x + i u_y).
// Ends without a barrier: the caller's next barrier makes sp visible.
// With PRE, the caller has already written r into z (natural order, pitch
// spectral_pitch(N)) and r is not read.
template <int N, typename TI, bool NAT = false, bool PRE = false>
__device__ __forceinline__ void spectral_precond(const TI (&r)[4][2], TI* __restrict__ z, TI* __restrict__ z2,
                                                 TI* __restrict__ sp, const SpectralRegs<N, TI>& g, bool own, int Ii,
                                                 int Ji) {
  constexpr int M = SpectralRegs<N, TI>::M;
  constexpr int H = N / 2;   // last inverse stage
  constexpr int TW = Tiles<N / 2>::TW;
  constexpr int ZP = spectral_pitch(N);
  // I and J opaque per call: the stage addresses (integer arithmetic on
  // them) are formed here rather than hoisted out of the PCG loop, where
  // they would hold some forty registers across the whole solve
  asm volatile("" : "+v"(Ii), "+v"(Ji));
  const unsigned I = static_cast<unsigned>(Ii), J = static_cast<unsigned>(Ji);
  if (!PRE && own) {
    TI* zo = own_pts<N>(z, I, J);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      zo[(k & 1) * 2 + (k >> 1) * 2 * ZP] = r[k][0], zo[(k & 1) * 2 + (k >> 1) * 2 * ZP + 1] = r[k][1];
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
    TI* zb = z2 + 2 * (J * ZP + I);
    const TI* tx = g.tw + 2 * I;
    const TI* ty = g.tw + 2 * J;
    const Cx<TI> wx = {tx[0], tx[1]}, wy = {ty[0], ty[1]};
    constexpr int DX = 2 * H, DY = 2 * H * ZP;
    const Cx<TI> a = {zb[0], zb[1]}, b = cmulc(Cx<TI>{zb[DX], zb[DX + 1]}, wx);
    const Cx<TI> c = {zb[DY], zb[DY + 1]}, d = cmulc(Cx<TI>{zb[DX + DY], zb[DX + DY + 1]}, wx);
    const Cx<TI> A = cadd(a, b), B = csub(a, b), C = cmulc(cadd(c, d), wy), D = cmulc(csub(c, d), wy);
    const Cx<TI> o00 = cadd(A, C), o10 = cadd(B, D), o01 = csub(A, C), o11 = csub(B, D);
    const bool pin = (I | J) == 0;
    if constexpr (NAT) {   // natural order: points (I, J) + {0, H}^2
      TI* sb = sp + 2 * (J * ZP + I);
      sb[0] = pin ? TI(0) : o00.re;
      sb[1] = pin ? TI(0) : o00.im;
      sb[DX] = o10.re, sb[DX + 1] = o10.im;
      sb[DY] = o01.re, sb[DY + 1] = o01.im;
      sb[DX + DY] = o11.re, sb[DX + DY + 1] = o11.im;
    } else {
      // node (x, y) -> block-major slot; +H along x or y is a constant offset
      TI* sb = sp + 4 * Tiles<N / 2>::bix(I >> 1, J >> 1) + (I & 1) + 2 * (J & 1);
      constexpr int OX = sp_at<N>(H, 0) - sp_at<N>(0, 0), OY = sp_at<N>(0, H) - sp_at<N>(0, 0);
      sb[0] = pin ? TI(0) : o00.re;
      sb[N * N] = pin ? TI(0) : o00.im;
      sb[OX] = o10.re, sb[N * N + OX] = o10.im;
      sb[OY] = o01.re, sb[N * N + OY] = o01.im;
      sb[OX + OY] = o11.re, sb[N * N + OX + OY] = o11.im;
    }
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
  constexpr int N = 48, NS = 16, ZP = spectral_pitch(N);
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
      zo[(k & 1) * 2 + (k >> 1) * 2 * ZP] = r[k][0], zo[(k & 1) * 2 + (k >> 1) * 2 * ZP + 1] = r[k][1];
  }
  __syncthreads();
  if (tid < NS * NS) {   // radix-3 x 3, forward: the lane's nine points, in place, one axis at a time
    const int x = tid % NS, y = tid / NS;
#pragma unroll 1
    for (int b = 0; b < 3; ++b) {   // along x
      Cx<TI> o[3];
      dft3(zld<TI>(z, x, y + NS * b, ZP), zld<TI>(z, x + NS, y + NS * b, ZP), zld<TI>(z, x + 2 * NS, y + NS * b, ZP), o,
           false);
#pragma unroll
      for (int mx = 0; mx < 3; ++mx) zst<TI>(z, x + NS * mx, y + NS * b, ZP, o[mx]);
    }
#pragma unroll 1
    for (int mx = 0; mx < 3; ++mx) {   // along y, then the twiddles
      Cx<TI> o[3];
      dft3(zld<TI>(z, x + NS * mx, y, ZP), zld<TI>(z, x + NS * mx, y + NS, ZP), zld<TI>(z, x + NS * mx, y + 2 * NS, ZP), o,
           false);
#pragma unroll
      for (int my = 0; my < 3; ++my) zst<TI>(z, x + NS * mx, y + NS * my, ZP, cmul(o[my], cmul(w48(x * mx), w48(y * my))));
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
        vv[mx] = cmulc(zld<TI>(z2, x + NS * mx, y + NS * my, ZP), cmul(w48(x * mx), w48(y * my)));
      dft3(vv[0], vv[1], vv[2], o, true);
#pragma unroll
      for (int a = 0; a < 3; ++a) zst<TI>(z2, x + NS * a, y + NS * my, ZP, o[a]);
    }
#pragma unroll 1
    for (int a = 0; a < 3; ++a) {
      Cx<TI> o[3];
      dft3(zld<TI>(z2, x + NS * a, y, ZP), zld<TI>(z2, x + NS * a, y + NS, ZP), zld<TI>(z2, x + NS * a, y + 2 * NS, ZP),
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

}  // namespace fe2
