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
#include "spectral2d.hpp"
#include "dense2d.hpp"

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
  //         (two values per thread, [WG][2] after the two four-value slots)
  st4(sx + 4 * (0 * WG + tid), fx[0][2], fy[0][2], fx[1][2], fy[1][2]);
  st4(sx + 4 * (1 * WG + tid), fx[2][0], fy[2][0], fx[2][1], fy[2][1]);
  sx[8 * WG + 2 * tid] = fx[2][2];
  sx[8 * WG + 2 * tid + 1] = fy[2][2];
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
  V gl[4], gb[4], gd[2];
  ld4(sx + 4 * (0 * WG + tl), gl);
  ld4(sx + 4 * (1 * WG + tb), gb);
  gd[0] = sx[8 * WG + 2 * td];
  gd[1] = sx[8 * WG + 2 * td + 1];
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
// [8][NF] element table in global memory, read-only for the whole launch.
// It is read through the constant address space, so that its reads are
// scalar loads into SGPRs wherever they sit (a plain global pointer read
// after a barrier or a store becomes a vector load, serialised through
// whatever VGPRs are left in the register-bound solve instantiations).
using const_f64 = __attribute__((address_space(4))) const double;
template <int N1, int N2>
__device__ __forceinline__ double bF_entry(const double* __restrict__ eb, const double* __restrict__ KwF,
                                           int di, int dj, int d, int j) {
  const const_f64* K = (const const_f64*)KwF;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) s += elem_scale<N1, N2>(eb, di, dj, q) * K[(2 * elem_cc(q) + d) * NF + j];
  return s;
}

}  // namespace

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
  return spectral && 4 * static_cast<size_t>(n1) * spectral_pitch(n1) > 12 * static_cast<size_t>(wg)
             ? 4 * static_cast<size_t>(n1) * spectral_pitch(n1)
             : 12 * static_cast<size_t>(wg);
}
__host__ __device__ constexpr size_t lin2d_xch_bytes(int n1, int n2, int wg, int nrhs, int ti_bytes, bool spectral) {
  return ((n1 | n2) & 1) == 0 && nrhs > 0 ? lin2d_xch_len(n1, n2, wg, spectral) * ti_bytes : 0;
}
__host__ __device__ constexpr size_t lin2d_lds_bytes_t(int n1, int n2, int wg, int nrhs, int ti_bytes,
                                                       bool spectral = false, bool dense = false) {
  // the dense form takes the place of the exchange slots (its inner solve
  // does not run the element-wise operator): factor, vector, scratch, flag
  return dense ? lin2d_xch_offset(n1, n2, wg, nrhs) + 4 * dense2d::dense_floats(dense2d::dense_md(n1, n2)) + 16
               : lin2d_xch_offset(n1, n2, wg, nrhs) + lin2d_xch_bytes(n1, n2, wg, nrhs, ti_bytes, spectral) +
                     (spectral ? 2 * static_cast<size_t>(lin2d_spectral_twiddles(n1)) * ti_bytes + n1 + 2 : 0);   // twiddles, partner map
}

// The spectral FP32 form is held to three work-groups of 256 lanes per CU
// (at most 168 VGPRs), the occupancy of the Jacobi form.
template <typename TI, bool FFT, int WG>
constexpr int kLin2dMinBlocks = (sizeof(TI) == 4 && FFT && WG == 256) ? 3 : (FFT && WG == 256) ? 2 : 1;

template <typename TI, int NRHS, int N1, int N2, int WG, bool FFT, bool DENSE = false>
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
  static_assert(!DENSE || (!FFT && sizeof(TI) == 4 && WG == 256), "dense solve: FP32 factor, 256 lanes");
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
  const int64_t fo = a.foff[b];
  double ssum = 0.0;
  // every load of the thread in flight at once, then the LDS writes (a loop
  // that waits for each load before the next would serialise the latencies)
  constexpr int PE = (NN + WG - 1) / WG;   // elements (and nodes) per thread
  uint8_t phv[PE];
#pragma unroll
  for (int q = 0; q < PE; ++q) {   // (clamped index: no branch around the loads)
    const int e = tid + q * WG;
    phv[q] = ph[e < NN ? e : NN - 1];
  }
  // assembly-only instantiation: the field w_b is loaded together with the
  // phase ids (one 16-byte load per node; fields start at even offsets) and
  // staged behind the same barrier
  constexpr bool PRE_W = NRHS == 0;
  const bool pre_w = PRE_W && (a.flags & RVE_ASSEMBLE);
  double2 wpre[PRE_W ? PE : 1];
  if constexpr (PRE_W) {
#pragma unroll
    for (int q = 0; q < PE; ++q) {
      const int n = tid + q * WG;
      if (pre_w && n < NN) wpre[q] = reinterpret_cast<const double2*>(a.w + fo)[n];
    }
  }
#pragma unroll
  for (int q = 0; q < PE; ++q) {
    const int e = tid + q * WG;
    if (e >= NN) continue;
    const double s = phv[q] ? mu1 : mu0;
    const int i = e % N1, j = e / N1;
    put_halo<N1, N2>(s_sc, i, j, s);
    if constexpr (sizeof(TI) == 4) put_halo<N1, N2>(s_sc32, i, j, static_cast<float>(s));
    ssum += s;
  }
  if constexpr (PRE_W) {
#pragma unroll
    for (int q = 0; q < PE; ++q) {
      const int n = tid + q * WG;
      if (!pre_w || n >= NN) continue;
      const int i = n % N1, j = n / N1;
      put_halo<N1, N2>(s_st, i, j, wpre[q].x);
      put_halo<N1, N2>(s_st + P::PN, i, j, wpre[q].y);
    }
  }
  __syncthreads();
  const double* eb = s_sc + base;
  const TI* ebI;
  if constexpr (sizeof(TI) == 4) ebI = reinterpret_cast<const TI*>(s_sc32 + base);
  else ebI = reinterpret_cast<const TI*>(s_sc + base);

  constexpr int64_t flen = 2 * NN;
  double* Xb = a.X + fo * (NF + 1);
  const double V = a.volume;
  double eps[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) eps[j] = a.macro[static_cast<size_t>(b) * NF + j];

  auto stage = [&](const double* src) {   // periodic field -> padded FP64 staging
    // one 16-byte load per node (columns start at even offsets); above 32^2
    // two nodes' loads are in flight before their LDS writes (a
    // load-then-write loop waits out an L2 round trip per load; at 32^2 the
    // second load's registers cost more spills than the wait saves).  The
    // assembly-only instantiation staged w_b with the phase ids.
    constexpr int SU = N1 * N2 > 1024 ? 2 : 1;
    for (int n0 = tid; n0 < NN; n0 += SU * WG) {
      double2 v[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int n = n0 + u * WG;
        if (n < NN) v[u] = reinterpret_cast<const double2*>(src)[n];
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int n = n0 + u * WG;
        if (n >= NN) continue;
        const int i = n % N1, j = n / N1;
        put_halo<N1, N2>(s_st, i, j, v[u].x);
        put_halo<N1, N2>(s_st + P::PN, i, j, v[u].y);
      }
    }
  };

  // ---- a3: residual and stress integral at (eps_b, w_b) ------------------
  double Pint[NF];
  // (only the assembly-only instantiation assembles: the host never sends
  // RVE_ASSEMBLE with right-hand sides)
  if (pre_w) {
    if constexpr (!PRE_W) {
      stage(a.w + fo);
      __syncthreads();
    }
    double y[4][2];
    #pragma unroll
    for (int k = 0; k < 4; ++k) mv_node64<N1, N2>(s_st + base, eb, kv64, k & 1, k >> 1, y[k]);
    double red[5] = {0.0, 0.0, 0.0, 0.0, ssum};
    // no lane-dependent branch surrounds the K_wF reads: nodes the thread
    // does not hold are masked by selects
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k & 1, dj = k >> 1;
      double rv2[2];
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        double bf[NF];
#pragma unroll
        for (int j = 0; j < NF; ++j) bf[j] = bF_entry<N1, N2>(eb, KwF, di, dj, d, j);
        double rv = y[k][d];
#pragma unroll
        for (int j = 0; j < NF; ++j) rv += bf[j] * eps[j];
        rv = dof[k] ? rv : 0.0;
        rv2[d] = rv;
        const double wv = s_st[d * P::PN + pidx[k]];
        red[0] += exists[k] ? rv * rv : 0.0;
#pragma unroll
        for (int j = 0; j < NF; ++j) red[1 + j] += exists[k] ? bf[j] * wv : 0.0;
      }
      if (exists[k]) *reinterpret_cast<double2*>(a.r + fo + 2 * node_of(k)) = make_double2(rv2[0], rv2[1]);
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
  if constexpr (FFT)
    spectral_setup<N1, TI>(sreg, ftab, s_x + lin2d_xch_bytes(N1, N2, WG, NRHS, static_cast<int>(sizeof(TI)), true) / sizeof(TI),
                           own, I, J);
  // dense form: K_ww assembled and factored once per RVE (FP32, matrix cores)
  constexpr int MD = DENSE ? dense2d::dense_md(N1, N2) : 16;
  float* dA = reinterpret_cast<float*>(smem + lin2d_xch_offset(N1, N2, WG, NRHS));
  float* dv = dA + static_cast<size_t>(MD) * dense2d::dense_pitch(MD);
  float* dscr = dv + MD;
  int* dflag = reinterpret_cast<int*>(dscr + 256);
  if constexpr (DENSE) {
    dense2d::dense_assemble<N1, N2>(dA, s_sc, kv64);
    if (!dense2d::dense_potrf<MD>(dA, dflag)) {   // K_ww not positive definite in FP32
      if (tid == 0) {
        atomicAdd(a.fail_count, 1);
        a.relres[b] = __builtin_inf();
        a.iters[b] = 0.0;
        a.mv64[b] = 0.0;
      }
      return;
    }
    for (int t = tid; t < MD; t += WG) dv[t] = 0.0f;   // padding unknowns stay zero
  }
  // ---- a6 folded into the refinement (FP32 spectral solve) ----------------
  // The energy-form entry E[i][j] = b_i . x_j + x_i . (b_j - K x_j) equals
  // E[j][i] for symmetric K, whatever the solve error.  So column j, at the
  // sweep that accepts it, supplies E[i][j] for i <= j from the K x_j and
  // the staged x_j it has just used (x_i of the finished columns from HBM),
  // and thread 0 writes C-bar entry (i, j) and its mirror; the residual
  // column gives P-hat.  No separate FP64 pass per column.
  constexpr bool FOLD = FFT && sizeof(TI) == 4;
  double* Cb = a.Cbar + static_cast<size_t>(b) * NF * NF;
  auto fold = [&](int jc, bool xz, const double (&rj)[4][2]) {
    double g[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) g[i] = 0.0;
    double xj[4][2];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int d = 0; d < 2; ++d) xj[k][d] = (xz || !dof[k]) ? 0.0 : s_st[d * P::PN + pidx[k]];
    // one column i at a time: its four own-node (x, y) pairs are loaded
    // together (16-byte loads, no lane-dependent branch around them, at
    // constant offsets from one address for even sizes, where every
    // thread's block lies inside the RVE; for odd sizes a node the thread
    // does not hold reads node 0), then summed in the order k, d as for
    // column jc itself
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      if (jc < NF && i > jc) continue;   // from the mirror, when column i is accepted
      double xi[4][2];
      if (i == jc) {
#pragma unroll
        for (int k = 0; k < 4; ++k) xi[k][0] = xj[k][0], xi[k][1] = xj[k][1];
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double2 v =
              *reinterpret_cast<const double2*>(Xb + i * flen + 2 * ((EVEN || exists[k]) ? node_of(k) : 0));
          xi[k][0] = v.x;
          xi[k][1] = v.y;
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (!dof[k]) continue;
        const int di = k & 1, dj = k >> 1;
#pragma unroll
        for (int d = 0; d < 2; ++d) g[i] += bF_entry<N1, N2>(eb, KwF, di, dj, d, i) * xj[k][d] + xi[k][d] * rj[k][d];
      }
    }
    wg_sum<NF, NW, RED_NV>(g, s_red, parity);
    if (tid == 0) {
      if (jc < NF) {
        for (int i = 0; i <= jc; ++i) {
          const double v = (ssum * a.KFF64[i * NF + jc] - g[i]) / V;
          Cb[i * NF + jc] = v;
          Cb[jc * NF + i] = v;
        }
      } else {
#pragma unroll
        for (int i = 0; i < NF; ++i) a.Phat[static_cast<size_t>(b) * NF + i] = (Pint[i] - g[i]) / V;
      }
    }
  };
  const bool warm = (a.flags & RVE_WARM) != 0;
  const double tin2 = a.tol_in * a.tol_in;
  const double tol2 = a.tol * a.tol;
  int iters = 0, nmv64 = 0;
  bool all_ok = true;
  double worst = 0.0;

#pragma unroll 1
  for (int kc = ronly ? NF : 0; kc < NRHS; ++kc) {
    double* xc = Xb + kc * flen;
    // warm start: previous X_F; x_r from zero.  A column that starts from
    // zero is not cleared in memory: the first correction is stored as the
    // column (no read-modify-write), and a column that needs no correction
    // is written as zeros when its loop ends
    bool xzero = !warm || kc >= NF;
    auto clear_col = [&]() {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (exists[k]) {
          xc[2 * node_of(k)] = 0.0;
          xc[2 * node_of(k) + 1] = 0.0;
        }
    };
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
        if (xzero) clear_col();
        if constexpr (FOLD) {
          if (!ronly) fold(kc, xzero, r64);
        }
        break;
      }
      if (sweep >= a.max_ir) {
        worst = rel > worst ? rel : worst;
        all_ok = false;
        if (xzero) clear_col();
        if constexpr (FOLD) {
          if (!ronly) fold(kc, xzero, r64);
        }
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
      TI xi[4][2];
      if constexpr (DENSE) {
        // the direct solve with the FP32 factor: r into the unknown vector,
        // forward and backward substitution, the correction back
        __syncthreads();   // the previous solve's readers of the vector are done
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d)
            if (dof[k]) dv[dense2d::dof_of(node_of(k), d)] = ri[k][d];
        __syncthreads();
        dense2d::dense_solve<MD>(dA, dv, dscr);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) xi[k][d] = dof[k] ? dv[dense2d::dof_of(node_of(k), d)] : TI(0);
        ++iters;
      } else {
      __syncthreads();   // staging reads finished before s_p is written
      TI uv[4][2], pv[4][2], sv[4][2];
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
          if constexpr (N1 == 48) spectral_precond48<TI>(rm, s_x, s_x + 2 * N1 * spectral_pitch(N1), s_p, sreg, own, I, J);
          else spectral_precond<N1, TI>(rm, s_x, s_x + 2 * N1 * spectral_pitch(N1), s_p, sreg, own, I, J);
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
      }   // (inner solve)
      // x64 += x_inner (FP64 accumulation in the output column; stored
      // directly when the column started from zero)
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 2; ++d)
          if (exists[k]) {
            const double dx = rnrm * static_cast<double>(xi[k][d]);
            double* xp = xc + 2 * node_of(k) + d;
            *xp = xzero ? dx : *xp + dx;
          }
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
#pragma unroll 1
  for (int jc = 0; jc < (FOLD ? 0 : NRHS); ++jc) {
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


// ---------------------------------------------------------------------------
// Multi-column solve: the n_F = 3 columns of X_F in one PCG loop
// ---------------------------------------------------------------------------
// Square 16 x 16 and 32 x 32 RVEs, FP32 inner precision, spectral
// preconditioner, three right-hand sides (the RVE residual column x_r is
// zero).  The three columns run as independent CGs in lock step: one
// preconditioner application per iteration transforms the three fields
// stage by stage (the stage addresses, twiddles and barriers are shared),
// one pass of the element-wise operator serves the three search directions,
// and the reductions carry one value per column.  A column that has
// converged drops out of the work (uniform branches), the others go on.
// The FP64 refinement treats the three columns together as well: every
// sweep forms the three FP64 residuals, and the accepted sweep's residuals
// give the condensation in the energy form for every entry,
// E[i][j] = b_i . x_j + x_i . (b_j - K x_j), without a further pass.
//
// LDS (byte offsets): reduction buffers [2][NW][MR_NV] doubles | element
// scales FP64 [PN] | FP32 [PN] | search directions u [3][2][N*N] FP32 |
// exchange slots [3][3][WG][4] FP32, aliased by the three transform fields
// [3][N*N][2] | twiddles, partner map.  The FP64 column of the refinement
// passes ([2][PN] doubles, padded periodic layout) aliases the u and
// exchange regions, which are free outside the inner solve.
__host__ __device__ constexpr size_t al16(size_t x) { return (x + 15) & ~static_cast<size_t>(15); }
constexpr int MR_C = 3;
constexpr int MR_NV = 2 * MR_C + MR_C * MR_C;   // FP64 sweep reduction: norms and energy-form products
template <int N, int WG>
struct MrLds {
  static constexpr size_t PN = static_cast<size_t>(pad_w(N)) * pad_w(N);
  static constexpr size_t red = 0;
  static constexpr size_t sc = al16(2 * static_cast<size_t>(WG / 64) * MR_NV * 8);
  static constexpr size_t sc32 = al16(sc + PN * 8);
  static constexpr size_t u = al16(sc32 + PN * 4);
  static constexpr size_t ulen = static_cast<size_t>(MR_C) * 2 * N * N * 4;
  static constexpr size_t x = al16(u + ulen);
  static constexpr size_t zlen = static_cast<size_t>(MR_C) * 2 * N * spectral_pitch(N);
  static constexpr size_t xlen = (static_cast<size_t>(MR_C) * 12 * WG > zlen ? static_cast<size_t>(MR_C) * 12 * WG : zlen) * 4;
  static constexpr size_t tw = x + xlen;
  static constexpr size_t total = tw + 2 * static_cast<size_t>(lin2d_spectral_twiddles(N)) * 4 + N + 2;
  static_assert(ulen + xlen >= 2 * PN * 8, "FP64 column does not fit the aliased region");
};

// u = M^-1 r for the three columns (see spectral_precond; every thread of
// the work-group calls it).  z: the columns' transform fields at stride
// 2 N^2; sp: the columns' block-major search directions at stride 2 N^2.
// All three columns are transformed (a converged column carries zeros):
// the stage addresses and twiddles are formed once per stage and the three
// columns' loads and butterflies interleave.  Without a second transform
// buffer, a barrier separates the symbol's partner reads from the
// inverse's first writes.
template <int N, int H, int TS, bool INV>
__device__ __forceinline__ void vr2_mc(float* __restrict__ z, const float* __restrict__ tw, unsigned I, unsigned J) {
  constexpr int ZS = 2 * N * spectral_pitch(N), ZP = spectral_pitch(N);
  const unsigned i = I + (I & ~(H - 1u)), j = J + (J & ~(H - 1u));
  float* zb = z + 2 * (j * ZP + i);
  const float* tx = tw + 2 * ((I & (H - 1u)) * TS);
  const float* ty = tw + 2 * ((J & (H - 1u)) * TS);
  const Cx<float> wx = {tx[0], tx[1]}, wy = {ty[0], ty[1]};
  constexpr int DX = 2 * H, DY = 2 * H * ZP;
#pragma unroll
  for (int c = 0; c < MR_C; ++c) {
    float* q = zb + c * ZS;
    const Cx<float> a0 = {q[0], q[1]}, b0 = {q[DX], q[DX + 1]};
    const Cx<float> c0 = {q[DY], q[DY + 1]}, d0 = {q[DX + DY], q[DX + DY + 1]};
    Cx<float> o00, o10, o01, o11;
    if constexpr (!INV) {
      const Cx<float> A = cadd(a0, b0), B = cmul(csub(a0, b0), wx), C = cadd(c0, d0), D = cmul(csub(c0, d0), wx);
      o00 = cadd(A, C);
      o01 = cmul(csub(A, C), wy);
      o10 = cadd(B, D);
      o11 = cmul(csub(B, D), wy);
    } else {
      const Cx<float> bb = cmulc(b0, wx), dd = cmulc(d0, wx);
      const Cx<float> A = cadd(a0, bb), B = csub(a0, bb), C = cmulc(cadd(c0, dd), wy), D = cmulc(csub(c0, dd), wy);
      o00 = cadd(A, C);
      o10 = cadd(B, D);
      o01 = csub(A, C);
      o11 = csub(B, D);
    }
    q[0] = o00.re, q[1] = o00.im;
    q[DX] = o10.re, q[DX + 1] = o10.im;
    q[DY] = o01.re, q[DY + 1] = o01.im;
    q[DX + DY] = o11.re, q[DX + DY + 1] = o11.im;
  }
}

template <int N>
__device__ __forceinline__ void spectral_precond_mc(const float (&r)[MR_C][4][2], float* __restrict__ z,
                                                    float* __restrict__ sp, const SpectralRegs<N, float>& g, bool own,
                                                    int Ii, int Ji) {
  constexpr int M = SpectralRegs<N, float>::M;
  constexpr int H = N / 2;   // last inverse stage
  constexpr int TW = Tiles<N / 2>::TW;
  constexpr int ZS = 2 * N * spectral_pitch(N), ZP = spectral_pitch(N);
  asm volatile("" : "+v"(Ii), "+v"(Ji));
  const unsigned I = static_cast<unsigned>(Ii), J = static_cast<unsigned>(Ji);
  if (own) {
    float* zo = own_pts<N>(z, I, J);
#pragma unroll
    for (int c = 0; c < MR_C; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        zo[c * ZS + (k & 1) * 2 + (k >> 1) * 2 * ZP] = r[c][k][0],
                                                    zo[c * ZS + (k & 1) * 2 + (k >> 1) * 2 * ZP + 1] = r[c][k][1];
  }
  __syncthreads();
  // forward stages h = N/2 .. 2
  auto fwd = [&](auto hc) {
    constexpr int HH = decltype(hc)::value;
    if (own) vr2_mc<N, HH, N / (2 * HH), false>(z, g.tw, I, J);
    if constexpr (HH > TW) __syncthreads();
    else wave_sync();
  };
  fwd(std::integral_constant<int, N / 2>{});
  fwd(std::integral_constant<int, N / 4>{});
  fwd(std::integral_constant<int, N / 8>{});
  if constexpr (M >= 5) fwd(std::integral_constant<int, N / 16>{});
  Cx<float> v[MR_C][4];
  if (own)
#pragma unroll
    for (int c = 0; c < MR_C; ++c) spectral_fwd1<N, float>(v[c], z + c * ZS, I, J);
  __syncthreads();
  if (own)
#pragma unroll
    for (int c = 0; c < MR_C; ++c) spectral_symbol<N, float>(v[c], z + c * ZS, g, I, J);
  __syncthreads();   // every partner read precedes the overwrites below
  if (own)
#pragma unroll
    for (int c = 0; c < MR_C; ++c) spectral_inv1<N, float>(v[c], z + c * ZS, I, J);
  // inverse stages h = 2 .. N/4, in place
  auto inv = [&](auto hc) {
    constexpr int HH = decltype(hc)::value;
    if constexpr (HH > TW) __syncthreads();
    else wave_sync();
    if (own) vr2_mc<N, HH, N / (2 * HH), true>(z, g.tw, I, J);
  };
  inv(std::integral_constant<int, 2>{});
  inv(std::integral_constant<int, 4>{});
  if constexpr (M >= 5) inv(std::integral_constant<int, 8>{});
  if constexpr (H > TW) __syncthreads();
  else wave_sync();
  if (own) {   // last inverse stage, h = N/2, into the search directions
    const float* tx = g.tw + 2 * I;
    const float* ty = g.tw + 2 * J;
    const Cx<float> wx = {tx[0], tx[1]}, wy = {ty[0], ty[1]};
    constexpr int DX = 2 * H, DY = 2 * H * ZP;
    constexpr int OX = sp_at<N>(H, 0) - sp_at<N>(0, 0), OY = sp_at<N>(0, H) - sp_at<N>(0, 0);
    const int so = 4 * Tiles<N / 2>::bix(I >> 1, J >> 1) + (I & 1) + 2 * (J & 1);
    const bool pin = (I | J) == 0;
    const float* zb0 = z + 2 * (J * ZP + I);
#pragma unroll
    for (int c = 0; c < MR_C; ++c) {
      const float* zb = zb0 + c * ZS;
      const Cx<float> a0 = {zb[0], zb[1]}, b0 = cmulc(Cx<float>{zb[DX], zb[DX + 1]}, wx);
      const Cx<float> c0 = {zb[DY], zb[DY + 1]}, d0 = cmulc(Cx<float>{zb[DX + DY], zb[DX + DY + 1]}, wx);
      const Cx<float> A = cadd(a0, b0), B = csub(a0, b0), C = cmulc(cadd(c0, d0), wy), D = cmulc(csub(c0, d0), wy);
      const Cx<float> o00 = cadd(A, C), o10 = cadd(B, D), o01 = csub(A, C), o11 = csub(B, D);
      float* sb = sp + c * (2 * N * N) + so;
      sb[0] = pin ? 0.0f : o00.re;
      sb[N * N] = pin ? 0.0f : o00.im;
      sb[OX] = o10.re, sb[N * N + OX] = o10.im;
      sb[OY] = o01.re, sb[N * N + OY] = o01.im;
      sb[OX + OY] = o11.re, sb[N * N + OX + OY] = o11.im;
    }
  }
}

// Wave-uniform values pinned to scalar registers.
__device__ __forceinline__ float uni(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uni(double v) {
  const long long t = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readfirstlane(static_cast<int>(t));
  const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(t >> 32));
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Work-group sums of MR_C per-lane partials around a caller's barrier.
template <int NW>
__device__ __forceinline__ const float* wsum_post_mc(const float (&v)[MR_C], double* s_red, int& parity) {
  float* buf = reinterpret_cast<float*>(s_red + parity * (NW * MR_NV));
  parity ^= 1;
  float w[MR_C];
#pragma unroll
  for (int c = 0; c < MR_C; ++c) w[c] = wave_sum_to_last(v[c]);
  if ((threadIdx.x & 63) == 63)
#pragma unroll
    for (int c = 0; c < MR_C; ++c) buf[(threadIdx.x >> 6) * MR_C + c] = w[c];
  return buf;
}
template <int NW>
__device__ __forceinline__ void wsum_collect_mc(const float* buf, float (&out)[MR_C]) {
#pragma unroll
  for (int c = 0; c < MR_C; ++c) {
    float t = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += buf[w * MR_C + c];
    out[c] = t;
  }
}

template <int N, int WG>
__global__ void __launch_bounds__(WG, 2) k_lin2d_mr(const Lin2DArgs a) {
  using P = Pad<N, N>;
  using L = MrLds<N, WG>;
  constexpr int NW = WG / 64;
  constexpr int NN = N * N;
  constexpr int NB = N / 2;
  constexpr int ZS = 2 * N * N;
  static_assert(NB * NB == WG || (N == 8 && WG == 64), "one 2x2 block per lane");
  const int tid = threadIdx.x;
  const int b = a.rve_list[blockIdx.x];
  if (a.skip && a.skip[b]) return;   // handled elsewhere (whole work-group)

  extern __shared__ __align__(16) unsigned char smem[];
  double* s_red = reinterpret_cast<double*>(smem + L::red);
  double* s_sc = reinterpret_cast<double*>(smem + L::sc);    // [PN] FP64 element scales
  float* s_sc32 = reinterpret_cast<float*>(smem + L::sc32);  // [PN] FP32 element scales
  float* s_u = reinterpret_cast<float*>(smem + L::u);        // [3][2][N*N] search directions
  float* s_x = reinterpret_cast<float*>(smem + L::x);        // exchange slots / transform fields
  double* s_st = reinterpret_cast<double*>(smem + L::u);     // [2][PN] FP64 column (refinement passes only)
  int parity = 0;

  double kv64[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) kv64[t] = a.kv64[t];
  const double* KwF = a.KwF64;   // [8][NF], uniform
  float mcI[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) mcI[t] = static_cast<float>(a.modes64[t]);

  // ---- ownership: wave tiles of 2x2 node blocks ---------------------------
  const bool own = tid < NB * NB;
  const int I = own ? Tiles<NB>::I_of(tid) : 0;
  const int J = own ? Tiles<NB>::J_of(tid) : 0;
  const int i0 = 2 * I, j0 = 2 * J;
  bool exists[4], dof[4];
  int pidx[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = i0 + (k & 1), j = j0 + (k >> 1);
    exists[k] = own;
    dof[k] = own && (i | j) != 0;   // corner node 0 is pinned
    pidx[k] = P::at(i, j);
  }
  const int base = P::at(i0 - 1, j0 - 1);
  auto node_of = [&](int k) { return (j0 + (k >> 1)) * N + i0 + (k & 1); };
  const int Il = (I + NB - 1) % NB, Jb = (J + NB - 1) % NB, Ir = (I + 1) % NB, Jt = (J + 1) % NB;
  const int t_l = Tiles<NB>::bix(Il, J), t_b = Tiles<NB>::bix(I, Jb), t_d = Tiles<NB>::bix(Il, Jb);
  const int b_own = Tiles<NB>::bix(I, J), b_r = Tiles<NB>::bix(Ir, J), b_t = Tiles<NB>::bix(I, Jt),
            b_d = Tiles<NB>::bix(Ir, Jt);

  // ---- element scales (mu of the phase), padded ---------------------------
  const double* par = a.params + static_cast<size_t>(b) * 4;
  const double mu0 = par[1], mu1 = par[3];
  const uint8_t* ph = a.phase + a.phase_off[b];
  double ssum = 0.0;
  constexpr int PE = (NN + WG - 1) / WG;
  uint8_t phv[PE];
#pragma unroll
  for (int q = 0; q < PE; ++q) {   // (clamped index: no branch around the loads)
    const int e = tid + q * WG;
    phv[q] = ph[e < NN ? e : NN - 1];
  }
#pragma unroll
  for (int q = 0; q < PE; ++q) {
    const int e = tid + q * WG;
    if (e >= NN) continue;
    const double s = phv[q] ? mu1 : mu0;
    put_halo<N, N>(s_sc, e % N, e / N, s);
    put_halo<N, N>(s_sc32, e % N, e / N, static_cast<float>(s));
    ssum += s;
  }
  SpectralRegs<N, float> sreg;
  spectral_setup<N, float>(sreg, a.fft_tab, s_x + L::xlen / 4, own, I, J);
  {
    double red[1] = {ssum};
    wg_sum<1, NW, MR_NV>(red, s_red, parity);   // (its barrier also publishes the scales and tables)
    ssum = uni(red[0]);
  }
  const double* eb = s_sc + base;
  float esc[2][2];   // scales of the thread's four elements
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2) esc[c][a2] = s_sc32[base + (c + 1) * P::PW + a2 + 1];

  const int64_t fo = a.foff[b];
  constexpr int64_t flen = 2 * NN;
  double* Xb = a.X + fo * (NF + 1);
  const double V = a.volume;

  // own nodes of a column in HBM (16-byte accesses: fields start at even offsets)
  auto ld_own = [&](const double* src, double (&v)[4][2]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double2 t = make_double2(0.0, 0.0);
      if (exists[k]) t = reinterpret_cast<const double2*>(src)[node_of(k)];
      v[k][0] = t.x;
      v[k][1] = t.y;
    }
  };
  auto st_own = [&](double* dst, const double (&v)[4][2]) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (exists[k]) reinterpret_cast<double2*>(dst)[node_of(k)] = make_double2(v[k][0], v[k][1]);
  };
  // cold start: the columns start from zero (and so does x_r, not solved here)
  if (!(a.flags & RVE_WARM)) {
    const double z0[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
    for (int c = 0; c < MR_C; ++c) st_own(Xb + c * flen, z0);
  }
  {
    const double z0[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    st_own(Xb + NF * flen, z0);
  }
  bool xzero = !(a.flags & RVE_WARM);   // every column zero (no FP64 operator needed)

  const float tinI = static_cast<float>(a.tol_in * a.tol_in);
  const double tol2 = a.tol * a.tol;
  int iters = 0, nmv64 = 0;
  bool all_ok = true;
  double worst = 0.0;
  bool act[MR_C];   // columns that still need an inner solve (uniform)

#pragma unroll 1
  for (int sweep = 0;; ++sweep) {
    // ---- FP64 residuals of the three columns, norms and energy products ----
    // E[i][c] = b_i . x_c + x_i . r_c: the x . r term is a correction of
    // relative size rve_tol, so it takes r in FP32 (the copy kept for the
    // inner solve) in a second pass over the columns.
    double red[MR_NV];
#pragma unroll
    for (int t = 0; t < MR_NV; ++t) red[t] = 0.0;
    float rf[MR_C][4][2];   // r_c (FP32) for the inner solve
#pragma unroll 1
    for (int c = 0; c < MR_C; ++c) {
      double y[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
      if (!xzero) {
        double xc[4][2];
        ld_own(Xb + c * flen, xc);
        __syncthreads();   // earlier readers of the FP64 column (and of u) done
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          put_halo<N, N>(s_st, i0 + (k & 1), j0 + (k >> 1), xc[k][0]);
          put_halo<N, N>(s_st + P::PN, i0 + (k & 1), j0 + (k >> 1), xc[k][1]);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) mv_node64<N, N>(s_st + base, eb, kv64, k & 1, k >> 1, y[k]);
        ++nmv64;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int di = k & 1, dj = k >> 1;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          double r = 0.0;
          if (dof[k]) {
            const double bk = bF_entry<N, N>(eb, KwF, di, dj, d, c);
            r = bk - y[k][d];
            red[2 * c] += r * r;
            red[2 * c + 1] += bk * bk;
          }
          rf[c][k][d] = static_cast<float>(r);
        }
      }
    }
    if (!xzero) {
#pragma unroll 1
      for (int c = 0; c < MR_C; ++c) {
        double xc[4][2];
        ld_own(Xb + c * flen, xc);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (!dof[k]) continue;
          const int di = k & 1, dj = k >> 1;
#pragma unroll
          for (int d = 0; d < 2; ++d)
#pragma unroll
            for (int i = 0; i < MR_C; ++i) {
              red[2 * MR_C + i * MR_C + c] += bF_entry<N, N>(eb, KwF, di, dj, d, i) * xc[k][d];
              red[2 * MR_C + c * MR_C + i] += xc[k][d] * static_cast<double>(rf[i][k][d]);
            }
        }
      }
    }
    wg_sum<MR_NV, NW, MR_NV>(red, s_red, parity);
    bool any = false;
    float rsc[MR_C];   // 1 / ||r_c|| (FP32) for the columns that go on
    double rnrm[MR_C];
#pragma unroll
    for (int c = 0; c < MR_C; ++c) {
      const double rel = red[2 * c + 1] > 0.0 ? sqrt(red[2 * c] / red[2 * c + 1]) : 0.0;
      const bool accept = red[2 * c + 1] == 0.0 || red[2 * c] <= tol2 * red[2 * c + 1];
      act[c] = !accept && sweep < a.max_ir;
      if (!act[c]) {
        worst = rel > worst ? rel : worst;
        if (!accept) all_ok = false;
      }
      any = any || act[c];
      rnrm[c] = uni(sqrt(red[2 * c]));
      rsc[c] = red[2 * c] > 0.0 ? static_cast<float>(1.0 / rnrm[c]) : 0.0f;
    }
    if (!any) {   // every column accepted (or given up): energy-form condensation
      if (tid == 0) {
        double* Cb = a.Cbar + static_cast<size_t>(b) * NF * NF;
#pragma unroll
        for (int i = 0; i < NF; ++i)
#pragma unroll
          for (int j = 0; j < NF; ++j)
            Cb[i * NF + j] = (ssum * a.KFF64[i * NF + j] - red[2 * MR_C + i * MR_C + j]) / V;
#pragma unroll   // x_r = 0: Phat = Pbar
        for (int i = 0; i < NF; ++i) a.Phat[static_cast<size_t>(b) * NF + i] = a.Pbar[static_cast<size_t>(b) * NF + i];
      }
      break;
    }
    // ---- inner PCG of the active columns on r_c / ||r_c|| (FP32) ----------
    // Every column passes through the transform and the operator (a column
    // that is not active carries zeros); only the updates are per column.
    unsigned actm = 0;   // active columns (uniform bit mask)
#pragma unroll
    for (int c = 0; c < MR_C; ++c) actm |= act[c] ? (1u << c) : 0u;
    actm = __builtin_amdgcn_readfirstlane(actm);
    const unsigned solvem = actm;
    float xi[MR_C][4][2], pv[MR_C][4][2], qv[MR_C][4][2];
    float gam0[MR_C], gam_old[MR_C];
#pragma unroll
    for (int c = 0; c < MR_C; ++c) {
      gam0[c] = 0.0f;
      gam_old[c] = 1.0f;
      const float sc = (actm >> c) & 1u ? rsc[c] : 0.0f;
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          rf[c][k][d] = dof[k] ? rf[c][k][d] * sc : 0.0f;
          xi[c][k][d] = pv[c][k][d] = qv[c][k][d] = 0.0f;
        }
    }
    __syncthreads();   // the FP64 column's readers done before u and the transforms overwrite it
#pragma unroll 1
    for (int it = 0;; ++it) {
      spectral_precond_mc<N>(rf, s_x, s_u, sreg, own, I, J);
      __syncthreads();   // u visible (and every read of the transform fields done)
      float gpart[MR_C], fo[MR_C][2][2][2];
#pragma unroll
      for (int c = 0; c < MR_C; ++c) {
        gpart[c] = 0.0f;
        float o[2][4];
#pragma unroll
        for (int d = 0; d < 2; ++d) ld4(s_u + c * ZS + d * NN + 4 * b_own, o[d]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) gpart[c] = fma(rf[c][k][d], o[d][k], gpart[c]);
        mv_modes_post<N, N, WG, float>(s_u + c * ZS, esc, mcI, s_x + c * 12 * WG, b_own, b_r, b_t, b_d, tid, fo[c]);
      }
      const float* rb = wsum_post_mc<NW>(gpart, s_red, parity);
      __syncthreads();   // exchange slots and the r.u wave totals visible
      float gam[MR_C];
      wsum_collect_mc<NW>(rb, gam);
#pragma unroll
      for (int c = 0; c < MR_C; ++c) gam[c] = uni(gam[c]);
      unsigned m = actm;
#pragma unroll
      for (int c = 0; c < MR_C; ++c) {
        if (it == 0) gam0[c] = gam[c];
        if (it >= a.max_it || !(gam[c] > tinI * gam0[c]) || !(gam[c] > 0.0f)) m &= ~(1u << c);
      }
      actm = __builtin_amdgcn_readfirstlane(m);
      if (actm == 0) break;
      float qpart[MR_C];
#pragma unroll
      for (int c = 0; c < MR_C; ++c) {
        float wv[4][2];
        mv_modes_gather<WG, float>(s_x + c * 12 * WG, fo[c], t_l, t_b, t_d, wv);
        const float beta = (it == 0 || !((actm >> c) & 1u)) ? 0.0f : gam[c] / gam_old[c];
        float uo[2][4];
#pragma unroll
        for (int d = 0; d < 2; ++d) ld4(s_u + c * ZS + d * NN + 4 * b_own, uo[d]);
        qpart[c] = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            pv[c][k][d] = fma_keep(pv[c][k][d], beta, uo[d][k]);
            qv[c][k][d] = fma_keep(qv[c][k][d], beta, wv[k][d]);
            qpart[c] = fma(pv[c][k][d], qv[c][k][d], qpart[c]);
          }
      }
      const float* qb = wsum_post_mc<NW>(qpart, s_red, parity);
      __syncthreads();
      float pq[MR_C];
      wsum_collect_mc<NW>(qb, pq);
#pragma unroll
      for (int c = 0; c < MR_C; ++c) pq[c] = uni(pq[c]);
      m = actm;
#pragma unroll
      for (int c = 0; c < MR_C; ++c)
        if (!(pq[c] > 0.0f)) m &= ~(1u << c);   // exact solution or loss of definiteness
      actm = __builtin_amdgcn_readfirstlane(m);
#pragma unroll
      for (int c = 0; c < MR_C; ++c) {
        const bool on = (actm >> c) & 1u;
        const float alpha = on ? gam[c] / pq[c] : 0.0f;
        iters += on ? 1 : 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            xi[c][k][d] = fma(alpha, pv[c][k][d], xi[c][k][d]);
            // (the pinned node's entry stays zero: it must not reach the transform)
            rf[c][k][d] = (on && dof[k]) ? fma(-alpha, qv[c][k][d], rf[c][k][d]) : 0.0f;
          }
        if (on) gam_old[c] = gam[c];
      }
    }
    // ---- x_c += ||r_c|| x_inner (FP64, own nodes in HBM) -------------------
#pragma unroll
    for (int c = 0; c < MR_C; ++c) {
      if (!((solvem >> c) & 1u)) continue;   // accepted (or given up): unchanged
      double v[4][2];
      ld_own(Xb + c * flen, v);
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 2; ++d) v[k][d] += rnrm[c] * static_cast<double>(xi[c][k][d]);
      st_own(Xb + c * flen, v);
    }
    xzero = false;
  }
  if (tid == 0) {
    a.relres[b] = worst;
    a.iters[b] = static_cast<double>(iters);
    a.mv64[b] = static_cast<double>(nmv64);
    if (!all_ok) atomicAdd(a.fail_count, 1);
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

template <typename TI, int NRHS, int N1, int N2, bool FFT = false, bool DENSE = false>
static int launch_t(const Lin2DArgs& a, int n_launch, hipStream_t s) {
  constexpr int WG = DENSE ? 256 : wg_for(N1, N2);
  constexpr size_t lds = lin2d_lds_bytes_t(N1, N2, WG, NRHS, static_cast<int>(sizeof(TI)), FFT, DENSE);
  static_assert(lds <= 160 * 1024, "RVE too large for the LDS-resident solver");
  static_assert(!FFT || N1 != 48 || WG == 576, "the 48-element transform assumes one block per lane");
  auto kern = &k_lin2d<TI, NRHS, N1, N2, WG, FFT, DENSE>;
  if (lds > 64 * 1024)
    FE2_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  hipLaunchKernelGGL(kern, dim3(n_launch), dim3(WG), lds, s, a);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

template <int N>
static int launch_mr(const Lin2DArgs& a, int n_launch, hipStream_t s) {
  constexpr int WG = (N / 2) * (N / 2);
  constexpr size_t lds = MrLds<N, WG>::total;
  static_assert(lds <= 80 * 1024, "two work-groups per CU");
  auto kern = &k_lin2d_mr<N, WG>;
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
  if (a.flags & RVE_ASSEMBLE) return set_error("assembly runs without right-hand sides"), FE2_EINVAL;
  if constexpr (lin2d_dense_size(N1, N2)) {
    if (a.flags & RVE_DENSE) {
      if (precision != FE2_PREC_FP32_IR) return set_error("the dense solve factors in FP32"), FE2_ENOTSUP;
      return nrhs == NF ? launch_t<float, NF, N1, N2, false, true>(a, n_launch, s)
                        : launch_t<float, NF + 1, N1, N2, false, true>(a, n_launch, s);
    }
  } else {
    if (a.flags & RVE_DENSE) return set_error("no dense solve for this RVE size"), FE2_ENOTSUP;
  }
  if constexpr (N1 == N2 && (N1 == 16 || N1 == 32)) {
    // the three columns of X_F in one loop (FP32 inner precision, spectral)
    if ((a.flags & RVE_FFT) && (a.flags & RVE_MC) && precision != FE2_PREC_FP64 && nrhs == NF &&
        !(a.flags & (RVE_RONLY | RVE_ASSEMBLE)) && a.fft_tab)
      return launch_mr<N1>(a, n_launch, s);
  }
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
