// RVE element integration, periodic null-space solve and condensation for
// two-dimensional finite-strain RVEs (Q4, plane strain, polyconvex phases),
// one work-group per RVE.
//
// Method (Hesch, Schmidt, Schuss, arXiv:2312.12771):
//   * micro gradient F~ = F_b + grad w~ (Eq. (11)); per phase the
//     Mooney-Rivlin family of Eqs. (7)-(8) in the plane-strain form of
//     Eq. (59): P = c0 F + c1 H, H = cof F (Eq. (1)), with c0 = 2(a+b),
//     c1 = 2bJ + k(J-1) - 2(a+2b)/J, and tangent
//     dP/dF = c0 I + c1 dH/dF + c1' H (x) H, c1' = 2b + k + 2(a+2b)/J^2
//     (the compressible Neo-Hookean law is a = mu/2, b = 0, k = lambda);
//   * micro residual r_b = sum_l eta_l G^T P~ (Eq. (35)), stress integral
//     (Eq. (17)), K_FF = int A;
//   * K_ww [X_F | x_r] = [K_wF | r_b] with the periodic null space of
//     condition (iii) in Eq. (15) (periodic nodes, pinned corner) and the
//     condensation of Eqs. (46)-(48).
//
// GPU design
//   * Element passes: thread t integrates elements t, t+WG, ... one at a
//     time (the register footprint is that of one element) and writes its
//     eight nodal force entries to LDS; every node then gathers the four
//     corner entries it receives.  No atomics, deterministic order.
//   * The tangent is never stored: each operator application recomputes F~,
//     J, H, c1, c1' at the four Gauss points from the linearisation state.
//     The inner (TI) operator reads the state and the search direction from
//     halo-padded LDS copies; the FP64 passes read w and x from global
//     memory (they run a few times per column only).
//   * K_wF columns are applied implicitly: the refinement residual of column
//     j is G^T A (e_j - grad x) per element, and K_Fw x = sum eta A grad x.
//   * Precision as in the small-strain kernel: inner PCG in TI, FP64
//     residual refinement, energy-form condensation.
//   * Preconditioner: Jacobi, or (square 8/16/32 RVEs) the inverse of the
//     periodic operator of a homogeneous small-strain reference medium
//     (spectral2d.hpp).  The tangent of a uniformly elliptic state is
//     spectrally equivalent to it, with constants set by the spread of the
//     tangent moduli, not by the mesh.
#include <type_traits>

#include "rve2d_common.hpp"
#include "spectral2d.hpp"

namespace fe2 {

using namespace rve2d;

namespace {

constexpr int NF = 4;   // F11, F12, F21, F22

// P = c0 F + c1 H and the coefficients of the tangent at gradient F
// (row-major); H = cof F in plane strain.
template <typename V>
__device__ __forceinline__ void law(const V (&F)[4], V c0, V b2, V k, V a2b2, V (&P)[4], V& c1, V& dc1,
                                    V (&H)[4]) {
  const V J = F[0] * F[3] - F[1] * F[2];
  H[0] = F[3];
  H[1] = -F[2];
  H[2] = -F[1];
  H[3] = F[0];
  const V rJ = V(1) / J;
  c1 = b2 * J + k * (J - V(1)) - a2b2 * rJ;
  dc1 = b2 + k + a2b2 * rJ * rJ;
#pragma unroll
  for (int t = 0; t < 4; ++t) P[t] = c0 * F[t] + c1 * H[t];
}

// tangent coefficients only (inner operator: P is not needed)
template <typename V>
__device__ __forceinline__ void law_tangent(const V (&F)[4], V b2, V k, V a2b2, V& c1, V& dc1) {
  const V J = F[0] * F[3] - F[1] * F[2];
  const V rJ = V(1) / J;
  c1 = b2 * J + k * (J - V(1)) - a2b2 * rJ;
  dc1 = b2 + k + a2b2 * rJ * rJ;
}

// s = A g, A = c0 I + c1 dH/dF + dc1 H (x) H; dH/dF g = (g22, -g21, -g12, g11)
// and H = (F22, -F21, -F12, F11)
template <typename V>
__device__ __forceinline__ void tangent_apply_F(V c0, V c1, V dc1, const V (&F)[4], const V (&g)[4], V (&s)[4]) {
  const V hg = dc1 * (F[3] * g[0] - F[2] * g[1] - F[1] * g[2] + F[0] * g[3]);
  s[0] = c0 * g[0] + c1 * g[3] + F[3] * hg;
  s[1] = c0 * g[1] - c1 * g[2] - F[2] * hg;
  s[2] = c0 * g[2] - c1 * g[1] - F[1] * hg;
  s[3] = c0 * g[3] + c1 * g[0] + F[0] * hg;
}

// dN_m/dX and dN_m/dY of corner m at Gauss point g (xi fastest) of a box
// element: s_x(m) (1 + s_y(m) eta_g) / (2 h1) and s_y(m) (1 + s_x(m) xi_g) / (2 h2).
__host__ __device__ constexpr double gp_fac(int s, int q) {
  return 1.0 + s * (2 * q - 1) * 0.57735026918962576451;
}
template <typename V>
__device__ __forceinline__ V dNx(int m, int g, V r2h1) {
  return V(sgn_x(m) * gp_fac(sgn_y(m), g >> 1)) * r2h1;
}
template <typename V>
__device__ __forceinline__ V dNy(int m, int g, V r2h2) {
  return V(sgn_y(m) * gp_fac(sgn_x(m), g & 1)) * r2h2;
}

// displacement gradient at Gauss point g from the element's nodal values
template <typename V>
__device__ __forceinline__ void grad_at(const V (&u)[4][2], int g, V r1, V r2, V (&G)[4]) {
  V g0 = V(0), g1 = V(0), g2 = V(0), g3 = V(0);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const V nx = dNx<V>(m, g, r1), ny = dNy<V>(m, g, r2);
    g0 += nx * u[m][0];
    g1 += ny * u[m][0];
    g2 += nx * u[m][1];
    g3 += ny * u[m][1];
  }
  G[0] = g0;
  G[1] = g1;
  G[2] = g2;
  G[3] = g3;
}

// f_m += wt G_m^T s
template <typename V>
__device__ __forceinline__ void add_force(V (&f)[4][2], int g, V r1, V r2, V wt, const V (&s)[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const V nx = dNx<V>(m, g, r1), ny = dNy<V>(m, g, r2);
    f[m][0] += wt * (nx * s[0] + ny * s[1]);
    f[m][1] += wt * (nx * s[2] + ny * s[3]);
  }
}

struct Phase {
  double c0, b2, k, a2b2;   // 2(a+b), 2b, k, 2(a+2b)
};

}  // namespace

// LDS layout: reduction buffers | phase ids | w in TI (padded) |
// union { FP64 element forces [8][NN],
//         TI element forces [8][NN] + TI search direction (padded) [2][PN] }
constexpr int RED_NV = 23;   // widest work-group reduction
__host__ __device__ constexpr size_t fin2d_red_doubles(int nw, int nrhs) {
  return 2 * static_cast<size_t>(nw) * RED_NV + 0 * nrhs;
}
__host__ __device__ constexpr size_t fin2d_pn(int n1, int n2) {
  return static_cast<size_t>(rve2d::pad_w(n1)) * rve2d::pad_w(n2);
}
__host__ __device__ constexpr size_t fin2d_off_ph(int wg, int nrhs) { return fin2d_red_doubles(wg / 64, nrhs) * 8; }
__host__ __device__ constexpr size_t fin2d_off_w(int n1, int n2, int wg, int nrhs) {
  return (fin2d_off_ph(wg, nrhs) + static_cast<size_t>(n1) * n2 + 15) & ~static_cast<size_t>(15);
}
__host__ __device__ constexpr size_t fin2d_off_u(int n1, int n2, int wg, int nrhs, size_t ti) {
  return (fin2d_off_w(n1, n2, wg, nrhs) + 2 * fin2d_pn(n1, n2) * ti + 15) & ~static_cast<size_t>(15);
}
// The force region holds the FP64 element forces [8][NN] during the FP64
// passes, and the inner forces [8][NN] plus the search direction [2][PN]
// (and, spectral, the two transform fields [2][N*pitch][2]) during the
// inner solve; the spectral twiddles and partner map follow it.
__host__ __device__ constexpr size_t fin2d_off_z(int n1, int n2, size_t ti) {
  return (8 * static_cast<size_t>(n1) * n2 * ti + 2 * fin2d_pn(n1, n2) * ti + 15) & ~static_cast<size_t>(15);
}
__host__ __device__ constexpr size_t fin2d_region(int n1, int n2, size_t ti, bool fft) {
  const size_t a = 8 * static_cast<size_t>(n1) * n2 * 8;
  const size_t b = fin2d_off_z(n1, n2, ti) + (fft ? 4 * static_cast<size_t>(n1) * spectral_pitch(n1) * ti : 0);
  return (a > b ? a : b + 15) & ~static_cast<size_t>(15);
}
__host__ __device__ constexpr size_t fin2d_lds_bytes_t(int n1, int n2, int wg, int nrhs, size_t ti, bool fft = false) {
  return fin2d_off_u(n1, n2, wg, nrhs, ti) + fin2d_region(n1, n2, ti, fft) +
         (fft ? 2 * static_cast<size_t>(lin2d_spectral_twiddles(n1)) * ti + n1 + 2 : 0);
}

// Occupancy: the FP32 instances are held to two work-groups per CU (256
// VGPRs per lane) so that the latency of the recomputed tangents overlaps
// across waves; the FP64 instances keep their full register budget.
template <typename T> constexpr int kFinMinBlocks = 1;
template <> constexpr int kFinMinBlocks<float> = 2;
template <typename TI, int NRHS, int N1, int N2, int WG, bool FFT>
__global__ void __launch_bounds__(WG, kFinMinBlocks<TI>) k_fin2d(const Fin2DArgs a) {
  using P = Pad<N1, N2>;
  constexpr int NW = WG / 64;
  constexpr int NN = N1 * N2;
  constexpr int NPT = (NN + WG - 1) / WG;   // owned nodes per thread
  const int tid = threadIdx.x;
  const int b = a.rve_list[blockIdx.x];
  if (a.skip && a.skip[b]) return;   // handled elsewhere (whole work-group)

  extern __shared__ __align__(16) unsigned char smem[];
  double* s_red = reinterpret_cast<double*>(smem);
  uint8_t* s_ph = smem + fin2d_off_ph(WG, NRHS);
  TI* s_w = reinterpret_cast<TI*>(smem + fin2d_off_w(N1, N2, WG, NRHS));   // [2][PN]
  unsigned char* s_u = smem + fin2d_off_u(N1, N2, WG, NRHS, sizeof(TI));
  double* s_ef = reinterpret_cast<double*>(s_u);   // [8][NN] FP64 element forces
  TI* s_efI = reinterpret_cast<TI*>(s_u);          // [8][NN] TI element forces
  TI* s_p = s_efI + 8 * NN;                        // [2][PN] TI search direction
  TI* s_z = reinterpret_cast<TI*>(s_u + fin2d_off_z(N1, N2, sizeof(TI)));   // spectral: [2][N*pitch][2]
  TI* s_tw = reinterpret_cast<TI*>(s_u + fin2d_region(N1, N2, sizeof(TI), FFT));   // spectral: twiddles, map
  int parity = 0;
  static_assert(!FFT || (N1 == N2 && (N1 == 8 || N1 == 16 || N1 == 32)), "spectral sizes: 8, 16, 32");
  // spectral preconditioner: the transform works on 2x2 node blocks, one
  // per thread in wave tiles (the nodes the thread owns for the operator
  // are another set; the residual passes through LDS in natural order)
  constexpr int NB = FFT ? N1 / 2 : 8;
  const bool sown = FFT && tid < NB * NB;
  const int sI = sown ? Tiles<NB>::I_of(tid) : 0, sJ = sown ? Tiles<NB>::J_of(tid) : 0;
  struct NoSpectral {};
  using SpecRegs = typename std::conditional<FFT, SpectralRegs<FFT ? N1 : 8, TI>, NoSpectral>::type;
  SpecRegs sreg;
  if constexpr (FFT) {
    const TI* ftab;
    if constexpr (sizeof(TI) == 4) ftab = reinterpret_cast<const TI*>(a.fft_tab);
    else ftab = reinterpret_cast<const TI*>(a.fft_tab64);
    spectral_setup<N1, TI>(sreg, ftab, s_tw, sown, sI, sJ);   // visible after the next barrier
  }

  // ---- material, geometry, state ---------------------------------------
  const double* par = a.params + static_cast<size_t>(b) * 6;
  Phase mp[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double al = par[3 * q], be = par[3 * q + 1], ka = par[3 * q + 2];
    mp[q].c0 = 2.0 * (al + be);
    mp[q].b2 = 2.0 * be;
    mp[q].k = ka;
    mp[q].a2b2 = 2.0 * (al + 2.0 * be);
  }
  const double r2h1 = 0.5 / a.h1, r2h2 = 0.5 / a.h2;
  const double wt = 0.25 * a.h1 * a.h2;
  double Fb[NF];
#pragma unroll
  for (int t = 0; t < NF; ++t) Fb[t] = a.macro[static_cast<size_t>(b) * NF + t];

  const uint8_t* ph = a.phase + a.phase_off[b];
  const int64_t fo = a.foff[b];
  constexpr int64_t flen = 2 * NN;
  const double* wb = a.w + fo;
  double* Xb = a.X + fo * (NF + 1);
  for (int n = tid; n < NN; n += WG) {
    const int i = n % N1, j = n / N1;
    s_ph[n] = ph[n];
    put_halo<N1, N2>(s_w, i, j, static_cast<TI>(wb[2 * n]));
    put_halo<N1, N2>(s_w + P::PN, i, j, static_cast<TI>(wb[2 * n + 1]));
  }

  // Owned nodes n = tid + k WG.  Node (i, j) is corner 0 of element (i, j),
  // 1 of (i-1, j), 2 of (i-1, j-1) and 3 of (i, j-1) (periodic).
  auto node_ok = [&](int k) { return tid + k * WG < NN; };
  auto gather = [&](const auto* ef, int k, int d) {
    const int n = tid + k * WG;
    const int i = n % N1, j = n / N1;
    const int im = i == 0 ? N1 - 1 : i - 1;
    const int jm = j == 0 ? N2 - 1 : j - 1;
    return ef[(2 * 0 + d) * NN + j * N1 + i] + ef[(2 * 1 + d) * NN + j * N1 + im] +
           ef[(2 * 2 + d) * NN + jm * N1 + im] + ef[(2 * 3 + d) * NN + jm * N1 + i];
  };
  // nodal values of element e from a global FP64 field (periodic numbering)
  auto elem_vals_g = [&](const double* f, int e, double (&v)[4][2]) {
    const int i = e % N1, j = e / N1;
    const int ip = i == N1 - 1 ? 0 : i + 1;
    const int jp = j == N2 - 1 ? 0 : j + 1;
    const int nd[4] = {j * N1 + i, j * N1 + ip, jp * N1 + ip, jp * N1 + i};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      v[m][0] = f[2 * nd[m]];
      v[m][1] = f[2 * nd[m] + 1];
    }
  };
  // nodal values of element e from a padded LDS field
  auto elem_vals_s = [&](const TI* f, int e, TI (&v)[4][2]) {
    const int o = P::at(e % N1, e / N1);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int om = o + cyo(m) * P::PW + cxo(m);
      v[m][0] = f[om];
      v[m][1] = f[P::PN + om];
    }
  };

  // ---- FP64 element passes ------------------------------------------------
  // mode 0: forces G^T P~ at the state; acc = [int P (4) | K_FF (16) | #(J<=0) |
  //         sum of the squared entries of a rounding bound of the element
  //         forces: G^T applied, with absolute values, to |c0 F| + (|2b J| +
  //         |k (J - 1)| + |2(a + 2b) / J|) |H|, the terms whose cancellation
  //         sets the FP64 rounding level of r_b]
  // mode 1: forces G^T A (e_kc - grad x) (kc < 0: -G^T A grad x) with x the
  //         global field xg (zero when xg is null); acc[0..3] = K_Fw x when
  //         want_k; acc[20] = sum of the squared element force entries
  // mode 2: diagonal entries of the element matrices
  auto pass64 = [&](auto mode_c, int kc, const double* xg, bool want_k, double (&acc)[22]) {
    constexpr int mode = decltype(mode_c)::value;
#pragma unroll
    for (int t = 0; t < 22; ++t) acc[t] = 0.0;
#pragma unroll 1
    for (int e = tid; e < NN; e += WG) {
      const Phase q = s_ph[e] ? mp[1] : mp[0];
      double we[4][2], xe[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
      elem_vals_g(wb, e, we);
      if constexpr (mode == 1) {
        if (xg) elem_vals_g(xg, e, xe);
      }
      double f[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
      double fa[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};   // mode 0: rounding bound of f
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        double F[4], Pk[4], H[4], c1, dc1, s[4];
        grad_at<double>(we, g, r2h1, r2h2, F);
#pragma unroll
        for (int t = 0; t < 4; ++t) F[t] += Fb[t];
        law<double>(F, q.c0, q.b2, q.k, q.a2b2, Pk, c1, dc1, H);
        if constexpr (mode == 0) {
          if (!(F[0] * F[3] - F[1] * F[2] > 0.0)) acc[20] += 1.0;
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[t] += wt * Pk[t];
          if (want_k) {
#pragma unroll
            for (int cj = 0; cj < 4; ++cj) {   // K_FF column cj = int A e_cj
              double ej[4] = {0, 0, 0, 0}, col[4];
              ej[cj] = 1.0;
              tangent_apply_F<double>(q.c0, c1, dc1, F, ej, col);
#pragma unroll
              for (int t = 0; t < 4; ++t) acc[4 + 4 * t + cj] += wt * col[t];
            }
          }
          add_force<double>(f, g, r2h1, r2h2, wt, Pk);
          const double J = F[0] * F[3] - F[1] * F[2];
          const double c1a = fabs(q.b2 * J) + fabs(q.k * (J - 1.0)) + fabs(q.a2b2 / J);
          double Pa[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) Pa[t] = fabs(q.c0 * F[t]) + c1a * fabs(H[t]);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const double nx = fabs(dNx<double>(m, g, r2h1)), ny = fabs(dNy<double>(m, g, r2h2));
            fa[m][0] += wt * (nx * Pa[0] + ny * Pa[1]);
            fa[m][1] += wt * (nx * Pa[2] + ny * Pa[3]);
          }
        } else if constexpr (mode == 1) {
          double gx[4], dd[4];
          grad_at<double>(xe, g, r2h1, r2h2, gx);
#pragma unroll
          for (int t = 0; t < 4; ++t) dd[t] = ((t == kc) ? 1.0 : 0.0) - gx[t];
          tangent_apply_F<double>(q.c0, c1, dc1, F, dd, s);
          add_force<double>(f, g, r2h1, r2h2, wt, s);
          if (want_k) {
            double kx[4];
            tangent_apply_F<double>(q.c0, c1, dc1, F, gx, kx);
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] += wt * kx[t];
          }
        } else {
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            // g = G_m e_d has (nx, ny) in the two rows of component d; the
            // dH/dF part vanishes on such g
            const double nx = dNx<double>(m, g, r2h1), ny = dNy<double>(m, g, r2h2);
            const double hx0 = H[0] * nx + H[1] * ny, hx1 = H[2] * nx + H[3] * ny;
            const double n2 = nx * nx + ny * ny;
            f[m][0] += wt * (q.c0 * n2 + dc1 * hx0 * hx0);
            f[m][1] += wt * (q.c0 * n2 + dc1 * hx1 * hx1);
          }
        }
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          s_ef[(2 * m + d) * NN + e] = f[m][d];
          if constexpr (mode == 1) acc[20] += f[m][d] * f[m][d];
          if constexpr (mode == 0) acc[21] += fa[m][d] * fa[m][d];
        }
    }
  };

  // ---- a3: residual, stress integral, K_FF --------------------------------
  const bool solve = (a.flags & RVE_SOLVE) != 0;
  double rsize2;     // squared rounding bound of the element-level terms of r_b
  __syncthreads();   // phases and state staged
  {
    double red[23];
    {
      double acc[22];
      pass64(std::integral_constant<int, 0>(), 0, nullptr, solve && !(a.flags & RVE_RONLY), acc);
#pragma unroll
      for (int t = 0; t < 20; ++t) red[t] = acc[t];
      red[21] = acc[20];
      red[22] = acc[21];
    }
    red[20] = 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      if (!node_ok(k)) continue;
      const int n = tid + k * WG;
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const double rv = n != 0 ? gather(s_ef, k, d) : 0.0;
        a.r[fo + 2 * n + d] = rv;
        red[20] += rv * rv;
      }
    }
    wg_sum<23, NW, RED_NV>(red, s_red, parity);
    rsize2 = red[22];
    if ((a.flags & RVE_ASSEMBLE) && tid == 0) {
#pragma unroll
      for (int t = 0; t < NF; ++t) a.Pbar[static_cast<size_t>(b) * NF + t] = red[t] / a.volume;
      a.rnorm2[b] = red[20];
      if (a.rsize2) a.rsize2[b] = rsize2;
    }
    if (!solve) return;
    if ((a.flags & RVE_RONLY) && red[20] <= a.thr2[b]) {   // in equilibrium: x_r = 0
#pragma unroll
      for (int k = 0; k < NPT; ++k)
        if (node_ok(k)) {
          Xb[NF * flen + 2 * (tid + k * WG)] = 0.0;
          Xb[NF * flen + 2 * (tid + k * WG) + 1] = 0.0;
        }
      if (tid == 0) {
        a.relres[b] = 0.0;
        a.iters[b] = 0.0;
        a.mv64[b] = 0.0;
      }
      return;
    }
    if (tid == 0 && !(a.flags & RVE_RONLY)) {   // condensation accumulates into these
#pragma unroll
      for (int t = 0; t < NF * NF; ++t) a.Cbar[static_cast<size_t>(b) * NF * NF + t] = red[4 + t];
#pragma unroll
      for (int t = 0; t < NF; ++t) a.Phat[static_cast<size_t>(b) * NF + t] = red[t];
    }
    if (red[21] > 0.0) {   // J <= 0 at some Gauss point: no admissible tangent
      if (tid == 0) {
        atomicAdd(a.fail_count, 1);
        a.relres[b] = __builtin_inf();
        a.iters[b] = 0.0;
        a.mv64[b] = 0.0;
      }
      return;
    }
  }

  if constexpr (NRHS == 0) {   // assemble-only instantiation
    return;
  } else {
  // ---- Jacobi diagonal ------------------------------------------------------
  TI dinv[NPT][2];
  if constexpr (FFT) {
#pragma unroll
    for (int k = 0; k < NPT; ++k) dinv[k][0] = dinv[k][1] = TI(0);
  } else {
    double acc[22];
    pass64(std::integral_constant<int, 2>(), 0, nullptr, false, acc);   // the gathers above precede the last barrier
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k)
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const int n = tid + k * WG;
        dinv[k][d] = (node_ok(k) && n != 0) ? static_cast<TI>(1.0 / gather(s_ef, k, d)) : TI(0);
      }
  }

  // ---- inner operator q = K p in TI ----------------------------------------
  const TI r1I = static_cast<TI>(r2h1), r2I = static_cast<TI>(r2h2), wtI = static_cast<TI>(wt);
  TI FbI[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) FbI[t] = static_cast<TI>(Fb[t]);
  auto matvec_ti = [&](TI (&qv)[NPT][2]) {
#pragma unroll 1
    for (int e = tid; e < NN; e += WG) {
      const Phase q = s_ph[e] ? mp[1] : mp[0];
      const TI c0 = static_cast<TI>(q.c0), b2 = static_cast<TI>(q.b2);
      const TI kk = static_cast<TI>(q.k), a2b2 = static_cast<TI>(q.a2b2);
      TI we[4][2], pe[4][2];
      elem_vals_s(s_w, e, we);
      elem_vals_s(s_p, e, pe);
      TI f[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        TI F[4], c1, dc1, gp[4], s[4];
        grad_at<TI>(we, g, r1I, r2I, F);
#pragma unroll
        for (int t = 0; t < 4; ++t) F[t] += FbI[t];
        law_tangent<TI>(F, b2, kk, a2b2, c1, dc1);
        grad_at<TI>(pe, g, r1I, r2I, gp);
        tangent_apply_F<TI>(c0, c1, dc1, F, gp, s);
        add_force<TI>(f, g, r1I, r2I, wtI, s);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int d = 0; d < 2; ++d) s_efI[(2 * m + d) * NN + e] = f[m][d];
    }
    __syncthreads();
    // the pinned corner (node 0) is no unknown: its row is dropped
#pragma unroll
    for (int k = 0; k < NPT; ++k)
#pragma unroll
      for (int d = 0; d < 2; ++d) qv[k][d] = (node_ok(k) && tid + k * WG != 0) ? gather(s_efI, k, d) : TI(0);
  };

  // u = M^-1 r at the owned nodes (pinned node zero): Jacobi, or the
  // spectral preconditioner (residual into the natural-order transform
  // field, transform, u read back from it; every thread calls it)
  auto precond = [&](const TI (&rr)[NPT][2], TI (&u)[NPT][2]) {
    if constexpr (FFT) {
      constexpr int ZP = spectral_pitch(N1);
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        if (!node_ok(k)) continue;
        const int n = tid + k * WG;
        TI* q = s_z + 2 * ((n / N1) * ZP + n % N1);
        q[0] = n != 0 ? rr[k][0] : TI(0);
        q[1] = n != 0 ? rr[k][1] : TI(0);
      }
      const TI none[4][2] = {};
      spectral_precond<N1, TI, true, true>(none, s_z, s_z + 2 * N1 * ZP, s_z, sreg, sown, sI, sJ);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int n = tid + k * WG;
        const TI* q = s_z + 2 * ((n / N1) * ZP + n % N1);
        u[k][0] = node_ok(k) ? q[0] : TI(0);
        u[k][1] = node_ok(k) ? q[1] : TI(0);
      }
    } else {
#pragma unroll
      for (int k = 0; k < NPT; ++k)
#pragma unroll
        for (int d = 0; d < 2; ++d) u[k][d] = dinv[k][d] * rr[k][d];
    }
  };

  // FP64 residual b - K x of column kc (x = 0 when xzero), and K_Fw x
  // (kfx[4] = sum of squared element-level force entries: the size of the
  // terms whose sum is the residual)
  auto residual64 = [&](int kc, bool xzero, double (&res)[NPT][2], double (&kfx)[5], bool want_kfx) {
    __syncthreads();   // earlier readers of the force buffer are done
    double acc[22];
    pass64(std::integral_constant<int, 1>(), kc < NF ? kc : -1, xzero ? nullptr : Xb + kc * flen, want_kfx, acc);
#pragma unroll
    for (int t = 0; t < 4; ++t) kfx[t] = acc[t];
    kfx[4] = acc[20];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k)
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const int n = tid + k * WG;
        double v = 0.0;
        if (node_ok(k) && n != 0) {
          v = gather(s_ef, k, d);
          if (kc == NF) v += a.r[fo + 2 * n + d];
        }
        res[k][d] = v;
      }
  };

  // ---- a5: PCG + FP64 refinement per column ---------------------------------
  const bool warm = (a.flags & RVE_WARM) != 0;
  const double tin2 = a.tol_in * a.tol_in;
  const double tol2 = a.tol * a.tol;
  int iters = 0, nmv64 = 0;
  bool all_ok = true;
  double worst = 0.0;

  const bool ronly = (a.flags & RVE_RONLY) != 0;
#pragma unroll 1
  for (int kc = ronly ? NF : 0; kc < NRHS; ++kc) {
    double* xc = Xb + kc * flen;
    bool xzero = !warm || kc >= NF;
    if (xzero) {
#pragma unroll
      for (int k = 0; k < NPT; ++k)
        if (node_ok(k)) {
          xc[2 * (tid + k * WG)] = 0.0;
          xc[2 * (tid + k * WG) + 1] = 0.0;
        }
    }
    double bb = -1.0;
#pragma unroll 1
    for (int sweep = 0;; ++sweep) {
      double res[NPT][2], kfx[5];
      residual64(kc, xzero, res, kfx, false);
      ++nmv64;
      double red[2] = {0.0, kfx[4]};
#pragma unroll
      for (int k = 0; k < NPT; ++k)
#pragma unroll
        for (int d = 0; d < 2; ++d) red[0] += res[k][d] * res[k][d];
      wg_sum<2, NW, RED_NV>(red, s_red, parity);
      if (bb < 0.0) {
        // Stopping test ||b - K x|| <= max(tol ||b||, 1e-14 S), S the size of
        // the element-level terms summed into b: a right-hand side that
        // cancels to rounding noise cannot be resolved further in FP64.
        // bb is the reference size this test divides by.
        double rb[2] = {red[0], red[1]};
        if (!xzero) {   // ||b||: one more pass from x = 0
          double r0[NPT][2], k0[5];
          residual64(kc, true, r0, k0, false);
          ++nmv64;
          rb[0] = 0.0;
          rb[1] = k0[4];
#pragma unroll
          for (int k = 0; k < NPT; ++k)
#pragma unroll
            for (int d = 0; d < 2; ++d) rb[0] += r0[k][d] * r0[k][d];
          wg_sum<2, NW, RED_NV>(rb, s_red, parity);
        }
        if (kc == NF) rb[1] += rsize2;
        bb = fmax(rb[0], 1e-28 / tol2 * rb[1]);
      }
      const double rel = bb > 0.0 ? sqrt(red[0] / bb) : 0.0;
      if (bb == 0.0 || red[0] <= tol2 * bb) {
        worst = rel > worst ? rel : worst;
        break;
      }
      if (sweep >= a.max_ir) {
        worst = rel > worst ? rel : worst;
        all_ok = false;
        break;
      }
      // inner PCG in TI on K d = res, from d = 0
      TI ri[NPT][2], xi[NPT][2], pown[NPT][2];
      bool indefinite = false;
      double rz, r0;
      __syncthreads();   // force buffer free before s_p (and the transform fields) are written
      {
#pragma unroll
        for (int k = 0; k < NPT; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) ri[k][d] = static_cast<TI>(res[k][d]);
        precond(ri, pown);
        double red2[2] = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < NPT; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            xi[k][d] = TI(0);
            const int n = tid + k * WG;
            if (node_ok(k)) put_halo<N1, N2>(s_p + d * P::PN, n % N1, n / N1, pown[k][d]);
            red2[0] += static_cast<double>(ri[k][d]) * static_cast<double>(pown[k][d]);
            red2[1] += static_cast<double>(ri[k][d]) * static_cast<double>(ri[k][d]);
          }
        wg_sum<2, NW, RED_NV>(red2, s_red, parity);
        rz = red2[0];
        r0 = red2[1];
      }
#pragma unroll 1
      for (int it = 0; it < a.max_it; ++it) {
        if (it > 0) __syncthreads();   // new search direction visible
        ++iters;
        TI q[NPT][2];
        matvec_ti(q);
        double pq[1] = {0.0};
#pragma unroll
        for (int k = 0; k < NPT; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) pq[0] += static_cast<double>(pown[k][d]) * static_cast<double>(q[k][d]);
        wg_sum<1, NW, RED_NV>(pq, s_red, parity);
        if (!(pq[0] > 0.0)) {   // breakdown: exact solution, or negative curvature
          indefinite = !(pq[0] == 0.0);
          break;
        }
        const TI alpha = static_cast<TI>(rz / pq[0]);
#pragma unroll
        for (int k = 0; k < NPT; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            xi[k][d] = fma(alpha, pown[k][d], xi[k][d]);
            ri[k][d] = fma(-alpha, q[k][d], ri[k][d]);
          }
        TI uz[NPT][2];
        precond(ri, uz);   // (its first barrier follows every read of s_p in this iteration)
        double red2[2] = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < NPT; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            const double rv = static_cast<double>(ri[k][d]);
            red2[0] += rv * static_cast<double>(uz[k][d]);
            red2[1] += rv * rv;
          }
        wg_sum<2, NW, RED_NV>(red2, s_red, parity);
        if (red2[1] <= tin2 * r0 || !(red2[0] > 0.0)) break;
        const TI beta = static_cast<TI>(red2[0] / rz);
        rz = red2[0];
        // every read of s_p in this iteration precedes the barrier of the
        // last work-group sum, so the new direction can be written now
#pragma unroll
        for (int k = 0; k < NPT; ++k)
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            pown[k][d] = fma(beta, pown[k][d], uz[k][d]);
            const int n = tid + k * WG;
            if (node_ok(k)) put_halo<N1, N2>(s_p + d * P::PN, n % N1, n / N1, pown[k][d]);
          }
      }
      if (indefinite) {   // K_ww is not positive definite here: PCG cannot solve it
        worst = __builtin_inf();
        all_ok = false;
        break;
      }
#pragma unroll
      for (int k = 0; k < NPT; ++k)
        if (node_ok(k)) {
          const int n = tid + k * WG;
          xc[2 * n] += static_cast<double>(xi[k][0]);
          xc[2 * n + 1] += static_cast<double>(xi[k][1]);
        }
      xzero = false;
    }
  }
  if constexpr (NRHS == NF) {
    double* xc = Xb + NF * flen;
#pragma unroll
    for (int k = 0; k < NPT; ++k)
      if (node_ok(k)) {
        xc[2 * (tid + k * WG)] = 0.0;
        xc[2 * (tid + k * WG) + 1] = 0.0;
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

  // ---- a6: condensation (energy form) ---------------------------------------
  //   C = (K_FF - K_Fw X_F - X_F^T (K_wF - K X_F)) / V,
  //   Phat = (int P - K_Fw x_r - X_F^T (r - K x_r)) / V;
  // column j needs (K_Fw x_j)_i and x_i . (b_j - K x_j), i < 4
  double* Cb = a.Cbar + static_cast<size_t>(b) * NF * NF;
  double* Pb = a.Phat + static_cast<size_t>(b) * NF;
#pragma unroll 1
  for (int jc = 0; jc < NRHS; ++jc) {
    double res[NPT][2], kfx[5];
    residual64(jc, false, res, kfx, true);
    ++nmv64;
    double g[2 * NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      g[i] = kfx[i];
      g[NF + i] = 0.0;
    }
    // column by column: the thread's NPT (x, y) pairs of column i are read
    // together (16-byte loads at a clamped node index, no lane-dependent
    // branch around them), then added in node order
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      double2 xv[NPT];
#pragma unroll
      for (int k = 0; k < NPT; ++k)
        xv[k] = *reinterpret_cast<const double2*>(Xb + i * flen + 2 * (node_ok(k) ? tid + k * WG : 0));
#pragma unroll
      for (int k = 0; k < NPT; ++k)
        if (node_ok(k)) g[NF + i] += xv[k].x * res[k][0] + xv[k].y * res[k][1];
    }
    wg_sum<2 * NF, NW, RED_NV>(g, s_red, parity);
    if (tid == 0) {
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        if (jc < NF) {
          Cb[i * NF + jc] -= g[i] + g[NF + i];
        } else {
          Pb[i] -= g[i] + g[NF + i];
        }
      }
    }
  }
  if (tid == 0) {
    a.relres[b] = worst;
    a.iters[b] = static_cast<double>(iters);
    a.mv64[b] = static_cast<double>(nmv64);
    if (!all_ok) atomicAdd(a.fail_count, 1);
    const double rV = 1.0 / a.volume;
#pragma unroll
    for (int i = 0; i < NF * NF; ++i) Cb[i] *= rV;
#pragma unroll
    for (int i = 0; i < NF; ++i) Pb[i] *= rV;
  }
  }
}

// ---------------------------------------------------------------------------
static constexpr int fin_wg(int n1, int n2) {
  // about four owned nodes per thread, at least one wave
  return n1 * n2 >= 1024 ? 256 : 64 * ((n1 * n2 / 4 + 63) / 64 > 0 ? (n1 * n2 / 4 + 63) / 64 : 1);
}

template <typename TI, int NRHS, int N1, int N2, bool FFT = false>
static int launch_t(const Fin2DArgs& a, int n_launch, hipStream_t s) {
  constexpr int WG = fin_wg(N1, N2);
  constexpr size_t lds = fin2d_lds_bytes_t(N1, N2, WG, NRHS, sizeof(TI), FFT);
  static_assert(lds <= 160 * 1024, "RVE too large for the LDS-resident finite-strain solver");
  static_assert(!FFT || (N1 / 2) * (N2 / 2) <= WG, "one transform block per thread");
  auto kern = &k_fin2d<TI, NRHS, N1, N2, WG, FFT>;
  if (lds > 64 * 1024)
    FE2_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  hipLaunchKernelGGL(kern, dim3(n_launch), dim3(WG), lds, s, a);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

template <int N1, int N2>
static int launch_n(const Fin2DArgs& a, int n_launch, int precision, int nrhs, hipStream_t s) {
  if (nrhs == 0) return launch_t<double, 0, N1, N2>(a, n_launch, s);   // assemble only (FP64)
  if constexpr (fin2d_spectral_size(N1, N2)) {
    if (a.flags & RVE_FFT) {
      if (!a.fft_tab || !a.fft_tab64) return set_error("spectral preconditioner table missing"), FE2_EINVAL;
      if (precision == FE2_PREC_FP64)
        return nrhs == NF ? launch_t<double, NF, N1, N2, true>(a, n_launch, s)
                          : launch_t<double, NF + 1, N1, N2, true>(a, n_launch, s);
      return nrhs == NF ? launch_t<float, NF, N1, N2, true>(a, n_launch, s)
                        : launch_t<float, NF + 1, N1, N2, true>(a, n_launch, s);
    }
  } else {
    if (a.flags & RVE_FFT) return set_error("no spectral preconditioner for this RVE size"), FE2_ENOTSUP;
  }
  if (precision == FE2_PREC_FP64)
    return nrhs == NF ? launch_t<double, NF, N1, N2>(a, n_launch, s) : launch_t<double, NF + 1, N1, N2>(a, n_launch, s);
  return nrhs == NF ? launch_t<float, NF, N1, N2>(a, n_launch, s) : launch_t<float, NF + 1, N1, N2>(a, n_launch, s);
}

#define FE2_FIN2D_SIZES(X) X(4, 4) X(6, 10) X(8, 8) X(15, 15) X(16, 16) X(30, 30) X(32, 32)

bool fin2d_supported(int n1, int n2) {
#define FE2_CASE(A, B) \
  if (n1 == A && n2 == B) return true;
  FE2_FIN2D_SIZES(FE2_CASE)
#undef FE2_CASE
  return false;
}

int launch_fin2d(const Fin2DArgs& a, int n_launch, int precision, int nrhs, hipStream_t s) {
  if (n_launch <= 0) return FE2_OK;
  if (nrhs != 0 && nrhs != NF && nrhs != NF + 1)
    return set_error("finite-strain kernel takes 0 (assemble), 4 or 5 right-hand sides"), FE2_EINVAL;
#define FE2_CASE(A, B) \
  if (a.n1 == A && a.n2 == B) return launch_n<A, B>(a, n_launch, precision, nrhs, s);
  FE2_FIN2D_SIZES(FE2_CASE)
#undef FE2_CASE
  set_error("RVE resolution has no compiled finite-strain kernel");
  return FE2_ENOTSUP;
}

}  // namespace fe2
