// RVE element integration, periodic null-space solve and condensation for
// three-dimensional small-strain RVEs (hex8 cubes, linear isotropic phases),
// one work-group per RVE.
//
// Method (Hesch, Schmidt, Schuss, arXiv:2312.12771), as for 2D:
//   * micro residual r_b = K_wF eps_b + K_ww w_b and stress integral
//     int sigma~ = K_FF eps_b + K_wF^T w_b (Eqs. (34)-(35), (17));
//   * solve K_ww [X_F | x_r] = [K_wF | r_b] with the periodic null space of
//     condition (iii) in Eq. (15) (periodic nodes, pinned corner node);
//   * condensation Cbar = (K_FF - K_wF^T X_F)/|Omega|,
//     Phat = (int sigma~ - K_wF^T x_r)/|Omega| (Eqs. (46)-(48)).
// Voigt order [11, 22, 33, 23, 13, 12] with engineering shear (nF = 6).
//
// GPU design
//   * Element stiffness mu_e * K_ref(lambda/mu); the hex8 cube K_ref has ten
//     distinct entries (kref3_id / kref3_sign), held in scalar registers.
//   * Node-centric operator: a node's row couples its 27 neighbours through
//     the 8 elements around it (64 element-corner pairs, 576 FMA per node);
//     each neighbour is loaded once from a halo-padded LDS copy of the
//     vector and feeds the per-element partial sums, which are scaled by the
//     element modulus at the end.  No scatter, no atomics, deterministic.
//   * Thread t owns nodes t, t + WG, ...; PCG vectors of the owned nodes
//     live in registers, the search direction and the FP64 staging buffer
//     (aliased) in LDS.
//   * Precision as in 2D: inner Jacobi PCG in TI, FP64 residual refinement,
//     energy-form condensation accumulated column by column.
#include <utility>

#include "elem3d.hpp"
#include "rve2d_common.hpp"

namespace fe2 {

namespace {

constexpr int NF = 6;

template <int N>
struct Pad3 {
  static constexpr int PW = N + 2;
  static constexpr int PP = PW * PW;
  static constexpr int PN = PP * PW;
  static __host__ __device__ constexpr int at(int i, int j, int k) { return (k + 1) * PP + (j + 1) * PW + (i + 1); }
};

// value of node/element (i, j, k) and its periodic halo images
template <int N, typename V>
__device__ __forceinline__ void put_halo3(V* f, int i, int j, int k, V v) {
  using P = Pad3<N>;
  const int ii[2] = {i, i == 0 ? N : (i == N - 1 ? -1 : -2)};
  const int jj[2] = {j, j == 0 ? N : (j == N - 1 ? -1 : -2)};
  const int kk[2] = {k, k == 0 ? N : (k == N - 1 ? -1 : -2)};
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a)
        if (ii[a] != -2 && jj[b] != -2 && kk[c] != -2) f[P::at(ii[a], jj[b], kk[c])] = v;
}

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1, so
// that table indices derived from I are constants (the 576-term operator is
// too large for the unroller's budget).
template <typename F, int... I>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

template <int R, int C, typename V>
__device__ __forceinline__ V kfma3(const V (&kv)[10], V x, V acc) {
  constexpr int id = kref3_id(R, C);
  if constexpr (kref3_sign(R, C) > 0) return fma(kv[id], x, acc);
  else return fma(-kv[id], x, acc);
}

// y = K v at one node: pb points at the node's padded entry of component x
// (y, z follow at +PN, +2PN); eb at the padded entry of element (i-1, j-1,
// k-1) of the phase array; s0, s1 the phase moduli.  Neighbour-major: each
// of the 27 neighbours is loaded once and feeds the partial sums z_q of the
// elements q it shares with the node.
template <int N, typename V>
__device__ __forceinline__ void mv_node(const V* __restrict__ pb, const uint8_t* __restrict__ eb, V s0, V s1,
                                        const V (&kv)[10], V (&y)[3]) {
  using P = Pad3<N>;
  V z[8][3];
#pragma unroll
  for (int q = 0; q < 8; ++q) z[q][0] = z[q][1] = z[q][2] = V(0);
  sfor<27>([&](auto oi) {
    constexpr int ox = decltype(oi)::value % 3 - 1;
    constexpr int oy = (decltype(oi)::value / 3) % 3 - 1;
    constexpr int oz = decltype(oi)::value / 9 - 1;
    constexpr int o = oz * P::PP + oy * P::PW + ox;
    const V v0 = pb[o], v1 = pb[P::PN + o], v2 = pb[2 * P::PN + o];
    sfor<8>([&](auto qi) {
      constexpr int q = decltype(qi)::value;
      constexpr int qa = q & 1, qb = (q >> 1) & 1, qc = q >> 2;
      constexpr int ma = ox + 1 - qa, mb = oy + 1 - qb, mc = oz + 1 - qc;
      if constexpr (ma >= 0 && ma <= 1 && mb >= 0 && mb <= 1 && mc >= 0 && mc <= 1) {
        constexpr int c = hcorner(1 - qa, 1 - qb, 1 - qc), m = hcorner(ma, mb, mc);
        sfor<3>([&](auto di) {
          constexpr int d = decltype(di)::value;
          V t = z[q][d];
          t = kfma3<3 * c + d, 3 * m>(kv, v0, t);
          t = kfma3<3 * c + d, 3 * m + 1>(kv, v1, t);
          t = kfma3<3 * c + d, 3 * m + 2>(kv, v2, t);
          z[q][d] = t;
        });
      }
    });
    if constexpr (decltype(oi)::value % 9 == 8) {   // one plane of neighbours loaded at a time
#pragma unroll
      for (int q = 0; q < 8; ++q) asm volatile("" : "+v"(z[q][0]), "+v"(z[q][1]), "+v"(z[q][2]) : : "memory");
    }
  });
  y[0] = y[1] = y[2] = V(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int qa = q & 1, qb = (q >> 1) & 1, qc = q >> 2;
    const V s = eb[qc * P::PP + qb * P::PW + qa] ? s1 : s0;
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d] = fma(s, z[q][d], y[d]);
  }
}

// The same operator element by element (three live accumulators; used for
// the FP64 passes, which run a few times per column).
template <int N, typename V>
__device__ __forceinline__ void mv_node_elem(const V* __restrict__ pb, const uint8_t* __restrict__ eb, V s0, V s1,
                                             const V (&kv)[10], V (&y)[3]) {
  using P = Pad3<N>;
  y[0] = y[1] = y[2] = V(0);
  sfor<8>([&](auto qi) {
    constexpr int q = decltype(qi)::value;
    constexpr int qa = q & 1, qb = (q >> 1) & 1, qc = q >> 2;
    constexpr int c = hcorner(1 - qa, 1 - qb, 1 - qc);
    V t[3] = {V(0), V(0), V(0)};
    sfor<8>([&](auto mi) {
      constexpr int m = decltype(mi)::value;
      constexpr int o = (qc - 1 + hbit(m, 2)) * P::PP + (qb - 1 + hbit(m, 1)) * P::PW + (qa - 1 + hbit(m, 0));
      const V v0 = pb[o], v1 = pb[P::PN + o], v2 = pb[2 * P::PN + o];
      sfor<3>([&](auto di) {
        constexpr int d = decltype(di)::value;
        t[d] = kfma3<3 * c + d, 3 * m>(kv, v0, t[d]);
        t[d] = kfma3<3 * c + d, 3 * m + 1>(kv, v1, t[d]);
        t[d] = kfma3<3 * c + d, 3 * m + 2>(kv, v2, t[d]);
      });
    });
    const V s = eb[qc * P::PP + qb * P::PW + qa] ? s1 : s0;
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d] = fma(s, t[d], y[d]);
    // One element's corner values live at a time: the empty asm consumes
    // this element's contribution and, with its memory clobber, keeps the
    // next element's loads behind it (otherwise every load is issued first
    // and every product sinks to the end).
    asm volatile("" : "+v"(y[0]), "+v"(y[1]), "+v"(y[2]) : : "memory");
  });
}

// Columns of K_wF at a node.  For a cube element of side h,
// K_wF[3c+d][j] = h^2/4 sum_f sigma_j[d][f] s_f(c) with sigma_j = C e_j
// (mu = 1), so the node's entries follow from g_f = sum_q mu_q s_f(c_q)
// over its 8 elements (c_q = the node's corner in element q):
//   normal j < 3:  h^2/4 g_d (rho + 2 delta_dj);
//   shear j = 3 (23), 4 (13), 5 (12): h^2/4 g_f for the component pair.
// (The setup checks this form against the quadrature tables.)
struct BFNode {
  double g[3];
  __device__ __forceinline__ double operator()(int d, int j, double rho, double h2q) const {
    if (j < 3) return h2q * g[d] * (rho + (d == j ? 2.0 : 0.0));
    const int p = (j == 3) ? 1 : 0, q = (j == 5) ? 1 : 2;   // component pair of the shear
    return d == p ? h2q * g[q] : (d == q ? h2q * g[p] : 0.0);
  }
};

template <int N>
__device__ __forceinline__ BFNode bf_node(const uint8_t* __restrict__ eb, double s0, double s1) {
  using P = Pad3<N>;
  BFNode r{{0.0, 0.0, 0.0}};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int qa = q & 1, qb = (q >> 1) & 1, qc = q >> 2;
    const double sc = eb[qc * P::PP + qb * P::PW + qa] ? s1 : s0;
    // the node is corner (1-qa, 1-qb, 1-qc): sign +1 where that bit is 1
    r.g[0] += (qa ? -sc : sc);
    r.g[1] += (qb ? -sc : sc);
    r.g[2] += (qc ? -sc : sc);
  }
  return r;
}

}  // namespace

// LDS layout: reduction buffers | phase ids with halo [PN] |
// search direction [3][PN] in TI aliased with the FP64 staging [3][PN].
constexpr int RED_NV = 12;   // widest work-group reduction
__host__ __device__ constexpr size_t lin3d_red_doubles(int nw) { return 2 * static_cast<size_t>(nw) * RED_NV; }
__host__ __device__ constexpr size_t lin3d_vec_offset(int n, int wg) {
  return (lin3d_red_doubles(wg / 64) * 8 + static_cast<size_t>(n + 2) * (n + 2) * (n + 2) + 15) &
         ~static_cast<size_t>(15);
}
__host__ __device__ constexpr size_t lin3d_lds_bytes_t(int n, int wg) {
  return lin3d_vec_offset(n, wg) + 3 * static_cast<size_t>(n + 2) * (n + 2) * (n + 2) * 8;
}

// Occupancy: FP32 instances are held to three work-groups per CU.
template <typename T> constexpr int kLin3dMinBlocks = 1;
template <> constexpr int kLin3dMinBlocks<float> = 3;
template <typename TI, int NRHS, int N, int WG>
__global__ void __launch_bounds__(WG, kLin3dMinBlocks<TI>) k_lin3d(const Lin2DArgs a) {
  using P = Pad3<N>;
  using rve2d::wg_sum;
  constexpr int NW = WG / 64;
  constexpr int NN = N * N * N;
  constexpr int NPT = (NN + WG - 1) / WG;
  const int tid = threadIdx.x;
  const int b = a.rve_list[blockIdx.x];
  if (a.skip && a.skip[b]) return;   // handled elsewhere (whole work-group)

  extern __shared__ __align__(16) unsigned char smem[];
  double* s_red = reinterpret_cast<double*>(smem);
  uint8_t* s_ph = smem + lin3d_red_doubles(NW) * 8;                 // [PN] element phases
  unsigned char* s_vec = smem + lin3d_vec_offset(N, WG);
  TI* s_p = reinterpret_cast<TI*>(s_vec);           // [3][PN] search direction
  double* s_st = reinterpret_cast<double*>(s_vec);   // [3][PN] FP64 staging (aliases s_p)
  int parity = 0;

  double kv64[10];
  TI kvI[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) {
    kv64[t] = a.kv64[t];
    kvI[t] = static_cast<TI>(kv64[t]);
  }
  const double* par = a.params + static_cast<size_t>(b) * 4;
  const double mu0 = par[1], mu1 = par[3];
  const double rho = par[0] / par[1];
  const double hh = cbrt(a.volume) / N;
  const double h2q = 0.25 * hh * hh;
  const TI mu0I = static_cast<TI>(mu0), mu1I = static_cast<TI>(mu1);
  const uint8_t* ph = a.phase + a.phase_off[b];
  double ssum = 0.0;
  for (int e = tid; e < NN; e += WG) {
    const int i = e % N, j = (e / N) % N, k = e / (N * N);
    put_halo3<N>(s_ph, i, j, k, ph[e]);
    ssum += ph[e] ? mu1 : mu0;
  }

  // owned nodes n = tid + kk WG
  auto node_ok = [&](int kk) { return tid + kk * WG < NN; };
  auto node_pad = [&](int kk) {
    const int n = tid + kk * WG;
    return P::at(n % N, (n / N) % N, n / (N * N));
  };
  const int64_t fo = a.foff[b];
  constexpr int64_t flen = 3 * NN;
  double* Xb = a.X + fo * (NF + 1);
  const double V = a.volume;
  double eps[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) eps[j] = a.macro[static_cast<size_t>(b) * NF + j];

  auto stage = [&](const double* src) {   // periodic field -> padded FP64 staging
    for (int n = tid; n < NN; n += WG) {
      const int i = n % N, j = (n / N) % N, k = n / (N * N);
#pragma unroll
      for (int d = 0; d < 3; ++d) put_halo3<N>(s_st + d * P::PN, i, j, k, src[3 * n + d]);
    }
  };
  // y = K x (FP64) at owned node kk from the staging buffer
  auto mv64 = [&](int kk, double (&y)[3]) {
    const int pn = node_pad(kk);
    mv_node_elem<N, double>(s_st + pn, s_ph + pn - P::PP - P::PW - 1, mu0, mu1, kv64, y);
  };
  auto bfn = [&](int kk) { return bf_node<N>(s_ph + node_pad(kk) - P::PP - P::PW - 1, mu0, mu1); };

  // ---- a3: residual and stress integral at (eps_b, w_b) ------------------
  double Pint[NF];
  if (a.flags & RVE_ASSEMBLE) {
    stage(a.w + fo);
    __syncthreads();
    double red[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, ssum};
#pragma unroll 1
    for (int kk = 0; kk < NPT; ++kk) {
      if (!node_ok(kk)) continue;
      const int n = tid + kk * WG;
      double y[3];
      mv64(kk, y);
      const BFNode bf = bfn(kk);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double rv = 0.0;
        if (n != 0) {
          rv = y[d];
#pragma unroll
          for (int j = 0; j < NF; ++j) rv += bf(d, j, rho, h2q) * eps[j];
        }
        a.r[fo + 3 * n + d] = rv;
        red[0] += rv * rv;
        const double wv = s_st[d * P::PN + node_pad(kk)];
#pragma unroll
        for (int j = 0; j < NF; ++j) red[1 + j] += bf(d, j, rho, h2q) * wv;
      }
    }
    wg_sum<8, NW, RED_NV>(red, s_red, parity);
    ssum = red[7];
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
    __syncthreads();   // phase halo complete
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
#pragma unroll
    for (int kk = 0; kk < NPT; ++kk)
      if (node_ok(kk))
#pragma unroll
        for (int d = 0; d < 3; ++d) Xb[NF * flen + 3 * (tid + kk * WG) + d] = 0.0;
    if (tid == 0) {
      a.relres[b] = 0.0;
      a.iters[b] = 0.0;
      a.mv64[b] = 0.0;
    }
    return;
  }

  // ---- a5: per column, FP64 refinement around the inner PCG --------------
  TI dinv[NPT];   // the diagonal is kv[0] * (sum of the 8 element moduli), equal for the 3 components
#pragma unroll
  for (int kk = 0; kk < NPT; ++kk) {
    const uint8_t* eb = s_ph + node_pad(kk) - P::PP - P::PW - 1;
    double sm = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) sm += eb[(q >> 2) * P::PP + ((q >> 1) & 1) * P::PW + (q & 1)] ? mu1 : mu0;
    dinv[kk] = (node_ok(kk) && tid + kk * WG != 0) ? static_cast<TI>(1.0 / (kv64[0] * sm)) : TI(0);
  }
  const bool warm = (a.flags & RVE_WARM) != 0;
  const double tin2 = a.tol_in * a.tol_in;
  const double tol2 = a.tol * a.tol;
  int iters = 0, nmv64 = 0;
  bool all_ok = true;
  double worst = 0.0;

#pragma unroll 1
  for (int kc = ronly ? NF : 0; kc < NRHS; ++kc) {
    double* xc = Xb + kc * flen;
    bool xzero = !warm || kc >= NF;
    if (xzero) {
#pragma unroll
      for (int kk = 0; kk < NPT; ++kk)
        if (node_ok(kk))
#pragma unroll
          for (int d = 0; d < 3; ++d) xc[3 * (tid + kk * WG) + d] = 0.0;
    }
#pragma unroll 1
    for (int sweep = 0;; ++sweep) {
      TI ri[NPT][3];
      double red[2] = {0.0, 0.0};
      __syncthreads();   // earlier readers of the staging / direction buffer are done
      if (!xzero) stage(xc);
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < NPT; ++kk) {
        double y[3] = {0.0, 0.0, 0.0};
        const bool dof = node_ok(kk) && tid + kk * WG != 0;
        if (!xzero && node_ok(kk)) mv64(kk, y);
        const BFNode bf = bfn(kk);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double r64 = 0.0;
          if (dof) {
            const double bk = (kc < NF) ? bf(d, kc, rho, h2q) : a.r[fo + 3 * (tid + kk * WG) + d];
            r64 = bk - y[d];
            red[0] += r64 * r64;
            red[1] += bk * bk;
          }
          ri[kk][d] = static_cast<TI>(r64);
        }
      }
      if (!xzero) ++nmv64;
      wg_sum<2, NW, RED_NV>(red, s_red, parity);
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
      __syncthreads();   // staging reads finished before s_p is written
      TI xi[NPT][3], pown[NPT][3];
      double rz, r0;
      {
        double red2[2] = {0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < NPT; ++kk)
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            xi[kk][d] = TI(0);
            pown[kk][d] = dinv[kk] * ri[kk][d];
            if (node_ok(kk)) {
              const int n = tid + kk * WG;
              put_halo3<N>(s_p + d * P::PN, n % N, (n / N) % N, n / (N * N), pown[kk][d]);
            }
            red2[0] += static_cast<double>(ri[kk][d]) * static_cast<double>(pown[kk][d]);
            red2[1] += static_cast<double>(ri[kk][d]) * static_cast<double>(ri[kk][d]);
          }
        wg_sum<2, NW, RED_NV>(red2, s_red, parity);
        rz = red2[0];
        r0 = red2[1];
      }
#pragma unroll 1
      for (int it = 0; it < a.max_it; ++it) {
        if (it > 0) __syncthreads();   // new search direction visible
        ++iters;
        TI q[NPT][3];
#pragma unroll
        for (int kk = 0; kk < NPT; ++kk) {
          q[kk][0] = q[kk][1] = q[kk][2] = TI(0);
          if (node_ok(kk) && tid + kk * WG != 0) {
            const int pn = node_pad(kk);
            mv_node<N, TI>(s_p + pn, s_ph + pn - P::PP - P::PW - 1, mu0I, mu1I, kvI, q[kk]);
            // keep the nodes' operator evaluations apart (see mv_node_elem)
            asm volatile("" : "+v"(q[kk][0]), "+v"(q[kk][1]), "+v"(q[kk][2]) : : "memory");
          }
        }
        double pq[1] = {0.0};
#pragma unroll
        for (int kk = 0; kk < NPT; ++kk)
#pragma unroll
          for (int d = 0; d < 3; ++d) pq[0] += static_cast<double>(pown[kk][d]) * static_cast<double>(q[kk][d]);
        wg_sum<1, NW, RED_NV>(pq, s_red, parity);
        if (!(pq[0] > 0.0)) break;   // breakdown (exact solution)
        const TI alpha = static_cast<TI>(rz / pq[0]);
        double red2[2] = {0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < NPT; ++kk)
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            xi[kk][d] = fma(alpha, pown[kk][d], xi[kk][d]);
            ri[kk][d] = fma(-alpha, q[kk][d], ri[kk][d]);
            const double rv = static_cast<double>(ri[kk][d]);
            red2[0] += rv * static_cast<double>(dinv[kk] * ri[kk][d]);
            red2[1] += rv * rv;
          }
        wg_sum<2, NW, RED_NV>(red2, s_red, parity);
        if (red2[1] <= tin2 * r0 || !(red2[0] > 0.0)) break;
        const TI beta = static_cast<TI>(red2[0] / rz);
        rz = red2[0];
        // all reads of s_p in this iteration precede the last barrier
#pragma unroll
        for (int kk = 0; kk < NPT; ++kk)
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            pown[kk][d] = fma(beta, pown[kk][d], dinv[kk] * ri[kk][d]);
            if (node_ok(kk)) {
              const int n = tid + kk * WG;
              put_halo3<N>(s_p + d * P::PN, n % N, (n / N) % N, n / (N * N), pown[kk][d]);
            }
          }
      }
#pragma unroll
      for (int kk = 0; kk < NPT; ++kk)
        if (node_ok(kk))
#pragma unroll
          for (int d = 0; d < 3; ++d) xc[3 * (tid + kk * WG) + d] += static_cast<double>(xi[kk][d]);
      xzero = false;
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
  if constexpr (NRHS == NF) {   // residual column not solved: x_r = 0
#pragma unroll
    for (int kk = 0; kk < NPT; ++kk)
      if (node_ok(kk))
#pragma unroll
        for (int d = 0; d < 3; ++d) Xb[NF * flen + 3 * (tid + kk * WG) + d] = 0.0;
  }

  // ---- a6: condensation (energy form), one column at a time --------------
  //   G1[i][j] = b_i . x_j,  G2[i][j] = x_i . (b_j - K x_j)
  double* Cb = a.Cbar + static_cast<size_t>(b) * NF * NF;
  double* Pb = a.Phat + static_cast<size_t>(b) * NF;
#pragma unroll 1
  for (int jc = 0; jc < NRHS; ++jc) {
    const double* xc = Xb + jc * flen;
    __syncthreads();   // global writes of X visible, staging free
    stage(xc);
    __syncthreads();
    ++nmv64;
    double g[2 * NF];
#pragma unroll
    for (int i = 0; i < 2 * NF; ++i) g[i] = 0.0;
#pragma unroll 1
    for (int kk = 0; kk < NPT; ++kk) {
      if (!node_ok(kk) || tid + kk * WG == 0) continue;
      const int n = tid + kk * WG;
      double y[3];
      mv64(kk, y);
      const BFNode bf = bfn(kk);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double bj = (jc < NF) ? bf(d, jc, rho, h2q) : a.r[fo + 3 * n + d];
        const double xj = s_st[d * P::PN + node_pad(kk)];
        const double res = bj - y[d];
#pragma unroll
        for (int i = 0; i < NF; ++i) {
          g[i] += bf(d, i, rho, h2q) * xj;
          g[NF + i] += Xb[i * flen + 3 * n + d] * res;
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
        for (int i = 0; i < NF; ++i) Pb[i] = (Pint[i] - g[i] - g[NF + i]) / V;
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
      for (int i = 0; i < NF; ++i) Pb[i] = Pint[i] / V;
    }
  }
  }
}

// ---------------------------------------------------------------------------
static constexpr int lin3d_wg(int n) {
  return n * n * n >= 1000 ? 256 : (n * n * n >= 512 ? 128 : 64);
}

template <typename TI, int NRHS, int N>
static int launch3_t(const Lin2DArgs& a, int n_launch, hipStream_t s) {
  constexpr int WG = lin3d_wg(N);
  constexpr size_t lds = lin3d_lds_bytes_t(N, WG);
  static_assert(lds <= 160 * 1024, "RVE too large for the LDS-resident 3D solver");
  auto kern = &k_lin3d<TI, NRHS, N, WG>;
  if (lds > 64 * 1024)
    FE2_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  hipLaunchKernelGGL(kern, dim3(n_launch), dim3(WG), lds, s, a);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

template <int N>
static int launch3_n(const Lin2DArgs& a, int n_launch, int precision, int nrhs, hipStream_t s) {
  if (nrhs == 0) return launch3_t<double, 0, N>(a, n_launch, s);   // assemble only (FP64)
  if (precision == FE2_PREC_FP64)
    return nrhs == NF ? launch3_t<double, NF, N>(a, n_launch, s) : launch3_t<double, NF + 1, N>(a, n_launch, s);
  return nrhs == NF ? launch3_t<float, NF, N>(a, n_launch, s) : launch3_t<float, NF + 1, N>(a, n_launch, s);
}

#define FE2_LIN3D_SIZES(X) X(4) X(6) X(8) X(10)

bool lin3d_supported(int n1, int n2, int n3) {
  if (n1 != n2 || n2 != n3) return false;
#define FE2_CASE(A) \
  if (n1 == A) return true;
  FE2_LIN3D_SIZES(FE2_CASE)
#undef FE2_CASE
  return false;
}

int launch_lin3d(const Lin2DArgs& a, int n_launch, int precision, int nrhs, hipStream_t s) {
  if (n_launch <= 0) return FE2_OK;
  if (nrhs != 0 && nrhs != NF && nrhs != NF + 1)
    return set_error("3D kernel takes 0 (assemble), 6 or 7 right-hand sides"), FE2_EINVAL;
#define FE2_CASE(A) \
  if (a.n1 == A) return launch3_n<A>(a, n_launch, precision, nrhs, s);
  FE2_LIN3D_SIZES(FE2_CASE)
#undef FE2_CASE
  set_error("RVE resolution has no compiled 3D kernel");
  return FE2_ENOTSUP;
}

}  // namespace fe2
