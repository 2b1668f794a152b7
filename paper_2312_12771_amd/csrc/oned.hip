// The 1+1-dimensional FE^2 problem of Sec. 5.1 on the GPU (FP64): a macro bar
// with Lagrange elements of order q, one RVE (0, 1) per macro Gauss point
// (Dirac basis, Eqs. (31)-(35)) or per macro element (piecewise-constant
// basis, Eqs. (constSolution1)-(constSolution2)), the micro energy
// lambda(X~) (F~^2 - 1), hence P~ = 2 lambda F~, and zero fluctuation at both
// RVE ends (condition (ii) of Eq. (15)).
//
// Every RVE has the same micro mesh and material, so the banded RVE stiffness
// K_ww, its coupling K_wF, K_FF and the sensitivity X_F = K_ww^-1 K_wF are
// built and factorised once at setup; the per-RVE work of a Newton step
// (residual, solve for x_r, condensation, update) runs one lane per RVE over
// vectors stored DOF-major (lane-contiguous), and the macro system goes to
// the block-cyclic-reduction band solver.
#include <cmath>
#include <new>
#include <vector>

#include "fe2_internal.hpp"
#include "macro.hpp"

using namespace fe2;

namespace {

constexpr int NG_MICRO = 5;   // Gauss-Legendre points per RVE element

// 5-point Gauss-Legendre rule on [-1, 1]
__device__ __constant__ double c_g5x[NG_MICRO] = {-0.90617984593866399280, -0.53846931010568309104, 0.0,
                                                  0.53846931010568309104, 0.90617984593866399280};
__device__ __constant__ double c_g5w[NG_MICRO] = {0.23692688505618908751, 0.47862867049936646804,
                                                  0.56888888888888888889, 0.47862867049936646804,
                                                  0.23692688505618908751};

// Lagrange shape functions of order q on [-1, 1], equally spaced nodes.
__host__ __device__ inline void shape1d(int q, double xi, double* N, double* dN) {
  if (q == 1) {
    N[0] = 0.5 * (1.0 - xi);
    N[1] = 0.5 * (1.0 + xi);
    dN[0] = -0.5;
    dN[1] = 0.5;
  } else {
    N[0] = 0.5 * xi * (xi - 1.0);
    N[1] = 1.0 - xi * xi;
    N[2] = 0.5 * xi * (xi + 1.0);
    dN[0] = xi - 0.5;
    dN[1] = -2.0 * xi;
    dN[2] = xi + 0.5;
  }
}

// Gauss points of the macro rule (q + 1 points) on [-1, 1].
__host__ __device__ inline void macro_gauss(int q, int g, double* x, double* w) {
  if (q == 1) {
    *x = g == 0 ? -0.57735026918962576451 : 0.57735026918962576451;
    *w = 1.0;
  } else {
    const double a = 0.77459666924148337704;
    *x = g == 0 ? -a : (g == 1 ? 0.0 : a);
    *w = g == 1 ? 8.0 / 9.0 : 5.0 / 9.0;
  }
}

struct OneD {
  int q, n_mac, n_mic, basis;
  int n_phi, n_int, n_gp, n_rve;
  double L, load, phi_l, phi_r;
  double h_mac, h_mic;
};

// ---------------------------------------------------------------------------
// setup: RVE matrices (one thread per interior RVE node), factorisation and
// the shared sensitivity (one thread)
// ---------------------------------------------------------------------------
// kw: lower band of K_ww, kw[i*(q+1) + d] = K(i, i-d) over interior nodes
// i = a - 1; kfw[i] = K_Fw; kff_part[e] = integral of 2 lambda over element e.
__global__ void k1d_micro(OneD o, const double* __restrict__ lam_gp, double* __restrict__ kw,
                          double* __restrict__ kfw, double* __restrict__ kff_part) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = o.q;
  const double j = 0.5 * o.h_mic;
  if (t < o.n_mic) {
    double s = 0.0;
    for (int l = 0; l < NG_MICRO; ++l) s += 2.0 * lam_gp[t * NG_MICRO + l] * c_g5w[l] * j;
    kff_part[t] = s;
  }
  if (t >= o.n_int) return;
  const int a = t + 1;   // global node of interior row t
  double band[3] = {0.0, 0.0, 0.0};
  double fw = 0.0;
  for (int e = (a - 1) / q - 1; e <= a / q; ++e) {
    if (e < 0 || e >= o.n_mic || a < q * e || a > q * e + q) continue;
    const int la = a - q * e;
    for (int l = 0; l < NG_MICRO; ++l) {
      double N[3], dN[3];
      shape1d(q, c_g5x[l], N, dN);
      const double w2 = 2.0 * lam_gp[e * NG_MICRO + l] * c_g5w[l] * j;
      const double da = dN[la] / j;
      fw += w2 * da;
      for (int lb = 0; lb <= la; ++lb) band[la - lb] += w2 * da * dN[lb] / j;
    }
  }
  for (int d = 0; d <= q; ++d) kw[t * (q + 1) + d] = (t - d >= 0) ? band[d] : 0.0;
  kfw[t] = fw;
}

// Banded Cholesky K_ww = L L^T (in place, lower band, bandwidth q) with
// reciprocal pivots, then X_F = K_ww^-1 K_wF and the shared condensed
// tangent Cbar = (K_FF - K_Fw X_F) / |Omega| (|Omega| = 1).  One thread: the
// RVE has at most a few thousand DOFs.  info = 1-based failing pivot.
__global__ void k1d_factor(OneD o, double* __restrict__ kw, double* __restrict__ rinv, const double* __restrict__ kfw,
                           double* __restrict__ xf, const double* __restrict__ kff_part, double* __restrict__ scal,
                           int* __restrict__ info) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int q = o.q, n = o.n_int, b1 = q + 1;
  for (int i = 0; i < n; ++i) {
    for (int d = q; d >= 1; --d) {       // L(i, i-d)
      if (i - d < 0) continue;
      double v = kw[i * b1 + d];
      for (int c = d + 1; c <= q; ++c)   // sum_k L(i,k) L(i-d,k), k = i-c
        if (i - c >= 0 && c - d <= q) v -= kw[i * b1 + c] * kw[(i - d) * b1 + (c - d)];
      kw[i * b1 + d] = v * rinv[i - d];
    }
    double dd = kw[i * b1];
    for (int c = 1; c <= q; ++c)
      if (i - c >= 0) dd -= kw[i * b1 + c] * kw[i * b1 + c];
    if (!(dd > 0.0)) {
      *info = i + 1;
      return;
    }
    kw[i * b1] = sqrt(dd);
    rinv[i] = 1.0 / kw[i * b1];
  }
  // forward and backward substitution for X_F
  for (int i = 0; i < n; ++i) {
    double v = kfw[i];
    for (int c = 1; c <= q; ++c)
      if (i - c >= 0) v -= kw[i * b1 + c] * xf[i - c];
    xf[i] = v * rinv[i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = xf[i];
    for (int c = 1; c <= q; ++c)
      if (i + c < n) v -= kw[(i + c) * b1 + c] * xf[i + c];
    xf[i] = v * rinv[i];
  }
  double kff = 0.0, fx = 0.0;
  for (int e = 0; e < o.n_mic; ++e) kff += kff_part[e];
  for (int i = 0; i < n; ++i) fx += kfw[i] * xf[i];
  scal[0] = kff;          // K_FF; the Voigt average C_V = K_FF / |Omega|
  scal[1] = kff - fx;     // Cbar (|Omega| = 1)
}

// ---------------------------------------------------------------------------
// macro geometry helpers
// ---------------------------------------------------------------------------
// derivative row B_g = dN/dX at Gauss point g of a macro element (uniform mesh)
__device__ inline void macro_B(const OneD& o, int g, double* B, double* wJ) {
  double x, w, N[3], dN[3];
  macro_gauss(o.q, g, &x, &w);
  shape1d(o.q, x, N, dN);
  const double J = 0.5 * o.h_mac;
  for (int a = 0; a <= o.q; ++a) B[a] = dN[a] / J;
  *wJ = w * J;
}

// gradient operator of RVE b: B_g (Dirac) or Bbar_e = sum_g wJ B_g / h (element)
__device__ inline int rve_B(const OneD& o, int b, double* B, double* vol) {
  if (o.basis == FE2_BASIS_ELEMENT) {
    for (int a = 0; a <= o.q; ++a) B[a] = 0.0;
    double v = 0.0;
    for (int g = 0; g < o.n_gp; ++g) {
      double Bg[3], wJ;
      macro_B(o, g, Bg, &wJ);
      for (int a = 0; a <= o.q; ++a) B[a] += wJ * Bg[a];
      v += wJ;
    }
    for (int a = 0; a <= o.q; ++a) B[a] /= v;
    *vol = v;
    return b;
  }
  double wJ;
  macro_B(o, b % o.n_gp, B, &wJ);
  *vol = wJ;
  return b / o.n_gp;
}

// ---------------------------------------------------------------------------
// per-RVE work: residual, solve for x_r with the shared factor, condensation
// ---------------------------------------------------------------------------
// Vectors are DOF-major: entry i of RVE b at [i * n_rve + b], so a wave reads
// 64 consecutive RVEs per DOF.
//
// r_b = K_wF F_b + K_ww w_b, one thread per (DOF, RVE): fully parallel.
__global__ void k1d_resid(OneD o, const double* __restrict__ phi, const double* __restrict__ w,
                          const double* __restrict__ kw, const double* __restrict__ kfw, double* __restrict__ r,
                          double* __restrict__ Fb) {
  const size_t t = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  const int nr = o.n_rve, n = o.n_int, q = o.q, b1 = q + 1;
  if (t >= static_cast<size_t>(n) * nr) return;
  const int i = static_cast<int>(t / nr), b = static_cast<int>(t % nr);
  double B[3], vol;
  const int e = rve_B(o, b, B, &vol);
  double F = 0.0;
  for (int a = 0; a <= q; ++a) F += B[a] * phi[q * e + a];
  if (i == 0) Fb[b] = F;
  double ri = kfw[i] * F + kw[i * b1] * w[t];
  for (int d = 1; d <= q; ++d) {
    if (i - d >= 0) ri += kw[i * b1 + d] * w[t - static_cast<size_t>(d) * nr];
    if (i + d < n) ri += kw[(i + d) * b1 + d] * w[t + static_cast<size_t>(d) * nr];
  }
  r[t] = ri;
}

// Forward and backward substitution with the shared Cholesky factor, one
// lane per RVE.  The factor, its reciprocal pivots and K_Fw are staged in LDS
// (the same for every lane); the recurrences are sequential in the DOF
// index, so the per-RVE loads of the next PF DOFs are issued before the
// current PF steps run (register double buffering), leaving two FMAs and a
// multiply per DOF on the chain.  Also ||r_b||^2, the stress integral and
// P_hat (|Omega| = 1).
constexpr int PF = 16;
template <int Q>
__global__ void __launch_bounds__(64) k1d_rve(OneD o, const double* __restrict__ r, const double* __restrict__ w,
                                              const double* __restrict__ kw, const double* __restrict__ rinv,
                                              const double* __restrict__ kfw, const double* __restrict__ scal,
                                              const double* __restrict__ Fb, double* __restrict__ xr,
                                              double* __restrict__ pbar, double* __restrict__ phat,
                                              double* __restrict__ rn2) {
  extern __shared__ double s_fac[];
  constexpr int B1 = Q + 1;
  const int n = o.n_int, nr = o.n_rve;
  // kw holds the lower band of K_ww (kw[i*(q+1) + d] = K(i, i-d), zero for
  // i < d) followed by the same band of its Cholesky factor
  double* Lf = s_fac;                                   // [n][Q+1]
  double* s_ri = s_fac + static_cast<size_t>(n) * B1;   // [n]
  double* s_kf = s_ri + n;                              // [n]
  for (int k = threadIdx.x; k < n * B1; k += blockDim.x) Lf[k] = kw[static_cast<size_t>(n) * B1 + k];
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    s_ri[k] = rinv[k];
    s_kf[k] = kfw[k];
  }
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nr) return;
  const double* rb = r + b;
  const double* wb = w + b;
  double* xb = xr + b;
  auto at = [&](int i) { return static_cast<size_t>(i) * nr; };
  double pint = Fb[b] * scal[0];
  double r2 = 0.0;
  // ---- forward: L y = r.  Full chunks [0, nf) without bounds tests (the
  // factor's entries above the first rows are zero), then the tail.
  double y1 = 0.0, y2 = 0.0;   // y_{i-1}, y_{i-2}
  const int nf = (n / PF) * PF;
  double rc[PF], wc[PF], rn[PF], wn[PF], out[PF];
  if (nf > 0) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      rc[j] = rb[at(j)];
      wc[j] = wb[at(j)];
    }
  }
  for (int i0 = 0; i0 < nf; i0 += PF) {
    if (i0 + PF < nf) {
#pragma unroll
      for (int j = 0; j < PF; ++j) {
        rn[j] = rb[at(i0 + PF + j)];
        wn[j] = wb[at(i0 + PF + j)];
      }
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int i = i0 + j;
      r2 += rc[j] * rc[j];
      pint += s_kf[i] * wc[j];
      double v = rc[j] - Lf[i * B1 + 1] * y1;
      if constexpr (Q == 2) v -= Lf[i * B1 + 2] * y2;
      const double yi = v * s_ri[i];
      out[j] = yi;
      y2 = y1;
      y1 = yi;
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) xb[at(i0 + j)] = out[j];
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      rc[j] = rn[j];
      wc[j] = wn[j];
    }
  }
  for (int i = nf; i < n; ++i) {
    const double ri = rb[at(i)];
    r2 += ri * ri;
    pint += s_kf[i] * wb[at(i)];
    double v = ri;
    if (i >= 1) v -= Lf[i * B1 + 1] * y1;
    if (Q == 2 && i >= 2) v -= Lf[i * B1 + 2] * y2;
    const double yi = v * s_ri[i];
    xb[at(i)] = yi;
    y2 = y1;
    y1 = yi;
  }
  // ---- backward: L^T x = y.  Tail [m, n) with bounds tests first, then full
  // chunks below m, where i + Q < n always holds.
  const int m = n > Q ? ((n - Q) / PF) * PF : 0;
  double x1 = 0.0, x2 = 0.0, fx = 0.0;   // x_{i+1}, x_{i+2}
  for (int i = n - 1; i >= m; --i) {
    double v = xb[at(i)];
    if (i + 1 < n) v -= Lf[(i + 1) * B1 + 1] * x1;
    if (Q == 2 && i + 2 < n) v -= Lf[(i + 2) * B1 + 2] * x2;
    const double xi = v * s_ri[i];
    xb[at(i)] = xi;
    fx += s_kf[i] * xi;
    x2 = x1;
    x1 = xi;
  }
  if (m > 0) {
#pragma unroll
    for (int j = 0; j < PF; ++j) rc[j] = xb[at(m - 1 - j)];
  }
  for (int i0 = m - 1; i0 >= 0; i0 -= PF) {
    if (i0 - PF >= 0) {
#pragma unroll
      for (int j = 0; j < PF; ++j) rn[j] = xb[at(i0 - PF - j)];
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int i = i0 - j;
      double v = rc[j] - Lf[(i + 1) * B1 + 1] * x1;
      if constexpr (Q == 2) v -= Lf[(i + 2) * B1 + 2] * x2;
      const double xi = v * s_ri[i];
      out[j] = xi;
      fx += s_kf[i] * xi;
      x2 = x1;
      x1 = xi;
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) xb[at(i0 - j)] = out[j];
#pragma unroll
    for (int j = 0; j < PF; ++j) rc[j] = rn[j];
  }
  pbar[b] = pint;
  phat[b] = pint - fx;
  rn2[b] = r2;
}

// ---------------------------------------------------------------------------
// macro element vectors and tangents, one thread per macro element
// ---------------------------------------------------------------------------
// Dirac: sigma_g = P_b, k = sum_g wJ B_g^T Cbar B_g.  Element: sigma_g = P_e +
// C_V (F_g - Fbar_e), k = sum_g wJ B_g^T C_V B_g + V_e Bbar^T (Cbar - C_V) Bbar.
__global__ void k1d_macro_elem(OneD o, const double* __restrict__ phi, const double* __restrict__ pbar,
                               const double* __restrict__ phat, const double* __restrict__ scal,
                               double* __restrict__ fe_true, double* __restrict__ fe_hat, double* __restrict__ ke) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= o.n_mac) return;
  const int q = o.q, nd = q + 1;
  const double CV = scal[0], Cb = scal[1];
  double ft[3] = {0, 0, 0}, fh[3] = {0, 0, 0}, k[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const bool element = o.basis == FE2_BASIS_ELEMENT;
  double Bbar[3] = {0, 0, 0}, V = 0.0, Fbar = 0.0;
  if (element) {
    rve_B(o, e, Bbar, &V);
    for (int a = 0; a < nd; ++a) Fbar += Bbar[a] * phi[q * e + a];
  }
  for (int g = 0; g < o.n_gp; ++g) {
    double B[3], wJ;
    macro_B(o, g, B, &wJ);
    double st, sh, C;
    if (element) {
      double Fg = 0.0;
      for (int a = 0; a < nd; ++a) Fg += B[a] * phi[q * e + a];
      st = pbar[e] + CV * (Fg - Fbar);
      sh = phat[e] + CV * (Fg - Fbar);
      C = CV;
    } else {
      const int b = e * o.n_gp + g;
      st = pbar[b];
      sh = phat[b];
      C = Cb;
    }
    for (int a = 0; a < nd; ++a) {
      ft[a] += wJ * B[a] * st;
      fh[a] += wJ * B[a] * sh;
      for (int c = 0; c < nd; ++c) k[a * nd + c] += wJ * B[a] * C * B[c];
    }
  }
  if (element)
    for (int a = 0; a < nd; ++a)
      for (int c = 0; c < nd; ++c) k[a * nd + c] += V * Bbar[a] * (Cb - CV) * Bbar[c];
  for (int a = 0; a < nd; ++a) {
    fe_true[e * nd + a] = ft[a];
    fe_hat[e * nd + a] = fh[a];
    for (int c = 0; c < nd; ++c) ke[(e * nd + a) * nd + c] = k[a * nd + c];
  }
}

// Row gather into the lower band (bandwidth q) with the two Dirichlet ends as
// identity rows (zero increment: the state satisfies the boundary data), the
// right-hand side -(F_hat - f_ext) and the true residual F_int - f_ext.
__global__ void k1d_macro_rows(OneD o, const double* __restrict__ fe_true, const double* __restrict__ fe_hat,
                               const double* __restrict__ ke, double* __restrict__ band, double* __restrict__ rhs,
                               double* __restrict__ rtrue, double* __restrict__ fint) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= o.n_phi) return;
  const int q = o.q, nd = q + 1, b1 = q + 1;
  double ft = 0.0, fh = 0.0, fext = 0.0;
  double row[3] = {0, 0, 0};   // K(A, A-d)
  for (int e = A / q - 1; e <= A / q; ++e) {
    if (e < 0 || e >= o.n_mac || A < q * e || A > q * e + q) continue;
    const int la = A - q * e;
    ft += fe_true[e * nd + la];
    fh += fe_hat[e * nd + la];
    for (int g = 0; g < o.n_gp; ++g) {   // consistent load of the uniform body force
      double x, w, N[3], dN[3];
      macro_gauss(q, g, &x, &w);
      shape1d(q, x, N, dN);
      fext += w * 0.5 * o.h_mac * o.load * N[la];
    }
    for (int lb = 0; lb <= la; ++lb) row[la - lb] += ke[(e * nd + la) * nd + lb];
  }
  const bool dir = (A == 0 || A == o.n_phi - 1);
  fint[A] = ft;
  rtrue[A] = dir ? 0.0 : ft - fext;
  // lower band storage of the block solver: entry (A, A-d) at [(A-d)][d];
  // slots (A, d) with A + d past the last row are padding and set to zero
  for (int d = 0; d <= q; ++d) {
    if (A + d >= o.n_phi) band[static_cast<size_t>(A) * b1 + d] = 0.0;
    if (A - d < 0) continue;
    const bool dcol = (A - d == 0 || A - d == o.n_phi - 1);
    double v = (dir || dcol) ? 0.0 : row[d];
    if (dir && d == 0) v = 1.0;
    band[static_cast<size_t>(A - d) * b1 + d] = v;
  }
  rhs[A] = dir ? 0.0 : fext - fh;
}

// w_b -= x_r + X_F dF_b with dF_b from the macro increment, one thread per
// (DOF, RVE).
__global__ void k1d_update(OneD o, const double* __restrict__ dphi, const double* __restrict__ xr,
                           const double* __restrict__ xf, double* __restrict__ w) {
  const size_t t = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (t >= static_cast<size_t>(o.n_int) * o.n_rve) return;
  const int i = static_cast<int>(t / o.n_rve), b = static_cast<int>(t % o.n_rve);
  double B[3], vol;
  const int e = rve_B(o, b, B, &vol);
  double dF = 0.0;
  for (int a = 0; a <= o.q; ++a) dF += B[a] * dphi[o.q * e + a];
  w[t] -= xr[t] + xf[i] * dF;
}

__global__ void k1d_axpy(int n, const double* __restrict__ x, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

// norms: [||[R_free; R_micro]||, ||R_free||, ||R_micro||, ||F_int||] with
// R_micro,b = vol_b / |Omega| r_b.  One work-group of 256 threads.
__global__ void __launch_bounds__(256) k1d_norms(OneD o, const double* __restrict__ rtrue,
                                                 const double* __restrict__ fint, const double* __restrict__ rn2,
                                                 double* __restrict__ out) {
  __shared__ double red[4][3];
  double s[3] = {0, 0, 0};
  for (int i = threadIdx.x; i < o.n_phi; i += blockDim.x) {
    s[0] += rtrue[i] * rtrue[i];
    s[2] += fint[i] * fint[i];
  }
  for (int b = threadIdx.x; b < o.n_rve; b += blockDim.x) {
    double B[3], vol;
    rve_B(o, b, B, &vol);
    s[1] += vol * vol * rn2[b];
  }
  for (int k = 0; k < 3; ++k) s[k] = wave_sum(s[k]);
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 3; ++k) red[threadIdx.x >> 6][k] = s[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[3] = {0, 0, 0};
    for (int wv = 0; wv < 4; ++wv)
      for (int k = 0; k < 3; ++k) t[k] += red[wv][k];
    out[0] = sqrt(t[0] + t[1]);
    out[1] = sqrt(t[0]);
    out[2] = sqrt(t[1]);
    out[3] = sqrt(t[2]);
  }
}

// initial state: phi linear between the boundary values, w = 0
__global__ void k1d_init(OneD o, double* __restrict__ phi, double* __restrict__ w, size_t wlen) {
  const size_t t = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (t < static_cast<size_t>(o.n_phi)) {
    const double s = static_cast<double>(t) / (o.n_phi - 1);
    phi[t] = (t + 1 == static_cast<size_t>(o.n_phi)) ? o.phi_r : o.phi_l + s * (o.phi_r - o.phi_l);
  }
  for (size_t k = t; k < wlen; k += static_cast<size_t>(gridDim.x) * blockDim.x) w[k] = 0.0;
}

// DOF-major [i][b] -> RVE-major [b][i]
__global__ void k1d_transpose(int n_int, int n_rve, const double* __restrict__ src, double* __restrict__ dst) {
  const size_t t = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (t >= static_cast<size_t>(n_int) * n_rve) return;
  const int b = static_cast<int>(t / n_int), i = static_cast<int>(t % n_int);
  dst[t] = src[static_cast<size_t>(i) * n_rve + b];
}

inline unsigned nb(size_t n, unsigned bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

template <typename T>
int alloc(T** p, size_t n) {
  *p = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(p), (n ? n : 1) * sizeof(T)) != hipSuccess) {
    set_error("hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
    return FE2_ENOMEM;
  }
  return FE2_OK;
}

}  // namespace

struct fe2_1d_ctx {
  OneD o{};
  double *lam = nullptr, *kw = nullptr, *rinv = nullptr, *kfw = nullptr, *xf = nullptr, *kffp = nullptr,
         *scal = nullptr;
  double *phi = nullptr, *w = nullptr, *xr = nullptr, *Fb = nullptr, *pbar = nullptr, *phat = nullptr,
         *rn2 = nullptr;
  double *fe_t = nullptr, *fe_h = nullptr, *ke = nullptr, *band = nullptr, *rhs = nullptr, *rtrue = nullptr,
         *fint = nullptr, *norms = nullptr, *ws = nullptr, *wtmp = nullptr;
  int* info = nullptr;
  double* norms_host = nullptr;
  BcrPlan plan;
};

namespace {

void free_1d(fe2_1d_ctx* h) {
  if (!h) return;
  void* ps[] = {h->lam, h->kw, h->rinv, h->kfw, h->xf, h->kffp, h->scal, h->phi, h->w, h->xr, h->Fb,
                h->pbar, h->phat, h->rn2, h->fe_t, h->fe_h, h->ke, h->band, h->rhs, h->rtrue, h->fint,
                h->norms, h->ws, h->wtmp, h->info};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (h->norms_host) (void)hipHostFree(h->norms_host);
  delete h;
}

int setup_1d(fe2_1d_ctx* h, const fe2_1d_desc* d, hipStream_t s) {
  OneD& o = h->o;
  o.q = d->order;
  o.n_mac = d->n_macro;
  o.n_mic = d->n_micro;
  o.basis = d->basis;
  o.n_phi = o.q * o.n_mac + 1;
  o.n_int = o.q * o.n_mic - 1;
  o.n_gp = o.q + 1;
  o.n_rve = o.basis == FE2_BASIS_ELEMENT ? o.n_mac : o.n_mac * o.n_gp;
  o.L = d->macro_length;
  o.load = d->body_load;
  o.phi_l = d->phi_left;
  o.phi_r = d->phi_right;
  o.h_mac = o.L / o.n_mac;
  o.h_mic = 1.0 / o.n_mic;
  const size_t b1 = o.q + 1, ni = o.n_int, nr = o.n_rve, wl = ni * nr;
  int rc;
  if ((rc = alloc(&h->lam, static_cast<size_t>(o.n_mic) * NG_MICRO))) return rc;
  FE2_HIP_CHECK(hipMemcpyAsync(h->lam, d->lambda_gp, sizeof(double) * o.n_mic * NG_MICRO, hipMemcpyHostToDevice, s));
  if ((rc = alloc(&h->kw, 2 * ni * b1))) return rc;   // K_ww band, then its factor
  if ((rc = alloc(&h->rinv, ni))) return rc;
  if ((rc = alloc(&h->kfw, ni))) return rc;
  if ((rc = alloc(&h->xf, ni))) return rc;
  if ((rc = alloc(&h->kffp, o.n_mic))) return rc;
  if ((rc = alloc(&h->scal, 2))) return rc;
  if ((rc = alloc(&h->phi, o.n_phi))) return rc;
  if ((rc = alloc(&h->w, wl))) return rc;
  if ((rc = alloc(&h->wtmp, wl))) return rc;
  if ((rc = alloc(&h->xr, wl))) return rc;
  if ((rc = alloc(&h->Fb, nr))) return rc;
  if ((rc = alloc(&h->pbar, nr))) return rc;
  if ((rc = alloc(&h->phat, nr))) return rc;
  if ((rc = alloc(&h->rn2, nr))) return rc;
  if ((rc = alloc(&h->fe_t, o.n_mac * b1))) return rc;
  if ((rc = alloc(&h->fe_h, o.n_mac * b1))) return rc;
  if ((rc = alloc(&h->ke, o.n_mac * b1 * b1))) return rc;
  if ((rc = alloc(&h->band, o.n_phi * b1))) return rc;
  if ((rc = alloc(&h->rhs, o.n_phi))) return rc;
  if ((rc = alloc(&h->rtrue, o.n_phi))) return rc;
  if ((rc = alloc(&h->fint, o.n_phi))) return rc;
  if ((rc = alloc(&h->norms, 4))) return rc;
  if ((rc = alloc(&h->info, 1))) return rc;
  h->plan = bcr_plan(o.n_phi, o.q);
  if ((rc = alloc(&h->ws, bcr_workspace_doubles(h->plan)))) return rc;
  if (hipHostMalloc(reinterpret_cast<void**>(&h->norms_host), 4 * sizeof(double)) != hipSuccess)
    return set_error("pinned host allocation failed"), FE2_ENOMEM;
  FE2_HIP_CHECK(hipMemsetAsync(h->info, 0, sizeof(int), s));
  hipLaunchKernelGGL(k1d_micro, dim3(nb(std::max(o.n_int, o.n_mic), 128)), dim3(128), 0, s, o, h->lam, h->kw,
                     h->kfw, h->kffp);
  FE2_HIP_CHECK(hipMemcpyAsync(h->kw + ni * b1, h->kw, sizeof(double) * ni * b1, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k1d_factor, dim3(1), dim3(64), 0, s, o, h->kw + ni * b1, h->rinv, h->kfw, h->xf, h->kffp,
                     h->scal, h->info);
  hipLaunchKernelGGL(k1d_init, dim3(std::min<unsigned>(4096, nb(std::max<size_t>(wl, o.n_phi), 256))), dim3(256), 0,
                     s, o, h->phi, h->w, wl);
  FE2_HIP_CHECK(hipGetLastError());
  int info = 0;
  FE2_HIP_CHECK(hipMemcpyAsync(&info, h->info, sizeof(int), hipMemcpyDeviceToHost, s));
  FE2_HIP_CHECK(hipStreamSynchronize(s));
  if (info) return set_error("RVE stiffness not positive definite at pivot " + std::to_string(info)), FE2_EINVAL;
  return FE2_OK;
}

}  // namespace

extern "C" {

int fe2_1d_setup(const fe2_1d_desc* d, void* stream, fe2_1d_handle* out) {
  if (!out) return set_error("null output handle"), FE2_EINVAL;
  *out = nullptr;
  if (!d) return set_error("null descriptor"), FE2_EINVAL;
  if (d->struct_size != static_cast<int32_t>(sizeof(fe2_1d_desc)))
    return set_error("struct_size does not match this library's fe2_1d_desc"), FE2_EINVAL;
  if (d->order != 1 && d->order != 2) return set_error("order must be 1 or 2"), FE2_EINVAL;
  if (d->basis != FE2_BASIS_DIRAC && d->basis != FE2_BASIS_ELEMENT) return set_error("unknown basis"), FE2_EINVAL;
  if (d->n_macro < 1 || d->n_micro < 1 || d->order * d->n_micro < 2)
    return set_error("need at least one macro element and one interior RVE node"), FE2_EINVAL;
  if (d->n_macro > (1 << 20)) return set_error("macro mesh too large"), FE2_EINVAL;
  // the RVE factor, pivots and K_Fw are staged in 64 KiB of LDS
  if ((static_cast<int64_t>(d->order) * d->n_micro - 1) * (d->order + 3) > 8192)
    return set_error("RVE too large: (order * n_micro - 1) * (order + 3) must not exceed 8192"), FE2_EINVAL;
  if (!(d->macro_length > 0.0) || !d->lambda_gp) return set_error("bad macro length or material table"), FE2_EINVAL;
  for (int k = 0; k < d->n_micro * NG_MICRO; ++k)
    if (!(d->lambda_gp[k] > 0.0)) return set_error("lambda must be positive"), FE2_EINVAL;
  fe2_1d_ctx* h = new (std::nothrow) fe2_1d_ctx();
  if (!h) return set_error("host allocation failed"), FE2_ENOMEM;
  const int rc = setup_1d(h, d, static_cast<hipStream_t>(stream));
  if (rc) {
    (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
    free_1d(h);
    return rc;
  }
  *out = h;
  return FE2_OK;
}

int fe2_1d_newton_step(fe2_1d_handle h, double* norms_host, void* stream) {
  if (!h) return set_error("null handle"), FE2_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const OneD& o = h->o;
  const size_t wl = static_cast<size_t>(o.n_int) * o.n_rve;
  hipLaunchKernelGGL(k1d_resid, dim3(nb(wl, 256)), dim3(256), 0, s, o, h->phi, h->w, h->kw, h->kfw, h->wtmp, h->Fb);
  const size_t lds = (static_cast<size_t>(o.n_int) * (o.q + 1) + 2 * o.n_int) * sizeof(double);
  hipLaunchKernelGGL(o.q == 1 ? k1d_rve<1> : k1d_rve<2>, dim3(nb(o.n_rve, 64)), dim3(64), lds, s, o, h->wtmp, h->w, h->kw, h->rinv, h->kfw,
                     h->scal, h->Fb, h->xr, h->pbar, h->phat, h->rn2);
  hipLaunchKernelGGL(k1d_macro_elem, dim3(nb(o.n_mac, 64)), dim3(64), 0, s, o, h->phi, h->pbar, h->phat, h->scal,
                     h->fe_t, h->fe_h, h->ke);
  hipLaunchKernelGGL(k1d_macro_rows, dim3(nb(o.n_phi, 64)), dim3(64), 0, s, o, h->fe_t, h->fe_h, h->ke, h->band,
                     h->rhs, h->rtrue, h->fint);
  hipLaunchKernelGGL(k1d_norms, dim3(1), dim3(256), 0, s, o, h->rtrue, h->fint, h->rn2, h->norms);
  FE2_HIP_CHECK(hipGetLastError());
  FE2_HIP_CHECK(hipMemsetAsync(h->info, 0, sizeof(int), s));
  const int rc = bcr_solve(h->plan, h->ws, h->band, h->rhs, h->info, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k1d_axpy, dim3(nb(o.n_phi, 256)), dim3(256), 0, s, o.n_phi, h->rhs, h->phi);
  hipLaunchKernelGGL(k1d_update, dim3(nb(wl, 256)), dim3(256), 0, s, o, h->rhs, h->xr, h->xf, h->w);
  FE2_HIP_CHECK(hipGetLastError());
  int info = 0;
  FE2_HIP_CHECK(hipMemcpyAsync(h->norms_host, h->norms, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  FE2_HIP_CHECK(hipMemcpyAsync(&info, h->info, sizeof(int), hipMemcpyDeviceToHost, s));
  FE2_HIP_CHECK(hipStreamSynchronize(s));
  if (info) return set_error("macro tangent not positive definite"), FE2_EINVAL;
  if (norms_host)
    for (int k = 0; k < 4; ++k) norms_host[k] = h->norms_host[k];
  return FE2_OK;
}

int fe2_1d_get_state(fe2_1d_handle h, double* phi_dev, double* w_dev, void* stream) {
  if (!h) return set_error("null handle"), FE2_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const OneD& o = h->o;
  if (phi_dev) FE2_HIP_CHECK(hipMemcpyAsync(phi_dev, h->phi, sizeof(double) * o.n_phi, hipMemcpyDeviceToDevice, s));
  if (w_dev) {
    const size_t n = static_cast<size_t>(o.n_int) * o.n_rve;
    hipLaunchKernelGGL(k1d_transpose, dim3(nb(n, 256)), dim3(256), 0, s, o.n_int, o.n_rve, h->w, w_dev);
    FE2_HIP_CHECK(hipGetLastError());
  }
  return FE2_OK;
}

int fe2_1d_query(fe2_1d_handle h, int which, int64_t* out) {
  if (!h || !out) return set_error("null argument"), FE2_EINVAL;
  switch (which) {
    case FE2_1D_Q_N_PHI: *out = h->o.n_phi; return FE2_OK;
    case FE2_1D_Q_N_RVE: *out = h->o.n_rve; return FE2_OK;
    case FE2_1D_Q_N_INT: *out = h->o.n_int; return FE2_OK;
    default: return set_error("unknown query"), FE2_EINVAL;
  }
}

int fe2_1d_destroy(fe2_1d_handle h) {
  if (!h) return FE2_OK;
  (void)hipDeviceSynchronize();
  free_1d(h);
  return FE2_OK;
}

}  // extern "C"
