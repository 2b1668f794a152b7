// Macro side of the monolithic FE^2 step (FP64 throughout), Hesch, Schmidt,
// Schuss, arXiv:2312.12771:
//   * reference tables of the RVE box element (setup);
//   * macro Gauss-point geometry and the macro gradient at every RVE
//     (Eqs. (25)-(28), (11));
//   * element tangents and residuals from the condensed Cbar_b, Phat_b and
//     the averaged Pbar_b (Eqs. (35), (39), (48));
//   * deterministic row-gather assembly into band storage with Dirichlet
//     elimination;
//   * banded Cholesky factorisation and solve in one work-group (the macro
//     system of Eq. (48));
//   * fluctuation update dw_b = -(x_r + X_F dF_b) (Eq. (49)) and the residual
//     norms of the convergence test;
//   * the piecewise-constant macro basis of the fluctuation (Eqs.
//     (constSolution1)-(constSolution2), small strain): RVE b = element e,
//     driven by the element-average strain, with the in-element strain
//     variation carried by the volume-averaged elasticity C_V.
#include "macro.hpp"
#include "elem3d.hpp"

namespace fe2 {

// ---------------------------------------------------------------------------
// setup: reference tables of a box element (2D: Q4, plane strain)
// ---------------------------------------------------------------------------
// K_ref = sum_gp w B^T C0 B, KwF = sum_gp w B^T C0, KFF = sum_gp w C0 with
// C0 = C(lambda = rho, mu = 1); then the ten distinct entries of K_ref and a
// consistency flag (every entry equals sign * kv[id]).
__global__ void k_ref_tables_2d(double h1, double h2, double rho, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double g = 0.57735026918962576451;   // 1/sqrt(3)
  const double C[3][3] = {{rho + 2.0, rho, 0.0}, {rho, rho + 2.0, 0.0}, {0.0, 0.0, 1.0}};
  const double xa[4] = {-1, 1, 1, -1}, ya[4] = {-1, -1, 1, 1};
  double K[8][8] = {};
  double KwF[8][3] = {};
  double KFF[3][3] = {};
  const double wt = 0.25 * h1 * h2;
  for (int gy = 0; gy < 2; ++gy)
    for (int gx = 0; gx < 2; ++gx) {
      const double xi = gx ? g : -g, eta = gy ? g : -g;
      double B[3][8] = {};
      for (int a = 0; a < 4; ++a) {
        const double dx = 0.25 * xa[a] * (1.0 + ya[a] * eta) * (2.0 / h1);
        const double dy = 0.25 * ya[a] * (1.0 + xa[a] * xi) * (2.0 / h2);
        B[0][2 * a] = dx;
        B[1][2 * a + 1] = dy;
        B[2][2 * a] = dy;
        B[2][2 * a + 1] = dx;
      }
      for (int r = 0; r < 8; ++r) {
        double CB[3];
        for (int i = 0; i < 3; ++i) CB[i] = C[i][0] * B[0][r] + C[i][1] * B[1][r] + C[i][2] * B[2][r];
        for (int c = 0; c < 8; ++c) K[r][c] += wt * (CB[0] * B[0][c] + CB[1] * B[1][c] + CB[2] * B[2][c]);
        for (int j = 0; j < 3; ++j) KwF[r][j] += wt * CB[j];
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) KFF[i][j] += wt * C[i][j];
    }
  double kv[10] = {};
  bool seen[10] = {};
  double err = 0.0, scale = 0.0;
  for (int r = 0; r < 8; ++r)
    for (int c = 0; c < 8; ++c) {
      const int id = kref_id(r, c);
      const double v = kref_sign(r, c) * K[r][c];
      if (!seen[id]) {
        kv[id] = v;
        seen[id] = true;
      }
      err = fmax(err, fabs(v - kv[id]));
      scale = fmax(scale, fabs(K[r][c]));
    }
  // Mode constants: for a box element the bilinear strain energy separates
  // into the projections of (u_x, u_y) on the corner patterns bx = (-1,1,1,-1),
  // by = (-1,-1,1,1) and g = (1,-1,1,-1): with X1 = bx.ux, Y2 = by.uy,
  // Sx = by.ux, Sy = bx.uy, Hx = g.ux, Hy = g.uy,
  //   G1 = k0 X1 + k1 Y2, G2 = k2 X1 + k3 Y2, G3 = k4 Sx + k5 Sy,
  //   G4 = k6 Sx + k7 Sy, G5 = k8 Hx, G6 = k9 Hy,
  //   f_x = bx G1 + by G3 + g G5,  f_y = bx G4 + by G2 + g G6.
  // Each constant is read off K applied to one pure pattern (a pattern has
  // squared norm 4 and is orthogonal to the others).
  const double pat[3][4] = {{-1, 1, 1, -1}, {-1, -1, 1, 1}, {1, -1, 1, -1}};   // bx, by, g
  auto apply = [&](int comp, int p, double f[8]) {   // f = K u, u_comp = pattern p
    for (int r = 0; r < 8; ++r) {
      f[r] = 0.0;
      for (int a = 0; a < 4; ++a) f[r] += K[r][2 * a + comp] * pat[p][a];
    }
  };
  auto proj = [&](const double f[8], int comp, int p) {
    double v = 0.0;
    for (int a = 0; a < 4; ++a) v += pat[p][a] * f[2 * a + comp];
    return v / 16.0;
  };
  double km[10], f[8];
  apply(0, 0, f);   // ux = bx: X1 = 4
  km[0] = proj(f, 0, 0);
  km[2] = proj(f, 1, 1);
  apply(1, 1, f);   // uy = by: Y2 = 4
  km[1] = proj(f, 0, 0);
  km[3] = proj(f, 1, 1);
  apply(0, 1, f);   // ux = by: Sx = 4
  km[4] = proj(f, 0, 1);
  km[6] = proj(f, 1, 0);
  apply(1, 0, f);   // uy = bx: Sy = 4
  km[5] = proj(f, 0, 1);
  km[7] = proj(f, 1, 0);
  apply(0, 2, f);   // ux = g: Hx = 4
  km[8] = proj(f, 0, 2);
  apply(1, 2, f);   // uy = g: Hy = 4
  km[9] = proj(f, 1, 2);
  // the mode form must reproduce every column of K
  for (int c = 0; c < 8; ++c) {
    double ux[4] = {}, uy[4] = {};
    (c & 1 ? uy : ux)[c / 2] = 1.0;
    double P[2][3];   // projections of ux, uy on bx, by, g
    for (int p = 0; p < 3; ++p) {
      P[0][p] = P[1][p] = 0.0;
      for (int a = 0; a < 4; ++a) {
        P[0][p] += pat[p][a] * ux[a];
        P[1][p] += pat[p][a] * uy[a];
      }
    }
    const double G1 = km[0] * P[0][0] + km[1] * P[1][1], G2 = km[2] * P[0][0] + km[3] * P[1][1];
    const double G3 = km[4] * P[0][1] + km[5] * P[1][0], G4 = km[6] * P[0][1] + km[7] * P[1][0];
    const double G5 = km[8] * P[0][2], G6 = km[9] * P[1][2];
    for (int a = 0; a < 4; ++a) {
      const double fx = pat[0][a] * G1 + pat[1][a] * G3 + pat[2][a] * G5;
      const double fy = pat[0][a] * G4 + pat[1][a] * G2 + pat[2][a] * G6;
      err = fmax(err, fmax(fabs(fx - K[2 * a][c]), fabs(fy - K[2 * a + 1][c])));
    }
  }
  // layout: kv[10] | KwF[24] | KFF[9] | consistency error | mode constants[10]
  for (int t = 0; t < 10; ++t) out[t] = kv[t];
  for (int r = 0; r < 8; ++r)
    for (int j = 0; j < 3; ++j) out[10 + 3 * r + j] = KwF[r][j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) out[34 + 3 * i + j] = KFF[i][j];
  out[43] = err / scale;
  for (int t = 0; t < 10; ++t) out[44 + t] = km[t];
}

// Reference tables of the hex8 box element (cube of side h, lambda = rho,
// mu = 1) by 2x2x2 Gauss quadrature, Voigt order [11,22,33,23,13,12] with
// engineering shear: out = kv[10] | KwF[24][6] | KFF[6][6] | consistency
// error of K against the ten-value structure of kref3_id / kref3_sign.
__global__ void k_ref_tables_3d(double h, double rho, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double g = 0.57735026918962576451;
  double C[6][6] = {};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i][j] = rho + (i == j ? 2.0 : 0.0);
  C[3][3] = C[4][4] = C[5][5] = 1.0;
  double K[24][24] = {};
  double KwF[24][6] = {};
  double KFF[6][6] = {};
  const double wt = 0.125 * h * h * h;
  for (int gp = 0; gp < 8; ++gp) {
    const double xi[3] = {(gp & 1) ? g : -g, (gp & 2) ? g : -g, (gp & 4) ? g : -g};
    double B[6][24] = {};
    for (int a = 0; a < 8; ++a) {
      double dN[3];
      for (int f = 0; f < 3; ++f) {
        double v = 0.125 * hsg(a, f) * (2.0 / h);
        for (int k = 0; k < 3; ++k)
          if (k != f) v *= 1.0 + hsg(a, k) * xi[k];
        dN[f] = v;
      }
      B[0][3 * a] = dN[0];
      B[1][3 * a + 1] = dN[1];
      B[2][3 * a + 2] = dN[2];
      B[3][3 * a + 1] = dN[2];
      B[3][3 * a + 2] = dN[1];
      B[4][3 * a] = dN[2];
      B[4][3 * a + 2] = dN[0];
      B[5][3 * a] = dN[1];
      B[5][3 * a + 1] = dN[0];
    }
    for (int r = 0; r < 24; ++r) {
      double CB[6];
      for (int i = 0; i < 6; ++i) {
        CB[i] = 0.0;
        for (int k = 0; k < 6; ++k) CB[i] += C[i][k] * B[k][r];
      }
      for (int c = 0; c < 24; ++c) {
        double v = 0.0;
        for (int i = 0; i < 6; ++i) v += CB[i] * B[i][c];
        K[r][c] += wt * v;
      }
      for (int j = 0; j < 6; ++j) KwF[r][j] += wt * CB[j];
    }
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) KFF[i][j] += wt * C[i][j];
  }
  double kv[10] = {};
  bool seen[10] = {};
  double err = 0.0, scale = 0.0;
  for (int r = 0; r < 24; ++r)
    for (int c = 0; c < 24; ++c) {
      const int id = kref3_id(r, c);
      const double v = kref3_sign(r, c) * K[r][c];
      if (!seen[id]) {
        kv[id] = v;
        seen[id] = true;
      }
      err = fmax(err, fabs(v - kv[id]));
      scale = fmax(scale, fabs(K[r][c]));
    }
  for (int t = 0; t < 10; ++t) out[t] = kv[t];
  for (int r = 0; r < 24; ++r)
    for (int j = 0; j < 6; ++j) out[10 + 6 * r + j] = KwF[r][j];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) out[154 + 6 * i + j] = KFF[i][j];
  out[190] = err / scale;
}

// ---------------------------------------------------------------------------
// macro Gauss-point geometry (setup)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ref_node(int dim, int a, double* xa) {
  const int cx = (a & 3) == 1 || (a & 3) == 2;
  const int cy = (a & 3) >= 2;
  xa[0] = cx ? 1.0 : -1.0;
  xa[1] = cy ? 1.0 : -1.0;
  if (dim == 3) xa[2] = a >= 4 ? 1.0 : -1.0;
}

// Quadratic 1D Lagrange polynomial on the nodes -1, 0, 1 (node index k = 0,
// 1, 2 for -1, 1, 0 as in the Q9 numbering below) and its derivative.
__device__ __forceinline__ void lagrange2(double x, int k, double* l, double* dl) {
  if (k == 0) {
    *l = 0.5 * x * (x - 1.0);
    *dl = x - 0.5;
  } else if (k == 1) {
    *l = 0.5 * x * (x + 1.0);
    *dl = x + 0.5;
  } else {
    *l = 1.0 - x * x;
    *dl = -2.0 * x;
  }
}

// Reference derivatives dN_a/dxi_J of the nen shape functions at xi, and the
// Gauss weight of point g.  Order 1: Q4 / hex8 at (+-1/sqrt3)^dim, weight 1.
// Order 2: biquadratic Q9 (tensor products of the quadratic Lagrange
// polynomials; corners, then mid-sides of the bottom, right, top and left
// edges, then the centre) at the 3x3 Gauss points +-sqrt(3/5), 0 with weights
// 5/9, 8/9, 5/9, xi fastest.
__device__ __forceinline__ double macro_ref_derivs(const MacroArgs& m, int g, double (*dxi)[3]) {
  const int dim = m.dim;
  if (m.order == 2) {
    const double gx[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
    const double gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    const int ix = g % 3, iy = g / 3;
    // 1D node index per Q9 node along xi and eta (0: -1, 1: +1, 2: 0)
    const int kx[9] = {0, 1, 1, 0, 2, 1, 2, 0, 2};
    const int ky[9] = {0, 0, 1, 1, 0, 2, 1, 2, 2};
    for (int a = 0; a < 9; ++a) {
      double lx, dlx, ly, dly;
      lagrange2(gx[ix], kx[a], &lx, &dlx);
      lagrange2(gx[iy], ky[a], &ly, &dly);
      dxi[a][0] = dlx * ly;
      dxi[a][1] = lx * dly;
    }
    return gw[ix] * gw[iy];
  }
  const double gq = 0.57735026918962576451;
  double xi[3];
  xi[0] = (g & 1) ? gq : -gq;
  xi[1] = (g & 2) ? gq : -gq;
  xi[2] = (g & 4) ? gq : -gq;
  for (int a = 0; a < m.nen; ++a) {
    double na[3];
    ref_node(dim, a, na);
    for (int J = 0; J < dim; ++J) {
      double v = (dim == 2) ? 0.25 : 0.125;
      for (int K = 0; K < dim; ++K) v *= (K == J) ? na[K] : (1.0 + na[K] * xi[K]);
      dxi[a][J] = v;
    }
  }
  return 1.0;
}

// Geometry of macro Gauss point q = e * n_gp + g: dN/dX and wdet = w_g det J.
__global__ void k_macro_geometry(MacroArgs m) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= m.n_qp) return;
  const int dim = m.dim, nen = m.nen, ngp = m.n_gp;
  const int e = b / ngp, g = b % ngp;
  double dxi[9][3];
  const double wg = macro_ref_derivs(m, g, dxi);
  double Jm[3][3] = {};
  for (int a = 0; a < nen; ++a) {
    const int node = m.conn[e * nen + a];
    for (int i = 0; i < dim; ++i)
      for (int J = 0; J < dim; ++J) Jm[i][J] += m.X[node * dim + i] * dxi[a][J];
  }
  double inv[3][3], det;
  if (dim == 2) {
    det = Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0];
    inv[0][0] = Jm[1][1] / det;
    inv[0][1] = -Jm[0][1] / det;
    inv[1][0] = -Jm[1][0] / det;
    inv[1][1] = Jm[0][0] / det;
  } else {
    det = Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) -
          Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0]) +
          Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
    inv[0][0] = (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) / det;
    inv[0][1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) / det;
    inv[0][2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) / det;
    inv[1][0] = (Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2]) / det;
    inv[1][1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) / det;
    inv[1][2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) / det;
    inv[2][0] = (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]) / det;
    inv[2][1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) / det;
    inv[2][2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) / det;
  }
  // dN/dX_J = sum_K dN/dxi_K (J^-1)_KJ
  for (int a = 0; a < nen; ++a)
    for (int J = 0; J < dim; ++J) {
      double v = 0.0;
      for (int K = 0; K < dim; ++K) v += dxi[a][K] * inv[K][J];
      m.dNdX[(static_cast<size_t>(b) * nen + a) * dim + J] = v;
    }
  m.wdet[b] = wg * det;
}

// Weight of RVE b in the micro residual rows: wdet of its Gauss point (Dirac
// basis) or the element volume V_e = sum_g wdet_g (element basis).
__global__ void k_rve_weight(MacroArgs m) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= m.n_rve) return;
  if (m.basis == FE2_BASIS_ELEMENT) {
    double v = 0.0;
    for (int g = 0; g < m.n_gp; ++g) v += m.wdet[b * m.n_gp + g];
    m.vol[b] = v;
  } else {
    m.vol[b] = m.wdet[b];
  }
}

// macro strain-displacement (small) or gradient (finite) operator entry
// B[i][col] at Gauss point q (= b with the Dirac basis), col = a*dim + c.
__device__ __forceinline__ double macro_B(const MacroArgs& m, int b, int i, int col) {
  const int dim = m.dim;
  const int a = col / dim, c = col % dim;
  const double* d = m.dNdX + (static_cast<size_t>(b) * m.nen + a) * dim;
  if (m.kin == FE2_FINITE_STRAIN) {   // row (p, J) = dim*p + J: dN_a/dX_J if p == c
    const int p = i / dim, J = i % dim;
    return p == c ? d[J] : 0.0;
  }
  if (dim == 2) {
    switch (i) {
      case 0: return c == 0 ? d[0] : 0.0;
      case 1: return c == 1 ? d[1] : 0.0;
      default: return c == 0 ? d[1] : d[0];
    }
  }
  switch (i) {   // [11, 22, 33, 23, 13, 12]
    case 0: return c == 0 ? d[0] : 0.0;
    case 1: return c == 1 ? d[1] : 0.0;
    case 2: return c == 2 ? d[2] : 0.0;
    case 3: return c == 1 ? d[2] : (c == 2 ? d[1] : 0.0);
    case 4: return c == 0 ? d[2] : (c == 2 ? d[0] : 0.0);
    default: return c == 0 ? d[1] : (c == 1 ? d[0] : 0.0);
  }
}

// Element-average operator Bbar[i][col] = sum_g wdet_g B_g[i][col] / V_e.
__device__ __forceinline__ double macro_Bbar(const MacroArgs& m, int e, int i, int col) {
  double v = 0.0;
  for (int g = 0; g < m.n_gp; ++g) {
    const int q = e * m.n_gp + g;
    v += m.wdet[q] * macro_B(m, q, i, col);
  }
  return v / m.vol[e];
}

// Gradient operator of RVE b: B_b (Dirac basis) or Bbar_e (element basis).
__device__ __forceinline__ double rve_B(const MacroArgs& m, int b, int i, int col) {
  return m.basis == FE2_BASIS_ELEMENT ? macro_Bbar(m, b, i, col) : macro_B(m, b, i, col);
}

__device__ __forceinline__ int elem_of_rve(const MacroArgs& m, int b) {
  return m.basis == FE2_BASIS_ELEMENT ? b : b / m.n_gp;
}

// Volume average C_V of the micro elasticity of RVE b (small strain, Voigt
// with engineering shear): (1 - phi) C(lambda_0, mu_0) + phi C(lambda_1, mu_1),
// phi the phase-1 fraction (all RVE elements have the same volume).
__device__ __forceinline__ void voigt_average(const MacroArgs& m, int b, double (&C)[36]) {
  const double* p = m.kpar + static_cast<size_t>(b) * 4;
  const double f = m.phi[b];
  const double lam = (1.0 - f) * p[0] + f * p[2];
  const double mu = (1.0 - f) * p[1] + f * p[3];
  const int nF = m.nF, nn = m.dim;   // normal components come first
  for (int i = 0; i < nF; ++i)
    for (int j = 0; j < nF; ++j) {
      double v = 0.0;
      if (i < nn && j < nn) v = lam + (i == j ? 2.0 * mu : 0.0);
      else if (i == j) v = mu;
      C[i * nF + j] = v;
    }
}

// a2: macro gradient of every RVE from the displacement u = q - X (element
// basis: the element average, exact for the RVE's residual, which is linear
// in the macro strain).
__global__ void k_macro_grad(MacroArgs m, const double* __restrict__ u, double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= m.n_rve) return;
  const int e = elem_of_rve(m, b);
  const int nd = m.nen * m.dim;
  for (int i = 0; i < m.nF; ++i) {
    double v = 0.0;
    for (int col = 0; col < nd; ++col) {
      const int node = m.conn[e * m.nen + col / m.dim];
      v += rve_B(m, b, i, col) * u[node * m.dim + col % m.dim];
    }
    if (m.kin == FE2_FINITE_STRAIN && (i / m.dim) == (i % m.dim)) v += 1.0;
    out[static_cast<size_t>(b) * m.nF + i] = v;
  }
}

// Element-basis residual row: P_g = P_e + C_V (eps_g - epsbar_e) at Gauss
// point g, from the current displacement u.
__device__ __noinline__ double elem_vec_row_element(const MacroArgs& m, const double* __restrict__ P,
                                                    const double* __restrict__ u, int e, int row) {
  const int nd = m.nen * m.dim, nF = m.nF;
  double ue[24], CV[36], eps[8][6], ebar[6];
  for (int col = 0; col < nd; ++col) ue[col] = u[m.conn[e * m.nen + col / m.dim] * m.dim + col % m.dim];
  voigt_average(m, e, CV);
  for (int i = 0; i < nF; ++i) ebar[i] = 0.0;
  for (int g = 0; g < m.n_gp; ++g) {
    const int q = e * m.n_gp + g;
    for (int i = 0; i < nF; ++i) {
      double s = 0.0;
      for (int col = 0; col < nd; ++col) s += macro_B(m, q, i, col) * ue[col];
      eps[g][i] = s;
      ebar[i] += m.wdet[q] * s;
    }
  }
  for (int i = 0; i < nF; ++i) ebar[i] /= m.vol[e];
  const double* Pe = P + static_cast<size_t>(e) * nF;
  double v = 0.0;
  for (int g = 0; g < m.n_gp; ++g) {
    const int q = e * m.n_gp + g;
    double s = 0.0;
    for (int i = 0; i < nF; ++i) {
      double pg = Pe[i];
      for (int j = 0; j < nF; ++j) pg += CV[i * nF + j] * (eps[g][j] - ebar[j]);
      s += macro_B(m, q, i, row) * pg;
    }
    v += m.wdet[q] * s;
  }
  return v;
}

// a7 (part): element residual vectors  f = sum_g wdet B^T P  for P = Pbar
// (true residual) and P = Phat (condensed right-hand side); the element
// basis uses the row form above.  One thread per (element, row).
__global__ void k_macro_elem_vec(MacroArgs m, const double* __restrict__ P, double* __restrict__ f,
                                 const double* __restrict__ u) {
  const int nd = m.nen * m.dim;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_elems * nd) return;
  const int e = t / nd, row = t % nd;
  if (m.basis == FE2_BASIS_ELEMENT) {
    f[t] = elem_vec_row_element(m, P, u, e, row);
    return;
  }
  double v = 0.0;
  for (int g = 0; g < m.n_gp; ++g) {
    const int b = e * m.n_gp + g;
    double s = 0.0;
    for (int i = 0; i < m.nF; ++i) s += macro_B(m, b, i, row) * P[static_cast<size_t>(b) * m.nF + i];
    v += m.wdet[b] * s;
  }
  f[t] = v;
}

// Element-basis tangent row: sum_g wdet_g B_g^T C_V B_g + V_e Bbar^T
// (Cbar_e - C_V) Bbar (its own function: the local C_V lives in private
// memory, which the Dirac path must not pay for).
__device__ __noinline__ void elem_mat_row_element(const MacroArgs& m, const double* __restrict__ Cb, int e, int row,
                                                  double* acc) {
  const int nd = m.nen * m.dim, nF = m.nF;
  double CV[36];
  voigt_average(m, e, CV);
  for (int g = 0; g < m.n_gp; ++g) {
    const int q = e * m.n_gp + g;
    double tj[6];
    for (int j = 0; j < nF; ++j) {
      double s = 0.0;
      for (int i = 0; i < nF; ++i) s += macro_B(m, q, i, row) * CV[i * nF + j];
      tj[j] = s * m.wdet[q];
    }
    for (int c = 0; c < nd; ++c) {
      double s = 0.0;
      for (int j = 0; j < nF; ++j) s += tj[j] * macro_B(m, q, j, c);
      acc[c] += s;
    }
  }
  const double* C = Cb + static_cast<size_t>(e) * nF * nF;
  double tj[6];
  for (int j = 0; j < nF; ++j) {
    double s = 0.0;
    for (int i = 0; i < nF; ++i) s += macro_Bbar(m, e, i, row) * (C[i * nF + j] - CV[i * nF + j]);
    tj[j] = s * m.vol[e];
  }
  for (int c = 0; c < nd; ++c) {
    double s = 0.0;
    for (int j = 0; j < nF; ++j) s += tj[j] * macro_Bbar(m, e, j, c);
    acc[c] += s;
  }
}

// a7 (part): element tangents  k = sum_g wdet B^T Cbar B (Dirac basis) or
// the element-basis form above, one thread per (element, row).
// Gradient operator with the element's dimension and kinematics fixed at
// compile time (the values macro_B computes for them).
template <int DIM, bool FINITE>
__device__ __forceinline__ double macro_B_t(const double* __restrict__ d, int i, int c) {
  if constexpr (FINITE) {
    return i / DIM == c ? d[i % DIM] : 0.0;
  } else if constexpr (DIM == 2) {
    return i == 0 ? (c == 0 ? d[0] : 0.0) : i == 1 ? (c == 1 ? d[1] : 0.0) : (c == 0 ? d[1] : d[0]);
  } else {
    switch (i) {   // [11, 22, 33, 23, 13, 12]
      case 0: return c == 0 ? d[0] : 0.0;
      case 1: return c == 1 ? d[1] : 0.0;
      case 2: return c == 2 ? d[2] : 0.0;
      case 3: return c == 1 ? d[2] : (c == 2 ? d[1] : 0.0);
      case 4: return c == 0 ? d[2] : (c == 2 ? d[0] : 0.0);
      default: return c == 0 ? d[1] : (c == 1 ? d[0] : 0.0);
    }
  }
}

// Row `row` of the element matrix, Dirac basis, the sizes fixed at compile
// time so that the row and the products stay in registers; the same sums in
// the same order as the general path of k_macro_elem_mat.
template <int DIM, int NEN, int NF, bool FINITE>
__device__ __forceinline__ void elem_mat_row_dirac(const MacroArgs& m, const double* __restrict__ Cb, int e, int row,
                                                   double* __restrict__ out) {
  constexpr int ND = NEN * DIM;
  double acc[ND];
#pragma unroll
  for (int c = 0; c < ND; ++c) acc[c] = 0.0;
  const int ra = row / DIM, rc = row % DIM;
  for (int g = 0; g < m.n_gp; ++g) {
    const int b = e * m.n_gp + g;
    const double* C = Cb + static_cast<size_t>(b) * NF * NF;
    const double* dN = m.dNdX + static_cast<size_t>(b) * NEN * DIM;
    double dr[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) dr[k] = dN[ra * DIM + k];
    double tj[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      double s2 = 0.0;
#pragma unroll
      for (int i = 0; i < NF; ++i) s2 += macro_B_t<DIM, FINITE>(dr, i, rc) * C[i * NF + j];
      tj[j] = s2 * m.wdet[b];
    }
#pragma unroll
    for (int a = 0; a < NEN; ++a) {
      double da[DIM];
#pragma unroll
      for (int k = 0; k < DIM; ++k) da[k] = dN[a * DIM + k];
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        double s2 = 0.0;
#pragma unroll
        for (int j = 0; j < NF; ++j) s2 += tj[j] * macro_B_t<DIM, FINITE>(da, j, c);
        acc[a * DIM + c] += s2;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < ND; ++c) out[c] = acc[c];
}

__global__ void k_macro_elem_mat(MacroArgs m, const double* __restrict__ Cb, double* __restrict__ ke) {
  const int nd = m.nen * m.dim;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_elems * nd) return;
  const int e = t / nd, row = t % nd;
  const int nF = m.nF;
  double acc[24];
  for (int c = 0; c < nd; ++c) acc[c] = 0.0;
  if (m.basis == FE2_BASIS_ELEMENT) {
    elem_mat_row_element(m, Cb, e, row, acc);
  } else {
    for (int g = 0; g < m.n_gp; ++g) {
      const int b = e * m.n_gp + g;
      const double* C = Cb + static_cast<size_t>(b) * nF * nF;
      double tj[9];
      for (int j = 0; j < nF; ++j) {
        double s = 0.0;
        for (int i = 0; i < nF; ++i) s += macro_B(m, b, i, row) * C[i * nF + j];
        tj[j] = s * m.wdet[b];
      }
      for (int c = 0; c < nd; ++c) {
        double s = 0.0;
        for (int j = 0; j < nF; ++j) s += tj[j] * macro_B(m, b, j, c);
        acc[c] += s;
      }
    }
  }
  for (int c = 0; c < nd; ++c) ke[static_cast<size_t>(t) * nd + c] = acc[c];
}

template <int DIM, int NEN, int NF, bool FINITE>
__global__ void k_macro_elem_mat_t(MacroArgs m, const double* __restrict__ Cb, double* __restrict__ ke) {
  constexpr int ND = NEN * DIM;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.n_elems * ND) return;
  elem_mat_row_dirac<DIM, NEN, NF, FINITE>(m, Cb, t / ND, t % ND, ke + static_cast<size_t>(t) * ND);
}

void launch_macro_elem_mat(const MacroArgs& m, const double* Cb, double* ke, hipStream_t s) {
  const int nd = m.nen * m.dim;
  const dim3 grid(static_cast<unsigned>((static_cast<size_t>(m.n_elems) * nd + 63) / 64)), block(64);
  const bool fin = m.kin == FE2_FINITE_STRAIN;
  if (m.basis != FE2_BASIS_ELEMENT) {   // sized kernels for the 2D element types (3D hex8 would spill)
    if (m.dim == 2 && m.nen == 4 && !fin && m.nF == 3)
      { hipLaunchKernelGGL((k_macro_elem_mat_t<2, 4, 3, false>), grid, block, 0, s, m, Cb, ke); return; }
    if (m.dim == 2 && m.nen == 4 && fin && m.nF == 4)
      { hipLaunchKernelGGL((k_macro_elem_mat_t<2, 4, 4, true>), grid, block, 0, s, m, Cb, ke); return; }
    if (m.dim == 2 && m.nen == 9 && !fin && m.nF == 3)
      { hipLaunchKernelGGL((k_macro_elem_mat_t<2, 9, 3, false>), grid, block, 0, s, m, Cb, ke); return; }
  }
  hipLaunchKernelGGL(k_macro_elem_mat, grid, block, 0, s, m, Cb, ke);
}

// Row-wise residual gather: R_true = F_int - lam f_ext, F_int, and the
// condensed right-hand side rhs = lam f_ext - sum f_hat (Dirichlet rows get
// their prescribed increment later).  One thread per DOF; contributions in a
// fixed order (deterministic).
__global__ void k_macro_rows_vec(MacroArgs m, const double* __restrict__ f_true,
                                 const double* __restrict__ f_hat, double lam,
                                 double* __restrict__ r_true, double* __restrict__ f_int,
                                 double* __restrict__ rhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.ndof) return;
  double ft = 0.0, fh = 0.0;
  for (int k = m.vec_ptr[i]; k < m.vec_ptr[i + 1]; ++k) {
    const int src = m.vec_src[k];
    ft += f_true[src];
    if (f_hat) fh += f_hat[src];
  }
  const double fe = m.f_ext ? lam * m.f_ext[i] : 0.0;
  if (f_int) f_int[i] = ft;
  if (r_true) r_true[i] = ft - fe;
  if (rhs) rhs[i] = fe - fh;
}

// Band assembly with Dirichlet elimination.  Row i gathers every nonzero
// K_ij from the element matrices; free/free entries with j <= i go to the
// lower band L[j*(bw+1) + (i-j)], free/Dirichlet entries move to the
// right-hand side, Dirichlet rows become identity rows with rhs = du_D.
__global__ void k_macro_rows_band(MacroArgs m, const double* __restrict__ ke, double dlam,
                                  double* __restrict__ band, double* __restrict__ rhs,
                                  double* __restrict__ kdense) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.ndof) return;
  const int bw1 = m.bw + 1;
  const bool diri = m.is_dir[i] != 0;
  double corr = 0.0;
  for (int k = m.nz_ptr[i]; k < m.nz_ptr[i + 1]; ++k) {
    const int j = m.nz_col[k];
    double v = 0.0;
    for (int s = m.nzc_ptr[k]; s < m.nzc_ptr[k + 1]; ++s) v += ke[m.nzc_src[s]];
    if (kdense) kdense[static_cast<size_t>(i) * m.ndof + j] = v;
    if (diri) continue;
    if (m.is_dir[j]) {
      corr += v * dlam * m.dir_full[j];
    } else if (j <= i) {
      band[static_cast<size_t>(j) * bw1 + (i - j)] = v;
    }
  }
  if (diri) {
    band[static_cast<size_t>(i) * bw1] = 1.0;
    rhs[i] = dlam * m.dir_full[i];
  } else {
    rhs[i] -= corr;
  }
}

__global__ void k_fill(double* p, size_t n, double v) {
  for (size_t t = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; t < n;
       t += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[t] = v;
}

__global__ void k_fill_i(int* p, size_t n, int v) {
  for (size_t t = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; t < n;
       t += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[t] = v;
}

// ---------------------------------------------------------------------------
// update and norms
// ---------------------------------------------------------------------------
__global__ void k_axpy(int n, const double* __restrict__ x, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

// a9: dF_b = B_b du_e (element basis: Bbar_e du_e); w_b -= x_r + X_F dF_b
// (generalized) or X_F dF_b (classical predictor).  One work-group per RVE.
// The products B_b[i][col] du_col run on one thread each (one dependent
// connectivity -> displacement load per thread instead of a chain of nd), and
// the first chunk of the RVE's columns is loaded before they are summed, so
// the stream over X and w does not wait for dF.  Every thread sums dF[i] over
// col in order from the shared products (same value on every thread).
template <int NF>
__global__ void __launch_bounds__(256) k_update_w(MacroArgs m, const double* __restrict__ du,
                                                  const int64_t* __restrict__ foff, const double* __restrict__ X,
                                                  double* __restrict__ w, int use_xr, const int* __restrict__ skip) {
  constexpr int U = 4;   // elements per thread and chunk
  const int b = blockIdx.x;
  if (skip && skip[b]) return;
  __shared__ double part[kUpdateMaxProducts];
  const int e = elem_of_rve(m, b);
  const int nd = m.nen * m.dim;
  for (int t = threadIdx.x; t < NF * nd; t += blockDim.x) {
    const int i = t / nd, col = t % nd;
    const int node = m.conn[e * m.nen + col / m.dim];
    part[t] = rve_B(m, b, i, col) * du[node * m.dim + col % m.dim];
  }
  const int64_t fo = foff[b];
  const int64_t flen = foff[b + 1] - fo;
  const double* Xb = X + fo * (NF + 1);
  const int64_t step = static_cast<int64_t>(U) * blockDim.x;
  double xv[U][NF + 1], wv[U];
  auto load = [&](int64_t t0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t t = t0 + static_cast<int64_t>(u) * blockDim.x;
      const bool in = t < flen;
      wv[u] = in ? w[fo + t] : 0.0;
#pragma unroll
      for (int j = 0; j < NF; ++j) xv[u][j] = in ? Xb[j * flen + t] : 0.0;
      xv[u][NF] = in && use_xr ? Xb[NF * flen + t] : 0.0;
    }
  };
  int64_t t0 = threadIdx.x;
  load(t0);
  __syncthreads();
  double dF[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    double v = 0.0;
    for (int col = 0; col < nd; ++col) v += part[i * nd + col];
    dF[i] = v;
  }
  while (true) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t t = t0 + static_cast<int64_t>(u) * blockDim.x;
      double dw = xv[u][NF];
#pragma unroll
      for (int j = 0; j < NF; ++j) dw += xv[u][j] * dF[j];
      if (t < flen) w[fo + t] = wv[u] - dw;
    }
    t0 += step;
    if (t0 >= flen) break;
    load(t0);
  }
}

int launch_update_w(const MacroArgs& m, int n_rve, const double* du, const int64_t* foff, const double* X,
                    double* w, int use_xr, const int* skip, hipStream_t s) {
  if (m.nF * m.nen * m.dim > kUpdateMaxProducts) return -1;
  switch (m.nF) {
    case 3: hipLaunchKernelGGL(k_update_w<3>, dim3(n_rve), dim3(256), 0, s, m, du, foff, X, w, use_xr, skip); break;
    case 4: hipLaunchKernelGGL(k_update_w<4>, dim3(n_rve), dim3(256), 0, s, m, du, foff, X, w, use_xr, skip); break;
    case 6: hipLaunchKernelGGL(k_update_w<6>, dim3(n_rve), dim3(256), 0, s, m, du, foff, X, w, use_xr, skip); break;
    case 9: hipLaunchKernelGGL(k_update_w<9>, dim3(n_rve), dim3(256), 0, s, m, du, foff, X, w, use_xr, skip); break;
    default: return -1;
  }
  return 0;
}

// Classical inner loop (Sec. 4.1): per-RVE stopping threshold
// thr2_b = tol^2 max(1, ||r_b^0||^2), the number of RVEs above it, and the
// Newton update w_b -= x_r of the RVEs' residual solves.
// Equilibrium threshold of the classical inner loop: ||r_b|| <= tol max(1,
// ||r_b^0||), but never below the rounding level 1e-14 S_b of the residual
// evaluation (S_b^2 = rsize2: summed squared element-level terms; may be null).
__global__ void k_micro_thr(int n_rve, const double* __restrict__ rnorm2, const double* __restrict__ rsize2,
                            double tol, double* __restrict__ thr2) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n_rve) thr2[b] = fmax(tol * tol * fmax(1.0, rnorm2[b]), rsize2 ? 1e-28 * rsize2[b] : 0.0);
}

__global__ void __launch_bounds__(1024) k_count_above(int n_rve, const double* __restrict__ rnorm2,
                                                      const double* __restrict__ thr2, const int* __restrict__ skip,
                                                      int* __restrict__ count) {
  __shared__ int part[16];
  int c = 0;
  for (int b = threadIdx.x; b < n_rve; b += blockDim.x) c += !(skip && skip[b]) && !(rnorm2[b] <= thr2[b]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < static_cast<int>(blockDim.x + 63) / 64; ++w) t += part[w];
    *count = t;
  }
}

__global__ void k_sub_xr(int nF, const int64_t* __restrict__ foff, const double* __restrict__ X,
                         const int* __restrict__ skip, double* __restrict__ w) {
  const int b = blockIdx.x;
  if (skip && skip[b]) return;
  const int64_t fo = foff[b];
  const int64_t flen = foff[b + 1] - fo;
  const double* xr = X + fo * (nF + 1) + nF * flen;
  for (int64_t t = threadIdx.x; t < flen; t += blockDim.x) w[fo + t] -= xr[t];
}

// RVEs whose last inner solve missed tol are excluded from further rounds
// (dead[b] = 1); count = number of RVEs excluded by this call.
__global__ void k_mark_dead(int n_rve, const double* __restrict__ relres, double tol, int* __restrict__ dead,
                            int* __restrict__ count) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_rve || dead[b]) return;
  if (!(relres[b] <= tol)) {
    dead[b] = 1;
    atomicAdd(count, 1);
  }
}

__global__ void k_copy_mask(int n, const int* __restrict__ src, int* __restrict__ dst) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n) dst[b] = src ? src[b] : 0;
}

// Norms of the convergence test: out = [||[R_free; R_micro]||, ||R_free||,
// ||R_micro||, ||F_int||] with R_micro,b = vol_b / |Omega| r_b (vol_b: wdet of
// the Gauss point, or the element volume with the element basis).
__global__ void __launch_bounds__(1024) k_norms(MacroArgs m, const double* __restrict__ r_true,
                                                const double* __restrict__ f_int,
                                                const double* __restrict__ rnorm2, double volume,
                                                double* __restrict__ out) {
  __shared__ double red[3][16];
  double s[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < m.ndof; i += blockDim.x) {
    if (!m.is_dir[i]) s[0] += r_true[i] * r_true[i];
    s[2] += f_int[i] * f_int[i];
  }
  for (int b = threadIdx.x; b < m.n_rve; b += blockDim.x) {
    const double sc = m.vol[b] / volume;
    s[1] += sc * sc * rnorm2[b];
  }
  for (int k = 0; k < 3; ++k) s[k] = wave_sum(s[k]);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < 3; ++k) red[k][wid] = s[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[3] = {0.0, 0.0, 0.0};
    for (int w = 0; w < static_cast<int>(blockDim.x + 63) / 64; ++w)
      for (int k = 0; k < 3; ++k) t[k] += red[k][w];
    out[0] = sqrt(t[0] + t[1]);
    out[1] = sqrt(t[0]);
    out[2] = sqrt(t[1]);
    out[3] = sqrt(t[2]);
  }
}

}  // namespace fe2
