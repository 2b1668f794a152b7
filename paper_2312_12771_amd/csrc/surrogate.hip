// Kernels of the RVE-response surrogate (finite strain, 2D): features,
// training targets, normalisation, decoding of network outputs into the
// homogenized stress and tangent, and the comparison with full RVE solves.
//
// Representation (frame-indifferent, so one network serves every rotation):
//   input  x = (E11, E22, E12, phi): Green-Lagrange strain E = (F^T F - I)/2
//          of the macro gradient and the inclusion volume fraction phi;
//   output y = (S11, S22, S12, D11, D22, D33, D12, D13, D23): second
//          Piola-Kirchhoff stress S and the symmetric Voigt matrix D of
//          dS/dE (S_v = D E_v with E_v = (E11, E22, 2 E12)).
// The macro quantities follow from P = F S and
//   A_iJkL = dP_iJ/dF_kL = delta_ik S_LJ + F_iM F_kN C_MJNL,
// C_MJNL = D[v(MJ)][v(NL)], v(11) = 0, v(22) = 1, v(12) = v(21) = 2.
#include "surrogate.hpp"

namespace fe2 {
namespace {

__device__ __forceinline__ int voigt(int a, int b) { return a == b ? a : 2; }

__device__ void features(const double* F, double phi, double x[4]) {
  // F row-major (F11, F12, F21, F22): (F^T F)_11 = F11^2 + F21^2, ...
  x[0] = 0.5 * (F[0] * F[0] + F[2] * F[2] - 1.0);
  x[1] = 0.5 * (F[1] * F[1] + F[3] * F[3] - 1.0);
  x[2] = 0.5 * (F[0] * F[1] + F[2] * F[3]);
  x[3] = phi;
}

// (S, D) -> P (4) and A (4x4, row (i,J) = 2i+J, column (k,L) = 2k+L)
__device__ void macro_from_sd(const double* F, const double S2[2][2], const double D[3][3], double P[4],
                              double A[16]) {
  for (int i = 0; i < 2; ++i)
    for (int J = 0; J < 2; ++J) P[2 * i + J] = F[2 * i] * S2[0][J] + F[2 * i + 1] * S2[1][J];
  for (int i = 0; i < 2; ++i)
    for (int J = 0; J < 2; ++J)
      for (int k = 0; k < 2; ++k)
        for (int L = 0; L < 2; ++L) {
          double v = (i == k) ? S2[L][J] : 0.0;
          for (int M = 0; M < 2; ++M)
            for (int N = 0; N < 2; ++N) v += F[2 * i + M] * F[2 * k + N] * D[voigt(M, J)][voigt(N, L)];
          A[(2 * i + J) * 4 + 2 * k + L] = v;
        }
}

}  // namespace

__global__ void k_phase_fraction(int n_rve, const int64_t* __restrict__ off, const uint8_t* __restrict__ phase,
                                 double* __restrict__ phi) {
  __shared__ int part[4];
  const int b = blockIdx.x;
  const int64_t o0 = off[b], o1 = off[b + 1];
  int c = 0;
  for (int64_t e = o0 + threadIdx.x; e < o1; e += blockDim.x) c += phase[e];
  for (int s = 32; s > 0; s >>= 1) c += __shfl_xor(c, s, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) phi[b] = static_cast<double>(part[0] + part[1] + part[2] + part[3]) / (o1 - o0);
}

// Network inputs of every point; a point is accepted while its features lie
// inside the training range.  A point that leaves the range is banned for
// the rest of the attachment (it stays on the RVE path), so that points at
// the edge of the range cannot switch between the network and the RVE
// solve from one Newton iteration to the next (a discontinuous residual).
__global__ void k_surr_features(int n, const double* __restrict__ F, const double* __restrict__ phi,
                                const double* __restrict__ norm, int* __restrict__ banned,
                                float* __restrict__ X, int* __restrict__ accept) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  double x[4];
  features(F + 4 * static_cast<size_t>(b), phi[b], x);
  bool range = true;
  for (int c = 0; c < 4; ++c) {
    const double lo = norm[c], hi = norm[4 + c];
    range = range && x[c] >= lo && x[c] <= hi;
    X[4 * static_cast<size_t>(b) + c] = static_cast<float>(2.0 * (x[c] - lo) / (hi - lo) - 1.0);
  }
  if (!range && banned) banned[b] = 1;
  accept[b] = (range && !(banned && banned[b])) ? 1 : 0;
}

__global__ void k_surr_decode(int n, const float* __restrict__ Y, const double* __restrict__ norm,
                              const double* __restrict__ F, const int* __restrict__ accept,
                              double* __restrict__ Pbar, double* __restrict__ Phat, double* __restrict__ Cbar,
                              double* __restrict__ rnorm2, double* __restrict__ surrP, double* __restrict__ surrC) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const double* mean = norm + 8;
  const double* sd = norm + 17;
  double y[9];
  for (int o = 0; o < 9; ++o) y[o] = mean[o] + sd[o] * static_cast<double>(Y[9 * static_cast<size_t>(b) + o]);
  const double S2[2][2] = {{y[0], y[2]}, {y[2], y[1]}};
  const double D[3][3] = {{y[3], y[6], y[7]}, {y[6], y[4], y[8]}, {y[7], y[8], y[5]}};
  double P[4], A[16];
  macro_from_sd(F + 4 * static_cast<size_t>(b), S2, D, P, A);
  for (int t = 0; t < 4; ++t) surrP[4 * static_cast<size_t>(b) + t] = P[t];
  for (int t = 0; t < 16; ++t) surrC[16 * static_cast<size_t>(b) + t] = A[t];
  if (!accept[b]) return;
  for (int t = 0; t < 4; ++t) {
    Pbar[4 * static_cast<size_t>(b) + t] = P[t];
    Phat[4 * static_cast<size_t>(b) + t] = P[t];
  }
  for (int t = 0; t < 16; ++t) Cbar[16 * static_cast<size_t>(b) + t] = A[t];
  rnorm2[b] = 0.0;
}

// Training pairs from RVE responses: x = features, t = (S, D) with
// S = F^-1 P and C_MJNL = F^-1_Mi F^-1_Nk (A_iJkL - delta_ik S_LJ),
// D averaged over the minor-symmetric entries.
__global__ void k_surr_targets(int n, const double* __restrict__ F, const double* __restrict__ P,
                               const double* __restrict__ A, const double* __restrict__ phi, double* __restrict__ X,
                               double* __restrict__ T) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const double* f = F + 4 * static_cast<size_t>(b);
  const double* p = P + 4 * static_cast<size_t>(b);
  const double* a = A + 16 * static_cast<size_t>(b);
  double x[4];
  features(f, phi[b], x);
  for (int c = 0; c < 4; ++c) X[4 * static_cast<size_t>(b) + c] = x[c];
  const double J = f[0] * f[3] - f[1] * f[2];
  const double Fi[2][2] = {{f[3] / J, -f[1] / J}, {-f[2] / J, f[0] / J}};
  double S[2][2];
  for (int M = 0; M < 2; ++M)
    for (int Jj = 0; Jj < 2; ++Jj) S[M][Jj] = Fi[M][0] * p[Jj] + Fi[M][1] * p[2 + Jj];
  double C[2][2][2][2];
  for (int M = 0; M < 2; ++M)
    for (int Jj = 0; Jj < 2; ++Jj)
      for (int N = 0; N < 2; ++N)
        for (int L = 0; L < 2; ++L) {
          double v = 0.0;
          for (int i = 0; i < 2; ++i)
            for (int k = 0; k < 2; ++k) {
              const double g = a[(2 * i + Jj) * 4 + 2 * k + L] - ((i == k) ? S[L][Jj] : 0.0);
              v += Fi[M][i] * Fi[N][k] * g;
            }
          C[M][Jj][N][L] = v;
        }
  auto Dv = [&](int r, int c) {   // average of the entries mapped to Voigt (r, c)
    const int rm[3][2] = {{0, 0}, {1, 1}, {0, 1}};
    double s = 0.0;
    int cnt = 0;
    for (int sr = 0; sr < (r == 2 ? 2 : 1); ++sr)
      for (int sc = 0; sc < (c == 2 ? 2 : 1); ++sc) {
        const int M = sr ? rm[r][1] : rm[r][0], Jj = sr ? rm[r][0] : rm[r][1];
        const int N = sc ? rm[c][1] : rm[c][0], L = sc ? rm[c][0] : rm[c][1];
        s += 0.5 * (C[M][Jj][N][L] + C[N][L][M][Jj]);
        ++cnt;
      }
    return s / cnt;
  };
  double* t = T + 9 * static_cast<size_t>(b);
  t[0] = S[0][0];
  t[1] = S[1][1];
  t[2] = 0.5 * (S[0][1] + S[1][0]);
  t[3] = Dv(0, 0);
  t[4] = Dv(1, 1);
  t[5] = Dv(2, 2);
  t[6] = Dv(0, 1);
  t[7] = Dv(0, 2);
  t[8] = Dv(1, 2);
}

// Per-column statistics over the rows with ok[row] != 0 (one block per
// column, fixed reduction order): out = [min | max | mean | std] of m columns.
__global__ void __launch_bounds__(256) k_col_stats(int n, int m, const double* __restrict__ V,
                                                   const double* __restrict__ ok, double* __restrict__ out) {
  __shared__ double smn[4], smx[4], ss[4], sq[4], sc[4];
  const int c = blockIdx.x;
  double mn = 1e300, mx = -1e300, s = 0.0, q = 0.0, cnt = 0.0;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    if (ok && !(ok[r] != 0.0)) continue;
    const double v = V[static_cast<size_t>(r) * m + c];
    mn = fmin(mn, v);
    mx = fmax(mx, v);
    s += v;
    q += v * v;
    cnt += 1.0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    mx = fmax(mx, __shfl_xor(mx, o, 64));
    s += __shfl_xor(s, o, 64);
    q += __shfl_xor(q, o, 64);
    cnt += __shfl_xor(cnt, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    smn[w] = mn;
    smx[w] = mx;
    ss[w] = s;
    sq[w] = q;
    sc[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      smn[0] = fmin(smn[0], smn[k]);
      smx[0] = fmax(smx[0], smx[k]);
      ss[0] += ss[k];
      sq[0] += sq[k];
      sc[0] += sc[k];
    }
    const double mean = sc[0] > 0.0 ? ss[0] / sc[0] : 0.0;
    const double var = sc[0] > 0.0 ? fmax(sq[0] / sc[0] - mean * mean, 0.0) : 0.0;
    out[c] = smn[0];
    out[m + c] = smx[0];
    out[2 * m + c] = mean;
    out[3 * m + c] = sqrt(var);
  }
}

// out = (V - shift) / scale (mode 0) or 2 (V - lo) / (hi - lo) - 1 (mode 1),
// as float
__global__ void k_normalize(int n, int m, const double* __restrict__ V, const double* __restrict__ a,
                            const double* __restrict__ bb, int mode, float* __restrict__ out) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<size_t>(n) * m) return;
  const int c = static_cast<int>(i % m);
  const double v = V[i];
  out[i] = static_cast<float>(mode == 0 ? (v - a[c]) / bb[c] : 2.0 * (v - a[c]) / (bb[c] - a[c]) - 1.0);
}

// error of the surrogate against full RVE results for the accepted points
__global__ void k_surr_compare(int n, const int* __restrict__ accept, const double* __restrict__ surrP,
                               const double* __restrict__ surrC, const double* __restrict__ Pbar,
                               const double* __restrict__ Cbar, double tol, double* __restrict__ err,
                               int* __restrict__ banned, int* __restrict__ n_rejected) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  if (!accept[b]) {
    err[b] = 0.0;
    return;
  }
  double dp = 0.0, np = 0.0, dc = 0.0, nc = 0.0;
  for (int t = 0; t < 4; ++t) {
    const double r = Pbar[4 * static_cast<size_t>(b) + t];
    dp += (surrP[4 * static_cast<size_t>(b) + t] - r) * (surrP[4 * static_cast<size_t>(b) + t] - r);
    np += r * r;
  }
  for (int t = 0; t < 16; ++t) {
    const double r = Cbar[16 * static_cast<size_t>(b) + t];
    dc += (surrC[16 * static_cast<size_t>(b) + t] - r) * (surrC[16 * static_cast<size_t>(b) + t] - r);
    nc += r * r;
  }
  // stress error relative to the tangent scale times the strain (the stress
  // vanishes at F = I), tangent error relative to the tangent
  const double e = fmax(sqrt(dp) / fmax(sqrt(np), 1e-3 * sqrt(nc)), sqrt(dc) / sqrt(nc));
  err[b] = e;
  if (!(e <= tol)) {
    banned[b] = 1;
    atomicAdd(n_rejected, 1);
  }
}

__global__ void k_zero_w_masked(const int64_t* __restrict__ foff, const int* __restrict__ mask, double* __restrict__ w) {
  const int b = blockIdx.x;
  if (!mask[b]) return;
  for (int64_t t = foff[b] + threadIdx.x; t < foff[b + 1]; t += blockDim.x) w[t] = 0.0;
}

__global__ void k_ok_flags(int n, const double* __restrict__ rnorm2, const double* __restrict__ thr2,
                           const double* __restrict__ relres, double tol, double* __restrict__ ok) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  ok[b] = (rnorm2[b] <= thr2[b] && relres[b] <= tol) ? 1.0 : 0.0;
}

}  // namespace fe2
