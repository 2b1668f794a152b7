// Internal declarations shared by the HIP translation units of libfe2.
// Device code targets gfx950 (CDNA4, 64-wide wavefronts) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/fe2.h"

namespace fe2 {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);

#define FE2_HIP_CHECK(expr)                                                    \
  do {                                                                         \
    hipError_t _e = (expr);                                                    \
    if (_e != hipSuccess) {                                                    \
      ::fe2::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));      \
      return FE2_EHIP;                                                         \
    }                                                                          \
  } while (0)

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap_idx(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum NV values over the work-group; every thread receives the totals.
// s_red must hold NW*NV doubles.  Deterministic: fixed order of the
// butterfly within a wave and of the waves.
template <int NV, int NW>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* s_red) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) s_red[wid * NV + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += s_red[w * NV + i];
    v[i] = t;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// kernel arguments
// ---------------------------------------------------------------------------
enum RveFlags : int {
  RVE_ASSEMBLE = 1,   // element integration: r_b, int P~ (a3)
  RVE_SOLVE = 2,      // PCG + refinement + condensation (a5, a6)
  RVE_WARM = 4,       // start from the solution stored in X
  RVE_RCOL = 8,       // solve the residual column (nF+1 right-hand sides)
  RVE_FFT = 16,       // homogeneous-reference (FFT) preconditioner
  RVE_RONLY = 32,     // solve the residual column only (x_r), no condensation;
                      // RVEs with rnorm2 <= thr2 are skipped (x_r = 0)
  RVE_MC = 64,        // spectral: the columns of X_F in one PCG loop where a
                      // kernel for the size exists (else one after another)
  RVE_DENSE = 128     // dense FP32 Cholesky on the matrix cores + FP64 refinement
};

// One launch handles the RVEs of one resolution class (same n1 x n2 and same
// lambda/mu ratio, hence the same reference element tables).
struct Lin2DArgs {
  int n1, n2;
  const int* rve_list;          // RVE ids of this launch
  const int64_t* phase_off;     // [n_rve+1]
  const uint8_t* phase;         // phase id per RVE element
  const double* params;         // [n_rve][2][2] (lambda, mu)
  const double* kv64;           // [10] distinct entries of the element stiffness, mu = 1
  const double* KwF64;          // [8*3] element coupling, mu = 1
  const double* KFF64;          // [9] element integral of C, mu = 1
  const double* modes64;        // [10] mode constants of the element stiffness, mu = 1
  const double* macro;          // [n_rve][3] macro strain
  const int64_t* foff;          // [n_rve+1] field offsets (doubles)
  const double* w;              // state fluctuation (periodic numbering)
  double* r;                    // RVE residual (written by ASSEMBLE)
  double* X;                    // solutions, (nF+1) fields per RVE
  double* Cbar;                 // [n_rve][3][3]
  double* Phat;                 // [n_rve][3]
  double* Pbar;                 // [n_rve][3]
  double* rnorm2;               // [n_rve] ||r_b||^2
  double* relres;               // [n_rve] final relative FP64 residual
  double* iters;                // [n_rve] inner PCG iterations (all columns)
  double* mv64;                 // [n_rve] FP64 operator applications
  int* fail_count;              // RVEs that missed tol
  const double* thr2;           // [n_rve] RVE_RONLY: skip RVEs with rnorm2 <= thr2
  const int* skip;              // [n_rve] or null: RVEs with skip[b] != 0 are left untouched
  const float* fft_tab;         // spectral preconditioner table, FP32 (RVE_FFT)
  const double* fft_tab64;      // the same table in FP64
  double volume;
  double tol, tol_in;
  int max_it, max_ir;
  int flags;
};

// Finite-strain 2D RVEs (plane strain, polyconvex phases).  One launch
// handles the RVEs of one resolution.
struct Fin2DArgs {
  int n1, n2;
  const int* rve_list;          // RVE ids of this launch
  const int64_t* phase_off;     // [n_rve+1]
  const uint8_t* phase;         // phase id per RVE element
  const double* params;         // [n_rve][2][3] (alpha, beta, kappa)
  const double* macro;          // [n_rve][4] macro gradient F_b, row-major
  const int64_t* foff;          // [n_rve+1] field offsets (doubles)
  const double* w;              // state fluctuation (periodic numbering)
  double* r;                    // RVE residual (written by ASSEMBLE)
  double* X;                    // solutions, (nF+1) fields per RVE
  double* Cbar;                 // [n_rve][4][4]
  double* Phat;                 // [n_rve][4]
  double* Pbar;                 // [n_rve][4]
  double* rnorm2;               // [n_rve] ||r_b||^2
  double* rsize2;               // [n_rve] squared size of the element-level terms of r_b (or null)
  double* relres;               // [n_rve] final relative FP64 residual
  double* iters;                // [n_rve] inner PCG iterations (all columns)
  double* mv64;                 // [n_rve] FP64 operator applications
  int* fail_count;              // RVEs that missed tol (or lost J > 0)
  const double* thr2;           // [n_rve] RVE_RONLY: skip RVEs with rnorm2 <= thr2
  const int* skip;              // [n_rve] or null: RVEs with skip[b] != 0 are left untouched
  const float* fft_tab;         // spectral preconditioner table, FP32 (RVE_FFT)
  const double* fft_tab64;      // the same table in FP64
  double h1, h2;                // element edge lengths
  double volume;
  double tol, tol_in;
  int max_it, max_ir;
  int flags;
};

// Surrogate network (mlp.hip): input (which = 0) or output width, batch cap
int mlp_width(fe2_mlp q, int which);
int mlp_max_batch(fe2_mlp q);

// Launchers (rve_lin2d.hip, rve_fin2d.hip)
// Square RVEs of 8, 16, 32 or 48 elements (finite strain: 8, 16, 32) run the
// PCG with the spectral preconditioner of a homogeneous reference medium
// when RVE_FFT is set;
// lin2d_spectral_table writes its table (alpha, Re beta, Im beta, 0 per
// position, then the twiddles e^{-2 pi i t / n}, t < lin2d_spectral_twiddles)
// for lambda/mu = rho: 4 n^2 + 2 lin2d_spectral_twiddles(n) doubles.
constexpr bool lin2d_spectral_size(int n1, int n2) {
  return n1 == n2 && (n1 == 8 || n1 == 16 || n1 == 32 || n1 == 48);
}
constexpr int lin2d_spectral_twiddles(int n) { return n == 48 ? 32 : n / 2; }
void lin2d_spectral_table(int n, double rho, double* out);
constexpr bool fin2d_spectral_size(int n1, int n2) { return n1 == n2 && (n1 == 8 || n1 == 16 || n1 == 32); }
// Dense direct RVE solve (2D small strain): RVEs whose reduced stiffness
// (2 n1 n2 - 2 unknowns, rounded up to 16) fits an LDS-resident FP32 factor
constexpr bool lin2d_dense_size(int n1, int n2) { return n1 >= 3 && n2 >= 3 && 2 * n1 * n2 - 2 <= 128; }
int launch_lin2d(const Lin2DArgs& a, int n_launch, int precision, int nrhs,
                 hipStream_t s);
bool lin2d_supported(int n1, int n2);
int launch_fin2d(const Fin2DArgs& a, int n_launch, int precision, int nrhs,
                 hipStream_t s);
// 3D small strain (rve_lin3d.hip): cubes n x n x n, reuses Lin2DArgs with
// n1 = n, KwF64 = [24][6], KFF64 = [6][6]
int launch_lin3d(const Lin2DArgs& a, int n_launch, int precision, int nrhs,
                 hipStream_t s);
bool lin3d_supported(int n1, int n2, int n3);
bool fin2d_supported(int n1, int n2);

}  // namespace fe2
