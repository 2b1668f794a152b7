// Kernels of the RVE-response surrogate (finite strain, 2D); see surrogate.hip.
#pragma once

#include "fe2_internal.hpp"

namespace fe2 {

// norm layout (doubles): in_lo[4] | in_hi[4] | out_mean[9] | out_std[9]
constexpr int SURR_NIN = 4, SURR_NOUT = 9, SURR_NORM = 26;

__global__ void k_phase_fraction(int n_rve, const int64_t* off, const uint8_t* phase, double* phi);
__global__ void k_surr_features(int n, const double* F, const double* phi, const double* norm, int* banned,
                                float* X, int* accept);
__global__ void k_surr_decode(int n, const float* Y, const double* norm, const double* F, const int* accept,
                              double* Pbar, double* Phat, double* Cbar, double* rnorm2, double* surrP, double* surrC);
__global__ void k_surr_targets(int n, const double* F, const double* P, const double* A, const double* phi, double* X,
                               double* T);
__global__ void k_col_stats(int n, int m, const double* V, const double* ok, double* out);
__global__ void k_normalize(int n, int m, const double* V, const double* a, const double* bb, int mode, float* out);
__global__ void k_surr_compare(int n, const int* accept, const double* surrP, const double* surrC, const double* Pbar,
                               const double* Cbar, double tol, double* err, int* banned, int* n_rejected);
__global__ void k_zero_w_masked(const int64_t* foff, const int* mask, double* w);
__global__ void k_ok_flags(int n, const double* rnorm2, const double* thr2, const double* relres, double tol,
                           double* ok);

}  // namespace fe2
