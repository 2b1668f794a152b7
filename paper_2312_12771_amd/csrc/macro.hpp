// Macro-side kernels of libfe2 (FP64): geometry, gradients, assembly,
// band assembly, update and norms.
#pragma once

#include "elem2d.hpp"
#include "fe2_internal.hpp"

namespace fe2 {

struct MacroArgs {
  int n_rve, dim, nen, n_gp, nF, kin, n_elems, ndof, bw;
  int basis;              // FE2_BASIS_DIRAC or FE2_BASIS_ELEMENT
  int order;              // macro element order: 1 (Q4 / hex8), 2 (Q9)
  int n_qp;               // macro Gauss points, n_elems * n_gp
  const int* conn;        // [n_elems][nen]
  const double* X;        // [n_nodes][dim]
  double* dNdX;           // [n_qp][nen][dim]
  double* wdet;           // [n_qp]
  double* vol;            // [n_rve] weight of the RVE's micro residual rows
  const double* kpar;     // [n_rve][2][2] (lambda, mu) per phase (small strain)
  const double* phi;      // [n_rve] phase-1 volume fraction
  const double* f_ext;    // [ndof] or null
  const int* is_dir;      // [ndof]
  const double* dir_full; // [ndof] prescribed value at load factor 1 (0 on free DOFs)
  const int* vec_ptr;     // [ndof+1] row -> element-vector entries
  const int* vec_src;     //          index e*nd + a
  const int* nz_ptr;      // [ndof+1] row -> nonzero columns
  const int* nz_col;
  const int* nzc_ptr;     // [nnz+1] nonzero -> element-matrix entries
  const int* nzc_src;     //          index (e*nd + a)*nd + c
};

__global__ void k_ref_tables_2d(double h1, double h2, double rho, double* out);
constexpr int REF2_TABLE = 54;    // kv[10] | KwF[8*3] | KFF[9] | error | mode constants[10]
__global__ void k_ref_tables_3d(double h, double rho, double* out);
constexpr int REF3_TABLE = 191;   // kv[10] | KwF[24*6] | KFF[36] | error
__global__ void k_macro_geometry(MacroArgs m);
__global__ void k_rve_weight(MacroArgs m);
__global__ void k_macro_grad(MacroArgs m, const double* __restrict__ u, double* __restrict__ out);
__global__ void k_macro_elem_vec(MacroArgs m, const double* __restrict__ P, double* __restrict__ f,
                                 const double* __restrict__ u);
__global__ void k_macro_elem_mat(MacroArgs m, const double* __restrict__ Cb, double* __restrict__ ke);
// the element matrices (a7): a sized kernel for the element types in use,
// the general one otherwise
void launch_macro_elem_mat(const MacroArgs& m, const double* Cb, double* ke, hipStream_t s);
__global__ void k_macro_rows_vec(MacroArgs m, const double* __restrict__ f_true,
                                 const double* __restrict__ f_hat, double lam,
                                 double* __restrict__ r_true, double* __restrict__ f_int,
                                 double* __restrict__ rhs);
__global__ void k_macro_rows_band(MacroArgs m, const double* __restrict__ ke, double dlam,
                                  double* __restrict__ band, double* __restrict__ rhs,
                                  double* __restrict__ kdense);
__global__ void k_fill(double* p, size_t n, double v);
__global__ void k_fill_i(int* p, size_t n, int v);
// Block cyclic reduction solve of a banded SPD system (bcr.hip).
struct BcrPlan {
  int n = 0, bw = 0, bs = 0, nb = 0;
  size_t d_len = 0, g_len = 0, inv_len = 0, f_len = 0;
};
BcrPlan bcr_plan(int n, int bw);
size_t bcr_workspace_doubles(const BcrPlan& p);
int bcr_max_bandwidth();
// band: lower band storage [n][bw+1] (read only); y: right-hand side in,
// solution out; info: 0 on entry, set to a 1-based pivot index when the
// matrix is not positive definite; ws: bcr_workspace_doubles(p) doubles.
int bcr_solve(const BcrPlan& p, double* ws, const double* band, double* y, int* info, hipStream_t s);
__global__ void k_axpy(int n, const double* __restrict__ x, double* __restrict__ y);
// a9 update of the RVE fields (one work-group per RVE); -1 for an nF or
// element beyond the kernel's shared product table
constexpr int kUpdateMaxProducts = 256;
int launch_update_w(const MacroArgs& m, int n_rve, const double* du, const int64_t* foff, const double* X,
                    double* w, int use_xr, const int* skip, hipStream_t s);
__global__ void k_micro_thr(int n_rve, const double* __restrict__ rnorm2, const double* __restrict__ rsize2, double tol,
                            double* __restrict__ thr2);
__global__ void k_count_above(int n_rve, const double* __restrict__ rnorm2,
                              const double* __restrict__ thr2, const int* __restrict__ skip,
                              int* __restrict__ count);
__global__ void k_sub_xr(int nF, const int64_t* __restrict__ foff, const double* __restrict__ X,
                         const int* __restrict__ skip, double* __restrict__ w);
__global__ void k_mark_dead(int n_rve, const double* __restrict__ relres, double tol, int* __restrict__ dead,
                            int* __restrict__ count);
__global__ void k_copy_mask(int n, const int* __restrict__ src, int* __restrict__ dst);
__global__ void k_norms(MacroArgs m, const double* __restrict__ r_true,
                        const double* __restrict__ f_int, const double* __restrict__ rnorm2,
                        double volume, double* __restrict__ out);

}  // namespace fe2
