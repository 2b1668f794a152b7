/*
 * fe2.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot path
 * of the monolithic FE^2 scheme of Hesch, Schmidt and Schuss, "Variational
 * formulation and monolithic solution of computational homogenization
 * methods" (arXiv:2312.12771).  Equation numbers follow the paper.
 *
 * For every macroscopic Gauss point b the library assembles the RVE attached
 * to b (Sec. 3, Eqs. (34)-(35)), reduces it with the periodic null space
 * (condition (iii) of Eq. (15)), solves the RVE system and condenses it to the
 * homogenized stress and tangent that enter the macro Newton step of the
 * generalized null-space scheme (Sec. 4.2, Eqs. (46)-(49)); the macro tangent
 * is then assembled and solved in FP64 and the fluctuations are updated.
 *
 * Conventions (all entry points)
 *   - Host arrays passed to fe2_setup are read during the call and copied;
 *     the caller keeps ownership.
 *   - Pointers named *_dev are device (HBM) pointers owned by the caller,
 *     contiguous float64 unless stated otherwise.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work on that stream and return without waiting, except
 *     where a host scalar is returned (fe2_newton_step waits for its norms).
 *   - Return values: FE2_OK (0) or FE2_CONVERGED (1) on success, a negative
 *     fe2_status on failure.  No exception crosses the ABI.  A failed call
 *     leaves the handle usable unless it returns FE2_ESTATE.  fe2_last_error()
 *     gives a human-readable reason for the last failure of this thread.
 *   - A handle is not thread-safe; use one handle per host thread.
 *
 * Numbering
 *   - Macro DOFs are node-major: dof = node*dim + component.
 *   - RVE b = element * 2^dim + g, Gauss points xi fastest (2 per direction);
 *     with FE2_BASIS_ELEMENT, RVE b = element.
 *   - RVE fields use the periodic node numbering of an n1 x n2 (x n3) grid,
 *     node (i,j,k) -> i + n1*(j + n2*k), DOF = node*dim + component; the
 *     corner node 0 carries the pinned fluctuation (always 0 in outputs).
 *     fe2_query(FE2_Q_FIELD_LEN) gives the total length over all RVEs and
 *     FE2_Q_FIELD_OFFSETS the per-RVE offsets (in units of doubles).
 *   - Macro kinematic components nF: small strain Voigt [11,22,12] (2D,
 *     engineering shear) or [11,22,33,23,13,12] (3D); finite strain the
 *     row-major deformation gradient [F11,F12,F21,F22].
 */
#ifndef FE2_H
#define FE2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FE2_ABI_VERSION 4

typedef enum fe2_status {
  FE2_OK = 0,
  FE2_CONVERGED = 1,   /* fe2_newton_step: residual below tolerance, no update made */
  FE2_EINVAL = -1,     /* invalid argument or descriptor */
  FE2_ENOMEM = -2,     /* device or host allocation failed */
  FE2_EHIP = -3,       /* a HIP runtime call failed */
  FE2_ENOCONV = -4,    /* an RVE solve missed its tolerance (see FE2_Q_FAILED_RVES) */
  FE2_ESTATE = -5,     /* handle unusable (earlier fatal error) */
  FE2_ENOTSUP = -6     /* combination not implemented */
} fe2_status;

enum { FE2_SMALL_STRAIN = 0, FE2_FINITE_STRAIN = 1 };
enum { FE2_LINEAR_ISO = 0, FE2_NEO_HOOKE = 1, FE2_MOONEY_RIVLIN = 2 };
enum { FE2_PREC_FP64 = 0, FE2_PREC_FP32_IR = 1, FE2_PREC_BF16_IR = 2 };
enum {
  FE2_SOLVER_AUTO = 0,
  FE2_SOLVER_PCG_JACOBI = 1,
  FE2_SOLVER_PCG_FFT = 2,
  FE2_SOLVER_DENSE = 3,
  FE2_SOLVER_PCG_FFT_MC = 4
};
enum { FE2_SCHEME_GENERALIZED = 0, FE2_SCHEME_CLASSICAL = 1, FE2_SCHEME_CLASSICAL_PLAIN = 2 };
/* Macro basis of the fluctuation: FE2_BASIS_DIRAC puts one RVE at every macro
 * Gauss point (Dirac approach, Eqs. (31)-(35)); FE2_BASIS_ELEMENT gives every
 * macro element one fluctuation field shared by its Gauss points (the
 * piecewise-constant approximation of Eqs. (constSolution1)-(constSolution2),
 * discontinuous across elements). */
enum { FE2_BASIS_DIRAC = 0, FE2_BASIS_ELEMENT = 1 };

/*
 * Problem description (Sec. 2 and Sec. 5.2 problem statement: macro body,
 * boundary data and loads, RVE with its phases and micro boundary condition,
 * discretisation, tolerances).
 *
 *  struct_size      sizeof(fe2_problem_desc) (ABI check)
 *  dim              2 (Q4, plane strain) or 3 (hex8)
 *  kinematics       FE2_SMALL_STRAIN or FE2_FINITE_STRAIN (2D only)
 *  material         FE2_LINEAR_ISO (small strain), FE2_NEO_HOOKE or
 *                   FE2_MOONEY_RIVLIN (finite strain)
 *  n_nodes, X       macro node coordinates [n_nodes][dim]
 *  n_elems, conn    macro connectivity [n_elems][nen]: nen = 2^dim for
 *                   macro_order 1 (Q4 counter-clockwise; hex8 bottom face then
 *                   top face), nen = 9 for macro_order 2 (Q9: corners
 *                   counter-clockwise, then the mid-side nodes of the bottom,
 *                   right, top and left edges, then the centre node)
 *  n_dir, dir_dofs, dir_vals   prescribed DOFs (strictly increasing) and their
 *                   values at load factor 1
 *  f_ext            external nodal forces at load factor 1 [n_nodes*dim] or NULL
 *  n_rve            number of RVEs: n_elems * (macro_order + 1)^dim
 *                   (FE2_BASIS_DIRAC, one per Gauss point, xi fastest) or
 *                   n_elems (FE2_BASIS_ELEMENT)
 *  rve_res          RVE resolutions [n_rve][dim], every entry >= 2
 *  rve_off          offsets into phase_id [n_rve+1]
 *  phase_id         phase (0 or 1) of every RVE element, lexicographic
 *  n_phase_params   parameters per phase: 2 (lambda, mu) for FE2_LINEAR_ISO
 *                   and FE2_NEO_HOOKE, 3 (alpha, beta, kappa) for
 *                   FE2_MOONEY_RIVLIN (the law of Eq. (59))
 *  phase_params     [n_rve][2][n_phase_params]; for FE2_LINEAR_ISO both
 *                   phases of an RVE must have the same lambda/mu (the
 *                   element stiffness is mu_e times one reference matrix of
 *                   that ratio), else FE2_ENOTSUP
 *  rve_size         side length of the cubic RVE cell (|Omega| = rve_size^dim)
 *  precision        FE2_PREC_FP64 (plain FP64 RVE solves) or FE2_PREC_FP32_IR
 *                   (FP32 PCG with FP64 residual refinement).
 *                   FE2_PREC_BF16_IR is declared and refused (FE2_ENOTSUP):
 *                   refinement around a solve with unit roundoff u contracts
 *                   only while cond(K_ww) * u < 1, and the RVE stiffnesses of
 *                   the paper's configurations have cond(K_ww) far above
 *                   1/u = 256 of bfloat16
 *  solver           preconditioner of the RVE PCG (2D small strain):
 *                   FE2_SOLVER_PCG_JACOBI (diagonal), FE2_SOLVER_PCG_FFT
 *                   (inverse of the periodic operator of a homogeneous
 *                   reference medium, applied by FFT in LDS; square RVEs of
 *                   8, 16, 32 or 48 elements only, else FE2_ENOTSUP; 48 runs
 *                   a radix-3 x 3 stage ahead of radix-2 x 2 stages) or
 *                   FE2_SOLVER_AUTO (FFT where the size allows it, Jacobi
 *                   otherwise), FFT and AUTO solving the columns one after
 *                   another; FE2_SOLVER_PCG_FFT_MC is the same preconditioner
 *                   with the three columns of X_F in one PCG loop (FP32_IR,
 *                   16 x 16 and 32 x 32 RVEs, three right-hand sides; other
 *                   cases fall back to one column at a time).  Finite
 *                   strain (2D) takes FFT on square RVEs of 8, 16 or 32
 *                   elements (reference medium: the small-strain limit of
 *                   the stiffer phase); 3D uses Jacobi, FFT there gives
 *                   FE2_ENOTSUP.  FE2_SOLVER_DENSE replaces the PCG by a
 *                   direct solve: K_ww assembled densely in LDS, factored
 *                   once per RVE by an FP32 Cholesky on the matrix cores and
 *                   applied inside the FP64 refinement (2D small strain,
 *                   FE2_PREC_FP32_IR, RVEs with 2 n1 n2 - 2 <= 128 unknowns
 *                   and n1, n2 >= 3; else FE2_ENOTSUP)
 *  scheme           FE2_SCHEME_GENERALIZED (Sec. 4.2) or _CLASSICAL (Sec. 4.1:
 *                   every RVE equilibrated at the current macro state, the
 *                   macro step on the condensed tangent, the fluctuations
 *                   moved with the macro increment by w -= X_F dF); or
 *                   _CLASSICAL_PLAIN, the same staggered scheme without that
 *                   predictor (the fluctuations carried unchanged into the
 *                   next inner loop)
 *  rve_tol          relative FP64 residual ||b - K x|| / ||b|| every RVE
 *                   solve must reach
 *  inner_tol        floor of the relative tolerance of one FP32 PCG sweep
 *                   (FP32_IR only; a sweep targets max(0.3*rve_tol, inner_tol),
 *                   <= 0 selects 1e-5)
 *  newton_tol       macro convergence: ||[R_macro; R_micro]|| <= newton_tol *
 *                   ||F_int||
 *  micro_tol        classical scheme: inner RVE Newton stops when
 *                   ||r_b|| <= micro_tol * max(1, ||r_b at entry||)
 *  max_pcg_it, max_ir, max_micro_it   iteration caps
 *  macro_basis      FE2_BASIS_DIRAC or FE2_BASIS_ELEMENT (small strain only:
 *                   FE2_ENOTSUP for finite strain)
 *  macro_order      Lagrange order of the macro elements: 1 (Q4 / hex8 with
 *                   2 Gauss points per direction, unit weights) or 2
 *                   (biquadratic Q9 with 3 Gauss points per direction and
 *                   weights 5/9, 8/9, 5/9; the order-2 setting of Sec. 5.1
 *                   carried to 2D).  Order 2 is 2D small strain with the
 *                   Dirac basis; other combinations give FE2_ENOTSUP.
 */
typedef struct fe2_problem_desc {
  int32_t struct_size;
  int32_t dim, kinematics, material;
  int32_t n_nodes;
  const double* X;
  int32_t n_elems;
  const int32_t* conn;
  int32_t n_dir;
  const int32_t* dir_dofs;
  const double* dir_vals;
  const double* f_ext;
  int32_t n_rve;
  const int32_t* rve_res;
  const int64_t* rve_off;
  const uint8_t* phase_id;
  int32_t n_phase_params;
  const double* phase_params;
  double rve_size;
  int32_t precision, solver, scheme;
  double rve_tol, inner_tol, newton_tol, micro_tol;
  int32_t max_pcg_it, max_ir, max_micro_it;
  int32_t macro_basis;
  int32_t macro_order;
} fe2_problem_desc;

typedef struct fe2_ctx* fe2_handle;

/* Build a handle on the current HIP device: copies the description to HBM,
 * builds the reference-element tables, the macro Gauss-point geometry and the
 * RVE work lists on the device (Sec. 3, Eqs. (25)-(29): macro basis and the
 * tensor-product fluctuation numbering), and zeroes the state (q = X, w~ = 0,
 * load factor 0).  Errors: FE2_EINVAL for an inconsistent description,
 * FE2_ENOTSUP for unsupported combinations, FE2_ENOMEM, FE2_EHIP. */
int fe2_setup(const fe2_problem_desc* desc, void* stream, fe2_handle* out);

/* Macro gradient at every Gauss point (Eq. (11): F_b = I + grad u, small
 * strain eps_b = sym grad u; with FE2_BASIS_ELEMENT the RVE of element e is
 * driven by the element average sum_g wdet_g eps_g / V_e, which is exact for
 * its micro residual because that residual is linear in eps) and RVE element
 * integration at the current
 * (q, w~): micro residual r_b (Eq. (35)) in the periodic numbering, the
 * integral of the micro stress (Eq. (17)) and, for finite strain, the micro
 * tangents used by the next solve.  Results stay in the handle
 * (fe2_get_rve_data). */
int fe2_assemble_rve(fe2_handle h, void* stream);

/* Solve K_ww [X_F | x_r] = [K_wF | r_b] for every RVE (the RVE blocks of L in
 * Eq. (42), reduced by the periodic null space) and condense (Eqs. (46)-(48)):
 *   Cbar_b = (K_FF - K_wF^T X_F) / |Omega|,
 *   Phat_b = (int P~ - K_wF^T x_r) / |Omega|.
 * Uses the data of the last fe2_assemble_rve.  Outputs: Cbar_dev
 * [n_rve][nF][nF], Phat_dev [n_rve][nF] (either may be NULL).  Returns
 * FE2_ENOCONV when an RVE missed rve_tol (results are still written). */
int fe2_condense(fe2_handle h, double* Cbar_dev, double* Phat_dev, void* stream);

/* One macro Newton iteration at target load factor `load_factor`
 * (generalized scheme: Eqs. (46)-(49); classical: Eqs. (43)-(45) with the
 * inner RVE equilibration of fe2_equilibrate_rve first).  Steps: macro
 * gradients, RVE integration, residual norms; if the handle's load factor
 * already equals load_factor and the norm satisfies newton_tol the call
 * returns FE2_CONVERGED without an update; otherwise RVE solves and
 * condensation, FP64 macro assembly with the prescribed increment
 * (load_factor - current) * dir_vals, FP64 direct solve of the banded
 * tangent (block cyclic reduction, see fe2_band_solve), update of
 * q and w~ (generalized: dw_b = -(x_r + X_F dF_b); classical predictor:
 * dw_b = -X_F dF_b).
 * norms_host (may be NULL) receives 4 doubles describing the state the call
 * started from: ||[R_macro(free); R_micro]||, ||R_macro(free)||,
 * ||R_micro||, ||F_int|| (R_micro,b = eta_b J_b / |Omega| r_b).  Waits for
 * the norms on `stream`.
 * With FE2_BASIS_ELEMENT (small strain) the Gauss-point stress of element e is
 * sigma_g = Pbar_e + C_V (eps_g - epsbar_e), C_V the volume average of the
 * micro elasticity (the RVE's fluctuation cannot follow the strain variation
 * inside the element), the element tangent is
 *   sum_g wdet_g B_g^T C_V B_g + V_e Bbar^T (Cbar_e - C_V) Bbar,
 * Bbar = sum_g wdet_g B_g / V_e, V_e = sum_g wdet_g, the micro residual
 * weight is V_e / |Omega|, and dw_e = -(x_r + X_F Bbar dq_e). */
int fe2_newton_step(fe2_handle h, double load_factor, double* norms_host, void* stream);

/* Inner RVE equilibration of the classical scheme (Sec. 4.1, the micro
 * Newton loop of Eqs. (43)-(44)) at the current macro displacement: every RVE
 * iterates w~_b <- w~_b - K_ww^-1 r_b until ||r_b|| <= micro_tol *
 * max(1, ||r_b^0||) (r_b^0 = residual at entry), at most max_micro_it
 * updates.  RVEs already in equilibrium are skipped.  iters_host (may be
 * NULL) receives the number of update rounds.  Waits on `stream` once per
 * round.  Returns FE2_ENOCONV when an RVE did not reach micro_tol or an inner
 * solve missed rve_tol; the fluctuations keep the last iterate. */
int fe2_equilibrate_rve(fe2_handle h, int* iters_host, void* stream);

/* Copy the state: u_dev [n_nodes*dim] macro displacement q - X; w_dev
 * [FE2_Q_FIELD_LEN] fluctuations (either may be NULL). */
int fe2_get_state(fe2_handle h, double* u_dev, double* w_dev, void* stream);

/* Overwrite the state (either pointer may be NULL = keep) and set the load
 * factor the prescribed values currently satisfy.  The next RVE solve starts
 * from zero (otherwise solves start from the previous X_F). */
int fe2_set_state(fe2_handle h, const double* u_dev, const double* w_dev,
                  double load_factor, void* stream);

/* Return to the reference state: q - X = 0 and every fluctuation w_b = 0
 * (the undeformed configuration of Sec. 2, where the first generalized
 * Newton iteration starts), at load factor `load_factor`.  The same result
 * as fe2_set_state with zero vectors, written by fill kernels on `stream`
 * (nothing read, nothing allocated, safe to capture in a HIP graph).  The
 * next RVE solve starts from zero. */
int fe2_reset_state(fe2_handle h, double load_factor, void* stream);

/* Intermediate results of the last assembly / condensation / step, copied to
 * caller memory:
 *   FE2_D_MACRO_GRAD  [n_rve][nF]        eps_b or F_b (a2)
 *   FE2_D_RESIDUAL    [FIELD_LEN]        r_b, periodic numbering (a3/a4)
 *   FE2_D_PBAR        [n_rve][nF]        int P~ / |Omega|
 *   FE2_D_SOLUTION    [FIELD_LEN*(nF+1)] per RVE nF+1 consecutive fields:
 *                                        X_F columns then x_r (a5)
 *   FE2_D_RVE_ITERS   [n_rve] (as double) PCG iterations of the last solve
 *                                        (FE2_SOLVER_DENSE: refinement sweeps)
 *   FE2_D_RVE_RELRES  [n_rve]            final relative FP64 residual
 *   FE2_D_MACRO_RHS   [n_nodes*dim]      condensed right-hand side
 *                                        sum G^T Phat - lambda f_ext (a7)
 *   FE2_D_MACRO_RTRUE [n_nodes*dim]      true residual sum G^T Pbar - lambda f_ext
 *   FE2_D_MACRO_DU    [n_nodes*dim]      last macro increment (a8)
 *   FE2_D_MACRO_KDENSE [ndof*ndof]       assembled macro tangent before
 *                                        Dirichlet elimination, dense (only
 *                                        when ndof <= 4096)
 *   FE2_D_CBAR, FE2_D_PHAT               as written by fe2_condense
 *   FE2_D_RVE_MV64    [n_rve] (as double) FP64 operator applications of the
 *                                        last solve (refinement residuals and
 *                                        the condensation pass) */
enum {
  FE2_D_MACRO_GRAD = 0, FE2_D_RESIDUAL = 1, FE2_D_PBAR = 2, FE2_D_SOLUTION = 3,
  FE2_D_RVE_ITERS = 4, FE2_D_RVE_RELRES = 5, FE2_D_MACRO_RHS = 6,
  FE2_D_MACRO_RTRUE = 7, FE2_D_MACRO_DU = 8, FE2_D_MACRO_KDENSE = 9,
  FE2_D_CBAR = 10, FE2_D_PHAT = 11, FE2_D_RVE_MV64 = 12,
  FE2_D_PHASE_FRACTION = 13,   /* [n_rve] volume fraction of phase 1 */
  FE2_D_SURR_ERR = 14          /* [n_rve] last fe2_surrogate_judge error per point */
};
int fe2_get_data(fe2_handle h, int which, double* dst_dev, void* stream);

/* Integer properties of a handle. */
enum {
  FE2_Q_NF = 0, FE2_Q_FIELD_LEN = 1, FE2_Q_NDOF = 2, FE2_Q_BANDWIDTH = 3,
  FE2_Q_FAILED_RVES = 4, FE2_Q_N_RVE = 5, FE2_Q_FIELD_OFFSETS = 6, /* into int64 out[n_rve+1] */
  FE2_Q_MICRO_ITERS = 7,  /* update rounds of the last inner equilibration */
  FE2_Q_SPECTRAL_RVES = 8 /* RVEs whose PCG uses the spectral preconditioner */
};
int fe2_query(fe2_handle h, int which, int64_t* out);

/* Phase timing of fe2_newton_step with HIP events recorded on the caller's
 * stream (tracing aid; off by default).  fe2_set_profiling(h, 1) enables and
 * clears the accumulators.  fe2_get_profile copies and clears 6 doubles:
 * accumulated milliseconds of [a2-a4 + norms, RVE solve and condensation
 * (a5-a6), macro assembly and banded solve (a7-a8), update (a9), whole
 * steps], and the number of timed steps that solved. */
int fe2_set_profiling(fe2_handle h, int enable);
/* Run the RVE solves, the macro assembly and solve and the update of each
 * generalized fe2_newton_step as one HIP graph launch (enable = 1) instead of
 * individual launches (0, the default).  A graph is captured the first time
 * a launch configuration occurs (right-hand sides, warm start, load factor
 * and its increment) and replayed afterwards; at most four are kept per
 * handle.  Results are identical to the individual launches.  With graphs on,
 * fe2_get_profile reports the solve, macro and update phases as one (the
 * solve entry holds their sum; the other two are zero).  The classical
 * scheme and the surrogate always launch individually. */
int fe2_set_graph(fe2_handle h, int enable);
/* Per-class override of the RVE solver, the choice of an autotuner (Sec.
 * 4.1: the RVE blocks of L are independent, so each resolution class may be
 * solved its own way).  Every RVE class of resolution n1 x n2 (x n3 in 3D;
 * n3 is ignored in 2D) runs with `solver` (FE2_SOLVER_*) instead of the
 * handle's: the preconditioner (Jacobi or spectral) and the right-hand sides
 * per PCG pass (FE2_SOLVER_PCG_FFT: one column at a time, _FFT_MC: the three
 * columns of X_F together), or the dense form.  FE2_EINVAL when no class has
 * that resolution or the solver is unknown; FE2_ENOTSUP when the class
 * cannot run it (spectral tables are built at setup only for spectral sizes
 * and solvers AUTO, FFT or FFT_MC; the dense form as in fe2_problem_desc).
 * Cached step graphs are dropped.  Results change only within the solve
 * tolerances. */
int fe2_set_class_solver(fe2_handle h, int n1, int n2, int n3, int solver);
int fe2_get_profile(fe2_handle h, double* out);

/* Release all device memory of the handle (waits for its work). */
int fe2_destroy(fe2_handle h);

/* FP64 direct solve of a symmetric positive definite banded system, the
 * macro linear solve of every Newton update (Eq. (47) for the generalized
 * scheme, Eq. (45) for the classical one).  band_dev: lower band storage,
 * A(i, j) for 0 <= i - j <= bw at band_dev[j * (bw + 1) + (i - j)], n * (bw + 1)
 * doubles, read only (entries with i >= n are ignored).  rhs_dev [n]: the
 * right-hand side on entry, the solution on return.  The matrix is cut into
 * blocks of the bandwidth (rounded up to 16) and solved by block cyclic
 * reduction.  Allocates and frees its own workspace (about 4 bs^2 doubles per
 * block) and waits for `stream`.  pivot_host (may be NULL) receives 0, or a
 * 1-based index of a non-positive pivot, in which case FE2_ENOCONV is
 * returned and rhs_dev is undefined.  FE2_ENOTSUP when bw exceeds 1120. */
int fe2_band_solve(int n, int bw, const double* band_dev, double* rhs_dev, int* pivot_host, void* stream);

/* fe2_band_solve without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and errors as fe2_band_solve, and
 * the same kernels; the workspace (about 5 bs^2 doubles per block of bs rows)
 * and the pivot report live in a static device array of 64 MiB that the
 * library holds on every GPU it runs on until the process ends.  Systems whose
 * workspace exceeds it fail with FE2_EINVAL before any device work (the 8450
 * unknowns of the 64 x 64 Q4 macro mesh at half bandwidth 133 need 50 MB).
 * Calls on one GPU share that array: calls that overlap on one device (two
 * streams or two threads) race and give undefined results.  Waits for
 * `stream`.  Nothing is allocated by the library on any path of the call. */
int fe2_band_solve_noalloc(int n, int bw, const double* band_dev, double* rhs_dev, int* pivot_host, void* stream);

/* The table of the RVE solver's spectral preconditioner (not an operation of
 * the paper: the inverse of the periodic Q4 stiffness of a homogeneous medium,
 * mu = 1 and lambda = rho, that preconditions the solve of Eq. (42)'s RVE
 * blocks), for inspection and testing; host memory, no GPU work.  n: RVE
 * elements per side, 8, 16, 32 or 48 (else FE2_ENOTSUP); rho > 0.  out_host
 * receives 4 n^2 + 2 t doubles: per position q * n + p of the transformed
 * field, (alpha, Re beta, Im beta, 0) with W(k) = alpha Z(k) + beta conj Z(-k)
 * at the frequency held there (bit-reversed along each axis; for n = 48,
 * position p holds 3 rev(p mod 16) + p / 16), then t twiddles
 * (cos, -sin)(2 pi k / n), t = 32 for n = 48 and n / 2 otherwise.
 * *len_out (may be NULL) receives the length; out_host may be NULL to query
 * it. */
int fe2_spectral_table(int n, double rho, double* out_host, int* len_out);

/* ------------------------------------------------------------------------
 * Surrogate network (not part of the paper): a multilayer perceptron that
 * stands in for the equilibrated RVE response of the nested scheme
 * (Sec. 4.1), trained on RVE solves of this library.  FP32 throughout.
 *   y = W_L h_{L-1} + b_L,  h_l = tanh(W_l h_{l-1} + b_l),  h_0 = x,
 * W_l of shape (sizes[l+1], sizes[l]) row-major; the flat parameter vector
 * holds W_0, b_0, W_1, b_1, ... (fe2_mlp_n_params floats).
 * Loss L = (1/B) sum_s sum_o w_o (y_so - t_so)^2.
 * All *_dev pointers are caller-owned device float32 arrays, row-major
 * [batch][width].  Calls enqueue on `stream` and return without waiting,
 * except fe2_mlp_loss_grad with loss_host != NULL.
 * ------------------------------------------------------------------------ */
typedef struct fe2_mlp_ctx* fe2_mlp;

/* n_layers weight layers (1..8), sizes[n_layers+1] widths (1..4096), buffers
 * for up to max_batch samples.  Parameters and Adam moments start at zero. */
int fe2_mlp_create(int n_layers, const int* sizes, int max_batch, void* stream, fe2_mlp* out);
int fe2_mlp_destroy(fe2_mlp m);
int fe2_mlp_n_params(fe2_mlp m, int64_t* out);
int fe2_mlp_set_params(fe2_mlp m, const float* theta_dev, void* stream);
int fe2_mlp_get_params(fe2_mlp m, float* theta_dev, void* stream);
/* Y_dev [batch][sizes[n_layers]] = network(X_dev [batch][sizes[0]]). */
int fe2_mlp_forward(fe2_mlp m, int batch, const float* X_dev, float* Y_dev, void* stream);
/* Loss and its gradient with respect to the parameters (kept in the handle
 * for fe2_mlp_adam_step; also copied to grad_dev when it is not NULL).
 * loss_host != NULL waits for the stream and returns the loss. */
int fe2_mlp_loss_grad(fe2_mlp m, int batch, const float* X_dev, const float* T_dev, const float* w_out_dev,
                      float* grad_dev, double* loss_host, void* stream);
/* One Adam step (Kingma and Ba, with bias correction) with the stored
 * gradient; the step counter starts at 1 after create or reset. */
int fe2_mlp_adam_step(fe2_mlp m, float lr, float beta1, float beta2, float eps, void* stream);
int fe2_mlp_reset_optimizer(fe2_mlp m, void* stream);

/* ------------------------------------------------------------------------
 * Surrogate of the equilibrated RVE response (2D finite strain).
 * Input x = (E11, E22, E12, phi): Green-Lagrange strain of the macro
 * gradient and the phase-1 volume fraction of the RVE; output
 * y = (S11, S22, S12, D11, D22, D33, D12, D13, D23): second Piola-Kirchhoff
 * stress and the symmetric Voigt matrix of dS/dE (tensor shear components,
 * S_v = D (E11, E22, 2 E12)).  The homogenized first Piola-Kirchhoff stress
 * and tangent follow as P = F S and A_iJkL = delta_ik S_LJ + F_iM F_kN C_MJNL.
 * Normalisation vector `norm` (26 doubles): in_lo[4], in_hi[4] (the network
 * sees 2 (x - lo) / (hi - lo) - 1 and the surrogate is used only inside
 * [lo, hi]), out_mean[9], out_std[9] (y = mean + std * network output).
 * ------------------------------------------------------------------------ */

/* Equilibrated RVE response at caller-given macro gradients (the material
 * point of the nested scheme, Sec. 4.1): F_dev [n_rve][nF]; every RVE is
 * equilibrated from its current fluctuation (fe2_equilibrate_rve rules) and
 * condensed.  Outputs (NULL = skip): P_dev [n_rve][nF] volume-averaged
 * stress, C_dev [n_rve][nF][nF] homogenized tangent, ok_dev [n_rve] 1.0 where
 * the RVE reached equilibrium and the condensation met rve_tol, else 0.0.
 * Returns FE2_ENOCONV when some RVE failed (the others are still valid). */
int fe2_rve_response(fe2_handle h, const double* F_dev, double* P_dev, double* C_dev, double* ok_dev,
                     void* stream);
/* Training pairs from RVE responses of this handle's RVE batch (FP64):
 * X_dev [n_rve][4] inputs, T_dev [n_rve][9] outputs as defined above. */
int fe2_surrogate_dataset(fe2_handle h, const double* F_dev, const double* P_dev, const double* C_dev,
                          double* X_dev, double* T_dev, void* stream);
/* Column statistics of V_dev [n][m] over the rows with ok_dev[row] != 0
 * (ok_dev may be NULL): out_dev [4][m] = min, max, mean, standard deviation. */
int fe2_surrogate_stats(int n, int m, const double* V_dev, const double* ok_dev, double* out_dev, void* stream);
/* out_dev [n][m] (float) = (V - a) / b (mode 0) or 2 (V - a) / (b - a) - 1
 * (mode 1), per column. */
int fe2_surrogate_normalize(int n, int m, const double* V_dev, const double* a_dev, const double* b_dev, int mode,
                            float* out_dev, void* stream);
/* Use the network in fe2_newton_step: every Gauss point whose input lies in
 * [in_lo, in_hi] and that the judge has not rejected takes (P, A) from the
 * network; the others run the classical RVE path (inner equilibration and
 * condensation).  The network must map 4 -> 9 and hold max_batch >= n_rve;
 * the handle keeps the pointer (detach before destroying the network). */
int fe2_surrogate_attach(fe2_handle h, fe2_mlp net, const double* norm_dev, void* stream);
int fe2_surrogate_detach(fe2_handle h);
/* Error judge at the current state: full RVE responses at every Gauss point
 * (surrogate points from w~ = 0) against the network's; a point with
 * max(|dP| / max(|P|, 1e-3 |A|), |dA| / |A|) > tol (Frobenius norms) is
 * rejected for the rest of the handle's life and keeps its equilibrated
 * fluctuation.  Returns the largest error and the number of points rejected
 * by this call. */
int fe2_surrogate_judge(fe2_handle h, double tol, double* max_err_host, int* n_rejected_host, void* stream);

/*
 * 1+1-dimensional FE^2 (Sec. 5.1): macro bar (0, macro_length) with n_macro
 * Lagrange elements of order `order` (1 or 2, equally spaced nodes), RVE
 * (0, 1) with n_micro elements of the same order, micro energy
 * lambda(X~) (F~^2 - 1) (so P~ = 2 lambda F~), uniform body load, prescribed
 * phi at both macro ends and zero fluctuation at both RVE ends (condition (ii)
 * of Eq. (15)).  The macro rule has order + 1 Gauss points per element; RVEs
 * sit at them (basis FE2_BASIS_DIRAC, RVE b = element * (order + 1) + g) or
 * one per macro element (FE2_BASIS_ELEMENT, RVE b = element).  The RVE is
 * integrated with 5 Gauss-Legendre points per element; lambda_gp gives lambda
 * at those points, [n_micro][5], points ordered from -0.906 to 0.906 on the
 * element's reference interval (read during setup and copied).
 * Limits: n_macro <= 2^20 and (order * n_micro - 1) * (order + 3) <= 8192
 * (the shared RVE factor is staged in 64 KiB of LDS).  Errors: FE2_EINVAL.
 */
typedef struct fe2_1d_desc {
  int32_t struct_size;
  int32_t order, n_macro, n_micro, basis;
  double macro_length, body_load, phi_left, phi_right;
  const double* lambda_gp;
} fe2_1d_desc;
typedef struct fe2_1d_ctx* fe2_1d_handle;

/* Set up the RVE matrices, factor the (shared) RVE stiffness once, and start
 * from phi linear between the boundary values and w~ = 0. */
int fe2_1d_setup(const fe2_1d_desc* desc, void* stream, fe2_1d_handle* out);
/* One generalized Newton iteration (Eqs. (46)-(49)) with the basis of the
 * handle: per-RVE residual and solve for x_r, condensation, FP64 macro
 * assembly and banded solve, update.  norms_host (may be NULL) receives the
 * norms of the state the call started from, as fe2_newton_step.  Waits on
 * `stream`. */
int fe2_1d_newton_step(fe2_1d_handle h, double* norms_host, void* stream);
/* phi_dev [order * n_macro + 1] nodal macro deformation; w_dev [n_rve][n_int]
 * fluctuation at the interior RVE nodes (n_int = order * n_micro - 1), in
 * node order; either may be NULL. */
int fe2_1d_get_state(fe2_1d_handle h, double* phi_dev, double* w_dev, void* stream);
enum { FE2_1D_Q_N_PHI = 0, FE2_1D_Q_N_RVE = 1, FE2_1D_Q_N_INT = 2 };
int fe2_1d_query(fe2_1d_handle h, int which, int64_t* out);
int fe2_1d_destroy(fe2_1d_handle h);

const char* fe2_strerror(int status);
const char* fe2_last_error(void);
int fe2_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FE2_H */
