// C ABI of libfe2 (see include/fe2.h): handle management, setup and the
// per-step orchestration of the RVE and macro kernels on a HIP stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "macro.hpp"
#include "surrogate.hpp"

namespace fe2 {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

template <typename T>
int dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) return FE2_OK;
  if (hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
    return FE2_ENOMEM;
  }
  return FE2_OK;
}

template <typename T>
int upload(T** p, const T* src, size_t n, hipStream_t s) {
  int rc = dalloc(p, n);
  if (rc) return rc;
  if (n) FE2_HIP_CHECK(hipMemcpyAsync(*p, src, n * sizeof(T), hipMemcpyHostToDevice, s));
  return FE2_OK;
}

inline unsigned nblk(size_t n, unsigned bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

struct RveClass {
  int n1 = 0, n2 = 0;
  double rho = 0.0;
  std::vector<int> rves;
  int* d_list = nullptr;
  double* d_tab = nullptr;   // 2D: kv[10] | KwF[24] | KFF[9] | err | modes[10]
  bool spectral = false;     // spectral preconditioner tables built for the class
  int solver = -1;           // per-class override of the handle's solver (-1: none)
  double* d_fft64 = nullptr; // its table, FP64 and FP32
  float* d_fft32 = nullptr;
};

}  // namespace
}  // namespace fe2

using namespace fe2;

struct fe2_ctx {
  // description
  int dim = 0, kin = 0, mat = 0, nF = 0, nen = 0, n_gp = 0, order = 1;
  int n_nodes = 0, n_elems = 0, n_rve = 0, ndof = 0, bw = 0, nnz = 0, n_pp = 0;
  int precision = 0, solver = 0, scheme = 0;
  int basis = FE2_BASIS_DIRAC, n_qp = 0;
  double rve_size = 1.0, volume = 1.0;
  double rve_tol = 1e-10, inner_tol = 1e-4, newton_tol = 1e-10, micro_tol = 1e-13;
  int max_pcg_it = 2000, max_ir = 8, max_micro_it = 30;
  bool broken = false;
  // macro
  int *conn = nullptr, *is_dir = nullptr, *vec_ptr = nullptr, *vec_src = nullptr;
  int *nz_ptr = nullptr, *nz_col = nullptr, *nzc_ptr = nullptr, *nzc_src = nullptr;
  double *X = nullptr, *dNdX = nullptr, *wdet = nullptr, *f_ext = nullptr, *dir_full = nullptr;
  double* vol = nullptr;          // [n_rve] micro residual weight (wdet or element volume)
  // RVE batch
  int64_t* phase_off = nullptr;
  uint8_t* phase = nullptr;
  double* params = nullptr;
  int64_t* foff = nullptr;
  std::vector<int64_t> h_foff;
  int64_t field_len = 0;
  std::vector<RveClass> classes;
  // state and results
  double lam = 0.0;
  double *u = nullptr, *w = nullptr, *r = nullptr, *Xs = nullptr;
  double *Cbar = nullptr, *Phat = nullptr, *Pbar = nullptr, *mgrad = nullptr, *rnorm2 = nullptr;
  double* rsize2 = nullptr;   // [n_rve] squared size of the element-level terms of r_b (finite strain)
  double *relres = nullptr, *iters = nullptr;
  int* fail_count = nullptr;
  int* info = nullptr;
  double *f_true = nullptr, *f_hat = nullptr, *ke = nullptr, *band = nullptr, *rhs = nullptr;
  double *du = nullptr, *r_true = nullptr, *f_int = nullptr, *norms_dev = nullptr, *kdense = nullptr;
  BcrPlan bcr;                 // block cyclic reduction of the banded macro tangent
  double* bcr_ws = nullptr;
  double* norms_host = nullptr;   // pinned [4]
  // phase timing (HIP events on the caller's stream)
  bool prof = false;
  hipEvent_t ev[8] = {};
  double prof_ms[8] = {};   // assemble+norms, RVE solve, macro assemble+solve, update, steps, solve launches
  double* mv64 = nullptr;
  int* flag_host = nullptr;       // pinned [3]
  double* thr2 = nullptr;         // [n_rve] inner-loop thresholds
  int* count = nullptr;           // [2] RVEs above their threshold, RVEs excluded
  int last_micro_its = 0;
  int* eq_skip = nullptr;         // [n_rve] RVEs excluded from the current inner loop
  const int* skip = nullptr;      // RVEs the RVE kernels leave alone (null: none)
  bool fixed_grad = false;        // macro gradients set by the caller, not from u
  // surrogate (finite strain): network, normalisation, per-point flags
  fe2_mlp surr_net = nullptr;
  double *surr_norm = nullptr, *phi = nullptr, *surrP = nullptr, *surrC = nullptr, *surr_err = nullptr;
  float *surr_X = nullptr, *surr_Y = nullptr;
  int *accept = nullptr, *banned = nullptr;
  double* okf = nullptr;          // [n_rve] fe2_rve_response status
  int last_failed = 0;
  bool have_solution = false;     // X holds the X_F of an earlier solve (warm start)
  // HIP graphs of the solve / macro / update sequence of a Newton step, one
  // per launch configuration (fe2_set_graph); captured on cap_stream
  struct StepGraph {
    int nrhs = 0, flags = 0;
    double lam = 0.0, dlam = 0.0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  std::vector<StepGraph> graphs;

  // the solver a class runs with, and whether that uses the spectral tables
  int class_solver(const RveClass& c) const { return c.solver >= 0 ? c.solver : solver; }
  bool class_fft(const RveClass& c) const {
    const int s = class_solver(c);
    return c.spectral && (s == FE2_SOLVER_AUTO || s == FE2_SOLVER_PCG_FFT || s == FE2_SOLVER_PCG_FFT_MC);
  }

  MacroArgs margs() const {
    MacroArgs m{};
    m.n_rve = n_rve;
    m.dim = dim;
    m.nen = nen;
    m.order = order;
    m.n_gp = n_gp;
    m.nF = nF;
    m.kin = kin;
    m.n_elems = n_elems;
    m.ndof = ndof;
    m.bw = bw;
    m.conn = conn;
    m.X = X;
    m.dNdX = dNdX;
    m.wdet = wdet;
    m.basis = basis;
    m.n_qp = n_qp;
    m.vol = vol;
    m.kpar = params;
    m.phi = phi;
    m.f_ext = f_ext;
    m.is_dir = is_dir;
    m.dir_full = dir_full;
    m.vec_ptr = vec_ptr;
    m.vec_src = vec_src;
    m.nz_ptr = nz_ptr;
    m.nz_col = nz_col;
    m.nzc_ptr = nzc_ptr;
    m.nzc_src = nzc_src;
    return m;
  }

  Fin2DArgs fargs(const RveClass& c, int flags) const {
    Fin2DArgs a{};
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.rve_list = c.d_list;
    a.phase_off = phase_off;
    a.phase = phase;
    a.params = params;
    a.macro = mgrad;
    a.foff = foff;
    a.w = w;
    a.r = r;
    a.X = Xs;
    a.Cbar = Cbar;
    a.Phat = Phat;
    a.Pbar = Pbar;
    a.rnorm2 = rnorm2;
    a.rsize2 = rsize2;
    a.relres = relres;
    a.iters = iters;
    a.mv64 = mv64;
    a.fail_count = fail_count;
    a.thr2 = thr2;
    a.skip = skip;
    a.h1 = rve_size / c.n1;
    a.h2 = rve_size / c.n2;
    a.volume = volume;
    a.tol = rve_tol;
    a.tol_in = precision == FE2_PREC_FP64 ? 0.5 * rve_tol : std::max(0.3 * rve_tol, inner_tol);
    a.max_it = max_pcg_it;
    a.max_ir = max_ir;
    a.fft_tab = c.d_fft32;
    a.fft_tab64 = c.d_fft64;
    a.flags = flags | (class_fft(c) ? RVE_FFT : 0);
    return a;
  }

  Lin2DArgs largs(const RveClass& c, int flags) const {
    Lin2DArgs a{};
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.rve_list = c.d_list;
    a.phase_off = phase_off;
    a.phase = phase;
    a.params = params;
    a.kv64 = c.d_tab;
    a.KwF64 = c.d_tab + 10;
    a.KFF64 = c.d_tab + (dim == 3 ? 154 : 34);
    a.modes64 = dim == 3 ? nullptr : c.d_tab + 44;
    a.macro = mgrad;
    a.foff = foff;
    a.w = w;
    a.r = r;
    a.X = Xs;
    a.Cbar = Cbar;
    a.Phat = Phat;
    a.Pbar = Pbar;
    a.rnorm2 = rnorm2;
    a.relres = relres;
    a.iters = iters;
    a.mv64 = mv64;
    a.fail_count = fail_count;
    a.thr2 = thr2;
    a.skip = skip;
    a.fft_tab = c.d_fft32;
    a.fft_tab64 = c.d_fft64;
    a.volume = volume;
    a.tol = rve_tol;
    a.tol_in = precision == FE2_PREC_FP64 ? 0.5 * rve_tol : std::max(0.3 * rve_tol, inner_tol);
    a.max_it = max_pcg_it;
    a.max_ir = max_ir;
    a.flags = flags | (class_fft(c) ? RVE_FFT : 0) |
              (class_fft(c) && class_solver(c) == FE2_SOLVER_PCG_FFT_MC ? RVE_MC : 0) |
              (class_solver(c) == FE2_SOLVER_DENSE ? RVE_DENSE : 0);
    return a;
  }
};

namespace {

void free_ctx(fe2_ctx* h) {
  if (!h) return;
  void* ptrs[] = {h->conn, h->is_dir, h->vec_ptr, h->vec_src, h->nz_ptr, h->nz_col, h->nzc_ptr,
                  h->nzc_src, h->X, h->dNdX, h->wdet, h->f_ext, h->dir_full, h->phase_off,
                  h->phase, h->params, h->foff, h->u, h->w, h->r, h->Xs, h->Cbar, h->Phat,
                  h->Pbar, h->mgrad, h->rnorm2, h->rsize2, h->relres, h->iters, h->fail_count, h->info,
                  h->f_true, h->f_hat, h->ke, h->band, h->rhs, h->du, h->r_true, h->f_int,
                  h->norms_dev, h->kdense, h->mv64, h->thr2, h->count, h->eq_skip, h->surr_norm, h->phi,
                  h->surrP, h->surrC, h->surr_err, h->surr_X, h->surr_Y, h->accept, h->banned, h->okf,
                  h->bcr_ws, h->vol};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (auto& c : h->classes) {
    if (c.d_list) (void)hipFree(c.d_list);
    if (c.d_tab) (void)hipFree(c.d_tab);
    if (c.d_fft64) (void)hipFree(c.d_fft64);
    if (c.d_fft32) (void)hipFree(c.d_fft32);
  }
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& g : h->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->norms_host) (void)hipHostFree(h->norms_host);
  if (h->flag_host) (void)hipHostFree(h->flag_host);
  delete h;
}

int validate(const fe2_problem_desc* d) {
  if (!d) return set_error("null descriptor"), FE2_EINVAL;
  if (d->struct_size != static_cast<int32_t>(sizeof(fe2_problem_desc)))
    return set_error("struct_size does not match this library's fe2_problem_desc"), FE2_EINVAL;
  if (d->dim != 2 && d->dim != 3) return set_error("dim must be 2 or 3"), FE2_EINVAL;
  if (d->n_nodes <= 0 || d->n_elems <= 0 || !d->X || !d->conn)
    return set_error("empty macro mesh"), FE2_EINVAL;
  if (d->macro_basis != FE2_BASIS_DIRAC && d->macro_basis != FE2_BASIS_ELEMENT)
    return set_error("unknown macro_basis"), FE2_EINVAL;
  if (d->macro_order != 1 && d->macro_order != 2) return set_error("macro_order must be 1 or 2"), FE2_EINVAL;
  if (d->macro_order == 2 && d->dim != 2)
    return set_error("quadratic macro elements are implemented in 2D (Q9)"), FE2_ENOTSUP;
  const int nen = d->macro_order == 2 ? 9 : (1 << d->dim);
  const int ngp = d->macro_order == 2 ? 9 : (1 << d->dim);
  const int rves_per_elem = d->macro_basis == FE2_BASIS_ELEMENT ? 1 : ngp;
  if (d->n_rve != d->n_elems * rves_per_elem)
    return set_error(d->macro_basis == FE2_BASIS_ELEMENT ? "n_rve must equal n_elems with the element basis"
                                                         : "n_rve must equal n_elems * (macro_order + 1)^dim"),
           FE2_EINVAL;
  if (!d->rve_res || !d->rve_off || !d->phase_id || !d->phase_params)
    return set_error("missing RVE arrays"), FE2_EINVAL;
  if (d->n_dir < 0 || (d->n_dir > 0 && (!d->dir_dofs || !d->dir_vals)))
    return set_error("bad Dirichlet arrays"), FE2_EINVAL;
  if (!(d->rve_size > 0.0)) return set_error("rve_size must be positive"), FE2_EINVAL;
  if (d->precision == FE2_PREC_BF16_IR)   // cond(K_ww) * 2^-8 > 1: the refinement would not contract
    return set_error("BF16 refinement cannot converge: cond(K_ww) of these RVEs exceeds 1/u = 256"), FE2_ENOTSUP;
  if (d->precision != FE2_PREC_FP64 && d->precision != FE2_PREC_FP32_IR)
    return set_error("unknown precision"), FE2_EINVAL;
  if (!(d->rve_tol > 0.0) || !(d->newton_tol >= 0.0)) return set_error("tolerances must be positive"), FE2_EINVAL;
  if (d->max_pcg_it <= 0 || d->max_ir < 0) return set_error("iteration caps must be positive"), FE2_EINVAL;
  for (int64_t k = 0; k < static_cast<int64_t>(d->n_elems) * nen; ++k)
    if (d->conn[k] < 0 || d->conn[k] >= d->n_nodes) return set_error("connectivity out of range"), FE2_EINVAL;
  for (int k = 0; k < d->n_dir; ++k) {
    if (d->dir_dofs[k] < 0 || d->dir_dofs[k] >= d->n_nodes * d->dim)
      return set_error("Dirichlet DOF out of range"), FE2_EINVAL;
    if (k && d->dir_dofs[k] <= d->dir_dofs[k - 1])
      return set_error("Dirichlet DOFs must be strictly increasing"), FE2_EINVAL;
  }
  if (d->rve_off[0] != 0) return set_error("rve_off[0] must be 0"), FE2_EINVAL;
  for (int b = 0; b < d->n_rve; ++b) {
    int64_t ne = 1;
    for (int c = 0; c < d->dim; ++c) {
      if (d->rve_res[b * d->dim + c] < 2) return set_error("RVE resolution below 2"), FE2_EINVAL;
      ne *= d->rve_res[b * d->dim + c];
    }
    if (d->rve_off[b + 1] - d->rve_off[b] != ne)
      return set_error("rve_off inconsistent with rve_res at RVE " + std::to_string(b)), FE2_EINVAL;
  }
  for (int64_t k = 0; k < d->rve_off[d->n_rve]; ++k)
    if (d->phase_id[k] > 1) return set_error("phase ids must be 0 or 1"), FE2_EINVAL;
  return FE2_OK;
}

// Macro sparsity, element-entry gather lists and half bandwidth.
int build_macro_lists(fe2_ctx* h, const fe2_problem_desc* d, hipStream_t s) {
  const int dim = h->dim, nen = h->nen, nd = nen * dim, ne = h->n_elems, ndof = h->ndof;
  std::vector<std::vector<int>> vec_rows(ndof);
  std::map<std::pair<int, int>, std::vector<int>> nz;
  int bw = 0;
  for (int e = 0; e < ne; ++e) {
    int edof[24];
    for (int a = 0; a < nen; ++a)
      for (int c = 0; c < dim; ++c) edof[a * dim + c] = d->conn[e * nen + a] * dim + c;
    for (int la = 0; la < nd; ++la) {
      vec_rows[edof[la]].push_back(e * nd + la);
      for (int lb = 0; lb < nd; ++lb) {
        nz[{edof[la], edof[lb]}].push_back((e * nd + la) * nd + lb);
        bw = std::max(bw, std::abs(edof[la] - edof[lb]));
      }
    }
  }
  std::vector<int> vptr(ndof + 1, 0), vsrc;
  for (int i = 0; i < ndof; ++i) {
    vptr[i + 1] = vptr[i] + static_cast<int>(vec_rows[i].size());
    vsrc.insert(vsrc.end(), vec_rows[i].begin(), vec_rows[i].end());
  }
  std::vector<int> zptr(ndof + 1, 0), zcol, cptr(1, 0), csrc;
  for (auto& kv : nz) {
    zptr[kv.first.first + 1]++;
    zcol.push_back(kv.first.second);
    csrc.insert(csrc.end(), kv.second.begin(), kv.second.end());
    cptr.push_back(static_cast<int>(csrc.size()));
  }
  for (int i = 0; i < ndof; ++i) zptr[i + 1] += zptr[i];
  h->bw = bw;
  h->nnz = static_cast<int>(zcol.size());
  int rc;
  if ((rc = upload(&h->vec_ptr, vptr.data(), vptr.size(), s))) return rc;
  if ((rc = upload(&h->vec_src, vsrc.data(), vsrc.size(), s))) return rc;
  if ((rc = upload(&h->nz_ptr, zptr.data(), zptr.size(), s))) return rc;
  if ((rc = upload(&h->nz_col, zcol.data(), zcol.size(), s))) return rc;
  if ((rc = upload(&h->nzc_ptr, cptr.data(), cptr.size(), s))) return rc;
  if ((rc = upload(&h->nzc_src, csrc.data(), csrc.size(), s))) return rc;
  // the host vectors die here: wait for the copies
  FE2_HIP_CHECK(hipStreamSynchronize(s));
  return FE2_OK;
}

int setup_impl(fe2_ctx* h, const fe2_problem_desc* d, hipStream_t s) {
  h->dim = d->dim;
  h->kin = d->kinematics;
  h->mat = d->material;
  h->order = d->macro_order;
  h->nen = h->order == 2 ? 9 : 1 << d->dim;
  h->n_gp = h->order == 2 ? 9 : 1 << d->dim;
  h->nF = d->kinematics == FE2_SMALL_STRAIN ? (d->dim == 2 ? 3 : 6) : d->dim * d->dim;
  h->n_nodes = d->n_nodes;
  h->n_elems = d->n_elems;
  h->n_rve = d->n_rve;
  h->basis = d->macro_basis;
  h->n_qp = d->n_elems * h->n_gp;
  h->ndof = d->n_nodes * d->dim;
  h->n_pp = d->n_phase_params;
  h->precision = d->precision;
  h->solver = d->solver;
  h->scheme = d->scheme;
  h->rve_size = d->rve_size;
  h->volume = std::pow(d->rve_size, d->dim);
  h->rve_tol = d->rve_tol;
  h->inner_tol = d->inner_tol > 0 ? d->inner_tol : 1e-5;
  h->newton_tol = d->newton_tol;
  h->micro_tol = d->micro_tol;
  h->max_pcg_it = d->max_pcg_it;
  h->max_ir = d->max_ir;
  h->max_micro_it = d->max_micro_it;

  // supported combinations
  const bool finite = h->kin == FE2_FINITE_STRAIN;
  if (h->dim == 3 && finite) return set_error("3D RVEs are supported for small strain only"), FE2_ENOTSUP;
  if (h->basis == FE2_BASIS_ELEMENT && finite)
    return set_error("the element basis of the fluctuation is implemented for small strain"), FE2_ENOTSUP;
  if (h->order == 2 && (finite || h->basis != FE2_BASIS_DIRAC))
    return set_error("Q9 macro elements are implemented for small strain with the Dirac basis"), FE2_ENOTSUP;
  if (!finite && (h->mat != FE2_LINEAR_ISO || h->n_pp != 2))
    return set_error("small strain takes FE2_LINEAR_ISO with (lambda, mu) per phase"), FE2_EINVAL;
  if (finite && !((h->mat == FE2_NEO_HOOKE && h->n_pp == 2) || (h->mat == FE2_MOONEY_RIVLIN && h->n_pp == 3)))
    return set_error("finite strain takes FE2_NEO_HOOKE (lambda, mu) or FE2_MOONEY_RIVLIN (alpha, beta, kappa)"),
           FE2_EINVAL;
  if (h->kin != FE2_SMALL_STRAIN && !finite) return set_error("unknown kinematics"), FE2_EINVAL;
  if (h->solver != FE2_SOLVER_AUTO && h->solver != FE2_SOLVER_PCG_JACOBI && h->solver != FE2_SOLVER_PCG_FFT &&
      h->solver != FE2_SOLVER_PCG_FFT_MC && h->solver != FE2_SOLVER_DENSE)
    return set_error("unknown solver"), FE2_EINVAL;
  if (h->solver == FE2_SOLVER_DENSE && (h->dim != 2 || finite || h->precision != FE2_PREC_FP32_IR))
    return set_error("the dense RVE solve is implemented for 2D small strain in FE2_PREC_FP32_IR"), FE2_ENOTSUP;
  if ((h->solver == FE2_SOLVER_PCG_FFT || h->solver == FE2_SOLVER_PCG_FFT_MC) && h->dim != 2)
    return set_error("the spectral preconditioner is implemented for 2D RVEs"), FE2_ENOTSUP;
  if (h->scheme != FE2_SCHEME_GENERALIZED && h->scheme != FE2_SCHEME_CLASSICAL &&
      h->scheme != FE2_SCHEME_CLASSICAL_PLAIN)
    return set_error("unknown scheme"), FE2_EINVAL;
  if (h->scheme != FE2_SCHEME_GENERALIZED && (!(h->micro_tol > 0.0) || h->max_micro_it <= 0))
    return set_error("the classical scheme needs micro_tol > 0 and max_micro_it > 0"), FE2_EINVAL;

  // Per-RVE material parameters as the kernels read them: (lambda, mu) per
  // phase for small strain, (alpha, beta, kappa) of the Eq. (59) family for
  // finite strain (Neo-Hooke: alpha = mu/2, beta = 0, kappa = lambda).
  const int npk = finite ? 3 : 2;
  std::vector<double> kpar(static_cast<size_t>(h->n_rve) * 2 * npk);
  for (int b = 0; b < h->n_rve; ++b)
    for (int q = 0; q < 2; ++q) {
      const double* p = d->phase_params + (static_cast<size_t>(b) * 2 + q) * h->n_pp;
      double* o = kpar.data() + (static_cast<size_t>(b) * 2 + q) * npk;
      if (!finite || h->mat == FE2_NEO_HOOKE) {
        if (!(p[1] > 0.0) || !(p[0] >= 0.0)) return set_error("need mu > 0 and lambda >= 0"), FE2_EINVAL;
      }
      if (!finite) {
        o[0] = p[0];
        o[1] = p[1];
      } else if (h->mat == FE2_NEO_HOOKE) {
        o[0] = 0.5 * p[1];
        o[1] = 0.0;
        o[2] = p[0];
      } else {
        if (!(p[0] + p[1] > 0.0) || !(p[1] >= 0.0) || !(p[2] >= 0.0) || !(p[0] + 2.0 * p[1] >= 0.0))
          return set_error("Mooney-Rivlin phases need alpha + beta > 0, beta >= 0, kappa >= 0"), FE2_EINVAL;
        o[0] = p[0];
        o[1] = p[1];
        o[2] = p[2];
      }
    }

  // RVE classes: (n1, n2, lambda/mu) for small strain, (n1, n2) for finite
  // strain (the finite-strain kernel evaluates the law per Gauss point)
  std::map<std::tuple<int, int, double>, int> key2cls;
  for (int b = 0; b < h->n_rve; ++b) {
    const int n1 = d->rve_res[b * h->dim], n2 = d->rve_res[b * h->dim + 1];
    const int n3 = h->dim == 3 ? d->rve_res[b * 3 + 2] : 1;
    double rho0 = 0.0;
    if (!finite) {
      const double* p = kpar.data() + static_cast<size_t>(b) * 4;
      rho0 = p[0] / p[1];
      const double rho1 = p[2] / p[3];
      if (std::fabs(rho0 - rho1) > 1e-12 * std::fabs(rho0))
        return set_error("both phases of an RVE must share lambda/mu"), FE2_ENOTSUP;
    }
    const bool ok = h->dim == 3 ? lin3d_supported(n1, n2, n3)
                                : (finite ? fin2d_supported(n1, n2) : lin2d_supported(n1, n2));
    if (!ok)
      return set_error("no compiled kernel for RVE resolution " + std::to_string(n1) + "x" + std::to_string(n2) +
                       (h->dim == 3 ? "x" + std::to_string(n3) : std::string())),
             FE2_ENOTSUP;
    if (h->solver == FE2_SOLVER_DENSE && !lin2d_dense_size(n1, n2))
      return set_error("the dense RVE solve needs n1, n2 >= 3 and 2 n1 n2 - 2 <= 128 unknowns"), FE2_ENOTSUP;
    if ((h->solver == FE2_SOLVER_PCG_FFT || h->solver == FE2_SOLVER_PCG_FFT_MC) &&
        !(finite ? fin2d_spectral_size(n1, n2) : lin2d_spectral_size(n1, n2)))
      return set_error(finite ? "the finite-strain spectral preconditioner needs square RVEs of 8, 16 or 32 elements"
                              : "the spectral preconditioner needs square RVEs of 8, 16, 32 or 48 elements"),
             FE2_ENOTSUP;
    auto key = std::make_tuple(n1, n2, rho0);
    auto it = key2cls.find(key);
    int ci;
    if (it == key2cls.end()) {
      ci = static_cast<int>(h->classes.size());
      key2cls[key] = ci;
      RveClass c;
      c.n1 = n1;
      c.n2 = n2;
      c.rho = rho0;
      if (finite) {
        // reference medium of the spectral preconditioner: lambda/mu of the
        // small-strain limit (mu = 2 (alpha + beta), lambda = kappa + 4 beta)
        // of the stiffer phase of the class's first RVE; any positive value
        // gives an SPD preconditioner, this one the closest reference
        const double* q = kpar.data() + static_cast<size_t>(b) * 6;
        const double mu0 = 2.0 * (q[0] + q[1]), mu1 = 2.0 * (q[3] + q[4]);
        const double* qs = mu1 > mu0 ? q + 3 : q;
        c.rho = (qs[2] + 4.0 * qs[1]) / (2.0 * (qs[0] + qs[1]));
      }
      h->classes.push_back(c);
    } else {
      ci = it->second;
    }
    h->classes[ci].rves.push_back(b);
  }

  int rc;
  if ((rc = upload(&h->X, d->X, static_cast<size_t>(h->n_nodes) * h->dim, s))) return rc;
  if ((rc = upload(&h->conn, d->conn, static_cast<size_t>(h->n_elems) * h->nen, s))) return rc;
  {
    std::vector<int> isd(h->ndof, 0);
    std::vector<double> dv(h->ndof, 0.0);
    for (int k = 0; k < d->n_dir; ++k) {
      isd[d->dir_dofs[k]] = 1;
      dv[d->dir_dofs[k]] = d->dir_vals[k];
    }
    if ((rc = upload(&h->is_dir, isd.data(), isd.size(), s))) return rc;
    if ((rc = upload(&h->dir_full, dv.data(), dv.size(), s))) return rc;
    FE2_HIP_CHECK(hipStreamSynchronize(s));
  }
  if (d->f_ext && (rc = upload(&h->f_ext, d->f_ext, h->ndof, s))) return rc;
  const int64_t n_ph = d->rve_off[h->n_rve];
  if ((rc = upload(&h->phase_off, d->rve_off, static_cast<size_t>(h->n_rve) + 1, s))) return rc;
  if ((rc = upload(&h->phase, d->phase_id, static_cast<size_t>(n_ph), s))) return rc;
  if ((rc = upload(&h->params, kpar.data(), kpar.size(), s))) return rc;
  h->h_foff.assign(h->n_rve + 1, 0);
  for (int b = 0; b < h->n_rve; ++b) {
    int64_t nn = 1;
    for (int c = 0; c < h->dim; ++c) nn *= d->rve_res[b * h->dim + c];
    h->h_foff[b + 1] = h->h_foff[b] + nn * h->dim;
  }
  h->field_len = h->h_foff[h->n_rve];
  if ((rc = upload(&h->foff, h->h_foff.data(), h->h_foff.size(), s))) return rc;
  if ((rc = build_macro_lists(h, d, s))) return rc;

  // device state and work buffers
  const size_t nr = h->n_rve, nF = h->nF, nd = static_cast<size_t>(h->nen) * h->dim;
  const size_t nq = h->n_qp;
  if ((rc = dalloc(&h->dNdX, nq * h->nen * h->dim))) return rc;
  if ((rc = dalloc(&h->wdet, nq))) return rc;
  if ((rc = dalloc(&h->vol, nr))) return rc;
  if ((rc = dalloc(&h->u, h->ndof))) return rc;
  if ((rc = dalloc(&h->w, h->field_len))) return rc;
  if ((rc = dalloc(&h->r, h->field_len))) return rc;
  if ((rc = dalloc(&h->Xs, static_cast<size_t>(h->field_len) * (nF + 1)))) return rc;
  if ((rc = dalloc(&h->Cbar, nr * nF * nF))) return rc;
  if ((rc = dalloc(&h->Phat, nr * nF))) return rc;
  if ((rc = dalloc(&h->Pbar, nr * nF))) return rc;
  if ((rc = dalloc(&h->mgrad, nr * nF))) return rc;
  if ((rc = dalloc(&h->rnorm2, nr))) return rc;
  if ((rc = dalloc(&h->rsize2, nr))) return rc;
  if ((rc = dalloc(&h->relres, nr))) return rc;
  if ((rc = dalloc(&h->iters, nr))) return rc;
  if ((rc = dalloc(&h->mv64, nr))) return rc;
  if ((rc = dalloc(&h->fail_count, 1))) return rc;
  if ((rc = dalloc(&h->info, 1))) return rc;
  if ((rc = dalloc(&h->f_true, static_cast<size_t>(h->n_elems) * nd))) return rc;
  if ((rc = dalloc(&h->f_hat, static_cast<size_t>(h->n_elems) * nd))) return rc;
  if ((rc = dalloc(&h->ke, static_cast<size_t>(h->n_elems) * nd * nd))) return rc;
  if ((rc = dalloc(&h->band, static_cast<size_t>(h->ndof) * (h->bw + 1)))) return rc;
  if ((rc = dalloc(&h->rhs, h->ndof))) return rc;
  if ((rc = dalloc(&h->du, h->ndof))) return rc;
  if ((rc = dalloc(&h->r_true, h->ndof))) return rc;
  if ((rc = dalloc(&h->f_int, h->ndof))) return rc;
  if ((rc = dalloc(&h->norms_dev, 4))) return rc;
  if ((rc = dalloc(&h->thr2, nr))) return rc;
  if ((rc = dalloc(&h->count, 2))) return rc;
  if ((rc = dalloc(&h->eq_skip, nr))) return rc;
  if ((rc = dalloc(&h->okf, nr))) return rc;
  if ((rc = dalloc(&h->phi, nr))) return rc;
  hipLaunchKernelGGL(k_phase_fraction, dim3(h->n_rve), dim3(256), 0, s, h->n_rve, h->phase_off, h->phase, h->phi);
  FE2_HIP_CHECK(hipGetLastError());
  if (hipHostMalloc(reinterpret_cast<void**>(&h->norms_host), 4 * sizeof(double)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&h->flag_host), 3 * sizeof(int)) != hipSuccess)
    return set_error("pinned host allocation failed"), FE2_ENOMEM;
  if (h->bw > bcr_max_bandwidth())
    return set_error("macro half bandwidth " + std::to_string(h->bw) + " exceeds the block solver's limit"),
           FE2_ENOTSUP;
  h->bcr = bcr_plan(h->ndof, h->bw);
  if ((rc = dalloc(&h->bcr_ws, bcr_workspace_doubles(h->bcr)))) return rc;

  // zero state
  hipLaunchKernelGGL(k_fill, dim3(nblk(h->ndof, 256)), dim3(256), 0, s, h->u, static_cast<size_t>(h->ndof), 0.0);
  hipLaunchKernelGGL(k_fill, dim3(std::min<unsigned>(4096, nblk(h->field_len, 256))), dim3(256), 0, s, h->w,
                     static_cast<size_t>(h->field_len), 0.0);
  hipLaunchKernelGGL(k_fill, dim3(std::min<unsigned>(4096, nblk(h->field_len * (nF + 1), 256))), dim3(256), 0, s,
                     h->Xs, static_cast<size_t>(h->field_len) * (nF + 1), 0.0);
  hipLaunchKernelGGL(k_fill, dim3(nblk(nr * nF, 256)), dim3(256), 0, s, h->Pbar, nr * nF, 0.0);
  hipLaunchKernelGGL(k_fill, dim3(nblk(h->ndof, 256)), dim3(256), 0, s, h->du, static_cast<size_t>(h->ndof), 0.0);
  FE2_HIP_CHECK(hipGetLastError());

  // macro geometry
  MacroArgs m = h->margs();
  hipLaunchKernelGGL(k_macro_geometry, dim3(nblk(nq, 128)), dim3(128), 0, s, m);
  hipLaunchKernelGGL(k_rve_weight, dim3(nblk(nr, 128)), dim3(128), 0, s, m);
  FE2_HIP_CHECK(hipGetLastError());

  // RVE classes: work lists and reference tables
  for (auto& c : h->classes) {
    if ((rc = upload(&c.d_list, c.rves.data(), c.rves.size(), s))) return rc;
    const bool want_fft =
        h->solver == FE2_SOLVER_PCG_FFT || h->solver == FE2_SOLVER_PCG_FFT_MC || h->solver == FE2_SOLVER_AUTO;
    if (finite) {   // FE2_SOLVER_AUTO: the spectral preconditioner wherever the size allows it
      if (want_fft && fin2d_spectral_size(c.n1, c.n2) && c.rho > 0.0) {
        const size_t nt = 4 * static_cast<size_t>(c.n1) * c.n1 + 2 * lin2d_spectral_twiddles(c.n1);
        std::vector<double> t64(nt);
        lin2d_spectral_table(c.n1, c.rho, t64.data());
        std::vector<float> t32(t64.begin(), t64.end());
        if ((rc = upload(&c.d_fft64, t64.data(), nt, s))) return rc;
        if ((rc = upload(&c.d_fft32, t32.data(), nt, s))) return rc;
        FE2_HIP_CHECK(hipStreamSynchronize(s));   // the host tables die here
        c.spectral = true;
      }
      continue;
    }
    double err = 0.0;
    if (h->dim == 3) {
      if ((rc = dalloc(&c.d_tab, REF3_TABLE))) return rc;
      hipLaunchKernelGGL(k_ref_tables_3d, dim3(1), dim3(64), 0, s, h->rve_size / c.n1, c.rho, c.d_tab);
      FE2_HIP_CHECK(hipGetLastError());
      FE2_HIP_CHECK(hipMemcpyAsync(&err, c.d_tab + REF3_TABLE - 1, sizeof(double), hipMemcpyDeviceToHost, s));
      FE2_HIP_CHECK(hipStreamSynchronize(s));
      if (!(err < 1e-12)) return set_error("reference element table inconsistent"), FE2_EHIP;
      continue;
    }
    // FE2_SOLVER_AUTO: the spectral preconditioner wherever the size allows it
    const bool want =
        h->solver == FE2_SOLVER_PCG_FFT || h->solver == FE2_SOLVER_PCG_FFT_MC || h->solver == FE2_SOLVER_AUTO;
    if (want && lin2d_spectral_size(c.n1, c.n2)) {
      const size_t nt = 4 * static_cast<size_t>(c.n1) * c.n1 + 2 * lin2d_spectral_twiddles(c.n1);
      std::vector<double> t64(nt);
      lin2d_spectral_table(c.n1, c.rho, t64.data());
      std::vector<float> t32(t64.begin(), t64.end());
      if ((rc = upload(&c.d_fft64, t64.data(), nt, s))) return rc;
      if ((rc = upload(&c.d_fft32, t32.data(), nt, s))) return rc;
      FE2_HIP_CHECK(hipStreamSynchronize(s));   // the host tables die here
      c.spectral = true;
    }
    if ((rc = dalloc(&c.d_tab, REF2_TABLE))) return rc;
    hipLaunchKernelGGL(k_ref_tables_2d, dim3(1), dim3(64), 0, s, h->rve_size / c.n1, h->rve_size / c.n2, c.rho,
                       c.d_tab);
    FE2_HIP_CHECK(hipGetLastError());
    FE2_HIP_CHECK(hipMemcpyAsync(&err, c.d_tab + 43, sizeof(double), hipMemcpyDeviceToHost, s));
    FE2_HIP_CHECK(hipStreamSynchronize(s));
    if (!(err < 1e-12)) return set_error("reference element table inconsistent"), FE2_EHIP;
  }
  FE2_HIP_CHECK(hipStreamSynchronize(s));
  h->lam = 0.0;
  return FE2_OK;
}

// one RVE class through the kernel of its kind
int launch_class(fe2_ctx* h, const RveClass& c, int flags, int n, int nrhs, hipStream_t s) {
  if (h->kin == FE2_FINITE_STRAIN) return launch_fin2d(h->fargs(c, flags), n, h->precision, nrhs, s);
  if (h->dim == 3) return launch_lin3d(h->largs(c, flags), n, h->precision, nrhs, s);
  return launch_lin2d(h->largs(c, flags), n, h->precision, nrhs, s);
}

int assemble_impl(fe2_ctx* h, hipStream_t s) {
  MacroArgs m = h->margs();
  if (!h->fixed_grad) {
    hipLaunchKernelGGL(k_macro_grad, dim3(nblk(h->n_rve, 128)), dim3(128), 0, s, m, h->u, h->mgrad);
    FE2_HIP_CHECK(hipGetLastError());
  }
  for (auto& c : h->classes) {
    const int n = static_cast<int>(c.rves.size());
    int rc = launch_class(h, c, RVE_ASSEMBLE, n, 0, s);
    if (rc) return rc;
  }
  return FE2_OK;
}

int solve_impl(fe2_ctx* h, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i, dim3(1), dim3(64), 0, s, h->fail_count, static_cast<size_t>(1), 0);
  const int flags = RVE_SOLVE | (h->have_solution ? RVE_WARM : 0);
  h->have_solution = true;
  for (auto& c : h->classes) {
    const int n = static_cast<int>(c.rves.size());
    int rc = launch_class(h, c, flags, n, nrhs, s);
    if (rc) return rc;
  }
  return FE2_OK;
}

// Classical inner loop at the current macro state (Sec. 4.1): RVE Newton
// iterations w_b -= K_ww^-1 r_b until ||r_b|| <= micro_tol max(1, ||r_b^0||).
// RVEs in h->skip are left alone; an RVE whose inner solve fails is excluded
// from further rounds (the others finish) and the call returns FE2_ENOCONV.
int equilibrate_impl(fe2_ctx* h, hipStream_t s) {
  const unsigned nb = nblk(h->n_rve, 256);
  const int* outer = h->skip;
  hipLaunchKernelGGL(k_copy_mask, dim3(nb), dim3(256), 0, s, h->n_rve, outer, h->eq_skip);
  hipLaunchKernelGGL(k_fill_i, dim3(1), dim3(64), 0, s, h->count + 1, static_cast<size_t>(1), 0);
  FE2_HIP_CHECK(hipGetLastError());
  h->skip = h->eq_skip;
  int rc = assemble_impl(h, s);
  if (!rc) {
    hipLaunchKernelGGL(k_micro_thr, dim3(nb), dim3(256), 0, s, h->n_rve, h->rnorm2,
                       h->kin == FE2_FINITE_STRAIN ? h->rsize2 : static_cast<const double*>(nullptr), h->micro_tol,
                       h->thr2);
    if (hipGetLastError() != hipSuccess) rc = (set_error("launch failed"), FE2_EHIP);
  }
  h->last_micro_its = 0;
  for (int it = 0; !rc; ++it) {
    hipLaunchKernelGGL(k_count_above, dim3(1), dim3(1024), 0, s, h->n_rve, h->rnorm2, h->thr2, h->eq_skip, h->count);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h->flag_host + 1, h->count, 2 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = (set_error("inner loop: HIP call failed"), FE2_EHIP);
      break;
    }
    const int active = h->flag_host[1], dead = h->flag_host[2];
    if (active == 0) {
      if (dead) {
        h->last_failed = dead;
        rc = (set_error(std::to_string(dead) + " inner RVE solves failed (missed rve_tol or indefinite)"),
              FE2_ENOCONV);
      }
      break;
    }
    if (it >= h->max_micro_it) {
      h->last_failed = active + dead;
      rc = (set_error(std::to_string(active) + " RVEs not in equilibrium after max_micro_it"), FE2_ENOCONV);
      break;
    }
    for (auto& c : h->classes) {
      const int n = static_cast<int>(c.rves.size());
      const int fl = RVE_SOLVE | RVE_RONLY;
      rc = launch_class(h, c, fl, n, h->nF + 1, s);
      if (rc) break;
    }
    if (rc) break;
    hipLaunchKernelGGL(k_mark_dead, dim3(nb), dim3(256), 0, s, h->n_rve, h->relres, h->rve_tol, h->eq_skip,
                       h->count + 1);
    hipLaunchKernelGGL(k_sub_xr, dim3(h->n_rve), dim3(256), 0, s, h->nF, h->foff, h->Xs, h->eq_skip, h->w);
    if (hipGetLastError() != hipSuccess) {
      rc = (set_error("inner loop: launch failed"), FE2_EHIP);
      break;
    }
    h->last_micro_its = it + 1;
    rc = assemble_impl(h, s);
  }
  h->skip = outer;
  return rc;
}

// Surrogate pass over all RVEs at the current u (a2 + network): features,
// inference, decoding into Pbar / Phat / Cbar of the accepted points; the
// accepted points become the skip set of the RVE kernels.
int surrogate_eval_impl(fe2_ctx* h, hipStream_t s) {
  MacroArgs m = h->margs();
  const unsigned nb = nblk(h->n_rve, 256);
  hipLaunchKernelGGL(k_macro_grad, dim3(nblk(h->n_rve, 128)), dim3(128), 0, s, m, h->u, h->mgrad);
  hipLaunchKernelGGL(k_surr_features, dim3(nb), dim3(256), 0, s, h->n_rve, h->mgrad, h->phi, h->surr_norm,
                     h->banned, h->surr_X, h->accept);
  FE2_HIP_CHECK(hipGetLastError());
  int rc = fe2_mlp_forward(h->surr_net, h->n_rve, h->surr_X, h->surr_Y, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_surr_decode, dim3(nb), dim3(256), 0, s, h->n_rve, h->surr_Y, h->surr_norm, h->mgrad,
                     h->accept, h->Pbar, h->Phat, h->Cbar, h->rnorm2, h->surrP, h->surrC);
  FE2_HIP_CHECK(hipGetLastError());
  h->skip = h->accept;
  return FE2_OK;
}

struct SkipReset {
  fe2_ctx* h;
  ~SkipReset() {
    h->skip = nullptr;
    h->fixed_grad = false;
  }
};

// Macro residual vectors and norms of the current assembly (no solve).
int residual_impl(fe2_ctx* h, double lam, hipStream_t s) {
  MacroArgs m = h->margs();
  const int nd = h->nen * h->dim;
  hipLaunchKernelGGL(k_macro_elem_vec, dim3(nblk(static_cast<size_t>(h->n_elems) * nd, 128)), dim3(128), 0, s, m,
                     h->Pbar, h->f_true, h->u);
  hipLaunchKernelGGL(k_macro_rows_vec, dim3(nblk(h->ndof, 128)), dim3(128), 0, s, m, h->f_true,
                     static_cast<const double*>(nullptr), lam, h->r_true, h->f_int, static_cast<double*>(nullptr));
  hipLaunchKernelGGL(k_norms, dim3(1), dim3(1024), 0, s, m, h->r_true, h->f_int, h->rnorm2, h->volume,
                     h->norms_dev);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

int macro_solve_impl(fe2_ctx* h, double lam, double dlam, hipStream_t s) {
  MacroArgs m = h->margs();
  const int nd = h->nen * h->dim;
  const size_t ne_rows = static_cast<size_t>(h->n_elems) * nd;
  hipLaunchKernelGGL(k_macro_elem_vec, dim3(nblk(ne_rows, 128)), dim3(128), 0, s, m, h->Phat, h->f_hat, h->u);
  launch_macro_elem_mat(m, h->Cbar, h->ke, s);
  hipLaunchKernelGGL(k_macro_rows_vec, dim3(nblk(h->ndof, 128)), dim3(128), 0, s, m, h->f_true, h->f_hat, lam,
                     static_cast<double*>(nullptr), static_cast<double*>(nullptr), h->rhs);
  const size_t nband = static_cast<size_t>(h->ndof) * (h->bw + 1);
  hipLaunchKernelGGL(k_fill, dim3(std::min<unsigned>(4096, nblk(nband, 256))), dim3(256), 0, s, h->band, nband, 0.0);
  hipLaunchKernelGGL(k_macro_rows_band, dim3(nblk(h->ndof, 128)), dim3(128), 0, s, m, h->ke, dlam, h->band, h->rhs,
                     h->kdense);
  hipLaunchKernelGGL(k_fill_i, dim3(1), dim3(64), 0, s, h->info, static_cast<size_t>(1), 0);
  FE2_HIP_CHECK(hipGetLastError());
  FE2_HIP_CHECK(hipMemcpyAsync(h->du, h->rhs, sizeof(double) * h->ndof, hipMemcpyDeviceToDevice, s));
  return bcr_solve(h->bcr, h->bcr_ws, h->band, h->du, h->info, s);
}

// The RVE solves, macro assembly and solve, and update of a generalized
// Newton step as one HIP graph launch on `s`.  Graphs are cached per launch
// configuration (right-hand sides, warm start, load factor and increment);
// every buffer they touch belongs to the handle, so a cached graph stays
// valid for the handle's lifetime.  Fills use kernels (no memset nodes).
int update_impl(fe2_ctx* h, int use_xr, hipStream_t s, bool move_w = true);
int graph_step_impl(fe2_ctx* h, int nrhs, double lam, double dlam, hipStream_t s) {
  const int flags = RVE_SOLVE | (h->have_solution ? RVE_WARM : 0);
  fe2_ctx::StepGraph* hit = nullptr;
  for (auto& g : h->graphs)
    if (g.nrhs == nrhs && g.flags == flags && g.lam == lam && g.dlam == dlam) hit = &g;
  if (!hit) {
    if (!h->cap_stream) FE2_HIP_CHECK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    constexpr size_t kMaxGraphs = 4;
    if (h->graphs.size() >= kMaxGraphs) {   // drop the oldest
      (void)hipGraphExecDestroy(h->graphs.front().exec);
      (void)hipGraphDestroy(h->graphs.front().graph);
      h->graphs.erase(h->graphs.begin());
    }
    fe2_ctx::StepGraph g;
    g.nrhs = nrhs;
    g.flags = flags;
    g.lam = lam;
    g.dlam = dlam;
    FE2_HIP_CHECK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
    int rc = solve_impl(h, nrhs, h->cap_stream);
    if (!rc) rc = macro_solve_impl(h, lam, dlam, h->cap_stream);
    if (!rc) rc = update_impl(h, nrhs > h->nF, h->cap_stream);
    const hipError_t ec = hipStreamEndCapture(h->cap_stream, &g.graph);
    if (rc) {
      if (g.graph) (void)hipGraphDestroy(g.graph);
      return rc;
    }
    if (ec != hipSuccess) return set_error(std::string("graph capture: ") + hipGetErrorString(ec)), FE2_EHIP;
    const hipError_t ei = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(g.graph);
      return set_error(std::string("graph instantiation: ") + hipGetErrorString(ei)), FE2_EHIP;
    }
    h->graphs.push_back(g);
    hit = &h->graphs.back();
  }
  h->have_solution = true;   // what solve_impl records on the host
  FE2_HIP_CHECK(hipGraphLaunch(hit->exec, s));
  return FE2_OK;
}

int update_impl(fe2_ctx* h, int use_xr, hipStream_t s, bool move_w) {
  MacroArgs m = h->margs();
  hipLaunchKernelGGL(k_axpy, dim3(nblk(h->ndof, 256)), dim3(256), 0, s, h->ndof, h->du, h->u);
  if (move_w && launch_update_w(m, static_cast<int>(h->n_rve), h->du, h->foff, h->Xs, h->w, use_xr, h->skip, s))
    return set_error("field update: unsupported nF or element"), FE2_ENOTSUP;
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

#define FE2_GUARD(h)                                                  \
  do {                                                                \
    if (!(h)) return set_error("null handle"), FE2_EINVAL;            \
    if ((h)->broken) return set_error("handle is unusable"), FE2_ESTATE; \
  } while (0)

// Workspace of fe2_band_solve_noalloc: one file-scope device array per GPU
// (bss of the code object, resident until the process ends).  Host code
// never names the array in a kernel argument or a copy: it resolves the
// device address once per device with hipGetSymbolAddress and uses that.
constexpr size_t kBandScratchBytes = size_t(64) << 20;
constexpr size_t kBandScratchHead = 256;   // pivot report, then the workspace doubles
static __device__ __align__(256) unsigned char scratch[kBandScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved on the first
// call there, with that device current).
int band_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return set_error("no usable current HIP device"), FE2_EHIP;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_error("hipGetSymbolAddress of the band-solve scratch failed"), FE2_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FE2_OK;
}

}  // namespace

extern "C" {

int fe2_abi_version(void) { return FE2_ABI_VERSION; }

const char* fe2_last_error(void) { return g_last_error.c_str(); }

const char* fe2_strerror(int st) {
  switch (st) {
    case FE2_OK: return "ok";
    case FE2_CONVERGED: return "converged";
    case FE2_EINVAL: return "invalid argument";
    case FE2_ENOMEM: return "out of memory";
    case FE2_EHIP: return "HIP runtime error";
    case FE2_ENOCONV: return "RVE solve did not converge";
    case FE2_ESTATE: return "handle unusable";
    case FE2_ENOTSUP: return "not supported";
    default: return "unknown status";
  }
}

int fe2_setup(const fe2_problem_desc* desc, void* stream, fe2_handle* out) {
  if (!out) return set_error("null output handle"), FE2_EINVAL;
  *out = nullptr;
  int rc = validate(desc);
  if (rc) return rc;
  fe2_ctx* h = new (std::nothrow) fe2_ctx();
  if (!h) return set_error("host allocation failed"), FE2_ENOMEM;
  rc = setup_impl(h, desc, static_cast<hipStream_t>(stream));
  if (rc) {
    (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
    free_ctx(h);
    return rc;
  }
  *out = h;
  return FE2_OK;
}

int fe2_assemble_rve(fe2_handle h, void* stream) {
  FE2_GUARD(h);
  return assemble_impl(h, static_cast<hipStream_t>(stream));
}

int fe2_condense(fe2_handle h, double* Cbar_dev, double* Phat_dev, void* stream) {
  FE2_GUARD(h);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = solve_impl(h, h->nF + 1, s);
  if (rc) return rc;
  const size_t nr = h->n_rve;
  if (Cbar_dev)
    FE2_HIP_CHECK(hipMemcpyAsync(Cbar_dev, h->Cbar, nr * h->nF * h->nF * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (Phat_dev)
    FE2_HIP_CHECK(hipMemcpyAsync(Phat_dev, h->Phat, nr * h->nF * sizeof(double), hipMemcpyDeviceToDevice, s));
  FE2_HIP_CHECK(hipMemcpyAsync(h->flag_host, h->fail_count, sizeof(int), hipMemcpyDeviceToHost, s));
  FE2_HIP_CHECK(hipStreamSynchronize(s));
  h->last_failed = h->flag_host[0];
  return h->last_failed ? (set_error(std::to_string(h->last_failed) + " RVE solves missed rve_tol"), FE2_ENOCONV)
                        : FE2_OK;
}

int fe2_newton_step(fe2_handle h, double load_factor, double* norms_host, void* stream) {
  FE2_GUARD(h);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  auto mark = [&](int i) {
    if (h->prof) (void)hipEventRecord(h->ev[i], s);
  };
  SkipReset reset{h};
  const bool surr = h->surr_net != nullptr;
  const bool classical = surr || h->scheme != FE2_SCHEME_GENERALIZED;
  // a2-a4 at the current state (classical: after the inner equilibration;
  // surrogate: network at the accepted points, inner equilibration at the
  // others) and the residual norms (a10)
  mark(0);
  if (surr && (rc = surrogate_eval_impl(h, s))) return rc;
  if ((rc = classical ? equilibrate_impl(h, s) : assemble_impl(h, s))) return rc;
  if ((rc = residual_impl(h, load_factor, s))) return rc;
  mark(1);
  FE2_HIP_CHECK(hipMemcpyAsync(h->norms_host, h->norms_dev, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  FE2_HIP_CHECK(hipStreamSynchronize(s));
  if (norms_host) std::memcpy(norms_host, h->norms_host, 4 * sizeof(double));
  const double dlam = load_factor - h->lam;
  if (dlam == 0.0 && h->norms_host[0] <= h->newton_tol * h->norms_host[3]) {
    if (h->prof) {
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, h->ev[0], h->ev[1]);
      h->prof_ms[0] += ms;
    }
    return FE2_CONVERGED;
  }
  // a5-a6: RVE solves; the residual column is dropped when every RVE
  // residual is exactly zero (first iteration from the reference state)
  // (classical: the RVEs are in equilibrium and only X_F is needed)
  const int nrhs = (classical || h->norms_host[2] == 0.0) ? h->nF : h->nF + 1;
  mark(2);
  if (h->use_graph && !classical) {
    // a5-a9 as one graph launch (phase marks 3 and 4 are not split)
    if ((rc = graph_step_impl(h, nrhs, load_factor, dlam, s))) return rc;
    mark(3);
    mark(4);
  } else {
    if ((rc = solve_impl(h, nrhs, s))) return rc;
    mark(3);
    // a7-a8: macro assembly and banded Cholesky solve with the increment
    if ((rc = macro_solve_impl(h, load_factor, dlam, s))) return rc;
    mark(4);
    // a9: update (the plain staggered scheme moves only the macro field)
    if ((rc = update_impl(h, nrhs > h->nF, s, surr || h->scheme != FE2_SCHEME_CLASSICAL_PLAIN))) return rc;
  }
  mark(5);
  FE2_HIP_CHECK(hipMemcpyAsync(h->flag_host, h->fail_count, sizeof(int), hipMemcpyDeviceToHost, s));
  FE2_HIP_CHECK(hipMemcpyAsync(h->flag_host + 1, h->info, sizeof(int), hipMemcpyDeviceToHost, s));
  FE2_HIP_CHECK(hipStreamSynchronize(s));
  h->lam = load_factor;
  h->last_failed = h->flag_host[0];
  if (h->prof) {
    float ms[5] = {};
    (void)hipEventElapsedTime(&ms[0], h->ev[0], h->ev[1]);
    (void)hipEventElapsedTime(&ms[1], h->ev[2], h->ev[3]);
    (void)hipEventElapsedTime(&ms[2], h->ev[3], h->ev[4]);
    (void)hipEventElapsedTime(&ms[3], h->ev[4], h->ev[5]);
    (void)hipEventElapsedTime(&ms[4], h->ev[0], h->ev[5]);
    for (int i = 0; i < 5; ++i) h->prof_ms[i] += ms[i];
    h->prof_ms[5] += 1.0;
  }
  if (h->flag_host[1] != 0)
    return set_error("macro tangent not positive definite at pivot " + std::to_string(h->flag_host[1])),
           FE2_ENOCONV;
  if (h->last_failed) return set_error(std::to_string(h->last_failed) + " RVE solves missed rve_tol"), FE2_ENOCONV;
  return FE2_OK;
}

int fe2_equilibrate_rve(fe2_handle h, int* iters_host, void* stream) {
  FE2_GUARD(h);
  if (!(h->micro_tol > 0.0) || h->max_micro_it <= 0)
    return set_error("inner equilibration needs micro_tol > 0 and max_micro_it > 0"), FE2_EINVAL;
  const int rc = equilibrate_impl(h, static_cast<hipStream_t>(stream));
  if (iters_host) *iters_host = h->last_micro_its;
  return rc;
}

int fe2_rve_response(fe2_handle h, const double* F_dev, double* P_dev, double* C_dev, double* ok_dev, void* stream) {
  FE2_GUARD(h);
  if (!F_dev) return set_error("null macro gradients"), FE2_EINVAL;
  if (!(h->micro_tol > 0.0) || h->max_micro_it <= 0)
    return set_error("the RVE response needs micro_tol > 0 and max_micro_it > 0"), FE2_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SkipReset reset{h};
  const size_t nr = h->n_rve, nF = h->nF;
  FE2_HIP_CHECK(hipMemcpyAsync(h->mgrad, F_dev, nr * nF * sizeof(double), hipMemcpyDeviceToDevice, s));
  h->fixed_grad = true;
  h->skip = nullptr;
  const int rc = equilibrate_impl(h, s);
  if (rc && rc != FE2_ENOCONV) return rc;
  h->skip = h->eq_skip;   // RVEs whose inner loop failed are not condensed
  int rc2 = solve_impl(h, h->nF, s);
  if (rc2) return rc2;
  hipLaunchKernelGGL(k_ok_flags, dim3(nblk(nr, 256)), dim3(256), 0, s, h->n_rve, h->rnorm2, h->thr2, h->relres,
                     h->rve_tol, h->okf);
  FE2_HIP_CHECK(hipGetLastError());
  if (P_dev) FE2_HIP_CHECK(hipMemcpyAsync(P_dev, h->Pbar, nr * nF * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (C_dev) FE2_HIP_CHECK(hipMemcpyAsync(C_dev, h->Cbar, nr * nF * nF * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (ok_dev) FE2_HIP_CHECK(hipMemcpyAsync(ok_dev, h->okf, nr * sizeof(double), hipMemcpyDeviceToDevice, s));
  FE2_HIP_CHECK(hipMemcpyAsync(h->flag_host, h->fail_count, sizeof(int), hipMemcpyDeviceToHost, s));
  FE2_HIP_CHECK(hipStreamSynchronize(s));
  if (rc == FE2_OK && h->flag_host[0] != 0) {
    h->last_failed = h->flag_host[0];
    return set_error(std::to_string(h->last_failed) + " RVE condensations missed rve_tol"), FE2_ENOCONV;
  }
  return rc;
}

int fe2_surrogate_dataset(fe2_handle h, const double* F_dev, const double* P_dev, const double* C_dev,
                          double* X_dev, double* T_dev, void* stream) {
  FE2_GUARD(h);
  if (h->kin != FE2_FINITE_STRAIN || h->dim != 2)
    return set_error("the surrogate covers 2D finite strain"), FE2_ENOTSUP;
  if (!F_dev || !P_dev || !C_dev || !X_dev || !T_dev) return set_error("null argument"), FE2_EINVAL;
  hipLaunchKernelGGL(k_surr_targets, dim3(nblk(h->n_rve, 128)), dim3(128), 0, static_cast<hipStream_t>(stream),
                     h->n_rve, F_dev, P_dev, C_dev, h->phi, X_dev, T_dev);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

int fe2_spectral_table(int n, double rho, double* out_host, int* len_out) {
  if (!lin2d_spectral_size(n, n)) return set_error("spectral table: n must be 8, 16, 32 or 48"), FE2_ENOTSUP;
  if (!(rho > 0.0)) return set_error("spectral table: rho must be positive"), FE2_EINVAL;
  const int len = 4 * n * n + 2 * lin2d_spectral_twiddles(n);
  if (len_out) *len_out = len;
  if (out_host) lin2d_spectral_table(n, rho, out_host);
  return FE2_OK;
}

int fe2_band_solve(int n, int bw, const double* band_dev, double* rhs_dev, int* pivot_host, void* stream) {
  if (pivot_host) *pivot_host = 0;
  if (n < 1 || bw < 0 || !band_dev || !rhs_dev)
    return set_error("invalid band solve arguments"), FE2_EINVAL;
  if (bw > bcr_max_bandwidth())
    return set_error("half bandwidth " + std::to_string(bw) + " exceeds the block solver's limit"), FE2_ENOTSUP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const BcrPlan plan = bcr_plan(n, bw);
  double* ws = nullptr;
  int* info = nullptr;
  int rc = dalloc(&ws, bcr_workspace_doubles(plan));
  if (rc) return rc;
  if (hipMalloc(reinterpret_cast<void**>(&info), sizeof(int)) != hipSuccess) {
    (void)hipFree(ws);
    return set_error("device allocation failed"), FE2_ENOMEM;
  }
  int piv = 0;
  hipLaunchKernelGGL(k_fill_i, dim3(1), dim3(64), 0, s, info, static_cast<size_t>(1), 0);
  rc = bcr_solve(plan, ws, band_dev, rhs_dev, info, s);
  if (!rc && (hipMemcpyAsync(&piv, info, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess))
    rc = (set_error("band solve failed on the device"), FE2_EHIP);
  (void)hipFree(ws);
  (void)hipFree(info);
  if (rc) return rc;
  if (pivot_host) *pivot_host = piv;
  if (piv) return set_error("matrix not positive definite at pivot " + std::to_string(piv)), FE2_ENOCONV;
  return FE2_OK;
}

int fe2_band_solve_noalloc(int n, int bw, const double* band_dev, double* rhs_dev, int* pivot_host, void* stream) {
  if (pivot_host) *pivot_host = 0;
  if (n < 1 || bw < 0 || !band_dev || !rhs_dev)
    return set_error("invalid band solve arguments"), FE2_EINVAL;
  if (bw > bcr_max_bandwidth())
    return set_error("half bandwidth " + std::to_string(bw) + " exceeds the block solver's limit"), FE2_ENOTSUP;
  const BcrPlan plan = bcr_plan(n, bw);
  const size_t need = kBandScratchHead + bcr_workspace_doubles(plan) * sizeof(double);
  if (need > kBandScratchBytes)
    return set_error("band solve needs " + std::to_string(need) + " bytes of workspace; the static scratch holds " +
                     std::to_string(kBandScratchBytes)),
           FE2_EINVAL;
  void* base = nullptr;
  int rc = band_scratch(&base);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int* info = static_cast<int*>(base);
  double* ws = reinterpret_cast<double*>(static_cast<unsigned char*>(base) + kBandScratchHead);
  // the pivot report must start at zero (a fill kernel, not a memset node)
  hipLaunchKernelGGL(k_fill_i, dim3(1), dim3(64), 0, s, info, static_cast<size_t>(1), 0);
  rc = bcr_solve(plan, ws, band_dev, rhs_dev, info, s);
  if (rc) return rc;
  int piv = 0;
  if (hipMemcpyAsync(&piv, info, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    return set_error("band solve failed on the device"), FE2_EHIP;
  }
  if (pivot_host) *pivot_host = piv;
  if (piv) return set_error("matrix not positive definite at pivot " + std::to_string(piv)), FE2_ENOCONV;
  return FE2_OK;
}

int fe2_surrogate_stats(int n, int m, const double* V_dev, const double* ok_dev, double* out_dev, void* stream) {
  if (n < 1 || m < 1 || !V_dev || !out_dev) return set_error("invalid statistics arguments"), FE2_EINVAL;
  hipLaunchKernelGGL(k_col_stats, dim3(m), dim3(256), 0, static_cast<hipStream_t>(stream), n, m, V_dev, ok_dev,
                     out_dev);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

int fe2_surrogate_normalize(int n, int m, const double* V_dev, const double* a_dev, const double* b_dev, int mode,
                            float* out_dev, void* stream) {
  if (n < 1 || m < 1 || !V_dev || !a_dev || !b_dev || !out_dev || (mode != 0 && mode != 1))
    return set_error("invalid normalisation arguments"), FE2_EINVAL;
  const size_t nn = static_cast<size_t>(n) * m;
  hipLaunchKernelGGL(k_normalize, dim3(nblk(nn, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), n, m, V_dev,
                     a_dev, b_dev, mode, out_dev);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

int fe2_surrogate_attach(fe2_handle h, fe2_mlp net, const double* norm_dev, void* stream) {
  FE2_GUARD(h);
  if (h->kin != FE2_FINITE_STRAIN || h->dim != 2)
    return set_error("the surrogate covers 2D finite strain"), FE2_ENOTSUP;
  if (!net || !norm_dev) return set_error("null argument"), FE2_EINVAL;
  if (mlp_width(net, 0) != SURR_NIN || mlp_width(net, 1) != SURR_NOUT)
    return set_error("the surrogate network must map 4 inputs to 9 outputs"), FE2_EINVAL;
  if (mlp_max_batch(net) < h->n_rve) return set_error("network max_batch below the number of RVEs"), FE2_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t nr = h->n_rve;
  int rc;
  if (!h->surr_norm) {
    if ((rc = dalloc(&h->surr_norm, SURR_NORM)) || (rc = dalloc(&h->surrP, nr * 4)) ||
        (rc = dalloc(&h->surrC, nr * 16)) || (rc = dalloc(&h->surr_err, nr)) || (rc = dalloc(&h->surr_X, nr * 4)) ||
        (rc = dalloc(&h->surr_Y, nr * 9)) || (rc = dalloc(&h->accept, nr)) || (rc = dalloc(&h->banned, nr)))
      return rc;
  }
  FE2_HIP_CHECK(hipMemcpyAsync(h->surr_norm, norm_dev, SURR_NORM * sizeof(double), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_fill_i, dim3(nblk(nr, 256)), dim3(256), 0, s, h->banned, nr, 0);
  hipLaunchKernelGGL(k_fill_i, dim3(nblk(nr, 256)), dim3(256), 0, s, h->accept, nr, 0);
  FE2_HIP_CHECK(hipGetLastError());
  h->surr_net = net;
  return FE2_OK;
}

int fe2_surrogate_detach(fe2_handle h) {
  FE2_GUARD(h);
  h->surr_net = nullptr;
  return FE2_OK;
}

int fe2_surrogate_judge(fe2_handle h, double tol, double* max_err_host, int* n_rejected_host, void* stream) {
  FE2_GUARD(h);
  if (!h->surr_net) return set_error("no surrogate attached"), FE2_ESTATE;
  if (!(tol > 0.0)) return set_error("tol must be positive"), FE2_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SkipReset reset{h};
  int rc = surrogate_eval_impl(h, s);
  if (rc) return rc;
  // full RVE responses at every point; the accepted points start from w = 0
  hipLaunchKernelGGL(k_zero_w_masked, dim3(h->n_rve), dim3(256), 0, s, h->foff, h->accept, h->w);
  FE2_HIP_CHECK(hipGetLastError());
  h->skip = nullptr;
  h->fixed_grad = true;
  const int rc_eq = equilibrate_impl(h, s);
  if (rc_eq && rc_eq != FE2_ENOCONV) return rc_eq;
  h->skip = h->eq_skip;
  if ((rc = solve_impl(h, h->nF, s))) return rc;
  hipLaunchKernelGGL(k_fill_i, dim3(1), dim3(64), 0, s, h->count, static_cast<size_t>(1), 0);
  hipLaunchKernelGGL(k_surr_compare, dim3(nblk(h->n_rve, 256)), dim3(256), 0, s, h->n_rve, h->accept, h->surrP,
                     h->surrC, h->Pbar, h->Cbar, tol, h->surr_err, h->banned, h->count);
  hipLaunchKernelGGL(k_col_stats, dim3(1), dim3(256), 0, s, h->n_rve, 1, h->surr_err,
                     static_cast<const double*>(nullptr), h->norms_dev);
  FE2_HIP_CHECK(hipGetLastError());
  double st[4];
  FE2_HIP_CHECK(hipMemcpyAsync(st, h->norms_dev, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  FE2_HIP_CHECK(hipMemcpyAsync(h->flag_host, h->count, sizeof(int), hipMemcpyDeviceToHost, s));
  FE2_HIP_CHECK(hipStreamSynchronize(s));
  if (max_err_host) *max_err_host = st[1];
  if (n_rejected_host) *n_rejected_host = h->flag_host[0];
  return rc_eq;
}

int fe2_get_state(fe2_handle h, double* u_dev, double* w_dev, void* stream) {
  FE2_GUARD(h);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (u_dev) FE2_HIP_CHECK(hipMemcpyAsync(u_dev, h->u, sizeof(double) * h->ndof, hipMemcpyDeviceToDevice, s));
  if (w_dev) FE2_HIP_CHECK(hipMemcpyAsync(w_dev, h->w, sizeof(double) * h->field_len, hipMemcpyDeviceToDevice, s));
  return FE2_OK;
}

int fe2_set_state(fe2_handle h, const double* u_dev, const double* w_dev, double load_factor, void* stream) {
  FE2_GUARD(h);
  h->have_solution = false;   // a new state: start the next solve from zero
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (u_dev) FE2_HIP_CHECK(hipMemcpyAsync(h->u, u_dev, sizeof(double) * h->ndof, hipMemcpyDeviceToDevice, s));
  if (w_dev) FE2_HIP_CHECK(hipMemcpyAsync(h->w, w_dev, sizeof(double) * h->field_len, hipMemcpyDeviceToDevice, s));
  h->lam = load_factor;
  return FE2_OK;
}

int fe2_reset_state(fe2_handle h, double load_factor, void* stream) {
  FE2_GUARD(h);
  h->have_solution = false;   // a new state: start the next solve from zero
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_fill, dim3(nblk(h->ndof, 256)), dim3(256), 0, s, h->u, static_cast<size_t>(h->ndof), 0.0);
  hipLaunchKernelGGL(k_fill, dim3(std::min<unsigned>(4096, nblk(h->field_len, 256))), dim3(256), 0, s, h->w,
                     static_cast<size_t>(h->field_len), 0.0);
  FE2_HIP_CHECK(hipGetLastError());
  h->lam = load_factor;
  return FE2_OK;
}

int fe2_get_data(fe2_handle h, int which, double* dst, void* stream) {
  FE2_GUARD(h);
  if (!dst) return set_error("null destination"), FE2_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t nr = h->n_rve, nF = h->nF;
  const double* src = nullptr;
  size_t n = 0;
  switch (which) {
    case FE2_D_MACRO_GRAD: src = h->mgrad; n = nr * nF; break;
    case FE2_D_RESIDUAL: src = h->r; n = h->field_len; break;
    case FE2_D_PBAR: src = h->Pbar; n = nr * nF; break;
    case FE2_D_SOLUTION: src = h->Xs; n = static_cast<size_t>(h->field_len) * (nF + 1); break;
    case FE2_D_RVE_ITERS: src = h->iters; n = nr; break;
    case FE2_D_RVE_RELRES: src = h->relres; n = nr; break;
    case FE2_D_RVE_MV64: src = h->mv64; n = nr; break;
    case FE2_D_PHASE_FRACTION: src = h->phi; n = nr; break;
    case FE2_D_SURR_ERR: src = h->surr_err; n = nr; break;
    case FE2_D_MACRO_RHS: src = h->rhs; n = h->ndof; break;
    case FE2_D_MACRO_RTRUE: src = h->r_true; n = h->ndof; break;
    case FE2_D_MACRO_DU: src = h->du; n = h->ndof; break;
    case FE2_D_CBAR: src = h->Cbar; n = nr * nF * nF; break;
    case FE2_D_PHAT: src = h->Phat; n = nr * nF; break;
    case FE2_D_MACRO_KDENSE: {
      if (h->ndof > 4096) return set_error("dense macro tangent only for ndof <= 4096"), FE2_EINVAL;
      const size_t nn = static_cast<size_t>(h->ndof) * h->ndof;
      if (!h->kdense) {
        int rc = dalloc(&h->kdense, nn);
        if (rc) return rc;
      }
      // rebuild from the element matrices of the last step (no Dirichlet change)
      MacroArgs m = h->margs();
      hipLaunchKernelGGL(k_fill, dim3(std::min<unsigned>(4096, nblk(nn, 256))), dim3(256), 0, s, h->kdense, nn, 0.0);
      const size_t nband = static_cast<size_t>(h->ndof) * (h->bw + 1);
      double* scratch_band = nullptr;
      double* scratch_rhs = nullptr;
      int rc = dalloc(&scratch_band, nband);
      if (rc) return rc;
      if ((rc = dalloc(&scratch_rhs, h->ndof))) {
        (void)hipFree(scratch_band);
        return rc;
      }
      hipLaunchKernelGGL(k_fill, dim3(nblk(h->ndof, 256)), dim3(256), 0, s, scratch_rhs,
                         static_cast<size_t>(h->ndof), 0.0);
      hipLaunchKernelGGL(k_macro_rows_band, dim3(nblk(h->ndof, 128)), dim3(128), 0, s, m, h->ke, 0.0, scratch_band,
                         scratch_rhs, h->kdense);
      FE2_HIP_CHECK(hipMemcpyAsync(dst, h->kdense, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
      FE2_HIP_CHECK(hipStreamSynchronize(s));
      (void)hipFree(scratch_band);
      (void)hipFree(scratch_rhs);
      return FE2_OK;
    }
    default: return set_error("unknown data selector"), FE2_EINVAL;
  }
  FE2_HIP_CHECK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  return FE2_OK;
}

int fe2_query(fe2_handle h, int which, int64_t* out) {
  FE2_GUARD(h);
  if (!out) return set_error("null output"), FE2_EINVAL;
  switch (which) {
    case FE2_Q_NF: *out = h->nF; return FE2_OK;
    case FE2_Q_FIELD_LEN: *out = h->field_len; return FE2_OK;
    case FE2_Q_NDOF: *out = h->ndof; return FE2_OK;
    case FE2_Q_BANDWIDTH: *out = h->bw; return FE2_OK;
    case FE2_Q_SPECTRAL_RVES: {
      int64_t n = 0;
      for (const auto& c : h->classes)
        if (h->class_fft(c)) n += static_cast<int64_t>(c.rves.size());
      *out = n;
      return FE2_OK;
    }
    case FE2_Q_FAILED_RVES: *out = h->last_failed; return FE2_OK;
    case FE2_Q_N_RVE: *out = h->n_rve; return FE2_OK;
    case FE2_Q_FIELD_OFFSETS: std::memcpy(out, h->h_foff.data(), h->h_foff.size() * sizeof(int64_t)); return FE2_OK;
    case FE2_Q_MICRO_ITERS: *out = h->last_micro_its; return FE2_OK;
    default: return set_error("unknown query"), FE2_EINVAL;
  }
}

int fe2_set_profiling(fe2_handle h, int enable) {
  FE2_GUARD(h);
  if (enable && !h->ev[0])
    for (auto& e : h->ev) FE2_HIP_CHECK(hipEventCreate(&e));
  h->prof = enable != 0;
  for (double& v : h->prof_ms) v = 0.0;
  return FE2_OK;
}

int fe2_set_class_solver(fe2_handle h, int n1, int n2, int n3, int solver) {
  FE2_GUARD(h);
  if (solver != FE2_SOLVER_AUTO && solver != FE2_SOLVER_PCG_JACOBI && solver != FE2_SOLVER_PCG_FFT &&
      solver != FE2_SOLVER_PCG_FFT_MC && solver != FE2_SOLVER_DENSE)
    return set_error("unknown solver"), FE2_EINVAL;
  const bool finite = h->kin == FE2_FINITE_STRAIN;
  int hits = 0;
  for (const auto& c : h->classes) {
    if (c.n1 != n1 || c.n2 != n2 || (h->dim == 3 && c.n1 != n3)) continue;
    ++hits;
    if ((solver == FE2_SOLVER_PCG_FFT || solver == FE2_SOLVER_PCG_FFT_MC) && !c.spectral)
      return set_error("no spectral tables for this class (size, or a handle set up with FE2_SOLVER_PCG_JACOBI)"),
             FE2_ENOTSUP;
    if (solver == FE2_SOLVER_DENSE &&
        (h->dim != 2 || finite || h->precision != FE2_PREC_FP32_IR || !lin2d_dense_size(n1, n2)))
      return set_error("the dense RVE solve is implemented for 2D small strain in FE2_PREC_FP32_IR up to 128 unknowns"),
             FE2_ENOTSUP;
  }
  if (!hits) return set_error("no RVE class of that resolution"), FE2_EINVAL;
  for (auto& c : h->classes)
    if (c.n1 == n1 && c.n2 == n2 && (h->dim != 3 || c.n1 == n3)) c.solver = solver;
  // cached step graphs hold the old launches
  for (auto& g : h->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  h->graphs.clear();
  return FE2_OK;
}

int fe2_set_graph(fe2_handle h, int enable) {
  FE2_GUARD(h);
  h->use_graph = enable != 0;
  return FE2_OK;
}

int fe2_get_profile(fe2_handle h, double* out) {
  FE2_GUARD(h);
  if (!out) return set_error("null output"), FE2_EINVAL;
  std::memcpy(out, h->prof_ms, 6 * sizeof(double));
  for (double& v : h->prof_ms) v = 0.0;
  return FE2_OK;
}

int fe2_destroy(fe2_handle h) {
  if (!h) return FE2_OK;
  (void)hipDeviceSynchronize();
  free_ctx(h);
  return FE2_OK;
}

}  // extern "C"
