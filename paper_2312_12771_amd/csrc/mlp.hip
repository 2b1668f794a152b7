// Multilayer perceptron of the RVE-response surrogate: forward pass, loss
// gradient by reverse-mode differentiation and Adam, all in FP32 on the GPU.
//
// Network: y = W_L h_{L-1} + b_L, h_l = tanh(W_l h_{l-1} + b_l), h_0 = x,
// W_l stored (out, in) row-major, flat parameter vector layer after layer
// (W_l then b_l).  Loss L = (1/B) sum_s sum_o w_o (y_so - t_so)^2.
//
// Every product is one strided tiled GEMM kernel (64 x 64 output tile, 256
// threads, 4 x 4 outputs per thread, K staged through LDS in chunks of 16):
//   forward      H_l = act(H_{l-1} W_l^T + b_l)          (M = batch)
//   data grad    dZ_{l-1} = (dZ_l W_l) * (1 - H_{l-1}^2)  (M = batch)
//   weight grad  dW_l = dZ_l^T H_{l-1}                    (M = out, split over
//                the batch into fixed chunks, partials summed in a fixed
//                order: deterministic)
// Activations of every layer are kept for the backward pass; buffers are
// sized for max_batch at creation.
#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "fe2_internal.hpp"

namespace fe2 {
namespace {

constexpr int TM = 64, TN = 64, TK = 16, GT = 256;
constexpr int SPLIT_ROWS = 256;   // batch rows per split of the weight gradient

enum Epi { EPI_TANH = 0, EPI_LINEAR = 1, EPI_DTANH = 2, EPI_STORE = 3 };

// C[z][m][n] = sum_{k in split z} A(m, k) B(k, n) (+ epilogue), with
// A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn].
template <int EPI>
__global__ void __launch_bounds__(GT) k_gemm(int M, int N, int K, const float* __restrict__ A, int sam, int sak,
                                             const float* __restrict__ B, int sbk, int sbn, float* __restrict__ C,
                                             int ldc, size_t split_stride, int kchunk, const float* __restrict__ bias,
                                             const float* __restrict__ aux, int ldaux) {
  __shared__ float As[TK][TM + 4];
  __shared__ float Bs[TK][TN + 4];
  const int t = threadIdx.x;
  const int tx = t % 16, ty = t / 16;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  float acc[4][4] = {};
  for (int k0 = kb; k0 < ke; k0 += TK) {
#pragma unroll
    for (int i = 0; i < TM * TK / GT; ++i) {
      const int e = t + i * GT;
      const int mm = e / TK, kk = e % TK;
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < M && k < ke) ? A[static_cast<size_t>(m) * sam + static_cast<size_t>(k) * sak] : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < TN * TK / GT; ++i) {
      const int e = t + i * GT;
      const int kk = e / TN, nn = e % TN;
      const int n = n0 + nn, k = k0 + kk;
      Bs[kk][nn] = (n < N && k < ke) ? B[static_cast<size_t>(k) * sbk + static_cast<size_t>(n) * sbn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  float* Cz = C + blockIdx.z * split_stride;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n >= N) continue;
      float v = acc[i][j];
      if constexpr (EPI == EPI_TANH) v = tanhf(v + bias[n]);
      if constexpr (EPI == EPI_LINEAR) v += bias[n];
      if constexpr (EPI == EPI_DTANH) {
        const float h = aux[static_cast<size_t>(m) * ldaux + n];
        v *= 1.0f - h * h;
      }
      Cz[static_cast<size_t>(m) * ldc + n] = v;
    }
  }
}

// partial column sums of dZ [B][n] over split z -> part[z*stride + n]
__global__ void k_colsum(int Bn, int n, const float* __restrict__ dZ, int kchunk, float* __restrict__ part,
                         size_t stride) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const int z = blockIdx.y;
  const int kb = z * kchunk, ke = min(Bn, kb + kchunk);
  float s = 0.0f;
  for (int k = kb; k < ke; ++k) s += dZ[static_cast<size_t>(k) * n + o];
  part[z * stride + o] = s;
}

// out[i] = sum_z part[z*stride + i], fixed order
__global__ void k_sum_splits(int nsplit, size_t n, const float* __restrict__ part, size_t stride,
                             float* __restrict__ out) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int z = 0; z < nsplit; ++z) s += part[z * stride + i];
  out[i] = s;
}

// output-layer seed of the backward pass and per-block loss partials
__global__ void __launch_bounds__(256) k_loss(int Bn, int n_out, const float* __restrict__ Y,
                                              const float* __restrict__ T, const float* __restrict__ w,
                                              float* __restrict__ dZ, double* __restrict__ part) {
  __shared__ double red[4];
  const size_t n = static_cast<size_t>(Bn) * n_out;
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (i < n) {
    const int o = static_cast<int>(i % n_out);
    const float d = Y[i] - T[i];
    dZ[i] = 2.0f * w[o] * d / static_cast<float>(Bn);
    l = static_cast<double>(w[o]) * d * d;
  }
  l = wave_sum(l);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) / Bn;
}

__global__ void __launch_bounds__(1024) k_sum_double(int n, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < static_cast<int>(blockDim.x / 64); ++k) t += red[k];
    *out = t;
  }
}

__global__ void k_adam(size_t n, float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_fill_f(float* p, size_t n, float v) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned nb(size_t n, unsigned bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

}  // namespace
}  // namespace fe2

using namespace fe2;

struct fe2_mlp_ctx {
  int L = 0;                       // weight layers
  std::vector<int> sizes;          // L + 1
  std::vector<size_t> woff;        // parameter offset of each layer
  size_t n_params = 0;
  int max_batch = 0, max_width = 0;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  float* acts = nullptr;           // h_1 .. h_{L-1}, then y: [B][sizes[l]] each
  std::vector<size_t> aoff;        // offsets into acts (index l = 1 .. L)
  float *dz0 = nullptr, *dz1 = nullptr;
  float* part = nullptr;           // weight-gradient split partials
  size_t part_stride = 0;
  int max_split = 0;
  double *loss_part = nullptr, *loss_dev = nullptr;
  double* loss_host = nullptr;     // pinned
  int step = 0;
};

namespace {

void free_mlp(fe2_mlp_ctx* q) {
  if (!q) return;
  void* p[] = {q->theta, q->grad, q->m, q->v, q->acts, q->dz0, q->dz1, q->part, q->loss_part, q->loss_dev};
  for (void* x : p)
    if (x) (void)hipFree(x);
  if (q->loss_host) (void)hipHostFree(q->loss_host);
  delete q;
}

template <typename T>
int dal(T** p, size_t n) {
  *p = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(p), (n ? n : 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return set_error("hipMalloc failed in the surrogate network"), FE2_ENOMEM;
  }
  return FE2_OK;
}

template <int EPI>
int gemm(int M, int N, int K, const float* A, int sam, int sak, const float* B, int sbk, int sbn, float* C, int ldc,
         size_t split_stride, int nsplit, int kchunk, const float* bias, const float* aux, int ldaux, hipStream_t s) {
  dim3 grid(nb(N, TN), nb(M, TM), nsplit);
  hipLaunchKernelGGL(k_gemm<EPI>, grid, dim3(GT), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, split_stride,
                     kchunk, bias, aux, ldaux);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

// forward pass of `batch` rows of X; activations stay in q->acts
int forward_impl(fe2_mlp_ctx* q, int batch, const float* X, hipStream_t s) {
  const float* h = X;
  for (int l = 0; l < q->L; ++l) {
    const int n_in = q->sizes[l], n_out = q->sizes[l + 1];
    const float* W = q->theta + q->woff[l];
    const float* bias = W + static_cast<size_t>(n_out) * n_in;
    float* out = q->acts + q->aoff[l + 1] * static_cast<size_t>(q->max_batch);
    int rc = (l + 1 < q->L) ? gemm<EPI_TANH>(batch, n_out, n_in, h, n_in, 1, W, 1, n_in, out, n_out, 0, 1, n_in,
                                             bias, nullptr, 0, s)
                            : gemm<EPI_LINEAR>(batch, n_out, n_in, h, n_in, 1, W, 1, n_in, out, n_out, 0, 1, n_in,
                                               bias, nullptr, 0, s);
    if (rc) return rc;
    h = out;
  }
  return FE2_OK;
}

int check_batch(fe2_mlp_ctx* q, int batch) {
  if (batch < 1 || batch > q->max_batch)
    return set_error("batch must be in [1, max_batch]"), FE2_EINVAL;
  return FE2_OK;
}

}  // namespace

namespace fe2 {
int mlp_width(fe2_mlp q, int which) { return which == 0 ? q->sizes.front() : q->sizes.back(); }
int mlp_max_batch(fe2_mlp q) { return q->max_batch; }
}  // namespace fe2

extern "C" {

int fe2_mlp_create(int n_layers, const int* sizes, int max_batch, void* stream, fe2_mlp* out) {
  if (!out) return set_error("null output handle"), FE2_EINVAL;
  *out = nullptr;
  if (n_layers < 1 || n_layers > 8 || !sizes || max_batch < 1)
    return set_error("need 1..8 layers, sizes[n_layers+1] and max_batch >= 1"), FE2_EINVAL;
  for (int l = 0; l <= n_layers; ++l)
    if (sizes[l] < 1 || sizes[l] > 4096) return set_error("layer widths must be in [1, 4096]"), FE2_EINVAL;
  fe2_mlp_ctx* q = new (std::nothrow) fe2_mlp_ctx();
  if (!q) return set_error("host allocation failed"), FE2_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  q->L = n_layers;
  q->sizes.assign(sizes, sizes + n_layers + 1);
  q->max_batch = max_batch;
  size_t off = 0, aw = 0;
  q->aoff.assign(n_layers + 1, 0);
  for (int l = 0; l < n_layers; ++l) {
    q->woff.push_back(off);
    off += static_cast<size_t>(sizes[l + 1]) * sizes[l] + sizes[l + 1];
    q->aoff[l + 1] = aw;
    aw += sizes[l + 1];
    q->max_width = std::max(q->max_width, std::max(sizes[l], sizes[l + 1]));
  }
  q->n_params = off;
  size_t max_wl = 0;
  for (int l = 0; l < n_layers; ++l) max_wl = std::max(max_wl, static_cast<size_t>(sizes[l + 1]) * (sizes[l] + 1));
  q->max_split = (max_batch + SPLIT_ROWS - 1) / SPLIT_ROWS;
  q->part_stride = max_wl;
  const size_t mb = static_cast<size_t>(max_batch);
  int rc = FE2_OK;
  if ((rc = dal(&q->theta, off)) || (rc = dal(&q->grad, off)) || (rc = dal(&q->m, off)) || (rc = dal(&q->v, off)) ||
      (rc = dal(&q->acts, aw * mb)) || (rc = dal(&q->dz0, q->max_width * mb)) ||
      (rc = dal(&q->dz1, q->max_width * mb)) || (rc = dal(&q->part, q->part_stride * q->max_split)) ||
      (rc = dal(&q->loss_part, nb(mb * q->max_width, 256))) || (rc = dal(&q->loss_dev, 1))) {
    free_mlp(q);
    return rc;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&q->loss_host), sizeof(double)) != hipSuccess) {
    free_mlp(q);
    return set_error("pinned host allocation failed"), FE2_ENOMEM;
  }
  for (float* p : {q->theta, q->grad, q->m, q->v}) hipLaunchKernelGGL(k_fill_f, dim3(nb(off, 256)), dim3(256), 0, s, p, off, 0.0f);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    free_mlp(q);
    return set_error("initialisation of the surrogate network failed"), FE2_EHIP;
  }
  *out = q;
  return FE2_OK;
}

int fe2_mlp_destroy(fe2_mlp q) {
  if (!q) return FE2_OK;
  (void)hipDeviceSynchronize();
  free_mlp(q);
  return FE2_OK;
}

int fe2_mlp_n_params(fe2_mlp q, int64_t* out) {
  if (!q || !out) return set_error("null argument"), FE2_EINVAL;
  *out = static_cast<int64_t>(q->n_params);
  return FE2_OK;
}

int fe2_mlp_set_params(fe2_mlp q, const float* theta_dev, void* stream) {
  if (!q || !theta_dev) return set_error("null argument"), FE2_EINVAL;
  FE2_HIP_CHECK(hipMemcpyAsync(q->theta, theta_dev, q->n_params * sizeof(float), hipMemcpyDeviceToDevice,
                               static_cast<hipStream_t>(stream)));
  return FE2_OK;
}

int fe2_mlp_get_params(fe2_mlp q, float* theta_dev, void* stream) {
  if (!q || !theta_dev) return set_error("null argument"), FE2_EINVAL;
  FE2_HIP_CHECK(hipMemcpyAsync(theta_dev, q->theta, q->n_params * sizeof(float), hipMemcpyDeviceToDevice,
                               static_cast<hipStream_t>(stream)));
  return FE2_OK;
}

int fe2_mlp_forward(fe2_mlp q, int batch, const float* X_dev, float* Y_dev, void* stream) {
  if (!q || !X_dev || !Y_dev) return set_error("null argument"), FE2_EINVAL;
  int rc = check_batch(q, batch);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((rc = forward_impl(q, batch, X_dev, s))) return rc;
  const int n_out = q->sizes[q->L];
  FE2_HIP_CHECK(hipMemcpyAsync(Y_dev, q->acts + q->aoff[q->L] * static_cast<size_t>(q->max_batch),
                               static_cast<size_t>(batch) * n_out * sizeof(float), hipMemcpyDeviceToDevice, s));
  return FE2_OK;
}

int fe2_mlp_loss_grad(fe2_mlp q, int batch, const float* X_dev, const float* T_dev, const float* w_out_dev,
                      float* grad_dev, double* loss_host, void* stream) {
  if (!q || !X_dev || !T_dev || !w_out_dev) return set_error("null argument"), FE2_EINVAL;
  int rc = check_batch(q, batch);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((rc = forward_impl(q, batch, X_dev, s))) return rc;
  const int L = q->L;
  const size_t mb = static_cast<size_t>(q->max_batch);
  const int n_out = q->sizes[L];
  const float* Y = q->acts + q->aoff[L] * mb;
  const unsigned nlb = nb(static_cast<size_t>(batch) * n_out, 256);
  hipLaunchKernelGGL(k_loss, dim3(nlb), dim3(256), 0, s, batch, n_out, Y, T_dev, w_out_dev, q->dz0, q->loss_part);
  hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(1024), 0, s, static_cast<int>(nlb), q->loss_part, q->loss_dev);
  FE2_HIP_CHECK(hipGetLastError());
  const int nsplit = (batch + SPLIT_ROWS - 1) / SPLIT_ROWS;
  float* dz = q->dz0;
  float* dzp = q->dz1;
  for (int l = L - 1; l >= 0; --l) {
    const int n_in = q->sizes[l], no = q->sizes[l + 1];
    const float* Hin = (l == 0) ? X_dev : q->acts + q->aoff[l] * mb;
    const float* W = q->theta + q->woff[l];
    // dW_l = dZ^T H_in (split over the batch), db_l = column sums of dZ
    if ((rc = gemm<EPI_STORE>(no, n_in, batch, dz, 1, no, Hin, n_in, 1, q->part, n_in, q->part_stride, nsplit,
                              SPLIT_ROWS, nullptr, nullptr, 0, s)))
      return rc;
    hipLaunchKernelGGL(k_colsum, dim3(nb(no, 64), nsplit), dim3(64), 0, s, batch, no, dz, SPLIT_ROWS,
                       q->part + static_cast<size_t>(no) * n_in, q->part_stride);
    const size_t nl = static_cast<size_t>(no) * (n_in + 1);
    hipLaunchKernelGGL(k_sum_splits, dim3(nb(nl, 256)), dim3(256), 0, s, nsplit, nl, q->part, q->part_stride,
                       q->grad + q->woff[l]);
    FE2_HIP_CHECK(hipGetLastError());
    if (l > 0) {   // dZ_{l-1} = (dZ_l W_l) * (1 - h_{l-1}^2)
      if ((rc = gemm<EPI_DTANH>(batch, n_in, no, dz, no, 1, W, n_in, 1, dzp, n_in, 0, 1, no, nullptr, Hin, n_in, s)))
        return rc;
      std::swap(dz, dzp);
    }
  }
  if (grad_dev)
    FE2_HIP_CHECK(hipMemcpyAsync(grad_dev, q->grad, q->n_params * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (loss_host) {
    FE2_HIP_CHECK(hipMemcpyAsync(q->loss_host, q->loss_dev, sizeof(double), hipMemcpyDeviceToHost, s));
    FE2_HIP_CHECK(hipStreamSynchronize(s));
    *loss_host = *q->loss_host;
  }
  return FE2_OK;
}

int fe2_mlp_adam_step(fe2_mlp q, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!q) return set_error("null handle"), FE2_EINVAL;
  if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return set_error("Adam needs lr > 0, 0 <= beta < 1, eps > 0"), FE2_EINVAL;
  q->step += 1;
  const float c1 = 1.0f - std::pow(beta1, static_cast<float>(q->step));
  const float c2 = 1.0f - std::pow(beta2, static_cast<float>(q->step));
  hipLaunchKernelGGL(k_adam, dim3(nb(q->n_params, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), q->n_params,
                     q->theta, q->grad, q->m, q->v, lr, beta1, beta2, eps, c1, c2);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

int fe2_mlp_reset_optimizer(fe2_mlp q, void* stream) {
  if (!q) return set_error("null handle"), FE2_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  q->step = 0;
  hipLaunchKernelGGL(k_fill_f, dim3(nb(q->n_params, 256)), dim3(256), 0, s, q->m, q->n_params, 0.0f);
  hipLaunchKernelGGL(k_fill_f, dim3(nb(q->n_params, 256)), dim3(256), 0, s, q->v, q->n_params, 0.0f);
  FE2_HIP_CHECK(hipGetLastError());
  return FE2_OK;
}

}  // extern "C"
