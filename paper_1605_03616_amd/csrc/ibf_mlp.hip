// Learned Chebyshev-order predictor: a small multilayer perceptron that models
// log10 of the IBF's achieved relative error (eq:relativeerr) from problem
// features and the order r (the paper reports that error against r in
// Tables 1, 3 and 4, essentially independent of N).  Training and inference
// run in these kernels; for an accuracy target the plan takes the loosest
// truncation tolerance, then the smallest r, whose predicted error plus a
// margin meets the target.
//
//   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = w3 . h2 + b3,
//   loss = mean (y - target)^2,  Adam with bias correction.
// Parameters are one flat FP32 vector:
//   [W1 (H x F row-major), b1 (H), W2 (H x H row-major), b2 (H), w3 (H), b3].
//
// Kernels:
//   k_mlp_forward   one thread per sample, parameters in LDS
//   k_mlp_grad      one 64-sample tile per block: forward, back-propagated
//                   deltas into LDS, then the block's gradient partial sums
//                   (one parameter per thread and pass) and its loss partial
//   k_mlp_reduce    fixed-order sum of the block partials (deterministic)
//   k_mlp_adam      elementwise Adam update
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "ibf_internal.h"

namespace ibf {
namespace {

constexpr int kF = IBF_MLP_FEATURES;
constexpr int kTile = 64;                 // samples per gradient block (one wave)

__host__ __device__ constexpr int mlp_params(int h) { return h * kF + h + h * h + h + h + 1; }

template <int H>
__device__ __forceinline__ void mlp_layers(const float* P, const float* x, float* h1, float* h2,
                                           float& y) {
  const float* W1 = P;
  const float* b1 = W1 + H * kF;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* w3 = b2 + H;
  const float b3 = w3[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    float z = b1[i];
#pragma unroll
    for (int f = 0; f < kF; ++f) z = fmaf(W1[i * kF + f], x[f], z);
    h1[i] = tanhf(z);
  }
  y = b3;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    float z = b2[i];
#pragma unroll
    for (int j = 0; j < H; ++j) z = fmaf(W2[i * H + j], h1[j], z);
    h2[i] = tanhf(z);
    y = fmaf(w3[i], h2[i], y);
  }
}

template <int H>
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ params,
                                                     const float* __restrict__ X, int64_t n,
                                                     float* __restrict__ Y) {
  constexpr int NP = mlp_params(H);
  __shared__ float P[NP];
  for (int e = threadIdx.x; e < NP; e += blockDim.x) P[e] = params[e];
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float x[kF], h1[H], h2[H], y;
#pragma unroll
  for (int f = 0; f < kF; ++f) x[f] = X[s * kF + f];
  mlp_layers<H>(P, x, h1, h2, y);
  Y[s] = y;
}

// work[block][0 .. NP-1] = the block's gradient partials, work[block][NP] = its loss partial
template <int H>
__global__ __launch_bounds__(kTile) void k_mlp_grad(const float* __restrict__ params,
                                                    const float* __restrict__ X,
                                                    const float* __restrict__ T, int64_t n,
                                                    float* __restrict__ work) {
  constexpr int NP = mlp_params(H);
  extern __shared__ __align__(16) float sm[];
  float* P = sm;                          // [NP]
  float* Xs = P + NP;                     // [kTile][kF]
  float* H1 = Xs + kTile * kF;            // [kTile][H]
  float* H2 = H1 + kTile * H;             // [kTile][H]
  float* D2 = H2 + kTile * H;             // [kTile][H]  delta at layer 2 (pre-tanh)
  float* D1 = D2 + kTile * H;             // [kTile][H]  delta at layer 1 (pre-tanh)
  float* DY = D1 + kTile * H;             // [kTile]
  float* SE = DY + kTile;                 // [kTile] squared errors / n
  for (int e = threadIdx.x; e < NP; e += blockDim.x) P[e] = params[e];
  __syncthreads();
  const int tid = threadIdx.x;
  const int64_t s = (int64_t)blockIdx.x * kTile + tid;
  const float inv_n = 1.0f / (float)n;
  float x[kF], h1[H], h2[H], y = 0.f;
  if (s < n) {
#pragma unroll
    for (int f = 0; f < kF; ++f) x[f] = X[s * kF + f];
    mlp_layers<H>(P, x, h1, h2, y);
  } else {
#pragma unroll
    for (int f = 0; f < kF; ++f) x[f] = 0.f;
#pragma unroll
    for (int i = 0; i < H; ++i) h1[i] = h2[i] = 0.f;
  }
  const float err = s < n ? y - T[s] : 0.f;
  const float dy = 2.0f * err * inv_n;                        // d loss / d y
  const float* W2 = P + H * kF + H;
  const float* w3 = W2 + H * H + H;
  float d2[H];
#pragma unroll
  for (int i = 0; i < H; ++i) d2[i] = dy * w3[i] * (1.0f - h2[i] * h2[i]);
#pragma unroll
  for (int j = 0; j < H; ++j) {
    float a = 0.f;
#pragma unroll
    for (int i = 0; i < H; ++i) a = fmaf(d2[i], W2[i * H + j], a);
    D1[tid * H + j] = a * (1.0f - h1[j] * h1[j]);
    H1[tid * H + j] = h1[j];
    H2[tid * H + j] = h2[j];
    D2[tid * H + j] = d2[j];
  }
#pragma unroll
  for (int f = 0; f < kF; ++f) Xs[tid * kF + f] = x[f];
  DY[tid] = dy;
  SE[tid] = err * err * inv_n;
  __syncthreads();
  // gradient partials: parameter e summed over the tile's samples
  float* out = work + (size_t)blockIdx.x * (NP + 1);
  for (int e = tid; e < NP; e += kTile) {
    float acc = 0.f;
    if (e < H * kF) {                                         // W1[i][f]
      const int i = e / kF, f = e % kF;
      for (int q = 0; q < kTile; ++q) acc = fmaf(D1[q * H + i], Xs[q * kF + f], acc);
    } else if (e < H * kF + H) {                              // b1[i]
      const int i = e - H * kF;
      for (int q = 0; q < kTile; ++q) acc += D1[q * H + i];
    } else if (e < H * kF + H + H * H) {                      // W2[i][j]
      const int r = e - H * kF - H, i = r / H, j = r % H;
      for (int q = 0; q < kTile; ++q) acc = fmaf(D2[q * H + i], H1[q * H + j], acc);
    } else if (e < H * kF + 2 * H + H * H) {                  // b2[i]
      const int i = e - H * kF - H - H * H;
      for (int q = 0; q < kTile; ++q) acc += D2[q * H + i];
    } else if (e < NP - 1) {                                  // w3[i]
      const int i = e - H * kF - 2 * H - H * H;
      for (int q = 0; q < kTile; ++q) acc = fmaf(DY[q], H2[q * H + i], acc);
    } else {                                                  // b3
      for (int q = 0; q < kTile; ++q) acc += DY[q];
    }
    out[e] = acc;
  }
  if (tid == 0) {
    float l = 0.f;
    for (int q = 0; q < kTile; ++q) l += SE[q];
    out[NP] = l;
  }
}

__global__ void k_mlp_reduce(const float* __restrict__ work, int nblk, int np,
                             float* __restrict__ grad, float* __restrict__ loss) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > np) return;
  float acc = 0.f;
  for (int b = 0; b < nblk; ++b) acc += work[(size_t)b * (np + 1) + e];
  if (e < np) grad[e] = acc;
  else if (loss) *loss = acc;
}

__global__ void k_mlp_adam(float* __restrict__ p, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, int np, float lr,
                           float beta1, float beta2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np) return;
  const float ge = g[e];
  const float me = beta1 * m[e] + (1.0f - beta1) * ge;
  const float ve = beta2 * v[e] + (1.0f - beta2) * ge * ge;
  m[e] = me;
  v[e] = ve;
  p[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
}

#define IBF_MLP_DISPATCH(h, LAUNCH)                                      \
  switch (h) {                                                           \
    case 8: LAUNCH(8); break;                                            \
    case 16: LAUNCH(16); break;                                          \
    default: LAUNCH(32); break;                                          \
  }

bool hidden_ok(int h) { return h == 8 || h == 16 || h == 32; }

int fail_arg(const char* msg) {
  set_error(msg);
  return IBF_ERR_INVALID_ARG;
}

}  // namespace
}  // namespace ibf

extern "C" {

int ibf_mlp_n_params(int n_hidden) {
  return ibf::hidden_ok(n_hidden) ? ibf::mlp_params(n_hidden) : -1;
}

int ibf_mlp_features(int64_t n, int phase_id, int r, double tol, float* out) {
  if (!out || n < 2 || r < 1 || !(tol > 0.0 && tol < 1.0))
    return ibf::fail_arg("ibf_mlp_features: bad argument");
  int L = 0;
  while (((int64_t)1 << L) < n) ++L;                          // tree depth ceil(log2 n)
  out[0] = (float)((double)n / (double)((int64_t)1 << L));    // width product of every pair
  out[1] = phase_id == IBF_PHASE_FIO1D ? 1.0f : 0.0f;
  out[2] = phase_id == IBF_PHASE_DFT ? 1.0f : 0.0f;
  out[3] = (float)(r / 16.0);
  out[4] = (float)(-std::log10(tol) / 16.0);
  return IBF_OK;
}

int ibf_mlp_forward(const float* params, int n_hidden, const float* X, int64_t n, float* Y,
                    void* stream) {
  if (!params || !X || !Y || n < 0 || !ibf::hidden_ok(n_hidden))
    return ibf::fail_arg("ibf_mlp_forward: bad argument");
  if (n == 0) return IBF_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid((unsigned)((n + 255) / 256));
#define IBF_LAUNCH_MF(HH) hipLaunchKernelGGL(ibf::k_mlp_forward<HH>, grid, dim3(256), 0, s, params, X, n, Y)
  IBF_MLP_DISPATCH(n_hidden, IBF_LAUNCH_MF);
#undef IBF_LAUNCH_MF
  IBF_HIP_CHECK(hipGetLastError());
  return IBF_OK;
}

int64_t ibf_mlp_grad_work(int n_hidden, int64_t n) {
  if (!ibf::hidden_ok(n_hidden) || n < 1) return -1;
  return ((n + ibf::kTile - 1) / ibf::kTile) * (ibf::mlp_params(n_hidden) + 1);
}

int ibf_mlp_loss_grad(const float* params, int n_hidden, const float* X, const float* T,
                      int64_t n, float* grad, float* loss, float* work, void* stream) {
  if (!params || !X || !T || !grad || !work || n < 1 || !ibf::hidden_ok(n_hidden))
    return ibf::fail_arg("ibf_mlp_loss_grad: bad argument");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int np = ibf::mlp_params(n_hidden);
  const int64_t nblk = (n + ibf::kTile - 1) / ibf::kTile;
  if (nblk > (1 << 30)) return ibf::fail_arg("ibf_mlp_loss_grad: too many samples");
  const size_t lds = sizeof(float) * ((size_t)np + ibf::kTile * (ibf::kF + 4 * (size_t)n_hidden + 2));
#define IBF_LAUNCH_MG(HH)                                                                  \
  hipLaunchKernelGGL(ibf::k_mlp_grad<HH>, dim3((unsigned)nblk), dim3(ibf::kTile), lds, s, \
                     params, X, T, n, work)
  IBF_MLP_DISPATCH(n_hidden, IBF_LAUNCH_MG);
#undef IBF_LAUNCH_MG
  IBF_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(ibf::k_mlp_reduce, dim3((unsigned)((np + 1 + 255) / 256)), dim3(256), 0, s,
                     work, (int)nblk, np, grad, loss);
  IBF_HIP_CHECK(hipGetLastError());
  return IBF_OK;
}

int ibf_mlp_adam(float* params, const float* grad, float* m, float* v, int n_params, int step,
                 float lr, float beta1, float beta2, float eps, void* stream) {
  if (!params || !grad || !m || !v || n_params < 1 || step < 1 || !(lr > 0.f) ||
      !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return ibf::fail_arg("ibf_mlp_adam: bad argument");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const float c1 = (float)(1.0 - std::pow((double)beta1, step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, step));
  hipLaunchKernelGGL(ibf::k_mlp_adam, dim3((unsigned)((n_params + 255) / 256)), dim3(256), 0, s,
                     params, grad, m, v, n_params, lr, beta1, beta2, eps, c1, c2);
  IBF_HIP_CHECK(hipGetLastError());
  return IBF_OK;
}

int ibf_mlp_select(const float* params, int n_hidden, int64_t n, int phase_id, double tol,
                   double margin, int rmin, int rmax, int* r_out, double* svd_tol_out,
                   void* stream) {
  if (!params || !r_out || !svd_tol_out || !ibf::hidden_ok(n_hidden) || rmin < 2 ||
      rmax > ibf::kMaxR || rmin > rmax || !(tol > 0.0 && tol < 1.0))
    return ibf::fail_arg("ibf_mlp_select: bad argument");
  *r_out = 0;
  *svd_tol_out = tol;
  // candidates in order of preference: the loosest truncation first (the
  // ranks, hence the stored entries, follow the truncation tolerance), then
  // the smallest r (the build's work grows with r)
  const double cand_tol[4] = {3.0 * tol, tol, tol / 3.0, tol / 10.0};
  const int nr = rmax - rmin + 1, nc = 4 * nr;
  std::vector<float> X((size_t)nc * ibf::kF), Y(nc);
  std::vector<int> valid(nc, 1);
  for (int c = 0; c < nc; ++c) {
    const double st = cand_tol[c / nr];
    if (!(st < 1.0)) {
      valid[c] = 0;
      continue;
    }
    const int rc = ibf_mlp_features(n, phase_id, rmin + c % nr, st,
                                    X.data() + (size_t)c * ibf::kF);
    if (rc) return rc;
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  float* d = nullptr;
  IBF_HIP_CHECK(ibf::dev_malloc(&d, sizeof(float) * (X.size() + Y.size())));
  int rc = IBF_OK;
  hipError_t e = hipMemcpyAsync(d, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    rc = ibf_mlp_forward(params, n_hidden, d, nc, d + X.size(), stream);
    if (!rc) {
      e = hipMemcpyAsync(Y.data(), d + X.size(), sizeof(float) * Y.size(),
                         hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
  }
  (void)ibf::dev_free(d);
  if (rc) return rc;
  IBF_HIP_CHECK(e);
  const double lt = std::log10(tol);
  for (int c = 0; c < nc; ++c)
    if (valid[c] && (double)Y[c] + margin <= lt) {
      *r_out = rmin + c % nr;
      *svd_tol_out = cand_tol[c / nr];
      break;
    }
  return IBF_OK;
}

}  // extern "C"
