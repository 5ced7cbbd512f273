// Application of the compressed IBF: u = Ubar Gbar^{L-l0} ... Gbar^{h+1}
// Hbar^{h} ... Hbar^{l0+1} Vbar^* g  (paper Sec. 4, eqn:IBFout), a sequence
// of block-sparse products.  Coefficient vectors live in ping-pong buffers
// laid out [pair][k][rhs]; pair p at level l is the bit string
// p = a 2^(L-l) + b (a: T_X box at level l, b: T_Omega box at level L-l).
// One butterfly stage maps inputs (a>>1, 2b), (a>>1, 2b+1) at level l-1 to
// output (a, b) at level l through a k_out x 2 k_in block.
#include <algorithm>
#include <cstdio>
#include <vector>

#include "ibf_device.h"

namespace ibf {
namespace {

constexpr int kBlock = 256;

template <typename VT> struct Zero;
template <> struct Zero<double2> { __device__ static double2 v() { return make_double2(0, 0); } };
template <> struct Zero<float2> { __device__ static float2 v() { return make_float2(0, 0); } };

// mu[p][k][n] = sum_{xi in leaf b} Vbar^*[xi][a][k] g[perm(xi)][n],  p = a 2^(L-l0) + b
template <typename VT, typename FT>
__global__ void k_apply_v(const VT* __restrict__ g, int64_t ldg, const int32_t* __restrict__ perm_xi,
                          const int32_t* __restrict__ xioff, const FT* __restrict__ vbar,
                          VT* __restrict__ mu, int L, int l0, int K, int nrhs, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int n = (int)(e % nrhs);
  const int k = (int)((e / nrhs) % K);
  const int64_t p = e / ((int64_t)nrhs * K);
  const int sh = L - l0;
  const int64_t a = p >> sh;
  const int64_t b = p & (((int64_t)1 << sh) - 1);
  VT acc = Zero<VT>::v();
  const int32_t j0 = xioff[b], j1 = xioff[b + 1];
  for (int32_t j = j0; j < j1; ++j) {
    const VT gv = g[(int64_t)n * ldg + perm_xi[j]];
    cfma(acc, load_factor(vbar, (((int64_t)j << l0) | a) * K + k), gv);
  }
  mu[e] = acc;
}

// out[p][t][n] = sum_c sum_s B[p][t][c kin + s] in[(a>>1, 2b+c)][s][n]
template <typename VT, typename FT>
__global__ void k_apply_stage(const VT* __restrict__ in, VT* __restrict__ out,
                              const FT* __restrict__ blk, int L, int l, int kin, int kout,
                              int nrhs, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int n = (int)(e % nrhs);
  const int t = (int)((e / nrhs) % kout);
  const int64_t p = e / ((int64_t)nrhs * kout);
  const int sh = L - l;
  const int64_t a = p >> sh;
  const int64_t b = p & (((int64_t)1 << sh) - 1);
  const int64_t in0 = ((a >> 1) << (sh + 1)) | (2 * b);
  const FT* row = blk + (p * kout + t) * 2 * kin;
  VT acc = Zero<VT>::v();
  for (int c = 0; c < 2; ++c) {
    const VT* src = in + (in0 + c) * kin * nrhs + n;
    for (int s = 0; s < kin; ++s) cfma(acc, load_factor(row, c * kin + s), src[(int64_t)s * nrhs]);
  }
  out[e] = acc;
}

// Middle block of the swept-in factorization: out[p][t][n] = sum_s Mdot[p][t][s] in[p][s][n]
template <typename VT, typename FT>
__global__ void k_apply_mid(const VT* __restrict__ in, VT* __restrict__ out,
                            const FT* __restrict__ mdot, int kin, int kout, int nrhs,
                            int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int n = (int)(e % nrhs);
  const int t = (int)((e / nrhs) % kout);
  const int64_t p = e / ((int64_t)nrhs * kout);
  const FT* row = mdot + (p * kout + t) * kin;
  const VT* src = in + p * kin * nrhs + n;
  VT acc = Zero<VT>::v();
  for (int s = 0; s < kin; ++s) cfma(acc, load_factor(row, s), src[(int64_t)s * nrhs]);
  out[e] = acc;
}

// u[perm(x)][n] = sum_b sum_k Ubar[x][b][k] mu[(a(x), b)][k][n]
template <typename VT, typename FT>
__global__ void k_apply_u(const VT* __restrict__ mu, VT* __restrict__ u, int64_t ldu,
                          const int32_t* __restrict__ perm_x, const int32_t* __restrict__ xleaf,
                          const FT* __restrict__ ubar, int l0, int K, int nrhs, int64_t nx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nx * nrhs) return;
  const int64_t i = e % nx;
  const int n = (int)(e / nx);
  const int64_t a = xleaf[i];
  VT acc = Zero<VT>::v();
  const int nb = 1 << l0;
  for (int b = 0; b < nb; ++b) {
    const int64_t p = (a << l0) | b;
    const FT* urow = ubar + ((i << l0) | b) * K;
    const VT* m = mu + p * K * nrhs + n;
    for (int k = 0; k < K; ++k) cfma(acc, load_factor(urow, k), m[(int64_t)k * nrhs]);
  }
  u[(int64_t)n * ldu + perm_x[i]] = acc;
}

inline unsigned nblocks(int64_t total) { return (unsigned)((total + kBlock - 1) / kBlock); }

// Records a hipEvent pair around each launch when profiling is requested.
struct LaunchTimer {
  ibf_profile* prof;
  hipStream_t s;
  std::vector<hipEvent_t> ev;
  explicit LaunchTimer(ibf_profile* p, hipStream_t st) : prof(p), s(st) {}
  ~LaunchTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  int begin() {
    if (!prof) return IBF_OK;
    if (prof->n_launches >= IBF_PROFILE_MAX) return IBF_OK;
    hipEvent_t a;
    IBF_HIP_CHECK(hipEventCreate(&a));
    ev.push_back(a);
    IBF_HIP_CHECK(hipEventRecord(a, s));
    return IBF_OK;
  }
  int end(const char* name, double flops, double bytes) {
    if (!prof || prof->n_launches >= IBF_PROFILE_MAX) return IBF_OK;
    hipEvent_t b;
    IBF_HIP_CHECK(hipEventCreate(&b));
    ev.push_back(b);
    IBF_HIP_CHECK(hipEventRecord(b, s));
    const int i = prof->n_launches++;
    std::snprintf(prof->name[i], sizeof(prof->name[i]), "%s", name);
    prof->flops[i] = flops;
    prof->bytes[i] = bytes;
    return IBF_OK;
  }
  int finish() {
    if (!prof) return IBF_OK;
    IBF_HIP_CHECK(hipStreamSynchronize(s));
    for (int i = 0; i < prof->n_launches; ++i)
      IBF_HIP_CHECK(hipEventElapsedTime(&prof->ms[i], ev[2 * i], ev[2 * i + 1]));
    return IBF_OK;
  }
};

template <typename VT, typename FT>
int apply_t(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs64,
            hipStream_t s, ibf_profile* prof) {
  const Geo& geo = p->geo;
  const int L = geo.L, l0 = geo.l0;
  const int nrhs = (int)nrhs64;
  int kmax = 1;
  for (int k : p->rank) kmax = std::max(kmax, k);
  for (int k : p->rank_in_g) kmax = std::max(kmax, k);
  for (int k : p->rank_in_h) kmax = std::max(kmax, k);
  const size_t need = (size_t)p->npairs * kmax * nrhs * sizeof(VT);
  if (need > p->work_bytes) {
    for (int i = 0; i < 2; ++i) {
      if (p->d_work[i]) (void)hipFree(p->d_work[i]);
      p->d_work[i] = nullptr;
    }
    p->work_bytes = 0;
    IBF_HIP_CHECK(hipMalloc(&p->d_work[0], need));
    IBF_HIP_CHECK(hipMalloc(&p->d_work[1], need));
    p->work_bytes = need;
  }
  VT* w[2] = {(VT*)p->d_work[0], (VT*)p->d_work[1]};
  LaunchTimer T(prof, s);
  const double fb = (double)sizeof(FT), vb = (double)sizeof(VT);
  int rc;
  {
    const int64_t total = p->npairs * p->k_vbar * nrhs;
    if ((rc = T.begin())) return rc;
    hipLaunchKernelGGL((k_apply_v<VT, FT>), dim3(nblocks(total)), dim3(kBlock), 0, s,
                       (const VT*)g, ldg, p->d_perm_xi, p->d_xioff, (const FT*)p->d_vbar, w[0],
                       L, l0, p->k_vbar, nrhs, total);
    const double nnz = (double)p->nnz_vbar;
    if ((rc = T.end("apply_v", 8.0 * nnz * nrhs,
                    nnz * fb + vb * nrhs * ((double)p->nxi + (double)total / nrhs))))
      return rc;
  }
  int cur = 0;
  auto launch_mid = [&]() -> int {
    const int64_t total = p->npairs * p->k_mid_g * nrhs;
    int rc2;
    if ((rc2 = T.begin())) return rc2;
    hipLaunchKernelGGL((k_apply_mid<VT, FT>), dim3(nblocks(total)), dim3(kBlock), 0, s, w[cur],
                       w[cur ^ 1], (const FT*)p->d_mdot, p->k_mid_h, p->k_mid_g, nrhs, total);
    const double nnz = (double)p->npairs * p->k_mid_g * p->k_mid_h;
    const double vec = (double)p->npairs * (p->k_mid_g + p->k_mid_h) * nrhs * vb;
    if ((rc2 = T.end("apply_mid", 8.0 * nnz * nrhs, nnz * fb + vec))) return rc2;
    cur ^= 1;
    return IBF_OK;
  };
  if (p->d_mdot && geo.h == l0)
    if ((rc = launch_mid())) return rc;
  for (const Stage& st : p->stages) {
    const int64_t total = p->npairs * st.k_out * nrhs;
    if ((rc = T.begin())) return rc;
    hipLaunchKernelGGL((k_apply_stage<VT, FT>), dim3(nblocks(total)), dim3(kBlock), 0, s,
                       w[cur], w[cur ^ 1], (const FT*)st.blk, L, st.level_out, st.k_in,
                       st.k_out, nrhs, total);
    const double nnz = (double)st.nnz;
    const double vec = (double)p->npairs * (st.k_in + st.k_out) * nrhs * vb;
    if ((rc = T.end("apply_stage", 8.0 * nnz * nrhs, nnz * fb + vec))) return rc;
    cur ^= 1;
    if (p->d_mdot && st.level_out == geo.h)
      if ((rc = launch_mid())) return rc;
  }
  {
    const int64_t total = p->nx * nrhs;
    if ((rc = T.begin())) return rc;
    hipLaunchKernelGGL((k_apply_u<VT, FT>), dim3(nblocks(total)), dim3(kBlock), 0, s, w[cur],
                       (VT*)u, ldu, p->d_perm_x, p->d_xleaf, (const FT*)p->d_ubar, l0,
                       p->k_ubar, nrhs, p->nx);
    const double nnz = (double)p->nnz_ubar;
    if ((rc = T.end("apply_u", 8.0 * nnz * nrhs,
                    nnz * fb + vb * nrhs * ((double)p->nx + (double)p->npairs * p->k_ubar))))
      return rc;
  }
  IBF_HIP_CHECK(hipGetLastError());
  return T.finish();
}

}  // namespace

int apply_plan(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs,
               hipStream_t s, ibf_profile* prof) {
  IBF_HIP_CHECK(hipSetDevice(p->device));
  if (nrhs > (1 << 20)) {
    set_error("ibf_apply: nrhs too large");
    return IBF_ERR_INVALID_ARG;
  }
  switch (p->precision) {
    case IBF_FP64: return apply_t<double2, double2>(p, g, ldg, u, ldu, nrhs, s, prof);
    case IBF_FP32: return apply_t<float2, float2>(p, g, ldg, u, ldu, nrhs, s, prof);
    default: return apply_t<float2, bf16x2c>(p, g, ldg, u, ldu, nrhs, s, prof);
  }
}

}  // namespace ibf
