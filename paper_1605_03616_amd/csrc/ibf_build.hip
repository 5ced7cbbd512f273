// Device construction of the compressed IBF.
//
// Every factor entry comes from its explicit formula (paper Sec. 3) and is
// consumed immediately by the compression that needs it (Sec. 4), so the
// preliminary factorization is never stored:
//   k_middle   -- switch blocks M~ = exp(2 pi i Phi(g^A_t, g^B_s)) (eqn:switchlocM)
//                 and their truncated SVD M~ = C R^*, Sigma^(1/2) on both sides
//                 (eq:KeqUMV with eq:lowrankSVD).
//   k_sweep_g  -- per output pair, W = [G_0 C_{PC0}, G_1 C_{PC1}] built from
//                 eqn:PIBF3 and factored W = C' Gbar with C' = U_k Sigma_k,
//                 Gbar = V_k^* (eqn:GC, eq:lowrankSVD3).
//   k_sweep_h  -- per input pair, Z = [H^*_{A0B<-PC} R_{A0B}, H^*_{A1B<-PC} R_{A1B}]
//                 from eqn:PIBF2, factored Z = R' Hbar (eqn:HR).
//   k_ubar     -- Ubar = U C at the X leaves (eqn:PIBFbf3 times C^L).
//   k_vbar     -- Vbar^* = R^* V^* at the Omega leaves (eqn:PIBF1, eqn:V0).
// All arithmetic is FP64; the stored factors are converted to the plan's
// storage precision at the end (k_pack_stage / k_ubar / k_vbar).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "ibf_kern.h"

namespace ibf {
namespace {

using kern::kBlock;
using kern::SweepArgs;
using kern::block_accumulate;

// ---------------------------------------------------------------------------
// RAII device buffer for build temporaries.
// ---------------------------------------------------------------------------
template <typename T>
struct DevBuf {
  T* ptr = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), n(o.n) { o.ptr = nullptr; o.n = 0; }
  ~DevBuf() { if (ptr) (void)ibf::dev_free(ptr); }
  hipError_t alloc(size_t count) {
    n = count;
    return ibf::dev_malloc((void**)&ptr, std::max<size_t>(count, 1) * sizeof(T));
  }
};

// ---------------------------------------------------------------------------
// Chebyshev nodes z_t = cos(t pi/(r-1))/2 and the child -> parent Lagrange
// matrices Lc[c][t][s] = M_t((2c-1)/4 + z_s/2) (paper Sec. 2.1 / eqn:PIBF2).
// Layout of `cheb`: z[r] then Lc[2][r][r].
// ---------------------------------------------------------------------------
__global__ void k_cheb(int r, double* cheb) {
  __shared__ double z[kMaxR];
  const int tid = threadIdx.x;
  if (tid < r) z[tid] = 0.5 * cos((double)tid * M_PI / (double)(r - 1));
  __syncthreads();
  if (tid < r) cheb[tid] = z[tid];
  for (int e = tid; e < 2 * r * r; e += blockDim.x) {
    int c = e / (r * r), t = (e / r) % r, s = e % r;
    double y;
    {
#pragma clang fp contract(off)
      y = (double)(2 * c - 1) / 4.0 + z[s] / 2.0;
    }
    cheb[r + e] = lagrange_t(z, r, t, y);
  }
}

// ---------------------------------------------------------------------------
// Conversion of one stage from the FP64 r x 2r staging layout [pair][t][c r + s]
// to the stored layout [pair][c k_in + s][t < kld] (input-major: the k_out
// entries that multiply one input coefficient are contiguous; rows padded with
// zeros to the even length kld so that a pair's block copies in 16-byte units)
// in the storage precision.
// ---------------------------------------------------------------------------
template <typename FT>
__global__ void k_pack_stage(const double2* stage, FT* out, int64_t npairs, int R, int kout,
                             int kin, int kld) {
  const int64_t per = (int64_t)kld * 2 * kin;
  const int64_t total = npairs * per;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / per;
    const int rem = (int)(e - p * per);
    const int cc = rem / kld;
    const int t = rem - cc * kld;
    const int c = cc / kin, s = cc - c * kin;
    store_factor(out, e, t < kout ? stage[(p * R + t) * 2 * R + c * R + s] : make_double2(0, 0));
  }
}

// ---------------------------------------------------------------------------
// Ubar = U C at level L-l0: one thread per (X point i, T_Omega box b @ l0).
//   U[x][t] = exp(2 pi i Phi(x, c_B)) M^A_t(x) exp(-2 pi i Phi(g^A_t, c_B))
// stored as ubar[(i 2^l0 + b) K + k].
// ---------------------------------------------------------------------------
template <typename FT>
__global__ void k_ubar(PhaseDesc ph, Geo geo, const double* cheb, const double* xs,
                       const int32_t* xleaf, int64_t nx, const double2* C, const int* rk,
                       int K, FT* ubar, unsigned long long* nnz) {
  __shared__ double z[kMaxR];
  const int R = geo.r;
  for (int e = threadIdx.x; e < R; e += blockDim.x) z[e] = cheb[e];
  __syncthreads();
  const int l0 = geo.l0, L = geo.L, la = L - l0;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long add = 0;
  if (e < (nx << l0)) {
    const int64_t i = e >> l0;
    const int64_t b = e & ((1 << l0) - 1);
    const int64_t a = xleaf[i];
    const int64_t p = (a << l0) | b;
    const double cA = box_cx(la, a), wA = box_wx(la);
    const double cB = box_cxi(geo, l0, b);
    const double x = xs[i];
    const double y = norm_pt(x, cA, wA);
    const double2 e0 = kval(ph, x, cB);
    double2 acc[kMaxR];
#pragma unroll
    for (int k = 0; k < kMaxR; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int t = 0; t < R; ++t) {
      const double m = lagrange_t(z, R, t, y);
      const double2 ut = cscale(cmul(e0, conjd(kval(ph, grid_pt(cA, wA, z[t]), cB))), m);
      const double2* Ct = C + (p * R + t) * R;
#pragma unroll
      for (int k = 0; k < kMaxR; ++k)
        if (k < K) cfma(acc[k], ut, Ct[k]);
    }
#pragma unroll
    for (int k = 0; k < kMaxR; ++k)
      if (k < K) store_factor(ubar, e * K + k, acc[k]);
    add = (unsigned long long)rk[p];
  }
  // counter of unpadded Ubar entries: sum over (point, b) of rank(pair)
  __shared__ unsigned long long s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  __syncthreads();
  if (add) atomicAdd(&s_sum, add);
  __syncthreads();
  if (threadIdx.x == 0 && s_sum) atomicAdd(nnz, s_sum);
}

// ---------------------------------------------------------------------------
// Vbar^* = R^* V^* at level l0: one thread per (Omega point j, T_X box a @ l0).
//   V^*[t][xi] = exp(-2 pi i Phi(c_A, g^B_t)) M^B_t(xi) exp(2 pi i Phi(c_A, xi))
// stored as vbar[(j 2^l0 + a) K + k].
// ---------------------------------------------------------------------------
template <typename FT>
__global__ void k_vbar(PhaseDesc ph, Geo geo, const double* cheb, const double* xis,
                       const int32_t* xileaf, int64_t nxi, const double2* Rm, const int* rk,
                       int K, FT* vbar, unsigned long long* nnz) {
  __shared__ double z[kMaxR];
  const int R = geo.r;
  for (int e = threadIdx.x; e < R; e += blockDim.x) z[e] = cheb[e];
  __syncthreads();
  const int l0 = geo.l0, L = geo.L, lb = L - l0;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long add = 0;
  if (e < (nxi << l0)) {
    const int64_t j = e >> l0;
    const int64_t a = e & ((1 << l0) - 1);
    const int64_t b = xileaf[j];
    const int64_t p = (a << lb) | b;
    const double cA = box_cx(l0, a);
    const double cB = box_cxi(geo, lb, b), wB = box_wxi(geo, lb);
    const double xi = xis[j];
    const double y = norm_pt(xi, cB, wB);
    const double2 e0 = kval(ph, cA, xi);
    double2 acc[kMaxR];
#pragma unroll
    for (int k = 0; k < kMaxR; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int t = 0; t < R; ++t) {
      const double m = lagrange_t(z, R, t, y);
      const double2 vt = cscale(cmul(conjd(kval(ph, cA, grid_pt(cB, wB, z[t]))), e0), m);
      const double2* Rt = Rm + (p * R + t) * R;
#pragma unroll
      for (int k = 0; k < kMaxR; ++k)
        if (k < K) cfma(acc[k], conjd(Rt[k]), vt);
    }
#pragma unroll
    for (int k = 0; k < kMaxR; ++k)
      if (k < K) store_factor(vbar, e * K + k, acc[k]);
    add = (unsigned long long)rk[p];
  }
  __shared__ unsigned long long s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  __syncthreads();
  if (add) atomicAdd(&s_sum, add);
  __syncthreads();
  if (threadIdx.x == 0 && s_sum) atomicAdd(nnz, s_sum);
}


template <typename FT>
__global__ void k_sweepin_mid(int R, int64_t npairs, const double2* cbar, const double2* rbar,
                              const int* rkG, const int* rkH, int KG, int KH, FT* mdot,
                              unsigned long long* nnz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long add = 0;
  if (e < npairs * KG * KH) {
    const int64_t p = e / (KG * KH);
    const int rem = (int)(e - p * KG * KH);
    const int t = rem / KH, s = rem - t * KH;
    double2 acc = make_double2(0.0, 0.0);
    for (int m = 0; m < R; ++m)
      cfma(acc, cbar[(p * R + t) * R + m], rbar[(p * R + m) * R + s]);
    store_factor(mdot, e, acc);
    if (rem == 0) add = (unsigned long long)rkG[p] * (unsigned long long)rkH[p];
  }
  __shared__ unsigned long long s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  __syncthreads();
  if (add) atomicAdd(&s_sum, add);
  __syncthreads();
  if (threadIdx.x == 0 && s_sum) atomicAdd(nnz, s_sum);
}

// Packs an outer factor [point][2^l0][r] FP64 into [point][2^l0][K] storage.
template <typename FT>
__global__ void k_pack_outer(const double2* src, FT* dst, int64_t rows, int R, int K) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < rows * K) {
    const int64_t i = e / K;
    const int k = (int)(e - i * K);
    store_factor(dst, e, src[i * R + k]);
  }
}

// Unpadded entries of an outer factor: sum over (point, box) of rank(pair).
__global__ void k_count_outer(const int32_t* leaf_of, int64_t npts, int l0, int shift_leaf,
                              const int* rk, unsigned long long* nnz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long add = 0;
  if (e < (npts << l0)) {
    const int64_t i = e >> l0;
    const int64_t o = e & ((1 << l0) - 1);
    const int64_t leaf = leaf_of[i];
    // U side: pair = leaf 2^l0 + o ; V side: pair = o 2^(L-l0) + leaf
    const int64_t p = shift_leaf ? ((o << shift_leaf) | leaf) : ((leaf << l0) | o);
    add = (unsigned long long)rk[p];
  }
  __shared__ unsigned long long s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  __syncthreads();
  if (add) atomicAdd(&s_sum, add);
  __syncthreads();
  if (threadIdx.x == 0 && s_sum) atomicAdd(nnz, s_sum);
}

// Per-pair ranks of one level kept for the apply (bytes; ranks are <= 16).
__global__ void k_save_rank(const int* rk, uint8_t* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (uint8_t)rk[i];
}

__global__ void k_eval(PhaseDesc ph, const double* x, const double* xi, int64_t n, double2* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = kval(ph, x[i], xi[i]);
}


// The quad records of a BF16X2 stage (the layout of Stage::qblk): one thread
// per 16-byte record (pair, child c, quad q, float f) gathers the hi and lo
// bf16 parts of float f of rows 4q .. 4q+3 of child c's block rows.
__global__ __launch_bounds__(kBlock) void k_quad_split(const bf16x2c* __restrict__ blk,
                                                       uint4* __restrict__ q, int64_t npairs,
                                                       int k_in, int k_ld) {
  const int nq = (k_in + 3) / 4, nf = 2 * k_ld;
  const int64_t total = npairs * 2 * nq * nf;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int f = (int)(i % nf);
    const int64_t cq = i / nf;
    const int qq = (int)(cq % nq);
    const int64_t pc = cq / nq;                               // pair * 2 + child
    const int c = (int)(pc & 1);
    const int64_t pair = pc >> 1;
    const unsigned short* b = reinterpret_cast<const unsigned short*>(blk) +
                              pair * (int64_t)(2 * k_in * k_ld) * 4;
    unsigned h[4], l[4];
    for (int k = 0; k < 4; ++k) {
      const int s = 4 * qq + k;
      h[k] = l[k] = 0u;
      if (s < k_in) {
        const int64_t e = ((int64_t)(c * k_in + s) * k_ld + (f >> 1)) * 4 + (f & 1);
        h[k] = b[e];
        l[k] = b[e + 2];
      }
    }
    q[i] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), l[0] | (l[1] << 16),
                      l[2] | (l[3] << 16));
  }
}

template <typename FT>
int pack_all(ibf_plan_t p, const std::vector<DevBuf<double2>>& stages, const double2* Cu,
             const double2* Rv, const int* rkU, const int* rkV, const double* cheb,
             unsigned long long* nnz_u, unsigned long long* nnz_v, hipStream_t s) {
  const Geo& geo = p->geo;
  const int l0 = geo.l0, L = geo.L, R = p->r;
  const size_t fb = sizeof(FT);
  p->nnz_stored = 0;
  for (int l = l0 + 1; l <= L - l0; ++l) {
    Stage st;
    st.level_out = l;
    st.k_out = p->rank[l - l0];
    st.k_in = p->rank[l - 1 - l0];
    st.k_ld = (st.k_out + 1) & ~1;
    const int64_t count = p->npairs * st.k_ld * 2 * st.k_in;
    st.bytes = (size_t)count * fb;
    IBF_HIP_CHECK(ibf::dev_malloc(&st.blk, st.bytes + kStageSlack));
    p->stages.push_back(st);
    const unsigned blocks = (unsigned)std::min<int64_t>((count + kBlock - 1) / kBlock, 1 << 20);
    hipLaunchKernelGGL((k_pack_stage<FT>), dim3(std::max(blocks, 1u)), dim3(kBlock), 0, s,
                       stages[l - l0 - 1].ptr, (FT*)st.blk, p->npairs, R, st.k_out, st.k_in,
                       st.k_ld);
    p->nnz_stored += count;
    // quad records for the per-pair-rank stages with BF16 split products
    if (std::is_same<FT, bf16x2c>::value && p->d_prank) {
      const int rc = make_quad_records(p->stages.back(), p->npairs, s);
      if (rc) return rc;
    }
  }
  // Ubar at level L-l0, Vbar at level l0
  p->k_ubar = p->rank[L - l0 - l0];
  p->k_vbar = p->rank[0];
  p->ubar_bytes = (size_t)(p->nx << l0) * p->k_ubar * fb;
  p->vbar_bytes = (size_t)(p->nxi << l0) * p->k_vbar * fb;
  IBF_HIP_CHECK(ibf::dev_malloc(&p->d_ubar, std::max<size_t>(p->ubar_bytes, 1)));
  IBF_HIP_CHECK(ibf::dev_malloc(&p->d_vbar, std::max<size_t>(p->vbar_bytes, 1)));
  {
    const int64_t n = p->nx << l0;
    hipLaunchKernelGGL((k_ubar<FT>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, p->phase, geo, cheb, p->d_xs, p->d_xleaf, p->nx, Cu, rkU, p->k_ubar,
                       (FT*)p->d_ubar, nnz_u);
    p->nnz_stored += n * p->k_ubar;
  }
  {
    const int64_t n = p->nxi << l0;
    hipLaunchKernelGGL((k_vbar<FT>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, p->phase, geo, cheb, p->d_xis, p->d_xileaf, p->nxi, Rv, rkV, p->k_vbar,
                       (FT*)p->d_vbar, nnz_v);
    p->nnz_stored += n * p->k_vbar;
  }
  IBF_HIP_CHECK(hipGetLastError());
  return IBF_OK;
}

// Sweep-in (Sec. 4.3) on the FP64 sweep-out results, then conversion of all
// factors to the storage precision.  `stages` hold the sweep-out blocks in
// the r x 2r staging layout and are rewritten in place.
template <typename FT>
int sweep_in_pack(ibf_plan_t p, std::vector<DevBuf<double2>>& stages, const double2* Cu,
                  const double2* Rv, const int* rkU, const int* rkV, const double* cheb,
                  hipStream_t s) {
  const Geo& geo = p->geo;
  const int L = geo.L, l0 = geo.l0, h = geo.h, R = p->r;
  const int nlev = L - 2 * l0 + 1, nst = L - 2 * l0;
  const int64_t np = p->npairs;
  const size_t fb = sizeof(FT);
  if (p->smax_x > 64 || p->smax_xi > 64) {
    set_error("ibf_build: sweep-in needs leaves of at most 64 points");
    return IBF_ERR_UNSUPPORTED;
  }
  DevBuf<double2> ub, vb, ud, vd, cb[2], rb[2];
  IBF_HIP_CHECK(ub.alloc((size_t)(p->nx << l0) * R));
  IBF_HIP_CHECK(ud.alloc((size_t)(p->nx << l0) * R));
  IBF_HIP_CHECK(vb.alloc((size_t)(p->nxi << l0) * R));
  IBF_HIP_CHECK(vd.alloc((size_t)(p->nxi << l0) * R));
  DevBuf<int> rkg[2], rkh[2], rmax_g, rmax_h;
  for (int i = 0; i < 2; ++i) {
    IBF_HIP_CHECK(cb[i].alloc((size_t)np * R * R));
    IBF_HIP_CHECK(rb[i].alloc((size_t)np * R * R));
    IBF_HIP_CHECK(rkg[i].alloc(np));
    IBF_HIP_CHECK(rkh[i].alloc(np));
  }
  IBF_HIP_CHECK(rmax_g.alloc(nlev));
  IBF_HIP_CHECK(rmax_h.alloc(nlev));
  DevBuf<unsigned long long> cnt, scratch;
  IBF_HIP_CHECK(cnt.alloc(nst + 3));
  IBF_HIP_CHECK(scratch.alloc(1));
  IBF_HIP_CHECK(hipMemsetAsync(rmax_g.ptr, 0, nlev * sizeof(int), s));
  IBF_HIP_CHECK(hipMemsetAsync(rmax_h.ptr, 0, nlev * sizeof(int), s));
  IBF_HIP_CHECK(hipMemsetAsync(cnt.ptr, 0, (nst + 3) * sizeof(unsigned long long), s));

  // outer factors in FP64 at width r
  {
    const int64_t n = p->nx << l0;
    hipLaunchKernelGGL((k_ubar<double2>), dim3((unsigned)((n + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, p->phase, geo, cheb, p->d_xs, p->d_xleaf, p->nx, Cu,
                       rkU, R, ub.ptr, scratch.ptr);
  }
  {
    const int64_t n = p->nxi << l0;
    hipLaunchKernelGGL((k_vbar<double2>), dim3((unsigned)((n + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, p->phase, geo, cheb, p->d_xis, p->d_xileaf, p->nxi, Rv,
                       rkV, R, vb.ptr, scratch.ptr);
  }
  // U side inward
  kern::sweepin_u(R, geo, p->tol, p->d_xoff, ub.ptr, ud.ptr, cb[0].ptr,
                 rkg[0].ptr, rmax_g.ptr + (L - 2 * l0), s);
  {
    const int64_t n = p->nx << l0;
    hipLaunchKernelGGL(k_count_outer, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, p->d_xleaf, p->nx, l0, 0, rkg[0].ptr, cnt.ptr + nst + 1);
  }
  int cg = 0;
  for (int l = L - l0; l > h; --l) {
    kern::sweepin_g(R, geo, p->tol, l, cb[cg].ptr, cb[cg ^ 1].ptr,
                   stages[l - l0 - 1].ptr, rkg[cg].ptr, rkg[cg ^ 1].ptr,
                   rmax_g.ptr + (l - 1 - l0), cnt.ptr + (l - l0 - 1), s);
    cg ^= 1;
  }
  // V side inward
  kern::sweepin_v(R, geo, p->tol, p->d_xioff, vb.ptr, vd.ptr, rb[0].ptr,
                 rkh[0].ptr, rmax_h.ptr, s);
  {
    const int64_t n = p->nxi << l0;
    hipLaunchKernelGGL(k_count_outer, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, p->d_xileaf, p->nxi, l0, L - l0, rkh[0].ptr, cnt.ptr + nst + 2);
  }
  int ch = 0;
  for (int l = l0 + 1; l <= h; ++l) {
    kern::sweepin_h(R, geo, p->tol, l, rb[ch].ptr, rb[ch ^ 1].ptr,
                   stages[l - l0 - 1].ptr, rkh[ch].ptr, rkh[ch ^ 1].ptr, rmax_h.ptr + (l - l0),
                   cnt.ptr + (l - l0 - 1), s);
    ch ^= 1;
  }
  IBF_HIP_CHECK(hipGetLastError());
  std::vector<int> rg(nlev), rh(nlev);
  IBF_HIP_CHECK(hipMemcpyAsync(rg.data(), rmax_g.ptr, nlev * sizeof(int), hipMemcpyDeviceToHost, s));
  IBF_HIP_CHECK(hipMemcpyAsync(rh.data(), rmax_h.ptr, nlev * sizeof(int), hipMemcpyDeviceToHost, s));
  IBF_HIP_CHECK(hipStreamSynchronize(s));
  for (auto& k : rg) k = std::max(k, 1);
  for (auto& k : rh) k = std::max(k, 1);
  p->rank_in_g = rg;
  p->rank_in_h = rh;

  p->nnz_stored = 0;
  for (int l = l0 + 1; l <= L - l0; ++l) {
    const std::vector<int>& rk = (l <= h) ? rh : rg;
    Stage st;
    st.level_out = l;
    st.k_out = rk[l - l0];
    st.k_in = rk[l - 1 - l0];
    st.nnz = 0;
    st.k_ld = (st.k_out + 1) & ~1;
    const int64_t count = np * st.k_ld * 2 * st.k_in;
    st.bytes = (size_t)count * fb;
    IBF_HIP_CHECK(ibf::dev_malloc(&st.blk, std::max<size_t>(st.bytes, 1)));
    p->stages.push_back(st);
    const unsigned blocks = (unsigned)std::min<int64_t>((count + kBlock - 1) / kBlock, 1 << 20);
    hipLaunchKernelGGL((k_pack_stage<FT>), dim3(std::max(blocks, 1u)), dim3(kBlock), 0, s,
                       stages[l - l0 - 1].ptr, (FT*)st.blk, np, R, st.k_out, st.k_in, st.k_ld);
    p->nnz_stored += count;
  }
  p->k_mid_g = rg[h - l0];
  p->k_mid_h = rh[h - l0];
  {
    const int64_t count = np * p->k_mid_g * p->k_mid_h;
    p->mdot_bytes = (size_t)count * fb;
    IBF_HIP_CHECK(ibf::dev_malloc(&p->d_mdot, std::max<size_t>(p->mdot_bytes, 1)));
    hipLaunchKernelGGL((k_sweepin_mid<FT>), dim3((unsigned)((count + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, R, np, cb[cg].ptr, rb[ch].ptr, rkg[cg].ptr,
                       rkh[ch].ptr, p->k_mid_g, p->k_mid_h, (FT*)p->d_mdot, cnt.ptr + nst);
    p->nnz_stored += count;
  }
  p->k_ubar = rg[L - 2 * l0];
  p->k_vbar = rh[0];
  p->ubar_bytes = (size_t)(p->nx << l0) * p->k_ubar * fb;
  p->vbar_bytes = (size_t)(p->nxi << l0) * p->k_vbar * fb;
  IBF_HIP_CHECK(ibf::dev_malloc(&p->d_ubar, std::max<size_t>(p->ubar_bytes, 1)));
  IBF_HIP_CHECK(ibf::dev_malloc(&p->d_vbar, std::max<size_t>(p->vbar_bytes, 1)));
  {
    const int64_t rows = p->nx << l0;
    hipLaunchKernelGGL((k_pack_outer<FT>),
                       dim3((unsigned)((rows * p->k_ubar + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, ud.ptr, (FT*)p->d_ubar, rows, R, p->k_ubar);
    p->nnz_stored += rows * p->k_ubar;
  }
  {
    const int64_t rows = p->nxi << l0;
    hipLaunchKernelGGL((k_pack_outer<FT>),
                       dim3((unsigned)((rows * p->k_vbar + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, vd.ptr, (FT*)p->d_vbar, rows, R, p->k_vbar);
    p->nnz_stored += rows * p->k_vbar;
  }
  IBF_HIP_CHECK(hipGetLastError());
  std::vector<unsigned long long> nn(nst + 3);
  IBF_HIP_CHECK(hipMemcpyAsync(nn.data(), cnt.ptr, nn.size() * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s));
  IBF_HIP_CHECK(hipStreamSynchronize(s));
  p->nnz_opt = 0;
  for (int i = 0; i < nst; ++i) {
    p->stages[i].nnz = (int64_t)nn[i];
    p->nnz_opt += (int64_t)nn[i];
  }
  p->nnz_ubar = (int64_t)nn[nst + 1];
  p->nnz_vbar = (int64_t)nn[nst + 2];
  p->nnz_opt += (int64_t)(nn[nst] + nn[nst + 1] + nn[nst + 2]);
  return IBF_OK;
}

template <typename T>
int upload(T** dst, const std::vector<T>& src) {
  if (*dst) return IBF_OK;
  IBF_HIP_CHECK(ibf::dev_malloc((void**)dst, std::max<size_t>(src.size(), 1) * sizeof(T)));
  if (!src.empty())
    IBF_HIP_CHECK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return IBF_OK;
}

}  // namespace

int make_quad_records(Stage& st, int64_t npairs, hipStream_t s) {
  const int64_t nrec = npairs * 2 * ((st.k_in + 3) / 4) * 2 * st.k_ld;
  st.qbytes = (size_t)nrec * sizeof(uint4);
  // + slack: with a stored input rank of 0 the clamped record loads of the
  // stage kernel read the first 32 records of the buffer
  IBF_HIP_CHECK(ibf::dev_malloc(&st.qblk, st.qbytes + kStageSlack));
  const unsigned qb = (unsigned)std::min<int64_t>((nrec + kBlock - 1) / kBlock, 1 << 20);
  hipLaunchKernelGGL(k_quad_split, dim3(std::max(qb, 1u)), dim3(kBlock), 0, s,
                     (const bf16x2c*)st.blk, (uint4*)st.qblk, npairs, st.k_in, st.k_ld);
  IBF_HIP_CHECK(hipGetLastError());
  return IBF_OK;
}

int build_plan(ibf_plan_t p, hipStream_t s) {
  IBF_HIP_CHECK(hipSetDevice(p->device));
  free_factors(p);
  int rc;
  if (p->learned && p->r == 0) {
    // order and truncation from the learned error model (a plan with no
    // predictor, or no qualifying candidate, falls back to r = 12 at tol)
    int r = 0;
    double st = p->target_tol;
    if (p->predictor) {
      rc = ibf_mlp_select(p->predictor, p->predictor_hidden, p->nxi, p->phase.kind, p->target_tol,
                          0.3, 2, kMaxR, &r, &st, s);
      if (rc) return rc;
    }
    if (r == 0) {
      r = 12;
      st = p->target_tol;
    }
    set_order(p, r, st);
  }
  if ((rc = upload(&p->d_xs, p->xs)) || (rc = upload(&p->d_xis, p->xis)) ||
      (rc = upload(&p->d_perm_x, p->perm_x)) || (rc = upload(&p->d_perm_xi, p->perm_xi)) ||
      (rc = upload(&p->d_xoff, p->xoff)) || (rc = upload(&p->d_xioff, p->xioff)) ||
      (rc = upload(&p->d_xleaf, p->xleaf)) || (rc = upload(&p->d_xileaf, p->xileaf)))
    return rc;

  const Geo geo = p->geo;
  const int L = geo.L, l0 = geo.l0, h = geo.h, R = p->r;
  const int nlev = L - 2 * l0 + 1;
  const int nst = L - 2 * l0;
  const int64_t np = p->npairs;

  DevBuf<double> cheb;
  IBF_HIP_CHECK(cheb.alloc(R + 2 * R * R));
  hipLaunchKernelGGL(k_cheb, dim3(1), dim3(256), 0, s, R, cheb.ptr);

  DevBuf<double2> Cb[2], Rb[2];
  DevBuf<int> rk_mid, rkG[2], rkH[2], rank_max;
  // unpadded-entry counters: [stage 0 .. nst-1], [nst] middle, [nst+1] ubar, [nst+2] vbar
  DevBuf<unsigned long long> nnz;
  for (int i = 0; i < 2; ++i) {
    IBF_HIP_CHECK(Cb[i].alloc((size_t)np * R * R));
    IBF_HIP_CHECK(Rb[i].alloc((size_t)np * R * R));
    IBF_HIP_CHECK(rkG[i].alloc(np));
    IBF_HIP_CHECK(rkH[i].alloc(np));
  }
  IBF_HIP_CHECK(rk_mid.alloc(np));
  IBF_HIP_CHECK(rank_max.alloc(nlev));
  IBF_HIP_CHECK(nnz.alloc(nst + 3));
  IBF_HIP_CHECK(hipMemsetAsync(rank_max.ptr, 0, nlev * sizeof(int), s));
  IBF_HIP_CHECK(hipMemsetAsync(nnz.ptr, 0, (nst + 3) * sizeof(unsigned long long), s));
  std::vector<DevBuf<double2>> stages(nst);
  for (int i = 0; i < nst; ++i) IBF_HIP_CHECK(stages[i].alloc((size_t)np * R * 2 * R));

  SweepArgs A{p->phase, geo, cheb.ptr, p->tol, np, rank_max.ptr, nnz.ptr + nst,
              p->caps.empty() ? nullptr : p->caps.data()};
  // per-pair ranks of every level, kept for the apply when no sweep-in follows
  uint8_t* prank = nullptr;
  if (!p->sweep_in) IBF_HIP_CHECK(ibf::dev_malloc(&prank, (size_t)nlev * np));
  p->d_prank = prank;
  auto save_rank = [&](const int* rk, int level) {
    if (prank)
      hipLaunchKernelGGL(k_save_rank, dim3((unsigned)((np + kBlock - 1) / kBlock)), dim3(kBlock),
                         0, s, rk, prank + (size_t)(level - l0) * np, np);
  };
  kern::middle(R, A, Cb[0].ptr, Rb[0].ptr, rk_mid.ptr, s);
  save_rank(rk_mid.ptr, h);

  // sweep toward U
  const double2* Ccur = Cb[0].ptr;
  const int* rkcur = rk_mid.ptr;
  int gi = 0;
  double2* Cout_last = Cb[0].ptr;
  const int* rkU = rk_mid.ptr;
  for (int l = h + 1; l <= L - l0; ++l) {
    double2* Cout = (Ccur == Cb[0].ptr) ? Cb[1].ptr : Cb[0].ptr;
    int* rkout = rkG[gi].ptr;
    kern::sweep_g(R, A, l, Ccur, Cout, stages[l - l0 - 1].ptr, rkcur, rkout,
                   nnz.ptr + (l - l0 - 1), s);
    save_rank(rkout, l);
    Ccur = Cout;
    Cout_last = Cout;
    rkcur = rkout;
    rkU = rkout;
    gi ^= 1;
  }
  // sweep toward V
  const double2* Rcur = Rb[0].ptr;
  rkcur = rk_mid.ptr;
  const int* rkV = rk_mid.ptr;
  int hi = 0;
  double2* Rout_last = Rb[0].ptr;
  for (int l = h; l >= l0 + 1; --l) {
    double2* Rout = (Rcur == Rb[0].ptr) ? Rb[1].ptr : Rb[0].ptr;
    int* rkout = rkH[hi].ptr;
    kern::sweep_h(R, A, l, Rcur, Rout, stages[l - l0 - 1].ptr, rkcur, rkout,
                   nnz.ptr + (l - l0 - 1), s);
    save_rank(rkout, l - 1);
    Rcur = Rout;
    Rout_last = Rout;
    rkcur = rkout;
    rkV = rkout;
    hi ^= 1;
  }
  IBF_HIP_CHECK(hipGetLastError());

  std::vector<int> rk_host(nlev);
  IBF_HIP_CHECK(hipMemcpyAsync(rk_host.data(), rank_max.ptr, nlev * sizeof(int),
                               hipMemcpyDeviceToHost, s));
  IBF_HIP_CHECK(hipStreamSynchronize(s));
  for (auto& k : rk_host) k = std::max(k, 1);
  p->rank = rk_host;
  p->rank_in_g.clear();
  p->rank_in_h.clear();

  if (p->sweep_in) {
    if (p->precision == IBF_FP64)
      rc = sweep_in_pack<double2>(p, stages, Cout_last, Rout_last, rkU, rkV, cheb.ptr, s);
    else if (p->precision == IBF_FP32)
      rc = sweep_in_pack<float2>(p, stages, Cout_last, Rout_last, rkU, rkV, cheb.ptr, s);
    else
      rc = sweep_in_pack<bf16x2c>(p, stages, Cout_last, Rout_last, rkU, rkV, cheb.ptr, s);
    if (rc) return rc;
    p->built = true;
    return IBF_OK;
  }

  if (p->precision == IBF_FP64)
    rc = pack_all<double2>(p, stages, Cout_last, Rout_last, rkU, rkV, cheb.ptr,
                           nnz.ptr + nst + 1, nnz.ptr + nst + 2, s);
  else if (p->precision == IBF_FP32)
    rc = pack_all<float2>(p, stages, Cout_last, Rout_last, rkU, rkV, cheb.ptr,
                          nnz.ptr + nst + 1, nnz.ptr + nst + 2, s);
  else
    rc = pack_all<bf16x2c>(p, stages, Cout_last, Rout_last, rkU, rkV, cheb.ptr,
                           nnz.ptr + nst + 1, nnz.ptr + nst + 2, s);
  if (rc) return rc;
  std::vector<unsigned long long> nn(nst + 3);
  IBF_HIP_CHECK(hipMemcpyAsync(nn.data(), nnz.ptr, nn.size() * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s));
  IBF_HIP_CHECK(hipStreamSynchronize(s));
  p->nnz_opt = 0;
  for (int i = 0; i < nst; ++i) {
    p->stages[i].nnz = (int64_t)nn[i];
    p->nnz_opt += (int64_t)nn[i];
  }
  p->nnz_ubar = (int64_t)nn[nst + 1];
  p->nnz_vbar = (int64_t)nn[nst + 2];
  p->nnz_opt += (int64_t)(nn[nst] + nn[nst + 1] + nn[nst + 2]);
  p->built = true;
  return IBF_OK;
}

// Direct product u(x_i) = sum_j K(x_i, xi_j) g_j in FP64 (the plain definition
// the factorization approximates): one thread per (row, right-hand side).
__global__ __launch_bounds__(256) void k_dense(PhaseDesc ph, const double* __restrict__ x,
                                               int64_t nx, const double* __restrict__ xi,
                                               int64_t nxi, const double2* __restrict__ g,
                                               int64_t ldg, double2* __restrict__ u, int64_t ldu) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i >= nx) return;
  const double xv = x[i];
  const double2* gc = g + c * ldg;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t j = 0; j < nxi; ++j) {
    const double2 k = kval(ph, xv, xi[j]);
    const double2 gv = gc[j];
    acc.x = fma(k.x, gv.x, fma(-k.y, gv.y, acc.x));
    acc.y = fma(k.x, gv.y, fma(k.y, gv.x, acc.y));
  }
  u[c * ldu + i] = acc;
}

int dense_apply(const PhaseDesc& ph, const double* x, int64_t nx, const double* xi, int64_t nxi,
                const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_dense, dim3((unsigned)((nx + 255) / 256), (unsigned)nrhs), dim3(256), 0, s,
                     ph, x, nx, xi, nxi, (const double2*)g, ldg, (double2*)u, ldu);
  IBF_HIP_CHECK(hipGetLastError());
  return IBF_OK;
}

// Squared norms for the relative error of eq:relativeerr: per column c,
// acc[2c] += sum |u - ref|^2 and acc[2c+1] += sum |ref|^2 over this block's
// rows (FP64 sums of the block, one atomic per block and column).
template <typename T>
__global__ __launch_bounds__(256) void k_err_sums(const T* __restrict__ u, int64_t ldu,
                                                  const T* __restrict__ ref, int64_t ldr,
                                                  int64_t n, double* acc) {
  const int64_t c = blockIdx.y;
  double d2 = 0.0, r2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T a = u[c * ldu + i], b = ref[c * ldr + i];
    const double dx = (double)a.x - (double)b.x, dy = (double)a.y - (double)b.y;
    d2 += dx * dx + dy * dy;
    r2 += (double)b.x * (double)b.x + (double)b.y * (double)b.y;
  }
  __shared__ double sd[256], sr[256];
  sd[threadIdx.x] = d2;
  sr[threadIdx.x] = r2;
  __syncthreads();
  for (int m = 128; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m) {
      sd[threadIdx.x] += sd[threadIdx.x + m];
      sr[threadIdx.x] += sr[threadIdx.x + m];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&acc[2 * c], sd[0]);
    atomicAdd(&acc[2 * c + 1], sr[0]);
  }
}

int rel_error(const void* u, int64_t ldu, const void* ref, int64_t ldr, int64_t n, int64_t nrhs,
              int precision, double* out, hipStream_t s) {
  DevBuf<double> acc;
  IBF_HIP_CHECK(acc.alloc((size_t)2 * nrhs));
  IBF_HIP_CHECK(hipMemsetAsync(acc.ptr, 0, sizeof(double) * 2 * nrhs, s));
  const unsigned bx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
  if (n > 0) {
    if (precision == IBF_FP64)
      hipLaunchKernelGGL((k_err_sums<double2>), dim3(bx, (unsigned)nrhs), dim3(256), 0, s,
                         (const double2*)u, ldu, (const double2*)ref, ldr, n, acc.ptr);
    else
      hipLaunchKernelGGL((k_err_sums<float2>), dim3(bx, (unsigned)nrhs), dim3(256), 0, s,
                         (const float2*)u, ldu, (const float2*)ref, ldr, n, acc.ptr);
    IBF_HIP_CHECK(hipGetLastError());
  }
  std::vector<double> h((size_t)2 * nrhs);
  IBF_HIP_CHECK(hipMemcpyAsync(h.data(), acc.ptr, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  IBF_HIP_CHECK(hipStreamSynchronize(s));
  double d2 = 0.0, r2 = 0.0, cmax = 0.0;
  for (int64_t c = 0; c < nrhs; ++c) {
    d2 += h[2 * c];
    r2 += h[2 * c + 1];
    const double e = h[2 * c + 1] > 0 ? std::sqrt(h[2 * c] / h[2 * c + 1]) : (h[2 * c] > 0 ? INFINITY : 0.0);
    cmax = std::max(cmax, e);
  }
  out[0] = r2 > 0 ? std::sqrt(d2 / r2) : (d2 > 0 ? INFINITY : 0.0);
  out[1] = cmax;
  return IBF_OK;
}

int eval_kernel(const PhaseDesc& ph, const double* x, const double* xi, int64_t n, void* out,
                hipStream_t s) {
  hipLaunchKernelGGL(k_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ph, x, xi, n,
                     (double2*)out);
  IBF_HIP_CHECK(hipGetLastError());
  return IBF_OK;
}

}  // namespace ibf

