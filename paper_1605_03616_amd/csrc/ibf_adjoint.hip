// Adjoint apply (ibf_apply_adjoint): v = K_IBF^* h.  With the pair labels
// transposed, (a, b) at level l <-> (b, a) at level L - l, the adjoint
// V^* H^* ... Mdot^* ... G^* U^* of the factorization (Sec. 4, eqn:IBFout /
// eqn:IBFin) is again a forward factorization: its V is conj(Ubar), its U is
// conj(Vbar), its points are the plan's with X and Omega exchanged, its stage
// with output level l' gathers, for output pair (A, B), the conjugate-
// transposed slices of the two forward blocks (2B + d, A >> 1), d = 0, 1, of
// the forward stage with output level L - l' + 1, and its middle block (at
// level L - h) is the conjugate transpose of Mdot at the transposed pair.  The
// transposed copies (with the per-pair ranks at the transposed labels, and
// the quad records of BF16X2 stages) are made on the first adjoint apply and
// run on the forward apply kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <type_traits>

#include "ibf_device.h"

namespace ibf {
namespace {
constexpr int kAdjBlock = 256;

// dst[e] = conj(src[e])
template <typename FT>
__global__ __launch_bounds__(kAdjBlock) void k_adjoint_conj(const FT* __restrict__ src,
                                                         FT* __restrict__ dst, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const auto v = load_factor(src, e);
  store_factor(dst, e, make_double2((double)v.x, -(double)v.y));
}

// adjoint stage block (A, B) at level lp: [d kin_a + t][kld_a], kin_a = the
// forward k_out, columns s < the forward k_in (zero beyond)
template <typename FT>
__global__ __launch_bounds__(kAdjBlock) void k_adjoint_stage(const FT* __restrict__ src,
                                                          FT* __restrict__ dst, int L, int lp,
                                                          int kin_f, int kout_f, int kld_f,
                                                          int kld_a, int64_t npairs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int rows = 2 * kout_f;
  if (e >= npairs * rows * kld_a) return;
  const int col = (int)(e % kld_a);
  const int row = (int)((e / kld_a) % rows);
  const int64_t pa = e / ((int64_t)kld_a * rows);
  const int d = row / kout_f, t = row - d * kout_f;
  const int sh = L - lp;                                      // bits of B
  const int64_t A = pa >> sh, B = pa & (((int64_t)1 << sh) - 1);
  // forward output level lf = L - lp + 1: pair (a, b), a = 2B + d, b = A >> 1
  const int64_t pf = ((2 * B + d) << (lp - 1)) | (A >> 1);
  const int c = (int)(A & 1);
  double2 v = make_double2(0.0, 0.0);
  if (col < kin_f) {
    const auto f =
        load_factor(src, pf * (2 * (int64_t)kin_f) * kld_f + (int64_t)(c * kin_f + col) * kld_f + t);
    v = make_double2((double)f.x, -(double)f.y);
  }
  store_factor(dst, e, v);
}

// adjoint middle block at transposed pair pa = A 2^h + B (A: L - h bits,
// B: h bits): [i < kh][j < kg] = conj(Mdot[B 2^(L-h) + A][j][i])
template <typename FT>
__global__ __launch_bounds__(kAdjBlock) void k_adjoint_mid(const FT* __restrict__ src,
                                                        FT* __restrict__ dst, int L, int h,
                                                        int kg, int kh, int64_t npairs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= npairs * kg * kh) return;
  const int j = (int)(e % kg);
  const int i = (int)((e / kg) % kh);
  const int64_t pa = e / ((int64_t)kg * kh);
  const int64_t A = pa >> h, B = pa & (((int64_t)1 << h) - 1);
  const int64_t pf = (B << (L - h)) | A;
  const auto f = load_factor(src, (pf * kg + j) * kh + i);
  store_factor(dst, e, make_double2((double)f.x, -(double)f.y));
}

// Per-pair ranks of the adjoint plan: its pair p' = A 2^l + B at level
// L - l (A: L - l bits, B: l bits) is the forward pair B 2^(L-l) + A at
// level l, whose coefficients have the same rank.
__global__ __launch_bounds__(kAdjBlock) void k_adjoint_prank(const uint8_t* __restrict__ src,
                                                          uint8_t* __restrict__ dst, int L,
                                                          int l0, int nlev, int64_t npairs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nlev * npairs) return;
  const int li = (int)(e / npairs);
  const int64_t pa = e - (int64_t)li * npairs;
  const int l = L - (l0 + li);                                // forward level
  const int64_t A = pa >> l, B = pa & (((int64_t)1 << l) - 1);
  dst[e] = src[(int64_t)(l - l0) * npairs + ((B << (L - l)) | A)];
}

}  // namespace

template <typename FT>
int make_adjoint_t(ibf_plan_t p, hipStream_t s) {
  const Geo& geo = p->geo;
  const int L = geo.L, l0 = geo.l0;
  auto a = new ibf_plan_s();
  a->dim = 1;
  a->nx = p->nxi;
  a->nxi = p->nx;
  a->device = p->device;
  a->phase = p->phase;
  a->r = p->r;
  a->leaf = p->leaf;
  a->precision = p->precision;
  a->tol = p->tol;
  a->geo = geo;
  a->geo.h = L - geo.h;
  a->npairs = p->npairs;
  a->nleaf = p->nleaf;
  a->smax_x = p->smax_xi;
  a->smax_xi = p->smax_x;
  a->d_xs = p->d_xis;
  a->d_xis = p->d_xs;
  a->d_perm_x = p->d_perm_xi;
  a->d_perm_xi = p->d_perm_x;
  a->d_xoff = p->d_xioff;
  a->d_xioff = p->d_xoff;
  a->d_xleaf = p->d_xileaf;
  a->d_xileaf = p->d_xleaf;
  a->rank.assign(p->rank.rbegin(), p->rank.rend());
  // sweep-in: the two sides exchange (and reverse) their ranks
  a->rank_in_h.assign(p->rank_in_g.rbegin(), p->rank_in_g.rend());
  a->rank_in_g.assign(p->rank_in_h.rbegin(), p->rank_in_h.rend());
  a->k_mid_g = p->k_mid_h;
  a->k_mid_h = p->k_mid_g;
  a->k_vbar = p->k_ubar;
  a->k_ubar = p->k_vbar;
  a->nnz_vbar = p->nnz_ubar;
  a->nnz_ubar = p->nnz_vbar;
  a->vbar_bytes = p->ubar_bytes;
  a->ubar_bytes = p->vbar_bytes;
  p->adj = a;                                                 // freed by free_adjoint on error
  auto conj_copy = [&](const void* src, void** dst, size_t bytes) -> int {
    IBF_HIP_CHECK(ibf::dev_malloc(dst, std::max<size_t>(bytes, 1)));
    const int64_t n = (int64_t)(bytes / sizeof(FT));
    if (n > 0)
      hipLaunchKernelGGL((k_adjoint_conj<FT>), dim3((unsigned)((n + kAdjBlock - 1) / kAdjBlock)),
                         dim3(kAdjBlock), 0, s, (const FT*)src, (FT*)*dst, n);
    IBF_HIP_CHECK(hipGetLastError());
    return IBF_OK;
  };
  int rc;
  if ((rc = conj_copy(p->d_ubar, &a->d_vbar, p->ubar_bytes))) return rc;
  if ((rc = conj_copy(p->d_vbar, &a->d_ubar, p->vbar_bytes))) return rc;
  for (int lp = l0 + 1; lp <= L - l0; ++lp) {
    const Stage& f = p->stages[(L - lp + 1) - l0 - 1];
    Stage st{};
    st.level_out = lp;
    st.k_out = f.k_in;
    st.k_in = f.k_out;
    st.k_ld = (st.k_out + 1) & ~1;
    st.nnz = f.nnz;
    st.bytes = (size_t)p->npairs * 2 * st.k_in * st.k_ld * sizeof(FT);
    a->stages.push_back(st);
    Stage& sa = a->stages.back();
    // + the stage slack: the per-pair-rank stage kernel reads whole rows past
    // a block's last row (as for the forward plan's blocks)
    IBF_HIP_CHECK(ibf::dev_malloc(&sa.blk, sa.bytes + kStageSlack));
    const int64_t n = (int64_t)p->npairs * 2 * st.k_in * st.k_ld;
    hipLaunchKernelGGL((k_adjoint_stage<FT>), dim3((unsigned)((n + kAdjBlock - 1) / kAdjBlock)),
                       dim3(kAdjBlock), 0, s, (const FT*)f.blk, (FT*)sa.blk, L, lp, f.k_in, f.k_out,
                       f.k_ld, st.k_ld, p->npairs);
    IBF_HIP_CHECK(hipGetLastError());
    // BF16X2 without the sweep-in: quad records for the BF16 split products
    if (std::is_same<FT, bf16x2c>::value && p->d_prank) {
      const int rc2 = make_quad_records(sa, p->npairs, s);
      if (rc2) return rc2;
    }
  }
  if (p->d_prank) {
    // the forward per-pair ranks at the transposed labels: the adjoint runs on
    // the per-pair-rank stage kernels as the forward apply does
    const int nlev = L - 2 * l0 + 1;
    const int64_t n = (int64_t)nlev * p->npairs;
    IBF_HIP_CHECK(ibf::dev_malloc(reinterpret_cast<void**>(&a->d_prank), (size_t)n));
    hipLaunchKernelGGL(k_adjoint_prank, dim3((unsigned)((n + kAdjBlock - 1) / kAdjBlock)),
                       dim3(kAdjBlock), 0, s, p->d_prank, a->d_prank, L, l0, nlev, p->npairs);
    IBF_HIP_CHECK(hipGetLastError());
  }
  if (p->d_mdot) {
    a->mdot_bytes = p->mdot_bytes;
    IBF_HIP_CHECK(ibf::dev_malloc(&a->d_mdot, std::max<size_t>(a->mdot_bytes, 1)));
    const int64_t n = p->npairs * p->k_mid_g * p->k_mid_h;
    if (n > 0)
      hipLaunchKernelGGL((k_adjoint_mid<FT>), dim3((unsigned)((n + kAdjBlock - 1) / kAdjBlock)),
                         dim3(kAdjBlock), 0, s, (const FT*)p->d_mdot, (FT*)a->d_mdot, L, geo.h,
                         p->k_mid_g, p->k_mid_h, p->npairs);
    IBF_HIP_CHECK(hipGetLastError());
  }
  a->built = true;
  return IBF_OK;
}

void free_adjoint(ibf_plan_t p) {
  ibf_plan_s* a = p->adj;
  if (!a) return;
  for (auto& st : a->stages) {
    if (st.blk) (void)ibf::dev_free(st.blk);
    if (st.qblk) (void)ibf::dev_free(st.qblk);
  }
  void* own[] = {a->d_vbar, a->d_ubar, a->d_mdot, a->d_work[0], a->d_work[1], a->d_prank};
  for (void* b : own)
    if (b) (void)ibf::dev_free(b);
  delete a;                                                   // the point maps are p's
  p->adj = nullptr;
}

int apply_adjoint(ibf_plan_t p, const void* h, int64_t ldh, void* v, int64_t ldv, int64_t nrhs,
                  hipStream_t s) {
  IBF_HIP_CHECK(hipSetDevice(p->device));
  if (!p->adj) {
    int rc;
    switch (p->precision) {
      case IBF_FP64: rc = make_adjoint_t<double2>(p, s); break;
      case IBF_FP32: rc = make_adjoint_t<float2>(p, s); break;
      default: rc = make_adjoint_t<bf16x2c>(p, s); break;
    }
    if (rc) {
      free_adjoint(p);
      return rc;
    }
  }
  return apply_plan(p->adj, h, ldh, v, ldv, nrhs, s);
}

}  // namespace ibf
