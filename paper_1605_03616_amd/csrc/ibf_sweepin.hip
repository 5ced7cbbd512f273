// Sweep-in compression kernels (paper Sec. 4.3, eqn:IBFin): from the outer
// factors toward the middle, each step a truncated SVD of a stacked block.
#include "ibf_kern.h"

namespace ibf {
namespace kern {
namespace {

// ---------------------------------------------------------------------------
// Sweep-in stage (paper Sec. 4.3, eqn:IBFin), outer factors toward the middle.
// Every SVD here is A = Q J^* by one-sided Jacobi with rows over lanes.
// ---------------------------------------------------------------------------

// U side, per X-leaf pair (a @ L-l0, b @ l0): Ubar (|A| x r) = Udot Cbar with
// Udot = U_k (= Q_j / sig_j), Cbar = Sigma_k V_k^* (= sig_j J^*)  (eq:lowrankSVD2).
// ubar64 / udot64: [x point][2^l0][r]; cbar: [pair][r][r].
template <int R, int G>
__global__ __launch_bounds__(kBlock) void k_sweepin_u(Geo geo, double tol, const int32_t* xoff,
                                                      const double2* ubar64, double2* udot64,
                                                      double2* cbar, int* rk, int* rank_max) {
  const int lane = threadIdx.x % G;
  const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int l0 = geo.l0;
  const int64_t npairs = (int64_t)1 << geo.L;
  const bool valid = p < npairs;
  const int64_t a = valid ? (p >> l0) : 0;
  const int64_t b = p & ((1 << l0) - 1);
  const int32_t x0 = xoff[a], cnt = valid ? xoff[a + 1] - x0 : 0;
  const bool row_ok = lane < cnt;
  double2 arow[R];
#pragma unroll
  for (int k = 0; k < R; ++k)
    arow[k] = row_ok ? ubar64[(((int64_t)(x0 + lane)) << l0 | b) * R + k] : make_double2(0.0, 0.0);
  double2 v[R];
  double sig[R];
  jacobi_svd<R, G>(arow, v, lane, cnt, sig);
  int pos[R];
  const int k = rank_positions<R>(sig, tol, pos);
  if (row_ok) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const bool keep = pos[j] < k;
      udot64[(((int64_t)(x0 + lane)) << l0 | b) * R + pos[j]] =
          keep ? cscale(arow[j], 1.0 / sig[j]) : make_double2(0.0, 0.0);
    }
  }
  if (valid && lane < R) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const bool keep = pos[j] < k;
      cbar[(p * R + pos[j]) * R + lane] = keep ? cscale(conjd(v[j]), sig[j]) : make_double2(0.0, 0.0);
    }
  }
  const bool leader = valid && lane == 0;
  if (leader) rk[p] = k;
  __shared__ unsigned long long dummy;
  block_accumulate(k, 0ull, leader, rank_max, &dummy);
}

// G side, stage l (input level l-1 -> output level l), processed for
// l = L-l0 .. h+1.  Per input pair q = (a', j = 2B + c):
//   Y = [Cbar_{A0 B} Gbar_{A0 B <- q}; Cbar_{A1 B} Gbar_{A1 B <- q}]  ((2r) x r)
//   Y = [Gdot_0; Gdot_1] Cbar_q,  Gdot = U_k, Cbar_q = Sigma_k V_k^*.
// The staging region (out_alpha, columns c r .. c r + r) is read and then
// overwritten by this group only.
template <int R, int G>
__global__ __launch_bounds__(kBlock) void k_sweepin_g(Geo geo, double tol, int l,
                                                      const double2* cbar_in, double2* cbar_out,
                                                      double2* stage, const int* rk_prev, int* rk,
                                                      int* rank_max, unsigned long long* nnz) {
  const int lane = threadIdx.x % G;
  const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int L = geo.L;
  const int64_t npairs = (int64_t)1 << L;
  const bool valid = q < npairs;
  const int shin = L - l + 1;
  const int64_t ap = q >> shin;
  const int64_t j = q & (((int64_t)1 << shin) - 1);
  const int64_t B = j >> 1;
  const int c = (int)(j & 1);
  const bool row_ok = valid && lane < 2 * R;
  const int alpha = row_ok ? lane / R : 0;
  const int tp = row_ok ? lane % R : 0;
  const int64_t out_a = ((2 * ap + alpha) << (L - l)) | B;
  double2 arow[R];
#pragma unroll
  for (int col = 0; col < R; ++col) arow[col] = make_double2(0.0, 0.0);
  if (row_ok) {
    const double2* crow = cbar_in + (out_a * R + tp) * R;
    const double2* gblk = stage + out_a * R * 2 * R + c * R;
    for (int m = 0; m < R; ++m) {
      const double2 cm = crow[m];
#pragma unroll
      for (int col = 0; col < R; ++col) cfma(arow[col], cm, gblk[m * 2 * R + col]);
    }
  }
  double2 v[R];
  double sig[R];
  jacobi_svd<R, G>(arow, v, lane, 2 * R, sig);
  int pos[R];
  const int k = rank_positions<R>(sig, tol, pos);
  if (row_ok) {
    double2* orow = stage + (out_a * R + tp) * 2 * R + c * R;
#pragma unroll
    for (int jx = 0; jx < R; ++jx) {
      const bool keep = pos[jx] < k;
      orow[pos[jx]] = keep ? cscale(arow[jx], 1.0 / sig[jx]) : make_double2(0.0, 0.0);
    }
  }
  if (valid && lane < R) {
#pragma unroll
    for (int jx = 0; jx < R; ++jx) {
      const bool keep = pos[jx] < k;
      cbar_out[(q * R + pos[jx]) * R + lane] =
          keep ? cscale(conjd(v[jx]), sig[jx]) : make_double2(0.0, 0.0);
    }
  }
  const bool leader = valid && lane == 0;
  unsigned long long add = 0;
  if (leader) {
    rk[q] = k;
    const int64_t o0 = ((2 * ap) << (L - l)) | B, o1 = ((2 * ap + 1) << (L - l)) | B;
    add = (unsigned long long)k * (unsigned long long)(rk_prev[o0] + rk_prev[o1]);
  }
  block_accumulate(k, add, leader, rank_max, nnz);
}

// V side, per pair (a @ l0, Omega leaf b): Vbar^* (r x |B|) = Rbar^* Vdot^*
// with A = Vbar (rows = points): Rbar^* = J_k Sigma_k, Vdot^* = (Q_j/sig_j)^*.
// vbar64 / vdot64: [xi point][2^l0][r]; rbar (Rbar^*): [pair][r][r].
template <int R, int G>
__global__ __launch_bounds__(kBlock) void k_sweepin_v(Geo geo, double tol, const int32_t* xioff,
                                                      const double2* vbar64, double2* vdot64,
                                                      double2* rbar, int* rk, int* rank_max) {
  const int lane = threadIdx.x % G;
  const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int l0 = geo.l0, lb = geo.L - l0;
  const int64_t npairs = (int64_t)1 << geo.L;
  const bool valid = p < npairs;
  const int64_t a = p >> lb;
  const int64_t b = valid ? (p & (((int64_t)1 << lb) - 1)) : 0;
  const int32_t j0 = xioff[b], cnt = valid ? xioff[b + 1] - j0 : 0;
  const bool row_ok = lane < cnt;
  double2 arow[R];
#pragma unroll
  for (int k = 0; k < R; ++k)
    arow[k] = row_ok ? conjd(vbar64[(((int64_t)(j0 + lane)) << l0 | a) * R + k])
                     : make_double2(0.0, 0.0);
  double2 v[R];
  double sig[R];
  jacobi_svd<R, G>(arow, v, lane, cnt, sig);
  int pos[R];
  const int k = rank_positions<R>(sig, tol, pos);
  if (row_ok) {
#pragma unroll
    for (int jx = 0; jx < R; ++jx) {
      const bool keep = pos[jx] < k;
      vdot64[(((int64_t)(j0 + lane)) << l0 | a) * R + pos[jx]] =
          keep ? cscale(conjd(arow[jx]), 1.0 / sig[jx]) : make_double2(0.0, 0.0);
    }
  }
  if (valid && lane < R) {
#pragma unroll
    for (int jx = 0; jx < R; ++jx) {
      const bool keep = pos[jx] < k;
      rbar[(p * R + lane) * R + pos[jx]] = keep ? cscale(v[jx], sig[jx]) : make_double2(0.0, 0.0);
    }
  }
  const bool leader = valid && lane == 0;
  if (leader) rk[p] = k;
  __shared__ unsigned long long dummy;
  block_accumulate(k, 0ull, leader, rank_max, &dummy);
}

// H side, stage l = l0+1 .. h, per output pair p = (a, b):
//   Y = [F_{p,0} Rbar^*_{in0}, F_{p,1} Rbar^*_{in1}]   (r x 2r)
//   Y = Rbar^*_p [Fdot_0, Fdot_1],  Rbar^*_p = U_k Sigma_k, Fdot = V_k^*.
// A = Y^* with rows i = c r + col.  The staging region of p is read and then
// overwritten by this group only.
template <int R, int G>
__global__ __launch_bounds__(kBlock) void k_sweepin_h(Geo geo, double tol, int l,
                                                      const double2* rbar_in, double2* rbar_out,
                                                      double2* stage, const int* rk_prev, int* rk,
                                                      int* rank_max, unsigned long long* nnz) {
  const int lane = threadIdx.x % G;
  const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int L = geo.L;
  const int64_t npairs = (int64_t)1 << L;
  const bool valid = p < npairs;
  const int sh = L - l;
  const int64_t a = p >> sh;
  const int64_t b = p & (((int64_t)1 << sh) - 1);
  const bool row_ok = valid && lane < 2 * R;
  const int c = row_ok ? lane / R : 0;
  const int col = row_ok ? lane % R : 0;
  const int64_t in_c = ((a >> 1) << (sh + 1)) | (2 * b + c);
  double2 rcol[R];
#pragma unroll
  for (int t = 0; t < R; ++t)
    rcol[t] = row_ok ? rbar_in[(in_c * R + t) * R + col] : make_double2(0.0, 0.0);
  double2 arow[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    double2 acc = make_double2(0.0, 0.0);
    if (row_ok) {
      const double2* frow = stage + (p * R + m) * 2 * R + c * R;
#pragma unroll
      for (int t = 0; t < R; ++t) cfma(acc, frow[t], rcol[t]);
    }
    arow[m] = conjd(acc);
  }
  double2 v[R];
  double sig[R];
  jacobi_svd<R, G>(arow, v, lane, 2 * R, sig);
  int pos[R];
  const int k = rank_positions<R>(sig, tol, pos);
  // every lane has read its F rows before any lane of the group writes
  if (row_ok) {
#pragma unroll
    for (int jx = 0; jx < R; ++jx) {
      const bool keep = pos[jx] < k;
      stage[(p * R + pos[jx]) * 2 * R + lane] =
          keep ? cscale(conjd(arow[jx]), 1.0 / sig[jx]) : make_double2(0.0, 0.0);
    }
  }
  if (valid && lane < R) {
#pragma unroll
    for (int jx = 0; jx < R; ++jx) {
      const bool keep = pos[jx] < k;
      rbar_out[(p * R + lane) * R + pos[jx]] =
          keep ? cscale(v[jx], sig[jx]) : make_double2(0.0, 0.0);
    }
  }
  const bool leader = valid && lane == 0;
  unsigned long long add = 0;
  if (leader) {
    rk[p] = k;
    const int64_t i0 = ((a >> 1) << (sh + 1)) | (2 * b);
    add = (unsigned long long)k * (unsigned long long)(rk_prev[i0] + rk_prev[i0 + 1]);
  }
  block_accumulate(k, add, leader, rank_max, nnz);
}

// Middle block Mdot = Cbar^h Rbar^{h*} (eqn:IBFin), packed directly into
// [pair][KG][KH] in the storage precision; counts unpadded entries.

template <int R>
void launch_sweepin_u(const Geo& geo, double tol, const int32_t* xoff, const double2* ub,
                      double2* ud, double2* cb, int* rk, int* rank_max, hipStream_t s) {
  const int64_t np = (int64_t)1 << geo.L;
  hipLaunchKernelGGL((k_sweepin_u<R, 64>), dim3((unsigned)((np * 64 + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, geo, tol, xoff, ub, ud, cb, rk, rank_max);
}
template <int R>
void launch_sweepin_v(const Geo& geo, double tol, const int32_t* xioff, const double2* vb,
                      double2* vd, double2* rb, int* rk, int* rank_max, hipStream_t s) {
  const int64_t np = (int64_t)1 << geo.L;
  hipLaunchKernelGGL((k_sweepin_v<R, 64>), dim3((unsigned)((np * 64 + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, geo, tol, xioff, vb, vd, rb, rk, rank_max);
}
template <int R>
void launch_sweepin_g(const Geo& geo, double tol, int l, const double2* cin, double2* cout,
                      double2* stage, const int* rkp, int* rk, int* rank_max,
                      unsigned long long* nnz, hipStream_t s) {
  constexpr int G = group_for<R>();
  const int64_t np = (int64_t)1 << geo.L;
  hipLaunchKernelGGL((k_sweepin_g<R, G>), dim3((unsigned)((np * G + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, geo, tol, l, cin, cout, stage, rkp, rk, rank_max, nnz);
}
template <int R>
void launch_sweepin_h(const Geo& geo, double tol, int l, const double2* rin, double2* rout,
                      double2* stage, const int* rkp, int* rk, int* rank_max,
                      unsigned long long* nnz, hipStream_t s) {
  constexpr int G = group_for<R>();
  const int64_t np = (int64_t)1 << geo.L;
  hipLaunchKernelGGL((k_sweepin_h<R, G>), dim3((unsigned)((np * G + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, geo, tol, l, rin, rout, stage, rkp, rk, rank_max, nnz);
}


}  // namespace

void sweepin_u(int R, const Geo& geo, double tol, const int32_t* xoff, const double2* ub,
               double2* ud, double2* cb, int* rk, int* rank_max, hipStream_t s) {
  IBF_DISPATCH_R(R, launch_sweepin_u, geo, tol, xoff, ub, ud, cb, rk, rank_max, s);
}
void sweepin_v(int R, const Geo& geo, double tol, const int32_t* xioff, const double2* vb,
               double2* vd, double2* rb, int* rk, int* rank_max, hipStream_t s) {
  IBF_DISPATCH_R(R, launch_sweepin_v, geo, tol, xioff, vb, vd, rb, rk, rank_max, s);
}
void sweepin_g(int R, const Geo& geo, double tol, int l, const double2* cin, double2* cout,
               double2* stage, const int* rkp, int* rk, int* rank_max, unsigned long long* nnz,
               hipStream_t s) {
  IBF_DISPATCH_R(R, launch_sweepin_g, geo, tol, l, cin, cout, stage, rkp, rk, rank_max, nnz, s);
}
void sweepin_h(int R, const Geo& geo, double tol, int l, const double2* rin, double2* rout,
               double2* stage, const int* rkp, int* rk, int* rank_max, unsigned long long* nnz,
               hipStream_t s) {
  IBF_DISPATCH_R(R, launch_sweepin_h, geo, tol, l, rin, rout, stage, rkp, rk, rank_max, nnz, s);
}

}  // namespace kern
}  // namespace ibf
