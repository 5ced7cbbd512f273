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
#include <cstring>
#include <vector>

#include "ibf_device.h"

namespace ibf {
namespace {

constexpr int kBlock = 256;

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
  ~DevBuf() { if (ptr) (void)hipFree(ptr); }
  hipError_t alloc(size_t count) {
    n = count;
    return hipMalloc((void**)&ptr, std::max<size_t>(count, 1) * sizeof(T));
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

template <int R>
__device__ inline void load_cheb(const double* cheb, double* z, double* Lc) {
  for (int e = threadIdx.x; e < R + 2 * R * R; e += blockDim.x) {
    double v = cheb[e];
    if (e < R) z[e] = v;
    else Lc[e - R] = v;
  }
  __syncthreads();
}

__device__ __forceinline__ double2 shfl2(double2 v, int src, int width) {
  return make_double2(__shfl(v.x, src, width), __shfl(v.y, src, width));
}

// Block-level reduction of the per-group rank (max) and a 64-bit counter.
__device__ inline void block_accumulate(int k, unsigned long long add, bool leader,
                                        int* rank_max_slot, unsigned long long* nnz) {
  __shared__ int s_max;
  __shared__ unsigned long long s_sum;
  if (threadIdx.x == 0) { s_max = 0; s_sum = 0ull; }
  __syncthreads();
  if (leader) {
    atomicMax(&s_max, k);
    atomicAdd(&s_sum, add);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(rank_max_slot, s_max);
    atomicAdd(nnz, s_sum);
  }
}

// ---------------------------------------------------------------------------
// Middle level: per pair (A at h, B at L-h), A = M~^* with rows s, then
// C = U_k Sigma^(1/2), R = V_k Sigma^(1/2)  (M~ = C R^*).
// ---------------------------------------------------------------------------
template <int R, int G>
__global__ __launch_bounds__(kBlock) void k_middle(PhaseDesc ph, Geo geo, const double* cheb,
                                                   double tol, int64_t npairs, double2* Cout,
                                                   double2* Rout, int* rk, int* rank_max,
                                                   unsigned long long* nnz) {
  __shared__ double z[R];
  __shared__ double Lc[2 * R * R];
  load_cheb<R>(cheb, z, Lc);
  const int lane = threadIdx.x % G;
  const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const bool valid = p < npairs;
  const int L = geo.L, h = geo.h;
  const int64_t a = p >> (L - h);
  const int64_t b = p & (((int64_t)1 << (L - h)) - 1);

  double2 arow[R];
  double2 v[R];
  const bool row_ok = valid && lane < R;
  const double cA = box_cx(h, a), wA = box_wx(h);
  const double cB = box_cxi(geo, L - h, b), wB = box_wxi(geo, L - h);
  const double gBs = grid_pt(cB, wB, z[row_ok ? lane : 0]);
#pragma unroll
  for (int t = 0; t < R; ++t) {
    double2 val = make_double2(0.0, 0.0);
    if (row_ok) val = conjd(kval(ph, grid_pt(cA, wA, z[t]), gBs));
    arow[t] = val;
  }
  double sig[R];
  jacobi_svd<R, G>(arow, v, lane, R, sig);
  int pos[R];
  const int k = rank_positions<R>(sig, tol, pos);
  if (valid && lane < R) {
    double2* Cp = Cout + (p * R + lane) * R;
    double2* Rp = Rout + (p * R + lane) * R;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const bool keep = pos[j] < k;
      const double sq = keep ? sqrt(sig[j]) : 0.0;
      Cp[pos[j]] = keep ? cscale(v[j], sq) : make_double2(0.0, 0.0);
      Rp[pos[j]] = keep ? cscale(arow[j], 1.0 / sq) : make_double2(0.0, 0.0);
    }
  }
  const bool leader = valid && lane == 0;
  if (leader) rk[p] = k;
  block_accumulate(k, (unsigned long long)k, leader, rank_max, nnz);
}

// ---------------------------------------------------------------------------
// Sweep toward U, output level l (h < l <= L-l0).  Output pair (A, B):
// A at level l (child alpha of P), B at level L-l with children C_c.
//   G_c[t][s] = exp(2 pi i Phi(g^A_t, c_C)) M^P_s(g^A_t) exp(-2 pi i Phi(g^P_s, c_C))
//   W = [G_0 C_{P C_0}, G_1 C_{P C_1}]   (r x 2r, zero-padded columns)
// Rows of A = W^* are indexed by i = c r + j (input child c, input column j).
// ---------------------------------------------------------------------------
template <int R, int G>
__global__ __launch_bounds__(kBlock) void k_sweep_g(PhaseDesc ph, Geo geo, const double* cheb,
                                                    double tol, int l, int64_t npairs,
                                                    const double2* Cin, double2* Cout,
                                                    double2* stage, const int* rk_in, int* rk_out,
                                                    int* rank_max, unsigned long long* nnz) {
  __shared__ double z[R];
  __shared__ double Lc[2 * R * R];
  load_cheb<R>(cheb, z, Lc);
  const int lane = threadIdx.x % G;
  const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const bool valid = p < npairs;
  const int L = geo.L;
  const int sh = L - l;
  const int64_t a = p >> sh;
  const int64_t b = p & (((int64_t)1 << sh) - 1);
  const int alpha = (int)(a & 1);
  const int64_t ap = a >> 1;
  const bool row_ok = valid && lane < 2 * R;
  const int c = row_ok ? lane / R : 0;
  const int jj = row_ok ? lane % R : 0;
  const int64_t in_c = (ap << (sh + 1)) | (2 * b + c);

  // phases: lane (c, jj) evaluates D1_c[jj] and D2_c[jj]
  const double cC = box_cxi(geo, L - l + 1, 2 * b + c);
  const double gA = grid_pt(box_cx(l, a), box_wx(l), z[jj]);
  const double gP = grid_pt(box_cx(l - 1, ap), box_wx(l - 1), z[jj]);
  const double2 d1 = valid ? kval(ph, gA, cC) : make_double2(0.0, 0.0);
  const double2 d2 = valid ? conjd(kval(ph, gP, cC)) : make_double2(0.0, 0.0);

  double2 y[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    double2 ds = shfl2(d2, c * R + s, G);
    double2 cv = row_ok ? Cin[(in_c * R + s) * R + jj] : make_double2(0.0, 0.0);
    y[s] = cmul(ds, cv);
  }
  double2 arow[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const double lx = Lc[(alpha * R + s) * R + t];   // M^P_s(g^A_t)
      acc.x = fma(lx, y[s].x, acc.x);
      acc.y = fma(lx, y[s].y, acc.y);
    }
    double2 dt = shfl2(d1, c * R + t, G);
    double2 w = cmul(dt, acc);
    arow[t] = row_ok ? conjd(w) : make_double2(0.0, 0.0);
  }
  double2 v[R];
  double sig[R];
  jacobi_svd<R, G>(arow, v, lane, 2 * R, sig);
  int pos[R];
  const int k = rank_positions<R>(sig, tol, pos);
  if (valid && lane < R) {
    double2* Cp = Cout + (p * R + lane) * R;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const bool keep = pos[j] < k;
      Cp[pos[j]] = keep ? cscale(v[j], sig[j]) : make_double2(0.0, 0.0);
    }
  }
  if (row_ok) {
    double2* Sp = stage + p * R * 2 * R;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const bool keep = pos[j] < k;
      Sp[pos[j] * 2 * R + lane] =
          keep ? cscale(conjd(arow[j]), 1.0 / sig[j]) : make_double2(0.0, 0.0);
    }
  }
  const bool leader = valid && lane == 0;
  unsigned long long add = 0;
  if (leader) {
    rk_out[p] = k;
    const int64_t in0 = (ap << (sh + 1)) | (2 * b);
    add = (unsigned long long)k * (unsigned long long)(rk_in[in0] + rk_in[in0 + 1]);
  }
  block_accumulate(k, add, leader, rank_max, nnz);
}

// ---------------------------------------------------------------------------
// Sweep toward V for stage l (l0 < l <= h): per input pair (P, C) at level
// l-1 with outputs (A_alpha, B) at level l, C = child c of B.
//   H_alpha[t][s] = exp(-2 pi i Phi(c_A, g^B_t)) M^B_t(g^C_s) exp(2 pi i Phi(c_A, g^C_s))
//   Z = [H_0^* R_{A0 B}, H_1^* R_{A1 B}],  A = Z^*,  A[i][s] with i = alpha r + j.
// ---------------------------------------------------------------------------
template <int R, int G>
__global__ __launch_bounds__(kBlock) void k_sweep_h(PhaseDesc ph, Geo geo, const double* cheb,
                                                    double tol, int l, int64_t npairs,
                                                    const double2* Rin, double2* Rout,
                                                    double2* stage, const int* rk_in, int* rk_out,
                                                    int* rank_max, unsigned long long* nnz) {
  __shared__ double z[R];
  __shared__ double Lc[2 * R * R];
  load_cheb<R>(cheb, z, Lc);
  const int lane = threadIdx.x % G;
  const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const bool valid = q < npairs;
  const int L = geo.L;
  const int shin = L - l + 1;
  const int64_t ap = q >> shin;
  const int64_t j = q & (((int64_t)1 << shin) - 1);
  const int64_t B = j >> 1;
  const int c = (int)(j & 1);
  const bool row_ok = valid && lane < 2 * R;
  const int alpha = row_ok ? lane / R : 0;
  const int jj = row_ok ? lane % R : 0;
  const int64_t out_a = ((2 * ap + alpha) << (L - l)) | B;

  const double cA = box_cx(l, 2 * ap + alpha);
  const double gB = grid_pt(box_cxi(geo, L - l, B), box_wxi(geo, L - l), z[jj]);
  const double gC = grid_pt(box_cxi(geo, L - l + 1, j), box_wxi(geo, L - l + 1), z[jj]);
  const double2 e1 = valid ? conjd(kval(ph, cA, gB)) : make_double2(0.0, 0.0);
  const double2 e2 = valid ? kval(ph, cA, gC) : make_double2(0.0, 0.0);

  double2 y[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    double2 et = shfl2(e1, alpha * R + t, G);
    double2 rv = row_ok ? Rin[(out_a * R + t) * R + jj] : make_double2(0.0, 0.0);
    y[t] = cmul(et, conjd(rv));
  }
  double2 arow[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const double lb = Lc[(c * R + t) * R + s];     // M^B_t(g^C_s)
      acc.x = fma(lb, y[t].x, acc.x);
      acc.y = fma(lb, y[t].y, acc.y);
    }
    double2 es = shfl2(e2, alpha * R + s, G);
    arow[s] = row_ok ? cmul(es, acc) : make_double2(0.0, 0.0);
  }
  double2 v[R];
  double sig[R];
  jacobi_svd<R, G>(arow, v, lane, 2 * R, sig);
  int pos[R];
  const int k = rank_positions<R>(sig, tol, pos);
  if (valid && lane < R) {
    double2* Rp = Rout + (q * R + lane) * R;
#pragma unroll
    for (int jx = 0; jx < R; ++jx) {
      const bool keep = pos[jx] < k;
      Rp[pos[jx]] = keep ? cscale(v[jx], sig[jx]) : make_double2(0.0, 0.0);
    }
  }
  if (row_ok) {
    double2* Sp = stage + (out_a * R + jj) * 2 * R + c * R;
#pragma unroll
    for (int jx = 0; jx < R; ++jx) {
      const bool keep = pos[jx] < k;
      Sp[pos[jx]] = keep ? cscale(arow[jx], 1.0 / sig[jx]) : make_double2(0.0, 0.0);
    }
  }
  const bool leader = valid && lane == 0;
  unsigned long long add = 0;
  if (leader) {
    rk_out[q] = k;
    const int64_t o0 = ((2 * ap) << (L - l)) | B;
    const int64_t o1 = ((2 * ap + 1) << (L - l)) | B;
    add = (unsigned long long)k * (unsigned long long)(rk_in[o0] + rk_in[o1]);
  }
  block_accumulate(k, add, leader, rank_max, nnz);
}

// ---------------------------------------------------------------------------
// Conversion of one stage from the FP64 r x 2r staging layout to the stored
// layout [pair][k_out][2 k_in] in the storage precision.
// ---------------------------------------------------------------------------
template <typename FT>
__global__ void k_pack_stage(const double2* stage, FT* out, int64_t npairs, int R, int kout,
                             int kin) {
  const int64_t per = (int64_t)kout * 2 * kin;
  const int64_t total = npairs * per;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / per;
    const int rem = (int)(e - p * per);
    const int t = rem / (2 * kin);
    const int cc = rem - t * 2 * kin;
    const int c = cc / kin, s = cc - c * kin;
    store_factor(out, e, stage[(p * R + t) * 2 * R + c * R + s]);
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

__global__ void k_eval(PhaseDesc ph, const double* x, const double* xi, int64_t n, double2* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = kval(ph, x[i], xi[i]);
}

// ---------------------------------------------------------------------------
// Launch helpers templated on r.
// ---------------------------------------------------------------------------
struct SweepArgs {
  PhaseDesc ph;
  Geo geo;
  const double* cheb;
  double tol;
  int64_t npairs;
  int* rank_max;
  unsigned long long* nnz;
};

template <int R>
constexpr int group_for() { return R <= 8 ? 16 : 32; }

template <int R>
void launch_middle(const SweepArgs& A, double2* C, double2* Rm, int* rk, hipStream_t s) {
  constexpr int G = group_for<R>();
  const int64_t threads = A.npairs * G;
  const unsigned blocks = (unsigned)((threads + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_middle<R, G>), dim3(blocks), dim3(kBlock), 0, s, A.ph, A.geo, A.cheb,
                     A.tol, A.npairs, C, Rm, rk, A.rank_max + (A.geo.h - A.geo.l0), A.nnz);
}

template <int R>
void launch_sweep_g(const SweepArgs& A, int l, const double2* Cin, double2* Cout,
                    double2* stage, const int* rk_in, int* rk_out, unsigned long long* nnz,
                    hipStream_t s) {
  constexpr int G = group_for<R>();
  const int64_t threads = A.npairs * G;
  const unsigned blocks = (unsigned)((threads + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_sweep_g<R, G>), dim3(blocks), dim3(kBlock), 0, s, A.ph, A.geo, A.cheb,
                     A.tol, l, A.npairs, Cin, Cout, stage, rk_in, rk_out,
                     A.rank_max + (l - A.geo.l0), nnz);
}

template <int R>
void launch_sweep_h(const SweepArgs& A, int l, const double2* Rin, double2* Rout,
                    double2* stage, const int* rk_in, int* rk_out, unsigned long long* nnz,
                    hipStream_t s) {
  constexpr int G = group_for<R>();
  const int64_t threads = A.npairs * G;
  const unsigned blocks = (unsigned)((threads + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_sweep_h<R, G>), dim3(blocks), dim3(kBlock), 0, s, A.ph, A.geo, A.cheb,
                     A.tol, l, A.npairs, Rin, Rout, stage, rk_in, rk_out,
                     A.rank_max + (l - 1 - A.geo.l0), nnz);
}

#define IBF_DISPATCH_R(r, FN, ...)                    \
  switch (r) {                                        \
    case 2: FN<2>(__VA_ARGS__); break;                \
    case 3: FN<3>(__VA_ARGS__); break;                \
    case 4: FN<4>(__VA_ARGS__); break;                \
    case 5: FN<5>(__VA_ARGS__); break;                \
    case 6: FN<6>(__VA_ARGS__); break;                \
    case 7: FN<7>(__VA_ARGS__); break;                \
    case 8: FN<8>(__VA_ARGS__); break;                \
    case 9: FN<9>(__VA_ARGS__); break;                \
    case 10: FN<10>(__VA_ARGS__); break;              \
    case 11: FN<11>(__VA_ARGS__); break;              \
    case 12: FN<12>(__VA_ARGS__); break;              \
    case 13: FN<13>(__VA_ARGS__); break;              \
    case 14: FN<14>(__VA_ARGS__); break;              \
    case 15: FN<15>(__VA_ARGS__); break;              \
    case 16: FN<16>(__VA_ARGS__); break;              \
    default: break;                                   \
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
    const int64_t count = p->npairs * st.k_out * 2 * st.k_in;
    st.bytes = (size_t)count * fb;
    IBF_HIP_CHECK(hipMalloc(&st.blk, std::max<size_t>(st.bytes, 1)));
    p->stages.push_back(st);
    const unsigned blocks = (unsigned)std::min<int64_t>((count + kBlock - 1) / kBlock, 1 << 20);
    hipLaunchKernelGGL((k_pack_stage<FT>), dim3(std::max(blocks, 1u)), dim3(kBlock), 0, s,
                       stages[l - l0 - 1].ptr, (FT*)st.blk, p->npairs, R, st.k_out, st.k_in);
    p->nnz_stored += count;
  }
  // Ubar at level L-l0, Vbar at level l0
  p->k_ubar = p->rank[L - l0 - l0];
  p->k_vbar = p->rank[0];
  p->ubar_bytes = (size_t)(p->nx << l0) * p->k_ubar * fb;
  p->vbar_bytes = (size_t)(p->nxi << l0) * p->k_vbar * fb;
  IBF_HIP_CHECK(hipMalloc(&p->d_ubar, std::max<size_t>(p->ubar_bytes, 1)));
  IBF_HIP_CHECK(hipMalloc(&p->d_vbar, std::max<size_t>(p->vbar_bytes, 1)));
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

template <typename T>
int upload(T** dst, const std::vector<T>& src) {
  if (*dst) return IBF_OK;
  IBF_HIP_CHECK(hipMalloc((void**)dst, std::max<size_t>(src.size(), 1) * sizeof(T)));
  if (!src.empty())
    IBF_HIP_CHECK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return IBF_OK;
}

}  // namespace

int build_plan(ibf_plan_t p, hipStream_t s) {
  IBF_HIP_CHECK(hipSetDevice(p->device));
  free_factors(p);
  int rc;
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

  SweepArgs A{p->phase, geo, cheb.ptr, p->tol, np, rank_max.ptr, nnz.ptr + nst};
  IBF_DISPATCH_R(R, launch_middle, A, Cb[0].ptr, Rb[0].ptr, rk_mid.ptr, s);

  // sweep toward U
  const double2* Ccur = Cb[0].ptr;
  const int* rkcur = rk_mid.ptr;
  int gi = 0;
  double2* Cout_last = Cb[0].ptr;
  const int* rkU = rk_mid.ptr;
  for (int l = h + 1; l <= L - l0; ++l) {
    double2* Cout = (Ccur == Cb[0].ptr) ? Cb[1].ptr : Cb[0].ptr;
    int* rkout = rkG[gi].ptr;
    IBF_DISPATCH_R(R, launch_sweep_g, A, l, Ccur, Cout, stages[l - l0 - 1].ptr, rkcur, rkout,
                   nnz.ptr + (l - l0 - 1), s);
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
    IBF_DISPATCH_R(R, launch_sweep_h, A, l, Rcur, Rout, stages[l - l0 - 1].ptr, rkcur, rkout,
                   nnz.ptr + (l - l0 - 1), s);
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

int eval_kernel(const PhaseDesc& ph, const double* x, const double* xi, int64_t n, void* out,
                hipStream_t s) {
  hipLaunchKernelGGL(k_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ph, x, xi, n,
                     (double2*)out);
  IBF_HIP_CHECK(hipGetLastError());
  return IBF_OK;
}

}  // namespace ibf
