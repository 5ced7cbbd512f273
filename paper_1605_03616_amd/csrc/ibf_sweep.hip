// Sweep-out compression kernels (paper Sec. 4.2): the middle-level
// factorization (eq:KeqUMV), the recursion toward U (eqn:GC) and toward V
// (eqn:HR).  Each preliminary block is evaluated from its explicit formula
// (Sec. 3: eqn:switchlocM, eqn:PIBF3, eqn:PIBF2) inside the kernel that
// compresses it.
#include "ibf_kern.h"

namespace ibf {
namespace kern {
namespace {

// ---------------------------------------------------------------------------
// Middle level: per pair (A at h, B at L-h), A = M~^* with rows s, then
// C = U_k Sigma^(1/2), R = V_k Sigma^(1/2)  (M~ = C R^*).
// ---------------------------------------------------------------------------
template <int R, int G>
__global__ __launch_bounds__(kBlock) void k_middle(PhaseDesc ph, Geo geo, const double* cheb,
                                                   double tol, int cap, int64_t npairs,
                                                   double2* Cout, double2* Rout, int* rk,
                                                   int* rank_max, unsigned long long* nnz) {
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
    if (row_ok) {
      // K(g^A_t, g^B_s) = a exp(2 pi i Phi): the amplitude enters here only
      const double gAt = grid_pt(cA, wA, z[t]);
      val = cscale(conjd(kval(ph, gAt, gBs)), ph.amp ? amp_val(ph, gAt, gBs) : 1.0);
    }
    arow[t] = val;
  }
  double sig[R];
  jacobi_svd<R, G>(arow, v, lane, R, sig);
  int pos[R];
  const int k = cap_rank<R>(sig, pos, rank_positions<R>(sig, tol, pos), cap);
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
                                                    double tol, int cap, int l, int64_t npairs,
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
  const int k = cap_rank<R>(sig, pos, rank_positions<R>(sig, tol, pos), cap);
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
// Up to r = 13 the register budget is that of 3 waves a SIMD, which the
// other sweep kernels reach by themselves (at r = 12: 178 -> 168 VGPRs with
// a few spills, measured 4 % off the build); larger r would spill more.
template <int R, int G>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(R <= 13 ? 3 : 1)))
void k_sweep_h(PhaseDesc ph, Geo geo, const double* cheb,
                                                    double tol, int cap, int l, int64_t npairs,
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
  const int k = cap_rank<R>(sig, pos, rank_positions<R>(sig, tol, pos), cap);
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


template <int R>
void launch_middle(const SweepArgs& A, double2* C, double2* Rm, int* rk, hipStream_t s) {
  constexpr int G = group_for<R>();
  const int64_t threads = A.npairs * G;
  const unsigned blocks = (unsigned)((threads + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_middle<R, G>), dim3(blocks), dim3(kBlock), 0, s, A.ph, A.geo, A.cheb,
                     A.tol, A.cap_at(A.geo.h), A.npairs, C, Rm, rk,
                     A.rank_max + (A.geo.h - A.geo.l0), A.nnz);
}

template <int R>
void launch_sweep_g(const SweepArgs& A, int l, const double2* Cin, double2* Cout,
                    double2* stage, const int* rk_in, int* rk_out, unsigned long long* nnz,
                    hipStream_t s) {
  constexpr int G = group_for<R>();
  const int64_t threads = A.npairs * G;
  const unsigned blocks = (unsigned)((threads + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_sweep_g<R, G>), dim3(blocks), dim3(kBlock), 0, s, A.ph, A.geo, A.cheb,
                     A.tol, A.cap_at(l), l, A.npairs, Cin, Cout, stage, rk_in, rk_out,
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
                     A.tol, A.cap_at(l - 1), l, A.npairs, Rin, Rout, stage, rk_in, rk_out,
                     A.rank_max + (l - 1 - A.geo.l0), nnz);
}


}  // namespace

void middle(int R, const SweepArgs& A, double2* C, double2* Rm, int* rk, hipStream_t s) {
  IBF_DISPATCH_R(R, launch_middle, A, C, Rm, rk, s);
}
void sweep_g(int R, const SweepArgs& A, int l, const double2* Cin, double2* Cout, double2* stage,
             const int* rk_in, int* rk_out, unsigned long long* nnz, hipStream_t s) {
  IBF_DISPATCH_R(R, launch_sweep_g, A, l, Cin, Cout, stage, rk_in, rk_out, nnz, s);
}
void sweep_h(int R, const SweepArgs& A, int l, const double2* Rin, double2* Rout, double2* stage,
             const int* rk_in, int* rk_out, unsigned long long* nnz, hipStream_t s) {
  IBF_DISPATCH_R(R, launch_sweep_h, A, l, Rin, Rout, stage, rk_in, rk_out, nnz, s);
}

}  // namespace kern
}  // namespace ibf
