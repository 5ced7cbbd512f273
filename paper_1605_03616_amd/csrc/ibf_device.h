// Device helpers: complex arithmetic, FP64 reduced phase, tree geometry,
// Chebyshev grids, Lagrange polynomials and the wave-group one-sided Jacobi
// SVD used by every compression step.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "ibf_internal.h"

namespace ibf {

// ---------------------------------------------------------------------------
// complex helpers (double2 / float2 as re, im)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) {
  return make_double2(a.x * s, a.y * s);
}
// acc += a * b
__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
__device__ __forceinline__ void cfma(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x));
  acc.y = fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y));
}

// ---------------------------------------------------------------------------
// Phase Phi(x, xi) reduced mod 1 (paper eqn:FIO kernel exp(2 pi i Phi)).
// Products of a coordinate and a frequency are reduced error-free with an
// FMA-based two-product, so the fractional part survives |Phi| ~ N.
// ---------------------------------------------------------------------------
__device__ inline double frac_prod(double a, double b) {
#pragma clang fp contract(off)
  double p = a * b;
  double e = fma(a, b, -p);
  double t = (p - rint(p)) + e;
  return t - rint(t);
}

__device__ inline double phase_frac(const PhaseDesc& P, double x, double xi) {
#pragma clang fp contract(off)
  double t;
  if (P.kind == IBF_PHASE_DFT) {
    t = P.p[0] * frac_prod(x, xi);
  } else if (P.kind == IBF_PHASE_FIO1D) {
    // c(x) = (p0 + p1 sin 2 pi x)/p2  (paper eqn:1D-FIO-kernal)
    double c = (P.p[0] + P.p[1] * sinpi(2.0 * x)) / P.p[2];
    t = frac_prod(x, xi) + frac_prod(c, fabs(xi));
  } else {  // separable
    t = frac_prod(P.p[0], x) + frac_prod(P.p[1], xi);
  }
  return t - rint(t);
}

// Amplitude a(x, xi) of the kernel a exp(2 pi i Phi) (paper eqn:FIO); 1 when
// the descriptor has none.  Real-valued families:
//   separable: (q0 + q1 sin 2 pi x + q2 cos 2 pi x)(q3 + q4 xi / sqrt(xi^2 + q5^2))
//   wave:      q0 + q1 cos(2 pi (x + xi / q2))
__device__ inline double amp_val(const PhaseDesc& P, double x, double xi) {
#pragma clang fp contract(off)
  if (P.amp == IBF_AMP_SEPARABLE) {
    const double fx = P.q[0] + P.q[1] * sinpi(2.0 * x) + P.q[2] * cospi(2.0 * x);
    const double fxi = P.q[3] + P.q[4] * xi / sqrt(xi * xi + P.q[5] * P.q[5]);
    return fx * fxi;
  }
  if (P.amp == IBF_AMP_WAVE) return P.q[0] + P.q[1] * cospi(2.0 * (x + xi / P.q[2]));
  return 1.0;
}

// exp(2 pi i Phi(x, xi))
__device__ inline double2 kval(const PhaseDesc& P, double x, double xi) {
  double t = phase_frac(P, x, xi);
  double s, c;
  sincospi(2.0 * t, &s, &c);
  return make_double2(c, s);
}

// ---------------------------------------------------------------------------
// Geometry (half-open dyadic boxes with geometric centres).
// ---------------------------------------------------------------------------
__device__ inline double box_cx(int level, int64_t a) {
#pragma clang fp contract(off)
  return ((double)a + 0.5) * ldexp(1.0, -level);
}
__device__ inline double box_wx(int level) { return ldexp(1.0, -level); }
__device__ inline double box_cxi(const Geo& g, int level, int64_t b) {
#pragma clang fp contract(off)
  double w = g.W / ldexp(1.0, level);
  return g.lo + ((double)b + 0.5) * w;
}
__device__ inline double box_wxi(const Geo& g, int level) { return g.W / ldexp(1.0, level); }
// grid point c + w z_t
__device__ inline double grid_pt(double c, double w, double z) {
#pragma clang fp contract(off)
  return c + w * z;
}
// normalised coordinate (pt - c)/w
__device__ inline double norm_pt(double pt, double c, double w) {
#pragma clang fp contract(off)
  return (pt - c) / w;
}

// Lagrange polynomial M_t(y) on nodes z[0..r) (paper Sec. 2.1, product form).
__device__ inline double lagrange_t(const double* z, int r, int t, double y) {
#pragma clang fp contract(off)
  double m = 1.0;
  for (int j = 0; j < r; ++j)
    if (j != t) m *= (y - z[j]) / (z[t] - z[j]);
  return m;
}

// ---------------------------------------------------------------------------
// Group reductions over G lanes (G a power of two, groups aligned in the
// wavefront, every lane of a group active).  Within a row of 16 lanes the
// partners come from DPP lane moves (quad permutes [1,0,3,2] and [2,3,0,1],
// the half-row and row mirrors), across rows from lane shuffles.  Every
// step pairs each lane with a partner that pairs back with it, so both add
// the same two values: the sums are bitwise identical in every lane of the
// group (the rotation decisions of a Jacobi sweep depend on it).
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_move<0xB1>(v);               // quad_perm [1,0,3,2]
  if constexpr (G >= 4) v += dpp_move<0x4E>(v);               // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += dpp_move<0x141>(v);              // row_half_mirror
  if constexpr (G >= 16) v += dpp_move<0x140>(v);             // row_mirror
  if constexpr (G >= 32) v += __shfl_xor(v, 16, G);
  if constexpr (G >= 64) v += __shfl_xor(v, 32, G);
  return v;
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of an n x R complex matrix A, n <= G,
// held one row per lane (lanes >= n hold zero rows).  On return a[] holds the
// rows of Q = A J with mutually orthogonal columns, v[] holds row `lane` of
// the unitary J (lanes < R), and sig[j] = ||Q_j||.  Then A = Q J^* and
// A^* = J Sigma Uhat^* with Uhat_j = Q_j / sig_j.
// ---------------------------------------------------------------------------
constexpr int kJacobiMaxSweeps = 30;

// One complex Jacobi rotation of columns (p, q): with gamma = a_p^H a_q =
// |gamma| e^{i phi}, rotate [a_p, e^{-i phi} a_q] by the real Jacobi angle
// that zeroes the off-diagonal of the 2 x 2 Gram matrix; J gets the same
// column operation.  Column norms are updated in closed form.
// Columns whose squared norm is below `small` (1e-30 of ||A||_F^2) are at
// rounding level: rotating them only shrinks noise toward subnormals, where
// exp(-i arg gamma) overflows, so they are left alone.
template <int G>
__device__ __forceinline__ void jacobi_rotate(double2& ap_, double2& aq_, double2& vp_,
                                              double2& vq_, double& np_, double& nq_,
                                              double thresh, double small, bool& rotated) {
  const double gr = group_sum<G>(ap_.x * aq_.x + ap_.y * aq_.y);
  const double gi = group_sum<G>(ap_.x * aq_.y - ap_.y * aq_.x);
  const double ag = sqrt(gr * gr + gi * gi);
  if (np_ > small && nq_ > small && ag > thresh * sqrt(np_ * nq_)) {
    const double zeta = (nq_ - np_) / (2.0 * ag);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t);
    const double s = c * t;
    const double2 e = make_double2(gr / ag, -gi / ag);   // exp(-i arg gamma)
    const double2 eq = cmul(e, aq_);
    const double2 ap = ap_;
    ap_ = make_double2(c * ap.x - s * eq.x, c * ap.y - s * eq.y);
    aq_ = make_double2(s * ap.x + c * eq.x, s * ap.y + c * eq.y);
    const double2 ev = cmul(e, vq_);
    const double2 vp = vp_;
    vp_ = make_double2(c * vp.x - s * ev.x, c * vp.y - s * ev.y);
    vq_ = make_double2(s * vp.x + c * ev.x, s * vp.y + c * ev.y);
    np_ -= t * ag;
    nq_ += t * ag;
    rotated = true;
  }
}

// Cyclic-by-rows sweep (p, q), p < q, expanded at compile time so that every
// register-array index is a constant.
template <int R, int G, int P, int Q>
__device__ __forceinline__ void jacobi_sweep(double2 (&a)[R], double2 (&v)[R], double (&nrm)[R],
                                             double thresh, double small, bool& rotated) {
  if constexpr (P < R - 1) {
    jacobi_rotate<G>(a[P], a[Q], v[P], v[Q], nrm[P], nrm[Q], thresh, small, rotated);
    if constexpr (Q + 1 < R)
      jacobi_sweep<R, G, P, Q + 1>(a, v, nrm, thresh, small, rotated);
    else
      jacobi_sweep<R, G, P + 1, P + 2>(a, v, nrm, thresh, small, rotated);
  }
}

template <int R, int G>
__device__ __forceinline__ void jacobi_svd(double2 (&a)[R], double2 (&v)[R], int lane,
                                  int n, double (&sig)[R]) {
  const double thresh = 4.0 * (double)(n > 8 ? n : 8) * 1.1102230246251565e-16;
#pragma unroll
  for (int j = 0; j < R; ++j) v[j] = make_double2(lane == j ? 1.0 : 0.0, 0.0);
  double nrm[R];
#pragma unroll
  for (int j = 0; j < R; ++j) nrm[j] = group_sum<G>(a[j].x * a[j].x + a[j].y * a[j].y);
  double fro2 = 0.0;
#pragma unroll
  for (int j = 0; j < R; ++j) fro2 += nrm[j];
  const double small = 1e-30 * fro2;

  for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
    bool rotated = false;
    jacobi_sweep<R, G, 0, 1>(a, v, nrm, thresh, small, rotated);
#pragma unroll
    for (int j = 0; j < R; ++j) nrm[j] = group_sum<G>(a[j].x * a[j].x + a[j].y * a[j].y);
    if (!__any(rotated)) break;
  }
#pragma unroll
  for (int j = 0; j < R; ++j) sig[j] = sqrt(nrm[j]);
}

// Position of column j in descending order of sig (ties by index), and the
// number of sig_j > tol * max sig.
template <int R>
__device__ __forceinline__ int rank_positions(const double (&sig)[R], double tol, int (&pos)[R]) {
  double smax = 0.0;
#pragma unroll
  for (int j = 0; j < R; ++j) smax = fmax(smax, sig[j]);
  int k = 0;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    int pj = 0;
#pragma unroll
    for (int i = 0; i < R; ++i)
      pj += (sig[i] > sig[j] || (sig[i] == sig[j] && i < j)) ? 1 : 0;
    pos[j] = pj;
    k += (smax > 0.0 && sig[j] > tol * smax) ? 1 : 0;
  }
  return k;
}

// Fixed-rank mode: at most `cap` of the k kept values (cap <= 0: no cap).  A
// cut that would split a cluster of equal singular values (the first dropped
// value >= (1 - 1e-10) times the last kept one) moves down until it does not:
// the kept subspace of a degenerate cluster is not unique.
template <int R>
__device__ __forceinline__ int cap_rank(const double (&sig)[R], const int (&pos)[R], int k,
                                        int cap) {
  if (cap <= 0 || cap >= k) return k;
  int kk = cap;
  for (int it = 0; it < R && kk > 1; ++it) {
    double first = 0.0, last = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      first = pos[j] == kk ? sig[j] : first;
      last = pos[j] == kk - 1 ? sig[j] : last;
    }
    if (first >= (1.0 - 1e-10) * last) --kk;
    else break;
  }
  return kk;
}

// ---------------------------------------------------------------------------
// Storage conversions
// ---------------------------------------------------------------------------
struct bf16x2c {   // one complex entry as bf16 hi + lo parts
  unsigned short rh, ih, rl, il;
};

__device__ inline unsigned short f2bf_rn(float f) {
  unsigned int u = __float_as_uint(f);
  unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

__device__ inline void store_factor(double2* base, int64_t i, double2 v) { base[i] = v; }
__device__ inline void store_factor(float2* base, int64_t i, double2 v) {
  base[i] = make_float2((float)v.x, (float)v.y);
}
__device__ inline void store_factor(bf16x2c* base, int64_t i, double2 v) {
  float re = (float)v.x, im = (float)v.y;
  unsigned short rh = f2bf_rn(re), ih = f2bf_rn(im);
  unsigned short rl = f2bf_rn((float)(v.x - (double)bf2f(rh)));
  unsigned short il = f2bf_rn((float)(v.y - (double)bf2f(ih)));
  base[i] = bf16x2c{rh, ih, rl, il};
}

__device__ __forceinline__ double2 load_factor(const double2* b, int64_t i) { return b[i]; }
__device__ __forceinline__ float2 load_factor(const float2* b, int64_t i) { return b[i]; }
__device__ __forceinline__ float2 load_factor(const bf16x2c* b, int64_t i) {
  bf16x2c v = b[i];
  return make_float2(bf2f(v.rh) + bf2f(v.rl), bf2f(v.ih) + bf2f(v.il));
}

}  // namespace ibf
