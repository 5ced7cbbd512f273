// Two-dimensional IBF on the boxes of the multiscale IBF (MIBF) of paper
// Sec. 5: Omega = [-W/2, W/2)^2 is split into coronas (eq:domaindecomp), each
// the union of 12 dyadic boxes, plus a centre square summed directly; every
// box carries its own IBF on quadtrees with tensor Chebyshev grids, and the
// results add up (eq:mba, eq:f1).
//
// Geometry of a box of side w (a power of two), L = log2 w: the pair (T_X box
// at level l, T_Omega box at level L - l) has width product 1 per coordinate.
// V pairs the Omega leaves (side 2^lV, level L - lV) with the T_X boxes at
// level lV; U pairs the T_X boxes at level L with the box itself; the middle
// level is h = floor((lV + L) / 2).  Boxes are Morton codes (child digit
// 2 c1 + c2), so the inputs of output pair (a, b) at level l are the four
// contiguous pairs (a >> 2, 4b + c) at level l - 1, and a pair index is
// p = a 4^(L-l) + b.  Tensor grid index t = t1 r + t2.
//
// Compression (Sec. 4.2): every block W (r^2 rows, its columns produced one
// at a time) is reduced to the triangular factor R of W^* = Q R by Givens
// rotations applied as each column arrives (backward stable), and the small
// R^* is orthogonalised by one-sided Jacobi in FP64: W = R^* Q^*, so the left
// singular vectors and singular values of W are those of R^*, accurate to
// rounding in FP64 (no Gram matrix, whose eigenvalues would lose singular
// values below about 1e-8 of the largest).  Rows on lanes: one 32-lane group
// per pair in registers for r <= 5 (r^2 <= 25), one wave per pair with the
// factor in LDS for r = 6 .. 9 (two rows a lane at r = 9).
//
// Kernels: k2_tables (Chebyshev nodes, tensor child->parent Lagrange
// matrices), k2_middle (eq:KeqUMV), k2_sweep_g (eqn:GC), k2_sweep_h (eqn:HR),
// k2_pack_stage, k2_vbar (eqn:V0), k2_ubar, k2_centre; apply (a thread per
// output row and chunk of right-hand sides): k2_apply_v_rows,
// k2_apply_stage_quad, k2_apply_u_tree (the boxes of one X tree together),
// k2_apply_centre_rows (k2_apply_v, k2_apply_stage, k2_apply_centre when the
// staged rows exceed LDS).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ibf_device.h"

namespace ibf {

struct Stage2 {
  int level, kin, kout, kld;
  void* blk;                   // [pair][c kin + s][kld], c = 0..3
  size_t bytes;
};

struct XTree2 {                // X points sorted into the level-L boxes (Morton)
  int L = 0;
  double* d_xs = nullptr;      // [sorted][2]
  int32_t* d_perm = nullptr;   // sorted -> caller
  int32_t* d_leaf = nullptr;   // leaf of each sorted point
};

struct Box2 {
  double o1 = 0, o2 = 0, w = 0;
  int L = 0, lV = 0, h = 0, xt = 0;
  int64_t m = 0;               // Omega points in the box
  double* d_xis = nullptr;     // [sorted][2]
  int32_t* d_perm_xi = nullptr;
  int32_t* d_xileaf = nullptr;
  int32_t* d_xioff = nullptr;  // Omega leaf CSR offsets (4^(L-lV) + 1)
  int smax_xi = 0;              // most points in one Omega leaf
  std::vector<Stage2> stages;  // H stages then G stages, in apply order
  void* d_vbar = nullptr;      // [Omega point][4^lV][K_V]
  void* d_ubar = nullptr;      // [X point (sorted at level L)][K_U]
  int K_V = 0, K_U = 0;
  size_t vbar_bytes = 0, ubar_bytes = 0;
  std::vector<int> rank;       // level maxima, index l - lV
  int64_t nnz_prelim = 0, nnz_opt = 0;
};

// one batched launch of the 2-D apply: V of every box, or stage j of every
// box that has one (descriptor array and block offsets in the plan's table)
struct Launch2 {
  size_t desc_off = 0, boff_off = 0, lds = 0;
  int count = 0;
  int64_t nblocks = 0;
};

struct Mibf2D {
  PhaseDesc ph{};
  int r = 0, R2 = 0, leaf_side = 0, precision = 0, device = 0;
  double tol = 0, W = 0;
  int ssamp = 0;               // > 0: sampled low-rank approximation (columns kept ~ ssamp)
  uint64_t sseed = 0;
  int64_t nx = 0, nxi = 0;
  double* d_x = nullptr;       // caller order [n][2]
  std::vector<XTree2> xtrees;
  std::vector<Box2> boxes;
  std::vector<double> xi_host; // caller order [n][2] (for the box point lists)
  std::vector<std::vector<int32_t>> box_pts;   // caller indices per box
  std::vector<int32_t> centre;                 // caller indices of the centre points
  int32_t* d_cidx = nullptr;
  void* d_kc = nullptr;        // [x][centre point] kernel values, storage precision
  double* d_z = nullptr;       // Chebyshev nodes [r]
  double* d_lc = nullptr;      // [4][R2][R2] child -> parent Lagrange matrices
  void* d_work = nullptr;      // per box two coefficient buffers (apply)
  size_t work_bytes = 0;
  // the boxes' V and stage launches run on worker streams forked from the
  // caller's stream; their U launches accumulate into u in box order
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> ev_u;  // per box: its stages done
  hipEvent_t ev_start = nullptr;
  // the whole launch sequence captured once per (g, u, leading dimensions,
  // nrhs, workspace) on a private stream and replayed on the caller's stream
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int64_t> graph_key;
  bool graph_failed = false;   // capture refused once: direct launches from then on
  // batched launches (V, then one launch per stage index over the boxes),
  // their table written for table_key = (nrhs, workspace); batched == false
  // when some box needs the unbatched kernels
  void* d_table = nullptr;
  size_t table_bytes = 0;
  std::vector<int64_t> table_key;
  std::vector<Launch2> launches;
  bool batched = false;
  bool built = false;
  int64_t nnz_prelim = 0, nnz_opt = 0, nnz_stored = 0, factor_bytes = 0;
  int maxL = 0;
};

namespace {

constexpr int kB2 = 256;
constexpr int kCentreSide = 16;            // centre square side (Sec. 6.3: down to 16 x 16)

struct BoxDev {
  PhaseDesc ph;
  double o1, o2, w;
  int L, lV, h, r;
  int ssamp;                   // > 0: column sampling of the compressed blocks (Sec. 2.1)
  uint64_t sseed;
};

// Randomized low-rank approximation by column sampling (Sec. 2.1): column j
// of pair p in block family `tag` (0 the middle, 1 + l the sweep toward U
// producing level l, 64 + l the one toward V producing level l - 1) is kept
// iff u < min(1, S / n) for its n real columns, u the top 53 bits of the
// (i + 1)-th output of SplitMix64 (Steele, Lea and Flood 2014) started at the
// seed, i = j + 2^9 p + 2^41 tag.  The kept columns' SVD stands for the
// block's, with singular values scaled by sqrt(n / kept).
__device__ __forceinline__ double splitmix64_u(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53;
}
__device__ __forceinline__ bool sample_kept(const BoxDev& B, int tag, int64_t pair, int col,
                                            int nreal) {
  if (B.ssamp <= 0) return true;
  const double rho = fmin(1.0, (double)B.ssamp / (double)(nreal > 1 ? nreal : 1));
  const uint64_t i = (uint64_t)col + ((uint64_t)pair << 9) + ((uint64_t)tag << 41);
  return splitmix64_u(B.sseed, i) < rho;
}
// sqrt(n / kept), 0 when nothing was kept
__device__ __forceinline__ double sample_scale(int nreal, int kept) {
  return kept > 0 ? sqrt((double)nreal / (double)kept) : 0.0;
}

// ---------------------------------------------------------------------------
// 2-D phase (Sec. 6.3) with exact mod-1 reduction of the coordinate products
// ---------------------------------------------------------------------------
__device__ inline double phase_frac2(const PhaseDesc& P, double x1, double x2, double k1,
                                     double k2) {
#pragma clang fp contract(off)
  double t;
  if (P.kind == IBF_PHASE_DFT) {
    t = P.p[0] * (frac_prod(x1, k1) + frac_prod(x2, k2));
  } else if (P.kind == IBF_PHASE_FIO2D) {
    const double s1 = sinpi(2.0 * x1), s2 = sinpi(2.0 * x2);
    const double q1 = cospi(2.0 * x1), q2 = cospi(2.0 * x2);
    const double c1 = (P.p[0] + P.p[1] * s1 * s2) / P.p[2];
    const double c2 = (P.p[0] + P.p[1] * q1 * q2) / P.p[2];
    const double a1 = c1 * k1, a2 = c2 * k2;
    const double root = sqrt(a1 * a1 + a2 * a2);
    t = frac_prod(x1, k1) + frac_prod(x2, k2) + (root - rint(root));
  } else {  // separable: p0 xi1 + p1 xi2
    t = frac_prod(P.p[0], k1) + frac_prod(P.p[1], k2);
  }
  return t - rint(t);
}

__device__ inline double2 kval2(const PhaseDesc& P, double x1, double x2, double k1, double k2) {
  const double t = phase_frac2(P, x1, x2, k1, k2);
  double s, c;
  sincospi(2.0 * t, &s, &c);
  return make_double2(c, s);
}

__device__ inline void morton_xy(int64_t code, int level, int64_t& i1, int64_t& i2) {
  i1 = 0;
  i2 = 0;
  for (int j = 0; j < level; ++j) {
    const int64_t d = (code >> (2 * j)) & 3;
    i1 |= (d >> 1) << j;
    i2 |= (d & 1) << j;
  }
}

__device__ inline void cx2(int level, int64_t a, double& c1, double& c2) {
#pragma clang fp contract(off)
  int64_t i1, i2;
  morton_xy(a, level, i1, i2);
  const double s = ldexp(1.0, -level);
  c1 = ((double)i1 + 0.5) * s;
  c2 = ((double)i2 + 0.5) * s;
}

__device__ inline void cxi2(const BoxDev& B, int level, int64_t b, double& c1, double& c2) {
#pragma clang fp contract(off)
  int64_t j1, j2;
  morton_xy(b, level, j1, j2);
  const double s = B.w / ldexp(1.0, level);
  c1 = B.o1 + ((double)j1 + 0.5) * s;
  c2 = B.o2 + ((double)j2 + 0.5) * s;
}

__device__ inline double gpt(double c, double w, double z) {
#pragma clang fp contract(off)
  return c + w * z;
}

// M_t(y) = M_t1(y1) M_t2(y2) on the tensor grid (t = t1 r + t2)
__device__ inline double lag2(const double* z, int r, int t, double y1, double y2) {
  return lagrange_t(z, r, t / r, y1) * lagrange_t(z, r, t % r, y2);
}

template <int G>
__device__ __forceinline__ double2 shfl2(double2 v, int src) {
  return make_double2(__shfl(v.x, src, G), __shfl(v.y, src, G));
}
template <int G>
__device__ __forceinline__ double2 csum(double2 v) {
  return make_double2(group_sum<G>(v.x), group_sum<G>(v.y));
}

// Lanes per pair of the build kernels for R2 tensor grid points.
template <int R2>
constexpr int group2() { return R2 <= 32 ? 32 : 64; }

// One column of a block W arrives (lane t holds W[t][m]): the row
// a = W[:, m]^* of A = W^* is folded into the upper-triangular R of A = Q R
// by R2 complex Givens rotations.  Lane k holds column k of R (rr[j] =
// R[j][k]) and a_k.  Rotation j mixes row j of R with a so that a_j becomes
// zero: with x = R[j][j], y = a_j, nu = sqrt(|x|^2 + |y|^2),
//   c = |x| / nu,  s = (x / |x|) conj(y) / nu   (c = 0, s = conj(y) / |y| if x = 0),
//   R[j][k] <- c R[j][k] + s a_k,  a_k <- -conj(s) R[j][k] + c a_k.
// Every lane computes c, s from the broadcast x, y (the same numbers); the
// lanes k < j hold zeros on both rows, which stay zero.
template <int R2, int G, int J = 0>
__device__ __forceinline__ void givens_fold(double2 (&rr)[R2], double2& a) {
  if constexpr (J < R2) {
    const double2 x = shfl2<G>(rr[J], J), y = shfl2<G>(a, J);
    const double ax2 = x.x * x.x + x.y * x.y, ay2 = y.x * y.x + y.y * y.y;
    const double ax = sqrt(ax2), nu = sqrt(ax2 + ay2);
    // branch-free: nu = 0 (nothing to eliminate) gives c = 1, s = 0; x = 0
    // gives c = 0, s = conj(y) / |y|
    const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
    const double c = nu > 0.0 ? ax * inv : 1.0;
    const double2 ph = ax > 0.0 ? make_double2(x.x / ax, x.y / ax) : make_double2(1.0, 0.0);
    const double2 sv = cscale(cmul(ph, conjd(y)), inv);
    const double2 rj = rr[J];
    rr[J] = cadd(cscale(rj, c), cmul(sv, a));
    a = cadd(cscale(a, c), cscale(cmul(conjd(sv), rj), -1.0));
    givens_fold<R2, G, J + 1>(rr, a);
  }
}

// Complex Jacobi rotation of columns (p, q) of a matrix held one row per lane.
template <int G>
__device__ __forceinline__ void jrot(double2& ap_, double2& aq_, double& np_, double& nq_,
                                     double thresh, double small, bool& rotated) {
  const double gr = group_sum<G>(ap_.x * aq_.x + ap_.y * aq_.y);
  const double gi = group_sum<G>(ap_.x * aq_.y - ap_.y * aq_.x);
  const double ag = sqrt(gr * gr + gi * gi);
  if (np_ > small && nq_ > small && ag > thresh * sqrt(np_ * nq_)) {
    const double zeta = (nq_ - np_) / (2.0 * ag);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t);
    const double s = c * t;
    const double2 e = make_double2(gr / ag, -gi / ag);
    const double2 eq = cmul(e, aq_);
    const double2 ap = ap_;
    ap_ = make_double2(c * ap.x - s * eq.x, c * ap.y - s * eq.y);
    aq_ = make_double2(s * ap.x + c * eq.x, s * ap.y + c * eq.y);
    np_ -= t * ag;
    nq_ += t * ag;
    rotated = true;
  }
}

template <int R, int G, int P, int Q>
__device__ __forceinline__ void jsweep(double2 (&a)[R], double (&nrm)[R], double thresh,
                                       double small, bool& rotated) {
  if constexpr (P < R - 1) {
    jrot<G>(a[P], a[Q], nrm[P], nrm[Q], thresh, small, rotated);
    if constexpr (Q + 1 < R)
      jsweep<R, G, P, Q + 1>(a, nrm, thresh, small, rotated);
    else
      jsweep<R, G, P + 1, P + 2>(a, nrm, thresh, small, rotated);
  }
}

// One-sided Jacobi on a matrix held one row per lane (columns in a[]):
// afterwards the columns are mutually orthogonal and lam[j] = ||column j||.
template <int R, int G>
__device__ __forceinline__ void jacobi_eig(double2 (&a)[R], double (&lam)[R]) {
  const double thresh = 4.0 * (double)(R > 8 ? R : 8) * 1.1102230246251565e-16;
  double nrm[R];
#pragma unroll
  for (int j = 0; j < R; ++j) nrm[j] = group_sum<G>(a[j].x * a[j].x + a[j].y * a[j].y);
  double fro2 = 0.0;
#pragma unroll
  for (int j = 0; j < R; ++j) fro2 += nrm[j];
  const double small = 1e-30 * fro2;
  for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
    bool rotated = false;
    jsweep<R, G, 0, 1>(a, nrm, thresh, small, rotated);
#pragma unroll
    for (int j = 0; j < R; ++j) nrm[j] = group_sum<G>(a[j].x * a[j].x + a[j].y * a[j].y);
    if (!__any(rotated)) break;
  }
#pragma unroll
  for (int j = 0; j < R; ++j) lam[j] = sqrt(nrm[j]);
}

// v[i] for a lane-dependent i without dynamic register indexing
template <int R, typename T>
__device__ __forceinline__ T sel(const T (&v)[R], int i) {
  T out = v[0];
#pragma unroll
  for (int j = 1; j < R; ++j)
    if (i == j) out = v[j];
  return out;
}

// ---------------------------------------------------------------------------
// Tables: Chebyshev nodes and the tensor child -> parent Lagrange matrices
//   lc[c][t][s] = M^B_t(g^{C_c}_s) = M_t1((2c1-1)/4 + z_s1/2) M_t2((2c2-1)/4 + z_s2/2)
// ---------------------------------------------------------------------------
__global__ void k2_tables(int r, double* z, double* lc) {
  double zz[kMaxR];
  for (int t = 0; t < r; ++t) zz[t] = 0.5 * cos((double)t * M_PI / (double)(r - 1));
  const int R2 = r * r;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < r) z[e] = zz[e];
  if (e >= 4 * R2 * R2) return;
  const int c = e / (R2 * R2), t = (e / R2) % R2, s = e % R2;
  const int c1 = c >> 1, c2 = c & 1;
  double y1, y2;
  {
#pragma clang fp contract(off)
    y1 = (double)(2 * c1 - 1) / 4.0 + zz[s / r] / 2.0;
    y2 = (double)(2 * c2 - 1) / 4.0 + zz[s % r] / 2.0;
  }
  lc[e] = lagrange_t(zz, r, t / r, y1) * lagrange_t(zz, r, t % r, y2);
}

// Thread -> (pair, lane) of the G-lane groups
#define IBF2_GROUP_INDEX                                                        \
  constexpr int G = group2<R2>();                                               \
  const int lane = threadIdx.x & (G - 1);                                       \
  const int64_t p = ((int64_t)blockIdx.x * kB2 + threadIdx.x) / G;              \
  if (p >= npairs) return;                                                      \
  const bool row = lane < R2;

// ---------------------------------------------------------------------------
// Middle level (eq:KeqUMV, eq:lowrankSVD): M~ = K(g^A_t, g^B_s) per pair at h,
// C = U_k S^(1/2), R = V_k S^(1/2) (both [pair][R2][R2], columns in
// descending singular-value order, zero beyond the rank).
// ---------------------------------------------------------------------------
template <int R2>
__global__ __launch_bounds__(kB2) void k2_middle(BoxDev B, const double* __restrict__ z,
                                                 double2* __restrict__ Cb,
                                                 double2* __restrict__ Rb,
                                                 int* __restrict__ rank, int* __restrict__ kmax,
                                                 unsigned long long* __restrict__ nnz,
                                                 int64_t npairs, double tol) {
  IBF2_GROUP_INDEX
  const int r = B.r, L = B.L, h = B.h;
  const int64_t a = p >> (2 * (L - h)), b = p & (((int64_t)1 << (2 * (L - h))) - 1);
  double ca1, ca2, cb1, cb2;
  cx2(h, a, ca1, ca2);
  cxi2(B, L - h, b, cb1, cb2);
  const double wa = ldexp(1.0, -h), wb = B.w / ldexp(1.0, L - h);
  const int tl = row ? lane : 0;
  const double ga1 = gpt(ca1, wa, z[tl / r]), ga2 = gpt(ca2, wa, z[tl % r]);
  // M^* = Q R by Givens rotations, one column of M at a time; gram = R^*
  double2 gram[R2];
#pragma unroll
  for (int j = 0; j < R2; ++j) gram[j] = make_double2(0.0, 0.0);
  int kept = 0;
  for (int s = 0; s < R2; ++s) {
    if (!sample_kept(B, 0, p, s, R2)) continue;
    ++kept;
    const double2 w = row ? kval2(B.ph, ga1, ga2, gpt(cb1, wb, z[s / r]), gpt(cb2, wb, z[s % r]))
                          : make_double2(0.0, 0.0);
    double2 av = conjd(w);
    givens_fold<R2, G>(gram, av);
  }
#pragma unroll
  for (int j = 0; j < R2; ++j) gram[j] = conjd(gram[j]);
  // columns of R^* orthogonalised: column j = sigma_j u_j, sig[j] = sigma_j
  double sig[R2];
  jacobi_eig<R2, G>(gram, sig);
  int pos[R2];
  const int k = rank_positions<R2>(sig, tol, pos);
  if (B.ssamp > 0) {                                     // sampled: scale to the block
    const double f = sample_scale(R2, kept);
#pragma unroll
    for (int j = 0; j < R2; ++j) {
      gram[j] = cscale(gram[j], f);
      sig[j] *= f;
    }
  }
  // C row t: u_j[t] sigma_j^(1/2)
  double2* crow = Cb + (p * R2 + tl) * R2;
#pragma unroll
  for (int j = 0; j < R2; ++j) {
    const bool keep = pos[j] < k && sig[j] > 0.0;
    const double sc = keep ? 1.0 / sqrt(sig[j]) : 0.0;
    if (row) crow[pos[j]] = cscale(gram[j], sc);
  }
  // R row s: (sum_t conj(M[t][s]) sigma_j u_j[t]) sigma_j^(-3/2) = v_j[s] sigma_j^(1/2);
  // lane j keeps column j
  const int my_pos = sel<R2>(pos, tl);
  const double my_sig = sel<R2>(sig, tl);
  const double my_sc = (my_pos < k && my_sig > 0.0) ? pow(my_sig, -1.5) : 0.0;
  for (int s = 0; s < R2; ++s) {
    const double2 mts = row ? kval2(B.ph, ga1, ga2, gpt(cb1, wb, z[s / r]), gpt(cb2, wb, z[s % r]))
                            : make_double2(0.0, 0.0);
    double2 mine = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < R2; ++j) {
      const double2 v = csum<G>(cmul(conjd(mts), gram[j]));
      if (lane == j) mine = v;
    }
    if (row) Rb[(p * R2 + s) * R2 + my_pos] = cscale(mine, my_sc);
  }
  if (lane == 0) {
    rank[p] = k;
    atomicMax(kmax, k);
    atomicAdd(nnz, (unsigned long long)k);
  }
}

// ---------------------------------------------------------------------------
// Sweep toward U (eqn:GC) at output level l: per output pair (a, b),
//   W = [G_c C^{l-1}_{(a>>2, 4b+c)}]_c,  G_c[t][s] = K(g^A_t, c_C) M^P_s(g^A_t) conj K(g^P_s, c_C),
//   W ~= C^l [Gbar_0 .. Gbar_3],  C^l = U_k S_k,  Gbar = S_k^-1 U_k^* W.
// Gbar goes to stage[p][c][t = output rank index][s = input rank index] (FP64).
// ---------------------------------------------------------------------------
template <int R2>
__global__ __launch_bounds__(kB2) void k2_sweep_g(BoxDev B, int l, const double* __restrict__ z,
                                                  const double* __restrict__ lc,
                                                  const double2* __restrict__ Cprev,
                                                  const int* __restrict__ rprev,
                                                  double2* __restrict__ Cout,
                                                  int* __restrict__ rout, int* __restrict__ kmax,
                                                  double2* __restrict__ stage,
                                                  unsigned long long* __restrict__ nnz,
                                                  int64_t npairs, double tol) {
  __shared__ double lcs[4 * R2 * R2];
  for (int e = threadIdx.x; e < 4 * R2 * R2; e += kB2) lcs[e] = lc[e];
  __syncthreads();
  IBF2_GROUP_INDEX
  const int r = B.r, L = B.L;
  const int sh = 2 * (L - l);
  const int64_t a = p >> sh, b = p & (((int64_t)1 << sh) - 1);
  const int64_t par = a >> 2;
  const int alpha = (int)(a & 3);
  const int64_t pin0 = (par << (sh + 2)) + 4 * b;
  double ca1, ca2, cp1, cp2;
  cx2(l, a, ca1, ca2);
  cx2(l - 1, par, cp1, cp2);
  const double wa = ldexp(1.0, -l), wp = ldexp(1.0, -(l - 1));
  const int tl = row ? lane : 0;
  const double ga1 = gpt(ca1, wa, z[tl / r]), ga2 = gpt(ca2, wa, z[tl % r]);
  const double gp1 = gpt(cp1, wp, z[tl / r]), gp2 = gpt(cp2, wp, z[tl % r]);
  const double* la = lcs + alpha * R2 * R2;             // la[s * R2 + t] = M^P_s(g^A_t)
  int kin[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) kin[c] = rprev[pin0 + c];
  // W_c[t][m] for this lane's row t
  auto wcol = [&](int c, int m, double2 at, double2 bs) -> double2 {
    const double2* cs = Cprev + (pin0 + c) * R2 * R2 + m;
    double2 acc = make_double2(0.0, 0.0);
    for (int s = 0; s < R2; ++s)
      cfma(acc, cscale(shfl2<G>(bs, s), la[s * R2 + tl]), cs[s * R2]);
    return row ? cmul(at, acc) : make_double2(0.0, 0.0);
  };
  double2 gram[R2];
#pragma unroll
  for (int j = 0; j < R2; ++j) gram[j] = make_double2(0.0, 0.0);
  double2 at[4], bs[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double cc1, cc2;
    cxi2(B, L - l + 1, 4 * b + c, cc1, cc2);
    at[c] = kval2(B.ph, ga1, ga2, cc1, cc2);
    bs[c] = conjd(kval2(B.ph, gp1, gp2, cc1, cc2));    // lane s holds B_s
  }
  // W^* = Q R by Givens rotations, one column of W at a time; gram = R^*
  const int nreal = kin[0] + kin[1] + kin[2] + kin[3];
  int kept = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    for (int m = 0; m < kin[c]; ++m) {
      if (!sample_kept(B, 1 + l, p, c * R2 + m, nreal)) continue;
      ++kept;
      double2 av = conjd(wcol(c, m, at[c], bs[c]));
      givens_fold<R2, G>(gram, av);
    }
#pragma unroll
  for (int j = 0; j < R2; ++j) gram[j] = conjd(gram[j]);
  double sig[R2];
  jacobi_eig<R2, G>(gram, sig);                          // column j = sigma_j u_j
  int pos[R2];
  const int k = rank_positions<R2>(sig, tol, pos);
  if (B.ssamp > 0) {
    const double f = sample_scale(nreal, kept);
#pragma unroll
    for (int j = 0; j < R2; ++j) {
      gram[j] = cscale(gram[j], f);
      sig[j] *= f;
    }
  }
  double2* crow = Cout + (p * R2 + tl) * R2;             // C^l = U_k S_k
#pragma unroll
  for (int j = 0; j < R2; ++j) {
    const bool keep = pos[j] < k && sig[j] > 0.0;
    if (row) crow[pos[j]] = keep ? gram[j] : make_double2(0.0, 0.0);
  }
  // Gbar row j = sigma_j^-1 u_j^* W = (sigma_j u_j)^* W sigma_j^-2
  const int my_pos = sel<R2>(pos, tl);
  const double my_sig = sel<R2>(sig, tl);
  const double my_sc = (my_pos < k && my_sig > 0.0) ? 1.0 / (my_sig * my_sig) : 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double2* st = stage + (p * 4 + c) * R2 * R2;
    for (int m = 0; m < R2; ++m) {
      if (m < kin[c]) {
        const double2 w = wcol(c, m, at[c], bs[c]);
        double2 mine = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < R2; ++j) {
          const double2 v = csum<G>(cmul(conjd(gram[j]), w));
          if (lane == j) mine = v;
        }
        if (row) st[my_pos * R2 + m] = cscale(mine, my_sc);
      } else if (row) {
        st[tl * R2 + m] = make_double2(0.0, 0.0);
      }
    }
  }
  if (lane == 0) {
    rout[p] = k;
    atomicMax(kmax, k);
    atomicAdd(nnz, (unsigned long long)k * (kin[0] + kin[1] + kin[2] + kin[3]));
  }
}

// ---------------------------------------------------------------------------
// Sweep toward V (eqn:HR) producing R^{l-1}: per input pair q = (P, C) at
// level l - 1 with C = 4B + c, the outputs are (A_alpha = 4P + alpha, B) at l:
//   Z = [H_alpha^* R^l_{(A_alpha, B)}]_alpha,
//   H_alpha^*[s][t] = conj K(c_A, g^C_s) M^B_t(g^C_s) K(c_A, g^B_t),
//   Z ~= R^{l-1} [Hbar_alpha],  R^{l-1} = U_k S_k,  Hbar^* rows = (Z^* U_k S_k^-1).
// The block of output (A_alpha, B), child c, row m (output rank index),
// column j (input rank index) goes to stage[pout][c][m][j].
// ---------------------------------------------------------------------------
template <int R2>
__global__ __launch_bounds__(kB2) void k2_sweep_h(BoxDev B, int l, const double* __restrict__ z,
                                                  const double* __restrict__ lc,
                                                  const double2* __restrict__ Rcur,
                                                  const int* __restrict__ rcur,
                                                  double2* __restrict__ Rnext,
                                                  int* __restrict__ rnext, int* __restrict__ kmax,
                                                  double2* __restrict__ stage,
                                                  unsigned long long* __restrict__ nnz,
                                                  int64_t npairs, double tol) {
  __shared__ double lcs[4 * R2 * R2];
  for (int e = threadIdx.x; e < 4 * R2 * R2; e += kB2) lcs[e] = lc[e];
  __syncthreads();
  IBF2_GROUP_INDEX
  const int r = B.r, L = B.L;
  const int shq = 2 * (L - l + 1);
  const int64_t q = p;
  const int64_t P = q >> shq, C = q & (((int64_t)1 << shq) - 1);
  const int64_t Bb = C >> 2;
  const int c = (int)(C & 3);
  double cc1, cc2, cb1, cb2;
  cxi2(B, L - l + 1, C, cc1, cc2);
  cxi2(B, L - l, Bb, cb1, cb2);
  const double wc = B.w / ldexp(1.0, L - l + 1), wb = B.w / ldexp(1.0, L - l);
  const int sl = row ? lane : 0;
  const double gc1 = gpt(cc1, wc, z[sl / r]), gc2 = gpt(cc2, wc, z[sl % r]);
  const double gb1 = gpt(cb1, wb, z[sl / r]), gb2 = gpt(cb2, wb, z[sl % r]);
  const double* lcc = lcs + c * R2 * R2;                 // lcc[t * R2 + s] = M^B_t(g^C_s)
  int64_t pout[4];
  int kout[4];
  double2 ds[4], et[4];
#pragma unroll
  for (int al = 0; al < 4; ++al) {
    const int64_t A = 4 * P + al;
    pout[al] = (A << (2 * (L - l))) + Bb;
    kout[al] = rcur[pout[al]];
    double ca1, ca2;
    cx2(l, A, ca1, ca2);
    ds[al] = conjd(kval2(B.ph, ca1, ca2, gc1, gc2));      // this lane's row s
    et[al] = kval2(B.ph, ca1, ca2, gb1, gb2);             // lane t holds E_t
  }
  auto zcol = [&](int al, int m) -> double2 {
    const double2* rs = Rcur + pout[al] * R2 * R2 + m;
    double2 acc = make_double2(0.0, 0.0);
    for (int t = 0; t < R2; ++t)
      cfma(acc, cscale(shfl2<G>(et[al], t), lcc[t * R2 + sl]), rs[t * R2]);
    return row ? cmul(ds[al], acc) : make_double2(0.0, 0.0);
  };
  // Z^* = Q R by Givens rotations, one column of Z at a time; gram = R^*
  double2 gram[R2];
#pragma unroll
  for (int j = 0; j < R2; ++j) gram[j] = make_double2(0.0, 0.0);
  const int nreal = kout[0] + kout[1] + kout[2] + kout[3];
  int kept = 0;
#pragma unroll
  for (int al = 0; al < 4; ++al)
    for (int m = 0; m < kout[al]; ++m) {
      if (!sample_kept(B, 64 + l, q, al * R2 + m, nreal)) continue;
      ++kept;
      double2 av = conjd(zcol(al, m));
      givens_fold<R2, G>(gram, av);
    }
#pragma unroll
  for (int j = 0; j < R2; ++j) gram[j] = conjd(gram[j]);
  double sig[R2];
  jacobi_eig<R2, G>(gram, sig);                          // column j = sigma_j u_j
  int pos[R2];
  const int k = rank_positions<R2>(sig, tol, pos);
  if (B.ssamp > 0) {
    const double f = sample_scale(nreal, kept);
#pragma unroll
    for (int j = 0; j < R2; ++j) {
      gram[j] = cscale(gram[j], f);
      sig[j] *= f;
    }
  }
  double2* rrow = Rnext + (q * R2 + sl) * R2;            // R^{l-1} = U_k S_k
#pragma unroll
  for (int j = 0; j < R2; ++j) {
    const bool keep = pos[j] < k && sig[j] > 0.0;
    if (row) rrow[pos[j]] = keep ? gram[j] : make_double2(0.0, 0.0);
  }
  const int my_pos = sel<R2>(pos, sl);
  const double my_sig = sel<R2>(sig, sl);
  const double my_sc = (my_pos < k && my_sig > 0.0) ? 1.0 / (my_sig * my_sig) : 0.0;
#pragma unroll
  for (int al = 0; al < 4; ++al) {
    double2* st = stage + (pout[al] * 4 + c) * R2 * R2;
    for (int m = 0; m < R2; ++m) {
      if (m < kout[al]) {
        const double2 w = zcol(al, m);
        double2 mine = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < R2; ++j) {
          const double2 v = csum<G>(cmul(conjd(gram[j]), w));
          if (lane == j) mine = v;
        }
        if (row) st[m * R2 + my_pos] = cscale(conjd(mine), my_sc);
      } else if (row) {
        st[m * R2 + sl] = make_double2(0.0, 0.0);
      }
    }
  }
  if (lane == 0) {
    rnext[q] = k;
    atomicMax(kmax, k);
    atomicAdd(nnz, (unsigned long long)k * (kout[0] + kout[1] + kout[2] + kout[3]));
  }
}

// ---------------------------------------------------------------------------
// Build kernels for 36 to 81 tensor grid points (r = 6 .. 9).  The arithmetic
// is that of the kernels above (streaming Givens QR of W^*, then one-sided
// Jacobi on R^*, one pair a wave), but the triangular factor R and then the
// columns of R^* live in LDS and the Givens folds and the Jacobi rotations
// run as loops: in registers they would need R2 complex values a lane and
// R2 (R2 - 1) / 2 unrolled rotations.  A lane holds the rows (and columns)
// k = lane + 64 h, h < RPL (two for 81 points).  Entry (j, k) of a wave's
// matrix is at LDS j S + k (S = 64, or R2 when a lane holds two); a block
// holds NW waves (pairs) of R2 S complex + R2 real values each.  The child
// -> parent Lagrange table is read from memory (it would not fit beside the
// factors).
// ---------------------------------------------------------------------------
constexpr int kWaveL = 64;
template <int R2>
constexpr int k2l_rpl() { return R2 > kWaveL ? 2 : 1; }
template <int R2>
constexpr int k2l_stride() { return R2 > kWaveL ? R2 : kWaveL; }
template <int R2>
constexpr size_t k2l_wave_lds() {                                 // 16-byte aligned per wave
  return ((size_t)R2 * k2l_stride<R2>() * sizeof(double2) + R2 * (sizeof(double) + sizeof(int)) +
          15) & ~(size_t)15;
}

__device__ __forceinline__ double rl_d(double v, int j) {        // lane j's v (j uniform)
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, j);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), j);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double2 rl2(double2 v, int j) {
  return make_double2(rl_d(v.x, j), rl_d(v.y, j));
}
// entry k (uniform) of a lane-distributed vector v[h] = component lane + 64 h
template <int RPL>
__device__ __forceinline__ double2 rl_k(const double2 (&v)[RPL], int k) {
  return (RPL > 1 && k >= kWaveL) ? rl2(v[RPL - 1], k - kWaveL) : rl2(v[0], k);
}

// givens_fold with R's rows in LDS (gm: the wave's matrix; row J at J S)
template <int R2>
__device__ __forceinline__ void givens_fold_l(double2* gm, int lane,
                                              double2 (&a)[k2l_rpl<R2>()]) {
  constexpr int RPL = k2l_rpl<R2>(), S = k2l_stride<R2>();
#pragma unroll 2
  for (int J = 0; J < R2; ++J) {
    double2 rj[RPL];
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
      const int k = lane + kWaveL * h;
      rj[h] = k < R2 ? gm[J * S + k] : make_double2(0.0, 0.0);
    }
    const double2 x = rl_k<RPL>(rj, J), y = rl_k<RPL>(a, J);
    const double ax2 = x.x * x.x + x.y * x.y, ay2 = y.x * y.x + y.y * y.y;
    const double ax = sqrt(ax2), nu = sqrt(ax2 + ay2);
    const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
    const double c = nu > 0.0 ? ax * inv : 1.0;
    const double2 ph = ax > 0.0 ? make_double2(x.x / ax, x.y / ax) : make_double2(1.0, 0.0);
    const double2 sv = cscale(cmul(ph, conjd(y)), inv);
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
      const int k = lane + kWaveL * h;
      if (k < R2) gm[J * S + k] = cadd(cscale(rj[h], c), cmul(sv, a[h]));
      a[h] = cadd(cscale(a[h], c), cscale(cmul(conjd(sv), rj[h]), -1.0));
    }
  }
}

// Complex Jacobi rotation of columns (p, q) whose rows are spread RPL a lane
template <int RPL>
__device__ __forceinline__ void jrot_l(double2 (&ap_)[RPL], double2 (&aq_)[RPL], double& np_,
                                       double& nq_, double thresh, double small, bool& rotated) {
  double pr = 0.0, pi = 0.0;
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    pr += ap_[h].x * aq_[h].x + ap_[h].y * aq_[h].y;
    pi += ap_[h].x * aq_[h].y - ap_[h].y * aq_[h].x;
  }
  const double gr = group_sum<kWaveL>(pr);
  const double gi = group_sum<kWaveL>(pi);
  const double ag = sqrt(gr * gr + gi * gi);
  if (np_ > small && nq_ > small && ag > thresh * sqrt(np_ * nq_)) {
    const double zeta = (nq_ - np_) / (2.0 * ag);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t);
    const double s = c * t;
    const double2 e = make_double2(gr / ag, -gi / ag);
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
      const double2 eq = cmul(e, aq_[h]);
      const double2 ap = ap_[h];
      ap_[h] = make_double2(c * ap.x - s * eq.x, c * ap.y - s * eq.y);
      aq_[h] = make_double2(s * ap.x + c * eq.x, s * ap.y + c * eq.y);
    }
    np_ -= t * ag;
    nq_ += t * ag;
    rotated = true;
  }
}

// jacobi_eig with the columns in LDS (column j at gm[j S + k], row k) and
// their squared norms in nl[j] (the same in every lane)
template <int R2>
__device__ __forceinline__ void jacobi_eig_l(double2* gm, double* nl, int lane) {
  constexpr int RPL = k2l_rpl<R2>(), S = k2l_stride<R2>();
  const double thresh = 4.0 * (double)(R2 > 8 ? R2 : 8) * 1.1102230246251565e-16;
  auto load = [&](int j, double2 (&v)[RPL]) {
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
      const int k = lane + kWaveL * h;
      v[h] = k < R2 ? gm[j * S + k] : make_double2(0.0, 0.0);
    }
  };
  auto store = [&](int j, const double2 (&v)[RPL]) {
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
      const int k = lane + kWaveL * h;
      if (k < R2) gm[j * S + k] = v[h];
    }
  };
  auto norms = [&]() {
    for (int j = 0; j < R2; ++j) {
      double2 v[RPL];
      load(j, v);
      double s2 = 0.0;
#pragma unroll
      for (int h = 0; h < RPL; ++h) s2 += v[h].x * v[h].x + v[h].y * v[h].y;
      nl[j] = group_sum<kWaveL>(s2);
    }
  };
  norms();
  double fro2 = 0.0;
  for (int j = 0; j < R2; ++j) fro2 += nl[j];
  const double small = 1e-30 * fro2;
  for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < R2 - 1; ++p) {
      double2 ap[RPL];
      load(p, ap);
      double np = nl[p];
      for (int q = p + 1; q < R2; ++q) {
        double2 aq[RPL];
        load(q, aq);
        double nq = nl[q];
        jrot_l<RPL>(ap, aq, np, nq, thresh, small, rotated);
        store(q, aq);
        nl[q] = nq;
      }
      store(p, ap);
      nl[p] = np;
    }
    norms();
    if (!__any(rotated)) break;
  }
}

// rank_positions on the LDS norms: pl[j] = position of column j in
// descending order of sigma_j = sqrt(nl[j]) (ties by index); returns the
// number of sigma_j > tol * max sigma (the same comparisons in the same
// precision as the register kernels)
template <int R2>
__device__ __forceinline__ int k2l_rank(const double* nl, int* pl, int lane, double tol) {
  double smax = 0.0;
  for (int i = 0; i < R2; ++i) smax = fmax(smax, sqrt(nl[i]));
  int k = 0;
  for (int i = 0; i < R2; ++i) k += (smax > 0.0 && sqrt(nl[i]) > tol * smax) ? 1 : 0;
#pragma unroll
  for (int h = 0; h < k2l_rpl<R2>(); ++h) {
    const int j = lane + kWaveL * h;
    if (j < R2) {
      const double sj = sqrt(nl[j]);
      int cnt = 0;
      for (int i = 0; i < R2; ++i) {
        const double si = sqrt(nl[i]);
        cnt += (si > sj || (si == sj && i < j)) ? 1 : 0;
      }
      pl[j] = cnt;
    }
  }
  return k;
}

// sampled blocks: the kept columns' singular values and left vectors scaled
// to the block's (after the rank and positions are taken from the unscaled
// values, as in the oracle)
template <int R2>
__device__ __forceinline__ void k2l_scale(double2* gm, double* nl, int lane, const BoxDev& B,
                                          int nreal, int kept) {
  if (B.ssamp <= 0) return;
  const double f = sample_scale(nreal, kept);
  for (int e = lane; e < R2 * k2l_stride<R2>(); e += kWaveL) gm[e] = cscale(gm[e], f);
  for (int j = 0; j < R2; ++j) nl[j] *= f * f;
}

// entry (j, row k) of the wave's matrix, zero past the rows
template <int R2>
__device__ __forceinline__ double2 k2l_at(const double2* gm, int j, int k) {
  return k < R2 ? gm[j * k2l_stride<R2>() + k] : make_double2(0.0, 0.0);
}
// sum over the rows of conj(column j) . w (w[h] at row lane + 64 h)
template <int R2>
__device__ __forceinline__ double2 k2l_dot(const double2* gm, int j, int lane,
                                           const double2 (&w)[k2l_rpl<R2>()]) {
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int h = 0; h < k2l_rpl<R2>(); ++h)
    acc = cadd(acc, cmul(conjd(k2l_at<R2>(gm, j, lane + kWaveL * h)), w[h]));
  return csum<kWaveL>(acc);
}

#define IBF2L_WAVE_INDEX                                                        \
  constexpr int RPL = k2l_rpl<R2>();                                            \
  extern __shared__ __align__(16) unsigned char smem2l[];                       \
  const int lane = threadIdx.x & (kWaveL - 1);                                  \
  const int wv = threadIdx.x / kWaveL;                                          \
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x / kWaveL) + wv;           \
  if (p >= npairs) return;                                                      \
  double2* gm = reinterpret_cast<double2*>(smem2l + wv * k2l_wave_lds<R2>());   \
  double* nl = reinterpret_cast<double*>(smem2l + wv * k2l_wave_lds<R2>() +     \
                                         (size_t)R2 * k2l_stride<R2>() * sizeof(double2)); \
  int* pl = reinterpret_cast<int*>(nl + R2);                                    \
  for (int e = lane; e < R2 * k2l_stride<R2>(); e += kWaveL) gm[e] = make_double2(0.0, 0.0);

template <int R2>
__global__ __launch_bounds__(256) void k2l_middle(BoxDev B, const double* __restrict__ z,
                                                  double2* __restrict__ Cb,
                                                  double2* __restrict__ Rb,
                                                  int* __restrict__ rank, int* __restrict__ kmax,
                                                  unsigned long long* __restrict__ nnz,
                                                  int64_t npairs, double tol) {
  IBF2L_WAVE_INDEX
  const int r = B.r, L = B.L, h0 = B.h;
  const int64_t a = p >> (2 * (L - h0)), b = p & (((int64_t)1 << (2 * (L - h0))) - 1);
  double ca1, ca2, cb1, cb2;
  cx2(h0, a, ca1, ca2);
  cxi2(B, L - h0, b, cb1, cb2);
  const double wa = ldexp(1.0, -h0), wb = B.w / ldexp(1.0, L - h0);
  double ga1[RPL], ga2[RPL];
  bool row[RPL];
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int t = lane + kWaveL * h;
    row[h] = t < R2;
    const int tl = row[h] ? t : 0;
    ga1[h] = gpt(ca1, wa, z[tl / r]);
    ga2[h] = gpt(ca2, wa, z[tl % r]);
  }
  auto mcol = [&](int s, double2 (&w)[RPL]) {
    const double gb1 = gpt(cb1, wb, z[s / r]), gb2 = gpt(cb2, wb, z[s % r]);
#pragma unroll
    for (int h = 0; h < RPL; ++h)
      w[h] = row[h] ? kval2(B.ph, ga1[h], ga2[h], gb1, gb2) : make_double2(0.0, 0.0);
  };
  int kept = 0;
  for (int s = 0; s < R2; ++s) {
    if (!sample_kept(B, 0, p, s, R2)) continue;
    ++kept;
    double2 av[RPL];
    mcol(s, av);
#pragma unroll
    for (int h = 0; h < RPL; ++h) av[h] = conjd(av[h]);
    givens_fold_l<R2>(gm, lane, av);
  }
  for (int e = lane; e < R2 * k2l_stride<R2>(); e += kWaveL) gm[e] = conjd(gm[e]);
  jacobi_eig_l<R2>(gm, nl, lane);
  const int k = k2l_rank<R2>(nl, pl, lane, tol);
  k2l_scale<R2>(gm, nl, lane, B, R2, kept);
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int t = lane + kWaveL * h;
    if (!row[h]) continue;
    double2* crow = Cb + (p * R2 + t) * R2;
    for (int j = 0; j < R2; ++j) {
      const double sj = sqrt(nl[j]);
      const int pj = pl[j];
      const bool keep = pj < k && sj > 0.0;
      const double sc = keep ? 1.0 / sqrt(sj) : 0.0;
      crow[pj] = cscale(k2l_at<R2>(gm, j, t), sc);
    }
  }
  for (int s = 0; s < R2; ++s) {
    double2 mts[RPL];
    mcol(s, mts);
#pragma unroll
    for (int h = 0; h < RPL; ++h) mts[h] = conjd(mts[h]);
    // column j of R^* dotted with conj(M[:, s]): lane j % 64 keeps it
    for (int j = 0; j < R2; ++j) {
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int h = 0; h < RPL; ++h)
        acc = cadd(acc, cmul(mts[h], k2l_at<R2>(gm, j, lane + kWaveL * h)));
      const double2 v = csum<kWaveL>(acc);
      if (lane == (j & (kWaveL - 1))) {
        const int pj = pl[j];
        const double sj = sqrt(nl[j]);
        const double sc = (pj < k && sj > 0.0) ? pow(sj, -1.5) : 0.0;
        Rb[(p * R2 + s) * R2 + pj] = cscale(v, sc);
      }
    }
  }
  if (lane == 0) {
    rank[p] = k;
    atomicMax(kmax, k);
    atomicAdd(nnz, (unsigned long long)k);
  }
}

template <int R2>
__global__ __launch_bounds__(256) void k2l_sweep_g(BoxDev B, int l, const double* __restrict__ z,
                                                   const double* __restrict__ lc,
                                                   const double2* __restrict__ Cprev,
                                                   const int* __restrict__ rprev,
                                                   double2* __restrict__ Cout,
                                                   int* __restrict__ rout, int* __restrict__ kmax,
                                                   double2* __restrict__ stage,
                                                   unsigned long long* __restrict__ nnz,
                                                   int64_t npairs, double tol) {
  IBF2L_WAVE_INDEX
  const int r = B.r, L = B.L;
  const int sh = 2 * (L - l);
  const int64_t a = p >> sh, b = p & (((int64_t)1 << sh) - 1);
  const int64_t par = a >> 2;
  const int alpha = (int)(a & 3);
  const int64_t pin0 = (par << (sh + 2)) + 4 * b;
  double ca1, ca2, cp1, cp2;
  cx2(l, a, ca1, ca2);
  cx2(l - 1, par, cp1, cp2);
  const double wa = ldexp(1.0, -l), wp = ldexp(1.0, -(l - 1));
  const double* la = lc + alpha * R2 * R2;               // la[s * R2 + t] = M^P_s(g^A_t)
  int kin[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) kin[c] = rprev[pin0 + c];
  bool row[RPL];
  int tl[RPL];
  double2 at[4][RPL], bs[4][RPL];
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int t = lane + kWaveL * h;
    row[h] = t < R2;
    tl[h] = row[h] ? t : 0;
    const double ga1 = gpt(ca1, wa, z[tl[h] / r]), ga2 = gpt(ca2, wa, z[tl[h] % r]);
    const double gp1 = gpt(cp1, wp, z[tl[h] / r]), gp2 = gpt(cp2, wp, z[tl[h] % r]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double cc1, cc2;
      cxi2(B, L - l + 1, 4 * b + c, cc1, cc2);
      at[c][h] = kval2(B.ph, ga1, ga2, cc1, cc2);
      bs[c][h] = conjd(kval2(B.ph, gp1, gp2, cc1, cc2));   // entry s = lane + 64 h: B_s
    }
  }
  // W_c[t][m] for this lane's rows t
  auto wcol = [&](int c, int m, double2 (&w)[RPL]) {
    const double2* cs = Cprev + (pin0 + c) * R2 * R2 + m;
    double2 acc[RPL];
#pragma unroll
    for (int h = 0; h < RPL; ++h) acc[h] = make_double2(0.0, 0.0);
    for (int s = 0; s < R2; ++s) {
      const double2 bsv = rl_k<RPL>(bs[c], s);
      const double2 cv = cs[s * R2];
#pragma unroll
      for (int h = 0; h < RPL; ++h) cfma(acc[h], cscale(bsv, la[s * R2 + tl[h]]), cv);
    }
#pragma unroll
    for (int h = 0; h < RPL; ++h) w[h] = row[h] ? cmul(at[c][h], acc[h]) : make_double2(0.0, 0.0);
  };
  const int nreal = kin[0] + kin[1] + kin[2] + kin[3];
  int kept = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    for (int m = 0; m < kin[c]; ++m) {
      if (!sample_kept(B, 1 + l, p, c * R2 + m, nreal)) continue;
      ++kept;
      double2 av[RPL];
      wcol(c, m, av);
#pragma unroll
      for (int h = 0; h < RPL; ++h) av[h] = conjd(av[h]);
      givens_fold_l<R2>(gm, lane, av);
    }
  for (int e = lane; e < R2 * k2l_stride<R2>(); e += kWaveL) gm[e] = conjd(gm[e]);
  jacobi_eig_l<R2>(gm, nl, lane);
  const int k = k2l_rank<R2>(nl, pl, lane, tol);
  k2l_scale<R2>(gm, nl, lane, B, nreal, kept);
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    if (!row[h]) continue;
    double2* crow = Cout + (p * R2 + tl[h]) * R2;        // C^l = U_k S_k
    for (int j = 0; j < R2; ++j) {
      const bool keep = pl[j] < k && sqrt(nl[j]) > 0.0;
      crow[pl[j]] = keep ? k2l_at<R2>(gm, j, tl[h]) : make_double2(0.0, 0.0);
    }
  }
  // Gbar row j = sigma_j^-2 (sigma_j u_j)^* W; lane j % 64 keeps column j
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double2* st = stage + (p * 4 + c) * R2 * R2;
    for (int m = 0; m < R2; ++m) {
      if (m < kin[c]) {
        double2 w[RPL];
        wcol(c, m, w);
        for (int j = 0; j < R2; ++j) {
          const double2 v = k2l_dot<R2>(gm, j, lane, w);
          if (lane == (j & (kWaveL - 1))) {
            const int pj = pl[j];
            const double sj = sqrt(nl[j]);
            const double sc = (pj < k && sj > 0.0) ? 1.0 / (sj * sj) : 0.0;
            st[pj * R2 + m] = cscale(v, sc);
          }
        }
      } else {
#pragma unroll
        for (int h = 0; h < RPL; ++h)
          if (row[h]) st[tl[h] * R2 + m] = make_double2(0.0, 0.0);
      }
    }
  }
  if (lane == 0) {
    rout[p] = k;
    atomicMax(kmax, k);
    atomicAdd(nnz, (unsigned long long)k * (kin[0] + kin[1] + kin[2] + kin[3]));
  }
}

template <int R2>
__global__ __launch_bounds__(256) void k2l_sweep_h(BoxDev B, int l, const double* __restrict__ z,
                                                   const double* __restrict__ lc,
                                                   const double2* __restrict__ Rcur,
                                                   const int* __restrict__ rcur,
                                                   double2* __restrict__ Rnext,
                                                   int* __restrict__ rnext, int* __restrict__ kmax,
                                                   double2* __restrict__ stage,
                                                   unsigned long long* __restrict__ nnz,
                                                   int64_t npairs, double tol) {
  IBF2L_WAVE_INDEX
  const int r = B.r, L = B.L;
  const int shq = 2 * (L - l + 1);
  const int64_t q = p;
  const int64_t P = q >> shq, C = q & (((int64_t)1 << shq) - 1);
  const int64_t Bb = C >> 2;
  const int c = (int)(C & 3);
  double cc1, cc2, cb1, cb2;
  cxi2(B, L - l + 1, C, cc1, cc2);
  cxi2(B, L - l, Bb, cb1, cb2);
  const double wc = B.w / ldexp(1.0, L - l + 1), wb = B.w / ldexp(1.0, L - l);
  const double* lcc = lc + c * R2 * R2;                  // lcc[t * R2 + s] = M^B_t(g^C_s)
  int64_t pout[4];
  int kout[4];
#pragma unroll
  for (int al = 0; al < 4; ++al) {
    const int64_t A = 4 * P + al;
    pout[al] = (A << (2 * (L - l))) + Bb;
    kout[al] = rcur[pout[al]];
  }
  bool row[RPL];
  int sl[RPL];
  double2 ds[4][RPL], et[4][RPL];
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int s = lane + kWaveL * h;
    row[h] = s < R2;
    sl[h] = row[h] ? s : 0;
    const double gc1 = gpt(cc1, wc, z[sl[h] / r]), gc2 = gpt(cc2, wc, z[sl[h] % r]);
    const double gb1 = gpt(cb1, wb, z[sl[h] / r]), gb2 = gpt(cb2, wb, z[sl[h] % r]);
#pragma unroll
    for (int al = 0; al < 4; ++al) {
      const int64_t A = 4 * P + al;
      double ca1, ca2;
      cx2(l, A, ca1, ca2);
      ds[al][h] = conjd(kval2(B.ph, ca1, ca2, gc1, gc2));  // row s of this lane
      et[al][h] = kval2(B.ph, ca1, ca2, gb1, gb2);         // entry t = lane + 64 h: E_t
    }
  }
  auto zcol = [&](int al, int m, double2 (&w)[RPL]) {
    const double2* rs = Rcur + pout[al] * R2 * R2 + m;
    double2 acc[RPL];
#pragma unroll
    for (int h = 0; h < RPL; ++h) acc[h] = make_double2(0.0, 0.0);
    for (int t = 0; t < R2; ++t) {
      const double2 ev = rl_k<RPL>(et[al], t);
      const double2 rv = rs[t * R2];
#pragma unroll
      for (int h = 0; h < RPL; ++h) cfma(acc[h], cscale(ev, lcc[t * R2 + sl[h]]), rv);
    }
#pragma unroll
    for (int h = 0; h < RPL; ++h) w[h] = row[h] ? cmul(ds[al][h], acc[h]) : make_double2(0.0, 0.0);
  };
  const int nreal = kout[0] + kout[1] + kout[2] + kout[3];
  int kept = 0;
#pragma unroll
  for (int al = 0; al < 4; ++al)
    for (int m = 0; m < kout[al]; ++m) {
      if (!sample_kept(B, 64 + l, q, al * R2 + m, nreal)) continue;
      ++kept;
      double2 av[RPL];
      zcol(al, m, av);
#pragma unroll
      for (int h = 0; h < RPL; ++h) av[h] = conjd(av[h]);
      givens_fold_l<R2>(gm, lane, av);
    }
  for (int e = lane; e < R2 * k2l_stride<R2>(); e += kWaveL) gm[e] = conjd(gm[e]);
  jacobi_eig_l<R2>(gm, nl, lane);
  const int k = k2l_rank<R2>(nl, pl, lane, tol);
  k2l_scale<R2>(gm, nl, lane, B, nreal, kept);
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    if (!row[h]) continue;
    double2* rrow = Rnext + (q * R2 + sl[h]) * R2;       // R^{l-1} = U_k S_k
    for (int j = 0; j < R2; ++j) {
      const bool keep = pl[j] < k && sqrt(nl[j]) > 0.0;
      rrow[pl[j]] = keep ? k2l_at<R2>(gm, j, sl[h]) : make_double2(0.0, 0.0);
    }
  }
#pragma unroll
  for (int al = 0; al < 4; ++al) {
    double2* st = stage + (pout[al] * 4 + c) * R2 * R2;
    for (int m = 0; m < R2; ++m) {
      if (m < kout[al]) {
        double2 w[RPL];
        zcol(al, m, w);
        for (int j = 0; j < R2; ++j) {
          const double2 v = k2l_dot<R2>(gm, j, lane, w);
          if (lane == (j & (kWaveL - 1))) {
            const int pj = pl[j];
            const double sj = sqrt(nl[j]);
            const double sc = (pj < k && sj > 0.0) ? 1.0 / (sj * sj) : 0.0;
            st[m * R2 + pj] = cscale(conjd(v), sc);
          }
        }
      } else {
#pragma unroll
        for (int h = 0; h < RPL; ++h)
          if (row[h]) st[m * R2 + sl[h]] = make_double2(0.0, 0.0);
      }
    }
  }
  if (lane == 0) {
    rnext[q] = k;
    atomicMax(kmax, k);
    atomicAdd(nnz, (unsigned long long)k * (kout[0] + kout[1] + kout[2] + kout[3]));
  }
}

// stored[p][c kin + s][t < kld] from stage[p][c][t][s] (FP64, R2 x R2 per child)
template <typename FT>
__global__ void k2_pack_stage(const double2* __restrict__ stage, FT* __restrict__ out,
                              int64_t npairs, int R2, int kin, int kout, int kld) {
  const int64_t per = (int64_t)4 * kin * kld;
  const int64_t total = npairs * per;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / per;
    const int rem = (int)(e - p * per);
    const int rowi = rem / kld, t = rem - rowi * kld;
    const int c = rowi / kin, s = rowi - c * kin;
    const double2 v = t < kout ? stage[((p * 4 + c) * R2 + t) * R2 + s] : make_double2(0.0, 0.0);
    store_factor(out, e, v);
  }
}

// Vbar = R^{lV *} V^* (eqn:V0): one thread per (Omega point i, T_X box a @ lV)
//   V^*[t][xi] = conj K(c_A, g^B_t) M^B_t(xi) K(c_A, xi)
template <int R2, typename FT>
__global__ __launch_bounds__(256) void k2_vbar(BoxDev B, const double* __restrict__ z, const double* __restrict__ xis,
                        const int32_t* __restrict__ xileaf, int64_t m,
                        const double2* __restrict__ Rb, const int* __restrict__ rk, int K,
                        FT* __restrict__ vbar, unsigned long long* __restrict__ nnz) {
  const int na = 1 << (2 * B.lV);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * na) return;
  const int64_t i = e / na;
  const int a = (int)(e % na);
  const int lO = B.L - B.lV;
  const int64_t b = xileaf[i];
  const int64_t p = ((int64_t)a << (2 * lO)) + b;
  double ca1, ca2, cb1, cb2;
  cx2(B.lV, a, ca1, ca2);
  cxi2(B, lO, b, cb1, cb2);
  const double wb = B.w / ldexp(1.0, lO);
  const double x1 = xis[2 * i], x2 = xis[2 * i + 1];
  double y1, y2;
  {
#pragma clang fp contract(off)
    y1 = (x1 - cb1) / wb;
    y2 = (x2 - cb2) / wb;
  }
  const double2 kx = kval2(B.ph, ca1, ca2, x1, x2);
  const int r = B.r;
  double2 acc[R2];
#pragma unroll
  for (int k = 0; k < R2; ++k) acc[k] = make_double2(0.0, 0.0);
  for (int t = 0; t < R2; ++t) {
    const double2 kb = conjd(kval2(B.ph, ca1, ca2, gpt(cb1, wb, z[t / r]), gpt(cb2, wb, z[t % r])));
    const double2 v = cscale(cmul(kb, kx), lag2(z, r, t, y1, y2));
    const double2* rr = Rb + (p * R2 + t) * R2;
#pragma unroll
    for (int k = 0; k < R2; ++k) cfma(acc[k], conjd(rr[k]), v);
  }
  FT* o = vbar + (i * na + a) * K;
#pragma unroll
  for (int k = 0; k < R2; ++k)
    if (k < K) store_factor(o, k, acc[k]);
  atomicAdd(nnz, (unsigned long long)rk[p]);
}

// Ubar = U C^L: one thread per X point (sorted into the level-L boxes)
//   U[x][t] = K(x, c_B) M^A_t(x) conj K(g^A_t, c_B),  B = the box itself
template <int R2, typename FT>
__global__ __launch_bounds__(256) void k2_ubar(BoxDev B, const double* __restrict__ z, const double* __restrict__ xs,
                        const int32_t* __restrict__ xleaf, int64_t n,
                        const double2* __restrict__ Cb, const int* __restrict__ rk, int K,
                        FT* __restrict__ ubar, unsigned long long* __restrict__ nnz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t a = xleaf[i];
  double ca1, ca2;
  cx2(B.L, a, ca1, ca2);
  const double wa = ldexp(1.0, -B.L);
  double cb1, cb2;
  {
#pragma clang fp contract(off)
    cb1 = B.o1 + B.w / 2.0;
    cb2 = B.o2 + B.w / 2.0;
  }
  const double x1 = xs[2 * i], x2 = xs[2 * i + 1];
  double y1, y2;
  {
#pragma clang fp contract(off)
    y1 = (x1 - ca1) / wa;
    y2 = (x2 - ca2) / wa;
  }
  const double2 kx = kval2(B.ph, x1, x2, cb1, cb2);
  const int r = B.r;
  double2 acc[R2];
#pragma unroll
  for (int k = 0; k < R2; ++k) acc[k] = make_double2(0.0, 0.0);
  for (int t = 0; t < R2; ++t) {
    const double2 kg =
        conjd(kval2(B.ph, gpt(ca1, wa, z[t / r]), gpt(ca2, wa, z[t % r]), cb1, cb2));
    const double2 u = cscale(cmul(kx, kg), lag2(z, r, t, y1, y2));
    const double2* cr = Cb + (a * R2 + t) * R2;
#pragma unroll
    for (int k = 0; k < R2; ++k) cfma(acc[k], u, cr[k]);
  }
  FT* o = ubar + i * K;
#pragma unroll
  for (int k = 0; k < R2; ++k)
    if (k < K) store_factor(o, k, acc[k]);
  atomicAdd(nnz, (unsigned long long)rk[a]);
}

// Centre block K_C[x][j] = K(x, xi_j) for the centre points (stored like a factor)
template <typename FT>
__global__ void k2_centre(PhaseDesc ph, const double* __restrict__ x, int64_t nx,
                          const double* __restrict__ xic, int nc, FT* __restrict__ kc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nx * nc) return;
  const int64_t i = e / nc;
  const int j = (int)(e % nc);
  store_factor(kc, e, kval2(ph, x[2 * i], x[2 * i + 1], xic[2 * j], xic[2 * j + 1]));
}

// ---------------------------------------------------------------------------
// Apply
// ---------------------------------------------------------------------------
template <typename VT> struct Zero2;
template <> struct Zero2<double2> { __device__ static double2 v() { return make_double2(0, 0); } };
template <> struct Zero2<float2> { __device__ static float2 v() { return make_float2(0, 0); } };

// mu[(a, b)][k][n] = sum_{xi in leaf b} Vbar[xi][a][k] g[xi][n]
template <typename VT, typename FT>
__global__ void k2_apply_v(const VT* __restrict__ g, int64_t ldg, const int32_t* __restrict__ perm,
                           const int32_t* __restrict__ off, const FT* __restrict__ vbar,
                           VT* __restrict__ mu, int lV, int lO, int K, int nrhs) {
  const int na = 1 << (2 * lV);
  const int64_t nb = (int64_t)1 << (2 * lO);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)na * nb * K * nrhs;
  if (e >= total) return;
  const int n = (int)(e % nrhs);
  const int k = (int)((e / nrhs) % K);
  const int64_t pp = e / ((int64_t)nrhs * K);          // pair (a, b) at level lV
  const int64_t a = pp / nb, b = pp % nb;
  VT acc = Zero2<VT>::v();
  for (int32_t i = off[b]; i < off[b + 1]; ++i)
    cfma(acc, load_factor(vbar, ((int64_t)i * na + a) * K + k), g[(int64_t)n * ldg + perm[i]]);
  mu[e] = acc;
}

// One quadtree stage (eqn:GC / eqn:HR applied): out[(a, b)][t][n] =
// sum_{row < 4 kin} F[(a, b)][row][t] in[(a >> 2, 4b) row][n].  The four
// outputs a = 4 (a >> 2) + d, d = 0..3, with the same b read the same 4 kin
// input rows (the four children 4b + c are adjacent pairs), so a block stages
// the input rows of QB such quads in LDS once, for a chunk of NR right-hand
// sides, and thread (quad, d, t) forms output row t of pair d for all NR
// columns: per input row one factor entry (the threads t of a pair read a
// contiguous factor row) and one broadcast LDS row.
template <typename VT, typename FT, int NR>
__device__ __forceinline__ void stage_quad_body(const VT* __restrict__ in, VT* __restrict__ out,
                                                const FT* __restrict__ blk, int L, int l,
                                                int kin, int kout, int kld, int nrhs, int qb,
                                                int nchunk, int64_t lb) {
  extern __shared__ __align__(16) unsigned char smem2[];
  VT* xs = reinterpret_cast<VT*>(smem2);                      // [qb][4 kin][NR]
  const int sh = 2 * (L - l);
  const int64_t nquad = (int64_t)1 << (2 * L - 2);
  const int64_t q0 = (lb / nchunk) * qb;
  const int n0 = (int)(lb % nchunk) * NR;
  const int nw = min(NR, nrhs - n0);
  const int rows = 4 * kin;
  // stage the quads' input rows (columns past the chunk are zero)
  for (int e = threadIdx.x; e < qb * rows * NR; e += kB2) {
    const int n = e % NR, r = (e / NR) % rows, qi = e / (NR * rows);
    const int64_t q = q0 + qi;
    VT v = Zero2<VT>::v();
    if (q < nquad && n < nw) {
      const int64_t pin0 = ((q >> sh) << (sh + 2)) + 4 * (q & (((int64_t)1 << sh) - 1));
      v = in[(pin0 * kin + r) * nrhs + n0 + n];
    }
    xs[e] = v;
  }
  __syncthreads();
  const int per = 4 * kout;                                   // threads a quad
  const int qi = threadIdx.x / per, rr = threadIdx.x - qi * per;
  const int64_t q = q0 + qi;
  if (qi >= qb || q >= nquad) return;
  const int d = rr / kout, t = rr - d * kout;
  const int64_t a = ((q >> sh) << 2) + d, b = q & (((int64_t)1 << sh) - 1);
  const int64_t pout = (a << sh) | b;
  const FT* f = blk + pout * rows * kld + t;
  const VT* x = xs + (size_t)qi * rows * NR;
  VT acc[NR];
#pragma unroll
  for (int n = 0; n < NR; ++n) acc[n] = Zero2<VT>::v();
  constexpr int U = 16;                                       // factor loads in flight
  int r = 0;
  for (; r + U <= rows; r += U) {
    VT fv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) fv[u] = load_factor(f, (int64_t)(r + u) * kld);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int n = 0; n < NR; ++n) cfma(acc[n], fv[u], x[(r + u) * NR + n]);
  }
  for (; r < rows; ++r) {
    const VT fv = load_factor(f, (int64_t)r * kld);
#pragma unroll
    for (int n = 0; n < NR; ++n) cfma(acc[n], fv, x[r * NR + n]);
  }
  VT* o = out + (pout * kout + t) * nrhs + n0;
#pragma unroll
  for (int n = 0; n < NR; ++n)
    if (n < nw) o[n] = acc[n];
}
template <typename VT, typename FT, int NR>
__global__ __launch_bounds__(kB2) void k2_apply_stage_quad(const VT* __restrict__ in,
                                                          VT* __restrict__ out,
                                                          const FT* __restrict__ blk, int L,
                                                          int l, int kin, int kout, int kld,
                                                          int nrhs, int qb, int nchunk) {
  stage_quad_body<VT, FT, NR>(in, out, blk, L, l, kin, kout, kld, nrhs, qb, nchunk,
                              blockIdx.x);
}

// Batched launches over the boxes: box p owns logical blocks [boff[p], boff[p+1]).
__device__ __forceinline__ int box_of_block(const int64_t* __restrict__ boff, int count,
                                            int64_t b) {
  int lo = 0, hi = count - 1;                                 // largest p with boff[p] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (boff[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// one box's quadtree stage in a batched launch (the boxes' stages of one
// index together: a box's stages run in launch order)
struct Stage2Desc {
  const void* in;
  void* out;
  const void* blk;
  int L, l, kin, kout, kld, qb;
};
template <typename VT, typename FT, int NR>
__global__ __launch_bounds__(kB2) void k2_batch_stage_quad(const Stage2Desc* __restrict__ ds,
                                                          const int64_t* __restrict__ boff,
                                                          int count, int nrhs, int nchunk) {
  const int p = box_of_block(boff, count, blockIdx.x);
  const Stage2Desc& D = ds[p];
  stage_quad_body<VT, FT, NR>(reinterpret_cast<const VT*>(D.in), reinterpret_cast<VT*>(D.out),
                              reinterpret_cast<const FT*>(D.blk), D.L, D.l, D.kin, D.kout, D.kld,
                              nrhs, D.qb, nchunk, (int64_t)blockIdx.x - boff[p]);
}

// out[(a, b)][t][n] = sum_{row < 4 kin} F[(a, b)][row][t] in[(a >> 2, 4b) row][n]
template <typename VT, typename FT>
__global__ void k2_apply_stage(const VT* __restrict__ in, VT* __restrict__ out,
                               const FT* __restrict__ blk, int L, int l, int kin, int kout,
                               int kld, int nrhs) {
  const int64_t npairs = (int64_t)1 << (2 * L);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= npairs * kout * nrhs) return;
  const int n = (int)(e % nrhs);
  const int t = (int)((e / nrhs) % kout);
  const int64_t p = e / ((int64_t)nrhs * kout);
  const int sh = 2 * (L - l);
  const int64_t a = p >> sh, b = p & (((int64_t)1 << sh) - 1);
  const int64_t pin0 = ((a >> 2) << (sh + 2)) + 4 * b;
  const FT* f = blk + p * 4 * kin * kld + t;
  const VT* x = in + pin0 * kin * nrhs + n;
  VT acc = Zero2<VT>::v();
  for (int row = 0; row < 4 * kin; ++row)
    cfma(acc, load_factor(f, (int64_t)row * kld), x[(int64_t)row * nrhs]);
  out[e] = acc;
}

// u[x][n] = sum_j K_C[x][j] g[centre_j][n]   (writes u; runs first)
template <typename VT, typename FT>
__global__ void k2_apply_centre(const FT* __restrict__ kc, int nc,
                                const int32_t* __restrict__ cidx, const VT* __restrict__ g,
                                int64_t ldg, int64_t nx, VT* __restrict__ u, int64_t ldu,
                                int nrhs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nx * nrhs) return;
  const int64_t i = e % nx;
  const int c = (int)(e / nx);
  VT acc = Zero2<VT>::v();
  for (int j = 0; j < nc; ++j)
    cfma(acc, load_factor(kc, i * nc + j), g[(int64_t)c * ldg + cidx[j]]);
  u[(int64_t)c * ldu + i] = acc;
}

// Row-per-thread forms of the leaf and centre products: thread = one output
// row for a chunk of NR right-hand sides (a factor entry is read once per
// chunk, the shared operand rows come from LDS).

// V for one Omega leaf b and RHS chunk: thread (a, k) forms mu[(a, b)][k][0..NR)
// over the leaf's points; the leaf's g rows are staged in LDS, and the threads
// of a point read its Vbar row [a][k] contiguously.
template <typename VT, typename FT, int NR>
__device__ __forceinline__ void v_rows_body(const VT* __restrict__ g, int64_t ldg,
                                            const int32_t* __restrict__ perm,
                                            const int32_t* __restrict__ off,
                                            const FT* __restrict__ vbar, VT* __restrict__ mu,
                                            int lV, int lO, int K, int nrhs, int nchunk,
                                            int64_t lb) {
  extern __shared__ __align__(16) unsigned char smem2[];
  VT* gl = reinterpret_cast<VT*>(smem2);                      // [smax][NR]
  const int na = 1 << (2 * lV);
  const int64_t nb = (int64_t)1 << (2 * lO);
  const int64_t b = lb / nchunk;
  const int n0 = (int)(lb % nchunk) * NR, nw = min(NR, nrhs - n0);
  const int32_t i0 = off[b], cnt = off[b + 1] - i0;
  for (int e = threadIdx.x; e < cnt * NR; e += kB2) {
    const int j = e / NR, n = e % NR;
    gl[e] = n < nw ? g[(int64_t)(n0 + n) * ldg + perm[i0 + j]] : Zero2<VT>::v();
  }
  __syncthreads();
  for (int item = threadIdx.x; item < na * K; item += kB2) {  // item = a K + k
    VT acc[NR];
#pragma unroll
    for (int n = 0; n < NR; ++n) acc[n] = Zero2<VT>::v();
    for (int j = 0; j < cnt; ++j) {
      const VT f = load_factor(vbar, (int64_t)(i0 + j) * na * K + item);
#pragma unroll
      for (int n = 0; n < NR; ++n) cfma(acc[n], f, gl[j * NR + n]);
    }
    const int a = item / K, k = item - a * K;
    VT* o = mu + (((int64_t)a * nb + b) * K + k) * nrhs + n0;
#pragma unroll
    for (int n = 0; n < NR; ++n)
      if (n < nw) o[n] = acc[n];
  }
}
template <typename VT, typename FT, int NR>
__global__ __launch_bounds__(kB2) void k2_apply_v_rows(const VT* __restrict__ g, int64_t ldg,
                                                      const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ off,
                                                      const FT* __restrict__ vbar,
                                                      VT* __restrict__ mu, int lV, int lO, int K,
                                                      int nrhs, int smax, int nchunk) {
  (void)smax;
  v_rows_body<VT, FT, NR>(g, ldg, perm, off, vbar, mu, lV, lO, K, nrhs, nchunk, blockIdx.x);
}
// V of every box in one launch
struct V2Desc {
  const int32_t* perm;
  const int32_t* off;
  const void* vbar;
  void* mu;
  int lV, lO, K;
};
template <typename VT, typename FT, int NR>
__global__ __launch_bounds__(kB2) void k2_batch_v_rows(const V2Desc* __restrict__ ds,
                                                      const int64_t* __restrict__ boff, int count,
                                                      const VT* __restrict__ g, int64_t ldg,
                                                      int nrhs, int nchunk) {
  const int p = box_of_block(boff, count, blockIdx.x);
  const V2Desc& D = ds[p];
  v_rows_body<VT, FT, NR>(g, ldg, D.perm, D.off, reinterpret_cast<const FT*>(D.vbar),
                          reinterpret_cast<VT*>(D.mu), D.lV, D.lO, D.K, nrhs, nchunk,
                          (int64_t)blockIdx.x - boff[p]);
}

// U of the boxes that share one X tree, in one launch: thread = one X point
// (the tree's sorted order), all NR columns of the chunk:
//   u[perm(i)][n] += sum_boxes sum_k Ubar_box[i][k] mu_box[leaf(i)][k][n]
// (the boxes in the order given, then one read-modify-write of u).
constexpr int kTreeBoxes = 16;
struct UTree {
  const void* mu[kTreeBoxes];
  const void* ubar[kTreeBoxes];
  int K[kTreeBoxes];
  int nb;
};
template <typename VT, typename FT, int NR>
__global__ __launch_bounds__(kB2) void k2_apply_u_tree(UTree T, const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ leaf, int64_t n,
                                                      VT* __restrict__ u, int64_t ldu, int nrhs,
                                                      int nchunk) {
  const int64_t i = (int64_t)(blockIdx.x / nchunk) * kB2 + threadIdx.x;
  const int n0 = (int)(blockIdx.x % nchunk) * NR, nw = min(NR, nrhs - n0);
  if (i >= n) return;
  const int64_t li = leaf[i];
  VT acc[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) acc[c] = Zero2<VT>::v();
  for (int bx = 0; bx < T.nb; ++bx) {
    const int K = T.K[bx];
    const VT* m = reinterpret_cast<const VT*>(T.mu[bx]) + li * K * nrhs + n0;
    const FT* ub = reinterpret_cast<const FT*>(T.ubar[bx]);
    // rows in batches of UB with all their loads issued before the products
    constexpr int UB = 4;
    int k = 0;
    for (; k + UB <= K; k += UB) {
      VT f[UB], mv[UB][NR];
#pragma unroll
      for (int b = 0; b < UB; ++b) {
        f[b] = load_factor(ub, i * K + k + b);
#pragma unroll
        for (int c = 0; c < NR; ++c) mv[b][c] = m[(int64_t)(k + b) * nrhs + min(c, nw - 1)];
      }
#pragma unroll
      for (int b = 0; b < UB; ++b)
#pragma unroll
        for (int c = 0; c < NR; ++c) cfma(acc[c], f[b], mv[b][c]);
    }
    for (; k < K; ++k) {
      const VT f = load_factor(ub, i * K + k);
#pragma unroll
      for (int c = 0; c < NR; ++c) cfma(acc[c], f, m[(int64_t)k * nrhs + min(c, nw - 1)]);
    }
  }
  const int64_t pi = perm[i];
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    if (c < nw) {
      VT* o = u + (int64_t)(n0 + c) * ldu + pi;
      VT cur = *o;
      cur.x += acc[c].x;
      cur.y += acc[c].y;
      *o = cur;
    }
  }
}

// Centre: u[x][n] = sum_j K_C[x][j] g[centre_j][n] for 256 consecutive x a
// block and NR columns.  The centre's g rows [nc][NR] sit in LDS; K_C is read
// in tiles of JT columns staged through LDS (coalesced row segments), then
// each thread runs its own row of the tile.
template <typename VT, typename FT, int NR>
__global__ __launch_bounds__(kB2) void k2_apply_centre_rows(const FT* __restrict__ kc, int nc,
                                                           const int32_t* __restrict__ cidx,
                                                           const VT* __restrict__ g, int64_t ldg,
                                                           int64_t nx, VT* __restrict__ u,
                                                           int64_t ldu, int nrhs, int nchunk) {
  constexpr int JT = 16;
  extern __shared__ __align__(16) unsigned char smem2[];
  VT* gc = reinterpret_cast<VT*>(smem2);                      // [nc][NR]
  VT* kt = gc + (size_t)nc * NR;                              // [kB2][JT + 1]
  const int64_t x0 = (int64_t)(blockIdx.x / nchunk) * kB2;
  const int n0 = (int)(blockIdx.x % nchunk) * NR, nw = min(NR, nrhs - n0);
  for (int e = threadIdx.x; e < nc * NR; e += kB2) {
    const int j = e / NR, n = e % NR;
    gc[e] = n < nw ? g[(int64_t)(n0 + n) * ldg + cidx[j]] : Zero2<VT>::v();
  }
  VT acc[NR];
#pragma unroll
  for (int n = 0; n < NR; ++n) acc[n] = Zero2<VT>::v();
  const int64_t xi = x0 + threadIdx.x;
  for (int j0 = 0; j0 < nc; j0 += JT) {
    __syncthreads();                                          // previous tile consumed
    for (int e = threadIdx.x; e < kB2 * JT; e += kB2) {
      const int r = e / JT, c = e % JT;
      const int64_t x = x0 + r;
      kt[r * (JT + 1) + c] = (x < nx && j0 + c < nc) ? load_factor(kc, x * nc + j0 + c)
                                                     : Zero2<VT>::v();
    }
    __syncthreads();
    const int jn = min(JT, nc - j0);
    for (int c = 0; c < jn; ++c) {
      const VT f = kt[threadIdx.x * (JT + 1) + c];
#pragma unroll
      for (int n = 0; n < NR; ++n) cfma(acc[n], f, gc[(j0 + c) * NR + n]);
    }
  }
  if (xi < nx) {
#pragma unroll
    for (int n = 0; n < NR; ++n)
      if (n < nw) u[(int64_t)(n0 + n) * ldu + xi] = acc[n];
  }
}

inline unsigned nblk(int64_t total) { return (unsigned)((total + kB2 - 1) / kB2); }

}  // namespace
}  // namespace ibf

// ===========================================================================
// Host side
// ===========================================================================
namespace ibf {
namespace {

#define IBF2_DISPATCH_R2(R2V, LAUNCH)                      \
  switch (R2V) {                                           \
    case 4: LAUNCH(4); break;                              \
    case 9: LAUNCH(9); break;                              \
    case 16: LAUNCH(16); break;                            \
    case 25: LAUNCH(25); break;                            \
    case 36: LAUNCH(36); break;                            \
    case 49: LAUNCH(49); break;                            \
    case 64: LAUNCH(64); break;                            \
    default: LAUNCH(81); break;                            \
  }
// register-resident compression kernels (r <= 5) / LDS-resident ones (r = 6 .. 8)
#define IBF2_DISPATCH_SMALL(R2V, LAUNCH)                   \
  switch (R2V) {                                           \
    case 4: LAUNCH(4); break;                              \
    case 9: LAUNCH(9); break;                              \
    case 16: LAUNCH(16); break;                            \
    default: LAUNCH(25); break;                            \
  }
#define IBF2_DISPATCH_BIG(R2V, LAUNCH)                     \
  switch (R2V) {                                           \
    case 36: LAUNCH(36); break;                            \
    case 49: LAUNCH(49); break;                            \
    case 64: LAUNCH(64); break;                            \
    default: LAUNCH(81); break;                            \
  }
// LDS bytes of one pair (wave) of the LDS-resident kernels, and pairs a
// block: as many as 160 KiB hold, at most 4
inline size_t k2l_lds_per_wave(int R2) {
  const size_t stride = R2 > kWaveL ? (size_t)R2 : (size_t)kWaveL;
  return ((size_t)R2 * stride * sizeof(double2) + (size_t)R2 * (sizeof(double) + sizeof(int)) +
          15) & ~(size_t)15;
}
inline int k2l_waves(int R2) {
  return (int)std::max<size_t>(1, std::min<size_t>(4, (160u << 10) / k2l_lds_per_wave(R2)));
}

int64_t morton_host(int64_t i1, int64_t i2, int level) {
  int64_t code = 0;
  for (int j = 0; j < level; ++j) code |= (((i1 >> j) & 1) * 2 + ((i2 >> j) & 1)) << (2 * j);
  return code;
}

// counting sort of codes in [0, nbin): perm (sorted -> input position), CSR offsets, bin per sorted
void sort_codes(const std::vector<int64_t>& code, int64_t nbin, std::vector<int32_t>& perm,
                std::vector<int32_t>& off, std::vector<int32_t>& bin) {
  off.assign(nbin + 1, 0);
  for (int64_t c : code) ++off[c + 1];
  for (int64_t b = 0; b < nbin; ++b) off[b + 1] += off[b];
  std::vector<int32_t> fill(off.begin(), off.end() - 1);
  perm.assign(code.size(), 0);
  bin.assign(code.size(), 0);
  for (size_t i = 0; i < code.size(); ++i) {
    const int32_t at = fill[code[i]]++;
    perm[at] = (int32_t)i;
    bin[at] = (int32_t)code[i];
  }
}

template <typename T>
int upload(T** d, const T* h, size_t n) {
  IBF_HIP_CHECK(ibf::dev_malloc(d, std::max<size_t>(n * sizeof(T), 1)));
  if (n) IBF_HIP_CHECK(hipMemcpy(*d, h, n * sizeof(T), hipMemcpyHostToDevice));
  return IBF_OK;
}

struct Scratch2 {
  double2* C[2] = {nullptr, nullptr};
  double2* R[2] = {nullptr, nullptr};
  int* rc[2] = {nullptr, nullptr};
  int* rr[2] = {nullptr, nullptr};
  double2* stage = nullptr;
  int* kmax = nullptr;                    // [2][64]: G side at [l], H side at [64 + l]
  unsigned long long* nnz = nullptr;
  ~Scratch2() {
    for (int i = 0; i < 2; ++i) {
      if (C[i]) (void)ibf::dev_free(C[i]);
      if (R[i]) (void)ibf::dev_free(R[i]);
      if (rc[i]) (void)ibf::dev_free(rc[i]);
      if (rr[i]) (void)ibf::dev_free(rr[i]);
    }
    if (stage) (void)ibf::dev_free(stage);
    if (kmax) (void)ibf::dev_free(kmax);
    if (nnz) (void)ibf::dev_free(nnz);
  }
};

int read_int(const int* d, int* h, hipStream_t s) {
  IBF_HIP_CHECK(hipMemcpyAsync(h, d, sizeof(int), hipMemcpyDeviceToHost, s));
  IBF_HIP_CHECK(hipStreamSynchronize(s));
  return IBF_OK;
}

template <typename FT>
int pack_stage(Box2& bx, Mibf2D& M, const double2* stage, int level, int kin, int kout,
               hipStream_t s) {
  Stage2 st;
  st.level = level;
  st.kin = kin;
  st.kout = kout;
  st.kld = (kout + 1) & ~1;
  const int64_t np = (int64_t)1 << (2 * bx.L);
  const int64_t count = np * 4 * kin * st.kld;
  st.bytes = (size_t)count * sizeof(FT);
  IBF_HIP_CHECK(ibf::dev_malloc(&st.blk, std::max<size_t>(st.bytes, 1)));
  const unsigned g = (unsigned)std::min<int64_t>((count + kB2 - 1) / kB2, 1 << 20);
  hipLaunchKernelGGL((k2_pack_stage<FT>), dim3(std::max(g, 1u)), dim3(kB2), 0, s, stage,
                     (FT*)st.blk, np, M.R2, kin, kout, st.kld);
  IBF_HIP_CHECK(hipGetLastError());
  bx.stages.push_back(st);
  M.nnz_stored += count;
  return IBF_OK;
}

template <typename FT>
int build2d_t(ibf_plan_t p, hipStream_t s) {
  Mibf2D& M = *p->mibf;
  const int R2 = M.R2, r = M.r;
  // tables and X points
  IBF_HIP_CHECK(ibf::dev_malloc(&M.d_z, sizeof(double) * r));
  IBF_HIP_CHECK(ibf::dev_malloc(&M.d_lc, sizeof(double) * 4 * R2 * R2));
  hipLaunchKernelGGL(k2_tables, dim3((4 * R2 * R2 + kB2 - 1) / kB2), dim3(kB2), 0, s, r, M.d_z,
                     M.d_lc);
  IBF_HIP_CHECK(hipGetLastError());
  // centre block
  const int nc = (int)M.centre.size();
  if (nc > 0) {
    std::vector<double> xic(2 * (size_t)nc);
    for (int j = 0; j < nc; ++j) {
      xic[2 * j] = M.xi_host[2 * (size_t)M.centre[j]];
      xic[2 * j + 1] = M.xi_host[2 * (size_t)M.centre[j] + 1];
    }
    double* d_xic = nullptr;
    int rc;
    if ((rc = upload(&d_xic, xic.data(), xic.size()))) return rc;
    if ((rc = upload(&M.d_cidx, M.centre.data(), M.centre.size()))) return rc;
    IBF_HIP_CHECK(ibf::dev_malloc(&M.d_kc, std::max<size_t>(sizeof(FT) * M.nx * nc, 1)));
    hipLaunchKernelGGL((k2_centre<FT>), dim3(nblk(M.nx * nc)), dim3(kB2), 0, s, M.ph, M.d_x,
                       M.nx, d_xic, nc, (FT*)M.d_kc);
    IBF_HIP_CHECK(hipGetLastError());
    IBF_HIP_CHECK(hipStreamSynchronize(s));
    (void)ibf::dev_free(d_xic);
    M.factor_bytes += (int64_t)(sizeof(FT) * M.nx * nc);
    M.nnz_opt += M.nx * nc;
    M.nnz_stored += M.nx * nc;
  }
  // scratch for the largest box
  const int64_t npmax = (int64_t)1 << (2 * M.maxL);
  Scratch2 S;
  const size_t bsz = sizeof(double2) * (size_t)npmax * R2 * R2;
  for (int i = 0; i < 2; ++i) {
    IBF_HIP_CHECK(ibf::dev_malloc(&S.C[i], bsz));
    IBF_HIP_CHECK(ibf::dev_malloc(&S.R[i], bsz));
    IBF_HIP_CHECK(ibf::dev_malloc(&S.rc[i], sizeof(int) * npmax));
    IBF_HIP_CHECK(ibf::dev_malloc(&S.rr[i], sizeof(int) * npmax));
  }
  IBF_HIP_CHECK(ibf::dev_malloc(&S.stage, 4 * bsz));
  IBF_HIP_CHECK(ibf::dev_malloc(&S.kmax, sizeof(int) * 128));
  IBF_HIP_CHECK(ibf::dev_malloc(&S.nnz, sizeof(unsigned long long)));

  int rc;
  for (Box2& bx : M.boxes) {
    const BoxDev B{M.ph, bx.o1, bx.o2, bx.w, bx.L, bx.lV, bx.h, r, M.ssamp, M.sseed};
    const int L = bx.L, lV = bx.lV, h = bx.h;
    const int64_t np = (int64_t)1 << (2 * L);
    const int G = R2 <= 32 ? 32 : 64;                        // lanes per pair (group2<R2>)
    const unsigned gg = (unsigned)((np * G + kB2 - 1) / kB2);
    std::vector<int> kg(L + 1, 0), kh(L + 1, 0);
    IBF_HIP_CHECK(hipMemsetAsync(S.kmax, 0, sizeof(int) * 128, s));
    IBF_HIP_CHECK(hipMemsetAsync(S.nnz, 0, sizeof(unsigned long long), s));
    const bool big = R2 > 25;
    const int nwl = k2l_waves(R2);
    const unsigned ggl = (unsigned)((np + nwl - 1) / nwl);
    const size_t ldsl = (size_t)nwl * k2l_lds_per_wave(R2);
#define IBF2_MIDDLE(RR)                                                                          \
  hipLaunchKernelGGL((k2_middle<RR>), dim3(gg), dim3(kB2), 0, s, B, M.d_z, S.C[0], S.R[0],      \
                     S.rc[0], S.kmax + h, S.nnz, np, M.tol)
#define IBF2L_MIDDLE(RR)                                                                         \
  hipLaunchKernelGGL((k2l_middle<RR>), dim3(ggl), dim3(kWaveL * nwl), ldsl, s, B, M.d_z, S.C[0], \
                     S.R[0], S.rc[0], S.kmax + h, S.nnz, np, M.tol)
    if (big) {
      IBF2_DISPATCH_BIG(R2, IBF2L_MIDDLE);
    } else {
      IBF2_DISPATCH_SMALL(R2, IBF2_MIDDLE);
    }
#undef IBF2_MIDDLE
#undef IBF2L_MIDDLE
    IBF_HIP_CHECK(hipGetLastError());
    IBF_HIP_CHECK(hipMemcpyAsync(S.rr[0], S.rc[0], sizeof(int) * np, hipMemcpyDeviceToDevice, s));
    if ((rc = read_int(S.kmax + h, &kg[h], s))) return rc;
    kh[h] = kg[h];
    // toward U
    int cc = 0;
    std::vector<Stage2> gst;
    for (int l = h + 1; l <= L; ++l) {
#define IBF2_SWG(RR)                                                                             \
  hipLaunchKernelGGL((k2_sweep_g<RR>), dim3(gg), dim3(kB2), 0, s, B, l, M.d_z, M.d_lc, S.C[cc], \
                     S.rc[cc], S.C[cc ^ 1], S.rc[cc ^ 1], S.kmax + l, S.stage, S.nnz, np, M.tol)
#define IBF2L_SWG(RR)                                                                            \
  hipLaunchKernelGGL((k2l_sweep_g<RR>), dim3(ggl), dim3(kWaveL * nwl), ldsl, s, B, l, M.d_z,     \
                     M.d_lc, S.C[cc], S.rc[cc], S.C[cc ^ 1], S.rc[cc ^ 1], S.kmax + l, S.stage,  \
                     S.nnz, np, M.tol)
      if (big) {
        IBF2_DISPATCH_BIG(R2, IBF2L_SWG);
      } else {
        IBF2_DISPATCH_SMALL(R2, IBF2_SWG);
      }
#undef IBF2_SWG
#undef IBF2L_SWG
      IBF_HIP_CHECK(hipGetLastError());
      if ((rc = read_int(S.kmax + l, &kg[l], s))) return rc;
      if ((rc = pack_stage<FT>(bx, M, S.stage, l, kg[l - 1], kg[l], s))) return rc;
      gst.push_back(bx.stages.back());
      bx.stages.pop_back();
      cc ^= 1;
    }
    // toward V
    int cr = 0;
    std::vector<Stage2> hst;
    for (int l = h; l > lV; --l) {
#define IBF2_SWH(RR)                                                                             \
  hipLaunchKernelGGL((k2_sweep_h<RR>), dim3(gg), dim3(kB2), 0, s, B, l, M.d_z, M.d_lc, S.R[cr], \
                     S.rr[cr], S.R[cr ^ 1], S.rr[cr ^ 1], S.kmax + 64 + l - 1, S.stage, S.nnz, \
                     np, M.tol)
#define IBF2L_SWH(RR)                                                                            \
  hipLaunchKernelGGL((k2l_sweep_h<RR>), dim3(ggl), dim3(kWaveL * nwl), ldsl, s, B, l, M.d_z,     \
                     M.d_lc, S.R[cr], S.rr[cr], S.R[cr ^ 1], S.rr[cr ^ 1], S.kmax + 64 + l - 1,  \
                     S.stage, S.nnz, np, M.tol)
      if (big) {
        IBF2_DISPATCH_BIG(R2, IBF2L_SWH);
      } else {
        IBF2_DISPATCH_SMALL(R2, IBF2_SWH);
      }
#undef IBF2_SWH
#undef IBF2L_SWH
      IBF_HIP_CHECK(hipGetLastError());
      if ((rc = read_int(S.kmax + 64 + l - 1, &kh[l - 1], s))) return rc;
      if ((rc = pack_stage<FT>(bx, M, S.stage, l, kh[l - 1], kh[l], s))) return rc;
      hst.push_back(bx.stages.back());
      bx.stages.pop_back();
      cr ^= 1;
    }
    // apply order: H stages lV+1..h, then G stages h+1..L
    bx.stages.clear();
    for (auto it = hst.rbegin(); it != hst.rend(); ++it) bx.stages.push_back(*it);
    for (auto& st : gst) bx.stages.push_back(st);
    bx.rank.assign(L - lV + 1, 0);
    for (int l = lV; l <= L; ++l) bx.rank[l - lV] = l <= h ? kh[l] : kg[l];
    // outer factors
    const XTree2& xt = M.xtrees[bx.xt];
    bx.K_V = std::max(kh[lV], 1);
    bx.K_U = std::max(kg[L], 1);
    const int na = 1 << (2 * lV);
    bx.vbar_bytes = sizeof(FT) * (size_t)bx.m * na * bx.K_V;
    bx.ubar_bytes = sizeof(FT) * (size_t)M.nx * bx.K_U;
    IBF_HIP_CHECK(ibf::dev_malloc(&bx.d_vbar, std::max<size_t>(bx.vbar_bytes, 1)));
    IBF_HIP_CHECK(ibf::dev_malloc(&bx.d_ubar, std::max<size_t>(bx.ubar_bytes, 1)));
    if (bx.m > 0) {
#define IBF2_VBAR(RR)                                                                            \
  hipLaunchKernelGGL((k2_vbar<RR, FT>), dim3(nblk(bx.m * na)), dim3(kB2), 0, s, B, M.d_z,       \
                     bx.d_xis, bx.d_xileaf, bx.m, S.R[cr], S.rr[cr], bx.K_V, (FT*)bx.d_vbar,    \
                     S.nnz)
      IBF2_DISPATCH_R2(R2, IBF2_VBAR);
#undef IBF2_VBAR
      IBF_HIP_CHECK(hipGetLastError());
    }
#define IBF2_UBAR(RR)                                                                            \
  hipLaunchKernelGGL((k2_ubar<RR, FT>), dim3(nblk(M.nx)), dim3(kB2), 0, s, B, M.d_z, xt.d_xs,   \
                     xt.d_leaf, M.nx, S.C[cc], S.rc[cc], bx.K_U, (FT*)bx.d_ubar, S.nnz)
    IBF2_DISPATCH_R2(R2, IBF2_UBAR);
#undef IBF2_UBAR
    IBF_HIP_CHECK(hipGetLastError());
    unsigned long long nn = 0;
    IBF_HIP_CHECK(hipMemcpyAsync(&nn, S.nnz, sizeof(nn), hipMemcpyDeviceToHost, s));
    IBF_HIP_CHECK(hipStreamSynchronize(s));
    bx.nnz_opt = (int64_t)nn;
    M.nnz_opt += bx.nnz_opt;
    M.nnz_stored += (int64_t)bx.m * na * bx.K_V + M.nx * bx.K_U;
    M.factor_bytes += (int64_t)(bx.vbar_bytes + bx.ubar_bytes);
    for (auto& st : bx.stages) M.factor_bytes += (int64_t)st.bytes;
  }
  M.built = true;
  return IBF_OK;
}

template <typename VT, typename FT>
int launch2d_t(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int nrhs,
               hipStream_t s, const std::vector<size_t>& off);

constexpr int kNR2 = 8;                                       // RHS columns a pass

// quads a block of the quad-grouped stage kernel: threads (4 kout each) and
// staged rows (<= 48 KB)
template <typename VT>
int stage_qb(const Stage2& st) {
  return std::max(1, std::min(kB2 / (4 * st.kout),
                              (int)((48 * 1024) / ((size_t)4 * st.kin * kNR2 * sizeof(VT)))));
}

// The batched launch plan and its descriptor table for nrhs right-hand sides
// and the current workspace (box ib's coefficient buffers at off[ib]).
// Written only when (nrhs, workspace) changes, after the stream has drained.
template <typename VT, typename FT>
int prepare_batched2d(ibf_plan_t p, int nrhs, const std::vector<size_t>& off, hipStream_t s) {
  Mibf2D& M = *p->mibf;
  const std::vector<int64_t> key = {nrhs, (int64_t)(uintptr_t)M.d_work};
  if (key == M.table_key) return IBF_OK;
  const int nbox = (int)M.boxes.size();
  const int nchunk = (nrhs + kNR2 - 1) / kNR2;
  bool ok = nbox > 0;
  size_t maxs = 0;
  for (const Box2& bx : M.boxes) maxs = std::max(maxs, bx.stages.size());
  std::vector<Launch2> launches(1 + maxs);
  std::vector<unsigned char> host;
  auto align16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
  auto buf = [&](int ib, int which) {
    char* wb = static_cast<char*>(M.d_work) + off[ib];
    return static_cast<void*>(wb + which * ((off[ib + 1] - off[ib]) / 2));
  };
  // V of every box
  {
    std::vector<V2Desc> d;
    std::vector<int64_t> bo{0};
    Launch2& x = launches[0];
    for (int ib = 0; ib < nbox; ++ib) {
      const Box2& bx = M.boxes[ib];
      const int lO = bx.L - bx.lV;
      d.push_back(V2Desc{bx.d_perm_xi, bx.d_xioff, bx.d_vbar, buf(ib, 0), bx.lV, lO, bx.K_V});
      bo.push_back(bo.back() + ((int64_t)1 << (2 * lO)) * nchunk);
      x.lds = std::max(x.lds, (size_t)bx.smax_xi * kNR2 * sizeof(VT));
    }
    x.count = nbox;
    x.nblocks = bo.back();
    x.desc_off = host.size();
    host.resize(align16(host.size() + d.size() * sizeof(V2Desc)));
    std::memcpy(host.data() + x.desc_off, d.data(), d.size() * sizeof(V2Desc));
    x.boff_off = host.size();
    host.resize(align16(host.size() + bo.size() * sizeof(int64_t)));
    std::memcpy(host.data() + x.boff_off, bo.data(), bo.size() * sizeof(int64_t));
    ok = ok && x.lds <= 64 * 1024;
  }
  // stage j of every box that has one: box ib reads buffer j % 2, writes the other
  for (size_t j = 0; j < maxs; ++j) {
    std::vector<Stage2Desc> d;
    std::vector<int64_t> bo{0};
    Launch2& x = launches[1 + j];
    for (int ib = 0; ib < nbox; ++ib) {
      const Box2& bx = M.boxes[ib];
      if (j >= bx.stages.size()) continue;
      const Stage2& st = bx.stages[j];
      const int qb = stage_qb<VT>(st);
      const size_t lds = (size_t)qb * 4 * st.kin * kNR2 * sizeof(VT);
      const int64_t nquad = (int64_t)1 << (2 * bx.L - 2);
      ok = ok && 4 * st.kout <= kB2 && lds <= 64 * 1024;
      d.push_back(Stage2Desc{buf(ib, (int)(j & 1)), buf(ib, (int)((j + 1) & 1)), st.blk, bx.L,
                             st.level, st.kin, st.kout, st.kld, qb});
      bo.push_back(bo.back() + (nquad + qb - 1) / qb * nchunk);
      x.lds = std::max(x.lds, lds);
    }
    x.count = (int)d.size();
    x.nblocks = bo.back();
    x.desc_off = host.size();
    host.resize(align16(host.size() + d.size() * sizeof(Stage2Desc)));
    std::memcpy(host.data() + x.desc_off, d.data(), d.size() * sizeof(Stage2Desc));
    x.boff_off = host.size();
    host.resize(align16(host.size() + bo.size() * sizeof(int64_t)));
    std::memcpy(host.data() + x.boff_off, bo.data(), bo.size() * sizeof(int64_t));
  }
  for (const Launch2& x : launches) ok = ok && x.nblocks < 0x7fffffff;
  M.batched = false;
  if (ok) {
    IBF_HIP_CHECK(hipStreamSynchronize(s));                   // no apply still reads the table
    if (host.size() > M.table_bytes) {
      if (M.d_table) IBF_HIP_CHECK(ibf::dev_free(M.d_table));
      M.d_table = nullptr;
      M.table_bytes = 0;
      IBF_HIP_CHECK(ibf::dev_malloc(&M.d_table, host.size()));
      M.table_bytes = host.size();
    }
    IBF_HIP_CHECK(hipMemcpy(M.d_table, host.data(), host.size(), hipMemcpyHostToDevice));
    M.launches = launches;
    M.batched = true;
  }
  M.table_key = key;
  return IBF_OK;
}

template <typename VT, typename FT>
int apply2d_t(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int nrhs,
              hipStream_t s) {
  Mibf2D& M = *p->mibf;
  const int nbox = (int)M.boxes.size();
  // one pair of coefficient buffers per box (boxes run concurrently)
  std::vector<size_t> off(nbox + 1, 0);
  for (int i = 0; i < nbox; ++i) {
    const Box2& bx = M.boxes[i];
    int kmx = 1;
    for (int k : bx.rank) kmx = std::max(kmx, k);
    const size_t one = ((((size_t)1 << (2 * bx.L)) * kmx * nrhs * sizeof(VT)) + 255) & ~(size_t)255;
    off[i + 1] = off[i] + 2 * one;
  }
  if (off[nbox] > M.work_bytes) {
    if (M.d_work) IBF_HIP_CHECK(ibf::dev_free(M.d_work));
    M.d_work = nullptr;
    M.work_bytes = 0;
    IBF_HIP_CHECK(ibf::dev_malloc(&M.d_work, off[nbox]));
    M.work_bytes = off[nbox];
  }
  if (M.streams.empty() && nbox > 0) {
    constexpr int kStreams = 8;
    for (int i = 0; i < std::min(kStreams, nbox); ++i) {
      hipStream_t st = nullptr;
      IBF_HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      M.streams.push_back(st);
    }
    IBF_HIP_CHECK(hipEventCreateWithFlags(&M.ev_start, hipEventDisableTiming));
    M.ev_u.assign(nbox, nullptr);
    for (int i = 0; i < nbox; ++i)
      IBF_HIP_CHECK(hipEventCreateWithFlags(&M.ev_u[i], hipEventDisableTiming));
  }
  {
    const int rc = prepare_batched2d<VT, FT>(p, nrhs, off, s);
    if (rc) return rc;
  }
  if (M.graph_failed || std::getenv("IBF_NO_GRAPH"))
    return launch2d_t<VT, FT>(p, g, ldg, u, ldu, nrhs, s, off);
  const std::vector<int64_t> key = {(int64_t)(uintptr_t)g, ldg, (int64_t)(uintptr_t)u, ldu,
                                    nrhs, (int64_t)(uintptr_t)M.d_work,
                                    (int64_t)(uintptr_t)M.d_table, (int64_t)M.batched};
  if (!M.exec || key != M.graph_key) {
    if (M.exec) (void)hipGraphExecDestroy(M.exec);
    if (M.graph) (void)hipGraphDestroy(M.graph);
    M.exec = nullptr;
    M.graph = nullptr;
    M.graph_key.clear();
    if (!M.cap) IBF_HIP_CHECK(hipStreamCreateWithFlags(&M.cap, hipStreamNonBlocking));
    IBF_HIP_CHECK(hipStreamBeginCapture(M.cap, hipStreamCaptureModeThreadLocal));
    const int lrc = launch2d_t<VT, FT>(p, g, ldg, u, ldu, nrhs, M.cap, off);
    hipGraph_t gr = nullptr;
    const hipError_t ec = hipStreamEndCapture(M.cap, &gr);
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = (lrc == IBF_OK && ec == hipSuccess && gr)
                              ? hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0)
                              : hipErrorUnknown;
    if (ei != hipSuccess) {
      // capture or instantiation refused: clear the error and launch directly
      if (gr) (void)hipGraphDestroy(gr);
      (void)hipGetLastError();
      M.graph_failed = true;
      return launch2d_t<VT, FT>(p, g, ldg, u, ldu, nrhs, s, off);
    }
    M.graph = gr;
    M.exec = ex;
    M.graph_key = key;
  }
  IBF_HIP_CHECK(hipGraphLaunch(M.exec, s));
  return IBF_OK;
}

// The launch sequence of one 2-D apply on stream s: the centre block, then
// per box V and the quadtree stages on a worker stream, then U per X tree
// back on s.
template <typename VT, typename FT>
int launch2d_t(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int nrhs,
               hipStream_t s, const std::vector<size_t>& off) {
  Mibf2D& M = *p->mibf;
  const int nbox = (int)M.boxes.size();
  const int nc = (int)M.centre.size();
  // the centre block writes every entry of u; the boxes then accumulate
  constexpr int NR = kNR2;
  const int nchunk = (nrhs + NR - 1) / NR;
  {
    const size_t lds = ((size_t)nc * NR + (size_t)kB2 * 17) * sizeof(VT);
    if (lds <= 64 * 1024) {
      hipLaunchKernelGGL((k2_apply_centre_rows<VT, FT, NR>),
                         dim3((unsigned)((M.nx + kB2 - 1) / kB2 * nchunk)), dim3(kB2), lds, s,
                         (const FT*)M.d_kc, nc, M.d_cidx, (const VT*)g, ldg, M.nx, (VT*)u, ldu,
                         nrhs, nchunk);
    } else {
      hipLaunchKernelGGL((k2_apply_centre<VT, FT>), dim3(nblk(M.nx * nrhs)), dim3(kB2), 0, s,
                         (const FT*)M.d_kc, nc, M.d_cidx, (const VT*)g, ldg, M.nx, (VT*)u, ldu,
                         nrhs);
    }
    IBF_HIP_CHECK(hipGetLastError());
  }
  std::vector<const void*> mu_final(nbox, nullptr);
  if (M.batched) {
    // one stream: V of every box, then stage j of every box per launch
    const char* base = static_cast<const char*>(M.d_table);
    {
      const Launch2& x = M.launches[0];
      hipLaunchKernelGGL((k2_batch_v_rows<VT, FT, NR>), dim3((unsigned)x.nblocks), dim3(kB2),
                         x.lds, s, reinterpret_cast<const V2Desc*>(base + x.desc_off),
                         reinterpret_cast<const int64_t*>(base + x.boff_off), x.count,
                         (const VT*)g, ldg, nrhs, nchunk);
      IBF_HIP_CHECK(hipGetLastError());
    }
    for (size_t j = 1; j < M.launches.size(); ++j) {
      const Launch2& x = M.launches[j];
      hipLaunchKernelGGL((k2_batch_stage_quad<VT, FT, NR>), dim3((unsigned)x.nblocks),
                         dim3(kB2), x.lds, s,
                         reinterpret_cast<const Stage2Desc*>(base + x.desc_off),
                         reinterpret_cast<const int64_t*>(base + x.boff_off), x.count, nrhs,
                         nchunk);
      IBF_HIP_CHECK(hipGetLastError());
    }
    for (int ib = 0; ib < nbox; ++ib) {
      char* wb = static_cast<char*>(M.d_work) + off[ib];
      mu_final[ib] = wb + (M.boxes[ib].stages.size() & 1) * ((off[ib + 1] - off[ib]) / 2);
    }
  } else {
  if (nbox) IBF_HIP_CHECK(hipEventRecord(M.ev_start, s));
  for (int ib = 0; ib < nbox; ++ib) {
    const Box2& bx = M.boxes[ib];
    hipStream_t bs = M.streams[ib % M.streams.size()];
    IBF_HIP_CHECK(hipStreamWaitEvent(bs, M.ev_start, 0));
    char* wb = static_cast<char*>(M.d_work) + off[ib];
    VT* w[2] = {reinterpret_cast<VT*>(wb), reinterpret_cast<VT*>(wb + (off[ib + 1] - off[ib]) / 2)};
    const int lO = bx.L - bx.lV;
    const int64_t npv = ((int64_t)1 << (2 * bx.lV)) * ((int64_t)1 << (2 * lO));
    {
      const size_t lds = (size_t)bx.smax_xi * NR * sizeof(VT);
      if (lds <= 64 * 1024) {
        const int64_t nleafb = (int64_t)1 << (2 * lO);
        hipLaunchKernelGGL((k2_apply_v_rows<VT, FT, NR>), dim3((unsigned)(nleafb * nchunk)),
                           dim3(kB2), lds, bs, (const VT*)g, ldg, bx.d_perm_xi, bx.d_xioff,
                           (const FT*)bx.d_vbar, w[0], bx.lV, lO, bx.K_V, nrhs, bx.smax_xi,
                           nchunk);
      } else {
        hipLaunchKernelGGL((k2_apply_v<VT, FT>), dim3(nblk(npv * bx.K_V * nrhs)), dim3(kB2), 0,
                           bs, (const VT*)g, ldg, bx.d_perm_xi, bx.d_xioff, (const FT*)bx.d_vbar,
                           w[0], bx.lV, lO, bx.K_V, nrhs);
      }
      IBF_HIP_CHECK(hipGetLastError());
    }
    int cur = 0;
    for (const Stage2& st : bx.stages) {
      const int64_t nquad = (int64_t)1 << (2 * bx.L - 2);
      const int qb = stage_qb<VT>(st);
      const size_t lds = (size_t)qb * 4 * st.kin * NR * sizeof(VT);
      const int64_t nb = (nquad + qb - 1) / qb * nchunk;
      if (4 * st.kout <= kB2 && lds <= 64 * 1024 && nb < 0x7fffffff) {
        hipLaunchKernelGGL((k2_apply_stage_quad<VT, FT, NR>), dim3((unsigned)nb), dim3(kB2),
                           lds, bs, w[cur], w[cur ^ 1], (const FT*)st.blk, bx.L, st.level,
                           st.kin, st.kout, st.kld, nrhs, qb, nchunk);
      } else {
        const int64_t np = (int64_t)1 << (2 * bx.L);
        hipLaunchKernelGGL((k2_apply_stage<VT, FT>), dim3(nblk(np * st.kout * nrhs)), dim3(kB2),
                           0, bs, w[cur], w[cur ^ 1], (const FT*)st.blk, bx.L, st.level, st.kin,
                           st.kout, st.kld, nrhs);
      }
      IBF_HIP_CHECK(hipGetLastError());
      cur ^= 1;
    }
    mu_final[ib] = w[cur];
    IBF_HIP_CHECK(hipEventRecord(M.ev_u[ib], bs));
  }
  }
  // U on the caller's stream, one launch per X tree (at most kTreeBoxes boxes
  // a launch), each after its boxes' stages: u accumulates in tree order,
  // then box order, and the caller's stream continues after the last one
  for (int t = 0; t < (int)M.xtrees.size(); ++t) {
    const XTree2& xt = M.xtrees[t];
    UTree T{};
    auto flush = [&]() -> int {
      if (!T.nb) return IBF_OK;
      hipLaunchKernelGGL((k2_apply_u_tree<VT, FT, NR>),
                         dim3((unsigned)((M.nx + kB2 - 1) / kB2 * nchunk)), dim3(kB2), 0, s, T,
                         xt.d_perm, xt.d_leaf, M.nx, (VT*)u, ldu, nrhs, nchunk);
      IBF_HIP_CHECK(hipGetLastError());
      T.nb = 0;
      return IBF_OK;
    };
    for (int ib = 0; ib < nbox; ++ib) {
      const Box2& bx = M.boxes[ib];
      if (bx.xt != t) continue;
      if (!M.batched) IBF_HIP_CHECK(hipStreamWaitEvent(s, M.ev_u[ib], 0));
      T.mu[T.nb] = mu_final[ib];
      T.ubar[T.nb] = bx.d_ubar;
      T.K[T.nb] = bx.K_U;
      if (++T.nb == kTreeBoxes) {
        int rc;
        if ((rc = flush())) return rc;
      }
    }
    int rc;
    if ((rc = flush())) return rc;
  }
  return IBF_OK;
}

}  // namespace

int plan2d(const ibf_desc* d, ibf_plan_t* out) {
  auto bad = [](const char* msg) {
    set_error(msg);
    return IBF_ERR_INVALID_ARG;
  };
  if (d->r < 2 || d->r > 9) {
    set_error("ibf_plan: dim 2 supports r = 2 .. 9 (r^2 <= 81 grid points per box)");
    return d->r < 2 ? IBF_ERR_INVALID_ARG : IBF_ERR_UNSUPPORTED;
  }
  if (!(d->tol > 0.0 && d->tol < 1.0)) return bad("ibf_plan: tol must lie in (0, 1)");
  int leaf_side = 0;
  for (int s = 1; s <= 8; s *= 2)
    if (s * s == d->leaf) leaf_side = s;
  if (leaf_side < 2) return bad("ibf_plan: dim 2 needs leaf = 4, 16 or 64 points (a square)");
  if (d->precision < IBF_FP64 || d->precision > IBF_BF16X2)
    return bad("ibf_plan: unknown precision");
  if (d->sweep_in > 0) {   // -1 (auto) resolves to off: grid leaves are full
    set_error("ibf_plan: the sweep-in stage is not provided for dim 2");
    return IBF_ERR_UNSUPPORTED;
  }
  if (d->sweep_in < -1) return bad("ibf_plan: sweep_in must be -1, 0 or 1");
  if (d->amp_id != IBF_AMP_NONE || d->fixed_ranks) {
    set_error("ibf_plan: amplitudes and fixed ranks are provided for dim 1");
    return IBF_ERR_UNSUPPORTED;
  }
  if (d->svd_samples < 0) return bad("ibf_plan: svd_samples < 0");
  const double W = d->omega_width;
  int Lw = 0;
  while ((double)((int64_t)1 << Lw) < W) ++Lw;
  if (!(W > 0) || (double)((int64_t)1 << Lw) != W || W < 2 * kCentreSide || Lw > 24)
    return bad("ibf_plan: dim 2 needs omega_width a power of two >= 32");
  if (d->omega_lo != -W / 2) return bad("ibf_plan: dim 2 needs omega_lo = -omega_width / 2");
  PhaseDesc ph{};
  ph.kind = d->phase_id;
  const double* pp = d->phase_params;
  const int np = d->n_params;
  if (np < 0 || np > kMaxParams || (np > 0 && !pp)) return bad("ibf_plan: bad phase parameters");
  switch (d->phase_id) {
    case IBF_PHASE_DFT:
      ph.p[0] = np >= 1 ? pp[0] : 1.0;
      if (ph.p[0] != 1.0 && ph.p[0] != -1.0) return bad("ibf_plan: DFT sign must be +1 or -1");
      break;
    case IBF_PHASE_FIO2D:
      ph.p[0] = np >= 1 ? pp[0] : 2.0;
      ph.p[1] = np >= 2 ? pp[1] : 1.0;
      ph.p[2] = np >= 3 ? pp[2] : 16.0;
      if (ph.p[2] == 0.0) return bad("ibf_plan: p2 == 0");
      break;
    case IBF_PHASE_SEPARABLE:
      ph.p[0] = np >= 1 ? pp[0] : 3.0;
      ph.p[1] = np >= 2 ? pp[1] : 0.3125;
      break;
    default:
      set_error("ibf_plan: unsupported phase for dim 2");
      return IBF_ERR_UNSUPPORTED;
  }
  auto M = new Mibf2D();
  M->ph = ph;
  M->r = d->r;
  M->R2 = d->r * d->r;
  M->leaf_side = leaf_side;
  M->precision = d->precision;
  M->device = d->device;
  M->tol = d->tol;
  M->ssamp = d->svd_samples;
  M->sseed = d->svd_seed;
  M->W = W;
  M->nx = d->n_x;
  M->nxi = d->n_xi;
  for (int64_t i = 0; i < 2 * d->n_x; ++i)
    if (!(d->x[i] >= 0.0 && d->x[i] < 1.0)) {
      delete M;
      return bad("ibf_plan: x outside [0, 1)^2");
    }
  M->xi_host.assign(d->xi, d->xi + 2 * d->n_xi);
  // coronas (eq:domaindecomp): boxes of side W / 2^(t+2) between the squares of
  // half-width W / 2^(t+1) and W / 2^(t+2); centre [-c/2, c/2)^2
  struct BoxGeo { double o1, o2, w; };
  std::vector<BoxGeo> geo;
  std::vector<int> first_box;           // index of the first box of corona t
  for (int t = 0;; ++t) {
    const double hw = W / std::ldexp(1.0, t + 1), w = W / std::ldexp(1.0, t + 2);
    if (!(hw > kCentreSide / 2) || w < leaf_side) break;
    first_box.push_back((int)geo.size());
    for (int i1 = 0; i1 < 4; ++i1)
      for (int i2 = 0; i2 < 4; ++i2) {
        if (i1 >= 1 && i1 <= 2 && i2 >= 1 && i2 <= 2) continue;
        geo.push_back({-hw + i1 * w, -hw + i2 * w, w});
      }
  }
  const double hc = W / std::ldexp(1.0, (int)first_box.size() + 1);   // centre half-side
  M->box_pts.assign(geo.size(), {});
  for (int64_t j = 0; j < d->n_xi; ++j) {
    const double k1 = d->xi[2 * j], k2 = d->xi[2 * j + 1];
    if (!(k1 >= -W / 2 && k1 < W / 2 && k2 >= -W / 2 && k2 < W / 2)) {
      delete M;
      return bad("ibf_plan: xi outside [omega_lo, omega_lo + omega_width)^2");
    }
    if (k1 >= -hc && k1 < hc && k2 >= -hc && k2 < hc) {
      M->centre.push_back((int32_t)j);
      continue;
    }
    int t = 0;
    while (k1 >= -W / std::ldexp(1.0, t + 2) && k1 < W / std::ldexp(1.0, t + 2) &&
           k2 >= -W / std::ldexp(1.0, t + 2) && k2 < W / std::ldexp(1.0, t + 2))
      ++t;                              // inside the next inner square
    const double hw = W / std::ldexp(1.0, t + 1), w = W / std::ldexp(1.0, t + 2);
    const int i1 = (int)std::floor((k1 + hw) / w), i2 = (int)std::floor((k2 + hw) / w);
    int idx = first_box[t];
    for (int a1 = 0; a1 < 4; ++a1)
      for (int a2 = 0; a2 < 4; ++a2) {
        if (a1 >= 1 && a1 <= 2 && a2 >= 1 && a2 <= 2) continue;
        if (a1 == i1 && a2 == i2) M->box_pts[idx].push_back((int32_t)j);
        ++idx;
      }
  }
  int lV = 0;
  while ((1 << lV) < leaf_side) ++lV;
  for (size_t i = 0; i < geo.size(); ++i) {
    Box2 bx;
    bx.o1 = geo[i].o1;
    bx.o2 = geo[i].o2;
    bx.w = geo[i].w;
    int L = 0;
    while ((double)(1 << L) < bx.w) ++L;
    bx.L = L;
    bx.lV = lV;
    bx.h = (lV + L) / 2;
    bx.m = (int64_t)M->box_pts[i].size();
    M->maxL = std::max(M->maxL, L);
    const int64_t R2 = M->R2;
    bx.nnz_prelim = bx.m * ((int64_t)1 << (2 * lV)) * R2 + M->nx * R2 +
                    (int64_t)(L - lV) * ((int64_t)1 << (2 * L)) * 4 * R2 * R2 +
                    ((int64_t)1 << (2 * L)) * R2 * R2;
    M->nnz_prelim += bx.nnz_prelim;
    M->boxes.push_back(bx);
  }
  M->nnz_prelim += M->nx * (int64_t)M->centre.size();
  auto pl = new ibf_plan_s();
  pl->dim = 2;
  pl->nx = d->n_x;
  pl->nxi = d->n_xi;
  pl->device = d->device;
  pl->phase = ph;
  pl->r = d->r;
  pl->leaf = d->leaf;
  pl->precision = d->precision;
  pl->tol = d->tol;
  pl->nnz_prelim = M->nnz_prelim;
  pl->mibf = M;
  // keep the caller's X for the device upload at build time
  pl->xs.assign(d->x, d->x + 2 * d->n_x);
  *out = pl;
  return IBF_OK;
}

int build2d(ibf_plan_t p, hipStream_t s) {
  Mibf2D& M = *p->mibf;
  IBF_HIP_CHECK(hipSetDevice(M.device));
  free2d_factors(p);
  int rc;
  if ((rc = upload(&M.d_x, p->xs.data(), p->xs.size()))) return rc;
  // X trees, one per distinct box depth
  for (Box2& bx : M.boxes) {
    int found = -1;
    for (size_t t = 0; t < M.xtrees.size(); ++t)
      if (M.xtrees[t].L == bx.L) found = (int)t;
    if (found < 0) {
      XTree2 xt;
      xt.L = bx.L;
      const int64_t nb = (int64_t)1 << bx.L;
      std::vector<int64_t> code(M.nx);
      for (int64_t i = 0; i < M.nx; ++i) {
        const int64_t i1 = std::min<int64_t>((int64_t)std::floor(p->xs[2 * i] * nb), nb - 1);
        const int64_t i2 = std::min<int64_t>((int64_t)std::floor(p->xs[2 * i + 1] * nb), nb - 1);
        code[i] = morton_host(i1, i2, bx.L);
      }
      std::vector<int32_t> perm, off, bin;
      sort_codes(code, nb * nb, perm, off, bin);
      std::vector<double> xs(2 * M.nx);
      for (int64_t i = 0; i < M.nx; ++i) {
        xs[2 * i] = p->xs[2 * (size_t)perm[i]];
        xs[2 * i + 1] = p->xs[2 * (size_t)perm[i] + 1];
      }
      if ((rc = upload(&xt.d_xs, xs.data(), xs.size()))) return rc;
      if ((rc = upload(&xt.d_perm, perm.data(), perm.size()))) return rc;
      if ((rc = upload(&xt.d_leaf, bin.data(), bin.size()))) return rc;
      M.xtrees.push_back(xt);
      found = (int)M.xtrees.size() - 1;
    }
    bx.xt = found;
  }
  // Omega points of every box, sorted into its leaves
  for (size_t i = 0; i < M.boxes.size(); ++i) {
    Box2& bx = M.boxes[i];
    const int lO = bx.L - bx.lV;
    const int64_t nb = (int64_t)1 << lO;
    const auto& pts = M.box_pts[i];
    std::vector<int64_t> code(pts.size());
    for (size_t j = 0; j < pts.size(); ++j) {
      const double k1 = M.xi_host[2 * (size_t)pts[j]], k2 = M.xi_host[2 * (size_t)pts[j] + 1];
      const int64_t j1 = std::min<int64_t>((int64_t)std::floor((k1 - bx.o1) * nb / bx.w), nb - 1);
      const int64_t j2 = std::min<int64_t>((int64_t)std::floor((k2 - bx.o2) * nb / bx.w), nb - 1);
      code[j] = morton_host(j1, j2, lO);
    }
    std::vector<int32_t> perm, off, bin;
    sort_codes(code, nb * nb, perm, off, bin);
    std::vector<double> xis(2 * pts.size());
    std::vector<int32_t> cperm(pts.size());
    for (size_t j = 0; j < pts.size(); ++j) {
      cperm[j] = pts[perm[j]];
      xis[2 * j] = M.xi_host[2 * (size_t)cperm[j]];
      xis[2 * j + 1] = M.xi_host[2 * (size_t)cperm[j] + 1];
    }
    if ((rc = upload(&bx.d_xis, xis.data(), xis.size()))) return rc;
    if ((rc = upload(&bx.d_perm_xi, cperm.data(), cperm.size()))) return rc;
    if ((rc = upload(&bx.d_xileaf, bin.data(), bin.size()))) return rc;
    if ((rc = upload(&bx.d_xioff, off.data(), off.size()))) return rc;
    bx.smax_xi = 0;
    for (size_t b = 0; b + 1 < off.size(); ++b)
      bx.smax_xi = std::max<int>(bx.smax_xi, off[b + 1] - off[b]);
  }
  M.nnz_opt = M.nnz_stored = M.factor_bytes = 0;
  switch (M.precision) {
    case IBF_FP64: rc = build2d_t<double2>(p, s); break;
    case IBF_FP32: rc = build2d_t<float2>(p, s); break;
    default: rc = build2d_t<bf16x2c>(p, s); break;
  }
  if (rc) return rc;
  IBF_HIP_CHECK(hipStreamSynchronize(s));
  p->nnz_opt = M.nnz_opt;
  p->nnz_stored = M.nnz_stored;
  p->built = true;
  return IBF_OK;
}

int apply2d(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs,
            hipStream_t s) {
  IBF_HIP_CHECK(hipSetDevice(p->mibf->device));
  if (nrhs > 65535) {
    set_error("ibf_apply: nrhs too large for dim 2");
    return IBF_ERR_INVALID_ARG;
  }
  switch (p->mibf->precision) {
    case IBF_FP64: return apply2d_t<double2, double2>(p, g, ldg, u, ldu, (int)nrhs, s);
    case IBF_FP32: return apply2d_t<float2, float2>(p, g, ldg, u, ldu, (int)nrhs, s);
    default: return apply2d_t<float2, bf16x2c>(p, g, ldg, u, ldu, (int)nrhs, s);
  }
}

void free2d_factors(ibf_plan_t p) {
  if (!p->mibf) return;
  Mibf2D& M = *p->mibf;
  auto fr = [](void* b) {
    if (b) (void)ibf::dev_free(b);
  };
  for (Box2& bx : M.boxes) {
    for (auto& st : bx.stages) fr(st.blk);
    bx.stages.clear();
    fr(bx.d_vbar);
    fr(bx.d_ubar);
    fr(bx.d_xis);
    fr(bx.d_perm_xi);
    fr(bx.d_xileaf);
    fr(bx.d_xioff);
    bx.d_vbar = bx.d_ubar = nullptr;
    bx.d_xis = nullptr;
    bx.d_perm_xi = bx.d_xileaf = bx.d_xioff = nullptr;
  }
  for (XTree2& xt : M.xtrees) {
    fr(xt.d_xs);
    fr(xt.d_perm);
    fr(xt.d_leaf);
  }
  M.xtrees.clear();
  fr(M.d_x);
  fr(M.d_cidx);
  fr(M.d_kc);
  fr(M.d_z);
  fr(M.d_lc);
  fr(M.d_work);
  for (hipStream_t st : M.streams) (void)hipStreamDestroy(st);
  M.streams.clear();
  for (hipEvent_t e : M.ev_u) (void)hipEventDestroy(e);
  M.ev_u.clear();
  if (M.ev_start) (void)hipEventDestroy(M.ev_start);
  M.ev_start = nullptr;
  if (M.exec) (void)hipGraphExecDestroy(M.exec);
  if (M.graph) (void)hipGraphDestroy(M.graph);
  if (M.cap) (void)hipStreamDestroy(M.cap);
  fr(M.d_table);
  M.d_table = nullptr;
  M.table_bytes = 0;
  M.table_key.clear();
  M.launches.clear();
  M.batched = false;
  M.exec = nullptr;
  M.graph = nullptr;
  M.cap = nullptr;
  M.graph_key.clear();
  M.d_x = nullptr;
  M.d_cidx = nullptr;
  M.d_kc = nullptr;
  M.d_z = M.d_lc = nullptr;
  M.d_work = nullptr;
  M.work_bytes = 0;
  M.built = false;
  p->built = false;
}

void destroy2d(ibf_plan_t p) {
  if (!p->mibf) return;
  const Mibf2D& M = *p->mibf;
  bool touched = M.d_x || M.d_z || M.d_kc || M.d_work || !M.xtrees.empty();
  for (const Box2& bx : M.boxes) touched = touched || bx.d_xis || bx.d_vbar;
  if (touched) {                       // a plan that never reached the device makes no HIP call
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(M.device);
    free2d_factors(p);
    (void)hipSetDevice(cur);
  }
  delete p->mibf;
  p->mibf = nullptr;
}

void query2d(ibf_plan_t p, ibf_info* info) {
  const Mibf2D& M = *p->mibf;
  info->L = M.maxL;
  info->l0 = M.boxes.empty() ? 0 : M.boxes[0].lV;
  info->h = 0;
  info->n_levels = 0;
  info->n_pairs = 0;
  for (const Box2& bx : M.boxes) info->n_pairs += (int64_t)1 << (2 * bx.L);
  info->nnz_prelim = M.nnz_prelim;
  info->nnz_opt = M.nnz_opt;
  info->nnz_stored = M.nnz_stored;
  info->factor_bytes = M.factor_bytes;
  info->build_ms = p->build_ms;
  // per-box level ranks of the outermost corona's first box
  if (!M.boxes.empty()) {
    const Box2& bx = M.boxes[0];
    info->n_levels = (int)bx.rank.size();
    for (size_t i = 0; i < bx.rank.size() && i < 64; ++i) info->rank[i] = bx.rank[i];
  }
}

// Direct 2-D product u(x_i) = sum_j exp(2 pi i Phi(x_i, xi_j)) g_j (the dense
// definition of Sec. 5 with the phases of Sec. 6.3) in FP64: one thread per
// (row, right-hand side); x and xi are [n][2].
__global__ __launch_bounds__(256) void k2_dense(PhaseDesc ph, const double* __restrict__ x,
                                                int64_t nx, const double* __restrict__ xi,
                                                int64_t nxi, const double2* __restrict__ g,
                                                int64_t ldg, double2* __restrict__ u,
                                                int64_t ldu) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i >= nx) return;
  const double x1 = x[2 * i], x2 = x[2 * i + 1];
  const double2* gc = g + c * ldg;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t j = 0; j < nxi; ++j) {
    const double2 k = kval2(ph, x1, x2, xi[2 * j], xi[2 * j + 1]);
    const double2 gv = gc[j];
    acc.x = fma(k.x, gv.x, fma(-k.y, gv.y, acc.x));
    acc.y = fma(k.x, gv.y, fma(k.y, gv.x, acc.y));
  }
  u[c * ldu + i] = acc;
}

int dense_apply_2d(const PhaseDesc& ph, const double* x, int64_t nx, const double* xi,
                   int64_t nxi, const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs,
                   hipStream_t s) {
  hipLaunchKernelGGL(k2_dense, dim3((unsigned)((nx + 255) / 256), (unsigned)nrhs), dim3(256), 0,
                     s, ph, x, nx, xi, nxi, (const double2*)g, ldg, (double2*)u, ldu);
  IBF_HIP_CHECK(hipGetLastError());
  return IBF_OK;
}

}  // namespace ibf
