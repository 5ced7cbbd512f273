// Application of the compressed IBF: u = U Gbar ... Gbar [Mdot] Hbar ... Hbar V^* g
// (paper Sec. 4, eqn:IBFout / eqn:IBFin), a sequence of block-sparse products.
//
// Coefficient vectors live in ping-pong buffers laid out [pair][k][rhs]; pair
// p at level l is the bit string p = a 2^(L-l) + b (a: T_X box at level l,
// b: T_Omega box at level L-l).  One butterfly stage maps the inputs
// (a>>1, 2b) and (a>>1, 2b+1) at level l-1 to the output (a, b) at level l
// through a k_out x 2 k_in block.  Fusing k consecutive stages closes over a
// contiguous group of 2^k input pairs, whose 2^k outputs land at stride
// 2^(L - l_end): one workgroup keeps such a group (for a chunk of the
// right-hand sides) in LDS across the k stages.
//
// Kernels:
//   k_apply_v      Omega leaf -> 2^l0 pairs:  mu = Vbar^* g   (per-leaf GEMM, LDS-staged)
//   k_apply_fused  k butterfly stages on one pair group in LDS
//   k_apply_mid    swept-in middle block Mdot (per pair)
//   k_apply_u      2^l0 pairs -> X leaf:  u = Ubar mu        (per-leaf GEMM, LDS-staged)
#include <algorithm>
#include <cstdio>
#include <vector>

#include "ibf_device.h"

namespace ibf {
namespace {

constexpr int kBlock = 256;
constexpr int kKmax = kMaxR;          // largest stored rank
constexpr int kNumXcd = 8;            // MI355X: 8 XCDs, each with its own L2

template <typename VT> struct Zero;
template <> struct Zero<double2> { __device__ static double2 v() { return make_double2(0, 0); } };
template <> struct Zero<float2> { __device__ static float2 v() { return make_float2(0, 0); } };

// Block index remapped so that consecutive logical blocks run on one XCD
// (hardware dispatches block i to XCD i mod 8): RHS chunks of one pair group
// then share an L2 for the factor blocks they all read.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t nblk) {
  const int64_t b = blockIdx.x;
  if (nblk % kNumXcd) return b;
  return (b % kNumXcd) * (nblk / kNumXcd) + b / kNumXcd;
}

// ---------------------------------------------------------------------------
// V: per (Omega leaf b, RHS chunk): mu[(a,b)][k][n] = sum_{xi in b} Vbar^*[xi][a][k] g[xi][n]
// LDS: g_leaf[cnt][NB], vbar_leaf[cnt][2^l0][K].
// ---------------------------------------------------------------------------
template <typename VT, typename FT>
__global__ __launch_bounds__(kBlock) void k_apply_v(
    const VT* __restrict__ g, int64_t ldg, const int32_t* __restrict__ perm_xi,
    const int32_t* __restrict__ xioff, const FT* __restrict__ vbar, VT* __restrict__ mu, int L,
    int l0, int K, int nrhs, int NB, int nchunk, int smax, int stage_factor) {
  extern __shared__ __align__(16) unsigned char smem[];
  VT* gl = reinterpret_cast<VT*>(smem);                       // [smax][NB]
  VT* vl = gl + (size_t)smax * NB;                            // [smax][2^l0][K] if staged
  const int64_t nblk = (int64_t)gridDim.x;
  const int64_t lb = xcd_logical_block(nblk);
  const int64_t b = lb / nchunk;
  const int chunk = (int)(lb % nchunk);
  const int nb0 = chunk * NB;
  const int nbw = min(NB, nrhs - nb0);
  const int32_t j0 = xioff[b], cnt = xioff[b + 1] - j0;
  const int na = 1 << l0;
  // gather g for the leaf (points fastest: contiguous in a column)
  for (int e = threadIdx.x; e < cnt * nbw; e += blockDim.x) {
    const int j = e % cnt, n = e / cnt;
    gl[j * NB + n] = g[(int64_t)(nb0 + n) * ldg + perm_xi[j0 + j]];
  }
  const FT* vsrc = vbar + (int64_t)j0 * na * K;
  if (stage_factor)
    for (int e = threadIdx.x; e < cnt * na * K; e += blockDim.x) vl[e] = load_factor(vsrc, e);
  __syncthreads();
  const int sh = L - l0;
  for (int item = threadIdx.x; item < na * nbw; item += blockDim.x) {
    const int n = item % nbw, a = item / nbw;
    VT acc[kKmax];
#pragma unroll
    for (int k = 0; k < kKmax; ++k) acc[k] = Zero<VT>::v();
    for (int j = 0; j < cnt; ++j) {
      const VT gv = gl[j * NB + n];
      const int64_t off = ((int64_t)j * na + a) * K;
      if (stage_factor) {
        const VT* vr = vl + off;
#pragma unroll
        for (int k = 0; k < kKmax; ++k)
          if (k < K) cfma(acc[k], vr[k], gv);
      } else {
#pragma unroll
        for (int k = 0; k < kKmax; ++k)
          if (k < K) cfma(acc[k], load_factor(vsrc, off + k), gv);
      }
    }
    const int64_t p = ((int64_t)a << sh) | b;
    VT* o = mu + p * K * nrhs + nb0 + n;
#pragma unroll
    for (int k = 0; k < kKmax; ++k)
      if (k < K) o[(int64_t)k * nrhs] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// Fused butterfly stages l_start .. l_start+nst-1 on one group of 2^nst
// contiguous input pairs (level l_start-1) and one RHS chunk.  In LDS the
// group's pair at level l_start-1+j has local index (alpha bits << (nst-j)) |
// (remaining child bits); a stage consumes the lowest child bit and appends
// an alpha bit.  Outputs of a stage are held in registers across a barrier
// and written back in place.  ranks[j] = K at level l_start-1+j.
// ---------------------------------------------------------------------------
struct FusedArgs {
  int L, l_start, nst, nrhs, NB, nchunk, ipt;
  int ranks[kMaxR + 1];
  const void* blk[kMaxR];
};

template <typename VT, typename FT>
__global__ __launch_bounds__(kBlock) void k_apply_fused(const VT* __restrict__ in,
                                                        VT* __restrict__ out, FusedArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  VT* S = reinterpret_cast<VT*>(smem);                        // [2^nst][Kmax_g][NB]
  const int k = A.nst, NB = A.NB, L = A.L;
  int kmaxg = 1;
  for (int j = 0; j <= k; ++j) kmaxg = max(kmaxg, A.ranks[j]);
  const int64_t nblk = (int64_t)gridDim.x;
  const int64_t lb = xcd_logical_block(nblk);
  const int64_t gid = lb / A.nchunk;
  const int chunk = (int)(lb % A.nchunk);
  const int nb0 = chunk * NB;
  const int nbw = min(NB, A.nrhs - nb0);
  const int nslot = 1 << k;
  const int nrhs = A.nrhs;
  const int sh_end = L - (A.l_start + k - 1);

  // load the group: slot c <- input pair (gid << k) | c
  {
    const int kin = A.ranks[0];
    const int64_t base = (gid << k) * kin * nrhs;
    for (int e = threadIdx.x; e < nslot * kin * nbw; e += blockDim.x) {
      const int n = e % nbw;
      const int rs = e / nbw;                                 // slot * kin + s
      S[(size_t)rs / kin * kmaxg * NB + (rs % kin) * NB + n] =
          in[base + (int64_t)rs * nrhs + nb0 + n];
    }
  }
  __syncthreads();
  const int64_t ap = gid >> sh_end;
  const int64_t bpp = gid & (((int64_t)1 << sh_end) - 1);
  for (int j = 0; j < k; ++j) {
    const int l = A.l_start + j;
    const int kin = A.ranks[j], kout = A.ranks[j + 1];
    const FT* blk = reinterpret_cast<const FT*>(A.blk[j]);
    const int rem = k - j - 1;                                // child bits left after this stage
    const int nitems = nslot * nbw;
    VT hold[2][kKmax];
    int hold_slot[2], hold_n[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      hold_slot[it] = -1;
      hold_n[it] = 0;
      const int item = threadIdx.x + it * blockDim.x;
      if (it < A.ipt && item < nitems) {
        const int n = item % nbw;
        const int locp = item / nbw;                          // output local index
        const int anew = locp >> rem;                         // alpha bits incl. the new one
        const int q = locp & ((1 << rem) - 1);
        const int abits = anew >> 1;
        const int loc0 = (abits << (rem + 1)) | (2 * q);
        const int64_t a_l = (ap << (j + 1)) | anew;
        const int64_t b_l = (bpp << rem) | q;
        const int64_t pout = (a_l << (L - l)) | b_l;
        // stored block layout: [pair][c kin + s][t]
        const FT* col0 = blk + pout * kout * 2 * kin;
        VT acc[kKmax];
#pragma unroll
        for (int t = 0; t < kKmax; ++t) acc[t] = Zero<VT>::v();
        for (int c = 0; c < 2; ++c) {
          const VT* src = S + (size_t)(loc0 + c) * kmaxg * NB + n;
          for (int s = 0; s < kin; ++s) {
            const VT xv = src[s * NB];
            const FT* col = col0 + (int64_t)(c * kin + s) * kout;
#pragma unroll
            for (int t = 0; t < kKmax; ++t)
              if (t < kout) cfma(acc[t], load_factor(col, t), xv);
          }
        }
#pragma unroll
        for (int t = 0; t < kKmax; ++t) hold[it][t] = acc[t];
        hold_slot[it] = locp;
        hold_n[it] = n;
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      if (hold_slot[it] >= 0) {
        VT* dst = S + (size_t)hold_slot[it] * kmaxg * NB + hold_n[it];
#pragma unroll
        for (int t = 0; t < kKmax; ++t)
          if (t < kout) dst[t * NB] = hold[it][t];
      }
    }
    __syncthreads();
  }
  // store: final slot loc -> output pair (ap << (k + sh_end)) | (loc << sh_end) | bpp
  {
    const int kout = A.ranks[k];
    for (int e = threadIdx.x; e < nslot * kout * nbw; e += blockDim.x) {
      const int n = e % nbw;
      const int rs = e / nbw;
      const int loc = rs / kout, t = rs % kout;
      const int64_t pout = (ap << (k + sh_end)) | ((int64_t)loc << sh_end) | bpp;
      out[(pout * kout + t) * nrhs + nb0 + n] = S[(size_t)loc * kmaxg * NB + t * NB + n];
    }
  }
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

// ---------------------------------------------------------------------------
// U: per (X leaf a, RHS chunk): u[perm(x)][n] = sum_b sum_k Ubar[x][b][k] mu[(a,b)][k][n]
// LDS: mu_leaf[2^l0][K][NB], ubar_leaf[cnt][2^l0 K + 1] (padded rows).
// ---------------------------------------------------------------------------
template <typename VT, typename FT>
__global__ __launch_bounds__(kBlock) void k_apply_u(
    const VT* __restrict__ mu, VT* __restrict__ u, int64_t ldu, const int32_t* __restrict__ perm_x,
    const int32_t* __restrict__ xoff, const FT* __restrict__ ubar, int l0, int K, int nrhs,
    int NB, int nchunk, int smax, int stage_factor) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nb = 1 << l0;
  const int urow = nb * K + 1;
  VT* ml = reinterpret_cast<VT*>(smem);                       // [nb][K][NB]
  VT* ul = ml + (size_t)nb * K * NB;                          // [smax][urow] if staged
  const int64_t nblk = (int64_t)gridDim.x;
  const int64_t lb = xcd_logical_block(nblk);
  const int64_t a = lb / nchunk;
  const int chunk = (int)(lb % nchunk);
  const int nb0 = chunk * NB;
  const int nbw = min(NB, nrhs - nb0);
  const int32_t x0 = xoff[a], cnt = xoff[a + 1] - x0;
  const int64_t p0 = a << l0;
  for (int e = threadIdx.x; e < nb * K * nbw; e += blockDim.x) {
    const int n = e % nbw, bk = e / nbw;
    ml[(size_t)bk * NB + n] = mu[(p0 * K + bk) * nrhs + nb0 + n];
  }
  const FT* usrc = ubar + (int64_t)x0 * nb * K;
  if (stage_factor)
    for (int e = threadIdx.x; e < cnt * nb * K; e += blockDim.x) {
      const int x = e / (nb * K), r = e % (nb * K);
      ul[(size_t)x * urow + r] = load_factor(usrc, e);
    }
  __syncthreads();
  for (int item = threadIdx.x; item < cnt * nbw; item += blockDim.x) {
    const int x = item % cnt, n = item / cnt;
    VT acc = Zero<VT>::v();
    if (stage_factor) {
      const VT* ur = ul + (size_t)x * urow;
      for (int bk = 0; bk < nb * K; ++bk) cfma(acc, ur[bk], ml[(size_t)bk * NB + n]);
    } else {
      const FT* ur = usrc + (int64_t)x * nb * K;
      for (int bk = 0; bk < nb * K; ++bk) cfma(acc, load_factor(ur, bk), ml[(size_t)bk * NB + n]);
    }
    u[(int64_t)(nb0 + n) * ldu + perm_x[x0 + x]] = acc;
  }
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

// RHS chunk width and fusion depth.  The group state 2^k x Kmax x NB of
// vector entries stays within kLdsBudget bytes, and every thread holds at most
// two output items (2^k * NB <= 2 * kBlock).
constexpr size_t kLdsBudget = 64 * 1024;

struct Schedule {
  int NB, nchunk;
};

Schedule rhs_schedule(int nrhs) {
  Schedule s;
  s.NB = std::min(nrhs, 32);
  s.nchunk = (nrhs + s.NB - 1) / s.NB;
  return s;
}

template <typename VT, typename FT>
int apply_t(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs64,
            hipStream_t s, ibf_profile* prof) {
  const Geo& geo = p->geo;
  const int L = geo.L, l0 = geo.l0, h = geo.h;
  const int nrhs = (int)nrhs64;
  const bool swept = p->d_mdot != nullptr;
  // stored rank of level l on the V/H side (l <= h) or the G/U side (l >= h);
  // they differ only at l = h, and only after the sweep-in
  auto rank_at = [&](int l, bool gside) -> int {
    if (!swept) return p->rank[l - l0];
    if (l < h || (l == h && !gside)) return p->rank_in_h[l - l0];
    return p->rank_in_g[l - l0];
  };
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
  const Schedule sc = rhs_schedule(nrhs);
  const int NB = sc.NB, nchunk = sc.nchunk;
  int rc;
  // V
  {
    const int K = p->k_vbar;
    int NBv = NB;
    while (NBv > 1 && (size_t)p->smax_xi * NBv * sizeof(VT) > kLdsBudget / 2) NBv /= 2;
    const int nchv = (nrhs + NBv - 1) / NBv;
    const size_t base = (size_t)p->smax_xi * NBv * sizeof(VT);
    const size_t fac = (size_t)p->smax_xi * (1 << l0) * K * sizeof(VT);
    if (base > kLdsBudget) {
      set_error("ibf_apply: an Omega leaf holds too many points for the apply kernels");
      return IBF_ERR_UNSUPPORTED;
    }
    const int stage_f = base + fac <= kLdsBudget ? 1 : 0;
    const size_t lds = base + (stage_f ? fac : 0);
    if ((rc = T.begin())) return rc;
    hipLaunchKernelGGL((k_apply_v<VT, FT>), dim3((unsigned)(p->nleaf * nchv)), dim3(kBlock),
                       lds, s, (const VT*)g, ldg, p->d_perm_xi, p->d_xioff, (const FT*)p->d_vbar,
                       w[0], L, l0, K, nrhs, NBv, nchv, p->smax_xi, stage_f);
    const double nnz = (double)p->nnz_vbar;
    if ((rc = T.end("apply_v", 8.0 * nnz * nrhs,
                    nnz * fb + vb * nrhs * ((double)p->nxi + (double)p->npairs * K))))
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
  // fused butterfly stages, split at the middle when a middle block exists
  auto run_stages = [&](int lo, int hi, bool gside) -> int {   // output levels lo..hi
    int l = lo;
    while (l <= hi) {
      int kk = 1;
      while (true) {   // grow the fused group while it fits
        const int next = kk + 1;
        if (l + next - 1 > hi) break;
        if (next > kMaxR - 1) break;
        if (((int64_t)1 << next) * NB > 2 * kBlock) break;
        if (next > L - l + 1) break;                          // group must fit the b bits
        int km = 1;
        for (int j = 0; j <= next; ++j) km = std::max(km, rank_at(l - 1 + j, gside));
        if (((size_t)1 << next) * km * NB * sizeof(VT) > kLdsBudget) break;
        kk = next;
      }
      FusedArgs A{};
      A.L = L;
      A.l_start = l;
      A.nst = kk;
      A.nrhs = nrhs;
      A.NB = NB;
      A.nchunk = nchunk;
      A.ipt = (int)(((((int64_t)1 << kk) * NB) + kBlock - 1) / kBlock);
      int km = 1;
      double nnz = 0, vec = 0;
      for (int j = 0; j <= kk; ++j) {
        A.ranks[j] = rank_at(l - 1 + j, gside);
        km = std::max(km, A.ranks[j]);
      }
      for (int j = 0; j < kk; ++j) {
        const Stage& st = p->stages[l + j - l0 - 1];
        A.blk[j] = st.blk;
        nnz += (double)st.nnz;
      }
      vec = (double)p->npairs * (A.ranks[0] + A.ranks[kk]) * nrhs * vb;
      const size_t lds = ((size_t)1 << kk) * km * NB * sizeof(VT);
      const int64_t ngroups = p->npairs >> kk;
      int rc2;
      if ((rc2 = T.begin())) return rc2;
      hipLaunchKernelGGL((k_apply_fused<VT, FT>), dim3((unsigned)(ngroups * nchunk)),
                         dim3(kBlock), lds, s, w[cur], w[cur ^ 1], A);
      if ((rc2 = T.end("apply_fused", 8.0 * nnz * nrhs, nnz * fb + vec))) return rc2;
      cur ^= 1;
      l += kk;
    }
    return IBF_OK;
  };
  if (swept) {
    if ((rc = run_stages(l0 + 1, h, false))) return rc;
    if ((rc = launch_mid())) return rc;
    if ((rc = run_stages(h + 1, L - l0, true))) return rc;
  } else {
    if ((rc = run_stages(l0 + 1, L - l0, true))) return rc;
  }
  // U
  {
    const int K = p->k_ubar;
    int NBu = NB;
    while (NBu > 1 && (size_t)(1 << l0) * K * NBu * sizeof(VT) > kLdsBudget / 2) NBu /= 2;
    const int nchu = (nrhs + NBu - 1) / NBu;
    const size_t base = (size_t)(1 << l0) * K * NBu * sizeof(VT);
    const size_t fac = (size_t)p->smax_x * ((1 << l0) * K + 1) * sizeof(VT);
    if (base > kLdsBudget) {
      set_error("ibf_apply: leaf size too large for the apply kernels");
      return IBF_ERR_UNSUPPORTED;
    }
    const int stage_f = base + fac <= kLdsBudget ? 1 : 0;
    const size_t lds = base + (stage_f ? fac : 0);
    if ((rc = T.begin())) return rc;
    hipLaunchKernelGGL((k_apply_u<VT, FT>), dim3((unsigned)(p->nleaf * nchu)), dim3(kBlock),
                       lds, s, w[cur], (VT*)u, ldu, p->d_perm_x, p->d_xoff, (const FT*)p->d_ubar,
                       l0, K, nrhs, NBu, nchu, p->smax_x, stage_f);
    const double nnz = (double)p->nnz_ubar;
    if ((rc = T.end("apply_u", 8.0 * nnz * nrhs,
                    nnz * fb + vb * nrhs * ((double)p->nx + (double)p->npairs * K))))
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
