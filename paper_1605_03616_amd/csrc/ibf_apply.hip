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
// right-hand sides) in LDS across the k stages, and stages each level's
// factor blocks for the group through LDS with coalesced loads.
//
// Kernels:
//   k_apply_v      Omega leaf -> 2^l0 pairs:  mu = Vbar^* g   (per-leaf product, LDS-staged)
//   k_apply_fused  k butterfly stages on one pair group in LDS (few right-hand
//                  sides, vector FMA)
//   k_apply_fused_mfma  the same for 32-column chunks in FP32 on MFMA
//                  (v_mfma_f32_4x4x1f32, 16 blocks = 2 slots x 8 groups of 4
//                  right-hand sides), persistent over the groups with the next
//                  groups' loads in flight during the current last stage
//   k_apply_mid    swept-in middle block Mdot (per pair)
//   k_apply_u      2^l0 pairs -> X leaf:  u = Ubar mu        (per-leaf product, LDS-staged)
#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "ibf_device.h"

namespace ibf {
namespace {

constexpr int kBlock = 256;
constexpr int kNumXcd = 8;             // MI355X: 8 XCDs, each with its own L2
constexpr size_t kLdsBudget = 64 * 1024;
constexpr size_t kLdsBudgetMfma = 80 * 1024;

typedef float v4f __attribute__((ext_vector_type(4)));

template <typename VT> struct Zero;
template <> struct Zero<double2> { __device__ static double2 v() { return make_double2(0, 0); } };
template <> struct Zero<float2> { __device__ static float2 v() { return make_float2(0, 0); } };

// Cooperative global -> LDS copy with UNR independent loads in flight per
// thread (a plain loop would wait on every load before its LDS store).
template <int UNR, typename T, typename LoadF, typename StoreF>
__device__ __forceinline__ void staged_copy(int total, LoadF load, StoreF store) {
  for (int e0 = threadIdx.x; e0 < total; e0 += UNR * kBlock) {
    T tmp[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int e = e0 + u * kBlock;
      if (e < total) tmp[u] = load(e);
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int e = e0 + u * kBlock;
      if (e < total) store(e, tmp[u]);
    }
  }
}

// Batched copy into an LDS array: map(e, off) loads element e and sets its
// destination offset; UNR loads are issued before any LDS store.
template <int UNR, typename T, typename MapF>
__device__ __forceinline__ void staged_copy_to(int total, T* base, MapF map) {
  for (int e0 = threadIdx.x; e0 < total; e0 += UNR * kBlock) {
    T tmp[UNR];
    int off[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int e = e0 + u * kBlock;
      off[u] = -1;
      if (e < total) tmp[u] = map(e, off[u]);
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      if (off[u] >= 0) base[off[u]] = tmp[u];
  }
}

// q / d and q % d for 0 <= q < 2^22 and 1 <= d <= 2^10 through a float
// reciprocal: (q + 1/2)/d sits at least 1/(2d) away from an integer, far
// beyond float rounding, so the truncation is exact.
struct FastDiv {
  int d;
  float inv;
  __device__ __forceinline__ explicit FastDiv(int dd) : d(dd), inv(1.0f / (float)dd) {}
  __device__ __forceinline__ int div(int q) const { return (int)(((float)q + 0.5f) * inv); }
  __device__ __forceinline__ void divmod(int q, int& qq, int& rr) const {
    qq = div(q);
    rr = q - qq * d;
  }
};

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
// LDS: g_leaf[smax][NB], and when it fits vbar_leaf[smax][2^l0][KT] (zero-padded).
// ---------------------------------------------------------------------------
struct VDesc {
  const void* g;
  int64_t ldg;
  const int32_t* perm_xi;
  const int32_t* xioff;
  const void* vbar;
  void* mu;
  int L, l0, K, nrhs, NB, nchunk, smax, stage_f;
  const uint8_t* prk;   // MFMA V: per-pair ranks at level l0; rows past a pair's
                        // rank are not written (null: every row is written)
};

template <typename VT, typename FT, int KT>
__device__ __forceinline__ void apply_v_body(const VDesc& d, int64_t lb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const VT* __restrict__ g = reinterpret_cast<const VT*>(d.g);
  const FT* __restrict__ vbar = reinterpret_cast<const FT*>(d.vbar);
  VT* __restrict__ mu = reinterpret_cast<VT*>(d.mu);
  const int32_t* __restrict__ perm_xi = d.perm_xi;
  const int32_t* __restrict__ xioff = d.xioff;
  const int64_t ldg = d.ldg;
  const int L = d.L, l0 = d.l0, K = d.K, nrhs = d.nrhs, NB = d.NB, nchunk = d.nchunk;
  const int smax = d.smax, stage_factor = d.stage_f;
  VT* gl = reinterpret_cast<VT*>(smem);                       // [smax][NB]
  VT* vl = gl + (size_t)smax * NB;                            // [smax][2^l0][KT]
  const int64_t b = lb / nchunk;
  const int chunk = (int)(lb % nchunk);
  const int nb0 = chunk * NB;
  const int nbw = min(NB, nrhs - nb0);
  const int32_t j0 = xioff[b], cnt = xioff[b + 1] - j0;
  const int na = 1 << l0;
  // gather g for the leaf (points fastest: contiguous within a column)
  if (cnt > 0) {
    // points fastest: contiguous within a column of g
    const FastDiv divC(cnt);
    staged_copy_to<8>(cnt * nbw, gl, [&](int e, int& off) {
      int n, j;
      divC.divmod(e, n, j);
      off = j * NB + n;
      return g[(int64_t)(nb0 + n) * ldg + perm_xi[j0 + j]];
    });
  }
  const FT* vsrc = vbar + (int64_t)j0 * na * K;
  if (stage_factor)
    staged_copy_to<8>(cnt * na * KT, vl, [&](int e, int& off) {
      const int ja = e / KT, k = e % KT;                      // KT is a compile-time constant
      off = e;
      return k < K ? load_factor(vsrc, (int64_t)ja * K + k) : Zero<VT>::v();
    });
  __syncthreads();
  const int sh = L - l0;
  for (int item = threadIdx.x; item < na * nbw; item += blockDim.x) {
    const int n = item % nbw, a = item / nbw;
    VT acc[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) acc[k] = Zero<VT>::v();
    for (int j = 0; j < cnt; ++j) {
      const VT gv = gl[j * NB + n];
      if (stage_factor) {
        const VT* vr = vl + ((size_t)j * na + a) * KT;
#pragma unroll
        for (int k = 0; k < KT; ++k) cfma(acc[k], vr[k], gv);
      } else {
        const int64_t off = ((int64_t)j * na + a) * K;
#pragma unroll
        for (int k = 0; k < KT; ++k) cfma(acc[k], load_factor(vsrc, off + min(k, K - 1)), gv);
      }
    }
    const int64_t p = ((int64_t)a << sh) | b;
    VT* o = mu + p * K * nrhs + nb0 + n;
#pragma unroll
    for (int k = 0; k < KT; ++k)
      if (k < K) o[(int64_t)k * nrhs] = acc[k];
  }
}

// Batched launches: problem p owns logical blocks [boff[p], boff[p+1]).
__device__ __forceinline__ int find_problem(const int64_t* __restrict__ boff, int count,
                                            int64_t b) {
  int lo = 0, hi = count - 1;                                 // largest p with boff[p] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (boff[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename VT, typename FT, int KT>
__global__ __launch_bounds__(kBlock) void k_apply_v(VDesc d) {
  apply_v_body<VT, FT, KT>(d, xcd_logical_block((int64_t)gridDim.x));
}
template <typename VT, typename FT, int KT>
__global__ __launch_bounds__(kBlock) void k_batch_v(const VDesc* __restrict__ ds,
                                                    const int64_t* __restrict__ boff, int count) {
  const int p = find_problem(boff, count, blockIdx.x);
  apply_v_body<VT, FT, KT>(ds[p], (int64_t)blockIdx.x - boff[p]);
}

// ---------------------------------------------------------------------------
// Fused butterfly stages l_start .. l_start+nst-1 on one group of 2^nst
// contiguous input pairs (level l_start-1) and one RHS chunk.  In LDS the
// group's pair at level l_start-1+j has local index (alpha bits << (nst-j)) |
// (remaining child bits); a stage consumes the lowest child bit and appends
// an alpha bit.  Outputs of a stage are held in registers across a barrier
// and written back in place; those of the last stage go straight to HBM.
// ranks[j] = stored K at level l_start-1+j; kld[j] = row length of stage j's
// stored blocks (each pair's block is 2 ranks[j] rows of kld[j] entries,
// contiguous in HBM and copied unchanged into LDS).
// ---------------------------------------------------------------------------
struct FusedArgs {
  int L, l_start, nst, nrhs, NB, nchunk, kmaxg;
  int ranks[kMaxR + 1];
  int kld[kMaxR];
  const void* blk[kMaxR];
  // MFMA launches only: the swept-in middle block Mdot [pair][kmid_out][kmid_in]
  // applied to each input pair before the first stage (null: none), in which
  // case the inputs hold kmid_in rows and ranks[0] == kmid_out
  const void* mid;
  int kmid_in, kmid_out;
};

// global output pair of local output slot `locp` after stage j (rem child bits left)
__device__ __forceinline__ int64_t fused_pout(int locp, int j, int rem, int64_t ap, int64_t bpp,
                                              int L, int l) {
  const int anew = locp >> rem;
  const int q = locp & ((1 << rem) - 1);
  const int64_t a_l = (ap << (j + 1)) | anew;
  const int64_t b_l = (bpp << rem) | q;
  return (a_l << (L - l)) | b_l;
}
// local slot of the first of the two inputs of output slot `locp`
__device__ __forceinline__ int fused_in0(int locp, int rem) {
  const int anew = locp >> rem;
  const int q = locp & ((1 << rem) - 1);
  return ((anew >> 1) << (rem + 1)) | (2 * q);
}

struct FusedDesc {
  const void* in;
  void* out;
  FusedArgs A;
};

// Few right-hand sides (vector path): the stage is a stream of factor blocks,
// each entry used by NB columns only.  One thread per output (slot, row t,
// column n), n fastest; it reads its factor row entries straight from HBM (the
// threads of one slot read whole rows together, and consecutive rows share
// cache lines) and the inputs from the LDS state, which ping-pongs between two
// buffers so that no output waits in registers.
template <typename VT, typename FT, int KT>
__device__ __forceinline__ void apply_fused_body(const FusedDesc& D, int64_t lb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const VT* __restrict__ in = reinterpret_cast<const VT*>(D.in);
  VT* __restrict__ out = reinterpret_cast<VT*>(D.out);
  const FusedArgs& A = D.A;
  const int k = A.nst, NB = A.NB, L = A.L, kmaxg = A.kmaxg;
  const int nslot = 1 << k;
  VT* S = reinterpret_cast<VT*>(smem);                        // [nslot][kmaxg][NB]
  VT* S1 = S + (size_t)nslot * kmaxg * NB;                    // second state buffer
  const int64_t gid = lb / A.nchunk;
  const int chunk = (int)(lb % A.nchunk);
  const int nb0 = chunk * NB;
  const int nbw = min(NB, A.nrhs - nb0);
  const int nrhs = A.nrhs;
  const int sh_end = L - (A.l_start + k - 1);
  const int64_t ap = gid >> sh_end;
  const int64_t bpp = gid & (((int64_t)1 << sh_end) - 1);
  // thread -> (column n, first row w) of the [row][NB] tiles it moves
  const int rstep = kBlock / NB;
  const int n = threadIdx.x % NB, w = threadIdx.x / NB;

  // load the group: slot c <- input pair (gid << k) | c; columns >= nbw are zero
  {
    const int kin = A.ranks[0];
    const VT* src = in + (gid << k) * kin * nrhs + nb0 + n;
    const int rows = nslot * kin;
    if (w < rstep) {
      int slot = 0, s = w;
      while (s >= kin) { s -= kin; ++slot; }
      for (int r0 = w; r0 < rows; r0 += 4 * rstep) {
        VT tmp[4];
        int off[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = r0 + u * rstep;
          off[u] = -1;
          if (r < rows) {
            tmp[u] = n < nbw ? src[(int64_t)r * nrhs] : Zero<VT>::v();
            off[u] = (slot * kmaxg + s) * NB + n;
          }
          s += rstep;
          while (s >= kin) { s -= kin; ++slot; }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (off[u] >= 0) S[off[u]] = tmp[u];
      }
    }
  }
  const FastDiv divNB(NB);
  __syncthreads();                                            // the gathered group is in S
  for (int j = 0; j < k; ++j) {
    const int l = A.l_start + j;
    const int kin = A.ranks[j], kout = A.ranks[j + 1], ke = A.kld[j];
    const int fs = 2 * kin * ke;
    const int rem = k - j - 1;
    const FT* __restrict__ blk = reinterpret_cast<const FT*>(A.blk[j]);
    const VT* Sin = (j & 1) ? S1 : S;
    VT* Sout = (j & 1) ? S : S1;
    const bool last = j == k - 1;
    const int items = nslot * kout * NB;
    const FastDiv divK(kout);
    for (int item = threadIdx.x; item < items; item += kBlock) {
      int r, nn, locp, t;
      divNB.divmod(item, r, nn);
      divK.divmod(r, locp, t);
      const int64_t pout = fused_pout(locp, j, rem, ap, bpp, L, l);
      const FT* f = blk + pout * fs + t;
      const VT* x = Sin + (size_t)fused_in0(locp, rem) * kmaxg * NB + nn;
      VT acc = Zero<VT>::v();
      for (int c = 0; c < 2; ++c) {
        const FT* fc = f + c * kin * ke;
        const VT* xc = x + (size_t)c * kmaxg * NB;
#pragma unroll 4
        for (int s2 = 0; s2 < kin; ++s2) cfma(acc, load_factor(fc, s2 * ke), xc[s2 * NB]);
      }
      if (!last) Sout[(size_t)(locp * kmaxg + t) * NB + nn] = acc;
      else if (nn < nbw) out[(pout * kout + t) * nrhs + nb0 + nn] = acc;
    }
    if (!last) __syncthreads();
  }
}

// LDS stride of a slot's staged factor block of fs entries: a multiple of 16
// entries plus 4, so that the A-operand reads of the slots that share a wave
// start 8 banks apart instead of on the same bank.
__device__ __forceinline__ int slot_stride(int fs) { return ((fs + 15) & ~15) + 4; }

// Factor blocks of one stage for the NV virtual slots of an MFMA block (NV /
// 2^k consecutive groups of 2^k slots): TPS = kBlock / NV threads per slot,
// thread t stages entries (t mod TPS) + TPS i of slot t / TPS, so each thread
// computes one block address per stage and loads move contiguous runs.  NL
// loads per thread cover blocks of up to 2 KT^2 entries (the launch's ranks
// are at most KT).
template <typename VT, typename FT, int KT, int NV>
struct SlotFactors {
  static constexpr int TPS = kBlock / NV;
  static constexpr int NL = (2 * KT * KT + TPS - 1) / TPS;
  VT v[NL];
  __device__ static __forceinline__ int slot() { return threadIdx.x / TPS; }
  // HBM block of stage j's factors for this thread's slot
  __device__ static __forceinline__ const FT* stage_block(const FT* blk, int fs, int k, int j,
                                                          int rem, int64_t gid0, int sh_end, int L,
                                                          int l) {
    const int u = slot();
    const int64_t g = gid0 + (u >> k);
    const int64_t ap = g >> sh_end, bpp = g & (((int64_t)1 << sh_end) - 1);
    return blk + fused_pout(u & ((1 << k) - 1), j, rem, ap, bpp, L, l) * fs;
  }
  // Every round loads (entries past the block re-read its last entry), so
  // loads and stores are straight-line code and the compiler can wait for
  // exactly the loads a store needs.
  __device__ __forceinline__ void load(const FT* src, int fs) {
    const int e = threadIdx.x % TPS;
#pragma unroll
    for (int i = 0; i < NL; ++i) v[i] = load_factor(src, min(e + TPS * i, fs - 1));
  }
  // Entries to F[slot] at slot_stride(fs); rounds past the block rewrite its
  // last entry with the same value.
  __device__ __forceinline__ void store(VT* F, int fs) const {
    const int u = slot(), e = threadIdx.x % TPS;
    VT* dst = F + u * slot_stride(fs);
#pragma unroll
    for (int i = 0; i < NL; ++i) dst[min(e + TPS * i, fs - 1)] = v[i];
  }
  // The fs entries form a [t][s] matrix of tk columns; store it transposed as
  // [s][tld] at slot_stride(tk tld).
  __device__ __forceinline__ void store_t(VT* F, int fs, int tk, int tld) const {
    const int u = slot(), e = threadIdx.x % TPS;
    VT* dst = F + u * slot_stride(tk * tld);
    const float inv = 1.0f / (float)tk;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int o = min(e + TPS * i, fs - 1);
      const int t = (int)(((float)o + 0.5f) * inv);           // o / tk (exact, o < 2^22)
      dst[(o - t * tk) * tld + t] = v[i];
    }
  }
};

// Multi-RHS FP32 variant on MFMA for RHS chunks of NBC = 32 or 16 columns.
// Each wave computes SPW = 64 / NBC virtual slots at once, and a block holds
// NV = 4 SPW of them (8 or 16): one group of NV pairs (log2 NV stages), or
// NV / 2^k consecutive groups of 2^k pairs side by side, for one RHS chunk.
// It is persistent: the block with logical index b takes logical blocks b,
// b + lstep, ... below lend (logical block = NV consecutive input pairs x
// chunk; the chunks of the same pairs are adjacent and so share the factor
// blocks through one XCD's L2).  While the last stage computes, the loads of
// the next block's input rows and first-stage factors are already in flight
// into registers, and each stage's computation overlaps the loads of the next
// stage's factors.
//
// Lane l of wave w belongs to virtual slot SPW w + l / NBC and carries RHS
// column l mod NBC.  The 16 MFMA blocks of v_mfma_f32_4x4x1f32 are groups of
// 4 columns, NBC / 4 per slot; A-operand row i = l & 3 is the raw float i of
// the slot's pair of complex factor entries (t = 2g, 2g+1): (re t0, im t0,
// re t1, im t1).  With P = sum f_i x_re and Q = sum f_i x_im, the complex
// outputs are
//   out[2g]   = (P0 - Q1, P1 + Q0),  out[2g+1] = (P2 - Q3, P3 + Q2).
template <typename VT, typename FT, int KT, int NBC, bool MID>
__device__ __forceinline__ void fused_mfma_body(const FusedDesc& D, int64_t lb, int64_t lstep,
                                                int64_t lend) {
  static_assert(sizeof(VT) == 8, "MFMA variant computes in FP32");
  static_assert(NBC == 32 || NBC == 16, "RHS chunks of 32 or 16 columns");
  constexpr int KG = KT / 2;                                  // row pairs (MFMA row groups)
  constexpr int NB = NBC;                                     // RHS columns per chunk
  constexpr int SPW = 64 / NBC;                               // slots per wave
  constexpr int NV = 4 * SPW;                                 // virtual slots per block
  constexpr int LNV = NV == 8 ? 3 : 4;
  // input rows held in flight per thread (row r goes to thread row r mod NV);
  // blocks with more input rows than NV XR copy the rest synchronously
  constexpr int XR = KT;
  extern __shared__ __align__(16) unsigned char smem[];
  const VT* __restrict__ in = reinterpret_cast<const VT*>(D.in);
  VT* __restrict__ out = reinterpret_cast<VT*>(D.out);
  const FusedArgs& A = D.A;
  const int k = A.nst, L = A.L, kmaxg = A.kmaxg, nrhs = A.nrhs, nchunk = A.nchunk;
  const int nslot = 1 << k;
  // S: the state of stage j as [virtual slot][ranks[j]][NB] (the 2 kin input
  // rows of an output slot are contiguous); F: the stage's factor blocks
  // [virtual slot][2 kin kld] at slot_stride, followed by 2 KT entries of
  // slack for reads past the last row
  VT* S = reinterpret_cast<VT*>(smem);
  VT* F = S + (size_t)NV * kmaxg * NB;
  const int sh_end = L - (A.l_start + k - 1);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = lane % NB, fi = lane & 3;
  const int vs = SPW * wave + lane / NB;                      // this lane's virtual slot
  const int grp = vs >> k, loc = vs & (nslot - 1);            // its group and local slot
  const int trow = threadIdx.x / NB;                          // row phase of the copies
  // A block's first factors: the swept-in middle block Mdot when the launch
  // applies it (staged transposed, [s][kldm]), else stage 0's blocks.  The
  // choice is a select, not a branch, so the staging stays straight-line.
  using SF = SlotFactors<VT, FT, KT, NV>;
  const FT* blk0 = reinterpret_cast<const FT*>(A.blk[0]);
  const FT* mdot = reinterpret_cast<const FT*>(A.mid);
  constexpr bool has_mid = MID;                               // A.mid set by the host
  const int kin0 = has_mid ? A.kmid_in : A.ranks[0];          // input rows per pair
  const int rows0 = NV * kin0;
  const int kmo = A.kmid_out, kldm = (A.kmid_out + 1) & ~1;
  const int fs0 = 2 * A.ranks[0] * A.kld[0];                  // a stage-0 block
  const int fsm = kmo * kin0, fsml = kin0 * kldm;             // an Mdot block: HBM, LDS
  const int fsf = has_mid ? fsm : fs0;
  auto first_src = [&](int64_t gid0) {
    if constexpr (MID) return mdot + ((gid0 << k) + SF::slot()) * (int64_t)fsm;
    else return SF::stage_block(blk0, fs0, k, 0, k - 1, gid0, sh_end, L, A.l_start);
  };

  struct Blk {
    int64_t gid0;                                             // first group
    int nb0, nbw;
  };
  auto decode = [&](int64_t l) {
    Blk g;
    const int64_t q = l / nchunk;
    g.gid0 = q << (LNV - k);
    g.nb0 = (int)(l - q * nchunk) * NB;
    g.nbw = min(NB, nrhs - g.nb0);
    return g;
  };
  SF fb;
  VT xin[XR];
  // The block's input rows are contiguous in HBM (pairs (gid0 << k) .. + NV,
  // kin0 rows each) and land contiguously in S; columns >= nbw read as zero.
  // The per-row offsets and bounds depend only on launch constants; passed
  // through an empty asm they are recomputed at each call instead of being
  // hoisted out of the block loop, where dozens of them would stay live in
  // registers across every stage.
  auto fetch = [&](const Blk& g) {
    int kin_v = kin0, fs_v = fsf, trow_v = trow;
    int64_t ld_v = nrhs;
    asm volatile("" : "+s"(kin_v), "+s"(fs_v), "+v"(trow_v), "+s"(ld_v));
    fb.load(first_src(g.gid0), fs_v);
    // straight-line loads (rows i >= kin0 re-read row kin0 - 1, columns past
    // the chunk re-read column 0 and are zeroed after the load)
    const bool ok = col < g.nbw;
    const VT* src = in + ((g.gid0 << k) * kin0 + trow_v) * ld_v + g.nb0 + (ok ? col : 0);
#pragma unroll
    for (int i = 0; i < XR; ++i) {
      const VT v = src[NV * min(i, kin_v - 1) * ld_v];
      xin[i] = ok ? v : Zero<VT>::v();
    }
  };
  auto deposit = [&](const Blk& g) {
    int kin_v = kin0, rows_v = rows0, fs_v = fsf, trow_v = trow;
    asm volatile("" : "+s"(kin_v), "+s"(rows_v), "+s"(fs_v), "+v"(trow_v));
    VT* dst = S + trow_v * NB + col;
    // rows i >= kin0 hold row kin0 - 1 again and rewrite it (straight-line)
#pragma unroll
    for (int i = 0; i < XR; ++i) dst[NV * min(i, kin_v - 1) * NB] = xin[i];
    if (rows_v > NV * XR) {
      const VT* src = in + (g.gid0 << k) * kin0 * nrhs + g.nb0 + col;
      for (int r = NV * XR + trow_v; r < rows_v; r += NV)
        S[r * NB + col] = col < g.nbw ? src[(int64_t)r * nrhs] : Zero<VT>::v();
    }
    if constexpr (MID) fb.store_t(F, fs_v, kin0, kldm);
    else fb.store(F, fs_v);
  };
  // P, Q += F-block rows times the nrows state rows from xp (the lane's
  // column); the factor rows start at fp (the lane's float fi), fstep floats
  // apart.  Software-pipelined: the LDS reads of the next row are in flight
  // while the MFMAs of the current row issue; for even nrows the last
  // iteration reads one row past the end, inside the LDS allocation and never
  // used.  (Starting the first row's MFMAs from an inline zero instead of
  // clearing the accumulators costs more registers than it saves.)
  // Only the first NG = ceil(kout / 2) row pairs are computed: the caller
  // picks NG = KG or KG - 1 for the stage (see run_product).
  auto product = [&](auto ng_c, const VT* xp, const float* fp, int fstep, int nrows,
                     v4f (&P)[KG], v4f (&Q)[KG]) {
    constexpr int NG = decltype(ng_c)::value;
    auto load_row = [&](const VT* x, const float* f, float (&Av)[KG], VT& X) {
      X = *x;
#pragma unroll
      for (int gq = 0; gq < NG; ++gq) Av[gq] = f[4 * gq];
    };
    auto mfma_row = [&](const float (&Av)[KG], const VT& X) {
#pragma unroll
      for (int gq = 0; gq < NG; ++gq) {
        P[gq] = __builtin_amdgcn_mfma_f32_4x4x1f32(Av[gq], X.x, P[gq], 0, 0, 0);
        Q[gq] = __builtin_amdgcn_mfma_f32_4x4x1f32(Av[gq], X.y, Q[gq], 0, 0, 0);
      }
    };
#pragma unroll
    for (int gq = 0; gq < NG; ++gq) {
      P[gq] = v4f{0.f, 0.f, 0.f, 0.f};
      Q[gq] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    float av[KG], bv[KG];
    VT xa, xb;
    load_row(xp, fp, av, xa);
    int left = nrows;
#pragma unroll 1
    for (; left >= 2; left -= 2) {
      load_row(xp + NB, fp + fstep, bv, xb);
      __builtin_amdgcn_sched_barrier(0);                      // keep the reads ahead
      mfma_row(av, xa);
      __builtin_amdgcn_sched_barrier(0);
      xp += 2 * NB;
      fp += 2 * fstep;
      load_row(xp, fp, av, xa);
      __builtin_amdgcn_sched_barrier(0);
      mfma_row(bv, xb);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (left) mfma_row(av, xa);                               // odd nrows: the last row
  };
  // stages whose output rank fits KT - 2 rows skip the last row pair: the
  // launch's KT covers its largest rank, the other stages' ranks are often
  // smaller (one uniform branch a stage)
  auto run_product = [&](int kout, const VT* xp, const float* fp, int fstep, int nrows,
                         v4f (&P)[KG], v4f (&Q)[KG]) {
    if constexpr (KG > 1) {
      if (kout <= KT - 2) {
        product(std::integral_constant<int, KG - 1>{}, xp, fp, fstep, nrows, P, Q);
        return;
      }
    }
    product(std::integral_constant<int, KG>{}, xp, fp, fstep, nrows, P, Q);
  };
  // the kout output rows of P, Q (this lane's slot and column) to S
  auto put_rows = [&](const v4f (&P)[KG], const v4f (&Q)[KG], int kout) {
    VT* dst = S + (size_t)vs * kout * NB + col;
#pragma unroll
    for (int gq = 0; gq < KG; ++gq) {
      if (2 * gq < kout) {
        const v4f p = P[gq], q = Q[gq];
        dst[(2 * gq) * NB] = make_float2(p[0] - q[1], p[1] + q[0]);
        if (2 * gq + 1 < kout) dst[(2 * gq + 1) * NB] = make_float2(p[2] - q[3], p[3] + q[2]);
      }
    }
  };

  Blk cur = decode(lb);
  fetch(cur);
  while (true) {
    deposit(cur);
    __syncthreads();
    const int64_t nlb = lb + lstep;
    const bool more = nlb < lend;
    const Blk nxt = more ? decode(nlb) : cur;
    const int64_t gme = cur.gid0 + grp;                       // this lane's group
    const int64_t ap = gme >> sh_end, bpp = gme & (((int64_t)1 << sh_end) - 1);
    if constexpr (MID) {
      // the middle block on each input pair (the lane's own slot), with
      // stage 0's factors in flight
      // fs0 laundered: its clamped offsets are not hoisted out of the
      // persistent loop (they would stay live in VGPRs across every stage)
      int fs0_v = fs0;
      asm volatile("" : "+s"(fs0_v));
      fb.load(SF::stage_block(blk0, fs0_v, k, 0, k - 1, cur.gid0, sh_end, L, A.l_start), fs0_v);
      v4f P[KG], Q[KG];
      run_product(kmo, S + (size_t)vs * kin0 * NB + col,
                  reinterpret_cast<const float*>(F + (size_t)vs * slot_stride(fsml)) + fi,
                  2 * kldm, kin0, P, Q);
      __syncthreads();                                        // S and F reads done
      put_rows(P, Q, kmo);
      asm volatile("" : "+s"(fs0_v));
      fb.store(F, fs0_v);
      __syncthreads();
    }
    // one stage; the last one is peeled off the stage loop so that the next
    // block's prefetched rows are live only during it
    auto stage = [&](int j, auto last_c) {
      constexpr bool LAST = decltype(last_c)::value;
      const int l = A.l_start + j;
      const int kin = A.ranks[j], kout = A.ranks[j + 1], ke = A.kld[j];
      const int fs = 2 * kin * ke;
      const int rem = k - j - 1;
      if constexpr (!LAST) {  // next stage's factor blocks: in flight during this stage
        const int fsn = 2 * kout * A.kld[j + 1];
        fb.load(SF::stage_block(reinterpret_cast<const FT*>(A.blk[j + 1]), fsn, k, j + 1, rem - 1,
                                cur.gid0, sh_end, L, l + 1),
                fsn);
      } else if (more) {      // the next block: in flight during the last stage
        fetch(nxt);
      }
      // the block product of this lane's slot over the 2 kin input rows of
      // its two children (adjacent slots, so contiguous rows in S)
      v4f P[KG], Q[KG];
      run_product(kout, S + (size_t)((grp << k) + fused_in0(loc, rem)) * kin * NB + col,
                  reinterpret_cast<const float*>(F + (size_t)vs * slot_stride(fs)) + fi, 2 * ke,
                  2 * kin, P, Q);
      if constexpr (!LAST) {
        // outputs replace inputs in S once every wave has read its inputs
        __syncthreads();
        put_rows(P, Q, kout);
        fb.store(F, 2 * kout * A.kld[j + 1]);
        __syncthreads();
      } else if (col < cur.nbw) {
        // last stage: rows of NB columns straight to HBM
        VT* dst = out + fused_pout(loc, j, 0, ap, bpp, L, l) * kout * nrhs + cur.nb0 + col;
#pragma unroll
        for (int gq = 0; gq < KG; ++gq) {
          if (2 * gq < kout) {
            const v4f p = P[gq], q = Q[gq];
            dst[(int64_t)(2 * gq) * nrhs] = make_float2(p[0] - q[1], p[1] + q[0]);
            if (2 * gq + 1 < kout)
              dst[(int64_t)(2 * gq + 1) * nrhs] = make_float2(p[2] - q[3], p[3] + q[2]);
          }
        }
      }
    };
    for (int j = 0; j + 1 < k; ++j) stage(j, std::false_type{});
    stage(k - 1, std::true_type{});
    if (!more) break;
    __syncthreads();                                          // last-stage LDS reads done
    lb = nlb;
    cur = nxt;
  }
}

template <typename VT, typename FT, int KT>
__global__ __launch_bounds__(kBlock) void k_apply_fused(FusedDesc D) {
  apply_fused_body<VT, FT, KT>(D, xcd_logical_block((int64_t)gridDim.x));
}
template <typename VT, typename FT, int KT>
__global__ __launch_bounds__(kBlock) void k_batch_fused(const FusedDesc* __restrict__ ds,
                                                        const int64_t* __restrict__ boff,
                                                        int count) {
  const int p = find_problem(boff, count, blockIdx.x);
  apply_fused_body<VT, FT, KT>(ds[p], (int64_t)blockIdx.x - boff[p]);
}
// persistent: a grid of resident blocks over `total` logical blocks
template <typename VT, typename FT, int KT, int NBC, bool MID>
__global__ __launch_bounds__(kBlock) void k_apply_fused_mfma(FusedDesc D, int64_t total) {
  fused_mfma_body<VT, FT, KT, NBC, MID>(D, xcd_logical_block((int64_t)gridDim.x),
                                        (int64_t)gridDim.x, total);
}
// (batched phases: one logical block per block; a member's launch carries the
// middle block when its descriptor has one)
template <typename VT, typename FT, int KT, int NBC>
__global__ __launch_bounds__(kBlock) void k_batch_fused_mfma(const FusedDesc* __restrict__ ds,
                                                             const int64_t* __restrict__ boff,
                                                             int count) {
  const int p = find_problem(boff, count, blockIdx.x);
  const int64_t lb = (int64_t)blockIdx.x - boff[p];
  if (ds[p].A.mid) fused_mfma_body<VT, FT, KT, NBC, true>(ds[p], lb, 1, lb + 1);
  else fused_mfma_body<VT, FT, KT, NBC, false>(ds[p], lb, 1, lb + 1);
}

// ---------------------------------------------------------------------------
// Butterfly stages on MFMA at each pair's own ranks (FP32 state, RHS chunks
// of 64 columns).  A level's blocks are stored at the level's largest rank
// with exact zero padding (rows past an input pair's rank, columns past the
// output pair's rank); at the 1-D FIO workloads the padding is about 40 % of
// the stored entries.  Here each wave owns one output pair of a stage and
// runs its product over exactly the two input pairs' ranks and the output
// pair's rank: the padding is neither read nor multiplied.
//
// A block of 64 * 2^k threads owns one group of 2^k contiguous input pairs
// (one RHS chunk) and carries it through k stages, one wave per slot, lane =
// RHS column; the group's state [slot][row][64] lives in LDS.  The kernel is
// persistent over groups: the next group's input rows and first factor rows
// are loaded into registers during the current group's last stage, and each
// stage's factor rows during the previous stage.
//
// Factor operands come straight from memory, two rows per coalesced 32-bit
// load (lanes 0-31 row s, lanes 32-63 row s + 1, float e of the row in lane
// e), and each v_mfma_f32_4x4x1f32 broadcasts the four floats of one (row,
// row pair g) to all 16 blocks (cbsz 4, abid 8 rsel + g): one register feeds
// the 2 x 8 (row, g) products of a window.  Per-pair ranks come from byte
// arrays kept by the build (prk[j][pair] at level l_start - 1 + j).
// ---------------------------------------------------------------------------
struct TightArgs {
  int L, l_start, nst, nrhs, nchunk;
  int KS;                            // rows per LDS slot: largest stored rank of the levels
  int rank_out;                      // 1: the output rows past a pair's rank are not written
                                     // (every reader of them skips them)
  int kst[kMaxR + 1];                // stored rank at level l_start - 1 + j (HBM row stride)
  int kld[kMaxR];                    // stored row length of stage j's blocks
  const void* blk[kMaxR];
  const void* qblk[kMaxR];           // split products: stage j's quad records
  const uint8_t* prk[kMaxR + 1];     // per-pair ranks at level l_start - 1 + j
};
struct TightDesc {
  const void* in;
  void* out;
  TightArgs A;
};

// Float fu + fl of a stored block, fu uniform across the wave (a scalar
// base) and fl the lane's offset (FP32 as stored; BF16X2 widened hi + lo;
// fu even, so the complex entry of fl alone picks the component)
// (the lane offset enters as a 32-bit byte offset, so the load takes the
// scalar-base + 32-bit-offset form: one VGPR per load in flight)
__device__ __forceinline__ float block_float(const float2* blk, int64_t fu, unsigned fl) {
  const char* b = reinterpret_cast<const char*>(reinterpret_cast<const float*>(blk) + fu);
  return *reinterpret_cast<const float*>(b + (fl * 4u));
}
__device__ __forceinline__ float block_float(const bf16x2c* blk, int64_t fu, unsigned fl) {
  const char* b = reinterpret_cast<const char*>(reinterpret_cast<const unsigned short*>(blk) + 2 * fu);
  const unsigned o = (4u * (fl >> 1) + (fl & 1u)) * 2u;
  return bf2f(*reinterpret_cast<const unsigned short*>(b + o)) +
         bf2f(*reinterpret_cast<const unsigned short*>(b + o + 4u));
}

// P[g], Q[g] += (row rsel of the window, row pair g) x (x_re, x_im) for g < NG:
// abid 8 rsel + g selects the four floats (re t0, im t0, re t1, im t1) of
// entries t = 2g, 2g + 1 held by lanes 32 rsel + 4g .. + 3.
template <int RS, int NG, int KG, int G = 0>
__device__ __forceinline__ void tight_row(float a, float2 x, v4f (&P)[KG], v4f (&Q)[KG]) {
  if constexpr (G < NG) {
    P[G] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, x.x, P[G], 4, 8 * RS + G, 0);
    Q[G] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, x.y, Q[G], 4, 8 * RS + G, 0);
    tight_row<RS, NG, KG, G + 1>(a, x, P, Q);
  }
}

// ---------------------------------------------------------------------------
// BF16 split products (BF16X2 plans).  A stored factor entry is bf16 hi + lo
// (the FP64 value rounded to bf16, then the rest rounded to bf16); the FP32
// state is split the same way when it is written to LDS.  One
// v_mfma_f32_4x4x4_16b_bf16 multiplies four state rows at once (the K index
// of the instruction runs over the rows), and a product is the three terms
// hi.hi + hi.lo + lo.hi accumulated in FP32 (the dropped lo.lo term is
// below 2^-16 of the product).  A block of 4 rows x 4 floats of the factor
// (the 4 floats (re t0, im t0, re t1, im t1) of an output row pair, K = the 4
// input rows) is broadcast from lanes 32 h + 4 g + i to all 16 blocks, as in
// the FP32 form above.
//
// State layout in LDS: per slot and 4-row quad, a record of 16 bytes a lane
// (column) for the hi parts {re rows 0-1, re rows 2-3, im rows 0-1, im rows
// 2-3} followed by the same for the lo parts: [slot][quad][hi|lo][64] uint4.
// Rows past a pair's rank inside its last quad hold zeros.
// ---------------------------------------------------------------------------
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned pack_bf16x2(float a, float b) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  typedef __bf16 b2v __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(unsigned, __builtin_convertvector((f2v){a, b}, b2v));
}
// hi = (bf16(a), bf16(b)) rounded to nearest even, lo = the same of the rests
// (a - hi is exact in FP32)
__device__ __forceinline__ void split_bf16(float a, float b, unsigned& hi, unsigned& lo) {
  hi = pack_bf16x2(a, b);
  lo = pack_bf16x2(a - __uint_as_float(hi << 16), b - __uint_as_float(hi & 0xffff0000u));
}

// P[g] += A x B_re, Q[g] += A x B_im for g < NG, A broadcast from block 8 H + g
template <int H, int NG, int KG, int G = 0>
__device__ __forceinline__ void split_terms(v4s a, v4s bre, v4s bim, v4f (&P)[KG], v4f (&Q)[KG]) {
  if constexpr (G < NG) {
    P[G] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, bre, P[G], 4, 8 * H + G, 0);
    Q[G] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, bim, Q[G], 4, 8 * H + G, 0);
    split_terms<H, NG, KG, G + 1>(a, bre, bim, P, Q);
  }
}
// one 4-row window: factor hi/lo (ah, al) against the state record (xh, xl)
template <int H, int NG, int KG>
__device__ __forceinline__ void split_window(uint2 ah, uint2 al, uint4 xh, uint4 xl,
                                             v4f (&P)[KG], v4f (&Q)[KG]) {
  const v4s Ah = __builtin_bit_cast(v4s, ah), Al = __builtin_bit_cast(v4s, al);
  const v4s Rh = __builtin_bit_cast(v4s, make_uint2(xh.x, xh.y));
  const v4s Ih = __builtin_bit_cast(v4s, make_uint2(xh.z, xh.w));
  const v4s Rl = __builtin_bit_cast(v4s, make_uint2(xl.x, xl.y));
  const v4s Il = __builtin_bit_cast(v4s, make_uint2(xl.z, xl.w));
  split_terms<H, NG, KG>(Ah, Rh, Ih, P, Q);
  split_terms<H, NG, KG>(Ah, Rl, Il, P, Q);
  split_terms<H, NG, KG>(Al, Rh, Ih, P, Q);
}
// a quad record from four complex rows (zeros past `live` rows)
__device__ __forceinline__ void split_quad(const float2 (&v)[4], uint4& h, uint4& l) {
  split_bf16(v[0].x, v[1].x, h.x, l.x);
  split_bf16(v[2].x, v[3].x, h.y, l.y);
  split_bf16(v[0].y, v[1].y, h.z, l.z);
  split_bf16(v[2].y, v[3].y, h.w, l.w);
}

// factor windows held in registers: FP32 form, 2 rows a window (one float a
// lane); split form, 8 rows a register pair (hi and lo, 4 bf16 a lane each)
template <bool SPLIT, int KT> struct TightWin { float a[KT]; };
template <int KT> struct TightWin<true, KT> {
  uint2 h[(KT + 3) / 4], l[(KT + 3) / 4];
};

template <typename FT, int KT, bool SPLIT>
__device__ __forceinline__ void tight_body(const TightDesc& D, int64_t lb, int64_t lstep,
                                           int64_t lend) {
  constexpr int NB = 64;
  constexpr int KG = KT / 2;                                  // most row pairs of an output
  constexpr int WC = KT / 2;                                  // most windows per child
  constexpr int WQ = (KT + 3) / 4;                            // split: most quads per child
  constexpr int WR = WQ;                                      // split: window registers (2 quads each)
  static_assert(!SPLIT || std::is_same<FT, bf16x2c>::value, "split products need BF16X2 factors");
  extern __shared__ __align__(16) unsigned char smem[];
  const float2* __restrict__ in = reinterpret_cast<const float2*>(D.in);
  float2* __restrict__ out = reinterpret_cast<float2*>(D.out);
  const TightArgs& A = D.A;
  const int L = A.L, nrhs = A.nrhs, nchunk = A.nchunk, KS = A.KS;
  const int K4 = A.nst;                                       // stages = log2(waves)
  float2* S = reinterpret_cast<float2*>(smem);                // [2^k][KS][64]
  uint4* S4 = reinterpret_cast<uint4*>(smem);                 // split: [2^k][KQ][2][64]
  const int KQ = (KS + 3) >> 2;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int half = lane >> 5, e = lane & 31;
  const int sh_end = L - (A.l_start + K4 - 1);

  struct Grp {
    int64_t gid;
    int nb0, nbw;
  };
  auto decode = [&](int64_t l) {
    Grp g;
    g.gid = l / nchunk;
    g.nb0 = (int)(l - g.gid * nchunk) * NB;
    g.nbw = min(NB, nrhs - g.nb0);
    return g;
  };
  // the global pairs of stage j: inputs of output slot w and the output
  struct StageWork {
    int64_t pout;
    int in0, kin0, kin1, kout;
  };
  auto stage_work = [&](const Grp& g, int j) {
    StageWork s;
    const int rem = K4 - j - 1;
    const int l = A.l_start + j;
    const int64_t gme = g.gid;
    const int64_t ap = gme >> sh_end, bpp = gme & (((int64_t)1 << sh_end) - 1);
    s.in0 = fused_in0(w, rem);
    int64_t p0, p1;
    if (j == 0) {
      p0 = (g.gid << K4) | s.in0;
      p1 = p0 + 1;
    } else {
      p0 = fused_pout(s.in0, j - 1, rem + 1, ap, bpp, L, l - 1);
      p1 = fused_pout(s.in0 + 1, j - 1, rem + 1, ap, bpp, L, l - 1);
    }
    s.kin0 = A.prk[j][p0];
    s.kin1 = A.prk[j][p1];
    s.pout = fused_pout(w, j, rem, ap, bpp, L, l);
    s.kout = A.prk[j + 1][s.pout];
    return s;
  };
  // factor windows of stage j for output pair pout: child c window i holds
  // rows 2i, 2i + 1 of child c's block rows (rows clamped to the child's
  // rank, so every window loads and the code is straight-line; the lanes
  // past a row's 2 kld floats read the next row or the slack past the
  // stage's blocks, and are never used)
  auto load_windows = [&](int j, const StageWork& s, TightWin<SPLIT, KT>& W) {
    const int kld = A.kld[j], Kin = A.kst[j];
    if constexpr (SPLIT) {
      // The 2 WQ quads of the two children, child 0 first, are numbered
      // v = c WQ + i; register m holds quads 2 m (lanes 0-31) and 2 m + 1
      // (lanes 32-63).  Lane 32 h + 4 g + i takes the record of float
      // f = 4 g + i of quad 2 m + h: bf16 hi and lo of rows 4 q .. 4 q + 3,
      // already in operand order.  f is clamped to the output pair's rank and
      // q to the quads of the child's rank (both inside the pair's records),
      // so the padding of the stored blocks is not read: the clamped loads
      // repeat a record already loaded and feed only unused blocks or rows
      // that meet zero state.
      const int nq = (Kin + 3) >> 2, nf = 2 * kld;
      const uint4* qb = reinterpret_cast<const uint4*>(A.qblk[j]) + s.pout * (int64_t)(2 * nq * nf);
      const int f = min(e, max(2 * s.kout - 1, 0));
#pragma unroll
      for (int m = 0; m < WR; ++m) {
        const int v = 2 * m + half, c = v >= WQ ? 1 : 0;
        const int qmax = max((((c ? s.kin1 : s.kin0) + 3) >> 2) - 1, 0);
        const int q = min(v - c * WQ, qmax);
        const uint4 d = qb[(c * nq + q) * nf + f];
        W.h[m] = make_uint2(d.x, d.y);
        W.l[m] = make_uint2(d.z, d.w);
      }
    } else {
      const int rowf = 2 * kld;                               // floats a row
      const FT* fb = reinterpret_cast<const FT*>(A.blk[j]) + s.pout * (int64_t)(2 * Kin * kld);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int rmax = max((c ? s.kin1 : s.kin0) - 1, 0);
#pragma unroll
        for (int i = 0; i < WC; ++i) {
          const int row = c * Kin + min(2 * i + half, rmax);
          W.a[c * WC + i] = block_float(fb, 0, (unsigned)(row * rowf + e));
        }
      }
    }
  };
  float2 xin[KT];
  // input rows of slot w of group g (rows past the pair's rank re-read its last row)
  auto fetch_inputs = [&](const Grp& g) {
    const int64_t pin = (g.gid << K4) | w;
    const int kin = A.prk[0][pin];
    const bool ok = lane < g.nbw;
    const float2* src = in + pin * A.kst[0] * (int64_t)nrhs + g.nb0 + (ok ? lane : 0);
    const int rmax = max(kin - 1, 0);
#pragma unroll
    for (int i = 0; i < KT; ++i) {
      const float2 v = src[(int64_t)min(i, rmax) * nrhs];
      xin[i] = ok ? v : make_float2(0.f, 0.f);
    }
  };
  auto deposit_inputs = [&](const Grp& g) {
    const int kin = A.prk[0][(g.gid << K4) | w];
    if constexpr (SPLIT) {
      uint4* dst = S4 + (size_t)w * KQ * 128 + lane;
#pragma unroll
      for (int q = 0; q < WQ; ++q) {
        if (4 * q < kin) {
          float2 v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int r = 4 * q + k;
            v[k] = make_float2(0.f, 0.f);
            if (r < KT) v[k] = r < kin ? xin[r < KT ? r : 0] : make_float2(0.f, 0.f);
          }
          uint4 h, l;
          split_quad(v, h, l);
          dst[q * 128] = h;
          dst[q * 128 + 64] = l;
        }
      }
      return;
    }
    float2* dst = S + (size_t)w * KS * NB + lane;
#pragma unroll
    for (int i = 0; i < KT; ++i)
      if (i < kin) dst[i * NB] = xin[i];
  };

  Grp cur = decode(lb);
  fetch_inputs(cur);
  TightWin<SPLIT, KT> aw, an;
  StageWork sw = stage_work(cur, 0);
  load_windows(0, sw, aw);
  deposit_inputs(cur);
  __syncthreads();
  while (true) {
    const int64_t nlb = lb + lstep;
    const bool more = nlb < lend;
    const Grp nxt = more ? decode(nlb) : cur;
#pragma unroll 1
    for (int j = 0; j < K4; ++j) {
      const bool last = j == K4 - 1;
      // this stage's factor rows (loaded during the previous stage) have
      // arrived; waiting here, before the next loads issue, spares the
      // products below waits on the loads still in flight
      __builtin_amdgcn_s_waitcnt(0x0F70);                     // vmcnt(0)
      // the next stage's (or the next group's first) factor rows: in flight
      // during this stage's products
      StageWork sn;
      if (!last) {
        sn = stage_work(cur, j + 1);
        load_windows(j + 1, sn, an);
      } else if (more) {
        sn = stage_work(nxt, 0);
        load_windows(0, sn, an);
        fetch_inputs(nxt);
      }
      const int ng = (sw.kout + 1) >> 1;
      v4f P[KG], Q[KG];
#pragma unroll
      for (int g = 0; g < KG; ++g) {
        P[g] = v4f{0.f, 0.f, 0.f, 0.f};
        Q[g] = v4f{0.f, 0.f, 0.f, 0.f};
      }
      // the rows of each child in windows of two, the last window first (a
      // chain of guarded blocks with one exit: an early exit from the
      // unrolled loop would have the compiler duplicate the rest of the stage
      // into every exit); the next window's state rows are read from LDS
      // while the current window's MFMAs issue.  One instantiation per output
      // row-pair count, chosen once per stage: no per-MFMA branches (uniform
      // branches take scalar-unit issue slots, which the SIMDs of a CU share)
      auto product = [&](auto ng_c) {
        constexpr int NG = decltype(ng_c)::value;
        if constexpr (SPLIT) {
          // the child's quads, the last first (a chain of guarded blocks);
          // a quad's state records are read from LDS just before its MFMAs
          // (the other waves of the SIMD keep the MFMA unit busy meanwhile)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const int nwin = ((c ? sw.kin1 : sw.kin0) + 3) >> 2;
            const uint4* X = S4 + (size_t)(sw.in0 + c) * KQ * 128 + lane;
#pragma unroll
            for (int i = WQ - 1; i >= 0; --i) {
              if (i < nwin) {
                const uint4 xh = X[i * 128], xl = X[i * 128 + 64];
                const int v = c * WQ + i;
                const uint2 ah = aw.h[v >> 1], al = aw.l[v >> 1];
                if (v & 1) split_window<1, NG, KG>(ah, al, xh, xl, P, Q);
                else split_window<0, NG, KG>(ah, al, xh, xl, P, Q);
              }
            }
          }
        } else {
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const int kin = c ? sw.kin1 : sw.kin0;
            const int nwin = (kin + 1) >> 1;
            const float2* X = S + (size_t)(sw.in0 + c) * KS * NB + lane;
            const int rl = max(2 * nwin - 2, 0);
            float2 x0 = X[rl * NB], x1 = X[(rl + 1) * NB];
#pragma unroll
            for (int i = WC - 1; i >= 0; --i) {
              if (i < nwin) {
                float2 y0 = x0, y1 = x1;
                if (i > 0) {
                  y0 = X[(2 * i - 2) * NB];
                  y1 = X[(2 * i - 1) * NB];
                }
                const float a = aw.a[c * WC + i];
                tight_row<0, NG, KG>(a, x0, P, Q);
                if (2 * i + 1 < kin) tight_row<1, NG, KG>(a, x1, P, Q);
                x0 = y0;
                x1 = y1;
              }
            }
          }
        }
      };
      switch (ng) {
        case 1: product(std::integral_constant<int, 1>{}); break;
        case 2: if constexpr (KG >= 2) product(std::integral_constant<int, 2>{}); break;
        case 3: if constexpr (KG >= 3) product(std::integral_constant<int, 3>{}); break;
        case 4: if constexpr (KG >= 4) product(std::integral_constant<int, 4>{}); break;
        case 5: if constexpr (KG >= 5) product(std::integral_constant<int, 5>{}); break;
        case 6: if constexpr (KG >= 6) product(std::integral_constant<int, 6>{}); break;
        case 7: if constexpr (KG >= 7) product(std::integral_constant<int, 7>{}); break;
        case 8: if constexpr (KG >= 8) product(std::integral_constant<int, 8>{}); break;
        default: break;                                       // rank 0: a zero output
      }
      __syncthreads();                                        // every wave read its inputs
      if (!last && SPLIT) {
        // outputs as quad records (rows past the output's rank zero)
        uint4* dst = S4 + (size_t)w * KQ * 128 + lane;
#pragma unroll
        for (int q = 0; q < (KG + 1) / 2; ++q) {
          if (4 * q < sw.kout) {
            float2 v[4];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
              const int g = 2 * q + s2;
              v4f pp = v4f{0.f, 0.f, 0.f, 0.f}, qq = v4f{0.f, 0.f, 0.f, 0.f};
              if (g < KG) {
                pp = P[g < KG ? g : 0];
                qq = Q[g < KG ? g : 0];
              }
              const bool l0 = 2 * g < sw.kout, l1 = 2 * g + 1 < sw.kout;
              v[2 * s2] = l0 ? make_float2(pp[0] - qq[1], pp[1] + qq[0]) : make_float2(0.f, 0.f);
              v[2 * s2 + 1] = l1 ? make_float2(pp[2] - qq[3], pp[3] + qq[2]) : make_float2(0.f, 0.f);
            }
            uint4 h, l;
            split_quad(v, h, l);
            dst[q * 128] = h;
            dst[q * 128 + 64] = l;
          }
        }
      } else if (!last) {
        float2* dst = S + (size_t)w * KS * NB + lane;
#pragma unroll
        for (int g = 0; g < KG; ++g) {
          if (2 * g < sw.kout) {
            const v4f pp = P[g], qq = Q[g];
            dst[(2 * g) * NB] = make_float2(pp[0] - qq[1], pp[1] + qq[0]);
            if (2 * g + 1 < sw.kout) dst[(2 * g + 1) * NB] = make_float2(pp[2] - qq[3], pp[3] + qq[2]);
          }
        }
      } else if (lane < cur.nbw) {
        // last stage: the output pair's rows to HBM at the stored row stride:
        // the rows of its rank, or all stored rows (zero past its rank)
        const int Kout = A.kst[K4];
        const int Kw = A.rank_out ? sw.kout : Kout;
        float2* dst = out + sw.pout * Kout * (int64_t)nrhs + cur.nb0 + lane;
#pragma unroll
        for (int g = 0; g < KG; ++g) {
          if (2 * g < Kw) {
            const v4f pp = P[g], qq = Q[g];
            const bool live = g < ng;
            dst[(int64_t)(2 * g) * nrhs] = live ? make_float2(pp[0] - qq[1], pp[1] + qq[0])
                                                : make_float2(0.f, 0.f);
            if (2 * g + 1 < Kw)
              dst[(int64_t)(2 * g + 1) * nrhs] = live ? make_float2(pp[2] - qq[3], pp[3] + qq[2])
                                                      : make_float2(0.f, 0.f);
          }
        }
      }
      if (!last || more) {
        sw = sn;
        aw = an;
      }
      if (!last) __syncthreads();                             // outputs in place
    }
    if (!more) break;
    deposit_inputs(nxt);
    __syncthreads();
    lb = nlb;
    cur = nxt;
  }
}

// a block of 64 * 2^nst threads, at most 16 waves (8 for KT > 12, whose
// registers would not fit 16 waves); persistent over `total` groups
template <int KT>
constexpr int tight_max_waves() { return KT > 12 ? 8 : 16; }
template <typename FT, int KT>
__global__ __launch_bounds__(64 * tight_max_waves<KT>()) void k_apply_tight(TightDesc D,
                                                                            int64_t total) {
  tight_body<FT, KT, false>(D, blockIdx.x, (int64_t)gridDim.x, total);
}
template <int KT>
__global__ __launch_bounds__(64 * tight_max_waves<KT>()) void k_apply_tight_split(TightDesc D,
                                                                                  int64_t total) {
  tight_body<bf16x2c, KT, true>(D, blockIdx.x, (int64_t)gridDim.x, total);
}

// Middle block of the swept-in factorization: out[p][t][n] = sum_s Mdot[p][t][s] in[p][s][n]
struct MidDesc {
  const void* in;
  void* out;
  const void* mdot;
  int kin, kout, nrhs;
  int64_t total;
};

template <typename VT, typename FT>
__global__ __launch_bounds__(kBlock) void k_apply_mid(MidDesc d) {
  const VT* __restrict__ in = reinterpret_cast<const VT*>(d.in);
  VT* __restrict__ out = reinterpret_cast<VT*>(d.out);
  const FT* __restrict__ mdot = reinterpret_cast<const FT*>(d.mdot);
  const int kin = d.kin, kout = d.kout, nrhs = d.nrhs;
  const int64_t total = d.total;
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
// LDS: mu_leaf[2^l0][K][NB], and when it fits ubar_leaf[smax][2^l0 K + 1] (padded rows).
// ---------------------------------------------------------------------------
struct UDesc {
  const void* mu;
  void* u;
  int64_t ldu;
  const int32_t* perm_x;
  const int32_t* xoff;
  const void* ubar;
  int l0, K, nrhs, NB, nchunk, smax, stage_f;
  const uint8_t* prk;   // MFMA U: per-pair ranks at level L - l0; rows past a
                        // pair's rank are not read (null: every row is read)
};

template <typename VT, typename FT>
__device__ __forceinline__ void apply_u_body(const UDesc& d, int64_t lb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const VT* __restrict__ mu = reinterpret_cast<const VT*>(d.mu);
  VT* __restrict__ u = reinterpret_cast<VT*>(d.u);
  const FT* __restrict__ ubar = reinterpret_cast<const FT*>(d.ubar);
  const int32_t* __restrict__ perm_x = d.perm_x;
  const int32_t* __restrict__ xoff = d.xoff;
  const int64_t ldu = d.ldu;
  const int l0 = d.l0, K = d.K, nrhs = d.nrhs, NB = d.NB, nchunk = d.nchunk;
  const int stage_factor = d.stage_f;
  const int nb = 1 << l0;
  const int urow = nb * K + 1;
  VT* ml = reinterpret_cast<VT*>(smem);                       // [nb][K][NB]
  VT* ul = ml + (size_t)nb * K * NB;                          // [smax][urow] if staged
  const int64_t a = lb / nchunk;
  const int chunk = (int)(lb % nchunk);
  const int nb0 = chunk * NB;
  const int nbw = min(NB, nrhs - nb0);
  const int32_t x0 = xoff[a], cnt = xoff[a + 1] - x0;
  const int64_t p0 = a << l0;
  {
    const FastDiv divW(nbw);
    const VT* src = mu + p0 * K * nrhs + nb0;
    staged_copy_to<8>(nb * K * nbw, ml, [&](int e, int& off) {
      int bk, n;
      divW.divmod(e, bk, n);
      off = bk * NB + n;
      return src[(int64_t)bk * nrhs + n];
    });
  }
  const FT* usrc = ubar + (int64_t)x0 * nb * K;
  if (stage_factor) {
    const FastDiv divR(nb * K);
    staged_copy_to<8>(cnt * nb * K, ul, [&](int e, int& off) {
      int x, r;
      divR.divmod(e, x, r);
      off = x * urow + r;
      return load_factor(usrc, e);
    });
  }
  __syncthreads();
  if (!stage_factor && nbw >= 16) {
    // two adjacent columns a thread: each factor entry is loaded and widened
    // once for both (point-major items; 16 RHS NUDFT: U 1.20 -> 0.95 ms; for
    // chunks of a few columns the single-column items below measured faster)
    const int nbh = (nbw + 1) >> 1;
    for (int item = threadIdx.x; item < cnt * nbh; item += blockDim.x) {
      const int x = item / nbh, n = 2 * (item - x * nbh);
      const int n1 = n + 1 < nbw ? n + 1 : n;
      VT acc0 = Zero<VT>::v(), acc1 = Zero<VT>::v();
      const FT* ur = usrc + (int64_t)x * nb * K;
      for (int bk = 0; bk < nb * K; ++bk) {
        const VT f = load_factor(ur, bk);
        cfma(acc0, f, ml[(size_t)bk * NB + n]);
        cfma(acc1, f, ml[(size_t)bk * NB + n1]);
      }
      const int64_t pi = perm_x[x0 + x];
      u[(int64_t)(nb0 + n) * ldu + pi] = acc0;
      if (n + 1 < nbw) u[(int64_t)(nb0 + n + 1) * ldu + pi] = acc1;
    }
    return;
  }
  // point-major items: a wave covers 64 / nbw points, so its lanes read few
  // distinct factor rows
  for (int item = threadIdx.x; item < cnt * nbw; item += blockDim.x) {
    const int x = item / nbw, n = item - x * nbw;
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

template <typename VT, typename FT>
__global__ __launch_bounds__(kBlock) void k_apply_u(UDesc d) {
  apply_u_body<VT, FT>(d, xcd_logical_block((int64_t)gridDim.x));
}
template <typename VT, typename FT>
__global__ __launch_bounds__(kBlock) void k_batch_u(const UDesc* __restrict__ ds,
                                                    const int64_t* __restrict__ boff, int count) {
  const int p = find_problem(boff, count, blockIdx.x);
  apply_u_body<VT, FT>(ds[p], (int64_t)blockIdx.x - boff[p]);
}

// ---------------------------------------------------------------------------
// V and U on MFMA (FP32 state, 64-column RHS chunks, leaves of at most 16
// points).  Both are small complex products per leaf with the same operand
// layout as the butterfly stages: lane l carries RHS column l, MFMA block
// b = l >> 2 a group of 4 columns, A-operand row i = l & 3 the raw float i of
// a pair of complex factor entries, and the outputs of a row pair follow from
// P = sum f_i x_re and Q = sum f_i x_im as
//   out[2g] = (P0 - Q1, P1 + Q0),  out[2g+1] = (P2 - Q3, P3 + Q2).
// ---------------------------------------------------------------------------
constexpr int kLeafMfma = 16;          // leaf points handled by the MFMA V / U
constexpr int kVChunk = 6;             // output row pairs per V accumulator set

// V: the leaf's output rows t = a K + k (R = 2^l0 K of them, in pairs) over
// its points.  LDS: g_leaf [16][65] (gathered, zero rows past the leaf's
// points; rows padded so that the gather's point-major stores spread over the
// banks) and Vbar [cnt][R] (+ slack for the last chunk's reads past R).
// Wave w computes row-pair chunks w, w + 4, ... with the 16 point rows of g
// held in registers.
template <typename FT>
__device__ __forceinline__ void apply_v_mfma_body(const VDesc& d, int64_t lb) {
  constexpr int NB = 64, CH = kVChunk, SM = kLeafMfma;
  extern __shared__ __align__(16) unsigned char smem[];
  const float2* __restrict__ g = reinterpret_cast<const float2*>(d.g);
  const FT* __restrict__ vbar = reinterpret_cast<const FT*>(d.vbar);
  float2* __restrict__ mu = reinterpret_cast<float2*>(d.mu);
  const int L = d.L, l0 = d.l0, K = d.K, nrhs = d.nrhs, nchunk = d.nchunk;
  const int64_t ldg = d.ldg;
  constexpr int GP = NB + 1;                                  // padded g row
  float2* gl = reinterpret_cast<float2*>(smem);               // [16][GP]
  float2* vl = gl + SM * GP;                                  // [cnt][R]
  const int64_t b = lb / nchunk;
  const int nb0 = (int)(lb - b * nchunk) * NB;
  const int nbw = min(NB, nrhs - nb0);
  const int32_t j0 = d.xioff[b], cnt = d.xioff[b + 1] - j0;
  const int R = K << l0;
  // gather g for the leaf (points fastest: contiguous within a column of g);
  // rows and columns outside the leaf and the chunk are zero
  staged_copy_to<8>(SM * NB, gl, [&](int e, int& off) {
    const int n = e >> 4, j = e & 15;
    off = j * GP + n;
    return (j < cnt && n < nbw) ? g[(int64_t)(nb0 + n) * ldg + d.perm_xi[j0 + j]]
                                : make_float2(0.f, 0.f);
  });
  const FT* vsrc = vbar + (int64_t)j0 * R;
  const int sh = L - l0;
  const FastDiv divK(K);
  // output row t = a K + k is written iff k is within the rank of pair
  // (a, b) (a byte a row after Vbar in LDS, computed while the copies load)
  unsigned char* rl = reinterpret_cast<unsigned char*>(vl + (size_t)SM * R + 2 * kVChunk);
  if (d.prk)
    for (int t = threadIdx.x; t < R; t += kBlock) {
      int a, k;
      divK.divmod(t, a, k);
      rl[t] = k < (int)d.prk[((int64_t)a << sh) | b] ? 1 : 0;
    }
  staged_copy_to<8>(cnt * R, vl, [&](int e, int& off) {
    off = e;
    return load_factor(vsrc, e);
  });
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int fi = lane & 3;
  float2 xr[SM];
#pragma unroll
  for (int j = 0; j < SM; ++j) xr[j] = gl[j * GP + lane];
  const int npair = R >> 1, nchk = (npair + CH - 1) / CH;
  for (int c = wave; c < nchk; c += 4) {
    v4f P[CH], Q[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      P[q] = v4f{0.f, 0.f, 0.f, 0.f};
      Q[q] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    const float* f = reinterpret_cast<const float*>(vl) + 4 * c * CH + fi;
#pragma unroll
    for (int j = 0; j < SM; ++j) {
      if (j < cnt) {
        float av[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) av[q] = f[2 * j * R + 4 * q];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          P[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[q], xr[j].x, P[q], 0, 0, 0);
          Q[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[q], xr[j].y, Q[q], 0, 0, 0);
        }
      }
    }
    if (lane < nbw) {
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        const int rp = c * CH + q;
        if (rp < npair) {
          const v4f pp = P[q], qq = Q[q];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            int a, k;
            divK.divmod(2 * rp + h, a, k);
            const int64_t pr = ((int64_t)a << sh) | b;
            if (!d.prk || rl[2 * rp + h])
              mu[(pr * K + k) * nrhs + nb0 + lane] =
                  h == 0 ? make_float2(pp[0] - qq[1], pp[1] + qq[0])
                         : make_float2(pp[2] - qq[3], pp[3] + qq[2]);
          }
        }
      }
    }
  }
}

// U: u[x][n] = sum_r Ubar[x][r] mu[p0 + r / K][r % K][n] over the R = 2^l0 K
// rows of the leaf's contiguous pairs (R a multiple of 16).  LDS: Ubar
// transposed to [R][17] (rows past the leaf's points are zero; the padding
// spreads the transposing stores over the banks) and four partial [16][64]
// tiles.  Wave w takes rows w R/4 .. (w+1) R/4 - 1 for all 16 points: its mu
// rows come straight from memory, all loads in flight at once, and each
// v_mfma_f32_4x4x1f32 broadcasts the four floats of one point pair of one
// row (lanes 0-31 hold row r, lanes 32-63 row r + 1, float e in lane e: the
// A block of point pair q is lanes 32 h + 4 q .. + 3, abid 8 h + q).  The
// four partial tiles are summed by the point-contiguous stores.
template <int H, int G = 0>
__device__ __forceinline__ void u_row(float a, float2 x, v4f (&P)[8], v4f (&Q)[8]) {
  if constexpr (G < 8) {
    P[G] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, x.x, P[G], 4, 8 * H + G, 0);
    Q[G] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, x.y, Q[G], 4, 8 * H + G, 0);
    u_row<H, G + 1>(a, x, P, Q);
  }
}

template <typename FT>
__device__ __forceinline__ void apply_u_mfma_body(const UDesc& d, int64_t lb) {
  constexpr int NB = 64, SM = kLeafMfma, RB = 8;
  static_assert(SM == 16, "one point pair per MFMA block: 8 pairs of a 32-float row");
  extern __shared__ __align__(16) unsigned char smem[];
  const float2* __restrict__ mu = reinterpret_cast<const float2*>(d.mu);
  float2* __restrict__ u = reinterpret_cast<float2*>(d.u);
  const FT* __restrict__ ubar = reinterpret_cast<const FT*>(d.ubar);
  const int l0 = d.l0, K = d.K, nrhs = d.nrhs, nchunk = d.nchunk;
  const int64_t ldu = d.ldu;
  const int R = K << l0;
  constexpr int UP = SM + 1;                                  // padded Ubar row
  float2* ul = reinterpret_cast<float2*>(smem);               // [R][UP]
  float2* ot = ul + (size_t)R * UP;                           // [4][16][64]
  const int64_t a = lb / nchunk;
  const int nb0 = (int)(lb - a * nchunk) * NB;
  const int nbw = min(NB, nrhs - nb0);
  const int32_t x0 = d.xoff[a], cnt = d.xoff[a + 1] - x0;
  const int64_t p0 = a << l0;
  const FT* usrc = ubar + (int64_t)x0 * R;
  const FastDiv divR(R);
  staged_copy_to<8>(R * SM, ul, [&](int e, int& off) {
    int x, r;
    divR.divmod(e, x, r);                                     // e = x R + r: reads coalesced
    off = r * UP + x;
    return x < cnt ? load_factor(usrc, e) : make_float2(0.f, 0.f);
  });
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int half = lane >> 5;
  const bool col = lane < nbw;
  const int rw = R >> 2, r0 = wave * rw;                      // this wave's rows (even count)
  const float2* src = mu + (p0 * K + r0) * nrhs + nb0 + lane;
  // the wave's mu rows, RB at a time, the first batch issued before the
  // barrier that publishes Ubar
  // rows past their pair's rank hold no data (their Ubar entries are zero)
  // and are not read: bit i of `live` is row r0 + i of this wave (rw <= 64
  // when ranks are given)
  uint64_t live = ~0ull;
  if (d.prk) {
    const FastDiv divK(K);
    int q = 0, k = 0;
    if (lane < rw) divK.divmod(r0 + lane, q, k);
    live = __ballot(lane >= rw || k < (int)d.prk[p0 + q]);
  }
  float2 xa[RB], xb[RB];
  auto load_rows = [&](int i0, float2 (&X)[RB]) {
#pragma unroll
    for (int i = 0; i < RB; ++i)
      X[i] = (col && i0 + i < rw && ((live >> ((i0 + i) & 63)) & 1ull))
                 ? src[(int64_t)(i0 + i) * nrhs]
                 : make_float2(0.f, 0.f);
  };
  load_rows(0, xa);
  __syncthreads();
  v4f P[8], Q[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    P[q] = v4f{0.f, 0.f, 0.f, 0.f};
    Q[q] = v4f{0.f, 0.f, 0.f, 0.f};
  }
  // A registers: float (lane & 31) of rows r0 + i + half, i even
  const float* f = reinterpret_cast<const float*>(ul) + (size_t)(r0 + half) * 2 * UP + (lane & 31);
  auto mfma_rows = [&](int i0, const float2 (&X)[RB]) {
#pragma unroll
    for (int i = 0; i < RB; i += 2) {
      if (i0 + i < rw) {
        const float av = f[(size_t)(i0 + i) * 2 * UP];
        u_row<0>(av, X[i], P, Q);
        u_row<1>(av, X[i + 1], P, Q);
      }
    }
  };
#pragma unroll 1
  for (int i0 = 0; i0 < rw; i0 += 2 * RB) {
    load_rows(i0 + RB, xb);
    mfma_rows(i0, xa);
    if (i0 + 2 * RB < rw) load_rows(i0 + 2 * RB, xa);
    mfma_rows(i0 + RB, xb);
  }
  // partial tile of this wave: point 2 q + h, column lane
  float2* pt = ot + (size_t)wave * SM * NB + lane;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const v4f pp = P[q], qq = Q[q];
    pt[(2 * q) * NB] = make_float2(pp[0] - qq[1], pp[1] + qq[0]);
    pt[(2 * q + 1) * NB] = make_float2(pp[2] - qq[3], pp[3] + qq[2]);
  }
  __syncthreads();
  // sum of the four partials, point-contiguous stores: item = n * 16 + x
  for (int item = threadIdx.x; item < SM * NB; item += kBlock) {
    const int x = item & 15, n = item >> 4;
    if (x < cnt && n < nbw) {
      float2 v = ot[x * NB + n];
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        const float2 t = ot[(size_t)w * SM * NB + x * NB + n];
        v.x += t.x;
        v.y += t.y;
      }
      u[(int64_t)(nb0 + n) * ldu + d.perm_x[x0 + x]] = v;
    }
  }
}

template <typename FT>
__global__ __launch_bounds__(kBlock) void k_apply_v_mfma(VDesc d) {
  apply_v_mfma_body<FT>(d, xcd_logical_block((int64_t)gridDim.x));
}
template <typename FT>
__global__ __launch_bounds__(kBlock) void k_batch_v_mfma(const VDesc* __restrict__ ds,
                                                         const int64_t* __restrict__ boff,
                                                         int count) {
  const int p = find_problem(boff, count, blockIdx.x);
  apply_v_mfma_body<FT>(ds[p], (int64_t)blockIdx.x - boff[p]);
}
template <typename FT>
__global__ __launch_bounds__(kBlock) void k_apply_u_mfma(UDesc d) {
  apply_u_mfma_body<FT>(d, xcd_logical_block((int64_t)gridDim.x));
}
template <typename FT>
__global__ __launch_bounds__(kBlock) void k_batch_u_mfma(const UDesc* __restrict__ ds,
                                                         const int64_t* __restrict__ boff,
                                                         int count) {
  const int p = find_problem(boff, count, blockIdx.x);
  apply_u_mfma_body<FT>(ds[p], (int64_t)blockIdx.x - boff[p]);
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
    if (!prof || prof->n_launches >= IBF_PROFILE_MAX) return IBF_OK;
    hipEvent_t a;
    IBF_HIP_CHECK(hipEventCreate(&a));
    ev.push_back(a);
    IBF_HIP_CHECK(hipEventRecord(a, s));
    return IBF_OK;
  }
  int end(const char* name, double flops, double bytes, double vec_bytes) {
    if (!prof || prof->n_launches >= IBF_PROFILE_MAX) return IBF_OK;
    hipEvent_t b;
    IBF_HIP_CHECK(hipEventCreate(&b));
    ev.push_back(b);
    IBF_HIP_CHECK(hipEventRecord(b, s));
    const int i = prof->n_launches++;
    std::snprintf(prof->name[i], sizeof(prof->name[i]), "%s", name);
    prof->flops[i] = flops;
    prof->bytes[i] = bytes;
    prof->vec_bytes[i] = vec_bytes;
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

// Kernel templates are instantiated for even KT = 2..16 (the padded row
// width of the staged factor blocks).
#define IBF_DISPATCH_KT(kt, LAUNCH)                 \
  switch (kt) {                                     \
    case 2: LAUNCH(2); break;                       \
    case 4: LAUNCH(4); break;                       \
    case 6: LAUNCH(6); break;                       \
    case 8: LAUNCH(8); break;                       \
    case 10: LAUNCH(10); break;                     \
    case 12: LAUNCH(12); break;                     \
    case 14: LAUNCH(14); break;                     \
    default: LAUNCH(16); break;                     \
  }

inline int even_kt(int k) { return std::min(16, std::max(2, (k + 1) & ~1)); }

// One kernel launch of an apply, with everything it needs.
enum LaunchKind { kLaunchV = 0, kLaunchFused = 1, kLaunchMid = 2, kLaunchU = 3, kLaunchTight = 4 };
struct Launch {
  LaunchKind kind;
  int kt = 2;
  bool mfma = false;
  bool split = false;                // per-pair-rank stages with BF16 split products
  size_t lds = 0;
  int64_t nblocks = 0;
  double flops = 0, bytes = 0, vec_bytes = 0;
  VDesc v{};
  FusedDesc f{};
  MidDesc m{};
  UDesc u{};
  TightDesc t{};
};

inline const char* launch_name(const Launch& x) {
  switch (x.kind) {
    case kLaunchV: return x.mfma ? "apply_v_mfma" : "apply_v";
    case kLaunchFused: return x.mfma ? "apply_fused_mfma" : "apply_fused";
    case kLaunchMid: return "apply_mid";
    case kLaunchTight: return x.split ? "apply_stage_tight_split" : "apply_stage_tight";
    default: return x.mfma ? "apply_u_mfma" : "apply_u";
  }
}

// Per-block LDS limit of the device (queried once per device).
inline int lds_limit(int device, int* out) {
  static int lds_max[64] = {0};
  int& lmax = lds_max[device & 63];
  if (!lmax) {
    int v = 0;
    IBF_HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    lmax = v > 0 ? v : 65536;
  }
  *out = lmax;
  return IBF_OK;
}

// The launch sequence of one apply of plan p: V, the fused butterfly stage
// groups (with the swept-in middle block between the two halves), U.
// Allocates the plan's ping-pong coefficient buffers when they are too small
// for nrhs, so it must run outside any graph capture.
template <typename VT, typename FT>
int make_schedule(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int nrhs,
                  std::vector<Launch>& seq, bool batch = false, void* const* ws = nullptr) {
  seq.clear();
  const Geo& geo = p->geo;
  const int L = geo.L, l0 = geo.l0, h = geo.h;
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
  if (!ws && need > p->work_bytes) {
    for (int i = 0; i < 2; ++i) {
      if (p->d_work[i]) (void)ibf::dev_free(p->d_work[i]);
      p->d_work[i] = nullptr;
    }
    p->work_bytes = 0;
    IBF_HIP_CHECK(ibf::dev_malloc(&p->d_work[0], need));
    IBF_HIP_CHECK(ibf::dev_malloc(&p->d_work[1], need));
    p->work_bytes = need;
  }
  // the ping-pong coefficient buffers: the plan's, or the caller's (the
  // allocation-free entry point passes two buffers of at least `need` bytes)
  void* w[2] = {ws ? ws[0] : p->d_work[0], ws ? ws[1] : p->d_work[1]};
  const double fb = (double)sizeof(FT), vb = (double)sizeof(VT);
  int lmax = 0, rc;
  if ((rc = lds_limit(p->device, &lmax))) return rc;
  const size_t budget_mfma = std::min<size_t>(kLdsBudgetMfma, (size_t)lmax);
  // Default rule: FP32-state stages with more than 8 RHS run on MFMA with
  // 32-column chunks (more than 16 RHS) or 16-column chunks; otherwise the
  // vector kernels take chunks of up to 32 columns.  A tuned schedule for this
  // nrhs (ibf_tune), or the candidate under trial, overrides the path, the
  // chunk width and the fusion depth.  The V and U leaf products use MFMA
  // from 32 RHS.
  Tuning tn{};
  if (p->trial_on) {
    tn = p->trial;
  } else {
    const auto it = p->tuned.find(nrhs);
    if (it != p->tuned.end()) tn = it->second;
  }
  bool mfma = sizeof(VT) == 8 && nrhs > 8;
  if (sizeof(VT) == 8 && tn.path == 1) mfma = false;
  if (sizeof(VT) == 8 && tn.path == 2) mfma = true;
  // stages at per-pair ranks (64-column chunks): the default from 64 RHS,
  // any FP32-state plan on path 3; needs the build's per-pair ranks (plans
  // without the sweep-in); not in batches
  const bool tight = sizeof(VT) == 8 && p->d_prank && !batch &&
                     ((tn.path == 0 && nrhs >= 64) || tn.path == 3 || tn.path == 4);
  // BF16X2 plans: the per-pair-rank stages multiply with BF16 split products
  // (path 4, and the default rule) or widen the factors to FP32 (path 3)
  const bool split = tight && std::is_same<FT, bf16x2c>::value && tn.path != 3 &&
                     std::all_of(p->stages.begin(), p->stages.end(),
                                 [](const Stage& st) { return st.qblk != nullptr; });
  const bool mfma_vu = sizeof(VT) == 8 && nrhs >= 32;
  const int NB = mfma ? (tn.chunk == 16 || tn.chunk == 32 ? tn.chunk : (nrhs > 16 ? 32 : 16))
                      : std::min(nrhs, 32);
  const int NV = kBlock / NB;                                 // MFMA virtual slots a block
  const int LNV = NV == 8 ? 3 : 4;
  const int nchunk = (nrhs + NB - 1) / NB;
  const int NBo = std::min(nrhs, 32);                         // outer (V, U) kernels
  // V
  {
    Launch x;
    x.kind = kLaunchV;
    const int K = p->k_vbar;
    x.kt = even_kt(K);
    const double nnz = (double)p->nnz_vbar;
    x.flops = 8.0 * nnz * nrhs;
    x.bytes = nnz * fb + vb * nrhs * (double)p->nxi;
    x.vec_bytes = vb * nrhs * (double)p->npairs * K;
    if (mfma_vu && p->smax_xi <= kLeafMfma && ((K << l0) & 1) == 0) {
      // MFMA leaf product, 64-column chunks
      const int R = K << l0;
      const int nchv = (nrhs + 63) / 64;
      x.mfma = true;
      // + a byte a row (the rows written before per-pair-rank stages)
      x.lds = ((size_t)kLeafMfma * 65 + (size_t)kLeafMfma * R + 2 * kVChunk) * sizeof(VT) + R;
      x.nblocks = p->nleaf * nchv;
      // before per-pair-rank stages, which read only the rows of each
      // pair's rank, the rows past it are not written
      x.v = VDesc{g, ldg, p->d_perm_xi, p->d_xioff, p->d_vbar, w[0], L, l0, K, nrhs, 64, nchv,
                  p->smax_xi, 1, tight ? p->d_prank : nullptr};
    } else {
      int NBv = NBo;
      while (NBv > 1 && (size_t)p->smax_xi * NBv * sizeof(VT) > kLdsBudget / 2) NBv /= 2;
      const int nchv = (nrhs + NBv - 1) / NBv;
      const size_t base = (size_t)p->smax_xi * NBv * sizeof(VT);
      const size_t fac = (size_t)p->smax_xi * (1 << l0) * x.kt * sizeof(VT);
      if (base > kLdsBudget) {
        set_error("ibf_apply: an Omega leaf holds too many points for the apply kernels");
        return IBF_ERR_UNSUPPORTED;
      }
      const int stage_f = base + fac <= kLdsBudget ? 1 : 0;
      x.lds = base + (stage_f ? fac : 0);
      x.nblocks = p->nleaf * nchv;
      x.v = VDesc{g, ldg, p->d_perm_xi, p->d_xioff, p->d_vbar, w[0], L, l0, K, nrhs, NBv, nchv,
                  p->smax_xi, stage_f, nullptr};
    }
    seq.push_back(x);
  }
  int cur = 0;
  auto add_mid = [&]() {
    Launch x;
    x.kind = kLaunchMid;
    const int64_t total = p->npairs * p->k_mid_g * nrhs;
    x.nblocks = (total + kBlock - 1) / kBlock;
    x.m = MidDesc{w[cur], w[cur ^ 1], p->d_mdot, p->k_mid_h, p->k_mid_g, nrhs, total};
    const double nnz = (double)p->npairs * p->k_mid_g * p->k_mid_h;
    x.flops = 8.0 * nnz * nrhs;
    x.bytes = nnz * fb;
    x.vec_bytes = (double)p->npairs * (p->k_mid_g + p->k_mid_h) * nrhs * vb;
    seq.push_back(x);
    cur ^= 1;
  };
  // LDS bytes of a fused block.  MFMA: 8 virtual slots (one group of 8 pairs or
  // 8 / 2^k groups side by side), state [8][kmaxg][32] + factors
  // [8][2 kmaxg kld] with kld <= kt, + 2 kt entries of slack (the compute loops
  // read whole kt-wide rows and one row past a block's end; entries past a row
  // feed only discarded outputs).  Vector path: a group of 2^k pairs in two
  // state buffers [2^k][kmaxg][NB], no factors.
  auto fused_lds = [&](int kk, int kmg, int kt) -> size_t {
    if (!mfma) return ((size_t)2 << kk) * kmg * NB * sizeof(VT);
    return ((size_t)NV * ((size_t)kmg * NB + (size_t)2 * kmg * kt + 20) + 2 * kt) * sizeof(VT);
  };
  // MFMA plans with the sweep-in apply the middle block inside the first
  // G-side launch (before its first stage) instead of a launch of its own
  bool fold_mid = false;
  auto add_stages = [&](int lo, int hi, bool gside) {   // output levels lo..hi
    int l = lo;
    if (tight) {
      while (l <= hi) {
        int kk = std::min(4, std::min(hi - l + 1, L - l + 1));
        if (tn.max_fused > 0) kk = std::min(kk, tn.max_fused);
        auto kmax_of = [&](int n) {
          int m = 1;
          for (int j = 0; j <= n; ++j) m = std::max(m, rank_at(l - 1 + j, gside));
          return m;
        };
        // LDS state: FP32 [2^k][km][64] + 4 rows (the product reads up to 3 rows
        // past a slot's live rows); split [2^k][quads][hi|lo][64] 16-byte records
        auto tight_lds = [&](int km_, int kk_) -> size_t {
          if (split) return ((size_t)((km_ + 3) / 4) << kk_) * 2 * 64 * 16;
          return (((size_t)km_ << kk_) + 4) * 64 * sizeof(VT);
        };
        // tiles above 12 rows run 8 waves a block (3 stages), and the state must fit LDS
        while (kk > 1 && ((even_kt(kmax_of(kk)) > 12 && kk > 3) ||
                          tight_lds(kmax_of(kk), kk) > (size_t)lmax))
          --kk;
        int km = kmax_of(kk);
        Launch x;
        x.kind = kLaunchTight;
        x.mfma = true;
        x.split = split;
        x.t.A.rank_out = 1;                                   // the next reader skips them
        TightArgs& T = x.t.A;
        T.L = L;
        T.l_start = l;
        T.nst = kk;
        T.nrhs = nrhs;
        T.nchunk = (nrhs + 63) / 64;
        km = 1;
        double nnz = 0;
        for (int j = 0; j <= kk; ++j) {
          T.kst[j] = rank_at(l - 1 + j, gside);
          T.prk[j] = p->d_prank + (size_t)(l - 1 + j - l0) * p->npairs;
          km = std::max(km, T.kst[j]);
        }
        for (int j = 0; j < kk; ++j) {
          const Stage& st = p->stages[l + j - l0 - 1];
          T.blk[j] = st.blk;
          T.qblk[j] = st.qblk;
          T.kld[j] = st.k_ld;
          nnz += (double)st.nnz;
        }
        T.KS = km;
        x.kt = even_kt(km);
        x.lds = tight_lds(km, kk);
        x.nblocks = (p->npairs >> kk) * T.nchunk;
        x.t.in = w[cur];
        x.t.out = w[cur ^ 1];
        x.flops = 8.0 * nnz * nrhs;
        x.bytes = nnz * fb;
        x.vec_bytes = (double)p->npairs * (T.kst[0] + T.kst[kk]) * nrhs * vb;
        seq.push_back(x);
        cur ^= 1;
        l += kk;
      }
      fold_mid = false;
      return;
    }
    while (l <= hi) {
      const bool mid_here = fold_mid && l == lo;
      int kk = 1;
      while (true) {   // grow the fused group while it fits
        const int next = kk + 1;
        if (l + next - 1 > hi) break;
        if (next > kMaxR - 1) break;
        if (next > L - l + 1) break;                          // group must fit the b bits
        if (tn.max_fused > 0 && next > tn.max_fused) break;
        // the default rule ends MFMA groups before a stage that fits a
        // smaller tile (its own launch then runs at the smaller tile, with
        // more resident waves): measured 2% faster on the random-point DFT
        const int split = tn.split ? tn.split : (mfma && tn.path == 0 ? 1 : 0);
        if (split) {
          // tile of the group so far against the tile of the stage to add
          int kg = mid_here ? p->k_mid_h : 1;
          for (int j = 0; j <= kk; ++j) kg = std::max(kg, rank_at(l - 1 + j, gside));
          const int ks = even_kt(std::max(rank_at(l + kk - 1, gside), rank_at(l + kk, gside)));
          if (ks < even_kt(kg) || (split == 2 && ks != even_kt(kg))) break;
        }
        int km = mid_here ? p->k_mid_h : 1;
        for (int j = 0; j <= next; ++j) km = std::max(km, rank_at(l - 1 + j, gside));
        // MFMA: at most NV slots a block; vector: at most 4 outputs per thread and stage
        if (mfma ? (next > LNV) : (((int64_t)1 << next) * km * NB > 4 * kBlock)) break;
        if (fused_lds(next, km, even_kt(km)) > (mfma ? budget_mfma : kLdsBudget)) break;
        kk = next;
      }
      Launch x;
      x.kind = kLaunchFused;
      x.mfma = mfma;
      FusedArgs& A = x.f.A;
      A.L = L;
      A.l_start = l;
      A.nst = kk;
      A.nrhs = nrhs;
      A.NB = NB;
      A.nchunk = nchunk;
      int km = 1, kom = 1;
      double nnz = 0;
      for (int j = 0; j <= kk; ++j) {
        A.ranks[j] = rank_at(l - 1 + j, gside);
        km = std::max(km, A.ranks[j]);
        if (j > 0) kom = std::max(kom, A.ranks[j]);
      }
      A.mid = nullptr;
      A.kmid_in = A.kmid_out = 0;
      int kin_launch = A.ranks[0];
      if (mid_here) {
        A.mid = p->d_mdot;
        A.kmid_in = p->k_mid_h;
        A.kmid_out = p->k_mid_g;
        km = std::max(km, p->k_mid_h);
        kin_launch = p->k_mid_h;
        nnz += (double)p->npairs * p->k_mid_g * p->k_mid_h;
      }
      A.kmaxg = km;
      for (int j = 0; j < kk; ++j) {
        const Stage& st = p->stages[l + j - l0 - 1];
        A.blk[j] = st.blk;
        A.kld[j] = st.k_ld;
        nnz += (double)st.nnz;
      }
      // (MFMA: KT also covers the launch's input rank, which bounds the
      // staged factor blocks at 2 KT^2 entries)
      x.kt = even_kt(mfma ? km : kom);
      x.lds = fused_lds(kk, km, x.kt);
      x.nblocks = (p->npairs >> (mfma ? LNV : kk)) * nchunk;
      x.f.in = w[cur];
      x.f.out = w[cur ^ 1];
      x.flops = 8.0 * nnz * nrhs;
      x.bytes = nnz * fb;
      x.vec_bytes = (double)p->npairs * (kin_launch + A.ranks[kk]) * nrhs * vb;
      seq.push_back(x);
      cur ^= 1;
      l += kk;
    }
    fold_mid = false;
  };
  if (swept) {
    add_stages(l0 + 1, h, false);
    // the first G-side launch starts from the middle block's output rank
    fold_mid = mfma && rank_at(h, true) == p->k_mid_g && h + 1 <= L - l0;
    if (!fold_mid) add_mid();
    add_stages(h + 1, L - l0, true);
  } else {
    add_stages(l0 + 1, L - l0, true);
  }
  // U
  {
    Launch x;
    x.kind = kLaunchU;
    const int K = p->k_ubar;
    const double nnz = (double)p->nnz_ubar;
    x.flops = 8.0 * nnz * nrhs;
    x.bytes = nnz * fb + vb * nrhs * (double)p->nx;
    x.vec_bytes = vb * nrhs * (double)p->npairs * K;
    if (mfma_vu && p->smax_x <= kLeafMfma && ((K << l0) % 16) == 0) {
      // MFMA leaf product, 64-column chunks
      const int R = K << l0;
      const int nchu = (nrhs + 63) / 64;
      x.mfma = true;
      x.lds = ((size_t)R * (kLeafMfma + 1) + (size_t)4 * kLeafMfma * 64) * sizeof(VT);
      x.nblocks = p->nleaf * nchu;
      // after per-pair-rank stages the rows past each pair's rank are not
      // written, and not read here
      x.u = UDesc{w[cur], u, ldu, p->d_perm_x, p->d_xoff, p->d_ubar, l0, K, nrhs, 64, nchu,
                  p->smax_x, 1,
                  tight && R <= 256 ? p->d_prank + (size_t)(L - 2 * l0) * p->npairs : nullptr};
    } else {
      int NBu = NBo;
      while (NBu > 1 && (size_t)(1 << l0) * K * NBu * sizeof(VT) > kLdsBudget / 2) NBu /= 2;
      const int nchu = (nrhs + NBu - 1) / NBu;
      const size_t base = (size_t)(1 << l0) * K * NBu * sizeof(VT);
      if (base > kLdsBudget) {
        set_error("ibf_apply: leaf size too large for the apply kernels");
        return IBF_ERR_UNSUPPORTED;
      }
      // the factor rows are read from memory (each by the nbw lanes of its
      // point): staging them sized the LDS by the largest leaf and cost
      // occupancy (measured slower)
      const int stage_f = 0;
      x.lds = base;
      x.nblocks = p->nleaf * nchu;
      x.u = UDesc{w[cur], u, ldu, p->d_perm_x, p->d_xoff, p->d_ubar, l0, K, nrhs, NBu, nchu,
                  p->smax_x, stage_f, nullptr};
    }
    // the last stage launch writes all stored rows unless this U skips the
    // rows past each pair's rank
    if (!seq.empty() && seq.back().kind == kLaunchTight && !(x.mfma && x.u.prk))
      seq.back().t.A.rank_out = 0;
    seq.push_back(x);
  }
  return IBF_OK;
}

// Blocks of a kernel that fit on the device at once (occupancy x CUs), for
// persistent launches; cached per kernel and LDS size.
inline int resident_blocks(const void* func, size_t lds, int64_t* out, int block = kBlock) {
  static std::mutex mu;
  static std::map<std::pair<std::pair<const void*, size_t>, int>, int64_t> cache;
  int dev = 0;
  IBF_HIP_CHECK(hipGetDevice(&dev));
  const auto key = std::make_pair(std::make_pair(func, lds), dev * 4096 + block);
  {
    std::lock_guard<std::mutex> g(mu);
    const auto it = cache.find(key);
    if (it != cache.end()) {
      *out = it->second;
      return IBF_OK;
    }
  }
  int per_cu = 0, ncu = 0;
  IBF_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, func, block, lds));
  IBF_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t n = (int64_t)std::max(1, per_cu) * std::max(1, ncu);
  {
    std::lock_guard<std::mutex> g(mu);
    cache[key] = n;
  }
  *out = n;
  return IBF_OK;
}

template <typename VT, typename FT>
int launch_one(const Launch& x, hipStream_t s) {
  const dim3 grid((unsigned)x.nblocks), blk(kBlock);
  switch (x.kind) {
    case kLaunchV:
      if (x.mfma) {
        if constexpr (sizeof(VT) == 8)
          hipLaunchKernelGGL((k_apply_v_mfma<FT>), grid, blk, x.lds, s, x.v);
        break;
      }
#define IBF_LAUNCH_V(KTC) hipLaunchKernelGGL((k_apply_v<VT, FT, KTC>), grid, blk, x.lds, s, x.v)
      IBF_DISPATCH_KT(x.kt, IBF_LAUNCH_V);
#undef IBF_LAUNCH_V
      break;
    case kLaunchFused:
      if (x.mfma) {
        if constexpr (sizeof(VT) == 8) {
#define IBF_LAUNCH_FMNM(KTC, NBC, MIDC)                                               \
  {                                                                                   \
    int64_t nres = 0;                                                                 \
    const int rc = resident_blocks(reinterpret_cast<const void*>(                      \
                                       &k_apply_fused_mfma<VT, FT, KTC, NBC, MIDC>),   \
                                   x.lds, &nres);                                     \
    if (rc) return rc;                                                                \
    const dim3 pgrid((unsigned)std::min<int64_t>(x.nblocks, nres));                    \
    hipLaunchKernelGGL((k_apply_fused_mfma<VT, FT, KTC, NBC, MIDC>), pgrid, blk, x.lds, \
                       s, x.f, x.nblocks);                                            \
  }
#define IBF_LAUNCH_FMN(KTC, NBC)               \
  if (x.f.A.mid) IBF_LAUNCH_FMNM(KTC, NBC, true) \
  else IBF_LAUNCH_FMNM(KTC, NBC, false)
#define IBF_LAUNCH_FM32(KTC) IBF_LAUNCH_FMN(KTC, 32)
#define IBF_LAUNCH_FM16(KTC) IBF_LAUNCH_FMN(KTC, 16)
          if (x.f.A.NB == 32) {
            IBF_DISPATCH_KT(x.kt, IBF_LAUNCH_FM32);
          } else {
            IBF_DISPATCH_KT(x.kt, IBF_LAUNCH_FM16);
          }
#undef IBF_LAUNCH_FM16
#undef IBF_LAUNCH_FM32
#undef IBF_LAUNCH_FMN
#undef IBF_LAUNCH_FMNM
        }
      } else {
#define IBF_LAUNCH_FV(KTC) \
  hipLaunchKernelGGL((k_apply_fused<VT, FT, KTC>), grid, blk, x.lds, s, x.f)
        IBF_DISPATCH_KT(x.kt, IBF_LAUNCH_FV);
#undef IBF_LAUNCH_FV
      }
      break;
    case kLaunchMid:
      hipLaunchKernelGGL((k_apply_mid<VT, FT>), grid, blk, 0, s, x.m);
      break;
    case kLaunchTight:
      if constexpr (sizeof(VT) == 8) {
        const int tb = 64 << x.t.A.nst;
#define IBF_LAUNCH_TIGHT(KTC)                                                                  \
  {                                                                                            \
    int64_t nres = 0;                                                                          \
    const int rc = resident_blocks(reinterpret_cast<const void*>(&k_apply_tight<FT, KTC>),     \
                                   x.lds, &nres, tb);                                          \
    if (rc) return rc;                                                                         \
    const dim3 pgrid((unsigned)std::min<int64_t>(x.nblocks, nres));                             \
    hipLaunchKernelGGL((k_apply_tight<FT, KTC>), pgrid, dim3(tb), x.lds, s, x.t, x.nblocks);   \
  }
#define IBF_LAUNCH_TIGHT_SPLIT(KTC)                                                            \
  {                                                                                            \
    int64_t nres = 0;                                                                          \
    const int rc = resident_blocks(reinterpret_cast<const void*>(&k_apply_tight_split<KTC>),   \
                                   x.lds, &nres, tb);                                          \
    if (rc) return rc;                                                                         \
    const dim3 pgrid((unsigned)std::min<int64_t>(x.nblocks, nres));                             \
    hipLaunchKernelGGL((k_apply_tight_split<KTC>), pgrid, dim3(tb), x.lds, s, x.t, x.nblocks); \
  }
        if constexpr (std::is_same<FT, bf16x2c>::value) {
          if (x.split) {
            IBF_DISPATCH_KT(x.kt, IBF_LAUNCH_TIGHT_SPLIT);
            break;
          }
        }
        IBF_DISPATCH_KT(x.kt, IBF_LAUNCH_TIGHT);
#undef IBF_LAUNCH_TIGHT
#undef IBF_LAUNCH_TIGHT_SPLIT
      }
      break;
    default:
      if (x.mfma) {
        if constexpr (sizeof(VT) == 8)
          hipLaunchKernelGGL((k_apply_u_mfma<FT>), grid, blk, x.lds, s, x.u);
        break;
      }
      hipLaunchKernelGGL((k_apply_u<VT, FT>), grid, blk, x.lds, s, x.u);
      break;
  }
  IBF_HIP_CHECK(hipGetLastError());
  return IBF_OK;
}

template <typename VT, typename FT>
int apply_t(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs,
            hipStream_t s, ibf_profile* prof, void* const* ws = nullptr) {
  // the launch list is rebuilt per call into a per-thread vector whose
  // capacity persists (no host allocation once it has grown)
  thread_local std::vector<Launch> seq;
  int rc;
  if ((rc = make_schedule<VT, FT>(p, g, ldg, u, ldu, (int)nrhs, seq, false, ws))) return rc;
  LaunchTimer T(prof, s);
  for (const Launch& x : seq) {
    if ((rc = T.begin())) return rc;
    if ((rc = launch_one<VT, FT>(x, s))) return rc;
    if ((rc = T.end(launch_name(x), x.flops, x.bytes, x.vec_bytes))) return rc;
  }
  return T.finish();
}

// ---------------------------------------------------------------------------
// Batched apply of many plans (uneven sizes and RHS counts).  Phase i of the
// batch holds launch i of every plan's sequence that has one: V for all, then
// the fused stage groups in order, then U for all (a plan with fewer groups
// waits for the U phase).  Each phase is one launch over the concatenated
// blocks of its plans; a block finds its plan by binary search over the
// per-plan block offsets.  The descriptors live in a device table written
// before each apply, so a captured graph of the phase launches replays for new
// vectors of the same RHS counts without recapture.
// ---------------------------------------------------------------------------
struct BatchPhase {
  LaunchKind kind;
  bool mfma;
  int nb;                                                    // MFMA stage chunk width
  int kt, count;
  size_t lds;
  int64_t nblocks;
  size_t desc_off, boff_off;                                 // byte offsets in the table
};

}  // namespace
}  // namespace ibf

struct ibf_batch_s {
  std::vector<ibf_plan_t> plans;
  int device = 0, precision = 0;
  hipStream_t cap = nullptr;                                 // capture stream
  void* d_table = nullptr;
  void* h_table = nullptr;                                   // pinned staging
  size_t table_cap = 0;
  hipEvent_t table_ev = nullptr;
  bool table_pending = false;
  std::vector<ibf::BatchPhase> phases;
  std::vector<int64_t> graph_key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace ibf {
namespace {

inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

template <typename VT, typename FT>
int launch_phase(const ibf_batch_s* b, const BatchPhase& ph, hipStream_t s) {
  const char* base = static_cast<const char*>(b->d_table);
  const int64_t* boff = reinterpret_cast<const int64_t*>(base + ph.boff_off);
  const dim3 grid((unsigned)ph.nblocks), blk(kBlock);
  switch (ph.kind) {
    case kLaunchV: {
      const VDesc* ds = reinterpret_cast<const VDesc*>(base + ph.desc_off);
      if (ph.mfma) {
        if constexpr (sizeof(VT) == 8)
          hipLaunchKernelGGL((k_batch_v_mfma<FT>), grid, blk, ph.lds, s, ds, boff, ph.count);
        break;
      }
#define IBF_LAUNCH_BV(KTC) \
  hipLaunchKernelGGL((k_batch_v<VT, FT, KTC>), grid, blk, ph.lds, s, ds, boff, ph.count)
      IBF_DISPATCH_KT(ph.kt, IBF_LAUNCH_BV);
#undef IBF_LAUNCH_BV
      break;
    }
    case kLaunchFused: {
      const FusedDesc* ds = reinterpret_cast<const FusedDesc*>(base + ph.desc_off);
      if (ph.mfma) {
        if constexpr (sizeof(VT) == 8) {
#define IBF_LAUNCH_BFM32(KTC)                                                           \
  hipLaunchKernelGGL((k_batch_fused_mfma<VT, FT, KTC, 32>), grid, blk, ph.lds, s, ds, boff, \
                     ph.count)
#define IBF_LAUNCH_BFM16(KTC)                                                           \
  hipLaunchKernelGGL((k_batch_fused_mfma<VT, FT, KTC, 16>), grid, blk, ph.lds, s, ds, boff, \
                     ph.count)
          if (ph.nb == 32) {
            IBF_DISPATCH_KT(ph.kt, IBF_LAUNCH_BFM32);
          } else {
            IBF_DISPATCH_KT(ph.kt, IBF_LAUNCH_BFM16);
          }
#undef IBF_LAUNCH_BFM16
#undef IBF_LAUNCH_BFM32
        }
      } else {
#define IBF_LAUNCH_BFV(KTC) \
  hipLaunchKernelGGL((k_batch_fused<VT, FT, KTC>), grid, blk, ph.lds, s, ds, boff, ph.count)
        IBF_DISPATCH_KT(ph.kt, IBF_LAUNCH_BFV);
#undef IBF_LAUNCH_BFV
      }
      break;
    }
    case kLaunchU: {
      const UDesc* ds = reinterpret_cast<const UDesc*>(base + ph.desc_off);
      if (ph.mfma) {
        if constexpr (sizeof(VT) == 8)
          hipLaunchKernelGGL((k_batch_u_mfma<FT>), grid, blk, ph.lds, s, ds, boff, ph.count);
        break;
      }
      hipLaunchKernelGGL((k_batch_u<VT, FT>), grid, blk, ph.lds, s, ds, boff, ph.count);
      break;
    }
    default:
      set_error("ibf_apply_batch: internal error (unexpected launch kind)");
      return IBF_ERR_DEVICE;
  }
  IBF_HIP_CHECK(hipGetLastError());
  return IBF_OK;
}

template <typename VT, typename FT>
int apply_batch_t(ibf_batch_s* b, const void* const* g, const int64_t* ldg, void* const* u,
                  const int64_t* ldu, const int64_t* nrhs, int use_graph, hipStream_t s) {
  const int count = (int)b->plans.size();
  std::vector<std::vector<Launch>> seqs(count);
  int rc;
  size_t nmax = 0;
  for (int i = 0; i < count; ++i) {
    if ((rc = make_schedule<VT, FT>(b->plans[i], g[i], ldg[i], u[i], ldu[i], (int)nrhs[i],
                                    seqs[i], true)))
      return rc;
    for (const Launch& x : seqs[i])
      if (x.kind == kLaunchMid) {
        set_error("ibf_apply_batch: plans built with the sweep-in are not batched");
        return IBF_ERR_UNSUPPORTED;
      }
    nmax = std::max(nmax, seqs[i].size());
  }
  // phase membership: V (launch 0), fused launch j (1..), U (last launch)
  std::vector<std::vector<const Launch*>> members;
  auto add_phase_members = [&](auto pick) {
    // one phase per kernel variant: vector, MFMA (V, U, or stages with 32- or
    // 16-column chunks)
    std::vector<const Launch*> mv, mf32, mf16;
    for (int i = 0; i < count; ++i) {
      const Launch* x = pick(seqs[i]);
      if (!x) continue;
      if (!x->mfma) mv.push_back(x);
      else if (x->kind == kLaunchFused && x->f.A.NB == 16) mf16.push_back(x);
      else mf32.push_back(x);
    }
    if (!mv.empty()) members.push_back(mv);
    if (!mf32.empty()) members.push_back(mf32);
    if (!mf16.empty()) members.push_back(mf16);
  };
  add_phase_members([](const std::vector<Launch>& q) { return &q.front(); });
  for (size_t j = 1; j + 1 < nmax; ++j)
    add_phase_members([j](const std::vector<Launch>& q) -> const Launch* {
      return j + 1 < q.size() ? &q[j] : nullptr;
    });
  add_phase_members([](const std::vector<Launch>& q) { return &q.back(); });
  // Table layout.  A phase runs every member at the phase's largest KT, so
  // the members' LDS footprints are recomputed at that KT: the V body stages
  // Vbar rows KT wide (when they fit), the fused body reads KT-wide rows.
  int lmax = 0;
  if ((rc = lds_limit(b->device, &lmax))) return rc;
  std::vector<BatchPhase> phases;
  std::vector<std::vector<Launch>> adj(members.size());
  size_t bytes = 0;
  for (size_t q = 0; q < members.size(); ++q) {
    const auto& m = members[q];
    BatchPhase ph{};
    ph.kind = m[0]->kind;
    ph.mfma = m[0]->mfma;
    ph.nb = m[0]->kind == kLaunchFused ? m[0]->f.A.NB : 0;
    ph.count = (int)m.size();
    const size_t dsz = ph.kind == kLaunchV ? sizeof(VDesc)
                       : ph.kind == kLaunchU ? sizeof(UDesc) : sizeof(FusedDesc);
    ph.desc_off = bytes;
    bytes = align16(bytes + dsz * m.size());
    ph.boff_off = bytes;
    bytes = align16(bytes + sizeof(int64_t) * (m.size() + 1));
    for (const Launch* x : m) {
      ph.kt = std::max(ph.kt, x->kt);
      ph.nblocks += x->nblocks;
    }
    for (const Launch* x : m) {
      Launch y = *x;
      if (y.kind == kLaunchV && !y.mfma) {
        const size_t base = (size_t)y.v.smax * y.v.NB * sizeof(VT);
        const size_t fac = (size_t)y.v.smax * ((size_t)1 << y.v.l0) * ph.kt * sizeof(VT);
        y.v.stage_f = base + fac <= kLdsBudget ? 1 : 0;
        y.lds = base + (y.v.stage_f ? fac : 0);
      } else if (y.kind == kLaunchFused && y.mfma) {
        const FusedArgs& A = y.f.A;
        const size_t nv = (size_t)kBlock / (size_t)A.NB;     // virtual slots a block
        y.lds = (nv * ((size_t)A.kmaxg * A.NB + (size_t)2 * A.kmaxg * ph.kt + 20) + 2 * ph.kt) *
                sizeof(VT);
      }
      ph.lds = std::max(ph.lds, y.lds);
      adj[q].push_back(y);
    }
    if (ph.nblocks > 0x7fffffff || ph.lds > (size_t)lmax) {
      set_error("ibf_apply_batch: a phase exceeds the grid or LDS limits of one launch");
      return IBF_ERR_UNSUPPORTED;
    }
    phases.push_back(ph);
  }
  if (bytes > b->table_cap) {
    if (b->table_pending) IBF_HIP_CHECK(hipEventSynchronize(b->table_ev));
    b->table_pending = false;
    if (b->d_table) IBF_HIP_CHECK(ibf::dev_free(b->d_table));
    if (b->h_table) IBF_HIP_CHECK(hipHostFree(b->h_table));
    b->d_table = b->h_table = nullptr;
    b->table_cap = 0;
    IBF_HIP_CHECK(ibf::dev_malloc(&b->d_table, bytes));
    IBF_HIP_CHECK(hipHostMalloc(&b->h_table, bytes, hipHostMallocDefault));
    b->table_cap = bytes;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_key.clear();
  }
  // the previous apply's table copy must have left the staging buffer
  if (b->table_pending) IBF_HIP_CHECK(hipEventSynchronize(b->table_ev));
  char* h = static_cast<char*>(b->h_table);
  for (size_t q = 0; q < phases.size(); ++q) {
    const auto& m = adj[q];
    int64_t* boff = reinterpret_cast<int64_t*>(h + phases[q].boff_off);
    int64_t acc = 0;
    for (size_t i = 0; i < m.size(); ++i) {
      boff[i] = acc;
      acc += m[i].nblocks;
      char* dst = h + phases[q].desc_off;
      switch (phases[q].kind) {
        case kLaunchV: reinterpret_cast<VDesc*>(dst)[i] = m[i].v; break;
        case kLaunchU: reinterpret_cast<UDesc*>(dst)[i] = m[i].u; break;
        default: reinterpret_cast<FusedDesc*>(dst)[i] = m[i].f; break;
      }
    }
    boff[m.size()] = acc;
  }
  IBF_HIP_CHECK(hipMemcpyAsync(b->d_table, b->h_table, bytes, hipMemcpyHostToDevice, s));
  IBF_HIP_CHECK(hipEventRecord(b->table_ev, s));
  b->table_pending = true;
  b->phases = phases;
  if (!use_graph) {
    for (const BatchPhase& ph : phases)
      if ((rc = launch_phase<VT, FT>(b, ph, s))) return rc;
    return IBF_OK;
  }
  // graph of the phase launches, keyed by everything that shapes them
  std::vector<int64_t> key;
  key.push_back((int64_t)(uintptr_t)b->d_table);
  for (const BatchPhase& ph : phases) {
    key.push_back(ph.kind);
    key.push_back(ph.mfma);
    key.push_back(ph.kt);
    key.push_back(ph.count);
    key.push_back((int64_t)ph.lds);
    key.push_back(ph.nblocks);
    key.push_back((int64_t)ph.desc_off);
    key.push_back((int64_t)ph.boff_off);
  }
  if (!b->exec || key != b->graph_key) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_key.clear();
    IBF_HIP_CHECK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int lrc = IBF_OK;
    for (const BatchPhase& ph : phases)
      if ((lrc = launch_phase<VT, FT>(b, ph, b->cap))) break;
    hipGraph_t gr = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->cap, &gr);
    if (lrc) {
      if (gr) (void)hipGraphDestroy(gr);
      return lrc;
    }
    IBF_HIP_CHECK(ec);
    b->graph = gr;
    IBF_HIP_CHECK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_key = key;
  }
  IBF_HIP_CHECK(hipGraphLaunch(b->exec, s));
  return IBF_OK;
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

// ---------------------------------------------------------------------------
// Allocation-free apply: the ping-pong coefficient buffers live in a static
// device array (one copy per device, held until the process ends) instead of
// the plan's workspace.  Host code never uses the array's name as a device
// address: its address on each device comes from hipGetSymbolAddress, taken
// once per device with that device current.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratch = (size_t)128 << 20;          // bytes, both buffers
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

int scratch_ptr(int device, unsigned char** out) {
  static std::mutex mu;
  static unsigned char* ptrs[64] = {nullptr};
  if (device < 0 || device >= 64) {
    set_error("ibf_apply_noalloc: device ordinal out of range");
    return IBF_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[device]) {
    void* ptr = nullptr;
    IBF_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    ptrs[device] = static_cast<unsigned char*>(ptr);
  }
  *out = ptrs[device];
  return IBF_OK;
}

int apply_plan_noalloc(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu,
                       int64_t nrhs, hipStream_t s) {
  IBF_HIP_CHECK(hipSetDevice(p->device));
  const size_t vb = complex_bytes(p->precision);
  int kmax = 1;
  for (int k : p->rank) kmax = std::max(kmax, k);
  for (int k : p->rank_in_g) kmax = std::max(kmax, k);
  for (int k : p->rank_in_h) kmax = std::max(kmax, k);
  const size_t half = (((size_t)p->npairs * kmax * (size_t)nrhs * vb) + 255) & ~(size_t)255;
  if (nrhs > (1 << 20) || 2 * half > kNoAllocScratch) {
    set_error("ibf_apply_noalloc: the coefficient buffers need " + std::to_string(2 * half) +
              " bytes, more than the " + std::to_string(kNoAllocScratch) +
              "-byte scratch array (use ibf_apply)");
    return IBF_ERR_INVALID_ARG;
  }
  unsigned char* base = nullptr;
  int rc;
  if ((rc = scratch_ptr(p->device, &base))) return rc;
  void* ws[2] = {base, base + half};
  switch (p->precision) {
    case IBF_FP64: return apply_t<double2, double2>(p, g, ldg, u, ldu, nrhs, s, nullptr, ws);
    case IBF_FP32: return apply_t<float2, float2>(p, g, ldg, u, ldu, nrhs, s, nullptr, ws);
    default: return apply_t<float2, bf16x2c>(p, g, ldg, u, ldu, nrhs, s, nullptr, ws);
  }
}

// The launch list a schedule produces (kernel, tile, grid, LDS, stage span
// and chunk width per launch): two knob settings with equal signatures run
// the same launches.
template <typename VT, typename FT>
int schedule_signature(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu,
                       int nrhs, std::vector<int64_t>& sig) {
  std::vector<Launch> seq;
  const int rc = make_schedule<VT, FT>(p, g, ldg, u, ldu, nrhs, seq);
  if (rc != IBF_OK) return rc;
  sig.clear();
  for (const Launch& x : seq) {
    sig.insert(sig.end(), {(int64_t)x.kind, (int64_t)x.kt, (int64_t)x.mfma, x.nblocks,
                           (int64_t)x.lds});
    if (x.kind == kLaunchFused) sig.insert(sig.end(), {x.f.A.l_start, x.f.A.nst, x.f.A.NB});
    if (x.kind == kLaunchTight)
      sig.insert(sig.end(), {x.t.A.l_start, x.t.A.nst, 64, (int64_t)x.split});
  }
  return IBF_OK;
}

int schedule_signature(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu,
                       int nrhs, std::vector<int64_t>& sig) {
  switch (p->precision) {
    case IBF_FP64: return schedule_signature<double2, double2>(p, g, ldg, u, ldu, nrhs, sig);
    case IBF_FP32: return schedule_signature<float2, float2>(p, g, ldg, u, ldu, nrhs, sig);
    default: return schedule_signature<float2, bf16x2c>(p, g, ldg, u, ldu, nrhs, sig);
  }
}

// Time every distinct candidate schedule for nrhs right-hand sides
// (interleaved rounds, median per candidate) and keep the fastest for later
// applies; the default rule is kept unless another is 2% faster.
int tune_plan(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs,
              hipStream_t s, ibf_tuning* best, ibf_tuning* dflt) {
  IBF_HIP_CHECK(hipSetDevice(p->device));
  std::vector<Tuning> cand;
  cand.push_back(Tuning{0, 0, 0, 0});                         // the default rule first
  cand.push_back(Tuning{0, 0, 0, 1});
  cand.push_back(Tuning{0, 0, 0, 2});
  cand.push_back(Tuning{1, 0, 0, 0});
  cand.push_back(Tuning{1, 0, 2, 0});
  if (p->precision != IBF_FP64) {
    const int chunks[2] = {32, 16};
    for (int c : chunks) {
      if (c == 32 && nrhs <= 16) continue;                    // half-empty 32-column chunks
      cand.push_back(Tuning{2, c, 0, 0});
      cand.push_back(Tuning{2, c, 0, 1});
      cand.push_back(Tuning{2, c, 0, 2});
      cand.push_back(Tuning{2, c, 3, 0});
      cand.push_back(Tuning{2, c, 2, 0});
    }
    if (p->d_prank && nrhs > 8) {                             // stages at per-pair ranks
      cand.push_back(Tuning{3, 0, 0, 0});
      cand.push_back(Tuning{3, 0, 3, 0});
      cand.push_back(Tuning{3, 0, 2, 0});
      if (p->precision == IBF_BF16X2) {                      // BF16 split products
        cand.push_back(Tuning{4, 0, 0, 0});
        cand.push_back(Tuning{4, 0, 3, 0});
        cand.push_back(Tuning{4, 0, 2, 0});
      }
    }
  }
  // the plan leaves trial mode and the events are released on every exit
  struct TrialOff {
    ibf_plan_t p;
    ~TrialOff() { p->trial_on = false; }
  } off{p};
  {  // drop knob settings that produce a launch list seen before
    std::vector<std::vector<int64_t>> seen;
    std::vector<Tuning> uniq;
    for (const Tuning& c : cand) {
      p->trial = c;
      p->trial_on = true;
      std::vector<int64_t> sig;
      const int r = schedule_signature(p, g, ldg, u, ldu, (int)nrhs, sig);
      if (r != IBF_OK) {
        if (uniq.empty()) return r;                           // the default rule must plan
        continue;
      }
      if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
      seen.push_back(sig);
      uniq.push_back(c);
    }
    cand.swap(uniq);
  }
  struct Guard {
    ibf_plan_t p;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Guard() {
      p->trial_on = false;
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } gd{p};
  IBF_HIP_CHECK(hipEventCreate(&gd.e0));
  IBF_HIP_CHECK(hipEventCreate(&gd.e1));
  const size_t nc = cand.size();
  // one untimed apply per candidate (workspace, clocks), then interleaved
  // timed rounds so that no candidate profits from coming later
  std::vector<bool> ok(nc, false);
  for (size_t i = 0; i < nc; ++i) {
    p->trial = cand[i];
    p->trial_on = true;
    const int r = apply_plan(p, g, ldg, u, ldu, nrhs, s);
    if (i == 0 && r != IBF_OK) return r;                      // the default rule must run
    ok[i] = r == IBF_OK;
  }
  constexpr int kRounds = 5;
  std::vector<std::vector<float>> t(nc);
  for (int k = 0; k < kRounds; ++k) {
    for (size_t i = 0; i < nc; ++i) {
      if (!ok[i]) continue;
      p->trial = cand[i];
      p->trial_on = true;
      IBF_HIP_CHECK(hipEventRecord(gd.e0, s));
      const int r = apply_plan(p, g, ldg, u, ldu, nrhs, s);
      if (r != IBF_OK) {
        if (i == 0) return r;
        ok[i] = false;
        continue;
      }
      IBF_HIP_CHECK(hipEventRecord(gd.e1, s));
      IBF_HIP_CHECK(hipEventSynchronize(gd.e1));
      float ms = 0;
      IBF_HIP_CHECK(hipEventElapsedTime(&ms, gd.e0, gd.e1));
      t[i].push_back(ms);
    }
  }
  p->trial_on = false;
  std::vector<float> med(nc, 0.f);
  for (size_t i = 0; i < nc; ++i) {
    if (!ok[i]) continue;
    std::vector<float> v = t[i];
    std::sort(v.begin(), v.end());
    med[i] = v[v.size() / 2];
  }
  // another candidate replaces the default rule only when it is 2% faster
  int ibest = 0;
  for (size_t i = 1; i < nc; ++i)
    if (ok[i] && med[i] < med[ibest] && med[i] < 0.98f * med[0]) ibest = (int)i;
  const float tbest = med[ibest], tdef = med[0];
  p->tuned[nrhs] = cand[ibest];
  if (best)
    *best = ibf_tuning{cand[ibest].path, cand[ibest].chunk, cand[ibest].max_fused, tbest,
                       cand[ibest].split};
  if (dflt) *dflt = ibf_tuning{0, 0, 0, tdef, 0};
  // leave u holding the product of the chosen schedule
  return apply_plan(p, g, ldg, u, ldu, nrhs, s);
}

}  // namespace ibf

extern "C" {

int ibf_tune(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs,
             void* stream, ibf_tuning* best, ibf_tuning* dflt) {
  if (!p) {
    ibf::set_error("ibf_tune: null plan");
    return IBF_ERR_INVALID_ARG;
  }
  if (!p->built) {
    ibf::set_error("ibf_tune: plan not built");
    return IBF_ERR_NOT_BUILT;
  }
  if (!g || !u || nrhs < 1 || ldg < p->nxi || ldu < p->nx) {
    ibf::set_error("ibf_tune: null vector, nrhs < 1 or leading dimension too small");
    return IBF_ERR_INVALID_ARG;
  }
  if (p->dim != 1) {
    ibf::set_error("ibf_tune: the schedule tuner is provided for 1-D plans");
    return IBF_ERR_UNSUPPORTED;
  }
  return ibf::tune_plan(p, g, ldg, u, ldu, nrhs, (hipStream_t)stream, best, dflt);
}

int ibf_apply_noalloc(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu,
                      int64_t nrhs, void* stream) {
  if (!p) {
    ibf::set_error("ibf_apply_noalloc: null plan");
    return IBF_ERR_INVALID_ARG;
  }
  if (!p->built) {
    ibf::set_error("ibf_apply_noalloc: plan not built");
    return IBF_ERR_NOT_BUILT;
  }
  if (!g || !u || nrhs < 1 || ldg < p->nxi || ldu < p->nx) {
    ibf::set_error("ibf_apply_noalloc: null vector, nrhs < 1 or leading dimension too small");
    return IBF_ERR_INVALID_ARG;
  }
  if (p->dim != 1) {
    ibf::set_error("ibf_apply_noalloc: provided for dim-1 plans");
    return IBF_ERR_UNSUPPORTED;
  }
  return ibf::apply_plan_noalloc(p, g, ldg, u, ldu, nrhs, (hipStream_t)stream);
}

int ibf_set_tuning(ibf_plan_t p, int64_t nrhs, const ibf_tuning* t) {
  if (!p || nrhs < 1) {
    ibf::set_error("ibf_set_tuning: null plan or nrhs < 1");
    return IBF_ERR_INVALID_ARG;
  }
  if (p->dim != 1) {
    ibf::set_error("ibf_set_tuning: schedules are provided for 1-D plans");
    return IBF_ERR_UNSUPPORTED;
  }
  if (!t) {
    p->tuned.erase(nrhs);
    return IBF_OK;
  }
  if (t->path < 0 || t->path > 4 || (t->chunk != 0 && t->chunk != 16 && t->chunk != 32) ||
      t->max_fused < 0 || t->split < 0 || t->split > 2) {
    ibf::set_error(
        "ibf_set_tuning: path outside 0..4, chunk not 0/16/32, max_fused < 0 or split outside "
        "0..2");
    return IBF_ERR_INVALID_ARG;
  }
  if ((t->path == 2 || t->path == 3) && p->precision == IBF_FP64) {
    ibf::set_error("ibf_set_tuning: no MFMA stage kernel for FP64 plans");
    return IBF_ERR_UNSUPPORTED;
  }
  if (t->path == 4 && p->precision != IBF_BF16X2) {
    ibf::set_error("ibf_set_tuning: BF16 split products (path 4) need a BF16X2 plan");
    return IBF_ERR_UNSUPPORTED;
  }
  p->tuned[nrhs] = ibf::Tuning{t->path, t->chunk, t->max_fused, t->split};
  return IBF_OK;
}

int ibf_batch_create(const ibf_plan_t* plans, int count, ibf_batch_t* out) {
  if (!out) {
    ibf::set_error("ibf_batch_create: NULL output");
    return IBF_ERR_INVALID_ARG;
  }
  *out = nullptr;
  if (!plans || count < 1) {
    ibf::set_error("ibf_batch_create: no plans");
    return IBF_ERR_INVALID_ARG;
  }
  for (int i = 0; i < count; ++i) {
    if (!plans[i] || !plans[i]->built) {
      ibf::set_error("ibf_batch_create: plan " + std::to_string(i) + " is NULL or not built");
      return IBF_ERR_INVALID_ARG;
    }
    if (plans[i]->precision != plans[0]->precision || plans[i]->device != plans[0]->device) {
      ibf::set_error("ibf_batch_create: plans differ in precision or device");
      return IBF_ERR_INVALID_ARG;
    }
  }
  ibf_batch_s* b = new ibf_batch_s;
  b->plans.assign(plans, plans + count);
  b->device = plans[0]->device;
  b->precision = plans[0]->precision;
  auto fail = [&](hipError_t e) {
    ibf::set_error(std::string("ibf_batch_create: ") + hipGetErrorString(e));
    ibf_batch_destroy(b);
    return IBF_ERR_DEVICE;
  };
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return fail(e);
  if ((e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) return fail(e);
  if ((e = hipEventCreateWithFlags(&b->table_ev, hipEventDisableTiming)) != hipSuccess)
    return fail(e);
  *out = b;
  return IBF_OK;
}

int ibf_apply_batch(ibf_batch_t b, const void* const* g, const int64_t* ldg, void* const* u,
                    const int64_t* ldu, const int64_t* nrhs, int flags, void* hip_stream) {
  if (!b || !g || !ldg || !u || !ldu || !nrhs) {
    ibf::set_error("ibf_apply_batch: NULL argument");
    return IBF_ERR_INVALID_ARG;
  }
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const ibf_plan_t p = b->plans[i];
    if (!g[i] || !u[i] || nrhs[i] < 1 || nrhs[i] > (1 << 20) || ldg[i] < p->nxi ||
        ldu[i] < p->nx) {
      ibf::set_error("ibf_apply_batch: bad vector, leading dimension or nrhs for plan " +
                     std::to_string(i));
      return IBF_ERR_INVALID_ARG;
    }
  }
  IBF_HIP_CHECK(hipSetDevice(b->device));
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int graph = (flags & IBF_BATCH_GRAPH) ? 1 : 0;
  switch (b->precision) {
    case IBF_FP64:
      return ibf::apply_batch_t<double2, double2>(b, g, ldg, u, ldu, nrhs, graph, s);
    case IBF_FP32:
      return ibf::apply_batch_t<float2, float2>(b, g, ldg, u, ldu, nrhs, graph, s);
    default:
      return ibf::apply_batch_t<float2, ibf::bf16x2c>(b, g, ldg, u, ldu, nrhs, graph, s);
  }
}

int ibf_batch_destroy(ibf_batch_t b) {
  if (!b) return IBF_OK;
  (void)hipSetDevice(b->device);
  if (b->table_pending && b->table_ev) (void)hipEventSynchronize(b->table_ev);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->table_ev) (void)hipEventDestroy(b->table_ev);
  if (b->d_table) (void)ibf::dev_free(b->d_table);
  if (b->h_table) (void)hipHostFree(b->h_table);
  delete b;
  return IBF_OK;
}

}  // extern "C"
