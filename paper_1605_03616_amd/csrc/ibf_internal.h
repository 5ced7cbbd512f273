// Internal declarations shared by the planner, the build and the apply code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/ibf.h"

namespace ibf {

constexpr int kMaxR = 16;          // Chebyshev points per box supported on device

// Apply schedule knobs (ibf_tune): path 0 default rule / 1 vector / 2 MFMA
// stage kernels, MFMA chunk width (0: by nrhs), most stages fused (0: as LDS
// allows), where fused groups end (0: as they fit; 1: before a stage whose
// own block rows fit a smaller tile; 2: before any stage of another tile)
struct Tuning {
  int path = 0, chunk = 0, max_fused = 0, split = 0;
};
constexpr int kMaxParams = 6;
// Bytes allocated past a stage's stored blocks and past its quad records:
// the per-pair-rank stage kernels read whole two-row windows (and rows past
// a pair's rank) without clamping, and clamped record loads of a stage with
// input rank 0 start at the buffer; what they read there is never used.
constexpr size_t kStageSlack = 8192;

struct PhaseDesc {
  int kind;
  double p[kMaxParams];
  int amp;                 // IBF_AMP_* (amplitude of eqn:FIO; enters the switch blocks only)
  double q[kMaxParams];
};

// Device-side geometry of one tree pair: T_X on [0,1), T_Omega on
// [lo, lo + W).  Box centres and widths are closed-form per level.
struct Geo {
  int L, l0, h, r;
  double lo, W;
};

void set_error(const std::string& msg);

// Device memory owned by plans and batches: from the caller's allocator when
// one is installed (ibf_set_allocator), else hipMalloc / hipFree.  A block is
// released through the allocator that made it.
hipError_t dev_malloc_raw(void** ptr, size_t bytes);
hipError_t dev_free(void* ptr);
template <typename T>
inline hipError_t dev_malloc(T** ptr, size_t bytes) {
  return dev_malloc_raw(reinterpret_cast<void**>(ptr), bytes);
}

// Stored factors of one compressed level stage, in the plan's precision.
struct Stage {
  int level_out;     // output coefficient level (l0+1 .. L-l0)
  int k_out, k_in;   // stored ranks
  int k_ld;          // row length: k_out rounded up to even, zero-padded
  void* blk;         // [pair][c k_in + s][k_ld] complex (input-major rows)
  size_t bytes;
  int64_t nnz;       // unpadded entries (each block at its own ranks)
  // BF16X2 plans with per-pair ranks: the same blocks for the BF16 split
  // products, [pair][c][quad q < ceil(k_in / 4)][float f < 2 k_ld] 16-byte
  // records {bf16 hi of rows 4q .. 4q+3, bf16 lo of the same rows} of float f
  // (re or im of entry f / 2; rows past k_in are zero); null otherwise
  void* qblk = nullptr;
  size_t qbytes = 0;
};

}  // namespace ibf

namespace ibf {
struct Mibf2D;            // 2-D multiscale plan (ibf2d.hip)
}

struct ibf_plan_s {
  ibf::Mibf2D* mibf = nullptr;   // dim == 2: the corona boxes and the centre block
  // descriptor
  int dim = 1;
  int64_t nx = 0, nxi = 0;
  int device = 0;
  ibf::PhaseDesc phase{};
  int r = 0, leaf = 0, precision = 0, sweep_in = 0;
  double tol = 0;
  // learned order (r <= 0 in the descriptor): chosen by ibf_build from the
  // predictor (device parameters, not owned), r = 12 without one
  bool learned = false;
  const float* predictor = nullptr;
  int predictor_hidden = 0;
  double target_tol = 0;       // the accuracy target of a learned plan
  int sweep_auto = 0;          // sweep_in = -1: decided when r is known
  std::vector<int> caps;       // fixed-rank caps per level l0..L-l0 (empty: none)
  ibf::Geo geo{};
  int64_t npairs = 0, nleaf = 0;

  // host geometry (sorted order)
  std::vector<double> xs, xis;
  std::vector<int32_t> perm_x, perm_xi;   // sorted position -> caller index
  std::vector<int32_t> xoff, xioff;       // leaf CSR offsets (nleaf + 1)
  std::vector<int32_t> xleaf, xileaf;     // leaf of each sorted point
  int smax_x = 0, smax_xi = 0;

  // device copies of the geometry
  double *d_xs = nullptr, *d_xis = nullptr;
  int32_t *d_perm_x = nullptr, *d_perm_xi = nullptr;
  int32_t *d_xoff = nullptr, *d_xioff = nullptr;
  int32_t *d_xleaf = nullptr, *d_xileaf = nullptr;

  // factors
  bool built = false;
  std::vector<int> rank;            // per coefficient level l0..L-l0 (index l - l0)
  std::vector<int> rank_in_g, rank_in_h;  // sweep-in ranks (same indexing)
  std::vector<ibf::Stage> stages;   // H stages then G stages, in apply order
  void* d_vbar = nullptr;           // [xi point][2^l0][K_l0]
  size_t vbar_bytes = 0;
  void* d_ubar = nullptr;           // [x point][2^l0][K_{L-l0}]
  size_t ubar_bytes = 0;
  void* d_mdot = nullptr;           // sweep-in middle block [pair][KG][KH] or null
  uint8_t* d_prank = nullptr;       // sweep-out rank of every pair: [level l0..L-l0][pair]
                                    // (plans without the sweep-in; read by the stage kernels
                                    // that skip each block's zero padding)
  size_t mdot_bytes = 0;
  int k_vbar = 0, k_ubar = 0, k_mid_g = 0, k_mid_h = 0;
  int64_t nnz_vbar = 0, nnz_ubar = 0;   // unpadded outer-factor entries
  int64_t nnz_prelim = 0, nnz_opt = 0, nnz_stored = 0;
  double build_ms = 0;

  // apply workspace (ping-pong coefficient buffers)
  void* d_work[2] = {nullptr, nullptr};
  size_t work_bytes = 0;
  // tuned schedules per nrhs (ibf_tune), and the candidate under trial
  std::map<int64_t, ibf::Tuning> tuned;
  ibf::Tuning trial{};
  bool trial_on = false;
  // the adjoint (ibf_apply_adjoint): a plan over the transposed pair labels
  // that shares this plan's point maps and owns conjugate-transposed copies
  // of the factors; made on the first adjoint apply, dropped with the factors
  ibf_plan_s* adj = nullptr;
};

namespace ibf {
int build_plan(ibf_plan_t p, hipStream_t s);
int apply_plan(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu,
               int64_t nrhs, hipStream_t s, ibf_profile* prof = nullptr);
int dense_apply(const PhaseDesc& ph, const double* x, int64_t nx, const double* xi, int64_t nxi,
                const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs, hipStream_t s);
// Quad records of a BF16X2 stage (Stage::qblk, allocated with the stage
// slack) from its stored blocks, on stream s.
int make_quad_records(Stage& st, int64_t npairs, hipStream_t s);
int dense_apply_2d(const PhaseDesc& ph, const double* x, int64_t nx, const double* xi,
                   int64_t nxi, const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs,
                   hipStream_t s);
int eval_kernel(const PhaseDesc& ph, const double* x, const double* xi,
                int64_t n, void* out, hipStream_t s);
int rel_error(const void* u, int64_t ldu, const void* ref, int64_t ldr, int64_t n, int64_t nrhs,
              int precision, double* out, hipStream_t s);
void free_factors(ibf_plan_t p);
void free_adjoint(ibf_plan_t p);
int apply_adjoint(ibf_plan_t p, const void* h, int64_t ldh, void* v, int64_t ldv, int64_t nrhs,
                  hipStream_t s);
// dim == 2 (multiscale IBF over coronal boxes)
int plan2d(const ibf_desc* d, ibf_plan_t* out);
int build2d(ibf_plan_t p, hipStream_t s);
int apply2d(ibf_plan_t p, const void* g, int64_t ldg, void* u, int64_t ldu, int64_t nrhs,
            hipStream_t s);
void free2d_factors(ibf_plan_t p);
void destroy2d(ibf_plan_t p);
void query2d(ibf_plan_t p, ibf_info* info);
size_t complex_bytes(int precision);
// the Chebyshev order and truncation of a dim-1 plan: sets r, tol, the
// preliminary entry count and the automatic sweep-in choice
void set_order(ibf_plan_t p, int r, double tol);
}  // namespace ibf

#define IBF_HIP_CHECK(expr)                                                   \
  do {                                                                        \
    hipError_t _e = (expr);                                                   \
    if (_e != hipSuccess) {                                                   \
      ibf::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));      \
      return (_e == hipErrorOutOfMemory) ? IBF_ERR_OOM : IBF_ERR_DEVICE;      \
    }                                                                         \
  } while (0)
