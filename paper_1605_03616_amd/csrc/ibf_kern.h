// Shared declarations of the construction kernels' translation units:
// device helpers used by several kernels and the host launchers of the
// r-templated compression kernels (dispatched on the runtime r).
#pragma once

#include "ibf_device.h"

namespace ibf {
namespace kern {

constexpr int kBlock = 256;

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
  const int* caps;     // host: fixed-rank cap per level l0..L-l0 (null: none)
  int cap_at(int level) const { return caps ? caps[level - geo.l0] : 0; }
};

template <int R>
constexpr int group_for() { return R <= 8 ? 16 : 32; }

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


// sweep-out (ibf_sweep.hip)
void middle(int R, const SweepArgs& A, double2* C, double2* Rm, int* rk, hipStream_t s);
void sweep_g(int R, const SweepArgs& A, int l, const double2* Cin, double2* Cout, double2* stage,
             const int* rk_in, int* rk_out, unsigned long long* nnz, hipStream_t s);
void sweep_h(int R, const SweepArgs& A, int l, const double2* Rin, double2* Rout, double2* stage,
             const int* rk_in, int* rk_out, unsigned long long* nnz, hipStream_t s);
// sweep-in (ibf_sweepin.hip)
void sweepin_u(int R, const Geo& geo, double tol, const int32_t* xoff, const double2* ub,
               double2* ud, double2* cb, int* rk, int* rank_max, hipStream_t s);
void sweepin_v(int R, const Geo& geo, double tol, const int32_t* xioff, const double2* vb,
               double2* vd, double2* rb, int* rk, int* rank_max, hipStream_t s);
void sweepin_g(int R, const Geo& geo, double tol, int l, const double2* cin, double2* cout,
               double2* stage, const int* rkp, int* rk, int* rank_max, unsigned long long* nnz,
               hipStream_t s);
void sweepin_h(int R, const Geo& geo, double tol, int l, const double2* rin, double2* rout,
               double2* stage, const int* rkp, int* rk, int* rank_max, unsigned long long* nnz,
               hipStream_t s);

}  // namespace kern
}  // namespace ibf
