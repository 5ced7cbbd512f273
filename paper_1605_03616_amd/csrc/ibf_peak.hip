// Measured peaks of the device for the roofline fractions: a plain streaming
// copy (HBM read + write bandwidth) and a loop of the FP32 MFMA instruction
// the butterfly stage kernels issue (v_mfma_f32_4x4x1f32, 16 blocks), timed
// with HIP events on the caller's stream.  Measurement support only; no part
// of the factorization.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "ibf_internal.h"

namespace ibf {
namespace {

constexpr int kPeakBlock = 256;

// dst[i] = src[i] over n float4: a block copies kCopyPer x kPeakBlock
// consecutive float4, each thread kCopyPer of them a block width apart with
// all its loads in flight before the stores
constexpr int kCopyPer = 4;
__global__ __launch_bounds__(kPeakBlock) void k_peak_copy(const float4* __restrict__ src,
                                                          float4* __restrict__ dst, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * kPeakBlock * kCopyPer + threadIdx.x;
  float4 v[kCopyPer];
#pragma unroll
  for (int j = 0; j < kCopyPer; ++j) {
    const int64_t i = base + (int64_t)j * kPeakBlock;
    if (i < n) v[j] = src[i];
  }
#pragma unroll
  for (int j = 0; j < kCopyPer; ++j) {
    const int64_t i = base + (int64_t)j * kPeakBlock;
    if (i < n) dst[i] = v[j];
  }
}

// iters rounds of 8 independent MFMA accumulations per wave; the sum of the
// accumulators is stored so that nothing is dropped
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kPeakBlock) void k_peak_mfma(float* __restrict__ out, int iters,
                                                          float a0, float b0) {
  v4f acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
  const float a = a0 + 1e-7f * (float)(threadIdx.x & 3), b = b0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, acc[j], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace
}  // namespace ibf

extern "C" int ibf_measure_peak(int what, void* hip_stream, double* result) {
  if (!result || (what != IBF_PEAK_HBM_COPY && what != IBF_PEAK_MFMA_F32)) {
    ibf::set_error("ibf_measure_peak: NULL result or unknown measurement");
    return IBF_ERR_INVALID_ARG;
  }
  *result = 0.0;
  hipStream_t s = (hipStream_t)hip_stream;
  int dev = 0;
  IBF_HIP_CHECK(hipGetDevice(&dev));
  int ncu = 0;
  IBF_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  struct Res {
    void* a = nullptr;
    void* b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Res() {
      if (a) (void)ibf::dev_free(a);
      if (b) (void)ibf::dev_free(b);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } r;
  IBF_HIP_CHECK(hipEventCreate(&r.e0));
  IBF_HIP_CHECK(hipEventCreate(&r.e1));
  constexpr int kReps = 5;
  float best = 0.f;
  double work = 0.0;
  if (what == IBF_PEAK_HBM_COPY) {
    const int64_t bytes = (int64_t)1 << 30;                  // 1 GiB each way
    const int64_t n4 = bytes / (int64_t)sizeof(float4);
    IBF_HIP_CHECK(ibf::dev_malloc(&r.a, (size_t)bytes));
    IBF_HIP_CHECK(ibf::dev_malloc(&r.b, (size_t)bytes));
    IBF_HIP_CHECK(hipMemsetAsync(r.a, 0, (size_t)bytes, s));
    const int64_t per_blk = (int64_t)ibf::kPeakBlock * ibf::kCopyPer;
    const dim3 grid((unsigned)((n4 + per_blk - 1) / per_blk)), blk(ibf::kPeakBlock);
    for (int k = 0; k <= kReps; ++k) {                        // the first run warms up
      IBF_HIP_CHECK(hipEventRecord(r.e0, s));
      hipLaunchKernelGGL(ibf::k_peak_copy, grid, blk, 0, s, (const float4*)r.a, (float4*)r.b, n4);
      IBF_HIP_CHECK(hipGetLastError());
      IBF_HIP_CHECK(hipEventRecord(r.e1, s));
      IBF_HIP_CHECK(hipEventSynchronize(r.e1));
      float ms = 0.f;
      IBF_HIP_CHECK(hipEventElapsedTime(&ms, r.e0, r.e1));
      if (k > 0 && (best == 0.f || ms < best)) best = ms;
    }
    work = 2.0 * (double)bytes;                               // read + write
    *result = work / (best * 1e-3) / 1e9;                     // GB/s
  } else {
    const int iters = 4096;
    const int nblk = std::max(1, ncu * 8);
    IBF_HIP_CHECK(ibf::dev_malloc(&r.a, sizeof(float) * (size_t)nblk * ibf::kPeakBlock));
    for (int k = 0; k <= kReps; ++k) {
      IBF_HIP_CHECK(hipEventRecord(r.e0, s));
      hipLaunchKernelGGL(ibf::k_peak_mfma, dim3((unsigned)nblk), dim3(ibf::kPeakBlock), 0, s,
                         (float*)r.a, iters, 1.0f, 1e-6f);
      IBF_HIP_CHECK(hipGetLastError());
      IBF_HIP_CHECK(hipEventRecord(r.e1, s));
      IBF_HIP_CHECK(hipEventSynchronize(r.e1));
      float ms = 0.f;
      IBF_HIP_CHECK(hipEventElapsedTime(&ms, r.e0, r.e1));
      if (k > 0 && (best == 0.f || ms < best)) best = ms;
    }
    // per wave and instruction: 16 blocks of 4 x 4 x 1, 2 flops each
    const double waves = (double)nblk * (ibf::kPeakBlock / 64);
    work = waves * iters * 8.0 * (16.0 * 4 * 4 * 1 * 2);
    *result = work / (best * 1e-3) / 1e12;                    // TFLOP/s
  }
  return IBF_OK;
}
