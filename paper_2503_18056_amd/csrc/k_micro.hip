// Machine-peak microbenchmarks, measured in the same process as the
// workload so that roofline fractions can be stated against what this GPU
// delivers as well as against the vendor figures:
//  - HBM: a streaming copy (16-byte loads and stores, grid-stride) of a
//    buffer much larger than the caches; bytes moved = 2 x the copy size;
//  - FP64 MFMA: v_mfma_f64_16x16x4f64 on register operands, four
//    independent accumulators per wavefront (no memory traffic in the loop);
//  - FP32 MFMA: v_mfma_f32_16x16x4f32, likewise.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/tt_kernels.h"

namespace tt {
void kernel_error(const std::string& m);  // the message of tt_kernel_last_error
}

namespace {

__global__ __launch_bounds__(256) void k_copy16(const float4* __restrict__ src,
                                                float4* __restrict__ dst, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_mfma_f64(int iters, double* __restrict__ out) {
  const double a = 1.0 + 1e-3 * (threadIdx.x & 7), b = 1.0 - 1e-3 * (threadIdx.x & 3);
  d4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  for (int it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c3, 0, 0, 0);
  }
  const d4 s = c0 + c1 + c2 + c3;
  out[blockIdx.x * (long long)blockDim.x + threadIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(256) void k_mfma_f32(int iters, double* __restrict__ out) {
  const float a = 1.0f + 1e-3f * (threadIdx.x & 7), b = 1.0f - 1e-3f * (threadIdx.x & 3);
  f4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  for (int it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c3, 0, 0, 0);
  }
  const f4 s = c0 + c1 + c2 + c3;
  out[blockIdx.x * (long long)blockDim.x + threadIdx.x] = (double)(s[0] + s[1] + s[2] + s[3]);
}

constexpr int MFMA_BLOCKS = 2048;  // 8 waves per CU on 256 CUs

}  // namespace

extern "C" {

size_t tt_kernel_microbench_workspace(int32_t which, size_t copy_bytes) {
  if (which == 0) return 2 * ((copy_bytes + 15) / 16 * 16);
  if (which == 1 || which == 2) return (size_t)MFMA_BLOCKS * 256 * sizeof(double);
  return 0;
}

tt_status tt_kernel_microbench(int32_t which, size_t copy_bytes, int32_t iters, void* ws,
                               size_t ws_bytes, double* result, void* stream) {
  if (!ws || !result || iters < 1 || (which < 0 || which > 2) || (which == 0 && copy_bytes < 16)) {
    tt::kernel_error("bad microbench arguments");
    return TT_ERR_INVALID_ARG;
  }
  if (ws_bytes < tt_kernel_microbench_workspace(which, copy_bytes)) {
    tt::kernel_error("workspace too small");
    return TT_ERR_OOM;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) {
    tt::kernel_error("hipEventCreate failed");
    return TT_ERR_DEVICE;
  }
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    tt::kernel_error("hipEventCreate failed");
    return TT_ERR_DEVICE;
  }
  const long long n16 = (long long)((copy_bytes + 15) / 16);
  float4* src = (float4*)ws;
  float4* dst = src + n16;
  auto launch = [&]() {
    if (which == 0) k_copy16<<<16384, 256, 0, s>>>(src, dst, n16);
    else if (which == 1) k_mfma_f64<<<MFMA_BLOCKS, 256, 0, s>>>(iters, (double*)ws);
    else k_mfma_f32<<<MFMA_BLOCKS, 256, 0, s>>>(iters, (double*)ws);
  };
  launch();  // first launch: code upload and clocks, not timed
  hipEventRecord(e0, s);
  const int reps = which == 0 ? iters : 1;
  for (int r = 0; r < reps; ++r) launch();
  hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) e = hipGetLastError();
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (e != hipSuccess) {
    tt::kernel_error(hipGetErrorString(e));
    return TT_ERR_DEVICE;
  }
  const double sec = ms * 1e-3;
  if (which == 0) {
    *result = 2.0 * (double)n16 * 16.0 * reps / sec / 1e9;  // GB/s
  } else {
    const double flops = (double)MFMA_BLOCKS * 4 /* waves */ * iters * 4 /* MFMAs */ *
                         (2.0 * 16 * 16 * 4);
    *result = flops / sec / 1e12;  // TFLOP/s
  }
  return TT_OK;
}

}  // extern "C"
