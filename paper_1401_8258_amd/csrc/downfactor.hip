// Time binning of a filterbank: downfactor every channel by 2 by summing adjacent samples
// (Ch. 2 Sec. "Direct Dedispersion", time binning above the diagonal DM; Sec. "Computing
// Larger DMs", the downfactor step). C-ABI entry point dd_downfactor.
//
// out[c][j] = A[c][2j] + A[c][2j+1] for j < floor(nsamp / 2), one FP32 add per output: u8
// codes and FP16 values are widened to FP32 first, so their sums are exact, and FP32
// inputs give the correctly rounded FP32 sum. Each lane reads 8 consecutive input samples
// (a wavefront 512, lane-contiguous vector loads when the row is aligned) and writes 4
// outputs; one read of the input and one write of half as many FP32 values: HBM-bound.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "dd_internal.h"

namespace {

constexpr int kDfThreads = 256;

template <typename T>
struct alignas(8 * sizeof(T)) Vec8 {
  T v[8];
};

__device__ __forceinline__ float widen(float x) { return x; }
__device__ __forceinline__ float widen(__half x) { return __half2float(x); }
__device__ __forceinline__ float widen(uint8_t x) { return (float)x; }

template <typename T>
__global__ __launch_bounds__(kDfThreads) void downfactor_rows(const T* __restrict__ in, int64_t nsamp, int64_t stride,
                                                              float* __restrict__ out, int64_t ostride) {
  const int64_t m = nsamp >> 1;  // outputs per row
  const int64_t j0 = ((int64_t)blockIdx.x * kDfThreads + threadIdx.x) * 4;
  if (j0 >= m) return;
  const T* row = in + (int64_t)blockIdx.y * stride;
  float* orow = out + (int64_t)blockIdx.y * ostride;
  float s[4];
  if (j0 + 3 < m && (reinterpret_cast<uintptr_t>(row) % (8 * sizeof(T))) == 0) {
    const Vec8<T> q = *reinterpret_cast<const Vec8<T>*>(row + 2 * j0);
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] = widen(q.v[2 * i]) + widen(q.v[2 * i + 1]);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      s[i] = j0 + i < m ? widen(row[2 * (j0 + i)]) + widen(row[2 * (j0 + i) + 1]) : 0.0f;
  }
  if (j0 + 3 < m && (reinterpret_cast<uintptr_t>(orow) & 15) == 0) {
    *reinterpret_cast<float4*>(orow + j0) = make_float4(s[0], s[1], s[2], s[3]);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (j0 + i < m) orow[j0 + i] = s[i];
  }
}

}  // namespace

extern "C" int dd_downfactor(const void* d_in, int32_t in_dtype, int64_t nchan, int64_t nsamp, int64_t in_row_stride,
                             float* d_out, int64_t out_row_stride, void* stream) {
  dd::clear_error();
  if (!d_in || !d_out) return dd::fail(DD_ERR_INVALID_ARG, "input and output must be non-NULL");
  if (in_dtype != DD_F32 && in_dtype != DD_F16 && in_dtype != DD_U8)
    return dd::fail(DD_ERR_INVALID_ARG, "unknown input dtype");
  if (nchan < 1 || nsamp < 2 || in_row_stride < nsamp)
    return dd::fail(DD_ERR_INVALID_ARG, "need nchan >= 1, nsamp >= 2 and in_row_stride >= nsamp");
  if (out_row_stride < nsamp / 2) return dd::fail(DD_ERR_INVALID_ARG, "out_row_stride < nsamp / 2");
  if (nchan > 65535) return dd::fail(DD_ERR_UNSUPPORTED, "at most 65535 channels per call");
  const int64_t blocks = (nsamp / 2 + 4 * kDfThreads - 1) / (4 * kDfThreads);
  if (blocks > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "series too long");
  const dim3 grid((unsigned)blocks, (unsigned)nchan);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (in_dtype == DD_F32)
    hipLaunchKernelGGL(downfactor_rows<float>, grid, dim3(kDfThreads), 0, st, static_cast<const float*>(d_in), nsamp,
                       in_row_stride, d_out, out_row_stride);
  else if (in_dtype == DD_F16)
    hipLaunchKernelGGL(downfactor_rows<__half>, grid, dim3(kDfThreads), 0, st, static_cast<const __half*>(d_in),
                       nsamp, in_row_stride, d_out, out_row_stride);
  else
    hipLaunchKernelGGL(downfactor_rows<uint8_t>, grid, dim3(kDfThreads), 0, st, static_cast<const uint8_t*>(d_in),
                       nsamp, in_row_stride, d_out, out_row_stride);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return dd::fail(DD_ERR_HIP, std::string("downfactor launch: ") + hipGetErrorString(e));
  return DD_OK;
}
