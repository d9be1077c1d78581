// Boxcar smoothing of (normalised) dedispersed series by successive addition of adjacent
// samples: the single-pulse search's smoothing, which downfactors the series by the
// boxcar width (Ch. 2 single-pulse detection; Ch. 6 template matching). C-ABI entry
// point dd_boxcar.
//
// Level k of a row holds s_k[j] = (x[j 2^k] + ... + x[j 2^k + 2^k - 1]) / sqrt(2^k) for
// j < floor(n / 2^k); levels are stored one after another in the output row, level k at
// offset sum_{i<k} floor(n / 2^i). Each lane takes 4 consecutive samples (a wavefront 256,
// loaded lane-contiguously) and forms every level from the one below by pairwise FP32
// sums: levels 1 and 2 in registers, levels 3 .. 6 across 2 .. 16 lanes by butterfly
// shuffles. Each input sample is read once and each output written once: an HBM-bound
// pass.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "dd_internal.h"

namespace {

constexpr int kBoxThreads = 256;
constexpr int kMaxLevel = 6;

__host__ __device__ inline int64_t level_offset(int64_t n, int k) {
  int64_t o = 0;
  for (int i = 0; i < k; ++i) o += n >> i;
  return o;
}

__global__ __launch_bounds__(kBoxThreads) void boxcar_rows(const float* __restrict__ x, int64_t n, int64_t stride,
                                                           int levels, float* __restrict__ out, int64_t ostride) {
  // lane l of the workgroup takes samples s0 .. s0 + 3: a wavefront covers 256 consecutive
  // samples, loaded lane-contiguously; no lane returns early, every lane takes part in the
  // cross-lane sums
  const int lane = threadIdx.x & 63;
  const int64_t s0 = ((int64_t)blockIdx.x * kBoxThreads + threadIdx.x) * 4;
  const float* row = x + (int64_t)blockIdx.y * stride;
  float* orow = out + (int64_t)blockIdx.y * ostride;
  float v[4];
  if (s0 + 3 < n && (reinterpret_cast<uintptr_t>(row) & 15) == 0) {
    const float4 q = *reinterpret_cast<const float4*>(row + s0);
    v[0] = q.x, v[1] = q.y, v[2] = q.z, v[3] = q.w;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = s0 + i < n ? row[s0 + i] : 0.0f;
  }
  // level 0 is the series itself
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (s0 + i < n) orow[s0 + i] = v[i];
  if (levels >= 1) {
    const int64_t off = n;
    const float norm = 0.70710678118654752f;
    const float a = v[0] + v[1], b = v[2] + v[3];
    const int64_t j = s0 >> 1;
    if (((j + 1) << 1) <= n) orow[off + j] = a * norm;
    if (((j + 2) << 1) <= n) orow[off + j + 1] = b * norm;
    float s = a + b;  // level 2: 4 samples
    if (levels >= 2 && ((s0 >> 2) + 1) << 2 <= n) orow[level_offset(n, 2) + (s0 >> 2)] = s * 0.5f;
    // levels 3 .. 6: the 8-, 16-, 32- and 64-sample windows span 2, 4, 8 and 16 lanes
#pragma unroll
    for (int k = 3; k <= kMaxLevel; ++k) {
      s += __shfl_xor(s, 1 << (k - 3), 64);
      if (k <= levels && (lane & ((1 << (k - 2)) - 1)) == 0) {
        const int64_t jk = s0 >> k;
        if (((jk + 1) << k) <= n) orow[level_offset(n, k) + jk] = s * (1.0f / sqrtf((float)(1 << k)));
      }
    }
  }
}

}  // namespace

extern "C" int dd_boxcar(const float* d_series, int64_t nrows, int64_t n, int64_t row_stride, int32_t levels,
                         float* d_out, int64_t out_row_stride, void* stream) {
  dd::clear_error();
  if (!d_series || !d_out) return dd::fail(DD_ERR_INVALID_ARG, "series and output must be non-NULL");
  if (nrows < 1 || n < 1 || row_stride < n)
    return dd::fail(DD_ERR_INVALID_ARG, "need nrows >= 1, n >= 1 and row_stride >= n");
  if (levels < 0 || levels > kMaxLevel)
    return dd::fail(DD_ERR_INVALID_ARG, "levels must be in 0..6 (boxcars of 1..64 samples)");
  if (out_row_stride < level_offset(n, levels + 1))
    return dd::fail(DD_ERR_INVALID_ARG, "output row shorter than the levels it holds");
  if (nrows > 65535) return dd::fail(DD_ERR_UNSUPPORTED, "at most 65535 rows per call");
  const int64_t blocks = (n + 4 * kBoxThreads - 1) / (4 * kBoxThreads);
  if (blocks > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "series too long");
  hipLaunchKernelGGL(boxcar_rows, dim3((unsigned)blocks, (unsigned)nrows), dim3(kBoxThreads), 0,
                     static_cast<hipStream_t>(stream), d_series, n, row_stride, (int)levels, d_out, out_row_stride);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return dd::fail(DD_ERR_HIP, std::string("boxcar launch: ") + hipGetErrorString(e));
  return DD_OK;
}
