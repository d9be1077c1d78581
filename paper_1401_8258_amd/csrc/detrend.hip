// Detrending and normalisation of dedispersed series (Sec. 3.5 "Signal Post-processing"),
// and its C-ABI entry point dd_detrend.
//
// One workgroup per series. Pass 1 sums x_t, x_t^2 and (t - tbar) x_t in FP64; the
// least-squares line is then b = sum (t - tbar) x_t / S_tt, S_tt = n(n^2 - 1)/12,
// a = mean - b*tbar, and since the residual is orthogonal to the line its sum of squares
// is sum (x - mean)^2 - b^2 S_tt. Pass 2 writes the residual x_t - (a + b t), divided by
// its population RMS when normalising. Every sum runs in a fixed order: each thread over
// its strided samples, then a fixed butterfly per wavefront and the four wavefronts in
// order, so results do not depend on anything but the input. Rows are read and written
// with 16-byte accesses when aligned. HBM-bound: two reads and one write of the series.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "dd_internal.h"

namespace {

constexpr int kDetrendThreads = 256;

__device__ __forceinline__ double wave_sum_tree(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 256-thread workgroup in a fixed tree; every thread gets the result.
__device__ double group_sum(double v, double* red) {
  v = wave_sum_tree(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();  // red[] from a previous call has been read
  if (lane == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(kDetrendThreads) void detrend_rows(float* __restrict__ x, int64_t n, int64_t stride,
                                                                int normalise, float* __restrict__ rms_out) {
  __shared__ double red[4];
  float* row = x + (int64_t)blockIdx.x * stride;
  const double tbar = 0.5 * (double)(n - 1);
  // 16-byte loads when the row is aligned: thread i takes samples 4i .. 4i+3 in order
  const int64_t n4 = (reinterpret_cast<uintptr_t>(row) & 15) == 0 ? n / 4 : 0;
  double sx = 0.0, sxx = 0.0, stx = 0.0;
  for (int64_t i = threadIdx.x; i < n4; i += kDetrendThreads) {
    const float4 q = reinterpret_cast<const float4*>(row)[i];
    const float e[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double v = (double)e[k];
      sx += v;
      sxx += v * v;
      stx += ((double)(4 * i + k) - tbar) * v;
    }
  }
  for (int64_t t = 4 * n4 + threadIdx.x; t < n; t += kDetrendThreads) {
    const double v = (double)row[t];
    sx += v;
    sxx += v * v;
    stx += ((double)t - tbar) * v;
  }
  sx = group_sum(sx, red);
  sxx = group_sum(sxx, red);
  stx = group_sum(stx, red);
  const double nn = (double)n;
  const double stt = nn * (nn * nn - 1.0) / 12.0;
  const double b = n > 1 ? stx / stt : 0.0;
  const double mean = sx / nn;
  const double a = mean - b * tbar;
  const double s2 = fmax((sxx - nn * mean * mean) - b * b * stt, 0.0);
  const double rms = sqrt(s2 / nn);
  const double scale = normalise && rms > 0.0 ? 1.0 / rms : 1.0;
  for (int64_t i = threadIdx.x; i < n4; i += kDetrendThreads) {
    float4 q = reinterpret_cast<float4*>(row)[i];
    const double t0 = (double)(4 * i);
    q.x = (float)(((double)q.x - (a + b * t0)) * scale);
    q.y = (float)(((double)q.y - (a + b * (t0 + 1.0))) * scale);
    q.z = (float)(((double)q.z - (a + b * (t0 + 2.0))) * scale);
    q.w = (float)(((double)q.w - (a + b * (t0 + 3.0))) * scale);
    reinterpret_cast<float4*>(row)[i] = q;
  }
  for (int64_t t = 4 * n4 + threadIdx.x; t < n; t += kDetrendThreads)
    row[t] = (float)(((double)row[t] - (a + b * (double)t)) * scale);
  if (rms_out && threadIdx.x == 0) rms_out[blockIdx.x] = (float)rms;
}

}  // namespace

extern "C" int dd_detrend(float* d_series, int64_t nrows, int64_t n, int64_t row_stride, int32_t normalise,
                          float* d_rms, void* stream) {
  dd::clear_error();
  if (!d_series) return dd::fail(DD_ERR_INVALID_ARG, "series must be non-NULL");
  if (nrows < 1 || n < 1 || row_stride < n)
    return dd::fail(DD_ERR_INVALID_ARG, "need nrows >= 1, n >= 1 and row_stride >= n");
  if (nrows > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "too many rows");
  hipLaunchKernelGGL(detrend_rows, dim3((unsigned)nrows), dim3(kDetrendThreads), 0,
                     static_cast<hipStream_t>(stream), d_series, n, row_stride, normalise ? 1 : 0, d_rms);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return dd::fail(DD_ERR_HIP, std::string("detrend launch: ") + hipGetErrorString(e));
  return DD_OK;
}
