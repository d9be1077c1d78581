// RFI mitigation of a filterbank before dedispersion (Ch. 3 Sec. "Bandpass Correction",
// "Channel Thresholding", "Spectrum Thresholding"). C-ABI entry points dd_bandpass,
// dd_bandpass_fit (host) and dd_rfi_clip.
//
// * bandpass_rows: one workgroup per channel sums the channel's samples in FP64 (fixed
//   order: per thread over strided samples, a butterfly per wavefront, the four wavefronts
//   in order) and writes the channel mean. One read of the input.
// * dd_bandpass_fit (host): least-squares polynomial over x = 2c/(nchan-1) - 1 by modified
//   Gram-Schmidt on the monomial columns (each orthogonalised twice); the fitted values are
//   the projection of the average onto their span.
// * chan_flag: one wavefront per (channel, window) sums the window in FP64 and flags a mean
//   further than the threshold from the channel's fitted value. chan_apply replaces every
//   sample of a flagged window or of a flagged window's neighbour by the fitted value.
// * spec_clip: each lane sums the spectra of 4 consecutive samples over channels in FP64,
//   in channel order, and replaces a whole spectrum by the fitted bandpass when its mean is
//   further than the threshold from the fit's mean. Lanes of a wavefront take consecutive
//   samples, so each channel read is one coalesced 1 KB line per wavefront.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "dd_internal.h"

namespace {

constexpr int kRfiThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(kRfiThreads) void bandpass_rows(const float* __restrict__ x, int64_t n, int64_t stride,
                                                             double* __restrict__ avg) {
  __shared__ double red[4];
  const float* row = x + (int64_t)blockIdx.x * stride;
  // 16-byte loads when the row is aligned; each thread adds its 4 samples in order
  const int64_t n4 = (reinterpret_cast<uintptr_t>(row) & 15) == 0 ? n / 4 : 0;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n4; i += kRfiThreads) {
    const float4 v = reinterpret_cast<const float4*>(row)[i];
    s += (double)v.x;
    s += (double)v.y;
    s += (double)v.z;
    s += (double)v.w;
  }
  for (int64_t t = 4 * n4 + threadIdx.x; t < n; t += kRfiThreads) s += (double)row[t];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) avg[blockIdx.x] = ((red[0] + red[1]) + (red[2] + red[3])) / (double)n;
}

// blockIdx.y = channel; each wavefront takes one window (the window index is uniform across
// the wavefront, so a wavefront past the last window leaves as a whole).
__global__ __launch_bounds__(kRfiThreads) void chan_flag(const float* __restrict__ x, int64_t n, int64_t stride,
                                                         int64_t window, int64_t nwin, const double* __restrict__ fit,
                                                         double thr, int32_t* __restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (kRfiThreads / 64) + (threadIdx.x >> 6);
  if (w >= nwin) return;
  const int64_t c = blockIdx.y;
  const float* row = x + c * stride;
  const int64_t t0 = w * window;
  const int64_t len = n - t0 < window ? n - t0 : window;
  double s = 0.0;
  // 16-byte loads when windows start on 16-byte boundaries: a wavefront reads 1 KB per step
  const int64_t len4 = (window & 3) == 0 && (reinterpret_cast<uintptr_t>(row) & 15) == 0 ? len / 4 : 0;
  const float4* p4 = reinterpret_cast<const float4*>(row + t0);
  for (int64_t i = lane; i < len4; i += 64) {
    const float4 v = p4[i];
    s += (double)v.x;
    s += (double)v.y;
    s += (double)v.z;
    s += (double)v.w;
  }
  for (int64_t i = 4 * len4 + lane; i < len; i += 64) s += (double)row[t0 + i];
  s = wave_sum(s);
  if (lane == 0) flags[c * nwin + w] = fabs(s / (double)len - fit[c]) > thr ? 1 : 0;
}

// One lane per (channel, window): a window with no flag on it or its neighbours leaves at
// once, so clean data costs only the flag reads; a replaced window is written by its lane.
__global__ __launch_bounds__(kRfiThreads) void chan_apply(float* __restrict__ x, int64_t n, int64_t stride,
                                                          int64_t window, int64_t nwin, const double* __restrict__ fit,
                                                          const int32_t* __restrict__ flags) {
  const int64_t w = (int64_t)blockIdx.x * kRfiThreads + threadIdx.x;
  if (w >= nwin) return;
  const int64_t c = blockIdx.y;
  const int32_t* f = flags + c * nwin;
  const bool hit = f[w] != 0 || (w > 0 && f[w - 1] != 0) || (w + 1 < nwin && f[w + 1] != 0);
  if (!hit) return;
  const int64_t t0 = w * window;
  const int64_t len = n - t0 < window ? n - t0 : window;
  const float v = (float)fit[c];
  float* row = x + c * stride + t0;
  for (int64_t i = 0; i < len; ++i) row[i] = v;
}

// Each lane takes 4 consecutive samples (16-byte loads when every row start is aligned);
// every sample's spectrum is summed over channels in channel order.
__global__ __launch_bounds__(kRfiThreads) void spec_clip(float* __restrict__ x, int64_t nchan, int64_t n,
                                                         int64_t stride, const double* __restrict__ fit,
                                                         double center, double thr) {
  const int64_t t0 = ((int64_t)blockIdx.x * kRfiThreads + threadIdx.x) * 4;
  if (t0 >= n) return;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  const bool vec = t0 + 3 < n && (stride & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
  if (vec) {
    for (int64_t c = 0; c < nchan; ++c) {
      const float4 v = *reinterpret_cast<const float4*>(x + c * stride + t0);
      s[0] += (double)v.x;
      s[1] += (double)v.y;
      s[2] += (double)v.z;
      s[3] += (double)v.w;
    }
  } else {
    for (int64_t c = 0; c < nchan; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (t0 + i < n) s[i] += (double)x[c * stride + t0 + i];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (t0 + i < n && fabs(s[i] / (double)nchan - center) > thr)
      for (int64_t c = 0; c < nchan; ++c) x[c * stride + t0 + i] = (float)fit[c];
}

hipError_t launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) dd::fail(DD_ERR_HIP, std::string(what) + " launch: " + hipGetErrorString(e));
  return e;
}

}  // namespace

extern "C" int dd_bandpass(const float* d_in, int64_t nchan, int64_t nsamp, int64_t row_stride, double* d_avg,
                           void* stream) {
  dd::clear_error();
  if (!d_in || !d_avg) return dd::fail(DD_ERR_INVALID_ARG, "input and average must be non-NULL");
  if (nchan < 1 || nsamp < 1 || row_stride < nsamp)
    return dd::fail(DD_ERR_INVALID_ARG, "need nchan >= 1, nsamp >= 1 and row_stride >= nsamp");
  if (nchan > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "too many channels");
  hipLaunchKernelGGL(bandpass_rows, dim3((unsigned)nchan), dim3(kRfiThreads), 0, static_cast<hipStream_t>(stream),
                     d_in, nsamp, row_stride, d_avg);
  return launched("bandpass") == hipSuccess ? DD_OK : DD_ERR_HIP;
}

extern "C" int dd_bandpass_fit(const double* avg, int32_t nchan, int32_t order, double* fit, double* rmse,
                               double* fit_mean) {
  dd::clear_error();
  if (!avg || !fit) return dd::fail(DD_ERR_INVALID_ARG, "avg and fit must be non-NULL");
  if (nchan < 1 || order < 0 || order >= nchan || order > 16)
    return dd::fail(DD_ERR_INVALID_ARG, "need nchan >= 1 and 0 <= order < nchan, order <= 16");
  const int n = nchan, m = order + 1;
  std::vector<double> x(n), q((size_t)m * n), col(n, 1.0);
  for (int c = 0; c < n; ++c) x[c] = n == 1 ? 0.0 : 2.0 * (double)c / (double)(n - 1) - 1.0;
  for (int j = 0; j < m; ++j) {
    if (j > 0)
      for (int c = 0; c < n; ++c) col[c] *= x[c];
    std::vector<double> v(col);
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        const double* qi = &q[(size_t)i * n];
        double d = 0.0;
        for (int c = 0; c < n; ++c) d += qi[c] * v[c];
        for (int c = 0; c < n; ++c) v[c] -= d * qi[c];
      }
    double nn = 0.0;
    for (int c = 0; c < n; ++c) nn += v[c] * v[c];
    nn = std::sqrt(nn);
    if (!(nn > 1e-12)) return dd::fail(DD_ERR_INVALID_ARG, "polynomial columns are degenerate for this order");
    for (int c = 0; c < n; ++c) q[(size_t)j * n + c] = v[c] / nn;
  }
  for (int c = 0; c < n; ++c) fit[c] = 0.0;
  for (int j = 0; j < m; ++j) {
    const double* qj = &q[(size_t)j * n];
    double d = 0.0;
    for (int c = 0; c < n; ++c) d += qj[c] * avg[c];
    for (int c = 0; c < n; ++c) fit[c] += d * qj[c];
  }
  double e2 = 0.0, s = 0.0;
  for (int c = 0; c < n; ++c) {
    e2 += (avg[c] - fit[c]) * (avg[c] - fit[c]);
    s += fit[c];
  }
  if (rmse) *rmse = std::sqrt(e2 / n);
  if (fit_mean) *fit_mean = s / n;
  return DD_OK;
}

extern "C" int dd_rfi_clip(float* d_data, int64_t nchan, int64_t nsamp, int64_t row_stride, const double* d_fit,
                           double chan_threshold, int64_t window, int32_t* d_flags, double fit_mean,
                           double spec_threshold, void* stream) {
  dd::clear_error();
  if (!d_data || !d_fit) return dd::fail(DD_ERR_INVALID_ARG, "data and fit must be non-NULL");
  if (nchan < 1 || nsamp < 1 || row_stride < nsamp)
    return dd::fail(DD_ERR_INVALID_ARG, "need nchan >= 1, nsamp >= 1 and row_stride >= nsamp");
  if (nchan > 65535) return dd::fail(DD_ERR_UNSUPPORTED, "at most 65535 channels per call");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (chan_threshold > 0.0) {
    if (window < 1 || !d_flags) return dd::fail(DD_ERR_INVALID_ARG, "channel clipping needs window >= 1 and flags");
    const int64_t nwin = (nsamp + window - 1) / window;
    const int64_t wblocks = (nwin + kRfiThreads / 64 - 1) / (kRfiThreads / 64);
    if (wblocks > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "series too long");
    hipLaunchKernelGGL(chan_flag, dim3((unsigned)wblocks, (unsigned)nchan), dim3(kRfiThreads), 0, st, d_data, nsamp,
                       row_stride, window, nwin, d_fit, chan_threshold, d_flags);
    if (launched("channel flag") != hipSuccess) return DD_ERR_HIP;
    const int64_t ablocks = (nwin + kRfiThreads - 1) / kRfiThreads;
    hipLaunchKernelGGL(chan_apply, dim3((unsigned)ablocks, (unsigned)nchan), dim3(kRfiThreads), 0, st, d_data, nsamp,
                       row_stride, window, nwin, d_fit, d_flags);
    if (launched("channel apply") != hipSuccess) return DD_ERR_HIP;
  }
  if (spec_threshold > 0.0) {
    const int64_t tblocks = (nsamp + 4 * kRfiThreads - 1) / (4 * kRfiThreads);
    if (tblocks > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "series too long");
    hipLaunchKernelGGL(spec_clip, dim3((unsigned)tblocks), dim3(kRfiThreads), 0, st, d_data, nchan, nsamp, row_stride,
                       d_fit, fit_mean, spec_threshold);
    if (launched("spectrum clip") != hipSuccess) return DD_ERR_HIP;
  }
  return DD_OK;
}
