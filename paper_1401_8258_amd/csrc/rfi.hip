// RFI mitigation of a filterbank before dedispersion (Ch. 3 Sec. "Bandpass Correction",
// "Channel Thresholding", "Spectrum Thresholding"). C-ABI entry points dd_bandpass,
// dd_bandpass_fit (host) and dd_rfi_clip for FP32 filterbanks; dd_bandpass_u8 and
// dd_rfi_clip_u8 for 8-bit codes (exact integer sums, replacement by the nearest code of
// the fit, no in-place correction: an 8-bit sample cannot hold x - fit).
//
// * bandpass_rows: one workgroup per channel sums the channel's samples in FP64 (fixed
//   order: per thread over strided samples, a butterfly per wavefront, the four wavefronts
//   in order) and writes the channel mean. One read of the input.
// * bandpass_windows: the same average together with every window's mean (the channel
//   stage's statistic), so the channel stage needs no read of its own: each wavefront sums
//   its windows four at a time (closed together by one transposing reduction) and the
//   channel total is the sum of its window sums in a fixed order.
// * bandpass_windows_u8: exact integer sums (v_sad_u8 over 16-byte loads). A 16-byte
//   aligned row whose window is 16 L bytes (L = 1, 2, ..., 64) is read in 1 KB lines, one
//   window per group of L lanes, four lines in flight per lane; other rows one window per
//   wavefront.
// * dd_bandpass_fit (host): least-squares polynomial over x = 2c/(nchan-1) - 1 by modified
//   Gram-Schmidt on the monomial columns (each orthogonalised twice); the fitted values are
//   the projection of the average onto their span.
// * chan_flag: one thread per window flags a window mean further than the threshold from
//   the channel's fitted value. chan_apply replaces every sample of a flagged window or of a
//   flagged window's neighbour by the fitted value (one lane per window, writing only
//   replaced windows); chan_correct does the same and also subtracts the fitted value from
//   every sample (a read and a write of the whole filterbank).
// * spec_clip: each lane sums the spectra of 4 consecutive samples over channels in FP64,
//   in channel order (the uncorrected values: corrected samples plus their channel's fitted
//   value), and replaces a whole spectrum by the fitted bandpass (0 when corrected) when its
//   mean is further than the threshold from the fit's mean. Lanes of a wavefront take
//   consecutive samples, so each channel read is one coalesced 1 KB line per wavefront.
//
// Order (Ch. 3): channel windows and then spectra are compared, uncorrected, with the fit
// and replaced by it; the fitted bandpass is subtracted last (in FP32, x - (float)fit).
#include <hip/hip_runtime.h>

#include <algorithm>
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

// blockIdx.x = channel. Wavefront k takes windows k, k + 4, ... in groups of four (the loads
// of a group are issued together); lanes take 16-byte chunks (or single samples) strided by
// 64, and each window's sum closes with a butterfly. Writes each window's mean and the
// channel mean (the window sums added in window order per wavefront, then the four
// wavefronts in order).
constexpr int kGroup = 4;  // windows per wavefront whose loads are in flight together (8 measured slower)
__global__ __launch_bounds__(kRfiThreads) void bandpass_windows(const float* __restrict__ x, int64_t n,
                                                                int64_t stride, int64_t window, int64_t nwin,
                                                                double* __restrict__ avg, double* __restrict__ means) {
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const float* row = x + (int64_t)blockIdx.x * stride;
  const bool vec4 = (window & 3) == 0 && (reinterpret_cast<uintptr_t>(row) & 15) == 0;
  double tot = 0.0;
  for (int64_t wg = (int64_t)wv; wg < nwin; wg += 4 * kGroup) {
    double s[kGroup];
    int64_t len[kGroup];
#pragma unroll
    for (int k = 0; k < kGroup; ++k) {
      s[k] = 0.0;
      const int64_t w = wg + 4 * k;
      const int64_t t0 = w * window;
      len[k] = w < nwin ? (n - t0 < window ? n - t0 : window) : 0;
    }
    const int64_t len4 = vec4 ? window / 4 : 0;
    for (int64_t i = lane; i < len4; i += 64) {
      float4 v[kGroup];
#pragma unroll
      for (int k = 0; k < kGroup; ++k)
        if (4 * i + 3 < len[k]) v[k] = reinterpret_cast<const float4*>(row + (wg + 4 * k) * window)[i];
#pragma unroll
      for (int k = 0; k < kGroup; ++k)
        if (4 * i + 3 < len[k]) {
          s[k] += (double)v[k].x;
          s[k] += (double)v[k].y;
          s[k] += (double)v[k].z;
          s[k] += (double)v[k].w;
        }
    }
#pragma unroll
    for (int k = 0; k < kGroup; ++k) {
      // samples not covered by whole 16-byte chunks (all of them without vec4)
      const int64_t start = vec4 ? 4 * (len[k] / 4) : 0;
      for (int64_t i = start + lane; i < len[k]; i += 64) s[k] += (double)row[(wg + 4 * k) * window + i];
    }
    // the four window sums in 7 shuffles instead of 4 x 6: across 32 lanes the lower half
    // keeps windows 0 and 1 and the upper half 2 and 3, across 16 lanes each quarter keeps
    // one, then a 16-lane butterfly; window k's sum ends in lanes 16k .. 16k + 15
    static_assert(kGroup == 4, "the transposing reduction takes four windows");
    const bool hi32 = (lane & 32) != 0, hi16 = (lane & 16) != 0;
    double k0 = hi32 ? s[2] : s[0], k1 = hi32 ? s[3] : s[1];
    k0 += __shfl_xor(hi32 ? s[0] : s[2], 32, 64);
    k1 += __shfl_xor(hi32 ? s[1] : s[3], 32, 64);
    double ws = (hi16 ? k1 : k0) + __shfl_xor(hi16 ? k0 : k1, 16, 64);
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) ws += __shfl_xor(ws, off, 64);
    const int mine = lane >> 4;  // the window this lane's sum belongs to
    const int64_t lm = mine == 0 ? len[0] : mine == 1 ? len[1] : mine == 2 ? len[2] : len[3];
    if ((lane & 15) == 0 && lm > 0) {
      tot += ws;
      means[(int64_t)blockIdx.x * nwin + wg + 4 * mine] = ws / (double)lm;
    }
  }
  tot = wave_sum(tot);  // the window sums sit in lanes 0, 16, 32 and 48
  if (lane == 0) red[wv] = tot;
  __syncthreads();
  if (threadIdx.x == 0) avg[blockIdx.x] = ((red[0] + red[1]) + (red[2] + red[3])) / (double)n;
}

// One thread per (channel, window): flags[c][w] = |mean - fit[c]| > thr.
__global__ __launch_bounds__(kRfiThreads) void chan_flag(const double* __restrict__ means, int64_t nwin,
                                                         const double* __restrict__ fit, double thr,
                                                         int32_t* __restrict__ flags) {
  const int64_t w = (int64_t)blockIdx.x * kRfiThreads + threadIdx.x;
  if (w >= nwin) return;
  const int64_t c = blockIdx.y;
  flags[c * nwin + w] = fabs(means[c * nwin + w] - fit[c]) > thr ? 1 : 0;
}

__device__ __forceinline__ bool replaced(const int32_t* f, int64_t w, int64_t nwin) {
  // the three flags are loaded together (indices clamped into the row, then masked)
  const int32_t self = f[w];
  const int32_t prev = f[w > 0 ? w - 1 : w];
  const int32_t next = f[w + 1 < nwin ? w + 1 : w];
  return (self | (w > 0 ? prev : 0) | (w + 1 < nwin ? next : 0)) != 0;
}

// One lane per (channel, window): a window with no flag on it or its neighbours leaves at
// once, so clean data costs only the flag reads; a replaced window is written by its lane.
__global__ __launch_bounds__(kRfiThreads) void chan_apply(float* __restrict__ x, int64_t n, int64_t stride,
                                                          int64_t window, int64_t nwin, const double* __restrict__ fit,
                                                          const int32_t* __restrict__ flags) {
  const int64_t w = (int64_t)blockIdx.x * kRfiThreads + threadIdx.x;
  if (w >= nwin) return;
  const int64_t c = blockIdx.y;
  if (!replaced(flags + c * nwin, w, nwin)) return;
  const int64_t t0 = w * window;
  const int64_t len = n - t0 < window ? n - t0 : window;
  const float v = (float)fit[c];
  float* row = x + c * stride + t0;
  for (int64_t i = 0; i < len; ++i) row[i] = v;
}

// Bandpass correction with the channel stage's replacement: every sample becomes
// x - (float)fit[c], or 0 in a replaced window. A workgroup takes 1024 consecutive samples
// of a channel, 4 per thread (16-byte accesses when the row is aligned); the replacement
// decisions of the windows it touches are taken once into shared memory. flags may be null
// (no channel stage).
constexpr int kCorrSamples = 4 * kRfiThreads;
__global__ __launch_bounds__(kRfiThreads) void chan_correct(float* __restrict__ x, int64_t n, int64_t stride,
                                                            int64_t window, int64_t nwin,
                                                            const double* __restrict__ fit,
                                                            const int32_t* __restrict__ flags) {
  __shared__ unsigned char rep[kCorrSamples + 2];
  const int64_t b0 = (int64_t)blockIdx.x * kCorrSamples;
  const int64_t c = blockIdx.y;
  float* row = x + c * stride;
  const int64_t wa = b0 / window;
  const int64_t wb = ((b0 + kCorrSamples < n ? b0 + kCorrSamples : n) - 1) / window;
  const int32_t* f = flags ? flags + c * nwin : nullptr;
  // the samples' load is issued before the window decisions are gathered, so its latency
  // overlaps theirs
  const int64_t t0 = b0 + 4 * threadIdx.x;
  const bool vec = t0 + 3 < n && (reinterpret_cast<uintptr_t>(row) & 15) == 0;
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (vec) v = *reinterpret_cast<const float4*>(row + t0);
  for (int64_t w = wa + threadIdx.x; w <= wb; w += kRfiThreads) rep[w - wa] = f && replaced(f, w, nwin) ? 1 : 0;
  __syncthreads();
  if (t0 >= n) return;
  const float fv = (float)fit[c];
  bool hit[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) hit[i] = t0 + i < n && rep[(t0 + i) / window - wa] != 0;
  if (vec) {
    v.x = hit[0] ? 0.f : v.x - fv;
    v.y = hit[1] ? 0.f : v.y - fv;
    v.z = hit[2] ? 0.f : v.z - fv;
    v.w = hit[3] ? 0.f : v.w - fv;
    *reinterpret_cast<float4*>(row + t0) = v;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (t0 + i < n) row[t0 + i] = hit[i] ? 0.f : row[t0 + i] - fv;
  }
}

// Each lane takes 4 consecutive samples (16-byte loads when every row start is aligned);
// every sample's spectrum is summed over channels in channel order. With `subtract` the
// data are corrected already: each value is summed with its channel's FP32 fitted value,
// giving back the uncorrected spectrum to compare, and a replaced spectrum becomes 0.
__global__ __launch_bounds__(kRfiThreads) void spec_clip(float* __restrict__ x, int64_t nchan, int64_t n,
                                                         int64_t stride, const double* __restrict__ fit,
                                                         double center, double thr, int subtract) {
  const int64_t t0 = ((int64_t)blockIdx.x * kRfiThreads + threadIdx.x) * 4;
  if (t0 >= n) return;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  const bool vec = t0 + 3 < n && (stride & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
  if (vec) {
    for (int64_t c = 0; c < nchan; ++c) {
      const float4 v = *reinterpret_cast<const float4*>(x + c * stride + t0);
      const double b = subtract ? (double)(float)fit[c] : 0.0;
      s[0] += (double)v.x + b;
      s[1] += (double)v.y + b;
      s[2] += (double)v.z + b;
      s[3] += (double)v.w + b;
    }
  } else {
    for (int64_t c = 0; c < nchan; ++c) {
      const double b = subtract ? (double)(float)fit[c] : 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (t0 + i < n) s[i] += (double)x[c * stride + t0 + i] + b;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (t0 + i < n && fabs(s[i] / (double)nchan - center) > thr)
      for (int64_t c = 0; c < nchan; ++c) x[c * stride + t0 + i] = subtract ? 0.f : (float)fit[c];
}

// ---- 8-bit codes. Sums of codes are exact integers, so every channel, window and spectrum
// mean is the exact sum divided once in FP64, whatever the order of the additions; the
// replacement value is the fitted bandpass rounded to the nearest code (halves away from
// zero) and clamped to 0..255.

__device__ __forceinline__ uint8_t fit_code(double f) {
  const double r = floor(f + 0.5);
  return (uint8_t)(r < 0.0 ? 0.0 : (r > 255.0 ? 255.0 : r));
}

// Sum of bytes [a, a + len) of a row: 16-byte loads (four v_sad_u8 each) where the span is
// 16-byte aligned, single bytes at its ragged ends; lanes strided by 64 chunks.
__device__ __forceinline__ uint64_t row_bytes_sum(const uint8_t* __restrict__ row, int64_t a, int64_t len,
                                                  int lane) {
  const uint8_t* p = row + a;
  int64_t head = (int64_t)((16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15);
  if (head > len) head = len;
  const int64_t nv = (len - head) / 16;
  uint64_t s = 0;
  if (lane < head) s += p[lane];
  const uint4* v = reinterpret_cast<const uint4*>(p + head);
  for (int64_t i = lane; i < nv; i += 64) {
    const uint4 q = v[i];
    unsigned acc = __builtin_amdgcn_sad_u8(q.x, 0u, 0u);
    acc = __builtin_amdgcn_sad_u8(q.y, 0u, acc);
    acc = __builtin_amdgcn_sad_u8(q.z, 0u, acc);
    acc = __builtin_amdgcn_sad_u8(q.w, 0u, acc);
    s += acc;
  }
  for (int64_t i = head + 16 * nv + lane; i < len; i += 64) s += p[i];
  return s;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums of the whole windows of a 16-byte aligned row whose window is 16 L bytes (L a power
// of two up to 64): lane groups of L lanes each own one window of every 1 KB line, and each
// lane keeps kLines lines' loads in flight. A window's sum (at most 1024 x 255) closes with
// a 32-bit butterfly inside its group; its first lane writes the mean (when means is not
// null) and adds the sum to `tot`. Lines are taken by the four wavefronts in turn.
constexpr int kLines = 4;
template <int L>
__device__ __forceinline__ void windows_aligned_u8(const uint8_t* __restrict__ row, int64_t nfull, int lane, int wv,
                                                   double* __restrict__ means, uint64_t& tot) {
  const uint4* v = reinterpret_cast<const uint4*>(row);
  const int64_t nchunk = nfull * L;  // 16-byte chunks of the whole windows
  const int64_t nline = (nchunk + 63) / 64;
  for (int64_t l0 = wv; l0 < nline; l0 += 4 * kLines) {
    uint4 q[kLines];
#pragma unroll
    for (int u = 0; u < kLines; ++u) {
      const int64_t ci = (l0 + 4 * u) * 64 + lane;
      q[u] = ci < nchunk ? v[ci] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < kLines; ++u) {
      unsigned sum = __builtin_amdgcn_sad_u8(q[u].x, 0u, 0u);
      sum = __builtin_amdgcn_sad_u8(q[u].y, 0u, sum);
      sum = __builtin_amdgcn_sad_u8(q[u].z, 0u, sum);
      sum = __builtin_amdgcn_sad_u8(q[u].w, 0u, sum);
#pragma unroll
      for (int off = L / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
      const int64_t ci = (l0 + 4 * u) * 64 + lane;
      if ((lane & (L - 1)) == 0 && ci < nchunk) {
        tot += sum;
        if (means) means[ci / L] = (double)sum / (double)(16 * L);
      }
    }
  }
}

// blockIdx.x = channel; the channel mean is its exact total over n. With window means
// (means not null): a 16-byte aligned row whose window is 16 L bytes (L a power of two up to
// 64) takes its whole windows through windows_aligned_u8 and its ragged last window through
// wavefront 0; any other row has wavefront k take windows k, k + 4, ... With no window
// means the total of an aligned row comes from 1 KB windows the same way.
__global__ __launch_bounds__(kRfiThreads) void bandpass_windows_u8(const uint8_t* __restrict__ x, int64_t n,
                                                                   int64_t stride, int64_t window, int64_t nwin,
                                                                   double* __restrict__ avg,
                                                                   double* __restrict__ means) {
  __shared__ uint64_t red[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint8_t* row = x + (int64_t)blockIdx.x * stride;
  double* mrow = means ? means + (int64_t)blockIdx.x * nwin : nullptr;
  uint64_t tot = 0;
  const int64_t win = means ? window : 1024;  // the windows the aligned path walks
  const int64_t L = win / 16;
  const bool aligned = (reinterpret_cast<uintptr_t>(row) & 15) == 0 && win % 16 == 0 && L <= 64 && (L & (L - 1)) == 0;
  if (aligned) {
    const int64_t nfull = n / win;
    switch (L) {
      case 1: windows_aligned_u8<1>(row, nfull, lane, wv, mrow, tot); break;
      case 2: windows_aligned_u8<2>(row, nfull, lane, wv, mrow, tot); break;
      case 4: windows_aligned_u8<4>(row, nfull, lane, wv, mrow, tot); break;
      case 8: windows_aligned_u8<8>(row, nfull, lane, wv, mrow, tot); break;
      case 16: windows_aligned_u8<16>(row, nfull, lane, wv, mrow, tot); break;
      case 32: windows_aligned_u8<32>(row, nfull, lane, wv, mrow, tot); break;
      default: windows_aligned_u8<64>(row, nfull, lane, wv, mrow, tot); break;
    }
    const int64_t t0 = nfull * win;
    if (wv == 0 && t0 < n) {  // the ragged last window
      const uint64_t ws = wave_sum_u64(row_bytes_sum(row, t0, n - t0, lane));
      if (lane == 0) {
        tot += ws;
        if (mrow) mrow[nfull] = (double)ws / (double)(n - t0);
      }
    }
    tot = wave_sum_u64(tot);  // the group sums sit in their first lanes
  } else {
    for (int64_t w = wv; w < nwin; w += 4) {
      const int64_t t0 = w * window;
      const int64_t len = n - t0 < window ? n - t0 : window;
      const uint64_t ws = wave_sum_u64(row_bytes_sum(row, t0, len, lane));
      tot += ws;
      if (mrow && lane == 0) mrow[w] = (double)ws / (double)len;
    }
  }
  if (lane == 0) red[wv] = tot;
  __syncthreads();
  if (threadIdx.x == 0) avg[blockIdx.x] = (double)(red[0] + red[1] + red[2] + red[3]) / (double)n;
}

// One lane per (channel, window), as chan_apply, writing the fitted code.
__global__ __launch_bounds__(kRfiThreads) void chan_apply_u8(uint8_t* __restrict__ x, int64_t n, int64_t stride,
                                                             int64_t window, int64_t nwin,
                                                             const double* __restrict__ fit,
                                                             const int32_t* __restrict__ flags) {
  const int64_t w = (int64_t)blockIdx.x * kRfiThreads + threadIdx.x;
  if (w >= nwin) return;
  const int64_t c = blockIdx.y;
  if (!replaced(flags + c * nwin, w, nwin)) return;
  const int64_t t0 = w * window;
  const int64_t len = n - t0 < window ? n - t0 : window;
  const uint8_t v = fit_code(fit[c]);
  uint8_t* row = x + c * stride + t0;
  for (int64_t i = 0; i < len; ++i) row[i] = v;
}

// Each lane takes 16 consecutive samples (one 16-byte load per channel when every row start
// is aligned, so a wavefront reads 1 KB of a channel at once) and sums their spectra over
// channels in exact integers: the four wavefronts of a workgroup take the same samples and
// every fourth channel each (four loads in flight per lane), and the first adds the others'
// sums from LDS. A spectrum whose mean is further than the threshold from the fit's mean
// takes the fitted codes.
__global__ __launch_bounds__(kRfiThreads) void spec_clip_u8(uint8_t* __restrict__ x, int64_t nchan, int64_t n,
                                                            int64_t stride, const double* __restrict__ fit,
                                                            double center, double thr) {
  __shared__ unsigned part[3][16][64];  // the partial sums of wavefronts 1..3
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t t0 = ((int64_t)blockIdx.x * 64 + lane) * 16;
  unsigned s[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) s[i] = 0;
  auto add16 = [&](const uint4 q) {
    const unsigned w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int b = 0; b < 4; ++b) s[4 * j + b] += (w4[j] >> (8 * b)) & 0xffu;
  };
  if (t0 < n) {
    // wavefront wv sums channels wv, wv + 4, ...: exact integers, so the order is free
    const bool vec = t0 + 15 < n && (stride & 15) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    if (vec) {
      int64_t c = wv;
      for (; c + 12 < nchan; c += 16) {  // four loads in flight
        uint4 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = *reinterpret_cast<const uint4*>(x + (c + 4 * u) * stride + t0);
#pragma unroll
        for (int u = 0; u < 4; ++u) add16(q[u]);
      }
      for (; c < nchan; c += 4) add16(*reinterpret_cast<const uint4*>(x + c * stride + t0));
    } else {
      for (int64_t c = wv; c < nchan; c += 4)
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (t0 + i < n) s[i] += x[c * stride + t0 + i];
    }
  }
  if (wv > 0)
#pragma unroll
    for (int i = 0; i < 16; ++i) part[wv - 1][i][lane] = s[i];
  __syncthreads();  // every wavefront has read its channels before any spectrum is replaced
  if (wv != 0 || t0 >= n) return;
#pragma unroll
  for (int i = 0; i < 16; ++i) s[i] += part[0][i][lane] + part[1][i][lane] + part[2][i][lane];
#pragma unroll
  for (int i = 0; i < 16; ++i)
    if (t0 + i < n && fabs((double)s[i] / (double)nchan - center) > thr)
      for (int64_t c = 0; c < nchan; ++c) x[c * stride + t0 + i] = fit_code(fit[c]);
}

hipError_t launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) dd::fail(DD_ERR_HIP, std::string(what) + " launch: " + hipGetErrorString(e));
  return e;
}

}  // namespace

extern "C" int dd_bandpass(const float* d_in, int64_t nchan, int64_t nsamp, int64_t row_stride, int64_t window,
                           double* d_avg, double* d_window_means, void* stream) {
  dd::clear_error();
  if (!d_in || !d_avg) return dd::fail(DD_ERR_INVALID_ARG, "input and average must be non-NULL");
  if (nchan < 1 || nsamp < 1 || row_stride < nsamp)
    return dd::fail(DD_ERR_INVALID_ARG, "need nchan >= 1, nsamp >= 1 and row_stride >= nsamp");
  if (window < 0 || (window > 0) != (d_window_means != nullptr))
    return dd::fail(DD_ERR_INVALID_ARG, "window means need window >= 1 and their buffer (or window 0 and NULL)");
  if (nchan > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "too many channels");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (window > 0)
    hipLaunchKernelGGL(bandpass_windows, dim3((unsigned)nchan), dim3(kRfiThreads), 0, st, d_in, nsamp, row_stride,
                       window, (nsamp + window - 1) / window, d_avg, d_window_means);
  else
    hipLaunchKernelGGL(bandpass_rows, dim3((unsigned)nchan), dim3(kRfiThreads), 0, st, d_in, nsamp, row_stride, d_avg);
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
                           double chan_threshold, int64_t window, const double* d_window_means, int32_t* d_flags,
                           double fit_mean, double spec_threshold, int32_t subtract_bandpass, void* stream) {
  dd::clear_error();
  if (!d_data || !d_fit) return dd::fail(DD_ERR_INVALID_ARG, "data and fit must be non-NULL");
  if (nchan < 1 || nsamp < 1 || row_stride < nsamp)
    return dd::fail(DD_ERR_INVALID_ARG, "need nchan >= 1, nsamp >= 1 and row_stride >= nsamp");
  if (nchan > 65535) return dd::fail(DD_ERR_UNSUPPORTED, "at most 65535 channels per call");
  const bool chan = chan_threshold > 0.0, sub = subtract_bandpass != 0;
  if (chan && (window < 1 || !d_flags || !d_window_means))
    return dd::fail(DD_ERR_INVALID_ARG, "channel clipping needs window >= 1, the window means and flags");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nwin = chan ? (nsamp + window - 1) / window : 1;
  if (chan) {
    const int64_t wblocks = (nwin + kRfiThreads - 1) / kRfiThreads;
    if (wblocks > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "series too long");
    hipLaunchKernelGGL(chan_flag, dim3((unsigned)wblocks, (unsigned)nchan), dim3(kRfiThreads), 0, st, d_window_means,
                       nwin, d_fit, chan_threshold, d_flags);
    if (launched("channel flag") != hipSuccess) return DD_ERR_HIP;
  }
  if (sub) {
    const int64_t tblocks = (nsamp + kCorrSamples - 1) / kCorrSamples;
    if (tblocks > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "series too long");
    hipLaunchKernelGGL(chan_correct, dim3((unsigned)tblocks, (unsigned)nchan), dim3(kRfiThreads), 0, st, d_data, nsamp,
                       row_stride, chan ? window : nsamp, nwin, d_fit, chan ? d_flags : nullptr);
    if (launched("channel correct") != hipSuccess) return DD_ERR_HIP;
  } else if (chan) {
    const int64_t ablocks = (nwin + kRfiThreads - 1) / kRfiThreads;
    hipLaunchKernelGGL(chan_apply, dim3((unsigned)ablocks, (unsigned)nchan), dim3(kRfiThreads), 0, st, d_data, nsamp,
                       row_stride, window, nwin, d_fit, d_flags);
    if (launched("channel apply") != hipSuccess) return DD_ERR_HIP;
  }
  if (spec_threshold > 0.0) {
    const int64_t tblocks = (nsamp + 4 * kRfiThreads - 1) / (4 * kRfiThreads);
    if (tblocks > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "series too long");
    hipLaunchKernelGGL(spec_clip, dim3((unsigned)tblocks), dim3(kRfiThreads), 0, st, d_data, nchan, nsamp, row_stride,
                       d_fit, fit_mean, spec_threshold, (int)sub);
    if (launched("spectrum clip") != hipSuccess) return DD_ERR_HIP;
  }
  return DD_OK;
}

extern "C" int dd_bandpass_u8(const uint8_t* d_in, int64_t nchan, int64_t nsamp, int64_t row_stride, int64_t window,
                              double* d_avg, double* d_window_means, void* stream) {
  dd::clear_error();
  if (!d_in || !d_avg) return dd::fail(DD_ERR_INVALID_ARG, "input and average must be non-NULL");
  if (nchan < 1 || nsamp < 1 || row_stride < nsamp)
    return dd::fail(DD_ERR_INVALID_ARG, "need nchan >= 1, nsamp >= 1 and row_stride >= nsamp");
  if (window < 0 || (window > 0) != (d_window_means != nullptr))
    return dd::fail(DD_ERR_INVALID_ARG, "window means need window >= 1 and their buffer (or window 0 and NULL)");
  if (nchan > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "too many channels");
  const int64_t win = window > 0 ? window : nsamp;
  hipLaunchKernelGGL(bandpass_windows_u8, dim3((unsigned)nchan), dim3(kRfiThreads), 0, static_cast<hipStream_t>(stream),
                     d_in, nsamp, row_stride, win, (nsamp + win - 1) / win, d_avg, d_window_means);
  return launched("bandpass (8-bit)") == hipSuccess ? DD_OK : DD_ERR_HIP;
}

extern "C" int dd_rfi_clip_u8(uint8_t* d_data, int64_t nchan, int64_t nsamp, int64_t row_stride, const double* d_fit,
                              double chan_threshold, int64_t window, const double* d_window_means, int32_t* d_flags,
                              double fit_mean, double spec_threshold, void* stream) {
  dd::clear_error();
  if (!d_data || !d_fit) return dd::fail(DD_ERR_INVALID_ARG, "data and fit must be non-NULL");
  if (nchan < 1 || nsamp < 1 || row_stride < nsamp)
    return dd::fail(DD_ERR_INVALID_ARG, "need nchan >= 1, nsamp >= 1 and row_stride >= nsamp");
  if (nchan > 65535) return dd::fail(DD_ERR_UNSUPPORTED, "at most 65535 channels per call");
  const bool chan = chan_threshold > 0.0;
  if (chan && (window < 1 || !d_flags || !d_window_means))
    return dd::fail(DD_ERR_INVALID_ARG, "channel clipping needs window >= 1, the window means and flags");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (chan) {
    const int64_t nwin = (nsamp + window - 1) / window;
    const int64_t wblocks = (nwin + kRfiThreads - 1) / kRfiThreads;
    if (wblocks > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "series too long");
    hipLaunchKernelGGL(chan_flag, dim3((unsigned)wblocks, (unsigned)nchan), dim3(kRfiThreads), 0, st, d_window_means,
                       nwin, d_fit, chan_threshold, d_flags);
    if (launched("channel flag") != hipSuccess) return DD_ERR_HIP;
    hipLaunchKernelGGL(chan_apply_u8, dim3((unsigned)wblocks, (unsigned)nchan), dim3(kRfiThreads), 0, st, d_data,
                       nsamp, row_stride, window, nwin, d_fit, d_flags);
    if (launched("channel apply (8-bit)") != hipSuccess) return DD_ERR_HIP;
  }
  if (spec_threshold > 0.0) {
    const int64_t tblocks = (nsamp + 16 * 64 - 1) / (16 * 64);  // 16 samples per lane of a wavefront
    if (tblocks > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "series too long");
    hipLaunchKernelGGL(spec_clip_u8, dim3((unsigned)tblocks), dim3(kRfiThreads), 0, st, d_data, nchan, nsamp,
                       row_stride, d_fit, fit_mean, spec_threshold);
    if (launched("spectrum clip (8-bit)") != hipSuccess) return DD_ERR_HIP;
  }
  return DD_OK;
}
