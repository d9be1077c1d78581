// Boxcar smoothing of (normalised) dedispersed series by successive addition of adjacent
// samples: the single-pulse search's smoothing, which downfactors the series by the
// boxcar width (Ch. 2 single-pulse detection; Ch. 6 template matching). C-ABI entry
// point dd_boxcar. Then boxcar template matching at every start offset with
// thresholding (dd_boxcar_search), below.
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
#include "dd_device.h"

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
  // level 0 is the series itself; whole 4-sample chunks of an aligned output row are
  // stored with one 16-byte (level 0) and one 8-byte (level 1, n even) store
  const bool ovec = (reinterpret_cast<uintptr_t>(orow) & 15) == 0 && s0 + 3 < n;
  if (ovec) {
    *reinterpret_cast<float4*>(orow + s0) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (s0 + i < n) orow[s0 + i] = v[i];
  }
  if (levels >= 1) {
    const int64_t off = n;
    const float norm = 0.70710678118654752f;
    const float a = v[0] + v[1], b = v[2] + v[3];
    const int64_t j = s0 >> 1;
    if (ovec && (n & 1) == 0) {
      *reinterpret_cast<float2*>(orow + off + j) = make_float2(a * norm, b * norm);
    } else {
      if (((j + 1) << 1) <= n) orow[off + j] = a * norm;
      if (((j + 2) << 1) <= n) orow[off + j + 1] = b * norm;
    }
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

// ------------------------------------------------------------------ boxcar search
//
// Template matching (Ch. 6 "Transient Surveys": boxcars of varying width convolved with each
// dedispersed series, then thresholded): for w = 2^j, j <= max_log2 <= 6, B_w[t] = x[t] +
// ... + x[t + w - 1] at every start t with t + w <= n, S/N_w[t] = (B_w[t] - w mean) /
// (rms sqrt(w)); a detection at (row, t) when the best width's S/N exceeds k (the smallest
// width on ties), reported with that width, B_w and S/N, rows in order and t ascending.
//
// One 256-thread workgroup per (row, segment of kSearchSeg starts). The segment and 64
// samples past it are read once into LDS with 16-byte loads (zeros past n, which no
// defined boxcar reads), 4 padding words after every 16 samples. Thread i then owns the 16
// consecutive starts 16 i .. 16 i + 15 and copies the 80 samples they need into registers
// (20 conflict-free ds_read_b128: threads 20 words apart cover all 64 banks per 16 lanes).
// Level j is formed in place from level j - 1 by B_2w[t] = B_w[t] + B_w[t + w] (a pairwise
// FP32 tree, the same order at every start), and after each level the thread updates the
// best S/N of its starts. S/N is FP32: w * mean is exact (w is a power of two), so the
// difference is rounded once, and the reciprocal 1 / (rms sqrt(w)) is formed in FP64 and
// rounded once. A counting pass, a scan of the counts and a writing pass that recomputes
// the segment place the detections; each pass reads the series once (HBM-bound).
constexpr int kSearchSeg = 4096;
constexpr int kSearchPer = kSearchSeg / kBoxThreads;  // consecutive starts per thread
constexpr int kSearchWin = kSearchPer + 64;           // samples a thread's starts need (80)
constexpr int kSearchSamples = kSearchSeg + 64;       // samples a segment needs
constexpr int kSearchLds = kSearchSamples / 16 * 20;  // LDS words with the padding

__device__ __forceinline__ int pad_pos(int a) { return a + 4 * (a >> 4); }

struct SearchArgs {
  const float* x;
  int64_t n, stride;
  const float* mean;  // null: 0 (normalised series)
  const float* rms;   // null: 1
  int max_log2;
  float k;
};

// Levels 0 .. max_log2 of one thread's window, in place, and the best S/N of its starts:
// start q takes width w when q + w <= lim (CHECKED; otherwise every width fits). The
// updates are selects, not branches: a start's best changes only on a strictly larger S/N,
// so ties keep the smaller width. COUNT: only the best S/N, as a maximum over the same S/N
// values (the counting pass needs neither the width nor the sum; the maximum decides
// "best > k" exactly as the selects do).
template <bool CHECKED, bool COUNT>
__device__ __forceinline__ void search_levels(float (&x)[kSearchWin], float (&best)[kSearchPer],
                                              int (&bj)[kSearchPer], float (&bval)[kSearchPer], int lim, float m,
                                              double r, int max_log2) {
#pragma unroll
  for (int j = 0; j <= kMaxLevel; ++j) {
    if (j > max_log2) break;
    const int w = 1 << j;
    if (j > 0) {
      // in place, ascending: B_w[t] for t + w <= kSearchWin from B_{w/2}[t], B_{w/2}[t + w/2]
#pragma unroll
      for (int t = 0; t + w <= kSearchWin; ++t) x[t] = x[t] + x[t + (w >> 1)];
    }
    // wave-uniform constants of the width, kept in scalar registers (readfirstlane of a
    // uniform value is exact), so a caller's loop does not hold them in vector registers
    const float mw = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(m * (float)w)));
    const float inv =
        __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int((float)(1.0 / (r * sqrt((double)w))))));
#pragma unroll
    for (int q = 0; q < kSearchPer; ++q) {
      const float snr = (x[q] - mw) * inv;
      if constexpr (COUNT) {
        if (!CHECKED || q + w <= lim) best[q] = __builtin_fmaxf(best[q], snr);
      } else {
        const bool up = snr > best[q] && (!CHECKED || q + w <= lim);
        bval[q] = up ? x[q] : bval[q];
        bj[q] = up ? j : bj[q];
        best[q] = up ? snr : best[q];
      }
    }
  }
}

// The best S/N over the widths (and, unless COUNT, its width index and boxcar sum) for this
// thread's starts of segment seg of row d; false when the row has no variance (the same for
// every thread of the workgroup, before any barrier).
template <bool COUNT>
__device__ __forceinline__ bool search_segment(const SearchArgs& A, int d, int64_t seg, float* buf,
                                               float (&best)[kSearchPer], int (&bj)[kSearchPer],
                                               float (&bval)[kSearchPer]) {
  const int tid = threadIdx.x;
  const int64_t b = seg * kSearchSeg;
  const float* row = A.x + (int64_t)d * A.stride + b;
  const float m = A.mean ? A.mean[d] : 0.0f;
  const double r = A.rms ? (double)A.rms[d] : 1.0;
#pragma unroll
  for (int q = 0; q < kSearchPer; ++q) {
    best[q] = -INFINITY;
    bj[q] = 0;
    bval[q] = 0.0f;
  }
  if (!(r > 0.0)) return false;
  const int64_t navail = A.n - b;  // samples of the row from the segment start on
  const bool vec = (reinterpret_cast<uintptr_t>(row) & 15) == 0;
  for (int i = tid; i < kSearchSamples / 4; i += kBoxThreads) {
    const int a = 4 * i;
    float4 v;
    if (vec && a + 3 < navail) {
      v = *reinterpret_cast<const float4*>(row + a);
    } else {
      v.x = a < navail ? row[a] : 0.0f;
      v.y = a + 1 < navail ? row[a + 1] : 0.0f;
      v.z = a + 2 < navail ? row[a + 2] : 0.0f;
      v.w = a + 3 < navail ? row[a + 3] : 0.0f;
    }
    *reinterpret_cast<float4*>(buf + pad_pos(a)) = v;
  }
  __syncthreads();
  float x[kSearchWin];
  const int a0 = kSearchPer * tid;
#pragma unroll
  for (int c = 0; c < kSearchWin / 4; ++c) {
    const float4 v = *reinterpret_cast<const float4*>(buf + pad_pos(a0 + 4 * c));
    x[4 * c] = v.x;
    x[4 * c + 1] = v.y;
    x[4 * c + 2] = v.z;
    x[4 * c + 3] = v.w;
  }
  // every start of every width lies inside the row unless this is the row's last segment
  const int lim = (int)min<int64_t>(A.n - (b + a0), (int64_t)kSearchWin);
  if (lim >= kSearchWin)
    search_levels<false, COUNT>(x, best, bj, bval, lim, m, r, A.max_log2);
  else
    search_levels<true, COUNT>(x, best, bj, bval, lim, m, r, A.max_log2);
  return true;
}

// Counting pass: workgroup (g, d) counts segments kCountSegs g .. kCountSegs (g + 1) - 1 of
// row d. A segment that lies wholly inside the row reaches LDS by DMA (one wavefront
// instruction per 64-sample run, 4 padding words after each run), double-buffered: the
// next segment's DMAs are in flight while this one is searched. A row's last, partial
// segment is loaded through registers. Each segment's count is the integer number of its
// starts whose best S/N exceeds k, decided as in the writing pass.
constexpr int kCountSegs = 8;                                 // segments per counting workgroup
constexpr int kRun = 64;                                      // samples per DMA instruction
constexpr int kRunPad = 4;                                    // LDS words after each run
constexpr int kRuns = kSearchSamples / kRun;                  // 65 runs per segment
constexpr int kRunWords = kRuns * (kRun + kRunPad);           // one buffer
static_assert(kSearchSamples % kRun == 0, "a segment is whole runs");
__device__ __forceinline__ int pad_run(int a) { return a + kRunPad * (a >> 6); }

__global__ __launch_bounds__(kBoxThreads) void boxcar_count(SearchArgs A, int64_t nseg, int32_t* __restrict__ cnt) {
  __shared__ __align__(16) float buf[2][kRunWords];
  __shared__ int wsum[2][kBoxThreads / 64];
  const int d = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: the DMAs' LDS address is scalar
  const int64_t seg0 = (int64_t)blockIdx.x * kCountSegs;
  const int nmine = (int)min<int64_t>(kCountSegs, nseg - seg0);  // >= 1: the grid covers nseg
  const float* row = A.x + (int64_t)d * A.stride;
  const float m = A.mean ? A.mean[d] : 0.0f;
  const double r = A.rms ? (double)A.rms[d] : 1.0;
  if (!(r > 0.0)) {  // no variance: no detections (the same for the whole workgroup)
    if (tid < nmine) cnt[(int64_t)d * nseg + seg0 + tid] = 0;
    return;
  }
  const int ndma = (kRuns - wv + 3) / 4;  // this wavefront's DMAs per segment: runs wv, wv + 4, ...
  auto full = [&](int64_t seg) { return A.n - seg * kSearchSeg >= kSearchSamples; };
  auto issue = [&](int64_t seg, int b) {  // a whole segment: every sample it reads is inside the row
    const float* src = row + seg * kSearchSeg;
    const unsigned lb = dd::lds_addr(&buf[b][0]);
    for (int rr = wv; rr < kRuns; rr += 4)
      dd::dma<4>(src, (unsigned)(4 * (rr * kRun + lane)),
                 __builtin_amdgcn_readfirstlane(lb + 4u * (unsigned)(rr * (kRun + kRunPad))));
  };
  // the row's last segment, through registers: -inf past the row, so that every window
  // reaching past it sums to -inf (or NaN) and never wins the maximum, the count the writing
  // pass's bound check gives
  auto load_regs = [&](int64_t seg, int b) {
    const int64_t navail = A.n - seg * kSearchSeg;
    const float* src = row + seg * kSearchSeg;
    for (int a = tid; a < kSearchSamples; a += kBoxThreads) buf[b][pad_run(a)] = a < navail ? src[a] : -INFINITY;
  };
  if (full(seg0)) issue(seg0, 0);
  else load_regs(seg0, 0);
  for (int j = 0; j < nmine; ++j) {
    const int64_t seg = seg0 + j;
    const int b = j & 1;
    const bool next_dma = j + 1 < nmine && full(seg + 1);
    if (next_dma) issue(seg + 1, b ^ 1);  // buffer b ^ 1 was last read before the previous barrier
    dd::wait_vm(next_dma ? ndma : 0);     // this segment's DMAs have landed (the next ones may not)
    __syncthreads();                      // ... for every wavefront; register-loaded samples too
    float x[kSearchWin];
    const int a0 = kSearchPer * tid;
#pragma unroll
    for (int c = 0; c < kSearchWin / 4; ++c) {
      const float4 v = *reinterpret_cast<const float4*>(&buf[b][pad_run(a0 + 4 * c)]);
      x[4 * c] = v.x;
      x[4 * c + 1] = v.y;
      x[4 * c + 2] = v.z;
      x[4 * c + 3] = v.w;
    }
    float best[kSearchPer];
    int bj[kSearchPer];
    float bval[kSearchPer];
#pragma unroll
    for (int q = 0; q < kSearchPer; ++q) best[q] = -INFINITY, bj[q] = 0, bval[q] = 0.0f;
    search_levels<false, true>(x, best, bj, bval, kSearchWin, m, r, A.max_log2);
    int c = 0;
#pragma unroll
    for (int q = 0; q < kSearchPer; ++q) c += best[q] > A.k ? 1 : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) wsum[b][wv] = c;
    __syncthreads();  // every wavefront is done with buffer b; the four counts are in LDS
    if (tid == 0) cnt[(int64_t)d * nseg + seg] = wsum[b][0] + wsum[b][1] + wsum[b][2] + wsum[b][3];
    if (j + 1 < nmine && !next_dma) load_regs(seg + 1, b ^ 1);
  }
}

// Detections in ascending t: thread i's starts precede thread i + 1's, so a thread's slot
// is the segment offset plus the exclusive prefix sum of the hit counts over threads
// (inclusive scan inside each wavefront, the wavefront totals through LDS).
__global__ __launch_bounds__(kBoxThreads) void boxcar_write(SearchArgs A, int64_t nseg, const int32_t* __restrict__ cnt,
                                                            const int64_t* __restrict__ offs, dd_pulse* __restrict__ out,
                                                            int64_t cap) {
  __shared__ __align__(16) float buf[kSearchLds];
  __shared__ int wtot[kBoxThreads / 64];
  const int d = blockIdx.y;
  const int64_t seg = blockIdx.x;
  const int64_t idx = (int64_t)d * nseg + seg;
  if (cnt[idx] == 0) return;  // the whole workgroup leaves together
  float best[kSearchPer];
  int bj[kSearchPer];
  float bval[kSearchPer];
  search_segment<false>(A, d, seg, buf, best, bj, bval);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int c = 0;
#pragma unroll
  for (int q = 0; q < kSearchPer; ++q) c += best[q] > A.k ? 1 : 0;
  int incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  int before = incl - c;
  for (int i = 0; i < w; ++i) before += wtot[i];
  int64_t pos = offs[idx] + before;
  const int64_t t0 = seg * kSearchSeg + kSearchPer * threadIdx.x;
#pragma unroll
  for (int q = 0; q < kSearchPer; ++q) {
    if (best[q] > A.k) {
      if (pos < cap) {
        dd_pulse o;
        o.row = d;
        o.width = 1 << bj[q];
        o.t = t0 + q;
        o.value = bval[q];
        o.snr = best[q];
        out[pos] = o;
      }
      ++pos;
    }
  }
}

struct SearchLayout {
  int64_t nseg, cnt_off, offs_off, total;
};

SearchLayout search_layout(int64_t nrows, int64_t n) {
  SearchLayout l{};
  l.nseg = (n + kSearchSeg - 1) / kSearchSeg;
  l.cnt_off = 0;
  l.offs_off = dd::align_up(nrows * l.nseg * 4);
  l.total = l.offs_off + dd::align_up(nrows * l.nseg * 8);
  return l;
}

}  // namespace

extern "C" int dd_boxcar_search_workspace(int64_t nrows, int64_t n, int64_t* ws_bytes) {
  dd::clear_error();
  if (!ws_bytes) return dd::fail(DD_ERR_INVALID_ARG, "ws_bytes is NULL");
  *ws_bytes = 0;
  if (nrows < 1 || n < 1) return dd::fail(DD_ERR_INVALID_ARG, "need nrows >= 1 and n >= 1");
  *ws_bytes = search_layout(nrows, n).total;
  return DD_OK;
}

extern "C" int dd_boxcar_search(const float* d_series, int64_t nrows, int64_t n, int64_t row_stride,
                                const float* d_mean, const float* d_rms, int32_t max_log2, float k_sigma,
                                dd_pulse* d_pulse, int64_t cap, int64_t* d_npulse, void* d_workspace,
                                int64_t ws_bytes, void* stream) {
  dd::clear_error();
  if (!d_series || !d_npulse || !d_workspace)
    return dd::fail(DD_ERR_INVALID_ARG, "series, count and workspace must be non-NULL");
  if (nrows < 1 || n < 1 || row_stride < n)
    return dd::fail(DD_ERR_INVALID_ARG, "need nrows >= 1, n >= 1 and row_stride >= n");
  if ((d_mean == nullptr) != (d_rms == nullptr))
    return dd::fail(DD_ERR_INVALID_ARG, "d_mean and d_rms must both be given or both be NULL");
  if (max_log2 < 0 || max_log2 > kMaxLevel)
    return dd::fail(DD_ERR_INVALID_ARG, "max_log2 must be in 0..6 (boxcars of 1..64 samples)");
  if (!std::isfinite(k_sigma)) return dd::fail(DD_ERR_INVALID_ARG, "k_sigma must be finite");
  if (cap < 0 || (cap > 0 && !d_pulse)) return dd::fail(DD_ERR_INVALID_ARG, "bad detection buffer");
  if (nrows > 65535) return dd::fail(DD_ERR_UNSUPPORTED, "at most 65535 rows per call");
  const SearchLayout l = search_layout(nrows, n);
  if (ws_bytes < l.total) return dd::fail(DD_ERR_WORKSPACE, "workspace smaller than dd_boxcar_search_workspace");
  if (l.nseg > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "series too long");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(d_workspace);
  int32_t* cnt = reinterpret_cast<int32_t*>(ws + l.cnt_off);
  int64_t* offs = reinterpret_cast<int64_t*>(ws + l.offs_off);
  const SearchArgs A{d_series, n, row_stride, d_mean, d_rms, (int)max_log2, k_sigma};
  const dim3 grid((unsigned)l.nseg, (unsigned)nrows);
  const dim3 cgrid((unsigned)((l.nseg + kCountSegs - 1) / kCountSegs), (unsigned)nrows);
  hipLaunchKernelGGL(boxcar_count, cgrid, dim3(kBoxThreads), 0, st, A, l.nseg, cnt);
  const int rc = dd::launch_count_scan(cnt, nrows * l.nseg, offs, d_npulse, st);
  if (rc) return rc;
  hipLaunchKernelGGL(boxcar_write, grid, dim3(kBoxThreads), 0, st, A, l.nseg, cnt, offs, d_pulse, cap);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return dd::fail(DD_ERR_HIP, std::string("boxcar search launch: ") + hipGetErrorString(e));
  return DD_OK;
}

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
