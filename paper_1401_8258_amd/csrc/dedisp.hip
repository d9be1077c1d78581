// HIP kernels for gfx950 and the C-ABI entry points that launch them.
//
// Kernels (all wave64):
//   dedisp_tile    Eq. bruteEquation over one (DM group, time tile) per workgroup.
//                  The channel vectors a group needs (Eq. channelDispersionEquation:
//                  tile length plus the in-group delay spread) are staged HBM -> LDS
//                  a few channels per barrier pair and shared by every wavefront of
//                  the workgroup; each wavefront accumulates its own DM trials in
//                  VGPRs. Delays are wave-uniform and come in through scalar loads.
//   stats_*        per-series mean and standard deviation over fixed 8192-sample
//                  segments (wavefront reductions, FP64), then an in-order finalize.
//   cand_*         n-sigma detections: per-segment counts, one exclusive scan, and an
//                  ordered ballot compaction, so candidates come out in (d, t) order.
//   ring_append    copies a block into a stream's per-channel ring (wrap-aware).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>

#include "dd_internal.h"

namespace {

constexpr int kMaxThreads = 512;

__device__ __forceinline__ float to_f32(float x) { return x; }
__device__ __forceinline__ float to_f32(__half x) { return __half2float(x); }
__device__ __forceinline__ float to_f32(uint8_t x) { return (float)x; }

// Input view: linear rows, or a per-channel ring of ring_len samples in which
// window position p lives at (win0 + p) mod ring_len.
struct InView {
  const void* ptr;
  int64_t row_stride;  // elements between channel rows
  int64_t nvalid;      // window positions [0, nvalid) hold data
  int64_t ring_len;    // 0 for linear input
  int64_t win0;        // ring only: global sample of window position 0
};

// One workgroup = W wavefronts x G DM trials each, over T = 64 * S output samples.
// Lane l of every wavefront owns outputs t0 + l + 64 s, s < S.
template <typename TIn, int G, int S, bool RING>
__global__ __launch_bounds__(kMaxThreads) void dedisp_tile(
    InView in, const int32_t* __restrict__ dtab, int ndm_pad, int nchan, int ndm,
    float* __restrict__ out, int64_t out_stride, int64_t nout, int len_max, int cc_n) {
  constexpr int T = 64 * S;
  extern __shared__ float smem[];
  const int nt = blockDim.x;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gw = G * (nt >> 6);  // DM trials per workgroup
  const int64_t t0 = (int64_t)blockIdx.x * T;
  const int dg = blockIdx.y * gw;
  const int dw = dg + w * G;
  const TIn* src = static_cast<const TIn*>(in.ptr);

  float acc[G][S];
  float part[G][S];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int s = 0; s < S; ++s) acc[g][s] = 0.f, part[g][s] = 0.f;

  for (int c0 = 0; c0 < nchan; c0 += cc_n) {
    const int n_here = min(cc_n, nchan - c0);
    __syncthreads();
    for (int cc = 0; cc < n_here; ++cc) {
      const int c = c0 + cc;
      const int32_t* row = dtab + (int64_t)c * ndm_pad;
      const int base = row[dg];
      const int len = T + row[dg + gw - 1] - base;
      const int64_t first = t0 + base;  // window position of element 0
      const TIn* rp = src + (int64_t)c * in.row_stride;
      float* dst = smem + cc * len_max;
      if constexpr (RING) {
        int64_t start = (in.win0 + first) % in.ring_len;
        for (int j = threadIdx.x; j < len; j += nt) {
          int64_t p = start + j;
          if (p >= in.ring_len) p -= in.ring_len;
          dst[j] = (first + j < in.nvalid) ? to_f32(rp[p]) : 0.f;
        }
      } else {
        for (int j = threadIdx.x; j < len; j += nt)
          dst[j] = (first + j < in.nvalid) ? to_f32(rp[first + j]) : 0.f;
      }
    }
    __syncthreads();
    for (int cc = 0; cc < n_here; ++cc) {
      const int c = c0 + cc;
      if ((c & (DD_CHAN_BLOCK - 1)) == 0 && c != 0) {
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int s = 0; s < S; ++s) acc[g][s] += part[g][s], part[g][s] = 0.f;
      }
      const int32_t* row = dtab + (int64_t)c * ndm_pad;
      const int base = row[dg];
      const float* v = smem + cc * len_max + lane;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int k = row[dw + g] - base;
#pragma unroll
        for (int s = 0; s < S; ++s) part[g][s] += v[k + 64 * s];
      }
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int s = 0; s < S; ++s) acc[g][s] += part[g][s];

#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int d = dw + g;
    if (d >= ndm) break;
    float* orow = out + (int64_t)d * out_stride;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int64_t t = t0 + lane + 64 * s;
      if (t < nout) orow[t] = acc[g][s];
    }
  }
}

// ------------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over a 256-thread block in a fixed tree; result valid in thread 0.
__device__ double block_sum256(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
  return r;
}

// Segment partial sums of (x - x0) and (x - x0)^2 with x0 = the row's first value.
__global__ __launch_bounds__(256) void stats_partial(const float* __restrict__ out, int64_t stride,
                                                     int64_t nout, int64_t nseg, double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t seg = blockIdx.x;
  const int d = blockIdx.y;
  const float* row = out + (int64_t)d * stride;
  const double x0 = row[0];
  const int64_t b = seg * dd::kStatSeg;
  const int64_t e = min(nout, b + dd::kStatSeg);
  double s = 0.0, ss = 0.0;
  for (int64_t t = b + threadIdx.x; t < e; t += 256) {
    const double x = (double)row[t] - x0;
    s += x;
    ss += x * x;
  }
  s = block_sum256(s, red);
  ss = block_sum256(ss, red);
  if (threadIdx.x == 0) {
    part[((int64_t)d * nseg + seg) * 2] = s;
    part[((int64_t)d * nseg + seg) * 2 + 1] = ss;
  }
}

// stat[d] = {mean, rms, threshold} in FP64; mean/rms also as FP32 outputs.
__global__ __launch_bounds__(256) void stats_finalize(const float* __restrict__ out, int64_t stride,
                                                      const double* __restrict__ part, int64_t nseg,
                                                      int ndm, int64_t nout, double k, float* mean,
                                                      float* rms, double* stat) {
  const int d = blockIdx.x * 256 + threadIdx.x;
  if (d >= ndm) return;
  double s = 0.0, ss = 0.0;
  for (int64_t g = 0; g < nseg; ++g) {
    s += part[((int64_t)d * nseg + g) * 2];
    ss += part[((int64_t)d * nseg + g) * 2 + 1];
  }
  const double n = (double)nout;
  const double ms = s / n;
  double var = ss / n - ms * ms;
  if (var < 0.0) var = 0.0;
  const double m = (double)out[(int64_t)d * stride] + ms;
  const double r = sqrt(var);
  mean[d] = (float)m;
  rms[d] = (float)r;
  stat[d * 3] = m;
  stat[d * 3 + 1] = r;
  stat[d * 3 + 2] = m + k * r;
}

__global__ __launch_bounds__(256) void cand_count(const float* __restrict__ out, int64_t stride, int64_t nout,
                                                  int64_t nseg, const double* __restrict__ stat,
                                                  int32_t* __restrict__ cnt) {
  __shared__ double red[4];
  const int64_t seg = blockIdx.x;
  const int d = blockIdx.y;
  const float* row = out + (int64_t)d * stride;
  const double thr = stat[d * 3 + 2];
  const int64_t b = seg * dd::kStatSeg;
  const int64_t e = min(nout, b + dd::kStatSeg);
  int n = 0;
  for (int64_t t = b + threadIdx.x; t < e; t += 256) n += ((double)row[t] > thr) ? 1 : 0;
  const double tot = block_sum256((double)n, red);
  if (threadIdx.x == 0) cnt[(int64_t)d * nseg + seg] = (int32_t)tot;
}

// Exclusive scan of n counts by one 1024-thread block; total to *ncand.
__global__ __launch_bounds__(1024) void cand_scan(const int32_t* __restrict__ cnt, int64_t n,
                                                  int64_t* __restrict__ offs, int64_t* __restrict__ ncand) {
  __shared__ int64_t part[1024];
  const int tid = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t b = min(n, tid * chunk), e = min(n, b + chunk);
  int64_t local = 0;
  for (int64_t i = b; i < e; ++i) local += cnt[i];
  part[tid] = local;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int64_t run = part[tid] - local;
  for (int64_t i = b; i < e; ++i) {
    offs[i] = run;
    run += cnt[i];
  }
  if (tid == 1023) *ncand = part[1023];
}

__global__ __launch_bounds__(256) void cand_write(const float* __restrict__ out, int64_t stride, int64_t nout,
                                                  int64_t nseg, const double* __restrict__ stat,
                                                  const int32_t* __restrict__ cnt,
                                                  const int64_t* __restrict__ offs, dd_cand* __restrict__ cand,
                                                  int64_t cap, int64_t t_base) {
  __shared__ int wtot[4];
  const int64_t seg = blockIdx.x;
  const int d = blockIdx.y;
  const int64_t idx = (int64_t)d * nseg + seg;
  if (cnt[idx] == 0) return;
  int64_t off = offs[idx];
  const float* row = out + (int64_t)d * stride;
  const double m = stat[d * 3], r = stat[d * 3 + 1], thr = stat[d * 3 + 2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t b = seg * dd::kStatSeg;
  const int64_t e = min(nout, b + dd::kStatSeg);
  for (int64_t c0 = b; c0 < e; c0 += 256) {
    const int64_t t = c0 + threadIdx.x;
    const float x = t < e ? row[t] : 0.f;
    const bool hit = t < e && (double)x > thr;
    const uint64_t mask = __ballot(hit);
    const int below = __popcll(mask & ((1ull << lane) - 1ull));
    __syncthreads();
    if (lane == 0) wtot[w] = __popcll(mask);
    __syncthreads();
    int before = 0;
    for (int i = 0; i < w; ++i) before += wtot[i];
    const int total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
    if (hit) {
      const int64_t pos = off + before + below;
      if (pos < cap) {
        dd_cand o;
        o.dm_index = d;
        o.reserved = 0;
        o.t = t_base + t;
        o.value = x;
        o.snr = r > 0.0 ? (float)(((double)x - m) / r) : 0.f;
        cand[pos] = o;
      }
    }
    off += total;
  }
}

template <typename TIn>
__global__ __launch_bounds__(256) void ring_append(const TIn* __restrict__ blk, int64_t in_stride, int64_t n,
                                                   TIn* __restrict__ ring, int64_t ring_len, int64_t pos0) {
  const int c = blockIdx.y;
  const TIn* s = blk + (int64_t)c * in_stride;
  TIn* r = ring + (int64_t)c * ring_len;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    int64_t p = pos0 + j;
    if (p >= ring_len) p -= ring_len;
    r[p] = s[j];
  }
}

// ------------------------------------------------------------------ host side

using KernFn = void (*)(InView, const int32_t*, int, int, int, float*, int64_t, int64_t, int, int);

template <typename TIn, bool RING>
KernFn pick(int g, int s) {
  if (g == 4 && s == 4) return dedisp_tile<TIn, 4, 4, RING>;
  if (g == 4 && s == 8) return dedisp_tile<TIn, 4, 8, RING>;
  if (g == 4 && s == 16) return dedisp_tile<TIn, 4, 16, RING>;
  if (g == 8 && s == 4) return dedisp_tile<TIn, 8, 4, RING>;
  if (g == 8 && s == 8) return dedisp_tile<TIn, 8, 8, RING>;
  if (g == 16 && s == 4) return dedisp_tile<TIn, 16, 4, RING>;
  return nullptr;
}

KernFn pick_kernel(int dtype, bool ring, int g, int s) {
  if (dtype == DD_F32) return ring ? pick<float, true>(g, s) : pick<float, false>(g, s);
  if (dtype == DD_F16) return ring ? pick<__half, true>(g, s) : pick<__half, false>(g, s);
  return ring ? pick<uint8_t, true>(g, s) : pick<uint8_t, false>(g, s);
}

int hip_fail(hipError_t e, const char* what) {
  return dd::fail(DD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct Outputs {
  float* out;
  int64_t out_stride;
  float* mean;
  float* rms;
  float k;
  dd_cand* cand;
  int64_t cap;
  int64_t* ncand;
  int64_t t_base;
};

int64_t lds_limit_bytes() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 65536;
  return v;
}

// Dedisperse nout outputs of a prepared input view, then stats and candidates.
int run_pipeline(const dd_plan* p, const InView& in, const int32_t* d_table, int64_t nout, const Outputs& o,
                 char* ws, const dd::WsLayout& l, hipStream_t st) {
  const int g = p->tiles.g, s = p->tiles.s, w = p->tiles.w;
  const int T = 64 * s;
  const int len_max = (int)dd::align_up((int64_t)T + p->max_span, 4);
  const int64_t lds_cap = lds_limit_bytes();
  int cc_n = p->tiles.cc;
  while (cc_n > 1 && (int64_t)cc_n * len_max * 4 > lds_cap) --cc_n;
  const int64_t lds = (int64_t)cc_n * len_max * 4;
  if (lds > lds_cap)
    return dd::fail(DD_ERR_UNSUPPORTED, "delay spread of one DM group (" + std::to_string(p->max_span) +
                                            " samples) does not fit in LDS; use fewer DMs per workgroup");
  KernFn k = pick_kernel(p->dtype, in.ring_len > 0, g, s);
  if (!k) return dd::fail(DD_ERR_UNSUPPORTED, "no kernel for this tuning");
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  }
  const int64_t ntiles = (nout + T - 1) / T;
  if (ntiles > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "too many time tiles");
  dim3 grid((unsigned)ntiles, (unsigned)p->ngroups);
  hipLaunchKernelGGL(k, grid, dim3(64 * w), (size_t)lds, st, in, d_table, p->ndm_pad, p->nchan, p->ndm, o.out,
                     o.out_stride, nout, len_max, cc_n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "dedisp_tile launch");

  if (o.mean && o.rms) {
    double* part = reinterpret_cast<double*>(ws + l.part_off);
    double* stat = reinterpret_cast<double*>(ws + l.thr_off);
    const int64_t nseg = (nout + dd::kStatSeg - 1) / dd::kStatSeg;
    hipLaunchKernelGGL(stats_partial, dim3((unsigned)nseg, (unsigned)p->ndm), dim3(256), 0, st, o.out,
                       o.out_stride, nout, nseg, part);
    hipLaunchKernelGGL(stats_finalize, dim3((unsigned)((p->ndm + 255) / 256)), dim3(256), 0, st, o.out,
                       o.out_stride, part, nseg, p->ndm, nout, (double)o.k, o.mean, o.rms, stat);
    if (o.k > 0.f && o.ncand) {
      int32_t* cnt = reinterpret_cast<int32_t*>(ws + l.cnt_off);
      int64_t* offs = reinterpret_cast<int64_t*>(ws + l.offs_off);
      hipLaunchKernelGGL(cand_count, dim3((unsigned)nseg, (unsigned)p->ndm), dim3(256), 0, st, o.out,
                         o.out_stride, nout, nseg, stat, cnt);
      hipLaunchKernelGGL(cand_scan, dim3(1), dim3(1024), 0, st, cnt, nseg * p->ndm, offs, o.ncand);
      hipLaunchKernelGGL(cand_write, dim3((unsigned)nseg, (unsigned)p->ndm), dim3(256), 0, st, o.out,
                         o.out_stride, nout, nseg, stat, cnt, offs, o.cand, o.cand ? o.cap : 0, o.t_base);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "statistics/candidate launch");
  }
  return DD_OK;
}

int check_outputs(const dd_plan* p, float* d_out, int64_t out_stride, int64_t nout, float* d_mean, float* d_rms,
                  float k, dd_cand* d_cand, int64_t cap, int64_t* d_ncand) {
  if (!d_out) return dd::fail(DD_ERR_INVALID_ARG, "d_out is NULL");
  if (out_stride < nout) return dd::fail(DD_ERR_INVALID_ARG, "out_row_stride < nout");
  if ((d_mean == nullptr) != (d_rms == nullptr))
    return dd::fail(DD_ERR_INVALID_ARG, "d_mean and d_rms must both be given or both be NULL");
  if (k > 0.f && d_ncand && !d_mean) return dd::fail(DD_ERR_INVALID_ARG, "candidates need d_mean and d_rms");
  if (cap < 0 || (cap > 0 && !d_cand)) return dd::fail(DD_ERR_INVALID_ARG, "bad candidate buffer");
  (void)p;
  return DD_OK;
}

}  // namespace

extern "C" {

int dd_plan_upload(const dd_plan* p, void* d_workspace, int64_t ws_bytes, void* stream) {
  dd::clear_error();
  if (!p || !d_workspace) return dd::fail(DD_ERR_INVALID_ARG, "plan and workspace must be non-NULL");
  const int64_t need = (int64_t)p->dev_table.size() * 4;
  if (ws_bytes < need) return dd::fail(DD_ERR_WORKSPACE, "workspace smaller than the delay table");
  hipError_t e = hipMemcpyAsync(d_workspace, p->dev_table.data(), (size_t)need, hipMemcpyHostToDevice,
                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (delay table)");
  return DD_OK;
}

int dd_dedisperse(const dd_plan* p, const void* d_in, int64_t nsamp, int64_t in_row_stride, float* d_out,
                  int64_t out_row_stride, float* d_mean, float* d_rms, float k_sigma, dd_cand* d_cand,
                  int64_t cand_cap, int64_t* d_ncand, void* d_workspace, int64_t ws_bytes, void* stream) {
  dd::clear_error();
  if (!p || !d_in || !d_workspace) return dd::fail(DD_ERR_INVALID_ARG, "plan, input and workspace are required");
  if (nsamp <= p->maxdelay)
    return dd::fail(DD_ERR_TOO_SHORT, "nsamp must exceed maxdelay (" + std::to_string(p->maxdelay) + ")");
  if (in_row_stride < nsamp) return dd::fail(DD_ERR_INVALID_ARG, "in_row_stride < nsamp");
  const int64_t nout = nsamp - p->maxdelay;
  int rc = check_outputs(p, d_out, out_row_stride, nout, d_mean, d_rms, k_sigma, d_cand, cand_cap, d_ncand);
  if (rc) return rc;
  const dd::WsLayout l = dd::workspace_layout(p, nsamp);
  if (ws_bytes < l.total) return dd::fail(DD_ERR_WORKSPACE, "workspace smaller than dd_plan_query asks for");
  InView in{d_in, in_row_stride, nsamp, 0, 0};
  Outputs o{d_out, out_row_stride, d_mean, d_rms, k_sigma, d_cand, cand_cap, d_ncand, 0};
  char* ws = static_cast<char*>(d_workspace);
  return run_pipeline(p, in, reinterpret_cast<const int32_t*>(ws + l.table_off), nout, o, ws, l,
                      static_cast<hipStream_t>(stream));
}

int dd_stream_create(const dd_plan* p, int64_t block_nsamp, void* d_ring, int64_t ring_bytes, void* stream,
                     dd_stream** out) {
  dd::clear_error();
  if (!out) return dd::fail(DD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!p || !d_ring) return dd::fail(DD_ERR_INVALID_ARG, "plan and ring must be non-NULL");
  if (block_nsamp < 1) return dd::fail(DD_ERR_INVALID_ARG, "block_nsamp must be >= 1");
  dd_plan_info info;
  dd_plan_query(p, block_nsamp, &info);
  dd::clear_error();
  if (ring_bytes < info.ring_bytes) return dd::fail(DD_ERR_WORKSPACE, "ring smaller than dd_plan_query asks for");
  dd_stream* s = new (std::nothrow) dd_stream();
  if (!s) return dd::fail(DD_ERR_INVALID_ARG, "out of host memory");
  s->plan = p;
  s->block = block_nsamp;
  s->ring_len = dd::align_up(block_nsamp + (int64_t)p->maxdelay, 64);
  s->ring = d_ring;
  hipError_t e = hipMemcpyAsync(d_ring, p->dev_table.data(), p->dev_table.size() * 4, hipMemcpyHostToDevice,
                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipMemcpyAsync (delay table)");
  }
  *out = s;
  return DD_OK;
}

void dd_stream_destroy(dd_stream* s) { delete s; }

int dd_stream_append(dd_stream* s, const void* d_block, int64_t nsamp, int64_t in_row_stride, int64_t seq,
                     void* stream, int64_t* t0_out, int64_t* nout_out) {
  dd::clear_error();
  if (t0_out) *t0_out = 0;
  if (nout_out) *nout_out = 0;
  if (!s || !d_block) return dd::fail(DD_ERR_INVALID_ARG, "stream and block must be non-NULL");
  if (seq != s->next_seq)
    return dd::fail(DD_ERR_SEQUENCE, "expected seq " + std::to_string(s->next_seq) + ", got " + std::to_string(seq));
  if (nsamp < 1 || nsamp > s->block) return dd::fail(DD_ERR_INVALID_ARG, "block size out of range");
  if (in_row_stride < nsamp) return dd::fail(DD_ERR_INVALID_ARG, "in_row_stride < nsamp");
  if (s->pending_n > 0) return dd::fail(DD_ERR_SEQUENCE, "previous window not dedispersed yet");
  const dd_plan* p = s->plan;
  char* ring = static_cast<char*>(s->ring) + dd::ring_table_bytes(p);
  const int64_t pos0 = s->received % s->ring_len;
  const unsigned gx = (unsigned)std::min<int64_t>((nsamp + 255) / 256, 1024);
  dim3 grid(gx, (unsigned)p->nchan);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->dtype == DD_F32)
    hipLaunchKernelGGL(ring_append<float>, grid, dim3(256), 0, st, static_cast<const float*>(d_block), in_row_stride,
                       nsamp, reinterpret_cast<float*>(ring), s->ring_len, pos0);
  else if (p->dtype == DD_F16)
    hipLaunchKernelGGL(ring_append<__half>, grid, dim3(256), 0, st, static_cast<const __half*>(d_block),
                       in_row_stride, nsamp, reinterpret_cast<__half*>(ring), s->ring_len, pos0);
  else
    hipLaunchKernelGGL(ring_append<uint8_t>, grid, dim3(256), 0, st, static_cast<const uint8_t*>(d_block),
                       in_row_stride, nsamp, reinterpret_cast<uint8_t*>(ring), s->ring_len, pos0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "ring_append launch");
  s->received += nsamp;
  s->next_seq += 1;
  const int64_t t1 = s->received - p->maxdelay;
  if (t1 <= s->emitted) return DD_FILLING;
  s->pending_t0 = s->emitted;
  s->pending_n = t1 - s->emitted;
  s->emitted = t1;
  if (t0_out) *t0_out = s->pending_t0;
  if (nout_out) *nout_out = s->pending_n;
  return DD_OK;
}

int dd_stream_push(dd_stream* s, const void* d_block, int64_t nsamp, int64_t in_row_stride, int64_t seq,
                   float* d_out, int64_t out_row_stride, float* d_mean, float* d_rms, float k_sigma,
                   dd_cand* d_cand, int64_t cand_cap, int64_t* d_ncand, void* d_workspace, int64_t ws_bytes,
                   void* stream, int64_t* t0_out, int64_t* nout_out) {
  dd::clear_error();
  if (t0_out) *t0_out = 0;
  if (nout_out) *nout_out = 0;
  if (!s || !d_workspace) return dd::fail(DD_ERR_INVALID_ARG, "stream and workspace must be non-NULL");
  const dd_plan* p = s->plan;
  int rc = check_outputs(p, d_out, out_row_stride, s->block, d_mean, d_rms, k_sigma, d_cand, cand_cap, d_ncand);
  if (rc) return rc;
  const dd::WsLayout l = dd::workspace_layout(p, s->block);
  if (ws_bytes < l.total) return dd::fail(DD_ERR_WORKSPACE, "workspace smaller than dd_plan_query asks for");
  int64_t t0 = 0, n = 0;
  rc = dd_stream_append(s, d_block, nsamp, in_row_stride, seq, stream, &t0, &n);
  if (rc != DD_OK) return rc;
  s->pending_n = 0;
  InView in{static_cast<char*>(s->ring) + dd::ring_table_bytes(p), s->ring_len, n + p->maxdelay, s->ring_len, t0};
  Outputs o{d_out, out_row_stride, d_mean, d_rms, k_sigma, d_cand, cand_cap, d_ncand, t0};
  rc = run_pipeline(p, in, static_cast<const int32_t*>(s->ring), n, o, static_cast<char*>(d_workspace), l,
                    static_cast<hipStream_t>(stream));
  if (rc) return rc;
  if (t0_out) *t0_out = t0;
  if (nout_out) *nout_out = n;
  return DD_OK;
}

int dd_batch_query(const dd_batch_item* items, int32_t n, int64_t* ws_bytes) {
  dd::clear_error();
  (void)items;
  (void)n;
  if (ws_bytes) *ws_bytes = 0;
  return dd::fail(DD_ERR_UNSUPPORTED, "batched launch not built yet");
}

int dd_batch_dedisperse(const dd_batch_item* items, int32_t n, void* d_workspace, int64_t ws_bytes, void* stream) {
  dd::clear_error();
  (void)items;
  (void)n;
  (void)d_workspace;
  (void)ws_bytes;
  (void)stream;
  return dd::fail(DD_ERR_UNSUPPORTED, "batched launch not built yet");
}

}  // extern "C"
