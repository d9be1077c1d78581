// Direct-read form of the dedispersion kernel for 8-bit input: gfx950, wave64.
//
// Eq. bruteEquation, D[d][t] = sum_c A[c][t + delay(c, d)], over one (S x 1024-sample time
// tile, group of G W DM trials) per workgroup of W wavefronts. Wavefront w owns trials
// dg + G w .. dg + G w + G - 1; lane l owns output samples t0 + 1024 u + 16 l .. + 15 of
// each sub-tile u < S. A second sub-tile reuses each trial's scalar offset work and halves
// the re-reads of a channel's delay range per output (one per 2048-sample tile).
//
// Nothing is staged in LDS. The input is held as four copies per channel, copy m shifted
// by m samples (copy m at position p holds sample p + m), so a trial whose window starts
// at sample s reads copy s & 3 at the 4-byte aligned position s - (s & 3). Per channel a
// wavefront then reads, per trial, one aligned 16-byte buffer load per lane (1 KB per
// wavefront) served by the L1 and L2 caches: the trials of a group and the groups of a
// tile read overlapping windows. (Loads at byte-aligned offsets move about a quarter of
// the bytes per clock that 4-byte aligned ones do, whatever their width.) This suits
// beams whose delays grow by many samples per DM trial (low frequencies, wide bands),
// where a window staged in LDS is shared by few trials. The loads of the next channel are
// in flight while the current one is summed.
//
// Sums: each dword of four codes splits into the 16-bit pairs (s0, s2) and (s1, s3) with a
// mask and a shift (plain VALU operations that issue at full rate); the pairs add with
// 32-bit adds and fold into 32-bit sums every 256 channels (255 * 256 < 2^16), so the sums
// are exact integers, equal to every other form's. The FP64 statistics partials of a
// (trial, 512-sample segment) are sums of exact integers below 2^53, so they do not depend
// on the order either.
//
// The copies: for a plain call a prep kernel writes them into the workspace, zero past the
// input's end and long enough for every window of the last tile; a stream's ring holds
// them directly (ring_append_quad), each copy a ring of the stream's ring length with a
// mirror of at least a tile past its end, so no window wraps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "dd_internal.h"
#include "dd_device.h"

namespace {

constexpr int kDrLane = 16;                // output samples per lane and sub-tile
constexpr int kDrTile = 64 * kDrLane;      // output samples per sub-tile
static_assert(kDrTile == 2 * dd::kTile, "a sub-tile is two statistics segments");
static_assert(kDrTile == dd::kDirectTile, "sub-tile disagrees with the plan");
// Buffer resource word 3 for raw (unswizzled, stride 0) buffers on gfx9-family devices.
constexpr int kRsrcWord3 = 0x00020000;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct DRParams {
  const uint8_t* quad;  // [nchan][4][lq]: copy m of channel c at quad + (4 c + m) lq
  int64_t lq;           // bytes per copy row
  int64_t ring_len;     // stream ring length (0: linear input, no wrap)
  int64_t w0;           // stream: ring position of window position 0
  const int32_t* dtab;  // [nchan][ndm_pad] delay of each trial (padded trials repeat the last DM)
  float* out;
  double* part;         // [ndm][nseg][2] per 512-sample segment, or null
  int64_t out_stride, nout, nitems, nseg;
  int nchan, ndm, ndm_pad, ngroups;
  int nw;               // wavefronts per workgroup
  int tiles_g;          // DM trials per wavefront
  int tiles_s;          // 1024-sample sub-tiles per wavefront tile
  int pad_;
};
static_assert(sizeof(DRParams) % 4 == 0, "DRParams is copied as dwords");

template <int G, int S>
struct DirectTile {
  uint32_t pr[G][S][8];    // 16-bit pairs: (s0, s2), (s1, s3) of dwords 0..3
  uint32_t acc[G][S][16];  // per sample

  __device__ __forceinline__ void fold() {
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int u = 0; u < S; ++u) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t a = pr[g][u][2 * k], b = pr[g][u][2 * k + 1];
          acc[g][u][4 * k] += a & 0xffffu;
          acc[g][u][4 * k + 2] += a >> 16;
          acc[g][u][4 * k + 1] += b & 0xffffu;
          acc[g][u][4 * k + 3] += b >> 16;
          pr[g][u][2 * k] = 0u;
          pr[g][u][2 * k + 1] = 0u;
        }
      }
    }
  }

  __device__ __forceinline__ void add(const u32x4 (&v)[G][S]) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int u = 0; u < S; ++u) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t x = v[g][u][k];
          pr[g][u][2 * k] += x & 0x00ff00ffu;
          pr[g][u][2 * k + 1] += (x >> 8) & 0x00ff00ffu;
        }
      }
    }
  }

  // the sub-tiles of a trial read consecutive 1 KB windows at one scalar offset (the
  // instruction's immediate offset adds 1024 per sub-tile)
  __device__ __forceinline__ void load(const DRParams& P, int c, int t0w, int lane, dd::ci32_t tab,
                                       u32x4 (&v)[G][S]) {
    const int64_t row4 = 4 * P.lq;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(P.quad + (int64_t)c * row4), (short)0, (int)row4, kRsrcWord3);
    const dd::ci32_t drow = tab + (int64_t)c * P.ndm_pad;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      int s = t0w + drow[g];
      if (P.ring_len && s >= (int)P.ring_len) s -= (int)P.ring_len;
      const int m = s & 3;
#pragma unroll
      for (int u = 0; u < S; ++u)
        v[g][u] = __builtin_amdgcn_raw_buffer_load_b128(rs, kDrLane * lane + kDrTile * u, m * (int)P.lq + (s - m), 0);
    }
  }

  __device__ __forceinline__ void run(const DRParams& P, int64_t tile, int grp) {
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t0 = tile * (kDrTile * S);
    const int dw = grp * G * P.nw + w * G;
    if (dw >= P.ndm_pad) return;  // a batched item regrouped to more wavefronts than its plan's
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int u = 0; u < S; ++u) {
#pragma unroll
        for (int q = 0; q < 8; ++q) pr[g][u][q] = 0u;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[g][u][q] = 0u;
      }
    }
    const dd::ci32_t tab = (dd::ci32_t)(P.dtab + dw);
    const int t0w = (int)(t0 + P.w0);  // window position 0 of this tile (ring: < ring_len + tile)
    const int nchan = P.nchan;
    u32x4 va[G][S], vb[G][S];
    load(P, 0, t0w, lane, tab, va);
    // channel pairs (c, c + 1): the loads of the next channel are issued before the adds
    for (int c = 0; c < nchan; c += 2) {
      if (c + 1 < nchan) load(P, c + 1, t0w, lane, tab, vb);
      if ((c & 255) == 0 && c != 0) fold();
      add(va);
      if (c + 1 >= nchan) break;
      if (c + 2 < nchan) load(P, c + 2, t0w, lane, tab, va);
      add(vb);
    }
    fold();

    const bool vec_ok = ((P.out_stride & 3) == 0) && ((reinterpret_cast<uintptr_t>(P.out) & 15) == 0);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int d = dw + g;
      if (d >= P.ndm) break;
      float* orow = P.out + (int64_t)d * P.out_stride;
#pragma unroll
      for (int u = 0; u < S; ++u) {
        const int64_t tb = t0 + kDrTile * u + kDrLane * lane;
        const int64_t seg = (t0 + kDrTile * u) / dd::kTile + (lane >> 5);
        float x[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) x[q] = (float)acc[g][u][q];
        if (vec_ok && tb + 15 < P.nout) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            *reinterpret_cast<float4*>(orow + tb + 4 * q) =
                make_float4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
        } else {
#pragma unroll
          for (int q = 0; q < 16; ++q)
            if (tb + q < P.nout) orow[tb + q] = x[q];
        }
        if (P.part) {
          double s1 = 0.0, s2 = 0.0;
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            if (tb + q < P.nout) {
              const double y = x[q];
              s1 += y;
              s2 += y * y;
            }
          }
          // each half wavefront covers one 512-sample segment
#pragma unroll
          for (int off = 16; off > 0; off >>= 1) {
            s1 += __shfl_xor(s1, off, 64);
            s2 += __shfl_xor(s2, off, 64);
          }
          if ((lane & 31) == 0 && seg < P.nseg) {
            P.part[((int64_t)d * P.nseg + seg) * 2] = s1;
            P.part[((int64_t)d * P.nseg + seg) * 2 + 1] = s2;
          }
        }
      }
    }
  }
};

// One work unit per workgroup; each XCD (workgroups lin, lin + 8, ...) takes a contiguous
// run of units, tile-major, so the DM groups of a tile share that XCD's L2.
template <int G, int S>
__global__ __launch_bounds__(512) void dedisp_direct(DRParams P) {
  const int64_t lin = blockIdx.x;
  const int64_t per = (P.nitems + 7) / 8;
  const int64_t item = (lin & 7) * per + (lin >> 3);
  if (item >= P.nitems) return;
  const int64_t tile = item / P.ngroups;
  const int grp = (int)(item - tile * P.ngroups);
  DirectTile<G, S> k;
  k.run(P, tile, grp);
}

// Several beams in one launch. XCD x (workgroups lin = x, x + 8, ...) walks the items in
// order and takes the x-th eighth of each item's units [item][tile][group] (a contiguous,
// tile-major run, as in a single launch), so at any time every XCD works on the same item
// and their reads of its input meet in the shared last-level cache, as they do when the
// items are launched one at a time. run[x][i] is the first of XCD x's workgroups on item
// i (run[x][n] the count); the item's own units begin at its offset plus x/8 of its units.
// The item's parameters are read through the scalar cache. A launch holds the items of one
// tile shape and wavefront count, each on its own plan's DM groups.
template <int G, int S>
__global__ __launch_bounds__(512) void dedisp_direct_batch(const DRParams* __restrict__ items,
                                                           const int64_t* __restrict__ run, int nitems) {
  typedef const __attribute__((address_space(4))) int64_t* ci64_t;
  const int64_t lin = blockIdx.x;
  const int x = (int)(lin & 7);
  const ci64_t rx = (ci64_t)(run + (int64_t)x * (nitems + 1));
  const int64_t k = lin >> 3;
  if (k >= rx[nitems]) return;
  int lo = 0, hi = nitems - 1;  // the last item whose run starts at or before k
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rx[mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  // wave-uniform copy of the item's record through scalar loads
  typedef const __attribute__((address_space(4))) uint32_t* cu32_t;
  const cu32_t src = (cu32_t)(items + lo);
  uint32_t wv[sizeof(DRParams) / 4];
#pragma unroll
  for (int j = 0; j < (int)(sizeof(DRParams) / 4); ++j) wv[j] = src[j];
  DRParams P;
  __builtin_memcpy(&P, wv, sizeof(DRParams));
  if (P.tiles_g != G || P.tiles_s != S) return;  // a launch holds the items of one tile shape
  const int64_t local = (P.nitems * x) / 8 + (k - rx[lo]);
  const int64_t tile = local / P.ngroups;
  const int grp = (int)(local - tile * P.ngroups);
  DirectTile<G, S> tk;
  tk.run(P, tile, grp);
}

// The four shifted copies of a linear input: copy m of row c at position p holds
// in[c][p + m], or 0 from nsamp on. One thread per 16 positions of all four copies.
__global__ __launch_bounds__(256) void quad_prep(const uint8_t* __restrict__ in, int64_t in_stride, int64_t nsamp,
                                                 uint8_t* __restrict__ quad, int64_t lq) {
  const int c = blockIdx.y;
  const int64_t p0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
  if (p0 >= lq) return;
  const uint8_t* row = in + (int64_t)c * in_stride;
  uint32_t b[19];
#pragma unroll
  for (int k = 0; k < 19; ++k) b[k] = p0 + k < nsamp ? (uint32_t)row[p0 + k] : 0u;
  uint8_t* q = quad + (int64_t)c * 4 * lq + p0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    uint4 v;
    v.x = b[m] | (b[m + 1] << 8) | (b[m + 2] << 16) | (b[m + 3] << 24);
    v.y = b[m + 4] | (b[m + 5] << 8) | (b[m + 6] << 16) | (b[m + 7] << 24);
    v.z = b[m + 8] | (b[m + 9] << 8) | (b[m + 10] << 16) | (b[m + 11] << 24);
    v.w = b[m + 12] | (b[m + 13] << 8) | (b[m + 14] << 16) | (b[m + 15] << 24);
    *reinterpret_cast<uint4*>(q + (int64_t)m * lq) = v;
  }
}

// A block of n samples (or zeros when blk is null) written into a stream ring of four
// shifted copies: sample j sits at ring position q = (pos0 + j) mod ring_len, and copy m
// holds ring position (p + m) mod ring_len at every p < lq, so the sample goes to
// p = (q - m) mod ring_len and its mirror images p + k ring_len below lq.
__global__ __launch_bounds__(256) void ring_append_quad(const uint8_t* __restrict__ blk, int64_t in_stride,
                                                        int64_t n, uint8_t* __restrict__ ring, int64_t lq,
                                                        int64_t ring_len, int64_t pos0) {
  const int c = blockIdx.y;
  uint8_t* r = ring + (int64_t)c * 4 * lq;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    const uint8_t v = blk ? blk[(int64_t)c * in_stride + j] : (uint8_t)0;
    const int64_t q = (pos0 + j) % ring_len;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      int64_t p = q - m;
      if (p < 0) p += ring_len;
      for (; p < lq; p += ring_len) r[(int64_t)m * lq + p] = v;
    }
  }
}

template <int G, int S>
void launch_gs(const DRParams& P, int64_t nblocks, hipStream_t st) {
  hipLaunchKernelGGL((dedisp_direct<G, S>), dim3((unsigned)nblocks), dim3(64 * P.nw), 0, st, P);
}

template <int G, int S>
void launch_batch_gs(const DRParams* rec, const int64_t* run, int count, int64_t nblocks, int waves,
                     hipStream_t st) {
  hipLaunchKernelGGL((dedisp_direct_batch<G, S>), dim3((unsigned)nblocks), dim3(64 * waves), 0, st, rec, run, count);
}

// The tile shapes the kernels are built for: (trials per wavefront, sub-tiles).
bool shape_ok(int g, int sub) { return (g == 1 || g == 2 || g == 4) && (sub == 1 || (sub == 2 && g <= 2)); }

}  // namespace

namespace dd {

namespace {

// Parameters of one direct-read launch; for linear input the prep kernel that writes the
// copies is enqueued first.
int prepare(const dd_plan* p, const InView& in, const int32_t* d_table, int64_t nout, float* out,
            int64_t out_stride, double* part, void* quad_ws, hipStream_t st, DRParams* P) {
  *P = DRParams{};
  if (in.ring_len > 0) {
    // a stream ring already holds the copies; row_stride is the copy row length
    P->quad = static_cast<const uint8_t*>(in.ptr);
    P->lq = in.row_stride;
    P->ring_len = in.ring_len;
    P->w0 = in.win0 % in.ring_len;
  } else {
    P->lq = direct_quad_row(in.nvalid);
    P->quad = static_cast<const uint8_t*>(quad_ws);
  }
  // buffer offsets are 32-bit: four copy rows per channel, and ring positions below 2^31
  if (4 * P->lq >= ((int64_t)1 << 31) || P->ring_len + kDirectTile >= ((int64_t)1 << 31))
    return fail(DD_ERR_UNSUPPORTED, "rows of 2^29 samples or more are not supported by the direct-read form");
  const int sub = p->tiles.s / kDrLane;
  if (!shape_ok(p->tiles.g, sub))
    return fail(DD_ERR_UNSUPPORTED, "direct-read form: unsupported (dms_per_wave, samples_per_lane)");
  if (in.ring_len == 0) {
    const dim3 grid((unsigned)((P->lq / 16 + 255) / 256), (unsigned)p->nchan);
    hipLaunchKernelGGL(quad_prep, grid, dim3(256), 0, st, static_cast<const uint8_t*>(in.ptr), in.row_stride,
                       in.nvalid, const_cast<uint8_t*>(P->quad), P->lq);
  }
  const int64_t ntiles = (nout + kDirectTile * sub - 1) / (kDirectTile * sub);
  P->dtab = d_table;
  P->out = out;
  P->part = part;
  P->out_stride = out_stride;
  P->nout = nout;
  P->nseg = (nout + kTile - 1) / kTile;
  P->nitems = ntiles * p->ngroups;
  P->nchan = p->nchan;
  P->ndm = p->ndm;
  P->ndm_pad = p->ndm_pad;
  P->ngroups = p->ngroups;
  P->nw = p->tiles.w;
  P->tiles_g = p->tiles.g;
  P->tiles_s = sub;
  return DD_OK;
}

}  // namespace

int launch_direct(const dd_plan* p, const InView& in, const int32_t* d_table, int64_t nout, float* out,
                  int64_t out_stride, double* part, void* quad_ws, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  DRParams P;
  int rc = prepare(p, in, d_table, nout, out, out_stride, part, quad_ws, st, &P);
  if (rc) return rc;
  const int64_t nblocks = (P.nitems + 7) / 8 * 8;
  if (nblocks > 0x7fffffff) return fail(DD_ERR_UNSUPPORTED, "too many work items");
  if (nblocks == 0) return DD_OK;
  const int shape = P.tiles_g * 10 + P.tiles_s;
  switch (shape) {
    case 11: launch_gs<1, 1>(P, nblocks, st); break;
    case 21: launch_gs<2, 1>(P, nblocks, st); break;
    case 41: launch_gs<4, 1>(P, nblocks, st); break;
    case 12: launch_gs<1, 2>(P, nblocks, st); break;
    default: launch_gs<2, 2>(P, nblocks, st); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DD_ERR_HIP, std::string("dedisp_direct launch: ") + hipGetErrorString(e));
  return DD_OK;
}

int64_t direct_batch_desc_bytes(int32_t n) {
  // the records, then per launch (a tile shape and wavefront count: at most n launches) the
  // XCD runs [8][items + 1]
  return align_up((int64_t)n * (int64_t)sizeof(DRParams)) + align_up((int64_t)8 * 8 * 2 * n);
}

// Direct-read batch items with at least this many (tile, DM group) units take a plain launch.
constexpr int64_t kDirectPlainUnits = 12288;

int launch_direct_batch(const std::vector<DirectItem>& items, void* d_desc, int64_t desc_bytes, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int32_t n = (int32_t)items.size();
  if (n == 0) return DD_OK;
  if (desc_bytes < direct_batch_desc_bytes(n)) return fail(DD_ERR_WORKSPACE, "batch workspace too small");
  std::vector<DRParams> all((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    const DirectItem& it = items[i];
    int rc = prepare(it.plan, it.in, it.table, it.nout, it.out, it.out_stride, it.part, it.quad_ws, st, &all[i]);
    if (rc) return rc;
  }
  // An item with many units takes the plain launch of its own (a large beam fills the GPU
  // by itself; the persistent loop pays off for many small items, such as serving blocks).
  std::vector<DRParams> rest;
  for (const DRParams& r : all) {
    if (r.nitems < kDirectPlainUnits) {
      rest.push_back(r);
      continue;
    }
    const int64_t nblocks = (r.nitems + 7) / 8 * 8;
    if (nblocks > 0x7fffffff) return fail(DD_ERR_UNSUPPORTED, "too many work items");
    switch (r.tiles_g * 10 + r.tiles_s) {
      case 11: launch_gs<1, 1>(r, nblocks, st); break;
      case 21: launch_gs<2, 1>(r, nblocks, st); break;
      case 41: launch_gs<4, 1>(r, nblocks, st); break;
      case 12: launch_gs<1, 2>(r, nblocks, st); break;
      default: launch_gs<2, 2>(r, nblocks, st); break;
    }
  }
  all.swap(rest);
  // records grouped by tile shape and wavefront count (one kernel instantiation and
  // workgroup size per launch: every item keeps its own tiles), then per group the XCD runs
  // after all the records
  std::vector<DRParams> P;
  std::vector<int64_t> run;
  struct Group { int g, sub, first, count, waves; int64_t run_at, longest; };
  std::vector<Group> groups;
  for (int shape : {11, 21, 41, 12, 22}) {
    const int g = shape / 10, sub = shape % 10;
    for (int w = 1; w <= 8; ++w) {
      Group gr{g, sub, (int)P.size(), 0, w, 0, 0};
      for (const DRParams& r : all)
        if (r.tiles_g == g && r.tiles_s == sub && r.nw == w) {
          P.push_back(r);
          ++gr.count;
        }
      if (gr.count == 0) continue;
      gr.run_at = (int64_t)run.size();
      for (int x = 0; x < 8; ++x) {
        int64_t k = 0;
        run.push_back(0);
        for (int i = 0; i < gr.count; ++i) {
          const int64_t u = P[gr.first + i].nitems;
          k += (u * (x + 1)) / 8 - (u * x) / 8;  // XCD x's eighth of item i
          run.push_back(k);
        }
        gr.longest = std::max(gr.longest, k);
      }
      groups.push_back(gr);
    }
  }
  char* bw = static_cast<char*>(d_desc);
  DRParams* dP = reinterpret_cast<DRParams*>(bw);
  int64_t* dS = reinterpret_cast<int64_t*>(bw + align_up((int64_t)n * (int64_t)sizeof(DRParams)));
  hipError_t e = hipSuccess;
  if (!P.empty()) {
    e = hipMemcpyAsync(dP, P.data(), P.size() * sizeof(DRParams), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dS, run.data(), run.size() * 8, hipMemcpyHostToDevice, st);
    if (e != hipSuccess)
      return fail(DD_ERR_HIP, std::string("hipMemcpyAsync (batch descriptors): ") + hipGetErrorString(e));
  }
  for (const Group& gr : groups) {
    const int64_t nblocks = 8 * gr.longest;
    if (nblocks > 0x7fffffff) return fail(DD_ERR_UNSUPPORTED, "too many work items");
    if (nblocks == 0) continue;
    const DRParams* rec = dP + gr.first;
    const int64_t* rn = dS + gr.run_at;
    switch (gr.g * 10 + gr.sub) {
      case 11: launch_batch_gs<1, 1>(rec, rn, gr.count, nblocks, gr.waves, st); break;
      case 21: launch_batch_gs<2, 1>(rec, rn, gr.count, nblocks, gr.waves, st); break;
      case 41: launch_batch_gs<4, 1>(rec, rn, gr.count, nblocks, gr.waves, st); break;
      case 12: launch_batch_gs<1, 2>(rec, rn, gr.count, nblocks, gr.waves, st); break;
      default: launch_batch_gs<2, 2>(rec, rn, gr.count, nblocks, gr.waves, st); break;
    }
  }
  e = hipGetLastError();
  if (e != hipSuccess) return fail(DD_ERR_HIP, std::string("dedisp_direct_batch launch: ") + hipGetErrorString(e));
  return DD_OK;
}

int append_direct(const dd_plan* p, const void* blk, int64_t in_stride, int64_t n, void* ring, int64_t lq,
                  int64_t ring_len, int64_t pos0, void* stream) {
  const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(ring_append_quad, dim3(gx, (unsigned)p->nchan), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const uint8_t*>(blk), in_stride, n, static_cast<uint8_t*>(ring), lq, ring_len,
                     pos0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DD_ERR_HIP, std::string("ring_append_quad launch: ") + hipGetErrorString(e));
  return DD_OK;
}

}  // namespace dd
