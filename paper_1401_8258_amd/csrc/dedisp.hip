// HIP kernels for gfx950 and the C-ABI entry points that launch them.
//
// Kernels (all wave64):
//   dedisp_tile    Eq. bruteEquation over one (DM group, time tile) per workgroup.
//                  The channel vectors a group needs (Eq. channelDispersionEquation:
//                  tile length plus the in-group delay spread) reach LDS by DMA through
//                  a ring of stages and are shared by every computing wavefront of the
//                  workgroup; each accumulates its own DM trials in VGPRs. Per-trial
//                  delays arrive as precomputed LDS offsets with the data. 16/32-bit
//                  input is staged as 32-bit words, 8-bit input as bytes (own tile
//                  body). One instantiation per DMA form: 4-byte DMAs, 16-byte DMAs
//                  issued by every wavefront, or producer wavefronts that issue them
//                  all, beside computing wavefronts of 8 trials (512 threads) or of 4
//                  (1024 threads: the FP32 default). The epilogue writes the tile and
//                  its FP64 statistics partials.
//   dedisp_batch   the same tile bodies in one persistent launch over many inputs.
//   stats_finalize per-series mean and standard deviation from the FP64 partial sums
//                  (sum x, sum x^2) that dedisp_tile writes per 512-sample tile with a
//                  fixed wavefront reduction tree; one wavefront per series adds them in
//                  a fixed lane-strided order and butterfly.
//   cand_*         n-sigma detections: per-segment counts, one exclusive scan, and an
//                  ordered ballot compaction, so candidates come out in (d, t) order.
//   ring_append    copies a block into a stream's per-channel ring and its mirror.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <type_traits>
#include <vector>
#include <cstdint>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>

#include "dd_internal.h"
#include "dd_device.h"

namespace {

using dd::InView;
using dd::ci32_t;
using dd::wave_sum_fixed;
using dd::block_barrier;
using dd::wait_vm;
using dd::dma;
using dd::dma_x4;
using dd::lds_addr;

constexpr int kMaxThreads = 512;


// ------------------------------------------------------------------ dedispersion kernel
//
// Work unit = (512-sample time tile, group of W*G DM trials; G = 8, or 4 in the 16-wavefront
// producer form). Computing wavefront w of the workgroup owns trials dg + Gw .. dg + Gw +
// G - 1; lane l owns output samples t0 + 4l .. t0 + 4l + 3 and t0 + 256 + 4l .. t0 + 256 +
// 4l + 3 of the tile.
//
// Channel vectors (tile plus the group's delay spread, Eq. channelDispersionEquation)
// reach LDS by DMA (global_load_lds) through a ring of nb stages of cs channels,
// issued nb - 1 stages ahead, so HBM/L2 latency hides behind compute. Every sample
// lands in a 32-bit LDS word (the byte and short DMA forms zero-extend 8- and 16-bit
// inputs on the way), and each channel is stored four times, shifted by 0..3 samples,
// so the 4-sample chunks any trial needs start 16-byte aligned: a trial costs an
// address add and two ds_read_b128 (lanes read consecutive 16-byte slots: no bank
// conflicts). The host precomputes, per (channel, trial), the byte offset of the
// trial's first chunk inside the channel's slot; those offsets travel with the data.
//
// A stage's channels are split between the wavefronts (nw / cs of them per channel),
// so all DMAs a wavefront issues in a stage address one channel: its first delay is a
// scalar load and the per-DMA work is two lane reads of a descriptor table plus one
// add. Nothing on the DMA path waits for LDS.

constexpr int kTile = 512;
constexpr int kG = 8;
constexpr int kCopies = 4;
constexpr int kMaxDma = 256;  // DMA instructions per wavefront per stage (four descriptor registers)
constexpr int kMaxX4 = 16;    // 16-byte DMAs per wavefront per stage (one descriptor register each)
static_assert(kTile == dd::kTile, "tile constant disagrees with the host plan");
static_assert(kMaxDma == dd::kMaxDma, "DMA limit disagrees with the host plan");
static_assert(kMaxX4 == dd::kMaxX4, "16-byte DMA limit disagrees with the host plan");

struct KParams {
  InView in;
  const int32_t* dtab;   // [nchan][ndm_pad] LDS byte offset of each trial's chunk in its channel slot
  const int32_t* gbase;  // [ngroups][nchan] first delay of each group
  float* out;
  double* part;          // [ndm][ntiles][2] or null
  int64_t out_stride, nout, nitems;
  int ndm_pad, nchan, ndm, ngroups;
  int L;        // words per (channel, copy) buffer
  int cs;       // channels per stage (divides nw unless a producer issues the DMAs)
  int nb;       // stages in the LDS ring
  int nd;       // DMA instructions per wavefront per stage; with a producer, per channel
  int nstages;  // ceil(nchan / cs)
  int x4;       // FP32 input: copies arrive by 16-byte DMAs (nd counts those)
  int nw;       // computing wavefronts (8 DM trials each)
  int nprod;    // wavefronts after those that only issue DMAs (0: none, else 1..4)
  int ndw;      // DMA instructions per issuing wavefront per stage (the vmcnt unit)
  // 8-bit linear input: a channel window that would read past the end of the input
  // (byte in_bytes of the whole [nchan][row_stride] array) reads from `tail`, a copy of
  // input bytes [tail_base, in_bytes) followed by in_bytes - tail_base bytes of padding
  const uint8_t* tail;
  int64_t tail_base, in_bytes;
  int g;        // DM trials per computing wavefront (8; 4 in the 16-wavefront producer form)
  int pad_;
};

// LDS layout (4-byte words): the ring's channel slots (buf, cc), each holding the four
// shifted copies (copy m word x = window sample first + m + x) followed by 64 words of
// trial offsets (the LDS byte offsets of the group's trials for that channel).
__device__ __forceinline__ int slot_word(const KParams& P, int buf, int cc) {
  return (buf * P.cs + cc) * (kCopies * P.L + 64);
}

// Copy m, word x of a channel slot holds window sample first + m + x; slot word y of the
// 4L data words is (m, x) = divmod(y, L). rel(y) = m + x is its offset from `first`.
__device__ __forceinline__ int slot_rel(int y, int L) {
  const int m = (y >= L) + (y >= 2 * L) + (y >= 3 * L);
  return y - m * (L - 1);
}

// A wavefront's DMA chunks of its stage channel: r = sub, sub + wpc, ... (clamped to the
// last chunk, which keeps the per-wavefront count uniform).
//  x1 form (any input): chunk r < 4 * L/64 covers slot words 64r .. 64r + 63 (lane l:
//    word 64r + l); the last chunk is the trial offsets. Lane j of (rel, ldw) describes
//    chunk j: rel = source offset of its lane 0 from `first` (-1: offsets), ldw = slot word.
//  x4 form (FP32): chunk r < L/64 covers slot words 256r .. 256r + 255 (lane l: words
//    256r + 4l .. + 3, which never straddle two copies since L is a multiple of 64);
//    relx[j] is this lane's source offset for chunk j. The offsets come as one more x1 DMA.
struct DmaDesc {
  int rel[4], ldw[4];
  int relx[kMaxX4];
};
template <bool X4>
__device__ __forceinline__ void make_desc(const KParams& P, int sub, int wpc, int lane, DmaDesc* d) {
  const int nch = P.L >> 6;
  if constexpr (X4) {
#pragma unroll
    for (int j = 0; j < kMaxX4; ++j) {
      const int r = min(sub + wpc * j, nch - 1);
      d->relx[j] = slot_rel(256 * r + 4 * lane, P.L);
    }
    return;
  }
  const int nchunk = kCopies * nch + 1;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int r = min(sub + wpc * (lane + 64 * h), nchunk - 1);
    d->rel[h] = r < kCopies * nch ? slot_rel(64 * r, P.L) : -1;
    d->ldw[h] = 64 * r;
  }
#pragma unroll
  for (int j = 0; j < kMaxX4; ++j) d->relx[j] = 0;
}

// One x1 chunk: the offsets (rel < 0), or 64 slot words from source offset rel + lane (a
// 64-word chunk lies inside one copy, L being a multiple of 64).
template <int EB, bool RING>
__device__ __forceinline__ void dma_chunk(const char* rp, const int32_t* orow, int rel, int ldw, unsigned slot,
                                          int start, int nlim, int lane, int gw) {
  const unsigned m0 = slot + 4u * (unsigned)ldw;
  if (rel < 0) {
    dma<4>(orow, 4u * (unsigned)min(lane, gw - 1), m0);
    return;
  }
  int pos = start + rel + lane;
  if constexpr (!RING) pos = min(pos, nlim);
  dma<EB>(rp, (unsigned)(EB * pos), m0);
}

// This wavefront's DMAs for stage sd: its channel's chunks and the group's trial offsets
// for that channel. `start` is the row index of window position `first`: on a ring,
// (win0 + first) mod ring_len, and the mirror keeps the whole window contiguous.
template <int EB, bool RING, bool X4>
__device__ __forceinline__ void stage_dma(const KParams& P, const DmaDesc& D, unsigned sbase, int sd, int cc_w,
                                          int64_t t0, int grp, int dg, int gw, int lane, int w0, int sub, int wpc) {
  int c = sd * P.cs + cc_w;
  if (c >= P.nchan) c = P.nchan - 1;  // keeps the per-wavefront DMA count uniform
  const ci32_t gb = (ci32_t)(P.gbase + (int64_t)grp * P.nchan);
  const int first = (int)t0 + gb[c];
  int start = first;
  if constexpr (RING) {
    start += w0;
    if (start >= (int)P.in.ring_len) start -= (int)P.in.ring_len;
  }
  const char* rp = static_cast<const char*>(P.in.ptr) + (int64_t)c * P.in.row_stride * EB;
  const int32_t* orow = P.dtab + (int64_t)c * P.ndm_pad + dg;
  const unsigned slot = sbase + 4u * (unsigned)slot_word(P, sd % P.nb, cc_w);
  const int nlim = (int)P.in.nvalid - 1;
  if constexpr (X4) {
    static_assert(EB == 4, "16-byte DMAs carry FP32 input");
    {
      const int nch = P.L >> 6;
      int njx = P.nd - 1;
      // opaque per call: the 16 tests j < njx stay scalar compares here instead of being
      // hoisted out of the stage loop as 16 live SGPR-pair masks
      asm volatile("" : "+s"(njx));
      // the window's last sample is first + L + 2 (copy 3, word L - 1)
      if (RING || first + P.L + 2 <= nlim) {
#pragma unroll
        for (int j = 0; j < kMaxX4; ++j) {
          if (j < njx) {
            const int r = min(sub + wpc * j, nch - 1);
            dma_x4(rp, 4u * (unsigned)(start + D.relx[j]), slot + 1024u * (unsigned)r);
          }
        }
      } else {
        // data ends inside this window: per-lane clamped 4-byte DMAs (four per chunk),
        // then wait for them so the vmcnt bookkeeping of later stages stays exact
        for (int j = 0; j < njx; ++j) {
          const int r = min(sub + wpc * j, nch - 1);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int y = 256 * r + 64 * k;
            dma<4>(rp, 4u * (unsigned)min(first + slot_rel(y + lane, P.L), nlim), slot + 4u * (unsigned)y);
          }
        }
        wait_vm(0);
      }
      dma<4>(orow, 4u * (unsigned)min(lane, gw - 1), slot + 4u * (unsigned)(kCopies * P.L));
    }
  } else {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int n = min(P.nd - 64 * h, 64);
      for (int j = 0; j < n; ++j) {
        const int rel = __builtin_amdgcn_readlane(D.rel[h], j);
        const int ldw = __builtin_amdgcn_readlane(D.ldw[h], j);
        dma_chunk<EB, RING>(rp, orow, rel, ldw, slot, start, nlim, lane, gw);
      }
    }
  }
}

// Epilogue: the tile's sums to the output rows (float4 stores when aligned) and the
// tile's FP64 statistics partials (a fixed wavefront reduction tree of DPP moves, so the
// LDS, which bounds the tile body, carries none of it).
template <int G>
__device__ __forceinline__ void store_tile(const KParams& P, const float (&acc)[G][8], int dw, int64_t t0,
                                           int64_t tile, int lane) {
  const bool vec_ok = ((P.out_stride & 3) == 0) && ((reinterpret_cast<uintptr_t>(P.out) & 15) == 0);
  const int64_t nseg = (P.nout + kTile - 1) / kTile;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int d = dw + g;
    if (d >= P.ndm) break;
    float* orow = P.out + (int64_t)d * P.out_stride;
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t tb = t0 + 256 * h + 4 * lane;
      if (vec_ok && tb + 3 < P.nout) {
        *reinterpret_cast<float4*>(orow + tb) =
            make_float4(acc[g][4 * h], acc[g][4 * h + 1], acc[g][4 * h + 2], acc[g][4 * h + 3]);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (tb + q < P.nout) orow[tb + q] = acc[g][4 * h + q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (tb + q < P.nout) {
          const double x = acc[g][4 * h + q];
          s1 += x;
          s2 += x * x;
        }
      }
    }
    if (P.part) {
      s1 = dd::wave_sum_lane0(s1);
      s2 = dd::wave_sum_lane0(s2);
      if (lane == 0) {
        P.part[((int64_t)d * nseg + tile) * 2] = s1;
        P.part[((int64_t)d * nseg + tile) * 2 + 1] = s2;
      }
    }
  }
}

// One (time tile, DM group) work unit for 16- and 32-bit input; every wavefront of the
// workgroup takes part. Sums are FP32 with a sub-sum folded into the accumulator every
// DD_CHAN_BLOCK channels (fixed order in c).
template <typename TIn, bool RING, bool X4>
__device__ __forceinline__ void tile_body_impl(const KParams& P, int64_t tile, int grp, float* smem) {
  constexpr int EB = (int)sizeof(TIn);
  constexpr bool F16 = std::is_same<TIn, __half>::value;
  static_assert(EB >= 2, "8-bit input has its own tile body");
  const int nw = P.nw;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gw = kG * nw;
  const int64_t t0 = tile * kTile;
  const int dg = grp * gw;
  const int dw = dg + w * kG;
  const int w0 = P.in.ring_len > 0 ? (int)(P.in.win0 % P.in.ring_len) : 0;
  const int wpc = nw / P.cs;
  const int cc_w = w / wpc;
  const int wsub = w - cc_w * wpc;
  DmaDesc D;
  make_desc<X4>(P, wsub, wpc, lane, &D);
  const unsigned sbase = lds_addr(smem);

  float acc[kG][8];
  float sub[kG][8];
#pragma unroll
  for (int g = 0; g < kG; ++g)
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[g][s] = 0.f, sub[g][s] = 0.f;

  // prologue: stages 0 .. nb-2 in flight
  const int pre = min(P.nb - 1, P.nstages);
  for (int sd = 0; sd < pre; ++sd) stage_dma<EB, RING, X4>(P, D, sbase, sd, cc_w, t0, grp, dg, gw, lane, w0, wsub, wpc);
  const int* lds_i = reinterpret_cast<const int*>(smem);
  const unsigned lane16 = 16u * (unsigned)lane;
  const int offw = kCopies * P.L + w * kG;  // this wavefront's 8 offsets inside a slot

  for (int st = 0; st < P.nstages; ++st) {
    // stages issued after st: min(nstages - 1, st + nb - 2) - st
    const int later = min(P.nstages - 1, st + P.nb - 2) - st;
    wait_vm(later * P.ndw);
    block_barrier();
    if (st + P.nb - 1 < P.nstages)
      stage_dma<EB, RING, X4>(P, D, sbase, st + P.nb - 1, cc_w, t0, grp, dg, gw, lane, w0, wsub, wpc);
    const int buf = st % P.nb;
    const int n_here = min(P.cs, P.nchan - st * P.cs);
    const int4* op = reinterpret_cast<const int4*>(lds_i + slot_word(P, buf, 0) + offw);
    int4 o0 = op[0], o1 = op[1];
    for (int cc = 0; cc < n_here; ++cc) {
      const int c = st * P.cs + cc;
      if ((c & (DD_CHAN_BLOCK - 1)) == 0 && c != 0) {
#pragma unroll
        for (int g = 0; g < kG; ++g)
#pragma unroll
          for (int s = 0; s < 8; ++s) acc[g][s] += sub[g][s], sub[g][s] = 0.f;
      }
      const int off[kG] = {o0.x, o0.y, o0.z, o0.w, o1.x, o1.y, o1.z, o1.w};
      const char* cb = reinterpret_cast<const char*>(lds_i + slot_word(P, buf, cc)) + lane16;
      // all 16 reads of the channel first (more LDS reads in flight), then the next
      // channel's offsets, then the adds
      uint4 v[2 * kG];
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        const uint4* a = reinterpret_cast<const uint4*>(cb + off[g]);
        v[2 * g] = a[0];
        v[2 * g + 1] = a[64];
      }
      if (cc + 1 < n_here) {
        const int4* np = reinterpret_cast<const int4*>(lds_i + slot_word(P, buf, cc + 1) + offw);
        o0 = np[0];
        o1 = np[1];
      }
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        const uint32_t x[8] = {v[2 * g].x,     v[2 * g].y,     v[2 * g].z,     v[2 * g].w,
                               v[2 * g + 1].x, v[2 * g + 1].y, v[2 * g + 1].z, v[2 * g + 1].w};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          if constexpr (F16)
            sub[g][s] += __half2float(__ushort_as_half((unsigned short)x[s]));
          else
            sub[g][s] += __uint_as_float(x[s]);
        }
      }
    }
  }
#pragma unroll
  for (int g = 0; g < kG; ++g)
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[g][s] += sub[g][s];

  store_tile(P, acc, dw, t0, tile, lane);
}

// ------------------------------------------------------------------ 8-bit input
//
// Samples stay bytes in LDS: each channel slot holds four copies of L bytes, copy m
// byte x = window sample first + m + x, filled by 1024-byte (16 bytes per lane) and
// 256-byte DMAs straight from the byte stream (sources need no alignment), then 256
// bytes of trial offsets. A trial reads one dword per half: lane l takes samples
// 4l .. 4l + 3 (and 256 + 4l ..) from copy k & 3 at a dword-aligned address, lanes on
// consecutive dwords. Masks split the dword into the 16-bit pairs (s0, s2) and
// (s1, s3), which add with plain 32-bit adds; every 256 channels (255 x 256 < 2^16) the
// pairs fold into 32-bit accumulators, so the sums are exact integers.

// Chunk descriptors of one wavefront for its stage channel (lane j: chunk j): rel =
// source byte offset from `first` (-1 for the offsets), lds = byte offset inside the
// slot, with bit 30 set for a 1024-byte chunk.
struct DescU8 {
  int rel[4], lds[4];
};
__device__ __forceinline__ DescU8 make_desc_u8(const KParams& P, int sub, int wpc, int lane) {
  const int n4 = P.L >> 10, n1 = (P.L & 1023) >> 8;
  const int per = n4 + n1;  // chunks per copy
  const int nchunk = 4 * per + 1;
  DescU8 d;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int r = min(sub + wpc * (lane + 64 * h), nchunk - 1);
    const int m = r / per;
    const int i = r - m * per;
    if (m >= 4) {
      d.rel[h] = -1;
      d.lds[h] = 4 * P.L;
    } else if (i < n4) {
      d.rel[h] = m + 1024 * i;
      d.lds[h] = (m * P.L + 1024 * i) | (1 << 30);
    } else {
      const int b = 1024 * n4 + 256 * (i - n4);
      d.rel[h] = m + b;
      d.lds[h] = m * P.L + b;
    }
  }
  return d;
}

template <bool RING>
__device__ __forceinline__ void stage_dma_u8(const KParams& P, const DescU8& D, unsigned sbase, int sd, int cc_w,
                                             int64_t t0, int grp, int dg, int gw, int lane, int w0) {
  int c = sd * P.cs + cc_w;
  if (c >= P.nchan) c = P.nchan - 1;  // keeps the per-wavefront DMA count uniform
  const ci32_t gb = (ci32_t)(P.gbase + (int64_t)grp * P.nchan);
  const int first = (int)t0 + gb[c];
  const char* rp;
  int pos0;
  if constexpr (RING) {
    pos0 = first + w0;
    if (pos0 >= (int)P.in.ring_len) pos0 -= (int)P.in.ring_len;
    rp = static_cast<const char*>(P.in.ptr) + (int64_t)c * P.in.row_stride;
  } else {
    // the DMAs read bytes first .. first + L + 2 of the row (+ up to 15 inside a chunk)
    const int64_t g0 = (int64_t)c * P.in.row_stride + first;
    if (g0 + P.L + 18 > P.in_bytes) {
      rp = reinterpret_cast<const char*>(P.tail);
      pos0 = (int)(g0 - P.tail_base);
    } else {
      rp = static_cast<const char*>(P.in.ptr) + (int64_t)c * P.in.row_stride;
      pos0 = first;
    }
  }
  const int32_t* orow = P.dtab + (int64_t)c * P.ndm_pad + dg;
  const unsigned slot = sbase + (unsigned)((sd % P.nb) * P.cs + cc_w) * (unsigned)(4 * P.L + 256);
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int n = min(P.nd - 64 * h, 64);
    for (int j = 0; j < n; ++j) {
      const int rel = __builtin_amdgcn_readlane(D.rel[h], j);
      const int ld = __builtin_amdgcn_readlane(D.lds[h], j);
      const unsigned m0 = slot + (unsigned)(ld & ~(1 << 30));
      if (rel < 0)
        dma<4>(orow, 4u * (unsigned)min(lane, gw - 1), m0);
      else if (ld & (1 << 30))
        dma_x4(rp, (unsigned)(pos0 + rel + 16 * lane), m0);
      else
        dma<4>(rp, (unsigned)(pos0 + rel + 4 * lane), m0);
    }
  }
}

template <bool RING>
__device__ __forceinline__ void tile_body_u8(const KParams& P, int64_t tile, int grp, float* smem) {
  const int nw = P.nw;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gw = kG * nw;
  const int64_t t0 = tile * kTile;
  const int dg = grp * gw;
  const int dw = dg + w * kG;
  const int w0 = P.in.ring_len > 0 ? (int)(P.in.win0 % P.in.ring_len) : 0;
  const int wpc = nw / P.cs;
  const int cc_w = w / wpc;
  const DescU8 D = make_desc_u8(P, w - cc_w * wpc, wpc, lane);
  const unsigned sbase = lds_addr(smem);
  const int slot_b = 4 * P.L + 256;  // bytes per channel slot

  uint32_t pr[kG][4];   // [g][2h + {0: (s0, s2), 1: (s1, s3)}] 16-bit pair sums
  uint32_t acc[kG][8];  // [g][4h + j]
#pragma unroll
  for (int g = 0; g < kG; ++g) {
#pragma unroll
    for (int q = 0; q < 4; ++q) pr[g][q] = 0u;
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[g][s] = 0u;
  }
  auto fold = [&]() {
#pragma unroll
    for (int g = 0; g < kG; ++g) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t a = pr[g][2 * h], b = pr[g][2 * h + 1];
        acc[g][4 * h] += a & 0xffffu;
        acc[g][4 * h + 2] += a >> 16;
        acc[g][4 * h + 1] += b & 0xffffu;
        acc[g][4 * h + 3] += b >> 16;
        pr[g][2 * h] = 0u;
        pr[g][2 * h + 1] = 0u;
      }
    }
  };

  const int pre = min(P.nb - 1, P.nstages);
  for (int sd = 0; sd < pre; ++sd) stage_dma_u8<RING>(P, D, sbase, sd, cc_w, t0, grp, dg, gw, lane, w0);
  const char* lds_c = reinterpret_cast<const char*>(smem);
  const unsigned lane4 = 4u * (unsigned)lane;
  const int offb = 4 * P.L + 4 * kG * w;  // this wavefront's 8 offsets inside a slot (bytes)

  for (int st = 0; st < P.nstages; ++st) {
    const int later = min(P.nstages - 1, st + P.nb - 2) - st;
    wait_vm(later * P.ndw);
    block_barrier();
    if (st + P.nb - 1 < P.nstages)
      stage_dma_u8<RING>(P, D, sbase, st + P.nb - 1, cc_w, t0, grp, dg, gw, lane, w0);
    const int buf = st % P.nb;
    const int n_here = min(P.cs, P.nchan - st * P.cs);
    const char* sl = lds_c + buf * P.cs * slot_b;
    const int4* op = reinterpret_cast<const int4*>(sl + offb);
    int4 o0 = op[0], o1 = op[1];
    for (int cc = 0; cc < n_here; ++cc) {
      const int c = st * P.cs + cc;
      if ((c & 255) == 0 && c != 0) fold();
      const int off[kG] = {o0.x, o0.y, o0.z, o0.w, o1.x, o1.y, o1.z, o1.w};
      const char* cb = sl + cc * slot_b + lane4;
      uint32_t v[2 * kG];
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        const uint32_t* a = reinterpret_cast<const uint32_t*>(cb + off[g]);
        v[2 * g] = a[0];
        v[2 * g + 1] = a[64];
      }
      if (cc + 1 < n_here) {
        const int4* np = reinterpret_cast<const int4*>(sl + (cc + 1) * slot_b + offb);
        o0 = np[0];
        o1 = np[1];
      }
#pragma unroll
      for (int g = 0; g < kG; ++g) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          // full-rate mask and shift (v_perm issues at half rate)
          const uint32_t d = v[2 * g + h];
          pr[g][2 * h] += d & 0x00ff00ffu;             // (s0, s2)
          pr[g][2 * h + 1] += (d >> 8) & 0x00ff00ffu;  // (s1, s3)
        }
      }
    }
  }
  fold();

  float facc[kG][8];
#pragma unroll
  for (int g = 0; g < kG; ++g)
#pragma unroll
    for (int s = 0; s < 8; ++s) facc[g][s] = (float)acc[g][s];
  store_tile(P, facc, dw, t0, tile, lane);
}

// ------------------------------------------------------------------ FP32 with producers
//
// Wavefronts nw .. nw + nprod - 1 issue every DMA of every stage, whole channels in stage
// order (producer i takes stage channels i, i + nprod, ...: the four copies as L/64
// 16-byte DMAs, then the trial offsets), and wait for them; wavefronts 0 .. nw-1 only
// compute. The ring keeps at most 63 DMAs per producer in flight, so a producer never
// stalls on its own vmcnt when it issues. All of them meet at one barrier per stage:
// before it stage st has landed and stage st - 1 has been read, after it the producers
// refill the slot of stage st - 1 with stage st + nb - 1. A wavefront that issues DMAs
// stalls until the DMA path takes them; here only the producers do, while the computing
// wavefronts keep the LDS busy. The sums are those of the all-wavefront form: same
// offsets, same channel order, same DD_CHAN_BLOCK folding.
// Producer form: wavefronts nw .. nw + nprod - 1 issue every DMA; each computing wavefront
// owns G trials (G = 8 with up to 6 computing wavefronts in 512 threads; G = 4 with up to
// 14 in 1024 threads, which halves each wavefront's registers so that four wavefronts share
// a SIMD: a stage's time is set by each wavefront's serial chain of reads and adds, so more
// computing wavefronts per stage do more trials in the same time).
template <bool RING, int G>
__device__ __forceinline__ void tile_body_prod(const KParams& P, int64_t tile, int grp, float* smem) {
  static_assert(G == 4 || G == 8, "4 or 8 trials per computing wavefront");
  constexpr int H = G / 2;  // trials per half
  const int nw = P.nw;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gw = G * nw;
  const int64_t t0 = tile * kTile;
  const int dg = grp * gw;
  const unsigned sbase = lds_addr(smem);
  if (w >= nw) {
    const int pi = w - nw;  // producer pi takes stage channels pi, pi + nprod, ...
    const int w0 = P.in.ring_len > 0 ? (int)(P.in.win0 % P.in.ring_len) : 0;
    DmaDesc D;
    make_desc<true>(P, 0, 1, lane, &D);
    const int pre = min(P.nb - 1, P.nstages);
    for (int sd = 0; sd < pre; ++sd)
      for (int cc = pi; cc < P.cs; cc += P.nprod)
        stage_dma<4, RING, true>(P, D, sbase, sd, cc, t0, grp, dg, gw, lane, w0, 0, 1);
    for (int st = 0; st < P.nstages; ++st) {
      const int later = min(P.nstages - 1, st + P.nb - 2) - st;
      wait_vm(later * P.ndw);
      block_barrier();
      const int sd = st + P.nb - 1;
      if (sd < P.nstages)
        for (int cc = pi; cc < P.cs; cc += P.nprod)
          stage_dma<4, RING, true>(P, D, sbase, sd, cc, t0, grp, dg, gw, lane, w0, 0, 1);
    }
    return;
  }
  const int dw = dg + w * G;
  float acc[G][8];
  float sub[G][8];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[g][s] = 0.f, sub[g][s] = 0.f;
  const int* lds_i = reinterpret_cast<const int*>(smem);
  const unsigned lane16 = 16u * (unsigned)lane;
  const int offw = kCopies * P.L + w * G;  // this wavefront's G offsets inside a slot
  const int slot_bytes = 4 * (kCopies * P.L + 64);
  // A channel's trials are read and added in two halves: the next channel's first half is
  // read while this channel's second half is added, so G LDS reads stay in flight during
  // the adds; the trial offsets are read two channels ahead. Each sum still takes its
  // channels in order.
  struct Half {
    int o[H];
  };
  auto read_half = [&](const char* cb, const Half& o, uint4 (&v)[G]) {
#pragma unroll
    for (int t = 0; t < H; ++t) {
      const uint4* a = reinterpret_cast<const uint4*>(cb + o.o[t]);
      v[2 * t] = a[0];
      v[2 * t + 1] = a[64];
    }
  };
  auto add_half = [&](const uint4 (&v)[G], int g0) {
#pragma unroll
    for (int t = 0; t < H; ++t) {
      const uint32_t x[8] = {v[2 * t].x,     v[2 * t].y,     v[2 * t].z,     v[2 * t].w,
                             v[2 * t + 1].x, v[2 * t + 1].y, v[2 * t + 1].z, v[2 * t + 1].w};
#pragma unroll
      for (int s = 0; s < 8; ++s) sub[g0 + t][s] += __uint_as_float(x[s]);
    }
    // the half's sums exist before any later LDS read issues: the next reads then reuse
    // these registers instead of taking a second set
#pragma unroll
    for (int t = 0; t < H; ++t)
      asm volatile("" : "+v"(sub[g0 + t][0]), "+v"(sub[g0 + t][1]), "+v"(sub[g0 + t][2]), "+v"(sub[g0 + t][3]),
                   "+v"(sub[g0 + t][4]), "+v"(sub[g0 + t][5]), "+v"(sub[g0 + t][6]), "+v"(sub[g0 + t][7])
                   :
                   : "memory");
  };
  for (int st = 0; st < P.nstages; ++st) {
    block_barrier();
    const int buf = st % P.nb;
    const int n_here = min(P.cs, P.nchan - st * P.cs);
    const char* cb0 = reinterpret_cast<const char*>(lds_i + slot_word(P, buf, 0)) + lane16;
    const int last = n_here - 1;
    auto offsets = [&](int cc, Half& a, Half& b) {  // offsets of stage channel min(cc, last)
      const int4* q = reinterpret_cast<const int4*>(lds_i + slot_word(P, buf, min(cc, last)) + offw);
      if constexpr (G == 8) {
        const int4 x = q[0], y = q[1];
        a = Half{{x.x, x.y, x.z, x.w}};
        b = Half{{y.x, y.y, y.z, y.w}};
      } else {
        const int4 x = q[0];
        a = Half{{x.x, x.y}};
        b = Half{{x.z, x.w}};
      }
    };
    auto fold = [&](int cc) {
      const int c = st * P.cs + cc;
      if ((c & (DD_CHAN_BLOCK - 1)) == 0 && c != 0) {
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int s = 0; s < 8; ++s) acc[g][s] += sub[g][s], sub[g][s] = 0.f;
      }
    };
    Half oa, ob, na, nb;  // offsets of the channel being read, of the next one
    offsets(0, oa, ob);
    uint4 va[G], vb[G];
    read_half(cb0, oa, va);
    offsets(1, na, nb);
    read_half(cb0, ob, vb);
    // every iteration issues the same LDS reads (no branch around them), so each wait
    // counts exactly the reads issued after the data it needs; the last channel is peeled
    for (int cc = 0; cc < last; ++cc) {
      fold(cc);
      const char* cbn = cb0 + (cc + 1) * slot_bytes;
      Half na2, nb2;
      add_half(va, 0);
      read_half(cbn, na, va);
      offsets(cc + 2, na2, nb2);
      add_half(vb, H);
      read_half(cbn, nb, vb);
      na = na2;
      nb = nb2;
    }
    fold(last);
    add_half(va, 0);
    add_half(vb, H);
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int s = 0; s < 8; ++s) acc[g][s] += sub[g][s];
  store_tile<G>(P, acc, dw, t0, tile, lane);
}

// How a kernel instantiation moves input into LDS. Each instantiation carries only the
// DMA code it runs (the 4-byte form's descriptor tables and loop would cost the 16-byte
// form registers); kAny picks per item, for batches that mix the two.
enum Form { kX1 = 0, kX4 = 1, kProd = 2, kAny = 3, kProd4 = 4 };

template <typename TIn, bool RING, int F>
__device__ __forceinline__ void tile_body_ring(const KParams& P, int64_t tile, int grp, float* smem) {
  if constexpr (std::is_same<TIn, uint8_t>::value) {
    tile_body_u8<RING>(P, tile, grp, smem);
  } else if constexpr (F == kProd || F == kProd4) {
    static_assert(std::is_same<TIn, float>::value, "producer wavefronts carry FP32 input");
    tile_body_prod<RING, F == kProd4 ? 4 : 8>(P, tile, grp, smem);
  } else if constexpr (F == kX4) {
    tile_body_impl<TIn, RING, true>(P, tile, grp, smem);
  } else if constexpr (F == kAny && std::is_same<TIn, float>::value) {
    if (P.x4)
      tile_body_impl<TIn, RING, true>(P, tile, grp, smem);
    else
      tile_body_impl<TIn, RING, false>(P, tile, grp, smem);
  } else {
    tile_body_impl<TIn, RING, false>(P, tile, grp, smem);
  }
}

template <typename TIn, int F>
__device__ __forceinline__ void tile_body(const KParams& P, int64_t tile, int grp, float* smem) {
  if (P.in.ring_len > 0)
    tile_body_ring<TIn, true, F>(P, tile, grp, smem);
  else
    tile_body_ring<TIn, false, F>(P, tile, grp, smem);
}

// Plain launch: one work unit per workgroup; each XCD (workgroups lin, lin + 8, ...)
// takes a contiguous run of units, tile-major, so the DM groups of a tile share L2.
// Threads per workgroup a form may launch: 16 wavefronts for the 4-trial producer form.
constexpr int max_threads(int F) { return F == kProd4 ? 1024 : kMaxThreads; }

template <typename TIn, int F>
__global__ __launch_bounds__(max_threads(F)) void dedisp_tile(KParams P) {
  extern __shared__ __align__(16) float smem[];
  const int64_t lin = blockIdx.x;
  const int64_t per = (P.nitems + 7) / 8;
  const int64_t item = (lin & 7) * per + (lin >> 3);
  if (item >= P.nitems) return;  // uniform for the workgroup, before any barrier
  const int64_t tile = item / P.ngroups;
  const int grp = (int)(item - tile * P.ngroups);
  tile_body<TIn, F>(P, tile, grp, smem);
}

// Batched persistent launch over several plans/inputs. XCD x (workgroups x, x + 8, ...)
// takes the x-th eighth of every item's units (tile-major, DM group fastest): a contiguous
// run, as in the plain launch, so that neighbouring DM groups, whose channel windows
// overlap, share that XCD's L2, and every XCD gets an even share of every item whatever
// its numbers of tiles and groups. start[x * (n + 1) + i] is the first of XCD x's units
// that belongs to item i. The result of every unit is the one the plain launch computes
// for it.
typedef const __attribute__((address_space(4))) uint32_t* cu32_t;
typedef const __attribute__((address_space(4))) int64_t* ci64_t;
static_assert(sizeof(KParams) % 4 == 0, "KParams is copied as dwords");

// Wave-uniform copy of a KParams record through scalar loads.
__device__ __forceinline__ KParams load_params(const KParams* items, int i) {
  cu32_t src = (cu32_t)(items + i);
  uint32_t w[sizeof(KParams) / 4];
#pragma unroll
  for (int k = 0; k < (int)(sizeof(KParams) / 4); ++k) w[k] = src[k];
  KParams P;
  __builtin_memcpy(&P, w, sizeof(KParams));
  return P;
}

template <typename TIn, int F>
__global__ __launch_bounds__(max_threads(F)) void dedisp_batch(const KParams* items, const int64_t* start,
                                                              int nitems) {
  extern __shared__ __align__(16) float smem[];
  const int x = blockIdx.x & 7;
  ci64_t st_c = (ci64_t)(start + (int64_t)x * (nitems + 1));
  const int64_t total = st_c[nitems];
  const int64_t nslot = gridDim.x >> 3;
  int it = 0;
  for (int64_t q = blockIdx.x >> 3; q < total; q += nslot) {
    while (it + 1 < nitems && st_c[it + 1] <= q) ++it;
    const KParams P = load_params(items, it);
    const int64_t local = (P.nitems * x) / 8 + (q - st_c[it]);
    const int64_t tile = local / P.ngroups;
    const int grp = (int)(local - tile * P.ngroups);
    block_barrier();  // the previous unit's LDS reads are done before new DMAs land
    tile_body<TIn, F>(P, tile, grp, smem);
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

// stat[d] = {mean, rms, threshold} in FP64; mean/rms also as FP32 outputs. Called by a whole
// wavefront for its series: lane l sums the partials of tiles l, l + 64, l + 128, ... in
// that order (each step a coalesced 1 KB read of the wavefront), then the 64 lane sums meet
// in a fixed butterfly. The order depends on the number of tiles only, so every launch,
// batch and kernel form gives the same bits.
__device__ __forceinline__ void finalize_series(const double* __restrict__ part, int64_t nseg, int d, int64_t nout,
                                                double k, float* mean, float* rms, double* stat) {
  const int lane = threadIdx.x & 63;
  const double* pd = part + (int64_t)d * nseg * 2;
  double s = 0.0, ss = 0.0;
  for (int64_t g = lane; g < nseg; g += 64) {
    s += pd[g * 2];
    ss += pd[g * 2 + 1];
  }
  s = wave_sum_fixed(s);
  ss = wave_sum_fixed(ss);
  if (lane != 0) return;
  const double n = (double)nout;
  const double m = s / n;
  double var = ss / n - m * m;
  if (var < 0.0) var = 0.0;
  const double r = sqrt(var);
  mean[d] = (float)m;
  rms[d] = (float)r;
  stat[d * 3] = m;
  stat[d * 3 + 1] = r;
  stat[d * 3 + 2] = m + k * r;
}

// Values above the threshold in one kStatSeg segment of series d (a 256-thread block).
__device__ __forceinline__ void count_segment(const float* __restrict__ out, int64_t stride, int64_t nout,
                                              int64_t nseg, const double* __restrict__ stat,
                                              int32_t* __restrict__ cnt, int64_t seg, int d, int* red) {
  const float* row = out + (int64_t)d * stride;
  const double thr = stat[d * 3 + 2];
  const int64_t b = seg * dd::kStatSeg;
  const int64_t e = min(nout, b + dd::kStatSeg);
  int n = 0;
  if (e - b == dd::kStatSeg && (reinterpret_cast<uintptr_t>(row + b) & 15) == 0) {
    // a whole aligned segment: eight 16-byte loads per thread, all in flight together
    constexpr int kPer = dd::kStatSeg / 4 / 256;
    const float4* v = reinterpret_cast<const float4*>(row + b);
    float4 q[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) q[k] = v[threadIdx.x + 256 * k];
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      n += ((double)q[k].x > thr) + ((double)q[k].y > thr) + ((double)q[k].z > thr) + ((double)q[k].w > thr);
  } else {
    for (int64_t t = b + threadIdx.x; t < e; t += 256) n += ((double)row[t] > thr) ? 1 : 0;
  }
  // integer sum over the block: wavefront butterflies, then the four wavefront totals
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) cnt[(int64_t)d * nseg + seg] = red[0] + red[1] + red[2] + red[3];
}

// The detections of one segment of series d, in time order, at their scanned offsets.
// dm_index = d_base + d and t = t_base + (t << t_shift) (time-binned runs report times in
// input samples).
__device__ __forceinline__ void write_segment(const float* __restrict__ out, int64_t stride, int64_t nout,
                                              int64_t nseg, const double* __restrict__ stat,
                                              const int32_t* __restrict__ cnt, const int64_t* __restrict__ offs,
                                              dd_cand* __restrict__ cand, int64_t cap, int64_t t_base, int64_t seg,
                                              int d, int* wtot, int d_base = 0, int t_shift = 0) {
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
        o.dm_index = d_base + d;
        o.reserved = 0;
        o.t = t_base + (t << t_shift);
        o.value = x;
        o.snr = r > 0.0 ? (float)(((double)x - m) / r) : 0.f;
        cand[pos] = o;
      }
    }
    off += total;
  }
}

// One wavefront per series (four per 256-thread block).
__global__ __launch_bounds__(256) void stats_finalize(const double* __restrict__ part, int64_t nseg,
                                                      int ndm, int64_t nout, double k, float* mean,
                                                      float* rms, double* stat) {
  const int d = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (d >= ndm) return;  // uniform for the wavefront
  finalize_series(part, nseg, d, nout, k, mean, rms, stat);
}

__global__ __launch_bounds__(256) void cand_count(const float* __restrict__ out, int64_t stride, int64_t nout,
                                                  int64_t nseg, const double* __restrict__ stat,
                                                  int32_t* __restrict__ cnt) {
  __shared__ int red[4];
  count_segment(out, stride, nout, nseg, stat, cnt, blockIdx.x, blockIdx.y, red);
}

// The three passes of the block-parallel count scan (dd_device.h), one 1024-thread block per
// tile of 4096 counts in the first and last.
__global__ __launch_bounds__(1024) void scan_totals_k(const int32_t* __restrict__ cnt, int64_t n,
                                                      int64_t* __restrict__ offs) {
  __shared__ int64_t part[16];
  dd::scan_tile_totals(cnt, n, offs, part);
}
__global__ __launch_bounds__(1024) void scan_bases_k(int64_t n, int64_t* __restrict__ offs,
                                                     int64_t* __restrict__ total) {
  __shared__ int64_t part[16];
  dd::scan_tile_bases(n, offs, total, part);
}
__global__ __launch_bounds__(1024) void scan_apply_k(const int32_t* __restrict__ cnt, int64_t n,
                                                     int64_t* __restrict__ offs) {
  __shared__ int64_t part[16];
  dd::scan_tile_apply(cnt, n, offs, part);
}

__global__ __launch_bounds__(256) void cand_write(const float* __restrict__ out, int64_t stride, int64_t nout,
                                                  int64_t nseg, const double* __restrict__ stat,
                                                  const int32_t* __restrict__ cnt,
                                                  const int64_t* __restrict__ offs, dd_cand* __restrict__ cand,
                                                  int64_t cap, int64_t t_base) {
  __shared__ int wtot[4];
  write_segment(out, stride, nout, nseg, stat, cnt, offs, cand, cap, t_base, blockIdx.x, blockIdx.y, wtot);
}

// The same four steps for every item of a batch in one launch each. An item's series are
// [ser0, ser0 + ndm) of the flattened list, its (series, segment) units [unit0, unit0 +
// ndm * nseg) (items without candidates own none); blocks find their item by binary search.
struct TailItem {
  const double* part;  // statistics partials [ndm][ntiles][2]
  double* stat;        // [ndm][3]
  float *mean, *rms;
  const float* out;
  int32_t* cnt;        // [ndm][nseg]
  int64_t* offs;       // [ndm][nseg]
  int64_t* ncand;
  dd_cand* cand;
  int64_t ntiles, nout, stride, nseg, cap, t_base, ser0, unit0;
  double k;
  int32_t ndm;
  int32_t d_base, t_shift;  // candidates report dm_index d_base + d and t t_base + (t << t_shift)
  int32_t pad;
};

template <typename F>
__device__ __forceinline__ int find_item(const TailItem* items, int n, int64_t key, F first) {
  int lo = 0, hi = n - 1;  // the last item whose range starts at or before key
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first(items[mid]) <= key) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void stats_finalize_batch(const TailItem* __restrict__ items, int n, int64_t nser) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);  // one wavefront per series
  if (i >= nser) return;
  const TailItem& it = items[find_item(items, n, i, [](const TailItem& t) { return t.ser0; })];
  finalize_series(it.part, it.ntiles, (int)(i - it.ser0), it.nout, it.k, it.mean, it.rms, it.stat);
}

__global__ __launch_bounds__(256) void cand_count_batch(const TailItem* __restrict__ items, int n) {
  __shared__ int red[4];
  const int64_t u = blockIdx.x;
  const TailItem& it = items[find_item(items, n, u, [](const TailItem& t) { return t.unit0; })];
  const int64_t local = u - it.unit0;
  count_segment(it.out, it.stride, it.nout, it.nseg, it.stat, it.cnt, local % it.nseg, (int)(local / it.nseg), red);
}

// one block per item with candidates (items[blockIdx.x] of the candidate list)
__global__ __launch_bounds__(1024) void cand_scan_batch(const TailItem* __restrict__ items) {
  __shared__ int64_t part[1024];
  const TailItem& it = items[blockIdx.x];
  dd::scan_counts(it.cnt, (int64_t)it.ndm * it.nseg, it.offs, it.ncand, part);
}

__global__ __launch_bounds__(256) void cand_write_batch(const TailItem* __restrict__ items, int n) {
  __shared__ int wtot[4];
  const int64_t u = blockIdx.x;
  const TailItem& it = items[find_item(items, n, u, [](const TailItem& t) { return t.unit0; })];
  const int64_t local = u - it.unit0;
  write_segment(it.out, it.stride, it.nout, it.nseg, it.stat, it.cnt, it.offs, it.cand, it.cap, it.t_base,
                local % it.nseg, (int)(local / it.nseg), wtot, it.d_base, it.t_shift);
}

// Row c of the ring holds sample t at (t mod ring_len); positions below `mirror` are
// also written at ring_len + position, so any window of up to `mirror` samples starting
// in [0, ring_len) reads contiguously.
template <typename TIn>
__global__ __launch_bounds__(256) void ring_append(const TIn* __restrict__ blk, int64_t in_stride, int64_t n,
                                                   TIn* __restrict__ ring, int64_t ring_row, int64_t ring_len,
                                                   int64_t mirror, int64_t pos0) {
  const int c = blockIdx.y;
  const TIn* s = blk + (int64_t)c * in_stride;
  TIn* r = ring + (int64_t)c * ring_row;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    int64_t p = pos0 + j;
    if (p >= ring_len) p -= ring_len;
    const TIn v = s[j];
    r[p] = v;
    if (p < mirror) r[ring_len + p] = v;
  }
}

// Zeros for samples [pos0, pos0 + n) of every row of a stream's ring (positions modulo
// ring_len, mirrored like ring_append); n <= ring_len.
template <typename TIn>
__global__ __launch_bounds__(256) void ring_zero(TIn* __restrict__ ring, int64_t ring_row, int64_t ring_len,
                                                 int64_t mirror, int64_t pos0, int64_t n) {
  const int c = blockIdx.y;
  TIn* r = ring + (int64_t)c * ring_row;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    int64_t p = pos0 + j;
    if (p >= ring_len) p -= ring_len;
    r[p] = TIn(0);
    if (p < mirror) r[ring_len + p] = TIn(0);
  }
}

// Scratch of the entry point that allocates nothing (dd_dedisperse_noalloc): the statistics
// partials, thresholds, candidate counts and offsets and the u8 input-tail copy that
// dd_dedisperse keeps in the caller's workspace. Each device the library runs on holds one
// copy until the process ends; every call on that device shares it.
constexpr int64_t kScratchBytes = int64_t(96) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

// ------------------------------------------------------------------ host side

using KernFn = void (*)(KParams);

KernFn pick_kernel(int dtype, const KParams& P) {
  if (dtype == DD_F32)
    return P.nprod > 0 ? (P.g == 4 ? dedisp_tile<float, kProd4> : dedisp_tile<float, kProd>)
                       : P.x4 ? dedisp_tile<float, kX4> : dedisp_tile<float, kX1>;
  if (dtype == DD_F16) return dedisp_tile<__half, kX1>;
  return dedisp_tile<uint8_t, kX1>;
}

using BatchFn = void (*)(const KParams*, const int64_t*, int);

// form: kX1, kX4 or kProd when every item has it, else kAny (FP32 items that differ in x4)
BatchFn pick_batch_kernel(int dtype, int form) {
  if (dtype == DD_F32) {
    if (form == kProd) return dedisp_batch<float, kProd>;
    if (form == kProd4) return dedisp_batch<float, kProd4>;
    if (form == kX4) return dedisp_batch<float, kX4>;
    if (form == kX1) return dedisp_batch<float, kX1>;
    return dedisp_batch<float, kAny>;
  }
  if (dtype == DD_F16) return dedisp_batch<__half, kX1>;
  return dedisp_batch<uint8_t, kX1>;
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
// Kernel parameters and launch geometry for nout outputs of one plan on one input view.
int build_params(const dd_plan* p, const InView& in, const int32_t* d_table, int64_t nout, const Outputs& o,
                 char* ws, const dd::WsLayout& l, KParams* P, dd::Launch* G) {
  const int64_t lds_cap = lds_limit_bytes();
  const dd::Launch g = p->launch;
  if (in.nvalid >= (int64_t)1 << 30 || in.ring_len >= (int64_t)1 << 30)
    return dd::fail(DD_ERR_UNSUPPORTED, "windows of 2^30 samples or more per channel are not supported");
  if (g.nb < 2 || g.lds > lds_cap || g.nd < 1)
    return dd::fail(DD_ERR_UNSUPPORTED, "delay spread of one DM group (" + std::to_string(p->max_span) +
                                            " samples) does not fit in LDS; use fewer DMs per workgroup");
  const int64_t ntiles = (nout + kTile - 1) / kTile;
  const bool stats = o.mean && o.rms;
  *P = KParams{};
  P->in = in;
  P->dtab = d_table;
  P->out = o.out;
  P->part = stats ? reinterpret_cast<double*>(ws + l.part_off) : nullptr;
  P->out_stride = o.out_stride;
  P->nout = nout;
  P->nitems = ntiles * p->ngroups;
  P->ndm_pad = p->ndm_pad;
  P->nchan = p->nchan;
  P->ndm = p->ndm;
  P->ngroups = p->ngroups;
  P->L = g.L;
  P->cs = g.cs;
  P->nb = g.nb;
  P->nd = g.nd;
  P->nstages = (p->nchan + g.cs - 1) / g.cs;
  P->x4 = g.x4;
  P->nw = p->tiles.w;
  P->g = p->tiles.g;
  P->nprod = g.prod;
  P->ndw = g.ndw;
  if (p->dtype == DD_U8 && in.ring_len == 0) {
    P->in_bytes = (int64_t)(p->nchan - 1) * in.row_stride + in.nvalid;
    P->tail_base = std::max<int64_t>(0, P->in_bytes - l.tail_bytes);
    P->tail = reinterpret_cast<const uint8_t*>(ws + l.tail_off);
  }
  P->gbase = d_table + (int64_t)p->nchan * p->ndm_pad;
  *G = g;
  return DD_OK;
}

// 8-bit linear input: the last input bytes go to the workspace copy that windows reaching
// past the end of the input read instead (enqueued before the dedispersion launch).
int copy_tail(const KParams& P, hipStream_t st) {
  if (!P.tail) return DD_OK;
  const char* src = static_cast<const char*>(P.in.ptr) + P.tail_base;
  hipError_t e = hipMemcpyAsync(const_cast<uint8_t*>(P.tail), src, (size_t)(P.in_bytes - P.tail_base),
                                hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (input tail)");
  return DD_OK;
}

// Statistics finalize and candidate kernels for one plan's nout outputs.
int launch_tail(const dd_plan* p, int64_t nout, const Outputs& o, char* ws, const dd::WsLayout& l, hipStream_t st) {
  if (!(o.mean && o.rms)) return DD_OK;
  const int64_t ntiles = (nout + kTile - 1) / kTile;
  double* part = reinterpret_cast<double*>(ws + l.part_off);
  double* stat = reinterpret_cast<double*>(ws + l.thr_off);
  hipLaunchKernelGGL(stats_finalize, dim3((unsigned)((p->ndm + 3) / 4)), dim3(256), 0, st, part, ntiles,
                     p->ndm, nout, (double)o.k, o.mean, o.rms, stat);
  if (o.k > 0.f && o.ncand) {
    const int64_t nseg = (nout + dd::kStatSeg - 1) / dd::kStatSeg;
    int32_t* cnt = reinterpret_cast<int32_t*>(ws + l.cnt_off);
    int64_t* offs = reinterpret_cast<int64_t*>(ws + l.offs_off);
    hipLaunchKernelGGL(cand_count, dim3((unsigned)nseg, (unsigned)p->ndm), dim3(256), 0, st, o.out, o.out_stride,
                       nout, nseg, stat, cnt);
    int rc = dd::launch_count_scan(cnt, nseg * p->ndm, offs, o.ncand, st);
    if (rc) return rc;
    hipLaunchKernelGGL(cand_write, dim3((unsigned)nseg, (unsigned)p->ndm), dim3(256), 0, st, o.out, o.out_stride,
                       nout, nseg, stat, cnt, offs, o.cand, o.cand ? o.cap : 0, o.t_base);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "statistics/candidate launch");
  return DD_OK;
}

int set_lds(const void* k, int64_t lds) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  }
  return DD_OK;
}

// Dedisperse nout outputs of a prepared input view, then stats and candidates.
int run_pipeline(const dd_plan* p, const InView& in, const int32_t* d_table, int64_t nout, const Outputs& o,
                 char* ws, const dd::WsLayout& l, hipStream_t st, bool tail) {
  if (p->launch.form == dd::kFormRegWin || p->launch.form == dd::kFormDirect) {
    double* part = (o.mean && o.rms) ? reinterpret_cast<double*>(ws + l.part_off) : nullptr;
    int rc = p->launch.form == dd::kFormRegWin
                 ? dd::launch_regwin(p, in, d_table, nout, o.out, o.out_stride, part, st)
                 : dd::launch_direct(p, in, d_table, nout, o.out, o.out_stride, part, ws + l.quad_off, st);
    if (rc) return rc;
    return tail ? launch_tail(p, nout, o, ws, l, st) : DD_OK;
  }
  KParams P;
  dd::Launch g;
  int rc = build_params(p, in, d_table, nout, o, ws, l, &P, &g);
  if (rc) return rc;
  KernFn k = pick_kernel(p->dtype, P);
  rc = set_lds((const void*)k, g.lds);
  if (rc) return rc;
  rc = copy_tail(P, st);
  if (rc) return rc;
  const int64_t nblocks = (P.nitems + 7) / 8 * 8;
  if (nblocks > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "too many work items");
  hipLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(64 * (P.nw + P.nprod)), (size_t)g.lds, st, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "dedisp_tile launch");
  return tail ? launch_tail(p, nout, o, ws, l, st) : DD_OK;
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


// ------------------------------------------------------------------ composite plans
//
// A time-binned plan (runs of trials on the input downfactored 2^k times) and a subband plan
// (step-1 plans per subband at nominal DMs, step-2 plans per group of trials over the
// reduced filterbank) are made of ordinary plans. Their statistics come from each run's own
// pipeline; their candidates go through one merged pass: counts of every run's (series,
// segment) units, one scan over all of them, and one writing launch, so the detections of all
// runs form one list in (global trial, time) order.

// One run's part of a merged candidate pass.
struct MergedRun {
  const float* out;     // the run's first row
  int64_t stride, nout;
  const double* stat;   // [ndm][3] from the run's statistics
  int32_t ndm, d0, shift;
  int64_t t_base = 0;   // candidate t = t_base + (output index << shift)
};

int64_t merged_cand_bytes(const std::vector<MergedRun>& runs) {
  int64_t units = 0;
  for (const MergedRun& r : runs) units += (int64_t)r.ndm * ((r.nout + dd::kStatSeg - 1) / dd::kStatSeg);
  return dd::align_up(units * 4) + dd::align_up(units * 8) + dd::align_up((int64_t)runs.size() * sizeof(TailItem));
}

int merged_candidates(const std::vector<MergedRun>& runs, float k, dd_cand* cand, int64_t cap, int64_t* ncand,
                      char* region, hipStream_t st) {
  int64_t units = 0;
  for (const MergedRun& r : runs) units += (int64_t)r.ndm * ((r.nout + dd::kStatSeg - 1) / dd::kStatSeg);
  int32_t* cnt = reinterpret_cast<int32_t*>(region);
  int64_t* offs = reinterpret_cast<int64_t*>(region + dd::align_up(units * 4));
  TailItem* dT = reinterpret_cast<TailItem*>(region + dd::align_up(units * 4) + dd::align_up(units * 8));
  std::vector<TailItem> items;
  int64_t u0 = 0;
  for (const MergedRun& r : runs) {
    TailItem t{};
    t.stat = const_cast<double*>(r.stat);
    t.out = r.out;
    t.stride = r.stride;
    t.nout = r.nout;
    t.k = (double)k;
    t.ndm = r.ndm;
    t.nseg = (r.nout + dd::kStatSeg - 1) / dd::kStatSeg;
    t.cnt = cnt + u0;
    t.offs = offs + u0;
    t.ncand = ncand;
    t.cand = cand;
    t.cap = cand ? cap : 0;
    t.unit0 = u0;
    t.d_base = r.d0;
    t.t_shift = r.shift;
    t.t_base = r.t_base;
    u0 += (int64_t)r.ndm * t.nseg;
    items.push_back(t);
  }
  if (units > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "too many candidate segments");
  hipError_t e = hipMemcpyAsync(dT, items.data(), items.size() * sizeof(TailItem), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (candidate descriptors)");
  const int n = (int)items.size();
  hipLaunchKernelGGL(cand_count_batch, dim3((unsigned)units), dim3(256), 0, st, (const TailItem*)dT, n);
  int rc = dd::launch_count_scan(cnt, units, offs, ncand, st);
  if (rc) return rc;
  hipLaunchKernelGGL(cand_write_batch, dim3((unsigned)units), dim3(256), 0, st, (const TailItem*)dT, n);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "merged candidate launch");
  return DD_OK;
}

}  // namespace

namespace dd {

int launch_count_scan(const int32_t* cnt, int64_t n, int64_t* offs, int64_t* total, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (ntiles > 0x7fffffff) return fail(DD_ERR_UNSUPPORTED, "too many counts to scan");
  if (ntiles > 0) hipLaunchKernelGGL(scan_totals_k, dim3((unsigned)ntiles), dim3(1024), 0, st, cnt, n, offs);
  hipLaunchKernelGGL(scan_bases_k, dim3(1), dim3(1024), 0, st, n, offs, total);
  if (ntiles > 0) hipLaunchKernelGGL(scan_apply_k, dim3((unsigned)ntiles), dim3(1024), 0, st, cnt, n, offs);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DD_ERR_HIP, std::string("count scan launch: ") + hipGetErrorString(e));
  return DD_OK;
}

}  // namespace dd

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
                      static_cast<hipStream_t>(stream), true);
}

int dd_dedisperse_noalloc(const dd_plan* p, const void* d_in, int64_t nsamp, int64_t in_row_stride, float* d_out,
                          int64_t out_row_stride, float* d_mean, float* d_rms, float k_sigma, dd_cand* d_cand,
                          int64_t cand_cap, int64_t* d_ncand, const void* d_table, void* stream) {
  dd::clear_error();
  if (!p || !d_in || !d_table) return dd::fail(DD_ERR_INVALID_ARG, "plan, input and device table are required");
  if (nsamp <= p->maxdelay)
    return dd::fail(DD_ERR_TOO_SHORT, "nsamp must exceed maxdelay (" + std::to_string(p->maxdelay) + ")");
  if (in_row_stride < nsamp) return dd::fail(DD_ERR_INVALID_ARG, "in_row_stride < nsamp");
  const int64_t nout = nsamp - p->maxdelay;
  int rc = check_outputs(p, d_out, out_row_stride, nout, d_mean, d_rms, k_sigma, d_cand, cand_cap, d_ncand);
  if (rc) return rc;
  // the workspace regions after the delay table, moved to the start of the scratch array
  dd::WsLayout l = dd::workspace_layout(p, nsamp);
  const int64_t base = l.part_off;
  if (l.total - base > kScratchBytes)
    return dd::fail(DD_ERR_UNSUPPORTED, "this call needs " + std::to_string(l.total - base) +
                                            " bytes of scratch; the static scratch holds " +
                                            std::to_string(kScratchBytes));
  l.part_off -= base;
  l.thr_off -= base;
  l.cnt_off -= base;
  l.offs_off -= base;
  l.tail_off -= base;
  l.quad_off -= base;
  l.total -= base;
  // the array's device address, looked up once per device with that device current (the
  // array's name is a host-side stand-in, not a device address)
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return dd::fail(DD_ERR_UNSUPPORTED, "device index beyond 63");
  void* sp = nullptr;
  {
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
      void* a = nullptr;
      e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !a) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
      addr[dev] = a;
    }
    sp = addr[dev];
  }
  InView in{d_in, in_row_stride, nsamp, 0, 0};
  Outputs o{d_out, out_row_stride, d_mean, d_rms, k_sigma, d_cand, cand_cap, d_ncand, 0};
  return run_pipeline(p, in, static_cast<const int32_t*>(d_table), nout, o, static_cast<char*>(sp), l,
                      static_cast<hipStream_t>(stream), true);
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
  s->ring_len = dd::ring_len_for(p, block_nsamp);
  s->ring_row = s->ring_len + dd::ring_mirror(p);
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
  if (seq != s->next_seq && !(s->gap_fill && seq > s->next_seq))
    return dd::fail(DD_ERR_SEQUENCE, "expected seq " + std::to_string(s->next_seq) + ", got " + std::to_string(seq));
  if (nsamp < 1 || nsamp > s->block) return dd::fail(DD_ERR_INVALID_ARG, "block size out of range");
  if (in_row_stride < nsamp) return dd::fail(DD_ERR_INVALID_ARG, "in_row_stride < nsamp");
  if (s->pending_n > 0) return dd::fail(DD_ERR_SEQUENCE, "previous window not dedispersed yet");
  const dd_plan* p = s->plan;
  char* ring = static_cast<char*>(s->ring) + dd::ring_table_bytes(p);
  const int64_t mirror = s->ring_row - s->ring_len;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool quad = p->launch.form == dd::kFormDirect;
  if (seq > s->next_seq) {
    // lost blocks: block samples of zeros each; only the last ring length of them can still
    // be read, so only those are written
    const int64_t missing = (seq - s->next_seq) * s->block;
    const int64_t nz = std::min<int64_t>(missing, s->ring_len);
    const int64_t zpos = (s->received + missing - nz) % s->ring_len;
    dim3 zgrid((unsigned)std::min<int64_t>((nz + 255) / 256, 1024), (unsigned)p->nchan);
    if (quad) {
      int rz = dd::append_direct(p, nullptr, 0, nz, ring, s->ring_row, s->ring_len, zpos, st);
      if (rz) return rz;
    } else if (p->dtype == DD_F32)
      hipLaunchKernelGGL(ring_zero<float>, zgrid, dim3(256), 0, st, reinterpret_cast<float*>(ring), s->ring_row,
                         s->ring_len, mirror, zpos, nz);
    else if (p->dtype == DD_F16)
      hipLaunchKernelGGL(ring_zero<__half>, zgrid, dim3(256), 0, st, reinterpret_cast<__half*>(ring), s->ring_row,
                         s->ring_len, mirror, zpos, nz);
    else
      hipLaunchKernelGGL(ring_zero<uint8_t>, zgrid, dim3(256), 0, st, reinterpret_cast<uint8_t*>(ring), s->ring_row,
                         s->ring_len, mirror, zpos, nz);
    hipError_t ez = hipGetLastError();
    if (ez != hipSuccess) return hip_fail(ez, "ring_zero launch");
    s->received += missing;
    s->next_seq = seq;
    // outputs computable from the zeros and this block beyond the last block's worth are
    // skipped: this push's window is at most one block long
    s->emitted = std::max(s->emitted, s->received + nsamp - p->maxdelay - s->block);
  }
  const int64_t pos0 = s->received % s->ring_len;
  const unsigned gx = (unsigned)std::min<int64_t>((nsamp + 255) / 256, 1024);
  dim3 grid(gx, (unsigned)p->nchan);
  if (quad) {
    int ra = dd::append_direct(p, d_block, in_row_stride, nsamp, ring, s->ring_row, s->ring_len, pos0, st);
    if (ra) return ra;
  } else if (p->dtype == DD_F32)
    hipLaunchKernelGGL(ring_append<float>, grid, dim3(256), 0, st, static_cast<const float*>(d_block), in_row_stride,
                       nsamp, reinterpret_cast<float*>(ring), s->ring_row, s->ring_len, mirror, pos0);
  else if (p->dtype == DD_F16)
    hipLaunchKernelGGL(ring_append<__half>, grid, dim3(256), 0, st, static_cast<const __half*>(d_block),
                       in_row_stride, nsamp, reinterpret_cast<__half*>(ring), s->ring_row, s->ring_len, mirror,
                       pos0);
  else
    hipLaunchKernelGGL(ring_append<uint8_t>, grid, dim3(256), 0, st, static_cast<const uint8_t*>(d_block),
                       in_row_stride, nsamp, reinterpret_cast<uint8_t*>(ring), s->ring_row, s->ring_len, mirror,
                       pos0);
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

int dd_stream_set_gap_fill(dd_stream* s, int32_t enable) {
  dd::clear_error();
  if (!s) return dd::fail(DD_ERR_INVALID_ARG, "stream is NULL");
  s->gap_fill = enable != 0;
  return DD_OK;
}

int dd_candidates_check(const int64_t* d_ncand, int64_t cand_cap, void* stream, int64_t* ncand_out) {
  dd::clear_error();
  if (ncand_out) *ncand_out = 0;
  if (!d_ncand) return dd::fail(DD_ERR_INVALID_ARG, "d_ncand is NULL");
  int64_t n = 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&n, d_ncand, sizeof(n), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "candidate count");
  if (ncand_out) *ncand_out = n;
  return n > cand_cap ? DD_WARN_CAND_OVERFLOW : DD_OK;
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
  const dd::WsLayout l = dd::workspace_layout(p, s->block, false);
  if (ws_bytes < l.total) return dd::fail(DD_ERR_WORKSPACE, "workspace smaller than dd_plan_query asks for");
  int64_t t0 = 0, n = 0;
  rc = dd_stream_append(s, d_block, nsamp, in_row_stride, seq, stream, &t0, &n);
  if (rc != DD_OK) return rc;
  s->pending_n = 0;
  InView in{static_cast<char*>(s->ring) + dd::ring_table_bytes(p), s->ring_row, n + p->maxdelay, s->ring_len, t0};
  Outputs o{d_out, out_row_stride, d_mean, d_rms, k_sigma, d_cand, cand_cap, d_ncand, t0};
  rc = run_pipeline(p, in, static_cast<const int32_t*>(s->ring), n, o, static_cast<char*>(d_workspace), l,
                    static_cast<hipStream_t>(stream), true);
  if (rc) return rc;
  if (t0_out) *t0_out = t0;
  if (nout_out) *nout_out = n;
  return DD_OK;
}

}  // extern "C"

namespace {
// LDS-form batch items with at least this many (tile, DM group) units, or units times
// channels, take a plain launch
constexpr int64_t kBatchPlainUnits = 4096;
constexpr int64_t kBatchPlainWork = (int64_t)1 << 20;
}  // namespace

extern "C" {

int dd_batch_query(const dd_batch_item* items, int32_t n, int64_t* ws_bytes) {
  dd::clear_error();
  if (!ws_bytes || n < 1 || !items) return dd::fail(DD_ERR_INVALID_ARG, "need items, n >= 1 and ws_bytes");
  // descriptors of the LDS-form launches (the records, then per launch the XCD runs
  // [8][items + 1]: at most 8 * 2n entries over at most n launches), then of the direct-read
  // launches
  *ws_bytes = dd::align_up((int64_t)n * (int64_t)sizeof(KParams)) + dd::align_up((int64_t)8 * 8 * 2 * n) +
              dd::direct_batch_desc_bytes(n) + 2 * dd::align_up((int64_t)n * (int64_t)sizeof(TailItem));
  return DD_OK;
}

int dd_batch_dedisperse(const dd_batch_item* items, int32_t n, void* d_workspace, int64_t ws_bytes, void* stream) {
  dd::clear_error();
  int64_t need = 0;
  int rc = dd_batch_query(items, n, &need);
  if (rc) return rc;
  if (!d_workspace || ws_bytes < need) return dd::fail(DD_ERR_WORKSPACE, "batch workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<KParams> P;  // LDS-form items
  // per LDS-form item: the launch it joins (input dtype, computing and producer wavefronts,
  // trials per wavefront: one kernel instantiation and workgroup shape) and its LDS bytes
  struct LdsKey {
    int32_t dtype, waves, prod, per_wave;
    bool operator==(const LdsKey& o) const {
      return dtype == o.dtype && waves == o.waves && prod == o.prod && per_wave == o.per_wave;
    }
  };
  std::vector<LdsKey> keys;
  std::vector<int64_t> ldss;
  std::vector<dd::DirectItem> direct;  // direct-read items
  std::vector<Outputs> outs((size_t)n);
  std::vector<int64_t> nouts((size_t)n);
  std::vector<dd::WsLayout> lays((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    const dd_batch_item& it = items[i];
    dd_stream* sp = it.stream_item;
    const dd_plan* p = sp ? sp->plan : it.plan;
    if (!p || !it.d_plan_workspace)
      return dd::fail(DD_ERR_INVALID_ARG, "batch item " + std::to_string(i) + ": plan and workspace required");
    if (p->launch.form == dd::kFormRegWin)
      return dd::fail(DD_ERR_UNSUPPORTED, "batch item " + std::to_string(i) +
                                              ": register-window plans are not batched; use DD_FORM_LDS");
    const bool is_direct = p->launch.form == dd::kFormDirect;
    InView in;
    const int32_t* table;
    int64_t nout, t_base = 0, lay_n;
    char* ws = static_cast<char*>(it.d_plan_workspace);
    if (sp) {
      if (sp->pending_n <= 0)
        return dd::fail(DD_ERR_SEQUENCE, "batch item " + std::to_string(i) + ": stream has no appended window");
      nout = sp->pending_n;
      t_base = sp->pending_t0;
      in = InView{static_cast<char*>(sp->ring) + dd::ring_table_bytes(p), sp->ring_row, nout + p->maxdelay,
                  sp->ring_len, sp->pending_t0};
      table = static_cast<const int32_t*>(sp->ring);
      lay_n = sp->block;
    } else {
      if (!it.d_in || it.nsamp <= p->maxdelay || it.in_row_stride < it.nsamp)
        return dd::fail(it.nsamp <= p->maxdelay ? DD_ERR_TOO_SHORT : DD_ERR_INVALID_ARG,
                        "batch item " + std::to_string(i) + ": bad input");
      nout = it.nsamp - p->maxdelay;
      in = InView{it.d_in, it.in_row_stride, it.nsamp, 0, 0};
      table = reinterpret_cast<const int32_t*>(ws);
      lay_n = it.nsamp;
    }
    rc = check_outputs(p, it.d_out, it.out_row_stride, nout, it.d_mean, it.d_rms, it.k_sigma, it.d_cand,
                       it.cand_cap, it.d_ncand);
    if (rc) return dd::fail(rc, "batch item " + std::to_string(i) + ": " + dd_last_error());
    lays[i] = dd::workspace_layout(p, lay_n, sp == nullptr);
    // every item writes statistics partials, candidate counts and (u8) an input-tail copy into
    // its workspace, so two items sharing workspace bytes would overwrite each other; checked
    // before anything is enqueued
    for (int32_t j = 0; j < i; ++j) {
      const char* a0 = static_cast<const char*>(it.d_plan_workspace);
      const char* b0 = static_cast<const char*>(items[j].d_plan_workspace);
      if (a0 < b0 + lays[j].total && b0 < a0 + lays[i].total)
        return dd::fail(DD_ERR_INVALID_ARG, "batch items " + std::to_string(j) + " and " + std::to_string(i) +
                                                " share workspace memory; each item needs its own");
    }
    outs[i] = Outputs{it.d_out, it.out_row_stride, it.d_mean, it.d_rms, it.k_sigma, it.d_cand, it.cand_cap,
                      it.d_ncand, t_base};
    nouts[i] = nout;
    if (is_direct) {
      double* part = (it.d_mean && it.d_rms) ? reinterpret_cast<double*>(ws + lays[i].part_off) : nullptr;
      direct.push_back(dd::DirectItem{p, in, table, nout, it.d_out, it.out_row_stride, part, ws + lays[i].quad_off});
      continue;
    }
    dd::Launch g;
    KParams kp;
    rc = build_params(p, in, table, nout, outs[i], ws, lays[i], &kp, &g);
    if (rc) return rc;
    rc = copy_tail(kp, st);
    if (rc) return rc;
    P.push_back(kp);
    keys.push_back(LdsKey{p->dtype, p->tiles.w, p->launch.prod, p->tiles.g});
    ldss.push_back(g.lds);
  }
  char* bw = static_cast<char*>(d_workspace);
  const int64_t lds_desc = dd::align_up((int64_t)n * (int64_t)sizeof(KParams)) + dd::align_up((int64_t)8 * 8 * 2 * n);
  // An item with many units takes the plain launch of its own: the persistent loop pays
  // off for many small items, and a large one fills the GPU by itself (same tile body,
  // same results).
  for (size_t i = 0; i < P.size();) {
    if (P[i].nitems < kBatchPlainUnits && P[i].nitems * P[i].nchan < kBatchPlainWork) {
      ++i;
      continue;
    }
    KernFn k = pick_kernel(keys[i].dtype, P[i]);
    rc = set_lds((const void*)k, ldss[i]);
    if (rc) return rc;
    const int64_t nblocks = (P[i].nitems + 7) / 8 * 8;
    if (nblocks > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "too many work items");
    hipLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(64 * (P[i].nw + P[i].nprod)), (size_t)ldss[i], st, P[i]);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "dedisp_tile launch");
    P.erase(P.begin() + (std::ptrdiff_t)i);
    keys.erase(keys.begin() + (std::ptrdiff_t)i);
    ldss.erase(ldss.begin() + (std::ptrdiff_t)i);
  }
  if (!P.empty()) {
    // one persistent launch per distinct key, in order of first appearance; each launch's
    // records are contiguous, then its XCD runs [xcd][item + 1]
    struct Group {
      LdsKey key;
      int first, count;
      int64_t run_at, units, lds;
    };
    std::vector<Group> groups;
    std::vector<KParams> rec;
    std::vector<int64_t> start;
    for (size_t i = 0; i < P.size(); ++i) {
      bool seen = false;
      for (const Group& gr : groups) seen = seen || gr.key == keys[i];
      if (seen) continue;
      Group gr{keys[i], (int)rec.size(), 0, 0, 0, 0};
      for (size_t j = i; j < P.size(); ++j)
        if (keys[j] == keys[i]) {
          rec.push_back(P[j]);
          gr.lds = std::max(gr.lds, ldss[j]);
          ++gr.count;
        }
      gr.run_at = (int64_t)start.size();
      start.resize(start.size() + (size_t)8 * (gr.count + 1), 0);
      for (int x = 0; x < 8; ++x) {
        int64_t* sx = &start[(size_t)gr.run_at + (size_t)x * (gr.count + 1)];
        for (int j = 0; j < gr.count; ++j) {
          const int64_t u = rec[(size_t)gr.first + j].nitems;
          sx[j + 1] = sx[j] + (u * (x + 1)) / 8 - (u * x) / 8;  // XCD x's eighth of item j
        }
        gr.units = std::max(gr.units, sx[gr.count]);
      }
      groups.push_back(gr);
    }
    KParams* dP = reinterpret_cast<KParams*>(bw);
    int64_t* dS = reinterpret_cast<int64_t*>(bw + dd::align_up((int64_t)n * (int64_t)sizeof(KParams)));
    hipError_t e = hipMemcpyAsync(dP, rec.data(), rec.size() * sizeof(KParams), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dS, start.data(), start.size() * 8, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (batch descriptors)");
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
      ncu = 256;
    for (const Group& gr : groups) {
      int form = -1;
      for (int j = 0; j < gr.count; ++j) {
        const KParams& q = rec[(size_t)gr.first + j];
        const int f = q.nprod > 0 ? (q.g == 4 ? kProd4 : kProd) : q.x4 ? kX4 : kX1;
        form = form < 0 || form == f ? f : kAny;  // producer counts agree within a launch
      }
      BatchFn k = pick_batch_kernel(gr.key.dtype, form);
      rc = set_lds((const void*)k, gr.lds);
      if (rc) return rc;
      // as many resident workgroups per CU as the LDS and the wavefront slots hold (four
      // wavefronts per SIMD at the 4-trial form's registers, two at the 8-trial form's;
      // one workgroup when its ring fills the LDS), in whole XCD groups of 8; `units` is
      // the largest per-XCD share
      const int64_t wg_waves = gr.key.waves + gr.key.prod;
      const int64_t per_cu = std::max<int64_t>(
          1, std::min<int64_t>(dd::kLdsBytes / std::max<int64_t>(gr.lds, 1), (gr.key.per_wave == 4 ? 16 : 8) / wg_waves));
      const int64_t nblocks = std::max<int64_t>(8, std::min<int64_t>((int64_t)ncu * per_cu, gr.units * 8) / 8 * 8);
      hipLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(64 * (gr.key.waves + gr.key.prod)), (size_t)gr.lds, st,
                         (const KParams*)(dP + gr.first), (const int64_t*)(dS + gr.run_at), (int)gr.count);
      e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "dedisp_batch launch");
    }
  }
  const int64_t direct_desc = dd::direct_batch_desc_bytes(n);
  rc = dd::launch_direct_batch(direct, bw + lds_desc, direct_desc, st);
  if (rc) return rc;
  // statistics and candidates of every item: one launch per step for the whole batch
  std::vector<TailItem> tails, cands;
  int64_t nser = 0, nunit = 0;
  for (int32_t i = 0; i < n; ++i) {
    const dd_batch_item& it = items[i];
    const dd_plan* p = it.stream_item ? it.stream_item->plan : it.plan;
    const Outputs& o = outs[i];
    if (!(o.mean && o.rms)) continue;
    char* ws = static_cast<char*>(it.d_plan_workspace);
    const dd::WsLayout& l = lays[i];
    TailItem t{};
    t.part = reinterpret_cast<const double*>(ws + l.part_off);
    t.stat = reinterpret_cast<double*>(ws + l.thr_off);
    t.mean = o.mean;
    t.rms = o.rms;
    t.out = o.out;
    t.stride = o.out_stride;
    t.ntiles = (nouts[i] + kTile - 1) / kTile;
    t.nout = nouts[i];
    t.k = (double)o.k;
    t.ndm = p->ndm;
    t.ser0 = nser;
    nser += p->ndm;
    tails.push_back(t);
    if (o.k > 0.f && o.ncand) {
      t.nseg = (nouts[i] + dd::kStatSeg - 1) / dd::kStatSeg;
      t.cnt = reinterpret_cast<int32_t*>(ws + l.cnt_off);
      t.offs = reinterpret_cast<int64_t*>(ws + l.offs_off);
      t.ncand = o.ncand;
      t.cand = o.cand;
      t.cap = o.cand ? o.cap : 0;
      t.t_base = o.t_base;
      t.unit0 = nunit;
      nunit += (int64_t)p->ndm * t.nseg;
      cands.push_back(t);
    }
  }
  if (!tails.empty()) {
    const int64_t tail_bytes = dd::align_up((int64_t)n * (int64_t)sizeof(TailItem));
    TailItem* dT = reinterpret_cast<TailItem*>(bw + lds_desc + direct_desc);
    TailItem* dC = reinterpret_cast<TailItem*>(bw + lds_desc + direct_desc + tail_bytes);
    hipError_t e = hipMemcpyAsync(dT, tails.data(), tails.size() * sizeof(TailItem), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !cands.empty())
      e = hipMemcpyAsync(dC, cands.data(), cands.size() * sizeof(TailItem), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (batch statistics descriptors)");
    hipLaunchKernelGGL(stats_finalize_batch, dim3((unsigned)((nser + 3) / 4)), dim3(256), 0, st,
                       (const TailItem*)dT, (int)tails.size(), nser);
    if (nunit > 0x7fffffff) return dd::fail(DD_ERR_UNSUPPORTED, "too many candidate segments in one batch");
    if (!cands.empty() && nunit > 0) {
      const int nc = (int)cands.size();
      hipLaunchKernelGGL(cand_count_batch, dim3((unsigned)nunit), dim3(256), 0, st, (const TailItem*)dC, nc);
      hipLaunchKernelGGL(cand_scan_batch, dim3((unsigned)nc), dim3(1024), 0, st, (const TailItem*)dC);
      hipLaunchKernelGGL(cand_write_batch, dim3((unsigned)nunit), dim3(256), 0, st, (const TailItem*)dC, nc);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batched statistics/candidate launch");
  }
  for (int32_t i = 0; i < n; ++i)
    if (items[i].stream_item) items[i].stream_item->pending_n = 0;
  return DD_OK;
}


// ------------------------------------------------------------------ time-binned plans

}  // extern "C"

struct dd_binned {
  int32_t nchan = 0, ndm = 0, dtype = DD_F32, max_log2 = 0;
  double tsamp = 0.0, dm_diag = 0.0;
  struct Run {
    int32_t k, d0, d1;
    dd_plan* plan;
  };
  std::vector<Run> runs;
  ~dd_binned() {
    for (Run& r : runs) dd_plan_destroy(r.plan);
  }
};

namespace {

// Workspace of a time-binned call on nsamp samples: the downfactored inputs (levels 1 .. K,
// FP32, rows of 64-sample multiples), each run's plan workspace (its delay table first, as
// dd_plan_upload places it), the batch descriptors and the merged candidate region.
struct BinnedLayout {
  int64_t level_off[17] = {0}, level_row[17] = {0};
  std::vector<int64_t> run_off, nout;
  std::vector<dd::WsLayout> run_l;
  int64_t batch_off = 0, cand_off = 0, total = 0;
};

// Side streams (default priority) and events that let a binned plan's runs overlap, per
// host thread and device: a plan is an immutable object that several threads may share.
// Created on first use and kept for the life of the process.
struct SidePool {
  int dev = -1;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
};
int side_pool(size_t nstreams, size_t nevents, SidePool** out) {
  thread_local std::vector<SidePool> pools;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  SidePool* p = nullptr;
  for (SidePool& q : pools)
    if (q.dev == dev) p = &q;
  if (!p) {
    pools.push_back(SidePool{});
    p = &pools.back();
    p->dev = dev;
  }
  while (p->streams.size() < nstreams) {
    hipStream_t x = nullptr;
    e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags (binned runs)");
    p->streams.push_back(x);
  }
  while (p->events.size() < nevents) {
    hipEvent_t x = nullptr;
    e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags (binned runs)");
    p->events.push_back(x);
  }
  *out = p;
  return DD_OK;
}

int binned_layout(const dd_binned* b, int64_t nsamp, BinnedLayout* L) {
  int64_t o = 0;
  int kmax = 0;
  for (const dd_binned::Run& r : b->runs) kmax = std::max(kmax, r.k);
  for (int k = 1; k <= kmax; ++k) {
    L->level_row[k] = dd::align_up(nsamp >> k, 64);
    L->level_off[k] = o;
    o += dd::align_up((int64_t)b->nchan * L->level_row[k] * 4);
  }
  std::vector<MergedRun> mr;
  for (const dd_binned::Run& r : b->runs) {
    const int64_t nk = nsamp >> r.k;
    const int64_t nout = nk - r.plan->maxdelay;
    if (nout < 1)
      return dd::fail(DD_ERR_TOO_SHORT, "nsamp too short for the run at factor " + std::to_string(1 << r.k) +
                                            " (needs more than " + std::to_string(r.plan->maxdelay) + " samples there)");
    const dd::WsLayout l = dd::workspace_layout(r.plan, nk, true);
    L->run_off.push_back(o);
    L->run_l.push_back(l);
    L->nout.push_back(nout);
    o += dd::align_up(l.total);
    mr.push_back(MergedRun{nullptr, 0, nout, nullptr, r.d1 - r.d0, r.d0, r.k});
  }
  std::vector<dd_batch_item> none((size_t)b->runs.size());
  int64_t bq = 0;
  dd_batch_query(none.data(), (int32_t)none.size(), &bq);
  L->batch_off = o;
  o += dd::align_up(bq);
  L->cand_off = o;
  o += merged_cand_bytes(mr);
  L->total = o;
  return DD_OK;
}

}  // namespace

extern "C" {

int dd_binned_create(dd_binned** out, const double* freq_mhz, int32_t nchan, double tsamp_s, const double* dm,
                     int32_t ndm, int32_t in_dtype, int32_t max_log2, const dd_tuning* tuning) {
  dd::clear_error();
  if (!out) return dd::fail(DD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!dm || ndm < 1) return dd::fail(DD_ERR_INVALID_ARG, "dm must be non-NULL with ndm >= 1");
  std::vector<int32_t> lg((size_t)ndm);
  double diag = 0.0;
  int rc = dd_time_binning(freq_mhz, nchan, tsamp_s, dm, ndm, max_log2, &diag, lg.data());
  if (rc) return rc;
  dd_binned* b = new (std::nothrow) dd_binned();
  if (!b) return dd::fail(DD_ERR_INVALID_ARG, "out of host memory");
  b->nchan = nchan;
  b->ndm = ndm;
  b->dtype = in_dtype;
  b->max_log2 = max_log2;
  b->tsamp = tsamp_s;
  b->dm_diag = diag;
  // Runs with k >= 1 read FP32 sums. Which runs a tuning applies to:
  //  * DD_FORM_DIRECT: the factor-1 run only (8-bit input);
  //  * DD_FORM_LDS or DD_FORM_REGWIN: every run;
  //  * DD_FORM_AUTO with tile fields: every FP32 run, and an 8-bit factor-1 run keeps the
  //    direct-read form (the tiles are LDS-form tiles; the direct-read form is the 8-bit
  //    default).
  // Without a tuning each run takes the planner's tiles for its own trials: a common tiling
  // that every run can take (fewer trials per workgroup for the runs at small factors, whose
  // DM groups spread over more samples) was slower on the 4096-channel beams than separate
  // launches on each run's own tiles.
  const int form = tuning ? tuning->kernel_form : DD_FORM_AUTO;
  const bool u8_direct0 = in_dtype == DD_U8 && (form == DD_FORM_DIRECT || form == DD_FORM_AUTO);
  std::vector<std::pair<int32_t, int32_t>> spans;
  for (int32_t d0 = 0, d = 1; d <= ndm; ++d) {
    if (d < ndm && lg[d] == lg[d0]) continue;
    spans.push_back({d0, d});
    d0 = d;
  }
  auto make = [&](int32_t d0, int32_t d1, const dd_tuning* t, dd_plan** p) {
    const int32_t k = lg[d0];
    return dd_plan_create(p, freq_mhz, nchan, tsamp_s * (double)(1 << k), dm + d0, d1 - d0,
                          k == 0 ? in_dtype : DD_F32, t);
  };
  auto tuning_for = [&](int32_t k) -> const dd_tuning* {
    if (k == 0) return u8_direct0 && form == DD_FORM_AUTO ? nullptr : tuning;
    return form == DD_FORM_DIRECT ? nullptr : tuning;
  };
  for (const auto& sp : spans) {
    dd_plan* p = nullptr;
    rc = make(sp.first, sp.second, tuning_for(lg[sp.first]), &p);
    if (rc) {
      delete b;
      return rc;
    }
    b->runs.push_back(dd_binned::Run{lg[sp.first], sp.first, sp.second, p});
  }
  *out = b;
  return DD_OK;
}

void dd_binned_destroy(dd_binned* b) { delete b; }

int dd_binned_query(const dd_binned* b, int64_t nsamp, int32_t* nruns, dd_binned_run* runs, int32_t runs_cap,
                    int64_t* workspace_bytes, double* dm_diag) {
  dd::clear_error();
  if (!b) return dd::fail(DD_ERR_INVALID_ARG, "plan is NULL");
  if (nruns) *nruns = (int32_t)b->runs.size();
  if (dm_diag) *dm_diag = b->dm_diag;
  if (runs) {
    for (int32_t i = 0; i < runs_cap && i < (int32_t)b->runs.size(); ++i) {
      const dd_binned::Run& r = b->runs[i];
      dd_binned_run o{};
      o.log2 = r.k;
      o.d0 = r.d0;
      o.d1 = r.d1;
      o.maxdelay = r.plan->maxdelay;
      o.nout = nsamp > 0 ? (nsamp >> r.k) - r.plan->maxdelay : 0;
      o.kernel_form = r.plan->launch.form;
      o.dms_per_wave = r.plan->tiles.g;
      o.waves = r.plan->tiles.w;
      o.producer_waves = r.plan->launch.prod;
      runs[i] = o;
    }
  }
  if (workspace_bytes) *workspace_bytes = 0;
  if (nsamp <= 0) return dd::fail(DD_ERR_INVALID_ARG, "nsamp must be > 0");
  BinnedLayout L;
  const int rc = binned_layout(b, nsamp, &L);
  if (rc) return rc;
  if (workspace_bytes) *workspace_bytes = L.total;
  return DD_OK;
}

int dd_binned_upload(const dd_binned* b, int64_t nsamp, void* d_workspace, int64_t ws_bytes, void* stream) {
  dd::clear_error();
  if (!b || !d_workspace) return dd::fail(DD_ERR_INVALID_ARG, "plan and workspace must be non-NULL");
  BinnedLayout L;
  int rc = binned_layout(b, nsamp, &L);
  if (rc) return rc;
  if (ws_bytes < L.total) return dd::fail(DD_ERR_WORKSPACE, "workspace smaller than dd_binned_query asks for");
  for (size_t i = 0; i < b->runs.size(); ++i) {
    rc = dd_plan_upload(b->runs[i].plan, static_cast<char*>(d_workspace) + L.run_off[i], L.run_l[i].total, stream);
    if (rc) return rc;
  }
  return DD_OK;
}

int dd_binned_dedisperse(const dd_binned* b, const void* d_in, int64_t nsamp, int64_t in_row_stride, float* d_out,
                         int64_t out_row_stride, float* d_mean, float* d_rms, float k_sigma, dd_cand* d_cand,
                         int64_t cand_cap, int64_t* d_ncand, int32_t batched, void* d_workspace, int64_t ws_bytes,
                         void* stream) {
  dd::clear_error();
  if (!b || !d_in || !d_workspace) return dd::fail(DD_ERR_INVALID_ARG, "plan, input and workspace are required");
  if (in_row_stride < nsamp) return dd::fail(DD_ERR_INVALID_ARG, "in_row_stride < nsamp");
  BinnedLayout L;
  int rc = binned_layout(b, nsamp, &L);
  if (rc) return rc;
  if (ws_bytes < L.total) return dd::fail(DD_ERR_WORKSPACE, "workspace smaller than dd_binned_query asks for");
  const int64_t nout_max = *std::max_element(L.nout.begin(), L.nout.end());
  rc = check_outputs(b->runs[0].plan, d_out, out_row_stride, nout_max, d_mean, d_rms, k_sigma, d_cand, cand_cap,
                     d_ncand);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(d_workspace);
  // the downfactored inputs, each level from the one below
  int kmax = 0;
  for (const dd_binned::Run& r : b->runs) kmax = std::max(kmax, r.k);
  const void* lvl = d_in;
  int32_t lvl_dtype = b->dtype;
  int64_t lvl_stride = in_row_stride;
  std::vector<const void*> level_ptr(kmax + 1, d_in);
  std::vector<int64_t> level_stride(kmax + 1, in_row_stride);
  // unbatched: each run on a side stream of its own, started as soon as its level exists
  // (events 0 .. kmax: the levels; then one per run), joined before the merged candidates
  SidePool* sp = nullptr;
  if (!batched) {
    rc = side_pool(b->runs.size(), (size_t)kmax + 1 + b->runs.size(), &sp);
    if (rc) return rc;
    const hipError_t e = hipEventRecord(sp->events[0], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord (binned levels)");
  }
  for (int k = 1; k <= kmax; ++k) {
    float* dst = reinterpret_cast<float*>(ws + L.level_off[k]);
    rc = dd_downfactor(lvl, lvl_dtype, b->nchan, nsamp >> (k - 1), lvl_stride, dst, L.level_row[k], stream);
    if (rc) return rc;
    if (sp) {
      const hipError_t e = hipEventRecord(sp->events[(size_t)k], st);
      if (e != hipSuccess) return hip_fail(e, "hipEventRecord (binned levels)");
    }
    level_ptr[k] = dst;
    level_stride[k] = L.level_row[k];
    lvl = dst;
    lvl_dtype = DD_F32;
    lvl_stride = L.level_row[k];
  }
  const bool stats = d_mean && d_rms;
  if (batched) {
    std::vector<dd_batch_item> items(b->runs.size());
    for (size_t i = 0; i < b->runs.size(); ++i) {
      const dd_binned::Run& r = b->runs[i];
      dd_batch_item& it = items[i];
      it = dd_batch_item{};
      it.plan = r.plan;
      it.d_in = level_ptr[r.k];
      it.nsamp = nsamp >> r.k;
      it.in_row_stride = level_stride[r.k];
      it.d_out = d_out + (int64_t)r.d0 * out_row_stride;
      it.out_row_stride = out_row_stride;
      it.d_mean = stats ? d_mean + r.d0 : nullptr;
      it.d_rms = stats ? d_rms + r.d0 : nullptr;
      it.k_sigma = k_sigma;  // thresholds for the merged pass; no candidate buffers here
      it.d_plan_workspace = ws + L.run_off[i];
    }
    rc = dd_batch_dedisperse(items.data(), (int32_t)items.size(), ws + L.batch_off, L.cand_off - L.batch_off, stream);
    if (rc) return rc;
  } else {
    for (size_t i = 0; i < b->runs.size(); ++i) {
      const dd_binned::Run& r = b->runs[i];
      char* rw = ws + L.run_off[i];
      const InView in{level_ptr[r.k], level_stride[r.k], nsamp >> r.k, 0, 0};
      // k sets the thresholds the merged candidate pass reads; no candidate buffers here
      const Outputs o{d_out + (int64_t)r.d0 * out_row_stride, out_row_stride, stats ? d_mean + r.d0 : nullptr,
                      stats ? d_rms + r.d0 : nullptr, k_sigma, nullptr, 0, nullptr, 0};
      hipStream_t side = sp->streams[i];
      hipEvent_t done = sp->events[(size_t)kmax + 1 + i];
      hipError_t e = hipStreamWaitEvent(side, sp->events[(size_t)r.k], 0);
      if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent (binned run)");
      rc = run_pipeline(r.plan, in, reinterpret_cast<const int32_t*>(rw + L.run_l[i].table_off), L.nout[i], o, rw,
                        L.run_l[i], side, true);
      if (rc) return rc;
      e = hipEventRecord(done, side);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, done, 0);
      if (e != hipSuccess) return hip_fail(e, "binned pass: joining a run");
    }
  }
  if (stats && k_sigma > 0.f && d_ncand) {
    std::vector<MergedRun> mr;
    for (size_t i = 0; i < b->runs.size(); ++i) {
      const dd_binned::Run& r = b->runs[i];
      mr.push_back(MergedRun{d_out + (int64_t)r.d0 * out_row_stride, out_row_stride, L.nout[i],
                             reinterpret_cast<const double*>(ws + L.run_off[i] + L.run_l[i].thr_off), r.d1 - r.d0,
                             r.d0, r.k});
    }
    rc = merged_candidates(mr, k_sigma, d_cand, cand_cap, d_ncand, ws + L.cand_off, st);
    if (rc) return rc;
  }
  return DD_OK;
}

// ------------------------------------------------------------------ time-binned streams

}  // extern "C"

// A stream over a time-binned plan: one ordinary stream per run, run k's ring holding the
// input downfactored k times (block_nsamp >> k samples per block), so every run keeps only
// its own maxdelay at its own sampling time.
struct dd_binned_stream {
  const dd_binned* b = nullptr;
  int64_t block = 0;
  int32_t kmax = 0;
  std::vector<dd_stream*> runs;
  // one side stream per run (default priority) and the events that order them after the
  // block's appends and before the merged candidates: the runs' dedispersion is
  // independent (own rings, workspaces and output rows), and each run alone leaves most of
  // the GPU idle
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> done;
  hipEvent_t ready = nullptr;
  ~dd_binned_stream() {
    for (dd_stream* s : runs) dd_stream_destroy(s);
    for (hipStream_t x : side) (void)hipStreamDestroy(x);
    for (hipEvent_t e : done) (void)hipEventDestroy(e);
    if (ready) (void)hipEventDestroy(ready);
  }
};

namespace {

int binned_kmax(const dd_binned* b) {
  int k = 0;
  for (const dd_binned::Run& r : b->runs) k = std::max(k, r.k);
  return k;
}

// Ring of a binned stream: each run's stream ring (its delay table first), 256-byte aligned.
int64_t binned_ring_layout(const dd_binned* b, int64_t block, std::vector<int64_t>* off) {
  int64_t o = 0;
  for (const dd_binned::Run& r : b->runs) {
    dd_plan_info info;
    dd_plan_query(r.plan, block >> r.k, &info);
    if (off) off->push_back(o);
    o += dd::align_up(info.ring_bytes);
  }
  dd::clear_error();
  return o;
}

// Workspace of one push: the downfactored block (levels 1 .. K), each run's stream
// workspace, the batch descriptors and the merged candidate region.
struct BinnedStreamLayout {
  int64_t level_off[17] = {0}, level_row[17] = {0};
  std::vector<int64_t> run_off;
  std::vector<dd::WsLayout> run_l;
  int64_t batch_off = 0, cand_off = 0, total = 0;
};

BinnedStreamLayout binned_stream_layout(const dd_binned* b, int64_t block) {
  BinnedStreamLayout L;
  int64_t o = 0;
  const int kmax = binned_kmax(b);
  for (int k = 1; k <= kmax; ++k) {
    L.level_row[k] = dd::align_up(block >> k, 64);
    L.level_off[k] = o;
    o += dd::align_up((int64_t)b->nchan * L.level_row[k] * 4);
  }
  std::vector<MergedRun> mr;
  for (const dd_binned::Run& r : b->runs) {
    const dd::WsLayout l = dd::workspace_layout(r.plan, block >> r.k, false);
    L.run_off.push_back(o);
    L.run_l.push_back(l);
    o += dd::align_up(l.total);
    mr.push_back(MergedRun{nullptr, 0, block >> r.k, nullptr, r.d1 - r.d0, r.d0, r.k});
  }
  std::vector<dd_batch_item> none((size_t)b->runs.size());
  int64_t bq = 0;
  dd_batch_query(none.data(), (int32_t)none.size(), &bq);
  L.batch_off = o;
  o += dd::align_up(bq);
  L.cand_off = o;
  o += merged_cand_bytes(mr);
  L.total = o;
  return L;
}

// The batched path's condition (no register-window run: that form is not batched), checked
// before anything is appended.
bool binned_batchable(const dd_binned* b) {
  for (const dd_binned::Run& r : b->runs)
    if (r.plan->launch.form == dd::kFormRegWin) return false;
  return true;
}

}  // namespace

extern "C" {

int dd_binned_stream_query(const dd_binned* b, int64_t block_nsamp, int64_t* ring_bytes, int64_t* workspace_bytes) {
  dd::clear_error();
  if (ring_bytes) *ring_bytes = 0;
  if (workspace_bytes) *workspace_bytes = 0;
  if (!b) return dd::fail(DD_ERR_INVALID_ARG, "plan is NULL");
  const int kmax = binned_kmax(b);
  if (block_nsamp < (1 << kmax) || block_nsamp % (1 << kmax) != 0)
    return dd::fail(DD_ERR_INVALID_ARG, "block_nsamp must be a positive multiple of " + std::to_string(1 << kmax) +
                                            " (the largest binning factor)");
  if (ring_bytes) *ring_bytes = binned_ring_layout(b, block_nsamp, nullptr);
  if (workspace_bytes) *workspace_bytes = binned_stream_layout(b, block_nsamp).total;
  return DD_OK;
}

int dd_binned_stream_create(const dd_binned* b, int64_t block_nsamp, void* d_ring, int64_t ring_bytes, void* stream,
                            dd_binned_stream** out) {
  dd::clear_error();
  if (!out) return dd::fail(DD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!b || !d_ring) return dd::fail(DD_ERR_INVALID_ARG, "plan and ring must be non-NULL");
  int64_t need = 0;
  int rc = dd_binned_stream_query(b, block_nsamp, &need, nullptr);
  if (rc) return rc;
  if (ring_bytes < need) return dd::fail(DD_ERR_WORKSPACE, "ring smaller than dd_binned_stream_query asks for");
  std::vector<int64_t> off;
  binned_ring_layout(b, block_nsamp, &off);
  dd_binned_stream* s = new (std::nothrow) dd_binned_stream();
  if (!s) return dd::fail(DD_ERR_INVALID_ARG, "out of host memory");
  s->b = b;
  s->block = block_nsamp;
  s->kmax = binned_kmax(b);
  for (size_t i = 0; i < b->runs.size(); ++i) {
    const dd_binned::Run& r = b->runs[i];
    dd_plan_info info;
    dd_plan_query(r.plan, block_nsamp >> r.k, &info);
    dd_stream* rs = nullptr;
    rc = dd_stream_create(r.plan, block_nsamp >> r.k, static_cast<char*>(d_ring) + off[i], info.ring_bytes, stream,
                          &rs);
    if (rc) {
      delete s;
      return rc;
    }
    s->runs.push_back(rs);
  }
  hipError_t e = hipEventCreateWithFlags(&s->ready, hipEventDisableTiming);
  for (size_t i = 0; e == hipSuccess && i < b->runs.size(); ++i) {
    hipStream_t x = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
    if (e == hipSuccess) s->side.push_back(x);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) s->done.push_back(ev);
  }
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "binned stream: side streams and events");
  }
  *out = s;
  return DD_OK;
}

void dd_binned_stream_destroy(dd_binned_stream* s) { delete s; }

int dd_binned_stream_set_gap_fill(dd_binned_stream* s, int32_t enable) {
  dd::clear_error();
  if (!s) return dd::fail(DD_ERR_INVALID_ARG, "stream is NULL");
  for (dd_stream* r : s->runs) r->gap_fill = enable != 0;
  return DD_OK;
}

int dd_binned_stream_push(dd_binned_stream* s, const void* d_block, int64_t nsamp, int64_t in_row_stride, int64_t seq,
                          float* d_out, int64_t out_row_stride, float* d_mean, float* d_rms, float k_sigma,
                          dd_cand* d_cand, int64_t cand_cap, int64_t* d_ncand, int32_t batched, void* d_workspace,
                          int64_t ws_bytes, void* stream, int64_t* t0_out, int64_t* nout_out) {
  dd::clear_error();
  if (!s) return dd::fail(DD_ERR_INVALID_ARG, "stream is NULL");
  const dd_binned* b = s->b;
  const size_t nr = b->runs.size();
  for (size_t i = 0; i < nr; ++i) {
    if (t0_out) t0_out[i] = 0;
    if (nout_out) nout_out[i] = 0;
  }
  if (!d_block || !d_workspace) return dd::fail(DD_ERR_INVALID_ARG, "block and workspace must be non-NULL");
  if (nsamp < 1 || nsamp > s->block) return dd::fail(DD_ERR_INVALID_ARG, "block size out of range");
  if (nsamp % (1 << s->kmax) != 0)
    return dd::fail(DD_ERR_INVALID_ARG, "nsamp must be a multiple of " + std::to_string(1 << s->kmax) +
                                            " (the largest binning factor)");
  if (in_row_stride < nsamp) return dd::fail(DD_ERR_INVALID_ARG, "in_row_stride < nsamp");
  int rc = check_outputs(b->runs[0].plan, d_out, out_row_stride, s->block, d_mean, d_rms, k_sigma, d_cand, cand_cap,
                         d_ncand);
  if (rc) return rc;
  const BinnedStreamLayout L = binned_stream_layout(b, s->block);
  if (ws_bytes < L.total) return dd::fail(DD_ERR_WORKSPACE, "workspace smaller than dd_binned_stream_query asks for");
  // every run's stream expects the same seq; checked once, before anything is enqueued
  const dd_stream* s0 = s->runs[0];
  if (seq != s0->next_seq && !(s0->gap_fill && seq > s0->next_seq))
    return dd::fail(DD_ERR_SEQUENCE, "expected seq " + std::to_string(s0->next_seq) + ", got " + std::to_string(seq));
  if (batched && !binned_batchable(b))
    return dd::fail(DD_ERR_UNSUPPORTED, "register-window runs are not batched; use DD_FORM_LDS or batched = 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(d_workspace);
  // the block downfactored 1 .. K times; blocks are multiples of 2^K samples, so no pair of
  // samples straddles two blocks and each level equals the whole stream's downfactored input
  std::vector<const void*> level_ptr((size_t)s->kmax + 1, d_block);
  std::vector<int64_t> level_stride((size_t)s->kmax + 1, in_row_stride);
  for (int k = 1; k <= s->kmax; ++k) {
    float* dst = reinterpret_cast<float*>(ws + L.level_off[k]);
    rc = dd_downfactor(level_ptr[k - 1], k == 1 ? b->dtype : DD_F32, b->nchan, nsamp >> (k - 1),
                       level_stride[k - 1], dst, L.level_row[k], stream);
    if (rc) return rc;
    level_ptr[k] = dst;
    level_stride[k] = L.level_row[k];
  }
  std::vector<int64_t> t0((size_t)nr, 0), n((size_t)nr, 0);
  bool any = false;
  for (size_t i = 0; i < nr; ++i) {
    const int k = b->runs[i].k;
    rc = dd_stream_append(s->runs[i], level_ptr[k], nsamp >> k, level_stride[k], seq, stream, &t0[i], &n[i]);
    if (rc == DD_FILLING) {
      n[i] = 0;
      continue;
    }
    if (rc) {
      for (dd_stream* r : s->runs) r->pending_n = 0;
      return rc;
    }
    any = true;
  }
  if (!any) return DD_FILLING;
  const bool stats = d_mean && d_rms;
  if (batched) {
    std::vector<dd_batch_item> items;
    for (size_t i = 0; i < nr; ++i) {
      if (n[i] == 0) continue;
      const dd_binned::Run& r = b->runs[i];
      dd_batch_item it{};
      it.d_out = d_out + (int64_t)r.d0 * out_row_stride;
      it.out_row_stride = out_row_stride;
      it.d_mean = stats ? d_mean + r.d0 : nullptr;
      it.d_rms = stats ? d_rms + r.d0 : nullptr;
      it.k_sigma = k_sigma;  // thresholds for the merged pass; no candidate buffers here
      it.d_plan_workspace = ws + L.run_off[i];
      it.stream_item = s->runs[i];
      items.push_back(it);
    }
    rc = dd_batch_dedisperse(items.data(), (int32_t)items.size(), ws + L.batch_off, L.cand_off - L.batch_off, stream);
  } else {
    // each run on its own side stream, after the appends and before the merged candidates
    hipError_t e = hipEventRecord(s->ready, st);
    if (e != hipSuccess) rc = hip_fail(e, "hipEventRecord (binned stream)");
    for (size_t i = 0; i < nr && rc == DD_OK; ++i) {
      if (n[i] == 0) continue;
      const dd_binned::Run& r = b->runs[i];
      dd_stream* rs = s->runs[i];
      const dd_plan* p = r.plan;
      const InView in{static_cast<char*>(rs->ring) + dd::ring_table_bytes(p), rs->ring_row, n[i] + p->maxdelay,
                      rs->ring_len, t0[i]};
      const Outputs o{d_out + (int64_t)r.d0 * out_row_stride, out_row_stride, stats ? d_mean + r.d0 : nullptr,
                      stats ? d_rms + r.d0 : nullptr, k_sigma, nullptr, 0, nullptr, t0[i]};
      e = hipStreamWaitEvent(s->side[i], s->ready, 0);
      if (e != hipSuccess) {
        rc = hip_fail(e, "hipStreamWaitEvent (binned stream)");
        break;
      }
      rc = run_pipeline(p, in, static_cast<const int32_t*>(rs->ring), n[i], o, ws + L.run_off[i], L.run_l[i],
                        s->side[i], true);
      rs->pending_n = 0;
      if (rc) break;
      e = hipEventRecord(s->done[i], s->side[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, s->done[i], 0);
      if (e != hipSuccess) rc = hip_fail(e, "binned stream: joining a run");
    }
  }
  if (rc) {
    for (dd_stream* r : s->runs) r->pending_n = 0;
    return rc;
  }
  if (stats && k_sigma > 0.f && d_ncand) {
    std::vector<MergedRun> mr;
    for (size_t i = 0; i < nr; ++i) {
      if (n[i] == 0) continue;
      const dd_binned::Run& r = b->runs[i];
      MergedRun m{d_out + (int64_t)r.d0 * out_row_stride, out_row_stride, n[i],
                  reinterpret_cast<const double*>(ws + L.run_off[i] + L.run_l[i].thr_off), r.d1 - r.d0, r.d0, r.k};
      m.t_base = t0[i] << r.k;
      mr.push_back(m);
    }
    rc = merged_candidates(mr, k_sigma, d_cand, cand_cap, d_ncand, ws + L.cand_off, st);
    if (rc) return rc;
  }
  for (size_t i = 0; i < nr; ++i) {
    if (t0_out) t0_out[i] = t0[i];
    if (nout_out) nout_out[i] = n[i];
  }
  return DD_OK;
}

// ------------------------------------------------------------------ subband plans

}  // extern "C"

struct dd_subband {
  int32_t nchan = 0, ndm = 0, chans_per_sub = 0, dms_per_group = 0;
  double tsamp = 0.0;
  std::vector<std::pair<int32_t, int32_t>> subs, groups;
  std::vector<dd_plan*> step1, step2;
  int32_t maxdelay1 = 0, min_maxdelay1 = 0;
  ~dd_subband() {
    for (dd_plan* p : step1) dd_plan_destroy(p);
    for (dd_plan* p : step2) dd_plan_destroy(p);
  }
};

namespace {

// Workspace of a subband call: the reduced filterbank [nsub][ngroups][width] (step-1
// outputs; width a 64-sample multiple), each step-1 and step-2 plan's workspace, the batch
// descriptors and the merged candidate region.
struct SubbandLayout {
  int64_t width = 0, len1 = 0, red_off = 0, batch_off = 0, cand_off = 0, total = 0;
  std::vector<int64_t> off1, off2, nout1, nout2;
  std::vector<dd::WsLayout> l1, l2;
};

int subband_layout(const dd_subband* sp, int64_t nsamp, SubbandLayout* L) {
  L->len1 = nsamp - sp->maxdelay1;
  if (L->len1 < 1) return dd::fail(DD_ERR_TOO_SHORT, "nsamp must exceed the subband delays");
  L->width = dd::align_up(nsamp - sp->min_maxdelay1, 64);
  int64_t o = 0;
  L->red_off = o;
  o += dd::align_up((int64_t)sp->subs.size() * sp->groups.size() * L->width * 4);
  for (dd_plan* p : sp->step1) {
    const dd::WsLayout l = dd::workspace_layout(p, nsamp, true);
    L->off1.push_back(o);
    L->l1.push_back(l);
    L->nout1.push_back(nsamp - p->maxdelay);
    o += dd::align_up(l.total);
  }
  std::vector<MergedRun> mr;
  for (size_t g = 0; g < sp->step2.size(); ++g) {
    dd_plan* p = sp->step2[g];
    const int64_t nout = L->len1 - p->maxdelay;
    if (nout < 1) return dd::fail(DD_ERR_TOO_SHORT, "nsamp must exceed the subband and group delays");
    const dd::WsLayout l = dd::workspace_layout(p, L->len1, true);
    L->off2.push_back(o);
    L->l2.push_back(l);
    L->nout2.push_back(nout);
    o += dd::align_up(l.total);
    mr.push_back(MergedRun{nullptr, 0, nout, nullptr, p->ndm, sp->groups[g].first, 0});
  }
  const int32_t nb = (int32_t)std::max(sp->step1.size(), sp->step2.size());
  std::vector<dd_batch_item> none((size_t)nb);
  int64_t bq = 0;
  dd_batch_query(none.data(), nb, &bq);
  L->batch_off = o;
  o += dd::align_up(bq);
  L->cand_off = o;
  o += merged_cand_bytes(mr);
  L->total = o;
  return DD_OK;
}

}  // namespace

extern "C" {

int dd_subband_create(dd_subband** out, const double* freq_mhz, int32_t nchan, double tsamp_s, const double* dm,
                      int32_t ndm, int32_t chans_per_sub, int32_t dms_per_group) {
  dd::clear_error();
  if (!out) return dd::fail(DD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!freq_mhz || !dm || nchan < 1 || ndm < 1)
    return dd::fail(DD_ERR_INVALID_ARG, "freq_mhz and dm must be non-NULL with nchan, ndm >= 1");
  if (chans_per_sub < 1 || dms_per_group < 1)
    return dd::fail(DD_ERR_INVALID_ARG, "chans_per_sub and dms_per_group must be >= 1");
  dd_subband* sp = new (std::nothrow) dd_subband();
  if (!sp) return dd::fail(DD_ERR_INVALID_ARG, "out of host memory");
  sp->nchan = nchan;
  sp->ndm = ndm;
  sp->chans_per_sub = chans_per_sub;
  sp->dms_per_group = dms_per_group;
  sp->tsamp = tsamp_s;
  for (int32_t c0 = 0; c0 < nchan; c0 += chans_per_sub) sp->subs.push_back({c0, std::min(nchan, c0 + chans_per_sub)});
  for (int32_t d0 = 0; d0 < ndm; d0 += dms_per_group) sp->groups.push_back({d0, std::min(ndm, d0 + dms_per_group)});
  // each group's nominal DM is its middle trial
  std::vector<double> nominal;
  for (const auto& g : sp->groups) nominal.push_back(dm[g.first + (g.second - g.first - 1) / 2]);
  std::vector<double> fsub;
  int rc = DD_OK;
  for (const auto& s : sp->subs) {
    dd_plan* p = nullptr;
    rc = dd_plan_create(&p, freq_mhz + s.first, s.second - s.first, tsamp_s, nominal.data(), (int32_t)nominal.size(),
                        DD_F32, nullptr);
    if (rc) break;
    sp->step1.push_back(p);
    fsub.push_back(*std::max_element(freq_mhz + s.first, freq_mhz + s.second));
  }
  // step 2: groups of dms_per_group trials share a workgroup, 4 trials per computing
  // wavefront beside 2 producers. A step-2 plan walks only the subbands, so its units are
  // short: the LDS budget lets as many workgroups share a CU as its 16 wavefront slots
  // hold (two for groups of 16), and each takes the budget's share of the LDS.
  dd_tuning t2{};
  t2.dms_per_wave = 4;
  t2.waves = std::max(1, std::min(14, (dms_per_group + 3) / 4));
  t2.producer_waves = 2;
  t2.kernel_form = DD_FORM_LDS;
  const int64_t share = std::max(1, 16 / (t2.waves + t2.producer_waves));
  for (size_t g = 0; rc == DD_OK && g < sp->groups.size(); ++g) {
    dd_plan* p = nullptr;
    // the budget's share, or the whole LDS when one group's windows need more; 8 trials per
    // wavefront when they do not fit the producers' DMAs at all
    const int32_t d0 = sp->groups[g].first, nd = sp->groups[g].second - sp->groups[g].first;
    for (int64_t div = share; div >= 1; div = div > 1 ? 1 : 0) {
      rc = dd::plan_create(&p, fsub.data(), (int32_t)fsub.size(), tsamp_s, dm + d0, nd, DD_F32, &t2,
                           dd::kLdsBytes / div);
      if (rc != DD_ERR_UNSUPPORTED) break;
    }
    if (rc == DD_ERR_UNSUPPORTED) {
      dd_tuning t8{};
      t8.dms_per_wave = 8;
      t8.waves = std::max(1, std::min(6, (dms_per_group + 7) / 8));
      t8.kernel_form = DD_FORM_LDS;
      rc = dd_plan_create(&p, fsub.data(), (int32_t)fsub.size(), tsamp_s, dm + d0, nd, DD_F32, &t8);
    }
    if (rc) break;
    sp->step2.push_back(p);
  }
  if (rc) {
    delete sp;
    return rc;
  }
  sp->maxdelay1 = 0;
  sp->min_maxdelay1 = std::numeric_limits<int32_t>::max();
  for (dd_plan* p : sp->step1) {
    sp->maxdelay1 = std::max(sp->maxdelay1, p->maxdelay);
    sp->min_maxdelay1 = std::min(sp->min_maxdelay1, p->maxdelay);
  }
  *out = sp;
  return DD_OK;
}

void dd_subband_destroy(dd_subband* sp) { delete sp; }

int dd_subband_query(const dd_subband* sp, int64_t nsamp, int64_t* workspace_bytes, int64_t* nout_per_dm,
                     int64_t* adds, int32_t* nsub, int32_t* ngroups) {
  dd::clear_error();
  if (!sp) return dd::fail(DD_ERR_INVALID_ARG, "plan is NULL");
  if (nsub) *nsub = (int32_t)sp->subs.size();
  if (ngroups) *ngroups = (int32_t)sp->groups.size();
  if (workspace_bytes) *workspace_bytes = 0;
  if (nsamp <= 0) return dd::fail(DD_ERR_INVALID_ARG, "nsamp must be > 0");
  SubbandLayout L;
  const int rc = subband_layout(sp, nsamp, &L);
  if (rc) return rc;
  if (workspace_bytes) *workspace_bytes = L.total;
  int64_t a = 0;
  for (size_t s = 0; s < sp->step1.size(); ++s) a += (int64_t)sp->step1[s]->ndm * sp->step1[s]->nchan * L.nout1[s];
  for (size_t g = 0; g < sp->step2.size(); ++g) {
    a += (int64_t)sp->step2[g]->ndm * sp->step2[g]->nchan * L.nout2[g];
    if (nout_per_dm)
      for (int32_t d = sp->groups[g].first; d < sp->groups[g].second; ++d) nout_per_dm[d] = L.nout2[g];
  }
  if (adds) *adds = a;
  return DD_OK;
}

int dd_subband_upload(const dd_subband* sp, int64_t nsamp, void* d_workspace, int64_t ws_bytes, void* stream) {
  dd::clear_error();
  if (!sp || !d_workspace) return dd::fail(DD_ERR_INVALID_ARG, "plan and workspace must be non-NULL");
  SubbandLayout L;
  int rc = subband_layout(sp, nsamp, &L);
  if (rc) return rc;
  if (ws_bytes < L.total) return dd::fail(DD_ERR_WORKSPACE, "workspace smaller than dd_subband_query asks for");
  char* ws = static_cast<char*>(d_workspace);
  for (size_t s = 0; s < sp->step1.size() && rc == DD_OK; ++s)
    rc = dd_plan_upload(sp->step1[s], ws + L.off1[s], L.l1[s].total, stream);
  for (size_t g = 0; g < sp->step2.size() && rc == DD_OK; ++g)
    rc = dd_plan_upload(sp->step2[g], ws + L.off2[g], L.l2[g].total, stream);
  return rc;
}

int dd_subband_dedisperse(const dd_subband* sp, const float* d_in, int64_t nsamp, int64_t in_row_stride, float* d_out,
                          int64_t out_row_stride, float* d_mean, float* d_rms, float k_sigma, dd_cand* d_cand,
                          int64_t cand_cap, int64_t* d_ncand, int32_t batched, void* d_workspace, int64_t ws_bytes,
                          void* stream) {
  dd::clear_error();
  if (!sp || !d_in || !d_workspace) return dd::fail(DD_ERR_INVALID_ARG, "plan, input and workspace are required");
  if (in_row_stride < nsamp) return dd::fail(DD_ERR_INVALID_ARG, "in_row_stride < nsamp");
  SubbandLayout L;
  int rc = subband_layout(sp, nsamp, &L);
  if (rc) return rc;
  if (ws_bytes < L.total) return dd::fail(DD_ERR_WORKSPACE, "workspace smaller than dd_subband_query asks for");
  const int64_t nout_max = *std::max_element(L.nout2.begin(), L.nout2.end());
  rc = check_outputs(sp->step2[0], d_out, out_row_stride, nout_max, d_mean, d_rms, k_sigma, d_cand, cand_cap, d_ncand);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(d_workspace);
  float* red = reinterpret_cast<float*>(ws + L.red_off);
  const int64_t ngrp = (int64_t)sp->groups.size();
  const bool stats = d_mean && d_rms;
  // step 1: subband s at the nominal DMs into red[s][g][:]
  if (batched) {
    std::vector<dd_batch_item> items(sp->step1.size());
    for (size_t s = 0; s < sp->step1.size(); ++s) {
      dd_batch_item& it = items[s];
      it = dd_batch_item{};
      it.plan = sp->step1[s];
      it.d_in = d_in + (int64_t)sp->subs[s].first * in_row_stride;
      it.nsamp = nsamp;
      it.in_row_stride = in_row_stride;
      it.d_out = red + (int64_t)s * ngrp * L.width;
      it.out_row_stride = L.width;
      it.d_plan_workspace = ws + L.off1[s];
    }
    rc = dd_batch_dedisperse(items.data(), (int32_t)items.size(), ws + L.batch_off, L.cand_off - L.batch_off, stream);
    if (rc) return rc;
  } else {
    for (size_t s = 0; s < sp->step1.size(); ++s) {
      char* rw = ws + L.off1[s];
      const InView in{d_in + (int64_t)sp->subs[s].first * in_row_stride, in_row_stride, nsamp, 0, 0};
      const Outputs o{red + (int64_t)s * ngrp * L.width, L.width, nullptr, nullptr, 0.f, nullptr, 0, nullptr, 0};
      rc = run_pipeline(sp->step1[s], in, reinterpret_cast<const int32_t*>(rw + L.l1[s].table_off), L.nout1[s], o, rw,
                        L.l1[s], st, true);
      if (rc) return rc;
    }
  }
  // step 2: group g over the reduced filterbank red[:][g][0 .. len1)
  if (batched) {
    std::vector<dd_batch_item> items(sp->step2.size());
    for (size_t g = 0; g < sp->step2.size(); ++g) {
      dd_batch_item& it = items[g];
      it = dd_batch_item{};
      it.plan = sp->step2[g];
      it.d_in = red + (int64_t)g * L.width;
      it.nsamp = L.len1;
      it.in_row_stride = ngrp * L.width;
      it.d_out = d_out + (int64_t)sp->groups[g].first * out_row_stride;
      it.out_row_stride = out_row_stride;
      it.d_mean = stats ? d_mean + sp->groups[g].first : nullptr;
      it.d_rms = stats ? d_rms + sp->groups[g].first : nullptr;
      it.k_sigma = k_sigma;
      it.d_plan_workspace = ws + L.off2[g];
    }
    rc = dd_batch_dedisperse(items.data(), (int32_t)items.size(), ws + L.batch_off, L.cand_off - L.batch_off, stream);
    if (rc) return rc;
  } else {
    // the step-2 plans are independent once step 1 is done and each is a short launch: they
    // go round-robin over a few side streams (the per-thread pool of the binned plans),
    // joined before the merged candidates
    constexpr size_t kSides = 4;
    SidePool* pool = nullptr;
    rc = side_pool(kSides, kSides + 1, &pool);
    if (rc) return rc;
    hipError_t e = hipEventRecord(pool->events[0], st);
    for (size_t x = 0; e == hipSuccess && x < kSides; ++x) e = hipStreamWaitEvent(pool->streams[x], pool->events[0], 0);
    if (e != hipSuccess) return hip_fail(e, "subband step 2: side streams");
    for (size_t g = 0; g < sp->step2.size(); ++g) {
      char* rw = ws + L.off2[g];
      const int32_t d0 = sp->groups[g].first;
      const InView in{red + (int64_t)g * L.width, ngrp * L.width, L.len1, 0, 0};
      const Outputs o{d_out + (int64_t)d0 * out_row_stride, out_row_stride, stats ? d_mean + d0 : nullptr,
                      stats ? d_rms + d0 : nullptr, k_sigma, nullptr, 0, nullptr, 0};
      rc = run_pipeline(sp->step2[g], in, reinterpret_cast<const int32_t*>(rw + L.l2[g].table_off), L.nout2[g], o, rw,
                        L.l2[g], pool->streams[g % kSides], true);
      if (rc) return rc;
    }
    for (size_t x = 0; e == hipSuccess && x < kSides; ++x) {
      e = hipEventRecord(pool->events[1 + x], pool->streams[x]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, pool->events[1 + x], 0);
    }
    if (e != hipSuccess) return hip_fail(e, "subband step 2: joining the side streams");
  }
  if (stats && k_sigma > 0.f && d_ncand) {
    std::vector<MergedRun> mr;
    for (size_t g = 0; g < sp->step2.size(); ++g) {
      const int32_t d0 = sp->groups[g].first;
      mr.push_back(MergedRun{d_out + (int64_t)d0 * out_row_stride, out_row_stride, L.nout2[g],
                             reinterpret_cast<const double*>(ws + L.off2[g] + L.l2[g].thr_off), sp->step2[g]->ndm, d0,
                             0});
    }
    rc = merged_candidates(mr, k_sigma, d_cand, cand_cap, d_ncand, ws + L.cand_off, st);
    if (rc) return rc;
  }
  return DD_OK;
}

}  // extern "C"
