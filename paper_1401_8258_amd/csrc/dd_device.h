// Device helpers shared by the dedispersion kernels (gfx950, wave64): input views,
// LDS DMA issue, explicit vmcnt waits, barriers and the fixed wavefront reduction.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dd_internal.h"

namespace dd {


typedef const __attribute__((address_space(4))) int32_t* ci32_t;

// Wavefront sum in a fixed butterfly (identical for every launch shape).
__device__ __forceinline__ double wave_sum_fixed(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One DPP move of a double (both halves), from the lane that CTRL names within the row.
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_double(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum over a whole wavefront (every lane active), valid in lane 0 only, with no LDS
// instruction: a butterfly over each 16-lane row by DPP moves, then lane 0 adds the four
// row sums. Row rotation by 8 pairs lane l with l ^ 8; after that step each row repeats
// with period 8, so rotation by 4 pairs l with a copy of l ^ 4, and quad permutations
// give xor 2 and xor 1. Lane 0 ends with the xor butterfly in the order 8, 4, 2, 1, 16,
// 32: (row 0 + row 1) + (row 2 + row 3). A fixed tree, so results depend on the inputs only.
__device__ __forceinline__ double wave_sum_lane0(double v) {
  v += dpp_double<0x128>(v);  // row_ror:8
  v += dpp_double<0x124>(v);  // row_ror:4
  v += dpp_double<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_double<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  return (v + readlane_double(v, 16)) + (readlane_double(v, 32) + readlane_double(v, 48));
}

// Exclusive scan of counts in tiles of 4096 by a 1024-thread block, each thread taking 4
// consecutive ones, so every load and store of a wavefront covers one contiguous span. A
// tile is scanned by wavefront shuffles and the 16 wavefront totals in LDS (part: at least
// 16 int64): offs[base + i] = carry + the counts before base + i in the tile. Returns the
// tile's total (in every thread).
constexpr int64_t kScanTile = 4096;
__device__ __forceinline__ int64_t scan_tile(const int32_t* __restrict__ cnt, int64_t n, int64_t base, int64_t carry,
                                             int64_t* __restrict__ offs, int64_t* part) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t i0 = base + 4 * tid;
  int c[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) c[k] = i0 + k < n ? cnt[i0 + k] : 0;
  const int64_t s = (int64_t)c[0] + c[1] + c[2] + c[3];
  int64_t incl = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) part[wv] = incl;
  __syncthreads();
  int64_t run = carry + incl - s, tile = 0;
  for (int k = 0; k < 16; ++k) {
    const int64_t p = part[k];
    run += k < wv ? p : 0;
    tile += p;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (i0 + k < n) offs[i0 + k] = run;
    run += c[k];
  }
  __syncthreads();  // every thread has read part before it is written again
  return tile;
}

// Exclusive scan of n counts by one 1024-thread block, tile after tile; the total to *total.
__device__ __forceinline__ void scan_counts(const int32_t* __restrict__ cnt, int64_t n, int64_t* __restrict__ offs,
                                            int64_t* __restrict__ total, int64_t* part) {
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += kScanTile) carry += scan_tile(cnt, n, base, carry, offs, part);
  if (threadIdx.x == 0) *total = carry;
}

// The same scan by many blocks, in three launches and no memory beyond offs (every
// candidate and detection compaction uses it; the offsets equal scan_counts's):
//  1. scan_tile_totals: block b parks the total of tile b in offs[4096 b];
//  2. scan_tile_bases (one block): an exclusive scan of those totals in place, the grand
//     total to *total;
//  3. scan_tile_apply: block b scans tile b from the base in offs[4096 b], rewriting that
//     slot with the same value.
__device__ __forceinline__ void scan_tile_totals(const int32_t* __restrict__ cnt, int64_t n,
                                                 int64_t* __restrict__ offs, int64_t* part) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int64_t i0 = base + 4 * tid;
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += i0 + k < n ? cnt[i0 + k] : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) part[wv] = s;
  __syncthreads();
  if (tid == 0) {
    int64_t t = 0;
    for (int k = 0; k < 16; ++k) t += part[k];
    offs[base] = t;
  }
}

__device__ __forceinline__ void scan_tile_bases(int64_t n, int64_t* __restrict__ offs, int64_t* __restrict__ total,
                                                int64_t* part) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < ntiles; c0 += 1024) {
    const int64_t k = c0 + tid;
    const int64_t v = k < ntiles ? offs[k * kScanTile] : 0;
    int64_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t u = __shfl_up(incl, off, 64);
      if (lane >= off) incl += u;
    }
    if (lane == 63) part[wv] = incl;
    __syncthreads();
    int64_t run = carry + incl - v, chunk = 0;
    for (int j = 0; j < 16; ++j) {
      const int64_t p = part[j];
      run += j < wv ? p : 0;
      chunk += p;
    }
    if (k < ntiles) offs[k * kScanTile] = run;
    carry += chunk;
    __syncthreads();
  }
  if (tid == 0) *total = carry;
}

__device__ __forceinline__ void scan_tile_apply(const int32_t* __restrict__ cnt, int64_t n,
                                                int64_t* __restrict__ offs, int64_t* part) {
  __shared__ int64_t base_off;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (threadIdx.x == 0) base_off = offs[base];
  __syncthreads();  // read before the tile's own offsets overwrite it
  scan_tile(cnt, n, base, base_off, offs, part);
}

__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

__device__ __forceinline__ void block_barrier() {
  compiler_fence();
  __builtin_amdgcn_s_barrier();
  compiler_fence();
}

// s_waitcnt vmcnt(n) with expcnt/lgkmcnt left open (gfx9 encoding), n in [0, 63].
#define DD_VMCNT(n) ((((n) & 15)) | (7 << 4) | (15 << 8) | ((((n) >> 4) & 3) << 14))
__device__ __forceinline__ void wait_vm(int n) {
  switch (n) {
#define DD_W4(b)                                                        \
  case b: __builtin_amdgcn_s_waitcnt(DD_VMCNT(b)); break;               \
  case b + 1: __builtin_amdgcn_s_waitcnt(DD_VMCNT(b + 1)); break;       \
  case b + 2: __builtin_amdgcn_s_waitcnt(DD_VMCNT(b + 2)); break;       \
  case b + 3: __builtin_amdgcn_s_waitcnt(DD_VMCNT(b + 3)); break;
    DD_W4(0) DD_W4(4) DD_W4(8) DD_W4(12) DD_W4(16) DD_W4(20) DD_W4(24) DD_W4(28)
    DD_W4(32) DD_W4(36) DD_W4(40) DD_W4(44) DD_W4(48) DD_W4(52) DD_W4(56) DD_W4(60)
#undef DD_W4
    default: __builtin_amdgcn_s_waitcnt(DD_VMCNT(0)); break;
  }
}

// One LDS DMA: lane i copies the element at base + voff into the 32-bit LDS word at
// lds + 4i (zero-extended for 1- and 2-byte elements). Issued from asm so the compiler
// neither serialises later LDS reads behind it nor counts it; the kernels wait for these
// with explicit vmcnt.
template <int EB>
__device__ __forceinline__ void dma(const void* base, unsigned voff, unsigned lds) {
  if constexpr (EB == 4)
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dword %0, %1" : : "v"(voff), "s"(base), "s"(lds) : "m0");
  else if constexpr (EB == 2)
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_ushort %0, %1" : : "v"(voff), "s"(base), "s"(lds) : "m0");
  else
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_ubyte %0, %1" : : "v"(voff), "s"(base), "s"(lds) : "m0");
}

// 16-byte LDS DMA: lane i copies 4 dwords from base + voff (4-byte aligned) to lds + 16i.
__device__ __forceinline__ void dma_x4(const void* base, unsigned voff, unsigned lds) {
  asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1" : : "v"(voff), "s"(base), "s"(lds) : "m0");
}

__device__ __forceinline__ unsigned lds_addr(const void* p) {
  return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

}  // namespace dd
