// Internal declarations shared by the host plan code and the HIP launch code.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dedisp.h"

namespace dd {

// Byte alignment of every region inside a workspace or ring.
constexpr int64_t kAlign = 256;
// Output samples per time tile of the dedispersion kernel; also the segment of
// the per-series statistics partials (fixed, so the reduction tree does not
// depend on the launch shape or on batching).
constexpr int64_t kTile = 512;
// Output samples per tile of the direct-read form (16 per lane): two statistics segments.
constexpr int64_t kDirectTile = 1024;
// Output samples per candidate-compaction segment.
constexpr int64_t kStatSeg = 8192;
// LDS of one gfx950 workgroup.
constexpr int64_t kLdsBytes = 160 * 1024;
// Most DMA instructions one wavefront issues per stage (its descriptor table spans four
// 64-lane registers).
constexpr int kMaxDma = 256;
// Most 16-byte DMAs one wavefront issues per stage for FP32 input (one descriptor
// register each); beyond that the 4-byte form is used.
constexpr int kMaxX4 = 16;
// Register-window form (FP32): DM trials per workgroup (8 wavefronts of 8) and channels
// per LDS stage; a wavefront's window holds at most kRwMaxChunks 4-sample chunks.
constexpr int kRwTrials = 64;
constexpr int kRwStage = 8;
constexpr int kRwMaxChunks = 12;
// Kernel forms (dd_tuning.kernel_form / dd_plan_info.kernel_form).
constexpr int kFormLds = 1;     // four shifted copies per channel in LDS, one LDS word per add
constexpr int kFormRegWin = 2;  // one copy per channel, register windows added in VGPR index mode
constexpr int kFormDirect = 3;  // 8-bit input read per trial through the caches, no LDS
// DD_FORM_AUTO picks the register-window form for FP32 plans it fits.
constexpr bool kAutoRegWin = false;

// Launch geometry of the dedispersion kernel.
struct Launch {
  int L;        // samples per (channel, copy) buffer (four copies shifted by 0..3 samples);
                // 32-bit words for 16/32-bit input, bytes for 8-bit input
  int cs;       // channels per stage (a divisor of the wavefront count unless prod > 0)
  int nb;       // stages in the LDS ring
  int nd;       // DMA instructions per stage channel share: per wavefront per stage, or
                // with a producer per channel
  int x4;       // FP32 data arrives by 16-byte DMAs
  int64_t lds;  // bytes
  int prod;     // wavefronts that only issue DMAs (0: every wavefront issues its share)
  int ndw;      // DMA instructions per issuing wavefront per stage (the vmcnt unit)
  int form;     // kFormLds, kFormRegWin or kFormDirect; for kFormRegWin, L is the samples a
                // slot's DMAs cover, nd the 16-byte DMAs per slot, cs = kRwStage; for
                // kFormDirect, L is the samples one wavefront load spans (the tile)
  int nch;      // kFormRegWin: 4-sample chunks per window (6, 8, 10 or 12)
};
Launch choose_launch(int32_t max_span, int nw, int nchan, int cs_req, int64_t lds_cap, int elem_bytes);
// FP32 input with nprod producer wavefronts issuing whole channels; nb = 0 if nothing fits.
Launch choose_launch_prod(int32_t max_span, int nchan, int cs_req, int64_t lds_cap, int nprod);

inline int64_t align_up(int64_t x, int64_t a = kAlign) { return (x + a - 1) / a * a; }

struct Tiles {
  int32_t g;   // DM trials per wavefront
  int32_t w;   // wavefronts per workgroup (each on its own G trials)
  int32_t s;   // output samples per lane (fixed: 8, two chunks of 4)
  int32_t cc;  // channels staged into LDS per barrier pair (0 = automatic)
  int32_t pw;  // producer wavefronts requested: -1 none, 0 automatic, 1 one
};

}  // namespace dd

struct dd_plan {
  int32_t nchan = 0, ndm = 0, dtype = DD_F32;
  double tsamp = 0.0;
  std::vector<double> freq, dm;
  std::vector<int32_t> delays;      // [nchan][ndm], Eq. deltaTEq
  int32_t maxdelay = 0;
  dd::Tiles tiles{};
  int32_t dms_per_group = 0;        // g * w
  int32_t ngroups = 0;
  int32_t ndm_pad = 0;              // ngroups * dms_per_group
  // device table: [nchan][ndm_pad] LDS byte offset of each trial's first chunk inside its
  // channel slot (padded trials repeat the last DM), then [ngroups][nchan] group first delays
  std::vector<int32_t> dev_table;
  int32_t max_span = 0;             // max over channels and groups of the in-group delay spread
  dd::Launch launch{};               // kernel geometry (fixed at plan time: the offsets depend on it)
  uint64_t id = 0;
};

struct dd_stream {
  const dd_plan* plan = nullptr;
  int64_t block = 0;        // largest block accepted
  int64_t ring_len = 0;     // R: samples per channel in the ring
  int64_t ring_row = 0;     // R + mirror: a channel row; [R, ring_row) repeats [0, ring_row - R)
  void* ring = nullptr;     // device: [table | ring data]
  int64_t received = 0;     // total samples appended
  int64_t next_seq = 0;
  int64_t emitted = 0;      // global output times already produced ([0, emitted))
  int64_t pending_t0 = 0, pending_n = 0;  // window appended but not yet dedispersed
  bool gap_fill = false;    // missing blocks become zeros instead of DD_ERR_SEQUENCE
};

namespace dd {

// Thread-local error message helpers (implemented in plan.cpp).
int fail(int code, const std::string& msg);
void clear_error();
// dd_plan_create with the LDS bytes one workgroup may take (csrc/plan.cpp); dd_plan_create
// passes kLdsBytes.
int plan_create(dd_plan** out, const double* freq_mhz, int32_t nchan, double tsamp_s, const double* dm,
                int32_t ndm, int32_t in_dtype, const dd_tuning* tuning, int64_t lds_cap);

// Workspace layout for one dd_dedisperse call.
struct WsLayout {
  int64_t table_off, table_bytes;
  int64_t part_off;    // double [ndm][ntile][2]: sum x, sum x^2 per 512-sample tile
  int64_t thr_off;     // double [ndm][3]: mean, rms, threshold
  int64_t cnt_off;     // int32 [ndm][nseg]
  int64_t offs_off;    // int64 [ndm][nseg]
  int64_t tail_off;    // 8-bit input: copy of the last tail_bytes of the input, then as many
  int64_t tail_bytes;  // bytes of padding (a window starting in the copy reads at most that far)
  int64_t quad_off;    // direct-read form, linear input: the four shifted copies of the input
  int64_t quad_bytes;
  int64_t nseg;        // candidate segments
  int64_t ntile;       // statistics segments
  int64_t total;
};
// Workspace of a call on n samples: linear input (dd_dedisperse) or a stream push of at
// most n samples (no region for the direct-read form's copies, which the ring holds).
WsLayout workspace_layout(const dd_plan* p, int64_t n, bool linear = true);
int64_t ring_table_bytes(const dd_plan* p);
// Samples after a ring row's R that mirror its start, so no channel window the kernel
// reads (at most launch.L + 3 samples from any start in [0, R)) wraps.
inline int64_t ring_mirror(const dd_plan* p) { return (int64_t)p->launch.L + 64; }
inline int64_t ring_len_for(const dd_plan* p, int64_t block) { return align_up(block + (int64_t)p->maxdelay, 64); }
// Rows a stream's ring keeps per channel: the direct-read form keeps its four shifted copies.
inline int64_t ring_copies(const dd_plan* p) { return p->launch.form == kFormDirect ? 4 : 1; }
int64_t elem_bytes(int32_t dtype);
// kFormRegWin device table: [ngroups][nchan] group first delays, then from this int32
// offset [ngroups][nchan][8 wavefronts] int4 {window byte offset, trial indices 0-3, 4-7, 0},
// followed by kRwStage - 1 channels of zero records.
bool plan_regwin(dd_plan* p, int64_t lds_cap);
inline int64_t rw_meta_offset(const dd_plan* p) { return ((int64_t)p->ngroups * p->nchan + 3) / 4 * 4; }
// Input view: linear rows, or a per-channel ring of ring_len samples in which
// window position p lives at (win0 + p) mod ring_len. A ring row continues past
// ring_len with a mirror of its start, so a window read from any start in
// [0, ring_len) is contiguous.
struct InView {
  const void* ptr;
  int64_t row_stride;  // elements between channel rows (ring: ring_len + mirror)
  int64_t nvalid;      // window positions [0, nvalid) hold data
  int64_t ring_len;    // 0 for linear input
  int64_t win0;        // ring only: global sample of window position 0
};
// Launch of the register-window kernel for nout outputs (statistics partials into part
// when non-null); defined with the kernel.
int launch_regwin(const dd_plan* p, const InView& in, const int32_t* d_table, int64_t nout, float* out,
                  int64_t out_stride, double* part, void* stream);
// Direct-read form (8-bit input): device table [nchan][ndm_pad] of plain delays (padded trials
// repeat the last DM). Fills the plan's tiles, groups, launch and table.
int plan_direct(dd_plan* p, const Tiles& t);
// Bytes per copy row of the direct-read form's copies of an nsamp-sample linear input: the
// last tile's windows (two sub-tiles at most) read at most 2 kDirectTile bytes past the
// last sample's position.
inline int64_t direct_quad_row(int64_t nsamp) { return align_up(nsamp + 2 * kDirectTile + 64, 64); }
// Linear input: writes the copies into quad_ws first. Ring input: in.ptr is the ring's
// copies, in.row_stride their row length.
int launch_direct(const dd_plan* p, const InView& in, const int32_t* d_table, int64_t nout, float* out,
                  int64_t out_stride, double* part, void* quad_ws, void* stream);
// One item of a batched direct-read launch (what launch_direct takes).
struct DirectItem {
  const dd_plan* plan;
  InView in;
  const int32_t* table;
  int64_t nout;
  float* out;
  int64_t out_stride;
  double* part;
  void* quad_ws;
};
// Bytes of device descriptors a batched direct-read launch of n items uploads.
int64_t direct_batch_desc_bytes(int32_t n);
int launch_direct_batch(const std::vector<DirectItem>& items, void* d_desc, int64_t desc_bytes, void* stream);
// n samples of a block (zeros when blk is null) into a direct-read stream ring of copy rows
// of lq bytes, starting at ring position pos0.
int append_direct(const dd_plan* p, const void* blk, int64_t in_stride, int64_t n, void* ring, int64_t lq,
                  int64_t ring_len, int64_t pos0, void* stream);
// Exclusive scan of n int32 counts into offs[n] (int64) and their total into *total, by
// many blocks in three launches that use no memory beyond offs (csrc/dedisp.hip).
int launch_count_scan(const int32_t* cnt, int64_t n, int64_t* offs, int64_t* total, void* stream);

}  // namespace dd
