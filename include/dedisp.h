/*
 * dedisp.h - C ABI of the MI355X brute-force dedispersion library (libdedisp.so).
 *
 * What it computes (Magro 2013, "A Real-Time, GPU-Based, Non-Imaging Back-End
 * for Radio Telescopes", Ch. 2 Sec. "Direct Dedispersion" and Ch. 3):
 *
 *   delays   Delta_t(d, c) = round(k_DM * DM(d) * (f_c^-2 - f_ref^-2) / t_samp),
 *            Eq. deltaTEq with the delay law of Eq. dispRelationshipEquation,
 *            k_DM = 4.15e3 s MHz^2 pc^-1 cm^3, f in MHz, f_ref = max_c f_c,
 *            evaluated in IEEE double on the host, rounded half away from zero.
 *   output   D[d][t] = sum_c A[c][t + Delta_t(d, c)], Eq. bruteEquation, for
 *            t in [0, nout), nout = nsamp - maxdelay, maxdelay = max Delta_t
 *            (the "maxshift" of Ch. 3 Sec. "Dedispersion").
 *   stats    mean_d and rms_d (population standard deviation) of each series,
 *            the normalisation of Ch. 3 Sec. "Signal Post-processing".
 *   cands    every (d, t) with D[d][t] > mean_d + k * rms_d, Ch. 3 Sec.
 *            "Detection and Candidate Selection", in ascending (d, t) order.
 *
 * Summation order (fixed, independent of tiling and of batching): channels are
 * summed in FP32 in order inside consecutive blocks of DD_CHAN_BLOCK channels
 * (c = 0..31, 32..63, ...); the block sums are added to the running series in
 * block order. u8 inputs are summed as raw codes in 32-bit integers (exact; the
output is that integer as FP32, exact below 2^24).
 *
 * Layouts: the filterbank is channel-major, time fastest ([nchan][row_stride],
 * Ch. 3 Sec. "Dedispersion" stores data after the transpose); the output is
 * DM-major ([ndm][out_row_stride]); delay tables are [nchan][ndm], DM fastest.
 *
 * Memory: every device pointer is owned by the caller. The library never
 * allocates device memory; it asks for a workspace size and uses the caller's
 * buffer. Host arrays passed in are copied; the caller keeps ownership.
 *
 * Errors: every call returns a status (0 ok, > 0 informational, < 0 error).
 * dd_last_error() gives the calling thread's message for the last failure. No
 * C++ exception crosses this boundary. Work is enqueued on the given HIP stream
 * (a hipStream_t passed as void*, NULL = the null stream) and the call returns
 * before the GPU finishes; faults inside a kernel surface at the caller's next
 * synchronisation.
 */
#ifndef DEDISP_H
#define DEDISP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DD_VERSION_MAJOR 1
#define DD_VERSION_MINOR 5  /* 1: dd_tuning.producer_waves, dd_plan_info.producer_waves;
                               2: dd_time_binning, dd_downfactor, dd_bandpass,
                                  dd_bandpass_fit, dd_rfi_clip;
                               3: dd_tuning.kernel_form, dd_plan_info.kernel_form and
                                  window_chunks (the register-window kernel form);
                                  dd_bandpass window means; dd_rfi_clip bandpass
                                  subtraction (subtract_bandpass) from the window means;
                                  DD_WARN_CAND_OVERFLOW, dd_candidates_check,
                                  dd_stream_set_gap_fill;
                               4: DD_FORM_DIRECT, dd_plan_info.stream_workspace_bytes,
                                  dd_boxcar_search, dd_binned_*, dd_subband_*;
                               5: dd_binned_stream_*, dd_bandpass_u8, dd_rfi_clip_u8 */
#define DD_CHAN_BLOCK 32

/* Status codes. */
enum {
  DD_OK = 0,
  DD_FILLING = 1,            /* stream push accepted, no output yet (ring still filling) */
  DD_WARN_CAND_OVERFLOW = 2, /* dd_candidates_check: more candidates qualified than cand_cap */
  DD_ERR_INVALID_ARG = -1,   /* a pointer, size or value is out of range */
  DD_ERR_TOO_SHORT = -2,     /* nsamp <= maxdelay: no output sample can be formed */
  DD_ERR_SEQUENCE = -3,      /* stream push out of order (seq must grow by one) */
  DD_ERR_WORKSPACE = -4,     /* workspace (or ring) smaller than dd_plan_query asks for */
  DD_ERR_HIP = -5,           /* a HIP runtime call failed (message in dd_last_error) */
  DD_ERR_UNSUPPORTED = -6    /* a tuning or shape the kernels cannot take */
};

/* Input storage types. All accumulate in FP32. */
enum { DD_F32 = 0, DD_F16 = 1, DD_U8 = 2 };

/* Kernel forms of the dedispersion step (dd_tuning.kernel_form). All compute the same
   sums in the same order (for 8-bit input the sums are exact integers), so their series
   are identical bit for bit; their statistics partials may group the FP64 additions
   differently (last-bit differences in mean/rms for FP32 and FP16 input). */
enum {
  DD_FORM_AUTO = 0,
  DD_FORM_LDS = 1,     /* each channel staged in LDS as four copies shifted by 0..3 samples;
                          every add reads its sample from LDS (all dtypes, any delay spread) */
  DD_FORM_REGWIN = 2,  /* FP32 only: each channel staged once; each lane loads a window of up
                          to 48 samples into registers and the 8 DM trials of its wavefront
                          add from it at their (wave-uniform) offsets. Needs the delay spread
                          of 8 consecutive trials plus 7 to stay within 40 samples in every
                          channel; groups of 64 trials, tuning fields other than the form
                          are ignored */
  DD_FORM_DIRECT = 3   /* 8-bit input only: nothing staged in LDS; the input is held as four
                          copies shifted by 0..3 samples (in the workspace for dd_dedisperse,
                          in the ring for streams: 4x the bytes of one copy), and per channel
                          each wavefront reads its trials' 1024-byte windows straight through
                          the L1/L2 caches (16 bytes per lane per trial, 4-byte aligned) and
                          sums them as exact integers. Suits beams whose delays grow by many
                          samples per trial (low frequencies, wide bands), where an LDS window
                          is shared by few trials. dms_per_wave 1, 2 or 4 (default 2), waves
                          1..8 (default 4), samples_per_lane 16; chan_stage and
                          producer_waves are ignored. Batched items of this form run in one
                          launch per tile shape and wavefront count, beside the LDS-form
                          items' launches */
};

typedef struct dd_plan dd_plan;
typedef struct dd_stream dd_stream;

/* Optional tile choice; zero fields take the library default. */
typedef struct dd_tuning {
  int32_t dms_per_wave;       /* DM trials each wavefront accumulates: 8, or 4 (FP32 input with
                                 producer wavefronts: up to 14 computing wavefronts in a
                                 1024-thread workgroup); 0 with waves 0: automatic (4 for FP32
                                 input when one DM group's windows fit the producers' DMAs,
                                 else 8) */
  int32_t waves;              /* computing wavefronts per workgroup, each on its own DMs
                                 (1..8, at most 8 - producer_waves; with 4 trials per
                                 wavefront 1..14, at most 16 - producer_waves) */
  int32_t samples_per_lane;   /* output samples per lane: 8 (the tile is 512 samples) */
  int32_t chan_stage;         /* channels per LDS stage (0..8; without a producer rounded
                                 down to a divisor of waves; 0 = automatic) */
  int32_t producer_waves;     /* wavefronts that only move input into LDS, FP32 input only:
                                 0 automatic (two for FP32 input when one DM group's channel
                                 windows fit 1024 words and waves allows, else none), -1 none
                                 (every wavefront issues its share of the DMAs), 1..4
                                 (waves + producer_waves <= 8; DD_ERR_UNSUPPORTED when the
                                 windows do not fit) */
  int32_t kernel_form;        /* DD_FORM_AUTO (the direct-read form for 8-bit input when no
                                 LDS-form tile field is set, else the LDS form), DD_FORM_LDS,
                                 DD_FORM_REGWIN (DD_ERR_UNSUPPORTED for
                                 other dtypes or a spread that does not fit) or DD_FORM_DIRECT
                                 (DD_ERR_UNSUPPORTED for other than 8-bit input) */
} dd_tuning;

typedef struct dd_plan_info {
  int32_t nchan, ndm, in_dtype, maxdelay;
  int64_t nsamp, nout;              /* for the queried nsamp */
  int64_t workspace_bytes;          /* for dd_dedisperse at this nsamp */
  int64_t ring_bytes;               /* for dd_stream_create with block_nsamp = nsamp */
  int32_t dms_per_wave, waves, samples_per_lane, max_span;  /* chosen tiles; LDS span */
  int64_t adds;                     /* ndm * nchan * nout: the algorithmic work */
  int32_t chan_stage;               /* channels per LDS stage requested (0 = automatic) */
  int32_t producer_waves;           /* chosen: wavefronts that only issue the LDS DMAs */
  /* launch geometry (fixed at plan creation for 160 KB of LDS per workgroup): shifted
     copies of each channel vector, samples per copy (32-bit words for 16/32-bit input,
     bytes for 8-bit input), channels per stage, stages in the LDS ring, LDS bytes per
     workgroup */
  int32_t launch_copies, launch_buf, launch_stage, launch_ring;
  int64_t launch_lds;
  int32_t kernel_form;              /* DD_FORM_LDS, DD_FORM_REGWIN or DD_FORM_DIRECT */
  int32_t window_chunks;            /* DD_FORM_REGWIN: 4-sample chunks per register window */
  int64_t stream_workspace_bytes;   /* for dd_stream_push on a stream of block_nsamp = nsamp
                                       (at most workspace_bytes: the direct-read form's copies
                                       of a plain call's input live in a stream's ring) */
} dd_plan_info;

/* One detection: (time, DM, intensity) of Ch. 3, plus (value - mean) / rms. */
typedef struct dd_cand {
  int32_t dm_index;
  int32_t reserved;
  int64_t t;          /* output sample (stream pushes: global output time) */
  float value;
  float snr;
} dd_cand;

/*
 * Build a plan (host only). freq_mhz[nchan] in any order (f_ref = the largest),
 * dm[ndm] >= 0 in non-decreasing order, tsamp_s > 0, in_dtype one of DD_F32/DD_F16/DD_U8, tuning may
 * be NULL. Computes the FP64 delay table (Eq. deltaTEq). Errors:
 * DD_ERR_INVALID_ARG for nchan < 1, ndm < 1, non-finite or non-positive
 * frequencies, tsamp <= 0, negative, non-finite or decreasing DMs, a delay above 2^31 - 1,
 * or an unknown dtype; DD_ERR_UNSUPPORTED for a tuning outside the listed
 * values, or when no launch geometry fits one DM group's delay spread in LDS. The plan
 * is immutable and may be shared between threads.
 */
int dd_plan_create(dd_plan** out, const double* freq_mhz, int32_t nchan, double tsamp_s,
                   const double* dm, int32_t ndm, int32_t in_dtype, const dd_tuning* tuning);

/* Free a plan (host memory only). NULL is a no-op. */
void dd_plan_destroy(dd_plan* plan);

/*
 * Sizes for a given nsamp: nout, workspace bytes, ring bytes, tiles.
 * DD_ERR_TOO_SHORT if nsamp <= maxdelay (info is still filled with maxdelay).
 */
int dd_plan_query(const dd_plan* plan, int64_t nsamp, dd_plan_info* info);

/* Copy the delay table, [nchan][ndm] int32 DM fastest, into host_out. */
int dd_plan_delays(const dd_plan* plan, int32_t* host_out);

/*
 * Prepare a workspace of ws_bytes (>= dd_plan_query's workspace_bytes) on the
 * current device: uploads this plan's delay table into it on the stream. The
 * workspace then belongs to this plan until the caller reuses the memory;
 * dd_dedisperse reads the table from it without checking its contents.
 */
int dd_plan_upload(const dd_plan* plan, void* d_workspace, int64_t ws_bytes, void* stream);

/*
 * Dedisperse one buffer (Eq. bruteEquation) and, optionally, reduce the series.
 *   d_in        [nchan][in_row_stride] elements of the plan's dtype, nsamp valid
 *   d_out       [ndm][out_row_stride] float, nout = nsamp - maxdelay written per row
 *   d_mean/d_rms  [ndm] float each, or both NULL to skip statistics and candidates
 *   k_sigma     threshold in units of rms; <= 0 (or d_ncand NULL) skips candidates
 *   d_cand      cand_cap entries; d_ncand (device int64) receives the total count.
 *               If the count exceeds cand_cap only the first cand_cap (in (d, t)
 *               order) are written, *d_ncand keeps the true count, and the next
 *               synchronising call, dd_candidates_check, returns DD_WARN_CAND_OVERFLOW.
 *   d_workspace prepared by dd_plan_upload, ws_bytes at least the queried size
 * Strides are in elements; in_row_stride >= nsamp, out_row_stride >= nout.
 */
int dd_dedisperse(const dd_plan* plan, const void* d_in, int64_t nsamp, int64_t in_row_stride,
                  float* d_out, int64_t out_row_stride, float* d_mean, float* d_rms,
                  float k_sigma, dd_cand* d_cand, int64_t cand_cap, int64_t* d_ncand,
                  void* d_workspace, int64_t ws_bytes, void* stream);

/*
 * dd_dedisperse for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same computation,
 * arguments and errors, with the delay table passed in (d_table: a buffer prepared once by
 * dd_plan_upload, read only) and the rest of the workspace (statistics partials,
 * thresholds, candidate counts and offsets, the u8 input-tail copy) taken from a static
 * device array of 96 MiB inside the library. The call makes no hipMalloc, hipFree or other
 * allocation. Each device the library runs on holds its own copy of the array until the
 * process ends; every call on a device shares it, so calls that overlap on one device
 * (on one stream or several) race and must not be issued. Nothing in the array needs to
 * start at zero. DD_ERR_UNSUPPORTED when the shape needs more scratch than the array holds
 * (the full 1024-channel, 2^20-sample, 2048-trial FP32 workload needs 67 MiB).
 */
int dd_dedisperse_noalloc(const dd_plan* plan, const void* d_in, int64_t nsamp, int64_t in_row_stride,
                          float* d_out, int64_t out_row_stride, float* d_mean, float* d_rms, float k_sigma,
                          dd_cand* d_cand, int64_t cand_cap, int64_t* d_ncand, const void* d_table, void* stream);

/*
 * Streaming (Ch. 3 Sec. "Dedispersion": the last maxshift spectra of a buffer are
 * carried into the next). A stream keeps a per-channel device ring of the last
 * maxdelay + block_nsamp samples (rounded up to 64), each row followed by a mirror of
 * its first launch_buf + 64 samples so that no channel window wraps, in the caller's
 * d_ring (ring_bytes >= dd_plan_query(plan, block_nsamp).ring_bytes). The ring also
 * holds the delay table, uploaded at creation on the given stream.
 */
int dd_stream_create(const dd_plan* plan, int64_t block_nsamp, void* d_ring, int64_t ring_bytes,
                     void* stream, dd_stream** out);

/*
 * Append one block (seq = 0, 1, 2, ... in order; nsamp <= block_nsamp samples in
 * [nchan][in_row_stride]) and dedisperse every output that became computable:
 * global output times [*t0_out, *t0_out + *nout_out), written to d_out rows from
 * column 0. Statistics and candidates cover those outputs only; candidate t is the
 * global output time. Returns DD_FILLING (nothing written) while the stream holds
 * fewer than maxdelay + 1 samples, DD_ERR_SEQUENCE for a wrong seq (nothing
 * changes). d_out needs at least block_nsamp columns. Not thread-safe per stream.
 */
int dd_stream_push(dd_stream* s, const void* d_block, int64_t nsamp, int64_t in_row_stride,
                   int64_t seq, float* d_out, int64_t out_row_stride, float* d_mean, float* d_rms,
                   float k_sigma, dd_cand* d_cand, int64_t cand_cap, int64_t* d_ncand,
                   void* d_workspace, int64_t ws_bytes, void* stream,
                   int64_t* t0_out, int64_t* nout_out);

/* Free a stream's host state (the ring is the caller's). NULL is a no-op. */
void dd_stream_destroy(dd_stream* s);

/*
 * Sequence gaps (Ch. 4 Sec. "Packet Receiver": lost packets leave zero-filled gaps that RFI
 * clipping then absorbs). With enable != 0, a push or append whose seq is larger than the
 * next expected one treats the missing blocks as block_nsamp samples of value 0 each: the
 * ring receives the zeros (only the last ring length of them is written) and the stream
 * time advances past them. Outputs made computable by the zero span alone are not
 * dedispersed: the window of that push is the last block_nsamp of the computable outputs,
 * so *t0_out jumps over the gap. A seq below the expected one is DD_ERR_SEQUENCE either way.
 * Default off (any gap is DD_ERR_SEQUENCE). Host only.
 */
int dd_stream_set_gap_fill(dd_stream* s, int32_t enable);

/*
 * Synchronise `stream` and read a candidate count written by dd_dedisperse, dd_stream_push
 * or dd_batch_dedisperse (d_ncand, device int64): *ncand_out (may be NULL) receives it.
 * Returns DD_WARN_CAND_OVERFLOW when it exceeds cand_cap (only the first cand_cap
 * candidates, in (d, t) order, were written), else DD_OK; DD_ERR_INVALID_ARG for a NULL
 * count; DD_ERR_HIP if the copy or the synchronisation fails (a fault of earlier work on
 * the stream surfaces here).
 */
int dd_candidates_check(const int64_t* d_ncand, int64_t cand_cap, void* stream, int64_t* ncand_out);

/*
 * Batched launch (uneven beams in few persistent launches). Each item names a plan, an
 * input already resident on the device, and its outputs; or a stream whose block has
 * already been appended with dd_stream_append. Items on the same kernel and workgroup shape
 * (LDS form: input dtype, computing and producer wavefronts, DM trials per wavefront;
 * direct-read form: DM trials per wavefront, samples per lane, wavefronts) run in one
 * launch that walks a device queue of (item, DM group, time tile) work, one launch per
 * distinct shape, each item on its own plan's tiles (an item of many units takes its plain
 * launch instead); then the statistics and candidates of all items take one launch per
 * step. The results equal those of one dd_dedisperse per
 * item, bit for bit. Register-window plans are refused (DD_ERR_UNSUPPORTED).
 */
typedef struct dd_batch_item {
  const dd_plan* plan;
  const void* d_in;            /* [nchan][in_row_stride]; ignored for stream items */
  int64_t nsamp, in_row_stride;
  float* d_out;
  int64_t out_row_stride;
  float* d_mean;
  float* d_rms;
  float k_sigma;
  int32_t reserved;
  dd_cand* d_cand;
  int64_t cand_cap;
  int64_t* d_ncand;
  void* d_plan_workspace;      /* prepared by dd_plan_upload for this item's plan */
  dd_stream* stream_item;      /* non-NULL: dedisperse this stream's pending window */
} dd_batch_item;

/* Workspace bytes the batch needs beyond the per-item plan workspaces. Each item's
   d_plan_workspace must be its own: items whose workspaces overlap are rejected with
   DD_ERR_INVALID_ARG (the statistics partials, candidate counts and u8 input-tail copy of
   one item would overwrite another's). For the same reason one workspace (or stream ring)
   must not serve two calls in flight at once, on one HIP stream or several. */
int dd_batch_query(const dd_batch_item* items, int32_t n, int64_t* ws_bytes);

int dd_batch_dedisperse(const dd_batch_item* items, int32_t n, void* d_workspace, int64_t ws_bytes,
                        void* stream);

/* Copy a block into a stream's ring without dedispersing (the batched path's first half). */
int dd_stream_append(dd_stream* s, const void* d_block, int64_t nsamp, int64_t in_row_stride,
                     int64_t seq, void* stream, int64_t* t0_out, int64_t* nout_out);

/*
 * Detrending and normalisation of dedispersed series, Ch. 3 Sec. "Signal
 * Post-processing": each of the nrows series in d_series ([nrows][row_stride] FP32,
 * device, caller-owned; the first n samples of a row are the series) loses its
 * least-squares line a + b*t over t = 0..n-1, in place. With normalise != 0 the residual
 * is then divided by its population standard deviation (a zero deviation leaves the zero
 * residual). d_rms (device [nrows] FP32, may be NULL) receives each residual's standard
 * deviation (from FP64 sums of x, x^2 and t*x: sum (x - mean)^2 - b^2 sum (t - tbar)^2).
 * Sums are FP64 in a fixed order, so results depend on the input only; one sample gives
 * a zero residual. Enqueued on `stream`. Errors: DD_ERR_INVALID_ARG for a
 * NULL series, nrows < 1, n < 1 or row_stride < n.
 */
int dd_detrend(float* d_series, int64_t nrows, int64_t n, int64_t row_stride, int32_t normalise,
               float* d_rms, void* stream);

/*
 * Boxcar levels of series, by successive addition of adjacent samples (Ch. 2 single-pulse
 * detection: the series is smoothed by adding groups of adjacent samples; Ch. 6: boxcar
 * templates downfactor the series). For k = 0..levels (levels <= 6: boxcars of 1..64
 * samples), level k of row r is s_k[j] = (x[j 2^k] + ... + x[j 2^k + 2^k - 1]) / sqrt(2^k)
 * for j < floor(n / 2^k), summed pairwise in FP32; a normalised series (dd_detrend) keeps
 * unit variance on every level. d_series: [nrows][row_stride] FP32 (first n samples);
 * d_out: [nrows][out_row_stride] FP32, levels one after another, level k at offset
 * sum_{i<k} floor(n / 2^i); out_row_stride must hold all levels. Both device,
 * caller-owned; enqueued on `stream`. Errors: DD_ERR_INVALID_ARG for NULL pointers,
 * nrows < 1, n < 1, row_stride < n, levels outside 0..6 or a short output row;
 * DD_ERR_UNSUPPORTED for more than 65535 rows.
 */
int dd_boxcar(const float* d_series, int64_t nrows, int64_t n, int64_t row_stride, int32_t levels,
              float* d_out, int64_t out_row_stride, void* stream);

/* One boxcar detection: row, start sample t, width (samples), boxcar sum, S/N. */
typedef struct dd_pulse {
  int32_t row;
  int32_t width;
  int64_t t;
  float value;
  float snr;
} dd_pulse;

/*
 * Boxcar template matching with thresholding (Ch. 6 Sec. "Transient Surveys": boxcar
 * templates of varying width convolved with each dedispersed series, then thresholded;
 * Ch. 2 Eq. pulseSNREquation: a matched boxcar's S/N grows as sqrt(width)). For widths
 * w = 2^j, j = 0 .. max_log2 (<= 6: 1..64 samples), at every start t of a row with
 * t + w <= n:
 *   B_w[t] = x[t] + ... + x[t + w - 1]            (FP32, pairwise: B_2w[t] = B_w[t] + B_w[t + w])
 *   S/N_w[t] = (B_w[t] - w mean) / (rms sqrt(w))  (FP32: w mean is exact, so the difference
 *                                                  is rounded once; 1 / (rms sqrt(w)) is formed
 *                                                  in FP64 and rounded once)
 * A detection at (row, t) when the largest S/N_w[t] over the widths defined there exceeds
 * k_sigma (the smallest width on ties); it is written as {row, w, t, B_w[t], S/N} in
 * ascending (row, t) order. Rows with rms <= 0 have no detections.
 * d_series: [nrows][row_stride] FP32 on the device (any [rows][n] array, e.g. the output
 * of dd_dedisperse); d_mean, d_rms: [nrows] FP32 (dd_dedisperse's statistics), or both
 * NULL for normalised rows (mean 0, rms 1, e.g. after dd_detrend with normalise).
 * d_pulse[cap] receives the detections; *d_npulse (device int64) their true count, which
 * may exceed cap (dd_candidates_check reads it and reports DD_WARN_CAND_OVERFLOW).
 * d_workspace: at least dd_boxcar_search_workspace bytes of device memory. Every buffer is
 * caller-owned; enqueued on `stream`, returns without waiting. The series is read twice
 * (a counting pass and a writing pass).
 * Errors: DD_ERR_INVALID_ARG for NULL series, count or workspace, nrows or n < 1,
 * row_stride < n, only one of d_mean/d_rms, max_log2 outside 0..6, non-finite k_sigma,
 * cap < 0 or cap > 0 with NULL d_pulse; DD_ERR_WORKSPACE for a short workspace;
 * DD_ERR_UNSUPPORTED for more than 65535 rows.
 */
int dd_boxcar_search_workspace(int64_t nrows, int64_t n, int64_t* ws_bytes);
int dd_boxcar_search(const float* d_series, int64_t nrows, int64_t n, int64_t row_stride, const float* d_mean,
                     const float* d_rms, int32_t max_log2, float k_sigma, dd_pulse* d_pulse, int64_t cap,
                     int64_t* d_npulse, void* d_workspace, int64_t ws_bytes, void* stream);

/*
 * Time binning above the diagonal DM (Ch. 2 Sec. "Direct Dedispersion": past the DM at
 * which the dispersion curve crosses one sample per channel, dedisperse at half the
 * sampling rate, again at twice that DM, and so on; Sec. "Computing Larger DMs" lists the
 * downfactor-then-dedisperse steps; Ch. 6 gives the same limit as dt f0^3 / (8300 df) and
 * counts ceil(log2(DM_max / DM_diag)) + 1 stages). Host only, no device memory.
 *   dm_diag = 1 / max over neighbouring channels a < b (frequency order) of
 *             (k_DM * (1/(a*a) - 1/(b*b))) / tsamp_s, each double operation rounded once;
 *             infinity for one channel. Written to *dm_diag_out when it is non-NULL.
 *   log2_out[d] = 0 for dm[d] <= dm_diag, else the smallest k <= max_log2 with
 *             dm[d] <= dm_diag * 2^k (max_log2 when none): trial d is dedispersed on the
 *             input downfactored k times (dd_downfactor) with a plan at sampling time
 *             2^k tsamp_s. DMs are non-decreasing, so each factor covers one run of trials.
 * freq_mhz[nchan], dm[ndm] and log2_out[ndm] are host arrays owned by the caller.
 * Errors: DD_ERR_INVALID_ARG for NULL arrays, nchan or ndm < 1, tsamp_s <= 0, non-finite
 * or non-positive frequencies, negative, non-finite or decreasing DMs, max_log2 outside
 * 0..16.
 */
int dd_time_binning(const double* freq_mhz, int32_t nchan, double tsamp_s, const double* dm, int32_t ndm,
                    int32_t max_log2, double* dm_diag_out, int32_t* log2_out);

/*
 * Downfactor a filterbank in time by 2 (Sec. "Computing Larger DMs": sum adjacent
 * samples): out[c][j] = A[c][2j] + A[c][2j+1] for j < floor(nsamp / 2), one FP32 add per
 * output after widening (u8 codes and FP16 values sum exactly; FP32 inputs give the
 * rounded FP32 sum). d_in: [nchan][in_row_stride] of in_dtype (DD_F32, DD_F16 or DD_U8),
 * nsamp valid per row; d_out: [nchan][out_row_stride] FP32, must not overlap d_in. Both
 * device, caller-owned; enqueued on `stream`. Repeating the call on its own output
 * gives the input downfactored 2^k times. Errors: DD_ERR_INVALID_ARG for NULL pointers,
 * an unknown dtype, nchan < 1, nsamp < 2, in_row_stride < nsamp or out_row_stride <
 * nsamp / 2; DD_ERR_UNSUPPORTED for more than 65535 channels.
 */
int dd_downfactor(const void* d_in, int32_t in_dtype, int64_t nchan, int64_t nsamp, int64_t in_row_stride,
                  float* d_out, int64_t out_row_stride, void* stream);

/*
 * Time-binned plan: brute-force dedispersion with time binning above the diagonal DM (Ch. 2
 * Sec. "Direct Dedispersion"; Sec. "Computing Larger DMs"). The trials are split into runs
 * by dd_time_binning; run k (trials whose factor is 2^k) is an ordinary plan at sampling
 * time 2^k tsamp_s over the input downfactored k times (dd_downfactor: FP32 sums; the
 * factor-1 run reads the input in in_dtype). A tuning of the 8-bit direct-read form
 * (DD_FORM_DIRECT) applies to the factor-1 run only; DD_FORM_LDS and DD_FORM_REGWIN to every
 * run; DD_FORM_AUTO with tile fields to every run except an 8-bit factor-1 run, which keeps
 * the direct-read form. Without a tuning each run takes the planner's choice for its own
 * trials.
 * Host object, immutable after creation; the caller keeps its arrays. Errors as
 * dd_time_binning and dd_plan_create.
 */
typedef struct dd_binned dd_binned;
typedef struct dd_binned_run {
  int32_t log2;        /* the run's factor is 2^log2 */
  int32_t d0, d1;      /* trials [d0, d1) */
  int32_t maxdelay;    /* in samples of the run (2^log2 tsamp_s) */
  int64_t nout;        /* (nsamp >> log2) - maxdelay for the queried nsamp */
  int32_t kernel_form, dms_per_wave, waves;
  int32_t producer_waves;  /* the run plan's producer wavefronts (LDS form; 0 otherwise) */
} dd_binned_run;
int dd_binned_create(dd_binned** out, const double* freq_mhz, int32_t nchan, double tsamp_s, const double* dm,
                     int32_t ndm, int32_t in_dtype, int32_t max_log2, const dd_tuning* tuning);
/* The runs (*nruns; up to runs_cap of them into runs[] when runs is non-NULL), the
   workspace an nsamp-sample call needs and the diagonal DM. DD_ERR_TOO_SHORT when some run
   would have no output (then *workspace_bytes is 0; the runs are still reported). */
int dd_binned_query(const dd_binned* b, int64_t nsamp, int32_t* nruns, dd_binned_run* runs, int32_t runs_cap,
                    int64_t* workspace_bytes, double* dm_diag);
/* Copies every run's delay table into a workspace for nsamp-sample calls. */
int dd_binned_upload(const dd_binned* b, int64_t nsamp, void* d_workspace, int64_t ws_bytes, void* stream);
/* One call over all runs. d_out: [ndm][out_row_stride] FP32; row d holds the nout of its
   run (samples at that run's sampling time), out_row_stride >= the largest run nout.
   d_mean/d_rms [ndm] as dd_dedisperse. Candidates of all runs form one list in ascending
   (trial, time) order: dm_index is the global trial, t the input sample where the binned
   sample starts (binned index << log2); *d_ncand the true count (as dd_dedisperse).
   batched != 0 runs the runs' dedispersion through one dd_batch_dedisperse call
   (DD_ERR_UNSUPPORTED when a run is in the register-window form); the results are the same
   bit for bit. Unbatched, each run runs on a side stream of its own as soon as its
   downfactored input exists, and `stream` waits for all of them. These side streams and
   their events (default priority) belong to the calling host thread and the current
   device, are created on first use and kept until the process ends. The workspace comes from dd_binned_upload for this
   nsamp. Errors as dd_dedisperse. */
int dd_binned_dedisperse(const dd_binned* b, const void* d_in, int64_t nsamp, int64_t in_row_stride, float* d_out,
                         int64_t out_row_stride, float* d_mean, float* d_rms, float k_sigma, dd_cand* d_cand,
                         int64_t cand_cap, int64_t* d_ncand, int32_t batched, void* d_workspace, int64_t ws_bytes,
                         void* stream);
void dd_binned_destroy(dd_binned* b);

/*
 * Streaming over a time-binned plan (Ch. 2 Sec. "Direct Dedispersion": time binning keeps
 * the long delays of low frequencies affordable; Ch. 3 Sec. "Dedispersion": the last
 * maxshift spectra of a buffer are carried into the next). Each run keeps its own stream
 * ring (as dd_stream_create) of the input downfactored 2^log2 times, so a run holds its
 * maxdelay at its own sampling time. block_nsamp and every pushed nsamp must be multiples of
 * 2^K, K the largest run log2: no pair of samples then straddles two blocks, and each run's
 * outputs equal those of dd_binned_dedisperse over the concatenated blocks, bit for bit.
 * dd_binned_stream_query gives the ring bytes (all runs' rings and delay tables, caller-owned
 * device memory) and the workspace one push needs; DD_ERR_INVALID_ARG for a block_nsamp that
 * is not a positive multiple of 2^K.
 */
typedef struct dd_binned_stream dd_binned_stream;
int dd_binned_stream_query(const dd_binned* b, int64_t block_nsamp, int64_t* ring_bytes, int64_t* workspace_bytes);
/* The binned plan must outlive the stream. Uploads every run's delay table into d_ring on
   `stream`. The object also creates, on the current device, one HIP stream (default
   priority) and one event per run, plus one more event: an unbatched push runs each run's
   dedispersion on its own stream, after the block's appends on the caller's stream, which
   then waits for all of them before the merged candidates. Use the object on the device
   it was created on; dd_binned_stream_destroy releases these as well. DD_ERR_HIP if they
   cannot be created. */
int dd_binned_stream_create(const dd_binned* b, int64_t block_nsamp, void* d_ring, int64_t ring_bytes, void* stream,
                            dd_binned_stream** out);
/*
 * Append one block (seq = 0, 1, 2, ...; nsamp <= block_nsamp samples in
 * [nchan][in_row_stride] of the plan's input dtype, nsamp a multiple of 2^K) and dedisperse
 * what became computable in each run: run i (in dd_binned_query order) writes outputs at
 * its own global output times [t0_out[i], t0_out[i] + nout_out[i]) (samples of that run's
 * sampling time) into d_out rows d0 .. d1-1 from column 0; nout_out[i] = 0 while that run
 * fills (its rows, mean and rms are then left alone). t0_out and nout_out hold one entry per
 * run and may be NULL. d_out needs block_nsamp columns. Statistics cover each run's window;
 * candidates of all runs with outputs form one list in (trial, time) order with dm_index
 * the global trial and t the input sample where the binned sample starts. Returns
 * DD_FILLING (nothing written, d_ncand untouched) while every run fills, DD_ERR_SEQUENCE
 * for a wrong seq (nothing changes), DD_ERR_UNSUPPORTED for batched != 0 when a run is in
 * the register-window form (as dd_binned_dedisperse). Not thread-safe per stream.
 */
int dd_binned_stream_push(dd_binned_stream* s, const void* d_block, int64_t nsamp, int64_t in_row_stride, int64_t seq,
                          float* d_out, int64_t out_row_stride, float* d_mean, float* d_rms, float k_sigma,
                          dd_cand* d_cand, int64_t cand_cap, int64_t* d_ncand, int32_t batched, void* d_workspace,
                          int64_t ws_bytes, void* stream, int64_t* t0_out, int64_t* nout_out);
/* Zero-filled sequence gaps on every run, as dd_stream_set_gap_fill. */
int dd_binned_stream_set_gap_fill(dd_binned_stream* s, int32_t enable);
/* Free the host state (the ring is the caller's). NULL is a no-op. */
void dd_binned_stream_destroy(dd_binned_stream* s);

/*
 * Subband plan: subband dedispersion (Ch. 2 Sec. "Subband Dedispersion"), an approximation of
 * Eq. bruteEquation. Trials are grouped in runs of dms_per_group; each group's nominal DM
 * is its middle trial. Step 1: each subband of chans_per_sub consecutive channels is
 * dedispersed at the nominal DMs (delays relative to the subband's highest frequency) into
 * a reduced filterbank [nsub][ngroups][width] in the workspace. Step 2: each group's trials
 * dedisperse its [nsub] rows of the reduced filterbank, the subbands standing at their
 * highest frequencies, over len1 = nsamp - (largest step-1 delay) samples (groups of up to 48
 * trials share a workgroup). FP32 input. Errors as dd_plan_create, and DD_ERR_INVALID_ARG
 * for chans_per_sub or dms_per_group < 1.
 */
typedef struct dd_subband dd_subband;
int dd_subband_create(dd_subband** out, const double* freq_mhz, int32_t nchan, double tsamp_s, const double* dm,
                      int32_t ndm, int32_t chans_per_sub, int32_t dms_per_group);
/* Workspace bytes for nsamp-sample calls, each trial's nout (nout_per_dm[ndm], optional,
   host), the channel-sample adds of both steps and the subband and group counts.
   DD_ERR_TOO_SHORT when a group would have no output. */
int dd_subband_query(const dd_subband* sp, int64_t nsamp, int64_t* workspace_bytes, int64_t* nout_per_dm,
                     int64_t* adds, int32_t* nsub, int32_t* ngroups);
int dd_subband_upload(const dd_subband* sp, int64_t nsamp, void* d_workspace, int64_t ws_bytes, void* stream);
/* One call over both steps; outputs and candidates as dd_binned_dedisperse (row d holds
   its group's nout; times in input samples). batched != 0 runs each step through one
   dd_batch_dedisperse call (same results bit for bit). Unbatched, the step-2 plans run on
   four side streams of the calling host thread (as dd_binned_dedisperse's) and `stream`
   waits for them. */
int dd_subband_dedisperse(const dd_subband* sp, const float* d_in, int64_t nsamp, int64_t in_row_stride, float* d_out,
                          int64_t out_row_stride, float* d_mean, float* d_rms, float k_sigma, dd_cand* d_cand,
                          int64_t cand_cap, int64_t* d_ncand, int32_t batched, void* d_workspace, int64_t ws_bytes,
                          void* stream);
void dd_subband_destroy(dd_subband* sp);

/*
 * RFI mitigation before dedispersion (Ch. 3 Sec. "Bandpass Correction", "Channel
 * Thresholding", "Spectrum Thresholding"), for FP32 filterbanks. A caller runs
 * dd_bandpass, copies the nchan averages to the host, fits them with dd_bandpass_fit,
 * uploads the fit and calls dd_rfi_clip.
 *
 * dd_bandpass: d_avg[c] = mean over t < nsamp of d_in[c][t] (the averaged bandpass), FP64
 * sums in a fixed order. With window >= 1 it also writes d_window_means[c][w], the mean of
 * samples [w window, (w + 1) window) (the last window may be shorter) for w <
 * ceil(nsamp / window): the channel stage's statistic, gathered in the same read of the
 * input (the channel total is then the sum of its window sums). d_in [nchan][row_stride]
 * FP32, d_avg [nchan] and d_window_means [nchan][ceil(nsamp/window)] FP64, all device.
 * Errors: DD_ERR_INVALID_ARG for NULL input or average, nchan or nsamp < 1, row_stride <
 * nsamp, or window and d_window_means not both given (window >= 1) or both absent (0).
 */
int dd_bandpass(const float* d_in, int64_t nchan, int64_t nsamp, int64_t row_stride, int64_t window, double* d_avg,
                double* d_window_means, void* stream);

/*
 * dd_bandpass_fit (host only): least-squares polynomial of degree `order` (0..16, below
 * nchan) in x = 2c/(nchan-1) - 1 (x = 0 for one channel) fitted to avg[nchan]; writes the
 * fitted values fit[nchan], and when non-NULL the RMSE between fit and avg (*rmse) and the
 * fit's mean over channels (*fit_mean). Host arrays, caller-owned. Errors:
 * DD_ERR_INVALID_ARG for NULL avg or fit, nchan < 1, or an order out of range.
 */
int dd_bandpass_fit(const double* avg, int32_t nchan, int32_t order, double* fit, double* rmse, double* fit_mean);

/*
 * dd_rfi_clip, in place on d_data [nchan][row_stride] FP32 (device), with d_fit [nchan]
 * FP64 (device) the fitted bandpass. The stages compare the uncorrected data with the fit:
 *   channel stage (chan_threshold > 0): window w of channel c (windows of `window` samples,
 *     the last may be shorter) is flagged when |d_window_means[c][w] - fit[c]| >
 *     chan_threshold (FP64), too high for RFI or too low for lost data; the means are
 *     dd_bandpass's for the same window. d_flags ([nchan][ceil(nsamp/window)] int32,
 *     device, caller-owned) receives the flags. Every sample of a flagged window or of a
 *     flagged window's neighbour takes the fitted value.
 *   spectrum stage (spec_threshold > 0), after the channel stage: a sample t whose mean
 *     over channels (FP64, in channel order) differs from fit_mean by more than
 *     spec_threshold takes the fitted value in every channel.
 *   bandpass correction (subtract_bandpass != 0, Ch. 3 Sec. "Bandpass Correction"): every
 *     sample becomes x - (float)fit[c] (one FP32 subtraction), so each channel's mean moves
 *     to about 0 and a replaced sample becomes exactly 0. Without it, replaced samples hold
 *     (float)fit[c] and the rest keep their values.
 * The channel replacement and the correction share one pass (a read and a write of the
 * filterbank); the spectrum stage reads it once more. With dd_bandpass that is three reads
 * of the input for the whole stage. Enqueued on `stream`. Errors: DD_ERR_INVALID_ARG for
 * NULL data or fit, nchan or nsamp < 1, row_stride < nsamp, or a channel stage without
 * window >= 1, window means and flags; DD_ERR_UNSUPPORTED for more than 65535 channels.
 */
int dd_rfi_clip(float* d_data, int64_t nchan, int64_t nsamp, int64_t row_stride, const double* d_fit,
                double chan_threshold, int64_t window, const double* d_window_means, int32_t* d_flags,
                double fit_mean, double spec_threshold, int32_t subtract_bandpass, void* stream);

/*
 * The same stage for 8-bit filterbanks (the codes of the serving beams). dd_bandpass_u8 is
 * dd_bandpass over d_in [nchan][row_stride] uint8: its sums are exact integers, so each
 * average and window mean is the exact sum divided once (FP64), in any summation order.
 * dd_rfi_clip_u8 is dd_rfi_clip on d_data [nchan][row_stride] uint8 in place, with the
 * replacement value of channel c the nearest code to fit[c] (halves away from zero),
 * clamped to 0..255, and the spectrum means exact sums over channels divided by nchan. It
 * makes no bandpass correction: an 8-bit sample cannot hold x - fit[c]. Subtracting a
 * per-channel constant from every sample lowers every dedispersed sample (Eq.
 * bruteEquation sums each channel once) by the same sum over channels of fit[c], which
 * moves each series' mean and leaves its RMS and its n-sigma candidates as they are; a
 * caller who wants the corrected values subtracts that constant from the outputs. Errors
 * as dd_bandpass and dd_rfi_clip.
 */
int dd_bandpass_u8(const uint8_t* d_in, int64_t nchan, int64_t nsamp, int64_t row_stride, int64_t window,
                   double* d_avg, double* d_window_means, void* stream);
int dd_rfi_clip_u8(uint8_t* d_data, int64_t nchan, int64_t nsamp, int64_t row_stride, const double* d_fit,
                   double chan_threshold, int64_t window, const double* d_window_means, int32_t* d_flags,
                   double fit_mean, double spec_threshold, void* stream);

/* Thread-local message for the last failing call on this thread ("" if none). */
const char* dd_last_error(void);

/* "major.minor" of the library. */
const char* dd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DEDISP_H */
