// Host side of the plan: validation, the FP64 delay table (Eq. deltaTEq), tile choice,
// workspace sizing. Built with -ffp-contract=off so each double operation rounds once.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "dd_internal.h"

namespace {

thread_local std::string g_err;
std::atomic<uint64_t> g_next_id{1};

// Approximate dispersion constant of Eq. dispRelationshipEquation (s MHz^2 pc^-1 cm^3).
constexpr double kDm = 4.15e3;

bool valid_tiles(const dd::Tiles& t) {
  auto in = [](int v, std::initializer_list<int> xs) {
    for (int x : xs) if (v == x) return true;
    return false;
  };
  // 8 trials per wavefront: at most 8 wavefronts (512 threads); 4 trials per wavefront (the
  // FP32 producer form only): at most 14 computing wavefronts, 16 with the producers
  const int maxw = t.g == 4 ? 16 : 8;
  return (t.g == 8 || t.g == 4) && t.w >= 0 && t.w <= (t.g == 4 ? 14 : 8) && t.s == 8 && t.cc >= 0 && t.cc <= 8 &&
         in(t.pw, {-1, 0, 1, 2, 3, 4}) && !(t.pw > 0 && t.w + t.pw > maxw);
}

// Largest in-group delay spread over all channels, for groups of gw trials with the last
// trial repeated as padding.
int32_t compute_span(const std::vector<int32_t>& delays, int32_t nchan, int32_t ndm, int gw) {
  const int ngroups = (ndm + gw - 1) / gw;
  int32_t span = 0;
  for (int32_t c = 0; c < nchan; ++c) {
    const int32_t* row = &delays[(size_t)c * ndm];
    for (int gi = 0; gi < ngroups; ++gi) {
      const int d0 = gi * gw, d1 = std::min(d0 + gw, (int)ndm) - 1;
      span = std::max(span, row[d1] - row[d0]);
    }
  }
  return span;
}

}  // namespace

namespace dd {

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
void clear_error() { g_err.clear(); }

int64_t elem_bytes(int32_t dtype) { return dtype == DD_F32 ? 4 : dtype == DD_F16 ? 2 : 1; }

WsLayout workspace_layout(const dd_plan* p, int64_t nout, bool linear) {
  WsLayout l{};
  l.table_off = 0;
  l.table_bytes = (int64_t)p->dev_table.size() * 4;
  l.nseg = nout > 0 ? (nout + kStatSeg - 1) / kStatSeg : 1;
  l.ntile = nout > 0 ? (nout + kTile - 1) / kTile : 1;
  int64_t o = align_up(l.table_bytes);
  l.part_off = o;
  o = align_up(o + (int64_t)p->ndm * l.ntile * 16);
  l.thr_off = o;
  o = align_up(o + (int64_t)p->ndm * 24);  // {mean, rms, threshold} per trial
  l.cnt_off = o;
  o = align_up(o + (int64_t)p->ndm * l.nseg * 4);
  l.offs_off = o;
  o = align_up(o + (int64_t)p->ndm * l.nseg * 8 + 8);
  l.tail_off = o;
  l.tail_bytes = p->dtype == DD_U8 && p->launch.form == kFormLds ? (int64_t)p->launch.L + 64 : 0;
  o = align_up(o + 2 * l.tail_bytes);
  l.quad_off = o;
  l.quad_bytes = linear && p->launch.form == kFormDirect ? 4 * (int64_t)p->nchan * direct_quad_row(nout) : 0;
  o = align_up(o + l.quad_bytes);
  l.total = o;
  return l;
}

int64_t ring_table_bytes(const dd_plan* p) { return align_up((int64_t)p->dev_table.size() * 4); }

// 8-bit input keeps its samples as bytes in LDS: four byte-shifted copies of L bytes
// (L a multiple of 256), filled by 1024-byte and 256-byte DMAs, plus 256 bytes of offsets.
Launch choose_launch_u8(int32_t max_span, int nw, int cs_req, int64_t lds_cap) {
  Launch best{};
  const int64_t L = (kTile + (int64_t)max_span + 255) / 256 * 256;
  const int64_t per_chan = 4 * L + 256;
  const int64_t nchunk = 4 * (L / 1024 + (L % 1024) / 256) + 1;
  const int cs_hi = cs_req > 0 ? std::min(cs_req, nw) : nw;
  int64_t best_score = -1;
  for (int cs = cs_hi; cs >= 1; --cs) {
    if (nw % cs) continue;
    const int wpc = nw / cs;
    const int64_t nd = (nchunk + wpc - 1) / wpc;
    if (nd > kMaxDma) continue;
    int nb = (int)std::min<int64_t>(lds_cap / (cs * per_chan), 16);
    while (nb > 2 && (int64_t)(nb - 2) * nd > 63) --nb;
    if (nb < 2) continue;
    if (cs_req > 0 && best_score >= 0) break;
    const int64_t score = (int64_t)std::min(nb * cs, 24) * 64 + cs;  // deep enough, then fewest barriers
    if (score > best_score) {
      best_score = score;
      best.L = (int)L;
      best.cs = cs;
      best.nb = nb;
      best.nd = (int)nd;
      best.x4 = 1;
    }
  }
  if (best_score < 0) return Launch{};
  best.lds = (int64_t)best.nb * best.cs * per_chan;
  best.ndw = best.nd;
  return best;
}

Launch choose_launch(int32_t max_span, int nw, int nchan, int cs_req, int64_t lds_cap, int elem_bytes) {
  if (elem_bytes == 1) return choose_launch_u8(max_span, nw, cs_req, lds_cap);
  Launch best{};
  (void)nchan;
  // words one channel copy covers: tile + group spread (lane reads end at k - m + 511)
  const int64_t L = (kTile + (int64_t)max_span + 63) / 64 * 64;  // whole 64-word DMA chunks
  // a channel's slot: four shifted copies plus the group's 64 trial offsets
  const int64_t per_chan = (4 * L + 64) * 4;
  const int64_t nchunk = 4 * (L / 64) + 1;
  const int cs_hi = cs_req > 0 ? std::min(cs_req, nw) : nw;
  int64_t best_score = -1;
  for (int cs = cs_hi; cs >= 1; --cs) {
    if (nw % cs) continue;  // each stage channel gets nw / cs whole wavefronts
    const int wpc = nw / cs;
    // FP32: 256-word chunks by 16-byte DMAs plus one offsets DMA; otherwise 64-word
    // chunks (the last one the offsets), split over the channel's wavefronts
    const int64_t njx = (L / 64 + wpc - 1) / wpc;
    const int x4 = elem_bytes == 4 && njx <= kMaxX4;
    const int64_t nd = x4 ? njx + 1 : (nchunk + wpc - 1) / wpc;
    if (nd > kMaxDma) continue;
    int nb = (int)std::min<int64_t>(lds_cap / (cs * per_chan), 16);
    // with later stages in flight the wait counts them (vmcnt <= 63); a two-stage ring
    // always waits for everything, so any DMA count is legal there
    while (nb > 2 && (int64_t)(nb - 2) * nd > 63) --nb;
    if (nb < 2) continue;
    if (cs_req > 0 && best_score >= 0) break;  // an explicit request takes the largest fitting divisor
    const int64_t score = (int64_t)nb * cs * 16 + cs;  // most channels in flight, then fewest barriers
    if (score > best_score) {
      best_score = score;
      best.L = (int)L;
      best.cs = cs;
      best.nb = nb;
      best.nd = (int)nd;
      best.x4 = x4;
    }
  }
  if (best_score < 0) return Launch{};
  best.lds = (int64_t)best.nb * best.cs * per_chan;
  best.ndw = best.nd;
  return best;
}

// FP32 input, one producer wavefront: it issues every channel of a stage whole (the four
// copies as L/64 16-byte DMAs, then the offsets), so any stage width works, and the
// computing wavefronts never wait on a DMA issue. A channel's copies must fit the 16
// per-lane descriptors (L <= 1024 words).
Launch choose_launch_prod(int32_t max_span, int nchan, int cs_req, int64_t lds_cap, int nprod) {
  Launch best{};
  const int64_t L = (kTile + (int64_t)max_span + 63) / 64 * 64;
  if (L / 64 > kMaxX4) return best;
  const int64_t per_chan = (4 * L + 64) * 4;
  const int nd = (int)(L / 64) + 1;
  // at least one channel per producer (stage channels past the last repeat it)
  const int cs_hi = cs_req > 0 ? cs_req : std::max(nprod, std::min(8, nchan));
  int64_t best_score = -1;
  for (int cs = cs_hi; cs >= 1; --cs) {
    if (cs % nprod) continue;  // each producer takes cs / nprod whole channels
    const int64_t ndw = (int64_t)(cs / nprod) * nd;
    int nb = (int)std::min<int64_t>(lds_cap / (cs * per_chan), 16);
    // every DMA of the nb - 1 stages ahead is in flight at once: a wavefront issues at
    // most 63 before it stalls (vmcnt), so the producer never waits to issue
    while (nb > 2 && (int64_t)(nb - 1) * ndw > 63) --nb;
    if (nb < 2 || ndw > 63) continue;
    if (cs_req > 0 && best_score >= 0) break;
    // the fewest barriers, then the deepest ring: the producers keep their DMAs ahead of
    // the computing wavefronts, so a double buffer of wide stages measured fastest
    const int64_t score = (int64_t)cs * 64 + nb;
    if (score > best_score) {
      best_score = score;
      best.L = (int)L;
      best.cs = cs;
      best.nb = nb;
      best.nd = nd;
      best.ndw = (int)ndw;
    }
  }
  if (best_score < 0) return Launch{};
  best.x4 = 1;
  best.prod = nprod;
  best.lds = (int64_t)best.nb * best.cs * per_chan;
  return best;
}

// Register-window form: groups of 64 trials (8 wavefronts of 8), one padded copy of each
// channel per LDS slot. Per (group, channel, wavefront) the table holds the window's LDS byte
// offset (a = the wavefront's first relative delay rounded down to 8: 12 words per 8
// samples, so 6a bytes) and the eight trials' register indices (relative delay - a), one
// byte each. Returns false when some window needs more than kRwMaxChunks chunks or the slots
// do not fit in LDS.
bool plan_regwin(dd_plan* p, int64_t lds_cap) {
  const int G = 8, NW = kRwTrials / 8;
  const int32_t nchan = p->nchan, ndm = p->ndm;
  const int ngroups = (ndm + kRwTrials - 1) / kRwTrials;
  std::vector<int32_t> tab;
  const int64_t moff = ((int64_t)ngroups * nchan + 3) / 4 * 4;
  // seven channels of zero records after the last group: a stage reads eight channels' records
  tab.assign((size_t)(moff + ((int64_t)ngroups * nchan + kRwStage - 1) * NW * 4), 0);
  int32_t max_idx = 0, max_a = 0, span = 0;
  for (int gi = 0; gi < ngroups; ++gi) {
    for (int32_t c = 0; c < nchan; ++c) {
      const int32_t* row = &p->delays[(size_t)c * ndm];
      auto dl = [&](int d) { return row[d < ndm ? d : ndm - 1]; };  // padded trials repeat the last DM
      const int32_t first = dl(gi * kRwTrials);
      tab[(size_t)gi * nchan + c] = first;
      span = std::max(span, dl(gi * kRwTrials + kRwTrials - 1) - first);
      for (int w = 0; w < NW; ++w) {
        const int d0 = gi * kRwTrials + G * w;
        const int32_t a = (dl(d0) - first) & ~7;
        uint32_t pk[2] = {0u, 0u};
        int32_t wmax = 0;
        for (int g = 0; g < G; ++g) {
          const int32_t idx = dl(d0 + g) - first - a;
          max_idx = std::max(max_idx, idx);
          wmax = std::max(wmax, idx);
          if (idx > 4 * kRwMaxChunks - 8) return false;
          pk[g / 4] |= (uint32_t)idx << (8 * (g % 4));
        }
        max_a = std::max(max_a, a);
        int32_t* m = &tab[(size_t)(moff + (((int64_t)gi * nchan + c) * NW + w) * 4)];
        m[0] = 6 * a;
        m[1] = (int32_t)pk[0];
        m[2] = (int32_t)pk[1];
        m[3] = (wmax + 8 + 3) / 4;  // chunks this wavefront's window needs in this channel
      }
    }
  }
  int nch = (max_idx + 8 + 3) / 4;
  nch = nch <= 6 ? 6 : nch <= 8 ? 8 : nch <= 10 ? 10 : 12;
  // samples the windows touch (lane 63 reads up to 8 * 63 + a + 4 nch - 1), and the 16-byte
  // DMAs that cover them: three 16-byte positions per 8 samples (two of data, one of padding)
  const int64_t need = 8 * 63 + (int64_t)max_a + 4 * nch;
  const int ndma = (int)((3 * ((need + 7) / 8) + 63) / 64);
  const int xs = 8 * ((64 * ndma - 1) / 3 + 1);
  const int64_t stage = (int64_t)kRwStage * 1024 * ndma;
  int nb = (int)std::min<int64_t>(lds_cap / stage, 8);
  while (nb > 2 && (int64_t)(nb - 2) * ndma > 63) --nb;  // a wait counts at most 63 DMAs
  if (nb < 2) return false;
  Launch l{};
  l.form = kFormRegWin;
  l.L = xs;
  l.cs = kRwStage;
  l.nb = nb;
  l.nd = ndma;
  l.ndw = ndma;
  l.x4 = 1;
  l.nch = nch;
  l.lds = (int64_t)nb * stage;
  p->launch = l;
  p->tiles = Tiles{G, NW, 8, kRwStage, -1};
  p->dms_per_group = kRwTrials;
  p->ngroups = ngroups;
  p->ndm_pad = ngroups * kRwTrials;
  p->max_span = span;
  p->dev_table.swap(tab);
  return true;
}

// Direct-read form: t.g trials per wavefront, t.w wavefronts per workgroup; the table is the
// plain delays per (channel, padded trial). A wavefront's loads span at most two 1024-sample
// sub-tiles, so a ring's mirror of launch.L + 64 samples covers every window that starts
// before the ring's end.
int plan_direct(dd_plan* p, const Tiles& t) {
  if (t.g != 1 && t.g != 2 && t.g != 4)
    return fail(DD_ERR_UNSUPPORTED, "the direct-read form takes dms_per_wave 1, 2 or 4");
  if (t.w < 1 || t.w > 8) return fail(DD_ERR_UNSUPPORTED, "the direct-read form takes waves 1..8");
  if (t.s != 16 && !(t.s == 32 && t.g <= 2))
    return fail(DD_ERR_UNSUPPORTED, "the direct-read form takes samples_per_lane 16, or 32 with dms_per_wave "
                                    "1 or 2");
  const int32_t nchan = p->nchan, ndm = p->ndm;
  p->tiles = Tiles{t.g, t.w, t.s, 0, -1};
  p->dms_per_group = t.g * t.w;
  p->ngroups = (ndm + p->dms_per_group - 1) / p->dms_per_group;
  p->ndm_pad = p->ngroups * p->dms_per_group;
  p->max_span = compute_span(p->delays, nchan, ndm, p->dms_per_group);
  Launch l{};
  l.form = kFormDirect;
  l.L = (int)(2 * kDirectTile);  // the widest wavefront tile (two sub-tiles)
  p->launch = l;
  p->dev_table.assign((size_t)nchan * p->ndm_pad, 0);
  for (int32_t c = 0; c < nchan; ++c) {
    const int32_t* row = &p->delays[(size_t)c * ndm];
    int32_t* drow = &p->dev_table[(size_t)c * p->ndm_pad];
    for (int32_t d = 0; d < p->ndm_pad; ++d) drow[d] = row[d < ndm ? d : ndm - 1];
  }
  return DD_OK;
}

}  // namespace dd

extern "C" {

const char* dd_last_error(void) { return g_err.c_str(); }

const char* dd_version(void) { return "1.5"; }

}  // extern "C"

namespace dd {

// dd_plan_create with the LDS bytes one workgroup may take (the ring and slots are sized
// within it; a smaller budget lets several workgroups share a CU).
int plan_create(dd_plan** out, const double* freq_mhz, int32_t nchan, double tsamp_s, const double* dm,
                int32_t ndm, int32_t in_dtype, const dd_tuning* tuning, int64_t lds_cap) {
  dd::clear_error();
  if (!out) return dd::fail(DD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!freq_mhz || !dm) return dd::fail(DD_ERR_INVALID_ARG, "freq_mhz and dm must be non-NULL");
  if (nchan < 1 || ndm < 1) return dd::fail(DD_ERR_INVALID_ARG, "nchan and ndm must be >= 1");
  if (!(tsamp_s > 0.0) || !std::isfinite(tsamp_s))
    return dd::fail(DD_ERR_INVALID_ARG, "tsamp must be finite and > 0");
  if (in_dtype != DD_F32 && in_dtype != DD_F16 && in_dtype != DD_U8)
    return dd::fail(DD_ERR_INVALID_ARG, "unknown input dtype");
  double fmax = 0.0;
  for (int32_t c = 0; c < nchan; ++c) {
    if (!std::isfinite(freq_mhz[c]) || !(freq_mhz[c] > 0.0))
      return dd::fail(DD_ERR_INVALID_ARG, "frequencies must be finite and > 0 (channel " +
                                              std::to_string(c) + ")");
    if (freq_mhz[c] > fmax) fmax = freq_mhz[c];
  }
  for (int32_t d = 0; d < ndm; ++d) {
    if (!std::isfinite(dm[d]) || dm[d] < 0.0)
      return dd::fail(DD_ERR_INVALID_ARG, "DMs must be finite and >= 0 (trial " + std::to_string(d) + ")");
    if (d > 0 && dm[d] < dm[d - 1])
      return dd::fail(DD_ERR_INVALID_ARG, "DM trials must be in non-decreasing order");
  }

  dd::Tiles t{8, 0, 8, 0, 0};
  const int form_req = tuning ? tuning->kernel_form : DD_FORM_AUTO;
  if (form_req != DD_FORM_AUTO && form_req != DD_FORM_LDS && form_req != DD_FORM_REGWIN &&
      form_req != DD_FORM_DIRECT)
    return dd::fail(DD_ERR_UNSUPPORTED, "unknown kernel_form");
  if (form_req == DD_FORM_REGWIN && in_dtype != DD_F32)
    return dd::fail(DD_ERR_UNSUPPORTED, "the register-window form takes FP32 input only");
  if (form_req == DD_FORM_DIRECT && in_dtype != DD_U8)
    return dd::fail(DD_ERR_UNSUPPORTED, "the direct-read form takes 8-bit input only");
  // the register-window form is the FP32 default when no tile field is set
  const bool tiles_set = tuning && (tuning->dms_per_wave || tuning->waves || tuning->samples_per_lane ||
                                    tuning->chan_stage || tuning->producer_waves);
  const bool try_regwin = in_dtype == DD_F32 && (form_req == DD_FORM_REGWIN ||
                                                 (form_req == DD_FORM_AUTO && !tiles_set && dd::kAutoRegWin));
  if (tuning) {
    if (tuning->dms_per_wave) t.g = tuning->dms_per_wave;
    if (tuning->waves) t.w = tuning->waves;
    if (tuning->samples_per_lane) t.s = tuning->samples_per_lane;
    t.cc = tuning->chan_stage;
    t.pw = tuning->producer_waves;
  }
  // 8-bit input takes the direct-read form unless the caller asks for another form or sets
  // an LDS-form tile field
  const bool direct = form_req == DD_FORM_DIRECT || (form_req == DD_FORM_AUTO && in_dtype == DD_U8 && !tiles_set);
  if (direct) {
    t.g = tuning && tuning->dms_per_wave ? tuning->dms_per_wave : 2;
    t.w = tuning && tuning->waves ? tuning->waves : 4;
    t.s = tuning && tuning->samples_per_lane ? tuning->samples_per_lane : 16;
  } else if (!valid_tiles(t)) {
    return dd::fail(DD_ERR_UNSUPPORTED, "unsupported tuning");
  }
  if (t.pw > 0 && in_dtype != DD_F32 && !direct)
    return dd::fail(DD_ERR_UNSUPPORTED, "producer wavefronts are available for FP32 input only");
  if (!direct && t.g == 4 && (in_dtype != DD_F32 || t.pw < 0))
    return dd::fail(DD_ERR_UNSUPPORTED, "4 DM trials per wavefront is the FP32 producer form only");

  dd_plan* p = new (std::nothrow) dd_plan();
  if (!p) return dd::fail(DD_ERR_INVALID_ARG, "out of host memory");
  p->nchan = nchan;
  p->ndm = ndm;
  p->dtype = in_dtype;
  p->tsamp = tsamp_s;
  p->freq.assign(freq_mhz, freq_mhz + nchan);
  p->dm.assign(dm, dm + ndm);
  p->delays.resize((size_t)nchan * ndm);

  // Eq. deltaTEq: x = ((k * DM) * (1/(f*f) - 1/(fr*fr))) / tsamp, round half away from zero.
  const double inv_ref = 1.0 / (fmax * fmax);
  int64_t maxd = 0;
  for (int32_t c = 0; c < nchan; ++c) {
    const double diff = 1.0 / (freq_mhz[c] * freq_mhz[c]) - inv_ref;
    for (int32_t d = 0; d < ndm; ++d) {
      const double x = ((kDm * dm[d]) * diff) / tsamp_s;
      const double fl = std::floor(x);
      const double r = fl + ((x - fl) >= 0.5 ? 1.0 : 0.0);
      if (!(r <= (double)std::numeric_limits<int32_t>::max())) {
        delete p;
        return dd::fail(DD_ERR_INVALID_ARG, "delay exceeds 2^31-1 samples");
      }
      const int32_t v = (int32_t)r;
      p->delays[(size_t)c * ndm + d] = v;
      if (v > maxd) maxd = v;
    }
  }
  p->maxdelay = (int32_t)maxd;

  if (direct) {
    const int rc = dd::plan_direct(p, t);
    if (rc) {
      delete p;
      return rc;
    }
    p->id = g_next_id.fetch_add(1);
    *out = p;
    return DD_OK;
  }
  if (try_regwin) {
    if (dd::plan_regwin(p, lds_cap)) {
      p->id = g_next_id.fetch_add(1);
      *out = p;
      return DD_OK;
    }
    if (form_req == DD_FORM_REGWIN) {
      delete p;
      return dd::fail(DD_ERR_UNSUPPORTED, "the delay spread of 8 consecutive DM trials does not fit the register "
                                          "window (at most 40 samples with the alignment)");
    }
  }
  // FP32 input: by default two producer wavefronts issue every LDS DMA beside the computing
  // ones, when one DM group's channel windows fit their 16-byte DMAs. Otherwise, and for
  // other input: 8 DM trials per wavefront, as many wavefronts as keep the LDS ring at least
  // 8 channels deep (unless the caller fixed the count).
  // With trials per wavefront and wavefronts left open, FP32 input first tries 4 trials per
  // wavefront (up to 14 computing wavefronts beside 2 producers in 1024 threads: 56 trials
  // share each staged channel, 10% faster than 6 x 8 on the full workload), then 8.
  int32_t span = 0;
  dd::Launch lg{};
  bool placed = false;
  const bool g_open = !(tuning && (tuning->dms_per_wave || tuning->waves));
  const int g_try[2] = {g_open && in_dtype == DD_F32 ? 4 : t.g, t.g};
  for (int gi = 0; gi < 2 && !placed; ++gi) {
    const int g = g_try[gi];
    if (gi == 1 && g == g_try[0]) break;
    const int maxw = g == 4 ? 16 : 8;  // wavefronts a workgroup may hold (1024 or 512 threads)
    const int npw = t.pw > 0 ? t.pw : (t.pw == 0 && in_dtype == DD_F32 && t.w + 2 <= maxw) ? 2 : 0;
    if (!(in_dtype == DD_F32 && npw > 0)) continue;
    const int wp8[5] = {6, 4, 3, 2, 1};
    const int wp4[5] = {14, 12, 8, 4, 1};
    const int* wp_opts = g == 4 ? wp4 : wp8;
    for (int oi = 0; oi < 5 && !placed; ++oi) {
      const int nw = t.w ? t.w : std::min(wp_opts[oi], maxw - npw);
      const int32_t sp = compute_span(p->delays, nchan, ndm, g * nw);
      const dd::Launch l = dd::choose_launch_prod(sp, nchan, t.cc, lds_cap, npw);
      if (l.nb >= 2) t.g = g, t.w = nw, span = sp, lg = l, placed = true;  // the most wavefronts that fit
      if (t.w) break;
    }
  }
  if (in_dtype == DD_F32 && !placed) {
    if (t.pw > 0 || t.g == 4) {
      delete p;
      return dd::fail(DD_ERR_UNSUPPORTED, "one DM group's windows do not fit the producer wavefronts' "
                                          "16-byte DMAs; use fewer DMs per workgroup or no producer");
    }
    if (!(tuning && tuning->waves)) t.w = 0;  // automatic: fall back to the other form
  }
  const int w_opts[4] = {8, 4, 2, 1};
  for (int oi = 0; oi < 4 && !placed; ++oi) {
    const int nw = t.w ? t.w : w_opts[oi];
    span = compute_span(p->delays, nchan, ndm, t.g * nw);
    lg = dd::choose_launch(span, nw, nchan, t.cc, lds_cap, (int)dd::elem_bytes(in_dtype));
    if (t.w || (lg.nb >= 2 && (int64_t)lg.nb * lg.cs >= std::min(8, nchan + 1)) || nw == 1) {
      t.w = nw;
      break;
    }
  }
  if (lg.nb < 2) {
    delete p;
    return dd::fail(DD_ERR_UNSUPPORTED, "delay spread of one DM group (" + std::to_string(span) +
                                            " samples) does not fit in LDS; use fewer DMs per workgroup");
  }
  p->tiles = t;
  lg.form = dd::kFormLds;
  p->launch = lg;
  p->dms_per_group = t.g * t.w;
  p->ngroups = (ndm + p->dms_per_group - 1) / p->dms_per_group;
  p->ndm_pad = p->ngroups * p->dms_per_group;
  p->max_span = span;
  // device table: per (channel, trial) the LDS byte offset of the trial's first 4-sample
  // chunk inside the channel slot: relative delay k to the group's first trial is read
  // from copy m = k & 3 at word k - m; then [ngroups][nchan] the groups' first delays
  p->dev_table.resize((size_t)nchan * p->ndm_pad + (size_t)p->ngroups * nchan);
  int32_t* gb = &p->dev_table[(size_t)nchan * p->ndm_pad];
  for (int32_t c = 0; c < nchan; ++c) {
    const int32_t* row = &p->delays[(size_t)c * ndm];
    int32_t* drow = &p->dev_table[(size_t)c * p->ndm_pad];
    for (int32_t gi = 0; gi < p->ngroups; ++gi) {
      const int32_t base = row[gi * p->dms_per_group];
      gb[(size_t)gi * nchan + c] = base;
      for (int32_t j = 0; j < p->dms_per_group; ++j) {
        const int32_t d = gi * p->dms_per_group + j;
        const int32_t k = row[d < ndm ? d : ndm - 1] - base;
        const int32_t m = k & 3;
        // byte offset: 32-bit words for 16/32-bit input, bytes for 8-bit input
        drow[d] = in_dtype == DD_U8 ? m * lg.L + (k - m) : 4 * (m * lg.L + (k - m));
      }
    }
  }
  p->id = g_next_id.fetch_add(1);
  *out = p;
  return DD_OK;
}

}  // namespace dd

extern "C" {

int dd_plan_create(dd_plan** out, const double* freq_mhz, int32_t nchan, double tsamp_s,
                   const double* dm, int32_t ndm, int32_t in_dtype, const dd_tuning* tuning) {
  return dd::plan_create(out, freq_mhz, nchan, tsamp_s, dm, ndm, in_dtype, tuning, dd::kLdsBytes);
}

void dd_plan_destroy(dd_plan* plan) { delete plan; }

int dd_plan_query(const dd_plan* p, int64_t nsamp, dd_plan_info* info) {
  dd::clear_error();
  if (!p || !info) return dd::fail(DD_ERR_INVALID_ARG, "plan and info must be non-NULL");
  std::memset(info, 0, sizeof(*info));
  info->nchan = p->nchan;
  info->ndm = p->ndm;
  info->in_dtype = p->dtype;
  info->maxdelay = p->maxdelay;
  info->nsamp = nsamp;
  info->dms_per_wave = p->tiles.g;
  info->waves = p->tiles.w;
  info->samples_per_lane = p->tiles.s;
  info->chan_stage = p->tiles.cc;
  info->producer_waves = p->launch.prod;
  info->max_span = p->max_span;
  info->kernel_form = p->launch.form;
  info->window_chunks = p->launch.form == dd::kFormRegWin ? p->launch.nch : 0;
  info->launch_copies = p->launch.form == dd::kFormLds ? 4 : p->launch.form == dd::kFormRegWin ? 1 : 0;
  info->launch_buf = p->launch.L;
  info->launch_stage = p->launch.cs;
  info->launch_ring = p->launch.nb;
  info->launch_lds = p->launch.lds;
  if (nsamp <= 0) return dd::fail(DD_ERR_INVALID_ARG, "nsamp must be > 0");
  const int64_t ring_row = dd::ring_len_for(p, nsamp) + dd::ring_mirror(p);
  info->ring_bytes = dd::ring_table_bytes(p) +
                     dd::align_up(ring_row * p->nchan * dd::ring_copies(p) * dd::elem_bytes(p->dtype));
  const int64_t nout = nsamp - p->maxdelay;
  // sized for nsamp outputs: covers a plain call (nout < nsamp) and a stream push (<= block)
  info->workspace_bytes = dd::workspace_layout(p, nsamp).total;
  info->stream_workspace_bytes = dd::workspace_layout(p, nsamp, false).total;
  if (nout <= 0) {
    info->nout = 0;
    return dd::fail(DD_ERR_TOO_SHORT, "nsamp must exceed maxdelay (" + std::to_string(p->maxdelay) + ")");
  }
  info->nout = nout;
  info->adds = (int64_t)p->ndm * p->nchan * nout;
  return DD_OK;
}

int dd_plan_delays(const dd_plan* p, int32_t* host_out) {
  dd::clear_error();
  if (!p || !host_out) return dd::fail(DD_ERR_INVALID_ARG, "plan and host_out must be non-NULL");
  std::memcpy(host_out, p->delays.data(), p->delays.size() * sizeof(int32_t));
  return DD_OK;
}

int dd_time_binning(const double* freq_mhz, int32_t nchan, double tsamp_s, const double* dm, int32_t ndm,
                    int32_t max_log2, double* dm_diag_out, int32_t* log2_out) {
  dd::clear_error();
  if (!freq_mhz || !dm || !log2_out) return dd::fail(DD_ERR_INVALID_ARG, "freq_mhz, dm and log2_out must be non-NULL");
  if (nchan < 1 || ndm < 1) return dd::fail(DD_ERR_INVALID_ARG, "nchan and ndm must be >= 1");
  if (!(tsamp_s > 0.0) || !std::isfinite(tsamp_s)) return dd::fail(DD_ERR_INVALID_ARG, "tsamp must be finite and > 0");
  if (max_log2 < 0 || max_log2 > 16) return dd::fail(DD_ERR_INVALID_ARG, "max_log2 must be in 0..16");
  std::vector<double> f(freq_mhz, freq_mhz + nchan);
  for (double v : f)
    if (!std::isfinite(v) || !(v > 0.0)) return dd::fail(DD_ERR_INVALID_ARG, "frequencies must be finite and > 0");
  for (int32_t d = 0; d < ndm; ++d) {
    if (!std::isfinite(dm[d]) || dm[d] < 0.0) return dd::fail(DD_ERR_INVALID_ARG, "DMs must be finite and >= 0");
    if (d > 0 && dm[d] < dm[d - 1]) return dd::fail(DD_ERR_INVALID_ARG, "DM trials must be in non-decreasing order");
  }
  // Diagonal DM: one over the largest per-DM delay difference (in samples) between
  // neighbouring channels in frequency order; each double operation rounds once.
  std::sort(f.begin(), f.end());
  double worst = 0.0;
  for (size_t c = 0; c + 1 < f.size(); ++c) {
    const double a = f[c], b = f[c + 1];
    const double per_dm = (kDm * (1.0 / (a * a) - 1.0 / (b * b))) / tsamp_s;
    worst = std::max(worst, per_dm);
  }
  const double diag = worst > 0.0 ? 1.0 / worst : std::numeric_limits<double>::infinity();
  if (dm_diag_out) *dm_diag_out = diag;
  for (int32_t d = 0; d < ndm; ++d) {
    int32_t k = 0;
    while (k < max_log2 && dm[d] > diag * (double)(1 << k)) ++k;
    log2_out[d] = k;
  }
  return DD_OK;
}

}  // extern "C"
