// C ABI of the fast-mode simulator (include/simradar.h): validation, launch
// plans, workspace layout and the calls that chain the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/simradar.h"
#include "launch.hpp"

using simk::ColPlan;
using simk::GridP;
using simk::RadarP;
using simk::RowPlan;
using simk::WinP;

struct sim_ctx {
  int device;
  sim_precision prec;
  const void* tw;      // the device's twiddle table of the context's precision
  void* ws;
  size_t ws_bytes;
  int row_bands;   // tuning: bands of the fused row pass (0 = default)
  int row_path;    // tuning: row path of the fused call (SIM_ROW_PATH_*)
  int acc_bands;   // tuning: most bands of the facet accumulate (0 = default)
  bool capturing;  // a batch is being captured into a graph
  // per-kernel timing: a pool of event pairs made by sim_profile_enable, so
  // that no compute call creates events
  bool profiling;
  std::vector<hipEvent_t> ev;   // pool, pairs (start, stop)
  std::vector<int> kind;        // kernel kind of each recorded pair
  size_t used;                  // pairs recorded
  uint64_t dropped;             // launches not timed (pool exhausted)
  int tab_slot;                 // slot of the look-up tables (-1: closed forms)
  // update lanes of sim_run_updates (SIM_TUNE_UPDATE_LANES): lane 0 is the
  // caller's stream, lanes 1.. have their own streams (default priority);
  // each lane has its own workspace slice
  int lanes;
  std::vector<hipStream_t> lane_st;
  std::vector<hipEvent_t> lane_ev;   // [0]: fork, [1 + l]: join of stream l
};

// Twiddle tables (entries [M, 2M) hold e^{+2 pi i m / M} for every power of
// two M <= kTwMax), one per precision, in the code object: every device the
// library runs on holds its own copy, filled once by the first sim_create on
// that device.  Host code uses them only through the addresses returned by
// hipGetSymbolAddress for that device.
__device__ __align__(256) float g_tw32[2 * simk::kTwEntries];
__device__ __align__(256) double g_tw64[2 * simk::kTwEntries];

// Scratch of sim_range_doppler_accumulate_noalloc: the band windows of
// partial spectra (at most kNoAllocBands bands of kSlots windows of at most
// 32 KiB: window_bins never makes one larger), then their headers and the
// band counters.  One copy per device, held until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for
// that device (device_setup).  Nothing in it has to start at zero: a call
// writes every header and counter it reads, and every window slot whose
// header it marks valid.
constexpr int kNoAllocBands = 256;
constexpr size_t kNoAllocWinBytes = (size_t)kNoAllocBands * 4 * 32 * 1024;
constexpr size_t kNoAllocHdrOff = kNoAllocWinBytes;
constexpr size_t kNoAllocCntOff = kNoAllocHdrOff + (size_t)kNoAllocBands * 4 * 16;
constexpr size_t kNoAllocBytes = kNoAllocCntOff + (size_t)kNoAllocBands * 8 * 4;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Parameter blocks of the look-up tables (sim_set_tables), one slot per
// context that has tables, per device; the kernels read the block through
// its device address.
constexpr int kTabSlots = 256;
__device__ __align__(256) simk::TabP g_tab_slots[kTabSlots];

namespace {

using simk::kLdsBudget;
constexpr size_t kWindowBudget = 32 * 1024;    // LDS of one window of partial spectra
constexpr int kSlots = 4;                      // window slots per band
constexpr int kMaxBands = 512;       // bands (blocks) of the fused row pass
constexpr int kMaxUpdateLanes = 4;   // update lanes of sim_run_updates
constexpr int kAccBands = 512;       // bands (blocks) of the facet accumulate
constexpr int kWsBands = kAccBands > kMaxBands ? kAccBands : kMaxBands;
constexpr int kProfilePairs = 8192;  // timed launches per profile record
static_assert(kNoAllocWinBytes == (size_t)kNoAllocBands * kSlots * kWindowBudget,
              "scratch sized for the windows of kNoAllocBands bands");
static_assert(kNoAllocBands <= kAccBands, "no more bands than the workspace path");

bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(long v) {
  int r = 0;
  while ((1L << r) < v) ++r;
  return r;
}
long floor_pow2(long v) {
  long r = 1;
  while ((r << 1) <= v) r <<= 1;
  return r;
}
size_t lpad(size_t i) { return i + (i >> 4); }
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
bool isfin(double v) { return std::isfinite(v); }

size_t csize(const sim_ctx* c) { return c->prec == SIM_PREC_FP64 ? 16 : 8; }

sim_status check_grid(const sim_ctx* c, const sim_grid* g) {
  if (!g) return SIM_ERR_ARG;
  if (!is_pow2(g->nx) || !is_pow2(g->ny)) return SIM_ERR_UNSUPPORTED;
  if (g->nx < 16 || g->nx > 8192 || g->ny < 16 || g->ny > 16384) return SIM_ERR_UNSUPPORTED;
  if (c->prec == SIM_PREC_FP64 && g->ny > 8192) return SIM_ERR_UNSUPPORTED;
  if (!(isfin(g->dx) && g->dx > 0 && isfin(g->dy) && g->dy > 0)) return SIM_ERR_ARG;
  if (!(isfin(g->x_origin) && isfin(g->y_origin))) return SIM_ERR_ARG;
  if (!(isfin(g->gravity) && g->gravity > 0)) return SIM_ERR_ARG;
  return SIM_OK;
}

sim_status check_radar(const sim_radar* r) {
  if (!r) return SIM_ERR_ARG;
  if (!(isfin(r->altitude) && r->altitude > 0 && isfin(r->velocity) && isfin(r->sat_x) &&
        isfin(r->sat_y0) && isfin(r->carrier_hz) && r->carrier_hz > 0 && isfin(r->prf_hz) &&
        r->prf_hz > 0 && isfin(r->gate_spacing) && r->gate_spacing > 0 &&
        isfin(r->window_start) && isfin(r->beamwidth_3db) && r->beamwidth_3db > 0 &&
        isfin(r->fresnel_sq) && r->fresnel_sq >= 0 && isfin(r->mss) && r->mss > 0))
    return SIM_ERR_ARG;
  if (r->n_gates < 1 || r->n_fast < 1) return SIM_ERR_ARG;
  if (r->window != SIM_WIN_SQRT_TRIANGLE && r->window != SIM_WIN_SQRT_RAISED_COSINE)
    return SIM_ERR_ARG;
  if (!is_pow2(r->n_doppler) || r->n_doppler < 2 || r->n_doppler > 2048)
    return SIM_ERR_UNSUPPORTED;
  if (r->n_gates > 65536) return SIM_ERR_UNSUPPORTED;
  return SIM_OK;
}

ColPlan col_plan(int nx, int ny, size_t cs) {
  ColPlan p;
  const int l = ilog2(ny);
  p.cpb = simk::col_cpb(l, (int)cs);
  p.threads = simk::col_threads(l, (int)cs);
  p.lds_bytes = simk::col_lds(l, (int)cs);
  if (p.cpb > nx) p.lds_bytes = (size_t)-1;   // strips wider than the grid: unsupported
  return p;
}

// Bins per window: the whole spectrum when it fits, else the largest power
// of two that fits the window budget and what the row transforms leave.
int window_bins(int G, int N, size_t cs, size_t fft_bytes) {
  size_t budget = kWindowBudget;
  const size_t left = kLdsBudget > fft_bytes + 512 ? kLdsBudget - fft_bytes - 512 : 0;
  if (left < budget) budget = left;
  const size_t per_bin = (size_t)G * cs;
  if (per_bin == 0 || budget < per_bin) return 0;
  const long wk = floor_pow2((long)(budget / per_bin));
  return wk >= N ? N : (int)wk;
}

RowPlan row_plan(int nx, size_t cs) {
  RowPlan p;
  const int l = ilog2(nx);
  p.rpb = simk::row_rpb(l);
  p.threads = simk::row_threads(l);
  p.fft_bytes = simk::row_fft_lds(l, (int)cs);
  p.front_bytes = p.fft_bytes + simk::row_stage_bytes(simk::row_stage_fused(l, (int)cs), l, (int)cs);
  p.acc_bytes = 0;
  return p;
}

struct WsLayout {
  size_t planes, part, hdr, bandcnt, facets, facet_stride, total;
};

// Bytes of the column pass's half planes.
size_t plane_bytes(const sim_grid* g, size_t cs) {
  return simk::kHalfPlanes * simk::half_plane_elems(ilog2(g->nx), ilog2(g->ny), (int)cs) * cs;
}

WsLayout ws_layout(const sim_grid* g, const sim_radar* r, size_t cs) {
  WsLayout L;
  const size_t P = (size_t)g->nx * g->ny;
  const int wk = window_bins(r->n_gates, r->n_doppler, cs, 0);
  size_t off = 0;
  L.planes = off;
  off = align256(off + plane_bytes(g, cs));
  L.part = off;
  off = align256(off + (size_t)kWsBands * kSlots * r->n_gates * (size_t)(wk > 0 ? wk : 1) * cs);
  L.hdr = off;
  off = align256(off + (size_t)kWsBands * kSlots * 16);
  L.bandcnt = off;
  off = align256(off + (size_t)kWsBands * 8 * 4);
  // facet fields of the split row path (9 planes of P reals)
  L.facets = off;
  L.facet_stride = align256(P * (cs / 2));
  off += 9 * L.facet_stride;
  L.total = off;
  return L;
}

// Facets per band and bands of the facet accumulate: the grid cut into at
// most max_bands bands of at least 1024 facets.
size_t acc_band_size(size_t P, int max_bands) {
  size_t band = (P + max_bands - 1) / max_bands;
  return band < 1024 ? 1024 : band;
}
int acc_band_count(size_t P, int max_bands) {
  const size_t band = acc_band_size(P, max_bands);
  return (int)((P + band - 1) / band);
}

void fill_grid(const sim_grid* g, GridP& gp) {
  gp.nx = g->nx;
  gp.ny = g->ny;
  gp.log2nx = ilog2(g->nx);
  gp.log2ny = ilog2(g->ny);
  gp.cwm = g->cwm ? 1 : 0;
  gp.dx = g->dx;
  gp.dy = g->dy;
  gp.x_origin = g->x_origin;
  gp.y_origin = g->y_origin;
  gp.gravity = g->gravity;
  gp.sqrt_g = std::sqrt(g->gravity);
}

// Platform positions, Doppler constant and amplitude constants.  The double
// expressions below are the ones the range and index arithmetic is defined
// with (evaluated once here, in this order).
void fill_radar(const sim_radar* r, const sim_grid* g, double t, RadarP& rp,
                const simk::TabP* tab = nullptr) {
  rp.tab = tab;
  rp.altitude = r->altitude;
  rp.sat_x = r->sat_x;
  rp.sat_y1 = r->sat_y0 + r->velocity * t;
  const double t2 = t + 1.0 / r->prf_hz;
  rp.sat_y2 = r->sat_y0 + r->velocity * t2;
  rp.k2 = 2.0 * r->carrier_hz / 299792458.0;
  rp.gate_spacing = r->gate_spacing;
  rp.window_start = r->window_start;
  rp.fresnel_over_mss = r->fresnel_sq / r->mss;
  rp.inv_mss = 1.0 / r->mss;
  const double sh = std::sin(0.5 * r->beamwidth_3db);
  const double gamma = (2.0 / std::log(2.0)) * sh * sh;
  rp.two_over_gamma = 2.0 / gamma;
  rp.cell_area = g->dx * g->dy;
  rp.G = r->n_gates;
  rp.N = r->n_doppler;
  rp.log2N = ilog2(r->n_doppler);
}

sim_status use_device(const sim_ctx* c) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return SIM_ERR_DEVICE;
  if (cur != c->device && hipSetDevice(c->device) != hipSuccess) return SIM_ERR_DEVICE;
  return SIM_OK;
}

// SIMRADAR_DEBUG=1 prints the HIP error behind every SIM_ERR_DEVICE.
sim_status dev_err(hipError_t e, const char* what) {
  if (e == hipSuccess) return SIM_OK;
  const char* dbg = std::getenv("SIMRADAR_DEBUG");
  if (dbg && dbg[0] == '1')
    std::fprintf(stderr, "simradar: %s: %s (%d)\n", what, hipGetErrorString(e), (int)e);
  return SIM_ERR_DEVICE;
}
#define dev(e) dev_err((e), #e)

// Roots of unity per size (entries [M, 2M) hold e^{+2 pi i m / M}),
// evaluated in long double and rounded once.
template <typename Real>
void make_twiddles(Real* host) {
  const long double two_pi = 6.283185307179586476925286766559L;
  host[0] = host[1] = (Real)0;
  for (int M = 1; M <= simk::kTwMax; M <<= 1) {
    for (int m = 0; m < M; ++m) {
      const long double a = two_pi * (long double)m / (long double)M;
      host[2 * (M + m)] = (Real)cosl(a);
      host[2 * (M + m) + 1] = (Real)sinl(a);
    }
  }
}

// Per-device state of the library's static device memory, set up once per
// device (by the first sim_create on it, with the device current).
constexpr int kMaxDevices = 64;
struct DeviceState {
  bool ready;
  void* tw32;
  void* tw64;
  void* scratch;   // device address of `scratch` on this device
  simk::TabP* tabs;              // device address of g_tab_slots
  bool tab_used[kTabSlots];      // slots held by live contexts
};
std::mutex g_dev_mutex;
DeviceState g_dev[kMaxDevices];

template <typename Real>
sim_status fill_twiddles(void* dst) {
  const size_t n = 2 * (size_t)simk::kTwEntries;
  Real* host = new (std::nothrow) Real[n];
  if (!host) return SIM_ERR_DEVICE;
  make_twiddles<Real>(host);
  const sim_status s = dev_err(hipMemcpy(dst, host, n * sizeof(Real), hipMemcpyHostToDevice),
                               "twiddle table upload");
  delete[] host;
  return s;
}

// Resolve the device addresses of the static tables on `device` (current)
// and fill the twiddles; idempotent.
sim_status device_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return SIM_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_dev_mutex);
  DeviceState& d = g_dev[device];
  if (d.ready) return SIM_OK;
  void* a = nullptr;
  void* b = nullptr;
  void* sc = nullptr;
  sim_status s = dev_err(hipGetSymbolAddress(&a, HIP_SYMBOL(g_tw32)), "twiddle table address");
  if (s == SIM_OK)
    s = dev_err(hipGetSymbolAddress(&b, HIP_SYMBOL(g_tw64)), "twiddle table address");
  if (s == SIM_OK)
    s = dev_err(hipGetSymbolAddress(&sc, HIP_SYMBOL(scratch)), "scratch address");
  void* tb = nullptr;
  if (s == SIM_OK)
    s = dev_err(hipGetSymbolAddress(&tb, HIP_SYMBOL(g_tab_slots)), "table slots address");
  if (s == SIM_OK && (!a || !b || !sc || !tb))
    s = dev_err(hipErrorInvalidSymbol, "static arrays");
  if (s == SIM_OK) s = fill_twiddles<float>(a);
  if (s == SIM_OK) s = fill_twiddles<double>(b);
  if (s != SIM_OK) return s;
  d.tw32 = a;
  d.tw64 = b;
  d.scratch = sc;
  d.tabs = (simk::TabP*)tb;
  for (bool& u : d.tab_used) u = false;
  d.ready = true;
  return SIM_OK;
}

// Device address of the context's table parameter block, or null.
const simk::TabP* ctx_tab(const sim_ctx* c) {
  return c->tab_slot >= 0 ? g_dev[c->device].tabs + c->tab_slot : nullptr;
}

void release_tab_slot(sim_ctx* c) {
  if (c->tab_slot < 0) return;
  std::lock_guard<std::mutex> lock(g_dev_mutex);
  g_dev[c->device].tab_used[c->tab_slot] = false;
  c->tab_slot = -1;
}

// The lane streams and events (after the work queued on them).
void release_lanes(sim_ctx* c) {
  if (!c->lane_st.empty() || !c->lane_ev.empty()) (void)use_device(c);
  for (hipStream_t st : c->lane_st) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (hipEvent_t e : c->lane_ev) (void)hipEventDestroy(e);
  c->lane_st.clear();
  c->lane_ev.clear();
  c->lanes = 1;
}

// Runs body(i, stream) for i in [0, count): on the caller's stream `st` when
// the context has one lane, else dealt round robin to its lanes (lane 0 is
// `st`; the lanes are forked from `st` by an event and joined back to it, so
// the whole is ordered on `st`, also under graph capture).  With ws_slice >
// 0 each lane enqueues with its own workspace slice (l * ws_slice; the
// workspace must hold one per lane).  Stops at the first error; always joins.
template <typename Body>
sim_status run_on_lanes(sim_ctx* ctx, int32_t count, size_t ws_slice, hipStream_t st, Body body) {
  const int NL = count > 1 ? std::min(ctx->lanes, (int)count) : 1;
  sim_status s = SIM_OK;
  if (NL == 1) {
    for (int32_t i = 0; i < count && s == SIM_OK; ++i) s = body(i, st);
    return s;
  }
  if (ws_slice && ctx->ws_bytes < (size_t)ctx->lanes * ws_slice) return SIM_ERR_WORKSPACE;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  s = dev(hipEventRecord(ctx->lane_ev[0], st));
  for (int l = 1; l < NL && s == SIM_OK; ++l)
    s = dev(hipStreamWaitEvent(ctx->lane_st[l - 1], ctx->lane_ev[0], 0));
  if (s != SIM_OK) return s;
  void* const ws0 = ctx->ws;
  const size_t ws_bytes0 = ctx->ws_bytes;
  if (ws_slice) ctx->ws_bytes = ws_slice;
  for (int32_t i = 0; i < count && s == SIM_OK; ++i) {
    const int l = i % NL;
    if (ws_slice) ctx->ws = (char*)ws0 + (size_t)l * ws_slice;
    s = body(i, l ? ctx->lane_st[l - 1] : st);
  }
  ctx->ws = ws0;
  ctx->ws_bytes = ws_bytes0;
  for (int l = 1; l < NL; ++l) {
    sim_status sj = dev(hipEventRecord(ctx->lane_ev[l], ctx->lane_st[l - 1]));
    if (sj == SIM_OK) sj = dev(hipStreamWaitEvent(st, ctx->lane_ev[l], 0));
    if (sj != SIM_OK && s == SIM_OK) s = sj;
  }
  return s;
}

// The facet set of update i of a stacked run (every field advanced by i
// fields of `field_bytes`).
sim_facets stacked_facets(const sim_facets& f, int32_t i, size_t field_bytes) {
  const size_t o = (size_t)i * field_bytes;
  sim_facets g;
  g.disp_x = (char*)f.disp_x + o;
  g.disp_y = (char*)f.disp_y + o;
  g.h = (char*)f.h + o;
  g.sx = (char*)f.sx + o;
  g.sy = (char*)f.sy + o;
  g.jac = (char*)f.jac + o;
  g.ddisp_x = (char*)f.ddisp_x + o;
  g.ddisp_y = (char*)f.ddisp_y + o;
  g.dh = (char*)f.dh + o;
  return g;
}

bool times_ok(const double* times, int32_t count) {
  if (!times) return false;
  for (int32_t i = 0; i < count; ++i)
    if (!isfin(times[i])) return false;
  return true;
}

bool facets_ok(const sim_facets* f) {
  if (!f) return false;
  void* const p[9] = {f->disp_x, f->disp_y, f->h, f->sx, f->sy, f->jac, f->ddisp_x, f->ddisp_y,
                      f->dh};
  for (void* q : p)
    if (!q) return false;
  return true;
}

WinP win_params(char* base, const sim_radar* r, const WsLayout& L, int wk, int n_bands,
                int band_size) {
  WinP wp;
  wp.WK = wk;
  wp.log2WK = ilog2(wk);
  wp.S = kSlots;
  wp.n_bands = n_bands;
  wp.band_rows = band_size;
  wp.part = base + L.part;
  wp.hdr = (int4*)(base + L.hdr);
  wp.bandcnt = (uint32_t*)(base + L.bandcnt);
  (void)r;
  return wp;
}

sim_status common_checks(sim_ctx* c, const sim_grid* g, const sim_radar* r, WsLayout* L) {
  if (!c) return SIM_ERR_ARG;
  sim_status s = check_grid(c, g);
  if (s != SIM_OK) return s;
  if (r) {
    s = check_radar(r);
    if (s != SIM_OK) return s;
    // the calls given a radar scatter facets, keeping one Doppler bin of all
    // gates in an LDS window: a size that cannot is unsupported, whatever
    // the workspace
    if (window_bins(r->n_gates, r->n_doppler, csize(c), 0) < 1) return SIM_ERR_UNSUPPORTED;
  }
  if (!c->ws) return SIM_ERR_WORKSPACE;
  if (r) {
    *L = ws_layout(g, r, csize(c));
    if (L->total > c->ws_bytes) return SIM_ERR_WORKSPACE;
  } else {
    const size_t need = align256(plane_bytes(g, csize(c)));
    if (need > c->ws_bytes) return SIM_ERR_WORKSPACE;
    L->planes = 0;
  }
  return SIM_OK;
}

// Bracket one kernel launch with events when profiling is on.  The events
// come from the pool made by sim_profile_enable; when it is exhausted the
// launch is not timed and counted as dropped.
struct ProfScope {
  sim_ctx* c;
  hipStream_t st;
  bool on;
  ProfScope(sim_ctx* c_, int kind, hipStream_t st_)
      : c(c_), st(st_), on(c_->profiling && !c_->capturing) {
    if (!on) return;
    if (c->used * 2 + 2 > c->ev.size()) {
      c->dropped++;
      on = false;
      return;
    }
    c->kind[c->used] = kind;
    (void)hipEventRecord(c->ev[2 * c->used], st);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(c->ev[2 * c->used + 1], st);
    c->used++;
  }
};

template <typename Real>
sim_status accumulate_fused(sim_ctx* c, const sim_grid* g, const void* spec0, bool prepared,
                            const sim_radar* r, double t, int32_t j, void* t_fast,
                            sim_counters* counters, int32_t* code, hipStream_t st,
                            const WsLayout& L) {
  GridP gp;
  RadarP rp;
  fill_grid(g, gp);
  fill_radar(r, g, t, rp, ctx_tab(c));
  const size_t cs = sizeof(Real) * 2;
  char* base = (char*)c->ws;
  void* planes = base + L.planes;
  const ColPlan cp = col_plan(g->nx, g->ny, cs);
  if (cp.lds_bytes > kLdsBudget) return SIM_ERR_UNSUPPORTED;
  RowPlan rpl = row_plan(g->nx, cs);
  const int wk = window_bins(r->n_gates, r->n_doppler, cs, rpl.front_bytes);
  if (wk < 1) return SIM_ERR_UNSUPPORTED;
  rpl.acc_bytes = rpl.front_bytes + (size_t)r->n_gates * wk * cs + simk::kWinCtxBytes;
  int target = rpl.threads <= 512 ? kMaxBands : kMaxBands / 2;
  if (c->row_bands > 0 && c->row_bands < target) target = c->row_bands;
  int n_bands, band_rows;
  if (g->ny >= rpl.rpb) {
    n_bands = g->ny / rpl.rpb < target ? g->ny / rpl.rpb : target;
    // rows per band: a whole number of row steps covering the grid
    band_rows = (g->ny + n_bands - 1) / n_bands;
    band_rows = (band_rows + rpl.rpb - 1) / rpl.rpb * rpl.rpb;
    n_bands = (g->ny + band_rows - 1) / band_rows;
  } else {
    n_bands = 1;
    band_rows = rpl.rpb;
  }
  const WinP wp = win_params((char*)c->ws, r, L, wk, n_bands, band_rows);
  void* Tj = (char*)t_fast + (size_t)j * r->n_gates * r->n_doppler * cs;
  sim_status s;
  {
    ProfScope p(c, SIM_KERNEL_SURFACE_COLPASS, st);
    s = dev(simk::launch_colpass<Real>(spec0, planes, gp, t, 1.0 / r->prf_hz, c->tw, prepared,
                                       st));
  }
  if (s != SIM_OK) return s;
  {
    ProfScope p(c, SIM_KERNEL_FUSED_ROWPASS, st);
    s = dev(simk::launch_rowpass_accumulate<Real>(planes, gp, rp, wp, Tj, code, rpl.acc_bytes,
                                                  c->tw, st));
  }
  if (s != SIM_OK) return s;
  ProfScope p(c, SIM_KERNEL_REDUCE_PARTIALS, st);
  return dev(simk::launch_reduce<Real>(rp, wp, Tj, (unsigned long long*)counters, st));
}

template <typename Real>
sim_status accumulate_facets(sim_ctx* c, const sim_grid* g, const sim_facets* f,
                             const sim_radar* r, double t, int32_t j, void* t_fast,
                             sim_counters* counters, int32_t* code, hipStream_t st,
                             const WsLayout& L, char* win_base = nullptr,
                             int max_bands = 0);

// Row path of the fused call: the fused row pass (facets never leave the
// chip), or the facet row pass into the workspace followed by the facet
// accumulate.  Automatic choice: the split path.  The fused row kernel holds
// nine facet fields per value slot in registers (about 245 VGPRs in float,
// spills in double and for 8192-wide rows), so a CU runs one block of it;
// the two split kernels keep several blocks per CU and measure faster even
// with the facet round trip through HBM (4096^2 float: 0.62 vs 0.68 ms per
// update for the row pass and accumulate; double: 1.18 vs 2.30 ms).
bool use_split(const sim_ctx* c, const sim_grid* g) {
  (void)g;
  if (c->row_path == SIM_ROW_PATH_FUSED) return false;
  return true;
}

sim_status surface_update_impl(sim_ctx* ctx, const sim_grid* grid, const void* spec0,
                               bool prepared, double t, double dt_pair, const sim_facets* out,
                               hipStream_t st);

template <typename Real>
sim_status accumulate_split(sim_ctx* c, const sim_grid* g, const void* spec0, bool prepared,
                            const sim_radar* r, double t, int32_t j, void* t_fast,
                            sim_counters* counters, int32_t* code, hipStream_t st,
                            const WsLayout& L) {
  char* fb = (char*)c->ws + L.facets;
  const size_t fs = L.facet_stride;
  sim_facets f;
  f.disp_x = fb + 0 * fs;
  f.disp_y = fb + 1 * fs;
  f.h = fb + 2 * fs;
  f.sx = fb + 3 * fs;
  f.sy = fb + 4 * fs;
  f.jac = fb + 5 * fs;
  f.ddisp_x = fb + 6 * fs;
  f.ddisp_y = fb + 7 * fs;
  f.dh = fb + 8 * fs;
  const sim_status s = surface_update_impl(c, g, spec0, prepared, t, 1.0 / r->prf_hz, &f, st);
  if (s != SIM_OK) return s;
  return accumulate_facets<Real>(c, g, &f, r, t, j, t_fast, counters, code, st, L);
}

// Facet accumulate of update j.  The band windows, their headers and the
// band counters are at the offsets of L from win_base (the context's
// workspace when NULL); the facets are cut into at most max_bands bands.
template <typename Real>
sim_status accumulate_facets(sim_ctx* c, const sim_grid* g, const sim_facets* f,
                             const sim_radar* r, double t, int32_t j, void* t_fast,
                             sim_counters* counters, int32_t* code, hipStream_t st,
                             const WsLayout& L, char* win_base, int max_bands) {
  GridP gp;
  RadarP rp;
  fill_grid(g, gp);
  fill_radar(r, g, t, rp, ctx_tab(c));
  const size_t cs = sizeof(Real) * 2;
  const int wk = window_bins(r->n_gates, r->n_doppler, cs, 0);
  if (wk < 1) return SIM_ERR_UNSUPPORTED;
  const size_t P = (size_t)g->nx * g->ny;
  if (max_bands <= 0) max_bands = c->acc_bands > 0 ? c->acc_bands : kAccBands;
  const int n_bands = acc_band_count(P, max_bands);
  const size_t band = acc_band_size(P, max_bands);
  const WinP wp = win_params(win_base ? win_base : (char*)c->ws, r, L, wk, n_bands, (int)band);
  const size_t lds = (size_t)r->n_gates * wk * cs + simk::kWinCtxBytes;
  void* const fp[9] = {f->disp_x, f->disp_y, f->h, f->sx, f->sy, f->jac, f->ddisp_x, f->ddisp_y,
                       f->dh};
  void* Tj = (char*)t_fast + (size_t)j * r->n_gates * r->n_doppler * cs;
  sim_status s;
  {
    ProfScope p(c, SIM_KERNEL_ACCUMULATE_FACETS, st);
    s = dev(simk::launch_accumulate_facets<Real>(fp, gp, rp, wp, Tj, code, lds, st));
  }
  if (s != SIM_OK) return s;
  ProfScope p(c, SIM_KERNEL_REDUCE_PARTIALS, st);
  return dev(simk::launch_reduce<Real>(rp, wp, Tj, (unsigned long long*)counters, st));
}

}  // namespace

extern "C" {

int sim_abi_version(void) { return SIM_ABI_VERSION; }

const char* sim_status_string(sim_status s) {
  switch (s) {
    case SIM_OK: return "ok";
    case SIM_ERR_ARG: return "invalid argument";
    case SIM_ERR_SHAPE: return "inconsistent shape or index";
    case SIM_ERR_UNSUPPORTED: return "unsupported size";
    case SIM_ERR_WORKSPACE: return "workspace missing or too small";
    case SIM_ERR_DEVICE: return "HIP device error";
  }
  return "unknown status";
}

sim_status sim_create(sim_ctx** ctx, int device, sim_precision precision) {
  if (!ctx) return SIM_ERR_ARG;
  *ctx = nullptr;
  if (precision != SIM_PREC_FP64 && precision != SIM_PREC_FP32_PHASE64) return SIM_ERR_ARG;
  int n = 0;
  if (dev(hipGetDeviceCount(&n)) != SIM_OK) return SIM_ERR_DEVICE;
  if (device < 0 || device >= n) return SIM_ERR_ARG;
  if (dev(hipSetDevice(device)) != SIM_OK) return SIM_ERR_DEVICE;
  int lds_max = 0;
  if (dev(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device)) !=
      SIM_OK)
    return SIM_ERR_DEVICE;
  if ((size_t)lds_max < kLdsBudget) {
    dev_err(hipErrorInvalidValue, "device LDS per block below the 159 KiB the kernels plan for");
    return SIM_ERR_UNSUPPORTED;
  }
  // the attribute only raises the dynamic-LDS cap; a runtime that does not
  // need it may refuse it, which is harmless
  if (simk::init_kernel_attributes(lds_max) != hipSuccess) (void)hipGetLastError();
  const sim_status sd = device_setup(device);
  if (sd != SIM_OK) return sd;
  sim_ctx* c = new (std::nothrow) sim_ctx;
  if (!c) return SIM_ERR_DEVICE;
  c->device = device;
  c->prec = precision;
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->tw = precision == SIM_PREC_FP64 ? g_dev[device].tw64 : g_dev[device].tw32;
  c->profiling = false;
  c->used = 0;
  c->dropped = 0;
  c->row_bands = 0;
  c->row_path = SIM_ROW_PATH_AUTO;
  c->acc_bands = 0;
  c->capturing = false;
  c->tab_slot = -1;
  c->lanes = 1;
  *ctx = c;
  return SIM_OK;
}

sim_status sim_destroy(sim_ctx* ctx) {
  if (!ctx) return SIM_OK;
  release_tab_slot(ctx);
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  release_lanes(ctx);
  delete ctx;
  return SIM_OK;
}

sim_status sim_get_precision(const sim_ctx* ctx, sim_precision* precision) {
  if (!ctx || !precision) return SIM_ERR_ARG;
  *precision = ctx->prec;
  return SIM_OK;
}

sim_status sim_workspace_size(const sim_ctx* ctx, const sim_grid* grid, const sim_radar* radar,
                              size_t* bytes) {
  if (!ctx || !bytes) return SIM_ERR_ARG;
  sim_status s = check_grid(ctx, grid);
  if (s != SIM_OK) return s;
  s = check_radar(radar);
  if (s != SIM_OK) return s;
  if (window_bins(radar->n_gates, radar->n_doppler, csize(ctx), 0) < 1) return SIM_ERR_UNSUPPORTED;
  const size_t one = ws_layout(grid, radar, csize(ctx)).total;
  *bytes = ctx->lanes > 1 ? (size_t)ctx->lanes * align256(one) : one;
  return SIM_OK;
}

sim_status sim_set_workspace(sim_ctx* ctx, void* device_ptr, size_t bytes) {
  if (!ctx) return SIM_ERR_ARG;
  if (bytes == 0) {
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    return SIM_OK;
  }
  if (!device_ptr || ((uintptr_t)device_ptr & 255) != 0) return SIM_ERR_ARG;
  ctx->ws = device_ptr;
  ctx->ws_bytes = bytes;
  return SIM_OK;
}

namespace {

sim_status surface_update_impl(sim_ctx* ctx, const sim_grid* grid, const void* spec0,
                               bool prepared, double t, double dt_pair, const sim_facets* out,
                               hipStream_t st) {
  GridP gp;
  fill_grid(grid, gp);
  const size_t cs = csize(ctx);
  const ColPlan cp = col_plan(grid->nx, grid->ny, cs);
  if (cp.lds_bytes > kLdsBudget) return SIM_ERR_UNSUPPORTED;
  void* const o[9] = {out->disp_x, out->disp_y, out->h, out->sx, out->sy, out->jac,
                      out->ddisp_x, out->ddisp_y, out->dh};
  void* planes = ctx->ws;
  const bool f64 = ctx->prec == SIM_PREC_FP64;
  sim_status s;
  {
    ProfScope p(ctx, SIM_KERNEL_SURFACE_COLPASS, st);
    s = f64 ? dev(simk::launch_colpass<double>(spec0, planes, gp, t, dt_pair, ctx->tw, prepared,
                                               st))
            : dev(simk::launch_colpass<float>(spec0, planes, gp, t, dt_pair, ctx->tw, prepared,
                                              st));
  }
  if (s != SIM_OK) return s;
  ProfScope p(ctx, SIM_KERNEL_SURFACE_ROWPASS, st);
  return f64 ? dev(simk::launch_rowpass_facets<double>(planes, gp, o, ctx->tw, st))
             : dev(simk::launch_rowpass_facets<float>(planes, gp, o, ctx->tw, st));
}

sim_status update_and_accumulate_impl(sim_ctx* ctx, const sim_grid* grid, const void* spec0,
                                      bool prepared, const sim_radar* radar, double t, int32_t j,
                                      void* t_fast, int32_t n_spec, sim_counters* counters,
                                      int32_t* facet_code, void* stream) {
  WsLayout L;
  sim_status s = common_checks(ctx, grid, radar, &L);
  if (s != SIM_OK) return s;
  if (!spec0 || !t_fast || !isfin(t)) return SIM_ERR_ARG;
  if (n_spec < 1 || j < 0 || j >= n_spec) return SIM_ERR_SHAPE;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const bool split = use_split(ctx, grid);
  if (ctx->prec == SIM_PREC_FP64)
    return split ? accumulate_split<double>(ctx, grid, spec0, prepared, radar, t, j, t_fast,
                                            counters, facet_code, st, L)
                 : accumulate_fused<double>(ctx, grid, spec0, prepared, radar, t, j, t_fast,
                                            counters, facet_code, st, L);
  return split ? accumulate_split<float>(ctx, grid, spec0, prepared, radar, t, j, t_fast,
                                         counters, facet_code, st, L)
               : accumulate_fused<float>(ctx, grid, spec0, prepared, radar, t, j, t_fast,
                                         counters, facet_code, st, L);
}

}  // namespace

sim_status sim_surface_update(sim_ctx* ctx, const sim_grid* grid, const void* spec0, double t,
                              double dt_pair, const sim_facets* out, void* stream) {
  WsLayout L;
  sim_status s = common_checks(ctx, grid, nullptr, &L);
  if (s != SIM_OK) return s;
  if (!spec0 || !facets_ok(out) || !isfin(t) || !isfin(dt_pair)) return SIM_ERR_ARG;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  return surface_update_impl(ctx, grid, spec0, false, t, dt_pair, out, (hipStream_t)stream);
}

sim_status sim_prepared_spectrum_size(const sim_ctx* ctx, const sim_grid* grid, size_t* bytes) {
  if (!ctx || !bytes) return SIM_ERR_ARG;
  const sim_status s = check_grid(ctx, grid);
  if (s != SIM_OK) return s;
  // the pair (c(k), c(-k)) of every mode kx >= 0 (half width of the planes)
  const size_t cs = csize(ctx);
  *bytes = 2 * simk::half_plane_elems(ilog2(grid->nx), ilog2(grid->ny), (int)cs) * cs;
  return SIM_OK;
}

sim_status sim_prepare_spectrum(sim_ctx* ctx, const sim_grid* grid, const void* spec0,
                                void* prepared, void* stream) {
  if (!ctx) return SIM_ERR_ARG;
  sim_status s = check_grid(ctx, grid);
  if (s != SIM_OK) return s;
  if (!spec0 || !prepared || ((uintptr_t)prepared & 15) != 0) return SIM_ERR_ARG;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  GridP gp;
  fill_grid(grid, gp);
  hipStream_t st = (hipStream_t)stream;
  ProfScope p(ctx, SIM_KERNEL_PREPARE, st);
  return ctx->prec == SIM_PREC_FP64
             ? dev(simk::launch_prepare_spectrum<double>(spec0, prepared, gp, st))
             : dev(simk::launch_prepare_spectrum<float>(spec0, prepared, gp, st));
}

sim_status sim_range_doppler_accumulate(sim_ctx* ctx, const sim_grid* grid,
                                        const sim_facets* facets, const sim_radar* radar,
                                        double t, int32_t j, void* t_fast, int32_t n_spec,
                                        sim_counters* counters, int32_t* facet_code,
                                        void* stream) {
  WsLayout L;
  sim_status s = common_checks(ctx, grid, radar, &L);
  if (s != SIM_OK) return s;
  if (!facets_ok(facets) || !t_fast || !isfin(t)) return SIM_ERR_ARG;
  if (n_spec < 1 || j < 0 || j >= n_spec) return SIM_ERR_SHAPE;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (ctx->prec == SIM_PREC_FP64)
    return accumulate_facets<double>(ctx, grid, facets, radar, t, j, t_fast, counters, facet_code,
                                     st, L);
  return accumulate_facets<float>(ctx, grid, facets, radar, t, j, t_fast, counters, facet_code,
                                  st, L);
}

sim_status sim_range_doppler_accumulate_noalloc(sim_ctx* ctx, const sim_grid* grid,
                                                const sim_facets* facets,
                                                const sim_radar* radar, double t, int32_t j,
                                                void* t_fast, int32_t n_spec,
                                                sim_counters* counters, int32_t* facet_code,
                                                void* stream) {
  if (!ctx) return SIM_ERR_ARG;
  sim_status s = check_grid(ctx, grid);
  if (s != SIM_OK) return s;
  s = check_radar(radar);
  if (s != SIM_OK) return s;
  if (!facets_ok(facets) || !t_fast || !isfin(t)) return SIM_ERR_ARG;
  if (n_spec < 1 || j < 0 || j >= n_spec) return SIM_ERR_SHAPE;
  const size_t cs = csize(ctx);
  const int wk = window_bins(radar->n_gates, radar->n_doppler, cs, 0);
  if (wk < 1) return SIM_ERR_UNSUPPORTED;
  // the windows of this call must fit the scratch (every supported size does)
  const int nb = acc_band_count((size_t)grid->nx * grid->ny, kNoAllocBands);
  if (nb > kNoAllocBands ||
      (size_t)nb * kSlots * radar->n_gates * (size_t)wk * cs > kNoAllocWinBytes)
    return SIM_ERR_WORKSPACE;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  char* base = (char*)g_dev[ctx->device].scratch;
  if (!base) return SIM_ERR_DEVICE;
  WsLayout L;
  std::memset(&L, 0, sizeof(L));
  L.part = 0;
  L.hdr = kNoAllocHdrOff;
  L.bandcnt = kNoAllocCntOff;
  hipStream_t st = (hipStream_t)stream;
  if (ctx->prec == SIM_PREC_FP64)
    return accumulate_facets<double>(ctx, grid, facets, radar, t, j, t_fast, counters,
                                     facet_code, st, L, base, kNoAllocBands);
  return accumulate_facets<float>(ctx, grid, facets, radar, t, j, t_fast, counters, facet_code,
                                  st, L, base, kNoAllocBands);
}

sim_status sim_update_and_accumulate(sim_ctx* ctx, const sim_grid* grid, const void* spec0,
                                     const sim_radar* radar, double t, int32_t j, void* t_fast,
                                     int32_t n_spec, sim_counters* counters,
                                     int32_t* facet_code, void* stream) {
  return update_and_accumulate_impl(ctx, grid, spec0, false, radar, t, j, t_fast, n_spec,
                                    counters, facet_code, stream);
}

sim_status sim_update_and_accumulate_prepared(sim_ctx* ctx, const sim_grid* grid,
                                              const void* prepared, const sim_radar* radar,
                                              double t, int32_t j, void* t_fast, int32_t n_spec,
                                              sim_counters* counters, int32_t* facet_code,
                                              void* stream) {
  return update_and_accumulate_impl(ctx, grid, prepared, true, radar, t, j, t_fast, n_spec,
                                    counters, facet_code, stream);
}

sim_status sim_run_updates(sim_ctx* ctx, const sim_grid* grid, const void* prepared,
                           const sim_radar* radar, int32_t j0, int32_t count,
                           const double* times, void* t_fast, int32_t n_spec,
                           sim_counters* counters, void* stream) {
  WsLayout L;
  sim_status s = common_checks(ctx, grid, radar, &L);
  if (s != SIM_OK) return s;
  if (!prepared || !t_fast || !times) return SIM_ERR_ARG;
  if (count < 1 || j0 < 0 || n_spec < 1 || j0 > n_spec - count) return SIM_ERR_SHAPE;
  if (!times_ok(times, count)) return SIM_ERR_ARG;
  // update j0 + i on lane i mod lanes with that lane's workspace slice;
  // updates write distinct spectra, the counters are added atomically
  return run_on_lanes(ctx, count, align256(L.total), (hipStream_t)stream,
                      [&](int32_t i, hipStream_t ls) {
                        return update_and_accumulate_impl(ctx, grid, prepared, true, radar,
                                                          times[i], j0 + i, t_fast, n_spec,
                                                          counters, nullptr, ls);
                      });
}

sim_status sim_range_doppler_accumulate_run(sim_ctx* ctx, const sim_grid* grid,
                                            const sim_facets* facets, const sim_radar* radar,
                                            int32_t j0, int32_t count, const double* times,
                                            void* t_fast, int32_t n_spec,
                                            sim_counters* counters, void* stream) {
  WsLayout L;
  sim_status s = common_checks(ctx, grid, radar, &L);
  if (s != SIM_OK) return s;
  if (!facets_ok(facets) || !t_fast || !times) return SIM_ERR_ARG;
  if (count < 1 || j0 < 0 || n_spec < 1 || j0 > n_spec - count) return SIM_ERR_SHAPE;
  if (!times_ok(times, count)) return SIM_ERR_ARG;
  const size_t field = (size_t)grid->nx * grid->ny * (csize(ctx) / 2);
  return run_on_lanes(ctx, count, align256(L.total), (hipStream_t)stream,
                      [&](int32_t i, hipStream_t ls) {
                        const sim_facets fi = stacked_facets(*facets, i, field);
                        return sim_range_doppler_accumulate(ctx, grid, &fi, radar, times[i],
                                                            j0 + i, t_fast, n_spec, counters,
                                                            nullptr, ls);
                      });
}

sim_status sim_segments_to_iq(sim_ctx* ctx, const sim_radar* radar, const void* t_fast,
                              int32_t n_spec, void* y, void* stream) {
  if (!ctx) return SIM_ERR_ARG;
  sim_status s = check_radar(radar);
  if (s != SIM_OK) return s;
  if (!t_fast || !y) return SIM_ERR_ARG;
  if (n_spec < 2) return SIM_ERR_SHAPE;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  const size_t cs = csize(ctx);
  const int N = radar->n_doppler;
  long gb = (long)(kLdsBudget / (4 * (size_t)N * cs));
  if (gb < 1) return SIM_ERR_UNSUPPORTED;
  if (gb > 64) gb = 64;
  if (gb > radar->n_gates) gb = radar->n_gates;
  hipStream_t st = (hipStream_t)stream;
  ProfScope p(ctx, SIM_KERNEL_SEGMENTS_TO_IQ, st);
  if (ctx->prec == SIM_PREC_FP64)
    return dev(simk::launch_segments_to_iq<double>(t_fast, y, radar->n_gates, N, ilog2(N),
                                                   radar->n_fast, radar->window, n_spec - 1,
                                                   (int)gb, ctx->tw, st));
  return dev(simk::launch_segments_to_iq<float>(t_fast, y, radar->n_gates, N, ilog2(N),
                                                radar->n_fast, radar->window, n_spec - 1, (int)gb,
                                                ctx->tw, st));
}

sim_status sim_waveform_loss(sim_ctx* ctx, const sim_radar* radar, const void* y,
                             int32_t n_pulses, const void* target, void* p, void* loss,
                             void* stream) {
  if (!ctx) return SIM_ERR_ARG;
  sim_status s = check_radar(radar);
  if (s != SIM_OK) return s;
  if (!y || !p || (loss && !target)) return SIM_ERR_ARG;
  if (n_pulses < 1) return SIM_ERR_SHAPE;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  ProfScope pf(ctx, SIM_KERNEL_ADJOINT, st);
  if (ctx->prec == SIM_PREC_FP64)
    return dev(simk::launch_waveform_loss<double>(y, n_pulses, radar->n_gates, target, p, loss, st));
  return dev(simk::launch_waveform_loss<float>(y, n_pulses, radar->n_gates, target, p, loss, st));
}

sim_status sim_waveform_loss_adjoint(sim_ctx* ctx, const sim_radar* radar, const void* y,
                                     int32_t n_pulses, const void* p, const void* target,
                                     const void* scale, void* y_bar, void* stream) {
  if (!ctx) return SIM_ERR_ARG;
  sim_status s = check_radar(radar);
  if (s != SIM_OK) return s;
  if (!y || !p || !target || !y_bar) return SIM_ERR_ARG;
  if (n_pulses < 1) return SIM_ERR_SHAPE;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  ProfScope pf(ctx, SIM_KERNEL_ADJOINT, st);
  if (ctx->prec == SIM_PREC_FP64)
    return dev(simk::launch_waveform_loss_adjoint<double>(y, p, target, scale, n_pulses,
                                                          radar->n_gates, y_bar, st));
  return dev(simk::launch_waveform_loss_adjoint<float>(y, p, target, scale, n_pulses,
                                                       radar->n_gates, y_bar, st));
}

sim_status sim_segments_to_iq_adjoint(sim_ctx* ctx, const sim_radar* radar, const void* y_bar,
                                      int32_t n_spec, void* t_fast_bar, void* stream) {
  if (!ctx) return SIM_ERR_ARG;
  sim_status s = check_radar(radar);
  if (s != SIM_OK) return s;
  if (!y_bar || !t_fast_bar) return SIM_ERR_ARG;
  if (n_spec < 2) return SIM_ERR_SHAPE;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  const size_t cs = csize(ctx);
  const int N = radar->n_doppler;
  long gb = (long)(kLdsBudget / (2 * (size_t)N * cs));
  if (gb < 1) return SIM_ERR_UNSUPPORTED;
  if (gb > 64) gb = 64;
  if (gb > radar->n_gates) gb = radar->n_gates;
  const int n_pulses = (n_spec - 1) * radar->n_fast;
  hipStream_t st = (hipStream_t)stream;
  ProfScope pf(ctx, SIM_KERNEL_ADJOINT, st);
  if (ctx->prec == SIM_PREC_FP64)
    return dev(simk::launch_segments_to_iq_adjoint<double>(y_bar, t_fast_bar, radar->n_gates, N,
                                                           radar->n_fast, n_pulses, radar->window,
                                                           n_spec, (int)gb, ctx->tw, st));
  return dev(simk::launch_segments_to_iq_adjoint<float>(y_bar, t_fast_bar, radar->n_gates, N,
                                                        radar->n_fast, n_pulses, radar->window,
                                                        n_spec, (int)gb, ctx->tw, st));
}

sim_status sim_range_doppler_accumulate_adjoint(sim_ctx* ctx, const sim_grid* grid,
                                                const sim_facets* facets,
                                                const sim_radar* radar, double t, int32_t j,
                                                const void* t_fast_bar, int32_t n_spec,
                                                void* grad_h, void* grad_sx, void* grad_sy,
                                                void* stream) {
  if (ctx && ctx->tab_slot >= 0) return SIM_ERR_UNSUPPORTED;   // closed forms only
  if (!ctx) return SIM_ERR_ARG;
  sim_status s = check_grid(ctx, grid);
  if (s != SIM_OK) return s;
  s = check_radar(radar);
  if (s != SIM_OK) return s;
  if (!facets_ok(facets) || !t_fast_bar || !grad_h || !grad_sx || !grad_sy || !isfin(t))
    return SIM_ERR_ARG;
  if (n_spec < 1 || j < 0 || j >= n_spec) return SIM_ERR_SHAPE;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  GridP gp;
  RadarP rp;
  fill_grid(grid, gp);
  fill_radar(radar, grid, t, rp);
  void* const fp[9] = {facets->disp_x, facets->disp_y, facets->h, facets->sx, facets->sy,
                       facets->jac, facets->ddisp_x, facets->ddisp_y, facets->dh};
  const size_t cs = csize(ctx);
  const void* Tj = (const char*)t_fast_bar + (size_t)j * radar->n_gates * radar->n_doppler * cs;
  hipStream_t st = (hipStream_t)stream;
  ProfScope pf(ctx, SIM_KERNEL_ADJOINT, st);
  if (ctx->prec == SIM_PREC_FP64)
    return dev(simk::launch_accumulate_adjoint<double>(fp, gp, rp, Tj, grad_h, grad_sx, grad_sy,
                                                       st));
  return dev(simk::launch_accumulate_adjoint<float>(fp, gp, rp, Tj, grad_h, grad_sx, grad_sy, st));
}

sim_status sim_range_doppler_accumulate_adjoint_run(sim_ctx* ctx, const sim_grid* grid,
                                                    const sim_facets* facets,
                                                    const sim_radar* radar, int32_t j0,
                                                    int32_t count, const double* times,
                                                    const void* t_fast_bar, int32_t n_spec,
                                                    void* grad_h, void* grad_sx, void* grad_sy,
                                                    void* stream) {
  if (ctx && ctx->tab_slot >= 0) return SIM_ERR_UNSUPPORTED;   // closed forms only
  if (!ctx) return SIM_ERR_ARG;
  sim_status s = check_grid(ctx, grid);
  if (s != SIM_OK) return s;
  s = check_radar(radar);
  if (s != SIM_OK) return s;
  if (!facets_ok(facets) || !t_fast_bar || !grad_h || !grad_sx || !grad_sy || !times)
    return SIM_ERR_ARG;
  if (count < 1 || j0 < 0 || n_spec < 1 || j0 > n_spec - count) return SIM_ERR_SHAPE;
  if (!times_ok(times, count)) return SIM_ERR_ARG;
  const size_t field = (size_t)grid->nx * grid->ny * (csize(ctx) / 2);
  // a per-facet gather into distinct gradient slices: no workspace
  return run_on_lanes(ctx, count, 0, (hipStream_t)stream, [&](int32_t i, hipStream_t ls) {
    const sim_facets fi = stacked_facets(*facets, i, field);
    const size_t o = (size_t)i * field;
    return sim_range_doppler_accumulate_adjoint(ctx, grid, &fi, radar, times[i], j0 + i,
                                                t_fast_bar, n_spec, (char*)grad_h + o,
                                                (char*)grad_sx + o, (char*)grad_sy + o, ls);
  });
}

sim_status sim_delay_doppler(sim_ctx* ctx, const sim_radar* radar, const void* y,
                             int32_t n_pulses, const sim_dd_params* params, void* beams,
                             void* centroid, void* beam_power, void* waveform, void* stream) {
  if (!ctx || !params) return SIM_ERR_ARG;
  sim_status s = check_radar(radar);
  if (s != SIM_OK) return s;
  const int M = params->burst, G = radar->n_gates;
  if (!is_pow2(M) || M < 2 || M > 256 || !is_pow2(G) || G < 2 || G > 2048)
    return SIM_ERR_UNSUPPORTED;
  if (n_pulses < M) return SIM_ERR_SHAPE;
  if (params->centroid_mode != SIM_DD_CENTROID_GIVEN &&
      params->centroid_mode != SIM_DD_CENTROID_ESTIMATE)
    return SIM_ERR_ARG;
  if (!isfin(params->centroid)) return SIM_ERR_ARG;
  if (params->migration && radar->velocity == 0.0) return SIM_ERR_ARG;
  if (!y || !beams || !centroid || !beam_power || !waveform) return SIM_ERR_ARG;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  const int nb = n_pulses / M;
  // range migration per squared beam Doppler (cycles per pulse), in gates
  double mig = 0.0;
  if (params->migration) {
    const double lam = 299792458.0 / radar->carrier_hz;
    const double a = radar->prf_hz * lam * radar->altitude / (2.0 * radar->velocity);
    mig = a * a / (2.0 * radar->altitude * radar->gate_spacing);
  }
  hipStream_t st = (hipStream_t)stream;
  ProfScope p(ctx, SIM_KERNEL_DELAY_DOPPLER, st);
  if (ctx->prec == SIM_PREC_FP64)
    return dev(simk::launch_delay_doppler<double>(
        y, G, M, nb, params->centroid_mode, params->centroid, mig, params->migration, beams,
        centroid, beam_power, waveform, ctx->tw, st));
  return dev(simk::launch_delay_doppler<float>(
      y, G, M, nb, params->centroid_mode, params->centroid, mig, params->migration, beams,
      centroid, beam_power, waveform, ctx->tw, st));
}

sim_status sim_set_tables(sim_ctx* ctx, const sim_tables* t) {
  if (!ctx) return SIM_ERR_ARG;
  if (!t || (!t->antenna && !t->nrcs)) {
    release_tab_slot(ctx);
    return SIM_OK;
  }
  if (t->antenna && !(t->nu >= 2 && t->nv >= 2 && isfin(t->u0) && isfin(t->v0) &&
                      isfin(t->du) && t->du > 0 && isfin(t->dv) && t->dv > 0))
    return SIM_ERR_ARG;
  if (t->nrcs && !(t->n_theta >= 2 && isfin(t->dtheta) && t->dtheta > 0)) return SIM_ERR_ARG;
  sim_status s = use_device(ctx);
  if (s != SIM_OK) return s;
  DeviceState& d = g_dev[ctx->device];
  if (ctx->tab_slot < 0) {
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    for (int i = 0; i < kTabSlots; ++i) {
      if (!d.tab_used[i]) {
        d.tab_used[i] = true;
        ctx->tab_slot = i;
        break;
      }
    }
    if (ctx->tab_slot < 0) return SIM_ERR_UNSUPPORTED;
  }
  simk::TabP p;
  std::memset(&p, 0, sizeof(p));
  p.ant = t->antenna;
  p.nrcs = t->nrcs;
  p.nu = t->antenna ? t->nu : 0;
  p.nv = t->antenna ? t->nv : 0;
  p.n_theta = t->nrcs ? t->n_theta : 0;
  p.u0 = t->u0;
  p.v0 = t->v0;
  p.inv_du = t->antenna ? 1.0 / t->du : 0.0;
  p.inv_dv = t->antenna ? 1.0 / t->dv : 0.0;
  p.inv_dtheta = t->nrcs ? 1.0 / t->dtheta : 0.0;
  // no kernel of this device may read the block while it changes
  s = dev(hipDeviceSynchronize());
  if (s != SIM_OK) return s;
  return dev(hipMemcpy(d.tabs + ctx->tab_slot, &p, sizeof(p), hipMemcpyHostToDevice));
}

sim_status sim_set_tuning(sim_ctx* ctx, int key, int value) {
  if (!ctx) return SIM_ERR_ARG;
  if (key == SIM_TUNE_ROW_BANDS) {
    if (value < 0 || value > kMaxBands || (value & (value - 1)) != 0) return SIM_ERR_ARG;
    ctx->row_bands = value;
    return SIM_OK;
  }
  if (key == SIM_TUNE_ROW_PATH) {
    if (value != SIM_ROW_PATH_AUTO && value != SIM_ROW_PATH_FUSED && value != SIM_ROW_PATH_SPLIT)
      return SIM_ERR_ARG;
    ctx->row_path = value;
    return SIM_OK;
  }
  if (key == SIM_TUNE_ACC_BANDS) {
    if (value < 0 || value > kAccBands || (value & (value - 1)) != 0 ||
        (value > 0 && value < 64))
      return SIM_ERR_ARG;
    ctx->acc_bands = value;
    return SIM_OK;
  }
  if (key == SIM_TUNE_UPDATE_LANES) {
    if (value < 1 || value > kMaxUpdateLanes) return SIM_ERR_ARG;
    if (value == ctx->lanes) return SIM_OK;
    sim_status s = use_device(ctx);
    if (s != SIM_OK) return s;
    release_lanes(ctx);
    bool ok = true;
    for (int l = 1; l < value && ok; ++l) {
      hipStream_t st = nullptr;
      ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
      if (ok) ctx->lane_st.push_back(st);
    }
    for (int i = 0; i < value && ok; ++i) {
      hipEvent_t e = nullptr;
      ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
      if (ok) ctx->lane_ev.push_back(e);
    }
    if (!ok) {
      (void)hipGetLastError();
      release_lanes(ctx);
      return SIM_ERR_DEVICE;
    }
    ctx->lanes = value;
    return SIM_OK;
  }
  return SIM_ERR_ARG;
}

sim_status sim_profile_enable(sim_ctx* ctx, int enable) {
  if (!ctx) return SIM_ERR_ARG;
  if (enable && ctx->ev.empty()) {
    sim_status s = use_device(ctx);
    if (s != SIM_OK) return s;
    ctx->ev.reserve(2 * (size_t)kProfilePairs);
    for (int i = 0; i < 2 * kProfilePairs; ++i) {
      hipEvent_t e;
      s = dev(hipEventCreate(&e));
      if (s != SIM_OK) {
        for (hipEvent_t x : ctx->ev) (void)hipEventDestroy(x);
        ctx->ev.clear();
        return s;
      }
      ctx->ev.push_back(e);
    }
    ctx->kind.assign(kProfilePairs, 0);
  }
  ctx->profiling = enable != 0;
  if (enable) {
    ctx->used = 0;
    ctx->dropped = 0;
  }
  return SIM_OK;
}

sim_status sim_profile_read(sim_ctx* ctx, sim_kernel_times* out) {
  if (!ctx || !out) return SIM_ERR_ARG;
  for (int k = 0; k < SIM_KERNEL_KINDS; ++k) {
    out->ms[k] = 0.0;
    out->launches[k] = 0;
  }
  out->dropped = ctx->dropped;
  if (ctx->used == 0) return SIM_OK;
  sim_status s = use_device(ctx);
  if (s != SIM_OK) return s;
  for (size_t i = 0; i < ctx->used; ++i) {
    s = dev(hipEventSynchronize(ctx->ev[2 * i + 1]));
    if (s != SIM_OK) return s;
    float ms = 0.f;
    s = dev(hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]));
    if (s != SIM_OK) return s;
    out->ms[ctx->kind[i]] += (double)ms;
    out->launches[ctx->kind[i]] += 1;
  }
  return SIM_OK;
}

}  // extern "C"

// Members run on up to kBatchLanes streams ("lanes") at once, each lane with
// its own slice of the workspace, so that the launches of small grids, which
// do not fill the GPU, overlap with the others.  Members are dealt to lanes
// largest first, each to the lane with the least work so far.
constexpr int kBatchLanes = 4;

struct sim_batch {
  sim_ctx* ctx;
  std::vector<sim_grid> grids;
  std::vector<sim_radar> radars;
  std::vector<int32_t> updates;
  std::vector<size_t> prep_off;   // prepared spectrum of each member in the workspace
  std::vector<int> lane_of;       // lane of each member
  std::vector<size_t> lane_off, lane_bytes;   // workspace slice of each lane
  std::vector<hipStream_t> lane_st;
  std::vector<hipEvent_t> lane_ev;            // join events
  hipEvent_t fork_ev;
  size_t ws_bytes;
  // captured graph and the pointers it was captured with
  hipGraphExec_t exec;
  bool have_graph;
  std::vector<void*> key;
  hipStream_t graph_stream;
  // persistent mode: members grouped by shape (grid sides, gates, bins);
  // each member's workspace slice; the per-update descriptors of every
  // class and the work counters of every launch in the workspace
  int mode;                                   // SIM_BATCH_*
  std::vector<std::vector<int>> classes;      // member indices per class
  std::vector<size_t> member_off;             // workspace slice of each member
  size_t desc_off, queue_off;
  std::vector<simk::BatchMember> desc;        // host copy, [update][member of class order]
  std::vector<size_t> desc_at;                // first descriptor of (update, class)
  std::vector<int> desc_n;                    // active members of (update, class)
  std::vector<void*> desc_key;                // pointers the descriptors were built for
  int jmax;
  std::vector<int> m_row_path, m_row_bands, m_acc_bands;   // per-member tuning (lanes mode)
};

namespace {

template <typename Real>
void build_descriptors(sim_batch* b, void* const* t_fast) {
  sim_ctx* c = b->ctx;
  const size_t cs = sizeof(Real) * 2;
  const int nc = (int)b->classes.size();
  b->desc.clear();
  b->desc_at.assign((size_t)(b->jmax + 1) * nc, 0);
  b->desc_n.assign((size_t)(b->jmax + 1) * nc, 0);
  for (int j = 0; j <= b->jmax; ++j) {
    for (int k = 0; k < nc; ++k) {
      b->desc_at[(size_t)j * nc + k] = b->desc.size();
      for (int r : b->classes[k]) {
        if (j > b->updates[r]) continue;
        const sim_grid* g = &b->grids[r];
        const sim_radar* rr = &b->radars[r];
        const WsLayout L = ws_layout(g, rr, cs);
        char* base = (char*)c->ws + b->member_off[r];
        const double t = ((double)j * rr->n_fast) / rr->prf_hz;
        simk::BatchMember m;
        std::memset(&m, 0, sizeof(m));
        GridP gp;
        fill_grid(g, gp);
        m.gp = simk::grid_with_tiles<Real>(gp);
        fill_radar(rr, g, t, m.rp, ctx_tab(c));
        const size_t P = (size_t)g->nx * g->ny;
        const int wk = window_bins(rr->n_gates, rr->n_doppler, cs, 0);
        m.wp = win_params(base, rr, L, wk, acc_band_count(P, kAccBands),
                          (int)acc_band_size(P, kAccBands));
        m.spec = (char*)c->ws + b->prep_off[r];
        m.planes = base + L.planes;
        for (int i = 0; i < 9; ++i) m.fac[i] = base + L.facets + (size_t)i * L.facet_stride;
        m.Tj = (char*)t_fast[r] + (size_t)j * rr->n_gates * rr->n_doppler * cs;
        m.t = t;
        m.dt = 1.0 / rr->prf_hz;
        b->desc.push_back(m);
        b->desc_n[(size_t)j * nc + k]++;
      }
    }
  }
}

// Persistent mode: every update j runs, per class, the four phases of the
// split row path as four persistent launches over all members of the class.
template <typename Real>
sim_status persistent_updates(sim_batch* b, hipStream_t st) {
  sim_ctx* c = b->ctx;
  const size_t cs = sizeof(Real) * 2;
  const int nc = (int)b->classes.size();
  const simk::BatchMember* dev_desc = (const simk::BatchMember*)((char*)c->ws + b->desc_off);
  int* queues = (int*)((char*)c->ws + b->queue_off);
  sim_status s = dev(simk::launch_clear(queues, (size_t)(b->jmax + 1) * nc * 4 * sizeof(int), st));
  for (int j = 0; j <= b->jmax && s == SIM_OK; ++j) {
    for (int k = 0; k < nc && s == SIM_OK; ++k) {
      const size_t at = b->desc_at[(size_t)j * nc + k];
      const int n = b->desc_n[(size_t)j * nc + k];
      if (n == 0) continue;
      const simk::BatchMember& m0 = b->desc[at];
      const int r0 = b->classes[k][0];
      const int wk = window_bins(b->radars[r0].n_gates, b->radars[r0].n_doppler, cs, 0);
      const size_t acc_lds = (size_t)b->radars[r0].n_gates * wk * cs + simk::kWinCtxBytes;
      ProfScope p(c, SIM_KERNEL_BATCHED_UPDATE, st);
      s = dev(simk::launch_update_batched<Real>(dev_desc + at, n, m0.gp, m0.rp, m0.wp, acc_lds,
                                                queues + 4 * ((size_t)j * nc + k), c->tw, st));
    }
  }
  return s;
}

sim_status batch_enqueue_persistent(sim_batch* b, void* const* spec0, void* const* t_fast,
                                    void* const* y, hipStream_t st) {
  sim_ctx* c = b->ctx;
  const int R = (int)b->grids.size();
  const size_t cs = csize(c);
  for (int r = 0; r < R; ++r) {
    const sim_radar& rr = b->radars[r];
    const size_t n = (size_t)(b->updates[r] + 1) * rr.n_gates * rr.n_doppler;
    ProfScope p(c, SIM_KERNEL_PREPARE, st);
    const sim_status s = dev(simk::launch_clear(t_fast[r], n * cs, st));
    if (s != SIM_OK) return s;
  }
  for (int r = 0; r < R; ++r) {
    const sim_status s = sim_prepare_spectrum(c, &b->grids[r], spec0[r],
                                              (char*)c->ws + b->prep_off[r], st);
    if (s != SIM_OK) return s;
  }
  sim_status s = c->prec == SIM_PREC_FP64 ? persistent_updates<double>(b, st)
                                          : persistent_updates<float>(b, st);
  for (int r = 0; r < R && s == SIM_OK && y; ++r) {
    if (!y[r]) continue;
    s = sim_segments_to_iq(c, &b->radars[r], t_fast[r], b->updates[r] + 1, y[r], st);
  }
  return s;
}

// The descriptors depend on the output pointers: rebuilt and uploaded when
// they change (after the stream has drained, so that no queued launch still
// reads the old ones).
sim_status batch_prepare_descriptors(sim_batch* b, void* const* t_fast, hipStream_t st) {
  std::vector<void*> key(t_fast, t_fast + b->grids.size());
  key.push_back(b->ctx->ws);
  if (key == b->desc_key && !b->desc.empty()) return SIM_OK;
  if (b->ctx->prec == SIM_PREC_FP64)
    build_descriptors<double>(b, t_fast);
  else
    build_descriptors<float>(b, t_fast);
  sim_status s = dev(hipStreamSynchronize(st));
  if (s != SIM_OK) return s;
  s = dev(hipMemcpy((char*)b->ctx->ws + b->desc_off, b->desc.data(),
                    b->desc.size() * sizeof(simk::BatchMember), hipMemcpyHostToDevice));
  if (s == SIM_OK) b->desc_key = key;
  return s;
}

sim_status batch_enqueue(sim_batch* b, void* const* spec0, void* const* t_fast, void* const* y,
                         hipStream_t st) {
  sim_ctx* c = b->ctx;
  const int R = (int)b->grids.size();
  const size_t cs = csize(c);
  int jmax = 0;
  for (int r = 0; r < R; ++r) jmax = b->updates[r] > jmax ? b->updates[r] : jmax;
  for (int r = 0; r < R; ++r) {
    const sim_radar& rr = b->radars[r];
    const size_t n = (size_t)(b->updates[r] + 1) * rr.n_gates * rr.n_doppler;
    ProfScope p(c, SIM_KERNEL_PREPARE, st);
    const sim_status s = dev(simk::launch_clear(t_fast[r], n * cs, st));
    if (s != SIM_OK) return s;
  }
  // each member's spectrum in the column-pass layout, once per run
  for (int r = 0; r < R; ++r) {
    const sim_status s = sim_prepare_spectrum(c, &b->grids[r], spec0[r],
                                              (char*)c->ws + b->prep_off[r], st);
    if (s != SIM_OK) return s;
  }
  // fork the lanes off the caller's stream (also under graph capture), run
  // each lane's members update-major on its stream with its workspace slice,
  // and join them back
  const int NL = (int)b->lane_st.size();
  sim_status s = dev(hipEventRecord(b->fork_ev, st));
  if (s != SIM_OK) return s;
  for (int l = 0; l < NL; ++l) {
    s = dev(hipStreamWaitEvent(b->lane_st[l], b->fork_ev, 0));
    if (s != SIM_OK) return s;
  }
  sim_status first = SIM_OK;
  for (int l = 0; l < NL && first == SIM_OK; ++l) {
    sim_ctx lc;                 // same device, twiddles and tuning, the lane's workspace
    lc.device = c->device;
    lc.prec = c->prec;
    lc.tw = c->tw;
    lc.ws = (char*)c->ws + b->lane_off[l];
    lc.ws_bytes = b->lane_bytes[l];
    lc.row_bands = c->row_bands;
    lc.row_path = c->row_path;
    lc.acc_bands = c->acc_bands;
    lc.capturing = c->capturing;
    lc.tab_slot = c->tab_slot;
    lc.lanes = 1;
    lc.profiling = false;
    lc.used = 0;
    lc.dropped = 0;
    hipStream_t ls = b->lane_st[l];
    for (int j = 0; j <= jmax && first == SIM_OK; ++j) {
      for (int r = 0; r < R; ++r) {
        if (b->lane_of[r] != l || j > b->updates[r]) continue;
        const sim_radar& rr = b->radars[r];
        const double t = ((double)j * rr.n_fast) / rr.prf_hz;
        lc.row_path = b->m_row_path[r] >= 0 ? b->m_row_path[r] : c->row_path;
        lc.row_bands = b->m_row_bands[r] >= 0 ? b->m_row_bands[r] : c->row_bands;
        lc.acc_bands = b->m_acc_bands[r] >= 0 ? b->m_acc_bands[r] : c->acc_bands;
        first = sim_update_and_accumulate_prepared(
            &lc, &b->grids[r], (char*)c->ws + b->prep_off[r], &rr, t, j, t_fast[r],
            b->updates[r] + 1, nullptr, nullptr, ls);
        if (first != SIM_OK) break;
      }
    }
    for (int r = 0; r < R && first == SIM_OK && y; ++r) {
      if (b->lane_of[r] != l || !y[r]) continue;
      first = sim_segments_to_iq(&lc, &b->radars[r], t_fast[r], b->updates[r] + 1, y[r], ls);
    }
  }
  // always join, so that a capture stays well formed
  for (int l = 0; l < NL; ++l) {
    s = dev(hipEventRecord(b->lane_ev[l], b->lane_st[l]));
    if (s == SIM_OK) s = dev(hipStreamWaitEvent(st, b->lane_ev[l], 0));
    if (s != SIM_OK && first == SIM_OK) first = s;
  }
  return first;
}

}  // namespace

extern "C" {

sim_status sim_batch_create(sim_ctx* ctx, int32_t n_real, const sim_grid* grids,
                            const sim_radar* radars, const int32_t* n_updates,
                            sim_batch** batch) {
  if (!batch) return SIM_ERR_ARG;
  *batch = nullptr;
  if (!ctx || n_real < 1 || !grids || !radars || !n_updates) return SIM_ERR_ARG;
  size_t ws = 0;
  for (int r = 0; r < n_real; ++r) {
    sim_status s = check_grid(ctx, &grids[r]);
    if (s != SIM_OK) return s;
    s = check_radar(&radars[r]);
    if (s != SIM_OK) return s;
    if (n_updates[r] < 1) return SIM_ERR_SHAPE;
    if (window_bins(radars[r].n_gates, radars[r].n_doppler, csize(ctx), 0) < 1)
      return SIM_ERR_UNSUPPORTED;
    const size_t need = ws_layout(&grids[r], &radars[r], csize(ctx)).total;
    ws = need > ws ? need : ws;
  }
  (void)ws;
  sim_status su = use_device(ctx);
  if (su != SIM_OK) return su;
  sim_batch* b = new (std::nothrow) sim_batch;
  if (!b) return SIM_ERR_DEVICE;
  b->ctx = ctx;
  b->grids.assign(grids, grids + n_real);
  b->radars.assign(radars, radars + n_real);
  b->updates.assign(n_updates, n_updates + n_real);
  // lanes: members largest first, each to the least loaded lane
  const int NL = n_real < kBatchLanes ? n_real : kBatchLanes;
  std::vector<double> load(NL, 0.0);
  std::vector<int> order(n_real);
  for (int r = 0; r < n_real; ++r) order[r] = r;
  auto work = [&](int r) {
    return (double)grids[r].nx * grids[r].ny * (double)(n_updates[r] + 1);
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
  b->lane_of.assign(n_real, 0);
  b->lane_bytes.assign(NL, 0);
  for (int r : order) {
    int best = 0;
    for (int l = 1; l < NL; ++l)
      if (load[l] < load[best]) best = l;
    b->lane_of[r] = best;
    load[best] += work(r);
    const size_t need = ws_layout(&grids[r], &radars[r], csize(ctx)).total;
    if (need > b->lane_bytes[best]) b->lane_bytes[best] = need;
  }
  // workspace: the lanes' slices, then every member's prepared spectrum
  size_t off = 0;
  for (int l = 0; l < NL; ++l) {
    b->lane_off.push_back(off);
    off = align256(off + b->lane_bytes[l]);
  }
  for (int r = 0; r < n_real; ++r) {
    size_t pb = 0;
    (void)sim_prepared_spectrum_size(ctx, &grids[r], &pb);
    b->prep_off.push_back(off);
    off = align256(off + pb);
  }
  // persistent mode: one workspace slice per member (the lanes' slices and
  // these are never in use together), then the descriptors and counters
  b->mode = SIM_BATCH_PERSISTENT;
  b->m_row_path.assign(n_real, -1);
  b->m_row_bands.assign(n_real, -1);
  b->m_acc_bands.assign(n_real, -1);
  b->jmax = 0;
  for (int r = 0; r < n_real; ++r) b->jmax = n_updates[r] > b->jmax ? n_updates[r] : b->jmax;
  for (int r = 0; r < n_real; ++r) {
    bool placed = false;
    for (auto& cl : b->classes) {
      const int q = cl[0];
      if (grids[q].nx == grids[r].nx && grids[q].ny == grids[r].ny &&
          radars[q].n_gates == radars[r].n_gates && radars[q].n_doppler == radars[r].n_doppler) {
        cl.push_back(r);
        placed = true;
        break;
      }
    }
    if (!placed) b->classes.push_back(std::vector<int>(1, r));
  }
  size_t poff = 0;
  for (int r = 0; r < n_real; ++r) {
    b->member_off.push_back(poff);
    poff = align256(poff + ws_layout(&grids[r], &radars[r], csize(ctx)).total);
  }
  // both modes start at offset 0: the prepared spectra move past the larger
  const size_t lanes_end = b->lane_off.empty() ? 0 : b->prep_off[0];
  if (poff > lanes_end) {
    const size_t shift = poff - lanes_end;
    for (size_t& o : b->prep_off) o += shift;
    off += shift;
  }
  b->desc_off = off;
  off = align256(off + (size_t)(b->jmax + 1) * n_real * sizeof(simk::BatchMember));
  b->queue_off = off;
  off = align256(off + (size_t)(b->jmax + 1) * b->classes.size() * 4 * sizeof(int));
  b->ws_bytes = off;
  bool ok = hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) == hipSuccess;
  for (int l = 0; l < NL && ok; ++l) {
    hipStream_t ls;
    hipEvent_t le;
    ok = hipStreamCreateWithFlags(&ls, hipStreamNonBlocking) == hipSuccess;
    if (!ok) break;
    b->lane_st.push_back(ls);
    ok = hipEventCreateWithFlags(&le, hipEventDisableTiming) == hipSuccess;
    if (ok) b->lane_ev.push_back(le);
  }
  if (!ok) {
    for (hipStream_t ls : b->lane_st) (void)hipStreamDestroy(ls);
    for (hipEvent_t le : b->lane_ev) (void)hipEventDestroy(le);
    delete b;
    return SIM_ERR_DEVICE;
  }
  b->have_graph = false;
  b->graph_stream = nullptr;
  *batch = b;
  return SIM_OK;
}

sim_status sim_batch_destroy(sim_batch* b) {
  if (!b) return SIM_OK;
  sim_status s = SIM_OK;
  if (use_device(b->ctx) != SIM_OK) s = SIM_ERR_DEVICE;
  if (b->have_graph && hipGraphExecDestroy(b->exec) != hipSuccess) s = SIM_ERR_DEVICE;
  for (hipStream_t ls : b->lane_st)
    if (hipStreamDestroy(ls) != hipSuccess) s = SIM_ERR_DEVICE;
  for (hipEvent_t le : b->lane_ev)
    if (hipEventDestroy(le) != hipSuccess) s = SIM_ERR_DEVICE;
  if (hipEventDestroy(b->fork_ev) != hipSuccess) s = SIM_ERR_DEVICE;
  delete b;
  return s;
}

sim_status sim_batch_set_mode(sim_batch* b, int mode) {
  if (!b) return SIM_ERR_ARG;
  if (mode != SIM_BATCH_LANES && mode != SIM_BATCH_PERSISTENT) return SIM_ERR_ARG;
  b->mode = mode;
  return SIM_OK;
}

sim_status sim_batch_set_tuning(sim_batch* b, int32_t member, int key, int value) {
  if (!b || member < 0 || member >= (int)b->grids.size()) return SIM_ERR_ARG;
  // a captured graph holds the launches of the old values
  if (b->have_graph) {
    (void)hipGraphExecDestroy(b->exec);
    b->have_graph = false;
  }
  if (key == SIM_TUNE_ROW_PATH) {
    if (value != SIM_ROW_PATH_AUTO && value != SIM_ROW_PATH_FUSED && value != SIM_ROW_PATH_SPLIT)
      return SIM_ERR_ARG;
    b->m_row_path[member] = value;
    return SIM_OK;
  }
  if (key == SIM_TUNE_ROW_BANDS) {
    if (value < 0 || value > kMaxBands || (value > 0 && !is_pow2(value))) return SIM_ERR_ARG;
    b->m_row_bands[member] = value;
    return SIM_OK;
  }
  if (key == SIM_TUNE_ACC_BANDS) {
    if (value < 0 || value > kAccBands || (value > 0 && (!is_pow2(value) || value < 64)))
      return SIM_ERR_ARG;
    b->m_acc_bands[member] = value;
    return SIM_OK;
  }
  return SIM_ERR_ARG;
}

sim_status sim_batch_workspace_size(const sim_batch* b, size_t* bytes) {
  if (!b || !bytes) return SIM_ERR_ARG;
  *bytes = b->ws_bytes;
  return SIM_OK;
}

sim_status sim_batch_run(sim_batch* b, void* const* spec0, void* const* t_fast, void* const* y,
                         int use_graph, void* stream) {
  if (!b || !spec0 || !t_fast) return SIM_ERR_ARG;
  const int R = (int)b->grids.size();
  for (int r = 0; r < R; ++r)
    if (!spec0[r] || !t_fast[r]) return SIM_ERR_ARG;
  sim_ctx* c = b->ctx;
  if (!c->ws) return SIM_ERR_WORKSPACE;
  if (c->ws_bytes < b->ws_bytes) return SIM_ERR_WORKSPACE;
  sim_status s = use_device(c);
  if (s != SIM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const bool pers = b->mode == SIM_BATCH_PERSISTENT;
  if (pers) {
    s = batch_prepare_descriptors(b, t_fast, st);
    if (s != SIM_OK) return s;
  }
  auto enqueue = [&]() {
    return pers ? batch_enqueue_persistent(b, spec0, t_fast, y, st)
                : batch_enqueue(b, spec0, t_fast, y, st);
  };
  if (!use_graph) return enqueue();
  if (!st) return SIM_ERR_ARG;
  std::vector<void*> key;
  key.push_back(c->ws);
  key.push_back((void*)(intptr_t)b->mode);
  for (int r = 0; r < R; ++r) {
    key.push_back(spec0[r]);
    key.push_back(t_fast[r]);
    key.push_back(y ? y[r] : nullptr);
  }
  if (!b->have_graph || key != b->key || b->graph_stream != st) {
    if (b->have_graph) {
      (void)hipGraphExecDestroy(b->exec);
      b->have_graph = false;
    }
    s = dev(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    if (s != SIM_OK) return s;
    c->capturing = true;
    const sim_status se = enqueue();
    c->capturing = false;
    hipGraph_t graph;
    s = dev(hipStreamEndCapture(st, &graph));
    if (se != SIM_OK) {
      if (s == SIM_OK) (void)hipGraphDestroy(graph);
      return se;
    }
    if (s != SIM_OK) return s;
    s = dev(hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    if (s != SIM_OK) return s;
    b->have_graph = true;
    b->key = key;
    b->graph_stream = st;
  }
  return dev(hipGraphLaunch(b->exec, st));
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Out-of-core runs (Sec. III.B, last two paragraphs): T_fast and Y stay in
// host memory and the device holds caches of K spectra.  The paper fills a
// device cache of spectra, copies it to host memory when full, and later
// copies parts of the spectra back to post-process them.  Here each chunk's
// IQ is formed on the device from the cache it has just filled (plus the
// last spectrum of the previous chunk), so no spectrum travels back to the
// device: per chunk of K update intervals, the compute stream fills one of
// two cache buffers and runs the post-processing; a copy stream moves that
// buffer's IQ (and spectra) to host memory while the next chunk computes into
// the other buffer.

struct sim_streamer {
  sim_ctx* ctx;
  sim_radar radar;
  int K;                       // update intervals per chunk
  size_t spec_bytes;           // one spectrum
  size_t cache_bytes;          // one of the two buffers
  hipStream_t copy_st;
  hipEvent_t computed[2], copied[2], done;
};

namespace {

size_t streamer_buffer_bytes(const sim_radar* r, int K, size_t cs) {
  const size_t spec = (size_t)r->n_gates * r->n_doppler * cs;
  const size_t y = (size_t)K * r->n_fast * r->n_gates * cs;
  return align256((size_t)(K + 1) * spec) + align256(y);
}

}  // namespace

extern "C" {

sim_status sim_streamer_destroy(sim_streamer* st);

sim_status sim_streamer_create(sim_ctx* ctx, const sim_radar* radar, int32_t chunk_updates,
                               sim_streamer** out) {
  if (!out) return SIM_ERR_ARG;
  *out = nullptr;
  if (!ctx) return SIM_ERR_ARG;
  sim_status s = check_radar(radar);
  if (s != SIM_OK) return s;
  if (chunk_updates < 1) return SIM_ERR_SHAPE;
  s = use_device(ctx);
  if (s != SIM_OK) return s;
  sim_streamer* st = new (std::nothrow) sim_streamer;
  if (!st) return SIM_ERR_DEVICE;
  st->ctx = ctx;
  st->radar = *radar;
  st->K = chunk_updates;
  st->spec_bytes = (size_t)radar->n_gates * radar->n_doppler * csize(ctx);
  st->cache_bytes = streamer_buffer_bytes(radar, chunk_updates, csize(ctx));
  // every handle starts null so that a partial set-up can be released
  st->copy_st = nullptr;
  st->done = nullptr;
  for (int b = 0; b < 2; ++b) st->computed[b] = st->copied[b] = nullptr;
  bool ok = hipStreamCreateWithFlags(&st->copy_st, hipStreamNonBlocking) == hipSuccess;
  for (int b = 0; b < 2 && ok; ++b) {
    ok = hipEventCreateWithFlags(&st->computed[b], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&st->copied[b], hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipEventCreateWithFlags(&st->done, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    (void)sim_streamer_destroy(st);
    return SIM_ERR_DEVICE;
  }
  *out = st;
  return SIM_OK;
}

sim_status sim_streamer_destroy(sim_streamer* st) {
  if (!st) return SIM_OK;
  sim_status s = use_device(st->ctx);
  if (st->copy_st) {
    if (hipStreamSynchronize(st->copy_st) != hipSuccess) s = SIM_ERR_DEVICE;
    if (hipStreamDestroy(st->copy_st) != hipSuccess) s = SIM_ERR_DEVICE;
  }
  for (int b = 0; b < 2; ++b) {
    if (st->computed[b] && hipEventDestroy(st->computed[b]) != hipSuccess) s = SIM_ERR_DEVICE;
    if (st->copied[b] && hipEventDestroy(st->copied[b]) != hipSuccess) s = SIM_ERR_DEVICE;
  }
  if (st->done && hipEventDestroy(st->done) != hipSuccess) s = SIM_ERR_DEVICE;
  delete st;
  return s;
}

sim_status sim_streamer_cache_size(const sim_streamer* st, size_t* bytes) {
  if (!st || !bytes) return SIM_ERR_ARG;
  *bytes = 2 * st->cache_bytes;
  return SIM_OK;
}

sim_status sim_streamer_run(sim_streamer* st, const sim_grid* grid, const void* prepared,
                            int32_t n_updates, void* t_fast_host, void* y_host, void* cache,
                            size_t cache_bytes, void* stream) {
  if (!st) return SIM_ERR_ARG;
  sim_ctx* c = st->ctx;
  const sim_radar* r = &st->radar;
  WsLayout L;
  sim_status s = common_checks(c, grid, r, &L);
  if (s != SIM_OK) return s;
  if (!prepared || !y_host || !cache) return SIM_ERR_ARG;
  if (((uintptr_t)cache & 255) != 0) return SIM_ERR_ARG;
  if (n_updates < 1) return SIM_ERR_SHAPE;
  if (cache_bytes < 2 * st->cache_bytes) return SIM_ERR_WORKSPACE;
  s = use_device(c);
  if (s != SIM_OK) return s;
  hipStream_t cs_ = (hipStream_t)stream;
  const int K = st->K;
  const size_t spec = st->spec_bytes;
  const size_t y_row = (size_t)r->n_gates * csize(c);        // one pulse
  const size_t y_off = align256((size_t)(K + 1) * spec);
  char* buf[2] = {(char*)cache, (char*)cache + st->cache_bytes};
  // both buffers start free: mark them copied on the copy stream, after
  // everything already queued on the caller's stream
  s = dev(hipEventRecord(st->done, cs_));
  if (s == SIM_OK) s = dev(hipStreamWaitEvent(st->copy_st, st->done, 0));
  for (int b = 0; b < 2 && s == SIM_OK; ++b) s = dev(hipEventRecord(st->copied[b], st->copy_st));
  const int n_chunks = (n_updates + K - 1) / K;
  for (int ch = 0; ch < n_chunks && s == SIM_OK; ++ch) {
    const int b = ch & 1;
    const int j0 = ch * K;                       // first spectrum of the chunk (slot 0)
    const int k = std::min(K, n_updates - j0);   // update intervals (segments) of the chunk
    char* specs = buf[b];
    char* ycache = buf[b] + y_off;
    s = dev(hipStreamWaitEvent(cs_, st->copied[b], 0));
    if (s != SIM_OK) break;
    // slot 0: spectrum j0, computed by the previous chunk (its last slot)
    if (ch == 0) {
      s = dev(simk::launch_clear(specs, spec, cs_));
      if (s == SIM_OK) {
        s = sim_update_and_accumulate_prepared(c, grid, prepared, r, 0.0, 0, specs, 1, nullptr,
                                               nullptr, cs_);
      }
    } else {
      const int kp = std::min(K, n_updates - (j0 - K));
      s = dev(hipMemcpyAsync(specs, buf[b ^ 1] + (size_t)kp * spec, spec,
                             hipMemcpyDeviceToDevice, cs_));
    }
    if (s != SIM_OK) break;
    s = dev(simk::launch_clear(specs + spec, (size_t)k * spec, cs_));
    for (int i = 1; i <= k && s == SIM_OK; ++i) {
      const int j = j0 + i;
      const double t = ((double)j * r->n_fast) / r->prf_hz;
      s = sim_update_and_accumulate_prepared(c, grid, prepared, r, t, i, specs, k + 1, nullptr,
                                             nullptr, cs_);
    }
    if (s == SIM_OK) s = sim_segments_to_iq(c, r, specs, k + 1, ycache, cs_);
    if (s == SIM_OK) s = dev(hipEventRecord(st->computed[b], cs_));
    if (s != SIM_OK) break;
    // copies of this chunk on the copy stream
    s = dev(hipStreamWaitEvent(st->copy_st, st->computed[b], 0));
    if (s == SIM_OK)
      s = dev(hipMemcpyAsync((char*)y_host + (size_t)j0 * r->n_fast * y_row, ycache,
                             (size_t)k * r->n_fast * y_row, hipMemcpyDeviceToHost, st->copy_st));
    if (s == SIM_OK && t_fast_host) {
      const int first = ch == 0 ? 0 : 1;
      s = dev(hipMemcpyAsync((char*)t_fast_host + (size_t)(j0 + first) * spec,
                             specs + (size_t)first * spec, (size_t)(k + 1 - first) * spec,
                             hipMemcpyDeviceToHost, st->copy_st));
    }
    if (s == SIM_OK) s = dev(hipEventRecord(st->copied[b], st->copy_st));
  }
  // join: the caller's stream waits for the last copies
  sim_status sj = dev(hipEventRecord(st->done, st->copy_st));
  if (sj == SIM_OK) sj = dev(hipStreamWaitEvent(cs_, st->done, 0));
  return s != SIM_OK ? s : sj;
}

}  // extern "C"

