// Host runtime and C-ABI of the pair-cascade PIC library (see include/pic.h).
//
// A gap is a batch of one.  The runtime validates parameters, carves the
// caller's device workspace into the per-gap arrays, fills the device
// descriptors, and enqueues the step kernels on the caller's stream (as a
// replayed HIP graph once the sequence is known).  It never allocates
// device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "pic.h"
#include "pic_device.hpp"
#include "pic_kernels.hpp"

using pic::GapDev;

namespace {

constexpr size_t kAlign = 256;
constexpr int kDefaultSort = 20;
// Steps a gap may run in total: conversion steps of photons are 32-bit and a
// photon converts at most 2^28 steps after its emission (the table limit).
constexpr int64_t kMaxSteps = ((int64_t)1 << 31) - ((int64_t)1 << 28) - 1;
// Steps whose plan holds fewer lepton chunks than this draw their emissions
// inside the push (measured on the 256-gap batch: the push emitting was 11%
// faster over the first 20 steps, about 1.4e4 chunks, and the emission
// kernel 16% faster over 200 steps, whose cascade peaks near 1e5 chunks).
constexpr int64_t kDefaultEmitSplit = 32768;
constexpr int kDefaultHist = 4096;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct GapLayout {
  size_t E, Ef, F, F_last, rho, table, sort_cnt[2], hist;
  size_t cell[2][2], off[2][2], p[2][2], id[2][2];
  size_t ph_rec[2], ph_step[2];
  size_t ph_bucket, ph_key;
  size_t end;
  int64_t table_len;
};

struct Layout {
  size_t gaps, wi, pwi, qwi, twi, cwi, items, emit_cnt, emit_ent, wg_emit, stripes, total;
  long long max_chunks, max_ph_chunks;
  std::vector<GapLayout> g;
  long long cell_items;
};

int grid_for_items(long long want) {
  const long long g = want < 64 ? 64 : (want > 2048 ? 2048 : want);
  return (int)((g + 7) / 8 * 8);
}

int offset_bits(int precision) { return precision == PIC_MIXED ? 24 : 40; }

// Steps the unsorted photon tail may grow before a re-sort sorts the store.
// Each step scans one key byte per tail photon, a sort moves about 64 bytes
// per stored photon, and photons stay about m = 1 / (1 - q) steps in the
// store (q = exp(-dt / (l_gamma dx))): scanning a tail of R a photons over a
// steps against sorting R (m + a) photons every a steps costs least near
// a = sqrt(128 m).
int photon_sort_age(const pic_gap_params& p) {
  if (!(p.l_gamma > 0.0)) return pic::kPhAgeMax;
  const double q = std::exp(-p.dt / (p.l_gamma * p.dx));
  const double m = 1.0 / (1.0 - q);
  const double a = std::sqrt(128.0 * m);
  return a >= (double)pic::kPhAgeMax ? pic::kPhAgeMax : (a < 1.0 ? 1 : (int)a);
}

// Photon conversion table T_k = floor(exp(-k dt / (l_gamma dx)) 2^32), until 0.
int64_t table_length(const pic_gap_params& p) {
  if (!(p.l_gamma > 0.0)) return 0;
  const double r = p.dt / (p.l_gamma * p.dx);
  // the entries vanish once k r > 32 ln 2; a length beyond any valid table
  // is clamped before the conversion to an integer
  const double len = std::ceil(32.0 * std::log(2.0) / r) + 3.0;
  return len < 0x1p40 ? (int64_t)len : (int64_t)1 << 40;
}

std::vector<uint32_t> build_table(const pic_gap_params& p) {
  std::vector<uint32_t> t;
  if (!(p.l_gamma > 0.0)) return t;
  const double r = p.dt / (p.l_gamma * p.dx);
  for (int64_t k = 0;; ++k) {
    const double v = std::floor(std::ldexp(std::exp(-((double)k * r)), 32));
    t.push_back(v >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)v);
    if (v == 0.0) break;
  }
  return t;
}

int hist_rows_of(const pic_gap_params& p) { return p.history_rows > 0 ? p.history_rows : kDefaultHist; }

// Lepton slots per species: the capacity (live leptons) plus a reserve for
// the slots absorbed leptons hold until the next re-sort.
int64_t slots_of(const pic_gap_params& p) { return p.capacity + p.capacity / 8 + 2048; }

pic_status validate(const pic_gap_params* p) {
  if (!p) return PIC_ERR_ARG;
  if (p->n_cells < 2 || p->n_cells > (1 << 22)) return PIC_ERR_ARG;
  if (!(p->dx > 0.0) || !(p->dt > 0.0) || !(p->dt < p->dx) || !std::isfinite(p->dx)) return PIC_ERR_ARG;
  if (p->boundary != PIC_BC_PERIODIC && p->boundary != PIC_BC_ABSORBING) return PIC_ERR_ARG;
  if (!std::isfinite(p->e0)) return PIC_ERR_ARG;
  if (!(p->gamma_thr > 1.0) || !(p->f > 0.0) || !(p->f < 1.0)) return PIC_ERR_ARG;
  if (std::isfinite(p->gamma_thr)) {
    if (!(p->f * p->gamma_thr >= 2.0)) return PIC_ERR_ARG;
    if (!((1.0 - p->f) * p->gamma_thr >= 1.0)) return PIC_ERR_ARG;
  }
  if (!(p->l_gamma >= 0.0) || !std::isfinite(p->l_gamma)) return PIC_ERR_ARG;
  if (!(p->weight >= 0.0) || !std::isfinite(p->weight)) return PIC_ERR_ARG;
  if (!std::isfinite(p->j_m)) return PIC_ERR_ARG;
  if (!(p->gamma_thr_spread >= 0.0) || !(p->gamma_thr_spread < 1.0)) return PIC_ERR_ARG;
  if (p->shape != PIC_SHAPE_LINEAR && p->shape != PIC_SHAPE_QUADRATIC) return PIC_ERR_ARG;
  if (p->shape == PIC_SHAPE_QUADRATIC && p->n_cells < 4) return PIC_ERR_ARG;
  if (p->gamma_thr_spread > 0.0 && std::isfinite(p->gamma_thr) &&
      !((1.0 - p->f - p->gamma_thr_spread) * p->gamma_thr >= 1.0))
    return PIC_ERR_ARG;
  if (p->capacity < 1 || slots_of(*p) >= (int64_t)1 << 31) return PIC_ERR_ARG;
  if (p->photon_capacity < 0 || p->photon_capacity >= (int64_t)1 << 31) return PIC_ERR_ARG;
  if (p->l_gamma > 0.0 && p->photon_capacity < 1) return PIC_ERR_ARG;
  if (p->precision != PIC_FP64 && p->precision != PIC_MIXED) return PIC_ERR_ARG;
  if (p->sort_every < 0 || p->diag_every < 0 || p->history_rows < 0) return PIC_ERR_ARG;
  if (table_length(*p) > (int64_t)1 << 28) return PIC_ERR_ARG;
  // Positions are int64 multiples of 2^-K cells: a photon's longest path
  // (the last step of the conversion table, dt/dx cells per step) and the
  // domain each stay below 2^62 of them, so a conversion point never
  // overflows.
  const double unit = std::ldexp(1.0, offset_bits(p->precision));
  if ((double)p->n_cells * unit > 0x1p62) return PIC_ERR_ARG;
  if (table_length(*p) > 0 &&
      (double)(table_length(*p) + 1) * (p->dt / p->dx * unit + 1.0) >= 0x1p62)
    return PIC_ERR_ARG;
  return PIC_OK;
}

// Lepton slots of a batch, both species; the per-step emitter prefix is
// 32-bit, so a batch holds fewer than 2^32.
bool batch_slots_ok(const pic_gap_params* prm, int B) {
  unsigned long long slots = 0;
  for (int i = 0; i < B; ++i) slots += 2ull * (unsigned long long)slots_of(prm[i]);
  return slots < (1ull << 32);
}

Layout make_layout(const pic_gap_params* prm, int B) {
  Layout L;
  size_t o = 0;
  L.gaps = o; o = align_up(o + sizeof(GapDev) * (size_t)B);
  L.wi = o; o = align_up(o + sizeof(long long) * (size_t)(B + 1));
  L.pwi = o; o = align_up(o + sizeof(long long) * (size_t)(B + 1));
  L.qwi = o; o = align_up(o + sizeof(long long) * (size_t)(B + 1));
  L.twi = o; o = align_up(o + sizeof(long long) * (size_t)(B + 1));
  L.cwi = o; o = align_up(o + sizeof(long long) * (size_t)(B + 1));
  L.items = o; o = align_up(o + sizeof(long long) * 3 * (size_t)B);
  L.cell_items = 0;
  // one emission slice per particle chunk the plan can hold
  L.max_chunks = 0;
  L.max_ph_chunks = 0;
  for (int i = 0; i < B; ++i) {
    L.max_chunks += 2 * ((slots_of(prm[i]) + pic::kChunk - 1) / pic::kChunk);
    L.max_ph_chunks += (prm[i].photon_capacity + pic::kPhChunk - 1) / pic::kPhChunk;
  }
  L.emit_cnt = o; o = align_up(o + sizeof(int32_t) * (size_t)L.max_chunks);
  L.emit_ent = o; o = align_up(o + sizeof(uint32_t) * (size_t)L.max_chunks * pic::kChunk);
  L.wg_emit = o; o = align_up(o + sizeof(uint32_t) * (size_t)pic::kPushGrid);
  L.stripes = o; o = align_up(o + sizeof(unsigned long long) * (size_t)B * 4 * pic::kStripes * pic::kStripeStride);
  const int prec = prm[0].precision;
  const size_t tb = prec == PIC_MIXED ? 4 : 8;
  const int hist = hist_rows_of(prm[0]);
  L.g.resize((size_t)B);
  for (int i = 0; i < B; ++i) {
    const pic_gap_params& p = prm[i];
    GapLayout& G = L.g[(size_t)i];
    const size_t nc = (size_t)p.n_cells, cap = (size_t)slots_of(p), pc = (size_t)p.photon_capacity;
    G.E = o; o = align_up(o + 8 * nc);
    G.Ef = o; o = align_up(o + 4 * nc);
    G.F = o; o = align_up(o + 8 * nc);
    G.F_last = o; o = align_up(o + 8 * nc);
    G.rho = o; o = align_up(o + 8 * (nc + 1));
    G.table_len = (int64_t)build_table(p).size();
    G.table = o; o = align_up(o + 4 * (size_t)G.table_len);
    // per-cell counts of the sorts, and the dead bucket of the tail sort
    for (int s = 0; s < 2; ++s) { G.sort_cnt[s] = o; o = align_up(o + 4 * (nc + 1)); }
    G.hist = o; o = align_up(o + sizeof(pic_history_row) * (size_t)hist);
    for (int b = 0; b < 2; ++b)
      for (int s = 0; s < 2; ++s) {
        G.cell[b][s] = o; o = align_up(o + 4 * cap);
        G.off[b][s] = o; o = align_up(o + tb * cap);
        G.p[b][s] = o; o = align_up(o + tb * cap);
        G.id[b][s] = o; o = align_up(o + 8 * cap);
      }
    for (int b = 0; b < 2; ++b) {
      G.ph_rec[b] = o; o = align_up(o + 16 * pc);
      G.ph_step[b] = o; o = align_up(o + 4 * pc);
    }
    G.ph_bucket = o; o = align_up(o + 4 * ((size_t)G.table_len + 1));
    // tail keys, read 16 at a time from 16-byte boundaries below the store's end
    G.ph_key = o; o = align_up(o + (pc + 15) / 16 * 16);
    G.end = o;
    L.cell_items += ((long long)p.n_cells + pic::kCellChunk - 1) / pic::kCellChunk;
  }
  L.total = o;
  return L;
}

template <typename T>
void fill_precision_constants(GapDev& G, const pic_gap_params& p) {
  const T gthr = (T)p.gamma_thr;
  const T gpair = (T)(p.f * p.gamma_thr);
  const T ghalf = gpair * (T)0.5;
  const T pchild = std::sqrt(ghalf * ghalf - (T)1);
  G.dtdx = (double)(T)(p.dt / p.dx);
  G.gthr = (double)gthr;
  // the lowest threshold a lepton can draw: the spread formula at 2u - 1 = -1
  G.thr_lo = (double)(T)(p.gamma_thr * (1.0 + p.gamma_thr_spread * -1.0));
  G.gpair = (double)gpair;
  G.pchild = (double)pchild;
  // a child's energy for the diagnostics, in binary64 from its momentum
  G.child_gamma64 = std::sqrt(1.0 + (double)pchild * (double)pchild);
}

}  // namespace

struct pic_gap {
  pic_batch* b;
  int idx;
  bool standalone;
};

// Online choice of the re-sort cadence (sort_every = 0).  Sorting never
// changes results, only cost: sorting often costs sort passes, sorting
// rarely lets chunks spread over more cells and leaves appended leptons
// unsorted longer.  Each candidate cadence S has its own captured graph (S
// steps and the sort); every replay is timed with events, read as replays
// complete (a call keeps at most kTuneAhead of them in flight, so the
// tuner also acts within one long call).  Periods of kTunePeriod replays
// start with a probe
// (current, challenger, current, challenger), the challenger alternating
// between half and twice the current cadence; comparing it with the replays
// beside it cancels the growth of the cascade, and a challenger faster per
// step by more than kTuneGain becomes the cadence.
constexpr int kTuneCand[] = {5, 10, 20, 40, 80};
constexpr int kTuneN = 5;
constexpr int kTuneStart = 2;  // 20 steps
constexpr int kTunePeriod = 16;
constexpr double kTuneGain = 0.02;
// Timed replays in flight at most: a long call waits for the oldest before
// enqueueing more, so the tuner reads its probes while the call runs (the
// device still has this many replays queued).
constexpr size_t kTuneAhead = 8;

struct Tuner {
  bool on = false;
  int cur = kTuneStart;
  int round = 0;            // probe rounds opened
  long long launches = 0;   // replays since tuning started
  int probe_ch = -1;        // challenger of the open round (-1: none)
  int got = 0;              // records of the open round read so far
  bool closed = true;
  double probe_cur = 0.0, probe_chal = 0.0;  // summed ms per step
  int switches = 0;
  struct Rec { hipEvent_t a, b; int ci; int round; };  // round -1: not a probe
  std::deque<Rec> pending;
  std::vector<hipEvent_t> spare;
};

struct pic_batch {
  int B = 0;
  int precision = 0, sort_every = kDefaultSort, diag_every = 1, hist_rows = kDefaultHist;
  Tuner tune;
  hipGraphExec_t tgraph[kTuneN] = {};
  hipGraph_t ttmpl[kTuneN] = {};
  long long since_sort = 0;  // steps enqueued since the last re-sort
  bool tail_sorts = false;   // some gap is wider than the push's tile (see launch_tail_sort)
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Layout L;
  std::vector<pic_gap_params> prm;
  std::vector<pic_gap> views;
  std::vector<int32_t> known_status;
  pic::StepLaunch launch{};
  long long host_step = 0;
  bool started = false;
  bool seed_sort = false;  // leptons were seeded since the last sort: sort them before stepping
  hipGraphExec_t graph = nullptr;
  hipGraph_t graph_tmpl = nullptr;
  bool graph_failed = false;
  // push-kernel timing
  bool profiling = false;
  std::vector<hipEvent_t> ev;   // start/stop pairs, reused
  size_t ev_used = 0;
  double prof_ms = 0.0;
  long long prof_launches = 0;
};

namespace {

GapDev* dgaps(pic_batch* b) { return reinterpret_cast<GapDev*>(b->ws + b->L.gaps); }

pic_status read_desc(pic_batch* b, int i, GapDev* out) {
  if (hipMemcpyAsync(out, dgaps(b) + i, sizeof(GapDev), hipMemcpyDeviceToHost, b->stream) != hipSuccess)
    return PIC_ERR_DEVICE;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return PIC_ERR_DEVICE;
  b->known_status[(size_t)i] = out->status;
  return PIC_OK;
}

pic_status write_desc(pic_batch* b, int i, const GapDev* in) {
  if (hipMemcpyAsync(dgaps(b) + i, in, sizeof(GapDev), hipMemcpyHostToDevice, b->stream) != hipSuccess)
    return PIC_ERR_DEVICE;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return PIC_ERR_DEVICE;
  return PIC_OK;
}

pic_status copy_to_host(pic_batch* b, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return PIC_OK;
  if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, b->stream) != hipSuccess) return PIC_ERR_DEVICE;
  return PIC_OK;
}

pic_status create_batch(const pic_gap_params* params, int n_gaps, void* d_ws, size_t ws_bytes,
                        void* hip_stream, pic_batch** out) {
  if (!params || !out || n_gaps < 1 || n_gaps > (1 << 16)) return PIC_ERR_ARG;
  *out = nullptr;
  for (int i = 0; i < n_gaps; ++i) {
    if (validate(&params[i]) != PIC_OK) return PIC_ERR_ARG;
    if (params[i].precision != params[0].precision || params[i].sort_every != params[0].sort_every ||
        params[i].diag_every != params[0].diag_every || params[i].history_rows != params[0].history_rows ||
        params[i].shape != params[0].shape)
      return PIC_ERR_ARG;
  }
  if (!batch_slots_ok(params, n_gaps)) return PIC_ERR_ARG;
  Layout L = make_layout(params, n_gaps);
  if (!d_ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0)
    return PIC_ERR_WORKSPACE;
  pic_batch* b = new (std::nothrow) pic_batch();
  if (!b) return PIC_ERR_ARG;
  b->B = n_gaps;
  b->precision = params[0].precision;
  b->sort_every = params[0].sort_every > 0 ? params[0].sort_every : kDefaultSort;
  b->tune.on = params[0].sort_every == 0;
  b->diag_every = params[0].diag_every > 0 ? params[0].diag_every : 1;
  b->hist_rows = hist_rows_of(params[0]);
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  b->ws = reinterpret_cast<char*>(d_ws);
  b->ws_bytes = ws_bytes;
  b->L = L;
  b->prm.assign(params, params + n_gaps);
  b->known_status.assign((size_t)n_gaps, PIC_OK);
  b->views.resize((size_t)n_gaps);
  for (int i = 0; i < n_gaps; ++i) b->views[(size_t)i] = pic_gap{b, i, false};

  std::vector<GapDev> host((size_t)n_gaps);
  std::vector<long long> cwi((size_t)n_gaps + 1, 0);
  char* ws = b->ws;
  pic_status st = PIC_OK;
  for (int i = 0; i < n_gaps && st == PIC_OK; ++i) {
    const pic_gap_params& p = params[i];
    const GapLayout& GL = L.g[(size_t)i];
    GapDev& G = host[(size_t)i];
    std::memset(&G, 0, sizeof G);
    G.n_cells = p.n_cells;
    G.boundary = p.boundary;
    G.K = offset_bits(p.precision);
    G.precision = p.precision;
    G.shape = p.shape;
    G.diag_every = b->diag_every;
    G.hist_rows = b->hist_rows;
    G.one = (int64_t)1 << G.K;
    G.domain = (int64_t)p.n_cells * G.one;
    G.photon_step = (int64_t)std::rint(std::ldexp(p.dt / p.dx, G.K));
    G.cap = p.capacity;
    G.slots = slots_of(p);
    G.emit_cnt = reinterpret_cast<int32_t*>(ws + L.emit_cnt);
    G.emit_ent = reinterpret_cast<uint32_t*>(ws + L.emit_ent);
    G.wg_emit = reinterpret_cast<uint32_t*>(ws + L.wg_emit);
    G.emit_split = kDefaultEmitSplit;
    G.ph_cap = p.photon_capacity;
    G.dt = p.dt;
    G.dx = p.dx;
    G.weight = p.weight;
    G.wq = std::ldexp(p.weight, -G.K);
    G.e0 = p.e0;
    G.jmdt = p.j_m * p.dt;
    G.sigma = p.gamma_thr_spread;
    G.gthr64 = p.gamma_thr;
    G.gpair64 = p.f * p.gamma_thr;
    G.seed = p.seed;
    if (p.precision == PIC_MIXED) fill_precision_constants<float>(G, p);
    else fill_precision_constants<double>(G, p);
    G.E = reinterpret_cast<double*>(ws + GL.E);
    G.Ef = reinterpret_cast<float*>(ws + GL.Ef);
    G.F = reinterpret_cast<long long*>(ws + GL.F);
    G.F_last = reinterpret_cast<long long*>(ws + GL.F_last);
    G.rho_acc = reinterpret_cast<long long*>(ws + GL.rho);
    G.table = reinterpret_cast<uint32_t*>(ws + GL.table);
    G.table_len = (int32_t)GL.table_len;
    for (int s = 0; s < 2; ++s) G.sort_cnt[s] = reinterpret_cast<int32_t*>(ws + GL.sort_cnt[s]);
    G.hist = reinterpret_cast<pic_history_row*>(ws + GL.hist);
    for (int bb = 0; bb < 2; ++bb) {
      for (int s = 0; s < 2; ++s) {
        G.cell[bb][s] = reinterpret_cast<int32_t*>(ws + GL.cell[bb][s]);
        G.off[bb][s] = ws + GL.off[bb][s];
        G.p[bb][s] = ws + GL.p[bb][s];
        G.id[bb][s] = reinterpret_cast<uint64_t*>(ws + GL.id[bb][s]);
      }
      G.ph_rec[bb] = reinterpret_cast<pic::PhotonRec*>(ws + GL.ph_rec[bb]);
      G.ph_step[bb] = reinterpret_cast<int32_t*>(ws + GL.ph_step[bb]);
    }
    G.ph_bucket = reinterpret_cast<int32_t*>(ws + GL.ph_bucket);
    G.ph_key = reinterpret_cast<uint8_t*>(ws + GL.ph_key);
    G.inv_lnq = p.l_gamma > 0.0 ? (float)(-p.l_gamma * p.dx / p.dt) : 0.0f;
    G.conv_c = p.l_gamma > 0.0 ? (float)(std::log(2.0) * p.l_gamma * p.dx / p.dt) : 0.0f;
    G.ph_age = photon_sort_age(p);
    cwi[(size_t)i + 1] = cwi[(size_t)i] + ((long long)p.n_cells + pic::kCellChunk - 1) / pic::kCellChunk;

    // initial field and zeroed flux; conversion table
    std::vector<double> E((size_t)p.n_cells, p.e0);
    if (hipMemcpy(G.E, E.data(), 8 * (size_t)p.n_cells, hipMemcpyHostToDevice) != hipSuccess) st = PIC_ERR_DEVICE;
    const std::vector<float> Ef((size_t)p.n_cells, (float)p.e0);
    if (st == PIC_OK && hipMemcpy(G.Ef, Ef.data(), 4 * (size_t)p.n_cells, hipMemcpyHostToDevice) != hipSuccess)
      st = PIC_ERR_DEVICE;
    std::vector<long long> z((size_t)p.n_cells + 1, 0);
    if (st == PIC_OK && hipMemcpy(G.F, z.data(), 8 * (size_t)p.n_cells, hipMemcpyHostToDevice) != hipSuccess) st = PIC_ERR_DEVICE;
    if (st == PIC_OK && hipMemcpy(G.F_last, z.data(), 8 * (size_t)p.n_cells, hipMemcpyHostToDevice) != hipSuccess) st = PIC_ERR_DEVICE;
    const std::vector<uint32_t> T = build_table(p);
    if (st == PIC_OK && !T.empty() &&
        hipMemcpy(G.table, T.data(), 4 * T.size(), hipMemcpyHostToDevice) != hipSuccess) st = PIC_ERR_DEVICE;
    const std::vector<int32_t> zb(T.size() + 1, 0);
    if (st == PIC_OK &&
        hipMemcpy(G.ph_bucket, zb.data(), 4 * zb.size(), hipMemcpyHostToDevice) != hipSuccess) st = PIC_ERR_DEVICE;
  }
  if (st == PIC_OK &&
      hipMemcpy(dgaps(b), host.data(), sizeof(GapDev) * (size_t)n_gaps, hipMemcpyHostToDevice) != hipSuccess)
    st = PIC_ERR_DEVICE;
  b->launch.gaps = dgaps(b);
  b->launch.wi = reinterpret_cast<long long*>(ws + L.wi);
  b->launch.pwi = reinterpret_cast<long long*>(ws + L.pwi);
  b->launch.qwi = reinterpret_cast<long long*>(ws + L.qwi);
  b->launch.twi = reinterpret_cast<long long*>(ws + L.twi);
  b->launch.cwi = reinterpret_cast<long long*>(ws + L.cwi);
  b->launch.items = reinterpret_cast<long long*>(ws + L.items);
  b->launch.cell_items = L.cell_items;
  b->launch.B = n_gaps;
  // Emission, conversion and the photon re-sort get grids sized to what the
  // batch can hold (about 16 chunks per workgroup when full), in whole
  // multiples of the 8 XCDs.
  b->launch.push_grid = pic::kPushGrid;
  b->launch.emit_grid = grid_for_items(L.max_chunks / 16);
  b->launch.conv_grid = grid_for_items(L.max_ph_chunks / 16);
  b->launch.ph_sort_grid = grid_for_items(L.max_ph_chunks / 16);
  b->launch.emit_cnt = reinterpret_cast<int32_t*>(ws + L.emit_cnt);
  b->launch.emit_ent = reinterpret_cast<uint32_t*>(ws + L.emit_ent);
  b->launch.wg_emit = reinterpret_cast<uint32_t*>(ws + L.wg_emit);
  b->launch.stripes = reinterpret_cast<unsigned long long*>(ws + L.stripes);
  b->launch.stream = b->stream;
  b->launch.spline = params[0].shape == PIC_SHAPE_QUADRATIC;
  b->launch.spread = false;
  for (int i = 0; i < n_gaps; ++i) b->launch.spread |= params[i].gamma_thr_spread > 0.0;
  // in gaps no wider than the push's tile every chunk fits it: no tail sorts
  for (int i = 0; i < n_gaps; ++i) b->tail_sorts |= params[i].n_cells > pic::kTile - 8;
  if (st == PIC_OK &&
      hipMemcpy(b->launch.cwi, cwi.data(), sizeof(long long) * cwi.size(), hipMemcpyHostToDevice) != hipSuccess)
    st = PIC_ERR_DEVICE;
  const std::vector<unsigned long long> zs((size_t)n_gaps * 4 * pic::kStripes * pic::kStripeStride, 0ull);
  if (st == PIC_OK && hipMemcpy(b->launch.stripes, zs.data(), sizeof(unsigned long long) * zs.size(),
                                hipMemcpyHostToDevice) != hipSuccess)
    st = PIC_ERR_DEVICE;
  if (st == PIC_OK && pic::launch_plan(b->launch) != hipSuccess) st = PIC_ERR_DEVICE;
  if (st == PIC_OK && hipStreamSynchronize(b->stream) != hipSuccess) st = PIC_ERR_DEVICE;
  if (st != PIC_OK) {
    delete b;
    return st;
  }
  *out = b;
  return PIC_OK;
}

pic_status append_counts(pic_batch* b, int g, long long add0, long long add1) {
  GapDev G;
  pic_status st = read_desc(b, g, &G);
  if (st != PIC_OK) return st;
  G.n[0] += (unsigned long long)add0; G.live[0] += (unsigned long long)add0;
  G.n[1] += (unsigned long long)add1; G.live[1] += (unsigned long long)add1;
  // the seed counts as the body of the first full re-sort, not as appended
  G.body_n[0] = G.n[0];
  G.body_n[1] = G.n[1];
  st = write_desc(b, g, &G);
  if (st != PIC_OK) return st;
  if (pic::launch_plan(b->launch) != hipSuccess) return PIC_ERR_DEVICE;
  return hipStreamSynchronize(b->stream) == hipSuccess ? PIC_OK : PIC_ERR_DEVICE;
}

// Folds the recorded event pairs into the running total (synchronises).
pic_status drain_events(pic_batch* b) {
  if (b->ev_used == 0) return PIC_OK;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return PIC_ERR_DEVICE;
  for (size_t i = 0; i + 1 < b->ev_used; i += 2) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, b->ev[i], b->ev[i + 1]) != hipSuccess) return PIC_ERR_DEVICE;
    b->prof_ms += ms;
    b->prof_launches += 1;
  }
  b->ev_used = 0;
  return PIC_OK;
}

// One step launched directly, with the push bracketed by events when
// profiling; the re-sort follows every sort_every steps.
pic_status eager_step(pic_batch* b) {
  const bool mixed = b->precision == PIC_MIXED;
  if (b->profiling) {
    if (b->ev_used + 2 > b->ev.size()) {
      if (b->ev.size() >= 8192) {
        pic_status st = drain_events(b);
        if (st != PIC_OK) return st;
      } else {
        for (int e = 0; e < 2; ++e) {
          // timing only: no system-scope fence (and its cache write-back)
          // when the push completes, which would be counted in its time
          hipEvent_t h;
          if (hipEventCreateWithFlags(&h, hipEventDisableSystemFence) != hipSuccess)
            return PIC_ERR_DEVICE;
          b->ev.push_back(h);
        }
      }
    }
    if (pic::launch_push(b->launch, mixed, b->ev[b->ev_used], b->ev[b->ev_used + 1]) != hipSuccess)
      return PIC_ERR_DEVICE;
    b->ev_used += 2;
    if (pic::launch_step_after_push(b->launch, mixed) != hipSuccess) return PIC_ERR_DEVICE;
  } else if (pic::launch_step(b->launch, mixed) != hipSuccess) {
    return PIC_ERR_DEVICE;
  }
  b->host_step += 1;
  b->since_sort += 1;
  if (b->since_sort >= b->sort_every) {
    if (pic::launch_sort(b->launch, mixed) != hipSuccess) return PIC_ERR_DEVICE;
    b->since_sort = 0;
  } else if (b->tail_sorts && b->since_sort % pic::kTailEvery == 0) {
    if (pic::launch_tail_sort(b->launch, mixed) != hipSuccess) return PIC_ERR_DEVICE;
  }
  return PIC_OK;
}

// Captures sort_every steps and the re-sort that ends them as one graph,
// with the sorts of the appended leptons every kTailEvery steps between.
// Every kernel reads its counts and plans from device memory, so the graph
// can be replayed at any step that is a multiple of sort_every.
bool build_graph(pic_batch* b, int S, hipGraph_t* tmpl, hipGraphExec_t* exec) {
  const bool mixed = b->precision == PIC_MIXED;
  if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed) != hipSuccess) return false;
  bool ok = true;
  for (int k = 1; k <= S && ok; ++k) {
    ok = pic::launch_step(b->launch, mixed) == hipSuccess;
    if (ok && b->tail_sorts && k < S && k % pic::kTailEvery == 0)
      ok = pic::launch_tail_sort(b->launch, mixed) == hipSuccess;
  }
  if (ok) ok = pic::launch_sort(b->launch, mixed) == hipSuccess;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (!ok || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return false;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return false;
  }
  *tmpl = g;
  *exec = x;
  return true;
}

// ---- cadence tuner
hipEvent_t tune_event(Tuner& t) {
  if (!t.spare.empty()) {
    hipEvent_t e = t.spare.back();
    t.spare.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Reads the timed replays that have completed (never blocks); the open
// round is decided once its four records are in (records of an earlier,
// abandoned round are dropped).
void tune_harvest(Tuner& t) {
  while (!t.pending.empty()) {
    Tuner::Rec r = t.pending.front();
    if (hipEventQuery(r.b) != hipSuccess) break;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    t.pending.pop_front();
    t.spare.push_back(r.a);
    t.spare.push_back(r.b);
    if (r.round != t.round || t.closed) continue;
    const double per_step = (double)ms / (double)kTuneCand[r.ci];
    if (r.ci == t.probe_ch) t.probe_chal += per_step;
    else t.probe_cur += per_step;
    if (++t.got == 4) {
      if (t.probe_chal < (1.0 - kTuneGain) * t.probe_cur) {
        t.cur = t.probe_ch;
        t.switches += 1;
      }
      t.closed = true;
    }
  }
}

// Candidate for the next replay; `round` is the probe round it belongs to
// (-1 outside probes).  A round opens at the start of every period.
int tune_pick(Tuner& t, int& round) {
  const long long pos = t.launches % kTunePeriod;
  round = -1;
  if (pos == 0) {
    const int dir = (t.round & 1) ? 1 : -1;
    int ch = t.cur + dir;
    if (ch < 0 || ch >= kTuneN) ch = t.cur - dir;
    t.round += 1;
    t.probe_ch = (ch >= 0 && ch < kTuneN) ? ch : -1;
    t.got = 0;
    t.closed = t.probe_ch < 0;
    t.probe_cur = t.probe_chal = 0.0;
  }
  if (!t.closed && pos < 4) {
    round = t.round;
    return (pos & 1) ? t.probe_ch : t.cur;
  }
  return t.cur;
}

// The seed, written in the order it was drawn, is sorted by cell group once before
// the first step, so that its chunks deposit through the LDS tile from the
// start (results do not depend on lepton order).
pic_status sort_seed(pic_batch* b) {
  if (!b->seed_sort) return PIC_OK;
  if (pic::launch_sort(b->launch, b->precision == PIC_MIXED) != hipSuccess) return PIC_ERR_DEVICE;
  b->seed_sort = false;
  return PIC_OK;
}

// Captures (and uploads) every graph the step sequence can replay: the
// candidate cadences of the tuner, or the one fixed cadence.
pic_status prepare_graphs(pic_batch* b) {
  if (b->stream == nullptr || b->profiling || b->graph_failed) return PIC_OK;
  if (b->tune.on) {
    for (int ci = 0; ci < kTuneN; ++ci) {
      if (b->tgraph[ci]) continue;
      if (!build_graph(b, kTuneCand[ci], &b->ttmpl[ci], &b->tgraph[ci])) {
        b->graph_failed = true;
        return PIC_OK;
      }
      if (hipGraphUpload(b->tgraph[ci], b->stream) != hipSuccess) return PIC_ERR_DEVICE;
    }
  } else if (!b->graph) {
    if (!build_graph(b, b->sort_every, &b->graph_tmpl, &b->graph)) {
      b->graph_failed = true;
      return PIC_OK;
    }
    if (hipGraphUpload(b->graph, b->stream) != hipSuccess) return PIC_ERR_DEVICE;
  }
  return PIC_OK;
}

pic_status enqueue_steps(pic_batch* b, int64_t n_steps) {
  if (n_steps > 0) {
    const pic_status st = sort_seed(b);
    if (st != PIC_OK) return st;
  }
  // graphs need a capturable (non-null) stream and no per-launch events
  const bool graphs = b->stream != nullptr && !b->profiling && !b->graph_failed;
  Tuner& t = b->tune;
  while (n_steps > 0) {
    if (t.on && b->since_sort == 0) {
      while (t.pending.size() >= kTuneAhead) {
        if (hipEventSynchronize(t.pending.front().b) != hipSuccess) return PIC_ERR_DEVICE;
        tune_harvest(t);
      }
      tune_harvest(t);
      int round = -1;
      const int ci = tune_pick(t, round);
      const int S = kTuneCand[ci];
      b->sort_every = S;  // eager steps that follow keep this cadence
      if (n_steps >= S) {
        // one timed replay: S steps and the re-sort, as a graph launch or,
        // without graphs (null stream, failed capture, per-push events), as
        // S eager steps
        if (graphs && !b->tgraph[ci] && !build_graph(b, S, &b->ttmpl[ci], &b->tgraph[ci])) {
          b->graph_failed = true;
          return enqueue_steps(b, n_steps);
        }
        hipEvent_t e0 = tune_event(t), e1 = tune_event(t);
        if (!e0 || !e1) return PIC_ERR_DEVICE;
        if (hipEventRecord(e0, b->stream) != hipSuccess) return PIC_ERR_DEVICE;
        if (graphs) {
          if (hipGraphLaunch(b->tgraph[ci], b->stream) != hipSuccess) return PIC_ERR_DEVICE;
          b->host_step += S;
        } else {
          for (int k = 0; k < S; ++k) {
            const pic_status st = eager_step(b);  // the S-th step re-sorts
            if (st != PIC_OK) {
              t.spare.push_back(e0);
              t.spare.push_back(e1);
              return st;
            }
          }
        }
        if (hipEventRecord(e1, b->stream) != hipSuccess) return PIC_ERR_DEVICE;
        t.pending.push_back(Tuner::Rec{e0, e1, ci, round});
        t.launches += 1;
        n_steps -= S;
        continue;
      }
      // fewer steps left than the cadence: finish them eagerly at this cadence
    }
    if (graphs && !t.on && b->since_sort == 0 && n_steps >= b->sort_every) {
      if (!b->graph && !build_graph(b, b->sort_every, &b->graph_tmpl, &b->graph)) {
        b->graph_failed = true;
        return enqueue_steps(b, n_steps);
      }
      if (hipGraphLaunch(b->graph, b->stream) != hipSuccess) return PIC_ERR_DEVICE;
      b->host_step += b->sort_every;
      n_steps -= b->sort_every;
    } else {
      pic_status st = eager_step(b);
      if (st != PIC_OK) return st;
      --n_steps;
    }
  }
  b->started = true;
  return PIC_OK;
}

}  // namespace

extern "C" {

pic_status pic_validate_params(const pic_gap_params* p) { return validate(p); }

size_t pic_workspace_bytes(const pic_gap_params* p) {
  if (validate(p) != PIC_OK) return 0;
  return make_layout(p, 1).total;
}

size_t pic_batch_workspace_bytes(const pic_gap_params* params, int32_t n_gaps) {
  if (!params || n_gaps < 1) return 0;
  for (int i = 0; i < n_gaps; ++i)
    if (validate(&params[i]) != PIC_OK) return 0;
  if (!batch_slots_ok(params, n_gaps)) return 0;
  return make_layout(params, n_gaps).total;
}

int32_t pic_batch_plan(const pic_gap_params* params, int32_t n_gaps, size_t budget_bytes,
                       uint8_t* admitted, size_t* ws_bytes) {
  if (!params || n_gaps < 1 || !admitted) return PIC_ERR_ARG;
  std::vector<pic_gap_params> acc;
  size_t used = 0;
  for (int i = 0; i < n_gaps; ++i) {
    admitted[i] = 0;
    if (validate(&params[i]) != PIC_OK) continue;
    acc.push_back(params[i]);
    if (!batch_slots_ok(acc.data(), (int)acc.size())) {
      acc.pop_back();
      continue;
    }
    const size_t need = make_layout(acc.data(), (int)acc.size()).total;
    if (need <= budget_bytes) {
      admitted[i] = 1;
      used = need;
    } else {
      acc.pop_back();
    }
  }
  if (ws_bytes) *ws_bytes = used;
  return (int32_t)acc.size();
}

pic_status pic_create_gap(const pic_gap_params* p, void* d_ws, size_t ws_bytes, void* hip_stream,
                          pic_gap** out) {
  if (!out) return PIC_ERR_ARG;
  *out = nullptr;
  pic_batch* b = nullptr;
  pic_status st = create_batch(p, 1, d_ws, ws_bytes, hip_stream, &b);
  if (st != PIC_OK) return st;
  b->views[0].standalone = true;
  *out = &b->views[0];
  return PIC_OK;
}

pic_status pic_create_batch(const pic_gap_params* params, int32_t n_gaps, void* d_ws,
                            size_t ws_bytes, void* hip_stream, pic_batch** out) {
  return create_batch(params, n_gaps, d_ws, ws_bytes, hip_stream, out);
}

pic_gap* pic_batch_gap(pic_batch* b, int32_t i) {
  if (!b || i < 0 || i >= b->B) return nullptr;
  return &b->views[(size_t)i];
}

int32_t pic_batch_size(const pic_batch* b) { return b ? b->B : 0; }

int32_t pic_offset_bits(const pic_gap* g) {
  if (!g) return PIC_ERR_ARG;
  return offset_bits(g->b->precision);
}

pic_status pic_seed_particles(pic_gap* g, int32_t mode, int64_t n_pairs, int32_t macro_per_pair,
                              double p0_minus, double p0_plus) {
  if (!g || n_pairs < 0 || macro_per_pair < 1) return PIC_ERR_ARG;
  if (mode != PIC_SEED_RANDOM && mode != PIC_SEED_LATTICE) return PIC_ERR_ARG;
  if (!std::isfinite(p0_minus) || !std::isfinite(p0_plus)) return PIC_ERR_ARG;
  pic_batch* b = g->b;
  if (b->started) return PIC_ERR_STATE;
  const long long N = (long long)n_pairs * (long long)macro_per_pair;
  if (n_pairs > 0 && N / n_pairs != macro_per_pair) return PIC_ERR_ARG;
  GapDev G;
  pic_status st = read_desc(b, g->idx, &G);
  if (st != PIC_OK) return st;
  // seed ids start at 0: a gap that already holds leptons would get
  // duplicate ids, and with them shared random streams
  if (G.n[0] != 0 || G.n[1] != 0) return PIC_ERR_STATE;
  if (N > G.cap) return PIC_ERR_CAPACITY;
  if (N == 0) return PIC_OK;
  if (pic::launch_seed(dgaps(b), g->idx, mode, N, p0_minus, p0_plus, (long long)G.n[0],
                       (long long)G.n[1], b->precision == PIC_MIXED, b->stream) != hipSuccess)
    return PIC_ERR_DEVICE;
  b->seed_sort = true;
  return append_counts(b, g->idx, N, N);
}

pic_status pic_seed_explicit(pic_gap* g, int32_t species, int64_t n, const int32_t* cell,
                             const double* off, const double* p, const uint64_t* id) {
  if (!g || species < 0 || species > 1 || n < 0) return PIC_ERR_ARG;
  if (n > 0 && (!cell || !off || !p || !id)) return PIC_ERR_ARG;
  pic_batch* b = g->b;
  if (b->started) return PIC_ERR_STATE;
  const pic_gap_params& prm = b->prm[(size_t)g->idx];
  for (int64_t i = 0; i < n; ++i) {
    if (cell[i] < 0 || cell[i] >= prm.n_cells) return PIC_ERR_ARG;
    if (!(off[i] >= 0.0) || !(off[i] < 1.0) || !std::isfinite(p[i])) return PIC_ERR_ARG;
  }
  GapDev G;
  pic_status st = read_desc(b, g->idx, &G);
  if (st != PIC_OK) return st;
  if ((long long)G.n[species] + n > G.cap) return PIC_ERR_CAPACITY;
  if (n == 0) return PIC_OK;
  const int K = offset_bits(b->precision);
  const size_t base = (size_t)G.n[species];
  const int bb = G.buf;
  std::vector<int32_t> c(cell, cell + n);
  std::vector<uint64_t> ids(id, id + n);
  hipError_t e = hipMemcpy(G.cell[bb][species] + base, c.data(), 4 * (size_t)n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(G.id[bb][species] + base, ids.data(), 8 * (size_t)n, hipMemcpyHostToDevice);
  if (b->precision == PIC_MIXED) {
    std::vector<float> o((size_t)n), pp((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
      o[(size_t)i] = (float)std::ldexp(std::floor(std::ldexp(off[i], K)), -K);
      pp[(size_t)i] = (float)p[i];
    }
    if (e == hipSuccess) e = hipMemcpy((float*)G.off[bb][species] + base, o.data(), 4 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((float*)G.p[bb][species] + base, pp.data(), 4 * (size_t)n, hipMemcpyHostToDevice);
  } else {
    std::vector<double> o((size_t)n), pp(p, p + n);
    for (int64_t i = 0; i < n; ++i) o[(size_t)i] = std::ldexp(std::floor(std::ldexp(off[i], K)), -K);
    if (e == hipSuccess) e = hipMemcpy((double*)G.off[bb][species] + base, o.data(), 8 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((double*)G.p[bb][species] + base, pp.data(), 8 * (size_t)n, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return PIC_ERR_DEVICE;
  b->seed_sort = true;
  return append_counts(b, g->idx, species == 0 ? n : 0, species == 1 ? n : 0);
}

pic_status pic_step_n(pic_gap* g, int64_t n_steps, pic_step_report* out) {
  if (!g || n_steps < 0) return PIC_ERR_ARG;
  if (!g->standalone) return PIC_ERR_STATE;
  pic_batch* b = g->b;
  if (n_steps > kMaxSteps - b->host_step) return PIC_ERR_ARG;
  if (b->known_status[0] != PIC_OK) return PIC_ERR_STATE;
  pic_status st = enqueue_steps(b, n_steps);
  if (st != PIC_OK) return st;
  if (out) {
    GapDev G;
    st = read_desc(b, 0, &G);
    if (st != PIC_OK) return st;
    out->steps_done = G.step;
    out->status = G.status;
    out->pushes = (int64_t)G.pushes;
  }
  return PIC_OK;
}

pic_status pic_batch_prepare(pic_batch* b) {
  if (!b) return PIC_ERR_ARG;
  if (b->started) return PIC_ERR_STATE;
  pic_status st = sort_seed(b);
  if (st == PIC_OK) st = prepare_graphs(b);
  if (st != PIC_OK) return st;
  return hipStreamSynchronize(b->stream) == hipSuccess ? PIC_OK : PIC_ERR_DEVICE;
}

pic_status pic_prepare(pic_gap* g) {
  if (!g || !g->standalone) return PIC_ERR_ARG;
  return pic_batch_prepare(g->b);
}

pic_status pic_batch_step_n(pic_batch* b, int64_t n_steps, pic_status* per_gap) {
  if (!b || n_steps < 0) return PIC_ERR_ARG;
  if (n_steps > kMaxSteps - b->host_step) return PIC_ERR_ARG;
  pic_status st = enqueue_steps(b, n_steps);
  if (st != PIC_OK) return st;
  if (per_gap) {
    std::vector<GapDev> all((size_t)b->B);
    if (hipMemcpyAsync(all.data(), dgaps(b), sizeof(GapDev) * (size_t)b->B, hipMemcpyDeviceToHost,
                       b->stream) != hipSuccess)
      return PIC_ERR_DEVICE;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return PIC_ERR_DEVICE;
    for (int i = 0; i < b->B; ++i) {
      per_gap[i] = all[(size_t)i].status;
      b->known_status[(size_t)i] = all[(size_t)i].status;
    }
  }
  return PIC_OK;
}

pic_status pic_read_fields(pic_gap* g, double* E, double* rho, int32_t n_cells) {
  if (!g) return PIC_ERR_ARG;
  pic_batch* b = g->b;
  GapDev G;
  pic_status st = read_desc(b, g->idx, &G);
  if (st != PIC_OK) return st;
  if (n_cells != G.n_cells) return PIC_ERR_ARG;
  if (E && copy_to_host(b, E, G.E, 8 * (size_t)n_cells) != PIC_OK) return PIC_ERR_DEVICE;
  if (rho) {
    std::vector<long long> acc((size_t)n_cells + 1);
    if (pic::launch_rho(dgaps(b), g->idx, G.rho_acc, n_cells + 1, b->precision == PIC_MIXED,
                        b->stream) != hipSuccess)
      return PIC_ERR_DEVICE;
    if (copy_to_host(b, acc.data(), G.rho_acc, 8 * acc.size()) != PIC_OK) return PIC_ERR_DEVICE;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return PIC_ERR_DEVICE;
    if (G.boundary == PIC_BC_PERIODIC) {
      acc[0] += acc[(size_t)n_cells];
      acc[(size_t)n_cells] = acc[0];
    }
    for (int32_t c = 0; c <= n_cells; ++c) rho[c] = G.wq * (double)acc[(size_t)c];
  }
  return hipStreamSynchronize(b->stream) == hipSuccess ? PIC_OK : PIC_ERR_DEVICE;
}

pic_status pic_read_fields_noalloc(pic_gap* g, double* E, double* rho, int32_t n_cells) {
  if (!g) return PIC_ERR_ARG;
  pic_batch* b = g->b;
  GapDev G;
  pic_status st = read_desc(b, g->idx, &G);
  if (st != PIC_OK) return st;
  if (n_cells != G.n_cells) return PIC_ERR_ARG;
  if (rho && (long long)n_cells + 1 > pic::kStaticNodes) return PIC_ERR_ARG;
  if (E && copy_to_host(b, E, G.E, 8 * (size_t)n_cells) != PIC_OK) return PIC_ERR_DEVICE;
  if (rho) {
    // the GPU that holds this gap, whose copy of the static scratch is used
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, b->ws) != hipSuccess) return PIC_ERR_DEVICE;
    long long* acc = nullptr;
    if (pic::static_scratch(attr.device, &acc) != hipSuccess) return PIC_ERR_DEVICE;
    if (pic::launch_rho(dgaps(b), g->idx, acc, n_cells + 1, b->precision == PIC_MIXED, b->stream) !=
        hipSuccess)
      return PIC_ERR_DEVICE;
    // the int64 accumulators land in the caller's buffer (same size) and are
    // turned into charges in place
    if (copy_to_host(b, rho, acc, 8 * ((size_t)n_cells + 1)) != PIC_OK) return PIC_ERR_DEVICE;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return PIC_ERR_DEVICE;
    int64_t first = 0, last = 0;
    std::memcpy(&first, rho, 8);
    std::memcpy(&last, rho + n_cells, 8);
    if (G.boundary == PIC_BC_PERIODIC) first = last = first + last;
    for (int32_t c = 0; c <= n_cells; ++c) {
      int64_t v;
      std::memcpy(&v, rho + c, 8);
      if (c == 0) v = first;
      if (c == n_cells) v = last;
      rho[c] = G.wq * (double)v;
    }
  }
  return hipStreamSynchronize(b->stream) == hipSuccess ? PIC_OK : PIC_ERR_DEVICE;
}

pic_status pic_phase_space(pic_gap* g, int32_t species, int32_t x_bins, int32_t p_bins, double p_min,
                           double p_max, int64_t* d_counts) {
  if (!g || !d_counts || species < 0 || species > 1 || x_bins < 1 || p_bins < 1) return PIC_ERR_ARG;
  if ((int64_t)x_bins * p_bins > ((int64_t)1 << 30)) return PIC_ERR_ARG;
  if (!std::isfinite(p_min) || !std::isfinite(p_max) || !(p_max > p_min)) return PIC_ERR_ARG;
  pic_batch* b = g->b;
  const double inv_dp = (double)p_bins / (p_max - p_min);
  if (pic::launch_phase(dgaps(b), g->idx, species, x_bins, p_bins, p_min, inv_dp,
                        reinterpret_cast<unsigned long long*>(d_counts), b->precision == PIC_MIXED,
                        b->stream) != hipSuccess)
    return PIC_ERR_DEVICE;
  return PIC_OK;
}

pic_status pic_event_map(pic_gap* g, int64_t* d_map, int32_t x_bins, int32_t steps_per_row, int32_t rows) {
  if (!g) return PIC_ERR_ARG;
  if (d_map && (x_bins < 1 || steps_per_row < 1 || rows < 1)) return PIC_ERR_ARG;
  if (d_map && (int64_t)x_bins * rows > ((int64_t)1 << 34)) return PIC_ERR_ARG;
  pic_batch* b = g->b;
  GapDev G;
  pic_status st = read_desc(b, g->idx, &G);
  if (st != PIC_OK) return st;
  if (d_map && pic::launch_zero(reinterpret_cast<long long*>(d_map), (long long)x_bins * rows, b->stream) != hipSuccess)
    return PIC_ERR_DEVICE;
  G.evmap = reinterpret_cast<unsigned long long*>(d_map);
  G.ev_x = d_map ? x_bins : 0;
  G.ev_steps = d_map ? steps_per_row : 1;
  G.ev_rows = d_map ? rows : 1;
  return write_desc(b, g->idx, &G);
}

pic_status pic_read_flux(pic_gap* g, int64_t* flux, int32_t n_cells) {
  if (!g || !flux) return PIC_ERR_ARG;
  pic_batch* b = g->b;
  GapDev G;
  pic_status st = read_desc(b, g->idx, &G);
  if (st != PIC_OK) return st;
  if (n_cells != G.n_cells) return PIC_ERR_ARG;
  if (copy_to_host(b, flux, G.F_last, 8 * (size_t)n_cells) != PIC_OK) return PIC_ERR_DEVICE;
  return hipStreamSynchronize(b->stream) == hipSuccess ? PIC_OK : PIC_ERR_DEVICE;
}

pic_status pic_read_moments(pic_gap* g, pic_moments* out) {
  if (!g || !out) return PIC_ERR_ARG;
  GapDev G;
  pic_status st = read_desc(g->b, g->idx, &G);
  if (st != PIC_OK) return st;
  std::memset(out, 0, sizeof *out);
  out->steps_done = G.step;
  out->status = G.status;
  out->n_minus = (int64_t)G.live[0];
  out->n_plus = (int64_t)G.live[1];
  out->n_photons = (int64_t)G.inflight;
  out->slots_minus = (int64_t)G.n[0];
  out->slots_plus = (int64_t)G.n[1];
  out->photon_slots = (int64_t)G.n_ph;
  out->pushes = (int64_t)G.pushes;
  out->last = G.last;
  out->push_emissions = (int64_t)G.push_emitted;
  return PIC_OK;
}

pic_status pic_read_history(pic_gap* g, pic_history_row* rows, int64_t max_rows, int64_t* n_out) {
  if (!g || max_rows < 0) return PIC_ERR_ARG;
  pic_batch* b = g->b;
  GapDev G;
  pic_status st = read_desc(b, g->idx, &G);
  if (st != PIC_OK) return st;
  const int64_t R = G.hist_rows;
  const int64_t avail = (int64_t)G.hist_count < R ? (int64_t)G.hist_count : R;
  if (n_out) *n_out = avail;
  if (!rows || max_rows == 0 || avail == 0) return PIC_OK;
  std::vector<pic_history_row> ring((size_t)R);
  if (copy_to_host(b, ring.data(), G.hist, sizeof(pic_history_row) * (size_t)R) != PIC_OK) return PIC_ERR_DEVICE;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return PIC_ERR_DEVICE;
  const int64_t first = (int64_t)G.hist_count - avail;
  const int64_t n = std::min(avail, max_rows);
  for (int64_t k = 0; k < n; ++k) rows[k] = ring[(size_t)((first + k) % R)];
  return PIC_OK;
}

pic_status pic_read_particles(pic_gap* g, int32_t species, int64_t max_n, int32_t* cell,
                              double* off, double* p, uint64_t* id, int64_t* n_out) {
  if (!g || species < 0 || species > 1 || max_n < 0) return PIC_ERR_ARG;
  pic_batch* b = g->b;
  GapDev G;
  pic_status st = read_desc(b, g->idx, &G);
  if (st != PIC_OK) return st;
  const size_t n = (size_t)G.n[species];
  const int bb = G.buf;
  const bool mixed = b->precision == PIC_MIXED;
  std::vector<int32_t> c(n);
  std::vector<uint64_t> ids(n);
  std::vector<double> o(n), pp(n);
  std::vector<float> of, pf;
  if (copy_to_host(b, c.data(), G.cell[bb][species], 4 * n) != PIC_OK) return PIC_ERR_DEVICE;
  if (copy_to_host(b, ids.data(), G.id[bb][species], 8 * n) != PIC_OK) return PIC_ERR_DEVICE;
  if (mixed) {
    of.resize(n); pf.resize(n);
    if (copy_to_host(b, of.data(), G.off[bb][species], 4 * n) != PIC_OK) return PIC_ERR_DEVICE;
    if (copy_to_host(b, pf.data(), G.p[bb][species], 4 * n) != PIC_OK) return PIC_ERR_DEVICE;
  } else {
    if (copy_to_host(b, o.data(), G.off[bb][species], 8 * n) != PIC_OK) return PIC_ERR_DEVICE;
    if (copy_to_host(b, pp.data(), G.p[bb][species], 8 * n) != PIC_OK) return PIC_ERR_DEVICE;
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess) return PIC_ERR_DEVICE;
  int64_t live = 0;
  for (size_t i = 0; i < n; ++i) {
    if (c[i] == pic::kDead) continue;
    if (live < max_n) {
      if (cell) cell[live] = c[i];
      if (off) off[live] = mixed ? (double)of[i] : o[i];
      if (p) p[live] = mixed ? (double)pf[i] : pp[i];
      if (id) id[live] = ids[i];
    }
    ++live;
  }
  if (n_out) *n_out = live;
  return PIC_OK;
}

pic_status pic_read_photons(pic_gap* g, int64_t max_n, int64_t* xq, int64_t* conv_step,
                            int32_t* dir, uint64_t* child, int64_t* n_out) {
  if (!g || max_n < 0) return PIC_ERR_ARG;
  pic_batch* b = g->b;
  GapDev G;
  pic_status st = read_desc(b, g->idx, &G);
  if (st != PIC_OK) return st;
  const size_t n = (size_t)G.n_ph;
  const int pb = G.phbuf;
  std::vector<pic::PhotonRec> rec(n);
  std::vector<int32_t> cs(n);
  if (copy_to_host(b, rec.data(), G.ph_rec[pb], 16 * n) != PIC_OK) return PIC_ERR_DEVICE;
  if (copy_to_host(b, cs.data(), G.ph_step[pb], 4 * n) != PIC_OK) return PIC_ERR_DEVICE;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return PIC_ERR_DEVICE;
  int64_t k = 0;
  for (size_t i = 0; i < n; ++i) {
    if ((long long)cs[i] < G.step) continue;  // converted or escaped, not yet reclaimed
    if (k < max_n) {
      if (xq) xq[k] = rec[i].x;
      if (conv_step) conv_step[k] = cs[i];
      if (dir) dir[k] = (rec[i].child & 1u) ? 1 : -1;
      if (child) child[k] = rec[i].child & ~(uint64_t)1;
    }
    ++k;
  }
  if (n_out) *n_out = k;
  return PIC_OK;
}

pic_status pic_set_fields(pic_gap* g, const double* E, int32_t n_cells) {
  if (!g || !E) return PIC_ERR_ARG;
  pic_batch* b = g->b;
  if (n_cells != b->prm[(size_t)g->idx].n_cells) return PIC_ERR_ARG;
  for (int32_t c = 0; c < n_cells; ++c)
    if (!std::isfinite(E[c])) return PIC_ERR_ARG;
  GapDev G;
  pic_status st = read_desc(b, g->idx, &G);
  if (st != PIC_OK) return st;
  if (hipMemcpy(G.E, E, 8 * (size_t)n_cells, hipMemcpyHostToDevice) != hipSuccess) return PIC_ERR_DEVICE;
  std::vector<float> Ef((size_t)n_cells);
  for (int32_t c = 0; c < n_cells; ++c) Ef[(size_t)c] = (float)E[c];
  if (hipMemcpy(G.Ef, Ef.data(), 4 * (size_t)n_cells, hipMemcpyHostToDevice) != hipSuccess) return PIC_ERR_DEVICE;
  return PIC_OK;
}

pic_status pic_destroy(pic_gap* g) {
  if (!g) return PIC_ERR_ARG;
  if (!g->standalone) return PIC_ERR_STATE;
  return pic_destroy_batch(g->b);
}

pic_status pic_destroy_batch(pic_batch* b) {
  if (!b) return PIC_ERR_ARG;
  pic_status st = hipStreamSynchronize(b->stream) == hipSuccess ? PIC_OK : PIC_ERR_DEVICE;
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->graph_tmpl) (void)hipGraphDestroy(b->graph_tmpl);
  for (int i = 0; i < kTuneN; ++i) {
    if (b->tgraph[i]) (void)hipGraphExecDestroy(b->tgraph[i]);
    if (b->ttmpl[i]) (void)hipGraphDestroy(b->ttmpl[i]);
  }
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  for (const Tuner::Rec& r : b->tune.pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (hipEvent_t e : b->tune.spare) (void)hipEventDestroy(e);
  delete b;
  return st;
}

pic_status pic_batch_profile_push(pic_batch* b, int32_t enable) {
  if (!b) return PIC_ERR_ARG;
  if (b->profiling && !enable) {
    pic_status st = drain_events(b);
    if (st != PIC_OK) return st;
  }
  b->profiling = enable != 0;
  b->ev_used = 0;
  b->prof_ms = 0.0;
  b->prof_launches = 0;
  return PIC_OK;
}

pic_status pic_batch_tuning(pic_batch* b, int32_t* sort_every, int32_t* autotuned,
                            int64_t* replays, int32_t* switches) {
  if (!b) return PIC_ERR_ARG;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return PIC_ERR_DEVICE;
  tune_harvest(b->tune);
  if (sort_every) *sort_every = b->tune.on ? kTuneCand[b->tune.cur] : b->sort_every;
  if (autotuned) *autotuned = b->tune.on ? 1 : 0;
  if (replays) *replays = b->tune.launches;
  if (switches) *switches = b->tune.switches;
  return PIC_OK;
}

pic_status pic_batch_emission_split(pic_batch* b, int64_t max_push_chunks) {
  if (!b || max_push_chunks < 0) return PIC_ERR_ARG;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return PIC_ERR_DEVICE;
  for (int i = 0; i < b->B; ++i) {
    GapDev G;
    pic_status st = read_desc(b, i, &G);
    if (st != PIC_OK) return st;
    G.emit_split = max_push_chunks;
    st = write_desc(b, i, &G);
    if (st != PIC_OK) return st;
  }
  return PIC_OK;
}

pic_status pic_emission_split(pic_gap* g, int64_t max_push_chunks) {
  if (!g) return PIC_ERR_ARG;
  return pic_batch_emission_split(g->b, max_push_chunks);
}

pic_status pic_tuning(pic_gap* g, int32_t* sort_every, int32_t* autotuned, int64_t* replays,
                      int32_t* switches) {
  if (!g) return PIC_ERR_ARG;
  return pic_batch_tuning(g->b, sort_every, autotuned, replays, switches);
}

pic_status pic_batch_read_push_time(pic_batch* b, double* ms, int64_t* launches) {
  if (!b) return PIC_ERR_ARG;
  pic_status st = drain_events(b);
  if (st != PIC_OK) return st;
  if (ms) *ms = b->prof_ms;
  if (launches) *launches = b->prof_launches;
  return PIC_OK;
}

pic_status pic_profile_push(pic_gap* g, int32_t enable) {
  if (!g || !g->standalone) return PIC_ERR_ARG;
  return pic_batch_profile_push(g->b, enable);
}

pic_status pic_read_push_time(pic_gap* g, double* ms, int64_t* launches) {
  if (!g || !g->standalone) return PIC_ERR_ARG;
  return pic_batch_read_push_time(g->b, ms, launches);
}

const char* pic_status_string(pic_status s) {
  switch (s) {
    case PIC_OK: return "ok";
    case PIC_ERR_ARG: return "invalid argument";
    case PIC_ERR_WORKSPACE: return "workspace too small or misaligned";
    case PIC_ERR_CAPACITY: return "particle or photon capacity exhausted";
    case PIC_ERR_DEVICE: return "HIP runtime error";
    case PIC_ERR_STATE: return "invalid call order or frozen gap";
    case PIC_ERR_NONFINITE: return "non-finite momentum";
    case PIC_ERR_EMISSION: return "more than 64 emissions in one step";
    case PIC_ERR_SLOTS: return "lepton slots held by absorbed leptons exhausted before the next re-sort";
    default: return "unknown status";
  }
}

}  // extern "C"
