// libprop C ABI: argument validation, transform planning, cached kernel
// spectra / chirp vectors / twiddle tables, per-stream workspace, and the
// pass sequences of every propagator and its adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <filesystem>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "libprop.h"
#include "cache.hpp"
#include "tune_cache.hpp"
#include "kernels.hpp"
#include "validate.hpp"

namespace lp {

static thread_local int g_last_hip = 0;

static int dev_err(hipError_t e) {
  g_last_hip = (int)e;
  return e == hipErrorOutOfMemory ? PROP_ENOMEM : PROP_EDEVICE;
}
#define LP_TRY(expr)                       \
  do {                                     \
    hipError_t e_ = (expr);                \
    if (e_ != hipSuccess) return dev_err(e_); \
  } while (0)
#define LP_RET(expr)          \
  do {                        \
    int r_ = (expr);          \
    if (r_ < 0) return r_;    \
  } while (0)

static const double kPi = 3.14159265358979323846;

// ------------------------------------------------------------- tracing --
// When enabled, every hot-path launch is bracketed by a pair of hipEvents
// recorded on the caller's stream, tagged with the pass name and its
// algorithmic bytes (compulsory reads + writes of that launch).
struct TraceRec {
  const char* name;
  hipEvent_t a, b;
  double bytes;
};
struct Tracer {
  bool on = false;
  std::string only;  // pass name to trace; empty: every pass
  std::vector<TraceRec> recs;
  std::vector<hipEvent_t> pool;
  bool want(const char* name) const { return on && (only.empty() || only == name); }
};
static Tracer& tracer() {
  static Tracer* t = new Tracer();
  return *t;
}
static bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}
static hipEvent_t take_event() {
  Tracer& t = tracer();
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
#define LP_TRACE(NAME, BYTES, S, EXPR)                                                  \
  do {                                                                                  \
    Tracer& tr_ = tracer();                                                             \
    hipEvent_t ea_ = nullptr, eb_ = nullptr;                                            \
    if (tr_.want(NAME) && !capturing(S)) {                                              \
      ea_ = take_event();                                                               \
      eb_ = take_event();                                                               \
      if (ea_) (void)hipEventRecord(ea_, S);                                            \
    }                                                                                   \
    hipError_t e_ = (EXPR);                                                             \
    if (ea_ && eb_) {                                                                   \
      (void)hipEventRecord(eb_, S);                                                     \
      tr_.recs.push_back(TraceRec{NAME, ea_, eb_, (double)(BYTES)});                    \
    }                                                                                   \
    if (e_ != hipSuccess) return dev_err(e_);                                           \
  } while (0)

// Twiddle table of the schedule that element type T runs at length n:
// stage s >= 1 holds W_{Ns R}^{r k} (forward sign), computed in long double,
// at off_s + k R + r (r = 0..R-1) in the per-thread layout, else at
// off_s + (r-1) Ns + k (r = 1..R-1); both the layout and the schedule follow
// the element type, as in the engine (tw_per_thread, SchedOf); sched 1: the
// length's alternative schedule.
template <typename T>
static bool make_twiddles(int n, int sched, std::vector<long double>& twr, std::vector<long double>& twi) {
  constexpr bool per_thread = tw_per_thread<T>();
  SchedInfo si;
  if (!sched_info(n, &si, sizeof(T) == 8, sched != 0)) return false;
  twr.clear();
  twi.clear();
  long ns = 1;
  for (int s = 0; s < si.nst; ++s) {
    const int R = si.rad[s];
    if (s > 0) {
      const long span = ns * R;
      auto put = [&](long k, int r) {
        const long m = (r * k) % span;
        const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)span;
        twr.push_back(cosl(ang));
        twi.push_back(sinl(ang));
      };
      if (per_thread) {
        for (long k = 0; k < ns; ++k)
          for (int r = 0; r < R; ++r) put(k, r);
      } else {
        for (int r = 1; r < R; ++r)
          for (long k = 0; k < ns; ++k) put(k, r);
      }
    }
    ns *= R;
  }
  if (twr.empty()) {
    twr.push_back(1.0L);
    twi.push_back(0.0L);
  }
  return true;
}

// --------------------------------------------------------------- context --
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct TwEntry {
  void* tw = nullptr;
};

// Tables generated on a stream carry an event recorded after their last
// generating kernel.  A call on another stream makes that stream wait for
// the event (on the device, no host synchronisation) until the host has
// seen it complete.
struct Ready {
  hipEvent_t ev = nullptr;
  hipStream_t gen = nullptr;
  bool done = true;
};

struct SpecEntry {
  void* q[4] = {nullptr, nullptr, nullptr, nullptr};  // kinds: H, (X/z)H, (Y/z)H, dH/dz
  int Mx = 0, My = 0;
  Ready ready;
};

struct ZoomEntry {
  void* pre = nullptr;
  void* post = nullptr;
  void* chat = nullptr;
  Ready ready;
};

using TwKey = std::tuple<int, int, int, int>;  // (device, element size, length, schedule)
using SpecKey = std::tuple<int, int, int, int, double, double, double, double, int>;
using ZoomKey = std::tuple<int, int, int, double, double, double, double, double, double, double, double, double,
                           int, int, int>;

// Autotuner record: per (device, element size, pass kind, length, lines,
// valid input length, kept output length, batch) the chosen launch variant
// and the measured time of each variant (ms; < 0 = not a distinct variant).
using TuneKey = std::tuple<int, int, int, int, int, int, int, int>;
struct TuneEntry {
  int variant = 0;
  float ms[kColVariants * kSchedVariants] = {-1.f, -1.f, -1.f, -1.f, -1.f, -1.f};
  bool from_file = false;  // read from the tuning cache file, not timed here
};
static_assert(kColVariants * kSchedVariants == kTuneCandidates, "tuning candidates");

// Tables a plan holds pins on (released by prop_plan_destroy).
struct Pins {
  std::vector<TwKey> tw;
  std::vector<SpecKey> spec;
  std::vector<ZoomKey> zoom;
};

// Default byte budget of the cached kernel spectra and zoom vectors
// (LIBPROP_CACHE_MB overrides it; prop_cache_set_limit at run time).
static size_t default_cache_limit() {
  const char* e = std::getenv("LIBPROP_CACHE_MB");
  const long long mb = e ? std::atoll(e) : 0;
  return mb > 0 ? (size_t)mb << 20 : (size_t)8 << 30;
}

struct Ctx {
  std::mutex mu;
  uint64_t epoch = 0;  // one per locked library call
  size_t limit = default_cache_limit();
  TableCache<TwKey, TwEntry> tws;
  TableCache<SpecKey, SpecEntry> specs;
  TableCache<ZoomKey, ZoomEntry> zooms;
  std::map<std::pair<int, hipStream_t>, Buf> work;
  std::map<std::pair<int, hipStream_t>, Buf> gen_scratch;  // complex128 table-generation scratch per stream
  std::map<TuneKey, TuneEntry> tuned;
  std::map<int, Buf> tune_a, tune_b;  // autotuner scratch per device
  Pins* pins = nullptr;               // set while a plan warms its tables
  uint64_t evict_syncs = 0;           // device synchronisations of eviction rounds
  // tuning cache file: records read (by architecture and shape), lines rejected
  std::string tune_path;
  bool tune_path_set = false, tune_loaded = false;
  std::map<std::tuple<std::string, int, int, int, int, int, int, int>, int> tune_file;
  int tune_rejected = 0;
};

static Ctx& ctx() {
  static Ctx* c = new Ctx();
  return *c;
}

// The library mutex, held for a whole call; each call is one cache epoch.
struct CtxLock {
  std::unique_lock<std::mutex> lk;
  CtxLock() : lk(ctx().mu) { ++ctx().epoch; }
};

static int cur_device(int* dev) {
  LP_TRY(hipGetDevice(dev));
  return PROP_OK;
}

static int ensure_buf(Buf& b, size_t bytes, hipStream_t s) {
  if (b.bytes >= bytes && b.p) return PROP_OK;
  if (b.p) {
    LP_TRY(hipStreamSynchronize(s));
    LP_TRY(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, 1 << 20);
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return dev_err(e);
  }
  b.bytes = want;
  return PROP_OK;
}

// ------------------------------------------------------ table lifetime --
static int ready_mark(Ready& r, hipStream_t s) {
  if (!r.ev) LP_TRY(hipEventCreateWithFlags(&r.ev, hipEventDisableTiming));
  LP_TRY(hipEventRecord(r.ev, s));
  r.gen = s;
  r.done = false;
  return PROP_OK;
}

static int ready_wait(Ready& r, hipStream_t s) {
  if (r.done || s == r.gen) return PROP_OK;  // complete, or ordered by the stream itself
  const hipError_t q = hipEventQuery(r.ev);
  if (q == hipSuccess) {
    r.done = true;
    return PROP_OK;
  }
  if (q != hipErrorNotReady) return dev_err(q);
  (void)hipGetLastError();
  LP_TRY(hipStreamWaitEvent(s, r.ev, 0));
  return PROP_OK;
}

static void release_spec(SpecEntry& e) {
  for (int k = 0; k < 4; ++k)
    if (e.q[k]) (void)hipFree(e.q[k]);
  if (e.ready.ev) (void)hipEventDestroy(e.ready.ev);
}

static void release_zoom(ZoomEntry& e) {
  (void)hipFree(e.pre);
  (void)hipFree(e.post);
  (void)hipFree(e.chat);
  if (e.ready.ev) (void)hipEventDestroy(e.ready.ev);
}

// Evict least recently used, unpinned spectra and zoom vectors of earlier
// calls until their bytes fall to `target`.  Kernels already enqueued may
// still read a victim, so one device synchronisation precedes each round's
// frees; rounds start above the budget and go down to 3/4 of it, so a
// distance-optimisation loop pays that synchronisation once per many new
// distances, not per call.
static void evict_tables(Ctx& C, size_t target) {
  bool synced = false;
  auto before = [&](size_t) {
    if (!synced) {
      (void)hipDeviceSynchronize();
      synced = true;
      ++C.evict_syncs;
    }
  };
  const size_t zb = C.zooms.bytes();
  C.specs.evict_to(target > zb ? target - zb : 0, C.epoch, before, release_spec);
  const size_t sb = C.specs.bytes();
  C.zooms.evict_to(target > sb ? target - sb : 0, C.epoch, before, release_zoom);
}

static void trim_tables(Ctx& C) {
  if (C.specs.bytes() + C.zooms.bytes() > C.limit) evict_tables(C, C.limit / 4 * 3);
}

// Device table allocation; on exhaustion every evictable table is dropped
// and the allocation tried once more.
static int table_alloc(Ctx& C, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    evict_tables(C, 0);
    e = hipMalloc(p, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return dev_err(e);
  }
  return PROP_OK;
}

template <typename T>
static int get_tw(int dev, int n, const cx<T>** tw, int sched = 0) {
  Ctx& C = ctx();
  const TwKey key{dev, (int)sizeof(T), n, sched};
  auto* slot = C.tws.find(key, C.epoch);
  if (!slot) {
    TwEntry e;
    std::vector<long double> wr, wi;
    if (!make_twiddles<T>(n, sched, wr, wi)) return PROP_ESHAPE;
    std::vector<cx<T>> h(wr.size());
    for (size_t i = 0; i < wr.size(); ++i) {
      h[i].x = (T)wr[i];
      h[i].y = (T)wi[i];
    }
    const size_t bytes = h.size() * sizeof(cx<T>);
    LP_RET(table_alloc(C, &e.tw, bytes));
    const hipError_t er = hipMemcpy(e.tw, h.data(), bytes, hipMemcpyHostToDevice);
    if (er != hipSuccess) {
      (void)hipFree(e.tw);
      return dev_err(er);
    }
    slot = C.tws.insert(key, e, bytes, C.epoch);
  }
  if (C.pins && C.tws.pin(key)) C.pins->tw.push_back(key);
  *tw = (const cx<T>*)slot->v.tw;
  return PROP_OK;
}

// ----------------------------------------------------- RS kernel spectra --
template <typename T>
static int get_rs_spectra(int dev, const prop_grid* g, double wl, double z, int kinds, hipStream_t s,
                          const cx<T>* q[4], int* Mx_out, int* My_out) {
  Ctx& C = ctx();
  const int Mx = fft_len(2 * g->nx - 1), My = fft_len(2 * g->ny - 1);
  *Mx_out = Mx;
  *My_out = My;
  const SpecKey key{dev, (int)sizeof(T), g->nx, g->ny, g->dx, g->dy, wl, z, 0};
  auto* slot = C.specs.find(key, C.epoch);
  if (!slot) {
    SpecEntry fresh;
    fresh.Mx = Mx;
    fresh.My = My;
    slot = C.specs.insert(key, fresh, 0, C.epoch);
  }
  SpecEntry& e = slot->v;
  bool need = false;
  for (int k = 0; k < 4; ++k) need |= ((kinds >> k) & 1) && e.q[k] == nullptr;
  if (need) {
    // generated on the caller's stream: the FP64 kernel samples, their FP64
    // transform and the half-table extraction share the stream's scratch,
    // which stream order keeps from being reused early
    const cx<double> *twx, *twy;
    LP_RET(get_tw<double>(dev, Mx, &twx));
    LP_RET(get_tw<double>(dev, My, &twy));
    Buf& sb = C.gen_scratch[{dev, s}];
    LP_RET(ensure_buf(sb, (size_t)Mx * My * sizeof(cx<double>), s));
    LP_RET(ready_wait(e.ready, s));
    cx<double>* full = (cx<double>*)sb.p;
    const size_t qbytes = (size_t)((Mx + 3) / 4 * 4) * (My / 2 + 1) * sizeof(cx<T>);
    const double k = 2.0 * kPi / wl;
    for (int kind = 0; kind < 4; ++kind) {
      if (!((kinds >> kind) & 1) || e.q[kind]) continue;
      void* qp = nullptr;
      LP_RET(table_alloc(C, &qp, qbytes));
      hipError_t er = launch_rs_kernel_wrapped(full, Mx, My, g->nx, g->ny, g->dx, g->dy, k, z, kind, s);
      if (er == hipSuccess)
        er = launch_fft_lines<double, -1>(Mx, false, full, full, Lines{0, Mx}, Lines{0, Mx}, My, Mx, Mx, 1.0, 1, twx, s);
      if (er == hipSuccess)
        er = launch_fft_lines<double, -1>(My, true, full, full, Lines{0, Mx}, Lines{0, Mx}, Mx, My, My, 1.0, 1, twy, s);
      if (er == hipSuccess) er = launch_extract_half<T>(full, (cx<T>*)qp, Mx, My, s);
      if (er != hipSuccess) {
        (void)hipFree(qp);
        return dev_err(er);
      }
      e.q[kind] = qp;
      C.specs.add_bytes(key, qbytes);
    }
    LP_RET(ready_mark(e.ready, s));
    trim_tables(C);
  } else {
    LP_RET(ready_wait(e.ready, s));
  }
  if (C.pins && C.specs.pin(key)) C.pins->spec.push_back(key);
  for (int kk = 0; kk < 4; ++kk) q[kk] = (const cx<T>*)e.q[kk];
  return PROP_OK;
}

// ----------------------------------------------------------- autotuner --
// The column and Bluestein passes have launch variants (col_pass_lines):
// lines per workgroup on the built-in schedule (bit-identical results) and,
// for FP32 lengths with an alternative schedule, the same on that schedule
// (different rounding).  When tuning is on, the first launch of each new
// shape takes its choice from the tuning cache file if that holds a valid
// record for this GPU architecture, and otherwise times every distinct
// candidate on scratch buffers of the same size (one warm-up and three
// timed launches each, HIP events on the caller's stream), keeps the
// fastest and appends it to the file.  Later launches of that shape reuse
// the choice, so a tuned plan keeps it for its lifetime.  Tuning is on with
// LIBPROP_AUTOTUNE=1 in the environment, or for the first execution of a
// plan created with PROP_PLAN_AUTOTUNE; never while the stream is being
// captured (the built-in variant 0 is used then).  Untuned calls never read
// the file.
enum { TUNE_RS_COLS = 0, TUNE_MIX2 = 1, TUNE_CZT_COLS = 2, TUNE_CZT_ROWS = 3 };
static thread_local bool t_tune_request = false;

static bool tune_enabled() {
  static const bool env = [] {
    const char* e = std::getenv("LIBPROP_AUTOTUNE");
    return e && std::atoi(e) != 0;
  }();
  return env || t_tune_request;
}

// Tuning cache file: prop_tune_cache_path's argument, else
// LIBPROP_TUNE_CACHE, else $XDG_CACHE_HOME/libprop/tune.txt or
// $HOME/.cache/libprop/tune.txt ("" disables it).
static std::string tune_file_path(Ctx& C) {
  if (C.tune_path_set) return C.tune_path;
  const char* e = std::getenv("LIBPROP_TUNE_CACHE");
  if (e) return e;
  const char* x = std::getenv("XDG_CACHE_HOME");
  if (x && *x) return std::string(x) + "/libprop/tune.txt";
  const char* h = std::getenv("HOME");
  if (h && *h) return std::string(h) + "/.cache/libprop/tune.txt";
  return "";
}

static std::string device_arch(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

// Valid candidate of its shape (the record's length must be a supported
// transform length and the variant one of that length's candidates).
static bool tune_record_usable(const TuneRecord& r) {
  if (fft_len(r.n) != r.n) return false;
  return (r.elem == 4 ? col_pass_lines<float>(r.kind, r.n, r.variant)
                      : col_pass_lines<double>(r.kind, r.n, r.variant)) > 0;
}

// Read the file once (a missing or unreadable file is empty; malformed or
// unusable lines are skipped and counted; a later line for a shape wins).
static void tune_file_load(Ctx& C) {
  if (C.tune_loaded) return;
  C.tune_loaded = true;
  const std::string path = tune_file_path(C);
  if (path.empty()) return;
  std::ifstream f(path);
  std::string line;
  while (f && std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    TuneRecord r;
    if (!parse_tune_record(line, &r) || !tune_record_usable(r)) {
      ++C.tune_rejected;
      continue;
    }
    C.tune_file[{r.arch, r.elem, r.kind, r.n, r.lines, r.n_in, r.n_out, r.batch}] = r.variant;
  }
}

static void tune_file_append(Ctx& C, const TuneRecord& r) {
  const std::string path = tune_file_path(C);
  if (path.empty()) return;
  std::error_code ec;
  const std::filesystem::path dir = std::filesystem::path(path).parent_path();
  if (!dir.empty()) std::filesystem::create_directories(dir, ec);
  std::ofstream f(path, std::ios::app);
  if (f) f << format_tune_record(r) << '\n';  // a cache: a failed write only costs a retune later
}

template <typename T, class Launch>
static int col_variant(int dev, int kind, int n, int nlines, int n_in, int n_out, int batch, size_t elems_a,
                       size_t elems_b, hipStream_t s, Launch launch, int* variant) {
  Ctx& C = ctx();
  const TuneKey key{dev, (int)sizeof(T), kind, n, nlines, n_in, n_out, batch};
  auto it = C.tuned.find(key);
  if (it != C.tuned.end()) {
    *variant = it->second.variant;
    return PROP_OK;
  }
  // untuned: the built-in variant (for RS column passes the bit-identical
  // one that fills the chip, rs_cols_fill_variant)
  *variant = kind == TUNE_RS_COLS ? rs_cols_fill_variant<T>(n, nlines, n_in, batch) : 0;
  if (!tune_enabled() || capturing(s)) return PROP_OK;
  TuneRecord rec;
  rec.arch = device_arch(dev);
  rec.elem = (int)sizeof(T);
  rec.kind = kind;
  rec.n = n;
  rec.lines = nlines;
  rec.n_in = n_in;
  rec.n_out = n_out;
  rec.batch = batch;
  tune_file_load(C);
  auto ft = C.tune_file.find({rec.arch, rec.elem, kind, n, nlines, n_in, n_out, batch});
  if (ft != C.tune_file.end()) {
    TuneEntry te;
    te.variant = ft->second;
    te.from_file = true;
    C.tuned[key] = te;
    *variant = te.variant;
    return PROP_OK;
  }
  Buf& ba = C.tune_a[dev];
  Buf& bb = C.tune_b[dev];
  LP_RET(ensure_buf(ba, std::max<size_t>(elems_a, 1) * sizeof(cx<T>), s));
  LP_RET(ensure_buf(bb, std::max<size_t>(elems_b, 1) * sizeof(cx<T>), s));
  LP_TRY(hipMemsetAsync(ba.p, 0, ba.bytes, s));
  LP_TRY(hipMemsetAsync(bb.p, 0, bb.bytes, s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  LP_TRY(hipEventCreate(&e0));
  hipError_t er = hipEventCreate(&e1);
  if (er != hipSuccess) {
    (void)hipEventDestroy(e0);
    return dev_err(er);
  }
  TuneEntry te;
  float best = 0.f;
  bool have = false;
  int seen[kTuneCandidates] = {};
  er = hipSuccess;
  for (int v = 0; v < kTuneCandidates && er == hipSuccess; ++v) {
    // distinct candidates only: a lines count already timed on the same
    // schedule gives the same launch
    const int lines = col_pass_lines<T>(kind, n, v);
    bool dup = lines <= 0;
    for (int u = (v / kColVariants) * kColVariants; u < v; ++u) dup = dup || seen[u] == lines;
    seen[v] = lines;
    if (dup) continue;
    er = launch(v, (cx<T>*)ba.p, (cx<T>*)bb.p);
    if (er == hipSuccess) er = hipEventRecord(e0, s);
    for (int rep = 0; rep < 3 && er == hipSuccess; ++rep) er = launch(v, (cx<T>*)ba.p, (cx<T>*)bb.p);
    if (er == hipSuccess) er = hipEventRecord(e1, s);
    if (er == hipSuccess) er = hipEventSynchronize(e1);
    float ms = 0.f;
    if (er == hipSuccess) er = hipEventElapsedTime(&ms, e0, e1);
    if (er != hipSuccess) break;
    te.ms[v] = ms / 3.f;
    if (!have || te.ms[v] < best) {
      best = te.ms[v];
      te.variant = v;
      have = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (er != hipSuccess) return dev_err(er);
  C.tuned[key] = te;
  *variant = te.variant;
  rec.variant = te.variant;
  C.tune_file[{rec.arch, rec.elem, kind, n, nlines, n_in, n_out, batch}] = te.variant;
  tune_file_append(C, rec);
  return PROP_OK;
}

// The tuned variant of a column or Bluestein pass and the twiddle table of
// the schedule it runs.  launch(var, tw, a, b) launches candidate var on
// scratch buffers a, b with twiddles tw.
template <typename T, class Launch>
static int tuned_pass(int dev, int kind, int n, int nlines, int n_in, int n_out, int batch, size_t elems_a,
                      size_t elems_b, hipStream_t s, Launch launch, int* variant, const cx<T>** tw) {
  const cx<T>* twc[kSchedVariants] = {nullptr, nullptr};
  LP_RET(get_tw<T>(dev, n, &twc[0], 0));
  const bool alt = col_pass_lines<T>(kind, n, kColVariants) > 0;
  if (alt && tune_enabled() && !capturing(s)) LP_RET(get_tw<T>(dev, n, &twc[1], 1));
  LP_RET(col_variant<T>(dev, kind, n, nlines, n_in, n_out, batch, elems_a, elems_b, s,
                        [&](int var, cx<T>* a, cx<T>* b) { return launch(var, twc[variant_sched(var)], a, b); },
                        variant));
  const int sc = variant_sched(*variant);
  if (sc && !twc[sc]) LP_RET(get_tw<T>(dev, n, &twc[sc], sc));
  *tw = twc[sc];
  return PROP_OK;
}

// --------------------------------------------------------- zoom vectors --
template <typename T>
static int get_zoom(int dev, const ZoomSpec& zs, hipStream_t s, const cx<T>** pre, const cx<T>** post,
                    const cx<T>** chat) {
  Ctx& C = ctx();
  const ZoomKey key{dev,    (int)sizeof(T), zs.sigma, zs.beta,  zs.x0,   zs.dx,   zs.X0,  zs.dX,
                    zs.qin, zs.qout,       zs.Kre,   zs.Kim,   zs.n_in, zs.n_out, zs.L};
  auto* slot = C.zooms.find(key, C.epoch);
  if (!slot) {
    ZoomEntry e;
    const cx<double>* twL;
    LP_RET(get_tw<double>(dev, zs.L, &twL));
    Buf& sb = C.gen_scratch[{dev, s}];
    LP_RET(ensure_buf(sb, (size_t)zs.L * sizeof(cx<double>), s));
    cx<double>* chirp = (cx<double>*)sb.p;
    const size_t bytes = ((size_t)zs.n_in + zs.n_out + zs.L) * sizeof(cx<T>);
    auto fail = [&](int r) {
      (void)hipFree(e.pre);
      (void)hipFree(e.post);
      (void)hipFree(e.chat);
      return r;
    };
    int r = table_alloc(C, &e.pre, (size_t)zs.n_in * sizeof(cx<T>));
    if (r == PROP_OK) r = table_alloc(C, &e.post, (size_t)zs.n_out * sizeof(cx<T>));
    if (r == PROP_OK) r = table_alloc(C, &e.chat, (size_t)zs.L * sizeof(cx<T>));
    if (r < 0) return fail(r);
    hipError_t er = launch_zoom_vectors<T>(zs, (cx<T>*)e.pre, (cx<T>*)e.post, chirp, s);
    if (er == hipSuccess)
      er = launch_fft_lines<double, -1>(zs.L, false, chirp, chirp, Lines{0, zs.L}, Lines{0, zs.L}, 1, zs.L, zs.L, 1.0,
                                        1, twL, s);
    if (er == hipSuccess) er = launch_convert<T>(chirp, (cx<T>*)e.chat, zs.L, s);
    if (er != hipSuccess) return fail(dev_err(er));
    r = ready_mark(e.ready, s);
    if (r < 0) return fail(r);
    slot = C.zooms.insert(key, e, bytes, C.epoch);
    trim_tables(C);
  } else {
    LP_RET(ready_wait(slot->v.ready, s));
  }
  if (C.pins && C.zooms.pin(key)) C.pins->zoom.push_back(key);
  *pre = (const cx<T>*)slot->v.pre;
  *post = (const cx<T>*)slot->v.post;
  *chat = (const cx<T>*)slot->v.chat;
  return PROP_OK;
}


// ------------------------------------------------------------- RS runs --
static size_t rs_work_bytes(prop_dtype t, const prop_grid* g, int batch) {
  return (size_t)rs_plane_elems(g->ny, fft_len(2 * g->nx - 1)) * batch * esize(t);
}

template <typename T>
static int rs_run(const void* in, void* out, const prop_grid* g, double wl, double z, int batch, hipStream_t s,
                  bool adjoint, void* work, int spec_kind = 0, const cx<T>* pg_u = nullptr, T* pg_grad = nullptr,
                  int pg_acc = 0, const Slm<T>* slm = nullptr) {
  int dev;
  LP_RET(cur_device(&dev));
  const cx<T>* q[4];
  int Mx, My;
  LP_RET(get_rs_spectra<T>(dev, g, wl, z, 1 << spec_kind, s, q, &Mx, &My));
  q[0] = q[spec_kind];
  const cx<T> *twx, *twy;
  LP_RET(get_tw<T>(dev, Mx, &twx));
  LP_RET(get_tw<T>(dev, My, &twy));
  const int nx = g->nx, ny = g->ny;
  const int64_t plane = rs_plane_elems(ny, Mx);
  cx<T>* W = (cx<T>*)work;
  const T scale = (T)(g->dx * g->dy / ((double)Mx * (double)My));
  // P1: row transforms of the ny input rows, zero-padded to Mx, into the
  // tiled workspace
  const double es = sizeof(cx<T>);
  const double qel = (double)Mx * (My / 2 + 1);  // half spectrum table
  // (a plan setup's SLM stage rides on this pass's loads in the forward)
  const double stage_bytes = (slm && slm->phase && !adjoint) ? (double)sizeof(T) * batch * ny * nx : 0.0;
  LP_TRACE("rs_rows_fwd", es * batch * ny * (double)(nx + Mx) + stage_bytes, s,
           (launch_rs_rows<T, -1>(Mx, (const cx<T>*)in, W, plane, ny, nx, T(1), batch, twx, s, nullptr, nullptr, 0,
                                  adjoint ? nullptr : slm)));
  // P2: column transform, kernel-spectrum multiply, inverse, first ny rows
  int v = 0;
  const cx<T>* twc = twy;
  LP_RET(tuned_pass<T>(dev, TUNE_RS_COLS, My, Mx, ny, ny, batch, (size_t)plane * batch, 0, s,
                       [&](int var, const cx<T>* tw, cx<T>* a, cx<T>*) {
                         return launch_rs_cols<T>(My, a, plane, Mx, ny, q[0], Mx, adjoint, batch, tw, s, var);
                       },
                       &v, &twc));
  LP_TRACE("rs_cols", es * (2.0 * batch * ny * Mx + qel), s,
           launch_rs_cols<T>(My, W, plane, Mx, ny, q[0], Mx, adjoint, batch, twc, s, v));
  // P3: inverse row transforms, crop to nx, scale dx dy / (Mx My)
  // inverse pass: reads the workspace rows, writes the field (and with the
  // fused phase gradient reads u, writes (and reads when accumulating) grad)
  // (and in the adjoint on its stores)
  const double inv_bytes =
      (double)batch * ny *
      (es * Mx + (out ? es * nx : 0.0) + (pg_grad ? (es + sizeof(T) * (pg_acc ? 2.0 : 1.0)) * nx : 0.0) +
       ((slm && slm->phase && adjoint) ? (double)sizeof(T) * nx : 0.0));
  LP_TRACE("rs_rows_inv", inv_bytes, s,
           (launch_rs_rows<T, 1>(Mx, W, (cx<T>*)out, plane, ny, nx, scale, batch, twx, s, pg_u, pg_grad, pg_acc,
                                 adjoint ? slm : nullptr)));
  return PROP_OK;
}

static int rs_entry(prop_dtype t, const void* in, void* out, const prop_grid* g, double wl, double z, int32_t batch,
                    void* stream, bool adjoint) {
  LP_RET(check_common(t, batch, wl));
  LP_RET(check_grid(g));
  if (!(z > 0) || !is_finite(z)) return PROP_EPARAM;
  if (fft_len(2 * g->nx - 1) < 0 || fft_len(2 * g->ny - 1) < 0) return PROP_ESHAPE;
  const int warn = sampling(g, wl, z);
  if (batch == 0) return warn;
  if (!in || !out) return PROP_ENULL;
  const size_t bytes = (size_t)g->nx * g->ny * batch * esize(t);
  LP_RET(check_alias({{in, bytes}}, {{out, bytes}}));
  CtxLock lk;
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, rs_work_bytes(t, g, batch), s));
  int r = t == PROP_C64 ? rs_run<float>(in, out, g, wl, z, batch, s, adjoint, wb.p)
                        : rs_run<double>(in, out, g, wl, z, batch, s, adjoint, wb.p);
  return r < 0 ? r : warn;
}

// ------------------------------------------------------------ VRS runs --
static size_t vrs_work_bytes(prop_dtype t, const prop_grid* g, int batch) { return 3 * rs_work_bytes(t, g, batch); }

template <typename T>
static int vrs_run(const void* const* ins, int nin, void* const* outs, int nout, const prop_grid* g, double wl,
                   double z, int batch, hipStream_t s, bool adjoint, void* work) {
  int dev;
  LP_RET(cur_device(&dev));
  const cx<T>* q[4];
  int Mx, My;
  LP_RET(get_rs_spectra<T>(dev, g, wl, z, 7, s, q, &Mx, &My));
  const cx<T> *twx, *twy;
  LP_RET(get_tw<T>(dev, Mx, &twx));
  LP_RET(get_tw<T>(dev, My, &twy));
  const int nx = g->nx, ny = g->ny;
  const int64_t pst = rs_plane_elems(ny, Mx);
  const size_t plane = (size_t)pst * batch;
  cx<T>* W[3];
  for (int i = 0; i < 3; ++i) W[i] = (cx<T>*)work + i * plane;
  const double es = sizeof(cx<T>);
  const double qel = (double)Mx * (My / 2 + 1);  // half spectrum table
  const double pl = (double)batch * ny * Mx;
  for (int i = 0; i < nin; ++i)
    LP_TRACE("rs_rows_fwd", es * batch * ny * (double)(nx + Mx), s,
             (launch_rs_rows<T, -1>(Mx, (const cx<T>*)ins[i], W[i], pst, ny, nx, T(1), batch, twx, s)));
  int vm = 0, vc = 0;
  LP_RET(col_variant<T>(dev, TUNE_MIX2, My, Mx, ny, ny, batch, (size_t)pst * batch, (size_t)pst * batch, s,
                        [&](int var, cx<T>* a, cx<T>* b) {
                          return launch_mix2_cols<T>(My, a, b, a, pst, Mx, ny, q[1], 1, T(-1), q[2], 2, T(-1),
                                                     false, Mx, batch, twy, s, var);
                        },
                        &vm));
  const cx<T>* twc = twy;
  if (!adjoint) {
    LP_RET(tuned_pass<T>(dev, TUNE_RS_COLS, My, Mx, ny, ny, batch, (size_t)pst * batch, 0, s,
                         [&](int var, const cx<T>* tw, cx<T>* a, cx<T>*) {
                           return launch_rs_cols<T>(My, a, pst, Mx, ny, q[0], Mx, false, batch, tw, s, var);
                         },
                         &vc, &twc));
    // E_z = -(Hx * E_x0 + Hy * E_y0) first (reads W0, W1), then E_x, E_y in place
    LP_TRACE("vrs_mix2", es * (3.0 * pl + 2.0 * qel), s,
             launch_mix2_cols<T>(My, W[0], W[1], W[2], pst, Mx, ny, q[1], 1, T(-1), q[2], 2, T(-1), false, Mx,
                                 batch, twy, s, vm));
    LP_TRACE("rs_cols", es * (2.0 * pl + qel), s,
             launch_rs_cols<T>(My, W[0], pst, Mx, ny, q[0], Mx, false, batch, twc, s, vc));
    LP_TRACE("rs_cols", es * (2.0 * pl + qel), s,
             launch_rs_cols<T>(My, W[1], pst, Mx, ny, q[0], Mx, false, batch, twc, s, vc));
  } else {
    // g_ex = H^H g_x - Hx^H g_z, g_ey = H^H g_y - Hy^H g_z (in place over W0, W1)
    LP_TRACE("vrs_mix2", es * (3.0 * pl + 2.0 * qel), s,
             launch_mix2_cols<T>(My, W[0], W[2], W[0], pst, Mx, ny, q[0], 0, T(1), q[1], 1, T(-1), true, Mx,
                                 batch, twy, s, vm));
    LP_TRACE("vrs_mix2", es * (3.0 * pl + 2.0 * qel), s,
             launch_mix2_cols<T>(My, W[1], W[2], W[1], pst, Mx, ny, q[0], 0, T(1), q[2], 2, T(-1), true, Mx,
                                 batch, twy, s, vm));
  }
  const T scale = (T)(g->dx * g->dy / ((double)Mx * (double)My));
  const int src[3] = {adjoint ? 0 : 0, 1, 2};
  for (int i = 0; i < nout; ++i)
    LP_TRACE("rs_rows_inv", es * batch * ny * (double)(nx + Mx), s,
             (launch_rs_rows<T, 1>(Mx, W[src[i]], (cx<T>*)outs[i], pst, ny, nx, scale, batch, twx, s)));
  return PROP_OK;
}

// ------------------------------------------------------------ CZT runs --
static ZoomSpec zoom_spec(int sigma, double beta, int n_in, double x0, double dx, int n_out, double X0, double dX,
                          double qin, double qout, double Kre, double Kim) {
  ZoomSpec z;
  z.sigma = sigma;
  z.beta = beta;
  z.x0 = x0;
  z.dx = dx;
  z.X0 = X0;
  z.dX = dX;
  z.qin = qin;
  z.qout = qout;
  z.Kre = Kre;
  z.Kim = Kim;
  z.n_in = n_in;
  z.n_out = n_out;
  z.L = fft_len(n_in + n_out - 1);
  return z;
}

static double first_x(const prop_grid* g) { return g->cx - (double)(g->nx / 2) * g->dx; }
static double first_y(const prop_grid* g) { return g->cy - (double)(g->ny / 2) * g->dy; }

// Separable zoom transform: rows (x) then columns (y) for "forward" shapes
// (input grid gi -> output grid go).  zx / zy describe the 1-D transforms.
template <typename T>
static int zoom2d_run(int dev, const cx<T>* in, cx<T>* out, int nxi, int nyi, int nxo, int nyo, const ZoomSpec& zx,
                      const ZoomSpec& zy, int batch, cx<T>* tmp, hipStream_t s, bool cols_first,
                      const cx<T>* pg_u = nullptr, T* pg_grad = nullptr, int pg_acc = 0,
                      const Slm<T>* slm = nullptr) {
  // a plan setup's SLM stage: on the first pass's loads (forward) or the
  // last pass's stores (adjoint)
  const bool st_on = slm && slm->active();
  const Slm<T>* st_first = st_on && !slm->adjoint ? slm : nullptr;
  const Slm<T>* st_last = st_on && slm->adjoint ? slm : nullptr;
  const cx<T> *prex, *postx, *chatx, *prey, *posty, *chaty;
  LP_RET(get_zoom<T>(dev, zx, s, &prex, &postx, &chatx));
  LP_RET(get_zoom<T>(dev, zy, s, &prey, &posty, &chaty));
  const cx<T> *twx, *twy;
  LP_RET(get_tw<T>(dev, zx.L, &twx));
  LP_RET(get_tw<T>(dev, zy.L, &twy));
  const double es = sizeof(cx<T>);
  // tuned row pass of nrows lines, n_in -> n_out points (rows of the input
  // or of the intermediate)
  auto rows_variant = [&](int nrows, int rin, int rout, int* vr, const cx<T>** twr) {
    const Lines ri{(int64_t)nrows * rin, rin}, ro{(int64_t)nrows * rout, rout};
    return tuned_pass<T>(dev, TUNE_CZT_ROWS, zx.L, nrows, rin, rout, batch, (size_t)ri.bstride * batch,
                         (size_t)ro.bstride * batch, s,
                         [&](int var, const cx<T>* tw, cx<T>* a, cx<T>* b) {
                           return launch_bluestein<T>(zx.L, false, a, b, ri, ro, nrows, rin, rout, prex, chatx, postx,
                                                      batch, tw, s, var);
                         },
                         vr, twr);
  };
  if (!cols_first) {
    // rows: [nyi][nxi] -> tmp [nyi][nxo]; cols: tmp -> out [nyo][nxo]
    int vr = 0;
    LP_RET(rows_variant(nyi, nxi, nxo, &vr, &twx));
    LP_TRACE("czt_rows", es * batch * nyi * (double)(nxi + nxo), s,
             launch_bluestein<T>(zx.L, false, in, tmp, Lines{(int64_t)nyi * nxi, nxi}, Lines{(int64_t)nyi * nxo, nxo},
                                 nyi, nxi, nxo, prex, chatx, postx, batch, twx, s, vr, nullptr, nullptr, 0, st_first));
    int v = 0;
    const Lines li{(int64_t)nyi * nxo, nxo}, lo{(int64_t)nyo * nxo, nxo};
    LP_RET(tuned_pass<T>(dev, TUNE_CZT_COLS, zy.L, nxo, nyi, nyo, batch, (size_t)li.bstride * batch,
                         (size_t)lo.bstride * batch, s,
                         [&](int var, const cx<T>* tw, cx<T>* a, cx<T>* b) {
                           return launch_bluestein<T>(zy.L, true, a, b, li, lo, nxo, nyi, nyo, prey, chaty, posty,
                                                      batch, tw, s, var);
                         },
                         &v, &twy));
    const double last_bytes =
        (double)batch * nxo *
        (es * nyi + (out ? es * nyo : 0.0) + (pg_grad ? (es + sizeof(T) * (pg_acc ? 2.0 : 1.0)) * nyo : 0.0));
    LP_TRACE("czt_cols", last_bytes, s,
             launch_bluestein<T>(zy.L, true, tmp, out, li, lo, nxo, nyi, nyo, prey, chaty, posty, batch, twy, s, v,
                                 pg_u, pg_grad, pg_acc, st_last));
  } else {
    // cols: [nyi][nxi] -> tmp [nyo][nxi]; rows: tmp -> out [nyo][nxo]
    int v = 0;
    const Lines li{(int64_t)nyi * nxi, nxi}, lo{(int64_t)nyo * nxi, nxi};
    LP_RET(tuned_pass<T>(dev, TUNE_CZT_COLS, zy.L, nxi, nyi, nyo, batch, (size_t)li.bstride * batch,
                         (size_t)lo.bstride * batch, s,
                         [&](int var, const cx<T>* tw, cx<T>* a, cx<T>* b) {
                           return launch_bluestein<T>(zy.L, true, a, b, li, lo, nxi, nyi, nyo, prey, chaty, posty,
                                                      batch, tw, s, var);
                         },
                         &v, &twy));
    LP_TRACE("czt_cols", es * batch * nxi * (double)(nyi + nyo), s,
             launch_bluestein<T>(zy.L, true, in, tmp, li, lo, nxi, nyi, nyo, prey, chaty, posty, batch, twy, s, v,
                                 nullptr, nullptr, 0, st_first));
    const double last_bytes =
        (double)batch * nyo *
        (es * nxi + (out ? es * nxo : 0.0) + (pg_grad ? (es + sizeof(T) * (pg_acc ? 2.0 : 1.0)) * nxo : 0.0));
    int vr = 0;
    LP_RET(rows_variant(nyo, nxi, nxo, &vr, &twx));
    LP_TRACE("czt_rows", last_bytes, s,
             launch_bluestein<T>(zx.L, false, tmp, out, Lines{(int64_t)nyo * nxi, nxi}, Lines{(int64_t)nyo * nxo, nxo},
                                 nyo, nxi, nxo, prex, chatx, postx, batch, twx, s, vr, pg_u, pg_grad, pg_acc,
                                 st_last));
  }
  return PROP_OK;
}

// dq: an extra quadratic phase exp(i dq (x^2 + y^2)) on the input grid,
// folded into the input-side chirp exactly (a thin lens of focal length f
// in front of the propagation: dq = -k / 2f).
static void czt_specs(const prop_grid* gi, const prop_grid* go, double wl, double z, bool adjoint, ZoomSpec* zx,
                      ZoomSpec* zy, double dq = 0.0) {
  const double k = 2.0 * kPi / wl;
  const double beta = 1.0 / (wl * z);
  const double a = gi->dx * gi->dy / (wl * z);
  const double Kre = a * std::sin(k * z), Kim = -a * std::cos(k * z);  // e^{ikz} dx dy / (i lambda z)
  const double q = k / (2.0 * z), qi = q + dq;
  if (!adjoint) {
    *zx = zoom_spec(-1, beta, gi->nx, first_x(gi), gi->dx, go->nx, first_x(go), go->dx, qi, q, 1.0, 0.0);
    *zy = zoom_spec(-1, beta, gi->ny, first_y(gi), gi->dy, go->ny, first_y(go), go->dy, qi, q, Kre, Kim);
  } else {
    *zx = zoom_spec(+1, beta, go->nx, first_x(go), go->dx, gi->nx, first_x(gi), gi->dx, -q, -qi, 1.0, 0.0);
    *zy = zoom_spec(+1, beta, go->ny, first_y(go), go->dy, gi->ny, first_y(gi), gi->dy, -q, -qi, Kre, -Kim);
  }
}

static void rw_specs(const prop_grid* gi, const prop_grid* go, double wl, const prop_lens* lens, bool adjoint,
                     ZoomSpec* zx, ZoomSpec* zy) {
  const double k = 2.0 * kPi / wl;
  const double f = lens->f;
  const double beta = 1.0 / (wl * f);
  const double a = k * f / (2.0 * kPi) * gi->dx * gi->dy / (f * f);
  const double Kre = a * std::sin(k * f), Kim = a * std::cos(k * f);  // i k f e^{-ikf}/(2 pi) dx dy / f^2
  if (!adjoint) {
    *zx = zoom_spec(+1, beta, gi->nx, first_x(gi), gi->dx, go->nx, first_x(go), go->dx, 0, 0, 1.0, 0.0);
    *zy = zoom_spec(+1, beta, gi->ny, first_y(gi), gi->dy, go->ny, first_y(go), go->dy, 0, 0, Kre, Kim);
  } else {
    *zx = zoom_spec(-1, beta, go->nx, first_x(go), go->dx, gi->nx, first_x(gi), gi->dx, 0, 0, 1.0, 0.0);
    *zy = zoom_spec(-1, beta, go->ny, first_y(go), go->dy, gi->ny, first_y(gi), gi->dy, 0, 0, Kre, -Kim);
  }
}

// scalar CZT with the caller holding the lock; tmp must hold
// batch * max(nyi*nxo, nyo*nxi) elements
template <typename T>
static int czt_core(int dev, const cx<T>* in, cx<T>* out, const prop_grid* gi, const prop_grid* go, double wl,
                    double z, int batch, cx<T>* tmp, hipStream_t s, bool adjoint, const cx<T>* pg_u = nullptr,
                    T* pg_grad = nullptr, int pg_acc = 0, const Slm<T>* slm = nullptr, double dq = 0.0) {
  ZoomSpec zx, zy;
  czt_specs(gi, go, wl, z, adjoint, &zx, &zy, dq);
  if (!adjoint) {
    const bool cols_first = (int64_t)go->ny * gi->nx < (int64_t)gi->ny * go->nx;
    return zoom2d_run<T>(dev, in, out, gi->nx, gi->ny, go->nx, go->ny, zx, zy, batch, tmp, s, cols_first, nullptr,
                         nullptr, 0, slm);
  }
  // with a fused phase gradient or SLM stage the row pass goes last, so that
  // the field and the gradient are read and written along contiguous rows
  const bool cols_first =
      (pg_grad || (slm && slm->active())) ? true : (int64_t)gi->ny * go->nx < (int64_t)go->ny * gi->nx;
  return zoom2d_run<T>(dev, in, out, go->nx, go->ny, gi->nx, gi->ny, zx, zy, batch, tmp, s, cols_first, pg_u,
                       pg_grad, pg_acc, slm);
}

static size_t czt_tmp_elems(const prop_grid* gi, const prop_grid* go) {
  return std::max((size_t)gi->ny * go->nx, (size_t)go->ny * gi->nx);
}

static size_t czt_work_bytes(prop_dtype t, const prop_grid* gi, const prop_grid* go, int batch) {
  return czt_tmp_elems(gi, go) * batch * esize(t);
}

template <typename T>
static int czt_run(const void* in, void* out, const prop_grid* gi, const prop_grid* go, double wl, double z, int batch,
                   hipStream_t s, bool adjoint, void* work) {
  int dev;
  LP_RET(cur_device(&dev));
  return czt_core<T>(dev, (const cx<T>*)in, (cx<T>*)out, gi, go, wl, z, batch, (cx<T>*)work, s, adjoint);
}

static int czt_entry(prop_dtype t, const void* in, void* out, const prop_grid* gi, const prop_grid* go, double wl,
                     double z, int32_t batch, void* stream, bool adjoint) {
  LP_RET(check_common(t, batch, wl));
  LP_RET(check_grid(gi));
  LP_RET(check_grid(go));
  if (!(z > 0) || !is_finite(z)) return PROP_EPARAM;
  LP_RET(check_czt_shapes(gi, go));
  if (batch == 0) return PROP_OK;
  if (!in || !out) return PROP_ENULL;
  const size_t bi = (size_t)gi->nx * gi->ny * batch * esize(t), bo = (size_t)go->nx * go->ny * batch * esize(t);
  if (!adjoint) LP_RET(check_alias({{in, bi}}, {{out, bo}}));
  else LP_RET(check_alias({{in, bo}}, {{out, bi}}));
  CtxLock lk;
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, czt_work_bytes(t, gi, go, batch), s));
  return t == PROP_C64 ? czt_run<float>(in, out, gi, go, wl, z, batch, s, adjoint, wb.p)
                       : czt_run<double>(in, out, gi, go, wl, z, batch, s, adjoint, wb.p);
}

// ------------------------------------------------- distance gradients --
// Blocks per batch item of an elementwise pass without a reduction.
static int item_blocks_host(int64_t npix, int batch) {
  const int64_t want = std::max<int64_t>(8, 4096 / std::max(batch, 1));
  return (int)std::max<int64_t>(1, std::min<int64_t>((npix + 255) / 256, want));
}

static int red_blocks(int64_t npix) { return (int)std::max<int64_t>(1, std::min<int64_t>((npix + 255) / 256, 256)); }

static size_t rs_grad_z_bytes(prop_dtype t, const prop_grid* g, int batch) {
  const size_t plane = (size_t)g->nx * g->ny * batch * esize(t);
  return rs_work_bytes(t, g, batch) + plane + (size_t)batch * red_blocks((int64_t)g->nx * g->ny) * sizeof(double) + 256;
}

// dL/dz = Re sum conj(g_out) dU/dz, dU/dz = RS with the kernel dH/dz.
template <typename T>
static int rs_grad_z_run(const void* u, const void* gout, double* dz, const prop_grid* g, double wl, double z, int batch,
                         hipStream_t s, void* work) {
  const int64_t npix = (int64_t)g->nx * g->ny;
  char* w = (char*)work;
  cx<T>* V = (cx<T>*)(w + rs_work_bytes(sizeof(T) == 4 ? PROP_C64 : PROP_C128, g, batch));
  double* partial = (double*)(((uintptr_t)(V + npix * batch) + 255) & ~(uintptr_t)255);
  LP_RET(rs_run<T>(u, V, g, wl, z, batch, s, false, work, 3));
  const int nblk = red_blocks(npix);
  LP_TRY(launch_redot<T>((const cx<T>*)gout, V, dz, partial, nblk, npix, batch, s));
  return PROP_OK;
}

static size_t rs_adjoint_grad_z_bytes(prop_dtype t, const prop_grid* g, int batch) {
  const int64_t plane = rs_plane_elems(g->ny, fft_len(2 * g->nx - 1));
  return std::max(2 * rs_work_bytes(t, g, batch) + (size_t)batch * red_blocks(plane) * sizeof(double) + 256,
                  rs_grad_z_bytes(t, g, batch));
}

// The adjoint of one RS step together with its distance gradient.  With
// V = RS of u with the kernel dH/dz, V = scale IFFT_rows(Cu) cropped to nx
// columns (Cu: the column pass of u's row transform with dH/dz, scale =
// dx dy / (Mx My)), and Parseval along each row gives
//   sum_{y, x < nx} conj(g[y, x]) V[y, x] = scale sum_{y, kx < Mx} conj(Rg[y, kx]) Cu[y, kx],
// Rg being the row transform of the zero-padded g, which is the adjoint's
// own first pass.  So dL/dz needs no inverse row pass: one dot product of
// the two workspaces (same tiled layout, every element written) before the
// adjoint's column pass overwrites Rg.  Where the workspace rows carry
// padding columns (Mx not a multiple of the tile width, nx = 1) the two
// computations run separately.
template <typename T>
static int rs_adjoint_grad_z_run(const void* gout, const void* u, void* gin, double* dz, const prop_grid* g,
                                 double wl, double z, int batch, hipStream_t s, void* work) {
  int dev;
  LP_RET(cur_device(&dev));
  const int nx = g->nx, ny = g->ny;
  if (fft_len(2 * nx - 1) % kTile != 0) {
    LP_RET(rs_grad_z_run<T>(u, gout, dz, g, wl, z, batch, s, work));
    return rs_run<T>(gout, gin, g, wl, z, batch, s, true, work);
  }
  const cx<T>* q[4];
  int Mx, My;
  LP_RET(get_rs_spectra<T>(dev, g, wl, z, 1 | 8, s, q, &Mx, &My));
  const cx<T> *twx, *twy;
  LP_RET(get_tw<T>(dev, Mx, &twx));
  LP_RET(get_tw<T>(dev, My, &twy));
  const int64_t plane = rs_plane_elems(ny, Mx);
  cx<T>* Wg = (cx<T>*)work;
  cx<T>* Wu = Wg + plane * batch;
  double* partial = (double*)(((uintptr_t)(Wu + plane * batch) + 255) & ~(uintptr_t)255);
  const double scale = g->dx * g->dy / ((double)Mx * (double)My);
  const double es = sizeof(cx<T>);
  const double qel = (double)Mx * (My / 2 + 1);
  LP_TRACE("rs_rows_fwd", es * batch * ny * (double)(nx + Mx), s,
           (launch_rs_rows<T, -1>(Mx, (const cx<T>*)gout, Wg, plane, ny, nx, T(1), batch, twx, s, nullptr, nullptr,
                                  0, nullptr)));
  LP_TRACE("rs_rows_fwd", es * batch * ny * (double)(nx + Mx), s,
           (launch_rs_rows<T, -1>(Mx, (const cx<T>*)u, Wu, plane, ny, nx, T(1), batch, twx, s, nullptr, nullptr, 0,
                                  nullptr)));
  // column passes: u with dH/dz (forward), then g with conj(H) (adjoint)
  for (int adj = 0; adj < 2; ++adj) {
    cx<T>* W = adj ? Wg : Wu;
    const cx<T>* spec = adj ? q[0] : q[3];
    int v = 0;
    const cx<T>* twc = twy;
    LP_RET(tuned_pass<T>(dev, TUNE_RS_COLS, My, Mx, ny, ny, batch, (size_t)plane * batch, 0, s,
                         [&](int var, const cx<T>* tw, cx<T>* a, cx<T>*) {
                           return launch_rs_cols<T>(My, a, plane, Mx, ny, spec, Mx, adj != 0, batch, tw, s, var);
                         },
                         &v, &twc));
    if (adj) {
      const int nblk = red_blocks(plane);
      LP_TRACE("rs_dz_dot", 2.0 * es * batch * (double)plane, s,
               launch_redot<T>(Wg, Wu, dz, partial, nblk, plane, batch, s, scale));
    }
    LP_TRACE("rs_cols", es * (2.0 * batch * ny * Mx + qel), s,
             launch_rs_cols<T>(My, W, plane, Mx, ny, spec, Mx, adj != 0, batch, twc, s, v));
  }
  LP_TRACE("rs_rows_inv", es * batch * ny * (double)(Mx + nx), s,
           (launch_rs_rows<T, 1>(Mx, Wg, (cx<T>*)gin, plane, ny, nx, (T)scale, batch, twx, s, nullptr, nullptr, 0,
                                 nullptr)));
  return PROP_OK;
}

static size_t czt_grad_z_bytes(prop_dtype t, const prop_grid* gi, const prop_grid* go, int batch, bool need_u) {
  const size_t ni = (size_t)gi->nx * gi->ny * batch, no = (size_t)go->nx * go->ny * batch;
  return (czt_tmp_elems(gi, go) * 3 * batch + 3 * ni + 3 * no + (need_u ? no : 0)) * esize(t) +
         (size_t)batch * red_blocks((int64_t)go->nx * go->ny) * sizeof(double) + 256;
}

// dL/dz = Re sum conj(g_out) dU/dz from U = C[u] and the three extra
// transforms C[|x|^2 u], C[x u], C[y u] (C = czt_propagate).
template <typename T>
static int czt_grad_z_run(const void* u, const void* uo, const void* gout, double* dz, const prop_grid* gi,
                          const prop_grid* go, double wl, double z, int batch, hipStream_t s, void* work) {
  const prop_dtype t = sizeof(T) == 4 ? PROP_C64 : PROP_C128;
  const size_t ni = (size_t)gi->nx * gi->ny * batch, no = (size_t)go->nx * go->ny * batch;
  cx<T>* P = (cx<T>*)work;  // 3 input planes
  cx<T>* Tt = P + 3 * ni;   // 3 output planes
  cx<T>* U = Tt + 3 * no;   // forward result when not given
  void* cw = U + (uo ? 0 : no);
  double* partial =
      (double*)(((uintptr_t)((char*)cw + czt_work_bytes(t, gi, go, 3 * batch)) + 255) & ~(uintptr_t)255);
  if (!uo) {
    LP_RET(czt_run<T>(u, U, gi, go, wl, z, batch, s, false, cw));
    uo = U;
  }
  LP_TRY(launch_czt_dz_prep<T>((const cx<T>*)u, P, gi->nx, gi->ny, gi->dx, gi->dy, gi->cx, gi->cy, batch, s));
  LP_RET(czt_run<T>(P, Tt, gi, go, wl, z, 3 * batch, s, false, cw));
  const int nblk = red_blocks((int64_t)go->nx * go->ny);
  LP_TRY(launch_czt_dz_reduce<T>((const cx<T>*)gout, (const cx<T>*)uo, Tt, go->nx, go->ny, go->dx, go->dy, go->cx,
                                 go->cy, 2.0 * kPi / wl, z, wl, dz, partial, nblk, batch, s));
  return PROP_OK;
}

// ----------------------------------------------------------- VCZT runs --
static size_t vczt_work_bytes(prop_dtype t, const prop_grid* gi, const prop_grid* go, bool lens, int batch) {
  const size_t ni = (size_t)gi->nx * gi->ny * batch, no = (size_t)go->nx * go->ny * batch;
  const size_t nt = czt_tmp_elems(gi, go) * batch;
  const size_t nm = (size_t)gi->ny * go->nx * batch;
  const size_t need = lens ? 3 * (ni + nm) : std::max(ni + no + nt, 2 * no + 3 * ni + nt);
  return need * esize(t);
}

template <typename T>
static int vczt_free_fwd(const void* ex, const void* ey, void* ox, void* oy, void* oz, const prop_grid* gi,
                         const prop_grid* go, double wl, double z, int batch, hipStream_t s, void* work) {
  int dev;
  LP_RET(cur_device(&dev));
  const size_t ni = (size_t)gi->nx * gi->ny * batch, no = (size_t)go->nx * go->ny * batch;
  cx<T>* prep = (cx<T>*)work;
  cx<T>* c2 = prep + ni;
  cx<T>* tmp = c2 + no;
  LP_TRY(launch_vczt_prep<T>((const cx<T>*)ex, (const cx<T>*)ey, prep, gi->nx, gi->ny, gi->dx, gi->dy, gi->cx, gi->cy,
                             batch, s));
  LP_RET(czt_core<T>(dev, (const cx<T>*)ex, (cx<T>*)ox, gi, go, wl, z, batch, tmp, s, false));
  LP_RET(czt_core<T>(dev, (const cx<T>*)ey, (cx<T>*)oy, gi, go, wl, z, batch, tmp, s, false));
  LP_RET(czt_core<T>(dev, prep, c2, gi, go, wl, z, batch, tmp, s, false));
  LP_TRY(launch_vczt_combine<T>((const cx<T>*)ox, (const cx<T>*)oy, c2, (cx<T>*)oz, go->nx, go->ny, go->dx, go->dy,
                                go->cx, go->cy, z, batch, s));
  return PROP_OK;
}

template <typename T>
static int vczt_free_adj(const void* gx, const void* gy, const void* gz, void* gex, void* gey, const prop_grid* gi,
                         const prop_grid* go, double wl, double z, int batch, hipStream_t s, void* work) {
  int dev;
  LP_RET(cur_device(&dev));
  const size_t ni = (size_t)gi->nx * gi->ny * batch, no = (size_t)go->nx * go->ny * batch;
  cx<T>* xg = (cx<T>*)work;
  cx<T>* yg = xg + no;
  cx<T>* a2 = yg + no;
  cx<T>* a3 = a2 + ni;
  cx<T>* a4 = a3 + ni;
  cx<T>* tmp = a4 + ni;
  LP_TRY(launch_vczt_adj_prep<T>((const cx<T>*)gz, xg, yg, go->nx, go->ny, go->dx, go->dy, go->cx, go->cy, z, batch,
                                 s));
  LP_RET(czt_core<T>(dev, (const cx<T>*)gx, (cx<T>*)gex, gi, go, wl, z, batch, tmp, s, true));
  LP_RET(czt_core<T>(dev, (const cx<T>*)gy, (cx<T>*)gey, gi, go, wl, z, batch, tmp, s, true));
  LP_RET(czt_core<T>(dev, xg, a2, gi, go, wl, z, batch, tmp, s, true));
  LP_RET(czt_core<T>(dev, yg, a3, gi, go, wl, z, batch, tmp, s, true));
  LP_RET(czt_core<T>(dev, (const cx<T>*)gz, a4, gi, go, wl, z, batch, tmp, s, true));
  LP_TRY(launch_vczt_adj_combine<T>((cx<T>*)gex, (cx<T>*)gey, a2, a3, a4, gi->nx, gi->ny, gi->dx, gi->dy, gi->cx,
                                    gi->cy, z, batch, s));
  return PROP_OK;
}

template <typename T>
static int rw_fwd(const void* ex, const void* ey, void* const* outs, const prop_grid* gi, const prop_grid* go,
                  double wl, const prop_lens* lens, int batch, hipStream_t s, void* work) {
  int dev;
  LP_RET(cur_device(&dev));
  const size_t ni = (size_t)gi->nx * gi->ny * batch;
  const size_t nm = (size_t)gi->ny * go->nx * batch;
  cx<T>* P = (cx<T>*)work;
  cx<T>* M = P + 3 * ni;
  const double es = sizeof(cx<T>);
  LP_TRACE("rw_pupil", es * 5.0 * ni, s,
           launch_pupil<T>((const cx<T>*)ex, (const cx<T>*)ey, P, P + ni, P + 2 * ni, gi->nx, gi->ny, gi->dx, gi->dy,
                           gi->cx, gi->cy, lens->f, lens->na, batch, (int64_t)gi->nx * gi->ny, false, s));
  ZoomSpec zx, zy;
  rw_specs(gi, go, wl, lens, false, &zx, &zy);
  const cx<T> *prex, *postx, *chatx, *prey, *posty, *chaty;
  LP_RET(get_zoom<T>(dev, zx, s, &prex, &postx, &chatx));
  LP_RET(get_zoom<T>(dev, zy, s, &prey, &posty, &chaty));
  const cx<T> *twx, *twy;
  LP_RET(get_tw<T>(dev, zx.L, &twx));
  LP_RET(get_tw<T>(dev, zy.L, &twy));
  const int nxi = gi->nx, nyi = gi->ny, nxo = go->nx, nyo = go->ny;
  LP_TRACE("rw_rows", es * 3.0 * batch * nyi * (double)(nxi + nxo), s,
           launch_bluestein<T>(zx.L, false, P, M, Lines{(int64_t)nyi * nxi, nxi}, Lines{(int64_t)nyi * nxo, nxo}, nyi,
                               nxi, nxo, prex, chatx, postx, 3 * batch, twx, s));
  const Lines li{(int64_t)nyi * nxo, nxo}, lo{(int64_t)nyo * nxo, nxo};
  int v = 0;
  LP_RET(tuned_pass<T>(dev, TUNE_CZT_COLS, zy.L, nxo, nyi, nyo, batch, (size_t)li.bstride * batch,
                       (size_t)lo.bstride * batch, s,
                       [&](int var, const cx<T>* tw, cx<T>* a, cx<T>* b) {
                         return launch_bluestein<T>(zy.L, true, a, b, li, lo, nxo, nyi, nyo, prey, chaty, posty,
                                                    batch, tw, s, var);
                       },
                       &v, &twy));
  for (int c = 0; c < 3; ++c)
    LP_TRACE("rw_cols", es * batch * nxo * (double)(nyi + nyo), s,
             launch_bluestein<T>(zy.L, true, M + c * nm, (cx<T>*)outs[c], li, lo, nxo, nyi, nyo, prey, chaty, posty,
                                 batch, twy, s, v));
  return PROP_OK;
}

template <typename T>
static int rw_adj(const void* const* gs, void* gex, void* gey, const prop_grid* gi, const prop_grid* go, double wl,
                  const prop_lens* lens, int batch, hipStream_t s, void* work) {
  int dev;
  LP_RET(cur_device(&dev));
  const size_t ni = (size_t)gi->nx * gi->ny * batch;
  const size_t nm = (size_t)gi->ny * go->nx * batch;
  cx<T>* P = (cx<T>*)work;
  cx<T>* M = P + 3 * ni;
  ZoomSpec zx, zy;
  rw_specs(gi, go, wl, lens, true, &zx, &zy);
  const cx<T> *prex, *postx, *chatx, *prey, *posty, *chaty;
  LP_RET(get_zoom<T>(dev, zx, s, &prex, &postx, &chatx));
  LP_RET(get_zoom<T>(dev, zy, s, &prey, &posty, &chaty));
  const cx<T> *twx, *twy;
  LP_RET(get_tw<T>(dev, zx.L, &twx));
  LP_RET(get_tw<T>(dev, zy.L, &twy));
  const int nxi = gi->nx, nyi = gi->ny, nxo = go->nx, nyo = go->ny;
  const double es = sizeof(cx<T>);
  const Lines li{(int64_t)nyo * nxo, nxo}, lo{(int64_t)nyi * nxo, nxo};
  int v = 0;
  LP_RET(tuned_pass<T>(dev, TUNE_CZT_COLS, zy.L, nxo, nyo, nyi, batch, (size_t)li.bstride * batch,
                       (size_t)lo.bstride * batch, s,
                       [&](int var, const cx<T>* tw, cx<T>* a, cx<T>* b) {
                         return launch_bluestein<T>(zy.L, true, a, b, li, lo, nxo, nyo, nyi, prey, chaty, posty,
                                                    batch, tw, s, var);
                       },
                       &v, &twy));
  for (int c = 0; c < 3; ++c)
    LP_TRACE("rw_cols", es * batch * nxo * (double)(nyi + nyo), s,
             launch_bluestein<T>(zy.L, true, (const cx<T>*)gs[c], M + c * nm, li, lo, nxo, nyo, nyi, prey, chaty,
                                 posty, batch, twy, s, v));
  LP_TRACE("rw_rows", es * 3.0 * batch * nyi * (double)(nxi + nxo), s,
           launch_bluestein<T>(zx.L, false, M, P, Lines{(int64_t)nyi * nxo, nxo}, Lines{(int64_t)nyi * nxi, nxi}, nyi,
                               nxo, nxi, prex, chatx, postx, 3 * batch, twx, s));
  LP_TRACE("rw_pupil", es * 5.0 * ni, s,
           launch_pupil<T>((const cx<T>*)gex, (const cx<T>*)gey, P, P + ni, P + 2 * ni, gi->nx, gi->ny, gi->dx, gi->dy,
                           gi->cx, gi->cy, lens->f, lens->na, batch, (int64_t)gi->nx * gi->ny, true, s));
  return PROP_OK;
}

// ---------------------------------------------------------- elementwise --
static double jones_cs(double theta, double* c, double* s) {
  *c = std::cos(theta);
  *s = std::sin(theta);
  return 0;
}

static void jones(double eta, double theta, double J[8]) {
  double c, s;
  jones_cs(theta, &c, &s);
  const double er = std::cos(eta), ei = std::sin(eta);
  // [[c^2 + e s^2, cs(1-e)], [cs(1-e), s^2 + e c^2]]
  J[0] = c * c + er * s * s; J[1] = ei * s * s;
  J[2] = c * s * (1 - er);   J[3] = -c * s * ei;
  J[4] = J[2];               J[5] = J[3];
  J[6] = s * s + er * c * c; J[7] = ei * c * c;
}

static void conj_transpose(const double J[8], double H[8]) {
  H[0] = J[0]; H[1] = -J[1];
  H[2] = J[4]; H[3] = -J[5];
  H[4] = J[2]; H[5] = -J[3];
  H[6] = J[6]; H[7] = -J[7];
}

static void jones_derivs(double eta, double theta, double d[16]) {
  double c, s;
  jones_cs(theta, &c, &s);
  const double er = std::cos(eta), ei = std::sin(eta);
  // dJ/deta = i e [[s^2, -cs], [-cs, c^2]],  i e = (-ei, er)
  const double ar = -ei, ai = er;
  const double m[4] = {s * s, -c * s, -c * s, c * c};
  for (int k = 0; k < 4; ++k) { d[2 * k] = ar * m[k]; d[2 * k + 1] = ai * m[k]; }
  // dJ/dtheta = (1 - e) [[-sin2t, cos2t], [cos2t, sin2t]]
  const double br = 1 - er, bi = -ei;
  const double s2 = std::sin(2 * theta), c2 = std::cos(2 * theta);
  const double n[4] = {-s2, c2, c2, s2};
  for (int k = 0; k < 4; ++k) { d[8 + 2 * k] = br * n[k]; d[8 + 2 * k + 1] = bi * n[k]; }
}


// ---------------------------------------------------------------- plans --
struct PlanSetup {
  prop_setup s;
  int ncomp_in = 1;
  bool modulated = false;  // vector ops: separate input-stage pass into umod
  bool fused = false;      // scalar ops: SLM stage fused into the first / last transform pass
  void* umod = nullptr;    // modulated input (ncomp_in planes) kept for the adjoint
  void* lens = nullptr;    // RS ops with lens_f: exp(-i q x^2) [nx] then exp(-i q y^2) [ny]
  int branch = 0;          // capture stream in graph mode
  double cost = 0.0;       // transform elements per execution (load balancing)
};

}  // namespace lp

struct prop_plan {
  prop_dtype t;
  int dev = 0;
  uint32_t flags = 0;
  std::vector<lp::PlanSetup> setups;
  int nbranch = 1;
  std::vector<lp::Buf> work;    // per branch
  std::vector<lp::Buf> gbuf;    // per branch: adjoint g_u planes
  std::vector<lp::Buf> mid;     // per branch: RS -> CZT intermediate of chained setups
  std::vector<hipStream_t> br;  // capture streams (graph mode)
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};  // forward, adjoint, forward + adjoint
  bool tuned[2] = {false, false};  // PROP_PLAN_AUTOTUNE: first execution tunes
  std::vector<int> order;          // graph mode: setups by decreasing cost
  lp::Pins pins;                   // cached tables this plan's kernels address
};

namespace lp {

// Drop a plan's pins (under the library lock); its tables become ordinary
// cache entries again.
static void unpin_all(Pins& p) {
  Ctx& C = ctx();
  for (auto& k : p.tw) C.tws.unpin(k);
  for (auto& k : p.spec) C.specs.unpin(k);
  for (auto& k : p.zoom) C.zooms.unpin(k);
  p.tw.clear();
  p.spec.clear();
  p.zoom.clear();
}

// After a device synchronisation every pinned table of the plan is complete.
static void mark_ready(Pins& p) {
  Ctx& C = ctx();
  for (auto& k : p.spec)
    if (auto* sl = C.specs.find(k, 0)) sl->v.ready.done = true;
  for (auto& k : p.zoom)
    if (auto* sl = C.zooms.find(k, 0)) sl->v.ready.done = true;
}

static int ncomp_in(int op) { return (op == PROP_OP_VRS || op == PROP_OP_VCZT) ? 2 : 1; }
static int ncomp_out(int op) { return (op == PROP_OP_VRS || op == PROP_OP_VCZT) ? 3 : 1; }
static bool vector_op(int op) { return op == PROP_OP_VRS || op == PROP_OP_VCZT; }
static bool czt_window(int op) { return op == PROP_OP_CZT || op == PROP_OP_VCZT || op == PROP_OP_RS_CZT; }

static int validate_setup(prop_dtype t, const prop_setup& s) {
  if (s.op < PROP_OP_RS || s.op > PROP_OP_RS_CZT) return PROP_ESHAPE;
  LP_RET(check_common(t, s.batch, s.wavelength));
  if (s.batch < 1) return PROP_ESHAPE;
  LP_RET(check_grid(&s.g_in));
  const bool lensmode = s.op == PROP_OP_VCZT && s.has_lens;
  if (czt_window(s.op)) {
    LP_RET(check_grid(&s.win));
    LP_RET(check_czt_shapes(&s.g_in, &s.win));
  }
  if (s.op == PROP_OP_RS || s.op == PROP_OP_VRS || s.op == PROP_OP_RS_CZT) LP_RET(check_rs_shape(&s.g_in));
  if (lensmode) LP_RET(check_lens(&s.lens));
  if (!lensmode && (!(s.z > 0) || !is_finite(s.z))) return PROP_EPARAM;
  if (s.op == PROP_OP_RS_CZT && (!(s.z2 > 0) || !is_finite(s.z2))) return PROP_EPARAM;
  if (!is_finite(s.lens_f) || s.lens_f < 0) return PROP_EPARAM;
  for (int c = 0; c < ncomp_in(s.op); ++c)
    if (!s.in[c]) return PROP_ENULL;
  for (int c = 0; c < ncomp_out(s.op); ++c)
    if (!s.out[c] || !s.gout[c]) return PROP_ENULL;
  return PROP_OK;
}

// Transform elements one execution of a setup touches (all passes, both
// directions alike): the weight of its load-balancing assignment.
static double rs_cost(const prop_grid& g) {
  const double Mx = fft_len(2 * g.nx - 1), My = fft_len(2 * g.ny - 1);
  return g.ny * Mx + Mx * My + g.ny * Mx;
}
static double czt_cost(const prop_grid& g, const prop_grid& w) {
  const double Lx = fft_len(g.nx + w.nx - 1), Ly = fft_len(g.ny + w.ny - 1);
  return g.ny * Lx + w.nx * Ly;
}
static double setup_cost(const prop_setup& s) {
  const double b = s.batch * (double)(ncomp_in(s.op) + ncomp_out(s.op));
  if (s.op == PROP_OP_RS || s.op == PROP_OP_VRS) return b * rs_cost(s.g_in);
  if (s.op == PROP_OP_RS_CZT) return b * (rs_cost(s.g_in) + czt_cost(s.g_in, s.win));
  return b * czt_cost(s.g_in, s.win);
}

static size_t setup_work_bytes(prop_dtype t, const prop_setup& s) {
  switch (s.op) {
    case PROP_OP_RS: return rs_work_bytes(t, &s.g_in, s.batch);
    case PROP_OP_VRS: return vrs_work_bytes(t, &s.g_in, s.batch);
    case PROP_OP_CZT: return czt_work_bytes(t, &s.g_in, &s.win, s.batch);
    case PROP_OP_RS_CZT:
      return std::max(rs_work_bytes(t, &s.g_in, s.batch), czt_work_bytes(t, &s.g_in, &s.win, s.batch));
    default: return vczt_work_bytes(t, &s.g_in, &s.win, s.has_lens != 0, s.batch);
  }
}

// Quadratic input phase dq (x^2 + y^2) of a thin lens of focal length f in
// front of a CZT (0: none); it folds exactly into the CZT input chirp.
static double lens_dq(double wl, double f) { return f > 0 ? -(2.0 * kPi / wl) / (2.0 * f) : 0.0; }

// The CZT of a setup: (grid, window, distance, lens folded in front).
static double czt_distance(const prop_setup& s) { return s.op == PROP_OP_RS_CZT ? s.z2 : s.z; }

// Fill the caches (spectra, chirps, twiddles) a setup needs, on stream s.
template <typename T>
static int warm_setup(int dev, const prop_setup& s, hipStream_t st) {
  const cx<T>* q[4];
  const cx<T>* tw;
  int Mx, My;
  const cx<T> *a, *b, *c;
  ZoomSpec zx, zy;
  if (s.op == PROP_OP_RS || s.op == PROP_OP_VRS || s.op == PROP_OP_RS_CZT) {
    LP_RET(get_rs_spectra<T>(dev, &s.g_in, s.wavelength, s.z, s.op == PROP_OP_VRS ? 7 : 1, st, q, &Mx, &My));
    LP_RET(get_tw<T>(dev, Mx, &tw));
    LP_RET(get_tw<T>(dev, My, &tw));
  }
  if (!czt_window(s.op)) return PROP_OK;
  for (int adj = 0; adj < 2; ++adj) {
    if (s.op == PROP_OP_VCZT && s.has_lens) rw_specs(&s.g_in, &s.win, s.wavelength, &s.lens, adj, &zx, &zy);
    else if (s.op == PROP_OP_VCZT) czt_specs(&s.g_in, &s.win, s.wavelength, s.z, adj, &zx, &zy);
    else czt_specs(&s.g_in, &s.win, s.wavelength, czt_distance(s), adj, &zx, &zy, lens_dq(s.wavelength, s.lens_f));
    LP_RET(get_zoom<T>(dev, zx, st, &a, &b, &c));
    LP_RET(get_zoom<T>(dev, zy, st, &a, &b, &c));
    LP_RET(get_tw<T>(dev, zx.L, &tw));
    LP_RET(get_tw<T>(dev, zy.L, &tw));
  }
  return PROP_OK;
}

// The fused SLM stage of a scalar setup: its phase, and for RS its input
// lens as separable factors (a CZT folds its lens into the chirp instead;
// a chained setup's lens sits between RS and CZT and folds likewise).
template <typename T>
static Slm<T> setup_slm(const PlanSetup& ps, bool adjoint) {
  Slm<T> st;
  st.phase = (const T*)ps.s.phase;
  st.pbs = (int64_t)ps.s.g_in.nx * ps.s.g_in.ny;
  st.nx = ps.s.g_in.nx;
  if (ps.lens) {
    st.lx = (const cx<T>*)ps.lens;
    st.ly = (const cx<T>*)ps.lens + ps.s.g_in.nx;
  }
  st.adjoint = adjoint;
  return st;
}

template <typename T>
static int run_setup(prop_plan* p, PlanSetup& ps, bool adjoint, hipStream_t st, int branch) {
  const prop_setup& s = ps.s;
  void* work = p->work[branch].p;
  const int64_t npix = (int64_t)s.g_in.nx * s.g_in.ny;
  const double q = s.lens_f > 0 ? (2.0 * kPi / s.wavelength) / (2.0 * s.lens_f) : 0.0;
  const int nin = ps.ncomp_in, nout = ncomp_out(s.op);
  const size_t plane = (size_t)npix * s.batch;
  const T* phase = (const T*)s.phase;
  int dev;
  LP_RET(cur_device(&dev));
  if (ps.fused || !vector_op(s.op)) {
    // scalar setups: SLM stage fused into the transforms, lens folded into
    // the CZT chirp (or separable factors in front of RS)
    const Slm<T> sf = setup_slm<T>(ps, false), sa = setup_slm<T>(ps, true);
    const Slm<T>* fwd = ps.fused ? &sf : nullptr;
    const Slm<T>* adj = ps.fused ? &sa : nullptr;
    const double dq = s.op == PROP_OP_RS ? 0.0 : lens_dq(s.wavelength, s.lens_f);
    cx<T>* mid = (cx<T>*)p->mid[branch].p;
    const cx<T>* v_in = (const cx<T>*)s.in[0];
    T* gph = (T*)s.grad_phase;
    if (!adjoint) {
      switch (s.op) {
        case PROP_OP_RS:
          return rs_run<T>(v_in, s.out[0], &s.g_in, s.wavelength, s.z, s.batch, st, false, work, 0, nullptr, nullptr,
                           0, fwd);
        case PROP_OP_CZT:
          return czt_core<T>(dev, v_in, (cx<T>*)s.out[0], &s.g_in, &s.win, s.wavelength, s.z, s.batch, (cx<T>*)work,
                             st, false, nullptr, nullptr, 0, fwd, dq);
        default:  // PROP_OP_RS_CZT
          LP_RET(rs_run<T>(v_in, mid, &s.g_in, s.wavelength, s.z, s.batch, st, false, work, 0, nullptr, nullptr, 0,
                           fwd));
          return czt_core<T>(dev, mid, (cx<T>*)s.out[0], &s.g_in, &s.win, s.wavelength, s.z2, s.batch,
                             (cx<T>*)work, st, false, nullptr, nullptr, 0, nullptr, dq);
      }
    }
    // adjoint: the last pass writes g_V = g_U conj(stage) into gin and the
    // phase gradient Im(g_U conj U) (V = the forward input, read again)
    void* gin = s.gin[0];
    if (!gin && !gph) return PROP_OK;
    const cx<T>* pgu = gph ? v_in : nullptr;
    switch (s.op) {
      case PROP_OP_RS:
        return rs_run<T>(s.gout[0], gin, &s.g_in, s.wavelength, s.z, s.batch, st, true, work, 0, pgu, gph, 0, adj);
      case PROP_OP_CZT:
        return czt_core<T>(dev, (const cx<T>*)s.gout[0], (cx<T>*)gin, &s.g_in, &s.win, s.wavelength, s.z, s.batch,
                           (cx<T>*)work, st, true, pgu, gph, 0, adj, dq);
      default:
        LP_RET(czt_core<T>(dev, (const cx<T>*)s.gout[0], mid, &s.g_in, &s.win, s.wavelength, s.z2, s.batch,
                           (cx<T>*)work, st, true, nullptr, nullptr, 0, nullptr, dq));
        return rs_run<T>(mid, gin, &s.g_in, s.wavelength, s.z, s.batch, st, true, work, 0, pgu, gph, 0, adj);
    }
  }
  // vector setups: a separate input stage pass keeps the modulated input
  if (!adjoint) {
    const void* u[2] = {s.in[0], s.in[1]};
    if (ps.modulated) {
      for (int c = 0; c < nin; ++c) {
        cx<T>* dst = (cx<T>*)ps.umod + c * plane;
        LP_TRACE("plan_input", (double)plane * (2 * sizeof(cx<T>) + (phase ? sizeof(T) : 0)), st,
                 launch_phase_stage<T>((const cx<T>*)s.in[c], phase, dst, s.g_in.nx, s.g_in.ny, s.g_in.dx, s.g_in.dy,
                                       s.g_in.cx, s.g_in.cy, q, s.batch, npix, st));
        u[c] = dst;
      }
    }
    if (s.op == PROP_OP_VRS) return vrs_run<T>(u, 2, s.out, 3, &s.g_in, s.wavelength, s.z, s.batch, st, false, work);
    if (s.has_lens) return rw_fwd<T>(u[0], u[1], s.out, &s.g_in, &s.win, s.wavelength, &s.lens, s.batch, st, work);
    return vczt_free_fwd<T>(u[0], u[1], s.out[0], s.out[1], s.out[2], &s.g_in, &s.win, s.wavelength, s.z, s.batch, st,
                            work);
  }
  // adjoint: g_u lands in gin directly when there is no input stage
  void* gu[2] = {s.gin[0], s.gin[1]};
  if (ps.modulated) {
    for (int c = 0; c < nin; ++c) gu[c] = (char*)p->gbuf[branch].p + c * plane * sizeof(cx<T>);
  }
  if (s.op == PROP_OP_VRS) {
    LP_RET(vrs_run<T>(s.gout, 3, gu, 2, &s.g_in, s.wavelength, s.z, s.batch, st, true, work));
  } else if (s.has_lens) {
    LP_RET(rw_adj<T>(s.gout, gu[0], gu[1], &s.g_in, &s.win, s.wavelength, &s.lens, s.batch, st, work));
  } else {
    LP_RET(vczt_free_adj<T>(s.gout[0], s.gout[1], s.gout[2], gu[0], gu[1], &s.g_in, &s.win, s.wavelength, s.z, s.batch,
                            st, work));
  }
  if (ps.modulated) {
    for (int c = 0; c < nin; ++c) {
      const cx<T>* u = (const cx<T>*)ps.umod + c * plane;
      LP_TRACE("plan_input_adj", (double)plane * 3 * sizeof(cx<T>), st,
               launch_phase_stage_adj<T>((const cx<T>*)gu[c], u, phase, (cx<T>*)s.gin[c], (T*)s.grad_phase, c > 0 ? 1 : 0,
                                         s.g_in.nx, s.g_in.ny, s.g_in.dx, s.g_in.dy, s.g_in.cx, s.g_in.cy, q, s.batch,
                                         npix, st));
    }
  }
  return PROP_OK;
}

// Enqueue all setups: sequentially on `st`, or over the plan's branch
// streams (fork/join through events) when `branched`.
static int plan_enqueue(prop_plan* p, bool adjoint, hipStream_t st, bool branched) {
  if (branched) {
    LP_TRY(hipEventRecord(p->fork, st));
    for (int b = 0; b < p->nbranch; ++b) LP_TRY(hipStreamWaitEvent(p->br[b], p->fork, 0));
  }
  for (size_t k = 0; k < p->setups.size(); ++k) {
    PlanSetup& ps = p->setups[branched ? p->order[k] : k];
    const int b = branched ? ps.branch : 0;
    const hipStream_t s = branched ? p->br[b] : st;
    LP_RET(p->t == PROP_C64 ? run_setup<float>(p, ps, adjoint, s, b) : run_setup<double>(p, ps, adjoint, s, b));
  }
  if (branched) {
    for (int b = 0; b < p->nbranch; ++b) {
      LP_TRY(hipEventRecord(p->join[b], p->br[b]));
      LP_TRY(hipStreamWaitEvent(st, p->join[b], 0));
    }
  }
  return PROP_OK;
}

// mode 0: forward, 1: adjoint, 2: forward then adjoint (one graph with
// PROP_PLAN_GRAPH; the adjoint's branches start once every forward branch
// has joined, exactly as two calls in a row)
static int plan_run(prop_plan* p, int mode, hipStream_t st) {
  if ((p->flags & PROP_PLAN_AUTOTUNE) && !capturing(st)) {
    // first execution of a direction runs eagerly with the autotuner on; a
    // graph is captured afterwards with the chosen variants
    const bool fwd_untuned = mode != 1 && !p->tuned[0], adj_untuned = mode != 0 && !p->tuned[1];
    if (fwd_untuned || adj_untuned) {
      for (int dir = 0; dir < 2; ++dir) {
        if ((dir == 0 && mode == 1) || (dir == 1 && mode == 0)) continue;
        t_tune_request = !p->tuned[dir];
        const int r = plan_enqueue(p, dir == 1, st, false);
        t_tune_request = false;
        LP_RET(r);
        p->tuned[dir] = true;
      }
      return PROP_OK;
    }
  }
  if (!(p->flags & PROP_PLAN_GRAPH)) {
    if (mode != 1) LP_RET(plan_enqueue(p, false, st, false));
    if (mode != 0) LP_RET(plan_enqueue(p, true, st, false));
    return PROP_OK;
  }
  hipGraphExec_t& ex = p->gexec[mode];
  if (!ex) {
    // capture on the first branch stream, forking to the others
    hipStream_t origin = p->br[0];
    hipGraph_t graph = nullptr;
    LP_TRY(hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal));
    int r = PROP_OK;
    if (mode != 1) r = plan_enqueue(p, false, origin, p->nbranch > 1);
    if (r >= 0 && mode != 0) r = plan_enqueue(p, true, origin, p->nbranch > 1);
    hipError_t e = hipStreamEndCapture(origin, &graph);
    if (r < 0) {
      if (graph) (void)hipGraphDestroy(graph);
      return r;
    }
    if (e != hipSuccess) return dev_err(e);
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      ex = nullptr;
      return dev_err(e);
    }
  }
  LP_TRY(hipGraphLaunch(ex, st));
  return PROP_OK;
}

// ------------------------------------------------------- detector loss --
static const int kSpotBlocks = 256;  // FP64 partial sums per batch item (fixed reduction order)

static int spot_loss_check(prop_dtype t, const void* ex, const void* ey, const void* ez, const prop_grid* win,
                           double wavelength, double w_fz, double* result, void* gx, void* gy, void* gz,
                           int32_t batch) {
  LP_RET(check_common(t, batch, wavelength));
  LP_RET(check_grid(win));
  if (!is_finite(w_fz)) return PROP_EPARAM;
  if (batch == 0) return PROP_OK;
  if (!ex || !ey || !result) return PROP_ENULL;
  if ((gx == nullptr) != (gy == nullptr)) return PROP_ENULL;
  const size_t b = (size_t)win->nx * win->ny * batch * esize(t);
  if (gx) {
    if (ez && gz) LP_RET(check_alias({{ex, b}, {ey, b}, {ez, b}}, {{gx, b}, {gy, b}, {gz, b}, {result, 64 * (size_t)batch}}));
    else LP_RET(check_alias({{ex, b}, {ey, b}}, {{gx, b}, {gy, b}, {result, 64 * (size_t)batch}}));
  }
  return PROP_OK;
}

static int spot_loss_launch(prop_dtype t, const void* ex, const void* ey, const void* ez, const prop_grid* win,
                            double wavelength, double w_fz, double* result, void* gx, void* gy, void* gz,
                            int32_t batch, double* partial, hipStream_t s) {
  hipError_t e = t == PROP_C64
                     ? launch_spot_loss<float>((const cx<float>*)ex, (const cx<float>*)ey, (const cx<float>*)ez,
                                               win->nx, win->ny, win->dx, win->dy, win->cx, win->cy, wavelength, w_fz,
                                               result, partial, kSpotBlocks, (cx<float>*)gx, (cx<float>*)gy,
                                               (cx<float>*)gz, batch, s)
                     : launch_spot_loss<double>((const cx<double>*)ex, (const cx<double>*)ey, (const cx<double>*)ez,
                                                win->nx, win->ny, win->dx, win->dy, win->cx, win->cy, wavelength,
                                                w_fz, result, partial, kSpotBlocks, (cx<double>*)gx, (cx<double>*)gy,
                                                (cx<double>*)gz, batch, s);
  return e == hipSuccess ? PROP_OK : dev_err(e);
}

// ---------------------------------------------- allocation-free scratch --
// Device memory of the allocation-free entry points: a file-scope array,
// one copy per GPU, held until the process ends.  In host code its name is
// only a stand-in; the device address comes from hipGetSymbolAddress, once
// per device with that device current, and only that address is used.
// Calls that overlap on one GPU share the array and race.
static const int kNoAllocMaxBatch = 256;
static __device__ __align__(256) double scratch[(size_t)kNoAllocMaxBatch * kSpotBlocks * 5];

static int noalloc_scratch(double** out) {
  static std::mutex mu;
  static void* addr[64] = {};
  int dev;
  LP_RET(cur_device(&dev));
  if (dev < 0 || dev >= 64) return PROP_EDEVICE;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    LP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return PROP_EDEVICE;
    addr[dev] = p;
  }
  *out = (double*)addr[dev];
  return PROP_OK;
}

}  // namespace lp

using namespace lp;

// =================================================================== ABI ==
extern "C" {

int rs_propagate(prop_dtype t, const void* u_in, void* u_out, const prop_grid* g, double wavelength, double z,
                 int32_t batch, void* stream) {
  return rs_entry(t, u_in, u_out, g, wavelength, z, batch, stream, false);
}

int rs_adjoint(prop_dtype t, const void* g_out, void* g_in, const prop_grid* g, double wavelength, double z,
               int32_t batch, void* stream) {
  return rs_entry(t, g_out, g_in, g, wavelength, z, batch, stream, true);
}

int rs_adjoint_phase_grad(prop_dtype t, const void* g_out, const void* u, void* g_u, void* grad, int32_t accumulate,
                          const prop_grid* g, double wavelength, double z, int32_t batch, void* stream) {
  LP_RET(check_common(t, batch, wavelength));
  LP_RET(check_grid(g));
  if (!(z > 0) || !is_finite(z)) return PROP_EPARAM;
  if (fft_len(2 * g->nx - 1) < 0 || fft_len(2 * g->ny - 1) < 0) return PROP_ESHAPE;
  const int warn = sampling(g, wavelength, z);
  if (batch == 0) return warn;
  if (!g_out || !u || !grad) return PROP_ENULL;
  const size_t bytes = (size_t)g->nx * g->ny * batch * esize(t);
  LP_RET(check_alias({{g_out, bytes}, {u, bytes}}, {{g_u, g_u ? bytes : 0}, {grad, bytes / 2}}));
  CtxLock lk;
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, rs_work_bytes(t, g, batch), s));
  const int r = t == PROP_C64 ? rs_run<float>(g_out, g_u, g, wavelength, z, batch, s, true, wb.p, 0,
                                              (const cx<float>*)u, (float*)grad, accumulate ? 1 : 0)
                              : rs_run<double>(g_out, g_u, g, wavelength, z, batch, s, true, wb.p, 0,
                                               (const cx<double>*)u, (double*)grad, accumulate ? 1 : 0);
  return r < 0 ? r : warn;
}

int czt_adjoint_phase_grad(prop_dtype t, const void* g_out, const void* u, void* g_u, void* grad, int32_t accumulate,
                           const prop_grid* g_in, const prop_grid* win, double wavelength, double z, int32_t batch,
                           void* stream) {
  LP_RET(check_common(t, batch, wavelength));
  LP_RET(check_grid(g_in));
  LP_RET(check_grid(win));
  if (!(z > 0) || !is_finite(z)) return PROP_EPARAM;
  LP_RET(check_czt_shapes(g_in, win));
  if (batch == 0) return PROP_OK;
  if (!g_out || !u || !grad) return PROP_ENULL;
  const size_t bi = (size_t)g_in->nx * g_in->ny * batch * esize(t), bo = (size_t)win->nx * win->ny * batch * esize(t);
  LP_RET(check_alias({{g_out, bo}, {u, bi}}, {{g_u, g_u ? bi : 0}, {grad, bi / 2}}));
  CtxLock lk;
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, czt_work_bytes(t, g_in, win, batch), s));
  return t == PROP_C64 ? czt_core<float>(dev, (const cx<float>*)g_out, (cx<float>*)g_u, g_in, win, wavelength, z, batch,
                                         (cx<float>*)wb.p, s, true, (const cx<float>*)u, (float*)grad,
                                         accumulate ? 1 : 0)
                       : czt_core<double>(dev, (const cx<double>*)g_out, (cx<double>*)g_u, g_in, win, wavelength, z,
                                          batch, (cx<double>*)wb.p, s, true, (const cx<double>*)u, (double*)grad,
                                          accumulate ? 1 : 0);
}

int rs_grad_z(prop_dtype t, const void* u_in, const void* g_out, double* dz, const prop_grid* g, double wavelength,
              double z, int32_t batch, void* stream) {
  LP_RET(check_common(t, batch, wavelength));
  LP_RET(check_grid(g));
  if (!(z > 0) || !is_finite(z)) return PROP_EPARAM;
  if (fft_len(2 * g->nx - 1) < 0 || fft_len(2 * g->ny - 1) < 0) return PROP_ESHAPE;
  const int warn = sampling(g, wavelength, z);
  if (batch == 0) return warn;
  if (!u_in || !g_out || !dz) return PROP_ENULL;
  CtxLock lk;
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, rs_grad_z_bytes(t, g, batch), s));
  const int r = t == PROP_C64 ? rs_grad_z_run<float>(u_in, g_out, dz, g, wavelength, z, batch, s, wb.p)
                              : rs_grad_z_run<double>(u_in, g_out, dz, g, wavelength, z, batch, s, wb.p);
  return r < 0 ? r : warn;
}

int rs_adjoint_grad_z(prop_dtype t, const void* g_out, const void* u_in, void* g_in, double* dz, const prop_grid* g,
                      double wavelength, double z, int32_t batch, void* stream) {
  LP_RET(check_common(t, batch, wavelength));
  LP_RET(check_grid(g));
  if (!(z > 0) || !is_finite(z)) return PROP_EPARAM;
  if (fft_len(2 * g->nx - 1) < 0 || fft_len(2 * g->ny - 1) < 0) return PROP_ESHAPE;
  const int warn = sampling(g, wavelength, z);
  if (batch == 0) return warn;
  if (!g_out || !u_in || !g_in || !dz) return PROP_ENULL;
  const size_t bytes = (size_t)g->nx * g->ny * batch * esize(t);
  LP_RET(check_alias({{g_out, bytes}, {u_in, bytes}}, {{g_in, bytes}, {dz, (size_t)batch * sizeof(double)}}));
  CtxLock lk;
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, rs_adjoint_grad_z_bytes(t, g, batch), s));
  const int r = t == PROP_C64
                    ? rs_adjoint_grad_z_run<float>(g_out, u_in, g_in, dz, g, wavelength, z, batch, s, wb.p)
                    : rs_adjoint_grad_z_run<double>(g_out, u_in, g_in, dz, g, wavelength, z, batch, s, wb.p);
  return r < 0 ? r : warn;
}

int czt_grad_z(prop_dtype t, const void* u_in, const void* u_out, const void* g_out, double* dz,
               const prop_grid* g_in, const prop_grid* win, double wavelength, double z, int32_t batch,
               void* stream) {
  LP_RET(check_common(t, batch, wavelength));
  LP_RET(check_grid(g_in));
  LP_RET(check_grid(win));
  if (!(z > 0) || !is_finite(z)) return PROP_EPARAM;
  LP_RET(check_czt_shapes(g_in, win));
  if (batch == 0) return PROP_OK;
  if (!u_in || !g_out || !dz) return PROP_ENULL;
  CtxLock lk;
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, czt_grad_z_bytes(t, g_in, win, batch, u_out == nullptr), s));
  return t == PROP_C64 ? czt_grad_z_run<float>(u_in, u_out, g_out, dz, g_in, win, wavelength, z, batch, s, wb.p)
                       : czt_grad_z_run<double>(u_in, u_out, g_out, dz, g_in, win, wavelength, z, batch, s, wb.p);
}

int czt_propagate(prop_dtype t, const void* u_in, void* u_out, const prop_grid* g_in, const prop_grid* win,
                  double wavelength, double z, int32_t batch, void* stream) {
  return czt_entry(t, u_in, u_out, g_in, win, wavelength, z, batch, stream, false);
}

int czt_adjoint(prop_dtype t, const void* g_out, void* g_in, const prop_grid* g_in_grid, const prop_grid* win,
                double wavelength, double z, int32_t batch, void* stream) {
  return czt_entry(t, g_out, g_in, g_in_grid, win, wavelength, z, batch, stream, true);
}

int vrs_propagate(prop_dtype t, const void* ex, const void* ey, void* ox, void* oy, void* oz, const prop_grid* g,
                  double wavelength, double z, int32_t batch, void* stream) {
  LP_RET(check_common(t, batch, wavelength));
  LP_RET(check_grid(g));
  if (!(z > 0) || !is_finite(z)) return PROP_EPARAM;
  if (fft_len(2 * g->nx - 1) < 0 || fft_len(2 * g->ny - 1) < 0) return PROP_ESHAPE;
  const int warn = sampling(g, wavelength, z);
  if (batch == 0) return warn;
  if (!ex || !ey || !ox || !oy || !oz) return PROP_ENULL;
  const size_t b = (size_t)g->nx * g->ny * batch * esize(t);
  LP_RET(check_alias({{ex, b}, {ey, b}}, {{ox, b}, {oy, b}, {oz, b}}));
  CtxLock lk;
  const void* ins[2] = {ex, ey};
  void* outs[3] = {ox, oy, oz};
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, vrs_work_bytes(t, g, batch), s));
  int r = t == PROP_C64 ? vrs_run<float>(ins, 2, outs, 3, g, wavelength, z, batch, s, false, wb.p)
                        : vrs_run<double>(ins, 2, outs, 3, g, wavelength, z, batch, s, false, wb.p);
  return r < 0 ? r : warn;
}

int vrs_adjoint(prop_dtype t, const void* gx, const void* gy, const void* gz, void* gex, void* gey, const prop_grid* g,
                double wavelength, double z, int32_t batch, void* stream) {
  LP_RET(check_common(t, batch, wavelength));
  LP_RET(check_grid(g));
  if (!(z > 0) || !is_finite(z)) return PROP_EPARAM;
  if (fft_len(2 * g->nx - 1) < 0 || fft_len(2 * g->ny - 1) < 0) return PROP_ESHAPE;
  const int warn = sampling(g, wavelength, z);
  if (batch == 0) return warn;
  if (!gx || !gy || !gz || !gex || !gey) return PROP_ENULL;
  const size_t b = (size_t)g->nx * g->ny * batch * esize(t);
  LP_RET(check_alias({{gx, b}, {gy, b}, {gz, b}}, {{gex, b}, {gey, b}}));
  CtxLock lk;
  const void* ins[3] = {gx, gy, gz};
  void* outs[2] = {gex, gey};
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, vrs_work_bytes(t, g, batch), s));
  int r = t == PROP_C64 ? vrs_run<float>(ins, 3, outs, 2, g, wavelength, z, batch, s, true, wb.p)
                        : vrs_run<double>(ins, 3, outs, 2, g, wavelength, z, batch, s, true, wb.p);
  return r < 0 ? r : warn;
}

int vczt_propagate(prop_dtype t, const void* ex, const void* ey, void* ox, void* oy, void* oz, const prop_grid* g_in,
                   const prop_grid* win, double wavelength, double z, const prop_lens* lens, int32_t batch,
                   void* stream) {
  LP_RET(check_common(t, batch, wavelength));
  LP_RET(check_grid(g_in));
  LP_RET(check_grid(win));
  LP_RET(check_lens(lens));
  if (!lens && (!(z > 0) || !is_finite(z))) return PROP_EPARAM;
  if (lens && !is_finite(z)) return PROP_EPARAM;
  LP_RET(check_czt_shapes(g_in, win));
  if (batch == 0) return PROP_OK;
  if (!ex || !ey || !ox || !oy || !oz) return PROP_ENULL;
  const size_t bi = (size_t)g_in->nx * g_in->ny * batch * esize(t), bo = (size_t)win->nx * win->ny * batch * esize(t);
  LP_RET(check_alias({{ex, bi}, {ey, bi}}, {{ox, bo}, {oy, bo}, {oz, bo}}));
  CtxLock lk;
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, vczt_work_bytes(t, g_in, win, lens != nullptr, batch), s));
  void* outs[3] = {ox, oy, oz};
  if (lens)
    return t == PROP_C64 ? rw_fwd<float>(ex, ey, outs, g_in, win, wavelength, lens, batch, s, wb.p)
                         : rw_fwd<double>(ex, ey, outs, g_in, win, wavelength, lens, batch, s, wb.p);
  return t == PROP_C64 ? vczt_free_fwd<float>(ex, ey, ox, oy, oz, g_in, win, wavelength, z, batch, s, wb.p)
                       : vczt_free_fwd<double>(ex, ey, ox, oy, oz, g_in, win, wavelength, z, batch, s, wb.p);
}

int vczt_adjoint(prop_dtype t, const void* gx, const void* gy, const void* gz, void* gex, void* gey,
                 const prop_grid* g_in, const prop_grid* win, double wavelength, double z, const prop_lens* lens,
                 int32_t batch, void* stream) {
  LP_RET(check_common(t, batch, wavelength));
  LP_RET(check_grid(g_in));
  LP_RET(check_grid(win));
  LP_RET(check_lens(lens));
  if (!lens && (!(z > 0) || !is_finite(z))) return PROP_EPARAM;
  if (lens && !is_finite(z)) return PROP_EPARAM;
  LP_RET(check_czt_shapes(g_in, win));
  if (batch == 0) return PROP_OK;
  if (!gx || !gy || !gz || !gex || !gey) return PROP_ENULL;
  const size_t bi = (size_t)g_in->nx * g_in->ny * batch * esize(t), bo = (size_t)win->nx * win->ny * batch * esize(t);
  LP_RET(check_alias({{gx, bo}, {gy, bo}, {gz, bo}}, {{gex, bi}, {gey, bi}}));
  CtxLock lk;
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, vczt_work_bytes(t, g_in, win, lens != nullptr, batch), s));
  if (lens) {
    const void* gs[3] = {gx, gy, gz};
    return t == PROP_C64 ? rw_adj<float>(gs, gex, gey, g_in, win, wavelength, lens, batch, s, wb.p)
                         : rw_adj<double>(gs, gex, gey, g_in, win, wavelength, lens, batch, s, wb.p);
  }
  return t == PROP_C64 ? vczt_free_adj<float>(gx, gy, gz, gex, gey, g_in, win, wavelength, z, batch, s, wb.p)
                       : vczt_free_adj<double>(gx, gy, gz, gex, gey, g_in, win, wavelength, z, batch, s, wb.p);
}

int prop_source_gaussian(prop_dtype t, void* out, const prop_grid* g, double w0, double amplitude, double lens_f,
                         double wavelength, int32_t batch, void* stream) {
  LP_RET(check_common(t, batch, wavelength));
  LP_RET(check_grid(g));
  if (!(w0 > 0) || !is_finite(w0) || !is_finite(amplitude) || !is_finite(lens_f) || lens_f < 0) return PROP_EPARAM;
  if (batch == 0) return PROP_OK;
  if (!out) return PROP_ENULL;
  const double k = 2.0 * kPi / wavelength;
  const hipStream_t s = (hipStream_t)stream;
  hipError_t e = t == PROP_C64 ? launch_source_gaussian<float>((cx<float>*)out, g->nx, g->ny, g->dx, g->dy, g->cx,
                                                               g->cy, w0, amplitude, lens_f, k, batch, s)
                               : launch_source_gaussian<double>((cx<double>*)out, g->nx, g->ny, g->dx, g->dy, g->cx,
                                                                g->cy, w0, amplitude, lens_f, k, batch, s);
  return e == hipSuccess ? PROP_OK : dev_err(e);
}

int prop_source_radial(prop_dtype t, void* ex, void* ey, const prop_grid* g, double w0, int32_t batch, void* stream) {
  LP_RET(check_common(t, batch, 1.0));
  LP_RET(check_grid(g));
  if (!(w0 > 0) || !is_finite(w0)) return PROP_EPARAM;
  if (batch == 0) return PROP_OK;
  if (!ex || !ey) return PROP_ENULL;
  const size_t b = (size_t)g->nx * g->ny * batch * esize(t);
  LP_RET(check_alias({}, {{ex, b}, {ey, b}}));
  const hipStream_t s = (hipStream_t)stream;
  hipError_t e = t == PROP_C64 ? launch_source_radial<float>((cx<float>*)ex, (cx<float>*)ey, g->nx, g->ny, g->dx,
                                                             g->dy, g->cx, g->cy, w0, batch, s)
                               : launch_source_radial<double>((cx<double>*)ex, (cx<double>*)ey, g->nx, g->ny, g->dx,
                                                              g->dy, g->cx, g->cy, w0, batch, s);
  return e == hipSuccess ? PROP_OK : dev_err(e);
}

static int modulate_run(prop_dtype t, const void* u_in, const void* phase, void* u_out, int64_t npix, int32_t batch,
                        int32_t phase_batch, void* stream, bool conj) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (npix < 0 || batch < 0) return PROP_ESHAPE;
  if (phase_batch != 1 && phase_batch != batch) return PROP_ESHAPE;
  if (npix == 0 || batch == 0) return PROP_OK;
  if (!u_in || !phase || !u_out) return PROP_ENULL;
  // in place (u_out == u_in) is allowed: elementwise
  const size_t b = (size_t)npix * batch * esize(t);
  if (u_out != u_in) LP_RET(check_alias({{u_in, b}}, {{u_out, b}}));
  LP_RET(check_alias({{phase, (size_t)npix * phase_batch * esize(t) / 2}}, {{u_out, b}}));
  const int64_t pbs = phase_batch == 1 ? 0 : npix;
  const hipStream_t s = (hipStream_t)stream;
  CtxLock lk;
  const double es = (double)esize(t);
  LP_TRACE("modulate", (double)npix * batch * 2.0 * es + (double)npix * phase_batch * es / 2, s,
           (t == PROP_C64 ? launch_modulate<float>((const cx<float>*)u_in, (const float*)phase, (cx<float>*)u_out,
                                                   npix, batch, pbs, s, conj)
                          : launch_modulate<double>((const cx<double>*)u_in, (const double*)phase,
                                                    (cx<double>*)u_out, npix, batch, pbs, s, conj)));
  return PROP_OK;
}

int prop_modulate(prop_dtype t, const void* u_in, const void* phase, void* u_out, int64_t npix, int32_t batch,
                  int32_t phase_batch, void* stream) {
  return modulate_run(t, u_in, phase, u_out, npix, batch, phase_batch, stream, false);
}

int prop_modulate_adjoint(prop_dtype t, const void* g_out, const void* phase, void* g_in, int64_t npix,
                          int32_t batch, int32_t phase_batch, void* stream) {
  return modulate_run(t, g_out, phase, g_in, npix, batch, phase_batch, stream, true);
}

int prop_phase_grad(prop_dtype t, const void* g_u, const void* u, void* grad, int64_t npix, int32_t batch,
                    int32_t accumulate, void* stream) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (npix < 0 || batch < 0) return PROP_ESHAPE;
  if (npix == 0 || batch == 0) return PROP_OK;
  if (!g_u || !u || !grad) return PROP_ENULL;
  const size_t b = (size_t)npix * batch * esize(t);
  LP_RET(check_alias({{g_u, b}, {u, b}}, {{grad, b / 2}}));
  const hipStream_t s = (hipStream_t)stream;
  CtxLock lk;
  LP_TRACE("phase_grad", (double)b * 2.0 + (double)b / 2 * (accumulate ? 2 : 1), s,
           (t == PROP_C64 ? launch_phase_grad<float>((const cx<float>*)g_u, (const cx<float>*)u, (float*)grad, npix,
                                                     batch, accumulate, s)
                          : launch_phase_grad<double>((const cx<double>*)g_u, (const cx<double>*)u, (double*)grad,
                                                      npix, batch, accumulate, s)));
  return PROP_OK;
}

// The planes of one port: all ncomp entries of a given array must be set.
static int port_planes(const void* const* arr, int ncomp, size_t bytes, Planes* out, std::vector<Span>* spans) {
  *out = Planes{{nullptr, nullptr, nullptr}};
  if (!arr) return PROP_OK;
  for (int k = 0; k < ncomp; ++k) {
    if (!arr[k]) return PROP_ENULL;
    out->p[k] = arr[k];
    spans->push_back({arr[k], bytes});
  }
  return PROP_OK;
}

int prop_phase_grad_sum(prop_dtype t, const void* g_u, const void* u, void* grad, int64_t npix, int32_t batch,
                        int32_t accumulate, void* stream) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (npix < 0 || batch < 0) return PROP_ESHAPE;
  if (npix == 0) return PROP_OK;
  if (!grad || (batch > 0 && (!g_u || !u))) return PROP_ENULL;
  const size_t b = (size_t)npix * batch * esize(t);
  LP_RET(check_alias({{g_u, b}, {u, b}}, {{grad, (size_t)npix * esize(t) / 2}}));
  const hipStream_t s = (hipStream_t)stream;
  LP_TRY(t == PROP_C64 ? launch_phase_grad_sum<float>((const cx<float>*)g_u, (const cx<float>*)u, (float*)grad, npix,
                                                      batch, accumulate, s)
                       : launch_phase_grad_sum<double>((const cx<double>*)g_u, (const cx<double>*)u, (double*)grad,
                                                       npix, batch, accumulate, s));
  return PROP_OK;
}

int prop_scale_items(prop_dtype t, const void* const* in, void* const* out, int32_t nplanes, const double* scale,
                     int64_t npix, int32_t batch, void* stream) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (nplanes < 1 || nplanes > 3 || npix < 0 || batch < 0) return PROP_ESHAPE;
  if (npix == 0 || batch == 0) return PROP_OK;
  if (!in || !out || !scale) return PROP_ENULL;
  const size_t bytes = (size_t)npix * batch * esize(t);
  std::vector<Span> ins = {{scale, 8 * (size_t)batch}}, outs;
  Planes pi, po;
  LP_RET(port_planes(in, nplanes, bytes, &pi, &ins));
  LP_RET(port_planes((const void* const*)out, nplanes, bytes, &po, &outs));
  // plane k may be written in place; any other overlap is rejected
  for (int k = 0; k < nplanes; ++k) {
    for (int m = 0; m < nplanes; ++m)
      if (!(m == k && out[k] == in[k]) && overlap(out[k], bytes, in[m], bytes)) return PROP_EALIAS;
    if (overlap(out[k], bytes, scale, 8 * (size_t)batch)) return PROP_EALIAS;
    for (int m = k + 1; m < nplanes; ++m)
      if (overlap(out[k], bytes, out[m], bytes)) return PROP_EALIAS;
  }
  const hipStream_t s = (hipStream_t)stream;
  LP_TRY(t == PROP_C64 ? launch_scale_items<float>(pi, po, nplanes, scale, npix, batch, s)
                       : launch_scale_items<double>(pi, po, nplanes, scale, npix, batch, s));
  return PROP_OK;
}

int prop_waveplate(prop_dtype t, const void* ex, const void* ey, void* ox, void* oy, double eta, double theta,
                   int64_t npix, int32_t batch, void* stream) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (!is_finite(eta) || !is_finite(theta)) return PROP_EPARAM;
  if (npix < 0 || batch < 0) return PROP_ESHAPE;
  if (npix == 0 || batch == 0) return PROP_OK;
  if (!ex || !ey || !ox || !oy) return PROP_ENULL;
  const size_t b = (size_t)npix * batch * esize(t);
  LP_RET(check_alias({{ex, b}, {ey, b}}, {{ox, b}, {oy, b}}));
  double J[8];
  jones(eta, theta, J);
  const hipStream_t s = (hipStream_t)stream;
  hipError_t e = t == PROP_C64 ? launch_jones<float>((const cx<float>*)ex, (const cx<float>*)ey, (cx<float>*)ox,
                                                     (cx<float>*)oy, J, npix, batch, s)
                               : launch_jones<double>((const cx<double>*)ex, (const cx<double>*)ey, (cx<double>*)ox,
                                                      (cx<double>*)oy, J, npix, batch, s);
  return e == hipSuccess ? PROP_OK : dev_err(e);
}

int prop_waveplate_adjoint(prop_dtype t, const void* gx, const void* gy, const void* ex, const void* ey, void* gex,
                           void* gey, double eta, double theta, double* dparams, int64_t npix, int32_t batch,
                           void* stream) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (!is_finite(eta) || !is_finite(theta)) return PROP_EPARAM;
  if (npix < 0 || batch < 0) return PROP_ESHAPE;
  if (npix == 0 || batch == 0) return PROP_OK;
  if (!gx || !gy || !ex || !ey || !gex || !gey || !dparams) return PROP_ENULL;
  const size_t b = (size_t)npix * batch * esize(t);
  LP_RET(check_alias({{gx, b}, {gy, b}, {ex, b}, {ey, b}}, {{gex, b}, {gey, b}, {dparams, 16 * (size_t)batch}}));
  double J[8], H[8], d[16];
  jones(eta, theta, J);
  conj_transpose(J, H);
  jones_derivs(eta, theta, d);
  CtxLock lk;
  int dev;
  LP_RET(cur_device(&dev));
  const hipStream_t s = (hipStream_t)stream;
  const int nblk = 256;
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, (size_t)nblk * batch * 2 * sizeof(double), s));
  hipError_t e;
  if (t == PROP_C64) {
    e = launch_jones<float>((const cx<float>*)gx, (const cx<float>*)gy, (cx<float>*)gex, (cx<float>*)gey, H, npix,
                            batch, s);
    if (e == hipSuccess)
      e = launch_jones_grad<float>((const cx<float>*)gx, (const cx<float>*)gy, (const cx<float>*)ex,
                                   (const cx<float>*)ey, d, dparams, (double*)wb.p, nblk, npix, batch, s);
  } else {
    e = launch_jones<double>((const cx<double>*)gx, (const cx<double>*)gy, (cx<double>*)gex, (cx<double>*)gey, H,
                             npix, batch, s);
    if (e == hipSuccess)
      e = launch_jones_grad<double>((const cx<double>*)gx, (const cx<double>*)gy, (const cx<double>*)ex,
                                    (const cx<double>*)ey, d, dparams, (double*)wb.p, nblk, npix, batch, s);
  }
  return e == hipSuccess ? PROP_OK : dev_err(e);
}

int prop_waveplate_batched(prop_dtype t, const void* ex, const void* ey, void* ox, void* oy, const double* params,
                           int64_t npix, int32_t batch, void* stream) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (npix < 0 || batch < 0) return PROP_ESHAPE;
  if (npix == 0 || batch == 0) return PROP_OK;
  if (!ex || !ey || !ox || !oy || !params) return PROP_ENULL;
  const size_t b = (size_t)npix * batch * esize(t);
  LP_RET(check_alias({{ex, b}, {ey, b}, {params, 16 * (size_t)batch}}, {{ox, b}, {oy, b}}));
  const hipStream_t s = (hipStream_t)stream;
  LP_TRY(t == PROP_C64 ? launch_jones_items<float>((const cx<float>*)ex, (const cx<float>*)ey, (cx<float>*)ox,
                                                   (cx<float>*)oy, params, false, npix, batch, s)
                       : launch_jones_items<double>((const cx<double>*)ex, (const cx<double>*)ey, (cx<double>*)ox,
                                                    (cx<double>*)oy, params, false, npix, batch, s));
  return PROP_OK;
}

int prop_waveplate_batched_adjoint(prop_dtype t, const void* gx, const void* gy, const void* ex, const void* ey,
                                   void* gex, void* gey, const double* params, double* dparams, int64_t npix,
                                   int32_t batch, void* stream) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (npix < 0 || batch < 0) return PROP_ESHAPE;
  if (npix == 0 || batch == 0) return PROP_OK;
  if (!gx || !gy || !gex || !params || (dparams && (!ex || !ey))) return PROP_ENULL;
  const size_t b = (size_t)npix * batch * esize(t);
  std::vector<Span> ins = {{gx, b}, {gy, b}, {params, 16 * (size_t)batch}};
  std::vector<Span> outs = {{gex, b}};
  if (gey) outs.push_back({gey, b});
  if (dparams) {
    ins.push_back({ex, b});
    ins.push_back({ey, b});
    outs.push_back({dparams, 16 * (size_t)batch});
  }
  LP_RET(check_alias(ins, outs));
  const hipStream_t s = (hipStream_t)stream;
  if (t == PROP_C64)
    LP_TRY(launch_jones_items<float>((const cx<float>*)gx, (const cx<float>*)gy, (cx<float>*)gex, (cx<float>*)gey,
                                     params, true, npix, batch, s));
  else
    LP_TRY(launch_jones_items<double>((const cx<double>*)gx, (const cx<double>*)gy, (cx<double>*)gex,
                                      (cx<double>*)gey, params, true, npix, batch, s));
  if (!dparams) return PROP_OK;
  CtxLock lk;
  int dev;
  LP_RET(cur_device(&dev));
  const int nblk = red_blocks(npix);
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, (size_t)nblk * batch * 2 * sizeof(double), s));
  LP_TRY(t == PROP_C64
             ? launch_jones_items_grad<float>((const cx<float>*)gx, (const cx<float>*)gy, (const cx<float>*)ex,
                                              (const cx<float>*)ey, params, dparams, (double*)wb.p, nblk, npix,
                                              batch, s)
             : launch_jones_items_grad<double>((const cx<double>*)gx, (const cx<double>*)gy, (const cx<double>*)ex,
                                               (const cx<double>*)ey, params, dparams, (double*)wb.p, nblk, npix,
                                               batch, s));
  return PROP_OK;
}

int prop_beam_splitter(prop_dtype t, const void* const* a, const void* const* b, void* const* c, void* const* d,
                       int32_t ncomp, const double* alpha, int64_t npix, int32_t batch, void* stream) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (ncomp < 1 || ncomp > 3 || npix < 0 || batch < 0) return PROP_ESHAPE;
  if (npix == 0 || batch == 0) return PROP_OK;
  if (!c || !d || !alpha) return PROP_ENULL;
  const size_t bytes = (size_t)npix * batch * esize(t);
  std::vector<Span> ins = {{alpha, 8 * (size_t)batch}}, outs;
  Planes pa, pb, pc, pd;
  LP_RET(port_planes(a, ncomp, bytes, &pa, &ins));
  LP_RET(port_planes(b, ncomp, bytes, &pb, &ins));
  LP_RET(port_planes((const void* const*)c, ncomp, bytes, &pc, &outs));
  LP_RET(port_planes((const void* const*)d, ncomp, bytes, &pd, &outs));
  LP_RET(check_alias(ins, outs));
  const hipStream_t s = (hipStream_t)stream;
  LP_TRY(t == PROP_C64 ? launch_beam_splitter<float>(pa, pb, pc, pd, ncomp, a != nullptr, b != nullptr, alpha, npix,
                                                     batch, s)
                       : launch_beam_splitter<double>(pa, pb, pc, pd, ncomp, a != nullptr, b != nullptr, alpha, npix,
                                                      batch, s));
  return PROP_OK;
}

int prop_beam_splitter_adjoint(prop_dtype t, const void* const* gc, const void* const* gd, const void* const* a,
                               const void* const* b, void* const* ga, void* const* gb, int32_t ncomp,
                               const double* alpha, double* dalpha, int64_t npix, int32_t batch, void* stream) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (ncomp < 1 || ncomp > 3 || npix < 0 || batch < 0) return PROP_ESHAPE;
  if (npix == 0 || batch == 0) return PROP_OK;
  if (!gc || !gd || !alpha) return PROP_ENULL;
  const size_t bytes = (size_t)npix * batch * esize(t);
  std::vector<Span> ins = {{alpha, 8 * (size_t)batch}}, outs;
  Planes pgc, pgd, pa, pb, pga, pgb;
  LP_RET(port_planes(gc, ncomp, bytes, &pgc, &ins));
  LP_RET(port_planes(gd, ncomp, bytes, &pgd, &ins));
  LP_RET(port_planes(dalpha ? a : nullptr, ncomp, bytes, &pa, &ins));
  LP_RET(port_planes(dalpha ? b : nullptr, ncomp, bytes, &pb, &ins));
  LP_RET(port_planes((const void* const*)ga, ncomp, bytes, &pga, &outs));
  LP_RET(port_planes((const void* const*)gb, ncomp, bytes, &pgb, &outs));
  if (dalpha) outs.push_back({dalpha, 8 * (size_t)batch});
  LP_RET(check_alias(ins, outs));
  const int flags = (a && dalpha ? 1 : 0) | (b && dalpha ? 2 : 0) | (ga ? 4 : 0) | (gb ? 8 : 0) | (dalpha ? 16 : 0);
  if (!(flags & 28)) return PROP_OK;
  const hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<CtxLock> lk;
  double* partial = nullptr;
  int nblk = item_blocks_host(npix, batch);
  if (dalpha) {
    lk.reset(new CtxLock());
    int dev;
    LP_RET(cur_device(&dev));
    nblk = red_blocks(npix);
    Buf& wb = ctx().work[{dev, s}];
    LP_RET(ensure_buf(wb, (size_t)nblk * batch * 2 * sizeof(double), s));
    partial = (double*)wb.p;
  }
  LP_TRY(t == PROP_C64 ? launch_beam_splitter_adj<float>(pgc, pgd, pa, pb, pga, pgb, ncomp, flags, alpha, dalpha,
                                                         partial, nblk, npix, batch, s)
                       : launch_beam_splitter_adj<double>(pgc, pgd, pa, pb, pga, pgb, ncomp, flags, alpha, dalpha,
                                                          partial, nblk, npix, batch, s));
  return PROP_OK;
}

int prop_spot_loss(prop_dtype t, const void* ex, const void* ey, const void* ez, const prop_grid* win,
                   double wavelength, double w_fz, double* result, void* gx, void* gy, void* gz, int32_t batch,
                   void* stream) {
  LP_RET(spot_loss_check(t, ex, ey, ez, win, wavelength, w_fz, result, gx, gy, gz, batch));
  if (batch == 0) return PROP_OK;
  CtxLock lk;
  int dev;
  LP_RET(cur_device(&dev));
  const hipStream_t s = (hipStream_t)stream;
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, (size_t)kSpotBlocks * batch * 5 * sizeof(double), s));
  return spot_loss_launch(t, ex, ey, ez, win, wavelength, w_fz, result, gx, gy, gz, batch, (double*)wb.p, s);
}

int prop_spot_loss_noalloc(prop_dtype t, const void* ex, const void* ey, const void* ez, const prop_grid* win,
                           double wavelength, double w_fz, double* result, void* gx, void* gy, void* gz,
                           int32_t batch, void* stream) {
  LP_RET(spot_loss_check(t, ex, ey, ez, win, wavelength, w_fz, result, gx, gy, gz, batch));
  if (batch > kNoAllocMaxBatch) return PROP_ELIMIT;
  if (batch == 0) return PROP_OK;
  double* partial = nullptr;
  LP_RET(noalloc_scratch(&partial));
  // every partial the final reduction reads is written first by this call:
  // nothing in the shared array needs clearing
  return spot_loss_launch(t, ex, ey, ez, win, wavelength, w_fz, result, gx, gy, gz, batch, partial,
                          (hipStream_t)stream);
}

int prop_sampling_check(const prop_grid* g, double wavelength, double z) {
  LP_RET(check_grid(g));
  if (!(wavelength > 0) || !is_finite(wavelength) || !(z > 0) || !is_finite(z)) return PROP_EPARAM;
  return sampling(g, wavelength, z);
}

int32_t prop_fft_length(int32_t n) { return fft_len(n); }

int prop_density_loss(prop_dtype t, const void* const* comps, int32_t ncomp, const void* const* dep, int32_t ndep,
                      double beta, int64_t npix, double eps, double* result, void* const* seeds,
                      void* const* dep_seeds, int32_t batch, void* stream) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (ncomp < 1 || ncomp > 3 || ndep < 0 || ndep > 3 || npix < 1 || batch < 0) return PROP_ESHAPE;
  if (!(eps >= 0.0 && eps <= 1.0) || !(beta >= 0.0 && beta <= 1.0)) return PROP_EPARAM;
  if (batch == 0) return PROP_OK;
  if (!comps || !result || (ndep > 0 && !dep)) return PROP_ENULL;
  for (int k = 0; k < ncomp; ++k)
    if (!comps[k]) return PROP_ENULL;
  for (int k = 0; k < ndep; ++k)
    if (!dep[k]) return PROP_ENULL;
  CtxLock lk;
  const hipStream_t s = (hipStream_t)stream;
  int dev;
  LP_RET(cur_device(&dev));
  const int nblk = red_blocks(npix);
  Buf& wb = ctx().work[{dev, s}];
  LP_RET(ensure_buf(wb, (size_t)3 * batch * nblk * sizeof(double), s));
  LP_TRY(t == PROP_C64 ? launch_density_loss<float>(comps, ncomp, dep, ndep, beta, npix, eps, result, (double*)wb.p,
                                                    nblk, seeds, dep_seeds, batch, s)
                       : launch_density_loss<double>(comps, ncomp, dep, ndep, beta, npix, eps, result, (double*)wb.p,
                                                     nblk, seeds, dep_seeds, batch, s));
  return PROP_OK;
}

int prop_adam_step(prop_dtype t, void* param, const void* grad, void* m, void* v, int64_t n, double lr, double beta1,
                   double beta2, double eps, double weight_decay, int32_t step, void* stream) {
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (n < 0 || step < 1) return PROP_ESHAPE;
  if (!(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0) ||
      !(weight_decay >= 0) || !is_finite(lr) || !is_finite(weight_decay))
    return PROP_EPARAM;
  if (n == 0) return PROP_OK;
  if (!param || !grad || !m || !v) return PROP_ENULL;
  const size_t b = (size_t)n * (t == PROP_C64 ? 4 : 8);
  LP_RET(check_alias({{grad, b}}, {{param, b}, {m, b}, {v, b}}));
  const hipStream_t s = (hipStream_t)stream;
  LP_TRY(t == PROP_C64 ? launch_adam<float>((float*)param, (const float*)grad, (float*)m, (float*)v, n, lr, beta1,
                                            beta2, eps, weight_decay, step, s)
                       : launch_adam<double>((double*)param, (const double*)grad, (double*)m, (double*)v, n, lr,
                                             beta1, beta2, eps, weight_decay, step, s));
  return PROP_OK;
}

int prop_softmin(const double* losses, int32_t ndet, double beta, double* value, double* weights, int32_t batch,
                 void* stream) {
  if (ndet < 1 || batch < 0) return PROP_ESHAPE;
  if (!(beta > 0.0) || !is_finite(beta)) return PROP_EPARAM;
  if (batch == 0) return PROP_OK;
  if (!losses || !value) return PROP_ENULL;
  LP_TRY(launch_softmin(losses, ndet, beta, value, weights, batch, (hipStream_t)stream));
  return PROP_OK;
}

int prop_track_best(const double* loss, double* best, int64_t* since, int32_t batch, void* stream) {
  if (batch < 0) return PROP_ESHAPE;
  if (batch == 0) return PROP_OK;
  if (!loss || !best || !since) return PROP_ENULL;
  const size_t nb = (size_t)batch;
  LP_RET(check_alias({{loss, nb * sizeof(double)}}, {{best, nb * sizeof(double)}, {since, nb * sizeof(int64_t)}}));
  LP_TRY(launch_track_best(loss, best, since, batch, (hipStream_t)stream));
  return PROP_OK;
}

int prop_sum_items(const double* in, double* out, int32_t n, int32_t m, void* stream) {
  if (n < 1 || m < 1) return PROP_ESHAPE;
  if (!in || !out) return PROP_ENULL;
  LP_RET(check_alias({{in, (size_t)n * m * sizeof(double)}}, {{out, (size_t)m * sizeof(double)}}));
  LP_TRY(launch_sum_items(in, out, n, m, (hipStream_t)stream));
  return PROP_OK;
}

int32_t prop_autotune_report(char* buf, int32_t cap) {
  CtxLock lk;
  Ctx& C = ctx();
  std::string out;
  static const char* kinds[] = {"rs_cols", "vrs_mix2", "czt_cols", "czt_rows"};
  for (const auto& kv : C.tuned) {
    const TuneKey& k = kv.first;
    const TuneEntry& e = kv.second;
    char line[320];
    const int esz = std::get<1>(k), kind = std::get<2>(k), n = std::get<3>(k);
    const int lines = esz == 4 ? col_pass_lines<float>(kind, n, e.variant) : col_pass_lines<double>(kind, n, e.variant);
    SchedInfo si;
    char sched[48] = "?";
    if (sched_info(n, &si, esz == 8, variant_sched(e.variant) != 0)) {
      int o = 0;
      for (int st = 0; st < si.nst && o < (int)sizeof sched - 8; ++st)
        o += std::snprintf(sched + o, sizeof sched - o, st ? "x%d" : "%d", si.rad[st]);
    }
    int m = std::snprintf(line, sizeof line,
                          "dev %d %s %s n=%d lines=%d in=%d out=%d batch=%d -> variant %d (schedule %s, %d per "
                          "workgroup; %s); ms",
                          std::get<0>(k), esz == 4 ? "c64" : "c128", kinds[kind], n, std::get<4>(k), std::get<5>(k),
                          std::get<6>(k), std::get<7>(k), e.variant, sched, lines, e.from_file ? "from file" : "timed");
    out.append(line, (size_t)std::max(0, std::min<int>(m, (int)sizeof line - 1)));
    for (int v = 0; v < kTuneCandidates; ++v) {
      m = e.ms[v] < 0 ? std::snprintf(line, sizeof line, " -") : std::snprintf(line, sizeof line, " %.4f", e.ms[v]);
      out.append(line, (size_t)std::max(0, std::min<int>(m, (int)sizeof line - 1)));
    }
    out.push_back('\n');
  }
  if (buf && cap > 0) {
    const size_t nc = std::min<size_t>(out.size(), (size_t)cap - 1);
    std::memcpy(buf, out.data(), nc);
    buf[nc] = 0;
  }
  return (int32_t)out.size() + 1;
}

void prop_cache_clear(void) {
  CtxLock lk;
  Ctx& C = ctx();
  (void)hipDeviceSynchronize();
  // tables pinned by live plans stay: their kernels and graphs address them
  C.tws.clear_unpinned([](TwEntry& e) { (void)hipFree(e.tw); });
  C.specs.clear_unpinned(release_spec);
  C.zooms.clear_unpinned(release_zoom);
  for (auto& kv : C.work) (void)hipFree(kv.second.p);
  for (auto& kv : C.gen_scratch) (void)hipFree(kv.second.p);
  for (auto& kv : C.tune_a) (void)hipFree(kv.second.p);
  for (auto& kv : C.tune_b) (void)hipFree(kv.second.p);
  C.tune_a.clear();
  C.tune_b.clear();
  C.tuned.clear();
  C.work.clear();
  C.gen_scratch.clear();
}

int32_t prop_tune_cache_path(const char* path) {
  CtxLock lk;
  Ctx& C = ctx();
  C.tune_path_set = path != nullptr;
  C.tune_path = path ? path : "";
  C.tune_loaded = false;
  C.tune_file.clear();
  C.tune_rejected = 0;
  tune_file_load(C);
  return (int32_t)C.tune_file.size();
}

int32_t prop_tune_cache_rejected(void) {
  CtxLock lk;
  return ctx().tune_rejected;
}

void prop_cache_set_limit(int64_t bytes) {
  CtxLock lk;
  Ctx& C = ctx();
  C.limit = bytes > 0 ? (size_t)bytes : default_cache_limit();
  if (C.specs.bytes() + C.zooms.bytes() > C.limit) evict_tables(C, C.limit);
}

void prop_cache_info(prop_cache_stats* out) {
  if (!out) return;
  CtxLock lk;
  Ctx& C = ctx();
  out->table_bytes = (int64_t)(C.specs.bytes() + C.zooms.bytes());
  out->limit = (int64_t)C.limit;
  out->spectra = (int64_t)C.specs.size();
  out->zooms = (int64_t)C.zooms.size();
  out->twiddles = (int64_t)C.tws.size();
  out->pinned = (int64_t)(C.specs.pinned() + C.zooms.pinned() + C.tws.pinned());
  out->evictions = (int64_t)(C.specs.evictions() + C.zooms.evictions());
  out->eviction_syncs = (int64_t)C.evict_syncs;
}

const char* prop_status_string(int status) {
  switch (status) {
    case PROP_OK: return "ok";
    case PROP_WUNDERSAMPLED: return "warning: propagation kernel under-sampled at the largest offset";
    case PROP_ENULL: return "error: null pointer";
    case PROP_ESHAPE: return "error: unsupported shape (size < 1, negative batch or transform length > 8192)";
    case PROP_EPARAM: return "error: invalid parameter (dtype, wavelength, distance, pitch, NA, focal length)";
    case PROP_EALIAS: return "error: output overlaps an input";
    case PROP_ENOMEM: return "error: device allocation failed";
    case PROP_EDEVICE: return "error: HIP call failed (see prop_last_device_error)";
    case PROP_ELIMIT: return "error: request exceeds the fixed scratch of an allocation-free entry point";
    default: return "unknown status";
  }
}


int prop_plan_create(prop_dtype t, const prop_setup* setups, int32_t n, uint32_t flags, prop_plan** plan) {
  if (!plan) return PROP_ENULL;
  *plan = nullptr;
  if (t != PROP_C64 && t != PROP_C128) return PROP_EPARAM;
  if (n < 1) return PROP_ESHAPE;
  if (!setups) return PROP_ENULL;
  for (int i = 0; i < n; ++i) LP_RET(validate_setup(t, setups[i]));
  CtxLock lk;
  prop_plan* p = new prop_plan();
  p->t = t;
  p->flags = flags;
  auto fail = [&](int r) {
    for (auto& b : p->work) (void)hipFree(b.p);
    for (auto& b : p->gbuf) (void)hipFree(b.p);
    for (auto& b : p->mid) (void)hipFree(b.p);
    for (auto& s : p->setups) {
      (void)hipFree(s.umod);
      (void)hipFree(s.lens);
    }
    for (auto s : p->br) (void)hipStreamDestroy(s);
    if (p->fork) (void)hipEventDestroy(p->fork);
    for (auto e : p->join) (void)hipEventDestroy(e);
    ctx().pins = nullptr;
    unpin_all(p->pins);
    delete p;
    return r;
  };
  int r = cur_device(&p->dev);
  if (r < 0) return fail(r);
  p->nbranch = (flags & PROP_PLAN_GRAPH) ? std::min(4, n) : 1;
  size_t wmax = 1, gmax = 1, mmax = 1;
  for (int i = 0; i < n; ++i) {
    PlanSetup ps;
    ps.s = setups[i];
    ps.ncomp_in = ncomp_in(ps.s.op);
    const bool staged = ps.s.phase != nullptr || ps.s.lens_f > 0;
    ps.modulated = staged && vector_op(ps.s.op);
    ps.fused = staged && !vector_op(ps.s.op);
    const size_t plane = (size_t)ps.s.g_in.nx * ps.s.g_in.ny * ps.s.batch * esize(t);
    if (ps.modulated) {
      hipError_t e = hipMalloc(&ps.umod, plane * ps.ncomp_in);
      if (e != hipSuccess) {
        p->setups.push_back(ps);
        return fail(dev_err(e));
      }
      gmax = std::max(gmax, plane * ps.ncomp_in);
    }
    if (ps.fused && ps.s.op == PROP_OP_RS && ps.s.lens_f > 0) {
      // separable thin-lens factors exp(-i k x^2 / 2f), exp(-i k y^2 / 2f),
      // evaluated in long double and rounded once to the element type
      const int nx = ps.s.g_in.nx, ny = ps.s.g_in.ny;
      const long double qq = (2.0L * 3.141592653589793238462643383279502884L / ps.s.wavelength) / (2.0L * ps.s.lens_f);
      std::vector<long double> re(nx + ny), im(nx + ny);
      for (int j = 0; j < nx + ny; ++j) {
        const long double x = j < nx ? (long double)ps.s.g_in.cx + (long double)(j - nx / 2) * ps.s.g_in.dx
                                     : (long double)ps.s.g_in.cy + (long double)(j - nx - ny / 2) * ps.s.g_in.dy;
        const long double ph = -qq * x * x;
        re[j] = cosl(ph);
        im[j] = sinl(ph);
      }
      const size_t lb = (size_t)(nx + ny) * esize(t);
      std::vector<char> hb(lb);
      for (int j = 0; j < nx + ny; ++j) {
        if (t == PROP_C64) {
          ((float*)hb.data())[2 * j] = (float)re[j];
          ((float*)hb.data())[2 * j + 1] = (float)im[j];
        } else {
          ((double*)hb.data())[2 * j] = (double)re[j];
          ((double*)hb.data())[2 * j + 1] = (double)im[j];
        }
      }
      hipError_t e = hipMalloc(&ps.lens, lb);
      if (e == hipSuccess) e = hipMemcpy(ps.lens, hb.data(), lb, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        p->setups.push_back(ps);
        return fail(dev_err(e));
      }
    }
    if (ps.s.op == PROP_OP_RS_CZT) mmax = std::max(mmax, plane);
    wmax = std::max(wmax, setup_work_bytes(t, ps.s));
    ps.cost = setup_cost(ps.s);
    p->setups.push_back(ps);
  }
  // branches: longest-first onto the least-loaded stream, so the concurrent
  // streams of a graph finish together
  p->order.resize(n);
  for (int i = 0; i < n; ++i) p->order[i] = i;
  std::stable_sort(p->order.begin(), p->order.end(),
                   [&](int a, int b) { return p->setups[a].cost > p->setups[b].cost; });
  std::vector<double> load(p->nbranch, 0.0);
  for (int i : p->order) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    p->setups[i].branch = b;
    load[b] += p->setups[i].cost;
  }
  p->work.resize(p->nbranch);
  p->gbuf.resize(p->nbranch);
  p->mid.resize(p->nbranch);
  for (int b = 0; b < p->nbranch; ++b) {
    // fault injection: the workspace allocation fails as on an exhausted device
    r = (flags & PROP_PLAN_FAULT_NOMEM) ? dev_err(hipErrorOutOfMemory) : ensure_buf(p->work[b], wmax, nullptr);
    if (r < 0) return fail(r);
    r = ensure_buf(p->gbuf[b], gmax, nullptr);
    if (r < 0) return fail(r);
    r = ensure_buf(p->mid[b], mmax, nullptr);
    if (r < 0) return fail(r);
  }
  // every table the setups use is computed now and pinned for the plan's
  // lifetime: its kernels (and captured graphs) address them directly
  ctx().pins = &p->pins;
  for (auto& ps : p->setups) {
    r = t == PROP_C64 ? warm_setup<float>(p->dev, ps.s, nullptr) : warm_setup<double>(p->dev, ps.s, nullptr);
    if (r < 0) return fail(r);
  }
  ctx().pins = nullptr;
  if (flags & PROP_PLAN_GRAPH) {
    for (int b = 0; b < p->nbranch; ++b) {
      hipStream_t s;
      hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
      if (e != hipSuccess) return fail(dev_err(e));
      p->br.push_back(s);
      hipEvent_t ev;
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) return fail(dev_err(e));
      p->join.push_back(ev);
    }
    hipError_t e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    if (e != hipSuccess) return fail(dev_err(e));
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail(dev_err(e));
  mark_ready(p->pins);
  *plan = p;
  return PROP_OK;
}

int prop_plan_forward(prop_plan* plan, void* stream) {
  if (!plan) return PROP_ENULL;
  CtxLock lk;
  return plan_run(plan, 0, (hipStream_t)stream);
}

int prop_plan_adjoint(prop_plan* plan, void* stream) {
  if (!plan) return PROP_ENULL;
  CtxLock lk;
  return plan_run(plan, 1, (hipStream_t)stream);
}

int prop_plan_step(prop_plan* plan, void* stream) {
  if (!plan) return PROP_ENULL;
  CtxLock lk;
  return plan_run(plan, 2, (hipStream_t)stream);
}

void prop_plan_destroy(prop_plan* plan) {
  if (!plan) return;
  CtxLock lk;
  (void)hipDeviceSynchronize();
  for (int k = 0; k < 3; ++k)
    if (plan->gexec[k]) (void)hipGraphExecDestroy(plan->gexec[k]);
  for (auto& b : plan->work) (void)hipFree(b.p);
  for (auto& b : plan->gbuf) (void)hipFree(b.p);
  for (auto& b : plan->mid) (void)hipFree(b.p);
  for (auto& s : plan->setups) {
    (void)hipFree(s.umod);
    (void)hipFree(s.lens);
  }
  for (auto s : plan->br) (void)hipStreamDestroy(s);
  if (plan->fork) (void)hipEventDestroy(plan->fork);
  for (auto e : plan->join) (void)hipEventDestroy(e);
  unpin_all(plan->pins);
  delete plan;
}

int prop_last_device_error(void) { return g_last_hip; }

void prop_trace_enable(int32_t on) {
  CtxLock lk;
  Tracer& t = tracer();
  for (auto& r : t.recs) {
    (void)hipEventSynchronize(r.b);
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
  }
  t.recs.clear();
  t.on = on != 0;
}

void prop_trace_only(const char* name) {
  CtxLock lk;
  tracer().only = name ? name : "";
}

int32_t prop_trace_read(prop_trace_stat* out, int32_t max) {
  CtxLock lk;
  Tracer& t = tracer();
  std::vector<prop_trace_stat> agg;
  int status = 0;
  for (auto& r : t.recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) status = -1;
    prop_trace_stat* e = nullptr;
    for (auto& a : agg)
      if (std::strncmp(a.name, r.name, sizeof(a.name)) == 0) e = &a;
    if (!e) {
      prop_trace_stat z;
      std::memset(&z, 0, sizeof(z));
      std::strncpy(z.name, r.name, sizeof(z.name) - 1);
      agg.push_back(z);
      e = &agg.back();
    }
    e->launches += 1;
    e->total_ms += ms;
    e->bytes += r.bytes;
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
  }
  t.recs.clear();
  if (status < 0) return PROP_EDEVICE;
  const int n = std::min<int>((int)agg.size(), max);
  for (int i = 0; i < n && out; ++i) out[i] = agg[i];
  return n;
}

}  // extern "C"
