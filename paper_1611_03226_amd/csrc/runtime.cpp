// Host runtime behind the dfhip.h C ABI: network registry (actors and FIFO
// channels, Sec. 2.2 / 3.2), all-or-nothing batch admission (the blocking
// reads and writes of Sec. 2.2), host push/pop, and the kernel chains that
// fire a batch.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "dfhip.h"
#include "host_logic.h"
#include "runtime.h"

using namespace dfh;

static thread_local std::string g_tls_error;

// ------------------------------------------------------------------ errors

df_status dfh::fail(df_graph *g, df_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (g) g->last_error = buf;
  g_tls_error = buf;
  return st;
}

df_status dfh::fail_hip(df_graph *g, hipError_t e, const char *what) {
  if (g) g->poisoned = true;
  return fail(g, DF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(g, expr)                                  \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return fail_hip((g), e_, #expr); \
  } while (0)

#define ENTER(g)                                                          \
  do {                                                                    \
    if (!(g)) return fail(nullptr, DF_EINVAL, "null graph");              \
    if ((g)->poisoned) return fail((g), DF_EDEVICE, "graph poisoned by an earlier HIP error"); \
    hipError_t e0_ = hipSetDevice((g)->device);                           \
    if (e0_ != hipSuccess) return fail_hip((g), e0_, "hipSetDevice");     \
  } while (0)

using host::next_pow2;

static host::SlotMap slot_map(const Fifo &f) {
  host::SlotMap m;
  m.cap = f.cap;
  m.period = f.period;
  m.delay = f.n_initial != 0;
  return m;
}

static int64_t dtype_bytes(int dt) {
  switch (dt) {
    case DF_C64: return 8;
    case DF_U8: return 1;
    case DF_I32: return 4;
    case DF_I64: return 8;
    default: return 0;
  }
}

// ------------------------------------------------------------------ graph

extern "C" const char *df_version(void) { return "dfhip 0.1 gfx950"; }

extern "C" int64_t df_paper_channel_bytes(int64_t token_bytes, int64_t rate, int32_t has_delay) {
  if (token_bytes < 1 || rate < 1) return -1;
  return token_bytes * (has_delay ? 3 * rate + 1 : 2 * rate);
}

extern "C" const char *df_last_error(const df_graph *g) {
  if (g) return g->last_error.c_str();
  return g_tls_error.c_str();
}

extern "C" df_status df_graph_create(df_graph **out, int device, void *stream) {
  if (!out) return fail(nullptr, DF_EINVAL, "df_graph_create: null output pointer");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(nullptr, DF_EDEVICE, "no HIP device available");
  if (device < 0 || device >= n) return fail(nullptr, DF_EINVAL, "device %d out of range (have %d)", device, n);
  df_graph *g = new (std::nothrow) df_graph();
  if (!g) return fail(nullptr, DF_ENOMEM, "host allocation failed");
  g->device = device;
  if ((e = hipSetDevice(device)) != hipSuccess) {
    delete g;
    return fail(nullptr, DF_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  }
  if (stream) {
    g->stream = (hipStream_t)stream;
    g->own_stream = false;
  } else {
    if ((e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking)) != hipSuccess) {
      delete g;
      return fail(nullptr, DF_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    g->own_stream = true;
  }
  const size_t idx_bytes = sizeof(int64_t) * kCtrWords * kMaxFifos;
  if ((e = hipMalloc(&g->idx_pool, idx_bytes)) != hipSuccess ||
      (e = hipMalloc(&g->err_dev, sizeof(int32_t) * 4)) != hipSuccess ||
      (e = hipMemset(g->idx_pool, 0, idx_bytes)) != hipSuccess ||
      (e = hipMemset(g->err_dev, 0, sizeof(int32_t) * 4)) != hipSuccess) {
    df_graph_destroy(g);
    return fail(nullptr, DF_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
  }
  if (const char *v = getenv("DFHIP_CHECK_INDICES")) g->check_indices = atoi(v) != 0;
  if (const char *v = getenv("DFHIP_LOG")) g->log_level = atoi(v);
  if (const char *v = getenv("DFHIP_SCAN_AHEAD")) g->no_scan_ahead = atoi(v) == 0;
  g->body_mx = dpd_body_mx_env();
  if (const char *v = getenv("DFHIP_TILE")) {
    // "tile_outputs,outputs_per_thread,blocks_per_cu" (0 keeps a default)
    int t = 0, k = 0, b = 0;
    if (sscanf(v, "%d,%d,%d", &t, &k, &b) < 1 || df_set_tile(g, t, k, b) != DF_OK) {
      df_graph_destroy(g);
      return fail(nullptr, DF_EINVAL, "DFHIP_TILE=\"%s\" is not tile,outputs_per_thread,blocks_per_cu", v);
    }
  }
  *out = g;
  return DF_OK;
}

static void free_actor(Actor &a) {
  (void)hipFree(a.h);
  (void)hipFree(a.hist);
  (void)hipFree(a.order);
  (void)hipFree(a.corr);
  (void)hipFree(a.ticket);
  (void)hipFree(a.prev);
  (void)hipFree(a.off);
  for (auto &sl : a.scan) {
    (void)hipFree(sl.B);
    (void)hipFree(sl.grp);
    (void)hipFree(sl.last);
    (void)hipFree(sl.err);
  }
  (void)hipFree(a.state);
  (void)hipFree(a.count);
  (void)hipFree(a.emit_off);
  (void)hipFree(a.bits);
  a = Actor();
}

extern "C" df_status df_graph_destroy(df_graph *g) {
  if (!g) return fail(nullptr, DF_EINVAL, "null graph");
  (void)hipSetDevice(g->device);
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  destroy_persistent(g);
  for (auto &pe : g->prof_pending) {
    (void)hipEventDestroy(pe.start);
    (void)hipEventDestroy(pe.stop);
  }
  for (auto ev : g->prof_pool) (void)hipEventDestroy(ev);
  for (auto &f : g->fifos) (void)hipFree(f.ring);
  for (auto &a : g->actors) free_actor(a);
  (void)hipFree(g->idx_pool);
  (void)hipFree(g->err_dev);
  if (g->copy_in) (void)hipStreamDestroy(g->copy_in);
  if (g->copy_out) (void)hipStreamDestroy(g->copy_out);
  if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
  return DF_OK;
}

df_status dfh::after_call(df_graph *g, df_status st) {
  if (st != DF_OK || !g->check_indices) return st;
  return sync_errors(g);
}

void dfh::dlog(const df_graph *g, int level, const char *fmt, ...) {
  if (!g || g->log_level < level) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  fprintf(stderr, "[dfhip] %s\n", buf);
}

extern "C" df_status df_sync(df_graph *g) {
  ENTER(g);
  return sync_errors(g);
}

df_status dfh::sync_errors(df_graph *g) {
  HIPCHK(g, hipStreamSynchronize(g->stream));
  int32_t err = 0;
  HIPCHK(g, hipMemcpy(&err, g->err_dev, sizeof err, hipMemcpyDeviceToHost));
  if (err & kErrIndex)
    return fail(g, DF_EINDEX, "a channel counter update broke read <= write <= read + capacity on the device");
  if (err & kErrControl) return fail(g, DF_ECONTROL, "a control token outside 0..n_branches_max was read on the device");
  return DF_OK;
}

// ------------------------------------------------------------------ FIFOs

// Register a channel of `cap` logical tokens (the admission capacity) over
// `slots` allocated slots; period > 0 selects the paper's layout.
static df_status make_fifo(df_graph *g, df_dtype dt, int64_t elems_per_token, int64_t cap, int64_t slots,
                           int64_t period, int64_t n_initial, const void *initial_host, int32_t *fifo_out) {
  const int64_t eb = dtype_bytes(dt);
  if ((int)g->fifos.size() >= kMaxFifos) return fail(g, DF_ENOMEM, "too many FIFOs (max %d)", kMaxFifos);
  Fifo f;
  f.dt = dt;
  f.elem_bytes = eb;
  f.elems_per_token = elems_per_token;
  f.token_bytes = eb * elems_per_token;
  f.cap = cap;
  f.mask = period ? 0 : cap - 1;
  f.period = period;
  f.slots = slots;
  f.n_initial = n_initial;
  const int id = (int)g->fifos.size();
  f.idx = g->idx_pool + kCtrWords * id;
  hipError_t e = hipMalloc(&f.ring, (size_t)(slots * f.token_bytes));
  if (e != hipSuccess) return fail(g, DF_ENOMEM, "channel allocation of %lld bytes failed",
                                   (long long)(slots * f.token_bytes));
  if (n_initial) {
    // initial tokens occupy positions 0..n_initial-1 (slot 0 in the paper's layout)
    if (initial_host)
      e = hipMemcpy(f.ring, initial_host, (size_t)(n_initial * f.token_bytes), hipMemcpyHostToDevice);
    else
      e = hipMemset(f.ring, 0, (size_t)(n_initial * f.token_bytes));
    if (e != hipSuccess) {
      (void)hipFree(f.ring);
      return fail_hip(g, e, "initial tokens");
    }
  }
  const int64_t init_idx[kCtrWords] = {0, n_initial, cap, 0};
  e = hipMemcpy(f.idx, init_idx, sizeof init_idx, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(f.ring);
    return fail_hip(g, e, "index init");
  }
  f.read_h = 0;
  f.write_lo = f.write_hi = n_initial;
  g->fifos.push_back(f);
  *fifo_out = id;
  return DF_OK;
}

extern "C" df_status df_fifo_create(df_graph *g, df_dtype dt, int64_t elems_per_token, int64_t capacity_tokens,
                                    int64_t n_initial, const void *initial_host, int32_t *fifo_out) {
  ENTER(g);
  if (!fifo_out) return fail(g, DF_EINVAL, "df_fifo_create: null output pointer");
  if (!dtype_bytes(dt)) return fail(g, DF_EINVAL, "df_fifo_create: bad dtype %d", (int)dt);
  if (elems_per_token < 1) return fail(g, DF_EINVAL, "df_fifo_create: elems_per_token must be >= 1");
  if (n_initial < 0 || capacity_tokens < 0) return fail(g, DF_EINVAL, "df_fifo_create: negative size");
  int64_t cap = capacity_tokens ? capacity_tokens : std::max<int64_t>(2 * n_initial, 1024);
  cap = next_pow2(cap);
  if (n_initial > cap) return fail(g, DF_EINVAL, "df_fifo_create: n_initial %lld exceeds capacity %lld",
                                   (long long)n_initial, (long long)cap);
  return make_fifo(g, dt, elems_per_token, cap, cap, 0, n_initial, initial_host, fifo_out);
}

extern "C" df_status df_fifo_create_paper(df_graph *g, df_dtype dt, int64_t elems_per_token, int64_t rate,
                                          int64_t n_initial, const void *initial_host, int32_t *fifo_out) {
  ENTER(g);
  if (!fifo_out) return fail(g, DF_EINVAL, "df_fifo_create_paper: null output pointer");
  if (!dtype_bytes(dt)) return fail(g, DF_EINVAL, "df_fifo_create_paper: bad dtype %d", (int)dt);
  if (elems_per_token < 1) return fail(g, DF_EINVAL, "df_fifo_create_paper: elems_per_token must be >= 1");
  if (rate < 1) return fail(g, DF_EINVAL, "df_fifo_create_paper: rate must be >= 1");
  if (n_initial != 0 && n_initial != 1)
    return fail(g, DF_EINVAL, "df_fifo_create_paper: the paper's layout holds 0 or 1 delay tokens");
  const int64_t period = n_initial ? 3 * rate : 2 * rate;
  return make_fifo(g, dt, elems_per_token, period, period + n_initial, period, n_initial, initial_host, fifo_out);
}

extern "C" int64_t df_fifo_bytes(df_graph *g, int32_t fifo) {
  if (!g || fifo < 0 || fifo >= (int)g->fifos.size()) return -1;
  const Fifo &f = g->fifos[fifo];
  return f.slots * f.token_bytes;
}

df_status dfh::refresh_fifo(df_graph *g, Fifo &f) {
  HIPCHK(g, hipStreamSynchronize(g->stream));
  int64_t idx[2];
  HIPCHK(g, hipMemcpy(idx, f.idx, sizeof idx, hipMemcpyDeviceToHost));
  f.read_h = idx[0];
  f.write_lo = f.write_hi = idx[1];
  return DF_OK;
}

extern "C" df_status df_fifo_status(df_graph *g, int32_t fifo, int64_t *read_idx, int64_t *write_idx,
                                    int64_t *capacity) {
  ENTER(g);
  if (fifo < 0 || fifo >= (int)g->fifos.size()) return fail(g, DF_EINVAL, "bad fifo id %d", fifo);
  Fifo &f = g->fifos[fifo];
  if (f.write_lo != f.write_hi) {
    df_status st = refresh_fifo(g, f);
    if (st) return st;
  }
  if (read_idx) *read_idx = f.read_h;
  if (write_idx) *write_idx = f.write_lo;
  if (capacity) *capacity = f.cap;
  return DF_OK;
}

extern "C" df_status df_fifo_info(df_graph *g, int32_t fifo, int32_t *dtype, int64_t *elems_per_token,
                                  int64_t *token_bytes) {
  if (!g) return fail(nullptr, DF_EINVAL, "null graph");
  if (fifo < 0 || fifo >= (int)g->fifos.size()) return fail(g, DF_EINVAL, "bad fifo id %d", fifo);
  const Fifo &f = g->fifos[fifo];
  if (dtype) *dtype = (int32_t)f.dt;
  if (elems_per_token) *elems_per_token = f.elems_per_token;
  if (token_bytes) *token_bytes = f.token_bytes;
  return DF_OK;
}

// ------------------------------------------------------------------ actors

extern "C" df_status df_actor_create(df_graph *g, df_actor_kind kind, const void *params, size_t params_size,
                                     int32_t *actor_out) {
  ENTER(g);
  if (!params || !actor_out) return fail(g, DF_EINVAL, "df_actor_create: null pointer");
  Actor a;
  a.kind = kind;
  hipError_t e;
  if (kind == DF_ACTOR_DPD) {
    // the struct without control_mode / reserved is accepted too (count tokens)
    const size_t short_size = offsetof(df_dpd_params, control_mode);
    if (params_size != sizeof(df_dpd_params) && params_size != short_size)
      return fail(g, DF_EINVAL, "df_actor_create: params_size mismatch");
    df_dpd_params p{};
    memcpy(&p, params, params_size);
    if (p.control_mode != DF_CTRL_COUNT && p.control_mode != DF_CTRL_MASK)
      return fail(g, DF_EINVAL, "bad control_mode %d", p.control_mode);
    if (p.n_branches_max < 1 || p.n_branches_max > kMaxBranches)
      return fail(g, DF_EINVAL, "n_branches_max %d outside 1..%d", p.n_branches_max, kMaxBranches);
    if (p.n_taps < 1 || p.n_taps > kMaxTaps) return fail(g, DF_EINVAL, "n_taps %d outside 1..%d", p.n_taps, kMaxTaps);
    if (p.firing_size < 1 || p.firing_size < p.n_taps - 1)
      return fail(g, DF_EINVAL, "firing_size %lld must be >= max(1, n_taps-1)", (long long)p.firing_size);
    if (p.history_mode != DF_HIST_BRANCH && p.history_mode != DF_HIST_SHARED)
      return fail(g, DF_EINVAL, "bad history_mode %d", p.history_mode);
    if (!p.coeffs) return fail(g, DF_EINVAL, "null coefficients");
    a.dp = p;
    a.dp.coeffs = nullptr;
    const size_t hb = sizeof(float2) * p.n_branches_max * p.n_taps;
    const size_t sb = sizeof(float2) * p.n_branches_max * std::max(p.n_taps - 1, 1);
    if ((e = hipMalloc(&a.h, hb)) != hipSuccess || (e = hipMalloc(&a.hist, sb)) != hipSuccess ||
        (e = hipMalloc(&a.scan[0].last, sizeof(int64_t) * p.n_branches_max)) != hipSuccess ||
        (e = hipMalloc(&a.scan[1].last, sizeof(int64_t) * p.n_branches_max)) != hipSuccess ||
        (e = hipMalloc(&a.scan[0].err, sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&a.scan[1].err, sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&a.ticket, sizeof(int32_t))) != hipSuccess) {
      free_actor(a);
      return fail(g, DF_ENOMEM, "actor allocation failed");
    }
    e = hipMemcpy(a.h, p.coeffs, hb, p.coeffs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(a.hist, 0, sb);
    if (e == hipSuccess) e = hipMemset(a.ticket, 0, sizeof(int32_t));
    for (auto &sl : a.scan)
      if (e == hipSuccess) e = hipMemset(sl.err, 0, sizeof(int32_t));
    if (e != hipSuccess) {
      free_actor(a);
      return fail_hip(g, e, "actor init");
    }
  } else if (kind == DF_ACTOR_MOTION) {
    if (params_size != sizeof(df_motion_params)) return fail(g, DF_EINVAL, "df_actor_create: params_size mismatch");
    const df_motion_params &p = *(const df_motion_params *)params;
    if (p.width < 1 || p.height < 1 || p.width > 65536 || p.height > 65536)
      return fail(g, DF_EINVAL, "bad frame size %dx%d", p.width, p.height);
    if (p.diff_threshold < 0 || p.diff_threshold > 255) return fail(g, DF_EINVAL, "diff_threshold outside 0..255");
    if (p.min_changed_permille < 0 || p.min_changed_permille > 1000)
      return fail(g, DF_EINVAL, "min_changed_permille outside 0..1000");
    if (p.self_delay != 0 && p.self_delay != 1) return fail(g, DF_EINVAL, "self_delay must be 0 or 1");
    a.mp = p;
    if (p.self_delay) {
      const size_t wh = (size_t)p.width * p.height;
      if ((e = hipMalloc(&a.state, wh)) != hipSuccess) return fail(g, DF_ENOMEM, "state allocation failed");
      if ((e = hipMemset(a.state, 0, wh)) != hipSuccess) {
        free_actor(a);
        return fail_hip(g, e, "state init");
      }
    }
  } else if (kind == DF_ACTOR_GAUSS5 || kind == DF_ACTOR_THRES || kind == DF_ACTOR_MED5) {
    if (params_size != sizeof(df_frame_params)) return fail(g, DF_EINVAL, "df_actor_create: params_size mismatch");
    const df_frame_params &p = *(const df_frame_params *)params;
    if (p.width < 1 || p.height < 1 || p.width > 65536 || p.height > 65536)
      return fail(g, DF_EINVAL, "bad frame size %dx%d", p.width, p.height);
    if (p.rate < 1) return fail(g, DF_EINVAL, "token rate must be >= 1");
    if (kind == DF_ACTOR_THRES && (p.threshold < 0 || p.threshold > 255))
      return fail(g, DF_EINVAL, "threshold outside 0..255");
    a.fp = p;
  } else {
    return fail(g, DF_EINVAL, "unknown actor kind %d", (int)kind);
  }
  *actor_out = (int32_t)g->actors.size();
  g->actors.push_back(a);
  return DF_OK;
}

// Port table: (dtype, elems per token, is_input); elems 0 = frame size.
struct PortSpec {
  df_dtype dt;
  bool frame;
  bool input;
  bool control;
};

static bool port_spec(const Actor &a, int port, PortSpec *ps) {
  if (a.kind == DF_ACTOR_DPD) {
    switch (port) {
      case DF_DPD_CTRL: *ps = {DF_I32, false, true, true}; return true;
      case DF_DPD_IN: *ps = {DF_C64, false, true, false}; return true;
      case DF_DPD_OUT: *ps = {DF_C64, false, false, false}; return true;
    }
  } else if (a.kind == DF_ACTOR_MOTION) {
    switch (port) {
      case DF_MD_CUR: *ps = {DF_U8, true, true, false}; return true;
      case DF_MD_PREV: *ps = {DF_U8, true, true, false}; return a.mp.self_delay == 0;
      case DF_MD_MASK: *ps = {DF_U8, true, false, false}; return true;
      case DF_MD_INDEX: *ps = {DF_I64, false, false, false}; return true;
    }
  } else if (a.kind == DF_ACTOR_GAUSS5 || a.kind == DF_ACTOR_THRES || a.kind == DF_ACTOR_MED5) {
    const int n_in = a.kind == DF_ACTOR_THRES ? 2 : 1;
    const int n_out = a.kind == DF_ACTOR_GAUSS5 ? 2 : 1;
    if (port < 0 || port >= n_in + n_out) return false;
    *ps = {DF_U8, true, port < n_in, false};
    return true;
  }
  return false;
}

// Pixels of a frame token of a frame actor.
static int64_t frame_elems(const Actor &a) {
  if (a.kind == DF_ACTOR_MOTION) return (int64_t)a.mp.width * a.mp.height;
  return (int64_t)a.fp.width * a.fp.height;
}

extern "C" df_status df_connect(df_graph *g, int32_t actor, int32_t port, int32_t fifo) {
  ENTER(g);
  if (actor < 0 || actor >= (int)g->actors.size()) return fail(g, DF_EINVAL, "bad actor id %d", actor);
  if (fifo < 0 || fifo >= (int)g->fifos.size()) return fail(g, DF_EINVAL, "bad fifo id %d", fifo);
  Actor &a = g->actors[actor];
  Fifo &f = g->fifos[fifo];
  PortSpec ps;
  if (!port_spec(a, port, &ps)) return fail(g, DF_EINVAL, "actor %d has no port %d", actor, port);
  if (f.period && !(a.kind == DF_ACTOR_GAUSS5 || a.kind == DF_ACTOR_THRES || a.kind == DF_ACTOR_MED5))
    return fail(g, DF_EINVAL, "channels in the paper's layout connect only to Gauss, Thres and Med actors");
  const int64_t want_elems = ps.frame ? frame_elems(a) : 1;
  if (f.dt != ps.dt || f.elems_per_token != want_elems)
    return fail(g, DF_EINVAL, "fifo %d token type does not match port %d", fifo, port);
  if (a.ports[port] >= 0) return fail(g, DF_ESTATE, "port %d of actor %d already connected", port, actor);
  if (ps.input) {
    if (f.reader >= 0) return fail(g, DF_ESTATE, "fifo %d already has a reader", fifo);
    if (f.writer == actor) return fail(g, DF_ESTATE, "an actor cannot read its own output channel");
    if (ps.control && f.n_initial)
      return fail(g, DF_ESTATE, "initial tokens are not allowed on a control channel");
    f.reader = actor;
    f.reader_port = port;
  } else {
    if (f.writer >= 0) return fail(g, DF_ESTATE, "fifo %d already has a writer", fifo);
    if (f.reader == actor) return fail(g, DF_ESTATE, "an actor cannot write its own input channel");
    f.writer = actor;
    f.writer_port = port;
  }
  a.ports[port] = fifo;
  return DF_OK;
}

extern "C" df_status df_port_rate(df_graph *g, int32_t actor, int32_t port, int64_t *rate) {
  if (!g) return fail(nullptr, DF_EINVAL, "null graph");
  if (actor < 0 || actor >= (int)g->actors.size()) return fail(g, DF_EINVAL, "bad actor id %d", actor);
  if (!rate) return fail(g, DF_EINVAL, "null output pointer");
  const Actor &a = g->actors[actor];
  PortSpec ps;
  if (!port_spec(a, port, &ps)) return fail(g, DF_EINVAL, "actor %d has no port %d", actor, port);
  if (a.kind == DF_ACTOR_DPD)
    *rate = port == DF_DPD_CTRL ? 1 : a.dp.firing_size;
  else if (a.kind == DF_ACTOR_MOTION)
    *rate = 1;
  else
    *rate = a.fp.rate;
  return DF_OK;
}

// ------------------------------------------------------------------ push / pop

// Copy n tokens between a channel (starting at token position pos) and a
// flat buffer, on stream `st` (the graph's stream when null), one
// hipMemcpyAsync per run of consecutive slots.
static hipError_t ring_copy(df_graph *g, Fifo &f, int64_t pos, void *flat, int64_t n, bool to_ring,
                            bool flat_on_device, hipStream_t st = nullptr) {
  if (!st) st = g->stream;
  const size_t tb = (size_t)f.token_bytes;
  const host::SlotMap m = slot_map(f);
  hipMemcpyKind kind = to_ring ? (flat_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice)
                               : (flat_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
  char *p = (char *)flat;
  for (int64_t done = 0; done < n;) {
    const host::Run run = host::next_run(m, pos + done, n - done, to_ring);
    hipError_t e = to_ring ? hipMemcpyAsync(f.ring + run.slot * tb, p + done * tb, run.count * tb, kind, st)
                           : hipMemcpyAsync(p + done * tb, f.ring + run.slot * tb, run.count * tb, kind, st);
    if (e != hipSuccess) return e;
    done += run.count;
  }
  return hipSuccess;
}

// The paper's delay-token layout: after writes of positions [pos, pos + n),
// copy slot P to slot 0 if one of them filled slot P (Sec. 3.2, Fig. 2).
// Admission keeps n <= P, so at most one position of the batch lands there.
static hipError_t paper_fixup(df_graph *g, const Fifo &f, int64_t pos, int64_t n) {
  if (!f.period || !f.n_initial) return hipSuccess;
  if (host::fixup_position(pos, n, f.period) < 0) return hipSuccess;
  const size_t tb = (size_t)f.token_bytes;
  return hipMemcpyAsync(f.ring, f.ring + f.period * tb, tb, hipMemcpyDeviceToDevice, g->stream);
}

extern "C" df_status df_push(df_graph *g, int32_t fifo, const void *src, int64_t n, int src_on_device) {
  ENTER(g);
  if (fifo < 0 || fifo >= (int)g->fifos.size()) return fail(g, DF_EINVAL, "bad fifo id %d", fifo);
  if (n < 0) return fail(g, DF_EINVAL, "negative token count");
  Fifo &f = g->fifos[fifo];
  if (f.writer >= 0) return fail(g, DF_ESTATE, "fifo %d is written by actor %d", fifo, f.writer);
  if (n == 0) return DF_OK;
  if (!src) return fail(g, DF_EINVAL, "null source");
  if (f.cap - (f.write_hi - f.read_h) < n)
    return fail(g, DF_EAGAIN, "fifo %d: %lld tokens do not fit (%lld free)", fifo, (long long)n,
                (long long)(f.cap - (f.write_hi - f.read_h)));
  if (f.reader >= 0 && f.reader_port == DF_DPD_CTRL && g->actors[f.reader].kind == DF_ACTOR_DPD &&
      !src_on_device) {
    const int32_t *v = (const int32_t *)src;
    const df_dpd_params &dp = g->actors[f.reader].dp;
    const int32_t hi = dp.control_mode == DF_CTRL_MASK ? (1 << dp.n_branches_max) - 1 : dp.n_branches_max;
    for (int64_t i = 0; i < n; ++i)
      if (v[i] < 0 || v[i] > hi)
        return fail(g, DF_EINVAL, "control token %d at %lld outside 0..%d", v[i], (long long)i, hi);
  }
  HIPCHK(g, ring_copy(g, f, f.write_hi, (void *)src, n, true, src_on_device != 0));
  HIPCHK(g, paper_fixup(g, f, f.write_hi, n));
  HIPCHK(g, launch_advance(f.idx + 1, n, g->err_dev, g->stream));
  f.write_lo += n;
  f.write_hi += n;
  if (!src_on_device) HIPCHK(g, hipStreamSynchronize(g->stream));
  return after_call(g, DF_OK);
}

extern "C" df_status df_pop(df_graph *g, int32_t fifo, void *dst, int64_t max_tokens, int dst_on_device,
                            int64_t *n_popped) {
  ENTER(g);
  if (n_popped) *n_popped = 0;
  if (fifo < 0 || fifo >= (int)g->fifos.size()) return fail(g, DF_EINVAL, "bad fifo id %d", fifo);
  if (max_tokens < 0) return fail(g, DF_EINVAL, "negative token count");
  Fifo &f = g->fifos[fifo];
  if (f.reader >= 0) return fail(g, DF_ESTATE, "fifo %d is read by actor %d", fifo, f.reader);
  if (f.write_lo != f.write_hi) {
    df_status st = refresh_fifo(g, f);
    if (st) return st;
  }
  const int64_t k = std::min(max_tokens, f.write_lo - f.read_h);
  if (k > 0) {
    if (!dst) return fail(g, DF_EINVAL, "null destination");
    HIPCHK(g, ring_copy(g, f, f.read_h, dst, k, false, dst_on_device != 0));
    HIPCHK(g, launch_advance(f.idx + 0, k, g->err_dev, g->stream));
    f.read_h += k;
    if (!dst_on_device) HIPCHK(g, hipStreamSynchronize(g->stream));
  }
  if (n_popped) *n_popped = k;
  return after_call(g, DF_OK);
}

// ------------------------------------------------------------------ firing

// Tokens available to the reader, refreshing a data-dependent producer's
// count from the device only when the guaranteed count is too small.
static df_status available(df_graph *g, Fifo &f, int64_t need, int64_t *avail) {
  *avail = f.write_lo - f.read_h;
  if (*avail < need && f.write_lo != f.write_hi) {
    df_status st = refresh_fifo(g, f);
    if (st) return st;
    *avail = f.write_lo - f.read_h;
  }
  return DF_OK;
}

static int64_t space_of(const Fifo &f) { return f.cap - (f.write_hi - f.read_h); }

static hipError_t grow(void **p, size_t bytes) {
  (void)hipFree(*p);
  *p = nullptr;
  return hipMalloc(p, bytes);
}

df_status dfh::ensure_dpd_scratch(df_graph *g, Actor &a, int64_t n) {
  if (n <= a.scratch_n) return DF_OK;
  HIPCHK(g, hipStreamSynchronize(g->stream));
  if (a.ahead >= 0) {                                // its results go with the old buffers
    HIPCHK(g, launch_fill_i32(a.scan[a.ahead].err, 0, 1, g->stream));
    a.ahead = -1;
  }
  const int64_t cap = std::max<int64_t>(next_pow2(n), 64);
  const int bm = a.dp.n_branches_max;
  if (grow((void **)&a.order, 2 * sizeof(int32_t) * cap) != hipSuccess ||
      grow((void **)&a.prev, sizeof(int64_t) * bm * cap) != hipSuccess ||
      grow((void **)&a.off, sizeof(int64_t) * bm * cap) != hipSuccess ||
      grow((void **)&a.corr, sizeof(float2) * std::max(a.dp.n_taps - 1, 1) * cap) != hipSuccess)
    return fail(g, DF_ENOMEM, "scratch allocation failed");
  for (auto &sl : a.scan) {
    if (grow((void **)&sl.B, sizeof(int32_t) * cap) != hipSuccess ||
        grow(&sl.grp, scan_scratch_bytes(1, cap, bm, true)) != hipSuccess)
      return fail(g, DF_ENOMEM, "scratch allocation failed");
    ScanArgs sa{};                                   // the scan's ticket starts at zero
    sa.n_segs = 1;
    sa.seg_firings = cap;
    sa.B_max = bm;
    scan_scratch_assign(sa, sl.grp, true);
    HIPCHK(g, launch_fill_i32(sa.ticket, 0, 1, g->stream));
  }
  a.scratch_n = cap;
  return DF_OK;
}

df_status dfh::dpd_admit(df_graph *g, Actor &a, int64_t n, int64_t *n_adm) {
  if (a.ports[DF_DPD_CTRL] < 0 || a.ports[DF_DPD_IN] < 0 || a.ports[DF_DPD_OUT] < 0)
    return fail(g, DF_ESTATE, "predistortion actor has unconnected ports");
  Fifo &fc = g->fifos[a.ports[DF_DPD_CTRL]];
  Fifo &fx = g->fifos[a.ports[DF_DPD_IN]];
  Fifo &fy = g->fifos[a.ports[DF_DPD_OUT]];
  const int64_t r = a.dp.firing_size;
  int64_t ac, ax;
  df_status st = available(g, fc, n, &ac);
  if (st) return st;
  st = available(g, fx, n * r, &ax);
  if (st) return st;
  *n_adm = std::min({n, ac, ax / r, space_of(fy) / r});
  return DF_OK;
}

// Scan of the batch of n firings whose control tokens start at position
// pos, into slot sl (tickets at zero); errors to err.
static ScanArgs scan_args(df_graph *g, Actor &a, Actor::ScanSlot &sl, int64_t pos, int64_t n, bool ordered,
                          int32_t *err) {
  const Fifo &fc = g->fifos[a.ports[DF_DPD_CTRL]];
  ScanArgs sa{};
  sa.ctrl = (const int32_t *)fc.ring;
  sa.ctrl_idx = nullptr;                             // the host's read position is exact
  sa.ctrl_pos = pos;
  sa.ctrl_mask = fc.mask;
  sa.seg_firings = n;
  sa.n_segs = 1;
  sa.B_max = a.dp.n_branches_max;
  sa.hist_mode = a.dp.history_mode;
  sa.ctrl_mode = a.dp.control_mode;
  sa.B_out = sl.B;
  sa.prev_out = a.prev;
  sa.off_out = a.off;
  sa.last_out = sl.last;
  sa.stride = a.scratch_n;
  sa.r = a.dp.firing_size;
  sa.err = err;
  scan_scratch_assign(sa, sl.grp, ordered);
  return sa;
}

df_status dfh::dpd_enqueue(df_graph *g, Actor &a, int64_t n, bool may_run_ahead) {
  Fifo &fc = g->fifos[a.ports[DF_DPD_CTRL]];
  Fifo &fx = g->fifos[a.ports[DF_DPD_IN]];
  Fifo &fy = g->fifos[a.ports[DF_DPD_OUT]];
  const int64_t r = a.dp.firing_size;
  const int bm = a.dp.n_branches_max, M = a.dp.n_taps;
  // tiled bodies: the head pass fills the prev/off tables from the group
  // table, and places the firings in processing order (grouped by Horner
  // length: pays off only for many workgroups)
  const bool heads_tables = dpd_tiled_shape(M);
  const bool ordered = heads_tables && n > 64;
  const int64_t pos = fc.read_h;

  // this batch's scan: the one run ahead if it assumed this batch, else a new one
  int s = a.cur ^ 1;
  int32_t *err_ahead = nullptr;
  bool scanned = false;
  if (a.ahead >= 0) {
    s = a.ahead;
    Actor::ScanSlot &sl = a.scan[s];
    if (a.ahead_pos == pos && a.ahead_n == n) {
      err_ahead = sl.err;                            // the head pass merges and clears it
      scanned = true;
      dlog(g, 2, "scan run ahead for %lld firings at %lld used", (long long)n, (long long)pos);
    } else {
      HIPCHK(g, launch_fill_i32(sl.err, 0, 1, g->stream));
      dlog(g, 2, "scan run ahead for %lld firings at %lld discarded", (long long)a.ahead_n, (long long)a.ahead_pos);
    }
    a.ahead = -1;
  }
  Actor::ScanSlot &sl = a.scan[s];
  if (!scanned)
    HIPCHK(g, launch_scan(scan_args(g, a, sl, pos, n, ordered, g->err_dev), g->stream, !heads_tables, false));
  ScanArgs sa{};                                     // where the scan left its tables
  sa.n_segs = 1;
  sa.seg_firings = n;
  sa.B_max = bm;
  scan_scratch_assign(sa, sl.grp, ordered);

  DpdArgs da{};
  da.x = (const float2 *)fx.ring;
  da.x_idx = fx.idx;
  da.x_mask = fx.mask;
  da.y = (float2 *)fy.ring;
  da.y_idx = fy.idx;
  da.y_mask = fy.mask;
  da.h = a.h;
  da.hist = a.hist;
  da.B = sl.B;
  da.order = ordered ? a.order : nullptr;
  da.prev = a.prev;
  da.prev_stride = a.scratch_n;
  da.seg_firings = n;
  da.n_firings = n;
  da.r = r;
  da.B_max = bm;
  da.M = M;
  da.corr = a.corr;
  da.masked = a.dp.control_mode == DF_CTRL_MASK;
  da.mx = g->body_mx;
  da.err = g->err_dev;
  da.err_ahead = err_ahead;
  if (heads_tables) {
    da.grp = sa.grp;
    da.tab_prev = a.prev;
    da.tab_off = a.off;
    da.hist_mode = a.dp.history_mode;
    da.obase = sa.lgrp;
    da.order_out = ordered ? a.order : nullptr;
  }
  // The next batch's scan, if its control tokens are already in the channel
  // (pushed before this batch): run by extra workgroups of the head pass into
  // the other slot (whose last readers, the previous batch's kernels, are
  // done), beside this batch's head corrections.
  const bool run_ahead = may_run_ahead && !g->no_scan_ahead && heads_tables && n > 64 &&
                         fc.write_lo - (pos + n) >= n;
  if (run_ahead) {
    const int t = s ^ 1;
    da.ahead = scan_args(g, a, a.scan[t], pos + n, n, ordered, a.scan[t].err);
    da.ahead_blocks = (int32_t)((scan_groups(1, n) + 3) / 4);
  }
  HIPCHK(g, launch_dpd_heads(da, g->stream));
  DpdCommitArgs ca{};
  ca.x = (const float2 *)fx.ring;
  ca.x_idx = fx.idx;
  ca.x_mask = fx.mask;
  ca.ctrl_idx = fc.idx;
  ca.y_idx = fy.idx;
  ca.hist = a.hist;
  ca.last = sl.last;
  ca.n_firings = n;
  ca.r = r;
  ca.B_max = bm;
  ca.M = M;
  ca.err = g->err_dev;
  // the tiled body's last workgroup commits the batch; the generic body
  // leaves it to a kernel of its own
  const bool fused = dpd_tiled_shape(M);
  if (fused) {
    da.ticket = a.ticket;
    da.commit = ca;
  }
  KTiming kt;
  HIPCHK(g, prof_pair(g, &kt, (int)(&a - g->actors.data())));
  HIPCHK(g, launch_dpd_body(da, g->stream, g->tile, g->outputs_per_thread, g->prof ? &kt : nullptr));
  if (!fused) HIPCHK(g, launch_dpd_commit(ca, g->stream));

  fc.read_h += n;
  fx.read_h += n * r;
  fy.write_lo += n * r;
  fy.write_hi += n * r;
  a.last_n = n;
  a.fired += n;
  a.cur = s;

  if (run_ahead) {
    a.ahead = s ^ 1;
    a.ahead_pos = pos + n;
    a.ahead_n = n;
  }
  return DF_OK;
}

static df_status fire_dpd(df_graph *g, Actor &a, int64_t n, int flags, int64_t *n_fired) {
  int64_t adm;
  df_status st = dpd_admit(g, a, n, &adm);
  if (st) return st;
  if (adm < n && !(flags & DF_FIRE_PARTIAL))
    return fail(g, DF_EAGAIN, "only %lld of %lld firings admissible", (long long)adm, (long long)n);
  n = adm;
  if (n_fired) *n_fired = n;
  if (n == 0) return DF_OK;
  st = ensure_dpd_scratch(g, a, n);
  if (st) return st;
  return dpd_enqueue(g, a, n, true);
}

static df_status fire_motion(df_graph *g, Actor &a, int64_t n, int flags, int64_t *n_fired) {
  const df_motion_params &p = a.mp;
  if (a.ports[DF_MD_CUR] < 0 || a.ports[DF_MD_MASK] < 0 || a.ports[DF_MD_INDEX] < 0 ||
      (!p.self_delay && a.ports[DF_MD_PREV] < 0))
    return fail(g, DF_ESTATE, "motion actor has unconnected ports");
  Fifo &fc = g->fifos[a.ports[DF_MD_CUR]];
  Fifo *fp = p.self_delay ? nullptr : &g->fifos[a.ports[DF_MD_PREV]];
  Fifo &fm = g->fifos[a.ports[DF_MD_MASK]];
  Fifo &fi = g->fifos[a.ports[DF_MD_INDEX]];
  int64_t ac, ap = n;
  df_status st = available(g, fc, n, &ac);
  if (st) return st;
  if (fp && (st = available(g, *fp, n, &ap))) return st;
  const int64_t adm = std::min({n, ac, ap, space_of(fm), space_of(fi)});
  if (adm < n && !(flags & DF_FIRE_PARTIAL))
    return fail(g, DF_EAGAIN, "only %lld of %lld firings admissible", (long long)adm, (long long)n);
  n = adm;
  if (n_fired) *n_fired = n;
  if (n == 0) return DF_OK;
  const int64_t wh = (int64_t)p.width * p.height;
  const int32_t wpr = (p.width + 31) / 32;
  const int64_t frame_bits = (int64_t)wpr * p.height * 4;
  // firings per chunk: grid limit of one launch, and <= 512 MiB of staged bits
  const int64_t chunk_max = std::max<int64_t>(1, std::min<int64_t>(65535, (512ll << 20) / frame_bits));
  const int64_t want = std::min(n, chunk_max);
  if (want > a.cnt_cap) {
    HIPCHK(g, hipStreamSynchronize(g->stream));
    const int64_t cap = std::min(next_pow2(want), chunk_max);
    if (grow((void **)&a.count, sizeof(int32_t) * cap) != hipSuccess ||
        grow((void **)&a.emit_off, sizeof(int64_t) * (cap + 1)) != hipSuccess ||
        grow((void **)&a.bits, (size_t)(frame_bits * cap)) != hipSuccess)
      return fail(g, DF_ENOMEM, "scratch allocation failed");
    a.cnt_cap = cap;
    // counts start at zero; every emit pass leaves the ones it used at zero
    HIPCHK(g, launch_fill_i32(a.count, 0, cap, g->stream));
  }
  for (int64_t done = 0; done < n; done += chunk_max) {
    const int64_t k = std::min(chunk_max, n - done);
    MotionArgs ma{};
    ma.cur = (const uint8_t *)fc.ring;
    ma.cur_idx = fc.idx;
    ma.cur_mask = fc.mask;
    ma.prev = fp ? (const uint8_t *)fp->ring : nullptr;
    ma.prev_idx = fp ? fp->idx : nullptr;
    ma.prev_mask = fp ? fp->mask : 0;
    ma.state = a.state;
    ma.out = (uint8_t *)fm.ring;
    ma.out_idx = fm.idx;
    ma.out_mask = fm.mask;
    ma.index_out = (int64_t *)fi.ring;
    ma.index_idx = fi.idx;
    ma.index_mask = fi.mask;
    ma.count = a.count;
    ma.emit_off = a.emit_off;
    ma.bits = a.bits;
    ma.words_per_row = wpr;
    ma.n = k;
    ma.frame_base = a.fired;
    ma.W = p.width;
    ma.H = p.height;
    ma.thr = p.diff_threshold;
    ma.permille = p.min_changed_permille;
    // the batch's last input frame becomes the self-delay state: copied by
    // the emit pass when the frame is whole 16-byte words per 32-pixel word
    const bool fast = (p.width % 32) == 0 && wh % 16 == 0;
    const uint8_t *last_frame = p.self_delay ? (const uint8_t *)fc.ring + ((fc.read_h + k - 1) & fc.mask) * wh : nullptr;
    ma.state_src = fast ? last_frame : nullptr;
    HIPCHK(g, prof_begin(g, (int)(&a - g->actors.data())));
    HIPCHK(g, launch_motion_count(ma, g->stream));
    HIPCHK(g, launch_motion_emit_scan(a.count, k, (int64_t)p.min_changed_permille * wh, a.emit_off, g->stream));
    HIPCHK(g, launch_motion_emit(ma, g->stream));
    HIPCHK(g, prof_end(g));
    if (last_frame && !fast)
      HIPCHK(g, hipMemcpyAsync(a.state, last_frame, (size_t)wh, hipMemcpyDeviceToDevice, g->stream));
    HIPCHK(g, launch_motion_commit(a.emit_off, k, fc.idx, fp ? fp->idx : nullptr, fm.idx, fi.idx, g->err_dev, g->stream));
    fc.read_h += k;
    if (fp) fp->read_h += k;
    fm.write_hi += k;
    fi.write_hi += k;
    a.fired += k;
  }
  a.last_n = n;
  return DF_OK;
}

// Gauss, Thres and Med: static actors, every port `rate` frames per firing
// (Sec. 4.1).  Ports: inputs first, then outputs; Gauss's second output is
// optional.
static df_status fire_frames(df_graph *g, Actor &a, int64_t n, int flags, int64_t *n_fired) {
  const df_frame_params &p = a.fp;
  const int n_in = a.kind == DF_ACTOR_THRES ? 2 : 1;
  const int n_out = a.kind == DF_ACTOR_GAUSS5 ? 2 : 1;
  for (int i = 0; i < n_in + 1; ++i)
    if (a.ports[i] < 0) return fail(g, DF_ESTATE, "frame actor has unconnected ports");
  Fifo *in[2] = {nullptr, nullptr}, *out[2] = {nullptr, nullptr};
  for (int i = 0; i < n_in; ++i) in[i] = &g->fifos[a.ports[i]];
  for (int i = 0; i < n_out; ++i)
    if (a.ports[n_in + i] >= 0) out[i] = &g->fifos[a.ports[n_in + i]];
  const int64_t r = p.rate;
  int64_t adm = n;
  for (int i = 0; i < n_in; ++i) {
    int64_t av;
    df_status st = available(g, *in[i], n * r, &av);
    if (st) return st;
    adm = std::min(adm, av / r);
  }
  for (int i = 0; i < n_out; ++i)
    if (out[i]) adm = std::min(adm, space_of(*out[i]) / r);
  if (adm < n && !(flags & DF_FIRE_PARTIAL))
    return fail(g, DF_EAGAIN, "only %lld of %lld firings admissible", (long long)adm, (long long)n);
  n = adm;
  if (n_fired) *n_fired = n;
  if (n == 0) return DF_OK;
  const int64_t k = n * r;
  MdpArgs ma{};
  ma.in0 = (const uint8_t *)in[0]->ring;
  ma.in0_idx = in[0]->idx;
  ma.in0_mask = chan_map(*in[0]);
  if (in[1]) {
    ma.in1 = (const uint8_t *)in[1]->ring;
    ma.in1_idx = in[1]->idx;
    ma.in1_mask = chan_map(*in[1]);
  }
  ma.out0 = (uint8_t *)out[0]->ring;
  ma.out0_idx = out[0]->idx;
  ma.out0_mask = chan_map(*out[0]);
  if (out[1]) {
    ma.out1 = (uint8_t *)out[1]->ring;
    ma.out1_idx = out[1]->idx;
    ma.out1_mask = chan_map(*out[1]);
  }
  ma.W = p.width;
  ma.H = p.height;
  ma.thr = p.threshold;
  ma.n_frames = k;
  KTiming kt;
  HIPCHK(g, prof_pair(g, &kt, (int)(&a - g->actors.data())));
  const KTiming *tp = g->prof ? &kt : nullptr;
  if (a.kind == DF_ACTOR_GAUSS5)
    HIPCHK(g, launch_gauss5(ma, g->stream, tp));
  else if (a.kind == DF_ACTOR_THRES)
    HIPCHK(g, launch_thres(ma, g->stream, tp));
  else
    HIPCHK(g, launch_med5(ma, g->stream, tp));
  for (int i = 0; i < n_out; ++i)
    if (out[i]) HIPCHK(g, paper_fixup(g, *out[i], out[i]->write_hi, k));
  int64_t *ctr[4];
  int nc = 0;
  for (int i = 0; i < n_in; ++i) ctr[nc++] = in[i]->idx + 0;
  for (int i = 0; i < n_out; ++i)
    if (out[i]) ctr[nc++] = out[i]->idx + 1;
  HIPCHK(g, launch_advance_n(ctr, nc, k, g->err_dev, g->stream));
  for (int i = 0; i < n_in; ++i) in[i]->read_h += k;
  for (int i = 0; i < n_out; ++i)
    if (out[i]) {
      out[i]->write_lo += k;
      out[i]->write_hi += k;
    }
  a.fired += n;
  a.last_n = n;
  return DF_OK;
}

static df_status fire_pipeline(df_graph *g, int32_t gauss, int32_t thres, int32_t med, int64_t n, int flags,
                               int64_t *n_fired) {
  ENTER(g);
  if (n_fired) *n_fired = 0;
  const int na = (int)g->actors.size();
  if (gauss < 0 || gauss >= na || thres < 0 || thres >= na || med < 0 || med >= na)
    return fail(g, DF_EINVAL, "bad actor id");
  if (n < 0) return fail(g, DF_EINVAL, "negative firing count");
  if (flags & ~(DF_FIRE_PARTIAL | DF_PIPE_SEPARATE)) return fail(g, DF_EINVAL, "bad flags 0x%x", flags);
  Actor &ga = g->actors[gauss], &ta = g->actors[thres], &ma = g->actors[med];
  if (ga.kind != DF_ACTOR_GAUSS5 || ta.kind != DF_ACTOR_THRES || ma.kind != DF_ACTOR_MED5)
    return fail(g, DF_EINVAL, "df_fire_pipeline takes a Gauss, a Thres and a Med actor");
  const int p_in = ga.ports[DF_GAUSS_IN], p_cur = ga.ports[DF_GAUSS_OUT], p_del = ga.ports[DF_GAUSS_OUT2];
  const int p_thr = ta.ports[DF_THRES_OUT], p_out = ma.ports[DF_MED_OUT];
  if (p_in < 0 || p_cur < 0 || p_thr < 0 || p_out < 0 || ta.ports[DF_THRES_CUR] < 0 || ta.ports[DF_THRES_PREV] < 0 ||
      ma.ports[DF_MED_IN] < 0)
    return fail(g, DF_ESTATE, "pipeline actors have unconnected ports");
  if (ta.ports[DF_THRES_CUR] != p_cur || ma.ports[DF_MED_IN] != p_thr)
    return fail(g, DF_EINVAL, "actors are not chained Gauss -> Thres -> Med");
  const df_frame_params &gp = ga.fp, &tp = ta.fp, &mp = ma.fp;
  if (gp.width != tp.width || gp.width != mp.width || gp.height != tp.height || gp.height != mp.height ||
      gp.rate != tp.rate || gp.rate != mp.rate)
    return fail(g, DF_EINVAL, "pipeline actors differ in frame size or rate");
  const int64_t r = gp.rate;
  // admission of the three firings in sequence: each inner channel receives
  // its batch before it is read, so only the input and the free space count
  Fifo &fin = g->fifos[p_in], &fcur = g->fifos[p_cur], &fthr = g->fifos[p_thr], &fout = g->fifos[p_out];
  Fifo *fdel = p_del >= 0 ? &g->fifos[p_del] : nullptr;
  int64_t av;
  df_status st = available(g, fin, n * r, &av);
  if (st) return st;
  int64_t adm = std::min({n, av / r, space_of(fcur) / r, space_of(fthr) / r, space_of(fout) / r});
  if (fdel) adm = std::min(adm, space_of(*fdel) / r);
  const int p_prev = ta.ports[DF_THRES_PREV];
  if (p_prev != p_del) {
    // Thres's previous-frame channel is not fed by this Gauss: its tokens
    // must already be there
    int64_t ap;
    st = available(g, g->fifos[p_prev], n * r, &ap);
    if (st) return st;
    adm = std::min(adm, ap / r);
  }
  if (adm < n && !(flags & DF_FIRE_PARTIAL))
    return fail(g, DF_EAGAIN, "only %lld of %lld firings admissible", (long long)adm, (long long)n);
  n = adm;
  if (n_fired) *n_fired = n;
  if (n == 0) return DF_OK;
  const bool fused = !(flags & DF_PIPE_SEPARATE) && fdel && p_prev == p_del &&
                     mdp_fused_supported(gp.width, gp.height) && fcur.write_lo == fcur.write_hi &&
                     fcur.write_lo == fcur.read_h && fthr.write_lo == fthr.write_hi && fthr.write_lo == fthr.read_h &&
                     fdel->write_lo == fdel->write_hi && fdel->write_lo - fdel->read_h == 1;
  if (!fused) {
    for (Actor *a : {&ga, &ta, &ma}) {
      int64_t k = 0;
      st = fire_frames(g, *a, n, 0, &k);
      if (st) return st;
    }
    return DF_OK;
  }
  const int64_t k = n * r;
  MdpFusedArgs fa{};
  fa.in = (const uint8_t *)fin.ring;
  fa.in_idx = fin.idx;
  fa.in_mask = chan_map(fin);
  fa.delay = (uint8_t *)fdel->ring;
  fa.delay_idx = fdel->idx;
  fa.delay_mask = chan_map(*fdel);
  fa.out = (uint8_t *)fout.ring;
  fa.out_idx = fout.idx;
  fa.out_mask = chan_map(fout);
  fa.W = gp.width;
  fa.H = gp.height;
  fa.thr = tp.threshold;
  fa.n_frames = k;
  KTiming kt;
  HIPCHK(g, prof_pair(g, &kt, gauss));
  HIPCHK(g, launch_mdp_fused(fa, g->stream, g->prof ? &kt : nullptr));
  // the one token the delay channel keeps is written at position write + k - 1
  HIPCHK(g, paper_fixup(g, *fdel, fdel->write_hi + k - 1, 1));
  HIPCHK(g, paper_fixup(g, fout, fout.write_hi, k));
  int64_t *ctr[8] = {fin.idx + 0, fcur.idx + 0, fcur.idx + 1, fdel->idx + 0, fdel->idx + 1,
                     fthr.idx + 0, fthr.idx + 1, fout.idx + 1};
  HIPCHK(g, launch_advance_n(ctr, 8, k, g->err_dev, g->stream));
  fin.read_h += k;
  for (Fifo *f : {&fcur, fdel, &fthr}) {
    f->read_h += k;
    f->write_lo += k;
    f->write_hi += k;
  }
  fout.write_lo += k;
  fout.write_hi += k;
  for (Actor *a : {&ga, &ta, &ma}) {
    a->fired += n;
    a->last_n = n;
  }
  return DF_OK;
}

extern "C" df_status df_fire_pipeline(df_graph *g, int32_t gauss, int32_t thres, int32_t med, int64_t n, int flags,
                                      int64_t *n_fired) {
  df_status st = fire_pipeline(g, gauss, thres, med, n, flags, n_fired);
  if (st == DF_OK) dlog(g, 1, "df_fire_pipeline %d -> %d -> %d n %lld", gauss, thres, med, (long long)n);
  return g && !g->poisoned ? after_call(g, st) : st;
}

extern "C" df_status df_fire(df_graph *g, int32_t actor, int64_t n, int flags, int64_t *n_fired) {
  ENTER(g);
  if (n_fired) *n_fired = 0;
  if (actor < 0 || actor >= (int)g->actors.size()) return fail(g, DF_EINVAL, "bad actor id %d", actor);
  if (n < 0) return fail(g, DF_EINVAL, "negative firing count");
  if (flags & ~DF_FIRE_PARTIAL) return fail(g, DF_EINVAL, "bad flags 0x%x", flags);
  Actor &a = g->actors[actor];
  dlog(g, 1, "df_fire actor %d kind %d n %lld flags 0x%x", actor, (int)a.kind, (long long)n, flags);
  if (a.kind == DF_ACTOR_DPD) return after_call(g, fire_dpd(g, a, n, flags, n_fired));
  if (a.kind == DF_ACTOR_MOTION) return after_call(g, fire_motion(g, a, n, flags, n_fired));
  return after_call(g, fire_frames(g, a, n, flags, n_fired));
}

// Host-to-host streaming through one predistortion actor with the three
// transfers overlapped: batch k's input copy (stream copy_in), batch k-1's
// firing (graph stream) and batch k-2's output copy (stream copy_out) run
// at once.  Events order every ring region between its writer and readers:
// an input copy waits for the firing that last read the slots it fills, a
// firing waits for its input copy and for the output copy that last drained
// the slots it writes, an output copy waits for its firing.
extern "C" df_status df_stream_dpd(df_graph *g, int32_t actor, const void *x_host, const int32_t *ctrl_host,
                                   void *y_host, int64_t n_batches, int64_t firings_per_batch) {
  ENTER(g);
  if (actor < 0 || actor >= (int)g->actors.size()) return fail(g, DF_EINVAL, "bad actor id %d", actor);
  Actor &a = g->actors[actor];
  if (a.kind != DF_ACTOR_DPD) return fail(g, DF_EINVAL, "not a predistortion actor");
  if (n_batches < 0 || firings_per_batch < 1) return fail(g, DF_EINVAL, "bad batch counts");
  if (a.ports[DF_DPD_CTRL] < 0 || a.ports[DF_DPD_IN] < 0 || a.ports[DF_DPD_OUT] < 0)
    return fail(g, DF_ESTATE, "predistortion actor has unconnected ports");
  if (n_batches == 0) return DF_OK;
  if (!x_host || !ctrl_host || !y_host) return fail(g, DF_EINVAL, "null pointer");
  Fifo &fc = g->fifos[a.ports[DF_DPD_CTRL]];
  Fifo &fx = g->fifos[a.ports[DF_DPD_IN]];
  Fifo &fy = g->fifos[a.ports[DF_DPD_OUT]];
  if (fc.writer >= 0 || fx.writer >= 0 || fy.reader >= 0)
    return fail(g, DF_ESTATE, "the actor's channels must be fed and drained by the host");
  if (fy.write_lo != fy.write_hi || fy.write_lo != fy.read_h || fc.write_hi != fc.read_h)
    return fail(g, DF_ESTATE, "output and control channels must be empty");
  const int64_t nb = firings_per_batch, ns = nb * a.dp.firing_size;
  if (fx.cap < 2 * ns + (fx.write_hi - fx.read_h) || fc.cap < 2 * nb || fy.cap < 2 * ns)
    return fail(g, DF_EINVAL, "channels must hold two batches (plus pending input tokens)");
  df_status st = ensure_dpd_scratch(g, a, nb);
  if (st) return st;
  if (!g->copy_in) HIPCHK(g, hipStreamCreateWithFlags(&g->copy_in, hipStreamNonBlocking));
  if (!g->copy_out) HIPCHK(g, hipStreamCreateWithFlags(&g->copy_out, hipStreamNonBlocking));
  std::vector<hipEvent_t> ev_in(n_batches), ev_fired(n_batches), ev_out(n_batches);
  for (int64_t k = 0; k < n_batches; ++k) {
    HIPCHK(g, hipEventCreateWithFlags(&ev_in[k], hipEventDisableTiming));
    HIPCHK(g, hipEventCreateWithFlags(&ev_fired[k], hipEventDisableTiming));
    HIPCHK(g, hipEventCreateWithFlags(&ev_out[k], hipEventDisableTiming));
  }
  hipEvent_t start;
  HIPCHK(g, hipEventCreateWithFlags(&start, hipEventDisableTiming));
  HIPCHK(g, hipEventRecord(start, g->stream));       // earlier work on the graph
  HIPCHK(g, hipStreamWaitEvent(g->copy_in, start, 0));
  HIPCHK(g, hipStreamWaitEvent(g->copy_out, start, 0));
  const int64_t x_read0 = fx.read_h, x_write0 = fx.write_hi, y0 = fy.write_hi;
  const char *xh = (const char *)x_host;
  const char *ch = (const char *)ctrl_host;
  char *yh = (char *)y_host;
  // the batch whose slots a write of positions up to `last` reuses: the one
  // holding position last - cap, if any (batches start at `base`, n apart)
  const auto reused = host::reused_batch;
  // The copy streams carry copies only; every counter update runs on the
  // graph stream, after the copy it accounts for (a kernel on a copy stream
  // would share a hardware queue with the firings and serialise them).
  int64_t y_drained = 0;          // batches whose output-copy has been accounted on the graph stream
  for (int64_t k = 0; k < n_batches; ++k) {
    // input: control tokens and samples of batch k
    int64_t j = std::max(reused(x_write0 + (k + 1) * ns - 1, fx.cap, x_read0, ns),
                         reused(fc.write_hi + nb - 1, fc.cap, fc.read_h - k * nb, nb));
    if (j >= k) return fail(g, DF_EINVAL, "channel too small for two batches");
    if (j >= 0) HIPCHK(g, hipStreamWaitEvent(g->copy_in, ev_fired[j], 0));
    HIPCHK(g, ring_copy(g, fc, fc.write_hi, (void *)(ch + k * nb * sizeof(int32_t)), nb, true, false, g->copy_in));
    HIPCHK(g, ring_copy(g, fx, fx.write_hi, (void *)(xh + k * ns * fx.token_bytes), ns, true, false, g->copy_in));
    HIPCHK(g, hipEventRecord(ev_in[k], g->copy_in));
    fc.write_lo += nb;
    fc.write_hi += nb;
    fx.write_lo += ns;
    fx.write_hi += ns;
    // firing of batch k, after its input copy (then the write counters move)
    // and after the output copy that last drained the slots it writes
    HIPCHK(g, hipStreamWaitEvent(g->stream, ev_in[k], 0));
    j = reused(y0 + (k + 1) * ns - 1, fy.cap, y0, ns);
    if (j >= k) return fail(g, DF_EINVAL, "channel too small for two batches");
    int64_t *ctr[3] = {fc.idx + 1, fx.idx + 1, fy.idx + 0};
    const int64_t delta[3] = {nb, ns, ns};
    int nc = 2;
    if (j >= 0) {
      HIPCHK(g, hipStreamWaitEvent(g->stream, ev_out[j], 0));
      if (j >= y_drained) {       // batches up to j are drained: move y's read counter
        nc = 3;
        ctr[2] = fy.idx + 0;
        const int64_t d = (j + 1 - y_drained) * ns;
        const int64_t deltas[3] = {nb, ns, d};
        HIPCHK(g, launch_advance_by(ctr, deltas, nc, g->err_dev, g->stream));
        y_drained = j + 1;
      } else {
        HIPCHK(g, launch_advance_by(ctr, delta, nc, g->err_dev, g->stream));
      }
    } else {
      HIPCHK(g, launch_advance_by(ctr, delta, nc, g->err_dev, g->stream));
    }
    st = dpd_enqueue(g, a, nb, false);
    if (st) return st;
    HIPCHK(g, hipEventRecord(ev_fired[k], g->stream));
    // output of batch k
    HIPCHK(g, hipStreamWaitEvent(g->copy_out, ev_fired[k], 0));
    HIPCHK(g, ring_copy(g, fy, fy.read_h, (void *)(yh + k * ns * fy.token_bytes), ns, false, false, g->copy_out));
    HIPCHK(g, hipEventRecord(ev_out[k], g->copy_out));
    fy.read_h += ns;
  }
  HIPCHK(g, hipStreamWaitEvent(g->stream, ev_in[n_batches - 1], 0));
  HIPCHK(g, hipStreamWaitEvent(g->stream, ev_out[n_batches - 1], 0));
  if (y_drained < n_batches) {
    int64_t *ctr[1] = {fy.idx + 0};
    const int64_t d[1] = {(n_batches - y_drained) * ns};
    HIPCHK(g, launch_advance_by(ctr, d, 1, g->err_dev, g->stream));
  }
  HIPCHK(g, hipStreamSynchronize(g->stream));
  for (int64_t k = 0; k < n_batches; ++k) {
    (void)hipEventDestroy(ev_in[k]);
    (void)hipEventDestroy(ev_fired[k]);
    (void)hipEventDestroy(ev_out[k]);
  }
  (void)hipEventDestroy(start);
  return after_call(g, DF_OK);
}

extern "C" df_status df_set_tile(df_graph *g, int32_t tile_outputs, int32_t outputs_per_thread,
                                 int32_t blocks_per_cu) {
  ENTER(g);
  if (outputs_per_thread != 0 && outputs_per_thread != 4 && outputs_per_thread != 8)
    return fail(g, DF_EINVAL, "outputs_per_thread must be 4 or 8");
  const int k = outputs_per_thread ? outputs_per_thread : g->outputs_per_thread;
  if (tile_outputs != 0 && (tile_outputs < 64 * k || tile_outputs > 512 * k || tile_outputs % (64 * k)))
    return fail(g, DF_EINVAL, "tile_outputs must be a multiple of %d in %d..%d", 64 * k, 64 * k, 512 * k);
  if (blocks_per_cu < 0 || blocks_per_cu > 16) return fail(g, DF_EINVAL, "blocks_per_cu outside 0..16");
  if (outputs_per_thread) g->outputs_per_thread = outputs_per_thread;
  if (tile_outputs) g->tile = tile_outputs;
  if (blocks_per_cu) g->blocks_per_cu = blocks_per_cu;
  return DF_OK;
}

extern "C" df_status df_debug_read_slots(df_graph *g, int32_t fifo, void *dst, int64_t max_bytes) {
  ENTER(g);
  if (fifo < 0 || fifo >= (int)g->fifos.size()) return fail(g, DF_EINVAL, "bad fifo id %d", fifo);
  const Fifo &f = g->fifos[fifo];
  const int64_t bytes = f.slots * f.token_bytes;
  if (!dst || max_bytes < bytes) return fail(g, DF_EINVAL, "destination holds fewer than %lld bytes", (long long)bytes);
  HIPCHK(g, hipStreamSynchronize(g->stream));
  HIPCHK(g, hipMemcpy(dst, f.ring, (size_t)bytes, hipMemcpyDeviceToHost));
  return DF_OK;
}

extern "C" df_status df_debug_set_counters(df_graph *g, int32_t fifo, int64_t read_idx, int64_t write_idx) {
  ENTER(g);
  if (fifo < 0 || fifo >= (int)g->fifos.size()) return fail(g, DF_EINVAL, "bad fifo id %d", fifo);
  Fifo &f = g->fifos[fifo];
  const int64_t v[2] = {read_idx, write_idx};
  HIPCHK(g, hipMemcpyAsync(f.idx, v, sizeof v, hipMemcpyHostToDevice, g->stream));
  HIPCHK(g, hipStreamSynchronize(g->stream));
  return DF_OK;
}

extern "C" df_status df_debug_last_batch(df_graph *g, int32_t actor, int32_t *rates, int64_t *offsets,
                                         int64_t *prev, int64_t cap, int64_t *n_out) {
  ENTER(g);
  if (actor < 0 || actor >= (int)g->actors.size()) return fail(g, DF_EINVAL, "bad actor id %d", actor);
  Actor &a = g->actors[actor];
  if (a.kind != DF_ACTOR_DPD) return fail(g, DF_EINVAL, "not a predistortion actor");
  const int64_t n = a.last_n;
  if (n_out) *n_out = n;
  if (n > cap) return fail(g, DF_EINVAL, "cap %lld < batch size %lld", (long long)cap, (long long)n);
  HIPCHK(g, hipStreamSynchronize(g->stream));
  const int bm = a.dp.n_branches_max;
  if (n == 0) return DF_OK;
  if (rates) {
    std::vector<int32_t> B(n);
    HIPCHK(g, hipMemcpy(B.data(), a.scan[a.cur].B, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    for (int b = 0; b < bm; ++b)
      for (int64_t j = 0; j < n; ++j) rates[b * cap + j] = in_set((uint32_t)B[j], b) ? (int32_t)a.dp.firing_size : 0;
  }
  for (int b = 0; b < bm; ++b) {
    if (offsets)
      HIPCHK(g, hipMemcpy(offsets + b * cap, a.off + b * a.scratch_n, sizeof(int64_t) * n, hipMemcpyDeviceToHost));
    if (prev)
      HIPCHK(g, hipMemcpy(prev + b * cap, a.prev + b * a.scratch_n, sizeof(int64_t) * n, hipMemcpyDeviceToHost));
  }
  return DF_OK;
}

// ------------------------------------------------------------------ profiling

static hipError_t take_event(df_graph *g, hipEvent_t *ev) {
  if (!g->prof_pool.empty()) {
    *ev = g->prof_pool.back();
    g->prof_pool.pop_back();
    return hipSuccess;
  }
  // timing-only events: no system-scope fence on record (df_profile_read
  // synchronizes the stream before reading them)
  return hipEventCreateWithFlags(ev, hipEventDisableSystemFence);
}

hipError_t dfh::prof_pair(df_graph *g, KTiming *t, int actor) {
  if (!g->prof) return hipSuccess;
  hipError_t e = take_event(g, &t->start);
  if (e == hipSuccess) e = take_event(g, &t->stop);
  if (e != hipSuccess) return e;
  g->prof_pending.push_back({t->start, t->stop, actor});
  return hipSuccess;
}

hipError_t dfh::prof_begin(df_graph *g, int actor) {
  if (!g->prof) return hipSuccess;
  hipEvent_t a, b;
  hipError_t e = take_event(g, &a);
  if (e == hipSuccess) e = take_event(g, &b);
  if (e != hipSuccess) return e;
  g->prof_pending.push_back({a, b, actor});
  return hipEventRecord(a, g->stream);
}

hipError_t dfh::prof_end(df_graph *g) {
  if (!g->prof || g->prof_pending.empty()) return hipSuccess;
  return hipEventRecord(g->prof_pending.back().stop, g->stream);
}

extern "C" df_status df_profile_enable(df_graph *g, int32_t enable) {
  ENTER(g);
  g->prof = enable != 0;
  return DF_OK;
}

// Sum and release the pending timings of `actor` (all of them when all_actors).
static df_status read_timings(df_graph *g, bool all_actors, int actor, double *total_ms, int64_t *n_launches) {
  HIPCHK(g, hipStreamSynchronize(g->stream));
  double t = 0.0;
  int64_t n = 0;
  std::vector<df_graph::ProfEntry> keep;
  for (auto &pe : g->prof_pending) {
    if (!all_actors && pe.actor != actor) {
      keep.push_back(pe);
      continue;
    }
    float ms = 0.f;
    HIPCHK(g, hipEventElapsedTime(&ms, pe.start, pe.stop));
    t += ms;
    ++n;
    g->prof_pool.push_back(pe.start);
    g->prof_pool.push_back(pe.stop);
  }
  if (total_ms) *total_ms = t;
  if (n_launches) *n_launches = n;
  g->prof_pending.swap(keep);
  return DF_OK;
}

extern "C" df_status df_profile_read(df_graph *g, double *total_ms, int64_t *n_launches) {
  ENTER(g);
  return read_timings(g, true, -1, total_ms, n_launches);
}

extern "C" df_status df_profile_read_actor(df_graph *g, int32_t actor, double *total_ms, int64_t *n_launches) {
  ENTER(g);
  if (actor < 0 || actor >= (int)g->actors.size()) return fail(g, DF_EINVAL, "bad actor id %d", actor);
  return read_timings(g, false, actor, total_ms, n_launches);
}
