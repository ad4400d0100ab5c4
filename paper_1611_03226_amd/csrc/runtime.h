// Host-side state of a network (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "common.h"
#include "dfhip.h"

namespace dfh {

constexpr int kMaxFifos = 16384;

// A FIFO channel as a device ring of `cap` tokens (power of two).  The
// device pair idx[0..1] = (read, write) token counters is authoritative;
// the host mirror read_h is exact (every reader has a statically known rate)
// and [write_lo, write_hi] brackets the write counter (equal unless the
// writer's production rate is data-dependent and not yet read back).
struct Fifo {
  df_dtype dt = DF_C64;
  int64_t elem_bytes = 0, elems_per_token = 0, token_bytes = 0;
  int64_t cap = 0, mask = 0;
  char *ring = nullptr;
  int64_t *idx = nullptr;
  int64_t read_h = 0, write_lo = 0, write_hi = 0;
  int64_t n_initial = 0;
  // the paper's layout (Sec. 3.2): period P (2r, or 3r with a delay token),
  // 0 for a ring; `slots` tokens are allocated (cap, or P + 1 with a delay)
  int64_t period = 0;
  int64_t slots = 0;
  int writer = -1, writer_port = -1;  // -1: the host
  int reader = -1, reader_port = -1;
};

// Slot map of a channel as the kernels take it (see read_slot / write_slot).
inline int64_t chan_map(const Fifo &f) {
  return f.period ? -(2 * f.period + (f.n_initial ? 1 : 0) + 2) : f.mask;
}

struct Actor {
  df_actor_kind kind = DF_ACTOR_DPD;
  int ports[4] = {-1, -1, -1, -1};
  int64_t fired = 0;     // firings so far
  int64_t last_n = 0;    // size of the last batch
  // predistortion
  df_dpd_params dp{};
  float2 *h = nullptr;       // [B_max][M]
  float2 *hist = nullptr;    // [B_max][M-1] carried branch histories
  int64_t scratch_n = 0;
  int32_t *order = nullptr;  // [scratch_n][2] (firing, branch set) grouped by Horner length
  float2 *corr = nullptr;    // [scratch_n][M-1] head corrections
  int64_t *prev = nullptr;   // [B_max][scratch_n]
  int64_t *off = nullptr;    // [B_max][scratch_n]
  int32_t *ticket = nullptr; // finished-workgroup counter of the body (commit by the last one)
  // Scan results of a batch, in two slots: the scan of the next batch (it
  // reads control tokens only) runs ahead, inside this batch's head pass,
  // and is used if the next batch starts where it assumed and has its size.
  struct ScanSlot {
    int32_t *B = nullptr;      // [scratch_n] validated branch sets
    void *grp = nullptr;       // scan scratch: ticket, group table, length table
    int64_t *last = nullptr;   // [B_max] last feeder of each branch
    int32_t *err = nullptr;    // control-token errors of a scan run ahead (merged when used)
  };
  ScanSlot scan[2];
  int cur = 0;                 // slot of the last batch
  int ahead = -1;              // slot holding a scan run ahead, or -1
  int64_t ahead_pos = 0, ahead_n = 0;
  // motion
  df_motion_params mp{};
  uint8_t *state = nullptr;  // previous frame (self-delay form)
  int32_t *count = nullptr;
  int64_t *emit_off = nullptr;
  uint32_t *bits = nullptr;  // bit-packed opened masks of a chunk of firings
  int64_t cnt_cap = 0;
  // Gauss / Thres / Med
  df_frame_params fp{};
};

struct Persistent;  // multi-instance batching state

}  // namespace dfh

struct df_graph {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t copy_in = nullptr, copy_out = nullptr;  // host transfers of df_stream_dpd (created on first use)
  bool no_scan_ahead = false;        // DFHIP_SCAN_AHEAD=0: no scan of the next batch in the head pass
  bool own_stream = false;
  bool poisoned = false;
  std::string last_error;
  std::vector<dfh::Fifo> fifos;
  std::vector<dfh::Actor> actors;
  int64_t *idx_pool = nullptr;   // device [kMaxFifos][kCtrWords] channel counter slots
  int32_t *err_dev = nullptr;    // sticky device error word
  int tile = 0;                  // 0 = default
  int outputs_per_thread = 4;
  bool body_mx = false;          // M = 16 bodies on the matrix cores (DFHIP_BODY=mx)
  int blocks_per_cu = 0;          // persistent grid; 0 = default
  dfh::Persistent *pers = nullptr;
  bool check_indices = false;    // DFHIP_CHECK_INDICES: every token-moving call syncs and reports device errors
  int log_level = 0;             // DFHIP_LOG: 1 = one line per firing call on stderr
  bool prof = false;                                   // record body-kernel events
  struct ProfEntry {
    hipEvent_t start, stop;
    int actor;  // -1: not one actor's launch (persistent batches)
  };
  std::vector<ProfEntry> prof_pending;
  std::vector<hipEvent_t> prof_pool;
};

namespace dfh {
df_status fail(df_graph *g, df_status st, const char *fmt, ...);
df_status fail_hip(df_graph *g, hipError_t e, const char *what);
df_status refresh_fifo(df_graph *g, Fifo &f);
// Synchronise and turn the sticky device error word into a status.
df_status sync_errors(df_graph *g);
// Result of a token-moving call: with DFHIP_CHECK_INDICES set, a successful
// call also synchronises and reports device errors.
df_status after_call(df_graph *g, df_status st);
// One diagnostic line on stderr when DFHIP_LOG >= level.
void dlog(const df_graph *g, int level, const char *fmt, ...);
df_status ensure_dpd_scratch(df_graph *g, Actor &a, int64_t n);
df_status dpd_admit(df_graph *g, Actor &a, int64_t n, int64_t *n_adm);
// One batch of n firings on the graph stream; with may_run_ahead, the head
// pass also scans the next batch of n firings (if its control tokens are in
// the channel).
df_status dpd_enqueue(df_graph *g, Actor &a, int64_t n, bool may_run_ahead);
void destroy_persistent(df_graph *g);

// Scratch of one stateless predistortion forward call: validated branch
// counts B [n], history sources prev [B_max][n], scan group table grp, head
// corrections corr [n][M-1] (n = S*len/r firings; without control tokens only
// corr, [S][M-1]).  Nothing in it needs to start at zero.
struct FwdScratch {
  int32_t *B = nullptr;
  int64_t *prev = nullptr;
  void *grp = nullptr;        // scan scratch (scan_scratch_bytes)
  float2 *corr = nullptr;
};
struct FwdScratchSize {
  size_t B = 0, prev = 0, grp = 0, corr = 0;
};
FwdScratchSize dpd_forward_scratch_size(int64_t S, int64_t len, int64_t r, int32_t B_max, int32_t M,
                                        bool with_ctrl);
hipError_t dpd_forward_enqueue(const FwdScratch &sc, hipStream_t s, const void *x, const int32_t *ctrl,
                               const void *h, void *y, int64_t S, int64_t len, int64_t r, int32_t B_max, int32_t M,
                               int32_t hist);
df_status check_dpd_forward_args(const void *x, const void *h, void *y, int64_t S, int64_t len, int64_t r,
                                 int32_t B_max, int32_t M, int32_t hist, bool *nothing);
// Event pair around body kernels when profiling is enabled (no-op otherwise).
hipError_t prof_begin(df_graph *g, int actor = -1);
// events for one timed launch of `actor` (none if profiling is off)
hipError_t prof_pair(df_graph *g, KTiming *t, int actor = -1);
hipError_t prof_end(df_graph *g);
}  // namespace dfh
