// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dfh {

constexpr int kMaxBranches = 16;
constexpr int kMaxTaps = 32;

// Sticky device error bits (an int32 in device memory per graph).
enum : int32_t { kErrControl = 1, kErrIndex = 2 };

// Channel counters: every channel owns one 32-byte-aligned slot of four
// int64 words in device memory, [0] read count, [1] write count,
// [2] capacity in tokens, [3] unused.  Kernels address the counters through
// a pointer to word 0 or word 1 of a slot.
constexpr int kCtrWords = 4;

__device__ __forceinline__ int64_t *chan_slot(int64_t *ctr) {
  return (int64_t *)((uintptr_t)ctr & ~(uintptr_t)(kCtrWords * sizeof(int64_t) - 1));
}

// Slot of token position p in a channel, from the channel's slot map m.
//   m >= 0: a ring of power-of-two capacity, m = capacity - 1 (m = -1: a
//           linear array, position = slot);
//   m <= -2: the paper's channel layout (Sec. 3.2, Eq. (1), Fig. 2) with
//           period P and d in {0, 1} delay tokens, m = -(2P + d + 2): P = 2r
//           slots (a double buffer) without a delay token; with one, 3r + 1
//           slots, P = 3r, the delay token in slot 0, writes filling slots
//           1..P in turn and reads taking slots 0..P-1 in turn (slot P is
//           copied to slot 0 after the write that fills it).
__device__ __host__ __forceinline__ int64_t read_slot(int64_t p, int64_t m) {
  if (m >= -1) return p & m;
  return p % ((-m - 2) >> 1);
}

__device__ __host__ __forceinline__ int64_t write_slot(int64_t p, int64_t m) {
  if (m >= -1) return p & m;
  const int64_t v = -m - 2, P = v >> 1;
  return (v & 1) ? 1 + (p - 1) % P : p % P;
}

// The ring invariant of a channel after a counter update: the reader never
// passes the writer, and the writer never runs more than a capacity ahead
// (read <= write <= read + capacity).  A violation sets the sticky kErrIndex.
__device__ __forceinline__ void check_chan(const int64_t *slot, int32_t *err) {
  const int64_t occ = slot[1] - slot[0];
  if ((occ < 0 || occ > slot[2]) && err) atomicOr(err, (int32_t)kErrIndex);
}

// ---------------------------------------------------------------- DPD
//
// Active branches of a firing as the kernels carry them: a bit set, bit b
// set when branch b runs (Sec. 4.2: the configuration selects which set of
// FIR filters takes part).  A count token B (the prefix reading) is the set
// {0, .., B-1}; a mask token is its own bits.  The Horner length of a set is
// its highest member + 1.
enum : int32_t { kCtrlCount = 0, kCtrlMask = 1 };

__device__ __host__ __forceinline__ uint32_t prefix_set(int B) { return B >= 32 ? ~0u : (1u << B) - 1u; }
__device__ __host__ __forceinline__ bool in_set(uint32_t s, int b) { return (s >> b) & 1u; }
__device__ __forceinline__ int set_len(uint32_t s) { return s ? 32 - __builtin_clz(s) : 0; }

// Validated branch set of control token v: count tokens 0..B_max, mask
// tokens 0..2^B_max - 1; anything else is the empty set and sets *bad.
__device__ __forceinline__ uint32_t token_set(int32_t v, int32_t mode, int32_t B_max, bool *bad) {
  const bool ok = mode == kCtrlMask ? (v >= 0 && v < (1 << B_max)) : (v >= 0 && v <= B_max);
  *bad = !ok;
  if (!ok) return 0u;
  return mode == kCtrlMask ? (uint32_t)v : prefix_set(v);
}
//
// One batch of predistortion firings.  Firing g (0 <= g < n_firings) reads
// r input samples starting at sample position xpos(g) and writes r output
// samples at ypos(g):
//   actor mode:      xpos(g) = R_x + g*r (ring, masked), ypos(g) = W_y + g*r
//   stateless mode:  xpos(g) = g*r, ypos(g) = g*r (rows of length
//                    seg_firings*r concatenated; no wrap: mask = -1)
// B[g] is the firing's validated branch set (nullptr: branches 0..B_const-1).
// prev[b*prev_stride + g] is the firing whose tail is branch b's FIR history
// (-1: carried state `hist` [b][M-1], nullptr history = zeros).  With
// prev == nullptr the history firing is g-1 inside its segment of
// seg_firings firings and -1 at a segment start.
// Batch commit of a single actor: advance the channel indices by the
// batch's token counts and carry each branch's history (the last M-1 input
// samples of its last feeding firing).
struct DpdCommitArgs {
  const float2 *x;
  int64_t *x_idx;
  int64_t x_mask;
  int64_t *ctrl_idx;
  int64_t *y_idx;
  float2 *hist;           // [B_max][M-1]
  const int64_t *last;    // [B_max]
  int64_t n_firings;
  int64_t r;
  int32_t B_max;
  int32_t M;
  int32_t *err;           // sticky error word (ring invariant), may be nullptr
};

// Control intake + offset scan over segments of firings (one wavefront per
// 64-firing group; the last group of a segment to finish scans the group
// tables of its segment).
struct ScanArgs {
  const int32_t *ctrl;    // control tokens (ring or linear)
  const int64_t *ctrl_idx;// device [read, write] or nullptr (position ctrl_pos)
  int64_t ctrl_pos;       // read position when ctrl_idx is nullptr
  int64_t ctrl_mask;      // ring mask, -1 for linear
  int64_t seg_firings;    // firings per segment (< 2^31)
  int32_t n_segs;
  int32_t B_max;
  int32_t hist_mode;      // 0 branch, 1 shared
  int32_t ctrl_mode;      // kCtrlCount or kCtrlMask
  int32_t *B_out;         // [n_segs*seg_firings] validated branch sets
  int64_t *prev_out;      // [B_max][stride]
  int64_t *off_out;       // [B_max][stride] (may be nullptr)
  int64_t *last_out;      // [n_segs][B_max] (may be nullptr)
  int64_t *grp;           // [scan_groups][B_max][2]: count and last feeder before each 64-firing group
  int32_t *lgrp;          // [scan_groups][B_max+1] (one segment) or nullptr: first processing slot of
                          // each Horner length in each group (firings grouped by length, longest first)
  int32_t *ticket;        // [n_segs] finished groups per segment; zero between scans
  int64_t stride;
  int64_t r;
  int32_t *err;           // sticky error word (may be nullptr)
};

struct DpdArgs {
  const float2 *x;
  const int64_t *x_idx;   // device [read, write] or nullptr (position 0)
  int64_t x_mask;
  float2 *y;
  const int64_t *y_idx;   // device [read, write] or nullptr
  int64_t y_mask;
  const float2 *h;        // [B_max][M]
  const float2 *hist;     // [B_max][M-1] or nullptr
  const int32_t *B;       // [n_firings] branch sets, or nullptr
  int32_t B_const;        // branch count of every firing when B is nullptr
  const int64_t *prev;    // [B_max][prev_stride] or nullptr
  int64_t prev_stride;
  int64_t seg_firings;
  int64_t n_firings;
  int64_t r;
  int32_t B_max;
  int32_t M;
  int32_t tile;           // outputs per workgroup (tiled kernel)
  int32_t tiles_per_firing;
  const int32_t *order;   // processing order, pairs (firing, branch set) grouped by Horner length, or nullptr
  float2 *corr;           // [n_firings][M-1] head corrections (tiled kernels)
  // With grp set (one segment), the head pass derives each firing's history
  // sources from the scan's group table and writes the prev/off tables itself.
  const int64_t *grp;     // [groups][B_max][2] from k_scan, or nullptr
  int64_t *tab_prev;      // [B_max][prev_stride]
  int64_t *tab_off;       // [B_max][prev_stride] or nullptr
  // ... and, with order_out, places each firing in the processing order from
  // the scan's length table
  const int32_t *obase;   // ScanArgs::lgrp
  int32_t *order_out;     // [n_firings][2] or nullptr
  int32_t hist_mode;
  int32_t masked;         // branch sets may be non-prefix (bit-mask control tokens)
  int32_t mx;             // M = 16 tiled body on the matrix cores (else the VALU form)
  int32_t *ticket;        // tiled kernel: the last workgroup to finish runs `commit` (nullptr: none)
  DpdCommitArgs commit;
  int32_t *err;           // sticky error word (head pass; may be nullptr)
  int32_t *err_ahead;     // errors of a scan run ahead of this batch: the head pass adds them to err
                          // and clears them (nullptr: none)
  // The head pass with tables can also run the scan of the next batch
  // (control tokens only): its first ahead_blocks workgroups do it.
  ScanArgs ahead;
  int32_t ahead_blocks;
};

// ---------------------------------------------------------------- motion
struct MotionArgs {
  const uint8_t *cur;     // ring of frames
  const int64_t *cur_idx;
  int64_t cur_mask;
  const uint8_t *prev;    // ring of frames (two-channel form) or nullptr
  const int64_t *prev_idx;
  int64_t prev_mask;
  uint8_t *state;         // previous frame (self-delay form)
  const uint8_t *state_src;  // the batch's last input frame, copied to state by the emit pass (or nullptr)
  uint8_t *out;           // mask ring
  const int64_t *out_idx;
  int64_t out_mask;
  int64_t *index_out;     // index ring
  const int64_t *index_idx;
  int64_t index_mask;
  int32_t *count;         // [n] opened-mask counts
  const int64_t *emit_off;// [n+1] exclusive scan of emit flags (emit pass)
  uint32_t *bits;         // bit-packed opened masks [n][H][W/32] (count pass)
  int64_t n;
  int64_t frame_base;     // global index of firing 0
  int32_t W, H, thr;
  int32_t permille;
  int32_t words_per_row;  // W/32 rounded up
};

// ---------------------------------------------------------------- adjoint
// Coefficient adjoint over firings laid out as in DpdArgs' stateless mode.
struct AdjArgs {
  const float2 *x;        // [n_firings * r]
  const float2 *G;        // [n_firings * r]
  const int32_t *B;       // [n_firings] branch sets, or nullptr (all B_max branches)
  const int64_t *prev;    // [B_max][prev_stride] or nullptr
  int64_t prev_stride;
  int64_t seg_firings;
  int64_t n_firings;
  int64_t r;
  int32_t B_max;
  int32_t M;
  int32_t chunk;          // outputs staged in LDS at a time (set by launch_adj)
  int32_t span;           // outputs per workgroup (chunks processed in turn)
  int32_t blocks_per_firing;
  float2 *partial;        // [B_max][M][n_firings*blocks_per_firing]
  float2 *grad;           // [B_max][M]
};

// Workgroups of `kernel` (threads, dynamic LDS bytes) resident on the whole
// current device at once (occupancy x compute units), cached per kernel shape.
int64_t resident_blocks(const void *kernel, int threads, size_t lds_bytes);

// ---------------------------------------------------------------- launchers
int64_t scan_groups(int64_t n_segs, int64_t seg_firings);   // 64-firing groups of a scan
// Scratch of one scan in bytes: segment tickets (int32 [n_segs]), group
// table (int64 [groups][B_max][2]), and for an ordered scan the length
// table (int32 [groups][B_max+1]); scan_scratch_assign points the ScanArgs
// fields into such a buffer (256-byte aligned regions, in that order).
size_t scan_scratch_bytes(int64_t n_segs, int64_t seg_firings, int32_t B_max, bool ordered);
void scan_scratch_assign(ScanArgs &a, void *scratch, bool ordered);
// tables: also write prev/off (else the head pass does); zero_tickets: clear
// the tickets first (a fill kernel) when the buffer is not known to be zero
hipError_t launch_scan(const ScanArgs &a, hipStream_t s, bool tables = true, bool zero_tickets = true);
// Optional start/stop events of one kernel launch (timing rides on the
// dispatch itself: hipExtLaunchKernel), or none.
struct KTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};

// One batch of a static frame actor of the motion-detection pipeline
// (Sec. 4.1): n_frames consecutive tokens of every port.  Frame f of the
// batch is slot read_slot(idx[0] + f, map) of an input channel (its read
// counter) and write_slot(idx[1] + f, map) of an output channel (its write
// counter); the *_mask fields hold each channel's slot map.
struct MdpArgs {
  const uint8_t *in0;    // Gauss / Med input, Thres current frame
  const int64_t *in0_idx;
  int64_t in0_mask;
  const uint8_t *in1;    // Thres previous frame
  const int64_t *in1_idx;
  int64_t in1_mask;
  uint8_t *out0;
  const int64_t *out0_idx;
  int64_t out0_mask;
  uint8_t *out1;         // Gauss second output or nullptr
  const int64_t *out1_idx;
  int64_t out1_mask;
  int32_t W, H;
  int32_t thr;
  int64_t n_frames;
};

// One fused batch of the chain Gauss -> Thres -> Med (n_frames frames):
// input frames from `in` (read counter), the previous Gauss frame of the
// batch's first frame from the delay channel's read slot, output frames to
// `out` (write counter), and the Gauss frame of the batch's last frame to the
// delay channel's slot write counter + n_frames - 1.
struct MdpFusedArgs {
  const uint8_t *in;
  const int64_t *in_idx;
  int64_t in_mask;
  uint8_t *delay;           // Gauss -> Thres delay channel
  const int64_t *delay_idx;
  int64_t delay_mask;
  uint8_t *out;
  const int64_t *out_idx;
  int64_t out_mask;
  int32_t W, H;
  int32_t thr;
  int64_t n_frames;
};
// The fused form needs W % 4 == 0 (returns hipErrorInvalidValue otherwise).
hipError_t launch_mdp_fused(const MdpFusedArgs &a, hipStream_t s, const KTiming *t = nullptr);
bool mdp_fused_supported(int32_t W, int32_t H);

hipError_t launch_gauss5(const MdpArgs &a, hipStream_t s, const KTiming *t = nullptr);
hipError_t launch_thres(const MdpArgs &a, hipStream_t s, const KTiming *t = nullptr);
hipError_t launch_med5(const MdpArgs &a, hipStream_t s, const KTiming *t = nullptr);
// Add delta to every counter ptr[0..n) (n <= 8) in one launch.
hipError_t launch_advance_n(int64_t *const *ptr, int n, int64_t delta, int32_t *err, hipStream_t s);
// Add delta[i] to counter ptr[i] (n <= 8) in one launch.
hipError_t launch_advance_by(int64_t *const *ptr, const int64_t *delta, int n, int32_t *err, hipStream_t s);

// The predistortion network with materialised branch channels (rows of
// nf firings of r samples; tables from the offset scan, off in samples).
struct DpdNetArgs {
  const float2 *x;       // [S][nf*r]
  float2 *y;             // [S][nf*r]
  const float2 *h;       // [B_max][M]
  const int32_t *B;      // [S*nf] validated branch counts
  const int64_t *off;    // [B_max][stride] channel offset of each firing's block
  int64_t stride;        // S*nf
  int64_t nf, r, S;
  int32_t B_max, M;
  float2 *chan;          // [B_max][S][nf*r] Poly -> FIR_b channels
  float2 *firo;          // [B_max][S][nf*r] FIR_b -> Adder channels
  int32_t mask_mode;     // tokens are bit masks (k_mask_tables validates them); B holds branch sets either way
};
hipError_t launch_dpd_network(const DpdNetArgs &a, hipStream_t s, const KTiming *t = nullptr);
// Tables for bit-mask control tokens: validated masks (out of range -> 0)
// into B [S*nf] and channel offsets into off [B_max][S*nf], from ctrl [S][nf].
hipError_t launch_mask_tables(const int32_t *ctrl, int32_t *B, int64_t *off, const DpdNetArgs &a, hipStream_t s);

bool dpd_tiled_shape(int M);
hipError_t launch_dpd_heads(const DpdArgs &a, hipStream_t s);
// Body form for M = 16 from the environment: the VALU form, or the
// matrix-core form with DFHIP_BODY=mx (measured slower on MI355X: the
// complex products and row combination it leaves on the VALU cost nearly
// as many instructions as Horner's rule).
bool dpd_body_mx_env();
hipError_t launch_dpd_body(const DpdArgs &a, hipStream_t s, int tile, int outputs_per_thread,
                           const KTiming *timing = nullptr);
hipError_t launch_dpd_commit(const DpdCommitArgs &a, hipStream_t s);
// Add delta to one counter (word 0 or 1 of a channel slot) and check the
// channel's ring invariant.
hipError_t launch_advance(int64_t *idx, int64_t delta, int32_t *err, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_motion_count(const MotionArgs &a, hipStream_t s);
hipError_t launch_motion_emit_scan(const int32_t *count, int64_t n, int64_t emit_threshold,
                                   int64_t *emit_off, hipStream_t s);
hipError_t launch_motion_emit(const MotionArgs &a, hipStream_t s);
hipError_t launch_adj(const AdjArgs &a, hipStream_t s);
hipError_t launch_stream_copy(const void *src, void *dst, int64_t bytes, hipStream_t s);
// Bandwidth reference of one access mix: 0 copy, 1 read only, 2 write only,
// 3 two reads one write (src holds 2*bytes).
hipError_t launch_hbm_ref(int mode, const void *src, void *dst, int64_t bytes, hipStream_t s);
hipError_t launch_mp_adj(const float2 *u, const float2 *a, const float2 *g, float2 *Gu, int64_t n_streams,
                         int64_t len, int K, int Q, hipStream_t s);
hipError_t launch_motion_commit(const int64_t *emit_off, int64_t n, int64_t *cur_idx, int64_t *prev_idx,
                                int64_t *out_idx, int64_t *index_idx, int32_t *err, hipStream_t s);

}  // namespace dfh
