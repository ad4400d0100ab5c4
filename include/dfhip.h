/*
 * dfhip.h - C ABI of the dynamic-data-rate actor library for AMD MI355X (gfx950).
 *
 * Implements batched firing of GPU-mapped actors whose token consumption and
 * production per firing are fixed by control tokens (Boutellier & Hautala,
 * "Executing Dynamic Data Rate Actor Networks on OpenCL Platforms", SiPS 2016,
 * Sec. 2.2 and 3).  An application is a network of actors and FIFO channels
 * (Sec. 2.2); it is built by calls to this API (Sec. 3.4: the network is
 * described by a C function calling the framework's library).
 *
 * General conventions
 *   - Every call returns df_status; DF_OK (0) on success, a negative code
 *     otherwise.  No exception or signal crosses this boundary.  After an
 *     error, df_last_error() gives a human-readable reason.
 *   - All device work of a graph is ordered on the graph's HIP stream.
 *   - Device-side FIFO read/write indices are authoritative; kernels read
 *     them from device memory, so batches can be enqueued (and captured in
 *     a HIP graph) without host round trips.
 *   - A graph is used from one host thread at a time.  Distinct graphs are
 *     independent.
 *   - A HIP runtime failure poisons the graph: every later call on it
 *     returns DF_EDEVICE.
 *   - Pointers marked "device" must point to memory of the graph's device;
 *     "host" pointers to ordinary host memory.  The caller keeps ownership
 *     of every buffer it passes; the library owns FIFO storage and actor
 *     state and frees them in df_graph_destroy.
 */
#ifndef DFHIP_H
#define DFHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct df_graph df_graph;
typedef int32_t df_status;

enum {
  DF_OK = 0,
  DF_EINVAL = -1,    /* bad argument, handle, port, size or token value          */
  DF_EAGAIN = -2,    /* not enough tokens or space for an all-or-nothing firing;
                        nothing changed                                          */
  DF_ENOMEM = -3,    /* device or host allocation failed                         */
  DF_ESTATE = -4,    /* call not valid in the current wiring / state             */
  DF_EDEVICE = -5,   /* HIP runtime error; the graph is poisoned                 */
  DF_ECONTROL = -6,  /* a control token read on the device was out of range
                        (sticky; reported by df_sync)                            */
  DF_EINDEX = -7     /* a channel counter update on the device broke the ring
                        invariant read <= write <= read + capacity (the
                        order-preserving channel of Sec. 3.2 would have lost
                        or re-read tokens; sticky; reported by df_sync)          */
};

typedef enum { DF_C64 = 1, DF_U8 = 2, DF_I32 = 3, DF_I64 = 4 } df_dtype;

typedef enum {
  DF_ACTOR_DPD = 1,
  DF_ACTOR_MOTION = 2,
  DF_ACTOR_GAUSS5 = 3,   /* paper's motion-detection pipeline, Sec. 4.1 */
  DF_ACTOR_THRES = 4,
  DF_ACTOR_MED5 = 5
} df_actor_kind;

/* Ports of the predistortion actor. */
enum { DF_DPD_CTRL = 0, DF_DPD_IN = 1, DF_DPD_OUT = 2 };
/* Ports of the motion actor. */
enum { DF_MD_CUR = 0, DF_MD_PREV = 1, DF_MD_MASK = 2, DF_MD_INDEX = 3 };

/* Ports of the pipeline actors of Sec. 4.1 (Gauss -> Thres -> Med). */
enum { DF_GAUSS_IN = 0, DF_GAUSS_OUT = 1, DF_GAUSS_OUT2 = 2 };
enum { DF_THRES_CUR = 0, DF_THRES_PREV = 1, DF_THRES_OUT = 2 };
enum { DF_MED_IN = 0, DF_MED_OUT = 1 };

/* FIR history of a predistortion branch across firings where it is inactive. */
enum {
  DF_HIST_BRANCH = 0, /* a branch's delay line advances only when the branch
                         fires: after a gap its history is the tail of its own
                         last active firing (the dataflow reading of Sec. 2.2
                         for separate FIR actors selected per firing, Sec. 4.2) */
  DF_HIST_SHARED = 1  /* every branch's history is the true input stream       */
};

/* df_fire flags */
enum { DF_FIRE_PARTIAL = 1 };  /* fire as many firings as are admissible (<= n) */
/* df_fire_many flags */
enum { DF_FIRE_PERSISTENT = 1, DF_FIRE_GRAPH = 2 };

/*
 * Predistortion actor (Sec. 4.2).  One firing consumes one control token B
 * (0 <= B <= n_branches_max) and firing_size samples, and produces
 * firing_size samples:
 *     y[t] = sum_{b<B} sum_{m<n_taps} h[b][m] * psi_b(s_b[t-m]),
 *     psi_b(x) = |x|^(2b) x   (odd order 2b+1),
 * where s_b is branch b's input sample stream under history_mode.  Branches
 * b >= B have token rate 0 in this firing (Sec. 2.2: a dynamic actor's
 * regular ports take rate 0 or r per firing, fixed by the control token).
 * control_mode DF_CTRL_COUNT reads B as above (the prefix of branches 0..B-1
 * active); DF_CTRL_MASK reads a token as a bit mask, branch b active when
 * bit b is set, 0 <= token < 2^n_branches_max: any set of branches (Sec. 4.2
 * lets the configuration actor select which set of FIR filters runs, and
 * Sec. 3.1 leaves the mapping of control tokens to rates open).  The sum
 * above then runs over the set's branches.
 * Constraint: firing_size >= n_taps - 1.
 */
/* How a predistortion actor reads its control tokens. */
enum { DF_CTRL_COUNT = 0, DF_CTRL_MASK = 1 };
typedef struct {
  int32_t n_branches_max;   /* 1..16                                            */
  int32_t n_taps;           /* 1..32                                            */
  int64_t firing_size;      /* r: samples consumed and produced per firing      */
  const void *coeffs;       /* complex64 [n_branches_max][n_taps], row-major,
                               host or device (coeffs_on_device); copied        */
  int32_t coeffs_on_device;
  int32_t history_mode;     /* DF_HIST_BRANCH or DF_HIST_SHARED                 */
  int32_t control_mode;     /* DF_CTRL_COUNT or DF_CTRL_MASK                    */
  int32_t reserved;         /* 0                                                */
} df_dpd_params;            /* df_actor_create also takes the struct without
                               the last two fields (count tokens)               */

/*
 * Motion actor (frame difference, threshold, 3x3 opening; Sec. 4.1 builds
 * motion detection from consecutive-frame subtraction with a threshold, the
 * previous frame arriving over a channel with one initial token).  One
 * firing consumes one frame from CUR and one from PREV and computes
 *     changed = |cur - prev| > diff_threshold,
 *     o = dilate3x3(erode3x3(changed))  (out-of-frame neighbours ignored),
 *     count = number of set pixels of o.
 * It produces one MASK token (u8 frame, 255 where o is set) and one INDEX
 * token (int64 frame number, counted from the actor's first firing) iff
 * 1000*count >= min_changed_permille*width*height; otherwise it produces no
 * output token (rate 0 on both output ports).
 * With self_delay = 1 the PREV port is not used: the actor keeps the
 * previous CUR frame as state (an all-zero frame before the first firing),
 * which equals a PREV channel fed the same frames with one zero initial token.
 */
typedef struct {
  int32_t width, height;            /* token = width*height bytes             */
  int32_t diff_threshold;           /* 25 in the reference workload           */
  int32_t min_changed_permille;     /* 1 => 0.1 % of the pixels               */
  int32_t self_delay;               /* 0: PREV port wired; 1: internal delay  */
} df_motion_params;

/*
 * Static frame actors of the paper's motion-detection pipeline (Sec. 4.1):
 * Src -> Gauss -> Thres -> Med -> Sink on 8-bit frames, one frame per
 * token, every port consuming or producing `rate` tokens per firing (4 in
 * the paper's GPU mapping).  Frames are row-major width*height bytes.
 *   Gauss (DF_ACTOR_GAUSS5): 5x5 binomial filter, weights (1,4,6,4,1) x
 *     (1,4,6,4,1) / 256, rounded as (sum + 128) >> 8; rows 0, 1, H-2, H-1
 *     are copied unfiltered; a neighbour column outside the frame takes the
 *     nearest in-frame column.  The same frames go to OUT and, if connected,
 *     OUT2 (the paper joins Gauss to Thres by two channels, one of them
 *     holding one initial token: the one-frame delay).
 *   Thres (DF_ACTOR_THRES): 255 where |cur - prev| > threshold, else 0.
 *   Med (DF_ACTOR_MED5): median of the pixel and its 4 edge neighbours, a
 *     neighbour outside the frame taking the nearest in-frame pixel.
 */
typedef struct {
  int32_t width, height;   /* 1..65536 each                                  */
  int32_t rate;            /* tokens per port per firing, >= 1               */
  int32_t threshold;       /* Thres: 0..255; ignored by Gauss and Med        */
} df_frame_params;

/* Bytes of a channel sized by the paper's rule, Eq. (1) of Sec. 3.2:
 * token_bytes * (3*rate + 1) with a delay token (the buffer of Fig. 2),
 * token_bytes * 2*rate without (a double buffer).  A host-side helper for
 * comparing footprints: this library's rings are sized by the caller
 * instead (a power of two of at least the batch), so that a batch of many
 * firings can sit in one channel.  Returns -1 for token_bytes < 1 or
 * rate < 1. */
int64_t df_paper_channel_bytes(int64_t token_bytes, int64_t rate, int32_t has_delay);

/* ------------------------------------------------------------------ graph */

/* Create an empty network on HIP device `hip_device`.  `hip_stream` is a
 * hipStream_t to order all work on (e.g. torch's current stream), or NULL
 * for a library-owned stream.  *g receives the handle.  Environment read
 * here: DFHIP_CHECK_INDICES (see df_sync), DFHIP_LOG=1|2 (a stderr line per
 * firing call and graph capture; 2 also per scan run ahead),
 * DFHIP_TILE=tile,outputs_per_thread,blocks_per_cu (as df_set_tile),
 * DFHIP_SCAN_AHEAD=0 (df_fire does not scan the next batch's control tokens
 * ahead; results are the same either way), DFHIP_BODY=mx (16-tap bodies on
 * the matrix cores: same results within the FP32 tolerance, rounded
 * differently from the default VALU form). */
df_status df_graph_create(df_graph **g, int hip_device, void *hip_stream);

/* Synchronise, free all FIFO storage, actor state and the owned stream. */
df_status df_graph_destroy(df_graph *g);

/* Wait for all enqueued work; report sticky device errors (DF_EINDEX, then
 * DF_ECONTROL).  Every kernel that advances a channel counter (push, pop,
 * batch commits) checks the channel's ring invariant afterwards.  With the
 * environment variable DFHIP_CHECK_INDICES=1 at df_graph_create, every
 * push, pop and firing call also synchronises and reports these errors
 * itself, so the failing call is the one that returns them. */
df_status df_sync(df_graph *g);

/* Reason for the last failing call on g (static storage, never NULL). */
const char *df_last_error(const df_graph *g);

/* Library version string, e.g. "dfhip 0.1 gfx950". */
const char *df_version(void);

/* ------------------------------------------------------------------ FIFOs */

/* Create an order-preserving channel (Sec. 3.2) as a device ring of
 * capacity_tokens tokens (rounded up to a power of two; 0 picks
 * max(2*n_initial, 1024)) of elems_per_token elements of type dt.
 * n_initial delay tokens are present before any firing (Sec. 2.2; the paper
 * allows 0 or 1, any number is accepted here): their values are read from
 * initial_host (host, n_initial tokens) or are zero when it is NULL.
 * *fifo_out receives the channel id.
 * Errors: DF_EINVAL (bad dtype/sizes, n_initial > capacity), DF_ENOMEM. */
df_status df_fifo_create(df_graph *g, df_dtype dt, int64_t elems_per_token,
                         int64_t capacity_tokens, int64_t n_initial,
                         const void *initial_host, int32_t *fifo_out);

/* Create a channel in the paper's own layout (Sec. 3.2): capacity exactly as
 * Eq. (1), for a channel whose every write and read moves `rate` tokens.
 * Without a delay token (n_initial = 0) it is a double buffer of 2*rate
 * slots.  With one (n_initial = 1) it has 3*rate + 1 slots and the access
 * pattern of Fig. 2: the delay token sits in slot 0, the writes fill slots
 * 1..3*rate in turn, the reads take slots 0..3*rate-1 in turn, and after the
 * write that fills slot 3*rate its token is copied to slot 0.  Token order
 * is that of any other channel; only the placement differs.  At most
 * 2*rate (3*rate) tokens are held at once, so a batch on such a channel
 * admits at most two firings.  Such a channel connects only to the frame
 * actors (Gauss, Thres, Med) and to the host; a device kernel addresses it
 * through the same slot rule.  initial_host: the delay token's value (NULL:
 * zeros).  Errors: DF_EINVAL (bad dtype or size, n_initial not 0 or 1,
 * rate < 1), DF_ENOMEM. */
df_status df_fifo_create_paper(df_graph *g, df_dtype dt, int64_t elems_per_token,
                               int64_t rate, int64_t n_initial, const void *initial_host,
                               int32_t *fifo_out);

/* Device bytes a channel allocates for its tokens (ring: capacity tokens;
 * paper layout: 2*rate or 3*rate + 1 tokens), or -1 for a bad id.  Host
 * only. */
int64_t df_fifo_bytes(df_graph *g, int32_t fifo);

/* Token counts of a channel.  Synchronises when the producer's rate is
 * data-dependent (the device indices are read back).  read/write indices
 * count tokens since creation; initial tokens occupy write indices
 * 0..n_initial-1.  Any output pointer may be NULL. */
df_status df_fifo_status(df_graph *g, int32_t fifo, int64_t *read_idx,
                         int64_t *write_idx, int64_t *capacity);

/* Element type and token shape of a channel: *dtype receives its df_dtype,
 * *elems_per_token the elements of one token and *token_bytes their bytes.
 * Lets a binding check that a buffer handed to df_push / df_pop holds the
 * tokens it claims.  Any output pointer may be NULL.  Host only; no device
 * work.  Errors: DF_EINVAL (bad fifo id). */
df_status df_fifo_info(df_graph *g, int32_t fifo, int32_t *dtype,
                       int64_t *elems_per_token, int64_t *token_bytes);

/* ------------------------------------------------------------------ actors */

/* Create an actor of `kind` with a parameter struct (df_dpd_params or
 * df_motion_params; params_size = sizeof that struct).  The actor's init
 * (Sec. 3.1) runs here: coefficients are copied, state zeroed.
 * Errors: DF_EINVAL (bad kind, size or parameter). */
df_status df_actor_create(df_graph *g, df_actor_kind kind, const void *params,
                          size_t params_size, int32_t *actor_out);

/* Connect an actor port to a channel.  A channel connects exactly one output
 * port to exactly one input port (Sec. 3.2); the host is the implicit writer
 * of channels no actor writes and the implicit reader of channels no actor
 * reads.  Token shape and dtype must match the port.  A channel with initial
 * tokens cannot feed a control port (Sec. 2.2).
 * Errors: DF_EINVAL (bad ids, port, dtype or token size), DF_ESTATE (port or
 * channel end already connected, initial tokens on a control channel). */
df_status df_connect(df_graph *g, int32_t actor, int32_t port, int32_t fifo);

/* Fixed token rate of one port of an actor (Sec. 2.2: tokens a firing moves
 * on that port; for the predistortion actor's branch-dependent rates the
 * data ports move firing_size samples every firing, the control port 1).
 * The motion actor's outputs are data-dependent: *rate receives the upper
 * bound 1.  Host only.  Errors: DF_EINVAL (bad actor id or port). */
df_status df_port_rate(df_graph *g, int32_t actor, int32_t port, int64_t *rate);

/* ------------------------------------------------------------------ tokens */

/* Append n_tokens tokens from src (host, or device when src_on_device) to a
 * channel the host writes.  A host push has finished reading src when the
 * call returns; a device push is stream-ordered (keep src alive until
 * df_sync).  Tokens written to a DPD control channel are checked to lie in
 * 0..n_branches_max (host pushes only).
 * Errors: DF_EAGAIN (not enough space; nothing written), DF_EINVAL (bad
 * token value, n_tokens < 0), DF_ESTATE (an actor writes this channel). */
df_status df_push(df_graph *g, int32_t fifo, const void *src, int64_t n_tokens,
                  int src_on_device);

/* Remove up to max_tokens tokens from a channel the host reads into dst
 * (host, or device when dst_on_device); *n_popped receives the number
 * moved.  A host pop has completed when the call returns; a device pop is
 * stream-ordered.  Errors: DF_ESTATE (an actor reads this channel). */
df_status df_pop(df_graph *g, int32_t fifo, void *dst, int64_t max_tokens,
                 int dst_on_device, int64_t *n_popped);

/* ------------------------------------------------------------------ firing */

/* Fire `actor` n_firings times, in order, as one batch (Sec. 2.2 firing rule
 * applied to every firing; the batch is a schedule of the same firings, so
 * results equal firing them one by one).  The batch runs as device kernels:
 * control intake and rate resolution, an offset scan over the per-firing
 * rates, the actor body, and a commit of the channel indices.
 * Reads and writes of the paper are blocking (Sec. 2.2); here admission is
 * all-or-nothing: if the statically known token counts (control tokens,
 * input tokens, worst-case output space) do not allow n_firings firings the
 * call returns DF_EAGAIN and changes nothing, unless flags has
 * DF_FIRE_PARTIAL, which fires the admissible prefix.  *n_fired (may be
 * NULL) receives the number fired.  Out-of-range control tokens found on the
 * device raise the sticky DF_ECONTROL and are treated as 0.
 * Errors: DF_EINVAL, DF_ESTATE (ports not all connected), DF_EAGAIN. */
df_status df_fire(df_graph *g, int32_t actor, int64_t n_firings, int flags,
                  int64_t *n_fired);

/* Fire many predistortion actors, actor[i] n_firings[i] times each (host
 * arrays of n_actors entries), as one batch of independent instances.
 * flags = 0: one df_fire per actor.  DF_FIRE_PERSISTENT: one persistent
 * kernel whose workgroups pull (instance, firing, tile) work items from a
 * device queue built by a segmented offset scan.  DF_FIRE_GRAPH (with
 * PERSISTENT): the scan -> persistent kernel -> commit chain is captured
 * once in a HIP graph for this actor list and replayed on later calls.
 * Admission is all-or-nothing over all instances (DF_EAGAIN).
 * Errors: DF_EINVAL (not DPD actors, duplicates, mixed n_taps), DF_ESTATE. */
df_status df_fire_many(df_graph *g, int32_t n_actors, const int32_t *actors,
                       const int64_t *n_firings, int flags);

/* Fire the chain Gauss -> Thres -> Med of Sec. 4.1 n_firings times: the same
 * as df_fire(gauss, n), df_fire(thres, n), df_fire(med, n) in that order
 * (same output tokens, same channel counters and pending tokens afterwards),
 * with admission over the whole chain (DF_EAGAIN, or the admissible prefix
 * with DF_FIRE_PARTIAL).  When the chain is wired as in the paper (Gauss OUT
 * and OUT2 to Thres CUR and PREV, Thres OUT to Med IN, equal frame
 * parameters), the Gauss->Thres current and Thres->Med channels are empty,
 * the delay channel holds exactly one token and the width is a multiple of
 * 4, one fused kernel fires the batch: the frames of the inner channels stay
 * on chip, and only the delay channel's one pending token (the last Gauss
 * frame) is written.  Otherwise, or with DF_PIPE_SEPARATE in flags, the three
 * actors fire one after the other.  A fused launch is timed as the Gauss
 * actor's.  *n_fired (may be NULL) receives the firings per actor.
 * Errors: DF_EINVAL (not such a chain), DF_ESTATE, DF_EAGAIN. */
enum { DF_PIPE_SEPARATE = 2 };
df_status df_fire_pipeline(df_graph *g, int32_t gauss, int32_t thres, int32_t med,
                           int64_t n_firings, int flags, int64_t *n_fired);

/* Stream host data through one predistortion actor: n_batches batches of
 * firings_per_batch firings, control tokens from ctrl_host (int32
 * [n_batches*firings_per_batch]), samples from x_host (complex64
 * [n_batches*firings_per_batch*firing_size]), outputs to y_host (same
 * size).  The same tokens as pushing, firing and popping each batch in turn,
 * but batch k's input copy, batch k-1's firing and batch k-2's output copy
 * run concurrently (two copy streams beside the graph's stream, ordered by
 * events; the analogue of GPP-mapped source/sink actors running beside the
 * GPU actors, Sec. 3.3).  Host buffers should be page-locked for the copies
 * to overlap.  The control and output channels must be empty and written /
 * read by the host; every channel must hold two batches (the input channel
 * two batches plus its pending tokens).  Returns when all outputs are in
 * y_host.  Errors: DF_EINVAL, DF_ESTATE, DF_EDEVICE. */
df_status df_stream_dpd(df_graph *g, int32_t actor, const void *x_host,
                        const int32_t *ctrl_host, void *y_host, int64_t n_batches,
                        int64_t firings_per_batch);

/* Tile configuration of the DPD body kernels: tile_outputs samples per
 * workgroup work item (a multiple of 64*outputs_per_thread, at most
 * 512*outputs_per_thread), outputs_per_thread (4 or 8), and the persistent
 * kernel's workgroups per compute unit (1..16).  0 keeps the current value.
 * Used by the autotuner.  Errors: DF_EINVAL. */
df_status df_set_tile(df_graph *g, int32_t tile_outputs, int32_t outputs_per_thread,
                      int32_t blocks_per_cu);

/* Kernel timing.  While enabled, every batch records HIP events on the
 * graph's stream around its actor-body kernels (predistortion body; motion
 * count + emit passes; Gauss, Thres and Med bodies; the persistent body
 * kernel, or the whole replayed graph when captured).  df_profile_read
 * synchronises, returns the summed time and number of timed launches since
 * the last read, and resets them.  df_profile_read_actor does the same for
 * the launches of one actor only (persistent batches belong to no actor)
 * and leaves the others pending.
 * Errors: DF_EINVAL, DF_EDEVICE. */
df_status df_profile_enable(df_graph *g, int32_t enable);
df_status df_profile_read(df_graph *g, double *total_ms, int64_t *n_launches);
df_status df_profile_read_actor(df_graph *g, int32_t actor, double *total_ms,
                                int64_t *n_launches);

/* Test hook: overwrite the device read and write counters of a channel
 * (the host's own bookkeeping is left alone), so that a test can drive the
 * ring invariant check of the next counter update.  Stream-ordered.
 * Errors: DF_EINVAL (bad fifo id), DF_EDEVICE. */
df_status df_debug_set_counters(df_graph *g, int32_t fifo, int64_t read_idx, int64_t write_idx);

/* Test hook: copy a channel's whole slot storage (df_fifo_bytes bytes,
 * slot-major) to host memory dst of max_bytes bytes, after the graph's
 * pending work; lets a test check where tokens sit (the Fig. 2 pattern).
 * Errors: DF_EINVAL (bad id, max_bytes too small), DF_EDEVICE. */
df_status df_debug_read_slots(df_graph *g, int32_t fifo, void *dst, int64_t max_bytes);

/* Test hook: per-firing tables of the last batch of a DPD actor (device
 * results copied to host arrays of at least cap entries per row):
 * rates [n_branches_max][n], offsets [n_branches_max][n] (token offset of
 * the firing's block on branch b's channel), prev [n_branches_max][n] (the
 * firing whose tail is branch b's FIR history, -1: carried state);
 * *n_out receives n.  Any array pointer may be NULL. */
df_status df_debug_last_batch(df_graph *g, int32_t actor, int32_t *rates,
                              int64_t *offsets, int64_t *prev, int64_t cap,
                              int64_t *n_out);

/* ------------------------------------------------------- stateless kernels */
/* Device-pointer entry points used by the autograd binding.  All run on
 * `stream` (a hipStream_t, NULL = default stream) and do not synchronise.
 * Each of the n_streams rows of length len is an independent predistortion
 * actor fired len/r times from zero state with no delay tokens.  ctrl is
 * int32 [n_streams][len/r] control tokens, or NULL for all branches active
 * in every firing.  x, y, G: complex64 [n_streams][len]; h, grad_h:
 * complex64 [B_max][M].  len must be a multiple of r, r >= M-1.
 * Errors: DF_EINVAL (sizes), DF_EDEVICE (launch failure). */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): the same
 * operation and arguments as df_dpd_forward, with identical results, but
 * its scratch (branch counts, history sources, scan group table, head
 * corrections) is a fixed device array of df_dpd_forward_noalloc_max_bytes()
 * bytes (12 MiB; enough for any call of up to 16384 firings, n_branches_max
 * <= 16, n_taps <= 32) that each GPU holds until the process ends.  Calls no
 * allocator.  A call needing more scratch returns DF_EINVAL and does nothing.
 * All calls on one GPU share that array: calls that overlap in time on one
 * GPU (different streams, or host threads) race and must be serialised by
 * the caller; calls ordered on one stream are safe.  Nothing in the array
 * needs clearing between calls. */
df_status df_dpd_forward_noalloc(void *stream, const void *x, const int32_t *ctrl,
                                 const void *h, void *y, int64_t n_streams, int64_t len,
                                 int64_t r, int32_t B_max, int32_t M, int32_t hist);
int64_t df_dpd_forward_noalloc_max_bytes(void);

/* y = DPD_h(x) (the predistortion actor body above). */
df_status df_dpd_forward(void *stream, const void *x, const int32_t *ctrl,
                         const void *h, void *y, int64_t n_streams, int64_t len,
                         int64_t r, int32_t B_max, int32_t M, int32_t hist);

/* The same y computed by the network of Sec. 4.2 as drawn: a Poly kernel
 * writing psi_b(x) of every firing to branch channel b (only for the
 * firing's active branches: the dynamic rates of Sec. 2.2), one FIR kernel
 * per branch over the samples its channel received, and an Adder kernel
 * summing the active branches' outputs at each firing's channel offsets.
 * ctrl_mode DF_CTRL_COUNT: a token B activates b < B (as everywhere else);
 * DF_CTRL_MASK: a token is a bit mask of active branches, any subset (Sec.
 * 4.2 lets the configuration actor select which set of FIR filters runs);
 * out-of-range tokens count as 0.  The 2*B_max*n_streams*len complex64
 * branch channels are allocated on `stream` for the call.  Branch history
 * only (the FIR actors' own delay lines, DF_HIST_BRANCH); ctrl must not be
 * NULL.  With count tokens the results equal df_dpd_forward's up to FP32
 * rounding order.  Errors as df_dpd_forward. */
df_status df_dpd_forward_network(void *stream, const void *x, const int32_t *ctrl,
                                 const void *h, void *y, int64_t n_streams, int64_t len,
                                 int64_t r, int32_t B_max, int32_t M, int32_t ctrl_mode);

/* Coefficient adjoint: grad_h[b][m] = sum over rows and samples n of
 * G[n] * conj(d y[n] / d h[b][m]), i.e. dL/dRe h + i dL/dIm h given
 * G[n] = dL/dRe y[n] + i dL/dIm y[n].  Deterministic (fixed reduction
 * order, no floating-point atomics).  grad_h is overwritten.
 * `work` is a device buffer of df_dpd_coeff_adjoint_work_bytes() bytes. */
df_status df_dpd_coeff_adjoint(void *stream, const void *x, const int32_t *ctrl,
                               const void *G, void *grad_h, int64_t n_streams,
                               int64_t len, int64_t r, int32_t B_max, int32_t M,
                               int32_t hist, void *work, int64_t work_bytes);
int64_t df_dpd_coeff_adjoint_work_bytes(int64_t n_streams, int64_t len, int64_t r,
                                        int32_t B_max, int32_t M);

/* Memory-polynomial input adjoint.  For v[n] = sum_k sum_q a[k][q]
 * |u[n-q]|^(2k) u[n-q] (a: complex64 [K][Q], orders 1,3,..,2K-1) and an
 * upstream gradient g = dL/dRe v + i dL/dIm v, writes
 * Gu = dL/dRe u + i dL/dIm u (Wirtinger chain rule).  u, g, Gu: complex64
 * [n_streams][len]; samples past a row's end contribute nothing. */
df_status df_mp_input_adjoint(void *stream, const void *u, const void *a,
                              const void *g, void *Gu, int64_t n_streams,
                              int64_t len, int32_t K, int32_t Q);

/* Measurement helper (no operation of the method): copies `bytes` bytes from
 * device buffer src to device buffer dst on `stream` (NULL: the null stream)
 * with a plain 16-byte-vector stream-copy kernel.  It is the reference
 * against which the actor kernels' bandwidth and HBM traffic counters are
 * scaled.  bytes must be a multiple of 16 and both pointers 16-byte
 * aligned (else DF_EINVAL); the buffers must not overlap and stay owned by
 * the caller, who keeps them alive until the stream has passed the copy. */
/* Measurement helper (no operation of the method): one HBM access mix over
 * `bytes` bytes on `stream`, for the achievable-bandwidth references.
 * mode 0: copy src -> dst (reads and writes `bytes`, same as df_stream_copy);
 * 1: read src only (dst receives at most 16 bytes);
 * 2: write dst only (src unused, may be NULL);
 * 3: dst[i] = src[i] ^ src[bytes + i] (reads 2*bytes from src, writes bytes).
 * bytes a multiple of 16, pointers 16-byte aligned, buffers owned by the
 * caller and alive until the stream has passed the call.
 * Errors: DF_EINVAL. */
df_status df_hbm_ref(void *stream, int32_t mode, const void *src, void *dst, int64_t bytes);

df_status df_stream_copy(void *stream, const void *src, void *dst,
                         int64_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* DFHIP_H */
