// Many predistortion instances fired as one batch.
//
// Every instance is an independent actor with its own channels, coefficients
// and control tokens; a batch fires instance i n_i times.  The chain is
//   prep:     exclusive scan of n_i (firing bases), work-queue reset
//   scan:     per-instance control intake and branch offset scan
//   order:    instances grouped by branch count, work-item bases in that order
//   body:     a persistent grid whose workgroups pull (instance, firing,
//             tile) work items from a device counter until none is left
//   commit:   per-instance channel indices and carried branch histories
// All counts live in device memory, so the chain can be captured once in a
// HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "common.h"
#include "dpd_tile.h"
#include "runtime.h"

namespace dfh {

struct InstDesc {
  const float2 *x;
  int64_t *x_idx;
  int64_t x_mask;
  float2 *y;
  int64_t *y_idx;
  int64_t y_mask;
  const int32_t *ctrl;
  int64_t *ctrl_idx;
  int64_t ctrl_mask;
  const float2 *h;
  float2 *hist;
  int64_t r;
  int32_t B_max;
  int32_t hist_mode;
  int32_t tpf;            // tiles per firing
  int32_t pad;
};

struct PersArgs {
  const InstDesc *inst;
  int32_t n_inst;
  int32_t Bg;             // largest n_branches_max of the instances
  const int64_t *n_fire;  // [n_inst]
  int64_t *fire_base;     // [n_inst + 1]
  int64_t *tile_base;     // [n_inst + 1] work-item bases in processing order
  int32_t *inst_order;    // [n_inst] processing order of the instances
  int32_t *B_all;         // [cap]
  int64_t *prev_all;      // [Bg][cap], instance-local firing index or -1
  int64_t *last_all;      // [n_inst][Bg]
  int64_t cap;
  int32_t *queue;
  int32_t *err;
  int32_t tile;
};

// One wavefront: exclusive scan of the firing counts (firing bases).
__global__ __launch_bounds__(64) void k_pers_prep(PersArgs a) {
  const int lane = threadIdx.x;
  int64_t cf = 0;
  for (int c = 0; c < a.n_inst; c += 64) {
    const int i = c + lane;
    const int64_t nf = i < a.n_inst ? a.n_fire[i] : 0;
    int64_t sf = nf;                               // inclusive wave scan
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t uf = __shfl_up(sf, d);
      if (lane >= d) sf += uf;
    }
    if (i < a.n_inst) a.fire_base[i] = cf + sf - nf;
    cf += __shfl(sf, 63);
  }
  if (lane == 0) {
    a.fire_base[a.n_inst] = cf;
    a.queue[0] = 0;
  }
}

// Processing order of the instances, grouped by the branch count of their
// first firing (largest first), and the work-item bases in that order.  The
// body compiles one unrolled code path per branch count; grouping keeps the
// workgroups resident on a compute unit on few paths (instruction cache).
// The order never changes a result.
__global__ __launch_bounds__(1024) void k_pers_order(PersArgs a) {
  __shared__ int32_t hist[kMaxBranches + 1], cursor[kMaxBranches + 1];
  __shared__ int64_t wsum[16];
  if (threadIdx.x <= kMaxBranches) hist[threadIdx.x] = 0;
  __syncthreads();
  auto key = [&](int i) { return a.n_fire[i] > 0 ? a.B_all[a.fire_base[i]] : 0; };
  for (int i = threadIdx.x; i < a.n_inst; i += blockDim.x) atomicAdd(&hist[key(i)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int v = kMaxBranches; v >= 0; --v) {
      cursor[v] = run;
      run += hist[v];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a.n_inst; i += blockDim.x) a.inst_order[atomicAdd(&cursor[key(i)], 1)] = i;
  __syncthreads();
  // exclusive scan of tiles over the ordered instances
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int64_t carry = 0;
  for (int c = 0; c < a.n_inst; c += blockDim.x) {
    const int k = c + threadIdx.x;
    int64_t nt = 0;
    if (k < a.n_inst) {
      const int i = a.inst_order[k];
      nt = a.n_fire[i] * a.inst[i].tpf;
    }
    int64_t sc = nt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t u = __shfl_up(sc, d);
      if (lane >= d) sc += u;
    }
    if (lane == 63) wsum[wid] = sc;
    __syncthreads();
    int64_t before = carry;
    for (int w = 0; w < wid; ++w) before += wsum[w];
    if (k < a.n_inst) a.tile_base[k] = before + sc - nt;
    int64_t total = 0;
    for (int w = 0; w < nw; ++w) total += wsum[w];
    __syncthreads();
    carry += total;
  }
  if (threadIdx.x == 0) a.tile_base[a.n_inst] = carry;
}

// One workgroup per instance, one wavefront per branch (as the single-actor
// scan): validated control tokens, history source firings, last feeders.
__global__ __launch_bounds__(1024) void k_pers_scan(PersArgs a) {
  const int i = blockIdx.x;
  const int b = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const InstDesc &d = a.inst[i];
  if (b >= d.B_max) return;
  const int64_t n = a.n_fire[i];
  const int64_t base = a.fire_base[i];
  const int64_t R = d.ctrl_idx[0];
  const uint64_t below_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  int64_t lastw = -1;
  for (int64_t c = 0; c < n; c += 64) {
    const int64_t j = c + lane;
    const bool in = j < n;
    int32_t B = 0;
    if (in) {
      int32_t v = d.ctrl[(R + j) & d.ctrl_mask];
      if (v < 0 || v > d.B_max) {
        if (b == 0) atomicOr(a.err, (int32_t)kErrControl);
        v = 0;
      }
      B = v;
      if (b == 0) a.B_all[base + j] = B;
    }
    const bool fed = in && (d.hist_mode == 1 || B > b);
    const uint64_t bal = __ballot(fed);
    const uint64_t below = bal & below_mask;
    if (in) a.prev_all[(int64_t)b * a.cap + base + j] = below ? (c + 63 - __clzll((long long)below)) : lastw;
    if (bal) lastw = c + 63 - __clzll((long long)bal);
  }
  if (lane == 0) a.last_all[(int64_t)i * a.Bg + b] = lastw;
}

// Persistent body: workgroups pull (instance, firing, tile) work items from
// the queue; the next item's window and histories are loaded into registers
// while the current item is computed from LDS.  The item number is made
// wavefront-uniform, so the instance table and the instance's coefficients
// are read with scalar loads.
template <int M, int K>
__global__ __launch_bounds__(512) void k_pers_body(PersArgs a) {
  extern __shared__ float2 lds[];   // [2*Bg*(M-1)] histories, window
  float2 *sq = lds, *sx = sq + lds_history(a.Bg, M);
  __shared__ int item_s;
  const auto *inst = as_const(a.inst);
  const auto *tile_base = as_const(a.tile_base);
  const int64_t total = tile_base[a.n_inst];
  if (threadIdx.x == 0) item_s = atomicAdd(a.queue, 1);
  __syncthreads();
  int64_t item = __builtin_amdgcn_readfirstlane(item_s);
  if (item >= total) return;                          // uniform: every wave leaves
  struct Item {
    int inst;
    int64_t gfire, Rx, j;
  };
  auto decode = [&](int64_t it, Item &d, TileJob &job) {
    int lo = 0, hi = a.n_inst - 1;                    // last ordered instance with base <= it
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tile_base[mid] <= it) lo = mid; else hi = mid - 1;
    }
    d.inst = as_const(a.inst_order)[lo];
    const auto &ds = inst[d.inst];
    const int64_t local = it - tile_base[lo];
    d.j = local / ds.tpf;
    d.gfire = as_const(a.fire_base)[d.inst] + d.j;
    d.Rx = as_const(ds.x_idx)[0];
    job.t0 = (local - d.j * ds.tpf) * a.tile;
    job.nout = (int)min((int64_t)a.tile, ds.r - job.t0);
    job.B = as_const(a.B_all)[d.gfire];
    job.head = (job.t0 == 0 && job.B > 0 && M > 1) ? 1 : 0;
    job.xb = d.Rx + d.j * ds.r;
    job.yb = as_const(ds.y_idx)[1] + d.j * ds.r;
  };
  auto prefetch = [&](const Item &d, const TileJob &job, TileRegs<M, K> &r) {
    const auto &ds = inst[d.inst];
    tile_prefetch<M, K>(r, job, ds.x, ds.x_mask, [&](int b, int64_t ii) {
      const int64_t pf = a.prev_all[(int64_t)b * a.cap + d.gfire];
      if (pf >= 0) return ds.x[(d.Rx + pf * ds.r + ds.r + ii) & ds.x_mask];
      return ds.hist[b * (M - 1) + (M - 1) + ii];
    });
  };
  Item cur;
  TileJob job;
  decode(item, cur, job);
  TileRegs<M, K> regs;
  prefetch(cur, job, regs);
  for (;;) {
    tile_commit<M, K>(sx, sq, regs, job);
    if (threadIdx.x == 0) item_s = atomicAdd(a.queue, 1);
    __syncthreads();
    const int64_t next = __builtin_amdgcn_readfirstlane(item_s);
    Item nd = cur;
    TileJob nj = job;
    if (next < total) {
      decode(next, nd, nj);
      prefetch(nd, nj, regs);
    }
    const cfloat2p hg = as_const(inst[cur.inst].h);
    if (job.head) {
      tile_head_sums<M>(sq, hg, job.B);
      __syncthreads();
    }
    tile_outputs<M, K>(sx, hg, sq, job, inst[cur.inst].y, inst[cur.inst].y_mask);
    if (next >= total) break;
    __syncthreads();
    cur = nd;
    job = nj;
  }
}

__global__ __launch_bounds__(256) void k_pers_commit(PersArgs a, int M) {
  const int i = blockIdx.x;
  const InstDesc &d = a.inst[i];
  const int64_t n = a.n_fire[i];
  if (n == 0) return;
  const int64_t Rx = d.x_idx[0];
  __syncthreads();
  const int L = M - 1;
  for (int t = threadIdx.x; t < d.B_max * L; t += blockDim.x) {
    const int b = t / L, k = t - b * L;
    const int64_t lf = a.last_all[(int64_t)i * a.Bg + b];
    if (lf >= 0) d.hist[b * L + k] = d.x[(Rx + lf * d.r + d.r - L + k) & d.x_mask];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    d.x_idx[0] = Rx + n * d.r;
    d.ctrl_idx[0] += n;
    d.y_idx[1] += n * d.r;
  }
}

// ------------------------------------------------------------------ host side

struct Persistent {
  std::vector<int32_t> actors;
  int M = 0, Bg = 0;
  InstDesc *inst = nullptr;
  int64_t *n_dev = nullptr;
  std::vector<int64_t> n_host;
  int64_t *fire_base = nullptr, *tile_base = nullptr, *prev_all = nullptr, *last_all = nullptr;
  int32_t *B_all = nullptr, *queue = nullptr, *inst_order = nullptr;
  int64_t cap = 0;
  int tile = 0, K = 0, bpc = 0, ncu = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void drop_graph(Persistent *p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

void destroy_persistent(df_graph *g) {
  Persistent *p = g->pers;
  if (!p) return;
  drop_graph(p);
  (void)hipFree(p->inst);
  (void)hipFree(p->n_dev);
  (void)hipFree(p->fire_base);
  (void)hipFree(p->tile_base);
  (void)hipFree(p->prev_all);
  (void)hipFree(p->last_all);
  (void)hipFree(p->B_all);
  (void)hipFree(p->queue);
  (void)hipFree(p->inst_order);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
  g->pers = nullptr;
}

template <int M, int K>
static hipError_t launch_pers_body(const PersArgs &a, int threads, int blocks, hipStream_t s) {
  const size_t lds = (size_t)(lds_window(a.tile + M - 1) + lds_history(a.Bg, M)) * sizeof(float2);
  hipLaunchKernelGGL((k_pers_body<M, K>), dim3(blocks), dim3(threads), lds, s, a);
  return hipGetLastError();
}

static hipError_t enqueue_chain(Persistent *p, const PersArgs &a, hipStream_t s, df_graph *prof_g) {
  if (a.Bg * (p->M - 1) > kHistRegs * (p->tile / p->K)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pers_prep, dim3(1), dim3(64), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pers_scan, dim3(a.n_inst), dim3(64 * a.Bg), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pers_order, dim3(1), dim3(1024), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int threads = p->tile / p->K;
  const int blocks = p->bpc * p->ncu;
  if (prof_g && (e = prof_begin(prof_g)) != hipSuccess) return e;
  if (p->M == 16 && p->K == 4) e = launch_pers_body<16, 4>(a, threads, blocks, s);
  else if (p->M == 16 && p->K == 8) e = launch_pers_body<16, 8>(a, threads, blocks, s);
  else if (p->M == 8 && p->K == 4) e = launch_pers_body<8, 4>(a, threads, blocks, s);
  else if (p->M == 8 && p->K == 8) e = launch_pers_body<8, 8>(a, threads, blocks, s);
  else if (p->M == 4 && p->K == 4) e = launch_pers_body<4, 4>(a, threads, blocks, s);
  else if (p->M == 4 && p->K == 8) e = launch_pers_body<4, 8>(a, threads, blocks, s);
  else return hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  if (prof_g && (e = prof_end(prof_g)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pers_commit, dim3(a.n_inst), dim3(256), 0, s, a, p->M);
  return hipGetLastError();
}

}  // namespace dfh

using namespace dfh;

#define HIPCHK(g, expr)                                    \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return fail_hip((g), e_, #expr); \
  } while (0)

extern "C" df_status df_fire_many(df_graph *g, int32_t n_actors, const int32_t *actors, const int64_t *n_firings,
                                  int flags) {
  if (!g) return fail(nullptr, DF_EINVAL, "null graph");
  if (g->poisoned) return fail(g, DF_EDEVICE, "graph poisoned by an earlier HIP error");
  HIPCHK(g, hipSetDevice(g->device));
  if (n_actors < 1 || !actors || !n_firings) return fail(g, DF_EINVAL, "df_fire_many: empty or null arrays");
  if (flags & ~(DF_FIRE_PERSISTENT | DF_FIRE_GRAPH)) return fail(g, DF_EINVAL, "bad flags 0x%x", flags);
  if ((flags & DF_FIRE_GRAPH) && !(flags & DF_FIRE_PERSISTENT))
    return fail(g, DF_EINVAL, "DF_FIRE_GRAPH requires DF_FIRE_PERSISTENT");
  std::vector<char> seen(g->actors.size(), 0);
  int M = -1, Bg = 0;
  int64_t max_r = 1, total = 0;
  for (int i = 0; i < n_actors; ++i) {
    const int id = actors[i];
    if (id < 0 || id >= (int)g->actors.size()) return fail(g, DF_EINVAL, "bad actor id %d", id);
    if (seen[id]) return fail(g, DF_EINVAL, "actor %d listed twice", id);
    seen[id] = 1;
    Actor &a = g->actors[id];
    if (a.kind != DF_ACTOR_DPD) return fail(g, DF_EINVAL, "actor %d is not a predistortion actor", id);
    if (n_firings[i] < 0) return fail(g, DF_EINVAL, "negative firing count");
    if (M < 0) M = a.dp.n_taps;
    if ((flags & DF_FIRE_PERSISTENT) && a.dp.n_taps != M)
      return fail(g, DF_EINVAL, "persistent batching needs one n_taps for all instances");
    Bg = std::max(Bg, a.dp.n_branches_max);
    max_r = std::max(max_r, a.dp.firing_size);
    total += n_firings[i];
    int64_t adm;
    df_status st = dpd_admit(g, a, n_firings[i], &adm);
    if (st) return st;
    if (adm < n_firings[i])
      return fail(g, DF_EAGAIN, "actor %d: only %lld of %lld firings admissible", id, (long long)adm,
                  (long long)n_firings[i]);
  }
  if (!(flags & DF_FIRE_PERSISTENT)) {
    for (int i = 0; i < n_actors; ++i) {
      if (!n_firings[i]) continue;
      Actor &a = g->actors[actors[i]];
      df_status st = ensure_dpd_scratch(g, a, n_firings[i]);
      if (st) return st;
      if ((st = dpd_enqueue(g, a, n_firings[i]))) return st;
    }
    return DF_OK;
  }
  if (M != 4 && M != 8 && M != 16) return fail(g, DF_EINVAL, "persistent batching supports n_taps 4, 8, 16");

  Persistent *p = g->pers;
  const bool same_list = p && p->actors.size() == (size_t)n_actors &&
                         std::equal(p->actors.begin(), p->actors.end(), actors);
  if (!same_list) {
    destroy_persistent(g);
    p = g->pers = new Persistent();
    p->actors.assign(actors, actors + n_actors);
    p->M = M;
    p->Bg = Bg;
    HIPCHK(g, hipDeviceGetAttribute(&p->ncu, hipDeviceAttributeMultiprocessorCount, g->device));
    HIPCHK(g, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HIPCHK(g, hipMalloc(&p->inst, sizeof(InstDesc) * n_actors));
    HIPCHK(g, hipMalloc(&p->n_dev, sizeof(int64_t) * n_actors));
    HIPCHK(g, hipMalloc(&p->fire_base, sizeof(int64_t) * (n_actors + 1)));
    HIPCHK(g, hipMalloc(&p->tile_base, sizeof(int64_t) * (n_actors + 1)));
    HIPCHK(g, hipMalloc(&p->last_all, sizeof(int64_t) * n_actors * Bg));
    HIPCHK(g, hipMalloc(&p->queue, sizeof(int32_t) * 64));
    HIPCHK(g, hipMalloc(&p->inst_order, sizeof(int32_t) * n_actors));
  }
  // Tile configuration: a multiple of 64*K outputs, no larger than needed.
  const int K = g->outputs_per_thread == 8 ? 8 : 4;
  int tile = g->tile > 0 ? g->tile : 1024;
  const int64_t rr = ((max_r + 64 * K - 1) / (64 * K)) * (64 * K);
  if (tile > rr) tile = (int)rr;
  tile = std::max(64 * K, std::min(512 * K, (tile / (64 * K)) * (64 * K)));
  // one history sample per thread
  while (tile / K < 512 && tile / K < Bg * (M - 1)) tile += 64 * K;
  const int bpc = g->blocks_per_cu > 0 ? g->blocks_per_cu : 4;
  bool rebuild = !same_list || tile != p->tile || K != p->K || bpc != p->bpc;
  if (total > p->cap) {
    HIPCHK(g, hipStreamSynchronize(g->stream));
    int64_t cap = 1024;
    while (cap < total) cap <<= 1;
    (void)hipFree(p->B_all);
    (void)hipFree(p->prev_all);
    p->B_all = nullptr;
    p->prev_all = nullptr;
    HIPCHK(g, hipMalloc(&p->B_all, sizeof(int32_t) * cap));
    HIPCHK(g, hipMalloc(&p->prev_all, sizeof(int64_t) * cap * Bg));
    p->cap = cap;
    rebuild = true;
  }
  if (rebuild) {
    HIPCHK(g, hipStreamSynchronize(g->stream));
    drop_graph(p);
    p->tile = tile;
    p->K = K;
    p->bpc = bpc;
    std::vector<InstDesc> desc(n_actors);
    for (int i = 0; i < n_actors; ++i) {
      Actor &a = g->actors[actors[i]];
      Fifo &fc = g->fifos[a.ports[DF_DPD_CTRL]];
      Fifo &fx = g->fifos[a.ports[DF_DPD_IN]];
      Fifo &fy = g->fifos[a.ports[DF_DPD_OUT]];
      InstDesc d{};
      d.x = (const float2 *)fx.ring;
      d.x_idx = fx.idx;
      d.x_mask = fx.mask;
      d.y = (float2 *)fy.ring;
      d.y_idx = fy.idx;
      d.y_mask = fy.mask;
      d.ctrl = (const int32_t *)fc.ring;
      d.ctrl_idx = fc.idx;
      d.ctrl_mask = fc.mask;
      d.h = a.h;
      d.hist = a.hist;
      d.r = a.dp.firing_size;
      d.B_max = a.dp.n_branches_max;
      d.hist_mode = a.dp.history_mode;
      d.tpf = (int32_t)((d.r + tile - 1) / tile);
      desc[i] = d;
    }
    HIPCHK(g, hipMemcpy(p->inst, desc.data(), sizeof(InstDesc) * n_actors, hipMemcpyHostToDevice));
    p->n_host.clear();
  }
  if (p->n_host.size() != (size_t)n_actors || !std::equal(p->n_host.begin(), p->n_host.end(), n_firings)) {
    // Counts changed: upload synchronously (the batch shape is normally stable).
    HIPCHK(g, hipStreamSynchronize(g->stream));
    HIPCHK(g, hipMemcpy(p->n_dev, n_firings, sizeof(int64_t) * n_actors, hipMemcpyHostToDevice));
    p->n_host.assign(n_firings, n_firings + n_actors);
  }
  PersArgs pa{};
  pa.inst = p->inst;
  pa.n_inst = n_actors;
  pa.Bg = p->Bg;
  pa.n_fire = p->n_dev;
  pa.fire_base = p->fire_base;
  pa.tile_base = p->tile_base;
  pa.B_all = p->B_all;
  pa.prev_all = p->prev_all;
  pa.last_all = p->last_all;
  pa.cap = p->cap;
  pa.queue = p->queue;
  pa.inst_order = p->inst_order;
  pa.err = g->err_dev;
  pa.tile = p->tile;
  if (flags & DF_FIRE_GRAPH) {
    if (!p->exec) {
      HIPCHK(g, hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue_chain(p, pa, p->cap_stream, nullptr);
      hipGraph_t graph = nullptr;
      hipError_t e2 = hipStreamEndCapture(p->cap_stream, &graph);
      if (e != hipSuccess) return fail_hip(g, e, "capture of the persistent chain");
      if (e2 != hipSuccess) return fail_hip(g, e2, "hipStreamEndCapture");
      p->graph = graph;
      HIPCHK(g, hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    }
    HIPCHK(g, prof_begin(g));
    HIPCHK(g, hipGraphLaunch(p->exec, g->stream));
    HIPCHK(g, prof_end(g));
  } else {
    HIPCHK(g, enqueue_chain(p, pa, g->stream, g));
  }
  for (int i = 0; i < n_actors; ++i) {
    Actor &a = g->actors[actors[i]];
    const int64_t n = n_firings[i], r = a.dp.firing_size;
    g->fifos[a.ports[DF_DPD_CTRL]].read_h += n;
    g->fifos[a.ports[DF_DPD_IN]].read_h += n * r;
    g->fifos[a.ports[DF_DPD_OUT]].write_lo += n * r;
    g->fifos[a.ports[DF_DPD_OUT]].write_hi += n * r;
    a.fired += n;
    a.last_n = 0;
  }
  return DF_OK;
}
