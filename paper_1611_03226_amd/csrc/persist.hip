// Many predistortion instances fired as one batch.
//
// Every instance is an independent actor with its own channels, coefficients
// and control tokens; a batch fires instance i n_i times.  The chain is
//   scan:     per instance: its firing and head-pass bases (sums of n_k over
//             the instances before it), control intake and branch offset
//             scan
//   order:    instances grouped by branch count, work-item bases in that order
//   heads + items (one launch): head corrections of every firing, and one
//             descriptor per (instance, firing, tile) work item in
//             processing order
//   body:     a persistent grid walking the work items with a grid stride
//   commit:   per-instance channel indices and carried branch histories
// (five kernels: every kernel boundary costs a few microseconds.  Folding
// the order into the scan's last workgroup was measured slower: each
// workgroup then has to publish its tables with a device-scope release,
// an L2 write-back here, and 1024 of those cost more than one boundary.)
// All counts live in device memory, so the chain can be captured once in a
// HIP graph and replayed.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
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
  int32_t ctrl_mode;      // kCtrlCount or kCtrlMask
};

// Work-item descriptor (what the body needs about one tile).
struct PItem {
  const float2 *x;
  float2 *y;
  const float2 *h;
  const float2 *corr;     // head corrections of the firing [M-1]
  int64_t x_mask, y_mask;
  int64_t xb, yb;         // ring positions of the firing's first input / output sample
  int32_t t0, nout;
  uint32_t set;           // the firing's branch set
  int32_t head;
};

static_assert(sizeof(PItem) % 4 == 0 && sizeof(PItem) / 4 <= 64, "descriptor fits one register");

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
  PItem *items;           // [items_cap]
  float2 *corr_all;       // [cap][M-1] head corrections
  int64_t *head_base;     // [n_inst + 1] first head-pass wavefront of each instance
  int32_t *head_inst;     // [heads] instance of each head-pass wavefront (4 firings each)
  int32_t M;
  int32_t *err;
  int32_t tile;
  int32_t masked;         // some instance reads bit-mask control tokens
};

// Processing order of the instances, grouped by the Horner length of their
// first firing's branch set (largest first), and the work-item bases in that
// order.  The
// body compiles one unrolled code path per branch count; grouping keeps the
// workgroups resident on a compute unit on few paths (instruction cache).
// The order never changes a result.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_pers_order(PersArgs a) {
  __shared__ int32_t hist[kMaxBranches + 1], cursor[kMaxBranches + 1];
  __shared__ int64_t wsum[16];
  if (threadIdx.x <= kMaxBranches) hist[threadIdx.x] = 0;
  __syncthreads();
  auto key = [&](int i) { return a.n_fire[i] > 0 ? set_len((uint32_t)a.B_all[a.fire_base[i]]) : 0; };
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

// Branch b's part of instance i's scan (one wavefront).
__device__ void pers_scan_branch(const PersArgs &a, const InstDesc &d, int i, int b, int64_t n, int64_t base,
                                 int64_t hbase) {
  const int lane = threadIdx.x & 63;
  const int64_t R = d.ctrl_idx[0];
  const uint64_t below_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  int64_t lastw = -1;
  for (int64_t c = 0; c < n; c += 64) {
    const int64_t j = c + lane;
    const bool in = j < n;
    uint32_t set = 0u;
    if (in) {
      bool bad;
      set = token_set(d.ctrl[(R + j) & d.ctrl_mask], d.ctrl_mode, d.B_max, &bad);
      if (bad && b == 0) atomicOr(a.err, (int32_t)kErrControl);
      if (b == 0) a.B_all[base + j] = (int32_t)set;
    }
    const bool fed = in && (d.hist_mode == 1 || in_set(set, b));
    const uint64_t bal = __ballot(fed);
    const uint64_t below = bal & below_mask;
    if (in) a.prev_all[(int64_t)b * a.cap + base + j] = below ? (c + 63 - __clzll((long long)below)) : lastw;
    if (bal) lastw = c + 63 - __clzll((long long)bal);
  }
  if (lane == 0) a.last_all[(int64_t)i * a.Bg + b] = lastw;
  if (b == 0)
    for (int64_t k = lane; k < (n + 3) / 4; k += 64) a.head_inst[hbase + k] = i;
}

// One workgroup per instance, one wavefront per branch (as the single-actor
// scan): validated control tokens, history source firings, last feeders.
// The workgroup first sums the firing counts of the instances before it
// (its firing base, and its first head-pass wavefront: four firings each).
__global__ __launch_bounds__(1024) void k_pers_scan(PersArgs a) {
  __shared__ int64_t part[2][16];
  const int i = blockIdx.x;
  const int b = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int lane = threadIdx.x & 63;
  const InstDesc &d = a.inst[i];
  int64_t sf = 0, sh = 0;
  for (int k = threadIdx.x; k < i; k += blockDim.x) {
    const int64_t nf = a.n_fire[k];
    sf += nf;
    sh += (nf + 3) / 4;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sf += __shfl_xor(sf, o), sh += __shfl_xor(sh, o);
  if (lane == 0) part[0][b] = sf, part[1][b] = sh;
  __syncthreads();
  int64_t base = 0, hbase = 0;
  for (int w = 0; w < nw; ++w) base += part[0][w], hbase += part[1][w];
  const int64_t n = a.n_fire[i];
  if (threadIdx.x == 0) {
    a.fire_base[i] = base;
    a.head_base[i] = hbase;
    if (i == a.n_inst - 1) {
      a.fire_base[a.n_inst] = base + n;
      a.head_base[a.n_inst] = hbase + (n + 3) / 4;
    }
  }
  if (b < d.B_max) pers_scan_branch(a, d, i, b, n, base, hbase);
}

// Work-item descriptors: item k (processing order) -> the last ordered
// instance whose tile base is <= k, its firing and tile.  Workgroup blk of
// nblk (256 threads each) strides over the items.
__device__ __forceinline__ void pers_items(const PersArgs &a, int64_t blk, int64_t nblk) {
  const int64_t total = a.tile_base[a.n_inst];
  for (int64_t it = blk * 256 + threadIdx.x; it < total; it += nblk * 256) {
    int lo = 0, hi = a.n_inst - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.tile_base[mid] <= it) lo = mid; else hi = mid - 1;
    }
    const int i = a.inst_order[lo];
    const InstDesc &d = a.inst[i];
    const int64_t local = it - a.tile_base[lo];
    const int64_t j = local / d.tpf;
    const int64_t t0 = (local - j * d.tpf) * a.tile;
    const int64_t gf = a.fire_base[i] + j;
    const uint32_t set = (uint32_t)a.B_all[gf];
    const int64_t Rx = d.x_idx[0];
    PItem p;
    p.x = d.x;
    p.y = d.y;
    p.h = d.h;
    p.corr = a.corr_all + gf * (a.M - 1);
    p.x_mask = d.x_mask;
    p.y_mask = d.y_mask;
    p.xb = Rx + j * d.r;
    p.yb = d.y_idx[1] + j * d.r;
    p.t0 = (int32_t)t0;
    p.nout = (int32_t)min((int64_t)a.tile, d.r - t0);
    p.set = set;
    p.head = (t0 == 0 && set != 0u) ? 1 : 0;
    a.items[it] = p;
  }
}

// Tile descriptors of the persistent batch: the work-item table.
struct ItemSrc {
  const PersArgs &a;
  static constexpr int kWords = (int)(sizeof(PItem) / 4);
  __device__ uint32_t fetch(int64_t it) const {
    const int lane = threadIdx.x & 63;
    return lane < kWords ? reinterpret_cast<const uint32_t *>(a.items + it)[lane] : 0u;
  }
  __device__ void expand(uint32_t dv, int64_t, Job &j) const {
    j.x = (const float2 *)qword_at(dv, offsetof(PItem, x) / 4);
    j.y = (float2 *)qword_at(dv, offsetof(PItem, y) / 4);
    j.h = (const float2 *)qword_at(dv, offsetof(PItem, h) / 4);
    j.corr = (const float2 *)qword_at(dv, offsetof(PItem, corr) / 4);
    j.x_mask = (int64_t)qword_at(dv, offsetof(PItem, x_mask) / 4);
    j.y_mask = (int64_t)qword_at(dv, offsetof(PItem, y_mask) / 4);
    j.xb = (int64_t)qword_at(dv, offsetof(PItem, xb) / 4);
    j.yb = (int64_t)qword_at(dv, offsetof(PItem, yb) / 4);
    j.t0 = (int)dword_at(dv, offsetof(PItem, t0) / 4);
    j.nout = (int)dword_at(dv, offsetof(PItem, nout) / 4);
    j.set = dword_at(dv, offsetof(PItem, set) / 4);
    j.B = set_len(j.set);
    j.head = (int)dword_at(dv, offsetof(PItem, head) / 4);
  }
};

// Head corrections of all instances' firings: one wavefront per four
// consecutive firings of one instance (rows), from the head-pass map.  The
// number of such wavefronts is read from the device (head_base[n_inst],
// written by the scan), and a fixed grid walks them with a stride, so the
// launch does not depend on the batch's firing counts.  The first
// head_blocks workgroups do that; the others write the work items.
template <int M>
__device__ __forceinline__ void pers_head(const PersArgs &a, int64_t w);

template <int M>
__global__ __launch_bounds__(256) void k_pers_heads_items(PersArgs a, int head_blocks) {
  if ((int)blockIdx.x >= head_blocks) {
    pers_items(a, blockIdx.x - head_blocks, gridDim.x - head_blocks);
    return;
  }
  const int64_t n_heads = as_const(a.head_base)[a.n_inst];
  const int64_t stride = (int64_t)head_blocks * 4;
  for (int64_t w = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); w < n_heads;
       w += stride)                                   // uniform per wavefront
    pers_head<M>(a, w);
}

template <int M>
__device__ __forceinline__ void pers_head(const PersArgs &a, int64_t w) {
  const int i = as_const(a.head_inst)[w];
  const auto *inst = as_const(a.inst) + i;
  const int64_t j0 = 4 * (w - as_const(a.head_base)[i]);
  const int64_t nf = as_const(a.n_fire)[i];
  const int64_t f0 = as_const(a.fire_base)[i] + j0;   // global firing of row 0
  const float2 *x = inst->x;
  const float2 *hist = inst->hist;
  const int64_t x_mask = inst->x_mask, r = inst->r;
  const int64_t Rx = as_const(inst->x_idx)[0];
  const auto B_of = [&](int row) { return j0 + row < nf ? (uint32_t)a.B_all[f0 + row] : 0u; };
  float cr = 0.f, ci = 0.f;
  head_correction<M, 4>(
      as_const(inst->h), B_of, [&](int row, int b) { return a.prev_all[(int64_t)b * a.cap + f0 + row]; },
      [&](int, int b, int64_t pf, int q) {
        if (pf >= 0) return x[(Rx + pf * r + r - (M - 1) + q) & x_mask];
        return hist[b * (M - 1) + q];
      },
      0, 1, [&](int, bool on, float sr, float si) {
        if (on) {
          cr += sr;
          ci += si;
        }
      });
  const int lane = threadIdx.x & 63, row = lane >> 4, q = lane & 15;
  if (head_live<M, 4>(B_of(row))) a.corr_all[(f0 + row) * (M - 1) + q] = make_float2(cr, ci);
}

// Persistent body: a grid-stride walk over the work items (run_tiles).
template <int M, int K, int BC, bool MASKED>
__global__ __launch_bounds__(512) void k_pers_body(PersArgs a) {
  extern __shared__ float2 lds[];   // [M-1] head corrections, window
  float2 *sc = lds, *sx = sc + lds_corr(M);
  ItemSrc src{a};
  run_tiles<M, K, BC, MASKED>(sx, sc, as_const(a.tile_base)[a.n_inst], src);
}

// The same walk with matrix-core tiles (M = 16).
template <int K, int BC, bool MASKED>
__global__ __launch_bounds__(512) void k_pers_body_mx(PersArgs a) {
  extern __shared__ float2 lds[];   // [15] head corrections, window, 4 row-sum rows, coefficients
  float2 *sc = lds, *sx = sc + lds_corr(16), *rb = sx + mx_window(a.tile), *sh = rb + 4 * mx_row(a.tile);
  ItemSrc src{a};
  run_tiles_mx<K, BC, MASKED>(sx, sc, rb, sh, as_const(a.tile_base)[a.n_inst], src);
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
    check_chan(d.x_idx, a.err);
    check_chan(d.ctrl_idx, a.err);
    check_chan(d.y_idx, a.err);
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
  float2 *corr_all = nullptr;
  int32_t *B_all = nullptr, *inst_order = nullptr;
  PItem *items = nullptr;
  int64_t *head_base = nullptr;
  int32_t *head_inst = nullptr;
  int64_t cap = 0, items_cap = 0, heads_cap = 0, n_heads = 0;
  int64_t captures = 0;   // graph captures so far (diagnostics)
  int tile = 0, K = 0, bpc = 0, ncu = 0;
  bool mx = false;         // M = 16 bodies on the matrix cores
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
  (void)hipFree(p->corr_all);
  (void)hipFree(p->last_all);
  (void)hipFree(p->B_all);
  (void)hipFree(p->items);
  (void)hipFree(p->head_base);
  (void)hipFree(p->head_inst);
  (void)hipFree(p->inst_order);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
  g->pers = nullptr;
}

template <int M, int K, int BC, bool MASKED>
static hipError_t launch_pers_body(const PersArgs &a, int threads, int blocks, hipStream_t s, const KTiming *t) {
  const size_t lds = (size_t)(lds_window(a.tile + M - 1) + lds_corr(M)) * sizeof(float2);
  if (t)
    hipExtLaunchKernelGGL((k_pers_body<M, K, BC, MASKED>), dim3(blocks), dim3(threads), lds, s, t->start, t->stop, 0, a);
  else
    hipLaunchKernelGGL((k_pers_body<M, K, BC, MASKED>), dim3(blocks), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <int K, int BC, bool MASKED>
static hipError_t launch_pers_body_mx(const PersArgs &a, int threads, int blocks, hipStream_t s, const KTiming *t) {
  const size_t lds = (size_t)mx_lds(a.tile) * sizeof(float2);
  if (t)
    hipExtLaunchKernelGGL((k_pers_body_mx<K, BC, MASKED>), dim3(blocks), dim3(threads), lds, s, t->start, t->stop, 0, a);
  else
    hipLaunchKernelGGL((k_pers_body_mx<K, BC, MASKED>), dim3(blocks), dim3(threads), lds, s, a);
  return hipGetLastError();
}

static hipError_t enqueue_chain(Persistent *p, const PersArgs &a, hipStream_t s, df_graph *prof_g) {
  hipLaunchKernelGGL(k_pers_scan, dim3(a.n_inst), dim3(64 * a.Bg), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pers_order, dim3(1), dim3(1024), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  {
    // head pass: a grid that covers the head-pass capacity in one sweep, at
    // most a few workgroups per compute unit (it strides over the device
    // count); work items: four workgroups per compute unit
    const int64_t want = (p->heads_cap + 3) / 4;
    const int hb = (int)std::max<int64_t>(1, std::min<int64_t>(want, 8 * p->ncu));
    const dim3 grid((unsigned)(hb + 4 * p->ncu));
    if (p->M == 16) hipLaunchKernelGGL(k_pers_heads_items<16>, grid, dim3(256), 0, s, a, hb);
    else if (p->M == 8) hipLaunchKernelGGL(k_pers_heads_items<8>, grid, dim3(256), 0, s, a, hb);
    else hipLaunchKernelGGL(k_pers_heads_items<4>, grid, dim3(256), 0, s, a, hb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int threads = p->tile / p->K;
  const int blocks = p->bpc * p->ncu;
  KTiming kt;
  if (prof_g && (e = prof_pair(prof_g, &kt)) != hipSuccess) return e;
  const KTiming *tp = (prof_g && prof_g->prof) ? &kt : nullptr;
  const bool small = a.Bg <= 10;
#define DF_PERS_MX(k)                                                                              \
  if (p->K == k)                                                                                   \
    e = a.masked ? launch_pers_body_mx<k, 16, true>(a, threads, blocks, s, tp)                    \
        : (small ? launch_pers_body_mx<k, 10, false>(a, threads, blocks, s, tp)                    \
                 : launch_pers_body_mx<k, 16, false>(a, threads, blocks, s, tp));               \
  else
#define DF_PERS(m, k)                                                                              \
  if (p->M == m && p->K == k)                                                                      \
    e = a.masked ? launch_pers_body<m, k, 16, true>(a, threads, blocks, s, tp)                    \
        : (small ? launch_pers_body<m, k, 10, false>(a, threads, blocks, s, tp)                    \
                 : launch_pers_body<m, k, 16, false>(a, threads, blocks, s, tp));               \
  else
  if (p->M == 16 && p->mx) {
    DF_PERS_MX(4) DF_PERS_MX(8) return hipErrorInvalidValue;
  } else {
    DF_PERS(16, 4) DF_PERS(16, 8) DF_PERS(8, 4) DF_PERS(8, 8) DF_PERS(4, 4) DF_PERS(4, 8)
    return hipErrorInvalidValue;
  }
#undef DF_PERS
#undef DF_PERS_MX
  if (e != hipSuccess) return e;
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

static df_status fire_many(df_graph *g, int32_t n_actors, const int32_t *actors, const int64_t *n_firings,
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
      if ((st = dpd_enqueue(g, a, n_firings[i], false))) return st;
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
    p->mx = g->body_mx;
    p->Bg = Bg;
    HIPCHK(g, hipDeviceGetAttribute(&p->ncu, hipDeviceAttributeMultiprocessorCount, g->device));
    HIPCHK(g, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HIPCHK(g, hipMalloc(&p->inst, sizeof(InstDesc) * n_actors));
    HIPCHK(g, hipMalloc(&p->n_dev, sizeof(int64_t) * n_actors));
    HIPCHK(g, hipMalloc(&p->fire_base, sizeof(int64_t) * (n_actors + 1)));
    HIPCHK(g, hipMalloc(&p->tile_base, sizeof(int64_t) * (n_actors + 1)));
    HIPCHK(g, hipMalloc(&p->last_all, sizeof(int64_t) * n_actors * Bg));
    HIPCHK(g, hipMalloc(&p->inst_order, sizeof(int32_t) * n_actors));
    HIPCHK(g, hipMalloc(&p->head_base, sizeof(int64_t) * (n_actors + 1)));
  }
  // Tile configuration: a multiple of 64*K outputs, no larger than needed.
  const int K = g->outputs_per_thread == 8 ? 8 : 4;
  int tile = g->tile > 0 ? g->tile : 1024;
  const int64_t rr = ((max_r + 64 * K - 1) / (64 * K)) * (64 * K);
  if (tile > rr) tile = (int)rr;
  tile = std::max(64 * K, std::min(512 * K, (tile / (64 * K)) * (64 * K)));
  const int bpc = g->blocks_per_cu > 0 ? g->blocks_per_cu : 4;
  bool rebuild = !same_list || tile != p->tile || K != p->K || bpc != p->bpc;
  if (total > p->cap) {
    HIPCHK(g, hipStreamSynchronize(g->stream));
    int64_t cap = 1024;
    while (cap < total) cap <<= 1;
    (void)hipFree(p->B_all);
    (void)hipFree(p->prev_all);
    (void)hipFree(p->corr_all);
    p->B_all = nullptr;
    p->prev_all = nullptr;
    p->corr_all = nullptr;
    HIPCHK(g, hipMalloc(&p->B_all, sizeof(int32_t) * cap));
    HIPCHK(g, hipMalloc(&p->prev_all, sizeof(int64_t) * cap * Bg));
    HIPCHK(g, hipMalloc(&p->corr_all, sizeof(float2) * cap * (M - 1)));
    p->cap = cap;
    rebuild = true;
  }
  int64_t n_items = 0;
  for (int i = 0; i < n_actors; ++i) {
    const int64_t r = g->actors[actors[i]].dp.firing_size;
    n_items += n_firings[i] * ((r + tile - 1) / tile);
  }
  if (n_items > p->items_cap) {
    HIPCHK(g, hipStreamSynchronize(g->stream));
    int64_t cap = 1024;
    while (cap < n_items) cap <<= 1;
    (void)hipFree(p->items);
    p->items = nullptr;
    HIPCHK(g, hipMalloc(&p->items, sizeof(PItem) * cap));
    p->items_cap = cap;
    rebuild = true;
  }
  int64_t n_heads = 0;
  for (int i = 0; i < n_actors; ++i) n_heads += (n_firings[i] + 3) / 4;
  if (n_heads > p->heads_cap) {
    HIPCHK(g, hipStreamSynchronize(g->stream));
    int64_t cap = 1024;
    while (cap < n_heads) cap <<= 1;
    (void)hipFree(p->head_inst);
    p->head_inst = nullptr;
    HIPCHK(g, hipMalloc(&p->head_inst, sizeof(int32_t) * cap));
    p->heads_cap = cap;
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
      d.ctrl_mode = a.dp.control_mode;
      d.tpf = (int32_t)((d.r + tile - 1) / tile);
      desc[i] = d;
    }
    HIPCHK(g, hipMemcpy(p->inst, desc.data(), sizeof(InstDesc) * n_actors, hipMemcpyHostToDevice));
    p->n_host.clear();
  }
  if (p->n_host.size() != (size_t)n_actors || !std::equal(p->n_host.begin(), p->n_host.end(), n_firings)) {
    // Counts changed: every kernel of the chain reads them from the device
    // (grids are sized by the capacities above), so a stream-ordered upload
    // is all it takes; a captured graph stays valid.  The copy is from
    // pageable memory, so n_firings may be reused once this call returns.
    HIPCHK(g, hipMemcpyAsync(p->n_dev, n_firings, sizeof(int64_t) * n_actors, hipMemcpyHostToDevice, g->stream));
    p->n_host.assign(n_firings, n_firings + n_actors);
    p->n_heads = n_heads;
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
  pa.items = p->items;
  pa.corr_all = p->corr_all;
  pa.head_base = p->head_base;
  pa.head_inst = p->head_inst;
  pa.M = p->M;
  pa.inst_order = p->inst_order;
  pa.err = g->err_dev;
  pa.tile = p->tile;
  pa.masked = 0;
  for (int i = 0; i < n_actors; ++i)
    if (g->actors[actors[i]].dp.control_mode == DF_CTRL_MASK) pa.masked = 1;
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
      ++p->captures;
      dlog(g, 1, "persistent chain captured (capture %lld)", (long long)p->captures);
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

extern "C" df_status df_fire_many(df_graph *g, int32_t n_actors, const int32_t *actors, const int64_t *n_firings,
                                  int flags) {
  df_status st = fire_many(g, n_actors, actors, n_firings, flags);
  if (st == DF_OK) dlog(g, 1, "df_fire_many %d actors flags 0x%x", n_actors, flags);
  return g && !g->poisoned ? after_call(g, st) : st;
}
