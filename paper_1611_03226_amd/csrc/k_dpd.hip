// Predistortion actor body and batch commit.
//
// Actor body (Sec. 4.2: a polynomial actor feeding parallel FIR filters
// whose active set a configuration actor selects, summed by an adder):
//   y[t] = sum_{b<B} sum_{m<M} h[b][m] * psi_b(s_b[t-m]),  psi_b(x) = |x|^(2b) x.
// Inside a firing every active branch reads the same samples, so the sum is
// evaluated per tap as a polynomial in p = |x|^2 (Horner over branches):
//   y[t] = sum_m x[t-m] * P_m(p[t-m]),   P_m(p) = sum_{b<B} h[b][m] p^b.
// Only the first M-1 outputs of a firing reach back into branch histories,
// which differ per branch (history source firing prev_b(g), or carried
// state); those terms are added by a per-branch correction.
#include <hip/hip_ext.h>

#include <cstdlib>
#include <cstring>

#include "common.h"
#include "dpd_tile.h"
#include "scan_dev.h"

namespace dfh {

__device__ __forceinline__ int64_t prev_of(const DpdArgs &a, int b, int64_t g) {
  if (a.prev) return a.prev[(int64_t)b * a.prev_stride + g];
  return (g % a.seg_firings) ? g - 1 : -1;
}

// Input sample at offset ii (< 0) before the start of firing g, as branch b
// sees it: tail of its history firing, carried state, or zero.
__device__ __forceinline__ float2 hist_sample(const DpdArgs &a, int64_t Rx, int b, int64_t g,
                                              int64_t pf, int64_t ii) {
  if (pf >= 0) return a.x[(Rx + pf * a.r + a.r + ii) & a.x_mask];
  if (a.hist) return a.hist[b * (a.M - 1) + (a.M - 1) + ii];
  return make_float2(0.f, 0.f);
}

// ------------------------------------------------------------------ generic
// One thread per output sample, direct form with per-branch sources.  Any
// B_max <= 16 and M <= 32.
__global__ __launch_bounds__(256) void k_dpd_generic(DpdArgs a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.n_firings * a.r) return;
  const int64_t g = t / a.r;
  const int64_t i = t - g * a.r;
  const uint32_t set = a.B ? (uint32_t)a.B[g] : prefix_set(a.B_const);
  const int64_t Rx = a.x_idx ? a.x_idx[0] : 0;
  const int64_t Wy = a.y_idx ? a.y_idx[1] : 0;
  float ar = 0.f, ai = 0.f;
  for (int b = 0; b < kMaxBranches; ++b) {
    if (!in_set(set, b)) continue;
    const int64_t pf = (i < a.M - 1) ? prev_of(a, b, g) : -1;
    for (int m = 0; m < a.M; ++m) {
      const int64_t ii = i - m;
      const float2 xv = ii >= 0 ? a.x[(Rx + g * a.r + ii) & a.x_mask]
                                : hist_sample(a, Rx, b, g, pf, ii);
      const float p = xv.x * xv.x + xv.y * xv.y;
      float pb = 1.f;
      for (int k = 0; k < b; ++k) pb *= p;
      const float sr = pb * xv.x, si = pb * xv.y;
      const float2 c = a.h[b * a.M + m];
      ar += c.x * sr - c.y * si;
      ai += c.x * si + c.y * sr;
    }
  }
  a.y[(Wy + t) & a.y_mask] = make_float2(ar, ai);
}

// ------------------------------------------------------------------ commit
// Advance the channel indices by the batch's token counts and carry each
// branch's history: the last M-1 input samples of its last feeding firing.
// One workgroup (a kernel of its own, or the body's last workgroup).
__device__ __forceinline__ void dpd_commit_block(const DpdCommitArgs &a) {
  const int64_t Rx = a.x_idx[0];
  __syncthreads();
  const int L = a.M - 1;
  for (int t = threadIdx.x; t < a.B_max * L; t += blockDim.x) {
    const int b = t / L, k = t - b * L;
    const int64_t lf = a.last[b];
    if (lf >= 0) a.hist[b * L + k] = a.x[(Rx + lf * a.r + a.r - L + k) & a.x_mask];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.x_idx[0] = Rx + a.n_firings * a.r;
    a.ctrl_idx[0] += a.n_firings;
    a.y_idx[1] += a.n_firings * a.r;
    check_chan(a.x_idx, a.err);
    check_chan(a.ctrl_idx, a.err);
    check_chan(a.y_idx, a.err);
  }
}

// ------------------------------------------------------------------ heads
// Head corrections of every firing with B > 0 (four firings per
// wavefront); corr[g][q], q < M-1.  Read by the tiled body.  With a group
// table (one segment) the wavefront also derives the history sources of its
// four firings and writes their prev/off table entries: the four firings lie
// in one 64-firing group, so a ballot of the group's feed flags per branch
// plus the group's entry (count and last feeder before it) gives them;
// with order_out it also writes the four firings' processing slots.
template <int M, bool TABLES>
__global__ __launch_bounds__(256) void k_dpd_heads(DpdArgs a) {
  // The workgroup's four wavefronts share four firings; wavefront w takes
  // branches w, w+4, w+8, w+12 (more wavefronts in flight, a quarter of the
  // serial work each); each branch's sum goes to LDS and one wavefront adds
  // them in increasing branch order, as a single pass would.
  __shared__ float2 part[kMaxBranches][64];
  if constexpr (TABLES) {
    if ((int)blockIdx.x < a.ahead_blocks) {          // the next batch's scan (whole workgroups)
      scan_dev::scan_group(a.ahead, (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
                           (a.ahead.seg_firings + 63) / 64);
      return;
    }
  }
  const int64_t hb = (int64_t)blockIdx.x - a.ahead_blocks;
  if (a.err_ahead && hb == 0 && threadIdx.x == 0) {
    const int32_t e = *a.err_ahead;
    if (e) {
      if (a.err) atomicOr(a.err, e);
      *a.err_ahead = 0;
    }
  }
  const int64_t g0 = hb * 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t Rx = a.x_idx ? as_const(a.x_idx)[0] : 0;
  const int lane = threadIdx.x & 63, row = lane >> 4, i = lane & 15;
  const int64_t g = g0 + row;                         // this lane's firing
  int64_t pf[kMaxBranches];
  if constexpr (TABLES) {
    const int64_t G = g0 >> 6;
    const int64_t gl = G * 64 + lane;                 // lane's firing of the group
    const bool gin = gl < a.n_firings;
    const uint32_t Bl = gin ? (a.B ? (uint32_t)a.B[gl] : prefix_set(a.B_const)) : 0u;
    const uint64_t below_mask = (1ull << ((g0 & 63) + row)) - 1;
#pragma unroll
    for (int b = 0; b < kMaxBranches; ++b) {
      pf[b] = -1;
      if (b >= a.B_max || (b & 3) != w) continue;     // uniform
      const uint64_t bal = __ballot(gin && (a.hist_mode == 1 || in_set(Bl, b)));
      const int64_t gi = 2 * (G * a.B_max + b);
      const int64_t cnt0 = as_const(a.grp)[gi], last0 = as_const(a.grp)[gi + 1];
      const uint64_t below = bal & below_mask;
      pf[b] = below ? G * 64 + 63 - __clzll((long long)below) : last0;
      if (i == b && g < a.n_firings) {
        const int64_t o = (int64_t)b * a.prev_stride + g;
        a.tab_prev[o] = pf[b];
        if (a.tab_off) a.tab_off[o] = a.r * (cnt0 + __popcll(below));
      }
    }
    if (a.order_out && w == 0) {
      // processing slot of each of the four firings: its length's first
      // slot in this group plus the firings of that length before it here
      const int NV = a.B_max + 1;
      const int Ll = gin ? set_len(Bl) : -1;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int lq = (int)(g0 & 63) + q;            // group lane of firing g0 + q
        if (g0 + q >= a.n_firings) break;             // uniform
        const uint32_t Sq = (uint32_t)__builtin_amdgcn_readlane((int)Bl, lq);
        const int Lq = set_len(Sq);
        const uint64_t bal = __ballot(Ll == Lq);
        if (lane == q) {
          const int64_t k = as_const(a.obase)[G * NV + Lq] + __popcll(bal & ((1ull << lq) - 1));
          a.order_out[2 * k] = (int32_t)(g0 + q);
          a.order_out[2 * k + 1] = (int32_t)Sq;
        }
      }
    }
  }
  const auto B_of = [&](int r) {
    const int64_t gr = g0 + r;
    return gr < a.n_firings ? (a.B ? (uint32_t)a.B[gr] : prefix_set(a.B_const)) : 0u;
  };
  head_correction<M, 4>(
      as_const(a.h), B_of,
      [&](int r, int b) {
        if constexpr (TABLES) return pf[b];              // this lane's row
        else return prev_of(a, b, g0 + r);
      },
      [&](int r, int b, int64_t p, int q) { return hist_sample(a, Rx, b, g0 + r, p, (int64_t)q - (M - 1)); },
      w, 4, [&](int b, bool, float sr, float si) { part[b][lane] = make_float2(sr, si); });
  __syncthreads();
  const uint32_t set = B_of(row);
  if (w == 0 && head_live<M, 4>(set)) {
    float cr = 0.f, ci = 0.f;
    for (int b = 0; b < kMaxBranches; ++b)
      if (in_set(set, b)) {
        cr += part[b][lane].x;
        ci += part[b][lane].y;
      }
    a.corr[g * (M - 1) + i] = make_float2(cr, ci);
  }
}

// ------------------------------------------------------------------ tiled
// Tile descriptors of a single actor's batch: tile k is tile k % tpf of the
// (k / tpf)-th firing in processing order (pairs (firing, branch set) from
// the scan, or firing order).
struct SingleSrc {
  const DpdArgs &a;
  int64_t Rx, Wy;
  __device__ uint32_t fetch(int64_t it) const {
    const int lane = threadIdx.x & 63;
    const int64_t k = it / a.tiles_per_firing;
    if (a.order) return lane < 2 ? (uint32_t)a.order[2 * k + lane] : 0u;
    if (lane == 0) return (uint32_t)k;
    if (lane == 1) return a.B ? (uint32_t)a.B[k] : prefix_set(a.B_const);
    return 0u;
  }
  __device__ void expand(uint32_t dv, int64_t it, Job &j) const {
    const int64_t k = it / a.tiles_per_firing;
    const int64_t tk = it - k * a.tiles_per_firing;
    const int64_t g = dword_at(dv, 0);
    const uint32_t set = dword_at(dv, 1);
    j.x = a.x;
    j.y = a.y;
    j.h = a.h;
    j.corr = a.corr + g * (a.M - 1);
    j.x_mask = a.x_mask;
    j.y_mask = a.y_mask;
    j.xb = Rx + g * a.r;
    j.yb = Wy + g * a.r;
    j.t0 = (int)(tk * a.tile);
    j.nout = (int)min((int64_t)a.tile, a.r - j.t0);
    j.set = set;
    j.B = set_len(set);
    j.head = (j.t0 == 0 && set != 0u) ? 1 : 0;
  }
};

// Grid-stride loop over the batch's tiles in the length-grouped firing order,
// pipelined as run_tiles describes.
template <int M, int K, int BC, bool MASKED>
__global__ __launch_bounds__(256) void k_dpd_tiled(DpdArgs a) {
  extern __shared__ float2 lds[];   // [M-1] head corrections, window
  float2 *sc = lds, *sx = sc + lds_corr(M);
  SingleSrc src{a, a.x_idx ? as_const(a.x_idx)[0] : 0, a.y_idx ? as_const(a.y_idx)[1] : 0};
  run_tiles<M, K, BC, MASKED>(sx, sc, a.n_firings * a.tiles_per_firing, src);
  if (!a.ticket) return;
  // The last workgroup to finish commits the batch: every other workgroup
  // has read the channel indices by then (it read them before finishing),
  // and the commit reads nothing another workgroup wrote, so a relaxed
  // counter suffices (a device-scope fence here would write back the L2).
  __shared__ int last_block;
  __syncthreads();
  if (threadIdx.x == 0)
    last_block = __hip_atomic_fetch_add(a.ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                 (int)gridDim.x - 1;
  __syncthreads();
  if (last_block) {
    dpd_commit_block(a.commit);
    if (threadIdx.x == 0) *a.ticket = 0;              // ready for the next batch
  }
}

// The same loop with matrix-core tiles (M = 16).
template <int K, int BC, bool MASKED>
__global__ __launch_bounds__(256) void k_dpd_tiled_mx(DpdArgs a) {
  extern __shared__ float2 lds[];   // [15] head corrections, window, 4 row-sum rows, coefficients
  float2 *sc = lds, *sx = sc + lds_corr(16), *rb = sx + mx_window(a.tile), *sh = rb + 4 * mx_row(a.tile);
  SingleSrc src{a, a.x_idx ? as_const(a.x_idx)[0] : 0, a.y_idx ? as_const(a.y_idx)[1] : 0};
  run_tiles_mx<K, BC, MASKED>(sx, sc, rb, sh, a.n_firings * a.tiles_per_firing, src);
  if (!a.ticket) return;
  __shared__ int last_block;                         // commit by the last workgroup, as above
  __syncthreads();
  if (threadIdx.x == 0)
    last_block = __hip_atomic_fetch_add(a.ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                 (int)gridDim.x - 1;
  __syncthreads();
  if (last_block) {
    dpd_commit_block(a.commit);
    if (threadIdx.x == 0) *a.ticket = 0;
  }
}

template <int K, int BC, bool MASKED>
static hipError_t launch_tiled_mx(const DpdArgs &a0, hipStream_t s, int tile, const KTiming *t) {
  DpdArgs a = a0;
  a.tile = tile;
  a.tiles_per_firing = (int32_t)((a.r + tile - 1) / tile);
  const int threads = tile / K;
  const size_t lds = (size_t)mx_lds(tile) * sizeof(float2);
  const int64_t items = a.n_firings * a.tiles_per_firing;
  if (items <= 0) return hipSuccess;
  const int64_t resident = resident_blocks((const void *)k_dpd_tiled_mx<K, BC, MASKED>, threads, lds);
  const int64_t blocks = items < resident ? items : resident;
  if (t)
    hipExtLaunchKernelGGL((k_dpd_tiled_mx<K, BC, MASKED>), dim3((unsigned)blocks), dim3(threads), lds, s, t->start,
                          t->stop, 0, a);
  else
    hipLaunchKernelGGL((k_dpd_tiled_mx<K, BC, MASKED>), dim3((unsigned)blocks), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <int M, int K, int BC, bool MASKED>
static hipError_t launch_tiled(const DpdArgs &a0, hipStream_t s, int tile, const KTiming *t) {
  DpdArgs a = a0;
  a.tile = tile;
  a.tiles_per_firing = (int32_t)((a.r + tile - 1) / tile);
  const int threads = tile / K;
  const size_t lds = (size_t)(lds_window(tile + M - 1) + lds_corr(M)) * sizeof(float2);
  const int64_t items = a.n_firings * a.tiles_per_firing;
  if (items <= 0) return hipSuccess;
  const int64_t resident = resident_blocks((const void *)k_dpd_tiled<M, K, BC, MASKED>, threads, lds);
  const int64_t blocks = items < resident ? items : resident;
  if (t)
    hipExtLaunchKernelGGL((k_dpd_tiled<M, K, BC, MASKED>), dim3((unsigned)blocks), dim3(threads), lds, s, t->start, t->stop,
                          0, a);
  else
    hipLaunchKernelGGL((k_dpd_tiled<M, K, BC, MASKED>), dim3((unsigned)blocks), dim3(threads), lds, s, a);
  return hipGetLastError();
}

bool dpd_tiled_shape(int M) { return M == 4 || M == 8 || M == 16; }

bool dpd_body_mx_env() {
  const char *v = getenv("DFHIP_BODY");
  return v && strcmp(v, "mx") == 0;
}

hipError_t launch_dpd_heads(const DpdArgs &a, hipStream_t s) {
  if (a.n_firings <= 0 || !dpd_tiled_shape(a.M)) return hipSuccess;
  if (!a.corr) return hipErrorInvalidValue;
  if (a.grp && (a.seg_firings != a.n_firings || !a.tab_prev)) return hipErrorInvalidValue;
  if (a.ahead_blocks < 0 || (a.ahead_blocks && (!a.grp || a.ahead.n_segs != 1 || !a.ahead.grp || !a.ahead.ticket ||
                                               a.ahead_blocks != (scan_groups(1, a.ahead.seg_firings) + 3) / 4)))
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)((a.n_firings + 3) / 4 + a.ahead_blocks));
#define DF_HEADS(m)                                                                     \
  if (a.M == m) {                                                                       \
    if (a.grp)                                                                          \
      hipLaunchKernelGGL((k_dpd_heads<m, true>), grid, dim3(256), 0, s, a);             \
    else                                                                                \
      hipLaunchKernelGGL((k_dpd_heads<m, false>), grid, dim3(256), 0, s, a);            \
  }
  DF_HEADS(16) else DF_HEADS(8) else DF_HEADS(4)
#undef DF_HEADS
  return hipGetLastError();
}

hipError_t launch_dpd_body(const DpdArgs &a, hipStream_t s, int tile, int outputs_per_thread, const KTiming *t) {
  if (a.n_firings <= 0) return hipSuccess;
  if (!dpd_tiled_shape(a.M)) {
    const int64_t total = a.n_firings * a.r;
    const dim3 grid((unsigned)((total + 255) / 256));
    if (t)
      hipExtLaunchKernelGGL(k_dpd_generic, grid, dim3(256), 0, s, t->start, t->stop, 0, a);
    else
      hipLaunchKernelGGL(k_dpd_generic, grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (!a.corr) return hipErrorInvalidValue;          // launch_dpd_heads fills it first
  // Tile: a multiple of 64*K outputs, at most 256 threads, no larger than
  // needed for one firing.
  const int K = outputs_per_thread == 8 ? 8 : 4;
  int tl = tile > 0 ? tile : 1024;
  const int64_t rr = ((a.r + 64 * K - 1) / (64 * K)) * (64 * K);
  if ((int64_t)tl > rr) tl = (int)rr;
  tl = (tl / (64 * K)) * (64 * K);
  if (tl < 64 * K) tl = 64 * K;
  if (tl / K > 256) tl = 256 * K;
  // compiled paths: Horner lengths up to 10 or up to 16; branch sets that are
  // not prefixes (bit-mask tokens) take the masked paths up to 16
  const bool small = a.B_max <= 10;
  if (a.M == 16 && a.mx) {
    if (K == 4)
      return a.masked ? launch_tiled_mx<4, 16, true>(a, s, tl, t)
                      : (small ? launch_tiled_mx<4, 10, false>(a, s, tl, t) : launch_tiled_mx<4, 16, false>(a, s, tl, t));
    return a.masked ? launch_tiled_mx<8, 16, true>(a, s, tl, t)
                    : (small ? launch_tiled_mx<8, 10, false>(a, s, tl, t) : launch_tiled_mx<8, 16, false>(a, s, tl, t));
  }
#define DF_TILED(m, k)                                                                      \
  if (a.M == m && K == k)                                                                   \
    return a.masked ? launch_tiled<m, k, 16, true>(a, s, tl, t)                             \
                    : (small ? launch_tiled<m, k, 10, false>(a, s, tl, t) : launch_tiled<m, k, 16, false>(a, s, tl, t));
  DF_TILED(16, 4) DF_TILED(16, 8) DF_TILED(8, 4) DF_TILED(8, 8) DF_TILED(4, 4) DF_TILED(4, 8)
#undef DF_TILED
  return hipErrorInvalidValue;
}

__global__ __launch_bounds__(1024) void k_dpd_commit(DpdCommitArgs a) { dpd_commit_block(a); }

hipError_t launch_dpd_commit(const DpdCommitArgs &a, hipStream_t s) {
  int threads = a.B_max * (a.M - 1);
  threads = threads < 64 ? 64 : (threads > 1024 ? 1024 : ((threads + 63) / 64) * 64);
  hipLaunchKernelGGL(k_dpd_commit, dim3(1), dim3(threads), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ small helpers
__global__ void k_advance(int64_t *idx, int64_t delta, int32_t *err) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    idx[0] += delta;
    check_chan(chan_slot(idx), err);
  }
}

hipError_t launch_advance(int64_t *idx, int64_t delta, int32_t *err, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, idx, delta, err);
  return hipGetLastError();
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace dfh
