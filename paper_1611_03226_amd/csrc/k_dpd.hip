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
#include "common.h"
#include "dpd_tile.h"

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
  const int B = a.B ? a.B[g] : a.B_const;
  const int64_t Rx = a.x_idx ? a.x_idx[0] : 0;
  const int64_t Wy = a.y_idx ? a.y_idx[1] : 0;
  float ar = 0.f, ai = 0.f;
  for (int b = 0; b < B; ++b) {
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

// ------------------------------------------------------------------ tiled
// Grid-stride loop over the batch's tiles (in the B-grouped firing order);
// each workgroup prefetches its next tile while computing the current one.
template <int M, int K>
__global__ __launch_bounds__(256) void k_dpd_tiled(DpdArgs a) {
  extern __shared__ float2 lds[];   // [2*B_max*(M-1)] histories, window
  float2 *sq = lds, *sx = sq + lds_history(a.B_max, M);
  const cfloat2p hg = as_const(a.h);
  const int64_t n_items = a.n_firings * a.tiles_per_firing;
  int64_t item = blockIdx.x;
  if (item >= n_items) return;                       // uniform
  const int64_t Rx = a.x_idx ? a.x_idx[0] : 0;
  const int64_t Wy = a.y_idx ? a.y_idx[1] : 0;
  auto job_of = [&](int64_t it, int64_t &g) {
    const int64_t k = it / a.tiles_per_firing;
    const int64_t tk = it - k * a.tiles_per_firing;
    g = a.order ? a.order[k] : k;
    TileJob j;
    j.t0 = tk * a.tile;
    j.nout = (int)min((int64_t)a.tile, a.r - j.t0);
    j.B = a.B ? a.B[g] : a.B_const;
    j.head = j.t0 == 0 && j.B > 0 && M > 1;
    j.xb = Rx + g * a.r;
    j.yb = Wy + g * a.r;
    return j;
  };
  int64_t g;
  TileJob job = job_of(item, g);
  TileRegs<M, K> regs;
  tile_prefetch<M, K>(regs, job, a.x, a.x_mask,
                      [&](int b, int64_t ii) { return hist_sample(a, Rx, b, g, prev_of(a, b, g), ii); });
  for (;;) {
    tile_commit<M, K>(sx, sq, regs, job);
    __syncthreads();
    const int64_t next = item + gridDim.x;
    int64_t ng = 0;
    TileJob nj = job;
    if (next < n_items) {
      nj = job_of(next, ng);
      tile_prefetch<M, K>(regs, nj, a.x, a.x_mask,
                          [&](int b, int64_t ii) { return hist_sample(a, Rx, b, ng, prev_of(a, b, ng), ii); });
    }
    if (job.head) {
      tile_head_sums<M>(sq, hg, job.B);
      __syncthreads();
    }
    tile_outputs<M, K>(sx, hg, sq, job, a.y, a.y_mask);
    if (next >= n_items) break;
    __syncthreads();
    item = next;
    job = nj;
    g = ng;
  }
}

template <int M, int K>
static hipError_t launch_tiled(const DpdArgs &a0, hipStream_t s, int tile) {
  DpdArgs a = a0;
  a.tile = tile;
  a.tiles_per_firing = (int32_t)((a.r + tile - 1) / tile);
  const int threads = tile / K;
  const size_t lds = (size_t)(lds_window(tile + M - 1) + lds_history(a.B_max, M)) * sizeof(float2);
  const int64_t items = a.n_firings * a.tiles_per_firing;
  if (items <= 0) return hipSuccess;
  const int64_t resident = resident_blocks((const void *)k_dpd_tiled<M, K>, threads, lds);
  const int64_t blocks = items < resident ? items : resident;
  hipLaunchKernelGGL((k_dpd_tiled<M, K>), dim3((unsigned)blocks), dim3(threads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_dpd_body(const DpdArgs &a, hipStream_t s, int tile, int outputs_per_thread) {
  if (a.n_firings <= 0) return hipSuccess;
  // Tile: a multiple of 64*K outputs, at most 256 threads, no larger than
  // needed for one firing.
  const int K = outputs_per_thread == 8 ? 8 : 4;
  int t = tile > 0 ? tile : 1024;
  const int64_t rr = ((a.r + 64 * K - 1) / (64 * K)) * (64 * K);
  if ((int64_t)t > rr) t = (int)rr;
  t = (t / (64 * K)) * (64 * K);
  if (t < 64 * K) t = 64 * K;
  if (t / K > 256) t = 256 * K;
  // the history prefetch gives each thread one sample: B_max*(M-1) <= threads
  const int need = a.B_max * (a.M - 1);
  while (t / K < need && t / K < 256) t += 64 * K;
  if (t / K < need) {
    const int64_t total = a.n_firings * a.r;
    hipLaunchKernelGGL(k_dpd_generic, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (a.M == 16 && K == 4) return launch_tiled<16, 4>(a, s, t);
  if (a.M == 16 && K == 8) return launch_tiled<16, 8>(a, s, t);
  if (a.M == 8 && K == 4) return launch_tiled<8, 4>(a, s, t);
  if (a.M == 8 && K == 8) return launch_tiled<8, 8>(a, s, t);
  if (a.M == 4 && K == 4) return launch_tiled<4, 4>(a, s, t);
  if (a.M == 4 && K == 8) return launch_tiled<4, 8>(a, s, t);
  const int64_t total = a.n_firings * a.r;
  hipLaunchKernelGGL(k_dpd_generic, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ commit
// Advance the channel indices by the batch's token counts and carry each
// branch's history: the last M-1 input samples of its last feeding firing.
__global__ __launch_bounds__(1024) void k_dpd_commit(DpdCommitArgs a) {
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
  }
}

hipError_t launch_dpd_commit(const DpdCommitArgs &a, hipStream_t s) {
  int threads = a.B_max * (a.M - 1);
  threads = threads < 64 ? 64 : (threads > 1024 ? 1024 : ((threads + 63) / 64) * 64);
  hipLaunchKernelGGL(k_dpd_commit, dim3(1), dim3(threads), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ small helpers
__global__ void k_advance(int64_t *idx, int64_t delta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) idx[0] += delta;
}

hipError_t launch_advance(int64_t *idx, int64_t delta, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, idx, delta);
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
