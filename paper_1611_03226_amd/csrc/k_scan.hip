// Control intake, rate resolution and offset scan for a batch of firings.
//
// Sec. 2.2: a dynamic actor first consumes one control token, which fixes
// the rate (0 or r) of each regular port for that firing.  For the
// predistortion actor the token B activates branches b < B.  From the
// per-firing rates this pass derives, for every branch b:
//   off_b(j)  = r * #{i < j : firing i feeds branch b}   (exclusive sum)
//   prev_b(j) = max{i < j : firing i feeds branch b}     (exclusive max, -1 none)
//   last_b    = max{i < n : firing i feeds branch b}
// where "feeds" is B_i > b (branch history) or always (shared history).
//
// One workgroup per segment of firings, which it walks in chunks of one
// firing per thread.  Per chunk and branch, a wavefront ballot of the feed
// flags gives the in-wavefront exclusive count (popcount of the bits below
// the lane) and last feeder (highest bit below the lane); the per-wavefront
// totals become exclusive prefixes in LDS, and the segment carries (count
// and last feeder so far) advance once per chunk.
#include "common.h"

namespace dfh {

constexpr int kScanThreads = 1024;
constexpr int kScanWaves = kScanThreads / 64;

__global__ __launch_bounds__(kScanThreads) void k_scan(ScanArgs a) {
  __shared__ int wsum[kScanWaves][kMaxBranches], wlast[kScanWaves][kMaxBranches];
  __shared__ int64_t carry_cnt[kMaxBranches], carry_last[kMaxBranches], chunk_cnt[kMaxBranches];
  __shared__ int chunk_last[kMaxBranches];
  const int seg = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int64_t R = a.ctrl_idx ? a.ctrl_idx[0] : 0;
  const int64_t g0 = (int64_t)seg * a.seg_firings;
  const uint64_t below_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  if (tid < a.B_max) carry_cnt[tid] = 0, carry_last[tid] = -1;
  for (int64_t c0 = 0; c0 < a.seg_firings; c0 += blockDim.x) {
    const int64_t j = c0 + tid;                       // segment-local firing
    const bool in = j < a.seg_firings;
    int Bv = 0;
    if (in) {
      Bv = a.ctrl[(R + g0 + j) & a.ctrl_mask];
      if (Bv < 0 || Bv > a.B_max) {
        if (a.err) atomicOr(a.err, (int32_t)kErrControl);
        Bv = 0;
      }
      a.B_out[g0 + j] = Bv;
    }
    // wavefront totals
    for (int b = 0; b < a.B_max; ++b) {
      const uint64_t bal = __ballot(in && (a.hist_mode == 1 || Bv > b));
      if (lane == 0) {
        wsum[wave][b] = __popcll(bal);
        wlast[wave][b] = bal ? 64 * wave + 63 - __clzll((long long)bal) : -1;
      }
    }
    __syncthreads();
    // per branch: totals over the chunk into the carries, and the
    // per-wavefront totals turned into exclusive prefixes (in place)
    if (tid < a.B_max) {
      int64_t cnt = 0;
      int wl = -1;
      for (int w = 0; w < nw; ++w) {
        const int s_ = wsum[w][tid], l_ = wlast[w][tid];
        wsum[w][tid] = (int)cnt;
        wlast[w][tid] = wl;
        cnt += s_;
        wl = max(wl, l_);
      }
      chunk_cnt[tid] = cnt;
      chunk_last[tid] = wl;
    }
    __syncthreads();
    for (int b = 0; b < a.B_max; ++b) {
      const uint64_t bal = __ballot(in && (a.hist_mode == 1 || Bv > b));
      const uint64_t below = bal & below_mask;
      const int64_t cnt = carry_cnt[b] + wsum[wave][b] + __popcll(below);
      const int wl = below ? 64 * wave + 63 - __clzll((long long)below) : wlast[wave][b];
      const int64_t last = wl >= 0 ? c0 + wl : carry_last[b];
      if (in) {
        const int64_t o = (int64_t)b * a.stride + g0 + j;
        a.prev_out[o] = last >= 0 ? g0 + last : -1;
        if (a.off_out) a.off_out[o] = a.r * cnt;
      }
    }
    __syncthreads();
    if (tid < a.B_max) {
      carry_cnt[tid] += chunk_cnt[tid];
      if (chunk_last[tid] >= 0) carry_last[tid] = c0 + chunk_last[tid];
    }
    __syncthreads();
  }
  if (tid < a.B_max && a.last_out)
    a.last_out[(int64_t)seg * a.B_max + tid] = carry_last[tid] >= 0 ? g0 + carry_last[tid] : -1;
}

// Processing order of a batch's firings, grouped by branch count B (largest
// first), as pairs (firing, B).  The body kernels compile one fully unrolled
// code path per B; grouping keeps the workgroups resident on a compute unit
// on one or two paths, so their instructions stay cached.  The order inside
// a group is irrelevant to the results (every firing's outputs are
// independent).
__global__ __launch_bounds__(1024) void k_order_by_b(const int32_t *B, int64_t n, int32_t B_max, int32_t *order) {
  __shared__ int32_t hist[kMaxBranches + 1], cursor[kMaxBranches + 1];
  if (threadIdx.x <= kMaxBranches) hist[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) atomicAdd(&hist[B[j]], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int v = B_max; v >= 0; --v) {
      cursor[v] = run;
      run += hist[v];
    }
  }
  __syncthreads();
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const int v = B[j];
    const int k = atomicAdd(&cursor[v], 1);
    order[2 * k] = (int32_t)j;
    order[2 * k + 1] = v;
  }
}

hipError_t launch_order_by_b(const int32_t *B, int64_t n, int32_t B_max, int32_t *order, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_order_by_b, dim3(1), dim3(1024), 0, s, B, n, B_max, order);
  return hipGetLastError();
}

int64_t resident_blocks(const void *kernel, int threads, size_t lds_bytes) {
  struct Entry {
    const void *k;
    int threads, dev;
    size_t lds;
    int64_t n;
  };
  static Entry cache[64];
  static int used = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  for (int i = 0; i < used; ++i)
    if (cache[i].k == kernel && cache[i].threads == threads && cache[i].lds == lds_bytes && cache[i].dev == dev)
      return cache[i].n;
  int per_cu = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds_bytes) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 1;
  const int64_t n = (int64_t)per_cu * ncu;
  if (used < 64) cache[used++] = Entry{kernel, threads, dev, lds_bytes, n};
  return n;
}

hipError_t launch_scan(const ScanArgs &a, hipStream_t s) {
  if (a.n_segs <= 0 || a.seg_firings <= 0) return hipSuccess;
  if (a.B_max < 1 || a.B_max > kMaxBranches) return hipErrorInvalidValue;
  // one firing per thread; small segments take fewer wavefronts
  int64_t waves = (a.seg_firings + 63) / 64;
  if (waves > kScanWaves) waves = kScanWaves;
  hipLaunchKernelGGL(k_scan, dim3(a.n_segs), dim3(64 * (unsigned)waves), 0, s, a);
  return hipGetLastError();
}

}  // namespace dfh
