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
// One workgroup per segment of firings, one wavefront per branch.  A
// 0/1 feed flag per lane makes both scans a ballot: the exclusive count is
// the popcount of the ballot bits below the lane, the exclusive max is the
// highest such bit, carried across 64-firing chunks.
#include "common.h"

namespace dfh {

__global__ __launch_bounds__(1024) void k_scan(ScanArgs a) {
  const int seg = blockIdx.x;
  const int b = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t R = a.ctrl_idx ? a.ctrl_idx[0] : 0;
  const int64_t g0 = (int64_t)seg * a.seg_firings;
  const uint64_t below_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  int64_t count = 0;
  int64_t lastw = -1;
  for (int64_t c = 0; c < a.seg_firings; c += 64) {
    const int64_t j = c + lane;
    const bool in = j < a.seg_firings;
    int32_t B = 0;
    if (in) {
      int32_t v = a.ctrl[(R + g0 + j) & a.ctrl_mask];
      if (v < 0 || v > a.B_max) {
        if (b == 0 && a.err) atomicOr(a.err, (int32_t)kErrControl);
        v = 0;
      }
      B = v;
      if (b == 0) a.B_out[g0 + j] = B;
    }
    const bool fed = in && (a.hist_mode == 1 || B > b);
    const uint64_t bal = __ballot(fed);
    const uint64_t below = bal & below_mask;
    if (in) {
      const int64_t pv = below ? (c + 63 - __clzll((long long)below)) : lastw;
      a.prev_out[(int64_t)b * a.stride + g0 + j] = pv >= 0 ? g0 + pv : -1;
      if (a.off_out)
        a.off_out[(int64_t)b * a.stride + g0 + j] = a.r * (count + __popcll(below));
    }
    count += __popcll(bal);
    if (bal) lastw = c + 63 - __clzll((long long)bal);
  }
  if (lane == 0 && a.last_out) a.last_out[(int64_t)seg * a.B_max + b] = lastw >= 0 ? g0 + lastw : -1;
}

// Processing order of a batch's firings, grouped by branch count B (largest
// first).  The body kernels compile one fully unrolled code path per B;
// grouping keeps the workgroups resident on a compute unit on one or two
// paths, so their instructions stay cached.  The order inside a group is
// irrelevant to the results (every firing's outputs are independent).
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
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) order[atomicAdd(&cursor[B[j]], 1)] = (int32_t)j;
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
  hipLaunchKernelGGL(k_scan, dim3(a.n_segs), dim3(64 * a.B_max), 0, s, a);
  return hipGetLastError();
}

}  // namespace dfh
