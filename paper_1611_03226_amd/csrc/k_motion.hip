// Motion actor body: frame difference, threshold, 3x3 opening, per-frame
// changed count and data-dependent emission.
//
// Sec. 4.1 subtracts consecutive frames (the previous one arriving over a
// channel with a one-frame initial token) and thresholds against a constant.
// Per firing j:
//   m0 = |cur - prev| > thr
//   e  = AND of m0 over the in-frame 3x3 neighbourhood   (erosion)
//   o  = OR  of e  over the in-frame 3x3 neighbourhood   (dilation)
//   count_j = sum o;  emit_j = 1000*count_j >= permille*W*H
// Emission depends on the whole frame, so the batch runs as
//   count pass -> scan of emit flags -> emit pass (recompute, write emitted
//   masks at their scanned output slots) -> commit of channel indices.
#include "common.h"

namespace dfh {

constexpr int TX = 64;   // tile width (outputs)
constexpr int TY = 16;   // tile height
constexpr int NTH = 256;

__device__ __forceinline__ const uint8_t *frame_ptr(const uint8_t *ring, int64_t pos, int64_t mask,
                                                    int64_t wh) {
  return ring + (pos & mask) * wh;
}

// Opened mask of the tile at (x0, y0) of firing j, left in o[TY][TX].
__device__ __forceinline__ void opened_tile(const MotionArgs &a, int64_t j, int x0, int y0,
                                            uint8_t (&m0)[TY + 4][TX + 4],
                                            uint8_t (&e)[TY + 2][TX + 2],
                                            uint8_t (&o)[TY][TX]) {
  const int64_t wh = (int64_t)a.W * a.H;
  const int64_t Rc = a.cur_idx[0];
  const uint8_t *cur = frame_ptr(a.cur, Rc + j, a.cur_mask, wh);
  const uint8_t *prev;
  if (a.prev) {
    prev = frame_ptr(a.prev, a.prev_idx[0] + j, a.prev_mask, wh);
  } else {
    prev = j == 0 ? a.state : frame_ptr(a.cur, Rc + j - 1, a.cur_mask, wh);
  }
  for (int idx = threadIdx.x; idx < (TY + 4) * (TX + 4); idx += NTH) {
    const int ly = idx / (TX + 4), lx = idx - ly * (TX + 4);
    const int y = y0 - 2 + ly, x = x0 - 2 + lx;
    uint8_t v = 1;                                   // outside: ignored by erosion
    if (y >= 0 && y < a.H && x >= 0 && x < a.W) {
      const int64_t off = (int64_t)y * a.W + x;
      const int d = abs((int)cur[off] - (int)prev[off]);
      v = d > a.thr;
    }
    m0[ly][lx] = v;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < (TY + 2) * (TX + 2); idx += NTH) {
    const int ly = idx / (TX + 2), lx = idx - ly * (TX + 2);
    const int y = y0 - 1 + ly, x = x0 - 1 + lx;
    uint8_t v = 0;                                   // outside: ignored by dilation
    if (y >= 0 && y < a.H && x >= 0 && x < a.W) {
      v = 1;
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) v &= m0[ly + dy][lx + dx];
    }
    e[ly][lx] = v;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < TY * TX; idx += NTH) {
    const int ly = idx / TX, lx = idx - ly * TX;
    uint8_t v = 0;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) v |= e[ly + dy][lx + dx];
    const int y = y0 + ly, x = x0 + lx;
    o[ly][lx] = (y < a.H && x < a.W) ? v : 0;
  }
  __syncthreads();
}

__global__ __launch_bounds__(NTH) void k_motion_count(MotionArgs a) {
  __shared__ uint8_t m0[TY + 4][TX + 4];
  __shared__ uint8_t e[TY + 2][TX + 2];
  __shared__ uint8_t o[TY][TX];
  __shared__ int wsum[NTH / 64];
  const int64_t j = blockIdx.z;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  opened_tile(a, j, x0, y0, m0, e, o);
  int c = 0;
  for (int idx = threadIdx.x; idx < TY * TX; idx += NTH) c += o[idx / TX][idx % TX];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < NTH / 64; ++w) t += wsum[w];
    if (t) atomicAdd(&a.count[j], t);
  }
}

__global__ __launch_bounds__(NTH) void k_motion_emit(MotionArgs a) {
  __shared__ uint8_t m0[TY + 4][TX + 4];
  __shared__ uint8_t e[TY + 2][TX + 2];
  __shared__ uint8_t o[TY][TX];
  const int64_t j = blockIdx.z;
  const int64_t slot = a.emit_off[j];
  if (slot < 0) return;                               // uniform: frame not emitted
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  opened_tile(a, j, x0, y0, m0, e, o);
  const int64_t wh = (int64_t)a.W * a.H;
  uint8_t *dst = a.out + ((a.out_idx[1] + slot) & a.out_mask) * wh;
  for (int idx = threadIdx.x; idx < TY * TX; idx += NTH) {
    const int ly = idx / TX, lx = idx - ly * TX;
    const int y = y0 + ly, x = x0 + lx;
    if (y < a.H && x < a.W) dst[(int64_t)y * a.W + x] = o[ly][lx] ? 255 : 0;
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
    a.index_out[(a.index_idx[1] + slot) & a.index_mask] = a.frame_base + j;
}

// Exclusive scan of emit flags: emit_off[j] = output slot of firing j or -1,
// emit_off[n] = number of emitted frames.  One wavefront, ballot-based.
__global__ __launch_bounds__(64) void k_emit_scan(const int32_t *count, int64_t n, int64_t thresh,
                                                  int64_t *off) {
  const int lane = threadIdx.x;
  const uint64_t below_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  int64_t carry = 0;
  for (int64_t c = 0; c < n; c += 64) {
    const int64_t j = c + lane;
    const bool f = j < n && 1000 * (int64_t)count[j] >= thresh;
    const uint64_t bal = __ballot(f);
    if (j < n) off[j] = f ? carry + __popcll(bal & below_mask) : -1;
    carry += __popcll(bal);
  }
  if (lane == 0) off[n] = carry;
}

__global__ void k_motion_commit(const int64_t *emit_off, int64_t n, int64_t *cur_idx, int64_t *prev_idx,
                                int64_t *out_idx, int64_t *index_idx) {
  if (threadIdx.x != 0) return;
  const int64_t total = emit_off[n];
  cur_idx[0] += n;
  if (prev_idx) prev_idx[0] += n;
  out_idx[1] += total;
  index_idx[1] += total;
}

hipError_t launch_motion_count(const MotionArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  dim3 grid((a.W + TX - 1) / TX, (a.H + TY - 1) / TY, (unsigned)a.n);
  hipLaunchKernelGGL(k_motion_count, grid, dim3(NTH), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_motion_emit_scan(const int32_t *count, int64_t n, int64_t thresh, int64_t *off,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_emit_scan, dim3(1), dim3(64), 0, s, count, n, thresh, off);
  return hipGetLastError();
}

hipError_t launch_motion_emit(const MotionArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  dim3 grid((a.W + TX - 1) / TX, (a.H + TY - 1) / TY, (unsigned)a.n);
  hipLaunchKernelGGL(k_motion_emit, grid, dim3(NTH), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_motion_commit(const int64_t *emit_off, int64_t n, int64_t *cur_idx, int64_t *prev_idx,
                                int64_t *out_idx, int64_t *index_idx, hipStream_t s) {
  hipLaunchKernelGGL(k_motion_commit, dim3(1), dim3(64), 0, s, emit_off, n, cur_idx, prev_idx, out_idx,
                     index_idx);
  return hipGetLastError();
}

}  // namespace dfh
