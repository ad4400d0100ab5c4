// Bodies of the static frame actors of the paper's motion-detection
// pipeline (Sec. 4.1): Gauss (5x5 binomial filter, two top and two bottom
// rows unfiltered), Thres (consecutive-frame difference against a fixed
// threshold) and Med (5-pixel median).  Each batch covers n_frames
// consecutive tokens of the actor's channels; see MdpArgs.
//
// Word path (width a multiple of 4): a work item is one 4-pixel word column
// of kRun consecutive output rows of one frame; consecutive lanes take
// consecutive columns, so every row load of a wave is one contiguous run of
// words.  The vertical window slides down the item in registers; the two
// neighbouring words give the horizontal halo, with the nearest in-frame
// pixel replicated at the left and right frame edges.  Pixels are processed
// four per word in 16-bit lanes (md_swar.h).  Any other width takes the byte
// path: one thread per pixel.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "common.h"
#include "md_swar.h"

namespace dfh {
namespace {

constexpr int kMdThreads = 256;
constexpr int kRun = 16;                   // output rows per word-path work item
constexpr int64_t kMaxBlocks = 1 << 23;    // per launch: threads stay below 2^31

__device__ inline const uint8_t *in_frame(const uint8_t *ring, const int64_t *idx, int64_t mask, int64_t f,
                                          int64_t WH) {
  return ring + ((idx[0] + f) & mask) * WH;
}

__device__ inline uint8_t *out_frame(uint8_t *ring, const int64_t *idx, int64_t mask, int64_t f, int64_t WH) {
  return ring + ((idx[1] + f) & mask) * WH;
}

// Word column `cx` of row `row` with its left and right neighbour words; at
// a frame edge the missing neighbour repeats the edge pixel.
struct Nbr {
  uint32_t l, m, r;
};

__device__ inline Nbr load_nbr(const uint32_t *row, int cx, int Wq) {
  Nbr n;
  n.m = row[cx];
  n.l = cx > 0 ? row[cx - 1] : (n.m & 0xFFu) * 0x01010101u;
  n.r = cx < Wq - 1 ? row[cx + 1] : (n.m >> 24) * 0x01010101u;
  return n;
}

// ------------------------------------------------------------------ Gauss

__global__ __launch_bounds__(kMdThreads) void k_gauss5_w(MdpArgs a, int64_t f0, int32_t n_runs, int32_t bpf) {
  const int64_t f = f0 + blockIdx.x / (uint32_t)bpf;
  const int32_t local = (int32_t)(blockIdx.x % (uint32_t)bpf) * kMdThreads + (int32_t)threadIdx.x;
  const int32_t Wq = a.W >> 2;
  const int32_t cx = local % Wq, run = local / Wq;
  if (run >= n_runs) return;
  const int64_t WH = (int64_t)a.W * a.H;
  const uint32_t *src = (const uint32_t *)in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH);
  uint32_t *dst = (uint32_t *)out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH);
  uint32_t *dst2 = a.out1 ? (uint32_t *)out_frame(a.out1, a.out1_idx, a.out1_mask, f, WH) : nullptr;
  const int H = a.H;
  const int y0 = run * kRun;
  const int yend = min(y0 + kRun, H);
  uint32_t he[5] = {0, 0, 0, 0, 0}, ho[5] = {0, 0, 0, 0, 0}, mid[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int r = 0; r < kRun + 4; ++r) {
    const int yy = min(max(y0 - 2 + r, 0), H - 1);
    const Nbr n = load_nbr(src + (int64_t)yy * Wq, cx, Wq);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      he[k] = he[k + 1];
      ho[k] = ho[k + 1];
      mid[k] = mid[k + 1];
    }
    // window bytes (p-2, p-1, p0, p1 | p2, p3, p4, p5)
    swar::hsum5(swar::funnel(n.m, n.l, 16), swar::funnel(n.r, n.m, 16), &he[4], &ho[4]);
    mid[4] = n.m;
    if (r >= 4) {
      const int y = y0 + r - 4;
      if (y < yend) {
        uint32_t v = mid[2];
        if (y >= 2 && y < H - 2)
          v = swar::interleave(swar::vround5(he[0], he[1], he[2], he[3], he[4]),
                               swar::vround5(ho[0], ho[1], ho[2], ho[3], ho[4]));
        const int64_t o = (int64_t)y * Wq + cx;
        __builtin_nontemporal_store(v, dst + o);
        if (dst2) __builtin_nontemporal_store(v, dst2 + o);
      }
    }
  }
}

__global__ __launch_bounds__(kMdThreads) void k_gauss5_b(MdpArgs a, int64_t f0, int32_t bpf) {
  const int64_t f = f0 + blockIdx.x / (uint32_t)bpf;
  const int64_t i = (int64_t)(blockIdx.x % (uint32_t)bpf) * kMdThreads + threadIdx.x;
  const int64_t WH = (int64_t)a.W * a.H;
  if (i >= WH) return;
  const uint8_t *src = in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH);
  const int W = a.W, H = a.H;
  const int y = (int)(i / W), x = (int)(i % W);
  uint32_t v = src[i];
  if (y >= 2 && y < H - 2) {
    const uint32_t w[5] = {1, 4, 6, 4, 1};
    uint32_t s = 128;
    for (int dy = 0; dy < 5; ++dy) {
      const uint8_t *row = src + (int64_t)(y + dy - 2) * W;
      for (int dx = 0; dx < 5; ++dx) s += w[dy] * w[dx] * row[min(max(x + dx - 2, 0), W - 1)];
    }
    v = s >> 8;
  }
  out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH)[i] = (uint8_t)v;
  if (a.out1) out_frame(a.out1, a.out1_idx, a.out1_mask, f, WH)[i] = (uint8_t)v;
}

// ------------------------------------------------------------------ Thres

__global__ __launch_bounds__(kMdThreads) void k_thres_v(MdpArgs a, int64_t f0, int32_t bpf) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const int64_t f = f0 + blockIdx.x / (uint32_t)bpf;
  const int64_t q = (int64_t)(blockIdx.x % (uint32_t)bpf) * kMdThreads + threadIdx.x;
  const int64_t WH = (int64_t)a.W * a.H;
  if (q >= WH / 16) return;
  const u32x4 c = __builtin_nontemporal_load((const u32x4 *)in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH) + q);
  const u32x4 p = __builtin_nontemporal_load((const u32x4 *)in_frame(a.in1, a.in1_idx, a.in1_mask, f, WH) + q);
  const uint32_t t = (uint32_t)a.thr;
  u32x4 o;
  o.x = swar::absdiff_gt(c.x, p.x, t);
  o.y = swar::absdiff_gt(c.y, p.y, t);
  o.z = swar::absdiff_gt(c.z, p.z, t);
  o.w = swar::absdiff_gt(c.w, p.w, t);
  __builtin_nontemporal_store(o, (u32x4 *)out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH) + q);
}

__global__ __launch_bounds__(kMdThreads) void k_thres_b(MdpArgs a, int64_t f0, int32_t bpf) {
  const int64_t f = f0 + blockIdx.x / (uint32_t)bpf;
  const int64_t i = (int64_t)(blockIdx.x % (uint32_t)bpf) * kMdThreads + threadIdx.x;
  const int64_t WH = (int64_t)a.W * a.H;
  if (i >= WH) return;
  const int c = in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH)[i];
  const int p = in_frame(a.in1, a.in1_idx, a.in1_mask, f, WH)[i];
  const int d = c > p ? c - p : p - c;
  out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH)[i] = d > a.thr ? 255 : 0;
}

// ------------------------------------------------------------------ Med

__global__ __launch_bounds__(kMdThreads) void k_med5_w(MdpArgs a, int64_t f0, int32_t n_runs, int32_t bpf) {
  const int64_t f = f0 + blockIdx.x / (uint32_t)bpf;
  const int32_t local = (int32_t)(blockIdx.x % (uint32_t)bpf) * kMdThreads + (int32_t)threadIdx.x;
  const int32_t Wq = a.W >> 2;
  const int32_t cx = local % Wq, run = local / Wq;
  if (run >= n_runs) return;
  const int64_t WH = (int64_t)a.W * a.H;
  const uint32_t *src = (const uint32_t *)in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH);
  uint32_t *dst = (uint32_t *)out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH);
  const int H = a.H;
  const int y0 = run * kRun;
  const int yend = min(y0 + kRun, H);
  uint32_t up = 0, lc = 0, mc = 0, rc = 0;   // row above; centre row and its neighbour words
#pragma unroll
  for (int r = 0; r < kRun + 2; ++r) {
    const int yy = min(max(y0 - 1 + r, 0), H - 1);
    const Nbr n = load_nbr(src + (int64_t)yy * Wq, cx, Wq);
    if (r >= 2) {
      const int y = y0 + r - 2;
      if (y < yend) {
        // left neighbours (p-1, p0, p1, p2), right neighbours (p1, p2, p3, p4)
        const uint32_t L = swar::funnel(mc, lc, 24), R = swar::funnel(rc, mc, 8);
        __builtin_nontemporal_store(swar::med5_bytes(mc, up, n.m, L, R), dst + (int64_t)y * Wq + cx);
      }
    }
    // the current centre row is the row above the next one
    up = mc;
    lc = n.l;
    mc = n.m;
    rc = n.r;
  }
}

__global__ __launch_bounds__(kMdThreads) void k_med5_b(MdpArgs a, int64_t f0, int32_t bpf) {
  const int64_t f = f0 + blockIdx.x / (uint32_t)bpf;
  const int64_t i = (int64_t)(blockIdx.x % (uint32_t)bpf) * kMdThreads + threadIdx.x;
  const int64_t WH = (int64_t)a.W * a.H;
  if (i >= WH) return;
  const uint8_t *src = in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH);
  const int W = a.W, H = a.H;
  const int y = (int)(i / W), x = (int)(i % W);
  const uint32_t c = src[i];
  const uint32_t u = src[(int64_t)max(y - 1, 0) * W + x];
  const uint32_t d = src[(int64_t)min(y + 1, H - 1) * W + x];
  const uint32_t l = src[(int64_t)y * W + max(x - 1, 0)];
  const uint32_t rr = src[(int64_t)y * W + min(x + 1, W - 1)];
  out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH)[i] = (uint8_t)swar::med5_bytes(c, u, d, l, rr);
}

// ------------------------------------------------------------------ launch

// Launch `kern` over all frames in chunks of at most kMaxBlocks workgroups,
// bpf workgroups per frame; timing events bracket the first and last chunk.
template <class K, class... Extra>
hipError_t launch_frames(K kern, const MdpArgs &a, int32_t bpf, hipStream_t s, const KTiming *t, Extra... extra) {
  const int64_t per_launch = kMaxBlocks / bpf > 0 ? kMaxBlocks / bpf : 1;
  for (int64_t f0 = 0; f0 < a.n_frames; f0 += per_launch) {
    const int64_t nf = a.n_frames - f0 < per_launch ? a.n_frames - f0 : per_launch;
    const dim3 grid((unsigned)(nf * bpf));
    const bool first = f0 == 0, last = f0 + per_launch >= a.n_frames;
    if (t && (first || last))
      hipExtLaunchKernelGGL(kern, grid, dim3(kMdThreads), 0, s, first ? t->start : nullptr,
                            last ? t->stop : nullptr, 0, a, f0, extra..., bpf);
    else
      hipLaunchKernelGGL(kern, grid, dim3(kMdThreads), 0, s, a, f0, extra..., bpf);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int32_t div_up32(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

__global__ void k_advance_n(int64_t *p0, int64_t *p1, int64_t *p2, int64_t *p3, int64_t delta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (p0) *p0 += delta;
    if (p1) *p1 += delta;
    if (p2) *p2 += delta;
    if (p3) *p3 += delta;
  }
}

}  // namespace

hipError_t launch_gauss5(const MdpArgs &a, hipStream_t s, const KTiming *t) {
  if (a.n_frames <= 0) return hipSuccess;
  if (a.W % 4 == 0) {
    const int32_t n_runs = div_up32(a.H, kRun);
    return launch_frames(k_gauss5_w, a, div_up32((int64_t)n_runs * (a.W / 4), kMdThreads), s, t, n_runs);
  }
  return launch_frames(k_gauss5_b, a, div_up32((int64_t)a.W * a.H, kMdThreads), s, t);
}

hipError_t launch_thres(const MdpArgs &a, hipStream_t s, const KTiming *t) {
  if (a.n_frames <= 0) return hipSuccess;
  const int64_t WH = (int64_t)a.W * a.H;
  if (WH % 16 == 0) return launch_frames(k_thres_v, a, div_up32(WH / 16, kMdThreads), s, t);
  return launch_frames(k_thres_b, a, div_up32(WH, kMdThreads), s, t);
}

hipError_t launch_med5(const MdpArgs &a, hipStream_t s, const KTiming *t) {
  if (a.n_frames <= 0) return hipSuccess;
  if (a.W % 4 == 0) {
    const int32_t n_runs = div_up32(a.H, kRun);
    return launch_frames(k_med5_w, a, div_up32((int64_t)n_runs * (a.W / 4), kMdThreads), s, t, n_runs);
  }
  return launch_frames(k_med5_b, a, div_up32((int64_t)a.W * a.H, kMdThreads), s, t);
}

hipError_t launch_advance_n(int64_t *const *ptr, int n, int64_t delta, hipStream_t s) {
  if (n < 1 || n > 4) return hipErrorInvalidValue;
  int64_t *p[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int i = 0; i < n; ++i) p[i] = ptr[i];
  hipLaunchKernelGGL(k_advance_n, dim3(1), dim3(64), 0, s, p[0], p[1], p[2], p[3], delta);
  return hipGetLastError();
}

}  // namespace dfh
