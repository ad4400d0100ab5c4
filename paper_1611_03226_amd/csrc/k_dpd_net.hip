// The predistortion network of Sec. 4.2 run as the paper draws it: a Poly
// actor P feeding one channel per branch, one FIR actor per branch, and an
// Adder A, each a kernel over a whole batch, with the branch channels
// materialised in device memory at the dynamic rates the control tokens set
// (branch b receives a firing's r samples only when b is in the firing's
// branch set: b < B for a count token, bit b for a mask token).
// Offsets into the branch channels come from the offset scan (k_scan
// tables, or k_mask_tables for bit-mask control tokens, which activate any
// set of branches).  This is the unfused counterpart of the fused body in
// k_dpd.hip, kept to show what the channels cost; it implements branch
// history only (each FIR actor's delay line holds its own last inputs).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "common.h"

namespace dfh {
namespace {

constexpr int kNetThreads = 256;

// The tables hold validated branch sets (from the offset scan, or from
// k_mask_tables for mask tokens).
__device__ inline bool active(int set, int b) { return in_set((uint32_t)set, b); }

// Poly and Adder: a workgroup per (firing, run of 256 V samples of it):
// the firing, its branch set and its channel offsets are uniform over the
// workgroup (scalar loads, no per-thread divisions); V = 2 samples per
// thread (16-byte accesses) when r is even, else 1.
template <int V>
__device__ __forceinline__ bool net_sample(const DpdNetArgs &a, int bpf, int64_t *gg, int64_t *i0) {
  *gg = blockIdx.x / (uint32_t)bpf;
  *i0 = (int64_t)(blockIdx.x - *gg * bpf) * (kNetThreads * V) + (int64_t)threadIdx.x * V;
  return *i0 < a.r;
}

template <int V>
__device__ __forceinline__ void net_load(const float2 *p, float2 (&v)[V]) {
  if constexpr (V == 2) {
    const float4 q = *reinterpret_cast<const float4 *>(p);
    v[0] = make_float2(q.x, q.y);
    v[1] = make_float2(q.z, q.w);
  } else {
    v[0] = *p;
  }
}

template <int V>
__device__ __forceinline__ void net_store(float2 *p, const float2 (&v)[V]) {
  if constexpr (V == 2) *reinterpret_cast<float4 *>(p) = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
  else *p = v[0];
}

// P: for every sample of every firing, psi_b(x) = |x|^(2b) x into channel b
// at the firing's offset, for b < B of the firing.
template <int V>
__global__ __launch_bounds__(kNetThreads) void k_net_poly(DpdNetArgs a, int bpf) {
  int64_t gg, i0;
  if (!net_sample<V>(a, bpf, &gg, &i0)) return;
  const int64_t row_len = a.nf * a.r, s = gg / a.nf;
  const int Bg = a.B[gg];
  float2 v[V];
  net_load<V>(a.x + gg * a.r + i0, v);
  float p[V];
#pragma unroll
  for (int k = 0; k < V; ++k) p[k] = fmaf(v[k].x, v[k].x, v[k].y * v[k].y);
#pragma unroll
  for (int b = 0; b < kMaxBranches; ++b) {
    if (b < a.B_max && active(Bg, b)) net_store<V>(a.chan + (b * a.S + s) * row_len + a.off[b * a.stride + gg] + i0, v);
#pragma unroll
    for (int k = 0; k < V; ++k) v[k] = make_float2(v[k].x * p[k], v[k].y * p[k]);
  }
}

// FIR_b: outputs over the K_b samples channel b received in row s (K_b = r
// times the number of firings with b < B), zero history before the row's
// first sample.  A workgroup takes kFirSpan consecutive outputs (eight per
// thread) and stages their inputs and the M-1 before them in LDS once (one
// global load per sample instead of M).
constexpr int kFirSpan = 8 * kNetThreads;

// MT: the tap count as a compile-time constant (4, 8, 16: coefficients in
// registers, taps unrolled), or 0 for any other count.
template <int MT>
__global__ __launch_bounds__(kNetThreads) void k_net_fir(DpdNetArgs a) {
  __shared__ float2 win[kFirSpan + kMaxTaps - 1];
  const int64_t row_len = a.nf * a.r;
  const int64_t t0 = (int64_t)blockIdx.x * kFirSpan;
  const int64_t bs = blockIdx.y;                      // b * S + s
  const int b = (int)(bs / a.S);
  const int64_t s = bs - (int64_t)b * a.S;
  const int64_t g_last = s * a.nf + a.nf - 1;
  const int64_t K = a.off[b * a.stride + g_last] + (active(a.B[g_last], b) ? a.r : 0);
  if (t0 >= K) return;                                // uniform per workgroup
  const int M = MT ? MT : a.M;
  const float2 *c = a.chan + bs * row_len;
  for (int i = threadIdx.x; i < kFirSpan + M - 1; i += kNetThreads) {
    const int64_t idx = t0 - (M - 1) + i;
    win[i] = idx >= 0 && idx < K ? c[idx] : make_float2(0.f, 0.f);
  }
  const float2 *hb = a.h + (int64_t)b * M;
  float2 hr[MT ? MT : 1];
#pragma unroll
  for (int m = 0; m < MT; ++m) hr[m] = hb[m];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kFirSpan / kNetThreads; ++j) {
    const int o = j * kNetThreads + threadIdx.x;
    if (t0 + o >= K) break;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int m = 0; m < (MT ? MT : kMaxTaps); ++m) {
      if (!MT && m >= M) break;
      const float2 h = MT ? hr[MT ? m : 0] : hb[m], u = win[o + (M - 1) - m];   // input t - m (zero before the row)
      acc.x = fmaf(h.x, u.x, fmaf(-h.y, u.y, acc.x));
      acc.y = fmaf(h.x, u.y, fmaf(h.y, u.x, acc.y));
    }
    a.firo[bs * row_len + t0 + o] = acc;
  }
}

// A: y = sum over b < B of FIR_b's output at the firing's offset.
template <int V>
__global__ __launch_bounds__(kNetThreads) void k_net_add(DpdNetArgs a, int bpf) {
  int64_t gg, i0;
  if (!net_sample<V>(a, bpf, &gg, &i0)) return;
  const int64_t row_len = a.nf * a.r, s = gg / a.nf;
  const int Bg = a.B[gg];
  // every branch's load is issued before the sums (unrolled, masked)
  float2 v[kMaxBranches][V];
#pragma unroll
  for (int b = 0; b < kMaxBranches; ++b) {
#pragma unroll
    for (int k = 0; k < V; ++k) v[b][k] = make_float2(0.f, 0.f);
    if (b < a.B_max && active(Bg, b)) net_load<V>(a.firo + (b * a.S + s) * row_len + a.off[b * a.stride + gg] + i0, v[b]);
  }
  float2 acc[V];
#pragma unroll
  for (int k = 0; k < V; ++k) {
    acc[k] = make_float2(0.f, 0.f);
#pragma unroll
    for (int b = 0; b < kMaxBranches; ++b) {
      acc[k].x += v[b][k].x;
      acc[k].y += v[b][k].y;
    }
  }
  net_store<V>(a.y + gg * a.r + i0, acc);
}

// Mask tables: one thread per (row, branch) walks the row's firings in
// order (an exclusive count of the firings whose mask has bit b).
__global__ __launch_bounds__(64) void k_mask_tables(const int32_t *ctrl, int32_t *B, int64_t *off, DpdNetArgs a) {
  const int64_t q = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (q >= a.S * a.B_max) return;
  const int64_t s = q / a.B_max;
  const int b = (int)(q - s * a.B_max);
  const int32_t lim = 1 << a.B_max;
  int64_t cnt = 0;
  for (int64_t g = 0; g < a.nf; ++g) {
    const int64_t gg = s * a.nf + g;
    int32_t m = ctrl[gg];
    if (m < 0 || m >= lim) m = 0;
    if (b == 0) B[gg] = m;
    off[b * a.stride + gg] = cnt * a.r;
    cnt += (m >> b) & 1;
  }
}

}  // namespace

hipError_t launch_mask_tables(const int32_t *ctrl, int32_t *B, int64_t *off, const DpdNetArgs &a, hipStream_t s) {
  const int64_t n = a.S * a.B_max;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mask_tables, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, ctrl, B, off, a);
  return hipGetLastError();
}

hipError_t launch_dpd_network(const DpdNetArgs &a, hipStream_t s, const KTiming *t) {
  const int64_t row_len = a.nf * a.r, total = a.S * row_len;
  if (total <= 0) return hipSuccess;
  // pairs: r even, and 16-byte aligned sample and output arrays (the
  // channels are this library's allocations)
  const bool pair = (a.r % 2) == 0 && ((reinterpret_cast<uintptr_t>(a.x) | reinterpret_cast<uintptr_t>(a.y)) & 15) == 0;
  const int per_block = kNetThreads * (pair ? 2 : 1);
  const int bpf = (int)((a.r + per_block - 1) / per_block);
  const int64_t nb = a.S * a.nf * (int64_t)bpf;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 g1((unsigned)nb);
  if (t) {
    if (pair) hipExtLaunchKernelGGL(k_net_poly<2>, g1, dim3(kNetThreads), 0, s, t->start, nullptr, 0, a, bpf);
    else hipExtLaunchKernelGGL(k_net_poly<1>, g1, dim3(kNetThreads), 0, s, t->start, nullptr, 0, a, bpf);
  } else {
    if (pair) hipLaunchKernelGGL(k_net_poly<2>, g1, dim3(kNetThreads), 0, s, a, bpf);
    else hipLaunchKernelGGL(k_net_poly<1>, g1, dim3(kNetThreads), 0, s, a, bpf);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 g2((unsigned)((row_len + kFirSpan - 1) / kFirSpan), (unsigned)(a.B_max * a.S));
  if (a.M == 16) hipLaunchKernelGGL(k_net_fir<16>, g2, dim3(kNetThreads), 0, s, a);
  else if (a.M == 8) hipLaunchKernelGGL(k_net_fir<8>, g2, dim3(kNetThreads), 0, s, a);
  else if (a.M == 4) hipLaunchKernelGGL(k_net_fir<4>, g2, dim3(kNetThreads), 0, s, a);
  else hipLaunchKernelGGL(k_net_fir<0>, g2, dim3(kNetThreads), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (t) {
    if (pair) hipExtLaunchKernelGGL(k_net_add<2>, g1, dim3(kNetThreads), 0, s, nullptr, t->stop, 0, a, bpf);
    else hipExtLaunchKernelGGL(k_net_add<1>, g1, dim3(kNetThreads), 0, s, nullptr, t->stop, 0, a, bpf);
  } else {
    if (pair) hipLaunchKernelGGL(k_net_add<2>, g1, dim3(kNetThreads), 0, s, a, bpf);
    else hipLaunchKernelGGL(k_net_add<1>, g1, dim3(kNetThreads), 0, s, a, bpf);
  }
  return hipGetLastError();
}

}  // namespace dfh
