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

// P: for every sample of every firing, psi_b(x) = |x|^(2b) x into channel b
// at the firing's offset, for b < B of the firing.
__global__ __launch_bounds__(kNetThreads) void k_net_poly(DpdNetArgs a) {
  const int64_t t = (int64_t)blockIdx.x * kNetThreads + threadIdx.x;
  const int64_t row_len = a.nf * a.r, total = a.S * row_len;
  if (t >= total) return;
  const int64_t s = t / row_len, rem = t - s * row_len, g = rem / a.r, i = rem - g * a.r;
  const int64_t gg = s * a.nf + g;
  const int Bg = a.B[gg];
  const float2 x = a.x[t];
  const float p = fmaf(x.x, x.x, x.y * x.y);
  float2 v = x;
#pragma unroll
  for (int b = 0; b < kMaxBranches; ++b) {
    if (b < a.B_max && active(Bg, b)) a.chan[(b * a.S + s) * row_len + a.off[b * a.stride + gg] + i] = v;
    v = make_float2(v.x * p, v.y * p);
  }
}

// FIR_b: outputs over the K_b samples channel b received in row s (K_b = r
// times the number of firings with b < B), zero history before the row's
// first sample.  A workgroup takes kFirSpan consecutive outputs (four per
// thread) and stages their inputs and the M-1 before them in LDS once (one
// global load per sample instead of M).
constexpr int kFirSpan = 4 * kNetThreads;

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
  for (int j = 0; j < 4; ++j) {
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
__global__ __launch_bounds__(kNetThreads) void k_net_add(DpdNetArgs a) {
  const int64_t t = (int64_t)blockIdx.x * kNetThreads + threadIdx.x;
  const int64_t row_len = a.nf * a.r, total = a.S * row_len;
  if (t >= total) return;
  const int64_t s = t / row_len, rem = t - s * row_len, g = rem / a.r, i = rem - g * a.r;
  const int64_t gg = s * a.nf + g;
  const int Bg = a.B[gg];
  // every branch's load is issued before the sums (unrolled, masked)
  float2 v[kMaxBranches];
#pragma unroll
  for (int b = 0; b < kMaxBranches; ++b) {
    v[b] = make_float2(0.f, 0.f);
    if (b < a.B_max && active(Bg, b)) v[b] = a.firo[(b * a.S + s) * row_len + a.off[b * a.stride + gg] + i];
  }
  float2 acc = make_float2(0.f, 0.f);
#pragma unroll
  for (int b = 0; b < kMaxBranches; ++b) {
    acc.x += v[b].x;
    acc.y += v[b].y;
  }
  a.y[t] = acc;
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
  const dim3 g1((unsigned)((total + kNetThreads - 1) / kNetThreads));
  if (t)
    hipExtLaunchKernelGGL(k_net_poly, g1, dim3(kNetThreads), 0, s, t->start, nullptr, 0, a);
  else
    hipLaunchKernelGGL(k_net_poly, g1, dim3(kNetThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 g2((unsigned)((row_len + kFirSpan - 1) / kFirSpan), (unsigned)(a.B_max * a.S));
  if (a.M == 16) hipLaunchKernelGGL(k_net_fir<16>, g2, dim3(kNetThreads), 0, s, a);
  else if (a.M == 8) hipLaunchKernelGGL(k_net_fir<8>, g2, dim3(kNetThreads), 0, s, a);
  else if (a.M == 4) hipLaunchKernelGGL(k_net_fir<4>, g2, dim3(kNetThreads), 0, s, a);
  else hipLaunchKernelGGL(k_net_fir<0>, g2, dim3(kNetThreads), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (t)
    hipExtLaunchKernelGGL(k_net_add, g1, dim3(kNetThreads), 0, s, nullptr, t->stop, 0, a);
  else
    hipLaunchKernelGGL(k_net_add, g1, dim3(kNetThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace dfh
