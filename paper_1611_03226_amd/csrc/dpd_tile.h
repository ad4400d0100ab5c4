// One tile of predistortion outputs inside one firing (device code shared by
// the single-actor batch kernel and the multi-instance persistent kernel).
//
// Inside a firing every active branch reads the same input samples, so the
// branch sum is evaluated per tap as a polynomial in p = |x|^2 (Horner over
// branches, Sec. 4.2 actor body):
//   y[t] = sum_m x[t-m] * P_m(p[t-m]),   P_m(p) = sum_{b<B} h[b][m] p^b.
// The samples before the firing start are staged as zeros; the taps that
// reach there read branch b's own history and are added per branch.
#pragma once

#include "common.h"

namespace dfh {

// LDS slot of window sample i: one pad slot per 8 samples, so the K-strided
// register-window reads of a wavefront fall on distinct banks.
__host__ __device__ constexpr int lds_slot(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int lds_window(int n) { return lds_slot(n) + 1; }

// h: the firing's coefficients staged in LDS ([B][M]); each tap reads its B
// coefficients with broadcast LDS loads (all lanes read the same address).
template <int M, int K, int B>
__device__ __forceinline__ void horner_taps(const float2 *h, const float2 (&w)[K + M - 1],
                                            const float (&p)[K + M - 1], float (&ar)[K], float (&ai)[K]) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    float hr[B], hi[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const float2 c = h[b * M + m];
      hr[b] = c.x;
      hi[b] = c.y;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int s = k + (M - 1) - m;
      float Pr = hr[B - 1], Pi = hi[B - 1];
#pragma unroll
      for (int b = B - 2; b >= 0; --b) {
        Pr = fmaf(Pr, p[s], hr[b]);
        Pi = fmaf(Pi, p[s], hi[b]);
      }
      ar[k] = fmaf(w[s].x, Pr, ar[k]);
      ar[k] = fmaf(-w[s].y, Pi, ar[k]);
      ai[k] = fmaf(w[s].x, Pi, ai[k]);
      ai[k] = fmaf(w[s].y, Pr, ai[k]);
    }
  }
}

// LDS float2 slots needed by dpd_tile beyond the window and coefficients: staged
// branch histories and their per-(branch, output) sums, [B_max][M-1] each.
__host__ __device__ constexpr int lds_history(int B_max, int M) { return 2 * B_max * (M > 1 ? M - 1 : 1); }

// Tile [t0, t0+nout) of the firing whose first input sample sits at ring
// position xb and first output at yb.  LDS: `sx` >= lds_window(nout+M-1)
// float2 (samples), `sh` >= B*M float2 (coefficients), `sq` >=
// lds_history(B, M) float2 (histories).
// hist(b, ii) returns branch b's input sample ii < 0 before the firing start.
// Contains up to three workgroup barriers (all uniform): every thread of the
// block must call it.  Every rounding step is an explicit fmaf or a single
// operation, so all kernels that instantiate this function produce
// bit-identical outputs.
template <int M, int K, class Hist>
__device__ __forceinline__ void dpd_tile(float2 *sx, float2 *sh, float2 *sq, const float2 *__restrict__ x,
                                         int64_t xb, int64_t x_mask, float2 *__restrict__ y, int64_t yb,
                                         int64_t y_mask, int64_t t0, int nout, int B,
                                         const float2 *__restrict__ h, Hist hist) {
  constexpr int L = M - 1;                              // history length
  const bool head = t0 == 0 && B > 0 && L > 0;           // uniform over the block
  for (int idx = threadIdx.x; idx < nout + M - 1; idx += blockDim.x) {
    const int64_t pos = t0 - (M - 1) + idx;
    sx[lds_slot(idx)] = pos >= 0 ? x[(xb + pos) & x_mask] : make_float2(0.f, 0.f);
  }
  for (int idx = threadIdx.x; idx < B * M; idx += blockDim.x) sh[idx] = h[idx];
  // branch b's history sample ii = i - L (i < L) before the firing start
  if (head)
    for (int idx = threadIdx.x; idx < B * L; idx += blockDim.x) sq[idx] = hist(idx / L, (int64_t)(idx % L - L));
  __syncthreads();
  if (head) {
    // history part of output q < L for branch b:
    //   sum_{m=q+1}^{M-1} h_b[m] psi_b(history sample q - m)
    float2 *hp = sq + B * L;
    for (int idx = threadIdx.x; idx < B * L; idx += blockDim.x) {
      const int b = idx / L, q = idx - b * L;
      float sr = 0.f, si = 0.f;
      for (int m = q + 1; m < M; ++m) {
        const float2 xv = sq[b * L + q - m + L];
        const float pp = fmaf(xv.x, xv.x, xv.y * xv.y);
        float pb = 1.f;
        for (int e = 0; e < b; ++e) pb *= pp;
        const float xr = pb * xv.x, xi = pb * xv.y;
        const float2 c = sh[b * M + m];
        sr = fmaf(c.x, xr, sr);
        sr = fmaf(-c.y, xi, sr);
        si = fmaf(c.x, xi, si);
        si = fmaf(c.y, xr, si);
      }
      hp[idx] = make_float2(sr, si);
    }
    __syncthreads();
  }
  const int q0 = threadIdx.x * K;
  if (q0 >= nout) return;
  float2 w[K + M - 1];
  float p[K + M - 1];
#pragma unroll
  for (int s = 0; s < K + M - 1; ++s) {
    w[s] = (q0 + s < nout + M - 1) ? sx[lds_slot(q0 + s)] : make_float2(0.f, 0.f);
    p[s] = fmaf(w[s].x, w[s].x, w[s].y * w[s].y);   // explicit: no contraction freedom
  }
  float ar[K], ai[K];
#pragma unroll
  for (int k = 0; k < K; ++k) ar[k] = ai[k] = 0.f;
  switch (B) {
#define DF_CASE(n) \
  case n: horner_taps<M, K, n>(sh, w, p, ar, ai); break;
    DF_CASE(1) DF_CASE(2) DF_CASE(3) DF_CASE(4) DF_CASE(5) DF_CASE(6) DF_CASE(7) DF_CASE(8)
    DF_CASE(9) DF_CASE(10) DF_CASE(11) DF_CASE(12) DF_CASE(13) DF_CASE(14) DF_CASE(15) DF_CASE(16)
#undef DF_CASE
    default: break;
  }
  if (head && q0 < L) {
    const float2 *hp = sq + B * L;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = q0 + k;
      if (q >= L || q >= nout) continue;
      for (int b = 0; b < B; ++b) {
        ar[k] += hp[b * L + q].x;
        ai[k] += hp[b * L + q].y;
      }
    }
  }
  const int64_t yo = yb + t0 + q0;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (q0 + k < nout) y[(yo + k) & y_mask] = make_float2(ar[k], ai[k]);
}

}  // namespace dfh
