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

// Tile [t0, t0+nout) of the firing whose first input sample sits at ring
// position xb and first output at yb.  `sx` is LDS of >= nout+M-1 float2 and
// `sh` LDS of >= B*M float2 (the coefficients are staged there).
// hist(b, ii) returns branch b's input sample ii < 0 before the firing start.
// Contains one workgroup barrier: every thread of the block must call it.
// Every rounding step is an explicit fmaf or a single operation, so all
// kernels that instantiate this function produce bit-identical outputs.
template <int M, int K, class Hist>
__device__ __forceinline__ void dpd_tile(float2 *sx, float2 *sh, const float2 *__restrict__ x, int64_t xb,
                                         int64_t x_mask, float2 *__restrict__ y, int64_t yb, int64_t y_mask,
                                         int64_t t0, int nout, int B, const float2 *__restrict__ h, Hist hist) {
  for (int idx = threadIdx.x; idx < nout + M - 1; idx += blockDim.x) {
    const int64_t pos = t0 - (M - 1) + idx;
    sx[idx] = pos >= 0 ? x[(xb + pos) & x_mask] : make_float2(0.f, 0.f);
  }
  for (int idx = threadIdx.x; idx < B * M; idx += blockDim.x) sh[idx] = h[idx];
  __syncthreads();
  const int q0 = threadIdx.x * K;
  if (q0 >= nout) return;
  float2 w[K + M - 1];
  float p[K + M - 1];
#pragma unroll
  for (int s = 0; s < K + M - 1; ++s) {
    w[s] = (q0 + s < nout + M - 1) ? sx[q0 + s] : make_float2(0.f, 0.f);
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
  if (t0 == 0 && q0 < M - 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = q0 + k;
      if (q >= M - 1 || q >= nout) continue;
      for (int b = 0; b < B; ++b) {
        for (int m = q + 1; m < M; ++m) {
          const float2 xv = hist(b, (int64_t)(q - m));
          const float pp = fmaf(xv.x, xv.x, xv.y * xv.y);
          float pb = 1.f;
          for (int e = 0; e < b; ++e) pb *= pp;
          const float sr = pb * xv.x, si = pb * xv.y;
          const float2 c = sh[b * M + m];
          ar[k] = fmaf(c.x, sr, ar[k]);
          ar[k] = fmaf(-c.y, si, ar[k]);
          ai[k] = fmaf(c.x, si, ai[k]);
          ai[k] = fmaf(c.y, sr, ai[k]);
        }
      }
    }
  }
  const int64_t yo = yb + t0 + q0;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (q0 + k < nout) y[(yo + k) & y_mask] = make_float2(ar[k], ai[k]);
}

}  // namespace dfh
