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

// Read-only device data seen through the constant address space: loads from
// it at wavefront-uniform addresses become scalar loads into SGPRs, which the
// FMAs read directly (no VGPRs, no LDS traffic for the coefficients).  Only
// memory that no kernel of the launch writes may be read this way.
typedef const __attribute__((address_space(4))) float2 *cfloat2p;

template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *as_const(const T *p) {
  return (const __attribute__((address_space(4))) T *)p;
}

// Element i of a constant-space complex array.
__device__ __forceinline__ float2 ldc(cfloat2p p, int i) {
  const __attribute__((address_space(4))) float *f = (const __attribute__((address_space(4))) float *)p;
  return make_float2(f[2 * i], f[2 * i + 1]);
}

// LDS slot of window sample i: one pad slot per 8 samples, so the K-strided
// register-window reads of a wavefront fall on distinct banks.
__host__ __device__ constexpr int lds_slot(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int lds_window(int n) { return lds_slot(n) + 1; }


// Taps of K consecutive outputs q0..q0+K-1.  Tap m of output q0+k reads
// window sample k+M-1-m, so iterating the taps in order slides a window of
// K samples (one new LDS read per tap; the shift is a register rename).
// Reads stay inside the window buffer (index < tile+M-1); in a partial tile,
// slots past the staged samples only feed outputs that are not stored.
// hg: the firing's coefficients [B][M] (uniform address: scalar loads).
// Software pipeline of depth one: tap m+1's coefficients and sample are
// loaded before tap m's arithmetic; a compiler fence after each tap keeps
// later loads from being hoisted (which would keep every tap's
// coefficients live at once and spill).
template <int M, int K, int B>
__device__ __forceinline__ void horner_taps(cfloat2p hg, const float2 *sx, int q0, float (&ar)[K],
                                            float (&ai)[K]) {
  float2 wv[K];
  float pv[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    wv[k] = sx[lds_slot(q0 + M - 1 + k)];
    pv[k] = fmaf(wv[k].x, wv[k].x, wv[k].y * wv[k].y);   // explicit: no contraction freedom
  }
  float2 hc[B];
#pragma unroll
  for (int b = 0; b < B; ++b) hc[b] = ldc(hg, b * M);
#pragma unroll
  for (int m = 0; m < M; ++m) {
    float2 hn[B];
    float2 wn = make_float2(0.f, 0.f);
    if (m + 1 < M) {
#pragma unroll
      for (int b = 0; b < B; ++b) hn[b] = ldc(hg, b * M + m + 1);
      wn = sx[lds_slot(q0 + M - 2 - m)];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float Pr = hc[B - 1].x, Pi = hc[B - 1].y;
#pragma unroll
      for (int b = B - 2; b >= 0; --b) {
        Pr = fmaf(Pr, pv[k], hc[b].x);
        Pi = fmaf(Pi, pv[k], hc[b].y);
      }
      ar[k] = fmaf(wv[k].x, Pr, ar[k]);
      ar[k] = fmaf(-wv[k].y, Pi, ar[k]);
      ai[k] = fmaf(wv[k].x, Pi, ai[k]);
      ai[k] = fmaf(wv[k].y, Pr, ai[k]);
    }
    asm volatile("" ::: "memory");
    if (m + 1 < M) {
#pragma unroll
      for (int b = 0; b < B; ++b) hc[b] = hn[b];
#pragma unroll
      for (int k = K - 1; k > 0; --k) {
        wv[k] = wv[k - 1];
        pv[k] = pv[k - 1];
      }
      wv[0] = wn;
      pv[0] = fmaf(wn.x, wn.x, wn.y * wn.y);
    }
  }
}

// LDS float2 slots for the branch histories and their per-(branch, output)
// sums, [B_max][M-1] each.
__host__ __device__ constexpr int lds_history(int B_max, int M) { return 2 * B_max * (M > 1 ? M - 1 : 1); }

// The tile pipeline.  A workgroup of NT threads computes tiles of K*NT
// consecutive outputs of one firing (B uniform over the tile).  For the next
// tile it first loads, into registers, its share of the input window
// (K*NT + M-1 samples) and, for the first tile of a firing, of the branch
// histories; while those loads are in flight it computes the current tile
// from LDS.  Every rounding step is an explicit fmaf or a single operation,
// so all kernels built from these pieces produce bit-identical outputs.

constexpr int kHistRegs = 1;   // history samples per thread: launchers keep B_max*(M-1) <= threads

struct TileJob {
  int64_t xb;      // ring position of the firing's first input sample
  int64_t yb;      // ring position of the firing's first output sample
  int64_t t0;      // first output of the tile within the firing
  int nout;        // outputs in the tile
  int B;           // active branches of the firing
  int head;        // first tile of a firing with active branches (0/1)
};

template <int M, int K>
struct TileRegs {
  float2 win[K + 1];
  float2 hst[kHistRegs];
};

// Loads of the next tile (issued early; consumed by tile_commit).
// hist(b, ii) returns branch b's input sample ii < 0 before the firing start.
template <int M, int K, class Hist>
__device__ __forceinline__ void tile_prefetch(TileRegs<M, K> &r, const TileJob &j, const float2 *__restrict__ x,
                                              int64_t x_mask, Hist hist) {
#pragma unroll
  for (int u = 0; u < K + 1; ++u) {
    const int idx = threadIdx.x + u * blockDim.x;
    const int64_t pos = j.t0 - (M - 1) + idx;
    r.win[u] = (idx < j.nout + M - 1 && pos >= 0) ? x[(j.xb + pos) & x_mask] : make_float2(0.f, 0.f);
  }
  constexpr int L = M - 1;
#pragma unroll
  for (int u = 0; u < kHistRegs; ++u) {
    const int idx = threadIdx.x + u * blockDim.x;
    r.hst[u] = (j.head && idx < j.B * L) ? hist(idx / L, (int64_t)(idx % L - L)) : make_float2(0.f, 0.f);
  }
}

// Registers -> LDS: the window into sx, the histories into sq.
template <int M, int K>
__device__ __forceinline__ void tile_commit(float2 *sx, float2 *sq, const TileRegs<M, K> &r, const TileJob &j) {
#pragma unroll
  for (int u = 0; u < K + 1; ++u) {
    const int idx = threadIdx.x + u * blockDim.x;
    if (idx < j.nout + M - 1) sx[lds_slot(idx)] = r.win[u];
  }
  constexpr int L = M - 1;
  if (j.head) {
#pragma unroll
    for (int u = 0; u < kHistRegs; ++u) {
      const int idx = threadIdx.x + u * blockDim.x;
      if (idx < j.B * L) sq[idx] = r.hst[u];
    }
  }
}

// History part of output q < M-1 for branch b (after the commit barrier):
//   hp[b][q] = sum_{m=q+1}^{M-1} h_b[m] psi_b(history sample q - m).
template <int M>
__device__ __forceinline__ void tile_head_sums(float2 *sq, cfloat2p hg, int B) {
  constexpr int L = M - 1;
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
      const float2 c = ldc(hg, b * M + m);
      sr = fmaf(c.x, xr, sr);
      sr = fmaf(-c.y, xi, sr);
      si = fmaf(c.x, xi, si);
      si = fmaf(c.y, xr, si);
    }
    hp[idx] = make_float2(sr, si);
  }
}

// The tile's outputs (window sx and history sums sq in LDS, coefficients hg
// [B][M]) to the output ring.
template <int M, int K>
__device__ __forceinline__ void tile_outputs(const float2 *sx, cfloat2p hg, const float2 *sq, const TileJob &j,
                                             float2 *__restrict__ y, int64_t y_mask) {
  constexpr int L = M - 1;
  const int q0 = threadIdx.x * K;
  if (q0 >= j.nout) return;
  float ar[K], ai[K];
#pragma unroll
  for (int k = 0; k < K; ++k) ar[k] = ai[k] = 0.f;
  switch (j.B) {
#define DF_CASE(n) \
  case n: horner_taps<M, K, n>(hg, sx, q0, ar, ai); break;
    DF_CASE(1) DF_CASE(2) DF_CASE(3) DF_CASE(4) DF_CASE(5) DF_CASE(6) DF_CASE(7) DF_CASE(8)
    DF_CASE(9) DF_CASE(10) DF_CASE(11) DF_CASE(12) DF_CASE(13) DF_CASE(14) DF_CASE(15) DF_CASE(16)
#undef DF_CASE
    default: break;
  }
  if (j.head && q0 < L) {
    const float2 *hp = sq + j.B * L;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = q0 + k;
      if (q >= L || q >= j.nout) continue;
      for (int b = 0; b < j.B; ++b) {
        ar[k] += hp[b * L + q].x;
        ai[k] += hp[b * L + q].y;
      }
    }
  }
  const int64_t yo = j.yb + j.t0 + q0;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (q0 + k < j.nout) y[(yo + k) & y_mask] = make_float2(ar[k], ai[k]);
}

}  // namespace dfh
