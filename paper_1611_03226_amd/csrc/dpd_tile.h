// One tile of predistortion outputs inside one firing (device code shared by
// the single-actor batch kernel and the multi-instance persistent kernel).
//
// Inside a firing every active branch reads the same input samples, so the
// branch sum is evaluated per tap as a polynomial in p = |x|^2 (Horner over
// branches, Sec. 4.2 actor body):
//   y[t] = sum_m x[t-m] * P_m(p[t-m]),   P_m(p) = sum_{b<B} h[b][m] p^b.
// With a branch set that is not a prefix, the coefficients of the inactive
// branches below the highest active one enter the polynomial as zeros.
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

// Element i, or +0 when `keep` is clear (all-ones / all-zero word: the
// select is a bitwise AND on the uniform coefficient words).
__device__ __forceinline__ float2 ldc_masked(cfloat2p p, int i, uint32_t keep) {
  const float2 v = ldc(p, i);
  return make_float2(__builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v.x) & keep),
                     __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v.y) & keep));
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
// MASKED: set is the firing's branch set (B = its Horner length) and the
// coefficients of branches outside it read as zero; without MASKED the set
// is the prefix 0..B-1 and the coefficients are used as loaded.
// Software pipeline of depth one: tap m+1's coefficients and sample are
// loaded before tap m's arithmetic; a compiler fence after each tap keeps
// later loads from being hoisted (which would keep every tap's
// coefficients live at once and spill).
template <int M, int K, int B, bool MASKED>
__device__ __forceinline__ void horner_taps(cfloat2p hg, uint32_t set, const float2 *sx, int q0, float (&ar)[K],
                                            float (&ai)[K]) {
  auto coef = [&](int b, int i) {
    if constexpr (MASKED) return ldc_masked(hg, i, 0u - ((set >> b) & 1u));
    else return ldc(hg, i);
  };
  float2 wv[K];
  float pv[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    wv[k] = sx[lds_slot(q0 + M - 1 + k)];
    pv[k] = fmaf(wv[k].x, wv[k].x, wv[k].y * wv[k].y);   // explicit: no contraction freedom
  }
  float2 hc[B];
#pragma unroll
  for (int b = 0; b < B; ++b) hc[b] = coef(b, b * M);
#pragma unroll
  for (int m = 0; m < M; ++m) {
    float2 hn[B];
    float2 wn = make_float2(0.f, 0.f);
    if (m + 1 < M) {
#pragma unroll
      for (int b = 0; b < B; ++b) hn[b] = coef(b, b * M + m + 1);
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

// LDS float2 slots for a firing's head corrections (M-1 outputs).
__host__ __device__ constexpr int lds_corr(int M) { return M > 1 ? M - 1 : 1; }

// Lane i of a 16-lane row receives lane i+S of the same row (0 past the
// row end): one DPP move.
template <int S>
__device__ __forceinline__ float row_shl(float v) {
  if constexpr (S == 0) {
    return v;
  } else {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x100 + S, 0xF, 0xF, true));
  }
}

// Taps m..M-1 of one branch's head correction for output i of the lane's
// row: psi of history sample i - m sits in lane (M-1) + i - m of the row.
// For m <= i (no history term) that lane is an idle lane of the row (psi 0)
// or past the row end (the shift yields 0), so every tap is summed.
template <int M, int m>
__device__ __forceinline__ void head_taps(cfloat2p hg, int b, float psr, float psi, float &sr, float &si) {
  const float2 c = ldc(hg, b * M + m);
  const float vr = row_shl<M - 1 - m>(psr), vi = row_shl<M - 1 - m>(psi);
  sr = fmaf(c.x, vr, sr);
  sr = fmaf(-c.y, vi, sr);
  si = fmaf(c.x, vi, si);
  si = fmaf(c.y, vr, si);
  if constexpr (m + 1 < M) head_taps<M, m + 1>(hg, b, psr, psi, sr, si);
}

// Head corrections of up to four firings of one actor (one wavefront; lane
// 16*row + i serves firing `row`, history sample / output i).  Outputs
// q < M-1 of a firing reach back before its first sample, where branch b
// reads its own history source (the tail of its last feeding firing, or the
// carried state).  The tile body stages zeros there; this adds the
// difference:
//   corr[q] = sum_{b<B} sum_{m=q+1}^{M-1} h_b[m] psi_b(src_b[q-m]),
// accumulated branch by branch.  All history loads are issued at once; psi
// values move inside a row by DPP row shifts; the coefficients are the same
// for every row (uniform scalar loads).
//   B_of(row) -> branch set of the row's firing (empty: no correction)
//   src_of(row, b) -> history source firing of branch b (-1: carried state)
//   sample(row, b, pf, i) -> sample i of branch b's history
// Only branches b_first, b_first + b_step, ... are evaluated (a head pass may
// split a firing's branches over several wavefronts); for each, in
// increasing b, emit(b, active, sr, si) receives the lane's sum over that
// branch's taps (active: b is in the row's branch set).  The correction of
// (row, output i) is the sum of the active branches' values in increasing
// b, starting from 0 (every caller keeps that order, so all head passes
// round alike); it is meaningful where head_live() holds.
template <int M, int ROWS>
__device__ __forceinline__ bool head_live(uint32_t set) {
  const int lane = threadIdx.x & 63, row = lane >> 4, i = lane & 15;
  return row < ROWS && i < M - 1 && set != 0u;
}

template <int M, int ROWS, class BOf, class SrcOf, class Sample, class Emit>
__device__ __forceinline__ void head_correction(cfloat2p hg, BOf B_of, SrcOf src_of, Sample sample, int b_first,
                                                int b_step, Emit emit) {
  constexpr int L = M - 1;
  static_assert(L < 16, "one row of 16 lanes per firing");
  const int lane = threadIdx.x & 63, row = lane >> 4, i = lane & 15;
  const bool live = row < ROWS && i < L;
  const uint32_t all = row < ROWS ? (uint32_t)B_of(row) : 0u;
  uint32_t pick = 0u;                                  // branches of this pass
  for (int b = b_first; b < kMaxBranches; b += b_step) pick |= 1u << b;
  const uint32_t set = all & pick;
  const int B = set_len(set);
  int Bw = B;                                          // largest Horner length of the wavefront
#pragma unroll
  for (int o = 16; o < 64; o <<= 1) Bw = max(Bw, __shfl_xor(Bw, o));
  Bw = __builtin_amdgcn_readfirstlane(Bw);
  int64_t pf[kMaxBranches];
#pragma unroll
  for (int b = 0; b < kMaxBranches; ++b) pf[b] = (in_set(set, b) && live) ? src_of(row, b) : -1;
  float2 xs[kMaxBranches];
#pragma unroll
  for (int b = 0; b < kMaxBranches; ++b)
    xs[b] = (in_set(set, b) && live) ? sample(row, b, pf[b], i) : make_float2(0.f, 0.f);
#pragma unroll
  for (int b = 0; b < kMaxBranches; ++b) {
    if (b >= Bw || !in_set(pick, b)) continue;         // uniform
    const float pp = fmaf(xs[b].x, xs[b].x, xs[b].y * xs[b].y);
    float pb = 1.f;
    for (int e = 0; e < b; ++e) pb *= pp;
    float sr = 0.f, si = 0.f;
    head_taps<M, 1>(hg, b, pb * xs[b].x, pb * xs[b].y, sr, si);
    emit(b, in_set(set, b), sr, si);
  }
}

// The tile pipeline.  A workgroup of NT threads computes tiles of K*NT
// consecutive outputs of one firing (B uniform over the tile), walking the
// batch's tiles with a grid stride.  Loads are issued well before their use:
// the descriptor of tile i+2 (one register, lane-distributed) and the window
// and head corrections of tile i+1 are loaded while tile i is computed.
// Samples before the firing start are staged as zeros; a firing's first
// M-1 outputs then add their head correction.  Every rounding step is an
// explicit fmaf or a single operation, so all kernels built from these
// pieces produce bit-identical outputs.

// Everything about one tile, uniform across the workgroup.
struct Job {
  const float2 *x;        // input ring
  float2 *y;              // output ring
  const float2 *h;        // coefficients [B][M] of the firing's actor
  const float2 *corr;     // the firing's head corrections [M-1] (used when head)
  int64_t x_mask, y_mask;
  int64_t xb, yb;         // ring positions of the firing's first input / output sample
  int t0;                 // first output of the tile within the firing
  int nout;               // outputs in the tile
  uint32_t set;           // active branches of the firing (bit set)
  int B;                  // its Horner length (highest active branch + 1)
  int head;               // first tile of a firing with active branches (0/1)
};

template <int M, int K>
struct TileRegs {
  float2 win[K + 1];
  float2 cv;              // head correction of output threadIdx.x (< M-1)
};

// Loads of tile j into registers (issued early, consumed by commit).
template <int M, int K>
__device__ __forceinline__ void load_tile(TileRegs<M, K> &r, const Job &j) {
#pragma unroll
  for (int u = 0; u < K + 1; ++u) {
    const int idx = threadIdx.x + u * blockDim.x;
    const int64_t pos = (int64_t)j.t0 - (M - 1) + idx;
    r.win[u] = (idx < j.nout + M - 1 && pos >= 0) ? j.x[(j.xb + pos) & j.x_mask] : make_float2(0.f, 0.f);
  }
  r.cv = (j.head && (int)threadIdx.x < M - 1) ? j.corr[threadIdx.x] : make_float2(0.f, 0.f);
}

template <int M, int K>
__device__ __forceinline__ void commit_tile(float2 *sx, float2 *sc, const TileRegs<M, K> &r, const Job &j) {
#pragma unroll
  for (int u = 0; u < K + 1; ++u) {
    const int idx = threadIdx.x + u * blockDim.x;
    if (idx < j.nout + M - 1) sx[lds_slot(idx)] = r.win[u];
  }
  if (j.head && (int)threadIdx.x < M - 1) sc[threadIdx.x] = r.cv;
}

// The tile's main arithmetic (window in sx) for this thread's K outputs.
// BC: largest Horner length compiled (10 or 16; fewer unrolled paths keep
// the register budget of the common configurations small).  MASKED: tiles
// may carry branch sets that are not prefixes (bit-mask control tokens).
template <int M, int K, int BC, bool MASKED>
__device__ __forceinline__ void tile_compute(const float2 *sx, cfloat2p hg, const Job &j, float (&ar)[K],
                                             float (&ai)[K]) {
  const int q0 = threadIdx.x * K;
#pragma unroll
  for (int k = 0; k < K; ++k) ar[k] = ai[k] = 0.f;
  if (q0 >= j.nout) return;
  switch (j.B) {
#define DF_CASE(n) \
  case n:                                                  \
    if constexpr (n <= BC) horner_taps<M, K, n, MASKED>(hg, j.set, sx, q0, ar, ai); \
    break;
    DF_CASE(1) DF_CASE(2) DF_CASE(3) DF_CASE(4) DF_CASE(5) DF_CASE(6) DF_CASE(7) DF_CASE(8)
    DF_CASE(9) DF_CASE(10) DF_CASE(11) DF_CASE(12) DF_CASE(13) DF_CASE(14) DF_CASE(15) DF_CASE(16)
#undef DF_CASE
    default: break;
  }
}

// Store this thread's outputs; in a firing's first tile, outputs q < M-1
// first add their head correction (staged in sc).
template <int M, int K>
__device__ __forceinline__ void tile_store(const float2 *sc, const Job &j, float (&ar)[K], float (&ai)[K]) {
  const int q0 = threadIdx.x * K;
  if (q0 >= j.nout) return;
  if (j.head && q0 < M - 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int q = q0 + k;
      if (q < M - 1 && q < j.nout) {
        ar[k] += sc[q].x;
        ai[k] += sc[q].y;
      }
    }
  }
  const int64_t yo = j.yb + j.t0 + q0;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (q0 + k < j.nout) j.y[(yo + k) & j.y_mask] = make_float2(ar[k], ai[k]);
}

// Word w of a lane-distributed descriptor (lane w holds word w).
__device__ __forceinline__ uint32_t dword_at(uint32_t dv, int w) {
  return (uint32_t)__builtin_amdgcn_readlane((int)dv, w);
}
__device__ __forceinline__ uint64_t qword_at(uint32_t dv, int w) {
  return (uint64_t)dword_at(dv, w) | ((uint64_t)dword_at(dv, w + 1) << 32);
}

// The whole pipelined loop over tiles blockIdx.x, +gridDim.x, ... < n_items.
// src.fetch(k) loads tile k's raw descriptor lane-distributed into one
// register (a vector load, two tiles ahead); src.expand(dv, k, job) turns it
// into the uniform Job (lane reads) when the tile's loads are issued.
template <int M, int K, int BC, bool MASKED, class Src>
__device__ __forceinline__ void run_tiles(float2 *sx, float2 *sc, int64_t n_items, Src &src) {
  const int64_t s = gridDim.x;
  int64_t item = blockIdx.x;
  if (item >= n_items) return;                       // uniform
  Job cur, nxt;
  src.expand(src.fetch(item), item, cur);
  TileRegs<M, K> regs;
  load_tile<M, K>(regs, cur);
  bool has_next = item + s < n_items;
  if (has_next) src.expand(src.fetch(item + s), item + s, nxt);
  for (;;) {
    commit_tile<M, K>(sx, sc, regs, cur);
    __syncthreads();
    const bool has_nn = item + 2 * s < n_items;
    if (has_next) load_tile<M, K>(regs, nxt);
    const uint32_t dv_nn = has_nn ? src.fetch(item + 2 * s) : 0u;
    float ar[K], ai[K];
    tile_compute<M, K, BC, MASKED>(sx, as_const(cur.h), cur, ar, ai);
    tile_store<M, K>(sc, cur, ar, ai);
    if (!has_next) break;
    __syncthreads();
    item += s;
    cur = nxt;
    if (has_nn) src.expand(dv_nn, item + s, nxt);
    has_next = has_nn;
  }
}

}  // namespace dfh
