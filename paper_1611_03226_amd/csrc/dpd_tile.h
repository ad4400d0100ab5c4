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



// ------------------------------------------------------------------ matrix cores
// Matrix-core form of a tile for M = 16 taps.  The per-tap polynomial is a
// matrix product: for a block of 16 window samples s and a chunk of four
// branches, Q[m][s] = sum_b h_b[m] p_s^b is one v_mfma_f32_16x16x4_f32
// (rows: taps m, columns: samples s, inner index: branches b; one product
// for the real and one for the imaginary part of h), accumulated over the
// ceil(B/4) chunks.  The rest stays on the VALU: Z[m][s] = x_s Q[m][s]
// (complex), and y[q] = sum_m Z[m][q + 15 - m] (window sample i = q + 15 - m
// for output q), taken in two steps.  Lane (row rho, column j) holds Z for
// taps 4 rho + r (r = 0..3, the product's accumulator layout) of sample j;
// shifting register r by r lanes inside the 16-lane row (DPP) aligns every
// value on lane u = j + r, so a row sums to
//   R_rho[16k + u] = sum_r Z[4 rho + r][16k + u - r]   (block k),
// with positions u >= 16 carried to the next block's first lanes.  Each
// R_rho is written to LDS, and after a barrier
//   y[q] = R_0[q + 15] + R_1[q + 11] + R_2[q + 7] + R_3[q + 3].
// The products are exact float products with float accumulation (the
// power-basis sum, not Horner's rule), so this form rounds differently from
// the VALU form; when it is selected (DFHIP_BODY=mx), every kernel that runs
// M = 16 bodies uses it, so the batching paths stay bit-identical.  On
// MI355X it is the slower form: the complex products, row combination,
// powers and LDS staging it leaves on the VALU cost nearly as many VALU
// instructions as Horner's rule (SQ_INSTS_VALU per launch 60 M + 4 M
// matrix products against 66 M), and the matrix products add latency.

typedef float mx4 __attribute__((ext_vector_type(4)));

// Lane i of a 16-lane row receives lane i-S of the same row (0 below the
// row start): one DPP move.
template <int S>
__device__ __forceinline__ float row_shr(float v) {
  if constexpr (S == 0) {
    return v;
  } else {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x110 + S, 0xF, 0xF, true));
  }
}

// Window and row-sum buffer sizes of a matrix-core tile (float2 slots): the
// blocks read window samples up to index tile + 30, and one block ahead.
__host__ __device__ constexpr int mx_window(int tile) { return lds_window(tile + 48); }
__host__ __device__ constexpr int mx_row(int tile) { return tile + 32; }
__host__ __device__ constexpr int mx_lds(int tile) { return lds_corr(16) + mx_window(tile) + 4 * mx_row(tile) + 256; }

// Coefficient operand of the tile's firing: lane l holds h_b[m] for branch
// b = 4c + l/16, tap m = l%16 (zero for branches outside the set).
struct MxCoef {
  float hr[4], hi[4];
};

// The operand passes through LDS (256 float2, written by wavefront 0 at the
// tile's commit), so that the block loop waits on LDS reads only, never on
// the next tile's global loads in flight.
__device__ __forceinline__ void mx_commit_coef(float2 *sh, const MxCoef &c) {
  if (threadIdx.x < 64) {
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[64 * k + threadIdx.x] = make_float2(c.hr[k], c.hi[k]);
  }
}

__device__ __forceinline__ void mx_read_coef(const float2 *sh, MxCoef &c) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float2 v = sh[64 * k + lane];
    c.hr[k] = v.x;
    c.hi[k] = v.y;
  }
}

template <bool MASKED>
__device__ __forceinline__ void mx_load_coef(MxCoef &c, const Job &j) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int b = 4 * k + (lane >> 4);
    const bool on = b < j.B && (!MASKED || in_set(j.set, b));
    const float2 v = on ? j.h[b * 16 + (lane & 15)] : make_float2(0.f, 0.f);
    c.hr[k] = v.x;
    c.hi[k] = v.y;
  }
}

// Row sums of window block k for this wavefront's lanes: main (lane u:
// position 16k + u) and the part past the block end (lanes 0..2: positions
// 16k + 16 + u, carried into the next block).
template <int NCH>
__device__ __forceinline__ void mx_block(const float2 xv, const MxCoef &c, float &mr, float &mi, float &nr, float &ni) {
  const int rho = (threadIdx.x & 63) >> 4;
  const float p = fmaf(xv.x, xv.x, xv.y * xv.y);
  const float p2 = p * p;
  // p^(4c + rho): p^rho selected without branches, times p^4 per chunk
  float bp = ((rho & 1) ? p : 1.f) * ((rho & 2) ? p2 : 1.f);
  const float p4 = p2 * p2;
  mx4 qr = {0.f, 0.f, 0.f, 0.f}, qi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    qr = __builtin_amdgcn_mfma_f32_16x16x4f32(c.hr[ch], bp, qr, 0, 0, 0);
    qi = __builtin_amdgcn_mfma_f32_16x16x4f32(c.hi[ch], bp, qi, 0, 0, 0);
    if (ch + 1 < NCH) bp *= p4;
  }
  float zr[4], zi[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    zr[r] = fmaf(xv.x, qr[r], -(xv.y * qi[r]));
    zi[r] = fmaf(xv.x, qi[r], xv.y * qr[r]);
  }
  mr = zr[0] + row_shr<1>(zr[1]);
  mi = zi[0] + row_shr<1>(zi[1]);
  mr = mr + row_shr<2>(zr[2]);
  mi = mi + row_shr<2>(zi[2]);
  mr = mr + row_shr<3>(zr[3]);
  mi = mi + row_shr<3>(zi[3]);
  nr = row_shl<15>(zr[1]) + row_shl<14>(zr[2]);
  ni = row_shl<15>(zi[1]) + row_shl<14>(zi[2]);
  nr = nr + row_shl<13>(zr[3]);
  ni = ni + row_shl<13>(zi[3]);
}

// Blocks [k0, k1) of the tile for this wavefront (block k0 - 1 first, for
// the part of its row sums that falls into block k0).
template <int NCH>
__device__ __forceinline__ void mx_blocks(const float2 *sx, float2 *rb, int rs, const MxCoef &c, int k0, int k1) {
  const int lane = threadIdx.x & 63, j = lane & 15, rho = lane >> 4;
  float cr = 0.f, ci = 0.f;                          // carried into lanes 0..2 from the block before
  if (k0 > 0) {
    float mr, mi;
    mx_block<NCH>(sx[lds_slot(16 * (k0 - 1) + j)], c, mr, mi, cr, ci);
  }
  float2 *dst = rb + rho * rs + j;
  float2 xv = sx[lds_slot(16 * k0 + j)];             // the next block's sample is read one block ahead
  for (int k = k0; k < k1; ++k) {
    const float2 xn = sx[lds_slot(16 * (k + 1) + j)];
    float mr, mi, nr, ni;
    mx_block<NCH>(xv, c, mr, mi, nr, ni);
    dst[16 * k] = make_float2(mr + cr, mi + ci);
    cr = nr;
    ci = ni;
    xv = xn;
  }
}

// The tile's outputs q = threadIdx.x + NT*kk from the row sums (and the
// head corrections of a firing's first M-1 outputs).
template <int K>
__device__ __forceinline__ void mx_store(const float2 *sc, const float2 *rb, int rs, const Job &j) {
  const int nt = blockDim.x;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int q = threadIdx.x + nt * kk;
    if (q >= j.nout) break;
    const float2 a = rb[q + 15], b = rb[rs + q + 11], c = rb[2 * rs + q + 7], d = rb[3 * rs + q + 3];
    float vr = a.x + b.x, vi = a.y + b.y;
    vr = vr + c.x;
    vi = vi + c.y;
    vr = vr + d.x;
    vi = vi + d.y;
    if (j.head && q < 15) {
      vr = vr + sc[q].x;
      vi = vi + sc[q].y;
    }
    j.y[(j.yb + j.t0 + q) & j.y_mask] = make_float2(vr, vi);
  }
}

// One tile on the matrix cores: the wavefronts split the tile's blocks,
// then every thread stores its outputs.
template <int K, int BC>
__device__ __forceinline__ void mx_tile(const float2 *sx, const float2 *sc, float2 *rb, const MxCoef &c, const Job &j) {
  const int rs = mx_row(K * (int)blockDim.x);
  const int nblk = (j.nout + 14) / 16 + 1;
  const int nw = blockDim.x >> 6, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int k0 = nblk * w / nw, k1 = nblk * (w + 1) / nw;
  const int nch = (j.B + 3) >> 2;
  if (j.B > 0) {
    switch (nch) {
      case 1: mx_blocks<1>(sx, rb, rs, c, k0, k1); break;
      case 2: mx_blocks<2>(sx, rb, rs, c, k0, k1); break;
      case 3: mx_blocks<3>(sx, rb, rs, c, k0, k1); break;
      default: if constexpr (BC > 12) mx_blocks<4>(sx, rb, rs, c, k0, k1); break;
    }
  }
  __syncthreads();
  if (j.B > 0) {
    mx_store<K>(sc, rb, rs, j);
  } else {                                           // no active branch: zeros
    for (int q = threadIdx.x; q < j.nout; q += blockDim.x) j.y[(j.yb + j.t0 + q) & j.y_mask] = make_float2(0.f, 0.f);
  }
}

// The pipelined tile loop (as run_tiles) with matrix-core tiles (M = 16).
// LDS: [15] head corrections, window (mx_window), 4 row-sum rows (mx_row),
// coefficient operand (256).
template <int K, int BC, bool MASKED, class Src>
__device__ __forceinline__ void run_tiles_mx(float2 *sx, float2 *sc, float2 *rb, float2 *sh, int64_t n_items,
                                             Src &src) {
  constexpr int M = 16;
  const int64_t s = gridDim.x;
  int64_t item = blockIdx.x;
  if (item >= n_items) return;                       // uniform
  Job cur, nxt;
  src.expand(src.fetch(item), item, cur);
  TileRegs<M, K> regs;
  MxCoef cl;                                         // coefficient loads of the tile to commit
  load_tile<M, K>(regs, cur);
  mx_load_coef<MASKED>(cl, cur);
  bool has_next = item + s < n_items;
  if (has_next) src.expand(src.fetch(item + s), item + s, nxt);
  for (;;) {
    commit_tile<M, K>(sx, sc, regs, cur);
    mx_commit_coef(sh, cl);
    __syncthreads();
    const bool has_nn = item + 2 * s < n_items;
    if (has_next) {
      load_tile<M, K>(regs, nxt);
      mx_load_coef<MASKED>(cl, nxt);
    }
    const uint32_t dv_nn = has_nn ? src.fetch(item + 2 * s) : 0u;
    MxCoef c;
    mx_read_coef(sh, c);
    mx_tile<K, BC>(sx, sc, rb, c, cur);
    if (!has_next) break;
    __syncthreads();
    item += s;
    cur = nxt;
    if (has_nn) src.expand(dv_nn, item + s, nxt);
    has_next = has_nn;
  }
}

}  // namespace dfh
