// Device side of the control intake and offset scan (Sec. 2.2), shared by
// the scan kernel and the head pass (which scans the next batch ahead).
// One wavefront per 64-firing group: the group's tokens validated, per
// branch a ballot of the feed flags gives its count and last feeder, per
// Horner length its firing count (ordered scans); the last group of a
// segment to finish turns the segment's tables into exclusive prefixes.
#pragma once

#include "common.h"

namespace dfh {
namespace scan_dev {

constexpr int kNV = kMaxBranches + 1;                // Horner lengths 0..kMaxBranches

// Inclusive wavefront scans with DPP: shifts by 1, 2, 4, 8 inside each row
// of 16 lanes (zero shifted in), then row 0's last lane into row 1 and row
// 2's into row 3 (row_bcast:15), then lane 31 into rows 2 and 3
// (row_bcast:31).
__device__ __forceinline__ int dpp_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// The same for max over values >= 0 (0 is the identity).
__device__ __forceinline__ int dpp_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));
  return v;
}

// Value of the lane below (0 into lane 0): wave_shr:1.
__device__ __forceinline__ int dpp_prev(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }

__device__ __forceinline__ int lane63(int v) { return __builtin_amdgcn_readlane(v, 63); }

// The segment's group table to exclusive prefixes (one wavefront; lane k
// holds group k0 + k of each chunk of 64 groups).  Counts and last feeders
// are segment-local int32 while scanning.  Loads are unconditional (of
// valid entries: branch 0 / length 0 / group 0 stand in past the ends) and
// masked after, so that all of a chunk's loads are in flight at once; a
// segment of at most 64 groups loads its length table with them.
__device__ inline void scan_segment(const ScanArgs &a, int64_t seg, int64_t gps) {
  const int lane = threadIdx.x & 63;
  const int64_t gb = seg * gps, g0 = seg * a.seg_firings;
  const int NV = a.B_max + 1;
  const bool one_chunk = gps <= 64;
  int x[kNV];                                        // length table row (one chunk)
  int cc[kMaxBranches], cl[kMaxBranches];            // carries (uniform)
#pragma unroll
  for (int b = 0; b < kMaxBranches; ++b) cc[b] = 0, cl[b] = -1;
  for (int64_t k0 = 0; k0 < gps; k0 += 64) {
    const int64_t k = k0 + lane;
    const bool ok = k < gps;
    int64_t *row = a.grp + 2 * (gb + (ok ? k : 0)) * a.B_max;
    int64_t cv[kMaxBranches], lv[kMaxBranches];
#pragma unroll
    for (int b = 0; b < kMaxBranches; ++b) {
      const int bb = b < a.B_max ? b : 0;
      cv[b] = row[2 * bb];
      lv[b] = row[2 * bb + 1];
    }
    if (one_chunk && a.lgrp) {
      const int32_t *lrow = a.lgrp + (ok ? k : 0) * NV;
#pragma unroll
      for (int v = 0; v < kNV; ++v) x[v] = lrow[v < NV ? v : 0];
    }
#pragma unroll
    for (int b = 0; b < kMaxBranches; ++b)
      if (b < a.B_max) {
        const int c = ok ? (int)cv[b] : 0;
        const int l = ok && lv[b] >= 0 ? (int)(lv[b] - g0) + 1 : 0;   // last feeder + 1, 0 for none
        const int cs = dpp_sum(c), ls = dpp_max(l);
        const int lx = dpp_prev(ls) - 1;             // exclusive, -1 for none
        if (ok) {
          const int last = lx >= 0 ? lx : cl[b];
          row[2 * b] = cc[b] + cs - c;
          row[2 * b + 1] = last >= 0 ? g0 + last : -1;
        }
        cc[b] += lane63(cs);
        const int lt = lane63(ls) - 1;
        if (lt >= 0) cl[b] = lt;
      }
  }
  if (a.last_out && lane < a.B_max) {
    int v = -1;
#pragma unroll
    for (int b = 0; b < kMaxBranches; ++b)
      if (b == lane) v = cl[b];
    a.last_out[seg * a.B_max + lane] = v >= 0 ? g0 + v : -1;
  }
  if (!a.lgrp) return;
  // length table (one segment): each group's first slot per length = slots
  // of all longer lengths + this length in earlier groups
  int tot[kNV], base[kNV];
  if (one_chunk) {
    const bool ok = lane < gps;
    int cs[kNV];
#pragma unroll
    for (int v = 0; v < kNV; ++v) {
      x[v] = ok ? x[v] : 0;
      cs[v] = dpp_sum(x[v]);
      tot[v] = lane63(cs[v]);
    }
    int run = 0;
#pragma unroll
    for (int v = kNV - 1; v >= 0; --v)
      if (v < NV) base[v] = run, run += tot[v];
    int32_t *lrow = a.lgrp + lane * NV;
#pragma unroll
    for (int v = 0; v < kNV; ++v)
      if (v < NV && ok) lrow[v] = base[v] + cs[v] - x[v];
    return;
  }
#pragma unroll
  for (int v = 0; v < kNV; ++v) tot[v] = 0;
  for (int64_t k0 = 0; k0 < gps; k0 += 64) {         // totals
    const int64_t k = k0 + lane;
    const bool ok = k < gps;
    const int32_t *lrow = a.lgrp + (ok ? k : 0) * NV;
#pragma unroll
    for (int v = 0; v < kNV; ++v) x[v] = lrow[v < NV ? v : 0];
#pragma unroll
    for (int v = 0; v < kNV; ++v)
      if (v < NV) tot[v] += lane63(dpp_sum(ok ? x[v] : 0));
  }
  int run = 0;
#pragma unroll
  for (int v = kNV - 1; v >= 0; --v)
    if (v < NV) base[v] = run, run += tot[v];
  for (int64_t k0 = 0; k0 < gps; k0 += 64) {         // first slots
    const int64_t k = k0 + lane;
    const bool ok = k < gps;
    int32_t *lrow = a.lgrp + (ok ? k : 0) * NV;
#pragma unroll
    for (int v = 0; v < kNV; ++v) x[v] = lrow[v < NV ? v : 0];
#pragma unroll
    for (int v = 0; v < kNV; ++v)
      if (v < NV) {
        const int xv = ok ? x[v] : 0;
        const int cs = dpp_sum(xv);
        if (ok) lrow[v] = base[v] + cs - xv;
        base[v] += lane63(cs);
      }
  }
}

// Group G of the scan (wave-uniform), one wavefront.
__device__ __forceinline__ void scan_group(const ScanArgs &a, int64_t G, int64_t n_groups) {
  if (G >= n_groups) return;                         // uniform per wavefront
  const int lane = threadIdx.x & 63;
  const int64_t gps = (a.seg_firings + 63) / 64;     // groups per segment
  const int64_t seg = G / gps, lg = G - seg * gps;
  const int64_t g0 = seg * a.seg_firings;
  const int64_t j = lg * 64 + lane;                  // segment-local firing
  const bool in = j < a.seg_firings;
  const int64_t R = a.ctrl_idx ? a.ctrl_idx[0] : a.ctrl_pos;
  const int32_t tok = in ? a.ctrl[(R + g0 + j) & a.ctrl_mask] : 0;
  bool bad;
  uint32_t set = token_set(tok, a.ctrl_mode, a.B_max, &bad);
  if (!in) set = 0u, bad = false;
  if (__ballot(bad) && lane == 0 && a.err) atomicOr(a.err, (int32_t)kErrControl);
  if (in) a.B_out[g0 + j] = (int32_t)set;
  // the group's count and last feeder of each branch (lane b keeps branch b's)
  int cnt = 0;
  int64_t last = -1;
  for (int b = 0; b < a.B_max; ++b) {
    const uint64_t bal = __ballot(in && (a.hist_mode == 1 || in_set(set, b)));
    if (lane == b) {
      cnt = __popcll(bal);
      last = bal ? g0 + lg * 64 + 63 - __clzll((long long)bal) : -1;
    }
  }
  if (lane < a.B_max) {
    a.grp[2 * (G * a.B_max + lane)] = cnt;
    a.grp[2 * (G * a.B_max + lane) + 1] = last;
  }
  if (a.lgrp) {                                      // firings of each Horner length
    const int NV = a.B_max + 1, L = in ? set_len(set) : -1;
    int c = 0;
    for (int v = 0; v < NV; ++v) {
      const uint64_t bal = __ballot(L == v);
      if (lane == v) c = __popcll(bal);
    }
    if (lane < NV) a.lgrp[G * NV + lane] = c;
  }
  // The segment's last group to finish scans its group tables: a release
  // fence orders this wavefront's table writes before its ticket increment,
  // an acquire fence after the last increment makes every group's visible.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  int done = 0;
  if (lane == 0)
    done = __hip_atomic_fetch_add(a.ticket + seg, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (int)(gps - 1);
  if (!__builtin_amdgcn_readfirstlane(done)) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  scan_segment(a, seg, gps);
  if (lane == 0) a.ticket[seg] = 0;                  // ready for the next scan
}

}  // namespace scan_dev
}  // namespace dfh
