// Control intake, rate resolution and offset scan for a batch of firings.
//
// Sec. 2.2: a dynamic actor first consumes one control token, which fixes
// the rate (0 or r) of each regular port for that firing.  For the
// predistortion actor the token B activates branches b < B.  From the
// per-firing rates this pass derives, for every branch b (a mask token
// activates the branches of its set bits instead; the kernels carry every
// token as its branch set):
//   off_b(j)  = r * #{i < j : firing i feeds branch b}   (exclusive sum)
//   prev_b(j) = max{i < j : firing i feeds branch b}     (exclusive max, -1 none)
//   last_b    = max{i < n : firing i feeds branch b}
// where "feeds" is "b active in firing i" (branch history) or always
// (shared history).
//
// k_scan_groups: one wavefront per 64-firing group, all groups in
// parallel.  A wavefront validates its group's tokens, and per branch a
// ballot of the feed flags gives the group's count and last feeder (group
// table).  The last wavefront of a segment to finish (a ticket counter
// with acquire/release ordering) turns the segment's group table into
// exclusive prefixes in place (sum and max over the groups in firing
// order, lane shuffles): per group, the count and last feeder before it.
// For an ordered scan (one segment) it does the same with the per-group
// counts of each Horner length (highest active branch + 1), which gives
// each length's first slot in each group of the processing order: the
// firings grouped by length, longest first, in firing order inside a
// length, as pairs (firing, branch set) for the body kernels (one unrolled
// code path per length: grouping keeps resident workgroups on one or two
// paths, so their instructions stay cached; the order never changes a
// result).  The head pass places each firing from that table and the rank
// of its length inside its group.
// k_scan_tables: one wavefront per group adds each firing's in-group part
// (popcount / highest bit of the ballot bits below its lane) and writes
// off_b, prev_b (paths without a head pass that does it).
#include <algorithm>

#include "scan_dev.h"

namespace dfh {

// One wavefront per 64-firing group (four per workgroup).
__global__ __launch_bounds__(256) void k_scan_groups(ScanArgs a, int64_t n_groups) {
  scan_dev::scan_group(a, (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), n_groups);
}

// One wavefront per 64-firing group: off_b and prev_b of its firings.
__global__ __launch_bounds__(256) void k_scan_tables(ScanArgs a, int64_t n_groups) {
  const int64_t G = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (G >= n_groups) return;                         // uniform per wavefront
  const int lane = threadIdx.x & 63;
  const int64_t gps = (a.seg_firings + 63) / 64;
  const int64_t seg = G / gps, lg = G - seg * gps;
  const int64_t g0 = seg * a.seg_firings;
  const int64_t j = lg * 64 + lane;                  // segment-local firing
  const bool in = j < a.seg_firings;
  const int Bv = in ? a.B_out[g0 + j] : 0;
  const uint64_t below_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int b = 0; b < a.B_max; ++b) {
    const uint64_t bal = __ballot(in && (a.hist_mode == 1 || in_set((uint32_t)Bv, b)));
    const uint64_t below = bal & below_mask;
    const int64_t gi = G * a.B_max + b;
    const int64_t cnt = a.grp[2 * gi] + __popcll(below);
    const int64_t last = below ? g0 + lg * 64 + 63 - __clzll((long long)below) : a.grp[2 * gi + 1];
    if (in) {
      const int64_t o = (int64_t)b * a.stride + g0 + j;
      a.prev_out[o] = last;
      if (a.off_out) a.off_out[o] = a.r * cnt;
    }
  }
}

int64_t scan_groups(int64_t n_segs, int64_t seg_firings) { return n_segs * ((seg_firings + 63) / 64); }

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t scan_scratch_bytes(int64_t n_segs, int64_t seg_firings, int32_t B_max, bool ordered) {
  const int64_t ng = std::max<int64_t>(scan_groups(n_segs, seg_firings), 1);
  size_t b = al256(sizeof(int32_t) * std::max<int64_t>(n_segs, 1)) + al256(2 * sizeof(int64_t) * (size_t)B_max * ng);
  if (ordered) b += al256(sizeof(int32_t) * (size_t)(B_max + 1) * ng);
  return b;
}

// Tickets first: their place depends only on the segment count, so a
// buffer sized for the largest batch keeps them (at zero) for any batch.
void scan_scratch_assign(ScanArgs &a, void *scratch, bool ordered) {
  const int64_t ng = std::max<int64_t>(scan_groups(a.n_segs, a.seg_firings), 1);
  char *p = (char *)scratch;
  a.ticket = (int32_t *)p;
  p += al256(sizeof(int32_t) * std::max<int64_t>(a.n_segs, 1));
  a.grp = (int64_t *)p;
  p += al256(2 * sizeof(int64_t) * (size_t)a.B_max * ng);
  a.lgrp = ordered ? (int32_t *)p : nullptr;
}

int64_t resident_blocks(const void *kernel, int threads, size_t lds_bytes) {
  struct Entry {
    const void *k;
    int threads, dev;
    size_t lds;
    int64_t n;
  };
  static Entry cache[64];
  static int used = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  for (int i = 0; i < used; ++i)
    if (cache[i].k == kernel && cache[i].threads == threads && cache[i].lds == lds_bytes && cache[i].dev == dev)
      return cache[i].n;
  int per_cu = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds_bytes) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 1;
  const int64_t n = (int64_t)per_cu * ncu;
  if (used < 64) cache[used++] = Entry{kernel, threads, dev, lds_bytes, n};
  return n;
}

hipError_t launch_scan(const ScanArgs &a, hipStream_t s, bool tables, bool zero_tickets) {
  if (a.n_segs <= 0 || a.seg_firings <= 0) return hipSuccess;
  if (a.B_max < 1 || a.B_max > kMaxBranches || !a.grp || !a.ticket) return hipErrorInvalidValue;
  if (a.seg_firings > INT32_MAX || (a.lgrp && a.n_segs != 1)) return hipErrorInvalidValue;
  if (zero_tickets) {
    hipError_t e = launch_fill_i32(a.ticket, 0, a.n_segs, s);
    if (e != hipSuccess) return e;
  }
  const int64_t ng = scan_groups(a.n_segs, a.seg_firings);
  hipLaunchKernelGGL(k_scan_groups, dim3((unsigned)((ng + 3) / 4)), dim3(256), 0, s, a, ng);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !tables) return e;          // else the head pass fills them
  hipLaunchKernelGGL(k_scan_tables, dim3((unsigned)((ng + 3) / 4)), dim3(256), 0, s, a, ng);
  return hipGetLastError();
}

}  // namespace dfh
