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
// Two kernels.  k_scan: one workgroup per segment of firings; a pass
// covers kScanChunks firings per thread (all control loads in flight at
// once):
//   A: per 64-firing group and branch, a ballot of the feed flags gives the
//      group's count and last feeder (LDS table);
//   B: one wavefront per branch scans that table (sum and max over the
//      groups in firing order, lane shuffles) and writes, per group, the
//      count and last feeder before it (global group table).
// With order_out, the batch's firings (one segment) are also grouped by B,
// largest first, as pairs (firing, B) for the body kernels (one unrolled
// code path per B: grouping keeps resident workgroups on one or two paths,
// so their instructions stay cached; the order never changes a result).
// k_scan_tables: one wavefront per group (all groups in parallel) adds each
// firing's in-group part (popcount / highest bit of the ballot bits below
// its lane) and writes off_b, prev_b.
#include "common.h"

namespace dfh {

constexpr int kScanThreads = 1024;
constexpr int kScanWaves = kScanThreads / 64;
constexpr int kScanChunks = 4;                 // kScanChunks * kScanWaves <= 64

__global__ __launch_bounds__(kScanThreads) void k_scan(ScanArgs a) {
  __shared__ int tot[kScanChunks * kScanWaves][kMaxBranches], lst[kScanChunks * kScanWaves][kMaxBranches];
  __shared__ int pass_cnt[kMaxBranches], pass_last[kMaxBranches];
  __shared__ int64_t carry_cnt[kMaxBranches], carry_last[kMaxBranches];
  __shared__ int tab[kScanChunks * kScanWaves][kMaxBranches + 1], pre[kScanChunks * kScanWaves][kMaxBranches + 1];
  __shared__ int cursor[kMaxBranches + 1], run[kMaxBranches + 1], pass_tot[kMaxBranches + 1];
  const int seg = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), nw = blockDim.x >> 6;
  const int64_t R = a.ctrl_idx ? a.ctrl_idx[0] : 0;
  const int64_t g0 = (int64_t)seg * a.seg_firings;
  const int64_t gps = (a.seg_firings + 63) / 64;     // groups per segment
  const int E = kScanChunks * nw;                    // groups per pass
  if (tid < a.B_max) carry_cnt[tid] = 0, carry_last[tid] = -1;
  const int64_t per_pass = (int64_t)kScanChunks * blockDim.x;
  int Bv[kScanChunks];
  for (int64_t p0 = 0; p0 < a.seg_firings; p0 += per_pass) {
#pragma unroll
    for (int c = 0; c < kScanChunks; ++c) {
      const int64_t j = p0 + (int64_t)c * blockDim.x + tid;   // segment-local firing
      int v = 0;
      if (j < a.seg_firings) {
        bool bad;
        v = (int)token_set(a.ctrl[(R + g0 + j) & a.ctrl_mask], a.ctrl_mode, a.B_max, &bad);
        if (bad && a.err) atomicOr(a.err, (int32_t)kErrControl);
      }
      Bv[c] = v;
    }
    __syncthreads();                            // carries and hist initialised / updated
#pragma unroll
    for (int c = 0; c < kScanChunks; ++c) {
      const int64_t j = p0 + (int64_t)c * blockDim.x + tid;
      if (j < a.seg_firings) a.B_out[g0 + j] = Bv[c];
    }
    // A: group counts and last feeders (pass-local index); row c*nw + wave
    // is the 64-firing group starting at p0 + c*blockDim + 64*wave
#pragma unroll
    for (int c = 0; c < kScanChunks; ++c) {
      const bool in = p0 + (int64_t)c * blockDim.x + tid < a.seg_firings;
      for (int b = 0; b < a.B_max; ++b) {
        const uint64_t bal = __ballot(in && (a.hist_mode == 1 || in_set((uint32_t)Bv[c], b)));
        if (lane == 0) {
          tot[c * nw + wave][b] = __popcll(bal);
          lst[c * nw + wave][b] = bal ? c * (int)blockDim.x + 64 * wave + 63 - __clzll((long long)bal) : -1;
        }
      }
    }
    __syncthreads();
    // B: exclusive scans over the groups, one wavefront per branch
    if (wave < a.B_max) {
      const int b = wave;
      const int row = lane;                       // group c*nw + w
      const int cnt = row < E ? tot[row][b] : 0;
      const int lastv = row < E ? lst[row][b] : -1;
      int cs = cnt, ls = lastv;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int tc = __shfl_up(cs, o), tl = __shfl_up(ls, o);
        if (lane >= o) cs += tc, ls = max(ls, tl);
      }
      int lx = __shfl_up(ls, 1);
      if (lane == 0) lx = -1;
      if (row < E) {
        const int c = row / nw, w = row - c * nw;
        const int64_t gstart = p0 + (int64_t)c * blockDim.x + 64 * w;   // first firing of the group
        if (gstart < a.seg_firings) {
          const int64_t gi = ((int64_t)seg * gps + gstart / 64) * a.B_max + b;
          const int64_t last = lx >= 0 ? p0 + lx : carry_last[b];
          a.grp[2 * gi] = carry_cnt[b] + (cs - cnt);
          a.grp[2 * gi + 1] = last >= 0 ? g0 + last : -1;
        }
      }
      if (lane == 63) pass_cnt[b] = cs, pass_last[b] = ls;
    }
    __syncthreads();
    if (tid < a.B_max) {
      carry_cnt[tid] += pass_cnt[tid];
      if (pass_last[tid] >= 0) carry_last[tid] = p0 + pass_last[tid];
    }
  }
  __syncthreads();
  if (tid < a.B_max && a.last_out)
    a.last_out[(int64_t)seg * a.B_max + tid] = carry_last[tid] >= 0 ? g0 + carry_last[tid] : -1;
  if (!a.order_out) return;
  // Group the firings by Horner length (largest first), in firing order
  // inside a length, with no atomics and no serial loops: the segment is
  // taken in passes of kScanChunks*blockDim firings (64 chunks of 64); per
  // chunk one ballot per length gives its count (LDS table) and each lane's
  // rank inside the chunk; wavefront v scans column v of the table over the
  // 64 chunks with lane shuffles.  Pass A only totals the lengths (to place
  // each length's run); pass B places the firings.
  const int NV = a.B_max + 1;                        // lengths 0..B_max
  const int E2 = kScanChunks * nw;                   // chunks per pass (64: one per lane)
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  // a segment of one pass still holds its tokens in registers
  const bool in_regs = a.seg_firings <= per_pass;
  auto sets_of = [&](int64_t p0, int (&S)[kScanChunks]) {
#pragma unroll
    for (int c = 0; c < kScanChunks; ++c) {
      const int64_t j = p0 + (int64_t)c * blockDim.x + tid;
      S[c] = j >= a.seg_firings ? -1 : (in_regs ? Bv[c] : a.B_out[g0 + j]);
    }
  };
  // chunk counts of one pass into tab[chunk][v]; ranks of this thread's firings
  auto count_pass = [&](const int (&S)[kScanChunks], int (&rank)[kScanChunks]) {
#pragma unroll
    for (int c = 0; c < kScanChunks; ++c) {
      const int L = S[c] >= 0 ? set_len((uint32_t)S[c]) : -1;
      int cnt = 0;
      rank[c] = 0;
      for (int v = 0; v < NV; ++v) {
        const uint64_t bal = __ballot(L == v);
        if (L == v) rank[c] = __popcll(bal & below);
        if (lane == v) cnt = __popcll(bal);
      }
      if (lane < NV) tab[c * nw + wave][lane] = cnt;
    }
  };
  // column scans: pre[chunk][v] = count of length v in earlier chunks of the
  // pass, pass_tot[v] = the pass's count of length v
  auto scan_columns = [&]() {
    for (int v = wave; v < NV; v += nw) {
      const int x = lane < E2 ? tab[lane][v] : 0;
      int sc = x;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(sc, o);
        if (lane >= o) sc += t;
      }
      if (lane < E2) pre[lane][v] = sc - x;
      if (lane == 63) pass_tot[v] = sc;
    }
  };
  int S[kScanChunks], rank[kScanChunks];
  if (tid <= kMaxBranches) run[tid] = 0;             // pass A: totals per length
  for (int64_t p0 = 0; p0 < a.seg_firings; p0 += per_pass) {
    sets_of(p0, S);
    count_pass(S, rank);
    __syncthreads();
    scan_columns();
    __syncthreads();
    if (tid < NV) run[tid] += pass_tot[tid];
    __syncthreads();
  }
  if (wave == 0) {                                   // cursor[v]: first slot of length v, longest first
    const int t = lane < NV ? run[lane] : 0;
    int sc = t;                                      // inclusive scan from the top length down
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_down(sc, o);
      if (lane + o < 64) sc += u;
    }
    if (lane < NV) cursor[lane] = sc - t;
  }
  __syncthreads();
  if (tid < NV) run[tid] = cursor[tid];              // pass B: place
  for (int64_t p0 = 0; p0 < a.seg_firings; p0 += per_pass) {
    sets_of(p0, S);
    count_pass(S, rank);
    __syncthreads();
    scan_columns();
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kScanChunks; ++c) {
      if (S[c] < 0) continue;
      const int L = set_len((uint32_t)S[c]);
      const int k = run[L] + pre[c * nw + wave][L] + rank[c];
      a.order_out[2 * k] = (int32_t)(p0 + (int64_t)c * blockDim.x + tid);
      a.order_out[2 * k + 1] = S[c];
    }
    __syncthreads();
    if (tid < NV) run[tid] += pass_tot[tid];
    __syncthreads();
  }
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

hipError_t launch_scan(const ScanArgs &a, hipStream_t s, bool tables) {
  if (a.n_segs <= 0 || a.seg_firings <= 0) return hipSuccess;
  if (a.B_max < 1 || a.B_max > kMaxBranches || !a.grp) return hipErrorInvalidValue;
  if (a.order_out && a.n_segs != 1) return hipErrorInvalidValue;
  // small segments take fewer wavefronts (kScanChunks firings per thread);
  // the group scan needs a wavefront per branch
  int64_t waves = (a.seg_firings + 64 * kScanChunks - 1) / (64 * kScanChunks);
  if (waves > kScanWaves) waves = kScanWaves;
  if (waves < a.B_max) waves = a.B_max;
  hipLaunchKernelGGL(k_scan, dim3(a.n_segs), dim3(64 * (unsigned)waves), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!tables) return hipSuccess;                    // the head pass fills them
  const int64_t ng = scan_groups(a.n_segs, a.seg_firings);
  hipLaunchKernelGGL(k_scan_tables, dim3((unsigned)((ng + 3) / 4)), dim3(256), 0, s, a, ng);
  return hipGetLastError();
}

}  // namespace dfh
