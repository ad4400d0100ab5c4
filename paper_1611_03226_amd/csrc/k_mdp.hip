// Bodies of the static frame actors of the paper's motion-detection
// pipeline (Sec. 4.1): Gauss (5x5 binomial filter, two top and two bottom
// rows unfiltered), Thres (consecutive-frame difference against a fixed
// threshold) and Med (5-pixel median).  Each batch covers n_frames
// consecutive tokens of the actor's channels; see MdpArgs.
//
// Word path (width a multiple of 4): a work item is a strip of V words (4V
// pixels; V = 4 when the width is a multiple of 16, else 1) of kRun
// consecutive output rows of one frame; consecutive lanes take consecutive
// strips, so every row load of a wave is one contiguous run.  The vertical
// window slides down the item in registers; the words left and right of the
// strip give the horizontal halo, with the nearest in-frame pixel repeated
// at the left and right frame edges.  Pixels are processed four per word in
// 16-bit lanes (md_swar.h).  Any other width takes the byte path: one thread
// per pixel.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "common.h"
#include "md_swar.h"

namespace dfh {
namespace {

constexpr int kMdThreads = 256;
constexpr int kWordThreads = 64;           // word-path workgroup: one wave, little padding per frame
constexpr int kRun = 16;                   // output rows per word-path work item
constexpr int64_t kMaxBlocks = 1 << 23;    // per launch: threads stay below 2^31

// Frame f of the batch in an input channel (from its read counter) or an
// output channel (from its write counter); `map` is the channel's slot map
// (a ring mask, or the paper's layout).
__device__ inline const uint8_t *in_frame(const uint8_t *ring, const int64_t *idx, int64_t map, int64_t f,
                                          int64_t WH) {
  return ring + read_slot(idx[0] + f, map) * WH;
}

__device__ inline uint8_t *out_frame(uint8_t *ring, const int64_t *idx, int64_t map, int64_t f, int64_t WH) {
  return ring + write_slot(idx[1] + f, map) * WH;
}

typedef __attribute__((address_space(1))) uint32_t gu32;

// A global pointer that is the same in every lane, held in scalar registers,
// so that loads and stores use the scalar base + 32-bit vector offset form.
__device__ inline gu32 *uniform_ptr(const void *p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (gu32 *)(((uint64_t)hi << 32) | lo);
}

// Frame and part of a word-path workgroup.  Workgroups are dispatched to the
// 8 XCDs round robin (workgroup b to XCD b % 8), each XCD with its own L2.
// Groups of 8 frames are laid out so that all bpf workgroups of a frame get
// the same b % 8: the rows two neighbouring parts of a frame share (the
// vertical halo) are then read through one L2.  A last group of fewer than
// 8 frames keeps the plain order.
struct FramePart {
  uint32_t frame, part;
};

__device__ inline FramePart frame_part(uint32_t b, uint32_t bpf) {
  const uint32_t nf = gridDim.x / bpf, group = 8 * bpf;
  const uint32_t g = b / group, rem = b % group;
  if (8 * (g + 1) <= nf) return {8 * g + rem % 8, rem / 8};
  return {b / bpf, b % bpf};
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) u32x4 gu32x4;

// Word columns of a word-path strip: its first word c0, V words, and the
// clamped neighbour words; at a frame edge the perm selectors repeat the
// edge pixel instead of using the missing neighbour, so every load is
// unconditional.
template <int V>
struct Strip {
  uint32_t c0, cl, cr;
  bool left_edge, right_edge;
  __device__ Strip(int s, int Wq) {
    c0 = (uint32_t)(s * V);
    left_edge = s == 0;
    right_edge = (s + 1) * V == Wq;
    cl = left_edge ? c0 : c0 - 1;
    cr = right_edge ? c0 + V - 1 : c0 + V;
  }
  // w[0] = left neighbour word, w[1..V] = the strip, w[V+1] = right neighbour
  __device__ void load(const gu32 *src, uint32_t row, uint32_t (&w)[V + 2]) const {
    if constexpr (V == 4) {
      const u32x4 m = *(const gu32x4 *)(src + row + c0);
      w[1] = m.x;
      w[2] = m.y;
      w[3] = m.z;
      w[4] = m.w;
    } else {
      w[1] = src[row + c0];
    }
    w[0] = src[row + cl];
    w[V + 1] = src[row + cr];
  }
  __device__ void store(gu32 *dst, uint32_t row, const uint32_t (&v)[V]) const {
    if constexpr (V == 4) {
      u32x4 m;
      m.x = v[0];
      m.y = v[1];
      m.z = v[2];
      m.w = v[3];
      __builtin_nontemporal_store(m, (gu32x4 *)(dst + row + c0));
    } else {
      __builtin_nontemporal_store(v[0], dst + row + c0);
    }
  }
};

// ------------------------------------------------------------------ Gauss

// FULL: H >= kRun, and the last run of a strip column starts at H - kRun
// (overlapping its predecessor, whose rows it rewrites with the same
// values), so no row of the loop is guarded.  TWO: write both outputs.
template <int V, bool TWO, bool FULL>
__global__ __launch_bounds__(kWordThreads) void k_gauss5_w(MdpArgs a, int64_t f0, int32_t n_runs, int32_t bpf) {
  const FramePart fp = frame_part(blockIdx.x, (uint32_t)bpf);
  const int64_t f = f0 + __builtin_amdgcn_readfirstlane(fp.frame);
  const int32_t local = (int32_t)__builtin_amdgcn_readfirstlane(fp.part) * kWordThreads + (int32_t)threadIdx.x;
  const int32_t Wq = a.W >> 2, Ws = Wq / V;
  const int32_t sx = local % Ws, run = local / Ws;
  if (run >= n_runs) return;
  const int64_t WH = (int64_t)a.W * a.H;
  const gu32 *src = uniform_ptr(in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH));
  gu32 *dst = uniform_ptr(out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH));
  gu32 *dst2 = TWO ? uniform_ptr(out_frame(a.out1, a.out1_idx, a.out1_mask, f, WH)) : nullptr;
  const int H = a.H;
  const int y0 = FULL ? min(run * kRun, H - kRun) : run * kRun;
  const int yend = min(y0 + kRun, H);
  const Strip<V> st(sx, Wq);
  const uint32_t sel_l0 = swar::win2_left(st.left_edge), sel_rV = swar::win2_right(st.right_edge);
  const uint32_t sel_l = swar::win2_left(false), sel_r = swar::win2_right(false);
  uint32_t he[V][5] = {}, ho[V][5] = {}, mid[V][5] = {};
#pragma unroll
  for (int r = 0; r < kRun + 4; ++r) {
    uint32_t w[V + 2];
    st.load(src, (uint32_t)(min(max(y0 - 2 + r, 0), H - 1) * Wq), w);
#pragma unroll
    for (int j = 0; j < V; ++j) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        he[j][k] = he[j][k + 1];
        ho[j][k] = ho[j][k + 1];
        mid[j][k] = mid[j][k + 1];
      }
      // window bytes (p-2, p-1, p0, p1 | p2, p3, p4, p5) of word j
      swar::hsum5(swar::perm(w[j + 1], w[j], j == 0 ? sel_l0 : sel_l),
                  swar::perm(w[j + 2], w[j + 1], j == V - 1 ? sel_rV : sel_r), &he[j][4], &ho[j][4]);
      mid[j][4] = w[j + 1];
    }
    if (r >= 4) {
      const int y = y0 + r - 4;
      if (FULL || y < yend) {
        const bool filtered = y >= 2 && y < H - 2;
        uint32_t v[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
          const uint32_t filt = swar::interleave(swar::vround5(he[j][0], he[j][1], he[j][2], he[j][3], he[j][4]),
                                                 swar::vround5(ho[j][0], ho[j][1], ho[j][2], ho[j][3], ho[j][4]));
          v[j] = filtered ? filt : mid[j][2];
        }
        st.store(dst, (uint32_t)(y * Wq), v);
        if (TWO) st.store(dst2, (uint32_t)(y * Wq), v);
      }
    }
  }
}

__global__ __launch_bounds__(kMdThreads) void k_gauss5_b(MdpArgs a, int64_t f0, int32_t bpf) {
  const int64_t f = f0 + blockIdx.x / (uint32_t)bpf;
  const int64_t i = (int64_t)(blockIdx.x % (uint32_t)bpf) * kMdThreads + threadIdx.x;
  const int64_t WH = (int64_t)a.W * a.H;
  if (i >= WH) return;
  const uint8_t *src = in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH);
  const int W = a.W, H = a.H;
  const int y = (int)(i / W), x = (int)(i % W);
  uint32_t v = src[i];
  if (y >= 2 && y < H - 2) {
    const uint32_t w[5] = {1, 4, 6, 4, 1};
    uint32_t s = 128;
    for (int dy = 0; dy < 5; ++dy) {
      const uint8_t *row = src + (int64_t)(y + dy - 2) * W;
      for (int dx = 0; dx < 5; ++dx) s += w[dy] * w[dx] * row[min(max(x + dx - 2, 0), W - 1)];
    }
    v = s >> 8;
  }
  out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH)[i] = (uint8_t)v;
  if (a.out1) out_frame(a.out1, a.out1_idx, a.out1_mask, f, WH)[i] = (uint8_t)v;
}

// ------------------------------------------------------------------ Thres

__global__ __launch_bounds__(kMdThreads) void k_thres_v(MdpArgs a, int64_t f0, int32_t bpf) {
  const int64_t f = f0 + __builtin_amdgcn_readfirstlane(blockIdx.x / (uint32_t)bpf);
  const int64_t q = (int64_t)(blockIdx.x % (uint32_t)bpf) * kMdThreads + threadIdx.x;
  const int64_t WH = (int64_t)a.W * a.H;
  if (q >= WH / 16) return;
  const u32x4 c = __builtin_nontemporal_load((const u32x4 *)in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH) + q);
  const u32x4 p = __builtin_nontemporal_load((const u32x4 *)in_frame(a.in1, a.in1_idx, a.in1_mask, f, WH) + q);
  const uint32_t t = (uint32_t)a.thr;
  u32x4 o;
  o.x = swar::absdiff_gt(c.x, p.x, t);
  o.y = swar::absdiff_gt(c.y, p.y, t);
  o.z = swar::absdiff_gt(c.z, p.z, t);
  o.w = swar::absdiff_gt(c.w, p.w, t);
  __builtin_nontemporal_store(o, (u32x4 *)out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH) + q);
}

__global__ __launch_bounds__(kMdThreads) void k_thres_b(MdpArgs a, int64_t f0, int32_t bpf) {
  const int64_t f = f0 + blockIdx.x / (uint32_t)bpf;
  const int64_t i = (int64_t)(blockIdx.x % (uint32_t)bpf) * kMdThreads + threadIdx.x;
  const int64_t WH = (int64_t)a.W * a.H;
  if (i >= WH) return;
  const int c = in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH)[i];
  const int p = in_frame(a.in1, a.in1_idx, a.in1_mask, f, WH)[i];
  const int d = c > p ? c - p : p - c;
  out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH)[i] = d > a.thr ? 255 : 0;
}

// ------------------------------------------------------------------ Med

template <int V, bool FULL>
__global__ __launch_bounds__(kWordThreads) void k_med5_w(MdpArgs a, int64_t f0, int32_t n_runs, int32_t bpf) {
  const FramePart fp = frame_part(blockIdx.x, (uint32_t)bpf);
  const int64_t f = f0 + __builtin_amdgcn_readfirstlane(fp.frame);
  const int32_t local = (int32_t)__builtin_amdgcn_readfirstlane(fp.part) * kWordThreads + (int32_t)threadIdx.x;
  const int32_t Wq = a.W >> 2, Ws = Wq / V;
  const int32_t sx = local % Ws, run = local / Ws;
  if (run >= n_runs) return;
  const int64_t WH = (int64_t)a.W * a.H;
  const gu32 *src = uniform_ptr(in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH));
  gu32 *dst = uniform_ptr(out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH));
  const int H = a.H;
  const int y0 = FULL ? min(run * kRun, H - kRun) : run * kRun;
  const int yend = min(y0 + kRun, H);
  const Strip<V> st(sx, Wq);
  const uint32_t sel_l0 = swar::win1_left(st.left_edge), sel_rV = swar::win1_right(st.right_edge);
  const uint32_t sel_l = swar::win1_left(false), sel_r = swar::win1_right(false);
  uint32_t up[V] = {}, cen[V + 2] = {};   // row above the centre row; centre row with its neighbour words
#pragma unroll
  for (int r = 0; r < kRun + 2; ++r) {
    uint32_t w[V + 2];
    st.load(src, (uint32_t)(min(max(y0 - 1 + r, 0), H - 1) * Wq), w);
    if (r >= 2) {
      const int y = y0 + r - 2;
      if (FULL || y < yend) {
        uint32_t v[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
          // left neighbours (p-1, p0, p1, p2), right neighbours (p1, p2, p3, p4) of word j
          const uint32_t L = swar::perm(cen[j + 1], cen[j], j == 0 ? sel_l0 : sel_l);
          const uint32_t R = swar::perm(cen[j + 2], cen[j + 1], j == V - 1 ? sel_rV : sel_r);
          v[j] = swar::med5_bytes(cen[j + 1], up[j], w[j + 1], L, R);
        }
        st.store(dst, (uint32_t)(y * Wq), v);
      }
    }
    // the current centre row is the row above the next one
#pragma unroll
    for (int j = 0; j < V; ++j) up[j] = cen[j + 1];
#pragma unroll
    for (int j = 0; j < V + 2; ++j) cen[j] = w[j];
  }
}

__global__ __launch_bounds__(kMdThreads) void k_med5_b(MdpArgs a, int64_t f0, int32_t bpf) {
  const int64_t f = f0 + blockIdx.x / (uint32_t)bpf;
  const int64_t i = (int64_t)(blockIdx.x % (uint32_t)bpf) * kMdThreads + threadIdx.x;
  const int64_t WH = (int64_t)a.W * a.H;
  if (i >= WH) return;
  const uint8_t *src = in_frame(a.in0, a.in0_idx, a.in0_mask, f, WH);
  const int W = a.W, H = a.H;
  const int y = (int)(i / W), x = (int)(i % W);
  const uint32_t c = src[i];
  const uint32_t u = src[(int64_t)max(y - 1, 0) * W + x];
  const uint32_t d = src[(int64_t)min(y + 1, H - 1) * W + x];
  const uint32_t l = src[(int64_t)y * W + max(x - 1, 0)];
  const uint32_t rr = src[(int64_t)y * W + min(x + 1, W - 1)];
  out_frame(a.out0, a.out0_idx, a.out0_mask, f, WH)[i] = (uint8_t)swar::med5_bytes(c, u, d, l, rr);
}

// ------------------------------------------------------------------ fused chain
//
// Gauss -> Thres -> Med in one pass over a batch: the frames of the two
// inner channels stay in registers.  A wavefront owns 62 consecutive words
// (lanes 1..62) of the flattened (row band, word column) sequence of a
// frame, plus one halo lane on each side, for kFuseRun output rows, and
// walks a range of consecutive frames: for each it computes the Gauss words
// of its band (rows y0-1 .. y0+R, sliding 5-row window; the 2 neighbour bytes
// on each side come from the adjacent lanes by DPP wave shifts), thresholds
// them against the previous frame's Gauss words kept in registers, and takes
// the 5-pixel median with the row above and below and the neighbour lanes'
// threshold words.  The previous Gauss frame of the first frame of a wave's
// range comes from the delay channel (first frame of the batch) or is
// recomputed from the previous input frame.  A band boundary inside a
// wavefront falls on a frame edge, where the perm selectors ignore the
// neighbour lane.  Lanes past the frame's words load clamped addresses and do
// not store; whole wavefronts past the range exit.
constexpr int kFuseRun = 16;
constexpr int kFuseOut = 62;

__device__ __forceinline__ uint32_t lane_below(uint32_t v) {   // value of lane l-1 (0 in lane 0)
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t lane_above(uint32_t v) {   // value of lane l+1 (0 in lane 63)
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xF, 0xF, true);
}

// One frame of a wavefront's band.  Gauss words of rows clamp(y0-1+j),
// j = 0..R+1, at word `col` are produced one per row step (sliding 5-row
// window).  WARM: only store them in gp (previous frame of the range).
// Otherwise each is thresholded against gp[j] (then replaces it), and once
// three threshold rows are known the median of the middle one is stored;
// with `keep` the Gauss words of rows y0..yend-1 also go to `dg` (the delay
// channel's token).
struct FuseLane {
  int y0, yend, H, Wq;
  uint32_t col, s2l, s2r, s1l, s1r, thr;
  bool store;
};

template <int R, bool WARM>
__device__ inline void fused_frame(const FuseLane &q, const uint32_t *src, uint32_t *dst, uint32_t *dg,
                                   uint32_t (&gpE)[R + 2], uint32_t (&gpO)[R + 2]) {
  uint32_t he[5] = {}, ho[5] = {}, mid[5] = {};
  uint32_t t_up = 0, t_c = 0;
  // recompute the row offsets per frame instead of holding them across the
  // frame loop (they would take ~40 registers)
  int y0 = q.y0;
  uint32_t col = q.col;
  asm volatile("" : "+v"(y0), "+v"(col));
  // every row of the band in flight at once: byte offsets from the
  // wavefront-uniform frame base, stepped by one row and clamped into the
  // frame in offset space (no multiply per row)
  const int row_bytes = 4 * q.Wq, last_row = (q.H - 1) * row_bytes;
  const int col_bytes = (int)col * 4;
  int off = (y0 - 3) * row_bytes;
  uint32_t rows[R + 6];
#pragma unroll
  for (int r = 0; r < R + 6; ++r, off += row_bytes)
    rows[r] = *(const uint32_t *)((const char *)src + (uint32_t)(min(max(off, 0), last_row) + col_bytes));
  int out_off = y0 * row_bytes + col_bytes;         // byte offset of output row y0
#pragma unroll
  for (int r = 0; r < R + 6; ++r) {
    const uint32_t w = rows[r];
    const uint32_t wl = lane_below(w), wr = lane_above(w);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      he[k] = he[k + 1];
      ho[k] = ho[k + 1];
      mid[k] = mid[k + 1];
    }
    swar::hsum5(swar::perm(w, wl, q.s2l), swar::perm(wr, w, q.s2r), &he[4], &ho[4]);
    mid[4] = w;
    if (r < 4) continue;
    const int j = r - 4;                          // Gauss / threshold row index
    const int t = y0 - 1 + j;                     // its frame row (clamped when used)
    // Gauss words kept split: even pixels in gE, odd pixels in gO
    const bool filtered = t >= 2 && t < q.H - 2;
    const uint32_t gE = filtered ? swar::vround5(he[0], he[1], he[2], he[3], he[4]) : mid[2] & swar::kLo;
    const uint32_t gO = filtered ? swar::vround5(ho[0], ho[1], ho[2], ho[3], ho[4]) : (mid[2] >> 8) & swar::kLo;
    if (WARM) {
      gpE[j] = gE;
      gpO[j] = gO;
      continue;
    }
    const uint32_t t_dn = swar::thres_split(gE, gO, gpE[j], gpO[j], q.thr);
    gpE[j] = gE;
    gpO[j] = gO;
    // frame row t = y0 + j - 1 is output row j - 1 of the band
    if (dg && j >= 1 && j <= R && t < q.yend && q.store)
      *(uint32_t *)((char *)dg + (uint32_t)(out_off + (j - 1) * row_bytes)) = swar::interleave(gE, gO);
    if (j >= 2) {
      // median of threshold row j-1 (frame row y0 + j - 2); its inputs are
      // 0x00/0xFF masks, so the median is the bitwise majority
      const uint32_t L = swar::perm(t_c, lane_below(t_c), q.s1l), Rt = swar::perm(lane_above(t_c), t_c, q.s1r);
      const int y = y0 + j - 2;
      if (q.store && y < q.yend)
        __builtin_nontemporal_store(swar::med5_masks(t_c, t_up, t_dn, L, Rt),
                                    (uint32_t *)((char *)dst + (uint32_t)(out_off + (j - 2) * row_bytes)));
    }
    t_up = t_c;
    t_c = t_dn;
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_mdp_fused(MdpFusedArgs a, int32_t waves_per_chunk, int32_t bpc,
                                                   int32_t frames_per_chunk) {
  const FramePart cp = frame_part(blockIdx.x, (uint32_t)bpc);   // (frame chunk, block of the chunk)
  const int32_t seg = (int32_t)cp.part * 4 + (int32_t)(threadIdx.x >> 6);
  if (seg >= waves_per_chunk) return;                            // whole wavefront
  const int lane = (int)(threadIdx.x & 63);
  FuseLane q;
  q.H = a.H;
  q.Wq = a.W >> 2;
  const int n_bands = (a.H + R - 1) / R;
  const int32_t N = n_bands * q.Wq;
  const int32_t i = seg * kFuseOut - 1 + lane;
  q.store = lane >= 1 && lane <= kFuseOut && i < N;
  const int32_t ic = min(max(i, 0), N - 1);
  const int cx = ic % q.Wq;
  q.y0 = (ic / q.Wq) * R;
  q.yend = min(q.y0 + R, a.H);
  q.col = (uint32_t)cx;
  q.s2l = swar::win2_left(cx == 0);
  q.s2r = swar::win2_right(cx == q.Wq - 1);
  q.s1l = swar::win1_left(cx == 0);
  q.s1r = swar::win1_right(cx == q.Wq - 1);
  q.thr = (uint32_t)a.thr;
  const int64_t WH = (int64_t)a.W * a.H;
  const int64_t f_begin = (int64_t)cp.frame * frames_per_chunk;
  const int64_t f_end = min(f_begin + frames_per_chunk, a.n_frames);
  const int64_t in0 = a.in_idx[0], out0 = a.out_idx[1], d_read = a.delay_idx[0], d_write = a.delay_idx[1];

  // Gauss words of the previous frame, rows clamp(y0-1+j), split into even
  // and odd pixels
  uint32_t gpE[R + 2], gpO[R + 2];
  if (f_begin == 0) {
    const uint32_t *pg = (const uint32_t *)(a.delay + read_slot(d_read, a.delay_mask) * WH);
#pragma unroll
    for (int j = 0; j < R + 2; ++j) {
      const uint32_t w = pg[(uint32_t)(min(max(q.y0 - 1 + j, 0), a.H - 1) * q.Wq) + q.col];
      gpE[j] = w & swar::kLo;
      gpO[j] = (w >> 8) & swar::kLo;
    }
  } else {
    fused_frame<R, true>(q, (const uint32_t *)(a.in + read_slot(in0 + f_begin - 1, a.in_mask) * WH), nullptr, nullptr,
                         gpE, gpO);
  }
  for (int64_t f = f_begin; f < f_end; ++f) {
    // the delay channel keeps the last frame's Gauss output as its one token
    uint32_t *dg = f == a.n_frames - 1 ? (uint32_t *)(a.delay + write_slot(d_write + a.n_frames - 1, a.delay_mask) * WH)
                                       : nullptr;
    fused_frame<R, false>(q, (const uint32_t *)(a.in + read_slot(in0 + f, a.in_mask) * WH),
                          (uint32_t *)(a.out + write_slot(out0 + f, a.out_mask) * WH), dg, gpE, gpO);
  }
}

// ------------------------------------------------------------------ launch

// Launch `kern` over all frames in chunks of at most kMaxBlocks workgroups,
// bpf workgroups per frame; timing events bracket the first and last chunk.
template <class K, class... Extra>
hipError_t launch_frames(K kern, int threads, const MdpArgs &a, int32_t bpf, hipStream_t s, const KTiming *t,
                         Extra... extra) {
  const int64_t per_launch = kMaxBlocks / bpf > 0 ? kMaxBlocks / bpf : 1;
  for (int64_t f0 = 0; f0 < a.n_frames; f0 += per_launch) {
    const int64_t nf = a.n_frames - f0 < per_launch ? a.n_frames - f0 : per_launch;
    const dim3 grid((unsigned)(nf * bpf));
    const bool first = f0 == 0, last = f0 + per_launch >= a.n_frames;
    if (t && (first || last))
      hipExtLaunchKernelGGL(kern, grid, dim3(threads), 0, s, first ? t->start : nullptr,
                            last ? t->stop : nullptr, 0, a, f0, extra..., bpf);
    else
      hipLaunchKernelGGL(kern, grid, dim3(threads), 0, s, a, f0, extra..., bpf);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int32_t div_up32(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

struct Counters {
  int64_t *p[8];
  int64_t d[8];
};

__global__ void k_advance_n(Counters c, int n, int32_t *err) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    for (int i = 0; i < n; ++i) *c.p[i] += c.d[i];
    for (int i = 0; i < n; ++i) check_chan(chan_slot(c.p[i]), err);
  }
}

}  // namespace

namespace {

template <int V>
hipError_t launch_gauss5_words(const MdpArgs &a, hipStream_t s, const KTiming *t) {
  const int32_t n_runs = div_up32(a.H, kRun);
  const int32_t bpf = div_up32((int64_t)n_runs * (a.W / (4 * V)), kWordThreads);
  const bool full = a.H >= kRun;
  if (a.out1)
    return full ? launch_frames(k_gauss5_w<V, true, true>, kWordThreads, a, bpf, s, t, n_runs)
                : launch_frames(k_gauss5_w<V, true, false>, kWordThreads, a, bpf, s, t, n_runs);
  return full ? launch_frames(k_gauss5_w<V, false, true>, kWordThreads, a, bpf, s, t, n_runs)
              : launch_frames(k_gauss5_w<V, false, false>, kWordThreads, a, bpf, s, t, n_runs);
}

template <int V>
hipError_t launch_med5_words(const MdpArgs &a, hipStream_t s, const KTiming *t) {
  const int32_t n_runs = div_up32(a.H, kRun);
  const int32_t bpf = div_up32((int64_t)n_runs * (a.W / (4 * V)), kWordThreads);
  return a.H >= kRun ? launch_frames(k_med5_w<V, true>, kWordThreads, a, bpf, s, t, n_runs)
                     : launch_frames(k_med5_w<V, false>, kWordThreads, a, bpf, s, t, n_runs);
}

}  // namespace

hipError_t launch_gauss5(const MdpArgs &a, hipStream_t s, const KTiming *t) {
  if (a.n_frames <= 0) return hipSuccess;
  if (a.W % 16 == 0) return launch_gauss5_words<4>(a, s, t);
  if (a.W % 4 == 0) return launch_gauss5_words<1>(a, s, t);
  return launch_frames(k_gauss5_b, kMdThreads, a, div_up32((int64_t)a.W * a.H, kMdThreads), s, t);
}

hipError_t launch_thres(const MdpArgs &a, hipStream_t s, const KTiming *t) {
  if (a.n_frames <= 0) return hipSuccess;
  const int64_t WH = (int64_t)a.W * a.H;
  if (WH % 16 == 0) return launch_frames(k_thres_v, kMdThreads, a, div_up32(WH / 16, kMdThreads), s, t);
  return launch_frames(k_thres_b, kMdThreads, a, div_up32(WH, kMdThreads), s, t);
}

hipError_t launch_med5(const MdpArgs &a, hipStream_t s, const KTiming *t) {
  if (a.n_frames <= 0) return hipSuccess;
  if (a.W % 16 == 0) return launch_med5_words<4>(a, s, t);
  if (a.W % 4 == 0) return launch_med5_words<1>(a, s, t);
  return launch_frames(k_med5_b, kMdThreads, a, div_up32((int64_t)a.W * a.H, kMdThreads), s, t);
}

hipError_t launch_advance_by(int64_t *const *ptr, const int64_t *delta, int n, int32_t *err, hipStream_t s) {
  if (n < 1 || n > 8) return hipErrorInvalidValue;
  Counters c{};
  for (int i = 0; i < n; ++i) {
    c.p[i] = ptr[i];
    c.d[i] = delta[i];
  }
  hipLaunchKernelGGL(k_advance_n, dim3(1), dim3(64), 0, s, c, n, err);
  return hipGetLastError();
}

hipError_t launch_advance_n(int64_t *const *ptr, int n, int64_t delta, int32_t *err, hipStream_t s) {
  if (n < 1 || n > 8) return hipErrorInvalidValue;
  const int64_t d[8] = {delta, delta, delta, delta, delta, delta, delta, delta};
  return launch_advance_by(ptr, d, n, err, s);
}

bool mdp_fused_supported(int32_t W, int32_t H) { return W % 4 == 0 && W >= 4 && H >= 1; }

hipError_t launch_mdp_fused(const MdpFusedArgs &a, hipStream_t s, const KTiming *t) {
  if (!mdp_fused_supported(a.W, a.H)) return hipErrorInvalidValue;
  if (a.n_frames <= 0) return hipSuccess;
  const int64_t n_bands = (a.H + kFuseRun - 1) / kFuseRun;
  const int64_t words = n_bands * (a.W / 4);
  const int32_t waves = (int32_t)((words + kFuseOut - 1) / kFuseOut);
  const int32_t bpc = (waves + 3) / 4;
  // frame ranges as short as possible while the whole grid stays resident
  // (one round of workgroups: no tail of a partly filled second round)
  const int64_t resident = resident_blocks((const void *)k_mdp_fused<kFuseRun>, 256, 0);
  const int64_t max_chunks = resident / bpc > 0 ? resident / bpc : 1;
  const int64_t fpc = (a.n_frames + max_chunks - 1) / max_chunks;
  const int64_t chunks = (a.n_frames + fpc - 1) / fpc;
  if (chunks * bpc > kMaxBlocks) return hipErrorInvalidValue;   // > 2^23 workgroups: not supported
  const dim3 grid((unsigned)(chunks * bpc));
  if (t)
    hipExtLaunchKernelGGL(k_mdp_fused<kFuseRun>, grid, dim3(256), 0, s, t->start, t->stop, 0, a, waves, bpc,
                          (int32_t)fpc);
  else
    hipLaunchKernelGGL(k_mdp_fused<kFuseRun>, grid, dim3(256), 0, s, a, waves, bpc, (int32_t)fpc);
  return hipGetLastError();
}

}  // namespace dfh
