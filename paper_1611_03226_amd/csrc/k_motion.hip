// Motion actor body: frame difference, threshold, 3x3 opening, per-frame
// changed count and data-dependent emission.
//
// Sec. 4.1 subtracts consecutive frames (the previous one arriving over a
// channel with a one-frame initial token) and thresholds against a constant.
// Per firing j:
//   m0 = |cur - prev| > thr
//   e  = AND of m0 over the in-frame 3x3 neighbourhood   (erosion)
//   o  = OR  of e  over the in-frame 3x3 neighbourhood   (dilation)
//   count_j = sum o;  emit_j = 1000*count_j >= permille*W*H
// Emission depends on the whole frame, so a batch runs
//   bits pass:   opened masks, bit-packed (32 pixels per word, transposed
//                bit order below), and counts
//   emit scan:   output slots of the emitted frames
//   expand pass: emitted masks as 0/255 bytes at their output slots
//   commit:      channel indices.
//
// Bits pass layout: a wavefront owns a band of rows of one frame chunk and
// one chunk of 62 consecutive 32-pixel words (lane l <-> word chunk*62+l-1;
// lanes 0 and 63 are halo words).  It sweeps the rows of the band (plus two
// above and below) keeping, per frame, the last horizontal-AND rows and
// horizontal-OR rows in registers:
//   hm(y)   = m0(y) & left(m0(y)) & right(m0(y))  (neighbour pixels; edge
//             bits from the neighbour lanes)
//   e(y-1)  = hm(y-2) & hm(y-1) & hm(y)
//   he(y-1) = e(y-1) | left(e(y-1)) | right(e(y-1))
//   o(y-2)  = he(y-3) | he(y-2) | he(y-1)
// Outside the frame m0 counts as set (erosion ignores it) and e as clear
// (dilation ignores it).  Erosion and dilation over a square are separable,
// so this equals the 3x3 definitions exactly.  In the self-delay form a
// wavefront handles F consecutive frames per row, so each input row is
// loaded once for F frames (F+1 row loads per F outputs).
#include "common.h"

namespace dfh {

constexpr int MW_CHUNK = 62;   // output words per wavefront

// 32 pixels of row y starting at pixel x0 (x0 < W); bytes past the row end
// read as 0.  `fast`: 16-byte loads (row starts and the word are aligned and
// the word lies inside the row).
__device__ __forceinline__ void load_word(const uint8_t *frame, int y, int x0, int W, bool fast, uint32_t (&v)[8]) {
  const uint8_t *p = frame + (int64_t)y * W + x0;
  if (fast) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 a = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    const u32x4 b = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p + 16));
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uint32_t w = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int x = x0 + 4 * k + i;
        if (x < W) w |= (uint32_t)p[4 * k + i] << (8 * i);
      }
      v[k] = w;
    }
  }
}

typedef short i16x2 __attribute__((ext_vector_type(2)));

// Word of the neighbouring lane, one DPP move each (no LDS round trip):
// lane l receives lane l-1 (lane 0: 0) / lane l+1 (lane 63: 0).  Lanes 0
// and 63 are halo words whose results are discarded.
__device__ __forceinline__ uint32_t from_lower_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xF, 0xF, true);   // wave_shr:1
}
__device__ __forceinline__ uint32_t from_upper_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xF, 0xF, true);   // wave_shl:1
}

// Mask words use a transposed bit order: pixel 4k + j of a word (dword k
// of its 32 bytes, byte j) is bit 8j + k.  The threshold's flags then
// gather with one byte permute and one shift-and-merge per dword, and the
// expand pass decodes a dword's four bytes with one mask and multiply.
__host__ __device__ constexpr int tbit(int x) { return 8 * (x & 3) + (x >> 2); }

// Natural-order mask (bit x = pixel x) to the transposed order.
__device__ __forceinline__ uint32_t to_tbits(uint32_t v) {
  uint32_t t = 0;
  for (int x = 0; x < 32; ++x) t |= ((v >> x) & 1u) << tbit(x);
  return t;
}

// Neighbour pixels in the transposed order: bit of pixel x receives pixel
// x+1 (right) or x-1 (left); across the word edge from the neighbouring
// lane's word (its pixel 0 is bit 0, its pixel 31 is bit 31).
__device__ __forceinline__ uint32_t tright(uint32_t m, uint32_t rw) {
  return (m >> 8) | ((m << 23) & 0x7F000000u) | (rw << 31);
}
__device__ __forceinline__ uint32_t tleft(uint32_t m, uint32_t lw) {
  return (m << 8) | ((m >> 23) & 0xFEu) | (lw >> 31);
}

// Even and odd bytes of a row's dwords spread into 16-bit lanes (byte
// permutes); in the self-delay form a frame's spread serves as the current
// frame of one output and the previous frame of the next.
struct Spread {
  i16x2 e[8], o[8];
};

__device__ __forceinline__ void spread(const uint32_t (&v)[8], Spread &s) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    s.e[k] = __builtin_bit_cast(i16x2, __builtin_amdgcn_perm(v[k], v[k], 0x0c020c00u));   // bytes 0, 2
    s.o[k] = __builtin_bit_cast(i16x2, __builtin_amdgcn_perm(v[k], v[k], 0x0c030c01u));   // bytes 1, 3
  }
}

// |cur - prev| > thr for the 32 pixels of a word (transposed order).  With
// d = cur - prev, a pixel is unchanged iff d - (thr+1) and -(thr+1) - d are
// both negative, i.e. bit 15 of their AND: pixels 0 and 2 of a dword in the
// even product's bits 15 and 31, pixels 1 and 3 in the odd one's.  One
// byte permute puts pixel j's flag in bit 7 of byte j, a shift by 7 - k and
// a mask move it to bit 8j + k; the word is inverted once.
__device__ __forceinline__ uint32_t thresh_tbits(const Spread &c, const Spread &p, i16x2 t1, i16x2 nt1) {
  uint32_t keep = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const i16x2 de = c.e[k] - p.e[k], dd = c.o[k] - p.o[k];
    const uint32_t ye = __builtin_bit_cast(uint32_t, de - t1) & __builtin_bit_cast(uint32_t, nt1 - de);
    const uint32_t yo = __builtin_bit_cast(uint32_t, dd - t1) & __builtin_bit_cast(uint32_t, nt1 - dd);
    const uint32_t g = __builtin_amdgcn_perm(yo, ye, 0x07030501u);   // ye.b1, yo.b1, ye.b3, yo.b3
    keep |= (g >> (7 - k)) & (0x01010101u << k);
  }
  return ~keep;
}

// Row y of the F+1 frames a wavefront needs: buf[f] is the previous frame of
// frame f and buf[f+1] its current frame (self-delay form: frames j0-1 ..
// j0+F-1 of the input channel, the first from the state for j0 = 0; the
// two-channel form has F = 1: buf[0] from the PREV channel, buf[1] from CUR).
// Every load is unconditional: callers clamp y into the frame and point the
// frames past the batch at its last frame (those results are masked).
template <int F, bool FAST>
__device__ __forceinline__ void load_rows(const uint8_t *const (&fr)[F + 1], int y, int x0, int W,
                                          uint32_t (&buf)[F + 1][8]) {
#pragma unroll
  for (int f = 0; f <= F; ++f) load_word(fr[f], y, x0, W, FAST, buf[f]);
}

// Coalesced form of one row of the F+1 frames (W a multiple of 32): the
// wavefront's 64 words are the 2 KiB from byte xs of the row; it loads them
// as two contiguous KiB spans (lane l: 16 bytes at xs + 16 l and at
// xs + 1024 + 16 l; spans outside the row read as 0) ...
template <int F>
__device__ __forceinline__ void load_spans(const uint8_t *const (&fr)[F + 1], int y, int xs, int W,
                                           uint32_t (&raw)[F + 1][8]) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int f = 0; f <= F; ++f)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int off = xs + 1024 * h + 16 * lane;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (off >= 0 && off < W) v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(fr[f] + (int64_t)y * W + off));
      raw[f][4 * h + 0] = v.x;
      raw[f][4 * h + 1] = v.y;
      raw[f][4 * h + 2] = v.z;
      raw[f][4 * h + 3] = v.w;
    }
}

// ... and passes them through LDS (stg: (F+1) x 512 words of this
// wavefront), so that each lane ends with its own 32 bytes (bytes 32 l ..
// 32 l + 31 of the span) in buf.
template <int F>
__device__ __forceinline__ void stage_spans(uint32_t *stg, const uint32_t (&raw)[F + 1][8], uint32_t (&buf)[F + 1][8]) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int f = 0; f <= F; ++f)
#pragma unroll
    for (int h = 0; h < 2; ++h)
      *reinterpret_cast<u32x4 *>(stg + 512 * f + 256 * h + 4 * lane) =
          u32x4{raw[f][4 * h], raw[f][4 * h + 1], raw[f][4 * h + 2], raw[f][4 * h + 3]};
#pragma unroll
  for (int f = 0; f <= F; ++f)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const u32x4 v = *reinterpret_cast<const u32x4 *>(stg + 512 * f + 8 * lane + 4 * h);
      buf[f][4 * h + 0] = v.x;
      buf[f][4 * h + 1] = v.y;
      buf[f][4 * h + 2] = v.z;
      buf[f][4 * h + 3] = v.w;
    }
}

// Work items in XCD-contiguous order: workgroups are dispatched to the 8
// XCDs round robin (workgroup b to XCD b % 8), so item k runs on XCD
// k / per_xcd, and the items an XCD runs in turn are consecutive: the bands
// of a frame group and the next frame groups.  A band's halo rows and the
// previous frame a frame group re-reads are then loaded by workgroups of one
// XCD at about the same time, and come from its L2.  Returns -1 for the
// padding workgroups of a grid rounded up to a multiple of 8.
__device__ __forceinline__ int xcd_item(int b, int n_items) {
  const int per_xcd = (n_items + 7) >> 3;
  const int k = (b & 7) * per_xcd + (b >> 3);
  return k < n_items ? k : -1;
}

template <int F, bool FAST>
__global__ __launch_bounds__(64) void k_motion_bits(MotionArgs a, int rows, int n_bands, int n_chunks, int n_items) {
  const int lane = threadIdx.x;
  const int blk = xcd_item(blockIdx.x, n_items);
  if (blk < 0) return;
  const int chunk = blk % n_chunks;
  const int band = (blk / n_chunks) % n_bands;
  const int64_t j0 = (int64_t)(blk / (n_chunks * n_bands)) * F;
  const int nfr = (int)min((int64_t)F, a.n - j0);
  const int H = a.H, W = a.W, wpr = a.words_per_row;
  const int c = chunk * MW_CHUNK + lane - 1;
  const bool word_in = c >= 0 && c < wpr;
  const bool out_lane = lane >= 1 && lane <= MW_CHUNK && word_in;
  const int x0 = word_in ? c * 32 : 0;
  const uint32_t valid = (c == wpr - 1 && (W & 31)) ? to_tbits((1u << (W & 31)) - 1u) : 0xFFFFFFFFu;
  const int64_t wh = (int64_t)W * H;
  const short t1s = (short)(a.thr + 1);
  const i16x2 t1 = {t1s, t1s}, nt1 = {(short)-t1s, (short)-t1s};
  const int y0 = band * rows, y1 = min(H, y0 + rows);
  uint32_t *__restrict__ bits = a.bits;

  // frame base pointers of the chunk (see load_rows)
  const uint8_t *fr[F + 1];
  {
    const int64_t Rc = a.cur_idx[0];
#pragma unroll
    for (int f = 0; f <= F; ++f) {
      if (a.prev) {
        fr[f] = f == 0 ? a.prev + ((a.prev_idx[0] + j0) & a.prev_mask) * wh : a.cur + ((Rc + j0) & a.cur_mask) * wh;
      } else {
        const int64_t j = j0 + min(f, nfr) - 1;            // past the batch: its last frame
        fr[f] = j < 0 ? a.state : a.cur + ((Rc + j) & a.cur_mask) * wh;
      }
    }
  }

  uint32_t hm2[F], hm1[F], he3[F], he2[F];
  int cnt[F];
#pragma unroll
  for (int f = 0; f < F; ++f) hm2[f] = hm1[f] = he3[f] = he2[f] = 0, cnt[f] = 0;

  auto process = [&](const uint32_t (&buf)[F + 1][8], int y) {
    const bool in = y >= 0 && y < H && word_in;
    const bool e_in = y - 1 >= 0 && y - 1 < H && word_in;
    Spread sp, sc;
    spread(buf[0], sp);
#pragma unroll
    for (int f = 0; f < F; ++f) {
      if (f >= nfr) break;                                  // uniform
      spread(buf[f + 1], sc);
      const uint32_t th = thresh_tbits(sc, sp, t1, nt1);
      sp = sc;
      const uint32_t m0 = in ? (th | ~valid) : 0xFFFFFFFFu; // outside the frame: set
      // horizontal AND with the neighbour words' edge bits
      const uint32_t lw = from_lower_lane(m0), rw = from_upper_lane(m0);
      const uint32_t hm = m0 & tleft(m0, lw) & tright(m0, rw);
      const uint32_t e = e_in ? (hm2[f] & hm1[f] & hm & valid) : 0u;   // e(y-1); outside: clear
      const uint32_t le = from_lower_lane(e), re = from_upper_lane(e);
      const uint32_t he = e | tleft(e, le) | tright(e, re);
      const uint32_t o = (he3[f] | he2[f] | he) & valid;    // o(y-2)
      const int yo = y - 2;
      if (yo >= y0 && yo < y1 && out_lane) {
        cnt[f] += __popc(o);
        bits[(j0 + f) * (int64_t)H * wpr + (int64_t)yo * wpr + c] = o;
      }
      hm2[f] = hm1[f];
      hm1[f] = hm;
      he3[f] = he2[f];
      he2[f] = he;
    }
  };

  // two register row buffers: the loads of the next row are in flight while
  // the current row is processed (rows outside the frame are not loaded)
  uint32_t A[F + 1][8], Bf[F + 1][8];
#pragma unroll
  for (int f = 0; f <= F; ++f)
#pragma unroll
    for (int k = 0; k < 8; ++k) A[f][k] = Bf[f][k] = 0;
  const int ylast = y1 + 1;
  if constexpr (FAST) {
    // coalesced spans: the next row's loads are in flight (raw) while the
    // current row, already staged through LDS, is processed
    __shared__ uint32_t stg[F + 1][512];
    const int xs = (chunk * MW_CHUNK - 1) * 32;
    auto clampy = [&](int y) { return min(max(y, 0), H - 1); };
    load_spans<F>(fr, clampy(y0 - 2), xs, W, Bf);
    stage_spans<F>(&stg[0][0], Bf, A);
    for (int y = y0 - 2; y <= ylast; ++y) {
      if (y + 1 <= ylast) load_spans<F>(fr, clampy(y + 1), xs, W, Bf);
      process(A, y);
      if (y + 1 > ylast) break;
      stage_spans<F>(&stg[0][0], Bf, A);
    }
  } else {
    auto rowload = [&](int y, uint32_t (&buf)[F + 1][8]) { load_rows<F, FAST>(fr, min(max(y, 0), H - 1), x0, W, buf); };
    rowload(y0 - 2, A);
    for (int y = y0 - 2; y <= ylast; y += 2) {
      if (y + 1 <= ylast) rowload(y + 1, Bf);
      process(A, y);
      if (y + 1 > ylast) break;
      if (y + 2 <= ylast) rowload(y + 2, A);
      process(Bf, y + 1);
    }
  }
#pragma unroll
  for (int f = 0; f < F; ++f) {
    int t = cnt[f];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (lane == 0 && f < nfr && t) atomicAdd(&a.count[j0 + f], t);
  }
}

// Expand the bit-packed mask of every emitted frame to 0/255 bytes at the
// frame's output slot.  One thread per 16-pixel half word, so the lanes of a
// wavefront store one contiguous 1 KiB span per instruction.
// The same pass leaves the batch's counts at zero for the next batch (the
// emit scan has read them) and, with state_src set, copies the batch's last
// frame to the self-delay state (grid row n: 16 bytes per thread; nothing in
// this pass reads the frames or the state).
template <bool FAST>
__global__ __launch_bounds__(256) void k_motion_expand(MotionArgs a) {
  const int64_t j = blockIdx.y;
  if (j == a.n) {
    const int64_t off = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    if (off < (int64_t)a.W * a.H) {
      typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
      const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(a.state_src + off));
      *reinterpret_cast<u32x4 *>(a.state + off) = v;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.count[j] = 0;
  const int64_t slot = a.emit_off[j];
  if (slot < 0) return;                                 // uniform: not emitted
  const int W = a.W, H = a.H, wpr = a.words_per_row;
  const int64_t wh = (int64_t)W * H;
  const int64_t hw = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    a.index_out[(a.index_idx[1] + slot) & a.index_mask] = a.frame_base + j;
  if (hw >= 2 * (int64_t)H * wpr) return;
  const int64_t wi = hw >> 1;
  const int half = (int)(hw & 1);
  const int y = (int)(wi / wpr), c = (int)(wi - (int64_t)y * wpr);
  const uint32_t o = a.bits[j * (int64_t)H * wpr + wi] >> (4 * half);
  const int x = c * 32 + 16 * half;
  uint8_t *dst = a.out + ((a.out_idx[1] + slot) & a.out_mask) * wh + (int64_t)y * W + x;
  uint32_t v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = ((o >> k) & 0x01010101u) * 0xFFu;   // dword k: pixel 4k + j <- bit 8j + k
  if (FAST) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 val = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(val, reinterpret_cast<u32x4 *>(dst));
  } else {
    const int n = min(16, W - x);
    for (int i = 0; i < n; ++i) dst[i] = (uint8_t)(v[i >> 2] >> (8 * (i & 3)));
  }
}

// Exclusive scan of emit flags: emit_off[j] = output slot of firing j or -1,
// emit_off[n] = number of emitted frames.  One wavefront, ballot-based.
__global__ __launch_bounds__(64) void k_emit_scan(const int32_t *count, int64_t n, int64_t thresh,
                                                  int64_t *off) {
  const int lane = threadIdx.x;
  const uint64_t below_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
  int64_t carry = 0;
  for (int64_t c = 0; c < n; c += 64) {
    const int64_t j = c + lane;
    const bool f = j < n && 1000 * (int64_t)count[j] >= thresh;
    const uint64_t bal = __ballot(f);
    if (j < n) off[j] = f ? carry + __popcll(bal & below_mask) : -1;
    carry += __popcll(bal);
  }
  if (lane == 0) off[n] = carry;
}

__global__ void k_motion_commit(const int64_t *emit_off, int64_t n, int64_t *cur_idx, int64_t *prev_idx,
                                int64_t *out_idx, int64_t *index_idx, int32_t *err) {
  if (threadIdx.x != 0) return;
  const int64_t total = emit_off[n];
  cur_idx[0] += n;
  if (prev_idx) prev_idx[0] += n;
  out_idx[1] += total;
  index_idx[1] += total;
  check_chan(cur_idx, err);
  if (prev_idx) check_chan(prev_idx, err);
  check_chan(out_idx, err);
  check_chan(index_idx, err);
}

constexpr int MOTION_ROWS = 32;  // rows per band

template <int F>
static hipError_t launch_bits(const MotionArgs &a, hipStream_t s, int64_t items, int rows, int n_bands,
                              int n_chunks) {
  if (items > 0x7ffffff0) return hipErrorInvalidValue;
  const bool fast = (a.W % 32) == 0 && ((int64_t)a.W * a.H) % 16 == 0;
  const dim3 grid((unsigned)((items + 7) / 8 * 8));
  if (fast)
    hipLaunchKernelGGL((k_motion_bits<F, true>), grid, dim3(64), 0, s, a, rows, n_bands, n_chunks, (int)items);
  else
    hipLaunchKernelGGL((k_motion_bits<F, false>), grid, dim3(64), 0, s, a, rows, n_bands, n_chunks, (int)items);
  return hipGetLastError();
}

// Frames per wavefront in the self-delay form: F + 1 row loads per F
// frames.  Measured on the 300-frame 1080p workload (bits pass + expand):
// F = 4 0.308 ms, F = 2 0.341 ms, F = 1 0.405 ms: the extra waves of smaller
// F do not pay for their extra frame reads.
constexpr int MOTION_F = 4;

hipError_t launch_motion_count(const MotionArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const int n_chunks = (a.words_per_row + MW_CHUNK - 1) / MW_CHUNK;
  const int rows = MOTION_ROWS;
  const int n_bands = (a.H + rows - 1) / rows;
  if (a.prev) return launch_bits<1>(a, s, (int64_t)n_chunks * n_bands * a.n, rows, n_bands, n_chunks);
  return launch_bits<MOTION_F>(a, s, (int64_t)n_chunks * n_bands * ((a.n + MOTION_F - 1) / MOTION_F), rows,
                               n_bands, n_chunks);
}

hipError_t launch_motion_emit_scan(const int32_t *count, int64_t n, int64_t thresh, int64_t *off,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_emit_scan, dim3(1), dim3(64), 0, s, count, n, thresh, off);
  return hipGetLastError();
}

hipError_t launch_motion_emit(const MotionArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const int64_t halves = 2 * (int64_t)a.H * a.words_per_row;
  const bool fast = (a.W % 32) == 0 && ((int64_t)a.W * a.H) % 16 == 0;
  // grid row n copies the state: 16 bytes per thread cover the frame when
  // the width is a multiple of 32 (halves * 16 = W * H)
  if (a.state_src && !fast) return hipErrorInvalidValue;
  dim3 grid((unsigned)((halves + 255) / 256), (unsigned)(a.n + (a.state_src ? 1 : 0)));
  if (fast)
    hipLaunchKernelGGL(k_motion_expand<true>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_motion_expand<false>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_motion_commit(const int64_t *emit_off, int64_t n, int64_t *cur_idx, int64_t *prev_idx,
                                int64_t *out_idx, int64_t *index_idx, int32_t *err, hipStream_t s) {
  hipLaunchKernelGGL(k_motion_commit, dim3(1), dim3(64), 0, s, emit_off, n, cur_idx, prev_idx, out_idx,
                     index_idx, err);
  return hipGetLastError();
}

}  // namespace dfh
