// Packed-byte arithmetic for the 8-bit frame actors of the motion-detection
// pipeline (Sec. 4.1): four pixels per 32-bit word, split into two words of
// 16-bit lanes (even pixels 0 and 2, odd pixels 1 and 3) so that sums and
// comparisons of up to 16 bits never carry into the neighbouring pixel.
// Host-compilable so the same code can be checked on the CPU.
#pragma once

#include <stdint.h>

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

namespace dfh {
namespace swar {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr uint32_t kLo = 0x00FF00FFu;

// Low 32 bits of the 64-bit value hi:lo shifted right by s (0 <= s < 32).
__host__ __device__ inline uint32_t funnel(uint32_t hi, uint32_t lo, int s) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> s);
}

// Byte permute: byte i of the result is byte sel[i] (0..7) of the 8-byte
// pool lo (bytes 0..3) : hi (bytes 4..7); a selector byte of 0x0C gives 0.
__host__ __device__ inline uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_perm(hi, lo, sel);
#else
  const uint64_t pool = ((uint64_t)hi << 32) | lo;
  uint32_t r = 0;
  for (int i = 0; i < 4; ++i) {
    const uint32_t s = (sel >> (8 * i)) & 0xFF;
    const uint32_t v = s < 8 ? (uint32_t)((pool >> (8 * s)) & 0xFF) : s == 0x0C ? 0u : 0xFFu;
    r |= v << (8 * i);
  }
  return r;
#endif
}

// Selectors for perm() building horizontal windows of the 4 pixels p0..p3
// of word m from its neighbour words l and r.  With `edge` set the pixels
// beyond the frame edge repeat the edge pixel (p-1 = p-2 = p0 on the left,
// p4 = p5 = p3 on the right).
//   perm(m, l, win2_left(e))  = (p-2, p-1, p0, p1)
//   perm(r, m, win2_right(e)) = (p2, p3, p4, p5)
//   perm(m, l, win1_left(e))  = (p-1, p0, p1, p2)
//   perm(r, m, win1_right(e)) = (p1, p2, p3, p4)
__host__ __device__ inline uint32_t win2_left(bool edge) { return edge ? 0x05040404u : 0x05040302u; }
__host__ __device__ inline uint32_t win2_right(bool edge) { return edge ? 0x03030302u : 0x05040302u; }
__host__ __device__ inline uint32_t win1_left(bool edge) { return edge ? 0x06050404u : 0x06050403u; }
__host__ __device__ inline uint32_t win1_right(bool edge) { return edge ? 0x03030201u : 0x04030201u; }

// Horizontal 5-tap binomial sums (1,4,6,4,1) of four pixels p0..p3 given
// the 8-byte window X = (p-2, p-1, p0, p1, p2, p3, p4, p5) as lo (bytes
// 0..3) and hi (bytes 4..7).  Returns the sums of (p0, p2) in *even and of
// (p1, p3) in *odd, one per 16-bit lane (each at most 255*16 = 4080).
__host__ __device__ inline void hsum5(uint32_t lo, uint32_t hi, uint32_t *even, uint32_t *odd) {
  // u[k]: bytes k and k+2 of X in the two 16-bit lanes, one byte permute
  // each (selector 0x0C writes a zero byte)
  const uint32_t u0 = lo & kLo;
  const uint32_t u1 = perm(hi, lo, 0x0C030C01u);
  const uint32_t u2 = perm(hi, lo, 0x0C040C02u);
  const uint32_t u3 = perm(hi, lo, 0x0C050C03u);
  const uint32_t u4 = hi & kLo;
  const uint32_t u5 = perm(hi, lo, 0x0C070C05u);
  *even = u0 + u4 + 4u * (u1 + u3) + 6u * u2;
  *odd = u1 + u5 + 4u * (u2 + u4) + 6u * u3;
}

// Vertical 5-tap binomial sum of horizontal sums, rounded (s + 128) >> 8,
// back to one byte per 16-bit lane.  Lanes stay below 65536: 4080*16 + 128.
__host__ __device__ inline uint32_t vround5(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e) {
  // 6c as 4c + 2c: c exceeds 24 bits, and a full 32-bit multiply is slow
  const uint32_t s = a + e + ((b + d + c) << 2) + (c << 1) + 0x00800080u;
  return (s >> 8) & kLo;
}

// Re-interleave even-pixel and odd-pixel lanes into one word of 4 pixels.
__host__ __device__ inline uint32_t interleave(uint32_t even, uint32_t odd) { return even | (odd << 8); }

// 0xFF in every byte lane where |a - b| > t, else 0 (t in 0..255).
__host__ __device__ inline uint32_t absdiff_gt(uint32_t a, uint32_t b, uint32_t t) {
  const uint32_t bias = (255u - t) * 0x00010001u;
  uint32_t m[2];
  for (int k = 0; k < 2; ++k) {
    const uint32_t x = (a >> (8 * k)) & kLo, y = (b >> (8 * k)) & kLo;
    // each lane: 256 + x - y (1..511), and 256 + y - x; + (255 - t) reaches
    // 512 (bit 9) exactly when the difference exceeds t
    const uint32_t p = ((x | 0x01000100u) - y + bias) >> 9;
    const uint32_t q = ((y | 0x01000100u) - x + bias) >> 9;
    m[k] = ((p | q) & 0x00010001u) * 0xFFu;
  }
  return interleave(m[0], m[1]);
}

__host__ __device__ inline u16x2 as_u16x2(uint32_t v) {
  u16x2 r;
  r.x = (unsigned short)(v & 0xFFFFu);
  r.y = (unsigned short)(v >> 16);
  return r;
}
__host__ __device__ inline uint32_t from_u16x2(u16x2 v) { return (uint32_t)v.x | ((uint32_t)v.y << 16); }

__host__ __device__ inline u16x2 vmin(u16x2 a, u16x2 b) { return __builtin_elementwise_min(a, b); }
__host__ __device__ inline u16x2 vmax(u16x2 a, u16x2 b) { return __builtin_elementwise_max(a, b); }

// Median of five values per 16-bit lane: the median of e and the two middle
// candidates max(min(a,b), min(c,d)) and min(max(a,b), max(c,d)).
__host__ __device__ inline u16x2 med5(u16x2 a, u16x2 b, u16x2 c, u16x2 d, u16x2 e) {
  const u16x2 f = vmax(vmin(a, b), vmin(c, d));
  const u16x2 g = vmin(vmax(a, b), vmax(c, d));
  return vmax(vmin(e, f), vmin(vmax(e, f), g));
}

// Threshold of pixels given in split form (even pixels 0, 2 in the 16-bit
// lanes of *E, odd pixels 1, 3 in *O, values 0..255): 0xFF in every byte
// where |cur - prev| > t (t in 0..255), else 0.  |d| + (255 - t) stays below
// 512, so bit 8 of each lane is the comparison.
__host__ __device__ inline uint32_t thres_split(uint32_t cE, uint32_t cO, uint32_t pE, uint32_t pO, uint32_t t) {
  const uint32_t bias = (255u - t) * 0x00010001u;
  const u16x2 ce = as_u16x2(cE), co = as_u16x2(cO), pe = as_u16x2(pE), po = as_u16x2(pO);
  const uint32_t dE = from_u16x2(vmax(ce, pe) - vmin(ce, pe));
  const uint32_t dO = from_u16x2(vmax(co, po) - vmin(co, po));
  const uint32_t bE = ((dE + bias) >> 8) & 0x00010001u, bO = ((dO + bias) >> 8) & 0x00010001u;
  const uint32_t ones = bE | (bO << 8);     // 0x00 / 0x01 per byte
  return (ones << 8) - ones;                // x 255, modulo 2^32
}

// Median of five 0x00/0xFF byte masks, per byte: with only two values the
// median is the majority, and the min/max network becomes AND/OR.
__host__ __device__ inline uint32_t med5_masks(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e) {
  const uint32_t f = (a & b) | (c & d);
  const uint32_t g = (a | b) & (c | d);
  return (e & f) | ((e | f) & g);
}

// Median of five words of four pixels each, per pixel.
__host__ __device__ inline uint32_t med5_bytes(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e) {
  uint32_t r[2];
  for (int k = 0; k < 2; ++k) {
    const int s = 8 * k;
    const u16x2 m = med5(as_u16x2((a >> s) & kLo), as_u16x2((b >> s) & kLo), as_u16x2((c >> s) & kLo),
                         as_u16x2((d >> s) & kLo), as_u16x2((e >> s) & kLo));
    r[k] = from_u16x2(m);
  }
  return interleave(r[0], r[1]);
}

}  // namespace swar
}  // namespace dfh
