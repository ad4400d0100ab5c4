// Host-side arithmetic of the runtime that involves no device: channel slot
// maps and the runs of consecutive slots a host copy covers, the slot-0 copy
// of the paper's delay-token layout, and the batch whose ring slots a
// streamed write reuses.  Plain C++ (no HIP), so that a host unit test can
// build it under AddressSanitizer / UndefinedBehaviorSanitizer.
#pragma once

#include <stdint.h>

namespace dfh {
namespace host {

inline int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// A channel's slots: a ring of `cap` (a power of two) slots, or the paper's
// layout of Sec. 3.2 with period P (2r, or 3r with one delay token: 3r + 1
// slots, writes filling slots 1..3r in turn, reads taking 0..3r-1).
struct SlotMap {
  int64_t cap = 0;      // ring capacity (period == 0)
  int64_t period = 0;   // paper layout period, 0 for a ring
  bool delay = false;   // paper layout with its one delay token
};

inline int64_t read_slot(const SlotMap &m, int64_t p) { return m.period ? p % m.period : (p & (m.cap - 1)); }

inline int64_t write_slot(const SlotMap &m, int64_t p) {
  if (!m.period) return p & (m.cap - 1);
  return m.delay ? 1 + (p - 1) % m.period : p % m.period;
}

// Exclusive end of the slots one run of a host copy may cover before the
// access pattern wraps to its first slot.
inline int64_t run_end(const SlotMap &m, bool to_ring) {
  if (!m.period) return m.cap;
  return (to_ring && m.delay) ? m.period + 1 : m.period;
}

// The next run of a copy of tokens [q, q + left): its first slot and length.
struct Run {
  int64_t slot, count;
};
inline Run next_run(const SlotMap &m, int64_t q, int64_t left, bool to_ring) {
  const int64_t slot = to_ring ? write_slot(m, q) : read_slot(m, q);
  const int64_t room = run_end(m, to_ring) - slot;
  return Run{slot, left < room ? left : room};
}

// Delay-token layout: the position in [pos, pos + n) whose write fills slot
// P (so that slot P must then be copied to slot 0), or -1.  Position 0 is the
// delay token itself and is never written.  With n <= P (what admission
// allows) there is at most one.
inline int64_t fixup_position(int64_t pos, int64_t n, int64_t P) {
  if (n <= 0 || P <= 0) return -1;
  const int64_t first = pos + ((P - (pos % P)) % P);   // first multiple of P at or after pos
  return (first < pos + n && first != 0) ? first : -1;
}

// Streamed writes: batches of n tokens start at `base`, n apart; a write
// whose last position is `last` reuses the ring slots of the batch holding
// position last - cap, if that position belongs to a batch.
inline int64_t reused_batch(int64_t last, int64_t cap, int64_t base, int64_t n) {
  const int64_t p = last - cap;
  return p < base ? -1 : (p - base) / n;
}

}  // namespace host
}  // namespace dfh
