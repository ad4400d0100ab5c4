// Host unit test of the runtime's device-free arithmetic (host_logic.h),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_logic.py.  Every check compares against a token-by-token
// model: a FIFO as a std::deque and the slot array a channel writes into.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "host_logic.h"

using namespace dfh::host;

static int failures = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      if (failures < 20) std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                    \
    }                                                                \
  } while (0)

// Push and pop random amounts through a channel of map m, writing token
// values into a slot array run by run (next_run) with the delay layout's
// slot-0 copy (fixup_position); every popped value must be the FIFO's.
static void fifo_through_slots(const SlotMap &m, int64_t capacity, std::mt19937_64 &rng) {
  const int64_t slots = m.period ? m.period + (m.delay ? 1 : 0) : m.cap;
  std::vector<int64_t> buf(slots, -1);
  std::deque<int64_t> model;
  int64_t w = 0, r = 0, next = 0;
  if (m.delay) {                                   // the delay token: position 0, slot 0
    buf[0] = -7;
    model.push_back(-7);
    w = 1;
  }
  for (int step = 0; step < 400; ++step) {
    const int64_t room = capacity - (w - r);
    const int64_t k = room ? (int64_t)(rng() % (room + 1)) : 0;
    for (int64_t done = 0; done < k;) {            // write k tokens
      const Run run = next_run(m, w + done, k - done, true);
      CHECK(run.count >= 1 && run.slot >= 0 && run.slot + run.count <= slots);
      for (int64_t i = 0; i < run.count; ++i) {
        CHECK(write_slot(m, w + done + i) == run.slot + i);
        buf[run.slot + i] = next + done + i;
      }
      done += run.count;
    }
    if (m.delay) {
      const int64_t f = fixup_position(w, k, m.period);
      if (f >= 0) buf[0] = buf[m.period];
    }
    for (int64_t i = 0; i < k; ++i) model.push_back(next + i);
    next += k;
    w += k;
    const int64_t avail = w - r;
    const int64_t n = avail ? (int64_t)(rng() % (avail + 1)) : 0;
    for (int64_t done = 0; done < n;) {            // read n tokens
      const Run run = next_run(m, r + done, n - done, false);
      CHECK(run.count >= 1 && run.slot >= 0 && run.slot + run.count <= slots);
      for (int64_t i = 0; i < run.count; ++i) {
        CHECK(read_slot(m, r + done + i) == run.slot + i);
        CHECK(buf[run.slot + i] == model.front());
        model.pop_front();
      }
      done += run.count;
    }
    r += n;
  }
}

int main() {
  std::mt19937_64 rng(12345);
  for (int64_t v : {1LL, 2LL, 3LL, 1000LL, 1024LL, 1025LL}) {
    const int64_t p = next_pow2(v);
    CHECK(p >= v && (p & (p - 1)) == 0 && (p == 1 || p / 2 < v));
  }
  for (int64_t cap : {1, 2, 8, 64}) {
    SlotMap m;
    m.cap = cap;
    fifo_through_slots(m, cap, rng);
  }
  for (int64_t rate = 1; rate <= 5; ++rate) {
    SlotMap dbl;
    dbl.period = 2 * rate;                          // double buffer of Eq. (1)
    fifo_through_slots(dbl, 2 * rate, rng);
    SlotMap tri;
    tri.period = 3 * rate;                          // delay-token buffer of Fig. 2
    tri.delay = true;
    fifo_through_slots(tri, 3 * rate, rng);
  }
  // the Fig. 2 pattern at rate 4: writes of four fill 1..4, 5..8, 9..12, 1..4
  SlotMap f2;
  f2.period = 12;
  f2.delay = true;
  CHECK(write_slot(f2, 1) == 1 && write_slot(f2, 12) == 12 && write_slot(f2, 13) == 1);
  CHECK(read_slot(f2, 0) == 0 && read_slot(f2, 11) == 11 && read_slot(f2, 12) == 0);
  CHECK(fixup_position(9, 4, 12) == 12 && fixup_position(1, 4, 12) == -1 && fixup_position(0, 3, 12) == -1);
  // fixup_position against brute force
  for (int64_t P = 1; P <= 9; ++P)
    for (int64_t pos = 0; pos < 40; ++pos)
      for (int64_t n = 0; n <= P; ++n) {
        int64_t want = -1;
        for (int64_t q = pos; q < pos + n; ++q)
          if (q != 0 && q % P == 0) { want = q; break; }
        CHECK(fixup_position(pos, n, P) == want);
      }
  // reused_batch against brute force: batches [base + k n, base + (k+1) n)
  for (int64_t cap : {4, 8, 16})
    for (int64_t n = 1; n <= 8; ++n)
      for (int64_t base = 0; base < 5; ++base)
        for (int64_t last = 0; last < 60; ++last) {
          const int64_t p = last - cap;
          int64_t want = -1;
          for (int64_t k = 0; k < 100 && p >= base; ++k)
            if (p >= base + k * n && p < base + (k + 1) * n) { want = k; break; }
          CHECK(reused_batch(last, cap, base, n) == want);
        }
  std::printf("host logic: %s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
