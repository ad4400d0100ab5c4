// Allocation-free variant of the stateless predistortion forward: its
// scratch (branch counts, history sources, scan group table, head
// corrections) lives in a fixed device array of this file instead of
// stream-ordered allocations, for callers that cannot allocate (code under
// HIP graph capture, serving loops that forbid allocation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "common.h"
#include "dfhip.h"
#include "runtime.h"

namespace {

// Largest scratch one call may use: any call of up to 16384 firings with
// n_branches_max <= 16 and n_taps <= 32 fits (at most 9.94 MiB: counts
// 64 KiB, history sources 2 MiB, head corrections 3.9 MiB, group table up
// to 4 MiB when every row is one firing).  Every GPU that runs the library
// holds one copy until the process ends.
constexpr size_t kScratchBytes = size_t(12) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
unsigned char *g_ptr[kMaxDevices] = {};

// The array's device address on the current device, looked up once per
// device with that device current (each GPU has its own copy).
hipError_t scratch_ptr(unsigned char **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = (unsigned char *)p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

using namespace dfh;

extern "C" int64_t df_dpd_forward_noalloc_max_bytes(void) { return (int64_t)kScratchBytes; }

extern "C" df_status df_dpd_forward_noalloc(void *stream, const void *x, const int32_t *ctrl, const void *h,
                                            void *y, int64_t S, int64_t len, int64_t r, int32_t B_max, int32_t M,
                                            int32_t hist) {
  bool nothing = false;
  df_status st = check_dpd_forward_args(x, h, y, S, len, r, B_max, M, hist, &nothing);
  if (st || nothing) return st;
  const FwdScratchSize z = dpd_forward_scratch_size(S, len, r, B_max, M, ctrl != nullptr);
  const size_t need = align256(z.corr) + align256(z.B) + align256(z.prev) + align256(z.grp);
  if (need > kScratchBytes)
    return fail(nullptr, DF_EINVAL,
                "df_dpd_forward_noalloc: this call needs %zu bytes of scratch, the fixed array holds %zu "
                "(use df_dpd_forward)", need, kScratchBytes);
  unsigned char *base = nullptr;
  hipError_t e = scratch_ptr(&base);
  if (e != hipSuccess) return fail_hip(nullptr, e, "df_dpd_forward_noalloc: scratch address");
  FwdScratch sc{};
  size_t off = 0;
  sc.corr = (float2 *)(base + off);
  off += align256(z.corr);
  if (z.B) sc.B = (int32_t *)(base + off);
  off += align256(z.B);
  if (z.prev) sc.prev = (int64_t *)(base + off);
  off += align256(z.prev);
  if (z.grp) sc.grp = base + off;
  e = dpd_forward_enqueue(sc, (hipStream_t)stream, x, ctrl, h, y, S, len, r, B_max, M, hist);
  if (e != hipSuccess) return fail_hip(nullptr, e, "df_dpd_forward_noalloc");
  return DF_OK;
}
