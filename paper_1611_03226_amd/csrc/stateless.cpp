// Stateless device-pointer entry points (used by the autograd binding):
// independent predistortion actors over the rows of a [n_streams][len]
// array, their coefficient adjoint, and the memory-polynomial input adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "dfhip.h"
#include "runtime.h"

using namespace dfh;

namespace {

df_status check_dpd_shape(int64_t S, int64_t len, int64_t r, int32_t B_max, int32_t M, int32_t hist) {
  if (S < 0 || len < 0) return fail(nullptr, DF_EINVAL, "negative size");
  if (r < 1 || len % r) return fail(nullptr, DF_EINVAL, "len %lld is not a multiple of r %lld", (long long)len,
                                    (long long)r);
  if (B_max < 1 || B_max > kMaxBranches) return fail(nullptr, DF_EINVAL, "B_max outside 1..%d", kMaxBranches);
  if (M < 1 || M > kMaxTaps) return fail(nullptr, DF_EINVAL, "M outside 1..%d", kMaxTaps);
  if (r < M - 1) return fail(nullptr, DF_EINVAL, "r must be >= M-1");
  if (hist != DF_HIST_BRANCH && hist != DF_HIST_SHARED) return fail(nullptr, DF_EINVAL, "bad history mode");
  return DF_OK;
}

// Per-firing tables for explicit control tokens (stream-ordered scratch).
struct Tables {
  int32_t *B = nullptr;
  int64_t *prev = nullptr;
  int64_t *off = nullptr;
  void *grp = nullptr;       // scan scratch
  int64_t n = 0;
};

hipError_t make_tables(const int32_t *ctrl, int64_t S, int64_t nf, int64_t r, int32_t B_max, int32_t hist,
                       hipStream_t s, Tables *t, bool offsets = false) {
  t->n = S * nf;
  hipError_t e = hipMallocAsync((void **)&t->B, sizeof(int32_t) * std::max<int64_t>(t->n, 1), s);
  if (e != hipSuccess) return e;
  e = hipMallocAsync((void **)&t->prev, sizeof(int64_t) * std::max<int64_t>(t->n, 1) * B_max, s);
  if (e != hipSuccess) return e;
  if (offsets) {
    e = hipMallocAsync((void **)&t->off, sizeof(int64_t) * std::max<int64_t>(t->n, 1) * B_max, s);
    if (e != hipSuccess) return e;
  }
  e = hipMallocAsync(&t->grp, scan_scratch_bytes(S, nf, B_max, false), s);
  if (e != hipSuccess) return e;
  ScanArgs sa{};
  sa.ctrl = ctrl;
  sa.ctrl_idx = nullptr;
  sa.ctrl_mask = -1;
  sa.seg_firings = nf;
  sa.n_segs = (int32_t)S;
  sa.B_max = B_max;
  sa.hist_mode = hist;
  sa.B_out = t->B;
  sa.prev_out = t->prev;
  sa.off_out = t->off;
  scan_scratch_assign(sa, t->grp, false);
  sa.stride = t->n;
  sa.r = r;
  return launch_scan(sa, s);
}

void free_tables(Tables *t, hipStream_t s) {
  if (t->B) (void)hipFreeAsync(t->B, s);
  if (t->prev) (void)hipFreeAsync(t->prev, s);
  if (t->off) (void)hipFreeAsync(t->off, s);
  if (t->grp) (void)hipFreeAsync(t->grp, s);
}

// outputs per adjoint workgroup (2048 balances the lane reduction against occupancy)
// Outputs per workgroup of the coefficient adjoint (processed in staged
// chunks; the span sets how many samples each lane reduction serves).
int adj_span(int64_t r) { return (int)std::min<int64_t>(2 * 2048, r); }

}  // namespace

// Bytes of each scratch region one forward call needs (see FwdScratch).
FwdScratchSize dfh::dpd_forward_scratch_size(int64_t S, int64_t len, int64_t r, int32_t B_max, int32_t M,
                                             bool with_ctrl) {
  FwdScratchSize z{};
  const int64_t L1 = std::max(M - 1, 1);
  if (!with_ctrl) {
    z.corr = sizeof(float2) * L1 * S;
    return z;
  }
  const int64_t nf = len / r, n = std::max<int64_t>(S * nf, 1);
  z.B = sizeof(int32_t) * n;
  z.prev = sizeof(int64_t) * n * B_max;
  z.grp = scan_scratch_bytes(S, nf, B_max, false);
  z.corr = sizeof(float2) * L1 * n;
  return z;
}

// The forward kernel chain over caller-provided scratch: control intake and
// offset scan (with control tokens), head corrections, tiled body.
hipError_t dfh::dpd_forward_enqueue(const FwdScratch &sc, hipStream_t s, const void *x, const int32_t *ctrl,
                                    const void *h, void *y, int64_t S, int64_t len, int64_t r, int32_t B_max,
                                    int32_t M, int32_t hist) {
  DpdArgs a{};
  a.x = (const float2 *)x;
  a.x_mask = -1;
  a.y = (float2 *)y;
  a.y_mask = -1;
  a.h = (const float2 *)h;
  a.B_max = B_max;
  a.M = M;
  a.corr = sc.corr;
  a.mx = dpd_body_mx_env();
  if (!ctrl) {
    // All branches active in every firing: a row is one convolution.
    a.B_const = B_max;
    a.seg_firings = 1;
    a.n_firings = S;
    a.r = len;
    hipError_t e = launch_dpd_heads(a, s);
    if (e == hipSuccess) e = launch_dpd_body(a, s, 0, 4);
    return e;
  }
  const int64_t nf = len / r, n = S * nf;
  ScanArgs sa{};
  sa.ctrl = ctrl;
  sa.ctrl_idx = nullptr;
  sa.ctrl_mask = -1;
  sa.seg_firings = nf;
  sa.n_segs = (int32_t)S;
  sa.B_max = B_max;
  sa.hist_mode = hist;
  sa.B_out = sc.B;
  sa.prev_out = sc.prev;
  sa.off_out = nullptr;
  scan_scratch_assign(sa, sc.grp, false);
  sa.stride = n;
  sa.r = r;
  hipError_t e = launch_scan(sa, s);
  if (e != hipSuccess) return e;
  a.B = sc.B;
  a.prev = sc.prev;
  a.prev_stride = n;
  a.seg_firings = nf;
  a.n_firings = n;
  a.r = r;
  e = launch_dpd_heads(a, s);
  if (e == hipSuccess) e = launch_dpd_body(a, s, 0, 4);
  return e;
}

df_status dfh::check_dpd_forward_args(const void *x, const void *h, void *y, int64_t S, int64_t len, int64_t r,
                                      int32_t B_max, int32_t M, int32_t hist, bool *nothing) {
  df_status st = check_dpd_shape(S, len, r, B_max, M, hist);
  if (st) return st;
  *nothing = S == 0 || len == 0;
  if (!*nothing && (!x || !h || !y)) return fail(nullptr, DF_EINVAL, "null pointer");
  return DF_OK;
}

extern "C" df_status df_dpd_forward(void *stream, const void *x, const int32_t *ctrl, const void *h, void *y,
                                    int64_t S, int64_t len, int64_t r, int32_t B_max, int32_t M, int32_t hist) {
  bool nothing = false;
  df_status st = check_dpd_forward_args(x, h, y, S, len, r, B_max, M, hist, &nothing);
  if (st || nothing) return st;
  hipStream_t s = (hipStream_t)stream;
  const FwdScratchSize z = dpd_forward_scratch_size(S, len, r, B_max, M, ctrl != nullptr);
  FwdScratch sc{};
  hipError_t e = hipMallocAsync((void **)&sc.corr, z.corr, s);
  if (e == hipSuccess && z.B) e = hipMallocAsync((void **)&sc.B, z.B, s);
  if (e == hipSuccess && z.prev) e = hipMallocAsync((void **)&sc.prev, z.prev, s);
  if (e == hipSuccess && z.grp) e = hipMallocAsync((void **)&sc.grp, z.grp, s);
  if (e == hipSuccess) e = dpd_forward_enqueue(sc, s, x, ctrl, h, y, S, len, r, B_max, M, hist);
  for (void *p : {(void *)sc.corr, (void *)sc.B, (void *)sc.prev, (void *)sc.grp})
    if (p) (void)hipFreeAsync(p, s);
  if (e != hipSuccess) return fail_hip(nullptr, e, "df_dpd_forward");
  return DF_OK;
}

extern "C" df_status df_dpd_forward_network(void *stream, const void *x, const int32_t *ctrl, const void *h, void *y,
                                            int64_t S, int64_t len, int64_t r, int32_t B_max, int32_t M,
                                            int32_t ctrl_mode) {
  df_status st = check_dpd_shape(S, len, r, B_max, M, DF_HIST_BRANCH);
  if (st) return st;
  if (ctrl_mode != DF_CTRL_COUNT && ctrl_mode != DF_CTRL_MASK) return fail(nullptr, DF_EINVAL, "bad ctrl_mode");
  if (S == 0 || len == 0) return DF_OK;
  if (!x || !ctrl || !h || !y) return fail(nullptr, DF_EINVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nf = len / r;
  Tables t;
  float2 *chan = nullptr, *firo = nullptr;
  const size_t chan_bytes = sizeof(float2) * (size_t)B_max * (size_t)S * (size_t)len;
  hipError_t e = hipSuccess;
  if (ctrl_mode == DF_CTRL_COUNT) {
    e = make_tables(ctrl, S, nf, r, B_max, DF_HIST_BRANCH, s, &t, true);
  } else {
    t.n = S * nf;
    e = hipMallocAsync((void **)&t.B, sizeof(int32_t) * t.n, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&t.off, sizeof(int64_t) * t.n * B_max, s);
  }
  if (e == hipSuccess) e = hipMallocAsync((void **)&chan, chan_bytes, s);
  if (e == hipSuccess) e = hipMallocAsync((void **)&firo, chan_bytes, s);
  if (e == hipSuccess) {
    DpdNetArgs a{};
    a.x = (const float2 *)x;
    a.y = (float2 *)y;
    a.h = (const float2 *)h;
    a.B = t.B;
    a.off = t.off;
    a.stride = t.n;
    a.nf = nf;
    a.r = r;
    a.S = S;
    a.B_max = B_max;
    a.M = M;
    a.chan = chan;
    a.firo = firo;
    a.mask_mode = ctrl_mode == DF_CTRL_MASK;
    if (a.mask_mode) e = launch_mask_tables(ctrl, t.B, t.off, a, s);
    if (e == hipSuccess) e = launch_dpd_network(a, s);
  }
  if (chan) (void)hipFreeAsync(chan, s);
  if (firo) (void)hipFreeAsync(firo, s);
  free_tables(&t, s);
  if (e != hipSuccess) return fail_hip(nullptr, e, "df_dpd_forward_network");
  return DF_OK;
}

extern "C" int64_t df_dpd_coeff_adjoint_work_bytes(int64_t S, int64_t len, int64_t r, int32_t B_max, int32_t M) {
  if (S <= 0 || len <= 0 || r <= 0 || B_max <= 0 || M <= 0) return 0;
  // Same firing decomposition as df_dpd_coeff_adjoint with explicit control
  // (the all-active case needs no more).
  const int64_t nf = len / r;
  const int c1 = adj_span(r);
  const int64_t blocks_ctrl = S * nf * ((r + c1 - 1) / c1);
  const int c2 = adj_span(len);
  const int64_t blocks_all = S * ((len + c2 - 1) / c2);
  return std::max(blocks_ctrl, blocks_all) * B_max * M * (int64_t)sizeof(float2);
}

extern "C" df_status df_dpd_coeff_adjoint(void *stream, const void *x, const int32_t *ctrl, const void *G,
                                         void *grad_h, int64_t S, int64_t len, int64_t r, int32_t B_max, int32_t M,
                                         int32_t hist, void *work, int64_t work_bytes) {
  df_status st = check_dpd_shape(S, len, r, B_max, M, hist);
  if (st) return st;
  if (!grad_h) return fail(nullptr, DF_EINVAL, "null grad_h");
  if (S > 0 && len > 0 && (!x || !G)) return fail(nullptr, DF_EINVAL, "null pointer");
  const int64_t need = df_dpd_coeff_adjoint_work_bytes(S, len, r, B_max, M);
  if (need > 0 && (!work || work_bytes < need))
    return fail(nullptr, DF_EINVAL, "work buffer of %lld bytes needed", (long long)need);
  hipStream_t s = (hipStream_t)stream;
  AdjArgs a{};
  a.x = (const float2 *)x;
  a.G = (const float2 *)G;
  a.B_max = B_max;
  a.M = M;
  a.partial = (float2 *)work;
  a.grad = (float2 *)grad_h;
  Tables t;
  hipError_t e = hipSuccess;
  if (S == 0 || len == 0) {
    a.n_firings = 0;
    a.blocks_per_firing = 1;
    e = launch_adj(a, s);
  } else if (!ctrl) {
    a.seg_firings = 1;
    a.n_firings = S;
    a.r = len;
    a.span = adj_span(len);
    a.blocks_per_firing = (int32_t)((len + a.span - 1) / a.span);
    e = launch_adj(a, s);
  } else {
    const int64_t nf = len / r;
    e = make_tables(ctrl, S, nf, r, B_max, hist, s, &t);
    if (e == hipSuccess) {
      a.B = t.B;
      a.prev = t.prev;
      a.prev_stride = t.n;
      a.seg_firings = nf;
      a.n_firings = S * nf;
      a.r = r;
      a.span = adj_span(r);
      a.blocks_per_firing = (int32_t)((r + a.span - 1) / a.span);
      e = launch_adj(a, s);
    }
    free_tables(&t, s);
  }
  if (e != hipSuccess) return fail_hip(nullptr, e, "df_dpd_coeff_adjoint");
  return DF_OK;
}

extern "C" df_status df_mp_input_adjoint(void *stream, const void *u, const void *a, const void *g, void *Gu,
                                        int64_t S, int64_t len, int32_t K, int32_t Q) {
  if (S < 0 || len < 0) return fail(nullptr, DF_EINVAL, "negative size");
  if (K < 1 || K > kMaxBranches || Q < 1 || Q > kMaxTaps) return fail(nullptr, DF_EINVAL, "bad K or Q");
  if (S == 0 || len == 0) return DF_OK;
  if (!u || !a || !g || !Gu) return fail(nullptr, DF_EINVAL, "null pointer");
  hipError_t e = launch_mp_adj((const float2 *)u, (const float2 *)a, (const float2 *)g, (float2 *)Gu, S, len, K, Q,
                               (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(nullptr, e, "df_mp_input_adjoint");
  return DF_OK;
}

extern "C" df_status df_hbm_ref(void *stream, int32_t mode, const void *src, void *dst, int64_t bytes) {
  if (mode < 0 || mode > 3) return fail(nullptr, DF_EINVAL, "mode must be 0..3");
  if (bytes < 0 || bytes % 16) return fail(nullptr, DF_EINVAL, "bytes must be a non-negative multiple of 16");
  if (bytes == 0) return DF_OK;
  if (!dst || (mode != 2 && !src)) return fail(nullptr, DF_EINVAL, "null pointer");
  if (((uintptr_t)src | (uintptr_t)dst) % 16) return fail(nullptr, DF_EINVAL, "pointers must be 16-byte aligned");
  hipError_t e = launch_hbm_ref(mode, src, dst, bytes, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(nullptr, e, "df_hbm_ref");
  return DF_OK;
}

extern "C" df_status df_stream_copy(void *stream, const void *src, void *dst, int64_t bytes) {
  if (bytes < 0 || bytes % 16) return fail(nullptr, DF_EINVAL, "bytes must be a non-negative multiple of 16");
  if (bytes == 0) return DF_OK;
  if (!src || !dst) return fail(nullptr, DF_EINVAL, "null pointer");
  if (((uintptr_t)src | (uintptr_t)dst) % 16) return fail(nullptr, DF_EINVAL, "pointers must be 16-byte aligned");
  hipError_t e = launch_stream_copy(src, dst, bytes, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(nullptr, e, "df_stream_copy");
  return DF_OK;
}
