// Adjoints for coefficient adaptation through a memory-polynomial PA.
//
// Gradients use the real-pair convention: for complex z, dL/dRe z + i dL/dIm z.
//
// Coefficient adjoint of the predistortion actor (y linear in h):
//   grad_h[b][m] = sum_n G[n] conj(psi_b(s_b[n-m])),  b < B of n's firing.
// Inside a firing the source sample is branch independent, so with
// z = G[n] conj(x[n-m]) and p = |x[n-m]|^2 each (n, m) pair feeds all
// branches through the running power z p^b.  Taps reaching before a firing
// start read branch b's own history and are added per branch.
// Reduction: fp32 partial sums per workgroup in a fixed order, then an fp64
// sum over workgroups in a fixed order (deterministic, no float atomics).
//
// Input adjoint of v[n] = sum_k sum_q a[k][q] phi_k(u[n-q]),
// phi_k(u) = |u|^(2k) u: with d phi/du = (k+1) p^k and
// d phi/du* = k p^(k-1) u^2 (p = |u|^2),
//   Gu[n] = sum_q g[n+q] conj(A_q) + conj(g[n+q]) Bw_q u^2,
//   A_q = sum_k a[k][q] (k+1) p^k,  Bw_q = sum_{k>=1} a[k][q] k p^(k-1).
#include "common.h"

namespace dfh {


__device__ __forceinline__ int64_t adj_prev(const AdjArgs &a, int b, int64_t g) {
  if (a.prev) return a.prev[(int64_t)b * a.prev_stride + g];
  return (g % a.seg_firings) ? g - 1 : -1;
}

// Lane reduce-scatter of N values per lane over the 64 lanes of a
// wavefront, in six steps; step k pairs each lane with a partner that
// differs in lane bit 32 >> k (and agrees in the bits split before): the
// lane with that bit set keeps the upper half of its values (padded to an
// even count with zeros), the other the lower half, each adding the
// partner's copy.  Steps 0 and 1 pair lanes 32 and 16 apart with the
// permlane swaps (a swap and an add per kept value); steps 2..5 use the
// DPP row mirror (lane 15 - l), half-row mirror (7 - l) and quad
// permutations (l ^ 2, l ^ 1) as partners (two selects and an add).  The
// partners' lane masks 32, 16, 15, 7, 2, 1 are independent, so after the
// six steps every kept value is summed over all 64 lanes exactly once, in
// a fixed order.
constexpr int rs_half(int n) { return (n + 1) / 2; }

template <int STEP, int N, int CAP>
__device__ __forceinline__ void rs_steps(float (&v)[CAP], int lane) {
  constexpr int H = rs_half(N);
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float lo = v[i];
    const float hi = i + H < N ? v[i + H] : 0.f;
    if constexpr (STEP < 2) {
      const auto sw = STEP == 0 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false)
                                : __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
      v[i] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
    } else {
      constexpr int ctrl = STEP == 2 ? 0x140 : STEP == 3 ? 0x141 : STEP == 4 ? 0x4E : 0xB1;
      const bool up = (lane & (32 >> STEP)) != 0;
      const float send = up ? lo : hi, keep = up ? hi : lo;
      v[i] = keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), ctrl, 0xF, 0xF, false));
    }
  }
  if constexpr (STEP < 5) rs_steps<STEP + 1, H>(v, lane);
}

// Values a lane holds after the six steps, and the original index of its
// j-th one (-1 for padding).
template <int N>
struct RsPlan {
  static constexpr int n0 = N, n1 = rs_half(n0), n2 = rs_half(n1), n3 = rs_half(n2), n4 = rs_half(n3),
                       n5 = rs_half(n4), kept = rs_half(n5);
  __device__ static int index(int j, int lane) {
    const int cnt[6] = {n0, n1, n2, n3, n4, n5};
    int t = j;
    bool ok = true;
    for (int k = 5; k >= 0; --k) {
      if (lane & (32 >> k)) t += rs_half(cnt[k]);
      ok = ok && t < cnt[k];
    }
    return ok ? t : -1;
  }
};

// Taps per wavefront of the coefficient adjoint for BM branches (8 taps,
// with twice the accumulators and half the wavefronts per SIMD, measured
// slower at 10 branches).
constexpr int adj_tpw(int) { return 4; }

// One workgroup per (firing, span of input samples); one wavefront per
// group of TPW taps.  Every (sample, output) pair with the output in the
// firing is counted by the workgroup that owns the sample (pairs with a
// sample before the firing start are added at the end from the branch
// histories).  The span is processed in chunks of four samples per thread
// staged in LDS with the G values of the outputs they reach, and lane l of
// a wavefront takes samples l, l+64, ... of each chunk.  For its sample a
// lane forms p^b once and accumulates G[s+m] conj(x_s) p^b into TPW taps x
// BM branches of independent registers; after the span the wavefront
// reduces over lanes (fixed order).  The next chunk's loads are in flight
// (in registers) while the current one is processed; a chunk's G window
// starts with the last M+TPW-2 values of the previous one.
template <int BM, int TPW>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(BM <= 10 ? 4 : 1))) void k_adj_partial(
    AdjArgs a) {
  extern __shared__ float2 lds[];
  const int M = a.M;
  const int64_t g = blockIdx.x / a.blocks_per_firing;
  const int64_t c = blockIdx.x - g * a.blocks_per_firing;
  const int64_t s0 = c * a.span;
  const int64_t s1 = min(s0 + a.span, a.r);
  const uint32_t set = a.B ? (uint32_t)a.B[g] : prefix_set(BM);
  const int B = set_len(set);
  const int64_t xb = g * a.r;
  // chunk of C samples at n0: sx[i] = x[n0+i] (zero past the span), sg[o] =
  // G[n0+o] for o < C+K (zero past the firing); K = M+TPW-2 covers the taps
  // of the last wavefront's group past M, whose sums are dropped
  const int nt = blockDim.x, tid = threadIdx.x;
  const int C = a.chunk;                  // 4 * nt, a multiple of 64
  const int K = M + TPW - 2;
  float2 *sx = lds;
  float2 *sg = lds + C;
  float2 *red = sg + C + K;               // [BM][M] reduced sums
  const int lane = threadIdx.x & 63;
  const int m0 = (threadIdx.x >> 6) * TPW;  // first tap of this wavefront
  constexpr int NV = 2 * TPW * BM;        // TPW taps x BM branches x (re, im)
  float v[NV];                            // v[q*2BM + 2b + c]
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = 0.f;
  float2 carry = make_float2(0.f, 0.f);   // sg[tid] (tid < K) of the next chunk
  if (tid < K && s0 + tid < a.r) carry = a.G[xb + s0 + tid];
  float2 rx[4], rg[4];                    // the next chunk's x[n0 + j*nt + tid], G[n0 + K + j*nt + tid]
  const auto fetch = [&](int64_t n0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t n = n0 + j * nt + tid;
      rx[j] = n < s1 ? a.x[xb + n] : make_float2(0.f, 0.f);
      rg[j] = n + K < a.r ? a.G[xb + n + K] : make_float2(0.f, 0.f);
    }
  };
  fetch(s0);
  for (int64_t n0 = s0; n0 < s1; n0 += C) {
    if (tid < K) sg[tid] = carry;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sx[j * nt + tid] = rx[j];
      sg[K + j * nt + tid] = rg[j];
    }
    __syncthreads();
    if (n0 + C < s1) fetch(n0 + C);
    // sample n0 + i, output n0 + i + m
#pragma unroll 2
    for (int i = lane; i < C; i += 64) {
      const float2 xv = sx[i];
      const float p = fmaf(xv.x, xv.x, xv.y * xv.y);
      float pw[BM];
      pw[0] = 1.f;
#pragma unroll
      for (int b = 1; b < BM; ++b) pw[b] = pw[b - 1] * p;
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        const float2 gv = sg[i + m0 + q];
        const float zr = fmaf(gv.x, xv.x, gv.y * xv.y);     // G conj(x)
        const float zi = fmaf(gv.y, xv.x, -(gv.x * xv.y));
#pragma unroll
        for (int b = 0; b < BM; ++b) {
          v[q * 2 * BM + 2 * b] = fmaf(zr, pw[b], v[q * 2 * BM + 2 * b]);
          v[q * 2 * BM + 2 * b + 1] = fmaf(zi, pw[b], v[q * 2 * BM + 2 * b + 1]);
        }
      }
    }
    if (tid < K) carry = sg[C + tid];    // read before anyone rewrites the window
    __syncthreads();
  }
  rs_steps<0, NV>(v, lane);
#pragma unroll
  for (int j = 0; j < RsPlan<NV>::kept; ++j) {
    const int idx = RsPlan<NV>::index(j, lane);
    if (idx < 0) continue;
    const int q = idx / (2 * BM), rem = idx - q * 2 * BM;
    if (m0 + q < M) reinterpret_cast<float *>(&red[(rem >> 1) * M + m0 + q])[rem & 1] = v[j];
  }
  // taps before the firing start read branch b's history source: the last
  // M-1 samples of its previous feeding firing (zeros if none), staged in
  // LDS by all threads at once
  float2 *hx = red + BM * M;              // [BM][M-1]
  if (s0 == 0) {
    for (int t = threadIdx.x; t < B * (M - 1); t += blockDim.x) {
      const int b = t / (M - 1), i = t - b * (M - 1);
      const int64_t pf = adj_prev(a, b, g);
      hx[t] = pf >= 0 ? a.x[pf * a.r + a.r - (M - 1) + i] : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < BM * M; t += blockDim.x) {
    const int b = t / M, mm = t - b * M;
    float sr = 0.f, si = 0.f;
    if (in_set(set, b)) {
      sr = red[t].x;
      si = red[t].y;
      if (s0 == 0) {
        // output i, tap mm reads history sample i - mm (< 0)
        for (int i = 0; i < mm && i < a.r; ++i) {
          const float2 xv = hx[b * (M - 1) + (M - 1) + i - mm];
          const float pp = fmaf(xv.x, xv.x, xv.y * xv.y);
          float pb = 1.f;
          for (int e = 0; e < b; ++e) pb *= pp;
          const float2 gv = a.G[xb + i];
          const float xr = pb * xv.x, xi = pb * xv.y;
          sr += gv.x * xr + gv.y * xi;
          si += gv.y * xr - gv.x * xi;
        }
      }
    }
    a.partial[(int64_t)t * gridDim.x + blockIdx.x] = make_float2(sr, si);
  }
}

// grad_h[b][m] = fp64 sum of the workgroup partials (stored [b][m][block]),
// fixed order: one workgroup per (b, m); thread t sums blocks t, t+256, ...,
// then a butterfly over each wavefront's lanes and the four wavefronts in
// order.
__global__ __launch_bounds__(256) void k_adj_reduce(const float2 *partial, int64_t n_blocks, float2 *grad) {
  __shared__ double wr[4], wi[4];
  const int e = blockIdx.x;               // b * M + m
  const float2 *src = partial + (int64_t)e * n_blocks;
  double ar = 0.0, ai = 0.0;
  int64_t k = threadIdx.x;
  for (; k + 768 < n_blocks; k += 1024) {  // four loads in flight
    const float2 v0 = src[k], v1 = src[k + 256], v2 = src[k + 512], v3 = src[k + 768];
    ar += v0.x;
    ai += v0.y;
    ar += v1.x;
    ai += v1.y;
    ar += v2.x;
    ai += v2.y;
    ar += v3.x;
    ai += v3.y;
  }
  for (; k < n_blocks; k += 256) {
    const float2 v = src[k];
    ar += v.x;
    ai += v.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ar += __shfl_xor(ar, o);
    ai += __shfl_xor(ai, o);
  }
  if ((threadIdx.x & 63) == 0) wr[threadIdx.x >> 6] = ar, wi[threadIdx.x >> 6] = ai;
  __syncthreads();
  if (threadIdx.x == 0)
    grad[e] = make_float2((float)(((wr[0] + wr[1]) + wr[2]) + wr[3]), (float)(((wi[0] + wi[1]) + wi[2]) + wi[3]));
}

hipError_t launch_adj(const AdjArgs &a, hipStream_t s) {
  const int64_t blocks = a.n_firings * a.blocks_per_firing;
  if (blocks > 0) {
    // one wavefront per adj_tpw(B_max) taps; chunks of four samples per
    // thread; LDS: samples, G window, reduced sums, history samples
    AdjArgs b = a;
    const auto lds_of = [&](int threads, int tpw) {
      b.chunk = 4 * threads;
      return sizeof(float2) * ((size_t)2 * b.chunk + (a.M + tpw - 2) + (size_t)a.B_max * (2 * a.M - 1));
    };
    switch (a.B_max) {
#define DF_CASE(n)                                                                                  \
  case n: {                                                                                         \
    const int threads = 64 * ((a.M + adj_tpw(n) - 1) / adj_tpw(n));                                 \
    const size_t lds = lds_of(threads, adj_tpw(n));                                                 \
    hipLaunchKernelGGL((k_adj_partial<n, adj_tpw(n)>), dim3((unsigned)blocks), dim3(threads), lds, s, b); \
  } break;
      DF_CASE(1) DF_CASE(2) DF_CASE(3) DF_CASE(4) DF_CASE(5) DF_CASE(6) DF_CASE(7) DF_CASE(8)
      DF_CASE(9) DF_CASE(10) DF_CASE(11) DF_CASE(12) DF_CASE(13) DF_CASE(14) DF_CASE(15) DF_CASE(16)
#undef DF_CASE
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adj_reduce, dim3(a.B_max * a.M), dim3(256), 0, s, a.partial, blocks, a.grad);
  return hipGetLastError();
}

// ------------------------------------------------------------------ PA input adjoint
__global__ __launch_bounds__(256) void k_mp_adj(const float2 *u, const float2 *a, const float2 *gin, float2 *Gu,
                                                int64_t n_streams, int64_t len, int K, int Q) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_streams * len) return;
  const int64_t s = t / len, n = t - s * len;
  const float2 uv = u[t];
  const float p = uv.x * uv.x + uv.y * uv.y;
  const float u2r = uv.x * uv.x - uv.y * uv.y, u2i = 2.f * uv.x * uv.y;
  float Gr = 0.f, Gi = 0.f;
  for (int q = 0; q < Q; ++q) {
    if (n + q >= len) break;
    const float2 gq = gin[s * len + n + q];
    float Ar = 0.f, Ai = 0.f, Br = 0.f, Bi = 0.f;
    float pk = 1.f, pkm1 = 1.f;                    // p^k, p^(k-1)
    for (int k = 0; k < K; ++k) {
      const float2 c = a[k * Q + q];
      Ar += c.x * (k + 1) * pk;
      Ai += c.y * (k + 1) * pk;
      if (k >= 1) {
        Br += c.x * k * pkm1;
        Bi += c.y * k * pkm1;
        pkm1 *= p;
      }
      pk *= p;
    }
    // gq conj(A)
    Gr += gq.x * Ar + gq.y * Ai;
    Gi += gq.y * Ar - gq.x * Ai;
    // conj(gq) Bw u^2
    const float wr = Br * u2r - Bi * u2i, wi = Br * u2i + Bi * u2r;
    Gr += gq.x * wr + gq.y * wi;
    Gi += gq.x * wi - gq.y * wr;
  }
  Gu[t] = make_float2(Gr, Gi);
}

hipError_t launch_mp_adj(const float2 *u, const float2 *a, const float2 *g, float2 *Gu, int64_t n_streams,
                         int64_t len, int K, int Q, hipStream_t s) {
  const int64_t total = n_streams * len;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mp_adj, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, u, a, g, Gu, n_streams,
                     len, K, Q);
  return hipGetLastError();
}

}  // namespace dfh
