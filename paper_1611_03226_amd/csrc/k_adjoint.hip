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

// One workgroup per (firing, chunk of outputs); one wavefront per group of 4
// taps; lane l of a wavefront takes input samples s = l, l+64, ... of the
// chunk's window.  For its sample a lane forms p^b once and accumulates
// G[s+m] conj(x_s) p^b into 4 taps x BM branches of independent registers;
// the wavefront then reduces over lanes (fixed shuffle order).
// One reduce-scatter step of the lane butterfly: lanes with bit 2*HALF set
// keep the upper HALF values, the others the lower HALF, each adding the
// partner's copy of the kept half.
template <int HALF>
__device__ __forceinline__ void butterfly_step(float (&v)[32], int lane) {
  constexpr int off = 2 * HALF;
  const bool upper = (lane & off) != 0;
#pragma unroll
  for (int i = 0; i < HALF; ++i) {
    const float send = upper ? v[i] : v[i + HALF];
    const float keep = upper ? v[i + HALF] : v[i];
    v[i] = keep + __shfl_xor(send, off);
  }
  if constexpr (HALF > 1) butterfly_step<HALF / 2>(v, lane);
}

template <int BM>
__global__ __launch_bounds__(512) void k_adj_partial(AdjArgs a) {
  extern __shared__ float2 lds[];
  const int M = a.M;
  const int64_t g = blockIdx.x / a.chunks_per_firing;
  const int64_t c = blockIdx.x - g * a.chunks_per_firing;
  const int64_t n0 = c * a.chunk;
  const int nout = (int)min((int64_t)a.chunk, a.r - n0);
  const uint32_t set = a.B ? (uint32_t)a.B[g] : prefix_set(BM);
  const int B = set_len(set);
  const int64_t xb = g * a.r;
  // G of the chunk's outputs, staged with M-1 zeros before and M+2 after, so
  // that every (sample, tap) pair of the loop below reads a defined value
  // (zero where the output lies outside the chunk, or the tap past M in the
  // last wavefront's group of 4) and the loop carries no bounds checks
  const int gpad = M - 1, gpost = M + 2;
  float2 *sx = lds;                       // window: nout + M - 1 samples
  float2 *sg = lds + a.chunk + M - 1 + gpad;
  float2 *red = sg + a.chunk + gpost;     // [BM][M] reduced sums
  for (int i = threadIdx.x; i < nout + M - 1; i += blockDim.x) {
    const int64_t pos = n0 - (M - 1) + i;
    sx[i] = pos >= 0 ? a.x[xb + pos] : make_float2(0.f, 0.f);
  }
  for (int i = threadIdx.x - gpad; i < nout + gpost; i += blockDim.x)
    sg[i] = (i >= 0 && i < nout) ? a.G[xb + n0 + i] : make_float2(0.f, 0.f);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int m0 = (threadIdx.x >> 6) * 4;  // first tap of this wavefront
  float accr[4][BM], acci[4][BM];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int b = 0; b < BM; ++b) accr[q][b] = acci[q][b] = 0.f;
  // window index i <-> input sample n0-(M-1)+i; output n = sample + m
  for (int i = lane; i < nout + M - 1; i += 64) {
    const float2 xv = sx[i];
    const float p = fmaf(xv.x, xv.x, xv.y * xv.y);
    float pw[BM];
    pw[0] = 1.f;
#pragma unroll
    for (int b = 1; b < BM; ++b) pw[b] = pw[b - 1] * p;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // output index within the chunk: -(M-1) <= o < nout + M + 2 (zeros outside)
      const int o = i - (M - 1) + m0 + q;
      const float2 gv = sg[o];
      const float zr = fmaf(gv.x, xv.x, gv.y * xv.y);     // G conj(x)
      const float zi = fmaf(gv.y, xv.x, -(gv.x * xv.y));
#pragma unroll
      for (int b = 0; b < BM; ++b) {
        accr[q][b] = fmaf(zr, pw[b], accr[q][b]);
        acci[q][b] = fmaf(zi, pw[b], acci[q][b]);
      }
    }
  }
  // Lane sums of the 2*BM values of each tap by a butterfly reduce-scatter
  // (fixed order): every step halves the values a lane holds, exchanging
  // the other half with the lane `off` apart; after the steps 32..2 lane l
  // holds value 16*b5 + 8*b4 + 4*b3 + 2*b2 + b1 (bits of l), summed over the
  // lanes that share bit 0, and a last exchange adds the pair.
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float v[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = i < 2 * BM ? ((i & 1) ? acci[q][i >> 1] : accr[q][i >> 1]) : 0.f;
    butterfly_step<16>(v, lane);
    const float tot = v[0] + __shfl_xor(v[0], 1);
    const int idx = ((lane >> 5) & 1) * 16 + ((lane >> 4) & 1) * 8 + ((lane >> 3) & 1) * 4 + ((lane >> 2) & 1) * 2 +
                    ((lane >> 1) & 1);
    if ((lane & 1) == 0 && idx < 2 * BM && m0 + q < M) {
      float *dst = reinterpret_cast<float *>(&red[(idx >> 1) * M + m0 + q]);
      dst[idx & 1] = tot;
    }
  }
  // taps before the firing start read branch b's history source: the last
  // M-1 samples of its previous feeding firing (zeros if none), staged in
  // LDS by all threads at once
  float2 *hx = red + BM * M;              // [BM][M-1]
  if (n0 == 0) {
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
      if (n0 == 0) {
        // output i, tap mm reads history sample i - mm (< 0)
        for (int i = 0; i < mm && i < nout; ++i) {
          const float2 xv = hx[b * (M - 1) + (M - 1) + i - mm];
          const float pp = fmaf(xv.x, xv.x, xv.y * xv.y);
          float pb = 1.f;
          for (int e = 0; e < b; ++e) pb *= pp;
          const float2 gv = sg[i];
          const float xr = pb * xv.x, xi = pb * xv.y;
          sr += gv.x * xr + gv.y * xi;
          si += gv.y * xr - gv.x * xi;
        }
      }
    }
    a.partial[(int64_t)blockIdx.x * a.B_max * M + t] = make_float2(sr, si);
  }
}

// grad_h[b][m] = fp64 sum of the workgroup partials, fixed order.
__global__ __launch_bounds__(256) void k_adj_reduce(const float2 *partial, int64_t n_blocks, int BM_stride,
                                                    float2 *grad) {
  __shared__ double sr[256], si[256];
  const int e = blockIdx.x;               // b * M + m
  double ar = 0.0, ai = 0.0;
  for (int64_t k = threadIdx.x; k < n_blocks; k += 256) {
    const float2 v = partial[k * BM_stride + e];
    ar += v.x;
    ai += v.y;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[e] = make_float2((float)sr[0], (float)si[0]);
}

hipError_t launch_adj(const AdjArgs &a, hipStream_t s) {
  const int64_t blocks = a.n_firings * a.chunks_per_firing;
  if (blocks > 0) {
    const int threads = 64 * ((a.M + 3) / 4);          // one wavefront per 4 taps
    const size_t lds = sizeof(float2) * ((size_t)2 * a.chunk + a.M - 1 + (a.M - 1) + (a.M + 2) +
                                         (size_t)a.B_max * (2 * a.M - 1));
    switch (a.B_max) {
#define DF_CASE(n) \
  case n: hipLaunchKernelGGL(k_adj_partial<n>, dim3((unsigned)blocks), dim3(threads), lds, s, a); break;
      DF_CASE(1) DF_CASE(2) DF_CASE(3) DF_CASE(4) DF_CASE(5) DF_CASE(6) DF_CASE(7) DF_CASE(8)
      DF_CASE(9) DF_CASE(10) DF_CASE(11) DF_CASE(12) DF_CASE(13) DF_CASE(14) DF_CASE(15) DF_CASE(16)
#undef DF_CASE
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adj_reduce, dim3(a.B_max * a.M), dim3(256), 0, s, a.partial, blocks, a.B_max * a.M,
                     a.grad);
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
