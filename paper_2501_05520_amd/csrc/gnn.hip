// Interaction-network edge classifier (Section 2.2.2, after Battaglia et al.):
//   h0 = phi_v0(x_i),  e0 = phi_e0([x_s, x_t])
//   for t = 1..T:  e <- e + phi_e([h_s, h_t, e]);   m_i = sum of e over edges at i;
//                  h <- h + phi_v([h, m])
//   p = sigmoid(phi_o([h_s, h_t, e]))
//
// MI355X layout.  The first layer of phi_e (and of phi_o) is factorised by its
// three input blocks: the per-node projections [h W_a | h W_b] are computed once
// per node by the node kernel (N x 2H) and gathered per edge, so each edge pays
// for two H x H products instead of a 3H x H one.  Edge states e live in HBM in
// the working precision and are rewritten in place each iteration; node states
// stay FP32.  In FP8 the edge states and the per-node projections are stored as
// E4M3 with per-tensor power-of-two scales (GnnScale) and the edge-side products
// (the e-block and the second layer of phi_e, the e-block of phi_o) run on FP8
// matrix cores; the node side (encoders, phi_v, the projections) runs in BF16.
// Aggregation is a gather, not a scatter: each node sums the states
// of its incident edges through CSR (by source) and CSC (by destination) index
// lists sorted by edge id, in a fixed order, so the sums are deterministic and an
// event gives the same scores alone or batched with others.
#include "kernels.h"
#include "mfma_tile.h"
#include <algorithm>
#include <type_traits>
#include <stdlib.h>

namespace {

// The encoders' first layers read the hit features (3 per hit, 6 per edge) and run in
// FP32 in every precision: one FP32 fragment block of k (16) covers them, costs about
// what one BF16 block would, and keeps the features' full precision (a trained
// encoder separates hits millimetres apart, which BF16 coordinates do not resolve).
constexpr int KIN = PrecF32::KB;              // padded width of the encoder inputs
constexpr int LDI = KIN + PrecF32::PAD;       // row stride of the FP32 input tile


template <class P, int H, int MT, int NW>
struct GnnShape {
  typedef typename P::act_t T;
  static constexpr int LDH = H + P::PAD;
  static constexpr int LD2 = 2 * H + P::PAD;
  static constexpr int MTW = MT / 16;
  static constexpr int NTW = H / 16 / NW;      // n-tiles per wave for N = H
  static constexpr int NTW2 = 2 * H / 16 / NW; // for N = 2H
  static_assert(NTW >= 1 && H % (16 * NW) == 0, "H must split over the waves");
};

template <class P>
__device__ __forceinline__ void load4(const typename P::act_t* p, float& a, float& b, float& c, float& d);
template <>
__device__ __forceinline__ void load4<PrecF32>(const float* p, float& a, float& b, float& c, float& d) {
  const float4 v = *(const float4*)p;
  a = v.x; b = v.y; c = v.z; d = v.w;
}
template <>
__device__ __forceinline__ void load4<PrecBF16>(const __bf16* p, float& a, float& b, float& c, float& d) {
  const bf16x4 v = *(const bf16x4*)p;
  a = (float)v[0]; b = (float)v[1]; c = (float)v[2]; d = (float)v[3];
}
template <>
__device__ __forceinline__ void load4<PrecX3>(const x3_t* p, float& a, float& b, float& c, float& d) {
  float v[4];
  PrecX3::unpack16(*(const uint4*)p, v);
  a = v[0]; b = v[1]; c = v[2]; d = v[3];
}

template <>
__device__ __forceinline__ void load4<PrecFP8>(const uint8_t* p, float& a, float& b, float& c, float& d) {
  const int v = *(const int*)p;
  const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(v, false);
  const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(v, true);
  a = lo[0]; b = lo[1]; c = hi[0]; d = hi[1];
}

template <class P>
constexpr bool is_fp8() { return std::is_same<P, PrecFP8>::value; }

// an edge state or node projection as stored: E4M3(v * s) in FP8, v itself otherwise
template <class P>
__device__ __forceinline__ void store_state4(typename P::act_t* p, float a, float b, float c, float d, float s) {
  if constexpr (is_fp8<P>()) P::store4_scaled(p, a, b, c, d, s);
  else P::store4(p, a, b, c, d);
}

// copy rows [row0, row0 + MT) of a [rows][H] act array into LDS (zero past `rows`):
// every load of the tile is requested before the first LDS write
template <class P, int H, int MT, int NT>
__device__ __forceinline__ void stage_rows(const typename P::act_t* __restrict__ g, int64_t row0, int64_t rows,
                                           typename P::act_t* lds, int ld) {
  constexpr int V = 16 / (int)sizeof(typename P::act_t);  // elements per 16-byte chunk
  constexpr int CPR = H / V;                               // chunks per row
  constexpr int IT = (MT * CPR + NT - 1) / NT;
  uint4 v[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int m = idx / CPR, c = idx - m * CPR;
    v[it] = make_uint4(0, 0, 0, 0);
    if (idx < MT * CPR && row0 + m < rows) v[it] = *(const uint4*)(g + (size_t)(row0 + m) * H + c * V);
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int m = idx / CPR, c = idx - m * CPR;
    if (idx < MT * CPR) *(uint4*)(lds + m * ld + c * V) = v[it];
  }
}

// product of an LDS activation tile with a layer of compile-time fan-in K
// (about 128 bytes of weight fragments per lane in flight: eight 16-byte
// fragments, four 32-byte ones)
template <class P, int MTW, int NTW, int K, bool INIT = false>
__device__ __forceinline__ void gemm_k(f32x4 (&acc)[MTW][NTW], const typename P::act_t* xs, int ldx,
                                       const DevLayer& L, int nt0) {
  constexpr int F = NTW * (int)(sizeof(typename P::frag_t) / 16);   // 16-byte units per k block
  tile_gemm_k<P, MTW, NTW, (K + P::KB - 1) / P::KB, (F >= 8 ? 1 : 8 / F), INIT>(acc, xs, ldx, L.w, L.nkb, nt0);
}

// ---------------------------------------------------------------------------
// node encoder: h0 = tanh(tanh(x W1 + b1) W2 + b2); proj = h0 [W_a | W_b]
// (products in P, projections stored in Q's format with scale ps)
// ---------------------------------------------------------------------------
template <class P, class Q, int H, int MT, int NW>
__global__ __launch_bounds__(NW * 64) void node_encode_kernel(const float* __restrict__ x, int n, DevLayer l1,
                                                              DevLayer l2, DevLayer lp, float* __restrict__ h,
                                                              typename Q::act_t* __restrict__ proj, float ps) {
  typedef GnnShape<P, H, MT, NW> S;
  typedef typename S::T T;
  __shared__ __align__(16) float xin[MT * LDI];
  __shared__ __align__(16) T a1[MT * S::LDH];
  __shared__ __align__(16) T a2[MT * S::LDH];
  const int wave = threadIdx.x >> 6, l = lane_id(), g = l >> 4, r = l & 15;
  const int ntiles = (n + MT - 1) / MT;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int row0 = t * MT;
    {
      constexpr int IT = (MT * KIN + NW * 64 - 1) / (NW * 64);
      float v[IT];
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = threadIdx.x + it * NW * 64;
        const int m = idx / KIN, k = idx - m * KIN;
        v[it] = (idx < MT * KIN && k < 3 && row0 + m < n) ? x[(size_t)(row0 + m) * 3 + k] : 0.f;
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = threadIdx.x + it * NW * 64;
        const int m = idx / KIN, k = idx - m * KIN;
        if (idx < MT * KIN) xin[m * LDI + k] = v[it];
      }
    }
    __syncthreads();
    f32x4 acc[S::MTW][S::NTW];
    gemm_k<PrecF32, S::MTW, S::NTW, 3, true>(acc, xin, LDI, l1, wave * S::NTW);
    tile_store_tanh<P>(acc, l1.bs, 1.f, a1, S::LDH, wave * S::NTW);
    __syncthreads();
    gemm_k<P, S::MTW, S::NTW, H, true>(acc, a1, S::LDH, l2, wave * S::NTW);
#pragma unroll
    for (int j = 0; j < S::NTW; ++j) {
      const int nn = (wave * S::NTW + j) * 16 + 4 * g;
      const float4 b = *(const float4*)(l2.bs + nn);
#pragma unroll
      for (int i = 0; i < S::MTW; ++i) {
        const int m = i * 16 + r;
        const float v0 = trk_tanh_log2(fmaf(acc[i][j][0], TRK_2LOG2E, b.x)), v1 = trk_tanh_log2(fmaf(acc[i][j][1], TRK_2LOG2E, b.y));
        const float v2 = trk_tanh_log2(fmaf(acc[i][j][2], TRK_2LOG2E, b.z)), v3 = trk_tanh_log2(fmaf(acc[i][j][3], TRK_2LOG2E, b.w));
        if (row0 + m < n) *(float4*)(h + (size_t)(row0 + m) * H + nn) = make_float4(v0, v1, v2, v3);
        P::store4(a2 + m * S::LDH + nn, v0, v1, v2, v3);
      }
    }
    __syncthreads();
    f32x4 accp[S::MTW][S::NTW2];
    gemm_k<P, S::MTW, S::NTW2, H, true>(accp, a2, S::LDH, lp, wave * S::NTW2);
#pragma unroll
    for (int j = 0; j < S::NTW2; ++j) {
      const int nn = (wave * S::NTW2 + j) * 16 + 4 * g;
#pragma unroll
      for (int i = 0; i < S::MTW; ++i) {
        const int m = i * 16 + r;
        if (row0 + m < n)
          store_state4<Q>(proj + (size_t)(row0 + m) * 2 * H + nn, accp[i][j][0], accp[i][j][1], accp[i][j][2],
                          accp[i][j][3], ps);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// edge encoder: e0 = tanh(tanh([x_s, x_t] W1 + b1) W2 + b2)
// (first layer in FP32, the second in P, states stored in Q's format with scale se)
// ---------------------------------------------------------------------------
template <class P, class Q, int H, int MT, int NW>
__global__ __launch_bounds__(NW * 64) void edge_encode_kernel(const float* __restrict__ x, int n,
                                                              const int* __restrict__ src, const int* __restrict__ dst,
                                                              int64_t m_cap, const int* d_m, DevLayer l1, DevLayer l2,
                                                              typename Q::act_t* __restrict__ e, int* d_err, float se) {
  typedef GnnShape<P, H, MT, NW> S;
  typedef typename S::T T;
  __shared__ __align__(16) float xin[MT * LDI];
  __shared__ __align__(16) T a1[MT * S::LDH];
  const int wave = threadIdx.x >> 6, l = lane_id(), g = l >> 4, r = l & 15;
  const int64_t m = d_m ? clamp_count(d_m, m_cap) : m_cap;
  const int64_t ntiles = (m + MT - 1) / MT;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * MT;
    {
      constexpr int IT = (MT * KIN + NW * 64 - 1) / (NW * 64);
      int node[IT];
      float v[IT];
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = threadIdx.x + it * NW * 64;
        const int mm = idx / KIN, k = idx - mm * KIN;
        node[it] = -1;
        if (idx < MT * KIN && k < 6 && row0 + mm < m) node[it] = k < 3 ? src[row0 + mm] : dst[row0 + mm];
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = threadIdx.x + it * NW * 64;
        const int k = idx % KIN;
        v[it] = 0.f;
        if ((unsigned)node[it] < (unsigned)n) v[it] = x[(size_t)node[it] * 3 + (k % 3)];
        else if (node[it] != -1 && d_err) atomicOr(d_err, TRK_ERRBIT_INDEX);
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = threadIdx.x + it * NW * 64;
        const int mm = idx / KIN, k = idx - mm * KIN;
        if (idx < MT * KIN) xin[mm * LDI + k] = v[it];
      }
    }
    __syncthreads();
    f32x4 acc[S::MTW][S::NTW];
    gemm_k<PrecF32, S::MTW, S::NTW, 6, true>(acc, xin, LDI, l1, wave * S::NTW);
    tile_store_tanh<P>(acc, l1.bs, 1.f, a1, S::LDH, wave * S::NTW);
    __syncthreads();
    gemm_k<P, S::MTW, S::NTW, H, true>(acc, a1, S::LDH, l2, wave * S::NTW);
#pragma unroll
    for (int j = 0; j < S::NTW; ++j) {
      const int nn = (wave * S::NTW + j) * 16 + 4 * g;
      const float4 b = *(const float4*)(l2.bs + nn);
#pragma unroll
      for (int i = 0; i < S::MTW; ++i) {
        const int64_t row = row0 + i * 16 + r;
        if (row < m)
          store_state4<Q>(e + (size_t)row * H + nn, trk_tanh_log2(fmaf(acc[i][j][0], TRK_2LOG2E, b.x)),
                          trk_tanh_log2(fmaf(acc[i][j][1], TRK_2LOG2E, b.y)),
                          trk_tanh_log2(fmaf(acc[i][j][2], TRK_2LOG2E, b.z)),
                          trk_tanh_log2(fmaf(acc[i][j][3], TRK_2LOG2E, b.w)), se);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// edge step: e <- e + tanh(tanh(e W_c + b1 + P_a[s] + P_b[t]) W2 + b2)
// edge output (OUT = true): p = sigmoid(tanh(e W_c + b1 + Q_a[s] + Q_b[t]) . w2 + b2)
// The gathered projections are summed into an FP32 LDS tile with coalesced row
// loads before the product; the hidden activation t1 reuses that tile.
// ---------------------------------------------------------------------------
// WPE: waves per SIMD the registers must allow (default: one workgroup's worth)
template <class P, int H, int MT, int NW, bool OUT, int WPE = NW / 4>
__global__ __launch_bounds__(NW * 64, WPE) void edge_kernel(typename P::act_t* __restrict__ e,
                                                       const typename P::act_t* __restrict__ proj,
                                                       const int* __restrict__ src, const int* __restrict__ dst,
                                                       int n, int64_t m_cap, const int* d_m, DevLayer lc, DevLayer l2,
                                                       DevVec lo, GnnScale sc, float* __restrict__ scores) {
  typedef GnnShape<P, H, MT, NW> S;
  typedef typename S::T T;
  constexpr int LDP = H + 4;                       // fp32 row stride of the gathered tile
  constexpr int V = 16 / (int)sizeof(T);           // act elements per 16-byte chunk
  __shared__ __align__(16) T et[MT * S::LDH];
  __shared__ __align__(16) float pre[MT * LDP];
  static_assert(MT * S::LDH * (int)sizeof(T) <= MT * LDP * 4, "t1 must fit in the gathered tile");
  __shared__ float zred[NW * MT];
  __shared__ int sidx[MT], didx[MT];
  T* t1 = (T*)pre;
  const int wave = threadIdx.x >> 6, l = lane_id(), g = l >> 4, r = l & 15;
  const int64_t m = d_m ? clamp_count(d_m, m_cap) : m_cap;
  const int64_t ntiles = (m + MT - 1) / MT;
  // product scales of the two layers, folded with the 2 log2(e) of the tanh epilogue
  // (the layers' dq is 1 unless FP8: the constant itself there)
  const float s1 = is_fp8<P>() ? lc.dq * TRK_2LOG2E : TRK_2LOG2E;
  const float s2 = is_fp8<P>() ? l2.dq * TRK_2LOG2E : TRK_2LOG2E;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * MT;
    {
      // the tile's edge ends are requested together with its state rows
      int a = 0, b = 0;
      const int mm = threadIdx.x;
      if (mm < MT && row0 + mm < m) {
        a = src[row0 + mm];
        b = dst[row0 + mm];
      }
      stage_rows<P, H, MT, NW * 64>(e, row0, m, et, S::LDH);
      if (mm < MT) {
        sidx[mm] = (unsigned)a < (unsigned)n ? a : 0;
        didx[mm] = (unsigned)b < (unsigned)n ? b : 0;
      }
    }
    __syncthreads();
    {
      // pre[m][c] = (proj[src_m][c] + proj[dst_m][H + c] + b1[c]) 2 log2(e): every gather of the
      // tile is requested before the first sum is written
      constexpr int CPR = H / V;
      constexpr int IT = (MT * CPR + NW * 64 - 1) / (NW * 64);
      uint4 ua[IT], ub[IT];
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = threadIdx.x + it * NW * 64;
        const int mm = idx / CPR, c = (idx - mm * CPR) * V;
        ua[it] = ub[it] = make_uint4(0, 0, 0, 0);
        if (idx < MT * CPR) {
          ua[it] = *(const uint4*)(proj + (size_t)sidx[mm] * 2 * H + c);
          ub[it] = *(const uint4*)(proj + (size_t)didx[mm] * 2 * H + H + c);
        }
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = threadIdx.x + it * NW * 64;
        const int mm = idx / CPR, c = (idx - mm * CPR) * V;
        if (idx < MT * CPR) {
          float pa[V], pb[V];
          P::unpack16(ua[it], pa);
          P::unpack16(ub[it], pb);
          if constexpr (is_fp8<P>()) {
#pragma unroll
            for (int q = 0; q < V; ++q) {
              pa[q] *= sc.inv_p;
              pb[q] *= sc.inv_p;
            }
          }
#pragma unroll
          for (int q = 0; q < V; q += 4) {
            // kept times 2 log2(e), the form the tanh epilogue consumes
            const float4 bb = *(const float4*)(lc.bs + c + q);
            *(float4*)(pre + mm * LDP + c + q) =
                make_float4(fmaf(pa[q] + pb[q], TRK_2LOG2E, bb.x),
                            fmaf(pa[q + 1] + pb[q + 1], TRK_2LOG2E, bb.y),
                            fmaf(pa[q + 2] + pb[q + 2], TRK_2LOG2E, bb.z),
                            fmaf(pa[q + 3] + pb[q + 3], TRK_2LOG2E, bb.w));
          }
        }
      }
    }
    __syncthreads();
    f32x4 acc[S::MTW][S::NTW];
    gemm_k<P, S::MTW, S::NTW, H, true>(acc, et, S::LDH, lc, wave * S::NTW);
    float part[S::MTW];
#pragma unroll
    for (int i = 0; i < S::MTW; ++i) part[i] = 0.f;
#pragma unroll
    for (int j = 0; j < S::NTW; ++j) {
      const int nn = (wave * S::NTW + j) * 16 + 4 * g;
      float4 w2 = make_float4(0.f, 0.f, 0.f, 0.f);
      if (OUT) w2 = *(const float4*)(lo.w + nn);
#pragma unroll
      for (int i = 0; i < S::MTW; ++i) {
        const int mm = i * 16 + r;
        const float4 pv = *(const float4*)(pre + mm * LDP + nn);
        const float v0 = trk_tanh_log2(fmaf(acc[i][j][0], s1, pv.x));
        const float v1 = trk_tanh_log2(fmaf(acc[i][j][1], s1, pv.y));
        const float v2 = trk_tanh_log2(fmaf(acc[i][j][2], s1, pv.z));
        const float v3 = trk_tanh_log2(fmaf(acc[i][j][3], s1, pv.w));
        if (OUT) part[i] += v0 * w2.x + v1 * w2.y + v2 * w2.z + v3 * w2.w;
        acc[i][j] = f32x4{v0, v1, v2, v3};
      }
    }
    if (OUT) {
#pragma unroll
      for (int i = 0; i < S::MTW; ++i) {
        part[i] += __shfl_xor(part[i], 16, 64);
        part[i] += __shfl_xor(part[i], 32, 64);
        if (g == 0) zred[wave * MT + i * 16 + r] = part[i];
      }
      __syncthreads();
      for (int mm = threadIdx.x; mm < MT; mm += blockDim.x) {
        float z = lo.b;
        for (int w = 0; w < NW; ++w) z += zred[w * MT + mm];
        if (row0 + mm < m) scores[row0 + mm] = trk_sigmoid(z);
      }
      __syncthreads();
    } else {
      __syncthreads();                 // every lane has read its part of pre
#pragma unroll
      for (int j = 0; j < S::NTW; ++j) {
        const int nn = (wave * S::NTW + j) * 16 + 4 * g;
#pragma unroll
        for (int i = 0; i < S::MTW; ++i)
          P::store4(t1 + (i * 16 + r) * S::LDH + nn, acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
      }
      __syncthreads();
            gemm_k<P, S::MTW, S::NTW, H, true>(acc, t1, S::LDH, l2, wave * S::NTW);
#pragma unroll
      for (int j = 0; j < S::NTW; ++j) {
        const int nn = (wave * S::NTW + j) * 16 + 4 * g;
        const float4 b = *(const float4*)(l2.bs + nn);
#pragma unroll
        for (int i = 0; i < S::MTW; ++i) {
          const int mm = i * 16 + r;
          const int64_t row = row0 + mm;
          float e0, e1, e2, e3;
          load4<P>(et + mm * S::LDH + nn, e0, e1, e2, e3);
          if constexpr (is_fp8<P>()) {
            e0 *= sc.inv_e; e1 *= sc.inv_e; e2 *= sc.inv_e; e3 *= sc.inv_e;
          }
          if (row < m)
            store_state4<P>(e + (size_t)row * H + nn, e0 + trk_tanh_log2(fmaf(acc[i][j][0], s2, b.x)),
                            e1 + trk_tanh_log2(fmaf(acc[i][j][1], s2, b.y)),
                            e2 + trk_tanh_log2(fmaf(acc[i][j][2], s2, b.z)),
                            e3 + trk_tanh_log2(fmaf(acc[i][j][3], s2, b.w)), sc.e);
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// aggregation: msg[i] = sum of the states of i's incident edges, the CSR (by
// source) list then the CSC (by destination) list, each in ascending edge order,
// taken as one list.  A wave serves one node at a time: one coalesced load brings
// up to 64 edge ids of the list, then its lanes form RPS groups that each read one
// edge row per step (16 bytes per lane); the groups' partial sums are combined in
// a fixed order, so the result does not depend on scheduling.  The list bounds of
// the wave's next node are requested while the current one is summed.
// ---------------------------------------------------------------------------
template <class P, int H>
__global__ __launch_bounds__(256) void aggregate_kernel(const typename P::act_t* __restrict__ e,
                                                        const int* __restrict__ sptr, const int* __restrict__ sidx,
                                                        const int* __restrict__ dptr, const int* __restrict__ didx,
                                                        int n, float* __restrict__ msg, float inv_e) {
  typedef typename P::act_t T;
  constexpr int V = 16 / (int)sizeof(T);   // columns per lane per row
  constexpr int LPR = H / V;               // lanes per row
  constexpr int RPS = 64 / LPR;            // rows per wave step
  static_assert(LPR >= 1 && LPR <= 64 && 64 % LPR == 0, "row split");
  const int l = lane_id();
  const int grp = l / LPR, col = (l % LPR) * V;
  const int waves = gridDim.x * (blockDim.x >> 6);
  int node = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  int bs = 0, es = 0, bd = 0, ed = 0;
  if (node < n) {
    bs = sptr[node]; es = sptr[node + 1];
    bd = dptr[node]; ed = dptr[node + 1];
  }
  for (; node < n; node += waves) {
    const int nxt = node + waves;
    int nbs = 0, nes = 0, nbd = 0, ned = 0;
    if (nxt < n) {
      nbs = sptr[nxt]; nes = sptr[nxt + 1];
      nbd = dptr[nxt]; ned = dptr[nxt + 1];
    }
    float acc[V];
#pragma unroll
    for (int q = 0; q < V; ++q) acc[q] = 0.f;
    const int cs = es - bs, tot = cs + (ed - bd);
    for (int base = 0; base < tot; base += 64) {
      const int cnt = min(64, tot - base);
      const int k0 = base + l;
      const int my = l < cnt ? (k0 < cs ? sidx[bs + k0] : didx[bd + k0 - cs]) : 0;
      const int steps = (cnt + RPS - 1) / RPS;   // uniform over the wave: the shuffle needs every lane
#pragma unroll 8
      for (int st = 0; st < steps; ++st) {
        const int k = grp + st * RPS;
        const int eid = __shfl(my, k < cnt ? k : 0, 64);
        if (k < cnt) {
          float v[V];
          P::unpack16(*(const uint4*)(e + (size_t)eid * H + col), v);
          if constexpr (is_fp8<P>()) {
#pragma unroll
            for (int q = 0; q < V; ++q) v[q] *= inv_e;
          }
#pragma unroll
          for (int q = 0; q < V; ++q) acc[q] += v[q];
        }
      }
    }
    // combine the row groups: lanes with the same column, fixed butterfly order
#pragma unroll
    for (int o = LPR; o < 64; o <<= 1)
#pragma unroll
      for (int q = 0; q < V; ++q) acc[q] += __shfl_xor(acc[q], o, 64);
    if (grp == 0) {
#pragma unroll
      for (int q = 0; q < V; q += 4)
        *(float4*)(msg + (size_t)node * H + col + q) = make_float4(acc[q], acc[q + 1], acc[q + 2], acc[q + 3]);
    }
    bs = nbs; es = nes; bd = nbd; ed = ned;
  }
}

// ---------------------------------------------------------------------------
// node step: h <- h + tanh(tanh([h, m] W1 + b1) W2 + b2) with m the aggregated
// messages; proj = h [W_a | W_b] for the next edge step (or the output head)
// (products in P, projections stored in Q's format with scale ps)
// ---------------------------------------------------------------------------
template <class P, class Q, int H, int MT, int NW>
__global__ __launch_bounds__(NW * 64) void node_step_kernel(float* __restrict__ h, const float* __restrict__ msg,
                                                            int n, DevLayer l1, DevLayer l2, DevLayer lp,
                                                            typename Q::act_t* __restrict__ proj, float ps) {
  typedef GnnShape<P, H, MT, NW> S;
  typedef typename S::T T;
  __shared__ __align__(16) T in[MT * S::LD2];
  __shared__ __align__(16) T t1[MT * S::LDH];
  const int wave = threadIdx.x >> 6, l = lane_id(), g = l >> 4, r = l & 15;
  const int ntiles = (n + MT - 1) / MT;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int row0 = t * MT;
    // staging of [h, m] as the working precision, and this lane's residual h values
    // (the layout of its outputs): every load of the tile is requested first
    constexpr int CPR = H / 4;                                  // float4 chunks per row
    constexpr int IT = (MT * CPR + NW * 64 - 1) / (NW * 64);
    float4 hv4[IT], mv4[IT], hres[S::MTW][S::NTW];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * NW * 64;
      const int mm = idx / CPR, c = (idx - mm * CPR) * 4;
      const int node = row0 + mm;
      hv4[it] = mv4[it] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (idx < MT * CPR && node < n) {
        hv4[it] = *(const float4*)(h + (size_t)node * H + c);
        mv4[it] = *(const float4*)(msg + (size_t)node * H + c);
      }
    }
#pragma unroll
    for (int i = 0; i < S::MTW; ++i)
#pragma unroll
      for (int j = 0; j < S::NTW; ++j) {
        const int node = row0 + i * 16 + r;
        const int nn = (wave * S::NTW + j) * 16 + 4 * g;
        hres[i][j] = node < n ? *(const float4*)(h + (size_t)node * H + nn) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * NW * 64;
      const int mm = idx / CPR, c = (idx - mm * CPR) * 4;
      if (idx < MT * CPR) {
        P::store4(in + mm * S::LD2 + c, hv4[it].x, hv4[it].y, hv4[it].z, hv4[it].w);
        P::store4(in + mm * S::LD2 + H + c, mv4[it].x, mv4[it].y, mv4[it].z, mv4[it].w);
      }
    }
    __syncthreads();
    f32x4 acc[S::MTW][S::NTW];
    gemm_k<P, S::MTW, S::NTW, 2 * H, true>(acc, in, S::LD2, l1, wave * S::NTW);
    tile_store_tanh<P>(acc, l1.bs, 1.f, t1, S::LDH, wave * S::NTW);
    __syncthreads();
    gemm_k<P, S::MTW, S::NTW, H, true>(acc, t1, S::LDH, l2, wave * S::NTW);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < S::NTW; ++j) {
      const int nn = (wave * S::NTW + j) * 16 + 4 * g;
      const float4 b = *(const float4*)(l2.bs + nn);
#pragma unroll
      for (int i = 0; i < S::MTW; ++i) {
        const int mm = i * 16 + r;
        const int node = row0 + mm;
        float4 hv = hres[i][j];
        hv.x += trk_tanh_log2(fmaf(acc[i][j][0], TRK_2LOG2E, b.x));
        hv.y += trk_tanh_log2(fmaf(acc[i][j][1], TRK_2LOG2E, b.y));
        hv.z += trk_tanh_log2(fmaf(acc[i][j][2], TRK_2LOG2E, b.z));
        hv.w += trk_tanh_log2(fmaf(acc[i][j][3], TRK_2LOG2E, b.w));
        if (node < n) *(float4*)(h + (size_t)node * H + nn) = hv;
        P::store4(in + mm * S::LD2 + nn, hv.x, hv.y, hv.z, hv.w);
      }
    }
    __syncthreads();
    f32x4 accp[S::MTW][S::NTW2];
    gemm_k<P, S::MTW, S::NTW2, H, true>(accp, in, S::LD2, lp, wave * S::NTW2);
#pragma unroll
    for (int j = 0; j < S::NTW2; ++j) {
      const int nn = (wave * S::NTW2 + j) * 16 + 4 * g;
#pragma unroll
      for (int i = 0; i < S::MTW; ++i) {
        const int node = row0 + i * 16 + r;
        if (node < n)
          store_state4<Q>(proj + (size_t)node * 2 * H + nn, accp[i][j][0], accp[i][j][1], accp[i][j][2],
                          accp[i][j][3], ps);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// incidence lists: for every node, the ids of the edges whose key (src or dst)
// is that node, ascending
// ---------------------------------------------------------------------------
// row pointers of edges sorted by key: ptr[i] = first edge whose key is >= i
__global__ void sorted_rowptr(const int* __restrict__ key, int64_t m_cap, const int* d_m, int n, int* ptr) {
  const int64_t m = d_m ? clamp_count(d_m, m_cap) : m_cap;
  GRID_STRIDE(i, (int64_t)n + 1) {
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (key[mid] < (int)i) lo = mid + 1; else hi = mid;
    }
    ptr[i] = (int)lo;
  }
}
__global__ void iota_kernel(int* __restrict__ out, int64_t m_cap, const int* d_m) {
  const int64_t m = d_m ? clamp_count(d_m, m_cap) : m_cap;
  GRID_STRIDE(e, m) out[e] = (int)e;
}

__global__ void incidence_count(const int* __restrict__ key, int64_t m_cap, const int* d_m, int n, int* cnt) {
  const int64_t m = d_m ? clamp_count(d_m, m_cap) : m_cap;
  GRID_STRIDE(e, m) {
    const int k = key[e];
    if ((unsigned)k < (unsigned)n) atomicAdd(&cnt[k], 1);
  }
}
__global__ void incidence_fill(const int* __restrict__ key, int64_t m_cap, const int* d_m, int n,
                               const int* __restrict__ ptr, int* cursor, int* raw) {
  const int64_t m = d_m ? clamp_count(d_m, m_cap) : m_cap;
  GRID_STRIDE(e, m) {
    const int k = key[e];
    if ((unsigned)k < (unsigned)n) raw[ptr[k] + atomicAdd(&cursor[k], 1)] = (int)e;
  }
}

// Grid of the aggregation: one node per wave, up to 65536 four-wave blocks (waves that
// finish early are replaced at once, which balances uneven degrees).
int agg_blocks(int n) { return blocks_for(n, 4, 65536); }

// the unrolled products read ceil(K / KB) fragment blocks per n-tile of each layer:
// the edge-side layers in P, the node side (encoders, node network, projections) in N
template <class P, class N, int H>
bool gnn_shapes_ok(const DevGNN& net) {
  auto nkb = [](int K, int KB) { return (K + KB - 1) / KB; };
  const DevLayer* edge_side[] = {&net.edge_c, &net.edge_2, &net.out_c};
  const DevLayer* node_side[] = {&net.node_enc2, &net.edge_enc2, &net.edge_ab, &net.node_2, &net.out_ab};
  for (const DevLayer* L : edge_side)
    if (L->nkb != nkb(H, P::KB)) return false;
  for (const DevLayer* L : node_side)
    if (L->nkb != nkb(H, N::KB)) return false;
  return net.H == H && net.node_enc1.nkb == nkb(3, N::KB) && net.edge_enc1.nkb == nkb(6, N::KB) &&
         net.node_1.nkb == nkb(2 * H, N::KB);
}

// P: precision of the edge-side products and of the stored edge states and
// projections; N: precision of the node-side products (N = P except in FP8)
template <class P, class N, int H, int MTE, int MTN, int NW, int EWPE = NW / 4>
void run_gnn(const DevGNN& net, const float* x, int n, const int* src, const int* dst, int64_t m_cap, const int* d_m,
             float* scores, GnnScratch& g, int n_cu, int* d_err, hipStream_t s, bool src_sorted) {
  typedef typename P::act_t T;
  T* proj = (T*)g.proj;
  T* e = (T*)g.e;
  const GnnScale sc = net.sc;
  launch_incidence(src, dst, m_cap, d_m, n, g, s, src_sorted);
  const int ngrid = (int)std::min<int64_t>((n + MTN - 1) / MTN, (int64_t)n_cu * 8);
  const int64_t etiles = (m_cap + MTE - 1) / MTE;
  const int egrid = (int)std::min<int64_t>(etiles, (int64_t)n_cu * 8);
  const DevLayer& first_proj = net.iters > 0 ? net.edge_ab : net.out_ab;
  if (ngrid > 0)
    node_encode_kernel<N, P, H, MTN, NW><<<ngrid, NW * 64, 0, s>>>(x, n, net.node_enc1, net.node_enc2, first_proj,
                                                                   g.h, proj, sc.p);
  if (egrid > 0)
    edge_encode_kernel<N, P, H, MTE, NW><<<egrid, NW * 64, 0, s>>>(x, n, src, dst, m_cap, d_m, net.edge_enc1,
                                                                   net.edge_enc2, e, d_err, sc.e);
  for (int it = 0; it < net.iters; ++it) {
    if (egrid > 0)
      edge_kernel<P, H, MTE, NW, false, EWPE><<<egrid, NW * 64, 0, s>>>(e, proj, src, dst, n, m_cap, d_m, net.edge_c,
                                                                  net.edge_2, net.out_2, sc, nullptr);
    const DevLayer& lp = it + 1 < net.iters ? net.edge_ab : net.out_ab;
    aggregate_kernel<P, H><<<agg_blocks(n), 256, 0, s>>>(e, g.rowptr, g.rowidx, g.cscptr, g.cscidx, n, g.msg,
                                                         sc.inv_e);
    if (ngrid > 0)
      node_step_kernel<N, P, H, MTN, NW><<<ngrid, NW * 64, 0, s>>>(g.h, g.msg, n, net.node_1, net.node_2, lp, proj,
                                                                   sc.p);
  }
  if (egrid > 0)
    edge_kernel<P, H, MTE, NW, true, EWPE><<<egrid, NW * 64, 0, s>>>(e, proj, src, dst, n, m_cap, d_m, net.out_c,
                                                               net.edge_2, net.out_2, sc, scores);
}

// Row tiles of the H=128 kernels: 64-edge tiles on eight waves with the edge kernel's
// registers held to four waves per SIMD, so that two workgroups share a CU; 64-node tiles
// for the node step, except in split BF16, whose node step takes 32-node tiles (its
// registers then also allow two workgroups per CU).
template <class P>
void run_gnn128(const DevGNN& net, const float* x, int n, const int* src, const int* dst, int64_t m_cap,
                const int* d_m, float* scores, GnnScratch& g, int n_cu, int* d_err, hipStream_t s, bool sorted) {
  if constexpr (std::is_same<P, PrecX3>::value)
    run_gnn<P, P, 128, 64, 32, 8, 4>(net, x, n, src, dst, m_cap, d_m, scores, g, n_cu, d_err, s, sorted);
  else if constexpr (std::is_same<P, PrecFP8>::value)
    run_gnn<P, PrecBF16, 128, 64, 64, 8, 4>(net, x, n, src, dst, m_cap, d_m, scores, g, n_cu, d_err, s, sorted);
  else
    run_gnn<P, P, 128, 64, 64, 8, 4>(net, x, n, src, dst, m_cap, d_m, scores, g, n_cu, d_err, s, sorted);
}

}  // namespace

void launch_incidence(const int* src, const int* dst, int64_t m_cap, const int* d_m, int n, GnnScratch& g,
                      hipStream_t s, bool src_sorted) {
  const int* keys[2] = {src, dst};
  int* ptrs[2] = {g.rowptr, g.cscptr};
  int* idxs[2] = {g.rowidx, g.cscidx};
  const int eb = blocks_for(m_cap, 256, 2048);
  for (int k = 0; k < 2; ++k) {
    if (k == 0 && src_sorted) {
      // edges already grouped by source in ascending edge order: the list of node i
      // is the edge range [lower_bound(src, i), lower_bound(src, i + 1))
      sorted_rowptr<<<blocks_for((int64_t)n + 1, 256), 256, 0, s>>>(src, m_cap, d_m, n, g.rowptr);
      iota_kernel<<<eb, 256, 0, s>>>(g.rowidx, m_cap, d_m);
      continue;
    }
    launch_fill_int(g.cnt, 0, n, s);
    if (m_cap > 0) incidence_count<<<eb, 256, 0, s>>>(keys[k], m_cap, d_m, n, g.cnt);
    launch_scan_excl(g.cnt, ptrs[k], n, nullptr, nullptr, g.tmp, s);
    launch_fill_int(g.cnt, 0, n, s);
    if (m_cap > 0) incidence_fill<<<eb, 256, 0, s>>>(keys[k], m_cap, d_m, n, ptrs[k], g.cnt, g.raw);
    launch_segment_sort(ptrs[k], g.raw, idxs[k], n, s);
  }
}

int launch_gnn(int prec, const DevGNN& net, const float* x, int n, const int* src, const int* dst, int64_t m_cap,
               const int* d_m, float* scores, GnnScratch& g, int n_cu, int* d_err, hipStream_t s, bool src_sorted) {
  if (n <= 0) return 0;
  const bool f32 = prec == TRK_PREC_F32;
  // split BF16 stores the same fragment blocks per k block as BF16; FP8 runs its
  // node side in BF16 and exists for H = 128 only (k in blocks of 128)
  if (prec == TRK_PREC_FP8) {
    if (net.H != 128 || !gnn_shapes_ok<PrecFP8, PrecBF16, 128>(net)) return -1;
    run_gnn128<PrecFP8>(net, x, n, src, dst, m_cap, d_m, scores, g, n_cu, d_err, s, src_sorted);
    return 0;
  }
  const bool ok = net.H == 128 ? (f32 ? gnn_shapes_ok<PrecF32, PrecF32, 128>(net)
                                      : gnn_shapes_ok<PrecBF16, PrecBF16, 128>(net))
                               : (f32 ? gnn_shapes_ok<PrecF32, PrecF32, 32>(net)
                                      : gnn_shapes_ok<PrecBF16, PrecBF16, 32>(net));
  if (!ok) return -1;
  if (prec == TRK_PREC_X3) {
    if (net.H == 128) { run_gnn128<PrecX3>(net, x, n, src, dst, m_cap, d_m, scores, g, n_cu, d_err, s, src_sorted); return 0; }
    if (net.H == 32) { run_gnn<PrecX3, PrecX3, 32, 64, 64, 1>(net, x, n, src, dst, m_cap, d_m, scores, g, n_cu, d_err, s, src_sorted); return 0; }
  } else if (prec == TRK_PREC_F32) {
    if (net.H == 128) { run_gnn128<PrecF32>(net, x, n, src, dst, m_cap, d_m, scores, g, n_cu, d_err, s, src_sorted); return 0; }
    if (net.H == 32) { run_gnn<PrecF32, PrecF32, 32, 64, 64, 1>(net, x, n, src, dst, m_cap, d_m, scores, g, n_cu, d_err, s, src_sorted); return 0; }
  } else {
    if (net.H == 128) { run_gnn128<PrecBF16>(net, x, n, src, dst, m_cap, d_m, scores, g, n_cu, d_err, s, src_sorted); return 0; }
    if (net.H == 32) { run_gnn<PrecBF16, PrecBF16, 32, 64, 64, 1>(net, x, n, src, dst, m_cap, d_m, scores, g, n_cu, d_err, s, src_sorted); return 0; }
  }
  return -1;
}
