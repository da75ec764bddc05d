// MFMA tile engine for the row-tile MLP kernels (gfx950, wave64).
//
// A layer computes out[m][n] = sum_k X[m][k] * W[k][n] for a tile of rows held in
// LDS.  The product is issued in transposed form, D = W^T X^T, so that the 16x16
// accumulator of a lane holds four consecutive output columns of one row:
//   lane l, register i  ->  row m = 16*mt + (l & 15),  column n = 16*nt + 4*(l >> 4) + i.
// Operand fragments per lane:
//   FP32 (v_mfma_f32_16x16x4_f32, four issues per 16-byte fragment): lane group
//        g = l>>4 carries k = 16*kb + 4g + s in issue s = 0..3;
//   BF16 (v_mfma_f32_16x16x32_bf16, 16 bytes): lane group g carries k = 32*kb + 8g + j, j = 0..7;
//   FP8  (v_mfma_scale_f32_16x16x128_f8f6f4 in E4M3 mode with unit block scales,
//        32 bytes): lane group g carries k = 128*kb + 32g + j, j = 0..31;
//   split BF16 (three v_mfma_f32_16x16x32_bf16 per block, 32 bytes): as BF16, the
//        high parts of the eight values then their low parts.
// Any assignment of k to (lane group, slot) is valid as long as the weight and the
// activation fragments agree, which lets each lane read 16 contiguous bytes of its
// activation row from LDS.  Weights are pre-arranged on the host into "fragment
// blocks": block (nt, kb) of a layer is 64 lanes x sizeof(fragment), stored at
// index nt * nkb + kb, so that a wave fetches one block with coalesced loads.
//
// Epilogues compute tanh(acc * dq + b): dq is 1 for FP32 and BF16 layers and the
// product of the inverse weight and activation scales for FP8 layers, so the
// dequantisation rides on the bias addition (one FMA either way).
#pragma once
#include "common.h"

#include <type_traits>

typedef int i32x8 __attribute__((ext_vector_type(8)));

struct PrecF32 {
  typedef float act_t;
  typedef uint4 frag_t;
  static constexpr int KB = 16;          // k per fragment block
  static constexpr int PAD = 4;          // row padding in elements (16 bytes)
  // four dependent issues into one accumulator (interleaving them over the
  // tile's accumulators measured slower on MI355X)
  static __device__ __forceinline__ void mma_first(f32x4& acc, const uint4& w, const uint4& x) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(w.x), __uint_as_float(x.x), f32x4{0.f, 0.f, 0.f, 0.f},
                                               0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(w.y), __uint_as_float(x.y), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(w.z), __uint_as_float(x.z), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(w.w), __uint_as_float(x.w), acc, 0, 0, 0);
  }
  static __device__ __forceinline__ void mma(f32x4& acc, const uint4& w, const uint4& x) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(w.x), __uint_as_float(x.x), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(w.y), __uint_as_float(x.y), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(w.z), __uint_as_float(x.z), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(w.w), __uint_as_float(x.w), acc, 0, 0, 0);
  }
  // store four consecutive columns
  static __device__ __forceinline__ void store4(float* p, float a, float b, float c, float d) {
    *(float4*)p = make_float4(a, b, c, d);
  }
  static __device__ __forceinline__ float load1(const float* p) { return *p; }
  static __device__ __forceinline__ float cvt(float v) { return v; }
  // element k of a row
  static __device__ __forceinline__ void store1(float* row, int k, float v) { row[k] = v; }
  // the values held by 16 bytes of a row
  static constexpr int V16 = 4;
  static __device__ __forceinline__ void unpack16(const uint4& u, float (&v)[V16]) {
    v[0] = __uint_as_float(u.x); v[1] = __uint_as_float(u.y); v[2] = __uint_as_float(u.z); v[3] = __uint_as_float(u.w);
  }
};

struct PrecBF16 {
  typedef __bf16 act_t;
  typedef uint4 frag_t;
  static constexpr int KB = 32;
  static constexpr int PAD = 8;
  static __device__ __forceinline__ void mma(f32x4& acc, const uint4& w, const uint4& x) {
    bf16x8 a = __builtin_bit_cast(bf16x8, w);
    bf16x8 b = __builtin_bit_cast(bf16x8, x);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  static __device__ __forceinline__ void mma_first(f32x4& acc, const uint4& w, const uint4& x) {
    bf16x8 a = __builtin_bit_cast(bf16x8, w);
    bf16x8 b = __builtin_bit_cast(bf16x8, x);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  }
  static __device__ __forceinline__ void store4(__bf16* p, float a, float b, float c, float d) {
    bf16x4 v = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
    *(bf16x4*)p = v;
  }
  static __device__ __forceinline__ float load1(const __bf16* p) { return (float)*p; }
  static __device__ __forceinline__ __bf16 cvt(float v) { return (__bf16)v; }
  static __device__ __forceinline__ void store1(__bf16* row, int k, float v) { row[k] = (__bf16)v; }
  static constexpr int V16 = 8;
  static __device__ __forceinline__ void unpack16(const uint4& u, float (&v)[V16]) {
    const bf16x8 b = __builtin_bit_cast(bf16x8, u);
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (float)b[q];
  }
};

// Split BF16: a value v is held as hi = bf16(v) and lo = bf16(v - hi) (both
// round-to-nearest-even): hi + lo is within 2^-18 of v relatively.  A product is
// formed from three BF16 products, hi*hi + hi*lo + lo*hi, accumulated in FP32; the
// dropped lo*lo term is below 2^-18 of the product, the order of the split's own
// representation error.  This is the three-term
// split of Henry, Tang and Heinecke (ARITH 2019), here on the BF16 matrix cores.
// Storage: in every group of four consecutive elements of a row (16 bytes), the
// four high parts, then the four low parts, so that 16-byte moves of a row move
// whole elements.  One element is the 4-byte unit x3_t.
struct x3_t {
  uint32_t bits;
};

struct PrecX3 {
  typedef x3_t act_t;
  typedef i32x8 frag_t;
  static constexpr int KB = 32;
  static constexpr int PAD = 4;
  static __device__ __forceinline__ void mma(f32x4& acc, const i32x8& w, const i32x8& x) {
    const bf16x8 wh = __builtin_bit_cast(bf16x8, __builtin_shufflevector(w, w, 0, 1, 2, 3));
    const bf16x8 wl = __builtin_bit_cast(bf16x8, __builtin_shufflevector(w, w, 4, 5, 6, 7));
    const bf16x8 xh = __builtin_bit_cast(bf16x8, __builtin_shufflevector(x, x, 0, 1, 2, 3));
    const bf16x8 xl = __builtin_bit_cast(bf16x8, __builtin_shufflevector(x, x, 4, 5, 6, 7));
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, xh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xh, acc, 0, 0, 0);
  }
  static __device__ __forceinline__ void mma_first(f32x4& acc, const i32x8& w, const i32x8& x) {
    const bf16x8 wh = __builtin_bit_cast(bf16x8, __builtin_shufflevector(w, w, 0, 1, 2, 3));
    const bf16x8 wl = __builtin_bit_cast(bf16x8, __builtin_shufflevector(w, w, 4, 5, 6, 7));
    const bf16x8 xh = __builtin_bit_cast(bf16x8, __builtin_shufflevector(x, x, 0, 1, 2, 3));
    const bf16x8 xl = __builtin_bit_cast(bf16x8, __builtin_shufflevector(x, x, 4, 5, 6, 7));
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, xh, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xh, acc, 0, 0, 0);
  }
  static __device__ __forceinline__ void split(float v, __bf16& h, __bf16& l) {
    h = (__bf16)v;
    l = (__bf16)(v - (float)h);
  }
  // four consecutive elements starting at a multiple of four
  static __device__ __forceinline__ void store4(x3_t* p, float a, float b, float c, float d) {
    bf16x4 h, l;
    __bf16 t0, t1;
    split(a, t0, t1); h[0] = t0; l[0] = t1;
    split(b, t0, t1); h[1] = t0; l[1] = t1;
    split(c, t0, t1); h[2] = t0; l[2] = t1;
    split(d, t0, t1); h[3] = t0; l[3] = t1;
    const uint2 hu = __builtin_bit_cast(uint2, h), lu = __builtin_bit_cast(uint2, l);
    *(uint4*)p = make_uint4(hu.x, hu.y, lu.x, lu.y);
  }
  static __device__ __forceinline__ void store1(x3_t* row, int k, float v) {
    __bf16* q = (__bf16*)(row + (k & ~3));
    __bf16 h, l;
    split(v, h, l);
    q[k & 3] = h;
    q[4 + (k & 3)] = l;
  }
  static constexpr int V16 = 4;
  static __device__ __forceinline__ void unpack16(const uint4& u, float (&v)[V16]) {
    const bf16x8 b = __builtin_bit_cast(bf16x8, u);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (float)b[q] + (float)b[4 + q];
  }
};

// OCP FP8 E4M3 (max 448).  Activations are tanh outputs (|a| <= 1) stored as
// E4M3(256 a): the static scale keeps them in the normal range down to |a| ~ 6e-5.
// Weights carry a per-tensor power-of-two scale chosen on the host.
struct PrecFP8 {
  typedef uint8_t act_t;
  typedef i32x8 frag_t;
  static constexpr int KB = 128;
  static constexpr int PAD = 16;
  static constexpr float ACT_SCALE = 256.f;
  static __device__ __forceinline__ void mma(f32x4& acc, const i32x8& w, const i32x8& x) {
    // format 0 (E4M3) for both operands, block scales 2^(127-127) = 1
    acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(w, x, acc, 0, 0, 0, 127, 0, 127);
  }
  static __device__ __forceinline__ void mma_first(f32x4& acc, const i32x8& w, const i32x8& x) {
    acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(w, x, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0, 127, 0, 127);
  }
  static __device__ __forceinline__ void store4(uint8_t* p, float a, float b, float c, float d) {
    int v = __builtin_amdgcn_cvt_pk_fp8_f32(a * ACT_SCALE, b * ACT_SCALE, 0, false);
    v = __builtin_amdgcn_cvt_pk_fp8_f32(c * ACT_SCALE, d * ACT_SCALE, v, true);
    *(int*)p = v;
  }
  // four E4M3 values of (s * a, s * b, s * c, s * d), element k at byte k
  static __device__ __forceinline__ void store4_scaled(uint8_t* p, float a, float b, float c, float d, float s) {
    int v = __builtin_amdgcn_cvt_pk_fp8_f32(a * s, b * s, 0, false);
    v = __builtin_amdgcn_cvt_pk_fp8_f32(c * s, d * s, v, true);
    *(int*)p = v;
  }
  // the sixteen E4M3 values held by 16 bytes of a row, as stored (scale not removed)
  static constexpr int V16 = 16;
  static __device__ __forceinline__ void unpack16(const uint4& u, float (&v)[V16]) {
    const int w[4] = {(int)u.x, (int)u.y, (int)u.z, (int)u.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(w[q], false);
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(w[q], true);
      v[4 * q] = lo[0];
      v[4 * q + 1] = lo[1];
      v[4 * q + 2] = hi[0];
      v[4 * q + 3] = hi[1];
    }
  }
};

template <class P>
__device__ __forceinline__ typename P::frag_t load_frag(const typename P::act_t* p) {
  if constexpr (std::is_same<P, PrecX3>::value) {
    // eight elements = two 16-byte groups (hi0..3 lo0..3, hi4..7 lo4..7)
    const uint4 a = *(const uint4*)p, b = *(const uint4*)(p + 4);
    return i32x8{(int)a.x, (int)a.y, (int)b.x, (int)b.y, (int)a.z, (int)a.w, (int)b.z, (int)b.w};
  } else if constexpr (sizeof(typename P::frag_t) == 16) {
    return *(const uint4*)p;
  } else {
    const uint4 a = *(const uint4*)p, b = *(const uint4*)(p + 16);
    return typename P::frag_t{(int)a.x, (int)a.y, (int)a.z, (int)a.w, (int)b.x, (int)b.y, (int)b.z, (int)b.w};
  }
}

template <int MTW, int NTW>
__device__ __forceinline__ void acc_zero(f32x4 (&acc)[MTW][NTW]) {
#pragma unroll
  for (int i = 0; i < MTW; ++i)
#pragma unroll
    for (int j = 0; j < NTW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// acc[i][j] += X[rows of m-tile i] * W[:, n-tile nt0 + j] over fragment blocks
// kb0 .. kb0 + nkb_run - 1 of a layer with nkb blocks per n-tile (INIT: acc = the
// product; the first block's issues take a zero accumulator, so acc needs no
// clearing; requires nkb_run >= 1, which every layer has).  xs: LDS activation
// tile (row-major, leading dimension ldx elements), row 0 = m-tile 0.
template <class P, int MTW, int NTW, bool INIT = false>
__device__ __forceinline__ void tile_gemm(f32x4 (&acc)[MTW][NTW], const typename P::act_t* xs, int ldx,
                                          const uint4* __restrict__ wb, int nkb, int nt0, int kb0,
                                          int nkb_run) {
  const int l = lane_id();
  const int g = l >> 4, r = l & 15;
  const typename P::act_t* xl = xs + r * ldx + g * (P::KB / 4);
  typedef typename P::frag_t F;
  const F* wl = (const F*)wb + (size_t)nt0 * nkb * 64 + l;
  if (!INIT && nkb_run <= 0) return;
  // one weight fragment per n-tile in flight: the fragment of n-tile j for the next k
  // block is requested as soon as the current one has been consumed
  F w[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) w[j] = wl[((size_t)j * nkb + kb0) * 64];
  // one k block; FIRST: the issues start from a zero accumulator
  auto block = [&](int kk, auto first) {
    const int kb = kb0 + kk;
    // the last block re-reads itself so that every load is unconditional and the
    // compiler can wait for each fragment individually
    const int kbn = kk + 1 < nkb_run ? kb + 1 : kb;
    F xf[MTW];
#pragma unroll
    for (int i = 0; i < MTW; ++i) xf[i] = load_frag<P>(xl + i * 16 * ldx + kb * P::KB);
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        if constexpr (decltype(first)::value) P::mma_first(acc[i][j], w[j], xf[i]);
        else P::mma(acc[i][j], w[j], xf[i]);
      }
      w[j] = wl[((size_t)j * nkb + kbn) * 64];
      // keep the issue order: n-tile j's products, then its next fragment request
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  int kk = 0;
  if constexpr (INIT) {
    block(0, std::true_type{});
    kk = 1;
  }
  for (; kk < nkb_run; ++kk) block(kk, std::false_type{});
}

// The same product for a compile-time number of k blocks NKB (the small square
// layers of the interaction network), fully unrolled: the weight fragments of the
// next DIST k blocks are in flight while the current one is multiplied, and the
// compiler can wait for each fragment individually.  nkb is the layer's stored
// block count per n-tile (the stride of the fragment array); NKB <= nkb.
template <class P, int MTW, int NTW, int NKB, int DIST, bool INIT = false>
__device__ __forceinline__ void tile_gemm_k(f32x4 (&acc)[MTW][NTW], const typename P::act_t* xs, int ldx,
                                            const uint4* __restrict__ wb, int nkb, int nt0) {
  typedef typename P::frag_t F;
  constexpr int D = DIST < NKB ? DIST : NKB;
  const int l = lane_id();
  const int g = l >> 4, r = l & 15;
  const typename P::act_t* xl = xs + r * ldx + g * (P::KB / 4);
  const F* wl = (const F*)wb + (size_t)nt0 * nkb * 64 + l;
  F w[D][NTW];
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int j = 0; j < NTW; ++j) w[d][j] = wl[((size_t)j * nkb + d) * 64];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) {
    F xf[MTW];
#pragma unroll
    for (int i = 0; i < MTW; ++i) xf[i] = load_frag<P>(xl + i * 16 * ldx + kb * P::KB);
#pragma unroll
    for (int j = 0; j < NTW; ++j) {
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        if (INIT && kb == 0) P::mma_first(acc[i][j], w[kb % D][j], xf[i]);
        else P::mma(acc[i][j], w[kb % D][j], xf[i]);
      }
      if (kb + D < NKB) w[kb % D][j] = wl[((size_t)j * nkb + kb + D) * 64];
    }
  }
}

// Epilogue: out = tanh(acc * dq + bias) written to an LDS tile (leading dimension
// ldo) in the storage format of P; bias_s is the bias times 2 log2(e).
template <class P, int MTW, int NTW>
__device__ __forceinline__ void tile_store_tanh(const f32x4 (&acc)[MTW][NTW], const float* __restrict__ bias_s,
                                                float dq, typename P::act_t* out, int ldo, int nt0) {
  const int l = lane_id();
  const int g = l >> 4, r = l & 15;
  const float s = dq * TRK_2LOG2E;
#pragma unroll
  for (int j = 0; j < NTW; ++j) {
    const int n = (nt0 + j) * 16 + 4 * g;
    const float4 b = *(const float4*)(bias_s + n);
#pragma unroll
    for (int i = 0; i < MTW; ++i) {
      const f32x4 a = acc[i][j];
      P::store4(out + (i * 16 + r) * ldo + n, trk_tanh_log2(fmaf(a[0], s, b.x)), trk_tanh_log2(fmaf(a[1], s, b.y)),
                trk_tanh_log2(fmaf(a[2], s, b.z)), trk_tanh_log2(fmaf(a[3], s, b.w)));
    }
  }
}
