// Internal device helpers shared by the gfx950 kernels of libtrk.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

#define TRK_WAVE 64

// ---------------------------------------------------------------------------
// Elementwise functions.  tanh and the logistic function are evaluated from
// the hardware base-2 exponential (v_exp_f32) and reciprocal (v_rcp_f32) with the
// identities tanh(x) = 1 - 2 / (exp(2x) + 1) and sigma(z) = 1 / (1 + exp(-z)),
// whose absolute error is a few float32 ulps of 1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float trk_exp(float x) {
  return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
}

// tanh(x) = 1 - 2 / (exp(2x) + 1), from y = 2 x log2(e): one exponential, one
// reciprocal.  No clamp is needed: for large y the exponential overflows to +inf,
// whose reciprocal is 0 (tanh = 1), and for very negative y it underflows to 0
// (tanh = -1).  Callers that compute a * s + b fold log2(e) into s and b.
constexpr float TRK_2LOG2E = 2.8853900817779268f;
__device__ __forceinline__ float trk_tanh_log2(float y) {
  return fmaf(-2.0f, __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(y) + 1.0f), 1.0f);
}
__device__ __forceinline__ float trk_tanh(float x) { return trk_tanh_log2(x * TRK_2LOG2E); }

__device__ __forceinline__ float trk_sigmoid(float z) {
  z = __builtin_amdgcn_fmed3f(z, -80.0f, 80.0f);
  return __builtin_amdgcn_rcpf(1.0f + trk_exp(-z));
}

// float <-> bf16, round to nearest even
__device__ __forceinline__ __bf16 f2bf(float x) { return (__bf16)x; }
__device__ __forceinline__ float bf2f(__bf16 x) { return (float)x; }

// ---------------------------------------------------------------------------
// Wave-level scans and reductions (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (l >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

// number of set lanes below this lane in a ballot mask
__device__ __forceinline__ int mask_rank(unsigned long long m) {
  const int l = lane_id();
  return __popcll(m & ((l == 0) ? 0ull : (~0ull >> (64 - l))));
}

// Relaxed device-scope atomic load (bypasses the per-CU cache)
__device__ __forceinline__ int load_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t clamp_count(const int* d_count, int64_t cap) {
  int64_t c = *d_count;
  return c < cap ? c : cap;
}

// ---------------------------------------------------------------------------
// Grid-stride helpers
// ---------------------------------------------------------------------------
#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)(n); i += (int64_t)gridDim.x * blockDim.x)

static inline int blocks_for(int64_t n, int threads, int max_blocks = 4096) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (int)b;
}
