// Roofline denominators measured on the device the library runs on: the dense
// matrix-core rate of each precision the kernels use, from a kernel that only
// issues independent MFMA chains from registers, and the HBM bandwidth of a plain
// coalesced copy.  The spec-sheet peaks are what the benchmark divides by; these
// give the fractions against what the part reaches.
#include "../../include/trk.h"
#include "common.h"
#include "mfma_tile.h"

namespace {

constexpr int PROBE_CHAINS = 8;   // independent accumulators per wave

template <int KIND>
__global__ __launch_bounds__(256) void mfma_probe_kernel(int64_t iters, float* __restrict__ sink) {
  const int l = lane_id();
  f32x4 acc[PROBE_CHAINS];
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
  // operands from the lane id, so that nothing folds at compile time
  const float fa = 1.f + 1e-3f * (float)l, fb = 1.f - 1e-3f * (float)l;
  bf16x8 ha, hb;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    ha[j] = (__bf16)(fa * (float)(j + 1));
    hb[j] = (__bf16)(fb * (float)(j + 1));
  }
  // E4M3 bytes around 1.0 (0x38) and 0.5 (0x30)
  const int va = 0x38383838 + (l & 7), vb = 0x30303030 + (l & 3);
  const i32x8 qa = {va, va, va, va, va, va, va, va};
  const i32x8 qb = {vb, vb, vb, vb, vb, vb, vb, vb};
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) {
      if constexpr (KIND == 0) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa, fb, acc[c], 0, 0, 0);
      else if constexpr (KIND == 1) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ha, hb, acc[c], 0, 0, 0);
      else acc[c] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(qa, qb, acc[c], 0, 0, 0, 127, 0, 127);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void copy_probe_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                         int64_t n16) {
  GRID_STRIDE(i, n16) dst[i] = src[i];
}

}  // namespace

extern "C" int trk_probe_mfma(int device, int precision, int64_t iters, double* tflops) {
  if (!tflops || iters < 1 || precision < TRK_FP32 || precision > TRK_FP8) return TRK_E_INVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TRK_E_INVAL;
  if (hipSetDevice(device) != hipSuccess) return TRK_E_DEVICE;
  int n_cu = 0;
  hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
  if (n_cu <= 0) n_cu = 256;
  const int blocks = n_cu * 8;   // eight 4-wave blocks per CU: eight waves per SIMD
  float* sink = nullptr;
  if (hipMalloc(&sink, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return TRK_E_NOMEM;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  auto launch = [&](int64_t n) {
    if (precision == TRK_FP32) mfma_probe_kernel<0><<<blocks, 256>>>(n, sink);
    else if (precision == TRK_BF16) mfma_probe_kernel<1><<<blocks, 256>>>(n, sink);
    else mfma_probe_kernel<2><<<blocks, 256>>>(n, sink);
  };
  launch(16);   // warm-up
  hipEventRecord(e0, nullptr);
  launch(iters);
  hipEventRecord(e1, nullptr);
  int rc = TRK_OK;
  float ms = 0.f;
  if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
      hipGetLastError() != hipSuccess)
    rc = TRK_E_DEVICE;
  const double per = precision == TRK_FP32 ? 2.0 * 16 * 16 * 4 : precision == TRK_BF16 ? 2.0 * 16 * 16 * 32
                                                                                      : 2.0 * 16 * 16 * 128;
  const double flops = (double)blocks * 4 * (double)iters * PROBE_CHAINS * per;
  *tflops = rc == TRK_OK && ms > 0.f ? flops / (ms * 1e-3) / 1e12 : 0.0;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(sink);
  return rc;
}

extern "C" int trk_probe_copy(const void* d_src, void* d_dst, size_t bytes, int reps, hipStream_t s,
                              double* gbps) {
  if (!d_src || !d_dst || !gbps || reps < 1 || bytes < 16 || bytes % 16) return TRK_E_INVAL;
  if (((uintptr_t)d_src | (uintptr_t)d_dst) & 15) return TRK_E_INVAL;
  const int64_t n16 = (int64_t)(bytes / 16);
  int dev = 0;
  hipGetDevice(&dev);
  int n_cu = 0;
  hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (n_cu <= 0) n_cu = 256;
  const int grid = blocks_for(n16, 256, n_cu * 16);
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  copy_probe_kernel<<<grid, 256, 0, s>>>((const uint4*)d_src, (uint4*)d_dst, n16);   // warm-up
  hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) copy_probe_kernel<<<grid, 256, 0, s>>>((const uint4*)d_src, (uint4*)d_dst, n16);
  hipEventRecord(e1, s);
  int rc = TRK_OK;
  float ms = 0.f;
  if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
      hipGetLastError() != hipSuccess)
    rc = TRK_E_DEVICE;
  // a copy reads and writes every byte
  *gbps = rc == TRK_OK && ms > 0.f ? 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9 : 0.0;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}
