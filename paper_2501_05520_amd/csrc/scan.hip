// Device-wide exclusive scan, order-preserving edge compaction and segmented
// rank sort.  Work counts may live in device memory: grids are sized by a
// capacity and blocks past the live count exit at once, so these can be chained
// behind producers without a host round trip.  All results are deterministic.
#include "kernels.h"
#include "common.h"

namespace {

constexpr int ST = 256;          // threads per block
constexpr int SPT = 16;          // items per thread
constexpr int CHUNK = ST * SPT;  // items per block

__device__ __forceinline__ int64_t live_count(int64_t cap, const int* d_n) {
  if (!d_n) return cap;
  const int64_t v = *d_n;
  return v < cap ? v : cap;
}

// exclusive scan of one value per thread over a 256-thread block; returns the
// exclusive prefix and the block total
__device__ __forceinline__ int block_scan(int v, int& total) {
  __shared__ int sh[ST / 64];
  const int incl = wave_incl_scan(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) sh[w] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < ST / 64; ++i) {
    const int s = sh[i];
    off += (i < w) ? s : 0;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return off + incl - v;
}

__global__ __launch_bounds__(ST) void scan_reduce(const int* __restrict__ in, int64_t n_cap, const int* d_n,
                                                  int* __restrict__ part) {
  const int64_t n = live_count(n_cap, d_n);
  const int64_t base = (int64_t)blockIdx.x * CHUNK + (int64_t)threadIdx.x * SPT;
  int s = 0;
  if ((int64_t)blockIdx.x * CHUNK < n) {
#pragma unroll
    for (int i = 0; i < SPT; ++i) s += (base + i < n) ? in[base + i] : 0;
  }
  int tot;
  block_scan(s, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single block: exclusive scan of part[0..nb) in place, part[nb] = total
__global__ __launch_bounds__(1024) void scan_parts(int* __restrict__ part, int nb, int* d_total,
                                                   int* out_last, int64_t n_cap, const int* d_n) {
  __shared__ int sh[16];
  __shared__ int carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? part[i] : 0;
    const int incl = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) sh[w] = incl;
    __syncthreads();
    int off = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
      off += (k < w) ? sh[k] : 0;
      tot += sh[k];
    }
    const int carry = carry_s;
    if (i < nb) part[i] = carry + off + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) carry_s = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[nb] = carry_s;
    if (d_total) *d_total = carry_s;
    if (out_last) out_last[live_count(n_cap, d_n)] = carry_s;
  }
}

__global__ __launch_bounds__(ST) void scan_apply(const int* __restrict__ in, int* __restrict__ out, int64_t n_cap,
                                                 const int* d_n, const int* __restrict__ part) {
  const int64_t n = live_count(n_cap, d_n);
  if ((int64_t)blockIdx.x * CHUNK >= n) return;
  const int64_t base = (int64_t)blockIdx.x * CHUNK + (int64_t)threadIdx.x * SPT;
  int v[SPT];
  int s = 0;
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  int tot;
  int run = block_scan(s, tot) + part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

__global__ __launch_bounds__(ST) void compact_count(const float* __restrict__ scores, float cut, int64_t m_cap,
                                                    const int* d_m, int* __restrict__ part) {
  const int64_t m = live_count(m_cap, d_m);
  const int64_t base = (int64_t)blockIdx.x * CHUNK + (int64_t)threadIdx.x * SPT;
  int s = 0;
  if ((int64_t)blockIdx.x * CHUNK < m) {
#pragma unroll
    for (int i = 0; i < SPT; ++i) s += (base + i < m && scores[base + i] > cut) ? 1 : 0;
  }
  int tot;
  block_scan(s, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(ST) void compact_scatter(const float* __restrict__ scores, float cut,
                                                      const int* __restrict__ src, const int* __restrict__ dst,
                                                      int64_t m_cap, const int* d_m, const int* __restrict__ part,
                                                      int* __restrict__ osrc, int* __restrict__ odst,
                                                      int64_t out_cap) {
  const int64_t m = live_count(m_cap, d_m);
  if ((int64_t)blockIdx.x * CHUNK >= m) return;
  const int64_t base = (int64_t)blockIdx.x * CHUNK + (int64_t)threadIdx.x * SPT;
  bool f[SPT];
  int s = 0;
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    f[i] = base + i < m && scores[base + i] > cut;
    s += f[i] ? 1 : 0;
  }
  int tot;
  int64_t pos = (int64_t)block_scan(s, tot) + part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    if (f[i]) {
      if (pos < out_cap) {
        osrc[pos] = src[base + i];
        odst[pos] = dst[base + i];
      }
      ++pos;
    }
  }
}

__global__ void fill_int(int* p, int v, int64_t n) {
  GRID_STRIDE(i, n) p[i] = v;
}
__global__ void set_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Rank sort of unique keys per segment: the key with r smaller keys in its segment goes
// to position r.  One wave per segment; segments up to SEG_LDS keys are staged in LDS.
constexpr int SEG_WAVES = 4;
constexpr int SEG_LDS = 1024;
__global__ __launch_bounds__(SEG_WAVES * 64) void segment_rank_sort(const int* __restrict__ ptr,
                                                                    const int* __restrict__ in,
                                                                    int* __restrict__ out, int nseg) {
  __shared__ int keys[SEG_WAVES][SEG_LDS];
  const int w = threadIdx.x >> 6, l = lane_id();
  for (int seg = blockIdx.x * SEG_WAVES + w; seg < nseg; seg += gridDim.x * SEG_WAVES) {
    const int b = ptr[seg], e = ptr[seg + 1], L = e - b;
    if (L <= 0) continue;
    if (L == 1) {
      if (l == 0) out[b] = in[b];
      continue;
    }
    if (L <= SEG_LDS) {
      for (int i = l; i < L; i += 64) keys[w][i] = in[b + i];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      for (int i = l; i < L; i += 64) {
        const int k = keys[w][i];
        int rank = 0;
        for (int j = 0; j < L; ++j) rank += keys[w][j] < k ? 1 : 0;
        out[b + rank] = k;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    } else {
      for (int i = l; i < L; i += 64) {
        const int k = in[b + i];
        int rank = 0;
        for (int j = 0; j < L; ++j) rank += in[b + j] < k ? 1 : 0;
        out[b + rank] = k;
      }
    }
  }
}

}  // namespace

int64_t scan_tmp_ints(int64_t n) { return n / CHUNK + 4; }

void launch_scan_excl(const int* in, int* out, int64_t n_cap, const int* d_n, int* d_total, int* tmp,
                      hipStream_t s) {
  const int nb = (int)((n_cap + CHUNK - 1) / CHUNK) > 0 ? (int)((n_cap + CHUNK - 1) / CHUNK) : 1;
  scan_reduce<<<nb, ST, 0, s>>>(in, n_cap, d_n, tmp);
  scan_parts<<<1, 1024, 0, s>>>(tmp, nb, d_total, out, n_cap, d_n);
  scan_apply<<<nb, ST, 0, s>>>(in, out, n_cap, d_n, tmp);
}

void launch_compact_edges(const float* scores, float cut, const int* src, const int* dst, int64_t m_cap,
                          const int* d_m, int* out_src, int* out_dst, int64_t out_cap, int* d_count, int* tmp,
                          hipStream_t s) {
  const int nb = (int)((m_cap + CHUNK - 1) / CHUNK) > 0 ? (int)((m_cap + CHUNK - 1) / CHUNK) : 1;
  compact_count<<<nb, ST, 0, s>>>(scores, cut, m_cap, d_m, tmp);
  scan_parts<<<1, 1024, 0, s>>>(tmp, nb, d_count, nullptr, 0, nullptr);
  compact_scatter<<<nb, ST, 0, s>>>(scores, cut, src, dst, m_cap, d_m, tmp, out_src, out_dst, out_cap);
}

void launch_fill_int(int* p, int v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  fill_int<<<blocks_for(n, 256), 256, 0, s>>>(p, v, n);
}

void launch_set_int(int* p, int64_t v, hipStream_t s) { set_int<<<1, 64, 0, s>>>(p, (int)v); }

void launch_segment_sort(const int* ptr, const int* in, int* out, int n, hipStream_t s) {
  if (n <= 0) return;
  const int grid = blocks_for(n, SEG_WAVES, 8192);
  segment_rank_sort<<<grid, SEG_WAVES * 64, 0, s>>>(ptr, in, out, n);
}
