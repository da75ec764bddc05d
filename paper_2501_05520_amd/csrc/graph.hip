// Fixed-radius candidate graph in the embedding space (Section 2.2.2: edges join
// spacepoints closer than a fixed radius in the latent space).
//
// Grid search in a 3-D projection.  The embedding (D <= 16 dims) is projected on
// three orthonormal directions - the leading principal axes of the batch,
// found by subspace iteration on its FP64 covariance.  An orthonormal projection
// does not increase distances, so two points closer than r fall in the same or
// adjacent cells of a cubic grid of edge >= r: every true neighbour of a point
// lies in the 27 cells around it.  Cells are keyed by (event, cx, cy, cz) and
// hashed into a table of buckets; a counting sort by bucket lays the points out
// cell-contiguously, and each entry keeps its exact cell key so that buckets
// shared by several cells are filtered exactly.
//
// Selection and canonical edges.  Point i selects the k_max nearest points j != i
// with d^2 < r^2 (FP32 squared distance, summed over dimensions in fixed order,
// hence bitwise symmetric), ordered by the 64-bit key (bits(d^2) << 32 | j).
// For saturated points the k_max-th key is found by an 8-pass radix select (over
// the keys staged in LDS when they fit).  The
// candidate edge set is the union of the selections as pairs (min, max):
//   pass 2 counts each pair once - point i owns (i, j) when it selects j > i, and
//          (j, i) when it selects j < i that does not select it back;
//   pass 3 writes the pairs into per-row slots, and a rank sort orders each row,
// giving the edge list sorted by (src, dst) independent of scheduling.
#include "kernels.h"
#include "common.h"

namespace {

constexpr int QW = 4;                 // waves per block in the query kernels
constexpr int EP = 16;                // padded embedding width
constexpr int NSLOT = 27;
constexpr double CELL_MARGIN = 1e-6;  // cell edge = r (1 + margin)

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ unsigned long long cell_key(int ev, int cx, int cy, int cz) {
  return ((unsigned long long)(ev & 0xFFFF) << 48) | ((unsigned long long)((cx + 32768) & 0xFFFF) << 32) |
         ((unsigned long long)((cy + 32768) & 0xFFFF) << 16) | (unsigned long long)((cz + 32768) & 0xFFFF);
}

__device__ __forceinline__ int clamp_cell(double v) {
  v = fmin(fmax(v, -32767.0), 32767.0);
  return (int)floor(v);
}

// ---------------------------------------------------------------------------
// Projection basis
// ---------------------------------------------------------------------------
constexpr int NSTAT = EP + EP * (EP + 1) / 2;  // sums and upper-triangle second moments
constexpr int STAT_T = 256;

__global__ __launch_bounds__(STAT_T) void stats_kernel(const float* __restrict__ emb, int n, int D,
                                                       double* __restrict__ part) {
  __shared__ float tile[STAT_T][EP + 1];
  double acc = 0.0;
  const int t = threadIdx.x;
  // thread t < NSTAT owns statistic t: t < EP -> sum e_t, else product e_a e_b (a <= b)
  int a = -1, b = -1;
  if (t < EP) {
    a = t;
  } else if (t < NSTAT) {
    int k = t - EP;
    a = 0;
    while (k >= EP - a) { k -= EP - a; ++a; }
    b = a + k;
  }
  for (int64_t base = (int64_t)blockIdx.x * STAT_T; base < n; base += (int64_t)gridDim.x * STAT_T) {
    const int64_t i = base + t;
    for (int k = 0; k < EP; ++k) tile[t][k] = (i < n && k < D) ? emb[i * D + k] : 0.f;
    __syncthreads();
    const int cnt = (int)min((int64_t)STAT_T, n - base);
    if (a >= 0) {
      if (b < 0)
        for (int r = 0; r < cnt; ++r) acc += (double)tile[r][a];
      else
        for (int r = 0; r < cnt; ++r) acc += (double)tile[r][a] * (double)tile[r][b];
    }
    __syncthreads();
  }
  if (t < NSTAT) part[(size_t)blockIdx.x * NSTAT + t] = acc;
}

// One block: sum partials (fixed order), form the covariance, run subspace
// iteration for the three leading eigenvectors on its fourth power and
// orthonormalise them (FP64).
// basis layout (doubles): [0..3*EP) directions, then cell edge, then spare.
__global__ __launch_bounds__(256) void basis_kernel(const double* __restrict__ part, int nblocks, int n, int D,
                                                    float radius, double* __restrict__ basis) {
  __shared__ double st[NSTAT];
  __shared__ double C[EP][EP];
  const int t = threadIdx.x;
  if (t < NSTAT) {
    double s = 0.0;
    for (int bk = 0; bk < nblocks; ++bk) s += part[(size_t)bk * NSTAT + t];
    st[t] = s;
  }
  __syncthreads();
  const double inv_n = n > 0 ? 1.0 / (double)n : 0.0;
  if (t < EP * EP) {
    const int a = t / EP, b = t % EP;
    double v = 0.0;
    if (a < D && b < D) {
      const int lo = a < b ? a : b, hi = a < b ? b : a;
      int idx = EP;
      for (int q = 0; q < lo; ++q) idx += EP - q;
      idx += hi - lo;
      v = st[idx] * inv_n - (st[a] * inv_n) * (st[b] * inv_n);
    }
    C[a][b] = v;
  }
  __syncthreads();
  // iterate with the fourth power of the trace-normalised covariance (same
  // eigenvectors, eigenvalue ratios to the fourth power: one step does the work of
  // four); its eigenvalues lie in [0, 1]
  __shared__ double C2[EP][EP];
  {
    double tr = 0.0;
    for (int q = 0; q < EP; ++q) tr += C[q][q];
    const double inv = tr > 0.0 ? 1.0 / tr : 1.0;
    const int a = t / EP, b = t % EP;
    double v = 0.0;
    for (int q = 0; q < EP; ++q) v += C[a][q] * C[q][b];
    __syncthreads();
    C2[a][b] = v * inv * inv;
    __syncthreads();
    v = 0.0;
    for (int q = 0; q < EP; ++q) v += C2[a][q] * C2[q][b];
    C[a][b] = v;
  }
  __syncthreads();
  // the iteration runs in one wave, in registers: lane l < 3 EP holds V[l / EP][l % EP]
  if (t >= 64) return;
  const int l = t, c = l / EP, k = l % EP;
  auto wave_sum = [](double d) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    return d;
  };
  // fixed dense start, distinct per column
  double v = (l < 3 * EP && k < D) ? cos(0.7 * (k + 1) * (c + 1) + 0.3 * c) : 0.0;
  for (int it = 0; it < 8; ++it) {
    double w = 0.0;
    for (int q = 0; q < EP; ++q) w += C[k][q] * __shfl(v, (c < 3 ? c : 3) * EP + q, 64);
    // keep a small multiple of the start vector so rank-deficient covariances still
    // leave three independent columns
    w += 1e-12 * v;
    // modified Gram-Schmidt on the three columns, in order
    for (int cc = 0; cc < 3; ++cc) {
      for (int p = 0; p < cc; ++p) {
        const double wp = __shfl(w, p * EP + k, 64);
        const double d = wave_sum(c == cc ? w * wp : 0.0);
        if (c == cc) w -= d * wp;
      }
      const double nn = wave_sum(c == cc ? w * w : 0.0);
      if (c == cc) w *= nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    }
    v = w;
  }
  // the columns must come out orthonormal; a degenerate run falls back to coordinate axes
  bool ok = true;
  for (int cc = 0; cc < 3; ++cc)
    for (int p = 0; p <= cc; ++p) {
      const double d = wave_sum(c == cc ? v * __shfl(v, p * EP + k, 64) : 0.0);
      ok = ok && fabs(d - (p == cc ? 1.0 : 0.0)) < 1e-9;
    }
  if (l < 3 * EP) basis[l] = ok ? v : (k == c ? 1.0 : 0.0);
  if (l == 0) basis[3 * EP] = (double)radius * (1.0 + CELL_MARGIN);
}

// ---------------------------------------------------------------------------
// Cells, histogram and counting sort by bucket
// ---------------------------------------------------------------------------
__global__ void cell_kernel(const float* __restrict__ emb, int n, int D, const int* __restrict__ ev,
                            const double* __restrict__ basis, int64_t tmask,
                            unsigned long long* __restrict__ cell, int* __restrict__ bucket,
                            int* __restrict__ hist) {
  GRID_STRIDE(i, n) {
    double p[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < D; ++k) {
      const double e = (double)emb[i * D + k];
      p[0] += basis[k] * e;
      p[1] += basis[EP + k] * e;
      p[2] += basis[2 * EP + k] * e;
    }
    const double cs = basis[3 * EP];
    const unsigned long long key =
        cell_key(ev ? ev[i] : 0, clamp_cell(p[0] / cs), clamp_cell(p[1] / cs), clamp_cell(p[2] / cs));
    const int b = (int)(mix64(key) & (unsigned long long)tmask);
    cell[i] = key;
    bucket[i] = b;
    atomicAdd(&hist[b], 1);
  }
}

// sorted_emb rows hold es = 4 ceil(D / 4) floats (12 for D = 12): the query passes
// read every candidate's row, so rows carry no padding beyond the last float4
__global__ void scatter_kernel(const float* __restrict__ emb, int n, int D, int es,
                               const unsigned long long* __restrict__ cell, const int* __restrict__ bucket,
                               const int* __restrict__ start, int* __restrict__ fill, int* __restrict__ sorted_id,
                               float* __restrict__ sorted_emb, unsigned long long* __restrict__ sorted_cell) {
  GRID_STRIDE(i, n) {
    const int b = bucket[i];
    const int pos = start[b] + atomicAdd(&fill[b], 1);
    sorted_id[pos] = (int)i;
    sorted_cell[pos] = cell[i];
    for (int k = 0; k < es; ++k) sorted_emb[(size_t)pos * es + k] = (k < D) ? emb[i * D + k] : 0.f;
  }
}

// ---------------------------------------------------------------------------
// Per-query candidate enumeration (one wave per query)
// ---------------------------------------------------------------------------
struct QueryCtx {
  const int* start;
  const int* sorted_id;
  const float* sorted_emb;   // [n][es]: the D coordinates, zero-padded to a multiple of 4
  const unsigned long long* sorted_cell;
  int64_t tmask;
  float r2;
  int nk4;                   // float4 chunks per point (es = 4 nk4 <= EP)
};

struct WaveSlots {
  unsigned long long key[NSLOT];
  int bstart[NSLOT];
  int pre[NSLOT + 1];
};

// Visits every candidate j != i of the query's 27 cells with d^2 < r^2, calling
// f(j, d2, valid) once per lane per step (valid = false for idle lanes) so that
// callers may use wave-wide operations inside f.
template <class F>
__device__ __forceinline__ void for_neighbours(const QueryCtx& qc, WaveSlots& ws, int i,
                                               unsigned long long qcell, const float (&qe)[EP], F&& f) {
  const int l = lane_id();
  int size = 0;
  if (l < NSLOT) {
    const int dx = l % 3 - 1, dy = (l / 3) % 3 - 1, dz = l / 9 - 1;
    const int cx = (int)((qcell >> 32) & 0xFFFF) - 32768 + dx;
    const int cy = (int)((qcell >> 16) & 0xFFFF) - 32768 + dy;
    const int cz = (int)(qcell & 0xFFFF) - 32768 + dz;
    const int evq = (int)(qcell >> 48);
    const unsigned long long key = cell_key(evq, cx, cy, cz);
    const int b = (int)(mix64(key) & (unsigned long long)qc.tmask);
    ws.key[l] = key;
    ws.bstart[l] = qc.start[b];
    size = qc.start[b + 1] - qc.start[b];
  }
  const int incl = wave_incl_scan(size);
  if (l < NSLOT) ws.pre[l + 1] = incl;
  if (l == 0) ws.pre[0] = 0;
  const int total = __shfl(incl, 63, 64);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int base = 0; base < total; base += 64) {
    const int fidx = base + l;
    int j = -1;
    float d2 = 0.f;
    bool ok = false;
    if (fidx < total) {
      int lo = 0, hi = NSLOT;  // find slot s with pre[s] <= fidx < pre[s+1]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ws.pre[mid] <= fidx) lo = mid; else hi = mid;
      }
      // entry lies inside a bucket, so the cell key, the id and the embedding of the
      // candidate are all requested at once and tested afterwards
      const int entry = ws.bstart[lo] + (fidx - ws.pre[lo]);
      const unsigned long long ck = qc.sorted_cell[entry];
      const int jj = qc.sorted_id[entry];
      const float4* pe = (const float4*)(qc.sorted_emb + (size_t)entry * 4 * qc.nk4);
      float4 v[EP / 4];
#pragma unroll
      for (int k4 = 0; k4 < EP / 4; ++k4) v[k4] = k4 < qc.nk4 ? pe[k4] : make_float4(0.f, 0.f, 0.f, 0.f);
      if (ck == ws.key[lo]) {
        j = jj;
        if (j != i) {
#pragma unroll
          for (int k4 = 0; k4 < EP / 4; ++k4) {
            float t;
            t = qe[4 * k4 + 0] - v[k4].x; d2 = fmaf(t, t, d2);
            t = qe[4 * k4 + 1] - v[k4].y; d2 = fmaf(t, t, d2);
            t = qe[4 * k4 + 2] - v[k4].z; d2 = fmaf(t, t, d2);
            t = qe[4 * k4 + 3] - v[k4].w; d2 = fmaf(t, t, d2);
          }
          ok = d2 < qc.r2;
        }
      }
    }
    f(j, d2, ok);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned long long sel_key(float d2, int j) {
  return ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned int)j;
}

// XCD-aware query walk: each of the 8 XCDs takes a contiguous eighth of the
// cell-sorted queries so that neighbouring queries share one L2.
#define FOR_QUERIES(q, n)                                                              \
  const int xcd_ = blockIdx.x & 7, bx_ = blockIdx.x >> 3, nbx_ = gridDim.x >> 3;      \
  const int64_t qlo_ = (int64_t)(n) * xcd_ / 8, qhi_ = (int64_t)(n) * (xcd_ + 1) / 8; \
  for (int64_t q = qlo_ + (int64_t)bx_ * QW + (threadIdx.x >> 6); q < qhi_; q += (int64_t)nbx_ * QW)

__device__ __forceinline__ void load_query(const QueryCtx& qc, int64_t q, int& i, unsigned long long& qcell,
                                           float (&qe)[EP]) {
  i = qc.sorted_id[q];
  qcell = qc.sorted_cell[q];
  const float4* pe = (const float4*)(qc.sorted_emb + (size_t)q * 4 * qc.nk4);
#pragma unroll
  for (int k4 = 0; k4 < EP / 4; ++k4) {
    const float4 v = k4 < qc.nk4 ? pe[k4] : make_float4(0.f, 0.f, 0.f, 0.f);
    qe[4 * k4] = v.x; qe[4 * k4 + 1] = v.y; qe[4 * k4 + 2] = v.z; qe[4 * k4 + 3] = v.w;
  }
}

// k_max-th smallest of a wave's keys by radix select, 8 bits per pass from the top.
// visit(g) calls g(key) for every key (per lane, any number of times per lane);
// hist is the wave's 256-bin LDS histogram.
template <class V>
__device__ __forceinline__ unsigned long long radix_select(int (&hist)[256], int k_max, V&& visit) {
  const int l = lane_id();
  unsigned long long prefix = 0;
  int rank = k_max - 1;
  for (int p = 0; p < 8; ++p) {
    const int shift = 56 - 8 * p;
    const unsigned long long hmask = p == 0 ? 0ull : (~0ull << (shift + 8));
    for (int b = l; b < 256; b += 64) hist[b] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    visit([&](unsigned long long k) {
      if ((k & hmask) == prefix) atomicAdd(&hist[(k >> shift) & 255], 1);
    });
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // lane l holds bins 4l .. 4l+3
    const int h0 = hist[4 * l], h1 = hist[4 * l + 1], h2 = hist[4 * l + 2], h3 = hist[4 * l + 3];
    const int s4 = h0 + h1 + h2 + h3;
    const int incl = wave_incl_scan(s4);
    const int excl = incl - s4;
    int digit = -1, below = 0;
    if (rank >= excl && rank < incl) {
      int cum = excl;
      if (rank < cum + h0) { digit = 4 * l; below = cum; }
      else if (rank < cum + h0 + h1) { digit = 4 * l + 1; below = cum + h0; }
      else if (rank < cum + h0 + h1 + h2) { digit = 4 * l + 2; below = cum + h0 + h1; }
      else { digit = 4 * l + 3; below = cum + h0 + h1 + h2; }
    }
    const unsigned long long m = ballot(digit >= 0);
    const int src_lane = __ffsll((long long)m) - 1;
    digit = __shfl(digit, src_lane, 64);
    below = __shfl(below, src_lane, 64);
    prefix |= (unsigned long long)digit << shift;
    rank -= below;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  return prefix;
}

// The within-r keys of a point are compacted into LDS during its counting pass
// (up to SEL_CAP of them), so that a saturated point's select reads LDS; a point
// with more neighbours than that enumerates its cells again in every select pass.
constexpr int SEL_CAP = 512;

// pass 1: within-r count and, for saturated points, the k_max-th selection key
__global__ __launch_bounds__(QW * 64) void query_count_kernel(QueryCtx qc, int n, int k_max, int* __restrict__ cnt,
                                                              unsigned long long* __restrict__ thr,
                                                              int* __restrict__ counters) {
  __shared__ WaveSlots slots[QW];
  __shared__ int hist[QW][256];
  __shared__ unsigned long long selk[QW][SEL_CAP];
  const int w = threadIdx.x >> 6, l = lane_id();
  FOR_QUERIES(q, n) {
    int i;
    unsigned long long qcell;
    float qe[EP];
    load_query(qc, q, i, qcell, qe);
    int c = 0;   // wave-uniform running count
    for_neighbours(qc, slots[w], i, qcell, qe, [&](int j, float d2, bool ok) {
      const unsigned long long m = ballot(ok);
      const int pos = c + mask_rank(m);
      if (ok && pos < SEL_CAP) selk[w][pos] = sel_key(d2, j);
      c += __popcll(m);
    });
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    unsigned long long t = ~0ull;
    if (c > k_max && c <= SEL_CAP) {
      t = radix_select(hist[w], k_max, [&](auto&& g) {
        for (int b = l; b < c; b += 64) g(selk[w][b]);
      });
    } else if (c > k_max) {
      t = radix_select(hist[w], k_max, [&](auto&& g) {
        for_neighbours(qc, slots[w], i, qcell, qe, [&](int j, float d2, bool ok) {
          if (ok) g(sel_key(d2, j));
        });
      });
    }
    if (l == 0) {
      cnt[i] = c;
      thr[i] = t;
      if (c > k_max) atomicAdd(&counters[1], 1);
    }
  }
}

// pass 2: per-row pair counts
__global__ __launch_bounds__(QW * 64) void query_rowcount_kernel(QueryCtx qc, int n,
                                                                 const unsigned long long* __restrict__ thr,
                                                                 int* __restrict__ rowcnt) {
  __shared__ WaveSlots slots[QW];
  const int w = threadIdx.x >> 6, l = lane_id();
  FOR_QUERIES(q, n) {
    int i;
    unsigned long long qcell;
    float qe[EP];
    load_query(qc, q, i, qcell, qe);
    const unsigned long long ti = thr[i];
    int own = 0;
    for_neighbours(qc, slots[w], i, qcell, qe, [&](int j, float d2, bool ok) {
      if (ok && sel_key(d2, j) <= ti) {
        if (j > i) ++own;
        else if (sel_key(d2, i) > thr[j]) atomicAdd(&rowcnt[j], 1);
      }
    });
    own = wave_sum(own);
    if (l == 0 && own) atomicAdd(&rowcnt[i], own);
  }
}

// pass 3: write the pairs into their rows (unordered within a row)
__global__ __launch_bounds__(QW * 64) void query_fill_kernel(QueryCtx qc, int n,
                                                             const unsigned long long* __restrict__ thr,
                                                             const int* __restrict__ rowptr, int* __restrict__ cursor,
                                                             int* __restrict__ out, int64_t cap) {
  __shared__ WaveSlots slots[QW];
  const int w = threadIdx.x >> 6, l = lane_id();
  FOR_QUERIES(q, n) {
    int i;
    unsigned long long qcell;
    float qe[EP];
    load_query(qc, q, i, qcell, qe);
    const unsigned long long ti = thr[i];
    const int64_t ri = rowptr[i];
    for_neighbours(qc, slots[w], i, qcell, qe, [&](int j, float d2, bool ok) {
      const bool sel = ok && sel_key(d2, j) <= ti;
      const bool mine = sel && j > i;
      const unsigned long long m = ballot(mine);
      int base = 0;
      if (m) {
        if (l == 0) base = atomicAdd(&cursor[i], __popcll(m));
        base = __shfl(base, 0, 64);
      }
      if (mine) {
        const int64_t pos = ri + base + mask_rank(m);
        if (pos < cap) out[pos] = j;
      }
      if (sel && j < i && sel_key(d2, i) > thr[j]) {
        const int64_t pos = (int64_t)rowptr[j] + atomicAdd(&cursor[j], 1);
        if (pos < cap) out[pos] = i;
      }
    });
  }
}

// rows: dst ascending per row, src = row id; rows extending past cap are skipped
__global__ __launch_bounds__(256) void row_sort_kernel(const int* __restrict__ rowptr, const int* __restrict__ in,
                                                       int* __restrict__ src, int* __restrict__ dst, int n,
                                                       int64_t cap) {
  __shared__ int keys[4][512];
  const int w = threadIdx.x >> 6, l = lane_id();
  for (int row = blockIdx.x * 4 + w; row < n; row += gridDim.x * 4) {
    const int b = rowptr[row], e = rowptr[row + 1], L = e - b;
    if (L <= 0 || e > cap) continue;
    if (L <= 512) {
      for (int k = l; k < L; k += 64) keys[w][k] = in[b + k];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int k = l; k < L; k += 64) {
        const int key = keys[w][k];
        int rank = 0;
        for (int t = 0; t < L; ++t) rank += keys[w][t] < key ? 1 : 0;
        dst[b + rank] = key;
        src[b + rank] = row;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      for (int k = l; k < L; k += 64) {
        const int key = in[b + k];
        int rank = 0;
        for (int t = 0; t < L; ++t) rank += in[b + t] < key ? 1 : 0;
        dst[b + rank] = key;
        src[b + rank] = row;
      }
    }
  }
}

}  // namespace

void launch_build_graph(const float* emb, int n, int D, float radius, int k_max, const int* ev, GraphScratch& g,
                        int* src, int* dst, int64_t cap, int n_cu, hipStream_t s) {
  launch_fill_int(g.counters, 0, 8, s);
  if (n <= 0) return;
  const int sblocks = g.stats_blocks;
  stats_kernel<<<sblocks, STAT_T, 0, s>>>(emb, n, D, g.stats);
  basis_kernel<<<1, 256, 0, s>>>(g.stats, sblocks, n, D, radius, g.basis);
  launch_fill_int(g.hist, 0, g.table, s);
  launch_fill_int(g.fill, 0, g.table, s);
  const int eb = blocks_for(n, 256);
  cell_kernel<<<eb, 256, 0, s>>>(emb, n, D, ev, g.basis, g.table - 1, g.cell, g.bucket, g.hist);
  launch_scan_excl(g.hist, g.start, g.table, nullptr, nullptr, g.tmp, s);
  const int nk4 = (D + 3) / 4;
  scatter_kernel<<<eb, 256, 0, s>>>(emb, n, D, 4 * nk4, g.cell, g.bucket, g.start, g.fill, g.sorted_id, g.sorted_emb,
                                    g.sorted_cell);
  QueryCtx qc{g.start, g.sorted_id, g.sorted_emb, g.sorted_cell, g.table - 1, radius * radius, nk4};
  int qgrid = (int)((n + QW - 1) / QW);
  if (qgrid > n_cu * 16) qgrid = n_cu * 16;
  qgrid = ((qgrid + 7) / 8) * 8;
  query_count_kernel<<<qgrid, QW * 64, 0, s>>>(qc, n, k_max, g.cnt, g.thr, g.counters);
  launch_fill_int(g.rowcnt, 0, n + 1, s);
  query_rowcount_kernel<<<qgrid, QW * 64, 0, s>>>(qc, n, g.thr, g.rowcnt);
  launch_scan_excl(g.rowcnt, g.rowptr, n, nullptr, &g.counters[0], g.tmp, s);
  launch_fill_int(g.cursor, 0, n, s);
  query_fill_kernel<<<qgrid, QW * 64, 0, s>>>(qc, n, g.thr, g.rowptr, g.cursor, g.unsorted, cap);
  row_sort_kernel<<<blocks_for(n, 4, 8192), 256, 0, s>>>(g.rowptr, g.unsorted, src, dst, n, cap);
}
