// Training path of the filter MLP and the interaction network (FP32): forward
// passes that keep what the backward needs, hand-written backward passes, the
// binary cross-entropy objective and an Adam update.
//
// Objective (the reading taken for the training configuration): mean binary
// cross-entropy with logits on the generator truth over the candidate edges
// (filter) plus the same over the filtered edges (interaction network); edge
// sets are held fixed.  The interaction-network backward keeps only the
// per-iteration node and edge states (h^t, e^t) from the forward pass and
// recomputes each iteration's internals from (h^{t-1}, e^{t-1}) when it gets
// there, so activation memory is (T+1) state copies instead of every layer of
// every iteration.
//
// Precision: an FP32 context trains with FP32 products; a BF16 context (the
// training configuration with BF16 activations) rounds the operands of every
// product - activations, deltas and the weight copies - to BF16 on the way into
// the matrix cores (v_mfma_f32_16x16x32_bf16) and accumulates in FP32, and keeps
// the activations that the forward pass stores for the backward (the filter's
// hidden layers, the encoders' hidden layers, the per-iteration states h^t and e^t,
// the output head's hidden layer, the embedding's hidden layers) in BF16, which
// halves that memory; the forward pass continues from the stored BF16 values, so
// forward and backward see the same numbers.  The master parameters, the Adam
// moments, the deltas and the element-wise arithmetic stay FP32.
//
// Building blocks, all on MFMA (v_mfma_f32_16x16x4_f32 or the BF16 form) or plain
// vector code:
//   rowgemm : out[r][:] = epi(X[r][:] W) for a row-major X (epilogues: store,
//             accumulate, +bias, tanh(+bias), times (1 - aux^2));
//   wgrad   : G[K(+1)][N] += X^T D over all rows, split over row chunks, partial
//             sums reduced in a fixed order (deterministic), the optional extra
//             row K being the bias gradient (column sums of D);
//   segsum  : per-node sums of edge rows over the CSR/CSC incidence lists (the
//             backward of a gather is again a fixed-order gather);
// the transposed weights needed by backward products are kept as their own
// fragment blocks, rebuilt with the forward ones whenever parameters change.
#include <vector>

#include "common.h"
#include "ctx.h"
#include "mfma_tile.h"

namespace {

enum { EPI_STORE = 0, EPI_ACC = 1, EPI_BIAS = 2, EPI_BIAS_TANH = 3, EPI_DTANH = 4, EPI_PAIR_TANH = 5,
       EPI_RES_TANH = 6 };   // EPI_RES_TANH: out = aux + tanh(acc + b), a residual update

// EPI_PAIR_TANH: out[r] = tanh(acc[r] + P[src[r]][0:N] + P[dst[r]][N:2N] + b), the first layer
// of an edge network on [h_s, h_t, e] with its per-node projections P = [h W_a | h W_b]
struct PairIn {
  const float* P = nullptr;
  const int* src = nullptr;
  const int* dst = nullptr;
  int n = 0;
};

}  // namespace

// A buffer of activations kept by a forward pass for its backward: FP32, or BF16
// in a BF16 context.  Transient FP32 buffers convert to it implicitly.
struct ActBuf {
  void* p = nullptr;
  int bf16 = 0;
  ActBuf() = default;
  ActBuf(std::nullptr_t) {}
  ActBuf(float* q) : p(q) {}
  ActBuf(const float* q) : p((void*)q) {}
  ActBuf(void* q, int b) : p(q), bf16(b) {}
  __device__ __forceinline__ float get(size_t i) const {
    return bf16 ? (float)((const __bf16*)p)[i] : ((const float*)p)[i];
  }
  __device__ __forceinline__ void set(size_t i, float v) const {
    if (bf16) ((__bf16*)p)[i] = (__bf16)v;
    else ((float*)p)[i] = v;
  }
  // four consecutive elements from a multiple of four (16 or 8 bytes)
  __device__ __forceinline__ float4 get4(size_t i) const {
    if (bf16) {
      const bf16x4 v = *(const bf16x4*)((const __bf16*)p + i);
      return make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    }
    return *(const float4*)((const float*)p + i);
  }
  __device__ __forceinline__ void set4(size_t i, float4 v) const {
    if (bf16) {
      bf16x4 b;
      b[0] = (__bf16)v.x; b[1] = (__bf16)v.y; b[2] = (__bf16)v.z; b[3] = (__bf16)v.w;
      *(bf16x4*)((__bf16*)p + i) = b;
    } else {
      *(float4*)((float*)p + i) = v;
    }
  }
  // the buffer from element `off` on
  ActBuf at(size_t off) const { return ActBuf((char*)p + off * (bf16 ? 2 : 4), bf16); }
};

namespace {

// node index clamped into [0, n): an out-of-range edge end reads node 0 instead of
// memory past the node arrays (the inference entry points report such edges)
__device__ __forceinline__ size_t node_of(int i, int n) { return (unsigned)i < (unsigned)n ? (size_t)i : 0; }

// ---------------------------------------------------------------------------
// fragment blocks from a view of parameter memory
// ---------------------------------------------------------------------------
struct MatView {
  const float* p = nullptr;  // base
  int r0 = 0;                // first row of the block in the stored matrix
  int ld = 0;                // row stride of the stored matrix
  int trans = 0;             // element (k, n) = trans ? p[(r0 + n) ld + k] : p[(r0 + k) ld + n]
  __device__ float at(int k, int n) const {
    return trans ? p[(size_t)(r0 + n) * ld + k] : p[(size_t)(r0 + k) * ld + n];
  }
};

// M[k][n] for k < K, n < N, built from A and B: mode 0 = A only, 1 = [A | B] side by side
// (B from column N1), 2 = [A ; B] stacked (B from row K1), 3 = A for the input
// [(u_s + u_t) / 2, u_s - u_t] of two halves of width `split` (rows [A_s + A_t;
// (A_s - A_t) / 2], the form the BF16 inference layers that read an edge's two ends use).
__global__ void frag_fill_kernel(uint4* out, int nkb, int nnt, int K, int N, MatView A, MatView B, int mode, int split,
                                 int bf16) {
  const int64_t nblk = (int64_t)nkb * nnt * 64;
  GRID_STRIDE(t, nblk) {
    const int lane = (int)(t % 64);
    const int64_t blk = t / 64;
    const int kb = (int)(blk % nkb), nt = (int)(blk / nkb);
    const int g = lane >> 4, n = nt * 16 + (lane & 15);
    auto val = [&](int k) -> float {
      if (k >= K || n >= N) return 0.f;
      if (mode == 1 && n >= split) return B.at(k, n - split);
      if (mode == 2 && k >= split) return B.at(k - split, n);
      if (mode == 3) return k < split ? A.at(k, n) + A.at(k + split, n) : 0.5f * (A.at(k - split, n) - A.at(k, n));
      return A.at(k, n);
    };
    uint4 o;
    if (!bf16) {
      float v[4];
      for (int s = 0; s < 4; ++s) v[s] = val(kb * 16 + 4 * g + s);
      o = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]), __float_as_uint(v[3]));
    } else {
      bf16x8 v;
      for (int j = 0; j < 8; ++j) v[j] = (__bf16)val(kb * 32 + 8 * g + j);
      o = __builtin_bit_cast(uint4, v);
    }
    out[t] = o;
  }
}

// bias (zero-padded to nout) and, when out_s is given, the same times 2 log2(e)
// (the inference epilogues' pre-scaled copy)
__global__ void bias_fill_kernel(float* out, float* out_s, int nout, const float* b, int N) {
  GRID_STRIDE(i, nout) {
    const float v = i < N ? b[i] : 0.f;
    out[i] = v;
    if (out_s) out_s[i] = v * TRK_2LOG2E;
  }
}

// ---------------------------------------------------------------------------
// rowgemm: out = epi(X W), X [m][K] row-major (ldx), W fragment blocks (FP32)
// ---------------------------------------------------------------------------

template <class P, int NW, int NTW, int RG_MT, int RG_KMAX>
__global__ __launch_bounds__(NW * 64) void rowgemm_kernel(ActBuf X, int ldx, int K, int64_t m, DevLayer W,
                                                             ActBuf out, int ldo, int N, int epi, ActBuf aux,
                                                             int ldaux, PairIn pr) {
  typedef typename P::act_t T;
  constexpr int LDX = RG_KMAX + P::PAD;
  constexpr int MTW = RG_MT / 16;
  constexpr int NT = NW * 64;
  __shared__ __align__(16) T xs[RG_MT * LDX];
  const int wave = threadIdx.x >> 6, l = lane_id(), g = l >> 4, r = l & 15;
  const int kpad = W.nkb * P::KB;
  const int64_t ntiles = (m + RG_MT - 1) / RG_MT;
  // four-element groups: X rows and widths that are multiples of four move as 16-byte
  // (FP32) or 8-byte (BF16) loads, eight per thread in flight; outputs likewise
  const bool vin = (K % 4 == 0) && (ldx % 4 == 0);
  const bool vout =
      (N % 4 == 0) && (ldo % 4 == 0) && ((epi != EPI_DTANH && epi != EPI_RES_TANH) || ldaux % 4 == 0);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * RG_MT;
    if (vin) {
      const int kq = kpad / 4;
      for (int base = threadIdx.x; base < RG_MT * kq; base += 8 * NT) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int idx = base + u * NT;
          const int mm = idx / kq, k = (idx - mm * kq) * 4;
          v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (idx < RG_MT * kq && row0 + mm < m && k < K) v[u] = X.get4((size_t)(row0 + mm) * ldx + k);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int idx = base + u * NT;
          const int mm = idx / kq, k = (idx - mm * kq) * 4;
          if (idx < RG_MT * kq) P::store4(xs + mm * LDX + k, v[u].x, v[u].y, v[u].z, v[u].w);
        }
      }
    } else {
      for (int idx = threadIdx.x; idx < RG_MT * kpad; idx += blockDim.x) {
        const int mm = idx / kpad, k = idx - mm * kpad;
        xs[mm * LDX + k] = P::cvt((row0 + mm < m && k < K) ? X.get((size_t)(row0 + mm) * ldx + k) : 0.f);
      }
    }
    __syncthreads();
    for (int nt0 = wave * NTW; nt0 < W.nnt; nt0 += NW * NTW) {
      f32x4 acc[MTW][NTW];
      tile_gemm<P, MTW, NTW, true>(acc, xs, LDX, W.w, W.nkb, nt0, 0, W.nkb);
#pragma unroll
      for (int j = 0; j < NTW; ++j) {
        const int n0 = (nt0 + j) * 16 + 4 * g;
        if (vout) {
          if (n0 >= N) continue;
          float4 b = make_float4(0.f, 0.f, 0.f, 0.f);
          if (epi == EPI_BIAS || epi == EPI_BIAS_TANH || epi == EPI_PAIR_TANH || epi == EPI_RES_TANH)
            b = *(const float4*)(W.b + n0);
#pragma unroll
          for (int i = 0; i < MTW; ++i) {
            const int64_t row = row0 + i * 16 + r;
            if (row >= m) continue;
            const size_t o = (size_t)row * ldo + n0;
            float4 v = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
            if (epi == EPI_ACC) {
              const float4 a = out.get4(o);
              v = make_float4(v.x + a.x, v.y + a.y, v.z + a.z, v.w + a.w);
            } else if (epi == EPI_BIAS) {
              v = make_float4(v.x + b.x, v.y + b.y, v.z + b.z, v.w + b.w);
            } else if (epi == EPI_BIAS_TANH) {
              v = make_float4(trk_tanh(v.x + b.x), trk_tanh(v.y + b.y), trk_tanh(v.z + b.z), trk_tanh(v.w + b.w));
            } else if (epi == EPI_DTANH) {
              const float4 a = aux.get4((size_t)row * ldaux + n0);
              v = make_float4(v.x * (1.f - a.x * a.x), v.y * (1.f - a.y * a.y), v.z * (1.f - a.z * a.z),
                              v.w * (1.f - a.w * a.w));
            } else if (epi == EPI_RES_TANH) {
              const float4 a = aux.get4((size_t)row * ldaux + n0);
              v = make_float4(a.x + trk_tanh(v.x + b.x), a.y + trk_tanh(v.y + b.y), a.z + trk_tanh(v.z + b.z),
                              a.w + trk_tanh(v.w + b.w));
            } else if (epi == EPI_PAIR_TANH) {
              const float4 ps = *(const float4*)(pr.P + node_of(pr.src[row], pr.n) * 2 * N + n0);
              const float4 pd = *(const float4*)(pr.P + node_of(pr.dst[row], pr.n) * 2 * N + N + n0);
              v = make_float4(trk_tanh(v.x + ps.x + pd.x + b.x), trk_tanh(v.y + ps.y + pd.y + b.y),
                              trk_tanh(v.z + ps.z + pd.z + b.z), trk_tanh(v.w + ps.w + pd.w + b.w));
            }
            out.set4(o, v);
          }
          continue;
        }
#pragma unroll
        for (int i = 0; i < MTW; ++i) {
          const int64_t row = row0 + i * 16 + r;
          if (row >= m) continue;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int n = n0 + c;
            if (n >= N) continue;
            float v = acc[i][j][c];
            const size_t o = (size_t)row * ldo + n;
            if (epi == EPI_ACC) v += out.get(o);
            else if (epi == EPI_BIAS) v += W.b[n];
            else if (epi == EPI_BIAS_TANH) v = trk_tanh(v + W.b[n]);
            else if (epi == EPI_DTANH) {
              const float a = aux.get((size_t)row * ldaux + n);
              v *= 1.f - a * a;
            } else if (epi == EPI_RES_TANH) {
              v = aux.get((size_t)row * ldaux + n) + trk_tanh(v + W.b[n]);
            } else if (epi == EPI_PAIR_TANH) {
              const float ps = pr.P[node_of(pr.src[row], pr.n) * 2 * N + n];
              const float pd = pr.P[node_of(pr.dst[row], pr.n) * 2 * N + N + n];
              v = trk_tanh(v + ps + pd + W.b[n]);
            }
            out.set(o, v);
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// wgrad: partial[chunk][k][n] = sum over the chunk's rows of X[r][k] D[r][n]; row K of
// the output is the column sum of D when with_bias.  X is dense (ldx) or, with
// gsrc, the pair [S[gsrc[r]], S[gdst[r]]] of width 2*gd.  Each workgroup stages
// WG_R rows of its X and D column blocks in LDS per step; the rows are split into
// enough chunks that several workgroups share each compute unit and hide one
// another's load latency.
// ---------------------------------------------------------------------------
constexpr int WG_T = 64;   // tile edge (k and n)
constexpr int WG_R = 64;   // rows staged per step

struct WgradIn {
  ActBuf X;
  int ldx;
  const int* gsrc;
  const int* gdst;
  const float* S;
  int gd, gn, K, with_bias;
  const float* D;
  int ldd, N;
};

// element (row, k) of X and (row, n) of D (zero past rend or the widths)
__device__ __forceinline__ void wgrad_value(const WgradIn& a, int64_t row, int64_t rend, int k, int n, float& xv,
                                            float& dv) {
  xv = dv = 0.f;
  if (row >= rend) return;
  if (k < a.K) {
    if (a.gsrc)
      xv = k < a.gd ? a.S[node_of(a.gsrc[row], a.gn) * a.gd + k] : a.S[node_of(a.gdst[row], a.gn) * a.gd + (k - a.gd)];
    else
      xv = a.X.get((size_t)row * a.ldx + k);
  } else if (k == a.K && a.with_bias) {
    xv = 1.f;
  }
  if (n < a.N) dv = a.D[(size_t)row * a.ldd + n];
}

// four consecutive columns from a multiple of four: X[row][k..k+3] (or the bias
// column), D[row][n..n+3]; used when every width and stride is a multiple of four
__device__ __forceinline__ float4 wgrad_x4(const WgradIn& a, int64_t row, int64_t rend, int k) {
  float4 xv = make_float4(0.f, 0.f, 0.f, 0.f);
  if (row >= rend) return xv;
  if (k < a.K) {
    if (a.gsrc)
      xv = k < a.gd ? *(const float4*)(a.S + node_of(a.gsrc[row], a.gn) * a.gd + k)
                    : *(const float4*)(a.S + node_of(a.gdst[row], a.gn) * a.gd + (k - a.gd));
    else
      xv = a.X.get4((size_t)row * a.ldx + k);
  } else if (k == a.K && a.with_bias) {
    xv.x = 1.f;
  }
  return xv;
}
__device__ __forceinline__ float4 wgrad_d4(const WgradIn& a, int64_t row, int64_t rend, int n) {
  if (row >= rend || n >= a.N) return make_float4(0.f, 0.f, 0.f, 0.f);
  return *(const float4*)(a.D + (size_t)row * a.ldd + n);
}
__device__ __forceinline__ void wgrad_value4(const WgradIn& a, int64_t row, int64_t rend, int k, int n, float4& xv,
                                             float4& dv) {
  xv = wgrad_x4(a, row, rend, k);
  dv = wgrad_d4(a, row, rend, n);
}

// whether the bias row (row K of the output) is summed apart: when K fills whole k
// tiles, a tile for that one row would cost as much as a full one
__host__ __device__ inline bool wgrad_fold(const WgradIn& a) { return a.with_bias && a.K % WG_T == 0; }

// whether wgrad_value4 applies
__host__ __device__ inline bool wgrad_vec(const WgradIn& a) {
  return a.K % 4 == 0 && a.N % 4 == 0 && a.ldd % 4 == 0 && (a.gsrc ? a.gd % 4 == 0 : a.ldx % 4 == 0);
}

// Tiles and row chunks over a one-dimensional grid.  Consecutive workgroups go to
// the eight XCDs in turn; the ids are dealt so that every tile of one row chunk
// lands on the same XCD, close together in time, where the tiles share the chunk's
// rows through that XCD's L2 (timed level with the plain order on these shapes).
// Padding ids past the last chunk leave at once.
struct WgradTile {
  int kt, nt, chunk;
};
__device__ __forceinline__ bool wgrad_tile(int ktiles, int ntiles, int chunks, WgradTile& t) {
  const int b = blockIdx.x, xcd = b & 7, slot = b >> 3;
  const int tiles = ktiles * ntiles;
  const int cw = slot / tiles, tl = slot - cw * tiles;
  t.chunk = cw * 8 + xcd;
  t.nt = tl / ktiles;
  t.kt = tl - t.nt * ktiles;
  return t.chunk < chunks;
}
inline int64_t wgrad_grid(int64_t tiles, int chunks) { return (int64_t)8 * ((chunks + 7) / 8) * tiles; }

__global__ __launch_bounds__(256) void wgrad_kernel(WgradIn a, int64_t m, int64_t rows_per_chunk,
                                                    float* __restrict__ partial, int ktiles, int ntiles,
                                                    int chunks) {
  WgradTile tile;
  if (!wgrad_tile(ktiles, ntiles, chunks, tile)) return;
  __shared__ float xs[WG_R][WG_T + 1];
  __shared__ float ds[WG_R][WG_T + 1];
  const int wave = threadIdx.x >> 6, l = lane_id(), g = l >> 4, r = l & 15;
  const int k0 = tile.kt * WG_T, n0 = tile.nt * WG_T;
  const int Kb = a.K + (a.with_bias ? 1 : 0);
  const int64_t rbeg = (int64_t)tile.chunk * rows_per_chunk;
  const int64_t rend = min(m, rbeg + rows_per_chunk);
  f32x4 acc[4];
  for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool vec = wgrad_vec(a);
  // a bias row that would start a k tile of its own is summed by the first k tile
  const bool fold = wgrad_fold(a) && tile.kt == 0;
  float bsum = 0.f;
  // vector path: four 16-byte groups of X and of D per thread, held in registers; the
  // next step's are requested once the barrier after the LDS writes has passed
  float4 xv[WG_R * WG_T / 1024], dv[WG_R * WG_T / 1024];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < WG_R * WG_T / 1024; ++u) {
      const int idx = threadIdx.x + u * 256;
      const int rr = idx / (WG_T / 4), c = (idx - rr * (WG_T / 4)) * 4;
      wgrad_value4(a, r0 + rr, rend, k0 + c, n0 + c, xv[u], dv[u]);
    }
  };
  if (vec && rbeg < rend) fetch(rbeg);
  for (int64_t rs = rbeg; rs < rend; rs += WG_R) {
    if (vec) {
#pragma unroll
      for (int u = 0; u < WG_R * WG_T / 1024; ++u) {
        const int idx = threadIdx.x + u * 256;
        const int rr = idx / (WG_T / 4), c = (idx - rr * (WG_T / 4)) * 4;
        xs[rr][c] = xv[u].x; xs[rr][c + 1] = xv[u].y; xs[rr][c + 2] = xv[u].z; xs[rr][c + 3] = xv[u].w;
        ds[rr][c] = dv[u].x; ds[rr][c + 1] = dv[u].y; ds[rr][c + 2] = dv[u].z; ds[rr][c + 3] = dv[u].w;
      }
    } else {
      for (int idx = threadIdx.x; idx < WG_R * WG_T; idx += blockDim.x) {
        const int rr = idx / WG_T, c = idx - rr * WG_T;
        float xv1, dv1;
        wgrad_value(a, rs + rr, rend, k0 + c, n0 + c, xv1, dv1);
        xs[rr][c] = xv1;
        ds[rr][c] = dv1;
      }
    }
    __syncthreads();
    if (vec && rs + WG_R < rend) fetch(rs + WG_R);
    if (fold && threadIdx.x < WG_T)
      for (int rr = 0; rr < WG_R; ++rr) bsum += ds[rr][threadIdx.x];
#pragma unroll 4
    for (int rr = 0; rr < WG_R; rr += 4) {
      // operands: k-row fragment from X^T (row = wave*16 + r), n fragments from D
      const float xa = xs[rr + g][wave * 16 + r];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float da = ds[rr + g][j * 16 + r];
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(da, xa, acc[j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // lane holds rows k = k0 + wave*16 + r, columns n = n0 + j*16 + 4g + c
  if (fold && threadIdx.x < WG_T && n0 + (int)threadIdx.x < a.N)
    partial[((size_t)tile.chunk * Kb + a.K) * a.N + n0 + threadIdx.x] = bsum;
  const int k = k0 + wave * 16 + r;
  if (k < (wgrad_fold(a) ? a.K : Kb)) {
    float* P = partial + ((size_t)tile.chunk * Kb + k) * a.N;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int n = n0 + j * 16 + 4 * g + c;
        if (n < a.N) P[n] = acc[j][c];
      }
  }
}

// The same partial products with BF16 operands: the staged rows are held
// transposed (column-major, rows contiguous), so that a lane's eight consecutive
// rows of one column are one 16-byte read; 32 rows per product.  Each thread of
// the first two waves stages eight consecutive rows of four X columns, each thread
// of the last two the same of D, and writes them as four 16-byte column runs; it
// requests the next step's rows right after those writes.
constexpr int WGB_LD = WG_R + 8;   // row stride of the transposed tiles (bf16 elements)

__global__ __launch_bounds__(256) void wgrad_bf16_kernel(WgradIn a, int64_t m, int64_t rows_per_chunk,
                                                         float* __restrict__ partial, int ktiles, int ntiles,
                                                         int chunks) {
  WgradTile tile;
  if (!wgrad_tile(ktiles, ntiles, chunks, tile)) return;
  __shared__ __align__(16) __bf16 xt[WG_T][WGB_LD];
  __shared__ __align__(16) __bf16 dt[WG_T][WGB_LD];
  const int wave = threadIdx.x >> 6, l = lane_id(), g = l >> 4, r = l & 15;
  const int k0 = tile.kt * WG_T, n0 = tile.nt * WG_T;
  const int Kb = a.K + (a.with_bias ? 1 : 0);
  const int64_t rbeg = (int64_t)tile.chunk * rows_per_chunk;
  const int64_t rend = min(m, rbeg + rows_per_chunk);
  f32x4 acc[4];
  for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool vec = wgrad_vec(a);
  // a bias row that would start a k tile of its own is summed by the first k tile
  const bool fold = wgrad_fold(a) && tile.kt == 0;
  float bsum = 0.f;
  static_assert(WG_R == 64 && WG_T == 64, "128 threads x 8 rows x 4 columns per operand");
  const bool isx = threadIdx.x < 128;                  // wave-uniform
  const int st_t = threadIdx.x & 127, cg = st_t & 15, rg = st_t >> 4;
  // the vector path holds a step's rows in registers: the next step's are requested
  // before the current step's products, so their latency is hidden behind them
  float4 v[8];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      v[j] = isx ? wgrad_x4(a, r0 + 8 * rg + j, rend, k0 + 4 * cg) : wgrad_d4(a, r0 + 8 * rg + j, rend, n0 + 4 * cg);
  };
  if (vec && rbeg < rend) fetch(rbeg);
  for (int64_t rs = rbeg; rs < rend; rs += WG_R) {
    if (vec) {
      __bf16 (*tile)[WGB_LD] = isx ? xt : dt;
      bf16x8 w0, w1, w2, w3;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        w0[j] = (__bf16)v[j].x; w1[j] = (__bf16)v[j].y;
        w2[j] = (__bf16)v[j].z; w3[j] = (__bf16)v[j].w;
      }
      *(bf16x8*)&tile[4 * cg][8 * rg] = w0;
      *(bf16x8*)&tile[4 * cg + 1][8 * rg] = w1;
      *(bf16x8*)&tile[4 * cg + 2][8 * rg] = w2;
      *(bf16x8*)&tile[4 * cg + 3][8 * rg] = w3;
      if (rs + WG_R < rend) fetch(rs + WG_R);
    } else {
      for (int idx = threadIdx.x; idx < WG_R * WG_T; idx += blockDim.x) {
        const int rr = idx / WG_T, c = idx - rr * WG_T;
        float xv, dv;
        wgrad_value(a, rs + rr, rend, k0 + c, n0 + c, xv, dv);
        xt[c][rr] = (__bf16)xv;
        dt[c][rr] = (__bf16)dv;
      }
    }
    __syncthreads();
    if (fold && threadIdx.x < WG_T)
      for (int rr = 0; rr < WG_R; ++rr) bsum += (float)dt[threadIdx.x][rr];
#pragma unroll
    for (int rr = 0; rr < WG_R; rr += 32) {
      // A: D^T rows (n = j*16 + r), B: X^T columns (k = wave*16 + r); lane group g
      // carries rows rr + 8g .. rr + 8g + 7
      const bf16x8 xb = *(const bf16x8*)&xt[wave * 16 + r][rr + 8 * g];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bf16x8 da = *(const bf16x8*)&dt[j * 16 + r][rr + 8 * g];
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(da, xb, acc[j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (fold && threadIdx.x < WG_T && n0 + (int)threadIdx.x < a.N)
    partial[((size_t)tile.chunk * Kb + a.K) * a.N + n0 + threadIdx.x] = bsum;
  const int k = k0 + wave * 16 + r;
  if (k < (wgrad_fold(a) ? a.K : Kb)) {
    float* P = partial + ((size_t)tile.chunk * Kb + k) * a.N;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int n = n0 + j * 16 + 4 * g + c;
        if (n < a.N) P[n] = acc[j][c];
      }
  }
}

// Wide FP32 layers (K and N multiples of 128): a 128 x 128 output tile per workgroup,
// so that each staged row of X and D feeds twice the products of the 64 x 64 tile.
// Wave w owns k rows [32w, 32w + 32) (two 16-row blocks) and all 128 n columns (eight
// blocks): per four staged rows it reads two X and eight D values for sixteen products.
// Sixteen rows are staged per step, each thread staging whole 16-byte groups of four
// columns.  A bias row (with_bias; K is a multiple of
// the tile) is summed by the k tile 0 workgroups.
constexpr int WT = 128;

__global__ __launch_bounds__(256) void wgrad128_kernel(WgradIn a, int64_t m, int64_t rows_per_chunk,
                                                       float* __restrict__ partial, int ktiles, int ntiles,
                                                       int chunks) {
  WgradTile tile;
  if (!wgrad_tile(ktiles, ntiles, chunks, tile)) return;
  constexpr int R = 16;                        // rows staged per step
  constexpr int GPT = R * (WT / 4) / 256;      // 16-byte groups per thread and operand
  constexpr int LDF = WT + 4;                  // row stride
  __shared__ __align__(16) float xs[R][LDF];
  __shared__ __align__(16) float ds[R][LDF];
  const int wave = threadIdx.x >> 6, l = lane_id(), g = l >> 4, r = l & 15;
  const int k0 = tile.kt * WT, n0 = tile.nt * WT;
  const int Kb = a.K + (a.with_bias ? 1 : 0);
  const int64_t rbeg = (int64_t)tile.chunk * rows_per_chunk;
  const int64_t rend = min(m, rbeg + rows_per_chunk);
  const bool fold = a.with_bias && tile.kt == 0;
  float bsum = 0.f;
  f32x4 acc[2][8];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // this thread's groups: column group cg (four columns), rows rg + 8 u
  const int cg = threadIdx.x % (WT / 4), rg = threadIdx.x / (WT / 4);
  // the next step's groups are requested once the barrier after the LDS writes has passed
  float4 xv[GPT], dv[GPT];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < GPT; ++u)
      wgrad_value4(a, r0 + rg + 8 * u, rend, k0 + 4 * cg, n0 + 4 * cg, xv[u], dv[u]);
  };
  if (rbeg < rend) fetch(rbeg);
  for (int64_t rs = rbeg; rs < rend; rs += R) {
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      *(float4*)&xs[rg + 8 * u][4 * cg] = xv[u];
      *(float4*)&ds[rg + 8 * u][4 * cg] = dv[u];
    }
    __syncthreads();
    if (rs + R < rend) fetch(rs + R);
    if (fold && threadIdx.x < WT)
      for (int rr = 0; rr < R; ++rr) bsum += ds[rr][threadIdx.x];
#pragma unroll
    for (int rr = 0; rr < R; rr += 4) {
      float xa[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) xa[i] = xs[rr + g][wave * 32 + i * 16 + r];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float da = ds[rr + g][j * 16 + r];
#pragma unroll
        for (int i = 0; i < 2; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(da, xa[i], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (fold && threadIdx.x < WT)
    partial[((size_t)tile.chunk * Kb + a.K) * a.N + n0 + threadIdx.x] = bsum;
  // lane holds k = k0 + 32 wave + 16 i + r and n = n0 + 16 j + 4 g + c
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int k = k0 + wave * 32 + i * 16 + r;
    float* P = partial + ((size_t)tile.chunk * Kb + k) * a.N;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      *(float4*)(P + n0 + j * 16 + 4 * g) = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
  }
}

// Wide layers in BF16 (K and N multiples of 128): the same 128 x 128 output tile with
// BF16 operands, 64 rows staged per step in tiles held transposed as in the 64 x 64
// BF16 kernel.  Thread t stages eight consecutive rows of four columns of X and the
// same of D (column group t mod 32, row group t / 32) as four 16-byte column runs
// each, and requests the next step's rows once the barrier after those writes has
// passed, so that they arrive while the step's products run (a barrier waits for
// every load still in flight).  Wave w owns k rows [32w, 32w + 32) and all 128 n
// columns: per 32 staged rows it reads two X and eight D fragments for sixteen
// products.  The k tile 0 workgroups sum the bias row (with_bias).
__global__ __launch_bounds__(256) void wgrad128_bf16_kernel(WgradIn a, int64_t m, int64_t rows_per_chunk,
                                                            float* __restrict__ partial, int ktiles, int ntiles,
                                                            int chunks) {
  WgradTile tile;
  if (!wgrad_tile(ktiles, ntiles, chunks, tile)) return;
  constexpr int R = 64;                        // rows staged per step
  constexpr int LDB = R + 8;                   // row stride of the transposed tiles (bf16)
  __shared__ __align__(16) __bf16 xt[WT][LDB];
  __shared__ __align__(16) __bf16 dt[WT][LDB];
  const int wave = threadIdx.x >> 6, l = lane_id(), g = l >> 4, r = l & 15;
  const int k0 = tile.kt * WT, n0 = tile.nt * WT;
  const int Kb = a.K + (a.with_bias ? 1 : 0);
  const int64_t rbeg = (int64_t)tile.chunk * rows_per_chunk;
  const int64_t rend = min(m, rbeg + rows_per_chunk);
  const bool fold = a.with_bias && tile.kt == 0;
  float bsum = 0.f;
  f32x4 acc[2][8];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  static_assert(R == 64 && WT == 128, "256 threads x 8 rows x 4 columns per operand");
  const int cg = threadIdx.x & 31, rg = threadIdx.x >> 5;
  float4 xv[8], dv[8];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      xv[j] = wgrad_x4(a, r0 + 8 * rg + j, rend, k0 + 4 * cg);
      dv[j] = wgrad_d4(a, r0 + 8 * rg + j, rend, n0 + 4 * cg);
    }
  };
  auto put = [&](__bf16 (*t)[LDB], const float4 (&v)[8]) {
    bf16x8 w0, w1, w2, w3;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      w0[j] = (__bf16)v[j].x; w1[j] = (__bf16)v[j].y;
      w2[j] = (__bf16)v[j].z; w3[j] = (__bf16)v[j].w;
    }
    *(bf16x8*)&t[4 * cg][8 * rg] = w0;
    *(bf16x8*)&t[4 * cg + 1][8 * rg] = w1;
    *(bf16x8*)&t[4 * cg + 2][8 * rg] = w2;
    *(bf16x8*)&t[4 * cg + 3][8 * rg] = w3;
  };
  if (rbeg < rend) fetch(rbeg);
  for (int64_t rs = rbeg; rs < rend; rs += R) {
    put(xt, xv);
    put(dt, dv);
    __syncthreads();
    if (rs + R < rend) fetch(rs + R);
    if (fold && threadIdx.x < WT)
      for (int rr = 0; rr < R; ++rr) bsum += (float)dt[threadIdx.x][rr];
#pragma unroll
    for (int rr = 0; rr < R; rr += 32) {
      bf16x8 xb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) xb[i] = *(const bf16x8*)&xt[wave * 32 + i * 16 + r][rr + 8 * g];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const bf16x8 da = *(const bf16x8*)&dt[j * 16 + r][rr + 8 * g];
#pragma unroll
        for (int i = 0; i < 2; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(da, xb[i], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (fold && threadIdx.x < WT)
    partial[((size_t)tile.chunk * Kb + a.K) * a.N + n0 + threadIdx.x] = bsum;
  // lane holds k = k0 + 32 wave + 16 i + r and n = n0 + 16 j + 4 g + c
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int k = k0 + wave * 32 + i * 16 + r;
    float* P = partial + ((size_t)tile.chunk * Kb + k) * a.N;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      *(float4*)(P + n0 + j * 16 + 4 * g) = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
  }
}

__global__ void wgrad_reduce_kernel(const float* __restrict__ partial, int chunks, int64_t count, float* __restrict__ grad) {
  GRID_STRIDE(i, count) {
    float s = 0.f;
#pragma unroll 8
    for (int c = 0; c < chunks; ++c) s += partial[(size_t)c * count + i];
    grad[i] += s;
  }
}

// per-node sums of rows of M [m][H] over incidence lists (src, dst or both), fixed order
__global__ void segsum_kernel(ActBuf M, int H, const int* __restrict__ p1, const int* __restrict__ i1,
                              const int* __restrict__ p2, const int* __restrict__ i2, int n, float* __restrict__ out,
                              int ldo, float sign2) {
  const int waves = gridDim.x * (blockDim.x >> 6);
  const int l = lane_id();
  for (int node = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); node < n; node += waves) {
    for (int c = l; c < H; c += 64) {
      float s = 0.f;
      if (p1)
        for (int k = p1[node]; k < p1[node + 1]; ++k) s += M.get((size_t)i1[k] * H + c);
      if (p2) {
        float s2 = 0.f;
        for (int k = p2[node]; k < p2[node + 1]; ++k) s2 += M.get((size_t)i2[k] * H + c);
        s += sign2 * s2;
      }
      out[(size_t)node * ldo + c] = s;
    }
  }
}

// The same sums, four columns per lane (16-byte loads of FP32 rows, 8-byte of BF16):
// LPR = H / 4 lanes per node, 64 / LPR nodes per wave; each column is summed in the
// same order as above, so the results are identical
template <int LPR>
__global__ void segsum4_kernel(ActBuf M, int H, const int* __restrict__ p1, const int* __restrict__ i1,
                               const int* __restrict__ p2, const int* __restrict__ i2, int n, float* __restrict__ out,
                               int ldo, float sign2) {
  constexpr int NPW = 64 / LPR;
  const int l = lane_id();
  const int c = (l % LPR) * 4;
  const int waves = gridDim.x * (blockDim.x >> 6);
  for (int base = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * NPW; base < n; base += waves * NPW) {
    const int node = base + l / LPR;
    if (node >= n) continue;
    float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
    if (p1) {
      const int kb = p1[node], ke = p1[node + 1];
#pragma unroll 4
      for (int k = kb; k < ke; ++k) {
        const float4 v = M.get4((size_t)i1[k] * H + c);
        sum.x += v.x; sum.y += v.y; sum.z += v.z; sum.w += v.w;
      }
    }
    if (p2) {
      float4 s2 = make_float4(0.f, 0.f, 0.f, 0.f);
      const int kb = p2[node], ke = p2[node + 1];
#pragma unroll 4
      for (int k = kb; k < ke; ++k) {
        const float4 v = M.get4((size_t)i2[k] * H + c);
        s2.x += v.x; s2.y += v.y; s2.z += v.z; s2.w += v.w;
      }
      sum.x += sign2 * s2.x; sum.y += sign2 * s2.y; sum.z += sign2 * s2.z; sum.w += sign2 * s2.w;
    }
    *(float4*)(out + (size_t)node * ldo + c) = sum;
  }
}

// ---------------------------------------------------------------------------
// elementwise kernels
// ---------------------------------------------------------------------------
// X[r] = [S[src[r]] | S[dst[r]]], width 2*d (ld = ldx)
__global__ void pair_gather_kernel(const float* S, int d, int n, const int* src, const int* dst, int64_t m, ActBuf X,
                                   int ldx) {
  GRID_STRIDE(i, m * 2 * d) {
    const int64_t r = i / (2 * d);
    const int c = (int)(i - r * 2 * d);
    X.set(r * ldx + c, c < d ? S[node_of(src[r], n) * d + c] : S[node_of(dst[r], n) * d + c - d]);
  }
}
// out[r][0:H] = A[r], out[r][H:2H] = B[r]
__global__ void concat_kernel(ActBuf A, const float* B, int64_t n, int H, float* out) {
  GRID_STRIDE(i, n * 2 * H) {
    const int64_t r = i / (2 * H);
    const int c = (int)(i - r * 2 * H);
    out[i] = c < H ? A.get(r * H + c) : B[r * H + c - H];
  }
}
// de[e] += dm[src[e]] + dm[dst[e]]   (dm rows with stride ldm, H columns)
__global__ void gather_add_kernel(const float* dm, int ldm, const int* src, const int* dst, int n, int64_t m, int H,
                                  float* de) {
  GRID_STRIDE(i, m * H) {
    const int64_t r = i / H;
    const int c = (int)(i - r * H);
    de[i] += dm[node_of(src[r], n) * ldm + c] + dm[node_of(dst[r], n) * ldm + c];
  }
}
// out[r][c] = dz[r] * w[c] * (1 - u[r][c]^2)
__global__ void outgrad_kernel(const float* dz, const float* w, ActBuf u, int64_t m, int H, float* out) {
  GRID_STRIDE(i, m * H) {
    const int64_t r = i / H;
    const int c = (int)(i - r * H);
    const float a = u.get(i);
    out[i] = dz[r] * w[c] * (1.f - a * a);
  }
}
// out[r][c] = a[r][c] + b[r * ldb + c], c < H
__global__ void add_cols_kernel(const float* a, const float* b, int ldb, int64_t n, int H, float* out) {
  GRID_STRIDE(i, n * H) {
    const int64_t r = i / H;
    const int c = (int)(i - r * H);
    out[i] = a[i] + b[(size_t)r * ldb + c];
  }
}
// out = d * (1 - a^2)
__global__ void dtanh_kernel(const float* d, ActBuf a, int64_t count, float* out) {
  GRID_STRIDE(i, count) {
    const float v = a.get(i);
    out[i] = d[i] * (1.f - v * v);
  }
}

// bce: per-block partial loss sums (fixed order) and dz = (sigmoid(z) - y) / m
__global__ __launch_bounds__(256) void bce_kernel(const float* z, const float* y, int64_t m, float* dz, float* part) {
  __shared__ float sh[256];
  float s = 0.f;
  GRID_STRIDE(i, m) {
    const float zi = z[i], yi = y[i];
    s += fmaxf(zi, 0.f) - zi * yi + log1pf(trk_exp(-fabsf(zi)));
    dz[i] = (trk_sigmoid(zi) - yi) / (float)m;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void bce_sum_kernel(const float* part, int nb, int64_t m, float* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < nb; ++i) s += part[i];
    *loss = m > 0 ? s / (float)m : 0.f;
  }
}

__global__ void adam_kernel(float* p, const float* gr, float* mo, float* ve, int64_t count, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  GRID_STRIDE(i, count) {
    const float gi = gr[i];
    const float mi = b1 * mo[i] + (1.f - b1) * gi;
    const float vi = b2 * ve[i] + (1.f - b2) * gi * gi;
    mo[i] = mi;
    ve[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// pair objective: counts of positive / negative pairs (block partials)
__global__ __launch_bounds__(256) void pair_count_kernel(const float* y, int64_t P, int* part) {
  __shared__ int sh[256];
  int c = 0;
  GRID_STRIDE(i, P) c += y[i] > 0.5f ? 1 : 0;
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void pair_count_sum_kernel(const int* part, int nb, int64_t P, int* counts) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int s = 0;
    for (int i = 0; i < nb; ++i) s += part[i];
    counts[0] = s;
    counts[1] = (int)(P - s);
  }
}
// per pair: g = coef * (e[a] - e[b]) with coef = 2/npos (positive) or
// -2 w max(0, margin - d) / d / nneg (negative, weight w); block partial sums of the loss
__global__ __launch_bounds__(256) void pair_grad_kernel(const float* __restrict__ emb, int D, int n,
                                                        const int* __restrict__ pa, const int* __restrict__ pb,
                                                        const float* __restrict__ y, int64_t P, float margin,
                                                        float neg_weight,
                                                        const int* __restrict__ counts, float* __restrict__ g,
                                                        float* __restrict__ part) {
  __shared__ float sh[256];
  const int npos = counts[0], nneg = counts[1];
  float lsum = 0.f;
  GRID_STRIDE(p, P) {
    const size_t a = node_of(pa[p], n), b = node_of(pb[p], n);
    float diff[16];
    float d2 = 0.f;
    for (int k = 0; k < D; ++k) {
      diff[k] = emb[a * D + k] - emb[b * D + k];
      d2 = fmaf(diff[k], diff[k], d2);
    }
    float coef = 0.f;
    if (y[p] > 0.5f) {
      lsum += d2 / (float)npos;
      coef = 2.f / (float)npos;
    } else {
      const float d = sqrtf(d2);
      const float h = fmaxf(0.f, margin - d);
      lsum += neg_weight * h * h / (float)nneg;
      if (h > 0.f && d > 0.f) coef = -2.f * neg_weight * h / d / (float)nneg;
    }
    for (int k = 0; k < D; ++k) g[(size_t)p * D + k] = coef * diff[k];
  }
  sh[threadIdx.x] = lsum;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

}  // namespace

// ===========================================================================
// host side
// ===========================================================================
struct LayerOff {
  int64_t w = 0, b = 0;  // float offsets of W[K][N] and b[N] in the flat parameter vector
  int K = 0, N = 0;
};

struct TrainState {
  int64_t n_params = 0;
  bool bf16 = false;   // BF16 operands for every product (a BF16 context)
  std::vector<LayerOff> filt, ne, ee, en, nn, out, emb;   // per network, per layer
  // fragment blocks for the training products (FP32, or BF16 in a BF16 context)
  void* fmem = nullptr;
  std::vector<DevLayer> filtF;       // forward layers 0..L (last: K x 1)
  std::vector<DevLayer> filtT;       // transposed hidden layers 1..L-1 (index l -> W_l^T)
  std::vector<DevLayer> embF, embT;  // embedding: forward 0..L, transposed 1..L
  DevLayer ne1, ne2, ee1, ee2, ec, eab, e2, n1, n2, oc, oab, o2;   // forward
  DevLayer ne2T, ee2T, ecT, eabT, e2T, n1T, n2T, ocT, oabT;        // transposed
  // buffers
  Arena arena;
  // activations kept from forward to backward (BF16 in a BF16 context)
  ActBuf fx0, fact, x6, ea1, na1, hck, eck, u, eact;
  float *fdel0 = nullptr, *fdel1 = nullptr;
  float *P = nullptr, *t1 = nullptr, *v = nullptr;
  float *de = nullptr, *dpre = nullptr, *dpre1 = nullptr, *msg = nullptr, *nin = nullptr, *q1 = nullptr, *q2 = nullptr;
  float *dh = nullptr, *dh2 = nullptr, *dq = nullptr, *dq1 = nullptr, *dnin = nullptr, *dP = nullptr, *tmpN = nullptr;
  float* partial = nullptr;
  int64_t partial_floats = 0;
  int n_cu = 256;   // compute units of the context's device (the weight-gradient grids)
  float* bce_part = nullptr;
  int64_t cap_c = 0, cap_f = 0, nmax = 0;
  // embedding training
  float *edel0 = nullptr, *edel1 = nullptr, *pg = nullptr;
  int* pcounts = nullptr;
  GnnScratch pairs;     // incidence lists of the pairs (by first and by second hit)
};

namespace {

void offsets_for(const trk_config& k, TrainState& T) {
  int64_t o = 0;
  auto net = [&](std::vector<LayerOff>& v, std::initializer_list<int> dims) {
    std::vector<int> d(dims);
    for (size_t i = 0; i + 1 < d.size(); ++i) {
      LayerOff L;
      L.K = d[i];
      L.N = d[i + 1];
      L.w = o;
      o += (int64_t)L.K * L.N;
      L.b = o;
      o += L.N;
      v.push_back(L);
    }
  };
  std::vector<int> fd;
  fd.push_back(2 * k.emb_dim);
  for (int i = 0; i < k.filt_layers; ++i) fd.push_back(k.filt_hidden);
  fd.push_back(1);
  {
    int64_t dummy = 0;
    (void)dummy;
    for (size_t i = 0; i + 1 < fd.size(); ++i) {
      LayerOff L;
      L.K = fd[i];
      L.N = fd[i + 1];
      L.w = o;
      o += (int64_t)L.K * L.N;
      L.b = o;
      o += L.N;
      T.filt.push_back(L);
    }
  }
  const int H = k.gnn_hidden;
  net(T.ne, {3, H, H});
  net(T.ee, {6, H, H});
  net(T.en, {3 * H, H, H});
  net(T.nn, {2 * H, H, H});
  net(T.out, {3 * H, H, 1});
  {
    std::vector<int> ed;
    ed.push_back(3);
    for (int i = 0; i < k.emb_layers; ++i) ed.push_back(k.emb_hidden);
    ed.push_back(k.emb_dim);
    for (size_t i = 0; i + 1 < ed.size(); ++i) {
      LayerOff L;
      L.K = ed[i];
      L.N = ed[i + 1];
      L.w = o;
      o += (int64_t)L.K * L.N;
      L.b = o;
      o += L.N;
      T.emb.push_back(L);
    }
  }
  T.n_params = o;
}

size_t frag_bytes(int K, int N) { return (size_t)((K + 15) / 16) * ((N + 15) / 16) * 64 * 16; }

struct FragAlloc {
  std::vector<std::pair<DevLayer*, std::pair<int, int>>> req;
  size_t total = 0;
  bool bf16 = false;   // BF16 blocks take k in 32s (the FP32 size is allocated either way)
  void add(DevLayer& L, int K, int N) {
    L.K = K;
    L.N = N;
    L.nkb = bf16 ? (K + 31) / 32 : (K + 15) / 16;
    L.nnt = (N + 15) / 16;
    req.push_back({&L, {K, N}});
    total += frag_bytes(K, N) + (size_t)L.nnt * 16 * 4 + 512;
  }
  void place(void* base) {
    size_t off = 0;
    for (auto& r : req) {
      r.first->w = (const uint4*)((char*)base + off);
      off += (frag_bytes(r.second.first, r.second.second) + 255) & ~(size_t)255;
      r.first->b = (const float*)((char*)base + off);
      off += ((size_t)r.first->nnt * 16 * 4 + 255) & ~(size_t)255;
    }
  }
};

void fill(const DevLayer& L, int K, int N, MatView A, MatView B, int mode, int split, const float* bias, int bf16,
          hipStream_t s) {
  const int64_t nblk = (int64_t)L.nkb * L.nnt * 64;
  frag_fill_kernel<<<blocks_for(nblk, 256), 256, 0, s>>>((uint4*)L.w, L.nkb, L.nnt, K, N, A, B, mode, split, bf16);
  bias_fill_kernel<<<blocks_for(L.nnt * 16, 256), 256, 0, s>>>((float*)L.b, (float*)L.bs, L.nnt * 16, bias,
                                                               bias ? N : 0);
}

MatView view(const float* P, const LayerOff& L, int r0 = 0, int trans = 0) {
  MatView v;
  v.p = P + L.w;
  v.r0 = r0;
  v.ld = L.N;
  v.trans = trans;
  return v;
}

// the staged row tile is sized for the layer's fan-in, so that narrow layers (the
// interaction network's, K <= 256) leave LDS for two to four workgroups per compute
// unit, which hide one another's staging loads; the wide layers (K of 512 and more),
// whose tile leaves room for one or two workgroups, run eight waves per workgroup
template <class P, int NW, int NTW, int MT, int KMAX>
void rowgemm_launch(ActBuf X, int ldx, int K, int64_t m, const DevLayer& W, ActBuf out, int ldo, int N, int epi,
                    ActBuf aux, int ldaux, const PairIn& pr, int resident, hipStream_t s) {
  const int64_t tiles = (m + MT - 1) / MT;
  const int grid = (int)std::min<int64_t>(tiles, resident);
  if (grid > 0)
    rowgemm_kernel<P, NW, NTW, MT, KMAX><<<grid, NW * 64, 0, s>>>(X, ldx, K, m, W, out, ldo, N, epi, aux, ldaux, pr);
}

template <class P, int NW, int MT, int KMAX>
void rowgemm_w(ActBuf X, int ldx, int K, int64_t m, const DevLayer& W, ActBuf out, int ldo, int N, int epi,
               ActBuf aux, int ldaux, const PairIn& pr, int resident, hipStream_t s) {
  const int per_wave = (W.nnt + NW - 1) / NW;
  if (per_wave <= 1) rowgemm_launch<P, NW, 1, MT, KMAX>(X, ldx, K, m, W, out, ldo, N, epi, aux, ldaux, pr, resident, s);
  else if (per_wave <= 2) rowgemm_launch<P, NW, 2, MT, KMAX>(X, ldx, K, m, W, out, ldo, N, epi, aux, ldaux, pr, resident, s);
  else rowgemm_launch<P, NW, 4, MT, KMAX>(X, ldx, K, m, W, out, ldo, N, epi, aux, ldaux, pr, resident, s);
}

template <class P>
void rowgemm_p(ActBuf X, int ldx, int K, int64_t m, const DevLayer& W, ActBuf out, int ldo, int N, int epi,
               ActBuf aux, int ldaux, const PairIn& pr, int n_cu, hipStream_t s) {
  const int kpad = W.nkb * P::KB;
  if (kpad <= 128)
    rowgemm_w<P, 4, 64, 128>(X, ldx, K, m, W, out, ldo, N, epi, aux, ldaux, pr, n_cu * 8, s);
  else if (kpad <= 256)
    rowgemm_w<P, 4, 64, 256>(X, ldx, K, m, W, out, ldo, N, epi, aux, ldaux, pr, n_cu * 4, s);
  else if (kpad <= 512)
    rowgemm_w<P, 8, 64, 512>(X, ldx, K, m, W, out, ldo, N, epi, aux, ldaux, pr, n_cu * 2, s);
  else
    rowgemm_w<P, 8, 32, 1024>(X, ldx, K, m, W, out, ldo, N, epi, aux, ldaux, pr, n_cu * 2, s);
}

// out = epi(X W) with W's blocks in the training precision (bf16: BF16 blocks)
void rowgemm(ActBuf X, int ldx, int K, int64_t m, const DevLayer& W, ActBuf out, int ldo, int N, int epi,
             ActBuf aux, int ldaux, int n_cu, hipStream_t s, bool bf16, const PairIn& pr = PairIn()) {
  if (bf16) rowgemm_p<PrecBF16>(X, ldx, K, m, W, out, ldo, N, epi, aux, ldaux, pr, n_cu, s);
  else rowgemm_p<PrecF32>(X, ldx, K, m, W, out, ldo, N, epi, aux, ldaux, pr, n_cu, s);
}

void wgrad(TrainState& T, ActBuf X, int ldx, const int* gsrc, const int* gdst, const float* S, int gd, int gn,
           int K, bool bias, const float* D, int ldd, int N, int64_t m, float* grad, hipStream_t s) {
  const int Kb = K + (bias ? 1 : 0);
  const int64_t count = (int64_t)Kb * N;
  // row chunks: enough workgroups to fill the chip several times over (at least 512
  // rows per chunk, at most 256 chunks), within the partial-sum buffer; the chunk
  // partition depends only on m and the shape, so the sums are reproducible
  const WgradIn a{X, ldx, gsrc, gdst, S, gd, gn, K, bias ? 1 : 0, D, ldd, N};
  // wide layers on 128 x 128 output tiles
  if (m > 0 && wgrad_vec(a) && K % WT == 0 && N % WT == 0 && K >= 2 * WT && N >= 2 * WT) {
    const int64_t tiles = (int64_t)(K / WT) * (N / WT);
    const int64_t want = std::max<int64_t>(1, (4 * (int64_t)T.n_cu + tiles - 1) / tiles);
    int chunks = (int)std::min<int64_t>({256, want, std::max<int64_t>(1, m / 512)});
    while (chunks > 1 && (int64_t)chunks * count > T.partial_floats) --chunks;
    const int64_t rpc = std::max<int64_t>(1, (m + chunks - 1) / chunks);
    if (T.bf16)
      wgrad128_bf16_kernel<<<wgrad_grid(tiles, chunks), 256, 0, s>>>(a, m, rpc, T.partial, K / WT, N / WT, chunks);
    else
      wgrad128_kernel<<<wgrad_grid(tiles, chunks), 256, 0, s>>>(a, m, rpc, T.partial, K / WT, N / WT, chunks);
    wgrad_reduce_kernel<<<blocks_for(count, 256), 256, 0, s>>>(T.partial, chunks, count, grad);
    return;
  }
  const int ktiles = ((wgrad_fold(a) ? K : Kb) + WG_T - 1) / WG_T;
  const int64_t tiles = (int64_t)ktiles * ((N + WG_T - 1) / WG_T);
  const int64_t want = std::max<int64_t>(1, (8 * (int64_t)T.n_cu + tiles - 1) / tiles);
  int chunks = (int)std::min<int64_t>({256, want, std::max<int64_t>(1, m / 512)});
  while (chunks > 1 && (int64_t)chunks * count > T.partial_floats) --chunks;
  const int64_t rpc = std::max<int64_t>(1, (m + chunks - 1) / chunks);
  const int ntiles = (N + WG_T - 1) / WG_T;
  if (m > 0) {
    if (T.bf16)
      wgrad_bf16_kernel<<<wgrad_grid(tiles, chunks), 256, 0, s>>>(a, m, rpc, T.partial, ktiles, ntiles, chunks);
    else
      wgrad_kernel<<<wgrad_grid(tiles, chunks), 256, 0, s>>>(a, m, rpc, T.partial, ktiles, ntiles, chunks);
    wgrad_reduce_kernel<<<blocks_for(count, 256), 256, 0, s>>>(T.partial, chunks, count, grad);
  }
}

void segsum(ActBuf M, int H, const int* p1, const int* i1, const int* p2, const int* i2, int n, float* out, int ldo,
            hipStream_t s, float sign2 = 1.f) {
  if (ldo % 4 == 0 && (H == 128 || H == 64)) {
    // 2 (H = 128) or 4 (H = 64) nodes per wave, four waves per block
    const int per_block = 4 * (H == 128 ? 2 : 4);
    if (H == 128)
      segsum4_kernel<32><<<blocks_for(n, per_block, 16384), 256, 0, s>>>(M, H, p1, i1, p2, i2, n, out, ldo, sign2);
    else
      segsum4_kernel<16><<<blocks_for(n, per_block, 16384), 256, 0, s>>>(M, H, p1, i1, p2, i2, n, out, ldo, sign2);
    return;
  }
  segsum_kernel<<<blocks_for(n, 4, 16384), 256, 0, s>>>(M, H, p1, i1, p2, i2, n, out, ldo, sign2);
}

template <class K, class... A>
void ew(K kernel, int64_t count, hipStream_t s, A... args) {
  if (count > 0) kernel<<<blocks_for(count, 256, 8192), 256, 0, s>>>(args...);
}

}  // namespace

// ---------------------------------------------------------------------------
// internal API used by trk_api.hip
// ---------------------------------------------------------------------------
int train_create(trk_ctx* c) {
  const trk_config& k = c->cfg;
  const bool all_f32 = c->prec == TRK_PREC_F32 && c->prec_emb == TRK_PREC_F32 && c->prec_gnn == TRK_PREC_F32;
  const bool all_bf16 = c->prec == TRK_PREC_BF16 && c->prec_emb == TRK_PREC_BF16 && c->prec_gnn == TRK_PREC_BF16;
  if (!all_f32 && !all_bf16) return TRK_E_INVAL;
  TrainState* T = new TrainState();
  c->train = T;
  T->bf16 = all_bf16;
  offsets_for(k, *T);
  const int H = k.gnn_hidden, F = k.filt_hidden, D = k.emb_dim, L = k.filt_layers;
  FragAlloc fa;
  fa.bf16 = T->bf16;
  T->filtF.resize(L + 1);
  T->filtT.resize(L + 1);
  for (int i = 0; i <= L; ++i) fa.add(T->filtF[i], T->filt[i].K, T->filt[i].N);
  for (int i = 1; i < L; ++i) fa.add(T->filtT[i], F, F);
  fa.add(T->ne1, 3, H); fa.add(T->ne2, H, H); fa.add(T->ee1, 6, H); fa.add(T->ee2, H, H);
  fa.add(T->ec, H, H); fa.add(T->eab, H, 2 * H); fa.add(T->e2, H, H);
  fa.add(T->n1, 2 * H, H); fa.add(T->n2, H, H);
  fa.add(T->oc, H, H); fa.add(T->oab, H, 2 * H); fa.add(T->o2, H, 1);
  fa.add(T->ne2T, H, H); fa.add(T->ee2T, H, H); fa.add(T->ecT, H, H); fa.add(T->eabT, 2 * H, H);
  fa.add(T->e2T, H, H); fa.add(T->n1T, H, 2 * H); fa.add(T->n2T, H, H); fa.add(T->ocT, H, H);
  fa.add(T->oabT, 2 * H, H);
  const int EL = k.emb_layers, EW = k.emb_hidden;
  T->embF.resize(EL + 1);
  T->embT.resize(EL + 1);
  for (int i = 0; i <= EL; ++i) fa.add(T->embF[i], T->emb[i].K, T->emb[i].N);
  for (int i = 1; i <= EL; ++i) fa.add(T->embT[i], T->emb[i].N, T->emb[i].K);
  if (hipMalloc(&T->fmem, fa.total) != hipSuccess) return TRK_E_NOMEM;
  fa.place(T->fmem);
  const int64_t CC = k.max_cand_edges, CF = k.max_kept_edges, NH = k.max_hits, It = k.gnn_iters;
  T->cap_c = CC;
  T->cap_f = CF;
  T->nmax = NH;
  Arena& a = T->arena;
  auto act = [&](ActBuf& b, size_t count) {
    b.bf16 = T->bf16 ? 1 : 0;
    a.add_bytes(b.p, count * (T->bf16 ? 2 : 4));
  };
  act(T->fx0, (size_t)CC * 2 * D);
  act(T->fact, (size_t)L * CC * F);
  a.add(T->fdel0, (size_t)CC * F);
  a.add(T->fdel1, (size_t)CC * F);
  act(T->x6, (size_t)CF * 6);
  act(T->ea1, (size_t)CF * H);
  act(T->na1, (size_t)NH * H);
  act(T->hck, (size_t)(It + 1) * NH * H);
  act(T->eck, (size_t)(It + 1) * CF * H);
  act(T->u, (size_t)CF * H);
  a.add(T->P, (size_t)NH * 2 * H);
  for (float** p : {&T->t1, &T->v, &T->de, &T->dpre, &T->dpre1}) a.add(*p, (size_t)CF * H);
  a.add(T->msg, (size_t)NH * H);
  a.add(T->nin, (size_t)NH * 2 * H);
  for (float** p : {&T->q1, &T->q2, &T->dh, &T->dh2, &T->dq, &T->dq1, &T->tmpN}) a.add(*p, (size_t)NH * H);
  a.add(T->dnin, (size_t)NH * 2 * H);
  a.add(T->dP, (size_t)NH * 2 * H);
  T->partial_floats = std::max<int64_t>((int64_t)16 * 513 * 512, (int64_t)8 * (EW + 1) * EW);
  T->n_cu = c->n_cu;
  act(T->eact, (size_t)EL * NH * EW);
  a.add(T->edel0, (size_t)NH * EW);
  a.add(T->edel1, (size_t)NH * EW);
  a.add(T->pg, (size_t)CC * k.emb_dim);
  a.add(T->pcounts, 8);
  a.add(T->pairs.rowptr, NH + 1);
  a.add(T->pairs.rowidx, CC);
  a.add(T->pairs.cscptr, NH + 1);
  a.add(T->pairs.cscidx, CC);
  a.add(T->pairs.raw, CC);
  a.add(T->pairs.cnt, NH);
  a.add(T->pairs.tmp, scan_tmp_ints(std::max<int64_t>(CC, NH + 1)));
  a.add(T->partial, (size_t)T->partial_floats);
  a.add(T->bce_part, 16384);
  if (a.commit() != hipSuccess) return TRK_E_NOMEM;
  return TRK_OK;
}

void train_destroy(trk_ctx* c) {
  if (!c->train) return;
  if (c->train->fmem) hipFree(c->train->fmem);
  if (c->train->arena.base) hipFree(c->train->arena.base);
  delete c->train;
  c->train = nullptr;
}

int64_t train_param_count(const trk_config& k) {
  TrainState T;
  offsets_for(k, T);
  return T.n_params;
}

// Rebuilds every fragment block (forward, transposed, and the inference layers of
// the context) from the flat parameter vector P (device).
int train_set_params(trk_ctx* c, const float* P, hipStream_t s) {
  TrainState& T = *c->train;
  const int H = c->cfg.gnn_hidden, L = c->cfg.filt_layers;
  MatView none;
  for (int i = 0; i <= L; ++i) {
    const LayerOff& o = T.filt[i];
    fill(T.filtF[i], o.K, o.N, view(P, o), none, 0, 0, P + o.b, T.bf16, s);
    if (i >= 1 && i < L) fill(T.filtT[i], o.N, o.K, view(P, o, 0, 1), none, 0, 0, nullptr, T.bf16, s);
  }
  fill(T.ne1, 3, H, view(P, T.ne[0]), none, 0, 0, P + T.ne[0].b, T.bf16, s);
  fill(T.ne2, H, H, view(P, T.ne[1]), none, 0, 0, P + T.ne[1].b, T.bf16, s);
  fill(T.ee1, 6, H, view(P, T.ee[0]), none, 0, 0, P + T.ee[0].b, T.bf16, s);
  fill(T.ee2, H, H, view(P, T.ee[1]), none, 0, 0, P + T.ee[1].b, T.bf16, s);
  fill(T.ec, H, H, view(P, T.en[0], 2 * H), none, 0, 0, P + T.en[0].b, T.bf16, s);
  fill(T.eab, H, 2 * H, view(P, T.en[0], 0), view(P, T.en[0], H), 1, H, nullptr, T.bf16, s);
  fill(T.e2, H, H, view(P, T.en[1]), none, 0, 0, P + T.en[1].b, T.bf16, s);
  fill(T.n1, 2 * H, H, view(P, T.nn[0]), none, 0, 0, P + T.nn[0].b, T.bf16, s);
  fill(T.n2, H, H, view(P, T.nn[1]), none, 0, 0, P + T.nn[1].b, T.bf16, s);
  fill(T.oc, H, H, view(P, T.out[0], 2 * H), none, 0, 0, P + T.out[0].b, T.bf16, s);
  fill(T.oab, H, 2 * H, view(P, T.out[0], 0), view(P, T.out[0], H), 1, H, nullptr, T.bf16, s);
  fill(T.o2, H, 1, view(P, T.out[1]), none, 0, 0, P + T.out[1].b, T.bf16, s);
  // transposed: element (k, n) of W^T is W[n][k]
  fill(T.ne2T, H, H, view(P, T.ne[1], 0, 1), none, 0, 0, nullptr, T.bf16, s);
  fill(T.ee2T, H, H, view(P, T.ee[1], 0, 1), none, 0, 0, nullptr, T.bf16, s);
  fill(T.ecT, H, H, view(P, T.en[0], 2 * H, 1), none, 0, 0, nullptr, T.bf16, s);
  fill(T.eabT, 2 * H, H, view(P, T.en[0], 0, 1), view(P, T.en[0], H, 1), 2, H, nullptr, T.bf16, s);
  fill(T.e2T, H, H, view(P, T.en[1], 0, 1), none, 0, 0, nullptr, T.bf16, s);
  fill(T.n1T, H, 2 * H, view(P, T.nn[0], 0, 1), none, 0, 0, nullptr, T.bf16, s);
  fill(T.n2T, H, H, view(P, T.nn[1], 0, 1), none, 0, 0, nullptr, T.bf16, s);
  fill(T.ocT, H, H, view(P, T.out[0], 2 * H, 1), none, 0, 0, nullptr, T.bf16, s);
  fill(T.oabT, 2 * H, H, view(P, T.out[0], 0, 1), view(P, T.out[0], H, 1), 2, H, nullptr, T.bf16, s);
  // the context's inference layers, in the context's precision
  const int inf_bf16 = c->prec == TRK_PREC_BF16 ? 1 : 0;
  auto same = [&](DevLayer& dst, const LayerOff& o, int r0, int K, MatView B = MatView(), int mode = 0) {
    fill(dst, K, o.N * (mode == 1 ? 2 : 1), view(P, o, r0), B, mode, o.N, mode == 1 ? nullptr : P + o.b, inf_bf16,
         s);
  };
  for (int i = 0; i <= c->cfg.emb_layers; ++i) {
    const LayerOff& o = T.emb[i];
    fill(T.embF[i], o.K, o.N, view(P, o), none, 0, 0, P + o.b, T.bf16, s);
    if (i >= 1) fill(T.embT[i], o.N, o.K, view(P, o, 0, 1), none, 0, 0, nullptr, T.bf16, s);
  }
  same(c->emb_in, T.emb[0], 0, 3);
  for (int i = 1; i < c->cfg.emb_layers; ++i) same(c->emb_hid.l[i - 1], T.emb[i], 0, T.emb[i].K);
  {  // a BF16 embedding's output layer is kept in FP32 (embed_kernel)
    const LayerOff& o = T.emb[c->cfg.emb_layers];
    fill(c->emb_out, o.K, o.N, view(P, o), none, 0, 0, P + o.b, c->cfg.emb_layers > 1 ? 0 : inf_bf16, s);
  }
  if (inf_bf16)   // the BF16 first layer reads the pair's mean and difference
    fill(c->filt_in, T.filt[0].K, T.filt[0].N, view(P, T.filt[0]), none, 3, T.filt[0].K / 2, P + T.filt[0].b, 1, s);
  else
    same(c->filt_in, T.filt[0], 0, T.filt[0].K);
  for (int i = 1; i < L; ++i) same(c->filt_hid.l[i - 1], T.filt[i], 0, T.filt[i].K);
  DevGNN& G = c->gnn;
  // the encoders' first layers are FP32 in every precision
  fill(G.node_enc1, 3, T.ne[0].N, view(P, T.ne[0]), none, 0, 0, P + T.ne[0].b, 0, s);
  same(G.node_enc2, T.ne[1], 0, H);
  fill(G.edge_enc1, 6, T.ee[0].N, view(P, T.ee[0]), none, 0, 0, P + T.ee[0].b, 0, s);
  same(G.edge_enc2, T.ee[1], 0, H);
  same(G.edge_c, T.en[0], 2 * H, H);
  same(G.edge_ab, T.en[0], 0, H, view(P, T.en[0], H), 1);
  same(G.edge_2, T.en[1], 0, H);
  same(G.node_1, T.nn[0], 0, 2 * H);
  same(G.node_2, T.nn[1], 0, H);
  same(G.out_c, T.out[0], 2 * H, H);
  same(G.out_ab, T.out[0], 0, H, view(P, T.out[0], H), 1);
  // single-output layers: weight vectors and the scalar biases (read back to the host)
  hipMemcpyAsync((void*)c->filt_out.w, P + T.filt[L].w, sizeof(float) * c->cfg.filt_hidden, hipMemcpyDeviceToDevice, s);
  hipMemcpyAsync((void*)G.out_2.w, P + T.out[1].w, sizeof(float) * H, hipMemcpyDeviceToDevice, s);
  float b2[2];
  hipMemcpyAsync(&b2[0], P + T.filt[L].b, sizeof(float), hipMemcpyDeviceToHost, s);
  hipMemcpyAsync(&b2[1], P + T.out[1].b, sizeof(float), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) return TRK_E_DEVICE;
  c->filt_out.b = b2[0];
  G.out_2.b = b2[1];
  return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE;
}

namespace {

bool train_ready(trk_ctx* c) { return c && c->train; }

}  // namespace

extern "C" {

int64_t trk_train_param_count(const trk_config* cfg) {
  if (!cfg) return -1;
  return train_param_count(*cfg);
}

int trk_train_set_params(trk_ctx* c, const float* d_params, hipStream_t s) {
  if (!train_ready(c) || !d_params) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  return train_set_params(c, d_params, s);
}

int trk_filter_train_fwd(trk_ctx* c, const float* d_emb, int64_t n, const int32_t* d_src, const int32_t* d_dst,
                         int64_t m, float* d_logits, hipStream_t s) {
  if (!train_ready(c) || n < 0 || n > c->cfg.max_hits || m < 0 || m > c->train->cap_c) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (m > 0 && (!d_emb || !d_src || !d_dst || !d_logits)) return TRK_E_INVAL;
  if (m == 0) return TRK_OK;
  TrainState& T = *c->train;
  const int D = c->cfg.emb_dim, F = c->cfg.filt_hidden, L = c->cfg.filt_layers;
  ew(pair_gather_kernel, m * 2 * D, s, d_emb, D, (int)n, d_src, d_dst, m, T.fx0, 2 * D);
  ActBuf a = T.fx0;
  int lda = 2 * D, K = 2 * D;
  for (int i = 0; i < L; ++i) {
    ActBuf o = T.fact.at((size_t)i * T.cap_c * F);
    rowgemm(a, lda, K, m, T.filtF[i], o, F, F, EPI_BIAS_TANH, nullptr, 0, c->n_cu, s, T.bf16);
    a = o;
    lda = F;
    K = F;
  }
  rowgemm(a, F, F, m, T.filtF[L], d_logits, 1, 1, EPI_BIAS, nullptr, 0, c->n_cu, s, T.bf16);
  return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE;
}

int trk_filter_train_bwd(trk_ctx* c, const float* d_emb, int64_t n, const int32_t* d_src, const int32_t* d_dst,
                         int64_t m, const float* d_dlogits, float* d_grads, hipStream_t s) {
  if (!train_ready(c) || n < 0 || n > c->cfg.max_hits || m < 0 || m > c->train->cap_c || !d_grads) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (m > 0 && (!d_emb || !d_src || !d_dst || !d_dlogits)) return TRK_E_INVAL;
  if (m == 0) return TRK_OK;
  TrainState& T = *c->train;
  const int D = c->cfg.emb_dim, F = c->cfg.filt_hidden, L = c->cfg.filt_layers;
  const ActBuf aL = T.fact.at((size_t)(L - 1) * T.cap_c * F);
  wgrad(T, aL, F, nullptr, nullptr, nullptr, 0, 0, F, true, d_dlogits, 1, 1, m, d_grads + T.filt[L].w, s);
  float* del = T.fdel0;
  float* nxt = T.fdel1;
  ew(outgrad_kernel, m * F, s, d_dlogits, c->filt_out.w, aL, m, F, del);
  for (int i = L - 1; i >= 0; --i) {
    if (i == 0)
      wgrad(T, nullptr, 0, d_src, d_dst, d_emb, D, (int)n, 2 * D, true, del, F, F, m, d_grads + T.filt[0].w, s);
    else
      wgrad(T, T.fact.at((size_t)(i - 1) * T.cap_c * F), F, nullptr, nullptr, nullptr, 0, 0, F, true, del, F, F, m,
            d_grads + T.filt[i].w, s);
    if (i >= 1) {
      rowgemm(del, F, F, m, T.filtT[i], nxt, F, F, EPI_DTANH, T.fact.at((size_t)(i - 1) * T.cap_c * F), F, c->n_cu, s,
              T.bf16);
      std::swap(del, nxt);
    }
  }
  return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE;
}

int trk_gnn_train_fwd(trk_ctx* c, const float* d_x, int64_t n, const int32_t* d_src, const int32_t* d_dst, int64_t m,
                      float* d_logits, hipStream_t s) {
  if (!train_ready(c) || n < 1 || n > c->cfg.max_hits || m < 0 || m > c->train->cap_f || !d_x) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (m > 0 && (!d_src || !d_dst || !d_logits)) return TRK_E_INVAL;
  TrainState& T = *c->train;
  GnnScratch& g = c->gs;
  const int H = c->cfg.gnn_hidden, It = c->cfg.gnn_iters;
  const int nn = (int)n;
  launch_incidence(d_src, d_dst, m, nullptr, nn, g, s);
  PairIn pair;
  pair.P = T.P;
  pair.src = d_src;
  pair.dst = d_dst;
  pair.n = nn;
  rowgemm(d_x, 3, 3, n, T.ne1, T.na1, H, H, EPI_BIAS_TANH, nullptr, 0, c->n_cu, s, T.bf16);
  rowgemm(T.na1, H, H, n, T.ne2, T.hck, H, H, EPI_BIAS_TANH, nullptr, 0, c->n_cu, s, T.bf16);
  ew(pair_gather_kernel, m * 6, s, d_x, 3, nn, d_src, d_dst, m, T.x6, 6);
  rowgemm(T.x6, 6, 6, m, T.ee1, T.ea1, H, H, EPI_BIAS_TANH, nullptr, 0, c->n_cu, s, T.bf16);
  rowgemm(T.ea1, H, H, m, T.ee2, T.eck, H, H, EPI_BIAS_TANH, nullptr, 0, c->n_cu, s, T.bf16);
  for (int t = 1; t <= It; ++t) {
    const ActBuf h = T.hck.at((size_t)(t - 1) * T.nmax * H);
    const ActBuf e = T.eck.at((size_t)(t - 1) * T.cap_f * H);
    const ActBuf h_new = T.hck.at((size_t)t * T.nmax * H);
    const ActBuf e_new = T.eck.at((size_t)t * T.cap_f * H);
    rowgemm(h, H, H, n, T.eab, T.P, 2 * H, 2 * H, EPI_STORE, nullptr, 0, c->n_cu, s, T.bf16);
    rowgemm(e, H, H, m, T.ec, T.t1, H, H, EPI_PAIR_TANH, nullptr, 0, c->n_cu, s, T.bf16, pair);
    rowgemm(T.t1, H, H, m, T.e2, e_new, H, H, EPI_RES_TANH, e, H, c->n_cu, s, T.bf16);
    segsum(e_new, H, g.rowptr, g.rowidx, g.cscptr, g.cscidx, nn, T.msg, H, s);
    ew(concat_kernel, n * 2 * H, s, h, T.msg, n, H, T.nin);
    rowgemm(T.nin, 2 * H, 2 * H, n, T.n1, T.q1, H, H, EPI_BIAS_TANH, nullptr, 0, c->n_cu, s, T.bf16);
    rowgemm(T.q1, H, H, n, T.n2, h_new, H, H, EPI_RES_TANH, h, H, c->n_cu, s, T.bf16);
  }
  const ActBuf hT = T.hck.at((size_t)It * T.nmax * H);
  const ActBuf eT = T.eck.at((size_t)It * T.cap_f * H);
  rowgemm(hT, H, H, n, T.oab, T.P, 2 * H, 2 * H, EPI_STORE, nullptr, 0, c->n_cu, s, T.bf16);
  if (m > 0) {
    rowgemm(eT, H, H, m, T.oc, T.u, H, H, EPI_PAIR_TANH, nullptr, 0, c->n_cu, s, T.bf16, pair);
    rowgemm(T.u, H, H, m, T.o2, d_logits, 1, 1, EPI_BIAS, nullptr, 0, c->n_cu, s, T.bf16);
  }
  return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE;
}

int trk_gnn_train_bwd(trk_ctx* c, const float* d_x, int64_t n, const int32_t* d_src, const int32_t* d_dst, int64_t m,
                      const float* d_dlogits, float* d_grads, hipStream_t s) {
  if (!train_ready(c) || n < 1 || n > c->cfg.max_hits || m < 0 || m > c->train->cap_f || !d_x || !d_grads)
    return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (m > 0 && (!d_src || !d_dst || !d_dlogits)) return TRK_E_INVAL;
  TrainState& T = *c->train;
  GnnScratch& g = c->gs;
  const int H = c->cfg.gnn_hidden, It = c->cfg.gnn_iters;
  const int nn = (int)n;
  float* G = d_grads;
  const ActBuf hT = T.hck.at((size_t)It * T.nmax * H);
  const ActBuf eT = T.eck.at((size_t)It * T.cap_f * H);
  PairIn pair;
  pair.P = T.P;
  pair.src = d_src;
  pair.dst = d_dst;
  pair.n = nn;
  // output head
  wgrad(T, T.u, H, nullptr, nullptr, nullptr, 0, 0, H, true, d_dlogits, 1, 1, m, G + T.out[1].w, s);
  float* du = T.dpre1;
  ew(outgrad_kernel, m * H, s, d_dlogits, c->gnn.out_2.w, T.u, m, H, du);
  segsum(du, H, g.rowptr, g.rowidx, nullptr, nullptr, nn, T.dP, 2 * H, s);
  segsum(du, H, g.cscptr, g.cscidx, nullptr, nullptr, nn, T.dP + H, 2 * H, s);
  wgrad(T, hT, H, nullptr, nullptr, nullptr, 0, 0, H, false, T.dP, 2 * H, H, n, G + T.out[0].w, s);
  wgrad(T, hT, H, nullptr, nullptr, nullptr, 0, 0, H, false, T.dP + H, 2 * H, H, n, G + T.out[0].w + (size_t)H * H, s);
  wgrad(T, eT, H, nullptr, nullptr, nullptr, 0, 0, H, true, du, H, H, m, G + T.out[0].w + (size_t)2 * H * H, s);
  float* dh = T.dh;
  float* dh2 = T.dh2;
  rowgemm(T.dP, 2 * H, 2 * H, n, T.oabT, dh, H, H, EPI_STORE, nullptr, 0, c->n_cu, s, T.bf16);
  rowgemm(du, H, H, m, T.ocT, T.de, H, H, EPI_STORE, nullptr, 0, c->n_cu, s, T.bf16);
  for (int t = It; t >= 1; --t) {
    const ActBuf h = T.hck.at((size_t)(t - 1) * T.nmax * H);
    const ActBuf e = T.eck.at((size_t)(t - 1) * T.cap_f * H);
    const ActBuf e_new = T.eck.at((size_t)t * T.cap_f * H);
    // recompute this iteration's internals from (h^{t-1}, e^{t-1})
    rowgemm(h, H, H, n, T.eab, T.P, 2 * H, 2 * H, EPI_STORE, nullptr, 0, c->n_cu, s, T.bf16);
    rowgemm(e, H, H, m, T.ec, T.t1, H, H, EPI_PAIR_TANH, nullptr, 0, c->n_cu, s, T.bf16, pair);
    rowgemm(T.t1, H, H, m, T.e2, T.v, H, H, EPI_BIAS_TANH, nullptr, 0, c->n_cu, s, T.bf16);
    segsum(e_new, H, g.rowptr, g.rowidx, g.cscptr, g.cscidx, nn, T.msg, H, s);
    ew(concat_kernel, n * 2 * H, s, h, T.msg, n, H, T.nin);
    rowgemm(T.nin, 2 * H, 2 * H, n, T.n1, T.q1, H, H, EPI_BIAS_TANH, nullptr, 0, c->n_cu, s, T.bf16);
    rowgemm(T.q1, H, H, n, T.n2, T.q2, H, H, EPI_BIAS_TANH, nullptr, 0, c->n_cu, s, T.bf16);
    // node update h^t = h + phi_v([h, msg])
    ew(dtanh_kernel, n * H, s, dh, T.q2, n * H, T.dq);
    wgrad(T, T.q1, H, nullptr, nullptr, nullptr, 0, 0, H, true, T.dq, H, H, n, G + T.nn[1].w, s);
    rowgemm(T.dq, H, H, n, T.n2T, T.dq1, H, H, EPI_DTANH, T.q1, H, c->n_cu, s, T.bf16);
    wgrad(T, T.nin, 2 * H, nullptr, nullptr, nullptr, 0, 0, 2 * H, true, T.dq1, H, H, n, G + T.nn[0].w, s);
    rowgemm(T.dq1, H, H, n, T.n1T, T.dnin, 2 * H, 2 * H, EPI_STORE, nullptr, 0, c->n_cu, s, T.bf16);
    ew(add_cols_kernel, n * H, s, dh, T.dnin, 2 * H, n, H, dh2);
    // messages: de^t += dmsg[src] + dmsg[dst]
    if (m > 0) ew(gather_add_kernel, m * H, s, T.dnin + H, 2 * H, d_src, d_dst, nn, m, H, T.de);
    // edge update e^t = e + phi_e([h_s, h_t, e])
    ew(dtanh_kernel, m * H, s, T.de, T.v, m * H, T.dpre);
    wgrad(T, T.t1, H, nullptr, nullptr, nullptr, 0, 0, H, true, T.dpre, H, H, m, G + T.en[1].w, s);
    rowgemm(T.dpre, H, H, m, T.e2T, T.dpre1, H, H, EPI_DTANH, T.t1, H, c->n_cu, s, T.bf16);
    wgrad(T, e, H, nullptr, nullptr, nullptr, 0, 0, H, true, T.dpre1, H, H, m, G + T.en[0].w + (size_t)2 * H * H, s);
    segsum(T.dpre1, H, g.rowptr, g.rowidx, nullptr, nullptr, nn, T.dP, 2 * H, s);
    segsum(T.dpre1, H, g.cscptr, g.cscidx, nullptr, nullptr, nn, T.dP + H, 2 * H, s);
    wgrad(T, h, H, nullptr, nullptr, nullptr, 0, 0, H, false, T.dP, 2 * H, H, n, G + T.en[0].w, s);
    wgrad(T, h, H, nullptr, nullptr, nullptr, 0, 0, H, false, T.dP + H, 2 * H, H, n, G + T.en[0].w + (size_t)H * H, s);
    rowgemm(T.dpre1, H, H, m, T.ecT, T.de, H, H, EPI_ACC, nullptr, 0, c->n_cu, s, T.bf16);
    rowgemm(T.dP, 2 * H, 2 * H, n, T.eabT, dh2, H, H, EPI_ACC, nullptr, 0, c->n_cu, s, T.bf16);
    std::swap(dh, dh2);
  }
  // encoders
  if (m > 0) {
    ew(dtanh_kernel, m * H, s, T.de, T.eck, m * H, T.dpre);
    wgrad(T, T.ea1, H, nullptr, nullptr, nullptr, 0, 0, H, true, T.dpre, H, H, m, G + T.ee[1].w, s);
    rowgemm(T.dpre, H, H, m, T.ee2T, T.dpre1, H, H, EPI_DTANH, T.ea1, H, c->n_cu, s, T.bf16);
    wgrad(T, T.x6, 6, nullptr, nullptr, nullptr, 0, 0, 6, true, T.dpre1, H, H, m, G + T.ee[0].w, s);
  }
  ew(dtanh_kernel, n * H, s, dh, T.hck, n * H, T.dq);
  wgrad(T, T.na1, H, nullptr, nullptr, nullptr, 0, 0, H, true, T.dq, H, H, n, G + T.ne[1].w, s);
  rowgemm(T.dq, H, H, n, T.ne2T, T.dq1, H, H, EPI_DTANH, T.na1, H, c->n_cu, s, T.bf16);
  wgrad(T, d_x, 3, nullptr, nullptr, nullptr, 0, 0, 3, true, T.dq1, H, H, n, G + T.ne[0].w, s);
  return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE;
}

int trk_embed_train_fwd(trk_ctx* c, const float* d_x, int64_t n, float* d_emb, hipStream_t s) {
  if (!train_ready(c) || n < 0 || n > c->cfg.max_hits || (n > 0 && (!d_x || !d_emb))) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (n == 0) return TRK_OK;
  TrainState& T = *c->train;
  const int EL = c->cfg.emb_layers, EW = c->cfg.emb_hidden, D = c->cfg.emb_dim;
  ActBuf a = d_x;
  int lda = 3, K = 3;
  for (int i = 0; i < EL; ++i) {
    ActBuf o = T.eact.at((size_t)i * T.nmax * EW);
    rowgemm(a, lda, K, n, T.embF[i], o, EW, EW, EPI_BIAS_TANH, nullptr, 0, c->n_cu, s, T.bf16);
    a = o;
    lda = EW;
    K = EW;
  }
  rowgemm(a, EW, EW, n, T.embF[EL], d_emb, D, D, EPI_BIAS, nullptr, 0, c->n_cu, s, T.bf16);
  return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE;
}

int trk_embed_train_bwd(trk_ctx* c, const float* d_x, int64_t n, const float* d_demb, float* d_grads, hipStream_t s) {
  if (!train_ready(c) || n < 0 || n > c->cfg.max_hits || !d_grads || (n > 0 && (!d_x || !d_demb))) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (n == 0) return TRK_OK;
  TrainState& T = *c->train;
  const int EL = c->cfg.emb_layers, EW = c->cfg.emb_hidden, D = c->cfg.emb_dim;
  auto act = [&](int i) { return T.eact.at((size_t)(i - 1) * T.nmax * EW); };   // a_i, i = 1..EL
  // output layer: emb = a_EL W + b (linear)
  wgrad(T, act(EL), EW, nullptr, nullptr, nullptr, 0, 0, EW, true, d_demb, D, D, n, d_grads + T.emb[EL].w, s);
  float* del = T.edel0;
  float* nxt = T.edel1;
  rowgemm(d_demb, D, D, n, T.embT[EL], del, EW, EW, EPI_DTANH, act(EL), EW, c->n_cu, s, T.bf16);
  for (int i = EL - 1; i >= 0; --i) {
    if (i == 0)
      wgrad(T, d_x, 3, nullptr, nullptr, nullptr, 0, 0, 3, true, del, EW, EW, n, d_grads + T.emb[0].w, s);
    else
      wgrad(T, act(i), EW, nullptr, nullptr, nullptr, 0, 0, EW, true, del, EW, EW, n, d_grads + T.emb[i].w, s);
    if (i >= 1) {
      rowgemm(del, EW, EW, n, T.embT[i], nxt, EW, EW, EPI_DTANH, act(i), EW, c->n_cu, s, T.bf16);
      std::swap(del, nxt);
    }
  }
  return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE;
}

int trk_pair_loss(trk_ctx* c, const float* d_emb, int64_t n, const int32_t* d_pa, const int32_t* d_pb,
                  const float* d_y, int64_t npairs, float margin, float neg_weight, float* d_demb, float* h_loss,
                  hipStream_t s) {
  if (!train_ready(c) || n < 1 || n > c->cfg.max_hits || npairs < 0 || npairs > c->train->cap_c || !d_emb || !d_demb)
    return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (npairs > 0 && (!d_pa || !d_pb || !d_y)) return TRK_E_INVAL;
  if (!(neg_weight >= 0.f) || !(margin >= 0.f)) return TRK_E_INVAL;
  TrainState& T = *c->train;
  const int D = c->cfg.emb_dim;
  const int nn = (int)n;
  if (h_loss) *h_loss = 0.f;
  if (npairs == 0) {
    launch_fill_int((int*)d_demb, 0, n * D, s);
    return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE;
  }
  const int nb = blocks_for(npairs, 256, 4096);
  pair_count_kernel<<<nb, 256, 0, s>>>(d_y, npairs, (int*)T.bce_part);
  pair_count_sum_kernel<<<1, 64, 0, s>>>((const int*)T.bce_part, nb, npairs, T.pcounts);
  pair_grad_kernel<<<nb, 256, 0, s>>>(d_emb, D, nn, d_pa, d_pb, d_y, npairs, margin, neg_weight, T.pcounts, T.pg,
                                         T.bce_part + 4096);
  bce_sum_kernel<<<1, 64, 0, s>>>(T.bce_part + 4096, nb, 1, T.bce_part + 12288);
  // node gradient: + sum over pairs where the node comes first, - sum where it comes second
  launch_incidence(d_pa, d_pb, npairs, nullptr, nn, T.pairs, s);
  segsum(T.pg, D, T.pairs.rowptr, T.pairs.rowidx, T.pairs.cscptr, T.pairs.cscidx, nn, d_demb, D, s, -1.f);
  if (h_loss) {
    if (hipMemcpyAsync(h_loss, T.bce_part + 12288, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess)
      return TRK_E_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return TRK_E_DEVICE;
  }
  return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE;
}

int trk_bce_with_logits(trk_ctx* c, const float* d_logits, const float* d_targets, int64_t m, float* d_dlogits,
                        float* h_loss, hipStream_t s) {
  if (!train_ready(c) || m < 0 || (m > 0 && (!d_logits || !d_targets || !d_dlogits))) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (h_loss) *h_loss = 0.f;
  if (m == 0) return TRK_OK;
  TrainState& T = *c->train;
  const int nb = blocks_for(m, 256, 4096);
  bce_kernel<<<nb, 256, 0, s>>>(d_logits, d_targets, m, d_dlogits, T.bce_part);
  bce_sum_kernel<<<1, 64, 0, s>>>(T.bce_part, nb, m, T.bce_part + 4096);
  if (h_loss) {
    if (hipMemcpyAsync(h_loss, T.bce_part + 4096, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess)
      return TRK_E_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return TRK_E_DEVICE;
  }
  return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE;
}

int trk_adam_update(trk_ctx* c, float* d_params, const float* d_grads, float* d_m, float* d_v, int64_t count, float lr,
                    float beta1, float beta2, float eps, int64_t step, hipStream_t s) {
  if (!c || count < 0 || step < 1 || (count > 0 && (!d_params || !d_grads || !d_m || !d_v))) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  if (count > 0) ew(adam_kernel, count, s, d_params, d_grads, d_m, d_v, count, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE;
}

}  // extern "C"
