// Fused row-tile MLP kernels: embedding over spacepoints and the edge filter
// (Section 2.2.2: the embedding MLP maps the three spacepoint features into the
// latent space; the filter MLP scores each candidate edge from the embeddings of
// its two ends).  A workgroup owns a tile of MT rows; every layer of the network
// runs on that tile with the activations resident in LDS, so hidden activations
// never travel to HBM.  Each wave owns a slab of output columns of every layer.
// Tiles are walked by a persistent grid whose row count may be read from device
// memory, so a kernel can be chained behind one that produced its row count.
// P is the precision of the square hidden layers (and of the embedding's output
// layer); P0 that of the narrow first layer (K = 3 or 2 * emb_dim), which is the
// same except in FP8 mode, where the first layer runs in BF16 because an FP8
// product consumes k in blocks of 128, and in split-BF16 mode, where it runs in
// FP32 (one k block either way).
#include "kernels.h"
#include "mfma_tile.h"
#include <stdlib.h>

namespace {

constexpr int KIN_MAX = 32;  // widest first-layer input: [emb_s, emb_t] with emb_dim <= 16

template <class P, class P0, int W, int MT, int NW>
struct MlpShape {
  typedef typename P::act_t T;
  typedef typename P0::act_t T0;
  static constexpr int LD = W + P::PAD;              // activation row stride (elements)
  static constexpr int LDI = KIN_MAX + P0::PAD;      // input row stride
  static constexpr int MTW = MT / 16;                // m-tiles per wave (all rows)
  static constexpr int NTW = W / 16 / NW;            // n-tiles per wave
  static constexpr int ACT_BYTES = MT * LD * (int)sizeof(T);
  static constexpr int RED_BYTES = NW * MT * 16 * 4;
  static constexpr int BUF_BYTES = ACT_BYTES > RED_BYTES ? ACT_BYTES : RED_BYTES;
  static_assert(NTW >= 1 && W % (16 * NW) == 0, "columns must split evenly over waves");
  static_assert(W % P::KB == 0, "hidden width must be a whole number of k blocks");
  static_assert(BUF_BYTES + MT * LDI * (int)sizeof(T0) <= 160 * 1024, "LDS budget");
};

// Embedding: emb[i][0..D) = L_out(tanh(... tanh(L_in(x_i)))).
template <class P, class P0, int W, int MT, int NW>
__global__ __launch_bounds__(NW * 64) void embed_kernel(const float* __restrict__ x, int n, DevLayer l_in,
                                                        LayerList hid, DevLayer l_out, int D,
                                                        float* __restrict__ emb) {
  typedef MlpShape<P, P0, W, MT, NW> S;
  typedef typename S::T T;
  typedef typename S::T0 T0;
  __shared__ __align__(16) unsigned char buf[S::BUF_BYTES];
  __shared__ __align__(16) T0 xin[MT * S::LDI];
  T* act = (T*)buf;
  float* red = (float*)buf;
  const int wave = threadIdx.x >> 6;
  const int l = lane_id(), g = l >> 4, r = l & 15;
  const int nt0 = wave * S::NTW;
  const int ntiles = (n + MT - 1) / MT;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int row0 = t * MT;
    for (int idx = threadIdx.x; idx < MT * P0::KB; idx += blockDim.x) {
      const int m = idx / P0::KB, k = idx - m * P0::KB;
      const float v = (k < 3 && row0 + m < n) ? x[(size_t)(row0 + m) * 3 + k] : 0.f;
      xin[m * S::LDI + k] = P0::cvt(v);
    }
    __syncthreads();
    f32x4 acc[S::MTW][S::NTW];
        tile_gemm<P0, S::MTW, S::NTW, true>(acc, xin, S::LDI, l_in.w, l_in.nkb, nt0, 0, l_in.nkb);
    tile_store_tanh<P>(acc, l_in.bs, l_in.dq, act, S::LD, nt0);
    __syncthreads();
    // BF16: the output layer reads the last hidden layer's FP32 tanh values straight
    // from the registers (FP32 products, weights in FP32 fragments), not the BF16 tile
    const bool fold = std::is_same<P, PrecBF16>::value && hid.n > 0;
    const int nfull = fold ? hid.n - 1 : hid.n;
    for (int h = 0; h < nfull; ++h) {
      tile_gemm<P, S::MTW, S::NTW, true>(acc, act, S::LD, hid.l[h].w, hid.l[h].nkb, nt0, 0, hid.l[h].nkb);
      __syncthreads();
      tile_store_tanh<P>(acc, hid.l[h].bs, hid.l[h].dq, act, S::LD, nt0);
      __syncthreads();
    }
    if (fold) {
      // The last hidden layer in two halves of each wave's columns (registers for one
      // half at a time).  Lane (g, r) holds h[16 i + r][16 J + 4 g + c] (J = the 16-column
      // block): for each c these are the second operand of an FP32 product over the k
      // chunk {16 J + 4 g' + c}, whose first operand, W_out[16 J + 4 g + c][r], is
      // component c of the FP32 fragment of k block J.
      const DevLayer& L = hid.l[hid.n - 1];
      const float sc = L.dq * TRK_2LOG2E;
      constexpr int NH = S::NTW / 2 > 0 ? S::NTW / 2 : 1;
      f32x4 o[S::MTW];
#pragma unroll
      for (int i = 0; i < S::MTW; ++i) o[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
      for (int half = 0; half * NH < S::NTW; ++half) {
        f32x4 ah[S::MTW][NH];
        tile_gemm<P, S::MTW, NH, true>(ah, act, S::LD, L.w, L.nkb, nt0 + half * NH, 0, L.nkb);
#pragma unroll
        for (int j = 0; j < NH; ++j) {
          const int J = nt0 + half * NH + j;
          const uint4 wf = l_out.w[(size_t)J * 64 + l];
          const float4 b = *(const float4*)(L.bs + J * 16 + 4 * g);
#pragma unroll
          for (int i = 0; i < S::MTW; ++i) {
            o[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(wf.x), trk_tanh_log2(fmaf(ah[i][j][0], sc, b.x)),
                                                        o[i], 0, 0, 0);
            o[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(wf.y), trk_tanh_log2(fmaf(ah[i][j][1], sc, b.y)),
                                                        o[i], 0, 0, 0);
            o[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(wf.z), trk_tanh_log2(fmaf(ah[i][j][2], sc, b.z)),
                                                        o[i], 0, 0, 0);
            o[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(wf.w), trk_tanh_log2(fmaf(ah[i][j][3], sc, b.w)),
                                                        o[i], 0, 0, 0);
          }
        }
      }
      __syncthreads();   // every wave has read the LDS tile the reduction buffer overlays
#pragma unroll
      for (int i = 0; i < S::MTW; ++i)
        *(float4*)(red + ((wave * MT + i * 16 + r) * 16 + 4 * g)) = make_float4(o[i][0], o[i][1], o[i][2], o[i][3]);
    }
    if (!fold) {
      // output layer: a single 16-column tile, its k range split over the waves
      f32x4 o[S::MTW][1];
      acc_zero(o);
      const int per = (l_out.nkb + NW - 1) / NW;
      const int kb0 = wave * per;
      const int run = min(per, l_out.nkb - kb0);
      tile_gemm<P, S::MTW, 1>(o, act, S::LD, l_out.w, l_out.nkb, 0, kb0, run);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < S::MTW; ++i)
        *(float4*)(red + ((wave * MT + i * 16 + r) * 16 + 4 * g)) =
            make_float4(o[i][0][0], o[i][0][1], o[i][0][2], o[i][0][3]);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < MT * D; idx += blockDim.x) {
      const int m = idx / D, c = idx - m * D;
      float s = 0.f;
      for (int w = 0; w < NW; ++w) s += red[(w * MT + m) * 16 + c];
      if (row0 + m < n) emb[(size_t)(row0 + m) * D + c] = fmaf(s, l_out.dq, l_out.b[c]);
    }
    __syncthreads();
  }
}

// Filter: scores[e] = sigmoid(out . tanh(L_last(... tanh(L_in([emb_src, emb_dst]))))).
// GPF: the next tile's gathered inputs are requested during the last layer's epilogue
// (edge ends first, under the epilogue's arithmetic; then the embedding values), so
// that the tile start does not wait for two dependent round trips to memory.
// A BF16 first layer (P0 = PrecBF16) reads the pair's FP32 mean and difference,
// [(e_s + e_t) / 2, e_s - e_t], rounded to BF16, with its weights stored for that form
// ([W_s + W_t; (W_s - W_t) / 2], the same function): the two ends of a candidate edge
// lie close together, and rounding each to BF16 before their difference is taken
// would lose that difference, which carries the edge's signal, to the rounding of
// the much larger coordinates.
template <class P, class P0, int W, int MT, int NW, bool GPF = false>
__global__ __launch_bounds__(NW * 64) void filter_kernel(const float* __restrict__ emb, int D,
                                                         const int* __restrict__ src, const int* __restrict__ dst,
                                                         int64_t m_host, const int* __restrict__ d_m, int64_t cap,
                                                         DevLayer l_in, LayerList hid, DevVec out,
                                                         float* __restrict__ scores, int n_nodes, int* d_err) {
  typedef MlpShape<P, P0, W, MT, NW> S;
  typedef typename S::T T;
  typedef typename S::T0 T0;
  __shared__ __align__(16) unsigned char buf[S::BUF_BYTES];
  __shared__ __align__(16) T0 xin[MT * S::LDI];
  __shared__ float zred[NW * MT];
  T* act = (T*)buf;
  const int wave = threadIdx.x >> 6;
  const int l = lane_id(), g = l >> 4, r = l & 15;
  const int nt0 = wave * S::NTW;
  const int64_t m = d_m ? clamp_count(d_m, cap) : m_host;
  const int64_t ntiles = (m + MT - 1) / MT;
  const int nlayers = 1 + hid.n;
  const int kin = 2 * D;
  const int kin_pad = l_in.nkb * P0::KB;
  constexpr bool MD = std::is_same<P0, PrecBF16>::value;
  // the gathered inputs held in registers between tiles (GPF): this thread's entries
  // idx = threadIdx.x + i * blockDim.x of the MT x kin_pad input tile (MD: of the
  // MT x D pairs of the two ends' values)
  constexpr int GI = (MT * (MD ? KIN_MAX / 2 : KIN_MAX) + NW * 64 - 1) / (NW * 64);
  int gnd[GI], gnd2[GI];
  bool gok[GI];
  float gv[GI], gv2[GI];
  auto gather_ends = [&](int64_t r0) {
#pragma unroll
    for (int i = 0; i < GI; ++i) {
      const int idx = threadIdx.x + i * NW * 64;
      if constexpr (MD) {
        const int mm = idx / D;
        const int64_t e = r0 + mm;
        gok[i] = idx < MT * D && e < m;
        gnd[i] = gok[i] ? src[e] : 0;
        gnd2[i] = gok[i] ? dst[e] : 0;
      } else {
        const int mm = idx / kin_pad, k = idx - mm * kin_pad;
        const int64_t e = r0 + mm;
        gok[i] = idx < MT * kin_pad && e < m && k < kin;
        gnd[i] = gok[i] ? ((k < D) ? src[e] : dst[e]) : 0;
      }
    }
  };
  auto gather_values = [&]() {
#pragma unroll
    for (int i = 0; i < GI; ++i) {
      const int idx = threadIdx.x + i * NW * 64;
      gv[i] = gv2[i] = 0.f;
      if constexpr (MD) {
        const int k = idx % D;
        if (gok[i]) {
          if ((unsigned)gnd[i] < (unsigned)n_nodes && (unsigned)gnd2[i] < (unsigned)n_nodes) {
            gv[i] = emb[(size_t)gnd[i] * D + k];
            gv2[i] = emb[(size_t)gnd2[i] * D + k];
          } else if (d_err) {
            atomicOr(d_err, TRK_ERRBIT_INDEX);
          }
        }
      } else {
        const int k = idx % kin_pad;
        if (gok[i]) {
          if ((unsigned)gnd[i] < (unsigned)n_nodes) gv[i] = emb[(size_t)gnd[i] * D + (k < D ? k : k - D)];
          else if (d_err) atomicOr(d_err, TRK_ERRBIT_INDEX);
        }
      }
    }
  };
  if constexpr (MD) {
    // the padding columns [2D, kin_pad) of the input tile stay zero
    for (int idx = threadIdx.x; idx < MT * (kin_pad - kin); idx += blockDim.x) {
      const int mm = idx / (kin_pad - kin), c = idx - mm * (kin_pad - kin);
      xin[mm * S::LDI + kin + c] = P0::cvt(0.f);
    }
  }
  if (GPF && (int64_t)blockIdx.x < ntiles) {
    gather_ends((int64_t)blockIdx.x * MT);
    gather_values();
  }
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t row0 = t * MT;
    if constexpr (GPF && MD) {
#pragma unroll
      for (int i = 0; i < GI; ++i) {
        const int idx = threadIdx.x + i * NW * 64;
        const int mm = idx / D, k = idx - mm * D;
        if (idx < MT * D) {
          xin[mm * S::LDI + k] = P0::cvt(0.5f * (gv[i] + gv2[i]));
          xin[mm * S::LDI + D + k] = P0::cvt(gv[i] - gv2[i]);
        }
      }
    } else if constexpr (GPF) {
#pragma unroll
      for (int i = 0; i < GI; ++i) {
        const int idx = threadIdx.x + i * NW * 64;
        const int mm = idx / kin_pad, k = idx - mm * kin_pad;
        if (idx < MT * kin_pad) xin[mm * S::LDI + k] = P0::cvt(gv[i]);
      }
    } else if constexpr (MD) {
      for (int idx = threadIdx.x; idx < MT * D; idx += blockDim.x) {
        const int mm = idx / D, k = idx - mm * D;
        const int64_t e = row0 + mm;
        float a = 0.f, b = 0.f;
        if (e < m) {
          const int sn = src[e], tn = dst[e];
          if ((unsigned)sn < (unsigned)n_nodes && (unsigned)tn < (unsigned)n_nodes) {
            a = emb[(size_t)sn * D + k];
            b = emb[(size_t)tn * D + k];
          } else if (d_err) {
            atomicOr(d_err, TRK_ERRBIT_INDEX);
          }
        }
        xin[mm * S::LDI + k] = P0::cvt(0.5f * (a + b));
        xin[mm * S::LDI + D + k] = P0::cvt(a - b);
      }
    } else {
      for (int idx = threadIdx.x; idx < MT * kin_pad; idx += blockDim.x) {
        const int mm = idx / kin_pad, k = idx - mm * kin_pad;
        const int64_t e = row0 + mm;
        float v = 0.f;
        if (e < m && k < kin) {
          const int node = (k < D) ? src[e] : dst[e];
          if ((unsigned)node < (unsigned)n_nodes) v = emb[(size_t)node * D + (k < D ? k : k - D)];
          else if (d_err) atomicOr(d_err, TRK_ERRBIT_INDEX);
        }
        xin[mm * S::LDI + k] = P0::cvt(v);
      }
    }
    __syncthreads();
    for (int layer = 0; layer < nlayers; ++layer) {
      const DevLayer& L = layer == 0 ? l_in : hid.l[layer - 1];
      f32x4 acc[S::MTW][S::NTW];
      if (layer == 0)
        tile_gemm<P0, S::MTW, S::NTW, true>(acc, xin, S::LDI, L.w, L.nkb, nt0, 0, L.nkb);
      else
        tile_gemm<P, S::MTW, S::NTW, true>(acc, act, S::LD, L.w, L.nkb, nt0, 0, L.nkb);
      if (layer + 1 < nlayers) {
        if (layer > 0) __syncthreads();
        tile_store_tanh<P>(acc, L.bs, L.dq, act, S::LD, nt0);
        __syncthreads();
      } else {
        // last hidden layer: fold the single-output layer into the epilogue
        float part[S::MTW];
        const float sc = L.dq * TRK_2LOG2E;
#pragma unroll
        for (int i = 0; i < S::MTW; ++i) part[i] = 0.f;
        float4 bq[S::NTW], wq[S::NTW];
#pragma unroll
        for (int j = 0; j < S::NTW; ++j) {
          const int n = (nt0 + j) * 16 + 4 * g;
          bq[j] = *(const float4*)(L.bs + n);
          wq[j] = *(const float4*)(out.w + n);
        }
        // the next tile's edge ends, requested after every load this epilogue waits for
        if constexpr (GPF) gather_ends(row0 + (int64_t)gridDim.x * MT);
#pragma unroll
        for (int j = 0; j < S::NTW; ++j) {
          const float4 b = bq[j];
          const float4 w = wq[j];
#pragma unroll
          for (int i = 0; i < S::MTW; ++i) {
            const f32x4 a = acc[i][j];
            part[i] += trk_tanh_log2(fmaf(a[0], sc, b.x)) * w.x + trk_tanh_log2(fmaf(a[1], sc, b.y)) * w.y +
                       trk_tanh_log2(fmaf(a[2], sc, b.z)) * w.z + trk_tanh_log2(fmaf(a[3], sc, b.w)) * w.w;
          }
        }
#pragma unroll
        for (int i = 0; i < S::MTW; ++i) {
          part[i] += __shfl_xor(part[i], 16, 64);
          part[i] += __shfl_xor(part[i], 32, 64);
          if (g == 0) zred[wave * MT + i * 16 + r] = part[i];
        }
        __syncthreads();
        if constexpr (GPF) gather_values();
        for (int mm = threadIdx.x; mm < MT; mm += blockDim.x) {
          float z = out.b;
          for (int w = 0; w < NW; ++w) z += zred[w * MT + mm];
          if (row0 + mm < m) scores[row0 + mm] = trk_sigmoid(z);
        }
        __syncthreads();
      }
    }
  }
}

template <class P, class P0, int W, int MT, int NW>
void launch_embed_t(const float* x, int n, const DevLayer& l_in, const LayerList& hid, const DevLayer& l_out,
                    int D, float* emb, int max_grid, hipStream_t s) {
  const int ntiles = (n + MT - 1) / MT;
  const int grid = ntiles < max_grid ? ntiles : max_grid;
  if (grid <= 0) return;
  embed_kernel<P, P0, W, MT, NW><<<grid, NW * 64, 0, s>>>(x, n, l_in, hid, l_out, D, emb);
}

template <class P, class P0, int W, int MT, int NW, bool GPF = false>
void launch_filter_t(const float* emb, int D, const int* src, const int* dst, int64_t m_host, const int* d_m,
                     int64_t cap, const DevLayer& l_in, const LayerList& hid, const DevVec& out, float* scores,
                     int n_nodes, int* d_err, int max_grid, hipStream_t s) {
  const int64_t m = d_m ? cap : m_host;
  const int64_t ntiles = (m + MT - 1) / MT;
  const int grid = (int)(ntiles < max_grid ? ntiles : max_grid);
  if (grid <= 0) return;
  filter_kernel<P, P0, W, MT, NW, GPF><<<grid, NW * 64, 0, s>>>(emb, D, src, dst, m_host, d_m, cap, l_in, hid, out, scores, n_nodes, d_err);
}

}  // namespace

// One tile shape per precision and width: eight-wave workgroups (one per CU) on 32
// rows (FP32, split BF16, FP8) or 64 rows (BF16) at the full width, four waves on 64
// rows at the tiny width.  Any other width is refused.
int launch_embed(int prec, int W, const float* x, int n, const DevLayer& l_in, const LayerList& hid,
                 const DevLayer& l_out, int D, float* emb, int n_cu, hipStream_t s) {
  if (prec == TRK_PREC_F32) {
    if (W == 1024) { launch_embed_t<PrecF32, PrecF32, 1024, 32, 8>(x, n, l_in, hid, l_out, D, emb, n_cu, s); return 0; }
    if (W == 64) { launch_embed_t<PrecF32, PrecF32, 64, 64, 4>(x, n, l_in, hid, l_out, D, emb, n_cu * 4, s); return 0; }
  } else if (prec == TRK_PREC_X3) {
    if (W == 1024) { launch_embed_t<PrecX3, PrecF32, 1024, 32, 8>(x, n, l_in, hid, l_out, D, emb, n_cu, s); return 0; }
    if (W == 64) { launch_embed_t<PrecX3, PrecF32, 64, 64, 4>(x, n, l_in, hid, l_out, D, emb, n_cu * 4, s); return 0; }
  } else if (prec == TRK_PREC_FP8) {
    if (W == 1024) { launch_embed_t<PrecFP8, PrecBF16, 1024, 32, 8>(x, n, l_in, hid, l_out, D, emb, n_cu, s); return 0; }
  } else {
    if (W == 1024) { launch_embed_t<PrecBF16, PrecBF16, 1024, 64, 8>(x, n, l_in, hid, l_out, D, emb, n_cu, s); return 0; }
    if (W == 64) { launch_embed_t<PrecBF16, PrecBF16, 64, 64, 4>(x, n, l_in, hid, l_out, D, emb, n_cu * 4, s); return 0; }
  }
  return -1;
}

// The FP32, split-BF16 and FP8 filters at the full width run 64-edge tiles on eight
// waves and request the next tile's gathered inputs during their last epilogue; the
// BF16 filter runs 128-edge tiles (no registers are left for that prefetch).
int launch_filter(int prec, int W, const float* emb, int D, const int* src, const int* dst, int64_t m_host,
                  const int* d_m, int64_t cap, const DevLayer& l_in, const LayerList& hid, const DevVec& out,
                  float* scores, int n_nodes, int* d_err, int n_cu, hipStream_t s) {
  if (prec == TRK_PREC_F32) {
    if (W == 512) { launch_filter_t<PrecF32, PrecF32, 512, 64, 8, true>(emb, D, src, dst, m_host, d_m, cap, l_in, hid, out, scores, n_nodes, d_err, n_cu, s); return 0; }
    if (W == 64) { launch_filter_t<PrecF32, PrecF32, 64, 64, 4>(emb, D, src, dst, m_host, d_m, cap, l_in, hid, out, scores, n_nodes, d_err, n_cu * 4, s); return 0; }
  } else if (prec == TRK_PREC_X3) {
    if (W == 512) { launch_filter_t<PrecX3, PrecF32, 512, 64, 8, true>(emb, D, src, dst, m_host, d_m, cap, l_in, hid, out, scores, n_nodes, d_err, n_cu, s); return 0; }
    if (W == 64) { launch_filter_t<PrecX3, PrecF32, 64, 64, 4>(emb, D, src, dst, m_host, d_m, cap, l_in, hid, out, scores, n_nodes, d_err, n_cu * 4, s); return 0; }
  } else if (prec == TRK_PREC_FP8) {
    if (W == 512) { launch_filter_t<PrecFP8, PrecBF16, 512, 64, 8, true>(emb, D, src, dst, m_host, d_m, cap, l_in, hid, out, scores, n_nodes, d_err, n_cu, s); return 0; }
  } else {
    if (W == 512) { launch_filter_t<PrecBF16, PrecBF16, 512, 128, 8>(emb, D, src, dst, m_host, d_m, cap, l_in, hid, out, scores, n_nodes, d_err, n_cu, s); return 0; }
    if (W == 64) { launch_filter_t<PrecBF16, PrecBF16, 64, 64, 4>(emb, D, src, dst, m_host, d_m, cap, l_in, hid, out, scores, n_nodes, d_err, n_cu * 4, s); return 0; }
  }
  return -1;
}
