// C ABI of libtrk.so: context lifecycle (create / execute / destroy, after the
// custom-backend lifecycle of Section 4.1), argument validation, the device
// arena, weight preparation and the chaining of the stage kernels of Section 2.2.2.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/trk.h"
#include "kernels.h"
#include "common.h"
#include "ctx.h"
#include "host_quant.h"

namespace {

// ---------------------------------------------------------------------------
// host-side weight preparation
// ---------------------------------------------------------------------------
struct HostLinear {
  int K = 0, N = 0;
  std::vector<float> w;  // [K][N]
  std::vector<float> b;  // [N]
};

uint16_t host_f2bf(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float host_bf2f(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

constexpr float FP8_ACT_SCALE = 256.f;   // storage scale of FP8 activations (|tanh| <= 1)

// fragment blocks of W[K][N]: block (nt, kb) at index nt * nkb + kb, 64 lanes x
// 16 bytes (FP32, BF16) or 32 bytes (FP8, values w * scale; split BF16, the high
// then the low parts).
std::vector<uint8_t> make_fragments(const float* w, int K, int N, int prec, int& nkb, int& nnt, float scale = 1.f) {
  const int KB = prec == TRK_PREC_F32 ? 16 : (prec == TRK_PREC_BF16 || prec == TRK_PREC_X3) ? 32 : 128;
  const int FB = (prec == TRK_PREC_FP8 || prec == TRK_PREC_X3) ? 32 : 16;
  nkb = (K + KB - 1) / KB;
  nnt = (N + 15) / 16;
  std::vector<uint8_t> out((size_t)nkb * nnt * 64 * FB, 0);
  for (int nt = 0; nt < nnt; ++nt)
    for (int kb = 0; kb < nkb; ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int g = lane >> 4, r = lane & 15, n = nt * 16 + r;
        uint8_t* dstp = out.data() + (((size_t)nt * nkb + kb) * 64 + lane) * FB;
        if (prec == TRK_PREC_FP8) {
          for (int j = 0; j < 32; ++j) {
            const int k = kb * 128 + 32 * g + j;
            dstp[j] = host_f2e4m3((k < K && n < N) ? w[(size_t)k * N + n] * scale : 0.f);
          }
        } else if (prec == TRK_PREC_F32) {
          float v[4];
          for (int s = 0; s < 4; ++s) {
            const int k = kb * 16 + 4 * g + s;
            v[s] = (k < K && n < N) ? w[(size_t)k * N + n] : 0.f;
          }
          memcpy(dstp, v, 16);
        } else if (prec == TRK_PREC_X3) {
          // the eight high parts, then the eight low parts
          uint16_t v[16];
          for (int j = 0; j < 8; ++j) {
            const int k = kb * 32 + 8 * g + j;
            const float x = (k < K && n < N) ? w[(size_t)k * N + n] : 0.f;
            v[j] = host_f2bf(x);
            v[8 + j] = host_f2bf(x - host_bf2f(v[j]));
          }
          memcpy(dstp, v, 32);
        } else {
          uint16_t v[8];
          for (int j = 0; j < 8; ++j) {
            const int k = kb * 32 + 8 * g + j;
            v[j] = host_f2bf((k < K && n < N) ? w[(size_t)k * N + n] : 0.f);
          }
          memcpy(dstp, v, 16);
        }
      }
  return out;
}

}  // namespace

namespace {

bool width_ok(int w, std::initializer_list<int> allowed) {
  for (int a : allowed)
    if (a == w) return true;
  return false;
}

int validate_config(const trk_config* c) {
  if (!c || c->abi_version != TRK_ABI_VERSION) return TRK_E_INVAL;
  if (!width_ok(c->emb_hidden, {64, 1024}) || c->emb_layers < 1 || c->emb_layers > 7) return TRK_E_INVAL;
  if (c->emb_dim < 1 || c->emb_dim > 16) return TRK_E_INVAL;
  if (!width_ok(c->filt_hidden, {64, 512}) || c->filt_layers < 1 || c->filt_layers > 7) return TRK_E_INVAL;
  if (!width_ok(c->gnn_hidden, {32, 128}) || c->gnn_iters < 0 || c->gnn_iters > 64) return TRK_E_INVAL;
  if (!(c->radius > 0.f) || c->k_max < 1 || c->k_max > 1024) return TRK_E_INVAL;
  if (c->precision < TRK_FP32 || c->precision > TRK_BF16X3_GNN_BF16) return TRK_E_INVAL;
  if ((c->precision == TRK_FP8 || c->precision == TRK_FP8_ALL) &&
      (c->emb_hidden % 128 || c->filt_hidden % 128 || c->gnn_hidden != 128))
    return TRK_E_INVAL;
  if (c->max_hits < 1 || c->max_hits > (1LL << 30)) return TRK_E_INVAL;
  if (c->max_cand_edges < 1 || c->max_cand_edges > (1LL << 31) - 1) return TRK_E_INVAL;
  if (c->max_kept_edges < 1 || c->max_kept_edges > (1LL << 31) - 1) return TRK_E_INVAL;
  if (c->max_events < 1 || c->max_events > 65535) return TRK_E_INVAL;
  if (c->max_hits * (int64_t)c->k_max > (1LL << 31) - 1) return TRK_E_INVAL;
  return TRK_OK;
}

struct BlobReader {
  const uint8_t* p;
  size_t left;
  bool ok = true;
  bool take(HostLinear& L, int K, int N) {
    const size_t need = ((size_t)K * N + N) * sizeof(float);
    if (!ok || left < need) return ok = false;
    L.K = K;
    L.N = N;
    L.w.resize((size_t)K * N);
    L.b.resize(N);
    memcpy(L.w.data(), p, (size_t)K * N * 4);
    memcpy(L.b.data(), p + (size_t)K * N * 4, (size_t)N * 4);
    p += need;
    left -= need;
    return true;
  }
};

// sub-matrix rows [r0, r0 + K) of L as a K x N layer, optional bias
HostLinear rows_of(const HostLinear& L, int r0, int K, bool bias) {
  HostLinear o;
  o.K = K;
  o.N = L.N;
  o.w.assign(L.w.begin() + (size_t)r0 * L.N, L.w.begin() + (size_t)(r0 + K) * L.N);
  o.b = bias ? L.b : std::vector<float>(L.N, 0.f);
  return o;
}

// The same layer for the input [(u_s + u_t) / 2, u_s - u_t] instead of [u_s, u_t]
// (u_s, u_t of width D): rows [W_s + W_t; (W_s - W_t) / 2].  Used where a BF16 layer
// reads the two ends of an edge, so that their difference is formed before rounding.
HostLinear mean_diff_form(const HostLinear& L, int D) {
  HostLinear o = L;
  for (int k = 0; k < D; ++k)
    for (int n = 0; n < L.N; ++n) {
      const double ws = L.w[(size_t)k * L.N + n], wt = L.w[(size_t)(D + k) * L.N + n];
      o.w[(size_t)k * L.N + n] = (float)(ws + wt);
      o.w[(size_t)(D + k) * L.N + n] = (float)(0.5 * (ws - wt));
    }
  return o;
}

// [rows a-block | rows b-block] side by side: K x 2N
HostLinear side_by_side(const HostLinear& L, int ra, int rb, int K) {
  HostLinear o;
  o.K = K;
  o.N = 2 * L.N;
  o.w.resize((size_t)K * o.N);
  for (int k = 0; k < K; ++k)
    for (int n = 0; n < L.N; ++n) {
      o.w[(size_t)k * o.N + n] = L.w[(size_t)(ra + k) * L.N + n];
      o.w[(size_t)k * o.N + L.N + n] = L.w[(size_t)(rb + k) * L.N + n];
    }
  o.b.assign(o.N, 0.f);
  return o;
}

struct WeightUpload {
  std::vector<uint8_t> bytes;
  struct Fix { DevLayer* L; size_t wofs, bofs, bsofs; };
  struct VecFix { DevVec* V; size_t wofs; };
  std::vector<Fix> fixes;
  std::vector<VecFix> vfixes;
  size_t put(const void* src, size_t n) {
    const size_t off = (bytes.size() + 255) & ~(size_t)255;
    bytes.resize(off + n);
    memcpy(bytes.data() + off, src, n);
    return off;
  }
  // act_scale: the storage scale of the FP8 activations the layer reads
  void layer(DevLayer& D, const HostLinear& L, int prec, float act_scale = FP8_ACT_SCALE) {
    D.K = L.K;
    D.N = L.N;
    const float scale = prec == TRK_PREC_FP8 ? fp8_weight_scale(L.w.data(), L.w.size()) : 1.f;
    // an FP8 layer reads FP8 activations (stored times act_scale) and FP8 weights
    D.dq = prec == TRK_PREC_FP8 ? 1.f / (scale * act_scale) : 1.f;
    std::vector<uint8_t> f = make_fragments(L.w.data(), L.K, L.N, prec, D.nkb, D.nnt, scale);
    std::vector<float> b((size_t)D.nnt * 16, 0.f), bs((size_t)D.nnt * 16, 0.f);
    for (int n = 0; n < L.N; ++n) {
      b[n] = L.b[n];
      bs[n] = (float)((double)L.b[n] * 2.8853900817779268);   // 2 log2(e)
    }
    const size_t wo = put(f.data(), f.size());
    const size_t bo = put(b.data(), b.size() * 4);
    const size_t bso = put(bs.data(), bs.size() * 4);
    fixes.push_back({&D, wo, bo, bso});
  }
  void vec(DevVec& V, const HostLinear& L) {  // L is K x 1
    V.K = L.K;
    std::vector<float> w(((size_t)L.K + 15) / 16 * 16, 0.f);
    for (int k = 0; k < L.K; ++k) w[k] = L.w[k];
    V.b = L.b[0];
    vfixes.push_back({&V, put(w.data(), w.size() * 4)});
  }
  void resolve(void* base) {
    for (auto& f : fixes) {
      f.L->w = (const uint4*)((char*)base + f.wofs);
      f.L->b = (const float*)((char*)base + f.bofs);
      f.L->bs = (const float*)((char*)base + f.bsofs);
    }
    for (auto& v : vfixes) v.V->w = (const float*)((char*)base + v.wofs);
  }
};

// Scales of the FP8 interaction network's stored tensors.  Every update adds a tanh
// to a tanh-initialised state, so |e|, |h| < T + 1 after T iterations; a projection
// column c of h W is then bounded by (T + 1) sum_k |W[k][c]| (with 1 % for the BF16
// roundings of h and W).  Each scale is the largest power of two that keeps its
// bound inside E4M3's 448, so no stored value saturates.
float pow2_scale_for(double bound) {
  return bound > 0 ? std::ldexp(1.f, (int)std::floor(std::log2(448.0 / bound))) : 1.f;
}

GnnScale gnn_state_scales(int iters, const HostLinear& eab, const HostLinear& oab) {
  const double hb = (double)(iters + 1);
  double colmax = 0;
  for (const HostLinear* L : {&eab, &oab})
    for (int n = 0; n < L->N; ++n) {
      double s = 0;
      for (int kk = 0; kk < L->K; ++kk) s += std::fabs((double)L->w[(size_t)kk * L->N + n]);
      colmax = std::max(colmax, s);
    }
  GnnScale sc;
  sc.e = pow2_scale_for(hb);
  sc.p = pow2_scale_for(hb * colmax * 1.01);
  sc.inv_e = 1.f / sc.e;
  sc.inv_p = 1.f / sc.p;
  return sc;
}

int load_weights(trk_ctx* c, const void* blob, size_t nbytes) {
  const trk_config& k = c->cfg;
  if (!blob || nbytes < 64) return TRK_E_WEIGHTS;
  uint32_t hdr[16];
  memcpy(hdr, blob, 64);
  if (hdr[0] != TRK_WEIGHTS_MAGIC || hdr[1] != TRK_ABI_VERSION) return TRK_E_WEIGHTS;
  const int32_t want[7] = {k.emb_hidden, k.emb_layers, k.emb_dim, k.filt_hidden, k.filt_layers, k.gnn_hidden,
                           k.gnn_iters};
  for (int i = 0; i < 7; ++i)
    if ((int32_t)hdr[2 + i] != want[i]) return TRK_E_WEIGHTS;
  BlobReader rd{(const uint8_t*)blob + 64, nbytes - 64};
  const int H = k.gnn_hidden, W = k.emb_hidden, F = k.filt_hidden, D = k.emb_dim;
  std::vector<HostLinear> emb(k.emb_layers + 1), filt(k.filt_layers + 1);
  for (int i = 0; i <= k.emb_layers; ++i)
    rd.take(emb[i], i == 0 ? 3 : W, i == k.emb_layers ? D : W);
  for (int i = 0; i <= k.filt_layers; ++i)
    rd.take(filt[i], i == 0 ? 2 * D : F, i == k.filt_layers ? 1 : F);
  HostLinear ne1, ne2, ee1, ee2, en1, en2, nn1, nn2, o1, o2;
  rd.take(ne1, 3, H); rd.take(ne2, H, H);
  rd.take(ee1, 6, H); rd.take(ee2, H, H);
  rd.take(en1, 3 * H, H); rd.take(en2, H, H);
  rd.take(nn1, 2 * H, H); rd.take(nn2, H, H);
  rd.take(o1, 3 * H, H); rd.take(o2, H, 1);
  if (!rd.ok || rd.left != 0) return TRK_E_WEIGHTS;

  const int prec = c->prec, prec_emb = c->prec_emb, prec_gnn = c->prec_gnn;
  // FP8 modes: FP8 for the layers that read a hidden activation tile of an FP8
  // MLP, BF16 for the narrow first layers and for the whole interaction network
  // (split BF16: FP32 for the narrow first MLP layers)
  const int prec_in = prec == TRK_PREC_FP8 ? TRK_PREC_BF16 : prec == TRK_PREC_X3 ? TRK_PREC_F32 : prec;
  const int prec_emb_in = prec_emb == TRK_PREC_FP8 ? TRK_PREC_BF16 : prec_emb == TRK_PREC_X3 ? TRK_PREC_F32 : prec_emb;
  WeightUpload up;
  up.layer(c->emb_in, emb[0], prec_emb_in);
  c->emb_hid.n = k.emb_layers - 1;
  for (int i = 1; i < k.emb_layers; ++i) up.layer(c->emb_hid.l[i - 1], emb[i], prec_emb);
  // a BF16 embedding's output layer runs in FP32 on the last hidden layer's FP32 values
  // (embed_kernel)
  up.layer(c->emb_out, emb[k.emb_layers], prec_emb == TRK_PREC_BF16 && k.emb_layers > 1 ? TRK_PREC_F32 : prec_emb);
  // a BF16 first layer reads the pair's mean and difference (filter_kernel)
  up.layer(c->filt_in, prec_in == TRK_PREC_BF16 ? mean_diff_form(filt[0], D) : filt[0], prec_in);
  c->filt_hid.n = k.filt_layers - 1;
  for (int i = 1; i < k.filt_layers; ++i) up.layer(c->filt_hid.l[i - 1], filt[i], prec);
  up.vec(c->filt_out, filt[k.filt_layers]);
  DevGNN& g = c->gnn;
  g.H = H;
  g.iters = k.gnn_iters;
  // FP8 interaction network: the edge-side layers (e-blocks of phi_e and phi_o, the
  // second layer of phi_e) in FP8, the node side in BF16; edge states and projections
  // stored as E4M3 with power-of-two scales from bounds (see gnn_state_scales)
  const bool gnn8 = prec_gnn == TRK_PREC_FP8;
  const int pn = gnn8 ? TRK_PREC_BF16 : prec_gnn;
  const HostLinear eab = side_by_side(en1, 0, H, H), oab = side_by_side(o1, 0, H, H);
  g.sc = gnn8 ? gnn_state_scales(k.gnn_iters, eab, oab) : GnnScale{};
  // the encoders' first layers read the hit features in FP32 (node_encode_kernel, edge_encode_kernel)
  up.layer(g.node_enc1, ne1, TRK_PREC_F32);
  up.layer(g.node_enc2, ne2, pn);
  up.layer(g.edge_enc1, ee1, TRK_PREC_F32);
  up.layer(g.edge_enc2, ee2, pn);
  up.layer(g.edge_c, rows_of(en1, 2 * H, H, true), prec_gnn, g.sc.e);
  up.layer(g.edge_ab, eab, pn);
  up.layer(g.edge_2, en2, prec_gnn);
  up.layer(g.node_1, nn1, pn);
  up.layer(g.node_2, nn2, pn);
  up.layer(g.out_c, rows_of(o1, 2 * H, H, true), prec_gnn, g.sc.e);
  up.layer(g.out_ab, oab, pn);
  up.vec(g.out_2, o2);
  if (hipMalloc(&c->wmem, up.bytes.size()) != hipSuccess) return TRK_E_NOMEM;
  if (hipMemcpy(c->wmem, up.bytes.data(), up.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) return TRK_E_DEVICE;
  up.resolve(c->wmem);
  return TRK_OK;
}

int64_t next_pow2(int64_t v) {
  int64_t p = 1024;
  while (p < v) p <<= 1;
  return p;
}

int alloc_scratch(trk_ctx* c) {
  const trk_config& k = c->cfg;
  const int64_t NH = k.max_hits, CC = k.max_cand_edges, CF = k.max_kept_edges;
  const int H = k.gnn_hidden;
  const size_t act = (c->prec_gnn == TRK_PREC_F32 || c->prec_gnn == TRK_PREC_X3) ? 4 : c->prec_gnn == TRK_PREC_FP8 ? 1 : 2;
  Arena& a = c->arena;
  GraphScratch& g = c->graph;
  GnnScratch& s = c->gs;
  g.table = next_pow2(2 * NH);
  g.stats_blocks = 256;
  const int64_t tmp_ints = std::max({scan_tmp_ints(CC), scan_tmp_ints(CF), scan_tmp_ints(g.table), scan_tmp_ints(NH + 1),
                                     scan_tmp_ints(256 * fit_sort_blocks(NH))});
  a.add(c->emb, (size_t)NH * k.emb_dim);
  a.add(c->cand_src, CC);
  a.add(c->cand_dst, CC);
  a.add(c->cand_scores, CC);
  a.add(c->filt_src, CF);
  a.add(c->filt_dst, CF);
  a.add(c->gnn_scores, CF);
  a.add(c->ev, NH);
  a.add(c->fit_cnt, NH + 1);
  a.add(c->fit_flag, NH + 1);
  a.add(c->fit_cidx, NH + 1);
  a.add(c->fit_start, NH + 1);
  a.add(c->fit_keys, NH);
  a.add(c->fit_keys2, NH);
  a.add(c->fit_raw, NH);
  a.add(c->fit_hits, NH);
  a.add(c->fit_hist, (size_t)256 * fit_sort_blocks(NH) + 1);
  a.add(c->fit_hoff, (size_t)256 * fit_sort_blocks(NH) + 1);
  a.add(c->offs, (size_t)k.max_events + 1);
  a.add(c->dev_words, 16);
  a.add(c->batch_counts, (size_t)k.max_events * 4);
  a.add(g.cell, NH);
  a.add(g.bucket, NH);
  a.add(g.sorted_id, NH);
  a.add(g.sorted_emb, (size_t)NH * 16);
  a.add(g.sorted_cell, NH);
  a.add(g.cnt, NH);
  a.add(g.thr, NH);
  a.add(g.rowcnt, NH + 1);
  a.add(g.rowptr, NH + 1);
  a.add(g.cursor, NH);
  a.add(g.unsorted, CC);
  a.add(g.hist, g.table);
  a.add(g.start, g.table + 1);
  a.add(g.fill, g.table);
  a.add(g.stats, (size_t)g.stats_blocks * 160);
  a.add(g.basis, 64);
  a.add(g.counters, 8);
  a.add(g.tmp, tmp_ints);
  a.add(s.h, (size_t)NH * H);
  a.add(s.msg, (size_t)NH * H);
  a.add_bytes(s.proj, (size_t)NH * 2 * H * act);
  a.add_bytes(s.e, (size_t)CF * H * act);
  a.add(s.rowptr, NH + 1);
  a.add(s.rowidx, CF);
  a.add(s.cscptr, NH + 1);
  a.add(s.cscidx, CF);
  a.add(s.raw, CF);
  a.add(s.cnt, NH);
  a.add(s.tmp, tmp_ints);
  if (a.commit() != hipSuccess) return TRK_E_NOMEM;
  if (hipHostMalloc((void**)&c->host_words, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->host_offs, sizeof(int64_t) * ((size_t)k.max_events + 1), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&c->host_counts, sizeof(int) * 4 * (size_t)k.max_events, hipHostMallocDefault) != hipSuccess)
    return TRK_E_NOMEM;
  return TRK_OK;
}

void read_stage_times(trk_ctx* c, float* out) {
  for (int i = 0; i < 8; ++i) out[i] = 0.f;
  if (!c->timing) return;
  for (int i = 0; i < 6; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_stage[i], c->ev_stage[i + 1]) == hipSuccess) out[i] = ms;
  }
}

int sync_words(trk_ctx* c, hipStream_t s) {
  // dev_words[0..8) then graph counters[0..8)
  if (hipMemcpyAsync(c->host_words, c->dev_words, 16 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
    return TRK_E_DEVICE;
  if (hipMemcpyAsync(c->host_words + 16, c->graph.counters, 8 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
    return TRK_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return TRK_E_DEVICE;
  return TRK_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) hipSetDevice(prev);
  }
};

int check_launch() { return hipGetLastError() == hipSuccess ? TRK_OK : TRK_E_DEVICE; }

// the whole chain on hits [0, n) of x; ev (nullable) gives the event of each hit
int run_chain(trk_ctx* c, const float* x, int n, const int* ev, int* labels, hipStream_t s) {
  const trk_config& k = c->cfg;
  int* err = &c->dev_words[0];
  int* n_filt = &c->dev_words[1];
  int* n_kept = &c->dev_words[2];
  auto mark = [&](int i) {
    if (c->timing) hipEventRecord(c->ev_stage[i], s);
  };
  launch_fill_int(c->dev_words, 0, 16, s);
  mark(0);
  if (launch_embed(c->prec_emb, k.emb_hidden, x, n, c->emb_in, c->emb_hid, c->emb_out, k.emb_dim, c->emb, c->n_cu, s))
    return TRK_E_INVAL;
  mark(1);
  launch_build_graph(c->emb, n, k.emb_dim, k.radius, k.k_max, ev, c->graph, c->cand_src, c->cand_dst,
                     k.max_cand_edges, c->n_cu, s);
  mark(2);
  const int* n_cand = &c->graph.counters[0];
  if (launch_filter(c->prec, k.filt_hidden, c->emb, k.emb_dim, c->cand_src, c->cand_dst, 0, n_cand,
                    k.max_cand_edges, c->filt_in, c->filt_hid, c->filt_out, c->cand_scores, n, err, c->n_cu, s))
    return TRK_E_INVAL;
  mark(3);
  launch_compact_edges(c->cand_scores, k.filter_cut, c->cand_src, c->cand_dst, k.max_cand_edges, n_cand, c->filt_src,
                       c->filt_dst, k.max_kept_edges, n_filt, c->graph.tmp, s);
  mark(4);
  // the filtered edges keep the radius graph's (source, destination) order
  if (launch_gnn(c->prec_gnn, c->gnn, x, n, c->filt_src, c->filt_dst, k.max_kept_edges, n_filt, c->gnn_scores, c->gs,
                 c->n_cu, err, s, true))
    return TRK_E_INVAL;
  mark(5);
  launch_components(n, c->filt_src, c->filt_dst, c->gnn_scores, k.score_cut, k.max_kept_edges, n_filt, labels,
                    n_kept, err, s);
  mark(6);
  return check_launch();
}

}  // namespace

extern "C" {

const char* trk_strerror(int status) {
  switch (status) {
    case TRK_OK: return "ok";
    case TRK_E_INVAL: return "invalid argument";
    case TRK_E_NOMEM: return "device memory allocation failed";
    case TRK_E_CAPACITY: return "edge count exceeds capacity";
    case TRK_E_DEVICE: return "HIP runtime error";
    case TRK_E_WEIGHTS: return "malformed weight blob";
    case TRK_E_EXPIRED: return "request deadline passed before it was run";
    case TRK_E_SHUTDOWN: return "server is shutting down";
    default: return "unknown status";
  }
}

int trk_create(const trk_config* cfg, const void* h_weights, size_t nbytes, int device_id, trk_ctx** out) {
  if (!out) return TRK_E_INVAL;
  *out = nullptr;
  int rc = validate_config(cfg);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device_id < 0 || device_id >= ndev) return TRK_E_INVAL;
  DeviceGuard guard(device_id);
  trk_ctx* c = new trk_ctx();
  c->cfg = *cfg;
  c->device = device_id;
  switch (cfg->precision) {
    // (embedding, filter, interaction network)
    case TRK_BF16: c->prec_emb = c->prec = c->prec_gnn = TRK_PREC_BF16; break;
    case TRK_FP8: c->prec_emb = TRK_PREC_BF16; c->prec = c->prec_gnn = TRK_PREC_FP8; break;
    case TRK_FP8_ALL: c->prec_emb = c->prec = c->prec_gnn = TRK_PREC_FP8; break;
    case TRK_BF16_EMB32: c->prec_emb = TRK_PREC_F32; c->prec = c->prec_gnn = TRK_PREC_BF16; break;
    case TRK_BF16X3: c->prec_emb = c->prec = c->prec_gnn = TRK_PREC_X3; break;
    case TRK_BF16X3_GNN_BF16: c->prec_emb = c->prec = TRK_PREC_X3; c->prec_gnn = TRK_PREC_BF16; break;
    default: c->prec_emb = c->prec = c->prec_gnn = TRK_PREC_F32;
  }
  hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device_id);
  if (c->n_cu <= 0) c->n_cu = 256;
  rc = load_weights(c, h_weights, nbytes);
  if (!rc) rc = alloc_scratch(c);
  c->timing = cfg->stage_timing != 0;
  if (!rc && cfg->training) rc = train_create(c);
  if (!rc && hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess) rc = TRK_E_DEVICE;
  for (int i = 0; i < 8 && !rc && c->timing; ++i)
    if (hipEventCreate(&c->ev_stage[i]) != hipSuccess) rc = TRK_E_DEVICE;
  if (rc) {
    trk_destroy(c);
    return rc;
  }
  *out = c;
  return TRK_OK;
}

void trk_destroy(trk_ctx* c) {
  if (!c) return;
  DeviceGuard guard(c->device);
  // every call on this context is ordered after the previous one, so its last
  // recorded completion covers all of its work (other contexts are not waited for)
  if (c->done) {
    if (c->used) hipEventSynchronize(c->done);
    hipEventDestroy(c->done);
  }
  train_destroy(c);
  if (c->arena.base) hipFree(c->arena.base);
  if (c->wmem) hipFree(c->wmem);
  if (c->host_words) hipHostFree(c->host_words);
  if (c->host_offs) hipHostFree(c->host_offs);
  if (c->host_counts) hipHostFree(c->host_counts);
  for (int i = 0; i < 8; ++i)
    if (c->ev_stage[i]) hipEventDestroy(c->ev_stage[i]);
  delete c;
}

int trk_embed(trk_ctx* c, const float* d_x, int64_t n, float* d_emb, hipStream_t s) {
  if (!c || n < 0 || n > c->cfg.max_hits || (n > 0 && (!d_x || !d_emb))) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (n == 0) return TRK_OK;
  DeviceGuard guard(c->device);
  if (launch_embed(c->prec_emb, c->cfg.emb_hidden, d_x, (int)n, c->emb_in, c->emb_hid, c->emb_out, c->cfg.emb_dim, d_emb,
                   c->n_cu, s))
    return TRK_E_INVAL;
  return check_launch();
}

int trk_build_graph(trk_ctx* c, const float* d_emb, int64_t n, int32_t* d_src, int32_t* d_dst, int64_t cap,
                    int64_t* h_n_edges, int64_t* h_n_saturated, hipStream_t s) {
  if (!c || !h_n_edges || n < 0 || n > c->cfg.max_hits || cap < 0) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (n > 0 && (!d_emb || (cap > 0 && (!d_src || !d_dst)))) return TRK_E_INVAL;
  *h_n_edges = 0;
  if (h_n_saturated) *h_n_saturated = 0;
  if (n == 0) return TRK_OK;
  DeviceGuard guard(c->device);
  const int64_t eff = std::min(cap, c->cfg.max_cand_edges);
  launch_build_graph(d_emb, (int)n, c->cfg.emb_dim, c->cfg.radius, c->cfg.k_max, nullptr, c->graph, d_src, d_dst, eff,
                     c->n_cu, s);
  if (check_launch()) return TRK_E_DEVICE;
  if (sync_words(c, s)) return TRK_E_DEVICE;
  const int64_t total = (uint32_t)c->host_words[16];
  *h_n_edges = total;
  if (h_n_saturated) *h_n_saturated = c->host_words[17];
  return total > eff ? TRK_E_CAPACITY : TRK_OK;
}

int trk_filter(trk_ctx* c, const float* d_emb, int64_t n, const int32_t* d_src, const int32_t* d_dst, int64_t m,
               float* d_scores, int32_t* d_kept_src, int32_t* d_kept_dst, int64_t cap, int64_t* h_n_kept,
               hipStream_t s) {
  if (!c || !h_n_kept || n < 0 || n > c->cfg.max_hits || m < 0 || cap < 0) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (m > 0 && (!d_emb || !d_src || !d_dst)) return TRK_E_INVAL;
  if (cap > 0 && (!d_kept_src || !d_kept_dst)) return TRK_E_INVAL;
  if (m > c->cfg.max_cand_edges) return TRK_E_INVAL;
  *h_n_kept = 0;
  if (m == 0) return TRK_OK;
  DeviceGuard guard(c->device);
  float* scores = d_scores ? d_scores : c->cand_scores;
  launch_fill_int(c->dev_words, 0, 16, s);
  if (launch_filter(c->prec, c->cfg.filt_hidden, d_emb, c->cfg.emb_dim, d_src, d_dst, m, nullptr, m, c->filt_in,
                    c->filt_hid, c->filt_out, scores, (int)n, &c->dev_words[0], c->n_cu, s))
    return TRK_E_INVAL;
  launch_compact_edges(scores, c->cfg.filter_cut, d_src, d_dst, m, nullptr, d_kept_src, d_kept_dst, cap,
                       &c->dev_words[1], c->graph.tmp, s);
  if (check_launch()) return TRK_E_DEVICE;
  if (sync_words(c, s)) return TRK_E_DEVICE;
  if (c->host_words[0] & TRK_ERRBIT_INDEX) return TRK_E_INVAL;
  *h_n_kept = (uint32_t)c->host_words[1];
  return *h_n_kept > cap ? TRK_E_CAPACITY : TRK_OK;
}

int trk_gnn(trk_ctx* c, const float* d_x, int64_t n, const int32_t* d_src, const int32_t* d_dst, int64_t m,
            float* d_scores, hipStream_t s) {
  if (!c || n < 0 || n > c->cfg.max_hits || m < 0 || m > c->cfg.max_kept_edges) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (n > 0 && !d_x) return TRK_E_INVAL;
  if (m > 0 && (!d_src || !d_dst || !d_scores)) return TRK_E_INVAL;
  if (n == 0) return m == 0 ? TRK_OK : TRK_E_INVAL;
  DeviceGuard guard(c->device);
  launch_fill_int(c->dev_words, 0, 16, s);
  if (launch_gnn(c->prec_gnn, c->gnn, d_x, (int)n, d_src, d_dst, m, nullptr, d_scores, c->gs, c->n_cu, &c->dev_words[0], s))
    return TRK_E_INVAL;
  if (check_launch()) return TRK_E_DEVICE;
  if (sync_words(c, s)) return TRK_E_DEVICE;
  return (c->host_words[0] & TRK_ERRBIT_INDEX) ? TRK_E_INVAL : TRK_OK;
}

int trk_components(trk_ctx* c, int64_t n, const int32_t* d_src, const int32_t* d_dst, const float* d_scores,
                   int64_t m, float cut, int32_t* d_labels, hipStream_t s) {
  if (!c || n < 0 || n > c->cfg.max_hits || m < 0 || m > (1LL << 31) - 1) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (n > 0 && !d_labels) return TRK_E_INVAL;
  if (m > 0 && (!d_src || !d_dst)) return TRK_E_INVAL;
  if (n == 0) return m == 0 ? TRK_OK : TRK_E_INVAL;
  DeviceGuard guard(c->device);
  launch_fill_int(c->dev_words, 0, 16, s);
  launch_components((int)n, d_src, d_dst, d_scores, cut, m, nullptr, d_labels, nullptr, &c->dev_words[0], s);
  if (check_launch()) return TRK_E_DEVICE;
  if (sync_words(c, s)) return TRK_E_DEVICE;
  return (c->host_words[0] & TRK_ERRBIT_INDEX) ? TRK_E_INVAL : TRK_OK;
}

int trk_event(trk_ctx* c, const float* d_x, int64_t n, int32_t* d_labels, trk_event_info* info, hipStream_t s) {
  if (!c || n < 0 || n > c->cfg.max_hits || (n > 0 && (!d_x || !d_labels))) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (info) memset(info, 0, sizeof(*info));
  if (n == 0) return TRK_OK;
  DeviceGuard guard(c->device);
  int rc = run_chain(c, d_x, (int)n, nullptr, d_labels, s);
  if (rc) return rc;
  if (sync_words(c, s)) return TRK_E_DEVICE;
  const int64_t n_cand = (uint32_t)c->host_words[16];
  const int64_t n_filt = (uint32_t)c->host_words[1];
  if (info) {
    info->n_hits = n;
    info->n_cand_edges = n_cand;
    info->n_filt_edges = n_filt;
    info->n_kept_edges = (uint32_t)c->host_words[2];
    info->n_saturated = c->host_words[17];
    read_stage_times(c, info->stage_ms);
  }
  if (n_cand > c->cfg.max_cand_edges || n_filt > c->cfg.max_kept_edges) return TRK_E_CAPACITY;
  if (c->host_words[0] & TRK_ERRBIT_INDEX) return TRK_E_DEVICE;
  return TRK_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches of events
// ---------------------------------------------------------------------------
namespace {

__global__ void event_ids_kernel(const int64_t* __restrict__ offs, int nev, int n, int* __restrict__ ev) {
  GRID_STRIDE(i, n) {
    int lo = 0, hi = nev;  // largest b with offs[b] <= i
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (offs[mid] <= i) lo = mid; else hi = mid;
    }
    ev[i] = lo;
  }
}

// labels to event-local ids; per-event counts of candidate, filtered and kept edges
__global__ void batch_finish_kernel(const int64_t* __restrict__ offs, const int* __restrict__ ev, int n,
                                    int* __restrict__ labels) {
  GRID_STRIDE(i, n) labels[i] -= (int)offs[ev[i]];
}

// first index e in [0, m) with key[e] >= v (key ascending)
__device__ __forceinline__ int64_t lower_bound_i(const int* key, int64_t m, int64_t v) {
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Per-event counts, one block per event, no atomics: the candidate and the filtered
// edges are sorted by source and every event owns a contiguous range of hit ids, so an
// event's edges form one contiguous range found by binary search.
__global__ __launch_bounds__(256) void event_counts_kernel(const int64_t* __restrict__ offs, const int* __restrict__ csrc,
                                                           int64_t ccap, const int* d_nc, const int* __restrict__ fsrc,
                                                           int64_t fcap, const int* d_nf, const float* __restrict__ scores,
                                                           float cut, const int* __restrict__ cnt, int k_max,
                                                           int* __restrict__ counts) {
  __shared__ int sh[2][4];
  const int b = blockIdx.x;
  const int64_t nc = clamp_count(d_nc, ccap), nf = clamp_count(d_nf, fcap);
  const int64_t h0 = offs[b], h1 = offs[b + 1];
  const int64_t c0 = lower_bound_i(csrc, nc, h0), c1 = lower_bound_i(csrc, nc, h1);
  const int64_t f0 = lower_bound_i(fsrc, nf, h0), f1 = lower_bound_i(fsrc, nf, h1);
  int kept = 0, sat = 0;
  for (int64_t e = f0 + threadIdx.x; e < f1; e += blockDim.x) kept += scores[e] > cut ? 1 : 0;
  for (int64_t i = h0 + threadIdx.x; i < h1; i += blockDim.x) sat += cnt[i] > k_max ? 1 : 0;
  kept = wave_sum(kept);
  sat = wave_sum(sat);
  if (lane_id() == 0) {
    sh[0][threadIdx.x >> 6] = kept;
    sh[1][threadIdx.x >> 6] = sat;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    counts[b * 4 + 0] = (int)(c1 - c0);
    counts[b * 4 + 1] = (int)(f1 - f0);
    counts[b * 4 + 2] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    counts[b * 4 + 3] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
  }
}

}  // namespace

extern "C" int trk_batch(trk_ctx* c, int32_t n_events, const float* d_x, const int64_t* h_offsets, int32_t* d_labels,
                         trk_event_info* infos, hipStream_t s) {
  if (!c || n_events < 0 || n_events > c->cfg.max_events || (n_events > 0 && !h_offsets)) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (n_events == 0) return TRK_OK;
  if (h_offsets[0] != 0) return TRK_E_INVAL;
  for (int b = 0; b < n_events; ++b)
    if (h_offsets[b + 1] < h_offsets[b]) return TRK_E_INVAL;
  const int64_t n = h_offsets[n_events];
  if (n > c->cfg.max_hits || (n > 0 && (!d_x || !d_labels))) return TRK_E_INVAL;
  if (infos) memset(infos, 0, sizeof(trk_event_info) * n_events);
  if (n == 0) return TRK_OK;
  DeviceGuard guard(c->device);
  // staged through pinned memory so the copy is asynchronous; the stream is idle here
  // with respect to the previous call's use of the staging buffer (that call synchronised)
  memcpy(c->host_offs, h_offsets, sizeof(int64_t) * (n_events + 1));
  if (hipMemcpyAsync(c->offs, c->host_offs, sizeof(int64_t) * (n_events + 1), hipMemcpyHostToDevice, s) != hipSuccess)
    return TRK_E_DEVICE;
  event_ids_kernel<<<blocks_for(n, 256), 256, 0, s>>>(c->offs, n_events, (int)n, c->ev);
  int rc = run_chain(c, d_x, (int)n, c->ev, d_labels, s);
  if (rc) return rc;
  if (infos) {
    const trk_config& k = c->cfg;
    event_counts_kernel<<<n_events, 256, 0, s>>>(c->offs, c->cand_src, k.max_cand_edges, &c->graph.counters[0],
                                                 c->filt_src, k.max_kept_edges, &c->dev_words[1], c->gnn_scores,
                                                 k.score_cut, c->graph.cnt, k.k_max, c->batch_counts);
  }
  batch_finish_kernel<<<blocks_for(n, 256), 256, 0, s>>>(c->offs, c->ev, (int)n, d_labels);
  if (check_launch()) return TRK_E_DEVICE;
  const int* counts = c->host_counts;
  if (infos && hipMemcpyAsync(c->host_counts, c->batch_counts, (size_t)n_events * 4 * sizeof(int),
                              hipMemcpyDeviceToHost, s) != hipSuccess)
    return TRK_E_DEVICE;
  if (sync_words(c, s)) return TRK_E_DEVICE;
  const int64_t n_cand = (uint32_t)c->host_words[16];
  const int64_t n_filt = (uint32_t)c->host_words[1];
  if (infos)
    for (int b = 0; b < n_events; ++b) {
      infos[b].n_hits = h_offsets[b + 1] - h_offsets[b];
      infos[b].n_cand_edges = counts[b * 4 + 0];
      infos[b].n_filt_edges = counts[b * 4 + 1];
      infos[b].n_kept_edges = counts[b * 4 + 2];
      infos[b].n_saturated = counts[b * 4 + 3];
      read_stage_times(c, infos[b].stage_ms);
    }
  if (n_cand > c->cfg.max_cand_edges || n_filt > c->cfg.max_kept_edges) return TRK_E_CAPACITY;
  if (c->host_words[0] & TRK_ERRBIT_INDEX) return TRK_E_DEVICE;
  return TRK_OK;
}
