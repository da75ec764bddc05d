// Internal definition of the context (shared by the C-ABI files).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

#include "../../include/trk.h"
#include "kernels.h"

// ---------------------------------------------------------------------------
// device arena: one allocation carved into 256-byte aligned pieces
// ---------------------------------------------------------------------------
struct Arena {
  std::vector<std::pair<void**, size_t>> req;
  void* base = nullptr;
  size_t total = 0;
  template <class T>
  void add(T*& p, size_t count) { req.push_back({(void**)&p, count * sizeof(T)}); }
  void add_bytes(void*& p, size_t bytes) { req.push_back({&p, bytes}); }
  hipError_t commit() {
    total = 0;
    for (auto& r : req) total += (r.second + 255) & ~(size_t)255;
    if (total == 0) total = 256;
    hipError_t e = hipMalloc(&base, total);
    if (e != hipSuccess) return e;
    size_t off = 0;
    for (auto& r : req) {
      *r.first = (char*)base + off;
      off += (r.second + 255) & ~(size_t)255;
    }
    return hipSuccess;
  }
};


struct TrainState;

struct trk_ctx {
  trk_config cfg;
  int device = 0;
  int n_cu = 256;
  int prec = TRK_PREC_F32;       // filter MLP
  int prec_emb = TRK_PREC_F32;   // embedding MLP
  int prec_gnn = TRK_PREC_F32;   // interaction network
  // weights
  void* wmem = nullptr;
  DevLayer emb_in, emb_out;
  LayerList emb_hid;
  DevLayer filt_in;
  LayerList filt_hid;
  DevVec filt_out;
  DevGNN gnn;
  // scratch
  Arena arena;
  float* emb = nullptr;
  int* cand_src = nullptr;
  int* cand_dst = nullptr;
  float* cand_scores = nullptr;
  int* filt_src = nullptr;
  int* filt_dst = nullptr;
  float* gnn_scores = nullptr;
  int* ev = nullptr;
  int64_t* offs = nullptr;
  int* dev_words = nullptr;  // [16]: 0 err bits, 1 filtered count, 2 kept count, 3.. per-event use
  int* batch_counts = nullptr;  // [max_events][4] per-event counts
  GraphScratch graph;
  GnnScratch gs;
  // helix fit (fit.hip): per-label counts, flags, candidate index, segment starts,
  // fill cursors, hit ids grouped by label (unsorted, sorted)
  int *fit_cnt = nullptr, *fit_flag = nullptr, *fit_cidx = nullptr, *fit_start = nullptr;
  int *fit_keys = nullptr, *fit_keys2 = nullptr, *fit_raw = nullptr, *fit_hits = nullptr;
  int *fit_hist = nullptr, *fit_hoff = nullptr;   // radix digit counts per block, their offsets
  int* host_words = nullptr;  // pinned mirror
  int64_t* host_offs = nullptr;  // pinned staging of batch offsets [max_events + 1]
  int* host_counts = nullptr;    // pinned per-event counts [max_events][4]
  hipEvent_t ev_stage[8] = {};
  bool timing = false;
  // the last call's completion and its stream (see CtxStreamScope)
  hipEvent_t done = nullptr;
  hipStream_t last_stream = nullptr;
  bool used = false;
  TrainState* train = nullptr;   // training buffers (trk_config.training != 0)
};

// Every entry point that enqueues work on a context holds one of these for the call:
// a call on a stream other than the previous call's first waits for that call's work
// (both would use the context's scratch), and the call's completion is recorded, so
// that trk_destroy waits for this context's own work only.
struct CtxStreamScope {
  trk_ctx* c;
  hipStream_t s;
  CtxStreamScope(trk_ctx* c_, hipStream_t s_) : c(c_), s(s_) {
    if (c->done && c->used && c->last_stream != s) hipStreamWaitEvent(s, c->done, 0);
  }
  ~CtxStreamScope() {
    if (c->done && hipEventRecord(c->done, s) == hipSuccess) {
      c->last_stream = s;
      c->used = true;
    }
  }
};

// training (train.hip)
int train_create(trk_ctx* c);
void train_destroy(trk_ctx* c);
int64_t train_param_count(const trk_config& k);
int train_set_params(trk_ctx* c, const float* P, hipStream_t s);
