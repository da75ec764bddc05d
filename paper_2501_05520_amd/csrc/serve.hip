// Serving loop on the GPU: the request scheduler of serve_core.h driving
// n_slots executor slots, each a context (weights + arena) with its own stream
// and pinned staging buffers; one batch of events per slot at a time through
// trk_batch.
#include <hip/hip_runtime.h>
#include <string.h>

#include <vector>

#include "../../include/trk.h"
#include "serve_core.h"
#include "service_core.h"

namespace {

struct GpuSlot {
  trk_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  float* h_x = nullptr;        // pinned [max_hits][3]
  int32_t* h_labels = nullptr; // pinned [max_hits]
  float* d_x = nullptr;
  int32_t* d_labels = nullptr;
  std::vector<int64_t> offs;
  std::vector<trk_event_info> infos;
};

struct GpuExec {
  int device = 0;
  std::vector<GpuSlot> slots;

  int run(int slot, std::vector<trk_serve::Request*>& batch) {
    GpuSlot& S = slots[slot];
    hipSetDevice(device);
    const int nb = (int)batch.size();
    S.offs.assign(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
      const trk_serve::Request* r = batch[b];
      if (r->n) memcpy(S.h_x + 3 * S.offs[b], r->x.data(), sizeof(float) * 3 * r->n);
      S.offs[b + 1] = S.offs[b] + r->n;
    }
    const int64_t n = S.offs[nb];
    S.infos.assign(nb, trk_event_info());
    if (n > 0 && hipMemcpyAsync(S.d_x, S.h_x, sizeof(float) * 3 * n, hipMemcpyHostToDevice, S.stream) != hipSuccess)
      return TRK_E_DEVICE;
    int rc = trk_batch(S.ctx, nb, S.d_x, S.offs.data(), S.d_labels, S.infos.data(), S.stream);
    if (rc != TRK_OK) return rc;
    if (n > 0) {
      if (hipMemcpyAsync(S.h_labels, S.d_labels, sizeof(int32_t) * n, hipMemcpyDeviceToHost, S.stream) != hipSuccess)
        return TRK_E_DEVICE;
      if (hipStreamSynchronize(S.stream) != hipSuccess) return TRK_E_DEVICE;
    }
    for (int b = 0; b < nb; ++b) {
      trk_serve::Request* r = batch[b];
      r->labels.assign(S.h_labels + S.offs[b], S.h_labels + S.offs[b + 1]);
      const trk_event_info& I = S.infos[b];
      r->counts[0] = I.n_hits;
      r->counts[1] = I.n_cand_edges;
      r->counts[2] = I.n_filt_edges;
      r->counts[3] = I.n_kept_edges;
      r->counts[4] = I.n_saturated;
      memcpy(r->stage_ms, I.stage_ms, sizeof(r->stage_ms));
      r->status = TRK_OK;
    }
    return TRK_OK;
  }
};

}  // namespace

struct trk_server {
  GpuExec exec;
  trk_serve::Server<GpuExec>* core = nullptr;
  uint64_t slot_bytes = 0;
  int64_t max_hits = 0;
};

namespace {

// the socket front end's view of a server
struct ServerBackend {
  trk_server* s;
  int submit(const float* x, int64_t n, double deadline_ms, int64_t* ticket) {
    return s->core->submit(x, n, deadline_ms, ticket);
  }
  int wait(int64_t ticket, int32_t* labels, int64_t* counts5, float* stage8, double* latency_ms) {
    return s->core->wait(ticket, labels, counts5, stage8, latency_ms);
  }
};

}  // namespace

struct trk_service {
  ServerBackend backend;
  trk_net::Service<ServerBackend>* svc = nullptr;
};

namespace {

void free_slots(trk_server* s) {
  for (GpuSlot& S : s->exec.slots) {
    if (S.ctx) trk_destroy(S.ctx);
    if (S.stream) hipStreamDestroy(S.stream);
    if (S.h_x) hipHostFree(S.h_x);
    if (S.h_labels) hipHostFree(S.h_labels);
    if (S.d_x) hipFree(S.d_x);
    if (S.d_labels) hipFree(S.d_labels);
  }
  s->exec.slots.clear();
}

}  // namespace

extern "C" {

int trk_server_create(const trk_config* cfg, const void* h_weights, size_t nbytes, int device_id,
                      const trk_server_config* scfg, trk_server** out) {
  if (!out || !cfg || !scfg) return TRK_E_INVAL;
  *out = nullptr;
  if (scfg->n_slots < 1 || scfg->n_slots > 16 || scfg->max_batch_events < 1 || scfg->max_batch_events > 65535 ||
      scfg->max_batch_hits < 1 || scfg->mem_budget_bytes == 0)
    return TRK_E_INVAL;
  trk_config c = *cfg;
  c.max_hits = scfg->max_batch_hits;
  c.max_events = scfg->max_batch_events;
  c.max_cand_edges = scfg->max_cand_edges > 0 ? scfg->max_cand_edges : scfg->max_batch_hits * (int64_t)cfg->k_max;
  c.max_kept_edges = scfg->max_kept_edges > 0 ? scfg->max_kept_edges : c.max_cand_edges;
  if (hipSetDevice(device_id) != hipSuccess) return TRK_E_INVAL;
  trk_server* s = new trk_server();
  s->exec.device = device_id;
  s->exec.slots.resize(scfg->n_slots);
  size_t free0 = 0, free1 = 0, total = 0;
  hipMemGetInfo(&free0, &total);
  int rc = TRK_OK;
  for (GpuSlot& S : s->exec.slots) {
    rc = trk_create(&c, h_weights, nbytes, device_id, &S.ctx);
    if (rc) break;
    const size_t nx = (size_t)c.max_hits;
    if (hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void**)&S.h_x, nx * 3 * sizeof(float), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&S.h_labels, nx * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&S.d_x, nx * 3 * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&S.d_labels, nx * sizeof(int32_t)) != hipSuccess) {
      rc = TRK_E_NOMEM;
      break;
    }
  }
  if (rc) {
    free_slots(s);
    delete s;
    return rc;
  }
  hipMemGetInfo(&free1, &total);
  s->slot_bytes = free0 > free1 ? (free0 - free1) / scfg->n_slots : 0;
  const uint64_t per_hit = scfg->bytes_per_hit ? scfg->bytes_per_hit
                                               : (uint64_t)(s->slot_bytes / (uint64_t)scfg->max_batch_hits) + 64;
  s->core = new trk_serve::Server<GpuExec>(&s->exec, scfg->n_slots, scfg->max_batch_events, scfg->max_batch_hits,
                                            scfg->mem_budget_bytes, per_hit, 4096);
  s->max_hits = scfg->max_batch_hits;
  *out = s;
  return TRK_OK;
}

int trk_server_submit(trk_server* s, const float* h_x, int64_t n, double deadline_ms, int64_t* ticket) {
  if (!s) return TRK_E_INVAL;
  return s->core->submit(h_x, n, deadline_ms, ticket);
}

int trk_server_wait(trk_server* s, int64_t ticket, int32_t* h_labels, trk_event_info* info, double* latency_ms) {
  if (!s) return TRK_E_INVAL;
  int64_t counts[5] = {0, 0, 0, 0, 0};
  float stage[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int rc = s->core->wait(ticket, h_labels, counts, stage, latency_ms);
  if (info) {
    info->n_hits = counts[0];
    info->n_cand_edges = counts[1];
    info->n_filt_edges = counts[2];
    info->n_kept_edges = counts[3];
    info->n_saturated = counts[4];
    memcpy(info->stage_ms, stage, sizeof(stage));
  }
  return rc;
}

int trk_server_stats(trk_server* s, trk_server_info* out) {
  if (!s || !out) return TRK_E_INVAL;
  const trk_serve::Stats st = s->core->stats();
  out->submitted = st.submitted;
  out->completed = st.completed;
  out->rejected = st.rejected;
  out->expired = st.expired;
  out->batches = st.batches;
  out->batched_events = st.batched_events;
  out->admitted_at_once = st.admitted_at_once;
  out->waited_for_memory = st.waited_for_memory;
  out->inflight_bytes = st.inflight_bytes;
  out->peak_inflight_bytes = st.peak_inflight_bytes;
  out->slot_bytes = s->slot_bytes;
  return TRK_OK;
}

int trk_service_start(trk_server* srv, const char* host, int port, trk_service** out, int* bound_port) {
  if (!srv || !out || port < 0 || port > 65535) return TRK_E_INVAL;
  *out = nullptr;
  trk_service* t = new trk_service();
  t->backend.s = srv;
  t->svc = new trk_net::Service<ServerBackend>(&t->backend, srv->max_hits);
  if (t->svc->start(host, port, bound_port) != 0) {
    delete t->svc;
    delete t;
    return TRK_E_INVAL;
  }
  *out = t;
  return TRK_OK;
}

void trk_service_stop(trk_service* t) {
  if (!t) return;
  t->svc->stop();
  delete t->svc;
  delete t;
}

void trk_server_destroy(trk_server* s) {
  if (!s) return;
  if (s->core) {
    s->core->shutdown();
    delete s->core;
  }
  hipSetDevice(s->exec.device);
  free_slots(s);
  delete s;
}

}  // extern "C"
