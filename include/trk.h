/*
 * trk.h - C ABI of the MI355X (gfx950) tracking-chain library libtrk.so.
 *
 * The per-event chain is the one of Section 2.2.2 of "Track reconstruction as a
 * service for collider physics" (arXiv:2501.05520): an embedding MLP over
 * spacepoints, a fixed-radius neighbour graph in the embedding space, an edge
 * filter MLP with a fixed threshold, an interaction-network edge classifier,
 * and a score cut followed by weakly connected components that turn the kept
 * edges into track candidates.  The lifecycle (create with configuration,
 * weights and device; execute per request; destroy) follows the custom-backend
 * lifecycle of Section 4.1.
 *
 * Conventions shared by every entry point
 *  - Return value: TRK_OK (0) or a negative trk_status.  trk_strerror() names it.
 *  - Arguments are validated on the host before anything is enqueued; on error
 *    nothing has been launched and outputs are untouched.
 *  - Pointers named d_* are device pointers (HBM of the context's device),
 *    owned by the caller, and must stay valid until the stream reaches the
 *    enqueued work.  Pointers named h_* are host pointers.
 *  - Work is enqueued on `stream` (NULL = the default stream).  Calls that
 *    return a count to the host (h_n_edges, h_n_kept, info) synchronise the
 *    stream before returning; the others do not.
 *  - Float data is IEEE float32, indices int32, row-major.
 *  - A context is used by one host thread at a time; its scratch memory is
 *    allocated once at creation from the max_* fields, so no entry point
 *    allocates device memory.
 *  - Capacity overflow is never truncated silently: the call returns
 *    TRK_E_CAPACITY and, where it has a count output, writes the required count.
 */
#ifndef TRK_H
#define TRK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRK_ABI_VERSION 1u
#define TRK_WEIGHTS_MAGIC 0x5754524Bu /* "KRTW" little-endian: 'K','R','T','W' */

typedef struct trk_ctx trk_ctx;

typedef enum {
  TRK_OK = 0,
  TRK_E_INVAL = -1,     /* bad argument: NULL pointer, size out of range, unsupported width */
  TRK_E_NOMEM = -2,     /* device allocation failed at trk_create */
  TRK_E_CAPACITY = -3,  /* an edge count exceeds the capacity given */
  TRK_E_DEVICE = -4,    /* a HIP runtime call failed */
  TRK_E_WEIGHTS = -5,   /* weight blob malformed or inconsistent with the configuration */
  TRK_E_EXPIRED = -7,   /* a served request's deadline passed before it was run */
  TRK_E_SHUTDOWN = -8,  /* the server is shutting down */
} trk_status;

typedef enum {
  TRK_FP32 = 0,  /* MLP and GNN matrix products in FP32 on MFMA */
  TRK_BF16 = 1,  /* matrix products in BF16 on MFMA, FP32 accumulation; activations stored BF16.
                  * The filter's first layer reads the FP32 mean and difference of the edge's two
                  * embeddings (rounded to BF16 after they are formed); the embedding's output
                  * layer runs in FP32 on the last hidden layer's FP32 values; the interaction
                  * network's encoders take the hit features in an FP32 first layer. */
  TRK_FP8 = 2,   /* the filter MLP's hidden layers in OCP FP8 E4M3 on MFMA with FP32 accumulation:
                  * weights with one power-of-two scale per tensor (largest |w| at most 448), tanh
                  * activations stored with the static scale 256; the interaction network's edge
                  * states and per-node projections stored as E4M3 with power-of-two scales fixed
                  * at creation from bounds, its edge-side products in FP8 and its node side in
                  * BF16; the filter's first layer and the embedding run as in TRK_BF16.  Needs
                  * emb_hidden and filt_hidden divisible by 128. */
  TRK_FP8_ALL = 3, /* TRK_FP8 plus the embedding MLP's hidden and output layers in FP8 */
  TRK_BF16_EMB32 = 4, /* filter and interaction network as in TRK_BF16, the embedding in FP32: the
                       * candidate graph is the FP32 one (the radius test is the step most
                       * sensitive to the embedding's precision) */
  TRK_BF16X3 = 5, /* every matrix product on the BF16 MFMA units in split form: each FP32 operand
                   * is carried as hi = bf16(v) plus lo = bf16(v - hi) (within 2^-18 of v) and a
                   * product is hi*hi + hi*lo + lo*hi with FP32 accumulation; activations are
                   * stored as the two parts (4 bytes).  The narrow first MLP layers run in FP32. */
  TRK_BF16X3_GNN_BF16 = 6, /* embedding and filter as in TRK_BF16X3, the interaction network as in
                            * TRK_BF16 (the score cut is the step least sensitive to precision) */
} trk_precision;

/* Model and sizing configuration, the analogue of a served model's config
 * (input shape, model, device; Section 4.1).  Network shapes:
 *   embedding  3 -> emb_hidden x emb_layers -> emb_dim        tanh on hidden layers
 *   filter     2*emb_dim -> filt_hidden x filt_layers -> 1    tanh on hidden layers
 *   interaction network, hidden H = gnn_hidden, gnn_iters message-passing steps:
 *     node encoder [3,H,H], edge encoder [6,H,H], edge network [3H,H,H],
 *     node network [2H,H,H] (tanh after every layer), output [3H,H,1].
 * Supported: emb_hidden in {64,1024}, emb_layers >= 1, emb_dim in 1..16,
 * filt_hidden in {64,512}, filt_layers >= 1, gnn_hidden in {32,128}, gnn_iters >= 0,
 * 1 <= k_max <= 1024, radius > 0. */
typedef struct {
  uint32_t abi_version;       /* TRK_ABI_VERSION */
  int32_t emb_hidden, emb_layers, emb_dim;
  int32_t filt_hidden, filt_layers;
  int32_t gnn_hidden, gnn_iters;
  float radius;               /* fixed radius r: an edge needs d^2 < r^2 */
  int32_t k_max;              /* at most k_max neighbours per spacepoint (nearest by (d^2, id)) */
  float filter_cut;           /* filter keeps p_f > filter_cut */
  float score_cut;            /* components use edges with p > score_cut */
  int32_t precision;          /* trk_precision */
  int64_t max_hits;           /* largest spacepoint count of one call (sum over a batch) */
  int64_t max_cand_edges;     /* capacity of candidate edges (radius graph) */
  int64_t max_kept_edges;     /* capacity of filtered edges (GNN input) */
  int32_t max_events;         /* largest batch of trk_batch */
  int32_t stage_timing;       /* non-zero: trk_event / trk_batch time each stage with HIP events */
  int32_t training;           /* non-zero: allocate the training buffers (TRK_FP32 or TRK_BF16 only) */
} trk_config;

/* Per-call counts reported by trk_event / trk_batch (all host memory). */
typedef struct {
  int64_t n_hits;
  int64_t n_cand_edges;       /* |E_c| */
  int64_t n_filt_edges;       /* |E_f| */
  int64_t n_kept_edges;       /* edges with GNN score > score_cut */
  int64_t n_saturated;        /* spacepoints with more than k_max neighbours within r */
  /* with stage_timing: milliseconds per stage, measured on the stream:
   * 0 embedding, 1 radius graph, 2 filter MLP, 3 filter cut (compaction),
   * 4 interaction network, 5 score cut + components; zero otherwise */
  float stage_ms[8];
} trk_event_info;

/* Weight blob: header of 16 uint32 (magic, abi_version, then the seven network
 * widths emb_hidden, emb_layers, emb_dim, filt_hidden, filt_layers, gnn_hidden,
 * gnn_iters, rest zero) followed by float32 tensors, each layer as W[fan_in][fan_out]
 * row-major then b[fan_out], networks in the order embedding, filter, node
 * encoder, edge encoder, edge network, node network, output head. */

/* Creates a context on device `device_id`: copies the weights (the blob is read
 * only during the call), derives the kernels' device layouts and precision
 * copies, and allocates all scratch memory.  Errors: TRK_E_INVAL (config),
 * TRK_E_WEIGHTS (blob), TRK_E_NOMEM, TRK_E_DEVICE. */
int trk_create(const trk_config* cfg, const void* h_weights, size_t nbytes, int device_id,
               trk_ctx** out);

/* Waits for the work this context enqueued (not for other contexts or streams) and
 * frees everything it owns.  NULL is a no-op.  Calls on one context are ordered:
 * a call on a stream other than the previous call's waits for that call's work,
 * since both use the context's scratch memory. */
void trk_destroy(trk_ctx* ctx);

/* Embedding (Section 2.2.2): d_emb[n][emb_dim] = MLP_emb(d_x[n][3]).  0 <= n <= max_hits. */
int trk_embed(trk_ctx* ctx, const float* d_x, int64_t n, float* d_emb, hipStream_t stream);

/* Fixed-radius graph (Section 2.2.2): candidate edges of the embedding
 * d_emb[n][emb_dim].  Spacepoint i selects the k_max nearest j != i with
 * d^2(i,j) < r^2 (FP32, ties by lower id); the output is the union of the
 * selections as undirected pairs src < dst, sorted by (src, dst), written to
 * d_src[0..E) and d_dst[0..E).  *h_n_edges receives E (synchronises).  If E > cap
 * returns TRK_E_CAPACITY with *h_n_edges = E and the outputs undefined.
 * h_n_saturated (optional) receives the count of spacepoints with more than k_max
 * neighbours within r. */
int trk_build_graph(trk_ctx* ctx, const float* d_emb, int64_t n, int32_t* d_src, int32_t* d_dst,
                    int64_t cap, int64_t* h_n_edges, int64_t* h_n_saturated, hipStream_t stream);

/* Allocation-free radius graph, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Computes exactly what trk_build_graph computes, with the graph
 * constants passed in instead of read from a context: emb_dim in [1, 16],
 * radius > 0, k_max in [1, 1024].  It needs no context and calls no allocating
 * routine: all of its scratch (35.2 MB) is one file-scope device array that
 * each device holds for the life of the process; its device address is looked up
 * on the first call on a device (the calling thread's current device, which
 * d_emb, d_src, d_dst and the stream must belong to).
 * Limits: n <= TRK_NOALLOC_MAX_HITS (else TRK_E_INVAL, nothing enqueued); at most
 * min(cap, TRK_NOALLOC_MAX_EDGES) edges are written: a larger total returns
 * TRK_E_CAPACITY with the total in *h_n_edges (as trk_build_graph does for cap).
 * Synchronises the stream.  Calls that overlap on one device share the array and
 * race: the caller serialises them (one stream, or its own ordering). */
#define TRK_NOALLOC_MAX_HITS 131072
#define TRK_NOALLOC_MAX_EDGES 4194304
int trk_build_graph_noalloc(const float* d_emb, int64_t n, int32_t emb_dim, float radius, int32_t k_max,
                            int32_t* d_src, int32_t* d_dst, int64_t cap, int64_t* h_n_edges,
                            int64_t* h_n_saturated, hipStream_t stream);

/* Edge filter (Section 2.2.2): p_f = sigmoid(MLP_f([emb_src, emb_dst])) for the m
 * edges (d_src, d_dst); writes d_scores[m] when non-NULL; copies the edges with
 * p_f > filter_cut, in input order, to d_kept_src/d_kept_dst and their count to
 * *h_n_kept (synchronises).  Kept count > cap: TRK_E_CAPACITY with *h_n_kept set.
 * Edge endpoints must lie in [0, n). */
int trk_filter(trk_ctx* ctx, const float* d_emb, int64_t n, const int32_t* d_src,
               const int32_t* d_dst, int64_t m, float* d_scores, int32_t* d_kept_src,
               int32_t* d_kept_dst, int64_t cap, int64_t* h_n_kept, hipStream_t stream);

/* Interaction network (Section 2.2.2, after Battaglia et al.): edge scores
 * d_scores[m] in (0,1) for the m edges (d_src, d_dst) over spacepoints d_x[n][3].
 * m <= max_kept_edges; endpoints in [0, n). */
int trk_gnn(trk_ctx* ctx, const float* d_x, int64_t n, const int32_t* d_src, const int32_t* d_dst,
            int64_t m, float* d_scores, hipStream_t stream);

/* Score cut and weakly connected components (Section 2.2.2): over the graph of
 * the m edges with d_scores[e] > cut (all m edges if d_scores is NULL),
 * d_labels[i] = the smallest spacepoint id in i's component. */
int trk_components(trk_ctx* ctx, int64_t n, const int32_t* d_src, const int32_t* d_dst,
                   const float* d_scores, int64_t m, float cut, int32_t* d_labels,
                   hipStream_t stream);

/* The whole chain for one event (Section 2.2.2, one request of Section 4.1):
 * d_x[n][3] -> d_labels[n], stages chained with device-resident counts and no
 * host round trip in between.  Synchronises the stream before returning, to
 * report overflow (TRK_E_CAPACITY) and, when info is non-NULL, the counts. */
int trk_event(trk_ctx* ctx, const float* d_x, int64_t n, int32_t* d_labels, trk_event_info* info,
              hipStream_t stream);

/* A batch of independent events packed back to back: event b owns spacepoints
 * [h_offsets[b], h_offsets[b+1]) of d_x.  One launch sequence serves the whole
 * batch; no edge joins two events.  d_labels[i] is the smallest id, counted from
 * the start of i's own event, in i's component, so each event's labels equal those
 * of trk_event on that event alone.  infos (optional) receives one record per
 * event.  Synchronises like trk_event. */
int trk_batch(trk_ctx* ctx, int32_t n_events, const float* d_x, const int64_t* h_offsets,
              int32_t* d_labels, trk_event_info* infos, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Serving loop: the analogue of the inference server of Section 2.3 (clients
 * send requests, the server batches them and runs them on its GPU) and of the
 * concurrent model instances of Section 4.2.1, in process.  Client threads submit
 * events (host memory); a request is admitted once the memory estimate of all
 * admitted, unfinished requests fits mem_budget_bytes (submission blocks until
 * then; a request whose estimate alone exceeds the budget is refused with
 * TRK_E_CAPACITY).  n_slots workers each own a context, a stream and staging
 * buffers; a free worker takes the queued requests in arrival order, up to
 * max_batch_events events and max_batch_hits spacepoints, and runs them as one
 * trk_batch, so requests arriving while batches run join the next batch and work of
 * different batches overlaps on the device.  Labels equal those of trk_event on
 * each event alone.  All server calls are thread-safe.
 * ---------------------------------------------------------------------- */
typedef struct trk_server trk_server;

typedef struct {
  int32_t n_slots;            /* concurrent batches, 1..16 */
  int32_t max_batch_events;   /* events per batch, 1..65535 */
  int64_t max_batch_hits;     /* spacepoints per batch (also the largest single request) */
  int64_t max_cand_edges;     /* per-slot capacities (0: max_batch_hits * k_max) */
  int64_t max_kept_edges;     /* (0: same as max_cand_edges) */
  uint64_t mem_budget_bytes;  /* admission budget over admitted, unfinished requests */
  uint64_t bytes_per_hit;     /* admission estimate per spacepoint (0: slot memory / max_batch_hits) */
} trk_server_config;

typedef struct {
  int64_t submitted, completed, rejected, expired, batches, batched_events;
  int64_t admitted_at_once, waited_for_memory;
  uint64_t inflight_bytes, peak_inflight_bytes;
  uint64_t slot_bytes;        /* device memory of one slot (context arena + weights + staging) */
} trk_server_info;

/* Creates a server with n_slots contexts on device_id; cfg's max_hits,
 * max_events and capacities are taken from scfg.  Errors as trk_create. */
int trk_server_create(const trk_config* cfg, const void* h_weights, size_t nbytes, int device_id,
                      const trk_server_config* scfg, trk_server** out);

/* Copies h_x[n][3] and enqueues it; *ticket identifies the request.  Blocks while
 * the budget is full.  deadline_ms > 0: the request expires (TRK_E_EXPIRED at
 * trk_server_wait) if not batched within that time.  n > max_batch_hits:
 * TRK_E_CAPACITY. */
int trk_server_submit(trk_server* srv, const float* h_x, int64_t n, double deadline_ms, int64_t* ticket);

/* Waits for a request and releases its ticket: writes h_labels[n] (host), the
 * counts and stage times (info, optional) and the latency from submission to
 * completion in ms (optional); returns the request's status. */
int trk_server_wait(trk_server* srv, int64_t ticket, int32_t* h_labels, trk_event_info* info,
                    double* latency_ms);

int trk_server_stats(trk_server* srv, trk_server_info* out);

/* Drains (runs every admitted request), stops the workers and frees the slots;
 * tickets not yet waited for are released.  Stop every service of the server first. */
void trk_server_destroy(trk_server* srv);

/* ------------------------------------------------------------------------
 * Roofline denominators measured on the device (not part of the chain; the
 * benchmark reports its fractions against these beside the spec-sheet peaks).
 * trk_probe_mfma: dense matrix-core rate of `precision` (TRK_FP32, TRK_BF16 or
 *   TRK_FP8: the v_mfma_f32_16x16x4_f32, 16x16x32_bf16 and 16x16x128 E4M3 forms the
 *   kernels use) from independent MFMA chains on every CU, `iters` steps each;
 *   *tflops (host) receives FLOP/s / 1e12.  Synchronous; allocates and frees a
 *   small result buffer.  TRK_E_INVAL for another precision or iters < 1.
 * trk_probe_copy: HBM bandwidth of a coalesced 16-byte copy of `bytes` (a
 *   multiple of 16, both pointers 16-byte aligned, device, caller-owned) from
 *   d_src to d_dst, `reps` times on `stream`; *gbps (host) = 2 * bytes * reps /
 *   time / 1e9 (read plus write).  Synchronises the stream.
 * ---------------------------------------------------------------------- */
int trk_probe_mfma(int device_id, int precision, int64_t iters, double* tflops);
int trk_probe_copy(const void* d_src, void* d_dst, size_t bytes, int reps, hipStream_t stream, double* gbps);

/* ------------------------------------------------------------------------
 * Downstream helix fit of track candidates (what consumes the chain's output,
 * Section 2.2.2): every label value carried by at least min_hits spacepoints of
 * d_x[n][3] (the chain's features, rho/1000 mm, phi/pi, z/1000 mm) is a candidate.
 * Per candidate, in ascending label order: the algebraic least-squares circle in
 * the transverse plane and the least-squares line z = z0 + s tan(lambda) over the
 * transverse arc length s, for a solenoid field of b_field_t tesla along z.
 * Outputs (device, caller-owned, capacity cap): d_cand_label[c], d_cand_nhits[c],
 * d_params[c][6] = (pT GeV, phi0 at the point of closest approach to the origin,
 * eta, z0 mm, charge +-1, mean squared transverse residual mm^2) in FP64.
 * *n_cands (host) = number of candidates; more than cap: TRK_E_CAPACITY (nothing
 * beyond cap written).  Labels must lie in [0, n) (trk_event's do), else
 * TRK_E_INVAL.  Hits with collinear or coincident transverse positions give NaN.
 * Synchronises the stream.
 * ---------------------------------------------------------------------- */
int trk_fit(trk_ctx* ctx, const float* d_x, int64_t n, const int32_t* d_labels, int32_t min_hits,
            double b_field_t, int32_t* d_cand_label, int32_t* d_cand_nhits, double* d_params, int64_t cap,
            int64_t* n_cands, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Out-of-process front end of a server (the network side of an inference
 * server, Section 2.3; Section 4 measures what the transfer adds): a TCP listener
 * on host:port (IPv4 dotted address, NULL = 127.0.0.1; port 0 = any free port,
 * written to *bound_port).  Each connection is served by its own thread, its
 * requests in order; requests of different connections meet in the server's
 * scheduler.  Wire format, little-endian:
 *   request : u32 0x5154524B, u32 0, i64 n, f64 deadline_ms, f32 x[n][3]
 *   response: u32 0x5254524B, i32 status, i64 n, f64 latency_ms (submission to
 *             completion), i64 counts[5] (n_hits, n_cand_edges, n_filt_edges,
 *             n_kept_edges, n_saturated), f32 stage_ms[8], then i32 labels[n] if
 *             status == 0
 * A bad magic, n < 0 or n > max_batch_hits gets status TRK_E_INVAL and the
 * connection is closed.  Returns TRK_E_INVAL when the address cannot be bound.
 * ---------------------------------------------------------------------- */
typedef struct trk_service trk_service;
int trk_service_start(trk_server* srv, const char* host, int port, trk_service** out, int* bound_port);

/* Stops listening, ends the connections (requests in progress complete) and frees
 * the service. */
void trk_service_stop(trk_service* svc);

/* ------------------------------------------------------------------------
 * Training of the filter MLP and the interaction network (contexts created with
 * training != 0, precision TRK_FP32 or TRK_BF16; in a TRK_BF16 context every product
 * of the forward and backward passes takes BF16 operands with FP32 accumulation,
 * while parameters, gradients, Adam moments and stored states stay FP32).
 * Objective, a reading of the training configuration:
 * binary cross-entropy with logits on truth labels, averaged over the candidate
 * edges (filter) and over the filtered edges (interaction network); the edge sets
 * are inputs held fixed.  Parameters live in one flat FP32 device vector: the
 * networks filter, node encoder, edge encoder, edge network, node network,
 * output head and embedding, each layer as W[fan_in][fan_out] then b[fan_out].  Gradients use the same layout.  A *_bwd call
 * uses the state of the preceding *_fwd call of the same context on the same
 * edges, and adds its gradients to d_grads.  The interaction-network backward
 * stores only the per-iteration node and edge states in the forward pass and
 * recomputes each iteration's internals during the backward pass.
 * ---------------------------------------------------------------------- */

/* Embedding (metric learning), a reading of the paper's statement that hits of
 * one particle end up close together in the latent space: pairs (a, b) labelled
 * y = 1 (same particle) or 0, objective
 *   L = mean_{y=1} d^2 + mean_{y=0} max(0, margin - d)^2,  d = |emb_a - emb_b|.
 * The embedding layers follow the output head in the flat parameter vector. */

/* Number of floats of the flat parameter (and gradient) vector. */
int64_t trk_train_param_count(const trk_config* cfg);

/* Loads the flat parameter vector (device) into every kernel layout of the
 * context, the inference path included; synchronises the stream. */
int trk_train_set_params(trk_ctx* ctx, const float* d_params, hipStream_t stream);

/* Filter logits z_f[m] of the edges (d_src, d_dst) over d_emb[n][emb_dim], keeping
 * the activations; m <= max_cand_edges. */
int trk_filter_train_fwd(trk_ctx* ctx, const float* d_emb, int64_t n, const int32_t* d_src,
                         const int32_t* d_dst, int64_t m, float* d_logits, hipStream_t stream);
/* Adds dL/dparams of the filter, given dL/dz_f[m], to d_grads. */
int trk_filter_train_bwd(trk_ctx* ctx, const float* d_emb, int64_t n, const int32_t* d_src,
                         const int32_t* d_dst, int64_t m, const float* d_dlogits, float* d_grads,
                         hipStream_t stream);
/* Interaction-network logits z_o[m], keeping the per-iteration states; m <= max_kept_edges. */
int trk_gnn_train_fwd(trk_ctx* ctx, const float* d_x, int64_t n, const int32_t* d_src,
                      const int32_t* d_dst, int64_t m, float* d_logits, hipStream_t stream);
/* Adds dL/dparams of the five interaction-network MLPs, given dL/dz_o[m], to d_grads. */
int trk_gnn_train_bwd(trk_ctx* ctx, const float* d_x, int64_t n, const int32_t* d_src,
                      const int32_t* d_dst, int64_t m, const float* d_dlogits, float* d_grads,
                      hipStream_t stream);
/* Embedding d_emb[n][emb_dim] of d_x[n][3], keeping the activations. */
int trk_embed_train_fwd(trk_ctx* ctx, const float* d_x, int64_t n, float* d_emb, hipStream_t stream);
/* Adds dL/dparams of the embedding, given dL/demb[n][emb_dim], to d_grads. */
int trk_embed_train_bwd(trk_ctx* ctx, const float* d_x, int64_t n, const float* d_demb, float* d_grads,
                        hipStream_t stream);
/* Pair objective of the embedding over npairs pairs (d_pa, d_pb, labels d_y in {0,1}),
 *   L = mean over positives of d^2 + neg_weight * mean over negatives of max(0, margin - d)^2
 * with d the distance of the two embeddings (metric learning: hits of one particle close
 * together in the latent space, Section 2.2.2); writes dL/demb into d_demb[n][emb_dim]
 * (overwritten) and, if h_loss, the loss (synchronises).  npairs <= max_cand_edges;
 * margin and neg_weight >= 0, else TRK_E_INVAL. */
int trk_pair_loss(trk_ctx* ctx, const float* d_emb, int64_t n, const int32_t* d_pa, const int32_t* d_pb,
                  const float* d_y, int64_t npairs, float margin, float neg_weight, float* d_demb,
                  float* h_loss, hipStream_t stream);
/* Mean binary cross-entropy with logits of z[m] against targets y[m] in {0,1}:
 * writes dL/dz = (sigmoid(z) - y) / m and, if h_loss, the loss (synchronises). */
int trk_bce_with_logits(trk_ctx* ctx, const float* d_logits, const float* d_targets, int64_t m,
                        float* d_dlogits, float* h_loss, hipStream_t stream);
/* One Adam step (Kingma and Ba) over count parameters with bias correction for
 * step >= 1; d_m and d_v are the moment vectors (start at zero). */
int trk_adam_update(trk_ctx* ctx, float* d_params, const float* d_grads, float* d_m, float* d_v,
                    int64_t count, float lr, float beta1, float beta2, float eps, int64_t step,
                    hipStream_t stream);

/* Static description of a status code. */
const char* trk_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* TRK_H */
