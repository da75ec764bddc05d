// Internal launcher declarations of libtrk.so (host side of each kernel file).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "layers.h"

// layer precisions (split BF16: FP32 values carried as two BF16 parts, see PrecX3)
enum { TRK_PREC_F32 = 0, TRK_PREC_BF16 = 1, TRK_PREC_FP8 = 2, TRK_PREC_X3 = 3 };
// bits of the device error word
enum { TRK_ERRBIT_CAPACITY = 1, TRK_ERRBIT_INDEX = 2 };

struct LayerList {
  DevLayer l[6];
  int n = 0;
};

// ---- mlp.hip ----
int launch_embed(int prec, int W, const float* x, int n, const DevLayer& l_in, const LayerList& hid,
                 const DevLayer& l_out, int D, float* emb, int n_cu, hipStream_t s);
int launch_filter(int prec, int W, const float* emb, int D, const int* src, const int* dst, int64_t m_host,
                  const int* d_m, int64_t cap, const DevLayer& l_in, const LayerList& hid, const DevVec& out,
                  float* scores, int n_nodes, int* d_err, int n_cu, hipStream_t s);

// ---- scan.hip ----
// Scratch needed by the scans / compactions for up to n elements (ints).
int64_t scan_tmp_ints(int64_t n);
// out[i] = sum_{j<i} in[j] for i <= n (out has n+1 entries; out[n] = total).
// n = min(*d_n, n_cap) if d_n, else n_cap.  Optional d_total receives the total.
void launch_scan_excl(const int* in, int* out, int64_t n_cap, const int* d_n, int* d_total, int* tmp,
                      hipStream_t s);
// Order-preserving compaction of edges with scores[e] > cut, e < m.
// m = min(*d_m, m_cap) if d_m else m_cap.  Writes *d_count = kept count (may exceed out_cap; only
// the first out_cap are written).
void launch_compact_edges(const float* scores, float cut, const int* src, const int* dst, int64_t m_cap,
                          const int* d_m, int* out_src, int* out_dst, int64_t out_cap, int* d_count, int* tmp,
                          hipStream_t s);
void launch_fill_int(int* p, int v, int64_t n, hipStream_t s);
void launch_set_int(int* p, int64_t v, hipStream_t s);

// ---- graph.hip ----
struct GraphScratch {
  // per spacepoint
  int* ev = nullptr;            // event id per hit (nullable: single event)
  float* proj = nullptr;        // [n][4] projected coordinates (xyz) + pad
  unsigned long long* cell = nullptr;  // [n] packed cell key
  int* bucket = nullptr;        // [n] hash bucket
  int* sorted_id = nullptr;     // [n]
  float* sorted_emb = nullptr;  // [n][16]
  unsigned long long* sorted_cell = nullptr;  // [n]
  int* cnt = nullptr;           // [n] within-r neighbour count
  unsigned long long* thr = nullptr;  // [n] selection threshold key (d2 bits << 32 | id)
  int* rowcnt = nullptr;        // [n+1]
  int* rowptr = nullptr;        // [n+1]
  int* cursor = nullptr;        // [n]
  int* unsorted = nullptr;      // [cap] dst of the unsorted rows
  // hash table
  int* hist = nullptr;          // [T]
  int* start = nullptr;         // [T+1]
  int* fill = nullptr;          // [T]
  int64_t table = 0;            // T (power of two)
  // basis
  double* stats = nullptr;      // block partial sums for mean / covariance
  double* basis = nullptr;      // [64]: three orthonormal directions (16 each), then the cell edge
  int* counters = nullptr;      // [8] device counters: 0 = E total, 1 = saturated, 2 = overflow
  int* tmp = nullptr;           // scan scratch
  int stats_blocks = 0;
};
// Builds the candidate graph of emb[n][D]; src/dst receive E = min(total, cap) rows; the device
// counter counters[0] receives the total (E may exceed cap: overflow).
void launch_build_graph(const float* emb, int n, int D, float radius, int k_max, const int* ev,
                        GraphScratch& g, int* src, int* dst, int64_t cap, int n_cu, hipStream_t s);

// ---- cc.hip ----
// labels[i] = min id of i's component over edges e < m (m from d_m if given) with scores[e] > cut
// (all if scores == nullptr).
void launch_components(int n, const int* src, const int* dst, const float* scores, float cut, int64_t m_cap,
                       const int* d_m, int* labels, int* d_kept, int* d_err, hipStream_t s);

// ---- gnn.hip ----
struct GnnScratch {
  float* h = nullptr;        // [n][H] node state fp32
  float* msg = nullptr;      // [n][H] aggregated messages fp32
  void* proj = nullptr;      // [n][2H] act type: per-node projections [h W1a | h W1b]
  void* e = nullptr;         // [cap][H] act type: edge state
  int* rowptr = nullptr;     // [n+1] CSR by src
  int* rowidx = nullptr;     // [cap] edge ids grouped by src, ascending
  int* cscptr = nullptr;     // [n+1] CSC by dst
  int* cscidx = nullptr;     // [cap] edge ids grouped by dst, ascending
  int* raw = nullptr;        // [cap] unsorted staging
  int* cnt = nullptr;        // [n] per-dst counts / cursors
  int* tmp = nullptr;        // scan scratch
};
// CSR (by src) and CSC (by dst) incidence lists of the edges into g, edge ids ascending per node
// src_sorted: the edges are ordered by source (ascending), so the source lists are
// edge ranges and need no construction
void launch_incidence(const int* src, const int* dst, int64_t m_cap, const int* d_m, int n, GnnScratch& g,
                      hipStream_t s, bool src_sorted = false);
int launch_gnn(int prec, const DevGNN& net, const float* x, int n, const int* src, const int* dst, int64_t m_cap,
               const int* d_m, float* scores, GnnScratch& g, int n_cu, int* d_err, hipStream_t s,
               bool src_sorted = false);

// segmented rank sort of unique int keys: for each segment [ptr[i], ptr[i+1]) of in, writes the
// keys ascending to out at the same positions.  n segments (from d_n if given).
void launch_segment_sort(const int* ptr, const int* in, int* out, int n, hipStream_t s);

// ---- fit.hip ----
// blocks of the stable radix sort that groups up to n hits by label
constexpr int FIT_SORT_CHUNK = 2048;
inline int64_t fit_sort_blocks(int64_t n) { return (n + FIT_SORT_CHUNK - 1) / FIT_SORT_CHUNK; }
