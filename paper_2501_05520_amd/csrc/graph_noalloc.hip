// Allocation-free variant of the radius-graph entry point (Section 2.2.2: the
// fixed-radius search that proposes the candidate edges in the embedding space).
// It runs the same kernels as trk_build_graph, with every scratch buffer carved
// out of one file-scope device array instead of a context's arena, so that a
// caller that cannot allocate device memory can build the graph with no context
// and no allocation.  Each device holds its own copy of the array for the life of
// the process; its address is looked up once per device and kept.
#include <mutex>

#include "../../include/trk.h"
#include "kernels.h"

namespace {

constexpr int64_t kMaxHits = TRK_NOALLOC_MAX_HITS;
constexpr int64_t kMaxEdges = TRK_NOALLOC_MAX_EDGES;
constexpr int64_t kTable = 2 * kMaxHits;        // cell hash table (a power of two >= 2 kMaxHits)
constexpr int kStatsBlocks = 256;               // blocks of the covariance pass, 160 doubles each
constexpr int64_t kScanInts = 65536;            // scan partials (far more than any scan here needs)
static_assert((kTable & (kTable - 1)) == 0, "the cell table must be a power of two");

constexpr size_t pad256(size_t b) { return (b + 255) & ~(size_t)255; }

// byte sizes of the scratch pieces, in carving order
constexpr size_t kPieces[] = {
    pad256(8 * kMaxHits),                  // cell keys
    pad256(4 * kMaxHits),                  // hash buckets
    pad256(4 * kMaxHits),                  // ids in cell order
    pad256(64 * kMaxHits),                 // embedding rows in cell order (16 floats)
    pad256(8 * kMaxHits),                  // cell keys in cell order
    pad256(4 * kMaxHits),                  // within-r counts
    pad256(8 * kMaxHits),                  // selection threshold keys
    pad256(4 * (kMaxHits + 1)),            // row counts
    pad256(4 * (kMaxHits + 1)),            // row starts
    pad256(4 * kMaxHits),                  // row fill cursors
    pad256(4 * kMaxEdges),                 // unsorted destinations
    pad256(4 * kTable),                    // bucket histogram
    pad256(4 * (kTable + 1)),              // bucket starts
    pad256(4 * kTable),                    // bucket fill cursors
    pad256(8 * kStatsBlocks * 160),        // covariance partial sums
    pad256(8 * 64),                        // basis
    pad256(4 * 8),                         // counters
    pad256(4 * kScanInts),                 // scan partials
};
constexpr size_t total_bytes() {
  size_t t = 0;
  for (size_t b : kPieces) t += b;
  return t;
}
constexpr size_t kScratchBytes = total_bytes();

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// per device: the device address of `scratch` (host code never uses the symbol's
// name as an address) and the compute-unit count
constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};
int g_n_cu[kMaxDevices] = {};

int scratch_of_current_device(unsigned char** ptr, int* n_cu) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TRK_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TRK_E_DEVICE;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return TRK_E_DEVICE;
    g_n_cu[dev] = cu > 0 ? cu : 256;
    g_ptr[dev] = (unsigned char*)p;
  }
  *ptr = g_ptr[dev];
  *n_cu = g_n_cu[dev];
  return TRK_OK;
}

GraphScratch carve(unsigned char* base) {
  GraphScratch g;
  size_t off = 0;
  int i = 0;
  auto next = [&]() {
    unsigned char* p = base + off;
    off += kPieces[i++];
    return (void*)p;
  };
  g.cell = (unsigned long long*)next();
  g.bucket = (int*)next();
  g.sorted_id = (int*)next();
  g.sorted_emb = (float*)next();
  g.sorted_cell = (unsigned long long*)next();
  g.cnt = (int*)next();
  g.thr = (unsigned long long*)next();
  g.rowcnt = (int*)next();
  g.rowptr = (int*)next();
  g.cursor = (int*)next();
  g.unsorted = (int*)next();
  g.hist = (int*)next();
  g.start = (int*)next();
  g.fill = (int*)next();
  g.stats = (double*)next();
  g.basis = (double*)next();
  g.counters = (int*)next();
  g.tmp = (int*)next();
  g.table = kTable;
  g.stats_blocks = kStatsBlocks;
  return g;
}

}  // namespace

extern "C" int trk_build_graph_noalloc(const float* d_emb, int64_t n, int32_t emb_dim, float radius, int32_t k_max,
                                       int32_t* d_src, int32_t* d_dst, int64_t cap, int64_t* h_n_edges,
                                       int64_t* h_n_saturated, hipStream_t s) {
  if (!h_n_edges || n < 0 || cap < 0 || emb_dim < 1 || emb_dim > 16 || !(radius > 0.f) || k_max < 1 ||
      k_max > 1024)
    return TRK_E_INVAL;
  if (n > kMaxHits) return TRK_E_INVAL;
  if (n > 0 && (!d_emb || (cap > 0 && (!d_src || !d_dst)))) return TRK_E_INVAL;
  *h_n_edges = 0;
  if (h_n_saturated) *h_n_saturated = 0;
  if (n == 0) return TRK_OK;
  if (scan_tmp_ints(kTable) > kScanInts || scan_tmp_ints(kMaxHits + 1) > kScanInts) return TRK_E_DEVICE;
  unsigned char* base = nullptr;
  int n_cu = 0;
  const int rc = scratch_of_current_device(&base, &n_cu);
  if (rc) return rc;
  GraphScratch g = carve(base);
  const int64_t eff = cap < kMaxEdges ? cap : kMaxEdges;
  // every buffer that must start at zero is cleared by a fill kernel inside the launch
  launch_build_graph(d_emb, (int)n, emb_dim, radius, k_max, nullptr, g, d_src, d_dst, eff, n_cu, s);
  if (hipGetLastError() != hipSuccess) return TRK_E_DEVICE;
  int words[2] = {0, 0};
  if (hipMemcpyAsync(words, g.counters, sizeof(words), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return TRK_E_DEVICE;
  const int64_t total = (uint32_t)words[0];
  *h_n_edges = total;
  if (h_n_saturated) *h_n_saturated = words[1];
  return total > eff ? TRK_E_CAPACITY : TRK_OK;
}
