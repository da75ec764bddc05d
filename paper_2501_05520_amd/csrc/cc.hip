// Score cut and weakly connected components (Section 2.2.2: the GNN edge scores go
// to a weakly-connected-components step that forms the track candidates).
//
// Lock-free union-find over the kept edges.  parent[] starts as the identity; an
// edge whose score passes the cut finds the roots of its two ends and links the
// larger root under the smaller one with a compare-and-swap that succeeds only
// while the larger is still a root.  Every write (link or path halving) replaces
// a parent by an ancestor, so parent[x] <= x always holds and the root of every
// tree is its smallest member: after a final pass of pointer jumping, the label of
// each spacepoint is the smallest id of its component, whatever the order in which
// edges were processed.
#include "kernels.h"
#include "common.h"
#include <stdlib.h>

namespace {

// Plain loads suffice: a parent value only ever moves to an ancestor, so a stale
// cached value is still an ancestor and the walk still ends at a root (if that
// root is stale, the compare-and-swap below fails and returns the current value).
// (Device-scope atomic loads and stores, which would see the links made on the
// other XCDs at once, measured 1.7x slower on MI355X.)
__device__ __forceinline__ int uf_find(int* parent, int x) {
  int p = parent[x];
  while (p != x) {
    const int gp = parent[p];
    if (gp != p) parent[x] = gp;  // path halving: gp is an ancestor of x
    x = p;
    p = gp;
  }
  return x;
}

__device__ __forceinline__ void uf_union(int* parent, int a, int b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a > b) { const int t = a; a = b; b = t; }
    // link root b under root a if b is still a root
    const int old = atomicCAS(&parent[b], b, a);
    if (old == b) return;
    b = old;  // b gained a parent meanwhile: continue from there
  }
}

__global__ void uf_init(int* parent, int n) {
  GRID_STRIDE(i, n) parent[i] = (int)i;
}

// Initial forest: every spacepoint points at the smallest id among itself and its
// kept neighbours with smaller ids (parent[x] <= x, same component), which links most
// of each component before the union pass.
__global__ void uf_init_min(int* parent, const int* __restrict__ src, const int* __restrict__ dst,
                            const float* __restrict__ scores, float cut, int64_t m_cap, const int* d_m, int n) {
  const int64_t m = d_m ? clamp_count(d_m, m_cap) : m_cap;
  GRID_STRIDE(e, m) {
    if (!scores || scores[e] > cut) {
      const int a = src[e], b = dst[e];
      if ((unsigned)a < (unsigned)n && (unsigned)b < (unsigned)n && a != b) {
        const int hi = a > b ? a : b, lo = a > b ? b : a;
        // a parent only decreases, so a (possibly stale) value <= lo makes the atomic moot
        if (parent[hi] > lo) atomicMin(&parent[hi], lo);
      }
    }
  }
}

// One round of root hooking: each kept edge whose ends have different parents
// points the larger parent at the smaller one (atomicMin keeps parent[x] <= x and
// the smaller candidate when several edges hook the same root).  After pointer
// jumping every spacepoint points at a root again; a few such rounds link most of
// each component using only fire-and-forget atomics, and the compare-and-swap
// pass below completes what is left.
__global__ void uf_hook_min(int* parent, const int* __restrict__ src, const int* __restrict__ dst,
                            const float* __restrict__ scores, float cut, int64_t m_cap, const int* d_m, int n) {
  const int64_t m = d_m ? clamp_count(d_m, m_cap) : m_cap;
  const int l = lane_id();
  // whole waves step through the edges together (the combining below needs every lane)
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < m; base += stride) {
    const int64_t e = base + l;
    int tgt = -1, val = 0x7fffffff;
    if (e < m && (!scores || scores[e] > cut)) {
      const int a = src[e], b = dst[e];
      if ((unsigned)a < (unsigned)n && (unsigned)b < (unsigned)n) {
        const int pa = parent[a], pb = parent[b];
        if (pa != pb) {
          tgt = pa > pb ? pa : pb;
          val = pa > pb ? pb : pa;
        }
      }
    }
    // edges are ordered by source, so neighbouring lanes often hook the same root:
    // runs of equal targets take their minimum by a segmented scan and only the
    // run's last lane issues the atomic
    // segmented inclusive min-scan; a run starts at lane 0 or where the target changes
    const int t_prev = __shfl_up(tgt, 1, 64);
    int head = (l == 0 || t_prev != tgt) ? 1 : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v_o = __shfl_up(val, o, 64), h_o = __shfl_up(head, o, 64);
      if (l >= o) {
        if (!head && v_o < val) val = v_o;
        head |= h_o;
      }
    }
    const int t_next = __shfl_down(tgt, 1, 64);
    const bool last = l == 63 || t_next != tgt;
    // skip the atomic when the target already points at val or lower (parents only
    // decrease, so a stale read errs on the side of issuing it)
    if (tgt >= 0 && last && parent[tgt] > val) atomicMin(&parent[tgt], val);
  }
}

__global__ void uf_hook(int* parent, const int* __restrict__ src, const int* __restrict__ dst,
                        const float* __restrict__ scores, float cut, int64_t m_cap, const int* d_m, int n,
                        int* d_kept, int* d_err) {
  const int64_t m = d_m ? clamp_count(d_m, m_cap) : m_cap;
  int kept = 0;
  GRID_STRIDE(e, m) {
    if (!scores || scores[e] > cut) {
      const int a = src[e], b = dst[e];
      if ((unsigned)a >= (unsigned)n || (unsigned)b >= (unsigned)n) {
        if (d_err) atomicOr(d_err, TRK_ERRBIT_INDEX);
        continue;
      }
      ++kept;
      uf_union(parent, a, b);
    }
  }
  if (d_kept) {
    kept = wave_sum(kept);
    if (lane_id() == 0 && kept) atomicAdd(d_kept, kept);
  }
}

__global__ void uf_compress(int* parent, int n) {
  GRID_STRIDE(i, n) {
    // all links were made by earlier kernels, so every value read here is an
    // ancestor and the walk ends at the current root
    int x = (int)i;
    int p = parent[x];
    while (p != x) {
      x = p;
      p = parent[x];
    }
    parent[i] = x;
  }
}

// atomicMin rounds before the compare-and-swap pass
constexpr int kHookRounds = 4;

}  // namespace

void launch_components(int n, const int* src, const int* dst, const float* scores, float cut, int64_t m_cap,
                       const int* d_m, int* labels, int* d_kept, int* d_err, hipStream_t s) {
  if (n <= 0) return;
  uf_init<<<blocks_for(n, 256), 256, 0, s>>>(labels, n);
  if (m_cap > 0) {
    uf_init_min<<<blocks_for(m_cap, 256, 2048), 256, 0, s>>>(labels, src, dst, scores, cut, m_cap, d_m, n);
    // the initial forest has chains of decreasing ids; pointing every spacepoint at
    // the end of its chain first keeps the finds of the union pass short
    uf_compress<<<blocks_for(n, 256), 256, 0, s>>>(labels, n);
    for (int round = 0; round < kHookRounds; ++round) {
      uf_hook_min<<<blocks_for(m_cap, 256, 2048), 256, 0, s>>>(labels, src, dst, scores, cut, m_cap, d_m, n);
      uf_compress<<<blocks_for(n, 256), 256, 0, s>>>(labels, n);
    }
  }
  if (m_cap > 0)
    uf_hook<<<blocks_for(m_cap, 256, 2048), 256, 0, s>>>(labels, src, dst, scores, cut, m_cap, d_m, n, d_kept, d_err);
  uf_compress<<<blocks_for(n, 256), 256, 0, s>>>(labels, n);
}
