"""FP64 CPU oracle of the per-event tracking chain of Section 2.2.2.

TEST INFRASTRUCTURE ONLY.  Nothing in the library or its Python binding may
import or call this module; only the tests, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the HIP path.

The chain (Section 2.2.2): an MLP embeds each spacepoint's three features into a
latent space; a fixed-radius search in that space proposes edges; a second MLP
scores each edge and a fixed threshold removes clearly fake ones; an
interaction network (Battaglia et al., cited there) scores the remaining edges;
the edges whose score passes the cut are split into weakly connected components,
each component being one track candidate.  The paper gives no widths,
thresholds or activation choices; the readings taken here are:

  * every MLP is Lin -> tanh -> ... -> Lin, with Lin(u) = u W + b, W stored
    [fan_in, fan_out]; the embedding and filter end in a linear layer, the
    interaction-network MLPs apply tanh after every layer except the output
    head's last one;
  * the radius test is strict, d^2 < r^2, on squared Euclidean distance;
  * a spacepoint keeps at most K neighbours, the K smallest by (d^2, id), self
    excluded; the candidate edge set is the union of these selections as
    undirected pairs (min id, max id), sorted;
  * the filter sees [emb_src, emb_dst] with src < dst, keeps p > c_f in edge
    order; the final cut keeps p > 0.5;
  * message aggregation sums an edge's state into both endpoints;
  * a component is labelled with its smallest spacepoint id.

All arithmetic is float64 on the float32 inputs and weights (upcast exactly).
Every function is a plain transcription of its definition; library routines
(matrix product, KD-tree range query, sparse connected components) serve only
as single steps.
"""
import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

CHUNK = 65536


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def sigmoid(z):
    """Logistic function 1 / (1 + exp(-z)), evaluated without overflow."""
    z = _f64(z)
    out = np.empty_like(z)
    pos = z >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-z[pos]))
    ez = np.exp(z[~pos])
    out[~pos] = ez / (1.0 + ez)
    return out


def mlp(u, layers, tanh_last=False):
    """Feed-forward MLP: Lin, then tanh between layers (and after the last one
    when tanh_last).  Section 2.2.2 (embedding and filtering MLPs)."""
    h = _f64(u)
    for li, (w, b) in enumerate(layers):
        h = h @ _f64(w) + _f64(b)
        if li < len(layers) - 1 or tanh_last:
            h = np.tanh(h)
    return h


def embed(x, nets):
    """Embedding stage of Section 2.2.2: emb = MLP_emb(x), linear output."""
    return mlp(x, nets["emb"])


def _pair_d2(emb, i, j):
    d = _f64(emb)[i] - _f64(emb)[j]
    return np.einsum("ij,ij->i", d, d)


def radius_pairs(emb, radius):
    """All unordered pairs (i < j) with d^2(i, j) < r^2 and their d^2 in FP64.
    Fixed-radius graph construction, Section 2.2.2."""
    e = _f64(emb)
    r = float(radius)
    if e.shape[0] < 2:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0)
    tree = cKDTree(e)
    pairs = tree.query_pairs(r * (1.0 + 1e-9), output_type="ndarray").astype(np.int64)
    if pairs.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0)
    i, j = pairs[:, 0], pairs[:, 1]
    d2 = np.concatenate([_pair_d2(e, i[s:s + CHUNK * 16], j[s:s + CHUNK * 16])
                         for s in range(0, i.size, CHUNK * 16)])
    keep = d2 < r * r
    i, j, d2 = i[keep], j[keep], d2[keep]
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    return lo, hi, d2


def select_neighbours(n, lo, hi, d2, k_max):
    """Directed selections Sel(i): the k_max smallest neighbours of i by (d^2, j).
    Returns (i, j, d2, rank) of every selected directed pair and the count of
    within-radius neighbours per spacepoint."""
    qi = np.concatenate([lo, hi])
    qj = np.concatenate([hi, lo])
    qd = np.concatenate([d2, d2])
    order = np.lexsort((qj, qd, qi))          # by i, then d^2, then j
    qi, qj, qd = qi[order], qj[order], qd[order]
    count = np.bincount(qi, minlength=n).astype(np.int64)
    start = np.zeros(n + 1, np.int64)
    start[1:] = np.cumsum(count)
    rank = np.arange(qi.size, dtype=np.int64) - start[qi]
    sel = rank < k_max
    return qi[sel], qj[sel], qd[sel], rank[sel], count


def radius_graph(emb, radius, k_max):
    """Candidate edges E_c of Section 2.2.2 under the K-cap reading: union of the
    directed selections as canonical (min, max) pairs, sorted by (src, dst)."""
    n = _f64(emb).shape[0]
    lo, hi, d2 = radius_pairs(emb, radius)
    si, sj, _, _, count = select_neighbours(n, lo, hi, d2, k_max)
    a, b = np.minimum(si, sj), np.maximum(si, sj)
    key = np.unique(a * np.int64(n) + b)
    return (key // n).astype(np.int64), (key % n).astype(np.int64), count


def filter_scores(emb, src, dst, nets):
    """Filtering stage of Section 2.2.2: p_f = sigmoid(MLP_f([emb_src, emb_dst]))."""
    e = _f64(emb)
    out = np.empty(len(src), np.float64)
    for s in range(0, len(src), CHUNK):
        u = np.concatenate([e[src[s:s + CHUNK]], e[dst[s:s + CHUNK]]], axis=1)
        out[s:s + CHUNK] = sigmoid(mlp(u, nets["filt"])[:, 0])
    return out


def filter_edges(scores, src, dst, cut):
    """Fixed threshold of Section 2.2.2: keep p_f > cut, in edge order."""
    keep = _f64(scores) > cut
    return np.asarray(src)[keep], np.asarray(dst)[keep]


def interaction_network(x, src, dst, nets, iters, return_states=False):
    """Interaction-network edge classifier (Section 2.2.2; Battaglia et al.).

    h0 = phi_v0(x_i), e0 = phi_e0([x_s, x_t]); for t = 1..T:
        e^t = e^{t-1} + phi_e([h_s, h_t, e^{t-1}])
        m_i = sum of e^t over edges with i as either endpoint
        h^t = h^{t-1} + phi_v([h^{t-1}, m])
    score = sigmoid(phi_o([h_s, h_t, e^T])).  Returns scores (and states)."""
    x = _f64(x)
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    n = x.shape[0]
    h = mlp(x, nets["node_enc"], tanh_last=True)
    e = mlp(np.concatenate([x[src], x[dst]], axis=1), nets["edge_enc"], tanh_last=True)
    states = [(h, e)]
    for _ in range(iters):
        e = e + mlp(np.concatenate([h[src], h[dst], e], axis=1), nets["edge_net"], tanh_last=True)
        m = np.zeros_like(h)
        np.add.at(m, src, e)
        np.add.at(m, dst, e)
        h = h + mlp(np.concatenate([h, m], axis=1), nets["node_net"], tanh_last=True)
        states.append((h, e))
    z = mlp(np.concatenate([h[src], h[dst], e], axis=1), nets["out"])[:, 0]
    p = sigmoid(z)
    return (p, states) if return_states else p


def components(n, src, dst, scores=None, cut=0.5):
    """Weakly connected components of the graph of kept edges (Section 2.2.2),
    each spacepoint labelled with the smallest id in its component; a
    spacepoint on no kept edge is its own component."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    if scores is not None:
        keep = _f64(scores) > cut
        src, dst = src[keep], dst[keep]
    g = coo_matrix((np.ones(src.size, np.int8), (src, dst)), shape=(n, n)).tocsr()
    _, comp = connected_components(g, directed=False)
    first = np.full(comp.max() + 1 if n else 0, n, np.int64)
    np.minimum.at(first, comp, np.arange(n, dtype=np.int64))
    return first[comp].astype(np.int32)


def candidates(labels, min_hits=3):
    """Track candidates: the spacepoint-id sets of components with >= min_hits members."""
    labels = np.asarray(labels)
    order = np.argsort(labels, kind="stable")
    ls = labels[order]
    cuts = np.flatnonzero(np.diff(ls)) + 1
    groups = np.split(order, cuts)
    return [tuple(sorted(g.tolist())) for g in groups if len(g) >= min_hits]


def event(x, nets, cfg):
    """Whole per-event chain; returns every intermediate."""
    n = np.asarray(x).shape[0]
    emb = embed(x, nets)
    src, dst, count = radius_graph(emb, np.float32(cfg.radius), cfg.k_max)
    pf = filter_scores(emb, src, dst, nets)
    fs, fd = filter_edges(pf, src, dst, np.float32(cfg.filter_cut))
    p = interaction_network(x, fs, fd, nets, cfg.gnn_iters)
    labels = components(n, fs, fd, p, np.float32(cfg.score_cut))
    return dict(emb=emb, src=src, dst=dst, nbr_count=count, filter_scores=pf,
                fsrc=fs, fdst=fd, gnn_scores=p, labels=labels)
