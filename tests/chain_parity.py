"""End-to-end parity of the GPU chain with the FP64 oracle (Section 2.2.2 chain).

The GPU chain is run twice: as one trk_event call and as the staged calls
(embed, build_graph, filter, gnn, components), and the two must give identical
labels and counts.  The oracle's chain is then followed step by step on the same
event, taking the GPU's decision only where the oracle's own value lies within
the stated tolerance of a threshold:

  * radius test and K-cap: a pair may differ only if its oracle distance is
    within the band of r or of a saturated point's K-th distance; the band is the
    FP32 distance band widened by the bound 2 sqrt(D) max|emb_gpu - emb_oracle|
    on how far the GPU's embedding moves a distance;
  * filter cut: every score within `score_tol` of the oracle's filter on the GPU's
    own embedding (itself checked against the oracle's), and the GPU's keep decision
    equal to the oracle's on every edge whose oracle score is more than `score_tol`
    from the cut;
  * interaction network and score cut: the same, on the GPU's filtered edges.

With those decisions the oracle's components must equal the GPU's labels bit for
bit.  Nothing here computes a side of a comparison: the numbers come from the
oracle's functions and from the library."""
import math

import numpy as np

import oracle
from tests.gpu_helpers import RADIUS_BAND, compare_edges


def staged(pipe, x):
    """The chain as separate entry-point calls (the GPU's intermediates)."""
    cfg = pipe.cfg
    n = x.shape[0]
    emb = pipe.embed(x)
    src, dst, nsat = pipe.build_graph(emb)
    pf, fs, fd = pipe.filter(emb, src, dst, cap=max(int(src.numel()), 1))
    q = pipe.gnn(x, fs, fd)
    labels = pipe.components(n, fs, fd, q, cfg.score_cut)
    out = dict(emb=emb, src=src, dst=dst, nsat=nsat, pf=pf, fsrc=fs, fdst=fd, q=q, labels=labels)
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


def chain_parity(pipe, x, nets, emb_tol, score_tol=1e-4, min_hits=3):
    """Asserts the whole-chain parity described above; returns the figures
    (margin counts, band differences, largest errors) for the record."""
    cfg = pipe.cfg
    x = np.asarray(x, np.float32)
    n = x.shape[0]
    g = staged(pipe, x)
    lab_ev, info = pipe.event(x)
    lab_ev = lab_ev.cpu().numpy()

    # (a) the one-call chain equals the staged calls
    assert np.array_equal(lab_ev, g["labels"]), "trk_event labels differ from the staged calls"
    assert info["n_cand_edges"] == g["src"].size and info["n_filt_edges"] == g["fsrc"].size
    assert info["n_kept_edges"] == int(np.sum(g["q"] > np.float32(cfg.score_cut)))
    assert info["n_saturated"] == g["nsat"]

    # embedding
    emb_o = oracle.embed(x, nets)
    d_emb = np.abs(g["emb"] - emb_o)
    rel = d_emb / np.maximum(1.0, np.abs(emb_o))
    assert rel.max() <= emb_tol, ("embedding", rel.max())

    # radius graph: differences only inside the widened bands
    rad = float(np.float32(cfg.radius))
    band = RADIUS_BAND + 2.0 * math.sqrt(cfg.emb_dim) * float(d_emb.max())
    lo, hi, d2 = oracle.radius_pairs(emb_o, rad)
    os_, od, cnt = oracle.radius_graph(emb_o, rad, cfg.k_max)
    ndiff, nbad, det = compare_edges(emb_o, g["src"], g["dst"], os_, od, rad, cfg.k_max, lo, hi, d2, band=band)
    assert nbad == 0, ("candidate edges outside the bands", det)
    assert abs(g["nsat"] - int((cnt > cfg.k_max).sum())) <= ndiff

    # filter on the GPU's candidate edges, fed the GPU's own embedding (checked above
    # against the oracle's): a filter that reads the small difference between an
    # edge's two ends multiplies the embedding's own FP32 error, so each stage is
    # compared on the same inputs, as in the stage tests; the figure on the oracle's
    # FP64 embedding is reported beside it
    pf_o = oracle.filter_scores(g["emb"], g["src"], g["dst"], nets)
    dpf = np.abs(g["pf"] - pf_o)
    assert dpf.size == 0 or dpf.max() <= score_tol, ("filter scores", dpf.max())
    pf_o64 = oracle.filter_scores(emb_o, g["src"], g["dst"], nets)
    dpf64 = np.abs(g["pf"] - pf_o64)
    cf = np.float32(cfg.filter_cut)
    keep_o = pf_o > cf
    keep_g = g["pf"] > cf
    margin_f = np.abs(pf_o - cf) <= score_tol
    assert np.array_equal(keep_g[~margin_f], keep_o[~margin_f]), "filter cut differs away from its margin"
    keep = np.where(margin_f, keep_g, keep_o)
    assert np.array_equal(g["fsrc"], g["src"][keep]) and np.array_equal(g["fdst"], g["dst"][keep])

    # interaction network on the GPU's filtered edges
    q_o = oracle.interaction_network(x, g["fsrc"], g["fdst"], nets, cfg.gnn_iters)
    dq = np.abs(g["q"] - q_o)
    assert dq.size == 0 or dq.max() <= score_tol, ("interaction-network scores", dq.max())
    sc = np.float32(cfg.score_cut)
    kept_o = q_o > sc
    kept_g = g["q"] > sc
    margin_s = np.abs(q_o - sc) <= score_tol
    assert np.array_equal(kept_g[~margin_s], kept_o[~margin_s]), "score cut differs away from its margin"
    kept = np.where(margin_s, kept_g, kept_o)

    # components of the substituted kept edges: identical labels
    lab_o = oracle.components(n, g["fsrc"][kept], g["fdst"][kept])
    assert np.array_equal(lab_ev, lab_o), "labels differ from the oracle's after the margin substitution"

    # for the record: how far the oracle's own chain is from the GPU's
    return dict(n=n, n_cand=int(g["src"].size), n_cand_oracle=int(os_.size), band_diffs=ndiff,
                n_filt=int(g["fsrc"].size), n_kept=info["n_kept_edges"],
                margin_filter=int(margin_f.sum()), margin_score=int(margin_s.sum()),
                flips_filter=int(np.sum(keep_g != keep_o)), flips_score=int(np.sum(kept_g != kept_o)),
                emb_rel_max=float(rel.max()), filter_dp_max=float(dpf.max()) if dpf.size else 0.0,
                filter_dp_max_on_fp64_embedding=float(dpf64.max()) if dpf64.size else 0.0,
                gnn_dp_max=float(dq.max()) if dq.size else 0.0,
                candidates=len(oracle.candidates(lab_ev, min_hits)))
