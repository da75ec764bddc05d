"""GPU parity of the split-BF16 mode (TRK_BF16X3: every product formed on the
BF16 matrix cores from the high and low BF16 parts of FP32 values) against the
FP64 oracle, held to the FP32 bars: scores within 1e-4, labels identical away
from the cuts.  The embedding carries the split's own error (each operand within
2^-18 relatively, against 2^-24 for FP32), so it gets a looser bound, and the
candidate graph is compared on the oracle's own embedding (stage-isolated).  At
pile-up 200 the embedding of every hit, sampled filter scores and a one-step
interaction network on ~1M edges are checked against the oracle at the same bars,
and the chain's labels are compared with the FP32 chain's."""
import numpy as np
import pytest
import torch

import oracle
from gen import TINY, MU200, make_weights, generate_event
from tests.chain_parity import chain_parity
from tests.gpu_helpers import label_agreement

pytestmark = pytest.mark.gpu

SCORE_TOL = 1e-4
# split operands carry 2^-18 relative error each, so a product term is off by at most
# about 3 * 2^-18 = 1.1e-5 of |w x|; a 1024-term sum of random-sign terms is about
# sqrt(1024) / 3 ~ 10 times smaller than the sum of its magnitudes, which puts the
# error of a wide layer's output near 1e-4 of its value in the worst case
EMB_TOL = 2e-4
SEEDS = [1, 2, 3, 4]


@pytest.fixture(scope="module")
def tiny_nets():
    return make_weights(TINY, 0)


@pytest.fixture(scope="module")
def tiny_pipe(tiny_nets):
    from paper_2501_05520_amd.trk import Pipeline
    p = Pipeline(TINY, tiny_nets, "bf16x3", max_hits=8192, max_events=4)
    yield p
    p.close()


@pytest.fixture(scope="module")
def tiny_ref(tiny_nets):
    out = {}
    for s in SEEDS:
        ev = generate_event(s, 1)
        out[s] = (ev, oracle.event(ev.x, tiny_nets, TINY))
    return out


@pytest.mark.parametrize("seed", SEEDS)
def test_tiny_stages(tiny_pipe, tiny_ref, tiny_nets, seed):
    ev, r = tiny_ref[seed]
    emb = tiny_pipe.embed(ev.x).cpu().numpy()
    de = np.abs(emb - r["emb"]) / np.maximum(1.0, np.abs(r["emb"]))
    assert de.max() <= EMB_TOL, de.max()
    e32 = r["emb"].astype(np.float32)
    p = tiny_pipe.filter(e32, r["src"], r["dst"])[0].cpu().numpy()
    assert np.abs(p - r["filter_scores"]).max() <= SCORE_TOL
    q = tiny_pipe.gnn(ev.x, r["fsrc"], r["fdst"]).cpu().numpy()
    assert np.abs(q - r["gnn_scores"]).max() <= SCORE_TOL


@pytest.mark.parametrize("seed", SEEDS)
def test_tiny_end_to_end(tiny_pipe, tiny_ref, tiny_nets, seed):
    """The split-BF16 chain end to end, held to the FP32 bars: trk_event equals the
    staged calls, and the oracle's chain with the GPU's decision taken only on
    margin edges (and on candidate pairs within the embedding error of the radius or
    K-th distance) gives identical labels; no fallback."""
    ev, r = tiny_ref[seed]
    st = chain_parity(tiny_pipe, ev.x, tiny_nets, EMB_TOL, SCORE_TOL)
    print(f"bf16x3 tiny seed {seed}: {st}")


@pytest.fixture(scope="module")
def mid():
    nets = make_weights(MU200, 0)
    ev = generate_event(300, 10)
    return nets, ev, oracle.event(ev.x, nets, MU200)


def test_mid_stages_full_network(mid):
    """Pile-up-10 event through the full-size network (embedding 3-1024x3-12, filter
    24-512x3-1, H=128 T=8), every stage against the oracle."""
    from paper_2501_05520_amd.trk import Pipeline
    nets, ev, r = mid
    p = Pipeline(MU200, nets, "bf16x3", max_hits=8192)
    emb = p.embed(ev.x).cpu().numpy()
    e32 = r["emb"].astype(np.float32)
    pf = p.filter(e32, r["src"], r["dst"])[0].cpu().numpy()
    q = p.gnn(ev.x, r["fsrc"], r["fdst"]).cpu().numpy()
    labels, info = p.event(ev.x)
    p.close()
    de = np.abs(emb - r["emb"]) / np.maximum(1.0, np.abs(r["emb"]))
    dpf, dq = np.abs(pf - r["filter_scores"]), np.abs(q - r["gnn_scores"])
    hit, jac = label_agreement(labels.cpu().numpy(), r["labels"])
    print(f"bf16x3 vs fp64 oracle: emb rel max {de.max():.3g}; filter |dp| max {dpf.max():.3g}; "
          f"gnn |dp| max {dq.max():.3g}; cand edges {info['n_cand_edges']} (oracle {r['src'].size}); "
          f"hit agreement {hit:.5f}")
    assert de.max() <= EMB_TOL
    assert dpf.max() <= SCORE_TOL and dq.max() <= SCORE_TOL
    assert hit >= 0.999


def test_mid_mixed_mode_filter_at_fp32_bar(mid):
    """TRK_BF16X3_GNN_BF16: embedding and filter in split BF16 (filter scores at the FP32
    bar), the interaction network in BF16 (its error reported)."""
    from paper_2501_05520_amd.trk import Pipeline
    nets, ev, r = mid
    p = Pipeline(MU200, nets, "bf16x3gnn16", max_hits=8192)
    e32 = r["emb"].astype(np.float32)
    pf = p.filter(e32, r["src"], r["dst"])[0].cpu().numpy()
    q = p.gnn(ev.x, r["fsrc"], r["fdst"]).cpu().numpy()
    p.close()
    dpf, dq = np.abs(pf - r["filter_scores"]), np.abs(q - r["gnn_scores"])
    print(f"bf16x3gnn16 vs fp64 oracle: filter |dp| max {dpf.max():.3g}; gnn |dp| max {dq.max():.3g} "
          f"p99 {np.percentile(dq, 99):.3g}")
    assert dpf.max() <= SCORE_TOL
    assert dq.max() < 0.2


@pytest.mark.parametrize("precision", ["bf16x3", "bf16x3gnn16"])
def test_mu200_agrees_with_fp32(precision):
    """The pile-up-200 chain in split BF16 against the FP32 chain: the track-candidate
    labels of at least 99.9 % of the hits are the same."""
    from paper_2501_05520_amd.trk import Pipeline
    nets = make_weights(MU200, 0)
    ev = generate_event(200, MU200.n_collisions)
    p32 = Pipeline(MU200, nets, "fp32", max_hits=ev.n)
    l32, i32 = p32.event(ev.x)
    l32 = l32.cpu().numpy()
    p32.close()
    px = Pipeline(MU200, nets, precision, max_hits=ev.n)
    lx, ix = px.event(ev.x)
    lx2, _ = px.event(ev.x)
    px.close()
    assert torch.equal(lx, lx2)
    hit, jac = label_agreement(lx.cpu().numpy(), l32)
    print(f"{precision} vs fp32 at mu=200: cand edges {ix['n_cand_edges']} vs {i32['n_cand_edges']}, filtered "
          f"{ix['n_filt_edges']} vs {i32['n_filt_edges']}, kept {ix['n_kept_edges']} vs {i32['n_kept_edges']}; "
          f"hit agreement {hit:.5f} jaccard {jac:.4f}")
    assert hit >= 0.999


# ------------------------------------------------- pile-up 200, sampled against the oracle
@pytest.fixture(scope="module")
def full_x3():
    from paper_2501_05520_amd.trk import Pipeline
    nets = make_weights(MU200, 0)
    ev = generate_event(200, MU200.n_collisions)
    p = Pipeline(MU200, nets, "bf16x3", max_hits=ev.n)
    yield nets, ev, oracle.embed(ev.x, nets), p
    p.close()


def test_full_embed_every_hit(full_x3):
    """The split-BF16 embedding of all 110,000 hits against the FP64 oracle."""
    nets, ev, emb_ref, p = full_x3
    emb = p.embed(ev.x).cpu().numpy()
    de = np.abs(emb - emb_ref) / np.maximum(1.0, np.abs(emb_ref))
    print(f"bf16x3 mu=200 embedding: rel max {de.max():.3g}, p99 {np.percentile(de, 99):.3g}")
    assert de.max() <= EMB_TOL


def test_full_filter_sampled(full_x3):
    """Split-BF16 filter scores at full size (the candidate graph of the oracle's
    embedding, ~3M edges), 20,000 sampled edges against the oracle at the FP32 bar."""
    nets, ev, emb_ref, p = full_x3
    e32 = emb_ref.astype(np.float32)
    src, dst, _ = p.build_graph(e32)
    src, dst = src.cpu().numpy(), dst.cpu().numpy()
    sc = p.filter(e32, src, dst)[0].cpu().numpy()
    idx = np.sort(np.random.default_rng(5).choice(src.size, 20000, replace=False))
    ref = oracle.filter_scores(e32, src[idx], dst[idx], nets)
    print(f"bf16x3 mu=200 filter: {src.size} edges, sampled |dp| max {np.abs(sc[idx] - ref).max():.3g}")
    assert src.size > 2_000_000
    assert np.abs(sc[idx] - ref).max() <= SCORE_TOL


def test_full_gnn_one_iteration(full_x3):
    """The split-BF16 interaction-network kernels at full size (~1M edges, one
    message-passing step), every score against the oracle at the FP32 bar."""
    from paper_2501_05520_amd.trk import Pipeline
    nets, ev, emb_ref, p = full_x3
    e32 = emb_ref.astype(np.float32)
    src, dst, _ = p.build_graph(e32)
    fs, fd = src.cpu().numpy()[::3], dst.cpu().numpy()[::3]
    cfg1 = MU200.with_(gnn_iters=1)
    nets1 = make_weights(cfg1, 0)
    p1 = Pipeline(cfg1, nets1, "bf16x3", max_hits=ev.n, max_cand_edges=4_000_000, max_kept_edges=4_000_000)
    q = p1.gnn(ev.x, fs, fd).cpu().numpy()
    p1.close()
    q_ref = oracle.interaction_network(ev.x, fs, fd, nets1, 1)
    print(f"bf16x3 mu=200 gnn (1 step, {fs.size} edges): |dp| max {np.abs(q - q_ref).max():.3g}")
    assert fs.size > 900_000
    assert np.abs(q - q_ref).max() <= SCORE_TOL
