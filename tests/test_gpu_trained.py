"""The chain on the trained weights (weights/trained_mu200.npz, written by the seeded
training recipe): end-to-end parity with the FP64 oracle on a pile-up-10 event, a
non-degenerate candidate set at pile-up 200 (thousands of candidates, tracks found
against the generator truth), and the served forms' candidate agreement with FP32."""
import hashlib
import json
import os

import numpy as np
import pytest

from gen import MU200, generate_event, load_trained
from tests.chain_parity import chain_parity
from tests.gpu_helpers import label_agreement

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "weights", "trained_mu200.npz")
RECORD = os.path.join(ROOT, "weights", "trained_mu200.json")


@pytest.fixture(scope="module")
def trained():
    with open(WEIGHTS, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    with open(RECORD) as fh:
        rec = json.load(fh)
    assert digest == rec["sha256"], "weights file differs from the one its record describes"
    cfg, nets = load_trained(WEIGHTS, MU200)
    return cfg, nets


def test_trained_end_to_end_parity(trained):
    """trk_event on the trained weights equals the staged calls, and the FP64 oracle's
    chain with the GPU's decision taken only on margin edges gives identical labels."""
    from paper_2501_05520_amd.trk import Pipeline
    cfg, nets = trained
    ev = generate_event(300, 10)
    p = Pipeline(cfg, nets, "fp32", max_hits=8192)
    st = chain_parity(p, ev.x, nets, emb_tol=1e-5, score_tol=1e-4)
    p.close()
    print(f"trained chain, pile-up 10: {st}")
    assert st["n_kept"] > 0 and st["candidates"] > 10


def test_trained_chain_finds_tracks(trained):
    """At pile-up 200 the trained chain gives a candidate set of ordinary track
    candidates (thousands, not a few giant components) that matches generated
    particles (double-majority matching)."""
    from paper_2501_05520_amd.evaluate_trained import match_candidates
    from paper_2501_05520_amd.trk import Pipeline
    cfg, nets = trained
    ev = generate_event(200, MU200.n_collisions)
    p = Pipeline(cfg, nets, "fp32", max_hits=ev.n)
    labels, info = p.event(ev.x)
    p.close()
    found, n_true, n_cand, fake = match_candidates(labels.cpu().numpy(), ev.pid)
    sizes = np.bincount(labels.cpu().numpy())
    print(f"trained chain, pile-up 200: {info['n_cand_edges']} candidate, {info['n_filt_edges']} filtered, "
          f"{info['n_kept_edges']} kept edges; {n_cand} candidates ({fake} fake), largest {sizes.max()} hits; "
          f"efficiency {found / n_true:.4f}")
    assert n_cand >= 1000 and sizes.max() < 1000 and found / n_true > 0.05


@pytest.mark.parametrize("precision", ["bf16x3", "bf16x3gnn16", "bf16", "fp8"])
def test_trained_served_forms_agreement(trained, precision):
    """Candidate exact-match Jaccard and hit agreement of each served form against
    FP32 at pile-up 200 on the trained weights (reported; the benchmark reports the
    ten-event figures).  The trained chain turns differences of 1e-5 into changed
    candidates: its filter cut sits where the scores are dense (about 4,000 edges per
    event within 1e-4 of it), and a changed filtered edge moves the interaction
    network's scores around it.  So even split BF16 changes about 3 % of the
    candidates (measured: Jaccard 0.967-0.974, hit agreement 0.996-0.997; FP32 itself
    differs from the exact chain in 0.3 % of its candidates, see the last test); the bars
    below only guard that figure (hit >= 0.99, Jaccard >= 0.9) and keep every form's
    hits mostly in their FP32 candidate."""
    from paper_2501_05520_amd.trk import Pipeline
    cfg, nets = trained
    ev = generate_event(201, MU200.n_collisions)
    p32 = Pipeline(cfg, nets, "fp32", max_hits=ev.n)
    l32, _ = p32.event(ev.x)
    p32.close()
    px = Pipeline(cfg, nets, precision, max_hits=ev.n)
    lx, ix = px.event(ev.x)
    px.close()
    hit, jac = label_agreement(lx.cpu().numpy(), l32.cpu().numpy())
    print(f"trained chain, {precision} vs fp32 at pile-up 200: hit agreement {hit:.6f}, candidate jaccard {jac:.6f} "
          f"(kept edges {ix['n_kept_edges']})")
    assert hit > 0.5
    if precision == "bf16x3":
        assert hit >= 0.99 and jac >= 0.9


def test_trained_scores_against_fp64_per_precision(trained):
    """Stage-isolated score errors on the trained weights against the FP64 oracle (the
    filter on the oracle's candidate edges and embedding, the interaction network on its
    filtered edges; pile-up-10 event).  FP32 holds the 1e-4 bar.  The trained networks
    amplify product roundings far more than the seeded ones (the interaction network's
    encoders separate hits millimetres apart): split BF16, whose products carry about
    2^-16 relative error against FP32's 2^-24, reaches 8.7e-5 at the 99th percentile and
    8.4e-4 at the maximum on these weights; the longer the network is trained the more it
    amplifies (1.6e-4 and 2.9e-4 at the maximum after 2,800 and 14,000 steps, where a CPU
    emulation of its roundings matched the first figure).  So its bar is the FP32 one,
    1e-4, at the 99th percentile, and 2e-3 at the maximum.
    BF16 gets regression guards only (filter 0.05, interaction network 0.3): its network's
    scores move by up to 0.21 on these weights (0.15-0.18 on the shorter-trained ones;
    with BF16 hit coordinates in its encoders they moved by up to 0.29)."""
    import oracle
    from paper_2501_05520_amd.trk import Pipeline
    cfg, nets = trained
    ev = generate_event(300, 10)
    r = oracle.event(ev.x, nets, cfg)
    e32 = r["emb"].astype(np.float32)
    err = {}
    for prec in ("fp32", "bf16x3", "bf16"):
        p = Pipeline(cfg, nets, prec, max_hits=ev.n)
        pf = p.filter(e32, r["src"], r["dst"])[0].cpu().numpy()
        q = p.gnn(ev.x, r["fsrc"], r["fdst"]).cpu().numpy()
        p.close()
        df, dq = np.abs(pf - r["filter_scores"]), np.abs(q - r["gnn_scores"])
        err[prec] = (df.max(), np.percentile(df, 99), dq.max(), np.percentile(dq, 99))
        print(f"trained {prec} vs fp64: filter max {df.max():.3g} p99 {np.percentile(df, 99):.3g}; "
              f"gnn max {dq.max():.3g} p99 {np.percentile(dq, 99):.3g} ({dq.size} edges)")
    assert r["fsrc"].size > 1000
    assert max(err["fp32"]) <= 1e-4
    assert err["bf16x3"][0] <= 1e-4 and err["bf16x3"][2] <= 2e-3
    assert err["bf16x3"][1] <= 1e-4 and err["bf16x3"][3] <= 1e-4
    assert err["bf16"][2] <= 0.3 and err["bf16"][0] <= 0.05


@pytest.mark.timeout(900)
def test_trained_fp32_against_the_exact_chain(trained):
    """How far FP32 itself is from exact arithmetic on the trained chain at pile-up
    200: the FP64 oracle's own chain (its own graph, cuts and components, no margin
    substitution) against trk_event in FP32.  Reported for the record (candidate
    exact-match Jaccard and hit agreement); the parity proper, with the GPU's decision
    taken on margin edges, is test_trained_end_to_end_parity.  Measured: hit agreement
    0.99953, candidate Jaccard 0.997 (the chain's thousands of margin edges make even
    FP32 change a few candidates); asserted with a margin: hit >= 0.999, Jaccard >= 0.99."""
    import oracle
    from paper_2501_05520_amd.trk import Pipeline
    cfg, nets = trained
    ev = generate_event(202, MU200.n_collisions)
    p = Pipeline(cfg, nets, "fp32", max_hits=ev.n)
    lab, info = p.event(ev.x)
    p.close()
    r = oracle.event(ev.x, nets, cfg)
    hit, jac = label_agreement(lab.cpu().numpy(), np.asarray(r["labels"]))
    print(f"trained chain, FP32 against the FP64 oracle's own chain at pile-up 200: hit agreement {hit:.6f}, "
          f"candidate jaccard {jac:.6f} (GPU {info['n_cand_edges']} / {info['n_filt_edges']} / {info['n_kept_edges']} "
          f"edges, oracle {r['src'].size} / {r['fsrc'].size} / {int(np.sum(r['gnn_scores'] > cfg.score_cut))})")
    assert hit >= 0.999 and jac >= 0.99
