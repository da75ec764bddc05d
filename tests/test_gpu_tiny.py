"""GPU parity on the tiny configuration (550 hits, 50 tracks): every stage is
fed the oracle's upstream output (stage-isolated) and compared element by
element with the FP64 oracle; then the whole chain end to end."""
import numpy as np
import pytest
import torch

import oracle
from gen import TINY, MU200, make_weights, generate_event, pack_events
from tests.chain_parity import chain_parity
from tests.gpu_helpers import compare_edges

pytestmark = pytest.mark.gpu

SEEDS = list(range(1, 9))
SCORE_TOL = 1e-4          # |p_gpu - p_oracle| in FP32
EMB_TOL = 2e-5            # relative to max(1, |emb|): FP32 accumulation over <= 64-term sums


@pytest.fixture(scope="module")
def nets():
    return make_weights(TINY, 0)


@pytest.fixture(scope="module")
def pipe(nets):
    from paper_2501_05520_amd.trk import Pipeline
    p = Pipeline(TINY, nets, "fp32", max_hits=8192, max_events=16)
    yield p
    p.close()


@pytest.fixture(scope="module")
def ref(nets):
    out = {}
    for s in SEEDS:
        ev = generate_event(s, 1)
        out[s] = (ev, oracle.event(ev.x, nets, TINY))
    return out


@pytest.mark.parametrize("seed", SEEDS)
def test_embed(pipe, ref, seed):
    ev, r = ref[seed]
    emb = pipe.embed(ev.x).cpu().numpy()
    err = np.abs(emb - r["emb"]) / np.maximum(1.0, np.abs(r["emb"]))
    assert err.max() <= EMB_TOL, err.max()


@pytest.mark.parametrize("seed", SEEDS)
def test_build_graph(pipe, ref, seed):
    ev, r = ref[seed]
    emb32 = r["emb"].astype(np.float32)
    src, dst, nsat = pipe.build_graph(emb32)
    src, dst = src.cpu().numpy(), dst.cpu().numpy()
    # canonical form: src < dst, sorted by (src, dst), no duplicates
    assert np.all(src < dst)
    key = src.astype(np.int64) * ev.n + dst
    assert np.all(np.diff(key) > 0)
    rad = float(np.float32(TINY.radius))
    lo, hi, d2 = oracle.radius_pairs(emb32, rad)
    os_, od, cnt = oracle.radius_graph(emb32, rad, TINY.k_max)
    ndiff, nbad, det = compare_edges(emb32, src, dst, os_, od, rad, TINY.k_max, lo, hi, d2)
    assert nbad == 0, det
    assert abs(nsat - int((cnt > TINY.k_max).sum())) <= ndiff


@pytest.mark.parametrize("seed", SEEDS)
def test_filter(pipe, ref, seed):
    ev, r = ref[seed]
    emb32 = r["emb"].astype(np.float32)
    scores, ks, kd = pipe.filter(emb32, r["src"], r["dst"])
    p_ref = oracle.filter_scores(emb32, r["src"], r["dst"], make_weights(TINY, 0))
    p = scores.cpu().numpy()
    assert np.abs(p - p_ref).max() <= SCORE_TOL
    # kept edges: the GPU's own cut of its own scores, in order
    keep = p > np.float32(TINY.filter_cut)
    assert np.array_equal(ks.cpu().numpy(), r["src"][keep]) and np.array_equal(kd.cpu().numpy(), r["dst"][keep])
    # against the oracle's cut: only edges within the tolerance of the cut may differ
    keep_ref = p_ref > np.float32(TINY.filter_cut)
    flip = keep != keep_ref
    assert np.all(np.abs(p_ref[flip] - TINY.filter_cut) <= SCORE_TOL)


@pytest.mark.parametrize("seed", SEEDS)
def test_gnn(pipe, ref, nets, seed):
    ev, r = ref[seed]
    p = pipe.gnn(ev.x, r["fsrc"], r["fdst"]).cpu().numpy()
    assert p.shape == r["gnn_scores"].shape
    assert np.abs(p - r["gnn_scores"]).max() <= SCORE_TOL


@pytest.mark.parametrize("seed", SEEDS)
def test_components_stage_isolated(pipe, ref, seed):
    ev, r = ref[seed]
    p32 = r["gnn_scores"].astype(np.float32)
    want = oracle.components(ev.n, r["fsrc"], r["fdst"], p32, np.float32(TINY.score_cut))
    got = pipe.components(ev.n, r["fsrc"], r["fdst"], p32, TINY.score_cut).cpu().numpy()
    assert np.array_equal(got, want)


def test_components_hand_graphs(pipe):
    cases = [
        (5, [(3, 4), (2, 3), (1, 2), (0, 1)], [0] * 5),
        (6, [(5, 0), (5, 1), (5, 2)], [0, 0, 0, 3, 4, 0]),
        (4, [(0, 1), (1, 2), (2, 3), (3, 0)], [0] * 4),
        (8, [(0, 1), (0, 2), (1, 2), (3, 4), (4, 5), (5, 6), (3, 6)], [0, 0, 0, 3, 3, 3, 3, 7]),
        (3, [], [0, 1, 2]),
    ]
    for n, edges, want in cases:
        s = [a for a, _ in edges]
        d = [b for _, b in edges]
        got = pipe.components(n, s, d, None).cpu().numpy().tolist()
        assert got == want, (n, edges)
    # a long chain whose ids descend along it
    n = 6000
    s = np.arange(n - 1, 0, -1)
    got = pipe.components(n, s, s - 1, None).cpu().numpy()
    assert np.all(got == 0)


def test_components_random_vs_oracle(pipe):
    rng = np.random.default_rng(7)
    for trial in range(5):
        n = int(rng.integers(100, 5000))
        m = int(rng.integers(0, 2 * n))
        s = rng.integers(0, n, m)
        d = rng.integers(0, n, m)
        sc = rng.uniform(0, 1, m).astype(np.float32)
        want = oracle.components(n, s, d, sc, np.float32(0.5))
        got = pipe.components(n, s, d, sc, 0.5).cpu().numpy()
        assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", SEEDS)
def test_event_end_to_end(pipe, ref, nets, seed):
    """trk_event equals the staged calls, and the oracle's chain with the GPU's
    decision taken only on margin edges gives identical labels (no fallback)."""
    ev, r = ref[seed]
    st = chain_parity(pipe, ev.x, nets, EMB_TOL, SCORE_TOL)
    print(f"tiny seed {seed}: {st}")
    assert st["n_cand"] == r["src"].size or st["band_diffs"] > 0


def test_deterministic(pipe, ref):
    ev, _ = ref[1]
    a, _ = pipe.event(ev.x)
    b, _ = pipe.event(ev.x)
    assert torch.equal(a, b)
    e1 = pipe.embed(ev.x)
    s1, d1, _ = pipe.build_graph(e1)
    sc1 = pipe.gnn(ev.x, s1, d1)
    sc2 = pipe.gnn(ev.x, s1, d1)
    assert torch.equal(sc1, sc2)


def test_batch_equals_alone(pipe, ref):
    evs = [ref[s][0] for s in SEEDS]
    x, offs = pack_events(evs)
    labels, infos = pipe.batch(x, offs)
    labels = labels.cpu().numpy()
    for b, ev in enumerate(evs):
        alone, info = pipe.event(ev.x)
        assert np.array_equal(labels[offs[b]:offs[b + 1]], alone.cpu().numpy())
        assert infos[b]["n_cand_edges"] == info["n_cand_edges"]
        assert infos[b]["n_filt_edges"] == info["n_filt_edges"]
        assert infos[b]["n_kept_edges"] == info["n_kept_edges"]
        assert infos[b]["n_saturated"] == info["n_saturated"]


def test_gnn_scores_alone_vs_disjoint_union(pipe, ref):
    (e1, r1), (e2, r2) = ref[1], ref[2]
    x = np.concatenate([e1.x, e2.x])
    s = np.concatenate([r1["fsrc"], r2["fsrc"] + e1.n])
    d = np.concatenate([r1["fdst"], r2["fdst"] + e1.n])
    both = pipe.gnn(x, s, d).cpu().numpy()
    a = pipe.gnn(e1.x, r1["fsrc"], r1["fdst"]).cpu().numpy()
    b = pipe.gnn(e2.x, r2["fsrc"], r2["fdst"]).cpu().numpy()
    assert np.array_equal(both, np.concatenate([a, b]))


def test_edge_cases(pipe):
    from paper_2501_05520_amd import trk
    # empty event
    labels, info = pipe.event(np.zeros((0, 3), np.float32))
    assert labels.numel() == 0 and info["n_hits"] == 0
    # single hit: no edges, own label
    labels, info = pipe.event(np.array([[0.5, 0.1, 0.2]], np.float32))
    assert labels.cpu().tolist() == [0] and info["n_cand_edges"] == 0
    # gnn with no edges
    assert pipe.gnn(np.zeros((4, 3), np.float32), [], []).numel() == 0
    # too many hits
    with pytest.raises(trk.TrkError) as e:
        pipe.event(np.zeros((9000, 3), np.float32))
    assert e.value.status == -1
    # out-of-range edge index is rejected, not read
    with pytest.raises(trk.TrkError) as e:
        pipe.components(4, [0, 7], [1, 2], None)
    assert e.value.status == -1


@pytest.mark.parametrize("precision", ["bf16", "bf16emb32", "bf16x3", "bf16x3gnn16", "fp8", "fp8all"])
def test_edge_cases_every_precision(nets, ref, precision):
    """The degenerate cases in every precision's kernels: an empty event, a single hit,
    the interaction network with no edge, and a filter cut that no score passes (every
    spacepoint is then its own component).  The FP8 forms need hidden widths in blocks
    of 128 (a context with the tiny network is refused), so they run on the full-size
    network with a pile-up-1 event."""
    from paper_2501_05520_amd.trk import Pipeline
    if precision.startswith("fp8"):
        cfg, nw, ev = MU200, make_weights(MU200, 0), generate_event(2, 1)
    else:
        cfg, nw, ev = TINY, nets, ref[2][0]
    p = Pipeline(cfg, nw, precision, max_hits=8192)
    labels, info = p.event(np.zeros((0, 3), np.float32))
    assert labels.numel() == 0 and info["n_hits"] == 0
    labels, info = p.event(np.array([[0.5, 0.1, 0.2]], np.float32))
    assert labels.cpu().tolist() == [0] and info["n_cand_edges"] == 0
    assert p.gnn(np.zeros((4, 3), np.float32), [], []).numel() == 0
    p.close()
    q = Pipeline(cfg.with_(filter_cut=1.0), nw, precision, max_hits=8192)
    labels, info = q.event(ev.x)
    q.close()
    assert info["n_filt_edges"] == 0 and info["n_kept_edges"] == 0
    assert np.array_equal(labels.cpu().numpy(), np.arange(ev.n))


def test_fp8_refuses_the_tiny_network(nets):
    """FP8 products take k in blocks of 128: a context whose filter (or embedding)
    hidden width is 64 is refused with TRK_E_INVAL instead of being run."""
    from paper_2501_05520_amd import trk
    for precision in ("fp8", "fp8all"):
        with pytest.raises(trk.TrkError) as e:
            trk.Pipeline(TINY, nets, precision, max_hits=8192)
        assert e.value.status == -1


def test_capacity_reported(pipe, ref):
    from paper_2501_05520_amd import trk
    ev, r = ref[1]
    emb = pipe.embed(ev.x)
    with pytest.raises(trk.TrkError) as e:
        pipe.build_graph(emb, cap=100)
    assert e.value.status == -3
    with pytest.raises(trk.TrkError) as e:
        pipe.filter(r["emb"].astype(np.float32), r["src"], r["dst"], cap=10)
    assert e.value.status == -3


def test_exact_ties_saturated(pipe):
    """80 copies of one embedding point plus 60 spread points: every copy has 79
    neighbours at distance exactly 0 (more than k_max = 64), so the K-cap is decided
    by the id order alone; both sides see d^2 = 0, so the edge sets must be equal."""
    rng = np.random.default_rng(11)
    emb = np.concatenate([np.tile(np.full((1, TINY.emb_dim), 0.25, np.float32), (80, 1)),
                          rng.uniform(-3, 3, (60, TINY.emb_dim)).astype(np.float32)])
    emb = emb[rng.permutation(emb.shape[0])]
    src, dst, nsat = pipe.build_graph(emb)
    os_, od, cnt = oracle.radius_graph(emb, np.float32(TINY.radius), TINY.k_max)
    assert np.array_equal(src.cpu().numpy(), os_) and np.array_equal(dst.cpu().numpy(), od)
    assert nsat == int((cnt > TINY.k_max).sum()) >= 80


def test_chain_with_no_filtered_edge(nets, ref):
    """A filter cut no score can pass: the interaction network gets no edge and every
    spacepoint is its own component."""
    from paper_2501_05520_amd.trk import Pipeline
    ev, _ = ref[2]
    p = Pipeline(TINY.with_(filter_cut=1.0), nets, "fp32", max_hits=8192)
    labels, info = p.event(ev.x)
    p.close()
    assert info["n_cand_edges"] > 0 and info["n_filt_edges"] == 0 and info["n_kept_edges"] == 0
    assert np.array_equal(labels.cpu().numpy(), np.arange(ev.n))
