"""The allocation-free radius graph (trk_build_graph_noalloc) against the context
entry point trk_build_graph on the same embeddings: identical edges and counts,
on two calls in a row (the second with a smaller input, so that the device array
still holds the first call's contents), and its limits."""
import numpy as np
import pytest
import torch

from gen import TINY, MU200, make_weights, generate_event

pytestmark = pytest.mark.gpu


def _both(pipe, emb, cfg):
    from paper_2501_05520_amd import trk
    src, dst, nsat = pipe.build_graph(emb)
    cap = int(pipe.config.max_cand_edges)
    s2 = torch.full((cap,), -1, dtype=torch.int32, device=emb.device)
    d2 = torch.full((cap,), -1, dtype=torch.int32, device=emb.device)
    ne, ns = trk.trk_build_graph_noalloc(emb, np.float32(cfg.radius), cfg.k_max, s2, d2)
    return (src, dst, nsat), (s2[:ne], d2[:ne], ns)


def test_noalloc_graph_equals_context_graph():
    from paper_2501_05520_amd.trk import Pipeline
    dev = torch.device("cuda", 0)
    # first call: a pile-up-200 event (110,000 hits, saturated points) through the
    # full-size embedding
    ev = generate_event(200, MU200.n_collisions)
    big = Pipeline(MU200, make_weights(MU200, 0), "fp32", max_hits=ev.n, max_cand_edges=4_194_304)
    emb = big.embed(torch.as_tensor(ev.x, device=dev))
    (a_s, a_d, a_n), (b_s, b_d, b_n) = _both(big, emb, MU200)
    big.close()
    print(f"pile-up 200: {ev.n} hits, {a_s.numel()} edges, {a_n} saturated")
    assert a_s.numel() > 2_000_000 and a_n > 0
    assert torch.equal(a_s, b_s) and torch.equal(a_d, b_d) and a_n == b_n
    # second call, smaller: a tiny event through the tiny embedding (other dim, radius, K)
    ev2 = generate_event(3, 1)
    small = Pipeline(TINY, make_weights(TINY, 0), "fp32", max_hits=8192)
    emb2 = small.embed(torch.as_tensor(ev2.x, device=dev))
    (a_s, a_d, a_n), (b_s, b_d, b_n) = _both(small, emb2, TINY)
    print(f"tiny: {ev2.n} hits, {a_s.numel()} edges, {a_n} saturated")
    assert a_s.numel() > 1000
    assert torch.equal(a_s, b_s) and torch.equal(a_d, b_d) and a_n == b_n
    small.close()


def test_noalloc_graph_limits():
    from paper_2501_05520_amd import trk
    dev = torch.device("cuda", 0)
    ev = generate_event(3, 1)
    small = trk.Pipeline(TINY, make_weights(TINY, 0), "fp32", max_hits=8192)
    emb = small.embed(torch.as_tensor(ev.x, device=dev))
    src, _, _ = small.build_graph(emb)
    small.close()
    total = src.numel()
    s = torch.empty(16, dtype=torch.int32, device=dev)
    d = torch.empty(16, dtype=torch.int32, device=dev)
    with pytest.raises(trk.TrkError) as e:             # capacity: the total is reported
        trk.trk_build_graph_noalloc(emb, TINY.radius, TINY.k_max, s, d)
    assert e.value.status == -3 and str(total) in str(e.value)
    too_many = torch.zeros((131073, TINY.emb_dim), dtype=torch.float32, device=dev)
    with pytest.raises(trk.TrkError) as e:             # more hits than the array holds
        trk.trk_build_graph_noalloc(too_many, TINY.radius, TINY.k_max, s, d)
    assert e.value.status == -1
    assert trk.trk_build_graph_noalloc(emb[:0], TINY.radius, TINY.k_max, s, d) == (0, 0)
