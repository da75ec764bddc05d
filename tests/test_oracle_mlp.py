"""Pins for the oracle's MLP stages (embedding, filter): a library Linear in
float64, and hand cases whose value is known without the code under test."""
import numpy as np
import torch

import oracle
from gen import TINY, MU200, make_weights, generate_event


def _torch_mlp(u, layers, tanh_last=False):
    h = torch.from_numpy(np.asarray(u, np.float64))
    for i, (w, b) in enumerate(layers):
        # torch's Linear stores weight as [out, in]: pass the transpose
        h = torch.nn.functional.linear(h, torch.from_numpy(w.astype(np.float64)).T.contiguous(),
                                       torch.from_numpy(b.astype(np.float64)))
        if i < len(layers) - 1 or tanh_last:
            h = torch.tanh(h)
    return h.numpy()


def test_embed_matches_torch_linear():
    nets = make_weights(TINY, 0)
    x = generate_event(1, 1).x
    assert np.allclose(oracle.embed(x, nets), _torch_mlp(x, nets["emb"]), rtol=0, atol=1e-13)


def test_filter_matches_torch_linear():
    nets = make_weights(TINY, 0)
    rng = np.random.default_rng(0)
    emb = rng.normal(size=(40, TINY.emb_dim)).astype(np.float32)
    src = rng.integers(0, 40, 200)
    dst = rng.integers(0, 40, 200)
    p = oracle.filter_scores(emb, src, dst, nets)
    u = np.concatenate([emb[src], emb[dst]], axis=1)
    z = _torch_mlp(u, nets["filt"])[:, 0]
    assert np.allclose(p, 1 / (1 + np.exp(-z)), atol=1e-14)


def test_mlp_hand_cases():
    x = np.array([[0.3, -0.2, 0.9], [1.5, 0.0, -2.0]])
    zero = [(np.zeros((3, 4), np.float32), np.array([1, 2, 3, 4], np.float32)),
            (np.zeros((4, 2), np.float32), np.array([-1, 5], np.float32))]
    assert np.array_equal(oracle.mlp(x, zero), np.tile([-1.0, 5.0], (2, 1)))
    ident = [(np.eye(3, dtype=np.float32), np.zeros(3, np.float32)),
             (np.eye(3, dtype=np.float32), np.zeros(3, np.float32))]
    assert np.allclose(oracle.mlp(x, ident), np.tanh(x), atol=0)
    assert np.allclose(oracle.mlp(x, ident, tanh_last=True), np.tanh(np.tanh(x)), atol=0)
    # a transposed weight would fail this non-square case
    w = np.arange(6, dtype=np.float32).reshape(3, 2)
    one = [(w, np.zeros(2, np.float32))]
    assert np.array_equal(oracle.mlp(x, one), x @ w)


def test_sigmoid_extremes():
    z = np.array([-800.0, -30.0, 0.0, 30.0, 800.0])
    p = oracle.sigmoid(z)
    assert p[2] == 0.5 and p[0] == 0.0 and p[4] == 1.0
    assert abs(p[1] - np.exp(-30) / (1 + np.exp(-30))) < 1e-25
    assert np.all(np.isfinite(p))


def test_filter_edges_strict_and_ordered():
    s = np.array([0, 0, 1, 2, 3])
    d = np.array([1, 4, 2, 3, 4])
    p = np.array([0.5, 0.7, 0.2, 0.50000001, 0.9])
    fs, fd = oracle.filter_edges(p, s, d, 0.5)
    assert fs.tolist() == [0, 2, 3] and fd.tolist() == [4, 3, 4]
