"""Pins for the oracle's hand-derived gradient of the training objective:
central finite differences in FP64 on the loss itself (computed by the forward
only), and the BCE closed form."""
import zlib

import numpy as np
import pytest

import oracle
from oracle import train as T
from gen import TINY, make_weights, generate_event


def _setup(seed=3, iters=2):
    cfg = TINY.with_(gnn_iters=iters)
    nets = make_weights(cfg, 0)
    ev = generate_event(seed, 1)
    r = oracle.event(ev.x, nets, cfg)
    return cfg, nets, ev, r


def _loss(nets, ev, r, iters):
    yc = T.edge_truth(ev.pid, r["src"], r["dst"])
    yf = T.edge_truth(ev.pid, r["fsrc"], r["fdst"])
    u = np.concatenate([r["emb"][r["src"]], r["emb"][r["dst"]]], axis=1)
    zf = oracle.mlp(u, nets["filt"])[:, 0]
    zg = T.gnn_forward(ev.x, r["fsrc"], r["fdst"], nets, iters)["z"]
    return T.bce_with_logits(zf, yc).mean() + T.bce_with_logits(zg, yf).mean()


def test_bce_closed_form():
    z = np.array([-50.0, -2.0, 0.0, 3.0, 60.0])
    y = np.array([1.0, 0.0, 1.0, 1.0, 0.0])
    p = 1 / (1 + np.exp(-z[1:4]))
    want = -(y[1:4] * np.log(p) + (1 - y[1:4]) * np.log(1 - p))
    got = T.bce_with_logits(z, y)
    assert np.allclose(got[1:4], want, rtol=1e-12)
    assert abs(got[0] - 50.0) < 1e-12 and abs(got[4] - 60.0) < 1e-12


@pytest.mark.parametrize("net", ["filt", "out", "edge_net", "node_net", "edge_enc", "node_enc"])
def test_gradient_matches_finite_differences(net):
    iters = 2
    cfg, nets, ev, r = _setup(iters=iters)
    nets = {k: [(w.astype(np.float64), b.astype(np.float64)) for w, b in v] for k, v in nets.items()}
    loss, _, grads = T.train_loss_and_grad(ev.x, ev.pid, r["emb"], (r["src"], r["dst"]), (r["fsrc"], r["fdst"]),
                                           nets, iters)
    assert abs(loss - _loss(nets, ev, r, iters)) < 1e-12
    rng = np.random.default_rng(zlib.crc32(net.encode()))   # stable across processes
    eps = 1e-6
    checked = 0
    for li, (w, b) in enumerate(nets[net]):
        for arr, garr in ((w, grads[net][li][0]), (b, grads[net][li][1])):
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + eps
                lp = _loss(nets, ev, r, iters)
                flat[idx] = old - eps
                lm = _loss(nets, ev, r, iters)
                flat[idx] = old
                fd = (lp - lm) / (2 * eps)
                an = garr.reshape(-1)[idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (net, li, idx, fd, an)
                checked += 1
    assert checked >= 12


def test_no_edges_gradient_is_zero_for_edge_nets():
    cfg, nets, ev, r = _setup()
    e0 = np.zeros(0, np.int64)
    loss, z, g = T.gnn_loss_and_grad(ev.x, e0, e0, np.zeros(0), nets, 2)
    assert loss == 0.0 and z.size == 0
    assert all(np.all(gw == 0) and np.all(gb == 0) for gw, gb in g["edge_net"])


def _pairs(ev, rng, n_neg=800):
    pid = ev.pid
    order = np.lexsort((ev.layer, pid))
    s = order[:-1]
    t = order[1:]
    same = (pid[s] == pid[t]) & (pid[s] > 0)
    pa, pb = list(s[same]), list(t[same])
    na = rng.integers(0, ev.n, n_neg)
    nb = rng.integers(0, ev.n, n_neg)
    keep = na != nb
    pa += list(na[keep])
    pb += list(nb[keep])
    y = np.concatenate([np.ones(int(same.sum())), (pid[na[keep]] == pid[nb[keep]]) & (pid[na[keep]] > 0)])
    return np.array(pa), np.array(pb), y.astype(np.float64)


def test_pair_loss_closed_form():
    e = np.array([[0.0, 0.0], [3.0, 4.0], [0.3, 0.4]])
    loss, g = T.pair_loss_and_grad(e, [0, 0], [1, 2], [1.0, 0.0], margin=1.0)
    # positive: d^2 = 25; negative: d = 0.5, hinge 0.5 -> 0.25
    assert abs(loss - 25.25) < 1e-12
    # d(d^2)/de0 = 2 (e0 - e1) = (-6, -8); negative: -2 * 0.5 / 0.5 * (e0 - e2) = (0.6, 0.8)
    assert np.allclose(g[0], [-6 + 0.6, -8 + 0.8]) and np.allclose(g[1], [6, 8]) and np.allclose(g[2], [-0.6, -0.8])
    # weight 10 on the negative term: 25 + 10 * 0.25, negative gradient scaled by 10
    loss, g = T.pair_loss_and_grad(e, [0, 0], [1, 2], [1.0, 0.0], margin=1.0, neg_weight=10.0)
    assert abs(loss - 27.5) < 1e-12
    assert np.allclose(g[0], [-6 + 6.0, -8 + 8.0]) and np.allclose(g[1], [6, 8]) and np.allclose(g[2], [-6.0, -8.0])


def test_embedding_gradient_matches_finite_differences():
    cfg = TINY
    nets = {k: [(w.astype(np.float64), b.astype(np.float64)) for w, b in v] for k, v in make_weights(cfg, 0).items()}
    ev = generate_event(4, 1)
    pa, pb, y = _pairs(ev, np.random.default_rng(1))
    margin, lam = 0.5, 3.0
    loss, emb, grads = T.embed_loss_and_grad(ev.x, pa, pb, y, margin, nets, neg_weight=lam)

    def L():
        e = oracle.mlp(ev.x, nets["emb"])
        return T.pair_loss_and_grad(e, pa, pb, y, margin, lam)[0]

    assert abs(L() - loss) < 1e-12
    rng = np.random.default_rng(5)
    eps = 1e-6
    for li, (w, b) in enumerate(nets["emb"]):
        for arr, garr in ((w, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, min(5, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + eps
                lp = L()
                flat[idx] = old - eps
                lm = L()
                flat[idx] = old
                fd = (lp - lm) / (2 * eps)
                assert abs(fd - garr.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (li, idx, fd)
