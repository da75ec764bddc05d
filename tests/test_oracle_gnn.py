"""Pins for the oracle's interaction network: an independent dense-incidence
formulation written with torch in float64, hand graphs, and disjoint-union
invariance."""
import numpy as np
import torch

import oracle
from gen import TINY, make_weights, generate_event


def _lin(u, layer):
    w, b = layer
    return u @ torch.from_numpy(w.astype(np.float64)) + torch.from_numpy(b.astype(np.float64))


def _net(u, layers, last_linear=False):
    for i, layer in enumerate(layers):
        u = _lin(u, layer)
        if not (last_linear and i == len(layers) - 1):
            u = torch.tanh(u)
    return u


def _dense_in(x, src, dst, nets, iters):
    """Interaction network with incidence matrices: B_s[e, i] = 1 iff src_e = i;
    the first edge-network layer is split into its three weight blocks."""
    x = torch.from_numpy(np.asarray(x, np.float64))
    n, m = x.shape[0], len(src)
    Bs = torch.zeros(m, n, dtype=torch.float64)
    Bd = torch.zeros(m, n, dtype=torch.float64)
    Bs[torch.arange(m), torch.as_tensor(src)] = 1.0
    Bd[torch.arange(m), torch.as_tensor(dst)] = 1.0
    h = _net(x, nets["node_enc"])
    w_e0, b_e0 = nets["edge_enc"][0]
    e = torch.tanh(Bs @ x @ torch.from_numpy(w_e0[:3].astype(np.float64))
                   + Bd @ x @ torch.from_numpy(w_e0[3:].astype(np.float64))
                   + torch.from_numpy(b_e0.astype(np.float64)))
    e = torch.tanh(_lin(e, nets["edge_enc"][1]))
    H = h.shape[1]
    w1, b1 = nets["edge_net"][0]
    W1 = torch.from_numpy(w1.astype(np.float64))
    for _ in range(iters):
        pre = (Bs @ h) @ W1[:H] + (Bd @ h) @ W1[H:2 * H] + e @ W1[2 * H:] + torch.from_numpy(b1.astype(np.float64))
        e = e + torch.tanh(_lin(torch.tanh(pre), nets["edge_net"][1]))
        mag = Bs.T @ e + Bd.T @ e
        h = h + _net(torch.cat([h, mag], dim=1), nets["node_net"])
    wo, bo = nets["out"][0]
    Wo = torch.from_numpy(wo.astype(np.float64))
    z = torch.tanh((Bs @ h) @ Wo[:H] + (Bd @ h) @ Wo[H:2 * H] + e @ Wo[2 * H:]
                   + torch.from_numpy(bo.astype(np.float64)))
    z = _lin(z, nets["out"][1])[:, 0]
    return torch.sigmoid(z).numpy(), h.numpy(), e.numpy()


def _tiny_graph(seed=1):
    ev = generate_event(seed, 1)
    nets = make_weights(TINY, 0)
    r = oracle.event(ev.x, nets, TINY)
    return ev, nets, r


def test_matches_dense_incidence_form():
    ev, nets, r = _tiny_graph()
    assert r["fsrc"].size > 100
    p, states = oracle.interaction_network(ev.x, r["fsrc"], r["fdst"], nets, TINY.gnn_iters, return_states=True)
    pd, hd, ed = _dense_in(ev.x, r["fsrc"], r["fdst"], nets, TINY.gnn_iters)
    assert np.allclose(p, pd, atol=1e-12)
    assert np.allclose(states[-1][0], hd, atol=1e-11)
    assert np.allclose(states[-1][1], ed, atol=1e-11)


def test_no_edges():
    nets = make_weights(TINY, 0)
    x = generate_event(2, 1).x[:20]
    e0 = np.zeros(0, np.int64)
    p, states = oracle.interaction_network(x, e0, e0, nets, 3, return_states=True)
    assert p.size == 0
    h = oracle.mlp(x, nets["node_enc"], tanh_last=True)
    for _ in range(3):
        h = h + oracle.mlp(np.concatenate([h, np.zeros_like(h)], axis=1), nets["node_net"], tanh_last=True)
    assert np.allclose(states[-1][0], h, atol=0)


def test_single_edge_and_path_by_hand():
    nets = make_weights(TINY, 0)
    x = np.array([[0.1, 0.2, -0.3], [0.5, -0.1, 0.7], [0.9, 0.4, 0.0]], np.float32)
    for src, dst in [([0], [1]), ([0, 1], [1, 2])]:
        p, _, _ = _dense_in(x, src, dst, nets, 2)
        assert np.allclose(oracle.interaction_network(x, src, dst, nets, 2), p, atol=1e-13)
    # on one edge, both endpoints receive the same message e
    x2 = x[:2]
    _, states = oracle.interaction_network(x2, [0], [1], nets, 1, return_states=True)
    h0, e0 = states[0]
    h1, e1 = states[1]
    for i in range(2):
        want = h0[i] + oracle.mlp(np.concatenate([h0[i], e1[0]])[None], nets["node_net"], tanh_last=True)[0]
        assert np.allclose(h1[i], want, atol=0)


def test_disjoint_union_invariance():
    nets = make_weights(TINY, 0)
    ev1, _, r1 = _tiny_graph(1)
    ev2, _, r2 = _tiny_graph(2)
    n1 = ev1.n
    x = np.concatenate([ev1.x, ev2.x])
    s = np.concatenate([r1["fsrc"], r2["fsrc"] + n1])
    d = np.concatenate([r1["fdst"], r2["fdst"] + n1])
    p = oracle.interaction_network(x, s, d, nets, TINY.gnn_iters)
    assert np.allclose(p[:r1["fsrc"].size], r1["gnn_scores"], atol=1e-14)
    assert np.allclose(p[r1["fsrc"].size:], r2["gnn_scores"], atol=1e-14)
