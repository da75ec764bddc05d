"""FP64 oracle of the training objective of the filter MLP and the interaction
network, and its hand-derived gradient.  TEST INFRASTRUCTURE ONLY (tests, smoke
check, CPU baseline).

The paper trains nothing in the service; the objective here is the reading
taken for the training configuration: binary cross-entropy with logits on the
generator's truth (an edge is true when both ends carry the same non-zero
particle id), averaged over the candidate edges for the filter and over the
filtered edges for the interaction network, the two terms summed.  The edge
sets are held fixed (the cuts are not differentiable).

  L = mean_{E_c} bce(z_f, y) + mean_{E_f} bce(z_o, y),
  bce(z, y) = max(z, 0) - z y + log(1 + exp(-|z|)),  d bce / dz = sigmoid(z) - y.

Gradients are returned for every weight and bias of the filter and of the five
interaction-network MLPs, in the layout of gen.weights.make_weights.
"""
import numpy as np

from .pipeline import sigmoid


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def bce_with_logits(z, y):
    z = _f64(z)
    y = _f64(y)
    return np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))


def edge_truth(pid, src, dst):
    pid = np.asarray(pid)
    return ((pid[src] == pid[dst]) & (pid[src] != 0)).astype(np.float64)


# ---------------------------------------------------------------------------
# MLP forward keeping activations, and its backward
# ---------------------------------------------------------------------------
def mlp_forward(u, layers, tanh_last):
    """Returns the list of layer outputs a_0 = u, a_1 .. a_L (after tanh where
    applied; the last one linear unless tanh_last)."""
    acts = [_f64(u)]
    for li, (w, b) in enumerate(layers):
        z = acts[-1] @ _f64(w) + _f64(b)
        if li < len(layers) - 1 or tanh_last:
            z = np.tanh(z)
        acts.append(z)
    return acts


def mlp_backward(acts, layers, tanh_last, d_out):
    """Gradient of a scalar with respect to the MLP's weights and input, given
    d_out = dL/d(output).  Returns ([(dW, db)...], d_input)."""
    grads = [None] * len(layers)
    d = _f64(d_out)
    for li in range(len(layers) - 1, -1, -1):
        if li < len(layers) - 1 or tanh_last:
            d = d * (1.0 - acts[li + 1] ** 2)          # through tanh: d tanh(z)/dz = 1 - tanh^2
        w, _ = layers[li]
        grads[li] = (acts[li].T @ d, d.sum(axis=0))
        d = d @ _f64(w).T
    return grads, d


# ---------------------------------------------------------------------------
# filter
# ---------------------------------------------------------------------------
def filter_loss_and_grad(emb, src, dst, y, nets):
    u = np.concatenate([_f64(emb)[src], _f64(emb)[dst]], axis=1)
    acts = mlp_forward(u, nets["filt"], tanh_last=False)
    z = acts[-1][:, 0]
    m = max(len(src), 1)
    loss = bce_with_logits(z, y).sum() / m
    dz = (sigmoid(z) - y) / m
    grads, _ = mlp_backward(acts, nets["filt"], False, dz[:, None])
    return loss, z, grads


# ---------------------------------------------------------------------------
# interaction network
# ---------------------------------------------------------------------------
def gnn_forward(x, src, dst, nets, iters):
    """Forward keeping every intermediate needed by the backward."""
    x = _f64(x)
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    st = {"x": x, "src": src, "dst": dst}
    st["node_enc"] = mlp_forward(x, nets["node_enc"], True)
    st["edge_enc"] = mlp_forward(np.concatenate([x[src], x[dst]], axis=1), nets["edge_enc"], True)
    h = st["node_enc"][-1]
    e = st["edge_enc"][-1]
    st["steps"] = []
    for _ in range(iters):
        ea = mlp_forward(np.concatenate([h[src], h[dst], e], axis=1), nets["edge_net"], True)
        e_new = e + ea[-1]
        msg = np.zeros_like(h)
        np.add.at(msg, src, e_new)
        np.add.at(msg, dst, e_new)
        na = mlp_forward(np.concatenate([h, msg], axis=1), nets["node_net"], True)
        h_new = h + na[-1]
        st["steps"].append({"h": h, "e": e, "edge_acts": ea, "node_acts": na})
        h, e = h_new, e_new
    st["h"], st["e"] = h, e
    st["out"] = mlp_forward(np.concatenate([h[src], h[dst], e], axis=1), nets["out"], False)
    st["z"] = st["out"][-1][:, 0]
    return st


def gnn_backward(st, nets, dz):
    """Gradients of the five MLPs given dL/dz_o."""
    src, dst, x = st["src"], st["dst"], st["x"]
    H = st["h"].shape[1]
    g = {}
    g["out"], du = mlp_backward(st["out"], nets["out"], False, _f64(dz)[:, None])
    dh = np.zeros_like(st["h"])
    np.add.at(dh, src, du[:, :H])
    np.add.at(dh, dst, du[:, H:2 * H])
    de = du[:, 2 * H:].copy()
    gsum = {k: None for k in ("edge_net", "node_net")}
    for step in reversed(st["steps"]):
        # node update h' = h + phi_v([h, msg])
        gn, dnin = mlp_backward(step["node_acts"], nets["node_net"], True, dh)
        dh_prev = dh + dnin[:, :H]
        dmsg = dnin[:, H:]
        # msg_i = sum of e' over edges at i  ->  de' += dmsg[src] + dmsg[dst]
        de = de + dmsg[src] + dmsg[dst]
        # edge update e' = e + phi_e([h_s, h_t, e])
        ge, dein = mlp_backward(step["edge_acts"], nets["edge_net"], True, de)
        np.add.at(dh_prev, src, dein[:, :H])
        np.add.at(dh_prev, dst, dein[:, H:2 * H])
        de = de + dein[:, 2 * H:]
        dh = dh_prev
        for name, gg in (("node_net", gn), ("edge_net", ge)):
            gsum[name] = gg if gsum[name] is None else [(a[0] + b[0], a[1] + b[1]) for a, b in zip(gsum[name], gg)]
    g["edge_net"] = gsum["edge_net"] or [(np.zeros_like(_f64(w)), np.zeros_like(_f64(b))) for w, b in nets["edge_net"]]
    g["node_net"] = gsum["node_net"] or [(np.zeros_like(_f64(w)), np.zeros_like(_f64(b))) for w, b in nets["node_net"]]
    g["edge_enc"], _ = mlp_backward(st["edge_enc"], nets["edge_enc"], True, de)
    g["node_enc"], _ = mlp_backward(st["node_enc"], nets["node_enc"], True, dh)
    return g


def gnn_loss_and_grad(x, src, dst, y, nets, iters):
    st = gnn_forward(x, src, dst, nets, iters)
    m = max(len(src), 1)
    loss = bce_with_logits(st["z"], y).sum() / m
    dz = (sigmoid(st["z"]) - y) / m
    return loss, st["z"], gnn_backward(st, nets, dz)


def train_loss_and_grad(x, pid, emb, cand, filt, nets, iters):
    """Total objective and gradients: cand = (src, dst) of E_c, filt = (src, dst) of E_f."""
    yc = edge_truth(pid, *cand)
    yf = edge_truth(pid, *filt)
    lf, zf, gf = filter_loss_and_grad(emb, cand[0], cand[1], yc, nets)
    lg, zg, gg = gnn_loss_and_grad(x, filt[0], filt[1], yf, nets, iters)
    gg["filt"] = gf
    return lf + lg, (zf, zg), gg


TRAINED_NETS = ("filt", "node_enc", "edge_enc", "edge_net", "node_net", "out")


# ---------------------------------------------------------------------------
# embedding (metric learning)
# ---------------------------------------------------------------------------
def pair_loss_and_grad(emb, pa, pb, y, margin, neg_weight=1.0):
    """Pair objective of the metric-learning embedding (a reading: the paper only
    says that hits of one particle end up close together in the latent space):
        L = mean over positive pairs of d^2
            + neg_weight * mean over negative pairs of max(0, margin - d)^2
    with d the Euclidean distance of the two embeddings.  Returns (L, dL/demb)."""
    e = _f64(emb)
    pa = np.asarray(pa, np.int64)
    pb = np.asarray(pb, np.int64)
    y = np.asarray(y) > 0.5
    diff = e[pa] - e[pb]
    d2 = np.einsum("ij,ij->i", diff, diff)
    d = np.sqrt(d2)
    npos, nneg = int(y.sum()), int((~y).sum())
    hinge = np.maximum(0.0, margin - d)
    loss = (d2[y].sum() / npos if npos else 0.0) + neg_weight * ((hinge[~y] ** 2).sum() / nneg if nneg else 0.0)
    coef = np.zeros_like(d)
    if npos:
        coef[y] = 2.0 / npos
    if nneg:
        act = (~y) & (hinge > 0) & (d > 0)
        coef[act] = -2.0 * neg_weight * hinge[act] / d[act] / nneg
    g = coef[:, None] * diff
    demb = np.zeros_like(e)
    np.add.at(demb, pa, g)
    np.add.at(demb, pb, -g)
    return loss, demb


def embed_loss_and_grad(x, pa, pb, y, margin, nets, neg_weight=1.0):
    acts = mlp_forward(x, nets["emb"], tanh_last=False)
    loss, demb = pair_loss_and_grad(acts[-1], pa, pb, y, margin, neg_weight)
    grads, _ = mlp_backward(acts, nets["emb"], False, demb)
    return loss, acts[-1], grads
