"""Emulation of the FP8 mode's quantised arithmetic on the CPU (test helper).

It applies the storage formats the FP8 mode uses to the same float32 weights
and inputs and evaluates the products in float64, so that a kernel mistake in
fragment layout or scaling shows up as a large error while legitimate
differences (float32 accumulation order, the tanh approximation, an activation
that lands on the other side of an E4M3 rounding boundary) stay small:
  * narrow first MLP layers: inputs and weights rounded to bfloat16 (nearest even);
    the filter's first layer, which reads both ends of an edge, takes their float32
    mean and difference [(u_s + u_t) / 2, u_s - u_t] with the weights
    [W_s + W_t; (W_s - W_t) / 2] (formed in float64, stored as float32), as the
    kernels do; the interaction network's encoders read the hit features unrounded
    (their first layers run in FP32);
  * hidden layers: weights W * s rounded to E4M3 with s the largest power of two
    such that max|W| * s <= 448; the activations they read, 256 * tanh(.), rounded
    to E4M3; the product is divided by 256 s;
  * the filter's single-output layer in float32 weights on unquantised tanh
    outputs; the embedding's output layer as a hidden layer.
E4M3 rounding is torch's float8_e4m3fn conversion (nearest even), after
clamping to +-448 as the saturating encoder does.
"""
import math

import numpy as np
import torch


def e4m3(a):
    t = torch.as_tensor(np.asarray(a, dtype=np.float32)).clamp(-448.0, 448.0)
    return t.to(torch.float8_e4m3fn).to(torch.float64).numpy()


def bf16(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def pow2_scale(w):
    amax = float(np.abs(np.asarray(w, np.float32)).max())
    return 1.0 if amax == 0.0 else 2.0 ** math.floor(math.log2(448.0 / amax))


def _fp8_layer(h, w, b):
    s = pow2_scale(w)
    q = e4m3(256.0 * h)
    wq = e4m3(np.asarray(w, np.float64) * s)
    return (q @ wq) / (256.0 * s) + np.asarray(b, np.float64)


def _bf16_layer(u, w, b):
    return bf16(u) @ bf16(w) + np.asarray(b, np.float64)


def _bf16_pair_layer(u_s, u_t, w, b):
    """A BF16 first layer over both ends of an edge, in its mean/difference form."""
    u_s = np.asarray(u_s, np.float32)
    u_t = np.asarray(u_t, np.float32)
    u = np.concatenate([np.float32(0.5) * (u_s + u_t), u_s - u_t], axis=1)
    w = np.asarray(w, np.float64)
    D = u_s.shape[1]
    wm = np.concatenate([w[:D] + w[D:2 * D], 0.5 * (w[:D] - w[D:2 * D])]).astype(np.float32)
    return _bf16_layer(u, wm, b)


def embed_bf16(x, nets):
    """The BF16 embedding: every hidden layer on BF16-rounded inputs and weights, its
    activations stored in BF16, except the last hidden layer's, which the output layer
    reads unrounded with float32 weights (products here in float64)."""
    layers = nets["emb"]
    h = np.asarray(x, np.float32)
    for w, b in layers[:-2]:
        h = np.tanh(_bf16_layer(h, w, b))
    w, b = layers[-2]
    h = np.tanh(_bf16_layer(h, w, b))                  # not rounded: read in FP32
    w, b = layers[-1]
    return h @ np.asarray(w, np.float64) + np.asarray(b, np.float64)


def embed_fp8(x, nets):
    layers = nets["emb"]
    h = np.tanh(_bf16_layer(x, *layers[0]))
    for w, b in layers[1:-1]:
        h = np.tanh(_fp8_layer(h, w, b))
    return _fp8_layer(h, *layers[-1])


def filter_fp8(emb, src, dst, nets):
    layers = nets["filt"]
    e = np.asarray(emb, np.float32)
    h = np.tanh(_bf16_pair_layer(e[src], e[dst], *layers[0]))
    for w, b in layers[1:-1]:
        h = np.tanh(_fp8_layer(h, w, b))
    w, b = layers[-1]
    z = h @ np.asarray(w, np.float64) + np.asarray(b, np.float64)
    return 1.0 / (1.0 + np.exp(-z[:, 0]))


# ---------------------------------------------------------------------------
# FP8 interaction network: edge states and per-node projections stored as
# E4M3(v * s) with power-of-two scales from bounds, the edge-side products (e-block
# and second layer of the edge network, e-block of the output head) in FP8 with
# activations E4M3(256 tanh), the node side (encoders, node network, projections)
# in BF16, FP32 node states and message sums.
# ---------------------------------------------------------------------------
def pow2_for_bound(bound):
    return 2.0 ** math.floor(math.log2(448.0 / bound)) if bound > 0 else 1.0


def gnn_state_scales(nets, iters):
    H = nets["node_enc"][1][0].shape[1]
    hb = float(iters + 1)
    colmax = 0.0
    for name in ("edge_net", "out"):
        w = np.asarray(nets[name][0][0], np.float64)
        colmax = max(colmax, np.abs(w[:H]).sum(axis=0).max(), np.abs(w[H:2 * H]).sum(axis=0).max())
    return pow2_for_bound(hb), pow2_for_bound(hb * colmax * 1.01)


def _q(v, s):
    return e4m3(np.asarray(v, np.float64) * s) / s


def _fp8_w(w):
    s = pow2_scale(w)
    return e4m3(np.asarray(w, np.float64) * s) / s


def gnn_fp8(x, src, dst, nets, iters):
    x = np.asarray(x, np.float32)
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    H = nets["node_enc"][1][0].shape[1]
    se, sp = gnn_state_scales(nets, iters)
    (n1w, n1b), (n2w, n2b) = nets["node_enc"]
    (e1w, e1b), (e2w, e2b) = nets["edge_enc"]
    (ew1, eb1), (ew2, eb2) = nets["edge_net"]
    (vw1, vb1), (vw2, vb2) = nets["node_net"]
    (ow1, ob1), (ow2, ob2) = nets["out"]
    f64 = lambda a: np.asarray(a, np.float64)

    def proj(h, w1):                        # [h W_a | h W_b] in BF16, stored as E4M3
        return _q(bf16(h) @ bf16(np.concatenate([w1[:H], w1[H:2 * H]], axis=1)), sp)

    # the encoders' first layers read the hit features in FP32 (products here in FP64)
    h = np.tanh(bf16(np.tanh(f64(x) @ f64(n1w) + f64(n1b))) @ bf16(n2w) + f64(n2b))
    pj = proj(h, ew1 if iters > 0 else ow1)
    u = np.concatenate([f64(x[src]), f64(x[dst])], axis=1)
    e = _q(np.tanh(bf16(np.tanh(u @ f64(e1w) + f64(e1b))) @ bf16(e2w) + f64(e2b)), se)
    wc, w2, woc = _fp8_w(ew1[2 * H:]), _fp8_w(ew2), _fp8_w(ow1[2 * H:])
    n = x.shape[0]
    for it in range(iters):
        t1 = np.tanh(e @ wc + pj[src, :H] + pj[dst, H:] + f64(eb1))
        t1 = e4m3(256.0 * t1) / 256.0
        e = _q(e + np.tanh(t1 @ w2 + f64(eb2)), se)
        m = np.zeros((n, H))
        np.add.at(m, src, e)
        np.add.at(m, dst, e)
        t = np.tanh(np.concatenate([bf16(h), bf16(m)], axis=1) @ bf16(vw1) + f64(vb1))
        h = h + np.tanh(bf16(t) @ bf16(vw2) + f64(vb2))
        pj = proj(h, ew1 if it + 1 < iters else ow1)
    v = np.tanh(e @ woc + pj[src, :H] + pj[dst, H:] + f64(ob1))
    z = v @ f64(ow2)[:, 0] + float(ob2[0])
    return 1.0 / (1.0 + np.exp(-z))
