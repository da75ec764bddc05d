"""Emulation of the FP8 mode's quantised arithmetic on the CPU (test helper).

It applies the storage formats the FP8 mode uses to the same float32 weights
and inputs and evaluates the products in float64, so that a kernel mistake in
fragment layout or scaling shows up as a large error while legitimate
differences (float32 accumulation order, the tanh approximation, an activation
that lands on the other side of an E4M3 rounding boundary) stay small:
  * narrow first layers: inputs and weights rounded to bfloat16 (nearest even);
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


def embed_fp8(x, nets):
    layers = nets["emb"]
    h = np.tanh(_bf16_layer(x, *layers[0]))
    for w, b in layers[1:-1]:
        h = np.tanh(_fp8_layer(h, w, b))
    return _fp8_layer(h, *layers[-1])


def filter_fp8(emb, src, dst, nets):
    layers = nets["filt"]
    e = np.asarray(emb, np.float32)
    u = np.concatenate([e[src], e[dst]], axis=1)
    h = np.tanh(_bf16_layer(u, *layers[0]))
    for w, b in layers[1:-1]:
        h = np.tanh(_fp8_layer(h, w, b))
    w, b = layers[-1]
    z = h @ np.asarray(w, np.float64) + np.asarray(b, np.float64)
    return 1.0 / (1.0 + np.exp(-z[:, 0]))
